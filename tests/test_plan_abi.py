"""Host-side checks of the C library: exported symbols, planner, argument errors.

None of these calls touch a GPU (the planner is host integer arithmetic and
argument errors are returned before any device work).
"""

import ctypes
import json
import math
import os
import re

import pytest

import mmp_inputs as gen
from oracle import paper_algorithms as pa
from tests.conftest import PRIMES

mmp = pytest.importorskip("paper_2601_07508_amd")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLDEN = os.path.join(ROOT, "tests", "golden")
TWO_T = 1 << 53


def header_functions():
    """Every function declared in include/*.h."""
    names = []
    for fn in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if fn.endswith(".h"):
            src = open(os.path.join(ROOT, "include", fn)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names += re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*\b([a-z_][a-z0-9_]*)\s*\(",
                                src, flags=re.M)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    names = header_functions()
    assert "mm_modp" in names and "mmp_plan" in names
    lib = mmp.lib()
    for name in names:
        assert hasattr(lib, name), name


def test_strerror_covers_all_codes():
    for code in range(0, -9, -1):
        s = mmp.strerror(code)
        assert s and s != "unknown status"
    assert mmp.strerror(12345) == "unknown status"


SUPPORTED = [(1, 1), (1, 2), (2, 1), (1, 3), (3, 1), (2, 2), (1, 4), (4, 1), (2, 3), (3, 2), (2, 4), (4, 2)]


def test_plan_matches_oracle_lambda_table():
    rows = json.load(open(os.path.join(GOLDEN, "lambda_table.json")))["rows"]
    checked = 0
    for r in rows:
        p, u, v = r["p"], r["u"], r["v"]
        if (u, v) not in SUPPORTED:
            continue
        if r["lambda"] < 1:
            with pytest.raises(mmp.MmpError) as e:
                mmp.plan(p, 64, 64, 64, u, v)
            assert e.value.status == -2
            continue
        pl = mmp.plan(p, 64, 64, 64, u, v)
        assert (pl["alpha"], pl["beta"], pl["lambda"]) == (r["alpha"], r["beta"], r["lambda"]), r
        checked += 1
    assert checked > 50


def _tight_lazy_ok(p, u, v, L):
    """Independent re-derivation: a block starting in [-p, 2p) with L products
    of words below alpha and beta stays within 2^t."""
    a, b = pa.iroot_ceil(p, u), pa.iroot_ceil(p, v)
    w = (p - 1) ** 2 if (u, v) == (1, 1) else (a - 1) * (b - 1)
    return L * w + 2 * p - 1 <= TWO_T


def _tight_biased_ok(p, u, v, L):
    """The same for the biased reduction: a block starting in
    [-2^t, -2^t + 4p) stays within [-2^t, 2^t]."""
    a, b = pa.iroot_ceil(p, u), pa.iroot_ceil(p, v)
    w = (p - 1) ** 2 if (u, v) == (1, 1) else (a - 1) * (b - 1)
    return -TWO_T + 4 * p - 1 + L * w <= TWO_T


@pytest.mark.parametrize("p", PRIMES[2:])
@pytest.mark.parametrize("uv", SUPPORTED)
@pytest.mark.parametrize("k", [1, 7, 100, 4096, 131072])
def test_plan_invariants(p, uv, k):
    u, v = uv
    lam = pa.block_size(p, u, v)
    if lam < 1:
        return
    for strict in (False, True):
        pl = mmp.plan(p, 256, 256, k, u, v, strict_fmod=strict)
        L, S = pl["kblock"], pl["slots"]
        assert 1 <= L <= lam
        assert S >= L and (S in (4, 8, 16) or (S % 4 == 0 and S == L and S >= 12))
        if pl["lazy"]:
            assert not strict
            if pl["biased"]:  # the signed range, for a block within the paper's lambda
                a_, b_ = pa.iroot_ceil(p, u), pa.iroot_ceil(p, v)
                w = (p - 1) ** 2 if (u, v) == (1, 1) else a_ * b_  # the paper's charge
                assert L * w + 2 * p - 1 > TWO_T  # the plain range would not do
                assert _tight_biased_ok(p, u, v, L)
            else:
                assert _tight_lazy_ok(p, u, v, L)
        else:
            assert not pl["biased"]
        assert pl["q"] == 1.0 / p
        assert pl["bk"] == 16 and pl["tile"] in (1, 2, 3)


def test_auto_choice_follows_bitsize():
    # Section 3.3: (1,1) for small primes; multiword beyond 26 bits; at 52
    # bits the (2,3)-product (the (2,2) block size is 1 there).
    F = mmp.FORM_FP64_WORDS
    pl = mmp.plan(1048573, 1024, 1024, 1024, form=F)
    assert (pl["u"], pl["v"]) == (1, 1)
    for b in range(27, 53):
        pl = mmp.plan(gen.prev_prime(1 << b), 2048, 2048, 2048, form=F)
        assert pa.block_size(pl["p"], pl["u"], pl["v"]) >= 1
        assert pl["u"] * pl["v"] >= 2
    pl = mmp.plan(4503599627370449, 2048, 2048, 2048, form=F)
    assert pl["u"] * pl["v"] == 6


def test_auto_form_choice():
    # AUTO compares the planner's time estimates of the two forms
    for b in (20, 25, 36, 50, 52):
        p = gen.prev_prime(1 << b)
        pl = mmp.plan(p, 4096, 4096, 4096)
        f64 = mmp.plan(p, 4096, 4096, 4096, form=mmp.FORM_FP64_WORDS)
        i8 = mmp.plan(p, 4096, 4096, 4096, form=mmp.FORM_INT8_WORDS)
        best = mmp.FORM_INT8_WORDS if i8["est_seconds"] < f64["est_seconds"] else mmp.FORM_FP64_WORDS
        assert pl["form"] == best
        assert i8["digits_a"] == (b + 7) // 8 and i8["workspace_bytes"] == i8["digits_a"] * 8192 * 4096
    # explicit words select the FP64 form
    assert mmp.plan(1125899906842597, 4096, 4096, 4096, 2, 2)["form"] == mmp.FORM_FP64_WORDS


def test_auto_orientation_skinny():
    p = 68719476731  # 36 bits: needs a (1, v) or (v, 1) split
    pl = mmp.plan(p, 16384, 32, 4096)  # n < m: extra words on B
    assert pl["v"] >= pl["u"]
    pl = mmp.plan(p, 32, 16384, 4096)
    assert pl["u"] >= pl["v"]


@pytest.mark.parametrize("args,status", [
    ((4, 1, 1), -1), ((1 << 52, 2, 2), -1), ((33554393, 5, 1), -1), ((33554393, 3, 3), -1),
    ((33554393, 1, 0), -1), ((2147483647, 1, 1), -2), ((4503599627370449, 1, 2), -2),
])
def test_plan_errors(args, status):
    p, u, v = args
    with pytest.raises(mmp.MmpError) as e:
        mmp.plan(p, 8, 8, 8, u, v)
    assert e.value.status == status


def test_forced_kblock():
    p = 1125899906842597  # (2,2): lambda = 7
    for L in range(1, 8):
        pl = mmp.plan(p, 64, 64, 64, 2, 2, force_kblock=L)
        assert pl["kblock"] == L and pl["slots"] >= L
    with pytest.raises(mmp.MmpError) as e:
        mmp.plan(p, 64, 64, 64, 2, 2, force_kblock=8)
    assert e.value.status == -2
    p = 68719476731  # (2,2): lambda = 131071
    assert mmp.plan(p, 64, 64, 64, 2, 2, force_kblock=4096)["slots"] == 4096
    assert mmp.plan(p, 64, 64, 64, 2, 2, force_kblock=100)["slots"] == 100  # 25 whole k-steps
    with pytest.raises(mmp.MmpError):
        mmp.plan(p, 64, 64, 64, 2, 2, force_kblock=102)  # > 16 and not whole k-steps


def test_forced_block_estimate_matches_the_planner_s_own():
    # forcing the block the planner would choose changes nothing, estimate included
    for p, shape in ((1125899906842597, (8192, 8192, 8192)), (68719476731, (4096, 4096, 4096)),
                     (33554393, (512, 512, 512))):
        auto = mmp.plan(p, *shape, form=1)
        forced = mmp.plan(p, *shape, auto["u"], auto["v"], form=1, force_kblock=auto["kblock"])
        for key in ("kblock", "slots", "lazy", "tile", "est_seconds"):
            assert forced[key] == pytest.approx(auto[key]), (p, key)


def test_batch_launch_option_range():
    o = mmp.MmpOpts()
    out = mmp.MmpPlan()
    for bad in (-1, 3):
        o.batch_launch = bad
        assert mmp.lib().mmp_plan(33554393, 1, 1, 8, 8, 8, ctypes.byref(o), ctypes.byref(out)) == -1
    o.batch_launch = 2
    assert mmp.lib().mmp_plan(33554393, 1, 1, 8, 8, 8, ctypes.byref(o), ctypes.byref(out)) == 0
    # a batch option: single products refuse it before any device work
    fake = ctypes.c_void_p(0x10000)
    assert mmp.lib().mm_modp_async(ctypes.byref(o), 33554393, 0, 0, 8, 8, 8, fake, 8, ctypes.c_void_p(0x20000000),
                                   8, ctypes.c_void_p(0x40000000), 8, None) == -1


def test_footprint_counts_word_copies():
    p, m, n, k = 1125899906842597, 1000, 700, 300
    fp = mmp.footprint(p, m, n, k, 2, 2)
    assert fp == 8 * (m * k + k * n + m * n) + 8 * (2 * m * k + 2 * k * n)


def test_argument_errors_before_device_work():
    lib = mmp.lib()
    # negative sizes, null pointers with non-empty shapes, bad leading dimension
    assert lib.mm_modp(33554393, 1, 1, -1, 4, 4, None, None, None) == -1
    assert lib.mm_modp(33554393, 1, 1, 4, 4, 4, None, None, None) == -1
    o = mmp.MmpOpts()
    fake = ctypes.c_void_p(0x1000)
    assert lib.mm_modp_async(ctypes.byref(o), 33554393, 1, 1, 4, 4, 4, fake, 3, ctypes.c_void_p(0x9000), 4,
                             ctypes.c_void_p(0x20000), 4, None) == -1
    # C overlapping A
    assert lib.mm_modp_async(ctypes.byref(o), 33554393, 1, 1, 4, 4, 4, fake, 4, ctypes.c_void_p(0x9000), 4,
                             ctypes.c_void_p(0x1008), 4, None) == -1
    # p out of range is rejected by the planner before any launch
    assert lib.mm_modp(3, 1, 1, 4, 4, 4, fake, ctypes.c_void_p(0x9000), ctypes.c_void_p(0x20000)) == -1
    # (1,1) at 31 bits has no block size
    assert lib.mm_modp(2147483647, 1, 1, 4, 4, 4, fake, ctypes.c_void_p(0x9000),
                       ctypes.c_void_p(0x20000)) == -2
    # a forced FP64 form whose A stage would span 2^31 bytes or more: refused on the host
    big_a, big_b, big_c = ctypes.c_void_p(0x10000), ctypes.c_void_p(0x7e0000000000), ctypes.c_void_p(0x7f0000000000)
    assert lib.mm_modp_async(ctypes.byref(o), 33554393, 1, 1, 64, 64, 4, big_a, 1 << 28, big_b, 64,
                             big_c, 64, None) == -1
    assert lib.mm_modp_async(ctypes.byref(o), 33554393, 1, 1, 64, 64, 4, big_a, 4, big_b, 1 << 27,
                             big_c, 64, None) == -1
    # empty products succeed without touching memory
    assert lib.mm_modp(33554393, 1, 1, 0, 4, 4, None, None, None) == 0
    assert lib.mm_modp(33554393, 1, 1, 4, 0, 4, None, None, None) == 0


def test_prepared_operand_host_checks():
    lib = mmp.lib()
    p = 68719476731  # 36 bits: 5 digits
    # digits x (outer rounded up to 16) x (inner rounded up to 64)
    assert lib.mmp_operand_bytes(p, 0, 10, 100) == 5 * 16 * 128
    assert lib.mmp_operand_bytes(p, 1, 100, 10) == 5 * 16 * 128
    assert lib.mmp_operand_bytes(p, 0, 3, 64) == 5 * 16 * 64
    assert lib.mmp_operand_bytes(p, 0, 32, 65) == 5 * 32 * 128
    assert lib.mmp_operand_bytes(p, 1, 65, 33) == 5 * 48 * 128
    for bad in ((p, 2, 10, 10), (p, 0, 0, 10), (p, 1, 10, -1), (3, 0, 10, 10)):
        assert lib.mmp_operand_bytes(*bad) == 0
    fake, buf = ctypes.c_void_p(0x1000), ctypes.c_void_p(0x100000)
    d = mmp.MmpOperand()
    need = 5 * 16 * 128
    # buffer too small, missing out, bad side, ld < cols: refused before any launch
    assert lib.mmp_prepare_operand(p, 0, fake, 10, 100, 100, buf, need - 1, ctypes.byref(d), None) == -1
    assert lib.mmp_prepare_operand(p, 0, fake, 10, 100, 100, buf, need, None, None) == -1
    assert lib.mmp_prepare_operand(p, 2, fake, 10, 100, 100, buf, need, ctypes.byref(d), None) == -1
    assert lib.mmp_prepare_operand(p, 0, fake, 10, 100, 99, buf, need, ctypes.byref(d), None) == -1
    # planes overlapping the matrix they are made from
    assert lib.mmp_prepare_operand(p, 0, fake, 10, 100, 100, ctypes.c_void_p(0x1000 + 800), need,
                                   ctypes.byref(d), None) == -1
    # the planner and the other entry points refuse prepared operands
    d.planes, d.p, d.side, d.digits, d.rows, d.cols, d.kp = 0x100000, p, 0, 5, 8, 8, 64
    o = mmp.MmpOpts()
    o.prepared_a = ctypes.pointer(d)
    out = mmp.MmpPlan()
    assert lib.mmp_plan(p, 0, 0, 8, 8, 8, ctypes.byref(o), ctypes.byref(out)) == -1
    job = mmp.MmpJob(p, 0, 0, 8, 8, 8, 0x1000, 8, 0x9000, 8, 0x20000, 8)
    assert lib.mm_modp_batched(ctypes.byref(job), 1, ctypes.byref(o), None) == -1
    A, B, C = ctypes.c_void_p(0x1000), ctypes.c_void_p(0x9000), ctypes.c_void_p(0x20000)

    def call(opts, m=8, n=8, k=8, pp=p, u=0):
        return lib.mm_modp_async(ctypes.byref(opts), pp, u, u, m, n, k, A, k, B, n, C, n, None)
    # planes that do not describe the operand: other modulus, shape, side or digits
    assert call(o, pp=1099511627689) == -1
    assert call(o, m=9) == -1
    assert call(o, k=70) == -1
    for field, val in (("side", 1), ("digits", 4), ("kp", 128), ("planes", None)):
        saved = getattr(d, field)
        setattr(d, field, val)
        assert call(o) == -1, field
        setattr(d, field, saved)
    # forced FP64 words or word counts with prepared planes
    o.form = mmp.FORM_FP64_WORDS
    assert call(o) == -1
    o.form = 0
    assert call(o, u=1) == -1
    o.centered_words = 1
    assert call(o) == -1


def test_crt_reconstruct_host_checks():
    lib = mmp.lib()
    vp, u64 = ctypes.c_void_p, ctypes.c_uint64
    ptrs = (vp * 3)(0x100000, 0x200000, 0x300000)
    out = vp(0x10000000)

    def call(moduli, m=4, n=4, ldc=4, ldo=4, limbs=4, C=ptrs, o=out):
        mods = (u64 * len(moduli))(*moduli)
        return lib.mmp_crt_reconstruct(C, ldc, mods, len(moduli), m, n, o, ldo, limbs, None)
    good = [1000003, 1000033, 1000037]
    assert call(good, m=0) == 0 and call(good, n=0) == 0          # empty: nothing launched
    assert call([6, 9, 5]) == -1                                   # not coprime
    assert call([1000003, 1 << 51, 7]) == -1                       # above 2^52 / 3
    assert call([1, 5, 7]) == -1                                   # below 2
    assert call(good, limbs=0) == -1                               # M needs one limb
    big = [(1 << 50) - 35, (1 << 50) - 27, (1 << 50) - 11]         # M near 2^150: three limbs
    assert call(big, limbs=2) == -1
    assert call(good, ldc=3) == -1 and call(good, ldo=3) == -1
    assert call(good, o=None) == -1
    assert call(good, C=(vp * 3)(0x100000, None, 0x300000)) == -1
    assert call(good, o=vp(0x100000 + 8)) == -1                    # out overlaps a residue matrix
    mods = (u64 * 65)(*([3] * 65))
    assert lib.mmp_crt_reconstruct(ptrs, 4, mods, 65, 4, 4, out, 4, 4, None) == -1
    assert lib.mmp_crt_reconstruct(ptrs, 4, mods, 0, 4, 4, out, 4, 4, None) == -1


# ------------------------------------------------------------------ schedule emulation
# The kernel accumulates L word products per block, reduces (correction-free
# when the plan says lazy), and finishes with a complete reduction and the
# Horner recombination.  This exact-integer emulation of that schedule on
# worst-case words checks that no partial sum leaves [-2^53, 2^53] for the
# planner's block, and that the result is the oracle's.


def _words(x, a, u):
    w = []
    for _ in range(u - 1):
        w.append(x % a)
        x //= a
    w.append(x)
    return w


def _lazy_reduce(x, p):
    q = 1.0 / p
    assert abs(x) <= TWO_T
    c = math.floor(float(x) * q)
    d = x - c * p
    assert -p <= d < 2 * p
    return d


def _emulate_entry(p, u, v, L, lazy, arow, bcol, biased=False):
    a_, b_ = pa.iroot_ceil(p, u), pa.iroot_ceil(p, v)
    K = TWO_T // p - 1
    k = len(arow)
    acc = [[0] * v for _ in range(u)]
    peak = 0
    for i in range(u):
        for j in range(v):
            s = -K * p if biased else 0
            for l0 in range(0, k, L):
                for l in range(l0, min(k, l0 + L)):
                    s += _words(arow[l], a_, u)[i] * _words(bcol[l], b_, v)[j]
                    peak = max(peak, abs(s))
                if biased:
                    s = _biased_reduce(s, p, K)
                else:
                    s = _lazy_reduce(s, p) if lazy else s % p
            acc[i][j] = s % p
    c = 0
    for i in reversed(range(u)):
        si = 0
        for j in reversed(range(v)):
            si = (si * b_ + acc[i][j]) % p
        c = (c * a_ + si) % p
    return c, peak


@pytest.mark.parametrize("p", [33554393, 67108859, 2147483647, 68719476731, 1099511627689,
                               1125899906842597, 4503599627370449])
def test_schedule_emulation_worst_case(p):
    for (u, v) in SUPPORTED:
        lam = pa.block_size(p, u, v)
        if lam < 1:
            continue
        pl = mmp.plan(p, 64, 64, 64, u, v)
        L = min(pl["kblock"], 64)
        a_ = pa.iroot_ceil(p, u)
        # entries whose words are all large: p - 1 and the largest x < p with low word alpha - 1
        x_lowmax = ((p - 1) // a_) * a_ - 1 if u > 1 else p - 1
        for x in {p - 1, x_lowmax}:
            k = 3 * L + 1
            arow = [x] * k
            bcol = [p - 1] * k
            c, peak = _emulate_entry(p, u, v, L, bool(pl["lazy"]), arow, bcol, bool(pl["biased"]))
            assert c == (k * x * (p - 1)) % p
            assert peak <= TWO_T


def test_paper_block_with_the_signed_range_at_50_bits():
    # (2,2) at p = 2^50 - 27: the paper's lambda is 7 (eq. cAcB).  A block of
    # 7 started in [-p, 2p) could pass 2^53 (2p + 7 alpha beta > 2^53), so the
    # plain correction-free reduction allows only 6; the biased one restarts
    # at the bottom of the signed range and allows the paper's 7, run as 7 of
    # 8 slots (two MFMA k-steps per reduction instead of one).
    p = 1125899906842597
    a_ = pa.iroot_ceil(p, 2)
    assert pa.block_size(p, 2, 2) == 7 and a_ == 1 << 25
    assert 7 * a_ * a_ + 2 * p - 1 > TWO_T
    pl = mmp.plan(p, 8192, 8192, 8192, 2, 2)
    assert (pl["kblock"], pl["slots"], pl["lazy"], pl["biased"], pl["extended"]) == (7, 8, 1, 1, 0)
    assert pl["kblock"] <= pl["lambda"] == 7
    # the negative control of the emulation: 8 terms from the same start pass 2^53
    K = TWO_T // p - 1
    worst = -K * p + 4 * p - 1
    assert worst + 7 * (a_ - 1) ** 2 <= TWO_T
    # strict reductions keep the paper's range and never bias
    st = mmp.plan(p, 8192, 8192, 8192, 2, 2, strict_fmod=True)
    assert st["biased"] == 0 and st["lazy"] == 0


# ------------------------------------------------------------------ extended block bound
# The opt-in extended bound accumulates over [-2^53, 2^53]: the in-loop
# reduction is c = floor(fl(x q + K)), d = x - c p with K = floor(2^53/p) - 1.
# Emulated exactly (one rounding for the fma), on worst-case words.


def _biased_reduce(x, p, K):
    q = 1.0 / p
    assert abs(x) <= TWO_T
    b = pa.fma(float(x), q, float(K))  # one rounding of x q + K
    c = math.floor(b)
    d = x - c * p
    assert -K * p - p <= d < -K * p + 2 * p
    assert -TWO_T <= d
    return d


def _emulate_extended(p, u, v, L, arow, bcol):
    a_, b_ = pa.iroot_ceil(p, u), pa.iroot_ceil(p, v)
    K = TWO_T // p - 1
    k = len(arow)
    out = [[0] * v for _ in range(u)]
    lo = hi = 0
    for i in range(u):
        for j in range(v):
            s = -K * p  # accumulator start, congruent to 0
            for l0 in range(0, k, L):
                for l in range(l0, min(k, l0 + L)):
                    s += _words(arow[l], a_, u)[i] * _words(bcol[l], b_, v)[j]
                    lo, hi = min(lo, s), max(hi, s)
                s = _biased_reduce(s, p, K)
            out[i][j] = s % p
    c = 0
    for i in reversed(range(u)):
        si = 0
        for j in reversed(range(v)):
            si = (si * b_ + out[i][j]) % p
        c = (c * a_ + si) % p
    return c, lo, hi


@pytest.mark.parametrize("p", [33554393, 67108859, 2147483647, 68719476731, 1125899906842597,
                               4503599627370449])
def test_extended_schedule_worst_case(p):
    for (u, v) in SUPPORTED:
        if pa.block_size(p, u, v) < 1:
            continue
        pl = mmp.plan(p, 64, 64, 4096, u, v, extended_block=True)
        paper = mmp.plan(p, 64, 64, 4096, u, v)
        L = pl["kblock"]
        a_, b_ = pa.iroot_ceil(p, u), pa.iroot_ceil(p, v)
        w = (p - 1) ** 2 if (u, v) == (1, 1) else a_ * b_
        if not pl["extended"]:  # the paper's bound was the better one here
            assert (pl["kblock"], pl["slots"]) == (paper["kblock"], paper["slots"])
            continue
        assert pl["lazy"] == 1
        assert L * w + 4 * p - 1 <= 2 * TWO_T  # the extended bound
        assert L >= paper["kblock"]  # never a worse block than the paper's
        Lk = min(L, 40)
        x_low = ((p - 1) // a_) * a_ - 1 if u > 1 else p - 1
        for x in {p - 1, x_low}:
            k = 3 * Lk + 1
            c, lo, hi = _emulate_extended(p, u, v, Lk, [x] * k, [p - 1] * k)
            assert c == (k * x * (p - 1)) % p
            assert -TWO_T <= lo and hi <= TWO_T


def test_extended_doubles_block_at_50_bits():
    p = 1125899906842597
    assert mmp.plan(p, 64, 64, 4096, 2, 2)["kblock"] == 7       # paper: lambda = 7, as 7 of 8 slots
    pl = mmp.plan(p, 64, 64, 4096, 2, 2, extended_block=True)
    assert pl["kblock"] == 12 and pl["lambda"] == 7             # extended: 12 allowed, 3 k-steps
    with pytest.raises(mmp.MmpError):
        mmp.plan(p, 64, 64, 64, 2, 2, extended_block=True, strict_fmod=True)


def test_tune_cache_roundtrip(tmp_path):
    # An entry read from a file steers AUTO plans of its class; clearing it
    # restores the planner's own choice.
    p = 1125899906842597  # 50 bits
    mmp.tune_cache_clear()
    own = mmp.plan(p, 1000, 1000, 1000)
    path = tmp_path / "tune.json"
    path.write_text('{"entries": [\n'
                    '  {"bits": 50, "lm": 10, "ln": 10, "lk": 10, "ext": 0, "form": 1, "u": 2, "v": 3, '
                    '"tile": 3, "kblock": 400, "ms": 1.0}\n]}\n')
    assert mmp.tune_cache_load(str(path)) == 1
    pl = mmp.plan(p, 1000, 1000, 1000)
    assert (pl["form"], pl["u"], pl["v"], pl["tile"], pl["kblock"]) == (1, 2, 3, 3, 400)
    other = mmp.plan(p, 3000, 1000, 1000)  # a different class is unaffected
    assert (other["form"], other["u"], other["v"]) == (own["form"], own["u"], own["v"])
    out = tmp_path / "saved.json"
    mmp.tune_cache_save(str(out))
    assert '"u": 2, "v": 3' in out.read_text()
    mmp.tune_cache_clear()
    pl = mmp.plan(p, 1000, 1000, 1000)
    assert (pl["form"], pl["u"], pl["v"]) == (own["form"], own["u"], own["v"])


def test_tune_cache_entry_that_does_not_fit_is_ignored(tmp_path):
    # a tuned block longer than this p's bound falls back to a fresh plan
    p = 1125899906842597
    path = tmp_path / "tune.json"
    path.write_text('{"entries": [\n'
                    '  {"bits": 50, "lm": 6, "ln": 6, "lk": 6, "ext": 0, "form": 1, "u": 2, "v": 2, '
                    '"tile": 1, "kblock": 64, "ms": 1.0}\n]}\n')
    mmp.tune_cache_clear()
    assert mmp.tune_cache_load(str(path)) == 1
    pl = mmp.plan(p, 64, 64, 64)
    assert not (pl["form"] == 1 and (pl["u"], pl["v"]) == (2, 2) and pl["kblock"] == 64)
    assert pl["form"] == 2 or pa.block_size(p, pl["u"], pl["v"]) >= pl["kblock"] or pl["extended"]
    mmp.tune_cache_clear()


# ------------------------------------------------------------------ centered words
# The opt-in centered words: x -> x - p when 2x > p, then a split with
# quotients rounded to nearest (floor of fl(t fl(1/a) + 1/2)), and
# the in-loop reduction c = floor(fl(x q + 1/2)), d = x - c p.  Emulated
# exactly in binary64 (Python floats are IEEE binary64 with round-to-nearest-
# even; pa.fma rounds once).


def _centered_words(x, p, a, u):
    # the kernel's split: r = floor(fl(t fl(1/a) + 1/2)), one rounding (fma)
    t = x - p if 2 * x > p else x
    ainv = 1.0 / a
    w = []
    for _ in range(u - 1):
        r = math.floor(pa.fma(float(t), ainv, 0.5))
        w.append(t - r * a)
        t = r
    w.append(t)
    return w


def _centered_word_bound(p, u):
    # the library's bound, restated: floor(a/2) + 1 below the top word,
    # floor(h / a^(u-1)) + 2 for the top word, h = floor(p/2) when u = 1
    h = p // 2
    if u == 1:
        return h
    a = pa.iroot_ceil(p, u)
    return max(a // 2 + 1, h // a ** (u - 1) + 2)


def _centered_reduce(x, p):
    assert abs(x) <= TWO_T
    b = pa.fma(float(x), 1.0 / p, 0.5)  # one rounding of x q + 1/2
    d = x - math.floor(b) * p
    assert abs(d) <= p // 2 + 3
    return d


def _emulate_centered(p, u, v, L, arow, bcol):
    a_, b_ = pa.iroot_ceil(p, u), pa.iroot_ceil(p, v)
    k = len(arow)
    wa = [_centered_words(x, p, a_, u) for x in arow]
    wb = [_centered_words(y, p, b_, v) for y in bcol]
    peak = 0
    out = [[0] * v for _ in range(u)]
    for i in range(u):
        for j in range(v):
            s = 0
            for l0 in range(0, k, L):
                for l in range(l0, min(k, l0 + L)):
                    s += wa[l][i] * wb[l][j]
                    peak = max(peak, abs(s))
                s = _centered_reduce(s, p)
            out[i][j] = s % p
    c = 0
    for i in reversed(range(u)):
        si = 0
        for j in reversed(range(v)):
            si = (si * b_ + out[i][j]) % p
        c = (c * a_ + si) % p
    return c, peak


def centered_worst_entries(p, u):
    """Entries whose centered words are all near their largest magnitude."""
    h = p // 2
    if u == 1:
        return [h, p - h]
    a = pa.iroot_ceil(p, u)
    low = sum(a ** i * (a // 2 - 1) for i in range(u - 1))
    top = (h - low) // a ** (u - 1)
    x = top * a ** (u - 1) + low
    assert 0 < x <= h
    return [x, p - x, h, p - h]


@pytest.mark.parametrize("p", [101, 1009, 65521, 100003])
@pytest.mark.parametrize("u", [2, 3, 4])
def test_centered_word_bound_brute_force(p, u):
    # every entry of a small field: the words recombine to x or x - p and
    # stay within the stated bound, which is reached up to its +1/+2 margin
    a = pa.iroot_ceil(p, u)
    bound = _centered_word_bound(p, u)
    big = 0
    for x in range(p):
        w = _centered_words(x, p, a, u)
        assert sum(a ** i * wi for i, wi in enumerate(w)) == (x - p if 2 * x > p else x)
        assert all(abs(wi) <= a // 2 + 1 for wi in w[:-1])
        assert abs(w[-1]) <= (p // 2) // a ** (u - 1) + 2
        big = max(big, max(abs(wi) for wi in w))
    assert bound - 2 <= big <= bound


@pytest.mark.parametrize("p", [33554393, 67108859, 134217689, 2147483647, 68719476731, 1099511627689,
                               1125899906842597, 4503599627370449])
def test_centered_schedule_worst_case(p):
    for (u, v) in SUPPORTED:
        try:
            pl = mmp.plan(p, 64, 64, 4096, u, v, centered_words=True)
        except mmp.MmpError:
            continue
        L = pl["kblock"]
        assert pl["centered"] == 1 and pl["lazy"] == 1 and pl["extended"] == 0
        W = _centered_word_bound(p, u) * _centered_word_bound(p, v)
        assert p // 2 + 4 + L * W <= TWO_T  # the centered bound
        Lk = min(L, 40)
        for x in centered_worst_entries(p, u):
            for y in centered_worst_entries(p, v):
                k = 2 * Lk + 3
                c, peak = _emulate_centered(p, u, v, Lk, [x] * k, [y] * k)
                assert c == (k * x * y) % p
                assert peak <= TWO_T


def test_centered_longest_block_is_the_bound():
    # the planner's block never exceeds the bound, and one more term would
    for p in [33554393, 1125899906842597, 68719476731]:
        for (u, v) in [(1, 1), (2, 2), (1, 3)]:
            W = _centered_word_bound(p, u) * _centered_word_bound(p, v)
            lam = (TWO_T - p // 2 - 4) // W
            if lam < 1:
                with pytest.raises(mmp.MmpError):
                    mmp.plan(p, 64, 64, 64, u, v, centered_words=True)
                continue
            L = min(lam, 1 << 20)
            if L > 16:
                L = L // 16 * 16
            mmp.plan(p, 64, 64, 64, u, v, centered_words=True, force_kblock=L)
            if lam <= 16:
                with pytest.raises(mmp.MmpError):
                    mmp.plan(p, 64, 64, 64, u, v, centered_words=True, force_kblock=lam + 1)


def test_centered_quadruples_block_at_50_bits():
    p = 1125899906842597
    pl = mmp.plan(p, 8192, 8192, 8192, 2, 2, centered_words=True)
    assert (pl["kblock"], pl["slots"], pl["centered"]) == (28, 28, 1)  # 29 allowed, 7 k-steps
    assert mmp.plan(p, 8192, 8192, 8192, 2, 2)["kblock"] == 7  # the paper's lambda, 7 of 8 slots
    # centered words reach one bit past the paper's (1,1) limit of 26 bits
    p27 = gen.prev_prime(1 << 27)
    assert pa.block_size(p27, 1, 1) < 1
    assert mmp.plan(p27, 64, 64, 64, 1, 1, centered_words=True)["kblock"] >= 1


@pytest.mark.parametrize("bad", [dict(extended_block=True), dict(strict_fmod=True), dict(form=2)])
def test_centered_option_conflicts(bad):
    with pytest.raises(mmp.MmpError):
        mmp.plan(1125899906842597, 64, 64, 64, 0 if bad.get("form") else 2, 0 if bad.get("form") else 2,
                 centered_words=True, **bad)


# ------------------------------------------------------------------ INT8 digit-weight fold
# The INT8 form folds its 2D - 1 int32 digit-weight accumulators with
# Horner's rule: t <- (256 t - c p) + w[s], c = floor(fl(256 t q + 1/2)).
# Emulated here step by step in binary64 (pa.fma rounds once): every
# intermediate must be an exactly representable integer and the result must
# be sum 256^s w[s] mod p.


def _fold_weights(w, p):
    q = 1.0 / p
    t = float(w[-1])
    for s in range(len(w) - 2, -1, -1):
        x = 256.0 * t
        assert x == 256 * int(t) and abs(x) < 2.0 ** 61
        c = math.floor(pa.fma(x, q, 0.5))
        d = int(x) - c * p  # the fma's exact result when representable
        assert abs(d) <= p // 2 + 2 ** 10 and float(d) == d
        t = float(d + w[s])
        assert t == d + w[s] and abs(t) < 2.0 ** 53
    c = math.floor(t * q)
    d = int(t) - c * p
    d = d - p if d >= p else d
    d = d + p if d < 0 else d
    return d


@pytest.mark.parametrize("p", [5, 7, 1048573, 2147483647, 68719476731, 1125899906842597,
                               4503599627370449])
def test_int8_fold_exact(p):
    lim = 2 ** 31 - 1
    rng = gen.uniform_mod(p % 1000, 91, 4000, 2 * lim + 1)
    vals = [int(x) - lim for x in rng]
    for nd in (1, 3, 5, 9, 13, 15):
        cases = [[lim] * nd, [-lim] * nd, [lim, -lim] * (nd // 2) + [lim] * (nd % 2)]
        cases += [vals[i * nd:(i + 1) * nd] for i in range(len(vals) // nd)][:60]
        for w in cases:
            want = sum(256 ** s * ws for s, ws in enumerate(w)) % p
            assert _fold_weights(w, p) == want


# The multi-modular (CRT) epilogue combines the weights once into exact
# groups of three, G_j = w[3j] + 256 w[3j+1] + 65536 w[3j+2], and folds them
# per modulus by Horner's rule with the scale 2^24, each step
# t <- (2^24 t - c p) + (G_j - c_j p) with round-to-nearest quotients.
# Emulated step by step in binary64 (pa.fma rounds once): every
# intermediate must be exact and within the bounds the kernel's comment
# derives, and the result must be sum 256^s w[s] mod p.


def _reduce_near(x, p, q):
    assert x == int(x) and abs(x) < 2.0 ** 80
    c = math.floor(pa.fma(x, q, 0.5))
    d = int(x) - c * p  # the fma's exact result when representable
    assert abs(d) < 2 ** 53 and float(d) == d
    return d


def _fold_groups(w, p):
    q = 1.0 / p
    nd = len(w)
    g = []
    for j in range((nd + 2) // 3):
        v = float(w[3 * j])
        if 3 * j + 1 < nd:
            v = pa.fma(256.0, float(w[3 * j + 1]), v)
        if 3 * j + 2 < nd:
            v = pa.fma(65536.0, float(w[3 * j + 2]), v)
        exact = sum(256 ** i * w[3 * j + i] for i in range(3) if 3 * j + i < nd)
        assert v == exact and abs(exact) < 2 ** 47.01
        g.append(v)
    bound = p * (1 + 2.0 ** -27) + 2
    t = _reduce_near(g[-1], p, q)
    assert abs(t) <= p / 2 + 1
    for j in range(len(g) - 2, -1, -1):
        x = 16777216.0 * float(t)
        assert x == 2 ** 24 * t
        r = _reduce_near(g[j], p, q)
        assert abs(r) <= p / 2 + 1
        t = _reduce_near(x, p, q) + r
        assert abs(t) <= bound and abs(t) < 2 ** 53
    c = math.floor(float(t) * q)
    d = t - c * p
    d = d - p if d >= p else d
    d = d + p if d < 0 else d
    assert 0 <= d < p
    return d


@pytest.mark.parametrize("p", [5, 7, 257, 1048573, 2147483647, 68719476731, 1125899906842597,
                               4503599627370449, 2 ** 52 - 1])
def test_crt_group_fold_exact(p):
    # any modulus 5 <= p < 2^52 (the last one is not prime: the fold does not care)
    lim = 2 ** 31 - 1
    rng = gen.uniform_mod(p % 1000, 92, 3000, 2 * lim + 1)
    vals = [int(x) - lim for x in rng]
    for nd in (1, 2, 3, 4, 5, 7, 9, 13, 15):
        cases = [[lim] * nd, [-lim] * nd, [lim, -lim] * (nd // 2) + [lim] * (nd % 2),
                 [-lim, lim] * (nd // 2) + [-lim] * (nd % 2), [0] * nd]
        cases += [vals[i * nd:(i + 1) * nd] for i in range(len(vals) // nd)][:40]
        for w in cases:
            want = sum(256 ** s * ws for s, ws in enumerate(w)) % p
            assert _fold_groups(w, p) == want


# When the groups are small next to p (Gmax <= (2^27 - 2) p, Gmax = 65793 K
# D 2^14 for K k-terms of D digits), Horner's rule runs over the unreduced
# groups directly, t <- (2^24 t - c p) + G_j from t = G_top: the persistent
# digit GEMM's short tiles (K <= 1024, D <= 7, p >= 2^16) and the CRT
# epilogue when every modulus of the launch allows it.  Emulated step by
# step at the extreme weights, at and above the smallest modulus allowed.


def _fold_direct(w, p, gmax):
    q = 1.0 / p
    nd = len(w)
    assert gmax <= (2 ** 27 - 2) * p
    g = []
    for j in range((nd + 2) // 3):
        v = float(w[3 * j])
        if 3 * j + 1 < nd:
            v = pa.fma(256.0, float(w[3 * j + 1]), v)
        if 3 * j + 2 < nd:
            v = pa.fma(65536.0, float(w[3 * j + 2]), v)
        exact = sum(256 ** i * w[3 * j + i] for i in range(3) if 3 * j + i < nd)
        assert v == exact and abs(exact) <= gmax
        g.append(exact)
    t = g[-1]
    for j in range(len(g) - 2, -1, -1):
        x = 16777216.0 * float(t)
        assert x == 2 ** 24 * t and abs(x / p) < 2 ** 51
        d = _reduce_near(x, p, q)
        assert abs(d) < p
        t = d + g[j]
        assert abs(t) <= p + gmax and abs(t) < 2 ** 53
    # the closing rounded reduction, then p added to a negative result
    assert abs(float(t) / p) <= 2 ** 27
    d = _reduce_near(float(t), p, q)
    assert abs(d) <= p / 2 + 1
    d = d + p if d < 0 else d
    assert 0 <= d < p
    return d


def _direct_cases(p, W, seed):
    rng = gen.uniform_mod(p % 1000, seed, 3000, 2 * W + 1)
    vals = [int(x) - W for x in rng]
    for nd in (5, 7, 9, 11, 13, 15):
        cases = [[W] * nd, [-W] * nd, [W, -W] * (nd // 2) + [W] * (nd % 2),
                 [-W, W] * (nd // 2) + [-W] * (nd % 2), [0] * nd, [W] + [0] * (nd - 1)]
        cases += [vals[i * nd:(i + 1) * nd] for i in range(len(vals) // nd)][:30]
        yield from cases


@pytest.mark.parametrize("p", [65537, 16777213, 2147483647, 68719476731, 1125899906842597,
                               4503599627370449, 2 ** 16, 2 ** 52 - 1])
def test_short_tile_fold_exact(p):
    # persistent tiles: K <= 1024 k-terms of at most 7 digit products, p >= 2^16
    W = 1024 * 7 * 2 ** 14
    for w in _direct_cases(p, W, 93):
        assert _fold_direct(w, p, 65793 * W) == sum(256 ** s * ws for s, ws in enumerate(w)) % p


@pytest.mark.parametrize("K,D", [(128, 8), (2048, 8), (16320, 8), (64, 1), (1024, 4)])
def test_crt_direct_fold_exact(K, D):
    # the CRT launcher takes fold_direct when 65793 K D 2^14 <= (2^27 - 2) p
    # for every modulus; checked at the smallest such p and above
    W = K * D * 2 ** 14
    gmax = 65793 * W
    pmin = max(5, -(-gmax // (2 ** 27 - 2)))
    for p in (pmin, pmin + 1, 2 * pmin + 7, 2 ** 31 - 1, 2 ** 52 - 1):
        if p < pmin or p >= 2 ** 52:
            continue
        for w in _direct_cases(p, W, 94):
            assert _fold_direct(w, p, gmax) == sum(256 ** s * ws for s, ws in enumerate(w)) % p


@pytest.mark.parametrize("shape", [(512, 512, 131072), (16384, 16384, 256), (4096, 4096, 4096), (64, 64, 1 << 20),
                                   (1000, 30, 50000), (10923, 32, 32768), (1024, 1024, 65536), (256, 2048, 65536)])
@pytest.mark.parametrize("form", [1, 2])
def test_split_policy(shape, form):
    # k-ranges only when the output tiles cannot fill 256 CUs twice, a power of
    # two (whole k-ranges per XCD from 8 on), each range at least 1024 (FP64)
    # or 2048 (INT8) k-terms.  FP64 words: the smallest count that gives four
    # rounds of 512 workgroups.  INT8 digits: the smallest that fills one
    # round, doubled while the last round is less than 90% full.
    m, n, k = shape
    p = 8388593
    pl = mmp.plan(p, m, n, k, form=form)
    s_ = pl["splits"]
    assert s_ >= 1 and s_ & (s_ - 1) == 0 and s_ <= 64
    bm, bn = (pl["bm"], pl["bn"]) if form == 1 else (64, 64)
    tiles = -(-m // bm) * -(-n // bn)
    per = 1024 if form == 1 else 2048
    cap = min(k // per, 64)
    if tiles >= 512:
        assert s_ == 1
    if s_ > 1:
        assert k // s_ >= per
        assert pl["workspace_bytes"] >= 8 * s_ * m * n
    if tiles < 512 and k >= 2 * per:
        if form == 1:
            assert tiles * s_ >= 4 * 512 or 2 * s_ > cap
            assert s_ == 1 or tiles * s_ // 2 < 4 * 512
        else:
            def fill(x):
                w = tiles * x
                return w / (512 * -(-w // 512))
            assert (tiles * s_ >= 512 and fill(s_) >= 0.9) or 2 * s_ > cap
            assert s_ == 1 or tiles * s_ // 2 < 512 or fill(s_ // 2) < 0.9


def test_static_entry_point_host_checks():
    # mm_modp_static refuses, on the host and before any device call, a caller
    # workspace, entry validation, and a plan whose workspace exceeds its
    # fixed array (the pointers below are never dereferenced)
    lib = mmp.lib()
    fake = ctypes.c_void_p(0x10000)
    fake2 = ctypes.c_void_p(0x20000000)
    fake3 = ctypes.c_void_p(0x40000000)
    p = 4503599627370449

    def call(m, n, k, **opts):
        o = mmp._opts(**opts)
        return lib.mm_modp_static(ctypes.byref(o), p, 0, 0, m, n, k, fake, k, fake2, n, fake3, n, None)

    o = mmp._opts()
    o.workspace = 0x1000
    o.workspace_bytes = 1 << 20
    assert lib.mm_modp_static(ctypes.byref(o), p, 0, 0, 8, 8, 8, fake, 8, fake2, 8, fake3, 8, None) == -1
    assert call(8, 8, 8, validate_entries=True) == -1
    m = n = 16384
    k = 4096
    assert mmp.plan(p, m, n, k, form=2, splits=1)["workspace_bytes"] > mmp.STATIC_SCRATCH_BYTES
    assert call(m, n, k, form=2, splits=1) == -4
