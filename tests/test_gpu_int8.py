"""GPU parity of the INT8-digit form against the exact oracle (tolerance 0).

The form writes every entry with D = ceil(bitsize(p) / 8) signed base-256
digits, multiplies digit planes on the INT8 matrix cores with exact int32
accumulation, and folds the digit weights into a binary64 residue mod p.
Its result must equal the definition C = A B mod p exactly.
"""

import sys

import numpy as np
import pytest

import mmp_inputs as gen
import oracle
from tests import freivalds

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
mmp = pytest.importorskip("paper_2601_07508_amd")

INT8 = mmp.FORM_INT8_WORDS


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def run(p, A, B, **opts):
    m, n = A.shape[0], B.shape[1]
    C = torch.full((m, n), -1.0, dtype=torch.float64, device="cuda")
    mmp.mm_modp_async(dev(A), dev(B), C, p, 0, 0, form=INT8, **opts)
    torch.cuda.synchronize()
    return C.cpu().numpy()


def assert_exact(got, want):
    w = want.astype(np.float64)
    bad = np.nonzero(got != w)
    assert bad[0].size == 0, f"{bad[0].size} mismatches, first at {bad[0][0]},{bad[1][0]}: {got[bad][0]} vs {w[bad][0]}"
    assert not np.any(np.signbit(got))


# one prime per digit count 1..7, plus both sides of byte boundaries
PRIMES = [5, 251, 257, 65521, 65537, 8388593, 16777213, 2147483647, 4294967291, 68719476731,
          1099511627689, 281474976710597, 1125899906842597, 4503599627370449]
SHAPES = [(1, 1, 1), (17, 33, 29), (64, 64, 64), (100, 70, 300), (130, 257, 67), (33, 40, 1000)]


@pytest.mark.parametrize("p", PRIMES)
def test_int8_parity(p):
    pl = mmp.plan(p, 64, 64, 64, form=INT8)
    assert pl["form"] == INT8 and pl["digits_a"] == (p.bit_length() + 7) // 8
    for (m, n, k) in SHAPES:
        say("int8", p, m, n, k)
        A = gen.random_matrix(p + m, 1, m, k, p)
        B = gen.random_matrix(p + n, 2, k, n, p)
        assert_exact(run(p, A, B), oracle.mm_modp(p, A, B))


@pytest.mark.parametrize("p", PRIMES)
def test_int8_worst_case_digits(p):
    # entries near p - 1, near the centring threshold and at the extremes of
    # a digit (x = 0x80..80, 0x7f..7f within [0, p))
    d = (p.bit_length() + 7) // 8
    cand = [p - 1, p - 2, 0, 1, (p - 1) // 2, (p + 1) // 2]
    top = int("7f" * d, 16)
    cand += [x % p for x in (top, top + 1, int("80" * d, 16), int("80" * d, 16) - 1)]
    vals = np.array(cand, dtype=np.uint64)
    m, n, k = 24, 20, 333
    A = vals[np.arange(m * k) % len(vals)].reshape(m, k)
    B = vals[(np.arange(k * n) * 7 + 3) % len(vals)].reshape(k, n)
    say("int8 worst", p)
    assert_exact(run(p, A, B), oracle.mm_modp(p, A, B))
    Aall = np.full((m, k), p - 1, dtype=np.uint64)
    assert_exact(run(p, Aall, np.full((k, n), p - 1, dtype=np.uint64)),
                 oracle.mm_modp(p, Aall, np.full((k, n), p - 1, dtype=np.uint64)))


@pytest.mark.parametrize("p", [65521, 2147483647, 1125899906842597, 4503599627370449])
def test_int8_folds_between_blocks(p):
    # a short int32 block forces several folds into the binary64 residue
    m, n, k = 70, 66, 700
    A = gen.random_matrix(1, 1, m, k, p)
    B = gen.random_matrix(1, 2, k, n, p)
    want = oracle.mm_modp(p, A, B)
    for kb in (64, 128, 192, 640):
        say("int8 fold", p, kb)
        assert_exact(run(p, A, B, force_kblock=kb), want)


# Entries that drive one digit-weight accumulator to the planner's exact
# extreme on every k-term (the witnesses of mmp_int8_bound): with k = K, one
# whole int32 block and no split, the accumulator ends at K * term_max (or
# K * term_min).  K is the longest block of 64-term stages within int32, so
# this reaches 99.8-99.99% of 2^31 (printed per case); 2K + 71 adds a second
# full block, a fold in between and a ragged tail.  The CPU tests show that
# K + 64 would wrap.
BLOCK_PRIMES = [251, 65521, 16777213, 4294967291, 1099511627689, 281474976710597, 281474976710655,
                1125899906842597, 4503599627370449]


@pytest.mark.parametrize("which", ["max", "min"])
@pytest.mark.parametrize("p", BLOCK_PRIMES)
def test_int8_block_at_its_exact_limit(p, which):
    b = mmp.int8_bound(p)
    K = b["kblock"]
    assert mmp.plan(p, 16, 24, 2 * K + 71, form=INT8)["kblock_int8"] == K
    a, c = b["witness_" + which]
    reach = K * b["term_" + which]
    assert -2**31 <= reach <= 2**31 - 1
    say("int8 block limit", p, which, "K", K, "accumulator", reach, f"= {reach / 2**31:+.5f} of 2^31")
    m, n = 16, 24
    for k in (K, 2 * K + 71):
        A = np.full((m, k), a % p, dtype=np.uint64)
        B = np.full((k, n), c % p, dtype=np.uint64)
        A[3, :] = p - 1  # other rows and columns with other digits
        B[:, 5] = (p - 1) // 2
        assert_exact(run(p, A, B, splits=1), oracle.mm_modp(p, A, B))


def test_int8_strided_and_stream():
    p = 1099511627689
    m, n, k = 70, 50, 90
    A = gen.random_matrix(8, 1, m, k, p)
    B = gen.random_matrix(8, 2, k, n, p)
    Ab = torch.zeros((m, k + 13), dtype=torch.float64, device="cuda")
    Bb = torch.zeros((k, n + 5), dtype=torch.float64, device="cuda")
    Cb = torch.full((m, n + 9), 7.0, dtype=torch.float64, device="cuda")
    Ab[:, :k] = dev(A)
    Bb[:, :n] = dev(B)
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    mmp.mm_modp_async(Ab[:, :k], Bb[:, :n], Cb[:, :n], p, stream=s, form=INT8)
    s.synchronize()
    out = Cb.cpu().numpy()
    assert_exact(out[:, :n], oracle.mm_modp(p, A, B))
    assert np.all(out[:, n:] == 7.0)
    # A's rows starting 8 bytes past a 16-byte boundary, even row stride:
    # the digitizing reads A's entries one by one
    Ae = torch.zeros((m, k + 4), dtype=torch.float64, device="cuda")
    Ae[:, 1:k + 1] = dev(A)
    C2 = torch.full((m, n), -1.0, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    assert Ae[:, 1:].data_ptr() % 16 == 8 and Ae.stride(0) % 2 == 0
    mmp.mm_modp_async(Ae[:, 1:k + 1], Bb[:, :n], C2, p, form=INT8)
    torch.cuda.synchronize()
    assert_exact(C2.cpu().numpy(), oracle.mm_modp(p, A, B))


@pytest.mark.parametrize("p", [8388593, 68719476731, 1125899906842597, 4503599627370449])
def test_int8_equals_fp64_form(p):
    m, n, k = 200, 190, 513
    A = gen.random_matrix(2, 1, m, k, p)
    B = gen.random_matrix(2, 2, k, n, p)
    C8 = run(p, A, B)
    C64 = torch.empty((m, n), dtype=torch.float64, device="cuda")
    mmp.mm_modp_async(dev(A), dev(B), C64, p, form=mmp.FORM_FP64_WORDS)
    torch.cuda.synchronize()
    assert np.array_equal(C8, C64.cpu().numpy())


@pytest.mark.parametrize("splits", [2, 5, 8])
def test_split_k_int8(splits):
    for p in (65521, 2147483647, 4503599627370449):
        m, n, k = 70, 90, 2000 + 37
        A = gen.random_matrix(splits, 1, m, k, p)
        B = gen.random_matrix(splits, 2, k, n, p)
        say("splitk int8", p, splits)
        assert mmp.plan(p, m, n, k, form=INT8, splits=splits)["splits"] == splits
        assert_exact(run(p, A, B, splits=splits), oracle.mm_modp(p, A, B))
    # with folds inside each k-range as well
    p = 1125899906842597
    A = gen.random_matrix(1, 1, 40, 3000, p)
    B = gen.random_matrix(1, 2, 3000, 30, p)
    assert_exact(run(p, A, B, splits=splits, force_kblock=128), oracle.mm_modp(p, A, B))


@pytest.mark.parametrize("p", [251, 65521, 8388593, 2147483647, 68719476731, 1125899906842597, 4503599627370449])
def test_prepared_operands(p):
    # digit planes made once (A, B or both) give the product of the plain call
    for (m, n, k) in ((17, 33, 29), (130, 70, 300), (33, 40, 1000)):
        A = gen.random_matrix(m + n, 1, m, k, p)
        B = gen.random_matrix(m + n, 2, k, n, p)
        want = oracle.mm_modp(p, A, B)
        dA, dB = dev(A), dev(B)
        pa = mmp.prepare_operand(dA, p, 0)
        pb = mmp.prepare_operand(dB, p, 1)
        # digits x (m rounded up to 16) x (k rounded up to 64)
        assert pa.planes.numel() == pa.desc.digits * (-(-m // 16) * 16) * (-(-k // 64) * 64)
        assert pb.planes.numel() == pb.desc.digits * (-(-n // 16) * 16) * (-(-k // 64) * 64)
        for kw in ({"prepared_a": pa}, {"prepared_b": pb}, {"prepared_a": pa, "prepared_b": pb},
                   {"prepared_a": pa, "splits": 3}, {"prepared_b": pb, "force_kblock": 64}):
            say("prepared", p, m, n, k, sorted(kw))
            C = torch.full((m, n), -1.0, dtype=torch.float64, device="cuda")
            mmp.mm_modp_async(dA, dB, C, p, **kw)
            torch.cuda.synchronize()
            assert_exact(C.cpu().numpy(), want)


def test_prepared_operand_strided_and_reused():
    # planes of a strided view; reused across several B, with a caller workspace
    p = 1099511627689
    m, n, k = 90, 50, 700
    Abig = gen.random_matrix(5, 1, m, k + 13, p)
    dAbig = dev(Abig)
    dA = dAbig[:, :k]
    pa = mmp.prepare_operand(dA, p, 0)
    ws = torch.empty(mmp.plan(p, m, n, k, form=INT8)["workspace_bytes"], dtype=torch.uint8, device="cuda")
    for t in range(3):
        B = gen.random_matrix(5, 10 + t, k, n, p)
        C = torch.full((m, n), -1.0, dtype=torch.float64, device="cuda")
        say("prepared reuse", t)
        mmp.mm_modp_async(dA, dev(B), C, p, prepared_a=pa, workspace=ws)
        torch.cuda.synchronize()
        assert_exact(C.cpu().numpy(), oracle.mm_modp(p, Abig[:, :k], B))


@pytest.mark.parametrize("p", [5, 251, 65521, 8388593, 2147483647, 68719476731, 281474976710597,
                               4503599627370449])
def test_int8_many_short_tiles(p):
    # a lone product of at least 4160 output tiles of 64 x 64 with whole k in
    # at most 16 k-stages, more than twice the workgroups the device holds at
    # once: the persistent kernel (one workgroup per resident slot walking
    # its tiles, the copy ring running across tiles); ragged m, n and k, k
    # of one stage and of exactly 16.  Checked on sampled rows (every
    # column) against the oracle, and every entry by Freivalds' check: a
    # tile's first stage waits only for its own copies after a whole tile's
    # stores, and edge tiles take the bounded store path, so an ordering
    # mistake would show in tiles that no sampled row meets.
    rng = np.random.default_rng(11)
    for (m, n, k) in ((4100, 4090, 300), (4160, 4096, 64), (4096, 4111, 1024), (8200, 2060, 17)):
        A = gen.random_matrix(m + k, 1, m, k, p)
        B = gen.random_matrix(m + k, 2, k, n, p)
        rows = np.unique(np.concatenate([[0, 1, 63, 64, m // 2, m - 65, m - 64, m - 1],
                                         rng.integers(0, m, 8)]))
        say("many short tiles", p, m, n, k)
        mmp.timers_enable(True)
        mmp.timers_read(reset=True)
        C = run(p, A, B)
        t = mmp.timers_read(reset=True)
        mmp.timers_enable(False)
        assert t.get("int8_gemm_persistent", (0, 0))[0] == 1, t
        assert t.get("int8_gemm", (0, 0))[0] == 0, t
        assert t.get("int8_digitize", (0, 0))[0] == 1, t  # both operands, one launch
        assert_exact(C[rows], oracle.mm_modp(p, A[rows], B))
        freivalds.check(p, A, B, C, seed=m + n + k, trials=2 if p > 1000 else 8)


@pytest.mark.parametrize("p", [251, 65521, 8388593, 2147483647, 68719476731, 281474976710597, 4503599627370449])
def test_int8_narrow_columns(p):
    # n <= 32 runs 64 x 32 tiles: every digit count, ragged m and k, n at and
    # below the tile width, split-K and short int32 blocks
    for (m, n, k) in ((1, 1, 1), (70, 32, 200), (129, 31, 77), (64, 16, 1000), (200, 1, 130)):
        A = gen.random_matrix(m * n, 1, m, k, p)
        B = gen.random_matrix(m * n, 2, k, n, p)
        want = oracle.mm_modp(p, A, B)
        say("int8 narrow", p, m, n, k)
        assert_exact(run(p, A, B), want)
        assert_exact(run(p, A, B, splits=3), want)
        if k >= 128:
            assert_exact(run(p, A, B, force_kblock=64), want)
    # all digits at their extremes
    m, n, k = 65, 32, 300
    Aall = np.full((m, k), p - 1, dtype=np.uint64)
    Ball = np.full((k, n), p - 1, dtype=np.uint64)
    assert_exact(run(p, Aall, Ball), oracle.mm_modp(p, Aall, Ball))


def test_int8_batch_mixed_widths():
    # one launch per digit count: narrow tiles only when every product has n <= 32
    p = 1099511627689
    shapes = [(50, 32, 100), (40, 20, 300), (30, 33, 90)]
    for sel in ([0, 1], [0, 1, 2]):
        jobs, want = [], []
        for i in sel:
            m, n, k = shapes[i]
            A = gen.random_matrix(i, 1, m, k, p)
            B = gen.random_matrix(i, 2, k, n, p)
            C = torch.full((m, n), -1.0, dtype=torch.float64, device="cuda")
            jobs.append((dev(A), dev(B), C, p, 0, 0))
            want.append(oracle.mm_modp(p, A, B))
        say("int8 batch widths", sel)
        mmp.mm_modp_batched(jobs, form=INT8)
        torch.cuda.synchronize()
        for (_, _, C, *_), w in zip(jobs, want):
            assert_exact(C.cpu().numpy(), w)
