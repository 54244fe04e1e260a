"""The INT8-digit form's exact int32 block (host logic, no GPU).

The digit GEMM accumulates, per output and digit weight s, the sums
sum_{i+j=s} a_i b_j of one k-term each in int32 (signed base-256 digits, the
low-precision words of Section 6).  The planner derives the block length K
(k-terms between folds into binary64) from the exact extremes of that sum
over the digit vectors the entries can take.  These tests

- model the digitizer's steps in Python integers and check them on every
  entry of small moduli and on seeded extremes of large ones;
- derive the extremes independently: brute force over all pairs for random
  digit-value intervals, and for the moduli of one to three digits from all
  reachable entries (convex hulls of their digit projections);
- check that entries reaching the planner's extremes exist at every size,
  that K keeps both extremes within int32, and that one more 64-term stage
  would not.
"""
import random

import numpy as np
import pytest

import mmp_inputs as gen
import paper_2601_07508_amd as mmp
from tests import int8_digit_model as dm

INT32_MAX = 2 ** 31 - 1

# moduli with one to three digits whose every entry is enumerated; several sit
# just past 127 R (the first moduli whose large entries become x - p)
SMALL = [5, 7, 127, 128, 131, 251, 255, 257, 32639, 32641, 32647, 40009, 65521, 65535, 65537, 131071,
         8355713, 16777213]
# larger moduli (seeded extremes): full-byte ones reach the widest digit range
LARGE = [16777259, 2147483647, 4294967291, 1099511627689, 68719476731, 281474976710597, 281474976710655,
         1125899906842597, 4503599627370449, 4503599627370495]


def _reachable(p):
    D = dm.digit_count(p)
    v = dm.residue_values_array(np.arange(p, dtype=np.int64), p, D)
    return D, v


def _column_ends(occ):
    """For an occupancy grid occ[x, y] of digits (offset by 128), the points
    (x, y_min) and (x, y_max) of every occupied column x: a set of points
    has the same convex hull as its columns' ends."""
    cols = np.nonzero(occ.any(axis=1))[0]
    ymin = occ[cols].argmax(axis=1)
    ymax = occ.shape[1] - 1 - occ[cols][:, ::-1].argmax(axis=1)
    pts = np.concatenate([np.stack([cols, ymin], 1), np.stack([cols, ymax], 1)]) - 128
    return pts


def _hull(P):
    occ = np.zeros((256, 256), dtype=bool)
    occ[P[:, 0] + 128, P[:, 1] + 128] = True
    return np.array(dm.hull_2d(_column_ends(occ)), dtype=np.int64)


def _exact_extremes_small(digs, D):
    """max and min of sum_{i+j=s} a_i b_j over all pairs of rows of digs (the
    reachable digit vectors), for D <= 3.  A linear function of b reaches
    its extremes over a finite set at vertices of the set's convex hull, and
    so does the resulting (convex) function of a, so only hull vertices of
    the projections need pairing."""
    hi, lo = None, None

    def upd(vals):
        nonlocal hi, lo
        vmax, vmin = int(np.max(vals)), int(np.min(vals))
        hi = vmax if hi is None else max(hi, vmax)
        lo = vmin if lo is None else min(lo, vmin)

    for s in range(2 * D - 1):
        pairs = [(i, s - i) for i in range(max(0, s - D + 1), min(s, D - 1) + 1)]
        if len(pairs) == 1:
            i, j = pairs[0]
            ea = np.array([digs[:, i].min(), digs[:, i].max()])
            eb = np.array([digs[:, j].min(), digs[:, j].max()])
            upd(np.outer(ea, eb))
        elif len(pairs) == 2:
            (i1, j1), (i2, j2) = pairs
            Ha = _hull(digs[:, [i1, i2]])
            Hb = _hull(digs[:, [j1, j2]])
            upd(Ha @ Hb.T)
        else:  # D = 3, s = 2: one hull of the low two digits per top digit
            assert D == 3 and len(pairs) == 3
            occ = np.zeros((256, 256, 256), dtype=bool)
            occ[digs[:, 2] + 128, digs[:, 0] + 128, digs[:, 1] + 128] = True
            verts = []  # rows (d0, d1, top) of every group's hull
            for t in np.nonzero(occ.any(axis=(1, 2)))[0]:
                H = dm.hull_2d(_column_ends(occ[t]))
                verts += [(h0, h1, t - 128) for h0, h1 in H]
            V = np.array(verts, dtype=np.int64)
            # a0 b2 + a1 b1 + a2 b0 over every pair of hull vertices
            upd(np.outer(V[:, 0], V[:, 2]) + np.outer(V[:, 1], V[:, 1]) + np.outer(V[:, 2], V[:, 0]))
    return hi, lo


# ---------------------------------------------------------------- the digit split


@pytest.mark.parametrize("p", SMALL + [16777259])
def test_digit_split_of_every_entry(p):
    D, v = _reachable(p)
    b = mmp.int8_bound(p)
    assert b["digits"] == D
    digs, carry = dm.digits_array(v, D)
    assert np.all(carry == 0), "a value needs more digits than the plan gives"
    assert digs.min() >= -128 and digs.max() <= 127
    back = np.zeros_like(v)
    for i in reversed(range(D)):
        back = back * 256 + digs[:, i]
    assert np.array_equal(back, v)
    assert np.all((v - np.arange(p)) % p == 0)
    assert int(v.min()) == b["lo"] and int(v.max()) == b["hi"]


def test_binary64_read_is_the_integer():
    rng = random.Random(5)
    xs = [0, 1, 2 ** 52 - 1, 2 ** 51, 2 ** 51 - 1] + [rng.randrange(2 ** 52) for _ in range(2000)]
    for x in xs:
        assert dm.read_binary64_integer(x) == x


@pytest.mark.parametrize("p", LARGE)
def test_digit_split_of_extreme_entries(p):
    D = dm.digit_count(p)
    R = dm.radix(D)
    top = 127 * R
    b = mmp.int8_bound(p)
    assert b["digits"] == D
    rng = random.Random(p)
    cand = {0, 1, 2, p - 1, p - 2, (p - 1) // 2, (p + 1) // 2}
    cand |= {x for x in (top - 1, top, top + 1, top + 2) if 0 <= x < p}
    for d in range(1, D + 1):  # digit patterns 0x80.., 0x7f.., and their neighbours
        for base in (int("80" * d, 16), int("7f" * d, 16), int("ff" * d, 16)):
            cand |= {(base + e) % p for e in (-1, 0, 1)}
    cand |= {rng.randrange(p) for _ in range(3000)}
    vals = []
    for x in sorted(cand):
        v = dm.residue_value(x, p, D)
        digs, carry = dm.digits_of(v, D)
        assert carry == 0 and all(-128 <= d <= 127 for d in digs)
        assert sum(d * 256 ** i for i, d in enumerate(digs)) == v and (v - x) % p == 0
        vals.append(v)
    assert b["lo"] <= min(vals) and max(vals) <= b["hi"]
    # the interval's ends are themselves entries' values
    assert b["hi"] == min(p - 1, top)
    assert b["lo"] == (top + 1 - p if p - 1 > top else 0)


@pytest.mark.parametrize("bits", list(range(1, 63)))
def test_integer_entries_fit_their_digits(bits):
    b = mmp.int8_bound(entry_bits=bits)
    D = b["digits"]
    assert (b["lo"], b["hi"]) == (0, 2 ** bits - 1)
    rng = random.Random(bits)
    top = 2 ** bits - 1
    if bits <= 18:
        xs = np.arange(2 ** bits, dtype=np.int64)
    else:
        xs = np.array([0, 1, top, top - 1, top // 2, top // 2 + 1] + [rng.randrange(2 ** bits) for _ in range(4000)],
                      dtype=np.int64)
    digs, carry = dm.digits_array(xs, D)
    assert np.all(carry == 0), f"{bits}-bit integers need more than {D} digits"
    # the fewest digits that do
    if D > 1:
        assert 127 * dm.radix(D - 1) < top


def test_digit_count_rule_for_integers_is_tight():
    # 2^b - 1 <= 127 R fails for b = 8D - 1 (127 R < 2^(8D-1) - 1): those
    # widths need one more digit than ceil((b + 1) / 8)
    for D in range(2, 9):
        b = 8 * D - 1
        if b > 62:
            continue
        assert 2 ** b - 1 > 127 * dm.radix(D)
        assert mmp.int8_bound(entry_bits=b)["digits"] == D + 1


# ---------------------------------------------------------------- the extremes


def _interval_cases():
    rng = random.Random(20260107508)
    cases = []
    for D in range(1, 9):
        R = dm.radix(D)
        lo_all, hi_all = -128 * R, 127 * R
        for _ in range(10):
            length = rng.randrange(1, 300)
            where = rng.random()
            if where < 0.25:
                lo = lo_all + rng.randrange(0, 600)
            elif where < 0.5:
                lo = hi_all - length - rng.randrange(0, 600)
            else:  # around a multiple of a power of 256
                unit = 256 ** rng.randrange(1, D + 1) if D > 1 else 256
                lo = rng.randrange(-(hi_all // unit), hi_all // unit + 1) * unit - rng.randrange(0, 300)
            lo = min(max(lo, lo_all), hi_all)
            hi = min(lo + length, hi_all)
            cases.append((D, lo, hi))
        cases.append((D, lo_all, lo_all + 200))
        cases.append((D, hi_all - 200, hi_all))
        cases.append((D, 0, 0))
    return cases


@pytest.mark.parametrize("D,lo,hi", _interval_cases())
def test_interval_extremes_by_brute_force(D, lo, hi):
    if D == 8 and (lo < -2 ** 63 or hi >= 2 ** 63):
        pytest.skip("outside int64")
    b = mmp.int8_interval_bound(D, lo, hi)
    digs, carry = dm.digits_array(np.arange(lo, hi + 1, dtype=np.int64), D)
    assert np.all(carry == 0)
    want_hi, want_lo = dm.pair_extremes(digs, digs, D)
    assert (b["term_max"], b["term_min"]) == (want_hi, want_lo)


@pytest.mark.parametrize("p", SMALL)
def test_extremes_over_every_entry(p):
    D, v = _reachable(p)
    digs = dm.digits_array(v, D)[0]  # distinct values have distinct digits
    want_hi, want_lo = _exact_extremes_small(digs, D)
    b = mmp.int8_bound(p)
    assert (b["term_max"], b["term_min"]) == (want_hi, want_lo)


def _check_witness(b, p, which):
    D = b["digits"]
    a, c = b["witness_" + which]
    s = b["weight_" + which]
    assert b["lo"] <= a <= b["hi"] and b["lo"] <= c <= b["hi"]
    da, ca = dm.digits_of(a, D)
    dc, cc = dm.digits_of(c, D)
    assert ca == 0 and cc == 0
    if p:  # the entries a mod p and c mod p really are read as a and c
        assert dm.residue_value(a % p, p, D) == a and dm.residue_value(c % p, p, D) == c
    assert dm.weight_sums(da, dc, D)[s] == b["term_" + which]


@pytest.mark.parametrize("p", SMALL + LARGE)
def test_extremes_are_reached_and_not_exceeded(p):
    b = mmp.int8_bound(p)
    _check_witness(b, p, "max")
    _check_witness(b, p, "min")
    # seeded search over reachable entries: random pairs, and pairs near the
    # witnesses (one digit changed), never pass the extremes
    D = b["digits"]
    rng = random.Random(p ^ 0x5EED)
    lo, hi = b["lo"], b["hi"]
    vals = [rng.randrange(lo, hi + 1) for _ in range(3000)]
    for w in b["witness_max"] + b["witness_min"]:
        for i in range(D):
            for e in (-3, -1, 1, 3):
                x = w + e * 256 ** i
                if lo <= x <= hi:
                    vals.append(x)
    digs, carry = dm.digits_array(np.array(vals, dtype=np.int64), D)
    assert np.all(carry == 0)
    got_hi, got_lo = dm.pair_extremes(digs, digs, D)
    assert got_hi <= b["term_max"] and got_lo >= b["term_min"]


@pytest.mark.parametrize("bits", [8, 15, 20, 31, 47, 55, 60, 62])
def test_integer_extremes_are_reached(bits):
    b = mmp.int8_bound(entry_bits=bits)
    _check_witness(b, 0, "max")
    _check_witness(b, 0, "min")


# ---------------------------------------------------------------- the block


def _wrap32(x):
    return (x + 2 ** 31) % 2 ** 32 - 2 ** 31


@pytest.mark.parametrize("p", SMALL + LARGE)
def test_block_is_the_longest_exact_one(p):
    b = mmp.int8_bound(p)
    K, tmax, tmin = b["kblock"], b["term_max"], b["term_min"]
    assert K % 64 == 0 and K >= 64
    # K k-terms at either extreme stay in int32 ...
    assert _wrap32(K * tmax) == K * tmax and K * tmax <= INT32_MAX
    assert _wrap32(K * tmin) == K * tmin
    # ... and one more 64-term stage at one of them wraps
    K2 = K + 64
    assert _wrap32(K2 * tmax) != K2 * tmax or _wrap32(K2 * tmin) != K2 * tmin
    # the planner's INT8 plan uses this block when k exceeds the block that
    # any entries allow (shorter products run as one block either way)
    D = b["digits"]
    K_any = (INT32_MAX // (D * 2 ** 14)) // 64 * 64
    assert mmp.plan(p, 64, 64, K_any + 1, form=mmp.FORM_INT8_WORDS)["kblock_int8"] == K
    assert mmp.plan(p, 64, 64, K_any, form=mmp.FORM_INT8_WORDS)["kblock_int8"] == K_any
    # a forced block beyond it is refused
    with pytest.raises(mmp.MmpError):
        mmp.plan(p, 64, 64, K_any + 1, form=mmp.FORM_INT8_WORDS, force_kblock=K2)


def test_block_never_shorter_than_the_any_entry_bound():
    # |d_i d_j| <= 2^14 and at most D products per weight give the block any
    # entries allow; the exact range is never worse
    for p in SMALL + LARGE:
        b = mmp.int8_bound(p)
        D = b["digits"]
        assert b["term_max"] <= D * 2 ** 14 and b["term_min"] >= -D * 128 * 127
        assert b["kblock"] >= (INT32_MAX // (D * 2 ** 14)) // 64 * 64


def test_crt_single_block_limit():
    # the multi-modular product forms the integer product in one int32 block
    # when k fits the exact block of its entries; beyond, it reduces per prime
    for bits in (20, 55, 60, 62):
        b = mmp.int8_bound(entry_bits=bits)
        K = b["kblock"]
        assert _wrap32(K * b["term_max"]) == K * b["term_max"]
        fast = mmp.workspace_crt(64, 64, K, bits, 4)
        slow = mmp.workspace_crt(64, 64, K + 1, bits, 4)
        assert fast > 0 and slow > fast
