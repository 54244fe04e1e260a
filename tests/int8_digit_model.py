"""A plain model of how the INT8-digit form turns entries into digits.

Test infrastructure: it restates, in Python integers, what the digitizing
kernels do to one entry, so that CPU tests can check every reachable digit
vector and the int32 block bound the planner derives from them.

- A residue x in [0, p) (stored as binary64) is read as an integer through
  its bit pattern after adding 2^52, then mapped to x' = x, or x - p when x
  exceeds 127 R, R = (256^D - 1) / 255, D = ceil(bitsize(p) / 8).
- An integer of the multi-modular product (below 2^entry_bits) is taken as
  it is.
- x' is written with D signed digits: the low byte read as int8 is the
  digit, and the exact quotient (x' - d) / 256 carries on.
- One k-term adds sum_{i+j=s} a_i b_j to the int32 accumulator of digit
  weight s (the digit products that share the weight 256^s).
"""
import struct

import numpy as np


def radix(D):
    return (256 ** D - 1) // 255


def digit_count(p):
    return (p.bit_length() + 7) // 8


def read_binary64_integer(x):
    """The digitizer's float-to-integer step for an integer 0 <= x < 2^52:
    the bit pattern of x + 2^52 minus that of 2^52."""
    bits = struct.unpack("<q", struct.pack("<d", float(x) + 4503599627370496.0))[0]
    return bits - 0x4330000000000000


def residue_value(x, p, D):
    v = read_binary64_integer(x)
    return v - p if v > 127 * radix(D) else v


def digits_of(v, D):
    """(digits, carry left after D digits); the carry is 0 when v fits."""
    out = []
    for _ in range(D):
        b = v & 0xFF
        d = b - 256 if b >= 128 else b
        out.append(d)
        v = (v - d) >> 8
    return out, v


def digits_array(values, D):
    """Digits of many int64 values at once (numpy; same steps as digits_of)."""
    v = np.asarray(values, dtype=np.int64).copy()
    out = np.empty((v.size, D), dtype=np.int64)
    for i in range(D):
        d = (v & 0xFF).astype(np.int64)
        d = np.where(d >= 128, d - 256, d)
        out[:, i] = d
        v = (v - d) >> 8
    return out, v


def residue_values_array(xs, p, D):
    """residue_value for many x (integers below 2^52, so the binary64 read is exact)."""
    x = np.asarray(xs, dtype=np.int64)
    top = 127 * radix(D)
    return np.where(x > top, x - p, x)


def weight_sums(a, b, D):
    """sum_{i+j=s} a_i b_j for s = 0 .. 2D - 2 (Python integers)."""
    return [sum(a[i] * b[s - i] for i in range(max(0, s - D + 1), min(s, D - 1) + 1)) for s in range(2 * D - 1)]


def pair_extremes(A, B, D):
    """Max and min over all pairs (rows of A, rows of B) and all weights of
    the weight sums, by brute force (numpy)."""
    best_hi, best_lo = None, None
    for s in range(2 * D - 1):
        W = np.zeros((A.shape[0], B.shape[0]), dtype=np.int64)
        for i in range(max(0, s - D + 1), min(s, D - 1) + 1):
            W += np.outer(A[:, i], B[:, s - i])
        hi, lo = int(W.max()), int(W.min())
        best_hi = hi if best_hi is None else max(best_hi, hi)
        best_lo = lo if best_lo is None else min(best_lo, lo)
    return best_hi, best_lo


def hull_2d(points):
    """Vertices of the convex hull of integer points (Andrew's monotone chain)."""
    pts = sorted(set(map(tuple, points)))
    if len(pts) <= 2:
        return pts

    def cross(o, a, b):
        return (a[0] - o[0]) * (b[1] - o[1]) - (a[1] - o[1]) * (b[0] - o[0])

    lower, upper = [], []
    for q in pts:
        while len(lower) >= 2 and cross(lower[-2], lower[-1], q) <= 0:
            lower.pop()
        lower.append(q)
    for q in reversed(pts):
        while len(upper) >= 2 and cross(upper[-2], upper[-1], q) <= 0:
            upper.pop()
        upper.append(q)
    return lower[:-1] + upper[:-1]


def int32_accumulate(terms):
    """Adds terms in two's-complement int32, as the MFMA accumulator does."""
    acc = 0
    for t in terms:
        acc = (acc + t + 2 ** 31) % 2 ** 32 - 2 ** 31
    return acc
