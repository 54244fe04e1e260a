"""The paper's floating-point algorithms, emulated step by step on the CPU.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Every quantity is an IEEE binary64 value held in a Python ``float``; Python's
float arithmetic is binary64 with round-to-nearest-even, which is the model
of Section 2 (t = 53, unit roundoff 2^-t, correctly rounded fma).  ``fma`` is
formed exactly with rationals and rounded once.  Matrices are lists of lists
of floats; these routines are meant for tiny matrices only.

Parameter formulas (exact integer arithmetic on Python ints):

* alpha = ceil(p^(1/u)) (Alg. 4, first step), as the smallest integer a with
  a^u >= p;
* block size lambda: eq. lambda-sw for (u, v) = (1, 1) with entries in F_p,
  else eq. cAcB (Prop. UVMW): the largest lambda with
  lambda * alpha * beta + p - 1 <= 2^t.
"""

from __future__ import annotations

import math
from fractions import Fraction

T_BITS = 53
TWO_T = 1 << T_BITS


# ------------------------------------------------------------- scalar helpers


def fma(a: float, b: float, c: float) -> float:
    """Correctly rounded a*b + c (Section 2, the fma assumption)."""
    if a == int(a) and b == int(b) and c == int(c):
        return float(int(a) * int(b) + int(c))  # int -> float rounds to nearest even
    return float(Fraction(a) * Fraction(b) + Fraction(c))


def iroot_ceil(p: int, u: int) -> int:
    """Smallest integer a >= 1 with a**u >= p (that is, ceil(p^(1/u)))."""
    if u == 1:
        return p
    a = max(1, int(round(p ** (1.0 / u))))
    while a ** u < p:
        a += 1
    while a > 1 and (a - 1) ** u >= p:
        a -= 1
    return a


def block_size(p: int, u: int, v: int, t: int = T_BITS) -> int:
    """The paper's block size lambda for a (u, v)-product (0 if none works).

    (1,1): eq. lambda-sw, floor((2^t - p + 1) / (p - 1)^2).
    otherwise: the largest lambda with lambda*alpha*beta + p - 1 <= 2^t (eq. cAcB).
    """
    two_t = 1 << t
    if u == 1 and v == 1:
        return max(0, (two_t - p + 1) // ((p - 1) ** 2))
    a, b = iroot_ceil(p, u), iroot_ceil(p, v)
    return max(0, (two_t - p + 1) // (a * b))


def bitsize_limit(u: int, v: int, t: int = T_BITS) -> int:
    """Largest b such that every prime of bitsize b admits lambda >= 1.

    This reads the third row of Table tab.summary: the limit on bitsize(p)
    is the largest b for which the block-size condition holds with
    lambda = 1 for every p < 2^b (and p < 2^(t-1), which Alg. 1 needs).
    The admissible p form an interval [5, p_max], so the limit is
    floor(log2(p_max + 1)).
    """
    lo, hi = 5, (1 << (t - 1)) - 1  # Prop. UVMW also needs p < 2^(t-1)
    if block_size(lo, u, v, t) < 1:
        return 0
    while lo < hi:  # largest p with lambda >= 1 (monotone in p)
        mid = (lo + hi + 1) // 2
        if block_size(mid, u, v, t) >= 1:
            lo = mid
        else:
            hi = mid - 1
    return (lo + 1).bit_length() - 1


# ------------------------------------------------------------- Algorithm 1


def fmod_alg1(x: float, p: float, q: float) -> float:
    """Alg. 1: d = x mod p with q = fl(1/p) (Section 2.1)."""
    b = x * q
    c = math.floor(b)
    d = fma(-float(c), p, x)
    if d >= p:
        d = d - p
    if d < 0:
        d = d + p
    return d


# ------------------------------------------------------------- Algorithm 2


def mulmod_alg2(x: float, y: float, p: float, q: float) -> float:
    """Alg. 2: e = x*y mod p through the error-free product h + l = x*y."""
    h = x * y
    l = fma(x, y, -h)
    b = h * q
    c = math.floor(b)
    d = fma(-float(c), p, h)
    e = d + l
    if e >= p:
        e = e - p
    if e < 0:
        e = e + p
    return e


# ------------------------------------------------------------- Algorithm 3


def block_product_alg3(C, A, B, p: int, lam: int):
    """Alg. 3: C = C + A B mod p, reducing C after every block of lam columns.

    The block product C + A_j B_j is formed entry by entry as a sequential
    chain of fma operations in increasing index order; when the block size
    satisfies Prop. blockProduct every intermediate value is an exactly
    representable integer, so this order is as good as any other.
    """
    m, k, n = len(A), len(B), len(B[0]) if B else 0
    pf = float(p)
    q = 1.0 / pf
    C = [row[:] for row in C]
    for j0 in range(0, k, lam):
        j1 = min(k, j0 + lam)
        for i in range(m):
            for c in range(n):
                acc = C[i][c]
                for l in range(j0, j1):
                    acc = fma(A[i][l], B[l][c], acc)
                C[i][c] = fmod_alg1(acc, pf, q)
    return C


# ------------------------------------------------------------- Algorithm 4


def mw_decompose_alg4(M, p: int, u: int):
    """Alg. 4: alpha = ceil(p^(1/u)) and words M_0..M_{u-1} with M = sum alpha^i M_i."""
    alpha = iroot_ceil(p, u)
    af = float(alpha)
    T = [row[:] for row in M]
    words = []
    for _ in range(u - 1):
        R = [[float(math.floor(x / af)) for x in row] for row in T]
        Mi = [[T[r][c] - af * R[r][c] for c in range(len(T[r]))] for r in range(len(T))]
        words.append(Mi)
        T = R
    words.append(T)
    return alpha, words


# ------------------------------------------------------------- Algorithms 5, 6


def _scale_mod(gamma: float, C, p: float, q: float):
    return [[mulmod_alg2(gamma, x, p, q) for x in row] for row in C]


def _powmod_alg2(base: int, e: int, p: float, q: float) -> float:
    """base^e mod p by repeated Alg. 2 with a reduction at every step."""
    r = 1.0
    b = float(base % int(p))
    for _ in range(e):
        r = mulmod_alg2(r, b, p, q)
    return r


def mw_product_alg5(A, B, p: int, u: int, v: int, lam: int):
    """Alg. 5 (in place, p prime): C = A B mod p from u x v word products."""
    pf = float(p)
    q = 1.0 / pf
    alpha, Aw = mw_decompose_alg4(A, p, u)
    beta, Bw = mw_decompose_alg4(B, p, v)
    m, n = len(A), len(B[0])
    C = [[0.0] * n for _ in range(m)]
    for i in range(u):
        for j in range(v):
            gamma = mulmod_alg2(_powmod_alg2(alpha, i, pf, q), _powmod_alg2(beta, j, pf, q), pf, q)
            delta = float(pow(int(gamma), -1, p))  # modular inverse (p prime)
            C = _scale_mod(delta, C, pf, q)
            C = block_product_alg3(C, Aw[i], Bw[j], p, lam)
            C = _scale_mod(gamma, C, pf, q)
    return C


def mw_product_alg6(A, B, p: int, u: int, v: int, lam: int):
    """Alg. 6 (concatenated): A_i [B_0 ... B_{v-1}] per i, then scale and add."""
    pf = float(p)
    q = 1.0 / pf
    alpha, Aw = mw_decompose_alg4(A, p, u)
    beta, Bw = mw_decompose_alg4(B, p, v)
    m, n = len(A), len(B[0])
    C = [[0.0] * n for _ in range(m)]
    Bcat = [sum((Bw[j][r] for j in range(v)), []) for r in range(len(B))]  # k x (n v)
    for i in range(u):
        Tcat = block_product_alg3([[0.0] * (n * v) for _ in range(m)], Aw[i], Bcat, p, lam)
        for j in range(v):
            gamma = mulmod_alg2(_powmod_alg2(alpha, i, pf, q), _powmod_alg2(beta, j, pf, q), pf, q)
            Tj = [row[j * n:(j + 1) * n] for row in Tcat]
            Tj = _scale_mod(gamma, Tj, pf, q)
            C = [[fmod_alg1(C[r][c] + Tj[r][c], pf, q) for c in range(n)] for r in range(m)]
    return C
