"""Pins for the CPU emulation of the paper's floating-point algorithms.

* Alg. 1 and Alg. 2 agree with integer "%" on the input ranges of
  Prop. fpModularReductionFMA and Prop. Joris (boundary values included).
* Alg. 4 reconstructs its input exactly, with words below alpha.
* Algs. 5 and 6 with the block size of Prop. UVMW equal the definition oracle.
* Negative control: one more than the paper's block size gives a wrong result
  on worst-case inputs, so the bound is tight and the emulation really
  rounds.
* Table tab.summary: the bitsize limits are reproduced exactly.
"""

import json
import math
import os

import numpy as np
import pytest

import mmp_inputs as gen
import oracle
from oracle import paper_algorithms as pa
from tests.conftest import PRIMES

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_fma_is_correctly_rounded():
    # 2^53 + 1 is a tie between 2^53 and 2^53 + 2: round to even gives 2^53.
    assert pa.fma(2.0**26, 2.0**27, 1.0) == 2.0**53
    assert pa.fma(2.0**26, 2.0**27, 3.0) == 2.0**53 + 4
    # the exact product is kept before the single rounding
    x = 2.0**30 + 1
    assert pa.fma(x, x, -(x * x)) == 1.0


def test_iroot_ceil_bruteforce():
    for p in [5, 7, 8, 9, 26, 27, 28, 63, 64, 65, 1000, 4096, 4097] + PRIMES:
        for u in range(1, 6):
            a = pa.iroot_ceil(p, u)
            assert a ** u >= p and (a == 1 or (a - 1) ** u < p)


@pytest.mark.parametrize("p", PRIMES[:-1])  # Alg. 1 needs p < 2^(t-1)
def test_alg1_fmod_range(p):
    q = 1.0 / p
    xmax = min(2**53, 2**51 * p)  # integers in F, x <= 2^(t-2) p
    xs = [0, 1, p - 1, p, p + 1, 2 * p - 1, 2 * p, xmax, xmax - 1, xmax - p]
    xs += [int(v) for v in gen.uniform_mod(p, 1, 2000, xmax + 1)]
    for x in xs:
        assert pa.fmod_alg1(float(x), float(p), q) == x % p


@pytest.mark.parametrize("p", PRIMES[:-1])
def test_alg2_mulmod_range(p):
    q = 1.0 / p
    bound = (2**52 * p) // 3  # x y <= 2^(t-1)/3 p
    ys = [0, 1, p - 1] + [int(v) for v in gen.uniform_mod(p, 2, 300, p)]
    alpha = pa.iroot_ceil(p, 2)
    for y in ys:
        for x in (1, 2, alpha, alpha - 1, p - 1, (p + 1) // 2):
            if x * y <= bound:
                assert pa.mulmod_alg2(float(x), float(y), float(p), q) == (x * y) % p


@pytest.mark.parametrize("p", PRIMES)
@pytest.mark.parametrize("u", [1, 2, 3, 4])
def test_alg4_decomposition(p, u):
    M = [[float(x) for x in gen.uniform_mod(p, u, 40, p)] + [0.0, float(p - 1)]]
    alpha, words = pa.mw_decompose_alg4(M, p, u)
    assert alpha == pa.iroot_ceil(p, u)
    for c in range(len(M[0])):
        assert sum(int(words[i][0][c]) * alpha**i for i in range(u)) == int(M[0][c])
        for i in range(u):
            w = words[i][0][c]
            assert w == int(w) and 0 <= w <= alpha - 1  # tight bound: words < alpha


def _tiny(p, m, k, n, seed):
    A = gen.random_matrix(seed, 1, m, k, p)
    B = gen.random_matrix(seed, 2, k, n, p)
    return A, B


CASES = [  # (p, u, v): a variant inside its bitsize limit
    (33554393, 1, 1), (67108859, 1, 1), (2147483647, 1, 2), (34359738337, 1, 2), (68719476731, 1, 3),
    (1099511627689, 2, 2), (1099511627689, 1, 4), (1125899906842597, 2, 2),
    (1125899906842597, 2, 3), (4503599627370449, 2, 3), (2147483647, 2, 1),
]


@pytest.mark.parametrize("p,u,v", CASES)
def test_alg5_alg6_equal_definition(p, u, v):
    lam = pa.block_size(p, u, v)
    assert lam >= 1
    for fill in ("uniform", "pmax"):
        m, k, n = 3, 2 * lam + 3 if lam < 20 else 9, 2
        if fill == "uniform":
            A, B = _tiny(p, m, k, n, p + u + v)
        else:
            A = np.full((m, k), p - 1, np.uint64)
            B = np.full((k, n), p - 1, np.uint64)
        want = oracle.mm_modp(p, A, B)
        Af = [[float(x) for x in row] for row in A]
        Bf = [[float(x) for x in row] for row in B]
        got5 = np.array(pa.mw_product_alg5(Af, Bf, p, u, v, lam), dtype=np.uint64)
        got6 = np.array(pa.mw_product_alg6(Af, Bf, p, u, v, lam), dtype=np.uint64)
        assert np.array_equal(got5, want)
        assert np.array_equal(got6, want)


@pytest.mark.parametrize("p,lam", [(33554393, 8), (67108859, 2)])
def test_alg3_single_word_bound_is_tight(p, lam):
    """Prop. blockProduct with eq. lambda-sw: lam works, lam + 1 fails on all-(p-1) inputs."""
    assert pa.block_size(p, 1, 1) == lam
    k = 64
    A = [[float(p - 1)] * k]
    B = [[float(p - 1)] for _ in range(k)]
    want = k % p
    assert pa.block_product_alg3([[0.0]], A, B, p, lam)[0][0] == want
    assert pa.block_product_alg3([[0.0]], A, B, p, lam + 1)[0][0] != want


def test_alg5_22_bound_is_tight():
    """(2,2) at p = 2^50 - 27: lambda = 7 is exact, 8 fails with maximal words."""
    p = 1125899906842597
    lam = pa.block_size(p, 2, 2)
    assert lam == 7
    alpha = pa.iroot_ceil(p, 2)
    x = p - 1  # high word alpha - 1 (the largest a word can be)
    assert x // alpha == alpha - 1
    k = 64
    A = [[float(x)] * k]
    B = [[float(x)] for _ in range(k)]
    want = (k * x * x) % p
    assert pa.mw_product_alg5(A, B, p, 2, 2, lam)[0][0] == want
    assert pa.mw_product_alg5(A, B, p, 2, 2, lam + 1)[0][0] != want


def test_table_summary_bitsize_limits():
    g = json.load(open(os.path.join(GOLDEN, "tab_summary.json")))
    for (u, v), flops, limit in zip(g["variants"], g["normalized_flops"], g["bitsize_limit_t53"]):
        assert u * v == flops
        assert pa.bitsize_limit(u, v) == limit, (u, v)
        assert pa.bitsize_limit(v, u) == limit


def test_single_word_limit_is_p_times_p_minus_1():
    # Corollary after eq. lambda-sw: lambda >= 1 exactly when p (p - 1) <= 2^t.
    pmax = max(p for p in range(94906200, 94906300) if p * (p - 1) <= 2**53)
    assert pa.block_size(pmax, 1, 1) == 1 and pa.block_size(pmax + 1, 1, 1) == 0
    assert abs(math.log2(pmax) - 26.5) < 0.01
