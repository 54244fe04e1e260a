"""Pins for the oracle's Chinese remainder reconstruction and product counts
(Section 5.2, eq. CRT2, eq. numprodMM, eq. numprodMW).

Checked against things other than the oracle's own formula:
* the classic textbook instance (residues 2, 3, 2 modulo 3, 5, 7 give 23);
* brute force: every X below M is recovered from its residues (X % m_i
  computed directly), for small prime and composite coprime moduli;
* large random X below the product of the CRT job's primes;
* the integer product of small 60-bit matrices (Python integers), recovered
  from the exact oracle's residues once M exceeds k (2^60 - 1)^2;
* eq. numprodMW's relation reproduces the (1, v) bitsize limits of Table
  tab.summary (tests/golden/tab_summary.json), and eq. numprodMM hand values.
"""

import json
import math
import os

import numpy as np
import pytest

import mmp_inputs as gen
import oracle
from oracle import crt

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_textbook_instance():
    assert crt.crt_reconstruct([2, 3, 2], [3, 5, 7]) == 23


@pytest.mark.parametrize("moduli", [[3, 5, 7, 11], [4, 9, 25], [2, 3], [7], [8, 27, 5]])
def test_bruteforce_every_value(moduli):
    M = math.prod(moduli)
    for X in range(M):
        assert crt.crt_reconstruct([X % m for m in moduli], moduli) == X


def test_not_coprime_rejected():
    with pytest.raises(ValueError):
        crt.crt_reconstruct([1, 1], [6, 9])


def test_large_values_job_primes():
    primes = gen.crt_primes()
    M = math.prod(primes)
    raw = gen.uniform_bits(77, 1, 40 * 24, 60)
    for t in range(40):
        # X assembled from 24 seeded 60-bit chunks, reduced below M
        X = 0
        for c in raw[t * 24:(t + 1) * 24]:
            X = (X << 60) | int(c)
        X %= M
        assert crt.crt_reconstruct([X % p for p in primes], primes) == X
    assert crt.crt_reconstruct([p - 1 for p in primes], primes) == M - 1
    assert crt.crt_reconstruct([0] * len(primes), primes) == 0


def _exact_product(A, B):
    A = [[int(x) for x in row] for row in np.asarray(A)]
    B = [[int(x) for x in row] for row in np.asarray(B)]
    m, k, n = len(A), len(B), len(B[0])
    return [[sum(A[i][l] * B[l][j] for l in range(k)) for j in range(n)] for i in range(m)]


@pytest.mark.parametrize("shape", [(3, 4, 5), (6, 2, 17), (1, 1, 1)])
def test_integer_product_from_residues(shape):
    m, n, k = shape
    bits = 60
    primes = gen.crt_primes()
    A = gen.uniform_bits(5, 1, m * k, bits).reshape(m, k)
    B = gen.uniform_bits(5, 2, k * n, bits).reshape(k, n)
    exact = _exact_product(A, B)
    s = crt.moduli_needed(primes, k, bits)
    assert s > 0 and math.prod(primes[:s]) > k * (2**bits - 1) ** 2 >= math.prod(primes[:s - 1])
    for use in (primes[:s], primes):
        res = [oracle.mm_modp(p, A % p, B % p) for p in use]
        got = crt.crt_matrix(res, use)
        assert [[int(x) for x in row] for row in got] == exact


def test_too_few_moduli_gives_the_residue_mod_M():
    # below eq. CRT2's bound the reconstruction is the product mod M, not the product
    A = np.full((1, 4), (1 << 60) - 1, dtype=np.uint64)
    B = np.full((4, 1), (1 << 60) - 1, dtype=np.uint64)
    exact = 4 * ((1 << 60) - 1) ** 2
    primes = gen.crt_primes()[:2]
    res = [oracle.mm_modp(p, A % p, B % p) for p in primes]
    got = int(crt.crt_matrix(res, primes)[0, 0])
    assert got == exact % math.prod(primes) and got != exact


def test_numprod_mw_reproduces_table_limits():
    tab = json.load(open(os.path.join(GOLDEN, "tab_summary.json")))
    limits = dict(zip(map(tuple, tab["variants"]), tab["bitsize_limit_t53"]))
    # eq. numprodMW for (1, v) at lambda = 1: v >= (1 + v) b / 53 up to the
    # table's limit, and not one bit beyond it
    for v in (1, 2, 3, 4):
        b = limits[(1, v)]
        assert v >= (1 + v) * b / 53 and v < (1 + v) * (b + 1) / 53
    # the least product count by bitsize
    assert [crt.numprod_mw(b, 1) for b in (20, 26, 27, 35, 36, 39, 40, 52)] == [1, 1, 2, 2, 3, 3, 4, 4]


def test_numprod_mm_values():
    assert crt.numprod_mm(50, 8192, 1) == 5        # ceil((200 + 26) / 53)
    assert crt.numprod_mm(50, 8192, 512) == 6      # ceil(226 / 44)
    assert crt.numprod_mm(31, 2048, 1) == 3        # ceil((124 + 22) / 53)


def test_multiword_needs_fewer_products_when_u_plus_v_at_most_4():
    # the paper's comparison: (1,2), (1,3), (2,2) need no more products than
    # the multimodular approach
    for lam in (1, 512):
        for b in range(20, 53):
            for k in (2**10, 2**13, 2**20):
                mw = crt.numprod_mw(b, lam)
                if mw and mw <= 4:
                    assert mw <= crt.numprod_mm(b, k, lam), (lam, b, k)
