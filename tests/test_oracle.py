"""Pins for the exact CPU oracle (the definition C = A B mod p, Section 1 eq. goal).

The oracle is checked against things other than itself:
* a second implementation on Python big integers (brute force, tiny sizes);
* algebraic identities of matrix products over Z/pZ;
* closed forms (all entries p - 1 gives k mod p, since (p-1)^2 = 1 mod p);
* Freivalds' check, A (B x) = C x mod p, evaluated with Python integers;
* planted mistakes: plausible wrong oracles fail at least one of these pins.
"""

import numpy as np
import pytest

import mmp_inputs as gen
import oracle
from tests.conftest import PRIMES


def brute(p, A, B):
    """Python big-integer product mod p (independent of the C oracle)."""
    A = [[int(x) for x in row] for row in np.asarray(A)]
    B = [[int(x) for x in row] for row in np.asarray(B)]
    m, k, n = len(A), len(B), len(B[0]) if len(B) else 0
    return np.array([[sum(A[i][l] * B[l][j] for l in range(k)) % p for j in range(n)]
                     for i in range(m)], dtype=np.uint64).reshape(m, n)


def rand(p, r, c, stream, seed=12345):
    return gen.random_matrix(seed, stream, r, c, p)


@pytest.mark.parametrize("p", PRIMES)
@pytest.mark.parametrize("shape", [(1, 1, 1), (2, 3, 5), (5, 8, 3), (8, 8, 8), (3, 1, 7)])
def test_bruteforce_tiny(p, shape):
    m, n, k = shape
    A = rand(p, m, k, 1, seed=p ^ m)
    B = rand(p, k, n, 2, seed=p ^ n)
    assert np.array_equal(oracle.mm_modp(p, A, B), brute(p, A, B))


@pytest.mark.parametrize("p", PRIMES)
def test_identity(p):
    A = rand(p, 7, 9, 1)
    assert np.array_equal(oracle.mm_modp(p, A, np.eye(9, dtype=np.uint64)), A)
    assert np.array_equal(oracle.mm_modp(p, np.eye(7, dtype=np.uint64), A), A)


@pytest.mark.parametrize("p", PRIMES)
def test_linearity_and_scalar(p):
    A = rand(p, 6, 11, 1)
    B1 = rand(p, 11, 5, 2)
    B2 = rand(p, 11, 5, 3)
    Bs = np.array((B1.astype(object) + B2.astype(object)) % p, dtype=np.uint64)
    lhs = oracle.mm_modp(p, A, Bs)
    rhs = (oracle.mm_modp(p, A, B1).astype(object) + oracle.mm_modp(p, A, B2).astype(object)) % p
    assert np.array_equal(lhs, np.array(rhs, dtype=np.uint64))
    c = (p * 2) // 3
    cA = np.array((A.astype(object) * c) % p, dtype=np.uint64)
    rhs = (oracle.mm_modp(p, A, B1).astype(object) * c) % p
    assert np.array_equal(oracle.mm_modp(p, cA, B1), np.array(rhs, dtype=np.uint64))


@pytest.mark.parametrize("p", PRIMES)
def test_associativity_and_transpose(p):
    A = rand(p, 5, 7, 1)
    B = rand(p, 7, 6, 2)
    C = rand(p, 6, 4, 3)
    ab_c = oracle.mm_modp(p, oracle.mm_modp(p, A, B), C)
    a_bc = oracle.mm_modp(p, A, oracle.mm_modp(p, B, C))
    assert np.array_equal(ab_c, a_bc)
    assert np.array_equal(oracle.mm_modp(p, A, B).T,
                          oracle.mm_modp(p, np.ascontiguousarray(B.T), np.ascontiguousarray(A.T)))


@pytest.mark.parametrize("p", PRIMES)
@pytest.mark.parametrize("k", [1, 2, 63, 1000])
def test_closed_forms(p, k):
    full = np.full((3, k), p - 1, dtype=np.uint64)
    fullB = np.full((k, 4), p - 1, dtype=np.uint64)
    assert np.all(oracle.mm_modp(p, full, fullB) == k % p)  # (p-1)^2 = 1 mod p
    ones = np.ones((3, k), dtype=np.uint64)
    assert np.all(oracle.mm_modp(p, ones, np.ones((k, 2), dtype=np.uint64)) == k % p)
    assert np.all(oracle.mm_modp(p, np.zeros((2, k), dtype=np.uint64), fullB) == 0)


def test_headroom_longest_k_largest_p():
    # The longest inner dimension of the workloads (2^17) at the largest
    # 52-bit prime: sum k (p-1)^2 < 2^121 must not overflow.
    p = 4503599627370449
    k = 131072
    A = np.full((2, k), p - 1, dtype=np.uint64)
    B = np.full((k, 2), p - 1, dtype=np.uint64)
    assert np.all(oracle.mm_modp(p, A, B) == k % p)
    x = p - 12345
    A2 = np.full((1, k), x, dtype=np.uint64)
    B2 = np.full((k, 1), x, dtype=np.uint64)
    assert int(oracle.mm_modp(p, A2, B2)[0, 0]) == (k * x * x) % p


def test_unreduced_entries_are_reduced_first():
    p = 2147483647
    A = gen.uniform_bits(3, 1, 4 * 9, 60).reshape(4, 9)
    B = gen.uniform_bits(3, 2, 9 * 5, 60).reshape(9, 5)
    assert np.array_equal(oracle.mm_modp(p, A, B), brute(p, A % np.uint64(p), B % np.uint64(p)))


def test_empty_and_degenerate_shapes():
    p = 33554393
    assert oracle.mm_modp(p, np.zeros((0, 4), np.uint64), np.zeros((4, 3), np.uint64)).shape == (0, 3)
    assert oracle.mm_modp(p, np.zeros((2, 4), np.uint64), np.zeros((4, 0), np.uint64)).shape == (2, 0)
    C = oracle.mm_modp(p, np.zeros((2, 0), np.uint64), np.zeros((0, 3), np.uint64))
    assert C.shape == (2, 3) and np.all(C == 0)


@pytest.mark.parametrize("p", [33554393, 68719476731, 1125899906842597])
def test_freivalds_medium(p):
    m, k, n = 40, 300, 37
    A = rand(p, m, k, 1)
    B = rand(p, k, n, 2)
    C = oracle.mm_modp(p, A, B)
    x = gen.uniform_mod(99, 5, n, p).astype(object)
    Bx = (B.astype(object).dot(x)) % p
    ABx = (A.astype(object).dot(Bx)) % p
    Cx = (C.astype(object).dot(x)) % p
    assert np.array_equal(ABx, Cx)


def test_entries_match_full():
    p = 1099511627689
    A = rand(p, 20, 50, 1)
    B = rand(p, 50, 30, 2)
    C = oracle.mm_modp(p, A, B)
    rows = np.array([0, 19, 7, 3, 19])
    cols = np.array([0, 29, 11, 0, 2])
    assert np.array_equal(oracle.mm_modp_entries(p, A, B, rows, cols), C[rows, cols])


# ----------------------------------------------------------------- planted mistakes
# Each mutant below is a plausible bug in a modular GEMM oracle.  The pins
# above must reject every one of them (the check runs the pin logic on the
# mutant, on the CPU).


def _mut_drop_last_term(p, A, B):
    return brute(p, A[:, :-1], B[:-1, :]) if A.shape[1] > 1 else np.zeros((A.shape[0], B.shape[1]), np.uint64)


def _mut_transposed_b(p, A, B):
    return brute(p, A, np.ascontiguousarray(B.T)) if B.shape[0] == B.shape[1] else brute(p, A, B) + np.uint64(1)


def _mut_u64_wraparound(p, A, B):
    # products and sums in wrapping 64-bit arithmetic, one "% p" at the end
    with np.errstate(over="ignore"):
        acc = np.zeros((A.shape[0], B.shape[1]), dtype=np.uint64)
        for l in range(A.shape[1]):
            acc += A[:, l:l + 1] * B[l:l + 1, :]
    return acc % np.uint64(p)


def _mut_no_reduction(p, A, B):
    return np.array(A.astype(object).dot(B.astype(object)) % (1 << 64), dtype=np.uint64)


def _mut_off_by_one_mod(p, A, B):
    return np.array(A.astype(object).dot(B.astype(object)) % (p - 1), dtype=np.uint64)


def _pins_pass(fn) -> bool:
    p = 1125899906842597
    try:
        A = rand(p, 5, 5, 1)
        B = rand(p, 5, 5, 2)
        if not np.array_equal(fn(p, A, B), brute(p, A, B)):
            return False
        k = 7
        if not np.all(fn(p, np.full((2, k), p - 1, np.uint64), np.full((k, 2), p - 1, np.uint64)) == k % p):
            return False
        if not np.array_equal(fn(p, A, np.eye(5, dtype=np.uint64)), A):
            return False
    except Exception:
        return False
    return True


@pytest.mark.parametrize("mutant", [_mut_drop_last_term, _mut_transposed_b, _mut_u64_wraparound,
                                    _mut_no_reduction, _mut_off_by_one_mod])
def test_pins_reject_planted_mistakes(mutant):
    assert _pins_pass(oracle.mm_modp)
    assert not _pins_pass(mutant)


def test_freivalds_check_catches_one_wrong_entry():
    # the whole-product check the full-size GPU tests use: an exact C passes,
    # and a C with one entry off by one (or with two rows swapped) fails
    from tests import freivalds
    p = 1125899906842597
    A = gen.random_matrix(31, 1, 300, 170, p)
    B = gen.random_matrix(31, 2, 170, 200, p)
    C = oracle.mm_modp(p, A, B)
    freivalds.check(p, A, B, C, seed=5)
    for (r, c) in [(0, 0), (299, 199), (123, 45)]:
        bad = C.copy()
        bad[r, c] = (int(bad[r, c]) + 1) % p
        with pytest.raises(AssertionError, match=f"first row {r}"):
            freivalds.check(p, A, B, bad, seed=5)
    swapped = C.copy()
    swapped[[10, 11]] = swapped[[11, 10]]
    with pytest.raises(AssertionError, match="2 rows"):
        freivalds.check(p, A, B, swapped, seed=5)
