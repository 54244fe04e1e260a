"""GPU parity of the Chinese remainder reconstruction (Section 5.2, eq. CRT2)
against the oracle's big-integer CRT and the exact integer product.

mmp_crt_reconstruct takes per-modulus residue matrices and writes, entry by
entry, the unique integer below the moduli's product as 64-bit limbs.  The
comparison is exact (integers).
"""

import math
import sys

import numpy as np
import pytest

import mmp_inputs as gen
import oracle
from oracle import crt as ocrt

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
mmp = pytest.importorskip("paper_2601_07508_amd")


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def to_ints(out):
    """(limbs, m, n) int64 tensor of 64-bit limbs -> object array of Python ints."""
    L = out.cpu().numpy().view(np.uint64)
    limbs, m, n = L.shape
    res = np.empty((m, n), dtype=object)
    for i in range(m):
        for j in range(n):
            x = 0
            for w in reversed(range(limbs)):
                x = (x << 64) | int(L[w, i, j])
            res[i, j] = x
    return res


def residues_of(X, moduli):
    """Residue matrices (float64 CUDA) of an object array of integers."""
    return [torch.tensor([[float(int(x) % p) for x in row] for row in X], dtype=torch.float64, device="cuda")
            for p in moduli]


P_MAX = (1 << 52) // 3
MODULI_SETS = {
    "one": [1000003],
    "textbook": [3, 5, 7],
    "composite": [4, 9, 25, 7, 11],
    "two_large": [P_MAX - 10, P_MAX - 11],  # consecutive integers are coprime
    "job_prefix3": gen.crt_primes()[:3],
    "job_16": gen.crt_primes()[:16],
    "job_32": gen.crt_primes(),
    "job_33": gen.crt_primes(count=33),
    "job_64": gen.crt_primes(count=64),
}


@pytest.mark.parametrize("name", sorted(MODULI_SETS))
def test_random_residues_match_oracle(name):
    moduli = MODULI_SETS[name]
    assert all(math.gcd(a, b) == 1 for i, a in enumerate(moduli) for b in moduli[i + 1:])
    M = math.prod(moduli)
    m, n = 9, 7
    raw = gen.uniform_bits(len(moduli), 3, m * n * 8, 63)
    X = np.empty((m, n), dtype=object)
    for e in range(m * n):
        x = 0
        for c in raw[e * 8:(e + 1) * 8]:
            x = (x << 63) | int(c)
        X.flat[e] = x % M
    X[0, 0], X[0, 1], X[1, 0] = 0, M - 1, 1  # edge values
    res = residues_of(X, moduli)
    say("crt reconstruct", name, len(moduli), mmp.crt_limbs(moduli))
    got = to_ints(mmp.crt_reconstruct(res, moduli))
    want = ocrt.crt_matrix([r.cpu().numpy().astype(np.uint64) for r in res], moduli)
    assert np.array_equal(got, want)
    assert np.array_equal(got, X)


def test_strided_inputs_extra_limbs_and_stream():
    moduli = gen.crt_primes()[:5]
    M = math.prod(moduli)
    m, n = 40, 33
    raw = gen.uniform_bits(9, 4, m * n * 4, 62)
    X = np.empty((m, n), dtype=object)
    for e in range(m * n):
        X.flat[e] = ((int(raw[4 * e]) << 186) | (int(raw[4 * e + 1]) << 124) | (int(raw[4 * e + 2]) << 62)
                     | int(raw[4 * e + 3])) % M
    big = [torch.full((m, n + 5), -7.0, dtype=torch.float64, device="cuda") for _ in moduli]
    for b, r in zip(big, residues_of(X, moduli)):
        b[:, :n] = r
    res = [b[:, :n] for b in big]
    limbs = mmp.crt_limbs(moduli) + 2
    out = torch.full((limbs, m, n + 3), 5, dtype=torch.int64, device="cuda")
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        mmp.crt_reconstruct(res, moduli, limbs=limbs, out=out[:, :, :n], stream=s)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    assert np.array_equal(to_ints(out[:, :, :n]), X)
    assert bool(torch.all(out[:, :, n:] == 5))  # columns past n untouched
    assert bool(torch.all(out[limbs - 2:, :, :n] == 0))


@pytest.mark.parametrize("shape", [(37, 29, 50), (64, 65, 130)])
def test_integer_product_end_to_end(shape):
    # uint64 A, B below 2^60 -> mm_modp_crt residues -> reconstruction = A B exactly
    m, n, k = shape
    bits = 60
    primes = gen.crt_primes()
    A = gen.uniform_bits(k, 1, m * k, bits).reshape(m, k)
    B = gen.uniform_bits(k, 2, k * n, bits).reshape(k, n)
    dA = torch.from_numpy(A.astype(np.int64)).cuda()
    dB = torch.from_numpy(B.astype(np.int64)).cuda()
    outs = [torch.empty((m, n), dtype=torch.float64, device="cuda") for _ in primes]
    mmp.mm_modp_crt(dA, dB, primes, outs, bits)
    s = ocrt.moduli_needed(primes, k, bits)
    say("crt end to end", shape, "moduli needed", s)
    few = to_ints(mmp.crt_reconstruct(outs[:s], primes[:s]))
    allp = to_ints(mmp.crt_reconstruct(outs, primes))
    Ai = [[int(x) for x in row] for row in A]
    Bi = [[int(x) for x in row] for row in B]
    exact = np.array([[sum(Ai[i][l] * Bi[l][j] for l in range(k)) for j in range(n)] for i in range(m)],
                     dtype=object)
    assert np.array_equal(few, exact)
    assert np.array_equal(allp, exact)


def test_crt_job_2048_reconstructed():
    # the multimodular job at its full size: 32 residues of the 2048^3 product
    # of 60-bit integers, reconstructed from all 32 moduli and from the
    # shortest prefix eq. CRT2 allows; sampled entries against the exact product
    job = gen.crt_job()
    A, B = job.a(), job.b()
    dA = torch.from_numpy(A.astype(np.int64)).cuda()
    dB = torch.from_numpy(B.astype(np.int64)).cuda()
    outs = [torch.empty((job.m, job.n), dtype=torch.float64, device="cuda") for _ in job.primes]
    mmp.mm_modp_crt(dA, dB, job.primes, outs, job.bits)
    s = ocrt.moduli_needed(job.primes, job.k, job.bits)
    say("crt job reconstruct", s, mmp.crt_limbs(job.primes))
    full = mmp.crt_reconstruct(outs, job.primes)
    few = mmp.crt_reconstruct(outs[:s], job.primes[:s])
    torch.cuda.synchronize()
    lf = few.shape[0]
    assert torch.equal(full[:lf], few) and bool(torch.all(full[lf:] == 0))
    rng = gen.uniform_mod(job.seed, 79, 2 * 128, 1 << 40)
    rows = [int(x) % job.m for x in rng[:128]] + [0, job.m - 1]
    cols = [int(x) % job.n for x in rng[128:]] + [job.n - 1, 0]
    L = few.cpu().numpy().view(np.uint64)
    for i, j in zip(rows, cols):
        exact = sum(int(A[i, l]) * int(B[l, j]) for l in range(job.k))
        got = sum(int(L[w, i, j]) << (64 * w) for w in range(lf))
        assert got == exact, (i, j)
