"""The benchmark workloads at full size, every output checked.

Each product runs through the same entry point and plan as the benchmark.
Every output is checked to be an integer in [0, p), and every output enters
Freivalds' check with the oracle as the checker: for seeded random vectors
x, A (B x) and C x mod p are formed by the oracle (products with one column)
and must agree.  A wrong entry of C makes its row of C x wrong except with
probability 1/p per trial (p prime), and two trials run.  The oracle also
recomputes whole sampled rows and columns plus random entries exactly; the
512^3 workload is small enough to compare in full.
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


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _compute(prob, **opts):
    A = prob.a()
    B = prob.b()
    dA = torch.from_numpy(A.astype(np.float64)).cuda()
    dB = torch.from_numpy(B.astype(np.float64)).cuda()
    C = torch.full((prob.m, prob.n), -1.0, dtype=torch.float64, device="cuda")
    mmp.mm_modp_async(dA, dB, C, prob.p, prob.u, prob.v, **opts)
    torch.cuda.synchronize()
    del dA, dB
    return A, B, C


def _check_sampled(prob, A, B, C, nrows=2, ncols=2, nrand=512):
    p = prob.p
    assert bool(torch.all((C >= 0) & (C < p) & (C == torch.floor(C))))
    assert not bool(torch.any(torch.signbit(C)))
    rng = gen.uniform_mod(prob.seed, 77, nrows + ncols + 2 * nrand, 1 << 62)
    rows = [int(x) % prob.m for x in rng[:nrows]] + [prob.m - 1]
    cols = [int(x) % prob.n for x in rng[nrows:nrows + ncols]] + [prob.n - 1]
    rr, cc = [], []
    for r in rows:
        rr += [r] * prob.n
        cc += list(range(prob.n))
    for c in cols:
        rr += list(range(prob.m))
        cc += [c] * prob.m
    rand = rng[nrows + ncols:]
    rr += [int(x) % prob.m for x in rand[:nrand]]
    cc += [int(x) % prob.n for x in rand[nrand:]]
    rr = np.array(rr, dtype=np.int64)
    cc = np.array(cc, dtype=np.int64)
    want = oracle.mm_modp_entries(p, A, B, rr, cc).astype(np.float64)
    got = C[torch.from_numpy(rr).cuda(), torch.from_numpy(cc).cuda()].cpu().numpy()
    bad = np.nonzero(got != want)[0]
    assert bad.size == 0, f"{bad.size} sampled mismatches, first ({rr[bad[0]]},{cc[bad[0]]})"


def _freivalds(p, A, B, C, seed):
    freivalds.check(p, A, B, C.cpu().numpy(), seed)


def test_square_512_b25_full():
    (prob,) = gen.config_problems(1)
    say("config", prob.tag, mmp.plan(prob.p, prob.m, prob.n, prob.k, prob.u, prob.v))
    A, B, C = _compute(prob)
    want = oracle.mm_modp(prob.p, A, B).astype(np.float64)
    assert np.array_equal(C.cpu().numpy(), want)


@pytest.mark.parametrize("idx", [0, 1])
def test_square_4096(idx):
    prob = gen.config_problems(2)[idx]
    say("config", prob.tag, mmp.plan(prob.p, prob.m, prob.n, prob.k, prob.u, prob.v))
    A, B, C = _compute(prob)
    _check_sampled(prob, A, B, C)
    _freivalds(prob.p, A, B, C, prob.seed)


# 8192^3 at p = 2^50 - 27: (2,2) words under the paper's bound (the benchmark's
# headline), the same under the extended and centered bounds, and the INT8
# digits; uniform entries and the all-(p-1) worst case
FORMS_8192 = {"paper": {}, "extended": {"extended_block": True}, "centered": {"centered_words": True},
              "int8": {"form": 2}}


@pytest.mark.parametrize("form", list(FORMS_8192))
@pytest.mark.parametrize("idx", [0, 1])
def test_square_8192_b50_22(idx, form):
    prob = gen.config_problems(3)[idx]
    opts = FORMS_8192[form]
    u, v = (0, 0) if form == "int8" else (prob.u, prob.v)
    say("config", prob.tag, form, mmp.plan(prob.p, prob.m, prob.n, prob.k, u, v, **opts))
    A, B = prob.a(), prob.b()
    dA = torch.from_numpy(A.astype(np.float64)).cuda()
    dB = torch.from_numpy(B.astype(np.float64)).cuda()
    C = torch.full((prob.m, prob.n), -1.0, dtype=torch.float64, device="cuda")
    mmp.mm_modp_async(dA, dB, C, prob.p, u, v, **opts)
    torch.cuda.synchronize()
    del dA, dB
    if prob.fill == "pmax":
        # (p-1)^2 = 1 mod p: every entry is k mod p
        assert bool(torch.all(C == float(prob.k % prob.p)))
    else:
        _check_sampled(prob, A, B, C, nrows=1, ncols=1, nrand=256)
        _freivalds(prob.p, A, B, C, prob.seed)


@pytest.mark.parametrize("idx", list(range(8)))
def test_sweep_shapes(idx):
    prob = gen.config_problems(4)[idx]
    say("config", prob.tag, mmp.plan(prob.p, prob.m, prob.n, prob.k, prob.u, prob.v))
    A, B, C = _compute(prob)
    _check_sampled(prob, A, B, C, nrows=1, ncols=1, nrand=512)
    _freivalds(prob.p, A, B, C, prob.seed)


def test_crt_2048_32_primes():
    job = gen.crt_job()
    A, B = job.a(), job.b()
    dA = torch.from_numpy(A.astype(np.int64)).cuda()
    dB = torch.from_numpy(B.astype(np.int64)).cuda()
    outs = [torch.full((job.m, job.n), -1.0, dtype=torch.float64, device="cuda") for _ in job.primes]
    say("crt config", job.m, job.n, job.k, len(job.primes), [p.bit_length() for p in job.primes])
    mmp.mm_modp_crt(dA, dB, job.primes, outs, job.bits)
    torch.cuda.synchronize()
    rng = gen.uniform_mod(job.seed, 78, 2 * 256, 1 << 40)
    rr = np.array([int(x) % job.m for x in rng[:256]] + [0, job.m - 1], dtype=np.int64)
    cc = np.array([int(x) % job.n for x in rng[256:]] + [job.n - 1, 0], dtype=np.int64)
    for p, C in zip(job.primes, outs):
        assert bool(torch.all((C >= 0) & (C < p) & (C == torch.floor(C))))
        want = oracle.mm_modp_entries(p, A, B, rr, cc).astype(np.float64)
        got = C[torch.from_numpy(rr).cuda(), torch.from_numpy(cc).cuda()].cpu().numpy()
        assert np.array_equal(got, want), p
        _freivalds(p, A, B, C, job.seed)  # the oracle reduces the integer entries mod p


@pytest.mark.parametrize("bits", [26, 50])
def test_unbalanced_10923x32768x32(bits):
    # the paper's second workload: both forms and the server with A resident
    prob = gen.unbalanced_problem(bits)
    A, B = prob.a(), prob.b()
    dA = torch.from_numpy(A.astype(np.float64)).cuda()
    dB = torch.from_numpy(B.astype(np.float64)).cuda()
    outs = []
    for form in (1, 2):
        C = torch.full((prob.m, prob.n), -1.0, dtype=torch.float64, device="cuda")
        say("unbalanced", bits, "form", form, mmp.plan(prob.p, prob.m, prob.n, prob.k, form=form))
        mmp.mm_modp_async(dA, dB, C, prob.p, form=form)
        outs.append(C)
    C = torch.full((prob.m, prob.n), -1.0, dtype=torch.float64, device="cuda")
    with mmp.Server(hbm_budget=32 << 30, max_slots=4) as srv:
        srv.register_operand(dA, prob.p, 0)
        assert srv.wait(srv.submit(dA, dB, C, prob.p), 120.0)[0] == 0
    outs.append(C)
    # A's digit planes prepared once, reused by direct calls
    pa = mmp.prepare_operand(dA, prob.p, 0)
    for _ in range(2):
        C = torch.full((prob.m, prob.n), -1.0, dtype=torch.float64, device="cuda")
        mmp.mm_modp_async(dA, dB, C, prob.p, prepared_a=pa)
        outs.append(C)
    torch.cuda.synchronize()
    assert all(torch.equal(outs[0], c) for c in outs[1:])
    _check_sampled(prob, A, B, outs[0], nrows=2, ncols=1, nrand=256)
    _freivalds(prob.p, A, B, outs[0], prob.seed)
