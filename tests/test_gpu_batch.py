"""Batched and multi-modular (CRT) products on the GPU, and graph capture.

Every output is compared with the exact oracle (tolerance 0); batched
results must also be identical to the same products run one by one.
"""

import sys

import numpy as np
import pytest

import mmp_inputs as gen
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
mmp = pytest.importorskip("paper_2601_07508_amd")


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def dev64(x):
    return torch.from_numpy(np.ascontiguousarray(x).astype(np.int64)).cuda()


def mixed_jobs(seed=1, count=20):
    """Uneven products: log-uniform dims, bitsizes 20..52, some with explicit words."""
    reqs = gen.serve_stream(count, 1.0, seed=seed, dim_lo=1, dim_hi=300)
    from oracle import paper_algorithms as pa
    out = []
    for i, r in enumerate(reqs):
        pr = r.problem
        u, v = 0, 0
        if i % 3 == 1:
            # explicit words where the paper's bound admits them
            for cand in ((1, 1), (1, 2), (2, 2), (2, 3)):
                if pa.block_size(pr.p, *cand) >= 1:
                    u, v = cand
                    break
        out.append((pr, u, v))
    return out


def test_batched_mixed_equals_oracle_and_single_calls():
    jobs = mixed_jobs()
    tensors = []
    for pr, u, v in jobs:
        A, B = pr.a(), pr.b()
        tensors.append((A, B, dev(A), dev(B), torch.full((pr.m, pr.n), -1.0, dtype=torch.float64, device="cuda")))
    batch = [(dA, dB, C, pr.p, u, v) for (pr, u, v), (_, _, dA, dB, C) in zip(jobs, tensors)]
    say("batched", [(pr.m, pr.n, pr.k, pr.p.bit_length(), u, v) for pr, u, v in jobs])
    mmp.mm_modp_batched(batch)
    torch.cuda.synchronize()
    for (pr, u, v), (A, B, dA, dB, C) in zip(jobs, tensors):
        want = oracle.mm_modp(pr.p, A, B).astype(np.float64)
        got = C.cpu().numpy()
        assert np.array_equal(got, want), (pr.m, pr.n, pr.k, pr.p, u, v)
        single = mmp.mm_modp(dA, dB, pr.p, u, v)
        torch.cuda.synchronize()
        assert torch.equal(single, C)


def test_batched_more_jobs_than_one_launch_and_degenerate():
    p = 1125899906842597
    jobs, host = [], []
    for i in range(40):  # 40 products of one configuration: three launches
        m, n, k = 17 + i, 9 + 2 * i, 31 + 3 * i
        A = gen.random_matrix(i, 1, m, k, p)
        B = gen.random_matrix(i, 2, k, n, p)
        C = torch.empty((m, n), dtype=torch.float64, device="cuda")
        jobs.append((dev(A), dev(B), C, p, 2, 2))
        host.append((A, B))
    z = torch.full((3, 4), 5.0, dtype=torch.float64, device="cuda")  # k = 0 -> zeros
    jobs.append((torch.zeros((3, 0), dtype=torch.float64, device="cuda"),
                 torch.zeros((0, 4), dtype=torch.float64, device="cuda"), z, p, 0, 0))
    mmp.mm_modp_batched(jobs)
    torch.cuda.synchronize()
    for (dA, dB, C, *_), (A, B) in zip(jobs[:40], host):
        assert np.array_equal(C.cpu().numpy(), oracle.mm_modp(p, A, B).astype(np.float64))
    assert torch.all(z == 0)


def test_batched_rejects_overlapping_outputs():
    p = 33554393
    A = torch.zeros((4, 4), dtype=torch.float64, device="cuda")
    C = torch.zeros((8, 4), dtype=torch.float64, device="cuda")
    with pytest.raises(mmp.MmpError) as e:
        mmp.mm_modp_batched([(A, A, C[:4], p, 1, 1), (A, A, C[2:6], p, 1, 1)])
    assert e.value.status == -1


def _crt_check(A, B, primes, outs, bits):
    for p, C in zip(primes, outs):
        want = oracle.mm_modp(p, A, B).astype(np.float64)
        got = C.cpu().numpy()
        assert np.array_equal(got, want), p


@pytest.mark.parametrize("bits,shape", [(60, (130, 96, 257)), (20, (65, 70, 1000)), (62, (40, 33, 64)),
                                        (8, (20, 20, 20)), (15, (33, 20, 100)), (55, (40, 70, 300))])
def test_crt_fast_path(bits, shape):
    m, n, k = shape
    primes = gen.crt_primes(count=32)
    A = gen.uniform_bits(bits, 1, m * k, bits).reshape(m, k)
    B = gen.uniform_bits(bits, 2, k * n, bits).reshape(k, n)
    outs = [torch.full((m, n), -1.0, dtype=torch.float64, device="cuda") for _ in primes]
    say("crt", bits, shape)
    mmp.mm_modp_crt(dev64(A), dev64(B), primes, outs, bits)
    torch.cuda.synchronize()
    _crt_check(A, B, primes, outs, bits)


# With p = 5 in the launch the epilogue reduces every group of three digit
# weights first; when every modulus is at least 65793 k D 2^14 / (2^27 - 2)
# (8225 here: k = 128, D = 8) it folds the groups directly.
@pytest.mark.parametrize("primes", [[4503599627370449, 1125899906842597, 2147483647, 5],
                                    [4503599627370449, 1125899906842597, 2147483647, 8231]])
def test_crt_extreme_entries(primes):
    bits = 62
    m, n, k = 16, 16, 128
    top = (1 << bits) - 1
    vals = np.array([top, 0, top - 1, 1 << 61, (1 << 61) - 1, 0x7F7F7F7F7F7F7F7F & top], dtype=np.uint64)
    A = vals[np.arange(m * k) % len(vals)].reshape(m, k)
    B = vals[(np.arange(k * n) * 5 + 1) % len(vals)].reshape(k, n)
    assert all(gen.is_prime(p) for p in primes)
    outs = [torch.empty((m, n), dtype=torch.float64, device="cuda") for _ in primes]
    mmp.mm_modp_crt(dev64(A), dev64(B), primes, outs, bits)
    torch.cuda.synchronize()
    _crt_check(A, B, primes, outs, bits)


# Widths 8D - 1 need D + 1 signed digits (2^(8D-1) - 1 > 127 (256^D - 1) / 255):
# the entries just below 2^bits, and the witnesses of the integer block's
# extremes over one whole block (k = K, the fast path's limit).
@pytest.mark.parametrize("bits", [15, 23, 55, 62])
def test_crt_widest_entries_and_block_limit(bits):
    b = mmp.int8_bound(entry_bits=bits)
    K = b["kblock"]
    primes = [4503599627370449, 1125899906842597, 2147483647, 65521]
    top = (1 << bits) - 1
    m, n = 8, 12
    vals = np.array([top, top - 1, top - 127, (1 << (bits - 1)), 0], dtype=np.uint64)
    for k, A, B in ((300, vals[np.arange(m * 300) % 5].reshape(m, 300), vals[(np.arange(300 * n) * 3) % 5].reshape(300, n)),
                    (K, np.full((m, K), b["witness_max"][0], dtype=np.uint64),
                     np.full((K, n), b["witness_max"][1], dtype=np.uint64))):
        say("crt widest", bits, k)
        outs = [torch.full((m, n), -1.0, dtype=torch.float64, device="cuda") for _ in primes]
        mmp.mm_modp_crt(dev64(A), dev64(B), primes, outs, bits)
        torch.cuda.synchronize()
        _crt_check(A, B, primes, outs, bits)


def test_crt_long_k_falls_back_to_reduced_products():
    bits = 60
    m, n, k = 24, 20, 20000  # beyond one exact int32 block of 8-digit integers
    primes = gen.crt_primes(count=5)
    A = gen.uniform_bits(3, 1, m * k, bits).reshape(m, k)
    B = gen.uniform_bits(3, 2, k * n, bits).reshape(k, n)
    outs = [torch.empty((m, n), dtype=torch.float64, device="cuda") for _ in primes]
    mmp.mm_modp_crt(dev64(A), dev64(B), primes, outs, bits)
    torch.cuda.synchronize()
    _crt_check(A, B, primes, outs, bits)


def test_crt_validates_entry_bound():
    A = torch.full((4, 4), 1 << 40, dtype=torch.int64, device="cuda")
    outs = [torch.empty((4, 4), dtype=torch.float64, device="cuda")]
    with pytest.raises(mmp.MmpError) as e:
        mmp.mm_modp_crt(A, A, [33554393], outs, 40, validate_entries=True)
    assert e.value.status == -3
    mmp.mm_modp_crt(A, A, [33554393], outs, 41, validate_entries=True)


def test_graph_capture_crt_and_batch_replays():
    bits = 60
    m, n, k = 96, 80, 300
    primes = gen.crt_primes(count=8)
    A = gen.uniform_bits(5, 1, m * k, bits).reshape(m, k)
    B = gen.uniform_bits(5, 2, k * n, bits).reshape(k, n)
    dA, dB = dev64(A), dev64(B)
    outs = [torch.zeros((m, n), dtype=torch.float64, device="cuda") for _ in primes]
    ws = torch.empty(mmp.workspace_crt(m, n, k, bits, len(primes)), dtype=torch.uint8, device="cuda")
    # batched products that use the INT8 form need a workspace too
    p = 1099511627689
    bA = gen.random_matrix(9, 1, 128, 200, p)
    bB = gen.random_matrix(9, 2, 200, 64, p)
    bC = torch.zeros((128, 64), dtype=torch.float64, device="cuda")
    bC2 = torch.zeros((128, 32), dtype=torch.float64, device="cuda")
    bjobs = [(dev(bA), dev(bB), bC, p, 0, 0), (dev(bA), dev(bB)[:, :32].contiguous(), bC2, p, 0, 0)]
    bws = torch.empty(max(mmp.workspace_batched(bjobs, form=mmp.FORM_INT8_WORDS), 1), dtype=torch.uint8,
                      device="cuda")
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):  # warm-up outside the graph (pool, kernels loaded)
        mmp.mm_modp_crt(dA, dB, primes, outs, bits, stream=s, workspace=ws)
        mmp.mm_modp_batched(bjobs, stream=s, workspace=bws, form=mmp.FORM_INT8_WORDS)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        mmp.mm_modp_crt(dA, dB, primes, outs, bits, stream=s, workspace=ws)
        mmp.mm_modp_batched(bjobs, stream=s, workspace=bws, form=mmp.FORM_INT8_WORDS)
    want = [oracle.mm_modp(pp, A, B).astype(np.float64) for pp in primes]
    wantb = oracle.mm_modp(p, bA, bB).astype(np.float64)
    for rep in range(3):
        for C in outs:
            C.fill_(-1.0)
        bC.fill_(-1.0)
        bC2.fill_(-1.0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for C, w in zip(outs, want):
            assert np.array_equal(C.cpu().numpy(), w), rep
        assert np.array_equal(bC.cpu().numpy(), wantb), rep
        assert np.array_equal(bC2.cpu().numpy(), wantb[:, :32]), rep
        # eager work between replays
        x = torch.randn(1000, device="cuda").sum()
        torch.cuda.synchronize()
        del x


def test_autotune_picks_a_correct_plan():
    for p, shape in [(1125899906842597, (256, 256, 512)), (8388593, (512, 128, 300)), (68719476731, (200, 300, 700))]:
        m, n, k = shape
        mmp.tune_cache_clear()
        best, tried = mmp.autotune(p, m, n, k)
        say("autotune", p, shape, tried, best)
        assert tried >= 2
        pl = mmp.plan(p, m, n, k)  # AUTO now follows the tuned choice
        assert (pl["form"], pl["u"], pl["v"], pl["tile"]) == (best["form"], best["u"], best["v"], best["tile"])
        A = gen.random_matrix(4, 1, m, k, p)
        B = gen.random_matrix(4, 2, k, n, p)
        C = mmp.mm_modp(dev(A), dev(B), p)
        torch.cuda.synchronize()
        assert np.array_equal(C.cpu().numpy(), oracle.mm_modp(p, A, B).astype(np.float64))
    mmp.tune_cache_clear()


def test_graph_capture_reconstruction_and_prepared_product_replays():
    # CRT residues + their reconstruction + a product with prepared A planes,
    # captured once and replayed with eager work in between
    bits = 60
    m, n, k = 70, 40, 256
    primes = gen.crt_primes(count=6)
    A = gen.uniform_bits(6, 1, m * k, bits).reshape(m, k)
    B = gen.uniform_bits(6, 2, k * n, bits).reshape(k, n)
    dA, dB = dev64(A), dev64(B)
    outs = [torch.zeros((m, n), dtype=torch.float64, device="cuda") for _ in primes]
    ws = torch.empty(mmp.workspace_crt(m, n, k, bits, len(primes)), dtype=torch.uint8, device="cuda")
    limbs = mmp.crt_limbs(primes)
    rec = torch.zeros((limbs, m, n), dtype=torch.int64, device="cuda")
    p = 1099511627689
    A2 = gen.random_matrix(8, 1, 90, 3000, p)
    B2 = gen.random_matrix(8, 2, 3000, 20, p)
    dA2, dB2 = dev(A2), dev(B2)
    C2 = torch.zeros((90, 20), dtype=torch.float64, device="cuda")
    pl = mmp.plan(p, 90, 20, 3000, form=mmp.FORM_INT8_WORDS)
    pws = torch.empty(pl["workspace_bytes"], dtype=torch.uint8, device="cuda")
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        pa = mmp.prepare_operand(dA2, p, 0, stream=s)

        def work():
            mmp.mm_modp_crt(dA, dB, primes, outs, bits, stream=s, workspace=ws)
            mmp.crt_reconstruct(outs, primes, out=rec, stream=s)
            mmp.mm_modp_async(dA2, dB2, C2, p, stream=s, prepared_a=pa, workspace=pws)
        work()  # warm-up outside the graph
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        work()
    exact = [[sum(int(A[i, l]) * int(B[l, j]) for l in range(k)) for j in range(n)] for i in range(m)]
    want2 = oracle.mm_modp(p, A2, B2).astype(np.float64)
    for rep in range(3):
        rec.fill_(-1)
        C2.fill_(-1.0)
        for C in outs:
            C.fill_(-1.0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        L = rec.cpu().numpy().view(np.uint64)
        got = [[sum(int(L[w, i, j]) << (64 * w) for w in range(limbs)) for j in range(n)] for i in range(m)]
        assert got == exact, rep
        assert np.array_equal(C2.cpu().numpy(), want2), rep
        x = torch.randn(1000, device="cuda").sum()
        torch.cuda.synchronize()
        del x


def _mix64(seed, count=64, dim_hi=700):
    """Products with bitsizes uniform in 20..52 (every digit count 3..7) and
    log-uniform dimensions: the serving mix at test size."""
    reqs = gen.serve_stream(count, 1.0, seed=seed, dim_lo=16, dim_hi=dim_hi)
    out = []
    for r in reqs:
        pr = r.problem
        A, B = pr.a(), pr.b()
        out.append((pr, A, B, dev(A), dev(B), torch.full((pr.m, pr.n), -1.0, dtype=torch.float64, device="cuda")))
    return out


def test_one_launch_batch_of_mixed_digit_counts():
    items = _mix64(91)
    digits = sorted({(pr.p.bit_length() + 7) // 8 for pr, *_ in items})
    say("mixed batch digit counts", digits, "bits", sorted({pr.p.bit_length() for pr, *_ in items}))
    assert len(digits) >= 4
    jobs = [(dA, dB, C, pr.p, 0, 0) for pr, A, B, dA, dB, C in items]
    torch.cuda.synchronize()
    mmp.timers_read(reset=True)
    mmp.timers_enable(True)
    mmp.mm_modp_batched(jobs, form=mmp.FORM_INT8_WORDS)
    torch.cuda.synchronize()
    mmp.timers_enable(False)
    t = mmp.timers_read(reset=True)
    say("timers", t)
    # the planes of all 64 products in one launch, their GEMM in one more
    assert t == {"int8_batch_digitize": (1, t["int8_batch_digitize"][1]), "int8_batch_gemm": (1, t["int8_batch_gemm"][1])}
    grouped = [torch.full_like(C, -2.0) for *_, C in items]
    mmp.mm_modp_batched([(dA, dB, G, pr.p, 0, 0) for (pr, A, B, dA, dB, C), G in zip(items, grouped)],
                        form=mmp.FORM_INT8_WORDS, batch_launch=1)
    torch.cuda.synchronize()
    for (pr, A, B, dA, dB, C), G in zip(items, grouped):
        want = oracle.mm_modp(pr.p, A, B).astype(np.float64)
        assert np.array_equal(C.cpu().numpy(), want), (pr.m, pr.n, pr.k, pr.p)
        assert torch.equal(C, G)


def test_one_launch_batch_more_than_64_and_ragged():
    # 70 products: two launches of each kernel; a k = 0 product is zero-filled
    items = _mix64(92, count=70, dim_hi=200)
    jobs = [(dA, dB, C, pr.p, 0, 0) for pr, A, B, dA, dB, C in items]
    z = torch.full((3, 4), 5.0, dtype=torch.float64, device="cuda")
    jobs.append((torch.zeros((3, 0), dtype=torch.float64, device="cuda"),
                 torch.zeros((0, 4), dtype=torch.float64, device="cuda"), z, 65521, 0, 0))
    mmp.timers_read(reset=True)
    mmp.timers_enable(True)
    mmp.mm_modp_batched(jobs, form=mmp.FORM_INT8_WORDS, batch_launch=2)
    torch.cuda.synchronize()
    mmp.timers_enable(False)
    t = mmp.timers_read(reset=True)
    assert t["int8_batch_digitize"][0] == 2 and t["int8_batch_gemm"][0] == 2
    for pr, A, B, dA, dB, C in items:
        assert np.array_equal(C.cpu().numpy(), oracle.mm_modp(pr.p, A, B).astype(np.float64))
    assert torch.all(z == 0)


def _replay_check(work, outs, wants, reps=3):
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        work(s)  # warm-up outside the graph
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        work(s)
    for rep in range(reps):
        for C in outs:
            C.fill_(-1.0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for C, w in zip(outs, wants):
            assert np.array_equal(C.cpu().numpy(), w), rep
        x = torch.randn(1000, device="cuda").sum()  # eager work between replays
        torch.cuda.synchronize()
        del x


def test_graph_capture_one_launch_batch_replays():
    items = _mix64(93, count=24, dim_hi=300)
    jobs = [(dA, dB, C, pr.p, 0, 0) for pr, A, B, dA, dB, C in items]
    ws = torch.empty(max(mmp.workspace_batched(jobs, form=mmp.FORM_INT8_WORDS), 1), dtype=torch.uint8,
                     device="cuda")
    wants = [oracle.mm_modp(pr.p, A, B).astype(np.float64) for pr, A, B, *_ in items]
    _replay_check(lambda s: mmp.mm_modp_batched(jobs, stream=s, workspace=ws, form=mmp.FORM_INT8_WORDS),
                  [C for *_, C in items], wants)


def test_graph_capture_fp64_word_batch_replays():
    # FP64-word products of several word pairs and blocks: no workspace
    cases = [(33554393, 1, 1), (8388593, 1, 2), (1125899906842597, 2, 2), (68719476731, 1, 3),
             (4503599627370449, 2, 3), (1099511627689, 2, 2)]
    items = []
    for i, (p, u, v) in enumerate(cases):
        m, n, k = 40 + 17 * i, 33 + 5 * i, 100 + 61 * i
        A = gen.random_matrix(100 + i, 1, m, k, p)
        B = gen.random_matrix(100 + i, 2, k, n, p)
        items.append((p, u, v, A, B, dev(A), dev(B), torch.zeros((m, n), dtype=torch.float64, device="cuda")))
    jobs = [(dA, dB, C, p, u, v) for p, u, v, A, B, dA, dB, C in items]
    assert mmp.workspace_batched(jobs) == 0
    wants = [oracle.mm_modp(p, A, B).astype(np.float64) for p, u, v, A, B, *_ in items]
    _replay_check(lambda s: mmp.mm_modp_batched(jobs, stream=s), [C for *_, C in items], wants)
