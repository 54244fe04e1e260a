#!/usr/bin/env python3
"""Benchmark: effective GFLOP/s of exact C = A B mod p on one MI355X.

One step is one call of the library's product entry point on resident
device inputs: plan, in-kernel word split, word products on the matrix
cores with in-loop modular reductions, recombination and the single store
of C (the whole method of Section 3.2).  Effective GFLOP/s is 2 m n k / t
(the paper's metric, Section 4.1).

Default workload: square m = n = k = 8192 with p the largest prime below
2^50, (u, v) = (2, 2) binary64 words on the FP64 matrix cores under the
paper's block bound (Prop. UVMW, eq. cAcB: lambda = 7); beside it the same
product under the other forms and bounds, its all-(p-1) worst case, the
4096^3 workloads at 36 and 26 bits, a served stream of mixed products and
the oracle on the host.  Other workloads by --config/--variant.

Prints one JSON line on stdout; progress goes to stderr.
"""

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_MFMA_PEAK_TFLOPS = 78.6  # MI355X dense FP64 matrix peak
INT8_MFMA_PEAK_TOPS = 5000.0
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# The sources that define each form's dominant kernel and its launch: a
# counter record taken on other sources than these is stale.
KERNEL_SOURCES = {
    1: ["fp64_words_kernel.h", "mmp_fp64_words.hip"],
    # the digit GEMM, its persistent form and their folds (the digitize passes
    # live in int8_digitize_kernel.h)
    2: ["int8_digits_kernel.h", "int8_digits_persistent.h", "int8_fold.h"],
}


def source_digest(form):
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2601_07508_amd", "csrc")
    for fn in KERNEL_SOURCES[form]:
        with open(os.path.join(d, fn), "rb") as f:
            h.update(fn.encode() + f.read())
    return h.hexdigest()[:16]


def traffic_for(workload, kernel, digest):
    """HBM bytes per launch from committed rocprofv3 counter runs, if they
    were taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path)).get(workload)
    except Exception:
        return None
    if not rec or rec.get("source_digest") != digest or not rec.get("kernel", "").startswith(kernel):
        return None
    return rec.get("hbm_bytes_per_launch")


def binding_roof(plan, m, n, k, work, peak, unit, kern_ms):
    """The roof that binds the dominant kernel, and its fraction.

    Algorithmic HBM bytes: the binary64 operands read once and C written
    once (FP64 words), or both operands' digit planes read once and C
    written once (INT8 digits).  The roof that binds is the one whose time
    at peak is the larger: the MFMA work (`work` at `peak` in `unit`) or
    those bytes at 8 TB/s."""
    mn, mk, kn = float(m) * n, float(m) * k, float(k) * n
    if plan["form"] == 1:
        alg_bytes = 8.0 * (mk + kn + mn)
    else:
        alg_bytes = plan["digits_a"] * mk + plan["digits_b"] * kn + 8.0 * mn
    if alg_bytes / (HBM_PEAK_GBS * 1e9) > work / (peak * 1e12):
        achieved = alg_bytes / (kern_ms * 1e-3) / 1e9 if kern_ms > 0 else 0.0
        bound, peak, unit = "hbm", HBM_PEAK_GBS, "GB/s"
    else:
        achieved = work / (kern_ms * 1e-3) / 1e12 if kern_ms > 0 else 0.0
        bound = "mfma"
    return {"bound": bound, "achieved": round(achieved, 3), "peak": peak, "unit": unit,
            "frac": round(achieved / peak, 4), "algorithmic_work_per_launch": work,
            "algorithmic_bytes_per_launch": alg_bytes}


def cpu_baseline(prob, A, B, budget_s=12.0):
    """The oracle, untuned, on the first rows of the same product."""
    import numpy as np

    import oracle

    rows = 8
    while True:  # grow the sample until it takes a sizeable share of the budget
        t0 = time.perf_counter()
        oracle.mm_modp(prob.p, np.ascontiguousarray(A[:rows]), B)
        t = time.perf_counter() - t0
        if t >= budget_s / 3 or rows >= prob.m:
            break
        rows = int(min(prob.m, max(2 * rows, rows * budget_s / max(t, 1e-3))))
    return {
        "value": 2.0 * rows * prob.n * prob.k / t / 1e9,
        "unit": "GFLOP/s",
        "cores": oracle.threads(),
        "cpu_model": _cpu_model(),
        "kind": "oracle",
        "sample": f"rows 0..{rows - 1} of the {prob.m}x{prob.n}x{prob.k} product "
                  f"({rows * prob.n} outputs, {t:.1f} s, 128-bit integer dot products)",
    }


def serving(mmp, torch, gen, count, loads):
    """Continuous-batching server on a Poisson stream of mixed products.

    Requests: m, n, k log-uniform in [64, 4096], bitsize uniform in [20, 52],
    p the largest prime below a random x of that bitsize, entries uniform in
    [0, p) generated on the device.  First a closed-loop pass (all requests
    at once) measures capacity; then open-loop passes submit at the given
    fractions of it and report request latency (submission to completion)
    percentiles beside throughput.
    """
    import threading

    import numpy as np

    reqs = gen.serve_stream(count, 1.0, seed=gen.BASE_SEED + 6)
    ops = []
    for i, r in enumerate(reqs):
        pr = r.problem
        g = torch.Generator(device="cuda")
        g.manual_seed(pr.seed)
        A = torch.randint(0, pr.p, (pr.m, pr.k), generator=g, device="cuda", dtype=torch.int64).double()
        B = torch.randint(0, pr.p, (pr.k, pr.n), generator=g, device="cuda", dtype=torch.int64).double()
        C = torch.empty((pr.m, pr.n), dtype=torch.float64, device="cuda")
        ops.append((pr, A, B, C))
    torch.cuda.synchronize()
    flops = sum(2.0 * pr.m * pr.n * pr.k for pr, *_ in ops)
    budget = 64 << 30

    def run(arrivals):
        lats = [0.0] * len(ops)
        tickets = [None] * len(ops)
        with mmp.Server(hbm_budget=budget, max_slots=64) as srv:
            t0 = time.perf_counter()

            def submitter():
                for i, (pr, A, B, C) in enumerate(ops):
                    if arrivals is not None:
                        while time.perf_counter() - t0 < arrivals[i]:
                            time.sleep(0)
                    tickets[i] = srv.submit(A, B, C, pr.p, ordered=False)  # inputs synchronised above

            th = threading.Thread(target=submitter)
            th.start()
            for i in range(len(ops)):
                while tickets[i] is None:
                    time.sleep(1e-5)
                st, lat = srv.wait(tickets[i], 600.0)
                if st != 0:
                    raise RuntimeError(f"request {i} failed: {st}")
                lats[i] = lat
            th.join()
            wall = time.perf_counter() - t0
            stats = srv.stats()
        return np.array(lats), wall, stats

    run(None)  # warm-up: kernels loaded, memory pool grown
    lat, wall, stats = run(None)
    capacity = len(ops) / wall
    out = {"requests": len(ops), "capacity_req_per_s": round(capacity, 1),
           "closed_loop_gflops": round(flops / wall / 1e9, 1),
           "closed_loop_p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 3),
           "closed_loop_p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 3),
           "max_batch": stats["max_batch"], "max_batches_in_flight": stats["max_inflight"],
           "max_requests_in_flight": stats["max_running"], "loads": {}}
    r = gen.raw_u64(gen.stream_key(gen.BASE_SEED + 6, 9), 0, len(ops)).astype(np.float64) / 2.0**64
    gaps = -np.log1p(-np.minimum(r, 1 - 1e-16))  # unit-rate exponential
    for f in loads:
        arrivals = np.cumsum(gaps) / (f * capacity)
        lat, wall, stats = run(arrivals)
        out["loads"][str(f)] = {"rate_req_per_s": round(f * capacity, 1),
                                "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 3),
                                "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 3),
                                "mean_ms": round(float(lat.mean()) * 1e3, 3),
                                "throughput_gflops": round(flops / wall / 1e9, 1),
                                "launches": stats["launches"], "max_batch": stats["max_batch"],
                                "max_batches_in_flight": stats["max_inflight"],
                                "max_requests_in_flight": stats["max_running"]}
    return out


def _residues_ok(torch, C, p):
    return bool(torch.all((C >= 0) & (C < p) & (C == torch.floor(C))))


def _time(torch, fn, warmup, steps, min_warm_s=0.25):
    """ms per call over `steps` back-to-back calls, after `warmup` calls and
    at least `min_warm_s` seconds of them: the first tens of milliseconds of
    a burst of short calls run at a clock the chip does not hold."""
    t0 = time.perf_counter()
    done = 0
    while done < warmup or time.perf_counter() - t0 < min_warm_s:
        fn()
        done += 1
        if done % 8 == 0:
            torch.cuda.synchronize()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def bench_unbalanced(args, mmp, torch, gen):
    """The paper's unbalanced workload (m = 10923, k = 32768, n = 32): A fixed
    across the iterations of block-Wiedemann, B new each time.  Per bitsize:
    the FP64 words (A's words are formed inside the kernel on every call), the
    INT8 digits with A digitised on every call, and the INT8 digits with A's
    digit planes prepared once (only B digitised per call, the paper's timing
    rule for this workload), directly and through a server with A registered.
    Outputs of all must agree."""
    import numpy as np

    for b in [int(x) for x in args.unbalanced.split(",")]:
        prob = gen.unbalanced_problem(b)
        p, m, n, k = prob.p, prob.m, prob.n, prob.k
        dA = torch.from_numpy(prob.a().astype(np.float64)).cuda()
        dB = torch.from_numpy(prob.b().astype(np.float64)).cuda()
        res, outs = {}, {}
        stream = torch.cuda.current_stream()
        for name, kw in (("fp64_words", {"form": 1}), ("int8_digits", {"form": 2})):
            C = torch.empty((m, n), dtype=torch.float64, device="cuda")
            pl = mmp.plan(p, m, n, k, **kw)
            ms = _time(torch, lambda: mmp.mm_modp_async(dA, dB, C, p, stream=stream, **kw), 2, args.steps)
            res[name] = {"ms": round(ms, 4), "eff_gflops": round(2.0 * m * n * k / ms / 1e6, 1),
                         "uv": [pl["u"], pl["v"]], "digits": pl["digits_a"], "tile": [pl["bm"], pl["bn"]],
                         "splits": pl["splits"]}
            outs[name] = C
        # A's digit planes prepared once (not timed, as in the paper); each
        # call digitises B, multiplies and reduces
        C = torch.empty((m, n), dtype=torch.float64, device="cuda")
        pa = mmp.prepare_operand(dA, p, 0)
        ms = _time(torch, lambda: mmp.mm_modp_async(dA, dB, C, p, stream=stream, prepared_a=pa), 2, args.steps)
        res["int8_digits_prepared_a"] = {"ms": round(ms, 4), "eff_gflops": round(2.0 * m * n * k / ms / 1e6, 1)}
        outs["int8_digits_prepared_a"] = C
        del pa
        # the same through the server with A registered: requests submitted
        # back to back, each waited for (adds the server's host round trip)
        C = torch.empty((m, n), dtype=torch.float64, device="cuda")
        with mmp.Server(hbm_budget=64 << 30, max_slots=4) as srv:
            srv.register_operand(dA, p, 0)
            for _ in range(2):
                srv.wait(srv.submit(dA, dB, C, p), 60.0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                srv.wait(srv.submit(dA, dB, C, p), 60.0)
            ms = (time.perf_counter() - t0) * 1e3 / args.steps
        res["int8_digits_server_resident_a"] = {"ms": round(ms, 4),
                                                "eff_gflops": round(2.0 * m * n * k / ms / 1e6, 1)}
        outs["int8_digits_server_resident_a"] = C
        same = all(torch.equal(outs["fp64_words"], c) for c in outs.values())
        ok = all(_residues_ok(torch, c, p) for c in outs.values())
        print(json.dumps({"workload": prob.tag, "bits": b, "p": p, "shape": [m, n, k], "forms": res,
                          "identical_outputs": bool(same), "residues_in_range": ok,
                          "note": "prepared-A: A's digit planes made once, untimed; server: per request, "
                                  "submit to completion"}),
              flush=True)
        del dA, dB, outs
        torch.cuda.empty_cache()
        if not (same and ok):
            sys.exit(1)


def bench_crt(args, mmp, torch, gen):
    """One integer pair against 32 primes of 31..50 bits (the CRT job)."""
    import numpy as np

    job = gen.crt_job()
    A, B = job.a(), job.b()
    dA = torch.from_numpy(A.astype(np.int64)).cuda()
    dB = torch.from_numpy(B.astype(np.int64)).cuda()
    outs = [torch.empty((job.m, job.n), dtype=torch.float64, device="cuda") for _ in job.primes]
    ms = _time(torch, lambda: mmp.mm_modp_crt(dA, dB, job.primes, outs, job.bits), args.warmup, args.steps)
    mmp.timers_read(reset=True)
    mmp.timers_enable(True)
    mmp.mm_modp_crt(dA, dB, job.primes, outs, job.bits)
    torch.cuda.synchronize()
    mmp.timers_enable(False)
    phases = mmp.timers_read(reset=True)
    for p, C in zip(job.primes, outs):
        if not _residues_ok(torch, C, p):
            log("RESULT OUT OF RANGE", p)
            sys.exit(1)
    mnk = float(job.m) * job.n * job.k
    d = (job.bits + 1 + 7) // 8
    gemm_ms = phases.get("crt_gemm", (1, 0.0))[1]
    # Chinese remainder reconstruction of the integer product: from all the
    # moduli, and from the shortest prefix whose product exceeds
    # k (2^bits - 1)^2 (eq. CRT2); the two must agree on every entry
    bound = job.k * ((1 << job.bits) - 1) ** 2
    M, s_min = 1, 0
    for i, p in enumerate(job.primes):
        M *= p
        if M > bound:
            s_min = i + 1
            break
    rec = {}
    outs_rec = {}
    for name, use in (("all_moduli", len(job.primes)), ("eq_crt2_moduli", s_min)):
        r_in, mods = outs[:use], job.primes[:use]
        limbs = mmp.crt_limbs(mods)
        o = torch.empty((limbs, job.m, job.n), dtype=torch.int64, device="cuda")
        t = _time(torch, lambda: mmp.crt_reconstruct(r_in, mods, out=o), 2, args.steps)
        rec[name] = {"moduli": use, "limbs": limbs, "ms": round(t, 4),
                     "entries_per_s": round(job.m * job.n / (t * 1e-3), 1)}
        outs_rec[name] = o
    lf = outs_rec["eq_crt2_moduli"].shape[0]
    same = bool(torch.equal(outs_rec["all_moduli"][:lf], outs_rec["eq_crt2_moduli"])) and \
        bool(torch.all(outs_rec["all_moduli"][lf:] == 0))
    if not same:
        log("RECONSTRUCTIONS DIFFER")
        sys.exit(1)
    rec["identical_low_limbs"] = same
    # product counts: eq. numprodMM (multimodular moduli) against the
    # multiword count (eq. numprodMW's least uv) and the planner's FP64 words
    counts = []
    for b in sorted({p.bit_length() for p in job.primes}):
        p = next(x for x in job.primes if x.bit_length() == b)
        row = {"bits": b}
        for lam in (1, 512):
            row[f"multimodular_lambda{lam}"] = math.ceil((4 * math.log2(p) + 2 * math.log2(job.k)) /
                                                        (53 - math.log2(lam)))
            row[f"multiword_lambda{lam}"] = min(
                (u * v for u, v in ((1, 1), (1, 2), (1, 3), (1, 4), (2, 2), (2, 3))
                 if u * v >= (u + v) * math.log2(p) / (53 - math.log2(lam))), default=None)
        pl = mmp.plan(p, job.m, job.n, job.k, form=1)
        row["planner_fp64_uv"] = pl["u"] * pl["v"]
        counts.append(row)
    print(json.dumps({
        "metric": "effective 2mnk GFLOP/s over all moduli of the CRT job",
        "value": round(len(job.primes) * 2 * mnk / (ms * 1e-3) / 1e9, 1), "unit": "GFLOP/s",
        "ms_per_step": round(ms, 4), "primes": len(job.primes), "entry_bits": job.bits,
        "config": {"workload": f"CRT {job.m}x{job.n}x{job.k}, entries < 2^{job.bits}, "
                               f"{len(job.primes)} primes of 31..50 bits"},
        "roofline": {"bound": "mfma", "kernel": "crt_gemm_kernel", "kernel_ms": round(gemm_ms, 4),
                     "achieved": round(2 * d * d * mnk / (gemm_ms * 1e-3) / 1e12, 2) if gemm_ms else None,
                     "peak": INT8_MFMA_PEAK_TOPS, "unit": "TOP/s"},
        "phases_ms": {k: round(v[1], 4) for k, v in phases.items()},
        "reconstruction": rec, "product_counts": counts}), flush=True)


def bench_autotune(args, mmp, torch, gen):
    """The eight skinny workloads (16384^2 x 256 and 512^2 x 131072 at 23, 31,
    40 and 52 bits) through the autotuner: per workload the tuned choice
    (form, words, tile, block) and its time per call against the planner's
    default plan, with outputs checked identical.  One JSON line per workload."""
    for prob in gen.config_problems(4):
        mmp.tune_cache_clear()
        default = mmp.plan(prob.p, prob.m, prob.n, prob.k)
        dA = torch.from_numpy(prob.a().astype("float64")).cuda()
        dB = torch.from_numpy(prob.b().astype("float64")).cuda()
        C0 = torch.empty((prob.m, prob.n), dtype=torch.float64, device="cuda")
        C1 = torch.empty_like(C0)
        t_default = _time(torch, lambda: mmp.mm_modp_async(dA, dB, C0, prob.p), 2, args.steps)
        t0 = time.perf_counter()
        best, tried = mmp.autotune(prob.p, prob.m, prob.n, prob.k)
        tune_s = time.perf_counter() - t0
        tuned = mmp.plan(prob.p, prob.m, prob.n, prob.k)  # AUTO follows the cache now
        t_tuned = _time(torch, lambda: mmp.mm_modp_async(dA, dB, C1, prob.p), 2, args.steps)
        torch.cuda.synchronize()

        def desc(pl):
            if pl["form"] == 2:
                return {"form": "int8_digits", "digits": pl["digits_a"], "splits": pl["splits"]}
            return {"form": "fp64_words", "uv": [pl["u"], pl["v"]], "tile": pl["tile"], "kblock": pl["kblock"],
                    "slots": pl["slots"], "splits": pl["splits"]}
        print(json.dumps({"workload": prob.tag, "shape": [prob.m, prob.n, prob.k], "p": prob.p,
                          "bits": prob.p.bit_length(), "candidates_timed": tried, "tune_s": round(tune_s, 2),
                          "default": desc(default), "default_ms": round(t_default, 4),
                          "tuned": desc(tuned), "tuned_ms": round(t_tuned, 4),
                          "identical": bool(torch.equal(C0, C1))}), flush=True)
        del dA, dB, C0, C1
        torch.cuda.empty_cache()
    mmp.tune_cache_clear()


def sweep_bits(args, mmp, torch, gen):
    """Both word forms on one shape for each bitsize: which one wins."""
    import numpy as np

    base = gen.config_problems(args.config)[args.variant]
    for b in [int(x) for x in args.sweep_bits.split(",")]:
        p = gen.largest_prime_below_pow2(b)
        A = gen.random_matrix(b, 1, base.m, base.k, p)
        B = gen.random_matrix(b, 2, base.k, base.n, p)
        dA = torch.from_numpy(A.astype(np.float64)).cuda()
        dB = torch.from_numpy(B.astype(np.float64)).cuda()
        res = {}
        outs = {}
        for name, kw in (("fp64_words", {"form": 1}), ("fp64_words_extended", {"form": 1, "extended_block": True}),
                         ("fp64_words_centered", {"form": 1, "centered_words": True}),
                         ("int8_digits", {"form": 2})):
            C = torch.empty((base.m, base.n), dtype=torch.float64, device="cuda")
            pl = mmp.plan(p, base.m, base.n, base.k, **kw)
            ms = _time(torch, lambda: mmp.mm_modp_async(dA, dB, C, p, stream=torch.cuda.current_stream(), **kw),
                       2, max(3, args.steps // 4))
            res[name] = {"ms": round(ms, 4), "eff_gflops": round(2.0 * base.m * base.n * base.k / ms / 1e6, 1),
                         "uv": [pl["u"], pl["v"]], "digits": pl["digits_a"], "kblock": pl["kblock"]}
            outs[name] = C
        same = all(torch.equal(outs["int8_digits"], c) for c in outs.values())
        win = min(res, key=lambda k: res[k]["ms"])
        print(json.dumps({"bits": b, "p": p, "shape": [base.m, base.n, base.k], "forms": res, "winner": win,
                          "identical_outputs": bool(same)}), flush=True)
        if not same:
            sys.exit(1)


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _leg(mmp, torch, dA, dB, p, u, v, steps, ref=None, **kw):
    """Times one form/bound of a product on resident inputs; returns its record
    and output.  Kernel time comes from the library's launch events."""
    m, k = dA.shape
    n = dB.shape[1]
    C = torch.empty((m, n), dtype=torch.float64, device="cuda")
    pl = mmp.plan(p, m, n, k, u, v, **kw)
    stream = torch.cuda.current_stream()
    ms = _time(torch, lambda: mmp.mm_modp_async(dA, dB, C, p, u, v, stream=stream, **kw), 2, steps)
    mmp.timers_read(reset=True)
    mmp.timers_enable(True)
    for _ in range(steps):
        mmp.mm_modp_async(dA, dB, C, p, u, v, stream=stream, **kw)
    torch.cuda.synchronize()
    mmp.timers_enable(False)
    phases = mmp.timers_read(reset=True)
    mnk = float(m) * n * k
    if pl["form"] == 1:
        phase, peak, work = "fp64_words", FP64_MFMA_PEAK_TFLOPS, 2.0 * pl["u"] * pl["v"] * mnk
        desc = {"form": "fp64_words", "dtype": "f64", "uv": [pl["u"], pl["v"]], "lambda": pl["lambda"],
                "kblock": pl["kblock"], "slots": pl["slots"], "biased_reduction": bool(pl["biased"]),
                "extended_block": bool(pl["extended"]), "centered_words": bool(pl["centered"])}
    else:
        phase = "int8_gemm_persistent" if "int8_gemm_persistent" in phases else "int8_gemm"
        peak, work = INT8_MFMA_PEAK_TOPS, 2.0 * pl["digits_a"] * pl["digits_b"] * mnk
        desc = {"form": "int8_digits", "dtype": "int8 digits, int32 accumulation, f64 fold",
                "digits": pl["digits_a"]}
    launches, tot = phases.get(phase, (0, 0.0))
    kms = tot / max(launches, 1)
    rec = dict(desc)
    rec.update({"ms": round(ms, 4), "eff_gflops": round(2.0 * mnk / (ms * 1e-3) / 1e9, 1),
                "kernel_ms": round(kms, 4),
                "kernel_frac_of_peak": round(work / (kms * 1e-3) / 1e12 / peak, 4) if kms > 0 else None})
    if ref is not None:
        rec["identical_to_headline"] = bool(torch.equal(C, ref))
    return rec, C


def extra_legs(args, mmp, torch, gen, prob, dA, dB, dC):
    """The headline product under the other forms and bounds, its all-(p-1)
    worst case, and the 4096^3 workloads at 36 and 26 bits."""
    steps = max(3, min(args.steps, 10))
    out = {}
    p = prob.p
    forms = {}
    for name, u, v, kw in (("fp64_words_lambda4", prob.u, prob.v, {"force_kblock": 4}),
                           ("fp64_words_extended_bound", prob.u, prob.v, {"extended_block": True}),
                           ("fp64_words_centered_words", prob.u, prob.v, {"centered_words": True}),
                           ("int8_digits", 0, 0, {"form": 2})):
        log("leg", name)
        forms[name], _ = _leg(mmp, torch, dA, dB, p, u, v, steps, ref=dC, **kw)
    out["same_workload_other_forms"] = forms
    # all entries p - 1: every word at its maximum; C = k mod p since (p-1)^2 = 1 mod p
    log("leg worst case")
    full = torch.full_like(dA, float(p - 1))
    want = float(prob.k % p)
    wc = {}
    for name, u, v, kw in (("fp64_words", prob.u, prob.v, {}), ("int8_digits", 0, 0, {"form": 2})):
        rec, C = _leg(mmp, torch, full, full, p, u, v, steps, **kw)
        rec["all_equal_k_mod_p"] = bool(torch.all(C == want))
        wc[name] = rec
    out["all_p_minus_1"] = wc
    del full
    # square 4096^3: 36 bits (the planner's choice, and the FP64 words it
    # would take), and 26 bits with the single word forced (lambda = 2)
    for tag, legs in ((0, (("auto", 0, 0, {}), ("fp64_words", 0, 0, {"form": 1}))),
                      (1, (("forced_uv11", 1, 1, {}), ("fp64_words", 0, 0, {"form": 1}),
                           ("int8_digits", 0, 0, {"form": 2})))):
        pr = gen.config_problems(2)[tag]
        log("workload", pr.tag)
        a = torch.from_numpy(pr.a().astype("float64")).cuda()
        b = torch.from_numpy(pr.b().astype("float64")).cuda()
        recs, ref = {}, None
        for name, u, v, kw in legs:
            rec, C = _leg(mmp, torch, a, b, pr.p, u, v, steps, ref=ref, **kw)
            if ref is None:
                ref = C
            else:
                rec["identical_to_first"] = rec.pop("identical_to_headline")
            recs[name] = rec
        out[pr.tag] = {"p": pr.p, "shape": [pr.m, pr.n, pr.k], "legs": recs}
        del a, b, ref
    torch.cuda.empty_cache()
    log("batched mix")
    out["batched_64_mixed"] = batched_mix(mmp, torch, gen, steps)
    torch.cuda.empty_cache()
    return out


def batched_mix(mmp, torch, gen, steps, count=64):
    """64 uneven products in one mm_modp_batched call (INT8 digits): m, n, k
    log-uniform in [64, 4096], bitsizes uniform in [20, 52] (digit counts
    3..7), entries uniform on the device.  The one-launch form (digit planes
    of all products in one launch, their GEMM in one persistent launch)
    against the grouped form (planes per product, a GEMM per digit count and
    16 products); outputs must agree."""
    reqs = gen.serve_stream(count, 1.0, seed=gen.BASE_SEED + 8)
    jobs, outs = [], {}
    flops = 0.0
    for r in reqs:
        pr = r.problem
        g = torch.Generator(device="cuda")
        g.manual_seed(pr.seed)
        A = torch.randint(0, pr.p, (pr.m, pr.k), generator=g, device="cuda", dtype=torch.int64).double()
        B = torch.randint(0, pr.p, (pr.k, pr.n), generator=g, device="cuda", dtype=torch.int64).double()
        jobs.append([A, B, None, pr.p, 0, 0])
        flops += 2.0 * pr.m * pr.n * pr.k
    rec = {"products": count, "bits": sorted({r.problem.p.bit_length() for r in reqs}),
           "digit_counts": sorted({(r.problem.p.bit_length() + 7) // 8 for r in reqs}),
           "total_2mnk": flops}
    for name, mode in (("one_launch", 0), ("grouped", 1)):
        Cs = [torch.empty((j[0].shape[0], j[1].shape[1]), dtype=torch.float64, device="cuda") for j in jobs]
        js = [(j[0], j[1], C, j[3], 0, 0) for j, C in zip(jobs, Cs)]
        ws = torch.empty(max(mmp.workspace_batched(js, form=2), 1), dtype=torch.uint8, device="cuda")
        call = lambda: mmp.mm_modp_batched(js, workspace=ws, form=2, batch_launch=mode)
        ms = _time(torch, call, 2, steps)
        mmp.timers_read(reset=True)
        mmp.timers_enable(True)
        call()
        torch.cuda.synchronize()
        mmp.timers_enable(False)
        ph = mmp.timers_read(reset=True)
        rec[name] = {"ms": round(ms, 4), "eff_gflops": round(flops / (ms * 1e-3) / 1e9, 1),
                     "launches": sum(v[0] for v in ph.values()),
                     "phases_ms": {k: round(v[1], 4) for k, v in ph.items()}}
        outs[name] = Cs
        del ws
    rec["identical"] = all(torch.equal(a, b) for a, b in zip(outs["one_launch"], outs["grouped"]))
    return rec


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", type=int, default=3, help="workload group 1..4")
    ap.add_argument("--variant", type=int, default=0, help="index inside the workload group")
    ap.add_argument("--form", type=int, default=0, help="0 auto, 1 FP64 words, 2 INT8 digits")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the other forms, the worst case and the 4096^3 legs of the default run")
    ap.add_argument("--serve", type=int, default=2000,
                    help="requests in the serving measurement (0: skip it)")
    ap.add_argument("--serve-loads", default="0.5,0.8,0.95",
                    help="comma-separated fractions of the measured capacity to offer")
    ap.add_argument("--batch-mix", action="store_true",
                    help="only the 64-product batch of mixed digit counts, one-launch and grouped forms")
    ap.add_argument("--autotune", action="store_true",
                    help="the eight skinny workloads through the autotuner, against the planner's default")
    ap.add_argument("--crt", action="store_true",
                    help="time the multi-modular job (2048^3 integers < 2^60 against 32 primes) instead")
    ap.add_argument("--sweep-bits", default="",
                    help="comma-separated bitsizes: time both forms on the workload's shape for each")
    ap.add_argument("--extended", action="store_true",
                    help="FP64 form: allow the extended (signed-range) block bound")
    ap.add_argument("--unbalanced", default="",
                    help="comma list of bitsizes: the unbalanced 10923x32768x32 workload, all forms")
    ap.add_argument("--centered", action="store_true",
                    help="FP64 form: centered words and their block bound")
    ap.add_argument("--force-kblock", type=int, default=0,
                    help="FP64 form: k-terms per block (0: the planner's)")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="instead of the product, time a plain device copy of this many bytes "
                         "(the reference kernel for scaling HBM counters)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(the product is measured on a single MI355X)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import mmp_inputs as gen
    import paper_2601_07508_amd as mmp

    if args.copy_bytes:
        src = torch.ones(args.copy_bytes // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(args.warmup):
            dst.copy_(src)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.steps):
            dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.steps
        print(json.dumps({"copy_bytes": args.copy_bytes, "ms": ms,
                          "GB/s (read+write)": 2 * args.copy_bytes / ms / 1e6}), flush=True)
        return

    if args.crt:
        return bench_crt(args, mmp, torch, gen)
    if args.autotune:
        return bench_autotune(args, mmp, torch, gen)
    if args.batch_mix:
        print(json.dumps(batched_mix(mmp, torch, gen, max(3, min(args.steps, 10)))), flush=True)
        return
    if args.sweep_bits:
        return sweep_bits(args, mmp, torch, gen)
    if args.unbalanced:
        return bench_unbalanced(args, mmp, torch, gen)

    prob = gen.config_problems(args.config)[args.variant]
    if args.form == 2:  # the INT8-digit form takes no word counts
        prob.u = prob.v = 0
    kw = dict(form=args.form, extended_block=args.extended, centered_words=args.centered,
              force_kblock=args.force_kblock)
    plan = mmp.plan(prob.p, prob.m, prob.n, prob.k, prob.u, prob.v, **kw)
    log("workload", prob.tag, "plan", plan)

    A = prob.a()
    B = prob.b()
    dA = torch.from_numpy(A.astype(np.float64)).cuda()
    dB = torch.from_numpy(B.astype(np.float64)).cuda()
    dC = torch.empty((prob.m, prob.n), dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()

    def step():
        mmp.mm_modp_async(dA, dB, dC, prob.p, prob.u, prob.v, stream=stream, **kw)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log("warmup done")

    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_wall0 = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    t_wall = time.perf_counter() - t_wall0
    ms = e0.elapsed_time(e1) / args.steps
    log(f"timed {args.steps} steps: {ms:.3f} ms/step (wall {t_wall:.3f} s)")

    # per-kernel device time: the library's event pairs around each launch, on
    # the stream the kernels run on, over the same number of steps
    mmp.timers_read(reset=True)
    mmp.timers_enable(True)
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    mmp.timers_enable(False)
    phases = mmp.timers_read(reset=True)
    log("phases", phases)

    # sanity of the last result (exactness is the tests' business): every
    # output an integer in [0, p)
    if not _residues_ok(torch, dC, prob.p):
        log("RESULT OUT OF RANGE")
        sys.exit(1)

    mnk = float(prob.m) * prob.n * prob.k
    eff = 2.0 * mnk / (ms * 1e-3) / 1e9
    digest = source_digest(plan["form"])
    workload = prob.tag
    if plan["form"] == 1:
        kernel, phase, peak, unit = "fp64_words_kernel", "fp64_words", FP64_MFMA_PEAK_TFLOPS, "TFLOP/s"
        work = 2.0 * plan["u"] * plan["v"] * mnk  # word flops per launch
        dtype = "f64"
        form_desc = (f"(u,v) = ({plan['u']},{plan['v']}) binary64 words on FP64 MFMA, k-block "
                     f"{plan['kblock']} of the bound {plan['lambda']}"
                     + (" (extended bound)" if plan["extended"] else
                        " (centered words)" if plan["centered"] else " (the paper's lambda)"))
    else:
        kernel, phase, peak, unit = "int8_digits_gemm_kernel", "int8_gemm", INT8_MFMA_PEAK_TOPS, "TOP/s"
        if "int8_gemm_persistent" in phases:  # many short tiles: the persistent form of the digit GEMM
            kernel, phase = "int8_digits_gemm_persistent_kernel", "int8_gemm_persistent"
        work = 2.0 * plan["digits_a"] * plan["digits_b"] * mnk  # digit-product int8 ops per launch
        dtype = "int8 digits, int32 accumulation, f64 fold"
        form_desc = f"{plan['digits_a']} signed 8-bit digits per entry on INT8 MFMA"
    launches, total_ms = phases.get(phase, (0, 0.0))
    kern_ms = total_ms / max(launches, 1)
    roofline = binding_roof(plan, prob.m, prob.n, prob.k, work, peak, unit, kern_ms)
    roofline.update({"traffic": traffic_for(workload, kernel, digest), "kernel": kernel,
                     "kernel_ms": round(kern_ms, 4)})
    shape = "square" if prob.m == prob.n == prob.k else "product"
    fill = ", all entries p - 1" if prob.fill == "pmax" else ""
    out = {
        "metric": "effective 2mnk GFLOP/s of C=AB mod p",
        "value": round(eff, 2),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic: seeded uniform integers in [0, p) stored as binary64" if not fill else
                "synthetic: every entry p - 1 (worst case) stored as binary64",
        "config": {
            "workload": f"{shape} {prob.m}x{prob.n}x{prob.k}, p = {prob.p} (largest prime below "
                        f"2^{prob.p.bit_length()}){fill}, {form_desc}, exact C = AB mod p",
            "m": prob.m, "n": prob.n, "k": prob.k, "p": prob.p, "bits": prob.p.bit_length(),
            "u": plan["u"], "v": plan["v"], "lambda": plan["lambda"], "kblock": plan["kblock"],
            "slots": plan["slots"], "biased_reduction": bool(plan["biased"]),
            "digits": plan["digits_a"], "extended_block": bool(plan["extended"]),
            "centered_words": bool(plan["centered"]),
            "form": "fp64_words" if plan["form"] == 1 else "int8_digits", "tile": plan["tile"],
        },
        "roofline": roofline,
        "phases_ms_per_step": {k: round(v[1] / max(args.steps, 1), 4) for k, v in phases.items()},
        "source_digest": digest,
    }
    default_run = (args.config == 3 and args.variant == 0 and args.form == 0 and not args.extended
                   and not args.centered and not args.force_kblock)
    if default_run and not args.no_extras:
        log("extra legs ...")
        out["extras"] = extra_legs(args, mmp, torch, gen, prob, dA, dB, dC)
    if args.serve > 0:
        log("serving ...")
        del dA, dB, dC
        torch.cuda.empty_cache()
        out["serving"] = serving(mmp, torch, gen, args.serve, [float(x) for x in args.serve_loads.split(",")])
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(prob, A, B)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
