"""Benchmark: MLMC level samples/s (field + solve) on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

One step = one pass of the whole hot path (normals, field DFTs, multigrid-
preconditioned CG solve, QoI) over one batch: the 4096 i.i.d. samples of
the single-level configuration Matern nu=1, lambda=0.1, sigma2=1 on 257^2
vertices (embedding 512^2), integral QoI, mixed precision (float field and
multigrid, double CG).  Each step draws new samples (seed 0, consecutive
sample indices).  Inputs are synthetic and generated on the device; the
plan set-up (eigenvalue DFT, masks) is timed separately, outside the timed
region.

Prints one JSON line on stdout; progress goes to stderr.
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLMC level samples/sec (field+solve) at 1 GPU, p50/p99 latency, % HBM roofline"
HBM_PEAK_GBS = 8000.0
# library kernel name -> device kernel symbol (mixed path) in rocprofv3 output
KERNEL_SYMBOL = {
    "mg_post_l0": "k_mg<float, 8, true, true, false, 64, false>",
    "mg_pre_l0": "k_mg<float, 8, false, true, false, 64, false>",
    "mg_post": "k_mg<float, 8, true, false, false, 64, false>",
    "mg_pre": "k_mg<float, 8, false, false, false, 64, false>",
    "mg_mid": "k_mg<float, 8, true, false, true, 128, true>",
    "mg_bottom": "k_bottom<float, 32, 256>",
    "pcg_dir": "k_pcg_dir<float>",
    "pcg_update": "k_pcg_update<false>",
    "pcg_init": "k_pcg_init<float>",
    "small_pcg": "k_small_pcg<float, 512, 32>",
    "small_direct": "k_small_direct<float>",
    "direct_lin": "k_direct_lin<float, 32, true>",
    "field_y": "k_field_y<float, 16, 0, 1>",
    "field_x": "k_field_x<float, 16, 0, 1, false>",
    "qoi": "k_qoi<float>",
}
# HBM traffic per launch from rocprofv3 FETCH_SIZE / WRITE_SIZE counters,
# scaled by a plain copy's counters; valid only for the kernel sources it
# was measured on (their SHA-256 is recorded with the figures).
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "c2_mixed_hbm_traffic.md")
# the kernels and the chunking (exec.cpp sizes the launches)
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2306_13493_amd", "csrc", f)
                  for f in ("solver.hip", "field.hip", "common.hpp", "fft_lds.hpp", "philox_bm.hpp", "exec.cpp")]


def sources_digest():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(symbol):
    """Calibrated HBM bytes per launch of `symbol`, or None when no counter
    figures exist for the current kernel sources."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    digest, row = None, None
    for line in open(TRAFFIC_FILE):
        if line.startswith("sources-sha256:"):
            digest = line.split(":", 1)[1].strip()
        cells = [c.strip() for c in line.strip().strip("|").split("|")]
        if len(cells) >= 5 and cells[0] == symbol:
            row = cells
    if digest != sources_digest() or row is None:
        return None
    return float(row[4])


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def dominant_roofline(prof, log, traffic_known=True, prof_all=None):
    """Roofline of the kernel with the largest total time in a launch
    profile (HIP events around each launch, algorithmic bytes per launch)
    and the per-kernel table.  prof_all, when given, is a profile of every
    kernel (prof then holds the dominant kernel's launches only): the
    table, the kernel's share and the whole-path rate come from it."""
    name, (launches, ms, nbytes) = max(prof.items(), key=lambda kv: kv[1][1])
    achieved = nbytes / (ms * 1e-3) / 1e9
    if prof_all is not None:
        prof = prof_all
        share_ms = prof_all[name][1]
    else:
        share_ms = ms
    total_ms = sum(v[1] for v in prof.values())
    symbol = KERNEL_SYMBOL.get(name, name)
    traffic = measured_traffic(symbol) if traffic_known else None
    roofline = {"bound": "hbm", "kernel": name, "symbol": symbol,
                "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": round(traffic) if traffic is not None else None,
                "avg_launch_us": round(ms * 1e3 / launches, 2), "launches": launches,
                "algorithmic_bytes_per_launch": round(nbytes / launches),
                "share_of_kernel_time": round(share_ms / total_ms, 4)}
    all_bytes = sum(v[2] for v in prof.values())
    kernels = {k: {"launches": v[0], "ms": round(v[1], 3),
                   "GBps": round(v[2] / (v[1] * 1e-3) / 1e9, 1) if v[1] > 0 else None}
               for k, v in sorted(prof.items(), key=lambda kv: -kv[1][1])}
    log("dominant kernel %s: %.1f GB/s (%.1f%% of 8 TB/s); whole path %.1f GB/s"
        % (name, achieved, 100 * achieved / HBM_PEAK_GBS, all_bytes / (total_ms * 1e-3) / 1e9))
    return roofline, kernels


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def c5_record(ces, ctx, W, log, steps=2):
    """The large flow-cell level (Matern nu=3/2, sigma2=2, lambda=0.01,
    2049^2 vertices, embedding 4096^2, outflow QoI, mixed precision) at its
    1024 samples per call: samples/s over `steps` timed calls (after one
    warm-up call and one call with the launch profiler on, which gives the
    live roofline of its dominant kernel), CG iterations, parity of sample
    0 (its field against the oracle's, and the device solve of its
    coefficient checked by the residual and flux balance of the flow cell
    under the oracle's element-by-element operator), and the oracle's time
    for the field of one sample (its SuperLU solve at 4.2 million unknowns
    takes minutes per sample and is not run here)."""
    import numpy as np
    import torch
    from oracle import fem as ofem, qoi as oqoi, sampler
    from paper_2306_13493_amd.workloads import to_oracle
    w = dict(W.C5)
    count = 1024
    t0 = time.perf_counter()
    plan = ctx.plan(ces.level_desc(**w))
    setup_ms = (time.perf_counter() - t0) * 1e3
    out = plan.sample(0, 0, count)
    torch.cuda.synchronize()
    log("C5: plan n=%d, warm-up call of %d samples done" % (plan.info.n, count))
    ces.profile_enable(True)
    torch.cuda.synchronize()
    out = plan.sample(0, count, count, out=out)
    torch.cuda.synchronize()
    prof = ces.profile_read()
    ces.profile_enable(False)
    roofline, kernels = dominant_roofline(prof, log, traffic_known=False)
    ts = []
    for k in range(steps):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        out = plan.sample(0, (k + 2) * count, count, out=out)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t1)
    it = out["iters"].cpu().numpy()
    ok = bool(np.all(out["status"].cpu().numpy() == 0))
    value = count / float(np.median(ts))
    log("C5: %d samples per call in %.3f s -> %.1f samples/s; CG iterations mean %.2f" % (count, np.median(ts),
                                                                                       value, it.mean()))
    # parity of sample 0
    m = w["m"]
    y0 = float(plan.sample(0, 0, 1)["y"].cpu().numpy()[0])
    zf, _ = plan.field(0, 0)
    z = zf.cpu().numpy()
    t1 = time.perf_counter()
    ref = sampler.Plan(to_oracle(w))
    t_setup = time.perf_counter() - t1
    t1 = time.perf_counter()
    zr, _ = ref.fields(0, 0)
    t_field = time.perf_counter() - t1
    field_err = float(np.max(np.abs(z - zr)) / np.max(np.abs(zr)))
    k = np.exp(z).astype(np.float32).astype(np.float64)   # the coefficient the mixed solver sees
    u, _ = plan.solve(torch.from_numpy(k).reshape(1, m + 1, m + 1).to("cuda"))
    uu = u.cpu().numpy().reshape(-1)
    A, b = ofem.assemble(k, m, 1.0)
    res = b - A @ uu
    i = np.arange((m + 1) ** 2) % (m + 1)
    free = (i > 0) & (i < m)
    r0 = b - A @ (i == 0).astype(np.float64)
    rel_res = float(np.linalg.norm(res[free]) / np.linalg.norm(r0[free]))
    balance = float(abs(res[i == 0].sum() + res[i == m].sum() - b.sum()))
    q = oqoi.outflux(uu, m, A, b)
    qoi_err = abs(y0 - q) / abs(q)
    log("C5 parity: field %.2e of max|Z|; residual %.2e of r0; flux balance %.2e; outflow QoI %.2e"
        % (field_err, rel_res, balance, qoi_err))
    return {
        "metric": "MLMC level samples/sec (field+solve), 2049^2 flow cell at 1 GPU", "value": round(value, 1),
        "unit": "samples/s", "samples_per_call": count, "calls_timed": steps,
        "ms_per_call": round(float(np.median(ts)) * 1e3, 1), "setup_ms": round(setup_ms, 1),
        "cg_iterations_mean": round(float(it.mean()), 3), "all_converged": ok,
        "config": {"workload": "Matern nu=3/2 sigma2=2 lambda=0.01, 2049x2049 vertices, embedding 4096x4096 "
                               "(nonnegative at 2m), flow cell (u=1 at x1=0, u=0 at x1=1), f=1, outflow QoI, "
                               "float field+multigrid, double CG to 1e-10, %d samples per call" % count},
        "roofline": roofline, "kernels": kernels,
        "parity_sample0": {"field_max_rel_diff": field_err, "field_bar": 1e-5,
                           "residual_rel_r0": rel_res, "flux_balance_abs": balance,
                           "outflow_qoi_rel_diff": qoi_err, "qoi_bar": 1e-6,
                           "operator": "oracle element-by-element P1 assembly on the float coefficient"},
        "cpu_oracle": {"kind": "oracle", "cores": 1, "cpu_model": cpu_model(),
                       "sample": "the field of sample 0 (normals, FP64 DFT at 4096^2, restriction)",
                       "setup_s": round(t_setup, 2), "field_s_per_sample": round(t_field, 2),
                       "solve_s_per_sample": None,
                       "note": "the oracle's SuperLU solve of one sample at 2049^2 took 678 s on one core of "
                               "the build container; far beyond this run's time, so not timed here"},
    }


def _oracle_worker(args):
    desc, seed, idx = args
    os.environ["OMP_NUM_THREADS"] = "1"
    from oracle import sampler
    p = sampler.Plan(desc)
    return [p.sample(seed, i)[0] for i in idx]


def cpu_baseline(workload, seed, nsamples, nproc):
    """The FP64 oracle timed on host cores over a bounded sample."""
    import multiprocessing as mp
    from paper_2306_13493_amd.workloads import to_oracle
    desc = to_oracle(workload)
    chunks = [list(range(r, nsamples, nproc)) for r in range(nproc)]
    t0 = time.perf_counter()
    ctx = mp.get_context("spawn")
    with ctx.Pool(nproc) as pool:
        parts = pool.map(_oracle_worker, [(desc, seed, c) for c in chunks])
    dt = time.perf_counter() - t0
    y = [0.0] * nsamples
    for c, v in zip(chunks, parts):
        for i, val in zip(c, v):
            y[i] = val
    return y, dt


def parity_per_result(ces, plan, w, seed, log):
    """Error of each result type of the benchmarked plan against the FP64
    oracle: the normals (bit-exact), the Gaussian field Z of two samples
    (relative to max |Z|) and the QoI (checked on the CPU-baseline samples
    by the caller)."""
    import numpy as np
    from oracle import normals as onm, sampler
    from paper_2306_13493_amd.workloads import to_oracle
    e = np.arange(0, 200000, dtype=np.uint64)
    g = ces.normals(seed, 5, w.get("stream", 0), 0, len(e)).cpu().numpy()
    g0, g1 = onm.normals(seed, 5, w.get("stream", 0), e)
    bitexact = bool(np.array_equal(g.view(np.uint64), np.stack([g0, g1], axis=1).view(np.uint64)))
    ref = sampler.Plan(to_oracle(w))
    worst = 0.0
    for i in (0, 1):
        zf, _ = plan.field(seed, i)
        zr, _ = ref.fields(seed, i)
        worst = max(worst, float(np.max(np.abs(zf.cpu().numpy() - zr)) / np.max(np.abs(zr))))
    log("parity: normals bit-exact %s (%d pairs); field max rel diff %.2e" % (bitexact, len(e), worst))
    return {"normals_bit_exact": bitexact, "normals_checked": int(len(e)), "field_max_rel_diff": worst,
            "field_bar": 1e-5, "qoi_bar": 1e-6}


def c3_batch(ces, ctx, W, log, reps=5):
    """Five MLMC levels (m = 16 .. 256, N = 20000/5000/1200/300/80) in one
    ces_sample_batch call, against the same levels one ces_sample call at a
    time; wall time per estimator round with results on the device."""
    import numpy as np
    import torch
    plans = [ctx.plan(ces.level_desc(**W.c3_level(l))) for l in range(len(W.C3_M))]
    reqs = [(p, 0, 0, n) for p, n in zip(plans, W.C3_N)]
    outs = ctx.sample_batch(reqs)
    seq = [p.sample(0, 0, n) for p, n in zip(plans, W.C3_N)]
    torch.cuda.synchronize()
    same = all(bool(torch.equal(a["y"], b["y"])) for a, b in zip(outs, seq))

    def timed(fn):
        ts = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            ts.append((time.perf_counter() - t0) * 1e3)
        return float(np.median(ts))

    default = list(ctx.schedule)
    t_default = timed(lambda: ctx.sample_batch(reqs, outs=outs))
    # the autotuner's schedule for this batch (a stored choice when
    # CESMLMC_AUTOTUNE_CACHE names a file that has one)
    tuned, tune_ms, _ = ctx.autotune(reqs, outs=outs)
    t_batch = timed(lambda: ctx.sample_batch(reqs, outs=outs))
    t_seq = timed(lambda: [p.sample(0, 0, n, out=o) for p, n, o in zip(plans, W.C3_N, seq)])
    torch.cuda.synchronize()
    same = same and all(bool(torch.equal(a["y"], b["y"])) for a, b in zip(outs, seq))
    total = sum(W.C3_N)
    log("C3 five-level batch: %.2f ms per round (%d level samples) under the tuned schedule %s (default %s: "
        "%.2f ms), one call per level %.2f ms; identical %s" % (t_batch, total, list(tuned), default, t_default,
                                                               t_seq, same))
    ctx.schedule = tuple(default)
    return {"ms_per_round": round(t_batch, 3), "level_samples_per_round": total,
            "level_samples_per_s": round(total / (t_batch * 1e-3), 1),
            "ms_one_call_per_level": round(t_seq, 3), "batch_equals_per_level_bitwise": same,
            "schedule": list(tuned), "schedule_fields": ["depth", "max_lanes", "chunk_samples", "graphs"],
            "default_schedule": default, "ms_per_round_default_schedule": round(t_default, 3)}


def serve(args):
    """Serving workload: replay the arrival trace (Poisson arrivals, mixed
    meshes 33^2 .. 1025^2, counts 1..256, a fresh covariance per request)
    into one server and drain.  Prints one JSON line."""
    import threading
    import numpy as np
    import torch
    import paper_2306_13493_amd as ces
    from paper_2306_13493_amd import workloads as W

    torch.cuda.init()
    ces.load()
    ctx = ces.Context(0)
    trace = W.c4_trace(duration_s=args.duration, rate=args.rate)
    log("serving trace: %d requests over %.1f s (rate %.0f/s), %d level samples"
        % (len(trace), args.duration, args.rate, sum(r["count"] for r in trace)))
    # warm the kernels on a throwaway server (first launches load code objects)
    warm = ces.Server(ctx)
    for m in (32, 64, 1024):
        warm.submit(dict(trace[0]["w"], m=m, level="single" if m == 32 else "pair"), 0, 0, 2)
    warm.drain()
    warm.close()
    srv = ces.Server(ctx, mem_budget=int(args.mem_gb * (1 << 30)), max_inflight=args.max_inflight)
    ids = [None] * len(trace)
    t0 = time.perf_counter()

    def replay():
        for i, r in enumerate(trace):
            d = r["t"] - (time.perf_counter() - t0)
            if d > 0:
                time.sleep(d)
            ids[i] = srv.submit(r["w"], r["seed"], r["first"], r["count"])

    th = threading.Thread(target=replay)
    th.start()
    last = time.perf_counter()
    while th.is_alive():
        th.join(timeout=5.0)
        st = srv.stats()
        log("t=%.1f s submitted %d completed %d admitted %d queued %d mem %.1f GB"
            % (time.perf_counter() - t0, st["submitted"], st["completed"], st["admitted"], st["queued"],
               st["mem_in_use"] / 2 ** 30))
    t_submit_end = time.perf_counter() - t0
    done = threading.Event()

    def drainer():
        srv.drain()
        done.set()

    dt = threading.Thread(target=drainer)
    dt.start()
    while not done.wait(timeout=10.0):
        st = srv.stats()
        log("draining: t=%.1f s completed %d / %d" % (time.perf_counter() - t0, st["completed"], st["submitted"]))
    dt.join()
    t_end = time.perf_counter() - t0
    st = srv.stats()
    lat = np.array([srv.poll(i)[1] for i in ids])
    states = np.array([srv.poll(i)[0] for i in ids])
    samples = sum(r["count"] for r in trace)
    srv.close()
    line = {
        "metric": "served level samples/sec at 1 GPU, p50/p99 request latency",
        "value": round(samples / t_end, 1), "unit": "samples/s", "n_gpus": 1,
        "higher_is_better": True, "data": "synthetic",
        "config": {"workload": "serving trace: Poisson arrivals %.0f/s for %.0f s; m uniform on 32..1024 "
                               "(pair (m, m/2) except single at 32), count 1..256, Matern nu in {1/2, 1, 3/2}, "
                               "lambda in [0.02, 0.3], tau 0, embedding grown up to 4x, mixed precision; then drain"
                               % (args.rate, args.duration),
                   "requests": len(trace), "level_samples": samples, "mem_budget_gb": args.mem_gb,
                   "max_inflight": args.max_inflight},
        "requests_per_s": round(len(trace) / t_end, 2),
        "latency_s": {"p50": round(float(np.percentile(lat, 50)), 4), "p99": round(float(np.percentile(lat, 99)), 4),
                      "max": round(float(lat.max()), 4), "per": "request, submit to results in host memory"},
        "wall_s": round(t_end, 2), "arrivals_end_s": round(t_submit_end, 2),
        "completed": int((states == 2).sum()), "failed": int((states < 0).sum()),
        "mem_peak_gb": round(st["mem_peak"] / 2 ** 30, 2),
    }
    print(json.dumps(line), flush=True)


def smoothing_study(args):
    """Smoothing error against the mesh (Section 4.1): the sample mean and
    variance of Q_h - Q~_h (both on one realisation) on meshes h = 1/8 ..
    1/256.  Separable exponential (lambda 0.3 and 0.1, sigma2 1, point QoI
    at (7/15, 7/15)) with tau = sqrt(s); Matern (nu 3/2, lambda 0.1 and
    0.03, sigma2 1, L2 QoI) with tau from the Matern rule, its constants
    from a pilot: alpha and C_alpha from the fit of |E[Q_h - Q_2h]|, C_s
    from E|Q_h - Q~_h| at tau = sqrt(s) divided by its bound.  Prints one
    JSON line."""
    import numpy as np
    import torch
    import paper_2306_13493_amd as ces

    torch.cuda.init()
    ces.load()
    ctx = ces.Context(0)
    meshes = [8, 16, 32, 64, 128, 256]
    n_smp = args.study_samples
    seed = 7
    t_start = time.perf_counter()

    def err(w, m, tau):
        full = ctx.plan(ces.level_desc(**dict(w, m=m, tau_fine=0, tau_coarse=0)))
        sm = ctx.plan(ces.level_desc(**dict(w, m=m, tau_fine=tau, tau_coarse=tau)))
        st = ces.smoothing_error(ctx, full, sm, seed, 0, n_smp)
        n, J = full.info.n, full.info.J
        full.close()
        sm.close()
        return st, n, J

    def slope(h, v):
        ok = [(a, b) for a, b in zip(h, v) if b > 0]
        if len(ok) < 2:
            return None
        x = np.log2([a for a, _ in ok])
        y = np.log2([b for _, b in ok])
        return float(np.polyfit(x, y, 1)[0])

    def table(w, taus):
        rows = []
        for m in meshes:
            probe = ctx.plan(ces.level_desc(**dict(w, m=m)))
            n, J = probe.info.n, probe.info.J
            probe.close()
            tau = taus(m, n, J)
            st, _, _ = err(w, m, tau)
            rows.append({"h": 1.0 / m, "n": n, "J": J, "tau": tau, "mean": st["mean"], "mean_abs": st["mean_abs"],
                         "var": st["var"], "mean_q": st["mean_q"]})
            log("  h=1/%-4d n=%-5d tau=%-7d E[Q-Q~]=% .3e E|Q-Q~|=%.3e V=%.3e" % (m, n, tau, st["mean"],
                                                                            st["mean_abs"], st["var"]))
        h = [r["h"] for r in rows]
        return {"rows": rows, "rate_mean_abs": slope(h, [abs(r["mean"]) for r in rows]),
                "rate_var": slope(h, [r["var"] for r in rows])}

    base = dict(precision="fp64", level="single")
    out = {}
    for lam in (0.3, 0.1):
        w = dict(base, cov="sepexp", lam=lam, qoi="point")
        log("separable exponential lambda=%g, point QoI, tau = sqrt(s)" % lam)
        out["sepexp_lambda_%g" % lam] = table(w, lambda m, n, J: n)
    for lam in (0.1, 0.03):
        w = dict(base, cov="matern", nu=1.5, lam=lam, qoi="l2")
        # pilot: |E[Q_h - Q_2h]| on pair levels, E|Q_h - Q~_h| at tau = sqrt(s)
        hs, dm, cs = [], [], []
        for m in (16, 32, 64):
            p = ctx.plan(ces.level_desc(**dict(w, m=m, level="pair")))
            y = p.sample(seed + 1, 0, n_smp)["y"].cpu().numpy()
            p.close()
            hs.append(1.0 / m)
            dm.append(abs(float(np.mean(y))))
        alpha = max(0.5, slope(hs, dm) or 1.0)
        c_alpha = float(np.mean([d / h ** alpha for h, d in zip(hs, dm)]))
        for m in (16, 32, 64):
            probe = ctx.plan(ces.level_desc(**dict(w, m=m)))
            n, J = probe.info.n, probe.info.J
            probe.close()
            st, _, _ = err(w, m, n)
            s = float(n) * n
            bound = s ** -0.5 * m * (s - n + 1.0) ** (-(1.0 + 1.5) / 2.0) * n
            cs.append(st["mean_abs"] / bound)
        c_s = float(np.mean(cs))
        log("Matern nu=1.5 lambda=%g, L2 QoI: pilot alpha=%.3f C_alpha=%.3e C_s=%.3e" % (lam, alpha, c_alpha, c_s))
        tab = table(w, lambda m, n, J: ces.tau_rule("matern", m, alpha, c_s / c_alpha, nu=1.5, J=J)[0])
        tab["pilot"] = {"alpha": alpha, "C_alpha": c_alpha, "C_s": c_s}
        out["matern_nu1.5_lambda_%g" % lam] = tab
    line = {"metric": "smoothing error E and V of Q_h - Q~_h against h (one realisation per sample)",
            "value": None, "unit": None, "n_gpus": 1, "data": "synthetic", "dtype": "f64",
            "config": {"workload": "meshes h = 1/8 .. 1/256, %d samples per mesh and form, seed %d" % (n_smp, seed)},
            "wall_s": round(time.perf_counter() - t_start, 2), "study": out}
    print(json.dumps(line), flush=True)


def estimators(args):
    """--workload mlqmc: the adaptive MLMC estimator and the multilevel QMC
    estimator (randomly shifted lattice rules, 16 shifts) on one level
    hierarchy (Matern nu 3/2, lambda 0.3, sigma2 1, L2 QoI, m = 8 .. 128,
    Hartley fields, mixed precision), timed to the same RMSE targets.
    Prints one JSON line."""
    import numpy as np
    import torch
    import paper_2306_13493_amd as ces

    torch.cuda.init()
    ces.load()
    ctx = ces.Context(0)
    nlev, shifts, s_dims, log2_points = 5, 16, 256, 11
    w = dict(cov="matern", nu=1.5, lam=0.3, sigma2=1.0, qoi="l2", field="hartley")
    descs = [dict(w, m=8 * 2 ** l, level="single" if l == 0 else "pair", stream=l) for l in range(nlev)]
    mc = [ctx.plan(ces.level_desc(**d)) for d in descs]
    qm = [ctx.plan(ces.level_desc(**d)) for d in descs]
    t0 = time.perf_counter()
    for p in qm:
        p.set_lattice(s=s_dims, log2_points=log2_points, shifts=shifts)
    cbc_s = time.perf_counter() - t0
    log("lattices: %d coordinates, 2^%d points, %d shifts per level; CBC + attach %.2f s" %
        (s_dims, log2_points, shifts, cbc_s))

    def cost(r):
        return float(sum(n * c for n, c in zip(r["n"], r["cost"])))

    def timed(fn):
        torch.cuda.synchronize()
        t = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        return r, time.perf_counter() - t

    # warm both paths (workspaces, graphs) at a loose target
    ces.mlmc_run(ctx, mc, eps=2e-3, l_start=2, n_pilot=100, seed=99)
    ces.mlqmc_run(ctx, qm, eps=2e-3, l_start=2, n_pilot=4, seed=99)
    rows = []
    for eps in (2e-4, 1e-4, 5e-5):
        a, ta = timed(lambda: ces.mlmc_run(ctx, mc, eps=eps, l_start=2, n_pilot=100, seed=1))
        b, tb = timed(lambda: ces.mlqmc_run(ctx, qm, eps=eps, l_start=2, n_pilot=4, seed=1))
        row = {"eps": eps,
               "mlmc": {"s": round(ta, 4), "estimate": a["estimate"], "sqrt_variance": a["variance"] ** 0.5,
                        "levels": a["levels"], "converged": a["converged"], "n": a["n"], "cost": cost(a)},
               "mlqmc": {"s": round(tb, 4), "estimate": b["estimate"], "sqrt_variance": b["variance"] ** 0.5,
                         "levels": b["levels"], "converged": b["converged"], "n": b["n"], "cost": cost(b)}}
        rows.append(row)
        log("eps=%.0e  MLMC %.3f s (N=%s, est %.6f)  MLQMC %.3f s (N=%s, est %.6f)" %
            (eps, ta, a["n"], a["estimate"], tb, b["n"], b["estimate"]))
    last = rows[-1]
    line = {"metric": "seconds to RMSE eps, multilevel QMC vs adaptive MLMC on the same levels",
            "value": last["mlqmc"]["s"], "unit": "s", "n_gpus": 1, "higher_is_better": False,
            "dtype": "f32+f64", "data": "synthetic",
            "config": {"workload": "Matern nu=3/2 lambda=0.3 sigma2=1, L2 QoI, levels m = 8..128, Hartley fields, "
                                   "mixed precision; QMC: %d lattice coordinates, CBC for 2^%d points, %d shifts"
                                   % (s_dims, log2_points, shifts)},
            "speedup_vs_mlmc": round(last["mlmc"]["s"] / max(last["mlqmc"]["s"], 1e-9), 2),
            "cost_ratio_vs_mlmc": round(last["mlmc"]["cost"] / max(last["mlqmc"]["cost"], 1.0), 2),
            "lattice_setup_s": round(cbc_s, 3), "rows": rows}
    print(json.dumps(line), flush=True)


def single_workload(args):
    """--workload c3: the five-level estimator round in one batched call;
    --workload c5: the 2049^2 flow-cell level (Matern 3/2, lambda 0.01,
    outflow QoI).  Prints one JSON line each (level samples per second)."""
    import numpy as np
    import torch
    import paper_2306_13493_amd as ces
    from paper_2306_13493_amd import workloads as W

    torch.cuda.init()
    ces.load()
    ctx = ces.Context(0)
    if args.workload == "c3":
        r = c3_batch(ces, ctx, W, log, reps=max(3, args.steps))
        line = {"metric": "MLMC level samples/sec, five-level batched round at 1 GPU",
                "value": r["level_samples_per_s"], "unit": "samples/s", "n_gpus": 1, "higher_is_better": True,
                "dtype": "f32+f64", "data": "synthetic",
                "config": {"workload": "C3: Matern nu=1/2 lambda=0.03, levels m = 16..256 (pairs above 16), "
                                       "N = 20000/5000/1200/300/80, tau = n below the finest level, mixed precision"},
                "c3_mlmc_batch": r}
        print(json.dumps(line), flush=True)
        return
    # C5: the 2049^2 flow cell at its 1024 samples per call
    r = c5_record(ces, ctx, W, log, steps=max(2, args.steps))
    line = {"metric": r.pop("metric"), "value": r.pop("value"), "unit": r.pop("unit"), "n_gpus": 1,
            "higher_is_better": True, "dtype": "f32+f64", "data": "synthetic", "config": r.pop("config")}
    line.update(r)
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--count", type=int, default=4096, help="samples per step")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--cpu-samples", type=int, default=0)
    ap.add_argument("--no-c3", action="store_true", help="skip the five-level batched estimator record")
    ap.add_argument("--no-c5", action="store_true", help="skip the 2049^2 flow-cell record")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run a plain 1 GiB device copy first (scale for HBM counters)")
    ap.add_argument("--study-samples", type=int, default=512, help="smoothing: samples per mesh and form")
    ap.add_argument("--workload", default="c2", choices=["c2", "c3", "c4", "c5", "smoothing", "mlqmc"],
                    help="c2: throughput of the single-level workload (default); c3: five-level batch; "
                         "c4: serving trace; c5: 2049^2 flow cell; smoothing: smoothing error against the mesh")
    ap.add_argument("--rate", type=float, default=200.0, help="c4: arrivals per second")
    ap.add_argument("--duration", type=float, default=30.0, help="c4: seconds of arrivals")
    ap.add_argument("--mem-gb", type=float, default=200.0, help="c4: server memory budget")
    ap.add_argument("--max-inflight", type=int, default=64, help="c4: admitted requests at most")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(samples would shard by index across GPUs). Use --gpus 1.", file=sys.stderr)
        sys.exit(2)

    if args.workload == "c4":
        serve(args)
        return
    if args.workload == "smoothing":
        smoothing_study(args)
        return
    if args.workload in ("c3", "c5"):
        single_workload(args)
        return
    if args.workload == "mlqmc":
        estimators(args)
        return

    import numpy as np
    import torch
    import paper_2306_13493_amd as ces
    from paper_2306_13493_amd import workloads as W

    torch.cuda.init()
    ces.load()
    if args.copy_calibration:
        a = torch.empty(256 << 20, dtype=torch.float32, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        log("copy calibration: 3 x %d bytes" % (a.numel() * 4))
        del a, b
    ctx = ces.Context(0)
    w = dict(W.C2)
    count = args.count
    t0 = time.perf_counter()
    plan = ctx.plan(ces.level_desc(**w))
    setup_ms = (time.perf_counter() - t0) * 1e3
    log("plan: n=%d J=%d setup %.1f ms" % (plan.info.n, plan.info.J, setup_ms))
    seed = 0
    step_id = 0
    out = None

    def step():
        nonlocal step_id, out
        out = plan.sample(seed, step_id * count, count, out=out)
        step_id += 1

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log("warmup done (%d steps)" % args.warmup)

    # one more untimed step with every launch profiled: the per-kernel
    # table and the dominant kernel; the timed steps then record HIP events
    # around that kernel's launches only (events around every launch cost
    # about 2% of the step)
    ces.profile_only(None)
    ces.profile_enable(True)
    step()
    torch.cuda.synchronize()
    prof_all = ces.profile_read()
    dominant = max(prof_all.items(), key=lambda kv: kv[1][1])[0]
    ces.profile_only(dominant)

    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    iters = []
    ces.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    first_step = step_id
    for k in range(args.steps):
        ev[k][0].record()
        step()
        ev[k][1].record()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = ces.profile_read()
    ces.profile_enable(False)
    ces.profile_only(None)
    step_ms = np.array([a.elapsed_time(b) for a, b in ev])
    it = out["iters"].cpu().numpy()
    status = out["status"].cpu().numpy()
    value = args.steps * count / elapsed
    log("timed: %d steps x %d samples in %.3f s -> %.1f samples/s; CG iterations mean %.2f max %d; failures %d"
        % (args.steps, count, elapsed, value, it.mean(), it.max(), int((status != 0).sum())))

    # the same number of steps again with the launch profiler off (the
    # timed steps carry the dominant kernel's HIP events), reported beside
    # `value`, which keeps the region the roofline comes from
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step()
    torch.cuda.synchronize()
    elapsed_np = time.perf_counter() - t0
    value_np = args.steps * count / elapsed_np
    log("unprofiled: %d steps in %.3f s -> %.1f samples/s" % (args.steps, elapsed_np, value_np))

    roofline, solver_kernels = dominant_roofline(prof, log, prof_all=prof_all)

    # parity of the timed path and the plain FP64 GPU path against the oracle
    extra = {}
    cpu = None
    if not args.no_cpu_baseline:
        # one process per core of the CPU share a one-GPU machine grants (16),
        # however many cores the host shows
        visible = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
        nproc = max(1, min(visible, 16))
        ns = args.cpu_samples or 4 * nproc
        log("cpu baseline: oracle on %d samples with %d processes ..." % (ns, nproc))
        y_ref, dt = cpu_baseline(w, seed, ns, nproc)
        y_ref = np.array(y_ref)
        # same samples on the GPU (indices 0 .. ns-1)
        g = plan.sample(seed, 0, ns)["y"].cpu().numpy()
        rel = float(np.max(np.abs(g - y_ref) / np.abs(y_ref)))
        cpu = {"value": round(ns / dt, 3), "unit": "samples/s", "cores": nproc, "kind": "oracle",
               "sample": "samples 0..%d of the same workload (seed 0), FP64 NumPy/SciPy (SuperLU), "
                         "%d processes x 1 thread, wall %.1f s" % (ns - 1, nproc, dt),
               "cpu_model": cpu_model(), "host_cpus_visible": os.cpu_count()}
        extra["parity_vs_oracle_max_rel"] = rel
        log("cpu baseline %.3f samples/s; GPU vs oracle max rel diff %.2e" % (ns / dt, rel))
    if not args.no_cpu_baseline:
        extra["parity_vs_oracle"] = parity_per_result(ces, plan, w, seed, log)
        extra["parity_vs_oracle"]["qoi_max_rel_diff"] = extra["parity_vs_oracle_max_rel"]
    if not args.no_fp64:
        p64 = ctx.plan(ces.level_desc(**dict(w, precision="fp64")))
        o64 = p64.sample(seed, 0, count)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        nrep = max(1, args.steps // 3)
        for r in range(nrep):
            o64 = p64.sample(seed, r * count, count, out=o64)
        torch.cuda.synchronize()
        v64 = nrep * count / (time.perf_counter() - t1)
        om = plan.sample(seed, (nrep - 1) * count, count)
        diff = float(torch.max(torch.abs(om["y"] - o64["y"]) / torch.abs(o64["y"])).item())
        # the plain FP64 path one sample per call (no batching), with the
        # default cycle and with the V-cycle (fewer launches per iteration)
        n1 = 32
        y1 = torch.empty(1, dtype=torch.float64, device="cuda")
        pv = ctx.plan(ces.level_desc(**dict(w, precision="fp64", cycle="v")))

        def one_per_call(pp):
            pp.lib.ces_sample(pp.handle, seed, 0, 1, ces._ptr(y1), None, None, None, None, ces._stream_ptr(None))
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for i in range(n1):
                pp.lib.ces_sample(pp.handle, seed, i, 1, ces._ptr(y1), None, None, None, None,
                                  ces._stream_ptr(None))
            torch.cuda.synchronize()
            return n1 / (time.perf_counter() - t1)

        v1 = one_per_call(p64)
        v1v = one_per_call(pv)
        extra["fp64_plain_path"] = {"value": round(v64, 1), "unit": "samples/s",
                                    "mixed_vs_fp64_max_rel_diff_Y": diff,
                                    "one_sample_per_call": {"value": round(v1, 1), "unit": "samples/s",
                                                            "samples": n1, "v_cycle": round(v1v, 1)}}
        log("plain FP64 path %.1f samples/s batched, %.1f samples/s one per call (%.1f with the V-cycle); "
            "mixed vs FP64 max rel diff %.2e" % (v64, v1, v1v, diff))

    if not args.no_c3:
        extra["c3_mlmc_batch"] = c3_batch(ces, ctx, W, log)
    if not args.no_c5:
        extra["c5_flowcell"] = c5_record(ces, ctx, W, log)

    line = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(float(elapsed * 1e3 / args.steps), 3),
        "unprofiled": {"value": round(value_np, 1), "ms_per_step": round(float(elapsed_np * 1e3 / args.steps), 3)},
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": "Matern nu=1 lambda=0.1 sigma2=1, 257x257 vertices, embedding 512x512 "
                               "(grown to nonnegative), %d i.i.d. samples per step, f=1, u=0 on the boundary, "
                               "QoI integral of u, float field+multigrid, double CG to 1e-10" % count,
                   "samples_per_step": count, "precision": "mixed"},
        "latency_ms": {"p50": round(float(np.percentile(step_ms, 50)), 3),
                       "p99": round(float(np.percentile(step_ms, 99)), 3),
                       "per": "step of %d samples" % count},
        "setup_ms": round(setup_ms, 2),
        "cg_iterations_mean": round(float(it.mean()), 3),
        "roofline": roofline,
        "kernels": solver_kernels,
        "cpu_baseline": cpu,
    }
    line.update(extra)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
