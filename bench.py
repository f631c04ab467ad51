#!/usr/bin/env python3
"""Adaptive FSAI setup + PCG time-to-solution on one MI355X.

One step = one adaptive FSAI setup of G plus one PCG solve of A x = b to rtol 1e-8 (x0 = 0) on
a synthetic workload already resident in HBM; the handle is destroyed after each step.
Default workload: the largest single-GPU configuration, a 27-point 3-dof heterogeneous SPD
operator on 150^3 nodes (10,125,000 unknowns, 809,238,528 nonzeros, log-normal sigma = 2 cell
coefficients), k_max = 15, s = 3, eps = 1e-2, G stored in FP32 with the per-row Cholesky and
the PCG in FP64.  The line also carries the 64^3 workload (786,432 unknowns, sigma = 1,
k_max = 10, s = 2, FP64) under ``context``.

Prints ONE JSON line.  ``value`` is the wall time of one solve (seconds, lower is better).
``roofline`` covers the kernel with the largest total event-measured time in one untimed
profiled step; inside the timed region only that kernel is bracketed by HIP events (on its
launch stream), and its average launch duration there gives ``achieved``.  ``kernels`` is the
per-kernel breakdown of the profiled step.  ``cpu_baseline`` times the FP64 CPU oracle on the
same workload (host cores): whole for up to 2M rows, on a stated sample above.
"""
from __future__ import annotations

import argparse
import contextlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "aFSAI setup+PCG s to rtol 1e-8, HBM GB/s; p50/p99 latency vs plain"
PEAK_HBM_GBS = 8000.0


BATCH_WORKLOADS = {"aniso_batch512": 512}


def batch_bench(args):
    """Batching form: one step = afsai_setup_batched + pcg_solve_batched over the whole batch of
    anisotropic 7-point systems (sides U{10..40}, k_max = 5, s = 1, eps = 1e-2, rtol = 1e-8);
    "plain" = the same systems set up and solved one after another with afsai_setup + pcg_solve."""
    import torch

    import paper_2010_14175_amd as af
    import synth

    nsys = BATCH_WORKLOADS[args.workload]
    probs = synth.aniso_batch(nsys=nsys, seed=3, side_lo=10, side_hi=40, kmax=5, s=1)
    A, off, b_h, _ = synth.block_diag(probs)
    print(f"[bench] workload {args.workload}: {nsys} systems, n={A.n} nnz={A.nnz}", file=sys.stderr, flush=True)
    dA = af.DeviceCSR.from_host(A)
    b = torch.from_numpy(b_h).cuda()
    x = torch.zeros_like(b)
    choice = None
    if args.tune:
        from paper_2010_14175_amd import tune

        choice = tune.autotune(dA, 5, 1, 1e-2, b, offsets=off, reps=2, cache=args.tune_cache)
        print(f"[bench] tuned: {choice}", file=sys.stderr, flush=True)

    def step():
        P = af.setup_batched(dA, off, 5, 1, 1e-2)
        x.zero_()
        _, infos = af.pcg_solve_batched(dA, P, off, b, x=x, rtol=1e-8)
        sinfo = P.info()
        P.close()
        return sinfo, infos

    ctx = tune.apply(choice) if choice else contextlib.nullcontext()
    with ctx:
        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        kern, kern_raw = {}, {}
        if not args.no_profile:
            # per-kernel breakdown from one untimed profiled step; inside the timed steps only
            # the dominant kernel carries events (on its launch stream)
            af.profile_only(None)
            af.profile_read(reset=True)
            af.profile_enable(True)
            step()
            torch.cuda.synchronize()
            af.profile_enable(False)
            kern_raw = af.profile_read(reset=True)
            kern = {k: {"launches": v[0], "total_ms": round(v[1], 3), "avg_us": round(v[1] / max(1, v[0]) * 1e3, 2)}
                    for k, v in kern_raw.items()}
            dom = max(kern_raw.items(), key=lambda kv: kv[1][1])[0]
            af.profile_only([dom])
            af.profile_enable(True)
        t0 = time.perf_counter()
        for _ in range(args.steps):
            sinfo, infos = step()
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t0) / args.steps
        kern_timed = {}
        if not args.no_profile:
            af.profile_enable(False)
            kern_timed = af.profile_read(reset=True)
            af.profile_only(None)
        # G of the batch for the per-system algorithmic bytes
        Pg = af.setup_batched(dA, off, 5, 1, 1e-2)
        g_rp = Pg.export()[0].cpu().numpy()
        Pg.close()
    its = np.array([i.iters for i in infos])
    worst = max(i.true_relres for i in infos)
    # plain form, one system after another (timed once after one warm-up system)
    singles = [(af.DeviceCSR.from_host(pb.A), torch.from_numpy(pb.b).cuda()) for pb in probs]
    af.pcg_solve(singles[0][0], af.setup(singles[0][0], 5, 1, 1e-2), singles[0][1])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for dk, bk in singles:
        Pk = af.setup(dk, 5, 1, 1e-2)
        af.pcg_solve(dk, Pk, bk, rtol=1e-8)
        Pk.close()
    torch.cuda.synchronize()
    plain = time.perf_counter() - t0
    print(f"[bench] {args.steps} steps: {sec * 1e3:.2f} ms/step batched (setup {sinfo.ms:.2f} ms, pcg "
          f"{infos[0].ms:.2f} ms, iterations {its.min()}..{its.max()}, worst true relres {worst:.2e}); "
          f"plain one by one {plain * 1e3:.1f} ms", file=sys.stderr, flush=True)
    # aggregate PCG bandwidth: every system's algorithmic bytes per iteration (A, G and G^T once,
    # row pointers, 15 vector passes) times its own iterations, over the batched solve's time
    a_rp = A.row_ptr
    sys_bytes = 0.0
    for k in range(nsys):
        o0, o1 = int(off[k]), int(off[k + 1])
        nk, nnz_a, nnz_g = o1 - o0, int(a_rp[o1] - a_rp[o0]), int(g_rp[o1] - g_rp[o0])
        per_it = 12.0 * nnz_a + 2 * (8 + 4) * nnz_g + 3 * 4 * (nk + 1) + 15 * 8 * nk
        sys_bytes += per_it * int(infos[k].iters)
    pcg_gbs = sys_bytes / (infos[0].ms * 1e-3) / 1e9
    pcg_roof = {"kernel": "pcg (all systems, aggregate)", "bound": "hbm", "achieved": round(pcg_gbs, 1),
                "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": round(pcg_gbs / PEAK_HBM_GBS, 4),
                "bytes": sys_bytes, "pcg_ms": round(infos[0].ms, 3)}
    roof = None
    if kern_timed:
        dom, (launches, ms) = max(kern_timed.items(), key=lambda kv: kv[1][1])
        avg_s = ms / launches * 1e-3
        byt = kernel_bytes(dom, A.n, A.nnz, int(g_rp[-1]), 8, 5, 6)
        ach = byt / avg_s / 1e9
        roof = {"kernel": dom, "bound": "hbm", "achieved": round(ach, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": round(ach / PEAK_HBM_GBS, 4), "traffic": measured_traffic(dom, args.workload),
                "bytes_per_launch": byt, "avg_launch_us": round(avg_s * 1e6, 2)}
    print(f"[bench] aggregate PCG {pcg_gbs:.0f} GB/s ({pcg_gbs / PEAK_HBM_GBS:.3f} of peak)", file=sys.stderr,
          flush=True)
    out = {"metric": METRIC, "value": round(sec, 6), "unit": "s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(sec * 1e3, 3), "higher_is_better": False, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": args.workload, "systems": nsys, "n": A.n, "nnz": A.nnz, "kmax": 5, "s": 1,
                      "eps": 1e-2, "rtol": 1e-8},
           "setup_ms": round(sinfo.ms, 3), "pcg_ms": round(infos[0].ms, 3), "iters_min": int(its.min()),
           "iters_max": int(its.max()), "worst_true_relres": worst, "plain_one_by_one_s": round(plain, 4),
           "speedup_vs_plain": round(plain / sec, 2), "roofline": roof, "pcg_roofline": pcg_roof, "kernels": kern,
           "tuned": choice, "cpu_baseline": None}
    print(json.dumps(out), flush=True)


def serve_bench(args):
    """Serving form: Poisson arrivals of SPD systems, n log-uniform in [1e4, 2e6], half 7-point
    (log-normal sigma = 1 cell coefficients, k_max = 5, s = 1), half 27-point 3-dof (the 64^3
    workload's construction, k_max = 10, s = 2), FP32 G, FP64 PCG to rtol 1e-8, x0 = 0.  Matrices come from
    a seeded pool of distinct systems; every request gets its own right-hand side b = A x with
    x ~ U(-1, 1).  The plain form serves one request at a time in arrival order (one slot);
    continuous batching admits up to 16 requests by memory.  Loads are 0.5 and 0.8 of the plain
    form's saturation throughput."""
    import torch

    import paper_2010_14175_amd as af
    import synth

    nreq, npool = args.requests, args.pool
    u = synth.uniform(4, 40, 3 * npool, 0.0, 1.0).reshape(npool, 3)
    pool = []
    for k in range(npool):
        n_want = math.exp(math.log(1e4) + u[k, 0] * (math.log(2e6) - math.log(1e4)))
        if u[k, 1] < 0.5:
            N = max(4, round(n_want ** (1 / 3)))
            A = synth.lap7_lognormal(N, N, N, 1.0, 100 + k)
            kind, kmax, s = "7pt", 5, 1
        else:
            N = max(3, round((n_want / 3) ** (1 / 3)))
            A = synth.elast27(N, 1.0, 200 + k)
            kind, kmax, s = "27pt", 10, 2
        pool.append((kind, kmax, s, af.DeviceCSR.from_host(A), A.n))
    print(f"[bench] serve: pool of {npool} systems, n = {sorted(p[4] for p in pool)}", file=sys.stderr, flush=True)
    pick = (synth.uniform(4, 41, nreq, 0.0, 1.0) * npool).astype(np.int64) % npool
    # right-hand sides on the device: b = A x, x ~ U(-1, 1) seeded per request
    gen = torch.Generator(device="cuda")
    bs = []
    for q in range(nreq):
        dA = pool[pick[q]][3]
        gen.manual_seed(1000 + q)
        xq = torch.rand(dA.n, dtype=torch.float64, device="cuda", generator=gen) * 2 - 1
        bs.append(af.spmv(dA, xq))
    torch.cuda.synchronize()

    def run(slots, arrivals, max_heavy=0):
        """Serves the requests arriving at `arrivals` (s) with `slots` slots; latency = completion
        minus arrival."""
        srv = af.Server(args.budget_gb * 2**30, slots, 5, 1, 1e-2, rtol=1e-8, g_prec=af.F32,
                        setup_threads=4 if slots > 1 else 1, max_heavy=max_heavy)
        xs = [torch.empty_like(b) for b in bs]
        t0 = time.perf_counter()
        sub, lat, bad = {}, [], 0
        q = done = 0
        while done < nreq:
            while q < nreq and arrivals[q] <= time.perf_counter() - t0:
                _, kmax, s_, dA, _ = pool[pick[q]]
                t = srv.submit(dA, bs[q], xs[q], kmax=kmax, s=s_)
                sub[t] = (arrivals[q], time.perf_counter() - t0)
                q += 1
            for r in srv.poll(wait_ms=0):
                arr, ts = sub.pop(r.ticket)
                lat.append((r.done_ms - r.submit_ms) / 1e3 + (ts - arr))
                bad += int(r.status != af.OK or not r.converged)
                done += 1
            if q < nreq:
                time.sleep(max(0.0, min(0.002, arrivals[q] - (time.perf_counter() - t0))))
            elif done < nreq:
                time.sleep(0.0005)
        span = time.perf_counter() - t0
        srv.close()
        return np.array(lat), span, bad

    # saturation throughput of the plain form: every request present at t = 0
    _, span0, bad0 = run(1, np.zeros(nreq))
    sat = nreq / span0
    print(f"[bench] plain saturation: {sat:.2f} solves/s ({span0:.1f} s for {nreq})", file=sys.stderr, flush=True)
    res = {"plain_saturation_solves_per_s": round(sat, 3)}
    rng_u = synth.uniform(4, 42, nreq, 1e-12, 1.0)
    for load in (0.5, 0.8):
        qps = load * sat
        arrivals = np.cumsum(-np.log(rng_u) / qps)
        runs = [("plain_fifo", 1, 0)] + [(f"continuous{k}", k, 0) for k in args.serve_slots]
        if args.serve_uncapped:
            runs += [(f"continuous{k}_uncapped", k, -1) for k in args.serve_slots]
        for mh in args.serve_heavy:
            runs += [(f"continuous{k}_heavy{mh}", k, mh) for k in args.serve_slots]
        for name, slots, mh in runs:
            lat, span, bad = run(slots, arrivals, mh)
            key = f"{name}@{load}"
            res[key] = {"qps": round(qps, 3), "slots": slots, "max_heavy": mh, "mean_s": round(float(lat.mean()), 4),
                        "p50_s": round(float(np.percentile(lat, 50)), 4),
                        "p99_s": round(float(np.percentile(lat, 99)), 4), "solves_per_s": round(nreq / span, 3),
                        "failed": bad}
            print(f"[bench] {key}: mean {res[key]['mean_s']} s, p50 {res[key]['p50_s']} s, p99 {res[key]['p99_s']} s, "
                  f"{res[key]['solves_per_s']} solves/s", file=sys.stderr, flush=True)
    best = min((k for k in res if k.startswith("continuous") and k.endswith("@0.8") and "_" not in k.split("@")[0]),
               key=lambda k: res[k]["p99_s"])
    out = {"metric": METRIC, "value": res[best]["p99_s"], "unit": f"s (p99 latency, {best})",
           "n_gpus": 1, "steps": nreq, "warmup": 0, "higher_is_better": False, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64 (G stored f32)", "data": "synthetic",
           "config": {"workload": "serve", "requests": nreq, "pool": npool, "n_range": [1e4, 2e6],
                      "budget_gb": args.budget_gb},
           "serving": res, "roofline": None, "cpu_baseline": None}
    print(json.dumps(out), flush=True)


def jacobi_bench(args):
    """aFSAI against Jacobi (k_max = 0: G = D^-1/2, M^-1 = D^-1) time to solution, rtol 1e-8,
    x0 = 0, on the 7-point 20^3 and 121^3 problems, the 27-point 64^3 workload and, with
    --with-largest, the 27-point 150^3 one.  One step = setup + PCG; median of the steps."""
    import torch

    import paper_2010_14175_amd as af

    names = ["poisson7_20", "poisson7_121", "elast27_64"] + (["elast27_150"] if args.with_largest else [])
    res = {}
    for name in names:
        pb = workloads()[name]()
        g_prec = af.F32 if name == "elast27_150" else af.F64
        dA = af.DeviceCSR.from_host(pb.A)
        b = torch.from_numpy(pb.b).cuda()
        x = torch.zeros_like(b)
        row = {"n": pb.n, "nnz": pb.A.nnz}
        for label, kmax in (("afsai", pb.kmax), ("jacobi", 0)):
            tot, st, pc, its = [], [], [], 0
            for k in range(args.warmup + args.steps):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                P = af.setup(dA, kmax, pb.s, pb.eps, g_prec=g_prec)
                x.zero_()
                _, info = af.pcg_solve(dA, P, b, x=x, rtol=pb.rtol, maxit=20 * pb.n)
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                sinfo = P.info()
                P.close()
                if k >= args.warmup:
                    tot.append((t1 - t0) * 1e3)
                    st.append(sinfo.ms)
                    pc.append(info.ms)
                its = info.iters
            row[label] = {"ms": round(float(np.median(tot)), 3), "setup_ms": round(float(np.median(st)), 3),
                          "pcg_ms": round(float(np.median(pc)), 3), "iters": its, "nnz_g": sinfo.nnz_g,
                          "true_relres": info.true_relres, "converged": info.converged}
            print(f"[bench] {name} {label}: {row[label]['ms']:.2f} ms (setup {row[label]['setup_ms']:.2f}, pcg "
                  f"{row[label]['pcg_ms']:.2f}), {its} iterations, true relres {info.true_relres:.2e}",
                  file=sys.stderr, flush=True)
        row["time_ratio"] = round(row["jacobi"]["ms"] / row["afsai"]["ms"], 3)
        row["iter_ratio"] = round(row["jacobi"]["iters"] / max(1, row["afsai"]["iters"]), 3)
        res[name] = row
    out = {"metric": "time to solution, Jacobi-PCG / aFSAI-PCG (rtol 1e-8)", "value": res["elast27_64"]["time_ratio"],
           "unit": "ratio", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "higher_is_better": True,
           "vs_baseline": None, "dtype": "f64", "data": "synthetic", "config": {"workload": "jacobi_compare"},
           "results": res}
    print(json.dumps(out), flush=True)


def spmm_bench(args):
    """Y = A X for blocks of 1, 2, 4 and 8 right-hand sides with A of the 27-point 64^3
    workload: the product kernel's time per block (HIP events on its launch stream, median of
    the steps) and per right-hand side, and its algorithmic bytes (every matrix entry once, X
    and Y once) over that time; beside it the wall time of a whole call, unprepared (A
    converted to its SELL layout in the call) and with a prepared A."""
    import torch

    import paper_2010_14175_amd as af
    import synth

    pb = workloads()["elast27_64"]()
    dA = af.DeviceCSR.from_host(pb.A)
    n, nnz = pb.n, pb.A.nnz
    X8 = torch.from_numpy(synth.uniform(13, 5, n * 8, -1.0, 1.0).reshape(n, 8)).cuda()
    M = af.PreparedMatrix(dA)

    def wall_ms(fn):
        ms = []
        for _ in range(args.steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            ms.append((time.perf_counter() - t0) * 1e3)
        return float(np.median(ms))

    res = {}
    for k in (1, 2, 4, 8):
        X = X8[:, :k].contiguous()
        Y = torch.empty_like(X)
        for _ in range(args.warmup):
            af.spmm(dA, X, Y)
        torch.cuda.synchronize()
        af.profile_only(["spmm_A"])
        us = []
        try:
            for _ in range(args.steps):
                af.profile_read(reset=True)
                af.profile_enable(True)
                af.spmm(dA, X, Y)
                af.profile_enable(False)
                us.append(af.profile_read(reset=True)["spmm_A"][1] * 1e3)
        finally:
            af.profile_enable(False)
            af.profile_only(None)
        t = float(np.median(us))
        byt = 12.0 * nnz + 4.0 * (n + 1) + 16.0 * k * n
        for _ in range(args.warmup):
            M.spmm(X, Y)
        w_un, w_pr = wall_ms(lambda: af.spmm(dA, X, Y)), wall_ms(lambda: M.spmm(X, Y))
        res[f"k{k}"] = {"us": round(t, 2), "us_per_rhs": round(t / k, 2), "gbs": round(byt / (t * 1e-6) / 1e9, 1),
                        "bytes": byt, "wall_us": round(w_un * 1e3, 1), "wall_us_prepared": round(w_pr * 1e3, 1)}
        print(f"[bench] spmm k={k}: {t:.1f} us ({t / k:.1f} us per right-hand side, "
              f"{res[f'k{k}']['gbs']} GB/s algorithmic); wall per call {w_un * 1e3:.1f} us, prepared "
              f"{w_pr * 1e3:.1f} us", file=sys.stderr, flush=True)
    # PCG over blocks (one setup reused): wall time of the solve per right-hand side, against
    # pcg_solve of one right-hand side
    P = af.setup(dA, pb.kmax, pb.s, pb.eps)
    Bt = torch.from_numpy(np.ascontiguousarray(
        np.column_stack([pb.A.to_scipy() @ synth.uniform(17, 3 + j, n, -1.0, 1.0) for j in range(8)]))).cuda()
    solves = {}
    b0 = Bt[:, 0].contiguous()
    for _ in range(args.warmup):
        af.pcg_solve(dA, P, b0, rtol=pb.rtol)
    ms = []
    for _ in range(args.steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, inf1 = af.pcg_solve(dA, P, b0, rtol=pb.rtol)
        torch.cuda.synchronize()
        ms.append((time.perf_counter() - t0) * 1e3)
    solves["pcg_solve"] = {"ms": round(float(np.median(ms)), 3), "iters": inf1.iters}
    for _ in range(args.warmup):
        M.pcg_solve(P, b0, rtol=pb.rtol)
    solves["pcg_solve_prepared"] = {"ms": round(wall_ms(lambda: M.pcg_solve(P, b0, rtol=pb.rtol)), 3)}
    for k in (1, 8):
        B = Bt[:, :k].contiguous()
        for _ in range(args.warmup):
            af.pcg_solve_multi(dA, P, B, rtol=pb.rtol)
        ms = []
        for _ in range(args.steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, infs = af.pcg_solve_multi(dA, P, B, rtol=pb.rtol)
            torch.cuda.synchronize()
            ms.append((time.perf_counter() - t0) * 1e3)
        t = float(np.median(ms))
        solves[f"multi_k{k}"] = {"ms": round(t, 3), "ms_per_rhs": round(t / k, 3),
                                 "iters": [i.iters for i in infs], "worst_true_relres": max(i.true_relres for i in infs)}
        print(f"[bench] pcg_solve_multi k={k}: {t:.2f} ms ({t / k:.2f} ms per right-hand side, iterations "
              f"{[i.iters for i in infs]})", file=sys.stderr, flush=True)
    print(f"[bench] pcg_solve: {solves['pcg_solve']['ms']:.2f} ms ({inf1.iters} iterations), prepared A "
          f"{solves['pcg_solve_prepared']['ms']:.2f} ms", file=sys.stderr, flush=True)
    P.close()
    M.close()
    res["pcg"] = solves
    out = {"metric": "SpMM time per right-hand side, k = 8 against k = 1", "value":
           round(res["k8"]["us_per_rhs"] / res["k1"]["us"], 4), "unit": "ratio", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "higher_is_better": False, "vs_baseline": None, "dtype": "f64",
           "data": "synthetic", "config": {"workload": "spmm", "n": n, "nnz": nnz}, "results": res}
    print(json.dumps(out), flush=True)


def workloads():
    import synth

    return {
        "elast27_64": lambda: synth.elasticity27(64, 1.0, 2, kmax=10, s=2),
        "poisson7_20": lambda: synth.poisson7(20, 1, kmax=5, s=1),
        "elast27_150": lambda: synth.elasticity27(150, 2.0, 5, kmax=15, s=3),
        "poisson7_121": lambda: synth.poisson7(121, 6, kmax=5, s=1),
    }


def kernel_bytes(name: str, n: int, nnz_a: int, nnz_g: int, w_g: int, kmax: int, mmax: int) -> float:
    """Algorithmic HBM bytes of one launch of each kernel (every matrix entry and vector element
    counted once per launch; caches assumed perfect for gathered vector entries)."""
    vec = 8.0 * n
    rp = 4.0 * (n + 1)
    table = {
        "spmv_A": 12.0 * nnz_a + rp + 2 * vec,           # A, x, y
        "spmv_A_dot": 12.0 * nnz_a + rp + 3 * vec,       # + w for the fused dot
        "spmv_G": (4.0 + w_g) * nnz_g + rp + 2 * vec,
        "spmv_GT_dot": (4.0 + w_g) * nnz_g + rp + 3 * vec,
        "update_xr": 6 * vec,                            # read x p r q, write x r
        "update_p": 3 * vec,                             # read z p, write p
        # setup: every growth step reads the rows of the pattern once (k_max passes over A at
        # most) and the padded per-row results are written once
        "afsai_rows": kmax * 12.0 * nnz_a + n * mmax * 12.0 + n * 24.0,
    }
    return table.get(name, float("nan"))


def cpu_baseline(pb, iters_hint: int, threads: int, x_gpu=None) -> dict:
    """The FP64 oracle on the whole workload: its setup of every row, then its PCG to rtol."""
    import oracle

    oracle.set_threads(threads)
    t0 = time.perf_counter()
    G = oracle.setup(pb.A, pb.kmax, pb.s, pb.eps, nthreads=threads)
    t1 = time.perf_counter()
    res = oracle.pcg(pb.A, G, pb.b, pb.rtol)
    t2 = time.perf_counter()
    return {"value": round(t2 - t0, 3), "unit": "s", "cores": threads, "kind": "oracle",
            "sample": (f"whole workload: oracle setup of all {pb.n} rows ({t1 - t0:.2f} s, {threads} threads) + "
                       f"oracle PCG to rtol {pb.rtol:g} ({res.iters} iterations, {t2 - t1:.2f} s; "
                       f"GPU took {iters_hint})"),
            "setup_s": round(t1 - t0, 3), "pcg_s": round(t2 - t1, 3), "iters": res.iters,
            "gpu_x_rel_err_vs_oracle": (float(np.linalg.norm(x_gpu - res.x) / np.linalg.norm(res.x))
                                        if x_gpu is not None else None)}


def leading_block(A, ns: int):
    """The leading principal ns x ns block of a CSR matrix (rows and columns below ns).  Rows of
    G depend only on A's entries of lower index, so its setup gives rows 0..ns-1 of G exactly."""
    import synth

    e = int(A.row_ptr[ns])
    col = A.col[:e]
    keep = col < ns
    rows = np.repeat(np.arange(ns, dtype=np.int64), np.diff(A.row_ptr[:ns + 1]))[keep]
    rp = np.zeros(ns + 1, np.int64)
    np.add.at(rp, rows + 1, 1)
    return synth.CSR(np.cumsum(rp).astype(np.int32), col[keep].astype(np.int32), A.val[:e][keep].astype(np.float64))


def cpu_baseline_sampled(pb, iters_gpu: int, nnz_g_gpu: int, threads: int, setup_stride: int = 64,
                         slab_div: int = 64, pcg_iters: int = 10) -> dict:
    """The FP64 oracle on a bounded sample of a workload too large to run whole (the oracle's
    setup of all 10.1M rows of the 150^3 problem alone takes minutes on the host):

    * setup: every ``setup_stride``-th row (rows are independent), timed, scaled by the number
      of rows;
    * PCG: ``pcg_iters`` oracle iterations on the leading principal block of n / slab_div rows
      with the oracle's G of that block (its rows are the first rows of the full G), the time
      per iteration scaled by the ratio of the whole problem's matrix entries (A, G and G^T) to
      the block's, times the GPU's iteration count."""
    import oracle

    oracle.set_threads(threads)
    n = pb.n
    rows = np.arange(0, n, setup_stride, dtype=np.int32)
    t0 = time.perf_counter()
    oracle.setup_rows(pb.A, pb.kmax, pb.s, pb.eps, rows=rows, nthreads=threads)
    t_rows = time.perf_counter() - t0
    setup_s = t_rows * n / len(rows)
    ns = n // slab_div
    As = leading_block(pb.A, ns)
    Gs = oracle.setup(As, pb.kmax, pb.s, pb.eps, nthreads=threads)
    bs = oracle.spmv(As, pb.x_true[:ns])
    t1 = time.perf_counter()
    r = oracle.pcg(As, Gs, bs, 1e-30, maxit=pcg_iters)
    t_it = (time.perf_counter() - t1) / max(1, r.iters)
    scale = (pb.A.nnz + 2.0 * nnz_g_gpu) / (As.nnz + 2.0 * Gs.nnz)
    pcg_s = t_it * scale * iters_gpu
    return {"value": round(setup_s + pcg_s, 3), "unit": "s", "cores": threads, "kind": "oracle",
            "sample": (f"oracle setup of every {setup_stride}th row ({len(rows)} of {n} rows, {t_rows:.2f} s, "
                       f"scaled by rows) + {r.iters} oracle PCG iterations on the leading {ns}-row principal block "
                       f"({t_it * 1e3:.1f} ms each, scaled by matrix entries x{scale:.1f} to the whole problem, times "
                       f"the GPU's {iters_gpu} iterations); {threads} threads"),
            "setup_s": round(setup_s, 3), "pcg_s": round(pcg_s, 3), "iters": iters_gpu,
            "sample_setup_s": round(t_rows, 3), "sample_pcg_s_per_iter": round(t_it, 5)}


COPY_BYTES = 1 << 30


def copy_check():
    """A plain device copy of COPY_BYTES, five times: its FETCH_SIZE / WRITE_SIZE per dispatch
    under rocprofv3 give the scale from counter units to bytes."""
    import torch

    a = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": COPY_BYTES, "dispatches": 5}), flush=True)


def kernel_source_hash(kernel: str) -> str | None:
    """Hash of the sources a kernel is built from (stored beside its counter summary, so that
    counter-derived traffic is only reported for the code that was measured)."""
    import hashlib

    files = {"afsai_rows": ["rows.hpp", "rows.hip", "rows_reg.hip", "rows_lds.hip", "rows_f32.hip", "rows_w.hpp",
                           "rows_w.hip", "rows_w_inst.hpp", "rows_w_g32.hip"]}.get(kernel)
    if not files:
        return None
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_2010_14175_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_value(kernel: str, workload: str, summary: str, key: str):
    """A value of the committed counter summary profiles/{kernel}_{workload}_{summary}.md, or
    None when there is none or the kernel's sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_{summary}.md")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and line.startswith("- "):
                k, v = line[2:].split(":", 1)
                vals[k.strip()] = v.strip().strip("`")
    if vals.get("source_hash") != kernel_source_hash(kernel):
        return None
    try:
        return float(vals[key])
    except (KeyError, ValueError):
        return None


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch from the committed FETCH_SIZE / WRITE_SIZE summary."""
    return measured_value(kernel, workload, "traffic", "hbm_bytes_per_launch")


# VALU issue: a wave64 VALU instruction occupies its SIMD for 4 cycles; 256 CUs x 4 SIMDs at
# 2.4 GHz
PEAK_VALU_GINST = 256 * 4 * 2.4 / 4


# G storage each workload is specified with (the 150^3 one: FP32 G with FP64 Cholesky + PCG)
WORKLOAD_G_PREC = {"elast27_150": "f32"}
# above this many rows the oracle is timed on a sample instead of the whole workload
CPU_WHOLE_MAX_ROWS = 2_000_000


def run_workload(af, pb, g_prec, args, steps: int, warmup: int, profile: bool, with_cpu: bool,
                 workload_name: str, with_forms: bool = False, forms_steps: int = 3) -> dict:
    """One workload: ``warmup`` untimed steps, one untimed profiled step (per-kernel breakdown,
    dominant kernel), then ``steps`` timed steps with events only around the dominant kernel.
    Returns the fields of the JSON line (without the common header)."""
    import torch

    dA = af.DeviceCSR.from_host(pb.A)
    b = torch.from_numpy(pb.b).cuda()
    x = torch.zeros_like(b)

    def step():
        P = af.setup(dA, pb.kmax, pb.s, pb.eps, g_prec=g_prec, setup_f32=args.setup_f32, grad_f32=args.grad_f32)
        x.zero_()
        _, info = af.pcg_solve(dA, P, b, x=x, rtol=pb.rtol)
        sinfo = P.info()
        P.close()
        return sinfo, info

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()

    kern_all = {}
    dom = None
    if profile:
        # one untimed step with every kernel timed: the per-kernel breakdown and the dominant
        # kernel; inside the timed region only the dominant kernel carries events
        af.profile_only(None)
        af.profile_read(reset=True)
        af.profile_enable(True)
        step()
        torch.cuda.synchronize()
        af.profile_enable(False)
        kern_all = af.profile_read(reset=True)
        dom = max(kern_all.items(), key=lambda kv: kv[1][1])[0]
        af.profile_only([dom])
        af.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    setup_ms, pcg_ms, its = [], [], []
    for k in range(steps):
        sinfo, info = step()
        setup_ms.append(sinfo.ms)
        pcg_ms.append(info.ms)
        its.append(info.iters)
        print(f"[bench] {workload_name} step {k + 1}/{steps}: setup {sinfo.ms:.1f} ms, pcg {info.ms:.1f} ms, "
              f"{info.iters} iterations", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kern = {}
    if profile:
        af.profile_enable(False)
        kern = af.profile_read(reset=True)
        af.profile_only(None)
    sec = (t1 - t0) / steps
    print(f"[bench] {workload_name}: {steps} steps: {sec * 1e3:.2f} ms/step (setup {np.mean(setup_ms):.2f} ms, "
          f"pcg {np.mean(pcg_ms):.2f} ms, {its[-1]} iterations, true relres {info.true_relres:.2e})",
          file=sys.stderr, flush=True)

    w_g = 4 if g_prec == af.F32 else 8
    roof = None
    issue_roof = None
    kern_report = {}
    for name, (launches, ms) in kern_all.items():
        byt = kernel_bytes(name, pb.n, pb.A.nnz, sinfo.nnz_g, w_g, pb.kmax, sinfo.mmax)
        avg_ms = ms / max(1, launches)
        kern_report[name] = {"launches": launches, "total_ms": round(ms, 3), "avg_us": round(avg_ms * 1e3, 2),
                             "gbs": round(byt / (avg_ms * 1e-3) / 1e9, 1) if avg_ms > 0 and byt == byt else None}
    if kern and dom in kern:
        launches, ms = kern[dom]
        avg_s = ms / launches * 1e-3
        byt = kernel_bytes(dom, pb.n, pb.A.nnz, sinfo.nnz_g, w_g, pb.kmax, sinfo.mmax)
        ach = byt / avg_s / 1e9
        roof = {"kernel": dom, "bound": "hbm", "achieved": round(ach, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": round(ach / PEAK_HBM_GBS, 4), "traffic": measured_traffic(dom, workload_name),
                "bytes_per_launch": byt, "avg_launch_us": round(avg_s * 1e6, 2)}
        # the same launch against the VALU issue rate, from the committed instruction count
        vi = measured_value(dom, workload_name, "sq_counters", "valu_insts_per_launch")
        if vi:
            g = vi / avg_s / 1e9
            issue_roof = {"kernel": dom, "bound": "valu_issue", "achieved": round(g, 1), "peak": PEAK_VALU_GINST,
                          "unit": "Ginst/s", "frac": round(g / PEAK_VALU_GINST, 4), "valu_insts_per_launch": vi}

    # whole-PCG achieved bandwidth from the per-iteration algorithmic bytes
    it_bytes = (kernel_bytes("spmv_A_dot", pb.n, pb.A.nnz, sinfo.nnz_g, w_g, pb.kmax, sinfo.mmax)
                + kernel_bytes("update_xr", pb.n, 0, 0, w_g, 0, 0)
                + kernel_bytes("spmv_G", pb.n, 0, sinfo.nnz_g, w_g, 0, 0)
                + kernel_bytes("spmv_GT_dot", pb.n, 0, sinfo.nnz_g, w_g, 0, 0)
                + kernel_bytes("update_p", pb.n, 0, 0, w_g, 0, 0))
    pcg_gbs = it_bytes * its[-1] / (np.mean(pcg_ms) * 1e-3) / 1e9

    cpu = None
    if with_cpu:
        threads = args.cpu_threads or int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or (os.cpu_count() or 1)
        print(f"[bench] cpu baseline: oracle on {threads} threads ...", file=sys.stderr, flush=True)
        if pb.n <= CPU_WHOLE_MAX_ROWS:
            cpu = cpu_baseline(pb, its[-1], threads, x.cpu().numpy())
        else:
            cpu = cpu_baseline_sampled(pb, its[-1], sinfo.nnz_g, threads)
        print(f"[bench] cpu baseline: {cpu['value']} s ({cpu['sample']})", file=sys.stderr, flush=True)

    forms = None
    if with_forms:
        forms = forms_compare(af, pb, dA, b, x, forms_steps)
    f32_eval = None
    if args.setup_f32:
        f32_eval = setup_f32_eval(af, pb, dA, b, x, its[-1])

    out = {
        "value": round(sec, 6),
        "ms_per_step": round(sec * 1e3, 3),
        "dtype": ("f32 setup, " if args.setup_f32 else "") + ("f32 gradient, " if args.grad_f32 else "")
                 + ("f64" if g_prec == af.F64 else "f64 (G stored f32)"),
        "config": {"workload": workload_name, "n": pb.n, "nnz": pb.A.nnz, "kmax": pb.kmax, "s": pb.s,
                   "eps": pb.eps, "rtol": pb.rtol, "g_prec": "f32" if g_prec == af.F32 else "f64",
                   "setup_prec": "f32" if args.setup_f32 else "f64",
                   "gradient_prec": "f32" if (args.setup_f32 or args.grad_f32) else "f64", "nnz_g": sinfo.nnz_g},
        "setup_ms": round(float(np.mean(setup_ms)), 3),
        "pcg_ms": round(float(np.mean(pcg_ms)), 3),
        "iters": its[-1],
        "true_relres": info.true_relres,
        "pcg_hbm_gbs": round(pcg_gbs, 1),
        "roofline": roof,
        "issue_roofline": issue_roof,
        "kernels": kern_report,
        "cpu_baseline": cpu,
    }
    if f32_eval:
        out["setup_f32_eval"] = f32_eval
    if forms:
        out["forms"] = forms
    return out


def forms_compare(af, pb, dA, b, x, steps: int) -> dict:
    """Time to solution (setup + PCG to rtol, median of ``steps`` after one warm-up) of the
    plain form (G and every setup step in FP64) against the precision forms: G stored and
    applied in FP32, and in addition the gradient reading FP32 values of A (the dense
    factorisation, the PCG recurrences and A stay FP64).  The FP32-gradient form's patterns
    are compared with the FP64 setup's row by row when G is small enough to export."""
    import torch

    kinds = {"plain_f64": dict(g_prec=af.F64), "g_f32": dict(g_prec=af.F32),
             "g_f32_grad_f32": dict(g_prec=af.F32, grad_f32=True)}
    res = {}
    for name, kw in kinds.items():
        runs = []
        for k in range(steps + 1):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            P = af.setup(dA, pb.kmax, pb.s, pb.eps, **kw)
            x.zero_()
            _, info = af.pcg_solve(dA, P, b, x=x, rtol=pb.rtol)
            torch.cuda.synchronize()
            wall = (time.perf_counter() - t0) * 1e3
            si = P.info()
            P.close()
            if k:
                runs.append((wall, si.ms, info.ms, info.iters, info.true_relres))
        w, su, pc, it, tr = (np.median([r[j] for r in runs]) for j in range(5))
        res[name] = {"ms": round(float(w), 3), "setup_ms": round(float(su), 3), "pcg_ms": round(float(pc), 3),
                     "iters": int(it), "true_relres": float(tr)}
    base = res["plain_f64"]["ms"]
    for name in kinds:
        res[name]["speedup_vs_plain"] = round(base / res[name]["ms"], 4)
    if pb.n <= CPU_WHOLE_MAX_ROWS:
        P64 = af.setup(dA, pb.kmax, pb.s, pb.eps)
        P32 = af.setup(dA, pb.kmax, pb.s, pb.eps, grad_f32=True)
        (r64, c64, _), (r32, c32, _) = ([t.cpu().numpy() for t in Pk.export()] for Pk in (P64, P32))
        P64.close()
        P32.close()
        same = int(np.sum([np.array_equal(c64[r64[i]:r64[i + 1]], c32[r32[i]:r32[i + 1]]) for i in range(pb.n)])) \
            if not np.array_equal(r64, r32) or not np.array_equal(c64, c32) else pb.n
        res["g_f32_grad_f32"]["rows_with_fp64_pattern"] = same / pb.n
    print(f"[bench] precision forms: {json.dumps(res)}", file=sys.stderr, flush=True)
    return res


def setup_f32_eval(af, pb, dA, b, x, iters_f32: int) -> dict:
    """The FP32 setup against the FP64 one (which equals the oracle's, tested): rows with the same
    pattern, element-wise and Frobenius relative error of G on them, PCG iterations of both."""
    P32 = af.setup(dA, pb.kmax, pb.s, pb.eps, setup_f32=True)
    P64 = af.setup(dA, pb.kmax, pb.s, pb.eps)
    (r32, c32, v32), (r64, c64, v64) = ([t.cpu().numpy() for t in Pk.export()] for Pk in (P32, P64))
    rows_same = 0
    gerr = None
    rel = np.array([np.nan])
    row_rel = np.array([np.nan])
    if np.array_equal(r32, r64):
        eq = c32 == c64
        row_of = np.repeat(np.arange(pb.n), np.diff(r64))
        bad = np.zeros(pb.n, bool)
        np.logical_or.at(bad, row_of[~eq], True)
        rows_same = int((~bad).sum())
        ok = ~bad[row_of]
        rel = np.abs(v32[ok] - v64[ok]) / np.maximum(np.abs(v64[ok]), 1e-300)
        # per row, relative to the row's largest entry (the parity tests' measure)
        d = np.maximum.reduceat(np.abs(v32 - v64), r64[:-1])
        m = np.maximum.reduceat(np.abs(v64), r64[:-1])
        row_rel = (d / m)[~bad]
        gerr = float(np.linalg.norm(v32[ok] - v64[ok]) / np.linalg.norm(v64[ok]))
    else:
        rows_same = int(sum(np.array_equal(c32[r32[i]:r32[i + 1]], c64[r64[i]:r64[i + 1]]) for i in range(pb.n)))
    x.zero_()
    _, i64 = af.pcg_solve(dA, P64, b, x=x, rtol=pb.rtol)
    P32.close()
    P64.close()
    ev = {"rows_same_pattern": rows_same / pb.n, "g_rel_err_same_rows_elementwise_max": float(np.nanmax(rel)),
          "g_rel_err_same_rows_rowmax_max": float(np.nanmax(row_rel)),
          "g_rel_err_same_rows_rowmax_p99": float(np.nanpercentile(row_rel, 99)),
          "g_rel_err_fro": gerr, "iters_f32_setup": iters_f32, "iters_f64_setup": i64.iters}
    print(f"[bench] FP32 setup: {100 * rows_same / pb.n:.4f}% rows with the FP64 pattern, iterations "
          f"{iters_f32} vs {i64.iters}, {ev}", file=sys.stderr, flush=True)
    return ev


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="elast27_150",
                    choices=sorted(list(workloads()) + list(BATCH_WORKLOADS) + ["serve", "jacobi_compare", "spmm"]))
    ap.add_argument("--with-largest", action="store_true", help="jacobi_compare: add the 150^3 27-point workload")
    ap.add_argument("--requests", type=int, default=600, help="serve: number of requests")
    ap.add_argument("--pool", type=int, default=16, help="serve: distinct systems the requests draw from")
    ap.add_argument("--budget-gb", type=int, default=96, help="serve: device memory budget of the servers")
    ap.add_argument("--serve-heavy", type=int, nargs="*", default=[],
                    help="serve: also run continuous batching with these limits of heavy requests at a time")
    ap.add_argument("--serve-uncapped", action="store_true",
                    help="serve: also run continuous batching without the limit of one heavy request at a time")
    ap.add_argument("--serve-slots", type=int, nargs="+", default=[2, 4],
                    help="serve: slot counts of the continuous-batching runs")
    ap.add_argument("--g-prec", default=None, choices=["f64", "f32"],
                    help="storage of G (default: the workload's own, FP32 for the 150^3 problem, else FP64)")
    ap.add_argument("--tune", action="store_true",
                    help="pick launch choices with the autotuner first (cached by shape) and apply them")
    ap.add_argument("--tune-cache", default=None, help="JSON cache of the autotuner (default: none, tune afresh)")
    ap.add_argument("--grad-f32", action="store_true",
                    help="precision form's gradient: FP32 values of A in the gradient, FP64 factorisation")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the comparison of the plain and precision forms at the 150^3 and 64^3 workloads")
    ap.add_argument("--setup-f32", action="store_true",
                    help="per-row setup arithmetic in FP32 (reports pattern agreement with the FP64 setup)")
    ap.add_argument("--per-entry-a", action="store_true",
                    help="A's SELL layout in the PCG with one column index per entry (AFSAI_OPT_SELL_RUNS = 1) "
                         "instead of one per run of three consecutive columns")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-threads", type=int, default=0)
    ap.add_argument("--no-profile", action="store_true", help="do not time kernels with HIP events")
    ap.add_argument("--no-context", action="store_true",
                    help="skip the 64^3 context run that the default (150^3) line carries")
    ap.add_argument("--copy-check", action="store_true",
                    help="only run a plain 1 GiB device copy five times (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.copy_check:
        copy_check()
        return

    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "row-stripe design is described but not built.", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2010_14175_amd as af

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    af.lib()
    if args.per_entry_a:
        af.set_option(af.OPT_SELL_RUNS, 1)

    if args.workload in BATCH_WORKLOADS:
        batch_bench(args)
        return
    if args.workload == "serve":
        serve_bench(args)
        return
    if args.workload == "jacobi_compare":
        jacobi_bench(args)
        return
    if args.workload == "spmm":
        spmm_bench(args)
        return
    t_gen = time.perf_counter()
    pb = workloads()[args.workload]()
    gp = args.g_prec or WORKLOAD_G_PREC.get(args.workload, "f64")
    g_prec = af.F32 if gp == "f32" else af.F64
    print(f"[bench] workload {pb.name}: n={pb.n} nnz={pb.A.nnz} kmax={pb.kmax} s={pb.s} eps={pb.eps} "
          f"g_prec={gp} (generated in {time.perf_counter() - t_gen:.1f} s)", file=sys.stderr, flush=True)
    forms = args.workload in ("elast27_150", "elast27_64") and not args.no_forms
    res = run_workload(af, pb, g_prec, args, args.steps, args.warmup, not args.no_profile,
                       not args.no_cpu_baseline, args.workload, with_forms=forms, forms_steps=2)
    context = None
    if args.workload == "elast27_150" and not args.no_context:
        # the 64^3 workload (786,432 rows, FP64 G) as context beside the headline
        del pb
        pc = workloads()["elast27_64"]()
        c = run_workload(af, pc, af.F64, args, min(args.steps, 5), 1, not args.no_profile, False, "elast27_64",
                         with_forms=not args.no_forms, forms_steps=5)
        context = {"elast27_64": {k: c[k] for k in ("ms_per_step", "setup_ms", "pcg_ms", "iters", "pcg_hbm_gbs",
                                                    "roofline", "config", "forms") if k in c}}
    out = {"metric": METRIC, "value": res.pop("value"), "unit": "s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": res.pop("ms_per_step"), "higher_is_better": False,
           "scaling": "weak", "vs_baseline": None, "dtype": res.pop("dtype"), "data": "synthetic",
           "config": res.pop("config")}
    out.update(res)
    if context:
        out["context"] = context
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
