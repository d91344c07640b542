"""Benchmark of the SIDM scattering step on one MI355X.

A step is the whole hot path through the C ABI: sidm_build_tree ->
sidm_find_ngb -> sidm_scatter_step -> sidm_pair_timestep, on inputs already
resident in HBM.  The default workload is the largest that fits one GPU: the
clustered periodic box of 256^3 = 16,777,216 particles (2000 NFW haloes and a
uniform background, Maxwellian velocities at the local Jeans dispersion,
constant sigma/m), all particles active, FP64.

Prints ONE JSON line.  value = active particles per second of whole steps
(K steps timed between two device synchronisations).  Inside the timed steps
only the dominant kernel is bracketed by the library's events (for the
roofline); the per-phase breakdown (phase_ms) comes from a window of a few
steps just before, with every phase bracketed.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "active particles/s per SIDM step (ngb+scatter); p50/p99 step latency at fixed rate"
HBM_PEAK_GBS = 8000.0


def make_workload(name: str):
    import workloads as W
    if name == "hernquist1e6":
        w = W.hernquist_bins(W.hernquist_halo(1_000_000))
        desc = ("isolated Hernquist halo G=M=a=1, N=1e6 (Eddington DF, r<100a), "
                "sigma/m=s0/(1+(w/0.5)^2)^2, power-of-two bins ~1/8 active, elastic, FP64")
    elif name == "uniform32k":
        w = W.uniform_box(32768)
        desc = "uniform periodic box 32^3, Maxwellian sigma_1D=1, const sigma/m, all active, FP64"
    elif name == "hernquist4e6_2state":
        w = W.hernquist_bins(W.hernquist_halo(4_000_000, ic_seed=104, philox_seed=4,
                                              two_state=True))
        desc = "two-state Hernquist halo N=4e6, ~1/8 active, delta=0.05 sigma_1D(a)^2, FP64"
    elif name == "hernquist4e6_2state_all":
        w = W.hernquist_halo(4_000_000, ic_seed=104, philox_seed=4, two_state=True)
        w.dt = np.full(w.n, 1e-3)
        desc = "two-state Hernquist halo N=4e6, all active, dt=1e-3, FP64"
    elif name == "clustered256":
        w = W.clustered_box()
        desc = ("clustered periodic box 256^3: 2000 NFW haloes (c=10, dN/dM~M^-1.9 over 3 "
                "decades, 70% of the mass) + uniform background, Maxwellian at the local "
                "Jeans dispersion, const sigma/m, all active, FP64")
    else:
        raise SystemExit(f"unknown workload {name}")
    return w, desc


def touched_count(ngb: np.ndarray, active: np.ndarray) -> int:
    return int(np.unique(np.concatenate([ngb.ravel(), active])).size)


def cpu_baseline(w, all_cores: bool, seconds_hint: float = 12.0) -> dict:
    """The CPU oracle as it stands, on a bounded sample of the same workload:
    the first n_s targets of the active list (all particles as neighbours),
    one full step (candidate gathering with scipy's k-d tree, the exact
    ranking, the scattering step, the timestep).  The k-d tree over all
    particles is built once and timed on its own; the rate is the whole
    active set's: N_a / (t_tree + t_sample N_a / n_s).  all_cores: the
    OpenMP build on every host core (scipy's queries too), else one core."""
    import oracle
    oracle.build(force=False)
    threads = oracle.use_openmp(0) if all_cores else 1
    if not all_cores:
        oracle.use_serial()
    workers = -1 if all_cores else 1
    try:
        t0 = time.perf_counter()
        kd = oracle.kd_tree(w.x, w.y, w.z, w.periodic, w.box)
        t_tree = time.perf_counter() - t0
        # a call costs fixed + per n_s (the fixed part copies the N-particle
        # arrays): samples growing (at most eightfold, aiming at seconds_hint)
        # until one takes seconds_hint; the last two give the line
        pts = []
        n_s = min(w.n_active, 2000)
        while True:
            t0 = time.perf_counter()
            oracle.full_step(w.subset_active(n_s), workers=workers, kd=kd)
            pts.append((n_s, time.perf_counter() - t0))
            if n_s == w.n_active or pts[-1][1] >= 0.8 * seconds_hint or len(pts) >= 6:
                break
            grow = min(8.0, max(2.0, seconds_hint / max(pts[-1][1], 1e-3)))
            n_s = min(w.n_active, int(n_s * grow))
    finally:
        oracle.use_serial()
    if len(pts) >= 2:
        (n1, t1), (n2, t2) = pts[-2], pts[-1]
        per = max((t2 - t1) / (n2 - n1), 1e-12)
        fixed = max(t1 - per * n1, 0.0)
    else:
        (n2, t2), = pts
        per, fixed = t2 / n2, 0.0
    rate = w.n_active / (t_tree + fixed + per * w.n_active)
    what = "all" if n2 == w.n_active else f"the first {n2}"
    return {"value": rate, "unit": "active particles/s", "cores": int(threads),
            "kind": "oracle",
            "sample": f"{what} of {w.n_active} active particles of the same workload (all {w.n} "
                      f"particles as neighbours), one full step (neighbours + scatter + timestep) "
                      f"in {t2:.2f} s; samples {[p[0] for p in pts]} fit t = {fixed:.3f} s + "
                      f"{per * 1e6:.2f} us per target; the k-d tree over all particles once in "
                      f"{t_tree:.2f} s; value = N_a / (t_tree + t_fixed + t_per N_a)"
                      + ("; OpenMP build, scipy queries on all cores" if all_cores else
                         "; one thread")}


def copy_probe(mib: int) -> None:
    """A plain copy of known size: its read and write bytes are exactly
    mib MiB each, which scales the counters of the other kernels."""
    import torch
    torch.cuda.set_device(0)
    n = mib * (1 << 20) // 8
    src = torch.arange(n, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ms = []
    for _ in range(3):
        ev[0].record()
        dst.copy_(src)
        ev[1].record()
        torch.cuda.synchronize()
        ms.append(ev[0].elapsed_time(ev[1]))
    assert bool(torch.equal(dst, src))
    print(json.dumps({"copy_probe_mib": mib, "bytes_read": n * 8, "bytes_written": n * 8,
                      "ms": ms, "gbs": 2 * n * 8 / (min(ms) * 1e-3) / 1e9}))


def run_serving(args) -> dict:
    """The served form: a Poisson stream of independent Hernquist haloes,
    continuous batching over slots, admission by HBM budget."""
    import concurrent.futures as cf
    import torch
    import workloads as W
    from paper_2607_05504_amd import FP64, MIXED
    from paper_2607_05504_amd.serve import Server, ServeConfig
    torch.cuda.set_device(0)
    reqs = W.serving_requests(args.requests, rate=args.rate, n_max=args.n_max, steps=args.req_steps)
    if args.ic_pool:
        # one Eddington sample of n_max particles; each request draws a rotated
        # random subset of it when it is admitted (a few ms of host time)
        pool = W.hernquist_halo(int(args.n_max), ic_seed=7)
        make = lambda r: W.request_workload_pooled(r, pool)
        print(f"[bench] serving: {len(reqs)} requests drawn from a pool of {pool.n}",
              file=sys.stderr, flush=True)
    else:
        # initial conditions generated before the stream starts (host work, not timed)
        with cf.ThreadPoolExecutor(8) as ex:
            wl = dict(zip([r.rid for r in reqs], ex.map(W.request_workload, reqs)))
        make = lambda r: wl[r.rid]
        print(f"[bench] serving: {len(reqs)} requests generated", file=sys.stderr, flush=True)
    prec = MIXED if args.precision == "mixed" else FP64
    # warm-up: one small request through the whole path
    srv = Server(ServeConfig(n_slots=args.slots, hbm_budget=args.budget_gib << 30, precision=prec,
                             progress_s=20.0 if args.ic_pool else 0.0))
    wreq = W.Request(rid=-1, arrival=0.0, n=10000, s0=W.hernquist_s0(), ic_seed=99, philox_seed=99,
                     steps=2)
    srv.run([wreq], W.request_workload)
    torch.cuda.synchronize()
    rep = srv.run(reqs, make)
    torch.cuda.synchronize()
    srv.close()
    n_steps = sum(r.steps for r in reqs)
    return {
        "metric": METRIC, "value": rep["throughput"], "unit": "active particles/s",
        "n_gpus": 1, "steps": n_steps, "warmup": 1,
        "ms_per_step": rep["wall_s"] * 1e3 / max(n_steps, 1),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32+f64", "data": "synthetic",
        "config": {"workload": "serving", "requests": len(reqs), "rate_per_s": args.rate,
                   "n_range": [1e4, args.n_max], "steps_per_request": args.req_steps,
                   "initial_conditions": "pooled subsets" if args.ic_pool else "per request",
                   "slots": args.slots, "hbm_budget_gib": args.budget_gib,
                   "precision": args.precision},
        "p50_step_ms": rep["p50_step_ms"], "p99_step_ms": rep["p99_step_ms"],
        "p50_request_s": rep["p50_request_s"], "p99_request_s": rep["p99_request_s"],
        "mean_admission_wait_s": rep["mean_admission_wait_s"],
        "max_admission_wait_s": rep["max_admission_wait_s"],
        "wall_s": rep["wall_s"], "particle_steps": rep["particle_steps"],
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="clustered256",
                    help="clustered256 (the largest single-GPU workload, the default), "
                         "hernquist1e6, hernquist4e6_2state, hernquist4e6_2state_all, "
                         "uniform32k, serving")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--precision", choices=("fp64", "mixed"), default="fp64",
                    help="mixed: FP32 neighbour test and probabilities on leaf-relative "
                         "offsets with FP64 rechecks in the bands, FP64 kicks")
    ap.add_argument("--traffic", default=os.path.join(ROOT, "profiles", "traffic.json"),
                    help="per-kernel HBM traffic measured with rocprofv3 counters")
    ap.add_argument("--estimator", choices=("one-sided", "overlap"), default="one-sided",
                    help="scattering-rate estimator: the fiducial one-sided kernel, or the "
                         "kernel overlap (partners r < h_i + h_j, tabulated overlap integral)")
    ap.add_argument("--max-ngb", type=int, default=384,
                    help="overlap estimator: partner buffer per active particle")
    ap.add_argument("--refit", action="store_true",
                    help="after the first step, reuse the tree's order (sidm_refit_tree)")
    ap.add_argument("--requests", type=int, default=200, help="serving: requests in the stream")
    ap.add_argument("--rate", type=float, default=20.0, help="serving: arrivals per second")
    ap.add_argument("--n-max", type=float, default=2e5, help="serving: largest halo (N)")
    ap.add_argument("--req-steps", type=int, default=64, help="serving: steps per request")
    ap.add_argument("--slots", type=int, default=8, help="serving: concurrent requests")
    ap.add_argument("--budget-gib", type=int, default=4, help="serving: HBM budget")
    ap.add_argument("--ic-pool", action="store_true",
                    help="serving: draw each request from one Eddington sample of n-max "
                         "particles (for streams too large to sample one by one)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB three times "
                         "(calibrates the HBM byte counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this library runs on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return
    if args.workload == "serving":
        print(json.dumps(run_serving(args)))
        return

    import torch
    from paper_2607_05504_amd import (EST_OVERLAP, FP64, MIXED, TIMING_ALL, TIMING_EVAL,
                                      TIMING_KNN, TIMING_OVERLAP, TIMING_TIMESTEP, Context,
                                      profsum, runner)

    torch.cuda.set_device(0)
    w, desc = make_workload(args.workload)
    ds = runner.upload(w, "cuda:0")
    overlap = args.estimator == "overlap"
    cfg = runner.config_for(w, precision=MIXED if args.precision == "mixed" else FP64,
                            estimator=EST_OVERLAP if overlap else 0)
    print(f"[bench] workload {args.workload}: n={w.n} active={w.n_active} "
          f"estimator {args.estimator}", file=sys.stderr, flush=True)
    if overlap:
        # every particle's h once before the timed steps (untimed, as the
        # inactive particles' h of earlier steps); each step then finds the
        # active particles' h and updates them before the overlap walk
        ctx = Context(cfg, w.n, w.n)
        out = runner.alloc_overlap(ds, w.n_ngb, args.max_ngb)

        def one_step(t, first=False):
            runner.run_overlap_step(ctx, ds, out, w.seed, t,
                                    smoothing="all" if first else "active")
    else:
        ctx = Context(cfg, w.n, w.n_active)
        out = runner.alloc_out(ds, w.n_ngb)

        def one_step(t, first=False):
            runner.run_step(ctx, ds, out, w.seed, t, refit=args.refit and not first)

    for t in range(args.warmup):
        one_step(w.step + t, first=t == 0)
    ctx.sync()
    torch.cuda.synchronize()

    # Per-phase breakdown from an instrumented window of steps before the
    # timed region: every phase bracketed by the library's events, which
    # leave the GPU idle a few microseconds at each bracket, so they stay out
    # of the timed steps.
    n_instr = max(3, min(args.steps, 10))
    ctx.timing_enable(TIMING_ALL)
    for t in range(n_instr):
        one_step(w.step + args.warmup + t, first=args.warmup + t == 0)
    tim_all = ctx.timing_read()
    ctx.timing_enable(0)
    ctx.sync()
    torch.cuda.synchronize()
    cand = ["knn", "eval", "timestep"] + (["overlap"] if overlap else [])
    dom = max(cand, key=lambda n: tim_all[n + "_ms"])
    dom_mask = {"knn": TIMING_KNN, "eval": TIMING_EVAL, "timestep": TIMING_TIMESTEP,
                "overlap": TIMING_OVERLAP}[dom]

    # timed region: K whole steps; per-step device time from one event at
    # each step boundary, and the dominant kernel's launches bracketed by the
    # library's events on its stream (the only phase timed in the region)
    ctx.timing_enable(dom_mask)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record()
    for t in range(args.steps):
        one_step(w.step + args.warmup + n_instr + t)
        ev[t + 1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    tim = ctx.timing_read()
    ctx.timing_enable(0)
    stats = ctx.sync()
    step_ms = np.array([ev[t].elapsed_time(ev[t + 1]) for t in range(args.steps)])

    na, k = w.n_active, w.n_ngb
    ms_per_step = wall * 1e3 / args.steps
    value = na / (wall / args.steps)
    if overlap:
        ngb_np = out.ngb_k.cpu().numpy()
        cnt = out.count.cpu().numpy()
        rows = out.ngb.cpu().numpy()
        n_t = touched_count(ngb_np, w.active)
        n_to = int(np.unique(np.concatenate([rows[rows >= 0], w.active])).size)
        c_tot = int(cnt.sum())
    else:
        ngb_np = out.ngb.cpu().numpy()
        n_t = touched_count(ngb_np, w.active)

    # algorithmic bytes per launch (FP64 form)
    knn_bytes = (4 + 4 * k + 8) * na + 24 * n_t
    if overlap:
        # walk: target index, x, h and the h update; rows and counts out;
        # partners' x and h; plus h of every particle into the tree's order
        ovl_bytes = (4 + 32 + 8 + 4) * na + 4 * c_tot + 32 * n_to + 20 * w.n
        eval_bytes = 20 * na + 4 * c_tot + 68 * n_to
        ts_bytes = 20 * na + 4 * c_tot + 32 * n_to
        kern_bytes = {"knn": knn_bytes, "overlap": ovl_bytes, "eval": eval_bytes,
                      "timestep": ts_bytes}
    else:
        eval_bytes = (4 * k + 20) * na + 52 * n_t
        ts_bytes = (4 * k + 20) * na + 24 * n_t
        kern_bytes = {"knn": knn_bytes, "eval": eval_bytes, "timestep": ts_bytes}
    dom_ms, dom_bytes = tim[dom + "_ms"], kern_bytes[dom]
    achieved = dom_bytes / (dom_ms * 1e-3) / 1e9
    traffic = None
    if os.path.exists(args.traffic):
        try:
            tr = json.load(open(args.traffic))
            key = args.workload if args.precision == "fp64" else args.workload + ":mixed"
            ent = tr.get(key, {}).get(dom)
            # a figure taken on another version of the kernel source is stale
            if ent and ent.get("source") == profsum.source_hash():
                traffic = ent.get("bytes_per_launch")
        except Exception:
            traffic = None
    roofline = {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                "algorithmic_bytes_per_launch": dom_bytes, "avg_launch_ms": dom_ms}

    # the active set is mapped once a step (the later calls reuse it)
    ngb_scatter_ms = (tim_all["knn_ms"] + tim_all["eval_ms"] + tim_all["resolve_ms"]
                      + tim_all["map_ms"])
    if overlap:
        ngb_scatter_ms += tim_all["overlap_ms"]
    res = {
        "metric": METRIC, "value": value, "unit": "active particles/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "description": desc, "n": w.n, "n_active": na,
                   "n_ngb": k, "precision": args.precision, "touched": n_t,
                   "tree": "refit" if args.refit else "rebuilt every step",
                   "estimator": args.estimator},
        "p50_step_ms": float(np.percentile(step_ms, 50)),
        "p99_step_ms": float(np.percentile(step_ms, 99)),
        "phase_ms": {kk: round(v, 5) for kk, v in tim_all.items() if kk.endswith("_ms")},
        "phase_window_steps": n_instr,
        "ngb_scatter_device_ms": ngb_scatter_ms,
        "ngb_scatter_rate": na / (ngb_scatter_ms * 1e-3) if ngb_scatter_ms > 0 else None,
        "events_last_step": stats["n_events"], "passes_last_step": stats["n_passes"],
        "rounds_last_step": stats["n_rounds"],
        "roofline": roofline,
    }
    if overlap:
        res["overlap_partners_mean"] = c_tot / max(na, 1)
        res["overlap_partners_max"] = int(cnt.max()) if na else 0
    if not args.no_cpu_baseline and not overlap:
        res["cpu_baseline"] = cpu_baseline(w, all_cores=True)
        res["cpu_baseline_single_core"] = cpu_baseline(w, all_cores=False)
    print(json.dumps(res))


if __name__ == "__main__":
    main()
