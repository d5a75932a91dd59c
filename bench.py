#!/usr/bin/env python3
"""MG-PCG throughput of the FCM p-multigrid solver on one MI355X.

Workload: 3D Poisson on the unit cube minus 8 seeded spherical voids, 32^3
cells, integrated-Legendre tensor basis p = 3 (848k unknowns for seed 0),
alpha = 1e-10, octree depth 3, u = 0 on the box faces, f = 1; FP32 V-cycle
inside FP64 CG (rtol 1e-10), patchwise additive Schwarz smoothing (one block
per grid node, omega = 1/18, Section 3.3).  One step = one complete solve of
a fresh seeded problem: classification, cut-cell integration, loads, Schwarz
inverses, coarse factorisation (setup) and the MG-preconditioned CG.  Step k
uses generator seed k; warm-up steps use seeds 1000+.

Prints one JSON line.  `value` is solves/s over the timed steps; p50/p99 are
per-solve latencies; the V-cycle throughput and the roofline of the dominant
V-cycle kernel (the finest-level GEMV over the unique patch inverses, HBM
bound) are timed with HIP events on the stream the library launches on,
after the timed region.
"""
import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MG-PCG solves/s + V-cycle DOF/s (%HBM roofline) at rel. err 1e-8; p50/p99 ms"
HBM_PEAK_GBS = 8000.0
# HBM traffic of one launch of the finest-level unique-patch GEMV on the seed-0
# 32^3 p = 3 problem, FP32 V-cycle: rocprofv3 FETCH_SIZE and WRITE_SIZE (KiB per
# dispatch) of `bench.py --steps 1 --warmup 0 --no-cpu-baseline --pmc-calibration`,
# each scaled by the reading of a 1 GiB elementwise copy (see
# profiles/patch_gemv_cube32_p3_traffic.md).  Valid for the kernel as profiled.
GEMV_TRAFFIC = {"bytes": 2.215e9}


def cpu_baseline(n_sample=6):
    """Oracle (FP64 NumPy/SciPy) MG-PCG, setup + solve, on the workload's geometry
    at a reduced grid; scaled to the full workload by the ratio of fine DOFs."""
    import fcm_inputs as fi
    from oracle import fcm, mg
    desc, opts = fi.voided_cube_poisson(0, n=n_sample, p=3)
    opts = dict(opts, smoother="patchwise", omega=1.0 / 18.0)
    t0 = time.perf_counter()
    disc = fcm.Discretization(desc)
    hier = mg.Hierarchy(disc, opts)
    _, it, _ = hier.pcg(disc.b)
    t = time.perf_counter() - t0
    full = 848071
    scale = full / disc.n_dofs
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": 1.0 / (t * scale), "unit": "solves/s", "cores": cores, "kind": "oracle",
            "sample": (f"oracle setup+MG-PCG (patchwise) of the same seeded voided cube at {n_sample}^3 cells, "
                       f"p=3 ({disc.n_dofs} DOFs, {it} iterations, {t:.1f} s), scaled by fine DOFs "
                       f"x{scale:.1f} to the 32^3 workload")}


def serve_bench(args):
    """Serving stream: seeded requests of mixed grids and orders arriving as a
    Poisson process, admitted by device-memory footprint and advanced together
    (one CG iteration per tick); compared with one-at-a-time plain FP64 solves."""
    import numpy as np
    import torch
    import fcm_inputs as fi
    from paper_2010_00881_amd import Server, Solver

    R = args.requests
    reqs = [fi.serving_request(i) for i in range(R)]
    arrivals = fi.arrival_times(args.rate, R)
    print(f"[bench] serving {R} requests at {args.rate}/s", file=sys.stderr, flush=True)
    srv = Server(memory_budget_bytes=int(args.budget_gb * (1 << 30)), max_active=args.slots,
                 n_streams=4)
    ids = []
    t0 = time.perf_counter()
    for i, (d, o) in enumerate(reqs):
        now = time.perf_counter() - t0
        if arrivals[i] > now:
            time.sleep(arrivals[i] - now)
        ids.append((srv.submit(d, dict(o, precision="mixed")), time.perf_counter() - t0))
    done = {}
    while len(done) < R:
        for k, (rid, ts) in enumerate(ids):
            if k not in done:
                r = srv.poll(rid, 0)
                if r is not None:
                    done[k] = (r, ts)
        time.sleep(0.002)
    srv.close()
    lat = [done[k][0]["latency_ms"] for k in range(R)]
    t_end = max(done[k][1] + done[k][0]["latency_ms"] / 1e3 for k in range(R))
    failed = [k for k in range(R) if done[k][0]["status"] != 0]
    served = R / t_end
    print("[bench] one-at-a-time plain FP64", file=sys.stderr, flush=True)
    t1 = time.perf_counter()
    its = []
    for d, o in reqs:
        s = Solver(d, dict(o, precision="fp64", use_graphs=0))
        _, info = s.pcg()
        torch.cuda.synchronize()
        its.append(info["iterations"])
        s.close()
    alone = R / (time.perf_counter() - t1)
    out = {
        "metric": "served MG-PCG solves/s (p50/p99 latency) vs one-at-a-time plain FP64",
        "value": served, "unit": "solves/s", "n_gpus": 1, "higher_is_better": True,
        "config": {"workload": f"serving_stream_{R}_requests", "rate_per_s": args.rate,
                   "slots": args.slots, "budget_gb": args.budget_gb},
        "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
        "one_at_a_time_fp64_solves_s": alone, "speedup": served / alone,
        "failed_requests": failed, "iterations_fp64": its,
    }
    print(json.dumps(out), flush=True)
    return 0


def mlhp_bench(args):
    """Multi-level hp sphere problem (8^3 base grid, p = 3, sphere r = 0.35,
    alpha = 1e-10, beta = 1e4, six seeded Gaussian sources) at refinement depth
    --mlhp-k (the paper's configuration uses 3, whose base-node patch inverses
    need ~700 GB; 1 and 2 fit one GPU): setup + FP64 MG-PCG per seed."""
    import torch
    import fcm_inputs as fi
    from paper_2010_00881_amd import Solver
    K = args.mlhp_k
    p = args.mlhp_p

    def one(seed):
        d, o = fi.sphere_multilevel(seed, n=8, k=K, p=p)
        d["quad_depth"] = 2
        t = time.perf_counter()
        s = Solver(d, dict(o, precision="fp64"))
        x, info = s.pcg()
        torch.cuda.synchronize()
        lat = (time.perf_counter() - t) * 1e3
        st = s.stats()
        n = s.n_dofs[-1]
        s.close()
        if info["status"] != 0:
            raise RuntimeError(f"seed {seed} did not converge: {info}")
        return lat, info, st, n

    print(f"[bench] multi-level hp K={K} p={p}: warmup", file=sys.stderr, flush=True)
    for w in range(args.warmup):
        one(1000 + w)
    print(f"[bench] timing {args.steps} steps", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    res = [one(sd) for sd in range(args.steps)]
    T = time.perf_counter() - t0
    lat = [r[0] for r in res]
    out = {
        "metric": "multi-level hp MG-PCG solves/s (setup + solve)", "value": args.steps / T,
        "unit": "solves/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": T * 1e3 / args.steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (seeded Gaussian sources, seeds 0..steps-1)",
        "config": {"workload": f"sphere_mlhp_8^3_k{K}_p{p}", "dofs": res[0][3],
                   "leaves": res[0][2]["n_kept"], "patches": res[0][2]["n_unique_blocks"],
                   "alpha": 1e-10, "beta": 1e4, "quad_depth": 2, "rtol": 1e-10},
        "p50_ms": statistics.median(lat),
        "setup_ms_median": statistics.median(r[1]["t_setup_ms"] for r in res),
        "solve_ms_median": statistics.median(r[1]["t_solve_ms"] for r in res),
        "iterations": [r[1]["iterations"] for r in res],
        "max_true_rel_res": max(r[1]["true_rel_res"] for r in res),
        "device_bytes": res[0][2]["device_bytes"],
    }
    print(json.dumps(out), flush=True)
    return 0


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=8)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", default="mixed", choices=["mixed", "fp64"])
    ap.add_argument("--n", type=int, default=32)
    ap.add_argument("--smoother", default="patchwise", choices=["patchwise", "elementwise"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--compare-fp64", action="store_true",
                    help="also time the plain FP64 form one problem at a time")
    ap.add_argument("--workload", default="cube", choices=["cube", "serving", "mlhp"],
                    help="cube: the 32^3 solve benchmark; serving: the request stream; "
                         "mlhp: the multi-level hp sphere problem")
    ap.add_argument("--mlhp-k", type=int, default=1)
    ap.add_argument("--mlhp-p", type=int, default=3)
    ap.add_argument("--requests", type=int, default=64)
    ap.add_argument("--rate", type=float, default=200.0)
    ap.add_argument("--slots", type=int, default=16)
    ap.add_argument("--budget-gb", type=float, default=96.0)
    ap.add_argument("--pmc-calibration", action="store_true",
                    help="finish with a 1 GiB elementwise copy (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU design is "
              "described in DESIGN.md and not built", file=sys.stderr)
        return 2

    if args.workload == "serving":
        return serve_bench(args)
    if args.workload == "mlhp":
        return mlhp_bench(args)

    import torch
    import fcm_inputs as fi
    from paper_2010_00881_amd import Solver

    def problem(seed, precision):
        d, o = fi.voided_cube_poisson(seed, n=args.n, p=3)
        return d, dict(o, precision=precision, smoother=args.smoother,
                       omega=1.0 / 18.0 if args.smoother == "patchwise" else 2.0 / 15.0)

    def run_steps(seeds, precision, keep_first=False):
        lat, its, setup, solve, errs = [], [], [], [], []
        first = None
        for sd in seeds:
            t = time.perf_counter()
            s = Solver(*problem(sd, precision))
            x, info = s.pcg()
            torch.cuda.synchronize()
            lat.append((time.perf_counter() - t) * 1e3)
            its.append(info["iterations"])
            setup.append(info["t_setup_ms"])
            solve.append(info["t_solve_ms"])
            errs.append(info["true_rel_res"])
            if info["status"] != 0:
                raise RuntimeError(f"solve of seed {sd} did not converge: {info}")
            if keep_first and sd == seeds[0]:
                first = s
            else:
                s.close()
            del x
        return lat, its, setup, solve, errs, first

    print(f"[bench] warmup {args.warmup} steps", file=sys.stderr, flush=True)
    run_steps([1000 + w for w in range(args.warmup)], args.precision)
    torch.cuda.synchronize()
    print(f"[bench] timing {args.steps} steps", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    lat, its, setup, solve, errs, s = run_steps(list(range(args.steps)), args.precision,
                                                keep_first=True)
    torch.cuda.synchronize()
    T = time.perf_counter() - t0
    value = args.steps / T

    # V-cycle throughput and dominant kernel on the seed-0 problem (the one the
    # committed counter profile covers), HIP events on the library's stream
    L = s.n_levels - 1
    n_fine = s.n_dofs[-1]
    ms_v, bytes_v = s.time_op("vcycle", reps=10)
    ms_s, bytes_s = s.time_op("smooth", level=L, reps=50)
    ms_r, bytes_r = s.time_op("residual", level=L, reps=50)
    ms_c, bytes_c = s.time_op("coarse", reps=10)
    if args.smoother == "patchwise":
        ms_k, bytes_k = s.time_op("smooth_stored", level=L, reps=50)
        dom = "patch_gemv_kernel (finest level, unique patch inverses)"
    else:
        ms_k, bytes_k = ms_s, bytes_s
        dom = "finest-level elementwise smoother"
    achieved = bytes_k / (ms_k * 1e-3) / 1e9
    st = s.stats()
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": T * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if args.precision == "mixed" else "f64",
        "data": "synthetic (seeded voided cube, seeds 0..steps-1)",
        "config": {"workload": f"cube_voids_poisson_{args.n}^3_p3", "n": args.n, "p": 3,
                   "dofs": n_fine, "precision": args.precision, "smoother": args.smoother,
                   "alpha": 1e-10,
                   "quad_depth": 3, "rtol": 1e-10, "parallelism": "none (1 GPU)"},
        "p50_ms": statistics.median(lat),
        "p99_ms": sorted(lat)[max(0, int(round(0.99 * len(lat))) - 1)],
        "setup_ms_median": statistics.median(setup),
        "solve_ms_median": statistics.median(solve),
        "iterations": its,
        "max_true_rel_res": max(errs),
        "vcycle_ms": ms_v,
        "vcycle_gdof_s": n_fine / (ms_v * 1e-3) / 1e9,
        "vcycle_hbm_frac": bytes_v / (ms_v * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "kernels": {
            "smooth_fine": {"ms": ms_s, "bytes": bytes_s,
                            "gbs": bytes_s / (ms_s * 1e-3) / 1e9},
            "stored_gemv_fine": {"ms": ms_k, "bytes": bytes_k},
            "residual_fine": {"ms": ms_r, "bytes": bytes_r,
                              "gbs": bytes_r / (ms_r * 1e-3) / 1e9},
            "coarse_solve": {"ms": ms_c, "bytes": bytes_c,
                             "gbs": bytes_c / (ms_c * 1e-3) / 1e9},
        },
        "problem": {k: st[k] for k in ("n_cut", "n_unique_blocks", "n_fp64_blocks",
                                        "coarse_blocks", "coarse_block_size", "device_bytes")},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": (GEMV_TRAFFIC["bytes"] / 1e9
                                 if GEMV_TRAFFIC["bytes"] is not None and args.n == 32
                                 and args.smoother == "patchwise" and args.precision == "mixed"
                                 else None),
                     "traffic_unit": "GB per launch (calibrated FETCH_SIZE + WRITE_SIZE)",
                     "algorithmic_gb": bytes_k / 1e9},
    }
    s.close()
    if args.compare_fp64:
        print("[bench] plain FP64 form, one problem at a time", file=sys.stderr, flush=True)
        t1 = time.perf_counter()
        lat64, *_ = run_steps(list(range(args.steps)), "fp64")
        torch.cuda.synchronize()
        out["fp64_form_solves_s"] = args.steps / (time.perf_counter() - t1)
    if not args.no_cpu_baseline:
        print("[bench] CPU oracle sample", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline()
    if args.pmc_calibration:
        a = torch.ones(256 * 2**20, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        torch.neg(a, out=b)          # reads 1 GiB, writes 1 GiB
        torch.cuda.synchronize()
        print("[bench] calibration copy: 1 GiB read, 1 GiB written", file=sys.stderr, flush=True)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
