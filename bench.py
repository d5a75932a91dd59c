#!/usr/bin/env python3
"""MG-PCG throughput of the FCM p-multigrid solver on one MI355X.

Default workload (the largest single-GPU configuration): 3D linear elasticity
(E = 1, nu = 0.3) on the unit cube minus 8 seeded spherical voids, 24^3
cells, integrated-Legendre tensor basis p = 4 (2,690,520 unknowns for seed
0), alpha = 1e-10, octree depth 3, clamped at z = 0, traction (0,0,-1) on
z = 1; patchwise additive Schwarz smoothing (blocks of up to 2187 unknowns,
omega = 1/27), FP32 smoother matrices inside the FP64 V-cycle and CG, rtol
1e-10.  One step = one complete solve of a fresh seeded problem:
classification, cut-cell integration, loads, Schwarz inverses, coarse
factorisation (setup) and the MG-preconditioned CG.  Step k uses generator
seed k; warm-up steps use seeds 1000+.  The plain FP64 form is timed on the
same seeds, and the 32^3 p = 3 Poisson cube (848,071 unknowns) is reported
beside it under "poisson_32".

Prints one JSON line.  `value` is solves/s over the timed steps; p50/p99 are
per-solve latencies; the V-cycle throughput and the roofline of the dominant
V-cycle kernel (the finest-level GEMV over the unique patch inverses, HBM
bound) are timed with HIP events on the stream the library launches on, on
the seed-0 problem, outside the timed region.
"""
import argparse
import json
import os
import platform
import statistics
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MG-PCG solves/s + V-cycle DOF/s (%HBM roofline) at rel. err 1e-8; p50/p99 ms"
HBM_PEAK_GBS = 8000.0
# HBM traffic per launch of the dominant kernel, from the committed rocprofv3
# counter profiles (FETCH_SIZE + WRITE_SIZE, KiB per dispatch, each scaled by
# the reading of a 1 GiB elementwise copy); constants of the kernels as
# profiled, reported as null for any other configuration.
GEMV_TRAFFIC = {
    "elasticity": 53.639e9,   # profiles/patch_gemv_band_elast24_p4_traffic.md
    "poisson": 2.230e9,       # profiles/patch_gemv_cube32_p3_traffic.md
}


def _cpu_model():
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                return line.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
    return platform.processor() or "unknown"


def _oracle_time(kind, n, threads):
    """Wall time of one oracle setup + MG-PCG (patchwise) of the seed-0
    problem at n^3 cells, with the BLAS thread count fixed, in a child
    process (thread counts are fixed at BLAS load)."""
    code = (
        "import sys, time; sys.path.insert(0, %r)\n"
        "import fcm_inputs as fi\n"
        "from oracle import fcm, mg\n"
        "if %r == 'elasticity':\n"
        "    d, o = fi.voided_cube_elasticity(0, n=%d, p=4)\n"
        "    o = dict(o, smoother='patchwise', omega=fi.patch_omega(3, 3))\n"
        "else:\n"
        "    d, o = fi.voided_cube_poisson(0, n=%d, p=3)\n"
        "    o = dict(o, smoother='patchwise', omega=fi.patch_omega(3, 1))\n"
        "t = time.perf_counter()\n"
        "disc = fcm.Discretization(d)\n"
        "h = mg.Hierarchy(disc, o)\n"
        "x, it, hist = h.pcg(disc.b)\n"
        "print(time.perf_counter() - t, disc.n_dofs, it)\n" % (ROOT, kind, n, n))
    env = dict(os.environ)
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        env[k] = str(threads)
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env,
                       timeout=600)
    if r.returncode != 0:
        raise RuntimeError(r.stderr[-2000:])
    t, dofs, it = r.stdout.split()
    return float(t), int(dofs), int(it)


def cpu_baseline(kind, full_dofs, sizes, cores):
    """The oracle (FP64 NumPy/SciPy, patchwise) timed on the host at small
    grids of the same seeded workload, with all `cores` BLAS threads and with
    one; the time per solve is extrapolated to the full workload along the
    power law t ~ dofs^beta fitted to the two largest all-core samples."""
    import math
    pts = [(n,) + _oracle_time(kind, n, cores) for n in sizes]
    t1, d1, _ = _oracle_time(kind, sizes[0], 1)
    (na, ta, da, _), (nb, tb, db, _) = pts[-2], pts[-1]
    beta = math.log(tb / ta) / math.log(db / da)
    t_full = tb * (full_dofs / db) ** beta
    t_full1 = t1 * (pts[-1][1] / pts[0][1]) * (full_dofs / db) ** beta
    return {"value": 1.0 / t_full, "unit": "solves/s", "cores": cores, "kind": "oracle",
            "cpu": _cpu_model(),
            "one_core_value": 1.0 / t_full1,
            "sample": ("oracle setup+MG-PCG (patchwise, FP64) of the seed-0 workload at " +
                       ", ".join(f"{n}^3 ({d} DOFs, {it} it, {t:.1f} s)" for n, t, d, it in pts) +
                       f" on {cores} threads, {sizes[0]}^3 on 1 thread {t1:.1f} s; extrapolated to "
                       f"{full_dofs} DOFs with t ~ dofs^{beta:.2f} fitted to the two largest samples")}


def serve_bench(args):
    """Serving stream: seeded requests of mixed grids and orders arriving as a
    Poisson process at each rate of --rate, admitted by device-memory footprint
    and advanced together (each admitted solve has one CG iteration in flight,
    replayed from its captured graph, on one of several streams); compared with
    the same requests solved one at a time in the plain FP64 form."""
    import numpy as np
    import torch
    import fcm_inputs as fi
    from paper_2010_00881_amd import Server, Solver

    R = args.requests
    reqs = [fi.serving_request(i) for i in range(R)]
    rates = [float(r) for r in str(args.rate).split(",")]
    runs = []
    for rate in rates:
        arrivals = fi.arrival_times(rate, R)
        print(f"[bench] serving {R} requests at {rate}/s", file=sys.stderr, flush=True)
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
                        if len(done) % 64 == 0:
                            print(f"[bench] {len(done)} of {R} done", file=sys.stderr, flush=True)
            time.sleep(0.002)
        srv.close()
        lat = [done[k][0]["latency_ms"] for k in range(R)]
        t_end = max(done[k][1] + done[k][0]["latency_ms"] / 1e3 for k in range(R))
        runs.append({"rate_per_s": rate, "solves_s": R / t_end, "makespan_s": t_end,
                     "p50_ms": float(np.percentile(lat, 50)),
                     "p99_ms": float(np.percentile(lat, 99)),
                     "failed_requests": [k for k in range(R) if done[k][0]["status"] != 0],
                     "iterations": [done[k][0]["iterations"] for k in range(R)]})
    print("[bench] one-at-a-time plain FP64", file=sys.stderr, flush=True)
    t1 = time.perf_counter()
    its, lat1 = [], []
    for k, (d, o) in enumerate(reqs):
        t = time.perf_counter()
        s = Solver(d, dict(o, precision="fp64", use_graphs=0))
        _, info = s.pcg()
        torch.cuda.synchronize()
        its.append(info["iterations"])
        s.close()
        lat1.append((time.perf_counter() - t) * 1e3)
        if (k + 1) % 64 == 0:
            print(f"[bench] {k + 1} of {R} alone", file=sys.stderr, flush=True)
    alone = R / (time.perf_counter() - t1)
    out = {
        "metric": "served MG-PCG solves/s (p50/p99 latency) vs one-at-a-time plain FP64",
        "value": runs[0]["solves_s"], "unit": "solves/s", "n_gpus": 1, "higher_is_better": True,
        "config": {"workload": f"serving_stream_{R}_requests", "rates_per_s": rates,
                   "slots": args.slots, "budget_gb": args.budget_gb, "precision": "mixed"},
        "runs": runs,
        "one_at_a_time_fp64_solves_s": alone,
        "one_at_a_time_fp64_p50_ms": float(np.percentile(lat1, 50)),
        "one_at_a_time_fp64_p99_ms": float(np.percentile(lat1, 99)),
        "speedup": [r["solves_s"] / alone for r in runs],
        "iterations_fp64": its,
    }
    print(json.dumps(out), flush=True)
    return 0


def batch_bench(args):
    """Throughput batch of the 16^2 p = 2 plate (856 unknowns each, seeds
    0..B-1): one problem at a time in the plain FP64 form against all B set up
    and then solved together, every CG step of all of them one graph launch
    (mixed form)."""
    import torch
    import fcm_inputs as fi
    from paper_2010_00881_amd import Solver
    from paper_2010_00881_amd.fcm import pcg_batched
    B = args.batch

    def prob(sd, prec):
        d, o = fi.plate_with_hole(sd)
        return d, dict(o, precision=prec)

    for sd in range(1000, 1000 + max(1, args.warmup)):   # warm-up: tuner, pool, code objects
        s = Solver(*prob(sd, "mixed"))
        s.pcg()
        s.close()
    print(f"[bench] batch of {B}: one at a time, FP64", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    solve1 = 0.0
    for sd in range(B):
        s = Solver(*prob(sd, "fp64"))
        _, info = s.pcg()
        solve1 += info["t_solve_ms"]
        s.close()
    torch.cuda.synchronize()
    t_alone = time.perf_counter() - t0
    print(f"[bench] batch of {B}: batched, mixed", file=sys.stderr, flush=True)
    t1 = time.perf_counter()
    solvers = [Solver(*prob(sd, "mixed")) for sd in range(B)]
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t1
    t2 = time.perf_counter()
    res = pcg_batched(solvers)
    torch.cuda.synchronize()
    t_solve = time.perf_counter() - t2
    bad = [k for k, (_, i) in enumerate(res) if i["status"] != 0]
    for s in solvers:
        s.close()
    out = {
        "metric": "batched MG-PCG solves/s (one graph launch per CG step) vs one at a time",
        "value": B / (t_setup + t_solve), "unit": "solves/s", "n_gpus": 1,
        "higher_is_better": True,
        "config": {"workload": f"plate16_p2_batch_{B}", "dofs_each": 856, "precision": "mixed"},
        "batched_solve_phase_s": t_solve, "batched_setup_phase_s": t_setup,
        "one_at_a_time_fp64_solves_s": B / t_alone,
        "one_at_a_time_fp64_solve_phase_s": solve1 / 1e3,
        "solve_phase_speedup": (solve1 / 1e3) / t_solve,
        "iterations": [i["iterations"] for _, i in res], "failed": bad,
    }
    print(json.dumps(out), flush=True)
    return 0


def mlhp_bench(args):
    """Multi-level hp sphere problem (8^3 base grid, p = 3, sphere r = 0.35,
    alpha = 1e-10, beta = 1e4, six seeded Gaussian sources) at refinement depth
    --mlhp-k (the paper's configuration uses 3, whose base-node patch inverses
    need ~700 GB; 1 and 2 fit one GPU): setup + MG-PCG per seed, in the form
    --precision (mixed: FP32 copies of the well-conditioned patch inverses)
    and, unless --no-fp64, in the plain FP64 form beside it."""
    import torch
    import fcm_inputs as fi
    from paper_2010_00881_amd import Solver
    K = args.mlhp_k
    p = args.mlhp_p

    def one(seed, precision):
        d, o = fi.sphere_multilevel(seed, n=8, k=K, p=p)
        d["quad_depth"] = 2
        t = time.perf_counter()
        s = Solver(d, dict(o, precision=precision))
        x, info = s.pcg()
        torch.cuda.synchronize()
        lat = (time.perf_counter() - t) * 1e3
        st = s.stats()
        n = s.n_dofs[-1]
        s.close()
        if info["status"] != 0:
            raise RuntimeError(f"seed {seed} did not converge: {info}")
        print(f"[bench] mlhp seed {seed} {precision}: {lat:.0f} ms (setup "
              f"{info['t_setup_ms']:.0f}, solve {info['t_solve_ms']:.0f}, {info['iterations']} it, "
              f"{n} unknowns, {st['n_unique_blocks'] - st['n_fp64_blocks']} FP32 patches)",
              file=sys.stderr, flush=True)
        return lat, info, st, n

    def timed(precision):
        t0 = time.perf_counter()
        res = [one(sd, precision) for sd in range(args.steps)]
        return res, time.perf_counter() - t0

    def summary(res):
        lat = [r[0] for r in res]
        return {"p50_ms": statistics.median(lat),
                "setup_ms_median": statistics.median(r[1]["t_setup_ms"] for r in res),
                "solve_ms_median": statistics.median(r[1]["t_solve_ms"] for r in res),
                "iterations": [r[1]["iterations"] for r in res],
                "max_true_rel_res": max(r[1]["true_rel_res"] for r in res)}

    print(f"[bench] multi-level hp K={K} p={p}: warmup", file=sys.stderr, flush=True)
    for w in range(args.warmup):
        one(1000 + w, args.precision)
    print(f"[bench] timing {args.steps} steps", file=sys.stderr, flush=True)
    res, T = timed(args.precision)
    st = res[0][2]
    out = {
        "metric": "multi-level hp MG-PCG solves/s (setup + solve)", "value": args.steps / T,
        "unit": "solves/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": T * 1e3 / args.steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32+f64" if args.precision == "mixed" else "f64",
        "data": "synthetic (seeded Gaussian sources, seeds 0..steps-1)",
        "config": {"workload": f"sphere_mlhp_8^3_k{K}_p{p}", "dofs": res[0][3],
                   "leaves": st["n_kept"], "patches": st["n_unique_blocks"],
                   "fp32_patches": st["n_unique_blocks"] - st["n_fp64_blocks"],
                   "precision": args.precision, "alpha": 1e-10, "beta": 1e4,
                   "quad_depth": 2, "rtol": 1e-10},
        "device_bytes": st["device_bytes"],
    }
    out.update(summary(res))
    if args.precision == "mixed" and not args.no_fp64:
        r64, T64 = timed("fp64")
        out["fp64_form_solves_s"] = args.steps / T64
        out["fp64_form"] = summary(r64)
        out["mixed_over_fp64"] = out["value"] / out["fp64_form_solves_s"]
    print(json.dumps(out), flush=True)
    return 0


COARSE = "blocktri"        # exact layer-block factorisation, or "hmg" (h-levels below p = 1)
SPACE = "tensor"           # element basis: tensor-product or trunk space


def _problem(kind, seed, n, precision, smoother="patchwise"):
    import fcm_inputs as fi
    if kind == "elasticity":
        d, o = fi.voided_cube_elasticity(seed, n=n, p=4)
        nf = 3
    else:
        d, o = fi.voided_cube_poisson(seed, n=n, p=3)
        nf = 1
    omega = fi.patch_omega(3, nf) if smoother == "patchwise" else 2.0 / 15.0
    d = dict(d, space=SPACE)
    return d, dict(o, precision=precision, smoother=smoother, omega=omega, coarse=COARSE)


def _run_steps(kind, n, seeds, precision, smoother="patchwise"):
    """Complete solves (setup + MG-PCG) of fresh problems; per-solve records."""
    import torch
    from paper_2010_00881_amd import Solver
    recs = []
    for sd in seeds:
        t = time.perf_counter()
        s = Solver(*_problem(kind, sd, n, precision, smoother))
        x, info = s.pcg()
        torch.cuda.synchronize()
        lat = (time.perf_counter() - t) * 1e3
        s.close()
        del x
        if info["status"] != 0:
            raise RuntimeError(f"{kind} solve of seed {sd} ({precision}) did not converge: {info}")
        recs.append({"lat": lat, "it": info["iterations"], "setup": info["t_setup_ms"],
                     "solve": info["t_solve_ms"], "res": info["true_rel_res"]})
        print(f"[bench] {kind} seed {sd} {precision}: {lat:.0f} ms (setup {info['t_setup_ms']:.0f}, "
              f"solve {info['t_solve_ms']:.0f}, {info['iterations']} it)", file=sys.stderr,
              flush=True)
    return recs


def _kernel_figures(kind, n, precision, smoother="patchwise"):
    """V-cycle and dominant-kernel timings (HIP events on the library's
    stream) on the seed-0 problem."""
    import torch
    from paper_2010_00881_amd import Solver
    s = Solver(*_problem(kind, 0, n, precision, smoother))
    torch.cuda.synchronize()
    L = s.n_levels - 1
    n_fine = s.n_dofs[-1]
    reps = 3 if kind == "elasticity" else 10
    ms_v, bytes_v = s.time_op("vcycle", reps=reps)
    ms_s, bytes_s = s.time_op("smooth", level=L, reps=5 * reps)
    ms_r, bytes_r = s.time_op("residual", level=L, reps=5 * reps)
    ms_c, bytes_c = s.time_op("coarse", reps=reps)
    if smoother == "patchwise":
        ms_k, bytes_k = s.time_op("smooth_stored", level=L, reps=5 * reps)
        dom = ("patch_gemv_band_kernel (finest level, unique patch inverses, band pairs)"
               if kind == "elasticity" else
               "patch_gemv_kernel (finest level, unique patch inverses)")
    else:
        ms_k, bytes_k = ms_s, bytes_s
        dom = "finest-level elementwise smoother"
    st = s.stats()
    s.close()
    torch.cuda.empty_cache()
    achieved = bytes_k / (ms_k * 1e-3) / 1e9
    traffic = GEMV_TRAFFIC.get(kind) if (precision == "mixed" and smoother == "patchwise"
                                         and SPACE == "tensor"
                                         and n == (24 if kind == "elasticity" else 32)) else None
    return {
        "dofs": n_fine,
        "vcycle_ms": ms_v,
        "vcycle_gdof_s": n_fine / (ms_v * 1e-3) / 1e9,
        "vcycle_hbm_frac": bytes_v / (ms_v * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "kernels": {
            "smooth_fine": {"ms": ms_s, "bytes": bytes_s, "gbs": bytes_s / (ms_s * 1e-3) / 1e9},
            "stored_gemv_fine": {"ms": ms_k, "bytes": bytes_k},
            "residual_fine": {"ms": ms_r, "bytes": bytes_r, "gbs": bytes_r / (ms_r * 1e-3) / 1e9},
            "coarse_solve": {"ms": ms_c, "bytes": bytes_c, "gbs": bytes_c / (ms_c * 1e-3) / 1e9},
        },
        "problem": {k: st[k] for k in ("n_cut", "n_unique_blocks", "n_fp64_blocks",
                                        "coarse_blocks", "coarse_block_size", "device_bytes")},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic / 1e9 if traffic is not None else None,
                     "traffic_unit": "GB per launch (calibrated FETCH_SIZE + WRITE_SIZE of the "
                                     "committed counter profile)",
                     "algorithmic_gb": bytes_k / 1e9},
    }


def _summary(recs):
    lat = [r["lat"] for r in recs]
    return {
        "latency_ms": lat,
        "p50_ms": statistics.median(lat),
        "p99_ms": sorted(lat)[max(0, int(round(0.99 * len(lat))) - 1)],
        "setup_ms_median": statistics.median(r["setup"] for r in recs),
        "solve_ms_median": statistics.median(r["solve"] for r in recs),
        "iterations": [r["it"] for r in recs],
        "max_true_rel_res": max(r["res"] for r in recs),
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", default="mixed", choices=["mixed", "fp64"])
    ap.add_argument("--workload", default="elasticity",
                    choices=["elasticity", "poisson", "serving", "batch", "mlhp"],
                    help="elasticity: the 24^3 p = 4 solve benchmark (default); poisson: the "
                         "32^3 p = 3 cube; serving: the request stream; mlhp: the multi-level "
                         "hp sphere problem")
    ap.add_argument("--n", type=int, default=None, help="cells per axis (24 / 32)")
    ap.add_argument("--smoother", default="patchwise", choices=["patchwise", "elementwise"])
    ap.add_argument("--space", default="tensor", choices=["tensor", "trunk"],
                    help="element basis (the trunk space keeps the modes whose bubble degrees "
                         "sum to at most p)")
    ap.add_argument("--coarse", default="blocktri", choices=["blocktri", "hmg"],
                    help="p = 1 level: exact layer-block factorisation or geometric h-levels")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true",
                    help="skip the plain FP64 form (one problem at a time)")
    ap.add_argument("--no-poisson", action="store_true",
                    help="skip the 32^3 Poisson figures beside the elasticity line")
    ap.add_argument("--mlhp-k", type=int, default=1)
    ap.add_argument("--mlhp-p", type=int, default=3)
    ap.add_argument("--requests", type=int, default=64)
    ap.add_argument("--rate", default="200", help="arrival rate(s) per s, comma separated")
    ap.add_argument("--batch", type=int, default=64, help="problems of the batch workload")
    ap.add_argument("--slots", type=int, default=16)
    ap.add_argument("--budget-gb", type=float, default=96.0)
    ap.add_argument("--pmc-calibration", action="store_true",
                    help="finish with a 1 GiB elementwise copy (counter calibration)")
    args = ap.parse_args()
    global COARSE, SPACE
    COARSE = args.coarse
    SPACE = args.space
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); a multi-GPU path is not "
              "built", file=sys.stderr)
        return 2

    if args.workload == "serving":
        return serve_bench(args)
    if args.workload == "batch":
        return batch_bench(args)
    if args.workload == "mlhp":
        return mlhp_bench(args)

    import torch
    kind = args.workload
    n = args.n or (24 if kind == "elasticity" else 32)
    label = (f"cube_voids_elasticity_{n}^3_p4" if kind == "elasticity"
             else f"cube_voids_poisson_{n}^3_p3")

    # The kernel figures come first and the warm-up solves after them, so that
    # the timed solves follow solves of their own kind (device memory is
    # handed out from a stream-ordered pool).
    print("[bench] kernel figures on the seed-0 problem", file=sys.stderr, flush=True)
    kf = _kernel_figures(kind, n, args.precision, args.smoother)
    torch.cuda.synchronize()
    print(f"[bench] {label}: warmup {args.warmup} steps", file=sys.stderr, flush=True)
    _run_steps(kind, n, [1000 + w for w in range(args.warmup)], args.precision, args.smoother)
    print(f"[bench] timing {args.steps} steps", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    recs = _run_steps(kind, n, list(range(args.steps)), args.precision, args.smoother)
    torch.cuda.synchronize()
    T = time.perf_counter() - t0
    out = {
        "metric": METRIC,
        "value": args.steps / T,
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
        "config": {"workload": label, "n": n, "p": 4 if kind == "elasticity" else 3,
                   "fields": 3 if kind == "elasticity" else 1, "dofs": kf["dofs"],
                   "precision": args.precision, "smoother": args.smoother,
                   "coarse": args.coarse, "space": args.space,
                   "omega": _problem(kind, 0, n, args.precision, args.smoother)[1]["omega"],
                   "alpha": 1e-10, "quad_depth": 3, "rtol": 1e-10,
                   "parallelism": "none (1 GPU)"},
    }
    out.update(_summary(recs))
    out.update({k: kf[k] for k in ("vcycle_ms", "vcycle_gdof_s", "vcycle_hbm_frac", "kernels",
                                   "problem", "roofline")})
    if not args.no_fp64 and args.precision == "mixed":
        print("[bench] plain FP64 form, one problem at a time", file=sys.stderr, flush=True)
        # one untimed FP64 solve first: its blocks are cut differently from the
        # mixed form's, and the first setup after the switch pays for that
        _run_steps(kind, n, [1000], "fp64", args.smoother)
        t1 = time.perf_counter()
        r64 = _run_steps(kind, n, list(range(args.steps)), "fp64", args.smoother)
        torch.cuda.synchronize()
        out["fp64_form_solves_s"] = args.steps / (time.perf_counter() - t1)
        out["fp64_form"] = _summary(r64)
        out["mixed_over_fp64"] = out["value"] / out["fp64_form_solves_s"]
    if kind == "elasticity" and not args.no_poisson:
        print("[bench] 32^3 p = 3 Poisson cube", file=sys.stderr, flush=True)
        _run_steps("poisson", 32, [1000, 1001], args.precision)
        pk = _kernel_figures("poisson", 32, args.precision)
        t2 = time.perf_counter()
        rp = _run_steps("poisson", 32, list(range(8)), args.precision)
        torch.cuda.synchronize()
        tp = time.perf_counter() - t2
        out["poisson_32"] = dict({"workload": "cube_voids_poisson_32^3_p3",
                                  "solves_s": 8 / tp, "steps": 8}, **_summary(rp), **pk)
    if kind == "elasticity" and not args.no_poisson and args.space == "tensor":
        # the same problems in the trunk space (the paper's 3D element)
        SPACE = "trunk"
        print("[bench] 24^3 p = 4 elasticity cube, trunk space", file=sys.stderr, flush=True)
        _run_steps(kind, n, [1000], args.precision, args.smoother)
        t4 = time.perf_counter()
        rt = _run_steps(kind, n, list(range(args.steps)), args.precision, args.smoother)
        torch.cuda.synchronize()
        out["elasticity_trunk"] = dict({"workload": "cube_voids_elasticity_24^3_p4_trunk",
                                        "solves_s": args.steps / (time.perf_counter() - t4),
                                        "steps": args.steps}, **_summary(rt))
        SPACE = args.space
    if kind == "elasticity" and not args.no_poisson:
        # the popcorn problem of Section 4.3 in the paper's configuration (trunk
        # space, p = 3, elementwise blocks) on a 32^3 embedding grid
        import fcm_inputs as fi
        from paper_2010_00881_amd import Solver
        print("[bench] popcorn 32^3 p = 3 trunk", file=sys.stderr, flush=True)
        recp = []
        for sd in range(-1, args.steps):
            d, o = fi.popcorn(32, 3, space="trunk")
            t5 = time.perf_counter()
            sp = Solver(d, dict(o, precision=args.precision))
            _, info = sp.pcg()
            torch.cuda.synchronize()
            lat = (time.perf_counter() - t5) * 1e3
            dofs_p = sp.n_dofs[-1]
            sp.close()
            if info["status"] != 0:
                raise RuntimeError(f"popcorn solve did not converge: {info}")
            if sd >= 0:   # the first solve is a warm-up
                recp.append({"lat": lat, "it": info["iterations"], "setup": info["t_setup_ms"],
                             "solve": info["t_solve_ms"], "res": info["true_rel_res"]})
        out["popcorn_32"] = dict({"workload": "popcorn_32^3_p3_trunk_elementwise",
                                  "dofs": dofs_p,
                                  "solves_s": 1e3 / statistics.mean(r["lat"] for r in recp)},
                                 **_summary(recp))
    if kind == "elasticity" and not args.no_poisson and args.coarse == "blocktri":
        # h-levels below p = 1 against the exact layer-block solve on a grid
        # where the latter's dense layer blocks (4225 unknowns) dominate
        big = {}
        for co in ("hmg", "blocktri"):
            COARSE = co
            print(f"[bench] 64^3 p = 3 Poisson cube, coarse {co}", file=sys.stderr, flush=True)
            _run_steps("poisson", 64, [1000], args.precision)
            t3 = time.perf_counter()
            r = _run_steps("poisson", 64, [0, 1], args.precision)
            torch.cuda.synchronize()
            big[co] = dict({"solves_s": 2 / (time.perf_counter() - t3)}, **_summary(r))
        COARSE = args.coarse
        out["poisson_64_coarse"] = {"workload": "cube_voids_poisson_64^3_p3", "steps": 2,
                                    "hmg": big["hmg"], "blocktri": big["blocktri"],
                                    "hmg_over_blocktri": big["hmg"]["solves_s"] /
                                    big["blocktri"]["solves_s"]}
    if not args.no_cpu_baseline:
        print("[bench] CPU oracle samples", file=sys.stderr, flush=True)
        cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        sizes = (2, 3) if kind == "elasticity" else (4, 6)
        out["cpu_baseline"] = cpu_baseline(kind, kf["dofs"], sizes, cores)
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
