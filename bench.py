"""Benchmark: AS-GenEO preconditioned CG on a 3M-DOF flat laminate, one MI355X.

One step = the whole path on one synthetic laminate: device mesh generation, element
assembly of K and f, overlapping decomposition, GenEO eigensolves and coarse space,
subdomain factorisations, and the PCG solve to rtol 1e-8.  Prints one JSON line.

Workload (the configuration the metric is quoted on): flat 50 x 50 mm laminate, 12 plies
[0/45/90/-45/0/45]s, 0.25 mm plies with 4 element layers and 0.05 mm resin interfaces with
1, 64 x 64 x 59 serendipity hexahedra, 3,005,925 DOFs (2,971,200 free), clamped at x = 0,
1 MPa traction at x = 50; 8 x 8 subdomains, overlap 2, GenEO threshold 0.1.
"""
from __future__ import annotations

import argparse
import json

import numpy as np
import os
import subprocess
import sys
import time

HW_QUEUES_SWEEP = 16
if any(a.startswith("--batch") for a in sys.argv[1:]):
    # The sweep's concurrent set-ups are chains of small launches on several streams each,
    # which HIP's default of 4 hardware queues serialises.  The runtime reads the count once,
    # when it starts, so it is set here, before anything can start it (--hw-queues N).
    _q = HW_QUEUES_SWEEP
    for _i, _a in enumerate(sys.argv[1:]):
        if _a == "--hw-queues" and _i + 2 < len(sys.argv):
            _q = int(sys.argv[_i + 2])
        elif _a.startswith("--hw-queues="):
            _q = int(_a.split("=", 1)[1])
    if not 1 <= _q <= 32:
        sys.exit("--hw-queues must be 1 to 32")
    os.environ["GPU_MAX_HW_QUEUES"] = str(_q)

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Solve time per 1M DOFs at rtol 1e-8 (FP64 vs mixed); CG iters; SpMV GB/s"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
# HBM bytes of one PCG subdomain band solve on this workload (FP64 or FP32 factors), from
# the FETCH_SIZE / WRITE_SIZE counters of `bench.py --traffic-probe [--precision mixed]`
# scaled by a 4 GiB copy.  Valid for the solve kernel as it stands: retake the counters
# when it changes.
SOLVE_TRAFFIC_BYTES = {"fp64": 136.0e9, "mixed": 67.4e9}


def run_step(gx, torch, cfg, precision):
    s = gx.Solver(stream=torch.cuda.current_stream())
    s.laminate(cfg)
    f = s.assemble()
    sv = cfg["solver"]
    part = s.partition(cfg, sv["px"], sv["py"])
    nev, n0 = s.geneo_setup(part, sv["px"] * sv["py"], overlap=sv["overlap"], tau=sv["tau"],
                            nev=sv["nev"], nev_max=sv["nev_max"], precision=precision)
    out = s.pcg(f, rtol=sv["rtol"], maxit=2000)
    return s, out, nev, n0


def cpu_baseline():
    """The oracle (plain CPU FP64) on a bounded sample of the same workload: the same
    laminate (layup, element layering, materials, loads) on a 6 x 6 in-plane mesh split
    into 2 x 2 subdomains with the same overlap, threshold and tolerance, timed end to end
    (assembly, decomposition, eigensolves, factorisations, PCG) on one thread."""
    import workloads
    from threadpoolctl import threadpool_limits
    from oracle import fem, pcg
    cfg = workloads.cfg1(nx=6, ny=6, px=2, py=2)
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        prob = fem.Problem(cfg)
        R = pcg.solve(cfg, prob=prob, rtol=cfg["solver"]["rtol"])
        t = time.perf_counter() - t0
    n = prob.n
    return {"value": t / (n / 1e6), "unit": "s/MDOF", "cores": 1, "kind": "oracle",
            "sample": f"6x6x59 elements of the same laminate: {n} free DOFs, 2x2 subdomains, "
                      f"overlap 2, tau 0.1, rtol 1e-8, {R['iters']} PCG iterations, "
                      f"{t:.1f} s wall on one thread"}


def sweep_in_child():
    """The 32-sample sweep (--batch 32 --precision mixed) in a child process of its own, so
    that it gets its hardware queues and the whole device; run before this process touches
    the GPU.  Returns the child's JSON line (or an error record)."""
    cmd = [sys.executable, os.path.join(ROOT, "bench.py"), "--batch", "32", "--precision",
           "mixed"]
    try:
        r = subprocess.run(cmd, capture_output=True, text=True, timeout=900)
    except subprocess.TimeoutExpired:
        return {"error": "sweep timed out"}
    lines = [l for l in r.stdout.splitlines() if l.startswith("{")]
    if r.returncode or not lines:
        return {"error": f"sweep exited with {r.returncode}", "stderr": r.stderr[-400:]}
    d = json.loads(lines[-1])
    keep = ("metric", "value", "unit", "config", "setup_s", "solve_s", "pcg_solves_per_s",
            "concurrent_setups", "hw_queues", "joint_solve_factor_bytes", "iters",
            "all_converged")
    return {k: d[k] for k in keep if k in d}


def batch_sweep(gx, torch, workloads, args):
    """The seeded sweep of wrinkled L-sections (amplitude in [0, 0.5] mm, wavelength in
    [2, 8] mm, 6 to 12 plies, 50k to 400k DOFs), mixed precision, rtol 1e-8: every sample
    meshed, assembled and set up, then all solved by one lockstep batched PCG."""
    prec = gx.GX_FP64 if args.precision == "fp64" else gx.GX_MIXED
    cfgs = [workloads.cfg4(i) for i in range(args.batch)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    batch = gx.Batch(cfgs, precision=prec)
    print(f"# {len(cfgs)} samples meshed and assembled; set-up, {args.concurrent} at a time",
          file=sys.stderr, flush=True)
    batch.setup(concurrent=args.concurrent,
                progress=lambda i, n: print(f"# set up {i + 1}/{n}", file=sys.stderr,
                                            flush=True))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    xs, it, rr, st = batch.solve(rtol=1e-8, maxit=3000)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    ndof = [3 * s.mesh["n_nodes"] for s in batch.solvers]
    entries = sum(s.stats()["interior_band_entries"] for s in batch.solvers)
    w = 8 if args.precision == "fp64" else 4
    line = {"metric": "batched sweep: samples per second (mesh, assembly, set-up and PCG)",
            "value": len(cfgs) / (t2 - t0), "unit": "samples/s", "n_gpus": 1,
            "higher_is_better": True, "data": "synthetic", "dtype": args.precision,
            "config": {"workload": f"{len(cfgs)} seeded wrinkled L-section samples",
                       "dofs_min": min(ndof), "dofs_max": max(ndof), "dofs_total": sum(ndof)},
            "setup_s": t1 - t0, "solve_s": t2 - t1, "pcg_solves_per_s": len(cfgs) / (t2 - t1),
            "concurrent_setups": args.concurrent,
            "hw_queues": os.environ.get("GPU_MAX_HW_QUEUES"), "interior_band_entries": entries,
            # factor read once per sweep by the joint subdomain solve, all samples active
            "joint_solve_factor_bytes": 2 * w * entries,
            "iters": it.tolist(), "all_converged": bool(np.all(st == 0))}
    batch.close()
    print(json.dumps(line), flush=True)


COPY_BYTES = 4 << 30      # calibration copy of the traffic probe (read and written once)


def traffic_probe(gx, torch, workloads, args):
    """The dispatches whose FETCH_SIZE / WRITE_SIZE counters give the subdomain solve's HBM
    traffic: one device-to-device copy of COPY_BYTES (known traffic, the calibration) and
    one launch of the PCG subdomain band solve on the bench workload."""
    cfg = workloads.cfg1()
    prec = gx.GX_MIXED if args.precision == "mixed" else gx.GX_FP64
    s, _, _, _ = run_step(gx, torch, cfg, prec)
    src = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    ms, nbytes = s.kernel_time(1, reps=1)
    print(json.dumps({"copy_bytes": COPY_BYTES, "solve_ms": ms, "solve_algorithmic_bytes": nbytes}),
          flush=True)


def verification_timing(gx, torch, workloads, args):
    """The corner-unfolding verification model of section 2.2 (graded mesh, resin edge
    strips, stiff end layer, end moment; --e1-sub squared subdomains, overlap 1) timed end to end:
    `warmup` untimed steps, then `steps` timed ones in the chosen precision."""
    cfg = workloads.verification_model(px=args.e1_sub, py=args.e1_sub)
    prec = gx.GX_MIXED if args.precision == "mixed" else gx.GX_FP64
    ms, s, out, n0 = timed_steps(gx, torch, cfg, prec, args.steps, args.warmup,
                                 "verification " + args.precision)
    nf = n_free(s)
    line = {"metric": "verification model: solve time per 1M DOFs at rtol 1e-8",
            "value": (ms / 1e3) / (nf / 1e6), "unit": "s/MDOF", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
            "higher_is_better": False, "data": "synthetic", "dtype": args.precision,
            "config": {"workload": cfg["name"] + " L-section R 6.6 mm, 3 mm limbs, W 15 mm, "
                                   "12 plies, graded 400 / 10, 2 mm resin strips, stiff end "
                                   f"layer, {args.e1_sub}x{args.e1_sub} subdomains, "
                                   "overlap 1, tau 0.1",
                       "n_dofs": int(3 * s.mesh["n_nodes"]), "n_free_dofs": nf},
            "cg_iters": out["iters"], "relres": out["relres"], "n0": int(n0),
            "phases_ms": s.phase_times(), "stats": s.stats()}
    s.close()
    print(json.dumps(line), flush=True)


def solution_diff(x, x_ref):
    import torch
    return float(torch.linalg.vector_norm(x - x_ref) / torch.linalg.vector_norm(x_ref))


def timed_steps(gx, torch, cfg, prec, steps, warmup, label):
    """warmup untimed steps, then `steps` timed ones (bracketed by device synchronisations);
    returns (ms per step, last solver, last PCG output, n0)."""
    for _ in range(warmup):
        s, out, nev, n0 = run_step(gx, torch, cfg, prec)
        print(f"# {label} warmup: {out['iters']} iterations, relres {out['relres']:.2e}",
              flush=True)
        del s
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        s, out, nev, n0 = run_step(gx, torch, cfg, prec)
        if k + 1 < steps:
            del s
        print(f"# {label} step {k}: {out['iters']} iterations", flush=True)
    torch.cuda.synchronize()
    return 1e3 * (time.perf_counter() - t0) / steps, s, out, n0


def n_free(s):
    return int(3 * s.mesh["n_nodes"] - 3 * s.mesh["clamped"].numel())


def precision_block(gx, torch, cfg, steps, warmup, x_fp64, ms_fp64, label):
    """The same workload with FP32 subdomain factors and solves (FP64 outer CG)."""
    ms, s, out, n0 = timed_steps(gx, torch, cfg, gx.GX_MIXED, steps, warmup, label)
    nf = n_free(s)
    solve_ms, solve_bytes = s.kernel_time(1, reps=5)
    blk = {"ms_per_step": ms, "value": (ms / 1e3) / (nf / 1e6), "unit": "s/MDOF",
           "steps": steps, "warmup": warmup, "cg_iters": out["iters"], "relres": out["relres"],
           "n0": int(n0), "speedup_vs_fp64": ms_fp64 / ms,
           "rel_diff_vs_fp64_solution": solution_diff(out["x"], x_fp64),
           "phases_ms": s.phase_times(), "stats": s.stats(),
           "subdomain_solve_ms": solve_ms,
           "subdomain_solve_GBps": solve_bytes / (solve_ms * 1e-3) / 1e9}
    s.close()
    return blk


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="fp64",
                    help="precision of --batch and --traffic-probe runs")
    ap.add_argument("--small", action="store_true", help="reduced 24x24 workload (testing)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision block")
    ap.add_argument("--no-sweep", action="store_true",
                    help="skip the 32-sample sweep (run first, in a child process)")
    ap.add_argument("--no-target", action="store_true",
                    help="skip the curved wrinkled L-section block (FP64 vs mixed)")
    ap.add_argument("--mixed-steps", type=int, default=5,
                    help="timed steps of each extra block, at most --steps")
    ap.add_argument("--batch", type=int, default=0,
                    help="instead: the seeded sweep of wrinkled L-sections, this many samples")
    ap.add_argument("--concurrent", type=int, default=6,
                    help="with --batch: set-ups run at a time")
    ap.add_argument("--hw-queues", type=int, default=HW_QUEUES_SWEEP,
                    help="with --batch: HIP hardware queues of the process (1 to 32)")
    ap.add_argument("--e1", action="store_true",
                    help="instead: the verification model of section 2.2 (432,768 elements, "
                         "5.36M DOFs) as a timing workload, in --precision")
    ap.add_argument("--e1-sub", type=int, default=8,
                    help="with --e1: subdomains per direction (8: 64 subdomains)")
    ap.add_argument("--traffic-probe", action="store_true",
                    help="instead: set up the workload, then launch one plain copy of "
                         "COPY_BYTES and one subdomain band solve (for hardware counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; --gpus must be 1 (the "
                                   "build targets a single MI355X; see the design notes for "
                                   "how the path would shard)"}))
        sys.exit(2)
    import torch
    import paper_1707_04228_amd as gx
    import workloads
    if args.batch:
        return batch_sweep(gx, torch, workloads, args)
    if args.traffic_probe:
        return traffic_probe(gx, torch, workloads, args)
    if args.e1:
        return verification_timing(gx, torch, workloads, args)

    sweep = None
    if not (args.no_sweep or args.small):
        print("# the 32-sample sweep, in a child process", file=sys.stderr, flush=True)
        sweep = sweep_in_child()
    cfg = workloads.cfg1(nx=24, ny=24, px=3, py=3) if args.small else workloads.cfg1()
    ms_step, s, out, n0 = timed_steps(gx, torch, cfg, gx.GX_FP64, args.steps, args.warmup,
                                      "fp64")
    nf = n_free(s)
    # live kernel measurements on the library's stream (HIP events)
    spmv_ms, spmv_bytes = s.kernel_time(0, reps=20)
    solve_ms, solve_bytes = s.kernel_time(1, reps=5)
    pre_ms, _ = s.kernel_time(2, reps=5)
    eig_ms, eig_bytes = s.kernel_time(4)          # recorded during the timed setup
    fac_ms, fac_flops = s.kernel_time(5, reps=1)  # the subdomain factorisation, alone
    bst = s.band_stats()
    phases = s.phase_times()
    stats = s.stats()
    x_fp64 = out["x"].clone()
    spmv_gbs = spmv_bytes / (spmv_ms * 1e-3) / 1e9
    solve_gbs = solve_bytes / (solve_ms * 1e-3) / 1e9
    stored_gbs = bst["solve_stored_bytes"] / (solve_ms * 1e-3) / 1e9
    eig_gbs = eig_bytes / (eig_ms * 1e-3) / 1e9
    fac_tflops = fac_flops / (fac_ms * 1e-3) / 1e12
    line = {
        "metric": METRIC,
        "value": (ms_step / 1e3) / (nf / 1e6),
        "unit": "s/MDOF",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": cfg["name"] + " flat 50x50 mm [0/45/90/-45/0/45]s laminate, "
                               "20-node serendipity hexes, 8x8 subdomains, overlap 2, "
                               "GenEO tau 0.1, rtol 1e-8",
                   "n_dofs": int(3 * s.mesh["n_nodes"]), "n_free_dofs": nf,
                   "precision": "fp64"},
        "cg_iters": out["iters"],
        "relres": out["relres"],
        "n0": int(n0),
        "spmv_GBps": spmv_gbs,
        "spmv_ms": spmv_ms,
        "subdomain_solve_GBps": solve_gbs,
        "subdomain_solve_ms": solve_ms,
        "precond_apply_ms": pre_ms,
        "phases_ms": phases,
        "stats": stats,
        "band_stats": bst,
        "roofline": {"bound": "hbm", "kernel": "k_band_solve_1 (PCG subdomain solves, "
                                               "forward+backward)",
                     "achieved": solve_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": solve_gbs / HBM_PEAK_GBS,
                     "traffic": SOLVE_TRAFFIC_BYTES["fp64"],
                     "bytes_per_launch": solve_bytes, "ms_per_launch": solve_ms,
                     "bytes": "envelope of the factors read once per sweep + 4 FP64 vector "
                              "passes",
                     "stored_bytes_per_launch": bst["solve_stored_bytes"],
                     "stored_GBps": stored_gbs},
        "eigensolve_roofline": {"bound": "hbm", "kernel": "k_band_solve_m (GenEO block solves)",
                                "achieved": eig_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                "frac": eig_gbs / HBM_PEAK_GBS, "bytes_per_launch": eig_bytes,
                                "ms_per_launch": eig_ms},
        "spmv_roofline": {"bound": "hbm", "kernel": "k_spmv", "achieved": spmv_gbs,
                          "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": spmv_gbs / HBM_PEAK_GBS},
        "factor_roofline": {"bound": "mfma", "kernel": "k_chain + k_far + k_syrk_wide (subdomain "
                                                       "band Cholesky, FP64)",
                            "achieved": fac_tflops, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                            "frac": fac_tflops / FP64_PEAK_TFLOPS, "flops": fac_flops,
                            "ms": fac_ms},
    }
    s.close()
    del s
    extra = min(args.mixed_steps, args.steps)
    if not args.no_mixed:
        line["mixed"] = precision_block(gx, torch, cfg, extra, 1, x_fp64, ms_step, "mixed")
        line["mixed"]["subdomain_solve_traffic"] = SOLVE_TRAFFIC_BYTES["mixed"]
    if not args.no_target:
        tcfg = workloads.cfg2()
        t64, s2, o2, n02 = timed_steps(gx, torch, tcfg, gx.GX_FP64, extra, 1, "target fp64")
        xt = o2["x"].clone()
        tblk = {"workload": tcfg["name"] + " curved L-section, R 5 mm, 40 mm limbs, "
                                           "wrinkle A 0.3 mm L 4 mm, end moment, 32x2 "
                                           "subdomains, overlap 2, tau 0.1, rtol 1e-8",
                "n_free_dofs": n_free(s2), "fp64_ms_per_step": t64,
                "fp64_cg_iters": o2["iters"], "fp64_phases_ms": s2.phase_times()}
        s2.close()
        del s2
        m = precision_block(gx, torch, tcfg, extra, 1, xt, t64, "target mixed")
        tblk.update({"mixed_ms_per_step": m["ms_per_step"], "mixed_cg_iters": m["cg_iters"],
                     "speedup_mixed_vs_fp64": m["speedup_vs_fp64"],
                     "mixed_rel_diff_vs_fp64_solution": m["rel_diff_vs_fp64_solution"],
                     "mixed_phases_ms": m["phases_ms"], "steps": extra})
        line["target"] = tblk
    if sweep is not None:
        line["sweep"] = sweep
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
