"""Benchmark: solves/s of the solve phase on one MI355X.

Workload (default): the 3D unit cube with a 100^3 two-point-flux host grid,
log-normal host permeability (sigma = 1, seed 0) and nine full fracture
planes (three per axis) with aperture 1e-4, for the four fracture
permeability pairs (K_par, kappa) in {1e-4, 1e4}^2; Dirichlet p = 1 / 0 on
x = 0 / 1.  One step = one complete solve (zero initial guess to true
relative residual 1e-8) of the next system in rotation.  Inputs and
hierarchies are resident in HBM before the clock starts.

The JSON line reports the plain-FP64 method as ``value`` and, beside it, the
mixed mode (FP32 preconditioner, FP64 outer loop and coarse solve) on the
same systems, per-solve latency percentiles, the roofline position of the
dominant kernel (timed with HIP events inside the library on the launch
stream) and the CPU oracle timed on a bounded sample on this host.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
PAIRS = [(1e-4, 1e-4), (1e-4, 1e4), (1e4, 1e-4), (1e4, 1e4)]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=4)
    p.add_argument("--n", type=int, default=100, help="host cells per side")
    p.add_argument("--seeds", type=int, default=1, help="log-normal seeds per (K_par, kappa) pair")
    p.add_argument("--vcycles", type=int, default=1, help="V-cycles per block solve (Section 3.3)")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-iters", type=int, default=10, help="oracle FGMRES iterations in the CPU sample")
    p.add_argument("--copy-probe-mb", type=int, default=0,
                   help="only run a device-to-device copy of this many MiB (5 times) and exit; used to "
                        "calibrate hardware traffic counters against a copy of known size")
    p.add_argument("--kernel-class", default="auto",
                   help="kernel class for the roofline object (auto = largest total time)")
    return p.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); this build has no "
              "multi-GPU path.", file=sys.stderr)
        sys.exit(2)

    import torch

    if args.copy_probe_mb:
        n = args.copy_probe_mb * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": n * 8, "copy_probe_bytes_written": n * 8, "launches": 5}))
        return

    import synth
    from paper_2206_03203_amd import _lib as L
    from paper_2206_03203_amd import tpfa
    from paper_2206_03203_amd import ktimer

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    systems = []
    t_asm = t_setup = 0.0
    for seed in range(args.seeds):
        for kp, ka in PAIRS:
            sc = synth.regular_3d(n=args.n, k_par=kp, kappa=ka, seed=seed)
            t0 = time.perf_counter()
            A, b, part = tpfa.assemble(sc)
            t1 = time.perf_counter()
            o64 = L.mdp_options_default(precision=L.MDP_FP64, vcycles=args.vcycles)
            o32 = L.mdp_options_default(precision=L.MDP_MIXED, vcycles=args.vcycles)
            hs = {"fp64": L.mdp_setup(A, part, o64, stream)}
            hs["mixed"] = L.mdp_setup_like(hs["fp64"], o32, stream)
            t2 = time.perf_counter()
            t_asm += t1 - t0
            t_setup += t2 - t1
            bt = torch.tensor(b, dtype=torch.float64, device=dev)
            xt = torch.zeros_like(bt)
            systems.append({"name": sc.name, "h": hs, "b": bt, "x": xt, "n": A.shape[0], "nnz": A.nnz})
            log(f"[bench] set up {sc.name}: n={A.shape[0]} nnz={A.nnz}")
    torch.cuda.synchronize()

    def run(prec, steps, record=None):
        lat, iters, res = [], [], []
        for k in range(steps):
            s = systems[k % len(systems)]
            t0 = time.perf_counter()
            rc, st = L.mdp_solve(s["h"][prec], s["b"], s["x"], stream)
            lat.append(time.perf_counter() - t0)
            iters.append(st[0]["iters"])
            res.append(st[0]["rel_res_true"])
            if st[0]["converged"] != 1:
                raise RuntimeError(f"{s['name']} {prec} did not converge: {st[0]}")
        return lat, iters, res

    out = {}
    for prec in ("fp64", "mixed"):
        run(prec, args.warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lat, iters, res = run(prec, args.steps)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        out[prec] = {"seconds": t1 - t0, "lat": lat, "iters": iters, "res": res}
        log(f"[bench] {prec}: {args.steps} solves in {t1 - t0:.3f}s, iters={sorted(set(iters))}")

    fp = out["fp64"]
    mx = out["mixed"]
    value = args.steps / fp["seconds"]
    mixed_value = args.steps / mx["seconds"]

    # Roofline: the same FP64 steps again, with HIP events recorded by the
    # library around every launch of each kernel class on its launch stream
    # (kept out of the timed passes above: the events lengthen the gaps
    # between kernels, not the kernels).
    torch.cuda.synchronize()
    ktimer.begin_all()
    t0 = time.perf_counter()
    run("fp64", args.steps)
    torch.cuda.synchronize()
    t_ev = time.perf_counter() - t0
    kt = ktimer.end_all()
    single = {c: v for c, v in kt.items() if c in ktimer.SINGLE_KERNEL}
    kclass = max(single, key=lambda c: single[c]["ms"]) if args.kernel_class == "auto" else args.kernel_class
    k = kt[kclass]
    achieved = k["bytes"] / (k["ms"] * 1e-3) / 1e9 if k["ms"] > 0 else 0.0
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                "kernel": kclass, "kernel_symbol": ktimer.SINGLE_KERNEL.get(kclass), "launches": k["launches"],
                "avg_launch_us": round(1e3 * k["ms"] / max(k["launches"], 1), 2),
                "bytes_per_launch": round(k["bytes"] / max(k["launches"], 1)),
                "timed_region": f"the {args.steps} FP64 steps repeated with per-launch HIP events "
                                f"({t_ev:.3f}s with events vs {fp['seconds']:.3f}s without)"}
    classes = {c: {"ms": round(v["ms"], 3), "launches": v["launches"],
                   "GB/s": round(v["bytes"] / (v["ms"] * 1e-3) / 1e9, 1) if v["ms"] > 0 else None}
               for c, v in kt.items()}

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(args, float(np.mean(fp["iters"])))

    for s in systems:
        for h in s["h"].values():
            L.mdp_destroy(h)

    def pct(a, q):
        return round(1e3 * float(np.percentile(a, q)), 3)

    line = {
        "metric": "solves/s to 1e-8 rel residual (FP64 method; mixed beside it)",
        "value": round(value, 3),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * fp["seconds"] / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"3d-unit-cube-{args.n}^3-9-planes-lognormal-host",
                   "systems": len(systems), "unknowns": systems[0]["n"], "nnz": systems[0]["nnz"],
                   "fracture_perm_pairs": PAIRS, "rtol": 1e-8, "vcycles": args.vcycles},
        "p50_ms": pct(fp["lat"], 50),
        "p99_ms": pct(fp["lat"], 99),
        "iters": sorted(set(fp["iters"])),
        "max_rel_res": max(fp["res"]),
        "mixed": {"value": round(mixed_value, 3), "unit": "solves/s", "dtype": "f32 preconditioner / f64 outer",
                  "ms_per_step": round(1e3 * mx["seconds"] / args.steps, 3), "p50_ms": pct(mx["lat"], 50),
                  "p99_ms": pct(mx["lat"], 99), "iters": sorted(set(mx["iters"])),
                  "max_rel_res": max(mx["res"]), "speedup_vs_fp64": round(mixed_value / value, 3)},
        "roofline": roofline,
        "kernel_classes": classes,
        "setup_s": {"assembly": round(t_asm, 2), "host_setup_and_upload": round(t_setup, 2)},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


def cpu_baseline(args, gpu_iters_per_solve):
    """The FP64 oracle on this host: set up the first system of the workload
    (untimed), time ``cpu_iters`` FGMRES iterations of its solve, and scale
    to solves/s with the GPU's mean iteration count per solve."""
    import synth
    from oracle import assembly as oa, solve as osv

    kp, ka = PAIRS[0]
    sc = synth.regular_3d(n=args.n, k_par=kp, kappa=ka, seed=0)
    log("[bench] cpu oracle: assembling and setting up (untimed)")
    t0 = time.perf_counter()
    A, b, part = oa.assemble(sc)
    M = osv.setup(A, part)
    t1 = time.perf_counter()
    log(f"[bench] cpu oracle setup {t1 - t0:.1f}s; timing {args.cpu_iters} iterations")
    opts = osv.SolveOptions(maxiter=args.cpu_iters)
    from threadpoolctl import threadpool_limits
    with threadpool_limits(limits=1):
        t2 = time.perf_counter()
        res, _, _ = osv.solve(A, b, part, opts, M=M)
        t3 = time.perf_counter()
    per_iter = (t3 - t2) / max(res.iters, 1)
    per_solve = per_iter * gpu_iters_per_solve
    return {"value": round(1.0 / per_solve, 5), "unit": "solves/s", "cores": 1, "kind": "oracle",
            "sample": f"FP64 oracle FGMRES on {sc.name} ({A.shape[0]} unknowns): first {res.iters} "
                      f"iterations timed ({t3 - t2:.1f}s), scaled by the GPU's mean "
                      f"{gpu_iters_per_solve:.1f} iterations per solve; oracle setup "
                      f"({t1 - t0:.1f}s) not timed",
            "host_cpu_count": os.cpu_count()}


if __name__ == "__main__":
    main()
