"""Benchmark: solves/s of the solve phase on one MI355X.

Headline workload (``value``): the 3D unit cube with a 100^3 two-point-flux
host grid, log-normal host permeability (sigma = 1, seeds 0, 1 and 2) and
nine full fracture planes (three per axis) with aperture 1e-4, for the four
fracture permeability pairs (K_par, kappa) in {1e-4, 1e4}^2: twelve systems;
Dirichlet p = 1 / 0 on x = 0 / 1.  Library defaults throughout (SA strength
threshold 0.02, ``--theta`` changes it for the headline, flux and 160^3
sections).  One step = one complete solve (zero initial guess to true
relative residual 1e-8) of the next system in rotation, plain FP64.  Inputs
and hierarchies are resident in HBM before the clock starts.

Beside it on the same JSON line: the mixed mode (FP32 preconditioner, FP64
outer loop and coarse solve) on the same systems, per-solve latency
percentiles, the four systems as one batch (``batched``), four right-hand
sides per call (``multi_rhs``), the error of every GPU result against the
FP64 oracle's solution of the same system (``err_vs_oracle``), the roofline
position of the dominant kernel and of every kernel class (HIP events inside
the library on the launch stream), and the CPU oracle timed on this host.
Further sections, each with its own set-up outside its clock:

* ``config1``: the 2D 32x32 grid with four full fracture lines, FP64;
* ``flux``: the headline's four systems in the paper's own block reading
  (subdomain pressures with explicit intersection lines and points on
  Omega, interface fluxes on Gamma), FP64 and mixed, with its own roofline
  pass;
* ``cube160``: the same cube at 160^3 (4.33M unknowns), FP64 and mixed,
  with its own roofline pass;
* ``batch``: 256 uneven 2D systems (side uniform in 64..512, 1..20 random
  fracture segments, log-uniform permeabilities in [1e-4, 1e4]), four
  right-hand sides each, mixed, one mdp_solve_batch call per step, beside the
  same pairs solved one system at a time;
* ``serve``: a pool of resident systems (half 2D as above, half 3D with side
  40..160 and 3..9 random planes), mixed, served by mdp_submit/mdp_poll under
  open-loop Poisson arrivals at 0.5, 0.8 and 0.95 of the saturated rate.

``--mode batch`` and ``--mode serve`` print those workloads alone, at full
size (serving: 64 systems, 2000 requests per rate).
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
DEFAULT_SEEDS = 3  # log-normal host permeability seeds 0, 1, 2 per pair: twelve headline systems


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=4)
    p.add_argument("--n", type=int, default=100, help="host cells per side")
    p.add_argument("--seeds", type=int, default=DEFAULT_SEEDS,
                   help="log-normal seeds per (K_par, kappa) pair (headline)")
    p.add_argument("--vcycles", type=int, default=1, help="V-cycles per block solve (Section 3.3)")
    p.add_argument("--restart", type=int, default=64, help="FGMRES restart length (at most 64)")
    p.add_argument("--theta", type=float, default=0.02,
                   help="strength threshold of the SA aggregation (reading R8)")
    p.add_argument("--max-coarse", type=int, default=400,
                   help="AMG: stop coarsening at this many unknowns (the coarsest is dense up to 2000)")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--copy-probe-mb", type=int, default=0,
                   help="only run a device-to-device copy of this many MiB (5 times) and exit; used to "
                        "calibrate hardware traffic counters against a copy of known size")
    p.add_argument("--kernel-class", default="auto",
                   help="kernel class for the roofline object (auto = largest total time)")
    p.add_argument("--mode", choices=["solve", "batch", "serve"], default="solve")
    p.add_argument("--block", choices=["lower", "diag", "upper"], default="lower",
                   help="block preconditioner: M_L (eq. 8, the paper's), or the inexact B_D / B_U of Section 3.2")
    p.add_argument("--smoother", choices=["l1jacobi", "gs"], default="l1jacobi",
                   help="V-cycle smoother: l1-Jacobi, or multicolour Gauss-Seidel (the paper's smoothing, Section 4)")
    p.add_argument("--graphs", action="store_true",
                   help="replay each Arnoldi step from a captured HIP graph instead of launching its kernels")
    p.add_argument("--no-autotune", action="store_true",
                   help="keep the fixed rule for sparse formats instead of timing candidates at setup")
    p.add_argument("--multi-rhs", type=int, default=2,
                   help="rounds over the systems with four right-hand sides each (0 = skip)")
    p.add_argument("--systems", type=int, default=256, help="batch mode: number of 2D systems")
    p.add_argument("--rhs", type=int, default=4, help="batch mode: right-hand sides per system")
    p.add_argument("--side-range", type=int, nargs=2, default=[64, 512],
                   help="batch mode: range of the 2D systems' side")
    p.add_argument("--pool", type=int, default=64, help="serve mode: resident systems (half 2D, half 3D)")
    p.add_argument("--requests", type=int, default=2000, help="serve mode: requests per arrival rate")
    p.add_argument("--slots", type=int, default=4, help="serve mode: server slots")
    p.add_argument("--budget-gb", type=float, default=64.0, help="serve mode: workspace memory budget")
    p.add_argument("--serve-grouping", action="store_true",
                   help="serve mode: solve queued requests of one system together (mdp_server_set_grouping)")
    p.add_argument("--cpu-seconds", type=float, default=20.0,
                   help="solve time after which the CPU oracle sample stops taking further systems")
    p.add_argument("--sections", default="config1,flux,cube160,batch,serve",
                   help="default mode: further workloads on the JSON line (comma list of config1, flux, "
                        "cube160, batch, serve; empty = the headline only)")
    p.add_argument("--dim-aware", action="store_true",
                   help="flux formulation: dimension-aware aggregation (mdp_setup_labeled, Section 3.3)")
    p.add_argument("--formulation", choices=["pressure", "flux"], default="pressure",
                   help="cube workload: host/fracture pressures (Gamma = fracture cells), or the paper's own "
                        "reading with explicit intersections and interface fluxes as Gamma")
    p.add_argument("--tune-file", default=None,
                   help="record the autotuner's format choices here and reuse the ones recorded (mdp_tune_file)")
    return p.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the library has no "
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

    from paper_2206_03203_amd import _lib as L
    if args.tune_file:
        L.mdp_tune_file(args.tune_file)

    if args.mode == "batch":
        print(json.dumps(mode_batch(args)), flush=True)
        return
    if args.mode == "serve":
        print(json.dumps(mode_serve(args)), flush=True)
        return

    t_start = time.perf_counter()
    line = run_cube(args, args.n, args.steps, args.warmup, headline=True)
    sections = [x for x in args.sections.split(",") if x]
    if "config1" in sections:
        line["config1"] = run_config1(args)
    if "flux" in sections and args.formulation == "pressure":
        c = run_cube(args, args.n, 8, 4, headline=False, formulation="flux")
        line["flux"] = {k: c[k] for k in ("value", "unit", "ms_per_step", "p50_ms", "p99_ms", "iters",
                                          "max_rel_res", "mixed", "roofline", "config", "setup_s")}
        line["flux"]["what"] = ("the same four systems in the paper's own block reading: Omega = pressures of "
                                "host, fracture, intersection-line and point cells, Gamma = interface fluxes; "
                                "value = FP64 solves/s, mixed beside it")
    if "cube160" in sections and args.n != 160:
        c = run_cube(args, 160, 8, 4, headline=False)
        line["cube160"] = {k: c[k] for k in ("value", "unit", "ms_per_step", "p50_ms", "p99_ms", "iters",
                                              "max_rel_res", "mixed", "roofline", "roofline_classes",
                                              "config", "setup_s")}
        line["cube160"]["what"] = ("the same four (K_par, kappa) systems at 160^3; value = FP64 solves/s, "
                                   "mixed beside it; eight timed solves per precision after four untimed")
    if "batch" in sections:
        bargs = argparse.Namespace(**vars(args))
        bargs.steps, bargs.warmup, bargs.no_cpu_baseline = 3, 1, True
        b = mode_batch(bargs, seq_steps=1)
        line["batch"] = {k: b[k] for k in ("value", "unit", "ms_per_step", "iters_mean", "iters_max",
                                           "max_rel_res", "sequential_mixed", "sequential_fp64",
                                           "speedup_vs_sequential_fp64", "speedup_vs_sequential_mixed",
                                           "roofline", "config", "setup_s")}
        line["batch"]["what"] = "256 uneven 2D systems x 4 right-hand sides, mixed, one mdp_solve_batch per step"
    if "serve" in sections:
        sargs = argparse.Namespace(**vars(args))
        sargs.pool, sargs.requests, sargs.no_cpu_baseline = 32, 200, True
        v = mode_serve(sargs)
        line["serve"] = {k: v[k] for k in ("value", "unit", "saturated", "poisson", "alone_service_ms",
                                           "config", "setup_s")}
        line["serve"]["what"] = ("served solves/s, mixed, pool of 32 resident systems (16 2D, 16 3D), "
                                 "200 Poisson requests per arrival rate; --mode serve runs 64 systems and "
                                 "2000 requests per rate")
    line["bench_wall_s"] = round(time.perf_counter() - t_start, 1)
    print(json.dumps(line), flush=True)


def run_cube(args, n, steps, warmup, headline, formulation=None):
    """The 3D cube workload at n^3: the four (K_par, kappa) systems set up in
    both precisions, timed FP64 and mixed passes of `steps` solves in
    rotation, a roofline pass, and (headline only) the batched and
    four-right-hand-side forms, the CPU oracle and the error of each result
    against the oracle's solution."""
    import torch
    import synth
    from paper_2206_03203_amd import _lib as L
    from paper_2206_03203_amd import tpfa, tpfa_flux

    formulation = formulation or args.formulation
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    systems = []
    info = None
    t_asm = t_setup = 0.0
    for seed in range(args.seeds if headline else 1):
        for kp, ka in PAIRS:
            sc = synth.regular_3d(n=n, k_par=kp, kappa=ka, seed=seed)
            t0 = time.perf_counter()
            if formulation == "flux":
                A, b, part, info = tpfa_flux.assemble_flux(sc)
            else:
                A, b, part = tpfa.assemble(sc)
            t1 = time.perf_counter()
            fl = (L.MDP_NO_AUTOTUNE if args.no_autotune else 0) | (L.MDP_GRAPHS if args.graphs else 0)
            bf = {"lower": L.MDP_BLOCK_LOWER, "diag": L.MDP_BLOCK_DIAG, "upper": L.MDP_BLOCK_UPPER}[args.block]
            sm = L.MDP_SMOOTH_GS if args.smoother == "gs" else L.MDP_SMOOTH_L1JACOBI
            o64 = L.mdp_options_default(precision=L.MDP_FP64, vcycles=args.vcycles, flags=fl, block_form=bf,
                                        max_coarse=args.max_coarse, restart=args.restart, smoother=sm,
                                        strength_theta=args.theta)
            o32 = L.mdp_options_default(precision=L.MDP_MIXED, vcycles=args.vcycles, flags=fl, block_form=bf,
                                        max_coarse=args.max_coarse, restart=args.restart, smoother=sm,
                                        strength_theta=args.theta)
            labels = info["labels"] if (formulation == "flux" and args.dim_aware) else None
            hs = {"fp64": L.mdp_setup(A, part, o64, stream, labels=labels)}
            hs["mixed"] = L.mdp_setup_like(hs["fp64"], o32, stream)
            t2 = time.perf_counter()
            t_asm += t1 - t0
            t_setup += t2 - t1
            bt = torch.tensor(b, dtype=torch.float64, device=dev)
            xt = torch.zeros_like(bt)
            systems.append({"name": sc.name, "sc": sc, "h": hs, "b": bt, "x": xt, "n": A.shape[0], "nnz": A.nnz})
            log(f"[bench] set up {sc.name}: n={A.shape[0]} nnz={A.nnz}")
    torch.cuda.synchronize()

    failed = set()

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
                if args.block == "lower":
                    raise RuntimeError(f"{s['name']} {prec} did not converge: {st[0]}")
                failed.add(s["name"])  # comparison forms: reported, not fatal
        return lat, iters, res

    out = {}
    for prec in ("fp64", "mixed"):
        run(prec, warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lat, iters, res = run(prec, steps)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        out[prec] = {"seconds": t1 - t0, "lat": lat, "iters": iters, "res": res}
        log(f"[bench] {n}^3 {prec}: {steps} solves in {t1 - t0:.3f}s, iters={sorted(set(iters))}")

    fp = out["fp64"]
    mx = out["mixed"]
    value = steps / fp["seconds"]
    mixed_value = steps / mx["seconds"]

    # Beside the one-at-a-time solves: the same systems solved together as
    # one block-diagonal batch (mdp_solve_batch), one launch per operation.
    batched = {}
    if headline and args.block == "lower":
        nb = max(1, steps // len(systems))
        for prec in ("fp64", "mixed"):
            hs = [s["h"][prec] for s in systems]
            bs = [s["b"] for s in systems]
            xs = [torch.zeros_like(s["b"]) for s in systems]
            L.mdp_solve_batch(hs, bs, xs, stream)  # builds the batch plan (untimed)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(nb):
                rc, st = L.mdp_solve_batch(hs, bs, xs, stream)
                if rc != L.MDP_OK:
                    raise RuntimeError(f"batched {prec} solve did not converge: rc={rc}")
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            batched[prec] = {"value": round(len(systems) * nb / dt, 3), "unit": "solves/s",
                             "ms_per_batch": round(1e3 * dt / nb, 3), "batches": nb,
                             "iters": [x["iters"] for x in st],
                             "max_rel_res": max(x["rel_res_true"] for x in st)}
            log(f"[bench] batched {prec}: {nb} batches of {len(systems)} in {dt:.3f}s")
        batched["what"] = "the same systems solved together as one block-diagonal batch"

    # Beside them: four right-hand sides per system (the Dirichlet data alone
    # and with three host source fields) in one mdp_solve call, which takes
    # the columns four at a time with each matrix read once for all four,
    # against the same columns solved one at a time.
    multi_rhs = {}
    mr_systems = systems[:len(PAIRS)]  # the first seed's four systems
    if headline and args.block == "lower" and args.multi_rhs and formulation == "pressure":
        for s in mr_systems:
            fs = [None] + [synth.host_sources(s["sc"], 100 + k) for k in range(3)]
            _, B, _ = tpfa.assemble(s["sc"], sources=fs)
            s["B4"] = torch.tensor(np.ascontiguousarray(B.T), dtype=torch.float64, device=dev)
        nr = args.multi_rhs
        for prec in ("fp64", "mixed"):
            xs = [torch.zeros_like(s["B4"]) for s in mr_systems]
            for s, x in zip(mr_systems, xs):
                L.mdp_solve(s["h"][prec], s["B4"], x, stream)  # builds the four-column plan (untimed)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            its = []
            for _ in range(nr):
                for s, x in zip(mr_systems, xs):
                    rc, st = L.mdp_solve(s["h"][prec], s["B4"], x, stream)
                    if rc != L.MDP_OK:
                        raise RuntimeError(f"{s['name']} {prec} four-column solve did not converge")
                    its += [c["iters"] for c in st]
            torch.cuda.synchronize()
            dt4 = time.perf_counter() - t0
            t0 = time.perf_counter()
            its1 = []
            for _ in range(nr):
                for s, x in zip(mr_systems, xs):
                    for k in range(s["B4"].shape[0]):
                        rc, st = L.mdp_solve(s["h"][prec], s["B4"][k], x[k], stream)
                        its1.append(st[0]["iters"])
            torch.cuda.synchronize()
            dt1 = time.perf_counter() - t0
            ns = nr * sum(s["B4"].shape[0] for s in mr_systems)
            mem = [L.mdp_multi_rhs_memory(s["h"][prec]) for s in mr_systems]
            multi_rhs[prec] = {"value": round(ns / dt4, 3), "unit": "solves/s",
                               "one_column_at_a_time": round(ns / dt1, 3),
                               "speedup": round(dt1 / dt4, 3), "solves": ns,
                               "iters": sorted(set(its)), "iters_one_at_a_time": sorted(set(its1)),
                               "handles_with_plan": sum(m["plan_bytes"] > 0 for m in mem),
                               "plan_gb": [round(m["plan_bytes"] / 1e9, 3) for m in mem],
                               "shared_workspace_gb": round(max(m["shared_bytes"] for m in mem) / 1e9, 3),
                               "held_gb": round(mem[-1]["held"] / 1e9, 3),
                               "budget_gb": round(mem[-1]["budget"] / 1e9, 3)}
            log(f"[bench] four right-hand sides {prec}: {ns} solves in {dt4:.3f}s "
                f"(one column at a time {dt1:.3f}s)")
        multi_rhs["what"] = ("the four systems of seed 0, each with four right-hand sides (Dirichlet data "
                             "alone and with three uniform host source fields) in one mdp_solve call")

    # Roofline: the same FP64 steps again, with HIP events recorded by the
    # library around every launch of each kernel class on its launch stream
    # (kept out of the timed passes above: the events lengthen the gaps
    # between kernels, not the kernels).
    roofline, classes = roofline_pass(lambda: run("fp64", steps), args.kernel_class,
                                      f"the {steps} FP64 steps repeated", fp["seconds"])
    if roofline["kernel_symbol"] and args.seeds == DEFAULT_SEEDS and args.vcycles == 1 and args.block == "lower" and \
            args.max_coarse == 400 and args.restart == 64 and formulation == "pressure" and args.smoother == "l1jacobi" \
            and args.theta == 0.02:
        roofline["traffic"] = measured_traffic(roofline["kernel_symbol"].split("<")[0], f"cube{n}", args.theta)

    # Each system's solution in both precisions against the oracle's solution
    # of the same system (the oracle solves are the CPU baseline's).
    cpu, errs = None, None
    if headline and not args.no_cpu_baseline and formulation == "pressure":
        items = [(synth.regular_3d(n=n, k_par=kp, kappa=ka, seed=0), None) for kp, ka in PAIRS]
        cpu, xo = cpu_full_solves(args, items, "seed 0")
        errs = []
        for s, (name, xor, it_o) in zip(systems, xo):
            e = {"system": name, "oracle_iters": it_o}
            for prec in ("fp64", "mixed"):
                x = torch.zeros_like(s["b"])
                rc, st = L.mdp_solve(s["h"][prec], s["b"], x, stream)
                xh = x.cpu().numpy()
                e[prec] = float(np.linalg.norm(xh - xor) / np.linalg.norm(xor))
                e[prec + "_iters"] = st[0]["iters"]
            errs.append(e)

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
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": round(1e3 * fp["seconds"] / steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"3d-unit-cube-{n}^3-9-planes-lognormal-host" +
                               ("-interface-fluxes" if formulation == "flux" else ""),
                   "formulation": formulation, "dim_aware": bool(formulation == "flux" and args.dim_aware),
                   "unknown_kinds": {k: v for k, v in info.items() if k != "labels"} if info else None,
                   "systems": len(systems), "unknowns": systems[0]["n"], "nnz": systems[0]["nnz"],
                   "fracture_perm_pairs": PAIRS, "rtol": 1e-8, "vcycles": args.vcycles,
                   "amg_max_coarse": args.max_coarse, "amg_theta": args.theta, "restart": args.restart,
                   "autotune": not args.no_autotune, "graphs": args.graphs, "smoother": args.smoother,
                   "block_preconditioner": args.block},
        "p50_ms": pct(fp["lat"], 50),
        "p99_ms": pct(fp["lat"], 99),
        "iters": sorted(set(fp["iters"])),
        "max_rel_res": max(fp["res"]),
        "not_converged": sorted(failed),
        "mixed": {"value": round(mixed_value, 3), "unit": "solves/s", "dtype": "f32 preconditioner / f64 outer",
                  "ms_per_step": round(1e3 * mx["seconds"] / steps, 3), "p50_ms": pct(mx["lat"], 50),
                  "p99_ms": pct(mx["lat"], 99), "iters": sorted(set(mx["iters"])),
                  "max_rel_res": max(mx["res"]), "speedup_vs_fp64": round(mixed_value / value, 3)},
        "batched": batched or None,
        "multi_rhs": multi_rhs or None,
        "err_vs_oracle": errs,
        "roofline": roofline,
        "roofline_classes": classes,
        "setup_s": {"assembly": round(t_asm, 2), "host_setup_and_upload": round(t_setup, 2)},
        "cpu_baseline": cpu,
    }
    return line


def run_config1(args):
    """The 2D 32x32 grid with four full fracture lines (K_par = kappa = 1e4,
    aperture 1e-4), FP64 and mixed: solves/s over 200 solves each, and the
    error against the oracle's solution."""
    import torch
    import synth
    from oracle import assembly as oa, solve as osv
    from paper_2206_03203_amd import _lib as L
    from paper_2206_03203_amd import tpfa

    stream = torch.cuda.current_stream()
    sc = synth.grid_2d_four_lines(32)
    A, b, part = tpfa.assemble(sc)
    Ao, bo, po = oa.assemble(sc)
    ref, _, _ = osv.solve(Ao, bo, po, osv.SolveOptions())
    bt = torch.tensor(b, dtype=torch.float64, device="cuda:0")
    out = {"workload": "2d-32x32-four-lines", "unknowns": A.shape[0], "nnz": A.nnz, "oracle_iters": ref.iters}
    for prec, pv in (("fp64", L.MDP_FP64), ("mixed", L.MDP_MIXED)):
        h = L.mdp_setup(A, part, L.mdp_options_default(precision=pv), stream)
        x = torch.zeros_like(bt)
        for _ in range(10):
            L.mdp_solve(h, bt, x, stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(200):
            rc, st = L.mdp_solve(h, bt, x, stream)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        xh = x.cpu().numpy()
        out[prec] = {"value": round(200 / dt, 2), "unit": "solves/s", "iters": st[0]["iters"],
                     "rel_res": st[0]["rel_res_true"],
                     "err_vs_oracle": float(np.linalg.norm(xh - ref.x) / np.linalg.norm(ref.x))}
        L.mdp_destroy(h)
    log(f"[bench] config1: {out}")
    return out


def roofline_pass(fn, kernel_class, what, seconds_plain, exact=None):
    """Run fn() once more with per-launch HIP events in the library and
    return (roofline object of the dominant single-symbol kernel class,
    per-class summary).  `exact`: the classes whose byte counts are exact
    (None = all); the others get no bandwidth figure."""
    import torch
    from paper_2206_03203_amd import ktimer

    torch.cuda.synchronize()
    ktimer.begin_all()
    t0 = time.perf_counter()
    fn()
    torch.cuda.synchronize()
    t_ev = time.perf_counter() - t0
    kt = ktimer.end_all()
    single = {c: v for c, v in kt.items() if c in ktimer.SINGLE_KERNEL and (exact is None or c in exact)}
    kclass = max(single, key=lambda c: single[c]["ms"]) if kernel_class == "auto" else kernel_class
    k = kt[kclass]
    achieved = k["bytes"] / (k["ms"] * 1e-3) / 1e9 if k["ms"] > 0 else 0.0
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                "kernel": kclass, "kernel_symbol": ktimer.SINGLE_KERNEL.get(kclass), "launches": k["launches"],
                "avg_launch_us": round(1e3 * k["ms"] / max(k["launches"], 1), 2),
                "bytes_per_launch": round(k["bytes"] / max(k["launches"], 1)),
                "timed_region": f"{what} with per-launch HIP events "
                                f"({t_ev:.3f}s with events vs {seconds_plain:.3f}s without)"}
    # every class against the same peak: the classes that are one kernel symbol,
    # and vcycle_other / other, which gather several kernels (their figure is
    # the class's bytes over its summed launch time)
    dom = max(kt, key=lambda c: kt[c]["ms"])
    classes = {}
    for c, v in kt.items():
        gbs = v["bytes"] / (v["ms"] * 1e-3) / 1e9 if v["ms"] > 0 and (exact is None or c in exact) else None
        classes[c] = {"ms": round(v["ms"], 3), "launches": v["launches"],
                      "avg_launch_us": round(1e3 * v["ms"] / max(v["launches"], 1), 2),
                      "GB/s": round(gbs, 1) if gbs is not None else None,
                      "frac": round(gbs / HBM_PEAK_GBS, 4) if gbs is not None else None,
                      "kernels": "one symbol" if c in ktimer.SINGLE_KERNEL else "several"}
    classes["largest_by_time"] = dom
    return roofline, classes


def kernel_source_hash() -> str:
    """SHA-256 over the device kernel sources (kernel bodies and the tile and
    block constants their launches use)."""
    import hashlib
    h = hashlib.sha256()
    for f in ("kernels.hpp", "types.hpp"):
        with open(os.path.join(ROOT, "paper_2206_03203_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(symbol: str, workload: str, theta: float):
    """HBM bytes per launch of kernel `symbol` on `workload` from the
    committed hardware-counter summary (FETCH_SIZE and WRITE_SIZE passes,
    scaled by a copy of known size), or None when there is none, the kernel
    sources changed since the counters were taken, or the counters were taken
    with another strength threshold (another hierarchy, other iteration
    counts, so another mix of Arnoldi steps)."""
    path = os.path.join(ROOT, "profiles", f"{symbol}_{workload}_traffic.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith((" ", "#")):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha256") != kernel_source_hash():
        return None
    try:
        if float(kv.get("amg_theta", "nan")) != theta:
            return None
    except ValueError:
        return None
    try:
        return float(kv["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def _pct(a, q):
    return round(1e3 * float(np.percentile(a, q)), 3) if len(a) else None


def _setup_pool(scs, sources_per_sys, precisions, stream, tag, flags=0, restart=64):
    """Assemble and set up every scenario; returns a list of dicts holding the
    handles (one per precision, sharing the host setup), the right-hand sides
    as a (nrhs, n) device tensor and the sizes."""
    import torch
    from paper_2206_03203_amd import _lib as L
    from paper_2206_03203_amd import tpfa

    out = []
    t_asm = t_set = 0.0
    t_last = time.perf_counter()
    for i, (sc, fs) in enumerate(zip(scs, sources_per_sys)):
        t0 = time.perf_counter()
        A, B, part = tpfa.assemble(sc, sources=fs)
        t1 = time.perf_counter()
        hs = {}
        first = None
        for prec in precisions:
            o = L.mdp_options_default(precision={"fp64": L.MDP_FP64, "mixed": L.MDP_MIXED}[prec], flags=flags,
                                      restart=restart)
            hs[prec] = L.mdp_setup(A, part, o, stream) if first is None else L.mdp_setup_like(first, o, stream)
            first = first or hs[prec]
        t2 = time.perf_counter()
        t_asm += t1 - t0
        t_set += t2 - t1
        b = torch.tensor(np.ascontiguousarray(B.T), dtype=torch.float64, device="cuda:0")
        out.append({"sc": sc, "h": hs, "b": b, "n": A.shape[0], "nnz": A.nnz, "fs": fs})
        if time.perf_counter() - t_last > 10 or i + 1 == len(scs):
            t_last = time.perf_counter()
            log(f"[bench] {tag}: set up {i + 1}/{len(scs)} systems")
    torch.cuda.synchronize()
    return out, t_asm, t_set


def _destroy_pool(pool):
    from paper_2206_03203_amd import _lib as L
    for s in pool:
        for h in s["h"].values():
            L.mdp_destroy(h)


def mode_batch(args, seq_steps=None):
    """Uneven 2D batch with several right-hand sides per system; returns the
    JSON object."""
    import torch
    import synth
    from paper_2206_03203_amd import _lib as L

    stream = torch.cuda.current_stream()
    scs = [synth.random_2d(s, n_range=tuple(args.side_range)) for s in range(args.systems)]
    srcs = [[synth.host_sources(sc, 4 * s + k) for k in range(args.rhs)] for s, sc in enumerate(scs)]
    fl = (L.MDP_NO_AUTOTUNE if args.no_autotune else 0) | (L.MDP_GRAPHS if args.graphs else 0)
    pool, t_asm, t_set = _setup_pool(scs, srcs, ("mixed", "fp64"), stream, "batch", fl, args.restart)
    pairs = sum(p["b"].shape[0] for p in pool)
    unknowns = sum(p["n"] * p["b"].shape[0] for p in pool)
    xs = [torch.zeros_like(p["b"]) for p in pool]

    def batch():
        rc, st = L.mdp_solve_batch([p["h"]["mixed"] for p in pool], [p["b"] for p in pool], xs, stream)
        if rc != L.MDP_OK:
            raise RuntimeError(f"batch did not converge: rc={rc}")
        return st

    def seq(prec):
        st_all = []
        for p, x in zip(pool, xs):
            rc, st = L.mdp_solve(p["h"][prec], p["b"], x, stream)
            if rc != L.MDP_OK:
                raise RuntimeError(f"{p['sc'].name} {prec} did not converge")
            st_all += st
        return st_all

    def timed(fn, steps, warm):
        for _ in range(warm):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            st = fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps, st

    log(f"[bench] batch: {len(pool)} systems, {pairs} pairs, {unknowns} unknowns in all")
    t_batch, st_b = timed(batch, args.steps, args.warmup)
    log(f"[bench] batch: {1e3 * t_batch:.1f} ms per batch")
    ns = seq_steps or max(1, args.steps // 2)
    t_seq, st_s = timed(lambda: seq("mixed"), ns, 1)
    log(f"[bench] sequential mixed: {1e3 * t_seq:.1f} ms per batch")
    t_seq64, st_64 = timed(lambda: seq("fp64"), ns, 1)
    log(f"[bench] sequential fp64: {1e3 * t_seq64:.1f} ms per batch")
    # In a batch the sparse products skip the rows of pairs that have stopped,
    # so only the Arnoldi classes (corrected per pair by the library) have
    # exact byte counts.
    roofline, classes = roofline_pass(batch, args.kernel_class, "one batch repeated", t_batch,
                                      exact=("arnoldi_dot", "arnoldi_axpy"))

    cpu = None
    if not args.no_cpu_baseline:
        cpu, _ = cpu_full_solves(args, [(p["sc"], p["fs"][0]) for p in pool], "first right-hand side")
    _destroy_pool(pool)
    its_b = [s["iters"] for s in st_b]
    its_s = [s["iters"] for s in st_s]
    line = {
        "metric": "solves/s to 1e-8 rel residual (batched, mixed precision)",
        "value": round(pairs / t_batch, 2),
        "unit": "solves/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(1e3 * t_batch, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 preconditioner / f64 outer", "data": "synthetic",
        "config": {"workload": f"2d-uneven-batch-{args.systems}x{args.rhs}", "systems": len(pool),
                   "pairs": pairs, "unknowns_total": unknowns, "side_range": list(args.side_range),
                   "segments_max": 20, "rtol": 1e-8, "restart": args.restart, "graphs": args.graphs},
        "iters_mean": round(float(np.mean(its_b)), 2), "iters_max": int(max(its_b)),
        "max_rel_res": max(s["rel_res_true"] for s in st_b),
        "sequential_mixed": {"value": round(pairs / t_seq, 2), "unit": "solves/s",
                             "iters_mean": round(float(np.mean(its_s)), 2)},
        "sequential_fp64": {"value": round(pairs / t_seq64, 2), "unit": "solves/s",
                            "iters_mean": round(float(np.mean([s["iters"] for s in st_64])), 2)},
        "speedup_vs_sequential_fp64": round(t_seq64 / t_batch, 3),
        "speedup_vs_sequential_mixed": round(t_seq / t_batch, 3),
        "roofline": roofline, "roofline_classes": classes,
        "setup_s": {"assembly": round(t_asm, 2), "host_setup_and_upload": round(t_set, 2)},
        "cpu_baseline": cpu,
    }
    return line


def mode_serve(args):
    """Open-loop Poisson arrivals over a pool of resident systems; returns
    the JSON object."""
    import torch
    import synth
    from paper_2206_03203_amd import _lib as L

    stream = torch.cuda.current_stream()
    half = args.pool // 2
    scs = [synth.random_2d(1000 + s) for s in range(half)]
    scs += [synth.random_3d(2000 + s) for s in range(args.pool - half)]
    nb = 4  # right-hand sides per system to draw requests from
    srcs = [[synth.host_sources(sc, 4 * (3000 + s) + k) for k in range(nb)] for s, sc in enumerate(scs)]
    pool, t_asm, t_set = _setup_pool(scs, srcs, ("mixed",), stream, "serve",
                                     L.MDP_NO_AUTOTUNE if args.no_autotune else 0, args.restart)
    budget = int(args.budget_gb * (1 << 30))
    srv = L.mdp_server_create(budget, args.slots)
    L.mdp_server_set_grouping(srv, args.serve_grouping)
    for p in pool:
        L.mdp_server_register(srv, p["h"]["mixed"])
    rng = np.random.default_rng(12345)

    def draw(k):
        ids = rng.integers(0, len(pool), size=k)
        cols = rng.integers(0, nb, size=k)
        return list(zip(ids.tolist(), cols.tolist()))

    def serve(reqs, arrivals):
        """Submit request i at arrivals[i] (seconds from start; None = all at
        once); return per-request latency (s), makespan (s), iterations."""
        xs = [torch.empty(pool[i]["n"], dtype=torch.float64, device="cuda:0") for i, _ in reqs]
        torch.cuda.synchronize()
        lat = [0.0] * len(reqs)
        iters = [0] * len(reqs)
        t_sub = [0.0] * len(reqs)
        inflight = {}
        nxt = 0
        t0 = time.perf_counter()
        t_log = t0
        while nxt < len(reqs) or inflight:
            now = time.perf_counter() - t0
            while nxt < len(reqs) and (arrivals is None or arrivals[nxt] <= now):
                i, c = reqs[nxt]
                t_sub[nxt] = time.perf_counter()
                inflight[L.mdp_submit(srv, pool[i]["h"]["mixed"], pool[i]["b"][c], xs[nxt])] = nxt
                nxt += 1
            for t in list(inflight):
                rc, st = L.mdp_poll(srv, t)
                if rc == L.MDP_PENDING:
                    continue
                j = inflight.pop(t)
                lat[j] = time.perf_counter() - t_sub[j]
                iters[j] = st[0]["iters"]
                if rc != L.MDP_OK:
                    raise RuntimeError(f"request {j} failed: rc={rc}")
            if time.perf_counter() - t_log > 20:
                t_log = time.perf_counter()
                log(f"[bench] serve: {nxt}/{len(reqs)} submitted, {len(inflight)} in flight")
            time.sleep(0.0002)
        return lat, time.perf_counter() - t0, iters

    # warm-up and saturated throughput (everything submitted at once)
    serve(draw(min(2 * len(pool), args.requests)), None)
    nsat = min(args.requests, 4 * len(pool))
    lat_sat, mk, it_sat = serve(draw(nsat), None)
    sat = nsat / mk
    log(f"[bench] serve: saturated {sat:.1f} solves/s")
    rates = {}
    for f in (0.5, 0.8, 0.95):
        lam = f * sat
        gaps = rng.exponential(1.0 / lam, size=args.requests)
        arr = np.cumsum(gaps) - gaps[0]
        lat, mk, its = serve(draw(args.requests), arr.tolist())
        rates[str(f)] = {"offered": round(lam, 2), "solves_per_s": round(args.requests / mk, 2),
                         "p50_ms": _pct(lat, 50), "p99_ms": _pct(lat, 99),
                         "mean_ms": round(1e3 * float(np.mean(lat)), 3),
                         "iters_mean": round(float(np.mean(its)), 2)}
        log(f"[bench] serve: rate {f}: {rates[str(f)]}")
    L.mdp_server_destroy(srv)

    # alone: each pool system solved once by itself (service time without queueing)
    alone = []
    for p in pool:
        x = torch.zeros(p["n"], dtype=torch.float64, device="cuda:0")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        L.mdp_solve(p["h"]["mixed"], p["b"][0], x, stream)
        alone.append(time.perf_counter() - t0)

    cpu = None
    if not args.no_cpu_baseline:
        cpu, _ = cpu_full_solves(args, [(p["sc"], p["fs"][0]) for p in pool], "first right-hand side")
    _destroy_pool(pool)
    line = {
        "metric": "served solves/s to 1e-8 rel residual with p50/p99 latency (mixed precision)",
        "value": round(sat, 2),
        "unit": "solves/s",
        "n_gpus": 1, "steps": nsat, "warmup": min(2 * len(pool), args.requests),
        "ms_per_step": round(1e3 / sat, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 preconditioner / f64 outer", "data": "synthetic",
        "config": {"workload": f"serving-pool-{len(pool)}-2d64-512-3d40-160", "slots": args.slots,
                   "grouping": bool(args.serve_grouping),
                   "budget_gb": args.budget_gb, "requests_per_rate": args.requests,
                   "unknowns_range": [min(p["n"] for p in pool), max(p["n"] for p in pool)]},
        "saturated": {"solves_per_s": round(sat, 2), "p50_ms": _pct(lat_sat, 50), "p99_ms": _pct(lat_sat, 99),
                      "iters_mean": round(float(np.mean(it_sat)), 2)},
        "poisson": rates,
        "alone_service_ms": {"p50": _pct(alone, 50), "p99": _pct(alone, 99),
                             "sequential_solves_per_s": round(len(alone) / sum(alone), 2)},
        "setup_s": {"assembly": round(t_asm, 2), "host_setup_and_upload": round(t_set, 2)},
        "cpu_baseline": cpu,
    }
    return line


def cpu_full_solves(args, items, which):
    """The FP64 oracle on this host, one core: full solves of the listed
    (scenario, source) items in order, each set up untimed, until
    ``cpu_seconds`` of solve time has been spent.  Returns the baseline
    object (solves/s) and the (name, solution, iterations) of each solve."""
    from oracle import assembly as oa, solve as osv
    from threadpoolctl import threadpool_limits

    spent, done, names, sols = 0.0, 0, [], []
    for sc, f in items:
        A, b, part = oa.assemble(sc.with_source(f))
        M = osv.setup(A, part)
        with threadpool_limits(limits=1):
            t0 = time.perf_counter()
            res, _, _ = osv.solve(A, b, part, osv.SolveOptions(), M=M)
            spent += time.perf_counter() - t0
        done += 1
        names.append(f"{sc.name}({A.shape[0]})")
        sols.append((sc.name, res.x, res.iters))
        log(f"[bench] cpu oracle: {sc.name} solved in {res.iters} iterations; {spent:.1f}s so far")
        if spent >= args.cpu_seconds:
            break
    shown = ", ".join(names[:4]) + (f", ... ({done - 4} more)" if done > 4 else "")
    return {"value": round(done / spent, 4), "unit": "solves/s", "cores": 1, "kind": "oracle",
            "sample": f"FP64 oracle, full solves of the first {done} systems ({which}): "
                      f"{shown}; {spent:.1f}s of solve time, setup not timed",
            "host_cpu_count": os.cpu_count()}, sols


if __name__ == "__main__":
    main()
