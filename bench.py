"""Benchmark: supernodal LL^T factorization + refined solve on one MI355X.

Workload: 3-D 7-point Laplacian on a 100^3 grid plus a diagonal shift 1e-3
(N = 1e6), one right-hand side uniform in [-1, 1].  A step is one pass of the
whole hot path with inputs resident in HBM: assembly, the persistent
factorization kernel (diagonal factorization, panel triangular solves,
sparse-GEMM updates from the device ready queue), triangular sweeps and FP64
residual/refinement to a componentwise backward error of 1e-14.  The FP64
mode is the headline; the FP32-factor + FP64-refinement mode is timed the
same way and reported as a speedup over it (factor + solve time).

value = algorithmic factorization flops (sum of squared exact column counts)
        / FP64 factorization time (HIP events around the factorize call).

Order of the run: the FP64 headline leg, then the oracle's CPU baseline,
then the other legs (FP32 + refinement, split-BF16 + refinement, L D L^T in
FP64 and FP32 + refinement, the deterministic accumulation mode in FP64,
the 512-system batch, then L U with static pivoting on the 80^3
convection-diffusion stencil with 4 right-hand sides in the three precision
modes, then L D L^T on the 40^3 clamped elasticity mesh with 8 right-hand
sides in FP64 and FP32 + refinement) while the wall-clock budget (--budget-s, counted from
the start of the process) leaves room for them; a leg that does not fit is
listed under "skipped".  Progress lines with the elapsed time go to stderr;
the one JSON line goes to stdout at the end.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

T_START = time.perf_counter()
ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6   # MI355X dense FP64 matrix peak


def log(msg):
    print("[%7.1f s] %s" % (time.perf_counter() - T_START, msg), file=sys.stderr, flush=True)


def measured_traffic():
    """HBM bytes per factorization from the committed rocprofv3 counter summary,
    or None when the factorization source changed since it was taken."""
    import hashlib
    try:
        kv = {}
        with open(os.path.join(ROOT, "profiles", "sched_kernel_traffic.txt")) as f:
            for ln in f:
                if "=" in ln and not ln.startswith("#"):
                    k, v = ln.strip().split("=", 1)
                    kv[k] = v
        with open(os.path.join(ROOT, "paper_1405_2636_amd", "csrc", "factor.hip"), "rb") as f:
            sha = hashlib.sha256(f.read()).hexdigest()[:16]
        if sha != kv["factor_hip_sha256_16"]:
            return None
        return (float(kv["fetch_kib"]) * float(kv["fetch_scale"]) + float(kv["write_kib"]) * float(kv["write_scale"])) * 1024.0
    except (OSError, KeyError, ValueError):
        return None


def host_cpu():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_count": os.cpu_count(), "cpu_model": model}


def cpu_baseline(p, budget_flops: float = 2.0e10):
    """The oracle (plain serial C, one core) on a bounded sample of the same
    workload: its own analysis of the full matrix, then the factorization of
    the largest subtree of the block elimination tree whose algorithmic flops
    fit the budget (leaves up to a separator block of that subtree: small and
    large blocks alike).  Only the factorization is timed; the subtree's
    assembly is timed apart and reported, not counted."""
    import numpy as np

    from oracle import oracle as O
    t0 = time.perf_counter()
    sym = O.analyze(p.n, p.colptr, p.rowind)
    t_an = time.perf_counter() - t0
    cc = sym.colcount.astype(np.float64)
    csum = np.concatenate([[0.0], np.cumsum(cc * cc)])
    first = O.subtree_first(sym)
    fcol, lcol = sym.fcol.astype(np.int64), sym.lcol.astype(np.int64)
    sub_flops = csum[lcol + 1] - csum[fcol[first]]
    fits = np.where(sub_flops <= budget_flops)[0]
    root = int(fits[np.argmax(sub_flops[fits])]) if len(fits) else 0
    k0 = int(first[root])
    fl = float(sub_flops[root])
    widths = lcol[k0:root + 1] - fcol[k0:root + 1] + 1
    _, t_asm, t_fac = O.factor_subtree(sym, p.colptr, p.rowind, p.values, root)
    return {"value": fl / t_fac / 1e9, "unit": "GFLOP/s", "cores": 1, "kind": "oracle",
            "sample": "oracle factorization of one subtree of the block elimination tree of the same matrix: "
                      "column blocks %d..%d of %d (widths 1..%d, %d columns), %.3e of %.3e algorithmic flops "
                      "in %.1f s; its assembly (%.1f s) and the oracle's analysis (%.1f s) not counted"
                      % (k0, root, len(lcol), int(widths.max()), int(widths.sum()), fl, sym.stats["flops_alg"],
                         t_fac, t_asm, t_an),
            "host": host_cpu()}


def copy_probe():
    """Three copies of 64 Mi doubles (512 MiB read + 512 MiB written each): the
    reference dispatch that scales rocprofv3's FETCH_SIZE / WRITE_SIZE."""
    import torch
    n = 64 * 1024 * 1024
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print("copied 3 x %d bytes" % (n * 8), flush=True)


def run_leg(torch, np, Solver, p, vals, b0, precision, steps, warmup, method="llt", adjoint=True,
            deterministic=False):
    """Warm-up, then `steps` timed passes of factorize + refined solve in one
    precision mode (and method: L L^T, L D L^T or L U).  Times are HIP events
    on the torch stream the library is called on; the kernel time is the
    library's own event pair around the scheduler kernel, on the same stream."""
    name = (precision if method == "llt" else precision + " " + method) + (" det" if deterministic else "")
    t0 = time.perf_counter()
    s = Solver(p.n, p.colptr, p.rowind, precision=precision, method=method, deterministic=deterministic)
    t_an = time.perf_counter() - t0
    info = s.info()
    log("[%s] analyze %.1f s: ncblk %d nnz(L) %d flops %.3e tasks %d"
        % (name, t_an, info["ncblk"], info["nnz_l"], info["flops_alg"], info["ntasks"]))
    stream = torch.cuda.current_stream()
    nrhs = 1 if b0.dim() == 1 else b0.shape[0]
    b = torch.empty_like(b0)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    for i in range(warmup):
        s.factorize(vals)
        b.copy_(b0)
        s.solve(b)
    torch.cuda.synchronize()
    log("[%s] %d warm-up steps done" % (name, warmup))
    fac_ms, sol_ms, ker_ms, oms, its = [], [], [], [], []
    for i in range(steps):
        ev[0].record(stream)
        s.factorize(vals)
        ev[1].record(stream)
        b.copy_(b0)
        _, si = s.solve(b)
        ev[2].record(stream)
        torch.cuda.synchronize()
        fac_ms.append(ev[0].elapsed_time(ev[1]))
        sol_ms.append(ev[1].elapsed_time(ev[2]))
        ker_ms.append(s.info()["factor_kernel_ms"])
        oms.append(si["omega"])
        its.append(si["ir_iters"])
    log("[%s] %d steps: factorize %.2f ms (kernel %.2f) solve %.2f ms omega %.2e ir %d"
        % (name, steps, float(np.median(fac_ms)), float(np.mean(ker_ms)), float(np.median(sol_ms)), max(oms),
           max(its)))
    out = {"factor_ms": float(np.median(fac_ms)), "solve_ms": float(np.median(sol_ms)),
           "kernel_ms": float(np.mean(ker_ms)), "omega": float(max(oms)), "ir_iters": int(max(its)),
           "flops": info["flops_alg"], "nnz_l": info["nnz_l"], "nrhs": nrhs, "analyze_s": t_an}
    if adjoint:
        # adjoint of the solve (backward pass of solve_autograd): db = A^{-1} xbar
        # with the same factor, then the value gradient on the pattern
        xbar = torch.ones_like(b0)
        adj_ms = []
        for i in range(3):
            ev[0].record(stream)
            db = xbar.clone()
            s.solve(db)
            s.values_grad(b, db)
            ev[1].record(stream)
            torch.cuda.synchronize()
            adj_ms.append(ev[0].elapsed_time(ev[1]))
        out["adjoint_ms"] = float(np.median(adj_ms))
    out["logdet"] = s.info()["logdet"]
    del s
    torch.cuda.synchronize()
    return out


def run_batch(torch, np, Solver, steps):
    """512 independent weighted 2-D grid Laplacians (sides 16..96, log-normal
    edge weights) factorized and solved together: one graph-replayed
    factorization launch, work decomposition chosen by the autotuner.  Both
    precision modes; times are medians over ``steps`` factorize + solve."""
    from gen import grid_batch
    ps = grid_batch(512)
    systems = [(p.n, p.colptr, p.rowind) for p in ps]
    vals = torch.tensor(np.concatenate([p.values for p in ps]), device="cuda")
    b0 = torch.tensor(np.concatenate([p.b[:, 0] for p in ps]), device="cuda")
    out = {"systems": len(ps), "n": int(sum(p.n for p in ps)), "nnz_a": int(sum(p.nnz for p in ps))}
    for prec in ("fp64", "fp32_ir"):
        t0 = time.perf_counter()
        s = Solver.batch(systems, precision=prec, graph=True, tune=True)
        t_an = time.perf_counter() - t0
        s.factorize(vals)   # tuning run
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        stream = torch.cuda.current_stream()
        fac, sol, om, its = [], [], [], []
        for i in range(steps):
            ev[0].record(stream)
            s.factorize(vals)
            ev[1].record(stream)
            b = b0.clone()
            _, si = s.solve(b)
            ev[2].record(stream)
            torch.cuda.synchronize()
            fac.append(ev[0].elapsed_time(ev[1]))
            sol.append(ev[1].elapsed_time(ev[2]))
            om.append(si["omega"])
            its.append(si["ir_iters"])
        inf = s.info()
        fl = inf["flops_alg"]
        out[prec] = {"analyze_s": t_an, "factor_ms": float(np.median(fac)), "solve_ms": float(np.median(sol)),
                     "factor_gflops": fl / (float(np.median(fac)) * 1e-3) / 1e9, "omega": float(max(om)),
                     "ir_iters": int(max(its)), "flops_alg": fl,
                     "tuned": {"tile": [inf["tile_rows"], inf["tile_cols"]], "hp_policy": inf["hp_policy"]}}
        log("[batch %s] factorize %.2f ms solve %.2f ms omega %.2e ir %d tile %s"
            % (prec, out[prec]["factor_ms"], out[prec]["solve_ms"], out[prec]["omega"], out[prec]["ir_iters"],
               out[prec]["tuned"]["tile"]))
        del s
    out["fp32_ir"]["speedup_vs_fp64"] = ((out["fp64"]["factor_ms"] + out["fp64"]["solve_ms"])
                                        / (out["fp32_ir"]["factor_ms"] + out["fp32_ir"]["solve_ms"]))
    return out


def run_update_bench(torch, np, ks, ms, precisions, streams, calls, gapped_modes, methods):
    """The update-kernel study of Section V-B (Fig. 2): `calls` updates
    C -= A B^T of a synthetic panel (A: m x k rows of inner dimension k, B
    its first k rows) into a dense m-row target or a gapped 2m-row one, per
    launch mode (1-3 streams round-robin, or 0 = all calls in one grid).
    GFLOP/s counts 2 k (m k - k (k - 1) / 2) flops per call (the target's
    diagonal block is updated on its lower triangle only)."""
    from gen import update_panels
    from paper_1405_2636_amd.spx import update_bench
    rows = []
    for prec in precisions:
        dt = torch.float64 if prec == "fp64" else torch.float32
        for method in methods:
            for gapped in gapped_modes:
                for k in ks:
                    for m in ms:
                        if m < k:
                            continue
                        P, rmap, ldc = update_panels(k, m, k, gapped, seed=m + k)
                        buf = torch.tensor(np.concatenate([P, np.zeros(ldc * k)]), dtype=dt, device="cuda")
                        rm = torch.tensor(rmap, device="cuda")
                        flops = 2.0 * k * (m * k - k * (k - 1) / 2)
                        row = {"precision": prec, "method": method, "gapped": gapped, "k": k, "m": m, "ldc": ldc}
                        for ns in streams:
                            update_bench(buf, rm, k, m, k, ldc, prec, method, 0, 2, ns)   # warm-up
                            t = update_bench(buf, rm, k, m, k, ldc, prec, method, 0, calls, ns)
                            row["gflops_%s" % ("grid" if ns == 0 else "s%d" % ns)] = calls * flops / (t * 1e-3) / 1e9
                        rows.append(row)
                        log("[update %s %s %s] k %d m %d: %s" % (
                            prec, method, "gapped" if gapped else "dense", k, m,
                            " ".join("%s %.0f" % (key[7:], v) for key, v in row.items() if key.startswith("gflops_"))))
                        del buf, rm
    return {"calls": calls, "rows": rows}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", type=int, default=2)
    ap.add_argument("--budget-s", type=float, default=420.0,
                    help="wall-clock seconds (from the start of the process) within which optional legs start")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the 512-system batch leg")
    ap.add_argument("--headline-only", action="store_true", help="only the FP64 leg (and the CPU baseline)")
    ap.add_argument("--batch-only", action="store_true",
                    help="only the 512-system batch leg (its JSON object on one line; for profiling)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run three plain device copies of 512 MiB (scale for the HBM byte counters)")
    ap.add_argument("--update-bench", action="store_true",
                    help="only the update-kernel study (Fig. 2 recipe): GFLOP/s per inner size k, height m, target "
                         "kind and launch mode, as one JSON line")
    ap.add_argument("--update-k", default="64,128,256")
    ap.add_argument("--update-m", default="256,512,1024,2048,4096,8192,16384")
    ap.add_argument("--update-precision", default="fp64,fp32_ir")
    ap.add_argument("--update-method", default="llt")
    ap.add_argument("--update-streams", default="1,2,3,0", help="streams per sweep point (0: all calls in one grid)")
    ap.add_argument("--update-target", default="dense,gapped")
    ap.add_argument("--update-calls", type=int, default=100)
    args = ap.parse_args()
    if args.copy_probe:
        copy_probe()
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only (no multi-GPU path: the factorization and its queue live on one device)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from gen import make_config
    from paper_1405_2636_amd import Solver

    log("imports done")
    if args.update_bench:
        ints = lambda t: [int(x) for x in t.split(",") if x]
        res = run_update_bench(torch, np, ints(args.update_k), ints(args.update_m), args.update_precision.split(","),
                               ints(args.update_streams), args.update_calls,
                               [t == "gapped" for t in args.update_target.split(",")], args.update_method.split(","))
        print(json.dumps({"update_bench": res}), flush=True)
        return
    if args.batch_only:
        print(json.dumps({"batch": run_batch(torch, np, Solver, args.steps)}), flush=True)
        return
    p = make_config(args.config)
    log("workload %s generated: n %d nnz %d" % (p.name, p.n, p.nnz))
    vals = torch.tensor(p.values, device="cuda")
    b0 = torch.tensor(np.ascontiguousarray(p.b[:, 0]), device="cuda")

    # headline: FP64 L L^T
    t_leg = time.perf_counter()
    r64 = run_leg(torch, np, Solver, p, vals, b0, "fp64", args.steps, args.warmup)
    leg_s = time.perf_counter() - t_leg
    flops = r64["flops"]
    achieved = flops / (r64["kernel_ms"] * 1e-3) / 1e12
    out = {
        "metric": "factorize GFLOP/s + solve ms at backward err 1e-14",
        "value": flops / (r64["factor_ms"] * 1e-3) / 1e9,
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r64["factor_ms"] + r64["solve_ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": p.name, "n": p.n, "nnz_a": int(p.nnz), "nnz_l": int(r64["nnz_l"]),
                   "flops_alg": flops, "nrhs": 1, "precision": "fp64"},
        "factor_ms": r64["factor_ms"],
        "solve_ms": r64["solve_ms"],
        "omega": r64["omega"],
        "ir_iters": r64["ir_iters"],
        "adjoint_ms": r64.get("adjoint_ms"),
        "logdet": r64["logdet"],
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP64_TFLOPS, "traffic": measured_traffic(),
                     "kernel": "sched_kernel<double, false>", "kernel_ms": r64["kernel_ms"]},
        "skipped": [],
    }
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(p)
        log("cpu baseline: %.2f GFLOP/s" % out["cpu_baseline"]["value"])

    def fits(est_s):
        return time.perf_counter() - T_START + est_s <= args.budget_s

    def speedup(r):
        return (r64["factor_ms"] + r64["solve_ms"]) / (r["factor_ms"] + r["solve_ms"])

    legs = [] if args.headline_only else (["fp32_ir", "bf16x3_ir", "ldlt_fp64", "ldlt_fp32_ir", "deterministic_fp64"]
                                          + ([] if args.no_batch else ["batch"])
                                          + ["lu_fp64", "lu_fp32_ir", "lu_bf16x3_ir", "c5_ldlt_fp64", "c5_ldlt_fp32_ir"])
    c3, c5 = {}, {}
    for leg in legs:
        est = 1.3 * leg_s if leg != "batch" else 90.0
        if not fits(est):
            out["skipped"].append(leg)
            log("[%s] skipped: %.0f s estimated, budget %.0f s" % (leg, est, args.budget_s))
            continue
        if leg in ("fp32_ir", "bf16x3_ir"):
            r = run_leg(torch, np, Solver, p, vals, b0, leg, args.steps, args.warmup, adjoint=False)
            out[leg] = {"factor_ms": r["factor_ms"], "solve_ms": r["solve_ms"],
                        "factor_gflops": flops / (r["factor_ms"] * 1e-3) / 1e9, "omega": r["omega"],
                        "ir_iters": r["ir_iters"], "kernel_ms": r["kernel_ms"], "speedup_vs_fp64": speedup(r)}
        elif leg in ("ldlt_fp64", "ldlt_fp32_ir", "deterministic_fp64"):
            prec = "fp32_ir" if leg == "ldlt_fp32_ir" else "fp64"
            r = run_leg(torch, np, Solver, p, vals, b0, prec, args.steps, args.warmup,
                        method="llt" if leg == "deterministic_fp64" else "ldlt", adjoint=False,
                        deterministic=leg == "deterministic_fp64")
            out[leg] = {"factor_ms": r["factor_ms"], "solve_ms": r["solve_ms"],
                        "factor_gflops": flops / (r["factor_ms"] * 1e-3) / 1e9, "omega": r["omega"],
                        "ir_iters": r["ir_iters"], "kernel_ms": r["kernel_ms"]}
            if prec == "fp64":
                out[leg]["kernel_frac_of_fp64_peak"] = flops / (r["kernel_ms"] * 1e-3) / 1e12 / PEAK_FP64_TFLOPS
            if leg == "ldlt_fp32_ir" and "ldlt_fp64" in out:
                out[leg]["speedup_vs_fp64"] = ((out["ldlt_fp64"]["factor_ms"] + out["ldlt_fp64"]["solve_ms"])
                                               / (r["factor_ms"] + r["solve_ms"]))
        elif leg == "batch":
            out["batch"] = run_batch(torch, np, Solver, args.steps)
        elif leg.startswith("lu_"):
            # L U with static pivoting on the 80^3 convection-diffusion stencil, 4 RHS
            if not c3:
                q = make_config(3)
                c3.update(p=q, vals=torch.tensor(q.values, device="cuda"),
                          b0=torch.tensor(np.ascontiguousarray(q.b.T), device="cuda"))
                out["convdiff80_lu"] = {"workload": q.name, "n": q.n, "nnz_a": int(q.nnz), "nrhs": 4}
            prec = leg[3:]
            r = run_leg(torch, np, Solver, c3["p"], c3["vals"], c3["b0"], prec, args.steps, args.warmup, method="lu",
                        adjoint=False)
            d = out["convdiff80_lu"]
            d["flops_alg"] = r["flops"]
            d[prec] = {"factor_ms": r["factor_ms"], "solve_ms": r["solve_ms"],
                       "factor_gflops": r["flops"] / (r["factor_ms"] * 1e-3) / 1e9, "omega": r["omega"],
                       "ir_iters": r["ir_iters"], "kernel_ms": r["kernel_ms"]}
            if prec == "fp64":
                d[prec]["kernel_frac_of_fp64_peak"] = r["flops"] / (r["kernel_ms"] * 1e-3) / 1e12 / PEAK_FP64_TFLOPS
            elif "fp64" in d:
                d[prec]["speedup_vs_fp64"] = ((d["fp64"]["factor_ms"] + d["fp64"]["solve_ms"])
                                              / (r["factor_ms"] + r["solve_ms"]))
        elif leg.startswith("c5_"):
            # L D L^T on the 40^3 clamped elasticity mesh, 8 RHS
            if not c5:
                q = make_config(5)
                c5.update(p=q, vals=torch.tensor(q.values, device="cuda"),
                          b0=torch.tensor(np.ascontiguousarray(q.b.T), device="cuda"))
                out["elasticity40_ldlt"] = {"workload": q.name, "n": q.n, "nnz_a": int(q.nnz), "nrhs": 8}
            prec = leg[len("c5_ldlt_"):]
            r = run_leg(torch, np, Solver, c5["p"], c5["vals"], c5["b0"], prec, args.steps, args.warmup,
                        method="ldlt", adjoint=False)
            d = out["elasticity40_ldlt"]
            d["flops_alg"] = r["flops"]
            d[prec] = {"factor_ms": r["factor_ms"], "solve_ms": r["solve_ms"],
                       "factor_gflops": r["flops"] / (r["factor_ms"] * 1e-3) / 1e9, "omega": r["omega"],
                       "ir_iters": r["ir_iters"], "kernel_ms": r["kernel_ms"]}
            if prec == "fp64":
                d[prec]["kernel_frac_of_fp64_peak"] = r["flops"] / (r["kernel_ms"] * 1e-3) / 1e12 / PEAK_FP64_TFLOPS
            elif "fp64" in d:
                d[prec]["speedup_vs_fp64"] = ((d["fp64"]["factor_ms"] + d["fp64"]["solve_ms"])
                                              / (r["factor_ms"] + r["solve_ms"]))
    log("done")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
