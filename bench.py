#!/usr/bin/env python3
"""Benchmark of the ASSS two-level solve on one MI355X.

One step = one complete solve of A x = b to true relative residual 1e-8
(FGMRES outer iteration, P^-1 through the SMW form around the inner mrs,
back-transform and true-residual check), with A, b and all preconditioner
data resident in HBM when the timed region starts.

Workload (default, the precision workload): 3D convection-diffusion, 7-point
first-order upwind on a 192^3 grid (n = 7,077,888, nnz = 49,324,032), Peclet
1000, wind (1, 0.5, 0.25), S on the pattern of Abar, k = 16 skew-Lanczos
vectors, b = A x*, x* ~ U(-1,1) (seeded draw of that workload).  The plain
FP64 solve is the headline value; the FP32-inner / FP64-outer solve of the
same system is reported beside it, each with the roofline of the inner step.

Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "time-to-1e-8 rel. residual + HBM GB/s; FP32-inner vs FP64 plain, 1 GPU"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def mrs_bytes_per_row(nh_per_row: float, k: int, v: int, vq: int = 0) -> float:
    """Algorithmic bytes of one inner mrs step per row: the strict upper
    triangle of J_tilde once ((v + 4) per entry), its row pointer (4), the k
    deflation vectors once (k vq, vq = v unless the basis is stored as FP32
    values), and ten vector streams of v bytes (read q, u, q_old, p_old2, x and
    a second q gather; write q', p, x; re-zero u)."""
    return nh_per_row * (v + 4) + 4 + k * (vq or v) + 10 * v


def workload_key(m: int, peclet: float, k: int, order: str) -> str:
    """Name of the committed profile summaries of one workload and inner order."""
    suffix = {"x-line tiles 4x4": "_linetiles4x4", "library grid order": "_gridorder"}.get(order, "")
    return f"convdiff3d_{m}_Pe{peclet:g}_k{k}{suffix}"


KERNEL_SOURCES = ("kernels.hip", "mrs_common.hpp", "kernels.hpp")


def kernel_sha() -> str:
    """sha256 of the inner step's source: the kernel file, the recurrence it
    shares with the other inner kernels, and their data structures."""
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2009_06954_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(precision: str, key: str, deflation: str = "explicit"):
    """HBM bytes per full inner step from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE summary of this workload (profiles/k_mrs_iter_<key>_traffic.json),
    if it was taken on the kernel source as it is now and for this form of the
    deflation basis; None otherwise."""
    name = key + ("_fp32basis" if deflation == "explicit_fp32_basis" else "")
    path = os.path.join(ROOT, "profiles", f"k_mrs_iter_{name}_traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f)
        sha = kernel_sha()
    except OSError:
        return None
    if rec.get("kernel_src_sha256") != sha or precision not in rec.get("kernels", {}):
        return None  # counters predate the current kernel
    return rec["kernels"][precision]["hbm_bytes"]


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            return next(l.split(":", 1)[1].strip() for l in f if l.startswith("model name"))
    except (OSError, StopIteration):
        return "unknown"


def oracle_solve_time(m: int, peclet: float, cfg: int, k: int, tol: float, inner_tol: float,
                      restart: int, repeats: int = 3):
    """The oracle (unchanged) on an m^3 instance of the workload family: setup
    once (not timed), then the best of `repeats` solves."""
    import oracle as O
    import workloads as W

    w = W.convdiff3d(m=m, peclet=peclet, cfg=cfg)
    t0 = time.perf_counter()
    st = O.setup(w.A, O.SetupOptions(k=k, s_pattern="abar"))
    setup_s = time.perf_counter() - t0
    best, info, x = float("inf"), None, None
    for _ in range(repeats):
        t0 = time.perf_counter()
        x, info = O.solve(st, w.b, O.SolveOptions(tol=tol, inner_tol=inner_tol, restart_m=restart))
        best = min(best, time.perf_counter() - t0)
    return {"m": m, "n": int(w.A.shape[0]), "solve_s": round(best, 4), "setup_s": round(setup_s, 2),
            "outer_its": int(info["outer_its"]), "inner_its": int(info["inner_its_total"]),
            "relres": float(info["relres_true"]), "_x": x}


def unit_cost(run: dict) -> float:
    """Oracle seconds per (row x inner step): the inner mrs dominates the
    solve, and its work per step is proportional to n."""
    return run["solve_s"] / (run["n"] * max(1, run["inner_its"]))


def cpu_baseline(sizes, peclet: float, cfg: int, k: int, tol: float, n_full: int, inner_full: int,
                 inner_tol: float, restart: int):
    """The oracle timed at two sizes of the same workload family on the host's
    cores (NumPy/SciPy as installed: sparse products on one thread, dense
    products on the BLAS thread pool).  The cost per (row x inner step) of the
    smaller size predicts the larger one (the check); the larger one's
    extrapolates to the full problem with the GPU solve's inner step count."""
    from threadpoolctl import threadpool_info

    runs = [oracle_solve_time(m, peclet, cfg, k, tol, inner_tol, restart) for m in sizes]
    xs = {r["m"]: r.pop("_x") for r in runs}
    small, large = runs[0], runs[-1]
    predicted = unit_cost(small) * large["n"] * large["inner_its"]
    pools = [{"api": d.get("internal_api"), "threads": d.get("num_threads")} for d in threadpool_info()]
    threads = max([p["threads"] or 1 for p in pools] + [1])
    value = unit_cost(large) * n_full * inner_full
    return {
        "value": round(value, 2), "unit": "s", "cores": threads, "kind": "oracle",
        "cpu_model": cpu_model(), "host_cpu_count": os.cpu_count(), "threadpools": pools,
        "runs": runs,
        "fit": {"model": "t = c * n * inner_its", "c_s": unit_cost(large),
                "check": {"predicted_large_from_small_s": round(predicted, 4),
                          "measured_large_s": large["solve_s"],
                          "ratio": round(predicted / large["solve_s"], 3)}},
        "sample": (f"oracle solves of convdiff3d m^3 Pe{peclet:g} for m in {list(sizes)} "
                   f"(best of 3, setup not timed); extrapolated to n={n_full} with the GPU's "
                   f"{inner_full} inner steps from the larger sample's cost per row and step"),
        "_x": xs,
    }


def oracle_parity(asss, torch, np, W, m, peclet, cfg, k, tol, inner_tol, restart, x_oracle):
    """The library on the same smaller instance of the workload family, in the
    benchmark's launch configuration (grid order, offset slots, FGMRES(restart),
    the same inner tolerance), FP64 and FP32 inner: relative error of each
    solution against the oracle's solution of the same system at the same
    tolerance, and against the oracle's x solved further (both sides at 1e-8
    differ from A^-1 b by up to kappa * tol)."""
    w = W.convdiff3d(m=m, peclet=peclet, cfg=cfg)
    h = asss.setup(w.A, k=k, s_pattern="abar", reorder="grid")
    b = torch.from_numpy(w.b).cuda()
    out = {"workload": f"convdiff3d_{m}^3_Pe{peclet:g}", "n": int(w.A.shape[0]), "tol": tol}
    xn = float(np.linalg.norm(x_oracle))
    for mixed in (False, True):
        x, inf = h.solve(b, tol=tol, inner_fp32=mixed, restart_m=restart, inner_tol=inner_tol)
        xg = x.cpu().numpy()
        key = "mixed" if mixed else "fp64"
        out[key + "_rel_err_vs_oracle"] = float(np.linalg.norm(xg - x_oracle) / xn)
        out[key + "_rel_err_vs_xstar"] = float(np.linalg.norm(xg - w.x_star) / np.linalg.norm(w.x_star))
        out[key + "_outer_its"] = inf["outer_its"]
    out["oracle_rel_err_vs_xstar"] = float(np.linalg.norm(x_oracle - w.x_star) / np.linalg.norm(w.x_star))
    h.close()
    return out


def batched(args, asss, torch, np, W):
    """64 uneven systems x 4 right-hand sides: the lockstep batch engine (one
    persistent work-queue launch per inner step for all systems, graph-replayed
    inner chunks, one host round trip per outer step) against the per-system
    workers and against solving the columns one at a time (same handles)."""
    ws = W.batched_implicit_euler(nsys=args.nsys, nrhs=4, cfg=3)
    log(f"batched: {len(ws)} systems, n from {min(w.A.shape[0] for w in ws)} to "
        f"{max(w.A.shape[0] for w in ws)}, total {sum(w.A.shape[0] for w in ws)}")
    t0 = time.perf_counter()
    hs = [asss.setup(w.A, k=8, s_pattern="tridiag", inner_fp32=not args.no_mixed, autotune=args.autotune)
          for w in ws]
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    log(f"setup {setup_s:.1f} s")
    Bs = [torch.from_numpy(np.ascontiguousarray(w.b.T)).cuda().t() for w in ws]
    kw = dict(tol=args.tol, inner_fp32=not args.no_mixed, restart_m=64, inner_tol=1e-2)
    nrhs = sum(B.shape[1] for B in Bs)

    def timed(mode, reps):
        asss.solve_batched(hs, Bs, batch_engine=mode, **kw)  # warm-up (the engine builds its batch data)
        torch.cuda.synchronize()
        best, infos = float("inf"), None
        for _ in range(reps):
            t0 = time.perf_counter()
            Xs, infos = asss.solve_batched(hs, Bs, batch_engine=mode, **kw)
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - t0)
        worst = max(i["relres_true"] for row in infos for i in row)
        conv = all(i["converged"] for row in infos for i in row)
        outer = max(i["outer_its"] for row in infos for i in row)
        log(f"{mode}: {best:.4f} s, worst relres {worst:.2e}, all converged {conv}, max outer {outer}")
        return best, worst, conv, Xs

    t_eng, worst_e, conv_e, Xe = timed("lockstep", max(1, args.steps))
    if args.engine_only:
        print(json.dumps({"engine_s": round(t_eng, 4), "worst_relres": worst_e, "converged": conv_e}), flush=True)
        return
    t_wrk, worst_w, conv_w, Xw = timed("workers", 1)
    diff = max(float(torch.linalg.norm(a - b) / torch.linalg.norm(b)) for a, b in zip(Xe, Xw))
    for h, B in zip(hs, Bs):  # warm-up of the single-column workspace
        h.solve(B[:, 0].contiguous(), **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for h, B in zip(hs, Bs):
        for j in range(B.shape[1]):
            h.solve(B[:, j].contiguous(), **kw)
    torch.cuda.synchronize()
    t_cols = time.perf_counter() - t0
    for h in hs:
        h.close()
    res = {"metric": "batched solve throughput (right-hand sides to 1e-8 per second)",
           "value": round(nrhs / t_eng, 3), "unit": "rhs/s", "n_gpus": 1, "higher_is_better": True,
           "dtype": "f32 inner / f64 outer" if not args.no_mixed else "f64", "data": "synthetic",
           "config": {"workload": f"implicit_euler_batched_{len(ws)}x4", "systems": len(ws),
                      "total_n": int(sum(w.A.shape[0] for w in ws)), "rhs": nrhs, "k": 8, "s_pattern": "tridiag",
                      "tol": args.tol, "outer": "fgmres(64)", "inner_tol": 1e-2, "engine": "lockstep"},
           "engine_s": round(t_eng, 4), "workers_s": round(t_wrk, 4), "column_by_column_s": round(t_cols, 3),
           "speedup_engine_vs_workers": round(t_wrk / t_eng, 3),
           "speedup_engine_vs_columns": round(t_cols / t_eng, 3),
           "worst_relres_engine": worst_e, "worst_relres_workers": worst_w,
           "all_converged": bool(conv_e and conv_w), "max_rel_diff_engine_vs_workers": diff,
           "setup_s": round(setup_s, 1), "autotune": bool(args.autotune)}
    print(json.dumps(res), flush=True)


def grad_bench(args, asss, torch, np, W):
    """Forward + backward of L = ||A^-1 b - x_t||^2 at n = 1e6 (A's values and b
    require gradients); the preconditioner is built once from A."""
    from paper_2009_06954_amd.autograd import LinearSolve
    w = W.implicit_euler_grid(m=1000, h=0.1, cfg=4)
    rng = np.random.default_rng(4)
    xt = torch.from_numpy(rng.standard_normal(w.A.shape[0])).cuda()
    t0 = time.perf_counter()
    op = LinearSolve(w.A, k=8, s_pattern="tridiag", tol=1e-10)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    times = []
    for it in range(args.warmup + args.steps):
        vals = torch.tensor(op.values0, requires_grad=True)
        b = torch.from_numpy(w.b.copy()).cuda().requires_grad_(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x = op(vals, b)
        L = ((x - xt) ** 2).sum()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        L.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        if it >= args.warmup:
            times.append((t1 - t0, t2 - t1))
    fwd = sum(t[0] for t in times) / len(times)
    bwd = sum(t[1] for t in times) / len(times)
    res = {"metric": "forward + backward time of a differentiable solve (s)", "value": round(fwd + bwd, 4),
           "unit": "s", "n_gpus": 1, "higher_is_better": False, "dtype": "f64", "data": "synthetic",
           "steps": args.steps, "warmup": args.warmup,
           "config": {"workload": "implicit_euler_1000x1000_h0.1", "n": int(w.A.shape[0]), "nnz": int(w.A.nnz),
                      "k": 8, "s_pattern": "tridiag", "tol": 1e-10, "outer": "fgmres(64)"},
           "forward_s": round(fwd, 4), "backward_s": round(bwd, 4), "setup_s": round(setup_s, 2),
           "forward_info": {k: op.last_info[k] for k in ("outer_its", "inner_its_total", "relres_true")},
           "grad_norm_values": float(vals.grad.norm()), "grad_norm_b": float(b.grad.norm())}
    op.close()
    print(json.dumps(res), flush=True)


def ildl_bench(args, asss, torch, np, W):
    """The general incomplete LDL^T preconditioner (precond = ILDL, Sec. 3;
    ildl(1e-2) as in the paper's experiments) against the diagonal reading on
    implicit-Euler grids (the 45 x 45 grid of the small parity workload and a
    100 x 100 one), S tridiagonal, k = 8, tol 1e-8, FGMRES(64), inner
    tolerance 1e-2; FP64.  The ILDL path runs both ways: with J_tilde formed
    at setup ("ildl", the default at these sizes: the inner step is the fused
    sliced kernel on the explicit operator) and with two level-scheduled
    triangular solves in one workgroup per inner step ("ildl_levels", whose
    time is the chain of levels: reported per level as well).  The oracle's
    ILDL solve of the 45 x 45 grid is timed beside it."""
    import oracle as O
    from oracle.ildl import IldlOptions
    out = {"metric": "time-to-1e-8 rel. residual with the incomplete LDL^T preconditioner", "unit": "s",
           "n_gpus": 1, "higher_is_better": False, "dtype": "f64", "data": "synthetic", "cases": []}
    kw = dict(tol=1e-8, restart_m=64, inner_tol=1e-2, max_outer=2000)
    for m in (45, 100):
        w = W.implicit_euler_grid(m=m, h=0.1, cfg=0)
        b = torch.from_numpy(w.b).cuda()
        rec = {"workload": f"implicit_euler_{m}x{m}_h0.1", "n": int(w.A.shape[0]), "k": 8, "s_pattern": "tridiag"}
        for name, skw in (("ildl", dict(precond="ildl", ildl_droptol=1e-2, ildl_explicit=True)),
                          ("ildl_levels", dict(precond="ildl", ildl_droptol=1e-2, ildl_explicit=False)),
                          ("diag", {})):
            t0 = time.perf_counter()
            h = asss.setup(w.A, k=8, s_pattern="tridiag", **skw)
            torch.cuda.synchronize()
            setup_s = time.perf_counter() - t0
            h.solve(b, **kw)  # warm-up
            best, inf = float("inf"), None
            for _ in range(max(1, args.steps)):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                x, inf = h.solve(b, **kw)
                torch.cuda.synchronize()
                best = min(best, time.perf_counter() - t0)
            err = float(torch.linalg.norm(x.cpu() - torch.from_numpy(w.x_star)) / np.linalg.norm(w.x_star))
            r = {"solve_s": round(best, 5), "setup_s": round(setup_s, 3), "outer_its": inf["outer_its"],
                 "inner_its": inf["inner_its_total"], "relres_true": inf["relres_true"], "rel_err_vs_xstar": err,
                 "inner_step_us": round(1e6 * inf["inner_kernel_s"] / max(1, inf["inner_its_total"]), 2)}
            if name == "ildl_levels":
                hi = h.info()
                lev = hi["ildl_levels_lower"] + hi["ildl_levels_upper"]
                r.update(levels_lower=hi["ildl_levels_lower"], levels_upper=hi["ildl_levels_upper"],
                         nnz_l=hi["ildl_nnz_l"], us_per_level=round(r["inner_step_us"] / max(1, lev), 3))
            rec[name] = r
            log(f"{rec['workload']} {name}: {r}")
            h.close()
        rec["speedup_ildl_vs_diag"] = round(rec["diag"]["solve_s"] / rec["ildl"]["solve_s"], 3)
        rec["speedup_explicit_vs_levels"] = round(rec["ildl_levels"]["solve_s"] / rec["ildl"]["solve_s"], 3)
        out["cases"].append(rec)
    out["value"] = out["cases"][0]["ildl"]["solve_s"]
    out["config"] = {"workload": out["cases"][0]["workload"], "precond": "ildl(1e-2)", "outer": "fgmres(64)",
                     "inner_tol": 1e-2, "tol": 1e-8}
    if not args.no_cpu_baseline:
        w = W.implicit_euler_grid(m=45, h=0.1, cfg=0)
        st = O.setup_ildl(w.A, O.SetupOptions(k=8, s_pattern="tridiag"), IldlOptions(droptol=1e-2))
        best = float("inf")
        for _ in range(3):
            t0 = time.perf_counter()
            _, info = O.solve(st, w.b, O.SolveOptions(tol=1e-8, restart_m=64, inner_tol=1e-2))
            best = min(best, time.perf_counter() - t0)
        out["cpu_baseline"] = {"value": round(best, 4), "unit": "s", "cores": os.cpu_count(), "kind": "oracle",
                               "sample": f"oracle ILDL solve of the 45 x 45 grid (best of 3, setup not timed; "
                                         f"{info['outer_its']} outer / {info['inner_its_total']} inner steps, dense "
                                         f"triangular solves)"}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--m", type=int, default=192, help="grid points per axis")
    ap.add_argument("--peclet", type=float, default=1000.0)
    ap.add_argument("--cfg", type=int, default=None,
                    help="seed of the x* draw (workload number): 2 for the 192^3 Pe 1000 precision "
                         "workload, 1 for the 128^3 Pe 100 one; default: 2 unless --m 128 --peclet 100")
    ap.add_argument("--k", type=int, default=16)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--restart", type=int, default=200, help="FGMRES restart length")
    ap.add_argument("--inner-tol", type=float, default=0.2,
                    help="inner mrs tolerance (0.2 minimises time-to-solution on the 3D workloads)")
    ap.add_argument("--max-outer", type=int, default=2000,
                    help="cap on outer iterations (profiling runs only; the result then does not reach tol)")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--fp32-basis-solve", action="store_true",
                    help="also run the FP64 solve with the FP32-valued deflation basis (a second setup)")
    ap.add_argument("--cpu-sizes", type=int, nargs=2, default=[16, 24],
                    help="grid sizes of the two oracle runs of the CPU baseline")
    ap.add_argument("--verbose", action="store_true")
    ap.add_argument("--probe", action="store_true",
                    help="profiling probe: setup, a 1 GiB device copy (counter calibration), then "
                         "--probe-steps fixed inner mrs steps in FP64 and in FP32; no solve")
    ap.add_argument("--probe-steps", type=int, default=50)
    ap.add_argument("--batched", action="store_true",
                    help="batched workload instead: 64 uneven implicit-Euler systems (n log-uniform in "
                         "[1e4, 5e5]), 4 right-hand sides each, FP32 inner / FP64 outer, tol 1e-8; "
                         "reports right-hand sides per second for the lockstep block solve and for "
                         "column-by-column solves")
    ap.add_argument("--nsys", type=int, default=64)
    ap.add_argument("--engine-only", action="store_true",
                    help="with --batched: time only the lockstep engine (profiling runs)")
    ap.add_argument("--grad", action="store_true",
                    help="differentiation workload instead: 1000 x 1000 implicit-Euler grid (n = 1e6), "
                         "loss ||x - x_t||^2, forward solve + backward (adjoint solve and dL/dA, dL/db) "
                         "through the autograd function, FP64, tol 1e-10")
    ap.add_argument("--ildl", action="store_true",
                    help="incomplete LDL^T workload instead: the ILDL preconditioner (ildl(1e-2)) against the "
                         "diagonal reading on 45 x 45 and 100 x 100 implicit-Euler grids, FP64, tol 1e-8")
    ap.add_argument("--outer", default="fgmres", choices=["fgmres", "tfqmr"])
    ap.add_argument("--deflation", default="explicit", choices=["explicit", "explicit_fp32_basis"],
                    help="explicit_fp32_basis: the Lanczos vectors rounded to FP32 values and used so "
                         "everywhere (same preconditioner, FP64 arithmetic, half the basis bytes)")
    ap.add_argument("--inner-order", choices=["natural", "tiles", "grid"], default="grid",
                    help="order of the inner system (a symmetric permutation of J_tilde that the "
                         "solution does not depend on): the library's own tiles of whole x-lines for a "
                         "detected 3D grid (reorder='grid', default), tiles passed by the caller (--tile "
                         "TYxTZ lines per tile, one tile per row block), or the grid's natural order")
    ap.add_argument("--tile", default="4x4")
    ap.add_argument("--natural", action="store_true",
                    help="also run one solve per precision with the inner system in the natural order")
    ap.add_argument("--autotune", choices=["on", "off"], default=None,
                    help="row-block autotuner at setup (times the inner step for several row-block "
                         "sizes and keeps the fastest).  Default: on for --batched, off for the 3D "
                         "workloads")
    args = ap.parse_args()
    args.autotune = (args.autotune == "on") if args.autotune else bool(args.batched)
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    if args.cfg is None:
        args.cfg = 1 if (args.m == 128 and args.peclet == 100.0) else 2

    import numpy as np
    import torch

    import paper_2009_06954_amd as asss
    import workloads as W

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    asss.load()
    torch.cuda.set_device(0)
    if args.batched:
        return batched(args, asss, torch, np, W)
    if args.grad:
        return grad_bench(args, asss, torch, np, W)
    if args.ildl:
        return ildl_bench(args, asss, torch, np, W)
    log(f"building workload m={args.m} Pe={args.peclet:g} (seed of workload {args.cfg})")
    w = W.convdiff3d(m=args.m, peclet=args.peclet, cfg=args.cfg)
    n, nnz = w.A.shape[0], w.A.nnz
    log(f"n={n} nnz={nnz}; setup (host preprocessing + device data)")
    t0 = time.perf_counter()
    order_kw = {}
    order_name = {"natural": "natural", "tiles": f"x-line tiles {args.tile}",
                  "grid": "library grid order"}[args.inner_order]
    if args.inner_order == "grid":
        order_kw["reorder"] = "grid"
    if args.inner_order == "tiles":
        ty, tz = (int(v) for v in args.tile.split("x"))
        order_kw["reorder"] = W.grid_line_tiles(args.m, ty, tz)
        if not args.autotune:
            order_kw["row_block"] = args.m * ty * tz  # one tile per row block
    h = asss.setup(w.A, k=args.k, s_pattern="abar", verbose=args.verbose, autotune=args.autotune,
                   deflation=args.deflation, **order_kw)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    hi = h.info()
    log(f"setup {setup_s:.2f} s: {hi}")
    key = workload_key(args.m, args.peclet, args.k, order_name)
    b = torch.from_numpy(w.b).cuda()
    xs = torch.from_numpy(w.x_star).cuda()
    x = torch.empty_like(b)

    def copy_rate():
        # practical roof: a 1 GiB device-to-device copy (read + write), best of
        # 5, HIP events on torch's stream, outside any timed region
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ms = []
        for _ in range(5):
            ev[0].record(); dst.copy_(src); ev[1].record(); torch.cuda.synchronize()
            ms.append(ev[0].elapsed_time(ev[1]))
        return 2 * src.numel() * 4, round(2 * src.numel() * 4 / (min(ms) * 1e-3) / 1e9, 1)

    if args.probe:
        copy_bytes, copy_gbs = copy_rate()
        out = {"probe": True, "workload": key, "copy_bytes": copy_bytes, "copy_GBs": copy_gbs}
        for mixed in (False, True):
            h.apply("mrs", b, fixed_inner_steps=5, inner_fp32=mixed)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            h.apply("mrs", b, fixed_inner_steps=args.probe_steps, inner_fp32=mixed)
            torch.cuda.synchronize()
            out["mrs_fp32" if mixed else "mrs_fp64"] = round((time.perf_counter() - t0) / args.probe_steps * 1e6, 1)
            log(f"probe {'fp32' if mixed else 'fp64'}: {out['mrs_fp32' if mixed else 'mrs_fp64']} us per step")
        out["handle"] = hi
        h.close()
        print(json.dumps(out), flush=True)
        return

    def run(mixed: bool, steps: int, warmup: int, h=h):
        for i in range(warmup):
            _, inf = h.solve(b, out=x, tol=args.tol, inner_fp32=mixed, restart_m=args.restart,
                             inner_tol=args.inner_tol, max_outer=args.max_outer, outer=args.outer)
            log(f"warmup {'mixed' if mixed else 'fp64'} {i}: {inf['solve_s']:.3f} s, "
                f"outer {inf['outer_its']}, inner {inf['inner_its_total']}, relres {inf['relres_true']:.2e}")
        torch.cuda.synchronize()
        infos = []
        t0 = time.perf_counter()
        for i in range(steps):
            _, inf = h.solve(b, out=x, tol=args.tol, inner_fp32=mixed, restart_m=args.restart,
                             inner_tol=args.inner_tol, max_outer=args.max_outer, outer=args.outer)
            infos.append(inf)
        torch.cuda.synchronize()
        total = time.perf_counter() - t0
        err = float(torch.linalg.norm(x - xs) / torch.linalg.norm(xs))
        for i, inf in enumerate(infos):
            log(f"step {'mixed' if mixed else 'fp64'} {i}: {inf['solve_s']:.3f} s, outer {inf['outer_its']}, "
                f"inner {inf['inner_its_total']}, relres {inf['relres_true']:.2e}, status {inf['status']}")
        return total, infos, err

    def roofline(infos, v, deflation):
        # kernel time of every launch (HIP events around each chunk of back-to-back
        # launches on the solve's stream) per full step: a solve also launches one
        # deferred-update step and, after its end, steps that return at once (the
        # outer step launches a chunk with a margin before it waits); their few
        # microseconds are charged to the full steps
        kern_s = sum(i["inner_kernel_s"] for i in infos)
        launches = sum(i["inner_launches"] for i in infos)
        steps = sum(i["inner_its_total"] for i in infos)
        avg = kern_s / max(1, steps)
        bpr = mrs_bytes_per_row(hi["nh"] / n, hi["k_eff"], v, 4 if deflation == "explicit_fp32_basis" else v)
        per_step = bpr * n
        achieved = per_step * steps / kern_s / 1e9
        traffic = measured_traffic("fp64" if v == 8 else "fp32", key, deflation)
        return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "traffic_unit": "HBM bytes per full step (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                "traffic_GBs": round(traffic * steps / kern_s / 1e9, 1) if traffic else None,
                "copy_ceiling_GBs": copy_gbs,
                "kernel": "k_mrs_iter (fused inner mrs step)",
                "bytes_per_step": int(per_step), "bytes_per_row": round(bpr, 1),
                "avg_step_us": round(avg * 1e6, 2), "launches": launches, "full_steps": steps}

    _, copy_gbs = copy_rate()
    total64, inf64, err64 = run(False, args.steps, args.warmup)
    t64 = total64 / args.steps
    x64 = x.clone()
    res = {
        "metric": METRIC, "value": round(t64, 5), "unit": "s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(1e3 * t64, 3), "higher_is_better": False,
        "scaling": "strong", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"convdiff3d_{args.m}^3_Pe{args.peclet:g}", "n": n, "nnz": nnz,
                   "k": args.k, "s_pattern": "abar", "tol": args.tol,
                   "outer": f"fgmres({args.restart})" if args.outer == "fgmres" else "tfqmr",
                   "inner_tol": args.inner_tol, "row_block": hi["row_block"],
                   "inner_order": order_name, "deflation": args.deflation,
                   "step_threads": {"fp64": hi.get("step_threads_fp64"), "fp32": hi.get("step_threads")}},
        "roofline": roofline(inf64, 8, args.deflation),
        "solve": {"outer_its": inf64[-1]["outer_its"], "inner_its": inf64[-1]["inner_its_total"],
                  "reorth_passes": inf64[-1]["reorth"],
                  "relres_true": inf64[-1]["relres_true"], "rel_err_vs_xstar": err64,
                  "inner_its_per_s": round(inf64[-1]["inner_its_total"] / inf64[-1]["solve_s"], 1)},
        "setup_s": round(setup_s, 2),
        "setup_host_s": round(inf64[-1]["setup_host_s"], 2),
        "setup_device_s": round(inf64[-1]["setup_device_s"], 2),
        "solve_s_per_step": [round(i["solve_s"], 4) for i in inf64],
    }
    if args.autotune:
        res["autotune"] = {"row_blocks": hi["tune_rows"], "inner_step_us": [round(t, 1) for t in hi["tune_us"]],
                           "tune_s": round(hi["tune_s"], 2)}
    if not args.no_mixed:
        total32, inf32, err32 = run(True, args.steps, args.warmup)
        t32 = total32 / args.steps
        res["mixed"] = {"value": round(t32, 5), "unit": "s",
                        "dtype": "f32 storage, f64 accumulation inner / f64 outer",
                        "speedup_vs_fp64": round(t64 / t32, 3), "roofline": roofline(inf32, 4, args.deflation),
                        "outer_its": inf32[-1]["outer_its"], "inner_its": inf32[-1]["inner_its_total"],
                        "relres_true": inf32[-1]["relres_true"], "rel_err_vs_xstar": err32,
                        "rel_diff_vs_fp64_solution": float(torch.linalg.norm(x - x64) / torch.linalg.norm(x64)),
                        "solve_s_per_step": [round(i["solve_s"], 4) for i in inf32]}
    if args.natural and args.inner_order != "natural":
        log("natural order of the inner system: setup and one solve per precision")
        hn = asss.setup(w.A, k=args.k, s_pattern="abar", deflation=args.deflation)
        nat = {"row_block": hn.info()["row_block"]}
        for mixed in ([False] if args.no_mixed else [False, True]):
            tn, infn, _ = run(mixed, 1, 1, h=hn)
            kk = "mixed" if mixed else "fp64"
            nat[kk + "_s"] = round(tn, 5)
            nat[kk + "_avg_step_us"] = round(1e6 * infn[-1]["inner_kernel_s"] / max(1, infn[-1]["inner_its_total"]), 2)
            nat[kk + "_inner_its"] = infn[-1]["inner_its_total"]
        hn.close()
        nat["speedup_of_order_fp64"] = round(nat["fp64_s"] / t64, 3)
        res["natural_order"] = nat
    if args.fp32_basis_solve and args.deflation == "explicit":
        # the FP64 solve with the deflation basis rounded to FP32 values (same
        # preconditioner P, FP64 arithmetic; the FP64 inner step reads the basis
        # as 4-byte values)
        log("FP64 solve with the FP32-valued deflation basis: setup and the same steps")
        tq0 = time.perf_counter()
        hq = asss.setup(w.A, k=args.k, s_pattern="abar", deflation="explicit_fp32_basis",
                        autotune=args.autotune, **order_kw)
        torch.cuda.synchronize()
        setup_q = time.perf_counter() - tq0
        tq, infq, errq = run(False, args.steps, args.warmup, h=hq)
        tq /= args.steps
        res["fp64_fp32_basis"] = {
            "value": round(tq, 5), "unit": "s", "dtype": "f64", "deflation": "explicit_fp32_basis",
            "speedup_vs_fp64": round(t64 / tq, 3), "roofline": roofline(infq, 8, "explicit_fp32_basis"),
            "outer_its": infq[-1]["outer_its"], "inner_its": infq[-1]["inner_its_total"],
            "relres_true": infq[-1]["relres_true"], "rel_err_vs_xstar": errq,
            "rel_diff_vs_fp64_solution": float(torch.linalg.norm(x - x64) / torch.linalg.norm(x64)),
            "solve_s_per_step": [round(i["solve_s"], 4) for i in infq], "setup_s": round(setup_q, 2)}
        hq.close()
    h.close()
    if not args.no_cpu_baseline:
        log(f"cpu baseline: oracle on convdiff3d {args.cpu_sizes[0]}^3 and {args.cpu_sizes[1]}^3")
        try:
            res["cpu_baseline"] = cpu_baseline(args.cpu_sizes, args.peclet, args.cfg, args.k, args.tol, n,
                                               inf64[-1]["inner_its_total"], args.inner_tol, args.restart)
        except Exception as e:  # the baseline must not hide the GPU result
            res["cpu_baseline"] = {"value": None, "error": repr(e)}
        xs = res["cpu_baseline"].pop("_x", None)
        if xs:
            mo = max(xs)
            log(f"error against the oracle on convdiff3d {mo}^3")
            try:
                res["oracle_parity"] = oracle_parity(asss, torch, np, W, mo, args.peclet, args.cfg, args.k,
                                                     args.tol, args.inner_tol, args.restart, xs[mo])
            except Exception as e:
                res["oracle_parity"] = {"error": repr(e)}
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
