#!/usr/bin/env python3
"""Benchmark of the repulsive-curves hot path on one MI355X.

Workload (default): a random smooth closed curve with 16,384 edges (Fourier
modes k = 1..8, coefficients N(0, 1/k^2), seed 0), tangent-point exponents
(alpha, beta) = (2, 4.5), pair kernels in FP32, barycenter + edge-length
constraints.  One step is one projected Sobolev step: energy and
differential, constraint and multigrid setup, projected PCG to a relative
FP64 residual of 1e-6, and the backtracking line search with constraint
projection.

Printed (one JSON line): edge-pair evaluations per second of the energy +
differential phase (ordered disjoint edge pairs / phase time), Sobolev steps
per second, the roofline of the dominant pair kernel (timed live with HIP
events on the library's stream), and the FP64 oracle timed on a bounded
sample on the host CPU.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# FP32 flops per ordered edge pair (four vertex pairs) of the two pair kernels,
# counted from their formulas; the transcendental operations (rsqrt, sqrt) are
# counted separately and not included.
FLOPS_PER_PAIR_TPE = 344   # energy + differential, 86 per vertex pair, 2 transcendentals
FLOPS_PER_PAIR_SOB = 198   # operator A = B + B0 applied to 3 right-hand sides
PEAK_FP32_TFLOPS = 157.3   # MI355X vector FP32 (packed); the non-packed issue limit is half


def ordered_disjoint_pairs(edges):
    import numpy as np

    e = np.asarray(edges)
    nE = len(e)
    deg = np.bincount(e.ravel())
    # pairs sharing a vertex: I = J, plus for every vertex the ordered pairs of distinct incident edges
    sharing = nE + int((deg * (deg - 1)).sum())
    return nE * nE - sharing


def cpu_baseline(g, e, alpha, beta, seconds=12.0):
    """The FP64 oracle's energy + differential on a bounded sample of target edges."""
    import numpy as np

    from oracle import tpe

    nE = len(e)
    cols = np.arange(nE)
    rows_done, t0 = 0, time.perf_counter()
    chunk = 64
    while time.perf_counter() - t0 < seconds and rows_done < nE:
        rows = np.arange(rows_done, min(nE, rows_done + chunk))
        tpe._block(g, e, alpha, beta, rows, cols, True)
        rows_done += len(rows)
    dt = time.perf_counter() - t0
    pairs = rows_done * nE
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count()
    return {
        "value": pairs / dt,
        "unit": "pairs/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"{rows_done} target edges x {nE} sources ({pairs:.3g} ordered pairs, FP64 numpy, one thread; "
                  f"{cores} host cores visible)",
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--edges", type=int, default=16384)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", default="step", choices=["step", "bh"],
                    help="step: projected Sobolev steps on the 16,384-edge knot (default); "
                         "bh: Barnes-Hut energy+differential on a 262,144-edge knot")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; multi-GPU runs are not supported "
                                   "(the sharding design is described in DESIGN.md)", "n_gpus": args.gpus}))
        sys.exit(2)

    if args.workload == "bh":
        return bench_bh(args)

    import numpy as np
    import torch

    import gen
    from paper_2006_07859_amd import (RC_C_BARYCENTER, RC_C_EDGE_LENGTH, RC_F32, RC_SOLVE_PCG_MG, Context,
                                      default_ls_opts, default_solve_opts)

    alpha, beta, n = 2.0, 4.5, args.edges
    g, e, _ = gen.fourier_knot(n, seed=0)
    g = gen.round_to_f32(g)
    P = ordered_disjoint_pairs(e)
    torch.cuda.init()
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    ctx = Context(len(g), e, alpha, beta, RC_F32)
    gamma = dev(g)
    ctx.rc_set_constraints(RC_C_BARYCENTER | RC_C_EDGE_LENGTH, gamma)
    so = default_solve_opts(solver=RC_SOLVE_PCG_MG, tol=1e-6, mg_min_vertices=256, cheb_degree=2, op_f64=1)
    ls = default_ls_opts()

    for _ in range(args.warmup):
        ctx.rc_step(gamma, so=so, ls=ls)
    torch.cuda.synchronize()
    ctx.rc_profile_enable(True)
    stats = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        st = ctx.rc_step(gamma, so=so, ls=ls)
        stats.append(st)
        print(f"[bench] step {k}: E {st['energy']:.6g} -> {st['energy_new']:.6g}, pcg {st['iterations']} it, "
              f"res {st['residual']:.2e}, tau {st['tau']:.3g}, eval {st['t_eval_ms']:.2f} ms, "
              f"solve {st['t_solve_ms']:.1f} ms, search {st['t_search_ms']:.1f} ms", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    T = time.perf_counter() - t0
    tpe_ms, tpe_n = ctx.rc_profile_read(0)
    sob_ms, sob_n = ctx.rc_profile_read(1)
    ctx.rc_profile_enable(False)

    t_eval = float(np.mean([s["t_eval_ms"] for s in stats])) * 1e-3
    value = P / t_eval
    tpe_avg = tpe_ms / max(tpe_n, 1) * 1e-3
    sob_avg = sob_ms / max(sob_n, 1) * 1e-3
    roof_tpe = FLOPS_PER_PAIR_TPE * P / tpe_avg / 1e12
    roof_sob = FLOPS_PER_PAIR_SOB * P / sob_avg / 1e12
    # the dominant kernel of the step is the one with the larger total time
    if sob_ms >= tpe_ms:
        dom = {"kernel": "k_sob_pairs<float> (operator, finest level)", "launches": sob_n,
               "avg_ms": sob_avg * 1e3, "flops_per_pair": FLOPS_PER_PAIR_SOB, "achieved_tflops": roof_sob}
    else:
        dom = {"kernel": "k_tpe_pairs<float> (energy+differential)", "launches": tpe_n,
               "avg_ms": tpe_avg * 1e3, "flops_per_pair": FLOPS_PER_PAIR_TPE, "achieved_tflops": roof_tpe}
    roofline = {
        "bound": "alu",
        "achieved": round(dom["achieved_tflops"], 3),
        "peak": PEAK_FP32_TFLOPS,
        "unit": "TFLOP/s",
        "frac": round(dom["achieved_tflops"] / PEAK_FP32_TFLOPS, 4),
        "traffic": None,
        "kernel": dom["kernel"],
        "avg_launch_ms": round(dom["avg_ms"], 4),
        "launches": dom["launches"],
    }
    out = {
        "metric": "edge-pair evals/s (energy+grad)",
        "value": value,
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": T / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"fourier knot, {n} edges, (alpha,beta)=(2,4.5), FP32 pair kernels, barycenter+edge-length "
                        f"constraints, multigrid PCG to 1e-6 FP64 residual, backtracking line search",
            "edges": n,
            "ordered_pairs": P,
        },
        "sobolev_steps_per_s": args.steps / T,
        "phases_ms": {
            "energy_differential": t_eval * 1e3,
            "setup_and_solve": float(np.mean([s["t_solve_ms"] for s in stats])),
            "line_search": float(np.mean([s["t_search_ms"] for s in stats])),
        },
        "pcg_iterations": [s["iterations"] for s in stats],
        "pcg_residual": [s["residual"] for s in stats],
        "projection_solve_iterations": [s["proj_solve_iterations"] for s in stats],
        "roofline": roofline,
        "roofline_energy_differential": {
            "kernel": "k_tpe_pairs<float>", "launches": tpe_n, "avg_launch_ms": round(tpe_avg * 1e3, 4),
            "achieved": round(roof_tpe, 3), "unit": "TFLOP/s", "frac": round(roof_tpe / PEAK_FP32_TFLOPS, 4),
            "pairs_per_s_kernel": P / tpe_avg,
        },
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(g, e, alpha, beta)
    ctx.close()
    print(json.dumps(out))


def bench_bh(args):
    """Barnes-Hut (theta = 0.25, leaves of 32) on a 262,144-edge knot, FP32."""
    import numpy as np
    import torch

    import gen
    from paper_2006_07859_amd import RC_F32, Context

    n = 262144 if args.edges == 16384 else args.edges
    alpha, beta, theta = 2.0, 4.5, 0.25
    g, e, _ = gen.fourier_knot(n, seed=0)
    g = gen.round_to_f32(g)
    P = ordered_disjoint_pairs(e)
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    ctx = Context(n, e, alpha, beta, RC_F32)
    gamma = dev(g)
    E = torch.zeros(1, dtype=torch.float64, device="cuda")
    dE = torch.zeros(n, 3, dtype=torch.float64, device="cuda")
    for _ in range(args.warmup):
        ctx.rc_bh_differential(gamma, theta, 32, E, dE)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ctx.rc_bh_differential(gamma, theta, 32, E, dE)
    torch.cuda.synchronize()
    T = (time.perf_counter() - t0) / args.steps
    work = ctx.rc_bh_last_work()
    # exact edge-midpoint sum (the theta -> 0 limit) for the error
    Em = torch.zeros(1, dtype=torch.float64, device="cuda")
    dEm = torch.zeros_like(dE)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ctx.rc_midpoint_differential(gamma, Em, dEm)
    torch.cuda.synchronize()
    Tm = time.perf_counter() - t1
    err_E = abs(E.item() - Em.item()) / abs(Em.item())
    err_G = (torch.linalg.norm(dE - dEm) / torch.linalg.norm(dEm)).item()
    out = {
        "metric": "exact-equivalent edge-pair evals/s (Barnes-Hut energy+grad)",
        "value": P / T,
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": T * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"fourier knot, {n} edges, (alpha,beta)=(2,4.5), Barnes-Hut theta=0.25, leaf 32, "
                               f"BVH built on the device every evaluation", "edges": n, "ordered_pairs": P},
        "interactions": work,
        "exact_midpoint_ms": Tm * 1e3,
        "error_vs_exact_midpoint": {"energy_rel": err_E, "differential_rel": err_G},
    }
    ctx.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
