#!/usr/bin/env python3
"""Benchmark of the repulsive-curves hot path on one MI355X.

Workload (default): a random smooth closed curve with 16,384 edges (Fourier
modes k = 1..8, coefficients N(0, 1/k^2), seed 0), tangent-point exponents
(alpha, beta) = (2, 4.5), pair kernels in FP32, barycenter + edge-length
constraints.  One step is one projected Sobolev step: energy and
differential, constraint and multigrid setup (BF16 assembled blocks as the
smoothers' operators), projected PCG to a relative FP64 residual of 1e-6 with
the FP64 matrix-free operator, and the backtracking line search with
constraint projection.  The same steps with the plain multigrid (FP32
matrix-free smoothers) are timed after it for comparison.

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

# FP32 flops of the energy + differential kernel.  For alpha = 2 on loops and
# paths the kernel evaluates the trapezoid sum regrouped by vertex pair: one
# pair of vertices (v, w) stands for the four vertex pairs of the four edge
# pairs at v and w, at 93 flops (32 + 4 FMAs, 18 multiplies, 3 subtractions in
# its gfx950 inner loop) and 2 transcendentals (rsqrt, sqrt) per vertex pair,
# and a closed curve has as many vertex pairs as edge pairs.  The edge-pair
# form it replaces took 280 algorithmic flops per edge pair (213 executed).
FLOPS_PER_PAIR_TPE = 93    # energy + differential, vertex-pair form (algorithmic = executed)
FLOPS_PER_PAIR_TPE_EXEC = 93
FLOPS_PER_EDGE_PAIR = 280  # energy + differential, edge-pair form (other exponents, batches)
# Operator A = B + B0 applied to 3 right-hand sides: about 100 flops per pair for
# the gather form; the FP32 kernel executes about 135 and 8 transcendentals per
# pair, the FP64 one about 190 with its powers from an FP32 estimate and Newton steps.
FLOPS_PER_PAIR_SOB = 100   # operator, algorithmic
# Edge-midpoint kernel k(x_I, x_J, T_I) l_I l_J and its partials for one ordered pair (Barnes-Hut leaf pairs
# and cluster interactions): 86 FP32 flops and 2 transcendentals as evaluated.
FLOPS_PER_PAIR_MID = 86
# block cluster tree near field, per edge pair (FP64): difference, squared distance, the two cross
# products and their squares (~40), the powers of |d| from an FP32 estimate and Newton steps (~12),
# the two kernels (~8), and 14 accumulated products (28)
FLOPS_PER_NEAR_PAIR_BCT = 90
PEAK_FP32_TFLOPS = 157.3   # MI355X vector FP32 (packed); the non-packed issue limit is half
PEAK_FP64_TFLOPS = 78.6    # MI355X vector FP64
PEAK_HBM_GBS = 8000.0      # MI355X HBM3E


CALIB_COPY_BYTES = 1 << 30  # the plain device copy that scales the HBM byte counters


def calibration_copy():
    """One device-to-device copy of CALIB_COPY_BYTES (1 GiB read + 1 GiB written): the reference
    dispatch against which rocprofv3's FETCH_SIZE / WRITE_SIZE counters of the other kernels are scaled."""
    import torch

    src = torch.ones(CALIB_COPY_BYTES // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


def traffic_record(kernel, edges):
    """HBM bytes per launch of `kernel` on the `edges`-edge workload from the rocprofv3 counter summaries under profiles/
    (FETCH_SIZE + WRITE_SIZE scaled by the copy calibration), or None when there is no record or a
    source file it was measured with has changed since."""
    import glob
    import hashlib

    key = kernel.split(" ")[0]
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        for line in open(path):
            if not line.startswith("traffic-record: "):
                continue
            rec = json.loads(line[len("traffic-record: "):])
            if rec["kernel"].split(" ")[0] != key or f"{edges} edges" not in rec["workload"]:
                continue
            for src, digest in rec["sources"].items():
                f = os.path.join(ROOT, src)
                if not os.path.exists(f) or hashlib.sha256(open(f, "rb").read()).hexdigest() != digest:
                    return None
            return rec["traffic_bytes"]
    return None


def ordered_disjoint_pairs(edges):
    import numpy as np

    e = np.asarray(edges)
    nE = len(e)
    deg = np.bincount(e.ravel())
    # pairs sharing a vertex: I = J, plus for every vertex the ordered pairs of distinct incident edges
    sharing = nE + int((deg * (deg - 1)).sum())
    return nE * nE - sharing


_ORACLE_ARGS = None


def _oracle_init(args):
    global _ORACLE_ARGS
    _ORACLE_ARGS = args


def _oracle_rows(r0, r1):
    """Energy + differential of the oracle for target edges r0 .. r1-1 against every source (one process)."""
    import numpy as np

    from oracle import tpe

    g, e, alpha, beta = _ORACLE_ARGS
    tpe._block(g, e, alpha, beta, np.arange(r0, r1), np.arange(len(e)), True)
    return (r1 - r0) * len(e)


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(g, e, alpha, beta, seconds=12.0, seconds_single=5.0, chunk=64):
    """The FP64 oracle's energy + differential on a bounded sample of target edges: on every host core
    available to this process (a process pool over blocks of `chunk` target edges, one single-threaded
    numpy process per core, at most 16), and on one core."""
    import concurrent.futures as cf
    import multiprocessing as mp

    nE = len(e)
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    workers = max(1, min(avail, 16))
    # one core
    _oracle_init((g, e, alpha, beta))
    rows1, t0 = 0, time.perf_counter()
    while time.perf_counter() - t0 < seconds_single and rows1 < nE:
        _oracle_rows(rows1, min(nE, rows1 + chunk))
        rows1 += chunk
    dt1 = time.perf_counter() - t0
    single = min(rows1, nE) * nE / dt1
    # all cores: single-threaded BLAS in every worker so that processes, not threads, share the cores
    keep = {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")}
    for k in keep:
        os.environ[k] = "1"
    ex = None
    pairs, dt, note = 0, 0.0, ""
    try:
        ex = cf.ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn"),
                                    initializer=_oracle_init, initargs=((g, e, alpha, beta),))
        # start the workers (numpy imports) before the clock starts
        warm = [ex.submit(_oracle_rows, 0, 1) for _ in range(workers)]
        cf.wait(warm, timeout=120)
        if not all(f.done() and f.exception() is None for f in warm):
            raise RuntimeError("oracle worker processes did not start")
        nxt, pending = 0, set()
        t0 = time.perf_counter()
        deadline = t0 + seconds + 120  # a block takes well under a minute; past this the pool is broken
        while True:
            while len(pending) < 2 * workers and time.perf_counter() - t0 < seconds:
                r0 = nxt % nE
                pending.add(ex.submit(_oracle_rows, r0, min(nE, r0 + chunk)))
                nxt += chunk
            if not pending:
                break
            if time.perf_counter() > deadline:
                raise RuntimeError("oracle worker processes stopped answering")
            done, pending = cf.wait(pending, timeout=10, return_when=cf.FIRST_COMPLETED)
            pairs += sum(f.result() for f in done)
        dt = time.perf_counter() - t0
    except Exception as exc:  # the all-core leg is a baseline only: report the one-core figure instead
        note = f"; all-core leg failed ({exc}), one-core figure reported"
        pairs, dt, workers = min(rows1, nE) * nE, dt1, 1
    finally:
        if ex is not None:
            procs = list(getattr(ex, "_processes", {}).values())
            ex.shutdown(wait=False, cancel_futures=True)
            for pr in procs:
                if pr.is_alive():
                    pr.kill()
        for k, v in keep.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    return {
        "value": pairs / dt,
        "unit": "pairs/s",
        "cores": workers,
        "kind": "oracle",
        "single_core_value": single,
        "sample": f"FP64 numpy oracle, energy + differential of blocks of {chunk} target edges x all {nE} sources: "
                  f"{pairs:.3g} ordered pairs in {dt:.1f} s on {workers} processes (one per core, "
                  f"single-threaded BLAS); one core: {min(rows1, nE) * nE:.3g} pairs in {dt1:.1f} s; "
                  f"{avail} host cores available, {_cpu_model()}{note}",
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--edges", type=int, default=16384)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true", help="default workload: skip the plain-multigrid comparison")
    ap.add_argument("--workload", default="step", choices=["step", "bh", "precision", "batch", "learned", "large"],
                    help="step: projected Sobolev steps on the 16,384-edge knot (default); "
                         "bh: Barnes-Hut energy+differential on a 262,144-edge knot; "
                         "precision: assembled 16-bit Sobolev block and a solve to 1e-8 on a 32,768-edge knot; "
                         "batch: 512 packing instances, one captured step; "
                         "learned: train the learned V-cycle smoother weights, then compare PCG preconditioners; "
                         "large: projected steps on a 262,144-edge knot with Barnes-Hut and the block cluster tree")
    ap.add_argument("--train-steps", type=int, default=1500, help="Adam steps of the learned smoother weights")
    ap.add_argument("--train-knots", type=int, default=24, help="knots whose flows give the training snapshots")
    ap.add_argument("--train-snapshots", type=int, default=40, help="snapshots per training knot")
    ap.add_argument("--batch-rows", type=int, default=32768, help="rows per Adam step")
    ap.add_argument("--tune-cache", default=None, help="JSON cache file of the batch tile autotuner")
    ap.add_argument("--fmt", default="bf16", choices=["bf16", "fp16"], help="16-bit format of the precision path")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; multi-GPU runs are not supported "
                                   "(the path is built and measured on one GPU's share)", "n_gpus": args.gpus}))
        sys.exit(2)

    if args.workload == "bh":
        return bench_bh(args)
    if args.workload == "precision":
        return bench_precision(args)
    if args.workload == "batch":
        return bench_batch(args)
    if args.workload == "learned":
        return bench_learned(args)
    if args.workload == "large":
        return bench_large(args)

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
    calibration_copy()
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    ctx = Context(len(g), e, alpha, beta, RC_F32)
    gamma = dev(g)
    ctx.rc_set_constraints(RC_C_BARYCENTER | RC_C_EDGE_LENGTH, gamma)
    # multigrid PCG: the Krylov recurrence on the assembled FP32 block, restarted from the FP64 matrix-free
    # true residual (the residual's judge) after each 1e-3 reduction; BF16 assembled blocks as the
    # smoothers' operators on every level with >= 512 vertices
    so = default_solve_opts(solver=RC_SOLVE_PCG_MG, tol=1e-6, mg_min_vertices=256, cheb_degree=2, op_f64=1,
                            lowp=1, lowp_band=16, lowp_min_vertices=512, lowp_outer=1, inner_tol=1e-3)
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
    lp_ms, lp_n = ctx.rc_profile_read(2)
    s64_ms, s64_n = ctx.rc_profile_read(4)
    a32_ms, a32_n = ctx.rc_profile_read(3)
    ctx.rc_profile_enable(False)

    t_eval = float(np.mean([s["t_eval_ms"] for s in stats])) * 1e-3
    value = P / t_eval
    tpe_avg = tpe_ms / max(tpe_n, 1) * 1e-3
    VP = len(g) * len(g)  # ordered vertex pairs the kernel visits (the near band's masked ones included)
    roof_tpe = FLOPS_PER_PAIR_TPE * VP / tpe_avg / 1e12
    # the timed kernels of the step (finest level), each against its own roofline
    kernels = [
        ("k_vp_pairs<float> (energy+differential, vertex-pair form)", tpe_ms, tpe_n, FLOPS_PER_PAIR_TPE * VP / 1e12, "alu",
         PEAK_FP32_TFLOPS, "TFLOP/s"),
        ("k_sob_pairs<float> (FP32 operator, finest level)", sob_ms, sob_n, FLOPS_PER_PAIR_SOB * P / 1e12, "alu",
         PEAK_FP32_TFLOPS, "TFLOP/s"),
        ("k_sob_pairs<double> (FP64 Krylov operator, finest level)", s64_ms, s64_n, FLOPS_PER_PAIR_SOB * P / 1e12,
         "alu", PEAK_FP64_TFLOPS, "TFLOP/s"),
        ("k_lowp_gemv<bf16> (smoother product, finest level)", lp_ms, lp_n, n * n * 2 / 1e9, "hbm", PEAK_HBM_GBS,
         "GB/s"),
        ("k_lowp_gemv32 (FP32 Krylov operator, finest level)", a32_ms, a32_n, n * n * 4 / 1e9, "hbm", PEAK_HBM_GBS,
         "GB/s"),
    ]
    rooflines = []
    for name, ms, nl, work, bound, peak, unit in kernels:
        if nl == 0:
            continue
        avg = ms / nl * 1e-3
        ach = work / avg
        rooflines.append({"bound": bound, "achieved": round(ach, 3), "peak": peak, "unit": unit,
                          "frac": round(ach / peak, 4), "traffic": traffic_record(name, n), "kernel": name,
                          "avg_launch_ms": round(avg * 1e3, 4), "launches": nl, "total_ms": round(ms, 2)})
    # the kernel behind `metric` (edge-pair evals/s of the energy + differential): the pair kernel, at the
    # algorithmic flops per pair and, beside it, at the flops its inner loop executes
    roofline = dict(rooflines[0])
    roofline["traffic_unit"] = "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)"
    roofline["flops_per_pair"] = FLOPS_PER_PAIR_TPE
    roofline["executed_flops_per_pair"] = FLOPS_PER_PAIR_TPE_EXEC
    roofline["executed_achieved"] = round(FLOPS_PER_PAIR_TPE_EXEC * VP / tpe_avg / 1e12, 3)
    roofline["vertex_pairs_per_launch"] = VP
    roofline["executed_frac"] = round(roofline["executed_achieved"] / PEAK_FP32_TFLOPS, 4)
    roofline["executed_frac_nonpacked"] = round(roofline["executed_achieved"] / (PEAK_FP32_TFLOPS / 2), 4)
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
                        f"constraints, multigrid PCG to 1e-6 FP64 residual (assembled FP32 Krylov operator, FP64 "
                        f"matrix-free true residual per 1e-3 sweep, BF16 assembled smoother blocks), "
                        f"backtracking line search",
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
        "refinement_sweeps": [s["sweeps"] for s in stats],
        "projection_solve_iterations": [s["proj_solve_iterations"] for s in stats],
        "roofline": roofline,
        "rooflines_timed_kernels": rooflines,
        "roofline_energy_differential": {
            "kernel": "k_vp_pairs<float>", "launches": tpe_n, "avg_launch_ms": round(tpe_avg * 1e3, 4),
            "achieved": round(roof_tpe, 3), "unit": "TFLOP/s", "frac": round(roof_tpe / PEAK_FP32_TFLOPS, 4),
            "pairs_per_s_kernel": P / tpe_avg, "flops_per_pair": FLOPS_PER_PAIR_TPE,
            "executed_flops_per_pair": FLOPS_PER_PAIR_TPE_EXEC,
            "executed_tflops": round(FLOPS_PER_PAIR_TPE_EXEC * VP / tpe_avg / 1e12, 3),
        },
    }
    # the same steps with the plain solver (FP32 matrix-free smoothers), from the same start
    ctx.close()
    if args.no_plain:
        if not args.no_cpu_baseline:
            out["cpu_baseline"] = cpu_baseline(g, e, alpha, beta)
        print(json.dumps(out))
        return
    ctx = Context(len(g), e, alpha, beta, RC_F32)
    gamma = dev(g)
    ctx.rc_set_constraints(RC_C_BARYCENTER | RC_C_EDGE_LENGTH, gamma)
    plain = default_solve_opts(solver=RC_SOLVE_PCG_MG, tol=1e-6, mg_min_vertices=256, cheb_degree=2, op_f64=1)
    ctx.rc_step(gamma, so=plain, ls=ls)
    torch.cuda.synchronize()
    tp = time.perf_counter()
    pst = [ctx.rc_step(gamma, so=plain, ls=ls) for _ in range(2)]
    torch.cuda.synchronize()
    Tp = (time.perf_counter() - tp) / 2
    out["plain_multigrid"] = {"sobolev_steps_per_s": 1.0 / Tp, "ms_per_step": Tp * 1e3,
                              "pcg_iterations": [s["iterations"] for s in pst],
                              "smoothers": "FP32 matrix-free operator on every level"}
    out["speedup_vs_plain"] = (args.steps / T) / (1.0 / Tp)
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
    ctx.rc_profile_enable(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ctx.rc_bh_differential(gamma, theta, 32, E, dE)
    torch.cuda.synchronize()
    T = (time.perf_counter() - t0) / args.steps
    trav_ms, trav_n = ctx.rc_profile_read(6)
    ctx.rc_profile_enable(False)
    work = ctx.rc_bh_last_work()
    # the traversal kernel against the FP32 vector peak: every cluster interaction and every leaf pair
    # visited is one evaluation of the edge-midpoint kernel and its partials (FLOPS_PER_PAIR_MID)
    trav_avg = trav_ms / max(trav_n, 1) * 1e-3
    interactions = work["far"] + work["near"]
    ach = FLOPS_PER_PAIR_MID * interactions / trav_avg / 1e12
    roofline = {"bound": "alu", "achieved": round(ach, 3), "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                "frac": round(ach / PEAK_FP32_TFLOPS, 4), "traffic": traffic_record("k_bh_traverse", n),
                "kernel": "k_bh_traverse<float> (Barnes-Hut traversal)", "avg_launch_ms": round(trav_avg * 1e3, 4),
                "launches": trav_n, "interactions_per_launch": interactions, "flops_per_interaction":
                FLOPS_PER_PAIR_MID}
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
        "roofline": roofline,
        "exact_midpoint_ms": Tm * 1e3,
        "error_vs_exact_midpoint": {"energy_rel": err_E, "differential_rel": err_G},
    }
    ctx.close()
    print(json.dumps(out))


def bench_large(args):
    """Projected Sobolev steps at 262,144 edges with the paper's large-curve
    approximations (App. B): Barnes-Hut energy and differential and trial
    energies (theta 0.25), multigrid PCG to a 1e-6 FP64 residual on block
    cluster tree operators (theta 0.25, every level of 16,384+ vertices),
    barycenter and edge-length constraints."""
    import numpy as np
    import torch

    import gen
    from paper_2006_07859_amd import (RC_C_BARYCENTER, RC_C_EDGE_LENGTH, RC_F32, RC_SOLVE_PCG_MG, Context,
                                      default_ls_opts, default_solve_opts)

    n = 262144 if args.edges == 16384 else args.edges
    alpha, beta, theta = 2.0, 4.5, 0.25
    g, e, _ = gen.fourier_knot(n, seed=0)
    g = gen.round_to_f32(g)
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    ctx = Context(n, e, alpha, beta, RC_F32)
    gamma = dev(g)
    ctx.rc_set_constraints(RC_C_BARYCENTER | RC_C_EDGE_LENGTH, gamma)
    so = default_solve_opts(solver=RC_SOLVE_PCG_MG, tol=1e-6, mg_min_vertices=256, cheb_degree=2, op_f64=1,
                            max_iter=200, bct_theta=theta, bct_min_vertices=8192)
    ls = default_ls_opts(bh_theta=theta)
    for _ in range(args.warmup):
        ctx.rc_step(gamma, so=so, ls=ls)
    torch.cuda.synchronize()
    stats = []
    t0 = time.perf_counter()
    for k in range(args.steps):
        st = ctx.rc_step(gamma, so=so, ls=ls)
        stats.append(st)
        print(f"[bench] large step {k}: E {st['energy']:.8g} -> {st['energy_new']:.8g}, pcg {st['iterations']} it, "
              f"res {st['residual']:.1e}, tau {st['tau']:.3g}, eval {st['t_eval_ms']:.1f} ms, solve "
              f"{st['t_solve_ms']:.1f} ms, search {st['t_search_ms']:.1f} ms", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    T = (time.perf_counter() - t0) / args.steps
    # the block cluster tree product at the final curve, timed alone on the context's stream
    ctx.rc_bct_build(gamma, theta, 32)
    bstats = ctx.rc_bct_stats()
    X = dev(np.random.default_rng(3).normal(size=(n, 3)))
    Y = torch.zeros_like(X)
    ctx.rc_sobolev_apply_bct(gamma, X, Y)
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(10):
        ctx.rc_sobolev_apply_bct(gamma, X, Y)
    ev1.record(stream)
    torch.cuda.synchronize()
    prod_ms = ev0.elapsed_time(ev1) / 10
    # the near field dominates the product: ~100 FP64 flops per near pair (kernel pair, 14 products)
    near_flops = FLOPS_PER_NEAR_PAIR_BCT * bstats["near_pairs"]
    ach = near_flops / (prod_ms * 1e-3) / 1e12
    out = {
        "metric": "projected Sobolev steps/s (262,144-edge knot, Barnes-Hut + block cluster tree)",
        "value": 1.0 / T,
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": T * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"fourier knot, {n} edges, (alpha,beta)=(2,4.5), barycenter+edge-length "
                               "constraints, Barnes-Hut energy/differential theta=0.25, multigrid PCG to 1e-6 on "
                               "block cluster tree operators theta=0.25 (levels of 8,192+ vertices)", "edges": n},
        "per_step": {"iterations": [s["iterations"] for s in stats], "tau": [s["tau"] for s in stats],
                     "t_eval_ms": [round(s["t_eval_ms"], 2) for s in stats],
                     "t_solve_ms": [round(s["t_solve_ms"], 1) for s in stats],
                     "t_search_ms": [round(s["t_search_ms"], 1) for s in stats]},
        "bct": bstats,
        "roofline": {"bound": "alu", "achieved": round(ach, 3), "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(ach / PEAK_FP64_TFLOPS, 4), "traffic": None,
                     "kernel": "block cluster tree product (all its launches; near-field FP64 flops)",
                     "avg_launch_ms": round(prod_ms, 4), "flops_per_near_pair": FLOPS_PER_NEAR_PAIR_BCT},
    }
    ctx.close()
    print(json.dumps(out))


def cpu_baseline_rows(g, e, alpha, beta, seconds=12.0):
    """The FP64 oracle producing rows of A (Sec. 4.2.2-4.2.3) and applying them to
    three columns, on a bounded sample of rows; reported as the 16-bit-equivalent
    bytes of A those rows amount to per second."""
    import numpy as np

    from oracle import sobolev

    n = len(g)
    X = np.random.default_rng(0).normal(size=(n, 3))
    done, t0 = 0, time.perf_counter()
    while time.perf_counter() - t0 < seconds and done < n:
        rows = list(range(done, min(n, done + 8)))
        R = sobolev.assemble_rows(g, e, alpha, beta, rows)
        _ = R @ X
        done += len(rows)
    dt = time.perf_counter() - t0
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count()
    return {
        "value": done * n * 2 / dt / 1e9,
        "unit": "GB/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"{done} rows of A (FP64 numpy assembly of the rows plus their product with 3 columns, one "
                  f"thread; {cores} host cores visible), counted as {n} x 2 bytes per row",
    }


def bench_precision(args):
    """Assembled 16-bit Sobolev block on a 32,768-edge knot: product bandwidth and
    the projected gradient solve to a relative FP64 residual of 1e-8."""
    import numpy as np
    import torch

    import gen
    from paper_2006_07859_amd import RC_C_BARYCENTER, RC_F32, RC_SOLVE_PCG_MG, Context, default_solve_opts

    n = 32768 if args.edges == 16384 else args.edges
    alpha, beta = 2.0, 4.5
    fmt = {"bf16": 1, "fp16": 2}[args.fmt]
    calibration_copy()
    g, e, _ = gen.fourier_knot(n, seed=0)
    g = gen.round_to_f32(g)
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    ctx = Context(n, e, alpha, beta, RC_F32)
    gamma = dev(g)
    ctx.rc_set_constraints(RC_C_BARYCENTER, gamma)
    E = torch.zeros(1, dtype=torch.float64, device="cuda")
    dE = torch.zeros(n, 3, dtype=torch.float64, device="cuda")
    out = torch.zeros_like(dE)
    so = default_solve_opts(solver=RC_SOLVE_PCG_MG, tol=1e-8, mg_min_vertices=256, cheb_degree=2, op_f64=1,
                            lowp=fmt, lowp_band=16, lowp_min_vertices=4096, lowp_outer=0, max_iter=300)

    def step():
        ctx.rc_differential(gamma, E, dE)
        return ctx.rc_sobolev_gradient(gamma, dE, out, so)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ctx.rc_profile_enable(True)
    stats = []
    t0 = time.perf_counter()
    for k in range(args.steps):
        st = step()
        stats.append(st)
        print(f"[bench] precision step {k}: pcg {st['iterations']} it, res {st['residual']:.2e}",
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    T = (time.perf_counter() - t0) / args.steps
    lp_ms, lp_n = ctx.rc_profile_read(2)
    ctx.rc_profile_enable(False)
    avg = lp_ms / max(lp_n, 1) * 1e-3
    bytes_per = n * n * 2  # algorithmic: every entry of the n x n block once, 2 bytes
    gbs = bytes_per / avg / 1e9

    # stand-alone products (the timed kernel alone) and the assembly
    X = dev(np.random.default_rng(1).normal(size=(n, 3)))
    Y = torch.zeros_like(X)
    torch.cuda.synchronize()
    ta = time.perf_counter()
    ctx.rc_lowp_assemble(gamma, fmt, 16, True)
    torch.cuda.synchronize()
    t_asm = time.perf_counter() - ta
    ctx.rc_profile_enable(True)
    for _ in range(20):
        ctx.rc_lowp_apply(X, Y)
        ctx.rc_lowp_apply(X, Y, True)
    m16, k16 = ctx.rc_profile_read(2)
    m32, k32 = ctx.rc_profile_read(3)
    ctx.rc_profile_enable(False)

    # the same solve with the FP64 matrix-free operator everywhere (plain multigrid PCG),
    # timed once, and its solution at a tighter residual for the error
    plain = default_solve_opts(solver=RC_SOLVE_PCG_MG, tol=1e-8, mg_min_vertices=256, cheb_degree=2, op_f64=1,
                               max_iter=300)
    ref = torch.zeros_like(dE)
    ctx.rc_differential(gamma, E, dE)
    torch.cuda.synchronize()
    tp = time.perf_counter()
    st_plain = ctx.rc_sobolev_gradient(gamma, dE, ref, plain)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - tp
    tight = default_solve_opts(solver=RC_SOLVE_PCG_MG, tol=2e-9, mg_min_vertices=256, op_f64=1, max_iter=400)
    ctx.rc_sobolev_gradient(gamma, dE, ref, tight)
    ctx.rc_sobolev_gradient(gamma, dE, out, so)
    err = (torch.linalg.norm(out - ref) / torch.linalg.norm(ref)).item()

    out_json = {
        "metric": "assembled-matvec HBM GB/s (16-bit Sobolev block x 3 columns, MFMA)",
        "value": gbs,
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": T * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.fmt,
        "data": "synthetic",
        "config": {"workload": f"fourier knot, {n} edges, (alpha,beta)=(2,4.5), barycenter constraint; one step = "
                               f"energy+differential, {args.fmt} block assembly (FP32 band 16), multigrid setup, "
                               f"projected PCG to 1e-8 FP64 residual with {args.fmt} smoothers on levels >= 4096 "
                               f"vertices and the FP64 matrix-free Krylov operator", "edges": n},
        "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": 8000.0, "unit": "GB/s",
                     "frac": round(gbs / 8000.0, 4), "traffic": traffic_record(f"k_lowp_gemv<{args.fmt}>", n),
                     "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                     "kernel": f"k_lowp_gemv<{args.fmt}> (finest level)", "launches": lp_n,
                     "avg_launch_ms": round(avg * 1e3, 4), "bytes_per_launch": bytes_per},
        "mfma_products_per_s": 1.0 / avg,
        "solve_to_1e-8": {"ms_per_step": T * 1e3, "pcg_iterations": [s["iterations"] for s in stats],
                          "refinement_sweeps": [s["sweeps"] for s in stats],
                          "residual": [s["residual"] for s in stats]},
        "plain_fp64_multigrid": {"ms": t_plain * 1e3, "pcg_iterations": st_plain["iterations"]},
        "error_vs_fp64": {"solution_rel": err, "reference": "FP64-operator multigrid PCG to 2e-9"},
        "assemble_ms": t_asm * 1e3,
        "product_kernels_ms": {f"{args.fmt}": m16 / max(k16, 1), "fp32": m32 / max(k32, 1)},
        "product_gbs": {f"{args.fmt}": bytes_per / (m16 / max(k16, 1) * 1e-3) / 1e9,
                        "fp32": 2 * bytes_per / (m32 / max(k32, 1) * 1e-3) / 1e9},
    }
    if not args.no_cpu_baseline:
        out_json["cpu_baseline"] = cpu_baseline_rows(g, e, alpha, beta)
    ctx.close()
    print(json.dumps(out_json))


def bench_batch(args):
    """512 packing instances (8-32 circles each, 200-8,000 edges, (alpha, beta) = (3, 6), sphere obstacle,
    barycenter + per-loop length constraints) stepped together; one step is one captured hipGraph."""
    import numpy as np
    import torch

    import gen
    from paper_2006_07859_amd import RC_F32, Batch, default_batch_opts

    alpha, beta = 3.0, 6.0
    insts = gen.packing_batch(512, seed=0)
    gs, es, voff, off = [], [], [0], 0
    for g, e, _ in insts:
        gs.append(g)
        es.append(np.asarray(e) + off)
        off += len(g)
        voff.append(off)
    g = np.concatenate(gs)
    e = np.concatenate(es).astype(np.int32)
    P = sum(ordered_disjoint_pairs(ei) for _, ei, _ in insts)
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    b = Batch(voff, e, alpha, beta, RC_F32)
    b.rc_set_obstacle((0.5, 0.5, 0.5), 0.25, 1.0)
    gamma = dev(g)
    tune = b.rc_batch_autotune(gamma, args.tune_cache)
    print(f"[bench] autotuned tiling {tune}", file=sys.stderr, flush=True)
    b.rc_batch_set_constraints(gamma)
    En = torch.zeros(512, dtype=torch.float64, device="cuda")
    dE = torch.zeros(len(g), 3, dtype=torch.float64, device="cuda")
    # energy + differential phase, kernel timed with HIP events
    b.rc_batch_energies(gamma, En, dE)
    b.rc_profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = 5
    for _ in range(reps):
        b.rc_batch_energies(gamma, En, dE)
    torch.cuda.synchronize()
    t_eval = (time.perf_counter() - t0) / reps
    tpe_ms, tpe_n = b.rc_profile_read(0)
    b.rc_profile_enable(False)
    tpe_avg = tpe_ms / max(tpe_n, 1) * 1e-3
    # captured steps
    opts = default_batch_opts(graph=1)
    for _ in range(args.warmup):
        b.rc_batch_step(gamma, opts, stats=False)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for k in range(args.steps):
        b.rc_batch_step(gamma, opts, stats=False)
    torch.cuda.synchronize()
    T = (time.perf_counter() - t1) / args.steps
    st = b.rc_batch_step(gamma, default_batch_opts(graph=1), stats=True)  # one more step, for its statistics
    ok = st[:, 5] == 0
    # the solves' operator alone: full-batch products with the assembled blocks, timed with HIP events
    Xr = dev(np.random.default_rng(2).normal(size=g.shape))
    Yr = torch.zeros_like(Xr)
    b.rc_batch_sobolev_apply(gamma, Xr, Yr, True)  # assembles at gamma
    b.rc_profile_enable(True)
    for _ in range(10):
        b.rc_batch_sobolev_apply(gamma, Xr, Yr, True)
    asm_ms, asm_n = b.rc_profile_read(5)
    b.rc_profile_enable(False)
    sizes = np.diff(np.asarray(voff)).astype(np.int64)
    asm_bytes = int((sizes * sizes).sum() * 4)  # every FP32 entry once
    asm_avg = asm_ms / max(asm_n, 1) * 1e-3
    asm_gbs = asm_bytes / asm_avg / 1e9
    achieved = FLOPS_PER_EDGE_PAIR * P / tpe_avg / 1e12  # (3, 6): the edge-pair form
    big = int(np.argmax(np.diff(voff)))
    out = {
        "metric": "aggregate edge-pair evals/s (energy+grad, 512-instance batch)",
        "value": P / t_eval,
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
        "config": {"workload": f"512 packing instances ({len(e)} edges, 8-32 circles each, 200-8,000 edges per "
                               f"instance), (alpha,beta)=(3,6), sphere obstacle, barycenter + per-loop length "
                               f"constraints; step = one captured hipGraph (energy, gradient by PCG on the "
                               f"assembled FP32 blocks with the two-level preconditioner, per-instance line search)", "edges": int(len(e)), "ordered_pairs": int(P)},
        "batch_steps_per_s": 1.0 / T,
        "energy_differential_ms": t_eval * 1e3,
        "tiling": tune,
        "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(achieved / PEAK_FP32_TFLOPS, 4), "traffic": None,
                     "kernel": "k_tpe_items<float> (persistent, energy+differential)", "launches": tpe_n,
                     "avg_launch_ms": round(tpe_avg * 1e3, 4)},
        "roofline_step_operator": {"bound": "hbm", "achieved": round(asm_gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                                   "frac": round(asm_gbs / PEAK_HBM_GBS, 4), "traffic": None,
                                   "kernel": "k_b_asm_apply (assembled per-instance FP32 blocks, whole batch)",
                                   "launches": asm_n, "avg_launch_ms": round(asm_avg * 1e3, 4),
                                   "bytes_per_launch": asm_bytes},
        "step_stats": {"accepted": int(ok.sum()), "pcg_iterations_mean": float(st[:, 3].mean()),
                       "pcg_iterations_max": float(st[:, 3].max()),
                       "energy_drop_mean": float(np.mean((st[ok, 0] - st[ok, 1]) / st[ok, 0]))},
    }
    if not args.no_cpu_baseline:
        gi, ei, _ = insts[big]
        out["cpu_baseline"] = cpu_baseline(gi, ei, alpha, beta)
        out["cpu_baseline"]["sample"] += f" (largest instance, {len(ei)} edges)"
    b.close()
    print(json.dumps(out))


def bench_learned(args):
    """Learned smoother weights of the multigrid V-cycle: (features, row l1 / diagonal
    ratio) rows of every smoothed level from snapshots of plain multigrid flows on
    knots of 1,024-4,096 edges, Adam regression on the GPU, then projected-gradient
    solves to 1e-6 on held-out knots of 4,096-16,384 edges: hand-set V-cycle
    (power-iteration interval), learned V-cycle (fixed interval), the untrained
    network (constant ratio 2.7) and Jacobi PCG, each the first solve on a fresh
    context (hierarchy built before the timed region), best of three."""
    import numpy as np
    import torch

    import gen
    from paper_2006_07859_amd import (RC_C_BARYCENTER, RC_F32, RC_SOLVE_PCG_JACOBI, RC_SOLVE_PCG_LEARNED,
                                      RC_SOLVE_PCG_MG, Context, Mlp, default_ls_opts, default_solve_opts)
    from paper_2006_07859_amd import _lib

    alpha, beta, n_min = 2.0, 4.5, 256
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")

    # data: snapshots along plain multigrid flows
    t0 = time.perf_counter()
    Xs, Rs = [], []
    snaps = 0
    knots = [(1024 * (1 + k % 4), 1000 + k) for k in range(args.train_knots)]
    for n, seed in knots:
        g, e, _ = gen.fourier_knot(n, seed=seed)
        c = Context(n, e, alpha, beta, RC_F32)
        gamma = dev(g)
        c.rc_set_constraints(RC_C_BARYCENTER, gamma)
        sizes = c.rc_learned_levels(128)
        N = sum(sizes)
        rows = N - sizes[-1]  # the smoothed levels
        for k in range(args.train_snapshots):
            X = torch.zeros(N, 8, dtype=torch.float32, device="cuda")
            R = torch.zeros(N, dtype=torch.float32, device="cuda")
            c.rc_learned_features(gamma, 128, X)
            c.rc_learned_targets(gamma, 128, R)
            Xs.append(X[:rows])
            Rs.append(R[:rows])
            snaps += 1
            if k + 1 < args.train_snapshots:
                c.rc_step(gamma, so=default_solve_opts(solver=RC_SOLVE_PCG_MG, tol=1e-6, mg_min_vertices=128),
                          ls=default_ls_opts())
        c.close()
        print(f"[bench] learned: knot n {n} seed {seed}: {args.train_snapshots} snapshots", file=sys.stderr,
              flush=True)
    X, R = torch.cat(Xs), torch.cat(Rs)
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    n_rows = int(X.shape[0])
    print(f"[bench] learned: {snaps} snapshots, {n_rows} rows in {t_data:.1f} s", file=sys.stderr, flush=True)

    # training: minibatch Adam regression
    theta0 = _init_params_host(_lib.mlp_n_params())
    mlp = Mlp(theta0)
    untrained = Mlp(theta0)
    g_t = torch.Generator(device="cuda").manual_seed(0)
    losses = []
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for it in range(args.train_steps):
        idx = torch.randint(0, n_rows, (args.batch_rows,), device="cuda", generator=g_t)
        losses.append(mlp.fit_step(X[idx].contiguous(), R[idx].contiguous(), 3e-3 if it < args.train_steps // 2 else 1e-3))
        if it % 200 == 0:
            print(f"[bench] learned: step {it} loss {losses[-1]:.5f}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t1
    head = float(np.mean(losses[:max(1, len(losses) // 10)]))
    tail = float(np.mean(losses[-max(1, len(losses) // 10):]))

    # held-out comparison
    kinds = [("multigrid", RC_SOLVE_PCG_MG, None), ("learned", RC_SOLVE_PCG_LEARNED, mlp),
             ("untrained", RC_SOLVE_PCG_LEARNED, untrained), ("jacobi", RC_SOLVE_PCG_JACOBI, None)]
    results, test_loss = {}, {}
    for n, seed in [(4096, 2001), (8192, 2002), (16384, 2003)]:
        g, e, _ = gen.fourier_knot(n, seed=seed)
        row = {}
        ref = None
        for name, kind, net in kinds:
            best, st_best = None, None
            for rep in range(3):
                c = Context(n, e, alpha, beta, RC_F32)
                gamma = dev(g)
                c.rc_set_constraints(RC_C_BARYCENTER, gamma)
                c.rc_learned_attach(net)
                sizes = c.rc_learned_levels(n_min)
                E = torch.zeros(1, dtype=torch.float64, device="cuda")
                dE = torch.zeros(n, 3, dtype=torch.float64, device="cuda")
                c.rc_differential(gamma, E, dE)
                if name == "learned" and rep == 0 and n <= 16384:
                    Nn = sum(sizes)
                    Xt = torch.zeros(Nn, 8, dtype=torch.float32, device="cuda")
                    Rt = torch.zeros(Nn, dtype=torch.float32, device="cuda")
                    c.rc_learned_features(gamma, n_min, Xt)
                    c.rc_learned_targets(gamma, n_min, Rt)
                    rows = Nn - sizes[-1]
                    test_loss[n] = {"trained": mlp.fit_step(Xt[:rows].contiguous(), Rt[:rows].contiguous(), 0.0),
                                    "untrained": untrained.fit_step(Xt[:rows].contiguous(), Rt[:rows].contiguous(),
                                                                    0.0)}
                out = torch.zeros_like(dE)
                so = default_solve_opts(solver=kind, tol=1e-6, mg_min_vertices=n_min, op_f64=1,
                                        max_iter=300 if kind == RC_SOLVE_PCG_JACOBI else 200, fallback_after=0)
                torch.cuda.synchronize()
                ts = time.perf_counter()
                st = c.rc_sobolev_gradient(gamma, dE, out, so, check=False)
                torch.cuda.synchronize()
                dt = (time.perf_counter() - ts) * 1e3
                if best is None or dt < best:
                    best, st_best = dt, st
                if name == "multigrid" and rep == 0:
                    ref = out.clone()
                err = (torch.linalg.norm(out - ref) / torch.linalg.norm(ref)).item()
                c.close()
            row[name] = {"iterations": int(st_best["iterations"]), "ms": round(best, 2),
                         "converged": st_best["status"] == 0, "residual": st_best["residual"],
                         "rel_diff_vs_multigrid": err}
            print(f"[bench] learned: n {n} {name}: {row[name]}", file=sys.stderr, flush=True)
        results[n] = row

    learned16 = results[16384]["learned"]
    value = 1e3 / learned16["ms"] if learned16["converged"] else 0.0
    out = {
        "metric": "projected-gradient solves/s to 1e-6 (learned V-cycle PCG, 16,384-edge knot)",
        "value": value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.train_steps,
        "warmup": 0,
        "ms_per_step": learned16["ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "fourier knots, (alpha,beta)=(2,4.5), barycenter constraint; training rows from "
                               "snapshots of plain multigrid flows on knots of 1,024-4,096 edges; held-out knots of "
                               "4,096, 8,192 and 16,384 edges solved to a relative FP64 residual of 1e-6, the first "
                               "solve on a fresh context, best of three",
                   "edges": 16384, "n_min": n_min},
        "training": {"snapshots": snaps, "rows": n_rows, "data_s": round(t_data, 2), "adam_steps": args.train_steps,
                     "batch_rows": args.batch_rows, "train_s": round(t_train, 2),
                     "loss_first_10pct": head, "loss_last_10pct": tail},
        "test_loss": {str(k): v for k, v in test_loss.items()},
        "comparison": {str(k): v for k, v in results.items()},
        "speedup_vs_multigrid": {str(k): round(v["multigrid"]["ms"] / v["learned"]["ms"], 3) for k, v in
                                 results.items()},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_solve(alpha, beta)
    mlp.close()
    untrained.close()
    print(json.dumps(out))


def _init_params_host(n_params):
    """Initial MLP parameters: He-scaled hidden layers (seeded), a small output
    layer and output bias log(expm1(1.7)), so that the network starts at the
    constant ratio 1 + 1.7."""
    import numpy as np

    rng = np.random.default_rng(0)
    f_in, w = 8, 64
    W1 = rng.normal(0.0, np.sqrt(2.0 / f_in), size=(f_in, w))
    W2 = rng.normal(0.0, np.sqrt(2.0 / w), size=(w, w))
    W3 = rng.normal(0.0, 0.01, size=w)
    theta = np.concatenate([W1.ravel(), np.zeros(w), W2.ravel(), np.zeros(w), W3, [np.log(np.expm1(1.7))]])
    assert theta.size == n_params
    return theta


def cpu_baseline_solve(alpha, beta, n=1024, seconds=12.0):
    """The FP64 oracle's projected gradient (dense assembly and saddle solve) on a
    smaller knot, repeated for a bounded time."""
    import gen
    from oracle import constraints as cons
    from oracle import solve, sobolev, tpe

    from threadpoolctl import threadpool_limits

    g, e, _ = gen.fourier_knot(n, seed=203)
    x0, _, _ = cons.reference_values(g, e)
    done, t0 = 0, time.perf_counter()
    with threadpool_limits(1):  # one BLAS thread, as reported
        while time.perf_counter() - t0 < seconds:
            A = sum(sobolev.assemble(g, e, alpha, beta))
            _, dE = tpe.differential(g, e, alpha, beta)
            _, C = cons.evaluate(g, e, cons.BARYCENTER, x0)
            solve.projected_gradient(A, C, dE)
            done += 1
    dt = time.perf_counter() - t0
    return {"value": done / dt, "unit": "solves/s", "cores": 1, "kind": "oracle",
            "sample": f"{done} dense FP64 projected-gradient solves (assembly, differential, saddle solve) on a "
                      f"{n}-edge knot, numpy, one thread"}


if __name__ == "__main__":
    main()
