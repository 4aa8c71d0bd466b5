"""Writes the oracle's energy, differential and projected Sobolev gradient of a
large Fourier knot to ``tests/golden/fourier<N>_seed<S>.npz``.

Calls only ``oracle/`` (and the seeded generator ``gen/``): the energy and
differential of eq. DiscreteEnergy / Sec. 4.1 (``oracle.tpe``), the rows of
A = B + B0 of Sec. 4.2 (``oracle.sobolev.assemble_rows``), the constraint
Jacobian of Sec. 7.1 (``oracle.constraints.jacobian_sparse``) and the saddle
solve of eq. GradientSaddlePointProblem through its structured Schur route
(``oracle.solve.projected_gradient_structured``).  The pair sums are spread
over a process pool by blocks of target edges / rows and added in block order.

The 16,384-edge knot (seed 0, (alpha, beta) = (2, 4.5), barycenter and edge
lengths) is the workload the benchmark measures; the 32,768-edge knot (seed 0,
barycenter only) is the precision-path workload.

    python tests/golden/make_fourier_knot.py --edges 16384 --constraints bary+edge
    python tests/golden/make_fourier_knot.py --edges 32768 --constraints bary

About 5 / 20 minutes on 8 cores, 8 / 20 GB of memory.
"""

from __future__ import annotations

import argparse
import hashlib
import multiprocessing as mp
import os
import sys
import tempfile
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import gen  # noqa: E402
from oracle import constraints as cons  # noqa: E402
from oracle import solve, sobolev, tpe  # noqa: E402

_G = None


def _init(args):
    global _G
    _G = args


def _energy_rows(r0, r1):
    g, e, a, b, _ = _G
    return tpe._block(g, e, a, b, np.arange(r0, r1), np.arange(len(e)), True)


def _a_rows(r0, r1):
    g, e, a, b, path = _G
    A = np.lib.format.open_memmap(path, mode="r+")
    A[r0:r1] = sobolev.assemble_rows(g, e, a, b, list(range(r0, r1)))
    A.flush()
    return r1 - r0


def input_hash(g, e):
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(g, dtype=np.float64).tobytes())
    h.update(np.ascontiguousarray(e, dtype=np.int32).tobytes())
    return h.hexdigest()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--edges", type=int, default=16384)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--alpha", type=float, default=2.0)
    ap.add_argument("--beta", type=float, default=4.5)
    ap.add_argument("--constraints", default="bary+edge", choices=["bary", "bary+edge"])
    ap.add_argument("--workers", type=int, default=min(8, os.cpu_count() or 1))
    args = ap.parse_args()
    n, a, b = args.edges, args.alpha, args.beta
    g, e, _ = gen.fourier_knot(n, seed=args.seed)
    g = gen.round_to_f32(g)
    mask = cons.BARYCENTER | (cons.EDGE_LENGTH if args.constraints == "bary+edge" else 0)
    tmp = tempfile.mkdtemp(prefix="rc_golden_")
    apath = os.path.join(tmp, "A.npy")
    np.lib.format.open_memmap(apath, mode="w+", dtype=np.float64, shape=(n, n)).flush()
    t0 = time.time()
    ctx = mp.get_context("fork")
    with ctx.Pool(args.workers, initializer=_init, initargs=((g, e, a, b, apath),)) as pool:
        blocks = [(r, min(n, r + 64)) for r in range(0, n, 64)]
        parts = pool.starmap(_energy_rows, blocks)
        E = float(sum(p[0] for p in parts))
        dE = np.zeros_like(g)
        for p in parts:
            dE += p[1]
        del parts
        print(f"energy + differential {time.time() - t0:.0f} s", flush=True)
        rows = [(r, min(n, r + 32)) for r in range(0, n, 32)]
        pool.starmap(_a_rows, rows)
        print(f"A {time.time() - t0:.0f} s", flush=True)
    A = np.array(np.load(apath, mmap_mode="r"))
    os.remove(apath)
    os.rmdir(tmp)
    x0 = cons.reference_values(g, e)[0]
    C = cons.jacobian_sparse(g, e, mask, x0)
    gt, lam = solve.projected_gradient_structured(A, C, dE)
    print(f"solve {time.time() - t0:.0f} s", flush=True)
    # checks of the saddle system itself (A applied in the difference form, as in the refinement)
    Ag = solve.apply_difference_form(A, gt)
    kkt = np.linalg.norm(Ag.ravel() + C.T @ lam - dE.ravel()) / np.linalg.norm(dE)
    feas = np.abs(C @ gt.ravel()).max() / np.abs(gt).max()
    descent = (float(np.sum(dE * gt)), float(np.sum(gt * Ag)))
    # the residual in the norm the library's solver stops on: ||P (dE - Abar g)|| / ||P dE||,
    # P = I - C^T (C C^T)^-1 C
    import scipy.sparse.linalg as spla

    lu = spla.splu((C @ C.T).tocsc())
    proj = lambda x: x - C.T @ lu.solve(C @ x)
    pres = np.linalg.norm(proj(dE.ravel() - Ag.ravel())) / np.linalg.norm(proj(dE.ravel()))
    print(f"E {E!r}  |dE| {np.linalg.norm(dE):.6g}  |g| {np.linalg.norm(gt):.6g}  KKT {kkt:.2e}  |Cg| {feas:.2e}  "
          f"projected residual {pres:.2e}  dE.g {descent[0]:.12g} g.Ag {descent[1]:.12g}", flush=True)
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"fourier{n}_seed{args.seed}.npz")
    np.savez(out, energy=np.array(E), dE=dE, g_tilde=gt, alpha=np.array(a), beta=np.array(b),
             mask=np.array(mask), input_sha256=np.array(input_hash(g, e)), kkt=np.array(kkt),
             projected_residual=np.array(pres))
    print(f"wrote {out}", flush=True)


if __name__ == "__main__":
    main()
