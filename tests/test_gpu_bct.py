"""Hierarchical product on a block cluster tree (App. B.2) against the oracle's
kernel-matrix form of A = B + B0 (App. B.3.4, oracle/sobolev.kernel_matrix_apply).

* theta -> 0: every block is a leaf summed exactly, so the product equals the
  kernel-matrix form to FP64 rounding (the parity of the approximation's
  limit);
* the error against it falls as theta falls (the approximation's own error,
  which the paper does not print: measured and bounded here);
* the approximate matrices are symmetric and annihilate constants for every
  theta (symmetric admissibility and kernels; the diagonal from the same row
  sums).
"""

import numpy as np
import pytest

import gen
from oracle import sobolev
from tests.gpu_util import banner, dev, host, relnorm, zeros

pytestmark = pytest.mark.gpu


def network():
    g1, e1, _ = gen.fourier_knot(500, seed=11)
    g2, e2, _ = gen.fourier_knot(300, seed=12)
    g2 = 0.5 * g2 + [3.0, 0.0, 0.0]
    t = np.linspace(0.0, 1.0, 201)
    g3 = np.stack([0.4 * np.cos(6 * t) - 3.0, 0.4 * np.sin(6 * t), 2.0 * t], 1)
    e3 = np.stack([np.arange(200), np.arange(1, 201)], 1)
    g = np.concatenate([g1, g2, g3])
    e = np.concatenate([e1, e2 + 500, e3 + 800]).astype(np.int32)
    return g, e


def oracle_apply(g, e, a, b, X):
    return np.stack([sobolev.kernel_matrix_apply(g, e, a, b, X[:, c]) for c in range(3)], 1)


def bct_apply(ctx, g, X, theta, leaf=32):
    gam = dev(g)
    ctx.rc_bct_build(gam, theta, leaf)
    Y = zeros(len(g), 3)
    ctx.rc_sobolev_apply_bct(gam, dev(X), Y)
    return host(Y), ctx.rc_bct_stats()


@pytest.mark.parametrize("alpha,beta", [(2.0, 4.5), (3.0, 6.0)])
def test_bct_limit_and_error_curve(lib, alpha, beta):
    from paper_2006_07859_amd import RC_F32, Context

    banner(f"block cluster tree product vs kernel-matrix form ({alpha},{beta})")
    g, e = network()
    X = np.random.default_rng(1).normal(size=g.shape)
    t = np.linspace(0, 1, len(g))
    Xs = np.stack([np.cos(2 * np.pi * t), np.sin(4 * np.pi * t), t * t], 1)  # smooth
    ctx = Context(len(g), e, alpha, beta, RC_F32)
    for name, V in (("random", X), ("smooth", Xs)):
        ref = oracle_apply(g, e, alpha, beta, V)
        Y0, st0 = bct_apply(ctx, g, V, 1e-6)
        assert st0["far_blocks"] == 0
        err0 = relnorm(Y0, ref)
        errs = []
        for theta in (0.1, 0.25, 0.5):
            Y, st = bct_apply(ctx, g, V, theta)
            errs.append(relnorm(Y, ref))
            print(f"  {name} theta {theta}: rel {errs[-1]:.2e}  far blocks {st['far_blocks']} near pairs "
                  f"{st['near_pairs']}")
        print(f"  {name} theta 1e-6 (all leaves exact): rel {err0:.2e}")
        assert err0 < 1e-12
        assert errs[0] < errs[1] < errs[2]
        assert errs[1] < 5e-2
    ctx.close()


def test_bct_symmetric_and_annihilates_constants(lib):
    from paper_2006_07859_amd import RC_F32, Context

    banner("block cluster tree product: symmetry and constants")
    g, e = network()
    rng = np.random.default_rng(2)
    U, V = rng.normal(size=g.shape), rng.normal(size=g.shape)
    ctx = Context(len(g), e, 2.0, 4.5, RC_F32)
    AU, _ = bct_apply(ctx, g, U, 0.5)
    AV, _ = bct_apply(ctx, g, V, 0.5)
    assert np.sum(V * AU) == pytest.approx(np.sum(U * AV), rel=1e-11)
    A1, _ = bct_apply(ctx, g, np.ones_like(U), 0.5)
    assert np.abs(A1).max() < 1e-10 * np.abs(AU).max()
    assert np.sum(U * AU) > 0
    ctx.close()


def test_bct_error_curve_32k(lib):
    """At 32,768 edges, against the same product with every block summed exactly (theta -> 0)."""
    import time

    import torch

    from paper_2006_07859_amd import RC_F32, Context

    n = 32768
    banner(f"block cluster tree error curve, fourier knot {n} edges")
    g, e, _ = gen.fourier_knot(n, seed=0)
    g = gen.round_to_f32(g)
    t = 2 * np.pi * np.arange(n) / n
    X = np.stack([np.cos(t), np.sin(2 * t), np.cos(3 * t)], 1) + 1e-3 * np.random.default_rng(3).normal(size=(n, 3))
    ctx = Context(n, e, 2.0, 4.5, RC_F32)
    ref, _ = bct_apply(ctx, g, X, 1e-6)
    prev, errs = None, {}
    for theta in (0.1, 0.25, 0.5):
        gam = dev(g)
        ctx.rc_bct_build(gam, theta, 32)
        Y = zeros(n, 3)
        Xd = dev(X)
        ctx.rc_sobolev_apply_bct(gam, Xd, Y)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(5):
            ctx.rc_sobolev_apply_bct(gam, Xd, Y)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / 5 * 1e3
        err = relnorm(host(Y), ref)
        st = ctx.rc_bct_stats()
        print(f"  theta {theta}: rel {err:.2e}  {ms:.2f} ms per product  far blocks {st['far_blocks']} near pairs "
              f"{st['near_pairs']} ({st['near_pairs'] / (n * n):.3%} of all pairs)")
        if prev is not None:
            assert err > prev
        prev = errs[theta] = err
    assert errs[0.1] < 1e-4 and errs[0.25] < 5e-3
    ctx.close()


def test_bct_projected_gradient_limit(lib):
    """The multigrid PCG solve with every smoothed level's operator on its own
    block cluster tree: as theta -> 0 its projected gradient is the oracle's
    dense saddle solution for the kernel-matrix form of A (eq.
    GradientSaddlePointProblem with A of App. B.3.4); at theta > 0 the gap
    follows the operator's error."""
    from paper_2006_07859_amd import (RC_C_BARYCENTER, RC_C_EDGE_LENGTH, RC_F32, RC_SOLVE_PCG_MG, Context,
                                      default_solve_opts)
    from oracle import constraints as cons
    from oracle import solve, tpe

    n, a, b = 2048, 2.0, 4.5
    banner(f"projected gradient on the block cluster tree, fourier knot {n} edges")
    g, e, _ = gen.fourier_knot(n, seed=0)
    g = gen.round_to_f32(g)
    mask = RC_C_BARYCENTER | RC_C_EDGE_LENGTH
    refs = cons.reference_values(g, e)
    _, dE = tpe.differential(g, e, a, b)
    A = sum(sobolev.assemble(g, e, a, b, quadrature="midpoint"))
    _, C = cons.evaluate(g, e, mask, *refs)
    g_ref, _ = solve.projected_gradient_structured(A, C, dE)
    ctx = Context(n, e, a, b, RC_F32)
    gam = dev(g)
    ctx.rc_set_constraints(mask, gam)
    errs = {}
    for theta in (1e-6, 0.1, 0.25):
        so = default_solve_opts(solver=RC_SOLVE_PCG_MG, tol=1e-10, mg_min_vertices=256, cheb_degree=2, op_f64=1,
                                max_iter=300, bct_theta=theta, bct_min_vertices=512)
        out = zeros(n, 3)
        st = ctx.rc_sobolev_gradient(gam, dev(dE), out, so)
        errs[theta] = relnorm(host(out), g_ref)
        print(f"  theta {theta}: {st['iterations']} iterations, res {st['residual']:.1e}, rel error {errs[theta]:.2e}")
    assert errs[1e-6] < 1e-7
    assert errs[0.1] < errs[0.25] < 2e-2
    ctx.close()


def test_bct_step_262k(lib):
    """A full projected Sobolev step at 262,144 edges with the paper's
    large-curve approximations (App. B): Barnes-Hut energy and differential
    (theta 0.25), multigrid PCG on the block cluster tree operator (theta 0.25)
    to 1e-6, projected line search with edge-length and barycenter restoration
    and Barnes-Hut trial energies: the step's energy is the Barnes-Hut energy
    at the curve, it falls, and the constraints hold at the new curve."""
    import time

    import torch

    from paper_2006_07859_amd import (RC_C_BARYCENTER, RC_C_EDGE_LENGTH, RC_F32, RC_SOLVE_PCG_MG, Context,
                                      default_ls_opts, default_solve_opts)

    n = 262144
    banner(f"projected Sobolev step on the block cluster tree, fourier knot {n} edges")
    g, e, _ = gen.fourier_knot(n, seed=0)
    g = gen.round_to_f32(g)
    ctx = Context(n, e, 2.0, 4.5, RC_F32)
    gam = dev(g)
    ctx.rc_set_constraints(RC_C_BARYCENTER | RC_C_EDGE_LENGTH, gam)
    so = default_solve_opts(solver=RC_SOLVE_PCG_MG, tol=1e-6, mg_min_vertices=256, cheb_degree=2, op_f64=1,
                            max_iter=200, bct_theta=0.25, bct_min_vertices=16384)
    ls = default_ls_opts(bh_theta=0.25)
    E_bh = torch.zeros(1, dtype=torch.float64, device="cuda")
    ctx.rc_bh_differential(dev(g), 0.25, 32, E_bh, zeros(n, 3))
    for k in range(2):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = ctx.rc_step(gam, so=so, ls=ls)
        if k == 0:
            assert st["energy"] == pytest.approx(float(E_bh.item()), rel=1e-12)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        print(f"  step {k}: {ms:.0f} ms  E {st['energy']:.8g} -> {st['energy_new']:.8g}  pcg {st['iterations']} it  "
              f"res {st['residual']:.1e}  tau {st['tau']:.3g}  eval {st['t_eval_ms']:.1f} ms  solve "
              f"{st['t_solve_ms']:.1f} ms  search {st['t_search_ms']:.1f} ms")
        assert st["energy_new"] < st["energy"]
        assert st["residual"] <= 1e-6
    phi = zeros(ctx.rc_constraint_count())
    ctx.rc_constraint_values(gam, phi)
    lbar = float(np.mean(np.linalg.norm(g[e[:, 1]] - g[e[:, 0]], axis=1)))
    assert np.abs(host(phi)[3:]).max() < 1e-9 * lbar  # the line search projects to 1e-10 mean edge lengths
    ctx.close()
