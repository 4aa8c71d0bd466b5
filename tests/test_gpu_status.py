"""The device-latched status word and rc_sync_status (C ABI conventions).

Each condition is forced from the host with a curve or an option that
produces it; no kernel faults.  A zero-length edge leaves T_I undefined
(Sec. 4, Notation); coincident vertices of disjoint edges make a pair's
kernel |T x d|^alpha / |d|^beta, and the energy (Sec. 4.1, Lemma
FiniteTangentPointEnergy), infinite.  The kernels latch these without
stopping the stream; the solver calls latch their own failures.
"""

import numpy as np
import pytest

import gen
from tests.gpu_util import banner, dev, zeros

pytestmark = pytest.mark.gpu

OK, DEGENERATE, NONFINITE, NOT_CONVERGED, PROJECTION, LINESEARCH = 0, 3, 4, 5, 6, 7


def flags():
    from paper_2006_07859_amd import _lib

    return _lib


@pytest.mark.parametrize("dtype", [0, 1])
def test_device_conditions_latch_and_clear(lib, dtype):
    from paper_2006_07859_amd import Context

    F = flags()
    g, e = gen.trefoil(256, seed=1)
    n = len(g)
    ctx = Context(n, e, 2.0, 4.5, dtype)
    E, dE = zeros(1), zeros(n, 3)

    banner(f"status clean dtype={dtype}")
    ctx.rc_differential(dev(g), E, dE)
    assert ctx.rc_sync_status() == (OK, 0)

    # coincident vertices of disjoint edges: one near along the loop (the FP64
    # band in FP32 contexts), one far apart (the FP32 tiles)
    for v, w in ((10, 30), (10, 140)):
        banner(f"status coincident vertices {v},{w} dtype={dtype}")
        gc = g.copy()
        gc[w] = gc[v]
        ctx.rc_differential(dev(gc), E, dE)
        st, f = ctx.rc_sync_status()
        assert st == DEGENERATE and f & F.RC_FLAG_PAIR_OVERFLOW, (st, f)
        assert not f & (F.RC_FLAG_ZERO_EDGE | F.RC_FLAG_INPUT_NONFINITE)
        # the word was cleared by the read
        assert ctx.rc_sync_status() == (OK, 0)

    banner(f"status zero-length edge dtype={dtype}")
    gz = g.copy()
    gz[11] = gz[10]
    ctx.rc_energy(dev(gz), E)
    st, f = ctx.rc_sync_status()
    assert st == DEGENERATE and f & F.RC_FLAG_ZERO_EDGE, (st, f)

    banner(f"status non-finite input dtype={dtype}")
    gn = g.copy()
    gn[5, 1] = np.nan
    ctx.rc_differential(dev(gn), E, dE)
    st, f = ctx.rc_sync_status()
    assert st == NONFINITE and f & F.RC_FLAG_INPUT_NONFINITE, (st, f)

    banner(f"status several calls before one read dtype={dtype}")
    ctx.rc_differential(dev(g), E, dE)
    ctx.rc_energy(dev(gz), E)
    ctx.rc_differential(dev(g), E, dE)
    st, f = ctx.rc_sync_status()
    assert st == DEGENERATE and f & F.RC_FLAG_ZERO_EDGE
    ctx.rc_differential(dev(g), E, dE)
    assert ctx.rc_sync_status() == (OK, 0)
    ctx.close()


def test_solver_conditions_latch(lib):
    from paper_2006_07859_amd import (RC_C_BARYCENTER, RC_C_EDGE_LENGTH, RC_F64, RC_SOLVE_DENSE, RC_SOLVE_PCG_JACOBI,
                                      Context, default_ls_opts, default_solve_opts)

    F = flags()
    g, e = gen.trefoil(96, seed=3)
    n = len(g)
    ctx = Context(n, e, 2.0, 4.0, RC_F64)
    E, dE, gt = zeros(1), zeros(n, 3), zeros(n, 3)
    ctx.rc_differential(dev(g), E, dE)

    banner("status not converged")
    ctx.rc_set_constraints(RC_C_BARYCENTER, dev(g))
    st = ctx.rc_sobolev_gradient(dev(g), dE, gt, default_solve_opts(solver=RC_SOLVE_PCG_JACOBI, tol=1e-14,
                                                                     max_iter=3), check=False)
    assert st["status"] == NOT_CONVERGED
    s, f = ctx.rc_sync_status()
    assert s == NOT_CONVERGED and f == F.RC_FLAG_NOT_CONVERGED, (s, f)

    dense = default_solve_opts(solver=RC_SOLVE_DENSE)
    ctx.rc_sobolev_gradient(dev(g), dE, gt, dense)
    assert ctx.rc_sync_status() == (OK, 0)

    banner("status projection")
    # edge-length constraints with no projection iteration allowed: no trial
    # step keeps every edge length, so the projection fails at every length
    ctx.rc_set_constraints(RC_C_BARYCENTER | RC_C_EDGE_LENGTH, dev(g))
    ctx.rc_sobolev_gradient(dev(g), dE, gt, dense)
    from paper_2006_07859_amd._lib import RcError

    with pytest.raises(RcError) as ei:
        ctx.rc_line_search_step(dev(g), E.item(), dE, gt, ls=default_ls_opts(max_proj_iter=0, max_backtracks=2),
                                so=dense)
    assert ei.value.status == PROJECTION
    s, f = ctx.rc_sync_status()
    assert s == PROJECTION and f == F.RC_FLAG_PROJECTION, (s, f)

    banner("status line search")
    # the projections succeed but no length meets an impossible Armijo constant
    with pytest.raises(RcError) as ei:
        ctx.rc_line_search_step(dev(g), E.item(), dE, gt, ls=default_ls_opts(c_armijo=1e6, max_backtracks=2),
                                so=dense)
    assert ei.value.status == LINESEARCH
    s, f = ctx.rc_sync_status()
    assert s == LINESEARCH and f == F.RC_FLAG_LINESEARCH, (s, f)
    ctx.close()


def test_constraint_setup_failure_reported(lib):
    """A constraint factorisation that breaks down is latched on the device during the set-up and
    reported by the call that prepared it: a non-finite vertex makes a pivot of the edge-length rows'
    tridiagonal block NaN, so rc_project and the multigrid gradient (whose set-up enqueues every
    level's factors without waiting) return RC_ERR_SINGULAR; the next call at a valid curve succeeds
    (the latch is cleared)."""
    from paper_2006_07859_amd import (RC_C_BARYCENTER, RC_C_EDGE_LENGTH, RC_F32, RC_SOLVE_PCG_MG, Context,
                                      default_solve_opts)
    from paper_2006_07859_amd._lib import RcError

    SINGULAR = 8
    g, e, _ = gen.fourier_knot(1024, seed=1)
    g = gen.round_to_f32(g)
    n = len(g)
    bad = g.copy()
    bad[100] = np.nan
    banner("constraint set-up failure: rc_project and multigrid gradient at a non-finite vertex")
    ctx = Context(n, e, 2.0, 4.5, RC_F32)
    ctx.rc_set_constraints(RC_C_BARYCENTER | RC_C_EDGE_LENGTH, dev(g))
    X, Y = dev(np.random.default_rng(0).normal(size=(n, 3))), zeros(n, 3)
    with pytest.raises(RcError) as ei:
        ctx.rc_project(dev(bad), X, Y)
    assert ei.value.status == SINGULAR
    ctx.rc_project(dev(g), X, Y)
    assert np.isfinite(Y.cpu().numpy()).all()
    E, dE, gt = zeros(1), zeros(n, 3), zeros(n, 3)
    ctx.rc_differential(dev(g), E, dE)
    so = default_solve_opts(solver=RC_SOLVE_PCG_MG, tol=1e-6, mg_min_vertices=256)
    with pytest.raises(RcError) as ei:
        ctx.rc_sobolev_gradient(dev(bad), dE, gt, so)
    assert ei.value.status == SINGULAR
    st = ctx.rc_sobolev_gradient(dev(g), dE, gt, so)
    assert st["residual"] < 1e-6
    ctx.rc_sync_status()  # clears the non-finite input flag latched by the failed calls
    ctx.close()
