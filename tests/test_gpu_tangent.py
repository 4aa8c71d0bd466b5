"""GPU parity of the tangent constraints of Sec. 7.1, read as the two rows
(u . T_I, v . T_I) over a fixed basis of the plane orthogonal to the
prescribed direction.

Against the oracle: the values Phi, the Euclidean projector onto null(C) (two
rows per tangent in the projector's dense block: the fused projector up to 8
rows, the general one above; with pinned vertices), the projected Sobolev
gradient of eq. GradientSaddlePointProblem from the dense, Jacobi-PCG,
multigrid-PCG and standalone multigrid solvers, and the step of Sec. 4.4
(dense: same step length, energy and curve; multigrid: turned tangents reached
within the projection tolerance).
"""

import numpy as np
import pytest

import gen
from oracle import constraints as cons
from oracle import solve, sobolev, tpe
from tests.gpu_util import banner, dev, host, relnorm, zeros

pytestmark = pytest.mark.gpu

BARY, TOTAL, EDGE = 1, 2, 4


def turned(T, th, seed):
    """Unit directions at angle th from the rows of T."""
    r = np.random.default_rng(seed).normal(size=T.shape)
    r -= (r * T).sum(1, keepdims=True) * T
    r /= np.linalg.norm(r, axis=1, keepdims=True)
    return np.cos(th) * T + np.sin(th) * r


def make(g, e, a, b, dtype, mask, tang, pins=None):
    from paper_2006_07859_amd import Context

    ctx = Context(len(g), e, a, b, dtype)
    ctx.rc_set_constraints(mask, dev(g))
    if pins is not None:
        ctx.rc_set_point_constraints(*pins)
    ctx.rc_set_tangent_constraints(*tang)
    return ctx


@pytest.mark.parametrize("mask,tedges,with_pins", [(BARY, [5, 150], False), (BARY | EDGE, [5, 150], False),
                                                   (BARY | EDGE, [5, 150, 299], False), (EDGE, [5, 150], True),
                                                   (BARY | EDGE, list(range(3, 300, 15)), False)])
def test_tangent_values_and_projector(lib, mask, tedges, with_pins):
    """(The last case has 20 tangents: 3 + 40 + 1 border rows, more than the device inverts, so the
    border Schur complement is inverted on the host.)"""
    from paper_2006_07859_amd import RC_F64

    n = 300
    banner(f"tangent constraints values/projector mask={mask} edges={tedges} pins={with_pins}")
    g, e = gen.trefoil(n, seed=2)
    _, T, _ = tpe.edge_geometry(g, e)
    te = np.array(tedges)
    X = turned(T[te], 0.05, 1) * 2.0  # (any length)
    pins = (np.array([40, 200]), g[[40, 200]]) if with_pins else None
    ctx = make(g, e, 2.0, 4.0, RC_F64, mask, (te, X), pins)
    refs = cons.reference_values(g, e)
    gp = g + 0.01 * np.random.default_rng(0).normal(size=g.shape)
    phi_ref, C = cons.evaluate(gp, e, mask, *refs, points=pins, tangent=(te, X))
    assert ctx.rc_constraint_count() == len(phi_ref)
    phi = zeros(ctx.rc_constraint_count())
    ctx.rc_constraint_values(dev(gp), phi)
    assert np.abs(host(phi) - phi_ref).max() < 1e-12 * (np.abs(phi_ref).max() + 1)
    Xv = np.random.default_rng(1).normal(size=g.shape)
    x = Xv.ravel()
    ref = x - C.T @ np.linalg.solve(C @ C.T, C @ x)
    Y = zeros(n, 3)
    ctx.rc_project(dev(gp), dev(Xv), Y)
    assert relnorm(host(Y).ravel(), ref) < 1e-11
    ctx.close()


def test_tangent_argument_errors(lib):
    from paper_2006_07859_amd import RC_F64, RcError

    g, e = gen.trefoil(64, seed=2)
    ctx = make(g, e, 2.0, 4.0, RC_F64, BARY, ([3], [[1.0, 0.0, 0.0]]))
    for te, X in (([64], [[1, 0, 0]]), ([-1], [[1, 0, 0]]), ([2, 2], [[1, 0, 0], [0, 1, 0]]), ([2], [[0, 0, 0]]),
                  ([2], [[np.nan, 1, 0]])):
        with pytest.raises(RcError):
            ctx.rc_set_tangent_constraints(te, X)
    assert ctx.rc_constraint_count() == 3 + 2
    ctx.rc_set_tangent_constraints([], [])
    assert ctx.rc_constraint_count() == 3
    ctx.close()


def oracle_gradient(g, e, a, b, mask, tang):
    refs = cons.reference_values(g, e)
    _, dE = tpe.differential(g, e, a, b)
    A = sum(sobolev.assemble(g, e, a, b))
    _, C = cons.evaluate(g, e, mask, *refs, tangent=tang)
    g_ref, _ = solve.projected_gradient(A, C, dE)
    return dE, C, g_ref


@pytest.mark.parametrize("mask", [BARY | EDGE, BARY])
def test_tangent_gradient_dense_and_jacobi(lib, mask):
    from paper_2006_07859_amd import RC_F64, RC_SOLVE_DENSE, RC_SOLVE_PCG_JACOBI, default_solve_opts

    n = 128
    banner(f"tangent-constrained gradient dense/jacobi mask={mask}")
    g, e = gen.trefoil(n, seed=3)
    _, T, _ = tpe.edge_geometry(g, e)
    tang = (np.array([0, 64]), T[[0, 64]])
    dE, C, g_ref = oracle_gradient(g, e, 2.0, 4.0, mask, tang)
    ctx = make(g, e, 2.0, 4.0, RC_F64, mask, tang)
    out = zeros(n, 3)
    ctx.rc_sobolev_gradient(dev(g), dev(dE), out, default_solve_opts(solver=RC_SOLVE_DENSE))
    assert relnorm(host(out), g_ref) < 1e-8
    st = ctx.rc_sobolev_gradient(dev(g), dev(dE), out,
                                 default_solve_opts(solver=RC_SOLVE_PCG_JACOBI, tol=1e-11, max_iter=6000))
    assert st["residual"] < 1e-11
    assert relnorm(host(out), g_ref) < 1e-7
    ctx.close()


def test_tangent_gradient_multigrid(lib):
    from paper_2006_07859_amd import RC_F32, RC_SOLVE_MG_FMG, RC_SOLVE_PCG_MG, default_solve_opts

    n = 2048
    banner(f"tangent-constrained multigrid gradient n={n}, barycenter + edge lengths + 2 tangents")
    g, e, _ = gen.fourier_knot(n, seed=1)
    g = gen.round_to_f32(g)
    _, T, _ = tpe.edge_geometry(g, e)
    tang = (np.array([3, 1001]), T[[3, 1001]])
    dE, C, g_ref = oracle_gradient(g, e, 2.0, 4.5, BARY | EDGE, tang)
    ctx = make(g, e, 2.0, 4.5, RC_F32, BARY | EDGE, tang)
    out = zeros(n, 3)
    st = ctx.rc_sobolev_gradient(dev(g), dev(dE), out,
                                 default_solve_opts(solver=RC_SOLVE_PCG_MG, tol=1e-9, op_f64=1, mg_min_vertices=256,
                                                    max_iter=400))
    print(f"  PCG-MG: {st['iterations']} iterations")
    assert relnorm(host(out), g_ref) < 1e-6
    assert st["iterations"] < 60
    st = ctx.rc_sobolev_gradient(dev(g), dev(dE), out,
                                 default_solve_opts(solver=RC_SOLVE_MG_FMG, tol=1e-8, op_f64=1, cheb_degree=6,
                                                    max_iter=400, mg_min_vertices=256))
    print(f"  FMG: {st['iterations']} V-cycles")
    assert relnorm(host(out), g_ref) < 1e-5
    ctx.close()


def test_tangent_step_dense_matches_oracle(lib):
    from paper_2006_07859_amd import RC_F64, RC_SOLVE_DENSE, default_solve_opts

    n = 128
    banner(f"tangent-constrained step dense trefoil{n}")
    g, e = gen.trefoil(n, seed=0)
    _, T, _ = tpe.edge_geometry(g, e)
    tang = (np.array([0, 64]), T[[0, 64]])
    refs = cons.reference_values(g, e)
    new_ref, info = solve.step(g, e, 2.0, 4.0, BARY | EDGE, refs, tangent=tang)
    ctx = make(g, e, 2.0, 4.0, RC_F64, BARY | EDGE, tang)
    gam = dev(g)
    st = ctx.rc_step(gam, so=default_solve_opts(solver=RC_SOLVE_DENSE))
    assert st["energy"] == pytest.approx(info["E0"], rel=1e-12)
    assert st["tau"] == info["tau"]
    assert st["energy_new"] == pytest.approx(info["E1"], rel=1e-10)
    assert relnorm(host(gam) - g, new_ref - g) < 1e-7
    ctx.close()


def test_tangent_step_multigrid_turns_tangents(lib):
    from paper_2006_07859_amd import RC_F32, RC_SOLVE_PCG_MG, default_solve_opts

    n = 1024
    banner(f"tangent-constrained step multigrid fourier{n}, tangents turned by 0.02 rad")
    g, e, _ = gen.fourier_knot(n, seed=2)
    g = gen.round_to_f32(g)
    _, T, _ = tpe.edge_geometry(g, e)
    te = np.array([10, 500])
    X = turned(T[te], 0.02, 5)
    ctx = make(g, e, 2.0, 4.5, RC_F32, BARY | EDGE, (te, X))
    gam = dev(g)
    st = ctx.rc_step(gam, so=default_solve_opts(solver=RC_SOLVE_PCG_MG, mg_min_vertices=256))
    assert st["tau"] > 0
    _, T1, _ = tpe.edge_geometry(host(gam), e)
    assert np.abs(T1[te] - X).max() < 1e-8
    ctx.close()
