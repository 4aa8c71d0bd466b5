"""GPU parity of the surface constraints of Sec. 7.1 (Phi = f(gamma_i), f the signed
distance of a sphere or a torus).

Against the oracle: the values Phi, the Euclidean projector onto null(C) (held
vertices eliminated by the tangent-plane weights; with and without barycenter,
edge lengths and pinned vertices), the projected Sobolev gradient of eq.
GradientSaddlePointProblem from the dense, Jacobi-PCG, multigrid-PCG and
standalone multigrid solvers, and the step of Sec. 4.4 (dense: same step length,
energy and curve; multigrid: a jittered curve lands back on the torus).
"""

import numpy as np
import pytest

import gen
from oracle import constraints as cons
from oracle import solve, sobolev, tpe
from tests.gpu_util import banner, dev, host, relnorm, zeros

pytestmark = pytest.mark.gpu

BARY, TOTAL, EDGE = 1, 2, 4
SPHERE, TORUS = 1, 2


def curve(kind, n, **kw):
    if kind == SPHERE:
        g, e = gen.tennis_ball(n, **kw)
        return g, e, [0.0, 0.0, 0.0, 1.0]
    g, e = gen.torus_knot(n, **kw)
    return g, e, [0.0, 0.0, 0.0, 1.0, 0.4]


def make(g, e, a, b, dtype, mask, surf, pins=None):
    from paper_2006_07859_amd import Context

    ctx = Context(len(g), e, a, b, dtype)
    ctx.rc_set_constraints(mask, dev(g))
    if pins is not None:
        ctx.rc_set_point_constraints(*pins)
    ctx.rc_set_surface_constraints(*surf)
    return ctx


CASES = [(SPHERE, 0, "all"), (SPHERE, BARY, "all"), (SPHERE, BARY | EDGE, "all"), (TORUS, BARY | EDGE, "even"),
         (TORUS, EDGE, "even+pins"), (TORUS, TOTAL, "all")]


@pytest.mark.parametrize("kind,mask,which", CASES)
def test_surface_values_and_projector(lib, kind, mask, which):
    from paper_2006_07859_amd import RC_F64

    n = 300
    banner(f"surface constraints values/projector kind={kind} mask={mask} {which}")
    g, e, par = curve(kind, n)
    held = np.arange(n) if which == "all" else np.arange(0, n, 2)
    pins = (np.array([1, 151]), g[[1, 151]]) if which.endswith("pins") else None
    ctx = make(g, e, 2.0, 4.0, RC_F64, mask, (kind, par, held), pins)
    refs = cons.reference_values(g, e)
    gp = g + 0.01 * np.random.default_rng(0).normal(size=g.shape)
    phi_ref, C = cons.evaluate(gp, e, mask, *refs, points=pins, surface=(kind, par, held))
    assert ctx.rc_constraint_count() == len(phi_ref)
    phi = zeros(ctx.rc_constraint_count())
    ctx.rc_constraint_values(dev(gp), phi)
    assert np.abs(host(phi) - phi_ref).max() < 1e-12 * (np.abs(phi_ref).max() + 1)
    X = np.random.default_rng(1).normal(size=g.shape)
    x = X.ravel()
    ref = x - C.T @ np.linalg.solve(C @ C.T, C @ x)
    Y = zeros(n, 3)
    ctx.rc_project(dev(gp), dev(X), Y)
    assert relnorm(host(Y).ravel(), ref) < 1e-11
    _, nrm = cons.surface_value(kind, par, gp[held])
    assert np.abs((host(Y)[held] * nrm).sum(1)).max() < 1e-12 * np.abs(x).max()
    ctx.close()


def test_surface_argument_errors(lib):
    from paper_2006_07859_amd import RC_F64, RcError

    g, e, par = curve(TORUS, 64)
    ctx = make(g, e, 2.0, 4.0, RC_F64, BARY, (TORUS, par, [0, 2]), ([5], [g[5]]))
    bad = [(3, par, [0]), (TORUS, [0, 0, 0, 0.3, 0.4], [0]), (SPHERE, [0, 0, 0, -1.0], [0]),
           (TORUS, par, [64]), (TORUS, par, [2, 2]), (TORUS, par, [5]), (TORUS, [0, np.inf, 0, 1, 0.4], [0])]
    for b in bad:
        with pytest.raises(RcError):
            ctx.rc_set_surface_constraints(*b)
    with pytest.raises(RcError):
        ctx.rc_set_point_constraints([2], [g[2]])  # held on the torus
    assert ctx.rc_constraint_count() == 3 + 3 + 2
    ctx.rc_set_surface_constraints(0, [], [])
    assert ctx.rc_constraint_count() == 3 + 3
    ctx.close()


def oracle_gradient(g, e, a, b, mask, surf):
    refs = cons.reference_values(g, e)
    _, dE = tpe.differential(g, e, a, b)
    A = sum(sobolev.assemble(g, e, a, b))
    _, C = cons.evaluate(g, e, mask, *refs, surface=surf)
    g_ref, _ = solve.projected_gradient(A, C, dE)
    return dE, C, g_ref


@pytest.mark.parametrize("kind,mask", [(SPHERE, BARY | EDGE), (SPHERE, 0), (TORUS, EDGE)])
def test_surface_gradient_dense_and_jacobi(lib, kind, mask):
    from paper_2006_07859_amd import RC_F64, RC_SOLVE_DENSE, RC_SOLVE_PCG_JACOBI, default_solve_opts

    n = 128
    banner(f"surface-constrained gradient dense/jacobi kind={kind} mask={mask}")
    g, e, par = curve(kind, n)
    surf = (kind, par, np.arange(n))
    dE, C, g_ref = oracle_gradient(g, e, 2.0, 4.0, mask, surf)
    ctx = make(g, e, 2.0, 4.0, RC_F64, mask, surf)
    out = zeros(n, 3)
    ctx.rc_sobolev_gradient(dev(g), dev(dE), out, default_solve_opts(solver=RC_SOLVE_DENSE))
    assert relnorm(host(out), g_ref) < 1e-8
    st = ctx.rc_sobolev_gradient(dev(g), dev(dE), out,
                                 default_solve_opts(solver=RC_SOLVE_PCG_JACOBI, tol=1e-11, max_iter=6000))
    assert st["residual"] < 1e-11
    assert relnorm(host(out), g_ref) < 1e-7
    ctx.close()


@pytest.mark.parametrize("kind,mask,n", [(TORUS, BARY | EDGE, 2048), (SPHERE, BARY, 2048)])
def test_surface_gradient_multigrid(lib, kind, mask, n):
    from paper_2006_07859_amd import RC_F32, RC_SOLVE_MG_FMG, RC_SOLVE_PCG_MG, default_solve_opts

    banner(f"surface-constrained multigrid gradient kind={kind} mask={mask} n={n}")
    g, e, par = curve(kind, n)
    g = gen.round_to_f32(g)
    surf = (kind, par, np.arange(n))
    dE, C, g_ref = oracle_gradient(g, e, 2.0, 4.5, mask, surf)
    ctx = make(g, e, 2.0, 4.5, RC_F32, mask, surf)
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


def test_surface_step_dense_matches_oracle(lib):
    from paper_2006_07859_amd import RC_F64, RC_SOLVE_DENSE, default_solve_opts

    n = 128
    banner(f"surface-constrained step dense tennis ball n={n}, edge lengths")
    g, e, par = curve(SPHERE, n)
    surf = (SPHERE, par, np.arange(n))
    refs = cons.reference_values(g, e)
    new_ref, info = solve.step(g, e, 2.0, 4.0, EDGE, refs, surface=surf)
    ctx = make(g, e, 2.0, 4.0, RC_F64, EDGE, surf)
    gam = dev(g)
    st = ctx.rc_step(gam, so=default_solve_opts(solver=RC_SOLVE_DENSE))
    assert st["energy"] == pytest.approx(info["E0"], rel=1e-12)
    assert st["tau"] == info["tau"]
    assert st["energy_new"] == pytest.approx(info["E1"], rel=1e-10)
    assert relnorm(host(gam) - g, new_ref - g) < 1e-7
    ctx.close()


def test_surface_step_multigrid_returns_to_torus(lib):
    from paper_2006_07859_amd import RC_F32, RC_SOLVE_PCG_MG, default_solve_opts

    n = 1024
    banner(f"surface-constrained step multigrid torus knot n={n}, jittered off the torus")
    g, e, par = curve(TORUS, n, seed=3, jitter_var=1e-6)
    g = gen.round_to_f32(g)
    surf = (TORUS, par, np.arange(n))
    ctx = make(g, e, 2.0, 4.5, RC_F32, BARY, surf)
    gam = dev(g)
    st = ctx.rc_step(gam, so=default_solve_opts(solver=RC_SOLVE_PCG_MG, mg_min_vertices=256))
    assert st["tau"] > 0
    f, _ = cons.surface_value(TORUS, par, host(gam))
    ell, _, _ = tpe.edge_geometry(g, e)
    assert np.abs(f).max() < 1e-8 * ell.mean()
    ctx.close()
