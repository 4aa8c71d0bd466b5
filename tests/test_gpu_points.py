"""GPU parity of the point constraints of Sec. 7.1 (Phi = gamma_i - x_i).

Against the oracle: the values Phi, the Euclidean projector onto null(C)
(x - C^+ C x; the pins are eliminated, so the fused projector serves up to 8
rows of barycenter, total length and loop cuts, the general one above: a
packing of 8+ loops), with a pinned pair of neighbours whose edge-length row is
implied by the pins, the projected Sobolev gradient of eq.
GradientSaddlePointProblem from the dense, Jacobi-PCG, multigrid-PCG and
standalone multigrid solvers, and the step of Sec. 4.4 (dense solver: same
step length, energy and curve; multigrid: the pins land on moved targets
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


def pins(n, m):
    return np.array([3, n // 2 + 1, n - 5, n // 4][:m])


def make(g, e, a, b, dtype, mask, pv, px):
    from paper_2006_07859_amd import Context

    ctx = Context(len(g), e, a, b, dtype)
    ctx.rc_set_constraints(mask, dev(g))
    ctx.rc_set_point_constraints(pv, px)
    return ctx


def projector_ref(C, x):
    """x - C^+ C x, the orthogonal projector onto null(C) (C may have dependent rows)."""
    return x - np.linalg.pinv(C, rcond=1e-10) @ (C @ x)


@pytest.mark.parametrize("mask,pv", [(0, [3]), (BARY, [3]), (BARY | EDGE, [3]), (BARY | EDGE, [3, 151, 295, 75]),
                                     (TOTAL, [3, 151, 295, 75]), (BARY | EDGE, [40, 41, 120]), (EDGE, [0, 299]),
                                     (BARY | EDGE, [0, 1])])
def test_point_values_and_projector(lib, mask, pv):
    from paper_2006_07859_amd import RC_F64

    n = 300
    m = len(pv)
    pv = np.array(pv)
    banner(f"point constraints values/projector mask={mask} pins={pv.tolist()}")
    g, e = gen.trefoil(n, seed=2)
    px = g[pv] + 0.01 * np.random.default_rng(7).normal(size=(m, 3))
    ctx = make(g, e, 2.0, 4.0, RC_F64, mask, pv, px)
    refs = cons.reference_values(g, e)
    gp = g + 0.01 * np.random.default_rng(0).normal(size=g.shape)
    phi_ref, C = cons.evaluate(gp, e, mask, *refs, points=(pv, px))
    assert ctx.rc_constraint_count() == len(phi_ref)
    phi = zeros(ctx.rc_constraint_count())
    ctx.rc_constraint_values(dev(gp), phi)
    assert np.abs(host(phi) - phi_ref).max() < 1e-12 * (np.abs(phi_ref).max() + 1)
    X = np.random.default_rng(1).normal(size=g.shape)
    x = X.ravel()
    ref = projector_ref(C, x)
    Y = zeros(n, 3)
    ctx.rc_project(dev(gp), dev(X), Y)
    assert relnorm(host(Y).ravel(), ref) < 1e-11
    assert np.abs(host(Y)[pv]).max() == 0.0
    # re-setting the other constraints keeps the pins; removing the pins drops their rows
    ctx.rc_set_constraints(mask, dev(g))
    assert ctx.rc_constraint_count() == len(phi_ref)
    ctx.rc_set_point_constraints([], [])
    assert ctx.rc_constraint_count() == len(phi_ref) - 3 * m
    ctx.close()


def test_point_projector_many_loops(lib):
    """A packing of 8+ circles with barycenter and edge-length constraints: 3 + one cut row per
    loop exceed the fused projector's 8 border rows, so the general projector runs with the
    pins masked."""
    from paper_2006_07859_amd import RC_F64

    g, e, sizes = gen.packing_instance(np.random.default_rng(11), e_min=400, e_max=600)
    n = len(g)
    assert len(sizes) >= 6
    banner(f"point constraints general projector, {len(sizes)} loops, n={n}")
    pv = np.array([1, int(sizes[0]) + 2, n - 3])
    ctx = make(g, e, 2.0, 4.0, RC_F64, BARY | EDGE, pv, g[pv])
    gp = g + 1e-3 * np.random.default_rng(2).normal(size=g.shape)
    _, C = cons.evaluate(gp, e, BARY | EDGE, *cons.reference_values(g, e), points=(pv, g[pv]))
    X = np.random.default_rng(3).normal(size=g.shape)
    Y = zeros(n, 3)
    ctx.rc_project(dev(gp), dev(X), Y)
    assert relnorm(host(Y).ravel(), projector_ref(C, X.ravel())) < 1e-11
    assert np.abs(host(Y)[pv]).max() == 0.0
    ctx.close()


def test_point_argument_errors(lib):
    from paper_2006_07859_amd import RC_F64, RcError

    g, e = gen.trefoil(64, seed=2)
    ctx = make(g, e, 2.0, 4.0, RC_F64, BARY, [], [])
    for pv in ([64], [-1], [5, 5]):
        with pytest.raises(RcError):
            ctx.rc_set_point_constraints(pv, [g[0]] * len(pv))
    with pytest.raises(RcError):
        ctx.rc_set_point_constraints(list(range(65)), [g[0]] * 65)
    with pytest.raises(RcError):
        ctx.rc_set_point_constraints([3], [[0.0, np.nan, 0.0]])
    assert ctx.rc_constraint_count() == 3
    ctx.close()


def oracle_gradient(g, e, a, b, mask, pv, px):
    """The oracle's projected gradient; edge-length rows whose two ends are both pinned are
    implied by the point rows and are dropped first (the same constraint set, independent rows)."""
    refs = cons.reference_values(g, e)
    _, dE = tpe.differential(g, e, a, b)
    A = sum(sobolev.assemble(g, e, a, b))
    _, C = cons.evaluate(g, e, mask, *refs, points=(pv, px))
    if mask & EDGE:
        nd = 3 * (mask & BARY) + (1 if mask & TOTAL else 0) + 3 * len(pv)
        implied = [nd + i for i, (u, v) in enumerate(e) if u in set(pv) and v in set(pv)]
        C = np.delete(C, implied, axis=0)
    g_ref, _ = solve.projected_gradient(A, C, dE)
    return dE, C, g_ref


@pytest.mark.parametrize("mask,pv", [(BARY | EDGE, [3, 65]), (EDGE, [3, 65]), (0, [3, 65]), (BARY | EDGE, [10, 11])])
def test_point_gradient_dense_and_jacobi(lib, mask, pv):
    from paper_2006_07859_amd import RC_F64, RC_SOLVE_DENSE, RC_SOLVE_PCG_JACOBI, default_solve_opts

    n = 128
    pv = np.array(pv)
    banner(f"point-constrained gradient dense/jacobi n={n} mask={mask} pins={pv.tolist()}")
    g, e = gen.trefoil(n, seed=3)
    dE, C, g_ref = oracle_gradient(g, e, 2.0, 4.0, mask, pv, g[pv])
    ctx = make(g, e, 2.0, 4.0, RC_F64, mask, pv, g[pv])
    out = zeros(n, 3)
    ctx.rc_sobolev_gradient(dev(g), dev(dE), out, default_solve_opts(solver=RC_SOLVE_DENSE))
    assert relnorm(host(out), g_ref) < 1e-8
    st = ctx.rc_sobolev_gradient(dev(g), dev(dE), out,
                                 default_solve_opts(solver=RC_SOLVE_PCG_JACOBI, tol=1e-11, max_iter=6000))
    assert st["residual"] < 1e-11
    assert relnorm(host(out), g_ref) < 1e-7
    assert np.abs(host(out)[pv]).max() == 0.0
    ctx.close()


@pytest.mark.parametrize("mask,m,n", [(BARY | EDGE, 2, 2048), (EDGE, 1, 2048), (0, 2, 1024)])
def test_point_gradient_multigrid(lib, mask, m, n):
    """Multigrid PCG and the standalone multigrid with pins (the coarse levels pin the vertices
    a pinned vertex interpolates from), with barycenter and edge lengths, edge lengths, and pins
    alone."""
    from paper_2006_07859_amd import RC_F32, RC_SOLVE_MG_FMG, RC_SOLVE_PCG_MG, default_solve_opts

    banner(f"point-constrained multigrid gradient n={n} mask={mask} pins={m}")
    g, e, _ = gen.fourier_knot(n, seed=1)
    g = gen.round_to_f32(g)
    pv = pins(n, m)
    dE, C, g_ref = oracle_gradient(g, e, 2.0, 4.5, mask, pv, g[pv])
    ctx = make(g, e, 2.0, 4.5, RC_F32, mask, pv, g[pv])
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
    assert np.abs(C @ host(out).ravel()).max() < 1e-9 * np.abs(host(out)).max()
    ctx.close()


def test_point_step_dense_matches_oracle(lib):
    from paper_2006_07859_amd import RC_F64, RC_SOLVE_DENSE, default_solve_opts

    n = 256
    banner(f"point-constrained step dense trefoil{n}, edge lengths + 2 pins")
    g, e = gen.trefoil(n, seed=0)
    pv = pins(n, 2)
    refs = cons.reference_values(g, e)
    new_ref, info = solve.step(g, e, 2.0, 4.0, EDGE, refs, points=(pv, g[pv]))
    ctx = make(g, e, 2.0, 4.0, RC_F64, EDGE, pv, g[pv])
    gam = dev(g)
    st = ctx.rc_step(gam, so=default_solve_opts(solver=RC_SOLVE_DENSE))
    assert st["energy"] == pytest.approx(info["E0"], rel=1e-12)
    assert st["tau"] == info["tau"]
    assert st["energy_new"] == pytest.approx(info["E1"], rel=1e-10)
    assert relnorm(host(gam) - g, new_ref - g) < 1e-7
    assert np.abs(host(gam)[pv] - g[pv]).max() < 1e-10 * refs[2].mean()
    ctx.close()


def test_point_step_multigrid_moves_pins(lib):
    """Targets moved off the curve by a fraction of an edge: the step's
    projection puts the pins on them (one increment suffices for a linear
    constraint) while keeping the edge lengths."""
    from paper_2006_07859_amd import RC_F32, RC_SOLVE_PCG_MG, default_solve_opts

    n = 1024
    banner(f"point-constrained step multigrid fourier{n}, moved pins")
    g, e, _ = gen.fourier_knot(n, seed=2)
    g = gen.round_to_f32(g)
    pv = pins(n, 2)
    ell, _, _ = tpe.edge_geometry(g, e)
    px = g[pv] + 0.2 * ell.mean() * np.array([[1.0, 0.0, 0.0], [0.0, -1.0, 0.0]])
    ctx = make(g, e, 2.0, 4.5, RC_F32, EDGE, pv, px)
    gam = dev(g)
    st = ctx.rc_step(gam, so=default_solve_opts(solver=RC_SOLVE_PCG_MG, mg_min_vertices=256))
    new = host(gam)
    assert st["tau"] > 0
    phi, _ = cons.evaluate(new, e, EDGE, *cons.reference_values(g, e), jacobian=False, points=(pv, px))
    assert np.abs(phi).max() < 1e-8 * ell.mean()
    ctx.close()
