"""GPU parity of constraints, projection, projected Sobolev gradient and step.

Compared with the FP64 oracle's dense saddle solves (eqs.
GradientSaddlePointProblem, ConstraintSaddlePointProblem) and its backtracking
step (Sec. 4.4).  The projected gradient is unique when A is definite on
null(C), so the solvers must agree with the oracle's solution.
"""

import numpy as np
import pytest

import gen
from oracle import constraints as cons
from oracle import solve, sobolev, tpe
from tests.gpu_util import banner, dev, host, relnorm, zeros

pytestmark = pytest.mark.gpu

BARY, TOTAL, EDGE = 1, 2, 4


def make(lib, g, e, a, b, dtype, mask):
    from paper_2006_07859_amd import Context

    ctx = Context(len(g), e, a, b, dtype)
    ctx.rc_set_constraints(mask, dev(g))
    return ctx


def oracle_system(g, e, a, b, mask):
    refs = cons.reference_values(g, e)
    E, dE = tpe.differential(g, e, a, b)
    A = sum(sobolev.assemble(g, e, a, b))
    phi, C = cons.evaluate(g, e, mask, *refs)
    return refs, E, dE, A, phi, C


@pytest.mark.parametrize("mask", [BARY, BARY | EDGE, BARY | TOTAL, EDGE])
def test_constraint_values_and_projector(lib, mask):
    from paper_2006_07859_amd import RC_F64

    banner(f"constraints mask={mask}")
    g, e = gen.trefoil(150, seed=2)
    ctx = make(lib, g, e, 2.0, 4.0, RC_F64, mask)
    refs = cons.reference_values(g, e)
    # values at a perturbed curve
    gp = g + 0.01 * np.random.default_rng(0).normal(size=g.shape)
    phi_ref, C = cons.evaluate(gp, e, mask, *refs)
    phi = zeros(ctx.rc_constraint_count())
    ctx.rc_constraint_values(dev(gp), phi)
    assert np.abs(host(phi) - phi_ref).max() < 1e-12 * (np.abs(phi_ref).max() + 1)
    # projector P = I - C^T (C C^T)^-1 C at gp
    X = np.random.default_rng(1).normal(size=g.shape)
    x = X.ravel()
    ref = x - C.T @ np.linalg.solve(C @ C.T, C @ x)
    Y = zeros(len(g), 3)
    ctx.rc_project(dev(gp), dev(X), Y)
    assert relnorm(host(Y).ravel(), ref) < 1e-11
    assert np.abs(C @ host(Y).ravel()).max() < 1e-10 * np.abs(x).max()


@pytest.mark.parametrize("mask", [BARY, BARY | EDGE])
def test_dense_gradient_c1(lib, mask):
    from paper_2006_07859_amd import RC_F64, RC_SOLVE_DENSE, default_solve_opts

    banner(f"dense projected gradient trefoil256 mask={mask}")
    g, e = gen.trefoil(256, seed=0)
    refs, E, dE, A, phi, C = oracle_system(g, e, 2.0, 4.0, mask)
    g_ref, _ = solve.projected_gradient(A, C, dE)
    ctx = make(lib, g, e, 2.0, 4.0, RC_F64, mask)
    out = zeros(256, 3)
    ctx.rc_sobolev_gradient(dev(g), dev(dE), out, default_solve_opts(solver=RC_SOLVE_DENSE))
    assert relnorm(host(out), g_ref) < 1e-8


def test_pcg_jacobi_small(lib):
    from paper_2006_07859_amd import RC_F64, RC_SOLVE_PCG_JACOBI, default_solve_opts

    banner("PCG jacobi f64 trefoil96")
    g, e = gen.trefoil(96, seed=4)
    refs, E, dE, A, phi, C = oracle_system(g, e, 2.0, 4.0, BARY | EDGE)
    g_ref, _ = solve.projected_gradient(A, C, dE)
    ctx = make(lib, g, e, 2.0, 4.0, RC_F64, BARY | EDGE)
    out = zeros(len(g), 3)
    st = ctx.rc_sobolev_gradient(dev(g), dev(dE), out,
                                 default_solve_opts(solver=RC_SOLVE_PCG_JACOBI, tol=1e-11, max_iter=4000))
    assert st["residual"] < 1e-11
    assert relnorm(host(out), g_ref) < 1e-7


@pytest.mark.parametrize("mask", [BARY, BARY | EDGE])
def test_pcg_multigrid(lib, mask):
    from paper_2006_07859_amd import RC_F32, RC_SOLVE_PCG_MG, default_solve_opts

    n = 2048
    banner(f"PCG multigrid f32 fourier{n} mask={mask}")
    g, e, _ = gen.fourier_knot(n, seed=1)
    g = gen.round_to_f32(g)
    refs, E, dE, A, phi, C = oracle_system(g, e, 2.0, 4.5, mask)
    g_ref, _ = solve.projected_gradient(A, C, dE)
    ctx = make(lib, g, e, 2.0, 4.5, RC_F32, mask)
    out = zeros(n, 3)
    # FP64 operator inside PCG: the solution is certified by the FP64 residual
    st = ctx.rc_sobolev_gradient(dev(g), dev(dE), out,
                                 default_solve_opts(solver=RC_SOLVE_PCG_MG, tol=1e-9, op_f64=1,
                                                    mg_min_vertices=256))
    assert st["iterations"] < 200
    assert relnorm(host(out), g_ref) < 1e-6
    assert st["iterations"] < 30  # projected multigrid: iteration count independent of n
    # FP32 operator with FP64 true-residual replacement: 1e-6 residual
    st = ctx.rc_sobolev_gradient(dev(g), dev(dE), out,
                                 default_solve_opts(solver=RC_SOLVE_PCG_MG, tol=1e-6, mg_min_vertices=256, op_f64=0))
    Ab = np.kron(A, np.eye(3))
    err = host(out).ravel() - g_ref.ravel()
    assert np.sqrt(err @ Ab @ err) / np.sqrt(g_ref.ravel() @ Ab @ g_ref.ravel()) < 1e-4


def test_bench_solver_options_match_oracle(lib):
    """The projected gradient with exactly the options the benchmark's step uses (multigrid PCG to a
    1e-6 FP64 residual, the Krylov recurrence on the assembled FP32 block refined by FP64 matrix-free
    true residuals every 1e-3, BF16 assembled blocks as the smoothers' operators on levels of >= 512
    vertices, Chebyshev degree 2, coarsest level 256) on a 2,048-edge knot with barycenter and
    edge-length constraints, against the oracle's dense saddle solve (eq. GradientSaddlePointProblem):
    normwise and A-norm error within the FP32 bound 1e-4 of the projected gradient."""
    from paper_2006_07859_amd import RC_F32, RC_SOLVE_PCG_MG, default_solve_opts

    n = 2048
    banner(f"bench solver options vs oracle, fourier{n} barycenter+edge lengths")
    g, e, _ = gen.fourier_knot(n, seed=5)
    g = gen.round_to_f32(g)
    refs, E, dE, A, phi, C = oracle_system(g, e, 2.0, 4.5, BARY | EDGE)
    g_ref, _ = solve.projected_gradient(A, C, dE)
    ctx = make(lib, g, e, 2.0, 4.5, RC_F32, BARY | EDGE)
    so = default_solve_opts(solver=RC_SOLVE_PCG_MG, tol=1e-6, mg_min_vertices=256, cheb_degree=2, op_f64=1,
                            lowp=1, lowp_band=16, lowp_min_vertices=512, lowp_outer=1, inner_tol=1e-3)
    out = zeros(n, 3)
    st = ctx.rc_sobolev_gradient(dev(g), dev(dE), out, so)
    assert st["residual"] < 1e-6 and st["sweeps"] >= 1
    Ab = np.kron(A, np.eye(3))
    err = host(out).ravel() - g_ref.ravel()
    a_err = np.sqrt(err @ Ab @ err) / np.sqrt(g_ref.ravel() @ Ab @ g_ref.ravel())
    n_err = relnorm(host(out), g_ref)
    print(f"  iterations {st['iterations']} sweeps {st['sweeps']} residual {st['residual']:.2e} "
          f"normwise {n_err:.2e} A-norm {a_err:.2e}")
    assert n_err < 1e-4 and a_err < 1e-4
    assert np.abs(C @ host(out).ravel()).max() < 1e-8 * np.abs(host(out)).max()


def test_step_dense_matches_oracle(lib):
    from paper_2006_07859_amd import RC_F64, RC_SOLVE_DENSE, default_solve_opts

    banner("step dense trefoil256 barycenter")
    g, e = gen.trefoil(256, seed=0)
    refs = cons.reference_values(g, e)
    new_ref, info = solve.step(g, e, 2.0, 4.0, BARY, refs)
    ctx = make(lib, g, e, 2.0, 4.0, RC_F64, BARY)
    gam = dev(g)
    st = ctx.rc_step(gam, so=default_solve_opts(solver=RC_SOLVE_DENSE))
    assert st["energy"] == pytest.approx(info["E0"], rel=1e-12)
    assert st["tau"] == info["tau"]
    assert st["energy_new"] == pytest.approx(info["E1"], rel=1e-10)
    assert relnorm(host(gam) - g, new_ref - g) < 1e-7


def test_step_multigrid_edge_lengths(lib):
    from paper_2006_07859_amd import RC_F32, RC_SOLVE_PCG_MG, default_solve_opts

    n = 1024
    banner(f"step multigrid f32 fourier{n} barycenter+edge lengths")
    g, e, _ = gen.fourier_knot(n, seed=2)
    g = gen.round_to_f32(g)
    ctx = make(lib, g, e, 2.0, 4.5, RC_F32, BARY | EDGE)
    gam = dev(g)
    E0 = tpe.energy(g, e, 2.0, 4.5)
    st = ctx.rc_step(gam, so=default_solve_opts(solver=RC_SOLVE_PCG_MG, mg_min_vertices=256))
    new = host(gam)
    E1 = tpe.energy(new, e, 2.0, 4.5)
    assert st["tau"] > 0 and E1 < E0
    assert st["energy_new"] == pytest.approx(E1, rel=1e-5)
    refs = cons.reference_values(g, e)
    phi, _ = cons.evaluate(new, e, BARY | EDGE, *refs, jacobian=False)
    ell, _, _ = tpe.edge_geometry(g, e)
    assert np.abs(phi[3:]).max() < 1e-8 * ell.mean()


@pytest.mark.parametrize("n", [1025, 1026, 1300, 3000, 16384, 16640, 40000])
def test_projector_long_loops(lib, n):
    """Edge-length + barycenter projector on long loops, across the partitions
    of the tridiagonal path solve: 1,024 path rows (one block, one-launch
    projector), 1,025 (five blocks, the last of one row), 1,299 and 2,999 (a
    ragged last block), 16,383 (64 blocks of 256), 16,639 (two rows per thread,
    a ragged last block) and 39,999 (three rows per thread).  Against the
    oracle's dense projector up to 3,000 edges; by its defining properties
    (C P x = 0, P P x = P x, symmetry) at every size."""
    from paper_2006_07859_amd import RC_F64

    banner(f"projector with edge-length rows, n={n}")
    g, e, _ = gen.fourier_knot(n, seed=4)
    ctx = make(lib, g, e, 2.0, 4.5, RC_F64, BARY | EDGE)
    gp = g + 1e-3 * np.random.default_rng(2).normal(size=g.shape) * np.linalg.norm(g[1] - g[0])
    rng = np.random.default_rng(3)
    X, Z = rng.normal(size=g.shape), rng.normal(size=g.shape)
    PX, PZ, PPX = zeros(n, 3), zeros(n, 3), zeros(n, 3)
    ctx.rc_project(dev(gp), dev(X), PX)
    ctx.rc_project(dev(gp), dev(Z), PZ)
    ctx.rc_project(dev(gp), PX, PPX)
    px, pz = host(PX), host(PZ)
    assert relnorm(host(PPX), px) < 1e-12
    assert (X * pz).sum() == pytest.approx((Z * px).sum(), rel=1e-11)
    # C y for the edge rows (T_I . (y_i2 - y_i1)) and the barycenter rows
    x0, _, _ = cons.reference_values(g, e)
    ell, T, xm = tpe.edge_geometry(gp, e)
    i1, i2 = e[:, 0], e[:, 1]
    edge_rows = (T * (px[i2] - px[i1])).sum(1)
    assert np.abs(edge_rows).max() < 1e-11 * np.abs(px).max()
    bary = (0.5 * ell[:, None] * (px[i1] + px[i2]) + (xm - x0) * edge_rows[:, None]).sum(0)
    assert np.abs(bary).max() < 1e-10 * ell.sum() * np.abs(px).max()
    if n <= 3000:
        _, C = cons.evaluate(gp, e, BARY | EDGE, *cons.reference_values(g, e))
        x = X.ravel()
        ref = x - C.T @ np.linalg.solve(C @ C.T, C @ x)
        assert relnorm(px.ravel(), ref) < 1e-11
    ctx.close()
