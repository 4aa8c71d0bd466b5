"""Pins of the oracle's constraints, saddle solves and step (Sec. 4.3-4.4, 7.1, App. B.3).

* The constraint Jacobians equal central differences of Phi.
* The full saddle solve and an independent route (augmented SPD block plus
  Schur complement) agree; the KKT conditions of eq.
  GradientSaddlePointProblem hold.
* Variational identity g^T Abar d = dE . d for every d in null(C), and the
  descent identity dE . g = g^T Abar g > 0.
* Scaling: g(lambda gamma) = lambda^(alpha - beta + 2 (beta - 1)/alpha) g(gamma).
* The projection increment of eq. ConstraintSaddlePointProblem equals the
  transformed solve of eq. SaddleSolutionTransformation.
* A step restores the constraints, satisfies the Armijo condition and lowers
  the energy.
* Point constraints: the saddle solve with pins alone equals the elimination
  onto the free vertices; one projection increment reaches moved pins exactly
  and moves the free vertices by the A-harmonic extension.
"""

import numpy as np
import pytest
import scipy.linalg as sla

import gen
from oracle import constraints as cons
from oracle import solve, sobolev, tpe

MASKS = [cons.BARYCENTER, cons.BARYCENTER | cons.EDGE_LENGTH, cons.BARYCENTER | cons.TOTAL_LENGTH]


def setup(n=40, seed=21, alpha=2.0, beta=4.5, mask=cons.BARYCENTER, scale=1.0):
    g, e = gen.trefoil(n, seed=seed)
    g = g * scale
    refs = cons.reference_values(g, e)
    E, dE = tpe.differential(g, e, alpha, beta)
    A = sum(sobolev.assemble(g, e, alpha, beta))
    phi, C = cons.evaluate(g, e, mask, *refs)
    return g, e, refs, E, dE, A, phi, C


@pytest.mark.parametrize("mask", MASKS)
def test_jacobian_matches_central_differences(mask):
    g, e, refs, *_ , C = setup(mask=mask)
    h = 1e-6
    for v, c in [(0, 0), (7, 2), (39, 1)]:
        gp, gm = g.copy(), g.copy()
        gp[v, c] += h
        gm[v, c] -= h
        fd = (cons.evaluate(gp, e, mask, *refs, jacobian=False)[0]
              - cons.evaluate(gm, e, mask, *refs, jacobian=False)[0]) / (2 * h)
        assert np.allclose(C[:, 3 * v + c], fd, rtol=1e-7, atol=1e-8)


@pytest.mark.parametrize("mask", MASKS)
def test_saddle_two_routes_and_kkt(mask):
    g, e, refs, E, dE, A, phi, C = setup(mask=mask)
    assert np.abs(phi).max() < 1e-12
    gt, lam = solve.projected_gradient(A, C, dE)
    gs, lams = solve.projected_gradient_schur(A, C, dE)
    assert np.abs(gt - gs).max() < 1e-10 * np.abs(gt).max()
    assert np.abs(lam - lams).max() < 1e-8 * (np.abs(lam).max() + 1)
    Abar = np.kron(A, np.eye(3))
    assert np.abs(C @ gt.ravel()).max() < 1e-10 * np.abs(gt).max()
    kkt = Abar @ gt.ravel() + C.T @ lam - dE.ravel()
    assert np.abs(kkt).max() < 1e-9 * np.abs(dE).max()
    # variational identity on null(C) and the descent identity
    N = sla.null_space(C)
    d = N @ np.random.default_rng(0).normal(size=N.shape[1])
    assert gt.ravel() @ Abar @ d == pytest.approx(dE.ravel() @ d, rel=1e-8)
    q = gt.ravel() @ Abar @ gt.ravel()
    assert q > 0 and np.sum(dE * gt) == pytest.approx(q, rel=1e-9)


@pytest.mark.parametrize("alpha,beta", [(2.0, 4.0), (2.0, 4.5), (3.0, 6.0)])
def test_gradient_scaling(alpha, beta):
    lam = 1.6
    g1 = solve.projected_gradient(*[setup(alpha=alpha, beta=beta)[i] for i in (5, 7, 4)])[0]
    g2 = solve.projected_gradient(*[setup(alpha=alpha, beta=beta, scale=lam)[i] for i in (5, 7, 4)])[0]
    expo = alpha - beta + 2 * (beta - 1) / alpha
    assert np.allclose(g2, lam ** expo * g1, rtol=1e-8, atol=1e-10 * np.abs(g2).max())


@pytest.mark.parametrize("mask", MASKS)
def test_projection_transform_and_step(mask):
    g, e, refs, E, dE, A, phi, C = setup(mask=mask)
    target = phi + np.random.default_rng(1).normal(size=phi.shape) * 1e-3
    x1 = solve.projection_increment(A, C, target)
    x2 = solve.projection_increment_transform(A, C, target)
    assert np.abs(x1 - x2).max() < 1e-10 * np.abs(x1).max()
    assert np.allclose(C @ x1.ravel(), -target, atol=1e-12)
    new, info = solve.step(g, e, 2.0, 4.5, mask, refs)
    assert info["ok"] and info["tau"] > 0
    ghat = info["g"] / np.linalg.norm(info["g"])
    assert info["E1"] <= info["E0"] - 0.01 * info["tau"] * np.sum(info["dE"] * ghat)
    assert info["E1"] < info["E0"]
    phi_new, _ = cons.evaluate(new, e, mask, *refs, jacobian=False)
    ell, _, _ = tpe.edge_geometry(new, e)
    assert np.abs(phi_new).max() < 1e-9 * ell.sum()
    assert tpe.energy(new, e, 2.0, 4.5) == pytest.approx(info["E1"], rel=1e-14)


def two_loops(seed=3):
    """Two disjoint jittered circles of 18 and 23 edges (a small packing)."""
    rng = np.random.default_rng(seed)
    parts, edges, off = [], [], 0
    for m, c in ((18, (0.0, 0.0, 0.0)), (23, (3.0, 0.5, -0.2))):
        t = 2 * np.pi * np.arange(m) / m
        p = np.stack([np.cos(t), np.sin(t), 0.3 * np.sin(2 * t)], 1) + np.asarray(c)
        parts.append(p + 0.01 * rng.normal(size=p.shape))
        edges.append(gen.loop_edges(m, off))
        off += m
    return np.concatenate(parts), np.concatenate(edges)


def test_loop_length_jacobian_and_identities():
    g, e = two_loops()
    x0, L0, l0 = cons.reference_values(g, e)
    Lq = cons.loop_lengths(g, e)
    assert len(Lq) == 2 and abs(Lq.sum() - L0) < 1e-12 * L0
    mask = cons.BARYCENTER | cons.LOOP_LENGTH
    phi, C = cons.evaluate(g, e, mask, x0, Lq=Lq)
    assert C.shape == (5, 3 * len(g)) and np.abs(phi).max() < 1e-12
    # central differences of Phi
    h = 1e-6
    for v, c in [(0, 0), (17, 2), (18, 1), (40, 0)]:
        gp, gm = g.copy(), g.copy()
        gp[v, c] += h
        gm[v, c] -= h
        fd = (cons.evaluate(gp, e, mask, x0, Lq=Lq, jacobian=False)[0]
              - cons.evaluate(gm, e, mask, x0, Lq=Lq, jacobian=False)[0]) / (2 * h)
        assert np.allclose(C[:, 3 * v + c], fd, rtol=1e-7, atol=1e-8)
    # a loop row only touches its own loop's vertices
    assert np.abs(C[3, 3 * 18:]).max() == 0 and np.abs(C[4, :3 * 18]).max() == 0
    # the loop rows sum to the total-length row
    _, Ct = cons.evaluate(g, e, cons.TOTAL_LENGTH, L0=L0)
    assert np.abs(C[3] + C[4] - Ct[0]).max() < 1e-14
    # on a single loop the loop-length row is the total-length row
    g1, e1 = gen.trefoil(30, seed=4)
    p1, C1 = cons.evaluate(g1, e1, cons.LOOP_LENGTH, Lq=cons.loop_lengths(g1, e1) + 0.1)
    p2, C2 = cons.evaluate(g1, e1, cons.TOTAL_LENGTH, L0=cons.reference_values(g1, e1)[1] + 0.1)
    assert np.allclose(p1, p2, atol=1e-14) and np.abs(C1 - C2).max() == 0


def test_loop_length_saddle_kkt():
    g, e = two_loops()
    x0, _, _ = cons.reference_values(g, e)
    Lq = cons.loop_lengths(g, e)
    _, dE = tpe.differential(g, e, 3.0, 6.0)
    A = sum(sobolev.assemble(g, e, 3.0, 6.0))
    _, C = cons.evaluate(g, e, cons.BARYCENTER | cons.LOOP_LENGTH, x0, Lq=Lq)
    gt, lam = solve.projected_gradient(A, C, dE)
    gs, _ = solve.projected_gradient_schur(A, C, dE)
    assert np.abs(gt - gs).max() < 1e-10 * np.abs(gt).max()
    assert np.abs(C @ gt.ravel()).max() < 1e-10 * np.abs(gt).max()
    kkt = np.kron(A, np.eye(3)) @ gt.ravel() + C.T @ lam - dE.ravel()
    assert np.abs(kkt).max() < 1e-9 * np.abs(dE).max()


def test_loop_length_step_restores_every_loop():
    # the projection's tolerance has one row per loop (1e-10 times its length)
    g, e = two_loops()
    refs = cons.reference_values(g, e) + (cons.loop_lengths(g, e),)
    mask = cons.BARYCENTER | cons.LOOP_LENGTH
    new, info = solve.step(g, e, 3.0, 6.0, mask, refs)
    assert info["ok"] and info["E1"] < info["E0"]
    phi, _ = cons.evaluate(new, e, mask, refs[0], Lq=refs[3], jacobian=False)
    assert np.abs(phi[3:]).max() <= 1e-10 * refs[3].max()
    assert np.abs(phi[:3]).max() <= 1e-10 * refs[1] * refs[2].mean()
    assert np.allclose(cons.loop_lengths(new, e), refs[3], rtol=1e-10)


@pytest.mark.parametrize("mask", MASKS)
def test_structured_route_and_sparse_jacobian(mask):
    # the structured solve used for curves too large for the dense saddle matrix
    g, e, refs, E, dE, A, phi, C = setup(n=60, mask=mask)
    Cs = cons.jacobian_sparse(g, e, mask, refs[0])
    assert np.abs(Cs.toarray() - C).max() == 0.0
    gt, lam = solve.projected_gradient(A, C, dE)
    for rho in (None, 1e-3 * np.abs(A).max()):
        gs, lams = solve.projected_gradient_structured(A, Cs, dE, rho=rho)
        assert np.abs(gs - gt).max() < 1e-10 * np.abs(gt).max()
        assert np.abs(lams - lam).max() < 1e-8 * (np.abs(lam).max() + 1)


def test_difference_form_product():
    g, e, refs, E, dE, A, phi, C = setup(n=50)
    u = np.random.default_rng(4).normal(size=(50, 3))
    assert np.allclose(solve.apply_difference_form(A, u, block=7), A @ u, rtol=1e-12, atol=1e-12 * np.abs(A @ u).max())


# --- point constraints (Sec. 7.1) -------------------------------------------


def pinned(n=40, seed=21, npt=2, shift=0.0):
    g, e = gen.trefoil(n, seed=seed)
    pv = np.array([3, 25][:npt])
    px = g[pv] + shift
    return g, e, (pv, px)


def test_point_rows_jacobian_order_and_sparse():
    g, e, pts = pinned(shift=0.01)
    refs = cons.reference_values(g, e)
    mask = cons.BARYCENTER | cons.TOTAL_LENGTH | cons.EDGE_LENGTH
    phi, C = cons.evaluate(g, e, mask, *refs, points=pts)
    assert C.shape[0] == 4 + 6 + len(e)
    # rows after barycenter and total length: gamma_i - x_i, identity Jacobian block
    assert np.allclose(phi[4:10], -0.01)
    h = 1e-6
    for v, c in [(3, 0), (25, 2), (7, 1)]:
        gp, gm = g.copy(), g.copy()
        gp[v, c] += h
        gm[v, c] -= h
        fd = (cons.evaluate(gp, e, mask, *refs, jacobian=False, points=pts)[0]
              - cons.evaluate(gm, e, mask, *refs, jacobian=False, points=pts)[0]) / (2 * h)
        assert np.allclose(C[:, 3 * v + c], fd, rtol=1e-7, atol=1e-8)
    assert np.abs(cons.jacobian_sparse(g, e, mask, refs[0], points=pts).toarray() - C).max() == 0.0


def test_point_constraints_reduce_to_the_free_block():
    """With point constraints alone the saddle system is the Dirichlet-type
    elimination: g vanishes at the pinned vertices and Abar_FF g_F = dE_F on
    the free ones (the pinned vertex removes the constant null space)."""
    g, e, pts = pinned(npt=1)
    _, dE = tpe.differential(g, e, 2.0, 4.5)
    A = sum(sobolev.assemble(g, e, 2.0, 4.5))
    _, C = cons.evaluate(g, e, 0, points=pts)
    gt, _ = solve.projected_gradient(A, C, dE)
    free = np.setdiff1d(np.arange(len(g)), pts[0])
    assert np.abs(gt[pts[0]]).max() < 1e-12 * np.abs(gt).max()
    gF = np.linalg.solve(A[np.ix_(free, free)], dE[free])
    assert np.abs(gt[free] - gF).max() < 1e-10 * np.abs(gF).max()


def test_point_projection_is_one_harmonic_step():
    """Pinned targets moved by d: one projection increment lands exactly on
    them (the constraint is linear), and the free vertices move by the
    A-harmonic extension x_F = -A_FF^-1 A_FP d of the pinned moves."""
    g, e, pts = pinned(npt=2)
    d = np.array([[0.01, -0.02, 0.005], [-0.01, 0.0, 0.02]])
    pts = (pts[0], pts[1] + d)
    refs = cons.reference_values(g, e)
    A = sum(sobolev.assemble(g, e, 2.0, 4.5))
    _, C = cons.evaluate(g, e, 0, *refs, points=pts)
    new, iters, ok = solve.project(g, e, A, C, 0, refs, points=pts)
    assert ok and iters == 1
    assert np.abs(new[pts[0]] - pts[1]).max() < 1e-14
    P, free = pts[0], np.setdiff1d(np.arange(len(g)), pts[0])
    xF = -np.linalg.solve(A[np.ix_(free, free)], A[np.ix_(free, P)] @ d)
    assert np.abs((new - g)[free] - xF).max() < 1e-10 * np.abs(d).max()


def test_point_constrained_step_keeps_pins():
    g, e, pts = pinned(n=48, npt=2)
    refs = cons.reference_values(g, e)
    mask = cons.EDGE_LENGTH  # (total length with edge lengths would be a dependent row)
    new, info = solve.step(g, e, 2.0, 4.5, mask, refs, points=pts)
    assert info["ok"] and info["E1"] < info["E0"]
    assert np.abs(new[pts[0]] - pts[1]).max() <= 1e-10 * refs[2].mean()
    assert np.abs(info["g"][pts[0]]).max() < 1e-12 * np.abs(info["g"]).max()
    assert np.abs(new - g).max() > 1e-4


def test_junction_graph_constraints_and_saddle():
    """A theta graph (two vertices of degree three): the edge-length and barycenter
    Jacobians equal central differences, and the saddle solve's two routes agree."""
    g, e = gen.theta_graph(8, seed=2)
    mask = cons.BARYCENTER | cons.EDGE_LENGTH
    refs = cons.reference_values(g, e)
    _, C = cons.evaluate(g, e, mask, *refs)
    h = 1e-6
    for v, c in [(0, 0), (1, 2), (5, 1)]:
        gp, gm = g.copy(), g.copy()
        gp[v, c] += h
        gm[v, c] -= h
        fd = (cons.evaluate(gp, e, mask, *refs, jacobian=False)[0]
              - cons.evaluate(gm, e, mask, *refs, jacobian=False)[0]) / (2 * h)
        assert np.allclose(C[:, 3 * v + c], fd, rtol=1e-7, atol=1e-8)
    _, dE = tpe.differential(g, e, 2.0, 4.5)
    A = sum(sobolev.assemble(g, e, 2.0, 4.5))
    gt, lam = solve.projected_gradient(A, C, dE)
    gs, _ = solve.projected_gradient_schur(A, C, dE)
    assert np.abs(gt - gs).max() < 1e-10 * np.abs(gt).max()
    assert np.abs(C @ gt.ravel()).max() < 1e-10 * np.abs(gt).max()


# --- surface constraints (Sec. 7.1) -----------------------------------------


def test_surface_values_closed_forms():
    c = np.array([0.3, -0.2, 0.5])
    u = np.array([2.0, -1.0, 2.0]) / 3.0
    f, gr = cons.surface_value(cons.SPHERE, [*c, 1.5], c + (1.5 + 0.01) * u)
    assert f[0] == pytest.approx(0.01, abs=1e-14) and np.allclose(gr[0], u, atol=1e-14)
    R, r = 1.0, 0.4
    pts = c + np.array([[R + r + 0.02, 0.0, 0.0], [0.0, R, r + 0.03], [-(R - r - 0.01), 0.0, 0.0]])
    f, gr = cons.surface_value(cons.TORUS, [*c, R, r], pts)
    assert np.allclose(f, [0.02, 0.03, 0.01], atol=1e-14)
    assert np.allclose(gr, [[1, 0, 0], [0, 0, 1], [1, 0, 0]], atol=1e-14)
    g, _ = gen.tennis_ball(64)
    assert np.abs(cons.surface_value(cons.SPHERE, [0, 0, 0, 1.0], g)[0]).max() < 1e-14
    g, _ = gen.torus_knot(64, R=R, r=r)
    assert np.abs(cons.surface_value(cons.TORUS, [0, 0, 0, R, r], g)[0]).max() < 1e-14


@pytest.mark.parametrize("kind", ["sphere", "torus"])
def test_surface_jacobian_gradient_and_step(kind):
    if kind == "sphere":
        g, e = gen.tennis_ball(48)
        surf = (cons.SPHERE, [0.0, 0.0, 0.0, 1.0], np.arange(48))
    else:
        g, e = gen.torus_knot(48)
        surf = (cons.TORUS, [0.0, 0.0, 0.0, 1.0, 0.4], np.arange(0, 48, 2))
    refs = cons.reference_values(g, e)
    mask = cons.BARYCENTER | cons.EDGE_LENGTH
    gj = g + 1e-3 * np.random.default_rng(1).normal(size=g.shape)
    phi, C = cons.evaluate(gj, e, mask, *refs, surface=surf)
    h = 1e-6
    for v, c in [(0, 0), (2, 2), (7, 1)]:
        gp, gm = gj.copy(), gj.copy()
        gp[v, c] += h
        gm[v, c] -= h
        fd = (cons.evaluate(gp, e, mask, *refs, jacobian=False, surface=surf)[0]
              - cons.evaluate(gm, e, mask, *refs, jacobian=False, surface=surf)[0]) / (2 * h)
        assert np.allclose(C[:, 3 * v + c], fd, rtol=1e-7, atol=1e-8)
    # at a curve on the surface the projected gradient is tangent to it at every held vertex
    _, dE = tpe.differential(g, e, 2.0, 4.5)
    A = sum(sobolev.assemble(g, e, 2.0, 4.5))
    _, C = cons.evaluate(g, e, mask, *refs, surface=surf)
    gt, _ = solve.projected_gradient(A, C, dE)
    gs, _ = solve.projected_gradient_schur(A, C, dE)
    assert np.abs(gt - gs).max() < 1e-10 * np.abs(gt).max()
    _, nrm = cons.surface_value(surf[0], surf[1], g[surf[2]])
    assert np.abs((gt[surf[2]] * nrm).sum(1)).max() < 1e-10 * np.abs(gt).max()
    new, info = solve.step(g, e, 2.0, 4.5, mask, refs, surface=surf)
    assert info["ok"] and info["E1"] < info["E0"]
    f, _ = cons.surface_value(surf[0], surf[1], new[surf[2]])
    assert np.abs(f).max() <= 1e-10 * refs[2].mean()


# --- tangent constraints (Sec. 7.1) -----------------------------------------


def test_tangent_basis_rule():
    u, v = cons.tangent_basis([0.0, 0.0, 2.0])
    assert np.allclose(u, [0, 1, 0], atol=0) and np.allclose(v, [-1, 0, 0], atol=0)
    for X in np.random.default_rng(4).normal(size=(5, 3)):
        u, v = cons.tangent_basis(X)
        Xn = X / np.linalg.norm(X)
        B = np.stack([u, v, Xn])
        assert np.allclose(B @ B.T, np.eye(3), atol=1e-14)
        assert np.allclose(np.cross(u, v), Xn, atol=1e-14)


def test_tangent_rows_values_jacobian_and_paper_form():
    g, e = gen.trefoil(40, seed=21)
    ell, T, _ = tpe.edge_geometry(g, e)
    I = 7
    X = T[I].copy()
    # the rows vanish at T_I = X; turning X by theta about u's orthogonal gives u . T = sin(theta)
    phi, C = cons.evaluate(g, e, 0, tangent=([I], [X]))
    assert np.abs(phi).max() < 1e-15
    u, v = cons.tangent_basis(X)
    th = 0.3
    Xr = np.cos(th) * X - np.sin(th) * u  # then T_I = cos(th) Xr + sin(th) u', u' . T_I = sin(th)
    phi_r, _ = cons.evaluate(g, e, 0, tangent=([I], [Xr]))
    ur, vr = cons.tangent_basis(Xr)
    assert np.allclose(phi_r, [ur @ T[I], vr @ T[I]], atol=1e-15)
    assert np.hypot(*phi_r) == pytest.approx(np.sin(th), rel=1e-12)
    # Jacobian against central differences, with another tangent and the barycenter rows
    tg = ([I, 20], [Xr, T[20] + 0.1])
    refs = cons.reference_values(g, e)
    _, C = cons.evaluate(g, e, cons.BARYCENTER, *refs, tangent=tg)
    h = 1e-6
    for vtx, c in [(7, 0), (8, 2), (20, 1), (21, 0), (3, 1)]:
        gp, gm = g.copy(), g.copy()
        gp[vtx, c] += h
        gm[vtx, c] -= h
        fd = (cons.evaluate(gp, e, cons.BARYCENTER, *refs, jacobian=False, tangent=tg)[0]
              - cons.evaluate(gm, e, cons.BARYCENTER, *refs, jacobian=False, tangent=tg)[0]) / (2 * h)
        assert np.allclose(C[:, 3 * vtx + c], fd, rtol=1e-7, atol=1e-8)
    # the paper's three rows T_I - X: their Jacobian (by differences of T_I) has rank 2 and the
    # same row space as the two rows read here
    J3 = np.zeros((3, 3 * len(g)))
    for vtx in e[I]:
        for c in range(3):
            gp, gm = g.copy(), g.copy()
            gp[vtx, c] += h
            gm[vtx, c] -= h
            J3[:, 3 * vtx + c] = (tpe.edge_geometry(gp, e)[1][I] - tpe.edge_geometry(gm, e)[1][I]) / (2 * h)
    _, C2 = cons.evaluate(g, e, 0, tangent=([I], [X]))
    assert np.linalg.matrix_rank(J3, tol=1e-6) == 2
    assert np.linalg.matrix_rank(np.vstack([J3, C2]), tol=1e-6) == 2


def test_tangent_constrained_step_keeps_tangents():
    g, e = gen.trefoil(48, seed=21)
    _, T, _ = tpe.edge_geometry(g, e)
    tg = ([0, 24], [T[0], T[24]])
    refs = cons.reference_values(g, e)
    new, info = solve.step(g, e, 2.0, 4.5, cons.BARYCENTER | cons.EDGE_LENGTH, refs, tangent=tg)
    assert info["ok"] and info["E1"] < info["E0"]
    _, T1, _ = tpe.edge_geometry(new, e)
    assert np.abs(T1[[0, 24]] - T[[0, 24]]).max() < 1e-9
    assert np.abs(new - g).max() > 1e-4
