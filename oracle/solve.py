"""Projected Sobolev gradient, constraint projection and the step, in float64 (oracle).

Test infrastructure only (see the package docstring).

Definitions (paper Sec. 4.3-4.4 and App. B.3.3-B.3.4):

* Eq. GradientSaddlePointProblem: ``[[Abar, C^T], [C, 0]] [g; lam] = [dE; 0]``
  with ``Abar`` the componentwise operator (eq. VectorInnerProduct).  In the
  vertex-major ordering used here ``Abar = kron(A, Id_3)``.
* Eq. ConstraintSaddlePointProblem: one projection iteration solves
  ``[[Abar, C^T], [C, 0]] [x; mu] = [0; -Phi(gamma~)]`` and sets
  ``gamma~ += x``; ``Abar`` and ``C`` stay those of the curve before the step
  (the factorisation of the gradient system is reused).
* App. B.3.4, eq. SaddleSolutionTransformation: the same x is
  ``x = z - y`` with ``z = C^T (C C^T)^-1 b`` and y the solution of the
  gradient-type system with right-hand side ``Abar z``.  Here the pseudoinverse
  is read as ``C^T (C C^T)^-1`` (the product printed in App. B.3.3 does not
  type-check as written).
* Sec. 4.4: normalise the projected gradient by its Euclidean norm, start at
  ``tau = 1`` and halve tau until the constraint projection succeeds and the
  Armijo condition ``E(gamma_new) <= E(gamma) - c tau <dE, g_hat>`` holds
  (backtracking in the sense of the cited textbook algorithm; constants
  ``c = 0.01`` and factor 1/2).
"""

from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from . import constraints as cons
from . import sobolev, tpe

__all__ = [
    "saddle_matrix",
    "projected_gradient",
    "projected_gradient_schur",
    "projected_gradient_structured",
    "apply_difference_form",
    "projection_increment",
    "projection_increment_transform",
    "project",
    "line_search",
    "step",
]


def saddle_matrix(A, C):
    Abar = np.kron(A, np.eye(3))
    k = C.shape[0]
    return np.block([[Abar, C.T], [C, np.zeros((k, k))]])


def projected_gradient(A, C, dE):
    """(g_tilde [V,3], lam) from the full saddle system (eq. GradientSaddlePointProblem)."""
    n = 3 * A.shape[0]
    rhs = np.concatenate([np.asarray(dE).ravel(), np.zeros(C.shape[0])])
    sol = sla.solve(saddle_matrix(A, C), rhs, assume_a="sym")
    return sol[:n].reshape(-1, 3), sol[n:]


def projected_gradient_schur(A, C, dE):
    """Same solution by a different route: augmented SPD block plus Schur complement.

    Because C g = 0, adding ``C^T C`` to ``Abar`` leaves the solution unchanged
    and makes the block positive definite (Abar is definite on null(C)).
    """
    Abar = np.kron(A, np.eye(3))
    H = Abar + C.T @ C
    cf = sla.cho_factor(H)
    b = np.asarray(dE).ravel()
    HinvCt = sla.cho_solve(cf, C.T)
    S = C @ HinvCt
    lam = np.linalg.solve(S, C @ sla.cho_solve(cf, b))
    g = sla.cho_solve(cf, b - C.T @ lam)
    return g.reshape(-1, 3), lam


def apply_difference_form(A, u, block=256):
    """A u as (A u)_v = sum_w A_vw (u_w - u_v): the increment tables of Sec.
    4.2.2-4.2.3 give every row of A a zero sum (B and B0 annihilate constants),
    so this is A u exactly, and for a smooth u it avoids the cancellation
    between the large diagonal and the off-diagonal terms of the plain product."""
    A = np.asarray(A)
    u = np.asarray(u, dtype=np.float64)
    out = np.zeros_like(u)
    for s in range(0, A.shape[0], block):
        rows = slice(s, min(A.shape[0], s + block))
        diff = u[None, :, :] - u[rows][:, None, :]
        out[rows] = np.einsum("vw,vwk->vk", A[rows], diff)
    return out


def projected_gradient_structured(A, C, dE, rho=None, refine=4):
    """Same solution for curves whose 3|V| x 3|V| saddle matrix does not fit: the
    component structure Abar = kron(A, Id_3) and A 1 = 0 are used instead of
    forming Abar.

    With ``H0 = A + rho 1 1^T / n`` (symmetric positive definite, since the null
    space of A is the constants) and ``U = kron(1 / sqrt(n), Id_3)``,
    ``Abar = kron(H0, Id_3) - rho U U^T``; the unknown ``mu = -rho U^T g`` turns the
    saddle system into the extended system
    ``[[Hbar, C^T, U], [C, 0, 0], [U^T, 0, Id_3 / rho]] [g; lam; mu] = [dE; 0; 0]``
    (``Hbar = kron(H0, Id_3)``), solved through its dense Schur complement of
    size k + 3, ``(F^T Hbar^-1 F - D) y = F^T Hbar^-1 b - c`` with
    ``F = [C^T, U]``, ``D = diag(0, Id_3 / rho)``; ``Hbar^-1`` is one Cholesky
    factor of H0 applied to each coordinate component.  The factorisations are
    then reused for ``refine`` steps of iterative refinement on the extended
    system's FP64 residual, with A applied in the difference form
    (``apply_difference_form``): at large sizes A is ill-conditioned enough
    (order 2s = 3.5) that one pass, or a residual taken with the plain product,
    leaves errors far above those of an iterative solver.  C may be dense or
    scipy.sparse.  Returns (g [V,3], lam).
    """
    import scipy.sparse as sp

    A = np.asarray(A, dtype=np.float64)
    n = A.shape[0]
    if rho is None:
        rho = float(np.mean(np.diag(A)))
    cf = sla.cho_factor(A + rho / n, lower=True)
    Cs = sp.csr_matrix(C)
    k = Cs.shape[0]
    U = sp.kron(np.ones((n, 1)) / np.sqrt(n), sp.identity(3), format="csr")
    F = sp.hstack([Cs.T, U], format="csr")              # 3n x (k + 3)
    S = np.zeros((k + 3, k + 3))
    for c in range(3):
        Fc = F[c::3]                                    # rows of component c: n x (k + 3)
        S += Fc.T @ sla.cho_solve(cf, Fc.toarray())     # F_c^T H0^-1 F_c
    S[k:, k:] -= np.eye(3) / rho
    lu = sla.lu_factor(S, overwrite_a=True)
    del S

    def solve_ext(b, c):
        Hb = sla.cho_solve(cf, b)
        y = sla.lu_solve(lu, F.T @ Hb.ravel() - c)
        return sla.cho_solve(cf, b - (F @ y).reshape(n, 3)), y

    b = np.asarray(dE, dtype=np.float64).reshape(n, 3)
    g, y = solve_ext(b, np.zeros(k + 3))
    for _ in range(refine):
        lam, mu = y[:k], y[k:]
        Hg = apply_difference_form(A, g) + (rho / n) * g.sum(0, keepdims=True)
        r1 = b - Hg - (F @ y).reshape(n, 3)
        r23 = -(F.T @ g.ravel()) - np.concatenate([np.zeros(k), mu / rho])
        dg, dy = solve_ext(r1, r23)
        g, y = g + dg, y + dy
    return g, y[:k]


def projection_increment(A, C, phi):
    """x solving [[Abar, C^T], [C, 0]] [x; mu] = [0; -phi] (eq. ConstraintSaddlePointProblem)."""
    n = 3 * A.shape[0]
    rhs = np.concatenate([np.zeros(n), -np.asarray(phi)])
    sol = sla.solve(saddle_matrix(A, C), rhs, assume_a="sym")
    return sol[:n].reshape(-1, 3)


def projection_increment_transform(A, C, phi):
    """Same x through eq. SaddleSolutionTransformation: x = z - y."""
    b = -np.asarray(phi)
    z = C.T @ np.linalg.solve(C @ C.T, b)
    Abar = np.kron(A, np.eye(3))
    y, _ = projected_gradient(A, C, Abar @ z)
    return (z - y.ravel()).reshape(-1, 3)


def _phi_tolerance(gamma, edges, mask, n_points=0, n_surface=0, n_tangent=0):
    """Per-row projection tolerance: 1e-10 l_mean (edge lengths, points, surface),
    1e-10 (the dimensionless tangent rows),
    1e-10 L l_mean (barycenter), 1e-10 L (total length) and 1e-10 L_q (length
    of loop q)."""
    ell, _, _ = tpe.edge_geometry(gamma, edges)
    lbar, L = ell.mean(), ell.sum()
    tol = []
    if mask & cons.BARYCENTER:
        tol += [1e-10 * L * lbar] * 3
    if mask & cons.TOTAL_LENGTH:
        tol += [1e-10 * L]
    tol += [1e-10 * lbar] * (3 * n_points + n_surface)
    tol += [1e-10] * (2 * n_tangent)
    if mask & cons.EDGE_LENGTH:
        tol += [1e-10 * lbar] * len(edges)
    if mask & cons.LOOP_LENGTH:
        tol += list(1e-10 * cons.loop_lengths(gamma, edges))
    return np.array(tol)


def project(gamma_t, edges, A, C, mask, refs, max_iter=10, tol=None, points=None, surface=None, tangent=None):
    """Iterate the projection increment from gamma_t; returns (gamma, iters, ok).

    ``refs`` is ``(x0, L0, l0)`` or ``(x0, L0, l0, Lq)`` with the loop-length
    targets ``Lq`` (needed when ``mask`` has LOOP_LENGTH); ``points`` =
    (vertices, targets) of the point constraints, ``surface`` = (kind,
    params, vertices) of the surface constraints, ``tangent`` = (edges,
    directions) of the tangent constraints."""
    x0, L0, l0 = refs[:3]
    Lq = refs[3] if len(refs) > 3 else None
    g = np.array(gamma_t, dtype=np.float64)
    npt = 0 if points is None else len(points[0])
    nsf = 0 if surface is None else len(surface[2])
    ntg = 0 if tangent is None else len(tangent[0])
    tol = _phi_tolerance(g, edges, mask, npt, nsf, ntg) if tol is None else tol
    for it in range(max_iter + 1):
        phi, _ = cons.evaluate(g, edges, mask, x0, L0, l0, jacobian=False, Lq=Lq, points=points, surface=surface,
                               tangent=tangent)
        if np.all(np.abs(phi) <= tol):
            return g, it, True
        if it == max_iter:
            break
        g = g + projection_increment(A, C, phi)
    return g, max_iter, False


def line_search(gamma, edges, alpha, beta, E0, dE, g_tilde, A, C, mask, refs,
                c_armijo=0.01, shrink=0.5, max_backtracks=30, tau0=1.0, points=None, surface=None, tangent=None):
    """Backtracking step of Sec. 4.4; returns (gamma_new, tau, E_new, info)."""
    ghat = g_tilde / np.linalg.norm(g_tilde)
    slope = float(np.sum(dE * ghat))
    tau = tau0
    for bt in range(max_backtracks + 1):
        cand = gamma - tau * ghat
        proj, iters, ok = project(cand, edges, A, C, mask, refs, points=points, surface=surface, tangent=tangent)
        if ok:
            E1 = tpe.energy(proj, edges, alpha, beta)
            if E1 <= E0 - c_armijo * tau * slope:
                return proj, tau, E1, dict(backtracks=bt, proj_iters=iters, ok=True)
        tau *= shrink
    return gamma, 0.0, E0, dict(backtracks=max_backtracks, proj_iters=0, ok=False)


def step(gamma, edges, alpha, beta, mask, refs, points=None, surface=None, tangent=None):
    """One projected Sobolev step: dE, A, C, g_tilde, line search."""
    E0, dE = tpe.differential(gamma, edges, alpha, beta)
    B, B0 = sobolev.assemble(gamma, edges, alpha, beta)
    A = B + B0
    x0, L0, l0 = refs[:3]
    _, C = cons.evaluate(gamma, edges, mask, x0, L0, l0, Lq=refs[3] if len(refs) > 3 else None, points=points,
                         surface=surface, tangent=tangent)
    g, _ = projected_gradient(A, C, dE)
    new, tau, E1, info = line_search(gamma, edges, alpha, beta, E0, dE, g, A, C, mask, refs, points=points,
                                     surface=surface, tangent=tangent)
    info.update(E0=E0, E1=E1, tau=tau, g=g, dE=dE)
    return new, info
