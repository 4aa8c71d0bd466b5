"""Learned multilevel preconditioner, in float64 (oracle).

Test infrastructure only (see the package docstring).

Not a construction of the paper.  It reuses the paper's multigrid hierarchy
(App. B.3.1: black/white coarsening of a closed curve, keeping every other
vertex, with prolongation J that copies kept vertices and averages the two
kept neighbours of a removed one) and forms the additive preconditioner

    M^-1 = sum_l P_l D_l P_l^T,   P_0 = Id,  P_l = J_1 ... J_l,

with positive diagonal scalings ``D_l = diag(y_{l,v} / diag(A_l)_v)``, where
A_l is the Sobolev operator of Sec. 4.2 rediscretised on level l and
``y_{l,v} > 0`` is the output of a small MLP (3 layers, width 64, ReLU, softplus
output) evaluated on per-vertex features.  ``y = 1`` is the hand-weighted
(Jacobi-scaled) multilevel preconditioner.  M^-1 is symmetric positive
definite for any parameters, and PCG applies it as ``P M^-1 P``.

Training minimises the relative A-norm error of one application to the
right-hand side of the projected gradient problem (eq.
GradientSaddlePointProblem), with g the exact projected gradient and the
application scaled by the best factor c (PCG does not see the scale of M):

    loss = min_c |c z - g|_A^2 / |g|_A^2 = 1 - <z, g>_A^2 / (|z|_A^2 |g|_A^2),
    z = P M^-1 P dE,  <x, y>_A = x^T Abar y.

Curves are single closed loops whose vertices are numbered along the loop.
"""

from __future__ import annotations

import numpy as np

from . import sobolev, tpe

__all__ = ["N_FEATURES", "WIDTH", "n_params", "init_params", "unpack", "forward", "backward", "adam_step",
           "hierarchy", "features", "level_diagonals", "apply_multilevel", "loss_and_grad"]

N_FEATURES = 8
WIDTH = 64
OFFSET = 4  # vertices at most this far apart along the loop are not "other parts" of the curve


def n_params(f_in=N_FEATURES, width=WIDTH):
    return f_in * width + width + width * width + width + width + 1


def unpack(theta, f_in=N_FEATURES, width=WIDTH):
    """Views (W1 [f_in, w], b1 [w], W2 [w, w], b2 [w], W3 [w], b3 [1]) of the flat parameters."""
    theta = np.asarray(theta)
    k = 0
    out = []
    for shape in ((f_in, width), (width,), (width, width), (width,), (width,), (1,)):
        n = int(np.prod(shape))
        out.append(theta[k:k + n].reshape(shape))
        k += n
    return out


def init_params(seed=0, f_in=N_FEATURES, width=WIDTH):
    """He-scaled hidden layers, a small output layer and an output bias with
    softplus(b3) = 1, so that the network starts at the hand-weighted scalings."""
    rng = np.random.default_rng(seed)
    W1 = rng.normal(0.0, np.sqrt(2.0 / f_in), size=(f_in, width))
    W2 = rng.normal(0.0, np.sqrt(2.0 / width), size=(width, width))
    W3 = rng.normal(0.0, 0.01, size=width)
    b3 = np.array([np.log(np.e - 1.0)])
    return np.concatenate([W1.ravel(), np.zeros(width), W2.ravel(), np.zeros(width), W3, b3])


def softplus(o):
    return np.logaddexp(0.0, o)


def forward(theta, X):
    """y = softplus(W3 . relu(W2^T relu(W1^T x + b1) + b2) + b3) for every row x of X."""
    W1, b1, W2, b2, W3, b3 = unpack(theta, X.shape[1])
    a1 = X @ W1 + b1
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ W2 + b2
    h2 = np.maximum(a2, 0.0)
    o = h2 @ W3 + b3[0]
    return softplus(o), (X, a1, h1, a2, h2, o)


def backward(theta, cache, dy):
    """Gradient of sum(dy * y) with respect to the flat parameters."""
    X, a1, h1, a2, h2, o = cache
    W1, b1, W2, b2, W3, b3 = unpack(theta, X.shape[1])
    do = dy / (1.0 + np.exp(-o))              # softplus' = logistic
    gW3 = h2.T @ do
    gb3 = np.array([do.sum()])
    dh2 = np.outer(do, W3) * (a2 > 0)
    gW2 = h1.T @ dh2
    gb2 = dh2.sum(0)
    dh1 = (dh2 @ W2.T) * (a1 > 0)
    gW1 = X.T @ dh1
    gb1 = dh1.sum(0)
    return np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3, gb3])


def adam_step(theta, grad, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba, Algorithm 1); t counts from 1."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def _prolongation(n):
    """J (n x nc) of one black/white coarsening of a closed loop of n vertices."""
    keep = list(range(0, n, 2))
    nc = len(keep)
    J = np.zeros((n, nc))
    for q, i0 in enumerate(keep):
        J[i0, q] = 1.0
        i1 = keep[q + 1] if q + 1 < nc else keep[0] + n
        for i in range(i0 + 1, i1):
            J[i % n, q] += 0.5
            J[i % n, (q + 1) % nc] += 0.5
    return J, keep


def hierarchy(gamma, n_min=256):
    """Level curves and prolongations: coarsen while the loop has more than n_min
    vertices (and at least 12)."""
    g = np.asarray(gamma, dtype=np.float64)
    gammas, Js = [g], []
    while len(g) > n_min and len(g) >= 12:
        J, keep = _prolongation(len(g))
        g = g[keep]
        gammas.append(g)
        Js.append(J)
    return gammas, Js


def _loop_edges(n):
    return np.stack([np.arange(n), (np.arange(n) + 1) % n], axis=1)


def level_diagonals(gammas, alpha, beta):
    return [np.diag(sum(sobolev.assemble(g, _loop_edges(len(g)), alpha, beta))) for g in gammas]


def features(gammas, diags):
    """Per-vertex features of every level, stacked level by level:
    level / (levels - 1); log of the mean incident edge length over the level's
    mean; turning angle; unit vertex tangent (3); log of the diagonal of A_l over
    its mean; log of the distance to the nearest vertex more than OFFSET steps
    away along the loop over the mean incident edge length."""
    L = len(gammas)
    rows = []
    for l, (g, dg) in enumerate(zip(gammas, diags)):
        n = len(g)
        ell, T, _ = tpe.edge_geometry(g, _loop_edges(n))
        lin, Tin = np.roll(ell, 1), np.roll(T, 1, axis=0)   # edge into v, and out of v
        lbar = 0.5 * (lin + ell)
        turn = np.arccos(np.clip((Tin * T).sum(1), -1.0, 1.0))
        tv = Tin + T
        tv /= np.linalg.norm(tv, axis=1)[:, None]
        d = np.linalg.norm(g[:, None, :] - g[None, :, :], axis=2)
        idx = np.arange(n)
        sep = np.abs(idx[:, None] - idx[None, :])
        sep = np.minimum(sep, n - sep)
        d[sep <= OFFSET] = np.inf
        F = np.empty((n, N_FEATURES))
        F[:, 0] = l / max(1, L - 1)
        F[:, 1] = np.log(lbar / ell.mean())
        F[:, 2] = turn
        F[:, 3:6] = tv
        F[:, 6] = np.log(dg / dg.mean())
        F[:, 7] = np.log(d.min(1) / lbar)
        rows.append(F)
    return np.concatenate(rows)


def apply_multilevel(Js, scal, r):
    """sum_l P_l diag(scal_l) P_l^T r for r [n0, 3]; scal is the list of
    per-level vertex scalings (D_l)."""
    us = [np.asarray(r, dtype=np.float64)]
    for J in Js:
        us.append(J.T @ us[-1])
    z = scal[-1][:, None] * us[-1]
    for l in range(len(Js) - 1, -1, -1):
        z = scal[l][:, None] * us[l] + Js[l] @ z
    return z


def loss_and_grad(theta, gamma, dE, g_ref, A, C, alpha, beta, n_min=256):
    """Relative A-norm error of the best-scaled P M^-1 P dE against the
    projected gradient g_ref, and its gradient with respect to the parameters."""
    gammas, Js = hierarchy(gamma, n_min)
    diags = level_diagonals(gammas, alpha, beta)
    X = features(gammas, diags)
    y, cache = forward(theta, X)
    sizes = [len(g) for g in gammas]
    cuts = np.cumsum([0] + sizes)
    scal = [y[cuts[l]:cuts[l + 1]] / diags[l] for l in range(len(sizes))]
    P = np.eye(C.shape[1]) - C.T @ np.linalg.solve(C @ C.T, C)
    Pd = (P @ np.asarray(dE).ravel()).reshape(-1, 3)
    z = (P @ apply_multilevel(Js, scal, Pd).ravel()).reshape(-1, 3)
    Ab = np.kron(A, np.eye(3))
    gr = np.asarray(g_ref).ravel()
    zr = z.ravel()
    Az, Ag = Ab @ zr, Ab @ gr
    a, b, c = zr @ Ag, zr @ Az, gr @ Ag
    loss = 1.0 - a * a / (b * c)
    w = (P @ ((2.0 * a / (b * c)) * ((a / b) * Az - Ag))).reshape(-1, 3)
    # d loss / d scal_l[v] = sum_c (P_l^T w)[v, c] (P_l^T P dE)[v, c]
    us, ws = [Pd], [w]
    for J in Js:
        us.append(J.T @ us[-1])
        ws.append(J.T @ ws[-1])
    dscal = [(ws[l] * us[l]).sum(1) for l in range(len(sizes))]
    dy = np.concatenate([dscal[l] / diags[l] for l in range(len(sizes))])
    return loss, backward(theta, cache, dy)
