"""Learned smoother weights of the multigrid V-cycle, in float64 (oracle).

Test infrastructure only (see the package docstring).

Not a construction of the paper.  It reuses the paper's multigrid hierarchy
(App. B.3.1: black/white coarsening of a closed curve, keeping every other
vertex) and its Jacobi-type smoothing, and learns the smoother's diagonal.
For the operator A_l of Sec. 4.2 rediscretised on level l, the ratio

    r_v = sum_w |A_l,vw| / A_l,vv   (>= 2: A annihilates constants)

makes D_r = diag(r_v A_l,vv) a Gershgorin bound (the spectrum of D_r^-1 A_l
lies in [0, 1]); with lambda_l its largest eigenvalue, the target

    T_v = r_v lambda_l

gives D = diag(T_v A_l,vv) whose D^-1 A_l tops out at exactly 1, so a
Chebyshev smoother on D^-1 A_l (and on its projected forms, whose spectra lie
inside) may take the fixed interval [frac, 1] instead of estimating the
largest eigenvalue.  A small MLP (3 layers, width 64, ReLU, softplus output)
maps per-vertex features to p = 1 + y and is trained by regression on T in
log space, with under-prediction (p < T, where the interval would fall short
of the spectrum) weighted by UNDER:

    loss = mean_v w_v (log p_v - log T_v)^2,   w_v = UNDER if p_v < T_v else 1.

Curves are single closed loops whose vertices are numbered along the loop.
"""

from __future__ import annotations

import numpy as np

from . import sobolev, tpe

__all__ = ["N_FEATURES", "WIDTH", "UNDER", "n_params", "init_params", "unpack", "forward", "backward", "adam_step",
           "hierarchy", "features", "level_diagonals", "level_operators", "l1_ratios", "targets", "fit_loss_and_grad"]

N_FEATURES = 8
WIDTH = 64
UNDER = 4.0  # weight of an under-predicted ratio in the regression loss


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


def init_params(seed=0, f_in=N_FEATURES, width=WIDTH, y0=1.7):
    """He-scaled hidden layers, a small output layer and an output bias with
    softplus(b3) = y0, so that the network starts near the constant ratio
    1 + y0."""
    rng = np.random.default_rng(seed)
    W1 = rng.normal(0.0, np.sqrt(2.0 / f_in), size=(f_in, width))
    W2 = rng.normal(0.0, np.sqrt(2.0 / width), size=(width, width))
    W3 = rng.normal(0.0, 0.01, size=width)
    b3 = np.array([np.log(np.expm1(y0))])
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


def level_operators(gammas, alpha, beta):
    """Dense A_l = B + B0 (Sec. 4.2, trapezoid weights) of every level."""
    return [sum(sobolev.assemble(g, _loop_edges(len(g)), alpha, beta)) for g in gammas]


def level_diagonals(gammas, alpha, beta):
    return [np.diag(A) for A in level_operators(gammas, alpha, beta)]


def l1_ratios(As):
    """r_v = sum_w |A_vw| / A_vv of every level, stacked finest first."""
    return np.concatenate([np.abs(A).sum(1) / np.diag(A) for A in As])


def targets(As):
    """T_v = r_v lambda_l of every level (lambda_l the largest eigenvalue of
    D_r^-1/2 A_l D_r^-1/2), stacked finest first."""
    out = []
    for A in As:
        r = np.abs(A).sum(1) / np.diag(A)
        s = 1.0 / np.sqrt(r * np.diag(A))
        lam = np.linalg.eigvalsh(s[:, None] * A * s[None, :])[-1]
        out.append(r * lam)
    return np.concatenate(out)


def features(gammas, diags):
    """Per-vertex features of every level, stacked level by level:
    log2(n_l) / 16; log of the mean incident edge length over the level's
    mean; turning angle; unit vertex tangent (3); log of the diagonal of A_l
    over its mean; log of the incoming over the outgoing edge length."""
    rows = []
    for g, dg in zip(gammas, diags):
        n = len(g)
        ell, T, _ = tpe.edge_geometry(g, _loop_edges(n))
        lin, Tin = np.roll(ell, 1), np.roll(T, 1, axis=0)   # edge into v, and out of v
        lbar = 0.5 * (lin + ell)
        turn = np.arccos(np.clip((Tin * T).sum(1), -1.0, 1.0))
        tv = Tin + T
        tv /= np.linalg.norm(tv, axis=1)[:, None]
        F = np.empty((n, N_FEATURES))
        F[:, 0] = np.log2(n) / 16.0
        F[:, 1] = np.log(lbar / ell.mean())
        F[:, 2] = turn
        F[:, 3:6] = tv
        F[:, 6] = np.log(dg / dg.mean())
        F[:, 7] = np.log(lin / ell)
        rows.append(F)
    return np.concatenate(rows)


def fit_loss_and_grad(theta, X, R):
    """The regression loss of p = 1 + y(X) on the targets R and its gradient
    with respect to the parameters."""
    y, cache = forward(theta, X)
    p = 1.0 + y
    e = np.log(p) - np.log(R)
    w = np.where(p < R, UNDER, 1.0)
    loss = float(np.mean(w * e * e))
    dy = 2.0 * w * e / p / len(R)
    return loss, backward(theta, cache, dy)
