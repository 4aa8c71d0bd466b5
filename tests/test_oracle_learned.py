"""Pins of the learned-smoother oracle (oracle/learned.py).

* MLP backward and the regression loss gradient against central differences.
* Adam's first step has the closed form -lr g / (|g| + eps) (bias correction
  makes m-hat = g and v-hat = g^2).
* The initial network outputs y0 = 1.7 (softplus(log(expm1(y0))) = y0, W3 small).
* The black/white prolongation keeps constants, copies kept vertices and
  halves the coarse size.
* The ratios r_v = sum_w |A_vw| / A_vv: A annihilates constants, so
  A_vv = -sum_{w != v} A_vw and r_v >= 2; they are invariant under rigid
  motions and scaling (A scales by one factor); with D = diag(r_v A_vv) every
  eigenvalue of D^-1 A lies in [0, 1] (Gershgorin).  The targets
  T_v = r_v lambda_l put the top of the spectrum of diag(T_v A_vv)^-1 A at 1
  exactly, and the weighted projection of the constrained smoother keeps it
  below.
* Features of a regular polygon take their closed forms; the scalar features
  are invariant under rigid motions and scaling, the tangent features rotate.
* The loss weights under-prediction by UNDER (a hand-computed case).
"""

import numpy as np
import pytest

import gen
from oracle import constraints as cons
from oracle import learned as lp


def test_mlp_backward_matches_central_differences():
    rng = np.random.default_rng(0)
    theta = lp.init_params(1) + 0.05 * rng.normal(size=lp.n_params())
    X = rng.normal(size=(7, lp.N_FEATURES))
    dy = rng.normal(size=7)
    y, cache = lp.forward(theta, X)
    g = lp.backward(theta, cache, dy)
    h = 1e-6
    for k in rng.choice(lp.n_params(), size=25, replace=False).tolist() + [lp.n_params() - 1]:
        tp, tm = theta.copy(), theta.copy()
        tp[k] += h
        tm[k] -= h
        fd = (dy @ lp.forward(tp, X)[0] - dy @ lp.forward(tm, X)[0]) / (2 * h)
        assert g[k] == pytest.approx(fd, rel=1e-6, abs=1e-9)


def test_initial_output_and_positivity():
    theta = lp.init_params(3)
    X = np.random.default_rng(1).normal(size=(50, lp.N_FEATURES))
    y, _ = lp.forward(theta, X)
    assert np.all(y > 0)
    assert lp.softplus(np.log(np.expm1(1.7))) == pytest.approx(1.7, abs=1e-14)
    assert np.abs(y - 1.7).max() < 0.2


def test_adam_first_steps_closed_form():
    rng = np.random.default_rng(2)
    theta = rng.normal(size=10)
    g = rng.normal(size=10)
    m = v = np.zeros(10)
    t1, m, v = lp.adam_step(theta, g, m, v, 1, 1e-2)
    assert np.allclose(t1 - theta, -1e-2 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)
    t2, m, v = lp.adam_step(t1, g, m, v, 2, 1e-2)  # same gradient again: same step
    assert np.allclose(t2 - t1, -1e-2 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)


@pytest.mark.parametrize("n", [1000, 999])
def test_prolongation(n):
    g = np.random.default_rng(3).normal(size=(n, 3))
    gammas, Js = lp.hierarchy(g, n_min=256)
    assert [len(x) for x in gammas] == ([1000, 500, 250] if n == 1000 else [999, 500, 250])
    for J, gc in zip(Js, gammas[1:]):
        assert np.allclose(J @ np.ones(J.shape[1]), 1.0)
        kept = np.where(J.max(1) == 1.0)[0]
        assert len(kept) == J.shape[1]
    assert np.array_equal(gammas[1], g[::2])


def test_ratios_bounds_and_invariance():
    g, e, _ = gen.fourier_knot(160, seed=4)
    gammas, _ = lp.hierarchy(g, n_min=40)
    As = lp.level_operators(gammas, 2.0, 4.5)
    r = lp.l1_ratios(As)
    assert len(r) == sum(len(x) for x in gammas)
    assert r.min() >= 2.0 - 1e-12
    # rigid motion and scaling
    q, _ = np.linalg.qr(np.random.default_rng(5).normal(size=(3, 3)))
    g2 = 2.5 * g @ q.T + 1.0
    r2 = lp.l1_ratios(lp.level_operators(lp.hierarchy(g2, n_min=40)[0], 2.0, 4.5))
    assert np.allclose(r, r2, rtol=1e-10)
    # Gershgorin: D = diag(r A_vv) puts the spectrum of D^-1 A in [0, 1]
    o = 0
    for A in As:
        n = len(A)
        D = r[o:o + n] * np.diag(A)
        o += n
        s = 1.0 / np.sqrt(D)
        ev = np.linalg.eigvalsh(s[:, None] * A * s[None, :])
        assert ev.min() > -1e-10 and ev.max() <= 1.0 + 1e-12
        assert ev.max() > 0.3
    # targets: the top eigenvalue of diag(T A_vv)^-1 A is 1
    T = lp.targets(As)
    o = 0
    for A in As:
        n = len(A)
        s = 1.0 / np.sqrt(T[o:o + n] * np.diag(A))
        o += n
        assert np.linalg.eigvalsh(s[:, None] * A * s[None, :])[-1] == pytest.approx(1.0, abs=1e-12)
    assert np.all(T <= r + 1e-12)


def test_weighted_projected_smoother_spectrum():
    """M = W - W C^T (C W C^T)^-1 C W with W = diag(T_v A_vv)^-1: the
    eigenvalues of M Abar lie in [0, lambda_max(W A)] = [0, 1] (barycenter and
    edge-length rows)."""
    g, e, _ = gen.fourier_knot(96, seed=6)
    A = lp.level_operators([g], 2.0, 4.5)[0]
    r = lp.targets([A])
    x0, _, l0 = cons.reference_values(g, e)
    _, C = cons.evaluate(g, e, cons.BARYCENTER | cons.EDGE_LENGTH, x0=x0, l0=l0)
    w = np.repeat(1.0 / (r * np.diag(A)), 3)
    W = np.diag(w)
    M = W - (W @ C.T) @ np.linalg.solve(C @ W @ C.T, C @ W)
    Ab = np.kron(A, np.eye(3))
    ev = np.linalg.eigvals(M @ Ab).real
    assert ev.min() > -1e-9 and ev.max() <= 1.0 + 1e-9


def test_features_regular_polygon_and_invariance():
    n = 64
    g, _ = gen.regular_ngon(n, 1.3, 0.2)
    gammas, Js = lp.hierarchy(g, n_min=20)
    diags = lp.level_diagonals(gammas, 2.0, 4.5)
    F = lp.features(gammas, diags)
    Fl = F[:n]
    assert np.allclose(Fl[:, 0], 6.0 / 16.0)
    assert np.allclose(Fl[:, 1], 0.0, atol=1e-12)
    assert np.allclose(Fl[:, 2], 2 * np.pi / n, atol=1e-12)
    assert np.allclose(Fl[:, 6], 0.0, atol=1e-10)
    assert np.allclose(Fl[:, 7], 0.0, atol=1e-12)
    assert np.allclose(F[n:n + 32, 0], 5.0 / 16.0)
    # rigid motion and scaling: scalar features unchanged, tangents rotated
    rng = np.random.default_rng(5)
    q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    h, _ = gen.fourier_knot(300, seed=2)[:2]
    hg, _ = lp.hierarchy(h, n_min=80)
    hr, _ = lp.hierarchy(0.7 * h @ q.T + 1.0, n_min=80)
    F1 = lp.features(hg, lp.level_diagonals(hg, 2.0, 4.5))
    F2 = lp.features(hr, lp.level_diagonals(hr, 2.0, 4.5))
    s = [0, 1, 2, 6, 7]
    assert np.allclose(F1[:, s], F2[:, s], atol=1e-8)
    assert np.allclose(F1[:, 3:6] @ q.T, F2[:, 3:6], atol=1e-10)


def test_fit_loss_hand_case_and_gradient():
    # hand case: with W1 = W2 = W3 = 0 the network outputs softplus(b3) everywhere
    theta = np.zeros(lp.n_params())
    theta[-1] = np.log(np.expm1(0.5))  # p = 1.5
    R = np.array([2.0, 1.2])
    loss, _ = lp.fit_loss_and_grad(theta, np.zeros((2, lp.N_FEATURES)), R)
    assert loss == pytest.approx((lp.UNDER * np.log(0.75) ** 2 + np.log(1.25) ** 2) / 2, rel=1e-12)
    # gradient against central differences
    rng = np.random.default_rng(9)
    theta = lp.init_params(7) + 0.05 * rng.normal(size=lp.n_params())
    X = rng.normal(size=(40, lp.N_FEATURES))
    R = rng.uniform(2.0, 3.0, size=40)
    loss, grad = lp.fit_loss_and_grad(theta, X, R)
    h = 1e-6
    for k in [0, 100, 600, 1000, 4000, lp.n_params() - 5, lp.n_params() - 1]:
        tp, tm = theta.copy(), theta.copy()
        tp[k] += h
        tm[k] -= h
        fd = (lp.fit_loss_and_grad(tp, X, R)[0] - lp.fit_loss_and_grad(tm, X, R)[0]) / (2 * h)
        assert grad[k] == pytest.approx(fd, rel=1e-5, abs=1e-10)
