"""Pins of the learned-preconditioner oracle (oracle/learned.py).

* MLP backward and the whole loss gradient against central differences.
* Adam's first step has the closed form -lr g / (|g| + eps) (bias correction
  makes m-hat = g and v-hat = g^2).
* The initial network outputs 1 (softplus(log(e - 1)) = 1 exactly, W3 small).
* The black/white prolongation keeps constants, copies kept vertices and
  halves the coarse size.
* The multilevel operator is symmetric positive definite.
* Features of a regular polygon take their closed forms; the scalar features
  are invariant under rigid motions, the tangent features rotate.
"""

import numpy as np
import pytest

import gen
from oracle import constraints as cons
from oracle import learned as lp
from oracle import sobolev, solve, tpe


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
    assert lp.softplus(np.log(np.e - 1.0)) == pytest.approx(1.0, abs=1e-15)
    assert np.abs(y - 1.0).max() < 0.2


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


def test_multilevel_operator_spd():
    rng = np.random.default_rng(4)
    g = rng.normal(size=(300, 3))
    _, Js = lp.hierarchy(g, n_min=40)
    sizes = [300] + [J.shape[1] for J in Js]
    scal = [rng.uniform(0.1, 2.0, size=s) for s in sizes]
    x, y = rng.normal(size=(300, 3)), rng.normal(size=(300, 3))
    Mx, My = lp.apply_multilevel(Js, scal, x), lp.apply_multilevel(Js, scal, y)
    assert (x * My).sum() == pytest.approx((y * Mx).sum(), rel=1e-12)
    assert (x * Mx).sum() > 0


def test_features_regular_polygon_and_invariance():
    n = 64
    g, _ = gen.regular_ngon(n, 1.3, 0.2)
    gammas, Js = lp.hierarchy(g, n_min=20)
    diags = lp.level_diagonals(gammas, 2.0, 4.5)
    F = lp.features(gammas, diags)
    Fl = F[:n]
    assert np.allclose(Fl[:, 0], 0.0)
    assert np.allclose(Fl[:, 1], 0.0, atol=1e-12)
    assert np.allclose(Fl[:, 2], 2 * np.pi / n, atol=1e-12)
    assert np.allclose(Fl[:, 6], 0.0, atol=1e-10)
    k = lp.OFFSET + 1
    assert np.allclose(Fl[:, 7], np.log(np.sin(k * np.pi / n) / np.sin(np.pi / n)), atol=1e-12)
    assert np.allclose(F[-len(gammas[-1]):, 0], 1.0)
    # rigid motion: scalar features unchanged, tangents rotated
    rng = np.random.default_rng(5)
    q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    h, _ = gen.fourier_knot(300, seed=2)[:2]
    hg, _ = lp.hierarchy(h, n_min=80)
    hr, _ = lp.hierarchy(h @ q.T + 1.0, n_min=80)
    F1 = lp.features(hg, lp.level_diagonals(hg, 2.0, 4.5))
    F2 = lp.features(hr, lp.level_diagonals(hr, 2.0, 4.5))
    s = [0, 1, 2, 6, 7]
    assert np.allclose(F1[:, s], F2[:, s], atol=1e-8)
    assert np.allclose(F1[:, 3:6] @ q.T, F2[:, 3:6], atol=1e-10)


def test_loss_gradient_matches_central_differences():
    g, e, _ = gen.fourier_knot(64, seed=6)
    A = sum(sobolev.assemble(g, e, 2.0, 4.5))
    x0, _, _ = cons.reference_values(g, e)
    _, C = cons.evaluate(g, e, cons.BARYCENTER, x0)
    _, dE = tpe.differential(g, e, 2.0, 4.5)
    g_ref, _ = solve.projected_gradient(A, C, dE)
    theta = lp.init_params(7) + 0.02 * np.random.default_rng(8).normal(size=lp.n_params())
    loss, grad = lp.loss_and_grad(theta, g, dE, g_ref, A, C, 2.0, 4.5, n_min=16)
    assert 0 < loss < 1
    h = 1e-6
    for k in [0, 100, 600, 1000, 4000, lp.n_params() - 5, lp.n_params() - 1]:
        tp, tm = theta.copy(), theta.copy()
        tp[k] += h
        tm[k] -= h
        fd = (lp.loss_and_grad(tp, g, dE, g_ref, A, C, 2.0, 4.5, n_min=16)[0]
              - lp.loss_and_grad(tm, g, dE, g_ref, A, C, 2.0, 4.5, n_min=16)[0]) / (2 * h)
        assert grad[k] == pytest.approx(fd, rel=1e-5, abs=1e-10)
