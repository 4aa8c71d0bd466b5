"""Pins of the penalty oracle (oracle/penalties.py, Sec. 7.1).

* Closed forms on a regular n-gon of circumradius R in the xy-plane:
  total length 2 n R sin(pi / n); length difference 0; field potential the
  perimeter for X normal to the plane, and half of it for X in the plane
  (sum_k sin^2(phi + 2 pi k / n) = n / 2 for n >= 3).
* An open path: only its interior vertices (degree two) enter the length
  difference, and a hand-computed three-edge case.
* Scaling: total length and field potential scale by lambda, the length
  difference by lambda^2; all three are invariant under translations and the
  field potential under rotations that fix X.
* Differentials against central differences of the energies.
"""

import numpy as np
import pytest

import gen
from oracle import penalties as pen


def ngon(n, R=1.3, phase=0.2):
    t = phase + 2 * np.pi * np.arange(n) / n
    g = np.stack([R * np.cos(t), R * np.sin(t), np.zeros(n)], 1)
    e = np.stack([np.arange(n), (np.arange(n) + 1) % n], 1)
    return g, e


@pytest.mark.parametrize("n", [3, 7, 64])
def test_regular_polygon_closed_forms(n):
    R = 1.3
    g, e = ngon(n, R)
    L = 2 * n * R * np.sin(np.pi / n)
    assert pen.total_length(g, e)[0] == pytest.approx(L, rel=1e-14)
    assert pen.length_difference(g, e)[0] == pytest.approx(0.0, abs=1e-24)
    assert pen.field_potential(g, e, [0, 0, 2.0])[0] == pytest.approx(L, rel=1e-14)
    assert pen.field_potential(g, e, [1.0, 0.3, 0])[0] == pytest.approx(L / 2, rel=1e-12)


def test_open_path_hand_case():
    g = np.array([[0, 0, 0], [1, 0, 0], [1, 2, 0], [1, 2, 3.0]])
    e = np.array([[0, 1], [1, 2], [2, 3]])
    # lengths 1, 2, 3; interior vertices 1 and 2: (1 - 2)^2 + (2 - 3)^2
    assert pen.length_difference(g, e)[0] == pytest.approx(2.0, rel=1e-15)
    assert pen.total_length(g, e)[0] == pytest.approx(6.0, rel=1e-15)
    # X = e_x: only the second and third edges are not parallel to it
    assert pen.field_potential(g, e, [1, 0, 0])[0] == pytest.approx(5.0, rel=1e-15)


def test_scaling_and_invariance():
    g, e, _ = gen.fourier_knot(50, seed=3)
    X = np.array([0.3, -0.5, 0.8])
    lam, t = 1.7, np.array([0.2, -1.0, 3.0])
    for f, k in ((lambda h: pen.total_length(h, e)[0], 1), (lambda h: pen.length_difference(h, e)[0], 2),
                 (lambda h: pen.field_potential(h, e, X)[0], 1)):
        assert f(lam * g + t) == pytest.approx(lam ** k * f(g), rel=1e-12)
    # a rotation about X leaves the field potential unchanged
    x = X / np.linalg.norm(X)
    K = np.array([[0, -x[2], x[1]], [x[2], 0, -x[0]], [-x[1], x[0], 0]])
    Q = np.eye(3) + np.sin(0.7) * K + (1 - np.cos(0.7)) * K @ K
    assert pen.field_potential(g @ Q.T, e, X)[0] == pytest.approx(pen.field_potential(g, e, X)[0], rel=1e-12)


def test_differentials_match_central_differences():
    g, e, _ = gen.fourier_knot(30, seed=5)
    g2 = np.concatenate([g, np.array([[3.0, 0, 0], [3.5, 0.2, 0.1], [4.0, -0.3, 0.4], [4.2, 0.5, 0.9]])])
    e2 = np.concatenate([e, np.array([[30, 31], [31, 32], [32, 33]])])
    X = [0.2, 0.9, -0.4]
    for f in (lambda h: pen.total_length(h, e2), lambda h: pen.length_difference(h, e2),
              lambda h: pen.field_potential(h, e2, X),
              lambda h: pen.penalties(h, e2, 0.5, 2.0, 1.5, X)):
        _, d = f(g2)
        h = 1e-6
        for v in (0, 7, 29, 30, 31, 33):
            for c in range(3):
                gp, gm = g2.copy(), g2.copy()
                gp[v, c] += h
                gm[v, c] -= h
                fd = (f(gp)[0] - f(gm)[0]) / (2 * h)
                assert d[v, c] == pytest.approx(fd, rel=1e-6, abs=1e-8)
