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
* Triangulated-surface potential: the generated meshes' areas; on refined
  spheres the centroid-quadrature field converges at second order to the
  closed-form shell potential of the sphere obstacle; its differential against
  central differences; scaling lambda^(3 - p) and rigid-motion invariance.
"""

import numpy as np
import pytest

import gen
from oracle import obstacle
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


# --- triangulated-surface potential (Sec. 7.1) -------------------------------


def test_triangle_samples_and_meshes():
    P, F = gen.icosphere(3, radius=0.5)
    cT, AT = pen.triangle_samples(P, F)
    assert len(F) == 8 * 4 ** 3 and np.allclose(np.linalg.norm(P, axis=1), 0.5)
    # inscribed polyhedron: its area approaches 4 pi R^2 from below
    assert 0.97 * np.pi < AT.sum() < np.pi
    P, F = gen.torus_mesh(64, 32, R=1.0, r=0.3)
    _, AT = pen.triangle_samples(P, F)
    assert AT.sum() == pytest.approx(4 * np.pi ** 2 * 1.0 * 0.3, rel=5e-3)


@pytest.mark.parametrize("p", [2.0, 2.5])
def test_surface_field_converges_to_the_sphere_closed_form(p):
    """On a refined triangulated sphere the centroid-quadrature field approaches the shell
    potential's closed form (the sphere obstacle's) at second order in the mesh size."""
    x = np.array([[1.7, 0.2, -0.3], [0.0, 0.0, 2.5]])
    exact = obstacle.shell_potential(np.linalg.norm(x, axis=1), 1.0, p)
    errs = []
    for lev in (3, 4, 5):
        P, F = gen.icosphere(lev)
        phi, _ = pen.surface_field(x, P, F, p)
        errs.append(np.abs(phi / exact - 1).max())
    # second order in the mesh size (each level halves it): the error falls about 4x per level
    assert 3.5 < errs[0] / errs[1] < 4.5 and 3.5 < errs[1] / errs[2] < 4.5 and errs[2] < 1.5e-3


def test_surface_potential_differential_and_scaling():
    g, e = gen.trefoil(24, seed=1)
    g = 0.3 * g + [0.0, 0.0, 2.2]
    P, F = gen.torus_mesh(12, 8, R=1.0, r=0.3)
    E, d = pen.surface_potential(g, e, P, F, 2.5)
    h = 1e-6
    for v, c in [(0, 0), (5, 2), (17, 1)]:
        gp, gm = g.copy(), g.copy()
        gp[v, c] += h
        gm[v, c] -= h
        fd = (pen.surface_potential(gp, e, P, F, 2.5)[0] - pen.surface_potential(gm, e, P, F, 2.5)[0]) / (2 * h)
        assert d[v, c] == pytest.approx(fd, rel=1e-6, abs=1e-9 * np.abs(d).max())
    # E(lambda gamma, lambda M) = lambda^(1 + 2 - p) E; a rigid motion of both leaves it unchanged
    assert pen.surface_potential(1.7 * g, e, 1.7 * P, F, 2.5)[0] == pytest.approx(1.7 ** 0.5 * E, rel=1e-12)
    q, _ = np.linalg.qr(np.random.default_rng(2).normal(size=(3, 3)))
    assert pen.surface_potential(g @ q.T + 1.0, e, P @ q.T + 1.0, F, 2.5)[0] == pytest.approx(E, rel=1e-12)
