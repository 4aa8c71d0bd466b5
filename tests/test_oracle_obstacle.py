"""Pins of the sphere-obstacle potential (Sec. 7.1, surface potential).

The closed-form shell integral is checked against a direct quadrature of the
surface integral over a fine Fibonacci point set on the sphere (equal-area
weights), and its penalty gradient against central differences.
"""

import numpy as np
import pytest

import gen
from oracle import obstacle


def fibonacci_sphere(n, R, c):
    i = np.arange(n) + 0.5
    phi = np.arccos(1 - 2 * i / n)
    th = np.pi * (1 + 5 ** 0.5) * i
    pts = np.stack([np.cos(th) * np.sin(phi), np.sin(th) * np.sin(phi), np.cos(phi)], 1)
    return c + R * pts, 4 * np.pi * R ** 2 / n


@pytest.mark.parametrize("p", [2.0, 2.5, 3.0])
def test_shell_closed_form_vs_quadrature(p):
    R, c = 0.25, np.array([0.5, 0.5, 0.5])
    pts, w = fibonacci_sphere(400_000, R, c)
    for r in (0.3, 0.45, 0.9):
        x = c + r * np.array([0.36, 0.48, 0.8])
        quad = w * np.sum(np.linalg.norm(pts - x, axis=1) ** (-p))
        assert obstacle.shell_potential(r, R, p) == pytest.approx(quad, rel=2e-4)


def test_shell_p3_simplifies():
    # p = 3: Psi(r) = 4 pi R^2 / (r (r^2 - R^2))
    r, R = np.linspace(0.3, 2.0, 7), 0.25
    assert np.allclose(obstacle.shell_potential(r, R, 3.0), 4 * np.pi * R ** 2 / (r * (r ** 2 - R ** 2)))


@pytest.mark.parametrize("p", [2.0, 3.0])
def test_penalty_gradient_central_differences(p):
    rng = np.random.default_rng(0)
    g, e = gen.regular_ngon(12, radius=0.15)
    g = g + [0.5, 0.5, 0.95] + 0.01 * rng.normal(size=g.shape)
    c, R = [0.5, 0.5, 0.5], 0.25
    G = obstacle.penalty_gradient(g, e, c, R, p)
    X = rng.normal(size=g.shape)
    h = 1e-6
    fd = (obstacle.penalty(g + h * X, e, c, R, p) - obstacle.penalty(g - h * X, e, c, R, p)) / (2 * h)
    assert np.sum(G * X) == pytest.approx(fd, rel=1e-7)
