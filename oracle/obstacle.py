"""Sphere-obstacle surface potential, in float64 (oracle).

Test infrastructure only (see the package docstring).

Paper Sec. 7.1 ("Surface potential") penalises a curve near a surface M with
``E_M = int_gamma int_M |x_M - gamma|^-(beta - alpha) dx_M dx_gamma``.  For M a
sphere of radius R and centre c, the inner surface integral at a point at
distance r > R from c has a closed form (integrate over the polar angle with
``u = r^2 + R^2 - 2 r R cos(theta)``):

    Psi(r) = (pi R / r) [ u^(1 - p/2) / (1 - p/2) ]_{u=(r-R)^2}^{(r+R)^2},  p = beta - alpha,

and ``(pi R / r) ln((r+R)^2 / (r-R)^2)`` when p = 2.  The outer integral is
taken with one midpoint sample per edge, as the paper discretises its other
per-edge potentials: ``E_M = sum_I l_I Psi(|x_I - c|)``.
"""

from __future__ import annotations

import numpy as np

from .tpe import edge_geometry

__all__ = ["shell_potential", "shell_potential_deriv", "penalty", "penalty_gradient"]


def shell_potential(r, R, p):
    r = np.asarray(r, dtype=np.float64)
    lo, hi = (r - R) ** 2, (r + R) ** 2
    if p == 2:
        return np.pi * R / r * np.log(hi / lo)
    q = 1.0 - 0.5 * p
    return np.pi * R / r * (hi ** q - lo ** q) / q


def shell_potential_deriv(r, R, p):
    """dPsi/dr of the closed form above."""
    r = np.asarray(r, dtype=np.float64)
    lo, hi = (r - R) ** 2, (r + R) ** 2
    if p == 2:
        F = np.log(hi / lo)
        dF = 2.0 / (r + R) - 2.0 / (r - R)
    else:
        q = 1.0 - 0.5 * p
        F = (hi ** q - lo ** q) / q
        dF = 2.0 * (r + R) * hi ** (q - 1.0) - 2.0 * (r - R) * lo ** (q - 1.0)
    return np.pi * R * (dF / r - F / r ** 2)


def penalty(gamma, edges, center, R, p, weight=1.0):
    ell, _, x = edge_geometry(gamma, edges)
    r = np.linalg.norm(x - np.asarray(center), axis=1)
    return float(weight * (ell * shell_potential(r, R, p)).sum())


def penalty_gradient(gamma, edges, center, R, p, weight=1.0):
    """d/dgamma of ``sum_I l_I Psi(|x_I - c|)`` (chain rule through l_I and x_I)."""
    g = np.asarray(gamma, dtype=np.float64)
    e = np.asarray(edges)
    ell, T, x = edge_geometry(g, e)
    dx = x - np.asarray(center)
    r = np.linalg.norm(dx, axis=1)
    psi, dpsi = shell_potential(r, R, p), shell_potential_deriv(r, R, p)
    G = np.zeros_like(g)
    for a, sgn in ((0, -1.0), (1, 1.0)):
        c = sgn * T * psi[:, None] + (ell * dpsi / r)[:, None] * 0.5 * dx
        np.add.at(G, e[:, a], weight * c)
    return G
