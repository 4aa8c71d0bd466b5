"""Curve penalties of Sec. 7.1, in float64 (oracle).

Test infrastructure only (see the package docstring).

Three soft terms that are added to the tangent-point energy (Sec. 7.1,
penalties), each with its differential with respect to the vertex positions:

* total length: sum over edges of l_I;
* length difference: sum over vertices v of degree two of (l_I - l_J)^2,
  I and J the two edges at v;
* field potential: sum over edges of l_I |T_I x X|^2 for a fixed unit vector
  X (a constant field; the paper's field is sampled at the edge midpoint,
  and a constant field does not depend on it);
* surface potential of a triangulated surface M (vertices P, triangles F):
  the double integral of |x_M - gamma|^-p, p = beta - alpha, over the curve
  and M, with one sample per edge (its midpoint x_I, weight l_I) and one per
  triangle (its centroid c_T, weight its area A_T):
  sum_I l_I phi(x_I), phi(x) = sum_T A_T |c_T - x|^-p.

The differentials follow from dl_I = T_I . (d gamma_i2 - d gamma_i1) and
dT_I = (I - T_I T_I^T)(d gamma_i2 - d gamma_i1) / l_I.
"""

from __future__ import annotations

import numpy as np

from .tpe import edge_geometry

__all__ = ["total_length", "length_difference", "field_potential", "penalties", "triangle_samples",
           "surface_field", "surface_potential"]


def _scatter(edges, nV, gI):
    """Vertex differential from per-edge gradients g_I with respect to the
    edge vector e_I = gamma_i2 - gamma_i1."""
    d = np.zeros((nV, 3))
    np.add.at(d, edges[:, 1], gI)
    np.add.at(d, edges[:, 0], -gI)
    return d


def total_length(gamma, edges):
    g, e = np.asarray(gamma, dtype=np.float64), np.asarray(edges)
    ell, T, _ = edge_geometry(g, e)
    return float(ell.sum()), _scatter(e, len(g), T)


def length_difference(gamma, edges):
    g, e = np.asarray(gamma, dtype=np.float64), np.asarray(edges)
    nV = len(g)
    ell, T, _ = edge_geometry(g, e)
    inc = [[] for _ in range(nV)]
    for I, (a, b) in enumerate(e):
        inc[a].append(I)
        inc[b].append(I)
    E = 0.0
    dl = np.zeros(len(e))  # dE / dl_I
    for v in range(nV):
        if len(inc[v]) != 2:
            continue
        I, J = inc[v]
        diff = ell[I] - ell[J]
        E += diff * diff
        dl[I] += 2.0 * diff
        dl[J] -= 2.0 * diff
    return float(E), _scatter(e, nV, dl[:, None] * T)


def field_potential(gamma, edges, X):
    g, e = np.asarray(gamma, dtype=np.float64), np.asarray(edges)
    X = np.asarray(X, dtype=np.float64)
    X = X / np.linalg.norm(X)
    ell, T, _ = edge_geometry(g, e)
    c = np.cross(T, X)
    E = float((ell * (c * c).sum(1)).sum())
    # l |T x X|^2 = l - (T.X)^2 l; with e = l T: d/de = T - 2 (T.X) X + (T.X)^2 T
    tx = T @ X
    gI = T - 2.0 * tx[:, None] * X[None, :] + (tx * tx)[:, None] * T
    return E, _scatter(e, len(g), gI)


def penalties(gamma, edges, w_length=0.0, w_diff=0.0, w_field=0.0, X=(0.0, 0.0, 1.0)):
    """Weighted sum of the three penalties and its differential."""
    g = np.asarray(gamma, dtype=np.float64)
    E, d = 0.0, np.zeros_like(g)
    for w, f in ((w_length, lambda: total_length(g, edges)), (w_diff, lambda: length_difference(g, edges)),
                 (w_field, lambda: field_potential(g, edges, X))):
        if w != 0.0:
            e_, d_ = f()
            E += w * e_
            d += w * d_
    return E, d


def triangle_samples(P, F):
    """Centroids c_T [nF][3] and areas A_T [nF] of the triangles F of the vertices P."""
    P = np.asarray(P, dtype=np.float64)
    F = np.asarray(F)
    a, b, c = P[F[:, 0]], P[F[:, 1]], P[F[:, 2]]
    return (a + b + c) / 3.0, 0.5 * np.linalg.norm(np.cross(b - a, c - a), axis=1)


def surface_field(x, P, F, p):
    """phi(x) = sum_T A_T |c_T - x|^-p at the points x [m][3], and its gradient
    p sum_T A_T |c_T - x|^(-p-2) (c_T - x)."""
    cT, AT = triangle_samples(P, F)
    x = np.asarray(x, dtype=np.float64).reshape(-1, 3)
    phi = np.zeros(len(x))
    grad = np.zeros((len(x), 3))
    for k in range(len(x)):
        d = cT - x[k]
        r2 = (d * d).sum(1)
        phi[k] = (AT * r2 ** (-0.5 * p)).sum()
        grad[k] = p * ((AT * r2 ** (-0.5 * p - 1.0))[:, None] * d).sum(0)
    return phi, grad


def surface_potential(gamma, edges, P, F, p):
    """E = sum_I l_I phi(x_I) and its vertex differential: at the edge's ends
    -+T_I phi(x_I) + (l_I / 2) grad phi(x_I) (x_I moves by half of each end)."""
    g, e = np.asarray(gamma, dtype=np.float64), np.asarray(edges)
    ell, T, x = edge_geometry(g, e)
    phi, grad = surface_field(x, P, F, p)
    E = float((ell * phi).sum())
    d = np.zeros_like(g)
    half = 0.5 * ell[:, None] * grad
    np.add.at(d, e[:, 1], T * phi[:, None] + half)
    np.add.at(d, e[:, 0], -T * phi[:, None] + half)
    return E, d
