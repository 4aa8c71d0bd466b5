"""Curve penalties of Sec. 7.1, in float64 (oracle).

Test infrastructure only (see the package docstring).

Three soft terms that are added to the tangent-point energy (Sec. 7.1,
penalties), each with its differential with respect to the vertex positions:

* total length: sum over edges of l_I;
* length difference: sum over vertices v of degree two of (l_I - l_J)^2,
  I and J the two edges at v;
* field potential: sum over edges of l_I |T_I x X|^2 for a fixed unit vector
  X (a constant field; the paper's field is sampled at the edge midpoint,
  and a constant field does not depend on it).

The differentials follow from dl_I = T_I . (d gamma_i2 - d gamma_i1) and
dT_I = (I - T_I T_I^T)(d gamma_i2 - d gamma_i1) / l_I.
"""

from __future__ import annotations

import numpy as np

from .tpe import edge_geometry

__all__ = ["total_length", "length_difference", "field_potential", "penalties"]


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
