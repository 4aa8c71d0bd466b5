"""Discrete tangent-point energy and its differential, in float64 (oracle).

Test infrastructure only (see the package docstring).

Definitions followed (paper Sec. 4, "Discretization"):

* Notation paragraph: for an edge I = (i1, i2),
  ``l_I = |g_i1 - g_i2|``, ``T_I = (g_i2 - g_i1) / l_I``, ``x_I = (g_i1 + g_i2)/2``.
* Eq. TangentPointKernel: ``k(p, q, T) = |T x (p - q)|^alpha / |p - q|^beta``.
* Eqs. DiscreteEnergy / DiscreteKernel: the energy is the double sum over
  ordered pairs of edges that share no vertex,
  ``E = sum_{I,J, I cap J = empty} l_I l_J * 1/4 sum_{i in I} sum_{j in J} k(g_i, g_j, T_I)``.
  Pairs sharing a vertex (I = J included) are omitted.
* Sec. 4.1: the differential is the vector of exact partial derivatives of
  that energy with respect to every vertex coordinate.  Here they are derived
  by hand with the chain rule through ``p``, ``q``, ``l_I``, ``l_J`` and
  ``T_I``, and scattered per ordered pair onto all four vertices.

The edge-midpoint variant ``E_mid = sum_{disjoint I,J} k(x_I, x_J, T_I) l_I l_J``
is the sum that the Barnes-Hut scheme of App. B.1.2 approximates; with the
admissibility parameter taken to zero every source edge is visited directly
and the scheme reproduces exactly this sum and its derivative.
"""

from __future__ import annotations

import numpy as np

__all__ = [
    "edge_geometry",
    "kernel",
    "energy",
    "differential",
    "energy_rows",
    "differential_at",
    "midpoint_energy",
    "midpoint_differential",
    "midpoint_rows",
]


def edge_geometry(gamma, edges):
    """Edge length, unit tangent and midpoint (Sec. 4, Notation)."""
    g = np.asarray(gamma, dtype=np.float64)
    e = np.asarray(edges)
    d = g[e[:, 1]] - g[e[:, 0]]
    ell = np.linalg.norm(d, axis=1)
    T = d / ell[:, None]
    x = 0.5 * (g[e[:, 0]] + g[e[:, 1]])
    return ell, T, x


def kernel(p, q, T, alpha, beta):
    """Tangent-point kernel |T x (p-q)|^alpha / |p-q|^beta (eq. TangentPointKernel)."""
    d = np.asarray(p, dtype=np.float64) - np.asarray(q, dtype=np.float64)
    c = np.cross(np.broadcast_to(T, d.shape), d)
    return np.linalg.norm(c, axis=-1) ** alpha / np.linalg.norm(d, axis=-1) ** beta


def _kernel_parts(d, T, alpha, beta):
    """k(d, T) and its partials with respect to d and to T (T not yet unit-constrained).

    With s = |T x d|^2 and r = |d|:  k = s^(alpha/2) r^(-beta),
    dk/dd = (alpha/2) s^(alpha/2-1) r^(-beta) ds/dd - beta k d / r^2,
    dk/dT = (alpha/2) s^(alpha/2-1) r^(-beta) ds/dT,
    ds/dd = 2 (|T|^2 d - (T.d) T),  ds/dT = 2 (|d|^2 T - (T.d) d).
    Where s = 0 the factor s^(alpha/2-1) multiplies a zero vector; the product
    is taken as 0 (its limit for alpha > 1).
    """
    c = np.cross(T, d)
    s = np.einsum("...k,...k->...", c, c)
    r2 = np.einsum("...k,...k->...", d, d)
    t = np.einsum("...k,...k->...", T, d)
    tt = np.einsum("...k,...k->...", T, T)
    rb = r2 ** (-0.5 * beta)
    k = s ** (0.5 * alpha) * rb
    with np.errstate(divide="ignore", invalid="ignore"):
        f = np.where(s > 0, 0.5 * alpha * s ** (0.5 * alpha - 1.0), 1.0 if alpha == 2 else 0.0)
    f = f * rb
    ds_dd = 2.0 * (tt[..., None] * d - t[..., None] * T)
    ds_dT = 2.0 * (r2[..., None] * T - t[..., None] * d)
    dk_dd = f[..., None] * ds_dd - (beta * k / r2)[..., None] * d
    dk_dT = f[..., None] * ds_dT
    return k, dk_dd, dk_dT


def _disjoint(edges, rows, cols):
    e = np.asarray(edges)
    a1, a2 = e[rows, 0][:, None], e[rows, 1][:, None]
    b1, b2 = e[cols, 0][None, :], e[cols, 1][None, :]
    return (a1 != b1) & (a1 != b2) & (a2 != b1) & (a2 != b2)


def _block(gamma, edges, alpha, beta, rows, cols, want_grad, per_row=False):
    """Energy (and scattered differential) of the ordered pairs rows x cols."""
    g = np.asarray(gamma, dtype=np.float64)
    e = np.asarray(edges)
    ell, T, _ = edge_geometry(g, e)
    mask = _disjoint(e, rows, cols)
    lI, lJ = ell[rows][:, None], ell[cols][None, :]
    TI = np.broadcast_to(T[rows][:, None, :], (len(rows), len(cols), 3))
    # kernel sum over the four vertex pairs (i_a, j_b); d = g_ia - g_jb
    K = np.zeros(mask.shape)
    pos = [np.zeros(mask.shape + (3,)) for _ in range(2)]    # sum_b dk/dd at i_a
    neg = [np.zeros(mask.shape + (3,)) for _ in range(2)]    # sum_a dk/dd at j_b
    dT = np.zeros(mask.shape + (3,))
    for a in range(2):
        p = g[e[rows, a]][:, None, :]
        for b in range(2):
            q = g[e[cols, b]][None, :, :]
            d = np.broadcast_to(p - q, mask.shape + (3,)).copy()
            d[~mask] = 1.0  # excluded pairs: any finite stand-in, zeroed below
            k, dk_dd, dk_dT = _kernel_parts(d, TI, alpha, beta)
            K += k
            if want_grad:
                pos[a] += dk_dd
                neg[b] += dk_dd
                dT += dk_dT
    K = np.where(mask, K, 0.0)
    if per_row:
        return (0.25 * lI * lJ * K).sum(axis=1)
    E = float((0.25 * lI * lJ * K).sum())
    if not want_grad:
        return E, None
    grad = np.zeros_like(g)
    m = mask[..., None]
    # target side: g_ia enters p, l_I and T_I
    Tr = T[rows][:, None, :]
    proj = dT - np.einsum("ijk,ijk->ij", dT, np.broadcast_to(Tr, dT.shape))[..., None] * Tr
    for a, sgn in ((0, -1.0), (1, 1.0)):
        c = (0.25 * lJ)[..., None] * (sgn * Tr * K[..., None] + lI[..., None] * pos[a] + sgn * proj)
        np.add.at(grad, e[rows, a], np.where(m, c, 0.0).sum(axis=1))
    # source side: g_jb enters q (with a minus sign) and l_J
    Tc = T[cols][None, :, :]
    for b, sgn in ((0, -1.0), (1, 1.0)):
        c = (0.25 * lI)[..., None] * (sgn * Tc * K[..., None] - lJ[..., None] * neg[b])
        np.add.at(grad, e[cols, b], np.where(m, c, 0.0).sum(axis=0))
    return E, grad


def _chunks(n, size):
    for s in range(0, n, size):
        yield np.arange(s, min(n, s + size))


def energy(gamma, edges, alpha, beta, chunk=64):
    """Discrete energy (eq. DiscreteEnergy), summed over target chunks."""
    nE = len(edges)
    cols = np.arange(nE)
    return float(sum(_block(gamma, edges, alpha, beta, r, cols, False)[0]
                     for r in _chunks(nE, chunk)))


def differential(gamma, edges, alpha, beta, chunk=64):
    """Energy and exact differential dE in R^{|V| x 3} (Sec. 4.1)."""
    nE = len(edges)
    cols = np.arange(nE)
    E, G = 0.0, np.zeros((len(gamma), 3))
    for r in _chunks(nE, chunk):
        e, g = _block(gamma, edges, alpha, beta, r, cols, True)
        E += e
        G += g
    return E, G


def energy_rows(gamma, edges, alpha, beta, rows):
    """Per-target-edge energy ``sum_J l_I l_J khat_IJ`` for the listed edges I."""
    cols = np.arange(len(edges))
    return _block(gamma, edges, alpha, beta, np.asarray(rows), cols, False, per_row=True)


def differential_at(gamma, edges, alpha, beta, vertices):
    """dE at selected vertices only: the pairs in which a vertex takes part.

    A vertex v enters the ordered pair (I, J) only if v is an endpoint of I or
    of J, never both (they share no vertex), so dE_v is the scatter of the
    pairs with I incident to v plus the pairs with J incident to v.
    """
    e = np.asarray(edges)
    cols = np.arange(len(e))
    out = np.zeros((len(vertices), 3))
    for n, v in enumerate(vertices):
        inc = np.nonzero((e[:, 0] == v) | (e[:, 1] == v))[0]
        _, g1 = _block(gamma, e, alpha, beta, inc, cols, True)
        _, g2 = _block(gamma, e, alpha, beta, cols, inc, True)
        out[n] = g1[v] + g2[v]
    return out


# ---------------------------------------------------------------------------
# Edge-midpoint variant (App. B.1.2, the sum that Barnes-Hut approximates)
# ---------------------------------------------------------------------------

def _mid_block(gamma, edges, alpha, beta, rows, cols, want_grad):
    g = np.asarray(gamma, dtype=np.float64)
    e = np.asarray(edges)
    ell, T, x = edge_geometry(g, e)
    mask = _disjoint(e, rows, cols)
    d = np.broadcast_to(x[rows][:, None, :] - x[cols][None, :, :], mask.shape + (3,)).copy()
    d[~mask] = 1.0
    lI, lJ = ell[rows][:, None], ell[cols][None, :]
    TI = np.broadcast_to(T[rows][:, None, :], d.shape)
    k, dk_dd, dk_dT = _kernel_parts(d, TI, alpha, beta)
    k = np.where(mask, k, 0.0)
    rowE = (lI * lJ * k).sum(axis=1)
    if not want_grad:
        return rowE, None
    grad = np.zeros_like(g)
    m = mask[..., None]
    Tr = T[rows][:, None, :]
    proj = dk_dT - np.einsum("ijk,ijk->ij", dk_dT, np.broadcast_to(Tr, dk_dT.shape))[..., None] * Tr
    for a, sgn in ((0, -1.0), (1, 1.0)):
        # x_I = (g_i1 + g_i2)/2 ; l_I ; T_I
        c = lJ[..., None] * (sgn * Tr * k[..., None] + lI[..., None] * 0.5 * dk_dd + sgn * proj)
        np.add.at(grad, e[rows, a], np.where(m, c, 0.0).sum(axis=1))
    Tc = T[cols][None, :, :]
    for b, sgn in ((0, -1.0), (1, 1.0)):
        c = lI[..., None] * (sgn * Tc * k[..., None] - lJ[..., None] * 0.5 * dk_dd)
        np.add.at(grad, e[cols, b], np.where(m, c, 0.0).sum(axis=0))
    return rowE, grad


def midpoint_energy(gamma, edges, alpha, beta, chunk=64):
    nE = len(edges)
    cols = np.arange(nE)
    return float(sum(_mid_block(gamma, edges, alpha, beta, r, cols, False)[0].sum()
                     for r in _chunks(nE, chunk)))


def midpoint_differential(gamma, edges, alpha, beta, chunk=64):
    nE = len(edges)
    cols = np.arange(nE)
    E, G = 0.0, np.zeros((len(gamma), 3))
    for r in _chunks(nE, chunk):
        rowE, g = _mid_block(gamma, edges, alpha, beta, r, cols, True)
        E += rowE.sum()
        G += g
    return E, G


def midpoint_rows(gamma, edges, alpha, beta, rows):
    """Per-target-edge midpoint energy and the target's own endpoint partials.

    Returns ``(rowE, dI)`` where ``dI[n, a]`` is the partial of
    ``sum_J [e_IJ + e_JI]`` (midpoint rule) with respect to ``g_{i_a}`` for
    the n-th listed edge I: the per-target quantity a Barnes-Hut traversal
    accumulates.
    """
    e = np.asarray(edges)
    rows = np.asarray(rows)
    cols = np.arange(len(e))
    rowE, _ = _mid_block(gamma, e, alpha, beta, rows, cols, False)
    dI = np.zeros((len(rows), 2, 3))
    for n, I in enumerate(rows):
        one = np.array([I])
        _, g1 = _mid_block(gamma, e, alpha, beta, one, cols, True)
        _, g2 = _mid_block(gamma, e, alpha, beta, cols, one, True)
        for a in range(2):
            v = e[I, a]
            dI[n, a] = g1[v] + g2[v]
    return rowE, dI
