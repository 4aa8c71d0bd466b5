"""Fractional Sobolev-Slobodeckij Gram matrices B and B0, in float64 (oracle).

Test infrastructure only (see the package docstring).

Definitions followed (paper Sec. 4.2 "Discrete Inner Product"):

* Orders: ``s = (beta - 1) / alpha`` (Sec. 3.2.1 / Lemma FiniteTangentPointEnergy)
  and ``sigma = s - 1``.
* Sec. 4.2.1: derivative of a vertex function on edge I is
  ``D_I u = (u_i2 - u_i1) / l_I * T_I``.
* Sec. 4.2.2, eq. DiscreteHighOrderPart: with
  ``w_IJ = 1/4 l_I l_J sum_{i in I, j in J} |g_i - g_j|^-(2 sigma + 1)``,
  ``u^T B v = sum_{disjoint I,J} w_IJ <D_I u - D_J u, D_I v - D_J v>`` and B is
  built by the printed increments over every ordered disjoint pair and every
  ``a, b in {1, 2}``.
* Sec. 4.2.3: with ``w0_IJ = 1/4 l_I l_J sum k_{2,4}(g_i, g_j, T_I) / |g_i - g_j|^(2 sigma + 1)``,
  ``u^T B0 v = sum w0_IJ (u_I - u_J)(v_I - v_J)`` (u_I the edge average) and B0
  is built by its printed +-w0/4 increments.  The low-order kernel is the
  (alpha, beta) = (2, 4) tangent-point kernel whatever the energy's exponents.
* Eq. VectorInnerProduct: ``A = B + B0`` acts on each coordinate component.
* App. B.3.4, eqs. LowOrderDecomposition / LowOrderKernel: the kernel-matrix
  form ``B0 u = E^T (diag(K 1) - K) E u`` with
  ``K_IJ = (k_{2,2 sigma+5}(x_I, x_J, T_I) + k_{2,2 sigma+5}(x_J, x_I, T_J)) l_I l_J``,
  and B likewise with the difference operator D and ``k_{0, 2 sigma + 1}``.
  This form samples the kernel at edge midpoints; ``assemble(...,
  quadrature="midpoint")`` gives the increment construction with the same
  midpoint weights so the two passages can be checked against each other.
"""

from __future__ import annotations

import numpy as np

from .tpe import edge_geometry, _disjoint

__all__ = [
    "orders",
    "assemble",
    "assemble_rows",
    "apply",
    "quad_high",
    "quad_low",
    "kernel_matrix_apply",
]


def orders(alpha, beta):
    """(s, sigma) with s = (beta-1)/alpha and sigma = s - 1."""
    s = (beta - 1.0) / alpha
    return s, s - 1.0


def _k24_over(d, T, expo):
    """k_{2,4}(p, q, T) / |p - q|^expo with d = p - q."""
    c = np.cross(T, d)
    r = np.linalg.norm(d, axis=-1)
    return np.einsum("...k,...k->...", c, c) / r ** 4 / r ** expo


def _weights(gamma, edges, alpha, beta, rows, cols, quadrature):
    """(w, w0, mask) for the ordered pairs rows x cols."""
    g = np.asarray(gamma, dtype=np.float64)
    e = np.asarray(edges)
    ell, T, x = edge_geometry(g, e)
    _, sigma = orders(alpha, beta)
    expo = 2.0 * sigma + 1.0
    mask = _disjoint(e, rows, cols)
    lIlJ = ell[rows][:, None] * ell[cols][None, :]
    TI = np.broadcast_to(T[rows][:, None, :], mask.shape + (3,))
    if quadrature == "trapezoid":
        acc, acc0 = np.zeros(mask.shape), np.zeros(mask.shape)
        for a in range(2):
            for b in range(2):
                d = g[e[rows, a]][:, None, :] - g[e[cols, b]][None, :, :]
                d = np.broadcast_to(d, mask.shape + (3,)).copy()
                d[~mask] = 1.0
                acc += np.linalg.norm(d, axis=-1) ** (-expo)
                acc0 += _k24_over(d, TI, expo)
        w = 0.25 * lIlJ * acc
        w0 = 0.25 * lIlJ * acc0
    elif quadrature == "midpoint":
        d = np.broadcast_to(x[rows][:, None, :] - x[cols][None, :, :], mask.shape + (3,)).copy()
        d[~mask] = 1.0
        w = lIlJ * np.linalg.norm(d, axis=-1) ** (-expo)
        w0 = lIlJ * _k24_over(d, TI, expo)
    else:
        raise ValueError(quadrature)
    return np.where(mask, w, 0.0), np.where(mask, w0, 0.0), mask


def _increments(gamma, edges, alpha, beta, rows, cols, quadrature):
    """Yield (row_index, col_index, value, part) of the printed increment tables."""
    e = np.asarray(edges)
    ell, T, _ = edge_geometry(gamma, e)
    w, w0, mask = _weights(gamma, e, alpha, beta, rows, cols, quadrature)
    II, JJ = np.nonzero(mask)
    I, J = rows[II], cols[JJ]
    wij, w0ij = w[II, JJ], w0[II, JJ]
    lI, lJ = ell[I], ell[J]
    TT = np.einsum("nk,nk->n", T[I], T[J])
    for a in range(2):
        for b in range(2):
            sgn = (-1.0) ** (a + b)
            ia, ib, ja, jb = e[I, a], e[I, b], e[J, a], e[J, b]
            # high-order table (Sec. 4.2.2)
            yield ia, ib, sgn * wij / lI ** 2, "B"
            yield ia, jb, -sgn * wij * TT / (lI * lJ), "B"
            yield ja, jb, sgn * wij / lJ ** 2, "B"
            yield ja, ib, -sgn * wij * TT / (lJ * lI), "B"
            # low-order table (Sec. 4.2.3)
            yield ia, ib, 0.25 * w0ij, "B0"
            yield ia, jb, -0.25 * w0ij, "B0"
            yield ja, ib, -0.25 * w0ij, "B0"
            yield ja, jb, 0.25 * w0ij, "B0"


def assemble(gamma, edges, alpha, beta, quadrature="trapezoid", chunk=128):
    """Dense (B, B0) in R^{|V| x |V|} from the increment tables."""
    nV, nE = len(gamma), len(edges)
    B, B0 = np.zeros((nV, nV)), np.zeros((nV, nV))
    cols = np.arange(nE)
    for s in range(0, nE, chunk):
        rows = np.arange(s, min(nE, s + chunk))
        for r, c, v, part in _increments(gamma, edges, alpha, beta, rows, cols, quadrature):
            np.add.at(B if part == "B" else B0, (r, c), v)
    return B, B0


def assemble_rows(gamma, edges, alpha, beta, vertices, quadrature="trapezoid"):
    """Rows ``vertices`` of A = B + B0, built from the increments that land in them.

    An increment lands in row v only when v is an endpoint of I or of J, so it
    is enough to visit the pairs with I incident to v and those with J
    incident to v (never both: the pairs are disjoint).
    """
    e = np.asarray(edges)
    nV = len(gamma)
    out = np.zeros((len(vertices), nV))
    allE = np.arange(len(e))
    for n, v in enumerate(vertices):
        inc = np.nonzero((e[:, 0] == v) | (e[:, 1] == v))[0]
        for rows, cols in ((inc, allE), (allE, inc)):
            for r, c, val, _ in _increments(gamma, e, alpha, beta, rows, cols, quadrature):
                sel = r == v
                np.add.at(out[n], c[sel], val[sel])
    return out


def apply(gamma, edges, alpha, beta, X):
    """A X for X in R^{|V| x m} (components share A, eq. VectorInnerProduct)."""
    B, B0 = assemble(gamma, edges, alpha, beta)
    return (B + B0) @ X


def quad_high(gamma, edges, alpha, beta, u, v=None):
    """The printed bilinear form sum w_IJ <D_I u - D_J u, D_I v - D_J v>."""
    v = u if v is None else v
    e = np.asarray(edges)
    ell, T, _ = edge_geometry(gamma, e)
    idx = np.arange(len(e))
    w, _, _ = _weights(gamma, e, alpha, beta, idx, idx, "trapezoid")
    Du = ((u[e[:, 1]] - u[e[:, 0]]) / ell)[:, None] * T
    Dv = ((v[e[:, 1]] - v[e[:, 0]]) / ell)[:, None] * T
    diffu = Du[:, None, :] - Du[None, :, :]
    diffv = Dv[:, None, :] - Dv[None, :, :]
    return float((w * np.einsum("ijk,ijk->ij", diffu, diffv)).sum())


def quad_low(gamma, edges, alpha, beta, u, v=None):
    """The printed bilinear form sum w0_IJ (u_I - u_J)(v_I - v_J)."""
    v = u if v is None else v
    e = np.asarray(edges)
    idx = np.arange(len(e))
    _, w0, _ = _weights(gamma, e, alpha, beta, idx, idx, "trapezoid")
    uI = 0.5 * (u[e[:, 0]] + u[e[:, 1]])
    vI = 0.5 * (v[e[:, 0]] + v[e[:, 1]])
    return float((w0 * (uI[:, None] - uI[None, :]) * (vI[:, None] - vI[None, :])).sum())


def kernel_matrix_apply(gamma, edges, alpha, beta, u):
    """(B_mid + B0_mid) u through the kernel-matrix form of App. B.3.4.

    Low order: ``E^T (diag(K 1) - K) E u`` with the k_{2, 2 sigma + 5} kernel
    matrix; high order: ``D^T (diag(K 1) - K) D u`` with the k_{0, 2 sigma + 1}
    kernel matrix acting on each of the three components of D u.
    Non-disjoint pairs are left out of K, as they are from the energy.
    """
    g = np.asarray(gamma, dtype=np.float64)
    e = np.asarray(edges)
    nV, nE = len(g), len(e)
    ell, T, x = edge_geometry(g, e)
    _, sigma = orders(alpha, beta)
    idx = np.arange(nE)
    mask = _disjoint(e, idx, idx)
    d = x[:, None, :] - x[None, :, :]
    d[~mask] = 1.0
    r = np.linalg.norm(d, axis=-1)
    c_IJ = np.cross(np.broadcast_to(T[:, None, :], d.shape), d)
    c_JI = np.cross(np.broadcast_to(T[None, :, :], d.shape), -d)
    k_lo = (np.einsum("ijk,ijk->ij", c_IJ, c_IJ) + np.einsum("ijk,ijk->ij", c_JI, c_JI)) / r ** (2 * sigma + 5)
    K_lo = np.where(mask, k_lo * ell[:, None] * ell[None, :], 0.0)
    k_hi = 2.0 / r ** (2 * sigma + 1)
    K_hi = np.where(mask, k_hi * ell[:, None] * ell[None, :], 0.0)
    Eavg = np.zeros((nE, nV))
    Eavg[idx, e[:, 0]] += 0.5
    Eavg[idx, e[:, 1]] += 0.5
    Dm = np.zeros((nE, 3, nV))
    for c in range(3):
        Dm[idx, c, e[:, 0]] -= T[:, c] / ell
        Dm[idx, c, e[:, 1]] += T[:, c] / ell
    low = Eavg.T @ ((np.diag(K_lo.sum(1)) - K_lo) @ (Eavg @ u))
    Du = np.einsum("ecv,v->ec", Dm, u)
    KD = (np.diag(K_hi.sum(1)) - K_hi) @ Du
    high = np.einsum("ecv,ec->v", Dm, KD)
    return high + low
