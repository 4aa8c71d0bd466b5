"""Constraints Phi(gamma) = 0 and their exact Jacobians, in float64 (oracle).

Test infrastructure only (see the package docstring).

Definitions (paper Sec. 7.1 "Constraints and Potentials"):

* Barycenter: ``Phi_b = sum_I l_I (x_I - x_0)`` (3 rows, unnormalised as
  printed).  Its Jacobian block at vertex v is
  ``sum_{I incident to v} [ (l_I / 2) Id_3 +- (x_I - x_0) T_I^T ]`` with ``+``
  when v is the edge's second endpoint and ``-`` when it is the first, since
  ``dl_I/dg_i2 = T_I = -dl_I/dg_i1`` and ``dx_I/dg_ia = Id_3 / 2``.
* Total length: ``Phi_L = L0 - sum_I l_I`` (1 row).
* Edge length: ``Phi_I = l0_I - l_I`` (one row per edge) with Jacobian
  ``+T_I`` at i1 and ``-T_I`` at i2.
* Point: ``Phi_{point,i} = gamma_i - x_i`` (3 rows per pinned vertex i, in
  the order the vertices are given), whose Jacobian is the identity block at
  vertex i and zero elsewhere.
* Surface: ``Phi_{surface,i} = f(gamma_i)`` for an implicit surface f = 0 (1 row
  per listed vertex), Jacobian row ``grad f(gamma_i)^T`` at vertex i.  Two
  surfaces, each by its signed distance (so that |grad f| = 1 and Phi has units
  of length): a sphere ``f = |x - c| - r`` and a torus about the axis through c
  along z, ``f = sqrt((rho - R)^2 + (z - c_z)^2) - r`` with rho the distance
  from that axis.
* Tangent: the paper writes ``Phi_{tangent,I} = T_I - X`` (3 rows), whose
  Jacobian has rank 2 only (T_I stays a unit vector).  Read here as the two
  independent rows ``(u . T_I, v . T_I)`` with (u, v) an orthonormal basis of
  the plane orthogonal to the unit direction X: ``u = (X x e_m) / |X x e_m|``
  with e_m the coordinate axis of the smallest |X_m| (the first on ties) and
  ``v = X x u``.  They vanish exactly when T_I is parallel to X (the branch
  T_I . X > 0 is the one a step from near X stays on).  Jacobian of u . T_I:
  ``(u - (u . T_I) T_I) / l_I`` at i2 and its negative at i1.
* Loop length: the total-length constraint applied to every connected
  component (closed loop) separately, ``Phi_q = L0_q - sum_{I in q} l_I``
  (one row per component, components ordered by their smallest vertex), as a
  packing of several curves keeps each curve's length.

Rows are stacked in the order barycenter, total length, points, surface,
tangents, edge lengths, loop lengths.  Points are passed as
``points=(vertices, targets)``, surfaces as ``surface=(kind, params,
vertices)`` (kind SPHERE with params (c_x, c_y, c_z, r), or TORUS with
(c_x, c_y, c_z, R, r)) and tangents as ``tangent=(edges, directions)`` beside
the flags (no flag of their own: an empty list is no such constraint).
Vectors in R^{3|V|} are vertex-major: entry ``3 v + c`` is coordinate c of
vertex v.
"""

from __future__ import annotations

import numpy as np

from .tpe import edge_geometry

__all__ = ["BARYCENTER", "TOTAL_LENGTH", "EDGE_LENGTH", "LOOP_LENGTH", "SPHERE", "TORUS", "reference_values",
           "components", "loop_lengths", "surface_value", "tangent_basis", "evaluate", "jacobian_sparse"]

BARYCENTER = 1
TOTAL_LENGTH = 2
EDGE_LENGTH = 4
LOOP_LENGTH = 8
SPHERE = 1
TORUS = 2


def surface_value(kind, params, x):
    """(f(x), grad f(x)) of the implicit surface at the points x [m][3]."""
    x = np.asarray(x, dtype=np.float64).reshape(-1, 3)
    p = np.asarray(params, dtype=np.float64)
    d = x - p[:3]
    if kind == SPHERE:
        r = np.linalg.norm(d, axis=1)
        return r - p[3], d / r[:, None]
    if kind == TORUS:
        rho = np.hypot(d[:, 0], d[:, 1])
        a = rho - p[3]
        q = np.hypot(a, d[:, 2])
        grad = np.stack([a / q * d[:, 0] / rho, a / q * d[:, 1] / rho, d[:, 2] / q], axis=1)
        return q - p[4], grad
    raise ValueError("unknown surface kind")


def tangent_basis(X):
    """(u, v): the orthonormal basis of the plane orthogonal to the unit vector X
    used by the tangent rows (u = X x e_m / |X x e_m|, e_m the axis of the
    smallest |X_m|, first on ties; v = X x u)."""
    X = np.asarray(X, dtype=np.float64)
    X = X / np.linalg.norm(X)
    m = int(np.argmin(np.abs(X)))
    em = np.zeros(3)
    em[m] = 1.0
    u = np.cross(X, em)
    u /= np.linalg.norm(u)
    return u, np.cross(X, u)


def reference_values(gamma, edges):
    """(x0, L0, l0) of a curve: the targets that make Phi(gamma) = 0.

    ``x0`` is the length-weighted barycenter ``sum l_I x_I / sum l_I``.
    """
    ell, _, x = edge_geometry(gamma, edges)
    return (ell[:, None] * x).sum(0) / ell.sum(), float(ell.sum()), ell.copy()


def components(edges, n_vertices):
    """Component index of every edge, components numbered by their smallest vertex."""
    e = np.asarray(edges)
    parent = list(range(n_vertices))

    def find(v):
        while parent[v] != v:
            parent[v] = parent[parent[v]]
            v = parent[v]
        return v

    for a, b in e:
        ra, rb = find(int(a)), find(int(b))
        if ra != rb:
            parent[max(ra, rb)] = min(ra, rb)
    roots = [find(int(a)) for a in e[:, 0]]
    order = {r: k for k, r in enumerate(sorted(set(roots)))}
    return np.array([order[r] for r in roots], dtype=np.int64)


def loop_lengths(gamma, edges):
    """Length of every component (the loop-length targets of gamma)."""
    ell, _, _ = edge_geometry(gamma, edges)
    comp = components(edges, len(gamma))
    return np.bincount(comp, weights=ell)


def evaluate(gamma, edges, mask, x0=None, L0=None, l0=None, jacobian=True, Lq=None, points=None, surface=None,
             tangent=None):
    """(Phi, C) for the constraint set ``mask`` (bitwise OR of the flags);
    ``Lq`` are the loop-length targets, ``points`` = (vertices, targets [m][3])
    the pinned vertices, ``surface`` = (kind, params, vertices) the vertices
    held on an implicit surface, ``tangent`` = (edges, directions [m][3]) the
    edges whose tangent is prescribed."""
    g = np.asarray(gamma, dtype=np.float64)
    e = np.asarray(edges)
    nV, nE = len(g), len(e)
    ell, T, x = edge_geometry(g, e)
    phis, jacs = [], []
    if mask & BARYCENTER:
        phis.append((ell[:, None] * (x - x0)).sum(0))
        if jacobian:
            Cb = np.zeros((3, 3 * nV))
            for I in range(nE):
                for a, sgn in ((0, -1.0), (1, 1.0)):
                    v = e[I, a]
                    Cb[:, 3 * v:3 * v + 3] += 0.5 * ell[I] * np.eye(3) + sgn * np.outer(x[I] - x0, T[I])
            jacs.append(Cb)
    if mask & TOTAL_LENGTH:
        phis.append(np.array([L0 - ell.sum()]))
        if jacobian:
            Cl = np.zeros((1, 3 * nV))
            for I in range(nE):
                Cl[0, 3 * e[I, 0]:3 * e[I, 0] + 3] += T[I]
                Cl[0, 3 * e[I, 1]:3 * e[I, 1] + 3] -= T[I]
            jacs.append(Cl)
    if points is not None and len(points[0]):
        pv = np.asarray(points[0], dtype=np.int64)
        px = np.asarray(points[1], dtype=np.float64).reshape(len(pv), 3)
        phis.append((g[pv] - px).ravel())
        if jacobian:
            Cp = np.zeros((3 * len(pv), 3 * nV))
            for j, v in enumerate(pv):
                Cp[3 * j:3 * j + 3, 3 * v:3 * v + 3] = np.eye(3)
            jacs.append(Cp)
    if surface is not None and len(surface[2]):
        sv = np.asarray(surface[2], dtype=np.int64)
        f, grad = surface_value(surface[0], surface[1], g[sv])
        phis.append(f)
        if jacobian:
            Cs = np.zeros((len(sv), 3 * nV))
            for j, v in enumerate(sv):
                Cs[j, 3 * v:3 * v + 3] = grad[j]
            jacs.append(Cs)
    if tangent is not None and len(tangent[0]):
        te = np.asarray(tangent[0], dtype=np.int64)
        X = np.asarray(tangent[1], dtype=np.float64).reshape(len(te), 3)
        Ct = np.zeros((2 * len(te), 3 * nV))
        ph = []
        for j, I in enumerate(te):
            for k, b in enumerate(tangent_basis(X[j])):
                ph.append(b @ T[I])
                r = (b - (b @ T[I]) * T[I]) / ell[I]
                Ct[2 * j + k, 3 * e[I, 1]:3 * e[I, 1] + 3] += r
                Ct[2 * j + k, 3 * e[I, 0]:3 * e[I, 0] + 3] -= r
        phis.append(np.array(ph))
        if jacobian:
            jacs.append(Ct)
    if mask & EDGE_LENGTH:
        phis.append(l0 - ell)
        if jacobian:
            Ce = np.zeros((nE, 3 * nV))
            for I in range(nE):
                Ce[I, 3 * e[I, 0]:3 * e[I, 0] + 3] = T[I]
                Ce[I, 3 * e[I, 1]:3 * e[I, 1] + 3] = -T[I]
            jacs.append(Ce)
    if mask & LOOP_LENGTH:
        comp = components(e, nV)
        nq = int(comp.max()) + 1
        phis.append(np.asarray(Lq, dtype=np.float64) - np.bincount(comp, weights=ell, minlength=nq))
        if jacobian:
            Cq = np.zeros((nq, 3 * nV))
            for I in range(nE):
                Cq[comp[I], 3 * e[I, 0]:3 * e[I, 0] + 3] += T[I]
                Cq[comp[I], 3 * e[I, 1]:3 * e[I, 1] + 3] -= T[I]
            jacs.append(Cq)
    phi = np.concatenate(phis) if phis else np.zeros(0)
    if not jacobian:
        return phi, None
    C = np.concatenate(jacs) if jacs else np.zeros((0, 3 * nV))
    return phi, C


def jacobian_sparse(gamma, edges, mask, x0=None, points=None):
    """The Jacobian C of ``evaluate`` for BARYCENTER, TOTAL_LENGTH, points and
    EDGE_LENGTH as a scipy.sparse CSR matrix, entry by entry from the same
    formulas (for curves too large for the dense k x 3|V| array)."""
    import scipy.sparse as sp

    g = np.asarray(gamma, dtype=np.float64)
    e = np.asarray(edges)
    nV, nE = len(g), len(e)
    ell, T, x = edge_geometry(g, e)
    rows, cols, vals = [], [], []
    k = 0
    if mask & BARYCENTER:
        # block at vertex v: sum over incident I of (l_I / 2) Id_3 +- (x_I - x0) T_I^T
        for a, sgn in ((0, -1.0), (1, 1.0)):
            v = e[:, a]
            for r in range(3):
                for c in range(3):
                    rows.append(np.full(nE, k + r))
                    cols.append(3 * v + c)
                    vals.append((0.5 * ell if r == c else 0.0) + sgn * (x[:, r] - x0[r]) * T[:, c])
        k += 3
    if mask & TOTAL_LENGTH:
        for a, sgn in ((0, 1.0), (1, -1.0)):
            for c in range(3):
                rows.append(np.full(nE, k))
                cols.append(3 * e[:, a] + c)
                vals.append(sgn * T[:, c])
        k += 1
    if points is not None and len(points[0]):
        pv = np.asarray(points[0], dtype=np.int64)
        m = 3 * len(pv)
        rows.append(k + np.arange(m))
        cols.append((3 * pv[:, None] + np.arange(3)[None, :]).ravel())
        vals.append(np.ones(m))
        k += m
    if mask & EDGE_LENGTH:
        I = np.arange(nE)
        for a, sgn in ((0, 1.0), (1, -1.0)):
            for c in range(3):
                rows.append(k + I)
                cols.append(3 * e[:, a] + c)
                vals.append(sgn * T[:, c])
        k += nE
    if not rows:
        return sp.csr_matrix((0, 3 * nV))
    vals = [np.broadcast_to(v, r.shape) for v, r in zip(vals, rows)]
    return sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(k, 3 * nV)).tocsr()
