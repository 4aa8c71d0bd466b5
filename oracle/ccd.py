"""First collision time of a moving curve, in float64 (oracle).

Test infrastructure only (see the package docstring).

Sec. 4.4 (Time Stepping): the line search may start from the first time
tau_max at which the curve, moved along the step direction, collides with
itself, which keeps it in its isotopy class; the search then starts at
(2/3) tau_max.  Here the curve moves as ``gamma(t) = gamma - t D`` (D the
normalised step direction, every vertex on a straight line), and a collision
is a contact between two edges that share no vertex (the pairs the energy
sums; edges sharing a vertex always touch there).

For two segments whose endpoints move linearly the first contact is found
exactly:

* the four endpoints must be coplanar, so t is a root of the cubic
  ``f(t) = det[p2 - p1, q1 - p1, q2 - p1](t)``; at each root in (0, T], in
  increasing order, the segments touch iff their distance is zero (to a
  relative tolerance), and the first such root is the contact time;
* if f vanishes identically (both segments move inside one fixed plane) the
  first contact is an endpoint of one segment reaching the other segment:
  the roots of ``n . ((a - p) x (b - p))(t)`` (a quadratic, n the plane's
  normal) for each endpoint p and opposite segment ab, checked for p lying
  within ab.

``first_collision_time`` is the minimum over all pairs of disjoint edges,
or None when no pair touches in (0, T].
"""

from __future__ import annotations

import numpy as np
from numpy.polynomial import polynomial as P

__all__ = ["segment_distance", "pair_contact_time", "first_collision_time"]

CONTACT_RTOL = 1e-9   # contact: segment distance <= CONTACT_RTOL * (pair scale)
PLANAR_RTOL = 1e-12   # f is identically zero when every coefficient term is below this relative size


def segment_distance(p1, p2, q1, q2):
    """Distance between the segments p1p2 and q1q2 (closest points, clamped)."""
    d1, d2, r = p2 - p1, q2 - q1, p1 - q1
    a, e, f = d1 @ d1, d2 @ d2, d2 @ r
    c, b = d1 @ r, d1 @ d2
    den = a * e - b * b
    s = np.clip((b * f - c * e) / den, 0.0, 1.0) if den > 1e-300 else 0.0
    u = (b * s + f) / e
    if u < 0.0:
        u, s = 0.0, np.clip(-c / a, 0.0, 1.0)
    elif u > 1.0:
        u, s = 1.0, np.clip((b - c) / a, 0.0, 1.0)
    return float(np.linalg.norm(p1 + s * d1 - (q1 + u * d2)))


def _lin(x0, v):
    """Coordinate polynomials (ascending coefficients) of x0 - t v."""
    return [np.array([x0[k], -v[k]]) for k in range(3)]


def _cross(A, B):
    return [P.polysub(P.polymul(A[1], B[2]), P.polymul(A[2], B[1])),
            P.polysub(P.polymul(A[2], B[0]), P.polymul(A[0], B[2])),
            P.polysub(P.polymul(A[0], B[1]), P.polymul(A[1], B[0]))]


def _dot(A, B):
    return P.polyadd(P.polyadd(P.polymul(A[0], B[0]), P.polymul(A[1], B[1])), P.polymul(A[2], B[2]))


def _sub(A, B):
    return [P.polysub(A[k], B[k]) for k in range(3)]


def _real_roots(c, T):
    c = np.trim_zeros(np.asarray(c, dtype=np.float64), "b")
    if len(c) <= 1:
        return []
    r = P.polyroots(c)
    r = np.real(r[np.abs(np.imag(r)) <= 1e-9 * (1.0 + np.abs(r))])
    return sorted(float(t) for t in r if 0.0 < t <= T)


def pair_contact_time(p1, p2, q1, q2, vp1, vp2, vq1, vq2, T):
    """First t in (0, T] at which the segments (p1 - t vp1)(p2 - t vp2) and
    (q1 - t vq1)(q2 - t vq2) touch, or None."""
    at = lambda x, v, t: x - t * v
    Pp1, Pp2, Pq1, Pq2 = _lin(p1, vp1), _lin(p2, vp2), _lin(q1, vq1), _lin(q2, vq2)
    a, b, c = _sub(Pp2, Pp1), _sub(Pq1, Pp1), _sub(Pq2, Pp1)
    f = _dot(a, _cross(b, c))
    speed = max(np.linalg.norm(v) for v in (vp1, vp2, vq1, vq2))
    scale = max(np.linalg.norm(p2 - p1), np.linalg.norm(q2 - q1), np.linalg.norm(q1 - p1)) + T * speed
    tol = CONTACT_RTOL * scale

    def touching(t):
        return segment_distance(at(p1, vp1, t), at(p2, vp2, t), at(q1, vq1, t), at(q2, vq2, t)) <= tol

    f = np.pad(f, (0, 4 - len(f)))
    if all(abs(f[k]) * T ** k <= PLANAR_RTOL * scale ** 3 for k in range(4)):
        # planar motion: an endpoint reaches the other segment
        n = np.cross(p2 - p1, q1 - p1)
        if np.linalg.norm(n) == 0.0:
            n = np.cross(p2 - p1, q2 - p1)
        n = n / np.linalg.norm(n)
        best = None
        for (x, vx), (y1, vy1), (y2, vy2) in (((p1, vp1), (q1, vq1), (q2, vq2)), ((p2, vp2), (q1, vq1), (q2, vq2)),
                                              ((q1, vq1), (p1, vp1), (p2, vp2)), ((q2, vq2), (p1, vp1), (p2, vp2))):
            X, Y1, Y2 = _lin(x, vx), _lin(y1, vy1), _lin(y2, vy2)
            g = _dot([np.array([n[k]]) for k in range(3)], _cross(_sub(Y1, X), _sub(Y2, X)))
            for t in _real_roots(g, T):
                if touching(t):
                    best = t if best is None else min(best, t)
                    break
        return best
    for t in _real_roots(f, T):
        if touching(t):
            return t
    return None


def _swept_boxes_overlap(g, v, e, T):
    """Pairs (I, J), I < J, whose boxes swept over [0, T] overlap.  A point of a
    segment at time t is a convex combination of its endpoints, each moving on a
    line, so it lies in the box of the four positions at 0 and T: pairs outside
    this list cannot touch."""
    ends = np.stack([g[e[:, 0]], g[e[:, 1]], g[e[:, 0]] - T * v[e[:, 0]], g[e[:, 1]] - T * v[e[:, 1]]], 1)
    lo, hi = ends.min(1), ends.max(1)
    pairs = []
    for I in range(len(e)):
        ok = np.all((lo[I] <= hi[I + 1:]) & (lo[I + 1:] <= hi[I]), axis=1)
        pairs.extend((I, I + 1 + int(j)) for j in np.nonzero(ok)[0])
    return pairs


def first_collision_time(gamma, edges, D, T, prune=False):
    """Minimum over pairs of edges sharing no vertex of their contact time
    in (0, T] when the curve moves as gamma - t D; None if there is none.
    prune=True visits only the pairs whose swept boxes overlap (the others
    cannot touch), for curves of a few thousand edges."""
    g = np.asarray(gamma, dtype=np.float64)
    v = np.asarray(D, dtype=np.float64)
    e = np.asarray(edges)
    best = None
    pairs = _swept_boxes_overlap(g, v, e, T) if prune else ((I, J) for I in range(len(e)) for J in range(I + 1, len(e)))
    for I, J in pairs:
        if {int(e[I, 0]), int(e[I, 1])} & {int(e[J, 0]), int(e[J, 1])}:
            continue
        i1, i2, j1, j2 = e[I, 0], e[I, 1], e[J, 0], e[J, 1]
        t = pair_contact_time(g[i1], g[i2], g[j1], g[j2], v[i1], v[i2], v[j1], v[j2], T)
        if t is not None and (best is None or t < best):
            best = t
    return best
