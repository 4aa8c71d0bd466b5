"""Seeded curve generators shaped like the workloads of the repulsive-curves paper.

Every generator returns ``(gamma, edges)``:

* ``gamma``: float64 array ``[n_vertices, 3]`` of vertex coordinates;
* ``edges``: int32 array ``[n_edges, 2]`` of oriented edges ``(i1, i2)``.

Random numbers come from ``numpy.random.default_rng(seed)`` (PCG64).  A normal
distribution written ``N(0, v)`` in a workload description takes ``v`` as the
variance.
"""

from __future__ import annotations

import numpy as np

__all__ = [
    "loop_edges",
    "trefoil",
    "fourier_knot",
    "regular_ngon",
    "packing_instance",
    "packing_batch",
    "round_to_f32",
    "theta_graph",
    "tennis_ball",
    "torus_knot",
    "icosphere",
    "torus_mesh",
    "star_graph",
]


def loop_edges(n: int, offset: int = 0) -> np.ndarray:
    """Edges of one closed loop over vertices ``offset .. offset+n-1``."""
    i = np.arange(n, dtype=np.int64)
    return np.stack([i + offset, (i + 1) % n + offset], axis=1).astype(np.int32)


def round_to_f32(gamma: np.ndarray) -> np.ndarray:
    """Round coordinates to the nearest float32 and return them as float64."""
    return np.asarray(gamma, dtype=np.float32).astype(np.float64)


def trefoil(n: int = 256, seed: int = 0, jitter_var: float = 1e-3):
    """Closed trefoil x = sin t + 2 sin 2t, y = cos t - 2 cos 2t, z = -sin 3t.

    ``n`` uniform samples ``t_i = 2 pi i / n`` plus i.i.d. Gaussian jitter of
    variance ``jitter_var`` on every coordinate.
    """
    t = 2.0 * np.pi * np.arange(n) / n
    g = np.stack([np.sin(t) + 2 * np.sin(2 * t),
                  np.cos(t) - 2 * np.cos(2 * t),
                  -np.sin(3 * t)], axis=1)
    rng = np.random.default_rng(seed)
    g = g + rng.normal(0.0, np.sqrt(jitter_var), size=g.shape)
    return g, loop_edges(n)


def regular_ngon(n: int, radius: float = 1.0, phase: float = 0.0):
    """Regular n-gon inscribed in a circle of the given radius in the xy-plane."""
    t = phase + 2.0 * np.pi * np.arange(n) / n
    g = np.stack([radius * np.cos(t), radius * np.sin(t), np.zeros(n)], axis=1)
    return g, loop_edges(n)


def _min_far_distance(g: np.ndarray, min_sep: int) -> float:
    """Smallest distance between vertices at least ``min_sep`` apart along the loop."""
    from scipy.spatial import cKDTree

    n = len(g)
    seg = np.linalg.norm(np.roll(g, -1, axis=0) - g, axis=1)
    tree = cKDTree(g)
    r = 40.0 * seg.mean()
    pairs = tree.query_pairs(r, output_type="ndarray")
    if len(pairs) == 0:
        return np.inf
    di = np.abs(pairs[:, 0] - pairs[:, 1])
    di = np.minimum(di, n - di)
    far = pairs[di >= min_sep]
    if len(far) == 0:
        return np.inf
    return float(np.min(np.linalg.norm(g[far[:, 0]] - g[far[:, 1]], axis=1)))


def fourier_knot(n: int, seed: int = 0, modes: int = 8, max_tries: int = 200,
                 clearance: float = 20.0):
    """Random smooth closed curve from Fourier modes ``k = 1..modes``.

    Per axis ``sum_k a_k cos(k t) + b_k sin(k t)`` with ``a_k, b_k ~ N(0, 1/k^2)``
    (standard deviation ``1/k``), sampled at ``t_i = 2 pi i / n``.  A draw is
    rejected, and the generator draws again from the same stream, when two
    vertices at least ``n/64`` apart along the loop come closer than
    ``clearance`` mean edge lengths, a distance capped at 1/400 of the curve
    length so that coarse curves stay admissible.  Returns
    ``(gamma, edges, tries)``.
    """
    rng = np.random.default_rng(seed)
    t = 2.0 * np.pi * np.arange(n) / n
    k = np.arange(1, modes + 1)
    ck, sk = np.cos(np.outer(t, k)), np.sin(np.outer(t, k))
    for attempt in range(1, max_tries + 1):
        a = rng.normal(0.0, 1.0, size=(modes, 3)) / k[:, None]
        b = rng.normal(0.0, 1.0, size=(modes, 3)) / k[:, None]
        g = ck @ a + sk @ b
        seg = np.linalg.norm(np.roll(g, -1, axis=0) - g, axis=1)
        if _min_far_distance(g, max(3, n // 64)) >= min(clearance * seg.mean(), seg.sum() / 400.0):
            return g, loop_edges(n), attempt
    raise RuntimeError(f"fourier_knot: no admissible draw in {max_tries} tries")


def _circle(center, radius, normal, n):
    normal = normal / np.linalg.norm(normal)
    helper = np.array([1.0, 0.0, 0.0]) if abs(normal[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
    u = np.cross(normal, helper)
    u /= np.linalg.norm(u)
    v = np.cross(normal, u)
    t = 2.0 * np.pi * np.arange(n) / n
    return center + radius * (np.outer(np.cos(t), u) + np.outer(np.sin(t), v))


def packing_instance(rng: np.random.Generator, obstacle_center=(0.5, 0.5, 0.5),
                     obstacle_radius=0.25, e_min=200, e_max=8000):
    """One packing instance: 8..32 circles around a sphere obstacle.

    The total edge count is log-uniform in ``[e_min, e_max]``; the loop count
    is uniform on 8..32, capped so that every loop has at least 8 edges, and
    edges are split in proportion to the radii.  Radii are ``U[0.05, 0.2]``,
    centres ``U[0,1]^3`` and normals uniform on the sphere; a circle is redrawn
    while its bounding sphere meets an earlier one or the obstacle (after many
    failures its radius shrinks).  Returns ``(gamma, edges, loop_sizes)``.
    """
    c0 = np.asarray(obstacle_center, dtype=np.float64)
    e_tot = int(round(np.exp(rng.uniform(np.log(e_min), np.log(e_max)))))
    n_loops = int(rng.integers(8, 33))
    n_loops = max(1, min(n_loops, e_tot // 8))
    placed = []
    for _ in range(n_loops):
        r = rng.uniform(0.05, 0.2)
        for attempt in range(2000):
            if attempt and attempt % 200 == 0:
                r *= 0.8
            c = rng.uniform(0.0, 1.0, size=3)
            if np.linalg.norm(c - c0) <= obstacle_radius + r:
                continue
            if all(np.linalg.norm(c - pc) > r + pr for pc, pr, _ in placed):
                break
        nrm = rng.normal(size=3)
        placed.append((c, r, nrm))
    radii = np.array([p[1] for p in placed])
    sizes = np.maximum(8, np.floor(e_tot * radii / radii.sum()).astype(int))
    gammas, edges, off = [], [], 0
    for (c, r, nrm), m in zip(placed, sizes):
        gammas.append(_circle(c, r, nrm, int(m)))
        edges.append(loop_edges(int(m), off))
        off += int(m)
    return np.concatenate(gammas), np.concatenate(edges).astype(np.int32), sizes


def packing_batch(n_instances: int = 512, seed: int = 0, **kw):
    """``n_instances`` independent packing instances from one seeded stream."""
    rng = np.random.default_rng(seed)
    return [packing_instance(rng, **kw) for _ in range(n_instances)]


def theta_graph(n_arc: int = 32, n_arcs: int = 3, seed: int = 0, jitter: float = 0.1):
    """A curve network with two junctions (Sec. 7.3): ``n_arcs`` arcs of ``n_arc`` edges each join
    vertex 0 at (-1, 0, 0) to vertex 1 at (1, 0, 0).

    Arc k runs through ``(-cos(pi t), r sin(pi t) cos(phi_k), r sin(pi t) sin(phi_k))``,
    ``t`` in [0, 1], with ``phi_k = 2 pi k / n_arcs`` and ``r = 0.8``, its interior
    vertices numbered consecutively after the two junctions; i.i.d. Gaussian jitter of
    standard deviation ``jitter`` times the arc's mean edge length moves the interior
    vertices.  Edges are oriented along t.
    """
    rng = np.random.default_rng(seed)
    pts = [np.array([-1.0, 0.0, 0.0]), np.array([1.0, 0.0, 0.0])]
    edges = []
    for k in range(n_arcs):
        phi = 2.0 * np.pi * k / n_arcs
        t = np.arange(0, n_arc + 1) / n_arc
        arc = np.stack([-np.cos(np.pi * t), 0.8 * np.sin(np.pi * t) * np.cos(phi),
                        0.8 * np.sin(np.pi * t) * np.sin(phi)], axis=1)
        h = np.linalg.norm(np.diff(arc, axis=0), axis=1).mean()
        arc = arc[1:-1] + rng.normal(0.0, jitter * h, size=(n_arc - 1, 3))
        first = len(pts)
        pts.extend(arc)
        ids = [0] + list(range(first, first + n_arc - 1)) + [1]
        edges.extend([ids[q], ids[q + 1]] for q in range(n_arc))
    return np.array(pts), np.array(edges, dtype=np.int32)


def tennis_ball(n: int = 256, a: float = 0.6, seed: int = 0, jitter_var: float = 0.0):
    """Closed curve on the unit sphere: ``(a cos t + b cos 3t, a sin t - b sin 3t,
    2 sqrt(a b) sin 2t)`` with ``b = 1 - a`` (its squared norm is (a + b)^2 = 1),
    ``n`` uniform samples of t plus i.i.d. Gaussian jitter of variance ``jitter_var``."""
    b = 1.0 - a
    t = 2.0 * np.pi * np.arange(n) / n
    g = np.stack([a * np.cos(t) + b * np.cos(3 * t), a * np.sin(t) - b * np.sin(3 * t),
                  2.0 * np.sqrt(a * b) * np.sin(2 * t)], axis=1)
    if jitter_var > 0:
        g = g + np.random.default_rng(seed).normal(0.0, np.sqrt(jitter_var), size=g.shape)
    return g, loop_edges(n)


def torus_knot(n: int = 256, p: int = 2, q: int = 3, R: float = 1.0, r: float = 0.4, seed: int = 0,
               jitter_var: float = 0.0):
    """(p, q) torus knot on the torus of radii (R, r) about the z axis:
    ``((R + r cos(q t)) cos(p t), (R + r cos(q t)) sin(p t), r sin(q t))``, ``n``
    uniform samples of t in [0, 2 pi) plus i.i.d. Gaussian jitter of variance ``jitter_var``."""
    t = 2.0 * np.pi * np.arange(n) / n
    g = np.stack([(R + r * np.cos(q * t)) * np.cos(p * t), (R + r * np.cos(q * t)) * np.sin(p * t),
                  r * np.sin(q * t)], axis=1)
    if jitter_var > 0:
        g = g + np.random.default_rng(seed).normal(0.0, np.sqrt(jitter_var), size=g.shape)
    return g, loop_edges(n)


def icosphere(level: int = 2, radius: float = 1.0, center=(0.0, 0.0, 0.0)):
    """Triangulated sphere: the octahedron's 8 faces split ``level`` times into 4
    (edge midpoints pushed out to the sphere).  Returns ``(P, F)``: vertices
    float64 [nP, 3] and triangles int32 [8 * 4^level, 3], outward oriented."""
    P = [np.array(v, dtype=np.float64) for v in
         ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1))]
    F = [(0, 2, 4), (2, 1, 4), (1, 3, 4), (3, 0, 4), (2, 0, 5), (1, 2, 5), (3, 1, 5), (0, 3, 5)]
    for _ in range(level):
        mid = {}

        def m(a, b):
            key = (min(a, b), max(a, b))
            if key not in mid:
                v = P[a] + P[b]
                P.append(v / np.linalg.norm(v))
                mid[key] = len(P) - 1
            return mid[key]

        F = [t for a, b, c in F for t in ((a, m(a, b), m(c, a)), (b, m(b, c), m(a, b)), (c, m(c, a), m(b, c)),
                                           (m(a, b), m(b, c), m(c, a)))]
    return radius * np.array(P) + np.asarray(center, dtype=np.float64), np.array(F, dtype=np.int32)


def torus_mesh(nu: int = 32, nv: int = 16, R: float = 1.0, r: float = 0.3, center=(0.0, 0.0, 0.0)):
    """Triangulated torus about the z axis: an ``nu`` x ``nv`` grid in the angles
    (u around the axis, v around the tube), two triangles per cell.  Returns ``(P, F)``."""
    u = 2.0 * np.pi * np.arange(nu) / nu
    v = 2.0 * np.pi * np.arange(nv) / nv
    U, V = np.meshgrid(u, v, indexing="ij")
    P = np.stack([(R + r * np.cos(V)) * np.cos(U), (R + r * np.cos(V)) * np.sin(U), r * np.sin(V)], axis=-1)
    P = P.reshape(-1, 3) + np.asarray(center, dtype=np.float64)
    idx = lambda i, j: (i % nu) * nv + (j % nv)
    F = []
    for i in range(nu):
        for j in range(nv):
            F.append((idx(i, j), idx(i + 1, j), idx(i + 1, j + 1)))
            F.append((idx(i, j), idx(i + 1, j + 1), idx(i, j + 1)))
    return P, np.array(F, dtype=np.int32)


def star_graph(n_arm: int = 64, n_arms: int = 3, seed: int = 0, jitter: float = 0.1):
    """A network with one junction: ``n_arms`` open arms of ``n_arm`` edges from vertex 0 at
    the origin; arm k runs along ``(t cos phi_k, t sin phi_k, 0.3 sin(pi t))``, t in (0, 1]
    (phi_k = 2 pi k / n_arms), plus i.i.d. Gaussian jitter of standard deviation ``jitter``
    times the arm's mean edge length on the arm vertices.  Edges are oriented outwards."""
    rng = np.random.default_rng(seed)
    pts = [np.zeros(3)]
    edges = []
    for k in range(n_arms):
        phi = 2.0 * np.pi * k / n_arms
        t = np.arange(0, n_arm + 1) / n_arm
        arm = np.stack([t * np.cos(phi), t * np.sin(phi), 0.3 * np.sin(np.pi * t)], axis=1)
        h = np.linalg.norm(np.diff(arm, axis=0), axis=1).mean()
        arm = arm[1:] + rng.normal(0.0, jitter * h, size=(n_arm, 3))
        first = len(pts)
        pts.extend(arm)
        ids = [0] + list(range(first, first + n_arm))
        edges.extend([ids[q], ids[q + 1]] for q in range(n_arm))
    return np.array(pts), np.array(edges, dtype=np.int32)
