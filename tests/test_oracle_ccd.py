"""Pins of the oracle's first collision time (Sec. 4.4, time stepping with the
first collision time tau_max).

* Closed forms: two segments approaching head on meet at distance / speed; a
  pass whose endpoints become coplanar beside the other segment is no
  contact; segments moving inside one plane meet when an endpoint reaches
  the other segment.
* Brute force on small random loops, by a route that shares nothing with the
  oracle's cubic: the determinant det[p2 - p1, q1 - p1, q2 - p1] evaluated
  directly (numpy.linalg.det) on a fine time grid, sign changes refined by
  Brent's method, and the contact decided by solving p1 + s a = q1 + u b in
  least squares (residual zero, s and u in [0, 1]).
* Invariances: rigid motion of curve and direction together; scaling the
  direction by c scales the time by 1/c.
"""

import numpy as np
import pytest
from scipy.optimize import brentq

import gen
from oracle import ccd


def test_head_on_and_miss_closed_forms():
    p1, p2 = np.array([0.0, 0, 0]), np.array([1.0, 0, 0])
    z = np.zeros(3)
    h, w = 0.7, 0.25
    q1, q2 = np.array([0.5, -1.0, h]), np.array([0.5, 1.0, h])
    v = np.array([0.0, 0.0, w])  # gamma - t v: the segment descends at speed w
    t = ccd.pair_contact_time(p1, p2, q1, q2, z, z, v, v, T=10.0)
    assert t == pytest.approx(h / w, rel=1e-12)
    # the same motion beside the first segment: coplanar at h / w, no contact
    q1m, q2m = q1 + [1.5, 0, 0], q2 + [1.5, 0, 0]
    assert ccd.pair_contact_time(p1, p2, q1m, q2m, z, z, v, v, T=10.0) is None
    # beyond the horizon: none
    assert ccd.pair_contact_time(p1, p2, q1, q2, z, z, v, v, T=0.99 * h / w) is None
    # both moving: the relative speed counts
    t2 = ccd.pair_contact_time(p1, p2, q1, q2, -v, -v, v, v, T=10.0)
    assert t2 == pytest.approx(h / (2 * w), rel=1e-12)


def test_planar_motion_endpoint_reaches_segment():
    p1, p2 = np.array([0.0, 0, 0]), np.array([1.0, 0, 0])
    z = np.zeros(3)
    q1, q2 = np.array([0.5, 1.0, 0.0]), np.array([0.3, 2.0, 0.0])
    v = np.array([0.0, 0.5, 0.0])  # moves towards y = 0 at speed 0.5
    assert ccd.pair_contact_time(p1, p2, q1, q2, z, z, v, v, T=10.0) == pytest.approx(2.0, rel=1e-12)
    # sliding past the end of the first segment: no contact
    q1s, q2s = q1 + [1.0, 0, 0], q2 + [1.0, 0, 0]
    assert ccd.pair_contact_time(p1, p2, q1s, q2s, z, z, v, v, T=10.0) is None


def brute_contact(p1, p2, q1, q2, vp1, vp2, vq1, vq2, T, grid=4000):
    at = lambda x, v, t: x - t * v

    def det(t):
        P1, P2, Q1, Q2 = at(p1, vp1, t), at(p2, vp2, t), at(q1, vq1, t), at(q2, vq2, t)
        return np.linalg.det(np.stack([P2 - P1, Q1 - P1, Q2 - P1]))

    def touch(t):
        P1, P2, Q1, Q2 = at(p1, vp1, t), at(p2, vp2, t), at(q1, vq1, t), at(q2, vq2, t)
        M = np.stack([P2 - P1, -(Q2 - Q1)], 1)
        su, *_ = np.linalg.lstsq(M, Q1 - P1, rcond=None)
        res = np.linalg.norm(M @ su - (Q1 - P1))
        scale = np.linalg.norm(P2 - P1) + np.linalg.norm(Q2 - Q1) + np.linalg.norm(Q1 - P1)
        return res <= 1e-8 * scale and -1e-9 <= su[0] <= 1 + 1e-9 and -1e-9 <= su[1] <= 1 + 1e-9

    ts = np.linspace(0.0, T, grid + 1)
    vals = np.array([det(t) for t in ts])
    for k in range(grid):
        if vals[k] == 0.0 and k > 0:
            if touch(ts[k]):
                return ts[k]
        elif vals[k] * vals[k + 1] < 0:
            t = brentq(det, ts[k], ts[k + 1], xtol=1e-15, rtol=1e-15)
            if touch(t):
                return t
    return None


def brute_first(g, e, D, T):
    best = None
    for I in range(len(e)):
        for J in range(I + 1, len(e)):
            if {int(e[I, 0]), int(e[I, 1])} & {int(e[J, 0]), int(e[J, 1])}:
                continue
            i1, i2, j1, j2 = e[I, 0], e[I, 1], e[J, 0], e[J, 1]
            t = brute_contact(g[i1], g[i2], g[j1], g[j2], D[i1], D[i2], D[j1], D[j2], T)
            if t is not None and (best is None or t < best):
                best = t
    return best


def random_case(seed, n=7):
    """A jittered loop moving towards its centroid (collapsing by t = 1) plus a random
    velocity per vertex, so that edges cross before the loop collapses."""
    rng = np.random.default_rng(100 + seed)
    t = 2 * np.pi * np.arange(n) / n
    g = np.stack([np.cos(t), np.sin(t), 0.3 * np.sin(2 * t)], 1) + 0.2 * rng.normal(size=(n, 3))
    D = (g - g.mean(0)) + 0.5 * rng.normal(size=(n, 3))
    return g, gen.loop_edges(n), D


@pytest.mark.parametrize("seed", range(8))
def test_random_loops_against_brute_force(seed):
    g, e, D = random_case(seed)
    T = 1.5
    ref = brute_first(g, e, D, T)
    got = ccd.first_collision_time(g, e, D, T)
    if ref is None:
        assert got is None
    else:
        assert got == pytest.approx(ref, rel=1e-9)


def test_some_random_cases_collide():
    # the brute-force comparison above is not vacuous: most of its cases collide
    hits = sum(ccd.first_collision_time(*random_case(seed), 1.5) is not None for seed in range(8))
    assert hits >= 5


def test_rigid_motion_and_speed_scaling():
    rng = np.random.default_rng(7)
    g, e = gen.trefoil(24, seed=2)
    D = rng.normal(size=g.shape)
    t0 = ccd.first_collision_time(g, e, D, 3.0)
    assert t0 is not None
    q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    assert ccd.first_collision_time(g @ q.T + 1.0, e, D @ q.T, 3.0) == pytest.approx(t0, rel=1e-10)
    assert ccd.first_collision_time(g, e, 2.5 * D, 3.0) == pytest.approx(t0 / 2.5, rel=1e-10)


def test_pruning_by_swept_boxes_keeps_the_result():
    for seed in range(4):
        g, e, D = random_case(seed, n=12)
        assert ccd.first_collision_time(g, e, D, 1.5, prune=True) == ccd.first_collision_time(g, e, D, 1.5)
