"""Pins of the oracle's Sobolev weights w_IJ, w0_IJ and of the barycenter
constraint that do not go through the oracle's own weight code.

* Brute force in 50-digit arithmetic (mpmath): the entries of B and B0 on
  small loops, written as plain loops over the weights exactly as Sec. 4.2.2
  (eq. DiscreteHighOrderPart: ``w_IJ = 1/4 l_I l_J sum_{i in I, j in J}
  |g_i - g_j|^-(2 sigma + 1)``) and Sec. 4.2.3 (``w0_IJ = 1/4 l_I l_J sum
  k_{2,4}(g_i, g_j, T_I) / |g_i - g_j|^(2 sigma + 1)``) define them, and the
  entries taken from the two bilinear forms those sections print
  (``sum w_IJ <D_I u - D_J u, D_I v - D_J v>`` and
  ``sum w0_IJ (u_I - u_J)(v_I - v_J)``) with unit vectors u, v.
* Two quadratures of one integral: the trapezoid weights of Sec. 4.2 and the
  edge-midpoint weights of App. B.3.4 (whose increment form is itself pinned
  to the appendix's kernel-matrix form) sample the same double integral, so on
  refined smooth curves the quadratic forms u^T B u and u^T B0 u of the two
  rules approach each other.  A wrong factor in either weight does not.
* Barycenter constraint (Sec. 7.1): ``Phi(g + t) = Phi(g) + L t`` and
  ``Phi(x0 + R (g - x0)) = R Phi(g)`` for a translation t and a rotation R,
  and the closed form of a regular polygon about a given centre.
* Edge-midpoint energy (the sum Barnes-Hut approximates, App. B.1.2) against
  a 50-digit brute force of its plain double sum.
"""

import mpmath
import numpy as np
import pytest

import gen
from oracle import constraints as cons
from oracle import sobolev as S
from oracle import tpe

PARAMS = [(2.0, 4.0), (2.0, 4.5), (3.0, 6.0)]


def random_loop(n, seed):
    rng = np.random.default_rng(seed)
    t = 2 * np.pi * np.arange(n) / n
    g = np.stack([np.cos(t), np.sin(t), 0.4 * np.sin(3 * t)], 1) + 0.12 * rng.normal(size=(n, 3))
    return g, gen.loop_edges(n)


def _mp_vec(v):
    return [mpmath.mpf(float(c)) for c in v]


def _mp_sub(a, b):
    return [a[k] - b[k] for k in range(3)]


def _mp_dot(a, b):
    return sum(a[k] * b[k] for k in range(3))


def _mp_cross(a, b):
    return [a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]]


def brute_force_gram(g, e, alpha, beta):
    """(B, B0) entries from the printed weights and bilinear forms, 50 digits."""
    mpmath.mp.dps = 50
    P = [_mp_vec(v) for v in g]
    nV, nE = len(g), len(e)
    sigma = (mpmath.mpf(beta) - 1) / mpmath.mpf(alpha) - 1
    expo = 2 * sigma + 1
    ell, T = [], []
    for I in range(nE):
        d = _mp_sub(P[e[I][1]], P[e[I][0]])
        L = mpmath.sqrt(_mp_dot(d, d))
        ell.append(L)
        T.append([c / L for c in d])
    B = [[mpmath.mpf(0)] * nV for _ in range(nV)]
    B0 = [[mpmath.mpf(0)] * nV for _ in range(nV)]
    for I in range(nE):
        for J in range(nE):
            if {int(e[I][0]), int(e[I][1])} & {int(e[J][0]), int(e[J][1])}:
                continue
            w = mpmath.mpf(0)
            w0 = mpmath.mpf(0)
            for i in (e[I][0], e[I][1]):
                for j in (e[J][0], e[J][1]):
                    d = _mp_sub(P[i], P[j])
                    r = mpmath.sqrt(_mp_dot(d, d))
                    c = _mp_cross(T[I], d)
                    w += r ** (-expo)
                    w0 += _mp_dot(c, c) / r ** 4 / r ** expo
            w *= ell[I] * ell[J] / 4
            w0 *= ell[I] * ell[J] / 4
            # D_K e_v = (delta(v, k2) - delta(v, k1)) / l_K T_K ; edge average of e_v
            for u in set([int(e[I][0]), int(e[I][1]), int(e[J][0]), int(e[J][1])]):
                Du = [mpmath.mpf(0)] * 3
                su_I = (int(u == e[I][1]) - int(u == e[I][0])) / ell[I]
                su_J = (int(u == e[J][1]) - int(u == e[J][0])) / ell[J]
                Du = [su_I * T[I][k] - su_J * T[J][k] for k in range(3)]
                au = (int(u == e[I][0]) + int(u == e[I][1]) - int(u == e[J][0]) - int(u == e[J][1])) / mpmath.mpf(2)
                for v in set([int(e[I][0]), int(e[I][1]), int(e[J][0]), int(e[J][1])]):
                    sv_I = (int(v == e[I][1]) - int(v == e[I][0])) / ell[I]
                    sv_J = (int(v == e[J][1]) - int(v == e[J][0])) / ell[J]
                    Dv = [sv_I * T[I][k] - sv_J * T[J][k] for k in range(3)]
                    av = (int(v == e[I][0]) + int(v == e[I][1]) - int(v == e[J][0]) - int(v == e[J][1])) / mpmath.mpf(2)
                    B[u][v] += w * _mp_dot(Du, Dv)
                    B0[u][v] += w0 * au * av
    to = lambda M: np.array([[float(x) for x in row] for row in M])
    return to(B), to(B0)


@pytest.mark.parametrize("n", [5, 8])
@pytest.mark.parametrize("alpha,beta", PARAMS)
def test_gram_entries_brute_force_mpmath(n, alpha, beta):
    g, e = random_loop(n, seed=40 + n)
    Bref, B0ref = brute_force_gram(g, e, alpha, beta)
    B, B0 = S.assemble(g, e, alpha, beta)
    assert np.abs(B - Bref).max() <= 1e-12 * np.abs(Bref).max()
    assert np.abs(B0 - B0ref).max() <= 1e-12 * np.abs(B0ref).max()
    # the independently computed entries keep the structure of the forms
    assert np.abs(Bref.sum(1)).max() <= 1e-13 * np.abs(Bref).max()
    assert np.abs(B0ref.sum(1)).max() <= 1e-13 * np.abs(B0ref).max()


def test_gram_entries_open_path_brute_force_mpmath():
    # an open path: its end vertices belong to one edge only
    g, _ = random_loop(7, seed=3)
    e = np.stack([np.arange(6), np.arange(1, 7)], 1).astype(np.int32)
    Bref, B0ref = brute_force_gram(g, e, 2.0, 4.5)
    B, B0 = S.assemble(g, e, 2.0, 4.5)
    assert np.abs(B - Bref).max() <= 1e-12 * np.abs(Bref).max()
    assert np.abs(B0 - B0ref).max() <= 1e-12 * np.abs(B0ref).max()


def smooth_knot(n):
    """(2,3) torus knot, uniformly sampled in its parameter (no jitter)."""
    t = 2 * np.pi * np.arange(n) / n
    r = 2.0 + np.cos(3 * t)
    g = np.stack([r * np.cos(2 * t), r * np.sin(2 * t), -np.sin(3 * t)], 1)
    return g, gen.loop_edges(n), t


@pytest.mark.parametrize("alpha,beta", PARAMS)
def test_trapezoid_and_midpoint_weights_sample_one_integral(alpha, beta):
    gaps_hi, gaps_lo = [], []
    for n in (96, 192, 384):
        g, e, t = smooth_knot(n)
        u = np.cos(t) + 0.5 * np.sin(2 * t) + 0.3 * np.cos(5 * t)
        Bt, B0t = S.assemble(g, e, alpha, beta, quadrature="trapezoid")
        Bm, B0m = S.assemble(g, e, alpha, beta, quadrature="midpoint")
        gaps_hi.append(abs(u @ Bt @ u / (u @ Bm @ u) - 1.0))
        gaps_lo.append(abs(u @ B0t @ u / (u @ B0m @ u) - 1.0))
    # the two rules converge to each other under refinement ...
    assert gaps_hi[0] > gaps_hi[1] > gaps_hi[2]
    assert gaps_lo[0] > gaps_lo[1] > gaps_lo[2]
    # ... and are already close (the gap shrinks like a power of h set by the
    # kernel's singularity, h^0.5 for (2, 4.5)): a factor slip in a weight
    # (2x, 3x, 1/4) is far outside
    assert gaps_hi[2] < 0.1
    assert gaps_lo[2] < 0.05


def test_barycenter_translation_rotation_and_polygon():
    g, e = random_loop(11, seed=5)
    x0, L0, l0 = cons.reference_values(g, e)
    x0 = x0 + np.array([0.2, -0.1, 0.3])  # a target that is not the curve's own
    phi, _ = cons.evaluate(g, e, cons.BARYCENTER, x0=x0, jacobian=False)
    L = float(np.linalg.norm(np.roll(g, -1, 0) - g, axis=1).sum())
    t = np.array([0.7, -1.3, 2.1])
    phi_t, _ = cons.evaluate(g + t, e, cons.BARYCENTER, x0=x0, jacobian=False)
    assert np.allclose(phi_t, phi + L * t, rtol=0, atol=1e-13 * L * 3)
    q, _ = np.linalg.qr(np.random.default_rng(2).normal(size=(3, 3)))
    Rg = (g - x0) @ q.T + x0
    phi_r, _ = cons.evaluate(Rg, e, cons.BARYCENTER, x0=x0, jacobian=False)
    assert np.allclose(phi_r, q @ phi, rtol=0, atol=1e-13 * L * 3)
    # regular polygon of circumradius R about c: l = 2 R sin(pi/n), midpoints on
    # a circle about c, so Phi(x0) = n l (c - x0)
    n, R = 9, 0.7
    c = np.array([0.3, 0.4, -0.2])
    gp, ep = gen.regular_ngon(n, radius=R)
    gp = gp + c
    lside = 2 * R * np.sin(np.pi / n)
    phi_p, _ = cons.evaluate(gp, ep, cons.BARYCENTER, x0=np.zeros(3), jacobian=False)
    assert np.allclose(phi_p, n * lside * c, rtol=1e-14, atol=1e-14)


def brute_force_midpoint_energy(g, e, alpha, beta):
    mpmath.mp.dps = 50
    P = [_mp_vec(v) for v in g]
    total = mpmath.mpf(0)
    for I in range(len(e)):
        for J in range(len(e)):
            if {int(e[I][0]), int(e[I][1])} & {int(e[J][0]), int(e[J][1])}:
                continue
            dI = _mp_sub(P[e[I][1]], P[e[I][0]])
            dJ = _mp_sub(P[e[J][1]], P[e[J][0]])
            lI, lJ = mpmath.sqrt(_mp_dot(dI, dI)), mpmath.sqrt(_mp_dot(dJ, dJ))
            T = [c / lI for c in dI]
            xI = [(P[e[I][0]][k] + P[e[I][1]][k]) / 2 for k in range(3)]
            xJ = [(P[e[J][0]][k] + P[e[J][1]][k]) / 2 for k in range(3)]
            d = _mp_sub(xI, xJ)
            c = _mp_cross(T, d)
            total += mpmath.sqrt(_mp_dot(c, c)) ** alpha / mpmath.sqrt(_mp_dot(d, d)) ** beta * lI * lJ
    return float(total)


@pytest.mark.parametrize("alpha,beta", PARAMS)
def test_midpoint_energy_brute_force_mpmath(alpha, beta):
    g, e = random_loop(9, seed=17)
    ref = brute_force_midpoint_energy(g, e, alpha, beta)
    assert tpe.midpoint_energy(g, e, alpha, beta) == pytest.approx(ref, rel=1e-13)


def test_gram_entries_junction_graph_brute_force_mpmath():
    # a theta graph: two vertices of degree three joined by three arcs (Sec. 7.3 networks)
    g, e = gen.theta_graph(3, seed=5, jitter=0.1)
    assert np.bincount(e.ravel()).max() == 3
    Bref, B0ref = brute_force_gram(g, e, 2.0, 4.5)
    B, B0 = S.assemble(g, e, 2.0, 4.5)
    assert np.abs(B - Bref).max() <= 1e-12 * np.abs(Bref).max()
    assert np.abs(B0 - B0ref).max() <= 1e-12 * np.abs(B0ref).max()
    assert np.abs(Bref.sum(1)).max() <= 1e-13 * np.abs(Bref).max()
