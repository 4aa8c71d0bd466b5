"""Pins of the oracle's Gram matrices B, B0 (Sec. 4.2) against independent facts.

* Polarization: the printed quadratic forms (eq. DiscreteHighOrderPart and the
  low-order form of Sec. 4.2.3) reproduce, entry by entry, the matrices built
  from the printed increment tables: a typo in either would break this.
* Two passages agree: with midpoint weights, the increment construction equals
  the kernel-matrix form of App. B.3.4 (eqs. LowOrderDecomposition /
  LowOrderKernel and the high-order analogue).
* Structure: A 1 = 0, symmetric, positive semidefinite, invariant under rigid
  motion, and scales as lambda^-(2 sigma + 1) (the exponent implied by
  Sec. 3.2 and App. A.3; App. A.3.2 prints it as 2s+1, read as 2 sigma + 1).
* Regular n-gon: A is circulant and its FFT eigenvalues equal eigvalsh(A).
"""

import numpy as np
import pytest

import gen
from oracle import sobolev as S

PARAMS = [(2.0, 4.0), (2.0, 4.5), (3.0, 6.0)]


@pytest.mark.parametrize("alpha,beta", PARAMS)
def test_polarization_reproduces_increment_tables(alpha, beta):
    g, e = gen.trefoil(16, seed=11)
    n = len(g)
    B, B0 = S.assemble(g, e, alpha, beta)
    eye = np.eye(n)
    Qh = lambda u: S.quad_high(g, e, alpha, beta, u)
    Ql = lambda u: S.quad_low(g, e, alpha, beta, u)
    rng = np.random.default_rng(0)
    pairs = [(i, i) for i in range(0, n, 5)] + [tuple(rng.integers(0, n, 2)) for _ in range(12)]
    for i, j in pairs:
        bij = 0.5 * (Qh(eye[i] + eye[j]) - Qh(eye[i]) - Qh(eye[j])) if i != j else Qh(eye[i])
        b0ij = 0.5 * (Ql(eye[i] + eye[j]) - Ql(eye[i]) - Ql(eye[j])) if i != j else Ql(eye[i])
        assert B[i, j] == pytest.approx(bij, rel=1e-11, abs=1e-12 * np.abs(B).max())
        assert B0[i, j] == pytest.approx(b0ij, rel=1e-11, abs=1e-12 * np.abs(B0).max())


@pytest.mark.parametrize("alpha,beta", PARAMS)
def test_structure(alpha, beta):
    g, e = gen.trefoil(48, seed=12)
    B, B0 = S.assemble(g, e, alpha, beta)
    for M in (B, B0, B + B0):
        scale = np.abs(M).max()
        assert np.abs(M - M.T).max() < 1e-14 * scale
        assert np.abs(M.sum(1)).max() < 1e-13 * scale
        assert np.linalg.eigvalsh(M).min() > -1e-12 * scale
    # B0 is a genuine low-order term: it is not a multiple of B
    assert np.linalg.matrix_rank(np.stack([B.ravel(), B0.ravel()])) == 2


@pytest.mark.parametrize("alpha,beta", PARAMS)
def test_scaling_and_rigid_motion(alpha, beta):
    g, e = gen.trefoil(32, seed=13)
    A = sum(S.assemble(g, e, alpha, beta))
    _, sigma = S.orders(alpha, beta)
    lam = 0.6
    As = sum(S.assemble(lam * g, e, alpha, beta))
    assert np.allclose(As, lam ** (-(2 * sigma + 1)) * A, rtol=1e-11, atol=1e-12 * np.abs(As).max())
    q, _ = np.linalg.qr(np.random.default_rng(1).normal(size=(3, 3)))
    Ar = sum(S.assemble(g @ q.T + 4.0, e, alpha, beta))
    assert np.allclose(Ar, A, rtol=1e-11, atol=1e-12 * np.abs(A).max())


@pytest.mark.parametrize("alpha,beta", PARAMS)
def test_ngon_circulant_fft_spectrum(alpha, beta):
    n = 40
    g, e = gen.regular_ngon(n, radius=0.8)
    A = sum(S.assemble(g, e, alpha, beta))
    for k in range(1, n):
        assert np.allclose(np.roll(A[0], k), A[k], rtol=1e-11, atol=1e-12 * np.abs(A).max())
    fft_eigs = np.sort(np.fft.fft(A[0]).real)
    assert np.allclose(fft_eigs, np.linalg.eigvalsh(A), rtol=1e-9, atol=1e-10 * np.abs(A).max())


@pytest.mark.parametrize("alpha,beta", PARAMS)
def test_midpoint_increments_equal_kernel_matrix_form(alpha, beta):
    g, e = gen.trefoil(30, seed=14)
    Bm, B0m = S.assemble(g, e, alpha, beta, quadrature="midpoint")
    u = np.random.default_rng(2).normal(size=len(g))
    ref = (Bm + B0m) @ u
    got = S.kernel_matrix_apply(g, e, alpha, beta, u)
    assert np.allclose(got, ref, rtol=1e-11, atol=1e-12 * np.abs(ref).max())


def test_rows_and_apply():
    g, e = gen.trefoil(24, seed=15)
    A = sum(S.assemble(g, e, 2, 4.5))
    R = S.assemble_rows(g, e, 2, 4.5, [0, 5, 23])
    assert np.allclose(R, A[[0, 5, 23]], rtol=1e-12, atol=1e-13 * np.abs(A).max())
    X = np.random.default_rng(3).normal(size=(24, 3))
    assert np.allclose(S.apply(g, e, 2, 4.5, X), A @ X)


def test_low_order_kernel_is_always_2_4():
    # w0 uses k_{2,4} whatever the energy exponents: with the same sigma,
    # two (alpha, beta) choices give the same B0
    g, e = gen.trefoil(20, seed=16)
    # sigma = (beta-1)/alpha - 1 is 0.75 for (2, 4.5) and for (4, 8)
    _, B0a = S.assemble(g, e, 2.0, 4.5)
    _, B0b = S.assemble(g, e, 4.0, 8.0)
    assert np.allclose(B0a, B0b, rtol=1e-13)
