"""GPU parity of the assembled 16-bit Sobolev block and the refined solve.

The stored operator A^ = D^1/2 (S^_off + diag sigma) D^1/2 is compared with the
FP64 oracle's A = B + B0 (Sec. 4.2.2-4.2.3):

* single product: every output entry lies within the rounding bound of the
  16-bit storage, u * sum_w |A_vw| (|x_w| + |x_v|) (the second term is the
  recomputed diagonal), plus FP32 accumulation over the column tiles and, for
  FP16, the absolute spacing of its subnormals;
* constants: A^ 1 = 0 up to FP32 accumulation;
* symmetry of the stored block;
* refined solve of the projected gradient problem (eq.
  GradientSaddlePointProblem): the FP64 true residual, recomputed on the CPU
  with the oracle's A and C, is below the tolerance, and the solution agrees
  with the oracle's dense saddle solve.
"""

import numpy as np
import pytest

import gen
from oracle import constraints as cons
from oracle import solve, sobolev, tpe
from tests.gpu_util import banner, dev, host, relnorm, zeros

pytestmark = pytest.mark.gpu

BARY = 1
UNIT = {1: 2.0 ** -8, 2: 2.0 ** -11}  # unit roundoff of BF16 and FP16
NAME = {1: "bf16", 2: "fp16"}


def product_bound(A, X, fmt, n):
    """Entrywise bound of |A^ X - A X| (see the module docstring)."""
    off = np.abs(A - np.diag(np.diag(A)))
    ax = np.abs(X)
    s = off @ ax + off.sum(axis=1)[:, None] * ax
    nkt = -(-n // 32)
    gamma = (nkt + 64) * 2.0 ** -24
    b = (UNIT[fmt] + gamma) * s
    if fmt == 2:
        d = np.sqrt(np.diag(A))
        b += 2.0 ** -24 * d[:, None] * (np.abs(d)[None, :] @ ax)
    return b


def rows_bound(R, rows, X, fmt, n):
    off = np.abs(R.copy())
    for k, v in enumerate(rows):
        off[k, v] = 0.0
    ax = np.abs(X)
    s = off @ ax + off.sum(axis=1)[:, None] * ax[rows]
    nkt = -(-n // 32)
    return (UNIT[fmt] + (nkt + 64) * 2.0 ** -24) * s


def ctx_for(g, e, a, b):
    from paper_2006_07859_amd import RC_F32, Context

    return Context(len(g), e, a, b, RC_F32)


@pytest.mark.parametrize("fmt", [1, 2])
@pytest.mark.parametrize("band", [0, 16, 40])
@pytest.mark.parametrize("alpha,beta", [(2.0, 4.5), (3.0, 6.0)])
def test_single_product_bound(lib, fmt, band, alpha, beta):
    n = 1000  # 63 row blocks, 32 column tiles: ragged in both directions
    banner(f"lowp product {NAME[fmt]} band={band} ({alpha},{beta}) fourier{n}")
    g, e, _ = gen.fourier_knot(n, seed=3)
    g = gen.round_to_f32(g)
    A = sum(sobolev.assemble(g, e, alpha, beta))
    ctx = ctx_for(g, e, alpha, beta)
    with32 = band > 0
    ctx.rc_lowp_assemble(dev(g), fmt, band, with32)
    X = np.random.default_rng(5).normal(size=(n, 3))
    Y = zeros(n, 3)
    ctx.rc_lowp_apply(dev(X), Y)
    y = host(Y)
    ref = A @ X
    err = np.abs(y - ref)
    bound = product_bound(A, X, fmt, n)
    print(f"  normwise rel err {relnorm(y, ref):.3e}  max err/bound {np.max(err / bound):.3f}")
    assert np.all(err <= bound)
    if with32:
        # FP32 block: entries outside the band evaluated in FP32 from FP32 coordinates
        # (a few ulps, more where chain-far vertices come close), stored without rounding
        ctx.rc_lowp_apply(dev(X), Y, True)
        y32 = host(Y)
        b32 = product_bound(A, X, 1, n) * (2.0 ** -18 / UNIT[1])
        print(f"  fp32 block: normwise rel err {relnorm(y32, ref):.3e}  max err/bound {np.max(np.abs(y32 - ref) / b32):.3f}")
        assert np.all(np.abs(y32 - ref) <= b32)
    # constants are annihilated up to FP32 accumulation
    ones = np.ones((n, 3))
    ctx.rc_lowp_apply(dev(ones), Y)
    s = np.abs(A - np.diag(np.diag(A))).sum(axis=1)
    assert np.all(np.abs(host(Y)) <= ((-(-n // 32)) + 64) * 2.0 ** -23 * 2 * s[:, None])
    # symmetry of the stored operator: x . A^ y = y . A^ x up to FP32 accumulation
    Z = np.random.default_rng(6).normal(size=(n, 3))
    ctx.rc_lowp_apply(dev(Z), Y)
    xy = float(np.sum(X * host(Y)))
    ctx.rc_lowp_apply(dev(X), Y)
    yx = float(np.sum(Z * host(Y)))
    scale = float(np.sum(np.abs(X) * (np.abs(A) @ np.abs(Z))))
    assert abs(xy - yx) <= 1e-5 * scale
    ctx.close()


def test_band_improves_single_product(lib):
    n = 1000
    banner(f"lowp band effect bf16 fourier{n}")
    g, e, _ = gen.fourier_knot(n, seed=3)
    g = gen.round_to_f32(g)
    A = sum(sobolev.assemble(g, e, 2.0, 4.5))
    ctx = ctx_for(g, e, 2.0, 4.5)
    # a smooth input: the regime where rounding of near entries matters most
    t = np.linspace(0, 2 * np.pi, n, endpoint=False)
    X = np.stack([np.cos(t), np.sin(2 * t), np.cos(3 * t)], axis=1)
    ref = A @ X
    errs = []
    for band in (0, 16):
        ctx.rc_lowp_assemble(dev(g), 1, band)
        Y = zeros(n, 3)
        ctx.rc_lowp_apply(dev(X), Y)
        errs.append(relnorm(host(Y), ref))
    print(f"  smooth-mode rel err band 0: {errs[0]:.3e}  band 16: {errs[1]:.3e}")
    assert errs[1] < errs[0]
    ctx.close()


@pytest.mark.parametrize("fmt", [1, 2])
def test_full_size_sampled_rows(lib, fmt):
    n = 32768
    banner(f"lowp product {NAME[fmt]} band=16 fourier{n} sampled rows")
    g, e, _ = gen.fourier_knot(n, seed=0)
    g = gen.round_to_f32(g)
    ctx = ctx_for(g, e, 2.0, 4.5)
    ctx.rc_lowp_assemble(dev(g), fmt, 16)
    X = np.random.default_rng(7).normal(size=(n, 3))
    Y = zeros(n, 3)
    ctx.rc_lowp_apply(dev(X), Y)
    y = host(Y)
    rows = [0, 5, 16001, 32767]
    R = sobolev.assemble_rows(g, e, 2.0, 4.5, rows)
    ref = R @ X
    bound = rows_bound(R, rows, X, fmt, n)
    err = np.abs(y[rows] - ref)
    print(f"  sampled max err/bound {np.max(err / bound):.3f}")
    assert np.all(err <= bound)
    # constants
    ctx.rc_lowp_apply(dev(np.ones((n, 3))), Y)
    s = np.abs(R).sum(axis=1) - np.abs(R[np.arange(len(rows)), rows])
    assert np.all(np.abs(host(Y)[rows]) <= ((n // 32) + 64) * 2.0 ** -23 * 2 * s[:, None])
    ctx.close()


OUTER = {0: "matrix-free FP64 Krylov", 1: "assembled FP32 Krylov + FP64 refinement"}
INNER = {0: 0.0, 1: 1e-2}  # refinement sweeps only where the Krylov operator is not FP64


@pytest.mark.parametrize("fmt,outer", [(1, 0), (2, 0), (1, 1), (2, 1)])
def test_refined_solve_matches_oracle(lib, fmt, outer):
    from paper_2006_07859_amd import RC_SOLVE_PCG_MG, default_solve_opts

    n = 2048
    banner(f"lowp solve {NAME[fmt]} smoothers, {OUTER[outer]}, fourier{n} barycenter")
    g, e, _ = gen.fourier_knot(n, seed=1)
    g = gen.round_to_f32(g)
    refs = cons.reference_values(g, e)
    _, dE = tpe.differential(g, e, 2.0, 4.5)
    A = sum(sobolev.assemble(g, e, 2.0, 4.5))
    _, C = cons.evaluate(g, e, BARY, *refs)
    g_ref, _ = solve.projected_gradient(A, C, dE)
    ctx = ctx_for(g, e, 2.0, 4.5)
    ctx.rc_set_constraints(BARY, dev(g))
    out = zeros(n, 3)
    o = default_solve_opts(solver=RC_SOLVE_PCG_MG, tol=1e-8, lowp=fmt, lowp_band=16, lowp_min_vertices=1024,
                           lowp_outer=outer, mg_min_vertices=256, inner_tol=INNER[outer], max_iter=400)
    st = ctx.rc_sobolev_gradient(dev(g), dev(dE), out, o)
    x = host(out).ravel()
    # residual of the projected system recomputed with the oracle's A and C
    Ab = np.kron(A, np.eye(3))
    P = lambda v: v - C.T @ np.linalg.solve(C @ C.T, C @ v)  # noqa: E731
    b = P(dE.ravel())
    res = np.linalg.norm(P(b - Ab @ x)) / np.linalg.norm(b)
    e_a = x - g_ref.ravel()
    aerr = np.sqrt(e_a @ Ab @ e_a) / np.sqrt(g_ref.ravel() @ Ab @ g_ref.ravel())
    print(f"  its {st['iterations']} sweeps {st['sweeps']} gpu res {st['residual']:.2e} oracle res {res:.2e}"
          f" rel err {relnorm(x, g_ref.ravel()):.2e} A-norm err {aerr:.2e}")
    assert st["residual"] < 1e-8
    assert res < 2e-8
    assert relnorm(x, g_ref.ravel()) < 1e-5
    assert aerr < 1e-6
    ctx.close()


@pytest.mark.parametrize("fmt,outer", [(1, 0), (2, 0), (2, 1)])
def test_full_size_refined_solve(lib, fmt, outer):
    from paper_2006_07859_amd import RC_SOLVE_PCG_MG, default_solve_opts

    n = 32768
    banner(f"lowp solve {NAME[fmt]} smoothers, {OUTER[outer]}, fourier{n} barycenter, FP64 comparison")
    g, e, _ = gen.fourier_knot(n, seed=0)
    g = gen.round_to_f32(g)
    ctx = ctx_for(g, e, 2.0, 4.5)
    gam = dev(g)
    ctx.rc_set_constraints(BARY, gam)
    E = zeros(1)
    dE = zeros(n, 3)
    ctx.rc_differential(gam, E, dE)
    out = zeros(n, 3)
    o = default_solve_opts(solver=RC_SOLVE_PCG_MG, tol=1e-8, lowp=fmt, lowp_band=16, lowp_min_vertices=4096,
                           lowp_outer=outer, mg_min_vertices=256, inner_tol=3 * INNER[outer], max_iter=400)
    st = ctx.rc_sobolev_gradient(gam, dE, out, o)
    print(f"  its {st['iterations']} sweeps {st['sweeps']} res {st['residual']:.2e}")
    assert st["residual"] < 1e-8
    # the same system solved with the FP64 matrix-free operator throughout, to a
    # tighter residual (the FP64 operator's own floor at this size is near 1e-10)
    ref = zeros(n, 3)
    st64 = ctx.rc_sobolev_gradient(gam, dE, ref, default_solve_opts(solver=RC_SOLVE_PCG_MG, tol=2e-9, op_f64=1,
                                                                    mg_min_vertices=256, max_iter=400))
    d = relnorm(host(out), host(ref))
    print(f"  fp64 its {st64['iterations']} res {st64['residual']:.2e}  rel diff {d:.2e}")
    assert d < 1e-5
    ctx.close()
