"""GPU parity of the pair kernels against the FP64 oracle, through the C ABI.

Energy and differential (Sec. 4.1), the edge-midpoint variant (App. B.1),
the operator A = B + B0 applied matrix-free, its diagonal and its dense
assembly (Sec. 4.2).  FP64 paths are held to 1e-12 (energy) / 1e-10
(differential, operator); FP32 paths to the stated 1e-5 energy and 1e-4
differential tolerances.  Sizes span several 256-edge tiles with a ragged
tail; the full 16,384-edge workload is checked on sampled vertices and by
invariances that hold at any size.
"""

import numpy as np
import pytest

import gen
from oracle import sobolev, tpe
from tests.gpu_util import banner, dev, host, relnorm, zeros

pytestmark = pytest.mark.gpu

PARAMS = [(2.0, 4.0), (2.0, 4.5), (3.0, 6.0), (2.5, 5.5)]


def ctx_for(lib, g, e, a, b, dtype):
    from paper_2006_07859_amd import Context

    return Context(len(g), e, a, b, dtype)


@pytest.mark.parametrize("alpha,beta", PARAMS)
def test_energy_differential_f64_trefoil(lib, alpha, beta):
    from paper_2006_07859_amd import RC_F64

    banner(f"energy+dE f64 trefoil256 ({alpha},{beta})")
    g, e = gen.trefoil(256, seed=0)
    E_ref, G_ref = tpe.differential(g, e, alpha, beta)
    ctx = ctx_for(lib, g, e, alpha, beta, RC_F64)
    E, dE = zeros(1), zeros(256, 3)
    ctx.rc_differential(dev(g), E, dE)
    E2 = zeros(1)
    ctx.rc_energy(dev(g), E2)
    assert host(E)[0] == pytest.approx(E_ref, rel=1e-12)
    assert host(E2)[0] == pytest.approx(E_ref, rel=1e-12)
    assert relnorm(host(dE), G_ref) < 1e-10


@pytest.mark.parametrize("alpha,beta", PARAMS)
def test_energy_differential_f32_ragged(lib, alpha, beta):
    from paper_2006_07859_amd import RC_F32

    n = 1000  # 4 tiles of 256 with a ragged tail
    banner(f"energy+dE f32 fourier{n} ({alpha},{beta})")
    g, e, _ = gen.fourier_knot(n, seed=3)
    g = gen.round_to_f32(g)
    E_ref, G_ref = tpe.differential(g, e, alpha, beta)
    ctx = ctx_for(lib, g, e, alpha, beta, RC_F32)
    E, dE = zeros(1), zeros(n, 3)
    ctx.rc_differential(dev(g), E, dE)
    assert host(E)[0] == pytest.approx(E_ref, rel=1e-5)
    assert relnorm(host(dE), G_ref) < 1e-4


def test_small_and_multi_component(lib):
    from paper_2006_07859_amd import RC_F32, RC_F64

    banner("energy+dE small loops, open path, several components")
    # two loops and an open path in one network, shuffled edge order
    g1, e1 = gen.trefoil(9, seed=1)
    g2, e2 = gen.regular_ngon(5, radius=0.7)
    g2 = g2 + [4.0, 0.0, 0.0]
    g3 = np.stack([np.linspace(0, 1, 6), np.full(6, 3.0), 0.2 * np.sin(np.arange(6))], 1)
    e3 = np.stack([np.arange(5), np.arange(1, 6)], 1)
    g = np.concatenate([g1, g2, g3])
    e = np.concatenate([e1, e2 + 9, e3 + 14]).astype(np.int32)
    e = e[np.random.default_rng(0).permutation(len(e))]
    for dt, tol in ((RC_F64, 1e-12), (RC_F32, 1e-5)):
        gg = g if dt == RC_F64 else gen.round_to_f32(g)
        E_ref, G_ref = tpe.differential(gg, e, 3.0, 6.0)
        ctx = ctx_for(lib, gg, e, 3.0, 6.0, dt)
        E, dE = zeros(1), zeros(len(g), 3)
        ctx.rc_differential(dev(gg), E, dE)
        assert host(E)[0] == pytest.approx(E_ref, rel=tol)
        assert relnorm(host(dE), G_ref) < 10 * tol


def test_f32_band_tiles_of_several_chains(lib):
    """FP32 energy + differential with the chain band on a network of two loops and an open path,
    each several 256-edge tiles long, in chain order and then shuffled: the tiles hold one chain
    (near and far along it, also across a loop's wrap), two chains, or chains whose ranges are
    disjoint, so every branch of the per-tile band classification runs against the oracle."""
    from paper_2006_07859_amd import RC_F32

    banner("energy+dE f32 two loops + open path, several tiles per chain")
    g1, e1, _ = gen.fourier_knot(700, seed=5)
    g2, e2, _ = gen.fourier_knot(600, seed=6)
    g2 = g2 + [4.0, 0.0, 0.0]
    t = np.linspace(0.0, 1.0, 401)
    g3 = np.stack([0.4 * np.cos(6 * t), 3.0 + 0.4 * np.sin(6 * t), 2.0 * t], 1)
    e3 = np.stack([np.arange(400), np.arange(1, 401)], 1)
    g = gen.round_to_f32(np.concatenate([g1, g2, g3]))
    e_ordered = np.concatenate([e1, e2 + 700, e3 + 1300]).astype(np.int32)
    e_shuffled = e_ordered[np.random.default_rng(1).permutation(len(e_ordered))]
    for e in (e_ordered, e_shuffled):
        E_ref, G_ref = tpe.differential(g, e, 2.0, 4.5)
        ctx = ctx_for(lib, g, e, 2.0, 4.5, RC_F32)
        E, dE = zeros(1), zeros(len(g), 3)
        ctx.rc_differential(dev(g), E, dE)
        assert host(E)[0] == pytest.approx(E_ref, rel=1e-5)
        assert relnorm(host(dE), G_ref) < 1e-4


@pytest.mark.parametrize("beta", [4.0, 4.5, 4.8])
def test_vertex_pair_form_against_edge_pair_form_and_oracle(lib, beta):
    """The alpha = 2 vertex-pair regrouping (default for FP32 chain graphs) and the edge-pair form, on
    one network holding a 1,000-edge knot, a 9-edge trefoil and a 5-gon (loops shorter than the near
    band, summed entirely in FP64), a 300-edge open path and a 5-edge open path, shuffled: both
    against the oracle at the FP32 tolerances, and against each other.  beta = 4.8 takes the general
    power path."""
    from paper_2006_07859_amd import RC_F32

    banner(f"energy+dE f32 vertex-pair vs edge-pair form, (2,{beta})")
    g1, e1, _ = gen.fourier_knot(1000, seed=7)
    g2, e2 = gen.trefoil(9, seed=2)
    g2 = 0.3 * g2 + [5.0, 0.0, 0.0]
    g3, e3 = gen.regular_ngon(5, radius=0.5)
    g3 = g3 + [0.0, 5.0, 0.0]
    t = np.linspace(0.0, 1.0, 301)
    g4 = np.stack([0.5 * np.cos(5 * t) - 4.0, 0.5 * np.sin(5 * t), 2.0 * t], 1)
    e4 = np.stack([np.arange(300), np.arange(1, 301)], 1)
    g5 = np.stack([np.linspace(0, 1, 6), np.full(6, -4.0), 0.2 * np.sin(np.arange(6))], 1)
    e5 = np.stack([np.arange(5), np.arange(1, 6)], 1)
    g = gen.round_to_f32(np.concatenate([g1, g2, g3, g4, g5]))
    e = np.concatenate([e1, e2 + 1000, e3 + 1009, e4 + 1014, e5 + 1315]).astype(np.int32)
    e = e[np.random.default_rng(3).permutation(len(e))]
    E_ref, G_ref = tpe.differential(g, e, 2.0, beta)
    out = {}
    for vp in (True, False):
        ctx = ctx_for(lib, g, e, 2.0, beta, RC_F32)
        ctx.rc_use_vertex_pairs(vp)
        E, dE, E2 = zeros(1), zeros(len(g), 3), zeros(1)
        ctx.rc_differential(dev(g), E, dE)
        ctx.rc_energy(dev(g), E2)
        assert host(E)[0] == pytest.approx(E_ref, rel=1e-5)
        assert host(E2)[0] == pytest.approx(host(E)[0], rel=1e-6)  # FP32 rounding of the two kernel variants
        assert relnorm(host(dE), G_ref) < 1e-4
        assert ctx.rc_sync_status() == (0, 0)
        out[vp] = (host(E)[0], host(dE))
        ctx.close()
    assert out[True][0] == pytest.approx(out[False][0], rel=2e-6)
    assert relnorm(out[True][1], out[False][1]) < 5e-5


@pytest.mark.parametrize("beta", [4.5, 4.8])
def test_vertex_pair_near_band_boundaries(lib, beta):
    """The FP64 near band of the vertex-pair form at its branch boundaries: loops of 64 to 67 vertices
    (a loop of at most 2 * 32 + 1 vertices is near in full, a longer one only within 32 steps, so
    the candidate window wraps onto itself or not) and open paths of 30 to 36 vertices (the window
    clamped at one end, at both, or at neither for the middle vertices), with pairs 3 to 32 steps
    apart in the vertex-pair form and closer ones in the edge-pair form; against the oracle at the
    FP32 tolerances and against the edge-pair form."""
    from paper_2006_07859_amd import RC_F32

    banner(f"energy+dE f32 vertex-pair near band boundaries, (2,{beta})")
    parts, edges, off = [], [], 0
    for k, m in enumerate((64, 65, 66, 67)):
        g, e = gen.trefoil(m, seed=10 + k)
        parts.append(0.4 * g + [3.0 * k, 0.0, 0.0])
        edges.append(e + off)
        off += m
    for k, m in enumerate((30, 33, 34, 35, 36)):
        t = np.linspace(0.0, 1.0, m)
        parts.append(np.stack([0.3 * np.cos(4 * t) + 3.0 * k, 4.0 + 0.3 * np.sin(4 * t), 1.5 * t], 1))
        edges.append(np.stack([np.arange(m - 1), np.arange(1, m)], 1) + off)
        off += m
    g = gen.round_to_f32(np.concatenate(parts))
    e = np.concatenate(edges).astype(np.int32)
    e = e[np.random.default_rng(4).permutation(len(e))]
    E_ref, G_ref = tpe.differential(g, e, 2.0, beta)
    out = {}
    for vp in (True, False):
        ctx = ctx_for(lib, g, e, 2.0, beta, RC_F32)
        ctx.rc_use_vertex_pairs(vp)
        E, dE = zeros(1), zeros(len(g), 3)
        ctx.rc_differential(dev(g), E, dE)
        assert host(E)[0] == pytest.approx(E_ref, rel=1e-5)
        assert relnorm(host(dE), G_ref) < 1e-4
        assert ctx.rc_sync_status() == (0, 0)
        out[vp] = (host(E)[0], host(dE))
        ctx.close()
    assert out[True][0] == pytest.approx(out[False][0], rel=2e-6)
    assert relnorm(out[True][1], out[False][1]) < 5e-5


def test_triangle_has_zero_energy(lib):
    from paper_2006_07859_amd import RC_F64

    g, e = gen.regular_ngon(3)
    ctx = ctx_for(lib, g, e, 2.0, 4.0, RC_F64)
    E, dE = zeros(1), zeros(3, 3)
    ctx.rc_differential(dev(g), E, dE)
    assert host(E)[0] == 0.0 and np.all(host(dE) == 0.0)


def test_full_size_16k_f32_sampled_and_invariants(lib):
    from paper_2006_07859_amd import RC_F32

    n = 16384
    banner(f"energy+dE f32 fourier{n} sampled")
    g, e, _ = gen.fourier_knot(n, seed=0)
    g = gen.round_to_f32(g)
    ctx = ctx_for(lib, g, e, 2.0, 4.5, RC_F32)
    E, dE = zeros(1), zeros(n, 3)
    ctx.rc_differential(dev(g), E, dE)
    G = host(dE)
    vs = [0, 4097, 12000, n - 1]
    ref = tpe.differential_at(g, e, 2.0, 4.5, vs)
    for v, r in zip(vs, ref):
        assert np.linalg.norm(G[v] - r) <= 1e-4 * np.linalg.norm(r)
    # exact identities of the full sum: translation, rotation, Euler homogeneity
    Gn = np.abs(G).max()
    assert np.abs(G.sum(0)).max() < 1e-5 * Gn * np.sqrt(n)
    Efull = host(E)[0]
    assert np.sum(g * G) == pytest.approx((2 + 2.0 - 4.5) * Efull, rel=1e-4)
    # scaling law E(lambda g) = lambda^(2 + alpha - beta) E(g) with an exact power-of-two scale
    E2 = zeros(1)
    ctx.rc_energy(dev(2.0 * g), E2)
    assert host(E2)[0] == pytest.approx(2.0 ** (2 + 2.0 - 4.5) * Efull, rel=1e-5)


@pytest.mark.parametrize("alpha,beta", [(2.0, 4.5), (3.0, 6.0)])
def test_midpoint_variant(lib, alpha, beta):
    from paper_2006_07859_amd import RC_F32, RC_F64

    banner(f"midpoint energy+dE ({alpha},{beta})")
    g, e, _ = gen.fourier_knot(700, seed=5)
    g = gen.round_to_f32(g)
    E_ref, G_ref = tpe.midpoint_differential(g, e, alpha, beta)
    for dt, te, tg in ((RC_F64, 1e-12, 1e-10), (RC_F32, 1e-5, 1e-4)):
        ctx = ctx_for(lib, g, e, alpha, beta, dt)
        E, dE = zeros(1), zeros(len(g), 3)
        ctx.rc_midpoint_differential(dev(g), E, dE)
        assert host(E)[0] == pytest.approx(E_ref, rel=te)
        assert relnorm(host(dE), G_ref) < tg


@pytest.mark.parametrize("alpha,beta", PARAMS)
def test_operator_apply_and_diag(lib, alpha, beta):
    from paper_2006_07859_amd import RC_F32, RC_F64

    n = 600
    banner(f"operator apply f64/f32 n={n} ({alpha},{beta})")
    g, e, _ = gen.fourier_knot(n, seed=7)
    g = gen.round_to_f32(g)
    B, B0 = sobolev.assemble(g, e, alpha, beta)
    A = B + B0
    X = np.random.default_rng(1).normal(size=(n, 3))
    ref = A @ X
    ctx = ctx_for(lib, g, e, alpha, beta, RC_F64)
    Y = zeros(n, 3)
    ctx.rc_sobolev_apply(dev(g), dev(X), Y, prec=RC_F64)
    assert relnorm(host(Y), ref) < 1e-10
    ctx.rc_sobolev_apply(dev(g), dev(X), Y, prec=RC_F32)
    assert relnorm(host(Y), ref) < 1e-5
    d = zeros(n)
    ctx.rc_sobolev_diag(dev(g), d)
    assert relnorm(host(d), np.diag(A)) < 1e-10
    # constants are annihilated
    ctx.rc_sobolev_apply(dev(g), dev(np.ones((n, 3))), Y, prec=RC_F64)
    assert np.abs(host(Y)).max() < 1e-9 * np.abs(A).max()


def test_operator_tiles_of_several_chains(lib):
    """The operator A = B + B0 applied matrix-free (FP64 and FP32) on two loops and an open path,
    each several 256-edge tiles long, in chain order and shuffled: tiles whose vertex ranges are
    disjoint skip the per-pair shared-vertex test, the others keep it."""
    from paper_2006_07859_amd import RC_F32, RC_F64

    banner("operator apply f64/f32 two loops + open path, several tiles per chain")
    g1, e1, _ = gen.fourier_knot(700, seed=5)
    g2, e2, _ = gen.fourier_knot(600, seed=6)
    g2 = g2 + [4.0, 0.0, 0.0]
    t = np.linspace(0.0, 1.0, 401)
    g3 = np.stack([0.4 * np.cos(6 * t), 3.0 + 0.4 * np.sin(6 * t), 2.0 * t], 1)
    e3 = np.stack([np.arange(400), np.arange(1, 401)], 1)
    g = gen.round_to_f32(np.concatenate([g1, g2, g3]))
    n = len(g)
    e_ordered = np.concatenate([e1, e2 + 700, e3 + 1300]).astype(np.int32)
    e_shuffled = e_ordered[np.random.default_rng(2).permutation(len(e_ordered))]
    X = np.random.default_rng(3).normal(size=(n, 3))
    B, B0 = sobolev.assemble(g, e_ordered, 2.0, 4.5)
    ref = (B + B0) @ X
    for e in (e_ordered, e_shuffled):
        ctx = ctx_for(lib, g, e, 2.0, 4.5, RC_F64)
        Y = zeros(n, 3)
        ctx.rc_sobolev_apply(dev(g), dev(X), Y, prec=RC_F64)
        assert relnorm(host(Y), ref) < 1e-10
        ctx.rc_sobolev_apply(dev(g), dev(X), Y, prec=RC_F32)
        assert relnorm(host(Y), ref) < 1e-5


@pytest.mark.parametrize("alpha,beta", [(2.0, 4.0), (2.0, 4.5), (3.0, 6.0)])
def test_dense_assembly(lib, alpha, beta):
    from paper_2006_07859_amd import RC_F64

    banner(f"dense assembly ({alpha},{beta})")
    g, e = gen.trefoil(256, seed=0)
    A_ref = sum(sobolev.assemble(g, e, alpha, beta))
    ctx = ctx_for(lib, g, e, alpha, beta, RC_F64)
    A = zeros(256, 256)
    ctx.rc_assemble_dense(dev(g), A)
    assert np.abs(host(A) - A_ref).max() < 1e-11 * np.abs(A_ref).max()


def test_operator_full_size_sampled(lib):
    from paper_2006_07859_amd import RC_F32

    n = 16384
    banner(f"operator f32 fourier{n} sampled rows")
    g, e, _ = gen.fourier_knot(n, seed=0)
    g = gen.round_to_f32(g)
    X = np.random.default_rng(2).normal(size=(n, 3))
    ctx = ctx_for(lib, g, e, 2.0, 4.5, RC_F32)
    Y = zeros(n, 3)
    ctx.rc_sobolev_apply(dev(g), dev(X), Y)
    rows = [5, 9000]
    R = sobolev.assemble_rows(g, e, 2.0, 4.5, rows)
    for k, v in enumerate(rows):
        ref = R[k] @ X
        assert np.linalg.norm(host(Y)[v] - ref) < 1e-4 * np.linalg.norm(ref)
