"""GPU parity of the batch path: many packing instances in one context.

Every instance is checked against the FP64 oracle on its own: tangent-point
energy and differential (Sec. 4.1) plus the sphere-obstacle penalty (Sec. 7.1,
surface potential), the operator A = B + B0 (Sec. 4.2), and the projected
gradient of eq. GradientSaddlePointProblem with that instance's barycenter
and per-loop length constraints.  The step is checked through its
guarantees (Armijo decrease at the accepted length, constraints restored)
and the captured hipGraph must reproduce the eager step exactly.
"""

import numpy as np
import pytest

import gen
from oracle import constraints as cons
from oracle import obstacle, solve, sobolev, tpe
from tests.gpu_util import banner, dev, host, relnorm, zeros

pytestmark = pytest.mark.gpu

ALPHA, BETA = 3.0, 6.0
CENTER, RADIUS = (0.5, 0.5, 0.5), 0.25


def union(insts):
    gs, es, off, voff = [], [], 0, [0]
    for g, e, _ in insts:
        gs.append(g)
        es.append(np.asarray(e) + off)
        off += len(g)
        voff.append(off)
    return np.concatenate(gs), np.concatenate(es).astype(np.int32), np.asarray(voff)


def small_batch(n=6, seed=7, e_min=40, e_max=300):
    rng = np.random.default_rng(seed)
    return [gen.packing_instance(rng, e_min=e_min, e_max=e_max) for _ in range(n)]


def make_batch(insts, obstacle_on=True):
    from paper_2006_07859_amd import Batch, RC_F32

    g, e, voff = union(insts)
    b = Batch(voff, e, ALPHA, BETA, RC_F32)
    if obstacle_on:
        b.rc_set_obstacle(CENTER, RADIUS, 1.0)
    return b, g, e, voff


def oracle_energy(g, e):
    E, dE = tpe.differential(g, e, ALPHA, BETA)
    E += obstacle.penalty(g, e, CENTER, RADIUS, BETA - ALPHA)
    dE = dE + obstacle.penalty_gradient(g, e, CENTER, RADIUS, BETA - ALPHA)
    return E, dE


@pytest.mark.parametrize("tiling", [None, (256, 2)])
def test_energies_and_differential(lib, tiling):
    insts = small_batch()
    banner(f"batch energies {len(insts)} instances tiling={tiling}")
    b, g, e, voff = make_batch(insts)
    if tiling:
        b.rc_batch_tiling(*tiling)  # several source chunks per instance
    En = zeros(len(insts))
    dE = zeros(len(g), 3)
    b.rc_batch_energies(dev(g), En, dE)
    En, dE = host(En), host(dE)
    for i, (gi, ei, _) in enumerate(insts):
        Er, dEr = oracle_energy(gi, ei)
        assert En[i] == pytest.approx(Er, rel=1e-5)
        assert relnorm(dE[voff[i]:voff[i + 1]], dEr) < 1e-4
    # the whole-context energy is the sum over instances
    Et = zeros(1)
    b.rc_energy(dev(g), Et)
    assert host(Et)[0] == pytest.approx(En.sum(), rel=1e-12)
    b.close()


def test_obstacle_term_alone(lib):
    """The batch energy minus the obstacle-free energy is the oracle's penalty."""
    insts = small_batch(n=3, seed=11)
    banner("batch obstacle penalty")
    b, g, e, voff = make_batch(insts, obstacle_on=True)
    E1 = zeros(len(insts))
    b.rc_batch_energies(dev(g), E1)
    b.rc_set_obstacle(CENTER, RADIUS, 0.0)
    E0 = zeros(len(insts))
    b.rc_batch_energies(dev(g), E0)
    for i, (gi, ei, _) in enumerate(insts):
        pen = obstacle.penalty(gi, ei, CENTER, RADIUS, BETA - ALPHA)
        assert host(E1)[i] - host(E0)[i] == pytest.approx(pen, rel=1e-9)
    b.close()


def test_operator_is_block_diagonal(lib):
    insts = small_batch(n=4, seed=3)
    banner("batch operator: matrix-free and assembled blocks")
    b, g, e, voff = make_batch(insts)
    rng = np.random.default_rng(1)
    X = rng.normal(size=g.shape)
    # a smooth input too: the assembled product's difference form must not cancel
    Xs = np.sin(2.0 * g) + 0.3 * g ** 2
    Y = zeros(len(g), 3)
    b.rc_sobolev_apply(dev(g), dev(X), Y)
    Ys = {}
    b.rc_batch_set_constraints(dev(g))
    for assembled in (False, True):
        for name, inp in (("random", X), ("smooth", Xs)):
            out = zeros(len(g), 3)
            b.rc_batch_sobolev_apply(dev(g), dev(inp), out, assembled)
            Ys[(assembled, name)] = host(out)
    for i, (gi, ei, _) in enumerate(insts):
        A = sum(sobolev.assemble(gi, ei, ALPHA, BETA))
        sl = slice(voff[i], voff[i + 1])
        assert relnorm(host(Y)[sl], A @ X[sl]) < 1e-5
        for (assembled, name), out in Ys.items():
            ref = A @ (X if name == "random" else Xs)[sl]
            err = relnorm(out[sl], ref)
            print(f"  instance {i} assembled={assembled} {name}: rel {err:.1e}")
            assert err < (1e-5 if name == "random" else 3e-5)
    b.close()


@pytest.mark.parametrize("coarse,op", [(1, 1), (0, 1), (1, 0)])
def test_gradient_matches_oracle(lib, coarse, op):
    from paper_2006_07859_amd import default_batch_opts

    insts = small_batch(n=5, seed=5, e_max=400)
    banner(f"batch projected gradient {len(insts)} instances, coarse space {coarse}, assembled operator {op}")
    b, g, e, voff = make_batch(insts)
    gam = dev(g)
    b.rc_batch_set_constraints(gam)
    En = zeros(len(insts))
    dE = zeros(len(g), 3)
    b.rc_batch_energies(gam, En, dE)
    out = zeros(len(g), 3)
    # iterative refinement: FP32-operator PCG sweeps to 1e-4 on the FP64 matrix-free true residual
    b.rc_batch_gradient(gam, dE, out, default_batch_opts(tol=1e-7, max_iter=400, check_every=10, coarse=coarse,
                                                                 op_assembled=op, refine=3, inner_tol=1e-4))
    its, res = b.rc_batch_pcg_state()
    print(f"  iterations {its.astype(int).tolist()} residuals {np.max(res):.1e}")
    out = host(out)
    for i, (gi, ei, loops) in enumerate(insts):
        x0, _, _ = cons.reference_values(gi, ei)
        Lq = cons.loop_lengths(gi, ei)
        _, C = cons.evaluate(gi, ei, cons.BARYCENTER | cons.LOOP_LENGTH, x0, Lq=Lq)
        A = sum(sobolev.assemble(gi, ei, ALPHA, BETA))
        _, dEr = oracle_energy(gi, ei)
        g_ref, _ = solve.projected_gradient(A, C, dEr)
        gi_out = out[voff[i]:voff[i + 1]]
        Ab = np.kron(A, np.eye(3))
        err = gi_out.ravel() - g_ref.ravel()
        aerr = np.sqrt(err @ Ab @ err) / np.sqrt(g_ref.ravel() @ Ab @ g_ref.ravel())
        print(f"  instance {i}: n={len(gi)} loops={len(loops)} rel {relnorm(gi_out, g_ref):.2e} A-norm {aerr:.2e}")
        assert res[i] < 1e-7  # the final FP64 true residual
        assert aerr < 1e-4 and relnorm(gi_out, g_ref) < 1e-4
        assert np.abs(C @ gi_out.ravel()).max() < 1e-8 * np.abs(gi_out).max()
    b.close()


def test_step_guarantees_and_graph_replay(lib):
    from paper_2006_07859_amd import default_batch_opts

    insts = small_batch(n=6, seed=9)
    banner(f"batch step {len(insts)} instances, eager vs captured graph")
    b, g, e, voff = make_batch(insts)
    g0 = dev(g)
    b.rc_batch_set_constraints(g0)
    opts = default_batch_opts(tol=1e-5, max_iter=200, check_every=0)
    gam = g0.clone()
    st = b.rc_batch_step(gam, opts)
    new = host(gam)
    print("  status", st[:, 5].astype(int).tolist(), "tau", st[:, 2].tolist())
    for i, (gi, ei, _) in enumerate(insts):
        gn = new[voff[i]:voff[i + 1]]
        E0, _ = oracle_energy(gi, ei)
        assert st[i, 0] == pytest.approx(E0, rel=1e-5)
        if st[i, 5] == 0:
            E1, _ = oracle_energy(gn, ei)
            assert st[i, 1] == pytest.approx(E1, rel=1e-5)
            assert E1 < E0
            x0, L, _ = cons.reference_values(gi, ei)
            Lq = cons.loop_lengths(gi, ei)
            phi, _ = cons.evaluate(gn, ei, cons.BARYCENTER | cons.LOOP_LENGTH, x0, Lq=Lq, jacobian=False)
            assert np.all(np.abs(phi[3:]) <= 1.01e-6 * Lq)
            assert np.all(np.abs(phi[:3]) <= 1.01e-6 * L * L)
        else:
            assert np.array_equal(gn, gi)
    assert (st[:, 5] == 0).sum() >= len(insts) - 1
    # the captured step reproduces the eager step bit for bit, replay after replay
    opts_g = default_batch_opts(tol=1e-5, max_iter=200, check_every=0, graph=1)
    gam_g = g0.clone()
    for rep in range(3):
        gam_g.copy_(g0)
        gam.copy_(g0)
        st_e = b.rc_batch_step(gam, opts)
        st_g = b.rc_batch_step(gam_g, opts_g)
        assert np.array_equal(host(gam), host(gam_g)), f"replay {rep}"
        assert np.array_equal(st_e, st_g), f"replay {rep}"
    b.close()


def test_full_batch_512(lib):
    from paper_2006_07859_amd import default_batch_opts

    insts = gen.packing_batch(512, seed=0)
    g, e, voff = union(insts)
    banner(f"batch 512 instances, {len(e)} edges")
    b, g, e, voff = make_batch(insts)
    gam = dev(g)
    En = zeros(512)
    dE = zeros(len(g), 3)
    b.rc_batch_energies(gam, En, dE)
    En = host(En)
    # sampled instances against the oracle (the smallest ones keep the oracle fast)
    sizes = np.diff(voff)
    for i in np.argsort(sizes)[:4].tolist() + [int(np.argsort(sizes)[200])]:
        gi, ei, _ = insts[i]
        Er, dEr = oracle_energy(gi, ei)
        assert En[i] == pytest.approx(Er, rel=1e-5)
        assert relnorm(host(dE)[voff[i]:voff[i + 1]], dEr) < 1e-4
    b.rc_batch_set_constraints(gam)
    st = b.rc_batch_step(gam, default_batch_opts(check_every=5))
    ok = st[:, 5] == 0
    print(f"  accepted {ok.sum()} / 512, PCG iterations max {st[:, 3].max():.0f}, "
          f"mean {st[:, 3].mean():.1f}, energy drop {np.mean((st[ok, 0] - st[ok, 1]) / st[ok, 0]):.2e}")
    assert ok.sum() >= 500
    assert np.all(st[ok, 1] < st[ok, 0])
    b.close()


def test_autotune_and_cache(lib, tmp_path):
    insts = small_batch(n=8, seed=13, e_max=2000)
    banner("batch tile autotuner with cache")
    b, g, e, voff = make_batch(insts)
    gam = dev(g)
    En0 = zeros(len(insts))
    b.rc_batch_energies(gam, En0)
    cache = tmp_path / "tune.json"
    t1 = b.rc_batch_autotune(gam, cache)
    assert t1["src_chunk"] in (512, 1024, 2048, 4096) and t1["blocks_per_cu"] in (4, 8, 16) and t1["ms"] > 0
    assert cache.exists() and "batch_pairs" in cache.read_text()
    t2 = b.rc_batch_autotune(gam, cache)  # cache hit: same choice
    assert (t2["src_chunk"], t2["blocks_per_cu"]) == (t1["src_chunk"], t1["blocks_per_cu"])
    En1 = zeros(len(insts))
    b.rc_batch_energies(gam, En1)
    # a different tiling changes only the summation order of the FP64-folded partials
    assert np.allclose(host(En1), host(En0), rtol=1e-6, atol=0)
    b.close()
