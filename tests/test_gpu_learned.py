"""GPU parity of the learned smoother weights against oracle/learned.py.

* MLP forward (FP16 weights and first hidden layer, FP32 accumulation)
  against the FP64 oracle run on the same FP16-rounded weights and inputs,
  within a first-order bound of the hidden layer's FP16 rounding.
* MLP backward against the oracle's gradient, Adam against its update.
* Level sizes, FP64 level diagonals and the features of every level.
* The training targets (row l1 / diagonal ratios of every level's operator
  times the top eigenvalue of the ratio-scaled operator) against the oracle's; one regression step's loss and gradient against the
  oracle's on the same network output.
* PCG with the learned V-cycle reaches the oracle's projected gradient.
* Trained on snapshots of plain flows, the learned V-cycle reaches 1e-6 on
  held-out knots of 4,096-16,384 edges in less wall time than the hand-set
  V-cycle (and Jacobi PCG does not reach it within its cap).
"""

import numpy as np
import pytest

import gen
from oracle import constraints as cons
from oracle import learned as lp
from oracle import solve, sobolev, tpe
from tests.gpu_util import banner, dev, host, relnorm, zeros

pytestmark = pytest.mark.gpu

ALPHA, BETA = 2.0, 4.5
U16 = 2.0 ** -11  # unit roundoff of FP16


def f32(a):
    import torch

    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32), device="cuda")


def theta16(theta):
    """Weights rounded to FP16 as the forward pass uses them; biases stay FP32."""
    t = np.asarray(theta, dtype=np.float32).astype(np.float64)
    out = t.copy()
    W1, b1, W2, b2, W3, b3 = lp.unpack(out)
    for w in (W1, W2, W3):
        w[...] = w.astype(np.float16).astype(np.float64)
    return out


def forward_bound(th, X):
    """First-order bound on |y_gpu - y_oracle| from rounding the first hidden
    layer to FP16 (softplus is 1-Lipschitz) plus FP32 accumulation."""
    W1, b1, W2, b2, W3, b3 = lp.unpack(th)
    y, (X_, a1, h1, a2, h2, o) = lp.forward(th, X)
    prop = np.abs(h1) @ np.abs(W2) @ np.abs(W3)
    acc = np.abs(X) @ np.abs(W1) @ np.abs(W2) @ np.abs(W3) + np.abs(h2) @ np.abs(W3) + abs(b3[0])
    return 1.05 * U16 * prop + 64 * 2.0 ** -24 * acc + 1e-6


def perturbed_params(seed, scale=0.1):
    return lp.init_params(seed) + scale * np.random.default_rng(seed + 100).normal(size=lp.n_params())


@pytest.mark.parametrize("N", [1000, 64, 1])
def test_mlp_forward(lib, N):
    from paper_2006_07859_amd import Mlp

    banner(f"MLP forward N={N}")
    rng = np.random.default_rng(N)
    theta = perturbed_params(1)
    X = rng.normal(size=(N, 8)).astype(np.float16).astype(np.float64)
    m = Mlp(theta)
    Y = f32(np.zeros(N))
    m.forward(f32(X), Y)
    th = theta16(theta)
    yr, _ = lp.forward(th, X)
    err = np.abs(host(Y) - yr)
    bound = forward_bound(th, X)
    print(f"  max err {err.max():.2e}, max bound {bound.max():.2e}")
    assert np.all(err <= bound)
    # get returns the FP32 master copy
    assert np.array_equal(m.get(), theta.astype(np.float32))
    m.close()


def test_mlp_backward_and_adam(lib):
    import torch

    from paper_2006_07859_amd import Mlp

    banner("MLP backward and Adam")
    rng = np.random.default_rng(5)
    N = 1777
    theta = perturbed_params(2)
    X = rng.normal(size=(N, 8)).astype(np.float16).astype(np.float64)
    th = theta16(theta)
    _, cache = lp.forward(th, X)
    # Rows with a ReLU input within the FP16 rounding of the first hidden layer
    # of zero may switch that unit on the device: they get no weight (dy = 0).
    W1, b1, W2, b2, W3, b3 = lp.unpack(th)
    a1, h1, a2 = cache[1], cache[2], cache[3]
    near = U16 * (np.abs(h1) @ np.abs(W2)) + 1e-5
    safe = np.all(np.abs(a2) > 4 * near, axis=1) & np.all(np.abs(a1) > 1e-5, axis=1)
    assert safe.sum() > N // 4
    dy = np.where(safe, rng.normal(size=N), 0.0)
    m = Mlp(theta)
    grad = torch.zeros(lp.n_params(), dtype=torch.float32, device="cuda")
    m.backward(f32(X), f32(dy), grad)
    gr = lp.backward(th, cache, dy.astype(np.float32).astype(np.float64))
    g = host(grad).astype(np.float64)
    names = ["W1", "b1", "W2", "b2", "W3", "b3"]
    k = 0
    for name, part in zip(names, lp.unpack(gr)):
        n = part.size
        e = relnorm(g[k:k + n], part.ravel())
        print(f"  {name}: rel {e:.2e}")
        assert e < 5e-3, name
        k += n
    # two Adam steps with that gradient against the oracle's update of the FP32 parameters
    t0 = theta.astype(np.float32).astype(np.float64)
    mm = vv = np.zeros(lp.n_params())
    t1, mm, vv = lp.adam_step(t0, g, mm, vv, 1, 1e-3)
    t2, mm, vv = lp.adam_step(t1, g, mm, vv, 2, 1e-3)
    m.adam(grad, 1e-3)
    m.adam(grad, 1e-3)
    got = m.get().astype(np.float64)
    assert np.abs(got - t2).max() < 2e-6 + 1e-6 * np.abs(t2).max()
    # set resets Adam: one step from the new point is again -lr sign(g)
    m.set(theta)
    m.adam(grad, 1e-3)
    step = m.get().astype(np.float64) - theta.astype(np.float32)
    big = np.abs(g) > 1e-4
    assert np.allclose(step[big], -1e-3 * np.sign(g[big]), rtol=1e-3, atol=1e-7)
    m.close()


def knot(n, seed):
    g, e, _ = gen.fourier_knot(n, seed=seed)
    return g, e


def context(g, e):
    from paper_2006_07859_amd import RC_C_BARYCENTER, RC_F32, Context

    ctx = Context(len(g), e, ALPHA, BETA, RC_F32)
    ctx.rc_set_constraints(RC_C_BARYCENTER, dev(g))
    return ctx


@pytest.mark.parametrize("n,n_min", [(1000, 64), (999, 40), (1024, 256)])
def test_levels_diagonals_features(lib, n, n_min):
    import torch

    banner(f"levels, diagonals and features n={n} n_min={n_min}")
    g, e = knot(n, 3)
    ctx = context(g, e)
    gammas, _ = lp.hierarchy(g, n_min)
    sizes = ctx.rc_learned_levels(n_min)
    assert sizes == [len(x) for x in gammas]
    N = sum(sizes)
    X = torch.zeros(N, 8, dtype=torch.float32, device="cuda")
    diag = zeros(N)
    ctx.rc_learned_features(dev(g), n_min, X, diag)
    diags = lp.level_diagonals(gammas, ALPHA, BETA)
    assert relnorm(host(diag), np.concatenate(diags)) < 1e-10
    for a, b in zip(np.split(host(diag), np.cumsum(sizes)[:-1]), diags):
        assert np.abs(a / b - 1).max() < 1e-10
    F = lp.features(gammas, diags)
    err = np.abs(host(X) - F)
    print("  max feature error per column", np.array2string(err.max(0), precision=1))
    assert np.all(err <= 2e-6 * (1 + np.abs(F)))
    ctx.close()


def test_targets_match_oracle(lib):
    import torch

    n, n_min = 1000, 100
    banner(f"learned-smoother targets n={n} n_min={n_min}")
    g, e = knot(n, 5)
    ctx = context(g, e)
    sizes = ctx.rc_learned_levels(n_min)
    R = torch.zeros(sum(sizes), dtype=torch.float32, device="cuda")
    ctx.rc_learned_targets(dev(g), n_min, R)
    gammas, _ = lp.hierarchy(g, n_min)
    ref = lp.targets(lp.level_operators(gammas, ALPHA, BETA))
    err = (host(R) - ref) / ref
    print(f"  sizes {sizes}, targets {ref.min():.3f}..{ref.max():.3f}, rel err {err.min():.1e}..{err.max():.1e}")
    # the power method's Rayleigh quotient approaches the top eigenvalue from below
    assert err.max() < 1e-6 and err.min() > -5e-3
    ctx.close()


def test_fit_step_matches_oracle(lib):
    import torch

    from paper_2006_07859_amd import Mlp

    banner("MLP regression step")
    rng = np.random.default_rng(11)
    theta = perturbed_params(4, 0.05)
    th = theta16(theta)
    X = rng.normal(size=(3000, 8)).astype(np.float16).astype(np.float64)
    _, cache = lp.forward(th, X)
    W1, b1, W2, b2, W3, b3 = lp.unpack(th)
    a1, h1, a2 = cache[1], cache[2], cache[3]
    near = U16 * (np.abs(h1) @ np.abs(W2)) + 1e-5
    safe = np.all(np.abs(a2) > 4 * near, axis=1) & np.all(np.abs(a1) > 1e-5, axis=1)
    X = X[safe]
    N = len(X)
    assert N > 500
    y_or, cache = lp.forward(th, X)
    # targets clear of the under/over switch at p = R
    R = (1.0 + y_or) * np.exp(np.where(rng.random(N) < 0.5, 1.0, -1.0) * rng.uniform(0.05, 0.4, size=N))
    R = np.maximum(R, 1.0 + 1e-3)
    m = Mlp(theta)
    Xd, Rd = f32(X), f32(R)
    Y = f32(np.zeros(N))
    m.forward(Xd, Y)
    y = host(Y).astype(np.float64)
    grad = torch.zeros(lp.n_params(), dtype=torch.float32, device="cuda")
    loss = m.fit_step(Xd, Rd, 0.0, grad)
    # the oracle's loss and gradient on the device's output y (the forward is checked separately)
    Rf = R.astype(np.float32).astype(np.float64)
    p = 1.0 + y
    ev = np.log(p) - np.log(Rf)
    w = np.where(p < Rf, lp.UNDER, 1.0)
    assert loss == pytest.approx(float(np.mean(w * ev * ev)), rel=1e-5)
    dy = 2.0 * w * ev / p / N
    gr = lp.backward(th, cache, dy)
    g = host(grad).astype(np.float64)
    k = 0
    for name, part in zip(["W1", "b1", "W2", "b2", "W3", "b3"], lp.unpack(gr)):
        e = relnorm(g[k:k + part.size], part.ravel())
        print(f"  {name}: rel {e:.2e}")
        assert e < 5e-3, name
        k += part.size
    # with lr > 0 the step is the Adam update of that gradient
    before = m.get().astype(np.float64)
    m.fit_step(Xd, Rd, 1e-3)
    step = m.get().astype(np.float64) - before
    big = np.abs(g) > 1e-4
    assert np.allclose(step[big], -1e-3 * np.sign(g[big]), rtol=1e-3, atol=1e-7)
    m.close()


def test_learned_vcycle_matches_oracle(lib):
    from paper_2006_07859_amd import (RC_C_BARYCENTER, RC_C_EDGE_LENGTH, RC_F32, RC_SOLVE_PCG_LEARNED, RC_SOLVE_PCG_MG,
                                      Context, Mlp, default_solve_opts)

    n = 2048
    banner(f"learned V-cycle PCG vs the oracle's projected gradient, n={n}")
    g, e = knot(n, 0)
    g = gen.round_to_f32(g)
    mask = cons.BARYCENTER | cons.EDGE_LENGTH
    refs = cons.reference_values(g, e)
    _, dE = tpe.differential(g, e, ALPHA, BETA)
    A = sum(sobolev.assemble(g, e, ALPHA, BETA))
    _, C = cons.evaluate(g, e, mask, *refs)
    g_ref, _ = solve.projected_gradient(A, C, dE)
    ctx = Context(n, e, ALPHA, BETA, RC_F32)
    ctx.rc_set_constraints(RC_C_BARYCENTER | RC_C_EDGE_LENGTH, dev(g))
    m = Mlp(lp.init_params(0))  # untrained: p ~ 2.7 everywhere
    ctx.rc_learned_attach(m)
    its = {}
    for kind in (RC_SOLVE_PCG_MG, RC_SOLVE_PCG_LEARNED):
        out = zeros(n, 3)
        so = default_solve_opts(solver=kind, tol=1e-10, mg_min_vertices=256, op_f64=1, max_iter=200, fallback_after=0)
        st = ctx.rc_sobolev_gradient(dev(g), dev(dE), out, so)
        err = relnorm(host(out), g_ref)
        its[kind] = st["iterations"]
        print(f"  solver {kind}: {st['iterations']} iterations, residual {st['residual']:.1e}, rel error {err:.1e}")
        assert err < 1e-7
    assert its[RC_SOLVE_PCG_LEARNED] <= its[RC_SOLVE_PCG_MG] + 3
    ctx.close()
    m.close()


def training_set(n_snap_per_knot=4):
    """(X, R) from snapshots of plain multigrid flows on knots of 1,024-2,048 edges."""
    import torch

    from paper_2006_07859_amd import (RC_C_BARYCENTER, RC_F32, RC_SOLVE_PCG_MG, Context, default_ls_opts,
                                      default_solve_opts)

    Xs, Rs = [], []
    for k, n in enumerate([1024, 1536, 2048] * 4):
        g, e = knot(n, 300 + k)
        ctx = Context(n, e, ALPHA, BETA, RC_F32)
        gam = dev(g)
        ctx.rc_set_constraints(RC_C_BARYCENTER, gam)
        sizes = ctx.rc_learned_levels(128)
        N = sum(sizes)
        for s in range(n_snap_per_knot):
            X = torch.zeros(N, 8, dtype=torch.float32, device="cuda")
            R = torch.zeros(N, dtype=torch.float32, device="cuda")
            ctx.rc_learned_features(gam, 128, X)
            ctx.rc_learned_targets(gam, 128, R)
            Xs.append(X[:N - sizes[-1]])  # smoothed levels only
            Rs.append(R[:N - sizes[-1]])
            if s + 1 < n_snap_per_knot:
                ctx.rc_step(gam, so=default_solve_opts(solver=RC_SOLVE_PCG_MG, tol=1e-6, mg_min_vertices=128),
                            ls=default_ls_opts())
        ctx.close()
    return torch.cat(Xs), torch.cat(Rs)


def test_learned_vcycle_wall_time(lib):
    import time

    import torch

    from paper_2006_07859_amd import (RC_C_BARYCENTER, RC_F32, RC_SOLVE_PCG_JACOBI, RC_SOLVE_PCG_LEARNED,
                                      RC_SOLVE_PCG_MG, Context, Mlp, default_solve_opts)

    banner("learned V-cycle: training on flow snapshots, held-out knots 4k-16k")
    X, R = training_set()
    N = X.shape[0]
    m = Mlp(lp.init_params(0))
    gen_t = torch.Generator(device="cuda").manual_seed(0)
    first = last = None
    for it in range(400):
        idx = torch.randint(0, N, (16384,), device="cuda", generator=gen_t)
        loss = m.fit_step(X[idx].contiguous(), R[idx].contiguous(), 3e-3)
        first = loss if first is None else first
        last = loss
    print(f"  {N} training rows, loss {first:.4f} -> {last:.4f}")
    assert last < 0.5 * first
    total = {"multigrid": 0.0, "learned": 0.0}
    for n, seed in [(4096, 401), (8192, 402), (16384, 403)]:
        g, e = knot(n, seed)
        E = torch.zeros(1, dtype=torch.float64, device="cuda")
        dE = zeros(n, 3)
        times, outs, its = {}, {}, {}
        for name, kind in (("multigrid", RC_SOLVE_PCG_MG), ("learned", RC_SOLVE_PCG_LEARNED),
                           ("jacobi", RC_SOLVE_PCG_JACOBI)):
            best = None
            for rep in range(3):  # a fresh context each time: the first solve at the curve
                ctx = Context(n, e, ALPHA, BETA, RC_F32)
                gam = dev(g)
                ctx.rc_set_constraints(RC_C_BARYCENTER, gam)
                ctx.rc_learned_attach(m)
                ctx.rc_learned_levels(256)  # hierarchy and buffers outside the timed region
                ctx.rc_differential(gam, E, dE)
                out = zeros(n, 3)
                so = default_solve_opts(solver=kind, tol=1e-6, mg_min_vertices=256, op_f64=1,
                                        max_iter=300 if kind == RC_SOLVE_PCG_JACOBI else 200, fallback_after=0)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                st = ctx.rc_sobolev_gradient(gam, dE, out, so, check=False)
                torch.cuda.synchronize()
                dt = (time.perf_counter() - t0) * 1e3
                best = dt if best is None else min(best, dt)
                ctx.close()
            times[name], outs[name], its[name] = best, out, (st["iterations"], st["status"])
        err = relnorm(host(outs["learned"]), host(outs["multigrid"]))
        print(f"  n {n}: multigrid {its['multigrid'][0]} it {times['multigrid']:.1f} ms, learned "
              f"{its['learned'][0]} it {times['learned']:.1f} ms (vs multigrid {err:.1e}), jacobi "
              f"{its['jacobi'][0]} it status {its['jacobi'][1]} {times['jacobi']:.1f} ms")
        assert its["multigrid"][1] == 0 and its["learned"][1] == 0
        assert its["jacobi"][1] != 0  # not converged within 300 iterations
        assert err < 1e-5
        for k in total:
            total[k] += times[k]
    print(f"  total: multigrid {total['multigrid']:.1f} ms, learned {total['learned']:.1f} ms")
    assert total["learned"] < total["multigrid"]
    m.close()
