"""GPU parity of the learned multilevel preconditioner against oracle/learned.py.

* MLP forward (FP16 weights and first hidden layer, FP32 accumulation)
  against the FP64 oracle run on the same FP16-rounded weights and inputs,
  within a first-order bound of the hidden layer's FP16 rounding.
* MLP backward against the oracle's gradient, Adam against its update.
* Level sizes, FP64 level diagonals and the features of every level.
* The multilevel application P (sum_l P_l D_l P_l^T) P against the oracle's,
  exactly up to rounding order, with hand-weighted and learned scalings.
* One training sample: loss and parameter gradient against the oracle's
  loss_and_grad; a short training run lowers the loss; PCG with either
  preconditioner reaches the oracle's projected gradient.
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


def oracle_projector(g, e):
    x0, _, _ = cons.reference_values(g, e)
    _, C = cons.evaluate(g, e, cons.BARYCENTER, x0)
    return np.eye(C.shape[1]) - C.T @ np.linalg.solve(C @ C.T, C), C


@pytest.mark.parametrize("learned", [False, True])
def test_multilevel_apply(lib, learned):
    import torch

    from paper_2006_07859_amd import Mlp

    n, n_min = 1000, 64
    banner(f"multilevel apply n={n} learned={learned}")
    g, e = knot(n, 4)
    ctx = context(g, e)
    m = None
    if learned:
        m = Mlp(perturbed_params(3))
        ctx.rc_learned_attach(m)
    sizes = ctx.rc_learned_levels(n_min)
    N = sum(sizes)
    scal = zeros(N)
    ctx.rc_learned_scalings(dev(g), n_min, scal)
    s = host(scal)
    gammas, Js = lp.hierarchy(g, n_min)
    diags = np.concatenate(lp.level_diagonals(gammas, ALPHA, BETA))
    if learned:
        # y = s diag from the network on the device features, within the forward bound
        X = torch.zeros(N, 8, dtype=torch.float32, device="cuda")
        ctx.rc_learned_features(dev(g), n_min, X)
        Xh = host(X).astype(np.float16).astype(np.float64)
        th = theta16(perturbed_params(3))
        yr, _ = lp.forward(th, Xh)
        assert np.all(np.abs(s * diags - yr) <= forward_bound(th, Xh) + 1e-9 * yr)
    else:
        assert np.abs(s * diags - 1).max() < 1e-10
    P, _ = oracle_projector(g, e)
    r = np.random.default_rng(7).normal(size=(n, 3))
    Y = zeros(n, 3)
    ctx.rc_learned_apply(dev(g), n_min, dev(r), Y)
    scal_l = np.split(s, np.cumsum(sizes)[:-1])
    Pr = (P @ r.ravel()).reshape(-1, 3)
    ref = (P @ lp.apply_multilevel(Js, scal_l, Pr).ravel()).reshape(-1, 3)
    assert relnorm(host(Y), ref) < 1e-12
    # symmetric positive definite on range(P)
    q = np.random.default_rng(8).normal(size=(n, 3))
    Yq = zeros(n, 3)
    ctx.rc_learned_apply(dev(g), n_min, dev(q), Yq)
    a, b = (q * host(Y)).sum(), (r * host(Yq)).sum()
    assert a == pytest.approx(b, rel=1e-11)
    assert (r * host(Y)).sum() > 0
    ctx.close()
    if m:
        m.close()


def gradient_problem(g, e):
    A = sum(sobolev.assemble(g, e, ALPHA, BETA))
    _, dE = tpe.differential(g, e, ALPHA, BETA)
    _, C = oracle_projector(g, e)
    g_ref, _ = solve.projected_gradient(A, C, dE)
    return A, C, dE, g_ref


def test_train_step_loss_and_gradient(lib):
    import torch

    from paper_2006_07859_amd import Mlp

    n, n_min = 512, 32
    banner(f"learned train step n={n}")
    g, e = knot(n, 5)
    A, C, dE, g_ref = gradient_problem(g, e)
    theta = perturbed_params(4, 0.05)
    ctx = context(g, e)
    m = Mlp(theta)
    ctx.rc_learned_attach(m)
    grad = torch.zeros(lp.n_params(), dtype=torch.float32, device="cuda")
    loss = ctx.rc_learned_train_step(dev(g), dev(dE), dev(g_ref), n_min, 0.0, grad)
    Lr, Gr = lp.loss_and_grad(theta16(theta), g, dE, g_ref, A, C, ALPHA, BETA, n_min=n_min)
    print(f"  loss {loss:.6f} oracle {Lr:.6f}, grad rel {relnorm(host(grad), Gr):.2e}")
    assert loss == pytest.approx(Lr, rel=2e-3)
    # FP16 hidden layers: the smooth error is ~1e-3, ReLU units near zero add a few 1e-3
    assert relnorm(host(grad), Gr) < 3e-2
    # lr = 0 leaves the parameters alone
    assert np.array_equal(m.get(), theta.astype(np.float32))
    ctx.close()
    m.close()


def test_training_lowers_loss_and_pcg_converges(lib):
    from paper_2006_07859_amd import (RC_SOLVE_PCG_LEARNED, RC_SOLVE_PCG_MULTILEVEL, Mlp,
                                      default_solve_opts)

    n, n_min = 512, 32
    banner("learned preconditioner: 120 training steps on 3 curves, then PCG")
    probs = []
    for seed in (10, 11, 12):
        g, e = knot(n, seed)
        probs.append((g, e) + gradient_problem(g, e))
    m = Mlp(lp.init_params(0))
    ctxs = []
    for g, e, *_ in probs:
        c = context(g, e)
        c.rc_learned_attach(m)
        ctxs.append(c)
    first, last = [], []
    for it in range(120):
        k = it % 3
        g, e, A, C, dE, g_ref = probs[k]
        L = ctxs[k].rc_learned_train_step(dev(g), dev(dE), dev(g_ref), n_min, 3e-3)
        if it < 3:
            first.append(L)
        elif it >= 117:
            last.append(L)
    print(f"  loss first pass {np.round(first, 4).tolist()} last pass {np.round(last, 4).tolist()}")
    assert np.mean(last) < 0.8 * np.mean(first)
    for kind in (RC_SOLVE_PCG_MULTILEVEL, RC_SOLVE_PCG_LEARNED):
        for (g, e, A, C, dE, g_ref), c in zip(probs, ctxs):
            out = zeros(n, 3)
            st = c.rc_sobolev_gradient(dev(g), dev(dE), out,
                                       default_solve_opts(solver=kind, tol=1e-9, max_iter=2000, mg_min_vertices=n_min,
                                                          fallback_after=0))
            assert st["fallback"] == 0
            Ab = np.kron(A, np.eye(3))
            err = host(out).ravel() - g_ref.ravel()
            aerr = np.sqrt(err @ Ab @ err / (g_ref.ravel() @ Ab @ g_ref.ravel()))
            print(f"  kind {kind}: iterations {st['iterations']} A-norm error {aerr:.1e}")
            assert aerr < 1e-6
    for c in ctxs:
        c.close()
    m.close()


def test_fallback_to_multigrid(lib):
    """A multilevel solve that runs out of iterations is redone with multigrid
    (forced from the host with a small iteration cap)."""
    from paper_2006_07859_amd import RC_SOLVE_PCG_MULTILEVEL, RcError, default_solve_opts

    n, n_min = 512, 32
    banner("multilevel PCG falls back to multigrid")
    g, e = knot(n, 21)
    A, C, dE, g_ref = gradient_problem(g, e)
    ctx = context(g, e)
    out = zeros(n, 3)
    so = default_solve_opts(solver=RC_SOLVE_PCG_MULTILEVEL, tol=1e-8, max_iter=30, mg_min_vertices=n_min)
    assert so.fallback_after == 10
    st = ctx.rc_sobolev_gradient(dev(g), dev(dE), out, so)
    print(f"  iterations {st['iterations']} fallback {st['fallback']}")
    assert st["fallback"] == 1 and st["iterations"] > 30 and st["residual"] < 1e-8
    Ab = np.kron(A, np.eye(3))
    err = host(out).ravel() - g_ref.ravel()
    assert np.sqrt(err @ Ab @ err / (g_ref.ravel() @ Ab @ g_ref.ravel())) < 1e-5
    so.fallback_after = 0
    with pytest.raises(RcError):
        ctx.rc_sobolev_gradient(dev(g), dev(dE), out, so)
    st = ctx.rc_sobolev_gradient(dev(g), dev(dE), out, so, check=False)
    assert st["status"] == 5 and st["fallback"] == 0 and st["iterations"] == 30
    ctx.close()


def test_rejects_unsupported_curves(lib):
    from paper_2006_07859_amd import RC_F32, Context, RcError

    banner("learned preconditioner argument checks")
    g, e = knot(200, 1)
    ctx = Context(len(g), e[::-1].copy(), ALPHA, BETA, RC_F32)  # edges not numbered along the loop
    with pytest.raises(RcError):
        ctx.rc_learned_levels(32)
    ctx.close()
    ctx = context(g, e)
    with pytest.raises(RcError):  # learned scalings need an attached MLP in the solver
        from paper_2006_07859_amd import RC_SOLVE_PCG_LEARNED, default_solve_opts

        ctx.rc_sobolev_gradient(dev(g), dev(g), zeros(200, 3), default_solve_opts(solver=RC_SOLVE_PCG_LEARNED))
    ctx.close()
