"""Barnes-Hut energy and differential (App. B.1) against the FP64 oracle.

* theta -> 0 makes every cluster inadmissible, so the traversal sums every
  disjoint pair directly: it must reproduce the exact edge-midpoint sum
  (the oracle's midpoint_energy / midpoint_differential) to FP32 rounding.
* The approximation error must shrink as theta decreases.
* At theta = 0.25 the paper prints no error value, so parity beyond these
  limits is unpinned: the test bounds the measured error loosely and the
  measured values are recorded in the design notes.
* The 262,144-edge workload is checked on sampled vertices against the
  oracle's per-target midpoint sums.
"""

import numpy as np
import pytest

import gen
from oracle import tpe
from tests.gpu_util import banner, dev, host, relnorm, zeros

pytestmark = pytest.mark.gpu


def run_bh(g, e, a, b, theta, leaf=32):
    from paper_2006_07859_amd import RC_F32, Context

    ctx = Context(len(g), e, a, b, RC_F32)
    E, dE = zeros(1), zeros(len(g), 3)
    ctx.rc_bh_differential(dev(g), theta, leaf, E, dE)
    work = ctx.rc_bh_last_work()
    ctx.close()
    return host(E)[0], host(dE), work


@pytest.mark.parametrize("alpha,beta", [(2.0, 4.5), (3.0, 6.0)])
def test_bh_small_theta_is_exact_midpoint(lib, alpha, beta):
    n = 1500
    banner(f"BH theta->0 fourier{n} ({alpha},{beta})")
    g, e, _ = gen.fourier_knot(n, seed=4)
    g = gen.round_to_f32(g)
    E_ref, G_ref = tpe.midpoint_differential(g, e, alpha, beta)
    for leaf in (8, 32, 64):
        E, G, work = run_bh(g, e, alpha, beta, 1e-6, leaf)
        assert work["far"] == 0
        assert E == pytest.approx(E_ref, rel=2e-5)
        assert relnorm(G, G_ref) < 2e-4


def test_bh_error_decreases_with_theta(lib):
    n = 3000
    banner(f"BH theta sweep fourier{n}")
    g, e, _ = gen.fourier_knot(n, seed=5)
    g = gen.round_to_f32(g)
    E_ref, G_ref = tpe.midpoint_differential(g, e, 2.0, 4.5)
    errs, fars = [], []
    for theta in (0.45, 0.25, 0.1, 0.03):
        E, G, work = run_bh(g, e, 2.0, 4.5, theta)
        errs.append((abs(E - E_ref) / E_ref, relnorm(G, G_ref)))
        fars.append(work["far"])
    print("theta errors (energy, differential):", errs, "far interactions:", fars)
    assert all(f > 0 for f in fars[:2])
    assert errs[0][1] > errs[1][1] > errs[2][1] > errs[3][1]
    assert errs[1][0] < 1e-2 and errs[1][1] < 5e-2  # theta = 0.25: measured, loosely bounded


def test_bh_full_size_sampled(lib):
    n = 262144
    banner(f"BH theta=0.25 fourier{n} sampled")
    g, e, _ = gen.fourier_knot(n, seed=0)
    g = gen.round_to_f32(g)
    E, G, work = run_bh(g, e, 2.0, 4.5, 0.25)
    exact_pairs = n * (n - 3)
    # far + near interactions visited: far fewer than the exact all-pairs count
    assert work["far"] + work["near"] < 0.05 * exact_pairs
    vs = [0, 100000, 200001]
    for v in vs:
        inc = np.nonzero((e[:, 0] == v) | (e[:, 1] == v))[0]
        _, dI = tpe.midpoint_rows(g, e, 2.0, 4.5, inc)
        ref = sum(dI[k, 0 if e[I, 0] == v else 1] for k, I in enumerate(inc))
        assert np.linalg.norm(G[v] - ref) < 5e-2 * np.linalg.norm(ref)
    assert np.isfinite(E) and E > 0


def test_bh_refit(lib):
    """Re-fitting the tree of the last build to a moved curve: with theta -> 0 the re-fitted
    traversal is the exact midpoint sum at the moved curve; at theta = 0.25 its error stays
    close to that of a tree built for the moved curve; without a tree the call is refused."""
    from paper_2006_07859_amd import RC_F32, Context, RcError

    n = 3000
    banner(f"BH re-fit fourier{n}")
    g, e, _ = gen.fourier_knot(n, seed=5)
    g = gen.round_to_f32(g)
    ell = np.linalg.norm(g[e[:, 1]] - g[e[:, 0]], axis=1).mean()
    t = np.linspace(0.0, 2.0 * np.pi, n, endpoint=False)
    move = 0.5 * ell * np.stack([np.sin(3 * t), np.cos(2 * t), np.sin(5 * t + 1.0)], 1)
    g2 = gen.round_to_f32(g + move)
    E_ref, G_ref = tpe.midpoint_differential(g2, e, 2.0, 4.5)
    ctx = Context(n, e, 2.0, 4.5, RC_F32)
    E, dE = zeros(1), zeros(n, 3)
    with pytest.raises(RcError):
        ctx.rc_bh_refit_differential(dev(g2), 0.25, E, dE)
    ctx.rc_bh_differential(dev(g), 1e-6, 32, E, dE)
    ctx.rc_bh_refit_differential(dev(g2), 1e-6, E, dE)
    assert ctx.rc_bh_last_work()["far"] == 0
    assert host(E)[0] == pytest.approx(E_ref, rel=2e-5)
    assert relnorm(host(dE), G_ref) < 2e-4
    ctx.rc_bh_differential(dev(g), 0.25, 32, E, dE)
    ctx.rc_bh_refit_differential(dev(g2), 0.25, E, dE)
    err_refit = (abs(host(E)[0] - E_ref) / E_ref, relnorm(host(dE), G_ref))
    E_b, G_b, _ = run_bh(g2, e, 2.0, 4.5, 0.25)
    err_build = (abs(E_b - E_ref) / E_ref, relnorm(G_b, G_ref))
    print(f"  theta 0.25 re-fit error {err_refit}, rebuilt {err_build}")
    assert err_refit[0] < 1e-2 and err_refit[1] < 5e-2
    assert err_refit[1] < 2.0 * err_build[1] + 1e-3
    ctx.close()
