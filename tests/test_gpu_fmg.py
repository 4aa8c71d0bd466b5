"""The paper's standalone multigrid (RC_SOLVE_MG_FMG, App. B.3.1): full-multigrid
initialisation and V-cycles with a projected CG smoother and an A-norm
minimising coarse-correction step, no outer Krylov method.  Its projected
gradient matches the oracle's dense saddle solution (eq.
GradientSaddlePointProblem) when driven to a small residual; the cycles it
needs for the paper's working tolerance (relative residual 1e-3) are
reported; and it drives rc_step."""

import numpy as np
import pytest

import gen
from oracle import constraints as cons
from oracle import solve, sobolev, tpe
from tests.gpu_util import banner, dev, host, relnorm, zeros

pytestmark = pytest.mark.gpu


def setup(n, seed=0):
    from paper_2006_07859_amd import RC_C_BARYCENTER, RC_C_EDGE_LENGTH, RC_F32, Context

    g, e, _ = gen.fourier_knot(n, seed=seed)
    g = gen.round_to_f32(g)
    ctx = Context(n, e, 2.0, 4.5, RC_F32)
    ctx.rc_set_constraints(RC_C_BARYCENTER | RC_C_EDGE_LENGTH, dev(g))
    return g, e, ctx


def test_fmg_matches_oracle(lib):
    from paper_2006_07859_amd import RC_SOLVE_MG_FMG, default_solve_opts

    n = 2048
    banner(f"standalone multigrid (FMG + CG-smoothed V-cycles) vs the oracle, n={n}")
    g, e, ctx = setup(n)
    mask = cons.BARYCENTER | cons.EDGE_LENGTH
    refs = cons.reference_values(g, e)
    _, dE = tpe.differential(g, e, 2.0, 4.5)
    A = sum(sobolev.assemble(g, e, 2.0, 4.5))
    _, C = cons.evaluate(g, e, mask, *refs)
    g_ref, _ = solve.projected_gradient(A, C, dE)
    out = zeros(n, 3)
    st = ctx.rc_sobolev_gradient(dev(g), dev(dE), out,
                                 default_solve_opts(solver=RC_SOLVE_MG_FMG, tol=1e-8, op_f64=1, cheb_degree=6,
                                                    max_iter=400, mg_min_vertices=256))
    err = relnorm(host(out), g_ref)
    print(f"  {st['iterations']} V-cycles, residual {st['residual']:.1e}, rel error {err:.1e}")
    assert err < 1e-5
    assert np.abs(C @ host(out).ravel()).max() < 1e-9 * np.abs(host(out)).max()
    ctx.close()


@pytest.mark.parametrize("n", [2048, 8192])
def test_fmg_paper_tolerance(lib, n):
    from paper_2006_07859_amd import RC_SOLVE_MG_FMG, RC_SOLVE_PCG_MG, default_solve_opts

    banner(f"standalone multigrid at the paper's 1e-3, n={n}")
    g, e, ctx = setup(n, seed=1)
    import torch

    E = torch.zeros(1, dtype=torch.float64, device="cuda")
    dE = zeros(n, 3)
    ctx.rc_differential(dev(g), E, dE)
    ref = zeros(n, 3)
    ctx.rc_sobolev_gradient(dev(g), dE, ref, default_solve_opts(solver=RC_SOLVE_PCG_MG, tol=1e-9, op_f64=1,
                                                                mg_min_vertices=256))
    out = zeros(n, 3)
    st = ctx.rc_sobolev_gradient(dev(g), dE, out, default_solve_opts(solver=RC_SOLVE_MG_FMG, tol=1e-3, op_f64=1,
                                                                     cheb_degree=6, max_iter=100,
                                                                     mg_min_vertices=256))
    err = relnorm(host(out), host(ref))
    print(f"  {st['iterations']} V-cycles to residual {st['residual']:.1e}; rel error vs converged {err:.1e}")
    assert st["residual"] < 1e-3
    assert st["iterations"] <= 15  # 7 at 2k and 8k when last run; the paper reports about 6
    assert err < 0.05
    ctx.close()


def test_step_with_fmg(lib):
    from paper_2006_07859_amd import RC_SOLVE_MG_FMG, default_ls_opts, default_solve_opts

    banner("rc_step with the standalone multigrid")
    g, e, ctx = setup(4096, seed=2)
    gam = dev(g)
    so = default_solve_opts(solver=RC_SOLVE_MG_FMG, tol=1e-3, op_f64=1, cheb_degree=6, max_iter=100,
                            mg_min_vertices=256)
    E = []
    for k in range(3):
        st = ctx.rc_step(gam, so=so, ls=default_ls_opts())
        E.append((st["energy"], st["energy_new"]))
        print(f"  step {k}: E {st['energy']:.8g} -> {st['energy_new']:.8g}, {st['iterations']} V-cycles, "
              f"tau {st['tau']:.3g}")
        assert st["energy_new"] < st["energy"]
    ctx.close()
