"""GPU parity of the triangulated-surface potential of Sec. 7.1.

With theta = 0 (every triangle summed) the energy and differential equal the
oracle's sum over (edge midpoint, triangle centroid) samples added to the
tangent-point energy (FP64 edge-pair path, and the FP32 vertex-pair path whose
penalties are FP64); with theta > 0 the tree's far-field error is measured
against that exact sum; a step with the potential lowers the total energy, and
a Barnes-Hut step rejects it.
"""

import numpy as np
import pytest

import gen
from oracle import penalties as pen
from oracle import tpe
from tests.gpu_util import banner, dev, host, relnorm, zeros

pytestmark = pytest.mark.gpu


def setup(n=256, level=3):
    g, e = gen.trefoil(n, seed=0)
    P, F = gen.icosphere(level, radius=0.5)  # inside the trefoil (|gamma| >= 1)
    return g, e, P, F


@pytest.mark.parametrize("dtype_name", ["f64", "f32"])
def test_surface_potential_exact_tree_matches_oracle(lib, dtype_name):
    from paper_2006_07859_amd import RC_F32, RC_F64, Context

    g, e, P, F = setup()
    dtype = RC_F64 if dtype_name == "f64" else RC_F32
    if dtype == RC_F32:
        g = gen.round_to_f32(g)
    banner(f"surface potential theta=0 vs oracle, trefoil256, icosphere {len(F)} triangles, {dtype_name}")
    w = 0.7
    E_t, d_t = tpe.differential(g, e, 2.0, 4.5)
    E_m, d_m = pen.surface_potential(g, e, P, F, 2.5)
    ctx = Context(len(g), e, 2.0, 4.5, dtype)
    ctx.rc_set_surface_potential(P, F, weight=w, theta=0.0)
    E, dE = zeros(1), zeros(len(g), 3)
    ctx.rc_differential(dev(g), E, dE)
    tol_e, tol_d = (1e-12, 1e-10) if dtype == RC_F64 else (1e-5, 1e-4)
    assert host(E)[0] == pytest.approx(E_t + w * E_m, rel=tol_e)
    assert relnorm(host(dE), d_t + w * d_m) < tol_d
    # the potential alone: the same context with the energy's share removed
    ctx2 = Context(len(g), e, 2.0, 4.5, dtype)
    E2, dE2 = zeros(1), zeros(len(g), 3)
    ctx2.rc_differential(dev(g), E2, dE2)
    pot = host(E)[0] - host(E2)[0]
    assert pot == pytest.approx(w * E_m, rel=1e-9 if dtype == RC_F64 else 1e-4)
    assert relnorm(host(dE) - host(dE2), w * d_m) < (1e-10 if dtype == RC_F64 else 1e-4)
    ctx.close()
    ctx2.close()


def test_surface_potential_tree_error(lib):
    """The far-field error of the tree against the exact sum, on a 4,096-edge knot beside a
    torus of 16,384 triangles (the tube 0.15 from the knot, 23 edge lengths): a node counts as one
    sample of its area at its area-weighted centre, so the error is second order in theta (the
    first-order term vanishes about that centre) and falls about 4x when theta halves."""
    from paper_2006_07859_amd import RC_F64, Context

    g, e, _ = gen.fourier_knot(4096, seed=2)
    c = g[np.argmax(g[:, 0])] + [0.65, 0.0, 0.0]  # the tube 0.15 from the knot's outermost point
    P, F = gen.torus_mesh(128, 64, R=0.4, r=0.1, center=c)
    banner(f"surface potential tree error, fourier4096 + torus {len(F)} triangles")
    ctxn = Context(len(g), e, 2.0, 4.5, RC_F64)
    En, Dn = zeros(1), zeros(len(g), 3)
    ctxn.rc_differential(dev(g), En, Dn)
    res = {}
    for theta in (0.0, 0.125, 0.25, 0.5):
        ctx = Context(len(g), e, 2.0, 4.5, RC_F64)
        ctx.rc_set_surface_potential(P, F, weight=1.0, theta=theta)
        E, D = zeros(1), zeros(len(g), 3)
        ctx.rc_differential(dev(g), E, D)
        res[theta] = (host(E)[0] - host(En)[0], host(D) - host(Dn))
        ctx.close()
    exact, dex = res[0.0]
    errs = {}
    for theta in (0.125, 0.25, 0.5):
        errs[theta] = (abs(res[theta][0] / exact - 1), relnorm(res[theta][1], dex))
        print(f"  theta {theta}: potential rel error {errs[theta][0]:.2e}, differential {errs[theta][1]:.2e}")
    assert errs[0.25][0] < 2e-2 and errs[0.25][1] < 4e-2
    for a, b in ((0.125, 0.25), (0.25, 0.5)):
        assert errs[b][0] > 2.5 * errs[a][0] and errs[b][1] > 2.5 * errs[a][1]
    ctxn.close()


def test_step_with_surface_potential(lib):
    from paper_2006_07859_amd import (RC_C_BARYCENTER, RC_F64, RC_SOLVE_DENSE, Context, RcError, default_ls_opts,
                                      default_solve_opts)

    g, e, P, F = setup(n=128, level=2)
    banner("step with the surface potential (dense solver)")
    w = 0.5
    E0 = tpe.energy(g, e, 2.0, 4.5) + w * pen.surface_potential(g, e, P, F, 2.5)[0]
    ctx = Context(len(g), e, 2.0, 4.5, RC_F64)
    ctx.rc_set_constraints(RC_C_BARYCENTER, dev(g))
    ctx.rc_set_surface_potential(P, F, weight=w)
    gam = dev(g)
    st = ctx.rc_step(gam, so=default_solve_opts(solver=RC_SOLVE_DENSE))
    assert st["energy"] == pytest.approx(E0, rel=1e-12)
    new = host(gam)
    E1 = tpe.energy(new, e, 2.0, 4.5) + w * pen.surface_potential(new, e, P, F, 2.5)[0]
    assert st["tau"] > 0 and E1 < E0
    assert st["energy_new"] == pytest.approx(E1, rel=1e-10)
    with pytest.raises(RcError):
        ctx.rc_step(gam, so=default_solve_opts(solver=RC_SOLVE_DENSE), ls=default_ls_opts(bh_theta=0.25))
    ctx.close()
