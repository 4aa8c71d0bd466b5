"""GPU parity of the Sec. 7.1 penalties (total length, length difference,
constant-field potential) against oracle/penalties.py, added to the
tangent-point energy and differential: FP64 on a loop plus an open path,
FP32 through the vertex-pair path (alpha = 2 loop), and inside rc_step."""

import numpy as np
import pytest

import gen
from oracle import penalties as pen
from oracle import tpe
from tests.gpu_util import banner, dev, host, relnorm, zeros

pytestmark = pytest.mark.gpu

W = dict(w_length=0.7, w_diff=1.3, w_field=0.9)
X = (0.3, -0.4, 0.85)


def network():
    g1, e1, _ = gen.fourier_knot(300, seed=21)
    t = np.linspace(0.0, 1.0, 81)
    g2 = np.stack([0.5 * np.cos(5 * t) + 4.0, 0.5 * np.sin(5 * t), 1.5 * t * t], 1)
    e2 = np.stack([np.arange(80), np.arange(1, 81)], 1) + 300
    return np.concatenate([g1, g2]), np.concatenate([e1, e2]).astype(np.int32)


def oracle(g, e, a, b):
    E, dE = tpe.differential(g, e, a, b)
    Ep, dp = pen.penalties(g, e, W["w_length"], W["w_diff"], W["w_field"], X)
    return E + Ep, dE + dp, Ep


@pytest.mark.parametrize("a,b", [(2.0, 4.5), (3.0, 6.0)])
def test_penalties_fp64(lib, a, b):
    import torch

    from paper_2006_07859_amd import RC_F64, Context

    banner(f"penalties FP64 ({a},{b})")
    g, e = network()
    E_ref, dE_ref, Ep = oracle(g, e, a, b)
    ctx = Context(len(g), e, a, b, RC_F64)
    ctx.rc_set_penalties(W["w_length"], W["w_diff"], W["w_field"], X)
    E = torch.zeros(1, dtype=torch.float64, device="cuda")
    dE = zeros(len(g), 3)
    ctx.rc_differential(dev(g), E, dE)
    print(f"  E {E.item():.12g} (penalties {Ep:.6g}); rel {abs(E.item() - E_ref) / E_ref:.1e}, "
          f"dE rel {relnorm(host(dE), dE_ref):.1e}")
    assert E.item() == pytest.approx(E_ref, rel=1e-12)
    assert relnorm(host(dE), dE_ref) < 1e-10
    E2 = torch.zeros(1, dtype=torch.float64, device="cuda")
    ctx.rc_energy(dev(g), E2)
    assert E2.item() == pytest.approx(E_ref, rel=1e-12)
    # removing them restores the plain energy
    ctx.rc_set_penalties(0.0, 0.0, 0.0)
    ctx.rc_energy(dev(g), E2)
    assert E2.item() == pytest.approx(E_ref - Ep, rel=1e-12)
    ctx.close()


def test_penalties_fp32_vertex_pairs(lib):
    import torch

    from paper_2006_07859_amd import RC_F32, Context

    n = 1000
    banner(f"penalties FP32 vertex-pair path, loop of {n}")
    g, e, _ = gen.fourier_knot(n, seed=22)
    g = gen.round_to_f32(g)
    E_ref, dE_ref, _ = oracle(g, e, 2.0, 4.5)
    ctx = Context(n, e, 2.0, 4.5, RC_F32)
    ctx.rc_set_penalties(W["w_length"], W["w_diff"], W["w_field"], X)
    E = torch.zeros(1, dtype=torch.float64, device="cuda")
    dE = zeros(n, 3)
    ctx.rc_differential(dev(g), E, dE)
    print(f"  E rel {abs(E.item() - E_ref) / E_ref:.1e}, dE rel {relnorm(host(dE), dE_ref):.1e}")
    assert E.item() == pytest.approx(E_ref, rel=1e-5)
    assert relnorm(host(dE), dE_ref) < 1e-4
    ctx.close()


def test_step_with_penalties(lib):
    import torch

    from paper_2006_07859_amd import (RC_C_BARYCENTER, RC_F64, RC_SOLVE_DENSE, Context, RcError, default_ls_opts,
                                      default_solve_opts)

    banner("rc_step with penalties")
    g, e, _ = gen.fourier_knot(200, seed=23)
    ctx = Context(len(g), e, 2.0, 4.5, RC_F64)
    gam = dev(g)
    ctx.rc_set_constraints(RC_C_BARYCENTER, gam)
    ctx.rc_set_penalties(W["w_length"], W["w_diff"], W["w_field"], X)
    E0 = oracle(g, e, 2.0, 4.5)[0]
    st = ctx.rc_step(gam, so=default_solve_opts(solver=RC_SOLVE_DENSE), ls=default_ls_opts())
    assert st["energy"] == pytest.approx(E0, rel=1e-12)
    E1 = oracle(host(gam), e, 2.0, 4.5)[0]
    assert st["energy_new"] == pytest.approx(E1, rel=1e-12)
    assert E1 < E0
    with pytest.raises(RcError):
        ctx.rc_step(gam, so=default_solve_opts(solver=RC_SOLVE_DENSE), ls=default_ls_opts(bh_theta=0.25))
    ctx.close()
