"""The paper's explicit-viscous RK4 (viscous and diffusive terms evaluated in every stage)
on the GPU against the oracle, alone and combined with the band-energy-hold forcing
(the paper's own scheme), and its closed form on a Beltrami flow."""
import numpy as np
import pytest

import oracle as ora
from tests.gpu_helpers import make_plan, rel_l2, set_params, to_numpy, torch_mod

pytestmark = pytest.mark.gpu


def _run(y0, prm, prec, dt, steps, graph=False, split=2):
    torch = torch_mod()
    N = y0.shape[-3]
    S = y0.shape[0] - 3
    plan = make_plan(N, S, prec)
    set_params(plan, 0, prm)
    st, ws = plan.new_state(), plan.new_workspace()
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        plan.set_graph(graph)
        plan.set_state(st, y0, 0)
        plan.step(st, ws, dt, split)
        plan.step(st, ws, dt, steps - split)
        got = to_numpy(plan.get_state(st, 0))
    stream.synchronize()
    return got


@pytest.mark.parametrize("N,S,prec,graph", [(32, 1, 64, False), (64, 2, 64, True), (64, 1, 32, False)])
def test_explicit_rk4_steps_match_oracle(N, S, prec, graph):
    y0 = ora.init_field(N, S, 12, 4.0, 1.0)
    prm = ora.Params(nu=0.01, schmidt=(1.0, 0.7)[:S], mean_grad=((0.0, 1.0, 0.0),) * S, power=0.1, k_force=2.0,
                     integrator="explicit")
    dt, steps = 0.004, 5
    got = _run(y0, prm, prec, dt, steps, graph)
    err = rel_l2(got, ora.step(y0, prm, dt, steps))
    assert err < (1e-12 if prec == 64 else 1e-5), err


def test_explicit_rk4_with_hold_forcing_and_cfl_matches_oracle():
    """The paper's scheme: explicit RK4, band energy held after the last stage, dt from
    Eq. (10) every step."""
    torch = torch_mod()
    N, S, steps = 32, 1, 4
    y0 = ora.init_field(N, S, 13, 4.0, 1.0)
    prm = ora.Params(nu=0.01, schmidt=(1.0,), mean_grad=((0.0, 1.0, 0.0),), k_force=2.0, forcing_mode="hold",
                     hold_energy=ora.band_energy(y0[:3], 2.0), integrator="explicit")
    ref = ora.step(y0, prm, None, steps, cfl=0.5)
    plan = make_plan(N, S, 64)
    set_params(plan, 0, prm)
    st, ws = plan.new_state(), plan.new_workspace()
    plan.set_state(st, y0, 0)
    plan.step(st, ws, -0.5, steps)
    got = to_numpy(plan.get_state(st, 0))
    torch.cuda.synchronize()
    assert rel_l2(got, ref) < 1e-12


def test_explicit_rk4_beltrami_follows_rk4_polynomial_on_gpu():
    N, k0, nu, h, n = 32, 3, 0.05, 0.07, 6
    x = 2.0 * np.pi * np.arange(N) / N
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    u = [np.sin(k0 * Z) + 0.4 * np.cos(k0 * Y), 0.7 * np.sin(k0 * X) + np.cos(k0 * Z),
         0.4 * np.sin(k0 * Y) + 0.7 * np.cos(k0 * X)]
    st0 = np.stack([ora.to_spectral(f) for f in u])
    prm = ora.Params(nu=nu, forcing=False, integrator="explicit")
    got = _run(st0, prm, 64, h, n)
    z = -nu * k0 * k0 * h
    amp = 1.0 + z + z * z / 2 + z ** 3 / 6 + z ** 4 / 24
    assert np.max(np.abs(got - st0 * amp ** n)) <= 1e-13 * np.max(np.abs(st0))
