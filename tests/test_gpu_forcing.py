"""The paper's deterministic band-energy-hold forcing (applied after the last stage) on
the GPU against the oracle, plus its exact invariants: the band energy after every step
is the target, and a Beltrami flow inside the band is stationary."""
import numpy as np
import pytest

import oracle as ora
from tests.gpu_helpers import make_plan, rel_l2, set_params, to_numpy, torch_mod

pytestmark = pytest.mark.gpu


def _hold_params(S, target, nu=0.01):
    return ora.Params(nu=nu, schmidt=(1.0, 0.7)[:S], mean_grad=((0.0, 1.0, 0.0),) * S, k_force=2.0,
                      forcing_mode="hold", hold_energy=target)


@pytest.mark.parametrize("N,S,prec,graph", [(32, 1, 64, False), (64, 2, 64, True), (32, 1, 32, False)])
def test_hold_forcing_steps_match_oracle(N, S, prec, graph):
    torch = torch_mod()
    y0 = ora.init_field(N, S, 8, 4.0, 1.0)
    target = 1.1 * ora.band_energy(y0[:3], 2.0)
    prm = _hold_params(S, target)
    dt, steps = 0.004, 5
    ref = ora.step(y0, prm, dt, steps)
    plan = make_plan(N, S, prec)
    set_params(plan, 0, prm)
    st, ws = plan.new_state(), plan.new_workspace()
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        plan.set_graph(graph)
        plan.set_state(st, y0, 0)
        plan.step(st, ws, dt, 2)
        plan.step(st, ws, dt, steps - 2)
        got = to_numpy(plan.get_state(st, 0))
    stream.synchronize()
    err = rel_l2(got, ref)
    assert err < (1e-12 if prec == 64 else 1e-5), err
    assert abs(ora.band_energy(got[:3], 2.0) - target) <= (1e-14 if prec == 64 else 1e-6) * target


def test_hold_forcing_keeps_beltrami_flow_stationary_on_gpu():
    torch = torch_mod()
    N, k0 = 32, 2
    x = 2.0 * np.pi * np.arange(N) / N
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    u = [np.sin(k0 * Z) + 0.4 * np.cos(k0 * Y), 0.7 * np.sin(k0 * X) + np.cos(k0 * Z),
         0.4 * np.sin(k0 * Y) + 0.7 * np.cos(k0 * X)]
    st0 = np.stack([ora.to_spectral(f) for f in u])
    prm = ora.Params(nu=0.05, k_force=2.0, forcing_mode="hold", hold_energy=ora.band_energy(st0, 2.0))
    plan = make_plan(N, 0, 64)
    set_params(plan, 0, prm)
    st, ws = plan.new_state(), plan.new_workspace()
    plan.set_state(st, st0, 0)
    plan.step(st, ws, 0.02, 6)
    got = to_numpy(plan.get_state(st, 0))
    torch.cuda.synchronize()
    assert np.max(np.abs(got - st0)) <= 1e-13 * np.max(np.abs(st0))


def test_mixed_forcing_modes_in_one_batch():
    """Slot 0 constant power, slot 1 hold: each matches its own oracle run."""
    torch = torch_mod()
    N, S, dt, steps = 32, 1, 0.004, 3
    a = ora.init_field(N, S, 21, 4.0, 1.0)
    b = ora.init_field(N, S, 22, 4.0, 1.0)
    pa = ora.Params(nu=0.01, schmidt=(1.0,), mean_grad=((0.0, 1.0, 0.0),), power=0.1, k_force=2.0)
    pb = _hold_params(S, 0.9 * ora.band_energy(b[:3], 2.0))
    plan = make_plan(N, S, 64, batch=2)
    set_params(plan, 0, pa)
    set_params(plan, 1, pb)
    st, ws = plan.new_state(), plan.new_workspace()
    plan.set_state(st, a, 0)
    plan.set_state(st, b, 1)
    plan.step(st, ws, dt, steps)
    ga, gb = to_numpy(plan.get_state(st, 0)), to_numpy(plan.get_state(st, 1))
    torch.cuda.synchronize()
    assert rel_l2(ga, ora.step(a, pa, dt, steps)) < 1e-12
    assert rel_l2(gb, ora.step(b, pb, dt, steps)) < 1e-12
