"""Stochastic band forcing (Ornstein-Uhlenbeck vector per band mode, the option of Sec. 2.3
after Eswaran & Pope) against the oracle drawing the same SplitMix64/Box-Muller normals.

The process starts at b = 0 when the workspace records are cleared, and every step draws
with its own dt, so the GPU runs one call from a fresh workspace and the oracle one call
from a fresh process.  CFL stepping makes the draws depend on the step size the GPU
computes itself.

Alvelius-type forcing (the other stochastic option of Sec. 2.3): a force drawn afresh each
step from y_n, normal to k, doing no work on the velocity of its step, with the power the
force-force term injects set to P; the GPU against the oracle drawing the same SplitMix64
angles, alone, with the paper's explicit RK4, in FP32, and beside other forcing modes in
one batch under graph replay.
"""
import numpy as np
import pytest

import oracle as ora
from paper_2012_04838_amd import psdns
from tests.gpu_helpers import make_plan, rel_l2, set_params, to_numpy, torch_mod

pytestmark = pytest.mark.gpu


def _prm(S, seed=17, sigma=0.4, tl=0.3, integrator="if"):
    return ora.Params(nu=0.02, schmidt=(1.0,) * S, mean_grad=((0.0, 1.0, 0.0),) * S, k_force=2.0,
                      forcing_mode="stochastic", stoch_sigma=sigma, stoch_tl=tl, stoch_seed=seed,
                      integrator=integrator)


@pytest.mark.parametrize("N,S,prec,integrator", [(32, 1, 64, "if"), (16, 0, 64, "if"), (32, 1, 64, "explicit"),
                                                 (32, 1, 32, "if")])
def test_stochastic_steps_match_oracle(N, S, prec, integrator):
    torch = torch_mod()
    prm = _prm(S, integrator=integrator)
    y0 = ora.init_field(N, S, 5, 3.0, 0.5)
    plan = make_plan(N, S, prec)
    set_params(plan, 0, prm)
    st, ws = plan.new_state(), plan.new_workspace()
    plan.set_state(st, y0, 0)
    steps = 4
    cfl = 0.5 if integrator == "if" else 0.2
    plan.step(st, ws, -cfl, steps)
    got = to_numpy(plan.get_state(st, 0))
    torch.cuda.synchronize()
    stoch = {"b": {}, "n": 0}
    ref = ora.step(y0, prm, None, steps, cfl=cfl, stoch_state=stoch)
    err = rel_l2(got, ref)
    # the forcing itself must matter at this size: the unforced run differs by far more
    ref0 = ora.step(y0, ora.Params(nu=prm.nu, schmidt=prm.schmidt, mean_grad=prm.mean_grad, forcing=False,
                                   integrator=integrator), None, steps, cfl=cfl)
    print(f"N={N} S={S} fp{prec} {integrator}: rel L2 {err:.2e} (forcing changes the field by "
          f"{rel_l2(ref0, ref):.2e})", flush=True)
    assert rel_l2(ref0, ref) > 1e-4
    assert err < (1e-12 if prec == 64 else 1e-5)
    assert plan.read_step_info(ws)[0]["steps"] == steps


def test_stochastic_process_continues_across_calls_and_restarts_on_clear():
    """Two calls continue one process (counter and b carried in the workspace); clearing the
    step records starts a fresh one."""
    torch = torch_mod()
    N, S, dt = 16, 1, 0.01
    prm = _prm(S, seed=3)
    y0 = ora.init_field(N, S, 8, 3.0, 0.5)
    plan = make_plan(N, S, 64)
    set_params(plan, 0, prm)
    st, ws = plan.new_state(), plan.new_workspace()
    plan.set_state(st, y0, 0)
    plan.step(st, ws, dt, 2)
    plan.step(st, ws, dt, 3)
    got = to_numpy(plan.get_state(st, 0))
    stoch = {"b": {}, "n": 0}
    ref = ora.step(y0, prm, dt, 2, stoch_state=stoch)
    ref = ora.step(ref, prm, dt, 3, stoch_state=stoch)
    assert rel_l2(got, ref) < 1e-12
    plan.clear_step_info(ws)
    plan.set_state(st, y0, 0)
    plan.step(st, ws, dt, 2)
    got2 = to_numpy(plan.get_state(st, 0))
    torch.cuda.synchronize()
    assert rel_l2(got2, ora.step(y0, prm, dt, 2)) < 1e-12


def test_stochastic_and_power_slots_in_one_batch_and_graph():
    """A stochastic slot beside a constant-power slot, stepped eagerly and by graph replay on
    a stream: each slot equals its oracle run."""
    torch = torch_mod()
    N, S, dt = 16, 1, 0.01
    ps = _prm(S, seed=11)
    pp = ora.Params(nu=0.02, schmidt=(1.0,), mean_grad=((0.0, 1.0, 0.0),), power=0.1, k_force=2.0)
    y0 = ora.init_field(N, S, 2, 3.0, 0.5)
    y1 = ora.init_field(N, S, 3, 3.0, 0.5)
    ref0 = ora.step(y0, ps, dt, 4)
    ref1 = ora.step(y1, pp, dt, 4)
    for graph in (False, True):
        plan = make_plan(N, S, 64, batch=2)
        set_params(plan, 0, ps)
        set_params(plan, 1, pp)
        st, ws = plan.new_state(), plan.new_workspace()
        stream = torch.cuda.Stream()
        with torch.cuda.stream(stream):
            plan.set_graph(graph)
            plan.set_state(st, y0, 0)
            plan.set_state(st, y1, 1)
            plan.step(st, ws, dt, 1)
            plan.step(st, ws, dt, 3)
            g0, g1 = to_numpy(plan.get_state(st, 0)), to_numpy(plan.get_state(st, 1))
        stream.synchronize()
        assert rel_l2(g0, ref0) < 1e-12, (graph, rel_l2(g0, ref0))
        assert rel_l2(g1, ref1) < 1e-12, (graph, rel_l2(g1, ref1))


def test_stochastic_parameters_are_validated():
    torch_mod()
    plan = make_plan(16, 0, 64)
    with pytest.raises(RuntimeError):
        plan.set_slot(0, nu=0.01, k_force=2.0, forcing=psdns.FORCING_STOCHASTIC, stoch_sigma=0.1, stoch_tl=0.0)
    with pytest.raises(RuntimeError):
        plan.set_slot(0, nu=0.01, k_force=5.0, forcing=psdns.FORCING_STOCHASTIC, stoch_sigma=0.1, stoch_tl=1.0)
    with pytest.raises(RuntimeError):
        plan.set_slot(0, nu=0.01, k_force=2.0, forcing=psdns.FORCING_STOCHASTIC, stoch_sigma=-1.0, stoch_tl=1.0)
    plan.set_slot(0, nu=0.01, k_force=4.5, forcing=psdns.FORCING_STOCHASTIC, stoch_sigma=0.1, stoch_tl=1.0)


def _alv(S, seed=23, power=0.2, integrator="if", k_force=2.0):
    return ora.Params(nu=0.02, schmidt=(1.0, 0.7)[:S], mean_grad=((0.0, 1.0, 0.0),) * S, k_force=k_force,
                      forcing_mode="alvelius", power=power, stoch_seed=seed, integrator=integrator)


@pytest.mark.parametrize("N,S,prec,integrator,kf", [(32, 1, 64, "if", 2.0), (16, 0, 64, "if", 2.0),
                                                    (32, 1, 64, "explicit", 2.0), (32, 1, 32, "if", 2.0),
                                                    (64, 2, 64, "if", 3.5)])
def test_alvelius_steps_match_oracle(N, S, prec, integrator, kf):
    torch = torch_mod()
    prm = _alv(S, integrator=integrator, k_force=kf)
    y0 = ora.init_field(N, S, 6, 3.0, 0.5)
    plan = make_plan(N, S, prec)
    set_params(plan, 0, prm)
    st, ws = plan.new_state(), plan.new_workspace()
    plan.set_state(st, y0, 0)
    steps = 4
    cfl = 0.5 if integrator == "if" else 0.2
    plan.step(st, ws, -cfl, steps)
    got = to_numpy(plan.get_state(st, 0))
    torch.cuda.synchronize()
    ref = ora.step(y0, prm, None, steps, cfl=cfl, stoch_state={"b": {}, "n": 0})
    err = rel_l2(got, ref)
    ref0 = ora.step(y0, ora.Params(nu=prm.nu, schmidt=prm.schmidt, mean_grad=prm.mean_grad, forcing=False,
                                   integrator=integrator), None, steps, cfl=cfl)
    print(f"Alvelius N={N} S={S} fp{prec} {integrator} k_F={kf}: rel L2 {err:.2e} (forcing changes the field "
          f"by {rel_l2(ref0, ref):.2e})", flush=True)
    assert rel_l2(ref0, ref) > 1e-4
    assert err < (1e-12 if prec == 64 else 1e-5)
    assert plan.read_step_info(ws)[0]["steps"] == steps


def test_alvelius_beside_other_forcing_modes_in_one_batch_and_graph():
    """Slots with Alvelius, Ornstein-Uhlenbeck and constant-power forcing in one batch, two
    calls stepped by graph replay on a stream: each slot equals its own oracle run, and
    clearing one slot's record restarts only that slot's draws."""
    torch = torch_mod()
    N, S, dt = 32, 1, 0.006
    prms = [_alv(S, seed=4), _prm(S, seed=5),
            ora.Params(nu=0.02, schmidt=(1.0,), mean_grad=((0.0, 1.0, 0.0),), power=0.1, k_force=2.0)]
    ys = [ora.init_field(N, S, 30 + i, 3.0, 0.5) for i in range(3)]
    plan = make_plan(N, S, 64, batch=3)
    st, ws = plan.new_state(), plan.new_workspace()
    for i in range(3):
        set_params(plan, i, prms[i])
        plan.set_state(st, ys[i], i)
    stream = torch.cuda.Stream()
    plan.set_graph(True)
    with torch.cuda.stream(stream):
        plan.step(st, ws, dt, 2)
        torch.cuda.synchronize()
        plan.step(st, ws, dt, 3)
    stream.synchronize()
    for i in range(3):
        ref = ora.step(ys[i], prms[i], dt, 5, stoch_state={"b": {}, "n": 0})
        got = to_numpy(plan.get_state(st, i))
        assert rel_l2(got, ref) < 1e-12, (i, rel_l2(got, ref))
    # restart slot 0 alone: its draws start again at step 1, the others continue
    plan.clear_slot_info(ws, 0)
    plan.set_state(st, ys[0], 0)
    mid1 = to_numpy(plan.get_state(st, 1))
    with torch.cuda.stream(stream):
        plan.step(st, ws, dt, 2)
    stream.synchronize()
    plan.set_graph(False)
    assert rel_l2(to_numpy(plan.get_state(st, 0)), ora.step(ys[0], prms[0], dt, 2)) < 1e-12
    stoch = {"b": {}, "n": 0}
    ref1 = ora.step(ys[1], prms[1], dt, 5, stoch_state=stoch)
    assert rel_l2(mid1, ref1) < 1e-12
    ref1 = ora.step(ref1, prms[1], dt, 2, stoch_state=stoch)
    assert rel_l2(to_numpy(plan.get_state(st, 1)), ref1) < 1e-12
    info = plan.read_step_info(ws)
    assert [r["steps"] for r in info] == [2, 7, 7]
    torch.cuda.synchronize()


def test_alvelius_parameters_are_validated():
    torch_mod()
    plan = make_plan(16, 0, 64)
    with pytest.raises(psdns.PsdnsError, match="k_force"):
        plan.set_slot(0, nu=0.01, power=0.1, k_force=5.5, forcing=psdns.FORCING_ALVELIUS)
    plan.set_slot(0, nu=0.01, power=0.1, k_force=4.5, forcing=psdns.FORCING_ALVELIUS)
