"""Failure detection and the smallest grid, through the C ABI on the GPU.

- Eq. (10): the step record's velocity scale is max over the grid of |u1| + |u2| + |u3|,
  checked on a field where that differs from the per-component maxima and from max |u|;
  a fixed step whose CFL number exceeds 1 raises PSDNS_FLAG_CFL, one below 1 does not.
- A slot poisoned with a NaN raises PSDNS_FLAG_NONFINITE for itself only: the other
  slots of the batch are bitwise equal to a run without the poisoned slot.
- N = 8 (K = 2, the smallest grid the ABI accepts): right-hand side and steps against
  the oracle at the FP64 bar.
"""
import math

import numpy as np
import pytest

import oracle as ora
from paper_2012_04838_amd import inputs
from tests.gpu_helpers import gpu_rhs, make_plan, rel_l2, set_params, to_numpy, torch_mod

pytestmark = pytest.mark.gpu

FLAG_NONFINITE, FLAG_CFL = 1, 2


def _grid(N):
    x = 2.0 * np.pi * np.arange(N) / N
    return np.meshgrid(x, x, x, indexing="ij")  # Z, Y, X


def _correlated_field(N, c=0.5):
    """u = (sin z, cos z, c sin x): max(|u1|+|u2|+|u3|) = sqrt(2) + c."""
    Z, Y, X = _grid(N)
    return np.stack([np.fft.rfftn(f, axes=(0, 1, 2)) for f in (np.sin(Z), np.cos(Z), c * np.sin(X))])


@pytest.mark.parametrize("prec", [64, 32])
def test_step_record_velocity_scale_and_cfl_dt(prec):
    torch = torch_mod()
    N, c, C = 32, 0.5, 0.5
    st_np = _correlated_field(N, c)
    want = math.sqrt(2.0) + c
    plan = make_plan(N, 0, prec)
    set_params(plan, 0, ora.Params(nu=0.01, forcing=False))
    st, ws = plan.new_state(), plan.new_workspace()
    plan.set_state(st, st_np, 0)
    plan.step(st, ws, -C, 1)
    info = plan.read_step_info(ws)[0]
    torch.cuda.synchronize()
    tol = 1e-14 if prec == 64 else 1e-6
    assert abs(info["max_u"] - want) <= tol * want, (info["max_u"], want)
    dx = 2.0 * math.pi / N
    assert abs(info["dt"] - C * dx / info["max_u"]) <= 1e-15 * info["dt"]
    assert info["flags"] == 0


def test_fixed_step_above_cfl_one_raises_flag():
    torch = torch_mod()
    N, c = 32, 0.5
    st_np = _correlated_field(N, c)
    dx = 2.0 * math.pi / N
    dt_one = dx / (math.sqrt(2.0) + c)  # CFL = 1 exactly
    plan = make_plan(N, 0, 64, batch=2)
    for i in range(2):
        set_params(plan, i, ora.Params(nu=0.01, forcing=False))
    st, ws = plan.new_state(), plan.new_workspace()
    plan.set_state(st, st_np, 0)
    plan.set_state(st, 0.5 * st_np, 1)  # half the velocity: CFL 0.6 at the same dt
    plan.step(st, ws, 1.2 * dt_one, 1)
    info = plan.read_step_info(ws)
    torch.cuda.synchronize()
    assert info[0]["flags"] & FLAG_CFL and not info[0]["flags"] & FLAG_NONFINITE
    assert info[1]["flags"] == 0
    # the flag is sticky until the record is cleared
    plan.set_state(st, 0.5 * st_np, 0)
    plan.step(st, ws, 1.2 * dt_one, 1)
    assert plan.read_step_info(ws)[0]["flags"] & FLAG_CFL
    plan.clear_slot_info(ws, 0)
    info = plan.read_step_info(ws)
    assert info[0]["flags"] == 0 and info[0]["steps"] == 0 and info[1]["steps"] == 2
    plan.step(st, ws, 1.2 * dt_one, 1)
    assert plan.read_step_info(ws)[0]["flags"] == 0


@pytest.mark.parametrize("prec", [64, 32])
def test_poisoned_slot_leaves_other_slots_bitwise_unchanged(prec):
    torch = torch_mod()
    N, S, B = 32, 1, 3
    prm = ora.Params(nu=0.01, schmidt=(0.7,), mean_grad=((0.0, 1.0, 0.0),), power=0.1, k_force=2.0)
    ys = []
    for i in range(B):
        y = ora.init_field(N, S, 20 + i, 4.0, 1.0)
        y[3:] = inputs.random_spectral_state(N, S, 30 + i, ora.kmax_retained(N), 4.0, 0.3)
        ys.append(y)
    bad = ys[1].copy()
    bad[0, 2, 1, 3] = np.nan
    results = []
    for poisoned in (False, True):
        plan = make_plan(N, S, prec, batch=B)
        st, ws = plan.new_state(), plan.new_workspace()
        for i in range(B):
            set_params(plan, i, prm)
            plan.set_state(st, bad if (poisoned and i == 1) else ys[i], i)
        plan.step(st, ws, -0.5, 4)
        info = plan.read_step_info(ws)
        results.append(([plan.get_state(st, i).clone() for i in range(B)], info))
    torch.cuda.synchronize()
    (clean, info_c), (pois, info_p) = results
    assert all(r["flags"] == 0 for r in info_c)
    assert info_p[1]["flags"] & FLAG_NONFINITE
    for i in (0, 2):
        assert info_p[i]["flags"] == 0
        assert torch.equal(pois[i], clean[i]), i
        assert info_p[i]["dt"] == info_c[i]["dt"] and info_p[i]["t"] == info_c[i]["t"]


@pytest.mark.parametrize("S", [0, 1])
def test_smallest_grid_rhs_and_steps_match_oracle(S):
    torch = torch_mod()
    N = 8
    prm = ora.Params(nu=0.02, schmidt=(0.7,)[:S], mean_grad=((0.0, 1.0, 0.0),)[:S], power=0.1, k_force=2.0)
    x = inputs.random_spectral_state(N, 3 + S, 50 + S, ora.kmax_retained(N), 10.0)
    # velocity solenoidal (the oracle projects the right-hand side, not the input)
    x[:3] = ora.project(x[:3])
    ref = ora.rhs(x, prm)
    got = gpu_rhs(x, prm, 64)
    assert rel_l2(got, ref) < 1e-12, rel_l2(got, ref)
    dt = ora.cfl_dt(x, 0.5)
    plan = make_plan(N, S, 64)
    set_params(plan, 0, prm)
    st, ws = plan.new_state(), plan.new_workspace()
    plan.set_state(st, x, 0)
    plan.step(st, ws, -0.5, 5)
    got = to_numpy(plan.get_state(st, 0))
    info = plan.read_step_info(ws)[0]
    torch.cuda.synchronize()
    ref, dts = ora.step(x, prm, nsteps=5, cfl=0.5, return_dts=True)
    assert abs(dts[0] - dt) < 1e-15 * dt
    assert rel_l2(got, ref) < 1e-12, rel_l2(got, ref)
    assert abs(info["t"] - sum(dts)) < 1e-13 * sum(dts)
