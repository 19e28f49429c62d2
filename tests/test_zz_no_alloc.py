"""The allocation-free entry point psdns_step_noalloc against psdns_step.

Called through the C ABI (ctypes binding).  Each call is compared with psdns_step on
a freshly cleared workspace from the same input: fields within the FP64 bar of 1e-12
relative L2 (FP32: 1e-5) and identical step records.  The calls run in a row on the
same static scratch, the second with a smaller plan (fewer fields, smaller grid, FP32),
the third repeating the first, so stale contents of the array never leak into a call.
"""
import ctypes

import numpy as np
import pytest

import oracle as ora
from paper_2012_04838_amd import inputs, psdns
from tests.gpu_helpers import make_plan, rel_l2, set_params, to_numpy, torch_mod

pytestmark = pytest.mark.gpu


def _case(N, S, prec, batch, dt, steps, seed, dealias="cube"):
    torch = torch_mod()
    prms = []
    for i in range(batch):
        prm = ora.Params(nu=0.01, schmidt=(0.7, 1.0)[:S], mean_grad=((0.0, 1.0, 0.0),) * S, power=0.1, k_force=2.0,
                         dealias=dealias)
        if i % 2 == 1:
            prm.forcing_mode, prm.stoch_sigma, prm.stoch_tl, prm.stoch_seed = "stochastic", 0.05, 0.4, 11 + i
        prms.append(prm)
    plan = make_plan(N, S, prec, batch, dealias=1 if dealias == "phase" else 0)
    st = plan.new_state()
    for i in range(batch):
        set_params(plan, i, prms[i])
        y = ora.init_field(N, S, seed + i, 4.0, 1.0, dealias=dealias)
        if S:
            y[3:] = (inputs.random_spectral_state(N, S, seed + 10 + i, ora.kmax_retained(N, dealias), 4.0, 0.3)
                     * ora.retained_mask(N, dealias))
        plan.set_state(st, y, i)
    st_na = st.clone()
    ws = plan.new_workspace()
    plan.step(st, ws, dt, steps)
    ref_info = plan.read_step_info(ws)
    info_dev = torch.zeros(batch * ctypes.sizeof(psdns.StepInfo), dtype=torch.uint8, device="cuda")
    plan.step_noalloc(st_na, dt, steps, info_dev)
    torch.cuda.synchronize()
    info = psdns.step_info_from_bytes(info_dev.cpu().numpy().tobytes(), batch)
    tol = 1e-12 if prec == 64 else 1e-5
    for i in range(batch):
        a, b = to_numpy(plan.get_state(st_na, i)), to_numpy(plan.get_state(st, i))
        err = rel_l2(a, b)
        print(f"N={N} S={S} fp{prec} slot {i}: rel L2 {err:.2e}, bitwise {np.array_equal(a, b)}", flush=True)
        assert err <= tol, (i, err)
        for k in ("t", "dt", "max_u", "steps", "flags", "active"):
            assert info[i][k] == ref_info[i][k], (i, k, info[i][k], ref_info[i][k])
    assert all(r["steps"] == steps and r["flags"] == 0 for r in info)
    del st, st_na, ws
    plan.close()


def test_noalloc_matches_step_on_calls_in_a_row():
    _case(64, 2, 64, 2, -0.5, 3, 3)      # CFL steps, one stochastic slot
    _case(32, 1, 32, 1, 0.004, 4, 7)     # a smaller input right after
    _case(64, 2, 64, 2, -0.5, 3, 3)      # the first again: records restart, no stale data


def test_noalloc_phase_shift_plan():
    # the paper's dealiasing: the kept unshifted products live in the scratch too
    _case(32, 1, 64, 2, -0.5, 3, 5, dealias="phase")
    _case(32, 2, 32, 1, -0.5, 2, 9, dealias="phase")


def test_noalloc_rejects_plans_beyond_the_scratch():
    torch_mod()
    plan = make_plan(256, 0, 32)
    assert plan.info.workspace_bytes > (256 << 20)
    st = plan.new_state()
    with pytest.raises(psdns.PsdnsError, match="static scratch"):
        plan.step_noalloc(st, 0.01, 1)
    plan.close()
