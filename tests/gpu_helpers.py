"""Helpers shared by the GPU tests: run the library on canonical numpy states."""
from __future__ import annotations

import numpy as np

import oracle as ora

CAPTURE_MANAGER = None  # set by conftest at session start


def progress(msg: str) -> None:
    """Print a progress line at once, past pytest's output capture, so that a long GPU
    test is visibly alive while it runs."""
    if CAPTURE_MANAGER is not None:
        with CAPTURE_MANAGER.global_and_fixture_disabled():
            print(msg, flush=True)
    else:
        print(msg, flush=True)


def torch_mod():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    return torch


def make_plan(N, S, prec, batch=1, dealias=0):
    from paper_2012_04838_amd import psdns
    return psdns.Plan(N, S, prec, batch, dealias)


def set_params(plan, slot, prm: "ora.Params", active=True):
    from paper_2012_04838_amd import psdns
    hold = prm.forcing and prm.forcing_mode == "hold"
    stoch = prm.forcing and prm.forcing_mode == "stochastic"
    alv = prm.forcing and prm.forcing_mode == "alvelius"
    mode = psdns.FORCING_HOLD if hold else (psdns.FORCING_STOCHASTIC if stoch else
                                            (psdns.FORCING_ALVELIUS if alv else psdns.FORCING_POWER))
    powered = prm.forcing and mode in (psdns.FORCING_POWER, psdns.FORCING_ALVELIUS)
    plan.set_slot(slot, nu=prm.nu, power=(prm.power if powered else 0.0),
                  k_force=prm.k_force, schmidt=list(prm.schmidt), mean_grad=[list(g) for g in prm.mean_grad],
                  active=active, forcing=mode, hold_energy=prm.hold_energy if hold else 0.0,
                  integrator=psdns.INTEGRATOR_EXPLICIT if prm.integrator == "explicit" else psdns.INTEGRATOR_IF,
                  stoch_sigma=prm.stoch_sigma if stoch else 0.0, stoch_tl=prm.stoch_tl if stoch else 1.0,
                  stoch_seed=prm.stoch_seed if (stoch or alv) else 0)


def poisoned_workspace(plan):
    """A workspace whose every byte is 0xFF (NaN in both precisions) before its records are
    cleared: a pass that reads workspace entries nobody wrote turns the result into NaN."""
    ws = plan.new_workspace()
    ws.fill_(255)
    plan.clear_step_info(ws)
    return ws


def to_numpy(t):
    return t.detach().cpu().numpy().astype(np.complex128)


def gpu_rhs(state_np, prm, prec=64):
    torch = torch_mod()
    N = state_np.shape[-3]
    S = state_np.shape[0] - 3
    plan = make_plan(N, S, prec, dealias=1 if prm.dealias == "phase" else 0)
    set_params(plan, 0, prm)
    st = plan.new_state()
    ws = poisoned_workspace(plan)
    out = plan.new_state()
    plan.set_state(st, state_np, 0)
    plan.rhs(st, out, ws)
    res = to_numpy(plan.get_state(out, 0))
    torch.cuda.synchronize()
    return res


def rel_l2(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def retained(x):
    N = x.shape[-3]
    return np.where(ora.retained_mask(N), x, 0.0)
