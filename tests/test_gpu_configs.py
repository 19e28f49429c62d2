"""The workload configurations at their own sizes.

- 256^3 FP64, S = 1 (k_p = 6, nu = 0.0015, Sc = 1, G = (0, 1, 0), P = 0.1 on k <= 2,
  CFL 0.5): GPU against the FP64 oracle after CFL-stepped RK4 steps, fields and the
  recorded statistics (eps, Re_lambda, velocity-derivative and scalar-gradient
  skewness).
- 512^3, S = 2 (k_p = 8, nu = 7e-4, Sc 0.7 and 1.0, G = (0, 1, 0) each), with the fixed
  dt = 0.5 dx / max(|u1|+|u2|+|u3|) of the FP64 initial field:
  * FP64 and FP32 GPU runs against the FP64 oracle after 2 steps (the oracle needs
    about 70 GB of host memory and a few minutes here): FP64 fields within 1e-12
    relative L2, FP32 within 1e-5; shell spectra of both within the per-shell bars;
  * FP32 against FP64 on the GPU over 10 and 200 steps: fields within 1e-5 relative L2
    after 10 steps; shell spectra within 1e-4 relative after 10 and 200 steps where the
    FP64 shell holds at least 1e-6 of the largest shell, and within 1e-10 K elsewhere.
- 1024^3, S = 1 (nu = 3e-4, Sc = 1, G = 1, CFL 0.5): the oracle does not fit a host at
  this size, so FP32-GPU is compared with FP64-GPU (10 steps, fields within 1e-5).
States are compared in the compact layout on the device.
"""
import math

import numpy as np
import pytest

import oracle as ora
from tests.gpu_helpers import make_plan, progress, rel_l2, set_params, to_numpy, torch_mod

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


def _log(msg):
    progress(f"[configs] {msg}")


def _device_rel_l2(torch, a32, b64):
    """Relative L2 of a FP32 compact state against a FP64 one (complex views)."""
    a = torch.view_as_complex(a32.view(torch.float32).view(-1, 2)).to(torch.complex128)
    b = torch.view_as_complex(b64.view(torch.float64).view(-1, 2))
    r = float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b))
    del a
    return r


def _shells_close(e32, e64, K, rel_tol=1e-4, abs_tol=1e-10):
    """Per-shell bar: relative rel_tol where the reference shell holds at least 1e-6 of
    the largest shell, absolute abs_tol * K elsewhere (shells below round-off)."""
    e32, e64 = np.asarray(e32), np.asarray(e64)
    big = e64 >= 1e-6 * e64.max()
    rel = np.abs(e32[big] - e64[big]) / e64[big]
    assert rel.max() <= rel_tol, rel.max()
    assert np.all(np.abs(e32[~big] - e64[~big]) <= abs_tol * K)
    return float(rel.max())


def test_256_fp64_cfl_steps_and_statistics_match_oracle():
    torch = torch_mod()
    N, S, steps = 256, 1, 10
    prm = ora.Params(nu=0.0015, schmidt=(1.0,), mean_grad=((0.0, 1.0, 0.0),), power=0.1, k_force=2.0)
    _log("256^3 oracle init and steps")
    y0 = ora.init_field(N, S, 2, 6.0, 1.0)
    ref = ora.step(y0, prm, None, steps, cfl=0.5)
    plan = make_plan(N, S, 64)
    set_params(plan, 0, prm)
    st, ws = plan.new_state(), plan.new_workspace()
    plan.init_field(st, ws, 0, seed=2, k_peak=6.0, kinetic_energy=1.0)
    assert rel_l2(to_numpy(plan.get_state(st, 0)), y0) < 1e-13
    plan.step(st, ws, -0.5, steps)
    got = to_numpy(plan.get_state(st, 0))
    sp = plan.spectra(st, ws)[0]
    torch.cuda.synchronize()
    err = rel_l2(got, ref)
    _log(f"256^3 FP64 after {steps} CFL steps: rel L2 {err:.2e}")
    assert err < 1e-12
    _log("256^3 oracle statistics")
    rs = ora.spectra(ref, prm)
    ph = ora.physical_stats(ref)
    for k in ("eps", "Re_lambda"):
        assert abs(sp[k] - rs[k]) <= 1e-10 * abs(rs[k]), (k, sp[k], rs[k])
    np.testing.assert_allclose(sp["vgt_skew"], ph["vgt_skew"], rtol=1e-8)
    np.testing.assert_allclose(sp["phi2_skew"], ph["phi2_skew"], rtol=1e-8, atol=1e-12)


def _pair(N, S, prm, seed, k_peak):
    plans = {}
    for prec in (32, 64):
        plan = make_plan(N, S, prec)
        set_params(plan, 0, prm)
        st, ws = plan.new_state(), plan.new_workspace()
        plan.init_field(st, ws, 0, seed=seed, k_peak=k_peak, kinetic_energy=1.0)
        plans[prec] = (plan, st, ws)
    return plans


@pytest.mark.timeout(1200)
def test_512_fp64_and_fp32_against_oracle():
    torch = torch_mod()
    N, S, steps = 512, 2, 2
    prm = ora.Params(nu=7e-4, schmidt=(0.7, 1.0), mean_grad=((0.0, 1.0, 0.0),) * 2, power=0.1, k_force=2.0)
    _log("512^3 S=2 oracle initial field")
    ref = ora.init_field(N, S, 3, 8.0, 1.0)
    dt = ora.cfl_dt(ref, 0.5)
    for n in range(steps):
        ref = ora.step(ref, prm, dt, 1)
        _log(f"512^3 oracle step {n + 1} of {steps} done (dt {dt:.6f})")
    rs = ora.spectra(ref, prm)
    for prec in (64, 32):
        plan = make_plan(N, S, prec)
        set_params(plan, 0, prm)
        st, ws = plan.new_state(), plan.new_workspace()
        plan.init_field(st, ws, 0, seed=3, k_peak=8.0, kinetic_energy=1.0)
        plan.step(st, ws, dt, steps)
        sp = plan.spectra(st, ws, 1)[0]
        info = plan.read_step_info(ws)[0]
        got = to_numpy(plan.get_state(st, 0))
        del st, ws
        plan.close()
        torch.cuda.empty_cache()
        eu, es = rel_l2(got[:3], ref[:3]), rel_l2(got[3:], ref[3:])
        del got
        _log(f"512^3 FP{prec} vs oracle after {steps} steps: velocity rel L2 {eu:.2e}, scalars {es:.2e}")
        tol = 1e-12 if prec == 64 else 1e-5
        assert eu < tol and es < tol, (prec, eu, es)
        assert info["flags"] == 0 and info["steps"] == steps
        rel_tol, abs_tol = (1e-10, 1e-14) if prec == 64 else (1e-4, 1e-10)
        r = _shells_close(sp["E"], rs["E"], rs["K"], rel_tol, abs_tol)
        for j in range(S):
            r = max(r, _shells_close(sp["E_phi"][j], rs["E_phi"][j], rs["K"], rel_tol, abs_tol))
        assert abs(sp["eps"] - rs["eps"]) <= rel_tol * rs["eps"]
        _log(f"512^3 FP{prec} vs oracle: max shell rel error {r:.2e}")


def test_512_fp32_against_fp64_fields_and_spectra():
    torch = torch_mod()
    N, S = 512, 2
    prm = ora.Params(nu=7e-4, schmidt=(0.7, 1.0), mean_grad=((0.0, 1.0, 0.0),) * 2, power=0.1, k_force=2.0)
    plans = _pair(N, S, prm, 3, 8.0)
    p64, s64, w64 = plans[64]
    p32, s32, w32 = plans[32]
    max_u = p64.spectra(s64, w64, 2)[0]["max_abs_u_sum"]
    dt = 0.5 * (2.0 * math.pi / N) / max_u
    _log(f"512^3 fixed dt {dt:.6f} from the FP64 initial field")
    for prec in (32, 64):
        p, s, w = plans[prec]
        p.step(s, w, dt, 10)
    torch.cuda.synchronize()
    err = _device_rel_l2(torch, s32, s64)
    _log(f"512^3 after 10 steps: FP32 vs FP64 rel L2 {err:.2e}")
    assert err < 1e-5
    sp64, sp32 = p64.spectra(s64, w64, 1)[0], p32.spectra(s32, w32, 1)[0]
    r = _shells_close(sp32["E"], sp64["E"], sp64["K"])
    for j in range(S):
        _shells_close(sp32["E_phi"][j], sp64["E_phi"][j], sp64["K"])
    _log(f"512^3 after 10 steps: max shell rel error {r:.2e}")
    for prec in (32, 64):
        p, s, w = plans[prec]
        p.step(s, w, dt, 190)
    torch.cuda.synchronize()
    sp64, sp32 = p64.spectra(s64, w64, 1)[0], p32.spectra(s32, w32, 1)[0]
    r = _shells_close(sp32["E"], sp64["E"], sp64["K"])
    for j in range(S):
        _shells_close(sp32["E_phi"][j], sp64["E_phi"][j], sp64["K"])
    _log(f"512^3 after 200 steps: max shell rel error {r:.2e}, "
         f"eps {sp32['eps']:.6e} vs {sp64['eps']:.6e}")
    assert abs(sp32["eps"] - sp64["eps"]) <= 1e-4 * sp64["eps"]
    for prec in (32, 64):
        info = plans[prec][0].read_step_info(plans[prec][2])[0]
        assert info["flags"] == 0 and info["steps"] == 200
    del plans, s32, s64, w32, w64
    torch.cuda.empty_cache()


def test_1024_fp32_against_fp64_gpu():
    torch = torch_mod()
    N, S = 1024, 1
    prm = ora.Params(nu=3e-4, schmidt=(1.0,), mean_grad=((0.0, 1.0, 0.0),), power=0.1, k_force=2.0)
    plans = _pair(N, S, prm, 4, 8.0)
    p64, s64, w64 = plans[64]
    p32, s32, w32 = plans[32]
    max_u = p64.spectra(s64, w64, 2)[0]["max_abs_u_sum"]
    dt = 0.5 * (2.0 * math.pi / N) / max_u
    for prec in (32, 64):
        p, s, w = plans[prec]
        p.step(s, w, dt, 10)
        torch.cuda.synchronize()
        _log(f"1024^3 FP{prec}: 10 steps done")
    err = _device_rel_l2(torch, s32, s64)
    _log(f"1024^3 after 10 steps: FP32 vs FP64 rel L2 {err:.2e}")
    assert err < 1e-5
    for prec in (32, 64):
        info = plans[prec][0].read_step_info(plans[prec][2])[0]
        assert info["flags"] == 0
    del plans, s32, s64, w32, w64
    torch.cuda.empty_cache()
