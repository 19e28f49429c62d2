"""The general kernels on the GPU against the oracle: grids whose N is not a power of two
(mixed-radix transforms with radices 2..13, the paper's N = 520 = 2^3 5 13 of Sec. 3.1),
and the paper's dealiasing (phase shift with spherical truncation, Sec. 2.3) at any N.

FP64 bar 1e-12 relative L2, FP32 1e-5.  Workspaces start filled with NaN bytes, so a pass
that reads an entry nobody wrote (e.g. modes of the bounding cube outside the sphere) fails.
Power-of-two grids with the phase shift step on the tuned kernels (their phase-shift stage)
and are checked here too, and against the general kernels on the same plan at 256^3 and 512^3.
Sizes: N = 24 (2^3 3), 40 (2^3 5), 52 (2^2 13),
56 (2^3 7), 44 (2^2 11) with the 2/3 rule; N = 16, 32, 64, 128 and 48 with the phase shift;
N = 150, 200, 260 and 390 (lines of 3, 4, 5 and 7 positions per lane and per thread);
N = 520 for one right-hand side and one step; N = 1024 (the longest lines, 16 positions)
against the tuned power-of-two kernels on the same plan.
"""
import math

import numpy as np
import pytest

import oracle as ora
from paper_2012_04838_amd import inputs, psdns
from tests.gpu_helpers import (gpu_rhs, make_plan, poisoned_workspace, progress, rel_l2, set_params, to_numpy,
                               torch_mod)

pytestmark = pytest.mark.gpu


def _prm(S, dealias="cube", **kw):
    sc = (1.0, 0.7, 2.0)[:S]
    g = ((0.0, 1.0, 0.0), (0.2, 1.0, -0.3), (1.0, 0.0, 0.0))[:S]
    return ora.Params(nu=kw.pop("nu", 0.01), schmidt=sc, mean_grad=g, power=0.1, k_force=2.0, dealias=dealias, **kw)


def _state(N, S, seed, dealias="cube", kp=4.0):
    y = ora.init_field(N, S, seed, kp, 1.0, dealias=dealias)
    if S:
        K = ora.kmax_retained(N, dealias)
        y[3:] = inputs.random_spectral_state(N, S, seed + 5, K, 4.0, 0.3) * ora.retained_mask(N, dealias)
    return y


def _run(N, S, prec, prm, y0, dt, nsteps, dealias):
    torch = torch_mod()
    plan = make_plan(N, S, prec, dealias=1 if dealias == "phase" else 0)
    # power-of-two grids step on the tuned kernels (their phase-shift stage), others on the
    # general ones
    assert plan.info.general == (0 if N & (N - 1) == 0 else 1)
    set_params(plan, 0, prm)
    st, ws = plan.new_state(), poisoned_workspace(plan)
    plan.set_state(st, y0, 0)
    plan.step(st, ws, dt, nsteps)
    got = to_numpy(plan.get_state(st, 0))
    info = plan.read_step_info(ws)[0]
    torch.cuda.synchronize()
    return got, info


@pytest.mark.parametrize("N,S", [(24, 1), (40, 2), (52, 0), (56, 1), (44, 1)])
def test_mixed_radix_rhs_matches_oracle(N, S):
    x = inputs.random_spectral_state(N, 3 + S, 60 + N, ora.kmax_retained(N), 5.0)
    prm = _prm(S)
    ref = ora.rhs(x, prm)
    got = gpu_rhs(x, prm, 64)
    err = rel_l2(got, ref)
    progress(f"[general] N={N} S={S} 2/3 rule rhs FP64 rel L2 {err:.2e}")
    assert err < 1e-12
    got32 = gpu_rhs(x, prm, 32)
    assert rel_l2(got32, ref) < 1e-5, rel_l2(got32, ref)


@pytest.mark.parametrize("N,S,prec", [(40, 1, 64), (52, 2, 64), (24, 1, 32)])
def test_mixed_radix_cfl_steps_match_oracle(N, S, prec):
    prm = _prm(S, nu=0.005)
    y0 = _state(N, S, 7)
    got, info = _run(N, S, prec, prm, y0, -0.5, 6, "cube")
    ref, dts = ora.step(y0, prm, nsteps=6, cfl=0.5, return_dts=True)
    err = rel_l2(got, ref)
    progress(f"[general] N={N} S={S} FP{prec} 6 CFL steps rel L2 {err:.2e}")
    assert err < (1e-12 if prec == 64 else 1e-5)
    assert abs(info["t"] - sum(dts)) < (1e-12 if prec == 64 else 1e-6) * sum(dts)


@pytest.mark.parametrize("N,S,prec", [(16, 1, 64), (32, 2, 64), (64, 1, 64), (48, 1, 64), (32, 1, 32),
                                     (128, 1, 64), (128, 2, 32)])
def test_phase_shift_rhs_matches_oracle(N, S, prec):
    K = ora.kmax_retained(N, "phase")
    x = inputs.random_spectral_state(N, 3 + S, 80 + N, K, 5.0) * ora.retained_mask(N, "phase")
    prm = _prm(S, "phase")
    ref = ora.rhs(x, prm)
    # the shifted evaluation matters at this size: the single-grid product differs
    single = ora.rhs(x, ora.Params(**{**prm.__dict__, "dealias": "cube"}))
    got = gpu_rhs(x, prm, prec)
    err = rel_l2(got, ref)
    progress(f"[general] N={N} S={S} phase shift rhs FP{prec} rel L2 {err:.2e} "
             f"(2/3-rule rhs differs by {rel_l2(single, ref):.2e})")
    assert err < (1e-12 if prec == 64 else 1e-5)


@pytest.mark.parametrize("N,S,integrator", [(32, 1, "if"), (48, 2, "if"), (32, 1, "explicit")])
def test_phase_shift_steps_match_oracle(N, S, integrator):
    prm = _prm(S, "phase", nu=0.01, integrator=integrator)
    y0 = _state(N, S, 9, "phase")
    cfl = 0.5 if integrator == "if" else 0.2
    got, info = _run(N, S, 64, prm, y0, -cfl, 5, "phase")
    ref, dts = ora.step(y0, prm, nsteps=5, cfl=cfl, return_dts=True)
    err = rel_l2(got, ref)
    progress(f"[general] N={N} S={S} phase shift {integrator} 5 CFL steps rel L2 {err:.2e}")
    assert err < 1e-12
    assert abs(info["dt"] - dts[-1]) < 1e-12 * dts[-1]


def test_phase_shift_initial_field_and_spectra_match_oracle():
    torch = torch_mod()
    N, S = 48, 1
    prm = _prm(S, "phase")
    plan = make_plan(N, S, 64, dealias=psdns.DEALIAS_PHASE_SPHERE)
    set_params(plan, 0, prm)
    st, ws = plan.new_state(), poisoned_workspace(plan)
    plan.init_field(st, ws, 0, seed=4, k_peak=5.0, kinetic_energy=1.0)
    got = to_numpy(plan.get_state(st, 0))
    ref = ora.init_field(N, S, 4, 5.0, 1.0, dealias="phase")
    assert rel_l2(got, ref) < 1e-14
    # modes of the sphere outside the 2/3 cube are populated, none outside the sphere
    assert np.any(got[:, ora.retained_mask(N, "phase") & ~ora.retained_mask(N)] != 0)
    assert np.all(got[:, ~ora.retained_mask(N, "phase")] == 0)
    y = _state(N, S, 11, "phase")
    plan.set_state(st, y, 0)
    sp = plan.spectra(st, ws)[0]
    torch.cuda.synchronize()
    rs = ora.spectra(y, prm)
    ph = ora.physical_stats(y)
    assert len(sp["E"]) == len(rs["E"]) == ora.n_shells(N, "phase")
    np.testing.assert_allclose(sp["E"], rs["E"], rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(sp["E_phi"], rs["E_phi"], rtol=1e-12, atol=1e-15)
    assert abs(sp["eps"] - rs["eps"]) <= 1e-12 * rs["eps"]
    np.testing.assert_allclose(sp["vgt_skew"], ph["vgt_skew"], rtol=1e-9)
    np.testing.assert_allclose(sp["phi2_skew"], ph["phi2_skew"], rtol=1e-9)
    assert abs(sp["max_abs_u_sum"] - ph["max_abs_u_sum"]) <= 1e-13 * ph["max_abs_u_sum"]


def test_general_plans_step_by_graph_replay_and_report_pressure_unsupported():
    torch = torch_mod()
    N, S, dt = 40, 1, 0.004
    prm = _prm(S, "phase")
    y0 = _state(N, S, 13, "phase")
    plan = make_plan(N, S, 64, dealias=psdns.DEALIAS_PHASE_SPHERE)
    set_params(plan, 0, prm)
    st, ws = plan.new_state(), poisoned_workspace(plan)
    plan.set_state(st, y0, 0)
    stream = torch.cuda.Stream()
    plan.set_graph(True)
    with torch.cuda.stream(stream):
        plan.step(st, ws, dt, 2)
        plan.step(st, ws, dt, 2)
    stream.synchronize()
    plan.set_graph(False)
    got = to_numpy(plan.get_state(st, 0))
    assert rel_l2(got, ora.step(y0, prm, dt, 4)) < 1e-12
    with pytest.raises(psdns.PsdnsError, match="general kernels"):
        plan.pressure(st, ws)
    torch.cuda.synchronize()


def test_alvelius_forcing_with_phase_shift_matches_oracle():
    N, S = 32, 1
    prm = _prm(S, "phase", forcing_mode="alvelius", stoch_seed=5)
    prm.power = 0.3
    y0 = _state(N, S, 15, "phase", kp=3.0)
    got, _ = _run(N, S, 64, prm, y0, -0.5, 4, "phase")
    ref = ora.step(y0, prm, None, 4, cfl=0.5, stoch_state={"b": {}, "n": 0})
    assert rel_l2(got, ref) < 1e-12, rel_l2(got, ref)


@pytest.mark.timeout(900)
def test_paper_grid_520_rhs_and_step_match_oracle():
    """N = 520 = 2^3 5 13 (Table 2 of the paper), one scalar: the right-hand side in FP64
    against the oracle, and one fixed step in FP32 against the oracle's FP64 step."""
    torch = torch_mod()
    N, S = 520, 1
    prm = _prm(S, nu=8e-4)
    progress("[general] 520^3 oracle initial field")
    y0 = ora.init_field(N, S, 2, 8.0, 1.0)
    y0[3:] = inputs.random_spectral_state(N, S, 3, ora.kmax_retained(N), 8.0, 0.3)
    progress("[general] 520^3 GPU right-hand side (FP64)")
    got = gpu_rhs(y0, prm, 64)
    torch.cuda.empty_cache()
    progress("[general] 520^3 oracle right-hand side")
    ref = ora.rhs(y0, prm)
    err = rel_l2(got, ref)
    del got, ref
    progress(f"[general] 520^3 rhs FP64 rel L2 {err:.2e}")
    assert err < 1e-12
    dt = ora.cfl_dt(y0, 0.5)
    got, info = _run(N, S, 32, prm, y0, dt, 1, "cube")
    torch.cuda.empty_cache()
    progress("[general] 520^3 oracle step")
    ref = ora.step(y0, prm, dt, 1)
    err = rel_l2(got, ref)
    progress(f"[general] 520^3 one step FP32 vs oracle rel L2 {err:.2e}")
    assert err < 1e-5 and info["flags"] == 0


@pytest.mark.timeout(600)
@pytest.mark.parametrize("N,S", [(150, 1), (200, 1), (260, 1), (390, 0)])
def test_general_kernels_at_every_line_length_match_oracle(N, S):
    """The x pass holds ceil(N/64) positions of a line per lane and the z-forward pass
    ceil(N/TT) per thread, each count compiled on its own: N = 150 (2 3 5^2), 200 (2^3 5^2),
    260 (2^2 5 13) and 390 (2 3 5 13) reach 3, 4, 5 and 7."""
    x = inputs.random_spectral_state(N, 3 + S, 70 + N, ora.kmax_retained(N), 8.0)
    prm = _prm(S)
    progress(f"[general] N={N} S={S} oracle right-hand side")
    ref = ora.rhs(x, prm)
    got = gpu_rhs(x, prm, 64)
    err = rel_l2(got, ref)
    got32 = gpu_rhs(x, prm, 32)
    err32 = rel_l2(got32, ref)
    progress(f"[general] N={N} S={S} rhs FP64 rel L2 {err:.2e}, FP32 {err32:.2e}")
    assert err < 1e-12
    assert err32 < 1e-5


@pytest.mark.timeout(900)
@pytest.mark.parametrize("S,prec", [(1, 32), (0, 64)])
def test_general_kernels_match_tuned_kernels_at_1024(S, prec):
    """N = 1024 with the 2/3 rule, the largest grid: the right-hand side and one CFL step of
    the general kernels (16 positions per lane and per thread in FP32) against the tuned
    power-of-two kernels on the same plan, state and workspace."""
    torch = torch_mod()
    N = 1024
    prm = ora.Params(nu=3e-4, schmidt=(1.0,)[:S], mean_grad=((0.0, 1.0, 0.0),)[:S], power=0.1, k_force=2.0)
    plan = make_plan(N, S, prec)
    assert plan.info.general == 0
    set_params(plan, 0, prm)
    st, ws = plan.new_state(), plan.new_workspace()
    progress(f"[general] 1024^3 S={S} FP{prec}: tuned kernels")
    plan.init_field(st, ws, 0, seed=4, k_peak=8.0, kinetic_energy=1.0)
    if S:
        plan.step(st, ws, -0.5, 1)  # scalar structure
    out_t, st_t = plan.new_state(), st.clone()
    plan.rhs(st, out_t, ws)
    plan.step(st_t, ws, -0.5, 1)
    dt_t = plan.read_step_info(ws)[0]["dt"]
    progress(f"[general] 1024^3 S={S} FP{prec}: general kernels")
    plan.use_general_kernels()
    assert plan.info.general == 1 and plan.info.n_schedules == 1
    out_g = plan.new_state()
    plan.rhs(st, out_g, ws)
    plan.step(st, ws, -0.5, 1)
    dt_g = plan.read_step_info(ws)[0]["dt"]
    real = torch.float32 if prec == 32 else torch.float64

    def rel(a, b):
        a, b = a.view(real), b.view(real)
        return float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b))

    e_rhs, e_step = rel(out_g, out_t), rel(st, st_t)
    tol = 1e-5 if prec == 32 else 1e-12
    progress(f"[general] 1024^3 S={S} FP{prec}: rhs rel L2 {e_rhs:.2e}, step {e_step:.2e}, "
             f"dt {dt_g:.6e} vs {dt_t:.6e}")
    assert e_rhs < tol and e_step < tol
    assert abs(dt_g - dt_t) <= (1e-6 if prec == 32 else 1e-13) * dt_t
    with pytest.raises(psdns.PsdnsError, match="general kernels"):
        plan.pressure(st, ws)
    del st, st_t, out_t, out_g, ws
    plan.close()
    torch.cuda.empty_cache()


@pytest.mark.timeout(900)
@pytest.mark.parametrize("S,prec", [(1, 32), (0, 64)])
def test_every_schedule_at_1024_matches_general_kernels(S, prec):
    """1024^3: the schedules differ most at this size (64-byte tiles of 8 elements per
    thread against 128-byte tiles of 16, one or two x-pass lines per block, register or LDS
    twiddles, one wavefront per column in schedule 7), and the per-pass tuner mixes them.
    The right-hand side of every schedule, and of the per-pass mix the FP32 tuner picks here
    (column passes on 128-byte tiles, the x pass in one-line blocks, the fused pass in
    schedule 7), against schedule 0's, and schedule 0's against the general kernels on the
    same state; one CFL step of the mix and of schedules 1, 4 and 7 against schedule 0, and
    a repeated step bitwise equal to the first."""
    torch = torch_mod()
    N = 1024
    prm = ora.Params(nu=3e-4, schmidt=(1.0,)[:S], mean_grad=((0.0, 1.0, 0.0),)[:S], power=0.1, k_force=2.0)
    plan = make_plan(N, S, prec)
    set_params(plan, 0, prm)
    st, ws, out = plan.new_state(), plan.new_workspace(), plan.new_state()
    plan.init_field(st, ws, 0, seed=4, k_peak=8.0, kinetic_energy=1.0)
    plan.set_schedule(0)
    if S:
        plan.step(st, ws, -0.5, 1)  # scalar structure
    real = torch.float32 if prec == 32 else torch.float64
    tol = 1e-5 if prec == 32 else 1e-12
    tag = f"[general] 1024^3 S={S} FP{prec}"

    def rel(a, b):
        a, b = a.view(real), b.view(real)
        return float(torch.linalg.vector_norm((a - b).double()) / torch.linalg.vector_norm(b.double()))

    def select(v):
        if v == "mix":
            plan.set_pass_schedules([1, 1, 4, 1, 7])
        else:
            plan.set_schedule(v)

    # each schedule against schedule 0 as it comes (one right-hand side kept)
    rhs0 = None
    for v in list(range(plan.n_schedules)) + ["mix"]:
        select(v)
        plan.rhs(st, out, ws)
        if rhs0 is None:
            rhs0 = out.clone()
            continue
        e = rel(out, rhs0)
        progress(f"{tag} schedule {v}: rhs rel L2 against schedule 0 {e:.2e}")
        assert e < tol, (v, e)
    y0, dt0 = None, None
    for v in (0, 1, 4, 7, "mix"):
        select(v)
        y = st.clone()
        plan.clear_step_info(ws)
        plan.step(y, ws, -0.5, 1)
        dt = plan.read_step_info(ws)[0]["dt"]
        if y0 is None:
            y0, dt0 = y, dt
            continue
        e = rel(y, y0)
        progress(f"{tag} schedule {v}: one CFL step rel L2 against schedule 0 {e:.2e}, dt {dt:.9e} vs {dt0:.9e}")
        assert e < tol / 10, (v, e)
        assert abs(dt - dt0) <= (1e-6 if prec == 32 else 1e-13) * dt0
        del y
    # the same step again on the same inputs repeats bitwise (schedule 0 and the mix)
    for v in (0, "mix"):
        select(v)
        ya, yb = st.clone(), st.clone()
        plan.step(ya, ws, -0.5, 1)
        plan.step(yb, ws, -0.5, 1)
        torch.cuda.synchronize()
        assert torch.equal(ya, yb), v
        if v == 0:
            assert torch.equal(ya, y0)
        del ya, yb
    progress(f"{tag}: repeated steps bitwise equal")
    plan.use_general_kernels()
    plan.rhs(st, out, ws)
    e = rel(rhs0, out)
    progress(f"{tag} schedule 0: rhs rel L2 against the general kernels {e:.2e}")
    assert e < tol
    del st, ws, out, rhs0, y0
    plan.close()
    torch.cuda.empty_cache()


@pytest.mark.timeout(900)
@pytest.mark.parametrize("N,S,prec", [(256, 2, 64), (512, 2, 32)])
def test_tuned_phase_shift_matches_general_kernels(N, S, prec):
    """The phase-shift dealiasing on the tuned kernels of a power-of-two grid (sphere of
    bounding K, shifted and unshifted evaluations) against the general kernels on the same
    plan, state and workspace: the right-hand side and one CFL step."""
    torch = torch_mod()
    prm = _prm(S, "phase", nu=7e-4)
    plan = make_plan(N, S, prec, dealias=psdns.DEALIAS_PHASE_SPHERE)
    assert plan.info.general == 0
    set_params(plan, 0, prm)
    st, ws = plan.new_state(), plan.new_workspace()
    progress(f"[general] {N}^3 S={S} FP{prec} phase shift: tuned kernels")
    plan.init_field(st, ws, 0, seed=6, k_peak=8.0, kinetic_energy=1.0)
    plan.step(st, ws, -0.5, 1)  # scalar structure
    out_t, st_t = plan.new_state(), st.clone()
    plan.rhs(st, out_t, ws)
    plan.step(st_t, ws, -0.5, 1)
    dt_t = plan.read_step_info(ws)[0]["dt"]
    plan.use_general_kernels()
    assert plan.info.general == 1
    out_g = plan.new_state()
    plan.rhs(st, out_g, ws)
    plan.step(st, ws, -0.5, 1)
    dt_g = plan.read_step_info(ws)[0]["dt"]
    real = torch.float32 if prec == 32 else torch.float64

    def rel(a, b):
        a, b = a.view(real), b.view(real)
        return float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b))

    e_rhs, e_step = rel(out_t, out_g), rel(st_t, st)
    tol = 1e-5 if prec == 32 else 1e-12
    progress(f"[general] {N}^3 S={S} FP{prec} phase shift: tuned vs general rhs rel L2 {e_rhs:.2e}, "
             f"step {e_step:.2e}, dt {dt_t:.6e} vs {dt_g:.6e}")
    assert e_rhs < tol and e_step < tol
    assert abs(dt_g - dt_t) <= (1e-6 if prec == 32 else 1e-13) * dt_g
    del st, st_t, out_t, out_g, ws
    plan.close()
    torch.cuda.empty_cache()


def test_tuned_phase_shift_graph_replay_matches_eager_bitwise():
    """The phase-shift stage on the tuned kernels runs the same launches eagerly and from a
    captured graph (it has no fused last stage), so replayed CFL steps equal eager ones
    bitwise, call after call, FP64 and FP32, and match the oracle."""
    torch = torch_mod()
    N, S = 32, 1
    prm = _prm(S, "phase")
    y0 = _state(N, S, 21, "phase", kp=3.0)
    for prec in (64, 32):
        stream = torch.cuda.Stream()
        with torch.cuda.stream(stream):
            pe = make_plan(N, S, prec, dealias=psdns.DEALIAS_PHASE_SPHERE)
            pg = make_plan(N, S, prec, dealias=psdns.DEALIAS_PHASE_SPHERE)
            assert pe.info.general == 0 and pg.info.general == 0
            for p in (pe, pg):
                set_params(p, 0, prm)
            se, we = pe.new_state(), pe.new_workspace()
            sg, wg = pg.new_state(), pg.new_workspace()
            pe.set_state(se, y0, 0)
            pg.set_state(sg, y0, 0)
            pg.set_graph(True)
            for rep in range(3):
                pe.step(se, we, -0.5, 2)
                pg.step(sg, wg, -0.5, 2)
                stream.synchronize()
                a, b = to_numpy(pe.get_state(se, 0)), to_numpy(pg.get_state(sg, 0))
                assert np.array_equal(a, b), (prec, rep, np.max(np.abs(a - b)))
        stream.synchronize()
        ref = ora.step(y0, prm, None, 6, cfl=0.5)
        err = rel_l2(a, ref)
        progress(f"[general] 32^3 phase shift FP{prec}: graph = eager bitwise over 3 calls, vs oracle {err:.2e}")
        assert err < (1e-12 if prec == 64 else 1e-5)
        del pe, pg
    torch.cuda.synchronize()
