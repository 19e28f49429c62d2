"""GPU spectra and statistics (Table 1, Eqs. (10)-(13)) against the CPU oracle."""
import numpy as np
import pytest

import oracle as ora
from paper_2012_04838_amd import inputs
from tests.gpu_helpers import make_plan, set_params, torch_mod

pytestmark = pytest.mark.gpu


def _state(N, S, seed):
    y = ora.init_field(N, S, seed, 4.0, 1.0)
    if S:
        y[3:] = inputs.random_spectral_state(N, S, seed + 7, ora.kmax_retained(N), 4.0, 0.4)
    # a small non-solenoidal part exercises the |k.u|^2 term of 2 nu <S:S>
    y[:3] += 0.05 * inputs.random_spectral_state(N, 3, seed + 9, ora.kmax_retained(N), 3.0, 0.1)
    return y


def _gpu_spectra(y, prm, prec, flags=3):
    torch_mod()
    N = y.shape[-3]
    S = y.shape[0] - 3
    plan = make_plan(N, S, prec)
    set_params(plan, 0, prm)
    st, ws = plan.new_state(), plan.new_workspace()
    plan.set_state(st, y, 0)
    a = plan.spectra_raw(st, ws, flags).cpu().numpy()
    b = plan.spectra_raw(st, ws, flags).cpu().numpy()
    from paper_2012_04838_amd import psdns
    return psdns.parse_spectra(a[0], int(plan.info.n_shells), S), a, b


def _close(got, ref, rtol):
    got, ref = np.asarray(got, float), np.asarray(ref, float)
    assert np.all(np.abs(got - ref) <= rtol * np.maximum(np.abs(ref), 1e-300) + 1e-300), (got, ref)


@pytest.mark.parametrize("N,S", [(32, 2), (64, 1), (16, 0)])
def test_spectra_fp64_match_oracle(N, S):
    prm = ora.Params(nu=0.013, schmidt=(1.0, 0.7)[:S], mean_grad=((0.0, 1.0, 0.0), (0.3, 1.0, -0.2))[:S])
    y = _state(N, S, 3 + N)
    got, a, b = _gpu_spectra(y, prm, 64)
    assert np.array_equal(a, b), "spectra must be bitwise reproducible"
    ref = ora.spectra(y, prm)
    phys = ora.physical_stats(y)
    Emax = ref["E"].max()
    big = ref["E"] > 1e-12 * Emax
    _close(got["E"][big], ref["E"][big], 1e-12)
    assert np.all(np.abs(got["E"] - ref["E"]) <= 1e-14 * Emax)
    for k in ("K", "eps", "u_rms", "lam", "Re_lambda", "eta", "l_o", "T_e"):
        _close(got[k], ref[k], 1e-12)
    for s in range(S):
        _close(got["E_phi"][s][ref["E_phi"][s] > 1e-12 * ref["E_phi"][s].max()],
               ref["E_phi"][s][ref["E_phi"][s] > 1e-12 * ref["E_phi"][s].max()], 1e-12)
    _close(got["phi_var"], ref["phi_var"], 1e-12)
    _close(got["chi"], ref["chi"], 1e-12)
    _close(got["production"], ref["production"], 1e-11)
    _close(got["vgt_m2"], phys["vgt_m2"], 1e-12)
    _close(got["vgt_skew"], phys["vgt_skew"], 1e-10)
    _close(got["vgt_flat"], phys["vgt_flat"], 1e-11)
    _close(got["max_abs_u_sum"], phys["max_abs_u_sum"], 1e-13)
    _close(got["phi2_skew"], phys["phi2_skew"], 1e-10)
    _close(got["phi2_flat"], phys["phi2_flat"], 1e-11)


def test_spectra_fp32_match_oracle_on_rounded_input():
    N, S = 64, 2
    prm = ora.Params(nu=0.01, schmidt=(1.0, 0.7), mean_grad=((0.0, 1.0, 0.0),) * 2)
    y = _state(N, S, 5).astype(np.complex64).astype(np.complex128)
    got, a, b = _gpu_spectra(y, prm, 32)
    assert np.array_equal(a, b)
    ref = ora.spectra(y, prm)
    phys = ora.physical_stats(y)
    big = ref["E"] > 1e-6 * ref["E"].max()
    _close(got["E"][big], ref["E"][big], 1e-10)   # FP32 data, FP64 sums
    for k in ("K", "eps", "Re_lambda"):
        _close(got[k], ref[k], 1e-10)
    _close(got["vgt_skew"], phys["vgt_skew"], 1e-4)
    _close(got["phi2_flat"], phys["phi2_flat"], 1e-4)


def test_moments_only_flag_leaves_shells_nan():
    N, S = 16, 1
    prm = ora.Params(nu=0.01, schmidt=(1.0,), mean_grad=((0.0, 1.0, 0.0),))
    got, _, _ = _gpu_spectra(_state(N, S, 2), prm, 64, flags=2)
    assert np.all(np.isnan(got["E"])) and np.isnan(got["K"])
    assert np.all(np.isfinite(got["vgt_skew"]))


def test_energy_budget_from_rhs_matches_spectra():
    """dK/dt from the GPU right-hand side equals P - eps from the GPU spectra (solenoidal u)."""
    torch = torch_mod()
    N, S = 64, 0
    prm = ora.Params(nu=0.02, power=0.1, k_force=2.0)
    plan = make_plan(N, S, 64)
    set_params(plan, 0, prm)
    st, out, ws = plan.new_state(), plan.new_state(), plan.new_workspace()
    plan.init_field(st, ws, 0, seed=4, k_peak=4.0, kinetic_energy=1.0)
    plan.rhs(st, out, ws)
    y = plan.get_state(st, 0).cpu().numpy()
    F = plan.get_state(out, 0).cpu().numpy()
    sp = plan.spectra(st, ws, 1)[0]
    w = ora.half_weights(N)
    dK = float(np.sum(w * np.real(np.conj(y) * F))) / float(N) ** 6
    assert abs(dK - (prm.power - sp["eps"])) < 1e-11 * sp["eps"]
    torch.cuda.synchronize()


@pytest.mark.parametrize("prec", [64, 32])
def test_shell_binning_of_hand_placed_modes(prec):
    """Single modes with |k|^2 = 1, 2, 3, 4, 5, 6, 8, 12, 13 fall in shells
    nint|k| = 1, 1, 2, 2, 2, 2, 3, 3, 4 (the table, not any binning code, decides);
    each mode carries a distinct energy on u1 and E(s) is the sum placed in shell s."""
    N = 16
    modes = [((1, 0, 0), 1), ((1, 1, 0), 1), ((1, 1, 1), 2), ((2, 0, 0), 2), ((2, 1, 0), 2),
             ((2, 1, 1), 2), ((2, 2, 0), 3), ((2, 2, 2), 3), ((3, 2, 0), 4)]
    y = np.zeros((3, N, N, N // 2 + 1), dtype=np.complex128)
    want = np.zeros(ora.n_shells(N))
    for i, ((kx, ky, kz), shell) in enumerate(modes):
        e = 0.01 * (i + 1)
        y[0, kz % N, ky % N, kx] = float(N) ** 3 * np.sqrt(e)
        want[shell] += e
    sp, _, _ = _gpu_spectra(y, ora.Params(nu=0.01), prec, flags=1)
    np.testing.assert_allclose(sp["E"], want, rtol=1e-14 if prec == 64 else 2e-7, atol=1e-17)
