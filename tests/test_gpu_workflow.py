"""The paper's workflow pieces on the GPU: the initial field from the paper's piecewise
spectrum, and starting the scalar from zero on a developed velocity field."""
import numpy as np
import pytest

import oracle as ora
from paper_2012_04838_amd import psdns
from tests.gpu_helpers import make_plan, rel_l2, set_params, to_numpy, torch_mod

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("N,S,prec", [(32, 1, 64), (64, 2, 64), (64, 0, 32)])
def test_paper_spectrum_initial_field_matches_oracle(N, S, prec):
    torch = torch_mod()
    plan = make_plan(N, S, prec)
    st, ws = plan.new_state(), plan.new_workspace()
    plan.init_field_spectrum(st, ws, 0, 9, psdns.SPECTRUM_PAPER, 3.0, 1.5)
    got = to_numpy(plan.get_state(st, 0))
    torch.cuda.synchronize()
    ref = ora.init_field(N, S, 9, 3.0, 1.5, spectrum="paper")
    assert rel_l2(got, ref) < (1e-14 if prec == 64 else 1e-7)


def test_scalar_restart_from_developed_velocity():
    """Velocity stepped alone, then phi reset to zero (psdns_zero_scalars) and both stepped:
    equal to the oracle doing the same."""
    torch = torch_mod()
    N, S, dt = 32, 1, 0.005
    prm = ora.Params(nu=0.01, schmidt=(1.0,), mean_grad=((0.0, 1.0, 0.0),), power=0.1, k_force=2.0)
    y = ora.init_field(N, S, 14, 4.0, 1.0)
    y[3] = 0.3 * y[0]  # some scalar content that the restart must discard
    plan = make_plan(N, S, 64)
    set_params(plan, 0, prm)
    st, ws = plan.new_state(), plan.new_workspace()
    plan.set_state(st, y, 0)
    plan.step(st, ws, dt, 3)
    plan.zero_scalars(st, 0)
    mid = to_numpy(plan.get_state(st, 0))
    plan.step(st, ws, dt, 3)
    got = to_numpy(plan.get_state(st, 0))
    torch.cuda.synchronize()
    ref = ora.step(y, prm, dt, 3)
    assert np.max(np.abs(mid[3])) == 0.0
    assert rel_l2(mid[:3], ref[:3]) < 1e-12
    ref[3] = 0.0
    ref = ora.step(ref, prm, dt, 3)
    assert rel_l2(got, ref) < 1e-12
