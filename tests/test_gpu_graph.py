"""Graph-replayed RK4 steps against eagerly launched ones (bitwise), with eager work and
synchronisation between replays, and slot parameters changed between replays."""
import numpy as np
import pytest

import oracle as ora
from tests.gpu_helpers import make_plan, set_params, to_numpy, torch_mod

pytestmark = pytest.mark.gpu


def test_graph_replays_match_eager_steps():
    torch = torch_mod()
    N, S = 32, 1
    prm = ora.Params(nu=0.01, schmidt=(1.0,), mean_grad=((0.0, 1.0, 0.0),), power=0.1, k_force=2.0)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        pe, pg = make_plan(N, S, 64, 2), make_plan(N, S, 64, 2)
        for p in (pe, pg):
            set_params(p, 0, prm)
            set_params(p, 1, prm)
        se, we = pe.new_state(), pe.new_workspace()
        sg, wg = pg.new_state(), pg.new_workspace()
        for p, st, ws in ((pe, se, we), (pg, sg, wg)):
            p.init_field(st, ws, 0, seed=5, k_peak=4.0)
            p.init_field(st, ws, 1, seed=6, k_peak=3.0)
        pg.set_graph(True)
        for rep in range(4):
            pe.step(se, we, -0.5, 2)
            pg.step(sg, wg, -0.5, 2)
            stream.synchronize()
            a = [to_numpy(pe.get_state(se, i)) for i in range(2)]
            b = [to_numpy(pg.get_state(sg, i)) for i in range(2)]
            stream.synchronize()
            for i in range(2):
                assert np.array_equal(a[i], b[i]), (rep, i)
            # eager work between replays, and a parameter change the replay must pick up
            _ = torch.ones(1000, device="cuda").sum().item()
            if rep == 1:
                prm2 = ora.Params(nu=0.02, schmidt=(0.5,), mean_grad=((1.0, 0.0, 0.0),), power=0.05)
                set_params(pe, 1, prm2)
                set_params(pg, 1, prm2)
        ie, ig = pe.read_step_info(we), pg.read_step_info(wg)
        assert ie[0]["steps"] == ig[0]["steps"] == 8
        assert ie[1]["t"] == ig[1]["t"]
    torch.cuda.synchronize()
