"""Serving loop: every request's result is the same alone and inside a mixed,
continuously batched workload; admission respects the HBM budget; slots are reused."""
import copy

import numpy as np
import pytest

from paper_2012_04838_amd import psdns
from paper_2012_04838_amd.serve import Request, Server, footprint_bytes, make_mix, summarize, viscosity_for
from tests.gpu_helpers import torch_mod

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("autotune", [False, True])
def test_result_same_alone_and_in_mix(autotune, tmp_path):
    """With one fixed schedule the result is bitwise the same alone and in the mix.  With
    the autotuner on, a group of another capacity may run another schedule (same
    transforms, other butterfly association), so the bar is the FP32 field tolerance."""
    torch = torch_mod()
    from paper_2012_04838_amd import tune

    cache = tune.TuneCache(str(tmp_path / "tune.json")) if autotune else None
    mix = make_mix(14, rate=200.0, seed=3, sizes=(32, 64), weights=(0.5, 0.5), steps=(3, 12), scalars=(0, 1, 2))
    picked = [0, 5, 9, 13]
    for i in picked:
        mix[i].keep_state = True
    # small groups force slot reuse and waiting
    srv = Server(capacity=lambda n: 3, autotune=autotune, tune_cache=cache)
    done = srv.run(copy.deepcopy(mix))
    srv.close()
    assert len(done) == len(mix)
    by_id = {r.rid: r for r in done}
    for i in picked:
        alone = copy.deepcopy(mix[i])
        alone.arrival = 0.0
        s2 = Server(capacity=lambda n: 1, autotune=autotune, tune_cache=cache)
        res = s2.run([alone])[0]
        s2.close()
        a, b = res.state, by_id[i].state
        assert a is not None and b is not None
        if autotune:
            err = np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel())
            assert err < 1e-5, (i, err)
            assert abs(res.spectra["K"] - by_id[i].spectra["K"]) <= 1e-5 * abs(by_id[i].spectra["K"])
        else:
            assert np.array_equal(a, b), (i, np.max(np.abs(a - b)))
            assert res.spectra["K"] == by_id[i].spectra["K"]
    torch.cuda.synchronize()


def test_admission_respects_budget_and_reuses_slots():
    torch = torch_mod()
    per = footprint_bytes(64, 1, 32, 2)
    reqs = [Request(rid=i, n=64, n_scalars=1, steps=4, seed=10 + i, nu=viscosity_for(64)) for i in range(5)]
    srv = Server(hbm_budget=int(1.5 * per), capacity=lambda n: 2, autotune=False)
    done = srv.run(reqs)
    assert len(done) == 5
    assert len(srv.groups) == 1 and srv.reserved() <= srv.budget
    # with two slots, at most two requests were ever admitted before the first finished
    admits = sorted(r.t_admit for r in done)
    finishes = sorted(r.t_done for r in done)
    assert admits[2] >= finishes[0]
    # a request that cannot fit the budget waits instead of over-committing
    big = Request(rid=99, n=128, n_scalars=0, steps=1, seed=1, nu=viscosity_for(128))
    srv.waiting.append(big)
    srv._admit()
    assert big in srv.waiting and not any(k[0] == 128 for k in srv.groups)
    srv.close()
    s = summarize(done, 1.0, srv.steps_done)
    assert s["p99_s"] >= s["p50_s"] > 0
    torch.cuda.synchronize()


def test_viscosity_for_matches_kmax_eta():
    for n in (64, 128, 256, 512):
        nu = viscosity_for(n)
        eta = (nu ** 3 / 0.1) ** 0.25
        assert abs(eta * n / 3.0 - 1.5) < 1e-12


def test_reused_slot_starts_a_fresh_stochastic_run():
    """A one-slot group serves three stochastically forced requests in turn, so each
    reuses the slot (and workspace) of the one before.  Each result is bitwise the one
    the request gives alone: the slot's step count (which keys the random draws) and its
    Ornstein-Uhlenbeck vectors start from zero for every new request."""
    torch = torch_mod()
    reqs = [Request(rid=i, n=32, n_scalars=1, steps=6, seed=40 + i, nu=viscosity_for(32), keep_state=True,
                    forcing=psdns.FORCING_STOCHASTIC, stoch_sigma=0.05, stoch_tl=0.5, stoch_seed=7)
            for i in range(3)]
    srv = Server(capacity=lambda n: 1, autotune=False)
    done = {r.rid: r for r in srv.run(copy.deepcopy(reqs))}
    assert len(srv.groups) == 1
    srv.close()
    for r in reqs:
        alone = Server(capacity=lambda n: 1, autotune=False)
        res = alone.run([copy.deepcopy(r)])[0]
        alone.close()
        assert not res.failed and not done[r.rid].failed
        assert np.array_equal(res.state, done[r.rid].state), r.rid
    torch.cuda.synchronize()


def test_diverging_run_is_reported_failed():
    """A request whose step record carries a flag (here a CFL number above 1 from a
    fixed CFL target of 1.5) comes back with `failed` set; the others of its mix do not."""
    torch = torch_mod()
    reqs = [Request(rid=0, n=32, n_scalars=0, steps=2, seed=5, nu=viscosity_for(32)),
            Request(rid=1, n=32, n_scalars=0, steps=2, seed=6, nu=viscosity_for(32), cfl=1.5)]
    srv = Server(capacity=lambda n: 2, autotune=False)
    done = {r.rid: r for r in srv.run(reqs)}
    srv.close()
    assert not done[0].failed and done[0].flags == 0
    assert done[1].failed and done[1].flags & psdns.FLAG_CFL
    assert summarize(list(done.values()), 1.0, 1.0)["failed"] == 1
    torch.cuda.synchronize()
