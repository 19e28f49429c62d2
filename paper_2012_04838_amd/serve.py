"""Continuous-batching request loop for DNS runs of mixed grid sizes on one GPU.

Each request is one realization: a seeded Rogallo initial field (Sec. 2.3) at N^3
with 0-4 scalars, stepped `steps` times by the integrating-factor RK4 with
dt from CFL (Eq. (10)), FP32.  Requests with the same (N, S, CFL) share one batched
plan (a "group"): every slot of the group is stepped by the same kernel
launches, each slot with its own parameters and its own dt.  Groups run on their
own HIP streams, so work of different sizes overlaps on the device.

Admission is by HBM footprint: a group reserves, for its slot capacity, the state,
the workspace and the plan's own tables (psdns_state_bytes + psdns_workspace_bytes +
psdns_plan_device_bytes, the library's whole device footprint) plus the buffers this
loop adds (the spectra records and the copies of finished states), and a request
waits until its group has a free slot or the memory budget allows creating the
group.  The CFL number is part of the group key because one launch steps every
slot of a group with the same CFL target.  Between launches a group retires
finished slots (their spectra record, step flags and, if asked, final state are
copied out; a run whose record carries a flag, a non-finite velocity or a CFL
number above 1, is returned with `failed` set) and admits waiting requests into
free slots; a launch advances the group by the largest number of steps after
which some slot changes state.
"""
from __future__ import annotations

import math
import time
from collections import deque
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Tuple

import numpy as np

from . import psdns, tune


def viscosity_for(n: int, power: float = 0.1, kmax_eta: float = 1.5) -> float:
    """nu such that kmax*eta = kmax_eta with kmax = N/3 (2/3 rule) and eps = P (stationary
    constant-power forcing): eta = (nu^3/eps)^(1/4) => nu = (eps (kmax_eta/kmax)^4)^(1/3)."""
    kmax = n / 3.0
    return (power * (kmax_eta / kmax) ** 4) ** (1.0 / 3.0)


@dataclass
class Request:
    rid: int
    n: int
    n_scalars: int
    steps: int
    seed: int
    nu: float
    arrival: float = 0.0          # seconds after the server start
    k_peak: float = 4.0
    cfl: float = 0.5
    power: float = 0.1
    k_force: float = 2.0
    schmidt: Tuple[float, ...] = (1.0, 0.7, 1.0, 1.0)
    keep_state: bool = False
    # forcing of the band (psdns.FORCING_POWER with `power`, or FORCING_STOCHASTIC)
    forcing: int = psdns.FORCING_POWER
    stoch_sigma: float = 0.0
    stoch_tl: float = 1.0
    stoch_seed: int = 0
    # filled in by the server
    t_admit: float = math.nan
    t_done: float = math.nan
    spectra: Optional[dict] = None
    state: Optional[np.ndarray] = None
    flags: int = 0                # PSDNS_FLAG_* bits of the run's step record
    failed: bool = False

    @property
    def latency(self) -> float:
        return self.t_done - self.arrival


def default_capacity(n: int) -> int:
    return {8: 32, 16: 32, 32: 32, 64: 16, 128: 8, 256: 4, 512: 2}.get(n, 1)


def footprint_bytes(n: int, s: int, precision: int, capacity: int) -> int:
    """Device bytes a group of `capacity` slots holds: the library's state, workspace and
    plan tables, the spectra records, and at most one canonical state copy per slot
    (finished states kept for the caller)."""
    lib_bytes = psdns.state_bytes(n, s, precision, capacity) + psdns.workspace_bytes(n, s, precision, capacity) + \
        psdns.plan_device_bytes(n, s, precision, capacity)
    ns = int(round(math.sqrt(3.0) * ((n - 1) // 3))) + 1
    spectra = capacity * (ns * (1 + s) + 8 + 4 * s + 16 + 3 * s) * 8
    canon = capacity * (3 + s) * n * n * (n // 2 + 1) * (8 if precision == 32 else 16)
    return lib_bytes + spectra + canon


class Group:
    """One batched plan for a given (N, S), with its buffers and stream."""

    def __init__(self, n: int, s: int, capacity: int, precision: int = 32, use_graph: bool = True,
                 tune_cache: Optional[tune.TuneCache] = None, autotune: bool = True, cfl: float = 0.5):
        import torch

        self.n, self.s, self.capacity, self.cfl = n, s, capacity, cfl
        self.stream = torch.cuda.Stream()
        with torch.cuda.stream(self.stream):
            self.plan = psdns.Plan(n, s, precision, capacity)
            self.state = self.plan.new_state()
            self.ws = self.plan.new_workspace()
            self.spec = torch.empty((capacity, int(self.plan.info.spectra_doubles)), dtype=torch.float64,
                                    device="cuda")
            if autotune:
                # schedule for this (N, S, capacity): timed on a zero field with every slot active
                self.state.zero_()
                for i in range(capacity):
                    self.plan.set_slot(i, nu=viscosity_for(n), active=True)
                tune.autotune(self.plan, self.state, self.ws, cache=tune_cache, reps=2)
        self.stream.synchronize()
        self.plan.set_graph(use_graph)
        self.footprint = footprint_bytes(n, s, precision, capacity)
        self.slots: List[Optional[Request]] = [None] * capacity
        self.remaining = [0] * capacity
        self.event = None          # completion of the last launch
        self.inflight = 0          # steps of the last launch
        for i in range(capacity):
            self.plan.set_slot(i, nu=0.0, active=False)

    def free_slot(self) -> int:
        for i, r in enumerate(self.slots):
            if r is None:
                return i
        return -1

    def busy(self) -> bool:
        return any(r is not None for r in self.slots)

    def close(self):
        self.plan.close()
        del self.state, self.ws, self.spec


class Server:
    """Admission, continuous batching and completion of DNS requests."""

    def __init__(self, hbm_budget: Optional[int] = None, precision: int = 32, use_graph: bool = True,
                 capacity=default_capacity, max_chunk: int = 16, autotune: bool = True,
                 tune_cache: Optional[tune.TuneCache] = None, launch_ms: float = 25.0):
        import torch

        if hbm_budget is None:
            free, _ = torch.cuda.mem_get_info()
            hbm_budget = int(0.8 * free)
        self.budget = hbm_budget
        self.precision = precision
        self.use_graph = use_graph
        self.capacity = capacity
        self.max_chunk = max_chunk
        # a launch covers about launch_ms of device time, so that a large group's steps do
        # not hold up small groups that share a hardware queue with it
        self.launch_ms = launch_ms
        self.autotune = autotune
        self.tune_cache = tune_cache if tune_cache is not None else (tune.TuneCache() if autotune else None)
        self.groups: Dict[Tuple[int, int], Group] = {}
        self.waiting: deque = deque()
        self.done: List[Request] = []
        self.t0 = time.perf_counter()
        self.steps_done = 0.0  # sum of N^3 * steps

    def now(self) -> float:
        return time.perf_counter() - self.t0

    def reserved(self) -> int:
        return sum(g.footprint for g in self.groups.values())

    def submit(self, req: Request) -> None:
        self.waiting.append(req)

    # ---------------------------------------------------------------- admission
    def _group_for(self, req: Request) -> Optional[Group]:
        key = (req.n, req.n_scalars, req.cfl)
        g = self.groups.get(key)
        if g is not None:
            return g
        need = footprint_bytes(req.n, req.n_scalars, self.precision, self.capacity(req.n))
        if self.reserved() + need > self.budget:
            # release idle groups to make room
            for k, og in list(self.groups.items()):
                if not og.busy() and og.event is None:
                    og.close()
                    del self.groups[k]
                    if self.reserved() + need <= self.budget:
                        break
        if self.reserved() + need > self.budget:
            return None
        g = Group(req.n, req.n_scalars, self.capacity(req.n), self.precision, self.use_graph,
                  tune_cache=self.tune_cache, autotune=self.autotune, cfl=req.cfl)
        self.groups[key] = g
        return g

    def _admit(self) -> None:
        now = self.now()
        keep = deque()
        while self.waiting:
            req = self.waiting.popleft()
            if req.arrival > now:
                keep.append(req)
                continue
            g = self._group_for(req)
            slot = g.free_slot() if g is not None and g.event is None else -1
            if slot < 0:
                keep.append(req)
                continue
            g.plan.set_slot(slot, nu=req.nu, power=req.power, k_force=req.k_force,
                            schmidt=req.schmidt[:req.n_scalars],
                            mean_grad=[(0.0, 1.0, 0.0)] * req.n_scalars, active=True, forcing=req.forcing,
                            stoch_sigma=req.stoch_sigma, stoch_tl=req.stoch_tl, stoch_seed=req.stoch_seed)
            import torch
            with torch.cuda.stream(g.stream):
                # also starts the slot's step record and stochastic forcing from zero
                g.plan.init_field(g.state, g.ws, slot, seed=req.seed, k_peak=req.k_peak, kinetic_energy=1.0)
            g.slots[slot] = req
            g.remaining[slot] = req.steps
            req.t_admit = now
        self.waiting = keep

    # ---------------------------------------------------------------- stepping
    def _launch(self, g: Group) -> None:
        import torch

        active = [i for i, r in enumerate(g.slots) if r is not None and g.remaining[i] > 0]
        if not active:
            return
        est_ms = 21.0 * (g.n / 512.0) ** 3 * (3 + g.s) / 5.0 * len(active)  # FP32 step time model
        by_time = max(1, int(self.launch_ms / max(est_ms, 1e-3)))
        chunk = min(min(g.remaining[i] for i in active), self.max_chunk, by_time)
        with torch.cuda.stream(g.stream):
            g.plan.step(g.state, g.ws, -g.cfl, chunk)
            ev = torch.cuda.Event()
            ev.record(g.stream)
        g.event, g.inflight = ev, chunk
        for i in active:
            g.remaining[i] -= chunk
            self.steps_done += float(g.n) ** 3 * chunk

    def _retire(self, g: Group) -> None:
        import torch

        finished = [i for i, r in enumerate(g.slots) if r is not None and g.remaining[i] == 0]
        if not finished:
            return
        with torch.cuda.stream(g.stream):
            raw = g.plan.spectra_raw(g.state, g.ws, psdns.SPECTRA_SHELLS | psdns.SPECTRA_MOMENTS)
            states = {i: g.plan.get_state(g.state, i) for i in finished if g.slots[i].keep_state}
            info = g.plan.read_step_info(g.ws)  # synchronises the group's stream
        g.stream.synchronize()
        raw = raw.cpu().numpy()
        now = self.now()
        for i in finished:
            req = g.slots[i]
            req.flags = int(info[i]["flags"])
            req.failed = req.flags != 0
            req.spectra = psdns.parse_spectra(raw[i], int(g.plan.info.n_shells), g.s)
            if i in states:
                req.state = states[i].cpu().numpy()
            req.t_done = now
            self.done.append(req)
            g.slots[i] = None
            g.plan.set_slot(i, nu=0.0, active=False)

    def tick(self) -> bool:
        """One pass of the loop; returns True while work remains."""
        self._admit()
        for g in list(self.groups.values()):
            if g.event is not None:
                if not g.event.query():
                    continue
                g.event = None
                self._retire(g)
        self._admit()
        for g in self.groups.values():
            if g.event is None:
                self._launch(g)
        return bool(self.waiting) or any(g.busy() for g in self.groups.values())

    def run(self, requests: List[Request], idle_sleep: float = 2e-4, progress_every: int = 0) -> List[Request]:
        import sys

        for r in requests:
            self.submit(r)
        self.t0 = time.perf_counter()
        reported = 0
        while self.tick():
            if progress_every and len(self.done) >= reported + progress_every:
                reported = len(self.done) - len(self.done) % progress_every
                print(f"[serve] {len(self.done)}/{len(requests)} done at {self.now():.1f} s", file=sys.stderr,
                      flush=True)
            if all(g.event is None or not g.event.query() for g in self.groups.values()):
                time.sleep(idle_sleep)
        return self.done

    def close(self):
        for g in self.groups.values():
            g.close()
        self.groups.clear()


# -------------------------------------------------------------------- workloads
def make_mix(n_requests: int, rate: float, seed: int = 0, sizes=(64, 128, 256, 512),
             weights=(0.4, 0.3, 0.2, 0.1), steps=(10, 200), scalars=(0, 1, 2)) -> List[Request]:
    """Poisson arrivals (rate per second) of requests drawn from the serving mix:
    N^3 with the given weights, S uniform over `scalars`, steps uniform in [lo, hi],
    nu from kmax*eta = 1.5, request i seeded with 1000 + i."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(n_requests):
        t += rng.exponential(1.0 / rate) if rate > 0 else 0.0
        n = int(rng.choice(sizes, p=np.asarray(weights) / np.sum(weights)))
        s = int(rng.choice(scalars))
        st = int(rng.integers(steps[0], steps[1] + 1))
        out.append(Request(rid=i, n=n, n_scalars=s, steps=st, seed=1000 + i, nu=viscosity_for(n), arrival=t))
    return out


def summarize(done: List[Request], wall: float, steps_n3: float) -> dict:
    lat = np.array([r.latency for r in done])
    out = {"requests": len(done), "wall_s": wall, "p50_s": float(np.percentile(lat, 50)),
           "p99_s": float(np.percentile(lat, 99)), "mean_s": float(lat.mean()),
           "requests_per_s": len(done) / wall, "N3_steps_per_s": steps_n3 / wall,
           "failed": int(sum(1 for r in done if r.failed))}
    per = {}
    for n in sorted({r.n for r in done}):
        ln = np.array([r.latency for r in done if r.n == n])
        work = sum(float(n) ** 3 * r.steps for r in done if r.n == n)
        per[str(n)] = {"requests": int(ln.size), "p50_s": float(np.percentile(ln, 50)),
                       "p99_s": float(np.percentile(ln, 99)), "N3_steps_per_s": work / wall}
    out["per_size"] = per
    return out


def main():
    import argparse
    import json

    ap = argparse.ArgumentParser(description="serve a Poisson mix of DNS requests on one GPU")
    ap.add_argument("--requests", type=int, default=100)
    ap.add_argument("--load", type=float, default=0.7, help="offered load as a fraction of measured capacity")
    ap.add_argument("--loads", type=str, default="",
                    help="comma-separated offered loads (a sweep); overrides --load")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--progress", type=int, default=50, help="report every this many completions (stderr)")
    args = ap.parse_args()
    loads = [float(v) for v in args.loads.split(",")] if args.loads else [args.load]
    # saturated capacity: every request present at t = 0
    sat = make_mix(args.requests, 0.0, args.seed)
    srv = Server()
    t = time.perf_counter()
    done = srv.run(sat, progress_every=args.progress)
    wall = time.perf_counter() - t
    cap = len(sat) / wall
    out = summarize(done, wall, srv.steps_done)
    out.update(load="saturated")
    srv.close()
    print(json.dumps(out), flush=True)
    for load in loads:
        mix = make_mix(args.requests, load * cap, args.seed)
        srv = Server()
        t = time.perf_counter()
        done = srv.run(mix, progress_every=args.progress)
        out = summarize(done, time.perf_counter() - t, srv.steps_done)
        out.update(saturated_requests_per_s=cap, load=load)
        srv.close()
        print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
