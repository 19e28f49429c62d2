"""Throughput benchmark: N^3 * RK4-steps/s of the pseudo-spectral DNS step on one GPU.

Workload: 512^3 grid, two passive scalars (Sc = 0.7, 1.0, mean gradient (0, 1, 0)
each), nu = 7e-4, constant power P = 0.1 on 0 < |k| <= 2, Rogallo initial field
with spectrum peak k_p = 8 and unit kinetic energy, RK4 with the integrating
factor and dt from CFL = 0.5 every step.  FP32 is the reported value; the same
run in FP64 is reported beside it.  Inputs are resident in HBM before timing.

Timing: the timed region is K steps replayed from a captured HIP graph on one stream
(value and ms_per_step).  Two further untimed passes of K steps give the median of
single graph replays (per-step events) and the per-kernel durations of eager steps
(per-kernel events, for the roofline).  A second leg runs 1024^3 with one scalar
(nu = 3e-4) in FP32 and FP64.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-fp64] [--no-tune]
                       [--n 512] [--scalars 2] [--no-1024] [--serve-requests R]
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "N³·RK4-steps/s at 512³ FP32 vs FP64 on 1 GPU; serve p50/p99 latency"
PEAK_HBM_GBS = 8000.0
NU, POWER, KF, KP = 7e-4, 0.1, 2.0, 8.0
SCHMIDT = (0.7, 1.0)
GRAD = ((0.0, 1.0, 0.0), (0.0, 1.0, 0.0))

# HBM bytes per launch of the 512^3 S=2 FP32 kernels from rocprofv3 --pmc FETCH_SIZE and
# WRITE_SIZE runs, each counter scaled by what it reads for a plain 1e9-byte device copy in
# the same process (FETCH_SIZE x 2.0, WRITE_SIZE x 1.0; the library's own streaming copy and
# the runtime's copy kernel read the same), by the schedule the kernel's pass runs in (the
# per-pass tuner times every schedule, so every one was counted).  The fused pass: the mean
# of its four stage instances, counted for schedule 0; the schedules whose stage-1 instance
# moves the same bytes (within 0.1%) share it.  The unfused z forward, which the default
# step does not run, was counted in an earlier pass over the same kernel code.  `src` is the
# digest of the kernel sources and build flags they were taken with; a different digest
# reports null.
_SAME = (0, 1, 2, 4, 5, 6)  # schedules with 128-byte kx tiles at this size (3 and 7: 64-byte)
MEASURED_TRAFFIC = {
    "src": "f7e3ddece4df755d",
    "workload": (512, 2, 32),
    "bytes": {
        "z_inverse": {**{v: 2982.9e6 for v in _SAME}, 3: 3068.8e6, 7: 3067.6e6},
        "y_inverse": {**{v: 6542.9e6 for v in _SAME}, 3: 7903.5e6, 7: 8371.0e6},
        "x_pass": {v: 6233.0e6 for v in range(8)},
        "y_forward": {**{v: 3046.9e6 for v in _SAME}, 3: 4044.8e6, 7: 3795.2e6},
        "z_forward_update": {0: 2848.8e6},
        "z_forward_update_inverse": {v: 5420.4e6 for v in _SAME},
    },
}


# the sources that define the step kernels of the table and their launch shapes (the host
# API that sequences them is left out)
KERNEL_SOURCES = ("common.hpp", "engine.hpp", "fft.hpp", "mem.hpp", "inst_n512.hip")


def kernel_source_digest() -> str:
    """sha256 over the sources of the step kernels and the build flags of the library."""
    import hashlib

    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2012_04838_amd", "csrc")
    for name in KERNEL_SOURCES:
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    with open(os.path.join(ROOT, "paper_2012_04838_amd", "build.py"), "rb") as f:
        h.update(f.read())
    return h.hexdigest()[:16]


# pass of each timed kernel (the schedule index that applies to it)
KERNEL_PASS = {"z_inverse": 0, "y_inverse": 1, "x_pass": 2, "y_forward": 3, "z_forward_update": 4,
               "z_forward_update_inverse": 4}


def measured_traffic(kernel: str, n: int, s: int, prec: int, pass_schedules):
    """Counter bytes per launch of a kernel, if they were taken on these sources, this
    workload and the schedule its pass runs in (spills and tile shapes change the traffic)."""
    t = MEASURED_TRAFFIC
    if (t["workload"] != (n, s, prec) or kernel not in t["bytes"] or kernel not in KERNEL_PASS
            or t["src"] != kernel_source_digest()):
        return None
    return t["bytes"][kernel].get(pass_schedules[KERNEL_PASS[kernel]])


def kernel_bytes(n: int, s: int, prec: int) -> dict:
    """Algorithmic HBM bytes per launch of each pass for one realization: every retained
    (or, between passes, every partially transformed) complex entry its fields must
    read and write once; padding columns are never touched."""
    K = (n - 1) // 3
    M, KX = 2 * K + 1, K + 1
    F, FA, FB = 3 + s, 5 + 2 * s, 6 + 3 * s
    cs = 8 if prec == 32 else 16
    hc, a_, b_ = M * M * KX, n * M * KX, n * n * KX
    return {
        "z_inverse": cs * (F * hc + FA * a_),
        "y_inverse": cs * (FA * a_ + FB * b_),
        "x_pass": cs * (FB * b_ + F * b_),
        "y_forward": cs * (F * b_ + F * a_),
        # average over the four stages of the state traffic (3, 4, 4, 2 field-sized passes)
        "z_forward_update": cs * (F * a_ + 3.25 * F * hc),
        # fused with the next stage's z inverse: no full y_stage write/read; state traffic
        # (reads 1, 2, 2, 1; writes 1, 1, 1, 1) plus the inverse output
        "z_forward_update_inverse": cs * (F * a_ + 2.5 * F * hc + FA * a_),
    }


def step_bytes(n: int, s: int, prec: int) -> float:
    """Algorithmic bytes of one RK4 step in the steady state of a multi-step call: every
    stage ends with the fused z-forward/update/z-inverse pass."""
    kb = kernel_bytes(n, s, prec)
    return 4.0 * (kb["y_inverse"] + kb["x_pass"] + kb["y_forward"] + kb["z_forward_update_inverse"])


def five_pass_step_bytes(n: int, s: int, prec: int) -> float:
    """The five-pass byte model of one RK4 step: five unfused passes per stage, each reading and
    writing its fields once (6+3S fields through the inverse passes, 3+S through the
    forward passes), retained modes only, and 13 (3+S) compact-state transfers per step
    for y_n, the accumulator and the stage input."""
    K = (n - 1) // 3
    M, KX = 2 * K + 1, K + 1
    F, FB = 3 + s, 6 + 3 * s
    hc, a_, b_ = M * M * KX, n * M * KX, n * n * KX
    entries = 4 * (F * hc + 2 * FB * a_ + 2 * FB * b_ + 2 * F * b_ + 2 * F * a_) + 13 * F * hc
    return entries * (8 if prec == 32 else 16)


def run_gpu(n, s, prec, steps, warmup, seed=3, tune_reps=3, schedule=-1, nu=None, schmidt=None):
    import torch

    from paper_2012_04838_amd import psdns

    plan = psdns.Plan(n, s, prec, 1)
    plan.set_slot(0, nu=NU if nu is None else nu, power=POWER, k_force=KF,
                  schmidt=SCHMIDT[:s] if schmidt is None else schmidt, mean_grad=GRAD[:s])
    st = plan.new_state()
    ws = plan.new_workspace()
    plan.init_field(st, ws, 0, seed=seed, k_peak=KP, kinetic_energy=1.0)
    sched = None
    if schedule >= 0:
        plan.set_schedule(schedule)
        sched = {"chosen": [schedule] * psdns.NUM_PASSES, "ms_per_stage": None}
    elif tune_reps > 0:
        # autotuner (outside the timed region): every compiled schedule as a whole on this
        # state, then the fastest schedule of each pass (the one the timed steps run)
        best, ms_each = plan.tune(st, ws, tune_reps)
        chosen, table = plan.tune_passes(st, ws, tune_reps)
        sched = {"chosen": chosen, "best_whole_schedule": best, "ms_per_stage": ms_each,
                 "ms_per_pass": {psdns.PASS_NAMES[p]: [row[p] for row in table] for p in range(psdns.NUM_PASSES)}}
    if sched is not None:
        sched["chosen_desc"] = {psdns.PASS_NAMES[p]: plan.schedule_info(v) for p, v in enumerate(plan.pass_schedules)}
    stream = torch.cuda.Stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(stream):
        # timed region: K steps replayed from the captured step graph
        plan.set_graph(True)
        plan.step(st, ws, -0.5, warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e0.record(stream)
        plan.step(st, ws, -0.5, steps)
        e1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ms = e0.elapsed_time(e1)
        # untimed pass: the same replays with an event pair around each (per-step median)
        plan.set_timing(True)
        plan.get_timing()
        plan.step(st, ws, -0.5, steps)
        graph_t = plan.get_timing(detail=True)
        # untimed pass: eager steps with an event pair around each kernel (roofline)
        plan.set_graph(False)
        plan.step(st, ws, -0.5, steps)
        timing = plan.get_timing()
        plan.set_timing(False)
    torch.cuda.synchronize()
    info = plan.read_step_info(ws)[0]
    ok = info["flags"] == 0 and math.isfinite(info["max_u"])
    del st, ws
    plan.close()
    torch.cuda.empty_cache()
    step = graph_t.get("step", {})
    return {"ms_total": ms, "wall_s": wall, "timing": timing, "info": info, "finite": ok, "schedule": sched,
            "graph_step_median_ms": step.get("median_ms"), "graph_step_min_ms": step.get("min_ms"),
            "graph_steps_timed": step.get("launches")}


def copy_reference(gbytes: float, reps: int = 5):
    """Copy bandwidth of a known size: torch's device copy and the library's own streaming
    kernel over a sweep of grid sizes (the best is the achievable-bandwidth reference);
    the torch copy is also the dispatch that scales the FETCH_SIZE / WRITE_SIZE counters."""
    import torch

    from paper_2012_04838_amd import psdns

    n = int(gbytes * 1e9) // 16 * 16
    a = torch.ones(n // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    ms = timed(lambda: b.copy_(a))
    out = {"bytes_read": n, "bytes_written": n, "ms": ms, "GBs": 2 * n / (ms * 1e-3) / 1e9}
    kern = {}
    for blocks in (1024, 4096, 16384, 65536, 262144):
        kms = timed(lambda: psdns.stream_copy(b.view(torch.uint8), a.view(torch.uint8), blocks))
        kern[str(blocks)] = 2 * n / (kms * 1e-3) / 1e9
    assert torch.equal(a, b)
    best = max(kern, key=lambda k: kern[k])
    out["stream_copy_GBs"] = kern
    out["stream_copy_best"] = {"blocks": int(best), "GBs": kern[best]}
    del a, b
    torch.cuda.empty_cache()
    return out


def serve_mix(n_requests: int, load: float, seed: int = 0):
    """Serving mix: Poisson arrivals of seeded DNS requests, N^3 in {64,128,256,512} with
    weights 0.4/0.3/0.2/0.1, 0-2 scalars, 10-200 RK4 steps, nu from kmax*eta = 1.5, FP32,
    continuous batching (paper_2012_04838_amd.serve).  The saturated capacity is measured
    first with every request present at t = 0; the timed run offers `load` of it."""
    import torch

    from paper_2012_04838_amd import serve

    sat = serve.make_mix(n_requests, 0.0, seed)
    srv = serve.Server()
    t = time.perf_counter()
    srv.run(sat)
    cap_wall = time.perf_counter() - t
    cap = len(sat) / cap_wall
    sat_rate = srv.steps_done / cap_wall
    srv.close()
    torch.cuda.empty_cache()
    mix = serve.make_mix(n_requests, load * cap, seed)
    srv = serve.Server()
    t = time.perf_counter()
    done = srv.run(mix)
    res = serve.summarize(done, time.perf_counter() - t, srv.steps_done)
    srv.close()
    torch.cuda.empty_cache()
    res.update(load=load, saturated_requests_per_s=cap, saturated_N3_steps_per_s=sat_rate,
               workload="N^3 in {64,128,256,512} w 0.4/0.3/0.2/0.1, S in {0,1,2}, 10-200 steps, FP32, CFL 0.5, "
                        "k_p = 4, nu: kmax*eta = 1.5, seeds 1000+i")
    return res


def _cpu_description():
    """CPU model, and the logical CPUs and physical cores this process may run on."""
    model, topo = None, {}
    try:
        cur = {}
        with open("/proc/cpuinfo") as f:
            for line in f.read().split("\n\n"):
                d = dict(kv.split(":", 1) for kv in line.split("\n") if ":" in kv)
                d = {k.strip(): v.strip() for k, v in d.items()}
                if "processor" in d:
                    topo[int(d["processor"])] = (d.get("physical id", "0"), d.get("core id", d["processor"]))
                    model = model or d.get("model name")
    except OSError:
        pass
    cpus = sorted(os.sched_getaffinity(0))
    phys = len({topo[c] for c in cpus if c in topo}) or None
    return {"cpu_model": model, "logical_cpus": len(cpus), "physical_cores": phys}


def cpu_baseline(n, s):
    """The FP64 oracle on this host: one right-hand-side evaluation at the benchmark size
    (a quarter of an RK4 step; the integrating-factor update adds well under 5%), scaled
    to steps/s; and, beside it, the small configurations in full: 32^3 (20 steps) and
    256^3 (3 CFL steps)."""
    import oracle as ora

    prm = ora.Params(nu=NU, schmidt=SCHMIDT[:s], mean_grad=GRAD[:s], power=POWER, k_force=KF)
    y = ora.init_field(n, s, 3, KP, 1.0)
    t0 = time.perf_counter()
    ora.nonlinear(y, prm)
    dt = time.perf_counter() - t0
    del y
    per_step = 4.0 * dt
    others = {}
    p1 = ora.Params(nu=0.01, schmidt=(1.0,), mean_grad=((0.0, 1.0, 0.0),), power=0.1, k_force=2.0)
    y1 = ora.init_field(32, 1, 1, 4.0, 1.0)
    t0 = time.perf_counter()
    ora.step(y1, p1, 0.005, 20)
    w1 = time.perf_counter() - t0
    others["32^3 S=1 FP64, 20 steps dt 0.005"] = {"s_per_step": w1 / 20, "N3_steps_per_s": 32 ** 3 * 20 / w1}
    p2 = ora.Params(nu=0.0015, schmidt=(1.0,), mean_grad=((0.0, 1.0, 0.0),), power=0.1, k_force=2.0)
    y2 = ora.init_field(256, 1, 2, 6.0, 1.0)
    t0 = time.perf_counter()
    ora.step(y2, p2, None, 3, cfl=0.5)
    w2 = time.perf_counter() - t0
    others["256^3 S=1 FP64, 3 CFL steps"] = {"s_per_step": w2 / 3, "N3_steps_per_s": 256 ** 3 * 3 / w2}
    del y1, y2
    out = {"value": n ** 3 / per_step, "unit": "N^3*RK4-steps/s", "cores": ora.FFT_WORKERS, "kind": "oracle",
           "sample": f"one FP64 oracle RHS evaluation at {n}^3 S={s} ({dt:.1f} s), x4 per RK4 step; "
                     f"scipy.fft with {ora.FFT_WORKERS} workers, numpy elementwise single-threaded",
           "other_configs": others}
    out.update(_cpu_description())
    return out


def batched_small(steps: int = 20, tune_reps: int = 2):
    """Saturated throughput of small grids in one batch: B independent realizations of N^3,
    S = 2, FP32, with B N^3 = 2^24 at every size (the work of an eighth of a 512^3 step),
    stepped together by graph replay with the per-pass tuned schedules.  Reports the
    batch's N^3*steps/s and its step bandwidth on this design's bytes."""
    import torch

    from paper_2012_04838_amd import psdns
    from paper_2012_04838_amd.serve import viscosity_for

    out = {}
    for n, b in ((64, 64), (128, 8), (256, 1)):
        plan = psdns.Plan(n, 2, 32, b)
        for i in range(b):
            plan.set_slot(i, nu=viscosity_for(n), power=POWER, k_force=KF, schmidt=SCHMIDT[:2], mean_grad=GRAD[:2])
        st, ws = plan.new_state(), plan.new_workspace()
        for i in range(b):
            plan.init_field(st, ws, i, seed=100 + i, k_peak=4.0, kinetic_energy=1.0)
        chosen = plan.tune_passes(st, ws, tune_reps)[0] if tune_reps > 0 else [0] * psdns.NUM_PASSES
        stream = torch.cuda.Stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        with torch.cuda.stream(stream):
            plan.set_graph(True)
            plan.step(st, ws, -0.5, 2)
            torch.cuda.synchronize()
            e0.record(stream)
            plan.step(st, ws, -0.5, steps)
            e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        info = plan.read_step_info(ws)
        gbs = b * step_bytes(n, 2, 32) / (ms * 1e-3) / 1e9
        out[str(n)] = {"batch": b, "ms_per_step": ms, "N3_steps_per_s": b * float(n) ** 3 / (ms * 1e-3),
                       "alg_GBs": gbs, "frac": gbs / PEAK_HBM_GBS, "schedule": chosen,
                       "finite": all(r["flags"] == 0 for r in info)}
        del st, ws
        plan.close()
        torch.cuda.empty_cache()
    return out


def options_leg(steps: int = 5):
    """The paper's options on the 512^3 S=2 FP32 workload (CFL 0.5): milliseconds per step
    of each by graph replay, beside the default path (integrating factor, constant power,
    2/3 rule) timed the same way, and the general kernels on the paper's own grid N = 520;
    then the cost of one pressure call and of one spectra-and-statistics call."""
    import torch

    from paper_2012_04838_amd import psdns

    cases = [
        ("default", 512, {}, {}),
        ("explicit_rk4", 512, {}, {"integrator": psdns.INTEGRATOR_EXPLICIT}),
        ("band_energy_hold", 512, {}, {"forcing": psdns.FORCING_HOLD, "hold_energy": 0.01}),
        ("stochastic_eswaran_pope", 512, {},
         {"forcing": psdns.FORCING_STOCHASTIC, "stoch_sigma": 0.05, "stoch_tl": 0.5, "stoch_seed": 7}),
        ("stochastic_alvelius", 512, {}, {"forcing": psdns.FORCING_ALVELIUS, "stoch_seed": 7}),
        ("phase_shift_sphere", 512, {"dealias": psdns.DEALIAS_PHASE_SPHERE}, {}),
        ("mixed_radix_520", 520, {}, {}),
    ]
    out = {}
    for name, n, pkw, skw in cases:
        plan = psdns.Plan(n, 2, 32, 1, **pkw)
        plan.set_slot(0, nu=NU, power=POWER, k_force=KF, schmidt=SCHMIDT[:2], mean_grad=GRAD[:2], **skw)
        st, ws = plan.new_state(), plan.new_workspace()
        plan.init_field(st, ws, 0, seed=3, k_peak=KP, kinetic_energy=1.0)
        plan.tune_passes(st, ws, 1)
        stream = torch.cuda.Stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        with torch.cuda.stream(stream):
            plan.set_graph(True)
            plan.step(st, ws, -0.5, 1)
            torch.cuda.synchronize()
            e0.record(stream)
            plan.step(st, ws, -0.5, steps)
            e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        rec = {"n": n, "ms_per_step": ms, "N3_steps_per_s": float(n) ** 3 / (ms * 1e-3),
               "general_kernels": bool(plan.info.general), "finite": plan.read_step_info(ws)[0]["flags"] == 0}
        if name == "default":
            # one call each of the pressure and of the spectra and statistics
            for what, fn in (("pressure_ms", lambda: plan.pressure(st, ws)),
                             ("spectra_ms", lambda: plan.spectra_raw(st, ws))):
                fn()
                torch.cuda.synchronize()
                e0.record()
                for _ in range(3):
                    fn()
                e1.record()
                torch.cuda.synchronize()
                rec[what] = e0.elapsed_time(e1) / 3
        out[name] = rec
        del st, ws
        plan.close()
        torch.cuda.empty_cache()
    base = out["default"]["ms_per_step"]
    for name, rec in out.items():
        if rec["n"] == 512:
            rec["vs_default"] = rec["ms_per_step"] / base
    return out


def leg_summary(r, n, s, prec, steps):
    """Throughput, step bandwidth under both byte models and the graph-replay median."""
    ms = r["ms_total"] / steps
    out = {"value": float(n) ** 3 / (ms * 1e-3), "ms_per_step": ms,
           "graph_step_median_ms": r["graph_step_median_ms"], "graph_step_min_ms": r["graph_step_min_ms"],
           "frac_five_pass_model": five_pass_step_bytes(n, s, prec) / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS,
           "frac_design_bytes": step_bytes(n, s, prec) / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS,
           "finite": r["finite"], "schedule": r["schedule"]["chosen"] if r["schedule"] else 0}
    kb = kernel_bytes(n, s, prec)
    tim = r["timing"]
    out["kernels"] = {k: {"launches": tim[k][0], "avg_ms": tim[k][1] / max(tim[k][0], 1),
                          "alg_GBs": (kb[k] / (tim[k][1] / tim[k][0] * 1e-3) / 1e9) if k in kb and tim[k][0] else None}
                      for k in tim if tim[k][0]}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--scalars", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-1024", action="store_true", help="skip the 1024^3 S=1 leg")
    ap.add_argument("--steps-1024", type=int, default=10)
    ap.add_argument("--no-small", action="store_true", help="skip the batched small-grid leg")
    ap.add_argument("--no-options", action="store_true", help="skip the leg of the paper's options")
    ap.add_argument("--copy-gb", type=float, default=1.0,
                    help="size of the copy-bandwidth reference (0 disables)")
    ap.add_argument("--serve-requests", type=int, default=40,
                    help="requests of the serving mix (Poisson arrivals at --serve-load of the measured "
                         "saturated capacity); 0 disables")
    ap.add_argument("--serve-load", type=float, default=0.7)
    ap.add_argument("--no-tune", action="store_true", help="run schedule 0 instead of the autotuned schedule")
    ap.add_argument("--schedule", type=int, default=-1, help="run this schedule (no tuning); -1 tunes")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); "
              "the library steps each field on one GPU and does not shard it.", file=sys.stderr)
        sys.exit(2)
    import torch

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    n, s = args.n, args.scalars
    copy = copy_reference(args.copy_gb) if args.copy_gb > 0 else None
    tr = 0 if args.no_tune else 3
    r32 = run_gpu(n, s, 32, args.steps, args.warmup, tune_reps=tr, schedule=args.schedule)
    print(f"[bench] fp32 done: {r32['ms_total'] / args.steps:.3f} ms/step", file=sys.stderr, flush=True)
    r64 = None
    if not args.no_fp64:
        r64 = run_gpu(n, s, 64, args.steps, args.warmup, tune_reps=tr, schedule=args.schedule)
        print(f"[bench] fp64 done: {r64['ms_total'] / args.steps:.3f} ms/step", file=sys.stderr, flush=True)

    leg32 = leg_summary(r32, n, s, 32, args.steps)
    ms32 = leg32["ms_per_step"]
    kb = kernel_bytes(n, s, 32)
    tim = r32["timing"]
    dom = max((k for k in kb), key=lambda k: tim.get(k, (0, 0.0))[1])
    launches, tot = tim[dom]
    avg_ms = tot / max(launches, 1)
    achieved = kb[dom] / (avg_ms * 1e-3) / 1e9
    chosen = r32["schedule"]["chosen"] if r32["schedule"] else [0] * 5
    traffic = measured_traffic(dom, n, s, 32, chosen)
    step_traffic = None
    if all(measured_traffic(k, n, s, 32, chosen) is not None
           for k in ("y_inverse", "x_pass", "y_forward", "z_forward_update_inverse")):
        step_traffic = 4.0 * sum(measured_traffic(k, n, s, 32, chosen)
                                 for k in ("y_inverse", "x_pass", "y_forward", "z_forward_update_inverse"))
    out = {
        "metric": METRIC,
        "value": leg32["value"],
        "unit": "N^3*RK4-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms32,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{n}^3 pseudo-spectral DNS RK4 step, FP32 (FP64 beside), S={s} "
                               f"(Sc {SCHMIDT[:s]}, G=(0,1,0)), nu={NU}, P={POWER} on 0<|k|<={KF:g}, "
                               f"Rogallo IC k_p={KP:g}, CFL 0.5; timed as graph replays", "n": n, "scalars": s,
                   "batch": 1},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": achieved / PEAK_HBM_GBS, "traffic": traffic,
                     "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-scaled)",
                     "traffic_GBs": traffic / (avg_ms * 1e-3) / 1e9 if traffic else None,
                     "alg_bytes_per_launch": kb[dom],
                     "timing": "kernel durations from an eager pass of the same K steps with per-kernel events"},
        "step_roofline": {"alg_GB_per_step": step_bytes(n, s, 32) / 1e9,
                          "achieved_GBs": step_bytes(n, s, 32) / (ms32 * 1e-3) / 1e9,
                          "frac": leg32["frac_design_bytes"],
                          "five_pass_model_GB_per_step": five_pass_step_bytes(n, s, 32) / 1e9,
                          "frac_five_pass_model": leg32["frac_five_pass_model"],
                          "counter_GB_per_step": step_traffic / 1e9 if step_traffic else None,
                          "frac_counter_bytes": (step_traffic / (ms32 * 1e-3) / 1e9 / PEAK_HBM_GBS)
                          if step_traffic else None},
        "graph_step_median_ms": leg32["graph_step_median_ms"],
        "graph_step_min_ms": leg32["graph_step_min_ms"],
        "kernels_fp32": leg32["kernels"],
        "schedule_fp32": r32["schedule"],
        "copy_reference": copy,
        "finite": r32["finite"],
    }
    if r64 is not None:
        leg64 = leg_summary(r64, n, s, 64, args.steps)
        out["fp64"] = {k: leg64[k] for k in ("value", "ms_per_step", "graph_step_median_ms", "frac_five_pass_model",
                                              "frac_design_bytes", "finite")}
        out["fp64"]["step_frac"] = leg64["frac_design_bytes"]
        out["fp32_over_fp64"] = leg64["ms_per_step"] / ms32
        out["schedule_fp64"] = r64["schedule"]
        out["kernels_fp64"] = leg64["kernels"]
    if not args.no_1024:
        # the 1024^3 configuration: one scalar (Sc 1, G = (0, 1, 0)), nu = 3e-4, CFL 0.5
        big = {}
        for prec in (32, 64):
            r = run_gpu(1024, 1, prec, args.steps_1024, 2, seed=4, tune_reps=2 if tr else 0,
                        schedule=args.schedule, nu=3e-4, schmidt=(1.0,))
            leg = leg_summary(r, 1024, 1, prec, args.steps_1024)
            big[f"fp{prec}"] = {k: leg[k] for k in ("value", "ms_per_step", "graph_step_median_ms",
                                                    "frac_five_pass_model", "frac_design_bytes", "finite", "schedule",
                                                    "kernels")}
            print(f"[bench] 1024^3 fp{prec} done: {leg['ms_per_step']:.2f} ms/step", file=sys.stderr, flush=True)
        big["fp32_over_fp64"] = big["fp64"]["ms_per_step"] / big["fp32"]["ms_per_step"]
        big["steps"] = args.steps_1024
        big["workload"] = "1024^3 S=1 (Sc 1, G=(0,1,0)), nu=3e-4, P=0.1 on 0<|k|<=2, Rogallo IC k_p=8, CFL 0.5"
        out["n1024"] = big
    if not args.no_options:
        out["options"] = options_leg()
        print("[bench] options done: " + ", ".join(f"{k} {v['ms_per_step']:.1f} ms" for k, v in out["options"].items()),
              file=sys.stderr, flush=True)
    if not args.no_small:
        out["batched_small"] = batched_small(tune_reps=2 if tr else 0)
        print("[bench] batched small grids done: " + ", ".join(
            f"{k}^3 x{v['batch']} {v['ms_per_step']:.2f} ms" for k, v in out["batched_small"].items()),
            file=sys.stderr, flush=True)
    if args.serve_requests > 0:
        out["serve"] = serve_mix(args.serve_requests, args.serve_load)
        print(f"[bench] serve done: p50 {out['serve']['p50_s']:.3f} s p99 {out['serve']['p99_s']:.3f} s",
              file=sys.stderr, flush=True)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(n, s)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
