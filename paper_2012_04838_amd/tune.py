"""Autotune cache for the step schedules.

`psdns_tune` times every compiled schedule (tile and radix choice of the step kernels) on
the caller's state and selects the fastest.  This module keeps that choice per (device,
N, S, precision, batch) in a JSON file, so a plan of a known shape starts with its
schedule without re-timing.  Keys also carry a signature of the compiled schedule
table, so a rebuilt library with different schedules does not reuse stale entries.
"""
from __future__ import annotations

import hashlib
import json
import os
import tempfile
from typing import Optional

DEFAULT_PATH = os.environ.get("PSDNS_TUNE_CACHE",
                              os.path.join(os.path.expanduser("~"), ".cache", "psdns", "tune.json"))


def schedule_signature(plan) -> str:
    """Digest of the plan's compiled schedule descriptions."""
    desc = [plan.schedule_info(i) for i in range(plan.n_schedules)]
    return hashlib.sha256(json.dumps(desc, sort_keys=True).encode()).hexdigest()[:12]


def cache_key(device: str, plan) -> str:
    return f"{device}|n{plan.n}|s{plan.n_scalars}|p{plan.precision}|b{plan.batch}|{schedule_signature(plan)}"


class TuneCache:
    """JSON map key -> {"schedule": i, "ms": [...]}; writes are atomic (rename)."""

    def __init__(self, path: Optional[str] = None):
        self.path = path or DEFAULT_PATH
        self._d = self._load()

    def _load(self) -> dict:
        try:
            with open(self.path) as f:
                d = json.load(f)
            return d if isinstance(d, dict) else {}
        except (OSError, ValueError):
            return {}

    def get(self, key: str) -> Optional[int]:
        e = self._d.get(key)
        if isinstance(e, dict) and isinstance(e.get("schedule"), int):
            return e["schedule"]
        return None

    def put(self, key: str, schedule: int, ms) -> None:
        """Record a choice; the file is best effort (an unwritable path keeps it in memory)."""
        self._d[key] = {"schedule": int(schedule), "ms": [float(v) for v in ms]}
        try:
            d = os.path.dirname(os.path.abspath(self.path))
            os.makedirs(d, exist_ok=True)
            fd, tmp = tempfile.mkstemp(dir=d, prefix=".tune-", suffix=".json")
            with os.fdopen(fd, "w") as f:
                json.dump(self._d, f, indent=1, sort_keys=True)
            os.replace(tmp, self.path)
        except OSError:
            pass


def autotune(plan, state, ws, cache: Optional[TuneCache] = None, reps: int = 3,
             device: Optional[str] = None) -> int:
    """Select the plan's schedule from the cache, or time all schedules on `state` and
    record the winner.  Returns the schedule index in use."""
    if device is None:
        import torch

        device = torch.cuda.get_device_name()
    key = cache_key(device, plan)
    if cache is not None:
        hit = cache.get(key)
        if hit is not None and 0 <= hit < plan.n_schedules:
            plan.set_schedule(hit)
            return hit
    best, ms = plan.tune(state, ws, reps)
    if cache is not None:
        cache.put(key, best, ms)
    return best
