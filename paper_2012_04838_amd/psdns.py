"""Thin ctypes binding of libpsdns.so (the C ABI in include/psdns.h).

Only argument marshalling lives here: every step of the computation runs in
the HIP kernels of the library.  PyTorch supplies device memory (tensors) and
the HIP stream of the current device.  If the library is not built, importing
fails loudly; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Sequence

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("PSDNS_LIB") or os.path.join(_PKG, "libpsdns.so")
MAX_SCALARS = 4

FLAG_NONFINITE = 1
FLAG_CFL = 2
SPECTRA_SHELLS = 1
SPECTRA_MOMENTS = 2

_c_int32 = ctypes.c_int32
_c_void_p = ctypes.c_void_p


class PlanParams(ctypes.Structure):
    _fields_ = [("n", _c_int32), ("n_scalars", _c_int32), ("precision", _c_int32), ("batch", _c_int32),
                ("dealias", _c_int32)]


DEALIAS_TWO_THIRDS = 0
DEALIAS_PHASE_SPHERE = 1


FORCING_POWER = 0
FORCING_HOLD = 1
FORCING_STOCHASTIC = 2
FORCING_ALVELIUS = 3
# passes of a right-hand-side evaluation (psdns_set_pass_schedules order)
PASS_Z_INVERSE, PASS_Y_INVERSE, PASS_X, PASS_Y_FORWARD, PASS_Z_FORWARD = range(5)
NUM_PASSES = 5
PASS_NAMES = ("z_inverse", "y_inverse", "x_pass", "y_forward", "z_forward")
INTEGRATOR_IF = 0
INTEGRATOR_EXPLICIT = 1
SPECTRUM_CONFIG = 0
SPECTRUM_PAPER = 1


class SlotParams(ctypes.Structure):
    _fields_ = [("nu", ctypes.c_double), ("power", ctypes.c_double), ("k_force", ctypes.c_double),
                ("schmidt", ctypes.c_double * MAX_SCALARS),
                ("mean_grad", (ctypes.c_double * 3) * MAX_SCALARS),
                ("forcing", _c_int32), ("integrator", _c_int32), ("hold_energy", ctypes.c_double),
                ("stoch_sigma", ctypes.c_double), ("stoch_tl", ctypes.c_double), ("stoch_seed", ctypes.c_uint64)]


class StepInfo(ctypes.Structure):
    _fields_ = [("t", ctypes.c_double), ("dt", ctypes.c_double), ("max_u", ctypes.c_double),
                ("steps", ctypes.c_int64), ("flags", _c_int32), ("active", _c_int32)]


class PlanInfo(ctypes.Structure):
    _fields_ = [(name, _c_int32) for name in ("n", "k_max", "m", "kx_count", "kx_pitch", "n_scalars",
                                             "precision", "batch", "n_shells", "spectra_doubles")] + \
               [("state_bytes", ctypes.c_int64), ("workspace_bytes", ctypes.c_int64),
                ("elems_col", _c_int32), ("elems_x", _c_int32), ("n_schedules", _c_int32),
                ("schedule", _c_int32), ("plan_bytes", ctypes.c_int64), ("dealias", _c_int32),
                ("general", _c_int32), ("pass_schedules", _c_int32 * 5)]


class ScheduleInfo(ctypes.Structure):
    _fields_ = [(name, _c_int32) for name in ("index", "elems_col", "col_width", "elems_fused", "fused_width",
                                             "elems_x", "x_lines")]


class KernelTiming(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", _c_int32), ("total_ms", ctypes.c_double),
                ("median_ms", ctypes.c_double), ("min_ms", ctypes.c_double)]


class PsdnsError(RuntimeError):
    pass


_lib = None

_SIGS = {
    "psdns_state_bytes": (ctypes.c_size_t, [ctypes.POINTER(PlanParams)]),
    "psdns_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(PlanParams)]),
    "psdns_plan_device_bytes": (ctypes.c_size_t, [ctypes.POINTER(PlanParams)]),
    "psdns_plan_create": (ctypes.c_int, [ctypes.POINTER(PlanParams), ctypes.POINTER(_c_void_p)]),
    "psdns_plan_destroy": (ctypes.c_int, [_c_void_p]),
    "psdns_plan_get_info": (ctypes.c_int, [_c_void_p, ctypes.POINTER(PlanInfo)]),
    "psdns_set_slot": (ctypes.c_int, [_c_void_p, _c_int32, ctypes.POINTER(SlotParams), _c_int32]),
    "psdns_init_field": (ctypes.c_int, [_c_void_p, _c_void_p, _c_void_p, _c_int32, ctypes.c_uint64,
                                        ctypes.c_double, ctypes.c_double, _c_void_p]),
    "psdns_init_field_spectrum": (ctypes.c_int, [_c_void_p, _c_void_p, _c_void_p, _c_int32, ctypes.c_uint64,
                                                 _c_int32, ctypes.c_double, ctypes.c_double, _c_void_p]),
    "psdns_zero_scalars": (ctypes.c_int, [_c_void_p, _c_void_p, _c_int32, _c_void_p]),
    "psdns_rhs": (ctypes.c_int, [_c_void_p, _c_void_p, _c_void_p, _c_void_p, _c_void_p]),
    "psdns_step": (ctypes.c_int, [_c_void_p, _c_void_p, _c_void_p, ctypes.c_double, _c_int32, _c_void_p]),
    "psdns_read_step_info": (ctypes.c_int, [_c_void_p, _c_void_p, ctypes.POINTER(StepInfo), _c_void_p]),
    "psdns_clear_step_info": (ctypes.c_int, [_c_void_p, _c_void_p, _c_void_p]),
    "psdns_clear_slot_info": (ctypes.c_int, [_c_void_p, _c_void_p, _c_int32, _c_void_p]),
    "psdns_get_state": (ctypes.c_int, [_c_void_p, _c_void_p, _c_int32, _c_void_p, _c_void_p]),
    "psdns_set_state": (ctypes.c_int, [_c_void_p, _c_void_p, _c_int32, _c_void_p, _c_void_p]),
    "psdns_spectra": (ctypes.c_int, [_c_void_p, _c_void_p, _c_void_p, _c_void_p, _c_int32, _c_void_p]),
    "psdns_set_graph": (ctypes.c_int, [_c_void_p, _c_int32]),
    "psdns_step_noalloc": (ctypes.c_int, [_c_void_p, _c_void_p, ctypes.c_double, _c_int32, _c_void_p, _c_void_p]),
    "psdns_pressure": (ctypes.c_int, [_c_void_p, _c_void_p, _c_void_p, _c_void_p, _c_void_p]),
    "psdns_run": (ctypes.c_int, [_c_void_p, _c_void_p, _c_void_p, ctypes.c_double, _c_int32, _c_int32, _c_void_p,
                                 _c_int32, _c_void_p]),
    "psdns_get_schedule_info": (ctypes.c_int, [_c_void_p, _c_int32, ctypes.POINTER(ScheduleInfo)]),
    "psdns_set_schedule": (ctypes.c_int, [_c_void_p, _c_int32]),
    "psdns_set_pass_schedules": (ctypes.c_int, [_c_void_p, ctypes.POINTER(_c_int32)]),
    "psdns_use_general_kernels": (ctypes.c_int, [_c_void_p]),
    "psdns_tune_passes": (ctypes.c_int, [_c_void_p, _c_void_p, _c_void_p, _c_int32, ctypes.POINTER(ctypes.c_double),
                                         ctypes.POINTER(_c_int32), _c_void_p]),
    "psdns_tune": (ctypes.c_int, [_c_void_p, _c_void_p, _c_void_p, _c_int32, ctypes.POINTER(ctypes.c_double),
                                  ctypes.POINTER(_c_int32), _c_void_p]),
    "psdns_set_timing": (ctypes.c_int, [_c_void_p, _c_int32]),
    "psdns_get_timing": (ctypes.c_int, [_c_void_p, ctypes.POINTER(KernelTiming), _c_int32,
                                        ctypes.POINTER(_c_int32)]),
    "psdns_stream_copy": (ctypes.c_int, [_c_void_p, _c_void_p, ctypes.c_size_t, _c_int32, _c_void_p]),
    "psdns_last_error": (ctypes.c_char_p, []),
}


def lib() -> ctypes.CDLL:
    """Load libpsdns.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run `python -m paper_2012_04838_amd.build` first")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(status: int) -> None:
    if status != 0:
        msg = lib().psdns_last_error().decode(errors="replace")
        raise PsdnsError(f"psdns error {status}: {msg}")


def _torch():
    import torch
    return torch


def _stream():
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr())


def plan_params(n: int, n_scalars: int = 0, precision: int = 64, batch: int = 1, dealias: int = 0) -> PlanParams:
    return PlanParams(n, n_scalars, precision, batch, dealias)


def state_bytes(n: int, n_scalars: int = 0, precision: int = 64, batch: int = 1, dealias: int = 0) -> int:
    p = plan_params(n, n_scalars, precision, batch, dealias)
    return int(lib().psdns_state_bytes(ctypes.byref(p)))


def workspace_bytes(n: int, n_scalars: int = 0, precision: int = 64, batch: int = 1, dealias: int = 0) -> int:
    p = plan_params(n, n_scalars, precision, batch, dealias)
    return int(lib().psdns_workspace_bytes(ctypes.byref(p)))


def plan_device_bytes(n: int, n_scalars: int = 0, precision: int = 64, batch: int = 1, dealias: int = 0) -> int:
    p = plan_params(n, n_scalars, precision, batch, dealias)
    return int(lib().psdns_plan_device_bytes(ctypes.byref(p)))


class Plan:
    """A plan for N^3 grids with S scalars, a precision (32/64) and `batch` slots.

    Device buffers are torch tensors the caller keeps alive: `new_state()` and
    `new_workspace()` allocate them with the sizes the library reports.
    """

    def __init__(self, n: int, n_scalars: int = 0, precision: int = 64, batch: int = 1, dealias: int = 0):
        self.n, self.n_scalars, self.precision, self.batch = n, n_scalars, precision, batch
        self.dealias = dealias
        self._p = plan_params(n, n_scalars, precision, batch, dealias)
        h = ctypes.c_void_p()
        _check(lib().psdns_plan_create(ctypes.byref(self._p), ctypes.byref(h)))
        self._h = h
        info = PlanInfo()
        _check(lib().psdns_plan_get_info(self._h, ctypes.byref(info)))
        self.info = info

    def close(self) -> None:
        if getattr(self, "_h", None):
            lib().psdns_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------------- buffers
    @property
    def n_fields(self) -> int:
        return 3 + self.n_scalars

    @property
    def complex_dtype(self):
        torch = _torch()
        return torch.complex64 if self.precision == 32 else torch.complex128

    def new_state(self):
        torch = _torch()
        return torch.zeros(int(self.info.state_bytes), dtype=torch.uint8, device="cuda")

    def new_workspace(self):
        """A workspace with its per-slot records cleared (psdns_clear_step_info)."""
        torch = _torch()
        ws = torch.empty(int(self.info.workspace_bytes), dtype=torch.uint8, device="cuda")
        self.clear_step_info(ws)
        return ws

    def canonical_shape(self):
        n = self.n
        return (self.n_fields, n, n, n // 2 + 1)

    # ---------------------------------------------------------------- calls
    def set_slot(self, slot: int, nu: float, power: float = 0.0, k_force: float = 2.0,
                 schmidt: Sequence[float] = (), mean_grad: Sequence[Sequence[float]] = (),
                 active: bool = True, forcing: int = FORCING_POWER, hold_energy: float = 0.0,
                 integrator: int = INTEGRATOR_IF, stoch_sigma: float = 0.0, stoch_tl: float = 1.0,
                 stoch_seed: int = 0) -> None:
        sp = SlotParams()
        sp.nu, sp.power, sp.k_force = nu, power, k_force
        sp.forcing, sp.hold_energy, sp.integrator = forcing, hold_energy, integrator
        sp.stoch_sigma, sp.stoch_tl, sp.stoch_seed = stoch_sigma, stoch_tl, stoch_seed
        for i in range(MAX_SCALARS):
            sp.schmidt[i] = schmidt[i] if i < len(schmidt) else 1.0
            g = mean_grad[i] if i < len(mean_grad) else (0.0, 0.0, 0.0)
            for d in range(3):
                sp.mean_grad[i][d] = g[d]
        _check(lib().psdns_set_slot(self._h, slot, ctypes.byref(sp), 1 if active else 0))

    def init_field(self, state, ws, slot: int, seed: int, k_peak: float, kinetic_energy: float = 1.0) -> None:
        _check(lib().psdns_init_field(self._h, _ptr(state), _ptr(ws), slot, seed, k_peak, kinetic_energy,
                                      _stream()))

    def init_field_spectrum(self, state, ws, slot: int, seed: int, spectrum: int, k_param: float,
                            kinetic_energy: float = 1.0) -> None:
        _check(lib().psdns_init_field_spectrum(self._h, _ptr(state), _ptr(ws), slot, seed, spectrum, k_param,
                                               kinetic_energy, _stream()))

    def zero_scalars(self, state, slot: int) -> None:
        _check(lib().psdns_zero_scalars(self._h, _ptr(state), slot, _stream()))

    def rhs(self, state, out, ws) -> None:
        _check(lib().psdns_rhs(self._h, _ptr(state), _ptr(out), _ptr(ws), _stream()))

    def step(self, state, ws, dt: float, nsteps: int = 1) -> None:
        """dt > 0: fixed step; dt < 0: CFL target -dt (Eq. (10))."""
        _check(lib().psdns_step(self._h, _ptr(state), _ptr(ws), dt, nsteps, _stream()))

    def step_noalloc(self, state, dt: float, nsteps: int = 1, info=None) -> None:
        """Steps without a caller workspace (the library's static scratch); `info`, if given,
        is a device uint8 tensor of batch * sizeof(StepInfo) bytes that receives the records
        (parse with step_info_from_bytes)."""
        _check(lib().psdns_step_noalloc(self._h, _ptr(state), dt, nsteps,
                                        _ptr(info) if info is not None else None, _stream()))

    def read_step_info(self, ws):
        arr = (StepInfo * self.batch)()
        _check(lib().psdns_read_step_info(self._h, _ptr(ws), arr, _stream()))
        return [dict(t=a.t, dt=a.dt, max_u=a.max_u, steps=a.steps, flags=a.flags, active=a.active) for a in arr]

    def clear_step_info(self, ws) -> None:
        _check(lib().psdns_clear_step_info(self._h, _ptr(ws), _stream()))

    def clear_slot_info(self, ws, slot: int) -> None:
        _check(lib().psdns_clear_slot_info(self._h, _ptr(ws), slot, _stream()))

    def get_state(self, state, slot: int = 0):
        """Canonical [field][kz][ky][kx] complex tensor (device) of one slot."""
        torch = _torch()
        out = torch.empty(self.canonical_shape(), dtype=self.complex_dtype, device="cuda")
        _check(lib().psdns_get_state(self._h, _ptr(state), slot, _ptr(out), _stream()))
        return out

    def set_state(self, state, canonical, slot: int = 0) -> None:
        torch = _torch()
        c = canonical
        if not isinstance(c, torch.Tensor):
            c = torch.from_numpy(np.ascontiguousarray(c))
        c = c.to(device="cuda", dtype=self.complex_dtype).contiguous()
        if tuple(c.shape) != self.canonical_shape():
            raise ValueError(f"canonical shape {tuple(c.shape)} != {self.canonical_shape()}")
        _check(lib().psdns_set_state(self._h, _ptr(state), slot, _ptr(c), _stream()))
        torch.cuda.current_stream().synchronize()  # keep c alive until the copy ran

    def spectra_raw(self, state, ws, flags: int = SPECTRA_SHELLS | SPECTRA_MOMENTS):
        """Device tensor [batch][spectra_doubles] of FP64 records (layout in include/psdns.h)."""
        torch = _torch()
        out = torch.empty((self.batch, int(self.info.spectra_doubles)), dtype=torch.float64, device="cuda")
        _check(lib().psdns_spectra(self._h, _ptr(state), _ptr(ws), _ptr(out), flags, _stream()))
        return out

    def spectra(self, state, ws, flags: int = SPECTRA_SHELLS | SPECTRA_MOMENTS):
        """Per-slot dicts of shell spectra and statistics (copies to the host)."""
        raw = self.spectra_raw(state, ws, flags).cpu().numpy()
        return [parse_spectra(r, int(self.info.n_shells), self.n_scalars) for r in raw]

    def run(self, state, ws, dt: float, nsteps: int, every: int, flags: int = SPECTRA_SHELLS | SPECTRA_MOMENTS):
        """Step with a statistics time series: returns records[r][slot] as dicts of
        parse_spectra plus "t", one record after every `every` steps."""
        torch = _torch()
        nrec = nsteps // every
        rec = int(self.info.spectra_doubles)
        buf = torch.empty((max(nrec, 1), self.batch * (1 + rec)), dtype=torch.float64, device="cuda")
        _check(lib().psdns_run(self._h, _ptr(state), _ptr(ws), dt, nsteps, every, _ptr(buf), flags, _stream()))
        raw = buf.cpu().numpy()
        out = []
        for r in range(nrec):
            t = raw[r, :self.batch]
            sp = raw[r, self.batch:].reshape(self.batch, rec)
            row = []
            for i in range(self.batch):
                d = parse_spectra(sp[i], int(self.info.n_shells), self.n_scalars)
                d["t"] = float(t[i])
                row.append(d)
            out.append(row)
        return out

    def pressure(self, state, ws):
        """Modified pressure of every slot: complex tensor [batch, N, N, N/2+1] (canonical layout)."""
        torch = _torch()
        out = torch.empty((self.batch, self.n, self.n, self.n // 2 + 1), dtype=self.complex_dtype, device="cuda")
        _check(lib().psdns_pressure(self._h, _ptr(state), _ptr(ws), _ptr(out), _stream()))
        return out

    def set_graph(self, enable: bool) -> None:
        """Replay RK4 steps from a captured HIP graph (non-default streams only)."""
        _check(lib().psdns_set_graph(self._h, 1 if enable else 0))

    # ---------------------------------------------------------------- schedules
    def _refresh_info(self) -> None:
        _check(lib().psdns_plan_get_info(self._h, ctypes.byref(self.info)))

    @property
    def n_schedules(self) -> int:
        return int(self.info.n_schedules)

    @property
    def schedule(self) -> int:
        """Schedule of every pass, or -1 when the passes run in different schedules."""
        return int(self.info.schedule)

    @property
    def pass_schedules(self) -> list:
        """Schedule of each pass (PASS_* order)."""
        return [int(v) for v in self.info.pass_schedules]

    def schedule_info(self, index: int) -> dict:
        si = ScheduleInfo()
        _check(lib().psdns_get_schedule_info(self._h, index, ctypes.byref(si)))
        return {name: int(getattr(si, name)) for name, _ in ScheduleInfo._fields_}

    def set_schedule(self, index: int) -> None:
        _check(lib().psdns_set_schedule(self._h, index))
        self._refresh_info()

    def set_pass_schedules(self, sched) -> None:
        """Schedule of each pass, PASS_* order (five indices in [0, n_schedules))."""
        if len(sched) != NUM_PASSES:
            raise ValueError(f"{NUM_PASSES} schedule indices expected")
        arr = (_c_int32 * NUM_PASSES)(*[int(v) for v in sched])
        _check(lib().psdns_set_pass_schedules(self._h, arr))
        self._refresh_info()

    def use_general_kernels(self) -> None:
        """Run this plan on the general (mixed-radix) kernels even on a power-of-two grid
        with the 2/3 rule (a cross-check of the two kernel families; irreversible)."""
        _check(lib().psdns_use_general_kernels(self._h))
        self._refresh_info()

    def tune_passes(self, state, ws, reps: int = 3):
        """Time every pass in every schedule on `state` and select the fastest schedule of
        each pass; returns (selection [NUM_PASSES], ms [n_schedules][NUM_PASSES])."""
        ms = (ctypes.c_double * (self.n_schedules * NUM_PASSES))()
        best = (_c_int32 * NUM_PASSES)()
        _check(lib().psdns_tune_passes(self._h, _ptr(state), _ptr(ws), reps, ms, best, _stream()))
        self._refresh_info()
        table = [[float(ms[i * NUM_PASSES + p]) for p in range(NUM_PASSES)] for i in range(self.n_schedules)]
        return [int(v) for v in best], table

    def tune(self, state, ws, reps: int = 3):
        """Time every schedule on `state` (steady-state RK stages), select the fastest;
        returns (best index, [ms per stage of each schedule])."""
        ms = (ctypes.c_double * self.n_schedules)()
        best = _c_int32()
        _check(lib().psdns_tune(self._h, _ptr(state), _ptr(ws), reps, ms, ctypes.byref(best), _stream()))
        self._refresh_info()
        return int(best.value), [float(v) for v in ms]

    def set_timing(self, enable: bool) -> None:
        _check(lib().psdns_set_timing(self._h, 1 if enable else 0))

    def get_timing(self, detail: bool = False):
        """{name: (launches, total ms)} since the last call; with detail, {name: dict of
        launches, total_ms, median_ms, min_ms}."""
        arr = (KernelTiming * 16)()
        cnt = _c_int32()
        _check(lib().psdns_get_timing(self._h, arr, 16, ctypes.byref(cnt)))
        if detail:
            return {arr[i].name.decode(): dict(launches=arr[i].launches, total_ms=arr[i].total_ms,
                                               median_ms=arr[i].median_ms, min_ms=arr[i].min_ms)
                    for i in range(cnt.value)}
        return {arr[i].name.decode(): (arr[i].launches, arr[i].total_ms) for i in range(cnt.value)}


def step_info_from_bytes(raw: bytes, batch: int):
    """Records written by psdns_step_noalloc (psdns_step_info[batch]) as dicts."""
    arr = (StepInfo * batch).from_buffer_copy(raw)
    return [dict(t=a.t, dt=a.dt, max_u=a.max_u, steps=a.steps, flags=a.flags, active=a.active) for a in arr]


def stream_copy(dst, src, blocks: int) -> None:
    """The library's streaming copy of src into dst (device uint8 tensors of equal size)."""
    n = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != n:
        raise ValueError("dst and src sizes differ")
    _check(lib().psdns_stream_copy(_ptr(dst), _ptr(src), n, blocks, _stream()))


def parse_spectra(r, ns: int, S: int) -> dict:
    """Named view of one psdns_spectra record."""
    b = ns * (1 + S)
    p = b + 8 + 4 * S
    d = {"E": r[:ns].copy(), "E_phi": r[ns:b].reshape(S, ns).copy()}
    for i, k in enumerate(("K", "eps", "u_rms", "lam", "Re_lambda", "eta", "l_o", "T_e")):
        d[k] = float(r[b + i])
    sc = r[b + 8:b + 8 + 4 * S].reshape(S, 4) if S else np.zeros((0, 4))
    d.update(phi_var=sc[:, 0].copy(), chi=sc[:, 1].copy(), production=sc[:, 2].copy(), prod_over_chi=sc[:, 3].copy())
    d.update(vgt_m2=r[p:p + 3].copy(), vgt_m3=r[p + 3:p + 6].copy(), vgt_m4=r[p + 6:p + 9].copy(),
             vgt_skew=r[p + 9:p + 12].copy(), vgt_flat=r[p + 12:p + 15].copy(), max_abs_u_sum=float(r[p + 15]))
    ph = r[p + 16:p + 16 + 3 * S].reshape(S, 3) if S else np.zeros((0, 3))
    d.update(phi2_m2=ph[:, 0].copy(), phi2_skew=ph[:, 1].copy(), phi2_flat=ph[:, 2].copy())
    return d
