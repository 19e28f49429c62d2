"""Host-side checks of the C ABI that need no GPU: every function declared in
include/psdns.h is exported, and argument validation fails cleanly."""
import ctypes
import os
import re

import pytest

from paper_2012_04838_amd import psdns

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "psdns.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(psdns_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    L = psdns.lib()
    names = declared_functions()
    assert len(names) >= 15
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    # every declared function has a binding signature
    assert set(names) <= set(psdns._SIGS), set(names) - set(psdns._SIGS)


def test_sizes_reject_invalid_params():
    assert psdns.state_bytes(34, 0, 64) == 0      # prime factor 17
    assert psdns.state_bytes(105, 0, 64) == 0     # odd
    assert psdns.state_bytes(6, 0, 64) == 0       # below 8
    assert psdns.state_bytes(512, 5, 64) == 0
    assert psdns.state_bytes(512, 2, 16) == 0
    assert psdns.workspace_bytes(2048, 0, 32) == 0
    assert psdns.plan_device_bytes(34, 0, 64) == 0
    assert psdns.state_bytes(64, 0, 64, dealias=2) == 0


def test_mixed_radix_and_phase_shift_plans_size_their_retained_sets():
    # N = 520 = 2^3 5 13 (the paper's grid) with the 2/3 rule: K = 173
    K = 173
    M, PX = 2 * K + 1, ((K + 1 + 15) // 16) * 16
    assert psdns.state_bytes(520, 1, 32) == 4 * M * M * PX * 8
    # phase shift with the sphere 9 |k|^2 < 2 N^2: bounding cube K = 30 at N = 64, and one
    # more buffer of the unshifted products (3 + S fields after the y forward pass)
    K = 30
    M, PX = 2 * K + 1, ((K + 1 + 15) // 16) * 16
    assert psdns.state_bytes(64, 2, 64, dealias=psdns.DEALIAS_PHASE_SPHERE) == 5 * M * M * PX * 16
    ws = psdns.workspace_bytes(64, 2, 64, dealias=psdns.DEALIAS_PHASE_SPHERE)
    assert ws >= ((9 + 5) * 64 * M * PX + 12 * 64 * 64 * PX + 2 * 5 * M * M * PX) * 16


def test_plan_device_bytes_cover_the_plan_tables():
    # twiddles (N complex) and one slot-parameter record per slot, each in 256-byte granules
    for n, s, prec, b in [(32, 1, 64, 1), (512, 2, 32, 3)]:
        got = psdns.plan_device_bytes(n, s, prec, b)
        assert got >= n * (8 if prec == 32 else 16) + b * 8 * 16
        assert got % 256 == 0
        assert got < psdns.workspace_bytes(n, s, prec, b)


def test_sizes_follow_the_compact_layout():
    for n, s, prec in [(32, 1, 64), (512, 2, 32), (1024, 1, 64)]:
        K = (n - 1) // 3
        M, PX = 2 * K + 1, ((K + 1 + 15) // 16) * 16
        cs = 8 if prec == 32 else 16
        assert psdns.state_bytes(n, s, prec) == (3 + s) * M * M * PX * cs
        ws = psdns.workspace_bytes(n, s, prec)
        assert ws >= ((5 + 2 * s) * n * M * PX + (6 + 3 * s) * n * n * PX + 2 * (3 + s) * M * M * PX) * cs
        assert psdns.state_bytes(n, s, prec, batch=3) == 3 * psdns.state_bytes(n, s, prec)


def test_plan_create_validates_before_touching_the_device():
    L = psdns.lib()
    h = ctypes.c_void_p()
    p = psdns.plan_params(34, 0, 64, 1)
    assert L.psdns_plan_create(ctypes.byref(p), ctypes.byref(h)) == -1
    assert b"prime factors" in L.psdns_last_error()
    p = psdns.plan_params(64, 0, 64, 1, 5)
    assert L.psdns_plan_create(ctypes.byref(p), ctypes.byref(h)) == -1
    assert b"dealias" in L.psdns_last_error()
    assert L.psdns_plan_create(None, ctypes.byref(h)) == -1
    assert L.psdns_plan_destroy(None) == 0
    assert L.psdns_step(None, None, None, 0.1, 1, None) == -1


@pytest.mark.parametrize("n", [8, 16, 32, 64, 128, 256, 512, 1024])
def test_every_size_has_device_code(n):
    # sizes are reported for every supported grid in both precisions
    for prec in (32, 64):
        assert psdns.workspace_bytes(n, 1, prec) > 0
