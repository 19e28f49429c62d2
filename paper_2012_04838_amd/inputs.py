"""Seeded synthetic spectral inputs.

Used by the tests, the smoke check and the benchmark to build the same input
for the GPU library and for the CPU reference.  It holds none of the
method's arithmetic: it only draws random complex coefficients, shapes their
magnitude with a smooth envelope, limits their support to a cube of
wavenumbers and mirrors the kx = 0 plane so that the coefficients describe
real fields.

Layout (the library's canonical layout): complex128 array
[field][kz: N][ky: N][kx: N//2 + 1]; index i along an axis stands for the
wavenumber i (i <= N/2) or i - N.
"""
from __future__ import annotations

import numpy as np


def _signed(N: int) -> np.ndarray:
    i = np.arange(N)
    return np.where(i <= N // 2, i, i - N)


def random_spectral_state(N: int, n_fields: int, seed: int, kmax: int,
                          k_envelope: float = 4.0, amplitude: float = 1.0) -> np.ndarray:
    """Random coefficients c_f(k) = amplitude * N^3 * g * exp(-|k|^2 / (2 k_envelope^2)),
    g standard complex Gaussian, for 0 < |k| with |kx|, |ky|, |kz| <= kmax; zero elsewhere.
    The kx = 0 plane satisfies c(0, -ky, -kz) = conj(c(0, ky, kz))."""
    rng = np.random.default_rng(seed)
    NX = N // 2 + 1
    s = _signed(N)
    kz = s[:, None, None]
    ky = s[None, :, None]
    kx = np.arange(NX)[None, None, :]
    support = (np.abs(kx) <= kmax) & (np.abs(ky) <= kmax) & (np.abs(kz) <= kmax)
    k2 = (kx * kx + ky * ky + kz * kz).astype(np.float64)
    support = support & (k2 > 0)
    env = np.exp(-k2 / (2.0 * k_envelope * k_envelope))
    shape = (n_fields, N, N, NX)
    c = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    c = c * (amplitude * float(N) ** 3 * env * support)
    # mirror the kx = 0 plane: keep (ky > 0) or (ky == 0 and kz > 0), conjugate into the rest
    plane = c[:, :, :, 0]
    keep = (ky[0, :, 0][None, :] > 0) | ((ky[0, :, 0][None, :] == 0) & (kz[:, 0, 0][:, None] > 0))
    jz, jy = np.nonzero(keep)
    mirrored = np.zeros_like(plane)
    mirrored[:, jz, jy] = plane[:, jz, jy]
    mirrored[:, (-jz) % N, (-jy) % N] = np.conj(plane[:, jz, jy])
    c[:, :, :, 0] = mirrored * support[:, :, 0][None]
    return c
