"""Plain FP64 CPU oracle for the Fourier pseudo-spectral DNS of forced isotropic
turbulence carrying passive scalars under a uniform mean gradient
(Akhavan-Safaei & Zayernouri, arXiv:2012.04838, Sec. 2).

TEST INFRASTRUCTURE ONLY.  This module is the slow, obviously correct
reference that the GPU library is checked against.  Only the test suite, the
smoke check and the CPU-baseline leg of the benchmark may import it; the
product path never does, and it shares no code with the HIP implementation.

Everything is float64 / complex128 and follows the paper's notation:

* periodic box [0, 2pi)^3 (Eq. (4); L = 2pi as in Sec. 3.1), N points per axis,
  grid x_j = 2 pi j / N;
* physical arrays are indexed [z][y][x] (x = x1 is the fastest axis);
  spectral arrays hold the half spectrum [kz][ky][kx] with kx = 0..N/2;
* wavenumber of index i is i for i <= N/2 and i - N otherwise, i.e. the set
  k_i = -N/2+1 .. N/2 of Sec. 2.2;
* the forward transform is unnormalised, phi_hat = sum_x phi e^{-i k.x}, and
  the inverse carries 1/N^3 (Eq. (5)).

The library FFT (scipy.fft) is used as a plain step; all other arithmetic is
written out here.  Readings of the paper where it is silent or differs from the
configuration this oracle serves are marked "reading:" in the docstrings.
"""
from __future__ import annotations

import math
import os
from dataclasses import dataclass, field
from typing import Sequence

import numpy as np
import scipy.fft as sfft

# Threads handed to scipy.fft (a plain library primitive; no blocking or fusion).
FFT_WORKERS = int(os.environ.get("PSDNS_ORACLE_FFT_WORKERS",
                                 os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)))


# --------------------------------------------------------------------------
# Grid, wavenumbers, truncation (Sec. 2.2, Eqs. (4)-(5))
# --------------------------------------------------------------------------
def wavenumbers_1d(N: int) -> np.ndarray:
    """Integer wavenumber of each FFT index: i for i <= N/2, else i - N (Sec. 2.2)."""
    i = np.arange(N)
    return np.where(i <= N // 2, i, i - N)


def kgrid(N: int):
    """Broadcastable (kx, ky, kz) integer arrays for the half spectrum [kz][ky][kx]."""
    k1 = wavenumbers_1d(N)
    kx = np.arange(N // 2 + 1)[None, None, :]
    ky = k1[None, :, None]
    kz = k1[:, None, None]
    return kx, ky, kz


def k_squared(N: int) -> np.ndarray:
    kx, ky, kz = kgrid(N)
    return (kx * kx + ky * ky + kz * kz).astype(np.float64)


def kmax_retained(N: int, dealias: str = "cube") -> int:
    """Largest retained |k_i|.

    "cube": the 2/3 rule, 3|k_i| < N  <=>  |k_i| <= (N-1)//3.
    reading: the configurations ask for the 2/3 rule (Orszag).
    "phase": the paper's scheme (Sec. 2.3, Sec. 3.1): phase shift with spherical
    truncation at k_max = sqrt(2) N / 3; the largest integer k with 9 k^2 < 2 N^2 bounds
    the retained sphere.
    """
    if dealias == "phase":
        k = 0
        while 9 * (k + 1) * (k + 1) < 2 * N * N:
            k += 1
        return k
    if dealias != "cube":
        raise ValueError(dealias)
    return (N - 1) // 3


def retained_mask(N: int, dealias: str = "cube") -> np.ndarray:
    """Boolean mask of the retained modes on the half spectrum: the cube |kx|,|ky|,|kz| <= K
    ("cube"), or the sphere |k| < sqrt(2) N / 3, i.e. 9 |k|^2 < 2 N^2 ("phase")."""
    if dealias == "phase":
        return 9 * k_squared(N) < 2 * N * N
    K = kmax_retained(N, dealias)
    kx, ky, kz = kgrid(N)
    return (np.abs(kx) <= K) & (np.abs(ky) <= K) & (np.abs(kz) <= K)


def half_weights(N: int) -> np.ndarray:
    """Multiplicity of each stored half-spectrum mode in a full-spectrum sum.

    Modes with kx = 0 or kx = N/2 are their own conjugate partners' plane and
    are counted once; every other stored mode stands for itself and its
    conjugate at -k and is counted twice.
    """
    w = np.full(N // 2 + 1, 2.0)
    w[0] = 1.0
    w[N // 2] = 1.0
    return w[None, None, :]


def to_physical(fhat: np.ndarray) -> np.ndarray:
    """Inverse of Eq. (5): phi(x) = N^-3 sum_k phi_hat e^{i k.x} (real field)."""
    N = fhat.shape[0]
    return sfft.irfftn(fhat, s=(N, N, N), axes=(0, 1, 2), workers=FFT_WORKERS)


def to_spectral(f: np.ndarray) -> np.ndarray:
    """Eq. (5): phi_hat_k = sum_x phi(x) e^{-i k.x} (half spectrum, unnormalised)."""
    return sfft.rfftn(f, axes=(0, 1, 2), workers=FFT_WORKERS)


def truncate(fhat: np.ndarray, dealias: str = "cube") -> np.ndarray:
    """Zero every mode outside the retained set (2/3-rule cube, or the sphere)."""
    N = fhat.shape[-3]
    return np.where(retained_mask(N, dealias), fhat, 0.0)


def shift_phase(N: int) -> np.ndarray:
    """e^{i k . Delta} on the half spectrum for the grid shift Delta = (pi/N)(1, 1, 1), half a
    grid cell along every axis: the spectrum of f(x + Delta) is f_hat(k) e^{i k . Delta}."""
    kx, ky, kz = kgrid(N)
    return np.exp(1j * math.pi * (kx + ky + kz) / N)


# --------------------------------------------------------------------------
# Parameters
# --------------------------------------------------------------------------
@dataclass
class Params:
    """Physical parameters of one realization.

    nu        kinematic viscosity (Eq. (1); the paper calls it "dynamic")
    schmidt   Schmidt number per scalar, D_s = nu / Sc_s (Sec. 2.3)
    mean_grad mean scalar gradient g_s = grad<Phi_s> per scalar (Eq. (3):
              g = (0, beta, 0))
    power     injected power P of the constant-power forcing
    k_force   forced band 0 < |k| <= k_F (Sec. 2.3)
    forcing   False gives decaying turbulence (Sec. 2.3)
    forcing_mode  "power": constant power P, A re-evaluated at every stage (reading of
              the configurations); "hold": the paper's deterministic scheme, applied
              after the last stage only, holding the band energy at hold_energy
    hold_energy   target band energy E_f of the "hold" mode
                  "stochastic": the stochastic band forcing the paper names as an option
              (Sec. 2.3, after Eswaran & Pope): an Ornstein-Uhlenbeck vector b(k) per
              band mode, forcing term P(k) b (see ou_update)
                  "alvelius": Alvelius' random band forcing, the other stochastic option of
              Sec. 2.3 (see alvelius_force): drawn afresh every step, no work against the
              velocity, power P (`power`) injected by the force-force term, SplitMix64 seed
              stoch_seed
    stoch_sigma   standard deviation of each real and imaginary part of b (normalised,
              physical Fourier coefficients of the forcing) in the stationary state of
              the "stochastic" mode
    stoch_tl      correlation time T_L of b
    stoch_seed    SplitMix64 seed of the normal draws
    dealias       "cube": the 2/3 rule (reading of the configurations); "phase": the paper's
              phase shift with spherical truncation at sqrt(2) N / 3 (Sec. 2.3, Sec. 3.1)
    integrator    "if": RK4 in the frame of the viscous/diffusive integrating factor
              (reading of the configurations); "explicit": the paper's classical RK4
              with the viscous and diffusive terms evaluated in every stage (Sec. 2.3)
    """
    nu: float
    schmidt: Sequence[float] = field(default_factory=tuple)
    mean_grad: Sequence[Sequence[float]] = field(default_factory=tuple)
    power: float = 0.0
    k_force: float = 2.0
    forcing: bool = True
    forcing_mode: str = "power"
    hold_energy: float = 0.0
    integrator: str = "if"
    stoch_sigma: float = 0.0
    stoch_tl: float = 1.0
    stoch_seed: int = 0
    dealias: str = "cube"

    @property
    def n_scalars(self) -> int:
        return len(self.schmidt)

    def diffusivities(self):
        """nu for the three velocity components, then D_s = nu/Sc_s."""
        return [self.nu] * 3 + [self.nu / sc for sc in self.schmidt]


# --------------------------------------------------------------------------
# Forcing amplitude (Eq. (1) term A U; band of Sec. 2.3)
# --------------------------------------------------------------------------
def band_energy(uhat: np.ndarray, k_force: float) -> float:
    """E_f = 1/2 <u.u> restricted to the shell 0 < |k| <= k_F (full-spectrum sum / N^6)."""
    N = uhat.shape[-3]
    k2 = k_squared(N)
    band = (k2 > 0) & (k2 <= k_force * k_force)
    e = 0.5 * np.sum(half_weights(N) * band * np.sum(np.abs(uhat) ** 2, axis=0))
    return float(e) / float(N) ** 6


def forcing_amplitude(uhat: np.ndarray, prm: Params) -> float:
    """A = P / (2 E_f), so that the forcing injects exactly P into 1/2<u.u>.

    reading: the configurations ask for constant-power forcing of the band
    0 < |k| <= k_F, applied as A * u_hat on that band and re-evaluated at every
    RK stage from the stage input; A = 0 when forcing is off or E_f = 0.
    """
    if not prm.forcing or prm.forcing_mode != "power" or prm.power == 0.0:
        return 0.0
    ef = band_energy(uhat, prm.k_force)
    return prm.power / (2.0 * ef) if ef > 0.0 else 0.0


def band_hold(uhat: np.ndarray, prm: Params) -> np.ndarray:
    """The paper's deterministic forcing (Sec. 2.3): evaluated once, after the last RK
    stage, it keeps the energy of the band 0 < |k| <= k_F constant.  Applied as an
    amplitude A over the step, exp(A h) = sqrt(E_target / E_f), i.e. the band modes of
    the velocity are scaled by sqrt(E_target / E_f); the rest of the field is untouched.

    reading: the target is the prescribed band energy hold_energy; nothing is done
    when E_f = 0.
    """
    ef = band_energy(uhat, prm.k_force)
    if ef <= 0.0:
        return uhat
    out = uhat.copy()
    mask = band_mask(uhat.shape[-3], prm.k_force)
    out[:, mask] *= math.sqrt(prm.hold_energy / ef)
    return out


def band_mask(N: int, k_force: float) -> np.ndarray:
    k2 = k_squared(N)
    return (k2 > 0) & (k2 <= k_force * k_force)


# --------------------------------------------------------------------------
# Stochastic band forcing (Sec. 2.3 names Eswaran & Pope's scheme as an option)
# --------------------------------------------------------------------------
def band_radius(N: int, k_force: float, dealias: str = "cube") -> int:
    """Largest integer kf with kf^2 <= k_force^2, capped at the retained K."""
    kf = 0
    while float(kf + 1) ** 2 <= k_force * k_force:
        kf += 1
    return min(kf, kmax_retained(N, dealias))


def stochastic_candidates(N: int, k_force: float, dealias: str = "cube"):
    """The wavevectors (kx >= 0, ky, kz) of the box |k_i| <= kf in the order that keys the
    random draws: candidate i = kx + (kf+1) ((ky+kf) + (2kf+1) (kz+kf)).  Returns the
    list of (i, kx, ky, kz) inside the band 0 < |k|^2 <= k_force^2 and the box size."""
    kf = band_radius(N, k_force, dealias)
    span = 2 * kf + 1
    out = []
    for kz in range(-kf, kf + 1):
        for ky in range(-kf, kf + 1):
            for kx in range(0, kf + 1):
                k2 = kx * kx + ky * ky + kz * kz
                if 0 < k2 <= k_force * k_force:
                    out.append((kx + (kf + 1) * ((ky + kf) + span * (kz + kf)), kx, ky, kz))
    return out, (kf + 1) * span * span


def standard_normal(seed: int, q: int) -> float:
    """Normal number q of the stream: Box-Muller on the uniforms 2q and 2q+1,
    sqrt(-2 ln(1 - u1)) cos(2 pi u2)."""
    u = uniform01(seed, np.array([2 * q, 2 * q + 1], dtype=np.uint64))
    return math.sqrt(-2.0 * math.log(1.0 - float(u[0]))) * math.cos(2.0 * math.pi * float(u[1]))


def ou_update(b: dict, h: float, n: int, N: int, prm: Params) -> dict:
    """Step n (1, 2, ... since the process started at b = 0) of the Ornstein-Uhlenbeck
    vector of every band mode, exact over the step h:

        b <- a b + sigma sqrt(1 - a^2) xi,   a = exp(-h / T_L),

    xi a complex 3-vector whose real and imaginary parts are independent standard
    normals (stationary variance sigma^2 per part).  The normal of part p of component
    c of candidate i is number ((n C + i) 3 + c) 2 + p of the stream (C candidates).
    On the plane kx = 0 the field must be real in physical space: b(0, -ky, -kz) is the
    conjugate of b(0, ky, kz), whose own draw is kept for ky > 0 or (ky = 0, kz > 0).

    reading: the paper names the stochastic scheme without giving its formulas; this is
    the Ornstein-Uhlenbeck process of Eswaran & Pope with one complex vector per mode,
    updated once per step with that step's h and held over the stages."""
    cands, C = stochastic_candidates(N, prm.k_force, prm.dealias)
    a = math.exp(-h / prm.stoch_tl)
    c = prm.stoch_sigma * math.sqrt(max(0.0, 1.0 - a * a))
    out = {}
    for i, kx, ky, kz in cands:
        if kx == 0 and (ky < 0 or (ky == 0 and kz < 0)):
            continue
        old = b.get((kx, ky, kz), np.zeros(3, dtype=np.complex128))
        xi = np.array([complex(standard_normal(prm.stoch_seed, ((n * C + i) * 3 + comp) * 2),
                               standard_normal(prm.stoch_seed, ((n * C + i) * 3 + comp) * 2 + 1))
                       for comp in range(3)])
        out[(kx, ky, kz)] = a * old + c * xi
    for i, kx, ky, kz in cands:
        if kx == 0 and (ky < 0 or (ky == 0 and kz < 0)):
            out[(kx, ky, kz)] = np.conj(out[(0, -ky, -kz)])
    return out


def stochastic_forcing_field(b: dict, N: int) -> np.ndarray:
    """The forcing term on the band, zero elsewhere (half spectrum).  b holds normalised
    (physical) Fourier coefficients of the forcing, so in the unnormalised spectral state
    of Eq. (5) the term is N^3 P(k) b(k)."""
    f = np.zeros((3, N, N, N // 2 + 1), dtype=np.complex128)
    n3 = float(N) ** 3
    for (kx, ky, kz), v in b.items():
        k = np.array([kx, ky, kz], dtype=np.float64)
        pv = v - k * (k @ v) / (k @ k)
        f[:, kz % N, ky % N, kx] = n3 * pv
    return f


def transverse_basis(kx: int, ky: int, kz: int):
    """Unit vectors e1, e2 orthogonal to k and to each other: e1 = k x z_hat / |k x z_hat|
    (x_hat when k is along z), e2 = k x e1 / |k| (the basis of the initial field)."""
    k = np.array([kx, ky, kz], dtype=np.float64)
    kp = math.hypot(kx, ky)
    e1 = np.array([1.0, 0.0, 0.0]) if kp == 0.0 else np.array([ky / kp, -kx / kp, 0.0])
    e2 = np.cross(k, e1) / math.sqrt(float(k @ k))
    return e1, e2


def alvelius_force(uhat: np.ndarray, h: float, n: int, prm: Params) -> np.ndarray:
    """Random band forcing after Alvelius (the second stochastic option Sec. 2.3 names),
    drawn afresh for step n (1, 2, ...) from the velocity u_hat at the start of the step
    and held over its four stages; zero outside the band 0 < |k| <= k_F.

    At every band mode the force lies in the plane normal to k:
        f = F (g_A e^{i theta1} e1 + g_B e^{i theta2} e2),   g_A = sin 2 phi, g_B = cos 2 phi,
    with phi and psi uniform on [0, 2 pi) (uniforms 2q and 2q+1 of SplitMix64(stoch_seed),
    q = n C + i for band candidate i of C, the keying of ou_update) and theta2 = theta1 + psi.
    theta1 solves Re(conj(u_hat) . f) = 0: with xi_j = u_hat . e_j,
        a = g_A Re xi1 + g_B (Re xi2 cos psi + Im xi2 sin psi),
        b = g_A Im xi1 + g_B (Im xi2 cos psi - Re xi2 sin psi),
        a cos theta1 + b sin theta1 = 0  ->  theta1 = atan2(-a, b)  (0 when a = b = 0),
    so the force does no work on the velocity of its step.  |f|^2 = F^2 at every mode
    (g_A^2 + g_B^2 = 1); F is the same for all band modes and fixed by the power P that
    the force-force term injects over a step of size h:
        (h / 2) sum_band w |f|^2 / N^6 = P   ->   F = N^3 sqrt(2 P / (h W)),  W = sum_band w
    (w the half-spectrum multiplicity).  On the plane kx = 0 the mode (0, -ky, -kz) takes
    the conjugate of (0, ky, kz), so the force is real.

    reading: the paper names Alvelius' scheme without its formulas.  This keeps its
    defining choices (force normal to k, uncorrelated in time, no work against the
    velocity mode by mode, power set by the force-force term, two random angles per mode)
    with a spectrum that is flat over the band modes."""
    N = uhat.shape[-3]
    cands, C = stochastic_candidates(N, prm.k_force, prm.dealias)
    f = np.zeros((3, N, N, N // 2 + 1), dtype=np.complex128)
    if prm.power <= 0.0 or not cands:
        return f
    W = float(sum(1 if kx == 0 else 2 for _, kx, _, _ in cands))
    amp = float(N) ** 3 * math.sqrt(2.0 * prm.power / (h * W))
    for i, kx, ky, kz in cands:
        if kx == 0 and (ky < 0 or (ky == 0 and kz < 0)):
            continue
        u01 = uniform01(prm.stoch_seed, np.array([2 * (n * C + i), 2 * (n * C + i) + 1], dtype=np.uint64))
        phi, psi = 2.0 * math.pi * float(u01[0]), 2.0 * math.pi * float(u01[1])
        ga, gb = math.sin(2.0 * phi), math.cos(2.0 * phi)
        e1, e2 = transverse_basis(kx, ky, kz)
        u = uhat[:, kz % N, ky % N, kx]
        xi1, xi2 = complex(u @ e1), complex(u @ e2)
        a = ga * xi1.real + gb * (xi2.real * math.cos(psi) + xi2.imag * math.sin(psi))
        b = ga * xi1.imag + gb * (xi2.imag * math.cos(psi) - xi2.real * math.sin(psi))
        th1 = math.atan2(-a, b) if (a != 0.0 or b != 0.0) else 0.0
        th2 = th1 + psi
        f[:, kz % N, ky % N, kx] = amp * (ga * complex(math.cos(th1), math.sin(th1)) * e1 +
                                          gb * complex(math.cos(th2), math.sin(th2)) * e2)
    for i, kx, ky, kz in cands:
        if kx == 0 and (ky < 0 or (ky == 0 and kz < 0)):
            f[:, kz % N, ky % N, 0] = np.conj(f[:, (-kz) % N, (-ky) % N, 0])
    return f


# --------------------------------------------------------------------------
# Right-hand side (Eqs. (6)-(8))
# --------------------------------------------------------------------------
def project(vhat: np.ndarray) -> np.ndarray:
    """Leray projection (I - k k^T/|k|^2) v_hat of Eq. (7); the k = 0 mode is set to 0."""
    N = vhat.shape[-3]
    kx, ky, kz = kgrid(N)
    k2 = k_squared(N)
    inv = np.where(k2 > 0, 1.0 / np.where(k2 > 0, k2, 1.0), 0.0)
    kdotv = kx * vhat[0] + ky * vhat[1] + kz * vhat[2]
    out = np.empty_like(vhat)
    out[0] = vhat[0] - kx * kdotv * inv
    out[1] = vhat[1] - ky * kdotv * inv
    out[2] = vhat[2] - kz * kdotv * inv
    out[:, k2 == 0] = 0.0
    return out


def product_spectra(state: np.ndarray, form: str = "rotational", phase: np.ndarray | None = None):
    """Untruncated spectra of the quadratic terms: (u x omega)^ ("rotational") or
    (u.grad u)^ ("convective") for the velocity, and (u.grad phi_s)^ per scalar, the
    products formed pointwise in physical space from inverse transforms.  With `phase`
    (shift_phase), the products are formed on the grid shifted by Delta: the inputs carry
    e^{i k . Delta} and the transformed products are multiplied back by its conjugate."""
    N = state.shape[-3]
    S = state.shape[0] - 3
    kx, ky, kz = kgrid(N)
    ik = (1j * kx, 1j * ky, 1j * kz)
    y = state if phase is None else state * phase
    back = 1.0 if phase is None else np.conj(phase)
    uhat = y[:3]
    u = [to_physical(uhat[i]) for i in range(3)]
    if form == "rotational":
        # omega_hat = i k x u_hat
        w1 = to_physical(ik[1] * uhat[2] - ik[2] * uhat[1])
        w2 = to_physical(ik[2] * uhat[0] - ik[0] * uhat[2])
        w3 = to_physical(ik[0] * uhat[1] - ik[1] * uhat[0])
        c = (u[1] * w3 - u[2] * w2, u[2] * w1 - u[0] * w3, u[0] * w2 - u[1] * w1)
        vel = [to_spectral(ci) * back for ci in c]
    elif form == "convective":
        # n_i = u_j d_j u_i from the nine gradients i k_j u_i_hat (Sec. 2.3)
        vel = []
        for i in range(3):
            acc = 0.0
            for j in range(3):
                acc = acc + u[j] * to_physical(ik[j] * uhat[i])
            vel.append(to_spectral(acc) * back)
    else:
        raise ValueError(form)
    adv = []
    for s in range(S):
        grad = [to_physical(ik[j] * y[3 + s]) for j in range(3)]
        adv.append(to_spectral(u[0] * grad[0] + u[1] * grad[1] + u[2] * grad[2]) * back)
    return vel, adv


def nonlinear(state: np.ndarray, prm: Params, form: str = "rotational",
              fvec: np.ndarray | None = None) -> np.ndarray:
    """Everything in dy/dt except the viscous/diffusive term -D_f |k|^2 y_f.

    state = (u1_hat, u2_hat, u3_hat, phi_1_hat, ..., phi_S_hat), half spectrum.

    Velocity (Eq. (7)): F_u = P(k) [ (u x omega)^ ]  + A 1_band u_hat, where the
    product is formed in physical space from inverse transforms, transformed
    forward and truncated to the retained set.  u x omega differs from
    -u.grad u by the gradient grad(|u|^2/2), which the projection removes
    (reading: the rotational form is the one the configurations name; the
    paper's convective form is available as form="convective").

    Scalars (Eq. (8), generalised mean gradient g_s):
    F_phi = -(u.grad phi)^ - g_s . u_hat.

    Dealiasing (prm.dealias): "cube" truncates each product to the 2/3-rule cube.
    "phase" is the paper's scheme (Sec. 2.3): every product is the mean of its values on
    the grid and on the grid shifted by half a cell along each axis, truncated to the
    sphere |k| < sqrt(2) N / 3.  The shift multiplies an alias term at k + N m (m in
    {-1, 0, 1}^3) by (-1)^(m1 + m2 + m3), so the mean cancels every alias with an odd
    number of wrapped components, and the sphere keeps those with two out of reach.

    The k = 0 mode of every field is held at zero (zero-mean fluctuations, Sec. 2.1).
    """
    N = state.shape[-3]
    S = state.shape[0] - 3
    mask = retained_mask(N, prm.dealias)
    uhat = state[:3]
    if prm.dealias == "phase":
        v0, a0 = product_spectra(state, form)
        v1, a1 = product_spectra(state, form, shift_phase(N))
        vel = [0.5 * (p + q) for p, q in zip(v0, v1)]
        adv = [0.5 * (p + q) for p, q in zip(a0, a1)]
    else:
        vel, adv = product_spectra(state, form)
    prod = np.stack([np.where(mask, v, 0.0) for v in vel])
    fu = project(prod) if form == "rotational" else -project(prod)

    A = forcing_amplitude(uhat, prm)
    if A != 0.0:
        fu = fu + A * band_mask(N, prm.k_force) * uhat
    if fvec is not None:
        fu = fu + fvec

    out = np.empty_like(state)
    out[:3] = fu
    for s in range(S):
        g = prm.mean_grad[s]
        out[3 + s] = -np.where(mask, adv[s], 0.0) - (g[0] * uhat[0] + g[1] * uhat[1] + g[2] * uhat[2])
    k2 = k_squared(N)
    out[:, k2 == 0] = 0.0
    out[:, ~mask] = 0.0
    return out


def linear_rates(N: int, prm: Params) -> np.ndarray:
    """L_f(k) = -D_f |k|^2 per field (the viscous/diffusive terms of Eqs. (7)-(8))."""
    k2 = k_squared(N)
    return np.stack([-d * k2 for d in prm.diffusivities()])


def rhs(state: np.ndarray, prm: Params, form: str = "rotational", fvec: np.ndarray | None = None) -> np.ndarray:
    """Full dy/dt of Eqs. (7)-(8): nonlinear + forcing + mean-gradient + viscous terms."""
    N = state.shape[-3]
    out = nonlinear(state, prm, form, fvec) + linear_rates(N, prm) * state
    out[:, ~retained_mask(N, prm.dealias)] = 0.0
    out[:, k_squared(N) == 0] = 0.0
    return out


# --------------------------------------------------------------------------
# Time stepping: RK4 with the viscous/diffusive integrating factor
# --------------------------------------------------------------------------
def max_abs_sum_velocity(state: np.ndarray) -> float:
    """max over grid points of |u1| + |u2| + |u3| (the velocity scale of Eq. (10))."""
    u = [to_physical(state[i]) for i in range(3)]
    return float(np.max(np.abs(u[0]) + np.abs(u[1]) + np.abs(u[2])))


def cfl_dt(state: np.ndarray, cfl: float) -> float:
    """dt such that Eq. (10) equals the target: dt = CFL * dx / max(|u1|+|u2|+|u3|), dx = 2pi/N.

    reading: dt is recomputed from y_n at the start of every step.
    """
    N = state.shape[-3]
    dx = 2.0 * math.pi / N
    return cfl * dx / max_abs_sum_velocity(state)


def step(state: np.ndarray, prm: Params, dt: float | None = None, nsteps: int = 1,
         cfl: float | None = None, form: str = "rotational", return_dts: bool = False,
         stoch_state: dict | None = None):
    """Advance nsteps with the classical RK4 of Sec. 2.2 applied in the frame of the
    viscous/diffusive integrating factor (Lawson's IF-RK4).

    With L the diagonal viscous/diffusive operator, v = e^{-L (t - t_n)} y obeys
    dv/dt = e^{-L (t - t_n)} Nl(e^{L (t - t_n)} v); one classical RK4 step on v gives

        k1 = Nl(y_n)
        y_a = E(h/2) (y_n + h/2 k1);           k2 = Nl(y_a)
        y_b = E(h/2) y_n + h/2 k2;             k3 = Nl(y_b)
        y_c = E(h) y_n + h E(h/2) k3;          k4 = Nl(y_c)
        y_{n+1} = E(h) y_n + h/6 (E(h) k1 + 2 E(h/2) (k2 + k3) + k4)

    with E(tau) = exp(L tau).  reading: the paper evaluates the viscous term
    explicitly in each stage; the configurations ask for the integrating factor.

    Either a fixed dt or a CFL target (dt from Eq. (10) at the start of each step).

    With the "stochastic" forcing, stoch_state = {"b": {mode: vector}, "n": steps so far}
    carries the Ornstein-Uhlenbeck process across calls (a fresh process when None):
    every step first draws b with its own h (ou_update), then holds P(k) b over the four
    stages.  With the "alvelius" forcing every step draws its force from y_n with its own
    h and step number stoch_state["n"] (alvelius_force) and holds it over the stages.
    """
    N = state.shape[-3]
    L = linear_rates(N, prm)
    y = state.copy()
    dts = []
    stoch = prm.forcing and prm.forcing_mode == "stochastic"
    alv = prm.forcing and prm.forcing_mode == "alvelius"
    if (stoch or alv) and stoch_state is None:
        stoch_state = {"b": {}, "n": 0}
    for _ in range(nsteps):
        h = dt if cfl is None else cfl_dt(y, cfl)
        dts.append(h)
        fvec = None
        if stoch:
            stoch_state["n"] += 1
            stoch_state["b"] = ou_update(stoch_state["b"], h, stoch_state["n"], N, prm)
            fvec = stochastic_forcing_field(stoch_state["b"], N)
        if alv:
            stoch_state["n"] += 1
            fvec = alvelius_force(y[:3], h, stoch_state["n"], prm)
        if prm.integrator == "explicit":
            # the paper's scheme (Sec. 2.3): classical RK4 on the full right-hand side
            k1 = rhs(y, prm, form, fvec)
            k2 = rhs(y + 0.5 * h * k1, prm, form, fvec)
            k3 = rhs(y + 0.5 * h * k2, prm, form, fvec)
            k4 = rhs(y + h * k3, prm, form, fvec)
            y = y + (h / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)
            if prm.forcing and prm.forcing_mode == "hold":
                y[:3] = band_hold(y[:3], prm)
            continue
        e1 = np.exp(L * h)
        eh = np.exp(L * (0.5 * h))
        k1 = nonlinear(y, prm, form, fvec)
        ya = eh * (y + 0.5 * h * k1)
        k2 = nonlinear(ya, prm, form, fvec)
        yb = eh * y + 0.5 * h * k2
        k3 = nonlinear(yb, prm, form, fvec)
        yc = e1 * y + h * eh * k3
        k4 = nonlinear(yc, prm, form, fvec)
        y = e1 * y + (h / 6.0) * (e1 * k1 + 2.0 * eh * (k2 + k3) + k4)
        if prm.forcing and prm.forcing_mode == "hold":
            y[:3] = band_hold(y[:3], prm)
    return (y, dts) if return_dts else y


# --------------------------------------------------------------------------
# Initial condition (Sec. 2.3: Rogallo's random solenoidal isotropic field)
# --------------------------------------------------------------------------
_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_MIX1 = np.uint64(0xBF58476D1CE4E5B9)
_MIX2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, counter: np.ndarray) -> np.ndarray:
    """Output number `counter` (0-based) of the SplitMix64 stream started from `seed`
    (Steele, Lea & Flood 2014): z = seed + (counter+1)*gamma, then the two
    xor-shift-multiply rounds and a final xor-shift.  All arithmetic mod 2^64."""
    c = np.asarray(counter, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + (c + np.uint64(1)) * _GAMMA
        z = (z ^ (z >> np.uint64(30))) * _MIX1
        z = (z ^ (z >> np.uint64(27))) * _MIX2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform01(seed: int, counter: np.ndarray) -> np.ndarray:
    """Top 53 bits of the SplitMix64 output as a double in [0, 1)."""
    return (splitmix64(seed, counter) >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def init_spectrum(kappa: np.ndarray, k_peak: float) -> np.ndarray:
    """Configured initial spectrum shape E(kappa) = kappa^4 exp(-2 (kappa/k_p)^2).

    reading: the configurations replace the paper's Eq. (9) spectrum with this one.
    """
    return kappa ** 4 * np.exp(-2.0 * (kappa / k_peak) ** 2)


def paper_spectrum(kappa: np.ndarray, k_f: float, u_rms: float = 1.0) -> np.ndarray:
    """The paper's initial spectrum (Sec. 2.3, after Lamorgese et al.):
    E = (u_rms^2 / k_F) (kappa/k_F)^2 for kappa <= k_F and (u_rms^2 / k_F) (kappa/k_F)^(-5/3) beyond."""
    q = np.asarray(kappa / k_f, dtype=np.float64)
    upper = np.where(q > 1.0, q, 1.0) ** (-5.0 / 3.0)
    return (u_rms * u_rms / k_f) * np.where(q <= 1.0, q * q, upper)


def init_field(N: int, n_scalars: int, seed: int, k_peak: float, kinetic_energy: float = 1.0,
               spectrum: str = "config", dealias: str = "cube") -> np.ndarray:
    """Rogallo-type random divergence-free isotropic velocity (Sec. 2.3) with phi = 0 (Sec. 2.3,
    scalar started from zero).

    For every retained k != 0 in the canonical half space (kx > 0; or kx = 0, ky > 0;
    or kx = ky = 0, kz > 0):
      a(k)  = sqrt(E(|k|) / (4 pi |k|^2))
      e1    = k x z_hat / |k x z_hat|  (x_hat when k is along z), e2 = k x e1 / |k|
      theta1, theta2, psi uniform in [0, 2pi) from SplitMix64(seed), counters 3*idx + (0,1,2)
      with idx the linear index of k in the dense [kz][ky][kx] half-spectrum array
      u_hat = N^3 a (e^{i theta1} cos(psi) e1 + e^{i theta2} sin(psi) e2)
    The kx = 0 plane is completed by u_hat(-k) = conj(u_hat(k)), and the field is
    scaled so that K = 1/2 <u.u> equals `kinetic_energy` (reading: "unit kinetic
    energy" of the configurations; the paper's TKE magnification is a factor on K).
    spectrum="paper" uses the paper's spectrum with k_F = k_peak instead of E(k) above.
    The modes are those of the retained set of `dealias` (cube or sphere).
    """
    NX = N // 2 + 1
    state = np.zeros((3 + n_scalars, N, N, NX), dtype=np.complex128)
    kx, ky, kz = kgrid(N)
    KX = np.broadcast_to(kx, (N, N, NX)).astype(np.float64)
    KY = np.broadcast_to(ky, (N, N, NX)).astype(np.float64)
    KZ = np.broadcast_to(kz, (N, N, NX)).astype(np.float64)
    canon = (KX > 0) | ((KX == 0) & (KY > 0)) | ((KX == 0) & (KY == 0) & (KZ > 0))
    sel = canon & retained_mask(N, dealias)
    iz, iy, ix = np.nonzero(sel)
    lin = (iz.astype(np.uint64) * np.uint64(N) + iy.astype(np.uint64)) * np.uint64(NX) + ix.astype(np.uint64)
    k1, k2, k3 = KX[sel], KY[sel], KZ[sel]
    kmag = np.sqrt(k1 * k1 + k2 * k2 + k3 * k3)
    espec = paper_spectrum(kmag, k_peak) if spectrum == "paper" else init_spectrum(kmag, k_peak)
    amp = np.sqrt(espec / (4.0 * math.pi * kmag * kmag))
    # e1 = k x z_hat / |k x z_hat| = (ky, -kx, 0)/sqrt(kx^2+ky^2)
    kp = np.sqrt(k1 * k1 + k2 * k2)
    along_z = kp == 0
    kp_safe = np.where(along_z, 1.0, kp)
    e1 = np.stack([np.where(along_z, 1.0, k2 / kp_safe),
                   np.where(along_z, 0.0, -k1 / kp_safe),
                   np.zeros_like(k1)])
    # e2 = k x e1 / |k|
    e2 = np.stack([k2 * e1[2] - k3 * e1[1],
                   k3 * e1[0] - k1 * e1[2],
                   k1 * e1[1] - k2 * e1[0]]) / kmag
    two_pi = 2.0 * math.pi
    th1 = two_pi * uniform01(seed, 3 * lin + np.uint64(0))
    th2 = two_pi * uniform01(seed, 3 * lin + np.uint64(1))
    psi = two_pi * uniform01(seed, 3 * lin + np.uint64(2))
    alpha = np.exp(1j * th1) * np.cos(psi)
    beta = np.exp(1j * th2) * np.sin(psi)
    scale = float(N) ** 3 * amp
    for c in range(3):
        state[c][sel] = scale * (alpha * e1[c] + beta * e2[c])
    # Hermitian completion of the kx = 0 plane: u_hat(0, -ky, -kz) = conj(u_hat(0, ky, kz))
    plane = state[:3, :, :, 0]
    m = sel[:, :, 0]
    jz, jy = np.nonzero(m)
    plane[:, (-jz) % N, (-jy) % N] = np.conj(plane[:, jz, jy])
    e = kinetic_energy_of(state)
    if e > 0:
        state[:3] *= math.sqrt(kinetic_energy / e)
    return state


# --------------------------------------------------------------------------
# Diagnostics (Table 1, Eqs. (11)-(13))
# --------------------------------------------------------------------------
def kinetic_energy_of(state: np.ndarray) -> float:
    """K = 1/2 <u.u> = 1/2 sum_k |u_hat|^2 / N^6 (Parseval with Eq. (5))."""
    N = state.shape[-3]
    return 0.5 * float(np.sum(half_weights(N) * np.sum(np.abs(state[:3]) ** 2, axis=0))) / float(N) ** 6


def shell_index(N: int) -> np.ndarray:
    """Shell s = nint(|k|) of every half-spectrum mode.  |k|^2 is an integer, so |k| is
    never a half-integer and the rounding has no ties.  reading: the paper does not
    state its binning."""
    return np.rint(np.sqrt(k_squared(N))).astype(np.int64)


def n_shells(N: int, dealias: str = "cube") -> int:
    """Shells s = 0 .. nint(sqrt(3) K), K the largest retained |k_i|."""
    K = kmax_retained(N, dealias)
    return int(round(math.sqrt(3.0) * K)) + 1


def pressure(state: np.ndarray) -> np.ndarray:
    """Modified pressure of Sec. 2.2 (the divergence of the momentum equation under
    continuity): p_hat = i k.(u.grad u)^ / |k|^2 on the retained modes, 0 at k = 0.

    u.grad u is formed in physical space from the nine gradients i k_j u_i_hat, then
    transformed forward and truncated to the retained cube, the same dealiasing as the
    right-hand side.  Returns one half-spectrum field.
    """
    N = state.shape[-3]
    kx, ky, kz = kgrid(N)
    ik = (1j * kx, 1j * ky, 1j * kz)
    uhat = state[:3]
    u = [to_physical(uhat[i]) for i in range(3)]
    nhat = []
    for i in range(3):
        acc = 0.0
        for j in range(3):
            acc = acc + u[j] * to_physical(ik[j] * uhat[i])
        nhat.append(truncate(to_spectral(acc)))
    k2 = k_squared(N)
    p = 1j * (kx * nhat[0] + ky * nhat[1] + kz * nhat[2]) / np.where(k2 > 0, k2, 1.0)
    p[k2 == 0] = 0.0
    p[~retained_mask(N)] = 0.0
    return p


def spectra(state: np.ndarray, prm: Params) -> dict:
    """Shell spectra and the Table 1 statistics, all from the spectral state.

    E(s)      = sum_{nint|k| = s} 1/2 |u_hat|^2 / N^6           (sums to K)
    E_phi(s)  = sum_{nint|k| = s} 1/2 |phi_hat|^2 / N^6         (sums to <phi^2>/2; reading)
    eps       = 2 nu <S:S> = nu sum (|k|^2 |u_hat|^2 + |k.u_hat|^2) / N^6   (Table 1)
    u_rms = sqrt(2K/3), lambda = u_rms sqrt(15 nu/eps), Re_lambda = lambda u_rms / nu,
    eta = (nu^3/eps)^(1/4), l_o = u_rms^3/eps, T_e = l_o/u_rms (Table 1)
    chi_s     = 2 D_s <grad phi . grad phi> = 2 D_s sum |k|^2 |phi_hat|^2 / N^6   (Eq. (13))
    prod_s    = -2 g_s . <phi u> = -2 sum Re(conj(phi_hat) g_s.u_hat) / N^6     (Eq. (13))
    """
    N = state.shape[-3]
    S = state.shape[0] - 3
    w = half_weights(N)
    mask = retained_mask(N, prm.dealias)
    wm = w * mask
    k2 = k_squared(N)
    kx, ky, kz = kgrid(N)
    inv_n6 = 1.0 / float(N) ** 6
    sh = shell_index(N)
    ns = n_shells(N, prm.dealias)
    eu = 0.5 * wm * np.sum(np.abs(state[:3]) ** 2, axis=0) * inv_n6
    E = np.bincount(sh.ravel(), weights=np.broadcast_to(eu, sh.shape).ravel(), minlength=ns)[:ns]
    Ephi = []
    for s in range(S):
        ep = 0.5 * wm * np.abs(state[3 + s]) ** 2 * inv_n6
        Ephi.append(np.bincount(sh.ravel(), weights=np.broadcast_to(ep, sh.shape).ravel(), minlength=ns)[:ns])
    Kin = float(np.sum(eu))
    kdotu = kx * state[0] + ky * state[1] + kz * state[2]
    eps = prm.nu * float(np.sum(wm * (k2 * np.sum(np.abs(state[:3]) ** 2, axis=0) + np.abs(kdotu) ** 2))) * inv_n6
    out = {"E": E, "E_phi": np.array(Ephi).reshape(S, ns), "K": Kin, "eps": eps}
    urms = math.sqrt(2.0 * Kin / 3.0)
    out["u_rms"] = urms
    if eps > 0:
        lam = urms * math.sqrt(15.0 * prm.nu / eps)
        out.update(lam=lam, Re_lambda=lam * urms / prm.nu, eta=(prm.nu ** 3 / eps) ** 0.25,
                   l_o=urms ** 3 / eps)
        out["T_e"] = out["l_o"] / urms if urms > 0 else float("nan")
    else:
        out.update(lam=float("nan"), Re_lambda=float("nan"), eta=float("nan"), l_o=float("nan"),
                   T_e=float("nan"))
    var, chi, prod = [], [], []
    for s in range(S):
        ph = state[3 + s]
        d = prm.nu / prm.schmidt[s]
        g = prm.mean_grad[s]
        var.append(float(np.sum(wm * np.abs(ph) ** 2)) * inv_n6)
        chi.append(2.0 * d * float(np.sum(wm * k2 * np.abs(ph) ** 2)) * inv_n6)
        gu = g[0] * state[0] + g[1] * state[1] + g[2] * state[2]
        prod.append(-2.0 * float(np.sum(wm * np.real(np.conj(ph) * gu))) * inv_n6)
    out.update(phi_var=np.array(var), chi=np.array(chi), production=np.array(prod))
    return out


def _moments(f: np.ndarray):
    m2 = float(np.mean(f ** 2))
    m3 = float(np.mean(f ** 3))
    m4 = float(np.mean(f ** 4))
    return m2, m3, m4


def physical_stats(state: np.ndarray) -> dict:
    """Skewness and flatness of the VGT diagonal du_i/dx_i (Eqs. (11)-(12)) and of the
    scalar gradient along x2, dphi_s/dx2 (Sec. 2.3), plus max(|u1|+|u2|+|u3|) of Eq. (10).
    The derivatives are spectral (i k_i u_i_hat) and have zero mean, so raw moments are
    the central moments the paper asks for."""
    N = state.shape[-3]
    S = state.shape[0] - 3
    kx, ky, kz = kgrid(N)
    ks = (kx, ky, kz)
    res = {"vgt_m2": [], "vgt_m3": [], "vgt_m4": [], "vgt_skew": [], "vgt_flat": []}
    for i in range(3):
        d = to_physical(1j * ks[i] * state[i])
        m2, m3, m4 = _moments(d)
        res["vgt_m2"].append(m2)
        res["vgt_m3"].append(m3)
        res["vgt_m4"].append(m4)
        res["vgt_skew"].append(m3 / m2 ** 1.5 if m2 > 0 else float("nan"))
        res["vgt_flat"].append(m4 / m2 ** 2 if m2 > 0 else float("nan"))
    res["phi2_skew"], res["phi2_flat"], res["phi2_m2"] = [], [], []
    for s in range(S):
        d = to_physical(1j * ky * state[3 + s])
        m2, m3, m4 = _moments(d)
        res["phi2_m2"].append(m2)
        res["phi2_skew"].append(m3 / m2 ** 1.5 if m2 > 0 else float("nan"))
        res["phi2_flat"].append(m4 / m2 ** 2 if m2 > 0 else float("nan"))
    res["max_abs_u_sum"] = max_abs_sum_velocity(state)
    return res


# --------------------------------------------------------------------------
# Second route to single RHS modes: the truncated Galerkin convolution
# --------------------------------------------------------------------------
def full_spectrum_dict(state: np.ndarray, K: int | None = None):
    """Retained full-spectrum coefficients as arrays over all k in the cube |k_i| <= K
    (default: the 2/3-rule K): values[f, kz+K, ky+K, kx+K], built from the half spectrum by
    u_hat(-k) = conj(u_hat(k))."""
    N = state.shape[-3]
    K = kmax_retained(N) if K is None else K
    M = 2 * K + 1
    F = state.shape[0]
    full = np.zeros((F, M, M, M), dtype=np.complex128)
    r = np.arange(-K, K + 1)
    # kx >= 0 straight from storage
    pos = state[:, :, :, : K + 1][:, r % N][:, :, r % N]
    full[:, :, :, K:] = pos
    # kx < 0: conj of the stored partner at (-kx, -ky, -kz)
    neg = state[:, :, :, 1: K + 1][:, (-r) % N][:, :, (-r) % N]
    full[:, :, :, :K] = np.conj(neg[:, :, :, ::-1])
    return full


def galerkin_mode(state: np.ndarray, prm: Params, k: Sequence[int], full: np.ndarray | None = None) -> np.ndarray:
    """Nonlinear RHS Nl(y) at one retained mode k, straight from its definition as a
    truncated Galerkin convolution (no FFT):

        (u x omega)^_k = N^-3 sum_{p + q = k; p, q retained} u_hat_p x (i q x u_hat_q)
        (u.grad phi)^_k = N^-3 sum_{p + q = k} u_hat_p . (i q) phi_hat_q

    The sums run over the cube |p_i|, |q_i| <= K that bounds the retained set of
    prm.dealias; the state is zero outside its retained set (cube or sphere), so only
    retained p and q contribute.  With either dealiasing every alias of such a product is
    removed, so this equals the pseudo-spectral product on retained modes exactly.
    Returns the vector over fields (3 + S) including forcing and mean-gradient terms.
    """
    N = state.shape[-3]
    K = kmax_retained(N, prm.dealias)
    S = state.shape[0] - 3
    if full is None:
        full = full_spectrum_dict(state, K)
    kx0, ky0, kz0 = (int(v) for v in k)
    # p ranges over the retained cube with q = k - p retained too: a box per axis
    def box(k0):
        lo, hi = max(-K, k0 - K), min(K, k0 + K)
        return np.arange(lo, hi + 1)
    pz, py, px = box(kz0), box(ky0), box(kx0)
    up = full[:3, pz[0] + K:pz[-1] + K + 1, py[0] + K:py[-1] + K + 1, px[0] + K:px[-1] + K + 1]
    # q = k - p runs backwards as p runs forwards along each axis
    uq = full[:, kz0 - pz[-1] + K:kz0 - pz[0] + K + 1,
              ky0 - py[-1] + K:ky0 - py[0] + K + 1,
              kx0 - px[-1] + K:kx0 - px[0] + K + 1][:, ::-1, ::-1, ::-1]
    qz = (kz0 - pz)[:, None, None]
    qy = (ky0 - py)[None, :, None]
    qx = (kx0 - px)[None, None, :]
    # omega_hat_q = i q x u_hat_q
    w1 = 1j * (qy * uq[2] - qz * uq[1])
    w2 = 1j * (qz * uq[0] - qx * uq[2])
    w3 = 1j * (qx * uq[1] - qy * uq[0])
    n3 = float(N) ** 3
    c = np.array([np.sum(up[1] * w3 - up[2] * w2),
                  np.sum(up[2] * w1 - up[0] * w3),
                  np.sum(up[0] * w2 - up[1] * w1)]) / n3
    kvec = np.array([kx0, ky0, kz0], dtype=np.float64)
    k2 = float(kvec @ kvec)
    out = np.zeros(3 + S, dtype=np.complex128)
    if k2 == 0:
        return out
    uk = full[:3, kz0 + K, ky0 + K, kx0 + K]
    out[:3] = c - kvec * (kvec @ c) / k2
    A = forcing_amplitude(state[:3], prm)
    if A != 0.0 and k2 <= prm.k_force ** 2:
        out[:3] += A * uk
    for s in range(S):
        ph = uq[3 + s]
        adv = np.sum((up[0] * 1j * qx + up[1] * 1j * qy + up[2] * 1j * qz) * ph) / n3
        g = prm.mean_grad[s]
        out[3 + s] = -adv - (g[0] * uk[0] + g[1] * uk[1] + g[2] * uk[2])
    return out


def mode_value(state: np.ndarray, k: Sequence[int]) -> np.ndarray:
    """Coefficient vector at wavevector k (any sign of kx) read from the half spectrum."""
    N = state.shape[-3]
    kx0, ky0, kz0 = (int(v) for v in k)
    if kx0 >= 0:
        return state[:, kz0 % N, ky0 % N, kx0]
    return np.conj(state[:, (-kz0) % N, (-ky0) % N, -kx0])
