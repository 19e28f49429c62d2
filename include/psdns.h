/*
 * psdns — pseudo-spectral DNS right-hand side and RK4 stepping on AMD MI355X (gfx950).
 *
 * Solves, on the periodic box [0, 2pi)^3 with N^3 points, the incompressible
 * Navier-Stokes equations with a forcing coefficient (Akhavan-Safaei &
 * Zayernouri, arXiv:2012.04838, Sec. 2.1, Eq. (1)) and S passive scalars with a
 * uniform mean gradient (Eq. (3)), in the Fourier pseudo-spectral form of
 * Sec. 2.2 (Eqs. (5)-(8)):
 *
 *   du_hat/dt   = P(k) (u x omega)^  + A 1_band u_hat  - nu |k|^2 u_hat
 *   dphi_hat/dt = -(u . grad phi)^   - g . u_hat       - (nu/Sc) |k|^2 phi_hat
 *
 * with P(k) = I - k k^T/|k|^2 the projection of Eq. (7), products formed in
 * physical space, 2/3-rule truncation |k_i| <= K = (N-1)/3 (or the paper's phase shift
 * with spherical truncation, PSDNS_DEALIAS_PHASE_SPHERE), A = P/(2 E_f)
 * (constant power P injected into the band 0 < |k| <= k_force), and the
 * classical RK4 of Sec. 2.2 applied with the viscous/diffusive integrating
 * factor.
 *
 * Conventions.
 *  - Spectral coefficients use the unnormalised forward transform of Eq. (5):
 *    phi_hat(k) = sum_x phi(x) exp(-i k.x), x_j = 2 pi j / N.
 *  - Canonical layout (get/set_state): per slot, [field][kz: N][ky: N][kx: N/2+1]
 *    interleaved complex, kx fastest; index i stands for wavenumber i (i <= N/2)
 *    or i - N.  Fields are u1, u2, u3, phi_1 .. phi_S.  Element type is
 *    float2 (precision 32) or double2 (precision 64).
 *  - The internal state layout is compact (retained modes only) and opaque;
 *    its size is psdns_state_bytes().  Slots (independent realizations) are
 *    stored back to back.
 *
 * Ownership.  The caller owns every buffer passed in (state, workspace, outputs)
 * and the HIP stream; all of them are device pointers unless stated.  A plan
 * owns only its small twiddle and parameter tables (psdns_plan_device_bytes), so
 * state + workspace + plan tables is the whole device footprint of a plan.
 *
 * Workspace records.  Besides transform buffers, a workspace carries per-slot records
 * that persist across calls: simulated time, step count and flags (psdns_step_info) and
 * the stochastic-forcing vectors.  The library cannot tell a fresh workspace from one it
 * has seen, so the caller clears the records with psdns_clear_step_info before the first
 * use of a workspace with a plan (and whenever its contents are unknown, e.g. memory
 * reused from another allocation).  psdns_init_field clears the record of its slot.
 *
 * Errors.  Every call returns a psdns_status; nothing is thrown across the ABI.
 * Argument errors are detected before anything is launched.  Launches are
 * asynchronous on the given stream (NULL = default stream); numerical trouble
 * (non-finite values, CFL > 1) is recorded in per-slot device flags read by
 * psdns_read_step_info.  psdns_last_error() returns a thread-local message
 * describing the last failure.
 */
#ifndef PSDNS_H
#define PSDNS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PSDNS_MAX_SCALARS 4

/* Device flag bits (psdns_step_info.flags). */
#define PSDNS_FLAG_NONFINITE 1 /* a velocity value was NaN or Inf at the start of a step */
#define PSDNS_FLAG_CFL 2       /* Eq. (10) CFL number exceeded 1 for the step size used */

typedef struct psdns_plan psdns_plan;

typedef enum {
  PSDNS_OK = 0,
  PSDNS_E_INVAL = -1,       /* invalid argument; nothing launched */
  PSDNS_E_NOMEM = -2,       /* allocation of plan-owned tables failed */
  PSDNS_E_HIP = -3,         /* a HIP runtime call failed */
  PSDNS_E_UNSUPPORTED = -4  /* valid request this library does not implement */
} psdns_status;

/* Dealiasing of the quadratic products (Sec. 2.3).
 * TWO_THIRDS:   the 2/3 rule: every product truncated to the cube |k_i| <= K = (N-1)/3.
 * PHASE_SPHERE: the paper's scheme: every product is the mean of its values on the grid and
 *               on the grid shifted by half a cell along each axis (inputs multiplied by
 *               exp(i pi (kx+ky+kz)/N), products by its conjugate), truncated to the sphere
 *               9 |k|^2 < 2 N^2 (|k| < sqrt(2) N / 3, Sec. 3.1); K is then the largest integer
 *               with 9 K^2 < 2 N^2 and the state holds the sphere inside the cube |k_i| <= K.
 *               Each right-hand side costs two evaluations of the products. */
#define PSDNS_DEALIAS_TWO_THIRDS 0
#define PSDNS_DEALIAS_PHASE_SPHERE 1

/* Plan geometry, fixed for the life of a plan.  Grids that are powers of two run the tuned
 * step kernels: with the 2/3 rule in every schedule, with PHASE_SPHERE in one schedule
 * (their phase-shift stage).  Any other even n whose prime factors are 2, 3, 5, 7, 11 and
 * 13 (the paper's n = 520 = 2^3 5 13, Sec. 3.1 and Table 2) runs general kernels built on
 * mixed-radix transforms (one schedule).  Plans with PHASE_SPHERE, and plans on the
 * general kernels, have no psdns_pressure (PSDNS_E_UNSUPPORTED). */
typedef struct {
  int32_t n;         /* points per axis: even, 8 <= n <= 1024, prime factors in {2, 3, 5, 7, 11, 13} */
  int32_t n_scalars; /* S, 0 <= S <= PSDNS_MAX_SCALARS */
  int32_t precision; /* 32 or 64: storage, transforms and products; reductions are FP64 */
  int32_t batch;     /* number of independent realizations (slots), >= 1 */
  int32_t dealias;   /* PSDNS_DEALIAS_TWO_THIRDS (0) or PSDNS_DEALIAS_PHASE_SPHERE */
} psdns_plan_params;

/* Forcing of the band 0 < |k| <= k_force (Eq. (1) term A U, Sec. 2.3).
 * POWER: constant power, A = P / (2 E_f) evaluated at every RK stage from the stage input.
 * HOLD:  the paper's deterministic scheme, evaluated once after the last stage of every
 *        step: the band modes of u are scaled by sqrt(hold_energy / E_f), which keeps the
 *        band energy at hold_energy (no forcing term inside the stages). */
/* STOCHASTIC: the stochastic scheme the paper names as an option (Sec. 2.3, after
 *        Eswaran & Pope).  Every band mode k (k_force <= PSDNS_STOCHASTIC_KF_MAX) carries a
 *        complex 3-vector b(k), an Ornstein-Uhlenbeck process advanced once per step with
 *        that step's dt:  b <- a b + stoch_sigma sqrt(1 - a^2) xi,  a = exp(-dt / stoch_tl),
 *        xi with independent standard normal real and imaginary parts, so each part has
 *        variance stoch_sigma^2 in the stationary state.  b holds normalised (physical)
 *        Fourier coefficients: the term N^3 P(k) b (the solenoidal part, in the
 *        unnormalised state of Eq. (5)) is added to the velocity right-hand side in every
 *        stage of the step.  On the plane kx = 0, b(0,-ky,-kz) = conj b(0,ky,kz) (a real
 *        forcing).
 *        Normals: Box-Muller, sqrt(-2 ln(1-u1)) cos(2 pi u2), on SplitMix64(stoch_seed)
 *        uniforms (top 53 bits) number 2q and 2q+1, q = ((n C + i) 3 + c) 2 + p for step n
 *        (1, 2, ... counted by the step record), candidate i = kx + (kf+1)((ky+kf) +
 *        (2kf+1)(kz+kf)) of C = (kf+1)(2kf+1)^2, component c, real/imaginary part p;
 *        kf = floor(k_force), capped at k_max.  b lives in the workspace: it is zero after
 *        psdns_clear_step_info, psdns_clear_slot_info and psdns_init_field of the slot. */
/* ALVELIUS: the other stochastic scheme the paper names (Sec. 2.3, after Alvelius): a force
 *        drawn afresh every step from y_n and held over the four stages of that step, zero
 *        outside the band (k_force below PSDNS_STOCHASTIC_KF_MAX + 1).  At band mode k
 *          f = F (g_A e^{i th1} e1 + g_B e^{i th2} e2),  e1 = k x z_hat / |k x z_hat| (x_hat
 *        for k along z), e2 = k x e1 / |k|, g_A = sin 2 phi, g_B = cos 2 phi, th2 = th1 + psi,
 *        phi = 2 pi u_{2q}, psi = 2 pi u_{2q+1} from the SplitMix64(stoch_seed) uniforms (top
 *        53 bits), q = n C + i (step n and candidate i of C as for STOCHASTIC), and
 *        th1 = atan2(-a, b) (0 if a = b = 0) with xi_j = u_hat . e_j,
 *          a = g_A Re xi1 + g_B (Re xi2 cos psi + Im xi2 sin psi),
 *          b = g_A Im xi1 + g_B (Im xi2 cos psi - Re xi2 sin psi),
 *        so that Re(conj(u_hat) . f) = 0: the force does no work on the velocity of its step.
 *        F = N^3 sqrt(2 power / (dt W)), W the band modes counted twice for kx > 0 and once
 *        for kx = 0, so that the force-force term injects `power`:
 *        (dt / 2) sum w |f|^2 / N^6 = power.  On kx = 0, f(0,-ky,-kz) = conj f(0,ky,kz). */
#define PSDNS_FORCING_POWER 0
#define PSDNS_FORCING_HOLD 1
#define PSDNS_FORCING_STOCHASTIC 2
#define PSDNS_FORCING_ALVELIUS 3
#define PSDNS_STOCHASTIC_KF_MAX 4

/* Time integrator (Sec. 2.2-2.3).
 * IF:       classical RK4 in the frame of the viscous/diffusive integrating factor
 *           exp(-D |k|^2 t) (Lawson): the linear terms are integrated exactly.
 * EXPLICIT: the paper's classical RK4 with the viscous and diffusive terms evaluated in
 *           every stage like the others (stable while D |k|^2 dt stays inside the RK4
 *           stability region, about 2.78). */
#define PSDNS_INTEGRATOR_IF 0
#define PSDNS_INTEGRATOR_EXPLICIT 1

/* Physical parameters of one slot (Sec. 2.1, Sec. 2.3, Table 2). */
typedef struct {
  double nu;                              /* kinematic viscosity, >= 0 */
  double power;                           /* forcing power P >= 0 (POWER, ALVELIUS); 0 gives decaying turbulence */
  double k_force;                         /* forced band 0 < |k| <= k_force */
  double schmidt[PSDNS_MAX_SCALARS];      /* Sc_s = nu / D_s, > 0 */
  double mean_grad[PSDNS_MAX_SCALARS][3]; /* g_s = grad <Phi_s>; Eq. (3) has (0, beta, 0) */
  int32_t forcing;                        /* PSDNS_FORCING_POWER (default 0), _HOLD, _STOCHASTIC or _ALVELIUS */
  int32_t integrator;                     /* PSDNS_INTEGRATOR_IF (default 0) or PSDNS_INTEGRATOR_EXPLICIT */
  double hold_energy;                     /* HOLD: target band energy E_f > 0 */
  double stoch_sigma;                     /* STOCHASTIC: stationary deviation of each part of b, >= 0 */
  double stoch_tl;                        /* STOCHASTIC: correlation time T_L > 0 */
  uint64_t stoch_seed;                    /* STOCHASTIC, ALVELIUS: SplitMix64 seed of the random draws */
} psdns_slot_params;

/* Per-slot stepping record (host copy). */
typedef struct {
  double t;        /* simulated time accumulated by psdns_step */
  double dt;       /* step size of the last step */
  double max_u;    /* max over grid points of |u1|+|u2|+|u3| at the start of the last step */
  int64_t steps;   /* steps taken */
  int32_t flags;   /* PSDNS_FLAG_* */
  int32_t active;  /* slot is stepped */
} psdns_step_info;

/* Sizes and layout facts of a plan. */
typedef struct {
  int32_t n, k_max, m, kx_count, kx_pitch, n_scalars, precision, batch;
  int32_t n_shells;        /* shells s = 0 .. n_shells-1 reported by psdns_spectra */
  int32_t spectra_doubles; /* doubles per slot written by psdns_spectra */
  int64_t state_bytes, workspace_bytes;
  int32_t elems_col, elems_x; /* FFT elements per thread of the column and x passes (schedule in use) */
  int32_t n_schedules;        /* step schedules compiled for this size (psdns_set_schedule) */
  int32_t schedule;           /* schedule in use, or -1 when the passes run in different ones */
  int64_t plan_bytes;         /* device bytes of the plan's own tables (psdns_plan_device_bytes) */
  int32_t dealias;            /* PSDNS_DEALIAS_* of the plan */
  int32_t general;            /* 1 when the plan steps on the general (mixed-radix) kernels */
  int32_t pass_schedules[5];  /* schedule of each pass, PSDNS_PASS_* order */
} psdns_plan_info;

/* Bytes of the compact spectral state y for all slots (caller allocates). 0 on invalid params. */
size_t psdns_state_bytes(const psdns_plan_params* p);
/* Bytes of the workspace needed by rhs/step/init/spectra (caller allocates). 0 on invalid params. */
size_t psdns_workspace_bytes(const psdns_plan_params* p);

/* Device bytes a plan allocates for its own twiddle and slot tables (rounded up to 256-byte
 * granules); with the state and the workspace, the whole device footprint.  0 on invalid params. */
size_t psdns_plan_device_bytes(const psdns_plan_params* p);

/* Create a plan (host metadata plus twiddle and slot tables on the current device).
 * All slots start active with nu = 0, P = 0, k_force = 2, Sc = 1, g = 0. */
psdns_status psdns_plan_create(const psdns_plan_params* p, psdns_plan** out);
psdns_status psdns_plan_destroy(psdns_plan* plan);
psdns_status psdns_plan_get_info(const psdns_plan* plan, psdns_plan_info* out);

/* Set the physical parameters of one slot and whether it is stepped (active != 0).
 * Synchronous upload; call between steps, not while work on the slot is queued. */
psdns_status psdns_set_slot(psdns_plan* plan, int32_t slot, const psdns_slot_params* prm, int32_t active);

/* Rogallo-type random solenoidal field (Sec. 2.3) with the configured spectrum
 * E(k) ~ k^4 exp(-2 (k/k_peak)^2), phases from SplitMix64(seed) keyed by the
 * canonical linear index, scaled to kinetic energy 1/2<u.u> = kinetic_energy;
 * scalars start at zero (Sec. 2.3).  Writes one slot of `state`; uses `ws`, and clears the
 * slot's step record and stochastic-forcing vector there (a new realization starts at t = 0). */
psdns_status psdns_init_field(psdns_plan* plan, void* state, void* ws, int32_t slot, uint64_t seed,
                              double k_peak, double kinetic_energy, void* hip_stream);

/* The same field from another initial spectrum shape (Sec. 2.3):
 *   PSDNS_SPECTRUM_CONFIG  E(k) ~ k^4 exp(-2 (k/k_param)^2)              (as psdns_init_field)
 *   PSDNS_SPECTRUM_PAPER   the paper's spectrum (after Lamorgese et al.) with k_F = k_param:
 *                          E(k) = (u_rms^2/k_F) (k/k_F)^2 for k <= k_F, (u_rms^2/k_F) (k/k_F)^(-5/3)
 *                          beyond; the shape only matters, the field is scaled to kinetic_energy. */
#define PSDNS_SPECTRUM_CONFIG 0
#define PSDNS_SPECTRUM_PAPER 1
psdns_status psdns_init_field_spectrum(psdns_plan* plan, void* state, void* ws, int32_t slot, uint64_t seed,
                                       int32_t spectrum, double k_param, double kinetic_energy, void* hip_stream);

/* Set the scalars of one slot to zero and keep its velocity: the paper's way of starting
 * the scalar on a developed velocity field (phi_0 = 0, Sec. 2.3).  Asynchronous. */
psdns_status psdns_zero_scalars(psdns_plan* plan, void* state, int32_t slot, void* hip_stream);

/* Full right-hand side dy/dt (Eqs. (7)-(8), including the viscous and diffusive
 * terms) of every active slot of `state`, written to `out` (state layout).
 * `out` must not alias `state`. */
psdns_status psdns_rhs(psdns_plan* plan, const void* state, void* out, void* ws, void* hip_stream);

/* Advance every active slot by nsteps RK4 steps with the viscous/diffusive
 * integrating factor.  dt > 0: fixed step; dt < 0: each step uses
 * dt = (-dt) * (2 pi / N) / max(|u1|+|u2|+|u3|), i.e. Eq. (10) with CFL = -dt,
 * evaluated from the state at the start of the step.  In place on `state`. */
psdns_status psdns_step(psdns_plan* plan, void* state, void* ws, double dt, int32_t nsteps,
                        void* hip_stream);

/* Allocation-free stepping, for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc).  The same steps as
 * psdns_step on a workspace cleared with psdns_clear_step_info, but the workspace is a
 * static device array of PSDNS_NOALLOC_MAX_WORKSPACE_BYTES inside the library (one per
 * GPU, held until the process ends), so the call allocates nothing and takes no `ws`;
 * the caller still passes the state (and, optionally, the record output).  Steps are
 * launched directly (no graph of the plan's own).
 *  - PSDNS_E_INVAL (nothing launched) if psdns_workspace_bytes of the plan exceeds
 *    PSDNS_NOALLOC_MAX_WORKSPACE_BYTES, if the current device is not the plan's, or for
 *    the arguments psdns_step rejects.
 *  - Every call starts the step records and stochastic-forcing vectors of all slots from
 *    zero (the array keeps the last call's contents otherwise).  If info_out is not NULL
 *    it is a device buffer of batch psdns_step_info records that receives the records of
 *    this call after its last step (stream-ordered; psdns_read_step_info does not see
 *    them).
 *  - All calls on one GPU share the array: calls that may overlap in time on one GPU
 *    (other streams, other threads or plans) race and must be ordered by the caller. */
#define PSDNS_NOALLOC_MAX_WORKSPACE_BYTES (256ull << 20)
psdns_status psdns_step_noalloc(psdns_plan* plan, void* state, double dt, int32_t nsteps, psdns_step_info* info_out,
                                void* hip_stream);

/* Step through a captured HIP graph (off by default).  When enabled, psdns_step on a
 * non-default stream captures the launches of one RK4 step the first time it sees a given
 * (state, ws, dt) and then replays that graph once per step; a different state, workspace
 * or dt re-captures.  Slot parameters and active flags are read by the kernels at replay
 * time, so psdns_set_slot needs no re-capture, except that switching slots into or out of
 * PSDNS_FORCING_HOLD changes the step structure and re-captures.  Steps on the default (NULL) stream are
 * launched directly.  Timing events are not recorded for replayed steps. */
psdns_status psdns_set_graph(psdns_plan* plan, int32_t enable);

/* Step schedules.  The step kernels of a size are compiled in several tile and radix
 * schedules: elements per thread of the column passes (the radix of their Stockham
 * stages), kx columns per column block, the same two for the z-update pass, and lines
 * per x-pass block.  All schedules compute the same transforms of Eq. (5) and the same
 * right-hand side; only the association order of the butterflies differs.  Schedule 0
 * is the default.  Choosing one changes no layout or buffer size. */
typedef struct {
  int32_t index;
  int32_t elems_col;   /* elements per thread of the z and y passes */
  int32_t col_width;   /* kx columns per block of the z and y passes */
  int32_t elems_fused; /* elements per thread of the z-forward/update pass */
  int32_t fused_width; /* kx columns per block of the z-forward/update pass */
  int32_t elems_x;     /* elements per lane of the x pass */
  int32_t x_lines;     /* (z, y) lines per x-pass block */
} psdns_schedule_info;
psdns_status psdns_get_schedule_info(const psdns_plan* plan, int32_t index, psdns_schedule_info* out);
/* Select the schedule used by rhs and step (a captured step graph is dropped and
 * re-captured on the next graph step).  PSDNS_E_INVAL for an index outside
 * [0, n_schedules). */
psdns_status psdns_set_schedule(psdns_plan* plan, int32_t index);
/* Autotuner: times `reps` RK stages of every active slot of `state` with each schedule
 * (after one untimed trial), selects the fastest and returns the mean milliseconds per
 * stage in host array ms_out[n_schedules] (may be NULL) and its index in *best (may be
 * NULL).  A trial is the stage of a multi-step call that every step repeats (forcing
 * amplitude, y inverse, x pass, y forward, z forward with the update and the next
 * stage's z inverse); it writes only workspace buffers that a step rebuilds (the
 * accumulator, the stage input, the transform buffers) and leaves `state` and the step
 * records untouched.  Synchronises the stream. */
psdns_status psdns_tune(psdns_plan* plan, const void* state, void* ws, int32_t reps, double* ms_out,
                        int32_t* best, void* hip_stream);

/* The passes of one right-hand-side evaluation (Sec. 2.2: the inverse transforms of Eq. (5)
 * axis by axis, the products, the forward transforms and the update).  Every schedule reads
 * and writes the same buffers in the same layouts, so each pass may run in its own. */
#define PSDNS_PASS_Z_INVERSE 0 /* z inverse of the stage input (first stage of a call)          */
#define PSDNS_PASS_Y_INVERSE 1
#define PSDNS_PASS_X 2         /* x inverse, the products and the CFL maximum, x forward        */
#define PSDNS_PASS_Y_FORWARD 3
#define PSDNS_PASS_Z_FORWARD 4 /* z forward, projection, forcing, stage update, next z inverse */
#define PSDNS_NUM_PASSES 5
/* Select the schedule of each pass: sched[PSDNS_NUM_PASSES] (host array), each in
 * [0, n_schedules), else PSDNS_E_INVAL.  psdns_set_schedule(i) sets every pass to i.  The
 * results are those of any schedule (the same transforms; only the association order of the
 * butterflies differs).  A captured step graph is dropped and re-captured. */
psdns_status psdns_set_pass_schedules(psdns_plan* plan, const int32_t* sched);
/* Run this plan on the general (mixed-radix) kernels even where the tuned power-of-two
 * kernels apply (a power-of-two n, either dealiasing): both families read and write the same
 * state and workspace layouts and compute the same right-hand side (Sec. 2.2, and the
 * phase-shift dealiasing of Sec. 2.3), so the one cross-checks the other on one grid, up to
 * the largest lines (n = 1024).  From then on the
 * plan reports general = 1, has one schedule, and psdns_pressure returns
 * PSDNS_E_UNSUPPORTED.  No-op on a plan that already runs the general kernels; a captured
 * step graph is dropped.  There is no way back. */
psdns_status psdns_use_general_kernels(psdns_plan* plan);
/* Autotuner per pass: times the passes of `reps` RK stages with each schedule (the trial of
 * psdns_tune, and the standalone z inverse) with an event pair around every kernel and
 * selects for each pass the lowest-index schedule within 1% of its fastest (schedules that
 * coincide at a size then resolve to the same choice on every run).  Returns the mean
 * milliseconds of every pass and schedule in host array ms_out[n_schedules *
 * PSDNS_NUM_PASSES] (schedule-major; may be NULL) and the selection in
 * best[PSDNS_NUM_PASSES] (may be NULL).  Leaves `state` and the step records untouched.
 * Synchronises the stream. */
psdns_status psdns_tune_passes(psdns_plan* plan, const void* state, void* ws, int32_t reps, double* ms_out,
                               int32_t* best, void* hip_stream);

/* Copy the per-slot stepping records to host memory `out[batch]` (synchronises the stream). */
psdns_status psdns_read_step_info(psdns_plan* plan, const void* ws, psdns_step_info* out, void* hip_stream);
/* Reset t, steps, flags and the stochastic-forcing vectors of every slot (asynchronous;
 * a kernel, so it may be recorded in a captured graph).  Required before the first use of
 * a workspace with a plan. */
psdns_status psdns_clear_step_info(psdns_plan* plan, void* ws, void* hip_stream);
/* The same for one slot only, e.g. when a slot is reused for a new run loaded with
 * psdns_set_state.  PSDNS_E_INVAL for a slot outside [0, batch). */
psdns_status psdns_clear_slot_info(psdns_plan* plan, void* ws, int32_t slot, void* hip_stream);

/* Convert one slot between the compact state and the canonical layout (device buffers).
 * get: modes outside the retained cube are written as zero.  set: they are ignored. */
psdns_status psdns_get_state(psdns_plan* plan, const void* state, int32_t slot, void* canonical_out,
                             void* hip_stream);
psdns_status psdns_set_state(psdns_plan* plan, void* state, int32_t slot, const void* canonical_in,
                             void* hip_stream);

/* Stepping with statistics time series (the records the paper writes at a user-defined
 * interval, Sec. 2.3): advances every active slot by nsteps steps exactly as psdns_step
 * (same dt rule), and after every `every` steps appends one record block to the device
 * buffer `records`: batch doubles of simulated time t per slot, then batch spectra
 * records (psdns_spectra layout, `flags` as there).  floor(nsteps / every) blocks of
 * batch * (1 + spectra_doubles) doubles are written; steps beyond the last full interval
 * run without a record.  Asynchronous on the stream. */
psdns_status psdns_run(psdns_plan* plan, void* state, void* ws, double dt, int32_t nsteps, int32_t every,
                       double* records, int32_t flags, void* hip_stream);

/* Modified pressure (Sec. 2.2): p_hat(k) = i k.(u.grad u)^(k) / |k|^2 on the retained
 * modes, p_hat(0) = 0, in the transform convention of Eq. (5) (unnormalised like the
 * state).  Evaluated as -(|u|^2/2)^ - i k.(u x omega)^ / |k|^2, which equals it because
 * u.grad u = grad(|u|^2/2) - u x omega and both products are dealiased by the same
 * truncation.  `canonical_out` (device) receives batch * N * N * (N/2+1) complex values:
 * per slot one field in the canonical layout, modes outside the retained cube and
 * inactive slots zero.  Uses the workspace transform buffers and accumulator (which
 * holds nothing between steps); asynchronous on the stream. */
psdns_status psdns_pressure(psdns_plan* plan, const void* state, void* ws, void* canonical_out, void* hip_stream);

/* Spectra and statistics of every slot (Table 1; Eqs. (11)-(13)), accumulated in FP64 with
 * a fixed summation order (bitwise reproducible).  `out` is a device buffer of
 * batch * psdns_plan_info.spectra_doubles doubles; with ns = n_shells and S scalars the
 * record of one slot is
 *   [0, ns)                     E(s) = sum over nint|k| = s of |u_hat|^2/2 / N^6 (sums to K)
 *   [ns*(1+j), ns*(2+j))        E_phi_j(s), same with phi_j (sums to <phi_j^2>/2)
 *   b = ns*(1+S): b+0 K = <u.u>/2, b+1 eps = 2 nu <S:S>, b+2 u_rms = sqrt(2K/3),
 *                 b+3 lambda = u_rms sqrt(15 nu/eps), b+4 Re_lambda = lambda u_rms/nu,
 *                 b+5 eta = (nu^3/eps)^(1/4), b+6 l_o = u_rms^3/eps, b+7 T_e = l_o/u_rms
 *   b+8+4j:       <phi_j^2>, chi_j = 2 D_j <|grad phi_j|^2>, production -2 g_j.<phi_j u>,
 *                 production/chi_j   (Eq. (13))
 *   p = b+8+4S:   p+0..2 <(du_i/dx_i)^2>, p+3..5 <(du_i/dx_i)^3>, p+6..8 <(du_i/dx_i)^4>,
 *                 p+9..11 skewness S_{u_i,i} (Eq. (11)), p+12..14 flatness K_{u_i,i} (Eq. (12)),
 *                 p+15 max(|u1|+|u2|+|u3|) (Eq. (10)),
 *                 p+16+3j <(dphi_j/dx2)^2>, skewness, flatness of dphi_j/dx2
 * flags: PSDNS_SPECTRA_SHELLS fills [0, p); PSDNS_SPECTRA_MOMENTS fills [p, end) (three
 * extra inverse transforms per velocity component and scalar); other entries are NaN.
 * Uses the workspace transform buffers; asynchronous on the stream. */
#define PSDNS_SPECTRA_SHELLS 1
#define PSDNS_SPECTRA_MOMENTS 2
psdns_status psdns_spectra(psdns_plan* plan, const void* state, void* ws, double* out, int32_t flags,
                           void* hip_stream);

/* Per-kernel timing with HIP events on the launch stream (off by default).  Entries are the
 * step kernels by name, "aux" (initial field, conversions, spectra, pressure) and "step":
 * one whole RK4 step of psdns_step, around each graph replay or around the launches of an
 * eager step (its kernels are timed inside it).  median_ms and min_ms are over the
 * launches since the previous psdns_get_timing. */
typedef struct {
  char name[32];
  int32_t launches;
  double total_ms;
  double median_ms;
  double min_ms;
} psdns_kernel_timing;
psdns_status psdns_set_timing(psdns_plan* plan, int32_t enable);
/* Synchronises the recorded events, accumulates and clears them. Fills up to max entries. */
psdns_status psdns_get_timing(psdns_plan* plan, psdns_kernel_timing* out, int32_t max, int32_t* count);

/* Streaming device-to-device copy of `bytes` with `blocks` blocks of 256 threads, each
 * thread keeping four 16-byte loads in flight (grid-stride).  Not part of the method: the
 * achievable HBM bandwidth that the transform passes are compared with.  `bytes` and both
 * pointers must be multiples of 16 and the buffers must not overlap (else PSDNS_E_INVAL).
 * Asynchronous on the stream. */
psdns_status psdns_stream_copy(void* dst, const void* src, size_t bytes, int32_t blocks, void* hip_stream);

/* Thread-local description of the last error (never NULL). */
const char* psdns_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PSDNS_H */
