// Shared host/device structures of the pseudo-spectral DNS library.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/psdns.h"

namespace psdns {

constexpr int kMaxScalars = PSDNS_MAX_SCALARS;

// Sizes of one plan.  Spectral arrays keep only the retained cube
// |k_i| <= K = (N-1)/3 (the 2/3 rule): ky and kz use the compact index
// c in [0, M), M = 2K+1 (c <= K means k = c, otherwise k = c - M), kx runs
// over 0..K and rows are padded to PX = K+1 rounded up to 16 entries.
struct Geom {
  int N, K, M, KX, PX;
  int S;                  // passive scalars
  int F;                  // spectral fields: 3 + S
  int FA;                 // fields after the z pass: 5 + 2S
  int FB;                 // fields after the y pass: 6 + 3S
  int batch;              // realizations (slots)
  long long st_field;     // complex entries per field in the compact state: M*M*PX
  long long a_field;      // per field after the z pass: N*M*PX   (rows at a_row(z, ky_c))
  long long b_field;      // per field after the y pass: N*N*PX   ([z][y][kx])
  int nblk_x;             // x-pass blocks per slot (partial maxima)
  int ns;                 // spectral shells 0 .. ns-1, ns = nint(sqrt(3) K) + 1
  int sphere;             // retained set: 0 the cube |k_i| <= K (2/3 rule); 1 the sphere
                          // 9 |k|^2 < 2 N^2 inside that cube (phase-shift dealiasing)
};

// Whether wavevector (kx, ky, kz), with |k_i| <= K, is retained.
__host__ __device__ inline bool retained(const Geom& g, int kx, int ky, int kz) {
  return !g.sphere || 9LL * ((long long)kx * kx + (long long)ky * ky + (long long)kz * kz) < 2LL * g.N * g.N;
}

// Layout of the plan's root table (plan precision, interleaved complex):
//   [0, N)               w_N^m = exp(-2 pi i m / N)
//   [N + kRootOff(R), +R) exp(-2 pi i m / R) for the odd radices R = 3, 5, 7, 11, 13
//   [N + kShiftOff, +N/2+1) exp(i pi k / N), k = 0 .. N/2 (the half-cell grid shift)
constexpr int kOddRadices[5] = {3, 5, 7, 11, 13};
__host__ __device__ constexpr int kRootOff(int R) {
  return R == 3 ? 0 : R == 5 ? 3 : R == 7 ? 8 : R == 11 ? 15 : 26;
}
constexpr int kShiftOff = 39;
__host__ __device__ constexpr long long root_table_entries(int N) { return (long long)N + kShiftOff + N / 2 + 1; }

// Row placement: row (kz_c, ky_c) of a state field and row (z, ky_c) of a field
// after the z pass both sit at (z M + ky_c) PX, so the two share their strides.
__host__ __device__ inline long long st_row(int kzc, int kyc, int M, int PX) {
  return ((long long)kzc * M + kyc) * PX;
}
__host__ __device__ inline long long a_row(int z, int kyc, int M, int PX) { return ((long long)z * M + kyc) * PX; }

// Static per-slot parameters, uploaded by psdns_set_slot.
struct SlotDev {
  double nu;
  double power;
  double kf2;                       // k_force^2
  double diff[3 + kMaxScalars];     // diffusivity of each spectral field
  double g[kMaxScalars][3];         // mean scalar gradients
  int active;
  int forcing;                      // PSDNS_FORCING_POWER, _HOLD, _STOCHASTIC or _ALVELIUS
  double hold;                      // target band energy of PSDNS_FORCING_HOLD
  int integrator;                   // PSDNS_INTEGRATOR_IF or PSDNS_INTEGRATOR_EXPLICIT
  int pad_;
  double sigma;                     // PSDNS_FORCING_STOCHASTIC: stationary deviation per part
  double tl;                        // PSDNS_FORCING_STOCHASTIC: correlation time
  unsigned long long seed;          // PSDNS_FORCING_STOCHASTIC and _ALVELIUS: SplitMix64 seed
};

// Band table of the stochastic forcings: per slot, kStochCand candidates of 12 FP64 (the
// Ornstein-Uhlenbeck vector b, or unused for Alvelius' force, then the forcing term, 3
// complex each), candidate
// i = kx + (kf+1)((ky+kf) + (2kf+1)(kz+kf)) for the slot's kf.
constexpr int kStochKfMax = PSDNS_STOCHASTIC_KF_MAX;
constexpr int kStochCand = (kStochKfMax + 1) * (2 * kStochKfMax + 1) * (2 * kStochKfMax + 1);

// Per-slot values written on the device while stepping (part of the workspace).
struct DynDev {
  double dt;         // step in use
  double A;          // forcing amplitude of the current stage input
  double max_u;      // max |u1|+|u2|+|u3| at the start of the last step
  double t;          // simulated time accumulated by psdns_step
  double scratch;    // reduction result used by init_field
  long long steps;   // steps taken by psdns_step
  int flags;         // PSDNS_FLAG_* bits, sticky until psdns_clear_step_info / psdns_clear_slot_info
  int pad_;
  // running max of |u1|+|u2|+|u3| over the grid during the stage-0 x pass, as the bits
  // of a non-negative double: their unsigned order is the numeric order (NaN above
  // everything), so an integer atomic max gives the exact, order-independent result
  unsigned long long umax;
};

enum KernelId {
  KID_FORCE = 0,
  KID_ZINV,
  KID_YINV,
  KID_XPASS,
  KID_DT,
  KID_YFWD,
  KID_ZFWD,
  KID_AUX,
  KID_ZFWDI,
  KID_STEP,  // one whole RK4 step (a graph replay or the launches of an eager step)
  KID_COUNT
};

// rhs_stage flags
constexpr int kStageZinv = 1;  // run the standalone z inverse of the stage input first
constexpr int kStageFuse = 2;  // the z-forward/update pass also inverts the next stage input
constexpr int kStagePrologue = 4;  // only the standalone z inverse (before replaying fused steps)

// Optional per-launch timing with HIP events (see psdns_set_timing).
struct Timer {
  virtual void begin(int kid, hipStream_t s) = 0;
  virtual void end(int kid, hipStream_t s) = 0;
  virtual ~Timer() {}
};

// The passes of a right-hand-side evaluation, each of which may run in its own schedule
// (index order of psdns_set_pass_schedules).
constexpr int kPassZInverse = 0;  // z inverse of the stage input (first stage of a call)
constexpr int kPassYInverse = 1;
constexpr int kPassX = 2;         // x inverse, products, x forward
constexpr int kPassYForward = 3;
constexpr int kPassZForward = 4;  // z forward, projection, forcing, stage update (and next z inverse)
constexpr int kNumPasses = 5;

struct Ctx {
  Geom g;
  const void* tw;          // w_N^m = exp(-2 pi i m/N), m = 0..N-1, in the plan precision
  const SlotDev* slots;    // device table [batch]
  DynDev* dyn;             // device [batch]
  double* fband;           // device [batch][kStochCand][12] FP64 (stochastic forcing: b, P(k) b)
  void* abuf;              // [batch][FA][N][M][PX]
  void* akeep;             // phase-shift dealiasing: forward product of the unshifted evaluation [batch][F][N][M][PX]
  void* bbuf;              // [batch][FB][N][N][PX]
  void* ystage;            // [batch][F][M][M][PX]
  void* acc;               // [batch][F][M][M][PX]
  double* part;            // x-pass partial maxima [batch][nblk_x] and reduction scratch
  long long part_len;      // doubles available at part
  double* stat;            // statistics partials (shell sums, moment partials)
  int nbm;                 // blocks of the moments kernels per slot
  int spectra_rec;         // doubles per slot of the spectra record
  Timer* timer;            // may be null
  int psched[kNumPasses];  // schedule of each pass (Ops::rhs_mixed)
};

// One evaluation of the nonlinear right-hand side at stage_in followed by the stage
// update (stage 0..3) or, for stage < 0, the full dy/dt into rhs_out.
typedef void (*RhsStageFn)(const Ctx&, void* state, const void* stage_in, int stage, void* rhs_out,
                           int want_max, double dt_arg, int flags, hipStream_t);

// Schedules (tile and radix choices) compiled for the step kernels of one size.
constexpr int kMaxSched = 8;
struct StepSched {
  int ec, ex;          // elements per thread of the column passes and of the x pass
  int col_w;           // kx columns per column block
  int fused_ec;        // elements per thread of the z-update pass
  int fused_w;         // kx columns per z-update block
  int x_lines;         // x-pass lines per block
  RhsStageFn rhs_stage;
};

// One (N, precision) instantiation of the device code.
struct Ops {
  int nsched;
  StepSched sched[kMaxSched];
  // the stage with each pass in the schedule Ctx::psched names (null: sched[0] only)
  RhsStageFn rhs_mixed;
  // the stage with the phase-shift dealiasing on the step kernels of this N (null: none)
  RhsStageFn rhs_phase;
  void (*init_field)(const Ctx&, void* state, int slot, uint64_t seed, double k_peak, int spectrum, double energy,
                     hipStream_t);
  void (*get_state)(const Ctx&, const void* state, int slot, void* canon, hipStream_t);
  void (*set_state)(const Ctx&, void* state, int slot, const void* canon, hipStream_t);
  void (*spectra)(const Ctx&, const void* state, double* out, int flags, hipStream_t);
  void (*pressure)(const Ctx&, const void* state, void* canon, const int* active, hipStream_t);
  // the hold forcing after the last stage of a step (slots in PSDNS_FORCING_HOLD)
  void (*band_hold)(const Ctx&, void* state, hipStream_t);
  void (*zero_scalars)(const Ctx&, void* state, int slot, hipStream_t);
};

template <int N>
Ops make_ops_f32();
template <int N>
Ops make_ops_f64();

}  // namespace psdns
