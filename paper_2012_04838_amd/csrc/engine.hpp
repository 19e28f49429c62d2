// Device kernels of one RK right-hand-side evaluation and its stage update,
// templated on the grid size N and the real type T (float or double).
//
// One evaluation is five passes over HBM (Sec. 2.2-2.3 of arXiv:2012.04838,
// restated for the 2/3 rule and the integrating factor):
//   z_inverse   compact state -> inverse along z of u_i and dz u_1, dz u_2, phi, dz phi
//   y_inverse   -> inverse along y, forming the y-derivatives needed by omega, grad phi
//   x_pass      per (z, y) line: inverse along x, u x omega and u.grad phi + g.u in
//               registers, forward along x (physical fields never reach HBM)
//   y_forward   -> forward along y, keep |ky| <= K
//   z_forward   -> forward along z, keep |kz| <= K, projection P(k), forcing A u_hat,
//               integrating-factor RK4 stage update
// Each kernel reads and writes every element of its fields exactly once.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "common.hpp"
#include "fft.hpp"
#include "mem.hpp"

namespace psdns {

// Tuning knobs (elements per thread, minimum waves per SIMD for the register
// allocator; 0 leaves the allocator free).
#ifndef PSDNS_EC32
#define PSDNS_EC32 8
#endif
#ifndef PSDNS_EC64
#define PSDNS_EC64 8
#endif
#ifndef PSDNS_COL_WAVES
#define PSDNS_COL_WAVES 0
#endif
#ifndef PSDNS_X_WAVES
#define PSDNS_X_WAVES 2
#endif
#if PSDNS_COL_WAVES > 0
#define PSDNS_COL_BOUNDS(...) __launch_bounds__((__VA_ARGS__), PSDNS_COL_WAVES)
#else
#define PSDNS_COL_BOUNDS(...) __launch_bounds__((__VA_ARGS__))
#endif
#if PSDNS_X_WAVES > 0
#define PSDNS_X_BOUNDS(...) __launch_bounds__((__VA_ARGS__), PSDNS_X_WAVES)
#else
#define PSDNS_X_BOUNDS(...) __launch_bounds__((__VA_ARGS__))
#endif

// minimum waves per SIMD of the y-forward and z-update passes (0: as the other column passes)
#ifndef PSDNS_YF_WAVES
#define PSDNS_YF_WAVES 0
#endif
#ifndef PSDNS_FUSED_WAVES
#define PSDNS_FUSED_WAVES 0
#endif
#if PSDNS_YF_WAVES > 0
#define PSDNS_YF_BOUNDS(...) __launch_bounds__((__VA_ARGS__), PSDNS_YF_WAVES)
#else
#define PSDNS_YF_BOUNDS(...) PSDNS_COL_BOUNDS(__VA_ARGS__)
#endif
#if PSDNS_FUSED_WAVES > 0
#define PSDNS_FUSED_BOUNDS(...) __launch_bounds__((__VA_ARGS__), PSDNS_FUSED_WAVES)
#else
#define PSDNS_FUSED_BOUNDS(...) PSDNS_COL_BOUNDS(__VA_ARGS__)
#endif

#ifndef PSDNS_COL_BYTES
#define PSDNS_COL_BYTES 128
#endif
#ifndef PSDNS_COL_MAXT
#define PSDNS_COL_MAXT 1024
#endif

// elements per thread of the fused z-forward/update/z-inverse pass
#ifndef PSDNS_EF32
#define PSDNS_EF32 8
#endif
#ifndef PSDNS_EF64
#define PSDNS_EF64 8
#endif

// row segment of the z-forward/update pass (both variants), in bytes
#ifndef PSDNS_FB32
#define PSDNS_FB32 PSDNS_COL_BYTES
#endif
#ifndef PSDNS_FB64
#define PSDNS_FB64 PSDNS_COL_BYTES
#endif

// Threads per column block: PSDNS_COL_MAXT, and at most 512 for FP32 columns longer than
// 512 points.  There 512-thread blocks of 32 (128-byte tiles) or 16 (64-byte tiles) elements
// per thread, with 256 registers each, beat 1024-thread blocks of 16 or 8 elements held in
// 128 registers, spills included (1024^3: z inverse 6.1 against 7.1 ms, y inverse 9.0
// against 9.7, y forward 3.8 against 4.2).
template <int N, typename T>
constexpr int col_max_threads() {
  return (N > 512 && sizeof(T) == 4 && PSDNS_COL_MAXT > 512) ? 512 : PSDNS_COL_MAXT;
}

// Geometry of a column pass: W columns (one row segment of BYTES bytes) per block,
// TC = N/EC threads per column, EC elements per thread.
template <int N, typename T, int E_REQ, int BYTES = PSDNS_COL_BYTES>
struct ColCfg {
  static constexpr int W = BYTES / (int)sizeof(cpx<T>);
  static constexpr int MAXT = col_max_threads<N, T>();
  // at least N * W / MAXT elements per thread, so a block stays within the cap
  static constexpr int EC1 = E_REQ * MAXT < N * W ? N * W / MAXT : E_REQ;
  static constexpr int EC = N < EC1 ? N : EC1;
  static constexpr int TC = N / EC;
  static constexpr int THREADS = W * TC;
  // 64-byte row segments: the two halves of a 128-byte row go to consecutive blocks of
  // one XCD (col_block), so that XCD's L2 serves the second half
  static constexpr bool PAIR = W * (int)sizeof(cpx<T>) == 64;
  static constexpr int STORE = store_policy(W * (int)sizeof(cpx<T>));  // cache policy of its stores
  static_assert(THREADS <= 1024, "column block too large");
  static_assert((W * N + N) * sizeof(cpx<T>) <= 160 * 1024, "column pass LDS exceeds 160 KB");
  // blocks along x of a grid covering ntile kx tiles
  static constexpr int grid_x(int ntile) { return PAIR ? (ntile + 1) / 2 * 2 : ntile; }
};

// LDS of a column pass: the exchange buffer, doubled (one barrier per exchange)
// when two buffers and the twiddle table fit in the 160 KB of a CU.
#ifndef PSDNS_COL_DB
#define PSDNS_COL_DB 1
#endif
#ifndef PSDNS_FUSED_DB
#define PSDNS_FUSED_DB 0
#endif
// velocity components of the z-update pass fetched one ahead of their transform
#ifndef PSDNS_FUSED_PF
#define PSDNS_FUSED_PF 1
#endif
#ifndef PSDNS_YF_DB
#define PSDNS_YF_DB PSDNS_COL_DB
#endif
template <int N, typename T, int W, bool EN = PSDNS_COL_DB>
struct ColLds {
  static constexpr bool kDouble = EN && (2 * W * N + N) * sizeof(cpx<T>) <= 160 * 1024;
  static constexpr int kEntries = (kDouble ? 2 : 1) * W * N;
  using View = LdsCol<T, W, kDouble ? W * N : 0>;
};

// Whether a column pass with E elements per thread and THREADS threads per block can
// hold the next field's elements (prefetch) next to its two working arrays within
// the per-thread register budget of the block (65536 per SIMD over its waves).
template <typename T, int E, int THREADS>
constexpr bool col_prefetch() {
  return 3 * E * (int)sizeof(cpx<T>) / 4 + 40 <= 131072 / THREADS;
}

// Step schedules the autotuner chooses from: the tile and radix choices of the step
// kernels.  ec: elements per thread of the column passes (the radix of their Stockham
// stages); bytes: row segment (kx tile) of a column block; ef, fb: the same for the
// z-update pass; xl2: lines per x-pass block relative to 256 threads, in halves.
struct Sched {
  int ec32, ec64, bytes, ef32, ef64, fb32, fb64, xl2;
  int xw = 0;    // x pass, FP32: minimum waves per SIMD for the register allocator (0: PSDNS_X_WAVES)
  int xreg = 1;  // x pass, FP32: stage twiddles held in registers (else read from LDS)
  int xpf = 1;   // x pass, FP32: first scalar pair loaded before the velocity transforms
};
// bytes 0: the default of the size, 128-byte rows up to N = 512 and 64-byte rows above,
// where 1024-thread blocks of 128-byte rows would exceed the register budget.
constexpr Sched kSched[] = {
    {PSDNS_EC32, PSDNS_EC64, 0, PSDNS_EF32, PSDNS_EF64, 0, 0, 2},  // default
    {4, 4, PSDNS_COL_BYTES, 4, 4, PSDNS_COL_BYTES, PSDNS_COL_BYTES, 2},                          // radix 4
    {16, 16, PSDNS_COL_BYTES, 16, 16, PSDNS_COL_BYTES, PSDNS_COL_BYTES, 2},                      // radix 16
    {PSDNS_EC32, PSDNS_EC64, 64, PSDNS_EF32, PSDNS_EF64, 64, 64, 2},                             // narrow tiles
    {PSDNS_EC32, PSDNS_EC64, PSDNS_COL_BYTES, PSDNS_EF32, PSDNS_EF64, PSDNS_FB32, PSDNS_FB64, 1},  // small x blocks
    // x pass at three waves per SIMD: twiddles from LDS, no early scalar loads
    {PSDNS_EC32, PSDNS_EC64, 0, PSDNS_EF32, PSDNS_EF64, 0, 0, 2, 3, 0, 0},
    // the same with the twiddles kept in registers
    {PSDNS_EC32, PSDNS_EC64, 0, PSDNS_EF32, PSDNS_EF64, 0, 0, 2, 3, 1, 0},
    // radix 16 on 64-byte tiles: at N = 1024 a column is one wavefront of 16 elements per
    // lane in 512-thread blocks, whose 256-register budget holds the fused pass unspilled
    // (in FP32 there the cap of col_max_threads gives schedules 0, 3, 5 and 6 this shape too)
    {16, 16, 64, 16, 16, 64, 64, 2},
};
constexpr int kNumSched = (int)(sizeof(kSched) / sizeof(kSched[0]));
static_assert(kNumSched <= kMaxSched, "schedule table exceeds the dispatch table");
// schedules compiled for a grid size
template <int N>
constexpr int sched_count() {
  return kNumSched;
}
template <int N>
constexpr int row_bytes(int b, int dflt) {
  return b > 0 ? b : (N > 512 ? 64 : dflt);
}

template <int N, typename T, int V = 0>
struct Cfg {
  static constexpr Sched D = kSched[V];
  static constexpr bool F32 = sizeof(T) == 4;
  using Col = ColCfg<N, T, F32 ? D.ec32 : D.ec64, row_bytes<N>(D.bytes, PSDNS_COL_BYTES)>;
  using Fused = ColCfg<N, T, F32 ? D.ef32 : D.ef64, row_bytes<N>(F32 ? D.fb32 : D.fb64, F32 ? PSDNS_FB32 : PSDNS_FB64)>;
  // columns per block and elements per thread of the column passes (z, y)
  static constexpr int W = Col::W;
  static constexpr int EC = Col::EC;
  static constexpr int TC = Col::TC;
  static constexpr int COL_THREADS = Col::THREADS;
  // x pass: 8 elements per lane; lines of N <= 512 stay inside one wavefront, a line of
  // N = 1024 spans two
  static constexpr int EX0 = 8;
  static constexpr int EX = N < EX0 ? N : EX0;
  static constexpr int TX = N / EX;
  static constexpr int LX0 = 256 / TX * D.xl2 / 2;
  static constexpr int LX = LX0 < 1 ? 1 : (LX0 > 64 ? 64 : LX0);
  static constexpr int X_THREADS = LX * TX;
  static constexpr int X_WAVES = (D.xw > 0 && F32) ? D.xw : PSDNS_X_WAVES;  // FP64 lines need the registers
  static constexpr int LP = LinePad<N>::value;
};

// Block placement of a column pass over (kx tile, row, slot).  Blocks are handed to the 8
// XCDs round-robin in launch order (block L to XCD L mod 8), and each XCD has its own L2.
// With PAIR (64-byte tiles) the launch order is permuted so that tiles 2q and 2q + 1 of a
// row, the two halves of its 128-byte segments, are consecutive blocks on one XCD (launch
// blocks 16 r' + x and 16 r' + 8 + x); the grid is 2 ceil(ntile / 2) blocks wide and a
// block past the last tile has ok = false.  The tail of fewer than 16 blocks keeps the
// launch order.
struct ColBlock {
  int tile, row, slot;
  bool ok;
};
template <bool PAIR>
__device__ __forceinline__ ColBlock col_block(int ntile, int nrow) {
  ColBlock b;
  if constexpr (PAIR) {
    const long long L = blockIdx.x + (long long)gridDim.x * (blockIdx.y + (long long)gridDim.y * blockIdx.z);
    const long long G = (long long)gridDim.x * gridDim.y * gridDim.z;
    long long lam = L;
    if (L < G / 16 * 16) {
      const long long x = L % 8, r = L / 8;
      lam = 16 * (r / 2) + 2 * x + (r % 2);
    }
    const int npairs = (ntile + 1) / 2;
    const long long p = lam / 2;
    b.tile = 2 * (int)(p % npairs) + (int)(lam % 2);
    const long long rr = p / npairs;
    b.row = (int)(rr % nrow);
    b.slot = (int)(rr / nrow);
    b.ok = b.tile < ntile;
  } else {
    b.tile = blockIdx.x;
    b.row = blockIdx.y;
    b.slot = blockIdx.z;
    b.ok = true;
  }
  return b;
}

// Largest retained |k_i| of the step kernels: the 2/3 rule's (N-1)/3 (DL = 0), or the
// largest K with 9 K^2 < 2 N^2 that bounds the phase-shift sphere (DL = 1, Sec. 3.1).
template <int N, int DL>
constexpr int kmax() {
  if constexpr (DL == 0) {
    return (N - 1) / 3;
  } else {
    int k = 0;
    while (9LL * (k + 1) * (k + 1) < 2LL * N * N) ++k;
    return k;
  }
}
// exp(i pi k / N), the half-cell shift of wavenumber k (|k| <= N/2), from the root table
template <typename T>
__device__ __forceinline__ cpx<T> shift_phase(const cpx<T>* __restrict__ tw_g, int N, int k) {
  const cpx<T> v = tw_g[N + kShiftOff + (k < 0 ? -k : k)];
  return k < 0 ? conj(v) : v;
}

// position n of an N-point line -> compact index (or -1 if the wavenumber is truncated)
__device__ __forceinline__ int compact_of(int n, int N, int K, int M) {
  return n <= K ? n : (n >= N - K ? n - N + M : -1);
}
// position n -> signed wavenumber
__device__ __forceinline__ int wave_of(int n, int N) { return n <= N / 2 ? n : n - N; }
// compact index -> signed wavenumber
__device__ __forceinline__ int wave_of_compact(int c, int K, int M) { return c <= K ? c : c - M; }
// the half-cell shift phases of the N positions of a line, exp(i pi k / N) with k their
// wavenumbers (conjugated with CONJ), copied to the block's LDS (the caller's next block
// barrier publishes them)
template <int N, bool CONJ, typename T>
__device__ __forceinline__ void stage_shift(cpx<T>* dst, const cpx<T>* __restrict__ tw_g) {
  for (int i = threadIdx.x; i < N; i += blockDim.x) {
    const cpx<T> v = shift_phase(tw_g, N, wave_of(i, N));
    dst[i] = CONJ ? conj(v) : v;
  }
}

template <typename T>
__device__ __forceinline__ cpx<T> czero() { return {T(0), T(0)}; }

// ---------------------------------------------------------------------------
// z inverse: columns along kz at fixed (ky, kx-tile).
// A fields: 0 U1, 1 U2, 2 U3, 3 dz U1, 4 dz U2, 5+2s Phi_s, 6+2s dz Phi_s
// (all carry the 1/N^3 of Eq. (5) so that physical values are the true ones).
// The next field's loads are issued before the current field is transformed.
// DL = 1 (phase-shift dealiasing): the retained set is the sphere 9|k|^2 < 2N^2 inside
// the cube |k_i| <= K, only its modes are read, and with shift the inputs carry
// exp(i pi kz / N) (the kx and ky parts are applied by the later passes).
// ---------------------------------------------------------------------------
template <int N, typename T, int V, int DL = 0>
__global__ void PSDNS_COL_BOUNDS(Cfg<N, T, V>::COL_THREADS)
k_z_inverse(const cpx<T>* __restrict__ st, cpx<T>* __restrict__ abuf, const cpx<T>* __restrict__ tw_g,
            const SlotDev* __restrict__ slots, Geom g, int shift = 0) {
  using C = Cfg<N, T, V>;
  constexpr int W = C::W, E = C::EC, TT = C::TC;
  constexpr int K = kmax<N, DL>();
  constexpr int M = 2 * K + 1;
  constexpr uint32_t CS = sizeof(cpx<T>);
  using L = ColLds<N, T, W>;
  __shared__ cpx<T> smem[L::kEntries];
  __shared__ cpx<T> stw[N];
  __shared__ cpx<T> sph[DL ? N : 1];
  const ColBlock cb = col_block<C::Col::PAIR>((g.KX + W - 1) / W, M);
  if (!cb.ok) return;
  const int slot = cb.slot;
  if (!slots[slot].active) return;
  if constexpr (DL) stage_shift<N, false>(sph, tw_g);
  stage_twiddles<N>(stw, tw_g);
  const cpx<T>* tw = stw;
  const int c = threadIdx.x % W;
  const int j = threadIdx.x / W;
  const int kx = cb.tile * W + c;
  const int kyc = cb.row;
  const bool valid = kx < g.KX;
  const typename L::View lds{smem + c};
  const T scale = T(1) / (T(N) * T(N) * T(N));
  // state rows (kz_c, ky_c) and A rows (z, ky_c) are both M PX entries apart along z
  const uint32_t rsb = (uint32_t)M * g.PX * CS;
  const uint32_t voff = ((uint32_t)j * M * g.PX + (uint32_t)kyc * g.PX + (uint32_t)kx) * CS;
  const cpx<T>* sslot = st + (long long)slot * g.F * g.st_field;
  cpx<T>* aslot = abuf + (long long)slot * g.FA * g.a_field;

  [[maybe_unused]] const int ky = wave_of_compact(kyc, K, M);
  auto load = [&](int f, cpx<T> (&v)[E]) {
    const Buf<T> b = make_buf<T>(sslot + (long long)f * g.st_field);
#pragma unroll
    for (int m = 0; m < E; ++m) {
      uint32_t vo, so;
      bool in = valid && compact_at<N, TT, K>(m, j, voff, rsb, vo, so);
      if constexpr (DL) in = in && retained(g, kx, ky, wave_of(j + TT * m, N));
      v[m] = in ? bload(b, vo, so) : czero<T>();
      if constexpr (DL)
        if (shift) v[m] = cmul(v[m], sph[j + TT * m]);
    }
  };
  auto store = [&](int f, const cpx<T> (&v)[E]) {
    if (!valid) return;
    const Buf<T> b = make_buf<T>(aslot + (long long)f * g.a_field);
#pragma unroll
    for (int m = 0; m < E; ++m) bstore<C::Col::STORE>(b, voff, (uint32_t)(TT * m) * rsb, v[m]);
  };
  cpx<T> a[E], d[E], nx[E];
  // transform the field held in a (and its z derivative into fd when fd >= 0)
  auto emit = [&](int f, int fd) {
#pragma unroll
    for (int m = 0; m < E; ++m) {
      a[m] = scale * a[m];
      if (fd >= 0) d[m] = mul_is(a[m], T(wave_of(j + TT * m, N)));
    }
    fft<N, E, true>(a, lds, j, tw);
    store(f, a);
    if (fd >= 0) {
      fft<N, E, true>(d, lds, j, tw);
      store(fd, d);
    }
  };
  // field cur into a (from the prefetch when enabled), then prefetch field nxt
  constexpr bool PF = col_prefetch<T, E, C::COL_THREADS>();
  auto advance = [&](int cur, int nxt) {
    if constexpr (PF) {
#pragma unroll
      for (int m = 0; m < E; ++m) a[m] = nx[m];
      if (nxt >= 0) load(nxt, nx);
    } else {
      load(cur, a);
    }
  };
  load(0, a);
  if constexpr (PF) load(1, nx);
  emit(0, 3);  // u1, dz u1
  advance(1, 2);
  emit(1, 4);  // u2, dz u2
  advance(2, g.S > 0 ? 3 : -1);
  emit(2, -1);  // u3
  for (int s = 0; s < g.S; ++s) {
    advance(3 + s, s + 1 < g.S ? 4 + s : -1);
    emit(5 + 2 * s, 6 + 2 * s);  // phi_s, dz phi_s
  }
}

// ---------------------------------------------------------------------------
// y inverse: columns along ky at fixed (z, kx-tile).
// B fields: 0 u1, 1 u2, 2 u3, 3 omega1 = dy u3 - dz u2, 4 dz u1, 5 dy u1,
//           6+3s phi_s, 7+3s dy phi_s, 8+3s dz phi_s   (x still spectral)
// The next field's loads are issued before the current field is transformed.
// DL = 1: the cube |ky| <= K of the phase-shift sphere; with shift the inputs carry
// exp(i pi ky / N).
// ---------------------------------------------------------------------------
template <int N, typename T, int V, int DL = 0>
__global__ void PSDNS_COL_BOUNDS(Cfg<N, T, V>::COL_THREADS)
k_y_inverse(const cpx<T>* __restrict__ abuf, cpx<T>* __restrict__ bbuf, const cpx<T>* __restrict__ tw_g,
            const SlotDev* __restrict__ slots, Geom g, int shift = 0) {
  using C = Cfg<N, T, V>;
  constexpr int W = C::W, E = C::EC, TT = C::TC;
  constexpr int K = kmax<N, DL>();
  constexpr int M = 2 * K + 1;
  constexpr uint32_t CS = sizeof(cpx<T>);
  using L = ColLds<N, T, W>;
  __shared__ cpx<T> smem[L::kEntries];
  __shared__ cpx<T> stw[N];
  __shared__ cpx<T> sph[DL ? N : 1];
  const ColBlock cb = col_block<C::Col::PAIR>((g.KX + W - 1) / W, N);
  if (!cb.ok) return;
  const int slot = cb.slot;
  if (!slots[slot].active) return;
  if constexpr (DL) stage_shift<N, false>(sph, tw_g);
  stage_twiddles<N>(stw, tw_g);
  const cpx<T>* tw = stw;
  const int c = threadIdx.x % W;
  const int j = threadIdx.x / W;
  const int kx = cb.tile * W + c;
  const int z = cb.row;
  const bool valid = kx < g.KX;
  const typename L::View lds{smem + c};
  // A rows (z, ky_c) and B rows (z, y) are both PX entries apart at fixed z
  const uint32_t rsb = (uint32_t)g.PX * CS;
  const uint32_t voff = ((uint32_t)j * g.PX + (uint32_t)kx) * CS;
  const cpx<T>* aplane = abuf + (long long)slot * g.FA * g.a_field + a_row(z, 0, M, g.PX);
  cpx<T>* bplane = bbuf + (long long)slot * g.FB * g.b_field + (long long)z * N * g.PX;

  auto kyv = [&](int m) { return T(wave_of(j + TT * m, N)); };
  auto load = [&](int f, cpx<T> (&v)[E]) {
    const Buf<T> b = make_buf<T>(aplane + (long long)f * g.a_field);
#pragma unroll
    for (int m = 0; m < E; ++m) {
      uint32_t vo, so;
      v[m] = (valid && compact_at<N, TT, K>(m, j, voff, rsb, vo, so)) ? bload<T, kPolicyStream>(b, vo, so)
                                                                        : czero<T>();
      if constexpr (DL)
        if (shift) v[m] = cmul(v[m], sph[j + TT * m]);
    }
  };
  auto store = [&](int f, const cpx<T> (&v)[E]) {
    if (!valid) return;
    const Buf<T> b = make_buf<T>(bplane + (long long)f * g.b_field);
#pragma unroll
    for (int m = 0; m < E; ++m) bstore<C::Col::STORE>(b, voff, (uint32_t)(TT * m) * rsb, v[m]);
  };
  cpx<T> a[E], d[E], nx[E];
  // field cur into a (from the prefetch when enabled), then prefetch field nxt
  constexpr bool PF = col_prefetch<T, E, C::COL_THREADS>();
  auto advance = [&](int cur, int nxt) {
    if constexpr (PF) {
#pragma unroll
      for (int m = 0; m < E; ++m) a[m] = nx[m];
      if (nxt >= 0) load(nxt, nx);
    } else {
      load(cur, a);
    }
  };
  // u1 and dy u1
  load(0, a);
  if constexpr (PF) load(1, nx);
#pragma unroll
  for (int m = 0; m < E; ++m) d[m] = mul_is(a[m], kyv(m));
  fft<N, E, true>(a, lds, j, tw);
  store(0, a);
  fft<N, E, true>(d, lds, j, tw);
  store(5, d);
  // u2
  advance(1, 2);
  load(4, d);
  fft<N, E, true>(a, lds, j, tw);
  store(1, a);
  // u3 and omega1 = dy u3 - dz u2
  advance(2, 3);
#pragma unroll
  for (int m = 0; m < E; ++m) d[m] = mul_is(a[m], kyv(m)) - d[m];
  fft<N, E, true>(a, lds, j, tw);
  store(2, a);
  fft<N, E, true>(d, lds, j, tw);
  store(3, d);
  // dz u1
  advance(3, g.S > 0 ? 5 : -1);
  fft<N, E, true>(a, lds, j, tw);
  store(4, a);
  for (int s = 0; s < g.S; ++s) {
    // phi_s and dy phi_s
    advance(5 + 2 * s, 6 + 2 * s);
#pragma unroll
    for (int m = 0; m < E; ++m) d[m] = mul_is(a[m], kyv(m));
    fft<N, E, true>(a, lds, j, tw);
    store(6 + 3 * s, a);
    fft<N, E, true>(d, lds, j, tw);
    store(7 + 3 * s, d);
    // dz phi_s
    advance(6 + 2 * s, s + 1 < g.S ? 7 + 2 * s : -1);
    fft<N, E, true>(a, lds, j, tw);
    store(8 + 3 * s, a);
  }
}

// ---------------------------------------------------------------------------
// x pass: one (z, y) line per TX lanes; a line never leaves its wavefront, so
// the exchanges inside a line only need wave-level ordering.  Two real fields
// f, g travel as one complex line h = f + i g through an N-point complex
// transform.  Lane j loads the unique half-spectrum entries kx = j + TX q of a
// line once; the conjugate-mirrored entries it needs (negative kx) come from
// the partner lane (kx = TX - j mod TX) by a cross-lane permute, and the
// forward post-processing pairs Z[k] with Z[N-k] the same way.
// Output (in place, first F fields of B): 0 c1, 1 c2, 2 c3 with c = u x omega,
// 3+s a_s = u.grad phi_s + g_s.u, forward transformed along x, kx <= K.
// ---------------------------------------------------------------------------
template <int B_, int E_, class Fn>
__device__ __forceinline__ void static_for(Fn&& fn) {
  if constexpr (B_ < E_) {
    fn(std::integral_constant<int, B_>{});
    static_for<B_ + 1, E_>(fn);
  }
}

template <typename T>
__device__ __forceinline__ cpx<T> shfl_c(cpx<T> v, int src) {
  return {__shfl(v.x, src), __shfl(v.y, src)};
}

// Lane-level helpers of the x pass: which unique half-spectrum entries a lane
// loads, and how it assembles its strided positions of h = f + i g.
template <int N, typename T, int K_ = (N - 1) / 3>
struct XLine {
  static constexpr int E = Cfg<N, T>::EX, TT = Cfg<N, T>::TX;
  static constexpr int K = K_;
  static constexpr int NQ = (K + 1 + TT - 1) / TT;  // unique entries per lane and field
  // a line inside one wavefront exchanges with its mirror lane by a cross-lane permute;
  // a line over several wavefronts goes through LDS (block barriers)
  static constexpr bool kMulti = TT > 64;
  static_assert((TT <= 64 && 64 % TT == 0) || TT % 64 == 0, "lines must tile wavefronts");
  static_assert(NQ < E, "retained band must be shorter than the line");
  using Sync = std::conditional_t<kMulti, BlockSync, WaveSync>;
  // LDS entries of the mirror exchange per block thread (kMulti)
  static constexpr int kXch = kMulti ? 2 * NQ : 0;
  int j, partner;  // partner: lane in the wavefront, or thread in the block (kMulti)
  cpx<T>* xs;      // exchange area [2 NQ][blockDim] (kMulti)
  __device__ __forceinline__ explicit XLine(int tid, cpx<T>* xch = nullptr)
      : j(tid % TT),
        partner(kMulti ? (tid - tid % TT) + ((TT - tid % TT) & (TT - 1))
                       : ((tid & 63) - tid % TT) + ((TT - tid % TT) & (TT - 1))),
        xs(xch) {}
  __device__ __forceinline__ void mirror1(const cpx<T> (&v)[NQ], cpx<T> (&p)[NQ]) const {
    if constexpr (kMulti) {
      const int nt = blockDim.x;
#pragma unroll
      for (int q = 0; q < NQ; ++q) xs[q * nt + threadIdx.x] = v[q];
      __syncthreads();
#pragma unroll
      for (int q = 0; q < NQ; ++q) p[q] = xs[q * nt + partner];
      __syncthreads();
    } else {
#pragma unroll
      for (int q = 0; q < NQ; ++q) p[q] = shfl_c(v[q], partner);
    }
  }
  // values of the mirror lane: p[q] = v[q] of thread `partner`, q < NQ (two arrays at once)
  __device__ __forceinline__ void mirror(const cpx<T> (&va)[NQ], const cpx<T> (&vb)[NQ], cpx<T> (&pa)[NQ],
                                         cpx<T> (&pb)[NQ]) const {
    if constexpr (kMulti) {
      const int nt = blockDim.x;
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        xs[q * nt + threadIdx.x] = va[q];
        xs[(NQ + q) * nt + threadIdx.x] = vb[q];
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        pa[q] = xs[q * nt + partner];
        pb[q] = xs[(NQ + q) * nt + partner];
      }
      __syncthreads();
    } else {
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        pa[q] = shfl_c(va[q], partner);
        pb[q] = shfl_c(vb[q], partner);
      }
    }
  }
  __device__ __forceinline__ T kx(int q) const { return T(j + TT * q); }
  // r[q] = entry kx = j + TT q of the line at p (zero beyond K); at kx = 0 only the
  // real part is kept, as a complex-to-real transform does.
  // (the line is the field buffer b at byte offset voff + the entry's kx * entry size;
  //  entry j + TT q adds the uniform q TT entries)
  __device__ __forceinline__ void load(const Buf<T>& b, uint32_t voff, cpx<T> (&r)[NQ]) const {
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int k = j + TT * q;
      r[q] = k <= K ? bload(b, voff, (uint32_t)(TT * q * (int)sizeof(cpx<T>))) : czero<T>();
    }
    if (j == 0) r[0].y = T(0);
  }
  // h at positions n = j + TT m from the half-spectrum entries of f (va) and g (vb):
  // n <= K: va + i vb;  n >= N - K: conj(va) + i conj(vb) of kx = N - n;  else 0
  __device__ __forceinline__ void build(const cpx<T> (&va)[NQ], const cpx<T> (&vb)[NQ], cpx<T> (&h)[E]) const {
    // multi-wave lines gather the mirror lane's entries through LDS first; single-wave
    // lines permute each one where it is needed (fewer live registers)
    cpx<T> ma[NQ], mb[NQ];
    if constexpr (kMulti) mirror(va, vb, ma, mb);
    static_for<0, E>([&](auto mc) {
      constexpr int m = decltype(mc)::value;
      const int n = j + TT * m;
      cpx<T> a = czero<T>(), b = czero<T>();
      if constexpr (TT * m <= K) {
        if (n <= K) {
          a = va[m];
          b = vb[m];
        }
      }
      if constexpr (TT * m + TT - 1 >= N - K) {
        constexpr int q1 = E - m - 1;  // slot of kx = N - n at the partner lane (j != 0)
        constexpr int q0 = E - m;      // own slot when j == 0
        cpx<T> pa = czero<T>(), pb = czero<T>();
        if constexpr (q1 < NQ) {
          if constexpr (kMulti) {
            pa = ma[q1];
            pb = mb[q1];
          } else {
            pa = shfl_c(va[q1], partner);
            pb = shfl_c(vb[q1], partner);
          }
        }
        if (j == 0) {
          if constexpr (q0 < NQ) {
            pa = va[q0];
            pb = vb[q0];
          } else {
            pa = czero<T>();
            pb = czero<T>();
          }
        }
        if (n >= N - K) {
          a = conj(pa);
          b = conj(pb);
        }
      }
      h[m] = a + mul_i(b);
    });
  }
};

// mode bits of the x pass
constexpr int kXMax = 1;       // partial maxima of |u1|+|u2|+|u3| (CFL)
constexpr int kXPressure = 2;  // with S = 0: forward field 3 is |u|^2/2 (pressure assembly)
constexpr int kXShift = 4;     // DL = 1: inputs times exp(i pi kx / N), outputs times its conjugate

template <int N, typename T, int V, int DL = 0>
__global__ void __launch_bounds__((Cfg<N, T, V>::X_THREADS), (Cfg<N, T, V>::X_WAVES))
k_x_pass(cpx<T>* __restrict__ bbuf, const cpx<T>* __restrict__ tw_g, const SlotDev* __restrict__ slots,
         DynDev* __restrict__ dyn, Geom g, int mode) {
  using C = Cfg<N, T, V>;
  constexpr int K = kmax<N, DL>();
  using XL = XLine<N, T, K>;
  using XS = typename XL::Sync;
  constexpr int E = C::EX, TT = C::TX, L = C::LX, LP = C::LP;
  [[maybe_unused]] const bool shifted = DL && (mode & kXShift);
  constexpr int NQ = XL::NQ;  // unique entries per lane and field
  __shared__ cpx<T> smem[L * LP];
  __shared__ cpx<T> stw[N];
  __shared__ double red[C::X_THREADS];
  __shared__ cpx<T> xch[XL::kXch > 0 ? XL::kXch * C::X_THREADS : 1];
  const int slot = blockIdx.y;
  if (!slots[slot].active) return;
  stage_twiddles<N>(stw, tw_g);
  const int li = threadIdx.x / TT;
  const int j = threadIdx.x % TT;
  // FP32 up to N = 512: the lane's twiddles live in registers for all nine transforms
  // of the line; FP64, and the 16-element lines of N = 1024, keep them in LDS to leave
  // registers for the line data.
  constexpr bool kLong = E > 8;
  constexpr bool kRegTw = sizeof(T) == 4 && !kLong && C::D.xreg;
  // FP32 short lines load every input up front; FP64 and 16-element lines load u3/omega1
  // and u1/u2 only when their transform comes (registers)
  constexpr bool kLate = kLong || sizeof(T) == 8;
  using TwT = std::conditional_t<kRegTw, TwReg<N, E, T>, const cpx<T>*>;
  TwT tw;
  if constexpr (kRegTw)
    tw = tw_fill<N, E>(j, stw);
  else
    tw = stw;
  const long long line = (long long)blockIdx.x * L + li;  // z * N + y
  const LdsLine<T, N, E> lds{smem + li * LP};
  // fields addressed from the block's first line; a lane's offset covers its line and kx
  const cpx<T>* bblock = bbuf + (long long)slot * g.FB * g.b_field + (long long)blockIdx.x * L * g.PX;
  const uint32_t voff = ((uint32_t)li * g.PX + (uint32_t)j) * (uint32_t)sizeof(cpx<T>);
  auto fbuf = [&](int f) { return make_buf<T>(bblock + (long long)f * g.b_field); };

  const XL xl(threadIdx.x, xch);
  // DL = 1 with the shift: the phases exp(i pi kx / N) of the lane's entries, read once
  [[maybe_unused]] cpx<T> xph[DL ? NQ : 1];
  if constexpr (DL) {
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int k = j + TT * q;
      xph[q] = (shifted && k <= K) ? shift_phase(tw_g, N, k) : cpx<T>{T(1), T(0)};
    }
  }
  auto load = [&](int f, cpx<T> (&r)[NQ]) {
    xl.load(fbuf(f), voff, r);
    if constexpr (DL) {
      if (shifted) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) r[q] = cmul(r[q], xph[q]);
      }
    }
  };
  auto build = [&](const cpx<T> (&va)[NQ], const cpx<T> (&vb)[NQ], cpx<T> (&h)[E]) { xl.build(va, vb, h); };
  auto kxq = [&](int q) { return T(j + TT * q); };

  // short lines load every input up front; 16-element lines load u3/omega1 and
  // u1/u2 only when their transform comes (registers)
  cpx<T> r0[NQ], r1[NQ], r2[NQ], r3[NQ], r4[NQ], r5[NQ];
  load(1, r1);
  load(2, r2);
  load(4, r4);
  load(5, r5);
  if constexpr (!kLate) {
    load(3, r3);
    load(0, r0);
  }
  cpx<T> h[E], va[NQ], vb[NQ];
  // omega2 = dz u1 - dx u3, omega3 = dx u2 - dy u1
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    va[q] = r4[q] - mul_is(r2[q], kxq(q));
    vb[q] = mul_is(r1[q], kxq(q)) - r5[q];
  }
  build(va, vb, h);
  fft<N, E, true, XS>(h, lds, j, tw);
  T w2p[E], w3p[E];
#pragma unroll
  for (int m = 0; m < E; ++m) {
    w2p[m] = h[m].x;
    w3p[m] = h[m].y;
  }
  // u3, omega1
  if constexpr (kLate) load(3, r3);
  build(r2, r3, h);
  fft<N, E, true, XS>(h, lds, j, tw);
  T u3p[E], w1p[E];
#pragma unroll
  for (int m = 0; m < E; ++m) {
    u3p[m] = h[m].x;
    w1p[m] = h[m].y;
  }
  // u1, u2
  if constexpr (kLate) load(0, r0);
  build(r0, r1, h);
  const int S = g.S;
  // first scalar pair's entries go in flight before the next transforms
  cpx<T> s0[NQ], s1[NQ], s2[NQ], s3[NQ], s4[NQ], s5[NQ];
  auto load_scalar_pair = [&](int s) {
    load(6 + 3 * s, s0);
    load(7 + 3 * s, s1);
    load(8 + 3 * s, s2);
    if (s + 1 < S) {
      load(9 + 3 * s, s3);
      load(10 + 3 * s, s4);
      load(11 + 3 * s, s5);
    }
  };
  constexpr bool kPrefetchScalars = sizeof(T) == 4 && !kLong && C::D.xpf;
  if (kPrefetchScalars && S > 0) load_scalar_pair(0);
  fft<N, E, true, XS>(h, lds, j, tw);
  T u1p[E], u2p[E], c1[E], c2[E], c3[E];
  T mx = T(0);
#pragma unroll
  for (int m = 0; m < E; ++m) {
    u1p[m] = h[m].x;
    u2p[m] = h[m].y;
    c1[m] = u2p[m] * w3p[m] - u3p[m] * w2p[m];
    c2[m] = u3p[m] * w1p[m] - u1p[m] * w3p[m];
    c3[m] = u1p[m] * w2p[m] - u2p[m] * w1p[m];
    const T sm = fabs(u1p[m]) + fabs(u2p[m]) + fabs(u3p[m]);
    mx = (sm > mx || sm != sm) ? sm : mx;  // keeps NaN
  }

  // forward transform of the real pair (p, q); store fields fp, fq at kx <= K
  auto forward_pair = [&](const T (&p)[E], const T (&q)[E], int fp, int fq) {
#pragma unroll
    for (int m = 0; m < E; ++m) h[m] = {p[m], q[m]};
    fft<N, E, false, XS>(h, lds, j, tw);
    cpx<T> hm[NQ], pm[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) hm[q] = h[E - q - 1];
    xl.mirror1(hm, pm);
    static_for<0, NQ>([&](auto sc) {
      constexpr int s = decltype(sc)::value;
      cpx<T> zm = pm[s];
      if (j == 0) zm = h[(E - s) % E];
      const cpx<T> zk = h[s];
      const cpx<T> zc = conj(zm);
      const int kx = j + TT * s;
      if (kx <= K) {
        const uint32_t so = (uint32_t)(TT * s * (int)sizeof(cpx<T>));
        cpx<T> pv = T(0.5) * (zk + zc), qv = mul_mi(T(0.5) * (zk - zc));
        if constexpr (DL) {
          if (shifted) {
            const cpx<T> e = conj(xph[s]);
            pv = cmul(pv, e);
            qv = cmul(qv, e);
          }
        }
        bstore(fbuf(fp), voff, so, pv);
        if (fq >= 0) bstore(fbuf(fq), voff, so, qv);
      }
    });
  };
  T zero[E];
#pragma unroll
  for (int m = 0; m < E; ++m) zero[m] = T(0);

  forward_pair(c1, c2, 0, 1);
  if (S == 0) {
    if (mode & kXPressure) {
      // kinetic energy density |u|^2/2, the gradient part of u.grad u in rotational form
      T q[E];
#pragma unroll
      for (int m = 0; m < E; ++m) q[m] = T(0.5) * (u1p[m] * u1p[m] + u2p[m] * u2p[m] + u3p[m] * u3p[m]);
      forward_pair(c3, q, 2, 3);
    } else {
      forward_pair(c3, zero, 2, -1);
    }
  } else {
    const SlotDev& sp = slots[slot];
    T as0[E], as1[E];
    // scalars in pairs (s, s+1): a_s = u.grad phi_s + g_s.u
    for (int s = 0; s < S; s += 2) {
      const bool two = s + 1 < S;
      // FP64: each transform's inputs are loaded just before it (registers)
      if constexpr (kLate) {
        load(6 + 3 * s, s0);
        load(7 + 3 * s, s1);
      } else if (s > 0 || !kPrefetchScalars) {
        load_scalar_pair(s);
      }
      {
        const T g0 = T(sp.g[s][0]), g1 = T(sp.g[s][1]), g2 = T(sp.g[s][2]);
#pragma unroll
        for (int q = 0; q < NQ; ++q) va[q] = mul_is(s0[q], kxq(q));
        build(va, s1, h);
        fft<N, E, true, XS>(h, lds, j, tw);
#pragma unroll
        for (int m = 0; m < E; ++m)
          as0[m] = u1p[m] * h[m].x + u2p[m] * h[m].y + (g0 * u1p[m] + g1 * u2p[m] + g2 * u3p[m]);
      }
      if (two) {
        const T g0 = T(sp.g[s + 1][0]), g1 = T(sp.g[s + 1][1]), g2 = T(sp.g[s + 1][2]);
        if constexpr (kLate) {
          load(9 + 3 * s, s3);
          load(10 + 3 * s, s4);
        }
#pragma unroll
        for (int q = 0; q < NQ; ++q) va[q] = mul_is(s3[q], kxq(q));
        build(va, s4, h);
        fft<N, E, true, XS>(h, lds, j, tw);
#pragma unroll
        for (int m = 0; m < E; ++m)
          as1[m] = u1p[m] * h[m].x + u2p[m] * h[m].y + (g0 * u1p[m] + g1 * u2p[m] + g2 * u3p[m]);
      }
      // z-derivatives of both scalars share one transform
      if constexpr (kLate) {
        load(8 + 3 * s, s2);
        if (two) load(11 + 3 * s, s5);
      }
      if (!two) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) s5[q] = czero<T>();
      }
      build(s2, s5, h);
      fft<N, E, true, XS>(h, lds, j, tw);
#pragma unroll
      for (int m = 0; m < E; ++m) {
        as0[m] += u3p[m] * h[m].x;
        as1[m] = two ? as1[m] + u3p[m] * h[m].y : as1[m];
      }
      if (s == 0) {
        forward_pair(c3, as0, 2, 3);
        if (two) {
          if (S > 2) {
#pragma unroll
            for (int m = 0; m < E; ++m) c3[m] = as1[m];  // park a_1 until a_2 exists
          } else {
            forward_pair(as1, zero, 4, -1);
          }
        }
      } else {
        forward_pair(c3, as0, 3 + s - 1, 3 + s);
        if (two) forward_pair(as1, zero, 3 + s + 1, -1);
      }
    }
  }

  if (mode & kXMax) {
    red[threadIdx.x] = (double)mx;
    __syncthreads();
    for (int o = C::X_THREADS / 2; o > 0; o >>= 1) {
      if ((int)threadIdx.x < o) {
        const double a = red[threadIdx.x], b = red[threadIdx.x + o];
        red[threadIdx.x] = (b > a || b != b) ? b : a;
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) atomicMax(&dyn[slot].umax, (unsigned long long)__double_as_longlong(red[0]));
  }
}

// ---------------------------------------------------------------------------
// y forward: columns along y at fixed (z, kx-tile); keeps |ky| <= K.
// The next field's loads are issued before the current field is transformed.
// ---------------------------------------------------------------------------
template <int N, typename T, int V, int DL = 0>
__global__ void PSDNS_YF_BOUNDS(Cfg<N, T, V>::COL_THREADS)
k_y_forward(const cpx<T>* __restrict__ bbuf, cpx<T>* __restrict__ abuf, const cpx<T>* __restrict__ tw_g,
            const SlotDev* __restrict__ slots, Geom g, int shift = 0, int afields = 0) {
  using C = Cfg<N, T, V>;
  constexpr int W = C::W, E = C::EC, TT = C::TC;
  constexpr int K = kmax<N, DL>();
  constexpr int M = 2 * K + 1;
  constexpr uint32_t CS = sizeof(cpx<T>);
  using L = ColLds<N, T, W, PSDNS_YF_DB>;
  __shared__ cpx<T> smem[L::kEntries];
  __shared__ cpx<T> stw[N];
  __shared__ cpx<T> sph[DL ? N : 1];
  const ColBlock cb = col_block<C::Col::PAIR>((g.KX + W - 1) / W, N);
  if (!cb.ok) return;
  const int slot = cb.slot;
  if (!slots[slot].active) return;
  if constexpr (DL) stage_shift<N, true>(sph, tw_g);
  stage_twiddles<N>(stw, tw_g);
  const cpx<T>* tw = stw;
  const int c = threadIdx.x % W;
  const int j = threadIdx.x / W;
  const int kx = cb.tile * W + c;
  const int z = cb.row;
  const bool valid = kx < g.KX;
  const typename L::View lds{smem + c};
  const uint32_t rsb = (uint32_t)g.PX * CS;
  const uint32_t voff = ((uint32_t)j * g.PX + (uint32_t)kx) * CS;
  const cpx<T>* bplane = bbuf + (long long)slot * g.FB * g.b_field + (long long)z * N * g.PX;
  // DL = 1: the output has afields fields per slot (A, or the kept unshifted products)
  const int ofields = DL ? afields : g.FA;
  cpx<T>* aplane = abuf + (long long)slot * ofields * g.a_field + a_row(z, 0, M, g.PX);
  auto load = [&](int f, cpx<T> (&v)[E]) {
    const Buf<T> b = make_buf<T>(bplane + (long long)f * g.b_field);
#pragma unroll
    for (int m = 0; m < E; ++m) v[m] = valid ? bload<T, kPolicyStream>(b, voff, (uint32_t)(TT * m) * rsb) : czero<T>();
  };
  cpx<T> a[E], nx[E];
  constexpr bool PF = col_prefetch<T, E, C::COL_THREADS>();
  load(0, a);
  for (int f = 0; f < g.F; ++f) {
    if constexpr (PF) {
      if (f > 0) {
#pragma unroll
        for (int m = 0; m < E; ++m) a[m] = nx[m];
      }
      if (f + 1 < g.F) load(f + 1, nx);
    } else if (f > 0) {
      load(f, a);
    }
    fft<N, E, false>(a, lds, j, tw);
    if (valid) {
      const Buf<T> b = make_buf<T>(aplane + (long long)f * g.a_field);
#pragma unroll
      for (int m = 0; m < E; ++m) {
        uint32_t vo, so;
        if (!compact_at<N, TT, K>(m, j, voff, rsb, vo, so)) continue;
        cpx<T> v = a[m];
        if constexpr (DL)
          if (shift) v = cmul(v, sph[j + TT * m]);
        bstore<C::Col::STORE>(b, vo, so, v);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// z forward + spectral assembly + integrating-factor RK4 stage update.
// stage 0..3 updates (y_n, acc, y_stage); stage < 0 writes dy/dt to rhs_out.
// ---------------------------------------------------------------------------
template <typename T>
struct StageArgs {
  cpx<T>* yn;
  cpx<T>* acc;
  cpx<T>* ys;
  const cpx<T>* sin;    // stage input (y_n at stage 0, y_stage otherwise)
  cpx<T>* rhs;          // stage < 0 only
  const double* fband;  // stochastic forcing table [batch][kStochCand][12] (b, P(k) b)
  int stage;
};

// Stage update of one mode.  Returns the input of the next stage (y_stage for
// stages 0-2, y_{n+1} after stage 3); y_stage is stored only when write_ys.  The
// mode sits at byte offsets (vo, so) inside the field that starts foff entries
// into each state array.  F is the right-hand side without the linear term
// -lk2 y (lk2 = D |k|^2).  Integrating factor (expl = false): the stage formulas of
// Lawson's RK4 with eh = exp(-lk2 h/2) and e1 = eh^2 (FP64, then cast).  Explicit: the
// same formulas with both factors 1 and F completed by -lk2 times the stage input,
// which is classical RK4 on the full right-hand side.  STG is the stage when known at
// compile time (0..3, or -1 for dy/dt), else -2 and the stage comes from the arguments.
template <int STG, int SP = kPolicyStream, typename T>
__device__ __forceinline__ cpx<T> rk_update(const StageArgs<T>& a, long long foff, uint32_t vo, uint32_t so, cpx<T> F,
                                            double lk2, double ehd, double h, bool write_ys, bool expl) {
  const int stage = STG >= -1 ? STG : a.stage;
  if (stage < 0) {
    const cpx<T> y = bload(make_buf<T>(a.sin + foff), vo, so);
    bstore<SP>(make_buf<T>(a.rhs + foff), vo, so, F - T(lk2) * y);
    return czero<T>();
  }
  const Buf<T> yn = make_buf<T>(a.yn + foff), acc = make_buf<T>(a.acc + foff);
  const cpx<T> y = stage < 3 ? bload(yn, vo, so) : czero<T>();
  T eh, e1;
  if (expl) {
    const cpx<T> yin = stage == 0 ? y : bload(make_buf<T>(a.sin + foff), vo, so);
    F = F - T(lk2) * yin;
    eh = e1 = T(1);
  } else {
    eh = T(ehd);
    e1 = T(ehd * ehd);
  }
  const T th = T(h);
  cpx<T> nxt;
  switch (stage) {
    case 0: {
      bstore<SP>(acc, vo, so, e1 * (y + (th / T(6)) * F));
      nxt = eh * (y + (th / T(2)) * F);
      break;
    }
    case 1: {
      bstore<SP>(acc, vo, so, bload(acc, vo, so) + ((th / T(3)) * eh) * F);
      nxt = eh * y + (th / T(2)) * F;
      break;
    }
    case 2: {
      bstore<SP>(acc, vo, so, bload(acc, vo, so) + ((th / T(3)) * eh) * F);
      nxt = e1 * y + (th * eh) * F;
      break;
    }
    default: {
      nxt = bload(acc, vo, so) + (th / T(6)) * F;
      bstore<SP>(yn, vo, so, nxt);
      return nxt;
    }
  }
  if (write_ys) bstore<SP>(make_buf<T>(a.ys + foff), vo, so, nxt);
  return nxt;
}

// The integrating-factor update split into its loads and its arithmetic and stores, so
// that a column issues the state loads of all its elements before any of its stores.
// Loads and stores share one completion counter, so a load waited for after a store
// also waits for that store; loading first keeps the stores out of those waits.
template <typename T>
struct RkIn {
  cpx<T> y, accv;  // y_n (stages 0-2) and the accumulator (stages 1-3)
};
template <int STG, typename T>
__device__ __forceinline__ RkIn<T> rk_load(const StageArgs<T>& a, long long foff, uint32_t vo, uint32_t so) {
  static_assert(STG >= 0 && STG <= 3, "integrating-factor stages only");
  RkIn<T> r{czero<T>(), czero<T>()};
  if constexpr (STG < 3) r.y = bload(make_buf<T>(a.yn + foff), vo, so);
  if constexpr (STG > 0) r.accv = bload(make_buf<T>(a.acc + foff), vo, so);
  return r;
}
// The stage formulas of rk_update (integrating factor) on values from rk_load; SP is the
// cache policy of the stores.
template <int STG, int SP = kPolicyStream, typename T>
__device__ __forceinline__ cpx<T> rk_apply(const StageArgs<T>& a, long long foff, uint32_t vo, uint32_t so,
                                           const RkIn<T>& in, cpx<T> F, double ehd, double h, bool write_ys) {
  const Buf<T> yn = make_buf<T>(a.yn + foff), acc = make_buf<T>(a.acc + foff);
  const T eh = T(ehd), e1 = T(ehd * ehd), th = T(h);
  const cpx<T> y = in.y;
  cpx<T> nxt;
  if constexpr (STG == 0) {
    bstore<SP>(acc, vo, so, e1 * (y + (th / T(6)) * F));
    nxt = eh * (y + (th / T(2)) * F);
  } else if constexpr (STG == 1) {
    bstore<SP>(acc, vo, so, in.accv + ((th / T(3)) * eh) * F);
    nxt = eh * y + (th / T(2)) * F;
  } else if constexpr (STG == 2) {
    bstore<SP>(acc, vo, so, in.accv + ((th / T(3)) * eh) * F);
    nxt = e1 * y + (th * eh) * F;
  } else {
    nxt = in.accv + (th / T(6)) * F;
    bstore<SP>(yn, vo, so, nxt);
    return nxt;
  }
  if (write_ys) bstore<SP>(make_buf<T>(a.ys + foff), vo, so, nxt);
  return nxt;
}

// FUSE: after the update, the next stage input (held in registers, in the same
// strided kz ownership the inverse transform starts from) is transformed back
// along z and written as the A fields of the next evaluation (the work of
// k_z_inverse); y_stage is then stored only on the forced band, where the next
// forcing amplitude and forcing term read it.  Fields go scalars first, in
// reverse order, then velocity, so that no A field is overwritten before this
// block has read its forward data.
//
// Addressing: A rows (z, ky_c) and state rows (kz_c, ky_c) are both M PX entries
// apart along z, so one per-thread byte offset (row j of the column) serves every
// field of both; element m adds a uniform multiple of the row stride.
//
// Integrating factor: exp(-D h |k|^2 / 2) = exp(-D h (kx^2 + ky^2) / 2) exp(-D h kz^2 / 2);
// the block tabulates the kz part in LDS for each diffusivity (velocity, each scalar)
// and each thread evaluates the first part once for its column, so that a mode costs one
// product instead of an exponential.
//
// STG: the stage (0..3) when the launch fixes it, so that the update compiles to straight
// code; -2 reads it from the arguments (the rarer unfused launches and dy/dt).
//
// DL = 1 (phase-shift dealiasing, unfused): A holds the products evaluated on the shifted
// grid and akeep those on the grid itself; each field is the mean of the two transforms,
// the shifted one brought back by exp(-i pi kz / N) (the kx and ky parts were applied by
// the x and y forward passes), and only modes inside the sphere 9|k|^2 < 2N^2 are updated.
template <int N, typename T, bool FUSE, int V, int STG, int DL = 0>
__global__ void PSDNS_FUSED_BOUNDS(Cfg<N, T, V>::Fused::THREADS)
k_z_forward_update(cpx<T>* __restrict__ abuf, StageArgs<T> sa, const cpx<T>* __restrict__ tw_g,
                   const SlotDev* __restrict__ slots, const DynDev* __restrict__ dyn, Geom g,
                   const cpx<T>* __restrict__ akeep = nullptr) {
  static_assert(!(FUSE && DL), "the phase-shift pass runs unfused");
  using C = typename Cfg<N, T, V>::Fused;
  constexpr int W = C::W, E = C::EC, TT = C::TC;
  constexpr int K = kmax<N, DL>();
  constexpr int M = 2 * K + 1;
  constexpr uint32_t CS = sizeof(cpx<T>);
  using L = ColLds<N, T, W, PSDNS_FUSED_DB>;
  __shared__ cpx<T> smem[L::kEntries];
  __shared__ cpx<T> stw[N];
  __shared__ double ez[(1 + kMaxScalars) * (K + 1)];  // exp(-D h kz^2 / 2), |kz| <= K
  __shared__ cpx<T> sph[DL ? N : 1];                  // exp(-i pi kz / N) at position n
  const ColBlock cb = col_block<C::PAIR>((g.KX + W - 1) / W, g.M);
  if (!cb.ok) return;
  const int slot = cb.slot;
  const SlotDev& sp = slots[slot];
  if (!sp.active) return;
  const double h = dyn[slot].dt;
  const bool expl = sp.integrator == PSDNS_INTEGRATOR_EXPLICIT;
  const int stage = STG >= -1 ? STG : sa.stage;
  const bool factors = !expl && stage >= 0;
  // The fused instances update integrating-factor slots only: the host runs a batch with
  // an explicit-integrator slot through the unfused pass.  Should such a slot reach a
  // fused instance, its stage input becomes non-finite, which its step record flags.
  auto guard = [&](cpx<T> v) {
    return (FUSE && expl) ? cpx<T>{T(__builtin_nan("")), T(__builtin_nan(""))} : v;
  };
  if (factors) {
    // diffusivity of class cls: velocity (sp.diff[0]) or scalar cls - 1 (sp.diff[2 + cls])
    for (int i = threadIdx.x; i < (1 + g.S) * (K + 1); i += blockDim.x) {
      const int cls = i / (K + 1), kz = i % (K + 1);
      ez[i] = exp(-0.5 * sp.diff[cls == 0 ? 0 : 2 + cls] * h * (double(kz) * kz));
    }
  }
  if constexpr (DL) stage_shift<N, true>(sph, tw_g);
  stage_twiddles<N>(stw, tw_g);  // its barrier also covers ez and sph
  const cpx<T>* tw = stw;
  const int c = threadIdx.x % W;
  const int j = threadIdx.x / W;
  const int kx = cb.tile * W + c;
  const int kyc = cb.row;
  const bool valid = kx < g.KX;
  const typename L::View lds{smem + c};
  const uint32_t rsb = (uint32_t)M * g.PX * CS;                       // z row stride (bytes)
  const uint32_t voff = ((uint32_t)j * M * g.PX + (uint32_t)kyc * g.PX + (uint32_t)kx) * CS;
  const cpx<T>* aslot = abuf + (long long)slot * g.FA * g.a_field;
  const long long sslot = (long long)slot * g.F * g.st_field;
  const int ky = wave_of_compact(kyc, g.K, g.M);
  const double A = dyn[slot].A;
  const T scale = T(1) / (T(N) * T(N) * T(N));

  const int kxy2 = kx * kx + ky * ky;
  // integrating factor of element m from its column's part exy (class cls)
  auto exy_of = [&](int cls) {
    return factors ? exp(-0.5 * sp.diff[cls == 0 ? 0 : 2 + cls] * h * double(kxy2)) : 1.0;
  };
  auto efac = [&](int cls, double exy, int m) {
    const int kz = wave_of(j + TT * m, N);
    return factors ? exy * ez[cls * (K + 1) + (kz < 0 ? -kz : kz)] : 1.0;
  };
  auto k2m = [&](int m) {
    const int kz = wave_of(j + TT * m, N);
    return double(kxy2 + kz * kz);
  };
  // forward data of A field f into v (the loads are issued; the transform comes later)
  auto fetch = [&](int f, cpx<T> (&v)[E]) {
    const Buf<T> b = make_buf<T>(aslot + (long long)f * g.a_field);
#pragma unroll
    for (int m = 0; m < E; ++m) v[m] = valid ? bload(b, voff, (uint32_t)(TT * m) * rsb) : czero<T>();
  };
  auto store_a = [&](int f, const cpx<T> (&v)[E]) {
    if (!valid) return;
    const Buf<T> b = make_buf<T>(aslot + (long long)f * g.a_field);
#pragma unroll
    for (int m = 0; m < E; ++m) bstore<C::STORE>(b, voff, (uint32_t)(TT * m) * rsb, v[m]);
  };
  // inverse z of the next stage input (scaled by 1/N^3) into A field f, and of i kz * it into fd
  auto inverse_out = [&](cpx<T> (&v)[E], int f, int fd, auto&& between) {
    cpx<T> d[E];
#pragma unroll
    for (int m = 0; m < E; ++m) {
      v[m] = scale * v[m];
      d[m] = mul_is(v[m], T(wave_of(j + TT * m, N)));
    }
    fft<N, E, true>(v, lds, j, tw);
    store_a(f, v);
    between();
    if (fd >= 0) {
      fft<N, E, true>(d, lds, j, tw);
      store_a(fd, d);
    }
  };
  auto nothing = [] {};
  // state offsets of element m (false where truncated or outside the kx range)
  auto state_at = [&](int m, uint32_t& vo, uint32_t& so) {
    bool in = valid && compact_at<N, TT, K>(m, j, voff, rsb, vo, so);
    if constexpr (DL) in = in && retained(g, kx, ky, wave_of(j + TT * m, N));
    return in;
  };
  // DL = 1: v (the transformed shifted product of field f) becomes the mean of the two
  // evaluations
  auto average = [&](int f, cpx<T> (&v)[E]) {
    if constexpr (DL) {
      __builtin_amdgcn_sched_barrier(0);  // the kept field's loads stay here (registers)
      cpx<T> u[E];
      const Buf<T> b = make_buf<T>(akeep + ((long long)slot * g.F + f) * g.a_field);
#pragma unroll
      for (int m = 0; m < E; ++m) u[m] = valid ? bload(b, voff, (uint32_t)(TT * m) * rsb) : czero<T>();
      fft<N, E, false>(u, lds, j, tw);
#pragma unroll
      for (int m = 0; m < E; ++m) v[m] = T(0.5) * (u[m] + cmul(v[m], sph[j + TT * m]));
      __builtin_amdgcn_sched_barrier(0);
    }
  };

  cpx<T> nx[E];
  if constexpr (FUSE) fetch(g.S > 0 ? 2 + g.S : 0, nx);
  // scalars: F = -a_hat (a already holds u.grad phi + g.u)
  for (int s = g.S - 1; s >= 0; --s) {
    cpx<T> a[E];
    if constexpr (FUSE) {
#pragma unroll
      for (int m = 0; m < E; ++m) a[m] = nx[m];
    } else {
      fetch(3 + s, a);
    }
    fft<N, E, false>(a, lds, j, tw);
    average(3 + s, a);
    const double dif = sp.diff[3 + s];
    const double exy = exy_of(1 + s);
    const long long foff = sslot + (long long)(3 + s) * g.st_field;
    if constexpr (FUSE) {
      // two batches of E/2 elements: their loads, then their arithmetic and stores
      constexpr int HB = E / 2;
      static_for<0, 2>([&](auto hc) {
        constexpr int h0 = decltype(hc)::value * HB;
        RkIn<T> in[HB];
#pragma unroll
        for (int q = 0; q < HB; ++q) {
          uint32_t vo, so;
          if (state_at(h0 + q, vo, so)) in[q] = rk_load<STG>(sa, foff, vo, so);
        }
#pragma unroll
        for (int q = 0; q < HB; ++q) {
          const int m = h0 + q;
          uint32_t vo, so;
          cpx<T> nxt = czero<T>();
          if (state_at(m, vo, so)) {
            const cpx<T> F = k2m(m) == 0.0 ? czero<T>() : czero<T>() - a[m];
            nxt = rk_apply<STG, C::STORE>(sa, foff, vo, so, in[q], F, efac(1 + s, exy, m), h, false);
          }
          a[m] = guard(nxt);
        }
        __builtin_amdgcn_sched_barrier(0);
      });
    } else {
#pragma unroll
      for (int m = 0; m < E; ++m) {
        uint32_t vo, so;
        cpx<T> nxt = czero<T>();
        if (state_at(m, vo, so)) {
          const double k2m_ = k2m(m);
          const cpx<T> F = k2m_ == 0.0 ? czero<T>() : czero<T>() - a[m];
          nxt = rk_update<STG, C::STORE>(sa, foff, vo, so, F, dif * k2m_, efac(1 + s, exy, m), h, true, expl);
        }
        a[m] = nxt;
      }
    }
    if constexpr (FUSE) inverse_out(a, 5 + 2 * s, 6 + 2 * s, [&] { fetch(s > 0 ? 2 + s : 0, nx); });
  }
  // velocity: F = P(k) c_hat + A 1_band u_hat
  {
    cpx<T> c1[E], c2[E], c3[E];
#if PSDNS_FUSED_PF
    if constexpr (DL) {
      // one component at a time: each with its kept transform, then the next
      fetch(0, c1);
      fft<N, E, false>(c1, lds, j, tw);
      average(0, c1);
      fetch(1, c2);
      fft<N, E, false>(c2, lds, j, tw);
      average(1, c2);
      fetch(2, c3);
      fft<N, E, false>(c3, lds, j, tw);
      average(2, c3);
    } else {
    // the next component's loads are in flight while the current one is transformed
    if constexpr (FUSE) {
#pragma unroll
      for (int m = 0; m < E; ++m) c1[m] = nx[m];
    } else {
      fetch(0, c1);
    }
    fetch(1, c2);
    fft<N, E, false>(c1, lds, j, tw);
    fetch(2, c3);
    fft<N, E, false>(c2, lds, j, tw);
    fft<N, E, false>(c3, lds, j, tw);
    }
#else
    fetch(0, c1);
    fft<N, E, false>(c1, lds, j, tw);
    fetch(1, c2);
    fft<N, E, false>(c2, lds, j, tw);
    fetch(2, c3);
    fft<N, E, false>(c3, lds, j, tw);
    average(0, c1);
    average(1, c2);
    average(2, c3);
#endif
    if ((sp.forcing == PSDNS_FORCING_STOCHASTIC || sp.forcing == PSDNS_FORCING_ALVELIUS) && valid) {
      // the stochastic forcing term of the band modes (solenoidal, from k_stochastic_update)
      // joins the transformed product; the projection below leaves it unchanged
      int kfs = 0;
      while ((double)(kfs + 1) * (kfs + 1) <= sp.kf2) ++kfs;
      if (kfs > g.K) kfs = g.K;
#pragma unroll
      for (int m = 0; m < E; ++m) {
        const double k2m_ = k2m(m);
        if (k2m_ > 0.0 && k2m_ <= sp.kf2) {
          const int kz = wave_of(j + TT * m, N);
          const double* f =
              sa.fband + ((long long)slot * kStochCand + kx + (kfs + 1) * ((ky + kfs) + (2 * kfs + 1) * (kz + kfs))) * 12 + 6;
          c1[m] = c1[m] + cpx<T>{T(f[0]), T(f[1])};
          c2[m] = c2[m] + cpx<T>{T(f[2]), T(f[3])};
          c3[m] = c3[m] + cpx<T>{T(f[4]), T(f[5])};
        }
      }
    }
    const double nu = sp.nu;
    const double exy = exy_of(0);
    const long long f1 = sslot, f2 = sslot + g.st_field, f3 = sslot + 2 * g.st_field;
    if constexpr (FUSE) {
      // P(k) c_hat + A 1_band u_hat in place of c1..c3 (before any store of the velocity
      // update), then the update one component at a time, each in two batches of E/2
      // elements (their loads, then their arithmetic and stores)
#pragma unroll
      for (int m = 0; m < E; ++m) {
        uint32_t vo, so;
        if (!state_at(m, vo, so)) continue;
        const double k2m_ = k2m(m);
        if (k2m_ == 0.0) {
          c1[m] = c2[m] = c3[m] = czero<T>();
          continue;
        }
        const T kzt = T(wave_of(j + TT * m, N)), kyt = T(ky), kxt = T(kx);
        const T ik2 = T(1) / T(k2m_);  // k2m_ is an integer below 2^24: exact in T
        const cpx<T> kdc = kxt * c1[m] + kyt * c2[m] + kzt * c3[m];
        c1[m] = c1[m] - (kxt * ik2) * kdc;
        c2[m] = c2[m] - (kyt * ik2) * kdc;
        c3[m] = c3[m] - (kzt * ik2) * kdc;
        if (A != 0.0 && k2m_ <= sp.kf2) {
          const T At = T(A);
          c1[m] = c1[m] + At * bload(make_buf<T>(sa.sin + f1), vo, so);
          c2[m] = c2[m] + At * bload(make_buf<T>(sa.sin + f2), vo, so);
          c3[m] = c3[m] + At * bload(make_buf<T>(sa.sin + f3), vo, so);
        }
      }
      auto component = [&](cpx<T> (&cv)[E], long long fo) {
        constexpr int HB = E / 2;
        static_for<0, 2>([&](auto hc) {
          constexpr int h0 = decltype(hc)::value * HB;
          RkIn<T> in[HB];
#pragma unroll
          for (int q = 0; q < HB; ++q) {
            uint32_t vo, so;
            if (state_at(h0 + q, vo, so)) in[q] = rk_load<STG>(sa, fo, vo, so);
          }
#pragma unroll
          for (int q = 0; q < HB; ++q) {
            const int m = h0 + q;
            uint32_t vo, so;
            cpx<T> nxt = czero<T>();
            if (state_at(m, vo, so)) {
              const double k2m_ = k2m(m);
              // the next stage reads y_stage on the band (forcing amplitude and term)
              const bool band = k2m_ > 0.0 && k2m_ <= sp.kf2;
              nxt = rk_apply<STG, C::STORE>(sa, fo, vo, so, in[q], cv[m], efac(0, exy, m), h, band);
            }
            cv[m] = guard(nxt);
          }
          __builtin_amdgcn_sched_barrier(0);
        });
      };
      component(c1, f1);
      __builtin_amdgcn_sched_barrier(0);
      component(c2, f2);
      __builtin_amdgcn_sched_barrier(0);
      component(c3, f3);
    } else {
#pragma unroll
      for (int m = 0; m < E; ++m) {
        uint32_t vo, so;
        cpx<T> n1 = czero<T>(), n2 = czero<T>(), n3 = czero<T>();
        if (state_at(m, vo, so)) {
          const double k2m_ = k2m(m);
          const int n = j + TT * m;
          const T kzt = T(wave_of(n, N)), kyt = T(ky), kxt = T(kx);
          cpx<T> F1, F2, F3;
          const bool band = k2m_ > 0.0 && k2m_ <= sp.kf2;
          if (k2m_ == 0.0) {
            F1 = F2 = F3 = czero<T>();
          } else {
            const T ik2 = T(1) / T(k2m_);  // k2m_ is an integer below 2^24: exact in T
            const cpx<T> kdc = kxt * c1[m] + kyt * c2[m] + kzt * c3[m];
            F1 = c1[m] - (kxt * ik2) * kdc;
            F2 = c2[m] - (kyt * ik2) * kdc;
            F3 = c3[m] - (kzt * ik2) * kdc;
            if (A != 0.0 && band) {
              const T At = T(A);
              F1 = F1 + At * bload(make_buf<T>(sa.sin + f1), vo, so);
              F2 = F2 + At * bload(make_buf<T>(sa.sin + f2), vo, so);
              F3 = F3 + At * bload(make_buf<T>(sa.sin + f3), vo, so);
            }
          }
          const double lk2 = nu * k2m_;
          const double ef = efac(0, exy, m);
          n1 = rk_update<STG, C::STORE>(sa, f1, vo, so, F1, lk2, ef, h, true, expl);
          n2 = rk_update<STG, C::STORE>(sa, f2, vo, so, F2, lk2, ef, h, true, expl);
          n3 = rk_update<STG, C::STORE>(sa, f3, vo, so, F3, lk2, ef, h, true, expl);
        }
        c1[m] = n1;
        c2[m] = n2;
        c3[m] = n3;
      }
    }
    if constexpr (FUSE) {
      inverse_out(c1, 0, 3, nothing);
      inverse_out(c2, 1, 4, nothing);
      inverse_out(c3, 2, -1, nothing);
    }
  }
}

// ---------------------------------------------------------------------------
// pressure (Sec. 2.2): with u.grad u = grad(|u|^2/2) - u x omega,
//   p_hat = i k.(u.grad u)^ / |k|^2 = -(|u|^2/2)^ - i k.c_hat / |k|^2,  c = u x omega,
// and p_hat(0) = 0.  A fields 0..3 hold c1, c2, c3 and |u|^2/2 after the y forward
// pass; the z forward transform is followed by this assembly, written to one compact
// field per slot (rows (kz_c, ky_c), PX apart in kx).
// ---------------------------------------------------------------------------
template <int N, typename T>
__global__ void PSDNS_COL_BOUNDS(Cfg<N, T>::COL_THREADS)
k_z_forward_pressure(const cpx<T>* __restrict__ abuf, cpx<T>* __restrict__ pout, const cpx<T>* __restrict__ tw_g,
                     const SlotDev* __restrict__ slots, Geom g) {
  using C = Cfg<N, T>;
  constexpr int W = C::W, E = C::EC, TT = C::TC;
  constexpr int K = (N - 1) / 3;
  constexpr int M = 2 * K + 1;
  constexpr uint32_t CS = sizeof(cpx<T>);
  using L = ColLds<N, T, W>;
  __shared__ cpx<T> smem[L::kEntries];
  __shared__ cpx<T> stw[N];
  const int slot = blockIdx.z;
  if (!slots[slot].active) return;
  stage_twiddles<N>(stw, tw_g);
  const cpx<T>* tw = stw;
  const int c = threadIdx.x % W;
  const int j = threadIdx.x / W;
  const int kx = blockIdx.x * W + c;
  const int kyc = blockIdx.y;
  const bool valid = kx < g.KX;
  const typename L::View lds{smem + c};
  const uint32_t rsb = (uint32_t)M * g.PX * CS;
  const uint32_t voff = ((uint32_t)j * M * g.PX + (uint32_t)kyc * g.PX + (uint32_t)kx) * CS;
  const cpx<T>* aslot = abuf + (long long)slot * g.FA * g.a_field;
  const int ky = wave_of_compact(kyc, K, M);
  cpx<T> v[E], kdc[E];
  auto load_fwd = [&](int f) {
    const Buf<T> b = make_buf<T>(aslot + (long long)f * g.a_field);
#pragma unroll
    for (int m = 0; m < E; ++m) v[m] = valid ? bload(b, voff, (uint32_t)(TT * m) * rsb) : czero<T>();
    fft<N, E, false>(v, lds, j, tw);
  };
  // k . c_hat, one component at a time
  load_fwd(0);
#pragma unroll
  for (int m = 0; m < E; ++m) kdc[m] = T(kx) * v[m];
  load_fwd(1);
#pragma unroll
  for (int m = 0; m < E; ++m) kdc[m] = kdc[m] + T(ky) * v[m];
  load_fwd(2);
#pragma unroll
  for (int m = 0; m < E; ++m) kdc[m] = kdc[m] + T(wave_of(j + TT * m, N)) * v[m];
  load_fwd(3);
  if (!valid) return;
  const Buf<T> out = make_buf<T>(pout + (long long)slot * g.st_field);
#pragma unroll
  for (int m = 0; m < E; ++m) {
    uint32_t vo, so;
    if (!compact_at<N, TT>(m, j, voff, rsb, vo, so)) continue;
    const int kz = wave_of(j + TT * m, N);
    const double k2 = double(kx) * kx + double(ky) * ky + double(kz) * kz;
    cpx<T> p = czero<T>();
    if (k2 > 0.0) p = czero<T>() - v[m] - mul_is(kdc[m], T(1.0 / k2));
    bstore<C::Col::STORE>(out, vo, so, p);
  }
}

// ---------------------------------------------------------------------------
// forcing amplitude A = P / (2 E_f), E_f = 1/2 sum_{0<|k|^2<=kf^2} |u_hat|^2 / N^6 (FP64)
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256)
k_forcing_amplitude(const cpx<T>* __restrict__ sin, const SlotDev* __restrict__ slots, DynDev* __restrict__ dyn,
                    Geom g) {
  __shared__ double red[256];
  const int slot = blockIdx.x;
  const SlotDev& sp = slots[slot];
  if (!sp.active) return;
  // every stage starts a fresh grid maximum (only stage 0's x pass contributes to it)
  if (threadIdx.x == 0) dyn[slot].umax = 0ull;
  if (sp.forcing != PSDNS_FORCING_POWER) {
    // the hold scheme acts after the last stage only (k_band_hold)
    if (threadIdx.x == 0) dyn[slot].A = 0.0;
    return;
  }
  int kf = 0;
  while ((double)(kf + 1) * (kf + 1) <= sp.kf2) ++kf;
  if (kf > g.K) kf = g.K;
  const int span = 2 * kf + 1;
  const int ncand = (kf + 1) * span * span;
  double e = 0.0;
  const cpx<T>* base = sin + (long long)slot * g.F * g.st_field;
  for (int i = threadIdx.x; i < ncand; i += 256) {
    const int kx = i % (kf + 1);
    const int ky = (i / (kf + 1)) % span - kf;
    const int kz = i / ((kf + 1) * span) - kf;
    const double k2 = double(kx) * kx + double(ky) * ky + double(kz) * kz;
    if (k2 == 0.0 || k2 > sp.kf2) continue;
    const int kyc = ky >= 0 ? ky : ky + g.M;
    const int kzc = kz >= 0 ? kz : kz + g.M;
    const long long o = st_row(kzc, kyc, g.M, g.PX) + kx;
    double s = 0.0;
    for (int f = 0; f < 3; ++f) {
      const cpx<T> v = base[o + f * g.st_field];
      s += double(v.x) * double(v.x) + double(v.y) * double(v.y);
    }
    e += (kx == 0 ? 0.5 : 1.0) * s;
  }
  red[threadIdx.x] = e;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double n3 = double(g.N) * g.N * g.N;
    const double ef = red[0] / (n3 * n3);
    dyn[slot].A = (sp.power > 0.0 && ef > 0.0) ? sp.power / (2.0 * ef) : 0.0;
  }
}

// ---------------------------------------------------------------------------
// band-energy hold (the paper's deterministic forcing, Sec. 2.3), after the last stage:
// E_f of y_{n+1} over 0 < |k|^2 <= kf^2 (FP64, the summation order of
// k_forcing_amplitude), then the band modes of u scaled by sqrt(target / E_f)
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256)
k_band_hold(cpx<T>* __restrict__ state, const SlotDev* __restrict__ slots, Geom g) {
  __shared__ double red[256];
  const int slot = blockIdx.x;
  const SlotDev& sp = slots[slot];
  if (!sp.active || sp.forcing != PSDNS_FORCING_HOLD) return;
  int kf = 0;
  while ((double)(kf + 1) * (kf + 1) <= sp.kf2) ++kf;
  if (kf > g.K) kf = g.K;
  const int span = 2 * kf + 1;
  const int ncand = (kf + 1) * span * span;
  cpx<T>* base = state + (long long)slot * g.F * g.st_field;
  auto mode_at = [&](int i, long long& o) {
    const int kx = i % (kf + 1);
    const int ky = (i / (kf + 1)) % span - kf;
    const int kz = i / ((kf + 1) * span) - kf;
    const double k2 = double(kx) * kx + double(ky) * ky + double(kz) * kz;
    const int kyc = ky >= 0 ? ky : ky + g.M;
    const int kzc = kz >= 0 ? kz : kz + g.M;
    o = st_row(kzc, kyc, g.M, g.PX) + kx;
    return !(k2 == 0.0 || k2 > sp.kf2) ? (kx == 0 ? 1 : 2) : 0;
  };
  double e = 0.0;
  for (int i = threadIdx.x; i < ncand; i += 256) {
    long long o;
    const int w = mode_at(i, o);
    if (!w) continue;
    double s = 0.0;
    for (int f = 0; f < 3; ++f) {
      const cpx<T> v = base[o + f * g.st_field];
      s += double(v.x) * double(v.x) + double(v.y) * double(v.y);
    }
    e += (w == 1 ? 0.5 : 1.0) * s;
  }
  red[threadIdx.x] = e;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  const double n3 = double(g.N) * g.N * g.N;
  const double ef = red[0] / (n3 * n3);
  if (!(ef > 0.0)) return;
  const T fac = T(sqrt(sp.hold / ef));
  for (int i = threadIdx.x; i < ncand; i += 256) {
    long long o;
    if (!mode_at(i, o)) continue;
    for (int f = 0; f < 3; ++f) base[o + f * g.st_field] = fac * base[o + f * g.st_field];
  }
}

// ---------------------------------------------------------------------------
// step size from the stage-0 maxima (Eq. (10)) and the step record
// ---------------------------------------------------------------------------
static __global__ void __launch_bounds__(256)
k_step_dt(const SlotDev* __restrict__ slots, DynDev* __restrict__ dyn, Geom g, double dt_arg) {
  const int slot = blockIdx.x;
  if (!slots[slot].active) return;
  if (threadIdx.x == 0) {
    DynDev& d = dyn[slot];
    const double m = __longlong_as_double((long long)d.umax);
    const double dx = 6.283185307179586476925286766559 / g.N;
    double dt = dt_arg;
    int fl = d.flags;
    if (!(m == m) || m > 1.79769313486231570e308) fl |= PSDNS_FLAG_NONFINITE;
    if (dt_arg < 0.0) dt = (m > 0.0 && m == m) ? (-dt_arg) * dx / m : 0.0;
    if (dt * m / dx > 1.0) fl |= PSDNS_FLAG_CFL;
    d.dt = dt;
    d.max_u = m;
    d.t += dt;
    d.steps += 1;
    d.flags = fl;
  }
}

// ---------------------------------------------------------------------------
// initial condition (Sec. 2.3, Rogallo construction; SplitMix64 phases)
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t splitmix64_at(uint64_t seed, uint64_t counter) {
  uint64_t z = seed + (counter + 1ull) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
__device__ __forceinline__ double unit_double(uint64_t x) { return double(x >> 11) * (1.0 / 9007199254740992.0); }

// ---------------------------------------------------------------------------
// stochastic band forcing (the option of Sec. 2.3 after Eswaran & Pope): once per step,
// after the step size is known, b <- a b + sigma sqrt(1 - a^2) xi for every band mode,
// a = exp(-dt / T_L), xi from Box-Muller normals keyed by (step, candidate, component,
// part); the modes (0, ky, kz) with ky < 0, or ky = 0 and kz < 0, then take the conjugate
// of their partner so that the forcing is real.  One block per slot.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double normal_at(uint64_t seed, uint64_t q) {
  const double u1 = unit_double(splitmix64_at(seed, 2 * q));
  const double u2 = unit_double(splitmix64_at(seed, 2 * q + 1));
  return sqrt(-2.0 * log(1.0 - u1)) * cos(6.283185307179586476925286766559 * u2);
}

// Alvelius-type band forcing (the second stochastic option of Sec. 2.3), drawn once per step
// from y_n with that step's h: at band mode k, f = F (g_A e^{i th1} e1 + g_B e^{i th2} e2),
// g_A = sin 2 phi, g_B = cos 2 phi, phi and psi uniform (SplitMix64 uniforms 2q, 2q + 1,
// q = n C + i), th2 = th1 + psi, th1 = atan2(-a, b) (0 when a = b = 0) so that
// Re(conj(u_hat) . f) = 0, with xi_j = u_hat . e_j and
//   a = g_A Re xi1 + g_B (Re xi2 cos psi + Im xi2 sin psi),
//   b = g_A Im xi1 + g_B (Im xi2 cos psi - Re xi2 sin psi);
// F = N^3 sqrt(2 P / (h W)), W the half-spectrum count of band modes, so that the
// force-force term injects P: (h/2) sum w |f|^2 / N^6 = P.  Written to the forcing-term
// entries of the band table.
template <typename T>
__device__ void alvelius_mode(int kx, int ky, int kz, const cpx<T>* __restrict__ ybase, long long stf, int M, int PX,
                              uint64_t seed, uint64_t q, double amp, double* __restrict__ e) {
  const double two_pi = 6.283185307179586476925286766559;
  const double phi = two_pi * unit_double(splitmix64_at(seed, 2 * q));
  const double psi = two_pi * unit_double(splitmix64_at(seed, 2 * q + 1));
  const double ga = sin(2.0 * phi), gb = cos(2.0 * phi);
  const double fx = kx, fy = ky, fz = kz;
  const double kmag = sqrt(fx * fx + fy * fy + fz * fz);
  const double kperp = sqrt(fx * fx + fy * fy);
  double e1[3], e2[3];
  if (kperp == 0.0) {
    e1[0] = 1.0; e1[1] = 0.0; e1[2] = 0.0;
  } else {
    e1[0] = fy / kperp; e1[1] = -fx / kperp; e1[2] = 0.0;
  }
  e2[0] = (fy * e1[2] - fz * e1[1]) / kmag;
  e2[1] = (fz * e1[0] - fx * e1[2]) / kmag;
  e2[2] = (fx * e1[1] - fy * e1[0]) / kmag;
  const int kyc = ky >= 0 ? ky : ky + M, kzc = kz >= 0 ? kz : kz + M;
  const long long o = st_row(kzc, kyc, M, PX) + kx;
  double x1r = 0.0, x1i = 0.0, x2r = 0.0, x2i = 0.0;
  for (int c = 0; c < 3; ++c) {
    const cpx<T> u = ybase[o + c * stf];
    x1r += double(u.x) * e1[c];
    x1i += double(u.y) * e1[c];
    x2r += double(u.x) * e2[c];
    x2i += double(u.y) * e2[c];
  }
  const double cp = cos(psi), sp = sin(psi);
  const double a = ga * x1r + gb * (x2r * cp + x2i * sp);
  const double b = ga * x1i + gb * (x2i * cp - x2r * sp);
  const double th1 = (a != 0.0 || b != 0.0) ? atan2(-a, b) : 0.0;
  const double th2 = th1 + psi;
  const double ar = amp * ga * cos(th1), ai = amp * ga * sin(th1);
  const double br = amp * gb * cos(th2), bi = amp * gb * sin(th2);
  for (int c = 0; c < 6; ++c) e[c] = 0.0;
  for (int c = 0; c < 3; ++c) {
    e[6 + 2 * c] = ar * e1[c] + br * e2[c];
    e[6 + 2 * c + 1] = ai * e1[c] + bi * e2[c];
  }
}

template <typename T>
__global__ void __launch_bounds__(256)
k_stochastic_update(const cpx<T>* __restrict__ yn, const SlotDev* __restrict__ slots, const DynDev* __restrict__ dyn,
                    double* __restrict__ fband, Geom g) {
  const int slot = blockIdx.x;
  const SlotDev& sp = slots[slot];
  if (!sp.active || (sp.forcing != PSDNS_FORCING_STOCHASTIC && sp.forcing != PSDNS_FORCING_ALVELIUS)) return;
  const bool alv = sp.forcing == PSDNS_FORCING_ALVELIUS;
  int kf = 0;
  while ((double)(kf + 1) * (kf + 1) <= sp.kf2) ++kf;
  if (kf > g.K) kf = g.K;
  const int span = 2 * kf + 1;
  const int ncand = (kf + 1) * span * span;
  const double h = dyn[slot].dt;
  const uint64_t n = (uint64_t)dyn[slot].steps;
  const double a = exp(-h / sp.tl);
  const double c = sp.sigma * sqrt(fmax(0.0, 1.0 - a * a));
  // per candidate: b (3 complex) then the forcing term (3 complex)
  double* tab = fband + (long long)slot * kStochCand * 12;
  auto decode = [&](int i, int& kx, int& ky, int& kz) {
    kx = i % (kf + 1);
    ky = (i / (kf + 1)) % span - kf;
    kz = i / ((kf + 1) * span) - kf;
    const double k2 = double(kx) * kx + double(ky) * ky + double(kz) * kz;
    return k2 > 0.0 && k2 <= sp.kf2;
  };
  double amp = 0.0;
  if (alv) {
    // W: band modes counted with their half-spectrum multiplicity (the same count on every thread)
    double wsum = 0.0;
    for (int i = 0; i < ncand; ++i) {
      int kx, ky, kz;
      if (decode(i, kx, ky, kz)) wsum += kx == 0 ? 1.0 : 2.0;
    }
    const double n3 = double(g.N) * g.N * g.N;
    amp = (sp.power > 0.0 && h > 0.0 && wsum > 0.0) ? n3 * sqrt(2.0 * sp.power / (h * wsum)) : 0.0;
  }
  const cpx<T>* ybase = yn + (long long)slot * g.F * g.st_field;
  for (int i = threadIdx.x; i < ncand; i += blockDim.x) {
    int kx, ky, kz;
    if (!decode(i, kx, ky, kz)) continue;
    if (kx == 0 && (ky < 0 || (ky == 0 && kz < 0))) continue;
    double* e = tab + i * 12;
    if (alv) {
      alvelius_mode<T>(kx, ky, kz, ybase, g.st_field, g.M, g.PX, sp.seed, n * (uint64_t)ncand + (uint64_t)i, amp, e);
      continue;
    }
    for (int comp = 0; comp < 3; ++comp) {
      const uint64_t q = ((n * (uint64_t)ncand + (uint64_t)i) * 3 + (uint64_t)comp) * 2;
      e[2 * comp] = a * e[2 * comp] + c * normal_at(sp.seed, q);
      e[2 * comp + 1] = a * e[2 * comp + 1] + c * normal_at(sp.seed, q + 1);
    }
    // the term in the unnormalised state: N^3 P(k) b
    const double n3 = double(g.N) * g.N * g.N;
    const double k[3] = {double(kx), double(ky), double(kz)};
    const double k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
    const double kbr = (k[0] * e[0] + k[1] * e[2] + k[2] * e[4]) / k2;
    const double kbi = (k[0] * e[1] + k[1] * e[3] + k[2] * e[5]) / k2;
    for (int comp = 0; comp < 3; ++comp) {
      e[6 + 2 * comp] = n3 * (e[2 * comp] - k[comp] * kbr);
      e[6 + 2 * comp + 1] = n3 * (e[2 * comp + 1] - k[comp] * kbi);
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < ncand; i += blockDim.x) {
    int kx, ky, kz;
    if (!decode(i, kx, ky, kz)) continue;
    if (!(kx == 0 && (ky < 0 || (ky == 0 && kz < 0)))) continue;
    const int p = (kf + 1) * ((-ky + kf) + span * (-kz + kf));  // candidate of (0, -ky, -kz)
    for (int r = 0; r < 12; r += 2) {
      tab[i * 12 + r] = tab[p * 12 + r];
      tab[i * 12 + r + 1] = -tab[p * 12 + r + 1];
    }
  }
}

// Initial energy spectrum shape E(kappa): kind 0 the configured kappa^4 exp(-2 (kappa/kp)^2);
// kind 1 the paper's spectrum (Sec. 2.3, after Lamorgese et al.) with kp = k_F:
// (1/k_F) (kappa/k_F)^2 up to k_F and (1/k_F) (kappa/k_F)^(-5/3) beyond (u_rms = 1).
static __device__ double init_spectrum(double kmag, double kp, int kind) {
  const double q = kmag / kp;
  if (kind == 1) return (q <= 1.0 ? q * q : pow(q, -5.0 / 3.0)) / kp;
  return kmag * kmag * kmag * kmag * exp(-2.0 * q * q);
}

// Coefficient vector of the canonical mode (kx, ky, kz) before the energy scaling.
static __device__ void rogallo_mode(int kx, int ky, int kz, int N, uint64_t seed, double kp, int kind,
                                    double (&re)[3], double (&im)[3]) {
  const double fx = kx, fy = ky, fz = kz;
  const double k2 = fx * fx + fy * fy + fz * fz;
  const double kmag = sqrt(k2);
  const double spec = init_spectrum(kmag, kp, kind);
  const double amp = sqrt(spec / (4.0 * 3.14159265358979323846 * kmag * kmag));
  const double kperp = sqrt(fx * fx + fy * fy);
  double e1[3], e2[3];
  if (kperp == 0.0) {
    e1[0] = 1.0; e1[1] = 0.0; e1[2] = 0.0;
  } else {
    e1[0] = fy / kperp; e1[1] = -fx / kperp; e1[2] = 0.0;
  }
  e2[0] = (fy * e1[2] - fz * e1[1]) / kmag;
  e2[1] = (fz * e1[0] - fx * e1[2]) / kmag;
  e2[2] = (fx * e1[1] - fy * e1[0]) / kmag;
  const int NX = N / 2 + 1;
  const uint64_t iz = (uint64_t)((kz % N + N) % N), iy = (uint64_t)((ky % N + N) % N);
  const uint64_t lin = (iz * (uint64_t)N + iy) * (uint64_t)NX + (uint64_t)kx;
  const double two_pi = 6.283185307179586476925286766559;
  const double th1 = two_pi * unit_double(splitmix64_at(seed, 3 * lin + 0));
  const double th2 = two_pi * unit_double(splitmix64_at(seed, 3 * lin + 1));
  const double psi = two_pi * unit_double(splitmix64_at(seed, 3 * lin + 2));
  const double ca = cos(psi), sa = sin(psi);
  const double ar = cos(th1) * ca, ai = sin(th1) * ca;
  const double br = cos(th2) * sa, bi = sin(th2) * sa;
  const double scale = double(N) * N * N * amp;
  for (int c = 0; c < 3; ++c) {
    re[c] = scale * (ar * e1[c] + br * e2[c]);
    im[c] = scale * (ai * e1[c] + bi * e2[c]);
  }
}

// coefficient of any retained mode (mirror modes of the kx = 0 plane by conjugation)
static __device__ void init_coeff(int kx, int ky, int kz, int N, uint64_t seed, double kp, int kind,
                                  double (&re)[3], double (&im)[3]) {
  if (kx == 0 && ky == 0 && kz == 0) {
    for (int c = 0; c < 3; ++c) re[c] = im[c] = 0.0;
    return;
  }
  const bool canon = kx > 0 || (kx == 0 && ky > 0) || (kx == 0 && ky == 0 && kz > 0);
  if (canon) {
    rogallo_mode(kx, ky, kz, N, seed, kp, kind, re, im);
  } else {
    rogallo_mode(0, -ky, -kz, N, seed, kp, kind, re, im);
    for (int c = 0; c < 3; ++c) im[c] = -im[c];
  }
}

static __global__ void __launch_bounds__(256)
k_init_energy(Geom g, uint64_t seed, double kp, int kind, double* __restrict__ part) {
  __shared__ double red[256];
  const long long nmodes = (long long)g.M * g.M * g.KX;
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  double e = 0.0;
  if (i < nmodes) {
    const int kx = (int)(i % g.KX);
    const int kyc = (int)((i / g.KX) % g.M);
    const int kzc = (int)(i / ((long long)g.KX * g.M));
    double re[3], im[3];
    const int ky = wave_of_compact(kyc, g.K, g.M), kz = wave_of_compact(kzc, g.K, g.M);
    init_coeff(kx, ky, kz, g.N, seed, kp, kind, re, im);
    double s = 0.0;
    for (int c = 0; c < 3; ++c) s += re[c] * re[c] + im[c] * im[c];
    e = retained(g, kx, ky, kz) ? (kx == 0 ? 0.5 : 1.0) * s : 0.0;
  }
  red[threadIdx.x] = e;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

static __global__ void __launch_bounds__(256)
k_init_scale(const double* __restrict__ part, int nblocks, double energy, int N, DynDev* __restrict__ d) {
  __shared__ double red[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < nblocks; i += 256) s += part[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double n3 = double(N) * N * N;
    const double k = red[0] / (n3 * n3);
    d->scratch = k > 0.0 ? sqrt(energy / k) : 0.0;
  }
}

template <typename T>
__global__ void __launch_bounds__(256)
k_init_write(cpx<T>* __restrict__ st, Geom g, int slot, uint64_t seed, double kp, int kind,
             const DynDev* __restrict__ d) {
  const long long nmodes = (long long)g.M * g.M * g.KX;
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i >= nmodes) return;
  const int kx = (int)(i % g.KX);
  const int kyc = (int)((i / g.KX) % g.M);
  const int kzc = (int)(i / ((long long)g.KX * g.M));
  double re[3], im[3];
  const int ky = wave_of_compact(kyc, g.K, g.M), kz = wave_of_compact(kzc, g.K, g.M);
  init_coeff(kx, ky, kz, g.N, seed, kp, kind, re, im);
  const double sc = retained(g, kx, ky, kz) ? d->scratch : 0.0;
  const long long o = st_row(kzc, kyc, g.M, g.PX) + kx;
  cpx<T>* base = st + (long long)slot * g.F * g.st_field;
  for (int c = 0; c < 3; ++c) base[o + c * g.st_field] = {T(sc * re[c]), T(sc * im[c])};
  for (int s = 0; s < g.S; ++s) base[o + (3 + s) * g.st_field] = czero<T>();
}

// ---------------------------------------------------------------------------
// canonical <-> compact conversion of one slot
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_fill_zero(cpx<T>* __restrict__ p, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = czero<T>();
}

template <typename T, bool TO_CANON>
__global__ void __launch_bounds__(256)
k_convert(cpx<T>* __restrict__ st, cpx<T>* __restrict__ canon, Geom g, int slot) {
  const long long per = (long long)g.M * g.M * g.KX;
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i >= per * g.F) return;
  const int f = (int)(i / per);
  const long long r = i % per;
  const int kx = (int)(r % g.KX);
  const int kyc = (int)((r / g.KX) % g.M);
  const int kzc = (int)(r / ((long long)g.KX * g.M));
  const int N = g.N, NX = N / 2 + 1;
  const int ky = wave_of_compact(kyc, g.K, g.M), kz = wave_of_compact(kzc, g.K, g.M);
  const int iy = (ky + N) % N;
  const int iz = (kz + N) % N;
  const long long oc = (((long long)f * N + iz) * N + iy) * NX + kx;
  const long long os = (long long)slot * g.F * g.st_field + (long long)f * g.st_field +
                       st_row(kzc, kyc, g.M, g.PX) + kx;
  // modes of the bounding cube outside a spherical retained set are not part of the state
  const bool in = retained(g, kx, ky, kz);
  if (TO_CANON)
    canon[oc] = in ? st[os] : czero<T>();
  else
    st[os] = in ? canon[oc] : czero<T>();
}

// ---------------------------------------------------------------------------
// spectra and statistics (Table 1, Eqs. (11)-(13)), all accumulated in FP64
// with a fixed summation order (bitwise reproducible, no floating atomics)
// ---------------------------------------------------------------------------
// per shell: [0] sum w |u|^2/2, [1] sum w (|k|^2 |u|^2 + |k.u|^2),
// per scalar s: [2+3s] sum w |phi|^2/2, [3+3s] sum w |k|^2 |phi|^2, [4+3s] sum w Re(conj(phi) g_s.u)
__host__ __device__ inline int shell_quantities(int S) { return 2 + 3 * S; }

__device__ __forceinline__ int isqrt_floor(long long v) {
  if (v <= 0) return 0;
  long long r = (long long)sqrt((double)v);
  while (r * r > v) --r;
  while ((r + 1) * (r + 1) <= v) ++r;
  return (int)r;
}

template <typename T>
__global__ void __launch_bounds__(256)
k_shell_sums(const cpx<T>* __restrict__ st, const SlotDev* __restrict__ slots, Geom g, double* __restrict__ part,
             int ns) {
  constexpr int MAXQ = 2 + 3 * kMaxScalars;
  __shared__ double red[MAXQ][256];
  const int sh = blockIdx.x;
  const int slot = blockIdx.y;
  const SlotDev& sp = slots[slot];
  const int S = g.S, Q = shell_quantities(S), K = g.K, M = g.M;
  const long long lo = sh == 0 ? 0 : (long long)sh * sh - sh + 1;  // nint(|k|) = sh <=> lo <= |k|^2 <= hi
  const long long hi = (long long)sh * sh + sh;
  int R = isqrt_floor(hi);
  if (R > K) R = K;
  const int span = 2 * R + 1;
  double acc[MAXQ];
#pragma unroll
  for (int q = 0; q < MAXQ; ++q) acc[q] = 0.0;
  const cpx<T>* base = st + (long long)slot * g.F * g.st_field;
  for (int p = threadIdx.x; p < span * span; p += 256) {
    const int kz = p / span - R, ky = p % span - R;
    const long long r2 = (long long)kz * kz + (long long)ky * ky;
    if (r2 > hi) continue;
    int x0 = lo - r2 > 0 ? isqrt_floor(lo - r2 - 1) + 1 : 0;  // smallest kx with kx^2 >= lo - r2
    int x1 = isqrt_floor(hi - r2);
    if (x1 > K) x1 = K;
    const int kzc = kz >= 0 ? kz : kz + M, kyc = ky >= 0 ? ky : ky + M;
    const long long row = st_row(kzc, kyc, M, g.PX);
    for (int kx = x0; kx <= x1; ++kx) {
      const long long o = row + kx;
      const double w = kx == 0 ? 1.0 : 2.0;
      const double k2 = double(r2) + double(kx) * kx;
      const cpx<T> a = base[o], b = base[o + g.st_field], c = base[o + 2 * g.st_field];
      const double u1r = a.x, u1i = a.y, u2r = b.x, u2i = b.y, u3r = c.x, u3i = c.y;
      const double uu = u1r * u1r + u1i * u1i + u2r * u2r + u2i * u2i + u3r * u3r + u3i * u3i;
      const double kur = kx * u1r + ky * u2r + kz * u3r, kui = kx * u1i + ky * u2i + kz * u3i;
      acc[0] += 0.5 * w * uu;
      acc[1] += w * (k2 * uu + kur * kur + kui * kui);
#pragma unroll
      for (int s = 0; s < kMaxScalars; ++s) {
        if (s >= S) break;
        const cpx<T> f = base[o + (3 + s) * g.st_field];
        const double fr = f.x, fi = f.y, ff = fr * fr + fi * fi;
        const double gur = sp.g[s][0] * u1r + sp.g[s][1] * u2r + sp.g[s][2] * u3r;
        const double gui = sp.g[s][0] * u1i + sp.g[s][1] * u2i + sp.g[s][2] * u3i;
        acc[2 + 3 * s] += 0.5 * w * ff;
        acc[3 + 3 * s] += w * k2 * ff;
        acc[4 + 3 * s] += w * (fr * gur + fi * gui);
      }
    }
  }
#pragma unroll
  for (int q = 0; q < MAXQ; ++q)
    if (q < Q) red[q][threadIdx.x] = acc[q];
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o)
      for (int q = 0; q < Q; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + o];
    __syncthreads();
  }
  if ((int)threadIdx.x < Q) part[((long long)slot * ns + sh) * Q + threadIdx.x] = red[threadIdx.x][0];
}

// Inverse z transform of up to 8 derived fields i k_axis * (field) of the state
// (axis 0: none, 1: x, 2: y, 3: z); same layout and scaling as k_z_inverse.
struct DerivSpec {
  int nf;
  int field[8];
  int axis[8];
};

template <int N, typename T>
__global__ void PSDNS_COL_BOUNDS(Cfg<N, T>::COL_THREADS)
k_stats_z(const cpx<T>* __restrict__ st, cpx<T>* __restrict__ abuf, const cpx<T>* __restrict__ tw_g, Geom g,
          DerivSpec spec) {
  using C = Cfg<N, T>;
  constexpr int W = C::W, E = C::EC, TT = C::TC;
  constexpr int K = (N - 1) / 3, M = 2 * K + 1;
  __shared__ cpx<T> smem[W * N];
  __shared__ cpx<T> stw[N];
  const int slot = blockIdx.z;
  stage_twiddles<N>(stw, tw_g);
  const cpx<T>* tw = stw;
  const int c = threadIdx.x % W, j = threadIdx.x / W;
  const int kx = blockIdx.x * W + c, kyc = blockIdx.y;
  const bool valid = kx < g.KX;
  const int ky = wave_of_compact(kyc, K, M);
  const LdsCol<T, W> lds{smem + c};
  const T scale = T(1) / (T(N) * T(N) * T(N));
  const cpx<T>* in = st + (long long)slot * g.F * g.st_field + kx;
  cpx<T>* out = abuf + (long long)slot * g.FA * g.a_field + kx;
  cpx<T> a[E];
  for (int f = 0; f < spec.nf; ++f) {
    const cpx<T>* p = in + (long long)spec.field[f] * g.st_field;
    const int ax = spec.axis[f];
#pragma unroll
    for (int m = 0; m < E; ++m) {
      const int kc = compact_of(j + TT * m, N, K, M);
      cpx<T> v = (valid && kc >= 0) ? scale * p[st_row(kc, kyc, M, g.PX)] : czero<T>();
      const T kk = ax == 1 ? T(kx) : ax == 2 ? T(ky) : T(wave_of(j + TT * m, N));
      a[m] = ax == 0 ? v : mul_is(v, kk);
    }
    fft<N, E, true>(a, lds, j, tw);
    if (valid) {
      cpx<T>* q = out + (long long)f * g.a_field;
#pragma unroll
      for (int m = 0; m < E; ++m) q[a_row(j + TT * m, kyc, M, g.PX)] = a[m];
    }
  }
}

// Plain inverse y transform of nf fields (A layout -> B layout).
template <int N, typename T>
__global__ void PSDNS_COL_BOUNDS(Cfg<N, T>::COL_THREADS)
k_stats_y(const cpx<T>* __restrict__ abuf, cpx<T>* __restrict__ bbuf, const cpx<T>* __restrict__ tw_g, Geom g,
          int nf) {
  using C = Cfg<N, T>;
  constexpr int W = C::W, E = C::EC, TT = C::TC;
  constexpr int K = (N - 1) / 3, M = 2 * K + 1;
  __shared__ cpx<T> smem[W * N];
  __shared__ cpx<T> stw[N];
  const int slot = blockIdx.z;
  stage_twiddles<N>(stw, tw_g);
  const cpx<T>* tw = stw;
  const int c = threadIdx.x % W, j = threadIdx.x / W;
  const int kx = blockIdx.x * W + c, z = blockIdx.y;
  const bool valid = kx < g.KX;
  const LdsCol<T, W> lds{smem + c};
  const cpx<T>* in = abuf + (long long)slot * g.FA * g.a_field + a_row(z, 0, M, g.PX) + kx;
  const long long krow = g.PX;
  cpx<T>* out = bbuf + (long long)slot * g.FB * g.b_field + (long long)z * N * g.PX + kx;
  cpx<T> a[E];
  for (int f = 0; f < nf; ++f) {
    const cpx<T>* p = in + (long long)f * g.a_field;
#pragma unroll
    for (int m = 0; m < E; ++m) {
      const int kc = compact_of(j + TT * m, N, K, M);
      a[m] = (valid && kc >= 0) ? p[kc * krow] : czero<T>();
    }
    fft<N, E, true>(a, lds, j, tw);
    if (valid) {
      cpx<T>* q = out + (long long)f * g.b_field;
#pragma unroll
      for (int m = 0; m < E; ++m) q[(long long)(j + TT * m) * g.PX] = a[m];
    }
  }
}

// x inverse of nf (<= 6) B fields per line; FP64 sums of f^2, f^3, f^4 for the
// fields [mom0, nf) and max |u1|+|u2|+|u3| when fields 0..2 are the velocity
// (with_max).  Fixed grid with a fixed line assignment; one partial record per block:
// [3 * (nf - mom0)] moments then the max.
template <int N, typename T>
__global__ void PSDNS_X_BOUNDS(Cfg<N, T>::X_THREADS)
k_x_moments(const cpx<T>* __restrict__ bbuf, const cpx<T>* __restrict__ tw_g, Geom g, int nf, int mom0,
            int with_max, double* __restrict__ part) {
  using C = Cfg<N, T>;
  using XL = XLine<N, T>;
  constexpr int E = C::EX, TT = C::TX, L = C::LX, LP = C::LP, NQ = XL::NQ;
  __shared__ cpx<T> smem[L * LP];
  __shared__ cpx<T> stw[N];
  __shared__ double red[C::X_THREADS];
  __shared__ cpx<T> xch[XL::kXch > 0 ? XL::kXch * C::X_THREADS : 1];
  const int slot = blockIdx.y;
  stage_twiddles<N>(stw, tw_g);
  const cpx<T>* tw = stw;
  const XL xl(threadIdx.x, xch);
  const int li = threadIdx.x / TT, j = xl.j;
  const LdsLine<T, N, E> lds{smem + li * LP};
  double mom[6][3];
#pragma unroll
  for (int f = 0; f < 6; ++f) mom[f][0] = mom[f][1] = mom[f][2] = 0.0;
  double mx = 0.0;
  const long long nlines = (long long)N * N;
  for (long long l0 = (long long)blockIdx.x * L; l0 < nlines; l0 += (long long)gridDim.x * L) {
    const cpx<T>* bblock = bbuf + (long long)slot * g.FB * g.b_field + l0 * g.PX;
    const uint32_t voff = ((uint32_t)li * g.PX + (uint32_t)j) * (uint32_t)sizeof(cpx<T>);
    T u12x[E], u12y[E];
#pragma unroll
    for (int f = 0; f < 6; f += 2) {
      if (f >= nf) break;
      cpx<T> ra[NQ], rb[NQ], h[E];
      xl.load(make_buf<T>(bblock + (long long)f * g.b_field), voff, ra);
      if (f + 1 < nf) {
        xl.load(make_buf<T>(bblock + (long long)(f + 1) * g.b_field), voff, rb);
      } else {
#pragma unroll
        for (int q = 0; q < NQ; ++q) rb[q] = czero<T>();
      }
      xl.build(ra, rb, h);
      fft<N, E, true, typename XL::Sync>(h, lds, j, tw);
#pragma unroll
      for (int m = 0; m < E; ++m) {
        const double vx = h[m].x, vy = h[m].y;
        if (f >= mom0) {
          const double v2 = vx * vx;
          mom[f][0] += v2;
          mom[f][1] += v2 * vx;
          mom[f][2] += v2 * v2;
        }
        if (f + 1 < nf && f + 1 >= mom0) {
          const double v2 = vy * vy;
          mom[f + 1][0] += v2;
          mom[f + 1][1] += v2 * vy;
          mom[f + 1][2] += v2 * v2;
        }
        if (with_max && f == 0) {
          u12x[m] = h[m].x;
          u12y[m] = h[m].y;
        }
        if (with_max && f == 2) {
          const double sm = fabs((double)u12x[m]) + fabs((double)u12y[m]) + fabs(vx);
          mx = (sm > mx || sm != sm) ? sm : mx;
        }
      }
    }
  }
  const int nm = nf - mom0;
  double* out = part + ((long long)slot * gridDim.x + blockIdx.x) * (3 * 6 + 1);
  for (int q = 0; q < 3 * nm + 1; ++q) {
    double v;
    if (q < 3 * nm) {
      // select mom[mom0 + q / 3][q % 3] without dynamic register indexing
      v = 0.0;
#pragma unroll
      for (int f = 0; f < 6; ++f)
#pragma unroll
        for (int r = 0; r < 3; ++r)
          if (f == mom0 + q / 3 && r == q % 3) v = mom[f][r];
    } else {
      v = mx;
    }
    red[threadIdx.x] = v;
    __syncthreads();
    for (int o = C::X_THREADS / 2; o > 0; o >>= 1) {
      if ((int)threadIdx.x < o) {
        const double a = red[threadIdx.x], b = red[threadIdx.x + o];
        red[threadIdx.x] = q < 3 * nm ? a + b : ((b > a || b != b) ? b : a);
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) out[q] = red[0];
    __syncthreads();
  }
}

// Final record of one slot (layout in include/psdns.h).
static __global__ void __launch_bounds__(256)
k_spectra_finalize(const double* __restrict__ shells, const double* __restrict__ mom1, const double* __restrict__ mom2,
                   int nbm, const SlotDev* __restrict__ slots, Geom g, int ns, int flags, double* __restrict__ out,
                   int rec) {
  const int slot = blockIdx.x;
  const SlotDev& sp = slots[slot];
  const int S = g.S, Q = shell_quantities(S);
  double* o = out + (long long)slot * rec;
  const double nan = __builtin_nan("");
  const double n3 = double(g.N) * g.N * g.N, n6 = n3 * n3;
  const int base = ns * (1 + S);
  const int pb = base + 8 + 4 * S;
  if (threadIdx.x == 0) {
    for (int i = 0; i < rec; ++i) o[i] = nan;
  }
  __syncthreads();
  if ((flags & 1) && threadIdx.x == 0) {
    const double* sh = shells + (long long)slot * ns * Q;
    double K = 0.0, diss = 0.0;
    for (int s = 0; s < ns; ++s) {
      o[s] = sh[s * Q + 0] / n6;
      K += sh[s * Q + 0];
      diss += sh[s * Q + 1];
    }
    K /= n6;
    const double eps = sp.nu * diss / n6;
    const double urms = sqrt(2.0 * K / 3.0);
    o[base + 0] = K;
    o[base + 1] = eps;
    o[base + 2] = urms;
    if (eps > 0.0) {
      const double lam = urms * sqrt(15.0 * sp.nu / eps);
      o[base + 3] = lam;
      o[base + 4] = lam * urms / sp.nu;
      o[base + 5] = pow(sp.nu * sp.nu * sp.nu / eps, 0.25);
      o[base + 6] = urms * urms * urms / eps;
      o[base + 7] = urms > 0.0 ? (urms * urms * urms / eps) / urms : nan;
    }
    for (int s = 0; s < S; ++s) {
      double var = 0.0, chi = 0.0, prod = 0.0;
      for (int h = 0; h < ns; ++h) {
        o[ns * (1 + s) + h] = sh[h * Q + 2 + 3 * s] / n6;
        var += sh[h * Q + 2 + 3 * s];
        chi += sh[h * Q + 3 + 3 * s];
        prod += sh[h * Q + 4 + 3 * s];
      }
      const double d = sp.diff[3 + s];
      o[base + 8 + 4 * s + 0] = 2.0 * var / n6;
      o[base + 8 + 4 * s + 1] = 2.0 * d * chi / n6;
      o[base + 8 + 4 * s + 2] = -2.0 * prod / n6;
      o[base + 8 + 4 * s + 3] = (-2.0 * prod / n6) / (2.0 * d * chi / n6);
    }
  }
  if ((flags & 2) && threadIdx.x == 0) {
    // first sweep: fields u1 u2 u3 | du1/dx1 du2/dx2 (moments of the last two) + max
    // second sweep: du3/dx3, dphi_s/dx2 (moments of all)
    double m1[2][3] = {{0, 0, 0}, {0, 0, 0}}, mx = 0.0;
    double m2[1 + kMaxScalars][3] = {};
    const int r1 = 3 * 2 + 1, r2 = 3 * (1 + S) + 1;
    for (int b = 0; b < nbm; ++b) {
      const double* p = mom1 + ((long long)slot * nbm + b) * (3 * 6 + 1);
      for (int f = 0; f < 2; ++f)
        for (int r = 0; r < 3; ++r) m1[f][r] += p[3 * f + r];
      const double v = p[r1 - 1];
      mx = (v > mx || v != v) ? v : mx;
      const double* q = mom2 + ((long long)slot * nbm + b) * (3 * 6 + 1);
      for (int f = 0; f < 1 + S; ++f)
        for (int r = 0; r < 3; ++r) m2[f][r] += q[3 * f + r];
      (void)r2;
    }
    const double* mm[3] = {m1[0], m1[1], m2[0]};
    for (int i = 0; i < 3; ++i) {
      const double a2 = mm[i][0] / n3, a3 = mm[i][1] / n3, a4 = mm[i][2] / n3;
      o[pb + i] = a2;
      o[pb + 3 + i] = a3;
      o[pb + 6 + i] = a4;
      o[pb + 9 + i] = a2 > 0 ? a3 / pow(a2, 1.5) : nan;
      o[pb + 12 + i] = a2 > 0 ? a4 / (a2 * a2) : nan;
    }
    o[pb + 15] = mx;
    for (int s = 0; s < S; ++s) {
      const double a2 = m2[1 + s][0] / n3, a3 = m2[1 + s][1] / n3, a4 = m2[1 + s][2] / n3;
      o[pb + 16 + 3 * s] = a2;
      o[pb + 17 + 3 * s] = a2 > 0 ? a3 / pow(a2, 1.5) : nan;
      o[pb + 18 + 3 * s] = a2 > 0 ? a4 / (a2 * a2) : nan;
    }
  }
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
struct TimedLaunch {
  Timer* t;
  int kid;
  hipStream_t s;
  TimedLaunch(Timer* t_, int k, hipStream_t s_) : t(t_), kid(k), s(s_) {
    if (t) t->begin(kid, s);
  }
  ~TimedLaunch() {
    if (t) t->end(kid, s);
  }
};

// The passes of one right-hand-side evaluation and stage update with schedule V.  Every
// schedule reads and writes the same buffers in the same layouts, so a stage may take
// each pass from a different schedule (Stage below).
template <int N, typename T, int V>
struct Step {
  using C = Cfg<N, T, V>;
  // x-pass blocks per slot, which is also the count of partial maxima k_step_dt reads
  static constexpr int kXBlocks = N * N / C::LX;
  static int ntile(const Geom& g) { return C::Col::grid_x((g.KX + C::W - 1) / C::W); }

  static void z_inverse(const Ctx& x, const cpx<T>* sin, hipStream_t s) {
    TimedLaunch tl(x.timer, KID_ZINV, s);
    k_z_inverse<N, T, V><<<dim3(ntile(x.g), x.g.M, x.g.batch), C::COL_THREADS, 0, s>>>(
        sin, static_cast<cpx<T>*>(x.abuf), static_cast<const cpx<T>*>(x.tw), x.slots, x.g);
  }
  static void y_inverse(const Ctx& x, hipStream_t s) {
    TimedLaunch tl(x.timer, KID_YINV, s);
    k_y_inverse<N, T, V><<<dim3(ntile(x.g), N, x.g.batch), C::COL_THREADS, 0, s>>>(
        static_cast<const cpx<T>*>(x.abuf), static_cast<cpx<T>*>(x.bbuf), static_cast<const cpx<T>*>(x.tw), x.slots,
        x.g);
  }
  // g carries nblk_x = kXBlocks
  static void x_pass(const Ctx& x, const Geom& g, int mode, hipStream_t s) {
    TimedLaunch tl(x.timer, KID_XPASS, s);
    k_x_pass<N, T, V><<<dim3(kXBlocks, g.batch), C::X_THREADS, 0, s>>>(
        static_cast<cpx<T>*>(x.bbuf), static_cast<const cpx<T>*>(x.tw), x.slots, x.dyn, g, mode);
  }
  static void y_forward(const Ctx& x, hipStream_t s) {
    TimedLaunch tl(x.timer, KID_YFWD, s);
    k_y_forward<N, T, V><<<dim3(ntile(x.g), N, x.g.batch), C::COL_THREADS, 0, s>>>(
        static_cast<const cpx<T>*>(x.bbuf), static_cast<cpx<T>*>(x.abuf), static_cast<const cpx<T>*>(x.tw), x.slots,
        x.g);
  }
  // fuse: every stage of a multi-step call, the stage fixed at compile time
  static void z_forward(const Ctx& x, const StageArgs<T>& sa, int stage, bool fuse, hipStream_t s) {
    const Geom& g = x.g;
    cpx<T>* A = static_cast<cpx<T>*>(x.abuf);
    const cpx<T>* tw = static_cast<const cpx<T>*>(x.tw);
    const dim3 grid_u(C::Fused::grid_x((g.KX + C::Fused::W - 1) / C::Fused::W), g.M, g.batch);
    constexpr int TU = C::Fused::THREADS;
    if (fuse) {
      TimedLaunch tl(x.timer, KID_ZFWDI, s);
      switch (stage) {
        case 0: k_z_forward_update<N, T, true, V, 0><<<grid_u, TU, 0, s>>>(A, sa, tw, x.slots, x.dyn, g); break;
        case 1: k_z_forward_update<N, T, true, V, 1><<<grid_u, TU, 0, s>>>(A, sa, tw, x.slots, x.dyn, g); break;
        case 2: k_z_forward_update<N, T, true, V, 2><<<grid_u, TU, 0, s>>>(A, sa, tw, x.slots, x.dyn, g); break;
        default: k_z_forward_update<N, T, true, V, 3><<<grid_u, TU, 0, s>>>(A, sa, tw, x.slots, x.dyn, g); break;
      }
    } else {
      TimedLaunch tl(x.timer, KID_ZFWD, s);
      k_z_forward_update<N, T, false, V, -2><<<grid_u, TU, 0, s>>>(A, sa, tw, x.slots, x.dyn, g);
    }
  }
};

// Calls fn(std::integral_constant<int, v>) for a schedule index v known only at run time.
template <int N, int I = 0, class Fn>
void with_sched(int v, Fn&& fn) {
  if constexpr (I < sched_count<N>()) {
    if (v == I)
      fn(std::integral_constant<int, I>{});
    else
      with_sched<N, I + 1>(v, fn);
  }
}

// One right-hand-side evaluation and stage update, each pass with the schedule that
// x.psched names for it.
// schedule of the x pass of the phase-shift stage: three waves per SIMD with the stage
// twiddles in LDS (its four half-spectrum entries per lane at N = 512 spill a little, and
// it still ran 5% faster than schedule 0's two waves)
#ifndef PSDNS_PHASE_X
#define PSDNS_PHASE_X 5
#endif
constexpr int kPhaseX = PSDNS_PHASE_X;

template <int N, typename T>
struct Stage {
  // flags: kStageZinv launches the standalone z inverse of stage_in first; kStageFuse makes
  // the last pass also produce the z-inverse of the next stage input.
  static void rhs_stage(const Ctx& x, void* state, const void* stage_in, int stage, void* rhs_out, int want_max,
                        double dt_arg, int flags, hipStream_t s) {
    // the x-pass block count (and so the partial-maximum count) follows its schedule
    Geom g = x.g;
    with_sched<N>(x.psched[kPassX], [&](auto v) { g.nblk_x = Step<N, T, decltype(v)::value>::kXBlocks; });
    const cpx<T>* sin = static_cast<const cpx<T>*>(stage_in);
    if (!(flags & kStagePrologue)) {
      TimedLaunch tl(x.timer, KID_FORCE, s);
      k_forcing_amplitude<T><<<g.batch, 256, 0, s>>>(sin, x.slots, x.dyn, g);
    }
    if (flags & kStageZinv)
      with_sched<N>(x.psched[kPassZInverse], [&](auto v) { Step<N, T, decltype(v)::value>::z_inverse(x, sin, s); });
    if (flags & kStagePrologue) return;
    with_sched<N>(x.psched[kPassYInverse], [&](auto v) { Step<N, T, decltype(v)::value>::y_inverse(x, s); });
    with_sched<N>(x.psched[kPassX],
                  [&](auto v) { Step<N, T, decltype(v)::value>::x_pass(x, g, want_max ? kXMax : 0, s); });
    if (stage == 0) {
      TimedLaunch tl(x.timer, KID_DT, s);
      k_step_dt<<<g.batch, 64, 0, s>>>(x.slots, x.dyn, g, dt_arg);
      // returns at once for slots without the stochastic forcing
      k_stochastic_update<T><<<g.batch, 256, 0, s>>>(static_cast<const cpx<T>*>(state), x.slots, x.dyn, x.fband, g);
    }
    with_sched<N>(x.psched[kPassYForward], [&](auto v) { Step<N, T, decltype(v)::value>::y_forward(x, s); });
    StageArgs<T> sa;
    sa.yn = static_cast<cpx<T>*>(state);
    sa.acc = static_cast<cpx<T>*>(x.acc);
    sa.ys = static_cast<cpx<T>*>(x.ystage);
    sa.sin = sin;
    sa.rhs = static_cast<cpx<T>*>(rhs_out);
    sa.fband = x.fband;
    sa.stage = stage;
    const bool fuse = (flags & kStageFuse) != 0;
    with_sched<N>(x.psched[kPassZForward],
                  [&](auto v) { Step<N, T, decltype(v)::value>::z_forward(x, sa, stage, fuse, s); });
  }

  // The paper's dealiasing (Sec. 2.3): the products are evaluated twice, on the grid
  // (y forward into akeep) and on the grid shifted by half a cell along each axis (into A),
  // and the z-forward pass takes their mean on the sphere 9|k|^2 < 2N^2 before projection,
  // forcing and the stage update.  The passes run with the sphere's bounding K, in
  // schedule 0 but for the x pass (kPhaseX) and the z forward (below); each stage runs its
  // own z inverses (no fusion), and the CFL maximum comes from the unshifted evaluation.
  static void rhs_phase(const Ctx& x, void* state, const void* stage_in, int stage, void* rhs_out, int want_max,
                        double dt_arg, int flags, hipStream_t s) {
    using C = Cfg<N, T, 0>;
    using St = Step<N, T, 0>;
    Geom g = x.g;
    g.nblk_x = Step<N, T, kPhaseX>::kXBlocks;
    const cpx<T>* sin = static_cast<const cpx<T>*>(stage_in);
    const cpx<T>* tw = static_cast<const cpx<T>*>(x.tw);
    cpx<T>* A = static_cast<cpx<T>*>(x.abuf);
    cpx<T>* B = static_cast<cpx<T>*>(x.bbuf);
    cpx<T>* keep = static_cast<cpx<T>*>(x.akeep);
    {
      TimedLaunch tl(x.timer, KID_FORCE, s);
      k_forcing_amplitude<T><<<g.batch, 256, 0, s>>>(sin, x.slots, x.dyn, g);
    }
    if (flags & kStagePrologue) return;
    const int nt = St::ntile(g);
    for (int p = 0; p < 2; ++p) {
      {
        TimedLaunch tl(x.timer, KID_ZINV, s);
        k_z_inverse<N, T, 0, 1><<<dim3(nt, g.M, g.batch), C::COL_THREADS, 0, s>>>(sin, A, tw, x.slots, g, p);
      }
      {
        TimedLaunch tl(x.timer, KID_YINV, s);
        k_y_inverse<N, T, 0, 1><<<dim3(nt, N, g.batch), C::COL_THREADS, 0, s>>>(A, B, tw, x.slots, g, p);
      }
      {
        TimedLaunch tl(x.timer, KID_XPASS, s);
        const int mode = (want_max && p == 0 ? kXMax : 0) | (p ? kXShift : 0);
        k_x_pass<N, T, kPhaseX, 1><<<dim3(Step<N, T, kPhaseX>::kXBlocks, g.batch), Cfg<N, T, kPhaseX>::X_THREADS, 0,
                                     s>>>(B, tw, x.slots, x.dyn, g, mode);
      }
      if (stage == 0 && p == 0) {
        TimedLaunch tl(x.timer, KID_DT, s);
        k_step_dt<<<g.batch, 64, 0, s>>>(x.slots, x.dyn, g, dt_arg);
        k_stochastic_update<T><<<g.batch, 256, 0, s>>>(static_cast<const cpx<T>*>(state), x.slots, x.dyn, x.fband, g);
      }
      {
        TimedLaunch tl(x.timer, KID_YFWD, s);
        k_y_forward<N, T, 0, 1><<<dim3(nt, N, g.batch), C::COL_THREADS, 0, s>>>(B, p ? A : keep, tw, x.slots, g, p,
                                                                                  p ? g.FA : g.F);
      }
    }
    StageArgs<T> sa;
    sa.yn = static_cast<cpx<T>*>(state);
    sa.acc = static_cast<cpx<T>*>(x.acc);
    sa.ys = static_cast<cpx<T>*>(x.ystage);
    sa.sin = sin;
    sa.rhs = static_cast<cpx<T>*>(rhs_out);
    sa.fband = x.fband;
    sa.stage = stage;
    // the sphere leaves more retained modes per thread than the 2/3 rule: the z-forward
    // pass takes the narrow tiles of schedule 3 (512-thread blocks, 256 registers)
    using CZ = typename Cfg<N, T, 3>::Fused;
    TimedLaunch tl(x.timer, KID_ZFWD, s);
    const dim3 grid_u(CZ::grid_x((g.KX + CZ::W - 1) / CZ::W), g.M, g.batch);
    k_z_forward_update<N, T, false, 3, -2, 1><<<grid_u, CZ::THREADS, 0, s>>>(A, sa, tw, x.slots, x.dyn, g, keep);
  }

  // the stage with every pass in schedule V
  template <int V>
  static void rhs_stage_of(const Ctx& x, void* state, const void* stage_in, int stage, void* rhs_out, int want_max,
                           double dt_arg, int flags, hipStream_t s) {
    Ctx y = x;
    for (int p = 0; p < kNumPasses; ++p) y.psched[p] = V;
    rhs_stage(y, state, stage_in, stage, rhs_out, want_max, dt_arg, flags, s);
  }
};

template <int N, typename T>
struct Engine {
  using C = Cfg<N, T>;

  static void init_field(const Ctx& x, void* state, int slot, uint64_t seed, double kp, int kind, double energy,
                         hipStream_t s) {
    const Geom& g = x.g;
    const long long nmodes = (long long)g.M * g.M * g.KX;
    const int nb = (int)((nmodes + 255) / 256);
    TimedLaunch tl(x.timer, KID_AUX, s);
    k_init_energy<<<nb, 256, 0, s>>>(g, seed, kp, kind, x.part);
    k_init_scale<<<1, 256, 0, s>>>(x.part, nb, energy, g.N, x.dyn + slot);
    k_init_write<T><<<nb, 256, 0, s>>>(static_cast<cpx<T>*>(state), g, slot, seed, kp, kind, x.dyn + slot);
  }

  static void get_state(const Ctx& x, const void* state, int slot, void* canon, hipStream_t s) {
    const Geom& g = x.g;
    const long long ncan = (long long)g.F * N * N * (N / 2 + 1);
    TimedLaunch tl(x.timer, KID_AUX, s);
    k_fill_zero<T><<<(unsigned)((ncan + 255) / 256), 256, 0, s>>>(static_cast<cpx<T>*>(canon), ncan);
    const long long n = (long long)g.F * g.M * g.M * g.KX;
    k_convert<T, true><<<(unsigned)((n + 255) / 256), 256, 0, s>>>(
        const_cast<cpx<T>*>(static_cast<const cpx<T>*>(state)), static_cast<cpx<T>*>(canon), g, slot);
  }

  static void set_state(const Ctx& x, void* state, int slot, const void* canon, hipStream_t s) {
    const Geom& g = x.g;
    const long long n = (long long)g.F * g.M * g.M * g.KX;
    TimedLaunch tl(x.timer, KID_AUX, s);
    k_convert<T, false><<<(unsigned)((n + 255) / 256), 256, 0, s>>>(
        static_cast<cpx<T>*>(state), const_cast<cpx<T>*>(static_cast<const cpx<T>*>(canon)), g, slot);
  }

  static void zero_scalars(const Ctx& x, void* state, int slot, hipStream_t s) {
    const Geom& g = x.g;
    const long long n = (long long)g.S * g.st_field;
    if (n == 0) return;
    cpx<T>* p = static_cast<cpx<T>*>(state) + (long long)slot * g.F * g.st_field + 3 * g.st_field;
    TimedLaunch tl(x.timer, KID_AUX, s);
    k_fill_zero<T><<<(unsigned)((n + 255) / 256), 256, 0, s>>>(p, n);
  }

  static void band_hold(const Ctx& x, void* state, hipStream_t s) {
    TimedLaunch tl(x.timer, KID_FORCE, s);
    k_band_hold<T><<<x.g.batch, 256, 0, s>>>(static_cast<cpx<T>*>(state), x.slots, x.g);
  }

  // pressure of every active slot into the canonical layout (one field per slot)
  static void pressure(const Ctx& x, const void* state, void* canon, const int* active, hipStream_t s) {
    using C0 = Cfg<N, T, 0>;
    const cpx<T>* st = static_cast<const cpx<T>*>(state);
    const cpx<T>* tw = static_cast<const cpx<T>*>(x.tw);
    cpx<T>* A = static_cast<cpx<T>*>(x.abuf);
    cpx<T>* B = static_cast<cpx<T>*>(x.bbuf);
    cpx<T>* P = static_cast<cpx<T>*>(x.acc);  // compact pressure, one field per slot
    // velocity only: the scalar fields are skipped (slot strides keep the real counts)
    Geom gp = x.g;
    gp.S = 0;
    gp.nblk_x = N * N / C0::LX;
    const int ntile = (gp.KX + C0::W - 1) / C0::W;
    const int gx = C0::Col::grid_x(ntile);  // the passes shared with the step place blocks by col_block
    TimedLaunch tl(x.timer, KID_AUX, s);
    k_z_inverse<N, T, 0><<<dim3(gx, gp.M, gp.batch), C0::COL_THREADS, 0, s>>>(st, A, tw, x.slots, gp);
    k_y_inverse<N, T, 0><<<dim3(gx, N, gp.batch), C0::COL_THREADS, 0, s>>>(A, B, tw, x.slots, gp);
    k_x_pass<N, T, 0><<<dim3(gp.nblk_x, gp.batch), C0::X_THREADS, 0, s>>>(B, tw, x.slots, x.dyn, gp, kXPressure);
    Geom gy = gp;
    gy.F = 4;  // c1, c2, c3, |u|^2/2
    k_y_forward<N, T, 0><<<dim3(gx, N, gp.batch), C0::COL_THREADS, 0, s>>>(B, A, tw, x.slots, gy);
    k_z_forward_pressure<N, T><<<dim3(ntile, gp.M, gp.batch), C0::COL_THREADS, 0, s>>>(A, P, tw, x.slots, gp);
    const long long per = (long long)N * N * (N / 2 + 1);
    k_fill_zero<T><<<(unsigned)((per * gp.batch + 255) / 256), 256, 0, s>>>(static_cast<cpx<T>*>(canon),
                                                                             per * gp.batch);
    Geom g1 = gp;
    g1.F = 1;
    const long long n = (long long)g1.M * g1.M * g1.KX;
    for (int slot = 0; slot < gp.batch; ++slot) {
      if (!active[slot]) continue;
      k_convert<T, true><<<(unsigned)((n + 255) / 256), 256, 0, s>>>(P, static_cast<cpx<T>*>(canon) + slot * per, g1,
                                                                     slot);
    }
  }

  static void spectra(const Ctx& x, const void* state, double* out, int flags, hipStream_t s) {
    const Geom& g = x.g;
    const cpx<T>* st = static_cast<const cpx<T>*>(state);
    const cpx<T>* tw = static_cast<const cpx<T>*>(x.tw);
    cpx<T>* A = static_cast<cpx<T>*>(x.abuf);
    cpx<T>* B = static_cast<cpx<T>*>(x.bbuf);
    const int ns = g.ns, Q = shell_quantities(g.S);
    double* shells = x.stat;
    double* mom1 = shells + (long long)g.batch * ns * Q;
    double* mom2 = mom1 + (long long)g.batch * x.nbm * (3 * 6 + 1);
    const int ntile = (g.KX + C::W - 1) / C::W;
    TimedLaunch tl(x.timer, KID_AUX, s);
    if (flags & 1) k_shell_sums<T><<<dim3(ns, g.batch), 256, 0, s>>>(st, x.slots, g, shells, ns);
    if (flags & 2) {
      DerivSpec d1{};
      d1.nf = 5;
      const int f1[5] = {0, 1, 2, 0, 1}, a1[5] = {0, 0, 0, 1, 2};
      for (int i = 0; i < 5; ++i) {
        d1.field[i] = f1[i];
        d1.axis[i] = a1[i];
      }
      k_stats_z<N, T><<<dim3(ntile, g.M, g.batch), C::COL_THREADS, 0, s>>>(st, A, tw, g, d1);
      k_stats_y<N, T><<<dim3(ntile, N, g.batch), C::COL_THREADS, 0, s>>>(A, B, tw, g, 5);
      k_x_moments<N, T><<<dim3(x.nbm, g.batch), C::X_THREADS, 0, s>>>(B, tw, g, 5, 3, 1, mom1);
      DerivSpec d2{};
      d2.nf = 1 + g.S;
      d2.field[0] = 2;
      d2.axis[0] = 3;
      for (int i = 0; i < g.S; ++i) {
        d2.field[1 + i] = 3 + i;
        d2.axis[1 + i] = 2;
      }
      k_stats_z<N, T><<<dim3(ntile, g.M, g.batch), C::COL_THREADS, 0, s>>>(st, A, tw, g, d2);
      k_stats_y<N, T><<<dim3(ntile, N, g.batch), C::COL_THREADS, 0, s>>>(A, B, tw, g, 1 + g.S);
      k_x_moments<N, T><<<dim3(x.nbm, g.batch), C::X_THREADS, 0, s>>>(B, tw, g, 1 + g.S, 0, 0, mom2);
    }
    k_spectra_finalize<<<g.batch, 256, 0, s>>>(shells, mom1, mom2, x.nbm, x.slots, g, ns, flags, out,
                                               x.spectra_rec);
  }

  template <int V>
  static void add_sched(Ops& o) {
    using CV = Cfg<N, T, V>;
    StepSched& d = o.sched[V];
    d.ec = CV::EC;
    d.ex = CV::EX;
    d.col_w = CV::W;
    d.fused_ec = CV::Fused::EC;
    d.fused_w = CV::Fused::W;
    d.x_lines = CV::LX;
    d.rhs_stage = &Stage<N, T>::template rhs_stage_of<V>;
  }

  template <int V, int NV>
  static void add_scheds(Ops& o) {
    if constexpr (V < NV) {
      add_sched<V>(o);
      add_scheds<V + 1, NV>(o);
    }
  }

  static Ops ops() {
    Ops o{};
    o.nsched = sched_count<N>();
    add_scheds<0, sched_count<N>()>(o);
    o.rhs_mixed = &Stage<N, T>::rhs_stage;
    o.rhs_phase = &Stage<N, T>::rhs_phase;
    o.init_field = &init_field;
    o.get_state = &get_state;
    o.set_state = &set_state;
    o.spectra = &spectra;
    o.pressure = &pressure;
    o.band_hold = &band_hold;
    o.zero_scalars = &zero_scalars;
    return o;
  }
};

}  // namespace psdns
