// General kernels of the right-hand side and its stage update for any even N whose prime
// factors are 2, 3, 5, 7, 11 and 13 (the paper's N = 520 = 2^3 5 13, Sec. 3.1), and for the
// paper's dealiasing: the mean of the products on the grid and on the grid shifted by half a
// cell, truncated to the sphere |k| < sqrt(2) N / 3 (Sec. 2.3).
//
// The passes and the layouts are those of the tuned power-of-two kernels (z inverse,
// y inverse, x pass with the products, y forward, z forward with projection, forcing and the
// integrating-factor RK4 update), with N, K and the retained set known only at run time.
// Transforms are Stockham stages of mixed radix that keep whole lines in LDS: W columns per
// block (one row segment of the kx tile), TT threads per column, each stage a loop over the
// N/R butterflies of radix R with a block barrier between stages.  These kernels favour
// generality over speed: the tuned kernels stay the path for power-of-two grids.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "common.hpp"
#include "fft.hpp"

namespace psdns {
namespace gen {

constexpr int kMaxStages = 16;
constexpr int kMaxOut = 3 * (6 + 3 * kMaxScalars);

// Radices of the transform stages of an N-point line: eights, then one four or two for
// the rest of the power of two, then the odd primes.
struct Factors {
  int n, nst;
  int r[kMaxStages];
};

inline Factors factor(int N) {
  Factors f{};
  f.n = N;
  int m = N;
  while (m % 8 == 0) {
    f.r[f.nst++] = 8;
    m /= 8;
  }
  if (m % 4 == 0) {
    f.r[f.nst++] = 4;
    m /= 4;
  }
  if (m % 2 == 0) {
    f.r[f.nst++] = 2;
    m /= 2;
  }
  for (int p : kOddRadices)
    while (m % p == 0) {
      f.r[f.nst++] = p;
      m /= p;
    }
  return f;
}

// In-register DFT of odd prime length R from the roots exp(-2 pi i m / R) (conjugated for
// the inverse): y_k = sum_n a_n w^(k n), paired as a_n + a_{R-n} and a_n - a_{R-n}.
template <int R, bool INV, typename T>
__device__ __forceinline__ void dft_odd(cpx<T> (&a)[R], const cpx<T> (&w)[R]) {
  cpx<T> s[R / 2 + 1], d[R / 2 + 1];
#pragma unroll
  for (int n = 1; n <= R / 2; ++n) {
    s[n] = a[n] + a[R - n];
    d[n] = a[n] - a[R - n];
  }
  cpx<T> y[R];
  cpx<T> y0 = a[0];
#pragma unroll
  for (int n = 1; n <= R / 2; ++n) y0 = y0 + s[n];
  y[0] = y0;
#pragma unroll
  for (int k = 1; k <= R / 2; ++k) {
    // w^(k n) = c + i s with c = Re w_{kn}, s = Im w_{kn}; the pair (n, R - n) contributes
    // c (a_n + a_{R-n}) + i s (a_n - a_{R-n}) to y_k and c (...) - i s (...) to y_{R-k}
    cpx<T> cr = a[0], ci = {T(0), T(0)};
#pragma unroll
    for (int n = 1; n <= R / 2; ++n) {
      const cpx<T> wk = w[(k * n) % R];
      const T c = wk.x, sn = INV ? -wk.y : wk.y;
      cr = cr + c * s[n];
      ci = ci + sn * d[n];
    }
    y[k] = cr + mul_i(ci);
    y[R - k] = cr - mul_i(ci);
  }
#pragma unroll
  for (int k = 0; k < R; ++k) a[k] = y[k];
}

// One Stockham stage of radix R from src to dst (LDS; element p of column c at p W + c):
// butterfly b < N/R takes positions b + r N/R, applies the twiddles w_N^(r kv N/(NS R)),
// kv = b mod NS, and writes positions (b / NS) NS R + kv + r NS.
template <int R, bool INV, typename T>
__device__ __forceinline__ void stage(const cpx<T>* src, cpx<T>* dst, int W, int c, int j, int TT, int N, int NS,
                                      const cpx<T>* __restrict__ tw) {
  const int nb = N / R;
  cpx<T> root[R];
  if constexpr (R % 2 == 1) {
#pragma unroll
    for (int m = 0; m < R; ++m) root[m] = tw[N + kRootOff(R) + m];
  }
  // b / NS from a float reciprocal: for b, NS <= 1024 the rounding error of (b + 1/2) / NS
  // stays far below its distance 1 / (2 NS) from the nearest integer, so the quotient is exact
  const float rns = 1.0f / float(NS);
  for (int b = j; b < nb; b += TT) {
    const int bq = int((float(b) + 0.5f) * rns);
    const int kv = b - bq * NS;
    cpx<T> a[R];
#pragma unroll
    for (int r = 0; r < R; ++r) a[r] = src[(b + r * nb) * W + c];
    if (NS > 1) {
      const int step = N / (NS * R);
#pragma unroll
      for (int r = 1; r < R; ++r) {
        cpx<T> w = tw[r * kv * step];
        if (INV) w.y = -w.y;
        a[r] = cmul(a[r], w);
      }
    }
    if constexpr (R % 2 == 1)
      dft_odd<R, INV>(a, root);
    else
      dft<R, INV>(a);
    const int base = bq * NS * R + kv;
#pragma unroll
    for (int r = 0; r < R; ++r) dst[(base + r * NS) * W + c] = a[r];
  }
}

// Full N-point transform of the W columns held in b0 (all threads of the block call it, or
// all lanes of one wavefront with Sync = WaveSync when the wave owns its lines alone).
// Returns the buffer (b0 or b1) that holds the result in natural order.
template <bool INV, typename Sync = BlockSync, typename T>
__device__ __forceinline__ cpx<T>* fft(cpx<T>* b0, cpx<T>* b1, const Factors& f, int W, int c, int j, int TT,
                       const cpx<T>* __restrict__ tw) {
  cpx<T>* src = b0;
  cpx<T>* dst = b1;
  int NS = 1;
  for (int st = 0; st < f.nst; ++st) {
    const int R = f.r[st];
    switch (R) {
      case 2: stage<2, INV>(src, dst, W, c, j, TT, f.n, NS, tw); break;
      case 3: stage<3, INV>(src, dst, W, c, j, TT, f.n, NS, tw); break;
      case 4: stage<4, INV>(src, dst, W, c, j, TT, f.n, NS, tw); break;
      case 5: stage<5, INV>(src, dst, W, c, j, TT, f.n, NS, tw); break;
      case 7: stage<7, INV>(src, dst, W, c, j, TT, f.n, NS, tw); break;
      case 8: stage<8, INV>(src, dst, W, c, j, TT, f.n, NS, tw); break;
      case 11: stage<11, INV>(src, dst, W, c, j, TT, f.n, NS, tw); break;
      default: stage<13, INV>(src, dst, W, c, j, TT, f.n, NS, tw); break;
    }
    Sync::sync();
    NS *= R;
    cpx<T>* t = src;
    src = dst;
    dst = t;
  }
  return src;
}

// exp(i pi k / N) for |k| <= N/2 (the half-cell shift along one axis), from the table
template <typename T>
__device__ __forceinline__ cpx<T> shift_of(const cpx<T>* __restrict__ tw, int N, int k) {
  const cpx<T> v = tw[N + kShiftOff + (k < 0 ? -k : k)];
  return k < 0 ? conj(v) : v;
}

// position n of a line -> signed wavenumber; compact index along ky/kz (-1 if |k| > K)
__device__ __forceinline__ int wave(int n, int N) { return n <= N / 2 ? n : n - N; }
__device__ __forceinline__ int compact(int k, int K, int M) { return k > K || k < -K ? -1 : (k >= 0 ? k : k + M); }

// Output fields of a column pass: out_o = sum over its terms of sgn (i k_axis)^[axis > 0]
// in_f, axis 0 none, 1 x, 2 y, 3 z (k of the column or of the line).
struct Spec {
  int nout;
  int nterm[kMaxOut];
  int f[kMaxOut][2];
  int axis[kMaxOut][2];
  float sgn[kMaxOut][2];
};

// Launch shape of the column passes: W columns (a row segment of the kx tile) and TT
// threads per column, with two line buffers per column in dynamic LDS.
struct Shape {
  int W, TT;
  size_t lds;
};
constexpr int kMaxPerThread = 16;  // positions n = j + TT m of a column held by one thread

inline Shape col_shape(int N, int csize) {
  Shape s{};
  s.W = csize == 8 ? 16 : 8;
  while (s.W > 1 && 2 * (size_t)s.W * N * csize > 150 * 1024) s.W /= 2;
  // threads per column: up to 128 (and 1024 per block), at least N / kMaxPerThread
  s.TT = 1024 / s.W < 128 ? 1024 / s.W : 128;
  if (s.TT > N / 2) s.TT = N / 2;
  s.lds = 2 * (size_t)s.W * N * csize;
  return s;
}

// ---------------------------------------------------------------------------
// z inverse: state columns along kz (compact rows) -> A fields, all N positions of z.
// shift: inputs carry exp(i pi kz / N) (the kx and ky parts are applied by the later passes).
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(1024)
k_z_inverse(const cpx<T>* __restrict__ st, cpx<T>* __restrict__ abuf, const cpx<T>* __restrict__ tw,
            const SlotDev* __restrict__ slots, Geom g, Factors fz, Spec sp, int W, int TT, int shift, T scale) {
  extern __shared__ char lds_raw[];
  cpx<T>* b0 = reinterpret_cast<cpx<T>*>(lds_raw);
  cpx<T>* b1 = b0 + (size_t)W * g.N;
  const int slot = blockIdx.z;
  if (!slots[slot].active) return;
  const int c = threadIdx.x % W, j = threadIdx.x / W;
  const int kx = blockIdx.x * W + c, kyc = blockIdx.y;
  const bool valid = kx < g.KX;
  const int N = g.N, M = g.M;
  const int ky = kyc <= g.K ? kyc : kyc - M;
  const cpx<T>* sbase = st + (long long)slot * g.F * g.st_field;
  cpx<T>* abase = abuf + (long long)slot * g.FA * g.a_field;
  for (int o = 0; o < sp.nout; ++o) {
    for (int n = j; n < N; n += TT) {
      const int kz = wave(n, N), kc = compact(kz, g.K, M);
      cpx<T> v = {T(0), T(0)};
      // only retained modes are read: the stage inputs hold nothing defined outside a sphere
      if (valid && kc >= 0 && retained(g, kx, ky, kz)) {
        for (int t = 0; t < sp.nterm[o]; ++t) {
          cpx<T> x = sbase[(long long)sp.f[o][t] * g.st_field + st_row(kc, kyc, M, g.PX) + kx];
          const int ax = sp.axis[o][t];
          if (ax) x = mul_is(x, T(ax == 1 ? kx : ax == 2 ? ky : kz));
          v = v + T(sp.sgn[o][t]) * x;
        }
        v = scale * v;
        if (shift) v = cmul(v, shift_of(tw, N, kz));
      }
      b0[n * W + c] = v;
    }
    __syncthreads();
    const cpx<T>* res = fft<true>(b0, b1, fz, W, c, j, TT, tw);
    if (valid)
      for (int n = j; n < N; n += TT) abase[(long long)o * g.a_field + a_row(n, kyc, M, g.PX) + kx] = res[n * W + c];
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// y inverse: A columns along ky (compact rows) at fixed z -> B fields, all N positions of y.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(1024)
k_y_inverse(const cpx<T>* __restrict__ abuf, cpx<T>* __restrict__ bbuf, const cpx<T>* __restrict__ tw,
            const SlotDev* __restrict__ slots, Geom g, Factors fy, Spec sp, int W, int TT, int shift) {
  extern __shared__ char lds_raw[];
  cpx<T>* b0 = reinterpret_cast<cpx<T>*>(lds_raw);
  cpx<T>* b1 = b0 + (size_t)W * g.N;
  const int slot = blockIdx.z;
  if (!slots[slot].active) return;
  const int c = threadIdx.x % W, j = threadIdx.x / W;
  const int kx = blockIdx.x * W + c, z = blockIdx.y;
  const bool valid = kx < g.KX;
  const int N = g.N, M = g.M;
  const cpx<T>* abase = abuf + (long long)slot * g.FA * g.a_field;
  cpx<T>* bbase = bbuf + (long long)slot * g.FB * g.b_field + (long long)z * N * g.PX;
  for (int o = 0; o < sp.nout; ++o) {
    for (int n = j; n < N; n += TT) {
      const int ky = wave(n, N), kc = compact(ky, g.K, M);
      cpx<T> v = {T(0), T(0)};
      if (valid && kc >= 0) {
        for (int t = 0; t < sp.nterm[o]; ++t) {
          cpx<T> x = abase[(long long)sp.f[o][t] * g.a_field + a_row(z, kc, M, g.PX) + kx];
          const int ax = sp.axis[o][t];
          if (ax) x = mul_is(x, T(ax == 1 ? kx : ky));
          v = v + T(sp.sgn[o][t]) * x;
        }
        if (shift) v = cmul(v, shift_of(tw, N, ky));
      }
      b0[n * W + c] = v;
    }
    __syncthreads();
    const cpx<T>* res = fft<true>(b0, b1, fy, W, c, j, TT, tw);
    if (valid)
      for (int n = j; n < N; n += TT) bbase[(long long)o * g.b_field + (long long)n * g.PX + kx] = res[n * W + c];
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// y forward: the first nf B fields along y (all N positions) at fixed z -> A (or the kept
// unshifted product), rows |ky| <= K; shift multiplies by exp(-i pi ky / N).
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(1024)
k_y_forward(const cpx<T>* __restrict__ bbuf, cpx<T>* __restrict__ aout, int a_fields, const cpx<T>* __restrict__ tw,
            const SlotDev* __restrict__ slots, Geom g, Factors fy, int nf, int W, int TT, int shift) {
  extern __shared__ char lds_raw[];
  cpx<T>* b0 = reinterpret_cast<cpx<T>*>(lds_raw);
  cpx<T>* b1 = b0 + (size_t)W * g.N;
  const int slot = blockIdx.z;
  if (!slots[slot].active) return;
  const int c = threadIdx.x % W, j = threadIdx.x / W;
  const int kx = blockIdx.x * W + c, z = blockIdx.y;
  const bool valid = kx < g.KX;
  const int N = g.N, M = g.M;
  const cpx<T>* bbase = bbuf + (long long)slot * g.FB * g.b_field + (long long)z * N * g.PX;
  cpx<T>* obase = aout + (long long)slot * a_fields * g.a_field;
  for (int f = 0; f < nf; ++f) {
    for (int n = j; n < N; n += TT)
      b0[n * W + c] = valid ? bbase[(long long)f * g.b_field + (long long)n * g.PX + kx] : cpx<T>{T(0), T(0)};
    __syncthreads();
    const cpx<T>* res = fft<false>(b0, b1, fy, W, c, j, TT, tw);
    if (valid)
      for (int n = j; n < N; n += TT) {
        const int ky = wave(n, N), kc = compact(ky, g.K, M);
        if (kc < 0) continue;
        cpx<T> v = res[n * W + c];
        if (shift) v = cmul(v, conj(shift_of(tw, N, ky)));
        obase[(long long)f * g.a_field + a_row(z, kc, M, g.PX) + kx] = v;
      }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// x pass: one wavefront per (z, y) line, lw lines per block.  Pairs of real fields travel as
// one complex line h = f + i g (half-spectrum entries kx <= K, their conjugates at N - kx);
// the products u x omega and u.grad phi_s + g_s.u are formed pointwise and transformed back,
// kx <= K written in place into the first F fields of B.  shift multiplies the inputs by
// exp(i pi kx / N) and the outputs by its conjugate; with umax the line's
// max |u1|+|u2|+|u3| joins the slot's maximum (Eq. (10)).
//
// The block copies the root table (stage twiddles, odd-radix roots, half-cell shifts) to
// LDS once for its lines; each wave then owns two line buffers and synchronises its
// transform stages alone.  Lane j keeps positions n = j + 64 q (q < P) of the physical
// fields in registers: u1 u2 u3, and c1 c2 c3 while they are formed; c1 and c2 are
// transformed as soon as they exist, and each scalar product then pairs with the field
// before it, so that at most six fields are live.
// ---------------------------------------------------------------------------
constexpr int kXMaxLines = 4;     // lines (wavefronts) per block

// positions per lane of the physical fields of an N-point line; the half spectrum
// kx <= K <= N/2 then needs at most P/2 + 1 entries per lane
inline int x_positions(int N) { return (N + 63) / 64; }
constexpr int kMaxPositions = 16;  // N <= 1024: 64 lanes per x line, 64 or more threads per z column
// lines per block: as many as fit two blocks in the 160 KB of a CU
inline int x_lines(int N, int csize) {
  int lw = kXMaxLines;
  while (lw > 1 && ((size_t)root_table_entries(N) + (size_t)lw * 2 * N) * csize > 80 * 1024) lw /= 2;
  return lw;
}
inline size_t x_lds_bytes(int N, int csize, int lw) {
  return ((size_t)root_table_entries(N) + (size_t)lw * 2 * N) * csize;
}

// waves per SIMD the register allocation of the x pass aims at (six fields of P positions
// per lane next to the transform stages)
template <typename T, int P>
constexpr int x_waves() {
  return sizeof(T) == 4 ? (P <= 4 ? 4 : P <= 12 ? 3 : 2) : (P <= 10 ? 2 : 1);
}

template <typename T, int P>
__global__ void __launch_bounds__(64 * kXMaxLines, (x_waves<T, P>()))
k_x_pass(cpx<T>* __restrict__ bbuf, const cpx<T>* __restrict__ tw_g, const SlotDev* __restrict__ slots,
         DynDev* __restrict__ dyn, Geom g, Factors fx, int shift, int umax) {
  extern __shared__ char lds_raw[];
  const int N = g.N, S = g.S, K = g.K;
  const int nt = (int)root_table_entries(N);
  cpx<T>* tw = reinterpret_cast<cpx<T>*>(lds_raw);
  const int slot = blockIdx.y;
  const SlotDev& sp = slots[slot];
  if (!sp.active) return;
  for (int i = threadIdx.x; i < nt; i += blockDim.x) tw[i] = tw_g[i];
  __syncthreads();
  const int lw = blockDim.x / 64, wv = threadIdx.x / 64, j = threadIdx.x % 64;
  const long long line = (long long)blockIdx.x * lw + wv;  // z * N + y
  if (line >= (long long)N * N) return;
  cpx<T>* b0 = tw + nt + (size_t)wv * 2 * N;
  cpx<T>* b1 = b0 + N;
  cpx<T>* lbase = bbuf + (long long)slot * g.FB * g.b_field + line * g.PX;
  // entry kx of the combination (field f, optional i kx factor, sign)
  auto entry = [&](int f, bool dx, T sg, int kx) {
    cpx<T> v = lbase[(long long)f * g.b_field + kx];
    if (dx) v = mul_is(v, T(kx));
    v = sg * v;
    if (shift) v = cmul(v, shift_of(tw, N, kx));
    return v;
  };
  // value of a real field at kx as a combination of up to two B fields: first (f1, dx1, s1),
  // second (f2, dx2, s2) with f2 < 0 for none
  struct Comb {
    int f1;
    bool dx1;
    T s1;
    int f2;
    bool dx2;
    T s2;
  };
  auto coeff = [&](const Comb& q, int kx) {
    if (q.f1 < 0) return cpx<T>{T(0), T(0)};
    cpx<T> v = entry(q.f1, q.dx1, q.s1, kx);
    if (q.f2 >= 0) v = v + entry(q.f2, q.dx2, q.s2, kx);
    if (kx == 0) v.y = T(0);
    return v;
  };
  // The transforms of a line run as one sequence of jobs through a single forward transform
  // (an inverse transform is the conjugate of the forward transform of the conjugate):
  //   0  inverse (u1, u2)
  //   1  inverse (u3, omega1), omega1 into C
  //   2  inverse (omega2, omega3), then c = u x omega into A, B, C
  //   3  forward of the pair (A, B) into output fields (fa, fb), fb < 0 for A alone
  //   4  inverse (dx phi_s, dy phi_s), then a_s = u1 dx phi_s + u2 dy phi_s + g_s.u into B
  //   5  inverse dz phi_s, then a_s += u3 dz phi_s
  // c1 and c2 are transformed first; c3 then waits in A for a_0, and every second scalar
  // product waits in A for the next.  For an inverse job a lane reads its half-spectrum entries
  // k = j + 64 q once, all of them before any is used, and writes position k and its conjugate
  // mirror N - k of the line.
  constexpr int Q = P / 2 + 1;
  T u1[P], u2[P], u3[P], A[P], B[P], C[P];
  double mx = 0.0;
  int job = 0, s = 0, fa = 0, fb = 1, pend = -1;
  while (job >= 0) {
    if (job == 3) {
#pragma unroll
      for (int i = 0; i < P; ++i) {
        const int n = j + 64 * i;
        if (n < N) b0[n] = {A[i], fb >= 0 ? B[i] : T(0)};
      }
    } else {
      Comb qa = {-1, false, T(0), -1, false, T(0)}, qb = qa;
      // B fields: 0 u1, 1 u2, 2 u3, 3 omega1, 4 dz u1, 5 dy u1, 6+3s phi_s, 7+3s dy phi_s, 8+3s dz phi_s
      switch (job) {
        case 0: qa = {0, false, T(1), -1, false, T(0)}; qb = {1, false, T(1), -1, false, T(0)}; break;
        case 1: qa = {2, false, T(1), -1, false, T(0)}; qb = {3, false, T(1), -1, false, T(0)}; break;
        // omega2 = dz u1 - dx u3, omega3 = dx u2 - dy u1
        case 2: qa = {4, false, T(1), 2, true, T(-1)}; qb = {1, true, T(1), 5, false, T(-1)}; break;
        case 4: qa = {6 + 3 * s, true, T(1), -1, false, T(0)}; qb = {7 + 3 * s, false, T(1), -1, false, T(0)}; break;
        default: qa = {8 + 3 * s, false, T(1), -1, false, T(0)}; break;
      }
      cpx<T> va[Q], vb[Q];
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const int k = j + 64 * q;
        va[q] = k <= K ? coeff(qa, k) : cpx<T>{T(0), T(0)};
        vb[q] = k <= K ? coeff(qb, k) : cpx<T>{T(0), T(0)};
      }
      for (int n = K + 1 + j; n < N - K; n += 64) b0[n] = {T(0), T(0)};
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const int k = j + 64 * q;
        if (k <= K) {
          b0[k] = conj(va[q] + mul_i(vb[q]));
          if (k > 0) b0[N - k] = conj(conj(va[q]) + mul_i(conj(vb[q])));
        }
      }
    }
    WaveSync::sync();
    const cpx<T>* r = fft<false, WaveSync>(b0, b1, fx, 1, 0, j, 64, tw);
    if (job == 3) {
      for (int k = j; k <= K; k += 64) {
        const cpx<T> zk = r[k], zc = conj(r[(N - k) % N]);
        cpx<T> Pv = T(0.5) * (zk + zc);
        cpx<T> Qv = mul_mi(T(0.5) * (zk - zc));
        if (shift) {
          const cpx<T> e = conj(shift_of(tw, N, k));
          Pv = cmul(Pv, e);
          Qv = cmul(Qv, e);
        }
        lbase[(long long)fa * g.b_field + k] = Pv;
        if (fb >= 0) lbase[(long long)fb * g.b_field + k] = Qv;
      }
    } else {
      // physical values of the pair: Re and Im of the inverse, the conjugate of r
      T rx[P], ry[P];
#pragma unroll
      for (int i = 0; i < P; ++i) {
        const int n = j + 64 * i;
        rx[i] = n < N ? r[n].x : T(0);
        ry[i] = n < N ? -r[n].y : T(0);
      }
      switch (job) {
        case 0:
#pragma unroll
          for (int i = 0; i < P; ++i) {
            u1[i] = rx[i];
            u2[i] = ry[i];
          }
          break;
        case 1:
#pragma unroll
          for (int i = 0; i < P; ++i) {
            u3[i] = rx[i];
            C[i] = ry[i];
          }
          break;
        case 2:
#pragma unroll
          for (int i = 0; i < P; ++i) {
            const T w1 = C[i], w2 = rx[i], w3 = ry[i];
            const T a = u1[i], b = u2[i], c = u3[i];
            A[i] = b * w3 - c * w2;
            B[i] = c * w1 - a * w3;
            C[i] = a * w2 - b * w1;
            const double sm = fabs((double)a) + fabs((double)b) + fabs((double)c);
            mx = (sm > mx || sm != sm) ? sm : mx;
          }
          break;
        case 4: {
          const T g0 = T(sp.g[s][0]), g1 = T(sp.g[s][1]), g2 = T(sp.g[s][2]);
#pragma unroll
          for (int i = 0; i < P; ++i)
            B[i] = u1[i] * rx[i] + u2[i] * ry[i] + (g0 * u1[i] + g1 * u2[i] + g2 * u3[i]);
          break;
        }
        default:
#pragma unroll
          for (int i = 0; i < P; ++i) B[i] += u3[i] * rx[i];
          break;
      }
    }
    WaveSync::sync();
    // the next job
    switch (job) {
      case 0: job = 1; break;
      case 1: job = 2; break;
      case 2: job = 3; fa = 0; fb = 1; break;
      case 3:
        if (fa == 0) {  // c1, c2 done: c3 (field 2) waits for a_0
#pragma unroll
          for (int i = 0; i < P; ++i) A[i] = C[i];
          pend = 2;
        } else {
          pend = -1;
        }
        if (s < S) {
          job = 4;
        } else if (pend >= 0) {
          fa = pend;
          fb = -1;
          pend = -1;
        } else {
          job = -1;
        }
        break;
      case 4: job = 5; break;
      default:
        if (pend >= 0) {  // the pending field and a_s
          fa = pend;
          fb = 3 + s;
          job = 3;
        } else {  // a_s waits for a_{s+1}, or goes alone after the last scalar
#pragma unroll
          for (int i = 0; i < P; ++i) A[i] = B[i];
          pend = 3 + s;
          if (s + 1 < S) {
            job = 4;
          } else {
            fa = pend;
            fb = -1;
            job = 3;
          }
        }
        ++s;
        break;
    }
  }
  if (umax) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const double b = __shfl_xor(mx, o);
      mx = (b > mx || b != b) ? b : mx;
    }
    if (j == 0) atomicMax(&dyn[slot].umax, (unsigned long long)__double_as_longlong(mx));
  }
}

// LDS of the line-moment kernel (two line buffers, six real lines, the reduction)
inline size_t moment_lds_bytes(int N, int csize, int threads) {
  const size_t real = csize / 2;
  return 2 * (size_t)N * csize + (size_t)6 * N * real + (N & 1) * real + (size_t)threads * sizeof(double);
}


// ---------------------------------------------------------------------------
// z forward + assembly + stage update.  Each field is transformed along z; with the phase
// shift the kept unshifted product (akeep) is transformed too and the mean
// (P0 + P1 exp(-i pi kz / N)) / 2 taken.  Modes outside the retained set are dropped; then
// F_u = P(k) c_hat + A 1_band u_hat (+ the stochastic band term), F_phi = -a_hat, and the
// update of the stage (dy/dt for stage < 0) exactly as the tuned kernels do it.
// ---------------------------------------------------------------------------
template <typename T>
struct GStage {
  cpx<T>* yn;
  cpx<T>* acc;
  cpx<T>* ys;
  const cpx<T>* sin;
  cpx<T>* rhs;
  const double* fband;
  int stage;
};

template <typename T>
__device__ __forceinline__ cpx<T> update(const GStage<T>& a, long long o, cpx<T> F, double lk2, double h, bool expl) {
  if (a.stage < 0) {
    a.rhs[o] = F - T(lk2) * a.sin[o];
    return {T(0), T(0)};
  }
  const cpx<T> y = a.stage < 3 ? a.yn[o] : cpx<T>{T(0), T(0)};
  T eh, e1;
  if (expl) {
    F = F - T(lk2) * (a.stage == 0 ? y : a.sin[o]);
    eh = e1 = T(1);
  } else {
    const double e = exp(-0.5 * lk2 * h);
    eh = T(e);
    e1 = T(e * e);
  }
  const T th = T(h);
  cpx<T> nxt;
  switch (a.stage) {
    case 0:
      a.acc[o] = e1 * (y + (th / T(6)) * F);
      nxt = eh * (y + (th / T(2)) * F);
      break;
    case 1:
      a.acc[o] = a.acc[o] + ((th / T(3)) * eh) * F;
      nxt = eh * y + (th / T(2)) * F;
      break;
    case 2:
      a.acc[o] = a.acc[o] + ((th / T(3)) * eh) * F;
      nxt = e1 * y + (th * eh) * F;
      break;
    default:
      nxt = a.acc[o] + (th / T(6)) * F;
      a.yn[o] = nxt;
      return nxt;
  }
  a.ys[o] = nxt;
  return nxt;
}

// Launch shape of the z-forward pass: blocks of at most 512 threads (64 columns of threads in
// FP32, 128 in FP64, and 8 or 4 columns), so that a thread may hold its P positions
// n = j + TT m of three fields (c1, c2 and the current one) in registers.
inline Shape zf_shape(int N, int csize) {
  Shape s{};
  s.TT = csize == 8 ? 64 : 128;
  if (s.TT > N / 2) s.TT = N / 2;
  s.W = csize == 8 ? 8 : 4;
  while (s.W > 1 && 2 * (size_t)s.W * N * csize > 150 * 1024) s.W /= 2;
  s.lds = 2 * (size_t)s.W * N * csize;
  return s;
}
inline int zf_positions(int N, int TT) { return (N + TT - 1) / TT; }

// The fields go through one transform call in a loop (scalars 0 .. S-1, each updated as soon
// as it is transformed, then the velocity components), each field once, or twice with the
// shift (abuf, then akeep).
template <typename T, int P>
__global__ void __launch_bounds__(512)
k_z_forward_update(const cpx<T>* __restrict__ abuf, const cpx<T>* __restrict__ akeep, GStage<T> sa,
                   const cpx<T>* __restrict__ tw, const SlotDev* __restrict__ slots, const DynDev* __restrict__ dyn,
                   Geom g, Factors fz, int W, int TT) {
  extern __shared__ char lds_raw[];
  cpx<T>* b0 = reinterpret_cast<cpx<T>*>(lds_raw);
  cpx<T>* b1 = b0 + (size_t)W * g.N;
  const int slot = blockIdx.z;
  const SlotDev& sp = slots[slot];
  if (!sp.active) return;
  const int c = threadIdx.x % W, j = threadIdx.x / W;
  const int kx = blockIdx.x * W + c, kyc = blockIdx.y;
  const bool valid = kx < g.KX;
  const int N = g.N, M = g.M, K = g.K;
  const int ky = kyc <= K ? kyc : kyc - M;
  const double h = dyn[slot].dt, A = dyn[slot].A;
  const bool expl = sp.integrator == PSDNS_INTEGRATOR_EXPLICIT;
  const cpx<T>* aslot = abuf + (long long)slot * g.FA * g.a_field;
  const cpx<T>* kslot = akeep ? akeep + (long long)slot * g.F * g.a_field : nullptr;
  const long long sslot = (long long)slot * g.F * g.st_field;
  auto mode_of = [&](int m, long long& o, double& k2) {
    const int n = j + TT * m;
    if (!valid || n >= N) return false;
    const int kz = wave(n, N), kc = compact(kz, K, M);
    if (kc < 0 || !retained(g, kx, ky, kz)) return false;
    o = st_row(kc, kyc, M, g.PX) + kx;
    k2 = double(kx) * kx + double(ky) * ky + double(kz) * kz;
    return true;
  };
  auto stage_of = [&](int f) {
    GStage<T> q = sa;
    const long long foff = sslot + (long long)f * g.st_field;
    q.yn += foff;
    q.acc += foff;
    q.ys += foff;
    q.sin += foff;
    q.rhs += sa.stage < 0 ? foff : 0;
    return q;
  };
  const int S = g.S, per = kslot ? 2 : 1;
  cpx<T> v[P], c1[P], c2[P];
  for (int t = 0; t < (S + 3) * per; ++t) {
    const int fi = t / per, half = t % per;
    const int f = fi < S ? 3 + fi : fi - S;  // A field: scalar fi, or velocity component fi - S
    const cpx<T>* src = (half ? kslot : aslot) + (long long)f * g.a_field;
    for (int n = j; n < N; n += TT)
      b0[n * W + c] = valid ? src[a_row(n, kyc, M, g.PX) + kx] : cpx<T>{T(0), T(0)};
    __syncthreads();
    const cpx<T>* r = fft<false>(b0, b1, fz, W, c, j, TT, tw);
#pragma unroll
    for (int m = 0; m < P; ++m) {
      const int n = j + TT * m;
      if (n < N) {
        const cpx<T> x = r[n * W + c];
        // with the shift abuf holds the shifted product and akeep the unshifted one
        v[m] = half ? T(0.5) * (x + cmul(v[m], conj(shift_of(tw, N, wave(n, N))))) : x;
      }
    }
    __syncthreads();
    if (half + 1 < per) continue;
    if (fi < S) {
      // scalar: F = -a_hat
      const double dif = sp.diff[f];
      const GStage<T> q = stage_of(f);
#pragma unroll
      for (int m = 0; m < P; ++m) {
        long long o;
        double k2;
        if (mode_of(m, o, k2)) {
          const cpx<T> F = k2 == 0.0 ? cpx<T>{T(0), T(0)} : cpx<T>{-v[m].x, -v[m].y};
          update(q, o, F, dif * k2, h, expl);
        }
      }
    } else if (f == 0) {
#pragma unroll
      for (int m = 0; m < P; ++m) c1[m] = v[m];
    } else if (f == 1) {
#pragma unroll
      for (int m = 0; m < P; ++m) c2[m] = v[m];
    }
  }
  // velocity (v holds c3): F = P(k) c_hat + A 1_band u_hat (+ the stochastic band term)
  int kfs = 0;
  while ((double)(kfs + 1) * (kfs + 1) <= sp.kf2) ++kfs;
  if (kfs > K) kfs = K;
  const bool stoch = sp.forcing == PSDNS_FORCING_STOCHASTIC || sp.forcing == PSDNS_FORCING_ALVELIUS;
  const GStage<T> q0 = stage_of(0), q1 = stage_of(1), q2 = stage_of(2);
#pragma unroll
  for (int m = 0; m < P; ++m) {
    long long o;
    double k2;
    if (!mode_of(m, o, k2)) continue;
    const int kz = wave(j + TT * m, N);
    cpx<T> F1 = {T(0), T(0)}, F2 = F1, F3 = F1;
    const bool band = k2 > 0.0 && k2 <= sp.kf2;
    if (k2 > 0.0) {
      cpx<T> p1 = c1[m], p2 = c2[m], p3 = v[m];
      if (stoch && band) {
        const double* e = sa.fband + ((long long)slot * kStochCand + kx + (kfs + 1) * ((ky + kfs) + (2 * kfs + 1) * (kz + kfs))) * 12 + 6;
        p1 = p1 + cpx<T>{T(e[0]), T(e[1])};
        p2 = p2 + cpx<T>{T(e[2]), T(e[3])};
        p3 = p3 + cpx<T>{T(e[4]), T(e[5])};
      }
      const T ik2 = T(1.0 / k2);
      const T kxt = T(kx), kyt = T(ky), kzt = T(kz);
      const cpx<T> kdc = kxt * p1 + kyt * p2 + kzt * p3;
      F1 = p1 - (kxt * ik2) * kdc;
      F2 = p2 - (kyt * ik2) * kdc;
      F3 = p3 - (kzt * ik2) * kdc;
      if (A != 0.0 && band) {
        const T At = T(A);
        F1 = F1 + At * q0.sin[o];
        F2 = F2 + At * q1.sin[o];
        F3 = F3 + At * q2.sin[o];
      }
    }
    const double lk2 = sp.nu * k2;
    update(q0, o, F1, lk2, h, expl);
    update(q1, o, F2, lk2, h, expl);
    update(q2, o, F3, lk2, h, expl);
  }
}

// ---------------------------------------------------------------------------
// moments of nf B fields along x lines (statistics): FP64 sums of f^2, f^3, f^4 of the
// fields [mom0, nf) and max |u1|+|u2|+|u3| when fields 0..2 are the velocity (with_max).
// A fixed grid of blocks walks the lines in a fixed order; one partial record per block:
// [3 (nf - mom0)] moments then the max, 3 6 + 1 doubles apart.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256)
k_x_moments(const cpx<T>* __restrict__ bbuf, const cpx<T>* __restrict__ tw, Geom g, Factors fx, int nf, int mom0,
            int with_max, double* __restrict__ part) {
  extern __shared__ char lds_raw[];
  const int N = g.N, K = g.K;
  cpx<T>* b0 = reinterpret_cast<cpx<T>*>(lds_raw);
  cpx<T>* b1 = b0 + N;
  T* uabs = reinterpret_cast<T*>(b1 + N);       // running |u1| + |u2| + |u3| per position
  double* red = reinterpret_cast<double*>(uabs + N + (N & 1));
  const int slot = blockIdx.y;
  const int TT = blockDim.x, j = threadIdx.x;
  double mom[6][3];
  for (int f = 0; f < 6; ++f) mom[f][0] = mom[f][1] = mom[f][2] = 0.0;
  double mx = 0.0;
  const long long nlines = (long long)N * N;
  for (long long line = blockIdx.x; line < nlines; line += gridDim.x) {
    const cpx<T>* lbase = bbuf + (long long)slot * g.FB * g.b_field + line * g.PX;
    for (int f = 0; f < nf; f += 2) {
      const int fb = f + 1 < nf ? f + 1 : -1;
      for (int n = j; n < N; n += TT) {
        cpx<T> h = {T(0), T(0)};
        const int kx = n <= K ? n : (n >= N - K ? N - n : -1);
        if (kx >= 0) {
          cpx<T> a = lbase[(long long)f * g.b_field + kx];
          cpx<T> b = fb >= 0 ? lbase[(long long)fb * g.b_field + kx] : cpx<T>{T(0), T(0)};
          if (kx == 0) {
            a.y = T(0);
            b.y = T(0);
          }
          h = n <= K ? a + mul_i(b) : conj(a) + mul_i(conj(b));
        }
        b0[n] = h;
      }
      __syncthreads();
      const cpx<T>* r = fft<true>(b0, b1, fx, 1, 0, j, TT, tw);
      for (int n = j; n < N; n += TT) {
        const double vx = r[n].x, vy = r[n].y;
#pragma unroll
        for (int q = 0; q < 6; ++q) {
          if (q == f && f >= mom0) {
            const double v2 = vx * vx;
            mom[q][0] += v2;
            mom[q][1] += v2 * vx;
            mom[q][2] += v2 * v2;
          }
          if (q == fb && fb >= mom0) {
            const double v2 = vy * vy;
            mom[q][0] += v2;
            mom[q][1] += v2 * vy;
            mom[q][2] += v2 * v2;
          }
        }
        if (with_max && f == 0) uabs[n] = T(fabs(vx) + fabs(vy));
        if (with_max && f == 2) {
          const double sm = (double)fabs(r[n].x) + (double)uabs[n];
          mx = (sm > mx || sm != sm) ? sm : mx;
        }
      }
      __syncthreads();
    }
  }
  const int nm = nf - mom0;
  double* out = part + ((long long)slot * gridDim.x + blockIdx.x) * (3 * 6 + 1);
  for (int q = 0; q < 3 * nm + 1; ++q) {
    double v = 0.0;
    if (q < 3 * nm) {
#pragma unroll
      for (int f = 0; f < 6; ++f)
#pragma unroll
        for (int r = 0; r < 3; ++r)
          if (f == mom0 + q / 3 && r == q % 3) v = mom[f][r];
    } else {
      v = mx;
    }
    red[j] = v;
    __syncthreads();
    for (int o = TT / 2; o > 0; o >>= 1) {
      if (j < o) {
        const double a = red[j], b = red[j + o];
        red[j] = q < 3 * nm ? a + b : ((b > a || b != b) ? b : a);
      }
      __syncthreads();
    }
    if (j == 0) out[q] = red[0];
    __syncthreads();
  }
}

}  // namespace gen
}  // namespace psdns
