// Register/LDS FFT engine for gfx950 (64-wide wavefronts).
//
// A length-N complex line is spread over TT = N/E threads; thread j holds the
// E elements at positions j + TT*m (m = 0..E-1).  The transform runs as
// Stockham autosort stages of radix R <= E (each thread performs E/R
// butterflies per stage); between stages the line is exchanged through LDS.
// The input and output ownership are the same strided pattern, so a batch of
// lines laid out with the line index contiguous in memory (columns) is read
// and written with fully coalesced 128-byte rows, and a contiguous line is
// read with consecutive lanes on consecutive elements.
//
// Sign convention: forward uses exp(-2 pi i n k / N) (the unnormalised forward
// transform of Eq. (5)); inverse uses exp(+2 pi i n k / N) without 1/N.
#pragma once
#include <hip/hip_runtime.h>

namespace psdns {

template <typename T>
struct alignas(2 * sizeof(T)) cpx {
  T x, y;
};

template <typename T>
__device__ __forceinline__ cpx<T> operator+(cpx<T> a, cpx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ cpx<T> operator-(cpx<T> a, cpx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__device__ __forceinline__ cpx<T> operator*(T s, cpx<T> a) { return {s * a.x, s * a.y}; }
template <typename T>
__device__ __forceinline__ cpx<T> cmul(cpx<T> a, cpx<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T>
__device__ __forceinline__ cpx<T> conj(cpx<T> a) { return {a.x, -a.y}; }
// multiply by +i and by -i
template <typename T>
__device__ __forceinline__ cpx<T> mul_i(cpx<T> a) { return {-a.y, a.x}; }
template <typename T>
__device__ __forceinline__ cpx<T> mul_mi(cpx<T> a) { return {a.y, -a.x}; }
// multiply by i*s for a real s
template <typename T>
__device__ __forceinline__ cpx<T> mul_is(cpx<T> a, T s) { return {-s * a.y, s * a.x}; }

// cos(pi m / 32), m = 0..16: a quarter wave of the 64th roots of unity.
__host__ __device__ constexpr double quarter_cos64(int m) {
  switch (m) {
    case 0: return 1.0;
    case 1: return 0.99518472667219688624;
    case 2: return 0.98078528040323044913;
    case 3: return 0.95694033573220886494;
    case 4: return 0.92387953251128675613;
    case 5: return 0.88192126434835502971;
    case 6: return 0.83146961230254523708;
    case 7: return 0.77301045336273696081;
    case 8: return 0.70710678118654752440;
    case 9: return 0.63439328416364549822;
    case 10: return 0.55557023301960222474;
    case 11: return 0.47139673682599764856;
    case 12: return 0.38268343236508977173;
    case 13: return 0.29028467725446236764;
    case 14: return 0.19509032201612826785;
    case 15: return 0.09801714032956060199;
    default: return 0.0;
  }
}

// cos(2 pi m / 64) for any integer m, by symmetry of the quarter wave.
__host__ __device__ constexpr double cos64(int m) {
  m &= 63;
  return m <= 16 ? quarter_cos64(m)
       : m <= 32 ? -quarter_cos64(32 - m)
       : m <= 48 ? -quarter_cos64(m - 32)
                 : quarter_cos64(64 - m);
}
__host__ __device__ constexpr double sin64(int m) { return cos64(m - 16); }

// a * exp(-+ 2 pi i m / 64) with m a compile-time constant after unrolling.
// The trivial roots become swaps/negations so no multiplication by 0 or 1 survives.
template <bool INV, typename T>
__device__ __forceinline__ cpx<T> rot64(cpx<T> a, int m) {
  m &= 63;
  if (m == 0) return a;
  if (m == 32) return {-a.x, -a.y};
  if (m == 16) return INV ? mul_i(a) : mul_mi(a);
  if (m == 48) return INV ? mul_mi(a) : mul_i(a);
  const T c = static_cast<T>(cos64(m));
  const T s = INV ? static_cast<T>(sin64(m)) : static_cast<T>(-sin64(m));
  return {a.x * c - a.y * s, a.x * s + a.y * c};
}

template <int R>
__device__ constexpr int bitrev(int i) {
  int r = 0;
  for (int b = 1; b < R; b <<= 1) {
    r = (r << 1) | (i & 1);
    i >>= 1;
  }
  return r;
}

// In-register R-point DFT (R a power of two, R <= 64): radix-2 decimation in
// frequency followed by the bit-reversal permutation (free in registers).
template <int R, bool INV, typename T>
__device__ __forceinline__ void dft(cpx<T> (&a)[R]) {
#pragma unroll
  for (int len = R; len >= 2; len >>= 1) {
    const int half = len >> 1;
#pragma unroll
    for (int s = 0; s < R; s += len) {
#pragma unroll
      for (int j = 0; j < half; ++j) {
        const cpx<T> u = a[s + j];
        const cpx<T> w = a[s + j + half];
        a[s + j] = u + w;
        a[s + j + half] = rot64<INV>(u - w, j * (64 / len));
      }
    }
  }
  cpx<T> b[R];
#pragma unroll
  for (int i = 0; i < R; ++i) b[i] = a[bitrev<R>(i)];
#pragma unroll
  for (int i = 0; i < R; ++i) a[i] = b[i];
}

// LDS views used for the inter-stage exchange; x is the running exchange index.
// Columns: element p of the line owned by lane column c sits at base[p * W].  With
// SPAN > 0 two buffers SPAN entries apart alternate between exchanges, so a buffer
// is only rewritten after the barrier of the following exchange, which every thread
// reaches after its reads: one barrier per exchange instead of two.
template <typename T, int W, int SPAN = 0>
struct LdsCol {
  static constexpr bool kDouble = SPAN > 0;
  cpx<T>* base;
  __device__ __forceinline__ void st(int p, cpx<T> v, int x) const { base[(x & 1) * SPAN + p * W] = v; }
  __device__ __forceinline__ cpx<T> ld(int p, int x) const { return base[(x & 1) * SPAN + p * W]; }
};
// Contiguous line (one line per E-element lane group): element p is stored at
// p ^ ((p >> log2 E) & min(31, N-1)).  The XOR swizzle keeps the Stockham writes
// (stride E between lanes in the first stage, runs of E lanes later) and the
// strided reads free of LDS bank conflicts for 32 and 64 banks of 4 bytes.
template <typename T, int N, int E>
struct LdsLine {
  cpx<T>* base;
  static constexpr int kShift = E == 1 ? 0 : E == 2 ? 1 : E == 4 ? 2 : E == 8 ? 3 : E == 16 ? 4 : E == 32 ? 5 : 6;
  static constexpr int kMask = N - 1 < 31 ? N - 1 : 31;
  static constexpr bool kDouble = false;
  static __device__ __forceinline__ int idx(int p) { return p ^ ((p >> kShift) & kMask); }
  __device__ __forceinline__ void st(int p, cpx<T> v, int = 0) const { base[idx(p)] = v; }
  __device__ __forceinline__ cpx<T> ld(int p, int = 0) const { return base[idx(p)]; }
};
template <int N>
struct LinePad {
  static constexpr int value = N + N / 16;
};

// Exchange synchronisation: the whole block (lines spread over several
// wavefronts) or one wavefront (every line owned by lanes of a single wave;
// LDS operations of a wave execute in order, so only compiler ordering is needed).
struct BlockSync {
  static __device__ __forceinline__ void sync() { __syncthreads(); }
};
struct WaveSync {
  static __device__ __forceinline__ void sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
};

// Number of stage twiddles one thread applies (all stages after the first).
template <int N, int E, int NS = 1>
__host__ __device__ constexpr int tw_count() {
  if constexpr (NS >= N) {
    return 0;
  } else {
    constexpr int R = (NS * E <= N) ? E : N / NS;
    constexpr int NB = E / R;
    return (NS > 1 ? NB * (R - 1) : 0) + tw_count<N, E, NS * R>();
  }
}

// The twiddles of one thread kept in registers: identical for every line the
// thread transforms, so they are read from the table once.
template <int N, int E, typename T>
struct TwReg {
  static constexpr int C = tw_count<N, E>() > 0 ? tw_count<N, E>() : 1;
  cpx<T> w[C];
};

template <int N, int E, int NS, int OFF, typename T>
__device__ __forceinline__ void tw_fill_stage(TwReg<N, E, T>& t, int j, const cpx<T>* __restrict__ tw) {
  if constexpr (NS < N) {
    constexpr int TT = N / E;
    constexpr int R = (NS * E <= N) ? E : N / NS;
    constexpr int NB = E / R;
    if constexpr (NS > 1) {
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const int kv = (j + TT * b) & (NS - 1);
#pragma unroll
        for (int r = 1; r < R; ++r) t.w[OFF + b * (R - 1) + r - 1] = tw[r * kv * (N / (NS * R))];
      }
      tw_fill_stage<N, E, NS * R, OFF + NB * (R - 1)>(t, j, tw);
    } else {
      tw_fill_stage<N, E, NS * R, OFF>(t, j, tw);
    }
  }
}

template <int N, int E, typename T>
__device__ __forceinline__ TwReg<N, E, T> tw_fill(int j, const cpx<T>* __restrict__ tw) {
  TwReg<N, E, T> t;
  tw_fill_stage<N, E, 1, 0>(t, j, tw);
  return t;
}

// stage twiddle of butterfly b, element r: from a table (pointer) or from registers
template <int N, int E, int OFF, int R, typename T>
__device__ __forceinline__ cpx<T> tw_get(const cpx<T>* __restrict__ tw, int b, int r, int idx) {
  return tw[idx];
}
template <int N, int E, int OFF, int R, typename T>
__device__ __forceinline__ cpx<T> tw_get(const TwReg<N, E, T>& t, int b, int r, int idx) {
  return t.w[OFF + b * (R - 1) + r - 1];
}

// Number of LDS exchanges of an N-point transform with E elements per thread.
template <int N, int E, int NS = 1>
__host__ __device__ constexpr int exchanges() {
  if constexpr (NS >= N) {
    return 0;
  } else {
    constexpr int R = (NS * E <= N) ? E : N / NS;
    return (NS * R == N ? 0 : 1) + exchanges<N, E, NS * R>();
  }
}

// One Stockham stage (and, recursively, the ones after it).
// NS = product of the radices already applied; OFF = twiddles used so far;
// XI = exchanges done so far.
template <int N, int E, bool INV, int NS, int OFF, class Sync, int XI = 0, typename T, class Lds, class Tw>
__device__ __forceinline__ void fft_stage(cpx<T> (&v)[E], const Lds& lds, int j, const Tw& tw) {
  if constexpr (NS < N) {
    constexpr int TT = N / E;
    constexpr int R = (NS * E <= N) ? E : N / NS;
    constexpr int NB = E / R;
    constexpr bool LAST = (NS * R == N);
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int vb = j + TT * b;
      const int kv = vb & (NS - 1);
      cpx<T> a[R];
#pragma unroll
      for (int r = 0; r < R; ++r) a[r] = v[b + r * NB];
      if constexpr (NS > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          cpx<T> w = tw_get<N, E, OFF, R, T>(tw, b, r, r * kv * (N / (NS * R)));
          if (INV) w.y = -w.y;
          a[r] = cmul(a[r], w);
        }
      }
      dft<R, INV>(a);
      if constexpr (LAST) {
#pragma unroll
        for (int r = 0; r < R; ++r) v[b + r * NB] = a[r];
      } else {
        const int base = (vb / NS) * NS * R + kv;
#pragma unroll
        for (int r = 0; r < R; ++r) lds.st(base + r * NS, a[r], XI);
      }
    }
    if constexpr (!LAST) {
      Sync::sync();
#pragma unroll
      for (int m = 0; m < E; ++m) v[m] = lds.ld(j + TT * m, XI);
      // with two buffers the trailing barrier is needed only where the next transform
      // would reuse this buffer first: after the last exchange of an odd count
      constexpr int NX = exchanges<N, E>();
      if constexpr (!Lds::kDouble || (XI + 1 == NX && NX % 2 == 1)) Sync::sync();
      fft_stage<N, E, INV, NS * R, (NS > 1 ? OFF + NB * (R - 1) : OFF), Sync, XI + 1>(v, lds, j, tw);
    }
  }
}

// Full N-point transform of the strided register line.  With BlockSync every
// thread of the block must call it; with WaveSync every lane of the wave.
// tw is either a pointer to w_N^m, m = 0..N-1 (normally a copy staged in LDS),
// or the thread's TwReg.
template <int N, int E, bool INV, class Sync = BlockSync, typename T, class Lds, class Tw>
__device__ __forceinline__ void fft(cpx<T> (&v)[E], const Lds& lds, int j, const Tw& tw) {
  fft_stage<N, E, INV, 1, 0, Sync>(v, lds, j, tw);
}

// Copy the N twiddles into LDS (block-wide; ends with a block barrier).
template <int N, typename T>
__device__ __forceinline__ void stage_twiddles(cpx<T>* dst, const cpx<T>* __restrict__ src) {
  for (int i = threadIdx.x; i < N; i += blockDim.x) dst[i] = src[i];
  __syncthreads();
}

}  // namespace psdns
