// Vector-memory access of the column passes through buffer resources.
//
// A column pass touches, per thread, E elements of one column in each of several
// fields.  With plain 64-bit pointers every element needs its own address pair in
// VGPRs; with a buffer resource the field base sits in SGPRs, the per-thread part of
// the offset is one VGPR shared by every element and field, and the per-element part
// (a multiple of the row stride, the same for all lanes) is an SGPR offset.  All
// offsets are byte offsets below 2^32 from the resource base, which is therefore set
// per field (and per plane where a field exceeds 4 GiB).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "fft.hpp"

namespace psdns {

// Word 3 of a gfx9 buffer descriptor for raw dword access (data format 32, no swizzle).
constexpr int kBufWord3 = 0x00020000;

// Cache policy of the buffer accesses (the instructions' nt bit).  Every pass writes each
// output element once and the next pass reads it from HBM, so stores of whole 128-byte
// lines are streamed (non-temporal).  A column pass with 64-byte row segments writes the
// two halves of each 128-byte line from two blocks of one XCD; those stores stay cached,
// so that the L2 joins the halves before the line goes to HBM (streamed, each half went
// out alone and the passes moved 8-36% more bytes).  Loads are streamed in the passes
// where that measured faster (the y passes), and left cached where it did not.
constexpr int kPolicyCached = 0;
constexpr int kPolicyStream = 2;
// store policy of a pass whose row segments are ROW_BYTES long
constexpr int store_policy(int row_bytes) { return row_bytes >= 128 ? kPolicyStream : kPolicyCached; }

typedef unsigned int u32x2_t __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4_t __attribute__((ext_vector_type(4)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));
typedef double f64x2_t __attribute__((ext_vector_type(2)));

template <typename T>
struct Buf {
  __amdgpu_buffer_rsrc_t r;
};

template <typename T>
__device__ __forceinline__ Buf<T> make_buf(const cpx<T>* base) {
  // stride 0 (raw buffer), no record limit below 4 GiB
  return {__builtin_amdgcn_make_buffer_rsrc(const_cast<cpx<T>*>(base), 0, -1, kBufWord3)};
}

// Loads go through a two-lane vector of T: taking the lanes of the raw dword vector
// one by one lets the optimiser split the access into single-dword loads.
template <typename T, int POLICY = kPolicyCached>
__device__ __forceinline__ cpx<T> bload(const Buf<T>& b, uint32_t voff, uint32_t soff) {
  if constexpr (sizeof(T) == 4) {
    const f32x2_t v =
        __builtin_bit_cast(f32x2_t, __builtin_amdgcn_raw_buffer_load_b64(b.r, (int)voff, (int)soff, POLICY));
    return {v.x, v.y};
  } else {
    const f64x2_t v =
        __builtin_bit_cast(f64x2_t, __builtin_amdgcn_raw_buffer_load_b128(b.r, (int)voff, (int)soff, POLICY));
    return {v.x, v.y};
  }
}

// A store of more than 64 bits of data needs one wait state before a VALU instruction
// may overwrite its data registers.  The compiler inserts it only for buffer stores
// whose SGPR offset is the constant 0, so the 128-bit (FP64) stores carry their whole
// offset in the VGPR; with the offset in an SGPR the overwrite was observed to corrupt
// stored values now and then.  64-bit (FP32) stores are not affected.
template <int POLICY = kPolicyStream, typename T>
__device__ __forceinline__ void bstore(const Buf<T>& b, uint32_t voff, uint32_t soff, cpx<T> v) {
  if constexpr (sizeof(T) == 4) {
    const f32x2_t w = {v.x, v.y};
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2_t, w), b.r, (int)voff, (int)soff, POLICY);
  } else {
    const f64x2_t w = {v.x, v.y};
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4_t, w), b.r, (int)(voff + soff), 0, POLICY);
  }
}

// Positions along a column of N points handled by a thread: element m of thread j
// is position n = j + TT m.  A compact column keeps the retained positions n <= K
// and n >= N - K only, at compact index n and n - N + M respectively (K = (N-1)/3 for
// the 2/3 rule, or the bounding K of the phase-shift sphere; M = 2K + 1).  For most m
// every thread of a column falls in the same class, so the compact row is j plus a
// uniform shift.
template <int N, int TT, int K_ = (N - 1) / 3>
struct ColPos {
  static constexpr int K = K_;
  static constexpr int M = 2 * K + 1;
  static constexpr bool low(int m) { return TT * m + TT - 1 <= K; }
  static constexpr bool high(int m) { return TT * m >= N - K; }
  static constexpr bool cut(int m) { return TT * m > K && TT * m + TT - 1 < N - K; }
  static constexpr int shift(int m) { return high(m) ? TT * m - N + M : TT * m; }
};

// Byte offsets (vo per thread, so uniform) of element m of a compact column whose
// rows are rsb bytes apart and whose row-0 offset for this thread is voff (that of
// row j).  Returns false where the element is truncated.
template <int N, int TT, int K_ = (N - 1) / 3>
__device__ __forceinline__ bool compact_at(int m, int j, uint32_t voff, uint32_t rsb, uint32_t& vo, uint32_t& so) {
  using P = ColPos<N, TT, K_>;
  if (P::cut(m)) return false;
  if (P::low(m) || P::high(m)) {
    vo = voff;
    so = (uint32_t)P::shift(m) * rsb;
    return true;
  }
  const int n = j + TT * m;
  const int kc = n <= P::K ? n : (n >= N - P::K ? n - N + P::M : -1);
  if (kc < 0) return false;
  // (kc - j) may be negative; the sum wraps to the true offset, which is below 2^32
  vo = voff + (uint32_t)(kc - j) * rsb;
  so = 0;
  return true;
}

}  // namespace psdns
