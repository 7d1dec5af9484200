// Device helpers shared by the DG volume kernels: vector types, MFMA operand
// gathers from D, BF16 splitting, wave-level synchronisation.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "dgvol_layout.hpp"

namespace dgvol {

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));

// The value of lane M of each row of 16 lanes, in every lane of that row
// (DPP row_newbcast on each 32-bit half).  Every lane of the wave must be active.
template <int M>
__device__ __forceinline__ double row_bcast_f64(double v) {
  static_assert(M >= 0 && M < 16, "lane within a row");
  const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
  const int lo = __builtin_amdgcn_mov_dpp((int)(unsigned int)b, 0x150 + M, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(unsigned int)(b >> 32), 0x150 + M, 0xf, 0xf, false);
  return __builtin_bit_cast(double, ((unsigned long long)(unsigned int)hi << 32) | (unsigned int)lo);
}
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int WAVE = 64;

// Wave-level barrier with LDS visibility (lanes of one wave exchanging data
// through LDS).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ------------------------------------------------------------------ FP64 A operands

// A operand of output tile T, k-step s, for lane `lane`, read from row-major D.
// FP64 result rows are 4q + g, so A row m holds slot q = m / 4 of lane group g = m % 4.
template <int NP>
__device__ __forceinline__ double afrag_f64(const double* __restrict__ D, int T, int s, int lane) {
  const int m = lane & 15, kk = lane >> 4;
  const int q = m >> 2, g = m & 3;
  const int sigma = 4 * T + q;
  const int a = slot_dir(sigma), i = slot_node(sigma, g), j = 4 * s + kk;
  return (sigma < Shape<NP>::SLOTS && i < NP && j < NP) ? D[(a * NP + i) * NP + j] : 0.0;
}

// A operand of the transposed product (adjoint): tile TJ over output nodes j,
// k-step sp over the slots of the stacked cotangent W.
template <int NP>
__device__ __forceinline__ double afragT_f64(const double* __restrict__ D, int TJ, int sp, int lane) {
  const int m = lane & 15, kk = lane >> 4;
  const int j = 16 * TJ + m;
  const int a = slot_dir(sp), i = slot_node(sp, kk);
  return (j < NP && i < NP) ? D[(a * NP + i) * NP + j] : 0.0;
}

template <int NP>
constexpr int fwd_table_doubles() { return Shape<NP>::MT * Shape<NP>::KS64 * WAVE; }

// XOR swizzle of the A table: entry `lane` of row (T, s) sits at
// lane ^ ((s & 3) << 2) ^ ((lane >> 4) & 3).  Both the forward reads (a row,
// all lanes) and the transposed reads (16 lanes spread over 4 rows and the 4
// lane groups of a row) then touch 16 distinct 8-byte banks per 16 lanes; with
// the first term alone the transposed reads were 4-way bank conflicts.
__device__ __forceinline__ int tswz(int lane, int s) { return lane ^ ((s & 3) << 2) ^ ((lane >> 4) & 3); }

// Output planes are written once and not read again by the launch; streaming
// (non-temporal) stores measured faster for them on MI355X than ordinary ones
// (1:3 read:write stream +2 %, split-BF16 forward 10-16 %).
template <class T>
__device__ __forceinline__ void store_stream(T* p, const T& v) { __builtin_nontemporal_store(v, p); }

// Raw buffer access: loads past the descriptor's byte range return zero and
// stores past it are dropped by the hardware range check, so a wave can issue
// every load and store of a partial tile unconditionally.  With no branches
// around them the compiler counts the memory operations in flight exactly and
// waits only for the ones an instruction needs.
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_range(const void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}
__device__ __forceinline__ double buffer_load_f64(__amdgpu_buffer_rsrc_t r, uint32_t byte_off) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)byte_off, 0, 0));
}
// streaming (non-temporal) store, as store_stream
__device__ __forceinline__ void buffer_store_stream_f64(__amdgpu_buffer_rsrc_t r, uint32_t byte_off, double v) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, (int)byte_off, 0, 2);
}
__device__ __forceinline__ void buffer_store_f64(__amdgpu_buffer_rsrc_t r, uint32_t byte_off, double v) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, (int)byte_off, 0, 0);
}
__device__ __forceinline__ float buffer_load_f32(__amdgpu_buffer_rsrc_t r, uint32_t byte_off) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)byte_off, 0, 0));
}
__device__ __forceinline__ void buffer_store_stream_f32(__amdgpu_buffer_rsrc_t r, uint32_t byte_off, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), r, (int)byte_off, 0, 2);
}
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
// VEC consecutive words as one 16-byte access (VEC * sizeof(T) == 16)
template <typename T, int VEC>
struct WordVec {
  T v[VEC];
};
template <typename T, int VEC>
__device__ __forceinline__ WordVec<T, VEC> buffer_load_vec(__amdgpu_buffer_rsrc_t r, uint32_t byte_off) {
  static_assert(VEC * sizeof(T) == 16, "16-byte access");
  return __builtin_bit_cast(WordVec<T, VEC>, __builtin_amdgcn_raw_buffer_load_b128(r, (int)byte_off, 0, 0));
}
template <typename T, int VEC>
__device__ __forceinline__ void buffer_store_stream_vec(__amdgpu_buffer_rsrc_t r, uint32_t byte_off,
                                                        const WordVec<T, VEC>& x) {
  __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, x), r, (int)byte_off, 0, 2);
}
__device__ __forceinline__ double buffer_load_word(__amdgpu_buffer_rsrc_t r, uint32_t off, double) {
  return buffer_load_f64(r, off);
}
__device__ __forceinline__ float buffer_load_word(__amdgpu_buffer_rsrc_t r, uint32_t off, float) {
  return buffer_load_f32(r, off);
}
__device__ __forceinline__ void buffer_store_stream_word(__amdgpu_buffer_rsrc_t r, uint32_t off, double v) {
  buffer_store_stream_f64(r, off, v);
}
__device__ __forceinline__ void buffer_store_stream_word(__amdgpu_buffer_rsrc_t r, uint32_t off, float v) {
  buffer_store_stream_f32(r, off, v);
}

// ------------------------------------------------------------------ BF16 split

struct alignas(16) Bf16x8Bits {
  uint16_t v[8];
};

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

// x = hi + lo + O(2^-18 |x|) with hi = bf16(x), lo = bf16(x - hi), for two
// values at once on the packed FP32 -> BF16 converter (round to nearest even;
// NaN stays NaN): elements e, e+1 of hi and lo as BF16 bit patterns.
__device__ __forceinline__ void split_bf16_pair(float x0, float x1, Bf16x8Bits& hi, Bf16x8Bits& lo, int e) {
  const uint32_t h = __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2{x0, x1}, bf16x2));
  const float r0 = x0 - __uint_as_float(h << 16);          // exact in FP32
  const float r1 = x1 - __uint_as_float(h & 0xffff0000u);
  const uint32_t l = __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2{r0, r1}, bf16x2));
  hi.v[e] = (uint16_t)(h & 0xffffu);
  hi.v[e + 1] = (uint16_t)(h >> 16);
  lo.v[e] = (uint16_t)(l & 0xffffu);
  lo.v[e + 1] = (uint16_t)(l >> 16);
}

__device__ __forceinline__ bf16x8 as_bf16x8(const Bf16x8Bits& x) { return __builtin_bit_cast(bf16x8, x); }

// A operand (8 consecutive k per lane) of tile T, k-step s of the BF16 MFMA,
// split into hi and lo parts.  BF16 result rows are 4g + q, so A row m holds
// slot q = m % 4 of lane group g = m / 4.
template <int NP>
__device__ __forceinline__ void afrag_bf16(const float* __restrict__ D, int T, int s, int lane,
                                           Bf16x8Bits& hi, Bf16x8Bits& lo) {
  const int m = lane & 15, kk = lane >> 4;
  const int g = m >> 2, q = m & 3;
  const int sigma = 4 * T + q;
  const int a = slot_dir(sigma), i = slot_node(sigma, g);
  const bool row_ok = sigma < Shape<NP>::SLOTS && i < NP;
#pragma unroll
  for (int e = 0; e < 8; e += 2) {
    const int j = 32 * s + 8 * kk + e;
    const float x0 = (row_ok && j < NP) ? D[(a * NP + i) * NP + j] : 0.0f;
    const float x1 = (row_ok && j + 1 < NP) ? D[(a * NP + i) * NP + j + 1] : 0.0f;
    split_bf16_pair(x0, x1, hi, lo, e);
  }
}

template <int NP>
constexpr int bf16_table_entries() { return Shape<NP>::MT * Shape<NP>::KS16 * WAVE; }

__host__ __device__ constexpr int align16(int bytes) { return (bytes + 15) & ~15; }

}  // namespace dgvol
