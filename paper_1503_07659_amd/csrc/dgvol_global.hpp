// The __global__ entry kernels of the library: single-group forward kernels
// (FP64, split-BF16), the mixed-order batched kernels and the bandwidth and
// matrix-core calibration kernels, with the per-form LDS sizes their launches use.  The
// adjoint and D-cotangent kernels live with their bodies (dgvol_adjoint.hpp,
// dgvol_gradd.hpp); the host-side launch code and the C ABI are in
// dgvol_kernels.hip.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "dgvol.h"
#include "dgvol_device.hpp"
#include "dgvol_forward.hpp"
#include "dgvol_forward_f32s.hpp"
#include "dgvol_layout.hpp"
#include "dgvol_variants.hpp"

namespace dgvol {

constexpr int ADJ_WPB = 8;

// body ids (DG_BODY_STAGED, DG_BODY_CHUNKREG in dgvol.h)
constexpr int BODY_STAGED = DG_BODY_STAGED;
constexpr int BODY_CHUNKREG = DG_BODY_CHUNKREG;
constexpr int BODY_LEAN = DG_BODY_STAGED_LEAN;
static_assert(BODY_STAGED == VB_S && BODY_CHUNKREG == VB_C && BODY_LEAN == VB_L, "body ids of the variant tables");

// Dynamic LDS of one workgroup of a variant.
template <int NP, int BODY, int WPB, int TILES>
constexpr int f64_lds() {
  return BODY != BODY_CHUNKREG ? fwd_f64_staged_lds<NP, WPB, TILES>() : fwd_f64_chunkreg_lds<NP, WPB, TILES>();
}
template <int NP, int BODY, int WPB, int TILES>
constexpr int f32s_lds() {
  return BODY == BODY_STAGED ? fwd_f32s_staged_lds<NP, WPB, TILES>() : fwd_f32s_chunkreg_lds<NP, WPB, TILES>();
}

// Every listed variant fits the 160 KiB of LDS of a CU.
#define DGVOL_LDS_CHECK64(NP, IDX, BODY, WPB, TILES, CLS) \
  static_assert(f64_lds<NP, BODY, WPB, TILES>() <= 160 * 1024, "FP64 variant exceeds the LDS");
#define DGVOL_LDS_CHECK32(NP, IDX, BODY, WPB, TILES, CLS) \
  static_assert(f32s_lds<NP, BODY, WPB, TILES>() <= 160 * 1024, "split-BF16 variant exceeds the LDS");
DGVOL_F64_VARIANTS(DGVOL_LDS_CHECK64)
DGVOL_F32S_VARIANTS(DGVOL_LDS_CHECK32)
#undef DGVOL_LDS_CHECK64
#undef DGVOL_LDS_CHECK32

template <int NP, int BODY, int WPB, int TILES>
__device__ __forceinline__ void fwd_f64_body(const FwdArgs<double>& p, uint32_t bid, uint32_t nblk, char* lds) {
  if constexpr (BODY == BODY_LEAN)
    fwd_f64_staged_body<NP, WPB, TILES, true>(p, bid, nblk, lds);
  else if constexpr (BODY == BODY_STAGED)
    fwd_f64_staged_body<NP, WPB, TILES>(p, bid, nblk, lds);
  else
    fwd_f64_chunkreg_body<NP, WPB, TILES>(p, bid, nblk, lds);
}
template <int NP, int BODY, int WPB, int TILES>
__device__ __forceinline__ void fwd_f32s_body(const FwdArgs<float>& p, uint32_t bid, uint32_t nblk, char* lds) {
  if constexpr (BODY == BODY_STAGED)
    fwd_f32s_staged_body<NP, WPB, TILES>(p, bid, nblk, lds);
  else
    fwd_f32s_chunkreg_body<NP, WPB, TILES>(p, bid, nblk, lds);
}

// ------------------------------------------------------------------ single-group kernels
//
// A 4-wave workgroup is held to 168 registers per lane (three workgroups per
// CU); without the bound the compiler takes registers up to one wave per SIMD.
// The lean staged body is held to 128 (two 8-wave workgroups per CU).
constexpr int min_waves_per_eu(int wpb, int body = VB_S) { return body == VB_L ? 4 : wpb == 4 ? 3 : 1; }

template <int NP, int BODY, int WPB, int TILES>
__global__ __launch_bounds__(WAVE* WPB)
__attribute__((amdgpu_waves_per_eu(min_waves_per_eu(WPB, BODY), 8))) void fwd_f64_kernel(FwdArgs<double> p) {
  extern __shared__ __attribute__((aligned(16))) char lds[];
  fwd_f64_body<NP, BODY, WPB, TILES>(p, blockIdx.x, gridDim.x, lds);
}

template <int NP, int BODY, int WPB, int TILES>
__global__ __launch_bounds__(WAVE* WPB)
__attribute__((amdgpu_waves_per_eu(min_waves_per_eu(WPB), 8))) void fwd_f32s_kernel(FwdArgs<float> p) {
  extern __shared__ __attribute__((aligned(16))) char lds[];
  fwd_f32s_body<NP, BODY, WPB, TILES>(p, blockIdx.x, gridDim.x, lds);
}

// ------------------------------------------------------------------ mixed-order batched kernels
//
// One persistent launch over up to MAX_GROUPS element groups of different
// orders.  Workgroups are split between groups on the host in proportion to
// each group's cost (a static partition: deterministic, no device-side queue,
// nothing to reset between launches, so the launch can be captured in a
// graph).  Block b belongs to the group g with wg_begin[g] <= b < wg_begin[g+1]
// and runs that group's variant with its rank and count within the group.
// There is one kernel per variant class (dgvol_variants.hpp); a batch whose
// groups fall into several classes is one launch per class.

constexpr int MAX_GROUPS = DG_MAX_GROUPS;

struct GroupDev {
  int32_t Np;
  int32_t variant;
  uint32_t ncols;
  uint32_t ntiles;
  int64_t plane;
  const void* D;
  const void* G;
  const void* u;
  void* out;
};

struct BatchArgs {
  GroupDev g[MAX_GROUPS];
  uint32_t wg_begin[MAX_GROUPS + 1];
  int32_t ngroups;
  uint32_t F;
};

template <typename T>
__device__ __forceinline__ FwdArgs<T> group_args(const GroupDev& gd, uint32_t F) {
  return FwdArgs<T>{static_cast<const T*>(gd.D), static_cast<const T*>(gd.G), static_cast<const T*>(gd.u),
                    static_cast<T*>(gd.out), gd.ncols, F, gd.plane, gd.ntiles};
}

__device__ __forceinline__ int find_group(const BatchArgs& a) {
  int gi = 0;
  while (gi + 1 < a.ngroups && blockIdx.x >= a.wg_begin[gi + 1]) ++gi;
  return gi;
}

constexpr int class_waves(int cls) { return cls == VCLASS_WAVE4 ? 4 : 8; }
// LIGHT is held to 128 registers per lane (4 waves per SIMD: two 8-wave
// workgroups per CU), WAVE4 to 168 (three 4-wave workgroups per CU)
constexpr int class_min_waves_per_eu(int cls) { return cls == VCLASS_LIGHT ? 4 : cls == VCLASS_WAVE4 ? 3 : 2; }

#define DGVOL_BCASE64(NP, IDX, BODY, WPB, TILES, CLS)                                   \
  case vkey(NP, IDX):                                                                   \
    if constexpr (CLS == C) fwd_f64_body<NP, BODY, WPB, TILES>(p, bid, nblk, lds);     \
    break;
#define DGVOL_BCASE32(NP, IDX, BODY, WPB, TILES, CLS)                                   \
  case vkey(NP, IDX):                                                                   \
    if constexpr (CLS == C) fwd_f32s_body<NP, BODY, WPB, TILES>(p, bid, nblk, lds);    \
    break;

template <int C>
__global__ __launch_bounds__(WAVE* class_waves(C))
__attribute__((amdgpu_waves_per_eu(class_min_waves_per_eu(C), 8))) void batched_f64_kernel(BatchArgs a) {
  extern __shared__ __attribute__((aligned(16))) char lds[];
  const int gi = find_group(a);
  const GroupDev& gd = a.g[gi];
  const uint32_t bid = blockIdx.x - a.wg_begin[gi];
  const uint32_t nblk = a.wg_begin[gi + 1] - a.wg_begin[gi];
  const FwdArgs<double> p = group_args<double>(gd, a.F);
  switch (vkey(gd.Np, gd.variant)) {
    DGVOL_F64_VARIANTS(DGVOL_BCASE64)
    default: break;
  }
}

template <int C>
__global__ __launch_bounds__(WAVE* class_waves(C))
__attribute__((amdgpu_waves_per_eu(class_min_waves_per_eu(C), 8))) void batched_f32s_kernel(BatchArgs a) {
  extern __shared__ __attribute__((aligned(16))) char lds[];
  const int gi = find_group(a);
  const GroupDev& gd = a.g[gi];
  const uint32_t bid = blockIdx.x - a.wg_begin[gi];
  const uint32_t nblk = a.wg_begin[gi + 1] - a.wg_begin[gi];
  const FwdArgs<float> p = group_args<float>(gd, a.F);
  switch (vkey(gd.Np, gd.variant)) {
    DGVOL_F32S_VARIANTS(DGVOL_BCASE32)
    default: break;
  }
}
#undef DGVOL_BCASE64
#undef DGVOL_BCASE32

// ------------------------------------------------------------------ stream calibration
//
// Reads n doubles once and writes `copies` scaled copies of them (dst[c*n + i]
// = (c + 1) * src[i]), with streaming (non-temporal) stores as the forward
// kernels store their output planes.  With copies = 1 this is a plain copy of
// known size (the scale of the hardware byte counters); with copies = 3 it
// moves bytes in the forward kernel's 1 : 3 read : write mix with no other
// work (the streaming ceiling for that mix).
//
// stream16_kernel: one pass, no loop: every thread moves STREAM_U independent
// 16-byte pairs (all loads issued before any store), and the grid covers the
// array once (hundreds of thousands of workgroups for the workload sizes).
// stream_kernel: the fallback for arrays that are not 16-byte aligned or of
// odd length, one 8-byte word per lane in a grid-stride loop.
constexpr int STREAM_U = 4;
constexpr int STREAM_BLOCK = 256;
typedef double f64x2 __attribute__((ext_vector_type(2)));

__global__ __launch_bounds__(STREAM_BLOCK) void stream16_kernel(const f64x2* __restrict__ src,
                                                                f64x2* __restrict__ dst, int64_t n2,
                                                                int32_t copies) {
  const int64_t base = (int64_t)blockIdx.x * (STREAM_BLOCK * STREAM_U) + threadIdx.x;
  f64x2 v[STREAM_U];
#pragma unroll
  for (int q = 0; q < STREAM_U; ++q) {
    const int64_t i = base + (int64_t)STREAM_BLOCK * q;
    v[q] = i < n2 ? src[i] : f64x2{0.0, 0.0};
  }
  for (int32_t c = 0; c < copies; ++c) {
    const double s = (double)(c + 1);
#pragma unroll
    for (int q = 0; q < STREAM_U; ++q) {
      const int64_t i = base + (int64_t)STREAM_BLOCK * q;
      if (i < n2) __builtin_nontemporal_store(v[q] * s, &dst[c * n2 + i]);
    }
  }
}

__global__ __launch_bounds__(256) void stream_kernel(const double* __restrict__ src, double* __restrict__ dst,
                                                     int64_t n, int32_t copies) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const double v = src[i];
    for (int32_t c = 0; c < copies; ++c) store_stream(&dst[c * n + i], (double)(c + 1) * v);
  }
}

// ------------------------------------------------------------------ matrix-core calibration
//
// Every wave runs `iters` rounds of four independent accumulator chains of
// v_mfma_f64_16x16x4f64 with register operands (no memory traffic in the
// loop), then writes one sum per lane, so the work cannot be dropped.  Each
// product depends on the previous one of its chain; the operands stay fixed
// (rewriting a source register of an MFMA in flight would stall the issue).
// Launched with 256 threads; the wider bound keeps the accumulators in VGPRs
// (with a 256-thread bound the compiler moves them through AGPRs every round).
__global__ __launch_bounds__(1024) void mfma_cal_kernel(double* __restrict__ sink, int32_t iters) {
  const int lane = threadIdx.x & 63;
  const double a = 1.0 + 1e-3 * lane, b = 1.0 - 1e-3 * lane;
  f64x4 c0 = f64x4{0.0, 0.0, 0.0, 0.0}, c1 = c0, c2 = c0, c3 = c0;
  for (int32_t it = 0; it < iters; ++it) {
    c0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c0, 0, 0, 0);
    c1 = __builtin_amdgcn_mfma_f64_16x16x4f64(b, a, c1, 0, 0, 0);
    c2 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, a, c2, 0, 0, 0);
    c3 = __builtin_amdgcn_mfma_f64_16x16x4f64(b, b, c3, 0, 0, 0);
  }
  double s = 0.0;
#pragma unroll
  for (int q = 0; q < 4; ++q) s += c0[q] + c1[q] + c2[q] + c3[q];
  sink[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

}  // namespace dgvol
