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

namespace dgvol {

constexpr int FWD_WPB = 8;   // waves per workgroup of every forward launch
constexpr int ADJ_WPB = 8;

// body ids (DG_BODY_STAGED, DG_BODY_CHUNKREG in dgvol.h)
constexpr int BODY_STAGED = DG_BODY_STAGED;
constexpr int BODY_CHUNKREG = DG_BODY_CHUNKREG;

template <int NP>
constexpr bool f64_staged_ok() { return fwd_f64_staged_lds<NP, FWD_WPB>() <= 160 * 1024; }

template <int NP, int BODY>
constexpr int f64_lds() {
  return BODY == BODY_STAGED ? fwd_f64_staged_lds<NP, FWD_WPB>() : fwd_f64_chunkreg_lds<NP, FWD_WPB>();
}
template <int NP, int BODY>
constexpr int f32s_lds() {
  return BODY == BODY_STAGED ? fwd_f32s_staged_lds<NP, FWD_WPB>() : fwd_f32s_chunkreg_lds<NP, FWD_WPB>();
}

// ------------------------------------------------------------------ single-group kernels

template <int NP, int BODY>
__global__ __launch_bounds__(WAVE* FWD_WPB) void fwd_f64_kernel(FwdArgs<double> p) {
  extern __shared__ __attribute__((aligned(16))) char lds[];
  if constexpr (BODY == BODY_STAGED)
    fwd_f64_staged_body<NP, FWD_WPB>(p, blockIdx.x, gridDim.x, lds);
  else
    fwd_f64_chunkreg_body<NP, FWD_WPB>(p, blockIdx.x, gridDim.x, lds);
}

template <int NP, int BODY>
__global__ __launch_bounds__(WAVE* FWD_WPB) void fwd_f32s_kernel(FwdArgs<float> p) {
  extern __shared__ __attribute__((aligned(16))) char lds[];
  if constexpr (BODY == BODY_STAGED)
    fwd_f32s_staged_body<NP, FWD_WPB>(p, blockIdx.x, gridDim.x, lds);
  else
    fwd_f32s_chunkreg_body<NP, FWD_WPB>(p, blockIdx.x, gridDim.x, lds);
}

// ------------------------------------------------------------------ mixed-order batched kernels
//
// One persistent launch over up to MAX_GROUPS element groups of different
// orders.  Workgroups are split between groups on the host in proportion to
// each group's cost (a static partition: deterministic, no device-side queue,
// nothing to reset between launches, so the launch can be captured in a
// graph).  Block b belongs to the group g with wg_begin[g] <= b < wg_begin[g+1]
// and runs that group's body with its rank and count within the group.

constexpr int MAX_GROUPS = DG_MAX_GROUPS;

struct GroupDev {
  int32_t Np;
  int32_t body;
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

#define DGVOL_CASE64(NPV) \
  case NPV * 2 + BODY_CHUNKREG: fwd_f64_chunkreg_body<NPV, FWD_WPB>(p, bid, nblk, lds); break;

__global__ __launch_bounds__(WAVE* FWD_WPB) void batched_f64_kernel(BatchArgs a) {
  extern __shared__ __attribute__((aligned(16))) char lds[];
  const int gi = find_group(a);
  const GroupDev& gd = a.g[gi];
  const uint32_t bid = blockIdx.x - a.wg_begin[gi];
  const uint32_t nblk = a.wg_begin[gi + 1] - a.wg_begin[gi];
  const FwdArgs<double> p = group_args<double>(gd, a.F);
  switch (gd.Np * 2 + gd.body) {
    case 4 * 2 + BODY_STAGED: fwd_f64_staged_body<4, FWD_WPB>(p, bid, nblk, lds); break;
    case 10 * 2 + BODY_STAGED: fwd_f64_staged_body<10, FWD_WPB>(p, bid, nblk, lds); break;
    case 20 * 2 + BODY_STAGED: fwd_f64_staged_body<20, FWD_WPB>(p, bid, nblk, lds); break;
    case 35 * 2 + BODY_STAGED: fwd_f64_staged_body<35, FWD_WPB>(p, bid, nblk, lds); break;
    case 56 * 2 + BODY_STAGED: fwd_f64_staged_body<56, FWD_WPB>(p, bid, nblk, lds); break;
    DGVOL_CASE64(4)
    DGVOL_CASE64(10)
    DGVOL_CASE64(20)
    DGVOL_CASE64(35)
    DGVOL_CASE64(56)
    DGVOL_CASE64(84)
    DGVOL_CASE64(120)
    default: break;
  }
}
#undef DGVOL_CASE64

#define DGVOL_CASE32(NPV)                                                                   \
  case NPV * 2 + BODY_STAGED: fwd_f32s_staged_body<NPV, FWD_WPB>(p, bid, nblk, lds); break; \
  case NPV * 2 + BODY_CHUNKREG: fwd_f32s_chunkreg_body<NPV, FWD_WPB>(p, bid, nblk, lds); break;

__global__ __launch_bounds__(WAVE* FWD_WPB) void batched_f32s_kernel(BatchArgs a) {
  extern __shared__ __attribute__((aligned(16))) char lds[];
  const int gi = find_group(a);
  const GroupDev& gd = a.g[gi];
  const uint32_t bid = blockIdx.x - a.wg_begin[gi];
  const uint32_t nblk = a.wg_begin[gi + 1] - a.wg_begin[gi];
  const FwdArgs<float> p = group_args<float>(gd, a.F);
  switch (gd.Np * 2 + gd.body) {
    DGVOL_CASE32(4)
    DGVOL_CASE32(10)
    DGVOL_CASE32(20)
    DGVOL_CASE32(35)
    DGVOL_CASE32(56)
    DGVOL_CASE32(84)
    DGVOL_CASE32(120)
    default: break;
  }
}
#undef DGVOL_CASE32

// ------------------------------------------------------------------ stream calibration
//
// Reads n doubles once and writes `copies` scaled copies of them (dst[c*n + i]
// = (c + 1) * src[i]) with contiguous 8-byte accesses, stored as the forward
// kernels store their output planes (streaming stores).  With copies = 1 this is
// a plain copy of known size (the scale of the hardware byte counters); with
// copies = 3 it moves bytes in the forward kernel's 1 : 3 read : write mix with
// no other work (the practical streaming ceiling for that mix).
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
