// The __global__ entry kernels of the library: single-group forward kernels
// (FP64, split-BF16) and the mixed-order batched kernels, with the per-form
// LDS sizes their launches use.  The bandwidth and matrix-core calibration
// kernels are in dgvol_calibrate.hpp.  The
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
// There is one kernel per launch class (dgvol_variants.hpp): ALL8 holds every
// 8-wave variant, the others one variant class each.

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
// workgroups per CU), WAVE4 to 168 (three 4-wave workgroups per CU), HEAVY and
// ALL8 to 256 (the heaviest bodies need them)
constexpr int class_min_waves_per_eu(int cls) { return cls == VCLASS_LIGHT ? 4 : cls == VCLASS_WAVE4 ? 3 : 2; }
// whether launch class C runs a variant of class CLS with WPB waves
constexpr bool class_runs(int C, int CLS, int WPB) { return C == CLS || (C == LCLASS_ALL8 && WPB == 8); }

#define DGVOL_BCASE64(NP, IDX, BODY, WPB, TILES, CLS)                                                \
  case vkey(NP, IDX):                                                                                \
    if constexpr (class_runs(C, CLS, WPB)) fwd_f64_body<NP, BODY, WPB, TILES>(p, bid, nblk, lds);    \
    break;
#define DGVOL_BCASE32(NP, IDX, BODY, WPB, TILES, CLS)                                                \
  case vkey(NP, IDX):                                                                                \
    if constexpr (class_runs(C, CLS, WPB)) fwd_f32s_body<NP, BODY, WPB, TILES>(p, bid, nblk, lds);   \
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

}  // namespace dgvol
