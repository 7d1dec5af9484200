// Host side of the DG volume derivative library for gfx950 (MI355X): launches and the C ABI.
//
// Forward:  out_b[i] = sum_a G[3a+b] (D_a u)[i]   for every (element, field) column.
// Adjoint:  gu = sum_a D_a^T W_a with W_a = sum_b G[3a+b] gout_b;
//           gG[3a+b] = sum_{f,i} gout_b[i] (D_a u)[i].
// Definitions, layouts and error behaviour are documented in include/dgvol.h;
// the forward data-movement schemes in dgvol_forward.hpp (FP64) and
// dgvol_forward_f32s.hpp (split-BF16), the adjoint in
// dgvol_adjoint.hpp, the D cotangent in dgvol_gradd.hpp, the register layout
// of the products in dgvol_layout.hpp, the entry kernels in dgvol_global.hpp.
// This file holds the host side: launch configuration, validation, the ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>

#include "dgvol.h"
#include "dgvol_adjoint.hpp"
#include "dgvol_adjoint_cr.hpp"
#include "dgvol_device.hpp"
#include "dgvol_forward.hpp"
#include "dgvol_forward_f32s.hpp"
#include "dgvol_global.hpp"
#include "dgvol_gradd.hpp"
#include "dgvol_layout.hpp"

namespace dgvol {

// ------------------------------------------------------------------ launch helpers

constexpr int MAX_DEVICES = 64;

static int current_device(int* err) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0) {
    *err = DG_EDEVICE;
    return -1;
  }
  return dev;
}

static int cu_count(int dev, int* err) {
  static std::atomic<int> cache[MAX_DEVICES];
  if (dev < MAX_DEVICES) {
    const int c = cache[dev].load(std::memory_order_relaxed);
    if (c > 0) return c;
  }
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) {
    *err = DG_EDEVICE;
    return 0;
  }
  if (dev < MAX_DEVICES) cache[dev].store(cus, std::memory_order_relaxed);
  return cus;
}

// Resident workgroups of `kernel` on the whole device (the persistent grid
// size).  Kernels that take all their LDS dynamically (dyn_lds >= 0) get their
// dynamic-LDS limit raised to the full 160 KiB, and are queried with the
// largest size of the request's class (so a cached count is never too large);
// kernels with static LDS only (dyn_lds < 0) are queried as they are.  The
// result is cached per kernel instance, device and class.
template <typename Kern>
static int resident_blocks(Kern kernel, int block, int dyn_lds, int* err) {
  static std::atomic<int> cache[MAX_DEVICES][5];
  const int dev = current_device(err);
  if (dev < 0) return 0;
  const int cls = dyn_lds < 0 ? 4 : dyn_lds <= 40960 ? 0 : dyn_lds <= 81920 ? 1 : dyn_lds <= 122880 ? 2 : 3;
  if (dev < MAX_DEVICES) {
    const int c = cache[dev][cls].load(std::memory_order_relaxed);
    if (c > 0) return c;
  }
  const int cus = cu_count(dev, err);
  if (*err != DG_OK) return 0;
  int probe = 0;
  if (dyn_lds >= 0) {
    // a failure here surfaces as a launch error of a kernel asking for more than the default limit
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                              160 * 1024);
    probe = cls == 0 ? 40960 : cls == 1 ? 81920 : cls == 2 ? 122880 : 160 * 1024;
  }
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, block, probe) != hipSuccess || per_cu <= 0)
    per_cu = 1;
  const int total = cus * per_cu;
  if (dev < MAX_DEVICES) cache[dev][cls].store(total, std::memory_order_relaxed);
  return total;
}

static inline uint32_t ceil_div(uint64_t a, uint64_t b) { return (uint32_t)((a + b - 1) / b); }

// Default body per order: LDS-staged where memory bounds the problem and D
// fits LDS, chunk-register where the matrix cores bound it.
static int default_body_f64(int Np) { return Np <= 56 ? BODY_STAGED : BODY_CHUNKREG; }
static int default_body_f32s(int Np) { return Np <= 84 ? BODY_STAGED : BODY_CHUNKREG; }

static bool body_ok_f64(int Np, int body) {
  if (body == BODY_CHUNKREG) return true;
  if (body != BODY_STAGED) return false;
  switch (Np) {
    case 4: return f64_staged_ok<4>();
    case 10: return f64_staged_ok<10>();
    case 20: return f64_staged_ok<20>();
    case 35: return f64_staged_ok<35>();
    case 56: return f64_staged_ok<56>();
    default: return false;
  }
}
static bool body_ok_f32s(int, int body) { return body == BODY_STAGED || body == BODY_CHUNKREG; }

template <int NP>
static int lds_f64(int body) {
  if constexpr (f64_staged_ok<NP>())
    return body == BODY_STAGED ? f64_lds<NP, BODY_STAGED>() : f64_lds<NP, BODY_CHUNKREG>();
  else
    return f64_lds<NP, BODY_CHUNKREG>();
}
template <int NP>
static int lds_f32s(int body) {
  return body == BODY_STAGED ? f32s_lds<NP, BODY_STAGED>() : f32s_lds<NP, BODY_CHUNKREG>();
}

static int lds_bytes(int form, int Np, int body) {
#define DGVOL_LDS(NPV) \
  case NPV: return form == DG_FORM_F64 ? lds_f64<NPV>(body) : lds_f32s<NPV>(body);
  switch (Np) {
    DGVOL_LDS(4)
    DGVOL_LDS(10)
    DGVOL_LDS(20)
    DGVOL_LDS(35)
    DGVOL_LDS(56)
    DGVOL_LDS(84)
    DGVOL_LDS(120)
  }
#undef DGVOL_LDS
  return 0;
}

// 16-column tiles one workgroup processes per step of its loop.
static inline uint32_t tiles_per_block(int form, int Np, int body) {
  if (body == BODY_STAGED) {
    if (form == DG_FORM_F64) return FWD_WPB * (Np <= 4 ? staged_tpi<4>() : Np <= 20 ? staged_tpi<20>() : 1);
    return FWD_WPB * (Np <= 4 ? f32s_tpi<4>() : Np <= 20 ? f32s_tpi<20>() : Np <= 35 ? f32s_tpi<35>() : 1);
  }
  if (form != DG_FORM_F64) return chunk_tpw<4, 4>();
  return Np >= 120 ? chunk_tpw<120, 8>() : chunk_tpw<4, 8>();
}

template <typename Kern, typename Args>
static dg_status launch_persistent(Kern kern, const Args& args, uint32_t ntiles, int form, int Np, int body,
                                   int lds, hipStream_t stream) {
  int err = DG_OK;
  const int cap = resident_blocks(kern, WAVE * FWD_WPB, lds, &err);
  if (err != DG_OK) return err;
  const uint32_t grid = std::min<uint32_t>(ceil_div(ntiles, tiles_per_block(form, Np, body)), (uint32_t)cap);
  hipLaunchKernelGGL(kern, dim3(grid), dim3(WAVE * FWD_WPB), (size_t)lds, stream, args);
  return hipGetLastError() == hipSuccess ? DG_OK : DG_ELAUNCH;
}

template <int NP>
static dg_status launch_fwd_f64(const FwdArgs<double>& p, hipStream_t stream) {
  if constexpr (f64_staged_ok<NP>()) {
    if (default_body_f64(NP) == BODY_STAGED)
      return launch_persistent(fwd_f64_kernel<NP, BODY_STAGED>, p, p.ntiles, DG_FORM_F64, NP, BODY_STAGED,
                               f64_lds<NP, BODY_STAGED>(), stream);
  }
  return launch_persistent(fwd_f64_kernel<NP, BODY_CHUNKREG>, p, p.ntiles, DG_FORM_F64, NP, BODY_CHUNKREG,
                           f64_lds<NP, BODY_CHUNKREG>(), stream);
}

template <int NP>
static dg_status launch_fwd_f32s(const FwdArgs<float>& p, hipStream_t stream) {
  if (default_body_f32s(NP) == BODY_STAGED)
    return launch_persistent(fwd_f32s_kernel<NP, BODY_STAGED>, p, p.ntiles, DG_FORM_F32S, NP, BODY_STAGED,
                             f32s_lds<NP, BODY_STAGED>(), stream);
  return launch_persistent(fwd_f32s_kernel<NP, BODY_CHUNKREG>, p, p.ntiles, DG_FORM_F32S, NP, BODY_CHUNKREG,
                           f32s_lds<NP, BODY_CHUNKREG>(), stream);
}

template <int NP>
static dg_status launch_adj_f64(const double* D, const double* G, const double* u, const double* gout,
                                double* gu, double* gG, int64_t K, int32_t F, hipStream_t stream) {
  const uint32_t E = F <= 16 ? (uint32_t)(16 / F) : 1u;
  const uint32_t nsub = F <= 16 ? 1u : ceil_div((uint64_t)F, 16);
  const uint32_t ntiles = ceil_div((uint64_t)K, E);
  int err = DG_OK;
  if constexpr (NP >= 84) {
    // two chunk-register passes: gu, then gG
    const uint64_t ncols = (uint64_t)K * (uint64_t)F;
    const uint32_t tiles_a = ceil_div(ncols, 16);
    auto ka = adjcr_gu_kernel<NP>;
    const int cap_a = resident_blocks(ka, WAVE * ADJCR_WPB, -1, &err);
    if (err != DG_OK) return err;
    hipLaunchKernelGGL(ka, dim3(std::min<uint32_t>(tiles_a, (uint32_t)cap_a)), dim3(WAVE * ADJCR_WPB), 0, stream, D, G,
                       gout, gu, (uint32_t)ncols, (uint32_t)F, (int64_t)ncols * NP, tiles_a);
    auto kb = adjcr_gG_kernel<NP>;
    const int cap_b = resident_blocks(kb, WAVE * ADJCR_WPB, -1, &err);
    if (err != DG_OK) return err;
    hipLaunchKernelGGL(kb, dim3(std::min<uint32_t>(ntiles, (uint32_t)cap_b)), dim3(WAVE * ADJCR_WPB), 0, stream, D, u,
                       gout, gG, (uint32_t)K, (uint32_t)F, (int64_t)ncols * NP, E, nsub, ntiles);
    return hipGetLastError() == hipSuccess ? DG_OK : DG_ELAUNCH;
  } else {
    if (F <= 16) {
      auto kern = adj_f64_staged_kernel<NP, ADJ_WPB>;
      const int cap = resident_blocks(kern, WAVE * ADJ_WPB, -1, &err);
      if (err != DG_OK) return err;
      const uint32_t grid = std::min<uint32_t>(ceil_div(ntiles, ADJ_WPB), (uint32_t)cap);
      hipLaunchKernelGGL(kern, dim3(grid), dim3(WAVE * ADJ_WPB), 0, stream, D, G, u, gout, gu, gG, (uint32_t)K,
                         (uint32_t)F, (int64_t)K * F * NP, E, ntiles);
    } else {
      auto kern = adj_f64_kernel<NP, ADJ_WPB>;
      const int cap = resident_blocks(kern, WAVE * ADJ_WPB, -1, &err);
      if (err != DG_OK) return err;
      const uint32_t grid = std::min<uint32_t>(ceil_div(ntiles, ADJ_WPB), (uint32_t)cap);
      hipLaunchKernelGGL(kern, dim3(grid), dim3(WAVE * ADJ_WPB), 0, stream, D, G, u, gout, gu, gG, (uint32_t)K,
                         (uint32_t)F, (int64_t)K * F * NP, E, nsub, ntiles);
    }
    return hipGetLastError() == hipSuccess ? DG_OK : DG_ELAUNCH;
  }
}

// Partial sums of the D cotangent: a pure function of the problem size, so
// the result does not depend on the device.
static uint32_t gd_parts(int64_t K, int32_t Np, int32_t F) {
  const uint32_t nunits = ceil_div((uint64_t)K * (uint64_t)F, GD_UNIT);
  return std::min<uint32_t>(nunits, gd_maxpart(Np));
}

template <int NP>
static dg_status launch_gd_f64(const double* G, const double* u, const double* gout, double* gD, double* work,
                               int64_t K, int32_t F, hipStream_t stream) {
  using S = GdShape<NP>;
  const uint64_t ncols = (uint64_t)K * (uint64_t)F;
  const uint32_t npart = gd_parts(K, NP, F);
  if (npart > 0) {
    const GdArgs p{G, u, gout, work, (uint32_t)ncols, (uint32_t)F, (int64_t)ncols * NP, ceil_div(ncols, GD_UNIT),
                   npart};
    // with NSPLIT > 1 the grid is rounded up to whole groups of 8 ranges (one per XCD)
    const uint32_t grid = S::NSPLIT == 1 ? npart : ceil_div(npart, 8) * 8 * S::NSPLIT;
    hipLaunchKernelGGL(gd_partial_kernel<NP>, dim3(grid), dim3(S::NTH), 0, stream, p);
  }
  const uint32_t n = 3u * NP * NP;
  hipLaunchKernelGGL(gd_reduce_kernel, dim3(ceil_div(n, 64)), dim3(64 * GD_RED_PG), 0, stream, work, gD, npart,
                     n);
  return hipGetLastError() == hipSuccess ? DG_OK : DG_ELAUNCH;
}

// Estimate of one 16-column tile (seconds), used to split workgroups between
// groups when the caller gives no measured cost: the spec roofline time
// (8 TB/s, spec matrix peak) divided by the fraction of it that the order's
// default body reached in single-order launches on MI355X (F = 3, at the
// autotuner's problem size: at least 2^15 tiles and 256 MB).  Only the ratios
// between groups matter.
static double tile_cost_estimate(int form, int Np, uint32_t F) {
  const double word = form == DG_FORM_F64 ? 8.0 : 4.0;
  const double bytes = 16.0 * word * (4.0 * Np + 9.0 / F);
  const double flops = 16.0 * Np * (6.0 * Np + 15.0);
  const double bw = 8.0e12;
  const double peak = form == DG_FORM_F64 ? 78.6e12 : 2.5e15 / 3.0;  // three BF16 passes
  double eff;
  switch (Np) {
    case 4: eff = form == DG_FORM_F64 ? 0.71 : 0.49; break;
    case 10: eff = form == DG_FORM_F64 ? 0.65 : 0.65; break;
    case 20: eff = form == DG_FORM_F64 ? 0.67 : 0.60; break;
    case 35: eff = form == DG_FORM_F64 ? 0.60 : 0.55; break;
    case 56: eff = form == DG_FORM_F64 ? 0.58 : 0.76; break;
    case 84: eff = form == DG_FORM_F64 ? 0.43 : 0.70; break;
    default: eff = form == DG_FORM_F64 ? 0.60 : 0.55; break;  // Np = 120
  }
  return std::max(bytes / bw, flops / peak) / eff;
}

// ------------------------------------------------------------------ validation

static inline bool aligned(const void* p, uintptr_t a) { return ((uintptr_t)p & (a - 1)) == 0; }

// Common checks; returns DG_OK, or an error.  *noop is set when K == 0.
static dg_status check_common(int64_t K, int32_t Np, int32_t F, bool* noop) {
  *noop = false;
  if (K < 0 || F < 1) return DG_EINVAL;
  if (!dg_supported_np(Np)) return DG_EUNSUPPORTED;
  // columns (K * F) are indexed in 32 bits
  if ((uint64_t)K * (uint64_t)F > (uint64_t)INT32_MAX) return DG_EINVAL;
  if (K == 0) *noop = true;
  return DG_OK;
}

}  // namespace dgvol

using namespace dgvol;

extern "C" {

int32_t dg_abi_version(void) { return DGVOL_ABI_VERSION; }

const char* dg_strerror(dg_status s) {
  switch (s) {
    case DG_OK: return "success";
    case DG_EINVAL:
      return "invalid argument (null or misaligned pointer, K < 0, F < 1, K*F too large, or a bad group table)";
    case DG_EUNSUPPORTED: return "unsupported node count Np (supported: 4, 10, 20, 35, 56, 84, 120), form or body";
    case DG_ELAUNCH: return "kernel launch failed";
    case DG_EDEVICE: return "could not query the current HIP device";
    default: return "unknown status";
  }
}

int32_t dg_supported_np(int32_t Np) {
  switch (Np) {
    case 4: case 10: case 20: case 35: case 56: case 84: case 120: return 1;
    default: return 0;
  }
}

int32_t dg_body_available(int32_t form, int32_t Np, int32_t body) {
  if (!dg_supported_np(Np)) return 0;
  if (form == DG_FORM_F64) return body_ok_f64(Np, body) ? 1 : 0;
  if (form == DG_FORM_F32S) return body_ok_f32s(Np, body) ? 1 : 0;
  return 0;
}

int32_t dg_default_body(int32_t form, int32_t Np) {
  if (!dg_supported_np(Np)) return -1;
  if (form == DG_FORM_F64) return default_body_f64(Np);
  if (form == DG_FORM_F32S) return default_body_f32s(Np);
  return -1;
}

#define DGVOL_DISPATCH(LAUNCH, ...)            \
  switch (Np) {                                \
    case 4: return LAUNCH<4>(__VA_ARGS__);     \
    case 10: return LAUNCH<10>(__VA_ARGS__);   \
    case 20: return LAUNCH<20>(__VA_ARGS__);   \
    case 35: return LAUNCH<35>(__VA_ARGS__);   \
    case 56: return LAUNCH<56>(__VA_ARGS__);   \
    case 84: return LAUNCH<84>(__VA_ARGS__);   \
    case 120: return LAUNCH<120>(__VA_ARGS__); \
  }                                            \
  return DG_EUNSUPPORTED;

dg_status dg_volume(const double* D, const double* G, const double* u, double* out, int64_t K, int32_t Np,
                    int32_t F, void* stream) {
  bool noop = false;
  const dg_status st = check_common(K, Np, F, &noop);
  if (st != DG_OK || noop) return st;
  if (!D || !G || !u || !out) return DG_EINVAL;
  if (!aligned(D, 8) || !aligned(G, 8) || !aligned(u, 8) || !aligned(out, 8)) return DG_EINVAL;
  const uint64_t ncols = (uint64_t)K * (uint64_t)F;
  const FwdArgs<double> p{D, G, u, out, (uint32_t)ncols, (uint32_t)F, (int64_t)ncols * Np, ceil_div(ncols, 16)};
  DGVOL_DISPATCH(launch_fwd_f64, p, (hipStream_t)stream)
}

dg_status dg_volume_f32s(const float* D, const float* G, const float* u, float* out, int64_t K, int32_t Np,
                         int32_t F, void* stream) {
  bool noop = false;
  const dg_status st = check_common(K, Np, F, &noop);
  if (st != DG_OK || noop) return st;
  if (!D || !G || !u || !out) return DG_EINVAL;
  if (!aligned(D, 4) || !aligned(G, 4) || !aligned(u, 4) || !aligned(out, 4)) return DG_EINVAL;
  const uint64_t ncols = (uint64_t)K * (uint64_t)F;
  const FwdArgs<float> p{D, G, u, out, (uint32_t)ncols, (uint32_t)F, (int64_t)ncols * Np, ceil_div(ncols, 16)};
  DGVOL_DISPATCH(launch_fwd_f32s, p, (hipStream_t)stream)
}

dg_status dg_volume_adjoint(const double* D, const double* G, const double* u, const double* gout, double* gu,
                            double* gG, int64_t K, int32_t Np, int32_t F, void* stream) {
  bool noop = false;
  const dg_status st = check_common(K, Np, F, &noop);
  if (st != DG_OK || noop) return st;
  if (!D || !G || !u || !gout || !gu || !gG) return DG_EINVAL;
  if (!aligned(D, 8) || !aligned(G, 8) || !aligned(u, 8) || !aligned(gout, 8) || !aligned(gu, 8) ||
      !aligned(gG, 8))
    return DG_EINVAL;
  DGVOL_DISPATCH(launch_adj_f64, D, G, u, gout, gu, gG, K, F, (hipStream_t)stream)
}

dg_status dg_volume_grad_d_workspace(int64_t K, int32_t Np, int32_t F, uint64_t* bytes) {
  if (!bytes) return DG_EINVAL;
  bool noop = false;
  const dg_status st = check_common(K, Np, F, &noop);
  if (st != DG_OK) return st;
  *bytes = (uint64_t)gd_parts(K, Np, F) * 3u * (uint64_t)Np * (uint64_t)Np * sizeof(double);
  return DG_OK;
}

dg_status dg_volume_grad_d(const double* G, const double* u, const double* gout, double* gD, void* work,
                           uint64_t work_bytes, int64_t K, int32_t Np, int32_t F, void* stream) {
  bool noop = false;
  const dg_status st = check_common(K, Np, F, &noop);
  if (st != DG_OK) return st;
  if (!gD || !aligned(gD, 8)) return DG_EINVAL;
  uint64_t need = 0;
  dg_volume_grad_d_workspace(K, Np, F, &need);
  if (!noop) {
    if (!G || !u || !gout || !work) return DG_EINVAL;
    if (!aligned(G, 8) || !aligned(u, 8) || !aligned(gout, 8) || !aligned(work, 8)) return DG_EINVAL;
    if (work_bytes < need) return DG_EINVAL;
  }
  DGVOL_DISPATCH(launch_gd_f64, G, u, gout, gD, static_cast<double*>(work), K, F, (hipStream_t)stream)
}

#undef DGVOL_DISPATCH

dg_status dg_volume_batched(const dg_group* groups, int32_t ngroups, int32_t F, int32_t form, void* stream) {
  if (ngroups < 0 || ngroups > DG_MAX_GROUPS || F < 1) return DG_EINVAL;
  if (form != DG_FORM_F64 && form != DG_FORM_F32S) return DG_EUNSUPPORTED;
  if (ngroups > 0 && !groups) return DG_EINVAL;
  const uintptr_t word = form == DG_FORM_F64 ? 8 : 4;
  BatchArgs a{};
  a.F = (uint32_t)F;
  double cost[DG_MAX_GROUPS];
  uint32_t max_blocks[DG_MAX_GROUPS];
  double total_cost = 0.0;
  int lds = 0;
  int ng = 0;
  for (int i = 0; i < ngroups; ++i) {
    const dg_group& gr = groups[i];
    bool noop = false;
    const dg_status st = check_common(gr.K, gr.Np, F, &noop);
    if (st != DG_OK) return st;
    if (gr.body != DG_BODY_AUTO && !dg_body_available(form, gr.Np, gr.body)) return DG_EUNSUPPORTED;
    if (noop) continue;
    if (!gr.D || !gr.G || !gr.u || !gr.out) return DG_EINVAL;
    if (!aligned(gr.D, word) || !aligned(gr.G, word) || !aligned(gr.u, word) || !aligned(gr.out, word))
      return DG_EINVAL;
    const int body = gr.body != DG_BODY_AUTO
                         ? gr.body
                         : (form == DG_FORM_F64 ? default_body_f64(gr.Np) : default_body_f32s(gr.Np));
    const uint64_t ncols = (uint64_t)gr.K * (uint64_t)F;
    GroupDev& gd = a.g[ng];
    gd.Np = gr.Np;
    gd.body = body;
    gd.ncols = (uint32_t)ncols;
    gd.ntiles = ceil_div(ncols, 16);
    gd.plane = (int64_t)ncols * gr.Np;
    gd.D = gr.D;
    gd.G = gr.G;
    gd.u = gr.u;
    gd.out = gr.out;
    const double per_tile = gr.cost > 0.0 ? gr.cost : tile_cost_estimate(form, gr.Np, (uint32_t)F);
    cost[ng] = per_tile * gd.ntiles;
    max_blocks[ng] = ceil_div(gd.ntiles, tiles_per_block(form, gr.Np, body));
    total_cost += cost[ng];
    lds = std::max(lds, lds_bytes(form, gr.Np, body));
    ++ng;
  }
  if (ng == 0) return DG_OK;
  a.ngroups = ng;
  int err = DG_OK;
  const int cap = form == DG_FORM_F64 ? resident_blocks(batched_f64_kernel, WAVE * FWD_WPB, lds, &err)
                                      : resident_blocks(batched_f32s_kernel, WAVE * FWD_WPB, lds, &err);
  if (err != DG_OK) return err;
  // Split the resident workgroups so that the largest cost per workgroup is as
  // small as possible (Jefferson / D'Hondt apportionment): every group gets the
  // whole part of its proportional share, at least one and at most what it can
  // use, then each workgroup left goes to the group with the largest cost per
  // workgroup.  Plain rounding of the shares can leave a small group one
  // workgroup short, and that group then finishes last.
  uint32_t nb[DG_MAX_GROUPS];
  uint32_t used = 0;
  for (int i = 0; i < ng; ++i) {
    const uint32_t share = (uint32_t)((double)cap * cost[i] / total_cost);
    nb[i] = std::max<uint32_t>(1u, std::min(share, max_blocks[i]));
    used += nb[i];
  }
  while (used < (uint32_t)cap) {
    int pick = -1;
    for (int i = 0; i < ng; ++i)
      if (nb[i] < max_blocks[i] && (pick < 0 || cost[i] * nb[pick] > cost[pick] * nb[i])) pick = i;
    if (pick < 0) break;
    ++nb[pick];
    ++used;
  }
  uint32_t begin = 0;
  for (int i = 0; i < ng; ++i) {
    a.wg_begin[i] = begin;
    begin += nb[i];
  }
  for (int i = ng; i <= MAX_GROUPS; ++i) a.wg_begin[i] = begin;
  if (form == DG_FORM_F64)
    hipLaunchKernelGGL(batched_f64_kernel, dim3(begin), dim3(WAVE * FWD_WPB), (size_t)lds, (hipStream_t)stream, a);
  else
    hipLaunchKernelGGL(batched_f32s_kernel, dim3(begin), dim3(WAVE * FWD_WPB), (size_t)lds, (hipStream_t)stream,
                       a);
  return hipGetLastError() == hipSuccess ? DG_OK : DG_ELAUNCH;
}

dg_status dg_stream_calibrate(const double* src, double* dst, int64_t n, int32_t copies, void* stream) {
  if (n < 0 || copies < 1 || copies > 3) return DG_EINVAL;
  if (n == 0) return DG_OK;
  if (!src || !dst || !aligned(src, 8) || !aligned(dst, 8)) return DG_EINVAL;
  int err = DG_OK;
  const int dev = current_device(&err);
  if (dev < 0) return err;
  const int cus = cu_count(dev, &err);
  if (err != DG_OK) return err;
  const int64_t want = (n + 255) / 256;
  const uint32_t grid = (uint32_t)std::min<int64_t>(want, (int64_t)cus * 64);
  hipLaunchKernelGGL(stream_kernel, dim3(grid), dim3(256), 0, (hipStream_t)stream, src, dst, n, copies);
  return hipGetLastError() == hipSuccess ? DG_OK : DG_ELAUNCH;
}

dg_status dg_mfma_calibrate(double* sink, int32_t iters, void* stream) {
  if (!sink || !aligned(sink, 8) || iters < 1) return DG_EINVAL;
  hipLaunchKernelGGL(mfma_cal_kernel, dim3(DG_MFMA_CAL_BLOCKS), dim3(256), 0, (hipStream_t)stream, sink, iters);
  return hipGetLastError() == hipSuccess ? DG_OK : DG_ELAUNCH;
}

}  // extern "C"
