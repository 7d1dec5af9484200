// Host side of the DG volume derivative library for gfx950 (MI355X): launches and the C ABI.
//
// Forward:  out_b[i] = sum_a G[3a+b] (D_a u)[i]   for every (element, field) column.
// Adjoint:  gu = sum_a D_a^T W_a with W_a = sum_b G[3a+b] gout_b;
//           gG[3a+b] = sum_{f,i} gout_b[i] (D_a u)[i].
// Definitions, layouts and error behaviour are documented in include/dgvol.h;
// the forward data-movement schemes in dgvol_forward.hpp (FP64) and
// dgvol_forward_f32s.hpp (split-BF16), the adjoint in
// dgvol_adjoint.hpp, the D cotangent in dgvol_gradd.hpp, the register layout
// of the products in dgvol_layout.hpp, the entry kernels in dgvol_global.hpp,
// the calibration kernels in dgvol_calibrate.hpp.
// This file holds the host side: launch configuration, validation, the ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <mutex>

#include "dgvol.h"
#include "dgvol_adjoint.hpp"
#include "dgvol_adjoint_cr.hpp"
#include "dgvol_calibrate.hpp"
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
// size) for a launch of `block` threads with `dyn_lds` bytes of dynamic LDS
// (dyn_lds < 0: the kernel has static LDS only).  A kernel with dynamic LDS
// gets its limit raised to the full 160 KiB before its first query on a
// device.  Counts are cached per (device, kernel address, block size, LDS
// bytes) in a small table, so every kernel instance has entries of its own
// and the occupancy of one instance never sets the grid of another.
struct OccEntry {
  int dev;
  const void* fn;
  int block;
  int lds;
  int total;
};
constexpr int OCC_SLOTS = 1024;
static std::mutex occ_mutex;
static OccEntry occ_table[OCC_SLOTS];
static int occ_used = 0;

static int resident_blocks_fn(const void* fn, int block, int dyn_lds, int* err) {
  const int dev = current_device(err);
  if (dev < 0) return 0;
  bool attr_set = false;
  {
    std::lock_guard<std::mutex> lock(occ_mutex);
    for (int i = 0; i < occ_used; ++i) {
      const OccEntry& e = occ_table[i];
      if (e.dev != dev || e.fn != fn) continue;
      attr_set = true;
      if (e.block == block && e.lds == dyn_lds) return e.total;
    }
  }
  const int cus = cu_count(dev, err);
  if (*err != DG_OK) return 0;
  if (dyn_lds >= 0 && !attr_set) {
    // a failure here surfaces as a launch error of a kernel asking for more than the default limit
    (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  }
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, block, dyn_lds < 0 ? 0 : dyn_lds) != hipSuccess ||
      per_cu <= 0)
    per_cu = 1;
  const int total = cus * per_cu;
  std::lock_guard<std::mutex> lock(occ_mutex);
  if (occ_used < OCC_SLOTS) occ_table[occ_used++] = OccEntry{dev, fn, block, dyn_lds, total};
  return total;
}

template <typename Kern>
static int resident_blocks(Kern kernel, int block, int dyn_lds, int* err) {
  return resident_blocks_fn(reinterpret_cast<const void*>(kernel), block, dyn_lds, err);
}

static inline uint32_t ceil_div(uint64_t a, uint64_t b) { return (uint32_t)((a + b - 1) / b); }

// ------------------------------------------------------------------ forward variants

// One compiled variant of the forward product (dgvol_variants.hpp).
struct VariantDesc {
  const void* fn;  // its single-group kernel
  int body;
  int wpb;
  int tiles;
  int cls;
  int lds;
};

static bool variant_desc(int form, int Np, int v, VariantDesc* d) {
#define DGVOL_VDESC64(NP, IDX, BODY, WPB, TILES, CLS)                                                   \
  case vkey(NP, IDX):                                                                                   \
    *d = VariantDesc{reinterpret_cast<const void*>(fwd_f64_kernel<NP, BODY, WPB, TILES>), BODY, WPB, TILES, \
                     CLS, f64_lds<NP, BODY, WPB, TILES>()};                                             \
    return true;
#define DGVOL_VDESC32(NP, IDX, BODY, WPB, TILES, CLS)                                                    \
  case vkey(NP, IDX):                                                                                    \
    *d = VariantDesc{reinterpret_cast<const void*>(fwd_f32s_kernel<NP, BODY, WPB, TILES>), BODY, WPB, TILES, \
                     CLS, f32s_lds<NP, BODY, WPB, TILES>()};                                             \
    return true;
  if (v < 0 || v >= 16) return false;
  if (form == DG_FORM_F64) {
    switch (vkey(Np, v)) { DGVOL_F64_VARIANTS(DGVOL_VDESC64) default: return false; }
  }
  if (form == DG_FORM_F32S) {
    switch (vkey(Np, v)) { DGVOL_F32S_VARIANTS(DGVOL_VDESC32) default: return false; }
  }
  return false;
#undef DGVOL_VDESC64
#undef DGVOL_VDESC32
}

static int variant_count(int form, int Np) {
  int c = 0;
#define DGVOL_VCOUNT(NP, IDX, BODY, WPB, TILES, CLS) \
  if (NP == Np) ++c;
  if (form == DG_FORM_F64) { DGVOL_F64_VARIANTS(DGVOL_VCOUNT) }
  if (form == DG_FORM_F32S) { DGVOL_F32S_VARIANTS(DGVOL_VCOUNT) }
#undef DGVOL_VCOUNT
  return c;
}

// 16-column tiles one workgroup takes per loop iteration, and the loop's
// workers (waves of the staged body, workgroups of the chunk-register body).
static inline uint32_t units_per_step(const VariantDesc& d) {
  return d.body != BODY_CHUNKREG ? (uint32_t)(d.wpb * d.tiles) : (uint32_t)d.tiles;
}
static inline uint32_t workers_per_block(const VariantDesc& d) {
  return d.body != BODY_CHUNKREG ? (uint32_t)d.wpb : 1u;
}

// The batched kernel of a launch class.
static const void* batched_fn(int form, int cls) {
  if (form == DG_FORM_F64) {
    switch (cls) {
      case VCLASS_LIGHT: return reinterpret_cast<const void*>(batched_f64_kernel<VCLASS_LIGHT>);
      case VCLASS_HEAVY: return reinterpret_cast<const void*>(batched_f64_kernel<VCLASS_HEAVY>);
      case VCLASS_WAVE4: return reinterpret_cast<const void*>(batched_f64_kernel<VCLASS_WAVE4>);
      default: return reinterpret_cast<const void*>(batched_f64_kernel<LCLASS_ALL8>);
    }
  }
  switch (cls) {
    case VCLASS_LIGHT: return reinterpret_cast<const void*>(batched_f32s_kernel<VCLASS_LIGHT>);
    case VCLASS_HEAVY: return reinterpret_cast<const void*>(batched_f32s_kernel<VCLASS_HEAVY>);
    case VCLASS_WAVE4: return reinterpret_cast<const void*>(batched_f32s_kernel<VCLASS_WAVE4>);
    default: return reinterpret_cast<const void*>(batched_f32s_kernel<LCLASS_ALL8>);
  }
}

// The launch class a group of variant d runs in: its variant class when the
// batch asks for one launch per class, else ALL8 for every 8-wave variant.
static inline int launch_class(const VariantDesc& d, bool by_class) {
  if (by_class) return d.cls;
  return d.wpb == 8 ? LCLASS_ALL8 : VCLASS_WAVE4;
}

// Persistent grid of a single-group launch of variant d over `ntiles` tiles.
static uint32_t single_grid(const VariantDesc& d, uint32_t ntiles, int* err, uint32_t* resident) {
  const int cap = resident_blocks_fn(d.fn, WAVE * d.wpb, d.lds, err);
  if (*err != DG_OK) return 0;
  if (resident) *resident = (uint32_t)cap;
  return std::min<uint32_t>(ceil_div(ntiles, units_per_step(d)), (uint32_t)cap);
}

template <typename T>
static dg_status launch_variant(const VariantDesc& d, const FwdArgs<T>& p, hipStream_t stream) {
  int err = DG_OK;
  const uint32_t grid = single_grid(d, p.ntiles, &err, nullptr);
  if (err != DG_OK) return err;
  FwdArgs<T> a = p;
  void* args[] = {&a};
  if (hipLaunchKernel(d.fn, dim3(grid), dim3(WAVE * d.wpb), args, (size_t)d.lds, stream) != hipSuccess)
    return DG_ELAUNCH;
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
    case 84: eff = form == DG_FORM_F64 ? 0.54 : 0.70; break;
    default: eff = form == DG_FORM_F64 ? 0.60 : 0.55; break;  // Np = 120
  }
  return std::max(bytes / bw, flops / peak) / eff;
}

// Kernels and grids of the adjoint for (NP, K, F): one staged kernel (runs of
// whole elements per wave, any F) below Np = 84, two chunk-register passes
// (gu, then gG) from Np = 84.
struct AdjPlan {
  int nk;                // kernels launched
  const void* fn[2];
  uint32_t block[2];     // threads per workgroup of each kernel
  uint32_t grid[2];
  uint32_t resident[2];
  uint32_t units[2];     // work units of each kernel
  uint32_t workers[2];   // loop workers per workgroup (waves, or the workgroup itself)
  uint32_t min_it[2];    // loop iterations of the least and the most loaded worker
  uint32_t max_it[2];
};

template <int NP>
static dg_status adj_plan(int64_t K, int32_t F, AdjPlan* pl) {
  int err = DG_OK;
  if constexpr (NP >= 84) {
    const uint32_t tiles_a = ceil_div((uint64_t)K * (uint64_t)F, 16);
    pl->nk = 2;
    pl->block[0] = WAVE * ADJCR_WPB;
    pl->block[1] = AdjCrB<NP>::NTH;
    pl->fn[0] = reinterpret_cast<const void*>(adjcr_gu_kernel<NP>);
    pl->fn[1] = reinterpret_cast<const void*>(adjcr_gG_kernel<NP>);
    pl->units[0] = tiles_a;
    pl->units[1] = tiles_a;  // the gG pass: runs of whole elements per workgroup, in 16-column tiles
    for (int i = 0; i < 2; ++i) {
      const int cap = resident_blocks_fn(pl->fn[i], pl->block[i], -1, &err);
      if (err != DG_OK) return err;
      pl->resident[i] = (uint32_t)cap;
      pl->grid[i] = std::min<uint32_t>(pl->units[i], (uint32_t)cap);
      pl->workers[i] = 1;
      pl->min_it[i] = pl->units[i] / pl->grid[i];
      pl->max_it[i] = ceil_div(pl->units[i], pl->grid[i]);
    }
    const uint64_t nw = pl->grid[1];
    pl->min_it[1] = (uint32_t)ceil_div((uint64_t)(K / nw) * (uint64_t)F, 16);
    pl->max_it[1] = (uint32_t)ceil_div(ceil_div((uint64_t)K, nw) * (uint64_t)F, 16);
  } else {
    pl->nk = 1;
    pl->block[0] = pl->block[1] = WAVE * ADJ_WPB;
    pl->fn[0] = reinterpret_cast<const void*>(adj_f64_staged_kernel<NP, ADJ_WPB>);
    const int cap = resident_blocks_fn(pl->fn[0], pl->block[0], -1, &err);
    if (err != DG_OK) return err;
    pl->resident[0] = (uint32_t)cap;
    pl->workers[0] = ADJ_WPB;
    // runs of whole elements per wave, taken as 16-column tiles
    const uint32_t tiles = ceil_div((uint64_t)K * (uint64_t)F, 16);
    pl->units[0] = tiles;
    pl->grid[0] = std::min<uint32_t>(ceil_div(tiles, ADJ_WPB), (uint32_t)cap);
    const uint64_t nw = (uint64_t)pl->grid[0] * ADJ_WPB;
    pl->min_it[0] = (uint32_t)ceil_div((uint64_t)(K / nw) * (uint64_t)F, 16);
    pl->max_it[0] = (uint32_t)ceil_div(ceil_div((uint64_t)K, nw) * (uint64_t)F, 16);
  }
  return DG_OK;
}

template <int NP>
static dg_status launch_adj_f64(const double* D, const double* G, const double* u, const double* gout,
                                double* gu, double* gG, int64_t K, int32_t F, hipStream_t stream) {
  AdjPlan pl;
  const dg_status st = adj_plan<NP>(K, F, &pl);
  if (st != DG_OK) return st;
  if constexpr (NP >= 84) {
    // two chunk-register passes: gu, then gG
    const uint64_t ncols = (uint64_t)K * (uint64_t)F;
    hipLaunchKernelGGL(adjcr_gu_kernel<NP>, dim3(pl.grid[0]), dim3(pl.block[0]), 0, stream, D, G, gout, gu,
                       (uint32_t)ncols, (uint32_t)F, (int64_t)ncols * NP, pl.units[0]);
    hipLaunchKernelGGL(adjcr_gG_kernel<NP>, dim3(pl.grid[1]), dim3(pl.block[1]), 0, stream, D, u, gout, gG, (uint32_t)K,
                       (uint32_t)F, (int64_t)ncols * NP);
  } else {
    hipLaunchKernelGGL((adj_f64_staged_kernel<NP, ADJ_WPB>), dim3(pl.grid[0]), dim3(pl.block[0]), 0, stream, D, G, u,
                       gout, gu, gG, (uint32_t)K, (uint32_t)F, (int64_t)K * F * NP);
  }
  return hipGetLastError() == hipSuccess ? DG_OK : DG_ELAUNCH;
}

// Partial sums of the D cotangent: a pure function of the problem size, so
// the result does not depend on the device.
static uint32_t gd_parts(int64_t K, int32_t Np, int32_t F) {
  const uint32_t nunits = ceil_div((uint64_t)K * (uint64_t)F, GD_UNIT);
  return std::min<uint32_t>(nunits, gd_maxpart(Np));
}

// Partial sums of the D cotangent into work[npart][3][Np][Np], then their
// fixed-order sum into gD.
template <int NP>
static dg_status launch_gd_f64(const double* G, const double* u, const double* gout, double* gD, double* work,
                               uint32_t npart, int64_t K, int32_t F, hipStream_t stream) {
  using S = GdShape<NP>;
  const uint64_t ncols = (uint64_t)K * (uint64_t)F;
  if (npart > 0) {
    const GdArgs p{G, u, gout, work, (uint32_t)ncols, (uint32_t)F, (int64_t)ncols * NP, ceil_div(ncols, GD_UNIT),
                   npart};
    if constexpr (NP == 56) {
      hipLaunchKernelGGL(gd_split56_kernel, dim3(npart), dim3(GdSplit56::NTH), 0, stream, p);
    } else {
      // with NSPLIT > 1 the grid is rounded up to whole groups of 8 ranges (one per XCD)
      const uint32_t grid = S::NSPLIT == 1 ? npart : ceil_div(npart, 8) * 8 * S::NSPLIT;
      hipLaunchKernelGGL(gd_partial_kernel<NP>, dim3(grid), dim3(S::NTH), 0, stream, p);
    }
  }
  const uint32_t n = 3u * NP * NP;
  hipLaunchKernelGGL(gd_reduce_kernel, dim3(ceil_div(n, 64)), dim3(64 * GD_RED_PG), 0, stream, work, gD, npart,
                     n);
  return hipGetLastError() == hipSuccess ? DG_OK : DG_ELAUNCH;
}

// ------------------------------------------------------------------ fixed scratch (dg_volume_grad_d_noalloc)

// The partial sums of the D cotangent for callers that cannot allocate.  Each
// device the library runs on holds its own copy until the process ends.  In
// host code `scratch` names a host-side stand-in, not device memory: kernels
// and copies get the device address that scratch_device_ptr() looks up once
// per device, never the symbol itself.
static __device__ __align__(256) double scratch[DG_GRAD_D_NOALLOC_SCRATCH_BYTES / sizeof(double)];
static std::mutex scratch_mutex;
static double* scratch_dev[MAX_DEVICES];

// Device address of `scratch` on the current device (looked up on the first
// call per device; the lookup allocates nothing).
static double* scratch_device_ptr(int* err) {
  const int dev = current_device(err);
  if (dev < 0) return nullptr;
  if (dev >= MAX_DEVICES) {
    *err = DG_EDEVICE;
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(scratch_mutex);
  if (!scratch_dev[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
      *err = DG_EDEVICE;
      return nullptr;
    }
    scratch_dev[dev] = static_cast<double*>(ptr);
  }
  return scratch_dev[dev];
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
    case DG_ESCRATCH:
      return "the problem needs more scratch than the fixed no-allocation buffer holds "
             "(DG_GRAD_D_NOALLOC_SCRATCH_BYTES); call dg_volume_grad_d with a workspace";
    default: return "unknown status";
  }
}

int32_t dg_supported_np(int32_t Np) {
  switch (Np) {
    case 4: case 10: case 20: case 35: case 56: case 84: case 120: return 1;
    default: return 0;
  }
}

int32_t dg_variant_count(int32_t form, int32_t Np) {
  if (!dg_supported_np(Np)) return 0;
  return variant_count(form, Np);
}

dg_status dg_variant_query(int32_t form, int32_t Np, int32_t variant, dg_variant_info* info) {
  if (!info) return DG_EINVAL;
  VariantDesc d;
  if (!dg_supported_np(Np) || !variant_desc(form, Np, variant, &d)) return DG_EUNSUPPORTED;
  *info = dg_variant_info{d.body, d.wpb, d.tiles, d.cls, d.lds};
  return DG_OK;
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

dg_status dg_volume_variant(int32_t form, int32_t variant, const void* D, const void* G, const void* u, void* out,
                            int64_t K, int32_t Np, int32_t F, void* stream) {
  bool noop = false;
  const dg_status st = check_common(K, Np, F, &noop);
  if (st != DG_OK) return st;
  if (form != DG_FORM_F64 && form != DG_FORM_F32S) return DG_EUNSUPPORTED;
  VariantDesc d;
  if (!variant_desc(form, Np, variant == DG_VARIANT_AUTO ? 0 : variant, &d)) return DG_EUNSUPPORTED;
  if (noop) return DG_OK;
  const uintptr_t word = form == DG_FORM_F64 ? 8 : 4;
  if (!D || !G || !u || !out) return DG_EINVAL;
  if (!aligned(D, word) || !aligned(G, word) || !aligned(u, word) || !aligned(out, word)) return DG_EINVAL;
  const uint64_t ncols = (uint64_t)K * (uint64_t)F;
  if (form == DG_FORM_F64) {
    const FwdArgs<double> p{static_cast<const double*>(D), static_cast<const double*>(G),
                            static_cast<const double*>(u), static_cast<double*>(out), (uint32_t)ncols, (uint32_t)F,
                            (int64_t)ncols * Np, ceil_div(ncols, 16)};
    return launch_variant(d, p, (hipStream_t)stream);
  }
  const FwdArgs<float> p{static_cast<const float*>(D), static_cast<const float*>(G), static_cast<const float*>(u),
                         static_cast<float*>(out), (uint32_t)ncols, (uint32_t)F, (int64_t)ncols * Np,
                         ceil_div(ncols, 16)};
  return launch_variant(d, p, (hipStream_t)stream);
}

dg_status dg_volume(const double* D, const double* G, const double* u, double* out, int64_t K, int32_t Np,
                    int32_t F, void* stream) {
  return dg_volume_variant(DG_FORM_F64, DG_VARIANT_AUTO, D, G, u, out, K, Np, F, stream);
}

dg_status dg_volume_f32s(const float* D, const float* G, const float* u, float* out, int64_t K, int32_t Np,
                         int32_t F, void* stream) {
  return dg_volume_variant(DG_FORM_F32S, DG_VARIANT_AUTO, D, G, u, out, K, Np, F, stream);
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
  DGVOL_DISPATCH(launch_gd_f64, G, u, gout, gD, static_cast<double*>(work), gd_parts(K, Np, F), K, F,
                 (hipStream_t)stream)
}

dg_status dg_volume_grad_d_noalloc(const double* G, const double* u, const double* gout, double* gD, int64_t K,
                                   int32_t Np, int32_t F, void* stream) {
  bool noop = false;
  const dg_status st = check_common(K, Np, F, &noop);
  if (st != DG_OK) return st;
  if (!gD || !aligned(gD, 8)) return DG_EINVAL;
  if (!noop) {
    if (!G || !u || !gout) return DG_EINVAL;
    if (!aligned(G, 8) || !aligned(u, 8) || !aligned(gout, 8)) return DG_EINVAL;
  }
  uint64_t need = 0;
  dg_volume_grad_d_workspace(K, Np, F, &need);
  if (need > DG_GRAD_D_NOALLOC_SCRATCH_BYTES) return DG_ESCRATCH;
  int err = DG_OK;
  double* work = scratch_device_ptr(&err);
  if (err != DG_OK) return err;
  DGVOL_DISPATCH(launch_gd_f64, G, u, gout, gD, work, gd_parts(K, Np, F), K, F, (hipStream_t)stream)
}

#undef DGVOL_DISPATCH

dg_status dg_volume_batched(const dg_group* groups, int32_t ngroups, int32_t F, int32_t form_flags,
                            void* stream) {
  if (ngroups < 0 || ngroups > DG_MAX_GROUPS || F < 1) return DG_EINVAL;
  if (form_flags & ~(0xff | DG_BATCH_BY_CLASS)) return DG_EUNSUPPORTED;
  const bool by_class = (form_flags & DG_BATCH_BY_CLASS) != 0;
  const int32_t form = form_flags & 0xff;
  if (form != DG_FORM_F64 && form != DG_FORM_F32S) return DG_EUNSUPPORTED;
  if (ngroups > 0 && !groups) return DG_EINVAL;
  const uintptr_t word = form == DG_FORM_F64 ? 8 : 4;
  // validate everything first (nothing is launched on error), then one launch per class
  VariantDesc desc[DG_MAX_GROUPS];
  bool live[DG_MAX_GROUPS];
  for (int i = 0; i < ngroups; ++i) {
    const dg_group& gr = groups[i];
    bool noop = false;
    const dg_status st = check_common(gr.K, gr.Np, F, &noop);
    if (st != DG_OK) return st;
    if (!variant_desc(form, gr.Np, gr.variant == DG_VARIANT_AUTO ? 0 : gr.variant, &desc[i]))
      return DG_EUNSUPPORTED;
    live[i] = !noop;
    if (noop) continue;
    if (!gr.D || !gr.G || !gr.u || !gr.out) return DG_EINVAL;
    if (!aligned(gr.D, word) || !aligned(gr.G, word) || !aligned(gr.u, word) || !aligned(gr.out, word))
      return DG_EINVAL;
  }
  for (int cls = 0; cls < NUM_LCLASSES; ++cls) {
    BatchArgs a{};
    a.F = (uint32_t)F;
    double step_cost[DG_MAX_GROUPS];  // estimated cost of one loop step of one workgroup
    uint32_t steps[DG_MAX_GROUPS];    // loop steps of the group (units over units per step)
    uint32_t max_blocks[DG_MAX_GROUPS];
    int lds = 0;
    int ng = 0;
    for (int i = 0; i < ngroups; ++i) {
      if (!live[i] || launch_class(desc[i], by_class) != cls) continue;
      const dg_group& gr = groups[i];
      const uint64_t ncols = (uint64_t)gr.K * (uint64_t)F;
      GroupDev& gd = a.g[ng];
      gd.Np = gr.Np;
      gd.variant = gr.variant == DG_VARIANT_AUTO ? 0 : gr.variant;
      gd.ncols = (uint32_t)ncols;
      gd.ntiles = ceil_div(ncols, 16);
      gd.plane = (int64_t)ncols * gr.Np;
      gd.D = gr.D;
      gd.G = gr.G;
      gd.u = gr.u;
      gd.out = gr.out;
      const double per_tile = gr.cost > 0.0 ? gr.cost : tile_cost_estimate(form, gr.Np, (uint32_t)F);
      step_cost[ng] = per_tile * units_per_step(desc[i]);
      steps[ng] = ceil_div(gd.ntiles, units_per_step(desc[i]));
      max_blocks[ng] = steps[ng];
      lds = std::max(lds, desc[i].lds);
      ++ng;
    }
    if (ng == 0) continue;
    a.ngroups = ng;
    int err = DG_OK;
    const void* fn = batched_fn(form, cls);
    const int block = WAVE * class_waves(cls);
    const int cap = resident_blocks_fn(fn, block, lds, &err);
    if (err != DG_OK) return err;
    // Split the resident workgroups so that the largest load of a workgroup is as
    // small as possible: every group starts with one workgroup, and each further
    // one goes to the group whose workgroups carry the largest load, at most as
    // many as the group has loop steps.  A workgroup's load is its loop steps
    // (the group's steps over its workgroups, rounded up) times the cost of a
    // step.  Giving each group the whole part of its proportional share first
    // had used up the workgroups on the floors and the groups bumped to one,
    // and left a small group (order 6 of the mixed batch) one workgroup short:
    // it then finished last.
    uint32_t nb[DG_MAX_GROUPS];
    uint32_t used = 0;
    for (int i = 0; i < ng; ++i) {
      nb[i] = 1;
      ++used;
    }
    auto load = [&](int i) { return step_cost[i] * (double)ceil_div(steps[i], nb[i]); };
    while (used < (uint32_t)cap) {
      int pick = -1;
      for (int i = 0; i < ng; ++i)
        if (nb[i] < max_blocks[i] && (pick < 0 || load(i) > load(pick))) pick = i;
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
    void* args[] = {&a};
    if (hipLaunchKernel(fn, dim3(begin), dim3(block), args, (size_t)lds, (hipStream_t)stream) != hipSuccess)
      return DG_ELAUNCH;
    if (hipGetLastError() != hipSuccess) return DG_ELAUNCH;
  }
  return DG_OK;
}

dg_status dg_launch_shape_query(int32_t op, int32_t form, int32_t Np, int32_t variant, int64_t K, int32_t F,
                                dg_launch_shape* shape) {
  if (!shape || K < 1 || F < 1) return DG_EINVAL;
  if (!dg_supported_np(Np)) return DG_EUNSUPPORTED;
  if ((uint64_t)K * (uint64_t)F > (uint64_t)INT32_MAX) return DG_EINVAL;
  int err = DG_OK;
  dg_launch_shape sh{};
  if (op == DG_OP_FORWARD || op == DG_OP_BATCHED || op == DG_OP_BATCHED_BY_CLASS) {
    VariantDesc d;
    if (!variant_desc(form, Np, variant == DG_VARIANT_AUTO ? 0 : variant, &d)) return DG_EUNSUPPORTED;
    const uint32_t ntiles = ceil_div((uint64_t)K * (uint64_t)F, 16);
    const uint32_t per = units_per_step(d);
    uint32_t cap = 0;
    if (op == DG_OP_FORWARD) {
      cap = (uint32_t)resident_blocks_fn(d.fn, WAVE * d.wpb, d.lds, &err);
      sh.block = WAVE * d.wpb;
    } else {
      const int lc = launch_class(d, op == DG_OP_BATCHED_BY_CLASS);
      sh.block = WAVE * class_waves(lc);
      cap = (uint32_t)resident_blocks_fn(batched_fn(form, lc), sh.block, d.lds, &err);
    }
    if (err != DG_OK) return err;
    sh.grid = std::min<uint32_t>(ceil_div(ntiles, per), cap);
    sh.lds_bytes = (uint32_t)d.lds;
    sh.resident = cap;
    sh.units = ntiles;
    sh.units_per_step = per;
    // the loop hands out runs of `tiles` tiles to grid x workers workers in turn
    const uint32_t runs = ceil_div(ntiles, (uint32_t)d.tiles);
    const uint32_t workers = sh.grid * workers_per_block(d);
    sh.min_iters = runs / workers;
    sh.max_iters = ceil_div(runs, workers);
  } else if (op == DG_OP_ADJOINT) {
    if (form != DG_FORM_F64) return DG_EUNSUPPORTED;
    AdjPlan pl;
    dg_status st = DG_EUNSUPPORTED;
    switch (Np) {
      case 4: st = adj_plan<4>(K, F, &pl); break;
      case 10: st = adj_plan<10>(K, F, &pl); break;
      case 20: st = adj_plan<20>(K, F, &pl); break;
      case 35: st = adj_plan<35>(K, F, &pl); break;
      case 56: st = adj_plan<56>(K, F, &pl); break;
      case 84: st = adj_plan<84>(K, F, &pl); break;
      case 120: st = adj_plan<120>(K, F, &pl); break;
    }
    if (st != DG_OK) return st;
    sh.grid = pl.grid[0];
    sh.block = pl.block[0];
    sh.lds_bytes = 0;
    sh.resident = pl.resident[0];
    sh.units = pl.units[0];
    sh.units_per_step = pl.workers[0];
    sh.min_iters = UINT32_MAX;
    sh.max_iters = 0;
    for (int i = 0; i < pl.nk; ++i) {
      sh.min_iters = std::min(sh.min_iters, pl.min_it[i]);
      sh.max_iters = std::max(sh.max_iters, pl.max_it[i]);
    }
  } else {
    return DG_EINVAL;
  }
  *shape = sh;
  return DG_OK;
}

dg_status dg_stream_calibrate(const double* src, double* dst, int64_t n, int32_t copies, void* stream) {
  if (n < 0 || copies < 1 || copies > 3) return DG_EINVAL;
  if (n == 0) return DG_OK;
  if (!src || !dst || !aligned(src, 8) || !aligned(dst, 8)) return DG_EINVAL;
  if (aligned(src, 16) && aligned(dst, 16) && n % 2 == 0) {
    const int64_t n2 = n / 2;
    const int64_t per_block = (int64_t)STREAM_BLOCK * STREAM_U;
    const int64_t grid = (n2 + per_block - 1) / per_block;
    if (grid > INT32_MAX) return DG_EINVAL;
    hipLaunchKernelGGL(stream16_kernel, dim3((uint32_t)grid), dim3(STREAM_BLOCK), 0, (hipStream_t)stream,
                       reinterpret_cast<const f64x2*>(src), reinterpret_cast<f64x2*>(dst), n2, copies);
    return hipGetLastError() == hipSuccess ? DG_OK : DG_ELAUNCH;
  }
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

dg_status dg_stream_calibrate_tiles(const double* src, double* dst, int64_t ntiles, int32_t tiles_per_wave,
                                    void* stream) {
  if (ntiles < 0 || ntiles > INT32_MAX / TSTREAM_TILE || tiles_per_wave < 0) return DG_EINVAL;
  if (ntiles == 0) return DG_OK;
  if (!src || !dst || !aligned(src, 8) || !aligned(dst, 8)) return DG_EINVAL;
  // dynamic LDS: the waves' tile buffers, or (persistent form) enough to hold one
  // workgroup per CU, as the order-4 forward kernel's registers do
  const int need = TSTREAM_WPB * TSTREAM_TILE * 8;
  const int lds = tiles_per_wave == 0 ? 100 * 1024 : need;
  const uint64_t waves_needed = (uint64_t)ntiles;
  uint32_t grid, iters;
  if (tiles_per_wave == 0) {
    int cerr = DG_OK;
    const int dev = current_device(&cerr);
    if (dev < 0) return cerr;
    const int cus = cu_count(dev, &cerr);
    if (cerr != DG_OK) return cerr;
    grid = (uint32_t)std::min<uint64_t>((uint64_t)cus, ceil_div(waves_needed, TSTREAM_WPB));
  } else {
    grid = ceil_div(waves_needed, (uint64_t)TSTREAM_WPB * (uint64_t)tiles_per_wave);
  }
  iters = ceil_div((uint64_t)ntiles, (uint64_t)grid * TSTREAM_WPB);
  // raises the kernel's dynamic-LDS limit on this device (once per device)
  int err = DG_OK;
  (void)resident_blocks_fn(reinterpret_cast<const void*>(tile_stream_kernel), WAVE * TSTREAM_WPB, lds, &err);
  if (err != DG_OK) return err;
  hipLaunchKernelGGL(tile_stream_kernel, dim3(grid), dim3(WAVE * TSTREAM_WPB), (size_t)lds, (hipStream_t)stream, src,
                     dst, (uint32_t)ntiles, (int64_t)ntiles * TSTREAM_TILE, iters);
  return hipGetLastError() == hipSuccess ? DG_OK : DG_ELAUNCH;
}

dg_status dg_mfma_calibrate(double* sink, int32_t iters, void* stream) {
  if (!sink || !aligned(sink, 8) || iters < 1) return DG_EINVAL;
  hipLaunchKernelGGL(mfma_cal_kernel, dim3(DG_MFMA_CAL_BLOCKS), dim3(256), 0, (hipStream_t)stream, sink, iters);
  return hipGetLastError() == hipSuccess ? DG_OK : DG_ELAUNCH;
}

dg_status dg_mfma_calibrate_beside(double* sink, int32_t iters, int32_t viters, int32_t mode, void* stream) {
  if (!sink || !aligned(sink, 8) || iters < 0 || viters < 0 || iters + (int64_t)viters < 1) return DG_EINVAL;
  const dim3 grid(DG_MFMA_BESIDE_BLOCKS), block(512);
  const hipStream_t s = (hipStream_t)stream;
  switch (mode) {
    case DG_BESIDE_NONE: hipLaunchKernelGGL(mfma_beside_kernel<0>, grid, block, 0, s, sink, iters, viters); break;
    case DG_BESIDE_FP64_FMA: hipLaunchKernelGGL(mfma_beside_kernel<1>, grid, block, 0, s, sink, iters, viters); break;
    case DG_BESIDE_INT: hipLaunchKernelGGL(mfma_beside_kernel<2>, grid, block, 0, s, sink, iters, viters); break;
    case DG_BESIDE_DPP: hipLaunchKernelGGL(mfma_beside_kernel<3>, grid, block, 0, s, sink, iters, viters); break;
    default: return DG_EINVAL;
  }
  return hipGetLastError() == hipSuccess ? DG_OK : DG_ELAUNCH;
}

}  // extern "C"
