// HIP kernels of the DG volume derivative for gfx950 (MI355X) and the C ABI.
//
// Forward:  out_b[i] = sum_a G[3a+b] (D_a u)[i]   for every (element, field) column.
// Adjoint:  gu = sum_a D_a^T W_a with W_a = sum_b G[3a+b] gout_b;
//           gG[3a+b] = sum_{f,i} gout_b[i] (D_a u)[i].
// Definitions, layouts and error behaviour are documented in include/dgvol.h.
//
// Design (one wave = 16 columns, persistent grid):
//  * D is staged once per workgroup in LDS, already permuted into the
//    per-lane MFMA A-operand order (one conflict-free 8-byte read per lane per
//    MFMA), when the table fits; otherwise A operands are gathered from D in
//    global memory (L2-resident).  This is the "precompute into on-chip storage
//    of a repeatedly fetched operand" of the paper's Section on substitution
//    rules for precomputation, done by hand.
//  * u is read once from HBM straight into B-operand registers.
//  * The stacked product [3Np x Np] . [Np x 16] runs on the FP64 matrix cores
//    (v_mfma_f64_16x16x4_f64), k = node, in chunks of 3 output tiles.
//  * The row permutation of dgvol_layout.hpp leaves (D_r u, D_s u, D_t u) of
//    one node in one lane, so the geometric-factor combine is fused into the
//    epilogue with no data exchange, and out is written once.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdint>

#include "dgvol.h"
#include "dgvol_layout.hpp"

namespace dgvol {

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int WAVE = 64;

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

// Tables up to this size are staged in LDS; larger D is read from global memory.
constexpr int LDS_TABLE_LIMIT = 96 * 1024;

template <int NP>
constexpr bool fwd_table_in_lds() { return fwd_table_doubles<NP>() * 8 <= LDS_TABLE_LIMIT; }

template <int NP>
constexpr bool adj_d_in_lds() { return 3 * NP * NP * 8 <= LDS_TABLE_LIMIT; }

// ------------------------------------------------------------------ forward FP64

template <int NP, int WPB>
__global__ __launch_bounds__(WAVE* WPB) void fwd_f64_kernel(
    const double* __restrict__ D, const double* __restrict__ G, const double* __restrict__ u,
    double* __restrict__ out, uint32_t ncols, uint32_t F, int64_t plane, uint32_t ntiles) {
  using Sh = Shape<NP>;
  constexpr bool ALDS = fwd_table_in_lds<NP>();
  constexpr int NFRAG = ALDS ? fwd_table_doubles<NP>() : 1;
  __shared__ double afr[NFRAG];
  const int lane = threadIdx.x & 63;
  if constexpr (ALDS) {
    for (int e = threadIdx.x; e < NFRAG; e += WAVE * WPB) {
      const int ts = e >> 6;
      afr[e] = afrag_f64<NP>(D, ts / Sh::KS64, ts % Sh::KS64, e & 63);
    }
    __syncthreads();
  }
  const int n = lane & 15, g = lane >> 4;
  const uint32_t wave = threadIdx.x >> 6;
  for (uint32_t t = blockIdx.x * WPB + wave; t < ntiles; t += gridDim.x * WPB) {
    const uint32_t col = t * 16 + n;
    const bool valid = col < ncols;
    const double* __restrict__ uc = u + (int64_t)col * NP;
    double b[Sh::KS64];
#pragma unroll
    for (int s = 0; s < Sh::KS64; ++s) {
      const int j = 4 * s + g;
      b[s] = (valid && j < NP) ? uc[j] : 0.0;
    }
    const uint32_t k = valid ? col / F : 0u;
    double gk[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) gk[c] = valid ? G[(int64_t)k * 9 + c] : 0.0;
    double* __restrict__ oc = out + (int64_t)col * NP;
#pragma unroll
    for (int ch = 0; ch < Sh::NCHUNK; ++ch) {
      f64x4 acc[3];
#pragma unroll
      for (int tt = 0; tt < 3; ++tt) acc[tt] = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int s = 0; s < Sh::KS64; ++s) {
#pragma unroll
        for (int tt = 0; tt < 3; ++tt) {
          const int T = 3 * ch + tt;
          if (T < Sh::MT) {
            double a;
            if constexpr (ALDS)
              a = afr[(T * Sh::KS64 + s) * WAVE + lane];
            else
              a = afrag_f64<NP>(D, T, s, lane);
            acc[tt] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b[s], acc[tt], 0, 0, 0);
          }
        }
      }
#pragma unroll
      for (int tau = 4 * ch; tau < 4 * ch + 4; ++tau) {
        if (tau < Sh::TRIP) {
          double R[3];
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            const int loc = 3 * tau + a - 12 * ch;
            R[a] = acc[loc >> 2][loc & 3];
          }
          const int i = 4 * tau + g;
          if (valid && i < NP) {
#pragma unroll
            for (int bb = 0; bb < 3; ++bb)
              oc[bb * plane + i] = gk[bb] * R[0] + gk[3 + bb] * R[1] + gk[6 + bb] * R[2];
          }
        }
      }
    }
  }
}

// ------------------------------------------------------------------ adjoint FP64
//
// Tiles are whole elements: E = max(1, 16 / F) elements per tile, split into
// nsub sub-tiles of 16 columns (nsub > 1 only when F > 16), so the per-element
// gG sums need no cross-wave reduction.  Per sub-tile and chunk of 4 node
// triples: recompute R = D u (forward fragments), read gout at the lane's
// nodes, accumulate gG partials, form W = G^T gout lane-locally, then feed the
// 12 W slots straight in as the B operand of the transposed product D^T W
// (the slot order of W is the k order of that product), accumulated over chunks.

template <int NP, int WPB>
__global__ __launch_bounds__(WAVE* WPB) void adj_f64_kernel(
    const double* __restrict__ D, const double* __restrict__ G, const double* __restrict__ u,
    const double* __restrict__ gout, double* __restrict__ gu, double* __restrict__ gG,
    uint32_t K, uint32_t F, int64_t plane, uint32_t E, uint32_t nsub, uint32_t ntiles) {
  using Sh = Shape<NP>;
  constexpr bool DLDS = adj_d_in_lds<NP>();
  constexpr int ND = DLDS ? 3 * NP * NP : 1;
  __shared__ double Dl[ND];
  __shared__ double red[WPB][16][9];
  if constexpr (DLDS) {
    for (int e = threadIdx.x; e < ND; e += WAVE * WPB) Dl[e] = D[e];
    __syncthreads();
  }
  const double* __restrict__ Dsrc = DLDS ? Dl : D;
  const int lane = threadIdx.x & 63;
  const int n = lane & 15, g = lane >> 4;
  const uint32_t wave = threadIdx.x >> 6;
  for (uint32_t t = blockIdx.x * WPB + wave; t < ntiles; t += gridDim.x * WPB) {
    const uint32_t k0 = t * E;
    double P[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) P[c] = 0.0;
    for (uint32_t sub = 0; sub < nsub; ++sub) {
      const uint32_t lc = sub * 16 + n;
      const uint32_t e = (F <= 16) ? lc / F : 0u;
      const uint32_t f = (F <= 16) ? lc - e * F : lc;
      const uint32_t k = k0 + e;
      const bool valid = ((F <= 16) ? (lc < E * F) : (lc < F)) && (k < K);
      const uint32_t col = valid ? k * F + f : 0u;
      const double* __restrict__ uc = u + (int64_t)col * NP;
      double b[Sh::KS64];
#pragma unroll
      for (int s = 0; s < Sh::KS64; ++s) {
        const int j = 4 * s + g;
        b[s] = (valid && j < NP) ? uc[j] : 0.0;
      }
      double gk[9];
#pragma unroll
      for (int c = 0; c < 9; ++c) gk[c] = valid ? G[(int64_t)k * 9 + c] : 0.0;
      f64x4 accj[Sh::MTJ];
#pragma unroll
      for (int tj = 0; tj < Sh::MTJ; ++tj) accj[tj] = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int ch = 0; ch < Sh::NCHUNK; ++ch) {
        f64x4 acc[3];
#pragma unroll
        for (int tt = 0; tt < 3; ++tt) acc[tt] = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int s = 0; s < Sh::KS64; ++s) {
#pragma unroll
          for (int tt = 0; tt < 3; ++tt) {
            const int T = 3 * ch + tt;
            if (T < Sh::MT) {
              const double a = afrag_f64<NP>(Dsrc, T, s, lane);
              acc[tt] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b[s], acc[tt], 0, 0, 0);
            }
          }
        }
        double W[12];
#pragma unroll
        for (int x = 0; x < 12; ++x) W[x] = 0.0;
#pragma unroll
        for (int tau = 4 * ch; tau < 4 * ch + 4; ++tau) {
          if (tau < Sh::TRIP) {
            double R[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
              const int loc = 3 * tau + a - 12 * ch;
              R[a] = acc[loc >> 2][loc & 3];
            }
            const int i = 4 * tau + g;
            const bool inb = valid && i < NP;
            double go[3];
#pragma unroll
            for (int bb = 0; bb < 3; ++bb)
              go[bb] = inb ? gout[bb * plane + (int64_t)col * NP + i] : 0.0;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
#pragma unroll
              for (int bb = 0; bb < 3; ++bb) P[3 * a + bb] += go[bb] * R[a];
              W[3 * (tau - 4 * ch) + a] = gk[3 * a] * go[0] + gk[3 * a + 1] * go[1] + gk[3 * a + 2] * go[2];
            }
          }
        }
#pragma unroll
        for (int sl = 0; sl < 12; ++sl) {
          const int sp = 12 * ch + sl;
          if (sp < Sh::SLOTS) {
#pragma unroll
            for (int tj = 0; tj < Sh::MTJ; ++tj) {
              const double a = afragT_f64<NP>(Dsrc, tj, sp, lane);
              accj[tj] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, W[sl], accj[tj], 0, 0, 0);
            }
          }
        }
      }
      double* __restrict__ guc = gu + (int64_t)col * NP;
#pragma unroll
      for (int tj = 0; tj < Sh::MTJ; ++tj) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int j = 16 * tj + 4 * q + g;
          if (valid && j < NP) guc[j] = accj[tj][q];
        }
      }
    }
    // gG: sum the four lane groups (same column), then the columns of each element.
#pragma unroll
    for (int c = 0; c < 9; ++c) {
      P[c] += __shfl_xor(P[c], 16);
      P[c] += __shfl_xor(P[c], 32);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (g == 0) {
#pragma unroll
      for (int c = 0; c < 9; ++c) red[wave][n][c] = P[c];
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (g == 0 && (uint32_t)n < E && k0 + n < K) {
      const uint32_t lo = (F <= 16) ? n * F : 0u;
      const uint32_t hi = (F <= 16) ? lo + F : 16u;
      for (int c = 0; c < 9; ++c) {
        double s = 0.0;
        for (uint32_t m = lo; m < hi; ++m) s += red[wave][m][c];
        gG[(int64_t)(k0 + n) * 9 + c] = s;
      }
    }
  }
}

// ------------------------------------------------------------------ split-BF16 forward

// Round FP32 to the nearest BF16 (ties to even) in integer arithmetic; returns
// the FP32 bit pattern with the low 16 bits clear.  NaN stays a quiet NaN.
__device__ __forceinline__ uint32_t bf16_rne_bits(float x) {
  const uint32_t b = __float_as_uint(x);
  if ((b & 0x7f800000u) == 0x7f800000u && (b & 0x007fffffu) != 0u) return (b | 0x00400000u) & 0xffff0000u;
  return (b + 0x7fffu + ((b >> 16) & 1u)) & 0xffff0000u;
}

// x = hi + lo + O(2^-18 |x|): hi = bf16(x), lo = bf16(x - hi), as BF16 bit patterns.
__device__ __forceinline__ void split_bf16(float x, uint16_t& hi, uint16_t& lo) {
  const uint32_t h = bf16_rne_bits(x);
  const float r = x - __uint_as_float(h);  // exact in FP32
  hi = (uint16_t)(h >> 16);
  lo = (uint16_t)(bf16_rne_bits(r) >> 16);
}

struct alignas(16) Bf16x8Bits {
  uint16_t v[8];
};

__device__ __forceinline__ bf16x8 as_bf16x8(const Bf16x8Bits& x) { return __builtin_bit_cast(bf16x8, x); }

// A operand (8 consecutive k per lane) of tile T, k-step s of the BF16 MFMA.
// BF16 result rows are 4g + q, so A row m holds slot q = m % 4 of lane group g = m / 4.
template <int NP>
__device__ __forceinline__ void afrag_bf16(const float* __restrict__ D, int T, int s, int lane,
                                           Bf16x8Bits& hi, Bf16x8Bits& lo) {
  const int m = lane & 15, kk = lane >> 4;
  const int g = m >> 2, q = m & 3;
  const int sigma = 4 * T + q;
  const int a = slot_dir(sigma), i = slot_node(sigma, g);
  const bool row_ok = sigma < Shape<NP>::SLOTS && i < NP;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int j = 32 * s + 8 * kk + e;
    const float x = (row_ok && j < NP) ? D[(a * NP + i) * NP + j] : 0.0f;
    split_bf16(x, hi.v[e], lo.v[e]);
  }
}

template <int NP>
constexpr int bf16_table_entries() { return Shape<NP>::MT * Shape<NP>::KS16 * WAVE; }

template <int NP>
constexpr bool bf16_table_in_lds() { return bf16_table_entries<NP>() * 32 <= LDS_TABLE_LIMIT; }

template <int NP, int WPB>
__global__ __launch_bounds__(WAVE* WPB) void fwd_f32s_kernel(
    const float* __restrict__ D, const float* __restrict__ G, const float* __restrict__ u,
    float* __restrict__ out, uint32_t ncols, uint32_t F, int64_t plane, uint32_t ntiles) {
  using Sh = Shape<NP>;
  constexpr bool ALDS = bf16_table_in_lds<NP>();
  constexpr int NT = ALDS ? bf16_table_entries<NP>() : 1;
  __shared__ Bf16x8Bits ahi[NT];
  __shared__ Bf16x8Bits alo[NT];
  const int lane = threadIdx.x & 63;
  if constexpr (ALDS) {
    for (int e = threadIdx.x; e < NT; e += WAVE * WPB) {
      const int ts = e >> 6;
      Bf16x8Bits h, l;
      afrag_bf16<NP>(D, ts / Sh::KS16, ts % Sh::KS16, e & 63, h, l);
      ahi[e] = h;
      alo[e] = l;
    }
    __syncthreads();
  }
  const int n = lane & 15, g = lane >> 4;
  const uint32_t wave = threadIdx.x >> 6;
  for (uint32_t t = blockIdx.x * WPB + wave; t < ntiles; t += gridDim.x * WPB) {
    const uint32_t col = t * 16 + n;
    const bool valid = col < ncols;
    const float* __restrict__ uc = u + (int64_t)col * NP;
    Bf16x8Bits bh[Sh::KS16], bl[Sh::KS16];
#pragma unroll
    for (int s = 0; s < Sh::KS16; ++s) {
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int j = 32 * s + 8 * g + e;
        const float x = (valid && j < NP) ? uc[j] : 0.0f;
        split_bf16(x, bh[s].v[e], bl[s].v[e]);
      }
    }
    const uint32_t k = valid ? col / F : 0u;
    float gk[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) gk[c] = valid ? G[(int64_t)k * 9 + c] : 0.0f;
    float* __restrict__ oc = out + (int64_t)col * NP;
#pragma unroll
    for (int ch = 0; ch < Sh::NCHUNK; ++ch) {
      f32x4 acc[3];
#pragma unroll
      for (int tt = 0; tt < 3; ++tt) acc[tt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int s = 0; s < Sh::KS16; ++s) {
#pragma unroll
        for (int tt = 0; tt < 3; ++tt) {
          const int T = 3 * ch + tt;
          if (T < Sh::MT) {
            Bf16x8Bits ah, al;
            if constexpr (ALDS) {
              ah = ahi[(T * Sh::KS16 + s) * WAVE + lane];
              al = alo[(T * Sh::KS16 + s) * WAVE + lane];
            } else {
              afrag_bf16<NP>(D, T, s, lane, ah, al);
            }
            // small cross terms first, then hi x hi
            acc[tt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(al), as_bf16x8(bh[s]), acc[tt], 0, 0, 0);
            acc[tt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(ah), as_bf16x8(bl[s]), acc[tt], 0, 0, 0);
            acc[tt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(ah), as_bf16x8(bh[s]), acc[tt], 0, 0, 0);
          }
        }
      }
#pragma unroll
      for (int tau = 4 * ch; tau < 4 * ch + 4; ++tau) {
        if (tau < Sh::TRIP) {
          float R[3];
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            const int loc = 3 * tau + a - 12 * ch;
            R[a] = acc[loc >> 2][loc & 3];
          }
          const int i = 4 * tau + g;
          if (valid && i < NP) {
#pragma unroll
            for (int bb = 0; bb < 3; ++bb)
              oc[bb * plane + i] = gk[bb] * R[0] + gk[3 + bb] * R[1] + gk[6 + bb] * R[2];
          }
        }
      }
    }
  }
}

// ------------------------------------------------------------------ launch helpers

constexpr int MAX_DEVICES = 64;

// Persistent grid size: resident blocks per CU (occupancy query) x CU count,
// cached per kernel instance and device.
template <typename Kern>
static int resident_blocks(Kern kernel, int block, int* err) {
  static std::atomic<int> cache[MAX_DEVICES];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0) {
    *err = DG_EDEVICE;
    return 0;
  }
  if (dev < MAX_DEVICES) {
    const int c = cache[dev].load(std::memory_order_relaxed);
    if (c > 0) return c;
  }
  int cus = 0, per_cu = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) {
    *err = DG_EDEVICE;
    return 0;
  }
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, block, 0) != hipSuccess || per_cu <= 0)
    per_cu = 1;
  const int total = cus * per_cu;
  if (dev < MAX_DEVICES) cache[dev].store(total, std::memory_order_relaxed);
  return total;
}

static inline uint32_t ceil_div(uint64_t a, uint64_t b) { return (uint32_t)((a + b - 1) / b); }

constexpr int FWD_WPB = 4;
constexpr int ADJ_WPB = 4;

template <int NP>
static dg_status launch_fwd_f64(const double* D, const double* G, const double* u, double* out, int64_t K,
                                int32_t F, hipStream_t stream) {
  const uint64_t ncols = (uint64_t)K * (uint64_t)F;
  const uint32_t ntiles = ceil_div(ncols, 16);
  auto kern = fwd_f64_kernel<NP, FWD_WPB>;
  int err = DG_OK;
  const int cap = resident_blocks(kern, WAVE * FWD_WPB, &err);
  if (err != DG_OK) return err;
  const uint32_t grid = std::min<uint32_t>(ceil_div(ntiles, FWD_WPB), (uint32_t)cap);
  hipLaunchKernelGGL(kern, dim3(grid), dim3(WAVE * FWD_WPB), 0, stream, D, G, u, out, (uint32_t)ncols,
                     (uint32_t)F, (int64_t)ncols * NP, ntiles);
  return hipGetLastError() == hipSuccess ? DG_OK : DG_ELAUNCH;
}

template <int NP>
static dg_status launch_adj_f64(const double* D, const double* G, const double* u, const double* gout,
                                double* gu, double* gG, int64_t K, int32_t F, hipStream_t stream) {
  const uint32_t E = F <= 16 ? (uint32_t)(16 / F) : 1u;
  const uint32_t nsub = F <= 16 ? 1u : ceil_div((uint64_t)F, 16);
  const uint32_t ntiles = ceil_div((uint64_t)K, E);
  auto kern = adj_f64_kernel<NP, ADJ_WPB>;
  int err = DG_OK;
  const int cap = resident_blocks(kern, WAVE * ADJ_WPB, &err);
  if (err != DG_OK) return err;
  const uint32_t grid = std::min<uint32_t>(ceil_div(ntiles, ADJ_WPB), (uint32_t)cap);
  hipLaunchKernelGGL(kern, dim3(grid), dim3(WAVE * ADJ_WPB), 0, stream, D, G, u, gout, gu, gG, (uint32_t)K,
                     (uint32_t)F, (int64_t)K * F * NP, E, nsub, ntiles);
  return hipGetLastError() == hipSuccess ? DG_OK : DG_ELAUNCH;
}

template <int NP>
static dg_status launch_fwd_f32s(const float* D, const float* G, const float* u, float* out, int64_t K,
                                 int32_t F, hipStream_t stream) {
  const uint64_t ncols = (uint64_t)K * (uint64_t)F;
  const uint32_t ntiles = ceil_div(ncols, 16);
  auto kern = fwd_f32s_kernel<NP, FWD_WPB>;
  int err = DG_OK;
  const int cap = resident_blocks(kern, WAVE * FWD_WPB, &err);
  if (err != DG_OK) return err;
  const uint32_t grid = std::min<uint32_t>(ceil_div(ntiles, FWD_WPB), (uint32_t)cap);
  hipLaunchKernelGGL(kern, dim3(grid), dim3(WAVE * FWD_WPB), 0, stream, D, G, u, out, (uint32_t)ncols,
                     (uint32_t)F, (int64_t)ncols * NP, ntiles);
  return hipGetLastError() == hipSuccess ? DG_OK : DG_ELAUNCH;
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
    case DG_EINVAL: return "invalid argument (null or misaligned pointer, K < 0, F < 1, or K*F too large)";
    case DG_EUNSUPPORTED: return "unsupported node count Np (supported: 4, 10, 20, 35, 56, 84, 120)";
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

dg_status dg_volume(const double* D, const double* G, const double* u, double* out, int64_t K, int32_t Np,
                    int32_t F, void* stream) {
  bool noop = false;
  const dg_status st = check_common(K, Np, F, &noop);
  if (st != DG_OK || noop) return st;
  if (!D || !G || !u || !out) return DG_EINVAL;
  if (!aligned(D, 8) || !aligned(G, 8) || !aligned(u, 8) || !aligned(out, 8)) return DG_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  switch (Np) {
    case 4: return launch_fwd_f64<4>(D, G, u, out, K, F, s);
    case 10: return launch_fwd_f64<10>(D, G, u, out, K, F, s);
    case 20: return launch_fwd_f64<20>(D, G, u, out, K, F, s);
    case 35: return launch_fwd_f64<35>(D, G, u, out, K, F, s);
    case 56: return launch_fwd_f64<56>(D, G, u, out, K, F, s);
    case 84: return launch_fwd_f64<84>(D, G, u, out, K, F, s);
    case 120: return launch_fwd_f64<120>(D, G, u, out, K, F, s);
  }
  return DG_EUNSUPPORTED;
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
  hipStream_t s = (hipStream_t)stream;
  switch (Np) {
    case 4: return launch_adj_f64<4>(D, G, u, gout, gu, gG, K, F, s);
    case 10: return launch_adj_f64<10>(D, G, u, gout, gu, gG, K, F, s);
    case 20: return launch_adj_f64<20>(D, G, u, gout, gu, gG, K, F, s);
    case 35: return launch_adj_f64<35>(D, G, u, gout, gu, gG, K, F, s);
    case 56: return launch_adj_f64<56>(D, G, u, gout, gu, gG, K, F, s);
    case 84: return launch_adj_f64<84>(D, G, u, gout, gu, gG, K, F, s);
    case 120: return launch_adj_f64<120>(D, G, u, gout, gu, gG, K, F, s);
  }
  return DG_EUNSUPPORTED;
}

dg_status dg_volume_f32s(const float* D, const float* G, const float* u, float* out, int64_t K, int32_t Np,
                         int32_t F, void* stream) {
  bool noop = false;
  const dg_status st = check_common(K, Np, F, &noop);
  if (st != DG_OK || noop) return st;
  if (!D || !G || !u || !out) return DG_EINVAL;
  if (!aligned(D, 4) || !aligned(G, 4) || !aligned(u, 4) || !aligned(out, 4)) return DG_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  switch (Np) {
    case 4: return launch_fwd_f32s<4>(D, G, u, out, K, F, s);
    case 10: return launch_fwd_f32s<10>(D, G, u, out, K, F, s);
    case 20: return launch_fwd_f32s<20>(D, G, u, out, K, F, s);
    case 35: return launch_fwd_f32s<35>(D, G, u, out, K, F, s);
    case 56: return launch_fwd_f32s<56>(D, G, u, out, K, F, s);
    case 84: return launch_fwd_f32s<84>(D, G, u, out, K, F, s);
    case 120: return launch_fwd_f32s<120>(D, G, u, out, K, F, s);
  }
  return DG_EUNSUPPORTED;
}

}  // extern "C"
