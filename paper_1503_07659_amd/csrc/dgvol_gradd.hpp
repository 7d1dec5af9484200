// Cotangent of the reference differentiation matrices, FP64.
//
// The forward map is linear in D, so for a cotangent gout of the three output
// planes the cotangent of D is a sum over every element column c = (k, f):
//   W_a[c][i]   = sum_b G[k][3a+b] gout[b][c][i]
//   gD[a][i][j] = sum_c W_a[c][i] u[c][j]
// Stacking the three directions, rows r = a Np + i, this is ONE contraction
//   gD[r][j] = sum_c W[c][r] u[c][j]          ([3Np x ncols] . [ncols x Np])
// whose reduction dimension is the (long) column axis.  It runs on the FP64
// matrix cores with the columns as the MFMA k dimension:
//
//   * the 3Np stacked rows form ceil(3Np/16) row tiles and the Np columns
//     ceil(Np/16) column blocks (stacking wastes less of a 16-row tile than
//     padding every direction separately);
//   * the columns are split into npart contiguous ranges; one workgroup owns
//     one range (at the two highest orders NSPLIT workgroups, each with a
//     share of the row tiles) and keeps its output tiles in accumulators
//     spread over its waves; with fewer tiles than waves the waves also split
//     the k steps and add their partial tiles at the end in a fixed order;
//   * per step the workgroup stages u[c][:] and W[c][rows] in LDS, row-major
//     per column; each thread stages a fixed column, so it needs the
//     geometric factors of one element only;
//   * the staging is software-pipelined over two LDS buffers: while the waves
//     multiply step s out of one buffer, each thread writes step s+1 (loaded
//     into registers during step s-1) into the other and requests step s+2
//     from memory, with one barrier per step;
//   * each workgroup writes its partial gD to work[part]; a second kernel adds
//     the partials in a fixed order.
//
// The partition depends only on (K, F, Np), never on the device, and every
// sum runs in a fixed order, so the result is reproducible bit for bit.
#pragma once

#include "dgvol_device.hpp"

namespace dgvol {

// Columns per partition unit; every staging step (16..128 columns) divides it.
constexpr int GD_UNIT = 128;
constexpr int GD_WPB = 8;

// Upper bound on the number of partial sums (a function of Np only).
__host__ __device__ constexpr uint32_t gd_maxpart(int np) { return np <= 35 ? 1024u : 512u; }

// Row stride in LDS: an odd multiple of 16 doubles, so the 16-lane row
// segments of an MFMA operand read start 128 bytes apart modulo 256 and two of
// them never share banks.
constexpr int gd_ld(int n16) { return (n16 / 16) % 2 == 1 ? n16 : n16 + 16; }

template <int NP>
struct GdShape {
  static constexpr int NTH = WAVE * GD_WPB;
  static constexpr int NB = (NP + 15) / 16;            // column blocks (j)
  static constexpr int RT = (3 * NP + 15) / 16;        // row tiles (stacked r = a Np + i)
  static constexpr int NSPLIT = NP >= 120 ? 4 : (NP >= 84 ? 2 : 1);
  static constexpr int RTS = (RT + NSPLIT - 1) / NSPLIT;  // row tiles per workgroup
  static constexpr int NTW = RTS * NB;                  // output tiles per workgroup
  static constexpr int KSPLIT = NTW >= GD_WPB ? 1 : (NTW == 1 ? 8 : (NTW == 2 ? 4 : 2));
  static constexpr int SLOTS = NTW * KSPLIT;            // (tile, k share) pairs
  static constexpr int TPW = (SLOTS + GD_WPB - 1) / GD_WPB;
  // columns per step: two staging buffers of at most 32 KB, so that two
  // workgroups fit the LDS of a CU
  static constexpr int CH = NP <= 4 ? 128 : (NP <= 10 ? 64 : (NP <= 35 ? 32 : 16));
  static constexpr int TPC = NTH / CH;                  // threads staging one column
  static constexpr int NXU = (NP + TPC - 1) / TPC;      // values per thread and plane
  static constexpr int LDU = gd_ld(16 * NB);
  static constexpr int LDW = gd_ld(16 * RTS);
  static constexpr int STAGE_DOUBLES = CH * (LDU + LDW);  // one staging buffer
  static constexpr int RED_DOUBLES = KSPLIT > 1 ? SLOTS * 256 : 0;
  static constexpr int LDS_DOUBLES = 2 * STAGE_DOUBLES > RED_DOUBLES ? 2 * STAGE_DOUBLES : RED_DOUBLES;
  static_assert(2 * LDS_DOUBLES * 8 <= 160 * 1024, "two workgroups per CU");
  static_assert(GD_UNIT % CH == 0 && CH % 4 == 0, "staging step");
  static_assert((CH / 4) % KSPLIT == 0, "k steps split evenly");
};

struct GdArgs {
  const double* G;
  const double* u;
  const double* gout;
  double* work;      // [npart][3][Np][Np]
  uint32_t ncols;    // K * F
  uint32_t F;
  int64_t plane;     // K * F * Np
  uint32_t nunits;   // ceil(ncols / GD_UNIT)
  uint32_t npart;
};

// Two workgroups per CU (at most 128 registers a lane) so that one stages
// while the other multiplies.
template <int NP>
__global__ __launch_bounds__(GdShape<NP>::NTH) __attribute__((amdgpu_waves_per_eu(4, 8)))
void gd_partial_kernel(GdArgs p) {
  using S = GdShape<NP>;
  constexpr int CH = S::CH;
  constexpr int SUB = GD_UNIT / CH;  // steps per partition unit
  __shared__ double lds[S::LDS_DOUBLES];
  // staging buffer b: u[c][j] at [b][c][LDU], W[c][r - r0] at [b][CH LDU + c LDW]
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  // Workgroups of one column range sit on one XCD (workgroups are dealt to
  // the 8 XCDs in turn), so the NSPLIT reads of a column hit one L2.
  uint32_t part, split;
  if constexpr (S::NSPLIT == 1) {
    part = blockIdx.x;
    split = 0;
  } else {
    const uint32_t j = blockIdx.x >> 3;
    split = j % S::NSPLIT;
    part = (j / S::NSPLIT) * 8 + (blockIdx.x & 7);
  }
  if (part >= p.npart) return;
  const uint32_t st_begin = (uint32_t)((uint64_t)part * p.nunits / p.npart) * SUB;
  const uint32_t st_end = (uint32_t)((uint64_t)(part + 1) * p.nunits / p.npart) * SUB;
  const int r0 = (int)split * S::RTS * 16;  // first stacked row of this workgroup
  const int r1 = min(r0 + S::RTS * 16, 3 * NP);

  // Pad entries (columns Np.. of u, rows r1-r0.. of W) feed only outputs that
  // are never stored; keep them finite.
  for (int x = tid; x < 2 * S::STAGE_DOUBLES; x += S::NTH) lds[x] = 0.0;
  __syncthreads();

  // this thread's column within a step and its first row
  const int cc = tid / S::TPC;
  const int rr = tid % S::TPC;
  double ru[S::NXU], rg0[S::NXU], rg1[S::NXU], rg2[S::NXU], rG[9];
  auto load = [&](uint32_t st) __attribute__((always_inline)) {
    const uint32_t col = st * CH + cc;
    const bool v = col < p.ncols;
    const int64_t base = (int64_t)col * NP;
#pragma unroll
    for (int q = 0; q < S::NXU; ++q) {
      const int i = rr + S::TPC * q;
      const bool ok = v && i < NP;
      ru[q] = ok ? p.u[base + i] : 0.0;
      rg0[q] = ok ? p.gout[base + i] : 0.0;
      rg1[q] = ok ? p.gout[p.plane + base + i] : 0.0;
      rg2[q] = ok ? p.gout[2 * p.plane + base + i] : 0.0;
    }
    const int64_t gb = (int64_t)(v ? col / p.F : 0u) * 9;
#pragma unroll
    for (int m = 0; m < 9; ++m) rG[m] = v ? p.G[gb + m] : 0.0;
  };

  // write the registers' step into staging buffer b
  auto stage = [&](int b) __attribute__((always_inline)) {
    double* ul = lds + b * S::STAGE_DOUBLES;
    double* wl = ul + CH * S::LDU;
#pragma unroll
    for (int q = 0; q < S::NXU; ++q) {
      const int i = rr + S::TPC * q;
      if (i < NP) {
        ul[cc * S::LDU + i] = ru[q];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          const int r = a * NP + i;
          if (r >= r0 && r < r1)
            wl[cc * S::LDW + (r - r0)] = rG[3 * a] * rg0[q] + rG[3 * a + 1] * rg1[q] + rG[3 * a + 2] * rg2[q];
        }
      }
    }
  };

  f64x4 acc[S::TPW];
#pragma unroll
  for (int t = 0; t < S::TPW; ++t) acc[t] = f64x4{0.0, 0.0, 0.0, 0.0};

  // prologue: step st_begin staged in buffer 0, step st_begin + 1 in registers
  if (st_begin < st_end) {
    load(st_begin);
    stage(0);
    if (st_begin + 1 < st_end) load(st_begin + 1);
  }
  __syncthreads();
  int cur = 0;
  for (uint32_t st = st_begin; st < st_end; ++st) {
    // the other buffer was last read by the products of the previous step,
    // which every wave finished before the barrier that ended it
    if (st + 1 < st_end) {
      stage(cur ^ 1);
      if (st + 2 < st_end) load(st + 2);
    }
    const double* ul = lds + cur * S::STAGE_DOUBLES;
    const double* wl = ul + CH * S::LDU;
#pragma unroll
    for (int t = 0; t < S::TPW; ++t) {
      const int slot = wave * S::TPW + t;
      if (slot < S::SLOTS) {
        const int T = slot / S::KSPLIT;
        const int ks = slot % S::KSPLIT;
        const int rt = T / S::NB;
        const int jb = T % S::NB;
        const double* wa = wl + rt * 16 + (lane & 15);
        const double* ub = ul + jb * 16 + (lane & 15);
#pragma unroll
        for (int kk = ks; kk < CH / 4; kk += S::KSPLIT) {
          const int c = 4 * kk + (lane >> 4);
          acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(wa[c * S::LDW], ub[c * S::LDU], acc[t], 0, 0, 0);
        }
      }
      // one slot's operands at a time: keeps the LDS reads from being hoisted
      // into registers for every slot at once
      __builtin_amdgcn_sched_barrier(0);
    }
    __syncthreads();  // the next step's staging is visible; this buffer is free
    cur ^= 1;
  }

  // Add the k shares of each tile (fixed order) and store the partial sum.
  double* w = p.work + (int64_t)part * 3 * NP * NP;
  auto store_tile = [&](int T, const f64x4& v) __attribute__((always_inline)) {
    const int rt = T / S::NB;
    const int jb = T % S::NB;
    const int j = jb * 16 + (lane & 15);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int r = r0 + rt * 16 + 4 * q + (lane >> 4);
      if (r < r1 && j < NP) w[(int64_t)r * NP + j] = v[q];
    }
  };
  if constexpr (S::KSPLIT == 1) {
#pragma unroll
    for (int t = 0; t < S::TPW; ++t) {
      const int slot = wave * S::TPW + t;
      if (slot < S::SLOTS) store_tile(slot, acc[t]);
    }
  } else {
    __syncthreads();  // staging buffers are reused for the k shares
#pragma unroll
    for (int t = 0; t < S::TPW; ++t) {
      const int slot = wave * S::TPW + t;
      if (slot < S::SLOTS) {
#pragma unroll
        for (int q = 0; q < 4; ++q) lds[(slot * 4 + q) * WAVE + lane] = acc[t][q];
      }
    }
    __syncthreads();
    for (int T = wave; T < S::NTW; T += GD_WPB) {
      f64x4 v = f64x4{0.0, 0.0, 0.0, 0.0};
      for (int ks = 0; ks < S::KSPLIT; ++ks) {
#pragma unroll
        for (int q = 0; q < 4; ++q) v[q] += lds[((T * S::KSPLIT + ks) * 4 + q) * WAVE + lane];
      }
      store_tile(T, v);
    }
  }
}

// gD[x] = sum over parts of work[part][x], x < n, in a fixed order.
// Block: 64 consecutive x by GD_RED_PG part groups; part group g adds parts
// g, g + GD_RED_PG, ... in ascending order, and the group sums are then added
// in ascending g.  With npart = 0 it writes zeros.
constexpr int GD_RED_PG = 16;

__global__ __launch_bounds__(64 * GD_RED_PG) void gd_reduce_kernel(const double* __restrict__ work,
                                                                  double* __restrict__ gD, uint32_t npart,
                                                                  uint32_t n) {
  __shared__ double part_sum[GD_RED_PG][64];
  const int xi = threadIdx.x & 63;
  const int g = threadIdx.x >> 6;
  const uint32_t x = blockIdx.x * 64 + xi;
  double s = 0.0;
  if (x < n) {
    for (uint32_t pt = g; pt < npart; pt += GD_RED_PG) s += work[(int64_t)pt * n + x];
  }
  part_sum[g][xi] = s;
  __syncthreads();
  if (g == 0 && x < n) {
    double t = 0.0;
#pragma unroll
    for (int h = 0; h < GD_RED_PG; ++h) t += part_sum[h][xi];
    gD[x] = t;
  }
}

}  // namespace dgvol
