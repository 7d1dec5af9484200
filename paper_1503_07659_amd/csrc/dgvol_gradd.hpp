// Cotangent of the reference differentiation matrices, FP64.
//
// The forward map is linear in D, so for a cotangent gout of the three output
// planes the cotangent of D is a sum over every element column c = (k, f):
//   W_a[c][i]   = sum_b G[k][3a+b] gout[b][c][i]
//   gD[a][i][j] = sum_c W_a[c][i] u[c][j]
// which is the contraction W_a^T u with the element columns as its (long)
// reduction dimension: a GEMM of shape [Np x ncols] . [ncols x Np] per
// direction.  It runs on the FP64 matrix cores with the columns as the MFMA
// k dimension:
//
//   * the columns are split into npart contiguous ranges of 32-column chunks
//     (staged 16 or 32 columns per step); one workgroup (two at the highest
//     order, each with half of the tiles) owns one range and keeps the
//     3 x ceil(Np/16)^2 output tiles of its partial sum in accumulators,
//     spread over its waves;
//   * per chunk the workgroup stages u[c][:] and W_a[c][:] (formed from gout
//     and G while staging) in LDS, row-major per column, and every wave feeds
//     its tiles' MFMAs from there: A[i][c] = W_a[c][i], B[c][j] = u[c][j];
//   * each workgroup writes its partial gD to work[part]; a second kernel adds
//     the partials in a fixed order.
//
// The partition depends only on (K, F, Np), never on the device, and every
// sum runs in a fixed order, so the result is reproducible bit for bit.
#pragma once

#include "dgvol_device.hpp"

namespace dgvol {

// Upper bound on the number of partial sums (workgroups of the first pass).
constexpr uint32_t GD_MAXPART = 512;
// Element columns staged per step: a multiple of the MFMA k (4) and a divisor
// of GD_CHUNK_MAX, which fixes the partition into chunks for every order.
constexpr int GD_CHUNK_MAX = 32;

template <int NP>
struct GdShape {
  static constexpr int CH = NP >= 84 ? 16 : 32;           // columns per step
  static constexpr int NB = (NP + 15) / 16;               // 16-row blocks of one matrix
  static constexpr int NPAD = 16 * NB;
  static constexpr int LD = (NB & 1) ? NPAD : NPAD + 16;  // LDS row stride: rows 4 apart never share banks
  static constexpr int WPB = 8;
  static constexpr int NTH = WAVE * WPB;
  static constexpr int NT = 3 * NB * NB;                   // 16x16 output tiles
  // Workgroups per column range, each owning 1/NSPLIT of the tiles: at the
  // highest order the accumulators of all tiles do not fit one workgroup's
  // registers, and that order is bound by the matrix cores, so reading its
  // columns twice costs little.
  static constexpr int NSPLIT = NP >= 120 ? 2 : 1;
  static constexpr int TPS = (NT + NSPLIT - 1) / NSPLIT;   // tiles per workgroup
  static constexpr int TPW = (TPS + WPB - 1) / WPB;        // tiles per wave
  static constexpr int NXE = CH * NP;                      // staged values per plane per step
  static constexpr int NX = (NXE + NTH - 1) / NTH;         // per thread
  static constexpr int LDS_DOUBLES = 4 * CH * LD + CH * 9;
};

struct GdArgs {
  const double* G;
  const double* u;
  const double* gout;
  double* work;      // [npart][3][Np][Np]
  uint32_t ncols;    // K * F
  uint32_t F;
  int64_t plane;     // K * F * Np
  uint32_t nchunks;  // ceil(ncols / GD_CHUNK_MAX)
  uint32_t npart;
};

template <int NP>
__global__ __launch_bounds__(GdShape<NP>::NTH) void gd_partial_kernel(GdArgs p) {
  using S = GdShape<NP>;
  constexpr int CH = S::CH;
  constexpr int SUB = GD_CHUNK_MAX / CH;  // steps per chunk
  __shared__ double lds[S::LDS_DOUBLES];
  double* ul = lds;                        // [CH][LD]      u[c][j]
  double* wl = lds + CH * S::LD;           // [3][CH][LD]   W_a[c][i]
  double* gl = lds + 4 * CH * S::LD;       // [CH][9]       G row of column c
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const uint32_t part = blockIdx.x / S::NSPLIT;
  const int t_first = (blockIdx.x % S::NSPLIT) * S::TPS + wave * S::TPW;  // this wave's first tile
  const int t_stop = min((int)(blockIdx.x % S::NSPLIT + 1) * S::TPS, S::NT);
  // this part's chunks, as steps of CH columns
  const uint32_t ch_begin = (uint32_t)((uint64_t)part * p.nchunks / p.npart) * SUB;
  const uint32_t ch_end = (uint32_t)((uint64_t)(part + 1) * p.nchunks / p.npart) * SUB;

  // Rows are padded from Np to LD; the pad only feeds output rows and columns
  // beyond Np, which are never stored, but keep it finite.
  constexpr int PADW = S::LD - NP;
  for (int x = tid; x < 4 * CH * PADW; x += S::NTH) lds[(x / PADW) * S::LD + NP + x % PADW] = 0.0;

  double ru[S::NX], rg0[S::NX], rg1[S::NX], rg2[S::NX];
  double rG = 0.0;
  auto load = [&](uint32_t ch) __attribute__((always_inline)) {
    const uint32_t col0 = ch * CH;
    const uint32_t cnt = col0 < p.ncols ? min((uint32_t)CH, p.ncols - col0) * NP : 0u;
    const int64_t base = (int64_t)col0 * NP;
#pragma unroll
    for (int q = 0; q < S::NX; ++q) {
      const uint32_t x = tid + S::NTH * q;
      const bool v = x < cnt;
      ru[q] = v ? p.u[base + x] : 0.0;
      rg0[q] = v ? p.gout[base + x] : 0.0;
      rg1[q] = v ? p.gout[p.plane + base + x] : 0.0;
      rg2[q] = v ? p.gout[2 * p.plane + base + x] : 0.0;
    }
    if (tid < CH * 9) {
      const uint32_t col = col0 + tid / 9;
      rG = col < p.ncols ? p.G[(int64_t)(col / p.F) * 9 + tid % 9] : 0.0;
    }
  };

  f64x4 acc[S::TPW];
#pragma unroll
  for (int t = 0; t < S::TPW; ++t) acc[t] = f64x4{0.0, 0.0, 0.0, 0.0};

  if (ch_begin < ch_end) load(ch_begin);
  for (uint32_t ch = ch_begin; ch < ch_end; ++ch) {
    __syncthreads();  // the previous chunk's products are done with the LDS
#pragma unroll
    for (int q = 0; q < S::NX; ++q) {
      const int x = tid + S::NTH * q;
      if (x < S::NXE) ul[(x / NP) * S::LD + x % NP] = ru[q];
    }
    if (tid < CH * 9) gl[tid] = rG;
    __syncthreads();
#pragma unroll
    for (int q = 0; q < S::NX; ++q) {
      const int x = tid + S::NTH * q;
      if (x < S::NXE) {
        const int c = x / NP, i = x % NP;
        const double* g = gl + 9 * c;
#pragma unroll
        for (int a = 0; a < 3; ++a)
          wl[(a * CH + c) * S::LD + i] = g[3 * a] * rg0[q] + g[3 * a + 1] * rg1[q] + g[3 * a + 2] * rg2[q];
      }
    }
    __syncthreads();
    if (ch + 1 < ch_end) load(ch + 1);
#pragma unroll
    for (int t = 0; t < S::TPW; ++t) {
      const int T = t_first + t;
      if (T < t_stop) {
        const int a = T / (S::NB * S::NB);
        const int ib = (T / S::NB) % S::NB;
        const int jb = T % S::NB;
        const double* wa = wl + a * CH * S::LD + ib * 16 + (lane & 15);
        const double* ub = ul + jb * 16 + (lane & 15);
#pragma unroll
        for (int kk = 0; kk < CH / 4; ++kk) {
          const int c = 4 * kk + (lane >> 4);
          acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(wa[c * S::LD], ub[c * S::LD], acc[t], 0, 0, 0);
        }
      }
      // one tile's operands at a time: keeps the LDS reads from being hoisted
      // into registers for every tile at once
      __builtin_amdgcn_sched_barrier(0);
    }
  }

  double* w = p.work + (int64_t)part * 3 * NP * NP;
#pragma unroll
  for (int t = 0; t < S::TPW; ++t) {
    const int T = t_first + t;
    if (T < t_stop) {
      const int a = T / (S::NB * S::NB);
      const int ib = (T / S::NB) % S::NB;
      const int jb = T % S::NB;
      const int j = jb * 16 + (lane & 15);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = ib * 16 + 4 * q + (lane >> 4);
        if (i < NP && j < NP) w[((int64_t)a * NP + i) * NP + j] = acc[t][q];
      }
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
