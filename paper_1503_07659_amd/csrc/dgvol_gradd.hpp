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

// ------------------------------------------------------------------ order 5: producer and consumer waves
//
// At Np = 56 the 44 output tiles (11 stacked row tiles x 4 column blocks) split
// evenly over the four SIMDs by column block.  The workgroup's waves take two
// roles: consumer wave jb (0..3, one per SIMD) owns column block jb with all
// 11 row tiles in its accumulators and reads 12 operands per 11 products;
// producer waves (4..7) load u, gout and G two steps ahead, form W and stage
// both into the LDS buffer of the next step.  One barrier per step.  Each
// output tile accumulates its k steps in column order, so the partial sums
// depend on (K, F) only.
struct GdSplit56 {
  static constexpr int NP = 56;
  static constexpr int WPB = 8;
  static constexpr int NTH = WAVE * WPB;
  static constexpr int NCONS = 4;                    // consumer waves (column blocks)
  static constexpr int NPRODT = NTH - NCONS * WAVE;  // producer threads
  static constexpr int NB = 4, RT = 11;
  static constexpr int CH = 16;                      // columns per step
  static constexpr int KST = CH / 4;                 // k steps per step
  static constexpr int LDU = gd_ld(16 * NB);
  static constexpr int LDW = gd_ld(16 * RT);
  static constexpr int STAGE_DOUBLES = CH * (LDU + LDW);
  static constexpr int TPC = NPRODT / CH;            // producer threads per column
  static constexpr int NXU = (NP + TPC - 1) / TPC;   // values per producer thread and plane
  static constexpr int DEPTH = 2;                    // steps the loads run ahead
  static_assert(GD_UNIT % CH == 0, "staging step");
  static_assert(2 * 2 * STAGE_DOUBLES * 8 <= 160 * 1024, "two workgroups per CU");
};

__global__ __launch_bounds__(GdSplit56::NTH) __attribute__((amdgpu_waves_per_eu(4, 8)))
void gd_split56_kernel(GdArgs p) {
  using S = GdSplit56;
  constexpr int NP = S::NP;
  constexpr int CH = S::CH;
  constexpr int SUB = GD_UNIT / CH;
  __shared__ double lds[2 * S::STAGE_DOUBLES];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const uint32_t wave = __builtin_amdgcn_readfirstlane((uint32_t)tid >> 6);
  const uint32_t part = blockIdx.x;
  if (part >= p.npart) return;
  const uint32_t st_begin = (uint32_t)((uint64_t)part * p.nunits / p.npart) * SUB;
  const uint32_t st_end = (uint32_t)((uint64_t)(part + 1) * p.nunits / p.npart) * SUB;
  const uint32_t nsteps = st_end - st_begin;

  // pad entries (columns Np.. of u, rows 3 Np.. of W) stay zero
  for (int x = tid; x < 2 * S::STAGE_DOUBLES; x += S::NTH) lds[x] = 0.0;
  __syncthreads();

  const bool consumer = wave < S::NCONS;
  // ---- producer state: u and gout DEPTH steps ahead (register set r % DEPTH),
  // the geometric factors one step ahead (one set).  Loads go through buffer
  // ranges of the column's valid words (past them: zeros, no access), so no
  // branch surrounds a load and the waits count exactly.
  const int pt = tid - S::NCONS * WAVE;  // producer thread (valid when !consumer)
  const int cc = consumer ? 0 : pt / S::TPC;
  const int rr = consumer ? 0 : pt % S::TPC;
  double ru[S::DEPTH][S::NXU], rg0[S::DEPTH][S::NXU], rg1[S::DEPTH][S::NXU], rg2[S::DEPTH][S::NXU];
  double rG[9];
  // The buffer ranges are the step's (wave-uniform base and size: one
  // descriptor per wave); a lane's node past Np reads a word of the next
  // column, which is never staged.
  auto load_ug = [&](uint32_t r, int d) __attribute__((always_inline)) {
    const uint32_t c0 = (st_begin + r) * CH;
    const uint32_t ncl = r < nsteps && c0 < p.ncols ? min((uint32_t)CH, p.ncols - c0) : 0u;
    const int64_t base = (int64_t)(ncl ? c0 : 0u) * NP;
    const uint32_t nb = ncl * NP * 8u;
    const __amdgpu_buffer_rsrc_t bu = buffer_range(p.u + base, nb);
    const __amdgpu_buffer_rsrc_t b0 = buffer_range(p.gout + base, nb);
    const __amdgpu_buffer_rsrc_t b1 = buffer_range(p.gout + p.plane + base, nb);
    const __amdgpu_buffer_rsrc_t b2 = buffer_range(p.gout + 2 * p.plane + base, nb);
#pragma unroll
    for (int q = 0; q < S::NXU; ++q) {
      const uint32_t off = (uint32_t)(cc * NP + rr + S::TPC * q) * 8u;
      ru[d][q] = buffer_load_f64(bu, off);
      rg0[d][q] = buffer_load_f64(b0, off);
      rg1[d][q] = buffer_load_f64(b1, off);
      rg2[d][q] = buffer_load_f64(b2, off);
    }
  };
  auto load_g = [&](uint32_t r) __attribute__((always_inline)) {
    const uint32_t c0 = (st_begin + r) * CH;
    const uint32_t ncl = r < nsteps && c0 < p.ncols ? min((uint32_t)CH, p.ncols - c0) : 0u;
    const uint32_t k0 = ncl ? c0 / p.F : 0u;
    const uint32_t nk = ncl ? (c0 + ncl - 1) / p.F - k0 + 1 : 0u;
    const __amdgpu_buffer_rsrc_t bg = buffer_range(p.G + (int64_t)k0 * 9, nk * 72u);
    const uint32_t ke = (c0 + (uint32_t)cc) / p.F - k0;  // this lane's element within the step
#pragma unroll
    for (int m = 0; m < 9; ++m) rG[m] = buffer_load_f64(bg, (ke * 9u + (uint32_t)m) * 8u);
  };
  auto stage = [&](int d, int b) __attribute__((always_inline)) {
    double* ul = lds + b * S::STAGE_DOUBLES;
    double* wl = ul + CH * S::LDU;
#pragma unroll
    for (int q = 0; q < S::NXU; ++q) {
      const int i = rr + S::TPC * q;
      if (i < NP) {
        ul[cc * S::LDU + i] = ru[d][q];
#pragma unroll
        for (int a = 0; a < 3; ++a)
          wl[cc * S::LDW + a * NP + i] = rG[3 * a] * rg0[d][q] + rG[3 * a + 1] * rg1[d][q] + rG[3 * a + 2] * rg2[d][q];
      }
    }
  };
  // Each role runs its own loop (so that the consumers' accumulators and the
  // producers' register sets are never live together), with the same barriers:
  // one after the prologue, one per step.  Step r sits in producer register set
  // r % DEPTH and staging buffer r % 2 (DEPTH = 2: both alternate with r).
  if (consumer) {
    // column block jb = wave, all row tiles
    f64x4 acc[S::RT];
#pragma unroll
    for (int t = 0; t < S::RT; ++t) acc[t] = f64x4{0.0, 0.0, 0.0, 0.0};
    const double* ub0 = lds + wave * 16 + (lane & 15);
    const double* wa0 = lds + CH * S::LDU + (lane & 15);
    __syncthreads();
    for (uint32_t r = 0; r < nsteps; ++r) {
      const int b = (int)(r & 1u);
      const double* ub = ub0 + b * S::STAGE_DOUBLES;
      const double* wa = wa0 + b * S::STAGE_DOUBLES;
      // rolling operands: after each product the register of its A operand is
      // refilled with the next k step's (one LDS read after each product)
      const int cl = lane >> 4;
      double av[S::RT];
      double bv = ub[cl * S::LDU];
#pragma unroll
      for (int t = 0; t < S::RT; ++t) av[t] = wa[cl * S::LDW + t * 16];
#pragma unroll
      for (int kk = 0; kk < S::KST; ++kk) {
        const int cn = 4 * (kk + 1) + cl;
        const double bn = kk + 1 < S::KST ? ub[cn * S::LDU] : 0.0;
#pragma unroll
        for (int t = 0; t < S::RT; ++t) {
          acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[t], bv, acc[t], 0, 0, 0);
          if (kk + 1 < S::KST) av[t] = wa[cn * S::LDW + t * 16];
        }
#pragma unroll
        for (int t = 0; t < S::RT; ++t) {
          __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // one product,
          __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);  // then one LDS read
        }
        __builtin_amdgcn_sched_barrier(0);
        bv = bn;
      }
      __syncthreads();  // the producers have staged step r + 1; buffer r % 2 is free
    }
    double* w = p.work + (int64_t)part * 3 * NP * NP;
    const int j = (int)wave * 16 + (lane & 15);
#pragma unroll
    for (int t = 0; t < S::RT; ++t) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = t * 16 + 4 * q + (lane >> 4);
        if (r < 3 * NP && j < NP) w[(int64_t)r * NP + j] = acc[t][q];
      }
    }
  } else {
    static_assert(S::DEPTH == 2, "register sets alternate with the step");
    if (nsteps > 0) {
      load_ug(0, 0);
      load_ug(1, 1);
      load_g(0);
      stage(0, 0);
      load_g(1);
      load_ug(2, 0);
    }
    __syncthreads();
    // iteration r stages step r + 1 (its G requested one iteration earlier, its u and
    // gout two), then requests G of step r + 2 and u, gout of step r + 3
    for (uint32_t r0 = 0; r0 < nsteps; r0 += 2) {
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const uint32_t r = r0 + j;
        if (r < nsteps) {
          stage(j ^ 1, j ^ 1);
          load_g(r + 2);
          load_ug(r + 3, j ^ 1);
          __syncthreads();
        }
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
