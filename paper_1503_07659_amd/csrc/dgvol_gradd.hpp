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

#include <type_traits>

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
  // directions whose W rows one workgroup holds (its geometric factors in registers)
  static constexpr int NDIR = NSPLIT > 1 ? 2 : 3;
  static constexpr bool dirs_fit() {
    for (int s = 0; s < NSPLIT; ++s) {
      const int r0 = s * RTS * 16, r1 = (s + 1) * RTS * 16 < 3 * NP ? (s + 1) * RTS * 16 : 3 * NP;
      if (r0 < r1 && (r1 - 1) / NP - r0 / NP + 1 > NDIR) return false;
    }
    return true;
  }
  static_assert(dirs_fit(), "a workgroup's rows span at most NDIR directions");
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
  // the workgroup's rows start in direction a_lo and span at most NDIR directions;
  // rG holds the geometric factors of those (rows 3 a .. 3 a + 2 of the element's 9)
  const int a_lo = S::NSPLIT > 1 ? r0 / NP : 0;
  double ru[S::NXU], rg0[S::NXU], rg1[S::NXU], rg2[S::NXU], rG[3 * S::NDIR];
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
    for (int d = 0; d < S::NDIR; ++d)
#pragma unroll
      for (int b = 0; b < 3; ++b) rG[3 * d + b] = v ? p.G[gb + 3 * min(a_lo + d, 2) + b] : 0.0;
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
        for (int d = 0; d < S::NDIR; ++d) {
          const int r = (a_lo + d) * NP + i;
          if (r >= r0 && r < r1)
            wl[cc * S::LDW + (r - r0)] = rG[3 * d] * rg0[q] + rG[3 * d + 1] * rg1[q] + rG[3 * d + 2] * rg2[q];
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
// At Np = 56 the workgroup's waves take two roles.  Consumer waves 0..3 (one
// per SIMD) hold the output tiles in their accumulators and run the products
// of each step from LDS (the tiling is described below).  Producer waves
// 4..7 load u and gout two steps ahead (16-byte accesses of node pairs) and
// G one step ahead (one factor per lane, handed to the column's 16-lane row
// by a DPP broadcast), form W and stage both into the LDS buffer of the next
// step.  One barrier per step.  Each output accumulates its k steps in column
// order, so the partial sums depend on (K, F) only.
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
  static constexpr int TPC = NPRODT / CH;            // producer threads per column (one DPP row)
  static constexpr int NPR = (NP / 2 + TPC - 1) / TPC;  // node pairs per producer thread and plane
  static constexpr int NXU = 2 * NPR;                // values per producer thread and plane
  static constexpr int DEPTH = 2;                    // steps the loads run ahead
  static_assert(GD_UNIT % CH == 0, "staging step");
  static_assert(2 * 2 * STAGE_DOUBLES * 8 <= 160 * 1024, "two workgroups per CU");
  static_assert(TPC * NXU <= LDU && 3 * NP + TPC * NXU - NP <= LDW, "nodes past Np land in the pads");
  static_assert(TPC == 16 && NP % 2 == 0 && LDU % 2 == 0 && LDW % 2 == 0, "16-byte pairs, rows of 16 lanes");
};

// The consumers' tiling of the [168 x 56] output (rows r = a Np + i, columns
// j) without padding.  Two matrix instructions run at the same flop rate:
// v_mfma_f64_16x16x4f64 (one 16 x 16 tile, lane i + 16k holds row i of A and
// column i of B for k step k) and v_mfma_f64_4x4x4f64 (four 4 x 4 blocks b,
// lane 16k + 4b + x holds row x of block b's A and column x of its B; the
// result of row i, column j of block b is in lane 16i + 4b + j).  Four kinds
// of products:
//   F(rt, cb)  16 x 16 tile, rows 16rt.., columns 16cb..      (rt < 10, cb < 3)
//   C(rt, cq)  16 x 4: block b = rows 16rt + 4b.., columns 4cq..  (cq = 12, 13)
//   R(rq, cb)  4 x 16: block b = rows 4rq.., columns 16cb + 4b..  (rq = 40, 41)
//   K          8 x 8: block b = rows 160 + 4(b >> 1).., columns 48 + 4(b & 1)..
// A C product reads the same A register as F(rt, .) and an R product the same
// B register as F(., cb), so the 168 x 56 outputs take 30 F + 20 C + 6 R + 1 K
// products with no padding, where 16-wide tiles alone execute 1.20x the useful
// products.  Consumer wave w < 3 takes F(0..8, w) and R(40, w) (592 matrix-core
// cycles per k step, 64 per F product and 16 per small one); wave 3 takes the
// C products, F(9, .), R(41, .) and K (576 cycles).
//
// Each product reads two operand slots (a slot is one row range of W or one
// column range of u, of one lane layout).  A slot's value for k step kk is
// read from LDS GD56_LEAD product cycles before its first use (at the start
// of the step at the latest), so only the values in flight are live.
struct Gd56Plan {
  static constexpr int MAXOP = 28, MAXSLOT = 20, MAXRD = 4 * MAXSLOT, MAXPOS = 4 * MAXOP + 1;
  int nop = 0, nslot = 0, nrd = 0;
  int kind[MAXOP] = {};       // 0 F, 1 C, 2 R, 3 K
  int p1[MAXOP] = {}, p2[MAXOP] = {};
  int acc[MAXOP] = {};        // accumulator index within the kind's bank (F or small)
  int sa[MAXOP] = {}, sb[MAXOP] = {};
  int nfull = 0, nsmall = 0;
  int stype[MAXSLOT] = {};    // lane layout: 0 A rows 16.., 1 B cols 16.., 2 A rows 4.., 3 B cols 4.., 4 A of K, 5 B of K
  int soff[MAXSLOT] = {};     // first row or column of the slot
  // reads in issue order: k step and slot; position = product index (over the
  // step's KST k steps) before which the read is issued
  int rd_kk[MAXRD] = {}, rd_slot[MAXRD] = {};
  int rd_begin[MAXPOS + 1] = {};  // reads issued before product n: rd_begin[n] .. rd_begin[n + 1] - 1
};

constexpr int GD56_LEAD = 320;
constexpr int gd56_cycles(int kind) { return kind == 0 ? 64 : 16; }

constexpr int gd56_slot(Gd56Plan& P, int type, int off) {
  for (int x = 0; x < P.nslot; ++x)
    if (P.stype[x] == type && P.soff[x] == off) return x;
  P.stype[P.nslot] = type;
  P.soff[P.nslot] = off;
  return P.nslot++;
}

constexpr void gd56_add(Gd56Plan& P, int kind, int p1, int p2) {
  const int o = P.nop++;
  P.kind[o] = kind;
  P.p1[o] = p1;
  P.p2[o] = p2;
  P.acc[o] = kind == 0 ? P.nfull++ : P.nsmall++;
  switch (kind) {
    case 0: P.sa[o] = gd56_slot(P, 0, 16 * p1); P.sb[o] = gd56_slot(P, 1, 16 * p2); break;
    case 1: P.sa[o] = gd56_slot(P, 0, 16 * p1); P.sb[o] = gd56_slot(P, 3, 4 * p2); break;
    case 2: P.sa[o] = gd56_slot(P, 2, 4 * p1); P.sb[o] = gd56_slot(P, 1, 16 * p2); break;
    default: P.sa[o] = gd56_slot(P, 4, 160); P.sb[o] = gd56_slot(P, 5, 48); break;
  }
}

constexpr Gd56Plan gd56_plan(int wv, int kst) {
  Gd56Plan P;
  if (wv < 3) {
    for (int rt = 0; rt < 9; ++rt) gd56_add(P, 0, rt, wv);
    gd56_add(P, 2, 40, wv);
  } else {
    for (int rt = 0; rt < 10; ++rt) {
      gd56_add(P, 1, rt, 12);
      gd56_add(P, 1, rt, 13);
      if (rt >= 7) {
        gd56_add(P, 0, 9, rt - 7);
        gd56_add(P, 2, 41, rt - 7);
      }
    }
    gd56_add(P, 3, 0, 0);
  }
  // read schedule over the step's kst k steps (products n = kk * nop + o)
  const int N = kst * P.nop;
  int pos[Gd56Plan::MAXRD] = {}, first[Gd56Plan::MAXRD] = {};
  for (int kk = 0; kk < kst; ++kk) {
    for (int x = 0; x < P.nslot; ++x) {
      int u = -1;
      for (int o = 0; o < P.nop && u < 0; ++o)
        if (P.sa[o] == x || P.sb[o] == x) u = kk * P.nop + o;
      int n = u, cyc = 0;
      while (n > 0 && cyc < GD56_LEAD) {
        --n;
        cyc += gd56_cycles(P.kind[n % P.nop]);
      }
      pos[P.nrd] = n;
      first[P.nrd] = u;
      P.rd_kk[P.nrd] = kk;
      P.rd_slot[P.nrd] = x;
      ++P.nrd;
    }
  }
  // order by position, then by first use (insertion sort)
  for (int i = 1; i < P.nrd; ++i)
    for (int j = i; j > 0 && (pos[j - 1] > pos[j] || (pos[j - 1] == pos[j] && first[j - 1] > first[j])); --j) {
      int t = pos[j]; pos[j] = pos[j - 1]; pos[j - 1] = t;
      t = first[j]; first[j] = first[j - 1]; first[j - 1] = t;
      t = P.rd_kk[j]; P.rd_kk[j] = P.rd_kk[j - 1]; P.rd_kk[j - 1] = t;
      t = P.rd_slot[j]; P.rd_slot[j] = P.rd_slot[j - 1]; P.rd_slot[j - 1] = t;
    }
  int m = 0;
  for (int n = 0; n <= N; ++n) {
    P.rd_begin[n] = m;
    while (m < P.nrd && pos[m] == n) ++m;
  }
  P.rd_begin[N + 1] = m;
  return P;
}

template <int WV>
struct Gd56Wave {
  static constexpr Gd56Plan P = gd56_plan(WV, GdSplit56::KST);
  static_assert(P.nop <= Gd56Plan::MAXOP && P.nslot <= Gd56Plan::MAXSLOT, "plan size");
  static_assert(P.nrd == GdSplit56::KST * P.nslot, "every slot read once per k step");
};

template <int I, int N, typename Fn>
__device__ __forceinline__ void gd_static_for(Fn& fn) {
  if constexpr (I < N) {
    fn(std::integral_constant<int, I>{});
    gd_static_for<I + 1, N>(fn);
  }
}

// One consumer wave: its products for every step of the range, then its part
// of the partial sum.
template <int WV>
__device__ __forceinline__ void gd56_consume(const double* __restrict__ lds, uint32_t nsteps, double* __restrict__ w,
                                             int lane) {
  using S = GdSplit56;
  using PW = Gd56Wave<WV>;
  constexpr int NP = S::NP;
  constexpr int NOP = PW::P.nop, NSLOT = PW::P.nslot, NFULL = PW::P.nfull, NSMALL = PW::P.nsmall;
  constexpr int N = S::KST * NOP;
  const int kq = lane >> 4;
  // per-lane word offset of each slot layout within a staging buffer (k step 0)
  const int lane_off[6] = {S::CH * S::LDU + kq * S::LDW + (lane & 15),
                           kq * S::LDU + (lane & 15),
                           S::CH * S::LDU + kq * S::LDW + (lane & 3),
                           kq * S::LDU + (lane & 3),
                           S::CH * S::LDU + kq * S::LDW + 4 * ((lane >> 3) & 1) + (lane & 3),
                           kq * S::LDU + 4 * ((lane >> 2) & 1) + (lane & 3)};
  f64x4 accf[NFULL > 0 ? NFULL : 1];
  double accs[NSMALL > 0 ? NSMALL : 1];
#pragma unroll
  for (int t = 0; t < NFULL; ++t) accf[t] = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int t = 0; t < NSMALL; ++t) accs[t] = 0.0;
  __syncthreads();
  for (uint32_t r = 0; r < nsteps; ++r) {
    const double* buf = lds + (int)(r & 1u) * S::STAGE_DOUBLES;
    double v[S::KST][NSLOT];
    auto product = [&](auto nc) __attribute__((always_inline)) {
      constexpr int n = decltype(nc)::value;
      // the reads placed before product n (all of them, for n == N)
      constexpr int rb = PW::P.rd_begin[n], re = PW::P.rd_begin[n + 1];
      auto read = [&](auto ic) __attribute__((always_inline)) {
        constexpr int m = rb + decltype(ic)::value;
        constexpr int kk = PW::P.rd_kk[m], x = PW::P.rd_slot[m];
        constexpr int ty = PW::P.stype[x];
        constexpr int ld = (ty == 0 || ty == 2 || ty == 4) ? S::LDW : S::LDU;
        v[kk][x] = buf[lane_off[ty] + 4 * kk * ld + PW::P.soff[x]];
      };
      gd_static_for<0, re - rb>(read);
      if constexpr (re > rb) __builtin_amdgcn_sched_group_barrier(0x100, re - rb, 0);
      if constexpr (n < N) {
        constexpr int kk = n / NOP, o = n % NOP;
        constexpr int a = PW::P.sa[o], b = PW::P.sb[o], t = PW::P.acc[o];
        if constexpr (PW::P.kind[o] == 0)
          accf[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(v[kk][a], v[kk][b], accf[t], 0, 0, 0);
        else
          accs[t] = __builtin_amdgcn_mfma_f64_4x4x4f64(v[kk][a], v[kk][b], accs[t], 0, 0, 0);
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
      }
    };
    gd_static_for<0, N + 1>(product);
    __builtin_amdgcn_sched_barrier(0);
    __syncthreads();  // the producers have staged step r + 1; buffer r % 2 is free
  }
  // partial sums: output row and column of each product's results
#pragma unroll
  for (int o = 0; o < NOP; ++o) {
    const int kind = PW::P.kind[o], p1 = PW::P.p1[o], p2 = PW::P.p2[o], t = PW::P.acc[o];
    const int b = (lane >> 2) & 3;
    if (kind == 0) {
#pragma unroll
      for (int q = 0; q < 4; ++q) w[(int64_t)(16 * p1 + 4 * q + kq) * NP + 16 * p2 + (lane & 15)] = accf[t][q];
    } else if (kind == 1) {
      w[(int64_t)(16 * p1 + 4 * b + kq) * NP + 4 * p2 + (lane & 3)] = accs[t];
    } else if (kind == 2) {
      w[(int64_t)(4 * p1 + kq) * NP + 16 * p2 + (lane & 15)] = accs[t];
    } else {
      w[(int64_t)(160 + 4 * (b >> 1) + kq) * NP + 48 + 4 * (b & 1) + (lane & 3)] = accs[t];
    }
  }
}

__global__ __launch_bounds__(GdSplit56::NTH) __attribute__((amdgpu_waves_per_eu(4, 8)))
void gd_split56_kernel(GdArgs p) {
  using S = GdSplit56;
  constexpr int NP = S::NP;
  constexpr int CH = S::CH;
  constexpr int SUB = GD_UNIT / CH;
  __shared__ __attribute__((aligned(16))) double lds[2 * S::STAGE_DOUBLES];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const uint32_t wave = __builtin_amdgcn_readfirstlane((uint32_t)tid >> 6);
  const uint32_t part = blockIdx.x;
  if (part >= p.npart) return;
  const uint32_t st_begin = (uint32_t)((uint64_t)part * p.nunits / p.npart) * SUB;
  const uint32_t st_end = (uint32_t)((uint64_t)(part + 1) * p.nunits / p.npart) * SUB;
  const uint32_t nsteps = st_end - st_begin;


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
    // nodes 2 (rr + 16 h) and the next one, as one 16-byte access per plane
#pragma unroll
    for (int h = 0; h < S::NPR; ++h) {
      const uint32_t off = (uint32_t)(cc * NP + 2 * (rr + S::TPC * h)) * 8u;
      const WordVec<double, 2> x = buffer_load_vec<double, 2>(bu, off);
      const WordVec<double, 2> y0 = buffer_load_vec<double, 2>(b0, off);
      const WordVec<double, 2> y1 = buffer_load_vec<double, 2>(b1, off);
      const WordVec<double, 2> y2 = buffer_load_vec<double, 2>(b2, off);
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        ru[d][2 * h + e] = x.v[e];
        rg0[d][2 * h + e] = y0.v[e];
        rg1[d][2 * h + e] = y1.v[e];
        rg2[d][2 * h + e] = y2.v[e];
      }
    }
  };
  // The 9 geometric factors of a column's element: lane rr of the column's
  // 16-lane row loads factor rr, and a row broadcast (DPP) hands each factor
  // to the whole row, instead of 16 lanes loading the same 72 bytes.
  double gv = 0.0;
  auto load_g = [&](uint32_t r) __attribute__((always_inline)) {
    const uint32_t c0 = (st_begin + r) * CH;
    const uint32_t ncl = r < nsteps && c0 < p.ncols ? min((uint32_t)CH, p.ncols - c0) : 0u;
    const uint32_t k0 = ncl ? c0 / p.F : 0u;
    const uint32_t nk = ncl ? (c0 + ncl - 1) / p.F - k0 + 1 : 0u;
    const __amdgpu_buffer_rsrc_t bg = buffer_range(p.G + (int64_t)k0 * 9, nk * 72u);
    const uint32_t ke = (c0 + (uint32_t)cc) / p.F - k0;  // this lane's element within the step
    gv = buffer_load_f64(bg, (ke * 9u + (uint32_t)min(rr, 8)) * 8u);
  };
  auto bcast_g = [&]() __attribute__((always_inline)) {
    rG[0] = row_bcast_f64<0>(gv);
    rG[1] = row_bcast_f64<1>(gv);
    rG[2] = row_bcast_f64<2>(gv);
    rG[3] = row_bcast_f64<3>(gv);
    rG[4] = row_bcast_f64<4>(gv);
    rG[5] = row_bcast_f64<5>(gv);
    rG[6] = row_bcast_f64<6>(gv);
    rG[7] = row_bcast_f64<7>(gv);
    rG[8] = row_bcast_f64<8>(gv);
  };
  auto stage = [&](int d, int b) __attribute__((always_inline)) {
    double* ul = lds + b * S::STAGE_DOUBLES;
    double* wl = ul + CH * S::LDU;
    bcast_g();
    // A node past Np (the last pair of some threads) is written to the pads
    // (u columns Np.., W rows 3 Np..), which no product reads: the writes need
    // no branch, so the waits for the loads stay exact.
#pragma unroll
    for (int h = 0; h < S::NPR; ++h) {
      const int i = 2 * (rr + S::TPC * h);
      const bool in = i < NP;
      *reinterpret_cast<f64x2*>(ul + cc * S::LDU + i) = f64x2{ru[d][2 * h], ru[d][2 * h + 1]};
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        f64x2 wv;
#pragma unroll
        for (int e = 0; e < 2; ++e)
          wv[e] = rG[3 * a] * rg0[d][2 * h + e] + rG[3 * a + 1] * rg1[d][2 * h + e] + rG[3 * a + 2] * rg2[d][2 * h + e];
        *reinterpret_cast<f64x2*>(wl + cc * S::LDW + (in ? a * NP + i : 3 * NP + i - NP)) = wv;
      }
    }
  };
  // Each role runs its own loop (so that the consumers' accumulators and the
  // producers' register sets are never live together), with the same barriers:
  // one after the prologue, one per step.  Step r sits in producer register set
  // r % DEPTH and staging buffer r % 2 (DEPTH = 2: both alternate with r).
  if (consumer) {
    double* w = p.work + (int64_t)part * 3 * NP * NP;
    switch (wave) {
      case 0: gd56_consume<0>(lds, nsteps, w, lane); break;
      case 1: gd56_consume<1>(lds, nsteps, w, lane); break;
      case 2: gd56_consume<2>(lds, nsteps, w, lane); break;
      default: gd56_consume<3>(lds, nsteps, w, lane); break;
    }
  } else {
    static_assert(S::DEPTH == 2, "register sets alternate with the step");
    // The producers' vector work (FP64 multiply-adds, loads) shares the SIMDs
    // with the consumers' matrix products, and every step waits for it at the
    // barrier: issue it first (measured: 4 % faster).
    __builtin_amdgcn_s_setprio(3);
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
    // (nsteps is a whole number of partition units, so even: the pair of
    // iterations needs no guard, and the waits for the loads stay exact)
    static_assert(SUB % 2 == 0, "steps come in pairs");
    for (uint32_t r0 = 0; r0 < nsteps; r0 += 2) {
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const uint32_t r = r0 + j;
        stage(j ^ 1, j ^ 1);
        load_g(r + 2);
        load_ug(r + 3, j ^ 1);
        __syncthreads();
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
