// Adjoint at the high orders (Np = 84, 120) in two chunk-register passes.
//
// At these orders D (170-345 KB in FP64) does not fit in LDS, so the single
// staged adjoint cannot hold its operand table.  As in the forward
// chunk-register body, the 8 waves of a workgroup each keep a share of D in
// registers for the whole launch, and the workgroup stages the columns it
// works on in LDS:
//
//   pass A (gu):  gu[c][j] = sum_{a,i} D[a][i][j] W_a[c][i],
//                 W_a[c][i] = sum_b G[k][3a+b] gout_b[c][i]   (k = c / F).
//     Wave w < ceil(Np/16) owns output rows j = 16w..16w+15 and keeps the A
//     operands of the transposed product (k = slot sp: direction sp % 3,
//     nodes 4 (sp/3) + lane group) for all 3 ceil(Np/4) k-steps (at Np = 84,
//     whose 6 tiles leave two waves spare, the spare waves take the last
//     k-steps of three tiles each).  Per 16
//     columns the workgroup forms W from gout and G (each thread stages a fixed
//     column, so it needs one element's geometric factors) into LDS, each wave
//     runs its k-steps, and gu leaves through an LDS tile as contiguous runs.
//   pass B (gG):  gG[k][3a+b] = sum_f sum_i gout_b[c][i] (D_a u)[c][i].
//     Wave w < NCH keeps the A operands of output chunk w (3 tiles, as the
//     forward chunk-register body; at Np = 84, 4 tiles in 4-wave workgroups),
//     recomputes D u for the chunk's slots from u staged in LDS, and reduces
//     it with gout at its lanes' nodes (at most 4 node triples).  Each
//     workgroup owns a run of whole elements and takes its columns as full
//     16-column tiles (whole-element tiles left 1 of 16 columns idle at F = 3);
//     an element that continues past a tile carries its partial sum into the
//     next one, so every element's sums finish inside one workgroup.  The
//     partial sums are added in a fixed order (lane groups, then waves, then
//     the element's columns in order), so gG is reproducible bit for bit.
//     The loop takes one barrier per tile: the u stage and the partial sums
//     are double-buffered, a tile's final sums are formed while the next
//     tile's products run, and u and gout are requested one tile ahead.
//
// gout is read twice (once per pass), u once; the matrix work equals the
// single-pass adjoint's.
#pragma once

#include <type_traits>

#include "dgvol_device.hpp"
#include "dgvol_layout.hpp"

namespace dgvol {

constexpr int ADJCR_WPB = 8;

// fn(integral_constant<I>), ..., fn(integral_constant<N - 1>), unrolled at compile time
template <int I, int N, typename Fn>
__device__ __forceinline__ void adjcr_static_for(Fn&& fn) {
  if constexpr (I < N) {
    fn(std::integral_constant<int, I>{});
    adjcr_static_for<I + 1, N>(fn);
  }
}

// ------------------------------------------------------------------ pass A: gu

template <int NP>
struct AdjCrA {
  static constexpr int NTH = WAVE * ADJCR_WPB;
  static constexpr int KT = Shape<NP>::SLOTS;         // k-steps (slots) of the transposed product
  static constexpr int MTJ = Shape<NP>::MTJ;          // output tiles (waves with work)
  static constexpr int LDW = 3 * NP + 1;              // odd row stride of the W stage
  static constexpr int TPC = NTH / 16;                // threads staging one column
  static constexpr int NX = (NP + TPC - 1) / TPC;     // nodes per thread
  static_assert(MTJ <= ADJCR_WPB, "one wave per output tile");
  // Np = 84 has 6 output tiles for 8 waves.  There each owner wave runs the
  // first KA k-steps of its tile, and the two spare waves run the last KB
  // k-steps of three tiles each into a second partial, so every SIMD carries
  // about the same number of products.
  static constexpr bool SPLIT = MTJ == 6 && ADJCR_WPB == 8;
  static constexpr int KA = SPLIT ? 48 : KT;
  static constexpr int KB = KT - KA;
  // at Np = 120 the last KL k-steps' operands wait in LDS, not registers
  static constexpr int KL = NP == 120 ? 12 : 0;
  static constexpr int KR = KA - KL;
  static_assert(!SPLIT || 3 * KB <= KA, "a helper wave's operands fit the owner's array");
};

template <int NP>
__global__ __launch_bounds__(WAVE* ADJCR_WPB) void adjcr_gu_kernel(const double* __restrict__ D,
                                                                  const double* __restrict__ G,
                                                                  const double* __restrict__ gout,
                                                                  double* __restrict__ gu, uint32_t ncols, uint32_t F,
                                                                  int64_t plane, uint32_t ntiles) {
  using S = AdjCrA<NP>;
  __shared__ double ws[16 * S::LDW];  // W[c][a Np + i]
  __shared__ double ostg[16 * NP];    // gu tile, column-major runs
  __shared__ double ostg2[S::SPLIT ? 16 * NP : 1];  // the helper waves' partial
  __shared__ double atl[S::KL ? ADJCR_WPB * S::KL * WAVE : 1];  // operand tail, per wave and lane
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int n = lane & 15, g = lane >> 4;
  const int w = tid >> 6;
  const bool mma = w < S::MTJ;
  const bool helper = S::SPLIT && !mma;
  const int hw = helper ? w - S::MTJ : 0;  // helper index: tiles 3 hw .. 3 hw + 2
  double areg[S::KA];
#pragma unroll
  for (int sp = 0; sp < S::KA; ++sp) {
    double a = 0.0;
    if (mma)
      a = afragT_f64<NP>(D, w, sp, lane);
    else if (helper && sp < 3 * S::KB)
      a = afragT_f64<NP>(D, 3 * hw + sp / S::KB, S::KA + sp % S::KB, lane);
    if (sp < S::KR)
      areg[sp] = a;
    else
      atl[(w * S::KL + sp - S::KR) * WAVE + lane] = a;  // read back by this lane only
  }

  // staging: thread (cc, rr) owns column cc of the tile and nodes rr + TPC x
  const int cc = tid / S::TPC, rr = tid % S::TPC;
  double r0[S::NX], r1[S::NX], r2[S::NX], rG[9];
  // Loads are unconditional, so the compiler's waits count exactly the
  // memory operations in flight: gout moves through one buffer range per
  // plane over the tile's columns (zero past it, and for padding nodes), G
  // from a clamped column (a tile past the end rereads the last one).
  auto load = [&](uint32_t t) __attribute__((always_inline)) {
    const uint32_t col = min(t * 16 + cc, ncols - 1);
    const uint32_t gbytes = min(16u, ncols - t * 16) * NP * 8u;
    __amdgpu_buffer_rsrc_t rgo[3];
#pragma unroll
    for (int b = 0; b < 3; ++b) rgo[b] = buffer_range(gout + b * plane + (int64_t)t * 16 * NP, gbytes);
#pragma unroll
    for (int x = 0; x < S::NX; ++x) {
      const int i = rr + S::TPC * x;
      const uint32_t off = i < NP ? (uint32_t)(cc * NP + i) * 8u : gbytes;
      r0[x] = buffer_load_f64(rgo[0], off);
      r1[x] = buffer_load_f64(rgo[1], off);
      r2[x] = buffer_load_f64(rgo[2], off);
    }
    const int64_t gb = (int64_t)(col / F) * 9;
#pragma unroll
    for (int m = 0; m < 9; ++m) rG[m] = G[gb + m];
  };
  // W of the loaded tile into the stage; done at the end of an iteration, after
  // its stores, so the wait for the loads does not cover those stores
  auto stage = [&]() __attribute__((always_inline)) {
#pragma unroll
    for (int x = 0; x < S::NX; ++x) {
      const int i = rr + S::TPC * x;
      if (i < NP) {
#pragma unroll
        for (int a = 0; a < 3; ++a)
          ws[cc * S::LDW + a * NP + i] = rG[3 * a] * r0[x] + rG[3 * a + 1] * r1[x] + rG[3 * a + 2] * r2[x];
      }
    }
  };
  constexpr int NST = (16 * NP + S::NTH - 1) / S::NTH;  // gu words stored per thread
  uint32_t t = blockIdx.x;
  load(min(t, ntiles - 1));
  stage();
  for (; t < ntiles; t += gridDim.x) {
    const uint32_t col0 = t * 16;
    const int cnt = (int)min(16u, ncols - col0) * NP;
    __syncthreads();
    load(min(t + gridDim.x, ntiles - 1));
    if (mma) {
      f64x4 acc = f64x4{0.0, 0.0, 0.0, 0.0};
      auto bval = [&](int sp) __attribute__((always_inline)) {
        const int i = 4 * (sp / 3) + g;
        const double v = ws[n * S::LDW + (sp % 3) * NP + min(i, NP - 1)];
        return i < NP ? v : 0.0;
      };
      double bcur = bval(0);
#pragma unroll
      for (int sp = 0; sp < S::KA; ++sp) {
        const double bnxt = sp + 1 < S::KA ? bval(sp + 1) : 0.0;
        const double a = sp < S::KR ? areg[sp] : atl[(w * S::KL + sp - S::KR) * WAVE + lane];
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bcur, acc, 0, 0, 0);
        bcur = bnxt;
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int j = 16 * w + 4 * q + g;
        if (j < NP) ostg[n * NP + j] = acc[q];
      }
    }
    if constexpr (S::SPLIT) {
      if (helper) {
        f64x4 acc[3];
#pragma unroll
        for (int r = 0; r < 3; ++r) acc[r] = f64x4{0.0, 0.0, 0.0, 0.0};
        auto bval = [&](int sp) __attribute__((always_inline)) {
          const int i = 4 * (sp / 3) + g;
          const double v = ws[n * S::LDW + (sp % 3) * NP + min(i, NP - 1)];
          return i < NP ? v : 0.0;
        };
        double bcur = bval(S::KA);
#pragma unroll
        for (int s2 = 0; s2 < S::KB; ++s2) {
          const double bnxt = s2 + 1 < S::KB ? bval(S::KA + s2 + 1) : 0.0;
#pragma unroll
          for (int r = 0; r < 3; ++r)
            acc[r] = __builtin_amdgcn_mfma_f64_16x16x4f64(areg[r * S::KB + s2], bcur, acc[r], 0, 0, 0);
          bcur = bnxt;
        }
#pragma unroll
        for (int r = 0; r < 3; ++r) {
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int j = 16 * (3 * hw + r) + 4 * q + g;
            if (j < NP) ostg2[n * NP + j] = acc[r][q];
          }
        }
      }
    }
    __syncthreads();
    const __amdgpu_buffer_rsrc_t ro = buffer_range(gu + (int64_t)col0 * NP, (uint32_t)cnt * 8u);
#pragma unroll
    for (int q = 0; q < NST; ++q) {
      const int x = tid + S::NTH * q;
      const int xc = min(x, 16 * NP - 1);
      if constexpr (S::SPLIT)
        buffer_store_f64(ro, (uint32_t)x * 8u, ostg[xc] + ostg2[xc]);
      else
        buffer_store_f64(ro, (uint32_t)x * 8u, ostg[xc]);
    }
    stage();
  }
}

// ------------------------------------------------------------------ pass B: gG

template <int NP>
struct AdjCrB {
  // Waves per workgroup and tiles per output chunk.  Np = 120: 8 waves of
  // 3-tile chunks (4 whole node triples per lane).  Np = 84: 4 waves of
  // 4-tile chunks, two workgroups per CU.  The two workgroups keep their own
  // barriers, so one's epilogue and barrier wait run beside the other's
  // products, where one 8-wave workgroup (2-tile chunks) left each SIMD's
  // matrix unit idle while both its waves finished a tile; and each tile's
  // shuffles and partial sums are shared by 4 waves, not 8.  (One tile for
  // each of 16 waves measured 8 % slower than 8 waves: twice the epilogue.)
  // The pass only sums gout * (D u) over nodes, so a chunk need not hold
  // whole triples.
  static constexpr int WPB = NP == 84 ? 4 : ADJCR_WPB;
  static constexpr int NTH = WAVE * WPB;
  static constexpr int KS = Shape<NP>::KS64;
  static constexpr int LD = NP + 1;                    // odd row stride of the u stage
  static constexpr int NLD = (16 * NP + NTH - 1) / NTH;
  static constexpr int TPC = NP == 84 ? 4 : 3;
  static constexpr int NCH = (Shape<NP>::MT + TPC - 1) / TPC;  // chunks (waves with work)
  static constexpr int SPC = 4 * TPC;                         // slots per chunk
  static constexpr int NTRI = SPC % 3 == 0 ? SPC / 3 : (SPC + 4) / 3;  // node triples a chunk touches
  static_assert(NCH <= WPB, "one wave per output chunk");
  // A operands kept in LDS instead of registers: the last KL k-steps of the
  // chunk's last tile and the last KL2 of the one before it (at Np = 84 the
  // whole last tile and 3 more, which fills two workgroups' 160 KiB)
  static constexpr int KL = NP == 120 ? 12 : (NP == 84 ? KS : 0);
  static constexpr int KR = KS - KL;
  static constexpr int KL2 = NP == 84 ? 3 : 0;
  static constexpr int KR2 = KS - KL2;
  static constexpr int NAT = KL + KL2;  // operands per lane in LDS
  static_assert(TPC >= 2 || KL2 == 0, "a second tile to take the tail from");
  // tiles of u and gout in flight (register sets): the registers hold one
  static constexpr int DEPTH = 1;
  // waves per SIMD the register budget must allow (two workgroups per CU at Np = 84)
  static constexpr int MINW = 2;
  static constexpr bool ALLW = NCH == WPB;  // every wave has a chunk
};

template <int NP>
__global__ __launch_bounds__(AdjCrB<NP>::NTH)
__attribute__((amdgpu_waves_per_eu(AdjCrB<NP>::MINW, 8))) void adjcr_gG_kernel(const double* __restrict__ D,
                                                                  const double* __restrict__ u,
                                                                  const double* __restrict__ gout,
                                                                  double* __restrict__ gG, uint32_t K, uint32_t F,
                                                                  int64_t plane) {
  using Sh = Shape<NP>;
  using S = AdjCrB<NP>;
  // double-buffered by tile parity: tile t's products read us[t & 1] and
  // write red[t & 1] while u of tile t + 1 is staged into the other buffer
  // and tile t - 1's sums are read from the other red, so one barrier per
  // tile separates every write from its reads
  __shared__ double us[2][16 * S::LD];
  __shared__ double red[2][S::WPB][16][9];  // per tile parity, wave and column
  __shared__ double cry[2][9];  // partial gG of an element continued in the next tile (slot by tile parity)
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int n = lane & 15, g = lane >> 4;
  const int w = tid >> 6;
  const bool mma = w < S::NCH;
  const int ch = mma ? w : 0;
  const int tau0 = S::SPC * ch / 3;  // first node triple of the chunk
  const int r0 = S::SPC * ch % 3;    // its first slot's direction
  __shared__ double atl[S::NAT ? S::WPB * S::NAT * WAVE : 1];  // operand tails, per wave and lane
  // where operand (tile tt of the chunk, k-step s) lives: -1 in registers, else its LDS slot
  auto tail_slot = [](int tt, int s) constexpr {
    return (tt == S::TPC - 1 && s >= S::KR) ? s - S::KR : (tt == S::TPC - 2 && s >= S::KR2) ? S::KL + s - S::KR2 : -1;
  };
  double areg[S::TPC][S::KS];
#pragma unroll
  for (int tt = 0; tt < S::TPC; ++tt) {
    const int T = S::TPC * ch + tt;
#pragma unroll
    for (int s = 0; s < S::KS; ++s) {
      const double a = (mma && T < Sh::MT) ? afrag_f64<NP>(D, T, s, lane) : 0.0;
      if (tail_slot(tt, s) < 0)
        areg[tt][s] = a;
      else
        atl[(w * S::NAT + tail_slot(tt, s)) * WAVE + lane] = a;  // read back by this lane only
    }
  }
  // this workgroup's run of elements [e_lo, e_hi), columns [c_lo, c_hi),
  // tiles 0 .. nrun - 1 of 16 columns from c_lo
  const uint32_t e_lo = (uint32_t)((uint64_t)blockIdx.x * K / gridDim.x);
  const uint32_t e_hi = (uint32_t)((uint64_t)(blockIdx.x + 1) * K / gridDim.x);
  const uint32_t c_lo = e_lo * F, c_hi = e_hi * F;
  const uint32_t nrun = (c_hi - c_lo + 15u) / 16u;
  // u and gout move through buffer ranges (32-bit offsets, zero past the
  // range, empty past the last tile), which frees the address registers of
  // the clamped 64-bit form
  // tile tt's u and gout wait in register set tt % DEPTH
  double ur[S::DEPTH][S::NLD];
  auto load_u = [&](uint32_t tt, auto R) __attribute__((always_inline)) {
    constexpr int r = decltype(R)::value;
    const bool any = tt < nrun;
    const uint32_t c0 = any ? c_lo + 16u * tt : 0u;
    const uint32_t cnt = any ? min(16u, c_hi - c0) * NP : 0u;
    const __amdgpu_buffer_rsrc_t ru = buffer_range(u + (int64_t)c0 * NP, cnt * 8u);
#pragma unroll
    for (int q = 0; q < S::NLD; ++q) ur[r][q] = buffer_load_f64(ru, (uint32_t)(tid + S::NTH * q) * 8u);
  };
  auto stage = [&](uint32_t b, auto R) __attribute__((always_inline)) {
    constexpr int r = decltype(R)::value;
#pragma unroll
    for (int q = 0; q < S::NLD; ++q) {
      const int x = tid + S::NTH * q;
      if (x < 16 * NP) us[b][(x / NP) * S::LD + (x % NP)] = ur[r][q];
    }
  };
  // this lane's gout values of a tile, requested a tile ahead of their use
  // (unconditional loads; padding nodes and columns past the tile read the
  // range's end, which loads zero)
  double go[S::DEPTH][S::NTRI][3];
  auto load_go = [&](uint32_t tt, auto R) __attribute__((always_inline)) {
    constexpr int r = decltype(R)::value;
    const bool any = tt < nrun;
    const uint32_t c0 = any ? c_lo + 16u * tt : 0u;
    const uint32_t gbytes = any ? min(16u, c_hi - c0) * NP * 8u : 0u;
    __amdgpu_buffer_rsrc_t rgo[3];
#pragma unroll
    for (int bb = 0; bb < 3; ++bb) rgo[bb] = buffer_range(gout + bb * plane + (int64_t)c0 * NP, gbytes);
#pragma unroll
    for (int x = 0; x < S::NTRI; ++x) {
      const int i = 4 * (tau0 + x) + g;
      const uint32_t off = (tau0 + x < Sh::TRIP && i < NP) ? (uint32_t)(n * NP + i) * 8u : gbytes;
#pragma unroll
      for (int bb = 0; bb < 3; ++bb) go[r][x][bb] = buffer_load_f64(rgo[bb], off);
    }
  };
  // products of tile tt and this wave's partial sums into red[tt & 1]
  auto work = [&](uint32_t tt, auto R) __attribute__((always_inline)) {
    constexpr int r = decltype(R)::value;
    const double* ub = us[tt & 1u];
    f64x4 acc[S::TPC];
#pragma unroll
    for (int k = 0; k < S::TPC; ++k) acc[k] = f64x4{0.0, 0.0, 0.0, 0.0};
    auto bval = [&](int s) __attribute__((always_inline)) {
      const int j = 4 * s + g;
      const double v = ub[n * S::LD + min(j, NP - 1)];
      return j < NP ? v : 0.0;
    };
    double bcur = bval(0);
#pragma unroll
    for (int s = 0; s < S::KS; ++s) {
      const double bnxt = s + 1 < S::KS ? bval(s + 1) : 0.0;
#pragma unroll
      for (int k = 0; k < S::TPC; ++k) {
        const double a = tail_slot(k, s) < 0 ? areg[k][s] : atl[(w * S::NAT + tail_slot(k, s)) * WAVE + lane];
        acc[k] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bcur, acc[k], 0, 0, 0);
      }
      bcur = bnxt;
    }
    // P[3a+b] = sum over this lane's nodes of gout_b * (D_a u)
    double P[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) P[c] = 0.0;
    // slot l of the chunk: direction (r0 + l) % 3 of its triple (r0 + l) / 3,
    // with r0 (wave-uniform) made a compile-time constant per branch.  Slots
    // past the last one need no test: their A rows and their gout (a triple
    // past the last node) are zero, so they add +0 to P, which leaves it as it is.
    auto accumulate = [&](auto R0) __attribute__((always_inline)) {
      constexpr int rr = decltype(R0)::value;
#pragma unroll
      for (int l = 0; l < S::SPC; ++l) {
        const int a = (rr + l) % 3, x = (rr + l) / 3;
        const double R = acc[l >> 2][l & 3];
        P[3 * a] += go[r][x][0] * R;
        P[3 * a + 1] += go[r][x][1] * R;
        P[3 * a + 2] += go[r][x][2] * R;
      }
    };
    if (S::SPC % 3 == 0 || r0 == 0)  // 3-tile chunks start on a whole triple
      accumulate(std::integral_constant<int, 0>{});
    else if (r0 == 1)
      accumulate(std::integral_constant<int, 1>{});
    else
      accumulate(std::integral_constant<int, 2>{});
#pragma unroll
    for (int c = 0; c < 9; ++c) {
      P[c] += __shfl_xor(P[c], 16);
      P[c] += __shfl_xor(P[c], 32);
    }
    if (g == 0) {
#pragma unroll
      for (int c = 0; c < 9; ++c) red[tt & 1u][w][n][c] = P[c];
    }
  };
  // output (j, c) of tile tt: element k0 + j, factor c: its columns in the tile in order,
  // each summed over the waves in order, after the partial sum carried from the previous
  // tile when the element began there; written when the element ends in this tile, else
  // carried into the next (slot by tile parity: the slot read was written one barrier
  // earlier, the slot written is read one barrier later)
  // The waves take turns (tile tt's outputs start at wave tt % WPB), so that
  // no SIMD carries every tile's sums.
  auto reduce = [&](uint32_t tt) __attribute__((always_inline)) {
    const uint32_t c0 = c_lo + 16u * tt;
    const uint32_t nc = min(16u, c_hi - c0);
    const uint32_t k0 = c0 / F;
    const uint32_t ne = (c0 + nc - 1u) / F - k0 + 1u;
    const uint32_t o = (uint32_t)(tid - WAVE * (int)(tt % S::WPB)) % (uint32_t)S::NTH;  // output index
    if (o < ne * 9) {
      const uint32_t j = o / 9u;
      const int c = (int)(o % 9u);
      const uint32_t ke = k0 + j;
      const uint32_t lo = max(ke * F, c0) - c0, hi = min((ke + 1u) * F, c0 + nc) - c0;
      double s = (j == 0 && ke * F < c0) ? cry[tt & 1u][c] : 0.0;
      for (uint32_t m = lo; m < hi; ++m) {
        double sw = 0.0;
        for (int ww = 0; ww < S::NCH; ++ww) sw += red[tt & 1u][ww][m][c];
        s += sw;
      }
      if ((ke + 1u) * F <= c0 + nc)
        gG[(int64_t)ke * 9 + c] = s;
      else
        cry[(tt + 1u) & 1u][c] = s;
    }
  };
  using I0 = std::integral_constant<int, 0>;
  load_u(0, I0{});
  stage(0, I0{});
  adjcr_static_for<0, S::DEPTH>([&](auto J) {
    constexpr int j = decltype(J)::value;
    load_u(j + 1, std::integral_constant<int, (j + 1) % S::DEPTH>{});
    if (S::ALLW || mma) load_go(j, J);
  });
  __syncthreads();
  // tile t: reduce tile t - 1, products of t, stage u of t + 1; after the barrier request
  // u of t + 1 + DEPTH and gout of t + DEPTH.  The loop runs whole rounds of DEPTH tiles; a
  // tile past the run reads zeros and is not reduced.
  auto step = [&](uint32_t t, auto P) __attribute__((always_inline)) {
    constexpr int p = decltype(P)::value;
    using N1 = std::integral_constant<int, (p + 1) % S::DEPTH>;
    if (t - 1u < nrun) reduce(t - 1u);
    if (S::ALLW || mma) work(t, P);
    stage((t + 1u) & 1u, N1{});
    __syncthreads();
    load_u(t + 1u + S::DEPTH, N1{});
    if (S::ALLW || mma) load_go(t + S::DEPTH, P);
  };
  for (uint32_t t = 0; t < nrun; t += S::DEPTH)
    adjcr_static_for<0, S::DEPTH>([&](auto P) { step(t + decltype(P)::value, P); });
  if (nrun > 0 && nrun % S::DEPTH == 0) reduce(nrun - 1);
}

}  // namespace dgvol
