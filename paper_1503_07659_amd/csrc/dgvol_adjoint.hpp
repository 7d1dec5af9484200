// Adjoint kernels of the DG volume derivative (reverse mode w.r.t. u and G).
//
//   W_a[i]      = sum_b G[3a+b] gout_b[i]
//   gu[j]       = sum_a sum_i D[a][i][j] W_a[i]          (transposed product)
//   gG[3a+b]    = sum_{f,i} gout_b[i] (D_a u)[i]          (D u recomputed)
#pragma once

#include "dgvol_device.hpp"

namespace dgvol {

// ------------------------------------------------------------------ adjoint FP64 (Np <= 56)
//
// Each wave owns a contiguous run of whole elements and takes its columns as
// full 16-column tiles (only the run's last tile can be short), so no product
// column is idle: whole-element tiles left 1 of 16 columns idle at F = 3 and
// 12 of 32 at F = 20.  An element that continues past a tile carries its
// partial gG sum into the next one, so every element's gG sums finish in one
// wave, in a fixed order, with no cross-wave reduction.  Per tile and chunk
// of 4 node triples: recompute R = D u (forward
// fragments), read gout at the lane's nodes, accumulate gG partials, form
// W = G^T gout lane-locally, then feed the 12 W slots straight in as the B
// operand of the transposed product D^T W (the slot order of W is the k order
// of that product), accumulated over chunks.
//
// The A table of the forward product is stored in LDS with an XOR swizzle
// (entry `lane` of row (T, s) sits at lane ^ ((s & 3) << 2)).  The forward
// product reads its row as a permutation (conflict-free); the transposed
// product D^T W reads the same table: the entry it needs for lane (m, kk),
// output tile TJ and slot sp is row ((sp>>2) KS + 4 TJ + (m>>2)), column
// (16 (m&3) + 4 (sp&3) + kk) ^ ((m>>2) << 2), i.e. a per-lane base (one of four,
// by sp & 3) plus a compile-time offset, with at most two lanes per bank.
// u comes in and gu goes out through the wave's LDS tile buffer as contiguous
// runs; gout is read at each lane's own nodes, one chunk ahead of its use.
template <int NP>
constexpr int adj_table_rows() {
  // the transposed product reads rows up to ((SLOTS - 1) / 4) KS + 4 MTJ - 1 (rows past
  // the forward table belong to output nodes j >= Np, whose results are discarded)
  using Sh = Shape<NP>;
  constexpr int need = ((Sh::SLOTS - 1) / 4) * Sh::KS64 + 4 * Sh::MTJ;
  return need > Sh::MT * Sh::KS64 ? need : Sh::MT * Sh::KS64;
}

template <int NP, int WPB>
constexpr int adj_staged_lds() {
  return adj_table_rows<NP>() * WAVE * 8 + WPB * 16 * (NP + 1) * 8 + 2 * WPB * 16 * 9 * 8 + WPB * 9 * 8;
}

template <int NP, int WPB>
__global__ __launch_bounds__(WAVE* WPB) __attribute__((amdgpu_waves_per_eu(2, 8))) void adj_f64_staged_kernel(
    const double* __restrict__ D, const double* __restrict__ G, const double* __restrict__ u,
    const double* __restrict__ gout, double* __restrict__ gu, double* __restrict__ gG, uint32_t K, uint32_t F,
    int64_t plane) {
  using Sh = Shape<NP>;
  constexpr int KS = Sh::KS64;
  constexpr int NFRAG = fwd_table_doubles<NP>();
  constexpr int NTAB = adj_table_rows<NP>() * WAVE;
  constexpr int LD = NP + 1;  // odd row stride of the tile buffer: B-operand reads spread over banks
  constexpr int TILE = 16 * NP;
  constexpr int NRAW = (TILE + WAVE - 1) / WAVE;
  __shared__ double afr[NTAB];
  __shared__ double stg_all[WPB * 16 * LD];
  __shared__ double red_all[WPB * 16 * 9];
  __shared__ double gks_all[WPB * 16 * 9];
  __shared__ double cry_all[WPB * 9];  // partial gG of an element continued in the next tile
  static_assert(adj_staged_lds<NP, WPB>() <= 160 * 1024, "LDS budget");
  for (int e = threadIdx.x; e < NTAB; e += WAVE * WPB) {
    const int row = e >> 6, l = e & 63;
    afr[row * WAVE + tswz(l, row % KS)] = e < NFRAG ? afrag_f64<NP>(D, row / KS, row % KS, l) : 0.0;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int n = lane & 15, g = lane >> 4;
  // wave-uniform (readfirstlane): the tile index and the buffer descriptors built
  // from it then live in scalar registers; a per-lane index makes the compiler
  // wrap every buffer access in a loop over the distinct descriptors
  const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  double* stg = stg_all + wave * 16 * LD;
  double* red = red_all + wave * 16 * 9;
  double* gks = gks_all + wave * 16 * 9;  // geometric factors of the tile's (at most 16) elements
  double* cry = cry_all + wave * 9;
  // per-lane LDS offsets: forward rows by s & 3, transposed rows by sp & 3
  int fo[4], tb[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    fo[r] = tswz(lane, r);
    tb[r] = (n >> 2) * WAVE + tswz(16 * (n & 3) + 4 * r + g, n >> 2);
  }
  // The last 16-row tile of either product, when at most two of its row
  // quads are real rows (slot quads of the forward product, output nodes of
  // the transposed one), runs as one v_mfma_f64_4x4x4f64 per real quad r
  // instead of one padded 16 x 16 product.  Block b of that instruction
  // takes rows 4r.. and columns 4b.. of the tile: its A operand is row 4r + x
  // of the tile's fragment (x = lane & 3, k = lane >> 4), its B operand is the
  // 16 x 16 product's B register unchanged, and its result lands where
  // component r of the 16 x 16 accumulator would.  Under the table's swizzle
  // the A entry sits at a per-lane base (fs, ts) plus a constant 4 (r ^ s).
  constexpr int FQ = Sh::SLOTS - 4 * (Sh::MT - 1);    // real row quads of the last forward tile
  constexpr int JQ = (NP - 16 * (Sh::MTJ - 1) + 3) / 4;  // real row quads of the last transposed tile
  constexpr bool FSPLIT = FQ <= 2, JSPLIT = JQ <= 2;
  constexpr int MTJF = JSPLIT ? Sh::MTJ - 1 : Sh::MTJ;  // transposed tiles run as 16 x 16 products
  const int fs = 16 * g + ((lane & 3) ^ g);
  const int ts = 16 * (lane & 3) + (g ^ (lane & 3));
  const uint32_t stride = gridDim.x * WPB;
  // this wave's run of elements [e_lo, e_hi), columns [c_lo, c_hi), tiles
  // 0 .. nrun - 1 of 16 columns from c_lo
  const uint32_t gw = blockIdx.x * WPB + wave;
  const uint32_t e_lo = (uint32_t)((uint64_t)gw * K / stride);
  const uint32_t e_hi = (uint32_t)((uint64_t)(gw + 1) * K / stride);
  const uint32_t c_lo = e_lo * F, c_hi = e_hi * F;
  const uint32_t nrun = (c_hi - c_lo + 15u) / 16u;
  uint32_t t = 0;
  // first column, valid columns, first element and element count of tile tt
  struct TileCols {
    uint32_t col0, ncol, k0, ne;
  };
  auto tile_cols = [&](uint32_t tt) __attribute__((always_inline)) {
    TileCols c;
    c.col0 = c_lo + 16u * tt;
    c.ncol = tt < nrun ? min(16u, c_hi - c.col0) : 0u;
    c.k0 = c.col0 / F;
    c.ne = c.ncol ? (c.col0 + c.ncol - 1u) / F - c.k0 + 1u : 0u;
    return c;
  };
  // u of the tile and the geometric factors of its elements (one contiguous
  // run of G), loaded one tile ahead
  constexpr int NGR = (16 * 9 + WAVE - 1) / WAVE;
  double raw[NRAW], graw[NGR];
  // At Np = 56 the kernel sits at the register limit; there u, G and gu move
  // through buffer ranges (past the range: zero loads, dropped stores; empty
  // past the last tile), so no branch surrounds a memory operation.  The
  // compiler then allocates without spilling (measured -15 %).  At the lower
  // orders the guarded form measured 1-4 % faster.
  constexpr bool BUF = NP >= 56;
  // the u run of tile tt and the geometric factors of its elements
  auto load_raw = [&](uint32_t tt) __attribute__((always_inline)) {
    const TileCols tc = tile_cols(tt);
    if constexpr (BUF) {
      const bool any = tc.ncol > 0;
      const __amdgpu_buffer_rsrc_t ru = buffer_range(any ? u + (int64_t)tc.col0 * NP : u, tc.ncol * NP * 8u);
#pragma unroll
      for (int q = 0; q < NRAW; ++q) raw[q] = buffer_load_f64(ru, (uint32_t)(lane + WAVE * q) * 8u);
      const __amdgpu_buffer_rsrc_t rg = buffer_range(any ? G + (int64_t)tc.k0 * 9 : G, tc.ne * 9 * 8u);
#pragma unroll
      for (int q = 0; q < NGR; ++q) graw[q] = buffer_load_f64(rg, (uint32_t)(lane + WAVE * q) * 8u);
    } else {
      if (tc.ncol == 0) return;
      const double* __restrict__ src = u + (int64_t)tc.col0 * NP;
      const int cnt = (int)tc.ncol * NP;
#pragma unroll
      for (int q = 0; q < NRAW; ++q) {
        const int x = lane + WAVE * q;
        const double v = src[min(x, cnt - 1)];
        raw[q] = x < cnt ? v : 0.0;
      }
      const double* __restrict__ gsrc = G + (int64_t)tc.k0 * 9;
#pragma unroll
      for (int q = 0; q < NGR; ++q) {
        const int x = lane + WAVE * q;
        graw[q] = x < (int)tc.ne * 9 ? gsrc[x] : 0.0;
      }
    }
  };
  // gG partial sums of the lane's column in the tile
  double P[9];
  load_raw(t);
  const float invF = 1.0f / (float)F;
  while (t < nrun) {
    const TileCols tcur = tile_cols(t);
    const uint32_t k0 = tcur.k0, ne = tcur.ne, ncolt = tcur.ncol, col0 = tcur.col0;
    const int cnt = (int)ncolt * NP;
#pragma unroll
    for (int q = 0; q < NRAW; ++q) {
      const int x = lane + WAVE * q;
      if (NRAW * WAVE == TILE || x < TILE) stg[(x / NP) * LD + (x % NP)] = raw[q];
    }
#pragma unroll
    for (int q = 0; q < NGR; ++q) {
      const int x = lane + WAVE * q;
      if (x < 16 * 9) gks[x] = graw[q];
    }
    wave_sync();
    const bool valid = (uint32_t)n < ncolt;
    // element of this lane's column within the tile: (col0 mod F + n) / F, exact in
    // float for these small integers (the + 0.5 keeps a whole quotient off its edge)
    const uint32_t e = valid ? (uint32_t)(((float)(col0 - k0 * F + (uint32_t)n) + 0.5f) * invF) : 0u;
    const uint32_t col = col0 + (valid ? n : 0);
    const double* ge = gks + e * 9;  // geometric factors of this column's element
    const double* __restrict__ goc = gout + (int64_t)col * NP;
    // (buffer form) the three gout planes of the tile's valid columns
    static_assert(!BUF || NP == 4 * Sh::TRIP, "every node of a lane group is a real node");
    __amdgpu_buffer_rsrc_t rgo[3];
    if constexpr (BUF) {
#pragma unroll
      for (int bb = 0; bb < 3; ++bb) rgo[bb] = buffer_range(gout + bb * plane + (int64_t)col0 * NP, ncolt * NP * 8u);
    }
    f64x4 accj[Sh::MTJ];
#pragma unroll
    for (int tj = 0; tj < Sh::MTJ; ++tj) accj[tj] = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int c = 0; c < 9; ++c) P[c] = 0.0;
#pragma unroll
    for (int ch = 0; ch < Sh::NCHUNK; ++ch) {
      // this lane's gout values for the chunk, requested before the forward
      // product (clamped addresses: unconditional loads); zeroed outside only
      // where they are used, after the product, so the wait for them does not
      // land in its first k-step
      double gor[4][3];
#pragma unroll
      for (int x = 0; x < 4; ++x) {
        const int i = 4 * (4 * ch + x) + g;
#pragma unroll
        for (int bb = 0; bb < 3; ++bb) {
          if constexpr (BUF)  // columns past the tile read zero; i < Np (Np = 4 TRIP)
            gor[x][bb] = 4 * ch + x < Sh::TRIP ? buffer_load_f64(rgo[bb], (uint32_t)(n * NP + i) * 8u) : 0.0;
          else
            gor[x][bb] = 4 * ch + x < Sh::TRIP ? goc[bb * plane + min(i, NP - 1)] : 0.0;
        }
      }
      __builtin_amdgcn_sched_barrier(0);
      f64x4 acc[3];
#pragma unroll
      for (int tt = 0; tt < 3; ++tt) acc[tt] = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int s = 0; s < KS; ++s) {
        const int j = 4 * s + g;
        const double bv = stg[n * LD + min(j, NP - 1)];
        const double b = j < NP ? bv : 0.0;
#pragma unroll
        for (int tt = 0; tt < 3; ++tt) {
          const int T = 3 * ch + tt;
          if (FSPLIT && T == Sh::MT - 1) {
#pragma unroll
            for (int r = 0; r < FQ; ++r)
              acc[tt][r] = __builtin_amdgcn_mfma_f64_4x4x4f64(afr[(T * KS + s) * WAVE + fs + 4 * (r ^ (s & 3))], b,
                                                              acc[tt][r], 0, 0, 0);
          } else if (T < Sh::MT) {
            acc[tt] = __builtin_amdgcn_mfma_f64_16x16x4f64(afr[(T * KS + s) * WAVE + fo[s & 3]], b, acc[tt], 0, 0, 0);
          }
        }
        __builtin_amdgcn_sched_barrier(0);
      }
      double go[4][3];
#pragma unroll
      for (int x = 0; x < 4; ++x) {
        const bool ok = BUF || (valid && 4 * (4 * ch + x) + g < NP);
#pragma unroll
        for (int bb = 0; bb < 3; ++bb) go[x][bb] = ok ? gor[x][bb] : 0.0;
      }
#pragma unroll
      for (int x = 0; x < 4; ++x) {
        const int tau = 4 * ch + x;
        if (tau < Sh::TRIP) {
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            const int loc = 3 * x + a;
            const double R = acc[loc >> 2][loc & 3];
#pragma unroll
            for (int bb = 0; bb < 3; ++bb) P[3 * a + bb] += go[x][bb] * R;
          }
        }
      }
      // W of the chunk's 12 slots at once, then the transposed product with its
      // operands read one slot ahead (one read after each product)
      double wv[12];
      {
        double gl[9];
#pragma unroll
        for (int c = 0; c < 9; ++c) gl[c] = ge[c];
#pragma unroll
        for (int sl = 0; sl < 12; ++sl) {
          const int x = sl / 3, a = sl % 3;
          wv[sl] = gl[3 * a] * go[x][0] + gl[3 * a + 1] * go[x][1] + gl[3 * a + 2] * go[x][2];
        }
      }
      // operand o of slot sp: 16 x 16 tiles tj = o < MTJF, then the 4 x 4 quads of the last tile
      constexpr int NJO = MTJF + (JSPLIT ? JQ : 0);
      auto top = [&](int sp, int o) {
        if (o < MTJF) return afr[((sp >> 2) * KS + 4 * o) * WAVE + tb[sp & 3]];
        const int r = o - MTJF;
        return afr[((sp >> 2) * KS + 4 * (Sh::MTJ - 1) + r) * WAVE + ts + 4 * ((sp & 3) ^ r)];
      };
      double tc[NJO], tn[NJO];
#pragma unroll
      for (int o = 0; o < NJO; ++o) tc[o] = top(12 * ch, o);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int sl = 0; sl < 12; ++sl) {
        const int sp = 12 * ch + sl;
        if (sp < Sh::SLOTS) {
          const bool more = sl + 1 < 12 && sp + 1 < Sh::SLOTS;
#pragma unroll
          for (int o = 0; o < NJO; ++o) {
            if (more) tn[o] = top(sp + 1, o);
            if (o < MTJF) {
              accj[o] = __builtin_amdgcn_mfma_f64_16x16x4f64(tc[o], wv[sl], accj[o], 0, 0, 0);
            } else {
              const int r = o - MTJF;
              accj[Sh::MTJ - 1][r] = __builtin_amdgcn_mfma_f64_4x4x4f64(tc[o], wv[sl], accj[Sh::MTJ - 1][r], 0, 0, 0);
            }
          }
#pragma unroll
          for (int o = 0; o < NJO; ++o) {
            __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
            __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
          }
          __builtin_amdgcn_sched_barrier(0);
#pragma unroll
          for (int o = 0; o < NJO; ++o) tc[o] = tn[o];
        }
      }
    }
    // gu through the tile buffer (after every lane's last B-operand read)
    wave_sync();
#pragma unroll
    for (int tj = 0; tj < Sh::MTJ; ++tj) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int j = 16 * tj + 4 * q + g;
        if (16 * tj + 16 <= NP || j < NP) stg[n * LD + min(j, NP - 1)] = accj[tj][q];
      }
    }
    wave_sync();
    if constexpr (BUF) {
      const __amdgpu_buffer_rsrc_t rgu = buffer_range(gu + (int64_t)col0 * NP, (uint32_t)cnt * 8u);
#pragma unroll
      for (int q = 0; q < NRAW; ++q) {
        const int x = lane + WAVE * q;
        const int xc = min(x, TILE - 1);
        buffer_store_f64(rgu, (uint32_t)x * 8u, stg[(xc / NP) * LD + (xc % NP)]);
      }
    } else {
      double* __restrict__ gdst = gu + (int64_t)col0 * NP;
#pragma unroll
      for (int q = 0; q < NRAW; ++q) {
        const int x = lane + WAVE * q;
        if (x < cnt) gdst[x] = stg[(x / NP) * LD + (x % NP)];
      }
    }
    // gG: four lane groups, then the columns of each element, in a fixed order
#pragma unroll
    for (int c = 0; c < 9; ++c) {
      P[c] += __shfl_xor(P[c], 16);
      P[c] += __shfl_xor(P[c], 32);
    }
    if (g == 0) {
#pragma unroll
      for (int c = 0; c < 9; ++c) red[n * 9 + c] = P[c];
    }
    wave_sync();
    {
      // lane j < ne: element k0 + j, over its columns in this tile in order, after the
      // partial sum carried from the previous tile when the element began there;
      // written when it ends here, else carried into the next tile (a tile that both
      // takes and passes on a carry holds one element, lane 0: it reads the carry
      // before the sync below and writes it after)
      const uint32_t ke = k0 + (uint32_t)n;
      const bool mine = g == 0 && (uint32_t)n < ne;
      const uint32_t cb = mine ? max(ke * F, col0) - col0 : 0u;
      const uint32_t ce = mine ? min((ke + 1u) * F, col0 + ncolt) - col0 : 0u;
      const bool from_prev = mine && n == 0 && ke * F < col0;
      const bool ends = (ke + 1u) * F <= col0 + ncolt;
      double sacc[9];
#pragma unroll
      for (int c = 0; c < 9; ++c) sacc[c] = from_prev ? cry[c] : 0.0;
      for (uint32_t cc = cb; cc < ce; ++cc) {
#pragma unroll
        for (int c = 0; c < 9; ++c) sacc[c] += red[cc * 9 + c];
      }
      wave_sync();  // every lane has read the previous carry
      if (mine) {
#pragma unroll
        for (int c = 0; c < 9; ++c) {
          if (ends)
            gG[(int64_t)ke * 9 + c] = sacc[c];
          else
            cry[c] = sacc[c];
        }
      }
    }
    wave_sync();
    ++t;
    load_raw(t);
  }
}

}  // namespace dgvol
