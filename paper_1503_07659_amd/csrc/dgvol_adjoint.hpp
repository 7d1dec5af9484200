// Adjoint kernels of the DG volume derivative (reverse mode w.r.t. u and G).
//
//   W_a[i]      = sum_b G[3a+b] gout_b[i]
//   gu[j]       = sum_a sum_i D[a][i][j] W_a[i]          (transposed product)
//   gG[3a+b]    = sum_{f,i} gout_b[i] (D_a u)[i]          (D u recomputed)
#pragma once

#include "dgvol_device.hpp"

namespace dgvol {

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
  constexpr bool DLDS = 3 * NP * NP * 8 <= 96 * 1024;
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
      // chunks in a loop, not unrolled: unrolled, the chunks' operands and W
      // slots overflow the registers (kilobytes of spill at Np = 84)
#pragma unroll 1
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
        for (int xx = 0; xx < 4; ++xx) {
          const int tau = 4 * ch + xx;
          if (tau < Sh::TRIP) {
            double R[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
              const int loc = 3 * xx + a;
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
              W[3 * xx + a] = gk[3 * a] * go[0] + gk[3 * a + 1] * go[1] + gk[3 * a + 2] * go[2];
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

// Staged adjoint kernel (Np <= 56, F <= 16).
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
  return adj_table_rows<NP>() * WAVE * 8 + WPB * 16 * (NP + 1) * 8 + 2 * WPB * 16 * 9 * 8;
}

template <int NP, int WPB>
__global__ __launch_bounds__(WAVE* WPB) __attribute__((amdgpu_waves_per_eu(2, 8))) void adj_f64_staged_kernel(
    const double* __restrict__ D, const double* __restrict__ G, const double* __restrict__ u,
    const double* __restrict__ gout, double* __restrict__ gu, double* __restrict__ gG, uint32_t K, uint32_t F,
    int64_t plane, uint32_t E, uint32_t ntiles) {
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
  static_assert(adj_staged_lds<NP, WPB>() <= 160 * 1024, "LDS budget");
  for (int e = threadIdx.x; e < NTAB; e += WAVE * WPB) {
    const int row = e >> 6, l = e & 63;
    afr[row * WAVE + tswz(l, row % KS)] = e < NFRAG ? afrag_f64<NP>(D, row / KS, row % KS, l) : 0.0;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int n = lane & 15, g = lane >> 4;
  const uint32_t wave = threadIdx.x >> 6;
  double* stg = stg_all + wave * 16 * LD;
  double* red = red_all + wave * 16 * 9;
  double* gks = gks_all + wave * 16 * 9;  // geometric factors of the tile's (at most 16) elements
  // per-lane LDS offsets: forward rows by s & 3, transposed rows by sp & 3
  int fo[4], tb[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    fo[r] = tswz(lane, r);
    tb[r] = (n >> 2) * WAVE + tswz(16 * (n & 3) + 4 * r + g, n >> 2);
  }
  const uint32_t stride = gridDim.x * WPB;
  uint32_t t = blockIdx.x * WPB + wave;
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
  auto load_raw = [&](uint32_t tt) __attribute__((always_inline)) {
    const uint32_t kk0 = tt * E;
    if constexpr (BUF) {
      const bool any = tt < ntiles;
      const uint32_t ne = any ? min(E, K - kk0) : 0u;
      const __amdgpu_buffer_rsrc_t ru = buffer_range(any ? u + (int64_t)kk0 * F * NP : u, ne * F * NP * 8u);
#pragma unroll
      for (int q = 0; q < NRAW; ++q) raw[q] = buffer_load_f64(ru, (uint32_t)(lane + WAVE * q) * 8u);
      const __amdgpu_buffer_rsrc_t rg = buffer_range(any ? G + (int64_t)kk0 * 9 : G, ne * 9 * 8u);
#pragma unroll
      for (int q = 0; q < NGR; ++q) graw[q] = buffer_load_f64(rg, (uint32_t)(lane + WAVE * q) * 8u);
    } else {
      if (tt >= ntiles) return;
      const uint32_t ne = min(E, K - kk0);
      const double* __restrict__ src = u + (int64_t)kk0 * F * NP;
      const int cnt = (int)(ne * F) * NP;
#pragma unroll
      for (int q = 0; q < NRAW; ++q) {
        const int x = lane + WAVE * q;
        const double v = src[min(x, cnt - 1)];
        raw[q] = x < cnt ? v : 0.0;
      }
      const double* __restrict__ gsrc = G + (int64_t)kk0 * 9;
#pragma unroll
      for (int q = 0; q < NGR; ++q) {
        const int x = lane + WAVE * q;
        graw[q] = x < (int)ne * 9 ? gsrc[x] : 0.0;
      }
    }
  };
  load_raw(t);
  for (; t < ntiles; t += stride) {
    const uint32_t k0 = t * E;
    const uint32_t ne = min(E, K - k0);
    const uint32_t ncolt = ne * F;
    const int cnt = (int)ncolt * NP;
    const uint32_t col0 = k0 * F;
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
    const uint32_t e = valid ? (uint32_t)n / F : 0u;
    const uint32_t col = col0 + (valid ? n : 0);
    const double* ge = gks + e * 9;  // geometric factors of this column's element
    const double* __restrict__ goc = gout + (int64_t)col * NP;
    f64x4 accj[Sh::MTJ];
#pragma unroll
    for (int tj = 0; tj < Sh::MTJ; ++tj) accj[tj] = f64x4{0.0, 0.0, 0.0, 0.0};
    double P[9];
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
        for (int bb = 0; bb < 3; ++bb) gor[x][bb] = 4 * ch + x < Sh::TRIP ? goc[bb * plane + min(i, NP - 1)] : 0.0;
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
          if (T < Sh::MT)
            acc[tt] = __builtin_amdgcn_mfma_f64_16x16x4f64(afr[(T * KS + s) * WAVE + fo[s & 3]], b, acc[tt], 0, 0, 0);
        }
        __builtin_amdgcn_sched_barrier(0);
      }
      double go[4][3];
#pragma unroll
      for (int x = 0; x < 4; ++x) {
        const bool ok = valid && 4 * (4 * ch + x) + g < NP;
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
      auto top = [&](int sp, int tj) { return afr[((sp >> 2) * KS + 4 * tj) * WAVE + tb[sp & 3]]; };
      double tc[Sh::MTJ], tn[Sh::MTJ];
#pragma unroll
      for (int tj = 0; tj < Sh::MTJ; ++tj) tc[tj] = top(12 * ch, tj);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int sl = 0; sl < 12; ++sl) {
        const int sp = 12 * ch + sl;
        if (sp < Sh::SLOTS) {
          const bool more = sl + 1 < 12 && sp + 1 < Sh::SLOTS;
#pragma unroll
          for (int tj = 0; tj < Sh::MTJ; ++tj) {
            if (more) tn[tj] = top(sp + 1, tj);
            accj[tj] = __builtin_amdgcn_mfma_f64_16x16x4f64(tc[tj], wv[sl], accj[tj], 0, 0, 0);
          }
#pragma unroll
          for (int tj = 0; tj < Sh::MTJ; ++tj) {
            __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
            __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
          }
          __builtin_amdgcn_sched_barrier(0);
#pragma unroll
          for (int tj = 0; tj < Sh::MTJ; ++tj) tc[tj] = tn[tj];
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
    // gG: four lane groups, then the F columns of each element, in a fixed order
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
    if (g == 0 && (uint32_t)n < ne) {
#pragma unroll
      for (int c = 0; c < 9; ++c) {
        double sacc = 0.0;
        for (uint32_t f = 0; f < F; ++f) sacc += red[(n * F + f) * 9 + c];
        gG[(int64_t)(k0 + n) * 9 + c] = sacc;
      }
    }
    wave_sync();
    load_raw(t + stride);
  }
}

}  // namespace dgvol
