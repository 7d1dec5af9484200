// Split-BF16 forward bodies (FP32 storage, three BF16 matrix-core passes,
// FP32 accumulation): the same data-movement schemes as the FP64 bodies in
// dgvol_forward.hpp, with FP32 words.
#pragma once

#include "dgvol_device.hpp"
#include "dgvol_forward.hpp"

namespace dgvol {

// ------------------------------------------------------------------ split-BF16 staged
//
// FP32 words; u is split into hi/lo BF16 in registers after the LDS pick-up, D
// once when its table is built (or on the fly when the table does not fit).
// Three BF16 MFMAs per (tile, k-step), cross terms first, FP32 accumulation.

template <int NP>
constexpr bool bf16_table_fits() { return bf16_table_entries<NP>() * 32 <= 96 * 1024; }

// Tiles per wave iteration of the split-BF16 staged body (TPI), by default:
// FP32 words halve the bytes of a tile, so more tiles per iteration than in
// FP64 are needed to keep enough bytes in flight.  Other counts are
// instantiated as tuning variants.
template <int NP>
constexpr int f32s_tpi() { return NP <= 4 ? 8 : (NP <= 20 ? 4 : (NP <= 35 ? 2 : 1)); }

template <int NP, int TPI>
constexpr int f32s_wave_floats() {
  return TPI * 16 * NP + (TPI > 1 ? TPI * 16 * 9 : 0);
}

template <int NP, int WPB, int TPI>
constexpr int fwd_f32s_staged_lds() {
  return (bf16_table_fits<NP>() ? 2 * bf16_table_entries<NP>() * 16 : 0) + WPB * f32s_wave_floats<NP, TPI>() * 4;
}

// u, out and every plane start 8-byte aligned: the staged split-BF16 body then
// moves pairs of floats (512-byte runs per instruction, as the FP64 body does).
__host__ __device__ inline bool f32_pairs_ok(const FwdArgs<float>& p) {
  return (((uintptr_t)p.u | (uintptr_t)p.out) % 8 == 0) && (p.plane % 2 == 0);
}

template <int NP, int WPB>
__device__ __forceinline__ void fwd_f32s_staged_single(const FwdArgs<float>& p, uint32_t bid, uint32_t nblk,
                                                       char* lds) {
  using Sh = Shape<NP>;
  constexpr bool ALDS = bf16_table_fits<NP>();
  constexpr int NTE = ALDS ? bf16_table_entries<NP>() : 0;
  constexpr int TILE = 16 * NP;  // even
  constexpr int NRAW = (TILE + WAVE - 1) / WAVE;
  constexpr int NPAIR = (TILE / 2 + WAVE - 1) / WAVE;
  constexpr int NREG = NRAW > 2 * NPAIR ? NRAW : 2 * NPAIR;
  Bf16x8Bits* ahi = reinterpret_cast<Bf16x8Bits*>(lds);
  Bf16x8Bits* alo = ahi + NTE;
  float* stg_all = reinterpret_cast<float*>(lds + 2 * NTE * 16);
  if constexpr (ALDS) {
    for (int e = threadIdx.x; e < NTE; e += WAVE * WPB) {
      const int ts = e >> 6;
      Bf16x8Bits h, l;
      afrag_bf16<NP>(p.D, ts / Sh::KS16, ts % Sh::KS16, e & 63, h, l);
      ahi[e] = h;
      alo[e] = l;
    }
    __syncthreads();
  }
  const bool pairs = f32_pairs_ok(p);
  const int lane = threadIdx.x & 63;
  const int n = lane & 15, g = lane >> 4;
  const uint32_t wave = threadIdx.x >> 6;
  float* stg = stg_all + wave * TILE;
  const uint32_t stride = nblk * WPB;
  uint32_t t = bid * WPB + wave;
  float raw[NREG];
  // a whole tile moves as pairs; a partial last tile word by word
  auto load_raw = [&](uint32_t tt) __attribute__((always_inline)) {
    const float* __restrict__ src = p.u + (int64_t)tt * TILE;
    const int cnt = (int)min(16u, p.ncols - tt * 16) * NP;
    if (pairs && cnt == TILE) {
#pragma unroll
      for (int q = 0; q < NPAIR; ++q) {
        const int x = lane + WAVE * q;
        if (x < TILE / 2) {
          const f32x2 v = reinterpret_cast<const f32x2*>(src)[x];
          raw[2 * q] = v[0];
          raw[2 * q + 1] = v[1];
        }
      }
    } else {
#pragma unroll
      for (int q = 0; q < NREG; ++q) {
        const int x = lane + WAVE * q;
        raw[q] = x < cnt ? src[x] : 0.0f;
      }
    }
  };
  if (t < p.ntiles) load_raw(t);
  for (; t < p.ntiles; t += stride) {
    const uint32_t col0 = t * 16;
    const int cnt = (int)min(16u, p.ncols - col0) * NP;
    const bool whole = pairs && cnt == TILE;
    if (whole) {
#pragma unroll
      for (int q = 0; q < NPAIR; ++q) {
        const int x = lane + WAVE * q;
        if (x < TILE / 2) reinterpret_cast<f32x2*>(stg)[x] = f32x2{raw[2 * q], raw[2 * q + 1]};
      }
    } else {
#pragma unroll
      for (int q = 0; q < NRAW; ++q) {
        const int x = lane + WAVE * q;
        if (x < TILE) stg[x] = raw[q];
      }
    }
    wave_sync();
    Bf16x8Bits bh[Sh::KS16], bl[Sh::KS16];
#pragma unroll
    for (int s = 0; s < Sh::KS16; ++s) {
#pragma unroll
      for (int e = 0; e < 8; e += 2) {
        const int j = 32 * s + 8 * g + e;
        split_bf16_pair(j < NP ? stg[n * NP + j] : 0.0f, j + 1 < NP ? stg[n * NP + j + 1] : 0.0f, bh[s], bl[s], e);
      }
    }
    const uint32_t col = col0 + n;
    const bool valid = col < p.ncols;
    const uint32_t k = valid ? col / p.F : 0u;
    float gk[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) gk[c] = valid ? p.G[(int64_t)k * 9 + c] : 0.0f;
    wave_sync();
    f32x4 acc[Sh::MT];
#pragma unroll
    for (int T = 0; T < Sh::MT; ++T) acc[T] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < Sh::KS16; ++s) {
#pragma unroll
      for (int T = 0; T < Sh::MT; ++T) {
        Bf16x8Bits ah, al;
        if constexpr (ALDS) {
          ah = ahi[(T * Sh::KS16 + s) * WAVE + lane];
          al = alo[(T * Sh::KS16 + s) * WAVE + lane];
        } else {
          afrag_bf16<NP>(p.D, T, s, lane, ah, al);
        }
        acc[T] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(al), as_bf16x8(bh[s]), acc[T], 0, 0, 0);
        acc[T] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(ah), as_bf16x8(bl[s]), acc[T], 0, 0, 0);
        acc[T] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(ah), as_bf16x8(bh[s]), acc[T], 0, 0, 0);
        __builtin_amdgcn_sched_barrier(0);
      }
    }
#pragma unroll
    for (int bb = 0; bb < 3; ++bb) {
#pragma unroll
      for (int tau = 0; tau < Sh::TRIP; ++tau) {
        const int i = 4 * tau + g;
        const int s0 = 3 * tau;
        const float v = gk[bb] * acc[s0 >> 2][s0 & 3] + gk[3 + bb] * acc[(s0 + 1) >> 2][(s0 + 1) & 3] +
                        gk[6 + bb] * acc[(s0 + 2) >> 2][(s0 + 2) & 3];
        if (i < NP) stg[n * NP + i] = v;
      }
      wave_sync();
      float* __restrict__ ob = p.out + bb * p.plane + (int64_t)col0 * NP;
      if (whole) {
#pragma unroll
        for (int q = 0; q < NPAIR; ++q) {
          const int x = lane + WAVE * q;
          if (x < TILE / 2) store_stream(&reinterpret_cast<f32x2*>(ob)[x], reinterpret_cast<const f32x2*>(stg)[x]);
        }
      } else {
#pragma unroll
        for (int q = 0; q < NRAW; ++q) {
          const int x = lane + WAVE * q;
          if (x < cnt) store_stream(&ob[x], stg[x]);
        }
      }
      wave_sync();
    }
    if (t + stride < p.ntiles) load_raw(t + stride);
  }
}

// Several tiles per iteration (FP32 words; see fwd_f64_staged_multi): a wave
// takes TPI consecutive tiles, one contiguous run of u and of each plane (moved
// as float pairs when aligned), and the geometric factors of their elements
// as one run.
template <int NP, int WPB, int TPI>
__device__ __forceinline__ void fwd_f32s_staged_multi(const FwdArgs<float>& p, uint32_t bid, uint32_t nblk,
                                                      char* lds) {
  using Sh = Shape<NP>;
  constexpr bool ALDS = bf16_table_fits<NP>();
  constexpr int NTE = ALDS ? bf16_table_entries<NP>() : 0;
  constexpr int TILE = 16 * NP;
  constexpr int RUN = TPI * TILE;  // even
  constexpr int NRAW = (RUN + WAVE - 1) / WAVE;
  constexpr int NPAIR = (RUN / 2 + WAVE - 1) / WAVE;
  constexpr int NREG = NRAW > 2 * NPAIR ? NRAW : 2 * NPAIR;
  constexpr int GW = TPI * 16 * 9;
  constexpr int NGR = (GW + WAVE - 1) / WAVE;
  Bf16x8Bits* ahi = reinterpret_cast<Bf16x8Bits*>(lds);
  Bf16x8Bits* alo = ahi + NTE;
  if constexpr (ALDS) {
    for (int e = threadIdx.x; e < NTE; e += WAVE * WPB) {
      const int ts = e >> 6;
      Bf16x8Bits h, l;
      afrag_bf16<NP>(p.D, ts / Sh::KS16, ts % Sh::KS16, e & 63, h, l);
      ahi[e] = h;
      alo[e] = l;
    }
    __syncthreads();
  }
  const bool pairs = f32_pairs_ok(p);
  const int lane = threadIdx.x & 63;
  const int n = lane & 15, g = lane >> 4;
  const uint32_t wave = threadIdx.x >> 6;
  float* su = reinterpret_cast<float*>(lds + 2 * NTE * 16) + wave * f32s_wave_floats<NP, TPI>();
  float* sg = su + RUN;
  const uint32_t nrun = (p.ntiles + TPI - 1) / TPI;
  const uint32_t stride = nblk * WPB;
  uint32_t t = bid * WPB + wave;
  float raw[NREG], graw[NGR];
  auto run_elems = [&](uint32_t tt, uint32_t& e0, int& ng) __attribute__((always_inline)) {
    const uint32_t c0 = tt * (16 * TPI);
    const uint32_t c1 = min(c0 + 16 * TPI, p.ncols) - 1;
    e0 = c0 / p.F;
    ng = (int)(c1 / p.F - e0 + 1) * 9;
  };
  auto load_run = [&](uint32_t tt) __attribute__((always_inline)) {
    const uint32_t c0 = tt * (16 * TPI);
    const float* __restrict__ src = p.u + (int64_t)c0 * NP;
    const int cnt = (int)min(16u * TPI, p.ncols - c0) * NP;
    if (pairs && cnt == RUN) {
#pragma unroll
      for (int q = 0; q < NPAIR; ++q) {
        const int x = lane + WAVE * q;
        if (x < RUN / 2) {
          const f32x2 v = reinterpret_cast<const f32x2*>(src)[x];
          raw[2 * q] = v[0];
          raw[2 * q + 1] = v[1];
        }
      }
    } else {
#pragma unroll
      for (int q = 0; q < NREG; ++q) {
        const int x = lane + WAVE * q;
        raw[q] = x < cnt ? src[x] : 0.0f;
      }
    }
    uint32_t e0;
    int ng;
    run_elems(tt, e0, ng);
    const float* __restrict__ gsrc = p.G + (int64_t)e0 * 9;
#pragma unroll
    for (int q = 0; q < NGR; ++q) {
      const int x = lane + WAVE * q;
      graw[q] = x < ng ? gsrc[x] : 0.0f;
    }
  };
  if (t < nrun) load_run(t);
  for (; t < nrun; t += stride) {
    const uint32_t col0 = t * (16 * TPI);
    const int cnt = (int)min(16u * TPI, p.ncols - col0) * NP;
    const bool whole = pairs && cnt == RUN;
    uint32_t e0;
    int ng;
    run_elems(t, e0, ng);
    if (whole) {
#pragma unroll
      for (int q = 0; q < NPAIR; ++q) {
        const int x = lane + WAVE * q;
        if (x < RUN / 2) reinterpret_cast<f32x2*>(su)[x] = f32x2{raw[2 * q], raw[2 * q + 1]};
      }
    } else {
#pragma unroll
      for (int q = 0; q < NRAW; ++q) {
        const int x = lane + WAVE * q;
        if (x < RUN) su[x] = raw[q];
      }
    }
#pragma unroll
    for (int q = 0; q < NGR; ++q) {
      const int x = lane + WAVE * q;
      if (x < GW) sg[x] = graw[q];
    }
    wave_sync();
    f32x4 acc[TPI][Sh::MT];
#pragma unroll
    for (int r = 0; r < TPI; ++r) {
#pragma unroll
      for (int T = 0; T < Sh::MT; ++T) acc[r][T] = f32x4{0.f, 0.f, 0.f, 0.f};
    }
    // one k-step at a time: the B halves of every tile, then each A fragment
    // read once for all TPI tiles
#pragma unroll
    for (int s = 0; s < Sh::KS16; ++s) {
      Bf16x8Bits bh[TPI], bl[TPI];
#pragma unroll
      for (int r = 0; r < TPI; ++r) {
#pragma unroll
        for (int e = 0; e < 8; e += 2) {
          const int j = 32 * s + 8 * g + e;
          split_bf16_pair(j < NP ? su[r * TILE + n * NP + j] : 0.0f, j + 1 < NP ? su[r * TILE + n * NP + j + 1] : 0.0f,
                          bh[r], bl[r], e);
        }
      }
#pragma unroll
      for (int T = 0; T < Sh::MT; ++T) {
        Bf16x8Bits ah, al;
        if constexpr (ALDS) {
          ah = ahi[(T * Sh::KS16 + s) * WAVE + lane];
          al = alo[(T * Sh::KS16 + s) * WAVE + lane];
        } else {
          afrag_bf16<NP>(p.D, T, s, lane, ah, al);
        }
#pragma unroll
        for (int r = 0; r < TPI; ++r) {
          acc[r][T] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(al), as_bf16x8(bh[r]), acc[r][T], 0, 0, 0);
          acc[r][T] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(ah), as_bf16x8(bl[r]), acc[r][T], 0, 0, 0);
          acc[r][T] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(ah), as_bf16x8(bh[r]), acc[r][T], 0, 0, 0);
        }
        __builtin_amdgcn_sched_barrier(0);
      }
    }
    wave_sync();
    if (t + stride < nrun) load_run(t + stride);
#pragma unroll
    for (int bb = 0; bb < 3; ++bb) {
#pragma unroll
      for (int r = 0; r < TPI; ++r) {
        const uint32_t col = col0 + 16 * r + n;
        const int ge = col < p.ncols ? (int)(col / p.F - e0) * 9 : 0;
        const float g0 = sg[ge + bb], g1 = sg[ge + 3 + bb], g2 = sg[ge + 6 + bb];
#pragma unroll
        for (int tau = 0; tau < Sh::TRIP; ++tau) {
          const int i = 4 * tau + g;
          const int s0 = 3 * tau;
          const float v = g0 * acc[r][s0 >> 2][s0 & 3] + g1 * acc[r][(s0 + 1) >> 2][(s0 + 1) & 3] +
                          g2 * acc[r][(s0 + 2) >> 2][(s0 + 2) & 3];
          if (i < NP) su[r * TILE + n * NP + i] = v;
        }
      }
      wave_sync();
      float* __restrict__ ob = p.out + bb * p.plane + (int64_t)col0 * NP;
      if (whole) {
#pragma unroll
        for (int q = 0; q < NPAIR; ++q) {
          const int x = lane + WAVE * q;
          if (x < RUN / 2) store_stream(&reinterpret_cast<f32x2*>(ob)[x], reinterpret_cast<const f32x2*>(su)[x]);
        }
      } else {
#pragma unroll
        for (int q = 0; q < NRAW; ++q) {
          const int x = lane + WAVE * q;
          if (x < cnt) store_stream(&ob[x], su[x]);
        }
      }
      wave_sync();
    }
    (void)ng;
  }
}

template <int NP, int WPB, int TPI>
__device__ __forceinline__ void fwd_f32s_staged_body(const FwdArgs<float>& p, uint32_t bid, uint32_t nblk,
                                                     char* lds) {
  if constexpr (TPI > 1)
    fwd_f32s_staged_multi<NP, WPB, TPI>(p, bid, nblk, lds);
  else
    fwd_f32s_staged_single<NP, WPB>(p, bid, nblk, lds);
}

// ------------------------------------------------------------------ split-BF16 chunk-register

template <int NP, int WPB, int TPW>
constexpr int fwd_f32s_chunkreg_lds() { return chunk_lds<NP, 4, TPW>(); }

template <int NP, int WPB, int TPW>
__device__ __forceinline__ void fwd_f32s_chunkreg_body(const FwdArgs<float>& p, uint32_t bid, uint32_t nblk,
                                                       char* lds) {
  using Sh = Shape<NP>;
  static_assert(WPB >= Sh::NCHUNK, "one wave per output chunk");
  constexpr int KS = Sh::KS16;
  constexpr int OLD = chunk_old<NP, 4>();
  constexpr int OSUP = TPW * 16 * OLD;
  const int lane = threadIdx.x & 63;
  const int n = lane & 15, g = lane >> 4;
  const int w = threadIdx.x >> 6;
  const bool mma = w < Sh::NCHUNK;
  const int ch = mma ? w : 0;
  Bf16x8Bits ah[3][KS], al[3][KS];
#pragma unroll
  for (int tt = 0; tt < 3; ++tt) {
    const int T = 3 * ch + tt;
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      if (mma && T < Sh::MT) {
        afrag_bf16<NP>(p.D, T, s, lane, ah[tt][s], al[tt][s]);
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) ah[tt][s].v[e] = al[tt][s].v[e] = 0;
      }
    }
  }
  // u is staged split: BF16 hi and lo planes, row stride LDB; the entries past
  // Np of every row are zeroed here once (staging never writes them)
  constexpr int LDB = chunk_ldb<NP>();
  constexpr int PLANE = TPW * 16 * LDB;  // elements of one plane
  {
    uint16_t* h = reinterpret_cast<uint16_t*>(lds);
    for (int x = threadIdx.x; x < TPW * 16 * (LDB - NP); x += WAVE * WPB) {
      const int c = x / (LDB - NP), j = NP + x % (LDB - NP);
      h[c * LDB + j] = 0;
      h[PLANE + c * LDB + j] = 0;
    }
  }
  auto put_u = [](char* us, int c, int i, float x) {
    uint16_t* h = reinterpret_cast<uint16_t*>(us);
    Bf16x8Bits hb, lb;
    split_bf16_pair(x, 0.0f, hb, lb, 0);
    h[c * LDB + i] = hb.v[0];
    h[PLANE + c * LDB + i] = lb.v[0];
  };
  auto chunk = [&](const char* usb, float* ostg, const float* gs, uint32_t col0, uint32_t k_lo) {
    if (!mma) return;
    const uint16_t* uh = reinterpret_cast<const uint16_t*>(usb);
#pragma unroll
    for (int tp = 0; tp < TPW; ++tp) {
      const int cl = tp * 16 + n;
      f32x4 acc[3];
#pragma unroll
      for (int tt = 0; tt < 3; ++tt) acc[tt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int s = 0; s < KS; ++s) {
        const Bf16x8Bits bh = *reinterpret_cast<const Bf16x8Bits*>(uh + cl * LDB + 32 * s + 8 * g);
        const Bf16x8Bits bl = *reinterpret_cast<const Bf16x8Bits*>(uh + PLANE + cl * LDB + 32 * s + 8 * g);
#pragma unroll
        for (int tt = 0; tt < 3; ++tt) {
          acc[tt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(al[tt][s]), as_bf16x8(bh), acc[tt], 0, 0, 0);
          acc[tt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(ah[tt][s]), as_bf16x8(bl), acc[tt], 0, 0, 0);
          acc[tt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(ah[tt][s]), as_bf16x8(bh), acc[tt], 0, 0, 0);
        }
      }
      const uint32_t col = col0 + cl;
      const int e = (int)(min(col, p.ncols - 1) / p.F - k_lo);
#pragma unroll
      for (int x = 0; x < 4; ++x) {
        const int tau = 4 * ch + x;
        const int i = 4 * tau + g;
        if (tau < Sh::TRIP && i < NP) {
          const int l0 = 3 * x;
#pragma unroll
          for (int bb = 0; bb < 3; ++bb)
            ostg[bb * OSUP + cl * OLD + i] = gs[e * 9 + bb] * acc[l0 >> 2][l0 & 3] +
                                           gs[e * 9 + 3 + bb] * acc[(l0 + 1) >> 2][(l0 + 1) & 3] +
                                           gs[e * 9 + 6 + bb] * acc[(l0 + 2) >> 2][(l0 + 2) & 3];
        }
      }
    }
  };
  chunkreg_loop<float, NP, WPB, KS, TPW>(p, bid, nblk, lds, chunk, put_u);
}

}  // namespace dgvol
