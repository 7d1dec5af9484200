// FP64 forward bodies of the DG volume derivative (device functions shared by
// the single-group kernels and the mixed-order batched kernel), and the
// chunk-register skeleton both forms use; the split-BF16 bodies are in
// dgvol_forward_f32s.hpp.
//
// out_b[i] = sum_a G[3a+b] (D_a u)[i] for every (element, field) column; a
// wave computes 16 columns at a time as the stacked product
// [3Np x Np] . [Np x 16] on the matrix cores with the output rows permuted so
// that each lane holds (D_r u, D_s u, D_t u) of one node (dgvol_layout.hpp);
// the geometric-factor combine is then lane-local and fused into the epilogue.
//
// Two data-movement schemes:
//  * staged (memory-bound orders): D lives in LDS as an A-operand table built
//    once per workgroup (the paper's precompute of a repeatedly fetched
//    operand into on-chip storage, Section 4.3); every wave owns whole
//    16-column tiles and moves u in and each output plane out through one LDS
//    buffer of 16 x Np words (rows padded to an odd stride at Np = 56), so all
//    global accesses are contiguous runs.
//  * chunk-register (matrix-core-bound orders, D too large for LDS): the
//    workgroup shares a run of 16-column tiles per iteration; wave w keeps the
//    A operands of output chunk w (3 tiles) in registers for the whole launch;
//    u and the geometric factors are staged per iteration in LDS and read by
//    all waves; the output planes are assembled in LDS.
// Each body takes its block index and block count explicitly and carves its
// LDS from one dynamic buffer, so the same code serves every launch shape.
#pragma once

#include <type_traits>

#include "dgvol_device.hpp"

namespace dgvol {

template <typename T>
struct FwdArgs {
  const T* D;
  const T* G;
  const T* u;
  T* out;
  uint32_t ncols;   // K * F
  uint32_t F;
  int64_t plane;    // K * F * Np (words between output planes)
  uint32_t ntiles;  // ceil(ncols / 16)
};

// ------------------------------------------------------------------ FP64 staged

// 16-column tiles a wave of the FP64 staged body takes per iteration (TPI),
// by default.  A tile of a low order is only 16 Np doubles, too few bytes in
// flight per wave to cover the memory latency; several tiles per iteration
// (with their geometric factors fetched as one contiguous run) raise that.
// Other counts are instantiated as tuning variants.
template <int NP>
constexpr int staged_tpi() { return NP <= 4 ? 4 : (NP <= 20 ? 2 : 1); }

// Per wave: the u / output staging buffer, plus, with several tiles per
// iteration, room for the geometric factors of up to 16 TPI elements.
template <int NP, int TPI>
constexpr int staged_wave_doubles() {
  // (Np >= 56: rows padded to an odd stride, see fwd_f64_staged_early)
  return TPI * 16 * (NP >= 56 ? NP + 1 : NP) + (TPI > 1 ? TPI * 16 * 9 : 0);
}

template <int NP, int WPB, int TPI>
constexpr int fwd_f64_staged_lds() {
  return align16(fwd_table_doubles<NP>() * 8) + WPB * staged_wave_doubles<NP, TPI>() * 8;
}

// LEAN: the register-lean form (two 8-wave workgroups per CU, at most 128
// registers a lane): each A operand is read from LDS right before its product
// instead of one k-step ahead, and the geometric factors are read after the
// products instead of being held through them.  The other resident workgroup
// covers the LDS latency this exposes.
template <int NP, int WPB, bool LEAN = false>
__device__ __forceinline__ void fwd_f64_staged_single(const FwdArgs<double>& p, uint32_t bid, uint32_t nblk,
                                                      char* lds) {
  using Sh = Shape<NP>;
  constexpr int NFRAG = fwd_table_doubles<NP>();
  constexpr int TILE = 16 * NP;
  // The next tile's u is requested after this tile's output stores (late):
  // the orders that use this form are bound by the streams, and there an early
  // request, holding its registers through the products, measured slower.
  constexpr int NRAW = (TILE + WAVE - 1) / WAVE;
  double* afr = reinterpret_cast<double*>(lds);
  double* stg_all = reinterpret_cast<double*>(lds + align16(NFRAG * 8));
  for (int e = threadIdx.x; e < NFRAG; e += WAVE * WPB) {
    const int ts = e >> 6;
    afr[e] = afrag_f64<NP>(p.D, ts / Sh::KS64, ts % Sh::KS64, e & 63);
  }
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int n = lane & 15, g = lane >> 4;
  // wave-uniform (readfirstlane): branches on it are scalar (measured: order 4
  // forward -0.7 %; the chunk-register bodies and the two-pass adjoint measured
  // slower with it)
  const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  double* stg = stg_all + wave * TILE;
  const uint32_t stride = nblk * WPB;
  uint32_t t = bid * WPB + wave;
  double raw[NRAW];
  auto load_raw = [&](uint32_t tt) {
    const double* __restrict__ src = p.u + (int64_t)tt * TILE;
    const int cnt = (int)min(16u, p.ncols - tt * 16) * NP;
#pragma unroll
    for (int q = 0; q < NRAW; ++q) {
      const int x = lane + WAVE * q;
      raw[q] = x < cnt ? src[x] : 0.0;
    }
  };
  if (t < p.ntiles) load_raw(t);
  for (; t < p.ntiles; t += stride) {
    const uint32_t col0 = t * 16;
    const int cnt = (int)min(16u, p.ncols - col0) * NP;
#pragma unroll
    for (int q = 0; q < NRAW; ++q) {
      const int x = lane + WAVE * q;
      if (x < TILE) stg[x] = raw[q];
    }
    wave_sync();
    double b[Sh::KS64];
#pragma unroll
    for (int s = 0; s < Sh::KS64; ++s) {
      const int j = 4 * s + g;
      b[s] = j < NP ? stg[n * NP + j] : 0.0;
    }
    const uint32_t col = col0 + n;
    const bool valid = col < p.ncols;
    const uint32_t k = valid ? col / p.F : 0u;
    double gk[9];
    if constexpr (!LEAN) {
#pragma unroll
      for (int c = 0; c < 9; ++c) gk[c] = valid ? p.G[(int64_t)k * 9 + c] : 0.0;
    }
    wave_sync();
    f64x4 acc[Sh::MT];
#pragma unroll
    for (int T = 0; T < Sh::MT; ++T) acc[T] = f64x4{0.0, 0.0, 0.0, 0.0};
    if constexpr (LEAN) {
#pragma unroll
      for (int s = 0; s < Sh::KS64; ++s) {
#pragma unroll
        for (int T = 0; T < Sh::MT; ++T)
          acc[T] = __builtin_amdgcn_mfma_f64_16x16x4f64(afr[(T * Sh::KS64 + s) * WAVE + lane], b[s], acc[T], 0, 0,
                                                       0);
        __builtin_amdgcn_sched_barrier(0);
      }
#pragma unroll
      for (int c = 0; c < 9; ++c) gk[c] = valid ? p.G[(int64_t)k * 9 + c] : 0.0;
    } else {
      // A operands are read one k-step ahead of the products that use them; the
      // scheduling barrier keeps the compiler from hoisting every read (which
      // would cost about two registers per MFMA).
      double a_cur[Sh::MT], a_nxt[Sh::MT];
#pragma unroll
      for (int T = 0; T < Sh::MT; ++T) a_cur[T] = afr[(T * Sh::KS64) * WAVE + lane];
#pragma unroll
      for (int s = 0; s < Sh::KS64; ++s) {
#pragma unroll
        for (int T = 0; T < Sh::MT; ++T) {
          if (s + 1 < Sh::KS64) a_nxt[T] = afr[(T * Sh::KS64 + s + 1) * WAVE + lane];
          acc[T] = __builtin_amdgcn_mfma_f64_16x16x4f64(a_cur[T], b[s], acc[T], 0, 0, 0);
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int T = 0; T < Sh::MT; ++T) a_cur[T] = a_nxt[T];
      }
    }
#pragma unroll
    for (int bb = 0; bb < 3; ++bb) {
#pragma unroll
      for (int tau = 0; tau < Sh::TRIP; ++tau) {
        const int i = 4 * tau + g;
        const int s0 = 3 * tau;
        const double v = gk[bb] * acc[s0 >> 2][s0 & 3] + gk[3 + bb] * acc[(s0 + 1) >> 2][(s0 + 1) & 3] +
                         gk[6 + bb] * acc[(s0 + 2) >> 2][(s0 + 2) & 3];
        if (i < NP) stg[n * NP + i] = v;
      }
      wave_sync();
      double* __restrict__ ob = p.out + bb * p.plane + (int64_t)col0 * NP;
#pragma unroll
      for (int q = 0; q < NRAW; ++q) {
        const int x = lane + WAVE * q;
        if (x < cnt) store_stream(&ob[x], stg[x]);
      }
      wave_sync();
    }
    if (t + stride < p.ntiles) load_raw(t + stride);
  }
}

// One tile per wave iteration for the matrix-bound order (Np = 56).  Loads
// and stores share one in-order completion counter, so a request for the next
// tile's u issued after this tile's output stores would only be usable once
// those stores have completed; here it is issued before the products (early)
// and holds its registers through them.  u and the output move through buffer
// ranges (no branches around the memory operations), and the next tile is
// staged at the end of an iteration, so that wait counts exactly the stores
// issued after the loads instead of waiting for them too.
template <int NP, int WPB>
__device__ __forceinline__ void fwd_f64_staged_early(const FwdArgs<double>& p, uint32_t bid, uint32_t nblk,
                                                     char* lds) {
  using Sh = Shape<NP>;
  constexpr int NFRAG = fwd_table_doubles<NP>();
  constexpr int TILE = 16 * NP;
  constexpr int NRAW = (TILE + WAVE - 1) / WAVE;
  // Odd row stride of the staging buffer: with stride 56 the B-operand reads and
  // the epilogue writes of the 16 columns met only 2 distinct 8-byte banks
  // (8-way conflicts; the work took 13 % longer).
  constexpr int LD = NP + 1;
  double* afr = reinterpret_cast<double*>(lds);
  double* stg_all = reinterpret_cast<double*>(lds + align16(NFRAG * 8));
  for (int e = threadIdx.x; e < NFRAG; e += WAVE * WPB) {
    const int ts = e >> 6;
    afr[e] = afrag_f64<NP>(p.D, ts / Sh::KS64, ts % Sh::KS64, e & 63);
  }
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int n = lane & 15, g = lane >> 4;
  // wave-uniform for certain: the buffer descriptors are built from it
  const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  double* stg = stg_all + wave * 16 * LD;
  const uint32_t stride = nblk * WPB;
  uint32_t t = bid * WPB + wave;
  double raw[NRAW];
  // tile tt's u through a buffer range of its valid words; past the last tile
  // the range is empty (zeros, no memory access)
  auto load_raw = [&](uint32_t tt) {
    const bool any = tt < p.ntiles;
    const uint32_t cnt = any ? min(16u, p.ncols - tt * 16) * NP : 0u;
    const __amdgpu_buffer_rsrc_t r = buffer_range(any ? p.u + (int64_t)tt * TILE : p.u, cnt * 8u);
#pragma unroll
    for (int q = 0; q < NRAW; ++q) raw[q] = buffer_load_f64(r, (uint32_t)(lane + WAVE * q) * 8u);
  };
  auto stage = [&]() {
#pragma unroll
    for (int q = 0; q < NRAW; ++q) {
      const int x = lane + WAVE * q;
      if (x < TILE) stg[(x / NP) * LD + x % NP] = raw[q];
    }
    wave_sync();
  };
  load_raw(t);
  stage();
  for (; t < p.ntiles; t += stride) {
    const uint32_t col0 = t * 16;
    const int cnt = (int)min(16u, p.ncols - col0) * NP;
    double b[Sh::KS64];
#pragma unroll
    for (int s = 0; s < Sh::KS64; ++s) {
      const int j = 4 * s + g;
      b[s] = j < NP ? stg[n * LD + j] : 0.0;
    }
    const uint32_t col = col0 + n;
    const uint32_t k = (col < p.ncols ? col : 0u) / p.F;
    double gk[9];  // (columns past the end read element 0; their results are not stored)
#pragma unroll
    for (int c = 0; c < 9; ++c) gk[c] = p.G[(int64_t)k * 9 + c];
    wave_sync();
    load_raw(t + stride);
    f64x4 acc[Sh::MT];
#pragma unroll
    for (int T = 0; T < Sh::MT; ++T) acc[T] = f64x4{0.0, 0.0, 0.0, 0.0};
    // A operands are read one k-step ahead of the products that use them, each
    // read right after a product (else the compiler sinks them all behind the
    // k-step's products and the next k-step waits on LDS latency).  The wave
    // raises its priority for the products, so that a wave in its epilogue
    // does not take issue slots from one in its products.
    double a_cur[Sh::MT], a_nxt[Sh::MT];
#pragma unroll
    for (int T = 0; T < Sh::MT; ++T) a_cur[T] = afr[(T * Sh::KS64) * WAVE + lane];
    __builtin_amdgcn_s_setprio(1);
#pragma unroll
    for (int s = 0; s < Sh::KS64; ++s) {
#pragma unroll
      for (int T = 0; T < Sh::MT; ++T) {
        if (s + 1 < Sh::KS64) a_nxt[T] = afr[(T * Sh::KS64 + s + 1) * WAVE + lane];
        acc[T] = __builtin_amdgcn_mfma_f64_16x16x4f64(a_cur[T], b[s], acc[T], 0, 0, 0);
      }
#pragma unroll
      for (int T = 0; T < Sh::MT; ++T) {
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // one MFMA,
        __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);  // then one LDS read
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int T = 0; T < Sh::MT; ++T) a_cur[T] = a_nxt[T];
    }
    __builtin_amdgcn_s_setprio(0);
#pragma unroll
    for (int bb = 0; bb < 3; ++bb) {
#pragma unroll
      for (int tau = 0; tau < Sh::TRIP; ++tau) {
        const int i = 4 * tau + g;
        const int s0 = 3 * tau;
        const double v = gk[bb] * acc[s0 >> 2][s0 & 3] + gk[3 + bb] * acc[(s0 + 1) >> 2][(s0 + 1) & 3] +
                         gk[6 + bb] * acc[(s0 + 2) >> 2][(s0 + 2) & 3];
        if (i < NP) stg[n * LD + i] = v;
      }
      wave_sync();
      const __amdgpu_buffer_rsrc_t ro = buffer_range(p.out + bb * p.plane + (int64_t)col0 * NP, (uint32_t)cnt * 8u);
#pragma unroll
      for (int q = 0; q < NRAW; ++q) {
        const int x = lane + WAVE * q;
        const int xc = min(x, TILE - 1);
        buffer_store_stream_f64(ro, (uint32_t)x * 8u, stg[(xc / NP) * LD + xc % NP]);
      }
      wave_sync();
    }
    stage();  // the next tile's u (its loads were issued before the products)
  }
}

// Several tiles per iteration (low orders).  A wave takes TPI consecutive
// tiles -- 16 TPI columns, one contiguous run of u and of each output plane --
// and fetches the geometric factors of their elements, which are contiguous in
// G, as one run too.  Both are loaded into registers one iteration ahead and
// staged through the wave's LDS buffer.
template <int NP, int WPB, int TPI>
__device__ __forceinline__ void fwd_f64_staged_multi(const FwdArgs<double>& p, uint32_t bid, uint32_t nblk,
                                                     char* lds) {
  using Sh = Shape<NP>;
  constexpr int NFRAG = fwd_table_doubles<NP>();
  constexpr int TILE = 16 * NP;
  constexpr int RUN = TPI * TILE;                  // doubles of u per iteration
  constexpr int NRAW = (RUN + WAVE - 1) / WAVE;
  constexpr int GW = TPI * 16 * 9;                 // G words of at most 16 TPI elements
  constexpr int NGR = (GW + WAVE - 1) / WAVE;
  double* afr = reinterpret_cast<double*>(lds);
  for (int e = threadIdx.x; e < NFRAG; e += WAVE * WPB) {
    const int ts = e >> 6;
    afr[e] = afrag_f64<NP>(p.D, ts / Sh::KS64, ts % Sh::KS64, e & 63);
  }
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int n = lane & 15, g = lane >> 4;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  double* su = reinterpret_cast<double*>(lds + align16(NFRAG * 8)) + wave * staged_wave_doubles<NP, TPI>();
  double* sg = su + RUN;
  const uint32_t nrun = (p.ntiles + TPI - 1) / TPI;
  const uint32_t stride = nblk * WPB;
  uint32_t t = bid * WPB + wave;
  double raw[NRAW], graw[NGR];
  // first element of the run and the number of its G words
  auto run_elems = [&](uint32_t tt, uint32_t& e0, int& ng) __attribute__((always_inline)) {
    const uint32_t c0 = tt * (16 * TPI);
    const uint32_t c1 = min(c0 + 16 * TPI, p.ncols) - 1;
    e0 = c0 / p.F;
    ng = (int)(c1 / p.F - e0 + 1) * 9;
  };
  // run tt's u and G through buffer ranges of their valid words (empty past
  // the last run), so the loads are unconditional
  auto load_run = [&](uint32_t tt) __attribute__((always_inline)) {
    const bool any = tt < nrun;
    const uint32_t c0 = tt * (16 * TPI);
    const uint32_t cnt = any ? min(16u * TPI, p.ncols - c0) * NP : 0u;
    const __amdgpu_buffer_rsrc_t ru = buffer_range(any ? p.u + (int64_t)c0 * NP : p.u, cnt * 8u);
#pragma unroll
    for (int q = 0; q < NRAW; ++q) raw[q] = buffer_load_f64(ru, (uint32_t)(lane + WAVE * q) * 8u);
    uint32_t e0 = 0;
    int ng = 0;
    if (any) run_elems(tt, e0, ng);
    const __amdgpu_buffer_rsrc_t rg = buffer_range(p.G + (int64_t)e0 * 9, (uint32_t)ng * 8u);
#pragma unroll
    for (int q = 0; q < NGR; ++q) graw[q] = buffer_load_f64(rg, (uint32_t)(lane + WAVE * q) * 8u);
  };
  auto stage = [&]() __attribute__((always_inline)) {
#pragma unroll
    for (int q = 0; q < NRAW; ++q) {
      const int x = lane + WAVE * q;
      if (x < RUN) su[x] = raw[q];
    }
#pragma unroll
    for (int q = 0; q < NGR; ++q) {
      const int x = lane + WAVE * q;
      if (x < GW) sg[x] = graw[q];
    }
    wave_sync();
  };
  load_run(t);
  stage();
  for (; t < nrun; t += stride) {
    const uint32_t col0 = t * (16 * TPI);
    const int cnt = (int)min(16u * TPI, p.ncols - col0) * NP;
    uint32_t e0;
    int ng;
    run_elems(t, e0, ng);
    double b[TPI][Sh::KS64];
#pragma unroll
    for (int r = 0; r < TPI; ++r) {
#pragma unroll
      for (int s = 0; s < Sh::KS64; ++s) {
        const int j = 4 * s + g;
        b[r][s] = j < NP ? su[r * TILE + n * NP + j] : 0.0;
      }
    }
    wave_sync();
    load_run(t + stride);
    f64x4 acc[TPI][Sh::MT];
#pragma unroll
    for (int r = 0; r < TPI; ++r) {
#pragma unroll
      for (int T = 0; T < Sh::MT; ++T) acc[r][T] = f64x4{0.0, 0.0, 0.0, 0.0};
    }
    // one k-step's A operands at a time, shared by the TPI tiles
#pragma unroll
    for (int s = 0; s < Sh::KS64; ++s) {
      double a[Sh::MT];
#pragma unroll
      for (int T = 0; T < Sh::MT; ++T) a[T] = afr[(T * Sh::KS64 + s) * WAVE + lane];
#pragma unroll
      for (int r = 0; r < TPI; ++r) {
#pragma unroll
        for (int T = 0; T < Sh::MT; ++T)
          acc[r][T] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[T], b[r][s], acc[r][T], 0, 0, 0);
      }
      __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int bb = 0; bb < 3; ++bb) {
#pragma unroll
      for (int r = 0; r < TPI; ++r) {
        const uint32_t col = col0 + 16 * r + n;
        const int ge = col < p.ncols ? (int)(col / p.F - e0) * 9 : 0;
        const double g0 = sg[ge + bb], g1 = sg[ge + 3 + bb], g2 = sg[ge + 6 + bb];
#pragma unroll
        for (int tau = 0; tau < Sh::TRIP; ++tau) {
          const int i = 4 * tau + g;
          const int s0 = 3 * tau;
          const double v = g0 * acc[r][s0 >> 2][s0 & 3] + g1 * acc[r][(s0 + 1) >> 2][(s0 + 1) & 3] +
                           g2 * acc[r][(s0 + 2) >> 2][(s0 + 2) & 3];
          if (i < NP) su[r * TILE + n * NP + i] = v;
        }
      }
      wave_sync();
      const __amdgpu_buffer_rsrc_t ro = buffer_range(p.out + bb * p.plane + (int64_t)col0 * NP, (uint32_t)cnt * 8u);
#pragma unroll
      for (int q = 0; q < NRAW; ++q) {
        const int x = lane + WAVE * q;
        buffer_store_stream_f64(ro, (uint32_t)x * 8u, su[min(x, RUN - 1)]);
      }
      wave_sync();
    }
    stage();  // the next run (its loads were issued before the products)
    (void)ng;
  }
}

template <int NP, int WPB, int TPI, bool LEAN = false>
__device__ __forceinline__ void fwd_f64_staged_body(const FwdArgs<double>& p, uint32_t bid, uint32_t nblk,
                                                    char* lds) {
  if constexpr (LEAN)
    fwd_f64_staged_single<NP, WPB, true>(p, bid, nblk, lds);
  else if constexpr (TPI > 1)
    fwd_f64_staged_multi<NP, WPB, TPI>(p, bid, nblk, lds);
  else if constexpr (NP >= 56)
    fwd_f64_staged_early<NP, WPB>(p, bid, nblk, lds);
  else
    fwd_f64_staged_single<NP, WPB>(p, bid, nblk, lds);
}

// ------------------------------------------------------------------ FP64 chunk-register

// Row stride of the staged u rows.  FP64: odd, so the 8-byte B-operand reads
// of a wave spread over the banks.  FP32: the smallest stride >= Np that is 4
// modulo 8 words, so each lane's 8 consecutive operand words are two aligned
// 16-byte reads and the 16 lanes of a read group start on distinct banks.
template <int NP, int WORD>
constexpr int chunk_ld() { return WORD == 8 ? NP + 1 : ((NP + 3) / 8) * 8 + 4; }

// Row stride of the output tile: each wave writes word (column n, node 4 tau + g)
// from all 64 lanes.  FP64: Np + 2 (Np = 0 mod 4), so the two half-wave groups of
// an 8-byte write hit distinct banks; FP32: a multiple of 4 that is 4 mod 8.
template <int NP, int WORD>
constexpr int chunk_old() { return WORD == 8 ? NP + 2 : ((NP + 3) / 8) * 8 + 4; }

// Column tiles the workgroup shares per iteration of the chunk-register bodies
// (TPW), by default: more tiles per iteration means fewer barriers per byte and
// more bytes in flight, at the cost of prefetch registers (FP64 at Np = 120
// has none to spare).  Other counts are instantiated as tuning variants.
template <int NP, int WORD>
constexpr int chunk_tpw() { return WORD == 4 ? 4 : (NP >= 120 ? 1 : 2); }

// Split-BF16: u is staged already split, as BF16 hi and lo planes with this
// row stride (elements): every k-step's 32 entries plus 8, so a row is 16
// modulo 32 bytes and the 16 lanes of a 16-byte read group start on distinct
// banks; the entries past Np stay zero.
template <int NP>
constexpr int chunk_ldb() { return Shape<NP>::KS16 * 32 + 8; }

// Bytes of the staged u of one iteration.
template <int NP, int WORD, int TPW>
constexpr int chunk_us_bytes() {
  return WORD == 8 ? TPW * 16 * chunk_ld<NP, WORD>() * WORD : 2 * TPW * 16 * chunk_ldb<NP>() * 2;
}

// FP64 at Np = 84 the 16 row tiles make 6 chunks (five of 3 tiles, one of 1)
// for 8 waves; as plain chunks two of the four SIMDs would carry 6 tiles and
// two 3.  There the two spare waves take the last k-steps of two chunks and
// write their partial outputs into a second output tile, which the stores add.
template <int NP, int WORD>
constexpr bool chunk_sum2() { return WORD == 8 && NP == 84; }

// Byte offset of the second output tile (after the u stage, the output tile
// and the geometric factors).
template <int NP, int WORD, int TPW>
constexpr int chunk_out2_offset() {
  return align16(chunk_us_bytes<NP, WORD, TPW>()) + align16(3 * TPW * 16 * chunk_old<NP, WORD>() * WORD) +
         align16(TPW * 16 * 9 * WORD);
}

template <int NP, int WORD, int TPW>
constexpr int chunk_lds() {
  return chunk_out2_offset<NP, WORD, TPW>() +
         (chunk_sum2<NP, WORD>() ? 3 * TPW * 16 * chunk_old<NP, WORD>() * WORD : 0);
}

template <int NP, int WPB, int TPW>
constexpr int fwd_f64_chunkreg_lds() { return chunk_lds<NP, 8, TPW>(); }

// Shared skeleton of the chunk-register bodies.  Per iteration the workgroup
// stages TPW consecutive 16-column tiles of u (padded rows) and the geometric
// factors of their elements in LDS, each compute wave runs its output chunk
// for the TPW tiles and writes the results into an LDS output tile, and all
// threads store the three planes as contiguous runs.  The next iteration's u
// and G are loaded into registers while this iteration computes.  All global
// loads and stores go through buffer ranges (no branches around them), so the
// compiler's waits count exactly the operations in flight; with conditional
// loads and stores every wait had become a wait for everything, including the
// previous iteration's stores (order 7 took 13 % longer).  The body lays out
// the staged u: put_u(us, column, node, value) stores one word of it (FP64:
// padded rows; split-BF16: the value split into BF16 hi and lo planes).
template <typename T, int NP, int WPB, int KS, int TPW, int VEC, typename ChunkFn, typename PutU>
__device__ __forceinline__ void chunkreg_loop_vec(const FwdArgs<T>& p, uint32_t bid, uint32_t nblk, char* lds,
                                                  ChunkFn&& chunk, PutU&& put_u) {
  constexpr int WORD = sizeof(T);
  constexpr int SUP = TPW * 16 * NP;        // words of one plane of the super-tile
  constexpr int OLD = chunk_old<NP, WORD>();
  constexpr int OSUP = TPW * 16 * OLD;      // words of one plane of the output tile
  constexpr int NT = WAVE * WPB;
  static_assert(NP % VEC == 0, "a vector never crosses a column");
  constexpr int NLD = (SUP / VEC + NT - 1) / NT;  // u vectors loaded per thread per iteration
  constexpr int GMAX = TPW * 16 * 9;        // geometric-factor words of at most TPW*16 elements
  constexpr int NG = (GMAX + NT - 1) / NT;  // G words loaded per thread per iteration
  char* us = lds;  // laid out by put_u (the body's staging of one u word)
  T* ostg = reinterpret_cast<T*>(lds + align16(chunk_us_bytes<NP, WORD, TPW>()));
  T* gs = reinterpret_cast<T*>(lds + align16(chunk_us_bytes<NP, WORD, TPW>()) + align16(3 * OSUP * WORD));
  constexpr bool SUM2 = chunk_sum2<NP, WORD>();
  const T* ostg2 = reinterpret_cast<const T*>(lds + chunk_out2_offset<NP, WORD, TPW>());
  const int tid = threadIdx.x;
  const uint32_t nsup = (p.ntiles + TPW - 1) / TPW;
  T ur[NLD][VEC];
  T gr[NG];
  // run s's u and geometric factors through buffer ranges of their valid words
  // (empty past the last run: zeros, no memory access), so the loads are
  // unconditional; a vector lies wholly inside or outside a range
  auto load = [&](uint32_t s) {
    const bool any = s < nsup;
    const uint32_t c0 = s * TPW * 16;
    const uint32_t ncl = any ? min((uint32_t)(TPW * 16), p.ncols - c0) : 0u;
    const __amdgpu_buffer_rsrc_t ru = buffer_range(any ? p.u + (int64_t)c0 * NP : p.u, ncl * NP * WORD);
#pragma unroll
    for (int q = 0; q < NLD; ++q) {
      const uint32_t off = (uint32_t)(tid + NT * q) * (VEC * WORD);
      if constexpr (VEC == 1) {
        ur[q][0] = buffer_load_word(ru, off, T());
      } else {
        const WordVec<T, VEC> v = buffer_load_vec<T, VEC>(ru, off);
#pragma unroll
        for (int e = 0; e < VEC; ++e) ur[q][e] = v.v[e];
      }
    }
    const uint32_t k_lo = any ? c0 / p.F : 0u;
    const uint32_t nk = any ? (c0 + ncl - 1) / p.F - k_lo + 1 : 0u;
    const __amdgpu_buffer_rsrc_t rg = buffer_range(any ? p.G + (int64_t)k_lo * 9 : p.G, nk * 9 * WORD);
#pragma unroll
    for (int q = 0; q < NG; ++q) gr[q] = buffer_load_word(rg, (uint32_t)(tid + NT * q) * WORD, T());
  };
  // staged at the end of an iteration (after its stores), so the wait for the
  // loads does not cover the stores issued after them
  auto stage = [&]() {
#pragma unroll
    for (int q = 0; q < NLD; ++q) {
      const int x0 = (tid + NT * q) * VEC;
      if (x0 < SUP) {
#pragma unroll
        for (int e = 0; e < VEC; ++e) put_u(us, x0 / NP, x0 % NP + e, ur[q][e]);
      }
    }
#pragma unroll
    for (int q = 0; q < NG; ++q)
      if (tid + NT * q < GMAX) gs[tid + NT * q] = gr[q];
  };
  uint32_t st = bid;
  load(st);
  stage();
  for (; st < nsup; st += nblk) {
    const uint32_t col0 = st * TPW * 16;
    const int cnt = (int)min((uint32_t)(TPW * 16), p.ncols - col0) * NP;
    const uint32_t k_lo = col0 / p.F;
    __syncthreads();
    load(st + nblk);
    chunk(us, ostg, gs, col0, k_lo);
    __syncthreads();
#pragma unroll
    for (int bb = 0; bb < 3; ++bb) {
      const __amdgpu_buffer_rsrc_t ro = buffer_range(p.out + bb * p.plane + (int64_t)col0 * NP, (uint32_t)cnt * WORD);
#pragma unroll
      for (int q = 0; q < NLD; ++q) {
        const int x0 = (tid + NT * q) * VEC;
        const int xc = min(x0, SUP - VEC);
        const int so = bb * OSUP + (xc / NP) * OLD + (xc % NP);
        const T* src = ostg + so;
        const T* src2 = ostg2 + so;  // read only with SUM2
        if constexpr (VEC == 1) {
          buffer_store_stream_word(ro, (uint32_t)x0 * WORD, SUM2 ? src[0] + src2[0] : src[0]);
        } else {
          WordVec<T, VEC> v;
#pragma unroll
          for (int e = 0; e < VEC; ++e) v.v[e] = SUM2 ? src[e] + src2[e] : src[e];
          buffer_store_stream_vec<T, VEC>(ro, (uint32_t)x0 * WORD, v);
        }
      }
    }
    stage();
  }
}

// FP64: pairs of doubles (16-byte accesses) where a column is a whole number
// of them and u, out start 16-byte aligned (planes then are too); single words
// otherwise.  Measured: pairs -4 % (order 7) and -5 % (order 6); four-float
// vectors made the split-BF16 body 2-3 % slower, so it moves single words.
template <typename T, int NP, int WPB, int KS, int TPW, typename ChunkFn, typename PutU>
__device__ __forceinline__ void chunkreg_loop(const FwdArgs<T>& p, uint32_t bid, uint32_t nblk, char* lds,
                                              ChunkFn&& chunk, PutU&& put_u) {
  constexpr int V = sizeof(T) == 8 ? 2 : 1;
  if constexpr (V > 1 && NP % V == 0) {
    if ((((uintptr_t)p.u | (uintptr_t)p.out) & 15u) == 0) {
      chunkreg_loop_vec<T, NP, WPB, KS, TPW, V>(p, bid, nblk, lds, chunk, put_u);
      return;
    }
  }
  chunkreg_loop_vec<T, NP, WPB, KS, TPW, 1>(p, bid, nblk, lds, chunk, put_u);
}

template <int NP, int WPB, int TPW>
__device__ __forceinline__ void fwd_f64_chunkreg_body(const FwdArgs<double>& p, uint32_t bid, uint32_t nblk,
                                                      char* lds) {
  using Sh = Shape<NP>;
  static_assert(WPB >= Sh::NCHUNK, "one wave per output chunk");
  constexpr int KS = Sh::KS64;
  constexpr int LD = chunk_ld<NP, 8>();
  constexpr int OLD = chunk_old<NP, 8>();
  constexpr int OSUP = TPW * 16 * OLD;
  const int lane = threadIdx.x & 63;
  const int n = lane & 15, g = lane >> 4;
  const int w = threadIdx.x >> 6;
  // Wave roles.  Without the split, wave w < NCHUNK runs chunk w whole.  With
  // it (Np = 84, chunks 0-4 of 3 tiles and chunk 5 of 1): waves 0 and 4 run
  // the first KH k-steps of chunks 0 and 4, waves 6 and 7 the rest of them
  // into the second output tile, and wave 5 its one tile, so that every SIMD
  // (waves s and s + 4) carries 84 tile k-steps where two carried 126.
  constexpr bool SPLIT = chunk_sum2<NP, 8>();
  static_assert(!SPLIT || (WPB == 8 && Sh::NCHUNK == 6 && Sh::MT == 16), "the split assumes 6 chunks on 8 waves");
  constexpr int KH = SPLIT ? 14 : KS;
  const bool helper = SPLIT && w >= 6;
  const bool mma = w < Sh::NCHUNK || helper;
  const int ch = helper ? (w == 6 ? 0 : 4) : (mma ? w : 0);
  // 0: whole chunk; 1: first KH k-steps; 2: k-steps from KH on; 3: one tile (the last chunk)
  const int role = !SPLIT ? 0 : helper ? 2 : (w == 0 || w == 4) ? 1 : w == 5 ? 3 : 0;
  // this wave's A operands, for the whole launch
  double areg[3][KS];
#pragma unroll
  for (int tt = 0; tt < 3; ++tt) {
    const int T = 3 * ch + tt;
#pragma unroll
    for (int s = 0; s < KS; ++s) areg[tt][s] = (mma && T < Sh::MT) ? afrag_f64<NP>(p.D, T, s, lane) : 0.0;
  }
  // the second output tile holds -0.0 wherever no helper writes (x + -0.0 == x)
  if constexpr (SPLIT) {
    double* o2 = reinterpret_cast<double*>(lds + chunk_out2_offset<NP, 8, TPW>());
    for (int x = threadIdx.x; x < 3 * OSUP; x += WAVE * WPB) o2[x] = -0.0;
  }
  double* ostg2 = reinterpret_cast<double*>(lds + chunk_out2_offset<NP, 8, TPW>());
  auto put_u = [](char* us, int c, int i, double v) { reinterpret_cast<double*>(us)[c * LD + i] = v; };
  auto chunk = [&](const char* usb, double* ostg, const double* gs, uint32_t col0, uint32_t k_lo) {
    if (!mma) return;
    const double* us = reinterpret_cast<const double*>(usb);
    double* dst = helper ? ostg2 : ostg;
#pragma unroll
    for (int tp = 0; tp < TPW; ++tp) {
      const int cl = tp * 16 + n;  // column within the super-tile
      f64x4 acc[3];
#pragma unroll
      for (int tt = 0; tt < 3; ++tt) acc[tt] = f64x4{0.0, 0.0, 0.0, 0.0};
      auto bval = [&](int s) {
        const int j = 4 * s + g;
        const double v = us[cl * LD + min(j, NP - 1)];
        return j < NP ? v : 0.0;
      };
      // tiles [0, NT) of the chunk over k-steps [S0, S1)
      auto run = [&](auto NTc, auto S0c, auto S1c) __attribute__((always_inline)) {
        constexpr int NTT = decltype(NTc)::value, S0 = decltype(S0c)::value, S1 = decltype(S1c)::value;
        double bcur = bval(S0);
#pragma unroll
        for (int s = S0; s < S1; ++s) {
          const double bnxt = s + 1 < S1 ? bval(s + 1) : 0.0;
#pragma unroll
          for (int tt = 0; tt < NTT; ++tt)  // a missing third tile of the last chunk has zero operands
            acc[tt] = __builtin_amdgcn_mfma_f64_16x16x4f64(areg[tt][s], bcur, acc[tt], 0, 0, 0);
          bcur = bnxt;
        }
      };
      using C0 = std::integral_constant<int, 0>;
      using C1 = std::integral_constant<int, 1>;
      using C3 = std::integral_constant<int, 3>;
      using CKH = std::integral_constant<int, KH>;
      using CKS = std::integral_constant<int, KS>;
      if (!SPLIT || role == 0)
        run(C3{}, C0{}, CKS{});
      else if (role == 1)
        run(C3{}, C0{}, CKH{});
      else if (role == 2)
        run(C3{}, CKH{}, CKS{});
      else
        run(C1{}, C0{}, CKS{});
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
            dst[bb * OSUP + cl * OLD + i] = gs[e * 9 + bb] * acc[l0 >> 2][l0 & 3] +
                                          gs[e * 9 + 3 + bb] * acc[(l0 + 1) >> 2][(l0 + 1) & 3] +
                                          gs[e * 9 + 6 + bb] * acc[(l0 + 2) >> 2][(l0 + 2) & 3];
        }
      }
    }
  };
  chunkreg_loop<double, NP, WPB, KS, TPW>(p, bid, nblk, lds, chunk, put_u);
}

}  // namespace dgvol
