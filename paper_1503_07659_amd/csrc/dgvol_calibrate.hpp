// Calibration kernels (not part of the DG computation): streaming bandwidth
// for the forward's 1 : 3 read : write mix, the forward's own tile traffic
// without its arithmetic, and the FP64 matrix-core rate.  Timed by the caller
// (bench.py), they give the attainable ceilings the kernels are compared with.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "dgvol_device.hpp"

namespace dgvol {

// ------------------------------------------------------------------ stream calibration
//
// Reads n doubles once and writes `copies` scaled copies of them (dst[c*n + i]
// = (c + 1) * src[i]), with streaming (non-temporal) stores as the forward
// kernels store their output planes.  With copies = 1 this is a plain copy of
// known size (the scale of the hardware byte counters); with copies = 3 it
// moves bytes in the forward kernel's 1 : 3 read : write mix with no other
// work (the streaming ceiling for that mix).
//
// stream16_kernel: one pass, no loop: every thread moves STREAM_U independent
// 16-byte pairs (all loads issued before any store), and the grid covers the
// array once (hundreds of thousands of workgroups for the workload sizes).
// stream_kernel: the fallback for arrays that are not 16-byte aligned or of
// odd length, one 8-byte word per lane in a grid-stride loop.
constexpr int STREAM_U = 4;
constexpr int STREAM_BLOCK = 256;
typedef double f64x2 __attribute__((ext_vector_type(2)));

__global__ __launch_bounds__(STREAM_BLOCK) void stream16_kernel(const f64x2* __restrict__ src,
                                                                f64x2* __restrict__ dst, int64_t n2,
                                                                int32_t copies) {
  const int64_t base = (int64_t)blockIdx.x * (STREAM_BLOCK * STREAM_U) + threadIdx.x;
  f64x2 v[STREAM_U];
#pragma unroll
  for (int q = 0; q < STREAM_U; ++q) {
    const int64_t i = base + (int64_t)STREAM_BLOCK * q;
    v[q] = i < n2 ? src[i] : f64x2{0.0, 0.0};
  }
  for (int32_t c = 0; c < copies; ++c) {
    const double s = (double)(c + 1);
#pragma unroll
    for (int q = 0; q < STREAM_U; ++q) {
      const int64_t i = base + (int64_t)STREAM_BLOCK * q;
      if (i < n2) __builtin_nontemporal_store(v[q] * s, &dst[c * n2 + i]);
    }
  }
}

__global__ __launch_bounds__(256) void stream_kernel(const double* __restrict__ src, double* __restrict__ dst,
                                                     int64_t n, int32_t copies) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const double v = src[i];
    for (int32_t c = 0; c < copies; ++c) store_stream(&dst[c * n + i], (double)(c + 1) * v);
  }
}

// tile_stream_kernel: the order-4 forward's traffic without its arithmetic.
// Each wave moves whole 16-column tiles (16 x 35 doubles, one contiguous run
// in, one run out per plane) through its LDS buffer as the forward does: the
// run is written to LDS, read back in B-operand order (column n, node
// 4 s + g), written back per plane in output order and read again for the
// streaming stores, with dst[c][t][x] = (c + 1) src[t][x].  The next tile's
// loads are issued before this tile's stores (exact waits, no branch around a
// memory operation).  Waves take tiles t = 8 block + wave + 8 grid it,
// it = 0 .. iters - 1: with one tile per wave (iters = 1) the grid covers the
// array once; with many, the waves form a persistent loop.
constexpr int TSTREAM_NP = 35;
constexpr int TSTREAM_TILE = 16 * TSTREAM_NP;
constexpr int TSTREAM_WPB = 8;

__global__ __launch_bounds__(WAVE* TSTREAM_WPB) void tile_stream_kernel(const double* __restrict__ src,
                                                                        double* __restrict__ dst, uint32_t ntiles,
                                                                        int64_t plane, uint32_t iters) {
  extern __shared__ __attribute__((aligned(16))) char lds_raw[];
  constexpr int TILE = TSTREAM_TILE, NP = TSTREAM_NP;
  constexpr int NR = (TILE + WAVE - 1) / WAVE;
  const int lane = threadIdx.x & 63;
  const int n = lane & 15, g = lane >> 4;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  double* stg = reinterpret_cast<double*>(lds_raw) + wave * TILE;
  auto tile_of = [&](uint32_t it) -> uint32_t {
    return it < iters ? blockIdx.x * TSTREAM_WPB + wave + it * gridDim.x * TSTREAM_WPB : 0xffffffffu;
  };
  double raw[NR];
  auto load = [&](uint32_t t) {
    const bool any = t < ntiles;
    const __amdgpu_buffer_rsrc_t r = buffer_range(any ? src + (int64_t)t * TILE : src, any ? TILE * 8u : 0u);
#pragma unroll
    for (int q = 0; q < NR; ++q) raw[q] = buffer_load_f64(r, (uint32_t)(lane + WAVE * q) * 8u);
  };
  auto stage = [&]() {
#pragma unroll
    for (int q = 0; q < NR; ++q) {
      const int x = lane + WAVE * q;
      if (x < TILE) stg[x] = raw[q];
    }
    wave_sync();
  };
  uint32_t it = 0;
  uint32_t t = tile_of(0);
  load(t);
  stage();
  while (t < ntiles) {
    double b[9];
#pragma unroll
    for (int s = 0; s < 9; ++s) b[s] = stg[n * NP + min(4 * s + g, NP - 1)];
    wave_sync();
    const uint32_t tn = tile_of(++it);
    load(tn);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
#pragma unroll
      for (int s = 0; s < 9; ++s) {
        if (4 * s + g < NP) stg[n * NP + 4 * s + g] = b[s] * (double)(c + 1);
      }
      wave_sync();
      const __amdgpu_buffer_rsrc_t ro = buffer_range(dst + c * plane + (int64_t)t * TILE, TILE * 8u);
#pragma unroll
      for (int q = 0; q < NR; ++q) {
        const int x = lane + WAVE * q;
        buffer_store_stream_f64(ro, (uint32_t)x * 8u, stg[min(x, TILE - 1)]);
      }
      wave_sync();
    }
    stage();
    t = tn;
  }
}

// ------------------------------------------------------------------ matrix-core calibration
//
// Every wave runs `iters` rounds of four independent accumulator chains of
// v_mfma_f64_16x16x4f64 with register operands (no memory traffic in the
// loop), then writes one sum per lane, so the work cannot be dropped.  Each
// product depends on the previous one of its chain; the operands stay fixed
// (rewriting a source register of an MFMA in flight would stall the issue).
// Launched with 256 threads; the wider bound keeps the accumulators in VGPRs
// (with a 256-thread bound the compiler moves them through AGPRs every round).
__global__ __launch_bounds__(1024) void mfma_cal_kernel(double* __restrict__ sink, int32_t iters) {
  const int lane = threadIdx.x & 63;
  const double a = 1.0 + 1e-3 * lane, b = 1.0 - 1e-3 * lane;
  f64x4 c0 = f64x4{0.0, 0.0, 0.0, 0.0}, c1 = c0, c2 = c0, c3 = c0;
  for (int32_t it = 0; it < iters; ++it) {
    c0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c0, 0, 0, 0);
    c1 = __builtin_amdgcn_mfma_f64_16x16x4f64(b, a, c1, 0, 0, 0);
    c2 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, a, c2, 0, 0, 0);
    c3 = __builtin_amdgcn_mfma_f64_16x16x4f64(b, b, c3, 0, 0, 0);
  }
  double s = 0.0;
#pragma unroll
  for (int q = 0; q < 4; ++q) s += c0[q] + c1[q] + c2[q] + c3[q];
  sink[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// ------------------------------------------------------------------ products beside vector work
//
// One 8-wave workgroup per CU.  Waves 0..3 (one per SIMD) run the four chains
// of mfma_cal_kernel for `iters` rounds; waves 4..7 (one per SIMD, beside
// them) run `viters` rounds of 16 independent vector instructions of one kind:
//   MODE 0 nothing, 1 v_fma_f64, 2 32-bit integer add then xor, 3 a DPP row
//   broadcast (row_newbcast) then an add.
// With iters = 0 only the vector work runs.  Comparing the times shows how
// much of the vector work overlaps the FP64 products on the same SIMD.
template <int MODE>
__global__ __launch_bounds__(1024) void mfma_beside_kernel(double* __restrict__ sink, int32_t iters,
                                                           int32_t viters) {
  const int lane = threadIdx.x & 63;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  double s = 0.0;
  if (wave < 4) {
    const double a = 1.0 + 1e-3 * lane, b = 1.0 - 1e-3 * lane;
    f64x4 c0 = f64x4{0.0, 0.0, 0.0, 0.0}, c1 = c0, c2 = c0, c3 = c0;
    for (int32_t it = 0; it < iters; ++it) {
      c0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c0, 0, 0, 0);
      c1 = __builtin_amdgcn_mfma_f64_16x16x4f64(b, a, c1, 0, 0, 0);
      c2 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, a, c2, 0, 0, 0);
      c3 = __builtin_amdgcn_mfma_f64_16x16x4f64(b, b, c3, 0, 0, 0);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) s += c0[q] + c1[q] + c2[q] + c3[q];
  } else if constexpr (MODE == 1) {
    double x[16];
#pragma unroll
    for (int t = 0; t < 16; ++t) x[t] = 1.0 + 1e-4 * (lane + t);
    for (int32_t it = 0; it < viters; ++it) {
#pragma unroll
      for (int t = 0; t < 16; ++t) x[t] = __builtin_fma(x[t], 0.999999, 1e-7);
    }
#pragma unroll
    for (int t = 0; t < 16; ++t) s += x[t];
  } else if constexpr (MODE == 2) {
    uint32_t x[16];
#pragma unroll
    for (int t = 0; t < 16; ++t) x[t] = (uint32_t)(lane + t);
    const uint32_t inc = (uint32_t)viters | 1u;
    for (int32_t it = 0; it < viters; ++it) {
#pragma unroll
      for (int t = 0; t < 16; ++t) x[t] = (x[t] + inc) ^ (uint32_t)t;
    }
#pragma unroll
    for (int t = 0; t < 16; ++t) s += (double)x[t];
  } else if constexpr (MODE == 3) {
    int x[16];
#pragma unroll
    for (int t = 0; t < 16; ++t) x[t] = lane * 16 + t;
    for (int32_t it = 0; it < viters; ++it) {
#pragma unroll
      for (int t = 0; t < 16; ++t) x[t] = __builtin_amdgcn_mov_dpp(x[t], 0x153, 0xf, 0xf, false) + t;
    }
#pragma unroll
    for (int t = 0; t < 16; ++t) s += (double)x[t];
  }
  sink[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

}  // namespace dgvol
