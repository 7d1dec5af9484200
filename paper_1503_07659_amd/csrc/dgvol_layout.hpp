// Register/LDS layout of the DG volume product on gfx950 matrix cores.
//
// The reference derivative of a column (one element, one field) is the product
// of the stacked matrices [D_r; D_s; D_t] (3Np x Np) with the column's nodal
// values u (Np).  Columns are processed 16 at a time: one wave computes
// [3Np x Np] . [Np x 16] on 16x16 MFMA tiles.
//
// FP64 uses v_mfma_f64_16x16x4_f64.  For lane l (n = l % 16, g = l / 16):
//   A operand: A[row = n][k = g]        B operand: B[k = g][col = n]
//   result   : reg q holds C[row = 4q + g][col = n]
// BF16 uses v_mfma_f32_16x16x32_bf16:
//   A operand: A[row = n][k = 8g + e]   B operand: B[k = 8g + e][col = n], e = 0..7
//   result   : reg q holds C[row = 4g + q][col = n]
// (both measured on the device with a layout probe).
//
// Row order.  The output rows are permuted so that every lane ends up holding
// all three reference derivatives (r, s, t) of the same node of its column:
// the chain-rule combine with the element's geometric factors is then purely
// lane-local.  Each lane group g owns 4 rows of every 16-row tile ("slots");
// slot sigma = 4T + q of tile T is assigned to direction a = sigma % 3 of node
// i = 4 * (sigma / 3) + g.  With TRIP = ceil(Np / 4) triples per lane group,
// MT = ceil(3 TRIP / 4) tiles hold every (a, i) pair; this equals the minimum
// ceil(3 Np / 16) for every supported Np except Np = 10 (3 tiles instead of 2).  Tiles are processed in chunks of 3
// (12 slots = 4 whole triples), so no triple straddles a chunk.
#pragma once

namespace dgvol {

template <int NP>
struct Shape {
  static constexpr int TRIP = (NP + 3) / 4;          // node triples per lane group
  static constexpr int SLOTS = 3 * TRIP;             // (node, direction) slots per lane group
  static constexpr int MT = (SLOTS + 3) / 4;         // 16-row tiles of the stacked product
  static constexpr int NCHUNK = (MT + 2) / 3;        // chunks of <= 3 tiles
  static constexpr int KS64 = (NP + 3) / 4;          // k-steps of the FP64 MFMA (k = 4)
  static constexpr int KS16 = (NP + 31) / 32;        // k-steps of the BF16 MFMA (k = 32)
  static constexpr int MTJ = (NP + 15) / 16;         // 16-row tiles of the transposed product (adjoint)
};

static_assert(Shape<35>::MT == 7, "Np=35 packs 105 rows into 7 tiles");
static_assert(Shape<120>::MT == 23, "Np=120 packs 360 rows into 23 tiles");
static_assert(Shape<20>::MT == 4 && Shape<56>::MT == 11 && Shape<84>::MT == 16, "tile counts");

// slot -> (direction, node) for lane group g
__host__ __device__ constexpr int slot_dir(int sigma) { return sigma % 3; }
__host__ __device__ constexpr int slot_node(int sigma, int g) { return 4 * (sigma / 3) + g; }

}  // namespace dgvol
