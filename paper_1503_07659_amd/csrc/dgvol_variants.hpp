// Instantiated launch shapes ("variants") of the forward product, per form and
// node count: which body moves the data (LDS-staged or chunk-register), how
// many waves a workgroup has, and how many 16-column tiles one loop iteration
// takes (per wave for the staged body, per workgroup for the chunk-register
// body).  Variant 0 of each list is the library's default; the others are
// the search space of the autotuner (the paper's autotuning use case, here
// applied to tile shapes).  A variant's index is its position in its list and
// is part of the ABI (dg_volume_variant, dg_group.variant).
//
// The mixed-order batched launch runs each group's variant inside one of a few
// batched kernels.  By default every 8-wave variant runs in one kernel that
// holds them all (the groups then run side by side); on request each group
// runs in its variant's class kernel ("classes"): a class holds the variants
// with one workgroup size and similar register needs, so that light bodies
// are not run at the occupancy of the heaviest one, at the price of one
// launch per class, one after the other.  Class LIGHT is compiled for at most 128
// registers per lane (two 8-wave workgroups per CU), HEAVY for at most 256,
// WAVE4 holds the 4-wave variants, compiled for at most 168 registers per lane
// (three 4-wave workgroups per CU).
//
// Each list entry is X(NP, INDEX, BODY, WPB, TILES, CLASS).
#pragma once

namespace dgvol {

constexpr int VCLASS_LIGHT = 0;
constexpr int VCLASS_HEAVY = 1;
constexpr int VCLASS_WAVE4 = 2;
constexpr int NUM_VCLASSES = 3;
// Launch classes of the batched kernels: the three variant classes, plus ALL8,
// which holds every 8-wave variant (the default batched launch runs all
// 8-wave groups side by side in one launch of it).
constexpr int LCLASS_ALL8 = NUM_VCLASSES;
constexpr int NUM_LCLASSES = NUM_VCLASSES + 1;

constexpr int VB_S = 0;  // DG_BODY_STAGED
constexpr int VB_C = 1;  // DG_BODY_CHUNKREG
constexpr int VB_L = 2;  // DG_BODY_STAGED_LEAN (FP64, one tile per wave iteration)

// ------------------------------------------------------------------ FP64
#define DGVOL_F64_V4(X)                            \
  X(4, 0, VB_S, 8, 4, VCLASS_LIGHT)                \
  X(4, 1, VB_S, 8, 2, VCLASS_LIGHT)                \
  X(4, 2, VB_S, 8, 8, VCLASS_HEAVY)                \
  X(4, 3, VB_S, 4, 4, VCLASS_WAVE4)                \
  X(4, 4, VB_C, 8, 2, VCLASS_LIGHT)                \
  X(4, 5, VB_C, 8, 4, VCLASS_LIGHT)
#define DGVOL_F64_V10(X)                           \
  X(10, 0, VB_S, 8, 2, VCLASS_LIGHT)               \
  X(10, 1, VB_S, 8, 1, VCLASS_LIGHT)               \
  X(10, 2, VB_S, 8, 4, VCLASS_HEAVY)               \
  X(10, 3, VB_S, 4, 2, VCLASS_WAVE4)               \
  X(10, 4, VB_C, 8, 2, VCLASS_LIGHT)               \
  X(10, 5, VB_C, 8, 4, VCLASS_LIGHT)
#define DGVOL_F64_V20(X)                           \
  X(20, 0, VB_S, 8, 2, VCLASS_HEAVY)               \
  X(20, 1, VB_S, 8, 1, VCLASS_LIGHT)               \
  X(20, 2, VB_S, 4, 2, VCLASS_WAVE4)               \
  X(20, 3, VB_S, 4, 1, VCLASS_WAVE4)               \
  X(20, 4, VB_C, 8, 2, VCLASS_LIGHT)               \
  X(20, 5, VB_C, 8, 1, VCLASS_LIGHT)                \
  X(20, 6, VB_L, 8, 1, VCLASS_LIGHT)
#define DGVOL_F64_V35(X)                           \
  X(35, 0, VB_S, 8, 1, VCLASS_HEAVY)               \
  X(35, 1, VB_S, 4, 1, VCLASS_WAVE4)               \
  X(35, 2, VB_C, 8, 2, VCLASS_LIGHT)               \
  X(35, 3, VB_C, 8, 1, VCLASS_LIGHT)               \
  X(35, 4, VB_L, 8, 1, VCLASS_LIGHT)
#define DGVOL_F64_V56(X)                           \
  X(56, 0, VB_S, 8, 1, VCLASS_HEAVY)               \
  X(56, 1, VB_C, 8, 2, VCLASS_HEAVY)               \
  X(56, 2, VB_C, 8, 1, VCLASS_HEAVY)
#define DGVOL_F64_V84(X)                           \
  X(84, 0, VB_C, 8, 2, VCLASS_HEAVY)               \
  X(84, 1, VB_C, 8, 1, VCLASS_HEAVY)
#define DGVOL_F64_V120(X)                          \
  X(120, 0, VB_C, 8, 1, VCLASS_HEAVY)

// ------------------------------------------------------------------ split-BF16
#define DGVOL_F32S_V4(X)                           \
  X(4, 0, VB_S, 8, 8, VCLASS_HEAVY)                \
  X(4, 1, VB_S, 8, 4, VCLASS_LIGHT)                \
  X(4, 2, VB_S, 4, 4, VCLASS_WAVE4)                \
  X(4, 3, VB_C, 8, 4, VCLASS_LIGHT)                \
  X(4, 4, VB_C, 8, 8, VCLASS_LIGHT)
#define DGVOL_F32S_V10(X)                          \
  X(10, 0, VB_S, 8, 4, VCLASS_HEAVY)               \
  X(10, 1, VB_S, 8, 2, VCLASS_LIGHT)               \
  X(10, 2, VB_S, 4, 2, VCLASS_WAVE4)               \
  X(10, 3, VB_C, 8, 4, VCLASS_LIGHT)               \
  X(10, 4, VB_C, 8, 2, VCLASS_LIGHT)
#define DGVOL_F32S_V20(X)                          \
  X(20, 0, VB_S, 8, 4, VCLASS_HEAVY)               \
  X(20, 1, VB_S, 8, 2, VCLASS_LIGHT)               \
  X(20, 2, VB_S, 4, 2, VCLASS_WAVE4)               \
  X(20, 3, VB_C, 8, 4, VCLASS_LIGHT)               \
  X(20, 4, VB_C, 8, 2, VCLASS_LIGHT)
#define DGVOL_F32S_V35(X)                          \
  X(35, 0, VB_S, 8, 2, VCLASS_HEAVY)               \
  X(35, 1, VB_S, 8, 1, VCLASS_LIGHT)               \
  X(35, 2, VB_S, 4, 1, VCLASS_WAVE4)               \
  X(35, 3, VB_C, 8, 4, VCLASS_LIGHT)               \
  X(35, 4, VB_C, 8, 2, VCLASS_LIGHT)
#define DGVOL_F32S_V56(X)                          \
  X(56, 0, VB_S, 8, 1, VCLASS_LIGHT)               \
  X(56, 1, VB_S, 4, 1, VCLASS_WAVE4)               \
  X(56, 2, VB_C, 8, 4, VCLASS_LIGHT)               \
  X(56, 3, VB_C, 8, 2, VCLASS_LIGHT)
#define DGVOL_F32S_V84(X)                          \
  X(84, 0, VB_S, 8, 1, VCLASS_HEAVY)               \
  X(84, 1, VB_C, 8, 4, VCLASS_HEAVY)               \
  X(84, 2, VB_C, 8, 2, VCLASS_HEAVY)
#define DGVOL_F32S_V120(X)                         \
  X(120, 0, VB_C, 8, 4, VCLASS_HEAVY)              \
  X(120, 1, VB_C, 8, 2, VCLASS_HEAVY)

#define DGVOL_F64_VARIANTS(X) \
  DGVOL_F64_V4(X) DGVOL_F64_V10(X) DGVOL_F64_V20(X) DGVOL_F64_V35(X) DGVOL_F64_V56(X) DGVOL_F64_V84(X) DGVOL_F64_V120(X)
#define DGVOL_F32S_VARIANTS(X)                                                                           \
  DGVOL_F32S_V4(X) DGVOL_F32S_V10(X) DGVOL_F32S_V20(X) DGVOL_F32S_V35(X) DGVOL_F32S_V56(X) DGVOL_F32S_V84(X) \
  DGVOL_F32S_V120(X)

// a (Np, variant) pair as one switch label
constexpr int vkey(int np, int idx) { return np * 16 + idx; }

}  // namespace dgvol
