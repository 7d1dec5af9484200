/*
 * dgvol -- nodal discontinuous-Galerkin volume derivative on MI355X (gfx950).
 *
 * The volume term of a nodal DG discretisation on affine tetrahedra (the
 * PDE-solver use case the paper lists in its Introduction as one of the
 * workloads that shaped its design).  For every element k and field f:
 *
 *     R_a[i]   = sum_j D[a][i][j] * u[k][f][j]        a in {r, s, t}
 *     out_b[i] = sum_a G[k][3a+b] * R_a[i]            b in {x, y, z}
 *
 * D are the reference differentiation matrices of the order-N element
 * (Np = (N+1)(N+2)(N+3)/6 nodes) and G[k] = J_k^{-1} are the element's
 * geometric factors (d r_a / d x_b).  The paper states no formulas for this
 * kernel; the definitions above are the standard chain rule for an affine
 * element.  Of the paper's transformations, the staging of D on chip is its
 * precompute of a repeatedly fetched operand (Section "Substitution rules
 * for precomputation"), and the product itself is the dense matrix-matrix
 * multiplication of its second worked example ("Some examples").
 *
 * Array layouts (dense, row-major, caller-owned device memory):
 *   D    [3][Np][Np]      D_r, D_s, D_t
 *   G    [K][9]           rx ry rz sx sy sz tx ty tz  (G[k][3a+b] = d r_a / d x_b)
 *   u    [K][F][Np]       element-major nodal values
 *   out  [3][K][F][Np]    the d/dx, d/dy, d/dz planes
 *
 * Conventions shared by every entry point:
 *   - All pointers are device pointers except where stated; the caller owns
 *     every buffer; the library allocates no device memory.
 *   - Calls are asynchronous and ordered on `stream` (a hipStream_t; NULL is
 *     the null stream).  Nothing synchronises the host.
 *   - Outputs are overwritten, never accumulated.  Outputs must not overlap
 *     any input or each other.
 *   - Arguments are validated before any HIP call; on error nothing is
 *     launched and no output is touched.
 *   - K == 0 is a no-op that returns DG_OK (pointers may then be NULL),
 *     except for dg_volume_grad_d and dg_volume_grad_d_noalloc, whose output
 *     gD is then set to zero.
 *   - Pointers must be aligned to their element size (8 bytes for double,
 *     4 bytes for float).
 *   - Supported node counts: Np in {4, 10, 20, 35, 56, 84, 120} (N = 1..7).
 *   - Results depend only on the inputs and Np/F, not on launch timing:
 *     repeated calls give bitwise identical outputs.
 */
#ifndef DGVOL_H
#define DGVOL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t dg_status;

#define DG_OK 0
#define DG_EINVAL (-1)        /* null pointer, K < 0, F < 1, misaligned pointer, bad size */
#define DG_EUNSUPPORTED (-2)  /* Np not a supported node count, or form not available */
#define DG_ELAUNCH (-3)       /* the HIP launch reported an error */
#define DG_EDEVICE (-4)       /* querying the current device failed */
#define DG_ESCRATCH (-5)      /* the problem needs more scratch than a fixed-scratch entry point holds */

#define DGVOL_ABI_VERSION 4

/* Forms (precisions) of the forward product. */
#define DG_FORM_F64 0   /* FP64 storage, FP64 matrix cores */
#define DG_FORM_F32S 1  /* FP32 storage, split-BF16 matrix cores (see dg_volume_f32s) */

/* Kernel bodies of the forward product (same results, different data movement). */
#define DG_BODY_STAGED 0      /* D in LDS, u and out staged through LDS per wave (memory-bound orders) */
#define DG_BODY_CHUNKREG 1    /* D held in registers, one output chunk per wave (matrix-core-bound orders) */
#define DG_BODY_STAGED_LEAN 2 /* as STAGED with at most 128 registers a lane (two 8-wave workgroups per CU) */

/* Variant (launch shape) selection: DG_VARIANT_AUTO is the library's default. */
#define DG_VARIANT_AUTO (-1)

#define DG_MAX_GROUPS 16

/* Version of this interface (DGVOL_ABI_VERSION of the built library).
 * Source: this library's interface. */
int32_t dg_abi_version(void);

/* Static description of a status code; never NULL.  Source: this library's
 * interface. */
const char *dg_strerror(dg_status status);

/* 1 if Np is a supported node count, else 0.  Source: the node count of a
 * degree-N nodal basis on the tetrahedron, Np = (N+1)(N+2)(N+3)/6; the range
 * N = 1..7 (Np = 4, 10, 20, 35, 56, 84, 120) is this library's. */
int32_t dg_supported_np(int32_t Np);

/*
 * Forward volume derivative in FP64.
 *   D    [3][Np][Np]   reference differentiation matrices (read)
 *   G    [K][9]        geometric factors (read)
 *   u    [K][F][Np]    nodal values (read)
 *   out  [3][K][F][Np] written: out[b][k][f][i] = sum_a G[k][3a+b] (D_a u[k][f])[i]
 * Source: the volume term of a nodal DG discretisation on affine elements, the
 * solver use case of the paper's Introduction (which gives no formula: this
 * is the chain rule through the element's affine map).  D is staged on chip
 * once per workgroup, the paper's precompute of a repeatedly fetched operand
 * (Section 4.3); the product is the matrix-matrix multiplication of
 * Section 5.2 with both operands staged through on-chip memory.
 * Errors: DG_EINVAL (null pointer with K > 0, K < 0, F < 1, misaligned),
 *         DG_EUNSUPPORTED (Np), DG_ELAUNCH.
 */
dg_status dg_volume(const double *D, const double *G, const double *u, double *out,
                    int64_t K, int32_t Np, int32_t F, void *stream);

/*
 * Adjoint (reverse mode) of dg_volume with respect to u and G, FP64.
 * Given the cotangent gout of out:
 *   gu[k][f][j]  = sum_a sum_i D[a][i][j] * W_a[i],  W_a[i] = sum_b G[k][3a+b] gout[b][k][f][i]
 *   gG[k][3a+b]  = sum_f sum_i gout[b][k][f][i] * (D_a u[k][f])[i]
 *   gout [3][K][F][Np] (read), gu [K][F][Np] (written), gG [K][9] (written).
 * D_a u is recomputed, not read.
 * Source: defined by this library, not by the paper: the reverse-mode
 * derivative of dg_volume, which is linear in u and in G.
 * Errors as for dg_volume.
 */
dg_status dg_volume_adjoint(const double *D, const double *G, const double *u,
                            const double *gout, double *gu, double *gG,
                            int64_t K, int32_t Np, int32_t F, void *stream);

/*
 * Cotangent of the reference differentiation matrices D, FP64.  The forward
 * map is linear in D; for the cotangent gout of out it is the sum over all
 * element columns (k, f)
 *   gD[a][i][j] = sum_k sum_f W_a[i] * u[k][f][j],
 *   W_a[i]      = sum_b G[k][3a+b] gout[b][k][f][i]   (as in dg_volume_adjoint),
 * i.e. the reverse-mode rule for a matrix product applied to the reference
 * derivative D_a u of every element and field.
 *   G [K][9], u [K][F][Np], gout [3][K][F][Np] (read); gD [3][Np][Np] (written,
 *   never accumulated; zeros when K == 0).
 *   work: device scratch of at least dg_volume_grad_d_workspace(K, Np, F)
 *   bytes, owned by the caller, 8-byte aligned; its contents on entry are
 *   ignored and on return are unspecified.  Calls that share one work buffer
 *   must be ordered on one stream.
 * The columns are split into a number of partial sums fixed by (K, F) alone
 * and added in a fixed order, so the result is the same bit for bit on every
 * run and every device.  No D argument: gD does not depend on D.
 * Source: defined by this library, not by the paper (reverse mode of the
 * matrix product in dg_volume).
 * Errors: DG_EINVAL (null or misaligned pointer, work_bytes too small,
 *         K < 0, F < 1), DG_EUNSUPPORTED (Np), DG_ELAUNCH.
 */
dg_status dg_volume_grad_d(const double *G, const double *u, const double *gout, double *gD,
                           void *work, uint64_t work_bytes,
                           int64_t K, int32_t Np, int32_t F, void *stream);

/* Scratch bytes dg_volume_grad_d needs for (K, Np, F), written to *bytes (may
 * be 0).  Pure host computation.  Source: this library's (the partition of
 * dg_volume_grad_d).  Errors: DG_EINVAL, DG_EUNSUPPORTED. */
dg_status dg_volume_grad_d_workspace(int64_t K, int32_t Np, int32_t F, uint64_t *bytes);

/*
 * dg_volume_grad_d for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation).
 * Same arguments, layouts and result as dg_volume_grad_d without the
 * workspace: the partial sums go to one fixed scratch array of
 * DG_GRAD_D_NOALLOC_SCRATCH_BYTES (64 MiB) that the library holds on every
 * device it runs on, until the process ends.  The partition of the columns is
 * that of dg_volume_grad_d, so the two give the same gD bit for bit.
 * A problem whose partial sums need more than the fixed scratch
 * (dg_volume_grad_d_workspace(K, Np, F) > DG_GRAD_D_NOALLOC_SCRATCH_BYTES,
 * which happens only at Np = 84 with K*F > 50 688 and at Np = 120 with
 * K*F > 24 832) is rejected with DG_ESCRATCH before anything is launched.
 * The call allocates nothing and calls no allocating routine; its first call
 * on a device looks up that device's copy of the scratch.
 * Every call on one device shares that device's scratch, which keeps the last
 * call's partial sums: calls that overlap in time on one device (on different
 * streams, or from host threads without ordering) race and give wrong
 * results; order them on one stream.
 * Errors: as dg_volume_grad_d (with no workspace checks), plus DG_ESCRATCH and
 *         DG_EDEVICE.
 */
#define DG_GRAD_D_NOALLOC_SCRATCH_BYTES (64ull << 20)
dg_status dg_volume_grad_d_noalloc(const double *G, const double *u, const double *gout, double *gD,
                                   int64_t K, int32_t Np, int32_t F, void *stream);

/*
 * Forward volume derivative with FP32 storage and split-BF16 products.
 * Same layouts as dg_volume with float elements.  Each FP32 operand x of the
 * product D_a u is split into x_hi = bf16(x) and x_lo = bf16(x - x_hi)
 * (round to nearest even); D_a u is formed as D_hi u_hi + D_hi u_lo + D_lo u_hi
 * on BF16 matrix cores with FP32 accumulation, and the G combine runs in FP32.
 * Stated accuracy against the FP64 result on the same (FP64) data: per output
 * plane, max|err| <= 2e-5 max|ref| and ||err||_2 <= 1e-5 ||ref||_2.
 * Source: a precision form defined by this library, not by the paper; the
 * data movement is that of dg_volume (Sections 4.3 and 5.2).
 * Errors as for dg_volume.
 */
dg_status dg_volume_f32s(const float *D, const float *G, const float *u, float *out,
                         int64_t K, int32_t Np, int32_t F, void *stream);

/*
 * One element group of a mixed-order batch (dg_volume_batched).  All pointers
 * are device pointers to arrays of the batch's form (double for DG_FORM_F64,
 * float for DG_FORM_F32S), laid out as for dg_volume.
 */
typedef struct dg_group {
  int32_t Np;          /* node count of the group's order */
  int32_t variant;     /* DG_VARIANT_AUTO or an index < dg_variant_count(form, Np) */
  int64_t K;           /* elements in the group (>= 0; 0 = skip) */
  const void *D;       /* [3][Np][Np] */
  const void *G;       /* [K][9] */
  const void *u;       /* [K][F][Np] */
  void *out;           /* [3][K][F][Np], written */
  double cost;         /* measured cost of one 16-column tile, any unit common to the
                          batch, used to split workgroups between groups; <= 0 selects
                          the library's estimate (spec roofline time of a tile over the
                          fraction of it the order's default body reaches) */
} dg_group;

/*
 * Forward volume derivative of up to DG_MAX_GROUPS element groups of
 * possibly different orders, sharing F.  `form` is DG_FORM_F64 or
 * DG_FORM_F32S, optionally ORed with DG_BATCH_BY_CLASS.  Each group runs its
 * variant.  By default every group whose variant has 8 waves per workgroup
 * runs in one persistent launch of a kernel that holds all such bodies, side
 * by side with the others (and 4-wave variants in one more launch).  With
 * DG_BATCH_BY_CLASS each group runs in the kernel of its variant's class
 * (dg_variant_info.batch_class), whose register budget fits that class, and
 * the batch makes one launch per class, in class order, on `stream`.
 * `groups` is a host array of `ngroups` descriptors; it is read during the
 * call only.  Within a launch, the resident workgroups are split between
 * groups so that the largest load of a workgroup (its loop steps times the
 * group's cost per step) is as small as possible: every group gets one, and
 * each further workgroup goes to the group whose workgroups carry the largest
 * load.  The
 * split is static: the launch needs no device-side state and can be captured
 * in a HIP graph.  Each group's out is exactly what dg_volume_variant would
 * write for that group alone with the same variant.
 * Source: the batching is this library's; the per-order choice of launch
 * shapes is the paper's autotuning use case (Introduction) applied to tile
 * shapes.
 * Errors: DG_EINVAL (ngroups outside 0..DG_MAX_GROUPS, F < 1, NULL groups
 * with ngroups > 0, a group failing the dg_volume argument checks),
 * DG_EUNSUPPORTED (form, unknown flag, Np or a variant not available for the
 * form and order), DG_EDEVICE, DG_ELAUNCH.  Groups with K = 0 are skipped.
 */
#define DG_BATCH_BY_CLASS 0x100
dg_status dg_volume_batched(const dg_group *groups, int32_t ngroups, int32_t F, int32_t form, void *stream);

/*
 * Launch shapes ("variants") of the forward product.  For each form and node
 * count the library is compiled with a short list of shapes that give the same
 * result with different data movement: the body (DG_BODY_STAGED: D in LDS,
 * every wave owns whole 16-column tiles; DG_BODY_CHUNKREG: D in registers,
 * the workgroup shares its tiles), the waves per workgroup, and the 16-column
 * tiles one loop iteration takes (per wave for the staged body, per workgroup
 * for the chunk-register body).  Variant 0 is the default that dg_volume and
 * dg_volume_f32s use; the others are the autotuner's search space (the paper's
 * autotuning use case, Introduction and Section 3, applied to tile shapes).
 */
typedef struct dg_variant_info {
  int32_t body;          /* DG_BODY_STAGED, DG_BODY_CHUNKREG or DG_BODY_STAGED_LEAN */
  int32_t waves;         /* waves (64 lanes) per workgroup */
  int32_t tiles;         /* 16-column tiles per loop iteration (per wave if staged, per workgroup if chunk-register) */
  int32_t batch_class;   /* its class: the batched kernel that runs it under DG_BATCH_BY_CLASS (0..2) */
  int32_t lds_bytes;     /* dynamic LDS per workgroup */
} dg_variant_info;

/* Number of variants for (form, Np); 0 if either is unsupported.  Pure host.
 * Source: the launch shapes are this library's; choosing among them per order
 * is the paper's autotuning use case (Introduction). */
int32_t dg_variant_count(int32_t form, int32_t Np);

/* Describe variant `variant` of (form, Np) into *info (host memory).  Pure host.
 * Source: as dg_variant_count.
 * Errors: DG_EINVAL (info NULL), DG_EUNSUPPORTED (form, Np or variant out of range). */
dg_status dg_variant_query(int32_t form, int32_t Np, int32_t variant, dg_variant_info *info);

/*
 * Forward product with an explicit variant: `form` DG_FORM_F64 (double
 * arrays, as dg_volume) or DG_FORM_F32S (float arrays, as dg_volume_f32s);
 * `variant` DG_VARIANT_AUTO or an index < dg_variant_count(form, Np).  The
 * result meets the same bound as the form's default entry point (FP64: the
 * same reference values up to summation order; split-BF16: the same stated
 * bound).  Source: the operation of dg_volume (FP64) or dg_volume_f32s; the
 * variants are this library's launch shapes (see dg_variant_count).
 * Errors as for dg_volume, plus DG_EUNSUPPORTED for the variant.
 */
dg_status dg_volume_variant(int32_t form, int32_t variant, const void *D, const void *G, const void *u,
                            void *out, int64_t K, int32_t Np, int32_t F, void *stream);

/*
 * Launch shape of an operation on the current device, computed on the host
 * without launching anything (it queries the device's occupancy for the
 * kernel).  A work unit is a 16-column tile.  The forward loops hand out
 * tiles round-robin; below Np = 84 the adjoint gives each wave a run of whole
 * elements, taken as 16-column tiles (at Np = 84, 120 its second pass gives
 * such a run to each workgroup).  min_iters is the loop iterations of the
 * least-loaded wave (or workgroup, for the workgroup-wide loops), taken over
 * every kernel the operation launches.  Source: this library's (a description
 * of its own launches, for tests and tuning).
 */
typedef struct dg_launch_shape {
  uint32_t grid;            /* workgroups launched (first kernel of the operation) */
  uint32_t block;           /* threads per workgroup */
  uint32_t lds_bytes;       /* dynamic LDS per workgroup */
  uint32_t resident;        /* workgroups the device holds at once (the persistent grid cap) */
  uint32_t units;           /* work units of the problem */
  uint32_t units_per_step;  /* units one workgroup takes per loop iteration */
  uint32_t min_iters;       /* loop iterations of the least-loaded wave, over the operation's kernels */
  uint32_t max_iters;       /* loop iterations of the most-loaded wave, over the operation's kernels */
} dg_launch_shape;

#define DG_OP_FORWARD 0   /* dg_volume_variant(form, variant, ...) */
#define DG_OP_BATCHED 1   /* dg_volume_batched with one group of this (Np, variant) */
#define DG_OP_ADJOINT 2   /* dg_volume_adjoint (form must be DG_FORM_F64; variant ignored) */
#define DG_OP_BATCHED_BY_CLASS 3  /* dg_volume_batched with DG_BATCH_BY_CLASS, one group of this (Np, variant) */

/* Errors: DG_EINVAL (shape NULL, op unknown, K < 1, F < 1), DG_EUNSUPPORTED
 * (form, Np or variant), DG_EDEVICE. */
dg_status dg_launch_shape_query(int32_t op, int32_t form, int32_t Np, int32_t variant, int64_t K, int32_t F,
                                dg_launch_shape *shape);

/*
 * Bandwidth calibration (not part of the DG computation).
 * Reads src[0..n) once and writes `copies` (1..3) scaled copies:
 * dst[c*n + i] = (c + 1) * src[i]; dst must hold copies * n doubles.
 * With copies = 1 it is a plain copy of known size, used to scale hardware
 * byte counters; with copies = 3 it moves bytes in the same 1 : 3 read : write
 * mix as dg_volume with no other work, which measures the practical streaming
 * ceiling for that mix.  Source: this library's (a measurement of the chip,
 * not DG work).  When src and dst are 16-byte aligned and n is even,
 * every thread moves several independent 16-byte pairs in a one-pass grid;
 * otherwise single words in a grid-stride loop.  Errors: DG_EINVAL (n < 0,
 * copies outside 1..3, null or misaligned pointer with n > 0), DG_EDEVICE,
 * DG_ELAUNCH.
 */
dg_status dg_stream_calibrate(const double *src, double *dst, int64_t n, int32_t copies, void *stream);

/*
 * Tile-stream calibration (not part of the DG computation): the data movement
 * of the order-4 FP64 forward (dg_volume at Np = 35) without its arithmetic.
 * src holds ntiles tiles of 560 doubles (16 columns x 35 nodes), dst three
 * planes of the same size: dst[c * 560 ntiles + 560 t + x] = (c + 1) src[560 t + x].
 * Every 64-lane wave moves whole tiles through its own LDS buffer as the
 * forward kernel does (one contiguous run in, three runs out, two LDS round
 * trips), prefetching the next tile's run before the current one's stores.
 * tiles_per_wave = m >= 1: a grid of ceil(ntiles / 8m) 8-wave workgroups, each
 * wave taking m tiles (m = 1: the grid covers the array once);
 * tiles_per_wave = 0: one 8-wave workgroup per CU looping over all tiles, the
 * launch shape of the forward kernel.  Timed by the caller, it separates the
 * cost of the launch shape from the cost of the arithmetic.  Source: this
 * library's (a measurement of the chip, not DG work).
 * Errors: DG_EINVAL (ntiles < 0 or too large, tiles_per_wave < 0, null or
 * misaligned pointer with ntiles > 0), DG_EDEVICE, DG_ELAUNCH.
 */
dg_status dg_stream_calibrate_tiles(const double *src, double *dst, int64_t ntiles, int32_t tiles_per_wave,
                                    void *stream);

/*
 * FP64 matrix-core calibration (not part of the DG computation).  Launches
 * DG_MFMA_CAL_BLOCKS workgroups of 256 threads (4 waves); every wave issues
 * `iters` rounds of 4 independent v_mfma_f64_16x16x4f64 (2048 flops each)
 * from registers, i.e. DG_MFMA_CAL_BLOCKS * 4 * iters * 4 * 2048 flops in all,
 * and writes one double per thread to sink[0 .. DG_MFMA_CAL_BLOCKS * 256).
 * Timed by the caller, it gives the attainable FP64 matrix rate of the device.
 * Source: this library's (a measurement of the chip, not DG work).
 * Errors: DG_EINVAL (null or misaligned sink, iters < 1), DG_ELAUNCH.
 */
#define DG_MFMA_CAL_BLOCKS 2048
dg_status dg_mfma_calibrate(double *sink, int32_t iters, void *stream);

/*
 * Calibration (not DG work): FP64 matrix products beside vector work on the
 * same SIMDs.  DG_MFMA_BESIDE_BLOCKS workgroups of 512 threads (8 waves).
 * Waves 0..3 run four independent chains of v_mfma_f64_16x16x4f64 for
 * `iters` rounds, as dg_mfma_calibrate.  Waves 4..7, one per SIMD beside
 * them, run `viters` rounds of 16 independent vector instructions of the kind
 * `mode`: DG_BESIDE_NONE (nothing), DG_BESIDE_FP64_FMA (v_fma_f64),
 * DG_BESIDE_INT (32-bit add, then xor), DG_BESIDE_DPP (row broadcast, then
 * add).  With iters = 0 only the vector work runs.  Each thread writes one
 * double to sink[0 .. DG_MFMA_BESIDE_BLOCKS * 512).
 * Source: defined by this library (a measurement of the chip, not DG work).
 * Errors: DG_EINVAL (null or misaligned sink, iters < 0, viters < 0, both
 *         zero, unknown mode), DG_ELAUNCH.
 */
#define DG_MFMA_BESIDE_BLOCKS 256
#define DG_BESIDE_NONE 0
#define DG_BESIDE_FP64_FMA 1
#define DG_BESIDE_INT 2
#define DG_BESIDE_DPP 3
dg_status dg_mfma_calibrate_beside(double *sink, int32_t iters, int32_t viters, int32_t mode, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* DGVOL_H */
