/*
 * FP64 CPU oracle for the nodal DG volume derivative -- TEST INFRASTRUCTURE.
 *
 * Only the tests, the smoke check and the CPU-baseline leg of the benchmark
 * load this library.  It shares no source with the HIP library.
 *
 * Layouts (all arrays dense, row-major, FP64 unless stated):
 *   D    [3][Np][Np]     reference derivative matrices D_r, D_s, D_t
 *   G    [K][9]          geometric factors, G[k][3a+b] = d r_a / d x_b
 *   u    [K][F][Np]      nodal field values, element-major
 *   out  [3][K][F][Np]   d/dx, d/dy, d/dz planes
 *   gout [3][K][F][Np]   cotangent of out
 *   gu   [K][F][Np]      cotangent of u
 *   gG   [K][9]          cotangent of G
 *   gD   [3][Np][Np]     cotangent of D
 *
 * The volume term of nodal DG on affine elements (the PDE-solver use case in
 * the paper's Introduction) is, for every element k and field f,
 *   R_a[i]   = sum_j D[a][i][j] u[k][f][j]              (reference derivative)
 *   out_b[i] = sum_a G[k][3a+b] R_a[i]                  (chain rule)
 * Its adjoint, for a cotangent gout of out, is
 *   W_a[i]       = sum_b G[k][3a+b] gout_b[i]
 *   gu[k][f][j]  = sum_a sum_i D[a][i][j] W_a[i]
 *   gG[k][3a+b]  = sum_f sum_i gout_b[k][f][i] R_a[k][f][i]
 *   gD[a][i][j]  = sum_k sum_f W_a[k][f][i] u[k][f][j]
 * All sums run in ascending index order; compiled with -ffp-contract=off so
 * every product is rounded before it is added.  Elements are independent and
 * are shared across OpenMP threads; each output is written by one thread.
 */
#include <stdint.h>
#include <string.h>
#include <omp.h>

int oracle_num_threads(void) { return omp_get_max_threads(); }

void oracle_volume(const double *D, const double *G, const double *u, double *out,
                   int64_t K, int32_t Np, int32_t F) {
    const int64_t plane = K * (int64_t)F * Np;
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < K; ++k) {
        const double *g = G + 9 * k;
        for (int32_t f = 0; f < F; ++f) {
            const int64_t col = (k * F + f) * (int64_t)Np;
            const double *uk = u + col;
            for (int32_t i = 0; i < Np; ++i) {
                double R[3];
                for (int a = 0; a < 3; ++a) {
                    const double *Drow = D + ((int64_t)a * Np + i) * Np;
                    double s = 0.0;
                    for (int32_t j = 0; j < Np; ++j) s += Drow[j] * uk[j];
                    R[a] = s;
                }
                for (int b = 0; b < 3; ++b)
                    out[b * plane + col + i] = g[b] * R[0] + g[3 + b] * R[1] + g[6 + b] * R[2];
            }
        }
    }
}

void oracle_volume_adjoint(const double *D, const double *G, const double *u, const double *gout,
                           double *gu, double *gG, int64_t K, int32_t Np, int32_t F) {
    const int64_t plane = K * (int64_t)F * Np;
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < K; ++k) {
        const double *g = G + 9 * k;
        double acc[9];
        double W[3][Np], R[3][Np];
        for (int c = 0; c < 9; ++c) acc[c] = 0.0;
        for (int32_t f = 0; f < F; ++f) {
            const int64_t col = (k * F + f) * (int64_t)Np;
            const double *uk = u + col;
            /* W_a = sum_b G_ab gout_b ; R_a = D_a u */
            for (int32_t i = 0; i < Np; ++i) {
                for (int a = 0; a < 3; ++a) {
                    W[a][i] = g[3 * a + 0] * gout[0 * plane + col + i]
                            + g[3 * a + 1] * gout[1 * plane + col + i]
                            + g[3 * a + 2] * gout[2 * plane + col + i];
                    const double *Drow = D + ((int64_t)a * Np + i) * Np;
                    double s = 0.0;
                    for (int32_t j = 0; j < Np; ++j) s += Drow[j] * uk[j];
                    R[a][i] = s;
                }
            }
            /* gu_j = sum_a sum_i D[a][i][j] W_a[i] */
            for (int32_t j = 0; j < Np; ++j) {
                double s = 0.0;
                for (int a = 0; a < 3; ++a)
                    for (int32_t i = 0; i < Np; ++i) s += D[((int64_t)a * Np + i) * Np + j] * W[a][i];
                gu[col + j] = s;
            }
            /* gG_ab += sum_i gout_b[i] R_a[i] */
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) {
                    double s = 0.0;
                    for (int32_t i = 0; i < Np; ++i) s += gout[b * plane + col + i] * R[a][i];
                    acc[3 * a + b] += s;
                }
        }
        for (int c = 0; c < 9; ++c) gG[9 * k + c] = acc[c];
    }
}

/* Cotangent of D: gD[a][i][j] = sum over (k, f) ascending of W_a[i] u[k][f][j],
 * with W_a[i] = sum_b G[k][3a+b] gout_b[k][f][i] as in the adjoint above.  The
 * reduction runs over every element, so each OpenMP thread owns whole rows
 * (a, i) of gD and recomputes their W values; the result does not depend on
 * the thread count. */
void oracle_volume_grad_d(const double *G, const double *u, const double *gout, double *gD,
                          int64_t K, int32_t Np, int32_t F) {
    const int64_t plane = K * (int64_t)F * Np;
#pragma omp parallel for schedule(static)
    for (int32_t r = 0; r < 3 * Np; ++r) {
        const int a = r / Np;
        const int32_t i = r % Np;
        double *row = gD + (int64_t)r * Np;
        for (int32_t j = 0; j < Np; ++j) row[j] = 0.0;
        for (int64_t k = 0; k < K; ++k) {
            const double *g = G + 9 * k;
            for (int32_t f = 0; f < F; ++f) {
                const int64_t col = (k * F + f) * (int64_t)Np;
                const double w = g[3 * a + 0] * gout[0 * plane + col + i]
                               + g[3 * a + 1] * gout[1 * plane + col + i]
                               + g[3 * a + 2] * gout[2 * plane + col + i];
                for (int32_t j = 0; j < Np; ++j) row[j] += w * u[col + j];
            }
        }
    }
}

/* Round an FP32 value to the nearest BF16 (ties to even), returned as FP32.
 * BF16 keeps the top 16 bits of the FP32 encoding.  NaN stays NaN (quiet),
 * infinities and overflow to infinity follow IEEE round-to-nearest-even. */
static float bf16_rne(float x) {
    uint32_t b;
    memcpy(&b, &x, 4);
    if ((b & 0x7f800000u) == 0x7f800000u && (b & 0x007fffffu) != 0) {
        b = (b | 0x00400000u) & 0xffff0000u;
    } else {
        uint32_t lsb = (b >> 16) & 1u;
        b = (b + 0x7fffu + lsb) & 0xffff0000u;
    }
    float y;
    memcpy(&y, &b, 4);
    return y;
}

void oracle_bf16_round(const float *x, float *y, int64_t n) {
    for (int64_t i = 0; i < n; ++i) y[i] = bf16_rne(x[i]);
}

/*
 * Split-BF16 three-pass product, emulated.  Each FP32 operand x is split as
 * x_hi = bf16(x), x_lo = bf16(x - x_hi) (the difference is exact in FP32), and
 * the product D u is replaced by D_hi u_hi + D_hi u_lo + D_lo u_hi (the
 * D_lo u_lo term is dropped).  Each BF16 x BF16 product is exact in FP64; the
 * oracle accumulates them in FP64 in ascending j and applies the chain rule in
 * FP64 with the FP32 geometric factors, so the only approximation it carries
 * is the one the three-pass split itself makes.  Inputs are FP32, output FP64.
 */
void oracle_volume_split_bf16(const float *D, const float *G, const float *u, double *out,
                              int64_t K, int32_t Np, int32_t F) {
    const int64_t plane = K * (int64_t)F * Np;
    const int64_t nD = 3 * (int64_t)Np * Np;
    float Dhi[nD], Dlo[nD];
    for (int64_t e = 0; e < nD; ++e) {
        Dhi[e] = bf16_rne(D[e]);
        Dlo[e] = bf16_rne(D[e] - Dhi[e]);
    }
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < K; ++k) {
        const float *g = G + 9 * k;
        float uhi[Np], ulo[Np];
        for (int32_t f = 0; f < F; ++f) {
            const int64_t col = (k * F + f) * (int64_t)Np;
            for (int32_t j = 0; j < Np; ++j) {
                uhi[j] = bf16_rne(u[col + j]);
                ulo[j] = bf16_rne(u[col + j] - uhi[j]);
            }
            for (int32_t i = 0; i < Np; ++i) {
                double R[3];
                for (int a = 0; a < 3; ++a) {
                    const int64_t row = ((int64_t)a * Np + i) * Np;
                    double s = 0.0;
                    for (int32_t j = 0; j < Np; ++j)
                        s += (double)Dhi[row + j] * (double)uhi[j]
                           + (double)Dhi[row + j] * (double)ulo[j]
                           + (double)Dlo[row + j] * (double)uhi[j];
                    R[a] = s;
                }
                for (int b = 0; b < 3; ++b)
                    out[b * plane + col + i] = (double)g[b] * R[0] + (double)g[3 + b] * R[1]
                                             + (double)g[6 + b] * R[2];
            }
        }
    }
}
