// Internal declarations shared by the qrx HIP sources (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <type_traits>
#include <stdint.h>
#include <stddef.h>

#include "qrx.h"

#define QRX_DEV __device__ __forceinline__

typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

namespace qrx {

// Device index of a handle (-1 if it has none).
int handle_device(qrx_handle h);
// QRX_OK when *o is a valid set of options for the batched path.
int batched_opts_check(const qrx_qr_opts *o);

// The compatible-system ratio ||r|| / (||A||_F ||x|| + ||b||) certifies a
// solution at tol for square systems, where eta_F is undefined (r is rounding
// noise); for m > n only at the rounding level of the residual, which is
// where the least-squares residual itself vanishes (a consistent system).
// Returned: the factor that scales the ratio onto the tol scale.
__host__ __device__ inline double compat_scale(int64_t m, int64_t n, double tol) {
    const double lim = 1e3 * 1.1102230246251565e-16;
    return (m == n || tol <= lim) ? 1.0 : tol / lim;
}

// Exponent E with v = f 2^E, f in [0.5, 1); the power of two 2^(target - E)
// brings max-abs v into [2^(target-1), 2^target). Zero / non-finite -> 1.
QRX_DEV float pow2_scale(float v, int target) {
    if (!(v > 0.0f) || !(v <= 3.0e38f)) return 1.0f;
    int e;
    frexpf(v, &e);
    return ldexpf(1.0f, target - e);
}

QRX_DEV float wave_sum_f(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}
QRX_DEV double wave_sum_d(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}
QRX_DEV float wave_max_f(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
    return v;
}

// Error-free transformations for double-double accumulation. Contraction is
// off inside them: fusing a product into a following sum (hi + a*b -> one
// FMA) would break the exact-error identities they rely on.
QRX_DEV void two_sum(double a, double b, double &s, double &e) {
#pragma clang fp contract(off)
    s = a + b;
    double bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}
QRX_DEV void dd_add(double &hi, double &lo, double v) {   // (hi, lo) += v
#pragma clang fp contract(off)
    double s, e;
    two_sum(hi, v, s, e);
    e += lo;
    hi = s + e;
    lo = e - (hi - s);
}
QRX_DEV void dd_add_prod(double &hi, double &lo, double a, double b) {  // += a*b exactly-ish
#pragma clang fp contract(off)
    const double p = a * b;
    const double pe = fma(a, b, -p);
    dd_add(hi, lo, p);
    lo += pe;
}

// Balanced partition of `units` units into `nblk` blocks: block i starts at
// unit floor(i*units/nblk); blocks differ in size by at most one unit.
__device__ __host__ inline int64_t part_start(int64_t i, int64_t units, int64_t nblk) {
    return (i * units) / nblk;
}
// Index of the block that contains unit u.
__device__ __host__ inline int64_t part_owner(int64_t u, int64_t units, int64_t nblk) {
    return ((u + 1) * nblk - 1) / units;
}

constexpr int kPanelThreads = 256;   // TSQR block rows = threads (one row each)
constexpr int kMaxLevels = 12;
constexpr int kTrsvBlock = 256;      // padding unit of the n-vectors and of X = R^{-1}

// TSQR level descriptors of one panel (passed by value to the Q-formation kernel).
struct TsqrLevels {
    int nlev;                          // number of tree levels above level 0 (0 = single block)
    int64_t nblk[kMaxLevels + 1];      // blocks at level l (level 0 = panel row blocks)
    float *stack[kMaxLevels + 1];      // stack[l] (l >= 1): (nblk[l-1]*nb) x nb, ld = nblk[l-1]*nb
};

// ---- kernel launchers (one per .hip file section) --------------------------
// scan.hip
hipError_t launch_scan(hipStream_t s, int64_t m, int64_t n, const float *A, int64_t lda,
                       float *W, int64_t ldw, float *colmax, double *colss, int *flags);
hipError_t launch_scan_vec(hipStream_t s, int64_t m, const double *b, int *flags);
hipError_t launch_norm_finalize(hipStream_t s, int64_t n, const double *colss, double *normA);
hipError_t launch_fill_f32(hipStream_t s, float *p, int64_t count, float v);
hipError_t launch_r_finalize(hipStream_t s, int64_t n, float *R, int64_t ldr, int *flags);
// C = A B for upper-triangular n x n A, B (FP32; FP64 accumulation), C lower part zero
hipError_t launch_triu_mul(hipStream_t s, int64_t n, const float *A, int64_t lda, const float *B,
                           int64_t ldb, float *C, int64_t ldc);
hipError_t launch_copy_mat(hipStream_t s, int64_t rows, int64_t cols, const float *src,
                           int64_t lds, float *dst, int64_t ldd);
hipError_t launch_status_out(hipStream_t s, const int *flags, int *status);

// panel.hip : one TSQR panel of width w <= nb (nb = 32), m rows, column-major ld.
hipError_t launch_tsqr_level(hipStream_t s, float *P, int64_t ld, int64_t rows, int w,
                             int64_t nblk, int unit, float *rnext, int64_t ld_rnext, int reorth,
                             const float *colmax);
hipError_t launch_tsqr_qform(hipStream_t s, float *P, int64_t ld, int64_t m, int w,
                             const TsqrLevels &lv);
hipError_t launch_copy_r_block(hipStream_t s, const float *src, int64_t ld_src, int w,
                               float *R, int64_t ldr, const float *colmax);

// gram.hip : Cholesky QR twice on an FP64 Gram matrix (panel of w <= 128 columns);
// ws holds gram_workspace_doubles(m, wmax) doubles for panels up to wmax (64 or
// 128) columns; its flag area (gram_counter) is zeroed once before the first panel.
// 16-bit operand copies a Gram panel of more than 32 columns writes with its Q (as pack_q
// does): column-major qc (ldc) and row-major qr (ldq) of sc * Q, lo parts for
// a split; prec 0 writes none.
struct PanelPack {
    uint16_t *qc, *qcl, *qr, *qrl;
    int64_t ldc, ldq;
    float sc;
    int prec;
};
// Whether launch_gram_panel writes the operand copies itself for width w.
bool gram_panel_packs(int w);
hipError_t launch_gram_panel(hipStream_t s, float *P, int64_t ld, int64_t m, int w, float *R,
                             int64_t ldr, double *ws, int reorth, const PanelPack &pack);
constexpr int kGramCounterInts = 64;   // ints at gram_counter, all 0 before the first panel
size_t gram_workspace_doubles(int64_t m, int wmax);
int *gram_counter(double *ws);

// gemm.hip : trailing products of one recursion node.
//   projection: Part[s] (k x n2, ld k) = Q1^T A2 over row split s.
//   reduce:     R12 = sum_s Part[s] (unscaled), written into R (ldr);
//               also per-column update scales and colmax reset.
//   update:     A2 -= Q1 R12, refreshes colmax of A2 columns.
hipError_t launch_projection(hipStream_t s, int prec, int scaling, int64_t m, int64_t k,
                             int64_t n2, const float *Q1, const float *A2, int64_t lda,
                             const float *colmax_a2, float *part, int splits);
hipError_t launch_proj_reduce(hipStream_t s, int prec, int scaling, int64_t k, int64_t n2,
                              const float *part, int splits, float *R12, int64_t ldr,
                              float *colmax_a2, float *uscale, float *Racc, int64_t ldacc,
                              uint16_t *Rh, uint16_t *Rl, int64_t ldh);
hipError_t launch_update(hipStream_t s, int prec, int scaling, int64_t m, int64_t k,
                         int64_t n2, const float *Q1, float *A2, int64_t lda,
                         const float *R12, int64_t ldr, const float *uscale,
                         float *colmax_a2, float *cmpart);
int64_t update_cmpart_slots(int64_t m);
hipError_t launch_colmax_reduce(hipStream_t s, int64_t n2, int64_t slots, const float *cmpart,
                                float *colmax);

// gemm_lp.hip : the same products in FP16 / BF16 / split FP16 on 16-bit operand
// copies. pack_q writes the copies of one panel's Q columns (times 2^14 when
// scaling): qc column-major (ldc), qr row-major (ldr), lo parts for split FP16;
// the pointers address the panel's first column. Projection reads qc at Q1's
// first column; the update reads qr there and Rh (k x n2, ld ldh) written by
// launch_proj_reduce.
hipError_t launch_pack_q(hipStream_t s, int prec, int scaling, int64_t m, int w, const float *Q,
                         int64_t ldq, uint16_t *qc, uint16_t *qcl, int64_t ldc, uint16_t *qr,
                         uint16_t *qrl, int64_t ldr);
hipError_t launch_projection_lp(hipStream_t s, int prec, int scaling, int64_t m, int64_t k,
                                int64_t n2, const uint16_t *qc, const uint16_t *qcl, int64_t ldc,
                                const float *A2, int64_t lda, const float *colmax, float *part,
                                int splits);
hipError_t launch_update_lp(hipStream_t s, int prec, int scaling, int64_t m, int64_t k,
                            int64_t n2, const uint16_t *qr, const uint16_t *qrl, int64_t ldq,
                            const uint16_t *rh, const uint16_t *rhl, int64_t ldh, float *A2,
                            int64_t lda, const float *uscale, float *colmax, float *cmpart);
// Row splits of a projection: about `target` workgroups (0 = default).
int projection_splits(int64_t m, int64_t k, int64_t n2, int prec, int target);
// Large-tile products (gemm_tn.hip): 256 x 256 tiles on 16-bit operands with
// 16-byte aligned rows; tn_eligible tells whether a product of rows x cols
// outputs can use them.
bool tn_eligible(int64_t rows, int64_t cols, int64_t ld_a, int64_t ld_b, const void *a,
                 const void *b);
int tn_projection_splits(int64_t m, int64_t k, int64_t n2, int target);
hipError_t launch_pack_cols(hipStream_t s, int prec, int scaling, int64_t m, int64_t n2,
                            const float *A2, int64_t lda, const float *colmax, uint16_t *bh,
                            uint16_t *bl, int64_t ldb);
hipError_t launch_projection_tn(hipStream_t s, int prec, int64_t m, int64_t k, int64_t n2,
                                const uint16_t *qc, const uint16_t *qcl, int64_t ldc,
                                const uint16_t *bh, const uint16_t *bl, int64_t ldb, float *part,
                                int splits);
hipError_t launch_update_tn(hipStream_t s, int prec, int scaling, int64_t m, int64_t k,
                            int64_t n2, const uint16_t *qr, const uint16_t *qrl, int64_t ldq,
                            const uint16_t *rh, const uint16_t *rhl, int64_t ldh, float *A2,
                            int64_t lda, const float *uscale, float *colmax, float *cmpart);

}  // namespace qrx
