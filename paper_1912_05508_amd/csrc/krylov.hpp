// Krylov launchers: the kernels around the persistent iteration (krylov.hip,
// trinv.hip) and the persistent iteration itself (krylov_loop.hip).
#pragma once
#include "qrx_internal.hpp"

namespace qrx {

hipError_t kr_zero(hipStream_t s, int64_t n, double *dst);
// trinv.hip: X = R^{-1} (np x np FP64, ld np; np a multiple of 256; T holds
// kr_trinv_tmp_doubles(np)), and out = X in (trans 0) or X^T in (trans 1),
// part holding kr_trmv_part_doubles(np).
hipError_t kr_trinv(hipStream_t s, int64_t n, int64_t np, const float *R, int64_t ldr, double *X,
                    double *T);
size_t kr_trinv_tmp_doubles(int64_t np);
size_t kr_trmv_part_doubles(int64_t np);
hipError_t kr_trmv(hipStream_t s, int64_t np, const double *X, const double *in, double *out,
                   double *part, int trans);
int kr_gemv_n_splits(int64_t m, int64_t n);
int kr_gemv_t_splits(int64_t m);
hipError_t kr_gemv_t(hipStream_t s, int64_t m, int64_t n, const float *A, int64_t lda,
                     const double *u, double *part);
hipError_t kr_combine_n(hipStream_t s, int64_t n, const double *part, int splits, double *z,
                        double *ssq);
// Xt = X^T for np x np FP64 matrices (ld np).
hipError_t kr_transpose(hipStream_t s, int64_t np, const double *X, double *Xt);

// krylov_loop.hip: the whole Krylov iteration as one persistent kernel.
struct KLoopArgs {
    int64_t m, n, np, lda;
    const float *A;                 // m x n FP32 (lda)
    const double *b;                // m
    const double *X, *Xt;           // R^{-1} and its transpose (np x np, ld np); null = identity
    const double *colss, *normA;    // column sums of squares and ||A||_F from the scan
    const int *flags;               // scan / factorisation status flags (bit 0 non-finite, 1 singular)
    double *x, *xbest, *u, *u2, *rc, *q, *r, *v, *vn, *t, *t2, *d, *z, *vt;   // np- or m-vectors
    double *xlo;                    // np: low parts of x (x + xlo accumulates the updates of
                                    // one restart in double-double; zero at each restart)
    double *pn, *pn2, *pt;          // GEMV partials: splits_n x m (two), splits_t x np
    double *pf;                     // one-pass partials of A^T u: n x grid (fused only)
    double *ssqA, *ssqB;            // kr_loop_ssq_doubles(m, np) each
    unsigned *bar;                  // 64 barrier words, zero at launch (word 2: abort flag;
                                    // bytes 16..23: the 64-bit arrival count)
    double *x_user;                 // n: receives the best certified iterate
    qrx_lls_info *info;             // device
    int splits_n, splits_t;
    int64_t cchunk;                 // GEMV-N columns per split
    int vec;                        // A 16-byte aligned with lda % 4 == 0
    int fused;                      // LSQR takes A t and A^T u~ in one pass over A (n <= kr_fused_max_n)
    int method, max_iter;
    double tol, cscale;
    long long *prof;                // null, or 2 * KP_COUNT entries: wall-clock ticks and
                                    // barrier count per phase (workgroup 0's view)
};
// Phases of the persistent Krylov kernel, for its per-phase timing.
enum {
    KP_INIT = 0, KP_CERTIFY, KP_RESTART, KP_TRMV_N, KP_GEMV_N, KP_COMBINE_M, KP_GEMV_T,
    KP_COMBINE_N, KP_TRMV_T, KP_UPDATE, KP_FUSED,
    // the four steps of a certification (KP_CERTIFY: returning to the best x)
    KP_CERT_GEMV_N, KP_CERT_RESID, KP_CERT_GEMV_T, KP_CERT_COMBINE, KP_COUNT
};
// Largest n for the one-pass LSQR products, and the most workgroups a
// persistent Krylov launch uses (the fused partials are sized for it).
constexpr int64_t kr_fused_max_n = 1024;
constexpr int kr_max_grid = 1024;
size_t kr_loop_ssq_doubles(int64_t m, int64_t np);
// Whether an m x n matrix with leading dimension lda (16-byte aligned, lda % 4
// == 0) can take the one-pass LSQR products (n <= kr_fused_max_n and the byte
// offsets of its loads within 32 bits).
bool kr_fused_ok(int64_t m, int64_t n, int64_t lda);
// Workgroups of the persistent launch (co-resident on `device`).
int kr_loop_grid(int device, int64_t m, int64_t n);
hipError_t kr_loop(hipStream_t s, const KLoopArgs &a, int grid);

}  // namespace qrx
