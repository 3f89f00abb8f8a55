// Krylov kernel launchers and the layout of the device-side scalar state.
#pragma once
#include "qrx_internal.hpp"

namespace qrx {

// Indices into the FP64 scalar state array (device memory).
enum {
    S_ALPHA = 0, S_BETA, S_RHOBAR, S_PHIBAR, S_XCOEF, S_DCOEF, S_DCOEF_NEXT, S_EST, S_FLAG,
    S_GAMMA_TOL,           // trigger slack: stop estimate <= tol * this
    S_RNORM, S_ZNORM, S_NORMA, S_ETA, S_CONV,
    S_DELTA, S_GAMMA, S_GAMMANEW, S_CGALPHA, S_CGBETA, S_RSS,
    S_XNORM, S_BNORM, S_SCORE,
    S_COUNT
};

hipError_t kr_copy(hipStream_t s, int64_t n, const double *src, double *dst);
hipError_t kr_zero(hipStream_t s, int64_t n, double *dst);
hipError_t kr_set(hipStream_t s, double *st, int idx, double v);
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
hipError_t kr_gemv_n(hipStream_t s, int64_t m, int64_t n, const float *A, int64_t lda,
                     const double *x, double *part, double *part2, int splits, int dd);
hipError_t kr_gemv_t(hipStream_t s, int64_t m, int64_t n, const float *A, int64_t lda,
                     const double *u, double *part);
hipError_t kr_combine_m(hipStream_t s, int64_t m, const double *part, int splits,
                        const double *st, int ci, int cdiv, double *y_inout, double *out,
                        double *ssq);
hipError_t kr_resid_combine(hipStream_t s, int64_t m, const double *b, const double *hi,
                            const double *lo, int splits, double *r, double *ssq);
hipError_t kr_combine_n(hipStream_t s, int64_t n, const double *part, int splits, double *z,
                        double *ssq);
hipError_t kr_axpby(hipStream_t s, int64_t n, const double *st, int ia, int ia_div,
                    const double *x, int ib, double bsign, const double *y, double *out,
                    double *ssq);
hipError_t kr_norm(hipStream_t s, const double *ssq, int64_t count, double *st, int idx, int do_sqrt);
hipError_t kr_lsqr_scalar(hipStream_t s, double *st, double tol);
hipError_t kr_lsqr_xd(hipStream_t s, int64_t n, const double *st, const double *t, double *d,
                      double *x, double *v, int first);
hipError_t kr_lsqr_shift(hipStream_t s, double *st);
hipError_t kr_eta(hipStream_t s, double *st, double tol, double cscale);
hipError_t kr_lsqr_restart(hipStream_t s, double *st, int phase);
hipError_t kr_cgls_alpha(hipStream_t s, double *st);
hipError_t kr_cgls_beta(hipStream_t s, double *st, double tol);
hipError_t kr_cgls_xr(hipStream_t s, int64_t m, int64_t n, const double *st, const double *t,
                      double *x, const double *q, double *r, double *ssq);

}  // namespace qrx
