// Kernels of the right-preconditioned Krylov least-squares iteration
// (Sec. 3.2.3, Alg. 5; LSQR as the default variant).
//
// Per iteration the operator B = A R^{-1} and its transpose are applied as
//   t = X v      (X = R^{-1} formed once in FP64, trinv.hip),
//   q = A t      (GEMV-N: FP32 A streamed once, FP64 FMA),
//   z = A^T u    (GEMV-T),
//   v = X^T z.
// Both GEMVs split their reduction dimension over workgroups and sum the
// FP64 partials in a fixed order (deterministic). The true residual
// r = b - A x is accumulated in double-double so the certified eta_F is not
// limited by FP64 cancellation.
#include "qrx_internal.hpp"
#include "krylov.hpp"

namespace qrx {

constexpr int KT = 256;

// ---- GEMV-N partials: part[s][r] = sum_{j in split s} A[r, j] x[j] --------
// mode 0: FP64 accumulation; mode 1: double-double (hi in part, lo in part2).
__global__ __launch_bounds__(KT) void gemv_n_kernel(int64_t m, int64_t n,
                                                    const float *__restrict__ A, int64_t lda,
                                                    const double *__restrict__ x, int64_t cchunk,
                                                    double *__restrict__ part,
                                                    double *__restrict__ part2, int vec, int dd) {
    const int64_t s = blockIdx.y;
    const int64_t r = ((int64_t)blockIdx.x * KT + threadIdx.x) * 4;
    const int64_t j0 = s * cchunk;
    const int64_t j1 = (j0 + cchunk < n) ? j0 + cchunk : n;
    double h[4] = {0, 0, 0, 0}, l[4] = {0, 0, 0, 0};
    if (r < m) {
        const bool v4 = vec && (r + 3 < m);
        int64_t j = j0;
        if (v4 && !dd) {
            // GU column loads in flight per wave (one at a time leaves HBM
            // latency-bound); the sums keep the column order of the loop below
            constexpr int GU = 8;
            for (; j + GU <= j1; j += GU) {
                float4 q[GU];
#pragma unroll
                for (int u = 0; u < GU; ++u)
                    q[u] = *reinterpret_cast<const float4 *>(A + (j + u) * lda + r);
#pragma unroll
                for (int u = 0; u < GU; ++u) {
                    const double xj = x[j + u];
                    h[0] = fma((double)q[u].x, xj, h[0]);
                    h[1] = fma((double)q[u].y, xj, h[1]);
                    h[2] = fma((double)q[u].z, xj, h[2]);
                    h[3] = fma((double)q[u].w, xj, h[3]);
                }
            }
        }
        for (; j < j1; ++j) {
            const double xj = x[j];
            const float *a = A + j * lda + r;
            float e[4];
            if (v4) {
                float4 q = *reinterpret_cast<const float4 *>(a);
                e[0] = q.x; e[1] = q.y; e[2] = q.z; e[3] = q.w;
            } else {
#pragma unroll
                for (int k = 0; k < 4; ++k) e[k] = (r + k < m) ? a[k] : 0.0f;
            }
            if (dd) {
#pragma unroll
                for (int k = 0; k < 4; ++k) dd_add_prod(h[k], l[k], (double)e[k], xj);
            } else {
#pragma unroll
                for (int k = 0; k < 4; ++k) h[k] = fma((double)e[k], xj, h[k]);
            }
        }
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (r + k < m) {
                part[s * m + r + k] = h[k];
                if (dd) part2[s * m + r + k] = l[k];
            }
    }
}

// ---- GEMV-T partials: part[s][j] = sum_{r in split s} A[r, j] u[r] --------
constexpr int GT_ROWS = 4096;   // rows per split (u slice kept in LDS)
constexpr int GT_COLS = 16;     // columns per workgroup (4 per wave)
__global__ __launch_bounds__(KT) void gemv_t_kernel(int64_t m, int64_t n,
                                                    const float *__restrict__ A, int64_t lda,
                                                    const double *__restrict__ u,
                                                    double *__restrict__ part, int vec) {
    __shared__ double us[GT_ROWS];
    const int64_t s = blockIdx.y;
    const int64_t rs = s * GT_ROWS;
    const int64_t re = (rs + GT_ROWS < m) ? rs + GT_ROWS : m;
    const int cnt = (int)(re - rs);
    for (int i = threadIdx.x; i < GT_ROWS; i += KT) us[i] = (i < cnt) ? u[rs + i] : 0.0;
    __syncthreads();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    constexpr int CW = GT_COLS / 4;   // columns per wave, swept together (one u read each)
    const int64_t j0 = (int64_t)blockIdx.x * GT_COLS + wv * CW;
    const float *a[CW];
    bool jin[CW];
#pragma unroll
    for (int q = 0; q < CW; ++q) {
        jin[q] = j0 + q < n;
        a[q] = A + (jin[q] ? j0 + q : n - 1) * lda + rs;   // out of range: read a valid column
    }
    double acc[CW];
#pragma unroll
    for (int q = 0; q < CW; ++q) acc[q] = 0.0;
    if (vec) {
        // rows i .. i + 3 of the lane's CW columns per block; two blocks' loads
        // in flight, then one, then the ragged end (rows in ascending order)
        auto block = [&](const float4 *e, int i) {
            const double u0 = us[i], u1 = us[i + 1], u2 = us[i + 2], u3 = us[i + 3];
#pragma unroll
            for (int q = 0; q < CW; ++q) {
                acc[q] = fma((double)e[q].x, u0, acc[q]);
                acc[q] = fma((double)e[q].y, u1, acc[q]);
                acc[q] = fma((double)e[q].z, u2, acc[q]);
                acc[q] = fma((double)e[q].w, u3, acc[q]);
            }
        };
        const int cnt4 = cnt & ~3;
        int i = lane * 4;
        for (; i + 256 < cnt4; i += 512) {
            float4 e0[CW], e1[CW];
#pragma unroll
            for (int q = 0; q < CW; ++q) e0[q] = *reinterpret_cast<const float4 *>(a[q] + i);
#pragma unroll
            for (int q = 0; q < CW; ++q) e1[q] = *reinterpret_cast<const float4 *>(a[q] + i + 256);
            block(e0, i);
            block(e1, i + 256);
        }
        for (; i < cnt4; i += 256) {
            float4 e0[CW];
#pragma unroll
            for (int q = 0; q < CW; ++q) e0[q] = *reinterpret_cast<const float4 *>(a[q] + i);
            block(e0, i);
        }
        if (i < cnt) {
            for (int k = 0; k < 4 && i + k < cnt; ++k)
#pragma unroll
                for (int q = 0; q < CW; ++q) acc[q] = fma((double)a[q][i + k], us[i + k], acc[q]);
        }
    } else {
        for (int i = lane; i < cnt; i += 64)
#pragma unroll
            for (int q = 0; q < CW; ++q) acc[q] = fma((double)a[q][i], us[i], acc[q]);
    }
#pragma unroll
    for (int q = 0; q < CW; ++q) {
        const double v = wave_sum_d(acc[q]);
        if (lane == 0 && jin[q]) part[s * n + j0 + q] = v;
    }
}

// ---- deterministic sum of `count` doubles by one workgroup -----------------
QRX_DEV double block_sum(const double *p, int64_t count) {
    __shared__ double sh[KT];
    double a = 0.0;
    for (int64_t i = threadIdx.x; i < count; i += KT) a += p[i];
    sh[threadIdx.x] = a;
    __syncthreads();
    for (int o = KT / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    double r = sh[0];
    __syncthreads();
    return r;
}

// Per-workgroup partial of sum(v^2) written to ssq[blockIdx.x].
QRX_DEV void block_ssq_out(double v2, double *ssq) {
    __shared__ double sh[KT / 64];
    double w = wave_sum_d(v2);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = w;
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0.0;
        for (int i = 0; i < KT / 64; ++i) a += sh[i];
        ssq[blockIdx.x] = a;
    }
}

// out[r] = sum_s part[s][r] + a * y[r]  (y may be null); ssq partials.
__global__ __launch_bounds__(KT) void combine_m_kernel(int64_t m, const double *__restrict__ part,
                                                       int splits, const double *__restrict__ coef,
                                                       int ci, int cdiv, double *__restrict__ y_inout,
                                                       double *__restrict__ out,
                                                       double *__restrict__ ssq) {
    const int64_t r = (int64_t)blockIdx.x * KT + threadIdx.x;
    double v2 = 0.0;
    if (r < m) {
        double s = 0.0;
        for (int q = 0; q < splits; ++q) s += part[(int64_t)q * m + r];
        if (y_inout) s -= (coef[ci] / (cdiv >= 0 ? coef[cdiv] : 1.0)) * y_inout[r];
        out[r] = s;
        v2 = s * s;
    }
    block_ssq_out(v2, ssq);
}

// r = b - sum_s (hi_s + lo_s) in double-double, rounded; ssq partials.
__global__ __launch_bounds__(KT) void resid_combine_kernel(int64_t m, const double *__restrict__ b,
                                                           const double *__restrict__ hi,
                                                           const double *__restrict__ lo,
                                                           int splits, double *__restrict__ r_out,
                                                           double *__restrict__ ssq) {
    const int64_t r = (int64_t)blockIdx.x * KT + threadIdx.x;
    double v2 = 0.0;
    if (r < m) {
        double h = b[r], l = 0.0;
        for (int q = 0; q < splits; ++q) {
            dd_add(h, l, -hi[(int64_t)q * m + r]);
            dd_add(h, l, -lo[(int64_t)q * m + r]);
        }
        double v = h + l;
        r_out[r] = v;
        v2 = v * v;
    }
    block_ssq_out(v2, ssq);
}

// z[j] = sum_s part[s][j]; ssq partials.
__global__ __launch_bounds__(KT) void combine_n_kernel(int64_t n, const double *__restrict__ part,
                                                       int splits, double *__restrict__ z,
                                                       double *__restrict__ ssq) {
    const int64_t j = (int64_t)blockIdx.x * KT + threadIdx.x;
    double v2 = 0.0;
    if (j < n) {
        // CU partials loaded at a time (n is small: few workgroups), added in split order
        constexpr int CU = 16;
        double s = 0.0;
        int q = 0;
        for (; q + CU <= splits; q += CU) {
            double pv[CU];
#pragma unroll
            for (int u = 0; u < CU; ++u) pv[u] = part[(int64_t)(q + u) * n + j];
#pragma unroll
            for (int u = 0; u < CU; ++u) s += pv[u];
        }
        for (; q < splits; ++q) s += part[(int64_t)q * n + j];
        z[j] = s;
        v2 = s * s;
    }
    block_ssq_out(v2, ssq);
}

// out[j] = a * x[j] + bsign * b * y[j] (coefficients from the state array;
// index -1 = 0, index -2 = 1; a is divided by st[ia_div] when ia_div >= 0);
// ssq partials of out.
__global__ __launch_bounds__(KT) void axpby_kernel(int64_t n, const double *__restrict__ st,
                                                   int ia, int ia_div, const double *__restrict__ x,
                                                   int ib, double bsign,
                                                   const double *__restrict__ y,
                                                   double *__restrict__ out,
                                                   double *__restrict__ ssq) {
    const int64_t j = (int64_t)blockIdx.x * KT + threadIdx.x;
    const double a = (ia == -2 ? 1.0 : (ia == -1 ? 0.0 : st[ia])) / (ia_div >= 0 ? st[ia_div] : 1.0);
    const double bb = bsign * (ib == -2 ? 1.0 : (ib == -1 ? 0.0 : st[ib]));
    double v2 = 0.0;
    if (j < n) {
        double v = a * x[j] + (y ? bb * y[j] : 0.0);
        out[j] = v;
        v2 = v * v;
    }
    if (ssq) block_ssq_out(v2, ssq);
}

// ---- scalar steps (single workgroup) ---------------------------------------
// st[IDX] = sqrt(sum ssq) (or the plain sum when do_sqrt = 0)
__global__ __launch_bounds__(KT) void norm_kernel(const double *__restrict__ ssq, int64_t count,
                                                  double *__restrict__ st, int idx, int do_sqrt) {
    double s = block_sum(ssq, count);
    if (threadIdx.x == 0) st[idx] = do_sqrt ? sqrt(s) : s;
}

// One LSQR scalar step (Paige & Saunders), after alpha = ||v~||, beta known.
__global__ void lsqr_scalar_kernel(double *st, double tol) {
    double alpha = st[S_ALPHA], beta = st[S_BETA];
    double rhobar = st[S_RHOBAR], phibar = st[S_PHIBAR];
    double rho = hypot(rhobar, beta);
    double c = rhobar / rho, s = beta / rho;
    double theta = s * alpha;
    st[S_RHOBAR] = -c * alpha;
    double phi = c * phibar;
    st[S_PHIBAR] = s * phibar;
    st[S_XCOEF] = phi / rho;
    st[S_DCOEF_NEXT] = theta / rho;
    double est = alpha * fabs(c);           // ||B^T r|| / ||r||
    st[S_EST] = est;
    st[S_FLAG] = (est <= tol * st[S_GAMMA_TOL] || alpha == 0.0 || beta == 0.0) ? 1.0 : 0.0;
}

// t-direction update d = t - dcoef * d, then x += xcoef * d; v = v~ / alpha.
__global__ __launch_bounds__(KT) void lsqr_xd_kernel(int64_t n, const double *__restrict__ st,
                                                     const double *__restrict__ t,
                                                     double *__restrict__ d,
                                                     double *__restrict__ x,
                                                     double *__restrict__ v, int first) {
    const int64_t j = (int64_t)blockIdx.x * KT + threadIdx.x;
    if (j < n) {
        double dj = first ? t[j] : t[j] - st[S_DCOEF] * d[j];
        d[j] = dj;
        x[j] = fma(st[S_XCOEF], dj, x[j]);
        const double a = st[S_ALPHA];
        v[j] = a > 0.0 ? v[j] / a : 0.0;
    }
}

__global__ void lsqr_shift_kernel(double *st) { st[S_DCOEF] = st[S_DCOEF_NEXT]; }

// eta_F = ||z|| / (||A||_F ||r||) from the certification pass, and the
// compatible-system ratio ||r|| / (||A||_F ||x|| + ||b||) times cscale (see
// compat_scale); the score is the smaller of the two (converged when score <= tol).
__global__ void eta_kernel(double *st, double tol, double cscale) {
    double nr = st[S_RNORM], nz = st[S_ZNORM], na = st[S_NORMA];
    double e = (nr > 0.0 && na > 0.0) ? nz / (na * nr) : 0.0;
    double den = na * st[S_XNORM] + st[S_BNORM];
    double s1 = den > 0.0 ? cscale * (nr / den) : 0.0;
    st[S_ETA] = e;
    st[S_SCORE] = fmin(e, s1);
    st[S_CONV] = (fmin(e, s1) <= tol) ? 1.0 : 0.0;
}

// LSQR (re)start from the certified residual r (length m) and z = A^T r:
// u = r (beta = ||r||), v~ = R^{-T} z / beta computed by the caller.
__global__ void lsqr_restart_scalar_kernel(double *st) {
    st[S_BETA] = st[S_RNORM];
    st[S_PHIBAR] = st[S_RNORM];
}
__global__ void lsqr_restart2_kernel(double *st) {
    st[S_RHOBAR] = st[S_ALPHA];
    st[S_DCOEF] = 0.0;
}

// CGLS scalars
__global__ void cgls_alpha_kernel(double *st) {   // alpha = gamma / delta
    double d = st[S_DELTA];
    st[S_CGALPHA] = d > 0.0 ? st[S_GAMMA] / d : 0.0;
}
__global__ void cgls_beta_kernel(double *st, double tol) {   // beta = gamma'/gamma
    double g1 = st[S_GAMMA], g = st[S_GAMMANEW];
    st[S_CGBETA] = g1 > 0.0 ? g / g1 : 0.0;
    st[S_GAMMA] = g;
    double nr = sqrt(st[S_RSS]);
    double est = nr > 0.0 ? sqrt(g) / nr : 0.0;   // ||R^{-T} A^T r|| / ||r||
    st[S_EST] = est;
    st[S_FLAG] = (est <= tol * st[S_GAMMA_TOL] || g == 0.0) ? 1.0 : 0.0;
}
// x += alpha t (n); r -= alpha q (m); ssq of r
__global__ __launch_bounds__(KT) void cgls_xr_kernel(int64_t m, int64_t n, const double *st,
                                                     const double *t, double *x, const double *q,
                                                     double *r, double *ssq) {
    const int64_t i = (int64_t)blockIdx.x * KT + threadIdx.x;
    const double a = st[S_CGALPHA];
    if (i < n) x[i] = fma(a, t[i], x[i]);
    double v2 = 0.0;
    if (i < m) {
        double v = fma(-a, q[i], r[i]);
        r[i] = v;
        v2 = v * v;
    }
    block_ssq_out(v2, ssq);
}

__global__ void set_kernel(double *st, int idx, double v) { st[idx] = v; }
__global__ __launch_bounds__(KT) void copy_kernel(int64_t n, const double *src, double *dst) {
    const int64_t j = (int64_t)blockIdx.x * KT + threadIdx.x;
    if (j < n) dst[j] = src[j];
}
__global__ __launch_bounds__(KT) void zero_kernel(int64_t n, double *dst) {
    const int64_t j = (int64_t)blockIdx.x * KT + threadIdx.x;
    if (j < n) dst[j] = 0.0;
}

// ---------------------------------------------------------------------------
static unsigned nb256(int64_t n) { return (unsigned)((n + KT - 1) / KT); }

hipError_t kr_copy(hipStream_t s, int64_t n, const double *src, double *dst) {
    hipLaunchKernelGGL(copy_kernel, dim3(nb256(n)), dim3(KT), 0, s, n, src, dst);
    return hipGetLastError();
}
hipError_t kr_zero(hipStream_t s, int64_t n, double *dst) {
    hipLaunchKernelGGL(zero_kernel, dim3(nb256(n)), dim3(KT), 0, s, n, dst);
    return hipGetLastError();
}
hipError_t kr_set(hipStream_t s, double *st, int idx, double v) {
    hipLaunchKernelGGL(set_kernel, dim3(1), dim3(1), 0, s, st, idx, v);
    return hipGetLastError();
}

int kr_gemv_n_splits(int64_t m, int64_t n) {
    const int64_t rb = (m + 1023) / 1024;
    int64_t s = (1024 + rb - 1) / rb;
    int64_t smax = (n + 63) / 64;
    if (s > smax) s = smax;
    if (s < 1) s = 1;
    if (s > 64) s = 64;
    return (int)s;
}
int kr_gemv_t_splits(int64_t m) { return (int)((m + GT_ROWS - 1) / GT_ROWS); }

hipError_t kr_gemv_n(hipStream_t s, int64_t m, int64_t n, const float *A, int64_t lda,
                     const double *x, double *part, double *part2, int splits, int dd) {
    const int64_t cchunk = (n + splits - 1) / splits;
    const int vec = ((((uintptr_t)A) & 15) == 0) && (lda % 4 == 0);
    hipLaunchKernelGGL(gemv_n_kernel, dim3((unsigned)((m + 1023) / 1024), splits), dim3(KT), 0, s,
                       m, n, A, lda, x, cchunk, part, part2, vec, dd);
    return hipGetLastError();
}

hipError_t kr_gemv_t(hipStream_t s, int64_t m, int64_t n, const float *A, int64_t lda,
                     const double *u, double *part) {
    const int vec = ((((uintptr_t)A) & 15) == 0) && (lda % 4 == 0);
    hipLaunchKernelGGL(gemv_t_kernel, dim3((unsigned)((n + GT_COLS - 1) / GT_COLS),
                                           kr_gemv_t_splits(m)),
                       dim3(KT), 0, s, m, n, A, lda, u, part, vec);
    return hipGetLastError();
}

hipError_t kr_combine_m(hipStream_t s, int64_t m, const double *part, int splits,
                        const double *st, int ci, int cdiv, double *y_inout, double *out,
                        double *ssq) {
    hipLaunchKernelGGL(combine_m_kernel, dim3(nb256(m)), dim3(KT), 0, s, m, part, splits, st, ci,
                       cdiv, y_inout, out, ssq);
    return hipGetLastError();
}
hipError_t kr_resid_combine(hipStream_t s, int64_t m, const double *b, const double *hi,
                            const double *lo, int splits, double *r, double *ssq) {
    hipLaunchKernelGGL(resid_combine_kernel, dim3(nb256(m)), dim3(KT), 0, s, m, b, hi, lo, splits,
                       r, ssq);
    return hipGetLastError();
}
hipError_t kr_combine_n(hipStream_t s, int64_t n, const double *part, int splits, double *z,
                        double *ssq) {
    hipLaunchKernelGGL(combine_n_kernel, dim3(nb256(n)), dim3(KT), 0, s, n, part, splits, z, ssq);
    return hipGetLastError();
}
hipError_t kr_axpby(hipStream_t s, int64_t n, const double *st, int ia, int ia_div,
                    const double *x, int ib, double bsign, const double *y, double *out,
                    double *ssq) {
    hipLaunchKernelGGL(axpby_kernel, dim3(nb256(n)), dim3(KT), 0, s, n, st, ia, ia_div, x, ib,
                       bsign, y, out, ssq);
    return hipGetLastError();
}
hipError_t kr_norm(hipStream_t s, const double *ssq, int64_t count, double *st, int idx, int do_sqrt) {
    hipLaunchKernelGGL(norm_kernel, dim3(1), dim3(KT), 0, s, ssq, count, st, idx, do_sqrt);
    return hipGetLastError();
}
hipError_t kr_lsqr_scalar(hipStream_t s, double *st, double tol) {
    hipLaunchKernelGGL(lsqr_scalar_kernel, dim3(1), dim3(1), 0, s, st, tol);
    return hipGetLastError();
}
hipError_t kr_lsqr_xd(hipStream_t s, int64_t n, const double *st, const double *t, double *d,
                      double *x, double *v, int first) {
    hipLaunchKernelGGL(lsqr_xd_kernel, dim3(nb256(n)), dim3(KT), 0, s, n, st, t, d, x, v, first);
    return hipGetLastError();
}
hipError_t kr_lsqr_shift(hipStream_t s, double *st) {
    hipLaunchKernelGGL(lsqr_shift_kernel, dim3(1), dim3(1), 0, s, st);
    return hipGetLastError();
}
hipError_t kr_eta(hipStream_t s, double *st, double tol, double cscale) {
    hipLaunchKernelGGL(eta_kernel, dim3(1), dim3(1), 0, s, st, tol, cscale);
    return hipGetLastError();
}
hipError_t kr_lsqr_restart(hipStream_t s, double *st, int phase) {
    if (phase == 0)
        hipLaunchKernelGGL(lsqr_restart_scalar_kernel, dim3(1), dim3(1), 0, s, st);
    else
        hipLaunchKernelGGL(lsqr_restart2_kernel, dim3(1), dim3(1), 0, s, st);
    return hipGetLastError();
}
hipError_t kr_cgls_alpha(hipStream_t s, double *st) {
    hipLaunchKernelGGL(cgls_alpha_kernel, dim3(1), dim3(1), 0, s, st);
    return hipGetLastError();
}
hipError_t kr_cgls_beta(hipStream_t s, double *st, double tol) {
    hipLaunchKernelGGL(cgls_beta_kernel, dim3(1), dim3(1), 0, s, st, tol);
    return hipGetLastError();
}
hipError_t kr_cgls_xr(hipStream_t s, int64_t m, int64_t n, const double *st, const double *t,
                      double *x, const double *q, double *r, double *ssq) {
    const int64_t mx = m > n ? m : n;
    hipLaunchKernelGGL(cgls_xr_kernel, dim3(nb256(mx)), dim3(KT), 0, s, m, n, st, t, x, q, r, ssq);
    return hipGetLastError();
}

}  // namespace qrx
