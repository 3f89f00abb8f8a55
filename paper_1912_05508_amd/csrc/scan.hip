// Input scan and small bookkeeping kernels.
//
// scan: one pass over A (m x n, column-major) computing per column the
// max-abs (for the power-of-two operand scaling of the low-precision
// products), the FP64 sum of squares (for ||A||_F of the normalised
// normal-equation error, Sec. 3.2.2) and a finite check; optionally writes a
// working copy W. One workgroup per column; streaming, HBM-bound
// (4 bytes read + 4 written per element with a copy).
#include "qrx_internal.hpp"

namespace qrx {

constexpr int kScanThreads = 256;

__global__ __launch_bounds__(kScanThreads) void scan_cols_kernel(
    int64_t m, const float *__restrict__ A, int64_t lda, float *__restrict__ W, int64_t ldw,
    float *__restrict__ colmax, double *__restrict__ colss, int *__restrict__ flags) {
    const int64_t j = blockIdx.x;
    const float *a = A + j * lda;
    float *w = W ? W + j * ldw : nullptr;
    float mx = 0.0f;
    double ss = 0.0;
    int bad = 0;
    const bool vec = ((((uintptr_t)a) & 15) == 0) && (!w || ((((uintptr_t)w) & 15) == 0));
    int64_t r0 = 0;
    if (vec) {
        const int64_t m4 = m & ~int64_t(3);
        for (int64_t r = int64_t(threadIdx.x) * 4; r < m4; r += kScanThreads * 4) {
            float4 v = *reinterpret_cast<const float4 *>(a + r);
            if (w) *reinterpret_cast<float4 *>(w + r) = v;
            float e[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                bad |= !isfinite(e[q]);
                mx = fmaxf(mx, fabsf(e[q]));
                ss = fma((double)e[q], (double)e[q], ss);
            }
        }
        r0 = m4;
    }
    for (int64_t r = r0 + threadIdx.x; r < m; r += kScanThreads) {
        float v = a[r];
        if (w) w[r] = v;
        bad |= !isfinite(v);
        mx = fmaxf(mx, fabsf(v));
        ss = fma((double)v, (double)v, ss);
    }
    __shared__ float smx[kScanThreads / 64];
    __shared__ double sss[kScanThreads / 64];
    __shared__ int sbad[kScanThreads / 64];
    mx = wave_max_f(mx);
    ss = wave_sum_d(ss);
    bad = __any(bad) ? 1 : 0;
    const int wv = threadIdx.x / 64;
    if ((threadIdx.x & 63) == 0) {
        smx[wv] = mx;
        sss[wv] = ss;
        sbad[wv] = bad;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        float M = smx[0];
        double S = sss[0];
        int B = sbad[0];
        for (int q = 1; q < kScanThreads / 64; ++q) {
            M = fmaxf(M, smx[q]);
            S += sss[q];
            B |= sbad[q];
        }
        colmax[j] = M;
        colss[j] = S;
        if (B) atomicOr(flags, 1);
    }
}

__global__ __launch_bounds__(kScanThreads) void scan_vec_kernel(int64_t m, const double *b,
                                                                int *flags) {
    int bad = 0;
    for (int64_t r = int64_t(blockIdx.x) * kScanThreads + threadIdx.x; r < m;
         r += int64_t(gridDim.x) * kScanThreads)
        bad |= !isfinite(b[r]);
    if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(flags, 1);
}

// ||A||_F = sqrt(sum_j colss[j]), fixed summation order (deterministic).
__global__ __launch_bounds__(256) void norm_finalize_kernel(int64_t n, const double *colss,
                                                            double *normA) {
    __shared__ double s[256];
    double acc = 0.0;
    for (int64_t j = threadIdx.x; j < n; j += 256) acc += colss[j];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) *normA = sqrt(s[0]);
}

__global__ void fill_f32_kernel(float *p, int64_t count, float v) {
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < count;
         i += int64_t(gridDim.x) * blockDim.x)
        p[i] = v;
}

// Zero the strictly-lower part of R and check its diagonal (a8): a zero or
// non-finite diagonal entry means A is not of full column rank in working
// precision -> flag bit 2 (QRX_ESINGULAR).
__global__ __launch_bounds__(256) void r_finalize_kernel(int64_t n, float *R, int64_t ldr,
                                                         int *flags) {
    const int64_t j = blockIdx.x;
    float *c = R + j * ldr;
    for (int64_t i = j + 1 + threadIdx.x; i < n; i += 256) c[i] = 0.0f;
    if (threadIdx.x == 0) {
        float d = c[j];
        if (!(d > 0.0f) || !isfinite(d)) atomicOr(flags, 2);
    }
}

// C = A B for upper-triangular A and B (n x n, FP32, column-major), FP64
// accumulation, into C (FP32, ldc) with its strictly-lower part zero: the R
// factor of a re-orthogonalised Q (R = R2 R). 64 x 64 tile per workgroup
// (4 x 4 outputs per thread, rows and columns 16 apart), K in stages of 32 over
// the range [i0, j0 + 63] where both triangles can be nonzero.
__global__ __launch_bounds__(256) void triu_mul_kernel(int64_t n, const float *__restrict__ A,
                                                       int64_t lda, const float *__restrict__ B,
                                                       int64_t ldb, float *__restrict__ C,
                                                       int64_t ldc) {
    __shared__ double As[32][65], Bs[32][65];   // As[k][i] = A(i0 + i, k0 + k), Bs[k][j]
    const int64_t i0 = (int64_t)blockIdx.x * 64, j0 = (int64_t)blockIdx.y * 64;
    const int t = threadIdx.x, ti = t % 16, tj = t / 16;
    double acc[4][4];
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[p][q] = 0.0;
    if (i0 <= j0) {
        const int64_t kend = (j0 + 64 < n) ? j0 + 64 : n;
        for (int64_t k0 = i0; k0 < kend; k0 += 32) {
            for (int e = t; e < 64 * 32; e += 256) {
                const int i = e % 64, k = e / 64;
                const int64_t gi = i0 + i, gk = k0 + k;
                As[k][i] = (gi < n && gk < n && gi <= gk) ? (double)A[gi + gk * lda] : 0.0;
                const int kk = e % 32, j = e / 32;
                const int64_t gk2 = k0 + kk, gj = j0 + j;
                Bs[kk][j] = (gk2 < n && gj < n && gk2 <= gj) ? (double)B[gk2 + gj * ldb] : 0.0;
            }
            __syncthreads();
            for (int k = 0; k < 32; ++k) {
                double a[4], b[4];
#pragma unroll
                for (int p = 0; p < 4; ++p) a[p] = As[k][ti + 16 * p];
#pragma unroll
                for (int q = 0; q < 4; ++q) b[q] = Bs[k][tj + 16 * q];
#pragma unroll
                for (int p = 0; p < 4; ++p)
#pragma unroll
                    for (int q = 0; q < 4; ++q) acc[p][q] = fma(a[p], b[q], acc[p][q]);
            }
            __syncthreads();
        }
    }
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int64_t i = i0 + ti + 16 * p, j = j0 + tj + 16 * q;
            if (i < n && j < n) C[i + j * ldc] = (i <= j) ? (float)acc[p][q] : 0.0f;
        }
}

// dst (rows x cols, ldd) = src (lds), FP32, column-major
__global__ __launch_bounds__(256) void copy_mat_kernel(int64_t rows, const float *__restrict__ src,
                                                       int64_t lds, float *__restrict__ dst,
                                                       int64_t ldd) {
    const int64_t j = blockIdx.y;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < rows; i += (int64_t)gridDim.x * 256)
        dst[i + j * ldd] = src[i + j * lds];
}

// Map the flag bits to one status value (non-finite input wins).
__global__ void status_out_kernel(const int *flags, int *status) {
    int f = *flags;
    *status = (f & 1) ? QRX_ENONFINITE : ((f & 2) ? QRX_ESINGULAR : QRX_OK);
}

hipError_t launch_scan(hipStream_t s, int64_t m, int64_t n, const float *A, int64_t lda,
                       float *W, int64_t ldw, float *colmax, double *colss, int *flags) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(scan_cols_kernel, dim3((unsigned)n), dim3(kScanThreads), 0, s, m, A,
                       lda, W, ldw, colmax, colss, flags);
    return hipGetLastError();
}

hipError_t launch_scan_vec(hipStream_t s, int64_t m, const double *b, int *flags) {
    int64_t blocks = (m + kScanThreads - 1) / kScanThreads;
    if (blocks > 1024) blocks = 1024;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(scan_vec_kernel, dim3((unsigned)blocks), dim3(kScanThreads), 0, s, m, b,
                       flags);
    return hipGetLastError();
}

hipError_t launch_norm_finalize(hipStream_t s, int64_t n, const double *colss, double *normA) {
    hipLaunchKernelGGL(norm_finalize_kernel, dim3(1), dim3(256), 0, s, n, colss, normA);
    return hipGetLastError();
}

hipError_t launch_fill_f32(hipStream_t s, float *p, int64_t count, float v) {
    if (count <= 0) return hipSuccess;
    int64_t blocks = (count + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(fill_f32_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, count, v);
    return hipGetLastError();
}

hipError_t launch_r_finalize(hipStream_t s, int64_t n, float *R, int64_t ldr, int *flags) {
    hipLaunchKernelGGL(r_finalize_kernel, dim3((unsigned)n), dim3(256), 0, s, n, R, ldr, flags);
    return hipGetLastError();
}

hipError_t launch_triu_mul(hipStream_t s, int64_t n, const float *A, int64_t lda, const float *B,
                           int64_t ldb, float *C, int64_t ldc) {
    if (n <= 0) return hipSuccess;
    const unsigned nb = (unsigned)((n + 63) / 64);
    if (nb > 65535) return hipErrorInvalidValue;
    hipLaunchKernelGGL(triu_mul_kernel, dim3(nb, nb), dim3(256), 0, s, n, A, lda, B, ldb, C, ldc);
    return hipGetLastError();
}

hipError_t launch_copy_mat(hipStream_t s, int64_t rows, int64_t cols, const float *src,
                           int64_t lds, float *dst, int64_t ldd) {
    if (rows <= 0 || cols <= 0) return hipSuccess;
    if (cols > 65535) return hipErrorInvalidValue;
    int64_t gx = (rows + 255) / 256;
    if (gx > 64) gx = 64;
    hipLaunchKernelGGL(copy_mat_kernel, dim3((unsigned)gx, (unsigned)cols), dim3(256), 0, s, rows,
                       src, lds, dst, ldd);
    return hipGetLastError();
}

hipError_t launch_status_out(hipStream_t s, const int *flags, int *status) {
    hipLaunchKernelGGL(status_out_kernel, dim3(1), dim3(1), 0, s, flags, status);
    return hipGetLastError();
}

}  // namespace qrx
