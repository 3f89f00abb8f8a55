// Kernels used around the persistent Krylov iteration (Sec. 3.2.3): the
// direct start's A^T b (GEMV-T with FP64 partials over row splits, then the
// column sums in a fixed order: deterministic) and the zero fill of the
// n-vectors. The iteration itself, with its products, certification and
// restarts, is the persistent kernel of krylov_loop.hip.
#include "qrx_internal.hpp"
#include "krylov.hpp"

namespace qrx {

constexpr int KT = 256;

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

__global__ __launch_bounds__(KT) void zero_kernel(int64_t n, double *dst) {
    const int64_t j = (int64_t)blockIdx.x * KT + threadIdx.x;
    if (j < n) dst[j] = 0.0;
}

// ---------------------------------------------------------------------------
static unsigned nb256(int64_t n) { return (unsigned)((n + KT - 1) / KT); }
hipError_t kr_zero(hipStream_t s, int64_t n, double *dst) {
    hipLaunchKernelGGL(zero_kernel, dim3(nb256(n)), dim3(KT), 0, s, n, dst);
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
hipError_t kr_gemv_t(hipStream_t s, int64_t m, int64_t n, const float *A, int64_t lda,
                     const double *u, double *part) {
    const int vec = ((((uintptr_t)A) & 15) == 0) && (lda % 4 == 0);
    hipLaunchKernelGGL(gemv_t_kernel, dim3((unsigned)((n + GT_COLS - 1) / GT_COLS),
                                           kr_gemv_t_splits(m)),
                       dim3(KT), 0, s, m, n, A, lda, u, part, vec);
    return hipGetLastError();
}
hipError_t kr_combine_n(hipStream_t s, int64_t n, const double *part, int splits, double *z,
                        double *ssq) {
    hipLaunchKernelGGL(combine_n_kernel, dim3(nb256(n)), dim3(KT), 0, s, n, part, splits, z, ssq);
    return hipGetLastError();
}

}  // namespace qrx
