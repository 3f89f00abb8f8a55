// TSQR panel factorisation (Sec. 3.1.3, eq. caqr) with modified Gram-Schmidt
// blocks (Alg. 4), run twice per block (re-orthogonalisation, Sec. 4.1.2).
//
// A panel of m rows and w <= 32 columns is cut into row blocks of at most 256
// rows (balanced: sizes differ by at most one row). One workgroup of 256
// threads factors one block, each thread holding one row of the block in
// registers; the inner products of each MGS step are reduced through LDS.
// Q of the block overwrites the block in place, its 32 x 32 R goes to the
// stack of the next level (step 2 of eq. caqr). The stack is factored the
// same way, in groups of at most 8 R factors, until one block remains
// (step 3). The Q-formation kernel then multiplies every level-0 block by the
// product of the tree Q slices above it (steps 4-5).
//
// Column scaling: level 0 multiplies column j by an exact power of two taken
// from its max-abs so that sums of squares neither underflow nor overflow in
// FP32; the final R is unscaled column by column (exact).
#include "qrx_internal.hpp"

namespace qrx {

constexpr int NB = 32;
constexpr int PT = kPanelThreads;   // 256 rows per block
constexpr int LDR = PT + 8;         // padded LDS row of the product buffer

// One MGS sweep over the w active columns held in q (one row per thread).
// Rm receives R row-major (Rm[k*NB + j]); rows/cols >= w stay zero.
QRX_DEV void mgs_sweep(float (&q)[NB], int w, float *red, float *rowv, float *Rm) {
    const int t = threadIdx.x;
#pragma unroll
    for (int k = 0; k < NB; ++k) {
        if (k < w) {
            const int V = NB - k;
            // products of column k with columns k..NB-1 of this row
#pragma unroll
            for (int j = k; j < NB; ++j) red[(j - k) * LDR + t] = q[k] * q[j];
            __syncthreads();
            // G consecutive threads reduce one value over the 256 rows
            int G = 64;
            while (G * V > PT) G >>= 1;
            if (t < V * G) {
                const int v = t / G, sub = t - v * G;
                const float *src = red + v * LDR + sub;
                float acc = 0.0f;
                for (int i = 0; i < PT; i += G) acc += src[i];
                for (int o = G >> 1; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
                if (sub == 0) rowv[(k & 1) * NB + k + v] = acc;
            }
            __syncthreads();
            const float *row = rowv + (k & 1) * NB;
            const float rkk = sqrtf(row[k]);
            const float inv = rkk > 0.0f ? 1.0f / rkk : 0.0f;
            q[k] *= inv;
#pragma unroll
            for (int j = k + 1; j < NB; ++j) {
                const float rkj = row[j] * inv;
                q[j] = fmaf(-rkj, q[k], q[j]);
                if (t == 0) Rm[k * NB + j] = rkj;
            }
            if (t == 0) Rm[k * NB + k] = rkk;
        }
    }
    __syncthreads();
}

// Factor block `blockIdx.x` of a (rows x w) matrix stored column-major at P
// (ld), partitioned into nblk balanced blocks of whole `unit`-row units.
// Q overwrites the block; R (NB x NB, zero-padded) is written to rnext rows
// [blk*NB, blk*NB+NB) (column-major, ld_rnext). colmax (level 0 only, may be
// null) gives the per-column max-abs used for the power-of-two scaling.
__global__ __launch_bounds__(PT) void tsqr_level_kernel(float *__restrict__ P, int64_t ld,
                                                        int64_t rows, int w, int64_t nblk,
                                                        int unit, float *__restrict__ rnext,
                                                        int64_t ld_rnext, int reorth,
                                                        const float *__restrict__ colmax) {
    __shared__ float red[NB * LDR];
    __shared__ float rowv[2 * NB];
    __shared__ float R1[NB * NB];
    __shared__ float R2[NB * NB];
    __shared__ float csc[NB];
    const int t = threadIdx.x;
    const int64_t blk = blockIdx.x;
    const int64_t units = rows / unit;
    const int64_t s = part_start(blk, units, nblk) * unit;
    const int64_t e = part_start(blk + 1, units, nblk) * unit;
    const int64_t r = s + t;
    for (int i = t; i < NB * NB; i += PT) {
        R1[i] = 0.0f;
        R2[i] = 0.0f;
    }
    if (t < NB) csc[t] = (colmax && t < w) ? pow2_scale(colmax[t], 0) : 1.0f;
    __syncthreads();
    float q[NB];
#pragma unroll
    for (int j = 0; j < NB; ++j) q[j] = (j < w && r < e) ? P[r + j * ld] * csc[j] : 0.0f;

    mgs_sweep(q, w, red, rowv, R1);
    if (reorth) mgs_sweep(q, w, red, rowv, R2);

    if (r < e) {
#pragma unroll
        for (int j = 0; j < NB; ++j)
            if (j < w) P[r + j * ld] = q[j];
    }
    // R = R2 R1 (both upper triangular), or R1 for a single sweep.
    for (int idx = t; idx < NB * NB; idx += PT) {
        const int i = idx % NB, j = idx / NB;
        float v = 0.0f;
        if (i <= j) {
            if (reorth) {
                for (int l = i; l <= j; ++l) v = fmaf(R2[i * NB + l], R1[l * NB + j], v);
            } else {
                v = R1[i * NB + j];
            }
        }
        rnext[(blk * NB + i) + j * ld_rnext] = v;
    }
}

// Steps 4-5 of eq. caqr: P_blk <- P_blk * M_blk with M_blk the product of the
// tree Q slices on the path from level-0 block blk to the root.
__global__ __launch_bounds__(PT) void tsqr_qform_kernel(float *__restrict__ P, int64_t ld,
                                                        int64_t m, int w, TsqrLevels lv) {
    __shared__ float M[NB * NB];
    __shared__ float T[NB * NB];
    const int t = threadIdx.x;
    const int64_t blk = blockIdx.x;
    int64_t g[kMaxLevels + 1];
    g[0] = blk;
    for (int l = 1; l <= lv.nlev; ++l) g[l] = part_owner(g[l - 1], lv.nblk[l - 1], lv.nblk[l]);
    // M = Q_top[rows of unit g[nlev-1]]
    {
        const int L = lv.nlev;
        const int64_t ldL = lv.nblk[L - 1] * NB;
        const float *S = lv.stack[L] + g[L - 1] * NB;
        for (int idx = t; idx < NB * NB; idx += PT) {
            const int i = idx % NB, j = idx / NB;
            M[i * NB + j] = S[i + j * ldL];
        }
    }
    __syncthreads();
    for (int l = lv.nlev - 1; l >= 1; --l) {
        const int64_t ldl = lv.nblk[l - 1] * NB;
        const float *S = lv.stack[l] + g[l - 1] * NB;
        for (int idx = t; idx < NB * NB; idx += PT) {
            const int i = idx % NB, j = idx / NB;
            float v = 0.0f;
            for (int c = 0; c < NB; ++c) v = fmaf(S[i + c * ldl], M[c * NB + j], v);
            T[i * NB + j] = v;
        }
        __syncthreads();
        for (int idx = t; idx < NB * NB; idx += PT) M[idx] = T[idx];
        __syncthreads();
    }
    const int64_t s = part_start(blk, m, lv.nblk[0]);
    const int64_t e = part_start(blk + 1, m, lv.nblk[0]);
    const int64_t r = s + t;
    if (r < e) {
        float q[NB];
#pragma unroll
        for (int j = 0; j < NB; ++j) q[j] = (j < w) ? P[r + j * ld] : 0.0f;
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            if (j < w) {
                float v = 0.0f;
#pragma unroll
                for (int c = 0; c < NB; ++c) v = fmaf(q[c], M[c * NB + j], v);
                P[r + j * ld] = v;
            }
        }
    }
}

// Write the panel's final R (NB x NB at src, ld_src) into the w x w diagonal
// block of R, undoing the power-of-two column scaling of level 0.
__global__ void copy_r_block_kernel(const float *__restrict__ src, int64_t ld_src, int w,
                                    float *__restrict__ R, int64_t ldr,
                                    const float *__restrict__ colmax) {
    const int i = threadIdx.x % NB, j = threadIdx.x / NB;
    if (i < w && j < w) {
        const float sc = colmax ? pow2_scale(colmax[j], 0) : 1.0f;
        R[i + (int64_t)j * ldr] = (i <= j) ? src[i + j * ld_src] / sc : 0.0f;
    }
}

hipError_t launch_tsqr_level(hipStream_t s, float *P, int64_t ld, int64_t rows, int w,
                             int64_t nblk, int unit, float *rnext, int64_t ld_rnext, int reorth,
                             const float *colmax) {
    hipLaunchKernelGGL(tsqr_level_kernel, dim3((unsigned)nblk), dim3(PT), 0, s, P, ld, rows, w,
                       nblk, unit, rnext, ld_rnext, reorth, colmax);
    return hipGetLastError();
}

hipError_t launch_tsqr_qform(hipStream_t s, float *P, int64_t ld, int64_t m, int w,
                             const TsqrLevels &lv) {
    hipLaunchKernelGGL(tsqr_qform_kernel, dim3((unsigned)lv.nblk[0]), dim3(PT), 0, s, P, ld, m,
                       w, lv);
    return hipGetLastError();
}

hipError_t launch_copy_r_block(hipStream_t s, const float *src, int64_t ld_src, int w,
                               float *R, int64_t ldr, const float *colmax) {
    hipLaunchKernelGGL(copy_r_block_kernel, dim3(1), dim3(NB * NB), 0, s, src, ld_src, w, R,
                       ldr, colmax);
    return hipGetLastError();
}

}  // namespace qrx
