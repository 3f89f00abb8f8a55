// Panel factorisation by Cholesky QR run twice with an FP64 Gram matrix.
//
// An alternative to the TSQR/MGS panel for the leaves of the recursion (the
// paper's panel is eq. caqr with Alg. 4 blocks; this one keeps its two-sweep
// re-orthogonalisation but replaces the per-column reductions by one Gram
// matrix per sweep). For a panel P (m x w, FP32, w <= 64):
//   pass 1: G1 = P^T P (FP64; products of FP32 values are exact in FP64),
//           R1 = chol(G1), Q1 = fl32(P R1^{-1})       (FP64 arithmetic)
//   pass 2: G2 = Q1^T Q1, R2 = chol(G2), Q = fl32(Q1 R2^{-1}), R = R2 R1.
// Rounding Q (not the operator) keeps the factorisation backward stable; the
// FP64 Gram keeps Cholesky accurate for condition numbers up to ~1e7, i.e. the
// whole range an FP32 panel can carry. A zero (or negative) pivot leaves the
// column of Q zero with R_kk = 0 (reported as singular when it reaches R).
//
// Kernels per pass: Gram partials over row chunks (FP64, register-blocked),
// a fixed-order sum of the partials (one wave per entry), a one-workgroup
// Cholesky + triangular inverse in LDS, and the row-block product P R^{-1}
// (FP64, register-blocked).
#include "qrx_internal.hpp"

namespace qrx {

constexpr int GRT = 256;     // threads per workgroup
constexpr int GCH = 32;      // rows per LDS stage in the Gram kernel
constexpr int QROWS = 64;    // rows per workgroup in the Q-formation kernel

__device__ __host__ inline int64_t upk(int i, int j) { return (int64_t)j * (j + 1) / 2 + i; }  // i <= j

// part[blk][upk(i,j)] = sum over this block's rows of P[r,i] P[r,j] (i <= j).
// Thread = (8 x 8 tile of G, row group); row groups are combined by a tree.
template <int W>
__global__ __launch_bounds__(GRT) void gram_partial_kernel(const float *__restrict__ P, int64_t ld,
                                                           int64_t m, int w, int64_t rows_per,
                                                           double *__restrict__ part) {
    constexpr int TS = 8;
    constexpr int TW = W / TS;
    constexpr int T = TW * TW;
    constexpr int G = GRT / T;             // row groups sharing a tile (4, 16 or 64)
    static_assert(G >= 1 && GRT % T == 0, "tile mapping");
    __shared__ float Ps[GCH][W + 4];
    __shared__ double red[(G > 1) ? (GRT / 2) * TS * TS : 1];
    const int t = threadIdx.x;
    const int tile = t % T, grp = t / T;
    const int ti = tile % TW, tj = tile / TW;
    const bool active = ti <= tj;
    const int64_t r0 = (int64_t)blockIdx.x * rows_per;
    const int64_t r1 = (r0 + rows_per < m) ? r0 + rows_per : m;
    double acc[TS][TS];
#pragma unroll
    for (int a = 0; a < TS; ++a)
#pragma unroll
        for (int b = 0; b < TS; ++b) acc[a][b] = 0.0;
    for (int64_t c0 = r0; c0 < r1; c0 += GCH) {
        __syncthreads();
        for (int idx = t; idx < GCH * W; idx += GRT) {
            const int rr = idx % GCH, cc = idx / GCH;
            const int64_t r = c0 + rr;
            Ps[rr][cc] = (r < r1 && cc < w) ? P[r + cc * ld] : 0.0f;
        }
        __syncthreads();
        if (active) {
            for (int rr = grp; rr < GCH; rr += G) {
                double a[TS], b[TS];
#pragma unroll
                for (int q = 0; q < TS; ++q) {
                    a[q] = (double)Ps[rr][ti * TS + q];
                    b[q] = (double)Ps[rr][tj * TS + q];
                }
#pragma unroll
                for (int x = 0; x < TS; ++x)
#pragma unroll
                    for (int y = 0; y < TS; ++y) acc[x][y] = fma(a[x], b[y], acc[x][y]);
            }
        }
    }
    double *out = part + (int64_t)blockIdx.x * (W * (W + 1) / 2);
    if constexpr (G > 1) {
        // tree over row groups: group g += group g + h, h = G/2, G/4, ..., 1
        for (int h = G / 2; h >= 1; h >>= 1) {
            __syncthreads();
            if (grp >= h && grp < 2 * h && active) {
                double *d = &red[((grp - h) * T + tile) * TS * TS];
#pragma unroll
                for (int x = 0; x < TS; ++x)
#pragma unroll
                    for (int y = 0; y < TS; ++y) d[x * TS + y] = acc[x][y];
            }
            __syncthreads();
            if (grp < h && active) {
                const double *d = &red[(grp * T + tile) * TS * TS];
#pragma unroll
                for (int x = 0; x < TS; ++x)
#pragma unroll
                    for (int y = 0; y < TS; ++y) acc[x][y] += d[x * TS + y];
            }
        }
    }
    if (grp == 0 && active) {
#pragma unroll
        for (int x = 0; x < TS; ++x)
#pragma unroll
            for (int y = 0; y < TS; ++y) {
                const int i = ti * TS + x, j = tj * TS + y;
                if (i <= j) out[upk(i, j)] = acc[x][y];
            }
    }
}

// G[e] = sum_b part[b][e]: one wave per entry, lanes stride the parts, then a
// fixed butterfly (deterministic).
__global__ __launch_bounds__(GRT) void gram_reduce_kernel(const double *__restrict__ part,
                                                          int64_t nparts, int64_t np,
                                                          double *__restrict__ G) {
    const int lane = threadIdx.x & 63;
    const int64_t e = (int64_t)blockIdx.x * (GRT / 64) + (threadIdx.x >> 6);
    if (e >= np) return;
    double s = 0.0;
    for (int64_t b = lane; b < nparts; b += 64) s += part[b * np + e];
    s = wave_sum_d(s);
    if (lane == 0) G[e] = s;
}

// One workgroup: R = chol(G) (upper, G = R^T R) and X = R^{-1}, both FP64
// (W x W, column-major), by one symmetric elimination of [G | I]: step k
// subtracts multiples of row k from the rows below it, which leaves U = D L^T
// in the upper triangle and L^{-1} (unit lower) in the strictly-lower
// triangle, so R = D^{-1/2} U and R^{-1} = L^{-T} D^{-1/2}. One barrier per
// step. If Rfinal != null, also writes the panel's R block (FP32, ldr):
// R Rprev when Rprev != null, else R. A pivot <= 0 gives a zero row of R and a
// zero column of X.
template <int W>
__global__ __launch_bounds__(GRT) void gram_chol_kernel(const double *__restrict__ Gp, int w,
                                                        double *__restrict__ Rout,
                                                        double *__restrict__ Xout,
                                                        const double *__restrict__ Rprev,
                                                        float *__restrict__ Rfinal, int64_t ldr) {
    constexpr int LS = W + 1;
    __shared__ double S[W * LS];      // S[i + j*LS]; upper: G -> U, strictly lower: L^{-1}
    __shared__ double dg[W];          // D_kk^{-1/2} (0 for a non-positive pivot)
    const int t = threadIdx.x;
    for (int idx = t; idx < W * W; idx += GRT) {
        const int i = idx % W, j = idx / W;
        S[i + j * LS] = (i <= j && j < w) ? Gp[upk(i, j)] : 0.0;
    }
    __syncthreads();
    for (int k = 0; k < w; ++k) {
        const double d = S[k + k * LS];
        if (d > 0.0) {
            const double inv = 1.0 / d;
            const int rem = w - k - 1;
            // rows i > k: upper part j >= i (trailing Gram) and lower part c <= k (L^{-1})
            const int nup = rem * rem, nlo = rem * (k + 1);
            for (int idx = t; idx < nup + nlo; idx += GRT) {
                if (idx < nup) {
                    const int i = k + 1 + idx % rem, j = k + 1 + idx / rem;
                    if (i <= j) S[i + j * LS] -= S[k + i * LS] * S[k + j * LS] * inv;
                } else {
                    const int q = idx - nup;
                    const int i = k + 1 + q % rem, c = q / rem;     // c <= k
                    const double lkc = (c == k) ? 1.0 : S[k + c * LS];
                    S[i + c * LS] -= S[k + i * LS] * inv * lkc;
                }
            }
        }
        __syncthreads();
    }
    if (t < W) {
        const double d = (t < w) ? S[t + t * LS] : 0.0;
        dg[t] = (d > 0.0) ? 1.0 / sqrt(d) : 0.0;
    }
    __syncthreads();
    for (int idx = t; idx < W * W; idx += GRT) {
        const int i = idx % W, j = idx / W;
        // R[i][j] = U[i][j] D_i^{-1/2};  X[i][j] = Linv[j][i] D_j^{-1/2} (i <= j)
        const bool up = i <= j && j < w;
        Rout[i + j * W] = up ? S[i + j * LS] * dg[i] : 0.0;
        Xout[i + j * W] = up ? ((i == j) ? 1.0 : S[j + i * LS]) * dg[j] : 0.0;
    }
    if (Rfinal) {
        for (int idx = t; idx < W * W; idx += GRT) {
            const int i = idx % W, j = idx / W;
            double v = 0.0;
            if (i <= j && j < w) {
                if (Rprev) {
                    for (int l = i; l <= j; ++l) v = fma(S[i + l * LS] * dg[i], Rprev[l + j * W], v);
                } else {
                    v = S[i + j * LS] * dg[i];
                }
            }
            if (i < w && j < w) Rfinal[i + (int64_t)j * ldr] = (float)v;
        }
    }
}

// In place: P[r, :] <- fl32(P[r, :] X), X = R^{-1} (FP64, upper, W x W).
// Workgroup = 64 rows; thread = 4 rows x (W/16) columns, FP64 accumulation.
template <int W>
__global__ __launch_bounds__(GRT) void gram_qform_kernel(float *__restrict__ P, int64_t ld,
                                                         int64_t m, int w,
                                                         const double *__restrict__ X) {
    constexpr int CT = W / 16;                 // columns per thread
    __shared__ double Xs[W * W];               // Xs[i * W + j] = X[i][j] (row-major)
    __shared__ double Ps[QROWS][W + 1];
    const int t = threadIdx.x;
    const int64_t r0 = (int64_t)blockIdx.x * QROWS;
    for (int idx = t; idx < W * W; idx += GRT) {
        const int i = idx / W, j = idx % W;
        Xs[idx] = X[i + j * W];
    }
    for (int idx = t; idx < QROWS * W; idx += GRT) {
        const int rr = idx % QROWS, cc = idx / QROWS;
        const int64_t r = r0 + rr;
        Ps[rr][cc] = (r < m && cc < w) ? (double)P[r + cc * ld] : 0.0;
    }
    __syncthreads();
    const int rg = t % 16, cg = t / 16;        // rows rg*4.., columns cg*CT..
    double acc[4][CT];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < CT; ++b) acc[a][b] = 0.0;
    for (int i = 0; i < w; ++i) {
        double p[4], x[CT];
#pragma unroll
        for (int a = 0; a < 4; ++a) p[a] = Ps[rg * 4 + a][i];
#pragma unroll
        for (int b = 0; b < CT; ++b) x[b] = Xs[i * W + cg * CT + b];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < CT; ++b) acc[a][b] = fma(p[a], x[b], acc[a][b]);
    }
#pragma unroll
    for (int b = 0; b < CT; ++b) {
        const int j = cg * CT + b;
        if (j < w) {
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                const int64_t r = r0 + rg * 4 + a;
                if (r < m) P[r + j * ld] = (float)acc[a][b];
            }
        }
    }
}

// ---------------------------------------------------------------------------
int gram_parts(int64_t m) {
    int64_t b = (m + 255) / 256;               // ~256 rows per partial
    if (b > 256) b = 256;
    if (b < 1) b = 1;
    return (int)b;
}

// Workspace (doubles): parts * W(W+1)/2 + W(W+1)/2 + 4 W^2
size_t gram_workspace_doubles(int64_t m, int W) {
    const size_t np = (size_t)W * (W + 1) / 2;
    return (size_t)gram_parts(m) * np + np + 4 * (size_t)W * W;
}

template <int W>
static hipError_t gram_go(hipStream_t s, float *P, int64_t ld, int64_t m, int w, float *R,
                          int64_t ldr, double *ws, int reorth) {
    const int64_t np = (int64_t)W * (W + 1) / 2;
    const int parts = gram_parts(m);
    const int64_t rows_per = (m + parts - 1) / parts;
    double *part = ws;
    double *G = part + (size_t)parts * np;
    double *R1 = G + np;
    double *X1 = R1 + W * W;
    double *R2 = X1 + W * W;
    double *X2 = R2 + W * W;
    const unsigned qb = (unsigned)((m + QROWS - 1) / QROWS);
    const unsigned rb = (unsigned)((np + 3) / 4);
    const int passes = reorth ? 2 : 1;
    for (int pass = 0; pass < passes; ++pass) {
        hipLaunchKernelGGL(gram_partial_kernel<W>, dim3(parts), dim3(GRT), 0, s, P, ld, m, w,
                           rows_per, part);
        hipLaunchKernelGGL(gram_reduce_kernel, dim3(rb), dim3(GRT), 0, s, part, (int64_t)parts, np, G);
        if (pass == 0)
            hipLaunchKernelGGL(gram_chol_kernel<W>, dim3(1), dim3(GRT), 0, s, G, w, R1, X1,
                               (const double *)nullptr, passes == 1 ? R : (float *)nullptr, ldr);
        else
            hipLaunchKernelGGL(gram_chol_kernel<W>, dim3(1), dim3(GRT), 0, s, G, w, R2, X2, R1, R,
                               ldr);
        hipLaunchKernelGGL(gram_qform_kernel<W>, dim3(qb), dim3(GRT), 0, s, P, ld, m, w,
                           pass == 0 ? X1 : X2);
    }
    return hipGetLastError();
}

hipError_t launch_gram_panel(hipStream_t s, float *P, int64_t ld, int64_t m, int w, float *R,
                             int64_t ldr, double *ws, int reorth) {
    if (w <= 16) return gram_go<16>(s, P, ld, m, w, R, ldr, ws, reorth);
    if (w <= 32) return gram_go<32>(s, P, ld, m, w, R, ldr, ws, reorth);
    return gram_go<64>(s, P, ld, m, w, R, ldr, ws, reorth);
}

}  // namespace qrx
