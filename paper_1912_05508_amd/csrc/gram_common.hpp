// Workgroup-level pieces of the Cholesky-QR panel (Gram sweep, Q formation,
// Cholesky elimination), shared by the panel kernels of gram.hip and by the
// one-workgroup-per-problem batched path.
#pragma once

#include "qrx_internal.hpp"

namespace qrx {
namespace gram {

constexpr int GT = 256;   // threads of a sweep workgroup
constexpr int CH = 64;    // rows per LDS chunk

__device__ __host__ inline int upk(int i, int j) { return j * (j + 1) / 2 + i; }  // i <= j

template <int W>
struct Lds {
    static constexpr int LDC = W + 2;                     // chunk row stride (16-byte aligned)
    static constexpr int XLD = W + 2;                     // row stride of X in LDS
    static constexpr int TW = W / 4;                      // Gram: 4 x 4 register tiles
    static constexpr int T = TW * TW;
    static constexpr int G = GT / T;                      // row groups sharing a tile (1, 4, 16)
    static constexpr int C_DOUBLES = CH * LDC;
    static constexpr int X_DOUBLES = W * XLD;
    static constexpr int RED_DOUBLES = (G > 1) ? (GT / 2) * 16 : 2;
    static_assert(GT % T == 0 && CH % G == 0 && GT == 4 * CH, "thread mapping");
};

// Xs (row-major, XLD) <- X (W x W, FP64, column-major, global). Caller syncs.
template <int W>
QRX_DEV void load_x(const double *__restrict__ X, double *Xs, int t) {
    for (int idx = t; idx < W * W; idx += GT) {
        const int i = idx % W, j = idx / W;
        Xs[i * Lds<W>::XLD + j] = X[idx];
    }
}

// One sweep of a workgroup over row chunks [ch0, ch1) of P (m x w, column-major,
// ld). DO_Q: rows <- fl32(rows X) with X upper triangular, in LDS (Xs, loaded
// and synced by the caller). DO_G: acc += this thread's 4 x 4 tile of
// (rows)^T (rows) in FP64 (of the rounded rows when DO_Q). The next chunk is
// prefetched into registers while the current one is computed.
template <int W, bool DO_Q, bool DO_G>
QRX_DEV void sweep(float *__restrict__ P, int64_t ld, int64_t m, int w, int64_t ch0, int64_t ch1,
                   const double *Xs, double *C, double (&acc)[4][4], int t) {
    using L = Lds<W>;
    constexpr int LDC = L::LDC, XLD = L::XLD, TW = L::TW, T = L::T, G = L::G;
    constexpr int LPT = CH * W / GT;           // chunk elements each thread stages
    constexpr int CB = W / 8;                  // Q formation: columns per block
    float pre[LPT];
    auto load = [&](int64_t ch) {
#pragma unroll
        for (int s = 0; s < LPT; ++s) {
            const int e = t + GT * s;
            const int rr = e % CH, cc = e / CH;
            const int64_t r = ch * CH + rr;
            pre[s] = (r < m && cc < w) ? P[r + cc * ld] : 0.0f;
        }
    };
    const int tile = t % T, grp = t / T;
    const int ti = tile % TW, tj = tile / TW;
    // Q formation: row qr of the chunk, column blocks cg (low) and 7 - cg (high), so
    // that every wave does the same share of the triangular product
    const int qr = t % CH, cg = t / CH;
    const int jlo = cg * CB, jhi = (7 - cg) * CB;

    if (ch0 < ch1) load(ch0);
    for (int64_t ch = ch0; ch < ch1; ++ch) {
        __syncthreads();
#pragma unroll
        for (int s = 0; s < LPT; ++s) {
            const int e = t + GT * s;
            C[(e % CH) * LDC + e / CH] = (double)pre[s];
        }
        __syncthreads();
        if (ch + 1 < ch1) load(ch + 1);
        if constexpr (DO_Q) {
            double lo[CB], hi[CB];
#pragma unroll
            for (int b = 0; b < CB; ++b) lo[b] = hi[b] = 0.0;
            const double *crow = C + qr * LDC;
            for (int i = 0; i < jlo + CB; ++i) {
                const double p = crow[i];
#pragma unroll
                for (int b = 0; b < CB; ++b) lo[b] = fma(p, Xs[i * XLD + jlo + b], lo[b]);
            }
            for (int i = 0; i < jhi + CB; ++i) {
                const double p = crow[i];
#pragma unroll
                for (int b = 0; b < CB; ++b) hi[b] = fma(p, Xs[i * XLD + jhi + b], hi[b]);
            }
            __syncthreads();
            const int64_t r = ch * CH + qr;
#pragma unroll
            for (int b = 0; b < CB; ++b) {
                const float vl = (float)lo[b], vh = (float)hi[b];
                C[qr * LDC + jlo + b] = (double)vl;
                C[qr * LDC + jhi + b] = (double)vh;
                if (r < m) {
                    if (jlo + b < w) P[r + (jlo + b) * ld] = vl;
                    if (jhi + b < w) P[r + (jhi + b) * ld] = vh;
                }
            }
            if constexpr (DO_G) __syncthreads();
        }
        if constexpr (DO_G) {
            for (int rr = grp; rr < CH; rr += G) {
                const double *row = C + rr * LDC;
                double a[4], b[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    a[q] = row[ti * 4 + q];
                    b[q] = row[tj * 4 + q];
                }
#pragma unroll
                for (int x = 0; x < 4; ++x)
#pragma unroll
                    for (int y = 0; y < 4; ++y) acc[x][y] = fma(a[x], b[y], acc[x][y]);
            }
        }
    }
}

// Sum the row groups' tiles (fixed tree) and write the upper triangle of the
// W x W Gram matrix to out[upk(i, j)] (global or LDS).
template <int W>
QRX_DEV void gram_store(double (&acc)[4][4], double *red, double *out, int t) {
    using L = Lds<W>;
    constexpr int TW = L::TW, T = L::T, G = L::G;
    const int tile = t % T, grp = t / T;
    const int ti = tile % TW, tj = tile / TW;
    if constexpr (G > 1) {
        for (int h = G / 2; h >= 1; h >>= 1) {
            __syncthreads();
            if (grp >= h && grp < 2 * h) {
                double *d = &red[((grp - h) * T + tile) * 16];
#pragma unroll
                for (int x = 0; x < 4; ++x)
#pragma unroll
                    for (int y = 0; y < 4; ++y) d[x * 4 + y] = acc[x][y];
            }
            __syncthreads();
            if (grp < h) {
                const double *d = &red[(grp * T + tile) * 16];
#pragma unroll
                for (int x = 0; x < 4; ++x)
#pragma unroll
                    for (int y = 0; y < 4; ++y) acc[x][y] += d[x * 4 + y];
            }
        }
    }
    if (grp == 0 && ti <= tj) {
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
            for (int y = 0; y < 4; ++y) {
                const int i = ti * 4 + x, j = tj * 4 + y;
                if (i <= j) out[upk(i, j)] = acc[x][y];
            }
    }
}

// Symmetric elimination of [G | I] in S (W x W, S[i + j*(W+1)], upper triangle
// holding G on entry) by NT threads: step k subtracts multiples of row k from
// the rows below it, leaving U = D L^T in the upper triangle and L^{-1} (unit
// lower) strictly below, so R = D^{-1/2} U and R^{-1} = L^{-T} D^{-1/2}.
// dg[k] = D_kk^{-1/2} (0 for a pivot <= 0: that row of R and column of R^{-1}
// are zero). Ends with a barrier.
template <int W, int NT>
QRX_DEV void chol_elim(double *S, double *dg, int w, int t) {
    constexpr int LS = W + 1;
    constexpr int NG = (NT / W < W) ? NT / W : W;   // column groups per row
    constexpr int QN = W / NG;
    static_assert(NT % W == 0 && W % NG == 0, "elimination mapping");
    const int ri = t % W, rg = t / W;
    for (int k = 0; k < w; ++k) {
        const double d = S[k + k * LS];
        if (d > 0.0 && rg < NG && ri > k) {
            // row ri of [U | L^{-1}] -= l * row k, on the L^{-1} part (c <= k) and the
            // U part (c >= ri); all reads first, then branch-free selects
            const double l = S[k + ri * LS] / d;
            double rk[QN], mine[QN];
#pragma unroll
            for (int q = 0; q < QN; ++q) {
                const int c = rg + NG * q;
                rk[q] = S[k + c * LS];
                mine[q] = S[ri + c * LS];
            }
#pragma unroll
            for (int q = 0; q < QN; ++q) {
                const int c = rg + NG * q;
                const double coef = (c == k) ? 1.0 : rk[q];
                mine[q] = (c <= k || c >= ri) ? fma(-l, coef, mine[q]) : mine[q];
            }
#pragma unroll
            for (int q = 0; q < QN; ++q) S[ri + (rg + NG * q) * LS] = mine[q];
        }
        __syncthreads();
    }
    if (t < W) {
        const double d = (t < w) ? S[t + t * LS] : 0.0;
        dg[t] = (d > 0.0) ? 1.0 / sqrt(d) : 0.0;
    }
    __syncthreads();
}

// R[i][j] = U[i][j] D_i^{-1/2} and X = R^{-1}[i][j] = Linv[j][i] D_j^{-1/2} (i <= j),
// zero elsewhere and beyond w.
template <int W>
QRX_DEV double chol_R(const double *S, const double *dg, int w, int i, int j) {
    return (i <= j && j < w) ? S[i + j * (W + 1)] * dg[i] : 0.0;
}
template <int W>
QRX_DEV double chol_X(const double *S, const double *dg, int w, int i, int j) {
    return (i <= j && j < w) ? ((i == j) ? 1.0 : S[j + i * (W + 1)]) * dg[j] : 0.0;
}

}  // namespace gram
}  // namespace qrx
