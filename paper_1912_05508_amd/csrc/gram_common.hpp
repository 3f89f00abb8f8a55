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

// ---------------------------------------------------------------------------
// Blocked Cholesky with the inverse of the factor, for W a multiple of 16:
// G = R^T R (R upper, R_kk > 0) and X = R^{-1}, both FP64 in LDS (column-
// major, stride W + 1). On entry S holds G in its upper triangle (zero beyond
// w); on exit S holds R in its upper triangle and Xs holds X (zero below the
// diagonal). A pivot <= 0 gives a zero row of R and a zero column of X.
// Per 16-column block: one wave factors the diagonal block and inverts it in
// registers (column per lane, values exchanged by cross-lane shuffles), then
// all threads form the block row of R and update the trailing matrix; the
// off-diagonal blocks of X follow by block products ordered by their distance
// from the diagonal. T is LDS scratch of max(16, (W/16 - 1) * 256) doubles.
// ---------------------------------------------------------------------------
// v in lane l, as a wave-uniform value (two v_readlane).
QRX_DEV double readlane_d(double v, int l) {
    const long long bits = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)bits, l);
    const int hi = __builtin_amdgcn_readlane((int)(bits >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// 1 / sqrt(d) for d > 0: hardware estimate plus one Newton step.
QRX_DEV double rsqrt_d(double d) {
    double y = __builtin_amdgcn_rsq(d);
    return y * fma(-0.5 * d * y, y, 1.5);
}

// One wave: Cholesky of the 16 x 16 block at (o, o) of S (upper triangle,
// updated in place to R) and its inverse into Xs. Lane j < 16 keeps column j
// in registers; the entries of the pivot row are read from their lanes with
// v_readlane. Lanes 16..63 compute copies and write nothing.
template <int LS>
QRX_DEV void diag16(double *S, double *Xs, int o, int lane) {
    const int j = lane & 15;
    const bool own = lane < 16;
    double col[16], x[16], rdi[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) col[i] = (i <= j) ? S[(o + i) + (o + j) * LS] : 0.0;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const double d = readlane_d(col[k], k);      // G'[k][k]
        const double rinv = (d > 0.0) ? rsqrt_d(d) : 0.0;
        rdi[k] = rinv;                               // 1 / R[k][k] (0 for a bad pivot)
        const double rkj = (j >= k) ? col[k] * rinv : 0.0;
#pragma unroll
        for (int i = k + 1; i < 16; ++i) {
            const double rki = readlane_d(col[k], i) * rinv;   // R[k][i]
            if (i <= j) col[i] = fma(-rki, rkj, col[i]);
        }
        col[k] = rkj;                                // R[k][j]
    }
    // column j of X: R x = e_j by back substitution
#pragma unroll
    for (int i = 15; i >= 0; --i) {
        double acc = (i == j) ? 1.0 : 0.0;
#pragma unroll
        for (int l = i + 1; l < 16; ++l) acc = fma(-readlane_d(col[i], l), x[l], acc);
        x[i] = (i <= j) ? acc * rdi[i] : 0.0;
    }
    if (own) {
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            if (i <= j) S[(o + i) + (o + j) * LS] = col[i];
            Xs[(o + i) + (o + j) * LS] = x[i];
        }
    }
}

template <int W, int NT>
QRX_DEV void chol_blocked(double *S, double *Xs, double *T, int t) {
    constexpr int LS = W + 1;
    constexpr int NB = W / 16;
    constexpr int PV = (16 * (W - 16) + NT - 1) / NT;     // panel entries per thread
    static_assert(W % 16 == 0 && NT >= 64, "blocked Cholesky shape");
    // zero the strictly-lower part of Xs (the blocks below the diagonal stay zero)
    for (int idx = t; idx < W * W; idx += NT) {
        const int i = idx % W, jj = idx / W;
        if (i > jj) Xs[i + jj * LS] = 0.0;
    }
    for (int K = 0; K < NB; ++K) {
        const int o = 16 * K, rest = W - o - 16;
        if (t < 64) diag16<LS>(S, Xs, o, t);
        __syncthreads();
        if (rest > 0) {
            // block row of R: R[o+i][c] = sum_{l <= i} X_KK[l][i] G'[o+l][c]
            double v[PV > 0 ? PV : 1];
#pragma unroll
            for (int q = 0; q < PV; ++q) {
                const int idx = t + q * NT;
                v[q] = 0.0;
                if (idx < 16 * rest) {
                    const int i = idx % 16, c = o + 16 + idx / 16;
                    double a4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                    for (int l = 0; l < 16; ++l)   // X_KK[l][i] = 0 for l > i
                        a4[l & 3] = fma(Xs[(o + l) + (o + i) * LS], S[(o + l) + c * LS], a4[l & 3]);
                    v[q] = (a4[0] + a4[1]) + (a4[2] + a4[3]);
                }
            }
            __syncthreads();
#pragma unroll
            for (int q = 0; q < PV; ++q) {
                const int idx = t + q * NT;
                if (idx < 16 * rest) S[(o + idx % 16) + (o + 16 + idx / 16) * LS] = v[q];
            }
            __syncthreads();
            // trailing update: G'[a][b] -= sum_i R[o+i][a] R[o+i][b], a <= b in the rest
            for (int idx = t; idx < rest * rest; idx += NT) {
                const int a = o + 16 + idx % rest, b = o + 16 + idx / rest;
                if (a <= b) {
                    double a4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                    for (int i = 0; i < 16; ++i)
                        a4[i & 3] = fma(S[(o + i) + a * LS], S[(o + i) + b * LS], a4[i & 3]);
                    S[a + b * LS] -= (a4[0] + a4[1]) + (a4[2] + a4[3]);
                }
            }
            __syncthreads();
        }
    }
    // off-diagonal blocks of X: X_IJ = -X_II sum_{L=I+1..J} R_IL X_LJ, by distance
    for (int d = 1; d < NB; ++d) {
        const int nblk = NB - d;
        for (int idx = t; idx < nblk * 256; idx += NT) {
            const int I = idx / 256, p = (idx % 256) % 16, q = (idx % 256) / 16;
            const int J = I + d;
            double a4[4] = {0.0, 0.0, 0.0, 0.0};
            for (int r = 16 * (I + 1); r <= 16 * J + 15; r += 4) {
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    a4[u] = fma(S[(16 * I + p) + (r + u) * LS], Xs[(r + u) + (16 * J + q) * LS], a4[u]);
            }
            T[idx] = (a4[0] + a4[1]) + (a4[2] + a4[3]);
        }
        __syncthreads();
        for (int idx = t; idx < nblk * 256; idx += NT) {
            const int I = idx / 256, p = (idx % 256) % 16, q = (idx % 256) / 16;
            const int J = I + d;
            double a4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int s2 = 0; s2 < 16; ++s2)   // X_II[p][s2] = 0 for s2 < p
                a4[s2 & 3] = fma(Xs[(16 * I + p) + (16 * I + s2) * LS], T[I * 256 + q * 16 + s2], a4[s2 & 3]);
            Xs[(16 * I + p) + (16 * J + q) * LS] = -((a4[0] + a4[1]) + (a4[2] + a4[3]));
        }
        __syncthreads();
    }
}

}  // namespace gram
}  // namespace qrx
