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
// All loads are issued before the first store (one round trip to memory: X
// was just written by another workgroup and is not in this CU's caches).
template <int W>
QRX_DEV void load_x(const double *__restrict__ X, double *Xs, int t) {
    constexpr int NQ = (W * W + GT - 1) / GT;
    double v[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const int idx = t + q * GT;
        v[q] = (idx < W * W) ? X[idx] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const int idx = t + q * GT;
        if (idx < W * W) Xs[(idx % W) * Lds<W>::XLD + idx / W] = v[q];
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
// 32-column sweeps on the FP64 matrix cores (v_mfma_f64_16x16x4f64: A operand
// lane l holds A[l % 16][l / 16], B operand B[l / 16][l % 16], result register
// v of lane l holds D[4 v + l / 16][l % 16]). The four-by-four register tiles
// of sweep() read two LDS values per two FMAs and leave the sweep bound by LDS;
// a matrix-core step reads one value per lane per operand for 1024 FMAs.
// Gram: wave w takes rows 16w .. 16w + 15 of each chunk (four steps of four
// rows) for the three upper 16 x 16 blocks (0,0), (0,1), (1,1); gram_store32
// adds the waves' sums at the end of the sweep. Q formation: wave w forms rows
// 16w .. 16w + 15 of rows X, its two column blocks over K up to the block's
// last column (X is upper triangular).
// ---------------------------------------------------------------------------
typedef double gd4 __attribute__((ext_vector_type(4)));
QRX_DEV gd4 mfma_f64(double a, double b, gd4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

template <bool DO_Q, bool DO_G>
QRX_DEV void sweep32(float *__restrict__ P, int64_t ld, int64_t m, int w, int64_t ch0, int64_t ch1,
                     const double *Xs, double *C, gd4 (&acc)[3], int t) {
    using L = Lds<32>;
    constexpr int LDC = L::LDC, XLD = L::XLD;
    constexpr int LPT = CH * 32 / GT;           // chunk elements each thread stages
    static_assert(GT == 256 && CH == 64, "four waves, 16 chunk rows each");
    const int lane = t & 63;
    const int wv = __builtin_amdgcn_readfirstlane(t >> 6);
    const int li = lane & 15, lk = lane >> 4;
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
            gd4 q[2];
#pragma unroll
            for (int Jb = 0; Jb < 2; ++Jb) {
                q[Jb] = gd4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int k4 = 0; k4 < 4 * (Jb + 1); ++k4) {
                    const double a = C[(16 * wv + li) * LDC + 4 * k4 + lk];
                    const double b = Xs[(4 * k4 + lk) * XLD + 16 * Jb + li];
                    q[Jb] = mfma_f64(a, b, q[Jb]);
                }
            }
            __syncthreads();   // every wave has read its rows of the chunk
#pragma unroll
            for (int Jb = 0; Jb < 2; ++Jb)
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    C[(16 * wv + 4 * v + lk) * LDC + 16 * Jb + li] = (double)(float)q[Jb][v];
            __syncthreads();
            // Q rows back to P, coalesced along the columns
#pragma unroll
            for (int s = 0; s < LPT; ++s) {
                const int e = t + GT * s;
                const int rr = e % CH, cc = e / CH;
                const int64_t r = ch * CH + rr;
                if (r < m && cc < w) P[r + cc * ld] = (float)C[rr * LDC + cc];
            }
        }
        if constexpr (DO_G) {
#pragma unroll
            for (int k4 = 0; k4 < 4; ++k4) {
                const double *row = C + (16 * wv + 4 * k4 + lk) * LDC + li;
                const double r0 = row[0], r1 = row[16];
                acc[0] = mfma_f64(r0, r0, acc[0]);
                acc[1] = mfma_f64(r0, r1, acc[1]);
                acc[2] = mfma_f64(r1, r1, acc[2]);
            }
        }
    }
}

// The waves' Gram sums of sweep32 added in a fixed order ((w0 + w2) + (w1 + w3))
// and the upper triangle of the 32 x 32 result written to out[upk(i, j)]
// (global or LDS); red holds 1536 doubles. Ends with a barrier.
QRX_DEV void gram_store32(gd4 (&acc)[3], double *red, double *out, int t) {
    const int lane = t & 63;
    const int wv = __builtin_amdgcn_readfirstlane(t >> 6);
    static_assert(Lds<32>::RED_DOUBLES >= 2 * 12 * 64, "reduction buffer");
    auto slot = [&](int s, int p, int v) { return red + ((s * 3 + p) * 4 + v) * 64 + lane; };
    __syncthreads();   // red may still be read by the caller's previous step
    if (wv >= 2) {
#pragma unroll
        for (int p = 0; p < 3; ++p)
#pragma unroll
            for (int v = 0; v < 4; ++v) *slot(wv - 2, p, v) = acc[p][v];
    }
    __syncthreads();
    if (wv < 2) {
#pragma unroll
        for (int p = 0; p < 3; ++p)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[p][v] += *slot(wv, p, v);
    }
    __syncthreads();
    if (wv == 1) {
#pragma unroll
        for (int p = 0; p < 3; ++p)
#pragma unroll
            for (int v = 0; v < 4; ++v) *slot(0, p, v) = acc[p][v];
    }
    __syncthreads();
    if (wv == 0) {
        const int Is[3] = {0, 0, 1}, Js[3] = {0, 1, 1};
#pragma unroll
        for (int p = 0; p < 3; ++p)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = 16 * Is[p] + 4 * v + (lane >> 4), j = 16 * Js[p] + (lane & 15);
                if (i <= j) out[upk(i, j)] = acc[p][v] + *slot(0, p, v);
            }
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Cholesky with the inverse of the factor: G = R^T R (R upper, R_kk > 0) and
// X = R^{-1}, FP64 in LDS (column-major, stride W + 1). On entry S holds G in
// its upper triangle (zero beyond w); on exit S holds R in its upper triangle
// and Xs holds X (zero below the diagonal). A pivot <= 0 gives a zero row of R
// and a zero column of X.
// Symmetric elimination on the augmented W x 2W matrix [G | I]: step k
// subtracts (entry k of row i) / pivot times row k from every row i > k; row k
// scaled by 1/sqrt(pivot) is then row k of R on the left and row k of R^{-T}
// on the right (the row operations that turn G into R turn I into R^{-T}).
// The matrix lives in registers, RB x CB entries per thread, and row k stays
// unscaled until the end. Row k is broadcast through a double-buffered row in
// LDS with its pivot in a slot of its own and its left entries up to the
// diagonal zeroed, so that rows <= k, whose entry in that row is zero, are
// left unchanged without a branch. Waves whose rows are all <= k skip the
// step; one barrier per step. Entries left of the diagonal take finite values
// that are never read. T is LDS scratch of 4W + 4 doubles (kCholT64 for
// W = 64 with 512 threads, which takes the blocked variant).
// ---------------------------------------------------------------------------
// 1 / sqrt(d) for d > 0: hardware estimate plus one Newton step.
QRX_DEV double rsqrt_d(double d) {
    double y = __builtin_amdgcn_rsq(d);
    return y * fma(-0.5 * d * y, y, 1.5);
}

// v in lane l, as a wave-uniform value (two v_readlane).
QRX_DEV double readlane_d(double v, int l) {
    const long long bits = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)bits, l);
    const int hi = __builtin_amdgcn_readlane((int)(bits >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// The same elimination for W = 64 and 512 threads, blocked by eight pivots.
// Wave b owns rows 8b .. 8b + 7 of [G | I] (two columns per lane). In round b
// these rows have every earlier pivot applied; each lane of wave b reads the
// 8 x 8 diagonal block D (through LDS), factors D = U^T U redundantly in
// registers, and applies U^{-T} to its two columns of the eight rows, which
// thereby become rows 8b .. 8b + 7 of [R | R^{-T}] (final, scaled). The wave
// publishes them; after one barrier each wave below subtracts, from each of
// its rows i, R[p][i] times row p for the eight rows p of the block (the
// Schur-complement update of both halves, by the symmetry of the remaining
// block). Eight barriers in all; the pivots of a block form one register-
// resident chain in a single wave.
constexpr int kCholT64 = 2 * 8 * 128 + 64;   // LDS scratch: two 8-row buffers, the block

QRX_DEV void chol_inv64_b8(double *S, double *Xs, double *T, int t) {
    constexpr int W = 64, LS = W + 1, RB = 8, RW = 2 * W;
    const int lane = t & 63;
    const int wv = __builtin_amdgcn_readfirstlane(t >> 6);
    const int i0 = wv * RB, j0 = 2 * lane;
    double M[RB][2];
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const int i = i0 + r, j = j0 + c;
            M[r][c] = (j < W) ? ((i <= j) ? S[i + j * LS] : S[j + i * LS])
                              : ((j - W == i) ? 1.0 : 0.0);
        }
    double *Dsh = T + 2 * RB * RW;
    __syncthreads();
    for (int b = 0; b < W / RB; ++b) {
        double *buf = T + (b & 1) * RB * RW;
        if (wv == b) {
            // the diagonal block: columns 8b .. 8b + 7 are in lanes 4b .. 4b + 3
            if ((lane >> 2) == b) {
#pragma unroll
                for (int r = 0; r < RB; ++r)
                    *(double2 *)&Dsh[r * RB + (j0 - RB * b)] = make_double2(M[r][0], M[r][1]);
            }
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            double D[RB][RB];
#pragma unroll
            for (int r = 0; r < RB; ++r)
#pragma unroll
                for (int c = 0; c < RB; c += 2) {
                    const double2 v = *(const double2 *)&Dsh[r * RB + c];
                    D[r][c] = v.x;
                    D[r][c + 1] = v.y;
                }
            // D = U^T U (upper part of D becomes U; a pivot <= 0 gives a zero row)
            double rinv[RB];
#pragma unroll
            for (int q = 0; q < RB; ++q) {
                const double d = D[q][q];
                const double ri = (d > 0.0) ? rsqrt_d(d) : 0.0;
                rinv[q] = ri;
#pragma unroll
                for (int c = q; c < RB; ++c) D[q][c] *= ri;
#pragma unroll
                for (int r = q + 1; r < RB; ++r)
#pragma unroll
                    for (int c = r; c < RB; ++c) D[r][c] = fma(-D[q][r], D[q][c], D[r][c]);
            }
            // rows <- U^{-T} rows: row q = (row q - sum_{p<q} U[p][q] row p) / U[q][q]
#pragma unroll
            for (int q = 0; q < RB; ++q)
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    double v = M[q][c];
#pragma unroll
                    for (int p2 = 0; p2 < q; ++p2) v = fma(-D[p2][q], M[p2][c], v);
                    M[q][c] = v * rinv[q];
                }
#pragma unroll
            for (int r = 0; r < RB; ++r)
                *(double2 *)&buf[r * RW + j0] = make_double2(M[r][0], M[r][1]);
        }
        __syncthreads();
        if (wv > b) {
            // rows i of this wave: M[i][.] -= sum_p R[p][i] R[p][.]
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                double mu[4][RB], rp[4][2];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const double *row = buf + (4 * h + q) * RW;
#pragma unroll
                    for (int r = 0; r < RB; r += 2) {
                        const double2 v = *(const double2 *)&row[i0 + r];
                        mu[q][r] = v.x;
                        mu[q][r + 1] = v.y;
                    }
                    const double2 v = *(const double2 *)&row[j0];
                    rp[q][0] = v.x;
                    rp[q][1] = v.y;
                }
#pragma unroll
                for (int q = 0; q < 4; ++q)
#pragma unroll
                    for (int r = 0; r < RB; ++r)
#pragma unroll
                        for (int c = 0; c < 2; ++c) M[r][c] = fma(-mu[q][r], rp[q][c], M[r][c]);
            }
        }
    }
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const int i = i0 + r, j = j0 + c;
            const double v = M[r][c];
            if (j < W) {
                if (i <= j) S[i + j * LS] = v;
            } else {
                const int a = j - W;   // X[a][i] = (R^{-T})[i][a]
                Xs[a + i * LS] = (a <= i) ? v : 0.0;
            }
        }
    __syncthreads();
}

template <int W, int NT>
QRX_DEV void chol_inv(double *S, double *Xs, double *T, int t) {
    if constexpr (W == 64 && NT == 512) {
        chol_inv64_b8(S, Xs, T, t);
        return;
    }
    constexpr int LS = W + 1;
    constexpr int E = 2 * W * W / NT;      // entries per thread
    constexpr int CB = E >= 2 ? 2 : 1;
    constexpr int RB = E / CB;
    constexpr int NCB = 2 * W / CB;
    constexpr int RL = 2 * W + 2;          // row buffer: 2W entries, the pivot, padding
    static_assert(E * NT == 2 * W * W && (W / RB) * NCB == NT && NT % 64 == 0,
                  "elimination thread mapping");
    const int i0 = (t / NCB) * RB, j0 = (t % NCB) * CB;
    // last row held by this wave (uniform)
    const int wlast = __builtin_amdgcn_readfirstlane(((t | 63) / NCB) * RB + RB - 1);
    double M[RB][CB], sc[RB];
#pragma unroll
    for (int r = 0; r < RB; ++r) {
        sc[r] = 0.0;
#pragma unroll
        for (int c = 0; c < CB; ++c) {
            const int i = i0 + r, j = j0 + c;
            M[r][c] = (j < W) ? ((i <= j) ? S[i + j * LS] : S[j + i * LS])
                              : ((j - W == i) ? 1.0 : 0.0);
        }
    }
    // row q = i0 + r of this thread into buffer q & 1: left entries j <= q zeroed,
    // the pivot in its own slot; the row is picked from M by selects
    auto put_row = [&](int q, int r) {
        double v[CB];
#pragma unroll
        for (int c = 0; c < CB; ++c) v[c] = M[0][c];
#pragma unroll
        for (int rr = 1; rr < RB; ++rr)
#pragma unroll
            for (int c = 0; c < CB; ++c) v[c] = (r == rr) ? M[rr][c] : v[c];
        double *dst = T + (q & 1) * RL;
#pragma unroll
        for (int c = 0; c < CB; ++c) {
            const int j = j0 + c;
            dst[j] = (j <= q) ? 0.0 : v[c];
            if (j == q) dst[2 * W] = v[c];
        }
    };
    if (i0 == 0) put_row(0, 0);
    __syncthreads();
    for (int k = 0; k < W; ++k) {
        const int rk = k - i0;            // row k in this thread's block when 0 <= rk < RB
        const bool own_k = rk >= 0 && rk < RB;
        if (wlast > k) {
            const double *row = T + (k & 1) * RL;
            const double d = row[2 * W];
            double rr[RB], rc[CB];
#pragma unroll
            for (int r = 0; r < RB; ++r) rr[r] = row[i0 + r];
#pragma unroll
            for (int c = 0; c < CB; ++c) rc[c] = row[j0 + c];
            const double rinv = (d > 0.0) ? rsqrt_d(d) : 0.0;
            const double dinv = rinv * rinv;
#pragma unroll
            for (int c = 0; c < CB; ++c) rc[c] *= dinv;
#pragma unroll
            for (int r = 0; r < RB; ++r)
#pragma unroll
                for (int c = 0; c < CB; ++c) M[r][c] = fma(-rr[r], rc[c], M[r][c]);
            if (k + 1 < W && rk + 1 >= 0 && rk + 1 < RB) put_row(k + 1, rk + 1);
            if (own_k) {
#pragma unroll
                for (int r = 0; r < RB; ++r) sc[r] = (rk == r) ? rinv : sc[r];
            }
        } else if (own_k) {
            // the wave is done, but this thread still needs its scale for row k
            const double d = T[(k & 1) * RL + 2 * W];
            const double rinv = (d > 0.0) ? rsqrt_d(d) : 0.0;
#pragma unroll
            for (int r = 0; r < RB; ++r) sc[r] = (rk == r) ? rinv : sc[r];
        }
        __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
        for (int c = 0; c < CB; ++c) {
            const int i = i0 + r, j = j0 + c;
            const double v = M[r][c] * sc[r];
            if (j < W) {
                if (i <= j) S[i + j * LS] = v;
            } else {
                const int a = j - W;   // X[a][i] = (R^{-T})[i][a]
                Xs[a + i * LS] = (a <= i) ? v : 0.0;
            }
        }
    __syncthreads();
}

}  // namespace gram
}  // namespace qrx
