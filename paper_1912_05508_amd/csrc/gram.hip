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
// Three sweeps over the rows and two small kernels per panel:
//   gram_pass<G>    Gram partials of P over row chunks
//   gram_chol       fixed-order sum of the partials; the last workgroup to
//                   finish factors G1 -> R1, X1 = R1^{-1}
//   gram_pass<Q,G>  Q1 = fl32(P X1) written in place, and the Gram partials of
//                   the rounded Q1 rows while they are still in LDS
//   gram_chol       G2 -> R2, X2, and R = R2 R1 (FP32) into the R block
//   gram_pass<Q>    Q = fl32(Q1 X2) in place
// A sweep stages 64-row chunks of the panel in LDS as FP64; a workgroup owns a
// contiguous run of chunks and prefetches the next chunk into registers while
// it computes on the current one. With one sweep (no re-orthogonalisation)
// the panel is gram_pass<G>, gram_chol (R1 into the R block), gram_pass<Q>.
#include "qrx_internal.hpp"

namespace qrx {

constexpr int GT = 256;          // threads per sweep workgroup
constexpr int CH = 64;           // rows per LDS chunk
constexpr int CT = 512;          // threads per reduce/Cholesky workgroup
constexpr int kMaxParts = 256;   // Gram partials (one per sweep workgroup)

__device__ __host__ inline int upk(int i, int j) { return j * (j + 1) / 2 + i; }  // i <= j

// One sweep over the rows of P (m x w, column-major, ld). DO_Q: rows <- fl32(rows X)
// with X upper triangular (W x W, FP64, column-major). DO_G: part[blockIdx] =
// upper triangle of (rows)^T (rows) over this workgroup's chunks, FP64.
template <int W, bool DO_Q, bool DO_G>
__global__ __launch_bounds__(GT) void gram_pass_kernel(float *__restrict__ P, int64_t ld,
                                                       int64_t m, int w, int64_t chunks_per,
                                                       const double *__restrict__ X,
                                                       double *__restrict__ part) {
    constexpr int LDC = W + 2;                 // row stride of the chunk (16-byte aligned rows)
    constexpr int XLD = W + 2;                 // row stride of X in LDS
    constexpr int LPT = CH * W / GT;           // chunk elements each thread stages
    constexpr int TW = W / 4;                  // Gram: 4 x 4 register tiles
    constexpr int T = TW * TW;
    constexpr int G = GT / T;                  // Gram: row groups sharing a tile (1, 4, 16)
    constexpr int CB = W / 8;                  // Q formation: columns per block
    constexpr int NP = W * (W + 1) / 2;
    static_assert(GT % T == 0 && CH % G == 0 && GT == 4 * CH, "thread mapping");
    __shared__ __align__(16) double C[CH * LDC];
    __shared__ __align__(16) double Xs[DO_Q ? W * XLD : 2];          // row-major X
    __shared__ __align__(16) double red[(DO_G && G > 1) ? (GT / 2) * 16 : 2];
    const int t = threadIdx.x;
    const int64_t nch = (m + CH - 1) / CH;
    const int64_t ch0 = (int64_t)blockIdx.x * chunks_per;
    const int64_t ch1 = (ch0 + chunks_per < nch) ? ch0 + chunks_per : nch;

    if constexpr (DO_Q) {
        for (int idx = t; idx < W * W; idx += GT) {
            const int i = idx % W, j = idx / W;
            Xs[i * XLD + j] = X[idx];
        }
    }
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
    double acc[4][4];
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) acc[x][y] = 0.0;
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
    if constexpr (DO_G) {
        if constexpr (G > 1) {
            // tree over the row groups: group g += group g + h for h = G/2, ..., 1
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
            double *out = part + (int64_t)blockIdx.x * NP;
#pragma unroll
            for (int x = 0; x < 4; ++x)
#pragma unroll
                for (int y = 0; y < 4; ++y) {
                    const int i = ti * 4 + x, j = tj * 4 + y;
                    if (i <= j) out[upk(i, j)] = acc[x][y];
                }
        }
    }
}

// G[e] = sum over the partials: a workgroup owns 64 entries (one per lane),
// its 8 waves sum interleaved subsets of the partials and the 8 sums are added
// in a fixed order (deterministic). The last workgroup to finish then computes
// R = chol(G) (upper, G = R^T R) and X = R^{-1}, both FP64 (W x W, column-
// major), by one symmetric elimination of [G | I]: step k subtracts multiples
// of row k from the rows below it, which leaves U = D L^T in the upper triangle
// and L^{-1} (unit lower) in the strictly-lower triangle, so R = D^{-1/2} U and
// R^{-1} = L^{-T} D^{-1/2}. One barrier per step. If Rfinal is set, it also
// writes the panel's R block (FP32, ldr): R Rprev when Rprev is set, else R.
// A pivot <= 0 gives a zero row of R and a zero column of X.
// *counter must be 0 on entry; the last workgroup leaves it 0.
template <int W>
__global__ __launch_bounds__(CT) void gram_chol_kernel(const double *__restrict__ part, int nparts,
                                                       int w, double *__restrict__ G,
                                                       int *__restrict__ counter,
                                                       double *__restrict__ Rout,
                                                       double *__restrict__ Xout,
                                                       const double *__restrict__ Rprev,
                                                       float *__restrict__ Rfinal, int64_t ldr) {
    constexpr int NP = W * (W + 1) / 2;
    constexpr int LS = W + 1;
    constexpr int NW = CT / 64;                     // waves
    constexpr int NG = (CT / W < W) ? CT / W : W;   // column groups per row in the elimination
    constexpr int QN = W / NG;
    __shared__ double S[W * LS];        // S[i + j*LS]; upper: G -> U, strictly lower: L^{-1}
    __shared__ double Rp[W * W];        // Rprev
    __shared__ double sums[NW * 64];
    __shared__ double dg[W];            // D_kk^{-1/2} (0 for a non-positive pivot)
    __shared__ int last;
    const int t = threadIdx.x;
    const int lane = t & 63, wv = t >> 6;
    const int e = blockIdx.x * 64 + lane;
    {
        double s = 0.0;
        if (e < NP)
            for (int b = wv; b < nparts; b += NW) s += part[(int64_t)b * NP + e];
        sums[wv * 64 + lane] = s;
    }
    __syncthreads();
    if (wv == 0 && e < NP) {
        double s = sums[lane];
#pragma unroll
        for (int q = 1; q < NW; ++q) s += sums[q * 64 + lane];
        G[e] = s;
    }
    __threadfence();
    __syncthreads();
    if (t == 0) last = (atomicAdd(counter, 1) == (int)gridDim.x - 1);
    __syncthreads();
    if (!last) return;
    __threadfence();
    if (t == 0) atomicExch(counter, 0);

    for (int idx = t; idx < W * W; idx += CT) {
        const int i = idx % W, j = idx / W;
        S[i + j * LS] = (i <= j && j < w) ? G[upk(i, j)] : 0.0;
        if (Rprev) Rp[idx] = Rprev[idx];
    }
    __syncthreads();
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
    for (int idx = t; idx < W * W; idx += CT) {
        const int i = idx % W, j = idx / W;
        // R[i][j] = U[i][j] D_i^{-1/2};  X[i][j] = Linv[j][i] D_j^{-1/2} (i <= j)
        const bool up = i <= j && j < w;
        Rout[idx] = up ? S[i + j * LS] * dg[i] : 0.0;
        Xout[idx] = up ? ((i == j) ? 1.0 : S[j + i * LS]) * dg[j] : 0.0;
    }
    if (Rfinal) {
        for (int idx = t; idx < W * W; idx += CT) {
            const int i = idx % W, j = idx / W;
            if (i >= w || j >= w) continue;
            double v = 0.0;
            if (i <= j) {
                if (Rprev) {
                    for (int l = i; l <= j; ++l) v = fma(S[i + l * LS], Rp[l + j * W], v);
                    v *= dg[i];
                } else {
                    v = S[i + j * LS] * dg[i];
                }
            }
            Rfinal[i + (int64_t)j * ldr] = (float)v;
        }
    }
}

// ---------------------------------------------------------------------------
struct GramSplit {
    int parts;
    int64_t chunks_per;
};

static GramSplit gram_split(int64_t m) {
    const int64_t nch = (m + CH - 1) / CH;
    int64_t parts = nch < kMaxParts ? nch : kMaxParts;
    if (parts < 1) parts = 1;
    const int64_t per = (nch + parts - 1) / parts;
    parts = (nch + per - 1) / per;
    if (parts < 1) parts = 1;
    return {(int)parts, per};
}

// Workspace (doubles): parts * W(W+1)/2 + W(W+1)/2 + 4 W^2, then one double
// whose first word is the completion counter of gram_chol.
size_t gram_workspace_doubles(int64_t m, int W) {
    const size_t np = (size_t)W * (W + 1) / 2;
    return (size_t)gram_split(m).parts * np + np + 4 * (size_t)W * W + 1;
}

int *gram_counter(double *ws, int64_t m) {
    return reinterpret_cast<int *>(ws + gram_workspace_doubles(m, 64) - 1);
}

template <int W>
static hipError_t gram_go(hipStream_t s, float *P, int64_t ld, int64_t m, int w, float *R,
                          int64_t ldr, double *ws, int reorth) {
    const int64_t np = (int64_t)W * (W + 1) / 2;
    const GramSplit sp = gram_split(m);
    double *part = ws;
    double *G = part + (size_t)sp.parts * np;
    double *R1 = G + np;
    double *X1 = R1 + W * W;
    double *R2 = X1 + W * W;
    double *X2 = R2 + W * W;
    int *counter = gram_counter(ws, m);
    const unsigned cb = (unsigned)((np + 63) / 64);
    hipLaunchKernelGGL((gram_pass_kernel<W, false, true>), dim3(sp.parts), dim3(GT), 0, s, P, ld,
                       m, w, sp.chunks_per, (const double *)nullptr, part);
    hipLaunchKernelGGL(gram_chol_kernel<W>, dim3(cb), dim3(CT), 0, s, (const double *)part,
                       sp.parts, w, G, counter, R1, X1, (const double *)nullptr,
                       reorth ? (float *)nullptr : R, ldr);
    if (!reorth) {
        hipLaunchKernelGGL((gram_pass_kernel<W, true, false>), dim3(sp.parts), dim3(GT), 0, s, P,
                           ld, m, w, sp.chunks_per, (const double *)X1, (double *)nullptr);
        return hipGetLastError();
    }
    hipLaunchKernelGGL((gram_pass_kernel<W, true, true>), dim3(sp.parts), dim3(GT), 0, s, P, ld,
                       m, w, sp.chunks_per, (const double *)X1, part);
    hipLaunchKernelGGL(gram_chol_kernel<W>, dim3(cb), dim3(CT), 0, s, (const double *)part,
                       sp.parts, w, G, counter, R2, X2, (const double *)R1, R, ldr);
    hipLaunchKernelGGL((gram_pass_kernel<W, true, false>), dim3(sp.parts), dim3(GT), 0, s, P, ld,
                       m, w, sp.chunks_per, (const double *)X2, (double *)nullptr);
    return hipGetLastError();
}

hipError_t launch_gram_panel(hipStream_t s, float *P, int64_t ld, int64_t m, int w, float *R,
                             int64_t ldr, double *ws, int reorth) {
    if (w <= 16) return gram_go<16>(s, P, ld, m, w, R, ldr, ws, reorth);
    if (w <= 32) return gram_go<32>(s, P, ld, m, w, R, ldr, ws, reorth);
    return gram_go<64>(s, P, ld, m, w, R, ldr, ws, reorth);
}

}  // namespace qrx
