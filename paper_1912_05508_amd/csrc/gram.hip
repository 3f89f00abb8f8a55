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
// Three sweeps over the rows and two small steps per panel:
//   gram_pass<G>    Gram partials of P over row chunks
//   gram_reduce     fixed-order sums of the partials in a few slices (many
//                   workgroups; skipped when there are only a few partials)
//   gram_chol       one workgroup: adds the slices, factors G1 -> R1,
//                   X1 = R1^{-1}
//   gram_pass<Q,G>  Q1 = fl32(P X1) written in place, and the Gram partials of
//                   the rounded Q1 rows while they are still in LDS
//   gram_reduce, gram_chol   G2 -> R2, X2, and R = R2 R1 (FP32) into the R block
//   gram_pass<Q>    Q = fl32(Q1 X2) in place
// The reductions pass their sums on through kernel boundaries, with no
// device-wide fences or counters.
// A sweep stages 64-row chunks of the panel in LDS as FP64; a workgroup owns a
// contiguous run of chunks and prefetches the next chunk into registers while
// it computes on the current one. 64-column panels compute their Gram blocks
// and Q formation on the FP64 matrix cores. With one sweep (no re-orthogonalisation)
// the panel is gram_pass<G>, gram_reduce, gram_chol (R1 into the R block),
// gram_pass<Q>.
#include "gram_common.hpp"

#include <algorithm>

namespace qrx {

using gram::CH;
using gram::GT;
using gram::upk;
constexpr int CT = 512;          // threads per reduce/Cholesky workgroup
constexpr int kMaxParts = 512;   // Gram partials (one per sweep workgroup)
constexpr int kMaxSlices = 8;    // first-level reduction workgroups per column block
constexpr int kSliceParts = 64;  // partials summed by one of them (8 per wave)
constexpr int kDirectParts = 8;  // at most this many partials go to gram_chol unreduced
static_assert(kMaxSlices <= kDirectParts, "gram_chol sums at most kDirectParts partials");

// ---------------------------------------------------------------------------
// 64-column sweeps on the FP64 matrix cores (v_mfma_f64_16x16x4f64: A operand
// lane l holds A[l % 16][l / 16], B operand B[l / 16][l % 16], result register
// v of lane l holds D[4 v + l / 16][l % 16]).
// Gram: the 10 upper 16 x 16 blocks (I, J) of rows^T rows are split over the 4
// waves (3, 3, 2, 2 blocks), each over all rows of the chunk in steps of 4.
// Q formation: wave Rb forms rows 16 Rb .. 16 Rb + 15 of rows X, its 4 column
// blocks over K up to the block's last column (X is upper triangular).
// ---------------------------------------------------------------------------
typedef double d4 __attribute__((ext_vector_type(4)));

QRX_DEV d4 mfma64(double a, double b, d4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// block pairs of wave wv: (I, J) = pair(wv, p) for p < npairs(wv)
QRX_DEV int npairs(int wv) { return wv < 2 ? 3 : 2; }
QRX_DEV void pair_of(int wv, int p, int &I, int &J) {
    // 0: (0,0) (0,1) (0,2)   1: (0,3) (1,1) (1,2)   2: (1,3) (2,2)   3: (2,3) (3,3)
    const int code = wv * 3 + p;
    const int Is[12] = {0, 0, 0, 0, 1, 1, 1, 2, 0, 2, 3, 0};
    const int Js[12] = {0, 1, 2, 3, 1, 2, 3, 2, 0, 3, 3, 0};
    I = Is[code];
    J = Js[code];
}

// v as a 16-bit operand element (and its low part for a split) at index i
QRX_DEV void store16(uint16_t *h, uint16_t *l, int64_t i, float v, int prec) {
    if (prec == QRX_BF16) {
        const __bf16 b = (__bf16)v;
        h[i] = *reinterpret_cast<const uint16_t *>(&b);
        return;
    }
    const _Float16 f = (_Float16)v;
    h[i] = *reinterpret_cast<const uint16_t *>(&f);
    if (prec == QRX_FP16X3) {
        const _Float16 g = (_Float16)(v - (float)f);
        l[i] = *reinterpret_cast<const uint16_t *>(&g);
    }
}

template <bool DO_Q, bool DO_G>
QRX_DEV void sweep64(float *__restrict__ P, int64_t ld, int64_t m, int w, int64_t ch0,
                     int64_t ch1, const double *Xs, double *C, d4 (&acc)[3], int t,
                     const PanelPack &pk) {
    using L = gram::Lds<64>;
    constexpr int LDC = L::LDC, XLD = L::XLD;
    constexpr int LPT = CH * 64 / GT;
    const int lane = t & 63;
    const int wv = __builtin_amdgcn_readfirstlane(t >> 6);
    const int li = lane & 15, lk = lane >> 4;
    const int np = npairs(wv);
    int PI[3], PJ[3];
#pragma unroll
    for (int p = 0; p < 3; ++p) pair_of(wv, p < np ? p : 0, PI[p], PJ[p]);
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
            const int Rb = wv;
            d4 q[4];
#pragma unroll
            for (int Jb = 0; Jb < 4; ++Jb) {
                q[Jb] = d4{0.0, 0.0, 0.0, 0.0};
                for (int k4 = 0; k4 < 4 * (Jb + 1); ++k4) {
                    const double a = C[(16 * Rb + li) * LDC + 4 * k4 + lk];
                    const double b = Xs[(4 * k4 + lk) * XLD + 16 * Jb + li];
                    q[Jb] = mfma64(a, b, q[Jb]);
                }
            }
            __syncthreads();   // every wave has read its rows of the chunk
#pragma unroll
            for (int Jb = 0; Jb < 4; ++Jb)
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    C[(16 * Rb + 4 * v + lk) * LDC + 16 * Jb + li] = (double)(float)q[Jb][v];
            __syncthreads();
            // Q1 rows back to P, coalesced along the columns
#pragma unroll
            for (int s = 0; s < LPT; ++s) {
                const int e = t + GT * s;
                const int rr = e % CH, cc = e / CH;
                const int64_t r = ch * CH + rr;
                if (r < m && cc < w) P[r + cc * ld] = (float)C[rr * LDC + cc];
            }
            if (pk.prec) {
                // the operand copies: column-major coalesced along the columns,
                // row-major along the rows (few in flight: registers are scarce here)
#pragma unroll 1
                for (int s = 0; s < LPT; ++s) {
                    const int e = t + GT * s;
                    const int rr = e % CH, cc = e / CH;
                    const int64_t r = ch * CH + rr;
                    if (r < m && cc < w)
                        store16(pk.qc, pk.qcl, r + cc * pk.ldc,
                                (float)C[rr * LDC + cc] * pk.sc, pk.prec);
                }
#pragma unroll 1
                for (int s = 0; s < LPT; ++s) {
                    const int e = t + GT * s;
                    const int cc = e % 64, rr = e / 64;
                    const int64_t r = ch * CH + rr;
                    if (r < m && cc < w)
                        store16(pk.qr, pk.qrl, r * pk.ldq + cc, (float)C[rr * LDC + cc] * pk.sc,
                                pk.prec);
                }
            }
        }
        if constexpr (DO_G) {
            for (int k4 = 0; k4 < CH / 4; ++k4) {
                const double *row = C + (4 * k4 + lk) * LDC + li;
#pragma unroll
                for (int p = 0; p < 3; ++p)
                    if (p < np) acc[p] = mfma64(row[16 * PI[p]], row[16 * PJ[p]], acc[p]);
            }
        }
    }
}

// this wave's Gram blocks into out[upk(i, j)], i <= j
QRX_DEV void gram_store64(const d4 (&acc)[3], double *out, int t) {
    const int lane = t & 63;
    const int wv = __builtin_amdgcn_readfirstlane(t >> 6);
    const int np = npairs(wv);
#pragma unroll
    for (int p = 0; p < 3; ++p) {
        if (p >= np) continue;
        int I, J;
        pair_of(wv, p, I, J);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int i = 16 * I + 4 * v + (lane >> 4), j = 16 * J + (lane & 15);
            if (i <= j) out[upk(i, j)] = acc[p][v];
        }
    }
}

// One sweep over this workgroup's row chunks of P (m x w, column-major, ld).
// DO_Q: rows <- fl32(rows X) with X upper triangular (W x W, FP64, column-
// major). DO_G: part[blockIdx] = upper triangle of (rows)^T (rows), FP64.
// R = Ra Rb for the panel's R block: both upper triangular (W x W, FP64,
// column-major, zero below the diagonal); Rfinal gets the w x w FP32 result
// (lower part zero), column stride ldr. Ra and Rb are staged in A and B (LDS).
struct RProd {
    const double *Ra, *Rb;
    float *Rfinal;
    int64_t ldr;
};

template <int W>
QRX_DEV void r_product(const RProd &rp, int w, double *A, double *B, int t) {
    constexpr int TW = W / 4;
    for (int idx = t; idx < W * W; idx += GT) {
        A[idx] = rp.Ra[idx];
        B[idx] = rp.Rb[idx];
    }
    __syncthreads();
    for (int tile = t; tile < TW * TW; tile += GT) {
        const int i0 = 4 * (tile % TW), j0 = 4 * (tile / TW);
        double v[4][4];
#pragma unroll
        for (int p = 0; p < 4; ++p)
#pragma unroll
            for (int q = 0; q < 4; ++q) v[p][q] = 0.0;
        for (int l = i0; l <= j0 + 3; ++l) {   // Ra[i][l] = 0 for l < i, Rb[l][j] = 0 for l > j
            double a[4], b[4];
#pragma unroll
            for (int p = 0; p < 4; ++p) a[p] = A[(i0 + p) + l * W];
#pragma unroll
            for (int q = 0; q < 4; ++q) b[q] = B[l + (j0 + q) * W];
#pragma unroll
            for (int p = 0; p < 4; ++p)
#pragma unroll
                for (int q = 0; q < 4; ++q) v[p][q] = fma(a[p], b[q], v[p][q]);
        }
#pragma unroll
        for (int p = 0; p < 4; ++p)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int i = i0 + p, j = j0 + q;
                if (i < w && j < w) rp.Rfinal[i + (int64_t)j * rp.ldr] = (float)v[p][q];
            }
    }
}

// The sweep of one workgroup over its chunks (see gram_pass_kernel).
template <int W, bool DO_Q, bool DO_G>
QRX_DEV void pass_body(float *__restrict__ P, int64_t ld, int64_t m, int w, int64_t chunks_per,
                       const double *__restrict__ X, double *__restrict__ part, const PanelPack &pk,
                       double *C, double *Xs, double *red, int t) {
    const int64_t nch = (m + CH - 1) / CH;
    const int64_t ch0 = (int64_t)blockIdx.x * chunks_per;
    const int64_t ch1 = (ch0 + chunks_per < nch) ? ch0 + chunks_per : nch;
    if constexpr (DO_Q) gram::load_x<W>(X, Xs, t);
    if constexpr (W == 64) {
        d4 acc[3];
#pragma unroll
        for (int p = 0; p < 3; ++p) acc[p] = d4{0.0, 0.0, 0.0, 0.0};
        sweep64<DO_Q, DO_G>(P, ld, m, w, ch0, ch1, Xs, C, acc, t, pk);
        if constexpr (DO_G) gram_store64(acc, part + (int64_t)blockIdx.x * (W * (W + 1) / 2), t);
        (void)red;
    } else if constexpr (W == 32) {
        gram::gd4 acc[3];
#pragma unroll
        for (int p = 0; p < 3; ++p) acc[p] = gram::gd4{0.0, 0.0, 0.0, 0.0};
        gram::sweep32<DO_Q, DO_G>(P, ld, m, w, ch0, ch1, Xs, C, acc, t);
        if constexpr (DO_G)
            gram::gram_store32(acc, red, part + (int64_t)blockIdx.x * (W * (W + 1) / 2), t);
    } else {
        double acc[4][4];
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
            for (int y = 0; y < 4; ++y) acc[x][y] = 0.0;
        gram::sweep<W, DO_Q, DO_G>(P, ld, m, w, ch0, ch1, Xs, C, acc, t);
        if constexpr (DO_G)
            gram::gram_store<W>(acc, red, part + (int64_t)blockIdx.x * (W * (W + 1) / 2), t);
    }
}

// The final sweep (DO_Q only) may carry the R product: one extra workgroup,
// the last, computes it while the others sweep. With skip set the sweep does
// nothing (an earlier step finished the panel). With nogram set, a DO_Q, DO_G
// sweep forms Q only (the first Cholesky factor was well conditioned enough
// that the panel needs no second pass).
template <int W, bool DO_Q, bool DO_G>
__global__ __launch_bounds__(GT, 2) void gram_pass_kernel(float *__restrict__ P, int64_t ld,
                                                       int64_t m, int w, int64_t chunks_per,
                                                       const double *__restrict__ X,
                                                       double *__restrict__ part,
                                                       const int *__restrict__ skip,
                                                       const int *__restrict__ nogram,
                                                       PanelPack pk, RProd rp) {
    if (skip && *skip) return;   // the panel is already finished
    using L = gram::Lds<W>;
    __shared__ __align__(16) double C[L::C_DOUBLES];
    __shared__ __align__(16) double Xs[DO_Q ? L::X_DOUBLES : 2];
    __shared__ __align__(16) double red[DO_G ? L::RED_DOUBLES : 2];
    const int t = threadIdx.x;
    if constexpr (DO_Q && !DO_G) {
        static_assert(L::C_DOUBLES >= W * W && L::X_DOUBLES >= W * W, "R product staging");
        if (rp.Rfinal && blockIdx.x == gridDim.x - 1) {
            r_product<W>(rp, w, C, Xs, t);
            return;
        }
    }
    if constexpr (DO_Q && DO_G) {
        if (nogram && *nogram) {
            pass_body<W, true, false>(P, ld, m, w, chunks_per, X, part, pk, C, Xs, red, t);
            return;
        }
    }
    pass_body<W, DO_Q, DO_G>(P, ld, m, w, chunks_per, X, part, pk, C, Xs, red, t);
}

// First level of the Gram reduction when there are many partials: workgroup
// (x, y) sums entries 64x .. 64x + 63 of the partials y, y + NS, y + 2 NS, ...
// (NS = gridDim.y) into lvl[y]; its 8 waves sum interleaved subsets and the 8
// sums are added in a fixed order (deterministic). A kernel of its own: the
// sums reach gram_chol through the kernel boundary, with no fence.
template <int W>
__global__ __launch_bounds__(CT) void gram_reduce_kernel(const double *__restrict__ part,
                                                         int nparts, double *__restrict__ lvl,
                                                         const int *__restrict__ skip) {
    if (skip && *skip) return;   // the panel is already finished
    constexpr int NP = W * (W + 1) / 2;
    constexpr int NW = CT / 64;
    constexpr int RB = 8;
    __shared__ double Ub[NW * 64];
    const int t = threadIdx.x;
    const int lane = t & 63, wv = t >> 6;
    const int e = blockIdx.x * 64 + lane;
    const int NS = gridDim.y, slice = blockIdx.y;
    const int K = (nparts - slice + NS - 1) / NS;   // partials slice + k NS, k < K
    double s = 0.0;
    if (e < NP) {
        int k = wv;
        for (; k + (RB - 1) * NW < K; k += RB * NW) {
            double v[RB];
#pragma unroll
            for (int q = 0; q < RB; ++q) v[q] = part[(int64_t)(slice + (k + q * NW) * NS) * NP + e];
#pragma unroll
            for (int q = 0; q < RB; ++q) s += v[q];
        }
        double v[RB];
#pragma unroll
        for (int q = 0; q < RB; ++q) {
            const int kq = k + q * NW;
            v[q] = kq < K ? part[(int64_t)(slice + kq * NS) * NP + e] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < RB; ++q) s += v[q];
    }
    Ub[wv * 64 + lane] = s;
    __syncthreads();
    if (wv == 0 && e < NP) {
        double g = Ub[lane];
#pragma unroll
        for (int q = 1; q < NW; ++q) g += Ub[q * 64 + lane];
        lvl[(int64_t)slice * NP + e] = g;
    }
}

// One workgroup: G = the sum of nparts partials (a few, after gram_reduce),
// added in partial order, then G = R^T R by gram::chol_inv, writing R and
// X = R^{-1} (FP64, W x W, column-major). If Rfinal is set, it also writes the
// panel's R block (FP32, ldr): R when Rprev is null; R Rprev when Rprev is set
// and prod is nonzero (prod 0 leaves that product to the final sweep).
// With skip set (second sweep: G is the Gram matrix of the rounded Q1), a G
// within tau of the identity in every entry means Q1 is already orthonormal
// to working accuracy: then R = Rprev is written, *skip = 1 and the final
// sweep does nothing; otherwise *skip = 0 and the factorisation proceeds.
//
// pre: if set and nonzero on entry, the panel is already finished (the kernel
// returns at once). kflag (first factorisation of a re-orthogonalised panel):
// the kernel bounds kappa_2 of the column-equilibrated factor R D^-1 (D the
// column norms of R, i.e. sqrt of the diagonal of G); at most ktau, one pass
// has left Q1 orthonormal to FP32 accuracy (Cholesky QR with an FP64 Gram
// matrix loses orthogonality like kappa^2 u64 of the equilibrated panel:
// 2^28 2^-53 < 2^-24), so it writes R into the panel's R block and *kflag = 1
// (the second pass then forms Q only and its Gram steps are skipped);
// otherwise *kflag = 0 and R is left to the second factorisation.
// nparts is at most kDirectParts (the callers reduce more partials first).
template <int W>
__global__ __launch_bounds__(CT) void gram_chol_kernel(const double *__restrict__ part, int nparts,
                                                       int w, double *__restrict__ Rout,
                                                       double *__restrict__ Xout,
                                                       const double *__restrict__ Rprev,
                                                       float *__restrict__ Rfinal, int64_t ldr,
                                                       int *__restrict__ skip, double tau,
                                                       int prod, const int *__restrict__ pre,
                                                       int *__restrict__ kflag, double ktau) {
    if (pre && *pre) return;
    constexpr int NP = W * (W + 1) / 2;
    constexpr int LS = W + 1;
    constexpr int NW = CT / 64;
    constexpr int NQ = (W * W + CT - 1) / CT;   // entries of a W x W matrix per thread
    constexpr int TP = (W == 64 && CT == 512) ? gram::kCholT64 : 4 * W + 4;   // pivot rows
    constexpr int U = (NW > TP) ? NW : TP;      // wave maxima, then pivot rows
    __shared__ double S[W * LS];       // G, then R (upper)
    __shared__ double Xs[W * LS];      // R^{-1}, then Rprev
    __shared__ __align__(16) double Ub[U];   // wave maxima, then pivot rows of the elimination
    __shared__ double dnb[W];          // column norms of the factor (single-pass bound)
    const int t = threadIdx.x;
    const int lane = t & 63, wv = t >> 6;
    // G = the sum of the partials, in partial order. Thread t takes the pairs
    // of packed entries 2k, 2k + 1 for k = t, t + CT, ...: 16-byte loads, all
    // in flight at once (one round trip to memory).
    constexpr int NP2 = NP / 2, NC = (NP2 + CT - 1) / CT;
    static_assert(NP % 2 == 0, "packed Gram blocks hold an even number of entries");
    double2 gv[NC];
    {
        const double2 *p2 = reinterpret_cast<const double2 *>(part);
        double2 v[kDirectParts][NC];
#pragma unroll
        for (int b = 0; b < kDirectParts; ++b)
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                const int k = t + c * CT;
                v[b][c] = (b < nparts && k < NP2) ? p2[(int64_t)b * NP2 + k] : make_double2(0.0, 0.0);
            }
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            gv[c] = v[0][c];
#pragma unroll
            for (int b = 1; b < kDirectParts; ++b) {
                gv[c].x += v[b][c].x;
                gv[c].y += v[b][c].y;
            }
        }
    }
    // S: G in the upper triangle (zero in columns >= w), zero below it
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const int idx = t + q * CT, i = idx % W, j = idx / W;
        if (idx < W * W && i > j) S[i + j * LS] = 0.0;
    }
    double dev = 0.0;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        const int k = t + c * CT;
        if (k >= NP2) continue;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int e = 2 * k + h;
            // e = j (j + 1) / 2 + i, 0 <= i <= j
            int j = (int)((sqrtf(8.0f * (float)e + 1.0f) - 1.0f) * 0.5f);
            if (j * (j + 1) / 2 > e) --j;
            if ((j + 1) * (j + 2) / 2 <= e) ++j;
            const int i = e - j * (j + 1) / 2;
            const double g = j < w ? (h ? gv[c].y : gv[c].x) : 0.0;
            S[i + j * LS] = g;
            if (j < w) {
                if (i == j) dnb[i] = sqrt(g);   // column norms of R
                const double e2 = fabs(g - (i == j ? 1.0 : 0.0));
                dev = fmax(dev, (e2 == e2) ? e2 : 1e300);   // a NaN entry never passes
            }
        }
    }
    if (skip) {
        // max |G - I| over the workgroup (fixed reduction; the flag is uniform)
#pragma unroll
        for (int o2 = 32; o2 > 0; o2 >>= 1) dev = fmax(dev, __shfl_xor(dev, o2));
        if (lane == 0) Ub[wv] = dev;
        __syncthreads();
        double mx = 0.0;
#pragma unroll
        for (int q = 0; q < NW; ++q) mx = fmax(mx, Ub[q]);
        const bool done = mx <= tau;   // NaN compares false: factorise
        if (t == 0) *skip = done ? 1 : 0;
        if (done) {
            double rv[NQ];
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                const int idx = t + q * CT;
                rv[q] = (idx < W * W) ? Rprev[idx] : 0.0;
            }
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                const int idx = t + q * CT, i = idx % W, j = idx / W;
                if (idx < W * W && i < w && j < w) Rfinal[i + (int64_t)j * ldr] = (float)rv[q];
            }
            return;
        }
    }
    __syncthreads();
    gram::chol_inv<W, CT>(S, Xs, Ub, t);
    for (int idx = t; idx < W * W; idx += CT) {
        const int i = idx % W, j = idx / W;
        const bool up = i <= j && j < w;
        Rout[idx] = up ? S[i + j * LS] : 0.0;
        Xout[idx] = up ? Xs[i + j * LS] : 0.0;
    }
    if (kflag) {
        // kappa_2(R D^-1) <= ||R D^-1||_F ||D X||_F = sqrt(w) ||D X||_F, the
        // columns of R D^-1 having unit norm. Cholesky's rounding errors are
        // relative to the columns' scale, so this, not kappa(R) itself, governs
        // the orthogonality of one pass. A zero or non-finite pivot never passes.
        double a = 0.0;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int idx = t + q * CT, i = idx % W, j = idx / W;
            if (idx < W * W && i <= j && j < w) {
                const double v = dnb[i] * Xs[i + j * LS];
                a = fma(v, v, a);
                if (i == j && !(S[i + i * LS] > 0.0 && dnb[i] > 0.0)) a = HUGE_VAL;
            }
        }
#pragma unroll
        for (int o2 = 32; o2 > 0; o2 >>= 1) a += __shfl_xor(a, o2);
        if (lane == 0) Ub[wv] = a;
        __syncthreads();
        double fro2 = Ub[0];
#pragma unroll
        for (int q = 1; q < NW; ++q) fro2 += Ub[q];
        const double est2 = (double)w * fro2;                      // >= kappa_2(R D^-1)^2
        const bool ok = est2 <= ktau * ktau;                        // NaN: keep the second pass
        if (t == 0) *kflag = ok ? 1 : 0;
        if (!ok) return;
    } else if (!Rfinal || (Rprev && !prod)) {
        return;
    }
    if (Rprev) {
        double rv[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int idx = t + q * CT;
            rv[q] = (idx < W * W) ? Rprev[idx] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int idx = t + q * CT;
            if (idx < W * W) Xs[(idx % W) + (idx / W) * LS] = rv[q];
        }
        __syncthreads();
    }
    // R (or R Rprev) in 2 x 4 tiles; the lower parts of S and Rprev are zero
    for (int tile = t; tile < (W / 2) * (W / 4); tile += CT) {
        const int i0 = 2 * (tile % (W / 2)), j0 = 4 * (tile / (W / 2));
        double v[2][4];
#pragma unroll
        for (int p2 = 0; p2 < 2; ++p2)
#pragma unroll
            for (int q = 0; q < 4; ++q) v[p2][q] = 0.0;
        if (Rprev) {
            for (int l = i0; l <= j0 + 3; ++l) {
                const double a0 = S[i0 + l * LS], a1 = S[i0 + 1 + l * LS];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const double bq = Xs[l + (j0 + q) * LS];
                    v[0][q] = fma(a0, bq, v[0][q]);
                    v[1][q] = fma(a1, bq, v[1][q]);
                }
            }
        } else {
#pragma unroll
            for (int p2 = 0; p2 < 2; ++p2)
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    v[p2][q] = (i0 + p2 <= j0 + q) ? S[(i0 + p2) + (j0 + q) * LS] : 0.0;
        }
#pragma unroll
        for (int p2 = 0; p2 < 2; ++p2)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int i = i0 + p2, j = j0 + q;
                if (i < w && j < w) Rfinal[i + (int64_t)j * ldr] = (float)v[p2][q];
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

// first-level workgroups per column block for nparts partials (0: none)
static int gram_slices(int nparts) {
    if (nparts <= kDirectParts) return 0;
    const int s = (nparts + kSliceParts - 1) / kSliceParts;
    return s > kMaxSlices ? kMaxSlices : s;
}

// 128-column panels: at most this many partials (two chunks per sweep workgroup
// at m = 32768; a partial is 66 KB)
constexpr int kLeafParts = 256;

static GramSplit leaf_split(int64_t m) {
    const int64_t nch = (m + CH - 1) / CH;
    int64_t parts = nch < kLeafParts ? nch : kLeafParts;
    if (parts < 1) parts = 1;
    const int64_t per = (nch + parts - 1) / parts;
    parts = (nch + per - 1) / per;
    if (parts < 1) parts = 1;
    return {(int)parts, per};
}

// Workspace (doubles): kGramCounterInts ints of flags (the skip flag of the
// second sweep at index 1, the rest spare), then parts * W(W+1)/2 (partials),
// 4 W^2 (R1, X1, R2, X2) and kMaxSlices * W(W+1)/2 (slice sums). Sized for
// panels up to wmax columns (64 or 128).
size_t gram_workspace_doubles(int64_t m, int wmax) {
    size_t n = 0;
    for (int W : {64, 128}) {
        if (W > wmax) break;
        const size_t np = (size_t)W * (W + 1) / 2;
        const size_t parts = W == 128 ? leaf_split(m).parts : gram_split(m).parts;
        n = std::max(n, parts * np + 4 * (size_t)W * W + kMaxSlices * np);
    }
    return kGramCounterInts / 2 + n;
}

int *gram_counter(double *ws) { return reinterpret_cast<int *>(ws); }

// Re-orthogonalisation is skipped when every entry of Q1^T Q1 is within this
// of the identity (a few FP32 rounding units: a second sweep could not do better).
constexpr double kSkipTau = 1.0 / (1 << 21);
// One Cholesky QR pass suffices when the bound of kappa_2(R1) is at most
// kCondTau (see gram_chol_kernel): kappa^2 u64 = 2^28 2^-53 stays below FP32
// rounding.
constexpr double kCondTau = 16384.0;

template <int W>
static hipError_t gram_go(hipStream_t s, float *P, int64_t ld, int64_t m, int w, float *R,
                          int64_t ldr, double *ws, int reorth, const PanelPack &pack) {
    PanelPack none = pack;
    none.prec = 0;
    const PanelPack &pk = (W == 64) ? pack : none;   // sweeps of width 64 write the copies
    const int64_t np = (int64_t)W * (W + 1) / 2;
    const GramSplit sp = gram_split(m);
    double *part = ws + kGramCounterInts / 2;
    double *R1 = part + (size_t)sp.parts * np;
    double *X1 = R1 + W * W;
    double *R2 = X1 + W * W;
    double *X2 = R2 + W * W;
    double *lvl = X2 + W * W;
    int *skip = gram_counter(ws) + 1;
    const unsigned cb = (unsigned)((np + 63) / 64);
    const int ns = gram_slices(sp.parts);
    // partials as gram_chol reads them: the slice sums when there are many
    const double *cpart = ns ? lvl : part;
    const int cparts = ns ? ns : sp.parts;
    auto reduce = [&](const int *pre) {
        if (ns)
            hipLaunchKernelGGL(gram_reduce_kernel<W>, dim3(cb, ns), dim3(CT), 0, s,
                               (const double *)part, sp.parts, lvl, pre);
    };
    const int *noskip = nullptr;
    hipLaunchKernelGGL((gram_pass_kernel<W, false, true>), dim3(sp.parts), dim3(GT), 0, s, P, ld,
                       m, w, sp.chunks_per, (const double *)nullptr, part, noskip, noskip, none,
                       RProd{});
    reduce(noskip);
    if (!reorth) {
        hipLaunchKernelGGL(gram_chol_kernel<W>, dim3(1), dim3(CT), 0, s, cpart, cparts, w, R1, X1,
                           (const double *)nullptr, R, ldr, (int *)nullptr, 0.0, 0, noskip,
                           (int *)nullptr, 0.0);
        hipLaunchKernelGGL((gram_pass_kernel<W, true, false>), dim3(sp.parts), dim3(GT), 0, s, P,
                           ld, m, w, sp.chunks_per, (const double *)X1, (double *)nullptr, noskip,
                           noskip, pk, RProd{});
        return hipGetLastError();
    }
    // first factorisation; when R1 is well conditioned it finishes the panel's R
    // and sets *skip: the second pass then forms Q only, and the second
    // reduction, factorisation and final sweep do nothing
    hipLaunchKernelGGL(gram_chol_kernel<W>, dim3(1), dim3(CT), 0, s, cpart, cparts, w, R1, X1,
                       (const double *)nullptr, R, ldr, (int *)nullptr, 0.0, 0, noskip, skip,
                       kCondTau);
    hipLaunchKernelGGL((gram_pass_kernel<W, true, true>), dim3(sp.parts), dim3(GT), 0, s, P, ld,
                       m, w, sp.chunks_per, (const double *)X1, part, noskip, (const int *)skip,
                       pk, RProd{});
    reduce(skip);
    // second factorisation (G2 of the rounded Q1): within kSkipTau of I it keeps
    // R = R1 and sets *skip; otherwise R = R2 R1 by one more workgroup of the
    // final sweep
    hipLaunchKernelGGL(gram_chol_kernel<W>, dim3(1), dim3(CT), 0, s, cpart, cparts, w, R2, X2,
                       (const double *)R1, R, ldr, skip, kSkipTau, 0, (const int *)skip,
                       (int *)nullptr, 0.0);
    const RProd rp{R2, R1, R, ldr};
    hipLaunchKernelGGL((gram_pass_kernel<W, true, false>), dim3(sp.parts + 1), dim3(GT), 0, s, P,
                       ld, m, w, sp.chunks_per, (const double *)X2, (double *)nullptr,
                       (const int *)skip, noskip, pk, rp);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// 128-column panels: one Cholesky QR over a whole 128-column leaf of the
// recursion, its halves A | B (64 columns each) kept as blocks.
//   G = [A B]^T [A B] in one sweep; R_AA = chol(G_AA), R_AB = R_AA^{-T} G_AB,
//   R_BB = chol(G_BB - R_AB^T R_AB); X = R^{-1} has X_AA = R_AA^{-1},
//   X_BB = R_BB^{-1}, X_AB = -X_AA R_AB X_BB; Q = [A B] X in one more sweep.
// This is Cholesky QR of the 128 columns (the same R as two 64-column panels
// with the B half projected onto and updated by Q_A in between, in exact
// arithmetic), with one Gram matrix and one elimination chain per sweep pair
// instead of two, and no separate projection and update for the B half.
// Sweeps: 8 waves per workgroup on 64-row chunks. LDS: the chunk as two FP64
// halves, and for Q formation X_AB (full) and X_AA, X_BB in one array: X_AA
// above the diagonal shifted one column right, X_BB transposed on and below
// the diagonal (reads outside a triangle are masked to zero).
// ---------------------------------------------------------------------------
namespace leaf {
constexpr int W = 128, H = 64, NT = 512, LD = 66;
constexpr int NP = W * (W + 1) / 2;   // 8256 Gram entries
constexpr int LPT = CH * W / NT;      // chunk elements per thread
constexpr int NPAIR = 36;             // upper 16 x 16 block pairs of a 128 x 128 Gram
constexpr int MAXP = 5;               // pairs per wave: p = wave + 8 q
constexpr int CD = CH * LD;           // doubles of one LDS block

// block pair p (0 <= p < 36) of the upper triangle: (I, J), I <= J, by columns
QRX_DEV void pair(int p, int &I, int &J) {
    int j = 0;
    while ((j + 1) * (j + 2) / 2 <= p) ++j;
    J = j;
    I = p - j * (j + 1) / 2;
}

// X (W x W, FP64, column-major, zero below the diagonal) into the LDS blocks
QRX_DEV void load_x(const double *__restrict__ X, double *XT, double *XAB, int t) {
#pragma unroll 2
    for (int idx = t; idx < H * H; idx += NT) {
        const int k = idx % H, j = idx / H;
        const double aa = X[k + j * W], ab = X[k + (H + j) * W], bb = X[(H + k) + (H + j) * W];
        XAB[k * LD + j] = ab;
        if (k <= j) {
            XT[k * LD + j + 1] = aa;
            XT[j * LD + k] = bb;
        }
    }
}

// One sweep over row chunks [ch0, ch1) of P (m x w, 64 < w <= 128). DO_Q: rows
// <- fl32(rows X) (X in XT, XAB), written back to P and, when pk.prec is set,
// to the 16-bit operand copies. DO_G: acc += this wave's Gram blocks of the
// (rounded) rows. The next chunk is prefetched into registers.
template <bool DO_Q, bool DO_G>
QRX_DEV void sweep(float *__restrict__ P, int64_t ld, int64_t m, int w, int64_t ch0, int64_t ch1,
                   const double *XT, const double *XAB, double *CA, double *CB,
                   d4 (&acc)[MAXP], int t, const PanelPack &pk) {
    const int lane = t & 63;
    const int wv = __builtin_amdgcn_readfirstlane(t >> 6);
    const int li = lane & 15, lk = lane >> 4;
    int PI[MAXP], PJ[MAXP];   // this wave's Gram block pairs
#pragma unroll
    for (int qq = 0; qq < MAXP; ++qq) pair(wv + 8 * qq < NPAIR ? wv + 8 * qq : 0, PI[qq], PJ[qq]);
    float pre[LPT];
    // element s of this thread: row e % CH, column e / CH = wave + 8 s (A half for s < 8)
    auto load = [&](int64_t ch) {
#pragma unroll
        for (int s = 0; s < LPT; ++s) {
            const int e = t + NT * s;
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
            const int e = t + NT * s;
            const int rr = e % CH, cc = e / CH;
            if (s < LPT / 2) CA[rr * LD + cc] = (double)pre[s];
            else CB[rr * LD + cc - H] = (double)pre[s];
        }
        __syncthreads();
        if (ch + 1 < ch1) load(ch + 1);
        if constexpr (DO_Q) {
            // rows 16 Rb .. 16 Rb + 15; part 0: Q_A (4 column blocks) and Q_B block 3,
            // part 1: Q_B blocks 0..2 (72 MFMAs each)
            const int Rb = wv & 3, part = wv >> 2;
            const double *rowA = CA + (16 * Rb + li) * LD, *rowB = CB + (16 * Rb + li) * LD;
            d4 q[4];
#pragma unroll
            for (int b = 0; b < 4; ++b) q[b] = d4{0.0, 0.0, 0.0, 0.0};
            if (part == 0) {
#pragma unroll
                for (int Jb = 0; Jb < 4; ++Jb) {
                    const int j = 16 * Jb + li;
#pragma unroll 2
                    for (int k4 = 0; k4 < 4 * Jb; ++k4)
                        q[Jb] = mfma64(rowA[4 * k4 + lk], XT[(4 * k4 + lk) * LD + j + 1], q[Jb]);
#pragma unroll
                    for (int k4 = 4 * Jb; k4 < 4 * Jb + 4; ++k4) {
                        const int k = 4 * k4 + lk;
                        q[Jb] = mfma64(rowA[k], k <= j ? XT[k * LD + j + 1] : 0.0, q[Jb]);
                    }
                }
            } else {
#pragma unroll
                for (int Jb = 0; Jb < 3; ++Jb) {
                    const int j = 16 * Jb + li;
#pragma unroll 2
                    for (int k4 = 0; k4 < 16; ++k4)
                        q[Jb] = mfma64(rowA[4 * k4 + lk], XAB[(4 * k4 + lk) * LD + j], q[Jb]);
#pragma unroll 2
                    for (int k4 = 0; k4 < 4 * Jb; ++k4)
                        q[Jb] = mfma64(rowB[4 * k4 + lk], XT[j * LD + 4 * k4 + lk], q[Jb]);
#pragma unroll
                    for (int k4 = 4 * Jb; k4 < 4 * Jb + 4; ++k4) {
                        const int k = 4 * k4 + lk;
                        q[Jb] = mfma64(rowB[k], k <= j ? XT[j * LD + k] : 0.0, q[Jb]);
                    }
                }
            }
            d4 qb3 = d4{0.0, 0.0, 0.0, 0.0};
            if (part == 0) {
                const int j = 48 + li;
#pragma unroll 2
                for (int k4 = 0; k4 < 16; ++k4)
                    qb3 = mfma64(rowA[4 * k4 + lk], XAB[(4 * k4 + lk) * LD + j], qb3);
#pragma unroll 2
                for (int k4 = 0; k4 < 16; ++k4) {
                    const int k = 4 * k4 + lk;   // k <= 63 < j + 1 except on the diagonal block
                    qb3 = mfma64(rowB[k], k <= j ? XT[j * LD + k] : 0.0, qb3);
                }
            }
            __syncthreads();   // every wave has read its rows of the chunk
            double *outq = part == 0 ? CA : CB;
#pragma unroll
            for (int Jb = 0; Jb < 4; ++Jb) {
                if (part == 1 && Jb == 3) break;
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    outq[(16 * Rb + 4 * v + lk) * LD + 16 * Jb + li] = (double)(float)q[Jb][v];
            }
            if (part == 0) {
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    CB[(16 * Rb + 4 * v + lk) * LD + 48 + li] = (double)(float)qb3[v];
            }
            __syncthreads();
            // Q rows back to P, coalesced along the columns
#pragma unroll
            for (int s = 0; s < LPT; ++s) {
                const int e = t + NT * s;
                const int rr = e % CH, cc = e / CH;
                const int64_t r = ch * CH + rr;
                const double v = (s < LPT / 2) ? CA[rr * LD + cc] : CB[rr * LD + cc - H];
                if (r < m && cc < w) P[r + cc * ld] = (float)v;
            }
            if (pk.prec) {
#pragma unroll 1
                for (int s = 0; s < LPT; ++s) {
                    const int e = t + NT * s;
                    const int rr = e % CH, cc = e / CH;
                    const int64_t r = ch * CH + rr;
                    const double v = (s < LPT / 2) ? CA[rr * LD + cc] : CB[rr * LD + cc - H];
                    if (r < m && cc < w)
                        store16(pk.qc, pk.qcl, r + cc * pk.ldc, (float)v * pk.sc, pk.prec);
                }
#pragma unroll 1
                for (int s = 0; s < LPT; ++s) {
                    const int e = t + NT * s;
                    const int cc = e % W, rr = e / W;
                    const int64_t r = ch * CH + rr;
                    const double v = cc < H ? CA[rr * LD + cc] : CB[rr * LD + cc - H];
                    if (r < m && cc < w)
                        store16(pk.qr, pk.qrl, r * pk.ldq + cc, (float)v * pk.sc, pk.prec);
                }
            }
        }
        if constexpr (DO_G) {
#pragma unroll 2
            for (int k4 = 0; k4 < CH / 4; ++k4) {
                const double *ra = CA + (4 * k4 + lk) * LD + li;
                const double *rb = CB + (4 * k4 + lk) * LD + li;
#pragma unroll
                for (int qq = 0; qq < MAXP; ++qq) {
                    if (wv + 8 * qq >= NPAIR) break;
                    const int I = PI[qq], J = PJ[qq];
                    const double a = I < 4 ? ra[16 * I] : rb[16 * (I - 4)];
                    const double b = J < 4 ? ra[16 * J] : rb[16 * (J - 4)];
                    acc[qq] = mfma64(a, b, acc[qq]);
                }
            }
        }
    }
}

// this wave's Gram blocks into out[upk(i, j)], i <= j
QRX_DEV void gram_store(const d4 (&acc)[MAXP], double *out, int t) {
    const int lane = t & 63;
    const int wv = __builtin_amdgcn_readfirstlane(t >> 6);
#pragma unroll
    for (int qq = 0; qq < MAXP; ++qq) {
        const int p = wv + 8 * qq;
        if (p >= NPAIR) break;
        int I, J;
        pair(p, I, J);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int i = 16 * I + 4 * v + (lane >> 4), j = 16 * J + (lane & 15);
            if (i <= j) out[upk(i, j)] = acc[qq][v];
        }
    }
}

// R = Ra Rb (both W x W upper triangular, FP64, column-major) into Rfinal
// (FP32, ldr, w x w), through LDS in two 64-deep slabs: A = Ra[:, kb..kb+63]
// (column-major, ld W), B = Rb[kb..kb+63, :] (column-major, ld H).
QRX_DEV void r_product(const RProd &rp, int w, double *L, int t) {
    double *A = L, *B = L + W * H;
    const int i0 = 4 * (t % 32), j0 = 8 * (t / 32);
    double v[4][8];
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 8; ++q) v[p][q] = 0.0;
    for (int kb = 0; kb < W; kb += H) {
        __syncthreads();
        for (int idx = t; idx < W * H; idx += NT) {
            A[idx] = rp.Ra[(idx % W) + (int64_t)(kb + idx / W) * W];
            B[idx] = rp.Rb[(kb + idx % H) + (int64_t)(idx / H) * W];
        }
        __syncthreads();
        const int lo = i0 > kb ? i0 : kb;
        const int hi = (j0 + 7 < kb + H - 1) ? j0 + 7 : kb + H - 1;
        for (int l = lo; l <= hi; ++l) {
            double a[4], b[8];
#pragma unroll
            for (int p = 0; p < 4; ++p) a[p] = A[(i0 + p) + (l - kb) * W];
#pragma unroll
            for (int q = 0; q < 8; ++q) b[q] = B[(l - kb) + (j0 + q) * H];
#pragma unroll
            for (int p = 0; p < 4; ++p)
#pragma unroll
                for (int q = 0; q < 8; ++q) v[p][q] = fma(a[p], b[q], v[p][q]);
        }
    }
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int i = i0 + p, j = j0 + q;
            if (i < w && j < w) rp.Rfinal[i + (int64_t)j * rp.ldr] = (float)v[p][q];
        }
}
}  // namespace leaf

// One sweep of a 128-column panel over this workgroup's chunks (as
// gram_pass_kernel); the final sweep may carry the R product in one extra
// workgroup, the last.
template <bool DO_Q, bool DO_G>
__global__ __launch_bounds__(leaf::NT, DO_Q ? 2 : 4) void gram_leaf_pass_kernel(
    float *__restrict__ P, int64_t ld, int64_t m, int w, int64_t chunks_per,
    const double *__restrict__ X, double *__restrict__ part, const int *__restrict__ skip,
    PanelPack pk, RProd rp) {
    using namespace leaf;
    if (skip && *skip) return;   // the first sweep already gave an orthonormal Q
    __shared__ __align__(16) double L[(DO_Q ? 4 : 2) * CD];
    double *CA = L, *CB = L + CD, *XT = L + 2 * CD, *XAB = L + 3 * CD;
    const int t = threadIdx.x;
    if constexpr (DO_Q && !DO_G) {
        static_assert(4 * CD >= 2 * W * H, "R product staging");
        if (rp.Rfinal && blockIdx.x == gridDim.x - 1) {
            r_product(rp, w, L, t);
            return;
        }
    }
    const int64_t nch = (m + CH - 1) / CH;
    const int64_t ch0 = (int64_t)blockIdx.x * chunks_per;
    const int64_t ch1 = (ch0 + chunks_per < nch) ? ch0 + chunks_per : nch;
    if constexpr (DO_Q) load_x(X, XT, XAB, t);
    d4 acc[MAXP];
#pragma unroll
    for (int qq = 0; qq < MAXP; ++qq) acc[qq] = d4{0.0, 0.0, 0.0, 0.0};
    sweep<DO_Q, DO_G>(P, ld, m, w, ch0, ch1, XT, XAB, CA, CB, acc, t, pk);
    if constexpr (DO_G) gram_store(acc, part + (int64_t)blockIdx.x * NP, t);
}

// One workgroup: G (128 x 128, the sum of nparts partials in partial order),
// then the blocked factorisation and inverse described above, writing R and X
// (FP64, 128 x 128, column-major, zero below the diagonal) and, if Rfinal is
// set and Rprev is null, the panel's R block (FP32, ldr). With skip set the
// orthogonality check of gram_chol_kernel runs first: on success R = Rprev
// goes to Rfinal; otherwise the product R Rprev is left to the final sweep.
__global__ __launch_bounds__(CT) void gram_chol_leaf_kernel(const double *__restrict__ part,
                                                            int nparts, int w,
                                                            double *__restrict__ Rout,
                                                            double *__restrict__ Xout,
                                                            const double *__restrict__ Rprev,
                                                            float *__restrict__ Rfinal,
                                                            int64_t ldr, int *__restrict__ skip,
                                                            double tau) {
    using leaf::H;
    using leaf::NP;
    using leaf::W;
    constexpr int LS = H + 1;
    constexpr int NW = CT / 64;
    constexpr int NQ = (NP + CT - 1) / CT;   // packed entries per thread
    constexpr int PB = 2;
    __shared__ double S[H * LS];     // G_AA -> R_AA, then X_BB
    __shared__ double Xs[H * LS];    // X_AA
    __shared__ double GAB[H * LS];   // G_AB -> R_AB
    __shared__ double GBB[H * LS];   // G_BB -> S_BB -> R_BB, then R_AB X_BB
    __shared__ __align__(16) double Ub[gram::kCholT64];
    const int t = threadIdx.x;
    const int lane = t & 63, wv = t >> 6;
    const bool rfin = Rfinal && !Rprev;   // R block written here (single pass)
    double gv[NQ];
    int ii[NQ], jj[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const int e = t + q * CT;
        int j = (int)((sqrt(8.0 * e + 1.0) - 1.0) * 0.5);
        while (j * (j + 1) / 2 > e) --j;
        while ((j + 1) * (j + 2) / 2 <= e) ++j;
        jj[q] = j;
        ii[q] = e - j * (j + 1) / 2;
        gv[q] = 0.0;
    }
    {
        int p = 0;
        for (; p + PB <= nparts; p += PB) {
            double v[PB][NQ];
#pragma unroll
            for (int b = 0; b < PB; ++b)
#pragma unroll
                for (int q = 0; q < NQ; ++q) {
                    const int e = t + q * CT;
                    v[b][q] = e < NP ? part[(int64_t)(p + b) * NP + e] : 0.0;
                }
#pragma unroll
            for (int b = 0; b < PB; ++b)
#pragma unroll
                for (int q = 0; q < NQ; ++q) gv[q] += v[b][q];
        }
        for (; p < nparts; ++p)
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                const int e = t + q * CT;
                if (e < NP) gv[q] += part[(int64_t)p * NP + e];
            }
    }
    double dev = 0.0;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const int e = t + q * CT;
        if (e >= NP) continue;
        const int i = ii[q], j = jj[q];
        if (j < H) S[i + j * LS] = gv[q];
        else if (i < H) GAB[i + (j - H) * LS] = gv[q];
        else GBB[(i - H) + (j - H) * LS] = gv[q];
        if (j < w) {
            const double e2 = fabs(gv[q] - (i == j ? 1.0 : 0.0));
            dev = fmax(dev, (e2 == e2) ? e2 : 1e300);   // a NaN entry never passes
        }
    }
    if (skip) {
#pragma unroll
        for (int o2 = 32; o2 > 0; o2 >>= 1) dev = fmax(dev, __shfl_xor(dev, o2));
        if (lane == 0) Ub[wv] = dev;
        __syncthreads();
        double mx = 0.0;
#pragma unroll
        for (int q = 0; q < NW; ++q) mx = fmax(mx, Ub[q]);
        const bool done = mx <= tau;   // NaN compares false: factorise
        if (t == 0) *skip = done ? 1 : 0;
        if (done) {
            for (int idx = t; idx < W * W; idx += CT) {
                const int i = idx % W, j = idx / W;
                if (i < w && j < w) Rfinal[i + (int64_t)j * ldr] = (float)Rprev[idx];
            }
            return;
        }
    }
    __syncthreads();
    // R_AA, X_AA
    gram::chol_inv<H, CT>(S, Xs, Ub, t);
    for (int idx = t; idx < H * H; idx += CT) {
        const int i = idx % H, j = idx / H;
        const bool up = i <= j;
        const double r = up ? S[i + j * LS] : 0.0;
        Rout[i + j * W] = r;
        Xout[i + j * W] = up ? Xs[i + j * LS] : 0.0;
        Rout[(H + i) + j * W] = 0.0;
        Xout[(H + i) + j * W] = 0.0;
        if (rfin) {
            if (i < w && j < w) Rfinal[i + (int64_t)j * ldr] = (float)r;
            if (H + i < w && j < w) Rfinal[(H + i) + (int64_t)j * ldr] = 0.0f;
        }
    }
    // 2 x 4 tiles of a 64 x 64 block per thread
    const int i0 = 2 * (t % 32), j0 = 4 * (t / 32);
    double v[2][4];
    auto zero = [&] {
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
            for (int q = 0; q < 4; ++q) v[p][q] = 0.0;
    };
    // R_AB = X_AA^T G_AB (X_AA[k][i] = 0 for k > i)
    zero();
    for (int k = 0; k <= i0 + 1; ++k) {
        const double a0 = Xs[k + i0 * LS], a1 = Xs[k + (i0 + 1) * LS];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const double b = GAB[k + (j0 + q) * LS];
            v[0][q] = fma(a0, b, v[0][q]);
            v[1][q] = fma(a1, b, v[1][q]);
        }
    }
    __syncthreads();   // every read of G_AB is done
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int i = i0 + p, j = j0 + q;
            GAB[i + j * LS] = v[p][q];
            Rout[i + (H + j) * W] = v[p][q];
            if (rfin && i < w && H + j < w) Rfinal[i + (int64_t)(H + j) * ldr] = (float)v[p][q];
        }
    __syncthreads();
    // S_BB = G_BB - R_AB^T R_AB (upper part; each thread its own entries)
    zero();
    for (int k = 0; k < H; ++k) {
        const double a0 = GAB[k + i0 * LS], a1 = GAB[k + (i0 + 1) * LS];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const double b = GAB[k + (j0 + q) * LS];
            v[0][q] = fma(a0, b, v[0][q]);
            v[1][q] = fma(a1, b, v[1][q]);
        }
    }
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int i = i0 + p, j = j0 + q;
            if (i <= j) GBB[i + j * LS] -= v[p][q];
        }
    __syncthreads();
    // R_BB (in GBB), X_BB (in S: R_AA is already out)
    gram::chol_inv<H, CT>(GBB, S, Ub, t);
    for (int idx = t; idx < H * H; idx += CT) {
        const int i = idx % H, j = idx / H;
        const bool up = i <= j;
        const double r = up ? GBB[i + j * LS] : 0.0;
        Rout[(H + i) + (H + j) * W] = r;
        Xout[(H + i) + (H + j) * W] = up ? S[i + j * LS] : 0.0;
        if (rfin && H + i < w && H + j < w) Rfinal[(H + i) + (int64_t)(H + j) * ldr] = (float)r;
    }
    // Y = R_AB X_BB (X_BB[k][j] = 0 for k > j)
    zero();
    for (int k = 0; k <= j0 + 3; ++k) {
        const double a0 = GAB[i0 + k * LS], a1 = GAB[(i0 + 1) + k * LS];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const double b = S[k + (j0 + q) * LS];
            v[0][q] = fma(a0, b, v[0][q]);
            v[1][q] = fma(a1, b, v[1][q]);
        }
    }
    __syncthreads();   // every read of R_BB is done
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q) GBB[(i0 + p) + (j0 + q) * LS] = v[p][q];
    __syncthreads();
    // X_AB = -X_AA Y (X_AA[i][k] = 0 for k < i)
    zero();
    for (int k = i0; k < H; ++k) {
        const double a0 = Xs[i0 + k * LS], a1 = Xs[(i0 + 1) + k * LS];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const double b = GBB[k + (j0 + q) * LS];
            v[0][q] = fma(a0, b, v[0][q]);
            v[1][q] = fma(a1, b, v[1][q]);
        }
    }
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q) Xout[(i0 + p) + (H + j0 + q) * W] = -v[p][q];
}

static hipError_t leaf_go(hipStream_t s, float *P, int64_t ld, int64_t m, int w, float *R,
                          int64_t ldr, double *ws, int reorth, const PanelPack &pk) {
    using leaf::NP;
    using leaf::NT;
    using leaf::W;
    const GramSplit sp = leaf_split(m);
    double *part = ws + kGramCounterInts / 2;
    double *R1 = part + (size_t)sp.parts * NP;
    double *X1 = R1 + W * W;
    double *R2 = X1 + W * W;
    double *X2 = R2 + W * W;
    double *lvl = X2 + W * W;
    int *skip = gram_counter(ws) + 1;
    const unsigned cb = (unsigned)((NP + 63) / 64);
    const int ns = gram_slices(sp.parts);
    const double *cpart = ns ? lvl : part;
    const int cparts = ns ? ns : sp.parts;
    auto reduce = [&] {
        if (ns)
            hipLaunchKernelGGL(gram_reduce_kernel<W>, dim3(cb, ns), dim3(CT), 0, s,
                               (const double *)part, sp.parts, lvl, (const int *)nullptr);
    };
    PanelPack none = pk;
    none.prec = 0;
    const int *noskip = nullptr;
    hipLaunchKernelGGL((gram_leaf_pass_kernel<false, true>), dim3(sp.parts), dim3(NT), 0, s, P, ld,
                       m, w, sp.chunks_per, (const double *)nullptr, part, noskip, none, RProd{});
    reduce();
    hipLaunchKernelGGL(gram_chol_leaf_kernel, dim3(1), dim3(CT), 0, s, cpart, cparts, w, R1, X1,
                       (const double *)nullptr, reorth ? (float *)nullptr : R, ldr,
                       (int *)nullptr, 0.0);
    if (!reorth) {
        hipLaunchKernelGGL((gram_leaf_pass_kernel<true, false>), dim3(sp.parts), dim3(NT), 0, s,
                           P, ld, m, w, sp.chunks_per, (const double *)X1, (double *)nullptr,
                           noskip, pk, RProd{});
        return hipGetLastError();
    }
    hipLaunchKernelGGL((gram_leaf_pass_kernel<true, true>), dim3(sp.parts), dim3(NT), 0, s, P, ld,
                       m, w, sp.chunks_per, (const double *)X1, part, noskip, pk, RProd{});
    reduce();
    hipLaunchKernelGGL(gram_chol_leaf_kernel, dim3(1), dim3(CT), 0, s, cpart, cparts, w, R2, X2,
                       (const double *)R1, R, ldr, skip, kSkipTau);
    // R = R2 R1 by one more workgroup of the final sweep
    const RProd rp{R2, R1, R, ldr};
    hipLaunchKernelGGL((gram_leaf_pass_kernel<true, false>), dim3(sp.parts + 1), dim3(NT), 0, s,
                       P, ld, m, w, sp.chunks_per, (const double *)X2, (double *)nullptr,
                       (const int *)skip, pk, rp);
    return hipGetLastError();
}

bool gram_panel_packs(int w) { return w > 32; }

hipError_t launch_gram_panel(hipStream_t s, float *P, int64_t ld, int64_t m, int w, float *R,
                             int64_t ldr, double *ws, int reorth, const PanelPack &pack) {
    if (w <= 16) return gram_go<16>(s, P, ld, m, w, R, ldr, ws, reorth, pack);
    if (w <= 32) return gram_go<32>(s, P, ld, m, w, R, ldr, ws, reorth, pack);
    if (w <= 64) return gram_go<64>(s, P, ld, m, w, R, ldr, ws, reorth, pack);
    if (w <= 128) return leaf_go(s, P, ld, m, w, R, ldr, ws, reorth, pack);
    return hipErrorInvalidValue;
}

}  // namespace qrx
