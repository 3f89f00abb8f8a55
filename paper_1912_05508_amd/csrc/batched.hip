// Batched least squares: many small problems, one workgroup per problem.
//
// Each problem runs the same method as the single-problem path (Alg. 2 with
// Cholesky-QR-twice panels, then the R-preconditioned LSQR of Sec. 3.2.3 with
// FP64 vectors and a double-double residual certification), but entirely
// inside one workgroup: the problems are small (n <= 256), so a workgroup
// streams its own matrix from HBM/L2 while 2 workgroups per CU keep the chip
// busy. Problems are launched longest-first (one workgroup each, grid = batch),
// so the hardware dispatcher balances the uneven sizes.
//
// bqr_kernel   scan (||A||_F, max column norm, finite check, working copy),
//              the recursion over a per-n schedule: 32-column panels by the
//              Gram sweeps of gram_common.hpp, nodes by in-workgroup MFMA
//              projection / update (FP32, or BF16 above the cutoff), then R
//              finalisation (strictly-lower part zeroed, diagonal checked).
// blsqr_kernel LSQR on A R^{-1}: triangular solves in 64-row blocks, each
//              diagonal block solved by one wave from registers (row or column
//              of R per lane, values passed by cross-lane shuffles), the rest
//              applied by all waves; GEMVs with FP64 accumulation; the
//              iteration is certified with b - A x in double-double and
//              restarted on the certified residual when needed.
#include "gemm_common.hpp"
#include "gram_common.hpp"
#include "batched.hpp"

namespace qrx {

constexpr int BT = 256;   // threads per workgroup
static_assert(BT == GT && BT == gram::GT, "one workgroup shape for every phase");

// LDS of the QR kernel (doubles): the panel phase needs the most.
constexpr int kPanelLds = gram::Lds<32>::C_DOUBLES + gram::Lds<32>::X_DOUBLES +
                          gram::Lds<32>::RED_DOUBLES + 528 + 2 * 32 * 33 + 256 + 32 * 32;
constexpr int kGemmLds = 2 * 128 * (64 + 8) * 2 / 8;   // two 128 x (BK+PAD) 16-bit tiles
static_assert(2 * 128 * (32 + 4) * 4 / 8 <= kGemmLds, "FP32 tiles fit");
constexpr int kBqrLds = kPanelLds > kGemmLds ? kPanelLds : kGemmLds;
// the LSQR phase reuses the same LDS: 8 n-vectors and a 64 x 65 FP32 block
static_assert(8 * 256 + (64 * 65 + 1) / 2 <= kBqrLds, "LSQR vectors fit the QR's LDS");

QRX_DEV bool al16(const void *p) { return (((uintptr_t)p) & 15) == 0; }

// Second panel sweep skipped when Q1^T Q1 is within this of I in every entry.
constexpr double kBSkipTau = 1.0 / (1 << 21);

// A value every lane holds alike, made uniform for the compiler: branches on it
// are then scalar branches. Loops and branches that contain barriers must be
// uniform in this sense, or the compiler may restructure them per lane.
QRX_DEV int uniform_i(int v) { return __builtin_amdgcn_readfirstlane(v); }
// The same for a trivially copyable value of whole 32-bit words (a descriptor
// loaded from device memory at a uniform address arrives in vector registers).
template <class T>
QRX_DEV T uniform_v(const T &v) {
    static_assert(sizeof(T) % 4 == 0, "whole words");
    constexpr int W = sizeof(T) / 4;
    unsigned w[W];
    __builtin_memcpy(w, &v, sizeof(T));
#pragma unroll
    for (int i = 0; i < W; ++i) w[i] = __builtin_amdgcn_readfirstlane(w[i]);
    T out;
    __builtin_memcpy(&out, w, sizeof(T));
    return out;
}
QRX_DEV double uniform_d(double v) {
    const unsigned long long b = __double_as_longlong(v);
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)(b & 0xffffffffu));
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(b >> 32));
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Sum over the workgroup (fixed order); every thread gets the result.
QRX_DEV double bsum(double v, double *sh) {
    v = wave_sum_d(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    return uniform_d((sh[0] + sh[1]) + (sh[2] + sh[3]));
}
QRX_DEV double bmax(double v, double *sh) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    return uniform_d(fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3])));
}

// ---------------------------------------------------------------------------
// In-workgroup trailing products (same tiles as the single-problem kernels).
// ---------------------------------------------------------------------------
// R12 (k x n2, ldr) = Q1^T A2 over K = m rows, TILE x TILE output tiles (4 waves
// of TILE/2 x TILE/2).
template <class Tr, int TILE>
QRX_DEV void wg_project(int64_t m, int k, int n2, const float *Q1, const float *A2, int64_t ld,
                        float *R12, int64_t ldr, typename Tr::E *As, typename Tr::E *Bs, int t) {
    using E = typename Tr::E;
    constexpr int BK = Tr::BK, LS = BK + Tr::PAD, FM = TILE / 32, FN = TILE / 32, WT = TILE / 2;
    const int lane = t & 63, wv = t >> 6, wm = wv % 2, wn = wv / 2;
    const bool vec = al16(Q1) && al16(A2) && (ld % 4 == 0);
    auto one = [](int64_t) { return 1.0f; };
    for (int i0 = 0; i0 < k; i0 += TILE)
        for (int j0 = 0; j0 < n2; j0 += TILE) {
            f32x4 acc[FM][FN];
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int j = 0; j < FN; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
            KLoader<BK, TILE> la, lb;
            la.load(Q1, ld, 0, m, i0, k, vec, t);
            lb.load(A2, ld, 0, m, j0, n2, vec, t);
            for (int64_t k0 = 0; k0 < m; k0 += BK) {
                __syncthreads();
                la.template store<E, LS>(As, i0, t, one);
                lb.template store<E, LS>(Bs, j0, t, one);
                __syncthreads();
                if (k0 + BK < m) {
                    la.load(Q1, ld, k0 + BK, m, i0, k, vec, t);
                    lb.load(A2, ld, k0 + BK, m, j0, n2, vec, t);
                }
                mma_stage<Tr, FM, FN>(As, Bs, wm * WT, wn * WT, acc, lane);
            }
#pragma unroll
            for (int fm = 0; fm < FM; ++fm)
#pragma unroll
                for (int fn = 0; fn < FN; ++fn) {
                    const int j = j0 + wn * WT + fn * 16 + (lane & 15);
                    const int ib = i0 + wm * WT + fm * 16 + 4 * (lane >> 4);
                    if (j < n2) {
#pragma unroll
                        for (int v = 0; v < 4; ++v)
                            if (ib + v < k) R12[(ib + v) + (int64_t)j * ldr] = acc[fm][fn][v];
                    }
                }
        }
    __syncthreads();
}

// A2 (m x n2) -= Q1 (m x k) R12 (k x n2), TILE-row x TILE-column tiles.
template <class Tr, int TILE>
QRX_DEV void wg_update(int64_t m, int k, int n2, const float *Q1, float *A2, int64_t ld,
                       const float *R12, int64_t ldr, typename Tr::E *As, typename Tr::E *Bs,
                       int t) {
    using E = typename Tr::E;
    constexpr int BK = Tr::BK, LS = BK + Tr::PAD, FM = TILE / 32, FN = TILE / 32, WT = TILE / 2;
    const int lane = t & 63, wv = t >> 6, wm = wv % 2, wn = wv / 2;
    const bool vecq = al16(Q1) && (ld % 4 == 0);
    const bool vecr = al16(R12) && (ldr % 4 == 0);
    const bool veca = al16(A2) && (ld % 4 == 0);
    auto one = [](int64_t) { return 1.0f; };
    for (int j0 = 0; j0 < n2; j0 += TILE)
        for (int64_t r0 = 0; r0 < m; r0 += TILE) {
            f32x4 acc[FM][FN];
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int j = 0; j < FN; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
            MLoader<BK, TILE> la;
            KLoader<BK, TILE> lb;
            la.load(Q1, ld, r0, m, 0, k, vecq, t);
            lb.load(R12, ldr, 0, k, j0, n2, vecr, t);
            for (int k0 = 0; k0 < k; k0 += BK) {
                __syncthreads();
                la.template store<E, LS>(As, t, 1.0f);
                lb.template store<E, LS>(Bs, j0, t, one);
                __syncthreads();
                if (k0 + BK < k) {
                    la.load(Q1, ld, r0, m, k0 + BK, k, vecq, t);
                    lb.load(R12, ldr, k0 + BK, k, j0, n2, vecr, t);
                }
                mma_stage<Tr, FM, FN>(As, Bs, wm * WT, wn * WT, acc, lane);
            }
#pragma unroll
            for (int fn = 0; fn < FN; ++fn) {
                const int j = j0 + wn * WT + fn * 16 + (lane & 15);
                if (j >= n2) continue;
#pragma unroll
                for (int fm = 0; fm < FM; ++fm) {
                    const int64_t rb = r0 + wm * WT + fm * 16 + 4 * (lane >> 4);
                    float *dst = A2 + (int64_t)j * ld + rb;
                    if (veca && rb + 3 < m) {
                        float4 x = *reinterpret_cast<float4 *>(dst);
                        x.x -= acc[fm][fn][0];
                        x.y -= acc[fm][fn][1];
                        x.z -= acc[fm][fn][2];
                        x.w -= acc[fm][fn][3];
                        *reinterpret_cast<float4 *>(dst) = x;
                    } else {
#pragma unroll
                        for (int v = 0; v < 4; ++v)
                            if (rb + v < m) dst[v] -= acc[fm][fn][v];
                    }
                }
            }
        }
    __syncthreads();
}

// Second pass of the in-workgroup panel skipped when the bound of kappa_2 of the
// column-equilibrated first factor is at most this (as in the single-problem
// panel: one Cholesky-QR pass with an FP64 Gram matrix then leaves Q at the
// FP32 rounding level).
constexpr double kBCondTau = 16384.0;

// The square of sqrt(||R D^-1||_1 ||R D^-1||_inf ||D X||_1 ||D X||_inf) >=
// kappa_2(R D^-1), D the column norms of R: R (upper triangular) in S and
// X = R^{-1} in Xc, column-major with stride 33, w <= 32 columns. Eight threads
// share a column (or row), four entries each. T: 36 doubles of scratch. The
// result is uniform.
QRX_DEV double equil_kappa2_32(const double *S, const double *Xc, int w, double *T, int t) {
    const int c = t >> 3, sub = t & 7;
    double a = 0.0;
    if (c < w) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int k = 4 * sub + e;
            const double v = k <= c ? S[k + c * 33] : 0.0;
            a = fma(v, v, a);
        }
    }
    a += __shfl_xor(a, 1);
    a += __shfl_xor(a, 2);
    a += __shfl_xor(a, 4);
    double *dn = T + 4;                           // T[0..3]: bmax scratch
    __syncthreads();
    if (c < w && sub == 0) dn[c] = sqrt(a);
    __syncthreads();
    double nr[4];
#pragma unroll
    for (int nm = 0; nm < 4; ++nm) {
        const bool isx = nm & 1, cols = nm < 2;
        const double *M = isx ? Xc : S;
        double s = 0.0;
        if (c < w) {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int k = 4 * sub + e;
                const bool in = cols ? (k <= c) : (k >= c && k < w);
                const int i = cols ? k : c, j = cols ? c : k;
                const double v = in ? fabs(M[i + j * 33]) : 0.0;
                s += in ? (isx ? v * dn[i] : v / dn[j]) : 0.0;
            }
        }
        s += __shfl_xor(s, 1);
        s += __shfl_xor(s, 2);
        s += __shfl_xor(s, 4);
        nr[nm] = bmax(s, T);
    }
    return (nr[0] * nr[2]) * (nr[1] * nr[3]);
}

// ---------------------------------------------------------------------------
// In-workgroup panel: Cholesky QR with FP64 Gram matrices (w <= 32), a second
// pass when the first factor is not well conditioned enough.
// ---------------------------------------------------------------------------
QRX_DEV void wg_panel(float *P, int64_t ld, int64_t m, int w, float *Rb, int64_t ldr, double *lds,
                      int t) {
    using L = gram::Lds<32>;
    double *C = lds;
    double *Xs = C + L::C_DOUBLES;          // X row-major for the sweeps
    double *red = Xs + L::X_DOUBLES;
    double *Gl = red + L::RED_DOUBLES;
    double *S = Gl + 528;                   // G, then R (column-major, stride 33)
    double *Xc = S + 32 * 33;               // R^{-1} (column-major, stride 33)
    double *T = Xc + 32 * 33;               // pivot rows of the elimination (and scratch)
    double *R1 = T + 256;                   // first-sweep R
    const int64_t nch = (m + gram::CH - 1) / gram::CH;
    gram::gd4 acc[3];
    auto zero = [&]() {
#pragma unroll
        for (int x = 0; x < 3; ++x) acc[x] = gram::gd4{0.0, 0.0, 0.0, 0.0};
    };
    auto factor = [&]() {   // Gl -> S -> R, Xc; X into the sweep layout
        for (int idx = t; idx < 32 * 32; idx += BT) {
            const int i = idx % 32, j = idx / 32;
            S[i + j * 33] = (i <= j && j < w) ? Gl[gram::upk(i, j)] : 0.0;
        }
        __syncthreads();
        gram::chol_inv<32, BT>(S, Xc, T, t);
        for (int idx = t; idx < 32 * 32; idx += BT) {
            const int i = idx % 32, j = idx / 32;
            Xs[i * L::XLD + j] = (i <= j && j < w) ? Xc[i + j * 33] : 0.0;
        }
    };
    zero();
    gram::sweep32<false, true>(P, ld, m, w, 0, nch, Xs, C, acc, t);
    gram::gram_store32(acc, red, Gl, t);
    __syncthreads();
    factor();
    for (int idx = t; idx < 32 * 32; idx += BT) {
        const int i = idx % 32, j = idx / 32;
        R1[idx] = (i <= j && j < w) ? S[i + j * 33] : 0.0;
    }
    // one pass suffices: R = R1, Q = fl32(P X1)
    const double est2 = equil_kappa2_32(S, Xc, w, T, t);
    if (est2 <= kBCondTau * kBCondTau) {   // NaN compares false: second pass
        for (int idx = t; idx < 32 * 32; idx += BT) {
            const int i = idx % 32, j = idx / 32;
            if (i < w && j < w) Rb[i + (int64_t)j * ldr] = (float)R1[idx];
        }
        gram::sweep32<true, false>(P, ld, m, w, 0, nch, Xs, C, acc, t);
        __syncthreads();
        return;
    }
    zero();
    gram::sweep32<true, true>(P, ld, m, w, 0, nch, Xs, C, acc, t);
    gram::gram_store32(acc, red, Gl, t);
    __syncthreads();
    // Q1 already orthonormal to working accuracy: R = R1, no second factorisation
    double dev = 0.0;
    for (int idx = t; idx < 528; idx += BT) {
        int j = 0;
        while ((j + 1) * (j + 2) / 2 <= idx) ++j;
        const int i = idx - j * (j + 1) / 2;
        if (j < w) {
            const double e2 = fabs(Gl[idx] - (i == j ? 1.0 : 0.0));
            dev = fmax(dev, (e2 == e2) ? e2 : 1e300);
        }
    }
    if (bmax(dev, T) <= kBSkipTau) {
        for (int idx = t; idx < 32 * 32; idx += BT) {
            const int i = idx % 32, j = idx / 32;
            if (i < w && j < w) Rb[i + (int64_t)j * ldr] = (float)R1[idx];
        }
        __syncthreads();
        return;
    }
    factor();
    // R = R2 R1 into the diagonal block (R2 in S, both upper triangular)
    for (int idx = t; idx < 32 * 32; idx += BT) {
        const int i = idx % 32, j = idx / 32;
        if (i < w && j < w) {
            double v = 0.0;
            for (int l = i; l <= j; ++l) v = fma(S[i + l * 33], R1[l + j * 32], v);
            Rb[i + (int64_t)j * ldr] = (float)v;
        }
    }
    gram::sweep32<true, false>(P, ld, m, w, 0, nch, Xs, C, acc, t);
    __syncthreads();
}

// ---------------------------------------------------------------------------
// One problem's QR in one workgroup: scan (||A||_F, largest column norm, finite
// check, working copy), the recursion over its schedule, R finalisation.
// ---------------------------------------------------------------------------

struct BProb {
    int64_t m, n, lda, ldw, ldr;
    const float *A;   // the problem matrix (read by the scan and by the Krylov products)
    float *W;         // working copy, Q on exit (== A for an in-place QR)
    float *R;         // n x n upper triangle, ldr
    const double *b;  // right-hand side (least squares)
    double *x;        // solution (least squares)
    double *u, *q;    // FP64 m-vectors (least squares)
    int op0, nops, tiles;
};

template <class Tr>
QRX_DEV BRes wg_qr(const BProb &p, const BOp *ops, int copy, double *lds, double *sh, int t_in) {
    const int t = t_in;
    const int lane = t & 63, wv = t >> 6;
    const int64_t m = p.m;
    const int n = (int)p.n;
    double ss_tot = 0.0, ss_max = 0.0;
    int bad = 0;
    for (int j = wv; j < n; j += BT / 64) {
        double s = 0.0;
        const float *a = p.A + (int64_t)j * p.lda;
        float *wcol = p.W + (int64_t)j * p.ldw;
        // four rows of the lane at a time (their loads in flight together)
        int64_t r = lane;
        for (; r + 3 * 64 < m; r += 4 * 64) {
            float v[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) v[k] = a[r + 64 * k];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                if (!(fabsf(v[k]) <= 3.4028235e38f)) bad = 1;
                s = fma((double)v[k], (double)v[k], s);
                if (copy) wcol[r + 64 * k] = v[k];
            }
        }
        for (; r < m; r += 64) {
            const float v = a[r];
            if (!(fabsf(v) <= 3.4028235e38f)) bad = 1;
            s = fma((double)v, (double)v, s);
            if (copy) wcol[r] = v;
        }
        s = wave_sum_d(s);
        ss_tot += s;
        ss_max = fmax(ss_max, s);
    }
    ss_tot = bsum(lane == 0 ? ss_tot : 0.0, sh);
    ss_max = bmax(ss_max, sh);
    bad = bsum(bad ? 1.0 : 0.0, sh) > 0.0;
    __syncthreads();

    if (!bad) {
        using E = typename Tr::E;
        for (int o = p.op0; o < p.op0 + p.nops; ++o) {
            const BOp op = uniform_v(ops[o]);
            float *Wc = p.W + (int64_t)op.c0 * p.ldw;
            // the lane index behind an empty asm statement: what the step derives
            // from it is computed here, not hoisted out of the loops over steps and
            // problems (where it would stay live across them and be spilled)
            int t = t_in;
            asm volatile("" : "+v"(t));
            if (op.kind == 0) {
                wg_panel(Wc, p.ldw, m, op.k, p.R + op.c0 + (int64_t)op.c0 * p.ldr, p.ldr, lds, t);
            } else {
                float *A2 = p.W + (int64_t)(op.c0 + op.k) * p.ldw;
                float *R12 = p.R + op.c0 + (int64_t)(op.c0 + op.k) * p.ldr;
                if (op.lowp) {
                    E *As = reinterpret_cast<E *>(lds);
                    E *Bs = As + 128 * (Tr::BK + Tr::PAD);
                    bool small = false;
                    if constexpr (Tr::BK == 64) {   // 64 x 64 tiles: 16-bit operands only
                        if (p.tiles == 1) {
                            small = true;
                            wg_project<Tr, 64>(m, op.k, op.n2, Wc, A2, p.ldw, R12, p.ldr, As, Bs, t);
                            wg_update<Tr, 64>(m, op.k, op.n2, Wc, A2, p.ldw, R12, p.ldr, As, Bs, t);
                        }
                    }
                    if (!small) {
                        wg_project<Tr, 128>(m, op.k, op.n2, Wc, A2, p.ldw, R12, p.ldr, As, Bs, t);
                        wg_update<Tr, 128>(m, op.k, op.n2, Wc, A2, p.ldw, R12, p.ldr, As, Bs, t);
                    }
                } else {
                    float *As = reinterpret_cast<float *>(lds);
                    float *Bs = As + 128 * (PF32::BK + PF32::PAD);
                    wg_project<PF32, 128>(m, op.k, op.n2, Wc, A2, p.ldw, R12, p.ldr, As, Bs, t);
                    wg_update<PF32, 128>(m, op.k, op.n2, Wc, A2, p.ldw, R12, p.ldr, As, Bs, t);
                }
            }
        }
    }
    // R finalisation: zero the strictly-lower part, check the diagonal
    int sing = 0;
    for (int idx = t; idx < n * n; idx += BT) {
        const int i = idx % n, j = idx / n;
        float *rij = p.R + i + (int64_t)j * p.ldr;
        if (i > j || bad) *rij = 0.0f;
        if (i == j && !bad) {
            const float d = *rij;
            if (!(d > 0.0f) || !(d <= 3.4028235e38f)) sing = 1;
        }
    }
    sing = bsum(sing ? 1.0 : 0.0, sh) > 0.0;
    __syncthreads();
    BRes r;
    r.status = bad ? QRX_ENONFINITE : (sing ? QRX_ESINGULAR : QRX_OK);
    r.normA = sqrt(ss_tot);
    r.rho = sqrt(ss_max);
    return r;
}

// ---------------------------------------------------------------------------
// LSQR kernel
// ---------------------------------------------------------------------------
struct BVec {   // n-vectors in LDS (kBMaxN each)
    double *x, *xb, *v, *t, *d, *z, *y, *xs;
};

// The loops over A and R below load in groups (KB entries of A, or four
// row steps) before they accumulate, so that a group's loads are in flight
// together; the sums keep their sequential order.
constexpr int KB = 16;

// out = R^{-1} in (trans 0) or R^{-T} in (trans 1); R FP32 upper (n x n, ldr),
// arithmetic in FP64. y is scratch, Rb holds a 64 x 65 block (LDS). Blocks of
// 64 rows: the diagonal block is staged in LDS and solved by wave 0 (one row
// per lane, solved values passed by cross-lane shuffles); all waves then apply
// the solved block to the remaining rows.
QRX_DEV void wg_trsv(const float *R, int64_t ldr, int n, const double *in, double *y, double *out,
                     float *Rb, int trans, int t) {
    const int lane = t & 63, wv = t >> 6;
    const int nblk = (n + 63) / 64;
    for (int i = t; i < kBMaxN; i += BT) y[i] = (i < n) ? in[i] : 0.0;
    for (int q = 0; q < nblk; ++q) {
        const int J = trans ? q : nblk - 1 - q;
        const int o = J * 64;
        const int bw = (n - o < 64) ? n - o : 64;
        // Rb[i * 65 + c] = block entry the lane i uses at step c:
        // R[o+i][o+c] (trans 0) or R[o+c][o+i] (trans 1)
        __syncthreads();
        {
            constexpr int NL = 64 * 64 / BT;
            float v[NL];
#pragma unroll
            for (int s2 = 0; s2 < NL; ++s2) {
                const int idx = t + s2 * BT, r = idx % 64, c = idx / 64;   // R[o+r][o+c], coalesced along r
                v[s2] = (r < bw && c < bw) ? R[(o + r) + (int64_t)(o + c) * ldr] : 0.0f;
            }
#pragma unroll
            for (int s2 = 0; s2 < NL; ++s2) {
                const int idx = t + s2 * BT, r = idx % 64, c = idx / 64;
                if (trans) Rb[c * 65 + r] = v[s2]; else Rb[r * 65 + c] = v[s2];
            }
        }
        __syncthreads();
        if (wv == 0) {
            const bool in_b = lane < bw;
            const float dgl = in_b ? Rb[lane * 65 + lane] : 1.0f;
            const double dinv = (dgl != 0.0f) ? 1.0 / (double)dgl : 0.0;
            double yi = y[o + lane];
            double xi = 0.0;
            for (int st = 0; st < bw; ++st) {
                const int c = trans ? st : bw - 1 - st;
                const double xc = __shfl(yi * dinv, c);
                if (lane == c) xi = xc;
                const bool upd = trans ? (lane > c) : (lane < c);
                if (upd) yi = fma(-(double)Rb[lane * 65 + c], xc, yi);
            }
            out[o + lane] = in_b ? xi : 0.0;
        }
        __syncthreads();
        if (!trans) {
            for (int r = t; r < o; r += BT) {
                double acc = 0.0;
                int c = 0;
                for (; c + KB <= bw; c += KB) {
                    float a[KB];
#pragma unroll
                    for (int k = 0; k < KB; ++k) a[k] = R[r + (int64_t)(o + c + k) * ldr];
#pragma unroll
                    for (int k = 0; k < KB; ++k) acc = fma((double)a[k], out[o + c + k], acc);
                }
                for (; c < bw; ++c) acc = fma((double)R[r + (int64_t)(o + c) * ldr], out[o + c], acc);
                y[r] -= acc;
            }
        } else {
            for (int j = o + 64 + t; j < n; j += BT) {
                double acc = 0.0;
                int c = 0;
                for (; c + KB <= bw; c += KB) {
                    float a[KB];
#pragma unroll
                    for (int k = 0; k < KB; ++k) a[k] = R[(o + c + k) + (int64_t)j * ldr];
#pragma unroll
                    for (int k = 0; k < KB; ++k) acc = fma((double)a[k], out[o + c + k], acc);
                }
                for (; c < bw; ++c) acc = fma((double)R[(o + c) + (int64_t)j * ldr], out[o + c], acc);
                y[j] -= acc;
            }
        }
    }
    __syncthreads();
    for (int i = n + t; i < kBMaxN; i += BT) out[i] = 0.0;
    __syncthreads();
}

// f(r) for the rows r = t, t + BT, ... of [0, m), four at a time: f is called
// as f(r, v) after the four loads v = src[r] of a group are issued together.
template <class F>
QRX_DEV void rows4(int64_t m, const double *src, int t, F f) {
    int64_t r = t;
    for (; r + 3 * BT < m; r += 4 * BT) {
        double v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) v[k] = src[r + k * BT];
#pragma unroll
        for (int k = 0; k < 4; ++k) f(r + k * BT, v[k]);
    }
    for (; r < m; r += BT) f(r, src[r]);
}

// u <- A t - alpha u (alpha = 0: u <- A t); returns ||u||^2. t in LDS. A
// thread takes two of its rows at a time (r and r + BT).
QRX_DEV double wg_gemv_n(const BProb &p, const double *tv, double alpha, double *u, double *sh,
                         int t) {
    double ss = 0.0;
    const int n = (int)p.n;
    auto finish = [&](int64_t r, double acc) {
        const double v = (alpha != 0.0) ? acc - alpha * u[r] : acc;
        u[r] = v;
        ss = fma(v, v, ss);
    };
    for (int64_t r = t; r < p.m; r += 2 * BT) {
        const int64_t r2 = r + BT;
        const bool two = r2 < p.m;
        const float *ar = p.A + r;
        const float *ar2 = p.A + (two ? r2 : r);
        double acc = 0.0, acc2 = 0.0;
        int j = 0;
        for (; j + KB <= n; j += KB) {
            float a[KB], b[KB];
#pragma unroll
            for (int k = 0; k < KB; ++k) {
                a[k] = ar[(int64_t)(j + k) * p.lda];
                b[k] = ar2[(int64_t)(j + k) * p.lda];
            }
#pragma unroll
            for (int k = 0; k < KB; ++k) {
                acc = fma((double)a[k], tv[j + k], acc);
                acc2 = fma((double)b[k], tv[j + k], acc2);
            }
        }
        for (; j < n; ++j) {
            acc = fma((double)ar[(int64_t)j * p.lda], tv[j], acc);
            acc2 = fma((double)ar2[(int64_t)j * p.lda], tv[j], acc2);
        }
        finish(r, acc);
        if (two) finish(r2, acc2);
    }
    return bsum(ss, sh);
}

// z <- A^T u (one wave per column, fixed reduction order); z in LDS. A wave
// takes two columns at a time (j and j + 4), sharing the loads of u.
QRX_DEV void wg_gemv_t(const BProb &p, const double *u, double *z, int t) {
    const int lane = t & 63, wv = t >> 6;
    constexpr int NWV = BT / 64;
    for (int j = wv; j < (int)p.n; j += 2 * NWV) {
        const int j2 = j + NWV;
        const bool two = j2 < (int)p.n;
        const float *a = p.A + (int64_t)j * p.lda;
        const float *a2 = p.A + (int64_t)(two ? j2 : j) * p.lda;
        double acc = 0.0, acc2 = 0.0;
        int64_t r = lane;
        for (; r + 7 * 64 < p.m; r += 8 * 64) {
            float av[8], bv[8];
            double uv[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                av[k] = a[r + 64 * k];
                bv[k] = a2[r + 64 * k];
                uv[k] = u[r + 64 * k];
            }
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                acc = fma((double)av[k], uv[k], acc);
                acc2 = fma((double)bv[k], uv[k], acc2);
            }
        }
        for (; r < p.m; r += 64) {
            const double uu = u[r];
            acc = fma((double)a[r], uu, acc);
            acc2 = fma((double)a2[r], uu, acc2);
        }
        acc = wave_sum_d(acc);
        acc2 = wave_sum_d(acc2);
        if (lane == 0) {
            z[j] = acc;
            if (two) z[j2] = acc2;
        }
    }
    __syncthreads();
}

// Certification of x: q = b - A x (double-double), z = A^T q; returns the score
// min(eta_F, cscale ||r|| / (||A||_F ||x|| + ||b||)) (see compat_scale) and sets
// eta, rnorm.
QRX_DEV double wg_certify(const BProb &p, const double *x, double *z, double *q, double normA,
                          double bnorm, double &eta, double &rnorm, double *sh, int t,
                          double tol) {
    double ss = 0.0;
    const int n = (int)p.n;
    // two of the thread's rows at a time (r and r + BT)
    for (int64_t r = t; r < p.m; r += 2 * BT) {
        const int64_t r2 = r + BT;
        const bool two = r2 < p.m;
        double h = p.b[r], l = 0.0;
        double h2 = two ? p.b[r2] : 0.0, l2 = 0.0;
        const float *ar = p.A + r;
        const float *ar2 = p.A + (two ? r2 : r);
        int j = 0;
        for (; j + KB <= n; j += KB) {
            float a[KB], b[KB];
#pragma unroll
            for (int k = 0; k < KB; ++k) {
                a[k] = ar[(int64_t)(j + k) * p.lda];
                b[k] = ar2[(int64_t)(j + k) * p.lda];
            }
#pragma unroll
            for (int k = 0; k < KB; ++k) {
                dd_add_prod(h, l, -(double)a[k], x[j + k]);
                dd_add_prod(h2, l2, -(double)b[k], x[j + k]);
            }
        }
        for (; j < n; ++j) {
            dd_add_prod(h, l, -(double)ar[(int64_t)j * p.lda], x[j]);
            dd_add_prod(h2, l2, -(double)ar2[(int64_t)j * p.lda], x[j]);
        }
        const double v = h + l;
        q[r] = v;
        ss = fma(v, v, ss);
        if (two) {
            const double v2 = h2 + l2;
            q[r2] = v2;
            ss = fma(v2, v2, ss);
        }
    }
    rnorm = sqrt(bsum(ss, sh));
    wg_gemv_t(p, q, z, t);
    double zz = 0.0, xx = 0.0;
    for (int j = t; j < (int)p.n; j += BT) {
        zz = fma(z[j], z[j], zz);
        xx = fma(x[j], x[j], xx);
    }
    zz = bsum(zz, sh);
    xx = bsum(xx, sh);
    eta = (rnorm > 0.0 && normA > 0.0) ? sqrt(zz) / (normA * rnorm) : 0.0;
    const double den = normA * sqrt(xx) + bnorm;
    const double s1 = den > 0.0 ? compat_scale(p.m, p.n, tol) * (rnorm / den) : 0.0;
    return fmin(eta, s1);
}

// One problem's R-preconditioned LSQR (Sec. 3.2.3) in one workgroup, from x = 0,
// certified with a double-double residual and restarted on it; writes x and *info.
QRX_DEV void wg_lsqr(const BProb &p, const BRes &qr, double tol, int max_iter, qrx_lls_info *info,
                     double *lds, double *sh, int t_in) {
    // the lane index is re-read through an empty asm statement in each outer and
    // inner iteration, so that what the steps derive from it is computed there
    // and not kept live (and spilled) across the whole solve
    int t = t_in;
    double *vecs = lds;   // 8 n-vectors, then the 64 x 65 block of the triangular solves
    float *Rb = reinterpret_cast<float *>(lds + 8 * kBMaxN);
    const int n = (int)p.n;
    BVec V;
    V.x = vecs;
    V.xb = vecs + kBMaxN;
    V.v = vecs + 2 * kBMaxN;
    V.t = vecs + 3 * kBMaxN;
    V.d = vecs + 4 * kBMaxN;
    V.z = vecs + 5 * kBMaxN;
    V.y = vecs + 6 * kBMaxN;
    V.xs = vecs + 7 * kBMaxN;
    for (int i = t; i < 8 * kBMaxN; i += BT) vecs[i] = 0.0;
    __syncthreads();
    if (qr.status != QRX_OK) {
        for (int j = t; j < n; j += BT) p.x[j] = 0.0;
        if (t == 0) {
            memset(info, 0, sizeof(*info));
            info->status = qr.status;
            info->normA_F = qr.normA;
        }
        __syncthreads();
        return;
    }
    const double normA = qr.normA;
    // the LSQR estimate bounds ||(A R^{-1})^T r|| / ||r||; the scaled test compares
    // it with the eta_F target through the largest column norm
    const double trig = normA > 0.0 ? qr.rho / normA : 1.0;
    double bb = 0.0;
    rows4(p.m, p.b, t, [&](int64_t, double v) { bb = fma(v, v, bb); });
    const double bnorm = sqrt(bsum(bb, sh));
    double gamma = 1.0, best = 1e300, eta = 0.0, rnorm = 0.0, best_eta = 0.0, best_rn = 0.0;
    double first_eta = 0.0;
    int iters = 0, restarts = 0, stall = 0, status = QRX_ENOCONV;
    for (int outer = 0;; ++outer) {
        t = t_in;
        asm volatile("" : "+v"(t));
        // certify the current x; q = residual, z = A^T q
        const double score = wg_certify(p, V.x, V.z, p.q, normA, bnorm, eta, rnorm, sh, t, tol);
        if (outer == 0) first_eta = eta;
        if (score < best) {
            if (score < 0.5 * best) stall = 0; else ++stall;
            best = score;
            best_eta = eta;
            best_rn = rnorm;
            for (int j = t; j < kBMaxN; j += BT) V.xb[j] = V.x[j];
        } else {
            ++stall;
        }
        __syncthreads();
        if (best <= tol) {
            status = QRX_OK;
            break;
        }
        if (iters >= max_iter || stall >= 3 || rnorm == 0.0) break;
        if (outer > 0) {
            ++restarts;
            gamma = fmax(0.5 * gamma, 0.01);
        }
        // LSQR on the correction: min || A R^{-1} y - q ||, x += R^{-1} y
        double beta = rnorm;
        rows4(p.m, p.q, t, [&](int64_t r, double v) { p.u[r] = v / beta; });
        for (int j = t; j < kBMaxN; j += BT) V.z[j] = V.z[j] / beta;   // A^T u
        __syncthreads();
        wg_trsv(p.R, p.ldr, n, V.z, V.y, V.v, Rb, 1, t);                     // v = R^{-T} A^T u
        double aa = 0.0;
        for (int j = t; j < kBMaxN; j += BT) aa = fma(V.v[j], V.v[j], aa);
        double alpha = sqrt(bsum(aa, sh));
        if (alpha == 0.0) break;
        for (int j = t; j < kBMaxN; j += BT) V.v[j] /= alpha;
        __syncthreads();
        wg_trsv(p.R, p.ldr, n, V.v, V.y, V.t, Rb, 0, t);                     // t = R^{-1} v
        for (int j = t; j < kBMaxN; j += BT) V.d[j] = V.t[j];
        __syncthreads();
        double phibar = beta, rhobar = alpha;
        const int every = 50;
        for (int it = 0; it < every && iters < max_iter; ++it) {
            t = t_in;
            asm volatile("" : "+v"(t));
            ++iters;
            const double b2 = wg_gemv_n(p, V.t, alpha, p.u, sh, t);   // u = A t - alpha u
            beta = sqrt(b2);
            if (beta > 0.0)
                rows4(p.m, p.u, t, [&](int64_t r, double v) { p.u[r] = v / beta; });
            __syncthreads();
            wg_gemv_t(p, p.u, V.z, t);                                   // z = A^T u
            wg_trsv(p.R, p.ldr, n, V.z, V.y, V.xs, Rb, 1, t);                // xs = R^{-T} z
            aa = 0.0;
            for (int j = t; j < kBMaxN; j += BT) {
                const double vj = V.xs[j] - beta * V.v[j];
                V.v[j] = vj;
                aa = fma(vj, vj, aa);
            }
            alpha = sqrt(bsum(aa, sh));
            if (alpha > 0.0)
                for (int j = t; j < kBMaxN; j += BT) V.v[j] /= alpha;
            const double rho = hypot(rhobar, beta);
            const double c = rhobar / rho, s = beta / rho;
            const double theta = s * alpha;
            rhobar = -c * alpha;
            const double phi = c * phibar;
            phibar = s * phibar;
            for (int j = t; j < kBMaxN; j += BT) V.x[j] = fma(phi / rho, V.d[j], V.x[j]);
            __syncthreads();
            wg_trsv(p.R, p.ldr, n, V.v, V.y, V.t, Rb, 0, t);                 // t = R^{-1} v
            for (int j = t; j < kBMaxN; j += BT) V.d[j] = V.t[j] - (theta / rho) * V.d[j];
            __syncthreads();
            const double est = alpha * fabs(c) * trig;
            if (est <= tol * gamma || alpha == 0.0 || beta == 0.0) break;
        }
    }
    for (int j = t; j < n; j += BT) p.x[j] = V.xb[j];
    if (t == 0) {
        info->status = status;
        info->iters = iters;
        info->restarts = restarts;
        info->accepted = status == QRX_OK ? (best_eta <= tol ? 1 : 2) : 0;
        info->eta_F = best_eta;
        info->resid_norm = best_rn;
        info->normA_F = normA;
        info->eta_start = first_eta;
        info->score = best;
    }
    __syncthreads();
}


// ---------------------------------------------------------------------------
// The persistent batched kernels: each workgroup takes the next problem from an
// atomic queue over the longest-first order until the queue is empty. The QR
// kernel factors it; for least squares a second kernel, with its own queue,
// runs LSQR on each factored problem. Both kernels hold two workgroups per CU.
// ---------------------------------------------------------------------------
// The next queue index for this workgroup (uniform: every lane gets it in a
// scalar register; read back through LDS it would count as divergent, and the
// loop around it holds barriers).
QRX_DEV int queue_next(unsigned *counter, int *s_idx, int t) {
    if (t == 0) *s_idx = (int)atomicAdd(counter, 1u);
    __syncthreads();
    const int idx = uniform_i(*s_idx);
    __syncthreads();
    return idx;
}

// Problem `pi` as the batched calls describe it (uniform values); false for a
// bad descriptor.
QRX_DEV bool load_problem(const BArgs &a, int pi, BProb &p) {
    const BEntry e = uniform_v(a.ent[pi]);
    p.m = e.m;
    p.n = e.n;
    p.A = uniform_v(a.A[pi]);
    p.lda = uniform_v(a.lda[pi]);
    p.op0 = e.op0;
    p.nops = e.nops;
    p.tiles = e.tiles;
    bool ok = p.A != nullptr && p.lda >= p.m;
    if (a.lls) {
        p.b = uniform_v(a.b[pi]);
        p.x = uniform_v(a.x[pi]);
        p.W = reinterpret_cast<float *>(a.work + e.w_off);
        p.ldw = e.ldw;
        p.R = reinterpret_cast<float *>(a.work + e.r_off);
        p.ldr = e.n;
        p.u = reinterpret_cast<double *>(a.work + e.v_off);
        p.q = p.u + e.m;
        ok = ok && p.b != nullptr && p.x != nullptr;
    } else {
        p.W = const_cast<float *>(p.A);
        p.ldw = p.lda;
        p.R = uniform_v(a.R[pi]);
        p.ldr = uniform_v(a.ldr[pi]);
        p.b = nullptr;
        p.x = nullptr;
        p.u = p.q = nullptr;
        ok = ok && p.R != nullptr && p.ldr >= p.n;
    }
    return ok;
}

// Phase 1 of a batch: every problem's QR, taken off the first work queue in the
// longest-first order. For least squares the factorisation's results go to the
// per-problem records of phase 2; a bad descriptor is reported here. Its
// registers are bounded for two workgroups per CU: a second workgroup hides
// the latency of the first's loads (4096 mixed problems: 38.5 -> 31.1 ms),
// which outweighs the registers it then spills (about 56 per lane).
template <class Tr>
__global__ __launch_bounds__(BT, 2) void bqr_queue_kernel(BArgs a) {
    __shared__ __align__(16) double lds[kBqrLds];
    __shared__ double sh[4];
    __shared__ int s_idx;
    const int t = threadIdx.x;
    // one loop, one back edge, no early exits: each pass takes one problem
    for (int idx = queue_next(a.counter, &s_idx, t); idx < a.batch;
         idx = queue_next(a.counter, &s_idx, t)) {
        const int pi = uniform_i(a.order[idx]);
        BProb p;
        const bool ok = load_problem(a, pi, p);
        if (ok) {
            const BRes r = wg_qr<Tr>(p, a.ops, a.lls, lds, sh, t);
            if (t == 0) {
                if (a.lls)
                    a.res[pi] = r;
                else
                    a.status[pi] = r.status;
            }
        } else if (t == 0) {
            if (a.lls) {
                memset(a.info + pi, 0, sizeof(qrx_lls_info));
                a.info[pi].status = QRX_EINVAL;
                a.res[pi].status = QRX_EINVAL;
            } else {
                a.status[pi] = QRX_EINVAL;
            }
        }
    }
}

// Phase 2 (least squares): every problem's LSQR, off the second work queue.
__global__ __launch_bounds__(BT) void blsqr_queue_kernel(BArgs a) {
    __shared__ __align__(16) double lds[8 * kBMaxN + (64 * 65 + 1) / 2];
    __shared__ double sh[4];
    __shared__ int s_idx;
    const int t = threadIdx.x;
    for (int idx = queue_next(a.counter + 1, &s_idx, t); idx < a.batch;
         idx = queue_next(a.counter + 1, &s_idx, t)) {
        const int pi = uniform_i(a.order[idx]);
        BProb p;
        if (load_problem(a, pi, p)) {
            const BRes r = uniform_v(a.res[pi]);
            wg_lsqr(p, r, a.tol, a.max_iter, a.info + pi, lds, sh, t);
        }
    }
}

// ---------------------------------------------------------------------------
// Workgroups of a persistent queue launch: what fits on the device at once,
// and no more than there are problems.
static int queue_grid(const void *kernel, int device, int batch) {
    int cus = 0, per = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess ||
        cus < 1)
        cus = 1;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, BT, 0) != hipSuccess || per < 1)
        per = 1;
    const int64_t g = (int64_t)per * cus;
    return (int)(batch < g ? batch : g);
}

hipError_t launch_bsolve(hipStream_t s, int device, int prec, const BArgs &a) {
    const void *qk = prec == QRX_BF16 ? (const void *)bqr_queue_kernel<PBF16>
                                      : (const void *)bqr_queue_kernel<PF32>;
    if (prec != QRX_FP32 && prec != QRX_BF16) return hipErrorInvalidValue;
    const int gq = queue_grid(qk, device, a.batch);
    if (prec == QRX_BF16)
        hipLaunchKernelGGL(bqr_queue_kernel<PBF16>, dim3((unsigned)gq), dim3(BT), 0, s, a);
    else
        hipLaunchKernelGGL(bqr_queue_kernel<PF32>, dim3((unsigned)gq), dim3(BT), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !a.lls) return e;
    const int gl = queue_grid((const void *)blsqr_queue_kernel, device, a.batch);
    hipLaunchKernelGGL(blsqr_queue_kernel, dim3((unsigned)gl), dim3(BT), 0, s, a);
    return hipGetLastError();
}

}  // namespace qrx
