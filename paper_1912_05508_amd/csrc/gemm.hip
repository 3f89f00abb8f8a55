// Trailing products of the recursive Gram-Schmidt QR (Alg. 2):
//   projection  R12 = Q1^T A2      (M = k, N = n2, K = m)
//   update      A2 <- A2 - Q1 R12  (M = m, N = n2, K = k)
// on the matrix cores (MFMA 16x16) with FP32 accumulation; operands are
// converted from the FP32 masters to FP16 / BF16 (round to nearest even) or
// kept in FP32 while they are staged into LDS (Sec. 3.1.2: the products are
// what the low-precision unit accelerates).
//
// Low-precision operand scaling: Q1 columns (max-abs <= 1) are multiplied by
// 2^14, each A2 column by the power of two that puts its max-abs in
// [2^13, 2^14), each R12 column likewise before the update; the epilogues
// divide the exact powers of two back out. This keeps small trailing columns
// out of the FP16 subnormal range.
//
// The projection splits K = m over grid.y (split-K) and writes FP32 partial
// products; a second kernel sums them in a fixed order (deterministic), writes
// R12 into R, derives the update scales and clears the column max-abs of A2.
// The update's epilogue subtracts in FP32 and, when a later step needs them,
// writes per-tile partial column max-abs values that a small kernel reduces
// (no atomics; deterministic).
#include "qrx_internal.hpp"

namespace qrx {

constexpr int GT = 256;  // threads per workgroup (4 waves)

struct PF32 {
    using E = float;
    static constexpr int KS = 4;    // K per MFMA
    static constexpr int BK = 32;   // K per LDS stage
    static constexpr int PAD = 4;
    static constexpr bool SPLIT = false;
};
struct PF16 {
    using E = _Float16;
    static constexpr int KS = 32;
    static constexpr int BK = 64;
    static constexpr int PAD = 8;
    static constexpr bool SPLIT = false;
};
struct PBF16 {
    using E = __bf16;
    static constexpr int KS = 32;
    static constexpr int BK = 64;
    static constexpr int PAD = 8;
    static constexpr bool SPLIT = false;
};
// Split FP16: x = hi + 2^-11 lo with hi = fl16(x), lo = fl16((x - hi) 2^11);
// x y ~ hi_x hi_y + 2^-11 (hi_x lo_y + lo_x hi_y), three FP16 MFMAs per step.
struct PF16X3 {
    using E = _Float16;
    static constexpr int KS = 32;
    static constexpr int BK = 64;
    static constexpr int PAD = 8;
    static constexpr bool SPLIT = true;
};
constexpr float kSplitLo = 2048.0f;          // 2^11
constexpr float kSplitLoInv = 1.0f / 2048.0f;

typedef _Float16 f16x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));

QRX_DEV void st4(float *d, float a, float b, float c, float e) {
    *reinterpret_cast<float4 *>(d) = make_float4(a, b, c, e);
}
QRX_DEV void st4(_Float16 *d, float a, float b, float c, float e) {
    f16x4 v = {(_Float16)a, (_Float16)b, (_Float16)c, (_Float16)e};
    *reinterpret_cast<f16x4 *>(d) = v;
}
QRX_DEV void st4(__bf16 *d, float a, float b, float c, float e) {
    bf16x4 v = {(__bf16)a, (__bf16)b, (__bf16)c, (__bf16)e};
    *reinterpret_cast<bf16x4 *>(d) = v;
}

// hi / lo parts of four values
QRX_DEV void st4_split(_Float16 *dh, _Float16 *dl, float a, float b, float c, float e) {
    const _Float16 ha = (_Float16)a, hb = (_Float16)b, hc = (_Float16)c, he = (_Float16)e;
    f16x4 vh = {ha, hb, hc, he};
    f16x4 vl = {(_Float16)((a - (float)ha) * kSplitLo), (_Float16)((b - (float)hb) * kSplitLo),
                (_Float16)((c - (float)hc) * kSplitLo), (_Float16)((e - (float)he) * kSplitLo)};
    *reinterpret_cast<f16x4 *>(dh) = vh;
    *reinterpret_cast<f16x4 *>(dl) = vl;
}

// One K-stage of MFMA work for a wave: FM x FN fragments of 16x16.
// As: [rows][BK+PAD] (K contiguous), Bs: [cols][BK+PAD].
template <class Tr, int FM, int FN>
QRX_DEV void mma_stage(const typename Tr::E *As, const typename Tr::E *Bs, int arow0, int bcol0,
                       f32x4 (&acc)[FM][FN], int lane) {
    constexpr int LS = Tr::BK + Tr::PAD;
    const int rl = lane & 15, kq = lane >> 4;
#pragma unroll
    for (int kk = 0; kk < Tr::BK; kk += Tr::KS) {
        if constexpr (Tr::KS == 4) {
            float a[FM], b[FN];
#pragma unroll
            for (int f = 0; f < FM; ++f) a[f] = As[(arow0 + f * 16 + rl) * LS + kk + kq];
#pragma unroll
            for (int f = 0; f < FN; ++f) b[f] = Bs[(bcol0 + f * 16 + rl) * LS + kk + kq];
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int j = 0; j < FN; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
        } else {
            using V8 = typename std::conditional<std::is_same<typename Tr::E, _Float16>::value,
                                                 f16x8, bf16x8>::type;
            V8 a[FM], b[FN];
#pragma unroll
            for (int f = 0; f < FM; ++f)
                a[f] = *reinterpret_cast<const V8 *>(As + (arow0 + f * 16 + rl) * LS + kk + kq * 8);
#pragma unroll
            for (int f = 0; f < FN; ++f)
                b[f] = *reinterpret_cast<const V8 *>(Bs + (bcol0 + f * 16 + rl) * LS + kk + kq * 8);
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int j = 0; j < FN; ++j) {
                    if constexpr (std::is_same<typename Tr::E, _Float16>::value)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a[i], b[j], acc[i][j], 0, 0, 0);
                    else
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
                }
        }
    }
}

// Split-FP16 K-stage: acc += hi*hi, acc2 += hi*lo + lo*hi.
template <int FM, int FN, int BK, int LS>
QRX_DEV void mma_stage_split(const _Float16 *Ah, const _Float16 *Al, const _Float16 *Bh,
                             const _Float16 *Bl, int arow0, int bcol0, f32x4 (&acc)[FM][FN],
                             f32x4 (&acc2)[FM][FN], int lane) {
    const int rl = lane & 15, kq = lane >> 4;
#pragma unroll
    for (int kk = 0; kk < BK; kk += 32) {
        f16x8 ah[FM], al[FM], bh[FN], bl[FN];
#pragma unroll
        for (int f = 0; f < FM; ++f) {
            const int o = (arow0 + f * 16 + rl) * LS + kk + kq * 8;
            ah[f] = *reinterpret_cast<const f16x8 *>(Ah + o);
            al[f] = *reinterpret_cast<const f16x8 *>(Al + o);
        }
#pragma unroll
        for (int f = 0; f < FN; ++f) {
            const int o = (bcol0 + f * 16 + rl) * LS + kk + kq * 8;
            bh[f] = *reinterpret_cast<const f16x8 *>(Bh + o);
            bl[f] = *reinterpret_cast<const f16x8 *>(Bl + o);
        }
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j) {
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah[i], bh[j], acc[i][j], 0, 0, 0);
                acc2[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah[i], bl[j], acc2[i][j], 0, 0, 0);
                acc2[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(al[i], bh[j], acc2[i][j], 0, 0, 0);
            }
    }
}

// Load a K-contiguous operand tile: C columns x BK rows of X (X[k + c*ld]),
// k in [k0, kend), c in [c0, cend); zero outside. Each thread owns NR float4s.
template <int BK, int C>
struct KLoader {
    static constexpr int CPC = BK / 4;         // float4 per column
    static constexpr int COLS_PER_PASS = GT / CPC;
    static constexpr int NR = C / COLS_PER_PASS;
    float4 v[NR];
    QRX_DEV void load(const float *X, int64_t ld, int64_t k0, int64_t kend, int64_t c0,
                      int64_t cend, bool vec, int t) {
        const int q = t % CPC, cc = t / CPC;
#pragma unroll
        for (int p = 0; p < NR; ++p) {
            const int64_t c = c0 + cc + p * COLS_PER_PASS;
            const int64_t k = k0 + 4 * q;
            float4 r = make_float4(0.f, 0.f, 0.f, 0.f);
            if (c < cend) {
                const float *src = X + c * ld + k;
                if (vec && k + 3 < kend) {
                    r = *reinterpret_cast<const float4 *>(src);
                } else {
                    if (k < kend) r.x = src[0];
                    if (k + 1 < kend) r.y = src[1];
                    if (k + 2 < kend) r.z = src[2];
                    if (k + 3 < kend) r.w = src[3];
                }
            }
            v[p] = r;
        }
    }
    // store to LDS [col][BK+PAD], column c multiplied by scale(c)
    template <class E, int LS, class F>
    QRX_DEV void store(E *S, int64_t c0, int t, F scale) const {
        const int q = t % CPC, cc = t / CPC;
#pragma unroll
        for (int p = 0; p < NR; ++p) {
            const int cl = cc + p * COLS_PER_PASS;
            const float s = scale(c0 + cl);
            st4(S + cl * LS + 4 * q, v[p].x * s, v[p].y * s, v[p].z * s, v[p].w * s);
        }
    }
    template <int LS, class F>
    QRX_DEV void store_split(_Float16 *Sh, _Float16 *Sl, int64_t c0, int t, F scale) const {
        const int q = t % CPC, cc = t / CPC;
#pragma unroll
        for (int p = 0; p < NR; ++p) {
            const int cl = cc + p * COLS_PER_PASS;
            const float s = scale(c0 + cl);
            st4_split(Sh + cl * LS + 4 * q, Sl + cl * LS + 4 * q, v[p].x * s, v[p].y * s,
                      v[p].z * s, v[p].w * s);
        }
    }
};

// Load an M-contiguous operand tile (X[r + i*ld], r rows x BK columns i) and
// store it transposed to LDS [r][BK+PAD]; each thread moves NB4 4x4 blocks.
template <int BK, int BM>
struct MLoader {
    static constexpr int RB = BM / 4;                 // 4-row groups
    static constexpr int NBLK = RB * (BK / 4);
    static constexpr int NB4 = NBLK / GT;
    float4 v[NB4][4];
    QRX_DEV void load(const float *X, int64_t ld, int64_t r0, int64_t rend, int64_t i0,
                      int64_t iend, bool vec, int t) {
#pragma unroll
        for (int p = 0; p < NB4; ++p) {
            const int b = t + p * GT;
            const int rb = b % RB, ib = b / RB;
            const int64_t r = r0 + 4 * rb;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int64_t i = i0 + 4 * ib + c;
                float4 x = make_float4(0.f, 0.f, 0.f, 0.f);
                if (i < iend) {
                    const float *src = X + i * ld + r;
                    if (vec && r + 3 < rend) {
                        x = *reinterpret_cast<const float4 *>(src);
                    } else {
                        if (r < rend) x.x = src[0];
                        if (r + 1 < rend) x.y = src[1];
                        if (r + 2 < rend) x.z = src[2];
                        if (r + 3 < rend) x.w = src[3];
                    }
                }
                v[p][c] = x;
            }
        }
    }
    template <class E, int LS>
    QRX_DEV void store(E *S, int t, float s) const {
#pragma unroll
        for (int p = 0; p < NB4; ++p) {
            const int b = t + p * GT;
            const int rb = b % RB, ib = b / RB;
            E *d = S + (4 * rb) * LS + 4 * ib;
            st4(d + 0 * LS, v[p][0].x * s, v[p][1].x * s, v[p][2].x * s, v[p][3].x * s);
            st4(d + 1 * LS, v[p][0].y * s, v[p][1].y * s, v[p][2].y * s, v[p][3].y * s);
            st4(d + 2 * LS, v[p][0].z * s, v[p][1].z * s, v[p][2].z * s, v[p][3].z * s);
            st4(d + 3 * LS, v[p][0].w * s, v[p][1].w * s, v[p][2].w * s, v[p][3].w * s);
        }
    }
    template <int LS>
    QRX_DEV void store_split(_Float16 *Sh, _Float16 *Sl, int t, float s) const {
#pragma unroll
        for (int p = 0; p < NB4; ++p) {
            const int b = t + p * GT;
            const int rb = b % RB, ib = b / RB;
            const int o = (4 * rb) * LS + 4 * ib;
            st4_split(Sh + o + 0 * LS, Sl + o + 0 * LS, v[p][0].x * s, v[p][1].x * s, v[p][2].x * s, v[p][3].x * s);
            st4_split(Sh + o + 1 * LS, Sl + o + 1 * LS, v[p][0].y * s, v[p][1].y * s, v[p][2].y * s, v[p][3].y * s);
            st4_split(Sh + o + 2 * LS, Sl + o + 2 * LS, v[p][0].z * s, v[p][1].z * s, v[p][2].z * s, v[p][3].z * s);
            st4_split(Sh + o + 3 * LS, Sl + o + 3 * LS, v[p][0].w * s, v[p][1].w * s, v[p][2].w * s, v[p][3].w * s);
        }
    }
};

// ---------------------------------------------------------------------------
// Projection: part[s][i + j*M] = sum_{r in split s} Q1[r, i] A2[r, j] (scaled)
// ---------------------------------------------------------------------------
template <class Tr, int BM, int BN, int WM, int WN>
__global__ __launch_bounds__(GT) void projection_kernel(int64_t K, int64_t M, int64_t N,
                                                        const float *__restrict__ Q1,
                                                        const float *__restrict__ A2,
                                                        int64_t ld, const float *__restrict__ colmax,
                                                        int scaling, int64_t kchunk,
                                                        float *__restrict__ part, int vec) {
    using E = typename Tr::E;
    constexpr int BK = Tr::BK, LS = BK + Tr::PAD;
    constexpr int FM = BM / WM / 16, FN = BN / WN / 16;
    constexpr int NS = Tr::SPLIT ? 2 : 1;
    __shared__ __attribute__((aligned(16))) E As[NS * BM * LS];
    __shared__ __attribute__((aligned(16))) E Bs[NS * BN * LS];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int wm = wv % WM, wn = wv / WM;
    const int64_t tiles_m = (M + BM - 1) / BM;
    const int64_t i0 = (blockIdx.x % tiles_m) * BM;
    const int64_t j0 = (blockIdx.x / tiles_m) * BN;
    const int64_t kb = blockIdx.y * kchunk;
    const int64_t ke = (kb + kchunk < K) ? kb + kchunk : K;
    const bool lowp = Tr::KS != 4;
    const float qs = (lowp && scaling) ? 16384.0f : 1.0f;

    f32x4 acc[FM][FN];
    f32x4 acc2[Tr::SPLIT ? FM : 1][Tr::SPLIT ? FN : 1];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    if constexpr (Tr::SPLIT) {
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j) acc2[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    }

    KLoader<BK, BM> la;
    KLoader<BK, BN> lb;
    if (kb < ke) {
        la.load(Q1, ld, kb, ke, i0, M, vec, t);
        lb.load(A2, ld, kb, ke, j0, N, vec, t);
    }
    auto bscale = [&](int64_t c) {
        return (lowp && scaling && c < N) ? pow2_scale(colmax[c], 14) : 1.0f;
    };
    for (int64_t k0 = kb; k0 < ke; k0 += BK) {
        __syncthreads();
        if constexpr (Tr::SPLIT) {
            la.template store_split<LS>(As, As + BM * LS, i0, t, [&](int64_t) { return qs; });
            lb.template store_split<LS>(Bs, Bs + BN * LS, j0, t, bscale);
        } else {
            la.template store<E, LS>(As, i0, t, [&](int64_t) { return qs; });
            lb.template store<E, LS>(Bs, j0, t, bscale);
        }
        __syncthreads();
        if (k0 + BK < ke) {
            la.load(Q1, ld, k0 + BK, ke, i0, M, vec, t);
            lb.load(A2, ld, k0 + BK, ke, j0, N, vec, t);
        }
        if constexpr (Tr::SPLIT)
            mma_stage_split<FM, FN, BK, LS>(As, As + BM * LS, Bs, Bs + BN * LS, wm * (BM / WM),
                                            wn * (BN / WN), acc, acc2, lane);
        else
            mma_stage<Tr, FM, FN>(As, Bs, wm * (BM / WM), wn * (BN / WN), acc, lane);
    }
    if constexpr (Tr::SPLIT) {
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j) acc[i][j] += acc2[i][j] * kSplitLoInv;
    }
    float *P = part + (int64_t)blockIdx.y * M * N;
#pragma unroll
    for (int fm = 0; fm < FM; ++fm)
#pragma unroll
        for (int fn = 0; fn < FN; ++fn) {
            const int64_t j = j0 + wn * (BN / WN) + fn * 16 + (lane & 15);
            const int64_t ib = i0 + wm * (BM / WM) + fm * 16 + 4 * (lane >> 4);
            if (j < N) {
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    if (ib + v < M) P[(ib + v) + j * M] = acc[fm][fn][v];
            }
        }
}

// R12[i, j] = unscale_j * sum_s part[s][i + j*M]; update scale of column j;
// with Racc, also Racc += R12 (second projection of a re-orthogonalised node).
__global__ __launch_bounds__(256) void proj_reduce_kernel(int64_t M, int64_t N,
                                                          const float *__restrict__ part,
                                                          int splits, float *__restrict__ R12,
                                                          int64_t ldr, float *__restrict__ colmax,
                                                          float *__restrict__ uscale, int lowp_scaled,
                                                          float *__restrict__ Racc, int64_t ldacc) {
    const int64_t j = blockIdx.x;
    __shared__ float smax[4];
    const float unscale = lowp_scaled ? 1.0f / (16384.0f * pow2_scale(colmax[j], 14)) : 1.0f;
    float mx = 0.0f;
    for (int64_t i = threadIdx.x; i < M; i += 256) {
        float s = 0.0f;
        for (int q = 0; q < splits; ++q) s += part[(int64_t)q * M * N + i + j * M];
        s *= unscale;
        R12[i + j * ldr] = s;
        if (Racc) Racc[i + j * ldacc] += s;
        mx = fmaxf(mx, fabsf(s));
    }
    mx = wave_max_f(mx);
    if ((threadIdx.x & 63) == 0) smax[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        float m2 = fmaxf(fmaxf(smax[0], smax[1]), fmaxf(smax[2], smax[3]));
        uscale[j] = lowp_scaled ? pow2_scale(m2, 14) : 1.0f;
    }
}

// ---------------------------------------------------------------------------
// Update: A2[r, j] -= sum_i Q1[r, i] R12[i, j]; refresh colmax of A2.
// ---------------------------------------------------------------------------
template <class Tr, int BM, int BN, int WM, int WN>
__global__ __launch_bounds__(GT) void update_kernel(int64_t M, int64_t N, int64_t K,
                                                    const float *__restrict__ Q1, int64_t ldq,
                                                    float *__restrict__ A2, int64_t lda,
                                                    const float *__restrict__ R12, int64_t ldr,
                                                    const float *__restrict__ uscale,
                                                    float *__restrict__ cmpart, int scaling,
                                                    int vecq, int vecr, int veca) {
    using E = typename Tr::E;
    constexpr int BK = Tr::BK, LS = BK + Tr::PAD;
    constexpr int FM = BM / WM / 16, FN = BN / WN / 16;
    constexpr int NS = Tr::SPLIT ? 2 : 1;
    __shared__ __attribute__((aligned(16))) E As[NS * BM * LS];
    __shared__ __attribute__((aligned(16))) E Bs[NS * BN * LS];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int wm = wv % WM, wn = wv / WM;
    const int64_t tiles_m = (M + BM - 1) / BM;
    const int64_t r0 = (blockIdx.x % tiles_m) * BM;
    const int64_t j0 = (blockIdx.x / tiles_m) * BN;
    const bool lowp = Tr::KS != 4;
    const bool scaled = lowp && scaling;
    const float qs = scaled ? 16384.0f : 1.0f;

    f32x4 acc[FM][FN];
    f32x4 acc2[Tr::SPLIT ? FM : 1][Tr::SPLIT ? FN : 1];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    if constexpr (Tr::SPLIT) {
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j) acc2[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    }

    MLoader<BK, BM> la;
    KLoader<BK, BN> lb;
    la.load(Q1, ldq, r0, M, 0, K, vecq, t);
    lb.load(R12, ldr, 0, K, j0, N, vecr, t);
    auto bscale = [&](int64_t c) { return (scaled && c < N) ? uscale[c] : 1.0f; };
    for (int64_t k0 = 0; k0 < K; k0 += BK) {
        __syncthreads();
        if constexpr (Tr::SPLIT) {
            la.template store_split<LS>(As, As + BM * LS, t, qs);
            lb.template store_split<LS>(Bs, Bs + BN * LS, j0, t, bscale);
        } else {
            la.template store<E, LS>(As, t, qs);
            lb.template store<E, LS>(Bs, j0, t, bscale);
        }
        __syncthreads();
        if (k0 + BK < K) {
            la.load(Q1, ldq, r0, M, k0 + BK, K, vecq, t);
            lb.load(R12, ldr, k0 + BK, K, j0, N, vecr, t);
        }
        if constexpr (Tr::SPLIT)
            mma_stage_split<FM, FN, BK, LS>(As, As + BM * LS, Bs, Bs + BN * LS, wm * (BM / WM),
                                            wn * (BN / WN), acc, acc2, lane);
        else
            mma_stage<Tr, FM, FN>(As, Bs, wm * (BM / WM), wn * (BN / WN), acc, lane);
    }
    if constexpr (Tr::SPLIT) {
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j) acc[i][j] += acc2[i][j] * kSplitLoInv;
    }
#pragma unroll
    for (int fn = 0; fn < FN; ++fn) {
        const int64_t j = j0 + wn * (BN / WN) + fn * 16 + (lane & 15);
        const bool jin = j < N;
        const float es = (scaled && jin) ? 1.0f / (16384.0f * uscale[j]) : 1.0f;
        float cmax = 0.0f;
#pragma unroll
        for (int fm = 0; fm < FM; ++fm) {
            const int64_t rb = r0 + wm * (BM / WM) + fm * 16 + 4 * (lane >> 4);
            if (jin) {
                float *dst = A2 + j * lda + rb;
                if (veca && rb + 3 < M) {
                    float4 x = *reinterpret_cast<float4 *>(dst);
                    x.x = fmaf(-es, acc[fm][fn][0], x.x);
                    x.y = fmaf(-es, acc[fm][fn][1], x.y);
                    x.z = fmaf(-es, acc[fm][fn][2], x.z);
                    x.w = fmaf(-es, acc[fm][fn][3], x.w);
                    *reinterpret_cast<float4 *>(dst) = x;
                    cmax = fmaxf(cmax, fmaxf(fmaxf(fabsf(x.x), fabsf(x.y)), fmaxf(fabsf(x.z), fabsf(x.w))));
                } else {
#pragma unroll
                    for (int v = 0; v < 4; ++v)
                        if (rb + v < M) {
                            float y = fmaf(-es, acc[fm][fn][v], dst[v]);
                            dst[v] = y;
                            cmax = fmaxf(cmax, fabsf(y));
                        }
                }
            }
        }
        if (cmpart) {
            // per-wave partial max of the updated column; reduced by colmax_reduce
            cmax = fmaxf(cmax, __shfl_xor(cmax, 16));
            cmax = fmaxf(cmax, __shfl_xor(cmax, 32));
            const int64_t slot = (blockIdx.x % tiles_m) * WM + wm;
            if (jin && lane < 16) cmpart[slot * N + j] = cmax;
        }
    }
}

// colmax[j] = max over slots of cmpart[slot * N + j] (one wave per column).
__global__ __launch_bounds__(256) void colmax_reduce_kernel(int64_t N, int64_t slots,
                                                            const float *__restrict__ cmpart,
                                                            float *__restrict__ colmax) {
    const int lane = threadIdx.x & 63;
    const int64_t j = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (j >= N) return;
    float mx = 0.0f;
    for (int64_t q = lane; q < slots; q += 64) mx = fmaxf(mx, cmpart[q * N + j]);
    mx = wave_max_f(mx);
    if (lane == 0) colmax[j] = mx;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static bool aligned16(const void *p) { return (((uintptr_t)p) & 15) == 0; }

int projection_splits(int64_t m, int64_t k, int64_t n2) {
    const int64_t tiles = ((k + 127) / 128) * ((n2 + 127) / 128);
    int64_t want = (1024 + tiles - 1) / tiles;                 // ~4 waves of 256 workgroups
    int64_t maxs = (m + 511) / 512;                            // >= 512 rows per split
    if (want > maxs) want = maxs;
    if (want < 1) want = 1;
    if (want > 256) want = 256;
    return (int)want;
}

template <class Tr, int BM, int BN, int WM, int WN>
static hipError_t proj_go(hipStream_t s, int64_t m, int64_t k, int64_t n2, const float *Q1,
                          const float *A2, int64_t lda, const float *colmax, float *part,
                          int splits, int scaling) {
    const int64_t tiles = ((k + BM - 1) / BM) * ((n2 + BN - 1) / BN);
    int64_t kchunk = (m + splits - 1) / splits;
    kchunk = ((kchunk + Tr::BK - 1) / Tr::BK) * Tr::BK;
    const int vec = aligned16(Q1) && aligned16(A2) && (lda % 4 == 0);
    hipLaunchKernelGGL((projection_kernel<Tr, BM, BN, WM, WN>), dim3((unsigned)tiles, splits),
                       dim3(GT), 0, s, m, k, n2, Q1, A2, lda, colmax, scaling, kchunk, part, vec);
    return hipGetLastError();
}

template <class Tr>
static hipError_t proj_dispatch(hipStream_t s, int64_t m, int64_t k, int64_t n2,
                                const float *Q1, const float *A2, int64_t lda,
                                const float *colmax, float *part, int splits, int scaling) {
    if (k >= 128 && n2 >= 128)
        return proj_go<Tr, 128, 128, 2, 2>(s, m, k, n2, Q1, A2, lda, colmax, part, splits, scaling);
    return proj_go<Tr, 64, 64, 2, 2>(s, m, k, n2, Q1, A2, lda, colmax, part, splits, scaling);
}

hipError_t launch_projection(hipStream_t s, int prec, int scaling, int64_t m, int64_t k,
                             int64_t n2, const float *Q1, const float *A2, int64_t lda,
                             const float *colmax, float *part, int splits) {
    switch (prec) {
        case QRX_FP16: return proj_dispatch<PF16>(s, m, k, n2, Q1, A2, lda, colmax, part, splits, scaling);
        case QRX_FP16X3: return proj_dispatch<PF16X3>(s, m, k, n2, Q1, A2, lda, colmax, part, splits, scaling);
        case QRX_BF16: return proj_dispatch<PBF16>(s, m, k, n2, Q1, A2, lda, colmax, part, splits, scaling);
        default: return proj_dispatch<PF32>(s, m, k, n2, Q1, A2, lda, colmax, part, splits, 0);
    }
}

hipError_t launch_proj_reduce(hipStream_t s, int prec, int scaling, int64_t k, int64_t n2,
                              const float *part, int splits, float *R12, int64_t ldr,
                              float *colmax, float *uscale, float *Racc, int64_t ldacc) {
    const int lowp_scaled = (prec != QRX_FP32) && scaling;
    hipLaunchKernelGGL(proj_reduce_kernel, dim3((unsigned)n2), dim3(256), 0, s, k, n2, part,
                       splits, R12, ldr, colmax, uscale, lowp_scaled, Racc, ldacc);
    return hipGetLastError();
}

template <class Tr, int BM, int BN, int WM, int WN>
static hipError_t upd_go(hipStream_t s, int64_t m, int64_t k, int64_t n2, const float *Q1,
                         float *A2, int64_t lda, const float *R12, int64_t ldr,
                         const float *uscale, float *colmax, float *cmpart, int scaling) {
    const int64_t tiles_m = (m + BM - 1) / BM;
    const int64_t tiles = tiles_m * ((n2 + BN - 1) / BN);
    const int vecq = aligned16(Q1) && (lda % 4 == 0);
    const int vecr = aligned16(R12) && (ldr % 4 == 0);
    const int veca = aligned16(A2) && (lda % 4 == 0);
    float *cp = colmax ? cmpart : nullptr;
    hipLaunchKernelGGL((update_kernel<Tr, BM, BN, WM, WN>), dim3((unsigned)tiles), dim3(GT), 0, s,
                       m, n2, k, Q1, lda, A2, lda, R12, ldr, uscale, cp, scaling, vecq, vecr,
                       veca);
    if (colmax)
        hipLaunchKernelGGL(colmax_reduce_kernel, dim3((unsigned)((n2 + 3) / 4)), dim3(256), 0, s,
                           n2, tiles_m * WM, cmpart, colmax);
    return hipGetLastError();
}

// Slots of partial column maxima the update may write (max over tile shapes).
int64_t update_cmpart_slots(int64_t m) { return ((m + 127) / 128) * 2 + ((m + 255) / 256) * 4; }

template <class Tr>
static hipError_t upd_dispatch(hipStream_t s, int64_t m, int64_t k, int64_t n2, const float *Q1,
                               float *A2, int64_t lda, const float *R12, int64_t ldr,
                               const float *uscale, float *colmax, float *cmpart, int scaling) {
    if (n2 >= 128)
        return upd_go<Tr, 128, 128, 2, 2>(s, m, k, n2, Q1, A2, lda, R12, ldr, uscale, colmax,
                                          cmpart, scaling);
    if (n2 > 32)
        return upd_go<Tr, 256, 64, 4, 1>(s, m, k, n2, Q1, A2, lda, R12, ldr, uscale, colmax,
                                         cmpart, scaling);
    return upd_go<Tr, 256, 32, 4, 1>(s, m, k, n2, Q1, A2, lda, R12, ldr, uscale, colmax, cmpart,
                                     scaling);
}

hipError_t launch_update(hipStream_t s, int prec, int scaling, int64_t m, int64_t k, int64_t n2,
                         const float *Q1, float *A2, int64_t lda, const float *R12,
                         int64_t ldr, const float *uscale, float *colmax, float *cmpart) {
    switch (prec) {
        case QRX_FP16: return upd_dispatch<PF16>(s, m, k, n2, Q1, A2, lda, R12, ldr, uscale, colmax, cmpart, scaling);
        case QRX_FP16X3: return upd_dispatch<PF16X3>(s, m, k, n2, Q1, A2, lda, R12, ldr, uscale, colmax, cmpart, scaling);
        case QRX_BF16: return upd_dispatch<PBF16>(s, m, k, n2, Q1, A2, lda, R12, ldr, uscale, colmax, cmpart, scaling);
        default: return upd_dispatch<PF32>(s, m, k, n2, Q1, A2, lda, R12, ldr, uscale, colmax, cmpart, 0);
    }
}

}  // namespace qrx
