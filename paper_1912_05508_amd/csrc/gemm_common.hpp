// Tile helpers shared by the trailing-product kernels: precision traits,
// FP32 -> FP16/BF16 (and split FP16) staging, operand loaders and the MFMA
// inner loops (16x16 MFMA, FP32 accumulation).
#pragma once

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
// Split FP16: x = hi + lo with hi = fl16(x), lo = fl16(x - hi);
// x y ~ hi_x hi_y + hi_x lo_y + lo_x hi_y, three FP16 MFMAs per step.
struct PF16X3 {
    using E = _Float16;
    static constexpr int KS = 32;
    static constexpr int BK = 64;
    static constexpr int PAD = 8;
    static constexpr bool SPLIT = true;
};
// FP16 / BF16 with 32-wide K stages (half the LDS per tile: two workgroups per
// CU); measured faster than 64-wide stages for the plain 16-bit products, slower
// for the split products.
struct PF16K32 {
    using E = _Float16;
    static constexpr int KS = 32;
    static constexpr int BK = 32;
    static constexpr int PAD = 8;
    static constexpr bool SPLIT = false;
};
struct PBF16K32 {
    using E = __bf16;
    static constexpr int KS = 32;
    static constexpr int BK = 32;
    static constexpr int PAD = 8;
    static constexpr bool SPLIT = false;
};

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
    f16x4 vl = {(_Float16)(a - (float)ha), (_Float16)(b - (float)hb), (_Float16)(c - (float)hc),
                (_Float16)(e - (float)he)};
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
    static_assert(NR >= 1 && NR * COLS_PER_PASS == C, "K loader mapping");
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
    static_assert(NB4 >= 1 && NB4 * GT == NBLK, "M loader mapping");
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


// Load a K-contiguous tile of 16-bit elements: ROWS rows x BK elements of X
// (row r, element k at X[r * ld + k]), k in [k0, kend), r in [r0, rend); zero
// outside. Each thread moves NL 16-byte pieces.
template <int BK, int ROWS>
struct ELoader {
    static constexpr int SEGS = BK / 8;             // 16-byte pieces per row
    static constexpr int NL = ROWS * SEGS / GT;
    static_assert(NL * GT == ROWS * SEGS, "loader mapping");
    uint4 v[NL];
    template <class E>
    QRX_DEV void load(const E *X, int64_t ld, int64_t k0, int64_t kend, int64_t r0, int64_t rend,
                      bool vec, int t) {
        static_assert(sizeof(E) == 2, "16-bit elements");
#pragma unroll
        for (int p = 0; p < NL; ++p) {
            const int idx = t + p * GT;
            const int row = idx / SEGS, seg = idx % SEGS;
            const int64_t r = r0 + row, k = k0 + seg * 8;
            uint4 x = make_uint4(0u, 0u, 0u, 0u);
            if (r < rend) {
                const E *src = X + r * ld + k;
                if (vec && k + 7 < kend) {
                    x = *reinterpret_cast<const uint4 *>(src);
                } else {
                    uint16_t h[8];
#pragma unroll
                    for (int q = 0; q < 8; ++q)
                        h[q] = (k + q < kend) ? reinterpret_cast<const uint16_t *>(src)[q] : 0;
                    x.x = h[0] | ((uint32_t)h[1] << 16);
                    x.y = h[2] | ((uint32_t)h[3] << 16);
                    x.z = h[4] | ((uint32_t)h[5] << 16);
                    x.w = h[6] | ((uint32_t)h[7] << 16);
                }
            }
            v[p] = x;
        }
    }
    // store to LDS [row][LS] (16-bit elements)
    template <class E, int LS>
    QRX_DEV void store(E *S, int t) const {
#pragma unroll
        for (int p = 0; p < NL; ++p) {
            const int idx = t + p * GT;
            const int row = idx / SEGS, seg = idx % SEGS;
            *reinterpret_cast<uint4 *>(S + row * LS + seg * 8) = v[p];
        }
    }
};

}  // namespace qrx
