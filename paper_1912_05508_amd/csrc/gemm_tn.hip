// Large-tile trailing products on 16-bit operands (FP16, BF16, split FP16).
//
// Both products of Alg. 2 are C = A B^T with A and B stored K-contiguous:
//   projection R12 = Q1^T A2: A = Qc (column i of Q1, rows = K), B = the
//     node's A2 packed to 16-bit with its column scales (pack_cols_kernel);
//   update A2 -= Q1 R12: A = Qr (row r of Q1, columns = K), B = Rh (column j
//     of the packed R12, rows = K).
// One workgroup of 8 waves computes a 256 x 256 tile (each wave 128 x 64 with
// 16x16x32 MFMAs, FP32 accumulation) through double-buffered, XOR-swizzled LDS
// stages (64 deep), one barrier per stage; workgroups go to the XCDs in contiguous tile
// ranges (rows of tiles that share an operand block run on one L2).
// Split FP16 (x = hi + lo, lo = fl16(x - hi)) stages the hi and lo tiles of
// both operands (32 deep) and issues hi*hi, hi*lo and lo*hi for every fragment
// pair into the same FP32 accumulator; the lo*lo term is dropped.
// The projection is split over K (blockIdx.y) into FP32 partials summed in a
// fixed order by proj_reduce; the update subtracts its tile from A2 in place
// (scaled back by 1 / (2^14 s_j)) and writes partial column max-abs values.
#include "gemm_common.hpp"

namespace qrx {

namespace tn {
constexpr int BM = 256, BN = 256;
constexpr int WM = 2, WN = 4, NT = WM * WN * 64;
constexpr int FM = BM / WM / 16, FN = BN / WN / 16;
constexpr int kXcds = 8;
// Stage geometry: plain products stage A and B 64 deep; split products stage
// A_hi, A_lo, B_hi, B_lo 32 deep (128 KB of LDS either way, double-buffered).
// Rows are unpadded; the 16-byte piece q of row r is stored at piece
// q ^ ((r / RP) mod QP), RP = rows per 256 bytes, so that the 16 rows a
// fragment read touches in one piece column hit 16 different bank groups.
template <bool SPLIT>
struct Geo {
    static constexpr int BK = SPLIT ? 32 : 64;
    static constexpr int NTILE = SPLIT ? 4 : 2;
    static constexpr int LS = BK;                     // row stride (16-bit elements)
    static constexpr int TS = BM * LS;                // one tile
    static constexpr int QP = BK / 8;                 // 16-byte pieces per row
    static constexpr int RP = 128 / BK;               // rows per 256 bytes
    static constexpr int PT = BM * QP / NT;           // pieces per thread and tile
    static_assert(BM == BN && PT * NT == BM * QP && QP * RP == 16, "loader mapping");
    QRX_DEV static int off(int r, int q) { return r * LS + ((q ^ ((r / RP) & (QP - 1))) * 8); }
};

QRX_DEV int64_t xcd_order(int64_t b, int64_t nt) {
    if (nt % kXcds) return b;
    return (b % kXcds) * (nt / kXcds) + b / kXcds;
}

// 8 elements of row r at column k of X (row-major in K, ld), zero outside
// [0, rend) x [0, kend); a full piece in range is one 16-byte load.
template <class E>
QRX_DEV uint4 piece(const E *X, int64_t ld, int64_t r, int64_t rend, int64_t k, int64_t kend) {
    uint4 x = make_uint4(0u, 0u, 0u, 0u);
    if (r < rend) {
        const E *src = X + r * ld + k;
        if (k + 8 <= kend) {
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
    return x;
}

template <class E, class V8>
QRX_DEV f32x4 mma(const V8 &a, const V8 &b, const f32x4 &c) {
    if constexpr (std::is_same<E, _Float16>::value)
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
    else
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
}  // namespace tn

// MODE 0 (projection): part[blockIdx.y][i + j M] = sum over this split's
// stages. MODE 1 (update): A2[i + j lda] -= es_j * sum (i < M rows of A2).
// SPLIT: hi*hi + hi*lo + lo*hi per fragment pair, one FP32 accumulator.
template <class E, int MODE, bool SPLIT>
__global__ __launch_bounds__(tn::NT) void tn_mma_kernel(
    int64_t M, int64_t N, int64_t K, const E *__restrict__ Ah, const E *__restrict__ Al,
    int64_t lda_op, const E *__restrict__ Bh, const E *__restrict__ Bl, int64_t ldb_op,
    int64_t stages_per_split, float *__restrict__ out, int64_t ldo,
    const float *__restrict__ uscale, float *__restrict__ cmpart, int scaled) {
    using namespace tn;
    using G = Geo<SPLIT>;
    constexpr int BK = G::BK, LS = G::LS, TS = G::TS, QP = G::QP, PT = G::PT, NTILE = G::NTILE;
    __shared__ __attribute__((aligned(16))) E L[2 * NTILE * TS];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int wm = wv % WM, wn = wv / WM;
    const int64_t tiles_m = (M + BM - 1) / BM, tiles_n = (N + BN - 1) / BN;
    const int64_t tile = xcd_order(blockIdx.x, tiles_m * tiles_n);
    int64_t tm, tnn;
    if (MODE == 0) {   // row tiles of one B block adjacent
        tm = tile % tiles_m;
        tnn = tile / tiles_m;
    } else {           // column tiles of one A row block adjacent
        tnn = tile % tiles_n;
        tm = tile / tiles_n;
    }
    const int64_t i0 = tm * BM, j0 = tnn * BN;
    const int64_t nk = (K + BK - 1) / BK;
    const int64_t s0 = (int64_t)blockIdx.y * stages_per_split;
    int64_t s1 = s0 + stages_per_split;
    if (s1 > nk) s1 = nk;

    f32x4 acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

    // tiles of a stage: plain (A, B); split (A_hi, A_lo, B_hi, B_lo)
    uint4 rg[NTILE][PT];
    auto gload = [&](int64_t s) {
        const int64_t k0 = s * BK;
#pragma unroll
        for (int x = 0; x < NTILE; ++x) {
            const bool isb = x >= NTILE / 2;
            const E *X = isb ? ((SPLIT && x == 3) ? Bl : Bh) : ((SPLIT && x == 1) ? Al : Ah);
            const int64_t ld = isb ? ldb_op : lda_op;
            const int64_t base = isb ? j0 : i0, rend = isb ? N : M;
#pragma unroll
            for (int p = 0; p < PT; ++p) {
                const int e = t + p * NT, r = e / QP, q = e % QP;
                rg[x][p] = piece(X, ld, base + r, rend, k0 + q * 8, K);
            }
        }
    };
    auto lstore = [&](int buf) {
#pragma unroll
        for (int x = 0; x < NTILE; ++x)
#pragma unroll
            for (int p = 0; p < PT; ++p) {
                const int e = t + p * NT, r = e / QP, q = e % QP;
                *reinterpret_cast<uint4 *>(L + (buf * NTILE + x) * TS + G::off(r, q)) = rg[x][p];
            }
    };
    using V8 = typename std::conditional<std::is_same<E, _Float16>::value, f16x8, bf16x8>::type;
    if (s0 < s1) {
        gload(s0);
        lstore(0);
    }
    __syncthreads();
    const int rl = lane & 15, kq = lane >> 4;
    for (int64_t s = s0; s < s1; ++s) {
        const int buf = (int)((s - s0) & 1);
        if (s + 1 < s1) gload(s + 1);
        const E *a = L + (buf * NTILE) * TS;
        const E *b = L + (buf * NTILE + NTILE / 2) * TS;
        const int ar = wm * (BM / WM) + rl, br = wn * (BN / WN) + rl;
        if constexpr (SPLIT) {
            V8 bh[FN], bl[FN];
#pragma unroll
            for (int f = 0; f < FN; ++f) {
                bh[f] = *reinterpret_cast<const V8 *>(b + G::off(br + f * 16, kq));
                bl[f] = *reinterpret_cast<const V8 *>(b + TS + G::off(br + f * 16, kq));
            }
#pragma unroll
            for (int i = 0; i < FM; ++i) {
                const V8 ah = *reinterpret_cast<const V8 *>(a + G::off(ar + i * 16, kq));
                const V8 al = *reinterpret_cast<const V8 *>(a + TS + G::off(ar + i * 16, kq));
#pragma unroll
                for (int j = 0; j < FN; ++j) {
                    acc[i][j] = mma<E>(ah, bh[j], acc[i][j]);
                    acc[i][j] = mma<E>(ah, bl[j], acc[i][j]);
                    acc[i][j] = mma<E>(al, bh[j], acc[i][j]);
                }
            }
        } else {
#pragma unroll
            for (int kk = 0; kk < BK; kk += 32) {
                V8 af[FM], bf[FN];
#pragma unroll
                for (int f = 0; f < FM; ++f)
                    af[f] = *reinterpret_cast<const V8 *>(a + G::off(ar + f * 16, kk / 8 + kq));
#pragma unroll
                for (int f = 0; f < FN; ++f)
                    bf[f] = *reinterpret_cast<const V8 *>(b + G::off(br + f * 16, kk / 8 + kq));
#pragma unroll
                for (int i = 0; i < FM; ++i)
#pragma unroll
                    for (int j = 0; j < FN; ++j) acc[i][j] = mma<E>(af[i], bf[j], acc[i][j]);
            }
        }
        if (s + 1 < s1) lstore(buf ^ 1);
        __syncthreads();
    }

    if constexpr (MODE == 0) {
        float *P = out + (int64_t)blockIdx.y * M * N;
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
    } else {
        const bool veca = ((ldo & 3) == 0) && ((((uintptr_t)out) & 15) == 0);
#pragma unroll
        for (int fn = 0; fn < FN; ++fn) {
            const int64_t j = j0 + wn * (BN / WN) + fn * 16 + (lane & 15);
            const bool jin = j < N;
            const float es = (scaled && jin) ? 1.0f / (16384.0f * uscale[j]) : 1.0f;
            float cmax = 0.0f;
#pragma unroll
            for (int fm = 0; fm < FM; ++fm) {
                const int64_t rb = i0 + wm * (BM / WM) + fm * 16 + 4 * (lane >> 4);
                if (jin) {
                    float *dst = out + j * ldo + rb;
                    if (veca && rb + 3 < M) {
                        float4 x = *reinterpret_cast<float4 *>(dst);
                        x.x = fmaf(-es, acc[fm][fn][0], x.x);
                        x.y = fmaf(-es, acc[fm][fn][1], x.y);
                        x.z = fmaf(-es, acc[fm][fn][2], x.z);
                        x.w = fmaf(-es, acc[fm][fn][3], x.w);
                        *reinterpret_cast<float4 *>(dst) = x;
                        cmax = fmaxf(cmax, fmaxf(fmaxf(fabsf(x.x), fabsf(x.y)),
                                                 fmaxf(fabsf(x.z), fabsf(x.w))));
                    } else {
#pragma unroll
                        for (int v = 0; v < 4; ++v)
                            if (rb + v < M) {
                                const float y = fmaf(-es, acc[fm][fn][v], dst[v]);
                                dst[v] = y;
                                cmax = fmaxf(cmax, fabsf(y));
                            }
                    }
                }
            }
            if (cmpart) {
                cmax = fmaxf(cmax, __shfl_xor(cmax, 16));
                cmax = fmaxf(cmax, __shfl_xor(cmax, 32));
                const int64_t slot = tm * WM + wm;
                if (jin && lane < 16) cmpart[slot * N + j] = cmax;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// A2 (m x n2, FP32, column-major lda) -> 16-bit copies scaled per column by
// s_j = 2^(14 - E_j) (max-abs of column j brought to [2^13, 2^14); 1 without
// scaling): Bh[j ldb + r] = fl(A2 s_j), and with a split Bl = fl16(A2 s_j - Bh).
// Eight rows per thread.
// ---------------------------------------------------------------------------
template <class E, bool SPLIT>
__global__ __launch_bounds__(256) void pack_cols_kernel(const float *__restrict__ A2, int64_t lda,
                                                        int64_t m, const float *__restrict__ colmax,
                                                        int scaling, E *__restrict__ Bh,
                                                        E *__restrict__ Bl, int64_t ldb) {
    const int64_t j = blockIdx.y;
    const int64_t r = ((int64_t)blockIdx.x * 256 + threadIdx.x) * 8;
    if (r >= m) return;
    const float s = scaling ? pow2_scale(colmax[j], 14) : 1.0f;
    const float *src = A2 + j * lda + r;
    float v[8];
    if (r + 8 <= m && ((((uintptr_t)src) & 15) == 0)) {
        const float4 a = reinterpret_cast<const float4 *>(src)[0];
        const float4 b = reinterpret_cast<const float4 *>(src)[1];
        v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
        v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
    } else {
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] = (r + q < m) ? src[q] : 0.0f;
    }
    using V8 = typename std::conditional<std::is_same<E, _Float16>::value, f16x8, bf16x8>::type;
    V8 h, l;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const float x = v[q] * s;
        h[q] = (E)x;
        if constexpr (SPLIT) l[q] = (E)(x - (float)h[q]);
    }
    E *dh = Bh + j * ldb + r;
    if (r + 8 <= m) {
        *reinterpret_cast<V8 *>(dh) = h;
        if constexpr (SPLIT) *reinterpret_cast<V8 *>(Bl + j * ldb + r) = l;
    } else {
        for (int q = 0; q < 8 && r + q < m; ++q) {
            dh[q] = h[q];
            if constexpr (SPLIT) Bl[j * ldb + r + q] = l[q];
        }
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static bool a16(const void *p) { return (((uintptr_t)p) & 15) == 0; }

bool tn_eligible(int64_t rows, int64_t cols, int64_t ld_a, int64_t ld_b, const void *a,
                 const void *b) {
    return rows >= 256 && cols >= 256 && ld_a % 8 == 0 && ld_b % 8 == 0 && a16(a) && a16(b);
}

int tn_projection_splits(int64_t m, int64_t k, int64_t n2, int target) {
    const int64_t tiles = ((k + tn::BM - 1) / tn::BM) * ((n2 + tn::BN - 1) / tn::BN);
    const int64_t tgt = target > 0 ? target : 256;   // default: one workgroup per CU
    int64_t want = (tgt + tiles - 1) / tiles;
    const int64_t maxs = (m + 511) / 512;          // at least 512 rows per split
    if (want > maxs) want = maxs;
    if (want < 1) want = 1;
    if (want > 64) want = 64;
    return (int)want;
}

hipError_t launch_pack_cols(hipStream_t s, int prec, int scaling, int64_t m, int64_t n2,
                            const float *A2, int64_t lda, const float *colmax, uint16_t *bh,
                            uint16_t *bl, int64_t ldb) {
    const dim3 g((unsigned)((m + 2047) / 2048), (unsigned)n2), b(256);
    switch (prec) {
        case QRX_FP16:
            hipLaunchKernelGGL((pack_cols_kernel<_Float16, false>), g, b, 0, s, A2, lda, m, colmax,
                               scaling, (_Float16 *)bh, (_Float16 *)nullptr, ldb);
            break;
        case QRX_BF16:
            hipLaunchKernelGGL((pack_cols_kernel<__bf16, false>), g, b, 0, s, A2, lda, m, colmax,
                               scaling, (__bf16 *)bh, (__bf16 *)nullptr, ldb);
            break;
        case QRX_FP16X3:
            hipLaunchKernelGGL((pack_cols_kernel<_Float16, true>), g, b, 0, s, A2, lda, m, colmax,
                               scaling, (_Float16 *)bh, (_Float16 *)bl, ldb);
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <class E, int MODE, bool SPLIT>
static hipError_t tn_go(hipStream_t s, int64_t M, int64_t N, int64_t K, const uint16_t *ah,
                        const uint16_t *al, int64_t lda_op, const uint16_t *bh,
                        const uint16_t *bl, int64_t ldb_op, int splits, float *out, int64_t ldo,
                        const float *uscale, float *cmpart, int scaled) {
    const int64_t tiles = ((M + tn::BM - 1) / tn::BM) * ((N + tn::BN - 1) / tn::BN);
    const int64_t total = (K + tn::Geo<SPLIT>::BK - 1) / tn::Geo<SPLIT>::BK;
    const int64_t per = (total + splits - 1) / splits;
    hipLaunchKernelGGL((tn_mma_kernel<E, MODE, SPLIT>), dim3((unsigned)tiles, (unsigned)splits),
                       dim3(tn::NT), 0, s, M, N, K, (const E *)ah, (const E *)al, lda_op,
                       (const E *)bh, (const E *)bl, ldb_op, per, out, ldo, uscale, cmpart,
                       scaled);
    return hipGetLastError();
}

template <int MODE>
static hipError_t tn_prec(hipStream_t s, int prec, int64_t M, int64_t N, int64_t K,
                          const uint16_t *ah, const uint16_t *al, int64_t lda_op,
                          const uint16_t *bh, const uint16_t *bl, int64_t ldb_op, int splits,
                          float *out, int64_t ldo, const float *uscale, float *cmpart, int scaled) {
    switch (prec) {
        case QRX_FP16:
            return tn_go<_Float16, MODE, false>(s, M, N, K, ah, al, lda_op, bh, bl, ldb_op, splits,
                                                out, ldo, uscale, cmpart, scaled);
        case QRX_BF16:
            return tn_go<__bf16, MODE, false>(s, M, N, K, ah, al, lda_op, bh, bl, ldb_op, splits,
                                              out, ldo, uscale, cmpart, scaled);
        case QRX_FP16X3:
            return tn_go<_Float16, MODE, true>(s, M, N, K, ah, al, lda_op, bh, bl, ldb_op, splits,
                                               out, ldo, uscale, cmpart, scaled);
        default: return hipErrorInvalidValue;
    }
}

// R12 partials: part[split][i + j k] = sum_r Qc[r][i] B[r][j] over the split's rows.
hipError_t launch_projection_tn(hipStream_t s, int prec, int64_t m, int64_t k, int64_t n2,
                                const uint16_t *qc, const uint16_t *qcl, int64_t ldc,
                                const uint16_t *bh, const uint16_t *bl, int64_t ldb, float *part,
                                int splits) {
    return tn_prec<0>(s, prec, k, n2, m, qc, qcl, ldc, bh, bl, ldb, splits, part, k, nullptr,
                      nullptr, 0);
}

hipError_t launch_colmax_reduce(hipStream_t s, int64_t n2, int64_t slots, const float *cmpart,
                                float *colmax);

// A2 -= Q1 R12 (scaled back per column), optional column max-abs of the result.
hipError_t launch_update_tn(hipStream_t s, int prec, int scaling, int64_t m, int64_t k,
                            int64_t n2, const uint16_t *qr, const uint16_t *qrl, int64_t ldq,
                            const uint16_t *rh, const uint16_t *rhl, int64_t ldh, float *A2,
                            int64_t lda, const float *uscale, float *colmax, float *cmpart) {
    float *cp = colmax ? cmpart : nullptr;
    const hipError_t e = tn_prec<1>(s, prec, m, n2, k, qr, qrl, ldq, rh, rhl, ldh, 1, A2, lda,
                                    uscale, cp, scaling);
    if (e != hipSuccess) return e;
    if (colmax) return launch_colmax_reduce(s, n2, ((m + tn::BM - 1) / tn::BM) * tn::WM, cmpart, colmax);
    return hipSuccess;
}

}  // namespace qrx
