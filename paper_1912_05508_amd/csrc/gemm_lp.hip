// Low-precision trailing products (FP16, BF16, split FP16) on pre-packed
// operand copies.
//
// The products of Alg. 2 read Q1 many times (once per tile row or column of
// the result), so each panel's Q columns are packed once, right after the
// panel, into 16-bit copies already multiplied by the Q scale 2^14:
//   Qc  column-major (rows contiguous): the K-contiguous A operand of the
//       projection R12 = Q1^T A2 (K = rows);
//   Qr  row-major (columns contiguous): the K-contiguous A operand of the
//       update A2 -= Q1 R12 (K = Q1 columns).
// The projection's reduce kernel packs R12 (times its column scales) the same
// way for the update. Both products then stage 16-byte pieces straight into
// double-buffered LDS tiles (one barrier per K stage); only A2, the FP32
// operand of the projection, is converted (and column-scaled) on the way in.
// Split FP16 keeps a second copy with the low parts lo = fl16(x - hi).
//
// Workgroups are handed to the 8 XCDs round-robin; the tile order gives each
// XCD a contiguous range of tiles, so the tiles that share an operand block
// run on one L2.
#include "gemm_common.hpp"

namespace qrx {

constexpr int kXcds = 8;

QRX_DEV int64_t xcd_tile(int64_t b, int64_t nt) {
    if (nt % kXcds) return b;
    return (b % kXcds) * (nt / kXcds) + b / kXcds;
}

// ---------------------------------------------------------------------------
// Projection: part[s][i + j*M] = sum_{r in split s} Qc[i][r] * A2[r, j] (scaled)
// ---------------------------------------------------------------------------
template <class Tr, int BM, int BN, int WM, int WN>
__global__ __launch_bounds__(GT) void proj_lp_kernel(int64_t K, int64_t M, int64_t N,
                                                     const typename Tr::E *__restrict__ Qc,
                                                     const typename Tr::E *__restrict__ Ql,
                                                     int64_t ldc, const float *__restrict__ A2,
                                                     int64_t lda, const float *__restrict__ colmax,
                                                     int scaling, int64_t kchunk,
                                                     float *__restrict__ part, int vecq, int veca) {
    using E = typename Tr::E;
    constexpr int BK = Tr::BK, LS = BK + Tr::PAD;
    constexpr int FM = BM / WM / 16, FN = BN / WN / 16;
    constexpr int NS = Tr::SPLIT ? 2 : 1;
    constexpr int ASZ = NS * BM * LS, BSZ = NS * BN * LS;
    __shared__ __attribute__((aligned(16))) E As[2 * ASZ];
    __shared__ __attribute__((aligned(16))) E Bs[2 * BSZ];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int wm = wv % WM, wn = wv / WM;
    const int64_t tiles_m = (M + BM - 1) / BM, tiles_n = (N + BN - 1) / BN;
    const int64_t tile = xcd_tile(blockIdx.x, tiles_m * tiles_n);
    const int64_t tm = tile % tiles_m, tn = tile / tiles_m;   // row tiles of one A2 block adjacent
    const int64_t i0 = tm * BM, j0 = tn * BN;
    const int64_t kb = blockIdx.y * kchunk;
    const int64_t ke = (kb + kchunk < K) ? kb + kchunk : K;
    const int64_t nst = (ke > kb) ? (ke - kb + BK - 1) / BK : 0;

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

    ELoader<BK, BM> la;
    ELoader<BK, Tr::SPLIT ? BM : 64> la2;
    KLoader<BK, BN> lb;
    auto bscale = [&](int64_t c) {
        return (scaling && c < N) ? pow2_scale(colmax[c], 14) : 1.0f;
    };
    auto gload = [&](int64_t k0) {
        la.load(Qc, ldc, k0, ke, i0, M, vecq, t);
        if constexpr (Tr::SPLIT) la2.load(Ql, ldc, k0, ke, i0, M, vecq, t);
        lb.load(A2, lda, k0, ke, j0, N, veca, t);
    };
    auto lstore = [&](int buf) {
        E *a = As + buf * ASZ;
        E *b = Bs + buf * BSZ;
        la.template store<E, LS>(a, t);
        if constexpr (Tr::SPLIT) {
            la2.template store<E, LS>(a + BM * LS, t);
            lb.template store_split<LS>(b, b + BN * LS, j0, t, bscale);
        } else {
            lb.template store<E, LS>(b, j0, t, bscale);
        }
    };
    if (nst > 0) {
        gload(kb);
        lstore(0);
    }
    __syncthreads();
    for (int64_t s = 0; s < nst; ++s) {
        const int buf = (int)(s & 1);
        if (s + 1 < nst) gload(kb + (s + 1) * BK);
        const E *a = As + buf * ASZ;
        const E *b = Bs + buf * BSZ;
        if constexpr (Tr::SPLIT)
            mma_stage_split<FM, FN, BK, LS>(a, a + BM * LS, b, b + BN * LS, wm * (BM / WM),
                                            wn * (BN / WN), acc, acc2, lane);
        else
            mma_stage<Tr, FM, FN>(a, b, wm * (BM / WM), wn * (BN / WN), acc, lane);
        if (s + 1 < nst) lstore(buf ^ 1);
        __syncthreads();
    }
    if constexpr (Tr::SPLIT) {
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j) acc[i][j] += acc2[i][j];
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

// ---------------------------------------------------------------------------
// Update: A2[r, j] -= es_j * sum_i Qr[r][i] Rh[i][j]; partial column max-abs.
// ---------------------------------------------------------------------------
template <class Tr, int BM, int BN, int WM, int WN>
__global__ __launch_bounds__(GT) void update_lp_kernel(int64_t M, int64_t N, int64_t K,
                                                       const typename Tr::E *__restrict__ Qr,
                                                       const typename Tr::E *__restrict__ Qrl,
                                                       int64_t ldq,
                                                       const typename Tr::E *__restrict__ Rh,
                                                       const typename Tr::E *__restrict__ Rhl,
                                                       int64_t ldh, float *__restrict__ A2,
                                                       int64_t lda, const float *__restrict__ uscale,
                                                       float *__restrict__ cmpart, int scaled,
                                                       int vec, int veca) {
    using E = typename Tr::E;
    constexpr int BK = Tr::BK, LS = BK + Tr::PAD;
    constexpr int FM = BM / WM / 16, FN = BN / WN / 16;
    constexpr int NS = Tr::SPLIT ? 2 : 1;
    constexpr int ASZ = NS * BM * LS, BSZ = NS * BN * LS;
    __shared__ __attribute__((aligned(16))) E As[2 * ASZ];
    __shared__ __attribute__((aligned(16))) E Bs[2 * BSZ];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int wm = wv % WM, wn = wv / WM;
    const int64_t tiles_m = (M + BM - 1) / BM, tiles_n = (N + BN - 1) / BN;
    const int64_t tile = xcd_tile(blockIdx.x, tiles_m * tiles_n);
    const int64_t tn = tile % tiles_n, tm = tile / tiles_n;   // column tiles of one row block adjacent
    const int64_t r0 = tm * BM, j0 = tn * BN;
    const int64_t nst = (K + BK - 1) / BK;

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

    ELoader<BK, BM> la;
    ELoader<BK, Tr::SPLIT ? BM : 64> la2;
    ELoader<BK, BN> lb;
    ELoader<BK, Tr::SPLIT ? BN : 64> lb2;
    auto gload = [&](int64_t k0) {
        la.load(Qr, ldq, k0, K, r0, M, vec, t);
        lb.load(Rh, ldh, k0, K, j0, N, vec, t);
        if constexpr (Tr::SPLIT) {
            la2.load(Qrl, ldq, k0, K, r0, M, vec, t);
            lb2.load(Rhl, ldh, k0, K, j0, N, vec, t);
        }
    };
    auto lstore = [&](int buf) {
        E *a = As + buf * ASZ;
        E *b = Bs + buf * BSZ;
        la.template store<E, LS>(a, t);
        lb.template store<E, LS>(b, t);
        if constexpr (Tr::SPLIT) {
            la2.template store<E, LS>(a + BM * LS, t);
            lb2.template store<E, LS>(b + BN * LS, t);
        }
    };
    if (nst > 0) {
        gload(0);
        lstore(0);
    }
    __syncthreads();
    for (int64_t s = 0; s < nst; ++s) {
        const int buf = (int)(s & 1);
        if (s + 1 < nst) gload((s + 1) * BK);
        const E *a = As + buf * ASZ;
        const E *b = Bs + buf * BSZ;
        if constexpr (Tr::SPLIT)
            mma_stage_split<FM, FN, BK, LS>(a, a + BM * LS, b, b + BN * LS, wm * (BM / WM),
                                            wn * (BN / WN), acc, acc2, lane);
        else
            mma_stage<Tr, FM, FN>(a, b, wm * (BM / WM), wn * (BN / WN), acc, lane);
        if (s + 1 < nst) lstore(buf ^ 1);
        __syncthreads();
    }
    if constexpr (Tr::SPLIT) {
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j) acc[i][j] += acc2[i][j];
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
            const int64_t slot = tm * WM + wm;
            if (jin && lane < 16) cmpart[slot * N + j] = cmax;
        }
    }
}

// ---------------------------------------------------------------------------
// Q packing: copies of sc * Q (m x w, FP32, column-major ldq) in 16-bit
// elements, column-major Qc (ldc) and row-major Qr (ldr); with a split, also
// the low parts. A workgroup moves 64 rows through LDS.
// ---------------------------------------------------------------------------
template <class E, bool SPLIT>
__global__ __launch_bounds__(256) void pack_q_kernel(const float *__restrict__ Q, int64_t ldq,
                                                     int64_t m, int w, float sc,
                                                     E *__restrict__ Qc, E *__restrict__ Qcl,
                                                     int64_t ldc, E *__restrict__ Qr,
                                                     E *__restrict__ Qrl, int64_t ldr) {
    __shared__ float T[64][65];
    const int t = threadIdx.x;
    const int64_t r0 = (int64_t)blockIdx.x * 64;
#pragma unroll 4
    for (int p = 0; p < 16; ++p) {
        const int idx = t + 256 * p;
        const int rr = idx % 64, cc = idx / 64;
        const int64_t r = r0 + rr;
        const bool in = r < m && cc < w;
        const float v = in ? Q[r + cc * ldq] * sc : 0.0f;
        T[rr][cc] = v;
        if (in) {
            const E h = (E)v;
            Qc[r + cc * ldc] = h;
            if constexpr (SPLIT) Qcl[r + cc * ldc] = (E)(v - (float)h);
        }
    }
    __syncthreads();
#pragma unroll 4
    for (int p = 0; p < 16; ++p) {
        const int idx = t + 256 * p;
        const int cc = idx % 64, rr = idx / 64;
        const int64_t r = r0 + rr;
        if (r < m && cc < w) {
            const float v = T[rr][cc];
            const E h = (E)v;
            Qr[r * ldr + cc] = h;
            if constexpr (SPLIT) Qrl[r * ldr + cc] = (E)(v - (float)h);
        }
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static bool al16(const void *p) { return (((uintptr_t)p) & 15) == 0; }

hipError_t launch_pack_q(hipStream_t s, int prec, int scaling, int64_t m, int w, const float *Q,
                         int64_t ldq, uint16_t *qc, uint16_t *qcl, int64_t ldc, uint16_t *qr,
                         uint16_t *qrl, int64_t ldr) {
    if (w > 64) return hipErrorInvalidValue;
    const float sc = scaling ? 16384.0f : 1.0f;
    const dim3 g((unsigned)((m + 63) / 64)), b(256);
    switch (prec) {
        case QRX_FP16:
            hipLaunchKernelGGL((pack_q_kernel<_Float16, false>), g, b, 0, s, Q, ldq, m, w, sc,
                               (_Float16 *)qc, (_Float16 *)nullptr, ldc, (_Float16 *)qr,
                               (_Float16 *)nullptr, ldr);
            break;
        case QRX_BF16:
            hipLaunchKernelGGL((pack_q_kernel<__bf16, false>), g, b, 0, s, Q, ldq, m, w, sc,
                               (__bf16 *)qc, (__bf16 *)nullptr, ldc, (__bf16 *)qr,
                               (__bf16 *)nullptr, ldr);
            break;
        case QRX_FP16X3:
            hipLaunchKernelGGL((pack_q_kernel<_Float16, true>), g, b, 0, s, Q, ldq, m, w, sc,
                               (_Float16 *)qc, (_Float16 *)qcl, ldc, (_Float16 *)qr,
                               (_Float16 *)qrl, ldr);
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <class Tr, int BM, int BN, int WM, int WN>
static hipError_t projlp_go(hipStream_t s, int64_t m, int64_t k, int64_t n2, const uint16_t *qc,
                            const uint16_t *qcl, int64_t ldc, const float *A2, int64_t lda,
                            const float *colmax, float *part, int splits, int scaling) {
    using E = typename Tr::E;
    const int64_t tiles = ((k + BM - 1) / BM) * ((n2 + BN - 1) / BN);
    int64_t kchunk = (m + splits - 1) / splits;
    kchunk = ((kchunk + Tr::BK - 1) / Tr::BK) * Tr::BK;
    const int vecq = al16(qc) && (!qcl || al16(qcl)) && (ldc % 8 == 0);
    const int veca = al16(A2) && (lda % 4 == 0);
    hipLaunchKernelGGL((proj_lp_kernel<Tr, BM, BN, WM, WN>), dim3((unsigned)tiles, splits),
                       dim3(GT), 0, s, m, k, n2, (const E *)qc, (const E *)qcl, ldc, A2, lda,
                       colmax, scaling, kchunk, part, vecq, veca);
    return hipGetLastError();
}

template <class Tr>
static hipError_t projlp_dispatch(hipStream_t s, int64_t m, int64_t k, int64_t n2,
                                  const uint16_t *qc, const uint16_t *qcl, int64_t ldc,
                                  const float *A2, int64_t lda, const float *colmax, float *part,
                                  int splits, int scaling) {
    // the tile rule of projection_tile
    if constexpr (!Tr::SPLIT) {
        if (k >= 512 && n2 >= 128)
            return projlp_go<Tr, 256, 128, 2, 2>(s, m, k, n2, qc, qcl, ldc, A2, lda, colmax, part,
                                                 splits, scaling);
    }
    if (k >= 256 && n2 >= 128)
        return projlp_go<Tr, 128, 128, 2, 2>(s, m, k, n2, qc, qcl, ldc, A2, lda, colmax, part,
                                             splits, scaling);
    return projlp_go<Tr, 64, 64, 2, 2>(s, m, k, n2, qc, qcl, ldc, A2, lda, colmax, part, splits,
                                       scaling);
}

hipError_t launch_projection_lp(hipStream_t s, int prec, int scaling, int64_t m, int64_t k,
                                int64_t n2, const uint16_t *qc, const uint16_t *qcl, int64_t ldc,
                                const float *A2, int64_t lda, const float *colmax, float *part,
                                int splits) {
    switch (prec) {
        case QRX_FP16: return projlp_dispatch<PF16K32>(s, m, k, n2, qc, qcl, ldc, A2, lda, colmax, part, splits, scaling);
        case QRX_BF16: return projlp_dispatch<PBF16K32>(s, m, k, n2, qc, qcl, ldc, A2, lda, colmax, part, splits, scaling);
        case QRX_FP16X3: return projlp_dispatch<PF16X3>(s, m, k, n2, qc, qcl, ldc, A2, lda, colmax, part, splits, scaling);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_colmax_reduce(hipStream_t s, int64_t n2, int64_t slots, const float *cmpart,
                                float *colmax);

template <class Tr, int BM, int BN, int WM, int WN>
static hipError_t updlp_go(hipStream_t s, int64_t m, int64_t k, int64_t n2, const uint16_t *qr,
                           const uint16_t *qrl, int64_t ldq, const uint16_t *rh,
                           const uint16_t *rhl, int64_t ldh, float *A2, int64_t lda,
                           const float *uscale, float *colmax, float *cmpart, int scaling) {
    using E = typename Tr::E;
    const int64_t tiles_m = (m + BM - 1) / BM;
    const int64_t tiles = tiles_m * ((n2 + BN - 1) / BN);
    const int vec = al16(qr) && al16(rh) && (!qrl || al16(qrl)) && (!rhl || al16(rhl)) &&
                    (ldq % 8 == 0) && (ldh % 8 == 0);
    const int veca = al16(A2) && (lda % 4 == 0);
    float *cp = colmax ? cmpart : nullptr;
    hipLaunchKernelGGL((update_lp_kernel<Tr, BM, BN, WM, WN>), dim3((unsigned)tiles), dim3(GT), 0,
                       s, m, n2, k, (const E *)qr, (const E *)qrl, ldq, (const E *)rh,
                       (const E *)rhl, ldh, A2, lda, uscale, cp, scaling, vec, veca);
    if (colmax) return launch_colmax_reduce(s, n2, tiles_m * WM, cmpart, colmax);
    return hipGetLastError();
}

template <class Tr>
static hipError_t updlp_dispatch(hipStream_t s, int64_t m, int64_t k, int64_t n2,
                                 const uint16_t *qr, const uint16_t *qrl, int64_t ldq,
                                 const uint16_t *rh, const uint16_t *rhl, int64_t ldh, float *A2,
                                 int64_t lda, const float *uscale, float *colmax, float *cmpart,
                                 int scaling) {
    // 128 x 128 tiles measured fastest for the large nodes
    if (n2 > 64)
        return updlp_go<Tr, 128, 128, 2, 2>(s, m, k, n2, qr, qrl, ldq, rh, rhl, ldh, A2, lda,
                                            uscale, colmax, cmpart, scaling);
    return updlp_go<Tr, 128, 64, 2, 1>(s, m, k, n2, qr, qrl, ldq, rh, rhl, ldh, A2, lda, uscale,
                                       colmax, cmpart, scaling);
}

hipError_t launch_update_lp(hipStream_t s, int prec, int scaling, int64_t m, int64_t k,
                            int64_t n2, const uint16_t *qr, const uint16_t *qrl, int64_t ldq,
                            const uint16_t *rh, const uint16_t *rhl, int64_t ldh, float *A2,
                            int64_t lda, const float *uscale, float *colmax, float *cmpart) {
    switch (prec) {
        case QRX_FP16: return updlp_dispatch<PF16K32>(s, m, k, n2, qr, qrl, ldq, rh, rhl, ldh, A2, lda, uscale, colmax, cmpart, scaling);
        case QRX_BF16: return updlp_dispatch<PBF16K32>(s, m, k, n2, qr, qrl, ldq, rh, rhl, ldh, A2, lda, uscale, colmax, cmpart, scaling);
        case QRX_FP16X3: return updlp_dispatch<PF16X3>(s, m, k, n2, qr, qrl, ldq, rh, rhl, ldh, A2, lda, uscale, colmax, cmpart, scaling);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace qrx
