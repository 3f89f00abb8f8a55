// Trailing products of the recursive Gram-Schmidt QR (Alg. 2):
//   projection  R12 = Q1^T A2      (M = k, N = n2, K = m)
//   update      A2 <- A2 - Q1 R12  (M = m, N = n2, K = k)
// on the matrix cores (MFMA 16x16) with FP32 accumulation. This file holds
// the FP32 products (FP32 MFMA) and the kernels shared with the low-precision
// products of gemm_lp.hip: the split-K reduce, which also packs R12 for a
// low-precision update, and the column max-abs reduce (Sec. 3.1.2: the
// products are what the low-precision unit accelerates).
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
#include "gemm_common.hpp"

namespace qrx {

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

// R12[i, j] = unscale_j * sum_s part[s][i + j*M]; update scale of column j;
// with Racc, also Racc += R12 (second projection of a re-orthogonalised node).
// With Rh, also the update's operand copy Rh[i + j*ldh] = fl(R12[i, j] scale_j)
// in FP16 / BF16 (eprec 1 / 2) or as an FP16 hi/lo pair (eprec 3, lo in Rl).
__global__ __launch_bounds__(256) void proj_reduce_kernel(int64_t M, int64_t N,
                                                          const float *__restrict__ part,
                                                          int splits, float *__restrict__ R12,
                                                          int64_t ldr, float *__restrict__ colmax,
                                                          float *__restrict__ uscale, int lowp_scaled,
                                                          float *__restrict__ Racc, int64_t ldacc,
                                                          uint16_t *__restrict__ Rh,
                                                          uint16_t *__restrict__ Rl, int64_t ldh,
                                                          int eprec) {
    const int64_t j = blockIdx.x;
    __shared__ float smax[4];
    __shared__ float us_s;
    __shared__ float gsum[256];
    const float unscale = lowp_scaled ? 1.0f / (16384.0f * pow2_scale(colmax[j], 14)) : 1.0f;
    const int64_t MN = M * N;
    const float *pj = part + j * M;
    // sum of splits [q0, q1) for row i, eight loads in flight, added in split order
    auto ssum = [&](int64_t i, int q0, int q1) {
        float s = 0.0f;
        int q = q0;
        for (; q + 8 <= q1; q += 8) {
            float v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = pj[(int64_t)(q + u) * MN + i];
#pragma unroll
            for (int u = 0; u < 8; ++u) s += v[u];
        }
        for (; q < q1; ++q) s += pj[(int64_t)q * MN + i];
        return s;
    };
    float mx = 0.0f;
    if (M <= 128 && splits > 1) {
        // short columns: G groups of threads sum consecutive ranges of the splits,
        // then the group sums are added in group order
        const int G = 256 / (int)M, gi = threadIdx.x / (int)M, i = threadIdx.x % (int)M;
        const int per = (splits + G - 1) / G;
        if (gi < G) {
            const int q0 = gi * per, q1 = (q0 + per < splits) ? q0 + per : splits;
            gsum[gi * M + i] = ssum(i, q0 < splits ? q0 : splits, q1);
        }
        __syncthreads();
        if (gi == 0) {
            float s = gsum[i];
            for (int g = 1; g < G; ++g) s += gsum[g * M + i];
            s *= unscale;
            R12[i + j * ldr] = s;
            if (Racc) Racc[i + j * ldacc] += s;
            mx = fabsf(s);
        }
    } else {
        for (int64_t i = threadIdx.x; i < M; i += 256) {
            float s = ssum(i, 0, splits) * unscale;
            R12[i + j * ldr] = s;
            if (Racc) Racc[i + j * ldacc] += s;
            mx = fmaxf(mx, fabsf(s));
        }
    }
    mx = wave_max_f(mx);
    if ((threadIdx.x & 63) == 0) smax[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        float m2 = fmaxf(fmaxf(smax[0], smax[1]), fmaxf(smax[2], smax[3]));
        const float us = lowp_scaled ? pow2_scale(m2, 14) : 1.0f;
        uscale[j] = us;
        us_s = us;
    }
    if (!Rh) return;
    __syncthreads();
    const float us = us_s;
    for (int64_t i = threadIdx.x; i < M; i += 256) {
        const float v = R12[i + j * ldr] * us;     // this thread's own value from above
        if (eprec == 2) {
            const __bf16 b = (__bf16)v;
            Rh[i + j * ldh] = *reinterpret_cast<const uint16_t *>(&b);
        } else {
            const _Float16 h = (_Float16)v;
            Rh[i + j * ldh] = *reinterpret_cast<const uint16_t *>(&h);
            if (eprec == 3) {
                const _Float16 l = (_Float16)(v - (float)h);
                Rl[i + j * ldh] = *reinterpret_cast<const uint16_t *>(&l);
            }
        }
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

// Split-K count of the projection: about 1024 workgroups over the output tiles
// (FP32: 128 x 128; low precision: 256 x 128 when k >= 256 and n2 >= 128,
// else 128 x 128), at least 256 rows per split, at most 256 splits.
// Output tile of a node's projection kernel: the dispatchers below (FP32 here,
// 16-bit in gemm_lp.hip) use the same rule.
void projection_tile(int64_t k, int64_t n2, int prec, int &tm, int &tn) {
    if (prec == QRX_FP32) {
        tm = tn = (k >= 128 && n2 >= 128) ? 128 : 64;
        return;
    }
    if (prec != QRX_FP16X3 && k >= 512 && n2 >= 128) {
        tm = 256;
        tn = 128;
    } else if (k >= 256 && n2 >= 128) {
        tm = tn = 128;
    } else {
        tm = tn = 64;
    }
}

// Split-K count of a projection: about `target` workgroups (default 512), at
// least 128 rows per split, at most 256 splits and at most 16 MB of FP32
// partials (each split writes a k x n2 block that proj_reduce reads back).
int projection_splits(int64_t m, int64_t k, int64_t n2, int prec, int target) {
    int tm, tn;
    projection_tile(k, n2, prec, tm, tn);
    const int64_t tiles = ((k + tm - 1) / tm) * ((n2 + tn - 1) / tn);
    const int64_t tgt = target > 0 ? target : 512;
    int64_t want = (tgt + tiles - 1) / tiles;
    const int64_t maxs = (m + 127) / 128;
    const int64_t cap = (int64_t)(16 << 20) / (4 * (k > 0 ? k : 1) * (n2 > 0 ? n2 : 1));
    if (want > maxs) want = maxs;
    if (want > cap) want = cap;
    if (want > 256) want = 256;
    if (want < 1) want = 1;
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
        case QRX_FP32: return proj_dispatch<PF32>(s, m, k, n2, Q1, A2, lda, colmax, part, splits, 0);
        default: return hipErrorInvalidValue;   // low precision: launch_projection_lp
    }
}

hipError_t launch_proj_reduce(hipStream_t s, int prec, int scaling, int64_t k, int64_t n2,
                              const float *part, int splits, float *R12, int64_t ldr,
                              float *colmax, float *uscale, float *Racc, int64_t ldacc,
                              uint16_t *Rh, uint16_t *Rl, int64_t ldh) {
    const int lowp_scaled = (prec != QRX_FP32) && scaling;
    hipLaunchKernelGGL(proj_reduce_kernel, dim3((unsigned)n2), dim3(256), 0, s, k, n2, part,
                       splits, R12, ldr, colmax, uscale, lowp_scaled, Racc, ldacc, Rh, Rl, ldh,
                       prec);
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
    if (colmax) return launch_colmax_reduce(s, n2, tiles_m * WM, cmpart, colmax);
    return hipGetLastError();
}

hipError_t launch_colmax_reduce(hipStream_t s, int64_t n2, int64_t slots, const float *cmpart,
                                float *colmax) {
    hipLaunchKernelGGL(colmax_reduce_kernel, dim3((unsigned)((n2 + 3) / 4)), dim3(256), 0, s, n2,
                       slots, cmpart, colmax);
    return hipGetLastError();
}

// Slots of partial column maxima the update may write (max over tile shapes).
int64_t update_cmpart_slots(int64_t m) { return ((m + 63) / 64) * 4; }

template <class Tr>
static hipError_t upd_dispatch(hipStream_t s, int64_t m, int64_t k, int64_t n2, const float *Q1,
                               float *A2, int64_t lda, const float *R12, int64_t ldr,
                               const float *uscale, float *colmax, float *cmpart, int scaling) {
    if (n2 >= 128)
        return upd_go<Tr, 128, 128, 2, 2>(s, m, k, n2, Q1, A2, lda, R12, ldr, uscale, colmax,
                                          cmpart, scaling);
    if (n2 > 32) {
        // 128-row tiles when 256-row tiles would not cover the chip twice
        if ((m + 255) / 256 >= 512)
            return upd_go<Tr, 256, 64, 4, 1>(s, m, k, n2, Q1, A2, lda, R12, ldr, uscale, colmax,
                                             cmpart, scaling);
        return upd_go<Tr, 128, 64, 4, 1>(s, m, k, n2, Q1, A2, lda, R12, ldr, uscale, colmax,
                                         cmpart, scaling);
    }
    return upd_go<Tr, 256, 32, 4, 1>(s, m, k, n2, Q1, A2, lda, R12, ldr, uscale, colmax, cmpart,
                                     scaling);
}

hipError_t launch_update(hipStream_t s, int prec, int scaling, int64_t m, int64_t k, int64_t n2,
                         const float *Q1, float *A2, int64_t lda, const float *R12,
                         int64_t ldr, const float *uscale, float *colmax, float *cmpart) {
    switch (prec) {
        case QRX_FP32: return upd_dispatch<PF32>(s, m, k, n2, Q1, A2, lda, R12, ldr, uscale, colmax, cmpart, 0);
        default: return hipErrorInvalidValue;   // low precision: launch_update_lp
    }
}

}  // namespace qrx
