// The whole right-preconditioned Krylov least-squares iteration (Sec. 3.2.3;
// LSQR by default, CGLS as in Alg. 5 with the readings of its listing) as one
// persistent kernel: the iteration, its stopping test, the certification with
// the true residual and the restarts on it all run on the device, so a solve
// enqueues no host round trip per iteration and can be recorded into a HIP
// graph.
//
// Every workgroup of the launch takes part in every phase (grid-stride loops
// over "virtual blocks"); phases are separated by a software grid barrier.
// Scalars (norms, the LSQR Givens step, the CGLS step lengths, the decisions
// to certify, restart or stop) are computed by every workgroup from the same
// partial sums in the same order, so all workgroups hold bit-identical values
// and take the same branches without a broadcast.
//
// Per LSQR iteration, with X = R^{-1} (FP64, formed once) and its transpose:
//   t = X v                   (triangular product, one wave per column of X^T)
//   u~ = A t - alpha u, z = A^T u~   (n <= 1024: both in one pass over A, partials
//                             per workgroup, then summed; otherwise a GEMV-N over
//                             column splits and a GEMV-T over row splits)
//   v~ = X^T z / beta - beta v, alpha = ||v~||   (one wave per column of X)
//   Givens step, d = t - (theta/rho) d, x += (phi/rho) d, v = v~ / alpha
// All sums are taken in a fixed order (deterministic results).
//
// Memory: values a phase produces are read by other workgroups only after a
// barrier. Uniform (workgroup-wide) reads of such values go through LDS,
// never through scalar loads: the scalar data cache is not refreshed by the
// barrier's acquire.
#include "qrx_internal.hpp"
#include "krylov.hpp"

namespace qrx {

namespace {

constexpr int LT = 512;            // threads per workgroup (8 waves: one workgroup per CU)
constexpr int GN_STAGE = 1024;     // GEMV-N input entries staged in LDS at a time
constexpr int GT_R = 4096;         // rows per GEMV-T split (u slice in LDS)
constexpr int GT_C = 4 * (LT / 64);  // columns per GEMV-T virtual block (4 per wave)
constexpr unsigned kSpinLimit = 1u << 24;   // barrier polls before giving up (seconds)

// ---- grid barrier -------------------------------------------------------------
// A 64-bit arrival count that only grows (bytes 16..23 of bar) and an abort
// flag (bar[2]); all zero at launch. Thread 0 releases the workgroup's writes
// (agent scope) with its arrival; the workgroups of barrier k (counting from 0)
// wait until the count reaches (k + 1) nwg, k being its own arrival's count
// divided by nwg. The arrivals are read-modify-writes of one location, so the
// value that ends the wait carries every arrival's release; the last arrival
// does not wait. A poll limit or an abort raised by another workgroup ends the
// wait with `false`, so every workgroup leaves even if the launch was not
// co-resident.
QRX_DEV bool grid_barrier(unsigned *bar, unsigned nwg, int *sflag) {
    __syncthreads();
    if (threadIdx.x == 0) {
        int ok = 1;
        unsigned long long *cnt = reinterpret_cast<unsigned long long *>(bar + 4);
        const unsigned long long prev =
            __hip_atomic_fetch_add(cnt, 1ull, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        const unsigned long long target = (prev / nwg + 1) * nwg;
        if (prev + 1 != target) {
            unsigned polls = 0;
            while (__hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
                if (__hip_atomic_load(bar + 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u ||
                    ++polls > kSpinLimit) {
                    __hip_atomic_store(bar + 2, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    ok = 0;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        *sflag = ok;
    }
    __syncthreads();
    return *sflag != 0;
}

// threadIdx.x behind an empty asm statement: values a phase derives from it
// are computed inside the phase instead of being hoisted to the start of the
// kernel, where they would stay live across every phase (and be spilled).
QRX_DEV int lane_id_opaque() {
    int t = (int)threadIdx.x;
    asm volatile("" : "+v"(t));
    return t;
}

// ---- workgroup reductions --------------------------------------------------------
// Sum of p[0..count) in a fixed order: thread-strided partial sums, then a tree.
QRX_DEV double wg_sum(const double *p, int64_t count, double *sh) {
    double a = 0.0;
    for (int64_t i = threadIdx.x; i < count; i += LT) a += p[i];
    sh[threadIdx.x] = a;
    __syncthreads();
    for (int o = LT / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

// Sum of one value per thread (wave sums, then waves in order) into *dst by thread 0.
QRX_DEV void wg_partial(double v, double *dst, double *sh) {
    const double w = wave_sum_d(v);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = w;
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0.0;
        for (int i = 0; i < LT / 64; ++i) a += sh[i];
        *dst = a;
    }
    __syncthreads();
}

QRX_DEV unsigned nblk(int64_t n) { return (unsigned)((n + LT - 1) / LT); }

// ---- phases ------------------------------------------------------------------------
// GEMV-N partials: pn[s][r] = sum_{j in split s} A[r, j] in[j] (dd: double-double,
// lo parts in pn2). Virtual block = 4 LT rows (4 per thread) x one column split.
QRX_DEV void ph_gemv_n(const KLoopArgs &K, const double *in, double *pn, double *pn2, int dd,
                       double *stage) {
    const int64_t m = K.m, n = K.n;
    const int64_t nrb = (m + 4 * LT - 1) / (4 * LT);
    const int64_t nvb = nrb * K.splits_n;
    for (int64_t vb = blockIdx.x; vb < nvb; vb += gridDim.x) {
        const int64_t rb = vb % nrb, s = vb / nrb;
        const int64_t r = (rb * LT + lane_id_opaque()) * 4;
        const int64_t j0 = s * K.cchunk;
        const int64_t j1 = (j0 + K.cchunk < n) ? j0 + K.cchunk : n;
        const bool act = r < m;
        const bool v4 = K.vec && (r + 3 < m);
        double h[4] = {0, 0, 0, 0}, l[4] = {0, 0, 0, 0};
        for (int64_t c0 = j0; c0 < j1; c0 += GN_STAGE) {
            const int64_t c1 = (c0 + GN_STAGE < j1) ? c0 + GN_STAGE : j1;
            __syncthreads();
            for (int64_t j = c0 + lane_id_opaque(); j < c1; j += LT) stage[j - c0] = in[j];
            __syncthreads();
            if (!act) continue;
            int64_t j = c0;
            if (v4) {
                constexpr int GU = 16;   // column loads in flight per thread
                for (; j + GU <= c1; j += GU) {
                    float4 q[GU];
#pragma unroll
                    for (int u = 0; u < GU; ++u)
                        q[u] = *reinterpret_cast<const float4 *>(K.A + (j + u) * K.lda + r);
                    if (dd) {
#pragma unroll
                        for (int u = 0; u < GU; ++u) {
                            const double xj = stage[j + u - c0];
                            dd_add_prod(h[0], l[0], (double)q[u].x, xj);
                            dd_add_prod(h[1], l[1], (double)q[u].y, xj);
                            dd_add_prod(h[2], l[2], (double)q[u].z, xj);
                            dd_add_prod(h[3], l[3], (double)q[u].w, xj);
                        }
                    } else {
#pragma unroll
                        for (int u = 0; u < GU; ++u) {
                            const double xj = stage[j + u - c0];
                            h[0] = fma((double)q[u].x, xj, h[0]);
                            h[1] = fma((double)q[u].y, xj, h[1]);
                            h[2] = fma((double)q[u].z, xj, h[2]);
                            h[3] = fma((double)q[u].w, xj, h[3]);
                        }
                    }
                }
            }
            for (; j < c1; ++j) {
                const double xj = stage[j - c0];
                const float *a = K.A + j * K.lda + r;
                float e[4];
                if (v4) {
                    const float4 q = *reinterpret_cast<const float4 *>(a);
                    e[0] = q.x; e[1] = q.y; e[2] = q.z; e[3] = q.w;
                } else {
#pragma unroll
                    for (int k = 0; k < 4; ++k) e[k] = (r + k < m) ? a[k] : 0.0f;
                }
                if (dd) {
#pragma unroll
                    for (int k = 0; k < 4; ++k) dd_add_prod(h[k], l[k], (double)e[k], xj);
                } else {
#pragma unroll
                    for (int k = 0; k < 4; ++k) h[k] = fma((double)e[k], xj, h[k]);
                }
            }
        }
        if (act) {
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (r + k < m) {
                    pn[s * m + r + k] = h[k];
                    if (dd) pn2[s * m + r + k] = l[k];
                }
        }
    }
}

// GEMV-T partials: pt[s][j] = sum_{r in split s} A[r, j] in[r]. Virtual block =
// GT_C columns (4 per wave) x one 4096-row split; the slice of `in` sits in LDS.
QRX_DEV void ph_gemv_t(const KLoopArgs &K, const double *in, double *pt, double *us) {
    const int64_t m = K.m, n = K.n;
    const int64_t ncg = (n + GT_C - 1) / GT_C;
    const int64_t nvb = ncg * K.splits_t;
    const int lane = lane_id_opaque() & 63, wv = lane_id_opaque() >> 6;
    constexpr int CW = 4;
    // split-major order: a workgroup's consecutive virtual blocks share their row
    // split whenever the grid is a multiple of the split count, so the slice of
    // `in` is staged once for all of them
    int64_t staged = -1;
    for (int64_t vb = blockIdx.x; vb < nvb; vb += gridDim.x) {
        const int64_t s = vb % K.splits_t, cg = vb / K.splits_t;
        const int64_t rs = s * GT_R;
        const int64_t re = (rs + GT_R < m) ? rs + GT_R : m;
        const int cnt = (int)(re - rs);
        if (s != staged) {
            __syncthreads();
            for (int i = lane_id_opaque(); i < GT_R; i += LT) us[i] = (i < cnt) ? in[rs + i] : 0.0;
            __syncthreads();
            staged = s;
        }
        const int64_t j0 = cg * GT_C + wv * CW;
        const float *a[CW];
        bool jin[CW];
#pragma unroll
        for (int q = 0; q < CW; ++q) {
            jin[q] = j0 + q < n;
            a[q] = K.A + (jin[q] ? j0 + q : n - 1) * K.lda + rs;
        }
        double acc[CW];
#pragma unroll
        for (int q = 0; q < CW; ++q) acc[q] = 0.0;
        if (K.vec) {
            auto block = [&](const float4 *e, int i) {
                const double u0 = us[i], u1 = us[i + 1], u2 = us[i + 2], u3 = us[i + 3];
#pragma unroll
                for (int q = 0; q < CW; ++q) {
                    acc[q] = fma((double)e[q].x, u0, acc[q]);
                    acc[q] = fma((double)e[q].y, u1, acc[q]);
                    acc[q] = fma((double)e[q].z, u2, acc[q]);
                    acc[q] = fma((double)e[q].w, u3, acc[q]);
                }
            };
            const int cnt4 = cnt & ~3;
            int i = lane * 4;
            for (; i + 256 < cnt4; i += 512) {
                float4 e0[CW], e1[CW];
#pragma unroll
                for (int q = 0; q < CW; ++q) e0[q] = *reinterpret_cast<const float4 *>(a[q] + i);
#pragma unroll
                for (int q = 0; q < CW; ++q)
                    e1[q] = *reinterpret_cast<const float4 *>(a[q] + i + 256);
                block(e0, i);
                block(e1, i + 256);
            }
            for (; i < cnt4; i += 256) {
                float4 e0[CW];
#pragma unroll
                for (int q = 0; q < CW; ++q) e0[q] = *reinterpret_cast<const float4 *>(a[q] + i);
                block(e0, i);
            }
            if (i < cnt) {
                for (int k = 0; k < 4 && i + k < cnt; ++k)
#pragma unroll
                    for (int q = 0; q < CW; ++q)
                        acc[q] = fma((double)a[q][i + k], us[i + k], acc[q]);
            }
        } else {
            for (int i = lane; i < cnt; i += 64)
#pragma unroll
                for (int q = 0; q < CW; ++q) acc[q] = fma((double)a[q][i], us[i], acc[q]);
        }
#pragma unroll
        for (int q = 0; q < CW; ++q) {
            const double v = wave_sum_d(acc[q]);
            if (lane == 0 && jin[q]) pt[s * n + j0 + q] = v;
        }
    }
}

// out[r] = sum_s pn[s][r] - coef * y[r] (y may be null); ssq[vb] = partial sum of out^2.
QRX_DEV void ph_combine_m(const KLoopArgs &K, double coef, double *y, double *out, double *ssq,
                          double *sh) {
    const int64_t m = K.m;
    const unsigned nvb = nblk(m);
    for (unsigned vb = blockIdx.x; vb < nvb; vb += gridDim.x) {
        const int64_t r = (int64_t)vb * LT + lane_id_opaque();
        double v2 = 0.0;
        if (r < m) {
            double s = 0.0;
            // four splits' partials loaded together, added in split order
            int q = 0;
            for (; q + 4 <= K.splits_n; q += 4) {
                double v[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) v[k] = K.pn[(int64_t)(q + k) * m + r];
#pragma unroll
                for (int k = 0; k < 4; ++k) s += v[k];
            }
            for (; q < K.splits_n; ++q) s += K.pn[(int64_t)q * m + r];
            if (y) s = fma(-coef, y[r], s);
            out[r] = s;
            v2 = s * s;
        }
        wg_partial(v2, ssq + vb, sh);
    }
}

// rc = b - sum_s (hi_s + lo_s) in double-double, rounded; ssq partials.
QRX_DEV void ph_resid(const KLoopArgs &K, double *ssq, double *sh) {
    const int64_t m = K.m;
    const unsigned nvb = nblk(m);
    for (unsigned vb = blockIdx.x; vb < nvb; vb += gridDim.x) {
        const int64_t r = (int64_t)vb * LT + lane_id_opaque();
        double v2 = 0.0;
        if (r < m) {
            double h = K.b[r], l = 0.0;
            // four splits' hi and lo partials loaded together, added in split order
            int q = 0;
            for (; q + 4 <= K.splits_n; q += 4) {
                double ph[4], pl[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    ph[k] = K.pn[(int64_t)(q + k) * m + r];
                    pl[k] = K.pn2[(int64_t)(q + k) * m + r];
                }
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    dd_add(h, l, -ph[k]);
                    dd_add(h, l, -pl[k]);
                }
            }
            for (; q < K.splits_n; ++q) {
                dd_add(h, l, -K.pn[(int64_t)q * m + r]);
                dd_add(h, l, -K.pn2[(int64_t)q * m + r]);
            }
            const double v = h + l;
            K.rc[r] = v;
            v2 = v * v;
        }
        wg_partial(v2, ssq + vb, sh);
    }
}

// z[j] = sum_s pt[s][j] (j < n), one wave per column (lanes take the splits
// lane, lane + 64, ... in order; fixed reduction order); optional ssq partials,
// one per virtual block of LT / 64 columns.
QRX_DEV void ph_combine_n(const KLoopArgs &K, double *ssq, double *sh) {
    const int64_t n = K.n;
    constexpr int NW = LT / 64;
    const int lane = lane_id_opaque() & 63, wv = lane_id_opaque() >> 6;
    const unsigned nvb = (unsigned)((n + NW - 1) / NW);
    for (unsigned vb = blockIdx.x; vb < nvb; vb += gridDim.x) {
        const int64_t j = (int64_t)vb * NW + wv;
        double e2 = 0.0;
        if (j < n) {
            double s = 0.0;
            for (int q = lane; q < K.splits_t; q += 64) s += K.pt[(int64_t)q * n + j];
            s = wave_sum_d(s);
            if (lane == 0) K.z[j] = s;
            e2 = s * s;
        }
        if (ssq) {
            if (lane == 0) sh[wv] = e2;
            __syncthreads();
            if (threadIdx.x == 0) {
                double a = 0.0;
                for (int w = 0; w < NW; ++w) a += sh[w];
                ssq[vb] = a;
            }
            __syncthreads();
        }
    }
}

// ssq partials of v[0..len) (256 entries per virtual block).
QRX_DEV void ph_ssq(const double *v, int64_t len, double *ssq, double *sh) {
    const unsigned nvb = nblk(len);
    for (unsigned vb = blockIdx.x; vb < nvb; vb += gridDim.x) {
        const int64_t j = (int64_t)vb * LT + lane_id_opaque();
        const double e = j < len ? v[j] : 0.0;
        wg_partial(e * e, ssq + vb, sh);
    }
}

// Elementwise loop over [0, len) in 256-entry virtual blocks (the same entries go
// to the same workgroup in every call with the same len).
template <class F>
QRX_DEV void ph_each(int64_t len, F f) {
    const unsigned nvb = nblk(len);
    for (unsigned vb = blockIdx.x; vb < nvb; vb += gridDim.x) {
        const int64_t j = (int64_t)vb * LT + lane_id_opaque();
        if (j < len) f(j);
    }
}

// Dot product of rows [i0, i1) of one column with `in`, by one wave (lane-strided,
// eight loads in flight, fixed reduction order).
QRX_DEV double col_dot(const double *col, const double *in, int64_t i0, int64_t i1, int lane) {
    double acc = 0.0;
    int64_t i = i0 + lane;
    for (; i + 7 * 64 < i1; i += 8 * 64) {
        double c[8], w[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            c[u] = col[i + u * 64];
            w[u] = in[i + u * 64];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) acc = fma(c[u], w[u], acc);
    }
    // the rest (fewer than eight per lane): loaded together, then added in order
    // (an entry past the end contributes fma(0, 0, acc) = acc)
    {
        double c[8], w[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int64_t k = i + (int64_t)u * 64;
            const bool in_range = k < i1;
            c[u] = in_range ? col[k] : 0.0;
            w[u] = in_range ? in[k] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) acc = fma(c[u], w[u], acc);
    }
    return wave_sum_d(acc);
}

// x += a * d for entry j, accumulated in double-double (x, xlo): over the
// thousands of updates of a restart, rounding x after each one would add a
// random walk of about sqrt(updates) * u |x| to it, which for a strongly
// column-scaled A already exceeds the 1e-10 backward-error target; the pair
// keeps x itself the rounded sum. The residual of a restart is that of x,
// so xlo is dropped (zeroed) when the next restart begins.
QRX_DEV void x_update(const KLoopArgs &K, int64_t j, double a, double d) {
    double hi = K.x[j], lo = K.xlo[j];
    dd_add_prod(hi, lo, a, d);
    K.x[j] = hi;
    K.xlo[j] = lo;
}

// Triangular products. Output entries come in pairs (c, np-1-c), whose two
// columns have np + 1 entries in all, so that every pair is the same work; a
// pair is split over WP waves of one workgroup (WP = 1..8, as many as the
// grid's waves allow), wave s taking entries [s T/WP, (s+1) T/WP) of the two
// columns laid end to end (T = np + 1), and the WP partial sums are added in
// wave order (fixed reduction order). Virtual block = 8 / WP pairs.
//   upper = 1: out[c] = sum_{i <= c} M[i, c] in[i]   (M = X: out = X^T in)
//   upper = 0: out[c] = sum_{i >= c} M[i, c] in[i]   (M = X^T: out = X in)
// each times `scale`. M == null stands for the identity. The epilogue receives
// (c, value) on one lane and returns the entry's contribution to the virtual
// block's ssq partial.
QRX_DEV int tri_waves_per_pair(int64_t np, unsigned G) {
    const int64_t npairs = np / 2;
    int wp = LT / 64;
    while (wp > 1 && (int64_t)wp * npairs > (LT / 64) * (int64_t)G) wp >>= 1;
    return wp;
}
QRX_DEV unsigned tri_vblocks(int64_t np, unsigned G) {
    const int pw = (LT / 64) / tri_waves_per_pair(np, G);
    return (unsigned)((np / 2 + pw - 1) / pw);
}

template <class E>
QRX_DEV void ph_tri(const KLoopArgs &K, const double *M, const double *in, int upper,
                    double scale, double *ssq, double *sh, E epi) {
    const int64_t np = K.np;
    const int lane = lane_id_opaque() & 63, wv = lane_id_opaque() >> 6;
    constexpr int NW = LT / 64;
    const int wp = __builtin_amdgcn_readfirstlane(tri_waves_per_pair(np, gridDim.x));
    const int pw = NW / wp;
    const int pp = wv / wp, sg = wv % wp;        // pair within the block, segment of the pair
    const int64_t npairs = np / 2;
    const int64_t nvb = (npairs + pw - 1) / pw;
    const int64_t T = np + 1;
    double *part = sh + NW;                      // [pair][segment][2]
    for (int64_t vb = blockIdx.x; vb < nvb; vb += gridDim.x) {
        const int64_t p = vb * pw + pp;
        const bool act = p < npairs;
        const int64_t c0 = p, c1 = np - 1 - p;
        // concatenated entries [0, L0) lie in column c0, [L0, T) in column c1
        const int64_t L0 = upper ? c0 + 1 : np - c0;
        const int64_t s0 = sg * T / wp, s1 = (sg + 1) * T / wp;
        double v0 = 0.0, v1 = 0.0;
        if (act) {
            if (M == nullptr) {
                if (sg == 0) {
                    v0 = in[c0];
                    v1 = in[c1];
                }
            } else {
                // the segment's share of column c0 (first stored row r0) ...
                const int64_t a0 = s0 < L0 ? s0 : L0, b0 = s1 < L0 ? s1 : L0;
                const int64_t r0 = upper ? 0 : c0;
                if (a0 < b0) v0 = col_dot(M + c0 * np, in, r0 + a0, r0 + b0, lane);
                // ... and of column c1
                const int64_t a1 = (s0 > L0 ? s0 : L0) - L0, b1 = (s1 > L0 ? s1 : L0) - L0;
                const int64_t r1 = upper ? 0 : c1;
                if (a1 < b1) v1 = col_dot(M + c1 * np, in, r1 + a1, r1 + b1, lane);
            }
        }
        if (wp > 1) {
            if (lane == 0) {
                part[(pp * wp + sg) * 2] = v0;
                part[(pp * wp + sg) * 2 + 1] = v1;
            }
            __syncthreads();
            if (sg == 0) {
                v0 = part[pp * wp * 2];
                v1 = part[pp * wp * 2 + 1];
                for (int q = 1; q < wp; ++q) {
                    v0 += part[(pp * wp + q) * 2];
                    v1 += part[(pp * wp + q) * 2 + 1];
                }
            }
            __syncthreads();
        }
        double e2 = 0.0;
        if (act && sg == 0 && lane == 0) {
            e2 += epi(c0, v0 * scale);
            e2 += epi(c1, v1 * scale);
        }
        if (ssq) {
            if (lane == 0) sh[wv] = e2;
            __syncthreads();
            if (threadIdx.x == 0) {
                double a = 0.0;
                for (int w = 0; w < NW; ++w) a += sh[w];
                ssq[vb] = a;
            }
            __syncthreads();
        }
    }
}

// ---- LSQR's two products with A in one pass -------------------------------------
// The bidiagonalisation needs A t and then A^T of the result; the second
// product over a row block needs only that block's entries of the first, so a
// block of A serves both while it is on chip: A is read once per iteration
// instead of twice. Blocks are FR rows; groups of FG = 32 / FR consecutive
// blocks (32 rows, whole 128-byte lines of each column) go to the workgroups in
// turn (group k to workgroup k mod G), so the blocks in flight across the chip
// are adjacent in memory. For the workgroup's blocks:
//   u~[r] = (A t)[r] - coef uo[r]          (written to un; uo is not modified)
//   ssqA[wg] = sum of u~[r]^2 over its rows
//   pf[j G + wg] = sum over its rows of A[r, j] u~[r]      (j < n)
// Wave w takes columns [w cw, (w + 1) cw), cw = FS KC with FS = 64 / FQ column
// groups per wave; lane (q, g) = (lane % FQ, lane / FQ), FQ = FR / 4, holds rows
// 4q .. 4q + 3 of its columns w cw + g + FS k, k < KC.
// The entries go from HBM straight into LDS (16 bytes per lane per load, no
// registers) through FNBUF buffers: FNBUF - 1 blocks are in flight while one
// is reduced. (Measured on the 262144 x 1024 workload: 16-row blocks in two
// buffers stream faster than 8-row blocks in four; the access pattern itself
// streams at about 5 TB/s without any arithmetic.)
constexpr int FR = 16;                                  // rows per block
constexpr int FQ = FR / 4;                              // lanes per column of a block
constexpr int FS = 64 / FQ;                             // column groups per wave
constexpr int FG = 32 / FR;                             // blocks per group
constexpr int FKC = (int)(kr_fused_max_n / (LT / 64) / FS);   // most loads per lane
constexpr int FNBUF = 2;                                // LDS buffers
// per wave and buffer: FKC loads x 64 lanes, then the block's FR entries of uo
// (FR / 2 lanes x 16 bytes)
constexpr int FWAVE_F4 = FKC * 64 + FR / 2;
constexpr int FBUF_F4 = 8 * FWAVE_F4;
constexpr int FUSED_LDS_DOUBLES = FNBUF * FBUF_F4 * 2;
constexpr int US_DOUBLES = FUSED_LDS_DOUBLES > GT_R ? FUSED_LDS_DOUBLES : GT_R;

typedef __attribute__((address_space(3))) void lvoid;
typedef float f4v __attribute__((ext_vector_type(4)));
typedef double d2v __attribute__((ext_vector_type(2)));

// s_waitcnt with vmcnt(N) alone (expcnt, lgkmcnt at their no-wait maxima);
// lgkmcnt(0) alone
template <int N>
QRX_DEV void wait_vm() {
    static_assert(N >= 0 && N < 64, "vmcnt range");
    __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | 0x0F70);
}
QRX_DEV void wait_lgkm0() { __builtin_amdgcn_s_waitcnt(0xC07F); }
// vmcnt(c) for a count known only at run time (c clamped to 0..15)
QRX_DEV void wait_vm_rt(int c) {
    switch (c <= 0 ? 0 : c >= 15 ? 15 : c) {
        case 0: wait_vm<0>(); break;
        case 1: wait_vm<1>(); break;
        case 2: wait_vm<2>(); break;
        case 3: wait_vm<3>(); break;
        case 4: wait_vm<4>(); break;
        case 5: wait_vm<5>(); break;
        case 6: wait_vm<6>(); break;
        case 7: wait_vm<7>(); break;
        case 8: wait_vm<8>(); break;
        case 9: wait_vm<9>(); break;
        case 10: wait_vm<10>(); break;
        case 11: wait_vm<11>(); break;
        case 12: wait_vm<12>(); break;
        case 13: wait_vm<13>(); break;
        case 14: wait_vm<14>(); break;
        default: wait_vm<15>(); break;
    }
}

// LDS byte address of a shared-memory pointer
QRX_DEV unsigned lds_addr(const void *p) {
    return (unsigned)(uintptr_t)(const __attribute__((address_space(3))) char *)p;
}

// A pointer every lane holds alike, in scalar registers
template <class T>
QRX_DEV T *uniform_ptr(T *p) {
    const uint64_t v = (uint64_t)(uintptr_t)p;
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)v);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(v >> 32));
    return (T *)(uintptr_t)(((uint64_t)hi << 32) | lo);
}

// Buffer descriptor of `bytes` bytes at p (32-bit data format, as the vector
// memory unit expects of raw buffers); a load past `bytes` returns zeros.
QRX_DEV __amdgpu_buffer_rsrc_t raw_rsrc(const void *p, int64_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes,
                                             0x00020000);
}

// LDS reads of the one-pass products, written out so that the compiler does
// not hold them behind the loads of later blocks still in flight (it cannot
// tell the buffers apart). Each group waits for its own reads before it ends,
// so no read is left in flight.
// KC 16-byte reads at a, a + 1024, ...
template <int KC>
QRX_DEV void lds_read_cols(unsigned a, f4v (&e)[KC]) {
    static_assert(KC == 1 || KC == 2 || KC == 4 || KC == 8, "column loads per lane");
    if constexpr (KC == 1) {
        asm volatile("ds_read_b128 %0, %1\n\ts_waitcnt lgkmcnt(0)"
                     : "=&v"(e[0]) : "v"(a) : "memory");
    } else if constexpr (KC == 2) {
        asm volatile("ds_read_b128 %0, %2\n\tds_read_b128 %1, %2 offset:1024\n\t"
                     "s_waitcnt lgkmcnt(0)"
                     : "=&v"(e[0]), "=&v"(e[1]) : "v"(a) : "memory");
    } else if constexpr (KC == 4) {
        asm volatile("ds_read_b128 %0, %4\n\tds_read_b128 %1, %4 offset:1024\n\t"
                     "ds_read_b128 %2, %4 offset:2048\n\tds_read_b128 %3, %4 offset:3072\n\t"
                     "s_waitcnt lgkmcnt(0)"
                     : "=&v"(e[0]), "=&v"(e[1]), "=&v"(e[2]), "=&v"(e[3]) : "v"(a) : "memory");
    } else {
        asm volatile("ds_read_b128 %0, %8\n\tds_read_b128 %1, %8 offset:1024\n\t"
                     "ds_read_b128 %2, %8 offset:2048\n\tds_read_b128 %3, %8 offset:3072\n\t"
                     "ds_read_b128 %4, %8 offset:4096\n\tds_read_b128 %5, %8 offset:5120\n\t"
                     "ds_read_b128 %6, %8 offset:6144\n\tds_read_b128 %7, %8 offset:7168\n\t"
                     "s_waitcnt lgkmcnt(0)"
                     : "=&v"(e[0]), "=&v"(e[1]), "=&v"(e[2]), "=&v"(e[3]), "=&v"(e[4]),
                       "=&v"(e[5]), "=&v"(e[6]), "=&v"(e[7])
                     : "v"(a) : "memory");
    }
}
// four doubles at a and a + 16
QRX_DEV void lds_read_d4(unsigned a, d2v &lo, d2v &hi) {
    asm volatile("ds_read_b128 %0, %2\n\tds_read_b128 %1, %2 offset:16\n\ts_waitcnt lgkmcnt(0)"
                 : "=&v"(lo), "=&v"(hi) : "v"(a) : "memory");
}
// four doubles at a + 8 FR w and a + 8 FR w + 16 for w = 0..3 (four waves' row
// partials of one row quad, as 8 pairs in wave order)
static_assert(FR == 16, "row partial layout of lds_read_red4");
QRX_DEV void lds_read_red4(unsigned a, d2v (&v)[8]) {
    asm volatile("ds_read_b128 %0, %8\n\tds_read_b128 %1, %8 offset:16\n\t"
                 "ds_read_b128 %2, %8 offset:128\n\tds_read_b128 %3, %8 offset:144\n\t"
                 "ds_read_b128 %4, %8 offset:256\n\tds_read_b128 %5, %8 offset:272\n\t"
                 "ds_read_b128 %6, %8 offset:384\n\tds_read_b128 %7, %8 offset:400\n\t"
                 "s_waitcnt lgkmcnt(0)"
                 : "=&v"(v[0]), "=&v"(v[1]), "=&v"(v[2]), "=&v"(v[3]), "=&v"(v[4]),
                   "=&v"(v[5]), "=&v"(v[6]), "=&v"(v[7])
                 : "v"(a) : "memory");
}

// KC loads per lane (n <= 8 FS KC). Load k of wave w lands at
// buf[w FWAVE_F4 + 64 k + lane]; one more load (lanes 0..FR/2-1) brings the
// block's FR uo entries to buf[w FWAVE_F4 + 64 KC ...], entry r of the block at
// double index r there. Each wave reads back only its own loads, after its own wait.
// Columns past n lie past the A descriptor and load zeros (their t entry is
// zero and their sums are never stored). red: 2 x 8 waves x FR doubles.
// The host takes this path only when n lda 4 and m 8 are below 2^31 and
// 8 FS KC lda 4 below 2^32 (kr_fused_ok), so no byte offset below wraps.
template <int KC>
QRX_DEV void fused_pass(const KLoopArgs &K, const double *t, double coef, const double *uo,
                        double *un, double *lds, double *red, unsigned *voffs, double *sh) {
    const int64_t m = K.m, n = K.n, lda = K.lda;
    const int G = gridDim.x, wg = blockIdx.x;
    const int lane = lane_id_opaque() & 63, wv = lane_id_opaque() >> 6;
    const int q = lane % FQ, g = lane / FQ;
    constexpr int CW = FS * KC;                  // columns per wave
    float4 *bufs = reinterpret_cast<float4 *>(lds);
    const int c0 = wv * CW + g;                  // this lane's first column
    // this lane's entries of t (zero past n)
    double tv[KC];
#pragma unroll
    for (int k = 0; k < KC; ++k) tv[k] = (c0 + FS * k < n) ? t[c0 + FS * k] : 0.0;
    __syncthreads();                             // the previous phase is done with lds
    const int64_t nfull = m / FR;                // blocks with all FR rows inside
    const int64_t nsb = (m + FR - 1) / FR;
    // the workgroup's i-th block: group wg + (i / FG) G, block i % FG of it
    auto blk_of = [&](int64_t i) -> int64_t { return FG * (wg + (i / FG) * (int64_t)G) + (i % FG); };
    int64_t nb = 0;                              // full blocks of this workgroup
    {
        const int64_t nq = nfull / FG;           // whole groups of full blocks
        const int64_t groups = nq > wg ? (nq - wg + G - 1) / G : 0;
        nb = FG * groups;
        // leftover full blocks (nfull % FG) start group nq
        if ((nfull % FG) && nq % G == wg) nb += nfull % FG;
    }
    // column loads this wave issues per block (those with a lane inside the
    // matrix: the lowest column of load k is wv CW + FS k); with the uo load,
    // nk + 1 load instructions per block and wave
    int nk = 0;
    {
        const int64_t lo = (int64_t)__builtin_amdgcn_readfirstlane(wv) * CW;
        nk = lo >= n ? 0 : (int)((n - lo + FS - 1) / FS);
        if (nk > KC) nk = KC;
    }
    // byte offset of load k from the block's first row: (4q + (c0 + FS k) lda) 4;
    // the lane's part, and the uniform part of k
    const unsigned voff = (unsigned)((4 * q + (int64_t)c0 * lda) * 4);
    const unsigned kstep = (unsigned)(FS * lda * 4);
    const float *A = uniform_ptr(K.A);
    const double *U = uniform_ptr(uo);
    // slots of columns past n hold zeros in every buffer (whatever a load past
    // the descriptor leaves there), so their products with t are exact zeros
#pragma unroll
    for (int b = 0; b < FNBUF; ++b)
#pragma unroll
        for (int k = 0; k < KC; ++k)
            if (c0 + FS * k >= n)
                bufs[b * FBUF_F4 + wv * FWAVE_F4 + k * 64 + lane] = make_float4(0.f, 0.f, 0.f, 0.f);
    voffs[lane_id_opaque()] = voff;
    const unsigned avoff = lds_addr(voffs + lane_id_opaque());
    __asm__ volatile("" ::: "memory");
    wait_lgkm0();
    auto issue = [&](int64_t sb, int b) {
        float4 *mine = bufs + b * FBUF_F4 + wv * FWAVE_F4;
        // A from the block's first row on; columns past n read zeros
        const __amdgpu_buffer_rsrc_t ra = raw_rsrc(A + sb * FR, (n * lda - sb * FR) * 4);
        // the previous reads of this buffer are complete (each read group waits
        // for itself); keep the loads after them in the schedule
        __asm__ volatile("" ::: "memory");
        // the lane's offset comes back from LDS here (kept there rather than in a
        // register across the loop, where it would be spilled to scratch and its
        // reload would wait for the loads in flight)
        unsigned vb;
        asm volatile("ds_read_b32 %0, %1\n\ts_waitcnt lgkmcnt(0)"
                     : "=v"(vb) : "v"(avoff) : "memory");
#pragma unroll
        for (int k = 0; k < KC; ++k)
            if (k < nk)
                __builtin_amdgcn_raw_ptr_buffer_load_lds(ra, (lvoid *)(mine + k * 64), 16,
                                                         vb + (unsigned)k * kstep, 0, 0, 0);
        // lanes 0..FR/2-1 bring uo of the block's rows (one load instruction per wave)
        const __amdgpu_buffer_rsrc_t ru = raw_rsrc(U + sb * FR, FR * 8);
        if (lane < FR / 2)
            __builtin_amdgcn_raw_ptr_buffer_load_lds(ru, (lvoid *)(mine + KC * 64), 16,
                                                     (unsigned)(16 * lane), 0, 0, 0);
    };
    double acc[KC];
#pragma unroll
    for (int k = 0; k < KC; ++k) acc[k] = 0.0;
    double ss = 0.0;
    int par = 0;
    // one block from buffer b: A t by rows, u~, then A^T u~ into acc
    auto block = [&](int64_t sb, int b) {
        const float4 *mine = bufs + b * FBUF_F4 + wv * FWAVE_F4;
        const unsigned amine = lds_addr(mine + lane);
        const int64_t r = sb * FR + 4 * q;
        double p[4] = {0.0, 0.0, 0.0, 0.0};
        {
            f4v e[KC];
            lds_read_cols<KC>(amine, e);
#pragma unroll
            for (int k = 0; k < KC; ++k) {
                p[0] = fma((double)e[k].x, tv[k], p[0]);
                p[1] = fma((double)e[k].y, tv[k], p[1]);
                p[2] = fma((double)e[k].z, tv[k], p[2]);
                p[3] = fma((double)e[k].w, tv[k], p[3]);
            }
        }
        // over the wave's FS column groups (lanes q + FQ g), then over the 8 waves
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int o = FQ; o < 64; o <<= 1) p[i] += __shfl_xor(p[i], o);
        double *rd = red + par * (8 * FR);
        if (g == 0) {
#pragma unroll
            for (int i = 0; i < 4; ++i) rd[wv * FR + 4 * q + i] = p[i];
        }
        // one barrier per block (the next block writes the other half of red).
        // The row partials are LDS writes, complete at lgkmcnt(0); a plain
        // barrier publishes them without waiting for the loads in flight.
        __asm__ volatile("" ::: "memory");
        wait_lgkm0();
        __builtin_amdgcn_s_barrier();
        __asm__ volatile("" ::: "memory");
        par ^= 1;
        double uu[4];
        {
            // wave w's partial of row 4q + i: pair 2 (w % 4) + i / 2, entry i % 2
            // of the read of waves 4 (w / 4) ..; summed in wave order
            double sacc[4];
            const unsigned ar = lds_addr(rd + 4 * q);
            {
                d2v pr[8];
                lds_read_red4(ar, pr);
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    sacc[i] = pr[i / 2][i % 2];
#pragma unroll
                    for (int w = 1; w < 4; ++w) sacc[i] += pr[2 * w + i / 2][i % 2];
                }
            }
            {
                d2v pr[8];
                lds_read_red4(ar + 4 * FR * 8, pr);
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int w = 0; w < 4; ++w) sacc[i] += pr[2 * w + i / 2][i % 2];
            }
            d2v u0, u1;
            lds_read_d4(lds_addr(reinterpret_cast<const double *>(mine + KC * 64) + 4 * q), u0, u1);
            const double uol[4] = {u0.x, u0.y, u1.x, u1.y};
#pragma unroll
            for (int i = 0; i < 4; ++i) uu[i] = (r + i < m) ? fma(-coef, uol[i], sacc[i]) : 0.0;
        }
        if (wv == 0 && g == 0) {
#pragma unroll
            for (int i = 0; i < 4; ++i)
                if (r + i < m) {
                    un[r + i] = uu[i];
                    ss = fma(uu[i], uu[i], ss);
                }
        }
        {
            f4v e[KC];
            lds_read_cols<KC>(amine, e);
#pragma unroll
            for (int k = 0; k < KC; ++k) {
                double v = acc[k];
                v = fma((double)e[k].x, uu[0], v);
                v = fma((double)e[k].y, uu[1], v);
                v = fma((double)e[k].z, uu[2], v);
                v = fma((double)e[k].w, uu[3], v);
                acc[k] = v;
            }
        }
    };
    // full blocks through FNBUF buffers: block i + FNBUF - 1 is issued before
    // block i is reduced; the wait lets the loads of the blocks issued after
    // block i stay in flight (nk + 1 instructions each; older stores of wave 0
    // are waited for as well, which only makes it stricter)
    for (int64_t i = 0; i < FNBUF - 1 && i < nb; ++i) issue(blk_of(i), (int)i);
    for (int64_t i = 0; i < nb; ++i) {
        if (i + FNBUF - 1 < nb) issue(blk_of(i + FNBUF - 1), (int)((i + FNBUF - 1) % FNBUF));
        const int64_t after = nb - 1 - i < FNBUF - 1 ? nb - 1 - i : FNBUF - 1;
        wait_vm_rt((int)after * (nk + 1));
        __asm__ volatile("" ::: "memory");
        block(blk_of(i), (int)(i % FNBUF));
    }
    // the last, partial block (m % FR rows) goes to the workgroup of its group
    if (nsb > nfull && (nfull / FG) % G == wg) {
        const int64_t sb = nfull;
        const int b = (int)(nb % FNBUF);
        float4 *mine = bufs + b * FBUF_F4 + wv * FWAVE_F4;
        const int64_t r = sb * FR + 4 * q;
        wait_vm<0>();
        __asm__ volatile("" ::: "memory");
#pragma unroll
        for (int k = 0; k < KC; ++k) {
            const int64_t c = c0 + FS * k;
            const float *col = A + (c < n ? c : n - 1) * lda;
            float4 e;
            e.x = r < m ? col[r] : 0.f;
            e.y = r + 1 < m ? col[r + 1] : 0.f;
            e.z = r + 2 < m ? col[r + 2] : 0.f;
            e.w = r + 3 < m ? col[r + 3] : 0.f;
            mine[k * 64 + lane] = e;
        }
        if (lane < FQ) {
            double *ul = reinterpret_cast<double *>(mine + KC * 64) + 4 * lane;
            const int64_t ru = sb * FR + 4 * lane;
#pragma unroll
            for (int i = 0; i < 4; ++i) ul[i] = ru + i < m ? U[ru + i] : 0.0;
        }
        __asm__ volatile("" ::: "memory");
        wait_lgkm0();
        __asm__ volatile("" ::: "memory");
        block(sb, b);
    }
    // acc over the FQ row groups of the wave (lanes FQ g + q, fixed butterfly order)
#pragma unroll
    for (int k = 0; k < KC; ++k)
#pragma unroll
        for (int o = 1; o < FQ; o <<= 1) acc[k] += __shfl_xor(acc[k], o);
    if (q == 0) {
#pragma unroll
        for (int k = 0; k < KC; ++k)
            if (c0 + FS * k < n) K.pf[(c0 + FS * k) * G + wg] = acc[k];
    }
    wg_partial(ss, K.ssqA + wg, sh);
}

QRX_DEV void ph_fused(const KLoopArgs &K, const double *t, double coef, const double *uo,
                      double *un, double *lds, double *red, unsigned *voffs, double *sh) {
    const int64_t kc = (K.n + 8 * FS - 1) / (8 * FS);
    if (kc <= 1) fused_pass<1>(K, t, coef, uo, un, lds, red, voffs, sh);
    else if (kc <= 2) fused_pass<2>(K, t, coef, uo, un, lds, red, voffs, sh);
    else if (kc <= 4) fused_pass<4>(K, t, coef, uo, un, lds, red, voffs, sh);
    else fused_pass<8>(K, t, coef, uo, un, lds, red, voffs, sh);
}


// z[j] = sum over the workgroups of pf[j G + w] (j < n), one wave per column,
// lanes over the workgroups in a fixed order.
QRX_DEV void ph_combine_f(const KLoopArgs &K) {
    const int64_t n = K.n;
    const int G = gridDim.x;
    constexpr int NW = LT / 64;
    const int lane = lane_id_opaque() & 63, wv = lane_id_opaque() >> 6;
    const unsigned nvb = (unsigned)((n + NW - 1) / NW);
    for (unsigned vb = blockIdx.x; vb < nvb; vb += gridDim.x) {
        const int64_t j = (int64_t)vb * NW + wv;
        if (j < n) {
            const double *pj = K.pf + j * G;
            double s = 0.0;
            for (int w = lane; w < G; w += 64) s += pj[w];
            s = wave_sum_d(s);
            if (lane == 0) K.z[j] = s;
        }
    }
}

__global__ __launch_bounds__(LT, 1) void krylov_loop_kernel(KLoopArgs K) {
    __shared__ __align__(16) double us[US_DOUBLES];   // GEMV-T slice; GEMV-N staging; one-pass buffers
    __shared__ double sh[LT];     // reductions
    __shared__ __align__(16) double fred[2 * 8 * FR];   // row partials of the one-pass products
    __shared__ unsigned fvoff[LT];                      // lane offsets of the one-pass loads
    __shared__ int sflag;
    __shared__ long long prof[2 * KP_COUNT];   // per-phase ticks and counts (workgroup 0)
    const unsigned G = gridDim.x;
    const int64_t m = K.m, n = K.n, np = K.np;
    const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
    const bool timed = K.prof != nullptr && lead;
    qrx_lls_info *info = K.info;
    long long tprev = 0;
    if (timed) {
        for (int i = 0; i < 2 * KP_COUNT; ++i) prof[i] = 0;
        tprev = wall_clock64();
    }
    // a barrier that also closes phase `ph` in the timing record
    auto bar_ph = [&](int ph) -> bool {
        const bool ok = grid_barrier(K.bar, G, &sflag);
        if (timed) {
            const long long now = wall_clock64();
            prof[ph] += now - tprev;
            prof[KP_COUNT + ph] += 1;
            tprev = now;
        }
        return ok;
    };
    auto flush_prof = [&]() {
        if (timed)
            for (int i = 0; i < 2 * KP_COUNT; ++i) K.prof[i] = prof[i];
    };
    auto fail_sync = [&]() {
        if (lead) {
            info->status = QRX_ESYNC;
            info->accepted = 0;
        }
        flush_prof();
    };

    if (lead) memset(info, 0, sizeof(*info));
    // ---- inputs already flagged by the scan / factorisation
    const int flags = K.flags[0];
    const double normA = K.normA[0];
    if (flags & 3) {
        if (lead) {
            info->status = (flags & 1) ? QRX_ENONFINITE : QRX_ESINGULAR;
            info->normA_F = normA;
        }
        flush_prof();
        return;
    }
    // rho ~ ||R||_2 for the stopping trigger: 1 for the identity, else the largest
    // column norm of A (a lower bound of ||A||_2 = ||R||_2)
    double rho = 1.0;
    if (K.X) {
        double mx = 0.0;
        for (int64_t j = threadIdx.x; j < n; j += LT) mx = fmax(mx, K.colss[j]);
        sh[threadIdx.x] = mx;
        __syncthreads();
        for (int o = LT / 2; o > 0; o >>= 1) {
            if ((int)threadIdx.x < o) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + o]);
            __syncthreads();
        }
        rho = sqrt(sh[0]);
        __syncthreads();
    }
    const double trig = normA > 0.0 ? rho / normA : 1.0;
    const double tol = K.tol;

    // ||b|| for the compatible-system test
    ph_ssq(K.b, m, K.ssqA, sh);
    if (!bar_ph(KP_INIT)) return fail_sync();
    const double bnorm = sqrt(wg_sum(K.ssqA, nblk(m), sh));

    // certification of the current x: rc = b - A x (double-double), z = A^T rc,
    // eta_F = ||z|| / (||A||_F ||rc||), compatible ratio, score = min of the two
    double rnorm = 0.0, eta = 0.0, score = 0.0;
    // The squares of the last phase (x in [0, nblk(np)), z after them) go to
    // ssqB: the phase after a certification (a restart) writes ssqA while
    // another workgroup may still be summing these.
    auto certify = [&]() -> bool {
        ph_gemv_n(K, K.x, K.pn, K.pn2, 1, us);
        if (!bar_ph(KP_CERT_GEMV_N)) return false;
        ph_resid(K, K.ssqA, sh);
        if (!bar_ph(KP_CERT_RESID)) return false;
        rnorm = sqrt(wg_sum(K.ssqA, nblk(m), sh));
        ph_gemv_t(K, K.rc, K.pt, us);
        if (!bar_ph(KP_CERT_GEMV_T)) return false;
        double *sz = K.ssqB + nblk(np);
        ph_combine_n(K, sz, sh);
        ph_ssq(K.x, np, K.ssqB, sh);
        if (!bar_ph(KP_CERT_COMBINE)) return false;
        const double znorm = sqrt(wg_sum(sz, (n + LT / 64 - 1) / (LT / 64), sh));
        const double xnorm = sqrt(wg_sum(K.ssqB, nblk(np), sh));
        eta = (rnorm > 0.0 && normA > 0.0) ? znorm / (normA * rnorm) : 0.0;
        const double den = normA * xnorm + bnorm;
        const double s1 = den > 0.0 ? K.cscale * (rnorm / den) : 0.0;
        score = fmin(eta, s1);
        return true;
    };

    if (!certify()) return fail_sync();
    const double eta_start = eta;
    double best = score, best_eta = eta, best_rn = rnorm;
    ph_each(np, [&](int64_t j) { K.xbest[j] = K.x[j]; });
    auto keep_if_better = [&]() {
        if (score < best) {
            best = score;
            best_eta = eta;
            best_rn = rnorm;
            ph_each(np, [&](int64_t j) { K.xbest[j] = K.x[j]; });
        }
    };

    int iters = 0, outers = 0, no_gain = 0;
    double prev = best, gam = 1.0;
    // LSQR state; the x and d updates of an iteration are applied by the next
    // one's first phase (pend), or by flush_update before x is read
    double alpha = 0.0, beta = 0.0, rhobar = 0.0, phibar = 0.0, dcoef = 0.0;
    double p_dcoef = 0.0, p_xcoef = 0.0;
    bool pend = false, p_first = true;
    double *tbuf[2] = {K.t, K.t2};
    int tsel = 0;
    const double *usrc = K.rc;   // u~_old of the one-pass products
    auto flush_update = [&]() -> bool {
        const double *tp = tbuf[tsel];
        const double pdc = p_dcoef, pxc = p_xcoef;
        const bool pfst = p_first;
        ph_each(np, [&](int64_t j) {
            const double dj = pfst ? tp[j] : fma(-pdc, K.d[j], tp[j]);
            K.d[j] = dj;
            x_update(K, j, pxc, dj);
        });
        pend = false;
        return bar_ph(KP_UPDATE);
    };
    // CGLS state
    double gamma = 0.0;
    const unsigned ntri = tri_vblocks(np, G);
    const int64_t mx_mn = m > n ? m : n;

    while (best > tol && iters < K.max_iter) {
        ++outers;
        // ---- restart on the certified residual rc and z = A^T rc
        if (K.method == 0) {
            // u = rc (beta = ||rc||); v~ = X^T z / beta, alpha = ||v~|| (v = v~ / alpha
            // is formed by the next t = X v phase)
            beta = rnorm;
            phibar = rnorm;
            const double ib = 1.0 / beta;
            // the one-pass products read u~_old = rc where it is (certification
            // rewrites rc only after a later iteration has moved u~ on)
            if (K.fused) usrc = K.rc;
            else ph_each(m, [&](int64_t i) { K.u[i] = K.rc[i]; });
            ph_tri(K, K.X, K.z, 1, 1.0, K.ssqA, sh, [&](int64_t c, double val) {
                const double w = ib * val;
                K.v[c] = w;
                K.xlo[c] = 0.0;
                return w * w;
            });
            if (!bar_ph(KP_RESTART)) return fail_sync();
            alpha = sqrt(wg_sum(K.ssqA, ntri, sh));
            rhobar = alpha;
            dcoef = 0.0;
            pend = false;
        } else {
            // r = rc; s = X^T z (in vt), p = s (in v), gamma = ||s||^2
            ph_each(m, [&](int64_t i) { K.r[i] = K.rc[i]; });
            ph_tri(K, K.X, K.z, 1, 1.0, K.ssqA, sh, [&](int64_t c, double val) {
                K.vt[c] = val;
                K.v[c] = val;
                K.xlo[c] = 0.0;
                return val * val;
            });
            if (!bar_ph(KP_RESTART)) return fail_sync();
            gamma = wg_sum(K.ssqA, ntri, sh);
        }
        bool first = true;
        double best_est = HUGE_VAL;
        int kin = 0, last_new = 0, next_check = 10;
        while (iters < K.max_iter && best > tol) {
            ++iters;
            ++kin;
            double est;
            if (K.method == 0) {
                // v = v~ / alpha (into vn) and t = X v; the x and d updates owed by
                // the previous iteration use its t (the other t buffer)
                const double ia = alpha > 0.0 ? 1.0 / alpha : 0.0;
                double *tn = tbuf[tsel ^ 1];
                const double *tp = tbuf[tsel];
                const double pdc = p_dcoef, pxc = p_xcoef;
                const bool pfst = p_first, pd = pend;
                ph_each(np, [&](int64_t j) {
                    K.vn[j] = ia * K.v[j];
                    if (pd) {
                        const double dj = pfst ? tp[j] : fma(-pdc, K.d[j], tp[j]);
                        K.d[j] = dj;
                        x_update(K, j, pxc, dj);
                    }
                });
                ph_tri(K, K.Xt, K.v, 0, ia, nullptr, sh, [&](int64_t c, double val) {
                    tn[c] = val;
                    return 0.0;
                });
                tsel ^= 1;
                pend = false;
                if (!bar_ph(KP_TRMV_N)) return fail_sync();
                if (K.fused) {
                    // u~ = A t - (alpha / beta) u~_old and z = A^T u~ in one pass
                    // over A; u~ alternates between two buffers
                    double *un = (usrc == K.u) ? K.u2 : K.u;
                    ph_fused(K, tn, alpha / beta, usrc, un, us, fred, fvoff, sh);
                    usrc = un;
                    if (!bar_ph(KP_FUSED)) return fail_sync();
                    beta = sqrt(wg_sum(K.ssqA, G, sh));
                    ph_combine_f(K);
                    if (!bar_ph(KP_COMBINE_N)) return fail_sync();
                } else {
                    ph_gemv_n(K, tn, K.pn, nullptr, 0, us);
                    if (!bar_ph(KP_GEMV_N)) return fail_sync();
                    // u~ = A t - (alpha / beta) u~_old, beta = ||u~||
                    ph_combine_m(K, alpha / beta, K.u, K.u, K.ssqA, sh);
                    if (!bar_ph(KP_COMBINE_M)) return fail_sync();
                    beta = sqrt(wg_sum(K.ssqA, nblk(m), sh));
                    ph_gemv_t(K, K.u, K.pt, us);
                    if (!bar_ph(KP_GEMV_T)) return fail_sync();
                    ph_combine_n(K, nullptr, sh);
                    if (!bar_ph(KP_COMBINE_N)) return fail_sync();
                }
                // v~ = X^T z / beta - beta v; alpha = ||v~||
                const double ib = 1.0 / beta, bb = beta;
                ph_tri(K, K.X, K.z, 1, 1.0, K.ssqA, sh, [&](int64_t c, double val) {
                    const double w = fma(-bb, K.vn[c], ib * val);
                    K.v[c] = w;
                    return w * w;
                });
                if (!bar_ph(KP_TRMV_T)) return fail_sync();
                alpha = sqrt(wg_sum(K.ssqA, ntri, sh));
                // Givens step (Paige & Saunders); d = t - (theta/rho) d and
                // x += (phi/rho) d are owed to the next t = X v phase
                const double rh = hypot(rhobar, beta);
                const double c = rhobar / rh, s = beta / rh;
                const double theta = s * alpha;
                rhobar = -c * alpha;
                const double phi = c * phibar;
                phibar = s * phibar;
                est = alpha * fabs(c);   // ||B^T r|| / ||r||
                pend = true;
                p_first = first;
                p_dcoef = dcoef;
                p_xcoef = phi / rh;
                dcoef = theta / rh;
                first = false;
            } else {
                // Alg. 5: t = X p; q = A t; alpha = gamma / ||q||^2; x += alpha t;
                // r -= alpha q; s = X^T A^T r; beta = ||s||^2 / gamma; p = s + beta p
                ph_tri(K, K.Xt, K.v, 0, 1.0, nullptr, sh, [&](int64_t c, double val) {
                    K.t[c] = val;
                    return 0.0;
                });
                if (!bar_ph(KP_TRMV_N)) return fail_sync();
                ph_gemv_n(K, K.t, K.pn, nullptr, 0, us);
                if (!bar_ph(KP_GEMV_N)) return fail_sync();
                ph_combine_m(K, 0.0, nullptr, K.q, K.ssqA, sh);
                if (!bar_ph(KP_COMBINE_M)) return fail_sync();
                const double delta = wg_sum(K.ssqA, nblk(m), sh);
                const double a = delta > 0.0 ? gamma / delta : 0.0;
                {
                    const unsigned nvb = nblk(mx_mn);
                    for (unsigned vb = blockIdx.x; vb < nvb; vb += G) {
                        const int64_t i = (int64_t)vb * LT + lane_id_opaque();
                        if (i < n) x_update(K, i, a, K.t[i]);
                        double v2 = 0.0;
                        if (i < m) {
                            const double v = fma(-a, K.q[i], K.r[i]);
                            K.r[i] = v;
                            v2 = v * v;
                        }
                        wg_partial(v2, K.ssqB + vb, sh);
                    }
                }
                if (!bar_ph(KP_UPDATE)) return fail_sync();
                const double rss = wg_sum(K.ssqB, nblk(mx_mn), sh);
                ph_gemv_t(K, K.r, K.pt, us);
                if (!bar_ph(KP_GEMV_T)) return fail_sync();
                ph_combine_n(K, nullptr, sh);
                if (!bar_ph(KP_COMBINE_N)) return fail_sync();
                ph_tri(K, K.X, K.z, 1, 1.0, K.ssqA, sh, [&](int64_t c, double val) {
                    K.vt[c] = val;
                    return val * val;
                });
                if (!bar_ph(KP_TRMV_T)) return fail_sync();
                const double gnew = wg_sum(K.ssqA, ntri, sh);
                const double cb = gamma > 0.0 ? gnew / gamma : 0.0;
                gamma = gnew;
                const double nr = sqrt(rss);
                est = nr > 0.0 ? sqrt(gnew) / nr : 0.0;   // ||R^{-T} A^T r|| / ||r||
                ph_each(np, [&](int64_t j) { K.v[j] = fma(cb, K.v[j], K.vt[j]); });
                if (!bar_ph(KP_UPDATE)) return fail_sync();
            }
            // ---- decisions (identical in every workgroup)
            if (est < 0.99 * best_est) {
                best_est = est;
                last_new = kin;
            }
            const bool finite = isfinite(est);
            const int stall_len = kin / 2 > 100 ? kin / 2 : 100;
            const bool cg_stall =
                K.method == 1 && ((kin - last_new) > stall_len || est > 100.0 * best_est);
            const bool leave = !finite || est * trig <= tol * gam || cg_stall ||
                               iters >= K.max_iter;
            // periodic check of the true residual without restarting: the
            // preconditioned estimate can stay far above tol once eta_F has
            // reached its floor (R^{-T} amplifies rounding-level residuals)
            const bool check = !leave && kin >= next_check;
            if ((leave || check) && pend) {
                if (!flush_update()) return fail_sync();
            }
            if (leave) break;
            if (check) {
                next_check = kin + (iters / 8 > 10 ? iters / 8 : 10);
                if (!certify()) return fail_sync();
                keep_if_better();
            }
        }
        if (best <= tol) break;
        // ---- certify; keep the best iterate, or go back to it
        if (!certify()) return fail_sync();
        if (score < best) {
            keep_if_better();
        } else {
            ph_each(np, [&](int64_t j) {
                K.x[j] = K.xbest[j];
                K.xlo[j] = 0.0;
            });
            if (!bar_ph(KP_CERTIFY)) return fail_sync();
            if (!certify()) return fail_sync();
        }
        no_gain = (best > 0.5 * prev) ? no_gain + 1 : 0;
        prev = best;
        if (no_gain >= 3) break;
        if (best > tol) gam = fmax(0.01, 0.5 * gam);
    }
    // the returned x is the best certified iterate (same entries as the copies above)
    ph_each(np, [&](int64_t j) {
        if (j < n) K.x_user[j] = K.xbest[j];
    });
    if (lead) {
        info->status = best <= tol ? QRX_OK : QRX_ENOCONV;
        info->accepted = best <= tol ? (best_eta <= tol ? 1 : 2) : 0;
        info->iters = iters;
        info->restarts = outers > 0 ? outers - 1 : 0;
        info->eta_F = best_eta;
        info->resid_norm = best_rn;
        info->normA_F = normA;
        info->eta_start = eta_start;
        info->score = best;
    }
    flush_prof();
}

}  // namespace

bool kr_fused_ok(int64_t m, int64_t n, int64_t lda) {
    if (n < 1 || n > kr_fused_max_n) return false;
    const int64_t kc = (n + 8 * FS - 1) / (8 * FS);
    const int64_t KC = kc <= 1 ? 1 : kc <= 2 ? 2 : kc <= 4 ? 4 : 8;
    return (double)n * (double)lda * 4.0 < 2147483648.0 && (double)m * 8.0 < 2147483648.0 &&
           (double)(8 * FS * KC) * (double)lda * 4.0 < 4294967296.0;
}

size_t kr_loop_ssq_doubles(int64_t m, int64_t np) {
    const int64_t len = (m > np ? m : np);
    const int64_t a = (len + LT - 1) / LT;              // elementwise virtual blocks
    const int64_t b = np / 2 + 1;                        // triangular products: up to one per column pair
    int64_t c = a > b ? a : b;
    if (c < kr_max_grid) c = kr_max_grid;               // one-pass products: one per workgroup
    // a certification's squares of x and z, side by side
    const int64_t d = (np + LT - 1) / LT + (np + LT / 64 - 1) / (LT / 64);
    if (c < d) c = d;
    return (size_t)(c + 1);
}

int kr_loop_grid(int device, int64_t m, int64_t n) {
    int cus = 0, per = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess ||
        cus < 1)
        cus = 1;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, krylov_loop_kernel, LT, 0) !=
            hipSuccess ||
        per < 1)
        per = 1;
    // one workgroup per CU: a grid barrier costs time in proportion to the
    // number of workgroups that arrive at it
    per = 1;
    // no more workgroups than the widest phase has virtual blocks
    const int64_t np = (n + kTrsvBlock - 1) / kTrsvBlock * kTrsvBlock;
    int64_t want = ((m + 4 * LT - 1) / (4 * LT)) * kr_gemv_n_splits(m, n);
    const int64_t gt = ((n + GT_C - 1) / GT_C) * kr_gemv_t_splits(m);
    const int64_t tri = (np / 2 + LT / 64 - 1) / (LT / 64);
    const int64_t el = ((m > np ? m : np) + LT - 1) / LT;
    for (int64_t v : {gt, tri, el})
        if (v > want) want = v;
    int64_t g = (int64_t)per * cus;
    if (want < g) g = want;
    if (g > kr_max_grid) g = kr_max_grid;
    return (int)(g < 1 ? 1 : g);
}

hipError_t kr_loop(hipStream_t s, const KLoopArgs &a, int grid) {
    hipLaunchKernelGGL(krylov_loop_kernel, dim3((unsigned)grid), dim3(LT), 0, s, a);
    return hipGetLastError();
}

}  // namespace qrx
