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
//   u~ = A t - alpha u        (GEMV-N partials over column splits, then summed)
//   z = A^T u~                (GEMV-T partials over row splits, then summed)
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
// bar[0] = arrivals, bar[1] = generation, bar[2] = abort flag; all zero at launch.
// Thread 0 releases the workgroup's writes (agent scope) with its arrival; the
// last arrival resets the count and bumps the generation; the others poll the
// generation. A poll limit or an abort raised by another workgroup ends the
// wait with `false`, so every workgroup leaves even if the launch was not
// co-resident.
QRX_DEV bool grid_barrier(unsigned *bar, unsigned nwg, int *sflag) {
    __syncthreads();
    if (threadIdx.x == 0) {
        int ok = 1;
        const unsigned g = __hip_atomic_load(bar + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const unsigned prev =
            __hip_atomic_fetch_add(bar, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        if (prev == nwg - 1) {
            __hip_atomic_store(bar, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(bar + 1, g + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            unsigned polls = 0;
            while (__hip_atomic_load(bar + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == g) {
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
        const int64_t r = (rb * LT + threadIdx.x) * 4;
        const int64_t j0 = s * K.cchunk;
        const int64_t j1 = (j0 + K.cchunk < n) ? j0 + K.cchunk : n;
        const bool act = r < m;
        const bool v4 = K.vec && (r + 3 < m);
        double h[4] = {0, 0, 0, 0}, l[4] = {0, 0, 0, 0};
        for (int64_t c0 = j0; c0 < j1; c0 += GN_STAGE) {
            const int64_t c1 = (c0 + GN_STAGE < j1) ? c0 + GN_STAGE : j1;
            __syncthreads();
            for (int64_t j = c0 + threadIdx.x; j < c1; j += LT) stage[j - c0] = in[j];
            __syncthreads();
            if (!act) continue;
            int64_t j = c0;
            if (v4 && !dd) {
                constexpr int GU = 16;   // column loads in flight per thread
                for (; j + GU <= c1; j += GU) {
                    float4 q[GU];
#pragma unroll
                    for (int u = 0; u < GU; ++u)
                        q[u] = *reinterpret_cast<const float4 *>(K.A + (j + u) * K.lda + r);
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
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
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
            for (int i = threadIdx.x; i < GT_R; i += LT) us[i] = (i < cnt) ? in[rs + i] : 0.0;
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
        const int64_t r = (int64_t)vb * LT + threadIdx.x;
        double v2 = 0.0;
        if (r < m) {
            double s = 0.0;
            for (int q = 0; q < K.splits_n; ++q) s += K.pn[(int64_t)q * m + r];
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
        const int64_t r = (int64_t)vb * LT + threadIdx.x;
        double v2 = 0.0;
        if (r < m) {
            double h = K.b[r], l = 0.0;
            for (int q = 0; q < K.splits_n; ++q) {
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
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
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
        const int64_t j = (int64_t)vb * LT + threadIdx.x;
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
        const int64_t j = (int64_t)vb * LT + threadIdx.x;
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
    for (; i < i1; i += 64) acc = fma(col[i], in[i], acc);
    return wave_sum_d(acc);
}

// Triangular products with one wave per output entry; each wave takes the pair
// (c, np-1-c) so the work per wave is balanced. Virtual block = one pair per wave.
//   upper = 1: out[c] = sum_{i <= c} M[i, c] in[i]   (M = X: out = X^T in)
//   upper = 0: out[c] = sum_{i >= c} M[i, c] in[i]   (M = X^T: out = X in)
// each times `scale`. M == null stands for the identity. The epilogue receives (c, value) on lane 0
// and returns the entry's contribution to the virtual block's ssq partial.
template <class E>
QRX_DEV void ph_tri(const KLoopArgs &K, const double *M, const double *in, int upper,
                    double scale, double *ssq, double *sh, E epi) {
    const int64_t np = K.np;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    constexpr int NW = LT / 64;
    const int64_t npairs = np / 2;
    const int64_t nvb = (npairs + NW - 1) / NW;
    for (int64_t vb = blockIdx.x; vb < nvb; vb += gridDim.x) {
        const int64_t p = vb * NW + wv;
        double e2 = 0.0;
        if (p < npairs) {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int64_t c = h == 0 ? p : np - 1 - p;
                double val;
                if (M == nullptr) {
                    val = in[c];
                } else {
                    const double *col = M + c * np;
                    val = upper ? col_dot(col, in, 0, c + 1, lane) : col_dot(col, in, c, np, lane);
                }
                val *= scale;
                if (lane == 0) e2 += epi(c, val);
            }
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

QRX_DEV unsigned tri_vblocks(int64_t np) { return (unsigned)((np / 2 + LT / 64 - 1) / (LT / 64)); }

__global__ __launch_bounds__(LT, 1) void krylov_loop_kernel(KLoopArgs K) {
    __shared__ double us[GT_R];   // GEMV-T slice; GEMV-N staging
    __shared__ double sh[LT];     // reductions
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
    auto certify = [&]() -> bool {
        ph_gemv_n(K, K.x, K.pn, K.pn2, 1, us);
        if (!bar_ph(KP_CERTIFY)) return false;
        ph_resid(K, K.ssqA, sh);
        if (!bar_ph(KP_CERTIFY)) return false;
        rnorm = sqrt(wg_sum(K.ssqA, nblk(m), sh));
        ph_gemv_t(K, K.rc, K.pt, us);
        if (!bar_ph(KP_CERTIFY)) return false;
        ph_combine_n(K, K.ssqA, sh);
        ph_ssq(K.x, np, K.ssqB, sh);
        if (!bar_ph(KP_CERTIFY)) return false;
        const double znorm = sqrt(wg_sum(K.ssqA, (n + LT / 64 - 1) / (LT / 64), sh));
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
    auto flush_update = [&]() -> bool {
        const double *tp = tbuf[tsel];
        const double pdc = p_dcoef, pxc = p_xcoef;
        const bool pfst = p_first;
        ph_each(np, [&](int64_t j) {
            const double dj = pfst ? tp[j] : fma(-pdc, K.d[j], tp[j]);
            K.d[j] = dj;
            K.x[j] = fma(pxc, dj, K.x[j]);
        });
        pend = false;
        return bar_ph(KP_UPDATE);
    };
    // CGLS state
    double gamma = 0.0;
    const unsigned ntri = tri_vblocks(np);
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
            ph_each(m, [&](int64_t i) { K.u[i] = K.rc[i]; });
            ph_tri(K, K.X, K.z, 1, 1.0, K.ssqA, sh, [&](int64_t c, double val) {
                const double w = ib * val;
                K.v[c] = w;
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
                        K.x[j] = fma(pxc, dj, K.x[j]);
                    }
                });
                ph_tri(K, K.Xt, K.v, 0, ia, nullptr, sh, [&](int64_t c, double val) {
                    tn[c] = val;
                    return 0.0;
                });
                tsel ^= 1;
                pend = false;
                if (!bar_ph(KP_TRMV_N)) return fail_sync();
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
                        const int64_t i = (int64_t)vb * LT + threadIdx.x;
                        if (i < n) K.x[i] = fma(a, K.t[i], K.x[i]);
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
            ph_each(np, [&](int64_t j) { K.x[j] = K.xbest[j]; });
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

size_t kr_loop_ssq_doubles(int64_t m, int64_t np) {
    const int64_t len = (m > np ? m : np);
    const int64_t a = (len + LT - 1) / LT;              // elementwise virtual blocks
    const int64_t b = (np + LT / 64 - 1) / (LT / 64);   // per-column (wave) virtual blocks
    return (size_t)((a > b ? a : b) + 1);
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
    return (int)(g < 1 ? 1 : g);
}

hipError_t kr_loop(hipStream_t s, const KLoopArgs &a, int grid) {
    hipLaunchKernelGGL(krylov_loop_kernel, dim3((unsigned)grid), dim3(LT), 0, s, a);
    return hipGetLastError();
}

}  // namespace qrx
