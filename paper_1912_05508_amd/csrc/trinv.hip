// The preconditioner of the Krylov iteration as an explicit FP64 inverse.
//
// Right preconditioning applies R^{-1} and R^{-T} twice per iteration
// (Sec. 3.2.3, Alg. 5) with the same R throughout, so X = R^{-1} is formed
// once (FP64, from the FP32 R) and each application is one triangular
// matrix-vector product: a bandwidth-bound stream over the n^2/2 entries of X
// instead of a chain of dependent triangular-solve steps. X and X^T are
// applied by the same matrix, so the preconditioned operator and its
// transpose stay exact transposes of each other.
//
// X is built by recursive block inversion on a 64-column grid:
//   [R11 R12; 0 R22]^{-1} = [X11, -X11 R12 X22; 0, X22],
// leaves are the 64 x 64 diagonal blocks (inverted by back substitution in
// FP64), and each node costs two triangular-times-dense FP64 products whose
// K ranges skip the zero triangle. Beyond n, R is taken as the identity, so X
// is the identity there and padded vector entries stay zero.
#include "qrx_internal.hpp"
#include "krylov.hpp"

#include <cstring>
#include <vector>

namespace qrx {

constexpr int IB = 64;     // leaf block
constexpr int TT = 256;    // threads

QRX_DEV double Rpad(const float *R, int64_t ldr, int64_t n, int64_t i, int64_t j) {
    if (i < n && j < n) return (double)R[i + j * ldr];
    return (i == j) ? 1.0 : 0.0;
}

// X[o:o+64, o:o+64] = inverse of R[o:o+64, o:o+64] (identity-padded), o = 64 b.
// One thread per column c: back substitution X(:, c) = R^{-1} e_c.
__global__ __launch_bounds__(IB) void inv_diag_kernel(int64_t n, const float *__restrict__ R,
                                                      int64_t ldr, double *__restrict__ X,
                                                      int64_t ldx) {
    __shared__ double Rs[IB * (IB + 1)];
    __shared__ double Xs[IB * (IB + 1)];
    const int64_t o = (int64_t)blockIdx.x * IB;
    const int c = threadIdx.x;
    for (int i = 0; i < IB; ++i) Rs[i + c * (IB + 1)] = Rpad(R, ldr, n, o + i, o + c);
    __syncthreads();
    for (int i = IB - 1; i >= 0; --i) {
        double v = 0.0;
        if (i <= c) {
            double s = (i == c) ? 1.0 : 0.0;
            for (int l = i + 1; l <= c; ++l) s -= Rs[i + l * (IB + 1)] * Xs[l + c * (IB + 1)];
            const double d = Rs[i + i * (IB + 1)];
            v = (d != 0.0) ? s / d : 0.0;
        }
        Xs[i + c * (IB + 1)] = v;
    }
    for (int i = 0; i < IB; ++i) X[(o + i) + (o + c) * ldx] = Xs[i + c * (IB + 1)];
}

// C (M x N, ldc) = alpha * A B, FP64 accumulation, M and N multiples of 64, K
// a multiple of 16. A is FP32 or FP64 (element (i, k) at A[i + k*lda], zero
// where i >= arl or k >= acl); B is FP64 (B[k + j*ldb]). TRI = 1: B is upper
// triangular (k <= j contributes); TRI = 2: A is upper triangular (k >= i
// contributes). On the FP64 matrix cores (v_mfma_f64_16x16x4f64: A operand
// lane l holds A[l % 16][l / 16], B operand B[l / 16][l % 16], result register
// v of lane l holds D[4 v + l / 16][l % 16]): 64 x 64 tile per workgroup, wave
// w the 32 x 32 quarter (rows 32 (w % 2), columns 32 (w / 2)) as 2 x 2 blocks
// of 16 x 16; K in stages of 16 through LDS, the next stage's loads in
// registers meanwhile. Each lane reads one LDS value per operand and block for
// 1024 FMAs per instruction, where 4 x 4 register tiles on the vector units
// read two values per two FMAs (the inverse at n = 8192, one launch per node
// and product: 11.8 ms against 13.4 ms with those).
typedef double tgd4 __attribute__((ext_vector_type(4)));
template <class TA, int TRI>
QRX_DEV void tri_tile(int64_t M, int64_t K, const TA *__restrict__ A, int64_t lda, int64_t arl,
                      int64_t acl, const double *__restrict__ B, int64_t ldb,
                      double *__restrict__ C, int64_t ldc, double alpha, int64_t tile) {
    constexpr int BT = 64, BK = 16, LS = BT + 4;
    constexpr int AQ = BT * BK / TT;               // A (and B) elements each thread stages
    __shared__ __align__(16) double As[BK * LS];   // As[k][i]
    __shared__ __align__(16) double Bs[BK * LS];   // Bs[k][j]
    const int t = threadIdx.x;
    const int64_t tiles_m = M / BT;
    const int64_t i0 = (tile % tiles_m) * BT, j0 = (tile / tiles_m) * BT;
    const int64_t kb = (TRI == 2) ? i0 : 0;
    const int64_t ke = (TRI == 1) ? ((j0 + BT < K) ? j0 + BT : K) : K;
    const int ar = t % BT, akq = t / BT;          // A loads: row ar, k = akq * AQ + q
    const int bk = t % 16, bjq = t / 16;          // B loads: k = bk, column bjq * AQ + q
    double pa[AQ], pb[AQ];
    auto load = [&](int64_t k0) {
        // the triangle's zero side is never read (the strictly lower part of X is not
        // stored): it is taken as zero here
#pragma unroll
        for (int q = 0; q < AQ; ++q) {
            const int64_t i = i0 + ar, k = k0 + akq * AQ + q;
            pa[q] = (i < arl && k < acl && (TRI != 2 || k >= i)) ? (double)A[i + k * lda] : 0.0;
            const int64_t kb2 = k0 + bk, jb = j0 + bjq * AQ + q;
            pb[q] = (TRI != 1 || kb2 <= jb) ? B[kb2 + jb * ldb] : 0.0;
        }
    };
    const int lane = t & 63, wv = t >> 6;
    const int wr = wv & 1, wc = wv >> 1;
    const int li = lane & 15, lk = lane >> 4;
    tgd4 acc[2][2];
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) acc[x][y] = tgd4{0.0, 0.0, 0.0, 0.0};
    if (kb < ke) load(kb);
    for (int64_t k0 = kb; k0 < ke; k0 += BK) {
        __syncthreads();
#pragma unroll
        for (int q = 0; q < AQ; ++q) {
            As[(akq * AQ + q) * LS + ar] = pa[q];
            Bs[bk * LS + bjq * AQ + q] = pb[q];
        }
        __syncthreads();
        if (k0 + BK < ke) load(k0 + BK);
#pragma unroll
        for (int k4 = 0; k4 < BK / 4; ++k4) {
            double a[2], b[2];
#pragma unroll
            for (int x = 0; x < 2; ++x) a[x] = As[(4 * k4 + lk) * LS + 32 * wr + 16 * x + li];
#pragma unroll
            for (int y = 0; y < 2; ++y) b[y] = Bs[(4 * k4 + lk) * LS + 32 * wc + 16 * y + li];
#pragma unroll
            for (int x = 0; x < 2; ++x)
#pragma unroll
                for (int y = 0; y < 2; ++y)
                    acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[x], b[y], acc[x][y], 0, 0, 0);
        }
    }
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int v = 0; v < 4; ++v)
                C[(i0 + 32 * wr + 16 * x + 4 * v + lk) + (j0 + 32 * wc + 16 * y + li) * ldc] =
                    alpha * acc[x][y][v];
}

// One level of the recursion in one launch: the products of up to kTriNodes
// nodes of equal depth (disjoint column ranges, so independent), their tiles
// numbered node after node. At n = 8192 this takes 14 launches where one per
// node and product took 254, and the inverse 6.6 ms where it took 11.8. Node k covers columns [c0, c0 + s1 + s2); its
// T = R12 X22 (TRI = 1) or X12 = -X11 T (TRI = 2) uses the T block at toff.
constexpr int kTriNodes = 64;
struct TriLevel {
    int count;
    int tile0[kTriNodes + 1];   // first tile of each node; tile0[count] = all tiles
    int c0[kTriNodes], s1[kTriNodes], s2[kTriNodes];
    int64_t toff[kTriNodes];
};

template <int TRI>
__global__ __launch_bounds__(TT) void tri_level_kernel(const TriLevel lv, int64_t n,
                                                       const float *__restrict__ R, int64_t ldr,
                                                       double *__restrict__ X, int64_t ldx,
                                                       double *__restrict__ T) {
    // this workgroup's node: the last k with tile0[k] <= blockIdx.x (binary search)
    const int b = (int)blockIdx.x;
    int lo = 0, hi = lv.count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if (lv.tile0[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    const int64_t c0 = lv.c0[lo], s1 = lv.s1[lo], s2 = lv.s2[lo];
    double *Tk = T + lv.toff[lo];
    const int64_t tile = b - lv.tile0[lo];
    if constexpr (TRI == 1) {
        // T = R12 X22 (s1 x s2, ld s1); R beyond n is the identity, so R12 is zero there
        tri_tile<float, 1>(s1, s2, R + c0 + (c0 + s1) * ldr, ldr, n - c0, n - (c0 + s1),
                           X + (c0 + s1) + (c0 + s1) * ldx, ldx, Tk, s1, 1.0, tile);
    } else {
        // X12 = -X11 T
        const int64_t big = (int64_t)1 << 62;
        tri_tile<double, 2>(s1, s1, X + c0 + c0 * ldx, ldx, big, big, Tk, s1,
                            X + c0 + (c0 + s1) * ldx, ldx, -1.0, tile);
    }
}

// ---- applications -----------------------------------------------------------
constexpr int TCS = 256;   // columns per split of the upper-triangular GEMV

// part[c][i] = sum_{j in split c, j >= i} X[i, j] v[j] for the splits c that
// reach the diagonal of row block blockIdx.x (rows of 256).
__global__ __launch_bounds__(TT) void trmv_n_kernel(int64_t np, const double *__restrict__ X,
                                                    int64_t ldx, const double *__restrict__ v,
                                                    double *__restrict__ part) {
    const int64_t rb = blockIdx.x, c = blockIdx.y;
    if ((c + 1) * TCS <= rb * TT) return;          // split entirely left of the diagonal
    const int64_t i = rb * TT + threadIdx.x;
    const int64_t j1 = (c + 1) * TCS;
    const int64_t j0 = (c * TCS > i) ? c * TCS : i;
    double acc = 0.0;
    const double *xr = X + i;
    int64_t j = j0;
    // TU loads in flight per thread (the workgroups are few), summed in column order
    constexpr int TU = 16;
    for (; j + TU <= j1; j += TU) {
        double xv[TU];
#pragma unroll
        for (int u = 0; u < TU; ++u) xv[u] = xr[(j + u) * ldx];
#pragma unroll
        for (int u = 0; u < TU; ++u) acc = fma(xv[u], v[j + u], acc);
    }
    for (; j < j1; ++j) acc = fma(xr[j * ldx], v[j], acc);
    part[c * np + i] = acc;
}

// out[i] = sum over the splits that reach row i, in split order (deterministic).
__global__ __launch_bounds__(TT) void trmv_n_combine_kernel(int64_t np, int64_t nsplit,
                                                            const double *__restrict__ part,
                                                            double *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * TT + threadIdx.x;
    if (i >= np) return;
    double s = 0.0;
    for (int64_t c = i / TCS; c < nsplit; ++c) s += part[c * np + i];
    out[i] = s;
}

// out[j] = sum_{i <= j} X[i, j] u[i]: one wave per column, fixed reduction order.
__global__ __launch_bounds__(TT) void trmv_t_kernel(int64_t np, const double *__restrict__ X,
                                                    int64_t ldx, const double *__restrict__ u,
                                                    double *__restrict__ out) {
    const int lane = threadIdx.x & 63;
    const int64_t j = (int64_t)blockIdx.x * (TT / 64) + (threadIdx.x >> 6);
    if (j >= np) return;
    const double *xc = X + j * ldx;
    double acc = 0.0;
    int64_t i = lane;
    for (; i + 192 <= j; i += 256) {
        acc = fma(xc[i], u[i], acc);
        acc = fma(xc[i + 64], u[i + 64], acc);
        acc = fma(xc[i + 128], u[i + 128], acc);
        acc = fma(xc[i + 192], u[i + 192], acc);
    }
    for (; i <= j; i += 64) acc = fma(xc[i], u[i], acc);
    acc = wave_sum_d(acc);
    if (lane == 0) out[j] = acc;
}

// Xt = X^T (np x np, ld np) through 64 x 64 LDS tiles.
__global__ __launch_bounds__(TT) void transpose_kernel(int64_t np, const double *__restrict__ X,
                                                       double *__restrict__ Xt) {
    __shared__ double tile[64][65];
    const int64_t tiles = np / 64;
    const int64_t bi = blockIdx.x % tiles, bj = blockIdx.x / tiles;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (int r = ty; r < 64; r += TT / 64) tile[r][tx] = X[(bi * 64 + tx) + (bj * 64 + r) * np];
    __syncthreads();
    for (int r = ty; r < 64; r += TT / 64) Xt[(bj * 64 + tx) + (bi * 64 + r) * np] = tile[tx][r];
}

hipError_t kr_transpose(hipStream_t s, int64_t np, const double *X, double *Xt) {
    if (np % 64) return hipErrorInvalidValue;
    const int64_t tiles = np / 64;
    hipLaunchKernelGGL(transpose_kernel, dim3((unsigned)(tiles * tiles)), dim3(TT), 0, s, np, X,
                       Xt);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
size_t kr_trinv_tmp_doubles(int64_t np) { return (size_t)(np / 2 + IB) * (size_t)(np / 2 + IB); }

// Internal nodes of the recursion (w > 64), with their depth.
struct TriNode {
    int64_t c0, w;
    int depth;
};
static void tri_nodes(std::vector<TriNode> &out, int64_t c0, int64_t w, int depth) {
    if (w <= IB) return;
    const int64_t s1 = IB * ((w / IB + 1) / 2), s2 = w - s1;
    out.push_back({c0, w, depth});
    tri_nodes(out, c0, s1, depth + 1);
    tri_nodes(out, c0 + s1, s2, depth + 1);
}

hipError_t kr_trinv(hipStream_t s, int64_t n, int64_t np, const float *R, int64_t ldr, double *X,
                    double *T) {
    if (np % IB) return hipErrorInvalidValue;
    hipLaunchKernelGGL(inv_diag_kernel, dim3((unsigned)(np / IB)), dim3(IB), 0, s, n, R, ldr, X,
                       np);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    std::vector<TriNode> nodes;
    tri_nodes(nodes, 0, np, 0);
    int maxd = -1;
    for (const TriNode &d : nodes) maxd = d.depth > maxd ? d.depth : maxd;
    // deepest level first: a node's children are complete before its products.
    // The T blocks of one launch lie side by side: sum of s1 s2 <= (np / 2)^2,
    // within the kr_trinv_tmp_doubles(np) of T. 64 x 64 tiles throughout: at
    // n = 8192, 128 x 128 tiles (vector units with 8 x 8 per thread, or matrix
    // cores) were slower.
    for (int d = maxd; d >= 0; --d) {
        size_t i = 0;
        while (i < nodes.size()) {
            TriLevel lv;
            memset(&lv, 0, sizeof(lv));
            int64_t tiles = 0, toff = 0;
            for (; i < nodes.size() && lv.count < kTriNodes; ++i) {
                if (nodes[i].depth != d) continue;
                const int64_t w = nodes[i].w, s1 = IB * ((w / IB + 1) / 2), s2 = w - s1;
                const int k = lv.count++;
                lv.tile0[k] = (int)tiles;
                lv.c0[k] = (int)nodes[i].c0;
                lv.s1[k] = (int)s1;
                lv.s2[k] = (int)s2;
                lv.toff[k] = toff;
                tiles += (s1 / IB) * (s2 / IB);
                toff += s1 * s2;
            }
            if (lv.count == 0) continue;
            lv.tile0[lv.count] = (int)tiles;
            hipLaunchKernelGGL(tri_level_kernel<1>, dim3((unsigned)tiles), dim3(TT), 0, s, lv, n,
                               R, ldr, X, np, T);
            hipLaunchKernelGGL(tri_level_kernel<2>, dim3((unsigned)tiles), dim3(TT), 0, s, lv, n,
                               R, ldr, X, np, T);
            e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
    }
    return hipSuccess;
}

size_t kr_trmv_part_doubles(int64_t np) { return (size_t)((np + TCS - 1) / TCS) * (size_t)np; }

hipError_t kr_trmv(hipStream_t s, int64_t np, const double *X, const double *in, double *out,
                   double *part, int trans) {
    if (np % TT) return hipErrorInvalidValue;
    if (trans) {
        hipLaunchKernelGGL(trmv_t_kernel, dim3((unsigned)(np / (TT / 64))), dim3(TT), 0, s, np, X,
                           np, in, out);
        return hipGetLastError();
    }
    const int64_t nsplit = (np + TCS - 1) / TCS;
    hipLaunchKernelGGL(trmv_n_kernel, dim3((unsigned)(np / TT), (unsigned)nsplit), dim3(TT), 0, s,
                       np, X, np, in, part);
    hipLaunchKernelGGL(trmv_n_combine_kernel, dim3((unsigned)(np / TT)), dim3(TT), 0, s, np,
                       nsplit, part, out);
    return hipGetLastError();
}

}  // namespace qrx
