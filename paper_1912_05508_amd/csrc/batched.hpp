// Descriptors of the batched path (device memory, written by the host).
#pragma once
#include "qrx_internal.hpp"

namespace qrx {

constexpr int kBMaxN = 256;        // largest n of a batched problem
constexpr int kBPanel = 32;        // panel width of the batched QR

struct BOp {          // one step of the recursion schedule (Alg. 2)
    int kind;         // 0 = panel of columns [c0, c0 + k); 1 = node (Q1 = [c0, c0+k), A2 = next n2)
    int c0, k, n2;
    int lowp;         // node products in the low precision (width > cutoff)
};

struct BProb {
    int64_t m, n, lda, ldw, ldr;
    const float *A;   // the problem matrix (read by the scan and by the Krylov products)
    float *W;         // working copy, Q on exit (== A for an in-place QR)
    float *R;         // n x n upper triangle, ldr
    const double *b;  // right-hand side (LLS)
    double *x;        // solution (LLS)
    double *u, *q;    // FP64 m-vectors (LLS)
    int op0, nops;    // slice of the schedule table
};

struct BOut {
    int status, iters, restarts, pad;
    double eta, rnorm, normA, rho;
};

hipError_t launch_bqr(hipStream_t s, int prec, int batch, const BProb *probs, const int *order,
                      const BOp *ops, int copy, BOut *out);
hipError_t launch_blsqr(hipStream_t s, int batch, const BProb *probs, const int *order,
                        double tol, int max_iter, BOut *out);

}  // namespace qrx
