// The batched path: a plan's device tables and the one persistent kernel.
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

// Per problem, built by a plan on the host and uploaded once.
struct BEntry {
    int64_t m, n;
    int64_t ldw;                   // leading dimension of the working copy (least squares)
    int64_t w_off, r_off, v_off;   // workspace byte offsets: working copy, R, u | q
    int op0, nops;                 // slice of the schedule table
    int tiles;                     // trailing-product tile of the low-precision nodes (0: 128, 1: 64)
    int pad;
};

// What a problem's QR hands to its LSQR (per-problem record in the workspace).
struct BRes {
    int status, pad;
    double normA, rho;
};

// Arguments of the persistent batched kernels (device arrays throughout).
struct BArgs {
    const BEntry *ent;
    const int *order;              // longest first
    const BOp *ops;
    int batch, lls;
    const float *const *A;         // problem matrices (QR: overwritten by Q)
    const int64_t *lda;
    float *const *R;               // QR: R outputs
    const int64_t *ldr;
    const double *const *b;        // least squares: right-hand sides and solutions
    double *const *x;
    char *work;                    // per-problem working storage (least squares)
    unsigned *counter;             // heads of the QR and LSQR work queues, zero at launch
    BRes *res;                     // least squares: per-problem QR results
    int *status;                   // QR: per-problem status
    qrx_lls_info *info;            // least squares: per-problem result
    double tol;
    int max_iter;
};

// The persistent batched launch: the QR work-queue kernel, then (least squares)
// the LSQR work-queue kernel, each with as many workgroups as fit on the device.
hipError_t launch_bsolve(hipStream_t s, int device, int prec, const BArgs &a);

}  // namespace qrx
