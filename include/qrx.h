/*
 * qrx -- mixed-precision QR factorisation and least-squares solver for
 * AMD Instinct MI355X (gfx950).
 *
 * Method (Zhang & Wu, "High Accuracy Low Precision QR Factorization and Least
 * Square Solver on GPU with TensorCore"):
 *   - QR by recursive blocked Gram-Schmidt (Alg. 2, eq. recqr): split the
 *     columns [A1 | A2], factor A1, R12 = Q1^T A2, A2 -= Q1 R12, factor A2.
 *     The two trailing products run on the matrix cores in FP16, BF16 or
 *     split FP16 with FP32 accumulation (Sec. 3.1.2); narrow panels at the
 *     leaves are orthogonalised twice (Sec. 4.1.2), by Cholesky QR on an FP64
 *     Gram matrix (default) or by a communication-avoiding TSQR with modified
 *     Gram-Schmidt blocks (eq. caqr, Alg. 4).
 *   - Least squares by a Krylov iteration (LSQR, or CGLS as in Alg. 5) on
 *     A R^{-1}, i.e. right-preconditioned by the low-precision R (Sec. 3.2.3),
 *     with FP64 vectors, R^{-1} formed once in FP64 and applied as a
 *     triangular matrix-vector product, and an FP64 (double-double
 *     accumulated) residual check.
 *
 * Conventions for every entry point:
 *   - Matrices are column-major. A is m x n with leading dimension lda >= m;
 *     R is n x n with ldr >= n. The problem needs m >= n >= 1 (Sec. 2.2:
 *     m > n and full column rank; m == n is accepted).
 *   - Matrix and vector pointers are DEVICE pointers owned by the caller; the
 *     library never frees them. `work` is an optional caller-owned device
 *     workspace of `work_bytes` bytes (query the size with the *_workspace_size
 *     call); with work == NULL the handle allocates and keeps its own.
 *   - Return values: QRX_OK (0) or a negative code detected on the host
 *     before any device work is enqueued (nothing is modified then).
 *     Numerical outcomes (positive codes) are reported through the status /
 *     info outputs described per call.
 *   - A handle is bound to one device and is not thread-safe: use one handle
 *     per host thread. Calls on one handle that use its own workspace (work ==
 *     NULL) share that workspace: issue them in stream order (one stream, or
 *     streams ordered by events). When a call needs a larger workspace the
 *     handle allocates a new one and keeps the old one alive until
 *     qrx_destroy, so work already queued (or recorded in a graph) that points
 *     at the old one stays valid.
 */
#ifndef QRX_H
#define QRX_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define QRX_OK          0
#define QRX_EINVAL     -1   /* bad argument (sizes, NULL pointer, enum, tolerance, workspace) */
#define QRX_ENOMEM     -2   /* device allocation by the handle failed */
#define QRX_EHIP       -3   /* a HIP runtime call or kernel launch failed */
#define QRX_ESINGULAR   1   /* R has a zero or non-finite diagonal entry: A is not of
                               full column rank in working precision (Sec. 2.2) */
#define QRX_ENONFINITE  2   /* A (or b) holds a NaN or Inf */
#define QRX_ENOCONV     3   /* the Krylov iteration reached max_iter above tol */
#define QRX_ESYNC       4   /* the persistent Krylov launch could not synchronise its
                               workgroups (another persistent launch held the device);
                               x is not written */

typedef struct qrx_handle_s *qrx_handle;

/* Operand precision of the trailing products R12 = Q1^T A2 and
 * A2 -= Q1 R12 (Alg. 2); accumulation is FP32 in every mode. QRX_FP16X3
 * splits each FP32 operand x into FP16 parts hi = fl16(x), lo = fl16(x - hi)
 * and forms hi*hi + hi*lo + lo*hi on the FP16 matrix cores (three products
 * per step, ~22-bit operands): near-FP32 accuracy at FP16 matrix-core rates. */
typedef enum { QRX_FP32 = 0, QRX_FP16 = 1, QRX_BF16 = 2, QRX_FP16X3 = 3 } qrx_prec;

/* QR options; an all-zero struct selects the defaults. */
typedef struct {
    int gemm_prec;        /* qrx_prec for recursion nodes wider than `cutoff` */
    int panel_width;      /* nb: leaf panel width; 1..128 for the Gram panel (0 = 64;
                             65..128 factor the panel as two 64-column blocks of one
                             Cholesky QR), 1..32 for the TSQR panel (0 = 32; Sec. 3.1.3
                             uses 32) */
    int cutoff;           /* c: nodes of width <= c use FP32 products (0 = 128, the
                             cutoff of Alg. 2); rounded up to a multiple of nb */
    int block_rows;       /* b: TSQR block rows, only 256 is supported (0 = 256; Sec. 3.1.3) */
    int no_col_scaling;   /* 1 = do not scale FP16/BF16 operand columns by powers of two */
    int panel_single_pass;/* 1 = one orthogonalisation sweep per panel instead of two */
    int panel_alg;        /* leaf panel: 0 = Cholesky QR twice on an FP64 Gram matrix
                             (default), 1 = TSQR with modified Gram-Schmidt blocks run
                             twice (eq. caqr with Alg. 4) */
    int node_reorth;      /* re-orthogonalise at every recursion node (project and update
                             twice, R12 accumulated; Sec. 4.1.2 remedy applied per node):
                             0 = default (off for qrx_qr_factor*, on for qrx_lls_solve),
                             1 = on, 2 = off */
    int gemm_tiles;       /* tiles of the low-precision trailing products: 0 = 256 x 256
                             tiles for nodes with at least 512 rows and columns of output
                             (default), 1 = 128-row tiles only. Batched plans: 0 = 128 x 128,
                             1 = 64 x 64 */
    int split_target;     /* workgroups a row-split projection aims at: 0 = default (256 with
                             256 x 256 tiles, 512 otherwise), else 16..8192 */
    int q_reorth;         /* 1 = re-orthogonalise the whole Q: factor Q again with the same
                             options (Q = Q2 R2) and return Q2 and R2 R (twice the time;
                             orthogonality no longer grows with the condition of A).
                             0 = off (default). Ignored by the least-squares calls;
                             must be 0 for the batched calls */
} qrx_qr_opts;

/* Least-squares options; an all-zero struct selects the defaults. */
typedef struct {
    qrx_qr_opts qr;
    int method;           /* 0 = LSQR (default), 1 = CGLS (Alg. 5) */
    double tol;           /* target for eta_F (0 = 1e-10); must be >= 0 */
    int max_iter;         /* Krylov iteration cap (0 = 200, the cap of Sec. 4.2.3) */
    int use_x0;           /* 1 = x holds the starting iterate on entry */
    int zero_start;       /* without use_x0: 0 = start from the direct solution
                             x0 = R^{-1} Q^T b of the factorisation (Alg. 1 with the
                             low-precision factors; default), 1 = start from x = 0. With a
                             caller-supplied R (qrx_lls_solve_with_R) the start is x = 0. */
} qrx_lls_opts;

/* Result of a least-squares solve, written by the device at the end of the
 * solve (valid once the stream has reached the end of the call). */
typedef struct {
    int status;           /* QRX_OK, QRX_ESINGULAR, QRX_ENONFINITE, QRX_ENOCONV or QRX_ESYNC */
    int iters;            /* Krylov iterations over all restarts */
    int restarts;         /* residual certifications that failed and restarted */
    int accepted;         /* the test that accepted x: 1 = eta_F <= tol; 2 = the
                             compatible-system ratio ||r|| / (||A||_F ||x|| + ||b||) <= tol
                             (for square systems, where eta_F is undefined, or a consistent
                             m > n system whose residual is at the rounding level); 0 = none */
    double eta_F;         /* ||A^T r|| / (||A||_F ||r||), r = b - A x, for the returned x */
    double resid_norm;    /* ||r||_2 */
    double normA_F;       /* ||A||_F */
    double eta_start;     /* eta_F of the starting iterate (for the default start: the
                             accuracy of the direct low-precision QR solve) */
    double score;         /* the certified score of x: min(eta_F, compatible ratio scaled
                             onto the tol scale); status is QRX_OK iff score <= tol */
} qrx_lls_info;

/* Per-kernel timing record (see qrx_timing_*). */
typedef struct {
    char name[40];
    int64_t launches;
    double total_ms;      /* sum of launch durations (HIP events on the launch stream) */
    double flops;         /* algorithmic flops summed over launches */
    double bytes;         /* algorithmic HBM bytes summed over launches */
} qrx_kernel_stat;

/* ---- handle ------------------------------------------------------------ */
int  qrx_create(qrx_handle *h, int device);
int  qrx_destroy(qrx_handle h);
const char *qrx_status_string(int status);

/* ---- QR ---------------------------------------------------------------- */
/* Bytes of device workspace qrx_qr_factor needs for (m, n, opts). */
int qrx_qr_workspace_size(qrx_handle h, int64_t m, int64_t n,
                          const qrx_qr_opts *opts, size_t *bytes);

/* Thin QR, A = Q R (Sec. 2.2; Alg. 2, eq. recqr, with re-orthogonalised
 * Cholesky-QR or TSQR leaf panels).
 * On entry A holds the matrix; on exit it holds Q (m x n, orthonormal columns
 * up to the precision of the mode). R receives the n x n upper-triangular
 * factor with positive diagonal; its strictly-lower part is set to zero.
 * `status` (device int, may be NULL) receives QRX_OK, QRX_ENONFINITE or
 * QRX_ESINGULAR when the stream reaches the end of the call. Asynchronous
 * on `stream`. */
int qrx_qr_factor(qrx_handle h, int64_t m, int64_t n, float *A, int64_t lda,
                  float *R, int64_t ldr, void *work, size_t work_bytes,
                  const qrx_qr_opts *opts, int *status, hipStream_t stream);

/* Out-of-place variant: A (const, lda) is read once by the input scan, which
 * writes the working copy into Q (m x n, ldq >= m); Q then receives the
 * orthonormal factor. Same R, status and stream semantics as qrx_qr_factor. */
int qrx_qr_factor_out(qrx_handle h, int64_t m, int64_t n, const float *A, int64_t lda,
                      float *Q, int64_t ldq, float *R, int64_t ldr, void *work,
                      size_t work_bytes, const qrx_qr_opts *opts, int *status,
                      hipStream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): qrx_qr_factor
 * with its workspace in a static device array of QRX_NOALLOC_SCRATCH_BYTES
 * bytes that the library holds on every GPU it runs on until the process ends.
 * Same arguments, results, status and stream semantics as qrx_qr_factor, minus
 * the workspace. Problems whose workspace (qrx_qr_workspace_size) exceeds the
 * array are rejected with QRX_EINVAL before anything is enqueued; so is a
 * handle with per-kernel timing on (timing creates HIP events). The call
 * allocates no device memory. Every call on a GPU shares that GPU's array and
 * its contents stay from the last call: calls that overlap in time on one GPU
 * (other streams or other handles) race; serialise them. */
#define QRX_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int qrx_qr_factor_noalloc(qrx_handle h, int64_t m, int64_t n, float *A, int64_t lda, float *R,
                          int64_t ldr, const qrx_qr_opts *opts, int *status,
                          hipStream_t stream);

/* ---- least squares ----------------------------------------------------- */
/* Bytes of device workspace qrx_lls_solve needs: the QR workspace, a working
 * copy of A, FP64 Krylov vectors, and X = R^{-1} as an FP64 np x np matrix
 * (np = n rounded up to a multiple of 256), i.e. about 8 n^2 + 4 m n bytes. */
int qrx_lls_workspace_size(qrx_handle h, int64_t m, int64_t n,
                           const qrx_lls_opts *opts, size_t *bytes);

/* x = argmin ||A x - b||_2 (Sec. 2.2, eq. opt:lls) by the QR of A followed
 * by a Krylov iteration on A R^{-1} (Sec. 3.2.3, Alg. 5), stopped when the
 * certified score (info->score) <= tol. A (FP32) and b (FP64, length m) are
 * not modified; x (FP64, length n) receives the solution (and holds x0 on
 * entry if use_x0). `info` is a DEVICE pointer to one qrx_lls_info (required).
 * Asynchronous on `stream`: the whole solve, including the iteration, its
 * stopping test and the certifications, is enqueued without any host
 * synchronisation (the iteration runs as one persistent kernel), so the call
 * can be recorded into a HIP graph. x and *info are valid when the stream
 * reaches the end of the call. Calls on one device must not overlap in time
 * (the persistent kernel expects the device's compute units to itself). */
int qrx_lls_solve(qrx_handle h, int64_t m, int64_t n, const float *A, int64_t lda,
                  const double *b, double *x, void *work, size_t work_bytes,
                  const qrx_lls_opts *opts, qrx_lls_info *info, hipStream_t stream);

/* The Krylov step alone with a caller-supplied preconditioner R (device,
 * FP32, n x n upper triangular, ldr >= n), or the identity when R == NULL.
 * Same kernels and semantics (asynchronous, device `info`) as qrx_lls_solve
 * after its factorisation. */
int qrx_lls_solve_with_R(qrx_handle h, int64_t m, int64_t n, const float *A, int64_t lda,
                         const float *R, int64_t ldr, const double *b, double *x,
                         void *work, size_t work_bytes, const qrx_lls_opts *opts,
                         qrx_lls_info *info, hipStream_t stream);

/* ---- batched: many small problems, persistent work-queue launches ---------
 * A batch is described once by a plan (host call, blocking, allocates the
 * plan's device tables): problem i has m[i] x n[i] with 1 <= n[i] <= 256 and
 * n[i] <= m[i] <= 2^31 (m, n are HOST arrays of length `batch`). The plan
 * checks the sizes (QRX_EINVAL), builds each problem's recursion schedule
 * (Alg. 2 with 32-column Cholesky-QR panels, re-orthogonalised, FP32 products
 * for nodes of width <= cutoff, BF16 products with FP32 accumulation and no
 * operand scaling above it), orders the problems longest first, and sizes the
 * workspace. cutoff and tiles are optional HOST arrays of per-problem values
 * (NULL: opts->qr.cutoff, 0 = 64, and opts->qr.gemm_tiles): the cutoff, and the
 * tile of the BF16 products (0 = 128 x 128, 1 = 64 x 64), e.g. as
 * qrx_tune_batched picks them per size class. opts->qr accepts gemm_prec
 * QRX_FP32 or QRX_BF16, panel_width 0 or 32, cutoff, gemm_tiles and
 * no_col_scaling; other QR options must be 0 (no TSQR panel, single-pass panel,
 * node or whole-Q re-orthogonalisation here). lls = 1 plans least squares
 * (LSQR only, method 0, no starting iterate; the iteration starts from x = 0;
 * tol and max_iter as in qrx_lls_opts), lls = 0 a QR factorisation. */
typedef struct qrx_batch_plan_s *qrx_batch_plan;
int qrx_batch_plan_create(qrx_handle h, int batch, const int64_t *m, const int64_t *n,
                          const int *cutoff, const int *tiles, const qrx_lls_opts *opts, int lls,
                          qrx_batch_plan *plan);
/* Bytes of device workspace the plan's batched call needs. */
int qrx_batch_plan_workspace_size(qrx_batch_plan plan, size_t *bytes);
int qrx_batch_plan_destroy(qrx_batch_plan plan);

/* The batched calls take DEVICE descriptor arrays of length `batch` (pointer
 * arrays of device pointers, leading dimensions, and per-problem outputs), in
 * the plan's problem order, and enqueue one fill kernel (the work-queue heads)
 * and the persistent kernels on `stream`: the QR kernel, whose workgroups each
 * take the next problem off an atomic queue over the longest-first order and
 * factor it, then (least squares) the LSQR kernel, which takes the problems off
 * a second queue in the same order and iterates each to the end. They are two
 * launches rather than one because each kernel is compiled for its own
 * register and LDS budget (the QR holds a 32-column panel and a product tile
 * per workgroup; LSQR needs a fraction of that): one kernel carrying the QR's
 * footprint through the LSQR phase took about twice as long.
 * Nothing is synchronised and nothing is allocated when `work` is given (or the
 * handle's workspace is already large enough), so the call can be recorded into
 * a HIP graph. Problems are independent: a singular, non-finite or invalid
 * problem (NULL pointer, lda < m, ldr < n, checked on the device) reports its
 * own status (QRX_ESINGULAR, QRX_ENONFINITE, QRX_EINVAL) and does not affect
 * the others. Outputs are valid when the stream reaches the end of the call. */

/* In place (plan made with lls = 0): A_i receives Q_i, R_i (n[i] x n[i],
 * ldr[i] >= n[i]) the upper-triangular factor; status[i] = QRX_OK,
 * QRX_ESINGULAR, QRX_ENONFINITE or QRX_EINVAL. */
int qrx_qr_factor_batched(qrx_handle h, qrx_batch_plan plan, float *const *A, const int64_t *lda,
                          float *const *R, const int64_t *ldr, void *work, size_t work_bytes,
                          int *status, hipStream_t stream);

/* x_i = argmin ||A_i x - b_i|| (plan made with lls = 1; b_i FP64 of length m[i],
 * x_i FP64 of length n[i]) by the batched QR followed by R-preconditioned LSQR
 * with FP64 vectors, certified with a double-double residual (score <= tol, as
 * qrx_lls_solve). A_i and b_i are not modified. info[i] as for qrx_lls_solve
 * (eta_start is the eta_F of x = 0). */
int qrx_lls_solve_batched(qrx_handle h, qrx_batch_plan plan, const float *const *A,
                          const int64_t *lda, const double *const *b, double *const *x,
                          void *work, size_t work_bytes, qrx_lls_info *info, hipStream_t stream);

/* ---- autotuning ---------------------------------------------------------
 * The paper fixes its blocking parameters (cutoff 128, 32-column panels, 256-row
 * TSQR blocks; Sec. 3.1.3); the tuner measures them per size class instead.
 * A size class is (device architecture, precision, panel algorithm or batched,
 * ceil(log2 m), ceil(log2 n)). */
typedef struct {
    int panel_width;      /* nb */
    int cutoff;           /* c */
    int gemm_tiles;       /* as in qrx_qr_opts */
    int split_target;     /* as in qrx_qr_opts (0 = default) */
    double ms;            /* median device time of one factorisation with these values */
    int trials;           /* configurations timed (0 when read from the cache) */
    int from_cache;       /* 1 = read from the cache file */
} qrx_tune_result;

/* Pick nb, c, the tile family and the projection split target for QR in the
 * precision (and panel algorithm) of *base: a coordinate search from the
 * defaults over nb in {32, 64, 128} (TSQR panel: {16, 32}), c in {64, 128, 256,
 * 512}, both tile families and split targets {128, 256, 512, 1024}, each
 * candidate timed with HIP events over `reps` runs (1..20) of
 * qrx_qr_factor_out on A (device, m x n, lda; not modified), median taken.
 * With cache_path (a JSON file, created if absent; NULL = no cache) a stored
 * entry for the size class is returned without measuring, and a new result
 * is stored. Allocates its own scratch (Q, R and workspace) and blocks. The
 * other fields of *base are kept as they are in every candidate.
 * Errors: QRX_EINVAL for bad sizes / options / reps, QRX_ENOMEM, QRX_EHIP, or
 * the first error of a candidate that fails for a reason other than an
 * unsupported option; a cache file that cannot be read or written gives
 * QRX_EINVAL after the measurement (out is filled). */
int qrx_tune(qrx_handle h, int64_t m, int64_t n, const float *A, int64_t lda,
             const qrx_qr_opts *base, int reps, const char *cache_path,
             qrx_tune_result *out, hipStream_t stream);

/* The batched counterpart, per size class: the problems of the batch are
 * grouped by (ceil(log2 m), ceil(log2 n)), and for each class the cutoff c in
 * {32, 64, 128, 256} and the BF16 product tile (128 or 64) are timed on that
 * class's problems as a sub-batch (copies; A is not modified), the median of
 * `reps` runs each; the best pair is stored per class in the cache (key kind 1,
 * "batched"; panel_width 32, cutoff c, gemm_tiles = the tile) and read from it
 * when present. A and lda are HOST arrays of device pointers and leading
 * dimensions. cutoff and tiles (HOST arrays of length batch, written) receive
 * each problem's values for qrx_batch_plan_create; *out sums the classes
 * (ms = sum of the chosen sub-batch times, trials = candidates timed,
 * from_cache = 1 when every class came from the cache). Blocks. */
int qrx_tune_batched(qrx_handle h, int batch, const int64_t *m, const int64_t *n,
                     const float *const *A, const int64_t *lda, const qrx_qr_opts *base,
                     int reps, const char *cache_path, int *cutoff, int *tiles,
                     qrx_tune_result *out, hipStream_t stream);

/* Host-only access to the tuning cache (no device work, no handle): the key
 * of a size class, "<arch>/<prec>/<kind>/m<ceil log2 m>/n<ceil log2 n>" with
 * kind 0 = "gram" (QR, Cholesky-QR panel), 1 = "batched", 2 = "tsqr" (QR,
 * TSQR panel), into buf (len bytes); look an entry up (QRX_OK, or 1 when the
 * file or the key is absent); store an entry (replacing the key's old one;
 * the file is rewritten whole through a temporary file). QRX_EINVAL for NULL
 * or bad arguments, a short buffer, or a file that is not a cache written by
 * this library. */
int qrx_tune_key(const char *arch, int64_t m, int64_t n, int prec, int kind, char *buf,
                 size_t len);
int qrx_tune_cache_get(const char *cache_path, const char *key, qrx_tune_result *out);
int qrx_tune_cache_put(const char *cache_path, const char *key, const qrx_tune_result *r);

/* ---- timing ------------------------------------------------------------ */
/* When enabled, every kernel launch is bracketed by HIP events on its
 * stream. qrx_timing_get synchronises those events and returns one record
 * per kernel name (at most `capacity`; `count` receives the number). */
int qrx_timing_enable(qrx_handle h, int enable);
int qrx_timing_reset(qrx_handle h);
int qrx_timing_get(qrx_handle h, qrx_kernel_stat *out, int capacity, int *count);

#ifdef __cplusplus
}
#endif
#endif /* QRX_H */
