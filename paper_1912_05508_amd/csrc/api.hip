// Host runtime of the qrx C ABI: argument validation, workspace carving, the
// static recursion schedule of Alg. 2, the TSQR level plan of eq. caqr, the
// Krylov driver of Sec. 3.2.3 and per-kernel timing.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "batched.hpp"
#include "krylov.hpp"
#include "qrx_internal.hpp"

using namespace qrx;

// ---------------------------------------------------------------------------
// handle
// ---------------------------------------------------------------------------
struct PendingTiming {
    std::string name;
    hipEvent_t a, b;
    double flops, bytes;
};

// Per-phase wall-clock record of one persistent Krylov launch (pinned host
// memory the kernel writes at its end), read by qrx_timing_get.
struct PendingPhases {
    long long *buf;
    double khz;                   // wall-clock ticks per millisecond
    int64_t m, n, np;
    int splits_n, splits_t, grid;
    int fused;                    // LSQR iterations take the one-pass products
};

struct qrx_handle_s {
    int device = -1;
    void *scratch_ptr = nullptr;   // this device's address of the static scratch array
    std::vector<PendingPhases> phase_pending;
    std::vector<long long *> phase_spare;
    void *pool = nullptr;
    size_t pool_bytes = 0;
    std::vector<void *> retired;    // outgrown pools, freed by qrx_destroy
    bool timing = false;
    std::vector<PendingTiming> pending;
    std::vector<hipEvent_t> spare;
    std::map<std::string, qrx_kernel_stat> stats;

    hipEvent_t ev() {
        if (!spare.empty()) {
            hipEvent_t e = spare.back();
            spare.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        hipEventCreate(&e);
        return e;
    }
};

namespace {

struct Rec {   // brackets one launch (or launch group) with events when timing is on
    qrx_handle h;
    hipStream_t s;
    hipEvent_t a = nullptr;
    Rec(qrx_handle h_, hipStream_t s_) : h(h_), s(s_) {
        if (h->timing) {
            a = h->ev();
            hipEventRecord(a, s);
        }
    }
    void end(const char *name, double flops, double bytes) {
        if (h->timing) {
            hipEvent_t b = h->ev();
            hipEventRecord(b, s);
            h->pending.push_back({name, a, b, flops, bytes});
        }
    }
};

#define QRX_TRY(expr)                                \
    do {                                             \
        hipError_t e__ = (expr);                     \
        if (e__ != hipSuccess) return QRX_EHIP;      \
    } while (0)

// bump allocator over a device buffer (or a size counter when base == null)
struct Carve {
    char *base;
    size_t off = 0;
    explicit Carve(void *b) : base((char *)b) {}
    template <class T>
    T *take(size_t count) {
        off = (off + 255) & ~size_t(255);
        T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
        off += count * sizeof(T);
        return p;
    }
};

int64_t round_up(int64_t v, int64_t q) { return (v + q - 1) / q * q; }

struct QrCfg {
    int prec, nb, c, reorth, scaling, alg, node_reorth, tiles, split_target, qreorth;
};

int resolve_qr(const qrx_qr_opts *o, QrCfg &c, bool lls = false) {
    qrx_qr_opts z;
    memset(&z, 0, sizeof(z));
    if (!o) o = &z;
    if (o->gemm_prec < 0 || o->gemm_prec > 3) return QRX_EINVAL;
    if (o->panel_alg < 0 || o->panel_alg > 1) return QRX_EINVAL;
    const int max_nb = o->panel_alg == 1 ? 32 : 128;
    if (o->panel_width < 0 || o->panel_width > max_nb) return QRX_EINVAL;
    if (o->cutoff < 0) return QRX_EINVAL;
    if (o->block_rows != 0 && o->block_rows != kPanelThreads) return QRX_EINVAL;
    if (o->no_col_scaling < 0 || o->no_col_scaling > 1) return QRX_EINVAL;
    if (o->panel_single_pass < 0 || o->panel_single_pass > 1) return QRX_EINVAL;
    c.prec = o->gemm_prec;
    c.alg = o->panel_alg;
    c.nb = o->panel_width ? o->panel_width : (c.alg == 1 ? 32 : 64);
    int cut = o->cutoff ? o->cutoff : 128;
    if (cut < c.nb) cut = c.nb;
    c.c = (int)round_up(cut, c.nb);
    if (o->node_reorth < 0 || o->node_reorth > 2) return QRX_EINVAL;
    c.node_reorth = o->node_reorth == 1 ? 1 : (o->node_reorth == 2 ? 0 : (lls ? 1 : 0));
    c.reorth = o->panel_single_pass ? 0 : 1;
    c.scaling = o->no_col_scaling ? 0 : 1;
    if (o->gemm_tiles < 0 || o->gemm_tiles > 1) return QRX_EINVAL;
    if (o->split_target != 0 && (o->split_target < 16 || o->split_target > 8192)) return QRX_EINVAL;
    c.tiles = o->gemm_tiles;
    c.split_target = o->split_target;
    if (o->q_reorth < 0 || o->q_reorth > 1) return QRX_EINVAL;
    c.qreorth = lls ? 0 : o->q_reorth;
    return QRX_OK;
}

struct Op {
    int kind;            // 0 = panel, 1 = node (projection + update)
    int64_t c0, k, n2;   // panel: columns [c0, c0 + k); node: Q1 = [c0, c0+k), A2 = [c0+k, c0+k+n2)
    int prec;
};

void plan_rec(int64_t c0, int64_t w, const QrCfg &c, std::vector<Op> &ops) {
    if (w <= c.nb) {
        ops.push_back({0, c0, w, 0, QRX_FP32});
        return;
    }
    const int64_t unit = (w > c.c) ? c.c : c.nb;
    const int64_t n1 = unit * ((w + 2 * unit - 1) / (2 * unit));
    plan_rec(c0, n1, c, ops);
    ops.push_back({1, c0, n1, w - n1, (w > c.c) ? c.prec : QRX_FP32});
    plan_rec(c0 + n1, w - n1, c, ops);
}

// TSQR level sizes for a panel of m rows (level 0 .. nlev).
void tsqr_sizes(int64_t m, int nb, std::vector<int64_t> &nblk) {
    nblk.clear();
    int64_t b0 = (m + kPanelThreads - 1) / kPanelThreads;
    nblk.push_back(b0);
    int64_t units = b0;
    while (nblk.back() > 1) {
        const int64_t rows = units * nb;
        const int64_t nb_l = (rows + kPanelThreads - 1) / kPanelThreads;
        nblk.push_back(nb_l);
        units = nb_l;
    }
}

struct QrWork {
    int *flags;
    float *colmax, *uscale, *part, *rtop, *stack_base, *rcorr, *cmpart;
    float *r2, *r3;   // whole-Q re-orthogonalisation: R2 and the product R2 R (n x n)
    double *colss, *normA, *gram;
    size_t stack_floats;
    // 16-bit operand copies for low-precision nodes (null when there are none):
    // Q column-major (ldc) and row-major (ldq), R12 of the current node (ld k)
    uint16_t *qc, *qcl, *qr, *qrl, *rh, *rhl;
    // the node's A2 packed to 16-bit (column-major, ldc) for large-tile projections
    uint16_t *a2h, *a2l;
    int64_t ldc, ldq;
};

// Whether a low-precision node's products take the large-tile kernels (their
// operands are the packed copies, aligned when the node's first column is a
// multiple of 8 and its width k is too).
bool tn_proj(const Op &o, int64_t m, const QrCfg &c) {
    return c.tiles == 0 && o.prec != QRX_FP32 && m >= 256 && o.k >= 512 && o.n2 >= 512 &&
           o.c0 % 8 == 0;
}
bool tn_upd(const Op &o, int64_t m, const QrCfg &c) {
    return c.tiles == 0 && o.prec != QRX_FP32 && m >= 256 && o.n2 >= 512 && o.c0 % 8 == 0 &&
           o.k % 8 == 0;
}
int node_splits(const Op &o, int64_t m, const QrCfg &c) {
    return tn_proj(o, m, c) ? tn_projection_splits(m, o.k, o.n2, c.split_target)
                            : projection_splits(m, o.k, o.n2, o.prec, c.split_target);
}

bool has_lowp_nodes(const QrCfg &c, const std::vector<Op> &ops) {
    for (const Op &o : ops)
        if (o.kind == 1 && o.prec != QRX_FP32) return true;
    (void)c;
    return false;
}

void carve_qr(Carve &cv, int64_t m, int64_t n, const QrCfg &c, const std::vector<Op> &ops,
              QrWork &w) {
    w.flags = cv.take<int>(4);
    w.r2 = cv.take<float>(c.qreorth ? (size_t)n * n : 1);
    w.r3 = cv.take<float>(c.qreorth ? (size_t)n * n : 1);
    w.colmax = cv.take<float>(n);
    w.uscale = cv.take<float>(n);
    w.colss = cv.take<double>(n);
    w.normA = cv.take<double>(1);
    size_t part = 1;
    for (const Op &o : ops)
        if (o.kind == 1) {
            const size_t s = node_splits(o, m, c);
            part = std::max(part, s * (size_t)o.k * (size_t)o.n2);
        }
    w.part = cv.take<float>(part);
    size_t rc = 1;
    if (c.node_reorth)
        for (const Op &o : ops)
            if (o.kind == 1) rc = std::max(rc, (size_t)o.k * (size_t)o.n2);
    w.rcorr = cv.take<float>(rc);
    w.cmpart = cv.take<float>((size_t)update_cmpart_slots(m) * (size_t)n);
    w.rtop = cv.take<float>(32 * 32);
    std::vector<int64_t> nblk;
    tsqr_sizes(m, 32, nblk);
    size_t st = 0;
    for (size_t l = 1; l < nblk.size(); ++l) st += (size_t)nblk[l - 1] * 32 * 32 + 64;
    w.stack_floats = st;
    w.stack_base = cv.take<float>(c.alg == 1 ? st + 1 : 1);
    w.gram = cv.take<double>(c.alg == 0 ? gram_workspace_doubles(m, c.nb > 64 ? 128 : 64) : 1);
    w.qc = w.qcl = w.qr = w.qrl = w.rh = w.rhl = w.a2h = w.a2l = nullptr;
    w.ldc = round_up(m, 8);
    w.ldq = round_up(n, 8);
    if (has_lowp_nodes(c, ops)) {
        const bool split = c.prec == QRX_FP16X3;
        size_t rsz = 1;
        for (const Op &o : ops)
            if (o.kind == 1 && o.prec != QRX_FP32) rsz = std::max(rsz, (size_t)o.k * (size_t)o.n2);
        w.qc = cv.take<uint16_t>((size_t)w.ldc * n);
        w.qr = cv.take<uint16_t>((size_t)m * w.ldq);
        w.rh = cv.take<uint16_t>(rsz);
        if (split) {
            w.qcl = cv.take<uint16_t>((size_t)w.ldc * n);
            w.qrl = cv.take<uint16_t>((size_t)m * w.ldq);
            w.rhl = cv.take<uint16_t>(rsz);
        }
        size_t a2 = 0;
        for (const Op &o : ops)
            if (o.kind == 1 && tn_proj(o, m, c)) a2 = std::max(a2, (size_t)w.ldc * (size_t)o.n2);
        if (a2) {
            w.a2h = cv.take<uint16_t>(a2);
            if (split) w.a2l = cv.take<uint16_t>(a2);
        }
    }
}

int run_panel_core(qrx_handle h, hipStream_t s, int64_t m, float *P, int64_t ld, int w,
                   float *R, int64_t ldr, const float *colmax, const QrCfg &c, QrWork &ws,
                   const PanelPack &pack);

// One leaf panel (columns [c0, c0 + w) of W), then its 16-bit operand copies.
int run_panel(qrx_handle h, hipStream_t s, int64_t m, float *W, int64_t ldw, int64_t c0, int w,
              float *R, int64_t ldr, const QrCfg &c, QrWork &ws) {
    float *P = W + c0 * ldw;
    // a 64-column Cholesky-QR panel writes the 16-bit operand copies with its Q
    PanelPack pack{};
    const bool fused = ws.qc && c.alg == 0 && gram_panel_packs(w);
    if (fused) {
        pack.qc = ws.qc + c0 * ws.ldc;
        pack.qcl = ws.qcl ? ws.qcl + c0 * ws.ldc : nullptr;
        pack.qr = ws.qr + c0;
        pack.qrl = ws.qrl ? ws.qrl + c0 : nullptr;
        pack.ldc = ws.ldc;
        pack.ldq = ws.ldq;
        pack.sc = c.scaling ? 16384.0f : 1.0f;
        pack.prec = c.prec;
    }
    int rc = run_panel_core(h, s, m, P, ldw, w, R + c0 + c0 * ldr, ldr, ws.colmax + c0, c, ws,
                            pack);
    if (rc) return rc;
    if (ws.qc && !fused) {
        Rec r(h, s);
        QRX_TRY(launch_pack_q(s, c.prec, c.scaling, m, w, P, ldw, ws.qc + c0 * ws.ldc,
                              ws.qcl ? ws.qcl + c0 * ws.ldc : nullptr, ws.ldc, ws.qr + c0,
                              ws.qrl ? ws.qrl + c0 : nullptr, ws.ldq));
        r.end("pack_q", 0.0, (4.0 + (ws.qcl ? 8.0 : 4.0)) * m * w);
    }
    return QRX_OK;
}

int run_panel_core(qrx_handle h, hipStream_t s, int64_t m, float *P, int64_t ld, int w, float *R,
                   int64_t ldr, const float *colmax, const QrCfg &c, QrWork &ws,
                   const PanelPack &pack) {
    if (c.alg == 0) {
        Rec r(h, s);
        QRX_TRY(launch_gram_panel(s, P, ld, m, w, R, ldr, ws.gram, c.reorth, pack));
        // FP64 work: Gram of P, Q formation, Gram of Q1 (m w(w+1)/2 FMA each); the
        // second Q formation runs only when Q1 is not yet orthonormal, so the
        // usual case is counted. Traffic model of a leaf panel (FP32): read the
        // panel, write Q, and read and write it once more, 16 m w bytes.
        r.end("gram_panel", (c.reorth ? 3.0 : 2.0) * m * (double)w * (w + 1), 16.0 * m * w);
        return QRX_OK;
    }
    constexpr int NB = 32;
    std::vector<int64_t> nblk;
    tsqr_sizes(m, NB, nblk);
    TsqrLevels lv;
    memset(&lv, 0, sizeof(lv));
    lv.nlev = (int)nblk.size() - 1;
    if (lv.nlev > kMaxLevels) return QRX_EINVAL;
    float *cur = ws.stack_base;
    for (int l = 0; l <= lv.nlev; ++l) lv.nblk[l] = nblk[l];
    for (int l = 1; l <= lv.nlev; ++l) {
        lv.stack[l] = cur;
        cur += nblk[l - 1] * NB * NB + 64;
    }
    const double flops_blk = (c.reorth ? 2.0 : 1.0) * 2.0 * 256.0 * w * w;
    {
        Rec r(h, s);
        float *rn = lv.nlev ? lv.stack[1] : ws.rtop;
        int64_t ldn = lv.nlev ? nblk[0] * NB : NB;
        QRX_TRY(launch_tsqr_level(s, P, ld, m, w, nblk[0], 1, rn, ldn, c.reorth, colmax));
        r.end("tsqr_leaf", flops_blk * nblk[0], 8.0 * m * w);
    }
    for (int l = 1; l <= lv.nlev; ++l) {
        Rec r(h, s);
        const int64_t rows = nblk[l - 1] * NB;
        float *rn = (l < lv.nlev) ? lv.stack[l + 1] : ws.rtop;
        int64_t ldn = (l < lv.nlev) ? nblk[l] * NB : NB;
        QRX_TRY(launch_tsqr_level(s, lv.stack[l], rows, rows, w, nblk[l], NB, rn, ldn, c.reorth,
                                  nullptr));
        r.end("tsqr_tree", flops_blk * nblk[l], 8.0 * rows * w);
    }
    if (lv.nlev > 0) {
        Rec r(h, s);
        QRX_TRY(launch_tsqr_qform(s, P, ld, m, w, lv));
        r.end("tsqr_qform", 2.0 * m * w * w, 8.0 * m * w);
    }
    {
        Rec r(h, s);
        QRX_TRY(launch_copy_r_block(s, ws.rtop, NB, w, R, ldr, colmax));
        r.end("copy_r", 0, 0);
    }
    return QRX_OK;
}

// The QR of W (m x n, ld ldw, in place -> Q) into R; colmax must hold the
// column max-abs of W on entry.
int run_qr(qrx_handle h, hipStream_t s, int64_t m, int64_t n, float *W, int64_t ldw, float *R,
           int64_t ldr, const QrCfg &c, const std::vector<Op> &ops, QrWork &ws) {
    if (c.alg == 0) QRX_TRY(launch_fill_f32(s, (float *)gram_counter(ws.gram), kGramCounterInts, 0.0f));
    for (const Op &o : ops) {
        if (o.kind == 0) {
            int rc = run_panel(h, s, m, W, ldw, o.c0, (int)o.k, R, ldr, c, ws);
            if (rc) return rc;
        } else {
            const float *Q1 = W + o.c0 * ldw;
            float *A2 = W + (o.c0 + o.k) * ldw;
            float *R12 = R + o.c0 + (o.c0 + o.k) * ldr;
            float *cm = ws.colmax + o.c0 + o.k;
            const int splits = node_splits(o, m, c);
            const bool big_p = tn_proj(o, m, c), big_u = tn_upd(o, m, c);
            // column max-abs of the updated A2 is read later only by scaled low-precision
            // projections inside A2 (width > cutoff) and by the TSQR panel's scaling
            float *cm_out = (c.alg == 1 || (o.n2 > c.c && o.prec != QRX_FP32 && c.scaling)) ? cm
                                                                                          : nullptr;
            const double fl = 2.0 * m * o.k * o.n2;
            static const char *pnames[4] = {"proj_fp32", "proj_fp16", "proj_bf16", "proj_fp16x3"};
            static const char *unames[4] = {"update_fp32", "update_fp16", "update_bf16", "update_fp16x3"};
            const char *pn = pnames[o.prec], *un = unames[o.prec];
            const bool lp = o.prec != QRX_FP32;
            const size_t esz = lp ? (o.prec == QRX_FP16X3 ? 4 : 2) : 4;   // bytes per Q element read
            // Rh = packed R12 (or correction) for the low-precision update
            uint16_t *rh = lp ? ws.rh : nullptr, *rhl = lp ? ws.rhl : nullptr;
            auto project = [&]() -> int {
                if (big_p) {
                    {
                        Rec r(h, s);
                        QRX_TRY(launch_pack_cols(s, o.prec, c.scaling, m, o.n2, A2, ldw, cm,
                                                 ws.a2h, ws.a2l, ws.ldc));
                        r.end("pack_a2", 0.0, (4.0 + (ws.a2l ? 4.0 : 2.0)) * m * o.n2);
                    }
                    Rec r(h, s);
                    QRX_TRY(launch_projection_tn(s, o.prec, m, o.k, o.n2, ws.qc + o.c0 * ws.ldc,
                                                 ws.qcl ? ws.qcl + o.c0 * ws.ldc : nullptr,
                                                 ws.ldc, ws.a2h, ws.a2l, ws.ldc, ws.part, splits));
                    r.end(pn, fl, (double)esz * m * (o.k + o.n2) + 4.0 * splits * o.k * o.n2);
                    return QRX_OK;
                }
                Rec r(h, s);
                if (lp)
                    QRX_TRY(launch_projection_lp(s, o.prec, c.scaling, m, o.k, o.n2,
                                                 ws.qc + o.c0 * ws.ldc,
                                                 ws.qcl ? ws.qcl + o.c0 * ws.ldc : nullptr, ws.ldc,
                                                 A2, ldw, cm, ws.part, splits));
                else
                    QRX_TRY(launch_projection(s, o.prec, c.scaling, m, o.k, o.n2, Q1, A2, ldw, cm,
                                              ws.part, splits));
                r.end(pn, fl, (double)esz * m * o.k + 4.0 * m * o.n2 + 4.0 * splits * o.k * o.n2);
                return QRX_OK;
            };
            auto update = [&](const float *Rm, int64_t ldm, float *cmo) -> int {
                Rec r(h, s);
                if (big_u)
                    QRX_TRY(launch_update_tn(s, o.prec, c.scaling, m, o.k, o.n2, ws.qr + o.c0,
                                             ws.qrl ? ws.qrl + o.c0 : nullptr, ws.ldq, rh, rhl,
                                             o.k, A2, ldw, ws.uscale, cmo, ws.cmpart));
                else if (lp)
                    QRX_TRY(launch_update_lp(s, o.prec, c.scaling, m, o.k, o.n2, ws.qr + o.c0,
                                             ws.qrl ? ws.qrl + o.c0 : nullptr, ws.ldq, rh, rhl,
                                             o.k, A2, ldw, ws.uscale, cmo, ws.cmpart));
                else
                    QRX_TRY(launch_update(s, o.prec, c.scaling, m, o.k, o.n2, Q1, A2, ldw, Rm,
                                          ldm, ws.uscale, cmo, ws.cmpart));
                r.end(un, fl, (double)esz * m * o.k + 8.0 * m * o.n2);
                return QRX_OK;
            };
            int rc = project();
            if (rc) return rc;
            {
                Rec r(h, s);
                QRX_TRY(launch_proj_reduce(s, o.prec, c.scaling, o.k, o.n2, ws.part, splits, R12,
                                           ldr, cm, ws.uscale, nullptr, 0, rh, rhl, o.k));
                r.end("proj_reduce", (double)splits * o.k * o.n2, 4.0 * (splits + 1) * o.k * o.n2);
            }
            rc = update(R12, ldr, (c.node_reorth && lp) ? cm : cm_out);
            if (rc) return rc;
            if (c.node_reorth) {
                // second projection of the updated A2 against Q1: C = Q1^T A2,
                // A2 -= Q1 C, R12 += C ("twice is enough")
                rc = project();
                if (rc) return rc;
                {
                    Rec r(h, s);
                    QRX_TRY(launch_proj_reduce(s, o.prec, c.scaling, o.k, o.n2, ws.part, splits,
                                               ws.rcorr, o.k, cm, ws.uscale, R12, ldr, rh, rhl,
                                               o.k));
                    r.end("proj_reduce", (double)splits * o.k * o.n2,
                          4.0 * (splits + 3) * o.k * o.n2);
                }
                rc = update(ws.rcorr, o.k, cm_out);
                if (rc) return rc;
            }
        }
    }
    return QRX_OK;
}

bool bad_ptr(const void *p) { return p == nullptr; }

int check_qr_args(qrx_handle h, int64_t m, int64_t n, int64_t lda, int64_t ldr) {
    if (!h) return QRX_EINVAL;
    if (n < 1 || m < n || lda < m || ldr < n) return QRX_EINVAL;
    if (n > (int64_t)1 << 30 || m > ((int64_t)1 << 40)) return QRX_EINVAL;
    return QRX_OK;
}

// The handle's workspace. A larger request allocates a new pool; the old one is
// kept (not freed) until qrx_destroy, because work already enqueued on some
// stream, or recorded into a HIP graph, may still point at it.
int ensure_pool(qrx_handle h, size_t bytes, void **out) {
    if (h->device < 0) return QRX_EHIP;
    if (h->pool_bytes < bytes) {
        void *p = nullptr;
        if (hipMalloc(&p, bytes) != hipSuccess) return QRX_ENOMEM;
        if (h->pool) h->retired.push_back(h->pool);
        h->pool = p;
        h->pool_bytes = bytes;
    }
    *out = h->pool;
    return QRX_OK;
}

// ---- Krylov workspace --------------------------------------------------------
struct KrWork {
    double *X, *Xt, *T, *tpart, *u, *u2, *r, *rc, *v, *vn, *t, *t2, *d, *z, *vt, *x, *xlo, *xbest, *q;
    double *part_n, *part_n2, *part_t, *part_f, *ssqA, *ssqB;
    unsigned *bar;
    int splits_n, splits_t;
};

void carve_kr(Carve &cv, int64_t m, int64_t n, bool precond, KrWork &k) {
    const int64_t np = round_up(n, kTrsvBlock);
    k.splits_n = kr_gemv_n_splits(m, n);
    k.splits_t = kr_gemv_t_splits(m);
    const size_t nn = precond ? (size_t)np * (size_t)np : 1;
    k.X = cv.take<double>(nn);
    k.Xt = cv.take<double>(nn);
    k.T = cv.take<double>(precond ? kr_trinv_tmp_doubles(np) : 1);
    k.tpart = cv.take<double>(kr_trmv_part_doubles(np));
    k.u = cv.take<double>(m);
    k.u2 = cv.take<double>(n <= kr_fused_max_n ? m : 1);
    k.r = cv.take<double>(m);
    k.rc = cv.take<double>(m);
    k.q = cv.take<double>(m);
    k.v = cv.take<double>(np);
    k.vn = cv.take<double>(np);
    k.t = cv.take<double>(np);
    k.t2 = cv.take<double>(np);
    k.d = cv.take<double>(np);
    k.z = cv.take<double>(np);
    k.vt = cv.take<double>(np);
    k.x = cv.take<double>(np);
    k.xlo = cv.take<double>(np);
    k.xbest = cv.take<double>(np);
    k.part_n = cv.take<double>((size_t)k.splits_n * m);
    k.part_n2 = cv.take<double>((size_t)k.splits_n * m);
    k.part_t = cv.take<double>((size_t)k.splits_t * np);
    // per-workgroup partials of the one-pass LSQR products (n <= kr_fused_max_n)
    k.part_f = cv.take<double>(n <= kr_fused_max_n ? (size_t)kr_max_grid * n : 1);
    k.ssqA = cv.take<double>(kr_loop_ssq_doubles(m, np));
    k.ssqB = cv.take<double>(kr_loop_ssq_doubles(m, np));
    k.bar = cv.take<unsigned>(64);
}

struct KrCfg {
    int method, max_iter;
    double tol;
    bool direct;   // start from x0 = R^{-1} Q^T b when Q is at hand
};

int resolve_lls(const qrx_lls_opts *o, KrCfg &k) {
    qrx_lls_opts z;
    memset(&z, 0, sizeof(z));
    if (!o) o = &z;
    if (o->method < 0 || o->method > 1) return QRX_EINVAL;
    if (!(o->tol >= 0.0) || !std::isfinite(o->tol)) return QRX_EINVAL;
    if (o->max_iter < 0) return QRX_EINVAL;
    if (o->use_x0 < 0 || o->use_x0 > 1) return QRX_EINVAL;
    if (o->zero_start < 0 || o->zero_start > 1) return QRX_EINVAL;
    k.direct = o->use_x0 == 0 && o->zero_start == 0;
    k.method = o->method;
    k.tol = o->tol > 0.0 ? o->tol : 1e-10;
    k.max_iter = o->max_iter ? o->max_iter : 200;
    return QRX_OK;
}

// Enqueues the Krylov step (Sec. 3.2.3): X = R^{-1} and its transpose, the
// start (x0 from the caller, the direct solution R^{-1} Q^T b of Alg. 1 with
// the computed factors, or zero), then the persistent iteration kernel, which
// writes x_user and *info. No host synchronisation.
int enqueue_krylov(qrx_handle h, hipStream_t s, int64_t m, int64_t n, const float *A,
                   int64_t lda, const float *R, int64_t ldr, const double *b, double *x_user,
                   bool use_x0, const float *Q, int64_t ldq, const KrCfg &cfg, KrWork &k,
                   const QrWork &ws, qrx_lls_info *info) {
    const int64_t np = round_up(n, kTrsvBlock);
    if (R) {
        Rec r(h, s);
        QRX_TRY(kr_trinv(s, n, np, R, ldr, k.X, k.T));
        QRX_TRY(kr_transpose(s, np, k.X, k.Xt));
        // recursive block inversion: ~np^3/3 FMA in FP64; the transpose moves 16 np^2 bytes
        r.end("trinv", 2.0 * (double)np * np * np / 3.0, 8.0 * np * np + 16.0 * np * np);
    }
    // the padded tails [n, np) of every n-vector must stay exactly zero
    for (double *vec : {k.x, k.xlo, k.xbest, k.v, k.vn, k.t, k.t2, k.d, k.z, k.vt})
        QRX_TRY(kr_zero(s, np, vec));
    if (use_x0) {
        QRX_TRY(hipMemcpyAsync(k.x, x_user, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    } else if (cfg.direct && Q && R) {
        // the direct solution of Alg. 1 with the computed factors: x0 = R^{-1} (Q^T b)
        Rec r(h, s);
        QRX_TRY(kr_gemv_t(s, m, n, Q, ldq, b, k.part_t));
        QRX_TRY(kr_combine_n(s, n, k.part_t, k.splits_t, k.z, k.ssqA));
        QRX_TRY(kr_trmv(s, np, k.X, k.z, k.x, k.tpart, 0));
        r.end("direct_start", 2.0 * m * n + (double)np * (np + 1),
              4.0 * m * n + 8.0 * m + 4.0 * np * (np + 1));
    }
    // barrier words cleared by a kernel (the call stays safe to record in a HIP graph)
    QRX_TRY(launch_fill_f32(s, reinterpret_cast<float *>(k.bar), 64, 0.0f));
    KLoopArgs a;
    memset(&a, 0, sizeof(a));
    a.m = m;
    a.n = n;
    a.np = np;
    a.lda = lda;
    a.A = A;
    a.b = b;
    a.X = R ? k.X : nullptr;
    a.Xt = R ? k.Xt : nullptr;
    a.colss = ws.colss;
    a.normA = ws.normA;
    a.flags = ws.flags;
    a.x = k.x;
    a.xbest = k.xbest;
    a.xlo = k.xlo;
    a.u = k.u;
    a.u2 = k.u2;
    a.rc = k.rc;
    a.q = k.q;
    a.r = k.r;
    a.v = k.v;
    a.vn = k.vn;
    a.t = k.t;
    a.t2 = k.t2;
    a.d = k.d;
    a.z = k.z;
    a.vt = k.vt;
    a.pn = k.part_n;
    a.pn2 = k.part_n2;
    a.pt = k.part_t;
    a.pf = k.part_f;
    a.ssqA = k.ssqA;
    a.ssqB = k.ssqB;
    a.bar = k.bar;
    a.x_user = x_user;
    a.info = info;
    a.splits_n = k.splits_n;
    a.splits_t = k.splits_t;
    a.cchunk = (n + k.splits_n - 1) / k.splits_n;
    a.vec = ((((uintptr_t)A) & 15) == 0) && (lda % 4 == 0);
    a.method = cfg.method;
    // the one-pass products address A and u by 32-bit byte offsets from their starts
    a.fused = cfg.method == 0 && a.vec && kr_fused_ok(m, n, lda);
    a.max_iter = cfg.max_iter;
    a.tol = cfg.tol;
    a.cscale = compat_scale(m, n, cfg.tol);
    const int grid = kr_loop_grid(h->device, m, n);
    if (h->timing) {
        long long *buf = nullptr;
        if (!h->phase_spare.empty()) {
            buf = h->phase_spare.back();
            h->phase_spare.pop_back();
        } else if (hipHostMalloc((void **)&buf, 2 * KP_COUNT * sizeof(long long)) != hipSuccess) {
            return QRX_ENOMEM;
        }
        memset(buf, 0, 2 * KP_COUNT * sizeof(long long));
        int khz = 0;
        hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, h->device);
        a.prof = buf;
        h->phase_pending.push_back({buf, khz > 0 ? (double)khz : 1e5, m, n, np, k.splits_n,
                                    k.splits_t, grid, a.fused});
    }
    Rec r(h, s);
    QRX_TRY(kr_loop(s, a, grid));
    r.end("krylov_loop", 0.0, 0.0);
    return QRX_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
// ---- batched: plans and the persistent work-queue launch ---------------------
struct qrx_batch_plan_s {
    int device = -1;
    int batch = 0, lls = 0, prec = 0, max_iter = 0;
    double tol = 0.0;
    size_t work_bytes = 0;         // counter + per-problem storage
    void *tables = nullptr;        // device: BEntry[batch] | int order[batch] | BOp ops[]
    BEntry *ent = nullptr;
    int *order = nullptr;
    BOp *ops = nullptr;
};

namespace {

int resolve_batched(const qrx_qr_opts *o, QrCfg &c) {
    qrx_qr_opts z;
    memset(&z, 0, sizeof(z));
    if (!o) o = &z;
    if (o->gemm_prec != QRX_FP32 && o->gemm_prec != QRX_BF16) return QRX_EINVAL;
    if (o->panel_alg != 0 || o->panel_single_pass != 0 || o->node_reorth == 1) return QRX_EINVAL;
    if (o->panel_width != 0 && o->panel_width != kBPanel) return QRX_EINVAL;
    if (o->cutoff < 0 || o->block_rows < 0) return QRX_EINVAL;
    if (o->no_col_scaling < 0 || o->no_col_scaling > 1) return QRX_EINVAL;
    if (o->gemm_tiles < 0 || o->gemm_tiles > 1) return QRX_EINVAL;
    if (o->split_target != 0 || o->q_reorth != 0) return QRX_EINVAL;
    c.prec = o->gemm_prec;
    c.alg = 0;
    c.nb = kBPanel;
    c.tiles = o->gemm_tiles;
    c.split_target = 0;
    int cut = o->cutoff ? o->cutoff : 64;
    if (cut < c.nb) cut = c.nb;
    c.c = (int)round_up(cut, c.nb);
    c.reorth = 1;
    c.scaling = 0;
    c.node_reorth = 0;
    c.qreorth = 0;
    return QRX_OK;
}

}  // namespace

namespace qrx {
int handle_device(qrx_handle h) { return h ? h->device : -1; }
int batched_opts_check(const qrx_qr_opts *o) {
    QrCfg c;
    return resolve_batched(o, c);
}
}  // namespace qrx

// Workspace of qrx_qr_factor_noalloc: a static device array (one per GPU, held
// until the process ends). In host code `scratch` names a host-side stand-in,
// not device memory: only the address hipGetSymbolAddress returns for the
// current device may be handed to kernels.
static __device__ __align__(256) unsigned char scratch[QRX_NOALLOC_SCRATCH_BYTES];

// That address for `device` (which must be current), looked up once per device.
static int scratch_address(int device, void **out) {
    static std::mutex mu;
    static std::map<int, void *> addr;
    std::lock_guard<std::mutex> lock(mu);
    auto it = addr.find(device);
    if (it == addr.end()) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr)
            return QRX_EHIP;
        it = addr.emplace(device, p).first;
    }
    *out = it->second;
    return QRX_OK;
}

extern "C" {

const char *qrx_status_string(int st) {
    switch (st) {
        case QRX_OK: return "QRX_OK: success";
        case QRX_EINVAL: return "QRX_EINVAL: invalid argument";
        case QRX_ENOMEM: return "QRX_ENOMEM: device allocation failed";
        case QRX_EHIP: return "QRX_EHIP: HIP runtime error";
        case QRX_ESINGULAR: return "QRX_ESINGULAR: R has a zero or non-finite diagonal entry";
        case QRX_ENONFINITE: return "QRX_ENONFINITE: input holds NaN or Inf";
        case QRX_ENOCONV: return "QRX_ENOCONV: iteration limit reached above tolerance";
        default: return "unknown qrx status";
    }
}

int qrx_create(qrx_handle *out, int device) {
    if (!out) return QRX_EINVAL;
    *out = nullptr;
    qrx_handle h = new qrx_handle_s();
    h->device = device;
    if (device >= 0) {
        int count = 0;
        if (hipGetDeviceCount(&count) != hipSuccess || device >= count ||
            hipSetDevice(device) != hipSuccess || scratch_address(device, &h->scratch_ptr)) {
            delete h;
            return QRX_EHIP;
        }
    }
    *out = h;
    return QRX_OK;
}

int qrx_destroy(qrx_handle h) {
    if (!h) return QRX_EINVAL;
    if (h->device >= 0) {
        hipSetDevice(h->device);
        for (auto &p : h->pending) {
            hipEventDestroy(p.a);
            hipEventDestroy(p.b);
        }
        for (auto e : h->spare) hipEventDestroy(e);
        if (h->pool) hipFree(h->pool);
        for (void *p : h->retired) hipFree(p);
        for (auto &p : h->phase_pending) hipHostFree(p.buf);
        for (long long *p : h->phase_spare) hipHostFree(p);
    }
    delete h;
    return QRX_OK;
}

int qrx_qr_workspace_size(qrx_handle h, int64_t m, int64_t n, const qrx_qr_opts *opts,
                          size_t *bytes) {
    if (!bytes) return QRX_EINVAL;
    int rc = check_qr_args(h, m, n, m, n);
    if (rc) return rc;
    QrCfg c;
    if ((rc = resolve_qr(opts, c))) return rc;
    std::vector<Op> ops;
    plan_rec(0, n, c, ops);
    Carve cv(nullptr);
    QrWork w;
    carve_qr(cv, m, n, c, ops, w);
    *bytes = cv.off + 256;
    return QRX_OK;
}

static int qr_common(qrx_handle h, int64_t m, int64_t n, const float *A, int64_t lda,
                     float *Q, int64_t ldq, float *R, int64_t ldr, void *work,
                     size_t work_bytes, const qrx_qr_opts *opts, int *status,
                     hipStream_t stream) {
    int rc = check_qr_args(h, m, n, lda, ldr);
    if (rc) return rc;
    if (ldq < m) return QRX_EINVAL;
    if (bad_ptr(A) || bad_ptr(R) || bad_ptr(Q)) return QRX_EINVAL;
    QrCfg c;
    if ((rc = resolve_qr(opts, c))) return rc;
    std::vector<Op> ops;
    plan_rec(0, n, c, ops);
    size_t need = 0;
    {
        Carve cv(nullptr);
        QrWork w;
        carve_qr(cv, m, n, c, ops, w);
        need = cv.off + 256;
    }
    if (work && work_bytes < need) return QRX_EINVAL;
    if (h->device < 0) return QRX_EHIP;
    if (hipSetDevice(h->device) != hipSuccess) return QRX_EHIP;
    if (!work) {
        if ((rc = ensure_pool(h, need, &work))) return rc;
    }
    Carve cv(work);
    QrWork ws;
    carve_qr(cv, m, n, c, ops, ws);
    // status flags cleared by a kernel (the call stays safe to record in a HIP graph)
    QRX_TRY(launch_fill_f32(stream, reinterpret_cast<float *>(ws.flags), 4, 0.0f));
    {
        Rec r(h, stream);
        const bool copy = (Q != A);
        QRX_TRY(launch_scan(stream, m, n, A, lda, copy ? Q : nullptr, ldq, ws.colmax, ws.colss,
                            ws.flags));
        r.end("scan", 0, (copy ? 8.0 : 4.0) * m * n);
    }
    if ((rc = run_qr(h, stream, m, n, Q, ldq, R, ldr, c, ops, ws))) return rc;
    {
        Rec r(h, stream);
        QRX_TRY(launch_r_finalize(stream, n, R, ldr, ws.flags));
        r.end("r_finalize", 0, 4.0 * n * n);
    }
    if (c.qreorth) {
        // whole-Q re-orthogonalisation: Q = Q2 R2 by the same factorisation, R <- R2 R
        {
            Rec r(h, stream);
            QRX_TRY(launch_scan(stream, m, n, Q, ldq, nullptr, ldq, ws.colmax, ws.colss,
                                ws.flags));
            r.end("scan", 0, 4.0 * m * n);
        }
        if ((rc = run_qr(h, stream, m, n, Q, ldq, ws.r2, n, c, ops, ws))) return rc;
        {
            Rec r(h, stream);
            QRX_TRY(launch_r_finalize(stream, n, ws.r2, n, ws.flags));
            QRX_TRY(launch_triu_mul(stream, n, ws.r2, n, R, ldr, ws.r3, n));
            QRX_TRY(launch_copy_mat(stream, n, n, ws.r3, n, R, ldr));
            r.end("q_reorth_r", 2.0 * n * n * n / 6.0, 20.0 * n * n);
        }
    }
    if (status) QRX_TRY(launch_status_out(stream, ws.flags, status));
    return QRX_OK;
}

int qrx_qr_factor(qrx_handle h, int64_t m, int64_t n, float *A, int64_t lda, float *R,
                  int64_t ldr, void *work, size_t work_bytes, const qrx_qr_opts *opts,
                  int *status, hipStream_t stream) {
    return qr_common(h, m, n, A, lda, A, lda, R, ldr, work, work_bytes, opts, status, stream);
}

int qrx_qr_factor_out(qrx_handle h, int64_t m, int64_t n, const float *A, int64_t lda,
                      float *Q, int64_t ldq, float *R, int64_t ldr, void *work,
                      size_t work_bytes, const qrx_qr_opts *opts, int *status,
                      hipStream_t stream) {
    return qr_common(h, m, n, A, lda, Q, ldq, R, ldr, work, work_bytes, opts, status, stream);
}

int qrx_qr_factor_noalloc(qrx_handle h, int64_t m, int64_t n, float *A, int64_t lda, float *R,
                          int64_t ldr, const qrx_qr_opts *opts, int *status,
                          hipStream_t stream) {
    if (!h) return QRX_EINVAL;
    if (h->timing) return QRX_EINVAL;   // per-kernel timing creates HIP events
    if (h->device < 0 || !h->scratch_ptr) return QRX_EHIP;
    // qr_common rejects a workspace smaller than the problem needs (QRX_EINVAL)
    return qr_common(h, m, n, A, lda, A, lda, R, ldr, h->scratch_ptr, QRX_NOALLOC_SCRATCH_BYTES,
                     opts, status, stream);
}

static int lls_sizes(int64_t m, int64_t n, const QrCfg &c, const std::vector<Op> &ops,
                     bool with_qr, bool precond, size_t *bytes) {
    Carve cv(nullptr);
    QrWork w;
    carve_qr(cv, m, n, c, ops, w);
    if (with_qr) {
        cv.take<float>((size_t)round_up(m, 64) * n);
        cv.take<float>((size_t)round_up(n, 64) * n);
    }
    KrWork k;
    carve_kr(cv, m, n, precond, k);
    *bytes = cv.off + 256;
    return QRX_OK;
}

int qrx_lls_workspace_size(qrx_handle h, int64_t m, int64_t n, const qrx_lls_opts *opts,
                           size_t *bytes) {
    if (!bytes) return QRX_EINVAL;
    int rc = check_qr_args(h, m, n, m, n);
    if (rc) return rc;
    QrCfg c;
    KrCfg kc;
    if ((rc = resolve_qr(opts ? &opts->qr : nullptr, c, true))) return rc;
    if ((rc = resolve_lls(opts, kc))) return rc;
    std::vector<Op> ops;
    plan_rec(0, n, c, ops);
    return lls_sizes(m, n, c, ops, true, true, bytes);
}

static int lls_common(qrx_handle h, int64_t m, int64_t n, const float *A, int64_t lda,
                      const float *Rin, int64_t ldr, bool with_qr, const double *b, double *x,
                      void *work, size_t work_bytes, const qrx_lls_opts *opts,
                      qrx_lls_info *info, hipStream_t stream) {
    int rc = check_qr_args(h, m, n, lda, with_qr ? n : ldr);
    if (rc) return rc;
    if (bad_ptr(A) || bad_ptr(b) || bad_ptr(x) || !info) return QRX_EINVAL;
    QrCfg c;
    KrCfg kc;
    if ((rc = resolve_qr(opts ? &opts->qr : nullptr, c, true))) return rc;
    if ((rc = resolve_lls(opts, kc))) return rc;
    std::vector<Op> ops;
    plan_rec(0, n, c, ops);
    const bool precond = with_qr || Rin != nullptr;
    size_t need = 0;
    lls_sizes(m, n, c, ops, with_qr, precond, &need);
    if (work && work_bytes < need) return QRX_EINVAL;
    if (h->device < 0) return QRX_EHIP;
    if (hipSetDevice(h->device) != hipSuccess) return QRX_EHIP;
    if (!work) {
        if ((rc = ensure_pool(h, need, &work))) return rc;
    }
    Carve cv(work);
    QrWork ws;
    carve_qr(cv, m, n, c, ops, ws);
    float *W = nullptr, *R = const_cast<float *>(Rin);
    int64_t ldw = round_up(m, 64), ldR = ldr;
    if (with_qr) {
        W = cv.take<float>((size_t)ldw * n);
        ldR = round_up(n, 64);
        R = cv.take<float>((size_t)ldR * n);
    }
    KrWork kw;
    carve_kr(cv, m, n, precond, kw);

    // status flags cleared by a kernel (the call stays safe to record in a HIP graph)
    QRX_TRY(launch_fill_f32(stream, reinterpret_cast<float *>(ws.flags), 4, 0.0f));
    {
        Rec r(h, stream);
        QRX_TRY(launch_scan(stream, m, n, A, lda, W, ldw, ws.colmax, ws.colss, ws.flags));
        QRX_TRY(launch_scan_vec(stream, m, b, ws.flags));
        QRX_TRY(launch_norm_finalize(stream, n, ws.colss, ws.normA));
        r.end("scan", 0, (with_qr ? 8.0 : 4.0) * m * n);
    }
    if (with_qr) {
        if ((rc = run_qr(h, stream, m, n, W, ldw, R, ldR, c, ops, ws))) return rc;
        Rec r(h, stream);
        QRX_TRY(launch_r_finalize(stream, n, R, ldR, ws.flags));
        r.end("r_finalize", 0, 4.0 * n * n);
    }
    return enqueue_krylov(h, stream, m, n, A, lda, R, ldR, b, x, opts && opts->use_x0,
                          with_qr ? W : nullptr, ldw, kc, kw, ws, info);
}

int qrx_lls_solve(qrx_handle h, int64_t m, int64_t n, const float *A, int64_t lda,
                  const double *b, double *x, void *work, size_t work_bytes,
                  const qrx_lls_opts *opts, qrx_lls_info *info, hipStream_t stream) {
    return lls_common(h, m, n, A, lda, nullptr, n, true, b, x, work, work_bytes, opts, info,
                      stream);
}

int qrx_lls_solve_with_R(qrx_handle h, int64_t m, int64_t n, const float *A, int64_t lda,
                         const float *R, int64_t ldr, const double *b, double *x, void *work,
                         size_t work_bytes, const qrx_lls_opts *opts, qrx_lls_info *info,
                         hipStream_t stream) {
    if (R && ldr < n) return QRX_EINVAL;
    return lls_common(h, m, n, A, lda, R, R ? ldr : n, false, b, x, work, work_bytes, opts, info,
                      stream);
}

int qrx_batch_plan_create(qrx_handle h, int batch, const int64_t *m, const int64_t *n,
                          const int *cutoff, const int *tiles, const qrx_lls_opts *opts, int lls,
                          qrx_batch_plan *plan) {
    if (!h || !plan || batch < 1 || !m || !n || (lls != 0 && lls != 1)) return QRX_EINVAL;
    *plan = nullptr;
    QrCfg c;
    int rc = resolve_batched(opts ? &opts->qr : nullptr, c);
    if (rc) return rc;
    KrCfg kc;
    memset(&kc, 0, sizeof(kc));
    if (lls) {
        if ((rc = resolve_lls(opts, kc))) return rc;
        if (opts && (opts->method != 0 || opts->use_x0)) return QRX_EINVAL;
    }
    std::vector<BEntry> ent(batch);
    std::vector<BOp> ops;
    std::map<std::pair<int64_t, int>, std::pair<int, int>> sched;   // (n, cutoff) -> slice
    std::vector<double> cost(batch);
    // the two work-queue heads, then the per-problem QR records (least squares)
    size_t off = 256 + (lls ? sizeof(BRes) * (size_t)batch : 0);
    auto take = [&](size_t bytes) {
        off = (off + 255) / 256 * 256;
        const size_t at = off;
        off += bytes;
        return (int64_t)at;
    };
    for (int i = 0; i < batch; ++i) {
        if (n[i] < 1 || n[i] > kBMaxN || m[i] < n[i] || m[i] > ((int64_t)1 << 31)) return QRX_EINVAL;
        int ci = cutoff ? cutoff[i] : c.c;
        if (ci < 1) return QRX_EINVAL;
        ci = (int)round_up(ci < c.nb ? c.nb : ci, c.nb);
        const int ti = tiles ? tiles[i] : c.tiles;
        if (ti < 0 || ti > 1) return QRX_EINVAL;
        auto key = std::make_pair(n[i], ci);
        auto it = sched.find(key);
        if (it == sched.end()) {
            QrCfg ck = c;
            ck.c = ci;
            std::vector<Op> o2;
            plan_rec(0, n[i], ck, o2);
            const int start = (int)ops.size();
            for (const Op &op : o2)
                ops.push_back({op.kind, (int)op.c0, (int)op.k, (int)op.n2,
                               op.kind == 1 && op.prec != QRX_FP32 ? 1 : 0});
            it = sched.emplace(key, std::make_pair(start, (int)o2.size())).first;
        }
        BEntry &e = ent[i];
        memset(&e, 0, sizeof(e));
        e.m = m[i];
        e.n = n[i];
        e.op0 = it->second.first;
        e.nops = it->second.second;
        e.tiles = ti;
        if (lls) {
            e.ldw = round_up(m[i], 4);
            e.w_off = take(sizeof(float) * (size_t)e.ldw * (size_t)n[i]);
            e.r_off = take(sizeof(float) * (size_t)n[i] * (size_t)n[i]);
            e.v_off = take(2 * sizeof(double) * (size_t)m[i]);
        }
        const double mm = (double)m[i], nn = (double)n[i];
        cost[i] = mm * nn * nn + (lls ? 40.0 * mm * nn : 0.0);
    }
    std::vector<int> order(batch);
    for (int i = 0; i < batch; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
    if (h->device < 0 || hipSetDevice(h->device) != hipSuccess) return QRX_EHIP;
    qrx_batch_plan p = new qrx_batch_plan_s();
    p->device = h->device;
    p->batch = batch;
    p->lls = lls;
    p->prec = c.prec;
    p->tol = kc.tol;
    p->max_iter = kc.max_iter;
    p->work_bytes = off + 256;
    const size_t eb = sizeof(BEntry) * (size_t)batch;
    const size_t ob = (sizeof(int) * (size_t)batch + 255) / 256 * 256;
    const size_t pb = sizeof(BOp) * ops.size();
    if (hipMalloc(&p->tables, eb + ob + pb) != hipSuccess) {
        delete p;
        return QRX_ENOMEM;
    }
    p->ent = reinterpret_cast<BEntry *>(p->tables);
    p->order = reinterpret_cast<int *>((char *)p->tables + eb);
    p->ops = reinterpret_cast<BOp *>((char *)p->tables + eb + ob);
    if (hipMemcpy(p->ent, ent.data(), eb, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(p->order, order.data(), sizeof(int) * (size_t)batch, hipMemcpyHostToDevice) !=
            hipSuccess ||
        hipMemcpy(p->ops, ops.data(), pb, hipMemcpyHostToDevice) != hipSuccess) {
        hipFree(p->tables);
        delete p;
        return QRX_EHIP;
    }
    *plan = p;
    return QRX_OK;
}

int qrx_batch_plan_workspace_size(qrx_batch_plan plan, size_t *bytes) {
    if (!plan || !bytes) return QRX_EINVAL;
    *bytes = plan->work_bytes;
    return QRX_OK;
}

int qrx_batch_plan_destroy(qrx_batch_plan plan) {
    if (!plan) return QRX_EINVAL;
    if (plan->tables) {
        hipSetDevice(plan->device);
        hipFree(plan->tables);
    }
    delete plan;
    return QRX_OK;
}

static int batched_common(qrx_handle h, qrx_batch_plan plan, int lls, const float *const *A,
                          const int64_t *lda, float *const *R, const int64_t *ldr,
                          const double *const *b, double *const *x, void *work,
                          size_t work_bytes, int *status, qrx_lls_info *info,
                          hipStream_t stream) {
    if (!h || !plan || plan->lls != lls || !A || !lda) return QRX_EINVAL;
    if (lls ? (!b || !x || !info) : (!R || !ldr || !status)) return QRX_EINVAL;
    if (h->device < 0 || h->device != plan->device) return QRX_EINVAL;
    if (work && work_bytes < plan->work_bytes) return QRX_EINVAL;
    if (hipSetDevice(h->device) != hipSuccess) return QRX_EHIP;
    int rc;
    if (!work && (rc = ensure_pool(h, plan->work_bytes, &work))) return rc;
    BArgs a;
    memset(&a, 0, sizeof(a));
    a.ent = plan->ent;
    a.order = plan->order;
    a.ops = plan->ops;
    a.batch = plan->batch;
    a.lls = lls;
    a.A = A;
    a.lda = lda;
    a.R = R;
    a.ldr = ldr;
    a.b = b;
    a.x = x;
    a.work = reinterpret_cast<char *>(work);
    a.counter = reinterpret_cast<unsigned *>(work);
    a.res = lls ? reinterpret_cast<BRes *>(reinterpret_cast<char *>(work) + 256) : nullptr;
    a.status = status;
    a.info = info;
    a.tol = plan->tol;
    a.max_iter = plan->max_iter;
    // the work-queue heads are cleared by a kernel (the call stays safe to record in a graph)
    QRX_TRY(launch_fill_f32(stream, reinterpret_cast<float *>(work), 2, 0.0f));
    Rec r(h, stream);
    QRX_TRY(launch_bsolve(stream, h->device, plan->prec, a));
    r.end(lls ? "batched_lls" : "batched_qr", 0.0, 0.0);
    return QRX_OK;
}

int qrx_qr_factor_batched(qrx_handle h, qrx_batch_plan plan, float *const *A, const int64_t *lda,
                          float *const *R, const int64_t *ldr, void *work, size_t work_bytes,
                          int *status, hipStream_t stream) {
    return batched_common(h, plan, 0, const_cast<const float *const *>(A), lda, R, ldr, nullptr,
                          nullptr, work, work_bytes, status, nullptr, stream);
}

int qrx_lls_solve_batched(qrx_handle h, qrx_batch_plan plan, const float *const *A,
                          const int64_t *lda, const double *const *b, double *const *x,
                          void *work, size_t work_bytes, qrx_lls_info *info, hipStream_t stream) {
    return batched_common(h, plan, 1, A, lda, nullptr, nullptr, b, x, work, work_bytes, nullptr,
                          info, stream);
}

int qrx_timing_enable(qrx_handle h, int enable) {
    if (!h) return QRX_EINVAL;
    h->timing = enable != 0;
    return QRX_OK;
}

static int drain_timing(qrx_handle h) {
    for (auto &p : h->pending) {
        if (hipEventSynchronize(p.b) != hipSuccess) return QRX_EHIP;
        float ms = 0.f;
        hipEventElapsedTime(&ms, p.a, p.b);
        qrx_kernel_stat &s = h->stats[p.name];
        if (s.launches == 0) {
            memset(&s, 0, sizeof(s));
            strncpy(s.name, p.name.c_str(), sizeof(s.name) - 1);
        }
        s.launches += 1;
        s.total_ms += ms;
        s.flops += p.flops;
        s.bytes += p.bytes;
        h->spare.push_back(p.a);
        h->spare.push_back(p.b);
    }
    h->pending.clear();
    // per-phase records of persistent Krylov launches (complete: their launch's
    // closing event has been waited for above)
    static const char *names[KP_COUNT] = {
        "krylov:init", "krylov:certify", "krylov:restart", "krylov:trmv_n", "krylov:gemv_n",
        "krylov:combine_m", "krylov:gemv_t", "krylov:combine_n", "krylov:trmv_t",
        "krylov:update", "krylov:fused_pass", "krylov:certify_gemv_n", "krylov:certify_resid",
        "krylov:certify_gemv_t", "krylov:certify_combine"};
    for (auto &p : h->phase_pending) {
        const double mn = (double)p.m * (double)p.n, tri = (double)p.np * (p.np + 1) / 2.0;
        for (int ph = 0; ph < KP_COUNT; ++ph) {
            const long long calls = p.buf[KP_COUNT + ph];
            if (calls == 0) continue;
            double fl = 0.0, by = 0.0;   // algorithmic work per call
            switch (ph) {
                case KP_GEMV_N: fl = 2.0 * mn; by = 4.0 * mn + 8.0 * p.splits_n * p.m; break;
                case KP_GEMV_T: fl = 2.0 * mn; by = 4.0 * mn + 8.0 * p.m + 8.0 * p.splits_t * p.n; break;
                case KP_TRMV_N:
                case KP_TRMV_T: fl = 2.0 * tri; by = 8.0 * tri + 16.0 * p.np; break;
                case KP_COMBINE_M: by = 8.0 * p.splits_n * p.m + 16.0 * p.m; break;
                case KP_COMBINE_N:
                    by = 8.0 * (p.fused ? p.grid : p.splits_t) * p.n + 8.0 * p.n;
                    break;
                // A once, u~_old read and u~ written, one n-vector of partials per workgroup
                case KP_FUSED: fl = 4.0 * mn; by = 4.0 * mn + 16.0 * p.m + 8.0 * p.grid * p.n; break;
                // certification: A x in double-double (hi and lo partials), the residual
                // from b and the partials, A^T r, the column sums
                case KP_CERT_GEMV_N: fl = 2.0 * mn; by = 4.0 * mn + 16.0 * p.splits_n * p.m; break;
                case KP_CERT_RESID: by = 16.0 * p.splits_n * p.m + 16.0 * p.m; break;
                case KP_CERT_GEMV_T: fl = 2.0 * mn; by = 4.0 * mn + 8.0 * p.m + 8.0 * p.splits_t * p.n; break;
                case KP_CERT_COMBINE: by = 8.0 * p.splits_t * p.n + 8.0 * p.n; break;
                default: break;
            }
            qrx_kernel_stat &s = h->stats[names[ph]];
            if (s.launches == 0) {
                memset(&s, 0, sizeof(s));
                strncpy(s.name, names[ph], sizeof(s.name) - 1);
            }
            s.launches += calls;
            s.total_ms += (double)p.buf[ph] / p.khz;
            s.flops += fl * calls;
            s.bytes += by * calls;
        }
        h->phase_spare.push_back(p.buf);
    }
    h->phase_pending.clear();
    return QRX_OK;
}

int qrx_timing_reset(qrx_handle h) {
    if (!h) return QRX_EINVAL;
    int rc = drain_timing(h);
    h->stats.clear();
    return rc;
}

int qrx_timing_get(qrx_handle h, qrx_kernel_stat *out, int capacity, int *count) {
    if (!h || !count || (capacity > 0 && !out)) return QRX_EINVAL;
    int rc = drain_timing(h);
    if (rc) return rc;
    int i = 0;
    for (auto &kv : h->stats) {
        if (i < capacity) out[i] = kv.second;
        ++i;
    }
    *count = i;
    return QRX_OK;
}

}  // extern "C"
