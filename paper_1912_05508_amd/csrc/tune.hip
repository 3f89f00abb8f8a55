// Autotuning of the blocking parameters, and its JSON cache.
//
// The paper fixes the recursion cutoff (128), the panel width (32) and the
// TSQR block (256 rows) for its GPU (Sec. 3.1.3). Here they are measured per
// size class: a coordinate search from the defaults, one parameter at a time
// (panel width, cutoff, tile family of the low-precision products, split
// target of the projections), each candidate timed with HIP events on the
// caller's stream, the median of `reps` runs kept; a candidate replaces the
// current choice when it is at least 1% faster. At most two passes.
// The cache is a small JSON file, one entry per line, keyed by
// "<arch>/<prec>/<gram|tsqr|batched>/m<ceil log2 m>/n<ceil log2 n>".
#include "qrx_internal.hpp"

#include <algorithm>
#include <map>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

namespace qrx {
namespace {

const char *prec_name(int p) {
    switch (p) {
        case QRX_FP32: return "fp32";
        case QRX_FP16: return "fp16";
        case QRX_BF16: return "bf16";
        case QRX_FP16X3: return "fp16x3";
        default: return nullptr;
    }
}

int ceil_log2(int64_t v) {
    int l = 0;
    while (((int64_t)1 << l) < v) ++l;
    return l;
}

struct Entry {
    std::string key;
    qrx_tune_result r;
};

// 0: parsed (entries may be empty), QRX_EINVAL: not a cache of this library.
int read_cache(const char *path, std::vector<Entry> &out, bool &exists) {
    out.clear();
    exists = false;
    FILE *f = fopen(path, "r");
    if (!f) return QRX_OK;
    exists = true;
    std::string text;
    char buf[4096];
    size_t got;
    while ((got = fread(buf, 1, sizeof(buf), f)) > 0) text.append(buf, got);
    fclose(f);
    if (text.find_first_not_of(" \t\r\n") == std::string::npos) return QRX_OK;   // empty file
    if (text.find("\"qrx_tune\"") == std::string::npos) return QRX_EINVAL;
    size_t pos = 0;
    while (pos < text.size()) {
        size_t eol = text.find('\n', pos);
        if (eol == std::string::npos) eol = text.size();
        const std::string line = text.substr(pos, eol - pos);
        pos = eol + 1;
        if (line.find("{\"key\": \"") == std::string::npos) continue;
        char key[256];
        Entry e;
        memset(&e.r, 0, sizeof(e.r));
        const int n = sscanf(line.c_str(),
                             " {\"key\": \"%255[^\"]\", \"panel_width\": %d, \"cutoff\": %d, "
                             "\"gemm_tiles\": %d, \"split_target\": %d, \"ms\": %lf}",
                             key, &e.r.panel_width, &e.r.cutoff, &e.r.gemm_tiles,
                             &e.r.split_target, &e.r.ms);
        if (n != 6) return QRX_EINVAL;
        e.key = key;
        out.push_back(e);
    }
    return QRX_OK;
}

int write_cache(const char *path, const std::vector<Entry> &es) {
    const std::string tmp = std::string(path) + ".tmp";
    FILE *f = fopen(tmp.c_str(), "w");
    if (!f) return QRX_EINVAL;
    fprintf(f, "{\"qrx_tune\": [\n");
    for (size_t i = 0; i < es.size(); ++i) {
        const qrx_tune_result &r = es[i].r;
        fprintf(f,
                "  {\"key\": \"%s\", \"panel_width\": %d, \"cutoff\": %d, \"gemm_tiles\": %d, "
                "\"split_target\": %d, \"ms\": %.6f}%s\n",
                es[i].key.c_str(), r.panel_width, r.cutoff, r.gemm_tiles, r.split_target, r.ms,
                i + 1 < es.size() ? "," : "");
    }
    fprintf(f, "]}\n");
    const bool ok = fclose(f) == 0;
    if (!ok || rename(tmp.c_str(), path) != 0) {
        remove(tmp.c_str());
        return QRX_EINVAL;
    }
    return QRX_OK;
}

bool device_arch(qrx_handle h, char *arch, size_t len) {
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, handle_device(h)) != hipSuccess) return false;
    size_t i = 0;
    for (; i + 1 < len && p.gcnArchName[i] && p.gcnArchName[i] != ':'; ++i) arch[i] = p.gcnArchName[i];
    arch[i] = 0;
    return i > 0;
}

// Median device time of `reps` runs of f() on stream s (after one warm-up run);
// a negative return is f's error.
template <class F>
int time_median(hipStream_t s, int reps, F f, double &ms) {
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess) return QRX_EHIP;
    if (hipEventCreate(&b) != hipSuccess) {
        hipEventDestroy(a);
        return QRX_EHIP;
    }
    int rc = f();
    std::vector<double> ts;
    for (int r = 0; rc == QRX_OK && r < reps; ++r) {
        if (hipEventRecord(a, s) != hipSuccess) { rc = QRX_EHIP; break; }
        rc = f();
        if (rc != QRX_OK) break;
        if (hipEventRecord(b, s) != hipSuccess || hipEventSynchronize(b) != hipSuccess) {
            rc = QRX_EHIP;
            break;
        }
        float t = 0.f;
        if (hipEventElapsedTime(&t, a, b) != hipSuccess) { rc = QRX_EHIP; break; }
        ts.push_back(t);
    }
    if (rc == QRX_OK && hipStreamSynchronize(s) != hipSuccess) rc = QRX_EHIP;
    hipEventDestroy(a);
    hipEventDestroy(b);
    if (rc != QRX_OK) return rc;
    std::sort(ts.begin(), ts.end());
    ms = ts[ts.size() / 2];
    return QRX_OK;
}

struct Cand {
    int nb, c, tiles, split;
    bool operator==(const Cand &o) const {
        return nb == o.nb && c == o.c && tiles == o.tiles && split == o.split;
    }
};

// Coordinate search: lists[p] are the values of parameter p; run(cand, ms)
// times one candidate (QRX_EINVAL = unsupported, skipped).
template <class Run>
int coord_search(const std::vector<std::vector<int>> &lists, Cand cur, Run run, Cand &best,
                 double &best_ms, int &trials) {
    trials = 0;
    int rc = run(cur, best_ms);
    ++trials;
    if (rc != QRX_OK) return rc;
    std::vector<Cand> seen{cur};
    for (int pass = 0; pass < 2; ++pass) {
        bool improved = false;
        for (size_t p = 0; p < lists.size(); ++p) {
            for (int v : lists[p]) {
                Cand c = cur;
                int *field = p == 0 ? &c.nb : p == 1 ? &c.c : p == 2 ? &c.tiles : &c.split;
                *field = v;
                if (std::find(seen.begin(), seen.end(), c) != seen.end()) continue;
                seen.push_back(c);
                double ms = 0.0;
                rc = run(c, ms);
                ++trials;
                if (rc == QRX_EINVAL) continue;
                if (rc != QRX_OK) return rc;
                if (ms < 0.99 * best_ms) {
                    best_ms = ms;
                    cur = c;
                    improved = true;
                }
            }
        }
        if (!improved) break;
    }
    best = cur;
    return QRX_OK;
}

int cache_lookup(const char *path, const char *key, qrx_tune_result *out) {
    std::vector<Entry> es;
    bool exists;
    const int rc = read_cache(path, es, exists);
    if (rc != QRX_OK) return rc;
    for (const Entry &e : es)
        if (e.key == key) {
            *out = e.r;
            out->trials = 0;
            out->from_cache = 1;
            return QRX_OK;
        }
    return 1;
}

}  // namespace
}  // namespace qrx

using namespace qrx;

extern "C" {

int qrx_tune_key(const char *arch, int64_t m, int64_t n, int prec, int kind, char *buf,
                 size_t len) {
    const char *pn = prec_name(prec);
    if (!arch || !buf || !pn || m < 1 || n < 1 || kind < 0 || kind > 2) return QRX_EINVAL;
    const char *tag = kind == 1 ? "batched" : (kind == 2 ? "tsqr" : "gram");
    const int w = snprintf(buf, len, "%s/%s/%s/m%d/n%d", arch, pn, tag, ceil_log2(m), ceil_log2(n));
    if (w < 0 || (size_t)w >= len) return QRX_EINVAL;
    for (const char *q = buf; *q; ++q)
        if (*q == '"' || *q == '\\' || *q == '\n') return QRX_EINVAL;
    return QRX_OK;
}

int qrx_tune_cache_get(const char *cache_path, const char *key, qrx_tune_result *out) {
    if (!cache_path || !key || !out) return QRX_EINVAL;
    return cache_lookup(cache_path, key, out);
}

int qrx_tune_cache_put(const char *cache_path, const char *key, const qrx_tune_result *r) {
    if (!cache_path || !key || !r) return QRX_EINVAL;
    for (const char *q = key; *q; ++q)
        if (*q == '"' || *q == '\\' || *q == '\n') return QRX_EINVAL;
    std::vector<Entry> es;
    bool exists;
    int rc = read_cache(cache_path, es, exists);
    if (rc != QRX_OK) return rc;
    bool found = false;
    for (Entry &e : es)
        if (e.key == key) {
            e.r = *r;
            found = true;
        }
    if (!found) es.push_back({key, *r});
    return write_cache(cache_path, es);
}

int qrx_tune(qrx_handle h, int64_t m, int64_t n, const float *A, int64_t lda,
             const qrx_qr_opts *base, int reps, const char *cache_path, qrx_tune_result *out,
             hipStream_t stream) {
    if (!h || !A || !out || n < 1 || m < n || lda < m || reps < 1 || reps > 20) return QRX_EINVAL;
    qrx_qr_opts b0;
    memset(&b0, 0, sizeof(b0));
    if (base) b0 = *base;
    size_t probe = 0;
    int rc = qrx_qr_workspace_size(h, m, n, &b0, &probe);   // validates the base options
    if (rc != QRX_OK) return rc;
    if (handle_device(h) < 0) return QRX_EHIP;
    memset(out, 0, sizeof(*out));
    char arch[64], key[256];
    if (!device_arch(h, arch, sizeof(arch))) return QRX_EHIP;
    rc = qrx_tune_key(arch, m, n, b0.gemm_prec, b0.panel_alg == 1 ? 2 : 0, key, sizeof(key));
    if (rc != QRX_OK) return rc;
    if (cache_path) {
        rc = cache_lookup(cache_path, key, out);
        if (rc == QRX_OK) return QRX_OK;
        if (rc != 1) return rc;
    }
    // candidate values; cutoffs below n so that the precision asked for is used
    const bool tsqr = b0.panel_alg == 1;
    std::vector<std::vector<int>> lists(4);
    lists[0] = tsqr ? std::vector<int>{16, 32} : std::vector<int>{32, 64, 128};
    for (int c : {64, 128, 256, 512})
        if (c < n || b0.gemm_prec == QRX_FP32) lists[1].push_back(c);
    lists[2] = {0, 1};
    lists[3] = {0, 128, 256, 512, 1024};
    Cand cur{b0.panel_width ? b0.panel_width : (tsqr ? 32 : 64), b0.cutoff ? b0.cutoff : 128,
             b0.gemm_tiles, b0.split_target};
    auto opts_of = [&](const Cand &c) {
        qrx_qr_opts o = b0;
        o.panel_width = c.nb;
        o.cutoff = c.c;
        o.gemm_tiles = c.tiles;
        o.split_target = c.split;
        return o;
    };
    // scratch: Q, R, status and the largest workspace of any candidate
    size_t wmax = 0;
    for (int nb : lists[0])
        for (int c : lists[1])
            for (int t : lists[2])
                for (int sp : lists[3]) {
                    const qrx_qr_opts o = opts_of(Cand{nb, c, t, sp});
                    size_t b = 0;
                    if (qrx_qr_workspace_size(h, m, n, &o, &b) == QRX_OK) wmax = std::max(wmax, b);
                }
    float *Q = nullptr, *R = nullptr;
    int *st = nullptr;
    void *work = nullptr;
    auto release = [&]() {
        if (Q) (void)hipFree(Q);
        if (R) (void)hipFree(R);
        if (st) (void)hipFree(st);
        if (work) (void)hipFree(work);
    };
    if (hipMalloc(&Q, sizeof(float) * (size_t)m * n) != hipSuccess ||
        hipMalloc(&R, sizeof(float) * (size_t)n * n) != hipSuccess ||
        hipMalloc(&st, sizeof(int)) != hipSuccess ||
        (wmax && hipMalloc(&work, wmax) != hipSuccess)) {
        release();
        return QRX_ENOMEM;
    }
    auto run = [&](const Cand &c, double &ms) -> int {
        const qrx_qr_opts o = opts_of(c);
        size_t b = 0;
        int r2 = qrx_qr_workspace_size(h, m, n, &o, &b);
        if (r2 != QRX_OK) return r2;
        return time_median(stream, reps, [&]() {
            return qrx_qr_factor_out(h, m, n, A, lda, Q, m, R, n, work, wmax, &o, st, stream);
        }, ms);
    };
    Cand best;
    double best_ms = 0.0;
    int trials = 0;
    rc = coord_search(lists, cur, run, best, best_ms, trials);
    release();
    if (rc != QRX_OK) return rc;
    out->panel_width = best.nb;
    out->cutoff = best.c;
    out->gemm_tiles = best.tiles;
    out->split_target = best.split;
    out->ms = best_ms;
    out->trials = trials;
    out->from_cache = 0;
    if (cache_path) return qrx_tune_cache_put(cache_path, key, out);
    return QRX_OK;
}

int qrx_tune_batched(qrx_handle h, int batch, const int64_t *m, const int64_t *n,
                     const float *const *A, const int64_t *lda, const qrx_qr_opts *base,
                     int reps, const char *cache_path, int *cutoff, int *tiles,
                     qrx_tune_result *out, hipStream_t stream) {
    if (!h || batch < 1 || !m || !n || !A || !lda || !cutoff || !tiles || !out || reps < 1 ||
        reps > 20)
        return QRX_EINVAL;
    qrx_lls_opts lo;
    memset(&lo, 0, sizeof(lo));
    if (base) lo.qr = *base;
    // sizes and options are checked before any device work
    for (int i = 0; i < batch; ++i)
        if (!A[i] || lda[i] < m[i] || n[i] < 1 || n[i] > 256 || m[i] < n[i] ||
            m[i] > ((int64_t)1 << 31))
            return QRX_EINVAL;
    if (batched_opts_check(&lo.qr) != QRX_OK) return QRX_EINVAL;
    if (handle_device(h) < 0) return QRX_EHIP;
    memset(out, 0, sizeof(*out));
    char arch[64];
    if (!device_arch(h, arch, sizeof(arch))) return QRX_EHIP;
    // size classes
    std::map<std::pair<int, int>, std::vector<int>> classes;
    for (int i = 0; i < batch; ++i)
        classes[std::make_pair(ceil_log2(m[i]), ceil_log2(n[i]))].push_back(i);
    bool all_cached = true;
    int trials = 0;
    double ms_sum = 0.0;
    hipEvent_t ea = nullptr, eb = nullptr;
    if (hipEventCreate(&ea) != hipSuccess || hipEventCreate(&eb) != hipSuccess) {
        if (ea) (void)hipEventDestroy(ea);
        return QRX_EHIP;
    }
    int rc = QRX_OK;
    for (auto &cl : classes) {
        const std::vector<int> &idx = cl.second;
        const int k = (int)idx.size();
        int64_t mmax = 0, nmax = 0, total = 0, rtot = 0;
        for (int i : idx) {
            mmax = std::max(mmax, m[i]);
            nmax = std::max(nmax, n[i]);
            total += m[i] * n[i];
            rtot += n[i] * n[i];
        }
        char key[256];
        if ((rc = qrx_tune_key(arch, mmax, nmax, lo.qr.gemm_prec, 1, key, sizeof(key)))) break;
        qrx_tune_result r;
        memset(&r, 0, sizeof(r));
        int found = 1;
        if (cache_path) {
            found = cache_lookup(cache_path, key, &r);
            if (found != QRX_OK && found != 1) {
                rc = found;
                break;
            }
        }
        if (found != QRX_OK) {
            all_cached = false;
            // the class's problems as a sub-batch of compact copies
            std::vector<int64_t> ms(k), ns(k), ldw(k), ldr(k);
            std::vector<float *> Aw(k), Rw(k);
            float *pristine = nullptr, *wk = nullptr, *Rb = nullptr;
            void *dev = nullptr, *work = nullptr;
            auto release = [&]() {
                for (void *q : {(void *)pristine, (void *)wk, (void *)Rb, dev, work})
                    if (q) (void)hipFree(q);
            };
            const size_t descb = (size_t)k * (2 * sizeof(void *) + 2 * sizeof(int64_t) + sizeof(int));
            if (hipMalloc(&pristine, sizeof(float) * (size_t)total) != hipSuccess ||
                hipMalloc(&wk, sizeof(float) * (size_t)total) != hipSuccess ||
                hipMalloc(&Rb, sizeof(float) * (size_t)rtot) != hipSuccess ||
                hipMalloc(&dev, descb) != hipSuccess) {
                release();
                rc = QRX_ENOMEM;
                break;
            }
            int64_t off = 0, roff = 0;
            for (int q = 0; q < k; ++q) {
                const int i = idx[q];
                ms[q] = m[i];
                ns[q] = n[i];
                if (hipMemcpy2DAsync(pristine + off, sizeof(float) * m[i], A[i],
                                     sizeof(float) * lda[i], sizeof(float) * m[i], n[i],
                                     hipMemcpyDeviceToDevice, stream) != hipSuccess) {
                    rc = QRX_EHIP;
                    break;
                }
                Aw[q] = wk + off;
                ldw[q] = m[i];
                Rw[q] = Rb + roff;
                ldr[q] = n[i];
                off += m[i] * n[i];
                roff += n[i] * n[i];
            }
            // device descriptor arrays: A | R | lda | ldr | status
            float **dA = reinterpret_cast<float **>(dev);
            float **dR = dA + k;
            int64_t *dlda = reinterpret_cast<int64_t *>(dR + k);
            int64_t *dldr = dlda + k;
            int *dst = reinterpret_cast<int *>(dldr + k);
            if (rc == QRX_OK &&
                (hipMemcpy(dA, Aw.data(), sizeof(void *) * k, hipMemcpyHostToDevice) != hipSuccess ||
                 hipMemcpy(dR, Rw.data(), sizeof(void *) * k, hipMemcpyHostToDevice) != hipSuccess ||
                 hipMemcpy(dlda, ldw.data(), sizeof(int64_t) * k, hipMemcpyHostToDevice) !=
                     hipSuccess ||
                 hipMemcpy(dldr, ldr.data(), sizeof(int64_t) * k, hipMemcpyHostToDevice) !=
                     hipSuccess))
                rc = QRX_EHIP;
            double best_ms = 1e300;
            int best_c = 64, best_t = 0;
            for (int c : {32, 64, 128, 256}) {
                if (rc != QRX_OK) break;
                if (c > 32 && c / 2 >= nmax) break;   // every node is already FP32
                for (int tl : {0, 1}) {
                    if (tl == 1 && c >= nmax) break;  // no low-precision node to tile
                    std::vector<int> cv(k, c), tv(k, tl);
                    qrx_batch_plan plan = nullptr;
                    if ((rc = qrx_batch_plan_create(h, k, ms.data(), ns.data(), cv.data(),
                                                    tv.data(), &lo, 0, &plan)))
                        break;
                    size_t wb = 0;
                    qrx_batch_plan_workspace_size(plan, &wb);
                    if (work) (void)hipFree(work);
                    work = nullptr;
                    if (hipMalloc(&work, wb) != hipSuccess) {
                        qrx_batch_plan_destroy(plan);
                        rc = QRX_ENOMEM;
                        break;
                    }
                    std::vector<double> ts;
                    for (int rep = 0; rep <= reps && rc == QRX_OK; ++rep) {
                        if (hipMemcpyAsync(wk, pristine, sizeof(float) * (size_t)total,
                                           hipMemcpyDeviceToDevice, stream) != hipSuccess ||
                            hipEventRecord(ea, stream) != hipSuccess) {
                            rc = QRX_EHIP;
                            break;
                        }
                        rc = qrx_qr_factor_batched(h, plan, dA, dlda, dR, dldr, work, wb, dst,
                                                   stream);
                        if (rc != QRX_OK) break;
                        float t = 0.f;
                        if (hipEventRecord(eb, stream) != hipSuccess ||
                            hipEventSynchronize(eb) != hipSuccess ||
                            hipEventElapsedTime(&t, ea, eb) != hipSuccess) {
                            rc = QRX_EHIP;
                            break;
                        }
                        if (rep > 0) ts.push_back(t);
                    }
                    qrx_batch_plan_destroy(plan);
                    if (rc != QRX_OK) break;
                    ++trials;
                    std::sort(ts.begin(), ts.end());
                    const double med = ts[ts.size() / 2];
                    if (med < best_ms) {
                        best_ms = med;
                        best_c = c;
                        best_t = tl;
                    }
                }
            }
            release();
            if (rc != QRX_OK) break;
            r.panel_width = 32;
            r.cutoff = best_c;
            r.gemm_tiles = best_t;
            r.split_target = 0;
            r.ms = best_ms;
            r.trials = trials;
            r.from_cache = 0;
            if (cache_path && (rc = qrx_tune_cache_put(cache_path, key, &r))) break;
        }
        ms_sum += r.ms;
        for (int i : idx) {
            cutoff[i] = r.cutoff;
            tiles[i] = r.gemm_tiles;
        }
    }
    (void)hipEventDestroy(ea);
    (void)hipEventDestroy(eb);
    if (rc != QRX_OK) return rc;
    out->panel_width = 32;
    out->cutoff = 0;
    out->gemm_tiles = 0;
    out->split_target = 0;
    out->ms = ms_sum;
    out->trials = trials;
    out->from_cache = all_cached ? 1 : 0;
    return QRX_OK;
}

}  // extern "C"
