// C ABI entry points of the library (declared in include/spmv.h).
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdlib>
#include <cstring>
#include <string>
#include <mutex>
#include <vector>

#include "common.hpp"

namespace spmv {

namespace {
thread_local std::string g_last_error;
}

void set_error(const char *fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
}

void clear_error() { g_last_error.clear(); }

void fail(spmv_status s, const char *fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    throw Error{s};
}

bool valid_format(spmv_format f) { return f >= SPMV_FMT_CSR && f <= SPMV_FMT_BELL; }

bool format_built(const spmv_matrix_s *h, spmv_format f) {
    switch (f) {
        case SPMV_FMT_CSR:
        case SPMV_FMT_COO: return true;
        case SPMV_FMT_ELL: return h->ell.built;
        case SPMV_FMT_HYB: return h->hyb.built;
        case SPMV_FMT_SELL: return h->sell.built;
        case SPMV_FMT_BELL: return h->bell.built;
    }
    return false;
}

void check_runnable(const spmv_matrix_s *h, spmv_format f) {
    if (!h) fail(SPMV_ERR_INVALID_ARG, "NULL handle");
    if (!valid_format(f)) fail(SPMV_ERR_INVALID_ARG, "bad format %d", (int)f);
    if (!format_built(h, f)) fail(SPMV_ERR_NOT_CONVERTED, "format %d not converted", (int)f);
}

// x (n_cols values) and y (n_rows values) are present where the matrix needs them
// and their byte ranges are disjoint.
void check_vectors(const spmv_matrix_s *h, const void *x, const void *y) {
    if (h->n_cols > 0 && !x) fail(SPMV_ERR_INVALID_ARG, "x is NULL");
    if (h->n_rows > 0 && !y) fail(SPMV_ERR_INVALID_ARG, "y is NULL");
    if (x && y && h->n_rows > 0 && h->n_cols > 0) {
        const size_t vs = dtype_size(h->dt);
        const char *xb = (const char *)x, *xe = xb + (size_t)h->n_cols * vs;
        const char *yb = (const char *)y, *ye = yb + (size_t)h->n_rows * vs;
        if (xb < ye && yb < xe) fail(SPMV_ERR_INVALID_ARG, "x and y overlap");
    }
}

void convert(spmv_matrix_s *h, spmv_format f, int32_t param, hipStream_t s) {
    switch (f) {
        case SPMV_FMT_CSR:
        case SPMV_FMT_COO: return;
        case SPMV_FMT_ELL: build_ell(h, s); return;
        case SPMV_FMT_HYB: build_hyb(h, param, s); return;
        case SPMV_FMT_SELL: build_sell(h, param, s); return;
        case SPMV_FMT_BELL:
            build_bell(h, param, s);
            // the variant must fit the new block size
            if (!variant_applicable(h, f, h->variant[f])) h->variant[f] = default_variant(h, f);
            return;
    }
}

double tune_format(spmv_matrix_s *h, spmv_format f, const void *x, void *y, int32_t reps, int flush,
                   int32_t *best_idx, hipStream_t s);  // timing.hip

namespace {

template <class V>
__global__ void fill_kernel(V *p, int64_t n, V v) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        p[i] = v;
}

int env_int(const char *name, int dflt) {
    const char *v = getenv(name);
    return v && *v ? atoi(v) : dflt;
}

// Timing-based choice: every applicable format converted, tuned and timed.
spmv_format select_exhaustive(spmv_matrix_s *h, float scores[SPMV_NUM_FORMATS], hipStream_t s) {
    const size_t vs = dtype_size(h->dt);
    DevBuf x, y;
    x.alloc(std::max<int64_t>(h->n_cols, 1) * vs);
    y.alloc(std::max<int64_t>(h->n_rows, 1) * vs);
    const int64_t nx = std::max<int32_t>(h->n_cols, 1);
    if (h->dt == SPMV_F64) fill_kernel<double><<<256, 256, 0, s>>>(x.as<double>(), nx, 1.0);
    else fill_kernel<float><<<256, 256, 0, s>>>(x.as<float>(), nx, 1.0f);
    SPMV_CHECK_LAUNCH();
    const int reps = std::max(1, env_int("SPMV_TUNE_REPS", 10));
    const int flush = env_int("SPMV_TUNE_FLUSH", 1);
    double best = INFINITY;
    spmv_format bf = SPMV_FMT_CSR;
    for (int fi = 0; fi < SPMV_NUM_FORMATS; ++fi) {
        const spmv_format f = (spmv_format)fi;
        double t = INFINITY;
        bool ok = true;
        if (!format_built(h, f)) {
            try {
                convert(h, f, -1, s);
            } catch (const Error &e) {
                if (e.status != SPMV_ERR_NOT_APPLICABLE) throw;
                ok = false;
                clear_error();
            }
        }
        if (ok) t = tune_format(h, f, x.p, y.p, reps, flush, nullptr, s);
        scores[fi] = (float)t;
        if (t < best) { best = t; bf = f; }
    }
    return bf;
}

// Fixed thresholds on the features (a baseline for the learned selector):
// HYB when a few rows are far longer than the rest and its COO tail stays
// small, COO (the column-sorted block kernel) for large matrices with rows of
// 16 or more entries, ELL when it pads little, CSR otherwise.
spmv_format select_rule(const float f[12], float votes[SPMV_NUM_FORMATS]) {
    const double nnz = f[1], mean = f[2], ell_ratio = f[7], mx = f[8], tail = f[11];
    spmv_format r = SPMV_FMT_CSR;
    if (mean > 0 && mx > 32 * mean && tail < 0.3) r = SPMV_FMT_HYB;
    else if (mean >= 16 && nnz >= 4e6) r = SPMV_FMT_COO;
    else if (ell_ratio >= 0.9) r = SPMV_FMT_ELL;
    for (int i = 0; i < SPMV_NUM_FORMATS; ++i) votes[i] = (i == (int)r) ? 1.f : 0.f;
    return r;
}

}  // namespace

bool prepare_variant(spmv_matrix_s *h, spmv_format f, int32_t idx, hipStream_t s) {
    if (!variant_applicable(h, f, idx)) return false;
    try {
        if (variant_needs_panel(f, idx) && !h->panel.built) build_panel(h, s);
        if (variant_needs_sorted(f, idx) && !h->sorted.built) build_sorted(h, s);
        if (const int T = variant_sorted_tiles(f, idx); T && !h->sorted_tiles[T == 4].built)
            build_sorted_tiles(h, T, s);
        if (variant_needs_split(f, idx) && !h->split.built) build_split(h, s);
        if (variant_needs_csr_blocks(f, idx) && !h->csr_blocks.built) build_csr_blocks(h, s);
        if (variant_needs_hyb_sorted(f, idx) && !h->hyb_sorted.built) build_hyb_sorted(h, s);
    } catch (const Error &e) {
        if (e.status != SPMV_ERR_NOT_APPLICABLE) throw;
        clear_error();
        return false;
    }
    return true;
}

spmv_status model_logits(const float *feats, float scores[SPMV_NUM_FORMATS], int *classes,
                         hipStream_t s);  // mlp.hip

// The network's choice: the highest logit over the formats it has classes for
// (ties to the lowest), ELL left out when its padding cap refuses it; a choice
// whose conversion is refused (SELL, BELL) gives way to the next highest.
spmv_format select_model(spmv_matrix_s *h, const float feats[12], float scores[SPMV_NUM_FORMATS],
                         hipStream_t s) {
    int nc = 0;
    const spmv_status st = model_logits(feats, scores, &nc, s);
    if (st != SPMV_OK) throw Error{st};
    bool allowed[SPMV_NUM_FORMATS];
    for (int i = 0; i < SPMV_NUM_FORMATS; ++i) allowed[i] = i < nc;
    const bool ell_ok = h->nnz == 0 ||
                        (int64_t)((h->n_rows + 63) / 64 * 64) * h->stats.max_len <= 8 * h->nnz;
    allowed[SPMV_FMT_ELL] = allowed[SPMV_FMT_ELL] && ell_ok;
    for (;;) {
        int best = SPMV_FMT_CSR;
        for (int i = 0; i < SPMV_NUM_FORMATS; ++i)
            if (allowed[i] && (!allowed[best] || scores[i] > scores[best])) best = i;
        const spmv_format f = (spmv_format)best;
        if (format_built(h, f)) return f;
        try {
            convert(h, f, -1, s);
            return f;
        } catch (const Error &e) {
            if (e.status != SPMV_ERR_NOT_APPLICABLE) throw;
            clear_error();
            allowed[best] = false;  // CSR and COO always exist, so this ends
        }
    }
}

}  // namespace spmv

using namespace spmv;

extern "C" void spmv_destroy(spmv_handle h) {
    if (!h) return;
    (void)hipDeviceSynchronize();
    delete h;
}

extern "C" spmv_status spmv_convert(spmv_handle h, spmv_format f, int32_t param, void *stream) {
    return guard([&] {
        if (!h) fail(SPMV_ERR_INVALID_ARG, "NULL handle");
        if (!valid_format(f)) fail(SPMV_ERR_INVALID_ARG, "bad format %d", (int)f);
        convert(h, f, param, (hipStream_t)stream);
        // a new HYB split drops the old tail's sorted copy: the current variant rebuilds it
        if (f == SPMV_FMT_HYB) (void)prepare_variant(h, f, h->variant[f], (hipStream_t)stream);
    });
}

extern "C" spmv_status spmv_run(spmv_handle h, spmv_format f, double alpha, const void *x,
                                double beta, void *y, void *stream) {
    return guard([&] {
        check_runnable(h, f);
        check_vectors(h, x, y);
        launch_spmv(h, f, h->variant[f], alpha, x, beta, y, (hipStream_t)stream);
    });
}

extern "C" spmv_status spmv_get_arrays(spmv_handle h, spmv_format f, spmv_arrays *v) {
    return guard([&] {
        check_runnable(h, f);
        if (!v) fail(SPMV_ERR_INVALID_ARG, "NULL view");
        memset(v, 0, sizeof(*v));
        v->format = f;
        v->dtype = h->dt;
        v->n_rows = h->n_rows;
        v->n_cols = h->n_cols;
        v->nnz = h->nnz;
        switch (f) {
            case SPMV_FMT_CSR:
                v->row_ptr = h->row_ptr.as<int32_t>();
                v->col = h->col.as<int32_t>();
                v->val = h->val.p;
                break;
            case SPMV_FMT_COO:
                v->row = h->row.as<int32_t>();
                v->col = h->col.as<int32_t>();
                v->val = h->val.p;
                break;
            case SPMV_FMT_ELL:
                v->K = h->ell.K;
                v->pitch = h->ell.pitch;
                v->ell_col = h->ell.col.as<int32_t>();
                v->ell_val = h->ell.val.p;
                break;
            case SPMV_FMT_HYB:
                v->K = h->hyb.K;
                v->pitch = h->hyb.pitch;
                v->nnz_tail = h->hyb.nnz_tail;
                v->ell_col = h->hyb.ell_col.as<int32_t>();
                v->ell_val = h->hyb.ell_val.p;
                v->tail_row = h->hyb.tail_row.as<int32_t>();
                v->tail_col = h->hyb.tail_col.as<int32_t>();
                v->tail_val = h->hyb.tail_val.p;
                break;
            case SPMV_FMT_SELL:
                v->sigma = h->sell.sigma;
                v->n_slices = h->sell.n_slices;
                v->slots = h->sell.slots;
                v->slice_ptr = h->sell.slice_ptr.as<int64_t>();
                v->perm = h->sell.sigma > 1 ? h->sell.perm.as<int32_t>() : nullptr;
                v->ell_col = h->sell.col.as<int32_t>();
                v->ell_val = h->sell.val.p;
                break;
            case SPMV_FMT_BELL:
                v->block = h->bell.b;
                v->K = h->bell.K;
                v->pitch = h->bell.pitch;
                v->slots = (int64_t)h->bell.K * h->bell.pitch;
                v->ell_col = h->bell.col.as<int32_t>();
                v->ell_val = h->bell.val.p;
                break;
        }
    });
}

extern "C" int32_t spmv_variant_count(spmv_format f, spmv_dtype dt) {
    if (!valid_format(f)) return 0;
    return variant_count(f, dt);
}

extern "C" spmv_status spmv_variant_describe(spmv_format f, spmv_dtype dt, int32_t idx,
                                             spmv_variant_info *out) {
    return guard([&] {
        if (!valid_format(f) || !out || !variant_describe(f, dt, idx, out))
            fail(SPMV_ERR_INVALID_ARG, "bad format/dtype/index");
    });
}

extern "C" spmv_status spmv_set_variant(spmv_handle h, spmv_format f, int32_t idx) {
    return guard([&] {
        if (!h || !valid_format(f)) fail(SPMV_ERR_INVALID_ARG, "bad handle or format");
        if (idx < 0 || idx >= variant_count(f, h->dt)) fail(SPMV_ERR_INVALID_ARG, "bad variant %d", idx);
        if (!prepare_variant(h, f, idx, nullptr))
            fail(SPMV_ERR_NOT_APPLICABLE, "variant %d does not apply to this matrix", idx);
        h->variant[f] = idx;
    });
}

extern "C" spmv_status spmv_get_variant(spmv_handle h, spmv_format f, int32_t *idx) {
    return guard([&] {
        if (!h || !valid_format(f) || !idx) fail(SPMV_ERR_INVALID_ARG, "bad argument");
        *idx = h->variant[f];
    });
}

extern "C" spmv_status spmv_stored_bytes(spmv_handle h, spmv_format f, int32_t variant,
                                         int64_t *bytes) {
    return guard([&] {
        check_runnable(h, f);
        if (!bytes) fail(SPMV_ERR_INVALID_ARG, "NULL bytes");
        const int32_t v = variant < 0 ? h->variant[f] : variant;
        if (v >= variant_count(f, h->dt)) fail(SPMV_ERR_INVALID_ARG, "variant %d out of range", v);
        const int64_t b = stored_bytes(h, f, v);
        if (b < 0) fail(SPMV_ERR_NOT_CONVERTED, "the layout of variant %d is not built", v);
        *bytes = b;
    });
}

extern "C" spmv_status spmv_features(spmv_handle h, float *out12, void *stream) {
    return guard([&] {
        if (!h || !out12) fail(SPMV_ERR_INVALID_ARG, "NULL argument");
        compute_features(h, out12, nullptr, (hipStream_t)stream);
    });
}

extern "C" spmv_status spmv_features_noalloc(spmv_handle h, float *out12, void *stream) {
    return guard([&] {
        if (!h || !out12) fail(SPMV_ERR_INVALID_ARG, "NULL argument");
        compute_features_noalloc(h, out12, (hipStream_t)stream);
    });
}

extern "C" spmv_status spmv_select_format(spmv_handle h, spmv_select_mode m, spmv_format *out,
                                          float *out_scores, void *stream) {
    return guard([&] {
        if (!h || !out) fail(SPMV_ERR_INVALID_ARG, "NULL argument");
        hipStream_t s = (hipStream_t)stream;
        float scores[SPMV_NUM_FORMATS] = {};
        spmv_format f = SPMV_FMT_CSR;
        if (m == SPMV_SELECT_EXHAUSTIVE) {
            f = select_exhaustive(h, scores, s);
        } else if (m == SPMV_SELECT_RULE || m == SPMV_SELECT_MODEL) {
            float feats[12];
            compute_features(h, feats, nullptr, s);
            if (m == SPMV_SELECT_RULE) {
                f = select_rule(feats, scores);
                if (f == SPMV_FMT_ELL && h->nnz > 0 &&
                    (int64_t)((h->n_rows + 63) / 64 * 64) * h->stats.max_len > 8 * h->nnz)
                    f = SPMV_FMT_CSR;
            } else {
                f = select_model(h, feats, scores, s);
            }
            if (!format_built(h, f)) convert(h, f, -1, s);
        } else {
            fail(SPMV_ERR_INVALID_ARG, "bad select mode %d", (int)m);
        }
        *out = f;
        if (out_scores) memcpy(out_scores, scores, sizeof(scores));
    });
}

namespace spmv {
namespace {

struct RuntimeModels {
    std::mutex mu;
    bool set[64] = {};
    float p[64][SPMV_RUNTIME_MODEL];
};

RuntimeModels &runtime_models() {
    static RuntimeModels *r = new RuntimeModels();  // lives until process exit
    return *r;
}

int runtime_device() {
    int d = 0;
    SPMV_HIP(hipGetDevice(&d));
    if (d < 0 || d >= 64) fail(SPMV_ERR_INVALID_ARG, "device id %d", d);
    return d;
}

// Time of one SpMV in format f (ms): exp of the run-time model's linear form over
// the selector's inputs.
double runtime_time_ms(const float *m, int f, const float feats[12]) {
    double z = m[f * 13 + 12];
    for (int i = 0; i < 12; ++i) {
        const bool lg = i <= 6 || i == 8 || i == 9;
        const double v = lg ? std::log2(1.0 + (double)feats[i]) : (double)feats[i];
        z += (double)m[f * 13 + i] * v;
    }
    return std::exp(z);
}

double runtime_convert_ms(const float *m, int f, const spmv_matrix_s *h) {
    if (f == SPMV_FMT_CSR || f == SPMV_FMT_COO) return 0.0;
    const float *c = m + SPMV_NUM_FORMATS * 13 + f * 3;
    return std::max(0.0, (double)c[0] + (double)c[1] * (h->nnz / 1e6) +
                             (double)c[2] * (h->n_rows / 1e6));
}

double now_ms() {
    return std::chrono::duration<double, std::milli>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

}  // namespace
}  // namespace spmv

extern "C" spmv_status spmv_runtime_set_model(const float *params, int64_t n) {
    return guard([&] {
        const int d = runtime_device();
        RuntimeModels &R = runtime_models();
        std::lock_guard<std::mutex> lk(R.mu);
        if (!params && n == 0) {
            R.set[d] = false;
            return;
        }
        if (!params || n != SPMV_RUNTIME_MODEL)
            fail(SPMV_ERR_INVALID_ARG, "expected %d floats, got %lld", SPMV_RUNTIME_MODEL, (long long)n);
        for (int i = 0; i < SPMV_RUNTIME_MODEL; ++i)
            if (!std::isfinite(params[i])) fail(SPMV_ERR_INVALID_ARG, "parameter %d is not finite", i);
        memcpy(R.p[d], params, sizeof(R.p[d]));
        R.set[d] = true;
    });
}

extern "C" spmv_status spmv_select_runtime(spmv_handle h, spmv_format current, int64_t iterations,
                                           spmv_runtime_decision *out, void *stream) {
    return guard([&] {
        if (!h || !out || iterations < 0) fail(SPMV_ERR_INVALID_ARG, "bad argument");
        check_runnable(h, current);
        hipStream_t s = (hipStream_t)stream;
        float m[SPMV_RUNTIME_MODEL];
        {
            const int d = runtime_device();
            RuntimeModels &R = runtime_models();
            std::lock_guard<std::mutex> lk(R.mu);
            if (!R.set[d]) fail(SPMV_ERR_NO_MODEL, "no run-time model on device %d", d);
            memcpy(m, R.p[d], sizeof(m));
        }
        spmv_runtime_decision r{};
        r.current = current;
        double t0 = now_ms();
        float feats[12];
        compute_features(h, feats, nullptr, s);
        r.features_ms = (float)(now_ms() - t0);
        t0 = now_ms();
        float scores[SPMV_NUM_FORMATS];
        int nc = 0;
        const spmv_status st = model_logits(feats, scores, &nc, s);
        if (st != SPMV_OK) throw Error{st};
        r.predict_ms = (float)(now_ms() - t0);
        bool allowed[SPMV_NUM_FORMATS];
        for (int i = 0; i < SPMV_NUM_FORMATS; ++i) allowed[i] = i < nc;
        allowed[SPMV_FMT_ELL] = allowed[SPMV_FMT_ELL] &&
                                (h->nnz == 0 || (int64_t)((h->n_rows + 63) / 64 * 64) *
                                                        h->stats.max_len <= 8 * h->nnz);
        r.t_current_ms = (float)runtime_time_ms(m, current, feats);
        for (;;) {
            int best = SPMV_FMT_CSR;
            for (int i = 0; i < SPMV_NUM_FORMATS; ++i)
                if (allowed[i] && (!allowed[best] || scores[i] > scores[best])) best = i;
            const spmv_format f = (spmv_format)best;
            r.predicted = f;
            r.t_predicted_ms = (float)runtime_time_ms(m, f, feats);
            r.convert_ms = format_built(h, f) ? 0.f : (float)runtime_convert_ms(m, f, h);
            r.gain_ms = ((double)r.t_current_ms - (double)r.t_predicted_ms) * (double)iterations;
            r.overhead_ms = (double)r.features_ms + (double)r.predict_ms + (double)r.convert_ms;
            r.chosen = current;
            r.converted = 0;
            if (f == current || !(r.gain_ms > r.overhead_ms)) break;  // the switch does not pay
            if (format_built(h, f)) {
                r.chosen = f;
                break;
            }
            try {
                convert(h, f, -1, s);
                r.chosen = f;
                r.converted = 1;
                break;
            } catch (const Error &e) {
                if (e.status != SPMV_ERR_NOT_APPLICABLE) throw;
                clear_error();
                allowed[best] = false;  // CSR and COO are always built, so this ends
            }
        }
        *out = r;
    });
}

extern "C" const char *spmv_status_string(spmv_status s) {
    switch (s) {
        case SPMV_OK: return "ok";
        case SPMV_ERR_INVALID_ARG: return "invalid argument";
        case SPMV_ERR_OUT_OF_BOUNDS: return "index out of bounds";
        case SPMV_ERR_DUPLICATE: return "duplicate entry";
        case SPMV_ERR_NOT_CONVERTED: return "format not converted";
        case SPMV_ERR_NOT_APPLICABLE: return "format not applicable";
        case SPMV_ERR_OOM: return "out of device memory";
        case SPMV_ERR_HIP: return "HIP runtime error";
        case SPMV_ERR_NO_MODEL: return "no selector model loaded";
    }
    return "unknown status";
}

extern "C" const char *spmv_last_error(void) { return g_last_error.c_str(); }
