/*
 * spmv.h - C ABI of the MI355X (gfx950) sparse matrix-vector library.
 *
 * The library computes y = alpha * A * x + beta * y (the SpMV product Y = A X
 * of the paper's background section on SpMV processing, with BLAS scaling)
 * for a sparse A held in one of the formats the run-time mode chooses
 * between, and picks the fastest format for a given matrix from its sparsity
 * features (paper, Method: run-time optimisation mode; sparsity features
 * table).
 *
 * Conventions for every function:
 *   - Indices are 0-based int32. Values are FP32 or FP64 (spmv_dtype).
 *   - A "device pointer" is memory allocated on the current HIP device
 *     (hipMalloc or torch). A "host pointer" is ordinary CPU memory.
 *   - `stream` is a hipStream_t passed as void*; NULL means the null stream.
 *     All device work is enqueued on it.
 *   - Every function returns a status and never throws or aborts across the
 *     ABI. spmv_last_error() gives a message for the calling thread.
 *   - Handles are owned by the library; spmv_create copies its inputs. A
 *     handle is not thread-safe: calls on one handle must not overlap, and
 *     runs of one handle enqueued on different streams must not execute at
 *     the same time (the COO kernels keep per-tile carries in the handle).
 *   - The current device at spmv_create is the handle's device; later calls
 *     on the handle must run with that device current.
 */
#ifndef SPMV_H
#define SPMV_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum spmv_status {
    SPMV_OK = 0,
    SPMV_ERR_INVALID_ARG = 1,   /* bad pointer, size, enum, x == y, ...          */
    SPMV_ERR_OUT_OF_BOUNDS = 2, /* a COO row/col index outside the matrix         */
    SPMV_ERR_DUPLICATE = 3,     /* two COO entries with the same (row, col)       */
    SPMV_ERR_NOT_CONVERTED = 4, /* format not built yet on this handle            */
    SPMV_ERR_NOT_APPLICABLE = 5,/* ELL padded size would exceed 8 * nnz           */
    SPMV_ERR_OOM = 6,           /* device allocation failed                       */
    SPMV_ERR_HIP = 7,           /* a HIP runtime call failed                      */
    SPMV_ERR_NO_MODEL = 8       /* selector weights not loaded                    */
} spmv_status;

/* Storage formats. The numbering is also the selector's class order. */
typedef enum spmv_format {
    SPMV_FMT_CSR = 0, /* row_ptr[n_rows+1], col[nnz], val[nnz], rows in order    */
    SPMV_FMT_COO = 1, /* row[nnz], col[nnz], val[nnz], sorted by (row, col)       */
    SPMV_FMT_ELL = 2, /* col/val [K][pitch], column-major, pitch = roundup(n,64)  */
    SPMV_FMT_HYB = 3, /* ELL part of width K_h + COO tail of the other entries    */
    SPMV_FMT_SELL = 4,/* sliced ELL: slices of 64 rows, each as wide as its longest
                         row (rounded up to 4 slots), slot pointers per slice, rows
                         optionally reordered by length inside windows (sigma)    */
    SPMV_FMT_BELL = 5 /* blocked ELL: ELL over dense b x b blocks, b = 2, 4 or 8  */
} spmv_format;
#define SPMV_NUM_FORMATS 6

typedef enum spmv_dtype { SPMV_F32 = 0, SPMV_F64 = 1 } spmv_dtype;

/* Kernel families behind the formats (a variant is one compiled instance). */
typedef enum spmv_kernel {
    SPMV_KERNEL_CSR_SCALAR = 0, /* one thread per row                             */
    SPMV_KERNEL_CSR_VECTOR = 1, /* `lanes` lanes of a wavefront per row           */
    SPMV_KERNEL_COO = 2,        /* nnz tiles, segmented reduction by row          */
    SPMV_KERNEL_ELL = 3,        /* `lanes` consecutive rows per thread            */
    SPMV_KERNEL_HYB = 4,        /* ELL part (`lanes` rows/thread) + COO tail; with
                                   pipelined = 1 the tail is added by the sorted-
                                   block COO kernel over a copy of the tail built
                                   by spmv_set_variant / spmv_tune / spmv_time /
                                   spmv_convert (its order of FP64 additions is not
                                   fixed, as for SPMV_KERNEL_COO_SORTED)          */
    SPMV_KERNEL_COO_PANEL = 5,  /* COO entries of each row group (one per wave)
                                   streamed in column-panel order, so an XCD's x
                                   gathers stay in a window of x; needs a second
                                   copy of the entries, built by spmv_set_variant
                                   / spmv_tune / spmv_time; n_cols < 2^23 - 1     */
    SPMV_KERNEL_COO_SORTED = 6, /* COO entries of each block of rows sorted by
                                   column, so a wave's gathers share cache lines;
                                   rows summed with LDS atomics across the block's
                                   16 waves: the order of the FP64 additions, and
                                   so the last bits of a result, may vary between
                                   runs; second copy of the entries as above;
                                   ksplit = 2 or 4 (column tiles): blocks 2 or 4
                                   times as tall, each block's entries in ksplit
                                   tiles by column range, run by as many
                                   workgroups; the other ranges' row sums are
                                   added to y by a second launch (4 tiles apply
                                   where one round of workgroups holds them)      */
    SPMV_KERNEL_COO_SPLIT = 7,  /* tiled COO run once per 2 MB column panel of x
                                   over a copy ordered by (panel, row, column), the
                                   first pass writing y, the others adding; only
                                   for matrices with more than one panel          */
    SPMV_KERNEL_SELL = 9,       /* SELL: one wavefront per slice, lane l on the
                                   slice's row l, four slots per 16-byte load;
                                   ksplit > 1: the waves of a workgroup share one
                                   slice, each taking every ksplit-th group       */
    SPMV_KERNEL_BELL = 10,      /* BELL: `lanes` rows of a block per thread (b /
                                   lanes threads per block row); a variant whose
                                   `lanes` exceeds the layout's b does not apply */
    SPMV_KERNEL_CSR_STREAM = 8  /* CSR over row blocks of at most 256 rows and
                                   2048 entries: a workgroup streams its block's
                                   entries with 16-byte loads, keeps the products
                                   in LDS and sums each row there in order (a row
                                   too long for the stage gets a workgroup of its
                                   own); the row blocks are computed on the host
                                   by spmv_set_variant / spmv_tune / spmv_time    */
} spmv_kernel;

typedef enum spmv_select_mode {
    SPMV_SELECT_MODEL = 0,      /* features -> selector network -> argmax         */
    SPMV_SELECT_EXHAUSTIVE = 1, /* convert all, tune and time all, take the best  */
    SPMV_SELECT_RULE = 2        /* fixed thresholds on the features               */
} spmv_select_mode;

typedef struct spmv_matrix_s *spmv_handle;
typedef struct spmv_batch_s *spmv_batch;

/* Description of one compiled kernel instance. */
typedef struct spmv_variant_info {
    int32_t kernel; /* spmv_kernel                                                */
    int32_t block;  /* workgroup size (threads)                                    */
    int32_t lanes;  /* CSR vector: lanes per row; ELL/HYB: rows per thread;
                       COO: entries per thread; CSR scalar: 1                      */
    int32_t unroll; /* independent loads in flight per lane                        */
    int32_t vec;    /* consecutive entries each lane reads with one load (1 or 4)  */
    int32_t pipelined; /* 0: plain; > 0: software pipelined (the next chunk's loads
                          in flight during the current gathers); for CSR the number
                          of rows each lane group walks as one stream, for ELL the
                          number of slots loaded ahead                            */
    int32_t ksplit;    /* ELL: waves of a workgroup sharing one block of rows, each
                          taking every ksplit-th slot (1 = one thread per row);
                          sorted-block COO: column tiles per block of rows         */
} spmv_variant_info;

/* Borrowed view of a format's device arrays; valid until spmv_destroy or a
 * re-conversion of that format. Fields a format does not use are 0 / NULL. */
typedef struct spmv_arrays {
    int32_t format, dtype, n_rows, n_cols;
    int64_t nnz;      /* stored entries of the matrix                           */
    int32_t K, pitch; /* ELL / HYB-ELL width and row pitch                       */
    int64_t nnz_tail; /* HYB: entries in the COO tail                            */
    const int32_t *row_ptr, *row, *col;
    const void *val;
    const int32_t *ell_col;
    const void *ell_val;
    const int32_t *tail_row, *tail_col;
    const void *tail_val;
    /* SELL: slot arrays in ell_col / ell_val; slice s holds slots
     * [slice_ptr[s], slice_ptr[s+1]), slot k of the row at position l of the
     * slice at slice_ptr[s] + (k / 4) * 256 + l * 4 + k % 4; perm[p] is the row
     * at position p (NULL when sigma == 1: position p is row p).
     * BELL: block columns in ell_col ([K][pitch], -1 = padding), block values
     * in ell_val (block (i, k) at (k * pitch + i) * b * b, row-major), with
     * K = most blocks in a block row, pitch = block rows rounded up to 64. */
    int32_t sigma, n_slices, block;  /* SELL sigma and slices; BELL edge b       */
    int64_t slots;                   /* SELL: slots; BELL: blocks (K * pitch)   */
    const int64_t *slice_ptr;
    const int32_t *perm;
} spmv_arrays;

/* ---- matrix lifetime ----------------------------------------------------- */

/* Ingest a COO matrix (the input format of the paper's run-time mode, Results:
 * run-time prediction overhead) and build its canonical COO and CSR forms on
 * the device (CSR: paper, Background, popular SpMV formats).
 *   row, col: int32[nnz], val: float[nnz] or double[nnz] per `dt`; host
 *   pointers if on_device == 0, device pointers otherwise; any order. The
 *   caller keeps ownership; the library copies them.
 *   n_rows, n_cols >= 0; 0 <= nnz <= INT32_MAX. nnz == 0 is legal.
 * Entries are sorted by (row, col). Explicit zeros are kept as entries.
 * Errors: INVALID_ARG (sizes, NULL pointers with nnz > 0, dtype),
 *         OUT_OF_BOUNDS (an index outside [0,n_rows) x [0,n_cols)),
 *         DUPLICATE (a repeated (row, col)), OOM, HIP.
 * Synchronises `stream`. On error *out is set to NULL. */
spmv_status spmv_create(spmv_handle *out, int32_t n_rows, int32_t n_cols, int64_t nnz,
                        const int32_t *row, const int32_t *col, const void *val, spmv_dtype dt,
                        int on_device, void *stream);

/* Free a handle and all its device arrays. NULL is ignored. Synchronises the
 * device. */
void spmv_destroy(spmv_handle h);

/* Build format `f` from the canonical CSR (paper, Background: ELL, BELL and
 * SELL, and the run-time mode's conversion step). CSR and COO exist after
 * spmv_create and return OK at once. `param` is the format's layout parameter.
 *   ELL: width K = longest row, pitch = roundup(n_rows, 64), slot (i, k) at
 *        k * pitch + i, padding slots hold col -1 and val +0.0. Returns
 *        NOT_APPLICABLE (and builds nothing) when pitch * K > 8 * nnz.
 *   HYB: ELL part of width K_h plus the remaining entries as a COO tail in
 *        (row, col) order. param < 0 chooses K_h by the Bell-Garland rule:
 *        the largest k such that at least T = min(n_rows, max(4096,
 *        ceil(n_rows/3))) rows hold k or more entries; param >= 0 forces it.
 *   SELL: param = sigma, the window inside which rows are reordered by
 *        descending length (stable): 1 keeps the row order (the paper's SELL),
 *        otherwise a positive multiple of 64; param < 0 takes whichever of 1
 *        and 16384 stores fewer bytes (slots * (4 + value size), plus 4 bytes
 *        per row for the order when sigma > 1; ties to 1). A slice's width is
 *        its longest row rounded up to a multiple of 4; padding col -1, +0.0.
 *   BELL: param = b in {2, 4, 8}; param < 0 takes, of the sizes within the
 *        cap, the one storing the fewest bytes (pitch * K * (4 + b*b*value
 *        size)), ties to the smaller, 2 if none. Absent entries of a stored
 *        block are +0.0, so a non-finite x value meeting one gives NaN.
 *   SELL and BELL return NOT_APPLICABLE when their slots (SELL) or stored
 *        values (BELL) exceed both 8 * nnz and 65536.
 * A failed conversion leaves the handle's other formats intact.
 * Errors: INVALID_ARG (bad param), NOT_APPLICABLE, OOM, HIP. Synchronises
 * `stream`. */
spmv_status spmv_convert(spmv_handle h, spmv_format f, int32_t param, void *stream);

/* y = alpha * A * x + beta * y with the handle's current variant for `f`
 * (paper, Background: SpMV processing on GPU). Asynchronous on `stream`.
 *   x: device pointer, n_cols values of the handle's dtype.
 *   y: device pointer, n_rows values; read only when beta != 0, so beta == 0
 *      ignores NaN or garbage in y. x and y must not overlap.
 *   alpha, beta: rounded to the handle's dtype.
 * Rows with no entries get y = beta * y (or 0 when beta == 0).
 * A run only launches kernels on `stream` (it never allocates, copies,
 * fills or synchronises; the variant's layout is built beforehand by
 * spmv_convert / spmv_set_variant / spmv_tune), so it may be captured into a
 * HIP graph and replayed.
 * Errors: INVALID_ARG (NULL x/y with a nonzero dimension, x and y overlap),
 *         NOT_CONVERTED, HIP (launch failure). */
spmv_status spmv_run(spmv_handle h, spmv_format f, double alpha, const void *x, double beta,
                     void *y, void *stream);

/* Borrowed device arrays of format `f` (see spmv_arrays). Errors:
 * INVALID_ARG, NOT_CONVERTED. */
spmv_status spmv_get_arrays(spmv_handle h, spmv_format f, spmv_arrays *view);

/* ---- kernel variants and timing (the paper's compile-time mode picks thread
 * block size and register/cache settings per matrix, Method: compile-time
 * optimisation mode; here each format has a set of compiled instances and the
 * fastest is chosen by timing) ---------------------------------------------- */

/* Number of compiled variants of format f for dtype dt (0 for a bad enum). */
int32_t spmv_variant_count(spmv_format f, spmv_dtype dt);

/* Describe variant `idx` of (f, dt). Errors: INVALID_ARG. */
spmv_status spmv_variant_describe(spmv_format f, spmv_dtype dt, int32_t idx,
                                  spmv_variant_info *out);

/* Select / query the variant spmv_run uses for format f on this handle.
 * A new handle starts with a default chosen from its row-length statistics.
 * Errors: INVALID_ARG. */
spmv_status spmv_set_variant(spmv_handle h, spmv_format f, int32_t idx);
spmv_status spmv_get_variant(spmv_handle h, spmv_format f, int32_t *idx);

/* Time `reps` runs of format f with variant `variant` (-1 = current) after
 * `warmup` untimed runs, y = 1 * A * x + 0 * y. If flush != 0 every timed run
 * is preceded by a 1 GiB read sweep that evicts L2 and the Infinity Cache.
 * Each run is bracketed by a pair of HIP events on `stream`.
 *   x, y: device pointers as for spmv_run (y is overwritten).
 *   out_ms: host pointer, float[reps], milliseconds per run.
 * Errors: INVALID_ARG, NOT_CONVERTED, OOM (flush buffer), HIP.
 * Synchronises `stream`. */
spmv_status spmv_time(spmv_handle h, spmv_format f, int32_t variant, const void *x, void *y,
                      int32_t warmup, int32_t reps, int flush, float *out_ms, void *stream);

/* Autotune format f: time every variant (median of `reps` runs, flushed if
 * flush != 0), make the fastest the handle's current variant, and return it.
 *   best_idx, best_ms: host pointers (may be NULL).
 * Errors: as spmv_time. Synchronises `stream`. */
spmv_status spmv_tune(spmv_handle h, spmv_format f, const void *x, void *y, int32_t reps,
                      int flush, int32_t *best_idx, float *best_ms, void *stream);

/* Bytes of the device arrays one run of format f with `variant` (-1 = the
 * current one) reads besides x and y: the layout that variant streams (the
 * format arrays, or the reordered copy it uses, with their padding) and its
 * pointer and order arrays; for column tiles also the other ranges' row sums
 * written and read back and y's second pass (2 (tiles - 1) + 2 values per
 * row). A run's algorithmic bytes are this plus n_cols values of x and n_rows
 * of y (twice when beta != 0).
 *   bytes: host pointer. Errors: INVALID_ARG, NOT_CONVERTED (the format, or
 *   the copy the variant reads, is not built). Touches no device memory. */
spmv_status spmv_stored_bytes(spmv_handle h, spmv_format f, int32_t variant, int64_t *bytes);

/* ---- energy, average power and efficiency (paper, Experimental Setup: GPU
 * performance monitoring -- energy, average power and MFLOPS per watt are
 * measured beside latency while the kernel repeats; Results of the run-time
 * optimisation mode -- the format moves power and efficiency) ------------- */

typedef struct spmv_energy_result {
    double seconds;         /* interval between the two counter updates (host clock)    */
    double joules;          /* board energy over that interval                           */
    double watts;           /* joules / seconds: average board power under the load      */
    int64_t runs;           /* SpMVs enqueued between the two updates                    */
    double ms_per_run;      /* HIP-event time of those runs back to back, per run        */
    double joules_per_run;  /* watts * ms_per_run: energy of one SpMV                    */
    double mflops_per_watt; /* 2 nnz / joules_per_run / 1e6                              */
} spmv_energy_result;

/* Run format f (variant, -1 = the current one) back to back with alpha = 1,
 * beta = 0 on `stream` and read the GPU's energy accumulator (amd-smi, matched
 * to the current HIP device by PCI id): after a 0.1 s warm period, wait for a
 * counter update, keep running for at least `seconds`, wait for the next
 * update; both updates fall inside the busy period. y is overwritten. The
 * board power includes the idle draw (see spmv_idle_power). The interval is
 * timed with the host clock at the two detections; one whose energy implies
 * no power or more than 5 kW holds a bad reading and is measured again (three
 * attempts).
 *   x, y: device pointers as for spmv_run. seconds in (0, 60]. out: host.
 * Errors: INVALID_ARG, NOT_CONVERTED, NOT_APPLICABLE (no energy counter for
 * this device, it did not advance, or the variant does not apply), HIP.
 * Synchronises `stream`; takes about seconds + 0.1 s + up to two counter
 * periods (about 1 s each on MI355X). */
spmv_status spmv_energy(spmv_handle h, spmv_format f, int32_t variant, const void *x, void *y,
                        double seconds, spmv_energy_result *out, void *stream);

/* Several formats of one matrix in one sweep (the energy labels of a matrix):
 * after a 0.1 s warm period and a counter update, formats[i] (variants[i], -1
 * or variants NULL = the current variant) runs back to back until `seconds`
 * have passed and the counter has moved again, and that update opens the next
 * format's interval, so the sweep takes about `count` counter periods (about
 * 1 s each on MI355X) instead of two per format. Runs of one format that spill
 * past its closing update (batches of about 1 ms) count towards the next. An
 * interval whose energy is inconsistent is measured again alone.
 *   formats, variants: host int32[count], 1 <= count <= 64. out: host
 *   spmv_energy_result[count]. Errors: as spmv_energy. Synchronises `stream`. */
spmv_status spmv_energy_formats(spmv_handle h, int32_t count, const int32_t *formats,
                                const int32_t *variants, const void *x, void *y, double seconds,
                                spmv_energy_result *out, void *stream);

/* Average board power over at least `seconds` between two counter updates,
 * with no work of this library (other work on the device counts).
 *   watts: host. Errors: INVALID_ARG, NOT_APPLICABLE, HIP. Synchronises the device. */
spmv_status spmv_idle_power(double seconds, double *watts);

/* ---- features and selection ---------------------------------------------- */

/* The 12 sparsity features of the matrix, computed on the device (paper,
 * Method: sparsity features table, extended), in this order:
 *   0 n_rows, 1 nnz, 2 mean row length, 3 population variance of row
 *   lengths, 4 standard deviation, 5 median row length (mean of the middle
 *   two when n is even), 6 mode (most frequent length, smallest on ties),
 *   7 ELL ratio nnz / (n * max), 8 max row length, 9 bandwidth max |i - j|,
 *   10 fill nnz / (n_rows * n_cols), 11 HYB tail fraction at the rule's K_h.
 * Quantities with an empty denominator are 0.
 *   out12: host pointer, float[12]. Synchronises `stream`. */
spmv_status spmv_features(spmv_handle h, float *out12, void *stream);

/* Longest row spmv_features_noalloc accepts. */
#define SPMV_FEATURES_NOALLOC_MAX_LEN 262143

/* For callers that cannot allocate device memory (tight serving loops,
 * harnesses that forbid hipMalloc): spmv_features with every temporary
 * (row-length histogram and its prefix sums, scan tile sums, statistics,
 * result words) in one file-scope device array of about 2 MiB per device,
 * held until the process ends. Calls no hipMalloc or hipFree; clears what it
 * uses with a fill kernel before each run. All calls on one device share that
 * array, so calls that overlap in time on one device (other threads or
 * streams) race; serialise them.
 *   out12: host pointer, float[12]; same values as spmv_features.
 * Errors: INVALID_ARG (NULL argument, or a row longer than
 * SPMV_FEATURES_NOALLOC_MAX_LEN), HIP. Synchronises `stream`. */
spmv_status spmv_features_noalloc(spmv_handle h, float *out12, void *stream);

/* Choose the format for this matrix (paper, Method: run-time optimisation
 * mode, steps 1-2; Predicting optimal configuration parameters).
 *   MODEL: features -> selector network -> argmax over applicable formats
 *          (requires spmv_selector_set_weights; else NO_MODEL).
 *   EXHAUSTIVE: convert every format, tune each, take the fastest median.
 *   RULE: fixed thresholds on the features.
 *   out: host pointer. out_scores: host float[SPMV_NUM_FORMATS] or NULL:
 *   logits (MODEL; -inf for a format the installed network has no class
 *   for), best median ms per format, +inf if not applicable (EXHAUSTIVE), or
 *   0/1 votes (RULE). The chosen format is converted before return.
 * Errors: INVALID_ARG, NO_MODEL, OOM, HIP. Synchronises `stream`. */
spmv_status spmv_select_format(spmv_handle h, spmv_select_mode m, spmv_format *out,
                               float *out_scores, void *stream);

/* ---- overhead-aware run-time mode (paper, Method: run-time optimisation mode,
 * step 3: the overhead of the switch is estimated and the matrix is converted
 * only when the gain pays for it; Results: run-time prediction overhead, the
 * regressors for the feature-extraction and conversion latencies) ----------
 *
 * A run-time model is SPMV_RUNTIME_MODEL floats: for each format f (0..5), 13
 * weights w[f] of a linear model of log(median SpMV time in ms) over the
 * selector's 12 inputs (log2(1 + v) on features 0-6, 8, 9; raw 7, 10, 11) plus
 * an intercept (w[f][12]); then, for each format, the conversion latency in ms
 * as c0 + c1 * (nnz / 1e6) + c2 * (n_rows / 1e6) (CSR and COO: no conversion). */
#define SPMV_RUNTIME_MODEL 96

typedef struct spmv_runtime_decision {
    int32_t current;       /* the format the caller runs now                          */
    int32_t predicted;     /* the selector network's choice                           */
    int32_t chosen;        /* predicted if converting pays, else current              */
    int32_t converted;     /* 1 when this call converted `chosen`                     */
    float features_ms;     /* measured: the features call                             */
    float predict_ms;      /* measured: the network's prediction                      */
    float convert_ms;      /* estimated conversion latency of `predicted` (0 if built) */
    float t_current_ms;    /* estimated time of one SpMV in the current format        */
    float t_predicted_ms;  /* estimated time of one SpMV in the predicted format      */
    double gain_ms;        /* (t_current - t_predicted) * iterations                  */
    double overhead_ms;    /* features + prediction + conversion                      */
} spmv_runtime_decision;

/* Install / forget the run-time model on the current device (host float[96];
 * NULL, 0 forgets it). Errors: INVALID_ARG (size, or a non-finite value). */
spmv_status spmv_runtime_set_model(const float *params, int64_t n);

/* Run-time mode for a matrix that will take `iterations` SpMVs: compute its
 * features (timed), ask the installed selector network for a format (timed),
 * estimate the per-SpMV times of the current and predicted formats and the
 * predicted format's conversion latency with the run-time model, and convert
 * only if (t_current - t_predicted) * iterations > features + prediction +
 * conversion. A predicted format whose conversion is refused gives way to the
 * network's next choice. `current` must be built (CSR and COO always are).
 *   out: host pointer. Errors: INVALID_ARG, NOT_CONVERTED (current),
 *   NO_MODEL (no selector network or no run-time model), OOM, HIP.
 * Synchronises `stream`. */
spmv_status spmv_select_runtime(spmv_handle h, spmv_format current, int64_t iterations,
                                spmv_runtime_decision *out, void *stream);

/* ---- batched SpMV: many CSR matrices in one persistent launch, captured in a
 * HIP graph (the stand-in for the paper's compile-time mode, Method:
 * compile-time optimisation mode, which fixes launch settings per matrix) -- */

typedef struct spmv_batch_config {
    int32_t block;           /* workgroup size (256)                                 */
    int32_t unroll;          /* 16-byte loads in flight per lane (1 or 2; 4 also for
                                tiling 2)                                            */
    int32_t passes_per_tile; /* a tile = this many passes of block/lanes rows        */
    int32_t blocks_per_cu;   /* persistent workgroups per compute unit               */
    int32_t lanes_divisor;   /* lanes per row = smallest power of two >=
                                row length / (4 * divisor), clamped to 2..64         */
    int32_t tiling;          /* 0: per matrix (lanes from the mean row length; y is
                                bit-equal to the single CSR vector launch with those
                                lanes and unroll); 1: per tile (lanes from the tile's
                                longest row; rows of >= 2048 entries get a tile of
                                their own reduced by the whole workgroup); 2: the
                                batch's sorted-block COO copy of every matrix, one
                                block (<= 4096 rows, entries sorted by column) per
                                1024-thread tile, largest first, unroll 1/2/4 = 4/8/16
                                entries per lane; the order of the FP64 row sums is
                                not fixed (see SPMV_KERNEL_COO_SORTED); needs a
                                second copy of every matrix's entries               */
    int32_t total_tiles;     /* row tiles over the whole batch                       */
    int32_t grid;            /* workgroups launched                                  */
    float tuned_ms;          /* median graph time of the chosen setting (0: untuned) */
} spmv_batch_config;

/* Build a batch over `count` (1..8192) CSR handles of one dtype on the current
 * device, with y_i = alpha_i * A_i * x_i + beta_i * y_i for each i.
 *   hs: host array of handles (borrowed: they must outlive the batch);
 *   xs, ys: host arrays of device pointers (x_i: n_cols_i values, y_i:
 *   n_rows_i values); no y_i may overlap any x_j or any other y_j (the x_i
 *   may be shared); alphas, betas: host arrays or NULL (1 and 0). If tune != 0 every setting of a small grid (unroll, tile size,
 *   workgroups per CU, lanes rule) is captured and timed and the fastest kept.
 * Errors: INVALID_ARG, OOM, HIP. Synchronises `stream`. */
spmv_status spmv_batch_create(spmv_batch *out, const spmv_handle *hs, int32_t count,
                              const void *const *xs, void *const *ys, const double *alphas,
                              const double *betas, int tune, void *stream);

/* One graph launch computing y_i = alpha_i * A_i * x_i + beta_i * y_i for every
 * matrix of the batch. Asynchronous on `stream`.
 *   alphas, betas: host double[count]; xs, ys: host arrays of count device
 *   pointers. Any of them may be NULL to keep the values the batch holds (from
 *   spmv_batch_create or an earlier run or update); given ones replace them for
 *   this and later runs (the descriptor upload is enqueued before the launch).
 * Runs on one stream must not overlap (they share the tile counter).
 * Errors: INVALID_ARG (as spmv_batch_create; the batch is left unchanged), HIP. */
spmv_status spmv_batch_run(spmv_batch b, const double *alphas, const void *const *xs,
                           const double *betas, void *const *ys, void *stream);

/* Re-point the batch (any array may be NULL to keep it); enqueued on `stream`
 * before later runs. Errors: INVALID_ARG (the batch is left unchanged), HIP. */
spmv_status spmv_batch_update(spmv_batch b, const void *const *xs, void *const *ys,
                              const double *alphas, const double *betas, void *stream);

/* The setting in use, and each matrix's lanes per row under the per-matrix
 * tiling (host int32[count] or NULL). Errors: INVALID_ARG. */
spmv_status spmv_batch_get_config(spmv_batch b, spmv_batch_config *out, int32_t *lanes);

/* Rebuild the batch's graph with the setting *cfg (block, total_tiles, grid and
 * tuned_ms are ignored): unroll 1 or 2 (or 4 with tiling 2), passes_per_tile >= 1,
 * blocks_per_cu >= 1, lanes_divisor >= 1, tiling 0, 1 or 2. Errors: INVALID_ARG,
 * NOT_APPLICABLE (tiling 2 on a matrix of more than 2^30 entries), OOM, HIP.
 * Synchronises `stream`. */
spmv_status spmv_batch_set_config(spmv_batch b, const spmv_batch_config *cfg, void *stream);

/* Free the batch (not its handles). NULL is ignored. Synchronises the device. */
void spmv_batch_destroy(spmv_batch b);

/* ---- the learned selector (paper, Method: predicting optimal configuration
 * parameters -- a classifier over the sparsity features; Setup, learning
 * algorithms: MLP with ReLU, Adam, learning rate 0.001, 200 epochs) -----------
 *
 * Network 12-64-64-C with ReLU, C = 4 classes (CSR, COO, ELL, HYB) or C = 6
 * (also SELL, BELL); classes are spmv_format values. A model is W1[64][12]
 * b1[64] W2[64][64] b2[64] W3[C][64] b3[C] (each W row-major [out][in]; 5252
 * parameters for C = 4, 5382 for C = 6) then the input standardisation
 * mean[12], std[12]. Inputs are the 12 features of spmv_features with
 * log2(1 + v) applied to features 0-6, 8 and 9, then (v - mean) / std. */

#define SPMV_SELECTOR_PARAMS 5252  /* C = 4 */
#define SPMV_SELECTOR_MODEL 5276
#define SPMV_SELECTOR_PARAMS6 5382 /* C = 6 */
#define SPMV_SELECTOR_MODEL6 5406

typedef struct spmv_train_opts {
    int32_t epochs;    /* passes over the data (200)                              */
    int32_t batch;     /* minibatch size; min(batch, n) is used (200)             */
    int32_t max_steps; /* stop after this many updates; <= 0 means no limit       */
    float lr;          /* Adam step size (1e-3)                                   */
    float l2;          /* L2 weight alpha; the loss adds alpha/(2B)*|W|^2 (1e-4)   */
    float beta1, beta2, eps; /* Adam (0.9, 0.999, 1e-8)                           */
    int32_t classes;   /* 4 or 6 (0 means 4)                                      */
} spmv_train_opts;

/* Train the selector on the device: mean softmax cross-entropy + L2, minibatch
 * Adam (Kingma and Ba, Algorithm 1) in the sample order perms gives for each
 * epoch; the standardisation statistics are the training set's mean and
 * population std (floored at 1e-6). One workgroup runs every step in one
 * launch (deterministic). The initial weights and the epoch orders are inputs
 * (the caller draws them; the library draws no random numbers).
 *   feats: device float[n][12] raw features; labels: device int32[n] in
 *   0..C-1; init_params: device float[params of C]; perms: device
 *   int32[epochs][n], each row a permutation of 0..n-1; out_model: device
 *   float[model of C]; out_losses: device float[number of steps] or NULL.
 * Errors: INVALID_ARG (also a label or order entry out of range), OOM, HIP.
 * Synchronises `stream`. */
spmv_status spmv_selector_train(const float *feats, const int32_t *labels, int32_t n,
                                const float *init_params, const int32_t *perms,
                                const spmv_train_opts *opts, float *out_model, float *out_losses,
                                void *stream);

/* Loss and gradient of one minibatch (the quantities a training step uses):
 *   params: device float[params of C]; classes: C (4 or 6); z: device
 *   float[b][12] already standardised; labels: device int32[b]; loss: device
 *   float[1]; grad: device float[params of C].
 * Asynchronous on `stream`. Errors: INVALID_ARG, HIP. */
spmv_status spmv_selector_loss_grad(const float *params, int32_t classes, const float *z,
                                    const int32_t *labels, int32_t b, float l2, float *loss,
                                    float *grad, void *stream);

/* Logits and chosen class for n feature vectors.
 *   model: device float[model of C] with classes = C, or NULL for the network
 *   installed on this device (classes 0 or its C); feats: device float[n][12]
 *   raw features; applicable: device uint8[n][C] (nonzero = format allowed) or
 *   NULL for all; logits: device float[n][C] or NULL; cls: device int32[n] or
 *   NULL (arg-max over allowed classes, ties to the lowest). Asynchronous.
 * Errors: INVALID_ARG, NO_MODEL, HIP. */
spmv_status spmv_selector_predict(const float *model, int32_t classes, const float *feats,
                                  int32_t n, const uint8_t *applicable, float *logits,
                                  int32_t *cls, void *stream);

/* Install / read the network MODEL selection uses on the current device.
 *   params: host float[n], n = 5276 (C = 4) or 5406 (C = 6);
 *   set_weights(NULL, 0) forgets it (MODEL selection then returns NO_MODEL).
 *   get_weights wants n equal to the installed model's size.
 * Errors: INVALID_ARG, NO_MODEL (get before set), HIP. Synchronous. */
spmv_status spmv_selector_set_weights(const float *params, int64_t n);
spmv_status spmv_selector_get_weights(float *params, int64_t n);
/* Classes of the network installed on the current device (0: none). */
int32_t spmv_selector_classes(void);

/* ---- diagnostics ------------------------------------------------------------ */

const char *spmv_status_string(spmv_status s);
/* Message of the calling thread's last failing call ("" if none). */
const char *spmv_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SPMV_H */
