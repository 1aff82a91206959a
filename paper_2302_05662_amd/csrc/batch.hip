// Batched SpMV: many CSR matrices of uneven sizes in one persistent launch,
// captured in a HIP graph, with its launch parameters chosen by timing.
//
// This stands in for the paper's compile-time mode (Method: compile-time
// optimisation mode picks the thread-block size and related settings per
// matrix): here a batch of matrices shares one launch whose unroll, tile size,
// grid size and lanes-per-row rule are picked by an autotuner.
//
// Work is split into tiles of consecutive rows of one matrix. A fixed grid of
// workgroups takes tiles from a device counter (atomicAdd) until the counter
// passes the last tile, so long and short matrices balance across the CUs and
// every workgroup reaches the exit. The counter is reset by a one-thread
// kernel node at the head of the graph. Each row is reduced by the same body
// as the single-matrix CSR vector kernel (csr_row_dot4), so a matrix's y is
// bit-equal to its single launch with the same lanes and unroll.
#include <algorithm>
#include <cmath>
#include <vector>

#include "common.hpp"
#include "device.hpp"

namespace spmv {
namespace {

constexpr int kBlock = 256;
constexpr int kMaxBatch = 8192;

struct BatchDesc {
    const int32_t *rp;
    const int32_t *col;
    const void *val;
    const void *x;
    void *y;
    int32_t n_rows;
    int32_t lanes_log2;    // lanes per row = 1 << lanes_log2 (1..6)
    int32_t rows_per_tile; // a multiple of 256 >> lanes_log2
    int32_t tile_begin;    // first tile of this matrix
    double alpha, beta;
};

__global__ void reset_counter(int32_t *counter) { *counter = 0; }

template <class V, int L, int UNROLL>
__device__ __forceinline__ void tile_pass(const BatchDesc &d, const int32_t *s_rp, int64_t r,
                                          int64_t row_end) {
    const int g = threadIdx.x / L, lane = threadIdx.x % L;
    const double acc = csr_row_dot4<V, L, UNROLL>(d.col, (const V *)d.val, (const V *)d.x,
                                                  s_rp[g], s_rp[g + 1], lane);
    const int64_t row = r + g;
    if (lane == 0 && row < row_end) store_y((V *)d.y, row, acc, (V)d.alpha, (V)d.beta);
}

template <class V, int UNROLL>
__global__ __launch_bounds__(kBlock) void batch_kernel(const BatchDesc *__restrict__ desc,
                                                       int32_t count, int32_t total_tiles,
                                                       int32_t *__restrict__ counter) {
    extern __shared__ int32_t s_begin[];        // tile_begin of every matrix
    __shared__ int32_t s_rp[kBlock / 2 + 1];    // row pointers of one pass (>= 2 lanes per row)
    __shared__ int32_t s_tile;
    for (int i = threadIdx.x; i < count; i += kBlock) s_begin[i] = desc[i].tile_begin;
    for (;;) {
        if (threadIdx.x == 0) s_tile = atomicAdd(counter, 1);
        __syncthreads();
        const int32_t t = s_tile;
        if (t >= total_tiles) break;
        int lo = 0, hi = count - 1;  // last matrix whose first tile is <= t
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (s_begin[mid] <= t) lo = mid; else hi = mid - 1;
        }
        const BatchDesc d = desc[lo];
        const int rpb = kBlock >> d.lanes_log2;  // rows per pass
        const int64_t row0 = (int64_t)(t - d.tile_begin) * d.rows_per_tile;
        const int64_t row_end = std::min<int64_t>(row0 + d.rows_per_tile, d.n_rows);
        for (int64_t r = row0; r < row_end; r += rpb) {
            for (int i = threadIdx.x; i <= rpb; i += kBlock) s_rp[i] = d.rp[std::min<int64_t>(r + i, row_end)];
            __syncthreads();
            switch (d.lanes_log2) {
                case 1: tile_pass<V, 2, UNROLL>(d, s_rp, r, row_end); break;
                case 2: tile_pass<V, 4, UNROLL>(d, s_rp, r, row_end); break;
                case 3: tile_pass<V, 8, UNROLL>(d, s_rp, r, row_end); break;
                case 4: tile_pass<V, 16, UNROLL>(d, s_rp, r, row_end); break;
                case 5: tile_pass<V, 32, UNROLL>(d, s_rp, r, row_end); break;
                default: tile_pass<V, 64, UNROLL>(d, s_rp, r, row_end); break;
            }
            __syncthreads();
        }
    }
}

using BatchKernel = void (*)(const BatchDesc *, int32_t, int32_t, int32_t *);

BatchKernel kernel_for(spmv_dtype dt, int unroll) {
    if (dt == SPMV_F64) return unroll == 2 ? batch_kernel<double, 2> : batch_kernel<double, 1>;
    return unroll == 2 ? batch_kernel<float, 2> : batch_kernel<float, 1>;
}

int lanes_log2_for(const spmv_matrix_s *h, int divisor) {
    // lanes x 4 entries per load ~ mean row length / divisor, within 2..64 lanes
    const double mean = h->n_rows ? (double)h->nnz / h->n_rows : 0.0;
    const double want = mean / (4.0 * divisor);
    int lg = 1;
    while (lg < 6 && (double)(1 << lg) < want) ++lg;
    return lg;
}

}  // namespace
}  // namespace spmv

struct spmv_batch_s {
    int device = 0;
    spmv_dtype dt = SPMV_F32;
    std::vector<spmv_matrix_s *> hs;
    std::vector<spmv::BatchDesc> desc;
    spmv::DevBuf d_desc, d_counter;
    spmv_batch_config cfg{};
    int num_cu = 0;
    hipStream_t capture_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;

    ~spmv_batch_s() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (capture_stream) (void)hipStreamDestroy(capture_stream);
    }
};

namespace spmv {
namespace {

// Fill the per-matrix tiling for a configuration; returns the total tile count.
int32_t plan_tiles(spmv_batch_s *b, const spmv_batch_config &c) {
    int64_t total = 0;
    for (size_t i = 0; i < b->hs.size(); ++i) {
        const spmv_matrix_s *h = b->hs[i];
        BatchDesc &d = b->desc[i];
        d.lanes_log2 = lanes_log2_for(h, c.lanes_divisor);
        d.rows_per_tile = (kBlock >> d.lanes_log2) * c.passes_per_tile;
        d.tile_begin = (int32_t)total;
        total += ceil_div(h->n_rows, d.rows_per_tile);
        if (total > INT32_MAX / 2) fail(SPMV_ERR_INVALID_ARG, "batch has too many tiles");
    }
    return (int32_t)total;
}

void upload_desc(spmv_batch_s *b, hipStream_t s) {
    SPMV_HIP(hipMemcpyAsync(b->d_desc.p, b->desc.data(), b->desc.size() * sizeof(BatchDesc),
                            hipMemcpyHostToDevice, s));
}

// (Re)build the graph {reset counter, persistent kernel} for configuration c.
void build_graph(spmv_batch_s *b, const spmv_batch_config &c, hipStream_t user) {
    spmv_batch_config cc = c;
    cc.total_tiles = plan_tiles(b, cc);
    cc.grid = std::max(1, std::min(cc.total_tiles, b->num_cu * cc.blocks_per_cu));
    cc.block = kBlock;
    upload_desc(b, user);
    SPMV_HIP(hipStreamSynchronize(user));
    if (b->exec) { SPMV_HIP(hipGraphExecDestroy(b->exec)); b->exec = nullptr; }
    if (b->graph) { SPMV_HIP(hipGraphDestroy(b->graph)); b->graph = nullptr; }
    hipStream_t cs = b->capture_stream;
    SPMV_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    reset_counter<<<1, 1, 0, cs>>>(b->d_counter.as<int32_t>());
    if (cc.total_tiles > 0) {
        BatchKernel k = kernel_for(b->dt, cc.unroll);
        const size_t lds = b->hs.size() * sizeof(int32_t);
        k<<<cc.grid, kBlock, lds, cs>>>(b->d_desc.as<BatchDesc>(), (int32_t)b->hs.size(),
                                        cc.total_tiles, b->d_counter.as<int32_t>());
    }
    hipError_t launch_err = hipGetLastError();
    hipGraph_t g = nullptr;
    hipError_t end_err = hipStreamEndCapture(cs, &g);
    if (launch_err != hipSuccess || end_err != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        fail(SPMV_ERR_HIP, "graph capture failed: %s / %s", hipGetErrorString(launch_err),
             hipGetErrorString(end_err));
    }
    b->graph = g;
    SPMV_HIP(hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0));
    b->cfg = cc;
}

double time_graph(spmv_batch_s *b, int reps, hipStream_t s) {
    hipEvent_t e0, e1;
    SPMV_HIP(hipEventCreate(&e0));
    SPMV_HIP(hipEventCreate(&e1));
    std::vector<float> ms;
    try {
        for (int i = 0; i < 2; ++i) SPMV_HIP(hipGraphLaunch(b->exec, s));
        for (int i = 0; i < reps; ++i) {
            SPMV_HIP(hipEventRecord(e0, s));
            SPMV_HIP(hipGraphLaunch(b->exec, s));
            SPMV_HIP(hipEventRecord(e1, s));
            SPMV_HIP(hipEventSynchronize(e1));
            float t = 0;
            SPMV_HIP(hipEventElapsedTime(&t, e0, e1));
            ms.push_back(t);
        }
    } catch (...) {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        throw;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    std::sort(ms.begin(), ms.end());
    return ms[ms.size() / 2];
}

void set_io(spmv_batch_s *b, const void *const *xs, void *const *ys, const double *alphas,
            const double *betas) {
    const size_t vs = dtype_size(b->dt);
    for (size_t i = 0; i < b->hs.size(); ++i) {
        const spmv_matrix_s *h = b->hs[i];
        BatchDesc &d = b->desc[i];
        if (xs) d.x = xs[i];
        if (ys) d.y = ys[i];
        if (alphas) d.alpha = alphas[i];
        if (betas) d.beta = betas[i];
        if ((h->n_cols > 0 && !d.x) || (h->n_rows > 0 && !d.y))
            fail(SPMV_ERR_INVALID_ARG, "matrix %zu: NULL x or y", i);
        if (d.x && d.y && h->n_rows > 0 && h->n_cols > 0) {
            const char *xb = (const char *)d.x, *xe = xb + (size_t)h->n_cols * vs;
            const char *yb = (const char *)d.y, *ye = yb + (size_t)h->n_rows * vs;
            if (xb < ye && yb < xe) fail(SPMV_ERR_INVALID_ARG, "matrix %zu: x and y overlap", i);
        }
    }
}

}  // namespace
}  // namespace spmv

using namespace spmv;

extern "C" spmv_status spmv_batch_create(spmv_batch *out, const spmv_handle *hs, int32_t count,
                                         const void *const *xs, void *const *ys,
                                         const double *alphas, const double *betas, int tune,
                                         void *stream) {
    if (out) *out = nullptr;
    spmv_batch_s *b = nullptr;
    spmv_status st = guard([&] {
        if (!out || !hs || !xs || !ys || count <= 0 || count > kMaxBatch)
            fail(SPMV_ERR_INVALID_ARG, "bad batch arguments (count %d, at most %d)", count, kMaxBatch);
        hipStream_t s = (hipStream_t)stream;
        b = new spmv_batch_s();
        SPMV_HIP(hipGetDevice(&b->device));
        SPMV_HIP(hipDeviceGetAttribute(&b->num_cu, hipDeviceAttributeMultiprocessorCount, b->device));
        b->dt = hs[0] ? hs[0]->dt : SPMV_F32;
        b->hs.assign(hs, hs + count);
        b->desc.resize(count);
        for (int32_t i = 0; i < count; ++i) {
            spmv_matrix_s *h = hs[i];
            if (!h) fail(SPMV_ERR_INVALID_ARG, "handle %d is NULL", i);
            if (h->dt != b->dt) fail(SPMV_ERR_INVALID_ARG, "handle %d has another dtype", i);
            if (h->device != b->device) fail(SPMV_ERR_INVALID_ARG, "handle %d is on another device", i);
            BatchDesc &d = b->desc[i];
            d.rp = h->row_ptr.as<int32_t>();
            d.col = h->col.as<int32_t>();
            d.val = h->val.p;
            d.n_rows = h->n_rows;
            d.alpha = 1.0;
            d.beta = 0.0;
        }
        set_io(b, xs, ys, alphas, betas);
        b->d_desc.alloc(count * sizeof(BatchDesc));
        b->d_counter.alloc(sizeof(int32_t));
        SPMV_HIP(hipStreamCreateWithFlags(&b->capture_stream, hipStreamNonBlocking));
        spmv_batch_config dflt{};
        dflt.unroll = 1;
        dflt.passes_per_tile = 4;
        dflt.blocks_per_cu = 8;
        dflt.lanes_divisor = 1;
        if (!tune) {
            build_graph(b, dflt, s);
            return;
        }
        // Time the candidates against scratch outputs, so that creating the
        // batch leaves the caller's y untouched whatever beta is.
        const size_t vs = dtype_size(b->dt);
        std::vector<size_t> off(count);
        size_t total = 0;
        for (int32_t i = 0; i < count; ++i) {
            off[i] = total;
            total += (size_t)ceil_div((int64_t)std::max(hs[i]->n_rows, 1) * vs, 256) * 256;
        }
        DevBuf scratch_y;
        scratch_y.alloc(total);
        SPMV_HIP(hipMemsetAsync(scratch_y.p, 0, total, s));
        std::vector<void *> real_y(count);
        for (int32_t i = 0; i < count; ++i) {
            real_y[i] = b->desc[i].y;
            b->desc[i].y = (char *)scratch_y.p + off[i];
        }
        double best = INFINITY;
        spmv_batch_config bc = dflt;
        for (int unroll : {1, 2})
            for (int passes : {1, 4, 16})
                for (int bpc : {4, 8})
                    for (int div : {1, 2}) {
                        spmv_batch_config c{};
                        c.unroll = unroll;
                        c.passes_per_tile = passes;
                        c.blocks_per_cu = bpc;
                        c.lanes_divisor = div;
                        build_graph(b, c, s);
                        const double t = time_graph(b, 5, s);
                        if (t < best) { best = t; bc = b->cfg; }
                    }
        SPMV_HIP(hipStreamSynchronize(s));
        for (int32_t i = 0; i < count; ++i) b->desc[i].y = real_y[i];
        build_graph(b, bc, s);
        b->cfg.tuned_ms = (float)best;
    });
    if (st == SPMV_OK) *out = b;
    else delete b;
    return st;
}

extern "C" spmv_status spmv_batch_run(spmv_batch b, void *stream) {
    return guard([&] {
        if (!b || !b->exec) fail(SPMV_ERR_INVALID_ARG, "NULL batch");
        SPMV_HIP(hipGraphLaunch(b->exec, (hipStream_t)stream));
    });
}

extern "C" spmv_status spmv_batch_update(spmv_batch b, const void *const *xs, void *const *ys,
                                         const double *alphas, const double *betas, void *stream) {
    return guard([&] {
        if (!b) fail(SPMV_ERR_INVALID_ARG, "NULL batch");
        std::vector<BatchDesc> keep = b->desc;
        try {
            set_io(b, xs, ys, alphas, betas);
        } catch (...) {
            b->desc = keep;
            throw;
        }
        upload_desc(b, (hipStream_t)stream);
    });
}

extern "C" spmv_status spmv_batch_get_config(spmv_batch b, spmv_batch_config *out, int32_t *lanes) {
    return guard([&] {
        if (!b || !out) fail(SPMV_ERR_INVALID_ARG, "NULL argument");
        *out = b->cfg;
        if (lanes)
            for (size_t i = 0; i < b->desc.size(); ++i) lanes[i] = 1 << b->desc[i].lanes_log2;
    });
}

extern "C" void spmv_batch_destroy(spmv_batch b) {
    if (!b) return;
    (void)hipDeviceSynchronize();
    delete b;
}
