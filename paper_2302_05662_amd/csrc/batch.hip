// Batched SpMV: many CSR matrices of uneven sizes in one persistent launch,
// captured in a HIP graph, with its launch parameters chosen by timing.
//
// This stands in for the paper's compile-time mode (Method: compile-time
// optimisation mode picks the thread-block size and related settings per
// matrix): here a batch of matrices shares one launch whose unroll, tiling,
// grid size and lanes-per-row rule are picked by an autotuner.
//
// Work is a list of tiles, each a range of consecutive rows of one matrix with
// the number of lanes that reduce each of its rows. A fixed grid of workgroups
// takes tiles from a device counter (atomicAdd) until the counter passes the
// last tile, so long and short matrices balance across the CUs and every
// workgroup reaches the exit. The counter is reset by a one-thread kernel node
// at the head of the graph.
//
// Two tilings: per matrix (every tile of a matrix uses the lanes of its mean
// row length; rows are then reduced exactly like the single-matrix CSR vector
// kernel, so y is bit-equal to a single launch with the same lanes and unroll),
// and per tile (a tile takes the lanes of its longest row, and a row of 2048 or
// more entries gets a tile of its own reduced by the whole workgroup), which
// keeps power-law rows from setting the tail. A third tiling uses the batch's
// own sorted-block COO copy of every matrix (blocks of up to 4096 rows, entries
// sorted by column, the row packed in the index or held in 16 bits beside it): a tile is one block, taken by a 1024-thread workgroup, and
// tiles are handed out largest first.
#include <algorithm>
#include <cmath>
#include <vector>

#include "common.hpp"
#include "device.hpp"

namespace spmv {
namespace {

constexpr int kBlock = 256;
constexpr int kMaxBatch = 8192;
constexpr int kBlockRow = 8;          // lanes_log2 value meaning "the whole workgroup"
constexpr int32_t kLongRow = 2048;    // entries from which a row gets its own tile
constexpr int kSortedBlock = kSortedWaves * kWave;  // workgroup size of the sorted tiling
constexpr int32_t kBatchSortedRows = 4096;          // rows per sorted block at most

struct BatchDesc {
    const int32_t *rp;
    const int32_t *col;
    const void *val;
    const void *x;
    void *y;
    int32_t n_rows;
    int32_t pad;
    double alpha, beta;
    // sorted-block copy (tiling 2)
    const int32_t *sblk;
    const int32_t *sidx;
    const void *sval;
    const uint16_t *srows16;  // rows inside the block, or null when packed in sidx
    const int32_t *sblk_row;  // first row of each block
    int64_t slast;  // last 16-byte-aligned load position of the copy
    int32_t scol_bits;
    int32_t spad;
};

struct BatchTile {
    int32_t matrix;
    int32_t row_begin;
    int32_t row_end;
    int32_t lanes_log2;  // 1..6: 2..64 lanes per row; kBlockRow: 256 lanes, one row per pass
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
                                                       const BatchTile *__restrict__ tiles,
                                                       int32_t n_tiles,
                                                       int32_t *__restrict__ counter) {
    __shared__ int32_t s_rp[kBlock / 2 + 1];  // row pointers of one pass (>= 2 lanes per row)
    __shared__ int32_t s_tile;
    __shared__ double s_part[kBlock / kWave];
    for (;;) {
        if (threadIdx.x == 0) s_tile = atomicAdd(counter, 1);
        __syncthreads();
        const int32_t t = s_tile;
        __syncthreads();  // every thread has read s_tile before thread 0 takes the next tile
        if (t >= n_tiles) break;
        const BatchTile tl = tiles[t];
        const BatchDesc d = desc[tl.matrix];
        if (tl.lanes_log2 == kBlockRow) {
            // one long row per pass, all 256 lanes: wave shuffles, then LDS across waves
            for (int64_t r = tl.row_begin; r < tl.row_end; ++r) {
                const int32_t s = d.rp[r], e = d.rp[r + 1];
                double p = csr_row_partial4<V, kBlock, UNROLL>(d.col, (const V *)d.val,
                                                               (const V *)d.x, s, e, threadIdx.x);
                p = group_sum<kWave>(p);
                if ((threadIdx.x & (kWave - 1)) == 0) s_part[threadIdx.x / kWave] = p;
                __syncthreads();
                if (threadIdx.x == 0) {
                    double tot = 0.0;
#pragma unroll
                    for (int w = 0; w < kBlock / kWave; ++w) tot += s_part[w];
                    store_y((V *)d.y, r, tot, (V)d.alpha, (V)d.beta);
                }
                __syncthreads();
            }
            continue;
        }
        const int rpb = kBlock >> tl.lanes_log2;  // rows per pass
        const int64_t row_end = tl.row_end;
        for (int64_t r = tl.row_begin; r < row_end; r += rpb) {
            for (int i = threadIdx.x; i <= rpb; i += kBlock)
                s_rp[i] = d.rp[std::min<int64_t>(r + i, row_end)];
            __syncthreads();
            switch (tl.lanes_log2) {
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

// Tiling 2: tile = one sorted block (matrix, block index in row_begin).
template <class V, int ITEMS>
__global__ __launch_bounds__(kSortedBlock) void batch_sorted_kernel(
    const BatchDesc *__restrict__ desc, const BatchTile *__restrict__ tiles, int32_t n_tiles,
    int32_t *__restrict__ counter) {
    __shared__ double s_y[kBatchSortedRows];
    __shared__ int32_t s_tile;
    for (;;) {
        if (threadIdx.x == 0) s_tile = atomicAdd(counter, 1);
        __syncthreads();
        const int32_t t = s_tile;
        __syncthreads();  // every thread has read s_tile before thread 0 takes the next tile
        if (t >= n_tiles) break;
        const BatchTile tl = tiles[t];
        const BatchDesc d = desc[tl.matrix];
        const int64_t row0 = d.sblk_row[tl.row_begin];
        const int nr = d.sblk_row[tl.row_begin + 1] - d.sblk_row[tl.row_begin];
        for (int i = threadIdx.x; i < nr; i += kSortedBlock) s_y[i] = 0.0;
        __syncthreads();
        const int64_t bs = d.sblk[tl.row_begin], be = d.sblk[tl.row_begin + 1];
        if (d.srows16)
            sorted_block_sum<V, ITEMS, kSortedWaves, true>(d.sidx, d.srows16, (const V *)d.sval,
                                                           (const V *)d.x, bs, be, d.scol_bits,
                                                           d.slast, s_y);
        else
            sorted_block_sum<V, ITEMS, kSortedWaves, false>(d.sidx, nullptr, (const V *)d.sval,
                                                            (const V *)d.x, bs, be, d.scol_bits,
                                                            d.slast, s_y);
        __syncthreads();
        for (int i = threadIdx.x; i < nr; i += kSortedBlock)
            store_y((V *)d.y, row0 + i, s_y[i], (V)d.alpha, (V)d.beta);
    }
}

using BatchKernel = void (*)(const BatchDesc *, const BatchTile *, int32_t, int32_t *);

BatchKernel kernel_for(spmv_dtype dt, int unroll, int tiling) {
    if (tiling == 2) {
        if (dt == SPMV_F64)
            return unroll == 4   ? batch_sorted_kernel<double, 16>
                   : unroll == 2 ? batch_sorted_kernel<double, 8>
                                 : batch_sorted_kernel<double, 4>;
        return unroll == 4   ? batch_sorted_kernel<float, 16>
               : unroll == 2 ? batch_sorted_kernel<float, 8>
                             : batch_sorted_kernel<float, 4>;
    }
    if (dt == SPMV_F64) return unroll == 2 ? batch_kernel<double, 2> : batch_kernel<double, 1>;
    return unroll == 2 ? batch_kernel<float, 2> : batch_kernel<float, 1>;
}

// Smallest lanes_log2 in 1..6 whose lanes x 4 entries per load reach len / divisor.
int lanes_log2_for_len(double len, int divisor) {
    const double want = len / (4.0 * divisor);
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
    std::vector<std::vector<int32_t>> row_ptr;  // host copies, for tiling
    std::vector<spmv::BatchDesc> desc;
    std::vector<int32_t> lanes;  // per matrix, for the per-matrix tiling
    std::vector<spmv::SortedPart> sorted;  // per matrix, built on first use of tiling 2
    spmv::DevBuf d_desc, d_tiles, d_counter;
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

std::vector<BatchTile> plan_tiles(spmv_batch_s *b, const spmv_batch_config &c) {
    std::vector<BatchTile> tiles;
    b->lanes.assign(b->hs.size(), 0);
    if (c.tiling == 2) {  // one tile per sorted block, largest first
        std::vector<std::pair<int32_t, BatchTile>> sized;
        for (size_t m = 0; m < b->hs.size(); ++m) {
            const std::vector<int32_t> &rp = b->row_ptr[m];
            const std::vector<int32_t> &st = b->sorted[m].row_start;
            for (int32_t k = 0; k < b->sorted[m].blocks; ++k) {
                const int32_t r0 = st[k], r1 = st[k + 1];
                sized.push_back({rp[r1] - rp[r0], BatchTile{(int32_t)m, k, r1, 0}});
            }
        }
        std::stable_sort(sized.begin(), sized.end(),
                         [](const auto &a, const auto &z) { return a.first > z.first; });
        for (const auto &e : sized) tiles.push_back(e.second);
        return tiles;
    }
    for (size_t m = 0; m < b->hs.size(); ++m) {
        const spmv_matrix_s *h = b->hs[m];
        const std::vector<int32_t> &rp = b->row_ptr[m];
        const int32_t n = h->n_rows;
        const int lg_mean = lanes_log2_for_len(n ? (double)h->nnz / n : 0.0, c.lanes_divisor);
        b->lanes[m] = 1 << lg_mean;
        const int32_t rows_per_tile = (kBlock >> lg_mean) * c.passes_per_tile;
        if (c.tiling == 0) {
            for (int32_t r = 0; r < n; r += rows_per_tile)
                tiles.push_back({(int32_t)m, r, std::min(n, r + rows_per_tile), lg_mean});
            continue;
        }
        int32_t r = 0;
        while (r < n) {
            if (rp[r + 1] - rp[r] >= kLongRow) {
                tiles.push_back({(int32_t)m, r, r + 1, kBlockRow});
                ++r;
                continue;
            }
            int32_t r_end = r, mx = 0;
            while (r_end < n && r_end - r < rows_per_tile && rp[r_end + 1] - rp[r_end] < kLongRow) {
                mx = std::max(mx, rp[r_end + 1] - rp[r_end]);
                ++r_end;
            }
            tiles.push_back({(int32_t)m, r, r_end,
                             std::max(lg_mean, lanes_log2_for_len(mx, c.lanes_divisor))});
            r = r_end;
        }
    }
    if (tiles.size() > (size_t)INT32_MAX / 2) fail(SPMV_ERR_INVALID_ARG, "batch has too many tiles");
    return tiles;
}

void upload_desc(spmv_batch_s *b, hipStream_t s) {
    SPMV_HIP(hipMemcpyAsync(b->d_desc.p, b->desc.data(), b->desc.size() * sizeof(BatchDesc),
                            hipMemcpyHostToDevice, s));
}

// The batch's own sorted-block COO copy of every matrix, built on first use of tiling 2.
void ensure_sorted(spmv_batch_s *b, hipStream_t s) {
    if (!b->sorted.empty()) return;
    std::vector<SortedPart> parts(b->hs.size());
    for (size_t m = 0; m < b->hs.size(); ++m) {
        // blocks of 4096 rows (fewer if the packed index holds at least 1024)
        const int32_t packed = sorted_packed_rows(b->hs[m]);
        const int32_t rows = std::min(
            {kBatchSortedRows, packed >= 1024 ? packed : kBatchSortedRows, sorted_max_rows(b->hs[m])});
        const int32_t n = b->hs[m]->n_rows;
        std::vector<int32_t> row_start;
        for (int64_t r = 0; r < n; r += rows) row_start.push_back((int32_t)r);
        row_start.push_back(n);
        build_sorted_into(b->hs[m], matrix_entries(b->hs[m]), b->row_ptr[m], row_start, parts[m], s);
    }
    b->sorted = std::move(parts);
    for (size_t m = 0; m < b->hs.size(); ++m) {
        const SortedPart &P = b->sorted[m];
        BatchDesc &d = b->desc[m];
        d.sblk = P.blk_ptr.as<int32_t>();
        d.sidx = P.idx.as<int32_t>();
        d.sval = P.val.p;
        d.srows16 = P.rows16.as<uint16_t>();
        d.slast = padded_count(P.stream) - 8;  // covers 4 and 8 entries per lane
        d.sblk_row = P.blk_row.as<int32_t>();
        d.scol_bits = P.col_bits;
    }
}

// (Re)build the graph {reset counter, persistent kernel} for configuration c.
void build_graph(spmv_batch_s *b, const spmv_batch_config &c, hipStream_t user) {
    spmv_batch_config cc = c;
    if (cc.tiling == 2) ensure_sorted(b, user);
    const std::vector<BatchTile> tiles = plan_tiles(b, cc);
    cc.total_tiles = (int32_t)tiles.size();
    cc.grid = std::max(1, std::min(cc.total_tiles, b->num_cu * cc.blocks_per_cu));
    cc.block = cc.tiling == 2 ? kSortedBlock : kBlock;
    SPMV_HIP(hipStreamSynchronize(user));  // no earlier run may still read the old tiles
    b->d_tiles.alloc(std::max<size_t>(tiles.size(), 1) * sizeof(BatchTile));
    if (!tiles.empty())
        SPMV_HIP(hipMemcpy(b->d_tiles.p, tiles.data(), tiles.size() * sizeof(BatchTile),
                           hipMemcpyHostToDevice));
    upload_desc(b, user);
    SPMV_HIP(hipStreamSynchronize(user));
    if (b->exec) { SPMV_HIP(hipGraphExecDestroy(b->exec)); b->exec = nullptr; }
    if (b->graph) { SPMV_HIP(hipGraphDestroy(b->graph)); b->graph = nullptr; }
    hipStream_t cs = b->capture_stream;
    SPMV_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    reset_counter<<<1, 1, 0, cs>>>(b->d_counter.as<int32_t>());
    if (cc.total_tiles > 0) {
        BatchKernel k = kernel_for(b->dt, cc.unroll, cc.tiling);
        k<<<cc.grid, cc.block, 0, cs>>>(b->d_desc.as<BatchDesc>(), b->d_tiles.as<BatchTile>(),
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
    }
    // One launch computes every product, so no y may share a byte with any x or
    // any other y (the x vectors may be shared: they are only read).
    struct Range {
        uintptr_t b, e;
        size_t i;
    };
    std::vector<Range> yr, xr;
    for (size_t i = 0; i < b->hs.size(); ++i) {
        const spmv_matrix_s *h = b->hs[i];
        const BatchDesc &d = b->desc[i];
        if (h->n_rows > 0) yr.push_back({(uintptr_t)d.y, (uintptr_t)d.y + (size_t)h->n_rows * vs, i});
        if (h->n_cols > 0) xr.push_back({(uintptr_t)d.x, (uintptr_t)d.x + (size_t)h->n_cols * vs, i});
    }
    std::sort(yr.begin(), yr.end(), [](const Range &a, const Range &c) { return a.b < c.b; });
    for (size_t k = 1; k < yr.size(); ++k)
        if (yr[k].b < yr[k - 1].e)
            fail(SPMV_ERR_INVALID_ARG, "y of matrices %zu and %zu overlap", yr[k - 1].i, yr[k].i);
    for (const Range &x : xr) {
        // the y ranges are disjoint and sorted: only the last one starting before x ends can meet it
        auto it = std::lower_bound(yr.begin(), yr.end(), x.e,
                                   [](const Range &a, uintptr_t v) { return a.b < v; });
        if (it != yr.begin() && (it - 1)->e > x.b)
            fail(SPMV_ERR_INVALID_ARG, "x of matrix %zu overlaps y of matrix %zu", x.i, (it - 1)->i);
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
        b->row_ptr.resize(count);
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
            b->row_ptr[i].resize((size_t)h->n_rows + 1);
            SPMV_HIP(hipMemcpy(b->row_ptr[i].data(), h->row_ptr.p, ((size_t)h->n_rows + 1) * 4,
                               hipMemcpyDeviceToHost));
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
        dflt.tiling = 1;
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
        std::vector<spmv_batch_config> grid_cfgs;
        for (int tiling : {0, 1})
            for (int unroll : {1, 2})
                for (int passes : {1, 4, 16})
                    for (int bpc : {4, 8})
                        for (int div : {1, 2}) {
                            spmv_batch_config c{};
                            c.tiling = tiling;
                            c.unroll = unroll;
                            c.passes_per_tile = passes;
                            c.blocks_per_cu = bpc;
                            c.lanes_divisor = div;
                            grid_cfgs.push_back(c);
                        }
        bool sorted_ok = true;
        for (int32_t i = 0; i < count; ++i) {
            try {
                (void)sorted_max_rows(hs[i]);
            } catch (const Error &e) {
                if (e.status != SPMV_ERR_NOT_APPLICABLE) throw;
                clear_error();
                sorted_ok = false;
            }
        }
        if (sorted_ok)
            for (int unroll : {1, 2, 4})
                for (int bpc : {1, 2}) {
                    spmv_batch_config c{};
                    c.tiling = 2;
                    c.unroll = unroll;
                    c.passes_per_tile = 1;
                    c.blocks_per_cu = bpc;
                    c.lanes_divisor = 1;
                    grid_cfgs.push_back(c);
                }
        for (const spmv_batch_config &gc : grid_cfgs) {
            build_graph(b, gc, s);
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

extern "C" spmv_status spmv_batch_run(spmv_batch b, const double *alphas, const void *const *xs,
                                      const double *betas, void *const *ys, void *stream) {
    return guard([&] {
        if (!b || !b->exec) fail(SPMV_ERR_INVALID_ARG, "NULL batch");
        if (alphas || xs || betas || ys) {
            std::vector<BatchDesc> keep = b->desc;
            try {
                set_io(b, xs, ys, alphas, betas);
            } catch (...) {
                b->desc = keep;
                throw;
            }
            upload_desc(b, (hipStream_t)stream);
        }
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
            for (size_t i = 0; i < b->lanes.size(); ++i) lanes[i] = b->lanes[i];
    });
}

extern "C" spmv_status spmv_batch_set_config(spmv_batch b, const spmv_batch_config *cfg,
                                             void *stream) {
    return guard([&] {
        if (!b || !cfg) fail(SPMV_ERR_INVALID_ARG, "NULL argument");
        const bool unroll_ok = cfg->unroll == 1 || cfg->unroll == 2 ||
                               (cfg->unroll == 4 && cfg->tiling == 2);
        if (!unroll_ok || cfg->passes_per_tile < 1 || cfg->blocks_per_cu < 1 ||
            cfg->lanes_divisor < 1 || cfg->tiling < 0 || cfg->tiling > 2)
            fail(SPMV_ERR_INVALID_ARG, "bad batch setting");
        build_graph(b, *cfg, (hipStream_t)stream);
    });
}

extern "C" void spmv_batch_destroy(spmv_batch b) {
    if (!b) return;
    (void)hipDeviceSynchronize();
    delete b;
}
