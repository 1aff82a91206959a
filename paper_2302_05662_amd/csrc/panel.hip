// Streaming COO SpMV over column-panel ordered entries.
//
// A format's entries may be kept in any order (paper, Background: sparse
// formats; COO stores explicit coordinates). This copy of the COO entries is
// ordered for MI355X's memory system: rows are split into groups, one per
// wavefront, and a group's entries are stored contiguously in column-panel
// order (16384 columns per panel, then row, then column). Every wavefront
// streams its own group with aligned 16-byte loads, the next chunk in flight
// while the current chunk's x gathers are outstanding, and all wavefronts of
// an XCD sweep x from the first panel to the last at about the same pace. A
// row-parallel CSR kernel gathers from all of x at once; here the gathers of
// an XCD fall in a moving window of x, so x vectors larger than one XCD's
// 4 MB L2 are still served from L2 rather than the Infinity Cache.
//
// Products are summed by row with a segmented scan across the wave; the row
// sums go into an FP64 accumulator in LDS that only this wave touches (one
// row can end two segments of a chunk, from two panels, so the add is a
// local atomic). Row totals are written once at the end as
// y = alpha * s + beta * y.
//
// The sorted-block COO kernel goes further: a workgroup owns a block of up to
// 16384 rows whose entries are sorted by column, and its 16 wavefronts stream
// its chunks in turn, each 256-entry chunk stored transposed so that one
// gather instruction reads 64 consecutive sorted entries. Those lanes read
// nearby columns and share cache lines (on a uniformly random matrix with ~33 entries per row
// and 256 blocks, about 4 entries per 128-byte line of x), so a gather moves a
// quarter of the lines a row-ordered kernel moves. Each product is added to
// the row's FP64 accumulator in LDS with a local atomic; the order in which
// the wavefronts' adds land is not fixed, so results may differ between runs
// in the last bits of the FP64 sums (FP32 outputs almost never change).
#include <algorithm>
#include <climits>

#include "common.hpp"
#include "device.hpp"

namespace spmv {
namespace {

constexpr int kB = 256;                   // builder workgroup size
constexpr int kNT = kPanelWaves * kWave;  // streaming kernel workgroup size
constexpr int kBlocksPerCu = 2;
constexpr uint32_t kColMask = (1u << kPanelColBits) - 1;

int grid_of_n(int64_t n) {
    return (int)std::min<int64_t>(std::max<int64_t>(ceil_div(n, kB), 1), 65536);
}

// ---- the kernel ----------------------------------------------------------------

template <class V, int ITEMS>
__global__ __launch_bounds__(kNT) void coo_panel_kernel(
    int32_t n_rows, int32_t rw, const int32_t *__restrict__ group_ptr,
    const int32_t *__restrict__ idx, const V *__restrict__ val, int64_t last_load,
    const V *__restrict__ x, V alpha, V beta, V *__restrict__ y) {
    constexpr int CH = kWave * ITEMS;
    __shared__ double s_y[kPanelWaves * kPanelRowsMax];
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int lane = threadIdx.x % kWave;
    const int64_t g = (int64_t)blockIdx.x * kPanelWaves + w;
    const int64_t row0 = g * rw;
    double *sy = s_y + w * kPanelRowsMax;
    for (int i = lane; i < rw; i += kWave) sy[i] = 0.0;
    const int64_t start = group_ptr[g], end = group_ptr[g + 1];

    using CI = Pack<int32_t, ITEMS>;
    using CV = Pack<V, ITEMS>;
    // Chunk at stream position q (a multiple of 4): lane l holds entries
    // q + ITEMS*l .. + ITEMS-1. The load address is clamped into the arrays;
    // entries at or past `end` are masked.
    auto load = [&](int64_t q, CI &c, CV &v) {
        const int64_t e = std::min<int64_t>(q + ITEMS * lane, last_load);
        c = ld_i32<ITEMS>(idx + e);
        v = ld_val<ITEMS>(val + e);
    };
    // Gathers of chunk q, then the loads of the next chunk, then the sums.
    auto step = [&](int64_t q, const CI &c, const CV &v, CI &cn, CV &vn) {
        V xv[ITEMS];
        bool ok[ITEMS];
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
            ok[j] = (q + ITEMS * lane + j < end) && c.v[j] != kPanelPad;
            xv[j] = x[ok[j] ? ((uint32_t)c.v[j] & kColMask) : 0u];
        }
        __builtin_amdgcn_sched_barrier(0);
        load(q + CH, cn, vn);
        __builtin_amdgcn_sched_barrier(0);
        int32_t r[ITEMS];
        double pr[ITEMS];
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
            r[j] = ok[j] ? (int32_t)((uint32_t)c.v[j] >> kPanelColBits) : -1;
            const double p = (double)v.v[j] * (double)xv[j];
            pr[j] = ok[j] ? p : 0.0;
        }
        int32_t prev_last = __shfl_up(r[ITEMS - 1], 1, kWave);
        if (lane == 0) prev_last = INT_MIN;
        int32_t next_first = __shfl_down(r[0], 1, kWave);
        if (lane == kWave - 1) next_first = INT_MIN;
        bool f = false;
        double s = 0.0;
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
            const bool head = (j == 0) ? (r[0] != prev_last) : (r[j] != r[j - 1]);
            if (head) { f = true; s = pr[j]; } else { s += pr[j]; }
        }
        bool fi = f;
        double si = s;
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) {
            const int of = __shfl_up((int)fi, d, kWave);
            const double os = __shfl_up(si, d, kWave);
            if (lane >= d) {
                if (!fi) si += os;
                fi = fi || of;
            }
        }
        double run = __shfl_up(si, 1, kWave);  // open segment entering this lane
        if (lane == 0) run = 0.0;
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
            const bool head = (j == 0) ? (r[0] != prev_last) : (r[j] != r[j - 1]);
            run = head ? pr[j] : run + pr[j];
            const bool tail = (j == ITEMS - 1) ? (r[j] != next_first) : (r[j] != r[j + 1]);
            if (tail && r[j] >= 0) atomicAdd(&sy[r[j]], run);
        }
    };
    CI cA, cB;
    CV vA, vB;
    load(start, cA, vA);
    for (int64_t q = start;;) {  // two steps per pass: the chunk buffers alternate
        if (q >= end) break;
        step(q, cA, vA, cB, vB);
        q += CH;
        if (q >= end) break;
        step(q, cB, vB, cA, vA);
        q += CH;
    }
    for (int i = lane; i < rw; i += kWave) {
        const int64_t row = row0 + i;
        if (row < n_rows) store_y(y, row, sy[i], alpha, beta);
    }
}

// ---- the builder ----------------------------------------------------------------

__global__ void panel_keys(const int32_t *__restrict__ row, const int32_t *__restrict__ col,
                           int64_t nnz, int32_t rw, int32_t panels, uint64_t *__restrict__ key,
                           uint32_t *__restrict__ perm) {
    for (int64_t k = (int64_t)blockIdx.x * kB + threadIdx.x; k < nnz; k += (int64_t)gridDim.x * kB) {
        key[k] = (uint64_t)(row[k] / rw) * (uint64_t)panels + (uint64_t)(col[k] / kPanelWidth);
        perm[k] = (uint32_t)k;
    }
}

// first[g] = entries of the row groups before g (rows are sorted, so this is
// the CSR row pointer at the group's first row); padded[g] = group size
// rounded up to a multiple of 4.
__global__ void panel_groups(const int32_t *__restrict__ row_ptr, int32_t n_rows, int64_t groups,
                             int32_t rw, int32_t *__restrict__ first, int32_t *__restrict__ padded) {
    for (int64_t t = (int64_t)blockIdx.x * kB + threadIdx.x; t <= groups;
         t += (int64_t)gridDim.x * kB) {
        const int64_t r0 = std::min<int64_t>(t * rw, n_rows);
        first[t] = row_ptr[r0];
        if (t < groups) {
            const int64_t r1 = std::min<int64_t>((t + 1) * rw, n_rows);
            padded[t] = (row_ptr[r1] - row_ptr[r0] + 3) & ~3;
        } else {
            padded[t] = 0;
        }
    }
}

template <class V>
__global__ void panel_scatter(const uint32_t *__restrict__ perm, int64_t nnz,
                              const int32_t *__restrict__ row, const int32_t *__restrict__ col,
                              const V *__restrict__ val, const int32_t *__restrict__ first,
                              const int32_t *__restrict__ start, int32_t rw,
                              int32_t *__restrict__ idx_out, V *__restrict__ val_out) {
    for (int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x; i < nnz; i += (int64_t)gridDim.x * kB) {
        const uint32_t e = perm[i];
        const int32_t r = row[e];
        const int64_t g = r / rw;
        // the sort keeps groups in order, so entry i is entry (i - first[g]) of group g
        const int64_t pos = (int64_t)start[g] + (i - first[g]);
        idx_out[pos] = (int32_t)(((uint32_t)(r % rw) << kPanelColBits) | (uint32_t)col[e]);
        val_out[pos] = val[e];
    }
}

template <class V, int ITEMS>
void launch_panel(const spmv_matrix_s *h, double alpha, const void *x, double beta, void *y,
                  hipStream_t s) {
    const PanelPart &P = h->panel;
    const int64_t cap = padded_count(P.stream);
    coo_panel_kernel<V, ITEMS><<<P.blocks, kNT, 0, s>>>(
        h->n_rows, P.rows_per_wave, P.group_ptr.as<int32_t>(), P.idx.as<int32_t>(), P.val.as<V>(),
        cap - ITEMS, (const V *)x, (V)alpha, (V)beta, (V *)y);
    SPMV_CHECK_LAUNCH();
}

// ---- sorted-block COO ------------------------------------------------------------

constexpr int kST = kSortedWaves * kWave;

// ACCUM: y += alpha * s for the rows the block has entries of (the HYB tail
// after its ELL part), else y = alpha * s + beta * y for every row.
template <class V, int ITEMS, bool ROW16, bool ACCUM>
__global__ __launch_bounds__(kST) void coo_sorted_kernel(
    const int32_t *__restrict__ blk_row, const int32_t *__restrict__ blk_order, int32_t col_bits,
    const int32_t *__restrict__ blk_ptr, const int32_t *__restrict__ idx,
    const uint16_t *__restrict__ rows16, const V *__restrict__ val, int64_t last_load,
    const V *__restrict__ x, V alpha, V beta, V *__restrict__ y) {
    __shared__ double s_y[kSortedRowsMax];
    const int32_t b = blk_order[blockIdx.x];
    const int64_t row0 = blk_row[b];
    const int nr = blk_row[b + 1] - blk_row[b];
    for (int i = threadIdx.x; i < nr; i += kST) s_y[i] = 0.0;
    __syncthreads();
    sorted_block_sum<V, ITEMS, kSortedWaves, ROW16>(idx, rows16, val, x, blk_ptr[b], blk_ptr[b + 1],
                                                    col_bits, last_load, s_y);
    __syncthreads();
    for (int i = threadIdx.x; i < nr; i += kST) {
        if constexpr (ACCUM) {
            if (s_y[i] != 0.0) y[row0 + i] = (V)((double)y[row0 + i] + (double)alpha * s_y[i]);
        } else {
            store_y(y, row0 + i, s_y[i], alpha, beta);
        }
    }
}

// Block holding row r: the last b with blk_row[b] <= r (blocks are never empty).
__device__ __forceinline__ int32_t sorted_block_of(const int32_t *__restrict__ blk_row,
                                                   int32_t blocks, int32_t r) {
    int32_t lo = 0, hi = blocks - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (blk_row[mid] <= r) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// key = (block << col_bits) | col: a block's entries sort together, by column.
__global__ void sorted_keys(const int32_t *__restrict__ row, const int32_t *__restrict__ col,
                            int64_t nnz, const int32_t *__restrict__ blk_row, int32_t blocks,
                            int32_t col_bits, uint64_t *__restrict__ key,
                            uint32_t *__restrict__ perm) {
    for (int64_t k = (int64_t)blockIdx.x * kB + threadIdx.x; k < nnz; k += (int64_t)gridDim.x * kB) {
        const int32_t b = sorted_block_of(blk_row, blocks, row[k]);
        key[k] = ((uint64_t)b << col_bits) | (uint64_t)col[k];
        perm[k] = (uint32_t)k;
    }
}

// first[b] = entries of the blocks before b; padded[b] = block b's stored
// length: a whole number of chunks.
__global__ void sorted_blocks(const int32_t *__restrict__ row_ptr,
                              const int32_t *__restrict__ blk_row, int64_t blocks,
                              int32_t *__restrict__ first, int32_t *__restrict__ padded) {
    for (int64_t t = (int64_t)blockIdx.x * kB + threadIdx.x; t <= blocks;
         t += (int64_t)gridDim.x * kB) {
        first[t] = row_ptr[blk_row[t]];
        int32_t len = 0;
        if (t < blocks) {
            const int64_t cnt = row_ptr[blk_row[t + 1]] - row_ptr[blk_row[t]];
            len = (int32_t)((cnt + kSortedChunk - 1) / kSortedChunk * kSortedChunk);
        }
        padded[t] = len;
    }
}

// Entry k of block b (in column order) goes to chunk k / 256, transposed inside
// it: row-major (64 lanes x 4) storage of the column-major order, so lane l's
// 16-byte group holds entries l, l+64, l+128, l+192.
// With rows16 set, the index is the column and the row inside the block goes to
// rows16 at the same position.
template <class V>
__global__ void sorted_scatter(const uint32_t *__restrict__ perm, int64_t nnz,
                               const int32_t *__restrict__ row, const int32_t *__restrict__ col,
                               const V *__restrict__ val, const int32_t *__restrict__ first,
                               const int32_t *__restrict__ start,
                               const int32_t *__restrict__ blk_row, int32_t blocks,
                               int32_t col_bits, int32_t *__restrict__ idx_out,
                               uint16_t *__restrict__ rows16, V *__restrict__ val_out) {
    for (int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x; i < nnz; i += (int64_t)gridDim.x * kB) {
        const uint32_t e = perm[i];
        const int32_t r = row[e];
        const int32_t b = sorted_block_of(blk_row, blocks, r);
        const uint32_t rin = (uint32_t)(r - blk_row[b]);
        const int64_t k = i - first[b], rr = k % kSortedChunk;
        const int64_t pos = (int64_t)start[b] + (k - rr) + (rr % kWave) * 4 + rr / kWave;
        if (rows16) {
            idx_out[pos] = col[e];
            rows16[pos] = (uint16_t)rin;
        } else {
            idx_out[pos] = (int32_t)((rin << col_bits) | (uint32_t)col[e]);
        }
        val_out[pos] = val[e];
    }
}

template <class V, int ITEMS, bool ACCUM = false>
void launch_sorted(const SortedPart &P, double alpha, const void *x, double beta, void *y,
                   hipStream_t s) {
    if (P.blocks == 0) return;
    const int64_t cap = padded_count(P.stream);
    if (P.row16)
        coo_sorted_kernel<V, ITEMS, true, ACCUM><<<P.blocks, kST, 0, s>>>(
            P.blk_row.as<int32_t>(), P.blk_order.as<int32_t>(), P.col_bits,
            P.blk_ptr.as<int32_t>(), P.idx.as<int32_t>(), P.rows16.as<uint16_t>(), P.val.as<V>(),
            cap - 4, (const V *)x, (V)alpha, (V)beta, (V *)y);
    else
        coo_sorted_kernel<V, ITEMS, false, ACCUM><<<P.blocks, kST, 0, s>>>(
            P.blk_row.as<int32_t>(), P.blk_order.as<int32_t>(), P.col_bits,
            P.blk_ptr.as<int32_t>(), P.idx.as<int32_t>(), nullptr, P.val.as<V>(), cap - 4,
            (const V *)x, (V)alpha, (V)beta, (V *)y);
    SPMV_CHECK_LAUNCH();
}

// ---- column tiles of the sorted-block layout -------------------------------------

// Workgroup i runs tile t = blk_order[i]: rows of block t >> tiles_log2, entries
// of column range h = t mod 2^tiles_log2. Range 0 writes y = alpha * s + beta * y,
// range h > 0 writes alpha * s to partial row h - 1 (sorted_tiles_combine adds
// them afterwards).
template <class V, int ITEMS, bool ROW16, bool DELTA>
__global__ __launch_bounds__(kST) void coo_tiles_kernel(
    const int32_t *__restrict__ blk_row, const int32_t *__restrict__ blk_order, int32_t col_bits,
    const int32_t *__restrict__ blk_ptr, const int32_t *__restrict__ idx,
    const uint16_t *__restrict__ rows16, const V *__restrict__ val, int64_t last_load,
    const int32_t *__restrict__ chunk_base, int64_t last_chunk, int32_t tiles_log2, int64_t pitch,
    const V *__restrict__ x, V alpha, V beta, V *__restrict__ y, V *__restrict__ partial) {
    __shared__ double s_y[kSortedRowsMax];
    const int32_t t = blk_order[blockIdx.x];
    const int32_t b = t >> tiles_log2, hh = t & ((1 << tiles_log2) - 1);
    const int64_t row0 = blk_row[b];
    const int nr = blk_row[b + 1] - blk_row[b];
    for (int i = threadIdx.x; i < nr; i += kST) s_y[i] = 0.0;
    __syncthreads();
    sorted_block_sum<V, ITEMS, kSortedWaves, ROW16, DELTA>(idx, rows16, val, x, blk_ptr[t],
                                                           blk_ptr[t + 1], col_bits, last_load,
                                                           s_y, chunk_base, last_chunk);
    __syncthreads();
    if (hh == 0) {
        for (int i = threadIdx.x; i < nr; i += kST) store_y(y, row0 + i, s_y[i], alpha, beta);
    } else {
        V *p = partial + (int64_t)(hh - 1) * pitch;
        for (int i = threadIdx.x; i < nr; i += kST) p[row0 + i] = (V)((double)alpha * s_y[i]);
    }
}

// y += the `parts` partial rows (the other column ranges' shares; partial h at
// h * pitch, pitch a multiple of 64), summed in FP64 in range order. With y
// 16-byte aligned (the partial rows always are), a thread adds 16 bytes of rows
// at a time, and the rows past the last whole group one by one.
template <class V>
__global__ void sorted_tiles_combine(int64_t n, int32_t parts, int64_t pitch,
                                     const V *__restrict__ partial, V *__restrict__ y) {
    constexpr int W = 16 / sizeof(V);
    typedef V vec_t __attribute__((ext_vector_type(W)));
    const int64_t tid = (int64_t)blockIdx.x * kB + threadIdx.x, stride = (int64_t)gridDim.x * kB;
    int64_t done = 0;
    if (((uintptr_t)y & 15) == 0) {
        const int64_t groups = n / W;
        for (int64_t g = tid; g < groups; g += stride) {
            const vec_t v = *(const vec_t *)(y + g * W);
            double acc[W];
#pragma unroll
            for (int j = 0; j < W; ++j) acc[j] = (double)v[j];
            for (int h = 0; h < parts; ++h) {
                const vec_t p = *(const vec_t *)(partial + h * pitch + g * W);
#pragma unroll
                for (int j = 0; j < W; ++j) acc[j] += (double)p[j];
            }
            vec_t out;
#pragma unroll
            for (int j = 0; j < W; ++j) out[j] = (V)acc[j];
            *(vec_t *)(y + g * W) = out;
        }
        done = groups * W;
    }
    for (int64_t r = done + tid; r < n; r += stride) {
        double acc = (double)y[r];
        for (int h = 0; h < parts; ++h) acc += (double)partial[h * pitch + r];
        y[r] = (V)acc;
    }
}

// key = (tile << col_bits) | col, tile = T * block + col / width.
__global__ void tiles_keys(const int32_t *__restrict__ row, const int32_t *__restrict__ col,
                           int64_t nnz, const int32_t *__restrict__ blk_row, int32_t blocks,
                           int32_t tiles, int32_t width, int32_t col_bits,
                           uint64_t *__restrict__ key, uint32_t *__restrict__ perm) {
    for (int64_t k = (int64_t)blockIdx.x * kB + threadIdx.x; k < nnz; k += (int64_t)gridDim.x * kB) {
        const int32_t b = sorted_block_of(blk_row, blocks, row[k]);
        const uint64_t t = (uint64_t)tiles * (uint64_t)b + (uint64_t)(col[k] / width);
        key[k] = (t << col_bits) | (uint64_t)col[k];
        perm[k] = (uint32_t)k;
    }
}

// first[t] = sorted keys below tile t's first key (t = 0 .. tiles); padded[t] =
// tile t's entries rounded up to whole chunks (padded[tiles] = 0).
__global__ void tiles_first(const uint64_t *__restrict__ skey, int64_t nnz, int64_t tiles,
                            int32_t col_bits, int32_t *__restrict__ first) {
    for (int64_t t = (int64_t)blockIdx.x * kB + threadIdx.x; t <= tiles;
         t += (int64_t)gridDim.x * kB) {
        const uint64_t want = (uint64_t)t << col_bits;
        int64_t lo = 0, hi = nnz;  // first position whose key >= want
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if (skey[mid] < want) lo = mid + 1; else hi = mid;
        }
        first[t] = (int32_t)lo;
    }
}

__global__ void tiles_padded(const int32_t *__restrict__ first, int64_t tiles,
                             int32_t *__restrict__ padded) {
    for (int64_t t = (int64_t)blockIdx.x * kB + threadIdx.x; t <= tiles;
         t += (int64_t)gridDim.x * kB) {
        const int64_t cnt = t < tiles ? first[t + 1] - first[t] : 0;
        padded[t] = (int32_t)((cnt + kSortedChunk - 1) / kSortedChunk * kSortedChunk);
    }
}

// Largest column span inside one chunk (last column less first) over all chunks.
__global__ void tiles_span(const uint64_t *__restrict__ skey, int64_t nnz,
                           const int32_t *__restrict__ first, int32_t col_bits,
                           uint32_t *__restrict__ span) {
    const uint64_t mask = (uint64_t(1) << col_bits) - 1;
    uint32_t best = 0;
    for (int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x; i < nnz; i += (int64_t)gridDim.x * kB) {
        const int64_t t = (int64_t)(skey[i] >> col_bits);
        const int64_t k = i - first[t];
        if (k % kSortedChunk != 0) continue;
        const int64_t last = std::min<int64_t>(i + kSortedChunk, first[t + 1]) - 1;
        best = std::max(best, (uint32_t)((skey[last] & mask) - (skey[i] & mask)));
    }
    if (best) atomicMax(span, best);
}

// Sorted position i goes to its tile's stream, transposed inside its chunk as in
// sorted_scatter. delta: index = row inside the block << col_bits | (column less
// the chunk's first column), and the chunk's first entry records that column;
// otherwise index = column and the row goes to rows16.
template <class V>
__global__ void tiles_scatter(const uint64_t *__restrict__ skey, const uint32_t *__restrict__ perm,
                              int64_t nnz, int32_t key_bits, const int32_t *__restrict__ row,
                              const V *__restrict__ val, const int32_t *__restrict__ first,
                              const int32_t *__restrict__ start,
                              const int32_t *__restrict__ blk_row, int32_t tiles_log2, bool delta,
                              int32_t col_bits, int32_t *__restrict__ idx_out,
                              uint16_t *__restrict__ rows16, int32_t *__restrict__ chunk_base,
                              V *__restrict__ val_out) {
    const uint64_t mask = (uint64_t(1) << key_bits) - 1;
    for (int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x; i < nnz; i += (int64_t)gridDim.x * kB) {
        const uint32_t e = perm[i];
        const int64_t t = (int64_t)(skey[i] >> key_bits);
        const uint32_t c = (uint32_t)(skey[i] & mask);
        const uint32_t rin = (uint32_t)(row[e] - blk_row[t >> tiles_log2]);
        const int64_t k = i - first[t], rr = k % kSortedChunk;
        const int64_t pos = (int64_t)start[t] + (k - rr) + (rr % kWave) * 4 + rr / kWave;
        if (delta) {
            const uint32_t c0 = (uint32_t)(skey[i - rr] & mask);
            idx_out[pos] = (int32_t)((rin << col_bits) | (c - c0));
            if (rr == 0) chunk_base[(start[t] + k) / kSortedChunk] = (int32_t)c;
        } else {
            idx_out[pos] = (int32_t)c;
            rows16[pos] = (uint16_t)rin;
        }
        val_out[pos] = val[e];
    }
}

template <class V, int ITEMS>
void launch_tiles(const SortedPart &P, int64_t n_rows, double alpha, const void *x, double beta,
                  void *y, hipStream_t s) {
    const int64_t cap = padded_count(P.stream);
    const int64_t last_chunk = std::max<int64_t>(P.stream / kSortedChunk - 1, 0);
    const int32_t grid = P.blocks * P.tiles;
    const int32_t tiles_log2 = P.tiles == 4 ? 2 : 1;
    if (P.delta)
        coo_tiles_kernel<V, ITEMS, false, true><<<grid, kST, 0, s>>>(
            P.blk_row.as<int32_t>(), P.blk_order.as<int32_t>(), P.col_bits,
            P.blk_ptr.as<int32_t>(), P.idx.as<int32_t>(), nullptr, P.val.as<V>(), cap - 4,
            P.chunk_base.as<int32_t>(), last_chunk, tiles_log2, P.pitch, (const V *)x, (V)alpha,
            (V)beta, (V *)y, P.partial.as<V>());
    else
        coo_tiles_kernel<V, ITEMS, true, false><<<grid, kST, 0, s>>>(
            P.blk_row.as<int32_t>(), P.blk_order.as<int32_t>(), P.col_bits,
            P.blk_ptr.as<int32_t>(), P.idx.as<int32_t>(), P.rows16.as<uint16_t>(), P.val.as<V>(),
            cap - 4, P.chunk_base.as<int32_t>(), last_chunk, tiles_log2, P.pitch, (const V *)x,
            (V)alpha, (V)beta, (V *)y, P.partial.as<V>());
    SPMV_CHECK_LAUNCH();
    sorted_tiles_combine<V><<<grid_of_n(ceil_div(n_rows, 16 / (int64_t)sizeof(V))), kB, 0, s>>>(
        n_rows, P.tiles - 1, P.pitch, P.partial.as<V>(), (V *)y);
    SPMV_CHECK_LAUNCH();
}

// ---- column-split COO ------------------------------------------------------------

__global__ void split_keys(const int32_t *__restrict__ col, int64_t nnz, int32_t width,
                           uint64_t *__restrict__ key, uint32_t *__restrict__ perm) {
    for (int64_t k = (int64_t)blockIdx.x * kB + threadIdx.x; k < nnz; k += (int64_t)gridDim.x * kB) {
        key[k] = (uint64_t)(col[k] / width);
        perm[k] = (uint32_t)k;
    }
}

// first[q] = number of sorted keys below q, for q = 0 .. n_keys.
__global__ void keys_first(const uint64_t *__restrict__ skey, int64_t nnz, int64_t n_keys,
                           int32_t *__restrict__ first) {
    for (int64_t q = (int64_t)blockIdx.x * kB + threadIdx.x; q <= n_keys;
         q += (int64_t)gridDim.x * kB) {
        int64_t lo = 0, hi = nnz;
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if (skey[mid] < (uint64_t)q) lo = mid + 1; else hi = mid;
        }
        first[q] = (int32_t)lo;
    }
}

template <class V>
__global__ void split_scatter(const uint64_t *__restrict__ skey, const uint32_t *__restrict__ perm,
                              int64_t nnz, const int32_t *__restrict__ row,
                              const int32_t *__restrict__ col, const V *__restrict__ val,
                              const int32_t *__restrict__ first, const int64_t *__restrict__ start,
                              int32_t *__restrict__ row_out, int32_t *__restrict__ col_out,
                              V *__restrict__ val_out) {
    for (int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x; i < nnz; i += (int64_t)gridDim.x * kB) {
        const uint64_t q = skey[i];
        const uint32_t e = perm[i];
        const int64_t pos = start[q] + (i - first[q]);
        row_out[pos] = row[e];
        col_out[pos] = col[e];
        val_out[pos] = val[e];
    }
}

}  // namespace

void build_split(spmv_matrix_s *h, hipStream_t s) {
    if (h->split.built) return;
    const int32_t width = split_width(h->dt);
    const int64_t panels = ceil_div(std::max<int64_t>(h->n_cols, 1), width);
    const int64_t nnz = h->nnz;
    if (panels < 2 || nnz > (int64_t)INT32_MAX / 2)
        fail(SPMV_ERR_NOT_APPLICABLE, "column-split COO needs more than %d columns", width);
    const size_t vs = dtype_size(h->dt);
    DevBuf keys, perm, first, dstart;
    keys.alloc(std::max<int64_t>(nnz, 1) * 8);
    perm.alloc(std::max<int64_t>(nnz, 1) * 4);
    first.alloc((panels + 1) * 4);
    if (nnz > 0) {
        split_keys<<<grid_of_n(nnz), kB, 0, s>>>(h->col.as<int32_t>(), nnz, width,
                                                 keys.as<uint64_t>(), perm.as<uint32_t>());
        SPMV_CHECK_LAUNCH();
        int bits = 0;
        while (bits < 64 && (uint64_t)(panels - 1) >> bits) ++bits;
        radix_sort_pairs(keys, perm, nnz, bits, s);
    }
    keys_first<<<grid_of_n(panels + 1), kB, 0, s>>>(keys.as<uint64_t>(), nnz, panels,
                                                    first.as<int32_t>());
    SPMV_CHECK_LAUNCH();
    std::vector<int32_t> hfirst(panels + 1);
    SPMV_HIP(hipMemcpyAsync(hfirst.data(), first.p, (panels + 1) * 4, hipMemcpyDeviceToHost, s));
    SPMV_HIP(hipStreamSynchronize(s));
    SplitPart P;
    P.panels = (int32_t)panels;
    P.width = width;
    P.start.assign(panels + 1, 0);
    P.count.assign(panels, 0);
    for (int64_t p = 0; p < panels; ++p) {
        P.count[p] = hfirst[p + 1] - hfirst[p];
        P.start[p + 1] = P.start[p] + (P.count[p] + 3) / 4 * 4;  // 16-byte aligned panels
    }
    const int64_t cap = padded_count(P.start[panels]);
    P.row.alloc(cap * 4);
    P.col.alloc(cap * 4);
    P.val.alloc(cap * vs);
    SPMV_HIP(hipMemsetAsync(P.row.p, 0, cap * 4, s));
    SPMV_HIP(hipMemsetAsync(P.col.p, 0, cap * 4, s));
    SPMV_HIP(hipMemsetAsync(P.val.p, 0, cap * vs, s));
    dstart.alloc((panels + 1) * 8);
    SPMV_HIP(hipMemcpyAsync(dstart.p, P.start.data(), (panels + 1) * 8, hipMemcpyHostToDevice, s));
    if (nnz > 0) {
        if (h->dt == SPMV_F64)
            split_scatter<double><<<grid_of_n(nnz), kB, 0, s>>>(
                keys.as<uint64_t>(), perm.as<uint32_t>(), nnz, h->row.as<int32_t>(),
                h->col.as<int32_t>(), h->val.as<double>(), first.as<int32_t>(),
                dstart.as<int64_t>(), P.row.as<int32_t>(), P.col.as<int32_t>(), P.val.as<double>());
        else
            split_scatter<float><<<grid_of_n(nnz), kB, 0, s>>>(
                keys.as<uint64_t>(), perm.as<uint32_t>(), nnz, h->row.as<int32_t>(),
                h->col.as<int32_t>(), h->val.as<float>(), first.as<int32_t>(),
                dstart.as<int64_t>(), P.row.as<int32_t>(), P.col.as<int32_t>(), P.val.as<float>());
        SPMV_CHECK_LAUNCH();
    }
    SPMV_HIP(hipStreamSynchronize(s));
    P.built = true;
    h->split = std::move(P);
}

namespace {
int sorted_col_bits(const spmv_matrix_s *h) {
    int col_bits = 1;
    while ((int64_t(1) << col_bits) <= h->n_cols) ++col_bits;  // n_cols < 2^col_bits
    return col_bits;
}
}  // namespace

int32_t sorted_max_rows(const spmv_matrix_s *h) {
    if (h->nnz > (int64_t)INT32_MAX / 2)
        fail(SPMV_ERR_NOT_APPLICABLE, "sorted-block COO holds at most 2^30 entries, not %lld",
             (long long)h->nnz);
    return kSortedRowsMax;
}

int32_t sorted_packed_rows(const spmv_matrix_s *h) {
    const int row_bits = 32 - sorted_col_bits(h);
    return row_bits < 1 ? 0 : (int32_t)std::min<int64_t>(kSortedRowsMax, int64_t(1) << row_bits);
}

std::vector<int32_t> sorted_balanced_rows(const std::vector<int32_t> &row_ptr, int32_t max_rows,
                                          int cus) {
    const int64_t n = (int64_t)row_ptr.size() - 1, nnz = n > 0 ? row_ptr[n] : 0;
    std::vector<int32_t> out;
    for (int64_t m = 1;; ++m) {
        const int64_t B = (int64_t)std::max(cus, 1) * m;
        // cuts at the rows where the entry count reaches b * nnz / B ...
        std::vector<int32_t> cut{0};
        for (int64_t b = 1; b < B; ++b) {
            const int64_t target = b * nnz / B;
            const int32_t r = (int32_t)(std::lower_bound(row_ptr.begin(), row_ptr.end(), target) -
                                        row_ptr.begin());
            if (r > cut.back() && r < n) cut.push_back(r);
        }
        if (n > cut.back()) cut.push_back((int32_t)n);
        // ... then blocks taller than max_rows split evenly
        out.assign(1, 0);
        for (size_t j = 1; j < cut.size(); ++j) {
            const int64_t a = cut[j - 1], h = cut[j] - a, k = ceil_div(h, max_rows);
            for (int64_t q = 1; q <= k; ++q) out.push_back((int32_t)(a + h * q / k));
        }
        if ((int64_t)out.size() - 1 <= B || m >= 64) return out;
    }
}

void build_sorted(spmv_matrix_s *h, hipStream_t s) {
    if (h->sorted.built) return;
    (void)sorted_max_rows(h);
    int cus = 0;
    SPMV_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, h->device));
    std::vector<int32_t> rp(h->n_rows + 1);
    SPMV_HIP(hipMemcpyAsync(rp.data(), h->row_ptr.p, rp.size() * 4, hipMemcpyDeviceToHost, s));
    SPMV_HIP(hipStreamSynchronize(s));
    // equal shares of the entries (a few long rows do not make one block the
    // slowest), as few blocks as possible, in whole rounds of one block per CU
    const std::vector<int32_t> row_start = sorted_balanced_rows(rp, kSortedRowsMax, cus);
    SortedPart P;
    build_sorted_into(h, matrix_entries(h), rp, row_start, P, s);
    h->sorted = std::move(P);
}

SortedEntries matrix_entries(const spmv_matrix_s *h) {
    return SortedEntries{h->nnz, h->row.as<int32_t>(), h->col.as<int32_t>(),
                         h->row_ptr.as<int32_t>(), h->val.p};
}

void build_hyb_sorted(spmv_matrix_s *h, hipStream_t s) {
    if (h->hyb_sorted.built) return;
    if (!h->hyb.built) fail(SPMV_ERR_NOT_CONVERTED, "HYB not converted");
    (void)sorted_max_rows(h);
    int cus = 0;
    SPMV_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, h->device));
    std::vector<int32_t> rp(h->n_rows + 1);
    SPMV_HIP(hipMemcpyAsync(rp.data(), h->hyb.tail_ptr.p, rp.size() * 4, hipMemcpyDeviceToHost, s));
    SPMV_HIP(hipStreamSynchronize(s));
    const std::vector<int32_t> row_start = sorted_balanced_rows(rp, kSortedRowsMax, cus);
    const SortedEntries tail{h->hyb.nnz_tail, h->hyb.tail_row.as<int32_t>(),
                             h->hyb.tail_col.as<int32_t>(), h->hyb.tail_ptr.as<int32_t>(),
                             h->hyb.tail_val.p};
    SortedPart P;
    build_sorted_into(h, tail, rp, row_start, P, s);
    h->hyb_sorted = std::move(P);
}

void build_sorted_into(const spmv_matrix_s *h, const SortedEntries &src,
                       const std::vector<int32_t> &row_ptr, const std::vector<int32_t> &row_start,
                       SortedPart &P, hipStream_t s) {
    const int32_t max_rows = sorted_max_rows(h);
    const int64_t n = h->n_rows, nnz = src.nnz;
    if ((int64_t)row_ptr.size() != n + 1 || row_start.empty() || row_start.front() != 0 ||
        row_start.back() != n)
        fail(SPMV_ERR_INVALID_ARG, "bad sorted block boundaries");
    const int64_t blocks = (int64_t)row_start.size() - 1;
    int32_t tallest = 0;
    for (int64_t b = 0; b < blocks; ++b) {
        const int32_t hgt = row_start[b + 1] - row_start[b];
        if (hgt < 1 || hgt > max_rows) fail(SPMV_ERR_INVALID_ARG, "bad sorted block height %d", hgt);
        tallest = std::max(tallest, hgt);
    }
    const int col_bits = sorted_col_bits(h);
    P = SortedPart{};
    P.col_bits = col_bits;
    P.rows = tallest;
    P.row16 = tallest > sorted_packed_rows(h);
    P.blocks = (int32_t)blocks;
    P.row_start = row_start;
    const size_t vs = dtype_size(h->dt);

    // workgroup order: largest block first, so the last round is the small blocks
    std::vector<int32_t> order(blocks);
    for (int64_t b = 0; b < blocks; ++b) order[b] = (int32_t)b;
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t c) {
        return row_ptr[row_start[a + 1]] - row_ptr[row_start[a]] >
               row_ptr[row_start[c + 1]] - row_ptr[row_start[c]];
    });
    P.blk_row.alloc((blocks + 1) * 4);
    P.blk_order.alloc(std::max<int64_t>(blocks, 1) * 4);
    SPMV_HIP(hipMemcpyAsync(P.blk_row.p, row_start.data(), (blocks + 1) * 4,
                            hipMemcpyHostToDevice, s));
    if (blocks > 0)
        SPMV_HIP(hipMemcpyAsync(P.blk_order.p, order.data(), blocks * 4, hipMemcpyHostToDevice, s));

    DevBuf keys, perm, first, start;
    first.alloc((blocks + 1) * 4);
    start.alloc((blocks + 1) * 4);
    sorted_blocks<<<grid_of_n(blocks + 1), kB, 0, s>>>(src.row_ptr, P.blk_row.as<int32_t>(), blocks,
                                                       first.as<int32_t>(), start.as<int32_t>());
    SPMV_CHECK_LAUNCH();
    exclusive_scan_i32(start.as<int32_t>(), start.as<int32_t>(), blocks + 1, s);
    int32_t total = 0;
    SPMV_HIP(hipMemcpyAsync(&total, start.as<int32_t>() + blocks, 4, hipMemcpyDeviceToHost, s));
    SPMV_HIP(hipStreamSynchronize(s));  // also keeps `order` alive until its copy is done
    P.stream = total;
    const int64_t cap = padded_count(total);
    P.idx.alloc(cap * 4);
    P.val.alloc(cap * vs);
    SPMV_HIP(hipMemsetAsync(P.idx.p, 0xFF, cap * 4, s));  // kPanelPad
    SPMV_HIP(hipMemsetAsync(P.val.p, 0, cap * vs, s));
    if (P.row16) {
        P.rows16.alloc(cap * 2);
        SPMV_HIP(hipMemsetAsync(P.rows16.p, 0, cap * 2, s));
    }
    if (nnz > 0) {
        keys.alloc(nnz * 8);
        perm.alloc(nnz * 4);
        sorted_keys<<<grid_of_n(nnz), kB, 0, s>>>(src.row, src.col, nnz, P.blk_row.as<int32_t>(),
                                                  P.blocks, col_bits, keys.as<uint64_t>(),
                                                  perm.as<uint32_t>());
        SPMV_CHECK_LAUNCH();
        int bits = col_bits;
        while (bits < 64 && (uint64_t)(blocks - 1) >> (bits - col_bits)) ++bits;
        radix_sort_pairs(keys, perm, nnz, bits, s);
        if (h->dt == SPMV_F64)
            sorted_scatter<double><<<grid_of_n(nnz), kB, 0, s>>>(
                perm.as<uint32_t>(), nnz, src.row, src.col, (const double *)src.val,
                first.as<int32_t>(), start.as<int32_t>(),
                P.blk_row.as<int32_t>(), P.blocks, col_bits, P.idx.as<int32_t>(),
                P.rows16.as<uint16_t>(), P.val.as<double>());
        else
            sorted_scatter<float><<<grid_of_n(nnz), kB, 0, s>>>(
                perm.as<uint32_t>(), nnz, src.row, src.col, (const float *)src.val,
                first.as<int32_t>(), start.as<int32_t>(),
                P.blk_row.as<int32_t>(), P.blocks, col_bits, P.idx.as<int32_t>(),
                P.rows16.as<uint16_t>(), P.val.as<float>());
        SPMV_CHECK_LAUNCH();
    }
    P.blk_ptr = std::move(start);
    SPMV_HIP(hipStreamSynchronize(s));
    P.built = true;
}

void build_sorted_tiles(spmv_matrix_s *h, int T, hipStream_t s) {
    if (T != 2 && T != 4) fail(SPMV_ERR_INVALID_ARG, "column tiles per block: 2 or 4, not %d", T);
    if (h->sorted_tiles[T == 4].built) return;
    (void)sorted_max_rows(h);
    int cus = 0;
    SPMV_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, h->device));
    std::vector<int32_t> rp(h->n_rows + 1);
    SPMV_HIP(hipMemcpyAsync(rp.data(), h->row_ptr.p, rp.size() * 4, hipMemcpyDeviceToHost, s));
    SPMV_HIP(hipStreamSynchronize(s));
    // blocks for 1/T of the CUs: their T tiles fill every CU once
    const int per_round = std::max(cus / T, 1);
    const std::vector<int32_t> row_start = sorted_balanced_rows(rp, kSortedRowsMax, per_round);
    const int64_t n = h->n_rows, nnz = h->nnz, blocks = (int64_t)row_start.size() - 1;
    if (T == 4 && blocks > per_round)
        fail(SPMV_ERR_NOT_APPLICABLE, "four column tiles need blocks of more than %d rows", kSortedRowsMax);
    const int64_t tiles = blocks * T;
    int32_t tallest = 0;
    for (int64_t b = 0; b < blocks; ++b) tallest = std::max(tallest, row_start[b + 1] - row_start[b]);
    const int key_bits = sorted_col_bits(h);
    const int32_t width = std::max<int32_t>((int32_t)ceil_div((int64_t)h->n_cols, T), 1);
    const size_t vs = dtype_size(h->dt);

    SortedPart P;
    P.tiles = T;
    P.pitch = ceil_div(std::max<int64_t>(n, 1), 64) * 64;
    P.blocks = (int32_t)blocks;
    P.rows = tallest;
    P.row_start = row_start;
    P.blk_row.alloc((blocks + 1) * 4);
    SPMV_HIP(hipMemcpyAsync(P.blk_row.p, row_start.data(), (blocks + 1) * 4, hipMemcpyHostToDevice, s));

    DevBuf keys, perm, first, start, span;
    first.alloc((tiles + 1) * 4);
    start.alloc((tiles + 1) * 4);
    span.alloc(4);
    keys.alloc(std::max<int64_t>(nnz, 1) * 8);
    perm.alloc(std::max<int64_t>(nnz, 1) * 4);
    SPMV_HIP(hipMemsetAsync(span.p, 0, 4, s));
    if (nnz > 0) {
        tiles_keys<<<grid_of_n(nnz), kB, 0, s>>>(h->row.as<int32_t>(), h->col.as<int32_t>(), nnz,
                                                 P.blk_row.as<int32_t>(), P.blocks, T, width,
                                                 key_bits, keys.as<uint64_t>(), perm.as<uint32_t>());
        SPMV_CHECK_LAUNCH();
        int bits = key_bits;
        while (bits < 64 && (uint64_t)(tiles - 1) >> (bits - key_bits)) ++bits;
        radix_sort_pairs(keys, perm, nnz, bits, s);
    }
    tiles_first<<<grid_of_n(tiles + 1), kB, 0, s>>>(keys.as<uint64_t>(), nnz, tiles, key_bits,
                                                    first.as<int32_t>());
    SPMV_CHECK_LAUNCH();
    tiles_padded<<<grid_of_n(tiles + 1), kB, 0, s>>>(first.as<int32_t>(), tiles, start.as<int32_t>());
    SPMV_CHECK_LAUNCH();
    exclusive_scan_i32(start.as<int32_t>(), start.as<int32_t>(), tiles + 1, s);
    if (nnz > 0) {
        tiles_span<<<grid_of_n(nnz), kB, 0, s>>>(keys.as<uint64_t>(), nnz, first.as<int32_t>(),
                                                 key_bits, span.as<uint32_t>());
        SPMV_CHECK_LAUNCH();
    }
    int32_t total = 0;
    uint32_t max_span = 0;
    std::vector<int32_t> hfirst(tiles + 1);
    SPMV_HIP(hipMemcpyAsync(&total, start.as<int32_t>() + tiles, 4, hipMemcpyDeviceToHost, s));
    SPMV_HIP(hipMemcpyAsync(&max_span, span.p, 4, hipMemcpyDeviceToHost, s));
    SPMV_HIP(hipMemcpyAsync(hfirst.data(), first.p, (tiles + 1) * 4, hipMemcpyDeviceToHost, s));
    SPMV_HIP(hipStreamSynchronize(s));
    // packed: row inside the block (tallest < 2^row_bits, so an index is never
    // all ones, the padding mark) above the column less its chunk's first
    int row_bits = 1;
    while ((int64_t(1) << row_bits) <= tallest) ++row_bits;
    const int delta_bits = 32 - row_bits;
    P.delta = delta_bits > 0 && (uint64_t)max_span < (uint64_t(1) << delta_bits) - 1;
    P.row16 = !P.delta;
    P.col_bits = P.delta ? delta_bits : key_bits;
    P.stream = total;

    // workgroup order: tiles of column range h at positions whose XCD (position
    // mod 8, as workgroups are dealt to the XCDs in turn) is in [8h/T, 8(h+1)/T),
    // so each XCD's L2 serves one range of x; larger tiles first within a range
    std::vector<std::vector<int32_t>> range(T);
    for (int64_t t = 0; t < tiles; ++t) range[t % T].push_back((int32_t)t);
    for (auto &v : range)
        std::stable_sort(v.begin(), v.end(), [&](int32_t a, int32_t c) {
            return hfirst[a + 1] - hfirst[a] > hfirst[c + 1] - hfirst[c];
        });
    std::vector<int32_t> order;
    std::vector<size_t> take(T, 0);
    for (int64_t w = 0; w < tiles; ++w) {
        int hh = (int)((w % 8) * T / 8);
        for (int k = 0; k < T && take[hh] == range[hh].size(); ++k) hh = (hh + 1) % T;
        order.push_back(range[hh][take[hh]++]);
    }
    P.blk_order.alloc(std::max<int64_t>(tiles, 1) * 4);
    if (tiles > 0)
        SPMV_HIP(hipMemcpyAsync(P.blk_order.p, order.data(), tiles * 4, hipMemcpyHostToDevice, s));

    const int64_t cap = padded_count(total);
    P.idx.alloc(cap * 4);
    P.val.alloc(cap * vs);
    P.chunk_base.alloc(std::max<int64_t>(total / kSortedChunk, 1) * 4);
    P.partial.alloc((T - 1) * P.pitch * vs);
    SPMV_HIP(hipMemsetAsync(P.idx.p, 0xFF, cap * 4, s));  // kPanelPad
    SPMV_HIP(hipMemsetAsync(P.val.p, 0, cap * vs, s));
    SPMV_HIP(hipMemsetAsync(P.chunk_base.p, 0, std::max<int64_t>(total / kSortedChunk, 1) * 4, s));
    if (P.row16) {
        P.rows16.alloc(cap * 2);
        SPMV_HIP(hipMemsetAsync(P.rows16.p, 0, cap * 2, s));
    }
    if (nnz > 0) {
        if (h->dt == SPMV_F64)
            tiles_scatter<double><<<grid_of_n(nnz), kB, 0, s>>>(
                keys.as<uint64_t>(), perm.as<uint32_t>(), nnz, key_bits, h->row.as<int32_t>(),
                h->val.as<double>(), first.as<int32_t>(), start.as<int32_t>(),
                P.blk_row.as<int32_t>(), T == 4 ? 2 : 1, P.delta, P.col_bits, P.idx.as<int32_t>(),
                P.rows16.as<uint16_t>(), P.chunk_base.as<int32_t>(), P.val.as<double>());
        else
            tiles_scatter<float><<<grid_of_n(nnz), kB, 0, s>>>(
                keys.as<uint64_t>(), perm.as<uint32_t>(), nnz, key_bits, h->row.as<int32_t>(),
                h->val.as<float>(), first.as<int32_t>(), start.as<int32_t>(),
                P.blk_row.as<int32_t>(), T == 4 ? 2 : 1, P.delta, P.col_bits, P.idx.as<int32_t>(),
                P.rows16.as<uint16_t>(), P.chunk_base.as<int32_t>(), P.val.as<float>());
        SPMV_CHECK_LAUNCH();
    }
    P.blk_ptr = std::move(start);
    SPMV_HIP(hipStreamSynchronize(s));  // also keeps `order` alive until its copy is done
    P.built = true;
    h->sorted_tiles[T == 4] = std::move(P);
}

void sorted_tiles_spmv(const spmv_matrix_s *h, int tiles, int items, double alpha, const void *x,
                       double beta, void *y, hipStream_t s) {
    const SortedPart &P = h->sorted_tiles[tiles == 4];
    if (!P.built) fail(SPMV_ERR_NOT_CONVERTED, "column-tile layout not built");
    if (h->n_rows == 0) return;
    if (h->dt == SPMV_F64) {
        if (items == 8) launch_tiles<double, 8>(P, h->n_rows, alpha, x, beta, y, s);
        else launch_tiles<double, 16>(P, h->n_rows, alpha, x, beta, y, s);
    } else {
        if (items == 8) launch_tiles<float, 8>(P, h->n_rows, alpha, x, beta, y, s);
        else launch_tiles<float, 16>(P, h->n_rows, alpha, x, beta, y, s);
    }
}

void sorted_spmv(const spmv_matrix_s *h, int items, double alpha, const void *x, double beta,
                 void *y, hipStream_t s) {
    if (!h->sorted.built) fail(SPMV_ERR_NOT_CONVERTED, "sorted-block COO layout not built");
    if (h->n_rows == 0) return;
    const SortedPart &P = h->sorted;
    if (h->dt == SPMV_F64) {
        if (items == 4) launch_sorted<double, 4>(P, alpha, x, beta, y, s);
        else if (items == 8) launch_sorted<double, 8>(P, alpha, x, beta, y, s);
        else launch_sorted<double, 16>(P, alpha, x, beta, y, s);
    } else {
        if (items == 4) launch_sorted<float, 4>(P, alpha, x, beta, y, s);
        else if (items == 8) launch_sorted<float, 8>(P, alpha, x, beta, y, s);
        else launch_sorted<float, 16>(P, alpha, x, beta, y, s);
    }
}

void hyb_sorted_tail(const spmv_matrix_s *h, int items, double alpha, const void *x, void *y,
                     hipStream_t s) {
    if (!h->hyb_sorted.built) fail(SPMV_ERR_NOT_CONVERTED, "sorted-block copy of the HYB tail not built");
    if (h->n_rows == 0 || h->hyb.nnz_tail == 0) return;
    const SortedPart &P = h->hyb_sorted;
    if (h->dt == SPMV_F64) {
        if (items == 8) launch_sorted<double, 8, true>(P, alpha, x, 0.0, y, s);
        else launch_sorted<double, 16, true>(P, alpha, x, 0.0, y, s);
    } else {
        if (items == 8) launch_sorted<float, 8, true>(P, alpha, x, 0.0, y, s);
        else launch_sorted<float, 16, true>(P, alpha, x, 0.0, y, s);
    }
}

void build_panel(spmv_matrix_s *h, hipStream_t s) {
    if (h->panel.built) return;
    const int64_t n = h->n_rows, nnz = h->nnz;
    if (h->n_cols >= (int32_t)kColMask || nnz > (int64_t)INT32_MAX / 2)
        fail(SPMV_ERR_NOT_APPLICABLE, "streaming COO needs fewer than %u columns", kColMask);
    int cus = 0;
    SPMV_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, h->device));
    PanelPart P;
    P.rows_per_wave = (int32_t)std::min<int64_t>(
        kPanelRowsMax,
        std::max<int64_t>(1, ceil_div(n, (int64_t)kPanelWaves * kBlocksPerCu * std::max(cus, 1))));
    P.blocks = (int32_t)ceil_div(n, (int64_t)kPanelWaves * P.rows_per_wave);
    const int64_t groups = (int64_t)P.blocks * kPanelWaves;
    const int32_t panels = (int32_t)std::max<int64_t>(1, ceil_div(h->n_cols, kPanelWidth));
    const size_t vs = dtype_size(h->dt);

    DevBuf keys, perm, first, start;
    first.alloc((groups + 1) * 4);
    start.alloc((groups + 1) * 4);
    panel_groups<<<grid_of_n(groups + 1), kB, 0, s>>>(h->row_ptr.as<int32_t>(), h->n_rows, groups,
                                                      P.rows_per_wave, first.as<int32_t>(),
                                                      start.as<int32_t>());
    SPMV_CHECK_LAUNCH();
    exclusive_scan_i32(start.as<int32_t>(), start.as<int32_t>(), groups + 1, s);
    int32_t total = 0;
    SPMV_HIP(hipMemcpyAsync(&total, start.as<int32_t>() + groups, 4, hipMemcpyDeviceToHost, s));
    SPMV_HIP(hipStreamSynchronize(s));
    P.stream = total;
    const int64_t cap = padded_count(total);
    P.idx.alloc(cap * 4);
    P.val.alloc(cap * vs);
    SPMV_HIP(hipMemsetAsync(P.idx.p, 0xFF, cap * 4, s));  // kPanelPad
    SPMV_HIP(hipMemsetAsync(P.val.p, 0, cap * vs, s));
    if (nnz > 0) {
        keys.alloc(nnz * 8);
        perm.alloc(nnz * 4);
        panel_keys<<<grid_of_n(nnz), kB, 0, s>>>(h->row.as<int32_t>(), h->col.as<int32_t>(), nnz,
                                                 P.rows_per_wave, panels, keys.as<uint64_t>(),
                                                 perm.as<uint32_t>());
        SPMV_CHECK_LAUNCH();
        const uint64_t n_keys = (uint64_t)groups * (uint64_t)panels;
        int bits = 0;
        while (bits < 64 && (n_keys - 1) >> bits) ++bits;
        radix_sort_pairs(keys, perm, nnz, bits, s);
        if (h->dt == SPMV_F64)
            panel_scatter<double><<<grid_of_n(nnz), kB, 0, s>>>(
                perm.as<uint32_t>(), nnz, h->row.as<int32_t>(), h->col.as<int32_t>(),
                h->val.as<double>(), first.as<int32_t>(), start.as<int32_t>(), P.rows_per_wave,
                P.idx.as<int32_t>(), P.val.as<double>());
        else
            panel_scatter<float><<<grid_of_n(nnz), kB, 0, s>>>(
                perm.as<uint32_t>(), nnz, h->row.as<int32_t>(), h->col.as<int32_t>(),
                h->val.as<float>(), first.as<int32_t>(), start.as<int32_t>(), P.rows_per_wave,
                P.idx.as<int32_t>(), P.val.as<float>());
        SPMV_CHECK_LAUNCH();
    }
    P.group_ptr = std::move(start);
    SPMV_HIP(hipStreamSynchronize(s));
    P.built = true;
    h->panel = std::move(P);
}

void panel_spmv(const spmv_matrix_s *h, int items, double alpha, const void *x, double beta,
                void *y, hipStream_t s) {
    if (!h->panel.built) fail(SPMV_ERR_NOT_CONVERTED, "streaming COO layout not built");
    if (h->n_rows == 0) return;
    if (h->dt == SPMV_F64) {
        if (items == 4) launch_panel<double, 4>(h, alpha, x, beta, y, s);
        else launch_panel<double, 8>(h, alpha, x, beta, y, s);
    } else {
        if (items == 4) launch_panel<float, 4>(h, alpha, x, beta, y, s);
        else launch_panel<float, 8>(h, alpha, x, beta, y, s);
    }
}

}  // namespace spmv
