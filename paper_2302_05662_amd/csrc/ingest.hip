// COO ingest on the device: bounds check, ordering check, stable LSD radix
// sort by (row, col), duplicate detection and CSR row pointers.
//
// Matrices arrive as COO (paper, Results: run-time prediction overhead notes
// that SuiteSparse stores them so); CSR is the paper's default format
// (Background: popular SpMV formats, CSR). Sorting by (row, col) makes COO and
// CSR share their column and value arrays.
#include <algorithm>
#include <cstring>
#include <vector>

#include "common.hpp"

namespace spmv {
namespace {

constexpr int kBlock = 256;
constexpr int kItems = 8;
constexpr int kTile = kBlock * kItems;  // 2048 elements per workgroup

enum : int { kFlagOutOfBounds = 1, kFlagNotCanonical = 2, kFlagDuplicate = 4 };

// ---- block-wide exclusive scan of one int per thread ---------------------------

__device__ int block_exclusive_scan(int v, int *total) {
    __shared__ int wave_sum[kBlock / kWave];
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    int x = v;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        int y = __shfl_up(x, d, kWave);
        if (lane >= d) x += y;
    }
    if (lane == kWave - 1) wave_sum[wave] = x;
    __syncthreads();
    int off = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kBlock / kWave; ++w) {
        int s = wave_sum[w];
        off += (w < wave) ? s : 0;
        tot += s;
    }
    __syncthreads();
    *total = tot;
    return off + x - v;
}

__global__ __launch_bounds__(kBlock) void scan_tile_sums(const int32_t *__restrict__ in, int64_t n,
                                                         int32_t *__restrict__ sums) {
    const int64_t base = (int64_t)blockIdx.x * kTile + (int64_t)threadIdx.x * kItems;
    int s = 0;
#pragma unroll
    for (int i = 0; i < kItems; ++i)
        if (base + i < n) s += in[base + i];
    int tot;
    block_exclusive_scan(s, &tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// out[k] = tile_offset + exclusive prefix within the tile. In-place is allowed.
__global__ __launch_bounds__(kBlock) void scan_tiles(const int32_t *in, int64_t n, int32_t *out,
                                                     const int32_t *__restrict__ tile_offset) {
    const int64_t base = (int64_t)blockIdx.x * kTile + (int64_t)threadIdx.x * kItems;
    int v[kItems];
    int s = 0;
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
        v[i] = (base + i < n) ? in[base + i] : 0;
        s += v[i];
    }
    int tot;
    int run = block_exclusive_scan(s, &tot) + (tile_offset ? tile_offset[blockIdx.x] : 0);
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
        if (base + i < n) out[base + i] = run;
        run += v[i];
    }
}

// ---- checks --------------------------------------------------------------------

__global__ __launch_bounds__(kBlock) void check_coo(const int32_t *__restrict__ row,
                                                    const int32_t *__restrict__ col, int64_t nnz,
                                                    int32_t n_rows, int32_t n_cols,
                                                    int32_t *__restrict__ flags) {
    int f = 0;
    for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < nnz;
         k += (int64_t)gridDim.x * kBlock) {
        int32_t r = row[k], c = col[k];
        if (r < 0 || r >= n_rows || c < 0 || c >= n_cols) f |= kFlagOutOfBounds;
        if (k > 0) {
            int32_t pr = row[k - 1], pc = col[k - 1];
            if (!(pr < r || (pr == r && pc < c))) f |= kFlagNotCanonical;
        }
    }
    if (f) atomicOr(flags, f);
}

__global__ __launch_bounds__(kBlock) void check_duplicates(const int32_t *__restrict__ row,
                                                           const int32_t *__restrict__ col,
                                                           int64_t nnz, int32_t *__restrict__ flags) {
    int f = 0;
    for (int64_t k = 1 + (int64_t)blockIdx.x * kBlock + threadIdx.x; k < nnz;
         k += (int64_t)gridDim.x * kBlock)
        if (row[k] == row[k - 1] && col[k] == col[k - 1]) f = kFlagDuplicate;
    if (f) atomicOr(flags, f);
}

// ---- LSD radix sort of 64-bit keys with a 32-bit payload -----------------------

__global__ __launch_bounds__(kBlock) void make_keys(const int32_t *__restrict__ row,
                                                    const int32_t *__restrict__ col, int64_t nnz,
                                                    int64_t n_cols, uint64_t *__restrict__ key,
                                                    uint32_t *__restrict__ idx) {
    for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < nnz;
         k += (int64_t)gridDim.x * kBlock) {
        key[k] = (uint64_t)row[k] * (uint64_t)n_cols + (uint64_t)col[k];
        idx[k] = (uint32_t)k;
    }
}

// Digit histogram of one tile, stored digit-major: hist[d * n_tiles + tile].
// An exclusive scan of that array gives every (digit, tile) its output start.
__global__ __launch_bounds__(kBlock) void radix_hist(const uint64_t *__restrict__ key, int64_t n,
                                                     int shift, int32_t *__restrict__ hist,
                                                     int n_tiles) {
    __shared__ int cnt[256];
    cnt[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kTile;
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
        int64_t k = base + (int64_t)i * kBlock + threadIdx.x;
        if (k < n) atomicAdd(&cnt[(key[k] >> shift) & 255u], 1);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * n_tiles + blockIdx.x] = cnt[threadIdx.x];
}

// Stable scatter of one tile. Element k of the tile sits in "row" i = k / 256,
// lane k % 256, so processing rows in order and waves in order keeps the
// input order among equal digits. Inside a wave, lanes with the same digit
// are found with eight ballots (one per digit bit).
__global__ __launch_bounds__(kBlock) void radix_scatter(
    const uint64_t *__restrict__ key_in, const uint32_t *__restrict__ idx_in,
    uint64_t *__restrict__ key_out, uint32_t *__restrict__ idx_out, int64_t n, int shift,
    const int32_t *__restrict__ offsets, int n_tiles) {
    constexpr int kWaves = kBlock / kWave;
    __shared__ int s_next[256];
    __shared__ int s_wave[kWaves][256];
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (kWave - lane));
    s_next[threadIdx.x] = offsets[(int64_t)threadIdx.x * n_tiles + blockIdx.x];
    const int64_t base = (int64_t)blockIdx.x * kTile;
    for (int i = 0; i < kItems; ++i) {
        const int64_t k = base + (int64_t)i * kBlock + threadIdx.x;
        const bool valid = k < n;
        uint64_t kv = valid ? key_in[k] : 0;
        uint32_t iv = valid ? idx_in[k] : 0;
        const int d = (int)((kv >> shift) & 255u);
#pragma unroll
        for (int w = 0; w < kWaves; ++w) s_wave[w][threadIdx.x] = 0;
        __syncthreads();
        uint64_t same = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1;
            const uint64_t m = __ballot(bit);
            same &= bit ? m : ~m;
        }
        const int rank = __popcll(same & lt_mask);
        if (valid && rank == 0) s_wave[wave][d] = __popcll(same);
        __syncthreads();
        {  // thread t owns digit t: hand out consecutive ranges wave by wave
            int run = s_next[threadIdx.x];
#pragma unroll
            for (int w = 0; w < kWaves; ++w) {
                int c = s_wave[w][threadIdx.x];
                s_wave[w][threadIdx.x] = run;
                run += c;
            }
            s_next[threadIdx.x] = run;
        }
        __syncthreads();
        if (valid) {
            const int pos = s_wave[wave][d] + rank;
            key_out[pos] = kv;
            idx_out[pos] = iv;
        }
        __syncthreads();
    }
}

template <class V>
__global__ __launch_bounds__(kBlock) void gather_entries(
    const uint32_t *__restrict__ perm, const int32_t *__restrict__ row_in,
    const int32_t *__restrict__ col_in, const V *__restrict__ val_in, int64_t nnz,
    int32_t *__restrict__ row_out, int32_t *__restrict__ col_out, V *__restrict__ val_out) {
    for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < nnz;
         k += (int64_t)gridDim.x * kBlock) {
        const uint32_t p = perm[k];
        row_out[k] = row_in[p];
        col_out[k] = col_in[p];
        val_out[k] = val_in[p];
    }
}

// row_ptr[r] = first position whose row is >= r (binary search on sorted rows).
__global__ __launch_bounds__(kBlock) void row_ptr_from_sorted(const int32_t *__restrict__ row,
                                                              int64_t nnz, int32_t n_rows,
                                                              int32_t *__restrict__ row_ptr) {
    for (int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x; r <= n_rows;
         r += (int64_t)gridDim.x * kBlock) {
        int64_t lo = 0, hi = nnz;
        while (lo < hi) {
            int64_t mid = (lo + hi) >> 1;
            if (row[mid] < r) lo = mid + 1; else hi = mid;
        }
        row_ptr[r] = (int32_t)lo;
    }
}

__global__ __launch_bounds__(kBlock) void max_row_len_kernel(const int32_t *__restrict__ row_ptr,
                                                             int32_t n_rows,
                                                             int32_t *__restrict__ out) {
    int m = 0;
    for (int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x; r < n_rows;
         r += (int64_t)gridDim.x * kBlock)
        m = max(m, row_ptr[r + 1] - row_ptr[r]);
    for (int d = kWave / 2; d > 0; d >>= 1) m = max(m, __shfl_xor(m, d, kWave));
    if ((threadIdx.x & (kWave - 1)) == 0 && m > 0) atomicMax(out, m);
}

int grid_for(int64_t n, int per_block = kBlock, int cap = 65536) {
    int64_t g = ceil_div(std::max<int64_t>(n, 1), per_block);
    return (int)std::min<int64_t>(g, cap);
}

int read_flags(const DevBuf &flags, hipStream_t s) {
    int32_t f = 0;
    SPMV_HIP(hipMemcpyAsync(&f, flags.p, sizeof(f), hipMemcpyDeviceToHost, s));
    SPMV_HIP(hipStreamSynchronize(s));
    return f;
}

// Sort (row, col, val) of `nnz` entries in [src] into the handle's arrays.
void sort_into_handle(spmv_matrix_s *h, const int32_t *row, const int32_t *col, const void *val,
                      hipStream_t s) {
    const int64_t nnz = h->nnz;
    const uint64_t span = (uint64_t)std::max(h->n_rows, 1) * (uint64_t)std::max(h->n_cols, 1);
    int bits = 0;
    while (bits < 64 && (span - 1) >> bits) ++bits;
    DevBuf keys, perm;
    keys.alloc(nnz * 8);
    perm.alloc(nnz * 4);
    make_keys<<<grid_for(nnz), kBlock, 0, s>>>(row, col, nnz, h->n_cols, keys.as<uint64_t>(),
                                               perm.as<uint32_t>());
    SPMV_CHECK_LAUNCH();
    radix_sort_pairs(keys, perm, nnz, bits, s);
    if (h->dt == SPMV_F64)
        gather_entries<double><<<grid_for(nnz), kBlock, 0, s>>>(
            perm.as<uint32_t>(), row, col, (const double *)val, nnz, h->row.as<int32_t>(),
            h->col.as<int32_t>(), h->val.as<double>());
    else
        gather_entries<float><<<grid_for(nnz), kBlock, 0, s>>>(
            perm.as<uint32_t>(), row, col, (const float *)val, nnz, h->row.as<int32_t>(),
            h->col.as<int32_t>(), h->val.as<float>());
    SPMV_CHECK_LAUNCH();
    SPMV_HIP(hipStreamSynchronize(s));
}

}  // namespace

// ---- shared helpers ------------------------------------------------------------

void radix_sort_pairs(DevBuf &keys, DevBuf &payload, int64_t n, int bits, hipStream_t s) {
    const int passes = (bits + 7) / 8;
    if (n <= 1 || passes == 0) return;
    DevBuf k1, p1, hist;
    k1.alloc(n * 8);
    p1.alloc(n * 4);
    const int n_tiles = (int)ceil_div(n, kTile);
    hist.alloc((int64_t)256 * n_tiles * 4);
    for (int p = 0; p < passes; ++p) {
        radix_hist<<<n_tiles, kBlock, 0, s>>>(keys.as<uint64_t>(), n, 8 * p, hist.as<int32_t>(),
                                              n_tiles);
        SPMV_CHECK_LAUNCH();
        exclusive_scan_i32(hist.as<int32_t>(), hist.as<int32_t>(), (int64_t)256 * n_tiles, s);
        radix_scatter<<<n_tiles, kBlock, 0, s>>>(keys.as<uint64_t>(), payload.as<uint32_t>(),
                                                 k1.as<uint64_t>(), p1.as<uint32_t>(), n, 8 * p,
                                                 hist.as<int32_t>(), n_tiles);
        SPMV_CHECK_LAUNCH();
        std::swap(keys, k1);
        std::swap(payload, p1);
    }
    SPMV_HIP(hipStreamSynchronize(s));  // the temporaries are freed on return
}

void exclusive_scan_i32(const int32_t *in, int32_t *out, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    const int64_t tiles = ceil_div(n, kTile);
    if (tiles == 1) {
        scan_tiles<<<1, kBlock, 0, s>>>(in, n, out, nullptr);
        SPMV_CHECK_LAUNCH();
        return;
    }
    if (tiles > INT32_MAX) fail(SPMV_ERR_INVALID_ARG, "scan too large");
    DevBuf sums;
    sums.alloc(tiles * 4);
    scan_tile_sums<<<(int)tiles, kBlock, 0, s>>>(in, n, sums.as<int32_t>());
    SPMV_CHECK_LAUNCH();
    exclusive_scan_i32(sums.as<int32_t>(), sums.as<int32_t>(), tiles, s);
    scan_tiles<<<(int)tiles, kBlock, 0, s>>>(in, n, out, sums.as<int32_t>());
    SPMV_CHECK_LAUNCH();
    SPMV_HIP(hipStreamSynchronize(s));  // `sums` is freed on return
}

void exclusive_scan_i32_ws(const int32_t *in, int32_t *out, int64_t n, int32_t *sums,
                           int64_t sums_cap, hipStream_t s) {
    if (n <= 0) return;
    const int64_t tiles = ceil_div(n, kTile);
    if (tiles == 1) {
        scan_tiles<<<1, kBlock, 0, s>>>(in, n, out, nullptr);
        SPMV_CHECK_LAUNCH();
        return;
    }
    if (tiles > kTile || tiles > sums_cap)
        fail(SPMV_ERR_INVALID_ARG, "scan of %lld elements needs %lld tile sums, workspace holds %lld",
             (long long)n, (long long)tiles, (long long)std::min<int64_t>(sums_cap, kTile));
    scan_tile_sums<<<(int)tiles, kBlock, 0, s>>>(in, n, sums);
    SPMV_CHECK_LAUNCH();
    scan_tiles<<<1, kBlock, 0, s>>>(sums, tiles, sums, nullptr);  // one tile: in place
    SPMV_CHECK_LAUNCH();
    scan_tiles<<<(int)tiles, kBlock, 0, s>>>(in, n, out, sums);
    SPMV_CHECK_LAUNCH();
}

int32_t device_max_row_len(const int32_t *row_ptr, int32_t n_rows, hipStream_t s) {
    if (n_rows <= 0) return 0;
    DevBuf out;
    out.alloc(4);
    SPMV_HIP(hipMemsetAsync(out.p, 0, 4, s));
    max_row_len_kernel<<<grid_for(n_rows, kBlock, 4096), kBlock, 0, s>>>(row_ptr, n_rows,
                                                                         out.as<int32_t>());
    SPMV_CHECK_LAUNCH();
    int32_t m = 0;
    SPMV_HIP(hipMemcpyAsync(&m, out.p, 4, hipMemcpyDeviceToHost, s));
    SPMV_HIP(hipStreamSynchronize(s));
    return m;
}

}  // namespace spmv

using namespace spmv;

extern "C" spmv_status spmv_create(spmv_handle *out, int32_t n_rows, int32_t n_cols, int64_t nnz,
                                   const int32_t *row, const int32_t *col, const void *val,
                                   spmv_dtype dt, int on_device, void *stream) {
    if (out) *out = nullptr;
    spmv_matrix_s *h = nullptr;
    spmv_status st = guard([&] {
        if (!out) fail(SPMV_ERR_INVALID_ARG, "out is NULL");
        if (n_rows < 0 || n_cols < 0 || nnz < 0 || nnz > INT32_MAX)
            fail(SPMV_ERR_INVALID_ARG, "bad sizes n_rows=%d n_cols=%d nnz=%lld", n_rows, n_cols,
                 (long long)nnz);
        if (dt != SPMV_F32 && dt != SPMV_F64) fail(SPMV_ERR_INVALID_ARG, "bad dtype %d", (int)dt);
        if (nnz > 0 && (!row || !col || !val)) fail(SPMV_ERR_INVALID_ARG, "NULL input array");
        if (nnz > 0 && ((int64_t)n_rows == 0 || (int64_t)n_cols == 0))
            fail(SPMV_ERR_OUT_OF_BOUNDS, "entries given for an empty matrix");
        hipStream_t s = (hipStream_t)stream;
        h = new spmv_matrix_s();
        SPMV_HIP(hipGetDevice(&h->device));
        h->n_rows = n_rows;
        h->n_cols = n_cols;
        h->nnz = nnz;
        h->dt = dt;
        const size_t vs = dtype_size(dt);
        const int64_t np = padded_count(nnz);
        h->row.alloc(np * 4);
        h->col.alloc(np * 4);
        h->val.alloc(np * vs);
        h->row_ptr.alloc(((int64_t)n_rows + 1) * 4);
        for (DevBuf *b : {&h->row, &h->col})  // padding past the last entry reads as 0
            SPMV_HIP(hipMemsetAsync(b->as<int32_t>() + nnz, 0, (np - nnz) * 4, s));
        SPMV_HIP(hipMemsetAsync((char *)h->val.p + nnz * vs, 0, (np - nnz) * vs, s));
        if (nnz > 0) {
            // Stage the input on the device.
            DevBuf in_row, in_col, in_val, flags;
            in_row.alloc(np * 4);
            in_col.alloc(np * 4);
            in_val.alloc(np * vs);
            flags.alloc(4);
            hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
            SPMV_HIP(hipMemcpyAsync(in_row.p, row, nnz * 4, kind, s));
            SPMV_HIP(hipMemcpyAsync(in_col.p, col, nnz * 4, kind, s));
            SPMV_HIP(hipMemcpyAsync(in_val.p, val, nnz * vs, kind, s));
            SPMV_HIP(hipMemsetAsync(flags.p, 0, 4, s));
            // zero the padding of the staged arrays (they may become the handle's)
            for (DevBuf *b : {&in_row, &in_col})
                SPMV_HIP(hipMemsetAsync(b->as<int32_t>() + nnz, 0, (np - nnz) * 4, s));
            SPMV_HIP(hipMemsetAsync((char *)in_val.p + nnz * vs, 0, (np - nnz) * vs, s));
            check_coo<<<grid_for(nnz, kBlock, 8192), kBlock, 0, s>>>(
                in_row.as<int32_t>(), in_col.as<int32_t>(), nnz, n_rows, n_cols,
                flags.as<int32_t>());
            SPMV_CHECK_LAUNCH();
            int f = read_flags(flags, s);
            if (f & kFlagOutOfBounds) fail(SPMV_ERR_OUT_OF_BOUNDS, "COO index outside the matrix");
            if (f & kFlagNotCanonical) {
                sort_into_handle(h, in_row.as<int32_t>(), in_col.as<int32_t>(), in_val.p, s);
                check_duplicates<<<grid_for(nnz, kBlock, 8192), kBlock, 0, s>>>(
                    h->row.as<int32_t>(), h->col.as<int32_t>(), nnz, flags.as<int32_t>());
                SPMV_CHECK_LAUNCH();
                if (read_flags(flags, s) & kFlagDuplicate)
                    fail(SPMV_ERR_DUPLICATE, "repeated (row, col) entry");
            } else {
                // Already strictly increasing in (row, col): keep the staged arrays.
                std::swap(h->row, in_row);
                std::swap(h->col, in_col);
                std::swap(h->val, in_val);
            }
        }
        row_ptr_from_sorted<<<grid_for((int64_t)n_rows + 1, kBlock, 8192), kBlock, 0, s>>>(
            h->row.as<int32_t>(), nnz, n_rows, h->row_ptr.as<int32_t>());
        SPMV_CHECK_LAUNCH();
        h->stats.max_len = device_max_row_len(h->row_ptr.as<int32_t>(), n_rows, s);
        h->coo_partials.alloc(coo_partials_bytes(nnz, dt));
        for (int f = 0; f < SPMV_NUM_FORMATS; ++f) h->variant[f] = default_variant(h, (spmv_format)f);
        SPMV_HIP(hipStreamSynchronize(s));
    });
    if (st == SPMV_OK) {
        *out = h;
    } else {
        delete h;
    }
    return st;
}
