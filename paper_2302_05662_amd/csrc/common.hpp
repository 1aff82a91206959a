// Internal runtime of the SpMV library: handle layout, error plumbing and
// small device helpers shared by the translation units. Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <vector>

#include <cstdint>
#include <cstdio>
#include <string>

#include "spmv.h"

namespace spmv {

// ---- errors -------------------------------------------------------------------

void set_error(const char *fmt, ...);
void clear_error();

struct Error {
    spmv_status status;
};

[[noreturn]] void fail(spmv_status s, const char *fmt, ...);

#define SPMV_HIP(call)                                                                     \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess)                                                              \
            ::spmv::fail(e_ == hipErrorOutOfMemory ? SPMV_ERR_OOM : SPMV_ERR_HIP,          \
                         "%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), __FILE__,  \
                         __LINE__);                                                        \
    } while (0)

#define SPMV_CHECK_LAUNCH() SPMV_HIP(hipGetLastError())

// Run `body` and turn thrown spmv::Error into a status.
template <class F>
spmv_status guard(F &&body) {
    try {
        clear_error();
        body();
        return SPMV_OK;
    } catch (const Error &e) {
        return e.status;
    } catch (...) {
        set_error("unexpected C++ exception");
        return SPMV_ERR_HIP;
    }
}

// ---- device memory ------------------------------------------------------------

// Owning device buffer (hipMalloc / hipFree).
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    DevBuf(DevBuf &&o) noexcept : p(o.p), bytes(o.bytes) { o.p = nullptr; o.bytes = 0; }
    DevBuf &operator=(DevBuf &&o) noexcept {
        if (this != &o) { release(); p = o.p; bytes = o.bytes; o.p = nullptr; o.bytes = 0; }
        return *this;
    }
    ~DevBuf() { release(); }
    void alloc(size_t n) {
        release();
        if (n == 0) return;
        hipError_t e = hipMalloc(&p, n);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            p = nullptr;
            fail(SPMV_ERR_OOM, "hipMalloc(%zu bytes) failed: %s", n, hipGetErrorString(e));
        }
        bytes = n;
    }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    template <class T> T *as() const { return static_cast<T *>(p); }
};

inline size_t dtype_size(spmv_dtype dt) { return dt == SPMV_F64 ? 8 : 4; }

// Streamed index/value arrays are allocated with at least one whole group of
// 16 entries past the last one (a multiple of 16, never empty), so a kernel may
// issue an aligned 16-byte load at any 4-aligned position <= nnz. The padding
// is zero-filled and never contributes to a result.
constexpr int64_t kArrayPad = 16;
inline int64_t padded_count(int64_t n) { return (n / kArrayPad + 1) * kArrayPad; }

// ---- the matrix handle ----------------------------------------------------------

struct EllPart {
    bool built = false;
    int32_t K = 0, pitch = 0;
    DevBuf col, val;
};

struct HybPart {
    bool built = false;
    int32_t K = 0, pitch = 0;
    int64_t nnz_tail = 0;
    DevBuf ell_col, ell_val, tail_row, tail_col, tail_val, partials;
    DevBuf tail_ptr;  // tail_ptr[r]: tail entries of the rows before r (n_rows + 1)
};

// Column-panel ordered copy of the COO entries for the streaming COO kernel.
// Rows are split into groups of `rows_per_wave` consecutive rows, one group per
// wavefront; a group's entries are stored contiguously, ordered by column panel
// (kPanelWidth columns), then row, then column, and the group's stream is padded
// to a multiple of 4 entries with index kPanelPad and value 0. An index packs
// the row inside its group (high 9 bits) and the global column (low 23 bits).
// group_ptr[g] .. group_ptr[g + 1] is group g's stream.
constexpr int kPanelWaves = 8;        // wavefronts (row groups) per workgroup
constexpr int kPanelRowsMax = 512;    // rows per group at most (LDS accumulators)
constexpr int kPanelColBits = 23;     // columns below 2^23 - 1
constexpr int32_t kPanelWidth = 16384;
constexpr int32_t kPanelPad = -1;

struct PanelPart {
    bool built = false;
    int32_t rows_per_wave = 0, blocks = 0;
    int64_t stream = 0;  // padded entries
    DevBuf idx, val, group_ptr;
};

// Column-sorted copy of the COO entries for the sorted-block COO kernel: rows
// are cut into blocks of consecutive rows, block b = rows [blk_row[b],
// blk_row[b + 1]) (one workgroup each, at most `rows` rows); a block's entries
// are stored sorted by column (then row) in whole 256-entry chunks, each
// transposed (see sorted_block_sum), padding with index kPanelPad and value 0.
// An index packs the row inside the block above the column, (row - first row)
// << col_bits | col with col_bits the bit length of n_cols, when the tallest
// block fits the bits left; otherwise (row16) the index is the column and the
// row inside the block is a uint16 in rows16. blk_ptr[b] .. blk_ptr[b + 1] is
// block b's stream; workgroup i takes block blk_order[i] (largest first).
constexpr int kSortedWaves = 16;       // wavefronts per workgroup
constexpr int kSortedRowsMax = 16384;  // rows per block at most (FP64 LDS accumulators)

//
// Column tiles (tiles = T, 2 or 4): each block's entries are split into T tiles
// by column range (width ceil(n_cols / T)), tile T b + h holding block b's
// entries of range h, each its own stream of whole chunks (blk_ptr and
// blk_order count tiles). Blocks are T times as tall as with one tile per block
// for the same number of workgroups, so each workgroup gathers from 1/T of x
// with T times the entries per line. A tile's index packs the row inside the
// block above the column less the first column of its chunk (delta;
// chunk_base[chunk]) when every chunk's column span fits the bits left, else
// (row16) the index is the column. Tile T b writes y = alpha * s + beta * y for
// its rows, tile T b + h (h > 0) writes alpha * s to partial[(h - 1) * pitch +
// row], and a second kernel adds the T - 1 partial rows to y.
struct SortedPart {
    bool built = false;
    bool row16 = false;
    bool delta = false;
    int32_t rows = 0;  // tallest block
    int32_t blocks = 0, col_bits = 0;
    int32_t tiles = 1;  // per block
    int64_t stream = 0, pitch = 0;  // pitch: rows per partial array
    std::vector<int32_t> row_start;  // host copy of blk_row
    DevBuf idx, val, blk_ptr, blk_row, blk_order, rows16, chunk_base, partial;
};

// Column-split copy of the COO entries: entries ordered by column panel (2 MB
// of x per panel), then row, then column; panel p's entries start at start[p]
// (a multiple of 4) and number count[p]. Three arrays like canonical COO.
struct SplitPart {
    bool built = false;
    int32_t panels = 0, width = 0;
    std::vector<int64_t> start, count;
    DevBuf row, col, val;
};
inline int32_t split_width(spmv_dtype dt) { return dt == SPMV_F64 ? (1 << 18) : (1 << 19); }

// SELL-C-sigma: slices of kSellSlice rows; slice s holds slots [slice_ptr[s],
// slice_ptr[s + 1]), its width (slots per row) a multiple of kSellGroup; slot k
// of the row at position l sits at slice_ptr[s] + (k / 4) * 256 + l * 4 + k % 4.
// perm[p] is the row at position p (only when sigma > 1).
constexpr int kSellSlice = 64;
constexpr int kSellGroup = 4;
constexpr int32_t kSellSigmaWide = 16384;
constexpr int64_t kSmallLayoutSlots = 65536;  // SELL / BELL layouts never refused

struct SellPart {
    bool built = false;
    int32_t sigma = 1, n_slices = 0;
    int64_t slots = 0;
    std::vector<int64_t> host_ptr;  // slice pointers (host copy)
    DevBuf slice_ptr, perm, col, val;
};

// BELL: b x b blocks, ELL over block rows: bcol[k * pitch + i] the block column
// (-1 padding), bval[(k * pitch + i) * b * b + r * b + c].
struct BellPart {
    bool built = false;
    int32_t b = 2, K = 0, pitch = 0, n_block_rows = 0;
    DevBuf col, val;
};

// Row-length statistics kept from ingest (used by defaults and features).
struct RowStats {
    int32_t max_len = 0;
};

}  // namespace spmv

namespace spmv {
// Row blocks of the CSR stream kernel: block b = rows [rows[b], rows[b + 1]),
// at most kCsrStreamRows rows whose entries, counted from the 4-aligned entry
// below the block's first, fit kCsrStreamCap; a row too long for that is a
// block of its own.
constexpr int kCsrStreamCap = 2048;
constexpr int kCsrStreamRows = 256;
struct CsrBlocks {
    bool built = false;
    int32_t blocks = 0;
    DevBuf rows;
};
}  // namespace spmv

struct spmv_matrix_s {
    int device = 0;
    int32_t n_rows = 0, n_cols = 0;
    int64_t nnz = 0;
    spmv_dtype dt = SPMV_F32;
    // canonical COO / CSR: row[nnz], col[nnz], val[nnz] sorted by (row, col);
    // row_ptr[n_rows + 1].
    spmv::DevBuf row, col, val, row_ptr;
    spmv::DevBuf coo_partials;  // per-tile carries of the COO kernel
    spmv::EllPart ell;
    spmv::HybPart hyb;
    spmv::PanelPart panel;    // built on first use of a streaming COO variant
    spmv::SortedPart sorted;  // built on first use of a sorted-block COO variant
    spmv::SortedPart hyb_sorted;  // the HYB tail's, built on first use of a sorted-tail HYB variant
    spmv::SortedPart sorted_tiles[2];  // column-tile copies ([0]: 2 tiles, [1]: 4), built on first use
    spmv::SplitPart split;    // built on first use of a column-split COO variant
    spmv::CsrBlocks csr_blocks;  // built on first use of a CSR stream variant
    spmv::SellPart sell;
    spmv::BellPart bell;
    spmv::RowStats stats;
    int32_t variant[SPMV_NUM_FORMATS] = {};
};

namespace spmv {

// ---- shared host-side helpers implemented in the .hip files ---------------------

// ingest.hip
void exclusive_scan_i32(const int32_t *in, int32_t *out, int64_t n, hipStream_t s);
// The same scan with caller-provided tile sums (at most min(sums_cap, 2048) of
// them, so n <= 2048 * 2048); allocates nothing and does not synchronise.
void exclusive_scan_i32_ws(const int32_t *in, int32_t *out, int64_t n, int32_t *sums,
                           int64_t sums_cap, hipStream_t s);
// Stable LSD radix sort of n 64-bit keys (the low `bits` bits) carrying a
// 32-bit payload; on return `keys` and `payload` hold the sorted pairs.
void radix_sort_pairs(DevBuf &keys, DevBuf &payload, int64_t n, int bits, hipStream_t s);
int32_t device_max_row_len(const int32_t *row_ptr, int32_t n_rows, hipStream_t s);

// convert.hip
void build_ell(spmv_matrix_s *h, hipStream_t s);
void build_hyb(spmv_matrix_s *h, int32_t hyb_k, hipStream_t s);
void build_sell(spmv_matrix_s *h, int32_t sigma, hipStream_t s);  // sigma < 0: rule
void build_bell(spmv_matrix_s *h, int32_t b, hipStream_t s);      // b < 0: rule
int32_t hyb_rule_width(spmv_matrix_s *h, hipStream_t s);

// panel.hip
void build_panel(spmv_matrix_s *h, hipStream_t s);  // NOT_APPLICABLE past the index limits
void panel_spmv(const spmv_matrix_s *h, int items, double alpha, const void *x, double beta,
                void *y, hipStream_t s);
void build_sorted(spmv_matrix_s *h, hipStream_t s);
// Tallest sorted block the packing allows for this matrix (NOT_APPLICABLE if none).
int32_t sorted_max_rows(const spmv_matrix_s *h);
// Rows per block that the packed index can hold (0: none); taller blocks use rows16.
int32_t sorted_packed_rows(const spmv_matrix_s *h);
// Block boundaries 0 = r_0 < r_1 < ... < r_B = n_rows with at most max_rows rows
// per block: cut at equal shares of the entries, in as few whole rounds of one
// block per CU as the height limit allows.
std::vector<int32_t> sorted_balanced_rows(const std::vector<int32_t> &row_ptr, int32_t max_rows,
                                          int cus);
// Entries a sorted-block copy is built from: the matrix's own (canonical COO and
// row pointers) or its HYB tail, row-sorted, with row pointers over all rows.
struct SortedEntries {
    int64_t nnz;
    const int32_t *row, *col, *row_ptr;
    const void *val;
};
SortedEntries matrix_entries(const spmv_matrix_s *h);
// Build a sorted-block copy of `src` (rows and columns of h) with the given block
// boundaries into P; row_ptr is a host copy of src's row pointers.
void build_sorted_into(const spmv_matrix_s *h, const SortedEntries &src,
                       const std::vector<int32_t> &row_ptr, const std::vector<int32_t> &row_start,
                       SortedPart &P, hipStream_t s);
// Sorted-block copy of the HYB tail (h->hyb_sorted), for the HYB variants that
// add the tail with the sorted-block kernel.
void build_hyb_sorted(spmv_matrix_s *h, hipStream_t s);
void hyb_sorted_tail(const spmv_matrix_s *h, int items, double alpha, const void *x, void *y,
                     hipStream_t s);
void build_split(spmv_matrix_s *h, hipStream_t s);  // NOT_APPLICABLE below two panels
void sorted_spmv(const spmv_matrix_s *h, int items, double alpha, const void *x, double beta,
                 void *y, hipStream_t s);
// Column-tile copy of the entries in `tiles` (2 or 4) tiles per block
// (h->sorted_tiles[tiles == 4]) and its SpMV (two launches). Four tiles are
// NOT_APPLICABLE where the blocks would need more than one round of workgroups.
void build_sorted_tiles(spmv_matrix_s *h, int tiles, hipStream_t s);
void sorted_tiles_spmv(const spmv_matrix_s *h, int tiles, int items, double alpha, const void *x,
                       double beta, void *y, hipStream_t s);

// kernels.hip
int32_t variant_count(spmv_format f, spmv_dtype dt);
bool variant_describe(spmv_format f, spmv_dtype dt, int32_t idx, spmv_variant_info *out);
int32_t default_variant(const spmv_matrix_s *h, spmv_format f);
// False when variant idx cannot run on the layout f holds now (BELL: more rows
// per thread than the block has).
bool variant_applicable(const spmv_matrix_s *h, spmv_format f, int32_t idx);
int64_t stored_bytes(const spmv_matrix_s *h, spmv_format f, int32_t idx);  // -1: not built
bool variant_needs_panel(spmv_format f, int32_t idx);
bool variant_needs_sorted(spmv_format f, int32_t idx);
int variant_sorted_tiles(spmv_format f, int32_t idx);  // column tiles the variant needs, 0: none
bool variant_needs_hyb_sorted(spmv_format f, int32_t idx);
bool variant_needs_split(spmv_format f, int32_t idx);
bool variant_needs_csr_blocks(spmv_format f, int32_t idx);
void build_csr_blocks(spmv_matrix_s *h, hipStream_t s);
// Make variant idx of f runnable: builds the reordered copy or block table the
// variant reads (streaming, sorted-block or column-split COO copy, CSR stream
// row blocks, sorted copy of the HYB tail) unless it is built. Returns false when
// that layout is not applicable to the matrix.
bool prepare_variant(spmv_matrix_s *h, spmv_format f, int32_t idx, hipStream_t s);
void launch_spmv(const spmv_matrix_s *h, spmv_format f, int32_t variant, double alpha,
                 const void *x, double beta, void *y, hipStream_t s);
int64_t coo_partials_bytes(int64_t nnz, spmv_dtype dt);

// features.hip
void compute_features(spmv_matrix_s *h, float out[12], int32_t *hyb_width, hipStream_t s);
// The same features with every temporary in a file-scope device array (no
// allocation); rows longer than SPMV_FEATURES_NOALLOC_MAX_LEN are refused.
void compute_features_noalloc(spmv_matrix_s *h, float out[12], hipStream_t s);

// timing.hip
void flush_caches(hipStream_t s);

// ---- device helpers -------------------------------------------------------------

constexpr int kWave = 64;
constexpr int kNumXcd = 8;

// Workgroups are dealt to the 8 XCDs round-robin (block b runs on XCD b % 8).
// This bijection gives each XCD one contiguous range of logical blocks, so
// neighbouring tiles (which share x entries for banded and stencil matrices)
// hit the same L2.
__device__ __forceinline__ int xcd_logical_block(int b, int nb) {
    int q = nb / kNumXcd, r = nb % kNumXcd;
    int x = b % kNumXcd, i = b / kNumXcd;
    return x * q + (x < r ? x : r) + i;
}

template <class T>
__device__ __forceinline__ T ld_stream(const T *p) {
    return __builtin_nontemporal_load(p);
}

constexpr int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

}  // namespace spmv
