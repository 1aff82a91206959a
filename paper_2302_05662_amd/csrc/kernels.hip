// SpMV kernels, y = alpha * A * x + beta * y, for the formats of the run-time
// mode (paper, Background: popular SpMV formats; HYB after Bell and Garland).
//
// All kernels stream the matrix arrays once with non-temporal loads (so they
// do not evict x from L2 / Infinity Cache) and gather x through the caches.
// FP32 matrices accumulate in FP64: the FP32 products are exact in FP64, and
// the one rounding at the end keeps long rows (50K entries) far inside a 1e-5
// per-row error budget whatever the lane split. SpMV is memory bound, so the
// wider accumulator costs no time.
#include <algorithm>
#include <climits>
#include <vector>

#include "common.hpp"
#include "device.hpp"

namespace spmv {
namespace {

// ---- CSR scalar: one thread per row ----------------------------------------------

template <class V, int BLOCK, int UNROLL>
__global__ __launch_bounds__(BLOCK) void csr_scalar_kernel(
    int32_t n_rows, const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
    const V *__restrict__ val, const V *__restrict__ x, V alpha, V beta, V *__restrict__ y) {
    const int b = xcd_logical_block(blockIdx.x, gridDim.x);
    const int64_t i = (int64_t)b * BLOCK + threadIdx.x;
    if (i >= n_rows) return;
    const int32_t s = rp[i], e = rp[i + 1];
    double acc[UNROLL];
#pragma unroll
    for (int u = 0; u < UNROLL; ++u) acc[u] = 0.0;
    int32_t j = s;
    for (; j + UNROLL <= e; j += UNROLL) {
        int32_t c[UNROLL];
        V v[UNROLL];
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) { c[u] = ld_stream(col + j + u); v[u] = ld_stream(val + j + u); }
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) acc[u] += (double)v[u] * (double)x[c[u]];
    }
    for (; j < e; ++j) acc[0] += (double)ld_stream(val + j) * (double)x[ld_stream(col + j)];
    double sum = acc[0];
#pragma unroll
    for (int u = 1; u < UNROLL; ++u) sum += acc[u];
    store_y(y, i, sum, alpha, beta);
}

// ---- CSR vector: L lanes of a wavefront per row ------------------------------------

template <class V, int BLOCK, int L, int UNROLL>
__global__ __launch_bounds__(BLOCK) void csr_vector_kernel(
    int32_t n_rows, const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
    const V *__restrict__ val, const V *__restrict__ x, V alpha, V beta, V *__restrict__ y) {
    constexpr int RPB = BLOCK / L;  // rows per workgroup
    __shared__ int32_t s_rp[RPB + 1];
    const int b = xcd_logical_block(blockIdx.x, gridDim.x);
    const int64_t row0 = (int64_t)b * RPB;
    for (int t = threadIdx.x; t <= RPB; t += BLOCK)
        s_rp[t] = rp[std::min<int64_t>(row0 + t, n_rows)];
    __syncthreads();
    const int g = threadIdx.x / L, lane = threadIdx.x % L;
    const int32_t s = s_rp[g], e = s_rp[g + 1];
    double acc = 0.0;
    int32_t j = s + lane;
    if constexpr (UNROLL > 1) {
        for (; j + (UNROLL - 1) * L < e; j += UNROLL * L) {
            int32_t c[UNROLL];
            V v[UNROLL];
#pragma unroll
            for (int u = 0; u < UNROLL; ++u) {
                c[u] = ld_stream(col + j + u * L);
                v[u] = ld_stream(val + j + u * L);
            }
#pragma unroll
            for (int u = 0; u < UNROLL; ++u) acc += (double)v[u] * (double)x[c[u]];
        }
    }
    for (; j < e; j += L) acc += (double)ld_stream(val + j) * (double)x[ld_stream(col + j)];
    acc = group_sum<L>(acc);
    const int64_t row = row0 + g;
    if (lane == 0 && row < n_rows) store_y(y, row, acc, alpha, beta);
}

// ---- CSR vector, 16-byte loads: L lanes per row, 4 consecutive entries per lane ----
//
// A lane reads entries [j, j + 4) with one aligned 16-byte load of col and one of
// val (two for FP64), starting from the row's first entry rounded down to a
// multiple of 4; entries outside the row are masked before x is touched. The
// arrays are padded to a multiple of 16 entries, so the last load stays inside.

template <class V, int BLOCK, int L, int UNROLL>
__global__ __launch_bounds__(BLOCK) void csr_vector4_kernel(
    int32_t n_rows, const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
    const V *__restrict__ val, const V *__restrict__ x, V alpha, V beta, V *__restrict__ y) {
    constexpr int RPB = BLOCK / L;
    __shared__ int32_t s_rp[RPB + 1];
    const int b = xcd_logical_block(blockIdx.x, gridDim.x);
    const int64_t row0 = (int64_t)b * RPB;
    for (int t = threadIdx.x; t <= RPB; t += BLOCK)
        s_rp[t] = rp[std::min<int64_t>(row0 + t, n_rows)];
    __syncthreads();
    const int g = threadIdx.x / L, lane = threadIdx.x % L;
    const double acc = csr_row_dot4<V, L, UNROLL>(col, val, x, s_rp[g], s_rp[g + 1], lane);
    const int64_t row = row0 + g;
    if (lane == 0 && row < n_rows) store_y(y, row, acc, alpha, beta);
}

// ---- CSR vector, software pipelined: each lane group walks PASSES rows -------------

template <class V, int BLOCK, int L, int PASSES>
__global__ __launch_bounds__(BLOCK) void csr_pipe_kernel(
    int32_t n_rows, const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
    const V *__restrict__ val, const V *__restrict__ x, V alpha, V beta, V *__restrict__ y) {
    constexpr int RPB = BLOCK / L;
    constexpr int ROWS = RPB * PASSES;
    __shared__ int32_t s_rp[ROWS + 1];
    const int b = xcd_logical_block(blockIdx.x, gridDim.x);
    const int64_t row0 = (int64_t)b * ROWS;
    for (int t = threadIdx.x; t <= ROWS; t += BLOCK)
        s_rp[t] = rp[std::min<int64_t>(row0 + t, n_rows)];
    __syncthreads();
    csr_rows_pipelined<V, L, RPB, PASSES>(col, val, x, s_rp, threadIdx.x / L, threadIdx.x % L,
                                          row0, n_rows, y, alpha, beta);
}

// ---- CSR stream: row blocks staged through LDS ------------------------------------
//
// Workgroup b takes row block b. Its entries, from the 4-aligned entry at or
// below the block's first, are loaded 4 at a time with 16-byte loads (threads
// take consecutive groups, so a wave reads 1 KB contiguous per value array);
// each product v * x[col] is formed in FP64 and kept in LDS, and after a barrier
// thread t adds row t's products in entry order and writes y. A block holding a
// single row longer than the stage instead has every thread accumulate every
// BLOCK*4-th group and the partial sums are added in a fixed tree.

template <class V, int BLOCK>
__global__ __launch_bounds__(BLOCK) void csr_stream_kernel(const int32_t *__restrict__ blk_rows,
                                                           const int32_t *__restrict__ rp,
                                                           const int32_t *__restrict__ col,
                                                           const V *__restrict__ val,
                                                           const V *__restrict__ x, V alpha, V beta,
                                                           V *__restrict__ y) {
    constexpr int CAP = kCsrStreamCap;
    static_assert(CAP % (4 * BLOCK) == 0, "whole 16-byte groups per thread");
    __shared__ double s_p[CAP];
    __shared__ double s_w[BLOCK / kWave];
    const int b = xcd_logical_block(blockIdx.x, gridDim.x);
    const int32_t r0 = blk_rows[b], r1 = blk_rows[b + 1];
    const int64_t e0 = rp[r0], e1 = rp[r1];
    const int64_t base = e0 & ~int64_t(3);
    if (e1 - base <= CAP) {
#pragma unroll
        for (int g = 0; g < CAP / (4 * BLOCK); ++g) {
            const int64_t q = base + (int64_t)(g * BLOCK + threadIdx.x) * 4;
            if (q < e1) {
                const Pack<int32_t, 4> c = ld_i32<4>(col + q);
                const Pack<V, 4> v = ld_val<4>(val + q);
                V xv[4];
                bool ok[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) ok[j] = q + j >= e0 && q + j < e1;
                gather_x<V, 4>(x, c.v, ok, xv);
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    s_p[q - base + j] = (double)v.v[j] * (double)xv[j];
            }
        }
        __syncthreads();
        // LP lanes per row (a power of two, block-uniform): lane q of a row adds its
        // products q, q + LP, ... and the LP partial sums meet in a fixed shuffle tree
        const int32_t nr = r1 - r0;
        int lp = 1;
        while (lp < 16 && nr * lp * 2 <= BLOCK) lp *= 2;
        for (int32_t t0 = 0; t0 < nr * lp; t0 += BLOCK) {
            const int32_t t = t0 + threadIdx.x;
            const int32_t r = t / lp, q = t % lp;
            double s = 0.0;
            if (r < nr) {
                const int64_t a0 = rp[r0 + r] - base, a1 = rp[r0 + r + 1] - base;
                for (int64_t k = a0 + q; k < a1; k += lp) s += s_p[k];
            }
            for (int off = lp / 2; off > 0; off >>= 1) s += __shfl_xor(s, off, kWave);
            if (r < nr && q == 0) store_y(y, r0 + r, s, alpha, beta);
        }
        return;
    }
    double s = 0.0;  // one long row: r1 == r0 + 1
    for (int64_t q = base + (int64_t)threadIdx.x * 4; q < e1; q += (int64_t)BLOCK * 4) {
        const Pack<int32_t, 4> c = ld_i32<4>(col + q);
        const Pack<V, 4> v = ld_val<4>(val + q);
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (q + j >= e0 && q + j < e1) s += (double)v.v[j] * (double)x[c.v[j]];
    }
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) s += __shfl_down(s, d, kWave);
    if (threadIdx.x % kWave == 0) s_w[threadIdx.x / kWave] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < BLOCK / kWave; ++w) t += s_w[w];
        store_y(y, r0, t, alpha, beta);
    }
}

// ---- ELL, software pipelined: the next slot's loads are in flight during the
// current slot's x gathers --------------------------------------------------------

template <class V, int BLOCK, int RPT, int DEPTH>
__global__ __launch_bounds__(BLOCK) void ell_pipe_kernel(int32_t n_rows, int32_t K, int32_t pitch,
                                                         const int32_t *__restrict__ ecol,
                                                         const V *__restrict__ evals,
                                                         const V *__restrict__ x, V alpha, V beta,
                                                         V *__restrict__ y) {
    const int b = xcd_logical_block(blockIdx.x, gridDim.x);
    const int64_t i0 = ((int64_t)b * BLOCK + threadIdx.x) * RPT;
    if (i0 >= n_rows) return;
    double acc[RPT];
#pragma unroll
    for (int q = 0; q < RPT; ++q) acc[q] = 0.0;
    using CI = Pack<int32_t, RPT>;
    using CV = Pack<V, RPT>;
    // slot k's gathers, then the load of slot `ahead` into (cn, vn), then slot k's
    // products (a select, not a branch, so every gather stays ahead of the load).
    // Buffers rotate by unrolling, never by copying a register a load is still
    // writing, so the wait before the products covers the gathers only.
    auto step = [&](const CI &c, const CV &v, int32_t ahead, CI &cn, CV &vn) {
        V xv[RPT];
        bool ok[RPT];
#pragma unroll
        for (int q = 0; q < RPT; ++q) ok[q] = c.v[q] >= 0;
        gather_x<V, RPT>(x, c.v, ok, xv);
        __builtin_amdgcn_sched_barrier(0);  // gathers issue before the prefetch ...
        const int64_t off = (int64_t)(ahead < K ? ahead : K - 1) * pitch + i0;
        cn = ld_i32<RPT>(ecol + off);
        vn = ld_val<RPT>(evals + off);
        __builtin_amdgcn_sched_barrier(0);  // ... and the prefetch before the products
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const double prod = (double)v.v[q] * (double)xv[q];
            acc[q] += ok[q] ? prod : 0.0;
        }
    };
    if (K > 0) {
        CI cA = ld_i32<RPT>(ecol + i0), cB, cC;
        CV vA = ld_val<RPT>(evals + i0), vB, vC;
        int32_t k = 0;
        if constexpr (DEPTH == 1) {
            for (;;) {
                step(cA, vA, k + 1, cB, vB);
                if (++k >= K) break;
                step(cB, vB, k + 1, cA, vA);
                if (++k >= K) break;
            }
        } else {
            const int64_t off1 = (int64_t)(K > 1 ? 1 : 0) * pitch + i0;
            cB = ld_i32<RPT>(ecol + off1);
            vB = ld_val<RPT>(evals + off1);
            for (;;) {
                step(cA, vA, k + 2, cC, vC);
                if (++k >= K) break;
                step(cB, vB, k + 2, cA, vA);
                if (++k >= K) break;
                step(cC, vC, k + 2, cB, vB);
                if (++k >= K) break;
            }
        }
    }
#pragma unroll
    for (int q = 0; q < RPT; ++q)
        if (i0 + q < n_rows) store_y(y, i0 + q, acc[q], alpha, beta);
}

// ---- ELL, slots split across the waves of a workgroup ----------------------------
//
// Wave w of the KS waves handles slots w, w + KS, w + 2 KS, ... of the same
// 64 * RPT rows (one contiguous 256-byte run per slot and wave), with the
// gather-then-prefetch order of the pipelined kernel; the KS partial sums are
// added in LDS in wave order. For wide, short matrices this gives KS times the
// waves of one thread per row.

template <class V, int KS, int RPT>
__global__ __launch_bounds__(64 * KS) void ell_ksplit_kernel(int32_t n_rows, int32_t K,
                                                             int32_t pitch,
                                                             const int32_t *__restrict__ ecol,
                                                             const V *__restrict__ evals,
                                                             const V *__restrict__ x, V alpha,
                                                             V beta, V *__restrict__ y) {
    __shared__ double s_acc[KS][64 * RPT];
    const int b = xcd_logical_block(blockIdx.x, gridDim.x);
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const int64_t i0 = ((int64_t)b * 64 + lane) * RPT;
    double acc[RPT];
#pragma unroll
    for (int q = 0; q < RPT; ++q) acc[q] = 0.0;
    using CI = Pack<int32_t, RPT>;
    using CV = Pack<V, RPT>;
    const bool live = i0 < n_rows;
    auto step = [&](const CI &c, const CV &v, int32_t ahead, CI &cn, CV &vn) {
        V xv[RPT];
        bool ok[RPT];
#pragma unroll
        for (int q = 0; q < RPT; ++q) ok[q] = c.v[q] >= 0;
        gather_x<V, RPT>(x, c.v, ok, xv);
        __builtin_amdgcn_sched_barrier(0);
        const int64_t off = (int64_t)(ahead < K ? ahead : w) * pitch + i0;
        cn = ld_i32<RPT>(ecol + off);
        vn = ld_val<RPT>(evals + off);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const double prod = (double)v.v[q] * (double)xv[q];
            acc[q] += ok[q] ? prod : 0.0;
        }
    };
    if (live && w < K) {
        CI cA = ld_i32<RPT>(ecol + (int64_t)w * pitch + i0), cB;
        CV vA = ld_val<RPT>(evals + (int64_t)w * pitch + i0), vB;
        int32_t k = w;
        for (;;) {
            step(cA, vA, k + KS, cB, vB);
            if ((k += KS) >= K) break;
            step(cB, vB, k + KS, cA, vA);
            if ((k += KS) >= K) break;
        }
    }
#pragma unroll
    for (int q = 0; q < RPT; ++q) s_acc[w][lane * RPT + q] = acc[q];
    __syncthreads();
    if (w == 0 && live) {
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            double t = s_acc[0][lane * RPT + q];
#pragma unroll
            for (int p = 1; p < KS; ++p) t += s_acc[p][lane * RPT + q];
            if (i0 + q < n_rows) store_y(y, i0 + q, t, alpha, beta);
        }
    }
}

// ---- ELL: RPT consecutive rows per thread, column-major slots ----------------------
//
// Slots are taken UNROLL at a time: the group's index and value loads are all
// issued first (a slot past K is not loaded), then every x gather of the group,
// then the products, so a thread waits for one load latency and one gather
// latency per group. Products are added in slot order.

template <class V, int BLOCK, int RPT, int UNROLL>
__global__ __launch_bounds__(BLOCK) void ell_kernel(int32_t n_rows, int32_t K, int32_t pitch,
                                                    const int32_t *__restrict__ ecol,
                                                    const V *__restrict__ evals,
                                                    const V *__restrict__ x, V alpha, V beta,
                                                    V *__restrict__ y) {
    const int b = xcd_logical_block(blockIdx.x, gridDim.x);
    const int64_t i0 = ((int64_t)b * BLOCK + threadIdx.x) * RPT;
    if (i0 >= n_rows) return;
    double acc[RPT];
#pragma unroll
    for (int q = 0; q < RPT; ++q) acc[q] = 0.0;
    for (int32_t k = 0; k < K; k += UNROLL) {
        Pack<int32_t, RPT> c[UNROLL];
        Pack<V, RPT> v[UNROLL];
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
            if (k + u < K) {  // uniform across the wavefront
                const int64_t off = (int64_t)(k + u) * pitch + i0;
                c[u] = ld_i32<RPT>(ecol + off);
                v[u] = ld_val<RPT>(evals + off);
            } else {
#pragma unroll
                for (int q = 0; q < RPT; ++q) {
                    c[u].v[q] = -1;
                    v[u].v[q] = V(0);
                }
            }
        }
        V xv[UNROLL][RPT];
        bool ok[UNROLL][RPT];
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
#pragma unroll
            for (int q = 0; q < RPT; ++q) ok[u][q] = c[u].v[q] >= 0;
            gather_x<V, RPT>(x, c[u].v, ok[u], xv[u]);
        }
        __builtin_amdgcn_sched_barrier(0);  // every gather of the group before the products
#pragma unroll
        for (int u = 0; u < UNROLL; ++u)
#pragma unroll
            for (int q = 0; q < RPT; ++q) {
                const double sum = acc[q] + (double)v[u].v[q] * (double)xv[u][q];
                acc[q] = ok[u][q] ? sum : acc[q];
            }
    }
#pragma unroll
    for (int q = 0; q < RPT; ++q)
        if (i0 + q < n_rows) store_y(y, i0 + q, acc[q], alpha, beta);
}

// ---- COO: nnz tiles, segmented reduction by row -------------------------------------
//
// Tile t holds entries [t*TILE, min(nnz, (t+1)*TILE)); thread j of the tile holds
// ITEMS consecutive entries. A row segment that lies inside one tile is summed by a
// block-wide segmented scan and written directly. A row that crosses a tile edge
// leaves one partial sum per tile (slot 2t: the tile's first row, slot 2t+1: its
// last row); coo_fixup adds them in tile order. Rows without entries are written
// by the entry that follows the gap. ACCUM adds alpha*s to y instead (HYB tail).

template <class V, int BLOCK, int ITEMS, bool ACCUM>
__global__ __launch_bounds__(BLOCK) void coo_tile_kernel(
    int64_t nnz, int32_t n_rows, const int32_t *__restrict__ row, const int32_t *__restrict__ col,
    const V *__restrict__ val, const V *__restrict__ x, V alpha, V beta, V *__restrict__ y,
    double *__restrict__ part) {
    constexpr int TILE = BLOCK * ITEMS;
    constexpr int WAVES = BLOCK / kWave;
    __shared__ int32_t s_first[BLOCK + 1];
    __shared__ int32_t s_last[BLOCK];
    __shared__ int s_wf[WAVES];
    __shared__ double s_ws[WAVES];

    const int64_t tile = blockIdx.x;
    const int64_t t0 = tile * TILE;
    const int64_t t1 = std::min<int64_t>(nnz, t0 + TILE);
    const int64_t k0 = t0 + (int64_t)threadIdx.x * ITEMS;
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;

    int32_t r[ITEMS];
    double p[ITEMS];
    int n_valid = 0;
    if (k0 + ITEMS <= t1) {
        Pack<int32_t, ITEMS> rr = ld_i32<ITEMS>(row + k0);
        Pack<int32_t, ITEMS> cc = ld_i32<ITEMS>(col + k0);
        Pack<V, ITEMS> vv = ld_val<ITEMS>(val + k0);
        constexpr int G = ITEMS < 4 ? ITEMS : 4;  // x runs of up to 4 entries
#pragma unroll
        for (int g = 0; g < ITEMS; g += G) {
            int32_t c4[G];
            bool ok[G];
            V xv[G];
#pragma unroll
            for (int i = 0; i < G; ++i) {
                c4[i] = cc.v[g + i];
                ok[i] = true;
            }
            gather_x<V, G>(x, c4, ok, xv);
#pragma unroll
            for (int i = 0; i < G; ++i) {
                r[g + i] = rr.v[g + i];
                p[g + i] = (double)vv.v[g + i] * (double)xv[i];
            }
        }
        n_valid = ITEMS;
    } else {
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const int64_t k = k0 + i;
            if (k < t1) {
                r[i] = ld_stream(row + k);
                p[i] = (double)ld_stream(val + k) * (double)x[ld_stream(col + k)];
                ++n_valid;
            } else {
                r[i] = INT_MAX;
                p[i] = 0.0;
            }
        }
    }
    s_first[threadIdx.x] = r[0];
    s_last[threadIdx.x] = n_valid ? r[n_valid - 1] : INT_MAX;
    if (threadIdx.x == 0) s_first[BLOCK] = INT_MAX;
    __syncthreads();

    // Row of the entry before this thread's first one (tile edge counts as a head).
    const int32_t prev_row = (threadIdx.x == 0) ? INT_MIN : s_last[threadIdx.x - 1];
    const int32_t next_row = s_first[threadIdx.x + 1];

    // Thread aggregate for the segmented scan: (a head occurred, sum since last head).
    bool f = false;
    double sum = 0.0;
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        if (i < n_valid) {
            const bool head = (i == 0) ? (r[0] != prev_row) : (r[i] != r[i - 1]);
            if (head) { f = true; sum = p[i]; } else { sum += p[i]; }
        }
    }
    // Inclusive segmented scan across the wave.
    bool fi = f;
    double si = sum;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const int of = __shfl_up((int)fi, d, kWave);
        const double os = __shfl_up(si, d, kWave);
        if (lane >= d) {
            if (!fi) si += os;
            fi = fi || of;
        }
    }
    if (lane == kWave - 1) { s_wf[wave] = fi; s_ws[wave] = si; }
    // Exclusive within the wave.
    int ef = __shfl_up((int)fi, 1, kWave);
    double es = __shfl_up(si, 1, kWave);
    if (lane == 0) { ef = 0; es = 0.0; }
    __syncthreads();
    // Prefix of the earlier waves.
    bool wf = false;
    double ws = 0.0;
    for (int w = 0; w < wave; ++w) {
        if (s_wf[w]) { wf = true; ws = s_ws[w]; } else { ws += s_ws[w]; }
    }
    double carry = ef ? es : ws + es;
    (void)wf;

    const int32_t r_first = row[t0];
    const int32_t r_last = row[t1 - 1];
    const bool open_start = t0 > 0 && row[t0 - 1] == r_first;
    const bool open_end = t1 < nnz && row[t1] == r_last;

    double acc = carry;
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        if (i < n_valid) {
            const bool head = (i == 0) ? (r[0] != prev_row) : (r[i] != r[i - 1]);
            acc = head ? p[i] : acc + p[i];
            const int32_t nxt = (i + 1 < n_valid) ? r[i + 1] : next_row;
            if (nxt != r[i]) {  // segment ends here (a tile edge always ends one)
                const bool first = open_start && r[i] == r_first;
                const bool last = open_end && r[i] == r_last;
                if (!first && !last) {
                    if constexpr (ACCUM) y[r[i]] = (V)((double)y[r[i]] + (double)alpha * acc);
                    else store_y(y, r[i], acc, alpha, beta);
                } else {
                    if (first) part[2 * tile] = acc;
                    if (last) part[2 * tile + 1] = acc;
                }
            }
        }
    }

    if constexpr (!ACCUM) {
        // Empty rows: the entry after a gap writes the rows in between.
        for (int i = 0; i < n_valid; ++i) {
            const int64_t k = k0 + i;
            int32_t before;
            if (i > 0) before = r[i - 1];
            else if (k == 0) before = -1;
            else if (threadIdx.x > 0) before = s_last[threadIdx.x - 1];
            else before = row[k - 1];
            for (int32_t g = before + 1; g < r[i]; ++g) store_y(y, g, 0.0, alpha, beta);
            if (k == nnz - 1)
                for (int32_t g = r[i] + 1; g < n_rows; ++g) store_y(y, g, 0.0, alpha, beta);
        }
    }
}

template <class V, int TILE, bool ACCUM>
__global__ __launch_bounds__(256) void coo_fixup(int64_t nnz, int64_t n_tiles,
                                                 const int32_t *__restrict__ row,
                                                 const double *__restrict__ part, V alpha, V beta,
                                                 V *__restrict__ y) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= n_tiles) return;
    const int64_t t0 = t * TILE, t1 = std::min<int64_t>(nnz, t0 + TILE);
    const int32_t r_first = row[t0], r_last = row[t1 - 1];
    const bool open_start = t0 > 0 && row[t0 - 1] == r_first;
    const bool open_end = t1 < nnz && row[t1] == r_last;
    if (!open_end) return;
    if (open_start && r_first == r_last) return;  // inside a chain, not its start
    double s = part[2 * t + 1];
    for (int64_t u = t + 1; u < n_tiles; ++u) {
        s += part[2 * u];
        const int64_t u1 = std::min<int64_t>(nnz, (u + 1) * TILE);
        if (!(u1 < nnz && row[u1 - 1] == r_last && row[u1] == r_last)) break;
    }
    if constexpr (ACCUM) y[r_last] = (V)((double)y[r_last] + (double)alpha * s);
    else store_y(y, r_last, s, alpha, beta);
}

// ---- SELL-C-sigma: one wavefront per slice of 64 rows --------------------------------
//
// Lane l owns the row at position l of its slice; each 16-byte load brings four
// consecutive slots of that row (the slice stores its rows' slots in runs of
// four), so a wavefront reads 1 KB contiguous per value array and group.
// UNROLL groups are loaded before their gathers are issued; with PIPE the next
// step's loads are in flight during the current gathers (buffers alternate by
// unrolling, as in the pipelined ELL kernel). KS > 1: the KS waves of a
// workgroup share one slice, wave w taking groups w, w + KS, ..., and their
// partial sums meet in LDS in wave order (for slices too wide for one wave).

template <class V, int UNROLL>
struct SellStep {
    Pack<int32_t, 4> c[UNROLL];
    Pack<V, 4> v[UNROLL];
};

template <class V, int UNROLL>
__device__ __forceinline__ void sell_load(SellStep<V, UNROLL> &st, const int32_t *__restrict__ col,
                                          const V *__restrict__ val, int64_t base, int32_t g,
                                          int32_t gstride, int32_t groups, int lane) {
#pragma unroll
    for (int u = 0; u < UNROLL; ++u) {
        const int32_t gu = g + u * gstride;
        const int64_t off = base + (int64_t)(gu < groups ? gu : 0) * (kSellSlice * kSellGroup) + lane * 4;
        st.c[u] = ld_i32<4>(col + off);
        st.v[u] = ld_val<4>(val + off);
        if (gu >= groups)
#pragma unroll
            for (int q = 0; q < 4; ++q) st.c[u].v[q] = -1;
    }
}

template <class V, int UNROLL>
__device__ __forceinline__ void sell_accumulate(const SellStep<V, UNROLL> &st,
                                                const V *__restrict__ x, double &acc) {
    V xv[UNROLL][4];
    bool ok[UNROLL][4];
#pragma unroll
    for (int u = 0; u < UNROLL; ++u) {
#pragma unroll
        for (int q = 0; q < 4; ++q) ok[u][q] = st.c[u].v[q] >= 0;
        gather_x<V, 4>(x, st.c[u].v, ok[u], xv[u]);
    }
#pragma unroll
    for (int u = 0; u < UNROLL; ++u)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const double prod = (double)st.v[u].v[q] * (double)xv[u][q];
            acc += ok[u][q] ? prod : 0.0;
        }
}

// Sum of the slots of one row of a slice, groups g0, g0 + gstride, ... < groups.
template <class V, int UNROLL, bool PIPE>
__device__ __forceinline__ double sell_row_sum(const int32_t *__restrict__ col,
                                               const V *__restrict__ val, const V *__restrict__ x,
                                               int64_t base, int32_t groups, int32_t g0,
                                               int32_t gstride, int lane) {
    double acc = 0.0;
    const int32_t step = UNROLL * gstride;
    if constexpr (!PIPE) {
        for (int32_t g = g0; g < groups; g += step) {
            SellStep<V, UNROLL> st;
            sell_load<V, UNROLL>(st, col, val, base, g, gstride, groups, lane);
            __builtin_amdgcn_sched_barrier(0);
            sell_accumulate<V, UNROLL>(st, x, acc);
        }
    } else {
        if (g0 >= groups) return 0.0;
        SellStep<V, UNROLL> A, B;
        sell_load<V, UNROLL>(A, col, val, base, g0, gstride, groups, lane);
        int32_t g = g0;
        for (;;) {
            // gathers of A, then B's loads, then A's products
            V xv[UNROLL][4];
            bool ok[UNROLL][4];
#pragma unroll
            for (int u = 0; u < UNROLL; ++u) {
#pragma unroll
                for (int q = 0; q < 4; ++q) ok[u][q] = A.c[u].v[q] >= 0;
                gather_x<V, 4>(x, A.c[u].v, ok[u], xv[u]);
            }
            __builtin_amdgcn_sched_barrier(0);
            const bool more = g + step < groups;
            sell_load<V, UNROLL>(B, col, val, base, more ? g + step : g0, gstride, groups, lane);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int u = 0; u < UNROLL; ++u)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const double prod = (double)A.v[u].v[q] * (double)xv[u][q];
                    acc += ok[u][q] ? prod : 0.0;
                }
            if (!more) break;
            g += step;
            // same body with the buffers swapped
#pragma unroll
            for (int u = 0; u < UNROLL; ++u) {
#pragma unroll
                for (int q = 0; q < 4; ++q) ok[u][q] = B.c[u].v[q] >= 0;
                gather_x<V, 4>(x, B.c[u].v, ok[u], xv[u]);
            }
            __builtin_amdgcn_sched_barrier(0);
            const bool more2 = g + step < groups;
            sell_load<V, UNROLL>(A, col, val, base, more2 ? g + step : g0, gstride, groups, lane);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int u = 0; u < UNROLL; ++u)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const double prod = (double)B.v[u].v[q] * (double)xv[u][q];
                    acc += ok[u][q] ? prod : 0.0;
                }
            if (!more2) break;
            g += step;
        }
    }
    return acc;
}

template <class V, int BLOCK, int UNROLL, bool PIPE, bool PERM>
__global__ __launch_bounds__(BLOCK) void sell_kernel(int32_t n_rows, int32_t n_slices,
                                                     const int64_t *__restrict__ slice_ptr,
                                                     const int32_t *__restrict__ perm,
                                                     const int32_t *__restrict__ col,
                                                     const V *__restrict__ val,
                                                     const V *__restrict__ x, V alpha, V beta,
                                                     V *__restrict__ y) {
    constexpr int WPB = BLOCK / kWave;
    const int b = xcd_logical_block(blockIdx.x, gridDim.x);
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int lane = threadIdx.x % kWave;
    const int64_t sl = (int64_t)b * WPB + w;
    if (sl >= n_slices) return;  // whole wavefronts
    const int64_t base = slice_ptr[sl];
    const int32_t groups = (int32_t)((slice_ptr[sl + 1] - base) / (kSellSlice * kSellGroup));
    const double acc = sell_row_sum<V, UNROLL, PIPE>(col, val, x, base, groups, 0, 1, lane);
    const int64_t p = sl * kSellSlice + lane;
    if (p < n_rows) store_y(y, PERM ? perm[p] : p, acc, alpha, beta);
}

template <class V, int KS, int UNROLL, bool PIPE, bool PERM>
__global__ __launch_bounds__(KS * 64) void sell_ksplit_kernel(int32_t n_rows, int32_t n_slices,
                                                              const int64_t *__restrict__ slice_ptr,
                                                              const int32_t *__restrict__ perm,
                                                              const int32_t *__restrict__ col,
                                                              const V *__restrict__ val,
                                                              const V *__restrict__ x, V alpha,
                                                              V beta, V *__restrict__ y) {
    __shared__ double s_acc[KS][kWave];
    const int64_t sl = xcd_logical_block(blockIdx.x, gridDim.x);
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int lane = threadIdx.x % kWave;
    const int64_t base = slice_ptr[sl];
    const int32_t groups = (int32_t)((slice_ptr[sl + 1] - base) / (kSellSlice * kSellGroup));
    s_acc[w][lane] = sell_row_sum<V, UNROLL, PIPE>(col, val, x, base, groups, w, KS, lane);
    __syncthreads();
    if (w == 0) {
        double t = s_acc[0][lane];
#pragma unroll
        for (int q = 1; q < KS; ++q) t += s_acc[q][lane];
        const int64_t p = sl * kSellSlice + lane;
        if (p < n_rows) store_y(y, PERM ? perm[p] : p, t, alpha, beta);
    }
}

// ---- BELL: ELL over b x b blocks ---------------------------------------------------
//
// B / RB threads share a block row; thread j of them owns rows j * RB ... j * RB
// + RB - 1 of it. Per slot it reads the block column (the same word for the
// block row's threads), its RB x B values (contiguous: a wavefront streams
// consecutive blocks) and the B consecutive x values of the block column with
// one vector load where the block lies inside the matrix. UNROLL slots are
// loaded before their products. Rows are summed in FP64 in block-column order.

template <class V, int N>
__device__ __forceinline__ void load_x_run(const V *__restrict__ x, int64_t c0, int32_t n_cols,
                                           V (&xv)[N]) {
    if (c0 + N <= n_cols) {
        const Pack<V, N> p = ld_xrun<V, N>(x + c0);
#pragma unroll
        for (int j = 0; j < N; ++j) xv[j] = p.v[j];
    } else {
#pragma unroll
        for (int j = 0; j < N; ++j) xv[j] = (c0 + j < n_cols) ? x[c0 + j] : V(0);
    }
}

template <class V, int B, int RB, int BLOCK, int UNROLL>
__global__ __launch_bounds__(BLOCK) void bell_kernel(int32_t n_rows, int32_t n_cols, int32_t K,
                                                     int32_t pitch, int32_t nbr,
                                                     const int32_t *__restrict__ bcol,
                                                     const V *__restrict__ bval,
                                                     const V *__restrict__ x, V alpha, V beta,
                                                     V *__restrict__ y) {
    constexpr int TPB = B / RB;  // threads per block row
    const int blk = xcd_logical_block(blockIdx.x, gridDim.x);
    const int64_t t = (int64_t)blk * BLOCK + threadIdx.x;
    const int64_t br = t / TPB;
    const int sub = (int)(t % TPB);
    if (br >= nbr) return;
    double acc[RB];
#pragma unroll
    for (int i = 0; i < RB; ++i) acc[i] = 0.0;
    for (int32_t k = 0; k < K; k += UNROLL) {
        int32_t bc[UNROLL];
        Pack<V, RB * B> v[UNROLL];
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
            const int32_t ku = k + u < K ? k + u : k;
            const int64_t slot = (int64_t)ku * pitch + br;
            bc[u] = k + u < K ? ld_stream(bcol + slot) : -1;
            v[u] = ld_val<RB * B>(bval + (slot * B + sub * RB) * B);
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
            if (bc[u] < 0) continue;  // padding: no x is read
            V xv[B];
            load_x_run<V, B>(x, (int64_t)bc[u] * B, n_cols, xv);
#pragma unroll
            for (int i = 0; i < RB; ++i)
#pragma unroll
                for (int j = 0; j < B; ++j) acc[i] += (double)v[u].v[i * B + j] * (double)xv[j];
        }
    }
#pragma unroll
    for (int i = 0; i < RB; ++i) {
        const int64_t r = br * B + sub * RB + i;
        if (r < n_rows) store_y(y, r, acc[i], alpha, beta);
    }
}

template <class V>
__global__ __launch_bounds__(256) void scale_y(int32_t n, V beta, V *__restrict__ y) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        y[i] = beta == V(0) ? V(0) : (V)((double)beta * (double)y[i]);
}

// ---- variant tables and launchers ------------------------------------------------

struct Args {
    const spmv_matrix_s *h;
    const void *x;
    void *y;
    double alpha, beta;
    hipStream_t s;
};

using Launcher = void (*)(const Args &);

struct Variant {
    spmv_variant_info info;
    Launcher f32, f64;
};

inline int grid_of(int64_t units, int per_block) {
    int64_t g = ceil_div(std::max<int64_t>(units, 1), per_block);
    if (g > INT32_MAX) fail(SPMV_ERR_INVALID_ARG, "grid too large");
    return (int)g;
}

// Column-split COO: one tiled COO pass per column panel of the split copy; the
// first pass writes every y_i (alpha*s + beta*y), the others add alpha*s.
template <class V, int ITEMS>
void coo_split_launch(const Args &a) {
    const spmv_matrix_s *h = a.h;
    const SplitPart &P = h->split;
    if (!P.built) fail(SPMV_ERR_NOT_CONVERTED, "column-split COO copy not built");
    if (h->n_rows == 0) return;
    for (int32_t p = 0; p < P.panels; ++p) {
        const int64_t off = P.start[p];
        const int32_t *row = P.row.as<int32_t>() + off, *col = P.col.as<int32_t>() + off;
        const V *val = P.val.as<V>() + off;
        if (p == 0)
            coo_launch_impl<V, ITEMS, false>(P.count[p], h->n_rows, row, col, val, a,
                                             h->coo_partials.as<double>());
        else
            coo_launch_impl<V, ITEMS, true>(P.count[p], h->n_rows, row, col, val, a,
                                            h->coo_partials.as<double>());
    }
}

template <class V>
void launch_coo_arrays(int64_t nnz, int32_t n_rows, const int32_t *row, const int32_t *col,
                       const V *val, const Args &a, double *part, int items, bool accum);

// BLOCK * ITEMS >= 512: the partial-sum buffer holds two slots per 512 entries.
template <class V, int ITEMS, bool ACCUM, int BLOCK = 256>
void coo_launch_impl(int64_t nnz, int32_t n_rows, const int32_t *row, const int32_t *col,
                     const V *val, const Args &a, double *part) {
    constexpr int TILE = BLOCK * ITEMS;
    static_assert(TILE >= 512 && BLOCK % kWave == 0, "tile size");
    const V al = (V)a.alpha, be = (V)a.beta;
    if (nnz == 0) {
        if (!ACCUM && n_rows > 0) {
            scale_y<V><<<std::min(grid_of(n_rows, 256), 4096), 256, 0, a.s>>>(n_rows, be, (V *)a.y);
            SPMV_CHECK_LAUNCH();
        }
        return;
    }
    const int64_t tiles = ceil_div(nnz, TILE);
    coo_tile_kernel<V, BLOCK, ITEMS, ACCUM><<<grid_of(nnz, TILE), BLOCK, 0, a.s>>>(
        nnz, n_rows, row, col, val, (const V *)a.x, al, be, (V *)a.y, part);
    SPMV_CHECK_LAUNCH();
    if (tiles > 1) {
        coo_fixup<V, TILE, ACCUM><<<grid_of(tiles, 256), 256, 0, a.s>>>(nnz, tiles, row, part, al,
                                                                       be, (V *)a.y);
        SPMV_CHECK_LAUNCH();
    }
}

template <class V>
void launch_coo_arrays(int64_t nnz, int32_t n_rows, const int32_t *row, const int32_t *col,
                       const V *val, const Args &a, double *part, int items, bool accum) {
#define COO_CASE(IT)                                                                         \
    if (items == IT) {                                                                       \
        if (accum) coo_launch_impl<V, IT, true>(nnz, n_rows, row, col, val, a, part);        \
        else coo_launch_impl<V, IT, false>(nnz, n_rows, row, col, val, a, part);             \
        return;                                                                              \
    }
    COO_CASE(2)
    COO_CASE(4)
    COO_CASE(8)
#undef COO_CASE
    fail(SPMV_ERR_INVALID_ARG, "bad COO items %d", items);
}

template <class V, int UNROLL>
void csr_scalar_launch(const Args &a) {
    const spmv_matrix_s *h = a.h;
    if (h->n_rows == 0) return;
    csr_scalar_kernel<V, 256, UNROLL><<<grid_of(h->n_rows, 256), 256, 0, a.s>>>(
        h->n_rows, h->row_ptr.as<int32_t>(), h->col.as<int32_t>(), h->val.as<V>(),
        (const V *)a.x, (V)a.alpha, (V)a.beta, (V *)a.y);
    SPMV_CHECK_LAUNCH();
}

template <class V, int L, int UNROLL>
void csr_vector_launch(const Args &a) {
    const spmv_matrix_s *h = a.h;
    if (h->n_rows == 0) return;
    constexpr int BLOCK = 256;
    csr_vector_kernel<V, BLOCK, L, UNROLL><<<grid_of(h->n_rows, BLOCK / L), BLOCK, 0, a.s>>>(
        h->n_rows, h->row_ptr.as<int32_t>(), h->col.as<int32_t>(), h->val.as<V>(),
        (const V *)a.x, (V)a.alpha, (V)a.beta, (V *)a.y);
    SPMV_CHECK_LAUNCH();
}

template <class V, int L, int UNROLL>
void csr_vector4_launch(const Args &a) {
    const spmv_matrix_s *h = a.h;
    if (h->n_rows == 0) return;
    constexpr int BLOCK = 256;
    csr_vector4_kernel<V, BLOCK, L, UNROLL><<<grid_of(h->n_rows, BLOCK / L), BLOCK, 0, a.s>>>(
        h->n_rows, h->row_ptr.as<int32_t>(), h->col.as<int32_t>(), h->val.as<V>(),
        (const V *)a.x, (V)a.alpha, (V)a.beta, (V *)a.y);
    SPMV_CHECK_LAUNCH();
}

// The same kernel at another workgroup size (the thread-block size the paper
// tunes in its compile-time mode).
template <class V, int BLOCK, int L, int UNROLL>
void csr_vector4_block_launch(const Args &a) {
    const spmv_matrix_s *h = a.h;
    if (h->n_rows == 0) return;
    static_assert(BLOCK % L == 0 && BLOCK >= kWave, "a workgroup holds whole lane groups");
    csr_vector4_kernel<V, BLOCK, L, UNROLL><<<grid_of(h->n_rows, BLOCK / L), BLOCK, 0, a.s>>>(
        h->n_rows, h->row_ptr.as<int32_t>(), h->col.as<int32_t>(), h->val.as<V>(),
        (const V *)a.x, (V)a.alpha, (V)a.beta, (V *)a.y);
    SPMV_CHECK_LAUNCH();
}

template <class V, int L, int PASSES>
void csr_pipe_launch(const Args &a) {
    const spmv_matrix_s *h = a.h;
    if (h->n_rows == 0) return;
    if (h->nnz == 0) {  // masked gathers read x[0]; with no entries x may be empty
        csr_vector4_launch<V, L, 1>(a);
        return;
    }
    constexpr int BLOCK = 256;
    csr_pipe_kernel<V, BLOCK, L, PASSES><<<grid_of(h->n_rows, BLOCK / L * PASSES), BLOCK, 0, a.s>>>(
        h->n_rows, h->row_ptr.as<int32_t>(), h->col.as<int32_t>(), h->val.as<V>(),
        (const V *)a.x, (V)a.alpha, (V)a.beta, (V *)a.y);
    SPMV_CHECK_LAUNCH();
}

template <class V, int BLOCK>
void csr_stream_launch(const Args &a) {
    const spmv_matrix_s *h = a.h;
    if (h->n_rows == 0) return;
    if (!h->csr_blocks.built) fail(SPMV_ERR_NOT_CONVERTED, "CSR stream row blocks not built");
    csr_stream_kernel<V, BLOCK><<<h->csr_blocks.blocks, BLOCK, 0, a.s>>>(
        h->csr_blocks.rows.as<int32_t>(), h->row_ptr.as<int32_t>(), h->col.as<int32_t>(),
        h->val.as<V>(), (const V *)a.x, (V)a.alpha, (V)a.beta, (V *)a.y);
    SPMV_CHECK_LAUNCH();
}

template <class V, int RPT, int DEPTH>
void ell_pipe_launch(const Args &a) {
    const spmv_matrix_s *h = a.h;
    if (h->n_rows == 0) return;
    constexpr int BLOCK = 256;
    ell_pipe_kernel<V, BLOCK, RPT, DEPTH><<<grid_of(ceil_div(h->n_rows, RPT), BLOCK), BLOCK, 0, a.s>>>(
        h->n_rows, h->ell.K, h->ell.pitch, h->ell.col.as<int32_t>(), h->ell.val.as<V>(),
        (const V *)a.x, (V)a.alpha, (V)a.beta, (V *)a.y);
    SPMV_CHECK_LAUNCH();
}

template <class V, int ITEMS, int BLOCK = 256>
void coo_launch(const Args &a) {
    const spmv_matrix_s *h = a.h;
    coo_launch_impl<V, ITEMS, false, BLOCK>(h->nnz, h->n_rows, h->row.as<int32_t>(),
                                            h->col.as<int32_t>(), h->val.as<V>(), a,
                                            h->coo_partials.as<double>());
}

template <class V, int RPT, int UNROLL, int BLOCK = 256>
void ell_arrays_launch(int32_t n_rows, int32_t K, int32_t pitch, const int32_t *ecol,
                       const V *evals, const Args &a) {
    if (n_rows == 0) return;
    ell_kernel<V, BLOCK, RPT, UNROLL><<<grid_of(ceil_div(n_rows, RPT), BLOCK), BLOCK, 0, a.s>>>(
        n_rows, K, pitch, ecol, evals, (const V *)a.x, (V)a.alpha, (V)a.beta, (V *)a.y);
    SPMV_CHECK_LAUNCH();
}

template <class V, int RPT, int UNROLL, int BLOCK = 256>
void ell_launch(const Args &a) {
    const spmv_matrix_s *h = a.h;
    ell_arrays_launch<V, RPT, UNROLL, BLOCK>(h->n_rows, h->ell.K, h->ell.pitch, h->ell.col.as<int32_t>(),
                                      h->ell.val.as<V>(), a);
}

template <class V, int KS, int RPT>
void ell_ksplit_launch(const Args &a) {
    const spmv_matrix_s *h = a.h;
    if (h->n_rows == 0) return;
    if (h->nnz == 0) {  // masked gathers read x[0]; with no entries x may be empty
        ell_launch<V, 1, 1>(a);
        return;
    }
    ell_ksplit_kernel<V, KS, RPT><<<grid_of(ceil_div(h->n_rows, RPT), 64), 64 * KS, 0, a.s>>>(
        h->n_rows, h->ell.K, h->ell.pitch, h->ell.col.as<int32_t>(), h->ell.val.as<V>(),
        (const V *)a.x, (V)a.alpha, (V)a.beta, (V *)a.y);
    SPMV_CHECK_LAUNCH();
}

// HYB with its ELL part split over KS waves per row block (wide, short ELL parts,
// e.g. HYB of a banded matrix, where the rule keeps every row in the ELL part).
template <class V, int KS, int RPT, int ITEMS>
void hyb_ksplit_launch(const Args &a) {
    const spmv_matrix_s *h = a.h;
    if (h->n_rows == 0) return;
    if (h->hyb.K == 0) {  // no slots: the plain kernel writes y = beta * y
        ell_arrays_launch<V, 1, 1>(h->n_rows, 0, h->hyb.pitch, h->hyb.ell_col.as<int32_t>(),
                                   h->hyb.ell_val.as<V>(), a);
    } else {
        ell_ksplit_kernel<V, KS, RPT><<<grid_of(ceil_div(h->n_rows, RPT), 64), 64 * KS, 0, a.s>>>(
            h->n_rows, h->hyb.K, h->hyb.pitch, h->hyb.ell_col.as<int32_t>(), h->hyb.ell_val.as<V>(),
            (const V *)a.x, (V)a.alpha, (V)a.beta, (V *)a.y);
        SPMV_CHECK_LAUNCH();
    }
    if (h->hyb.nnz_tail > 0)
        coo_launch_impl<V, ITEMS, true>(h->hyb.nnz_tail, h->n_rows, h->hyb.tail_row.as<int32_t>(),
                                        h->hyb.tail_col.as<int32_t>(), h->hyb.tail_val.as<V>(), a,
                                        h->hyb.partials.as<double>());
}

template <class V, int RPT, int ITEMS, int BLOCK = 256>
void hyb_launch(const Args &a) {
    const spmv_matrix_s *h = a.h;
    ell_arrays_launch<V, RPT, 4, BLOCK>(h->n_rows, h->hyb.K, h->hyb.pitch, h->hyb.ell_col.as<int32_t>(),
                                 h->hyb.ell_val.as<V>(), a);
    if (h->hyb.nnz_tail > 0)
        coo_launch_impl<V, ITEMS, true>(h->hyb.nnz_tail, h->n_rows, h->hyb.tail_row.as<int32_t>(),
                                        h->hyb.tail_col.as<int32_t>(), h->hyb.tail_val.as<V>(), a,
                                        h->hyb.partials.as<double>());
}

// HYB with its COO tail added by the sorted-block kernel (accumulate mode) after
// the ELL part.
template <class V, int RPT, int ITEMS>
void hyb_sorted_launch(const Args &a) {
    const spmv_matrix_s *h = a.h;
    if (!h->hyb_sorted.built) fail(SPMV_ERR_NOT_CONVERTED, "sorted-block copy of the HYB tail not built");
    ell_arrays_launch<V, RPT, 4>(h->n_rows, h->hyb.K, h->hyb.pitch, h->hyb.ell_col.as<int32_t>(),
                                 h->hyb.ell_val.as<V>(), a);
    hyb_sorted_tail(h, ITEMS, a.alpha, a.x, a.y, a.s);
}

template <class V, int BLOCK, int UNROLL, bool PIPE>
void sell_launch(const Args &a) {
    const spmv_matrix_s *h = a.h;
    const SellPart &P = h->sell;
    if (h->n_rows == 0 || P.n_slices == 0) return;
    constexpr int WPB = BLOCK / kWave;
    const int grid = grid_of(P.n_slices, WPB);
    if (P.sigma > 1)
        sell_kernel<V, BLOCK, UNROLL, PIPE, true><<<grid, BLOCK, 0, a.s>>>(
            h->n_rows, P.n_slices, P.slice_ptr.as<int64_t>(), P.perm.as<int32_t>(),
            P.col.as<int32_t>(), P.val.as<V>(), (const V *)a.x, (V)a.alpha, (V)a.beta, (V *)a.y);
    else
        sell_kernel<V, BLOCK, UNROLL, PIPE, false><<<grid, BLOCK, 0, a.s>>>(
            h->n_rows, P.n_slices, P.slice_ptr.as<int64_t>(), nullptr, P.col.as<int32_t>(),
            P.val.as<V>(), (const V *)a.x, (V)a.alpha, (V)a.beta, (V *)a.y);
    SPMV_CHECK_LAUNCH();
}

template <class V, int KS, int UNROLL, bool PIPE>
void sell_ksplit_launch(const Args &a) {
    const spmv_matrix_s *h = a.h;
    const SellPart &P = h->sell;
    if (h->n_rows == 0 || P.n_slices == 0) return;
    if (P.sigma > 1)
        sell_ksplit_kernel<V, KS, UNROLL, PIPE, true><<<P.n_slices, KS * kWave, 0, a.s>>>(
            h->n_rows, P.n_slices, P.slice_ptr.as<int64_t>(), P.perm.as<int32_t>(),
            P.col.as<int32_t>(), P.val.as<V>(), (const V *)a.x, (V)a.alpha, (V)a.beta, (V *)a.y);
    else
        sell_ksplit_kernel<V, KS, UNROLL, PIPE, false><<<P.n_slices, KS * kWave, 0, a.s>>>(
            h->n_rows, P.n_slices, P.slice_ptr.as<int64_t>(), nullptr, P.col.as<int32_t>(),
            P.val.as<V>(), (const V *)a.x, (V)a.alpha, (V)a.beta, (V *)a.y);
    SPMV_CHECK_LAUNCH();
}

template <class V, int B, int RB, int BLOCK, int UNROLL>
void bell_launch_b(const Args &a) {
    const spmv_matrix_s *h = a.h;
    const BellPart &P = h->bell;
    if constexpr (RB > B) {
        fail(SPMV_ERR_NOT_APPLICABLE, "BELL variant with %d rows per thread on %dx%d blocks", RB, B, B);
    } else {
        const int64_t threads = (int64_t)P.n_block_rows * (B / RB);
        bell_kernel<V, B, RB, BLOCK, UNROLL><<<grid_of(threads, BLOCK), BLOCK, 0, a.s>>>(
            h->n_rows, h->n_cols, P.K, P.pitch, P.n_block_rows, P.col.as<int32_t>(), P.val.as<V>(),
            (const V *)a.x, (V)a.alpha, (V)a.beta, (V *)a.y);
        SPMV_CHECK_LAUNCH();
    }
}

template <class V, int RB, int BLOCK, int UNROLL>
void bell_launch(const Args &a) {
    const spmv_matrix_s *h = a.h;
    if (!h->bell.built) fail(SPMV_ERR_NOT_CONVERTED, "BELL not converted");
    if (h->n_rows == 0) return;
    switch (h->bell.b) {
        case 2: bell_launch_b<V, 2, RB, BLOCK, UNROLL>(a); return;
        case 4: bell_launch_b<V, 4, RB, BLOCK, UNROLL>(a); return;
        case 8: bell_launch_b<V, 8, RB, BLOCK, UNROLL>(a); return;
    }
    fail(SPMV_ERR_INVALID_ARG, "BELL block size %d", h->bell.b);
}

#define V2(kind, blk, lanes, unr, fn) \
    Variant{{kind, blk, lanes, unr, 1, 0, 1}, fn<float>, fn<double>}
#define V4(kind, blk, lanes, unr, fn) \
    Variant{{kind, blk, lanes, unr, 4, 0, 1}, fn<float>, fn<double>}
#define VN(kind, blk, lanes, unr, vec, fn) \
    Variant{{kind, blk, lanes, unr, vec, 0, 1}, fn<float>, fn<double>}
#define VP(kind, blk, lanes, vec, pipe, fn) \
    Variant{{kind, blk, lanes, 1, vec, pipe, 1}, fn<float>, fn<double>}
#define VK(kind, blk, rpt, ks, fn) \
    Variant{{kind, blk, rpt, 1, rpt, 1, ks}, fn<float>, fn<double>}
#define VT(kind, blk, items, tiles, fn) \
    Variant{{kind, blk, items, 1, 4, 1, tiles}, fn<float>, fn<double>}

template <class V> void csr_s1(const Args &a) { csr_scalar_launch<V, 1>(a); }
template <class V> void csr_s4(const Args &a) { csr_scalar_launch<V, 4>(a); }
#define CSRV(L, U) \
    template <class V> void csr_v##L##_##U(const Args &a) { csr_vector_launch<V, L, U>(a); }
CSRV(2, 1) CSRV(2, 2) CSRV(2, 4)
CSRV(4, 1) CSRV(4, 2) CSRV(4, 4)
CSRV(8, 1) CSRV(8, 2) CSRV(8, 4)
CSRV(16, 1) CSRV(16, 2) CSRV(16, 4)
CSRV(32, 1) CSRV(32, 2) CSRV(32, 4)
CSRV(64, 1) CSRV(64, 2) CSRV(64, 4)
#undef CSRV
#define CSRV4(L, U) \
    template <class V> void csr_w##L##_##U(const Args &a) { csr_vector4_launch<V, L, U>(a); }
CSRV4(2, 1) CSRV4(2, 2)
CSRV4(4, 1) CSRV4(4, 2)
CSRV4(8, 1) CSRV4(8, 2)
CSRV4(16, 1) CSRV4(16, 2)
CSRV4(32, 1) CSRV4(32, 2)
CSRV4(64, 1) CSRV4(64, 2)
#undef CSRV4
#define CSRP(L, P) \
    template <class V> void csr_p##L##_##P(const Args &a) { csr_pipe_launch<V, L, P>(a); }
CSRP(2, 2) CSRP(2, 4)
CSRP(4, 2) CSRP(4, 4)
CSRP(8, 2) CSRP(8, 4)
CSRP(16, 2) CSRP(16, 4)
CSRP(32, 2) CSRP(32, 4)
CSRP(64, 2) CSRP(64, 4)
#undef CSRP
#define CSRB(B, L, U) \
    template <class V> void csr_b##B##_##L##_##U(const Args &a) { csr_vector4_block_launch<V, B, L, U>(a); }
CSRB(64, 4, 2) CSRB(128, 4, 2) CSRB(512, 4, 2) CSRB(1024, 4, 2)
CSRB(64, 16, 2) CSRB(128, 16, 2) CSRB(512, 16, 2) CSRB(1024, 16, 2)
#undef CSRB
template <class V> void ell_p1(const Args &a) { ell_pipe_launch<V, 1, 1>(a); }
template <class V> void ell_p2(const Args &a) { ell_pipe_launch<V, 2, 1>(a); }
template <class V> void ell_p4(const Args &a) { ell_pipe_launch<V, 4, 1>(a); }
template <class V> void ell_q2(const Args &a) { ell_pipe_launch<V, 2, 2>(a); }
template <class V> void ell_q4(const Args &a) { ell_pipe_launch<V, 4, 2>(a); }
template <class V> void ell_k2_2(const Args &a) { ell_ksplit_launch<V, 2, 2>(a); }
template <class V> void ell_k4_1(const Args &a) { ell_ksplit_launch<V, 4, 1>(a); }
template <class V> void ell_k4_2(const Args &a) { ell_ksplit_launch<V, 4, 2>(a); }
template <class V> void ell_k4_4(const Args &a) { ell_ksplit_launch<V, 4, 4>(a); }
template <class V> void coo_2(const Args &a) { coo_launch<V, 2>(a); }
template <class V> void coo_4(const Args &a) { coo_launch<V, 4>(a); }
template <class V> void coo_8(const Args &a) { coo_launch<V, 8>(a); }
template <class V> void coo_panel_4(const Args &a) { panel_spmv(a.h, 4, a.alpha, a.x, a.beta, a.y, a.s); }
template <class V> void coo_panel_8(const Args &a) { panel_spmv(a.h, 8, a.alpha, a.x, a.beta, a.y, a.s); }
template <class V> void coo_sorted_4(const Args &a) { sorted_spmv(a.h, 4, a.alpha, a.x, a.beta, a.y, a.s); }
template <class V> void coo_sorted_8(const Args &a) { sorted_spmv(a.h, 8, a.alpha, a.x, a.beta, a.y, a.s); }
template <class V> void coo_sorted_16(const Args &a) { sorted_spmv(a.h, 16, a.alpha, a.x, a.beta, a.y, a.s); }
template <class V> void coo_tiles_8(const Args &a) { sorted_tiles_spmv(a.h, 2, 8, a.alpha, a.x, a.beta, a.y, a.s); }
template <class V> void coo_tiles_16(const Args &a) { sorted_tiles_spmv(a.h, 2, 16, a.alpha, a.x, a.beta, a.y, a.s); }
template <class V> void coo_tiles4_8(const Args &a) { sorted_tiles_spmv(a.h, 4, 8, a.alpha, a.x, a.beta, a.y, a.s); }
template <class V> void coo_tiles4_16(const Args &a) { sorted_tiles_spmv(a.h, 4, 16, a.alpha, a.x, a.beta, a.y, a.s); }
template <class V> void coo_split_4(const Args &a) { coo_split_launch<V, 4>(a); }
template <class V> void coo_split_8(const Args &a) { coo_split_launch<V, 8>(a); }
template <class V> void csr_stream_256(const Args &a) { csr_stream_launch<V, 256>(a); }
template <class V> void csr_stream_512(const Args &a) { csr_stream_launch<V, 512>(a); }
template <class V> void ell_1_1(const Args &a) { ell_launch<V, 1, 1>(a); }
template <class V> void ell_1_2(const Args &a) { ell_launch<V, 1, 2>(a); }
template <class V> void ell_2_1(const Args &a) { ell_launch<V, 2, 1>(a); }
template <class V> void ell_2_2(const Args &a) { ell_launch<V, 2, 2>(a); }
template <class V> void ell_4_1(const Args &a) { ell_launch<V, 4, 1>(a); }
template <class V> void ell_4_2(const Args &a) { ell_launch<V, 4, 2>(a); }
template <class V> void ell_1_4(const Args &a) { ell_launch<V, 1, 4>(a); }
template <class V> void ell_2_4(const Args &a) { ell_launch<V, 2, 4>(a); }
template <class V> void ell_1_8(const Args &a) { ell_launch<V, 1, 8>(a); }
template <class V> void ell_2_8(const Args &a) { ell_launch<V, 2, 8>(a); }
template <class V> void ell_4_4(const Args &a) { ell_launch<V, 4, 4>(a); }
template <class V> void ell_4_8(const Args &a) { ell_launch<V, 4, 8>(a); }
template <class V> void hyb_1_4(const Args &a) { hyb_launch<V, 1, 4>(a); }
template <class V> void hyb_s1_8(const Args &a) { hyb_sorted_launch<V, 1, 8>(a); }
template <class V> void hyb_s2_8(const Args &a) { hyb_sorted_launch<V, 2, 8>(a); }
template <class V> void hyb_s2_16(const Args &a) { hyb_sorted_launch<V, 2, 16>(a); }
template <class V> void hyb_1_8(const Args &a) { hyb_launch<V, 1, 8>(a); }
template <class V> void hyb_2_4(const Args &a) { hyb_launch<V, 2, 4>(a); }
template <class V> void hyb_4_4(const Args &a) { hyb_launch<V, 4, 4>(a); }
template <class V> void hyb_4_8(const Args &a) { hyb_launch<V, 4, 8>(a); }
template <class V> void hyb_s4_8(const Args &a) { hyb_sorted_launch<V, 4, 8>(a); }
template <class V> void hyb_k4_2(const Args &a) { hyb_ksplit_launch<V, 4, 2, 8>(a); }
template <class V> void hyb_k4_4(const Args &a) { hyb_ksplit_launch<V, 4, 4, 8>(a); }
// the paper's thread-block-size knob on ELL, tiled COO and HYB's ELL part
#define BLKV(name, call) \
    template <class V> void name(const Args &a) { call(a); }
BLKV(ell_b64_4_2, (ell_launch<V, 4, 2, 64>)) BLKV(ell_b128_4_2, (ell_launch<V, 4, 2, 128>))
BLKV(ell_b512_4_2, (ell_launch<V, 4, 2, 512>)) BLKV(ell_b1024_4_2, (ell_launch<V, 4, 2, 1024>))
BLKV(ell_b64_2_4, (ell_launch<V, 2, 4, 64>)) BLKV(ell_b128_2_4, (ell_launch<V, 2, 4, 128>))
BLKV(ell_b512_2_4, (ell_launch<V, 2, 4, 512>)) BLKV(ell_b1024_2_4, (ell_launch<V, 2, 4, 1024>))
BLKV(coo_b64_8, (coo_launch<V, 8, 64>)) BLKV(coo_b128_4, (coo_launch<V, 4, 128>))
BLKV(coo_b512_4, (coo_launch<V, 4, 512>)) BLKV(coo_b1024_4, (coo_launch<V, 4, 1024>))
BLKV(coo_b1024_2, (coo_launch<V, 2, 1024>))
BLKV(hyb_b128_2_8, (hyb_launch<V, 2, 8, 128>)) BLKV(hyb_b512_2_8, (hyb_launch<V, 2, 8, 512>))
BLKV(hyb_b1024_2_8, (hyb_launch<V, 2, 8, 1024>)) BLKV(hyb_b64_1_8, (hyb_launch<V, 1, 8, 64>))
#undef BLKV
template <class V> void hyb_2_8(const Args &a) { hyb_launch<V, 2, 8>(a); }

#define SELLV(B, U, P) \
    template <class V> void sell_##B##_##U##_##P(const Args &a) { sell_launch<V, B, U, P>(a); }
SELLV(256, 1, 0) SELLV(256, 2, 0) SELLV(256, 4, 0) SELLV(256, 1, 1) SELLV(256, 2, 1) SELLV(256, 4, 1)
SELLV(64, 2, 0) SELLV(128, 2, 0) SELLV(512, 2, 0) SELLV(1024, 2, 0)
#undef SELLV
template <class V> void sell_k4(const Args &a) { sell_ksplit_launch<V, 4, 1, true>(a); }
template <class V> void sell_k16(const Args &a) { sell_ksplit_launch<V, 16, 1, true>(a); }
#define BELLV(R, B, U) \
    template <class V> void bell_##R##_##B##_##U(const Args &a) { bell_launch<V, R, B, U>(a); }
BELLV(1, 256, 1) BELLV(2, 256, 1) BELLV(4, 256, 1) BELLV(1, 256, 2) BELLV(2, 256, 2) BELLV(4, 256, 2)
BELLV(1, 64, 1) BELLV(1, 128, 1) BELLV(1, 512, 1) BELLV(1, 1024, 1)
BELLV(2, 64, 1) BELLV(2, 128, 1) BELLV(2, 512, 1) BELLV(2, 1024, 1)
BELLV(1, 256, 4) BELLV(1, 128, 2) BELLV(1, 64, 2) BELLV(2, 256, 4)
#undef BELLV

#define VS(blk, unr, pipe, ks, fn) \
    Variant{{SPMV_KERNEL_SELL, blk, 1, unr, 4, pipe, ks}, fn<float>, fn<double>}
#define VB(blk, rb, unr, fn) \
    Variant{{SPMV_KERNEL_BELL, blk, rb, unr, 0, 0, 1}, fn<float>, fn<double>}

const std::vector<Variant> &table(spmv_format f) {
    static const std::vector<Variant> csr = {
        V2(SPMV_KERNEL_CSR_SCALAR, 256, 1, 1, csr_s1),
        V2(SPMV_KERNEL_CSR_SCALAR, 256, 1, 4, csr_s4),
        V2(SPMV_KERNEL_CSR_VECTOR, 256, 2, 1, csr_v2_1),
        V2(SPMV_KERNEL_CSR_VECTOR, 256, 2, 2, csr_v2_2),
        V2(SPMV_KERNEL_CSR_VECTOR, 256, 2, 4, csr_v2_4),
        V2(SPMV_KERNEL_CSR_VECTOR, 256, 4, 1, csr_v4_1),
        V2(SPMV_KERNEL_CSR_VECTOR, 256, 4, 2, csr_v4_2),
        V2(SPMV_KERNEL_CSR_VECTOR, 256, 4, 4, csr_v4_4),
        V2(SPMV_KERNEL_CSR_VECTOR, 256, 8, 1, csr_v8_1),
        V2(SPMV_KERNEL_CSR_VECTOR, 256, 8, 2, csr_v8_2),
        V2(SPMV_KERNEL_CSR_VECTOR, 256, 8, 4, csr_v8_4),
        V2(SPMV_KERNEL_CSR_VECTOR, 256, 16, 1, csr_v16_1),
        V2(SPMV_KERNEL_CSR_VECTOR, 256, 16, 2, csr_v16_2),
        V2(SPMV_KERNEL_CSR_VECTOR, 256, 16, 4, csr_v16_4),
        V2(SPMV_KERNEL_CSR_VECTOR, 256, 32, 1, csr_v32_1),
        V2(SPMV_KERNEL_CSR_VECTOR, 256, 32, 2, csr_v32_2),
        V2(SPMV_KERNEL_CSR_VECTOR, 256, 32, 4, csr_v32_4),
        V2(SPMV_KERNEL_CSR_VECTOR, 256, 64, 1, csr_v64_1),
        V2(SPMV_KERNEL_CSR_VECTOR, 256, 64, 2, csr_v64_2),
        V2(SPMV_KERNEL_CSR_VECTOR, 256, 64, 4, csr_v64_4),
        V4(SPMV_KERNEL_CSR_VECTOR, 256, 2, 1, csr_w2_1),
        V4(SPMV_KERNEL_CSR_VECTOR, 256, 2, 2, csr_w2_2),
        V4(SPMV_KERNEL_CSR_VECTOR, 256, 4, 1, csr_w4_1),
        V4(SPMV_KERNEL_CSR_VECTOR, 256, 4, 2, csr_w4_2),
        V4(SPMV_KERNEL_CSR_VECTOR, 256, 8, 1, csr_w8_1),
        V4(SPMV_KERNEL_CSR_VECTOR, 256, 8, 2, csr_w8_2),
        V4(SPMV_KERNEL_CSR_VECTOR, 256, 16, 1, csr_w16_1),
        V4(SPMV_KERNEL_CSR_VECTOR, 256, 16, 2, csr_w16_2),
        V4(SPMV_KERNEL_CSR_VECTOR, 256, 32, 1, csr_w32_1),
        V4(SPMV_KERNEL_CSR_VECTOR, 256, 32, 2, csr_w32_2),
        V4(SPMV_KERNEL_CSR_VECTOR, 256, 64, 1, csr_w64_1),
        V4(SPMV_KERNEL_CSR_VECTOR, 256, 64, 2, csr_w64_2),
        VP(SPMV_KERNEL_CSR_VECTOR, 256, 2, 4, 2, csr_p2_2),
        VP(SPMV_KERNEL_CSR_VECTOR, 256, 2, 4, 4, csr_p2_4),
        VP(SPMV_KERNEL_CSR_VECTOR, 256, 4, 4, 2, csr_p4_2),
        VP(SPMV_KERNEL_CSR_VECTOR, 256, 4, 4, 4, csr_p4_4),
        VP(SPMV_KERNEL_CSR_VECTOR, 256, 8, 4, 2, csr_p8_2),
        VP(SPMV_KERNEL_CSR_VECTOR, 256, 8, 4, 4, csr_p8_4),
        VP(SPMV_KERNEL_CSR_VECTOR, 256, 16, 4, 2, csr_p16_2),
        VP(SPMV_KERNEL_CSR_VECTOR, 256, 16, 4, 4, csr_p16_4),
        VP(SPMV_KERNEL_CSR_VECTOR, 256, 32, 4, 2, csr_p32_2),
        VP(SPMV_KERNEL_CSR_VECTOR, 256, 32, 4, 4, csr_p32_4),
        VP(SPMV_KERNEL_CSR_VECTOR, 256, 64, 4, 2, csr_p64_2),
        VP(SPMV_KERNEL_CSR_VECTOR, 256, 64, 4, 4, csr_p64_4),
        V4(SPMV_KERNEL_CSR_VECTOR, 64, 4, 2, csr_b64_4_2),
        V4(SPMV_KERNEL_CSR_VECTOR, 128, 4, 2, csr_b128_4_2),
        V4(SPMV_KERNEL_CSR_VECTOR, 512, 4, 2, csr_b512_4_2),
        V4(SPMV_KERNEL_CSR_VECTOR, 1024, 4, 2, csr_b1024_4_2),
        V4(SPMV_KERNEL_CSR_VECTOR, 64, 16, 2, csr_b64_16_2),
        V4(SPMV_KERNEL_CSR_VECTOR, 128, 16, 2, csr_b128_16_2),
        V4(SPMV_KERNEL_CSR_VECTOR, 512, 16, 2, csr_b512_16_2),
        V4(SPMV_KERNEL_CSR_VECTOR, 1024, 16, 2, csr_b1024_16_2),
        VN(SPMV_KERNEL_CSR_STREAM, 256, 1, 1, 4, csr_stream_256),
        VN(SPMV_KERNEL_CSR_STREAM, 512, 1, 1, 4, csr_stream_512),
    };
    static const std::vector<Variant> coo = {
        VN(SPMV_KERNEL_COO, 256, 2, 1, 2, coo_2),
        VN(SPMV_KERNEL_COO, 256, 4, 1, 4, coo_4),
        VN(SPMV_KERNEL_COO, 256, 8, 1, 4, coo_8),
        VP(SPMV_KERNEL_COO_PANEL, 512, 4, 4, 1, coo_panel_4),
        VP(SPMV_KERNEL_COO_PANEL, 512, 8, 4, 1, coo_panel_8),
        VP(SPMV_KERNEL_COO_SORTED, 1024, 4, 4, 1, coo_sorted_4),
        VP(SPMV_KERNEL_COO_SORTED, 1024, 8, 4, 1, coo_sorted_8),
        VP(SPMV_KERNEL_COO_SORTED, 1024, 16, 4, 1, coo_sorted_16),
        VN(SPMV_KERNEL_COO_SPLIT, 256, 4, 1, 4, coo_split_4),
        VN(SPMV_KERNEL_COO_SPLIT, 256, 8, 1, 4, coo_split_8),
        VN(SPMV_KERNEL_COO, 64, 8, 1, 4, coo_b64_8), VN(SPMV_KERNEL_COO, 128, 4, 1, 4, coo_b128_4),
        VN(SPMV_KERNEL_COO, 512, 4, 1, 4, coo_b512_4), VN(SPMV_KERNEL_COO, 1024, 4, 1, 4, coo_b1024_4),
        VN(SPMV_KERNEL_COO, 1024, 2, 1, 2, coo_b1024_2),
        VT(SPMV_KERNEL_COO_SORTED, 1024, 8, 2, coo_tiles_8),
        VT(SPMV_KERNEL_COO_SORTED, 1024, 16, 2, coo_tiles_16),
        VT(SPMV_KERNEL_COO_SORTED, 1024, 8, 4, coo_tiles4_8),
        VT(SPMV_KERNEL_COO_SORTED, 1024, 16, 4, coo_tiles4_16),
    };
    static const std::vector<Variant> ell = {
        VN(SPMV_KERNEL_ELL, 256, 1, 1, 1, ell_1_1), VN(SPMV_KERNEL_ELL, 256, 1, 2, 1, ell_1_2),
        VN(SPMV_KERNEL_ELL, 256, 2, 1, 2, ell_2_1), VN(SPMV_KERNEL_ELL, 256, 2, 2, 2, ell_2_2),
        VN(SPMV_KERNEL_ELL, 256, 4, 1, 4, ell_4_1), VN(SPMV_KERNEL_ELL, 256, 4, 2, 4, ell_4_2),
        VP(SPMV_KERNEL_ELL, 256, 1, 1, 1, ell_p1), VP(SPMV_KERNEL_ELL, 256, 2, 2, 1, ell_p2),
        VP(SPMV_KERNEL_ELL, 256, 4, 4, 1, ell_p4),
        VP(SPMV_KERNEL_ELL, 256, 2, 2, 2, ell_q2), VP(SPMV_KERNEL_ELL, 256, 4, 4, 2, ell_q4),
        VK(SPMV_KERNEL_ELL, 128, 2, 2, ell_k2_2), VK(SPMV_KERNEL_ELL, 256, 1, 4, ell_k4_1),
        VK(SPMV_KERNEL_ELL, 256, 2, 4, ell_k4_2), VK(SPMV_KERNEL_ELL, 256, 4, 4, ell_k4_4),
        VN(SPMV_KERNEL_ELL, 256, 1, 8, 1, ell_1_8), VN(SPMV_KERNEL_ELL, 256, 2, 8, 2, ell_2_8),
        VN(SPMV_KERNEL_ELL, 256, 4, 4, 4, ell_4_4), VN(SPMV_KERNEL_ELL, 256, 4, 8, 4, ell_4_8),
        VN(SPMV_KERNEL_ELL, 256, 1, 4, 1, ell_1_4), VN(SPMV_KERNEL_ELL, 256, 2, 4, 2, ell_2_4),
        VN(SPMV_KERNEL_ELL, 64, 4, 2, 4, ell_b64_4_2), VN(SPMV_KERNEL_ELL, 128, 4, 2, 4, ell_b128_4_2),
        VN(SPMV_KERNEL_ELL, 512, 4, 2, 4, ell_b512_4_2), VN(SPMV_KERNEL_ELL, 1024, 4, 2, 4, ell_b1024_4_2),
        VN(SPMV_KERNEL_ELL, 64, 2, 4, 2, ell_b64_2_4), VN(SPMV_KERNEL_ELL, 128, 2, 4, 2, ell_b128_2_4),
        VN(SPMV_KERNEL_ELL, 512, 2, 4, 2, ell_b512_2_4), VN(SPMV_KERNEL_ELL, 1024, 2, 4, 2, ell_b1024_2_4),
    };
    static const std::vector<Variant> hyb = {
        VN(SPMV_KERNEL_HYB, 256, 1, 4, 1, hyb_1_4), VN(SPMV_KERNEL_HYB, 256, 1, 8, 1, hyb_1_8),
        VN(SPMV_KERNEL_HYB, 256, 2, 4, 2, hyb_2_4), VN(SPMV_KERNEL_HYB, 256, 2, 8, 2, hyb_2_8),
        // pipelined = 1: the tail goes through the sorted-block COO kernel
        Variant{{SPMV_KERNEL_HYB, 256, 1, 8, 1, 1, 1}, hyb_s1_8<float>, hyb_s1_8<double>},
        Variant{{SPMV_KERNEL_HYB, 256, 2, 8, 2, 1, 1}, hyb_s2_8<float>, hyb_s2_8<double>},
        Variant{{SPMV_KERNEL_HYB, 256, 2, 16, 2, 1, 1}, hyb_s2_16<float>, hyb_s2_16<double>},
        VN(SPMV_KERNEL_HYB, 128, 2, 8, 2, hyb_b128_2_8), VN(SPMV_KERNEL_HYB, 512, 2, 8, 2, hyb_b512_2_8),
        VN(SPMV_KERNEL_HYB, 1024, 2, 8, 2, hyb_b1024_2_8), VN(SPMV_KERNEL_HYB, 64, 1, 8, 1, hyb_b64_1_8),
        VN(SPMV_KERNEL_HYB, 256, 4, 4, 4, hyb_4_4), VN(SPMV_KERNEL_HYB, 256, 4, 8, 4, hyb_4_8),
        Variant{{SPMV_KERNEL_HYB, 256, 4, 8, 4, 1, 1}, hyb_s4_8<float>, hyb_s4_8<double>},
        Variant{{SPMV_KERNEL_HYB, 256, 2, 8, 2, 0, 4}, hyb_k4_2<float>, hyb_k4_2<double>},
        Variant{{SPMV_KERNEL_HYB, 256, 4, 8, 4, 0, 4}, hyb_k4_4<float>, hyb_k4_4<double>},
    };
    static const std::vector<Variant> sell = {
        VS(256, 1, 0, 1, sell_256_1_0), VS(256, 2, 0, 1, sell_256_2_0), VS(256, 4, 0, 1, sell_256_4_0),
        VS(256, 1, 1, 1, sell_256_1_1), VS(256, 2, 1, 1, sell_256_2_1), VS(256, 4, 1, 1, sell_256_4_1),
        VS(64, 2, 0, 1, sell_64_2_0), VS(128, 2, 0, 1, sell_128_2_0), VS(512, 2, 0, 1, sell_512_2_0),
        VS(1024, 2, 0, 1, sell_1024_2_0),
        VS(256, 1, 1, 4, sell_k4), VS(1024, 1, 1, 16, sell_k16),
    };
    static const std::vector<Variant> bell = {
        VB(256, 1, 1, bell_1_256_1), VB(256, 2, 1, bell_2_256_1), VB(256, 4, 1, bell_4_256_1),
        VB(256, 1, 2, bell_1_256_2), VB(256, 2, 2, bell_2_256_2), VB(256, 4, 2, bell_4_256_2),
        VB(64, 1, 1, bell_1_64_1), VB(128, 1, 1, bell_1_128_1), VB(512, 1, 1, bell_1_512_1),
        VB(1024, 1, 1, bell_1_1024_1),
        VB(64, 2, 1, bell_2_64_1), VB(128, 2, 1, bell_2_128_1), VB(512, 2, 1, bell_2_512_1),
        VB(1024, 2, 1, bell_2_1024_1),
        VB(256, 1, 4, bell_1_256_4), VB(128, 1, 2, bell_1_128_2), VB(64, 1, 2, bell_1_64_2),
        VB(256, 2, 4, bell_2_256_4),
    };
    static const std::vector<Variant> none;
    switch (f) {
        case SPMV_FMT_CSR: return csr;
        case SPMV_FMT_COO: return coo;
        case SPMV_FMT_ELL: return ell;
        case SPMV_FMT_HYB: return hyb;
        case SPMV_FMT_SELL: return sell;
        case SPMV_FMT_BELL: return bell;
    }
    return none;
}

}  // namespace

// Smallest COO tile is 256 threads x 2 entries.
int64_t coo_partials_bytes(int64_t nnz, spmv_dtype) {
    return 2 * std::max<int64_t>(1, ceil_div(nnz, 512)) * (int64_t)sizeof(double);
}

int32_t variant_count(spmv_format f, spmv_dtype dt) {
    if (dt != SPMV_F32 && dt != SPMV_F64) return 0;
    return (int32_t)table(f).size();
}

bool variant_describe(spmv_format f, spmv_dtype dt, int32_t idx, spmv_variant_info *out) {
    const auto &t = table(f);
    if (dt != SPMV_F32 && dt != SPMV_F64) return false;
    if (idx < 0 || idx >= (int32_t)t.size()) return false;
    if (out) *out = t[idx].info;
    return true;
}

int32_t default_variant(const spmv_matrix_s *h, spmv_format f) {
    switch (f) {
        case SPMV_FMT_CSR: {
            // lanes per row ~ mean row length, two loads in flight per lane
            const double mean = h->n_rows ? (double)h->nnz / h->n_rows : 0.0;
            int L = 2;
            while (L < 64 && L < mean) L *= 2;
            const auto &t = table(f);
            for (int32_t i = 0; i < (int32_t)t.size(); ++i)
                if (t[i].info.kernel == SPMV_KERNEL_CSR_VECTOR && t[i].info.lanes == L &&
                    t[i].info.unroll == 2)
                    return i;
            return 0;
        }
        case SPMV_FMT_COO: return 1;
        case SPMV_FMT_ELL: return 0;
        case SPMV_FMT_HYB: return 0;
        case SPMV_FMT_SELL: return 1;  // two groups per step, 256 threads
        case SPMV_FMT_BELL: {
            // a whole 2 x 2 block per thread, one row of a larger block per thread
            const int rb = (h->bell.built && h->bell.b == 2) ? 2 : 1;
            const auto &t = table(f);
            for (int32_t i = 0; i < (int32_t)t.size(); ++i)
                if (t[i].info.lanes == rb && t[i].info.block == 256 && t[i].info.unroll == 1) return i;
            return 0;
        }
    }
    return 0;
}

// Bytes of the device arrays one run of (f, idx) reads besides x and y: the
// layout the variant streams, with its padding and its pointer and order arrays.
// -1 when that layout is not built.
int64_t stored_bytes(const spmv_matrix_s *h, spmv_format f, int32_t idx) {
    const auto &t = table(f);
    if (idx < 0 || idx >= (int32_t)t.size()) return -1;
    const spmv_variant_info &info = t[idx].info;
    const int64_t v = (int64_t)dtype_size(h->dt), n = h->n_rows, nnz = h->nnz;
    auto sorted_bytes = [&](const SortedPart &P) -> int64_t {
        if (!P.built) return -1;
        return P.stream * (4 + v + (P.row16 ? 2 : 0)) + 3 * (int64_t)(P.blocks + 1) * 4;
    };
    switch (info.kernel) {
        case SPMV_KERNEL_CSR_SCALAR:
        case SPMV_KERNEL_CSR_VECTOR: return (n + 1) * 4 + nnz * (4 + v);
        case SPMV_KERNEL_CSR_STREAM:
            if (!h->csr_blocks.built) return -1;
            return (n + 1) * 4 + nnz * (4 + v) + (int64_t)(h->csr_blocks.blocks + 1) * 4;
        case SPMV_KERNEL_COO: return nnz * (8 + v);
        case SPMV_KERNEL_COO_PANEL:
            if (!h->panel.built) return -1;
            return h->panel.stream * (4 + v) +
                   (ceil_div(n, std::max(h->panel.rows_per_wave, 1)) + 1) * 4;
        case SPMV_KERNEL_COO_SORTED: {
            if (info.ksplit == 1) return sorted_bytes(h->sorted);
            const SortedPart &P = h->sorted_tiles[info.ksplit == 4];
            if (!P.built) return -1;
            // the tiles' streams and pointers, chunk bases, and the other ranges'
            // row sums written and read back with y read and written again
            return P.stream * (4 + v + (P.row16 ? 2 : 0)) + (P.delta ? P.stream / kSortedChunk * 4 : 0) +
                   (int64_t)(P.blocks + 1) * 4 + 2 * (int64_t)(P.blocks * P.tiles + 1) * 4 +
                   2 * (int64_t)(P.tiles - 1) * n * v + 2 * n * v;
        }
        case SPMV_KERNEL_COO_SPLIT: {
            if (!h->split.built) return -1;
            int64_t e = 0;
            for (int64_t c : h->split.count) e += c;
            return e * (8 + v);
        }
        case SPMV_KERNEL_ELL:
            if (!h->ell.built) return -1;
            return (int64_t)h->ell.K * h->ell.pitch * (4 + v);
        case SPMV_KERNEL_HYB: {
            if (!h->hyb.built) return -1;
            const int64_t ell = (int64_t)h->hyb.K * h->hyb.pitch * (4 + v);
            if (info.pipelined == 1) {
                const int64_t tb = h->hyb.nnz_tail > 0 ? sorted_bytes(h->hyb_sorted) : 0;
                return tb < 0 ? -1 : ell + tb;
            }
            return ell + h->hyb.nnz_tail * (8 + v);
        }
        case SPMV_KERNEL_SELL:
            if (!h->sell.built) return -1;
            return h->sell.slots * (4 + v) + (int64_t)(h->sell.n_slices + 1) * 8 +
                   (h->sell.sigma > 1 ? 4 * n : 0);
        case SPMV_KERNEL_BELL: {
            if (!h->bell.built) return -1;
            const int64_t slots = (int64_t)h->bell.K * h->bell.pitch;
            return slots * 4 + slots * h->bell.b * h->bell.b * v;
        }
    }
    return -1;
}

bool variant_applicable(const spmv_matrix_s *h, spmv_format f, int32_t idx) {
    const auto &t = table(f);
    if (idx < 0 || idx >= (int32_t)t.size()) return false;
    if (f == SPMV_FMT_BELL && h->bell.built) return t[idx].info.lanes <= h->bell.b;
    return true;
}

bool variant_needs_panel(spmv_format f, int32_t idx) {
    const auto &t = table(f);
    return idx >= 0 && idx < (int32_t)t.size() && t[idx].info.kernel == SPMV_KERNEL_COO_PANEL;
}

bool variant_needs_split(spmv_format f, int32_t idx) {
    const auto &t = table(f);
    return idx >= 0 && idx < (int32_t)t.size() && t[idx].info.kernel == SPMV_KERNEL_COO_SPLIT;
}

bool variant_needs_csr_blocks(spmv_format f, int32_t idx) {
    const auto &t = table(f);
    return idx >= 0 && idx < (int32_t)t.size() && t[idx].info.kernel == SPMV_KERNEL_CSR_STREAM;
}

void build_csr_blocks(spmv_matrix_s *h, hipStream_t s) {
    if (h->csr_blocks.built) return;
    const int64_t n = h->n_rows;
    std::vector<int32_t> rp(n + 1);
    SPMV_HIP(hipMemcpyAsync(rp.data(), h->row_ptr.p, rp.size() * 4, hipMemcpyDeviceToHost, s));
    SPMV_HIP(hipStreamSynchronize(s));
    std::vector<int32_t> rows{0};
    for (int64_t r = 0; r < n;) {
        const int64_t base = rp[r] & ~int64_t(3);
        int64_t e = r + 1;  // a row too long for the stage stays alone
        if (rp[r + 1] - base <= kCsrStreamCap)
            while (e < n && e - r < kCsrStreamRows && rp[e + 1] - base <= kCsrStreamCap) ++e;
        rows.push_back((int32_t)e);
        r = e;
    }
    CsrBlocks B;
    B.blocks = (int32_t)rows.size() - 1;
    B.rows.alloc(rows.size() * 4);
    SPMV_HIP(hipMemcpyAsync(B.rows.p, rows.data(), rows.size() * 4, hipMemcpyHostToDevice, s));
    SPMV_HIP(hipStreamSynchronize(s));
    B.built = true;
    h->csr_blocks = std::move(B);
}

bool variant_needs_hyb_sorted(spmv_format f, int32_t idx) {
    const auto &t = table(f);
    return idx >= 0 && idx < (int32_t)t.size() && t[idx].info.kernel == SPMV_KERNEL_HYB &&
           t[idx].info.pipelined == 1;
}

bool variant_needs_sorted(spmv_format f, int32_t idx) {
    const auto &t = table(f);
    return idx >= 0 && idx < (int32_t)t.size() && t[idx].info.kernel == SPMV_KERNEL_COO_SORTED &&
           t[idx].info.ksplit == 1;
}

int variant_sorted_tiles(spmv_format f, int32_t idx) {
    const auto &t = table(f);
    return idx >= 0 && idx < (int32_t)t.size() && t[idx].info.kernel == SPMV_KERNEL_COO_SORTED &&
                   t[idx].info.ksplit > 1
               ? t[idx].info.ksplit
               : 0;
}

void launch_spmv(const spmv_matrix_s *h, spmv_format f, int32_t variant, double alpha,
                 const void *x, double beta, void *y, hipStream_t s) {
    const auto &t = table(f);
    if (variant < 0 || variant >= (int32_t)t.size())
        fail(SPMV_ERR_INVALID_ARG, "variant %d out of range for format %d", variant, (int)f);
    Args a{h, x, y, alpha, beta, s};
    if (h->dt == SPMV_F64) t[variant].f64(a);
    else t[variant].f32(a);
}

}  // namespace spmv
