// COO SpMV over row blocks and column panels, with x staged in LDS.
//
// A format's entries may be kept in any order (paper, Background: sparse
// formats; COO stores explicit coordinates). This copy of the COO entries is
// ordered for MI355X's memory system: a workgroup owns 16 consecutive row
// groups (one per wavefront) and walks the column panels its rows touch, each
// panel being 64 KB of x loaded once into LDS with 16-byte loads. The x
// gathers then hit LDS instead of moving a 128-byte L2 line per 4-byte
// element, which is what bounds a row-parallel CSR kernel on matrices whose
// columns are spread over a vector that does not fit one CU's L1.
//
// Each wavefront streams its own entries (16-byte loads of packed indices and
// values, the next chunk in flight while the current one is reduced) and sums
// them by row with a segmented scan across the wave; the row sums go into an
// FP64 accumulator in LDS that only this wave touches, so the order of every
// addition is fixed and the result is deterministic. Row totals are written
// once at the end as y = alpha * s + beta * y.
#include <algorithm>
#include <climits>

#include "common.hpp"
#include "device.hpp"

namespace spmv {
namespace {

constexpr int kB = 256;                         // builder workgroup size
constexpr int kNT = kPanelWaves * kWave;        // panel kernel workgroup size
constexpr int64_t kMaxKeys = int64_t(1) << 26;  // (group, panel) runs at most

int grid_of_n(int64_t n) { return (int)std::min<int64_t>(std::max<int64_t>(ceil_div(n, kB), 1), 65536); }

// ---- the kernel ----------------------------------------------------------------

template <class V, int ITEMS, bool XVEC>
__global__ __launch_bounds__(kNT) void coo_panel_kernel(
    int32_t n_rows, int32_t n_cols, int32_t rw, int32_t panels,
    const int32_t *__restrict__ blk_ptr, const int32_t *__restrict__ blk_panel,
    const int32_t *__restrict__ run_ptr, const int32_t *__restrict__ idx,
    const V *__restrict__ val, const V *__restrict__ x, V alpha, V beta, V *__restrict__ y) {
    constexpr int W = (int)(65536 / sizeof(V));
    constexpr int CH = kWave * ITEMS;
    constexpr int XV = 16 / (int)sizeof(V);
    constexpr int XL = W / XV / kNT;
    typedef V X16 __attribute__((ext_vector_type(XV)));
    __shared__ X16 s_x[W / XV];
    __shared__ double s_y[kPanelWaves * kPanelRowsMax];
    const V *sxv = (const V *)s_x;

    const int b = xcd_logical_block(blockIdx.x, gridDim.x);
    const int w = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int64_t row0 = ((int64_t)b * kPanelWaves + w) * rw;
    double *sy = s_y + w * kPanelRowsMax;
    for (int i = lane; i < rw; i += kWave) sy[i] = 0.0;
    const int32_t *rp = run_ptr + ((int64_t)b * kPanelWaves + w) * (panels + 1);
    const int32_t k0 = blk_ptr[b], k1 = blk_ptr[b + 1];
    const int64_t end = rp[panels];
    int64_t pos = rp[0];

    using CI = Pack<int32_t, ITEMS>;
    using CV = Pack<V, ITEMS>;
    // Chunk at stream position q: lane l holds entries q + ITEMS*l .. + ITEMS-1.
    // Runs are padded to multiples of 4, so a chunk lane is whole or absent.
    auto load = [&](int64_t q, CI &c, CV &v) {
        const int64_t e = q + ITEMS * lane;
        if (e < end) {
            c = ld_i32<ITEMS>(idx + e);
            v = ld_val<ITEMS>(val + e);
        } else {
#pragma unroll
            for (int j = 0; j < ITEMS; ++j) { c.v[j] = kPanelPad; v.v[j] = V(0); }
        }
    };
    X16 xr[XL];
    auto load_x = [&](int p) {
        const int64_t c0 = (int64_t)p * W;
#pragma unroll
        for (int j = 0; j < XL; ++j) {
            const int64_t c = c0 + (int64_t)(threadIdx.x + j * kNT) * XV;
            if (XVEC && c + XV <= n_cols) {
                xr[j] = *(const X16 *)(x + c);
            } else {
#pragma unroll
                for (int q = 0; q < XV; ++q) xr[j][q] = (c + q < n_cols) ? x[c + q] : V(0);
            }
        }
    };
    // Entries of the chunk inside [lo, hi) belong to the panel in LDS. They
    // are sorted by row, so each row is one segment; its last entry adds the
    // segment's sum to the row's accumulator.
    auto process = [&](const CI &c, const CV &v, int64_t q, int64_t lo, int64_t hi) {
        int32_t r[ITEMS];
        double pr[ITEMS];
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
            const int64_t e = q + ITEMS * lane + j;
            const uint32_t u = (uint32_t)c.v[j];
            const bool ok = e >= lo && e < hi && c.v[j] != kPanelPad;
            r[j] = ok ? (int32_t)(u >> 16) : -1;
            const V xv = sxv[ok ? (u & 0xFFFFu) : 0u];
            pr[j] = ok ? (double)v.v[j] * (double)xv : 0.0;
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
            if (tail && r[j] >= 0) sy[r[j]] += run;
        }
    };

    CI c0, c1;
    CV v0, v1;
    load(pos, c0, v0);
    load(pos + CH, c1, v1);
    if (k0 < k1) load_x(blk_panel[k0]);
    for (int k = k0; k < k1; ++k) {
        const int p = blk_panel[k];
        __syncthreads();  // every wave is done with the previous panel
#pragma unroll
        for (int j = 0; j < XL; ++j) s_x[threadIdx.x + j * kNT] = xr[j];
        __syncthreads();
        if (k + 1 < k1) load_x(blk_panel[k + 1]);
        const int64_t lo = rp[p], hi = rp[p + 1];
        while (pos < hi) {
            process(c0, v0, pos, lo, hi);
            if (pos + CH > hi) break;  // the chunk continues into a later panel
            pos += CH;
            c0 = c1;
            v0 = v1;
            load(pos + CH, c1, v1);
        }
    }
    for (int i = lane; i < rw; i += kWave) {
        const int64_t row = row0 + i;
        if (row < n_rows) store_y(y, row, sy[i], alpha, beta);
    }
}

// ---- the builder ----------------------------------------------------------------

__global__ void panel_keys(const int32_t *__restrict__ row, const int32_t *__restrict__ col,
                           int64_t nnz, int32_t rw, int32_t panels, int32_t width,
                           uint64_t *__restrict__ key, uint32_t *__restrict__ perm) {
    for (int64_t k = (int64_t)blockIdx.x * kB + threadIdx.x; k < nnz; k += (int64_t)gridDim.x * kB) {
        key[k] = (uint64_t)(row[k] / rw) * (uint64_t)panels + (uint64_t)(col[k] / width);
        perm[k] = (uint32_t)k;
    }
}

// first[q] = number of sorted keys below q, for q = 0 .. n_keys.
__global__ void panel_first(const uint64_t *__restrict__ skey, int64_t nnz, int64_t n_keys,
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

__global__ void panel_padded(const int32_t *__restrict__ first, int64_t n_keys,
                             int32_t *__restrict__ padded) {
    for (int64_t q = (int64_t)blockIdx.x * kB + threadIdx.x; q <= n_keys;
         q += (int64_t)gridDim.x * kB)
        padded[q] = q < n_keys ? (first[q + 1] - first[q] + 3) & ~3 : 0;
}

template <class V>
__global__ void panel_scatter(const uint64_t *__restrict__ skey, const uint32_t *__restrict__ perm,
                              int64_t nnz, const int32_t *__restrict__ row,
                              const int32_t *__restrict__ col, const V *__restrict__ val,
                              const int32_t *__restrict__ first, const int32_t *__restrict__ start,
                              int32_t rw, int32_t width, int32_t *__restrict__ idx_out,
                              V *__restrict__ val_out) {
    for (int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x; i < nnz; i += (int64_t)gridDim.x * kB) {
        const uint64_t q = skey[i];
        const uint32_t e = perm[i];
        const int64_t pos = (int64_t)start[q] + (i - first[q]);
        idx_out[pos] = (int32_t)(((uint32_t)(row[e] % rw) << 16) | (uint32_t)(col[e] % width));
        val_out[pos] = val[e];
    }
}

__global__ void panel_run_ptr(const int32_t *__restrict__ start, int64_t groups, int32_t panels,
                              int32_t *__restrict__ run_ptr) {
    const int64_t n = groups * (panels + 1);
    for (int64_t t = (int64_t)blockIdx.x * kB + threadIdx.x; t < n; t += (int64_t)gridDim.x * kB) {
        const int64_t g = t / (panels + 1), p = t % (panels + 1);
        run_ptr[t] = start[g * panels + p];
    }
}

// flag[b * panels + p] = 1 when any group of block b has an entry in panel p.
__global__ void panel_flags(const int32_t *__restrict__ first, int32_t blocks, int32_t panels,
                            int32_t *__restrict__ flag) {
    const int64_t n = (int64_t)blocks * panels;
    for (int64_t t = (int64_t)blockIdx.x * kB + threadIdx.x; t <= n; t += (int64_t)gridDim.x * kB) {
        int any = 0;
        if (t < n) {
            const int64_t b = t / panels, p = t % panels;
            for (int w = 0; w < kPanelWaves; ++w) {
                const int64_t q = (b * kPanelWaves + w) * panels + p;
                any |= first[q + 1] > first[q];
            }
        }
        flag[t] = any;
    }
}

__global__ void panel_lists(const int32_t *__restrict__ fpos, int32_t blocks, int32_t panels,
                            int32_t *__restrict__ blk_panel, int32_t *__restrict__ blk_ptr) {
    const int64_t n = (int64_t)blocks * panels;
    for (int64_t t = (int64_t)blockIdx.x * kB + threadIdx.x; t < n; t += (int64_t)gridDim.x * kB)
        if (fpos[t + 1] > fpos[t]) blk_panel[fpos[t]] = (int32_t)(t % panels);
    for (int64_t b = (int64_t)blockIdx.x * kB + threadIdx.x; b <= blocks;
         b += (int64_t)gridDim.x * kB)
        blk_ptr[b] = fpos[b * panels];
}

template <class V, int ITEMS>
void launch_panel(const spmv_matrix_s *h, double alpha, const void *x, double beta, void *y,
                  hipStream_t s) {
    const PanelPart &P = h->panel;
    const bool xvec = ((uintptr_t)x % 16) == 0;
#define PANEL_ARGS                                                                              \
    h->n_rows, h->n_cols, P.rows_per_wave, P.panels, P.blk_ptr.as<int32_t>(),                   \
        P.blk_panel.as<int32_t>(), P.run_ptr.as<int32_t>(), P.idx.as<int32_t>(), P.val.as<V>(), \
        (const V *)x, (V)alpha, (V)beta, (V *)y
    if (xvec) coo_panel_kernel<V, ITEMS, true><<<P.blocks, kNT, 0, s>>>(PANEL_ARGS);
    else coo_panel_kernel<V, ITEMS, false><<<P.blocks, kNT, 0, s>>>(PANEL_ARGS);
#undef PANEL_ARGS
    SPMV_CHECK_LAUNCH();
}

}  // namespace

void build_panel(spmv_matrix_s *h, hipStream_t s) {
    if (h->panel.built) return;
    int cus = 0;
    SPMV_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, h->device));
    const int32_t width = panel_width(h->dt);
    const int64_t n = h->n_rows, nnz = h->nnz;
    PanelPart P;
    P.rows_per_wave = (int32_t)std::min<int64_t>(
        kPanelRowsMax, std::max<int64_t>(1, ceil_div(n, (int64_t)kPanelWaves * std::max(cus, 1))));
    P.blocks = (int32_t)ceil_div(n, (int64_t)kPanelWaves * P.rows_per_wave);
    P.panels = (int32_t)std::max<int64_t>(1, ceil_div(h->n_cols, width));
    const int64_t groups = (int64_t)P.blocks * kPanelWaves;
    const int64_t n_keys = groups * P.panels;
    if (n_keys > kMaxKeys || groups * (P.panels + 1) > kMaxKeys || nnz > (int64_t)INT32_MAX / 2)
        fail(SPMV_ERR_NOT_APPLICABLE, "panel layout needs %lld runs (at most %lld)",
             (long long)n_keys, (long long)kMaxKeys);
    const size_t vs = dtype_size(h->dt);

    DevBuf keys, perm, first, start;
    first.alloc((n_keys + 1) * 4);
    start.alloc((n_keys + 1) * 4);
    if (nnz > 0) {
        keys.alloc(nnz * 8);
        perm.alloc(nnz * 4);
        panel_keys<<<grid_of_n(nnz), kB, 0, s>>>(h->row.as<int32_t>(), h->col.as<int32_t>(), nnz,
                                                 P.rows_per_wave, P.panels, width,
                                                 keys.as<uint64_t>(), perm.as<uint32_t>());
        SPMV_CHECK_LAUNCH();
        int bits = 0;
        while (bits < 64 && (uint64_t)(n_keys - 1) >> bits) ++bits;
        radix_sort_pairs(keys, perm, nnz, bits, s);
    }
    panel_first<<<grid_of_n(n_keys + 1), kB, 0, s>>>(keys.as<uint64_t>(), nnz, n_keys,
                                                     first.as<int32_t>());
    SPMV_CHECK_LAUNCH();
    panel_padded<<<grid_of_n(n_keys + 1), kB, 0, s>>>(first.as<int32_t>(), n_keys,
                                                      start.as<int32_t>());
    SPMV_CHECK_LAUNCH();
    exclusive_scan_i32(start.as<int32_t>(), start.as<int32_t>(), n_keys + 1, s);
    int32_t total = 0;
    SPMV_HIP(hipMemcpyAsync(&total, start.as<int32_t>() + n_keys, 4, hipMemcpyDeviceToHost, s));
    SPMV_HIP(hipStreamSynchronize(s));
    P.stream = total;

    const int64_t cap = padded_count(total);
    P.idx.alloc(cap * 4);
    P.val.alloc(cap * vs);
    SPMV_HIP(hipMemsetAsync(P.idx.p, 0xFF, cap * 4, s));  // kPanelPad
    SPMV_HIP(hipMemsetAsync(P.val.p, 0, cap * vs, s));
    if (nnz > 0) {
        if (h->dt == SPMV_F64)
            panel_scatter<double><<<grid_of_n(nnz), kB, 0, s>>>(
                keys.as<uint64_t>(), perm.as<uint32_t>(), nnz, h->row.as<int32_t>(),
                h->col.as<int32_t>(), h->val.as<double>(), first.as<int32_t>(), start.as<int32_t>(),
                P.rows_per_wave, width, P.idx.as<int32_t>(), P.val.as<double>());
        else
            panel_scatter<float><<<grid_of_n(nnz), kB, 0, s>>>(
                keys.as<uint64_t>(), perm.as<uint32_t>(), nnz, h->row.as<int32_t>(),
                h->col.as<int32_t>(), h->val.as<float>(), first.as<int32_t>(), start.as<int32_t>(),
                P.rows_per_wave, width, P.idx.as<int32_t>(), P.val.as<float>());
        SPMV_CHECK_LAUNCH();
    }
    P.run_ptr.alloc(std::max<int64_t>(groups * (P.panels + 1), 1) * 4);
    if (groups > 0) {
        panel_run_ptr<<<grid_of_n(groups * (P.panels + 1)), kB, 0, s>>>(
            start.as<int32_t>(), groups, P.panels, P.run_ptr.as<int32_t>());
        SPMV_CHECK_LAUNCH();
    }
    // per-block lists of the panels that hold entries
    const int64_t nf = (int64_t)P.blocks * P.panels;
    DevBuf flag;
    flag.alloc((nf + 1) * 4);
    panel_flags<<<grid_of_n(nf + 1), kB, 0, s>>>(first.as<int32_t>(), P.blocks, P.panels,
                                                 flag.as<int32_t>());
    SPMV_CHECK_LAUNCH();
    exclusive_scan_i32(flag.as<int32_t>(), flag.as<int32_t>(), nf + 1, s);
    int32_t listed = 0;
    SPMV_HIP(hipMemcpyAsync(&listed, flag.as<int32_t>() + nf, 4, hipMemcpyDeviceToHost, s));
    SPMV_HIP(hipStreamSynchronize(s));
    P.blk_panel.alloc(std::max<int64_t>(listed, 1) * 4);
    P.blk_ptr.alloc(((int64_t)P.blocks + 1) * 4);
    panel_lists<<<grid_of_n(std::max<int64_t>(nf, (int64_t)P.blocks + 1)), kB, 0, s>>>(
        flag.as<int32_t>(), P.blocks, P.panels, P.blk_panel.as<int32_t>(), P.blk_ptr.as<int32_t>());
    SPMV_CHECK_LAUNCH();
    SPMV_HIP(hipStreamSynchronize(s));
    P.built = true;
    h->panel = std::move(P);
}

void panel_spmv(const spmv_matrix_s *h, int items, double alpha, const void *x, double beta,
                void *y, hipStream_t s) {
    if (!h->panel.built) fail(SPMV_ERR_NOT_CONVERTED, "panel layout of COO not built");
    if (h->n_rows == 0) return;
    if (h->dt == SPMV_F64) {
        if (items == 2) launch_panel<double, 2>(h, alpha, x, beta, y, s);
        else launch_panel<double, 4>(h, alpha, x, beta, y, s);
    } else {
        if (items == 2) launch_panel<float, 2>(h, alpha, x, beta, y, s);
        else launch_panel<float, 4>(h, alpha, x, beta, y, s);
    }
}

}  // namespace spmv
