// CSR -> ELL and CSR -> HYB conversion on the device (paper, Background:
// ELL keeps an m x max_nnz data matrix and a matching column-index matrix;
// the run-time mode converts the input to the predicted format). HYB, an ELL
// part plus a COO tail, follows Bell and Garland (SC'09).
//
// Layout: slot (i, k) of a width-K ELL block sits at k * pitch + i with pitch =
// roundup(n_rows, 64), so a wavefront reading slot k of 64 consecutive rows
// touches one contiguous 256-byte (FP32) run. Padding slots hold column -1
// and value +0.0. Every array is a bit copy of the canonical CSR.
#include <algorithm>

#include "common.hpp"

namespace spmv {
namespace {

constexpr int kBlock = 256;
constexpr int64_t kEllFillCap = 8;  // padded ELL slots may be at most 8 * nnz

template <class V>
__global__ __launch_bounds__(kBlock) void ell_fill(int32_t n_rows, int32_t pitch, int32_t K,
                                                   const int32_t *__restrict__ rp,
                                                   const int32_t *__restrict__ col,
                                                   const V *__restrict__ val,
                                                   int32_t *__restrict__ ecol,
                                                   V *__restrict__ eval) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= pitch) return;
    int32_t s = 0, len = 0;
    if (i < n_rows) {
        s = rp[i];
        len = rp[i + 1] - s;
    }
    for (int64_t k = blockIdx.y; k < K; k += gridDim.y) {
        const int64_t slot = k * pitch + i;
        if (k < len) {
            ecol[slot] = col[s + k];
            eval[slot] = val[s + k];
        } else {
            ecol[slot] = -1;
            eval[slot] = V(0);
        }
    }
}

__global__ __launch_bounds__(kBlock) void tail_counts(int32_t n_rows, int32_t K,
                                                      const int32_t *__restrict__ rp,
                                                      int32_t *__restrict__ cnt) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n_rows) cnt[i] = max(0, rp[i + 1] - rp[i] - K);
    if (i == n_rows) cnt[i] = 0;
}

template <class V>
__global__ __launch_bounds__(kBlock) void tail_scatter(int64_t nnz, int32_t K,
                                                       const int32_t *__restrict__ row,
                                                       const int32_t *__restrict__ col,
                                                       const V *__restrict__ val,
                                                       const int32_t *__restrict__ rp,
                                                       const int32_t *__restrict__ off,
                                                       int32_t *__restrict__ trow,
                                                       int32_t *__restrict__ tcol,
                                                       V *__restrict__ tval) {
    for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < nnz;
         e += (int64_t)gridDim.x * kBlock) {
        const int32_t r = row[e];
        const int32_t k = (int32_t)(e - rp[r]);
        if (k >= K) {
            const int64_t pos = (int64_t)off[r] + (k - K);
            trow[pos] = r;
            tcol[pos] = col[e];
            tval[pos] = val[e];
        }
    }
}

void fill_ell(const spmv_matrix_s *h, int32_t K, int32_t pitch, DevBuf &ecol, DevBuf &eval,
              hipStream_t s) {
    const size_t vs = dtype_size(h->dt);
    ecol.alloc((int64_t)K * pitch * 4);
    eval.alloc((int64_t)K * pitch * vs);
    if (K == 0 || pitch == 0) return;
    dim3 grid((unsigned)ceil_div(pitch, kBlock), (unsigned)std::min<int64_t>(K, 65535));
    if (h->dt == SPMV_F64)
        ell_fill<double><<<grid, kBlock, 0, s>>>(h->n_rows, pitch, K, h->row_ptr.as<int32_t>(),
                                                 h->col.as<int32_t>(), h->val.as<double>(),
                                                 ecol.as<int32_t>(), eval.as<double>());
    else
        ell_fill<float><<<grid, kBlock, 0, s>>>(h->n_rows, pitch, K, h->row_ptr.as<int32_t>(),
                                                h->col.as<int32_t>(), h->val.as<float>(),
                                                ecol.as<int32_t>(), eval.as<float>());
    SPMV_CHECK_LAUNCH();
}

int32_t ell_pitch(int32_t n_rows) { return (int32_t)(ceil_div(n_rows, 64) * 64); }

int bit_length(uint64_t v) {
    int b = 0;
    while (b < 64 && (v >> b)) ++b;
    return b;
}

int grid_for(int64_t n, int64_t cap = 65536) {
    return (int)std::max<int64_t>(1, std::min<int64_t>(ceil_div(n, kBlock), cap));
}

// ---- SELL-C-sigma ----------------------------------------------------------------

// Width of every slice: one wavefront per slice takes the longest of its rows
// (perm[p] is the row at position p, or p itself when perm is NULL), rounded up
// to a whole number of 4-slot groups.
__global__ __launch_bounds__(kBlock) void sell_widths(int32_t n_rows, int32_t n_slices,
                                                      const int32_t *__restrict__ rp,
                                                      const int32_t *__restrict__ perm,
                                                      int32_t *__restrict__ width) {
    const int64_t sl = (int64_t)blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave;
    if (sl >= n_slices) return;
    const int lane = threadIdx.x % kWave;
    const int64_t p = sl * kSellSlice + lane;
    int32_t len = 0;
    if (p < n_rows) {
        const int32_t r = perm ? perm[p] : (int32_t)p;
        len = rp[r + 1] - rp[r];
    }
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) len = max(len, __shfl_xor(len, d, kWave));
    if (lane == 0) width[sl] = (len + kSellGroup - 1) / kSellGroup * kSellGroup;
}

// Keys ordering rows by window of sigma rows, then by descending length; the
// stable sort keeps row order among equal lengths.
__global__ __launch_bounds__(kBlock) void sell_order_keys(int32_t n_rows, int32_t sigma,
                                                          int32_t max_len, int len_bits,
                                                          const int32_t *__restrict__ rp,
                                                          uint64_t *__restrict__ keys,
                                                          uint32_t *__restrict__ payload) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n_rows;
         i += (int64_t)gridDim.x * kBlock) {
        const uint32_t len = (uint32_t)(rp[i + 1] - rp[i]);
        keys[i] = ((uint64_t)(i / sigma) << len_bits) | (uint64_t)((uint32_t)max_len - len);
        payload[i] = (uint32_t)i;
    }
}

__global__ __launch_bounds__(kBlock) void invert_order(int32_t n, const int32_t *__restrict__ perm,
                                                       int32_t *__restrict__ pos) {
    for (int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x; p < n; p += (int64_t)gridDim.x * kBlock)
        pos[perm[p]] = (int32_t)p;
}

template <class V>
__global__ __launch_bounds__(kBlock) void pad_slots(int64_t n, int32_t *__restrict__ c,
                                                    V *__restrict__ v) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
        c[i] = -1;
        v[i] = V(0);
    }
}

// Entry e of row r, the k-th of its row, goes to slot k of position pos[r].
template <class V>
__global__ __launch_bounds__(kBlock) void sell_scatter(int64_t nnz, const int32_t *__restrict__ row,
                                                       const int32_t *__restrict__ col,
                                                       const V *__restrict__ val,
                                                       const int32_t *__restrict__ rp,
                                                       const int32_t *__restrict__ pos,
                                                       const int64_t *__restrict__ slice_ptr,
                                                       int32_t *__restrict__ scol,
                                                       V *__restrict__ sval) {
    for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < nnz;
         e += (int64_t)gridDim.x * kBlock) {
        const int32_t r = row[e];
        const int64_t k = e - rp[r];
        const int64_t p = pos ? pos[r] : r;
        const int64_t slot = slice_ptr[p / kSellSlice] + (k / kSellGroup) * (kSellSlice * kSellGroup) +
                             (p % kSellSlice) * kSellGroup + k % kSellGroup;
        scol[slot] = col[e];
        sval[slot] = val[e];
    }
}

// ---- BELL ------------------------------------------------------------------------

__global__ __launch_bounds__(kBlock) void bell_keys(int64_t nnz, int32_t b, int64_t nbc,
                                                    const int32_t *__restrict__ row,
                                                    const int32_t *__restrict__ col,
                                                    uint64_t *__restrict__ keys,
                                                    uint32_t *__restrict__ payload) {
    for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < nnz;
         e += (int64_t)gridDim.x * kBlock) {
        keys[e] = (uint64_t)(row[e] / b) * (uint64_t)nbc + (uint64_t)(col[e] / b);
        payload[e] = (uint32_t)e;
    }
}

// 1 where a sorted key starts a new block
__global__ __launch_bounds__(kBlock) void bell_heads(int64_t n, const uint64_t *__restrict__ keys,
                                                     int32_t *__restrict__ head) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
        head[i] = (i == 0 || keys[i] != keys[i - 1]) ? 1 : 0;
}

// For every block (a head): its block row's first block id and block count.
__global__ __launch_bounds__(kBlock) void bell_rows(int64_t n, int64_t nbc,
                                                    const uint64_t *__restrict__ keys,
                                                    const int32_t *__restrict__ head,
                                                    const int32_t *__restrict__ before,
                                                    int32_t *__restrict__ first,
                                                    int32_t *__restrict__ count,
                                                    int32_t *__restrict__ kmax) {
    int32_t m = 0;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
        if (!head[i]) continue;
        const int64_t br = (int64_t)(keys[i] / (uint64_t)nbc);
        if (i == 0 || (int64_t)(keys[i - 1] / (uint64_t)nbc) != br) first[br] = before[i];
        const int32_t c = atomicAdd(&count[br], 1) + 1;
        m = max(m, c);
    }
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) m = max(m, __shfl_xor(m, d, kWave));
    if ((threadIdx.x & (kWave - 1)) == 0 && m > 0) atomicMax(kmax, m);
}

template <class V>
__global__ __launch_bounds__(kBlock) void bell_place(int64_t n, int32_t b, int64_t nbc, int32_t pitch,
                                                     const uint64_t *__restrict__ keys,
                                                     const uint32_t *__restrict__ payload,
                                                     const int32_t *__restrict__ head,
                                                     const int32_t *__restrict__ before,
                                                     const int32_t *__restrict__ first,
                                                     const int32_t *__restrict__ row,
                                                     const int32_t *__restrict__ col,
                                                     const V *__restrict__ val,
                                                     int32_t *__restrict__ bcol,
                                                     V *__restrict__ bval) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
        const int64_t br = (int64_t)(keys[i] / (uint64_t)nbc);
        const int32_t bc = (int32_t)(keys[i] % (uint64_t)nbc);
        const int32_t id = before[i] + head[i] - 1;  // block id of this entry
        const int64_t slot = (int64_t)(id - first[br]) * pitch + br;
        if (head[i]) bcol[slot] = bc;
        const uint32_t e = payload[i];
        bval[slot * b * b + (row[e] % b) * b + col[e] % b] = val[e];
    }
}

// Blocks of one size: the sorted block keys of every entry with their block ids,
// and the per-block-row first ids; K = most blocks in a block row.
struct BellBlocks {
    int32_t b = 0, K = 0, nbr = 0;
    int64_t nbc = 0;
    DevBuf keys, payload, head, before, first;
};

BellBlocks bell_blocks(const spmv_matrix_s *h, int32_t b, hipStream_t s) {
    BellBlocks B;
    B.b = b;
    B.nbr = (int32_t)ceil_div(h->n_rows, b);
    B.nbc = (int64_t)h->n_cols / b + 1;
    const int64_t n = h->nnz;
    if (n == 0) return B;
    B.keys.alloc(n * 8);
    B.payload.alloc(n * 4);
    bell_keys<<<grid_for(n), kBlock, 0, s>>>(n, b, B.nbc, h->row.as<int32_t>(), h->col.as<int32_t>(),
                                            B.keys.as<uint64_t>(), B.payload.as<uint32_t>());
    SPMV_CHECK_LAUNCH();
    radix_sort_pairs(B.keys, B.payload, n, bit_length((uint64_t)B.nbr * (uint64_t)B.nbc - 1), s);
    B.head.alloc(n * 4);
    B.before.alloc(n * 4);
    bell_heads<<<grid_for(n), kBlock, 0, s>>>(n, B.keys.as<uint64_t>(), B.head.as<int32_t>());
    SPMV_CHECK_LAUNCH();
    exclusive_scan_i32(B.head.as<int32_t>(), B.before.as<int32_t>(), n, s);
    B.first.alloc((int64_t)std::max(B.nbr, 1) * 4);
    DevBuf count, kmax;
    count.alloc((int64_t)std::max(B.nbr, 1) * 4);
    kmax.alloc(4);
    SPMV_HIP(hipMemsetAsync(count.p, 0, (int64_t)std::max(B.nbr, 1) * 4, s));
    SPMV_HIP(hipMemsetAsync(kmax.p, 0, 4, s));
    bell_rows<<<grid_for(n, 4096), kBlock, 0, s>>>(n, B.nbc, B.keys.as<uint64_t>(), B.head.as<int32_t>(),
                                                  B.before.as<int32_t>(), B.first.as<int32_t>(),
                                                  count.as<int32_t>(), kmax.as<int32_t>());
    SPMV_CHECK_LAUNCH();
    SPMV_HIP(hipMemcpyAsync(&B.K, kmax.p, 4, hipMemcpyDeviceToHost, s));
    SPMV_HIP(hipStreamSynchronize(s));
    return B;
}

bool bell_within_cap(const spmv_matrix_s *h, const BellBlocks &B) {
    const int64_t values = (int64_t)ell_pitch(B.nbr) * B.K * B.b * B.b;
    return h->nnz == 0 || values <= std::max<int64_t>(kEllFillCap * h->nnz, kSmallLayoutSlots);
}

}  // namespace

void build_sell(spmv_matrix_s *h, int32_t sigma_in, hipStream_t s) {
    if (sigma_in == 0 || (sigma_in > 1 && sigma_in % kSellSlice != 0))
        fail(SPMV_ERR_INVALID_ARG, "SELL sigma %d: 1, a positive multiple of %d, or < 0 for the rule",
             sigma_in, kSellSlice);
    const int32_t n = h->n_rows;
    const int32_t n_slices = (int32_t)ceil_div(n, kSellSlice);
    const size_t vs = dtype_size(h->dt);
    DevBuf width;
    width.alloc((int64_t)std::max(n_slices, 1) * 4);
    auto widths_of = [&](const int32_t *perm) {
        std::vector<int32_t> w(n_slices);
        if (n_slices == 0) return w;
        sell_widths<<<(int)ceil_div(n_slices, kBlock / kWave), kBlock, 0, s>>>(
            n, n_slices, h->row_ptr.as<int32_t>(), perm, width.as<int32_t>());
        SPMV_CHECK_LAUNCH();
        SPMV_HIP(hipMemcpyAsync(w.data(), width.p, (size_t)n_slices * 4, hipMemcpyDeviceToHost, s));
        SPMV_HIP(hipStreamSynchronize(s));
        return w;
    };
    auto order_of = [&](int32_t sigma, DevBuf &perm) {
        DevBuf keys;
        keys.alloc((int64_t)std::max(n, 1) * 8);
        perm.alloc((int64_t)std::max(n, 1) * 4);
        const int len_bits = bit_length((uint64_t)h->stats.max_len);
        sell_order_keys<<<grid_for(n), kBlock, 0, s>>>(n, sigma, h->stats.max_len, len_bits,
                                                       h->row_ptr.as<int32_t>(), keys.as<uint64_t>(),
                                                       perm.as<uint32_t>());
        SPMV_CHECK_LAUNCH();
        const int bits = len_bits + bit_length((uint64_t)(n > 0 ? (n - 1) / sigma : 0));
        radix_sort_pairs(keys, perm, n, bits, s);  // synchronises
    };
    auto total = [](const std::vector<int32_t> &w) {
        int64_t t = 0;
        for (int32_t x : w) t += x;
        return t * kSellSlice;
    };
    SellPart P;
    std::vector<int32_t> w;
    if (sigma_in == 1 || n == 0) {
        P.sigma = sigma_in < 0 ? 1 : sigma_in;  // with no rows every order is the same
        w = widths_of(nullptr);
    } else {
        const int32_t sig = sigma_in < 0 ? kSellSigmaWide : sigma_in;
        DevBuf perm;
        order_of(sig, perm);
        std::vector<int32_t> ws = widths_of(perm.as<int32_t>());
        if (sigma_in < 0) {
            std::vector<int32_t> w1 = widths_of(nullptr);
            const int64_t b1 = total(w1) * (int64_t)(4 + vs);
            const int64_t b2 = total(ws) * (int64_t)(4 + vs) + 4 * (int64_t)n;
            if (b2 < b1) { P.sigma = sig; w = ws; P.perm = std::move(perm); }
            else { P.sigma = 1; w = w1; }
        } else {
            P.sigma = sig;
            w = ws;
            P.perm = std::move(perm);
        }
    }
    P.n_slices = n_slices;
    P.slots = total(w);
    if (h->nnz > 0 && P.slots > std::max<int64_t>(kEllFillCap * h->nnz, kSmallLayoutSlots))
        fail(SPMV_ERR_NOT_APPLICABLE, "SELL would hold %lld slots for %lld entries",
             (long long)P.slots, (long long)h->nnz);
    P.host_ptr.assign(n_slices + 1, 0);
    for (int32_t i = 0; i < n_slices; ++i) P.host_ptr[i + 1] = P.host_ptr[i] + (int64_t)w[i] * kSellSlice;
    P.slice_ptr.alloc((int64_t)(n_slices + 1) * 8);
    SPMV_HIP(hipMemcpyAsync(P.slice_ptr.p, P.host_ptr.data(), (size_t)(n_slices + 1) * 8,
                            hipMemcpyHostToDevice, s));
    P.col.alloc(std::max<int64_t>(P.slots, kSellSlice * kSellGroup) * 4);
    P.val.alloc(std::max<int64_t>(P.slots, kSellSlice * kSellGroup) * vs);
    DevBuf pos;
    if (P.sigma > 1) {
        pos.alloc((int64_t)std::max(n, 1) * 4);
        invert_order<<<grid_for(n), kBlock, 0, s>>>(n, P.perm.as<int32_t>(), pos.as<int32_t>());
        SPMV_CHECK_LAUNCH();
    }
    if (P.slots > 0) {
        if (h->dt == SPMV_F64) {
            pad_slots<double><<<grid_for(P.slots), kBlock, 0, s>>>(P.slots, P.col.as<int32_t>(), P.val.as<double>());
            SPMV_CHECK_LAUNCH();
            if (h->nnz > 0)
                sell_scatter<double><<<grid_for(h->nnz), kBlock, 0, s>>>(
                    h->nnz, h->row.as<int32_t>(), h->col.as<int32_t>(), h->val.as<double>(),
                    h->row_ptr.as<int32_t>(), pos.as<int32_t>(), P.slice_ptr.as<int64_t>(),
                    P.col.as<int32_t>(), P.val.as<double>());
        } else {
            pad_slots<float><<<grid_for(P.slots), kBlock, 0, s>>>(P.slots, P.col.as<int32_t>(), P.val.as<float>());
            SPMV_CHECK_LAUNCH();
            if (h->nnz > 0)
                sell_scatter<float><<<grid_for(h->nnz), kBlock, 0, s>>>(
                    h->nnz, h->row.as<int32_t>(), h->col.as<int32_t>(), h->val.as<float>(),
                    h->row_ptr.as<int32_t>(), pos.as<int32_t>(), P.slice_ptr.as<int64_t>(),
                    P.col.as<int32_t>(), P.val.as<float>());
        }
        SPMV_CHECK_LAUNCH();
    }
    SPMV_HIP(hipStreamSynchronize(s));
    P.built = true;
    h->sell = std::move(P);
}

void build_bell(spmv_matrix_s *h, int32_t b_in, hipStream_t s) {
    if (b_in >= 0 && b_in != 2 && b_in != 4 && b_in != 8)
        fail(SPMV_ERR_INVALID_ARG, "BELL block size %d: 2, 4, 8, or < 0 for the rule", b_in);
    const size_t vs = dtype_size(h->dt);
    BellBlocks best;
    if (b_in > 0) {
        best = bell_blocks(h, b_in, s);
    } else {
        int64_t best_bytes = -1;
        for (int32_t b : {2, 4, 8}) {
            BellBlocks B = bell_blocks(h, b, s);
            if (!bell_within_cap(h, B)) continue;
            const int64_t bytes = (int64_t)ell_pitch(B.nbr) * B.K * (int64_t)(4 + (int64_t)b * b * vs);
            if (best_bytes < 0 || bytes < best_bytes) { best_bytes = bytes; best = std::move(B); }
        }
        if (best_bytes < 0) best = bell_blocks(h, 2, s);
    }
    if (!bell_within_cap(h, best))
        fail(SPMV_ERR_NOT_APPLICABLE, "BELL %dx%d would hold %lld values for %lld entries", best.b,
             best.b, (long long)ell_pitch(best.nbr) * best.K * best.b * best.b, (long long)h->nnz);
    BellPart P;
    P.b = best.b;
    P.K = h->nnz > 0 ? best.K : 0;
    P.n_block_rows = best.nbr;
    P.pitch = ell_pitch(best.nbr);
    const int64_t slots = (int64_t)P.K * P.pitch;
    const int64_t values = slots * P.b * P.b;
    P.col.alloc(slots * 4);
    P.val.alloc(values * vs);
    if (slots > 0) {
        const int64_t n = h->nnz;
        if (h->dt == SPMV_F64) {
            pad_slots<double><<<grid_for(slots), kBlock, 0, s>>>(slots, P.col.as<int32_t>(), P.val.as<double>());
            SPMV_CHECK_LAUNCH();
            SPMV_HIP(hipMemsetAsync(P.val.p, 0, values * vs, s));
            bell_place<double><<<grid_for(n), kBlock, 0, s>>>(
                n, P.b, best.nbc, P.pitch, best.keys.as<uint64_t>(), best.payload.as<uint32_t>(),
                best.head.as<int32_t>(), best.before.as<int32_t>(), best.first.as<int32_t>(),
                h->row.as<int32_t>(), h->col.as<int32_t>(), h->val.as<double>(), P.col.as<int32_t>(),
                P.val.as<double>());
        } else {
            pad_slots<float><<<grid_for(slots), kBlock, 0, s>>>(slots, P.col.as<int32_t>(), P.val.as<float>());
            SPMV_CHECK_LAUNCH();
            SPMV_HIP(hipMemsetAsync(P.val.p, 0, values * vs, s));
            bell_place<float><<<grid_for(n), kBlock, 0, s>>>(
                n, P.b, best.nbc, P.pitch, best.keys.as<uint64_t>(), best.payload.as<uint32_t>(),
                best.head.as<int32_t>(), best.before.as<int32_t>(), best.first.as<int32_t>(),
                h->row.as<int32_t>(), h->col.as<int32_t>(), h->val.as<float>(), P.col.as<int32_t>(),
                P.val.as<float>());
        }
        SPMV_CHECK_LAUNCH();
    }
    SPMV_HIP(hipStreamSynchronize(s));
    P.built = true;
    h->bell = std::move(P);
}

void build_ell(spmv_matrix_s *h, hipStream_t s) {
    const int32_t K = h->stats.max_len;
    const int32_t pitch = ell_pitch(h->n_rows);
    if (h->nnz > 0 && (int64_t)pitch * K > kEllFillCap * h->nnz)
        fail(SPMV_ERR_NOT_APPLICABLE, "ELL would hold %lld slots for %lld entries",
             (long long)pitch * K, (long long)h->nnz);
    EllPart e;
    e.K = h->nnz > 0 ? K : 0;
    e.pitch = pitch;
    fill_ell(h, e.K, pitch, e.col, e.val, s);
    SPMV_HIP(hipStreamSynchronize(s));
    e.built = true;
    h->ell = std::move(e);
}

void build_hyb(spmv_matrix_s *h, int32_t hyb_k, hipStream_t s) {
    const int32_t K = hyb_k >= 0 ? hyb_k : hyb_rule_width(h, s);
    HybPart p;
    p.K = K;
    p.pitch = ell_pitch(h->n_rows);
    fill_ell(h, K, p.pitch, p.ell_col, p.ell_val, s);
    // COO tail: entries at position >= K of their row, in canonical order.
    DevBuf off;
    off.alloc(((int64_t)h->n_rows + 1) * 4);
    tail_counts<<<(unsigned)ceil_div((int64_t)h->n_rows + 1, kBlock), kBlock, 0, s>>>(
        h->n_rows, K, h->row_ptr.as<int32_t>(), off.as<int32_t>());
    SPMV_CHECK_LAUNCH();
    exclusive_scan_i32(off.as<int32_t>(), off.as<int32_t>(), (int64_t)h->n_rows + 1, s);
    int32_t total = 0;
    SPMV_HIP(hipMemcpyAsync(&total, off.as<int32_t>() + h->n_rows, 4, hipMemcpyDeviceToHost, s));
    SPMV_HIP(hipStreamSynchronize(s));
    p.nnz_tail = total;
    const size_t vs = dtype_size(h->dt);
    const int64_t tp = padded_count(total);
    p.tail_row.alloc(tp * 4);
    p.tail_col.alloc(tp * 4);
    p.tail_val.alloc(tp * vs);
    if (tp > total) {
        SPMV_HIP(hipMemsetAsync(p.tail_row.as<int32_t>() + total, 0, (tp - total) * 4, s));
        SPMV_HIP(hipMemsetAsync(p.tail_col.as<int32_t>() + total, 0, (tp - total) * 4, s));
        SPMV_HIP(hipMemsetAsync((char *)p.tail_val.p + total * vs, 0, (tp - total) * vs, s));
    }
    p.partials.alloc(coo_partials_bytes(total, h->dt));
    if (total > 0) {
        const int grid = (int)std::min<int64_t>(ceil_div(h->nnz, kBlock), 65536);
        if (h->dt == SPMV_F64)
            tail_scatter<double><<<grid, kBlock, 0, s>>>(
                h->nnz, K, h->row.as<int32_t>(), h->col.as<int32_t>(), h->val.as<double>(),
                h->row_ptr.as<int32_t>(), off.as<int32_t>(), p.tail_row.as<int32_t>(),
                p.tail_col.as<int32_t>(), p.tail_val.as<double>());
        else
            tail_scatter<float><<<grid, kBlock, 0, s>>>(
                h->nnz, K, h->row.as<int32_t>(), h->col.as<int32_t>(), h->val.as<float>(),
                h->row_ptr.as<int32_t>(), off.as<int32_t>(), p.tail_row.as<int32_t>(),
                p.tail_col.as<int32_t>(), p.tail_val.as<float>());
        SPMV_CHECK_LAUNCH();
    }
    SPMV_HIP(hipStreamSynchronize(s));
    p.tail_ptr = std::move(off);  // the exclusive scan: the tail's row pointers
    p.built = true;
    h->hyb = std::move(p);
    h->hyb_sorted = SortedPart{};  // a copy of the previous tail is stale
}

}  // namespace spmv
