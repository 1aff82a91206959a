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

}  // namespace

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
