// Sparsity features on the device (paper, Method: sparsity features table:
// n, nnz, average, variance, ELL ratio, median, mode and standard deviation of
// the row lengths), extended with the longest row, the bandwidth, the fill
// and the HYB tail fraction.
//
// Everything derives from one histogram of row lengths: the median and the
// Bell-Garland HYB width are order statistics read off its prefix sums, the
// mode is its arg-max, and the tail size is a weighted sum over its bins.
// Integer statistics are exact; the moments are formed in FP64 from the
// exact integer sums.
#include <algorithm>
#include <mutex>

#include "common.hpp"

namespace spmv {
namespace {

constexpr int kBlock = 256;
constexpr int kLdsBins = 8192;  // bins kept per workgroup in LDS; longer rows go to global

struct Stats {
    unsigned long long sum_sq;    // sum of len^2
    unsigned long long mode_key;  // (count << 32) | (0xffffffff - len): max = mode, smallest len
    unsigned long long tail;      // sum over rows of max(0, len - K_h)
    int32_t median_lo, median_hi, hyb_width, bandwidth;
};

__global__ __launch_bounds__(kBlock) void length_histogram(int32_t n_rows,
                                                           const int32_t *__restrict__ rp,
                                                           int32_t n_bins,
                                                           int32_t *__restrict__ hist,
                                                           Stats *__restrict__ st) {
    __shared__ int32_t s_hist[kLdsBins];
    __shared__ unsigned long long s_sq[kBlock / kWave];
    const int lds_bins = min(n_bins, kLdsBins);
    for (int b = threadIdx.x; b < lds_bins; b += kBlock) s_hist[b] = 0;
    __syncthreads();
    unsigned long long sq = 0;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n_rows;
         i += (int64_t)gridDim.x * kBlock) {
        const int32_t len = rp[i + 1] - rp[i];
        sq += (unsigned long long)len * (unsigned long long)len;
        if (len < lds_bins) atomicAdd(&s_hist[len], 1);
        else atomicAdd(&hist[len], 1);
    }
    for (int d = kWave / 2; d > 0; d >>= 1) sq += __shfl_xor(sq, d, kWave);
    if ((threadIdx.x & (kWave - 1)) == 0) s_sq[threadIdx.x / kWave] = sq;
    __syncthreads();
    for (int b = threadIdx.x; b < lds_bins; b += kBlock)
        if (s_hist[b]) atomicAdd(&hist[b], s_hist[b]);
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int w = 0; w < kBlock / kWave; ++w) t += s_sq[w];
        if (t) atomicAdd(&st->sum_sq, t);
    }
}

// For each bin l, rows ranked cum[l] .. cum[l] + hist[l] - 1 (ascending length)
// have length l. Exactly one bin holds each requested rank.
__global__ __launch_bounds__(kBlock) void order_statistics(int32_t n_bins,
                                                           const int32_t *__restrict__ hist,
                                                           const int32_t *__restrict__ cum,
                                                           int64_t rank_lo, int64_t rank_hi,
                                                           int64_t rank_hyb,
                                                           Stats *__restrict__ st) {
    unsigned long long best = 0;
    for (int64_t l = (int64_t)blockIdx.x * kBlock + threadIdx.x; l < n_bins;
         l += (int64_t)gridDim.x * kBlock) {
        const int64_t c = hist[l];
        if (c == 0) continue;
        const int64_t a = cum[l];
        if (a <= rank_lo && rank_lo < a + c) st->median_lo = (int32_t)l;
        if (a <= rank_hi && rank_hi < a + c) st->median_hi = (int32_t)l;
        if (rank_hyb >= 0 && a <= rank_hyb && rank_hyb < a + c) st->hyb_width = (int32_t)l;
        const unsigned long long key =
            ((unsigned long long)c << 32) | (unsigned long long)(0xffffffffu - (uint32_t)l);
        best = key > best ? key : best;
    }
    for (int d = kWave / 2; d > 0; d >>= 1) {
        unsigned long long o = __shfl_xor(best, d, kWave);
        best = o > best ? o : best;
    }
    if ((threadIdx.x & (kWave - 1)) == 0 && best) atomicMax(&st->mode_key, best);
}

__global__ __launch_bounds__(kBlock) void tail_size(int32_t n_bins, const int32_t *__restrict__ hist,
                                                    Stats *__restrict__ st) {
    const int32_t K = st->hyb_width;
    unsigned long long t = 0;
    for (int64_t l = (int64_t)blockIdx.x * kBlock + threadIdx.x; l < n_bins;
         l += (int64_t)gridDim.x * kBlock)
        if (l > K) t += (unsigned long long)hist[l] * (unsigned long long)(l - K);
    for (int d = kWave / 2; d > 0; d >>= 1) t += __shfl_xor(t, d, kWave);
    if ((threadIdx.x & (kWave - 1)) == 0 && t) atomicAdd(&st->tail, t);
}

__global__ __launch_bounds__(kBlock) void bandwidth_kernel(int64_t nnz,
                                                           const int32_t *__restrict__ row,
                                                           const int32_t *__restrict__ col,
                                                           Stats *__restrict__ st) {
    int32_t m = 0;
    for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < nnz;
         k += (int64_t)gridDim.x * kBlock)
        m = max(m, abs(row[k] - col[k]));
    for (int d = kWave / 2; d > 0; d >>= 1) m = max(m, __shfl_xor(m, d, kWave));
    if ((threadIdx.x & (kWave - 1)) == 0 && m > 0) atomicMax(&st->bandwidth, m);
}

__global__ void assemble_features(int32_t n, int32_t n_cols, int64_t nnz, int32_t max_len,
                                  const Stats *__restrict__ st, float *__restrict__ out,
                                  int32_t *__restrict__ hyb_width_out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double f[12];
    for (int i = 0; i < 12; ++i) f[i] = 0.0;
    f[0] = n;
    f[1] = (double)nnz;
    if (n > 0) {
        const double mean = (double)nnz / n;
        double var = (double)st->sum_sq / n - mean * mean;
        var = var < 0.0 ? 0.0 : var;
        f[2] = mean;
        f[3] = var;
        f[4] = sqrt(var);
        f[5] = 0.5 * ((double)st->median_lo + (double)st->median_hi);
        f[6] = (double)(0xffffffffu - (uint32_t)(st->mode_key & 0xffffffffull));
        f[7] = max_len > 0 ? (double)nnz / ((double)n * max_len) : 0.0;
        f[8] = max_len;
        if (nnz > 0) {
            f[9] = st->bandwidth;
            f[11] = (double)st->tail / (double)nnz;
        }
        f[10] = n_cols > 0 ? (double)nnz / ((double)n * (double)n_cols) : 0.0;
    }
    for (int i = 0; i < 12; ++i) out[i] = (float)f[i];
    *hyb_width_out = n > 0 ? st->hyb_width : 0;
}

// Rows needed for the HYB ELL part: T = min(n, max(4096, ceil(n / 3))).
int64_t hyb_rows(int64_t n) { return std::min<int64_t>(n, std::max<int64_t>(4096, (n + 2) / 3)); }

struct FeatureRun {
    float feats[12];
    int32_t hyb_width;
};

// Device memory one feature run works in: the histogram and its prefix sums
// (n_bins each), the scan's tile sums, the statistics and the 13-word result.
struct FeatureWork {
    int32_t *hist, *cum, *sums;
    int64_t sums_cap;
    Stats *st;
    float *out;  // 12 features, then the HYB width as an int32
};

__global__ __launch_bounds__(kBlock) void zero_words(int64_t n, uint32_t *__restrict__ p) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
        p[i] = 0u;
}

// Clears the histogram and the statistics with a fill kernel (no memset node
// lands in a caller's graph), then runs the feature kernels and copies the
// result to the host (synchronises). `ws` selects the scan with caller-given
// tile sums; otherwise the scan allocates its own.
FeatureRun run_features_in(spmv_matrix_s *h, const FeatureWork &w, bool ws, hipStream_t s) {
    const int32_t n = h->n_rows;
    const int32_t n_bins = h->stats.max_len + 1;
    zero_words<<<(int)std::min<int64_t>(ceil_div(n_bins, kBlock), 1024), kBlock, 0, s>>>(
        n_bins, (uint32_t *)w.hist);
    SPMV_CHECK_LAUNCH();
    static_assert(sizeof(Stats) % 4 == 0, "Stats is cleared as words");
    zero_words<<<1, kBlock, 0, s>>>(sizeof(Stats) / 4, (uint32_t *)w.st);
    SPMV_CHECK_LAUNCH();
    if (n > 0) {
        const int g = (int)std::min<int64_t>(ceil_div(n, kBlock), 1024);
        length_histogram<<<g, kBlock, 0, s>>>(n, h->row_ptr.as<int32_t>(), n_bins, w.hist, w.st);
        SPMV_CHECK_LAUNCH();
        if (ws) exclusive_scan_i32_ws(w.hist, w.cum, n_bins, w.sums, w.sums_cap, s);
        else exclusive_scan_i32(w.hist, w.cum, n_bins, s);
        const int gb = (int)std::min<int64_t>(ceil_div(n_bins, kBlock), 1024);
        order_statistics<<<gb, kBlock, 0, s>>>(n_bins, w.hist, w.cum, (n - 1) / 2, n / 2,
                                               n - hyb_rows(n), w.st);
        SPMV_CHECK_LAUNCH();
        tail_size<<<gb, kBlock, 0, s>>>(n_bins, w.hist, w.st);
        SPMV_CHECK_LAUNCH();
        if (h->nnz > 0) {
            const int ge = (int)std::min<int64_t>(ceil_div(h->nnz, kBlock), 2048);
            bandwidth_kernel<<<ge, kBlock, 0, s>>>(h->nnz, h->row.as<int32_t>(),
                                                   h->col.as<int32_t>(), w.st);
            SPMV_CHECK_LAUNCH();
        }
    }
    assemble_features<<<1, 64, 0, s>>>(n, h->n_cols, h->nnz, h->stats.max_len, w.st, w.out,
                                       (int32_t *)(w.out + 12));
    SPMV_CHECK_LAUNCH();
    FeatureRun r;
    SPMV_HIP(hipMemcpyAsync(r.feats, w.out, 12 * sizeof(float), hipMemcpyDeviceToHost, s));
    SPMV_HIP(hipMemcpyAsync(&r.hyb_width, w.out + 12, 4, hipMemcpyDeviceToHost, s));
    SPMV_HIP(hipStreamSynchronize(s));
    return r;
}

FeatureRun run_features(spmv_matrix_s *h, hipStream_t s) {
    const int32_t n_bins = h->stats.max_len + 1;
    DevBuf hist, cum, st, out;
    hist.alloc((int64_t)n_bins * 4);
    cum.alloc((int64_t)n_bins * 4);
    st.alloc(sizeof(Stats));
    out.alloc(12 * sizeof(float) + sizeof(int32_t));
    const FeatureWork w{hist.as<int32_t>(), cum.as<int32_t>(), nullptr, 0, st.as<Stats>(),
                        out.as<float>()};
    return run_features_in(h, w, false, s);
}

// ---- the allocation-free variant -------------------------------------------------
//
// One file-scope device array serves every call on a device: histogram and
// prefix sums of up to kNoAllocBins bins, the scan's tile sums, the statistics
// and the result. Host code reaches it only through the address
// hipGetSymbolAddress returns for the current device.

constexpr int64_t kNoAllocBins = SPMV_FEATURES_NOALLOC_MAX_LEN + 1;
constexpr int64_t kScanTile = 2048;  // elements per scan tile (the scan's workgroup tile)
constexpr int64_t kNoAllocSums = (kNoAllocBins + kScanTile - 1) / kScanTile;
constexpr int64_t align256(int64_t b) { return (b + 255) / 256 * 256; }
constexpr int64_t kOffHist = 0;
constexpr int64_t kOffCum = kOffHist + align256(kNoAllocBins * 4);
constexpr int64_t kOffSums = kOffCum + align256(kNoAllocBins * 4);
constexpr int64_t kOffStats = kOffSums + align256(kNoAllocSums * 4);
constexpr int64_t kOffOut = kOffStats + align256(sizeof(Stats));
constexpr int64_t kScratchBytes = kOffOut + align256(13 * 4);
static_assert(kNoAllocSums <= kScanTile, "two-level scan");

__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per device.
unsigned char *scratch_on_current_device() {
    int dev = 0;
    SPMV_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) fail(SPMV_ERR_INVALID_ARG, "device %d beyond %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        SPMV_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) fail(SPMV_ERR_HIP, "no device address for the feature scratch array");
        g_scratch_ptr[dev] = p;
    }
    return (unsigned char *)g_scratch_ptr[dev];
}

}  // namespace

void compute_features(spmv_matrix_s *h, float out[12], int32_t *hyb_width, hipStream_t s) {
    FeatureRun r = run_features(h, s);
    for (int i = 0; i < 12; ++i) out[i] = r.feats[i];
    if (hyb_width) *hyb_width = r.hyb_width;
}

int32_t hyb_rule_width(spmv_matrix_s *h, hipStream_t s) { return run_features(h, s).hyb_width; }

void compute_features_noalloc(spmv_matrix_s *h, float out[12], hipStream_t s) {
    if ((int64_t)h->stats.max_len + 1 > kNoAllocBins)
        fail(SPMV_ERR_INVALID_ARG,
             "longest row has %d entries; the allocation-free feature call takes at most %d",
             h->stats.max_len, SPMV_FEATURES_NOALLOC_MAX_LEN);
    unsigned char *base = scratch_on_current_device();
    const FeatureWork w{(int32_t *)(base + kOffHist), (int32_t *)(base + kOffCum),
                        (int32_t *)(base + kOffSums), kNoAllocSums, (Stats *)(base + kOffStats),
                        (float *)(base + kOffOut)};
    const FeatureRun r = run_features_in(h, w, true, s);
    for (int i = 0; i < 12; ++i) out[i] = r.feats[i];
}

}  // namespace spmv
