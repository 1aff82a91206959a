// Learned format selector: a 12-64-64-4 ReLU network over the sparsity
// features (paper, Method: predicting optimal configuration parameters -- a
// multi-class classifier over the features; Setup, learning algorithms: an
// MLP trained with ReLU, Adam, learning rate 0.001 and 200 epochs).
//
// One wavefront evaluates one sample: lane j owns hidden unit j of both hidden
// layers, so every weight row maps onto the 64 lanes. The weights live in LDS,
// W2 both row-major (for the backward product W2^T * delta) and transposed
// (for the forward product W2 * h1), so both products read consecutive banks.
// Training runs every epoch in one launch of one workgroup: per minibatch each
// wave accumulates the gradient of its samples in registers, the waves add
// theirs into LDS in a fixed order (deterministic), and the threads apply Adam
// (Kingma and Ba, Algorithm 1) to the parameters in place.
//
// Parameter layout (floats): W1[64][12] b1[64] W2[64][64] b2[64] W3[4][64] b3[4]
// (5252 values), followed by the input standardisation mean[12] and std[12].
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "common.hpp"

namespace spmv {
namespace {

constexpr int kIn = 12, kH = 64, kOut = 4;
constexpr int oW1 = 0, oB1 = oW1 + kH * kIn, oW2 = oB1 + kH, oB2 = oW2 + kH * kH,
              oW3 = oB2 + kH, oB3 = oW3 + kOut * kH, kParams = oB3 + kOut;  // 5252
constexpr int oMean = kParams, oStd = kParams + kIn, kModel = kParams + 2 * kIn;  // 5276
static_assert(kParams == 5252 && kModel == 5276, "parameter layout");
constexpr int kWaves = 8;
constexpr int kThreads = kWaves * kWave;
constexpr float kStdFloor = 1e-6f;

// Feature columns that enter as log2(1 + v): counts and lengths (n, nnz, mean,
// var, std, median, mode, max, bandwidth); ratios stay raw.
__device__ __forceinline__ bool log_feature(int i) { return i <= 6 || i == 8 || i == 9; }

struct Net {
    float W1T[kIn][kH];  // W1 transposed: [input][unit]
    float b1[kH];
    float W2[kH][kH];    // [unit of layer 2][unit of layer 1]
    float W2T[kH][kH];   // [unit of layer 1][unit of layer 2]
    float b2[kH];
    float W3[kOut][kH];
    float b3[kOut];
};

__device__ void load_net(Net &n, const float *__restrict__ p) {
    for (int t = threadIdx.x; t < kParams; t += blockDim.x) {
        const float w = p[t];
        if (t < oB1) { int j = t / kIn, i = t % kIn; n.W1T[i][j] = w; }
        else if (t < oW2) n.b1[t - oB1] = w;
        else if (t < oB2) { int q = t - oW2, j = q / kH, k = q % kH; n.W2[j][k] = w; n.W2T[k][j] = w; }
        else if (t < oW3) n.b2[t - oB2] = w;
        else if (t < oB3) { int q = t - oW3; n.W3[q / kH][q % kH] = w; }
        else n.b3[t - oB3] = w;
    }
}

__device__ __forceinline__ void store_param(Net &n, int t, float w) {
    if (t < oB1) { int j = t / kIn, i = t % kIn; n.W1T[i][j] = w; }
    else if (t < oW2) n.b1[t - oB1] = w;
    else if (t < oB2) { int q = t - oW2, j = q / kH, k = q % kH; n.W2[j][k] = w; n.W2T[k][j] = w; }
    else if (t < oW3) n.b2[t - oB2] = w;
    else if (t < oB3) { int q = t - oW3; n.W3[q / kH][q % kH] = w; }
    else n.b3[t - oB3] = w;
}

__device__ __forceinline__ float param_of(const Net &n, int t) {
    if (t < oB1) return n.W1T[t % kIn][t / kIn];
    if (t < oW2) return n.b1[t - oB1];
    if (t < oB2) { int q = t - oW2; return n.W2[q / kH][q % kH]; }
    if (t < oW3) return n.b2[t - oB2];
    if (t < oB3) { int q = t - oW3; return n.W3[q / kH][q % kH]; }
    return n.b3[t - oB3];
}

__device__ __forceinline__ bool is_weight(int t) {
    return t < oB1 || (t >= oW2 && t < oB2) || (t >= oW3 && t < oB3);
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

struct Forward {
    float z[kIn];
    float a1, a2, h2;
    float logits[kOut];
};

// Forward pass of one sample by one wave; h1 of all lanes is left in sh1.
__device__ void forward(const Net &n, const float *__restrict__ zin, float *sh1, Forward &f) {
    const int j = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int i = 0; i < kIn; ++i) f.z[i] = zin[i];
    float a = n.b1[j];
#pragma unroll
    for (int i = 0; i < kIn; ++i) a += n.W1T[i][j] * f.z[i];
    f.a1 = a;
    sh1[j] = fmaxf(a, 0.f);
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    float b = n.b2[j];
#pragma unroll 8
    for (int k = 0; k < kH; ++k) b += n.W2T[k][j] * sh1[k];
    f.a2 = b;
    f.h2 = fmaxf(b, 0.f);
#pragma unroll
    for (int c = 0; c < kOut; ++c) f.logits[c] = wave_sum(n.W3[c][j] * f.h2) + n.b3[c];
}

// Gradient accumulators of one wave (lane j holds row j of every weight matrix).
struct Grad {
    float dW1[kIn];
    float db1;
    float dW2[kH];
    float db2;
    float dW3[kOut];
    float db3[kOut];
    float loss;
};

__device__ void zero_grad(Grad &g) {
#pragma unroll
    for (int i = 0; i < kIn; ++i) g.dW1[i] = 0.f;
#pragma unroll
    for (int k = 0; k < kH; ++k) g.dW2[k] = 0.f;
#pragma unroll
    for (int c = 0; c < kOut; ++c) { g.dW3[c] = 0.f; g.db3[c] = 0.f; }
    g.db1 = g.db2 = g.loss = 0.f;
}

// Adds one sample's cross-entropy gradient, scaled by inv_b, to g. Inactive
// waves pass valid = false and only take part in the lockstep LDS traffic.
__device__ void backward(const Net &n, const Forward &f, int label, float inv_b, bool valid,
                         const float *sh1, float *sda, Grad &g) {
    const int j = threadIdx.x & (kWave - 1);
    float mx = f.logits[0];
#pragma unroll
    for (int c = 1; c < kOut; ++c) mx = fmaxf(mx, f.logits[c]);
    float e[kOut], se = 0.f;
#pragma unroll
    for (int c = 0; c < kOut; ++c) { e[c] = expf(f.logits[c] - mx); se += e[c]; }
    float dz[kOut];
#pragma unroll
    for (int c = 0; c < kOut; ++c) dz[c] = valid ? (e[c] / se - (c == label ? 1.f : 0.f)) * inv_b : 0.f;
    float picked = 0.f;  // logit of the label, selected without a dynamic register index
#pragma unroll
    for (int c = 0; c < kOut; ++c) picked = (c == label) ? f.logits[c] : picked;
    if (valid) g.loss += (logf(se) + mx - picked) * inv_b;
    float dh2 = 0.f;
#pragma unroll
    for (int c = 0; c < kOut; ++c) {
        g.dW3[c] += dz[c] * f.h2;
        g.db3[c] += dz[c];
        dh2 += n.W3[c][j] * dz[c];
    }
    const float da2 = f.a2 > 0.f ? dh2 : 0.f;
    g.db2 += da2;
#pragma unroll
    for (int k = 0; k < kH; ++k) g.dW2[k] += da2 * sh1[k];
    sda[j] = da2;
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    float dh1 = 0.f;
#pragma unroll 8
    for (int q = 0; q < kH; ++q) dh1 += n.W2[q][j] * sda[q];
    const float da1 = f.a1 > 0.f ? dh1 : 0.f;
    g.db1 += da1;
#pragma unroll
    for (int i = 0; i < kIn; ++i) g.dW1[i] += da1 * f.z[i];
}

// Waves add their accumulators into grad[] one after another (fixed order).
__device__ void reduce_grad(const Grad &g, float *grad, float *loss_acc) {
    const int j = threadIdx.x & (kWave - 1);
    const int w = threadIdx.x / kWave;
    for (int t = threadIdx.x; t < kParams; t += blockDim.x) grad[t] = 0.f;
    if (threadIdx.x == 0) *loss_acc = 0.f;
    __syncthreads();
    for (int turn = 0; turn < kWaves; ++turn) {
        if (w == turn) {
#pragma unroll
            for (int i = 0; i < kIn; ++i) grad[oW1 + j * kIn + i] += g.dW1[i];
            grad[oB1 + j] += g.db1;
#pragma unroll
            for (int k = 0; k < kH; ++k) grad[oW2 + j * kH + k] += g.dW2[k];
            grad[oB2 + j] += g.db2;
#pragma unroll
            for (int c = 0; c < kOut; ++c) grad[oW3 + c * kH + j] += g.dW3[c];
            if (j == 0) {
#pragma unroll
                for (int c = 0; c < kOut; ++c) grad[oB3 + c] += g.db3[c];
                *loss_acc += g.loss;
            }
        }
        __syncthreads();
    }
}

// Gradient of the mean cross-entropy over samples [0, B) of Z (standardised),
// plus the L2 term l2/(2B) * |W|^2, into grad[]. Returns the loss in *loss.
__device__ void batch_gradient(const Net &n, const float *__restrict__ Z,
                               const int32_t *__restrict__ labels, const int32_t *__restrict__ idx,
                               int B, float l2, float *sh1_all, float *sda_all, float *grad,
                               float *loss) {
    const int w = threadIdx.x / kWave;
    float *sh1 = sh1_all + w * kH;
    float *sda = sda_all + w * kH;
    Grad g;
    zero_grad(g);
    const float inv_b = 1.f / (float)B;
    const int rounds = (B + kWaves - 1) / kWaves;
    for (int r = 0; r < rounds; ++r) {
        const int s = r * kWaves + w;
        const bool valid = s < B;
        const int sample = valid ? (idx ? idx[s] : s) : 0;
        Forward f;
        forward(n, Z + (int64_t)sample * kIn, sh1, f);
        backward(n, f, valid ? labels[sample] : 0, inv_b, valid, sh1, sda, g);
    }
    __shared__ float s_loss;
    reduce_grad(g, grad, &s_loss);
    // L2 on the weights (not the biases), and its share of the loss.
    __shared__ float s_w2[kWaves];
    float w2 = 0.f;
    for (int t = threadIdx.x; t < kParams; t += blockDim.x) {
        if (is_weight(t)) {
            const float p = param_of(n, t);
            grad[t] += l2 * inv_b * p;
            w2 += p * p;
        }
    }
    w2 = wave_sum(w2);
    if ((threadIdx.x & (kWave - 1)) == 0) s_w2[w] = w2;
    __syncthreads();
    if (threadIdx.x == 0) {
        float t = 0.f;
        for (int q = 0; q < kWaves; ++q) t += s_w2[q];
        *loss = s_loss + 0.5f * l2 * inv_b * t;
    }
    __syncthreads();
}

__global__ __launch_bounds__(kThreads) void loss_grad_kernel(const float *__restrict__ params,
                                                             const float *__restrict__ Z,
                                                             const int32_t *__restrict__ labels,
                                                             int B, float l2,
                                                             float *__restrict__ loss_out,
                                                             float *__restrict__ grad_out) {
    __shared__ Net n;
    __shared__ float sh1[kWaves * kH], sda[kWaves * kH], grad[kParams];
    __shared__ float loss;
    load_net(n, params);
    __syncthreads();
    batch_gradient(n, Z, labels, nullptr, B, l2, sh1, sda, grad, &loss);
    for (int t = threadIdx.x; t < kParams; t += blockDim.x) grad_out[t] = grad[t];
    if (threadIdx.x == 0) *loss_out = loss;
}

// Standardised inputs: Z = (T - mean) / std, T = transformed features, with the
// training mean and population std (floored) computed here in FP64.
__global__ __launch_bounds__(kThreads) void standardize_kernel(const float *__restrict__ F, int N,
                                                               float *__restrict__ Z,
                                                               float *__restrict__ model) {
    __shared__ double s_sum[kIn][kWaves], s_sq[kIn][kWaves];
    __shared__ float s_mean[kIn], s_std[kIn];
    const int w = threadIdx.x / kWave;
    for (int i = 0; i < kIn; ++i) {
        double a = 0.0, b = 0.0;
        for (int s = threadIdx.x; s < N; s += blockDim.x) {
            double v = F[(int64_t)s * kIn + i];
            if (log_feature(i)) v = log2(1.0 + v);
            a += v;
            b += v * v;
        }
        for (int off = kWave / 2; off > 0; off >>= 1) {
            a += __shfl_xor(a, off, kWave);
            b += __shfl_xor(b, off, kWave);
        }
        if ((threadIdx.x & (kWave - 1)) == 0) { s_sum[i][w] = a; s_sq[i][w] = b; }
    }
    __syncthreads();
    if (threadIdx.x < kIn) {
        const int i = threadIdx.x;
        double a = 0.0, b = 0.0;
        for (int q = 0; q < kWaves; ++q) { a += s_sum[i][q]; b += s_sq[i][q]; }
        const double mean = a / N;
        double var = b / N - mean * mean;
        var = var > 0.0 ? var : 0.0;
        const float sd = fmaxf((float)sqrt(var), kStdFloor);
        s_mean[i] = (float)mean;
        s_std[i] = sd;
        model[oMean + i] = (float)mean;
        model[oStd + i] = sd;
    }
    __syncthreads();
    for (int64_t q = threadIdx.x; q < (int64_t)N * kIn; q += blockDim.x) {
        const int i = (int)(q % kIn);
        double v = F[q];
        if (log_feature(i)) v = log2(1.0 + v);
        Z[q] = (float)((v - s_mean[i]) / s_std[i]);
    }
}

struct TrainArgs {
    int N, epochs, batch, max_steps;
    float lr, l2, beta1, beta2, eps;
};

__global__ __launch_bounds__(kThreads) void train_kernel(const float *__restrict__ Z,
                                                         const int32_t *__restrict__ labels,
                                                         const int32_t *__restrict__ perms,
                                                         TrainArgs a, float *__restrict__ model,
                                                         float *__restrict__ m,
                                                         float *__restrict__ v,
                                                         float *__restrict__ losses) {
    __shared__ Net n;
    __shared__ float sh1[kWaves * kH], sda[kWaves * kH], grad[kParams];
    __shared__ float loss;
    load_net(n, model);
    for (int t = threadIdx.x; t < kParams; t += blockDim.x) { m[t] = 0.f; v[t] = 0.f; }
    __syncthreads();
    const int B = a.batch < a.N ? a.batch : a.N;
    int step = 0;
    for (int ep = 0; ep < a.epochs && step < a.max_steps; ++ep) {
        const int32_t *order = perms + (int64_t)ep * a.N;
        for (int s0 = 0; s0 < a.N && step < a.max_steps; s0 += B) {
            const int b = (a.N - s0) < B ? (a.N - s0) : B;
            batch_gradient(n, Z, labels, order + s0, b, a.l2, sh1, sda, grad, &loss);
            ++step;
            const double bc1 = 1.0 - pow((double)a.beta1, step);
            const double bc2 = 1.0 - pow((double)a.beta2, step);
            for (int t = threadIdx.x; t < kParams; t += blockDim.x) {
                const float gt = grad[t];
                const float mt = a.beta1 * m[t] + (1.f - a.beta1) * gt;
                const float vt = a.beta2 * v[t] + (1.f - a.beta2) * gt * gt;
                m[t] = mt;
                v[t] = vt;
                const float mhat = (float)(mt / bc1);
                const float vhat = (float)(vt / bc2);
                store_param(n, t, param_of(n, t) - a.lr * mhat / (sqrtf(vhat) + a.eps));
            }
            if (threadIdx.x == 0 && losses) losses[step - 1] = loss;
            __syncthreads();
        }
    }
    for (int t = threadIdx.x; t < kParams; t += blockDim.x) model[t] = param_of(n, t);
}

// Every entry of the epoch orders must index a training sample.
__global__ __launch_bounds__(256) void check_orders(const int32_t *__restrict__ perms, int64_t total,
                                                    int32_t n, int32_t *__restrict__ bad) {
    int f = 0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < total; i += (int64_t)gridDim.x * 256)
        f |= (perms[i] < 0 || perms[i] >= n);
    if (f) atomicOr(bad, 1);
}

// One wave per sample: logits, masked arg-max (ties to the lowest class).
__global__ __launch_bounds__(kThreads) void predict_kernel(const float *__restrict__ model,
                                                           const float *__restrict__ F, int N,
                                                           const uint8_t *__restrict__ applicable,
                                                           uint32_t mask_all,
                                                           float *__restrict__ logits,
                                                           int32_t *__restrict__ cls) {
    __shared__ Net n;
    __shared__ float sh1[kWaves * kH];
    __shared__ float s_mean[kIn], s_std[kIn];
    load_net(n, model);
    if (threadIdx.x < kIn) { s_mean[threadIdx.x] = model[oMean + threadIdx.x]; s_std[threadIdx.x] = model[oStd + threadIdx.x]; }
    __syncthreads();
    const int w = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
    for (int s = blockIdx.x * kWaves + w; s < N; s += gridDim.x * kWaves) {
        float z[kIn];
#pragma unroll
        for (int i = 0; i < kIn; ++i) {
            double v = F[(int64_t)s * kIn + i];
            if (log_feature(i)) v = log2(1.0 + v);
            z[i] = (float)((v - s_mean[i]) / s_std[i]);
        }
        Forward f;
        forward(n, z, sh1 + w * kH, f);
        if (lane == 0) {
            int best = -1;
            float bv = 0.f;
            for (int c = 0; c < kOut; ++c) {
                if (logits) logits[(int64_t)s * kOut + c] = f.logits[c];
                const bool ok = applicable ? applicable[(int64_t)s * kOut + c] != 0 : ((mask_all >> c) & 1u);
                if (ok && (best < 0 || f.logits[c] > bv)) { best = c; bv = f.logits[c]; }
            }
            if (cls) cls[s] = best < 0 ? 0 : best;
        }
        __builtin_amdgcn_wave_barrier();
    }
}

// ---- process-wide selector weights, one copy per device ---------------------------

struct Weights {
    std::mutex mu;
    DevBuf buf[64];
    bool set[64] = {};
};

Weights &weights() {
    static Weights *w = new Weights();  // lives until process exit
    return *w;
}

int current_device() {
    int d = 0;
    SPMV_HIP(hipGetDevice(&d));
    if (d < 0 || d >= 64) fail(SPMV_ERR_INVALID_ARG, "device id %d", d);
    return d;
}

}  // namespace

spmv_status select_model(spmv_matrix_s *h, const float *feats, spmv_format *out, float *scores,
                         hipStream_t s) {
    const int d = current_device();
    Weights &W = weights();
    const float *model;
    {
        std::lock_guard<std::mutex> lk(W.mu);
        if (!W.set[d]) {
            set_error("no selector weights loaded on device %d", d);
            return SPMV_ERR_NO_MODEL;
        }
        model = W.buf[d].as<float>();
    }
    const bool ell_ok = h->nnz == 0 || (int64_t)((h->n_rows + 63) / 64 * 64) * h->stats.max_len <= 8 * h->nnz;
    const uint32_t mask = 0xBu | (ell_ok ? 0x4u : 0u);
    DevBuf io;
    io.alloc(kIn * 4 + kOut * 4 + 4);
    float *dF = io.as<float>();
    float *dL = dF + kIn;
    int32_t *dC = (int32_t *)(dL + kOut);
    SPMV_HIP(hipMemcpyAsync(dF, feats, kIn * 4, hipMemcpyHostToDevice, s));
    predict_kernel<<<1, kThreads, 0, s>>>(model, dF, 1, nullptr, mask, dL, dC);
    SPMV_CHECK_LAUNCH();
    float lg[kOut];
    int32_t c = 0;
    SPMV_HIP(hipMemcpyAsync(lg, dL, sizeof(lg), hipMemcpyDeviceToHost, s));
    SPMV_HIP(hipMemcpyAsync(&c, dC, 4, hipMemcpyDeviceToHost, s));
    SPMV_HIP(hipStreamSynchronize(s));
    for (int i = 0; i < kOut; ++i) scores[i] = lg[i];
    *out = (spmv_format)c;
    return SPMV_OK;
}

}  // namespace spmv

using namespace spmv;

extern "C" spmv_status spmv_selector_set_weights(const float *params, int64_t n) {
    return guard([&] {
        const int d = current_device();
        Weights &W = weights();
        std::lock_guard<std::mutex> lk(W.mu);
        if (!params && n == 0) {  // forget the model on this device
            W.set[d] = false;
            return;
        }
        if (!params || n != kModel) fail(SPMV_ERR_INVALID_ARG, "expected %d floats, got %lld", kModel, (long long)n);
        if (!W.buf[d].p) W.buf[d].alloc(kModel * 4);
        SPMV_HIP(hipMemcpy(W.buf[d].p, params, kModel * 4, hipMemcpyHostToDevice));
        W.set[d] = true;
    });
}

extern "C" spmv_status spmv_selector_get_weights(float *params, int64_t n) {
    return guard([&] {
        if (!params || n != kModel) fail(SPMV_ERR_INVALID_ARG, "expected %d floats", kModel);
        const int d = current_device();
        Weights &W = weights();
        std::lock_guard<std::mutex> lk(W.mu);
        if (!W.set[d]) fail(SPMV_ERR_NO_MODEL, "no selector weights loaded on device %d", d);
        SPMV_HIP(hipMemcpy(params, W.buf[d].p, kModel * 4, hipMemcpyDeviceToHost));
    });
}

extern "C" spmv_status spmv_selector_predict(const float *model, const float *feats, int32_t n,
                                             const uint8_t *applicable, float *logits,
                                             int32_t *cls, void *stream) {
    return guard([&] {
        if (n < 0 || (n > 0 && !feats)) fail(SPMV_ERR_INVALID_ARG, "bad feats / n");
        const float *m = model;
        if (!m) {
            const int d = current_device();
            Weights &W = weights();
            std::lock_guard<std::mutex> lk(W.mu);
            if (!W.set[d]) fail(SPMV_ERR_NO_MODEL, "no selector weights loaded on device %d", d);
            m = W.buf[d].as<float>();
        }
        if (n == 0) return;
        const int grid = (int)std::min<int64_t>(ceil_div(n, kWaves), 1024);
        predict_kernel<<<grid, kThreads, 0, (hipStream_t)stream>>>(m, feats, n, applicable, 0xFu,
                                                                     logits, cls);
        SPMV_CHECK_LAUNCH();
    });
}

extern "C" spmv_status spmv_selector_loss_grad(const float *params, const float *z,
                                               const int32_t *labels, int32_t b, float l2,
                                               float *loss, float *grad, void *stream) {
    return guard([&] {
        if (!params || !z || !labels || !loss || !grad || b <= 0)
            fail(SPMV_ERR_INVALID_ARG, "bad argument");
        loss_grad_kernel<<<1, kThreads, 0, (hipStream_t)stream>>>(params, z, labels, b, l2, loss, grad);
        SPMV_CHECK_LAUNCH();
    });
}

extern "C" spmv_status spmv_selector_train(const float *feats, const int32_t *labels, int32_t n,
                                           const float *init_params, const int32_t *perms,
                                           const spmv_train_opts *opts, float *out_model,
                                           float *out_losses, void *stream) {
    return guard([&] {
        if (!feats || !labels || !init_params || !perms || !opts || !out_model || n <= 0)
            fail(SPMV_ERR_INVALID_ARG, "bad argument");
        if (opts->epochs <= 0 || opts->batch <= 0) fail(SPMV_ERR_INVALID_ARG, "bad epochs / batch");
        hipStream_t s = (hipStream_t)stream;
        DevBuf Z, mv, bad;
        bad.alloc(4);
        SPMV_HIP(hipMemsetAsync(bad.p, 0, 4, s));
        const int64_t total = (int64_t)opts->epochs * n;
        check_orders<<<(int)std::min<int64_t>(ceil_div(total, 256), 2048), 256, 0, s>>>(
            perms, total, n, bad.as<int32_t>());
        SPMV_CHECK_LAUNCH();
        int32_t hb = 0;
        SPMV_HIP(hipMemcpyAsync(&hb, bad.p, 4, hipMemcpyDeviceToHost, s));
        SPMV_HIP(hipStreamSynchronize(s));
        if (hb) fail(SPMV_ERR_INVALID_ARG, "perms holds an index outside [0, %d)", n);
        Z.alloc((int64_t)n * kIn * 4);
        mv.alloc(2 * (int64_t)kParams * 4);
        SPMV_HIP(hipMemcpyAsync(out_model, init_params, kParams * 4, hipMemcpyDeviceToDevice, s));
        standardize_kernel<<<1, kThreads, 0, s>>>(feats, n, Z.as<float>(), out_model);
        SPMV_CHECK_LAUNCH();
        TrainArgs a{n, opts->epochs, opts->batch, opts->max_steps > 0 ? opts->max_steps : INT32_MAX,
                    opts->lr, opts->l2, opts->beta1, opts->beta2, opts->eps};
        train_kernel<<<1, kThreads, 0, s>>>(Z.as<float>(), labels, perms, a, out_model,
                                            mv.as<float>(), mv.as<float>() + kParams, out_losses);
        SPMV_CHECK_LAUNCH();
        SPMV_HIP(hipStreamSynchronize(s));
    });
}
