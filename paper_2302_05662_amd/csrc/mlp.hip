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

constexpr int kIn = 12, kH = 64;
// Parameter offsets of a network with NOUT classes (4: CSR, COO, ELL, HYB; 6: also
// SELL and BELL).
template <int NOUT>
struct Layout {
    static constexpr int oW1 = 0, oB1 = oW1 + kH * kIn, oW2 = oB1 + kH, oB2 = oW2 + kH * kH,
                         oW3 = oB2 + kH, oB3 = oW3 + NOUT * kH, kParams = oB3 + NOUT;
    static constexpr int oMean = kParams, oStd = kParams + kIn, kModel = kParams + 2 * kIn;
};
static_assert(Layout<4>::kParams == SPMV_SELECTOR_PARAMS && Layout<4>::kModel == SPMV_SELECTOR_MODEL,
              "parameter layout");
static_assert(Layout<6>::kParams == SPMV_SELECTOR_PARAMS6 && Layout<6>::kModel == SPMV_SELECTOR_MODEL6,
              "parameter layout");
constexpr int kMaxOut = 6;
constexpr int kWaves = 8;
constexpr int kThreads = kWaves * kWave;
constexpr float kStdFloor = 1e-6f;

// Feature columns that enter as log2(1 + v): counts and lengths (n, nnz, mean,
// var, std, median, mode, max, bandwidth); ratios stay raw.
__device__ __forceinline__ bool log_feature(int i) { return i <= 6 || i == 8 || i == 9; }

template <int NOUT>
struct Net {
    float W1T[kIn][kH];  // W1 transposed: [input][unit]
    float b1[kH];
    float W2[kH][kH];    // [unit of layer 2][unit of layer 1]
    float W2T[kH][kH];   // [unit of layer 1][unit of layer 2]
    float b2[kH];
    float W3[NOUT][kH];
    float b3[NOUT];
};

template <int NOUT>
__device__ void load_net(Net<NOUT> &n, const float *__restrict__ p) {
    using L = Layout<NOUT>;
    for (int t = threadIdx.x; t < L::kParams; t += blockDim.x) {
        const float w = p[t];
        if (t < L::oB1) { int j = t / kIn, i = t % kIn; n.W1T[i][j] = w; }
        else if (t < L::oW2) n.b1[t - L::oB1] = w;
        else if (t < L::oB2) { int q = t - L::oW2, j = q / kH, k = q % kH; n.W2[j][k] = w; n.W2T[k][j] = w; }
        else if (t < L::oW3) n.b2[t - L::oB2] = w;
        else if (t < L::oB3) { int q = t - L::oW3; n.W3[q / kH][q % kH] = w; }
        else n.b3[t - L::oB3] = w;
    }
}

template <int NOUT>
__device__ __forceinline__ void store_param(Net<NOUT> &n, int t, float w) {
    using L = Layout<NOUT>;
    if (t < L::oB1) { int j = t / kIn, i = t % kIn; n.W1T[i][j] = w; }
    else if (t < L::oW2) n.b1[t - L::oB1] = w;
    else if (t < L::oB2) { int q = t - L::oW2, j = q / kH, k = q % kH; n.W2[j][k] = w; n.W2T[k][j] = w; }
    else if (t < L::oW3) n.b2[t - L::oB2] = w;
    else if (t < L::oB3) { int q = t - L::oW3; n.W3[q / kH][q % kH] = w; }
    else n.b3[t - L::oB3] = w;
}

template <int NOUT>
__device__ __forceinline__ float param_of(const Net<NOUT> &n, int t) {
    using L = Layout<NOUT>;
    if (t < L::oB1) return n.W1T[t % kIn][t / kIn];
    if (t < L::oW2) return n.b1[t - L::oB1];
    if (t < L::oB2) { int q = t - L::oW2; return n.W2[q / kH][q % kH]; }
    if (t < L::oW3) return n.b2[t - L::oB2];
    if (t < L::oB3) { int q = t - L::oW3; return n.W3[q / kH][q % kH]; }
    return n.b3[t - L::oB3];
}

template <int NOUT>
__device__ __forceinline__ bool is_weight(int t) {
    using L = Layout<NOUT>;
    return t < L::oB1 || (t >= L::oW2 && t < L::oB2) || (t >= L::oW3 && t < L::oB3);
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

template <int NOUT>
struct Forward {
    float z[kIn];
    float a1, a2, h2;
    float logits[NOUT];
};

// Forward pass of one sample by one wave; h1 of all lanes is left in sh1.
template <int NOUT>
__device__ void forward(const Net<NOUT> &n, const float *__restrict__ zin, float *sh1, Forward<NOUT> &f) {
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
    for (int c = 0; c < NOUT; ++c) f.logits[c] = wave_sum(n.W3[c][j] * f.h2) + n.b3[c];
}

// Gradient accumulators of one wave (lane j holds row j of every weight matrix).
template <int NOUT>
struct Grad {
    float dW1[kIn];
    float db1;
    float dW2[kH];
    float db2;
    float dW3[NOUT];
    float db3[NOUT];
    float loss;
};

template <int NOUT>
__device__ void zero_grad(Grad<NOUT> &g) {
#pragma unroll
    for (int i = 0; i < kIn; ++i) g.dW1[i] = 0.f;
#pragma unroll
    for (int k = 0; k < kH; ++k) g.dW2[k] = 0.f;
#pragma unroll
    for (int c = 0; c < NOUT; ++c) { g.dW3[c] = 0.f; g.db3[c] = 0.f; }
    g.db1 = g.db2 = g.loss = 0.f;
}

// Adds one sample's cross-entropy gradient, scaled by inv_b, to g. Inactive
// waves pass valid = false and only take part in the lockstep LDS traffic.
template <int NOUT>
__device__ void backward(const Net<NOUT> &n, const Forward<NOUT> &f, int label, float inv_b, bool valid,
                         const float *sh1, float *sda, Grad<NOUT> &g) {
    const int j = threadIdx.x & (kWave - 1);
    float mx = f.logits[0];
#pragma unroll
    for (int c = 1; c < NOUT; ++c) mx = fmaxf(mx, f.logits[c]);
    float e[NOUT], se = 0.f;
#pragma unroll
    for (int c = 0; c < NOUT; ++c) { e[c] = expf(f.logits[c] - mx); se += e[c]; }
    float dz[NOUT];
#pragma unroll
    for (int c = 0; c < NOUT; ++c) dz[c] = valid ? (e[c] / se - (c == label ? 1.f : 0.f)) * inv_b : 0.f;
    float picked = 0.f;  // logit of the label, selected without a dynamic register index
#pragma unroll
    for (int c = 0; c < NOUT; ++c) picked = (c == label) ? f.logits[c] : picked;
    if (valid) g.loss += (logf(se) + mx - picked) * inv_b;
    float dh2 = 0.f;
#pragma unroll
    for (int c = 0; c < NOUT; ++c) {
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
template <int NOUT>
__device__ void reduce_grad(const Grad<NOUT> &g, float *grad, float *loss_acc) {
    using L = Layout<NOUT>;
    const int j = threadIdx.x & (kWave - 1);
    const int w = threadIdx.x / kWave;
    for (int t = threadIdx.x; t < L::kParams; t += blockDim.x) grad[t] = 0.f;
    if (threadIdx.x == 0) *loss_acc = 0.f;
    __syncthreads();
    for (int turn = 0; turn < kWaves; ++turn) {
        if (w == turn) {
#pragma unroll
            for (int i = 0; i < kIn; ++i) grad[L::oW1 + j * kIn + i] += g.dW1[i];
            grad[L::oB1 + j] += g.db1;
#pragma unroll
            for (int k = 0; k < kH; ++k) grad[L::oW2 + j * kH + k] += g.dW2[k];
            grad[L::oB2 + j] += g.db2;
#pragma unroll
            for (int c = 0; c < NOUT; ++c) grad[L::oW3 + c * kH + j] += g.dW3[c];
            if (j == 0) {
#pragma unroll
                for (int c = 0; c < NOUT; ++c) grad[L::oB3 + c] += g.db3[c];
                *loss_acc += g.loss;
            }
        }
        __syncthreads();
    }
}

// Gradient of the mean cross-entropy over samples [0, B) of Z (standardised),
// plus the L2 term l2/(2B) * |W|^2, into grad[]. Returns the loss in *loss.
template <int NOUT>
__device__ void batch_gradient(const Net<NOUT> &n, const float *__restrict__ Z,
                               const int32_t *__restrict__ labels, const int32_t *__restrict__ idx,
                               int B, float l2, float *sh1_all, float *sda_all, float *grad,
                               float *loss) {
    const int w = threadIdx.x / kWave;
    float *sh1 = sh1_all + w * kH;
    float *sda = sda_all + w * kH;
    using L = Layout<NOUT>;
    Grad<NOUT> g;
    zero_grad(g);
    const float inv_b = 1.f / (float)B;
    const int rounds = (B + kWaves - 1) / kWaves;
    for (int r = 0; r < rounds; ++r) {
        const int s = r * kWaves + w;
        const bool valid = s < B;
        const int sample = valid ? (idx ? idx[s] : s) : 0;
        Forward<NOUT> f;
        forward(n, Z + (int64_t)sample * kIn, sh1, f);
        backward(n, f, valid ? labels[sample] : 0, inv_b, valid, sh1, sda, g);
    }
    __shared__ float s_loss;
    reduce_grad(g, grad, &s_loss);
    // L2 on the weights (not the biases), and its share of the loss.
    __shared__ float s_w2[kWaves];
    float w2 = 0.f;
    for (int t = threadIdx.x; t < L::kParams; t += blockDim.x) {
        if (is_weight<NOUT>(t)) {
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

template <int NOUT>
__global__ __launch_bounds__(kThreads) void loss_grad_kernel(const float *__restrict__ params,
                                                             const float *__restrict__ Z,
                                                             const int32_t *__restrict__ labels,
                                                             int B, float l2,
                                                             float *__restrict__ loss_out,
                                                             float *__restrict__ grad_out) {
    using L = Layout<NOUT>;
    __shared__ Net<NOUT> n;
    __shared__ float sh1[kWaves * kH], sda[kWaves * kH], grad[L::kParams];
    __shared__ float loss;
    load_net(n, params);
    __syncthreads();
    batch_gradient(n, Z, labels, nullptr, B, l2, sh1, sda, grad, &loss);
    for (int t = threadIdx.x; t < L::kParams; t += blockDim.x) grad_out[t] = grad[t];
    if (threadIdx.x == 0) *loss_out = loss;
}

// Standardised inputs: Z = (T - mean) / std, T = transformed features, with the
// training mean and population std (floored) computed here in FP64.
template <int NOUT>
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
        model[Layout<NOUT>::oMean + i] = (float)mean;
        model[Layout<NOUT>::oStd + i] = sd;
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

template <int NOUT>
__global__ __launch_bounds__(kThreads) void train_kernel(const float *__restrict__ Z,
                                                         const int32_t *__restrict__ labels,
                                                         const int32_t *__restrict__ perms,
                                                         TrainArgs a, float *__restrict__ model,
                                                         float *__restrict__ m,
                                                         float *__restrict__ v,
                                                         float *__restrict__ losses) {
    using L = Layout<NOUT>;
    __shared__ Net<NOUT> n;
    __shared__ float sh1[kWaves * kH], sda[kWaves * kH], grad[L::kParams];
    __shared__ float loss;
    load_net(n, model);
    for (int t = threadIdx.x; t < L::kParams; t += blockDim.x) { m[t] = 0.f; v[t] = 0.f; }
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
            for (int t = threadIdx.x; t < L::kParams; t += blockDim.x) {
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
    for (int t = threadIdx.x; t < L::kParams; t += blockDim.x) model[t] = param_of(n, t);
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
template <int NOUT>
__global__ __launch_bounds__(kThreads) void predict_kernel(const float *__restrict__ model,
                                                           const float *__restrict__ F, int N,
                                                           const uint8_t *__restrict__ applicable,
                                                           uint32_t mask_all,
                                                           float *__restrict__ logits,
                                                           int32_t *__restrict__ cls) {
    using L = Layout<NOUT>;
    __shared__ Net<NOUT> n;
    __shared__ float sh1[kWaves * kH];
    __shared__ float s_mean[kIn], s_std[kIn];
    load_net(n, model);
    if (threadIdx.x < kIn) { s_mean[threadIdx.x] = model[L::oMean + threadIdx.x]; s_std[threadIdx.x] = model[L::oStd + threadIdx.x]; }
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
        Forward<NOUT> f;
        forward(n, z, sh1 + w * kH, f);
        if (lane == 0) {
            int best = -1;
            float bv = 0.f;
            for (int c = 0; c < NOUT; ++c) {
                if (logits) logits[(int64_t)s * NOUT + c] = f.logits[c];
                const bool ok = applicable ? applicable[(int64_t)s * NOUT + c] != 0 : ((mask_all >> c) & 1u);
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
    int classes[64] = {};  // 0: none installed
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

int classes_of_model_size(int64_t n) {
    if (n == Layout<4>::kModel) return 4;
    if (n == Layout<6>::kModel) return 6;
    return 0;
}

int64_t model_size(int classes) { return classes == 6 ? Layout<6>::kModel : Layout<4>::kModel; }

void launch_predict(int classes, const float *model, const float *feats, int n,
                    const uint8_t *applicable, uint32_t mask_all, float *logits, int32_t *cls,
                    hipStream_t s) {
    const int grid = (int)std::min<int64_t>(ceil_div(n, kWaves), 1024);
    if (classes == 6)
        predict_kernel<6><<<grid, kThreads, 0, s>>>(model, feats, n, applicable, mask_all, logits, cls);
    else
        predict_kernel<4><<<grid, kThreads, 0, s>>>(model, feats, n, applicable, mask_all, logits, cls);
    SPMV_CHECK_LAUNCH();
}

}  // namespace

// Logits of the installed network for one feature vector; scores[f] = -inf for a
// format the network has no class for. *classes receives its class count.
spmv_status model_logits(const float *feats, float scores[SPMV_NUM_FORMATS], int *classes,
                         hipStream_t s) {
    const int d = current_device();
    Weights &W = weights();
    const float *model;
    int nc;
    {
        std::lock_guard<std::mutex> lk(W.mu);
        if (!W.classes[d]) {
            set_error("no selector weights loaded on device %d", d);
            return SPMV_ERR_NO_MODEL;
        }
        model = W.buf[d].as<float>();
        nc = W.classes[d];
    }
    DevBuf io;
    io.alloc(kIn * 4 + kMaxOut * 4);
    float *dF = io.as<float>();
    float *dL = dF + kIn;
    SPMV_HIP(hipMemcpyAsync(dF, feats, kIn * 4, hipMemcpyHostToDevice, s));
    launch_predict(nc, model, dF, 1, nullptr, 0u, dL, nullptr, s);
    float lg[kMaxOut];
    SPMV_HIP(hipMemcpyAsync(lg, dL, (size_t)nc * 4, hipMemcpyDeviceToHost, s));
    SPMV_HIP(hipStreamSynchronize(s));
    for (int i = 0; i < SPMV_NUM_FORMATS; ++i) scores[i] = i < nc ? lg[i] : -INFINITY;
    *classes = nc;
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
            W.classes[d] = 0;
            return;
        }
        const int nc = classes_of_model_size(n);
        if (!params || !nc)
            fail(SPMV_ERR_INVALID_ARG, "expected %d (4 classes) or %d (6 classes) floats, got %lld",
                 Layout<4>::kModel, Layout<6>::kModel, (long long)n);
        if (!W.buf[d].p) W.buf[d].alloc(Layout<6>::kModel * 4);
        SPMV_HIP(hipMemcpy(W.buf[d].p, params, n * 4, hipMemcpyHostToDevice));
        W.classes[d] = nc;
    });
}

extern "C" int32_t spmv_selector_classes(void) {
    int d = 0;
    if (hipGetDevice(&d) != hipSuccess || d < 0 || d >= 64) {
        (void)hipGetLastError();
        return 0;
    }
    Weights &W = weights();
    std::lock_guard<std::mutex> lk(W.mu);
    return W.classes[d];
}

extern "C" spmv_status spmv_selector_get_weights(float *params, int64_t n) {
    return guard([&] {
        const int d = current_device();
        Weights &W = weights();
        std::lock_guard<std::mutex> lk(W.mu);
        if (!W.classes[d]) fail(SPMV_ERR_NO_MODEL, "no selector weights loaded on device %d", d);
        const int64_t want = model_size(W.classes[d]);
        if (!params || n != want) fail(SPMV_ERR_INVALID_ARG, "expected %lld floats", (long long)want);
        SPMV_HIP(hipMemcpy(params, W.buf[d].p, want * 4, hipMemcpyDeviceToHost));
    });
}

extern "C" spmv_status spmv_selector_predict(const float *model, int32_t classes, const float *feats,
                                             int32_t n, const uint8_t *applicable, float *logits,
                                             int32_t *cls, void *stream) {
    return guard([&] {
        if (n < 0 || (n > 0 && !feats)) fail(SPMV_ERR_INVALID_ARG, "bad feats / n");
        const float *m = model;
        int nc = classes;
        if (!m) {
            const int d = current_device();
            Weights &W = weights();
            std::lock_guard<std::mutex> lk(W.mu);
            if (!W.classes[d]) fail(SPMV_ERR_NO_MODEL, "no selector weights loaded on device %d", d);
            if (nc != 0 && nc != W.classes[d])
                fail(SPMV_ERR_INVALID_ARG, "the installed network has %d classes, not %d", W.classes[d], nc);
            m = W.buf[d].as<float>();
            nc = W.classes[d];
        }
        if (nc != 4 && nc != 6) fail(SPMV_ERR_INVALID_ARG, "classes must be 4 or 6, got %d", nc);
        if (n == 0) return;
        launch_predict(nc, m, feats, n, applicable, (1u << nc) - 1u, logits, cls, (hipStream_t)stream);
    });
}

extern "C" spmv_status spmv_selector_loss_grad(const float *params, int32_t classes, const float *z,
                                               const int32_t *labels, int32_t b, float l2,
                                               float *loss, float *grad, void *stream) {
    return guard([&] {
        if (!params || !z || !labels || !loss || !grad || b <= 0)
            fail(SPMV_ERR_INVALID_ARG, "bad argument");
        if (classes == 6)
            loss_grad_kernel<6><<<1, kThreads, 0, (hipStream_t)stream>>>(params, z, labels, b, l2, loss, grad);
        else if (classes == 4)
            loss_grad_kernel<4><<<1, kThreads, 0, (hipStream_t)stream>>>(params, z, labels, b, l2, loss, grad);
        else
            fail(SPMV_ERR_INVALID_ARG, "classes must be 4 or 6, got %d", classes);
        SPMV_CHECK_LAUNCH();
    });
}

namespace {

// Every entry of the epoch orders must index a training sample, every label a class.
__global__ __launch_bounds__(256) void check_labels(const int32_t *__restrict__ labels, int32_t n,
                                                    int32_t classes, int32_t *__restrict__ bad) {
    int f = 0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        f |= (labels[i] < 0 || labels[i] >= classes);
    if (f) atomicOr(bad, 2);
}

template <int NOUT>
void train_impl(const float *feats, const int32_t *labels, int32_t n, const float *init_params,
                const int32_t *perms, const spmv_train_opts *opts, float *out_model,
                float *out_losses, hipStream_t s) {
    using L = Layout<NOUT>;
    DevBuf Z, mv, bad;
    bad.alloc(4);
    SPMV_HIP(hipMemsetAsync(bad.p, 0, 4, s));
    const int64_t total = (int64_t)opts->epochs * n;
    check_orders<<<(int)std::min<int64_t>(ceil_div(total, 256), 2048), 256, 0, s>>>(
        perms, total, n, bad.as<int32_t>());
    SPMV_CHECK_LAUNCH();
    check_labels<<<(int)std::min<int64_t>(ceil_div(n, 256), 2048), 256, 0, s>>>(labels, n, NOUT,
                                                                                 bad.as<int32_t>());
    SPMV_CHECK_LAUNCH();
    int32_t hb = 0;
    SPMV_HIP(hipMemcpyAsync(&hb, bad.p, 4, hipMemcpyDeviceToHost, s));
    SPMV_HIP(hipStreamSynchronize(s));
    if (hb & 1) fail(SPMV_ERR_INVALID_ARG, "perms holds an index outside [0, %d)", n);
    if (hb & 2) fail(SPMV_ERR_INVALID_ARG, "a label is outside [0, %d)", NOUT);
    Z.alloc((int64_t)n * kIn * 4);
    mv.alloc(2 * (int64_t)L::kParams * 4);
    SPMV_HIP(hipMemcpyAsync(out_model, init_params, L::kParams * 4, hipMemcpyDeviceToDevice, s));
    standardize_kernel<NOUT><<<1, kThreads, 0, s>>>(feats, n, Z.as<float>(), out_model);
    SPMV_CHECK_LAUNCH();
    TrainArgs a{n, opts->epochs, opts->batch, opts->max_steps > 0 ? opts->max_steps : INT32_MAX,
                opts->lr, opts->l2, opts->beta1, opts->beta2, opts->eps};
    train_kernel<NOUT><<<1, kThreads, 0, s>>>(Z.as<float>(), labels, perms, a, out_model,
                                              mv.as<float>(), mv.as<float>() + L::kParams, out_losses);
    SPMV_CHECK_LAUNCH();
    SPMV_HIP(hipStreamSynchronize(s));
}

}  // namespace

extern "C" spmv_status spmv_selector_train(const float *feats, const int32_t *labels, int32_t n,
                                           const float *init_params, const int32_t *perms,
                                           const spmv_train_opts *opts, float *out_model,
                                           float *out_losses, void *stream) {
    return guard([&] {
        if (!feats || !labels || !init_params || !perms || !opts || !out_model || n <= 0)
            fail(SPMV_ERR_INVALID_ARG, "bad argument");
        if (opts->epochs <= 0 || opts->batch <= 0) fail(SPMV_ERR_INVALID_ARG, "bad epochs / batch");
        const int nc = opts->classes == 0 ? 4 : opts->classes;
        if (nc == 6)
            train_impl<6>(feats, labels, n, init_params, perms, opts, out_model, out_losses, (hipStream_t)stream);
        else if (nc == 4)
            train_impl<4>(feats, labels, n, init_params, perms, opts, out_model, out_losses, (hipStream_t)stream);
        else
            fail(SPMV_ERR_INVALID_ARG, "classes must be 4 or 6, got %d", opts->classes);
    });
}
