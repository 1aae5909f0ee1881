// Learned candidate-buffer sizing: a small FP32 MLP (22 -> H -> H -> K, ReLU, sigmoid output)
// trained on the GPU with hand-written forward / backward / Adam kernels.
//
// Features of a design request: log(A)/log(2000), the 20 amino-acid fractions, lambda/4.
// Targets: for K bins of right endpoints b by relative position layer(b)/n, the fraction of the
// worst-case candidate slots (states c with layer(c) <= layer(b)-5) that the exact DP retains in
// C_b (eq. 6), summed per bin.  Loss: mean squared error over samples and outputs.
// Every reduction runs in a fixed order (one thread owns one output value), so gradients are
// deterministic.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <vector>

#include "../../include/sparsedesign.h"
#include "sd_device.h"

namespace sd {

constexpr int kFeat = 22;

struct MlpShape {
    int H, K;
    int o_w1, o_b1, o_w2, o_b2, o_w3, o_b3, total;
};

MlpShape mlp_shape(int H, int K) {
    MlpShape s;
    s.H = H;
    s.K = K;
    s.o_w1 = 0;
    s.o_b1 = s.o_w1 + H * kFeat;
    s.o_w2 = s.o_b1 + H;
    s.o_b2 = s.o_w2 + H * H;
    s.o_w3 = s.o_b2 + H;
    s.o_b3 = s.o_w3 + K * H;
    s.total = s.o_b3 + K;
    return s;
}

// layer forward: out[s][j] = act(sum_i W[j][i] * in[s][i] + b[j]); act 0 relu, 1 sigmoid
__global__ void k_dense_fwd(const float* __restrict__ W, const float* __restrict__ b, const float* __restrict__ in,
                            float* __restrict__ out, int n, int nin, int nout, int act) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n * nout) return;
    const int s = idx / nout, j = idx % nout;
    float z = b[j];
    for (int i = 0; i < nin; i++) z = fmaf(W[j * nin + i], in[s * nin + i], z);
    out[idx] = act == 0 ? fmaxf(z, 0.f) : 1.f / (1.f + expf(-z));
}

// output delta for MSE through the sigmoid: d = 2/(n*K) * (yhat - y) * yhat * (1 - yhat)
__global__ void k_out_delta(const float* __restrict__ yhat, const float* __restrict__ y, float* __restrict__ d,
                            int total, float scale) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    const float p = yhat[idx];
    d[idx] = scale * (p - y[idx]) * p * (1.f - p);
}

// back-propagate a delta through W (nout x nin) into the previous ReLU layer's pre-activation:
// dprev[s][i] = (sum_j W[j][i] * d[s][j]) * [act[s][i] > 0]
__global__ void k_dense_bwd_data(const float* __restrict__ W, const float* __restrict__ d,
                                 const float* __restrict__ act, float* __restrict__ dprev, int n, int nin, int nout) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n * nin) return;
    const int s = idx / nin, i = idx % nin;
    float g = 0.f;
    for (int j = 0; j < nout; j++) g = fmaf(W[j * nin + i], d[s * nout + j], g);
    dprev[idx] = act[idx] > 0.f ? g : 0.f;
}

// weight / bias gradients: gW[j][i] = sum_s d[s][j] * in[s][i], gb[j] = sum_s d[s][j]
__global__ void k_dense_bwd_weights(const float* __restrict__ d, const float* __restrict__ in, float* __restrict__ gW,
                                    float* __restrict__ gb, int n, int nin, int nout) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx < nout * nin) {
        const int j = idx / nin, i = idx % nin;
        float g = 0.f;
        for (int s = 0; s < n; s++) g = fmaf(d[s * nout + j], in[s * nin + i], g);
        gW[idx] = g;
    } else if (idx < nout * nin + nout) {
        const int j = idx - nout * nin;
        float g = 0.f;
        for (int s = 0; s < n; s++) g += d[s * nout + j];
        gb[j] = g;
    }
}

__global__ void k_mse(const float* __restrict__ yhat, const float* __restrict__ y, float* __restrict__ loss,
                      int total) {
    // single block, fixed-order tree reduction
    __shared__ float red[256];
    float acc = 0.f;
    for (int i = threadIdx.x; i < total; i += blockDim.x) {
        const float e = yhat[i] - y[i];
        acc += e * e;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *loss = red[0] / (float)total;
}

__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m, float* __restrict__ v,
                       int n, float lr, float b1, float b2, float eps, float c1, float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

}  // namespace sd

using namespace sd;

struct sd_sizer {
    sd_context* ctx;
    MlpShape sh;
    float* P = nullptr;  // params (device)
    float* G = nullptr;  // grads
    float* M = nullptr;  // Adam first moment
    float* Vm = nullptr; // Adam second moment
    int64_t adam_t = 0;
    std::vector<float> host;  // host copy of the parameters (prediction on the host side)
};

namespace {
thread_local std::string g_mlp_err;
int cdiv(int a, int b) { return (a + b - 1) / b; }

struct Work {
    float *X = nullptr, *Y = nullptr, *H1 = nullptr, *H2 = nullptr, *O = nullptr, *D3 = nullptr,
          *D2 = nullptr, *D1 = nullptr, *loss = nullptr;
    hipError_t alloc(int n, int H, int K) {
        size_t tot = (size_t)n * (kFeat + K + 3 * H + 2 * K + H) + 1;
        float* base = nullptr;
        hipError_t e = hipMalloc(&base, tot * sizeof(float));
        if (e != hipSuccess) return e;
        X = base;
        Y = X + (size_t)n * kFeat;
        H1 = Y + (size_t)n * K;
        H2 = H1 + (size_t)n * H;
        O = H2 + (size_t)n * H;
        D3 = O + (size_t)n * K;
        D2 = D3 + (size_t)n * K;
        D1 = D2 + (size_t)n * H;
        loss = D1 + (size_t)n * H;
        return hipSuccess;
    }
    ~Work() {
        if (X) hipFree(X);
    }
};

// forward (and optionally backward) on n samples already in W.X / W.Y
hipError_t fwd_bwd(sd_sizer* z, Work& W, int n, bool backward, hipStream_t st) {
    const MlpShape& s = z->sh;
    const int H = s.H, K = s.K;
    float* P = z->P;
    hipLaunchKernelGGL(k_dense_fwd, dim3(cdiv(n * H, 256)), dim3(256), 0, st, P + s.o_w1, P + s.o_b1, W.X, W.H1, n, kFeat, H, 0);
    hipLaunchKernelGGL(k_dense_fwd, dim3(cdiv(n * H, 256)), dim3(256), 0, st, P + s.o_w2, P + s.o_b2, W.H1, W.H2, n, H, H, 0);
    hipLaunchKernelGGL(k_dense_fwd, dim3(cdiv(n * K, 256)), dim3(256), 0, st, P + s.o_w3, P + s.o_b3, W.H2, W.O, n, H, K, 1);
    if (W.Y) hipLaunchKernelGGL(k_mse, dim3(1), dim3(256), 0, st, W.O, W.Y, W.loss, n * K);
    if (!backward) return hipGetLastError();
    float* G = z->G;
    hipLaunchKernelGGL(k_out_delta, dim3(cdiv(n * K, 256)), dim3(256), 0, st, W.O, W.Y, W.D3, n * K, 2.f / (float)(n * K));
    hipLaunchKernelGGL(k_dense_bwd_weights, dim3(cdiv(K * H + K, 256)), dim3(256), 0, st, W.D3, W.H2, G + s.o_w3, G + s.o_b3, n, H, K);
    hipLaunchKernelGGL(k_dense_bwd_data, dim3(cdiv(n * H, 256)), dim3(256), 0, st, P + s.o_w3, W.D3, W.H2, W.D2, n, H, K);
    hipLaunchKernelGGL(k_dense_bwd_weights, dim3(cdiv(H * H + H, 256)), dim3(256), 0, st, W.D2, W.H1, G + s.o_w2, G + s.o_b2, n, H, H);
    hipLaunchKernelGGL(k_dense_bwd_data, dim3(cdiv(n * H, 256)), dim3(256), 0, st, P + s.o_w2, W.D2, W.H1, W.D1, n, H, H);
    hipLaunchKernelGGL(k_dense_bwd_weights, dim3(cdiv(H * kFeat + H, 256)), dim3(256), 0, st, W.D1, W.X, G + s.o_w1, G + s.o_b1, n, kFeat, H);
    return hipGetLastError();
}

sd_status mlp_fail(sd_status s, const std::string& m) {
    g_mlp_err = m;
    return s;
}
}  // namespace

extern "C" sd_status sd_sizer_create(sd_context* ctx, int hidden, int n_out, uint64_t seed, sd_sizer** out) {
    if (!ctx || !out || hidden <= 0 || hidden > 1024 || n_out <= 0 || n_out > 64) return mlp_fail(SD_E_ARG, "bad sizer shape");
    *out = nullptr;
    sd_sizer* z = new (std::nothrow) sd_sizer();
    if (!z) return SD_E_NOMEM;
    z->ctx = ctx;
    z->sh = mlp_shape(hidden, n_out);
    const int T = z->sh.total;
    hipError_t e = hipSetDevice(ctx->device);
    float* base = nullptr;
    if (e == hipSuccess) e = hipMalloc(&base, sizeof(float) * 4 * (size_t)T);
    if (e != hipSuccess) {
        delete z;
        return mlp_fail(SD_E_NOMEM, "sizer allocation");
    }
    z->P = base;
    z->G = base + T;
    z->M = base + 2 * (size_t)T;
    z->Vm = base + 3 * (size_t)T;
    // He-style uniform initialisation from a 64-bit LCG; biases zero
    z->host.assign(T, 0.f);
    uint64_t st = seed * 6364136223846793005ull + 1442695040888963407ull;
    auto uni = [&]() {
        st = st * 6364136223846793005ull + 1442695040888963407ull;
        return (float)((st >> 40) * (1.0 / 16777216.0)) * 2.f - 1.f;
    };
    const MlpShape& s = z->sh;
    for (int i = 0; i < hidden * kFeat; i++) z->host[s.o_w1 + i] = uni() * sqrtf(6.f / kFeat);
    for (int i = 0; i < hidden * hidden; i++) z->host[s.o_w2 + i] = uni() * sqrtf(6.f / hidden);
    for (int i = 0; i < n_out * hidden; i++) z->host[s.o_w3 + i] = uni() * sqrtf(6.f / hidden);
    std::vector<float> zeros(3 * (size_t)T, 0.f);
    e = hipMemcpy(z->P, z->host.data(), sizeof(float) * T, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(z->G, zeros.data(), sizeof(float) * 3 * (size_t)T, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        hipFree(base);
        delete z;
        return mlp_fail(SD_E_DEVICE, "sizer upload");
    }
    *out = z;
    return SD_OK;
}

extern "C" void sd_sizer_free(sd_sizer* z) {
    if (!z) return;
    if (z->P) hipFree(z->P);
    delete z;
}

extern "C" int64_t sd_sizer_num_params(const sd_sizer* z) { return z ? z->sh.total : 0; }

extern "C" sd_status sd_sizer_get_params(const sd_sizer* z, float* flat) {
    if (!z || !flat) return mlp_fail(SD_E_ARG, "null argument");
    hipError_t e = hipMemcpy(flat, z->P, sizeof(float) * z->sh.total, hipMemcpyDeviceToHost);
    return e == hipSuccess ? SD_OK : mlp_fail(SD_E_DEVICE, "sizer download");
}

extern "C" sd_status sd_sizer_set_params(sd_sizer* z, const float* flat) {
    if (!z || !flat) return mlp_fail(SD_E_ARG, "null argument");
    z->host.assign(flat, flat + z->sh.total);
    hipError_t e = hipMemcpy(z->P, flat, sizeof(float) * z->sh.total, hipMemcpyHostToDevice);
    return e == hipSuccess ? SD_OK : mlp_fail(SD_E_DEVICE, "sizer upload");
}

// loss and full parameter gradient on n samples (MSE, same layout as sd_sizer_get_params)
extern "C" sd_status sd_sizer_gradient(sd_sizer* z, int n, const float* X, const float* Y, float* loss,
                                       float* grad) {
    if (!z || n <= 0 || !X || !Y || !loss || !grad) return mlp_fail(SD_E_ARG, "null argument");
    Work W;
    hipError_t e = W.alloc(n, z->sh.H, z->sh.K);
    hipStream_t st = z->ctx->stream;
    if (e == hipSuccess) e = hipMemcpyAsync(W.X, X, sizeof(float) * n * kFeat, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(W.Y, Y, sizeof(float) * n * z->sh.K, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = fwd_bwd(z, W, n, true, st);
    if (e == hipSuccess) e = hipMemcpyAsync(loss, W.loss, sizeof(float), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipMemcpyAsync(grad, z->G, sizeof(float) * z->sh.total, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    return e == hipSuccess ? SD_OK : mlp_fail(SD_E_DEVICE, hipGetErrorString(e));
}

// full-batch Adam for `steps` iterations; *final_loss is the loss before the last update
extern "C" sd_status sd_sizer_train(sd_sizer* z, int n, const float* X, const float* Y, int steps, float lr,
                                    float* final_loss) {
    if (!z || n <= 0 || !X || !Y || steps < 0) return mlp_fail(SD_E_ARG, "bad training arguments");
    Work W;
    hipError_t e = W.alloc(n, z->sh.H, z->sh.K);
    hipStream_t st = z->ctx->stream;
    if (e == hipSuccess) e = hipMemcpyAsync(W.X, X, sizeof(float) * n * kFeat, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(W.Y, Y, sizeof(float) * n * z->sh.K, hipMemcpyHostToDevice, st);
    const float b1 = 0.9f, b2 = 0.999f;
    for (int it = 0; it < steps && e == hipSuccess; it++) {
        e = fwd_bwd(z, W, n, true, st);
        z->adam_t++;
        const float c1 = 1.f - powf(b1, (float)z->adam_t), c2 = 1.f - powf(b2, (float)z->adam_t);
        if (e == hipSuccess)
            hipLaunchKernelGGL(k_adam, dim3(cdiv(z->sh.total, 256)), dim3(256), 0, st, z->P, z->G, z->M, z->Vm,
                               z->sh.total, lr, b1, b2, 1e-8f, c1, c2);
        if (e == hipSuccess) e = hipGetLastError();
    }
    float l = 0.f;
    if (e == hipSuccess && final_loss) e = hipMemcpyAsync(&l, W.loss, sizeof(float), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e == hipSuccess) {
        z->host.resize(z->sh.total);
        e = hipMemcpy(z->host.data(), z->P, sizeof(float) * z->sh.total, hipMemcpyDeviceToHost);
    }
    if (e != hipSuccess) return mlp_fail(SD_E_DEVICE, hipGetErrorString(e));
    if (final_loss) *final_loss = l;
    return SD_OK;
}

// GPU forward on n samples
extern "C" sd_status sd_sizer_predict(sd_sizer* z, int n, const float* X, float* Yhat) {
    if (!z || n <= 0 || !X || !Yhat) return mlp_fail(SD_E_ARG, "null argument");
    Work W;
    hipError_t e = W.alloc(n, z->sh.H, z->sh.K);
    hipStream_t st = z->ctx->stream;
    float* y = W.Y;
    W.Y = nullptr;  // no loss
    if (e == hipSuccess) e = hipMemcpyAsync(W.X, X, sizeof(float) * n * kFeat, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = fwd_bwd(z, W, n, false, st);
    W.Y = y;
    if (e == hipSuccess) e = hipMemcpyAsync(Yhat, W.O, sizeof(float) * n * z->sh.K, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    return e == hipSuccess ? SD_OK : mlp_fail(SD_E_DEVICE, hipGetErrorString(e));
}

extern "C" sd_status sd_sizer_features(const char* protein, double lambda_kcal, float out[22]) {
    if (!protein || !out) return mlp_fail(SD_E_ARG, "null argument");
    static const char* aa = "ACDEFGHIKLMNPQRSTVWY";
    const int A = (int)strlen(protein);
    if (A <= 0) return SD_E_PROTEIN;
    int cnt[20] = {0};
    for (int k = 0; k < A; k++) {
        const char* p = strchr(aa, protein[k]);
        if (p && protein[k]) cnt[p - aa]++;
    }
    out[0] = (float)(log((double)A) / log(2000.0));
    for (int i = 0; i < 20; i++) out[1 + i] = (float)cnt[i] / (float)A;
    out[21] = (float)(lambda_kcal / 4.0);
    return SD_OK;
}

// Host-side forward with the trained parameters (same arithmetic order as the kernels), used by
// the library's sizing policy; defined here so the policy needs no device round trip.
namespace sd {
void sizer_predict_host(const sd_sizer* z, const float* x, float* y) {
    const MlpShape& s = z->sh;
    const float* P = z->host.data();
    std::vector<float> h1(s.H), h2(s.H);
    for (int j = 0; j < s.H; j++) {
        float a = P[s.o_b1 + j];
        for (int i = 0; i < kFeat; i++) a = fmaf(P[s.o_w1 + j * kFeat + i], x[i], a);
        h1[j] = fmaxf(a, 0.f);
    }
    for (int j = 0; j < s.H; j++) {
        float a = P[s.o_b2 + j];
        for (int i = 0; i < s.H; i++) a = fmaf(P[s.o_w2 + j * s.H + i], h1[i], a);
        h2[j] = fmaxf(a, 0.f);
    }
    for (int j = 0; j < s.K; j++) {
        float a = P[s.o_b3 + j];
        for (int i = 0; i < s.H; i++) a = fmaf(P[s.o_w3 + j * s.H + i], h2[i], a);
        y[j] = 1.f / (1.f + expf(-a));
    }
}
int sizer_bins(const sd_sizer* z) { return z->sh.K; }
}  // namespace sd

extern "C" sd_status sd_sizer_predict_host(const sd_sizer* z, int n, const float* X, float* Yhat) {
    if (!z || n <= 0 || !X || !Yhat) return mlp_fail(SD_E_ARG, "null argument");
    for (int i = 0; i < n; i++) sd::sizer_predict_host(z, X + (size_t)i * kFeat, Yhat + (size_t)i * z->sh.K);
    return SD_OK;
}
