// mlp.hip -- the learned plan selector's network: a multilayer perceptron
// with two hidden ReLU layers, trained on the GPU with these kernels.
//
//   a1 = relu(W1 x + b1),  a2 = relu(W2 a1 + b2),  y = w3 . a2 + b3
//   loss = mean_b (y_b - t_b)^2
//
// Parameters are one float vector:
//   W1 [H][D], b1 [H], W2 [H][H], b2 [H], w3 [H], b3 [1].
// The gradient is computed in two steps: per-sample deltas (one workgroup
// per sample), then one thread per parameter summing over the minibatch in
// sample order, so results are deterministic (no atomics).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <vector>

#include "../../include/offt.h"
#include "offt_internal.h"
#include "plan_impl.h"

namespace offt {

struct MlpLayout {
    int D, H;
    int64_t W1, b1, W2, b2, w3, b3, P;
    __host__ __device__ MlpLayout(int d, int h) : D(d), H(h) {
        W1 = 0;
        b1 = W1 + (int64_t)H * D;
        W2 = b1 + H;
        b2 = W2 + (int64_t)H * H;
        w3 = b2 + H;
        b3 = w3 + H;
        P = b3 + 1;
    }
};

// One workgroup (H threads) per sample.  A1/A2 may be null (inference).
__global__ void mlp_forward_kernel(const float* __restrict__ p, const float* __restrict__ X,
                                   const int32_t* __restrict__ idx, int B, int D, int H, float* __restrict__ Y,
                                   float* __restrict__ A1, float* __restrict__ A2) {
    extern __shared__ float sh[];   // x[D], a1[H], a2[H]
    const MlpLayout lay(D, H);
    const int b = blockIdx.x;
    if (b >= B) return;
    const int j = threadIdx.x;
    const int64_t row = idx ? idx[b] : b;
    float* x = sh;
    float* a1 = sh + D;
    float* a2 = a1 + H;
    for (int k = j; k < D; k += H) x[k] = X[row * D + k];
    __syncthreads();
    float s = p[lay.b1 + j];
    for (int k = 0; k < D; ++k) s += p[lay.W1 + (int64_t)j * D + k] * x[k];
    a1[j] = s > 0.f ? s : 0.f;
    __syncthreads();
    s = p[lay.b2 + j];
    for (int i = 0; i < H; ++i) s += p[lay.W2 + (int64_t)j * H + i] * a1[i];
    a2[j] = s > 0.f ? s : 0.f;
    if (A1) A1[(int64_t)b * H + j] = a1[j];
    if (A2) A2[(int64_t)b * H + j] = a2[j];
    __syncthreads();
    if (j == 0) {
        float y = p[lay.b3];
        for (int i = 0; i < H; ++i) y += p[lay.w3 + i] * a2[i];
        Y[b] = y;
    }
}

// Per-sample deltas of the mean squared error: dy_b = 2 (y_b - t_b) / B,
// G2[b][j] = dy_b w3[j] [a2 > 0], G1[b][i] = (sum_j G2[b][j] W2[j][i]) [a1 > 0].
__global__ void mlp_delta_kernel(const float* __restrict__ p, const float* __restrict__ T,
                                 const int32_t* __restrict__ idx, int B, int D, int H,
                                 const float* __restrict__ Y, const float* __restrict__ A1,
                                 const float* __restrict__ A2, float* __restrict__ DY, float* __restrict__ G1,
                                 float* __restrict__ G2) {
    extern __shared__ float sh[];   // g2[H]
    const MlpLayout lay(D, H);
    const int b = blockIdx.x;
    if (b >= B) return;
    const int j = threadIdx.x;
    const int64_t row = idx ? idx[b] : b;
    const float dy = 2.f * (Y[b] - T[row]) / (float)B;
    const float g2 = A2[(int64_t)b * H + j] > 0.f ? dy * p[lay.w3 + j] : 0.f;
    sh[j] = g2;
    G2[(int64_t)b * H + j] = g2;
    if (j == 0) DY[b] = dy;
    __syncthreads();
    float s = 0.f;
    for (int k = 0; k < H; ++k) s += sh[k] * p[lay.W2 + (int64_t)k * H + j];
    G1[(int64_t)b * H + j] = A1[(int64_t)b * H + j] > 0.f ? s : 0.f;
}

// One thread per parameter: gradient summed over the minibatch in order.
__global__ void mlp_grad_kernel(const float* __restrict__ X, const int32_t* __restrict__ idx, int B, int D, int H,
                                const float* __restrict__ A1, const float* __restrict__ A2,
                                const float* __restrict__ DY, const float* __restrict__ G1,
                                const float* __restrict__ G2, float* __restrict__ grad) {
    const MlpLayout lay(D, H);
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= lay.P) return;
    float s = 0.f;
    if (q < lay.b1) {                       // W1[j][k]
        const int64_t j = q / D, k = q % D;
        for (int b = 0; b < B; ++b) {
            const int64_t row = idx ? idx[b] : b;
            s += G1[(int64_t)b * H + j] * X[row * D + k];
        }
    } else if (q < lay.W2) {                // b1[j]
        const int64_t j = q - lay.b1;
        for (int b = 0; b < B; ++b) s += G1[(int64_t)b * H + j];
    } else if (q < lay.b2) {                // W2[j][i]
        const int64_t r = q - lay.W2, j = r / H, i = r % H;
        for (int b = 0; b < B; ++b) s += G2[(int64_t)b * H + j] * A1[(int64_t)b * H + i];
    } else if (q < lay.w3) {                // b2[j]
        const int64_t j = q - lay.b2;
        for (int b = 0; b < B; ++b) s += G2[(int64_t)b * H + j];
    } else if (q < lay.b3) {                // w3[j]
        const int64_t j = q - lay.w3;
        for (int b = 0; b < B; ++b) s += DY[b] * A2[(int64_t)b * H + j];
    } else {                                // b3
        for (int b = 0; b < B; ++b) s += DY[b];
    }
    grad[q] = s;
}

// loss = mean_b (y_b - t_b)^2, one workgroup.
__global__ void mlp_loss_kernel(const float* __restrict__ Y, const float* __restrict__ T,
                                const int32_t* __restrict__ idx, int B, float* __restrict__ loss) {
    __shared__ float part[256];
    float s = 0.f;
    for (int b = threadIdx.x; b < B; b += blockDim.x) {
        const int64_t row = idx ? idx[b] : b;
        const float d = Y[b] - T[row];
        s += d * d;
    }
    part[threadIdx.x] = s;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *loss = part[0] / (float)B;
}

// Adam (Kingma & Ba 2015) with bias correction; step >= 1.
__global__ void mlp_adam_kernel(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                                float* __restrict__ v, int64_t P, float lr, float beta1, float beta2, float eps,
                                float corr1, float corr2) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= P) return;
    const float gq = g[q];
    const float mq = beta1 * m[q] + (1.f - beta1) * gq;
    const float vq = beta2 * v[q] + (1.f - beta2) * gq * gq;
    m[q] = mq;
    v[q] = vq;
    p[q] -= lr * (mq / corr1) / (sqrtf(vq / corr2) + eps);
}

}  // namespace offt

struct offt_mlp_s {
    int D = 0, H = 0, max_batch = 0;
    int64_t P = 0;
    float* params = nullptr;
    float* m = nullptr;
    float* v = nullptr;
    float* A1 = nullptr;
    float* A2 = nullptr;
    float* Y = nullptr;
    float* DY = nullptr;
    float* G1 = nullptr;
    float* G2 = nullptr;
    int64_t step = 0;
    std::vector<void*> allocs;
};

using namespace offt;

static void mlp_free(offt_mlp_s* m) {
    if (!m) return;
    for (void* d : m->allocs) (void)hipFree(d);
    delete m;
}

// SplitMix64 draw j of stream `key` mapped to [-1, 1).
static float mlp_uniform(uint64_t key, uint64_t j) {
    uint64_t z = key + (j + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (float)((double)(z >> 11) * 0x1.0p-52 - 1.0);
}

extern "C" {

int64_t offt_mlp_nparams(int in_dim, int hidden) {
    if (in_dim < 1 || hidden < 1 || hidden > 256) return OFFT_ERR_INVALID_ARG;
    return MlpLayout(in_dim, hidden).P;
}

void offt_mlp_init_params(int in_dim, int hidden, uint64_t seed, float* host_out) {
    // He-uniform weights (bound sqrt(6 / fan_in)), zero biases
    const MlpLayout lay(in_dim, hidden);
    for (int64_t q = 0; q < lay.P; ++q) host_out[q] = 0.f;
    const float s1 = std::sqrt(6.f / (float)in_dim), s2 = std::sqrt(6.f / (float)hidden);
    for (int64_t q = lay.W1; q < lay.b1; ++q) host_out[q] = s1 * mlp_uniform(seed, (uint64_t)q);
    for (int64_t q = lay.W2; q < lay.b2; ++q) host_out[q] = s2 * mlp_uniform(seed, (uint64_t)q);
    for (int64_t q = lay.w3; q < lay.b3; ++q) host_out[q] = s2 * mlp_uniform(seed, (uint64_t)q);
}

offt_mlp_t offt_mlp_create(int in_dim, int hidden, int max_batch, const float* host_params, uint64_t seed) {
    if (in_dim < 1 || hidden < 1 || hidden > 256 || max_batch < 1) { set_error(OFFT_ERR_INVALID_ARG); return nullptr; }
    int rc = check_device();
    if (rc != OFFT_SUCCESS) { set_error(rc); return nullptr; }
    offt_mlp_s* m = new offt_mlp_s();
    m->D = in_dim;
    m->H = hidden;
    m->max_batch = max_batch;
    m->P = MlpLayout(in_dim, hidden).P;
    auto alloc = [&](float** p, size_t n) {
        void* d = nullptr;
        if (hipMalloc(&d, n * sizeof(float)) != hipSuccess) { (void)hipGetLastError(); return false; }
        m->allocs.push_back(d);
        *p = static_cast<float*>(d);
        return true;
    };
    const size_t bh = (size_t)max_batch * hidden;
    if (!alloc(&m->params, m->P) || !alloc(&m->m, m->P) || !alloc(&m->v, m->P) || !alloc(&m->A1, bh) ||
        !alloc(&m->A2, bh) || !alloc(&m->Y, max_batch) || !alloc(&m->DY, max_batch) || !alloc(&m->G1, bh) ||
        !alloc(&m->G2, bh)) {
        mlp_free(m);
        set_error(OFFT_ERR_OUT_OF_MEMORY);
        return nullptr;
    }
    std::vector<float> init(m->P);
    if (host_params) memcpy(init.data(), host_params, sizeof(float) * m->P);
    else offt_mlp_init_params(in_dim, hidden, seed, init.data());
    if (hipMemcpy(m->params, init.data(), sizeof(float) * m->P, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(m->m, 0, sizeof(float) * m->P) != hipSuccess || hipMemset(m->v, 0, sizeof(float) * m->P) != hipSuccess) {
        mlp_free(m);
        set_error(OFFT_ERR_HIP);
        return nullptr;
    }
    set_error(OFFT_SUCCESS);
    return m;
}

int offt_mlp_destroy(offt_mlp_t m) {
    mlp_free(m);
    set_error(OFFT_SUCCESS);
    return OFFT_SUCCESS;
}

int offt_mlp_get_params(offt_mlp_t m, float* host_out) {
    if (!m || !host_out) { set_error(OFFT_ERR_INVALID_ARG); return OFFT_ERR_INVALID_ARG; }
    const int rc = hipMemcpy(host_out, m->params, sizeof(float) * m->P, hipMemcpyDeviceToHost) == hipSuccess
                       ? OFFT_SUCCESS : OFFT_ERR_HIP;
    set_error(rc);
    return rc;
}

int offt_mlp_set_params(offt_mlp_t m, const float* host_in) {
    if (!m || !host_in) { set_error(OFFT_ERR_INVALID_ARG); return OFFT_ERR_INVALID_ARG; }
    const int rc = hipMemcpy(m->params, host_in, sizeof(float) * m->P, hipMemcpyHostToDevice) == hipSuccess
                       ? OFFT_SUCCESS : OFFT_ERR_HIP;
    m->step = 0;
    (void)hipMemset(m->m, 0, sizeof(float) * m->P);
    (void)hipMemset(m->v, 0, sizeof(float) * m->P);
    set_error(rc);
    return rc;
}

int offt_mlp_forward(offt_mlp_t m, const float* X, const int32_t* idx, int B, float* y, void* stream) {
    if (!m || !X || !y || B < 1) { set_error(OFFT_ERR_INVALID_ARG); return OFFT_ERR_INVALID_ARG; }
    hipStream_t s = static_cast<hipStream_t>(stream);
    const size_t lds = sizeof(float) * (m->D + 2 * m->H);
    // one workgroup per row, at most 65535 workgroups per launch; the forward
    // pass alone keeps no activations
    for (int b0 = 0; b0 < B; b0 += 65535) {
        const int nb = std::min(65535, B - b0);
        hipLaunchKernelGGL(mlp_forward_kernel, dim3(nb), dim3(m->H), lds, s, m->params,
                           idx ? X : X + (int64_t)b0 * m->D, idx ? idx + b0 : nullptr, nb, m->D, m->H, y + b0,
                           nullptr, nullptr);
        if (hipGetLastError() != hipSuccess) { set_error(OFFT_ERR_HIP); return OFFT_ERR_HIP; }
    }
    set_error(OFFT_SUCCESS);
    return OFFT_SUCCESS;
}

int offt_mlp_gradient(offt_mlp_t m, const float* X, const float* T, const int32_t* idx, int B, float* grad,
                      float* loss, void* stream) {
    if (!m || !X || !T || !grad || B < 1 || B > m->max_batch) {
        set_error(OFFT_ERR_INVALID_ARG);
        return OFFT_ERR_INVALID_ARG;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    const size_t lds = sizeof(float) * (m->D + 2 * m->H);
    hipLaunchKernelGGL(mlp_forward_kernel, dim3(B), dim3(m->H), lds, s, m->params, X, idx, B, m->D, m->H, m->Y,
                       m->A1, m->A2);
    hipLaunchKernelGGL(mlp_delta_kernel, dim3(B), dim3(m->H), sizeof(float) * m->H, s, m->params, T, idx, B, m->D,
                       m->H, m->Y, m->A1, m->A2, m->DY, m->G1, m->G2);
    const int threads = 256;
    hipLaunchKernelGGL(mlp_grad_kernel, dim3((unsigned)((m->P + threads - 1) / threads)), dim3(threads), 0, s, X, idx,
                       B, m->D, m->H, m->A1, m->A2, m->DY, m->G1, m->G2, grad);
    if (loss) hipLaunchKernelGGL(mlp_loss_kernel, dim3(1), dim3(256), 0, s, m->Y, T, idx, B, loss);
    const int rc = hipGetLastError() == hipSuccess ? OFFT_SUCCESS : OFFT_ERR_HIP;
    set_error(rc);
    return rc;
}

int offt_mlp_adam(offt_mlp_t m, const float* grad, float lr, float beta1, float beta2, float eps, void* stream) {
    if (!m || !grad || !(lr > 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) ||
        !(eps > 0.f)) {
        set_error(OFFT_ERR_INVALID_ARG);
        return OFFT_ERR_INVALID_ARG;
    }
    m->step += 1;
    const float c1 = 1.f - std::pow(beta1, (float)m->step);
    const float c2 = 1.f - std::pow(beta2, (float)m->step);
    const int threads = 256;
    hipLaunchKernelGGL(mlp_adam_kernel, dim3((unsigned)((m->P + threads - 1) / threads)), dim3(threads), 0,
                       static_cast<hipStream_t>(stream), m->params, grad, m->m, m->v, m->P, lr, beta1, beta2, eps,
                       c1, c2);
    const int rc = hipGetLastError() == hipSuccess ? OFFT_SUCCESS : OFFT_ERR_HIP;
    set_error(rc);
    return rc;
}

}  // extern "C"
