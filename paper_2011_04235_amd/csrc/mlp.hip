// Per-block rank predictor: a 16-64-64-1 network (ReLU, ReLU, sigmoid) trained on the GPU
// with mean squared error on the kept fraction f = s_i / min(m_i, n_i), and Adam.
//
// Packed FP32 parameters (5313): W1 (64 x 16, row-major), b1 (64), W2 (64 x 64), b2 (64),
// W3 (64), b3. Samples are rows of X (N x 16). Gradients are summed over samples in a fixed
// order (per-chunk partial sums, then chunks in order): no floating-point atomics.
#include <cmath>

#include "device_common.h"
#include "kernels.h"

namespace fastpi {

constexpr int NF = 16, NH1 = 64, NH2 = 64;
constexpr int OW1 = 0, OB1 = OW1 + NH1 * NF, OW2 = OB1 + NH1, OB2 = OW2 + NH2 * NH1,
              OW3 = OB2 + NH2, OB3 = OW3 + NH2, NPARAM = OB3 + 1;
constexpr int ACT = NH1 + NH2;          // stored activations per sample
constexpr int DZ = 1 + NH2 + NH1;       // stored deltas per sample: dz3, dz2, dz1
constexpr int WG_CHUNK = 512;           // samples per partial-gradient chunk

int mlp_param_count() { return NPARAM; }

// one thread per sample; parameters staged in LDS (read as broadcasts)
__global__ __launch_bounds__(256) void k_mlp_forward(int64_t N, const float* __restrict__ X,
                                                     const float* __restrict__ th,
                                                     float* __restrict__ f, float* __restrict__ act) {
    __shared__ float P[NPARAM];
    for (int e = threadIdx.x; e < NPARAM; e += blockDim.x) P[e] = th[e];
    __syncthreads();
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= N) return;
    float x[NF];
#pragma unroll
    for (int k = 0; k < NF; ++k) x[k] = X[i * NF + k];
    float h1[NH1];
#pragma unroll 4
    for (int j = 0; j < NH1; ++j) {
        float z = P[OB1 + j];
#pragma unroll
        for (int k = 0; k < NF; ++k) z += P[OW1 + j * NF + k] * x[k];
        h1[j] = z > 0.f ? z : 0.f;
    }
    float z3 = P[OB3];
    for (int j = 0; j < NH2; ++j) {
        float z = P[OB2 + j];
#pragma unroll
        for (int k = 0; k < NH1; ++k) z += P[OW2 + j * NH1 + k] * h1[k];
        const float h2 = z > 0.f ? z : 0.f;
        z3 += P[OW3 + j] * h2;
        if (act) act[i * ACT + NH1 + j] = h2;
    }
    if (act) {
#pragma unroll 4
        for (int j = 0; j < NH1; ++j) act[i * ACT + j] = h1[j];
    }
    f[i] = 1.f / (1.f + expf(-z3));
}

// per-sample deltas of the mean squared error: dz3 = (2/N)(f - y) f (1 - f),
// dz2 = dz3 W3 . [z2 > 0], dz1 = (W2^T dz2) . [z1 > 0]
__global__ __launch_bounds__(256) void k_mlp_delta(int64_t N, const float* __restrict__ y,
                                                   const float* __restrict__ th,
                                                   const float* __restrict__ act,
                                                   const float* __restrict__ f, float* __restrict__ dz) {
    __shared__ float P[NPARAM];
    for (int e = threadIdx.x; e < NPARAM; e += blockDim.x) P[e] = th[e];
    __syncthreads();
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const float fi = f[i];
    const float d3 = (2.f / static_cast<float>(N)) * (fi - y[i]) * fi * (1.f - fi);
    float d2[NH2];
#pragma unroll 4
    for (int j = 0; j < NH2; ++j) {
        const float h2 = act[i * ACT + NH1 + j];
        d2[j] = h2 > 0.f ? d3 * P[OW3 + j] : 0.f;
    }
    float* out = dz + i * DZ;
    out[0] = d3;
#pragma unroll 4
    for (int j = 0; j < NH2; ++j) out[1 + j] = d2[j];
    for (int k = 0; k < NH1; ++k) {
        float s = 0.f;
#pragma unroll
        for (int j = 0; j < NH2; ++j) s += P[OW2 + j * NH1 + k] * d2[j];
        out[1 + NH2 + k] = act[i * ACT + k] > 0.f ? s : 0.f;
    }
}

// partial gradient of every parameter over one chunk of samples (one thread per parameter,
// samples visited in order)
__global__ __launch_bounds__(256) void k_mlp_wgrad(int64_t N, const float* __restrict__ X,
                                                   const float* __restrict__ act,
                                                   const float* __restrict__ dz,
                                                   float* __restrict__ part) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= NPARAM) return;
    const int64_t i0 = static_cast<int64_t>(blockIdx.y) * WG_CHUNK;
    const int64_t i1 = min(N, i0 + WG_CHUNK);
    float g = 0.f;
    if (p < OB1) {
        const int j = (p - OW1) / NF, k = (p - OW1) % NF;
        for (int64_t i = i0; i < i1; ++i) g += dz[i * DZ + 1 + NH2 + j] * X[i * NF + k];
    } else if (p < OW2) {
        const int j = p - OB1;
        for (int64_t i = i0; i < i1; ++i) g += dz[i * DZ + 1 + NH2 + j];
    } else if (p < OB2) {
        const int j = (p - OW2) / NH1, k = (p - OW2) % NH1;
        for (int64_t i = i0; i < i1; ++i) g += dz[i * DZ + 1 + j] * act[i * ACT + k];
    } else if (p < OW3) {
        const int j = p - OB2;
        for (int64_t i = i0; i < i1; ++i) g += dz[i * DZ + 1 + j];
    } else if (p < OB3) {
        const int k = p - OW3;
        for (int64_t i = i0; i < i1; ++i) g += dz[i * DZ] * act[i * ACT + NH1 + k];
    } else {
        for (int64_t i = i0; i < i1; ++i) g += dz[i * DZ];
    }
    part[static_cast<int64_t>(blockIdx.y) * NPARAM + p] = g;
}

__global__ void k_mlp_reduce(const float* __restrict__ part, int nchunk, float* __restrict__ grad) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= NPARAM) return;
    float g = 0.f;
    for (int c = 0; c < nchunk; ++c) g += part[static_cast<int64_t>(c) * NPARAM + p];
    grad[p] = g;
}

// Adam (Kingma & Ba): m <- b1 m + (1-b1) g, v <- b2 v + (1-b2) g^2,
// theta <- theta - lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)
__global__ void k_mlp_adam(float* __restrict__ th, const float* __restrict__ g, float* __restrict__ m,
                           float* __restrict__ v, float lr, float b1, float b2, float eps, float c1,
                           float c2) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= NPARAM) return;
    const float gi = g[p];
    const float mi = b1 * m[p] + (1.f - b1) * gi;
    const float vi = b2 * v[p] + (1.f - b2) * gi * gi;
    m[p] = mi;
    v[p] = vi;
    th[p] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

size_t mlp_scratch_floats(int64_t N) {
    const int64_t nchunk = (N + WG_CHUNK - 1) / WG_CHUNK;
    return static_cast<size_t>(N * ACT + N * DZ + N + nchunk * NPARAM + 64);
}

void launch_mlp_forward(int64_t N, const float* X, const float* th, float* f, float* act,
                        hipStream_t st) {
    if (N <= 0) return;
    hipLaunchKernelGGL(k_mlp_forward, dim3(static_cast<unsigned>((N + 255) / 256)), dim3(256), 0, st, N, X,
                       th, f, act);
}

void launch_mlp_gradient(int64_t N, const float* X, const float* y, const float* th, float* grad,
                         float* scratch, hipStream_t st) {
    if (N <= 0) return;
    float* act = scratch;
    float* dz = act + N * ACT;
    float* f = dz + N * DZ;
    float* part = f + N;
    const int nchunk = static_cast<int>((N + WG_CHUNK - 1) / WG_CHUNK);
    const unsigned nb = static_cast<unsigned>((N + 255) / 256);
    hipLaunchKernelGGL(k_mlp_forward, dim3(nb), dim3(256), 0, st, N, X, th, f, act);
    hipLaunchKernelGGL(k_mlp_delta, dim3(nb), dim3(256), 0, st, N, y, th, act, f, dz);
    hipLaunchKernelGGL(k_mlp_wgrad, dim3((NPARAM + 255) / 256, nchunk), dim3(256), 0, st, N, X, act, dz, part);
    hipLaunchKernelGGL(k_mlp_reduce, dim3((NPARAM + 255) / 256), dim3(256), 0, st, part, nchunk, grad);
}

void launch_mlp_adam(float* th, const float* g, float* m, float* v, int64_t step, float lr,
                     hipStream_t st) {
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float c1 = 1.f - std::pow(b1, static_cast<float>(step));
    const float c2 = 1.f - std::pow(b2, static_cast<float>(step));
    hipLaunchKernelGGL(k_mlp_adam, dim3((NPARAM + 255) / 256), dim3(256), 0, st, th, g, m, v, lr, b1, b2, eps,
                       c1, c2);
}

}  // namespace fastpi
