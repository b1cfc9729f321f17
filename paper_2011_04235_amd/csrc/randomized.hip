// Kernels of the randomized inner solver (Section 3.3: a randomized truncated SVD with power
// iterations for the incremental updates at low target rank): the Gaussian test matrix from a
// counter-based generator, and the column scaling that turns the eigenvectors of a basis'
// Gram matrix into its orthonormalizing factor.
#include "kernels.h"

namespace fastpi {

namespace {

// Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC 2011): four 32-bit counter words, a 64-bit
// key, ten rounds of two 32x32->64 multiplications, the key bumped by the Weyl constants
// between rounds.
__device__ inline void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
    constexpr uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u, W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += W0;
            k1 += W1;
        }
        const uint64_t p0 = static_cast<uint64_t>(M0) * c[0];
        const uint64_t p1 = static_cast<uint64_t>(M1) * c[2];
        const uint32_t hi0 = static_cast<uint32_t>(p0 >> 32), lo0 = static_cast<uint32_t>(p0);
        const uint32_t hi1 = static_cast<uint32_t>(p1 >> 32), lo1 = static_cast<uint32_t>(p1);
        const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
    }
}

// out[e] for e < count, row-major: pair i = e / 2 draws counter (i low, i high, 0, 0) under key
// (seed, stream); two 53-bit uniforms u1 in (0, 1], u2 in [0, 1) and the Box-Muller transform
// give sqrt(-2 ln u1) cos(2 pi u2) (even e) and sqrt(-2 ln u1) sin(2 pi u2) (odd e).
__global__ __launch_bounds__(256) void k_gauss(double* __restrict__ out, int64_t count, uint32_t seed,
                                               uint32_t stream) {
    const int64_t pairs = (count + 1) / 2;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < pairs;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        uint32_t c[4] = {static_cast<uint32_t>(i), static_cast<uint32_t>(static_cast<uint64_t>(i) >> 32), 0u, 0u};
        philox4x32_10(c, seed, stream);
        const double two26 = 67108864.0, two_m53 = 1.1102230246251565e-16;
        const double u1 = (static_cast<double>(c[0] >> 5) * two26 + static_cast<double>(c[1] >> 6) + 1.0) * two_m53;
        const double u2 = (static_cast<double>(c[2] >> 5) * two26 + static_cast<double>(c[3] >> 6)) * two_m53;
        const double rad = sqrt(-2.0 * log(u1));
        const double ang = (2.0 * M_PI) * u2;
        out[2 * i] = rad * cos(ang);
        if (2 * i + 1 < count) out[2 * i + 1] = rad * sin(ang);
    }
}

// S[:, j] = V[:, j] / sqrt(d_j) for d_j > cut * d_0, else 0 (V: k x k row-major eigenvectors
// of a Gram matrix, d descending).
__global__ __launch_bounds__(256) void k_scale_cols(const double* __restrict__ V, const double* __restrict__ d,
                                                    int64_t k, double cut, double* __restrict__ S) {
    const double lim = cut * d[0];
    for (int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; e < k * k;
         e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const double dj = d[e % k];
        S[e] = dj > lim ? V[e] / sqrt(dj) : 0.0;
    }
}

// One workgroup per column of V (rows x cols, row-major): negate the column unless its entry
// of largest magnitude (the first such entry on ties) is positive.
__global__ __launch_bounds__(256) void k_sign_fix(double* __restrict__ V, int64_t rows, int64_t cols) {
    __shared__ double s_v[4];
    __shared__ int64_t s_i[4];
    const int64_t j = blockIdx.x;
    double bv = -1.0;
    int64_t bi = rows;
    for (int64_t i = threadIdx.x; i < rows; i += blockDim.x) {
        const double a = fabs(V[i * cols + j]);
        if (a > bv) {   // rows ascend per thread: keeps the first on ties
            bv = a;
            bi = i;
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        const double ov = __shfl_xor(bv, off, 64);
        const int64_t oi = __shfl_xor(bi, off, 64);
        if (ov > bv || (ov == bv && oi < bi)) {
            bv = ov;
            bi = oi;
        }
    }
    const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
    if (lane == 0) {
        s_v[wave] = bv;
        s_i[wave] = bi;
    }
    __syncthreads();
    double v = s_v[0];
    int64_t i0 = s_i[0];
    for (int w = 1; w < 4; ++w)
        if (s_v[w] > v || (s_v[w] == v && s_i[w] < i0)) {
            v = s_v[w];
            i0 = s_i[w];
        }
    if (i0 >= rows) return;
    const bool flip = V[i0 * cols + j] < 0.0;
    __syncthreads();   // every thread has read the leading entry before any is negated
    if (flip)
        for (int64_t i = threadIdx.x; i < rows; i += blockDim.x) V[i * cols + j] = -V[i * cols + j];
}

unsigned grid_for(int64_t work) {
    const int64_t g = (work + 255) / 256;
    return static_cast<unsigned>(std::max<int64_t>(1, std::min<int64_t>(g, 65536)));
}

}  // namespace

void launch_gauss(double* out, int64_t count, uint32_t seed, uint32_t stream, hipStream_t st) {
    if (count <= 0) return;
    hipLaunchKernelGGL(k_gauss, dim3(grid_for((count + 1) / 2)), dim3(256), 0, st, out, count, seed, stream);
}

void launch_sign_fix(double* V, int64_t rows, int64_t cols, hipStream_t st) {
    if (rows <= 0 || cols <= 0) return;
    hipLaunchKernelGGL(k_sign_fix, dim3(static_cast<unsigned>(cols)), dim3(256), 0, st, V, rows, cols);
}

void launch_scale_cols(const double* V, const double* d, int64_t k, double cut, double* S, hipStream_t st) {
    if (k <= 0) return;
    hipLaunchKernelGGL(k_scale_cols, dim3(grid_for(k * k)), dim3(256), 0, st, V, d, k, cut, S);
}

}  // namespace fastpi
