// Dense FP64 contractions of the update and apply steps (Eqs. 2-3, Problem 1).
//
// On gfx950 the FP64 matrix-core peak equals the FP64 vector-FMA peak (78.6 TFLOP/s), so
// these are register-tiled FMA kernels: a 256-thread workgroup computes a 64 x 64 tile of C,
// each thread a 4 x 4 micro-tile, with 16-deep slices of A and B staged in LDS. The compute
// type Tc is double (FP64 path) or float (mixed path: operands rounded to FP32 on load,
// products accumulated in FP32, results stored as FP64).
//
//   gemm_tn : C_part[z] = A[kz]^T B[kz]  (A: K x M, B: K x N, both row-major; split over K)
//   gemm_nn : C[ci(i)] = A[ai(i)] B        (A: M x K row-major with optional row gather,
//                                            B: K x N row-major, optional C row scatter)
//   gemm_nt : C = A B^T                    (A: M x K, B: N x K, both row-major)
#include "device_common.h"
#include "kernels.h"

namespace fastpi {

constexpr int TM = 64, TN = 64, TK = 16;

template <typename Tc>
__global__ __launch_bounds__(256) void k_gemm_tn(const double* __restrict__ A, int64_t lda,
                                                 const double* __restrict__ B, int64_t ldb,
                                                 int64_t M, int64_t N, int64_t K, int64_t kchunk,
                                                 double* __restrict__ Cpart) {
    __shared__ Tc As[TK][TM + 2];
    __shared__ Tc Bs[TK][TN + 2];
    const int64_t i0 = static_cast<int64_t>(blockIdx.x) * TM;
    const int64_t j0 = static_cast<int64_t>(blockIdx.y) * TN;
    const int64_t kb = static_cast<int64_t>(blockIdx.z) * kchunk;
    const int64_t ke = min(K, kb + kchunk);
    const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
    Tc acc[4][4] = {};
    for (int64_t k0 = kb; k0 < ke; k0 += TK) {
        for (int e = threadIdx.x; e < TK * TM; e += 256) {
            const int kk = e / TM, ii = e % TM;
            const int64_t k = k0 + kk, i = i0 + ii;
            As[kk][ii] = static_cast<Tc>((k < ke && i < M) ? A[k * lda + i] : 0.0);
        }
        for (int e = threadIdx.x; e < TK * TN; e += 256) {
            const int kk = e / TN, jj = e % TN;
            const int64_t k = k0 + kk, j = j0 + jj;
            Bs[kk][jj] = static_cast<Tc>((k < ke && j < N) ? B[k * ldb + j] : 0.0);
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < TK; ++kk) {
            Tc a[4], b[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                a[u] = As[kk][ty * 4 + u];
                b[u] = Bs[kk][tx * 4 + u];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[u][v] += a[u] * b[v];
        }
        __syncthreads();
    }
    double* C = Cpart + static_cast<int64_t>(blockIdx.z) * M * N;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int64_t i = i0 + ty * 4 + u;
        if (i >= M) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int64_t j = j0 + tx * 4 + v;
            if (j < N) C[i * N + j] = static_cast<double>(acc[u][v]);
        }
    }
}

// C[i*ldc + j] = rs[i] * cs[j] * sum_z Cpart[z][i][j]  (rs, cs may be null = 1)
__global__ void k_reduce_parts(const double* __restrict__ Cpart, int nsplit, int64_t M, int64_t N,
                               double* __restrict__ C, int64_t ldc, const double* __restrict__ rs,
                               const double* __restrict__ cs) {
    const int64_t n = M * N;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; e < n; e += stride) {
        double acc = 0;
        for (int z = 0; z < nsplit; ++z) acc += Cpart[static_cast<int64_t>(z) * n + e];
        const int64_t i = e / N, j = e % N;
        if (rs) acc *= rs[i];
        if (cs) acc *= cs[j];
        C[i * ldc + j] = acc;
    }
}

template <typename Tc, bool TB>
__global__ __launch_bounds__(256) void k_gemm_nn(const double* __restrict__ A, int64_t lda,
                                                 const int* __restrict__ arow,
                                                 const double* __restrict__ B, int64_t ldb,
                                                 int64_t M, int64_t N, int64_t K,
                                                 double* __restrict__ C, int64_t ldc,
                                                 const int* __restrict__ crow) {
    __shared__ Tc As[TK][TM + 2];
    __shared__ Tc Bs[TK][TN + 2];
    const int64_t i0 = static_cast<int64_t>(blockIdx.x) * TM;
    const int64_t j0 = static_cast<int64_t>(blockIdx.y) * TN;
    const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
    Tc acc[4][4] = {};
    for (int64_t k0 = 0; k0 < K; k0 += TK) {
        for (int e = threadIdx.x; e < TK * TM; e += 256) {
            const int ii = e / TK, kk = e % TK;
            const int64_t k = k0 + kk, i = i0 + ii;
            double v = 0.0;
            if (k < K && i < M) {
                const int64_t ar = arow ? arow[i] : i;
                v = A[ar * lda + k];
            }
            As[kk][ii] = static_cast<Tc>(v);
        }
        for (int e = threadIdx.x; e < TK * TN; e += 256) {
            if (TB) {   // B is N x K row-major: read along k
                const int jj = e / TK, kk = e % TK;
                const int64_t k = k0 + kk, j = j0 + jj;
                Bs[kk][jj] = static_cast<Tc>((k < K && j < N) ? B[j * ldb + k] : 0.0);
            } else {
                const int kk = e / TN, jj = e % TN;
                const int64_t k = k0 + kk, j = j0 + jj;
                Bs[kk][jj] = static_cast<Tc>((k < K && j < N) ? B[k * ldb + j] : 0.0);
            }
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < TK; ++kk) {
            Tc a[4], b[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                a[u] = As[kk][ty * 4 + u];
                b[u] = Bs[kk][tx * 4 + u];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[u][v] += a[u] * b[v];
        }
        __syncthreads();
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int64_t i = i0 + ty * 4 + u;
        if (i >= M) continue;
        const int64_t ci = crow ? crow[i] : i;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int64_t j = j0 + tx * 4 + v;
            if (j < N) C[ci * ldc + j] = static_cast<double>(acc[u][v]);
        }
    }
}

// products big enough for the 128 x 128 matrix-core tiles go there
static bool use_mfma(int64_t M, int64_t N, int64_t K) { return M >= 128 && N >= 64 && K >= 64; }

int gemm_tn_splits(int64_t M, int64_t N, int64_t K, bool fp32, int ncu) {
    // chunks of at least 256 rows of K
    const int64_t smax = std::max<int64_t>(1, std::min<int64_t>(256, (K + 255) / 256));
    if (M <= 0 || N <= 0) return 1;   // empty product (e.g. a core of rank 0)
    if (use_mfma(M, N, K)) {
        // matrix cores: whole waves of the resident workgroups (two per CU in FP32, one in
        // FP64). s minimises the estimated time: the waves times one workgroup's share of a
        // tile (2 * 128^2 * K / s flops at ~120 GFLOP/s per resident workgroup), plus the s
        // partials written and summed (16 M N bytes each at ~4 TB/s)
        const int64_t tiles = ((M + 127) / 128) * ((N + 127) / 128);
        const int64_t slots = static_cast<int64_t>(fp32 ? 2 : 1) * std::max(1, ncu);
        const double t_tile = 2.0 * 128.0 * 128.0 * static_cast<double>(K) / 1.2e11;
        const double t_part = 16.0 * static_cast<double>(M) * static_cast<double>(N) / 4.0e12;
        int64_t best_s = 1;
        double best = 1e30;
        for (int64_t s = 1; s <= smax; ++s) {
            const double c = static_cast<double>((tiles * s + slots - 1) / slots) * t_tile / static_cast<double>(s) +
                             static_cast<double>(s) * t_part;
            if (c < best - 1e-12) {
                best = c;
                best_s = s;
            }
        }
        return static_cast<int>(best_s);
    }
    // FMA kernel: enough 64 x 64 tiles to cover the chip (~4 workgroups per CU)
    const int64_t tiles = ((M + TM - 1) / TM) * ((N + TN - 1) / TN);
    return static_cast<int>(std::max<int64_t>(1, std::min<int64_t>((1024 + tiles - 1) / tiles, smax)));
}

void launch_sum_parts(const double* part, int nsplit, int64_t M, int64_t N, double* C, int64_t ldc, hipStream_t st) {
    const int64_t n = M * N;
    if (n <= 0) return;
    hipLaunchKernelGGL(k_reduce_parts, dim3(static_cast<unsigned>(std::min<int64_t>((n + 255) / 256, 8192))), dim3(256),
                       0, st, part, nsplit, M, N, C, ldc, nullptr, nullptr);
}

void launch_gemm_tn(const double* A, int64_t lda, const double* B, int64_t ldb, int64_t M,
                    int64_t N, int64_t K, double* C, int64_t ldc, const double* rs,
                    const double* cs, double* part, int nsplit, hipStream_t st, bool fp32) {
    if (M <= 0 || N <= 0) return;
    if (use_mfma(M, N, K)) {
        launch_mfma_gemm(true, false, A, lda, B, ldb, M, N, K, part, N, nsplit, M * N, st, fp32);
        const int64_t n = M * N;
        hipLaunchKernelGGL(k_reduce_parts, dim3(static_cast<unsigned>(std::min<int64_t>((n + 255) / 256, 8192))),
                           dim3(256), 0, st, part, nsplit, M, N, C, ldc, rs, cs);
        return;
    }
    const int64_t kchunk = ((K + nsplit - 1) / nsplit + TK - 1) / TK * TK;
    dim3 grid(static_cast<unsigned>((M + TM - 1) / TM), static_cast<unsigned>((N + TN - 1) / TN),
              static_cast<unsigned>(nsplit));
    if (fp32)
        hipLaunchKernelGGL(k_gemm_tn<float>, grid, dim3(256), 0, st, A, lda, B, ldb, M, N, K,
                           std::max<int64_t>(kchunk, TK), part);
    else
        hipLaunchKernelGGL(k_gemm_tn<double>, grid, dim3(256), 0, st, A, lda, B, ldb, M, N, K,
                           std::max<int64_t>(kchunk, TK), part);
    const int64_t n = M * N;
    hipLaunchKernelGGL(k_reduce_parts, dim3(static_cast<unsigned>(std::min<int64_t>((n + 255) / 256, 8192))),
                       dim3(256), 0, st, part, nsplit, M, N, C, ldc, rs, cs);
}

void launch_gemm_nn(const double* A, int64_t lda, const int* arow, const double* B, int64_t ldb,
                    int64_t M, int64_t N, int64_t K, double* C, int64_t ldc, const int* crow,
                    hipStream_t st, bool fp32, KernelTimer* timer, int kind) {
    if (M <= 0 || N <= 0) return;
    if (use_mfma(M, N, K)) {
        if (arow || crow)
            launch_mfma_gemm_rows(A, lda, arow, B, ldb, M, N, K, C, ldc, crow, st, fp32);
        else
            launch_mfma_gemm(false, false, A, lda, B, ldb, M, N, K, C, ldc, 1, 0, st, fp32, timer, kind);
        return;
    }
    dim3 grid(static_cast<unsigned>((M + TM - 1) / TM), static_cast<unsigned>((N + TN - 1) / TN));
    if (fp32)
        hipLaunchKernelGGL((k_gemm_nn<float, false>), grid, dim3(256), 0, st, A, lda, arow, B, ldb, M, N, K, C,
                           ldc, crow);
    else
        hipLaunchKernelGGL((k_gemm_nn<double, false>), grid, dim3(256), 0, st, A, lda, arow, B, ldb, M, N, K, C,
                           ldc, crow);
}

void launch_gemm_nt(const double* A, int64_t lda, const double* B, int64_t ldb, int64_t M, int64_t N,
                    int64_t K, double* C, int64_t ldc, hipStream_t st, bool fp32, KernelTimer* timer) {
    if (M <= 0 || N <= 0) return;
    if (use_mfma(M, N, K)) {
        launch_mfma_gemm(false, true, A, lda, B, ldb, M, N, K, C, ldc, 1, 0, st, fp32, timer, KT_GEMM_NT);
        return;
    }
    dim3 grid(static_cast<unsigned>((M + TM - 1) / TM), static_cast<unsigned>((N + TN - 1) / TN));
    const int* none = nullptr;
    if (fp32)
        FASTPI_LAUNCH(timer, KT_GEMM_NT, (k_gemm_nn<float, true>), grid, dim3(256), 0, st, A, lda, none, B, ldb, M,
                      N, K, C, ldc, none);
    else
        FASTPI_LAUNCH(timer, KT_GEMM_NT, (k_gemm_nn<double, true>), grid, dim3(256), 0, st, A, lda, none, B, ldb,
                      M, N, K, C, ldc, none);
}

}  // namespace fastpi
