// Dense products on the matrix cores: C = op(A) op(B) with FP64 storage, computed by
// v_mfma_f64_16x16x4f64 (Tc = double) or v_mfma_f32_16x16x4f32 (Tc = float, the mixed form:
// operands rounded to FP32 on their way into LDS, FP32 accumulation).
//
// Workgroup tile 128 x 128, 256 threads = 4 waves in a 2 x 2 grid, each wave a 64 x 64 block
// of 4 x 4 MFMA tiles (16 accumulators of 4 values per lane). K advances in slices of 16:
// the next slice is loaded from global memory into registers while the current one is
// multiplied out of LDS. LDS holds both operands k-major (As[k][m], Bs[k][n]), so a
// fragment load (16 consecutive m or n per k) is conflict-free; rows are padded by 4.
//
// MFMA 16x16x4 operand layout (gfx950, checked on the device): lane l supplies
// A[i = l % 16][k = l / 16] and B[k = l / 16][j = l % 16]; its 4 results r = 0..3 are
// D[i][j = l % 16] with i = 4 (l / 16) + r for the FP32 instruction and i = 4 r + l / 16 for
// the FP64 one.
//
// op(A): TA = false, A is M x K row-major (lda); TA = true, A is stored K x M (A^T row-major).
// op(B): TB = false, B is K x N row-major (ldb); TB = true, B is stored N x K.
// Split K: blockIdx.z takes rows [z kchunk, (z + 1) kchunk) of K and writes C + z * cstride.
// GA (with TA = TB = false, no split): row i of A is row arow[i] of the stored A and row i
// of C goes to row crow[i] (either map may be null: the identity).
#include "device_common.h"
#include "kernels.h"

namespace fastpi {

namespace {

constexpr int MT = 128, NT = 128, KT = 16, PAD = 4;

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

template <typename Tc>
struct Mfma;

template <>
struct Mfma<double> {
    typedef v4d acc_t;
    static __device__ __forceinline__ acc_t step(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lk, int r) { return 4 * r + lk; }
};

template <>
struct Mfma<float> {
    typedef v4f acc_t;
    static __device__ __forceinline__ acc_t step(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lk, int r) { return 4 * lk + r; }
};

template <typename Tc, bool TA, bool TB, bool GA>
__global__ __launch_bounds__(256) void k_mfma_gemm(const double* __restrict__ A, int64_t lda,
                                                   const double* __restrict__ B, int64_t ldb, int64_t M,
                                                   int64_t N, int64_t K, int64_t kchunk, double* __restrict__ C,
                                                   int64_t ldc, int64_t cstride, const int* __restrict__ arow,
                                                   const int* __restrict__ crow) {
    static_assert(!GA || (!TA && !TB), "row maps only for C = A B");
    typedef typename Mfma<Tc>::acc_t acc_t;
    __shared__ Tc As[KT][MT + PAD];
    __shared__ Tc Bs[KT][NT + PAD];
    const int tid = threadIdx.x, lane = tid % 64, w = tid / 64;
    const int wm = w / 2, wn = w % 2;
    // Tile order: workgroups are dealt to the 8 XCDs round robin by their linear id, and each
    // XCD has its own L2. The linear id is remapped so that each XCD gets a contiguous range
    // of tiles, numbered with the N tile fastest: the tiles sharing a row band of op(A) then
    // run on one XCD and reuse it from that L2 (op(B) stays in the shared MALL).
    const int nx = gridDim.x, ny = gridDim.y;
    const int ntile = nx * ny;
    const int lin = blockIdx.x + nx * blockIdx.y;
    const int per = ntile / 8, extra = ntile % 8, xcd = lin % 8, slot = lin / 8;
    const int tile = (xcd < extra ? xcd * (per + 1) : extra * (per + 1) + (xcd - extra) * per) + slot;
    const int64_t i0 = static_cast<int64_t>(tile / ny) * MT;
    const int64_t j0 = static_cast<int64_t>(tile % ny) * NT;
    const int64_t kb = static_cast<int64_t>(blockIdx.z) * kchunk;
    const int64_t ke = min(K, kb + kchunk);
    C += static_cast<int64_t>(blockIdx.z) * cstride;

    // each thread moves 8 elements of each operand per slice; with GA its 8 rows of A
    // (i0 + tid / 16 + 16 u) are mapped once
    int64_t arow_u[GA ? 8 : 1];
    if (GA) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int64_t i = i0 + tid / KT + 16 * u;
            arow_u[u] = (i < M && arow) ? static_cast<int64_t>(arow[i]) : i;
        }
    }
    double ra[8], rb[8];
    auto load = [&](int64_t k0) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = tid + 256 * u;
            int kk, ii;
            if (TA) {   // stored K x M: contiguous along m
                kk = e / MT;
                ii = e % MT;
            } else {    // M x K: contiguous along k
                ii = e / KT;
                kk = e % KT;
            }
            const int64_t k = k0 + kk, i = i0 + ii;
            if (GA)
                ra[u] = (k < ke && i < M) ? A[arow_u[u] * lda + k] : 0.0;
            else
                ra[u] = (k < ke && i < M) ? (TA ? A[k * lda + i] : A[i * lda + k]) : 0.0;
            int jj, kk2;
            if (TB) {   // stored N x K: contiguous along k
                jj = e / KT;
                kk2 = e % KT;
            } else {    // K x N: contiguous along n
                kk2 = e / NT;
                jj = e % NT;
            }
            const int64_t k2 = k0 + kk2, j = j0 + jj;
            rb[u] = (k2 < ke && j < N) ? (TB ? B[j * ldb + k2] : B[k2 * ldb + j]) : 0.0;
        }
    };
    auto store = [&]() {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = tid + 256 * u;
            if (TA) As[e / MT][e % MT] = static_cast<Tc>(ra[u]);
            else As[e % KT][e / KT] = static_cast<Tc>(ra[u]);
            if (TB) Bs[e % KT][e / KT] = static_cast<Tc>(rb[u]);
            else Bs[e / NT][e % NT] = static_cast<Tc>(rb[u]);
        }
    };

    acc_t acc[4][4];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[r][c] = acc_t{0, 0, 0, 0};

    const int lr = lane % 16, lk = lane / 16;
    if (kb < ke) load(kb);
    for (int64_t k0 = kb; k0 < ke; k0 += KT) {
        store();
        __syncthreads();
        if (k0 + KT < ke) load(k0 + KT);
#pragma unroll
        for (int k4 = 0; k4 < KT; k4 += 4) {
            Tc a[4], b[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) a[r] = As[k4 + lk][wm * 64 + r * 16 + lr];
#pragma unroll
            for (int c = 0; c < 4; ++c) b[c] = Bs[k4 + lk][wn * 64 + c * 16 + lr];
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int c = 0; c < 4; ++c) acc[r][c] = Mfma<Tc>::step(a[r], b[c], acc[r][c]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int64_t j = j0 + wn * 64 + c * 16 + lr;
            if (j >= N) continue;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t i = i0 + wm * 64 + r * 16 + Mfma<Tc>::row(lk, v);
                if (i >= M) continue;
                const int64_t ci = (GA && crow) ? static_cast<int64_t>(crow[i]) : i;
                C[ci * ldc + j] = static_cast<double>(acc[r][c][v]);
            }
        }
}

}  // namespace

// C (M x N, ldc) = op(A) op(B) over K, on the matrix cores; nsplit > 1 writes nsplit partial
// products of K chunks to C + z * cstride (the caller sums them).
void launch_mfma_gemm(bool ta, bool tb, const double* A, int64_t lda, const double* B, int64_t ldb, int64_t M,
                      int64_t N, int64_t K, double* C, int64_t ldc, int nsplit, int64_t cstride, hipStream_t st,
                      bool fp32, KernelTimer* timer, int kind) {
    if (M <= 0 || N <= 0) return;
    const int* arow = nullptr;
    const int* crow = nullptr;
    nsplit = std::max(1, nsplit);
    const int64_t kchunk = std::max<int64_t>(KT, ((K + nsplit - 1) / nsplit + KT - 1) / KT * KT);
    dim3 grid(static_cast<unsigned>((M + MT - 1) / MT), static_cast<unsigned>((N + NT - 1) / NT),
              static_cast<unsigned>(nsplit));
#define FASTPI_MG(TC, TAV, TBV, GAV)                                                                           \
    FASTPI_LAUNCH(timer, kind, (k_mfma_gemm<TC, TAV, TBV, GAV>), grid, dim3(256), 0, st, A, lda, B, ldb, M, N, K,  \
                  kchunk, C, ldc, cstride, arow, crow)
    if (fp32) {
        if (ta) {
            if (tb) FASTPI_MG(float, true, true, false); else FASTPI_MG(float, true, false, false);
        } else {
            if (tb) FASTPI_MG(float, false, true, false); else FASTPI_MG(float, false, false, false);
        }
    } else {
        if (ta) {
            if (tb) FASTPI_MG(double, true, true, false); else FASTPI_MG(double, true, false, false);
        } else {
            if (tb) FASTPI_MG(double, false, true, false); else FASTPI_MG(double, false, false, false);
        }
    }
#undef FASTPI_MG
}

// C[crow(i)] = A[arow(i)] B (C = A B with a row gather of A and a row scatter of C; either
// map may be null), on the matrix cores, unsplit.
void launch_mfma_gemm_rows(const double* A, int64_t lda, const int* arow, const double* B, int64_t ldb, int64_t M,
                           int64_t N, int64_t K, double* C, int64_t ldc, const int* crow, hipStream_t st, bool fp32) {
    if (M <= 0 || N <= 0) return;
    dim3 grid(static_cast<unsigned>((M + MT - 1) / MT), static_cast<unsigned>((N + NT - 1) / NT), 1);
    const int64_t kchunk = std::max<int64_t>(KT, (K + KT - 1) / KT * KT);
    if (fp32)
        hipLaunchKernelGGL((k_mfma_gemm<float, false, false, true>), grid, dim3(256), 0, st, A, lda, B, ldb, M, N, K,
                           kchunk, C, ldc, int64_t{0}, arow, crow);
    else
        hipLaunchKernelGGL((k_mfma_gemm<double, false, false, true>), grid, dim3(256), 0, st, A, lda, B, ldb, M, N, K,
                           kchunk, C, ldc, int64_t{0}, arow, crow);
}

}  // namespace fastpi
