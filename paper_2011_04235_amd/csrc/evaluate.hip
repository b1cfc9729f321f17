// Evaluation of the multi-label regression (Application 1) on held-out rows: the score
// vector yhat = Z^T x of each test row, its k top-ranked labels and the top-k precision
// counts of the accuracy experiment (Section 4).
//
// One workgroup per test row (a grid-stride loop over rows). The scores live in LDS when
// L <= kTopkLdsLabels, else in a per-workgroup slice of a device scratch buffer; every label's
// score is accumulated over the row's stored entries in CSR order with one rounded multiply
// and one rounded add per entry, so the integer decision below is taken on scores of a
// stated precision and order. Labels are ranked by repeated workgroup argmax (ties go to the
// lower label); a taken label's score is replaced by NaN, which never wins a comparison.
#include "kernels.h"

namespace fastpi {

namespace {

constexpr int kEvalThreads = 256;
constexpr int kEvalWaves = kEvalThreads / 64;

struct KList {
    int n;
    int k[kTopkMaxKs];
};

// (a, ia) ranks before (b, ib): a higher score, or an equal score at a lower label.
// A NaN score ranks before nothing.
__device__ inline bool ranks_before(double a, int ia, double b, int ib) {
    return a > b || (a == b && ia < ib);
}

template <bool GLOBAL>
__global__ __launch_bounds__(kEvalThreads) void k_topk_hits(
    int64_t rows, int64_t n, int64_t L, const int64_t* __restrict__ a_rowptr, const int* __restrict__ a_col,
    const double* __restrict__ a_val, const double* __restrict__ Z,
    const int64_t* __restrict__ y_rowptr, const int* __restrict__ y_col, KList ks, int kmax,
    int* __restrict__ hits, double* __restrict__ scratch) {
#pragma clang fp contract(off)
    extern __shared__ double s_lds[];
    __shared__ double s_bv[kEvalWaves];
    __shared__ int s_bi[kEvalWaves];
    __shared__ int s_top[kTopkMaxK];
    __shared__ int s_hit[kTopkMaxK];
    double* s_score = GLOBAL ? scratch + static_cast<int64_t>(blockIdx.x) * L : s_lds;
    const int tid = threadIdx.x, lane = tid % 64, wave = tid / 64;
    for (int64_t row = blockIdx.x; row < rows; row += gridDim.x) {
        const int64_t eb = a_rowptr[row], ee = a_rowptr[row + 1];
        // a column outside [0, n) marks the row invalid: its counts are -1
        bool bad = false;
        for (int64_t e = eb; e < ee; ++e) bad |= a_col[e] < 0 || a_col[e] >= n;
        if (bad) {
            if (tid < ks.n) hits[row * ks.n + tid] = -1;
            continue;
        }
        for (int64_t l = tid; l < L; l += kEvalThreads) {
            double acc = 0.0;
            for (int64_t e = eb; e < ee; ++e) {
                const double prod = a_val[e] * Z[static_cast<int64_t>(a_col[e]) * L + l];
                acc = acc + prod;
            }
            s_score[l] = acc;
        }
        __syncthreads();
        const int Li = static_cast<int>(L);
        for (int t = 0; t < kmax; ++t) {
            double bv = 0.0;
            int bi = Li;   // sentinel: no label yet
            for (int l = tid; l < Li; l += kEvalThreads) {
                const double v = s_score[l];
                if (bi == Li ? (v == v) : ranks_before(v, l, bv, bi)) {
                    bv = v;
                    bi = l;
                }
            }
    #pragma unroll
            for (int off = 32; off > 0; off >>= 1) {
                const double ov = __shfl_xor(bv, off, 64);
                const int oi = __shfl_xor(bi, off, 64);
                if (oi != Li && (bi == Li || ranks_before(ov, oi, bv, bi))) {
                    bv = ov;
                    bi = oi;
                }
            }
            if (lane == 0) {
                s_bv[wave] = bv;
                s_bi[wave] = bi;
            }
            __syncthreads();
            if (tid == 0) {
                double v = s_bv[0];
                int i = s_bi[0];
                for (int w = 1; w < kEvalWaves; ++w)
                    if (s_bi[w] != Li && (i == Li || ranks_before(s_bv[w], s_bi[w], v, i))) {
                        v = s_bv[w];
                        i = s_bi[w];
                    }
                s_top[t] = i < Li ? i : -1;
                if (i < Li) s_score[i] = __builtin_nan("");
            }
            __syncthreads();
        }
        // hit flags of the ranked labels against the row's positives
        const int64_t yb = y_rowptr[row], ye = y_rowptr[row + 1];
        if (tid < kmax) {
            const int lab = s_top[tid];
            int h = 0;
            if (lab >= 0)
                for (int64_t e = yb; e < ye; ++e) h |= (y_col[e] == lab) ? 1 : 0;
            s_hit[tid] = h;
        }
        __syncthreads();
        if (tid < ks.n) {
            const int k = ks.k[tid];
            int c = 0;
            for (int t = 0; t < k && t < kmax; ++t) c += s_hit[t];
            hits[row * ks.n + tid] = c;
        }
        __syncthreads();
    }
}

}  // namespace

int64_t topk_scratch_doubles(int64_t rows, int64_t L) {
    return L <= kTopkLdsLabels ? 0 : std::min<int64_t>(rows, kTopkGlobalGrid) * L;
}

void launch_topk_hits(int64_t rows, int64_t n, int64_t L, const int64_t* a_rowptr, const int* a_col,
                      const double* a_val, const double* Z, const int64_t* y_rowptr, const int* y_col,
                      int nk, const int* ks_host, int kmax, int* hits, double* scratch, hipStream_t st) {
    if (rows <= 0 || nk <= 0) return;
    KList kl{};
    kl.n = nk;
    for (int i = 0; i < nk; ++i) kl.k[i] = ks_host[i];
    if (L <= kTopkLdsLabels) {
        const size_t shmem = static_cast<size_t>(std::max<int64_t>(L, 1)) * sizeof(double);
        const unsigned grid = static_cast<unsigned>(std::min<int64_t>(rows, 1 << 20));
        hipLaunchKernelGGL((k_topk_hits<false>), dim3(grid), dim3(kEvalThreads), shmem, st, rows, n, L, a_rowptr,
                           a_col, a_val, Z, y_rowptr, y_col, kl, kmax, hits, nullptr);
    } else {
        const unsigned grid = static_cast<unsigned>(std::min<int64_t>(rows, kTopkGlobalGrid));
        hipLaunchKernelGGL((k_topk_hits<true>), dim3(grid), dim3(kEvalThreads), 0, st, rows, n, L, a_rowptr, a_col,
                           a_val, Z, y_rowptr, y_col, kl, kmax, hits, scratch);
    }
}

}  // namespace fastpi
