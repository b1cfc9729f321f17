// Evaluation of the multi-label regression (Application 1) on held-out rows: the score
// vector yhat = Z^T x of each test row, its k top-ranked labels and the top-k precision
// counts of the accuracy experiment (Section 4).
//
// Two kernels per chunk of test rows:
//  - scores: one wave per (row, 64-label slice), a lane per label. Each label's score is
//    accumulated over the row's stored entries in CSR order with one rounded multiply and
//    one rounded add per entry, so the integer decision below is taken on scores of a
//    stated precision and order. Rows have power-law lengths; splitting a row over its label
//    slices keeps the longest dependency chain at one row's entry count, and the entry loop
//    keeps two groups of kUnroll independent loads of Z in flight ahead of the ordered adds.
//  - selection: one wave per row. The t-th ranked label is the best of those ranking
//    strictly after the (t-1)-th (higher score, or equal score at a lower label), so the
//    scores are never written back; non-finite scores are never ranked. A ballot of the hit
//    flags of the ranked labels gives every top-k count at once.
#include "kernels.h"

namespace fastpi {

namespace {

constexpr int kEvalThreads = 256;
constexpr int kEvalWaves = kEvalThreads / 64;
constexpr int kUnroll = 16;

struct KList {
    int n;
    int k[kTopkMaxKs];
};

// (a, ia) ranks before (b, ib): a higher score, or an equal score at a lower label.
__device__ inline bool ranks_before(double a, int ia, double b, int ib) {
    return a > b || (a == b && ia < ib);
}

__device__ inline double readlane_f64(double v, int lane) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane(static_cast<int>(b), lane);
    const int hi = __builtin_amdgcn_readlane(static_cast<int>(b >> 32), lane);
    return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}

// z[u] = Z[c_{g+u}, l] for the 16 entries of group g (columns broadcast from lane g+u; lanes
// past the row's end hold column 0, so every load stays in bounds)
__device__ inline void load_group(double (&z)[kUnroll], const double* Zl, int64_t L, int myc, int g) {
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) z[u] = Zl[static_cast<int64_t>(__builtin_amdgcn_readlane(myc, g + u)) * L];
}

// acc += x_e z_e over the group's entries below cnt, in entry order
__device__ inline double sum_group(double acc, const double (&z)[kUnroll], double myx, int g, int cnt) {
#pragma clang fp contract(off)
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
        const double prod = readlane_f64(myx, g + u) * z[u];
        const double next = acc + prod;
        acc = (g + u < cnt) ? next : acc;
    }
    return acc;
}

__global__ __launch_bounds__(kEvalThreads) void k_topk_scores(
    int64_t row0, int64_t nrows, int64_t n, int64_t L, const int64_t* __restrict__ a_rowptr,
    const int* __restrict__ a_col, const double* __restrict__ a_val, const double* __restrict__ Z,
    double* __restrict__ S) {
    const int lane = threadIdx.x % 64;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
    const int64_t slices = (L + 63) / 64;
    const int64_t unit = static_cast<int64_t>(blockIdx.x) * kEvalWaves + wave;
    if (unit >= nrows * slices) return;
    const int64_t rl = unit / slices;
    const int64_t l = (unit - rl * slices) * 64 + lane;
    const int64_t row = row0 + rl;
    const int64_t eb = a_rowptr[row], ee = a_rowptr[row + 1];
    const double* Zl = Z + (l < L ? l : 0);
    double acc = 0.0;
    double za[kUnroll], zb[kUnroll];
    // 64 entries at a time: one coalesced load of their columns and values, then groups of
    // 16 loads of Z, the next group in flight while the current one is summed
    for (int64_t e0 = eb; e0 < ee; e0 += 64) {
        const int cnt = static_cast<int>(ee - e0 < 64 ? ee - e0 : 64);
        int myc = 0;
        double myx = 0.0;
        if (lane < cnt) {
            myc = a_col[e0 + lane];
            myx = a_val[e0 + lane];
        }
        myc = (myc >= 0 && myc < n) ? myc : 0;   // such a row is reported invalid by the selection
        load_group(za, Zl, L, myc, 0);
        for (int g = 0; g < cnt; g += 2 * kUnroll) {
            if (g + kUnroll < cnt) load_group(zb, Zl, L, myc, g + kUnroll);
            acc = sum_group(acc, za, myx, g, cnt);
            if (g + 2 * kUnroll < cnt) load_group(za, Zl, L, myc, g + 2 * kUnroll);
            if (g + kUnroll < cnt) acc = sum_group(acc, zb, myx, g + kUnroll, cnt);
        }
    }
    if (l < L) S[rl * L + l] = acc;
}

__global__ __launch_bounds__(kEvalThreads) void k_topk_select(
    int64_t row0, int64_t nrows, int64_t n, int64_t L, const int64_t* __restrict__ a_rowptr,
    const int* __restrict__ a_col, const double* __restrict__ S, const int64_t* __restrict__ y_rowptr,
    const int* __restrict__ y_col, KList ks, int kmax, int* __restrict__ hits) {
    const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
    const int64_t rl = static_cast<int64_t>(blockIdx.x) * kEvalWaves + wave;
    if (rl >= nrows) return;
    const int64_t row = row0 + rl;
    // a column outside [0, n) marks the row invalid: its counts are -1
    bool bad = false;
    for (int64_t e = a_rowptr[row] + lane; e < a_rowptr[row + 1]; e += 64) bad |= a_col[e] < 0 || a_col[e] >= n;
    if (__any(bad)) {
        if (lane < ks.n) hits[row * ks.n + lane] = -1;
        return;
    }
    const double* Sr = S + rl * L;
    const int Li = static_cast<int>(L);
    double pv = 0.0;
    int pi = -1;    // previous pick; -1: none yet
    int mine = -1;  // the label ranked at position `lane`
    for (int t = 0; t < kmax; ++t) {
        double bv = 0.0;
        int bi = Li;   // sentinel: no candidate
        for (int l = lane; l < Li; l += 64) {
            const double v = Sr[l];
            if (!(v == v) || (pi >= 0 && !ranks_before(pv, pi, v, l))) continue;   // NaN, or not after
            if (bi == Li || ranks_before(v, l, bv, bi)) {
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
        if (bi == Li) break;   // fewer than kmax finite scores
        if (lane == t) mine = bi;
        pv = bv;
        pi = bi;
    }
    // hit flag of the label at position `lane` against the row's positives
    int h = 0;
    if (mine >= 0)
        for (int64_t e = y_rowptr[row]; e < y_rowptr[row + 1]; ++e) h |= (y_col[e] == mine) ? 1 : 0;
    const unsigned long long mask = __ballot(h);
    if (lane < ks.n) {
        const int k = ks.k[lane];
        const unsigned long long lo = k >= 64 ? ~0ull : ((1ull << k) - 1ull);
        hits[row * ks.n + lane] = __popcll(mask & lo);
    }
}

}  // namespace

int64_t topk_scratch_doubles(int64_t rows, int64_t L) {
    const int64_t per = std::max<int64_t>(L, 1);
    return std::min<int64_t>(rows, std::max<int64_t>(1, kTopkScoreDoubles / per)) * per;
}

void launch_topk_hits(int64_t rows, int64_t n, int64_t L, const int64_t* a_rowptr, const int* a_col,
                      const double* a_val, const double* Z, const int64_t* y_rowptr, const int* y_col,
                      int nk, const int* ks_host, int kmax, int* hits, double* scratch, hipStream_t st,
                      KernelTimer* timer) {
    if (rows <= 0 || nk <= 0) return;
    KList kl{};
    kl.n = nk;
    for (int i = 0; i < nk; ++i) kl.k[i] = ks_host[i];
    const int64_t chunk = topk_scratch_doubles(rows, L) / std::max<int64_t>(L, 1);
    const int64_t slices = (L + 63) / 64;
    const double* S = scratch;
    for (int64_t r0 = 0; r0 < rows; r0 += chunk) {
        const int64_t nr = std::min(chunk, rows - r0);
        if (slices > 0) {
            const int64_t units = nr * slices;
            FASTPI_LAUNCH(timer, KT_TOPK, k_topk_scores,
                          dim3(static_cast<unsigned>((units + kEvalWaves - 1) / kEvalWaves)), dim3(kEvalThreads), 0,
                          st, r0, nr, n, L, a_rowptr, a_col, a_val, Z, scratch);
        }
        FASTPI_LAUNCH(timer, KT_TOPK, k_topk_select, dim3(static_cast<unsigned>((nr + kEvalWaves - 1) / kEvalWaves)),
                      dim3(kEvalThreads), 0, st, r0, nr, n, L, a_rowptr, a_col, S, y_rowptr, y_col, kl, kmax, hits);
    }
}

}  // namespace fastpi
