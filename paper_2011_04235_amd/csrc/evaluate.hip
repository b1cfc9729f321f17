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

// Label SpMM of the sparse-label apply, C = diag-scaled Y^T U (L x r), with every labelled
// row of U read from memory once per call. The labelled rows (lrows) are cut into blocks of
// at most kLabelBlockRows rows and kLabelBlockPos positives (block b: lrows[bstart[b],
// bstart[b+1])). A frequent label is split into sub-labels (label l owns sub-labels vbase[l] ..
// vbase[l+1] - 1; the i-th of its positives in a block goes to sub-label i mod K_l), so that no
// run is long. Within a block the positives are sorted by sub-label, then by row (prow: the
// row's position in the block, each block's run of entries starting at bbase[b], 16-byte
// aligned); the block's runs, one per sub-label present, are listed in sub-label order (run i:
// sub-label rv[i], entries re[i] .. re[i+1] - 1 relative to bbase[b]; each block's list ends
// with a sentinel whose re is the block's count); rg[b * (ngroup + 1) + g] is the first run of
// the block with a sub-label of group g (2048 sub-labels a group).
// A workgroup of kLabelThreads threads owns kLabelCols columns of U, one group of sub-labels
// (accumulated in LDS) and a chunk of consecutive blocks: it stages each block's slice of U
// (two threads to a row) and its row indices in LDS (the next two blocks already loading into
// registers), and each thread sums the staged rows of the runs dealt to it and adds the sum to
// its sub-label's accumulator. A sub-label has one run per
// block and the blocks are taken in order between barriers, so every sum runs in a fixed order.
// The chunks' partial sums (part, nchunk x Lv x r) are added in chunk order, and a label's
// sub-labels in order, by k_label_reduce, which also applies the column scale cs.
namespace {

constexpr int kLabelRows = kLabelBlockRows;
constexpr int kLabelCols = 8;
constexpr int kLabelGroup = kLabelSubGroup;
constexpr int kLabelThreads = 2 * kLabelRows;   // two threads stage each row of a block

__global__ __launch_bounds__(kLabelThreads) void k_label_spmm(const int32_t* __restrict__ lrows, const int32_t* __restrict__ bstart,
                                                    const int32_t* __restrict__ bbase, const int32_t* __restrict__ rg,
                                                    const int32_t* __restrict__ rv, const int32_t* __restrict__ re,
                                                    const uint8_t* __restrict__ prow,
                                                    const double* __restrict__ pval,
                                                    const double* __restrict__ U, int64_t r, int64_t Lv,
                                                    int64_t nblk, int64_t bpc, int ncb, int ngroup, int nchunk,
                                                    double* __restrict__ part) {
    // XCD-grouped tile order (workgroups go to the 8 XCDs round robin by linear id): each XCD
    // takes a contiguous range of tiles numbered chunk-major, column block fastest, so the
    // workgroups sharing a chunk's tables run under one L2
    const int ntile = ncb * ngroup * nchunk;
    const int lin = blockIdx.x;
    const int per = ntile / 8, extra = ntile % 8, xcd = lin % 8, slot = lin / 8;
    const int tile = (xcd < extra ? xcd * (per + 1) : extra * (per + 1) + (xcd - extra) * per) + slot;
    const int cb = tile % ncb;
    const int g = (tile / ncb) % ngroup;
    const int p = tile / (ncb * ngroup);
    const int t = threadIdx.x;
    const int64_t c0 = static_cast<int64_t>(cb) * kLabelCols;
    const int64_t b0 = static_cast<int64_t>(p) * bpc;
    const int64_t b1 = min(nblk, b0 + bpc);
    const int v0 = g * kLabelGroup;
    const int nv = static_cast<int>(min<int64_t>(kLabelGroup, Lv - v0));
    __shared__ double acc[kLabelGroup][kLabelCols];
    __shared__ double Us[kLabelRows + 1][kLabelCols + 1];   // padded rows; row kLabelRows stays 0
    __shared__ uint2 Ps[kLabelBlockPos / 8 + 2];            // the block's row indices (+ slack)
    for (int e = t; e < kLabelGroup * kLabelCols; e += kLabelThreads) (&acc[0][0])[e] = 0.0;
    if (t < kLabelCols) Us[kLabelRows][t] = 0.0;
    // blocks ahead, in registers (a ring of three: two in flight while one is processed): half
    // of a U slice row, 8 bytes of row indices and the first two runs of this thread
    struct Ahead {
        double u[kLabelCols / 2];
        uint2 p;
        int32_t base, r0, r1, va, vb, e0a, e0b, e1a, e1b;   // runs t and t + kLabelThreads of the block
    };
    Ahead ra, rb, rc;   // three named slots (no indexing, so they stay in registers)
    auto fetch = [&](int64_t b, Ahead& A) __attribute__((always_inline)) {
        const int32_t k0 = bstart[b], k1 = bstart[b + 1];
        const int row = t / 2, h = (t % 2) * (kLabelCols / 2);
        const int64_t i = row < k1 - k0 ? lrows[k0 + row] : -1;
#pragma unroll
        for (int c = 0; c < kLabelCols / 2; ++c)
            A.u[c] = (i >= 0 && c0 + h + c < r) ? U[i * r + c0 + h + c] : 0.0;
        A.base = bbase[b];
        const int32_t npos = bbase[b + 1] - A.base;
        A.p = 8 * t < npos ? *reinterpret_cast<const uint2*>(prow + A.base + 8 * t) : make_uint2(0, 0);
        A.r0 = rg[b * (ngroup + 1) + g];
        A.r1 = rg[b * (ngroup + 1) + g + 1];
        const int32_t ra0 = A.r0 + t, rb0 = A.r0 + t + kLabelThreads;
        A.va = ra0 < A.r1 ? rv[ra0] : 0;
        A.e0a = ra0 < A.r1 ? re[ra0] : 0;
        A.e1a = ra0 < A.r1 ? re[ra0 + 1] : 0;
        A.vb = rb0 < A.r1 ? rv[rb0] : 0;
        A.e0b = rb0 < A.r1 ? re[rb0] : 0;
        A.e1b = rb0 < A.r1 ? re[rb0 + 1] : 0;
    };
    auto process = [&](const Ahead& A) __attribute__((always_inline)) {
        __syncthreads();   // the previous block's staged data is no longer read
#pragma unroll
        for (int c = 0; c < kLabelCols / 2; ++c) Us[t / 2][(t % 2) * (kLabelCols / 2) + c] = A.u[c];
        Ps[t] = A.p;
        __syncthreads();
        const uint8_t* ps = reinterpret_cast<const uint8_t*>(Ps);
        // one run: its positives' staged rows summed four at a time (their loads issue
        // together; past the run's end the zero row is added, which leaves the sum unchanged),
        // in order, then the sum added to the sub-label's accumulator
        auto run = [&](int32_t v, int32_t e0, int32_t e1) __attribute__((always_inline)) {
            double sum[kLabelCols];
#pragma unroll
            for (int c = 0; c < kLabelCols; ++c) sum[c] = 0.0;
            for (int32_t e = e0; e < e1; e += 4) {
                int j[4];
                double w[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const bool in = e + q < e1;
                    j[q] = in ? ps[e + q] : kLabelRows;
                    w[q] = in ? (pval ? pval[A.base + e + q] : 1.0) : 0.0;
                }
#pragma unroll
                for (int q = 0; q < 4; ++q)
#pragma unroll
                    for (int c = 0; c < kLabelCols; ++c) sum[c] += w[q] * Us[j[q]][c];
            }
            double* a = acc[v - v0];
#pragma unroll
            for (int c = 0; c < kLabelCols; ++c) a[c] += sum[c];
        };
        if (A.r0 + t < A.r1) run(A.va, A.e0a, A.e1a);
        if (A.r0 + t + kLabelThreads < A.r1) run(A.vb, A.e0b, A.e1b);
        for (int32_t ri = A.r0 + t + 2 * kLabelThreads; ri < A.r1; ri += kLabelThreads) run(rv[ri], re[ri], re[ri + 1]);
    };
    if (b0 < b1) fetch(b0, ra);
    if (b0 + 1 < b1) fetch(b0 + 1, rb);
    for (int64_t b = b0; b < b1; b += 3) {
        if (b + 2 < b1) fetch(b + 2, rc);
        process(ra);
        if (b + 1 >= b1) break;
        if (b + 3 < b1) fetch(b + 3, ra);
        process(rb);
        if (b + 2 >= b1) break;
        if (b + 4 < b1) fetch(b + 4, rb);
        process(rc);
    }
    __syncthreads();
    for (int e = t; e < nv * kLabelCols; e += kLabelThreads) {
        const int v = e / kLabelCols, c = e % kLabelCols;
        if (c0 + c < r) part[(static_cast<int64_t>(p) * Lv + v0 + v) * r + c0 + c] = acc[v][c];
    }
}

// C[l] = cs .* sum over chunks p, then over label l's sub-labels v in [vbase[l], vbase[l+1]),
// of part[p][v] (Lv sub-labels in all)
__global__ void k_label_reduce(const double* __restrict__ part, int nchunk, const int32_t* __restrict__ vbase,
                               int64_t Lv, int64_t L, int64_t r, const double* __restrict__ cs,
                               double* __restrict__ C) {
    const int64_t l = blockIdx.x;
    const int64_t k = static_cast<int64_t>(blockIdx.y) * blockDim.x + threadIdx.x;
    if (l >= L || k >= r) return;
    const int32_t v0 = vbase[l], v1 = vbase[l + 1];
    double acc = 0.0;
    for (int p = 0; p < nchunk; ++p)
        for (int32_t v = v0; v < v1; ++v) acc += part[(static_cast<int64_t>(p) * Lv + v) * r + k];
    C[l * r + k] = cs ? acc * cs[k] : acc;
}

}  // namespace

int label_spmm_chunks(int64_t nblk, int64_t r, int64_t Lv) {
    if (nblk <= 0) return 0;
    const int64_t ncb = (r + kLabelCols - 1) / kLabelCols;
    const int64_t ngroup = (Lv + kLabelGroup - 1) / kLabelGroup;
    // one workgroup per compute unit at most (the accumulators take most of the LDS, and a
    // second round would leave the chip mostly idle), each chunk at least one block
    const int64_t want = 256 / (ncb * ngroup);
    return static_cast<int>(std::max<int64_t>(1, std::min<int64_t>({want, nblk, 64})));
}

int label_slots(int64_t L) { return static_cast<int>((L + kLabelGroup - 1) / kLabelGroup * kLabelGroup); }

int label_groups(int64_t Lv) { return static_cast<int>((Lv + kLabelGroup - 1) / kLabelGroup); }

void launch_label_spmm(const LabelBlocks& lb, const double* U, int64_t r, int64_t L, const double* cs, double* C,
                       double* part, hipStream_t st, KernelTimer* timer) {
    if (r <= 0 || L <= 0) return;
    const int nchunk = label_spmm_chunks(lb.nblk, r, lb.Lv);
    if (nchunk == 0) {
        launch_fill(C, L * r, 0.0, st);
        return;
    }
    const int ncb = static_cast<int>((r + kLabelCols - 1) / kLabelCols);
    const int ngroup = label_groups(lb.Lv);
    const int64_t bpc = (lb.nblk + nchunk - 1) / nchunk;
    const unsigned tiles = static_cast<unsigned>(ncb) * static_cast<unsigned>(ngroup) * static_cast<unsigned>(nchunk);
    FASTPI_LAUNCH(timer, KT_LABEL_SPMM, k_label_spmm, dim3(tiles), dim3(kLabelThreads), 0, st, lb.lrows, lb.bstart, lb.bbase, lb.rg,
                  lb.rv, lb.re, lb.prow, lb.pval, U, r, lb.Lv, lb.nblk, bpc, ncb, ngroup, nchunk, part);
    FASTPI_LAUNCH(timer, KT_LABEL_SPMM, k_label_reduce, dim3(static_cast<unsigned>(L), static_cast<unsigned>((r + 255) / 256)),
                  dim3(256), 0, st, part, nchunk, lb.vbase, lb.Lv, L, r, cs, C);
}

}  // namespace fastpi
