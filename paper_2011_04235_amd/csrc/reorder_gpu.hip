// Hub-and-spoke reordering on the GPU (Section 3.2, Algorithm 2), with the same result as the
// host reordering bit for bit (the tie-break readings are the ones stated in fastpi.h).
//
// The bipartite graph lives on the device as CSR (rows) and CSC (columns) with stored zeros
// dropped. Every iteration, driven by the host (a few words read back per step):
//  1. degrees of the alive nodes inside the current graph;
//  2. hubs: the ceil(k|V|) alive nodes of highest degree, ties to the lower index. A degree
//     histogram gives the threshold degree D and the count above it; the nodes of degree D
//     are taken in index order through a prefix count; the hubs are then sorted by
//     (degree desc, index asc) and take the highest free ids in that order;
//  3. connected components of what remains, by min-label propagation with pointer jumping:
//     node codes are row i -> i and column j -> m + j, and every node ends with the smallest
//     code of its component. That code is the component's seed in the scan order (rows by
//     index, then columns), so ordering components by it is their discovery order;
//  4. the giant component (most nodes, the first found on ties) continues; every other
//     component is a diagonal block, its rows and its columns in ascending index order, the
//     blocks in discovery order: a sort of (code, index) keys gives each node its id.
#include <vector>

#include "host_internal.h"
#include "kernels.h"

namespace fastpi {

namespace {

constexpr int kThreads = 256;
constexpr int kScanBlock = 1024;   // elements per block of the two-level scan

unsigned grid_of(int64_t n, int per = kThreads) {
    const int64_t g = (n + per - 1) / per;
    return static_cast<unsigned>(std::max<int64_t>(1, std::min<int64_t>(g, 1 << 20)));
}

#define GRID_STRIDE(i, n)                                                                       \
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < (n); \
         i += static_cast<int64_t>(gridDim.x) * blockDim.x)

// ---- graph build -----------------------------------------------------------------------
// nonzero-valued entries per row (all entries when val is null)
__global__ void k_row_keep(const int64_t* __restrict__ rowptr, const double* __restrict__ val, int64_t m,
                           int* __restrict__ cnt) {
    GRID_STRIDE(i, m) {
        int c = 0;
        for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) c += (val == nullptr || val[e] != 0.0) ? 1 : 0;
        cnt[i] = c;
    }
}

__global__ void k_row_fill(const int64_t* __restrict__ rowptr, const int* __restrict__ col,
                           const double* __restrict__ val, int64_t m, const int64_t* __restrict__ rp,
                           int* __restrict__ rc, int* __restrict__ ccnt) {
    GRID_STRIDE(i, m) {
        int64_t o = rp[i];
        for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e)
            if (val == nullptr || val[e] != 0.0) {
                rc[o++] = col[e];
                atomicAdd(&ccnt[col[e]], 1);
            }
    }
}

// CSC from the kept CSR; the order inside a column is immaterial (degrees and components
// do not depend on it)
__global__ void k_col_fill(const int64_t* __restrict__ rp, const int* __restrict__ rc, int64_t m,
                           int* __restrict__ cpos, int* __restrict__ cr) {
    GRID_STRIDE(i, m) {
        for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
            const int slot = atomicAdd(&cpos[rc[e]], 1);
            cr[slot] = static_cast<int>(i);
        }
    }
}

// ---- scans -----------------------------------------------------------------------------
// exclusive scan of int values (n <= 2^31) into int64 offsets, in three passes
__global__ __launch_bounds__(kThreads) void k_scan_block_sums(const int* __restrict__ in, int64_t n,
                                                              int64_t* __restrict__ sums) {
    __shared__ int64_t s[kThreads];
    const int64_t b0 = static_cast<int64_t>(blockIdx.x) * kScanBlock;
    int64_t acc = 0;
    for (int64_t i = b0 + threadIdx.x; i < b0 + kScanBlock && i < n; i += kThreads) acc += in[i];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int off = kThreads / 2; off > 0; off >>= 1) {
        if (static_cast<int>(threadIdx.x) < off) s[threadIdx.x] += s[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) sums[blockIdx.x] = s[0];
}

// exclusive scan of the block sums in place (one workgroup, sequential chunks); total -> sums[nb]
__global__ __launch_bounds__(kThreads) void k_scan_sums(int64_t* __restrict__ sums, int64_t nb) {
    __shared__ int64_t s[kThreads];
    __shared__ int64_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int64_t c0 = 0; c0 < nb; c0 += kThreads) {
        const int64_t i = c0 + threadIdx.x;
        const int64_t v = i < nb ? sums[i] : 0;
        s[threadIdx.x] = v;
        __syncthreads();
        for (int off = 1; off < kThreads; off <<= 1) {
            const int64_t add = static_cast<int>(threadIdx.x) >= off ? s[threadIdx.x - off] : 0;
            __syncthreads();
            s[threadIdx.x] += add;
            __syncthreads();
        }
        if (i < nb) sums[i] = carry + s[threadIdx.x] - v;
        __syncthreads();
        if (threadIdx.x == kThreads - 1) carry += s[kThreads - 1];
        __syncthreads();
    }
    if (threadIdx.x == 0) sums[nb] = carry;
}

// out[i] = base + block offset + exclusive prefix inside the block
__global__ __launch_bounds__(kThreads) void k_scan_apply(const int* __restrict__ in, int64_t n,
                                                         const int64_t* __restrict__ sums, int64_t base,
                                                         int64_t* __restrict__ out) {
    __shared__ int64_t s[kThreads];
    const int64_t b0 = static_cast<int64_t>(blockIdx.x) * kScanBlock;
    constexpr int PER = kScanBlock / kThreads;
    int64_t loc[PER];
    int64_t acc = 0;
    for (int u = 0; u < PER; ++u) {
        const int64_t i = b0 + static_cast<int64_t>(threadIdx.x) * PER + u;
        loc[u] = acc;
        acc += i < n ? in[i] : 0;
    }
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int off = 1; off < kThreads; off <<= 1) {
        const int64_t add = static_cast<int>(threadIdx.x) >= off ? s[threadIdx.x - off] : 0;
        __syncthreads();
        s[threadIdx.x] += add;
        __syncthreads();
    }
    const int64_t excl = s[threadIdx.x] - acc + sums[blockIdx.x] + base;
    for (int u = 0; u < PER; ++u) {
        const int64_t i = b0 + static_cast<int64_t>(threadIdx.x) * PER + u;
        if (i < n) out[i] = excl + loc[u];
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) out[n] = base + sums[gridDim.x];
}

// ---- degrees and hubs ------------------------------------------------------------------
__global__ void k_degrees(const int64_t* __restrict__ ptr, const int* __restrict__ idx, int64_t cnt,
                          const unsigned char* __restrict__ alive_self,
                          const unsigned char* __restrict__ alive_other, int* __restrict__ deg,
                          int* __restrict__ hist) {
    GRID_STRIDE(v, cnt) {
        if (!alive_self[v]) {
            deg[v] = -1;
            continue;
        }
        int d = 0;
        for (int64_t e = ptr[v]; e < ptr[v + 1]; ++e) d += alive_other[idx[e]];
        deg[v] = d;
        atomicAdd(&hist[d], 1);
    }
}

// One workgroup: the threshold degree D with count(deg > D) < h <= count(deg >= D), written
// as out[0] = D, out[1] = h - count(deg > D) (nodes of degree D to take, lowest index first).
__global__ __launch_bounds__(1024) void k_hub_threshold(const int* __restrict__ hist, int64_t maxdeg, int64_t h,
                                                        int64_t* __restrict__ out) {
    __shared__ int64_t s[1024];
    const int64_t bins = maxdeg + 1;
    const int64_t chunk = (bins + 1023) / 1024;
    // chunk t covers degrees from the top: [bins - (t+1) chunk, bins - t chunk)
    const int64_t hi = bins - static_cast<int64_t>(threadIdx.x) * chunk;
    const int64_t lo = hi - chunk;
    int64_t acc = 0;
    for (int64_t d = hi - 1; d >= lo && d >= 0; --d) acc += hist[d];
    s[threadIdx.x] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t above = 0;
        int64_t D = 0, take = 0;
        bool found = false;
        for (int t = 0; t < 1024 && !found; ++t) {
            if (above + s[t] >= h) {
                const int64_t thi = bins - static_cast<int64_t>(t) * chunk;
                for (int64_t d = thi - 1; d >= thi - chunk && d >= 0; --d) {
                    if (above + hist[d] >= h) {
                        D = d;
                        take = h - above;
                        found = true;
                        break;
                    }
                    above += hist[d];
                }
            } else {
                above += s[t];
            }
        }
        out[0] = found ? D : 0;
        out[1] = found ? take : 0;
    }
}

__global__ void k_eq_flags(const int* __restrict__ deg, int64_t cnt, const int64_t* __restrict__ thr,
                           int* __restrict__ flag) {
    const int D = static_cast<int>(thr[0]);
    GRID_STRIDE(v, cnt) flag[v] = deg[v] == D ? 1 : 0;
}

// hubs: degree above D, or degree D within the first `take` of them in index order; their
// sort keys (degree desc, index asc) go to keys[slot] through an atomic slot counter
__global__ void k_hub_keys(const int* __restrict__ deg, int64_t cnt, const int64_t* __restrict__ thr,
                           const int64_t* __restrict__ eqrank, unsigned long long* __restrict__ keys,
                           int* __restrict__ nkeys) {
    const int D = static_cast<int>(thr[0]);
    const int64_t take = thr[1];
    GRID_STRIDE(v, cnt) {
        const int d = deg[v];
        if (d < 0) continue;
        if (d > D || (d == D && eqrank[v] < take)) {
            const int slot = atomicAdd(nkeys, 1);
            keys[slot] = (static_cast<unsigned long long>(0x7FFFFFFF - d) << 32) | static_cast<unsigned long long>(v);
        }
    }
}

// hub r (in key order) takes id hi - r and leaves the graph
__global__ void k_hub_assign(const unsigned long long* __restrict__ keys, int64_t h, int64_t hi,
                             int* __restrict__ pi, unsigned char* __restrict__ alive) {
    GRID_STRIDE(r, h) {
        const int v = static_cast<int>(keys[r] & 0xFFFFFFFFull);
        pi[v] = static_cast<int>(hi - r);
        alive[v] = 0;
    }
}

// ---- bitonic sort of 64-bit keys (padded to a power of two with all-ones) ---------------
__global__ void k_bitonic_global(unsigned long long* __restrict__ a, int64_t n, int64_t j, int64_t k) {
    GRID_STRIDE(i, n) {
        const int64_t l = i ^ j;
        if (l > i) {
            const unsigned long long x = a[i], y = a[l];
            const bool up = (i & k) == 0;
            if ((x > y) == up) {
                a[i] = y;
                a[l] = x;
            }
        }
    }
}

// all stages with stride j < 2048 of pass k, in LDS (one workgroup per 4096 keys)
__global__ __launch_bounds__(1024) void k_bitonic_local(unsigned long long* __restrict__ a, int64_t n, int64_t k,
                                                        int64_t jstart) {
    __shared__ unsigned long long s[4096];
    const int64_t base = static_cast<int64_t>(blockIdx.x) * 4096;
    for (int t = threadIdx.x; t < 4096; t += 1024) s[t] = base + t < n ? a[base + t] : ~0ull;
    __syncthreads();
    for (int64_t j = jstart; j > 0; j >>= 1) {
        for (int t = threadIdx.x; t < 4096; t += 1024) {
            const int l = t ^ static_cast<int>(j);
            if (l > t) {
                const int64_t gi = base + t;
                const bool up = (gi & k) == 0;
                const unsigned long long x = s[t], y = s[l];
                if ((x > y) == up) {
                    s[t] = y;
                    s[l] = x;
                }
            }
        }
        __syncthreads();
    }
    for (int t = threadIdx.x; t < 4096; t += 1024)
        if (base + t < n) a[base + t] = s[t];
}

__global__ void k_fill_u8(unsigned char* __restrict__ a, int64_t n, unsigned char v) {
    GRID_STRIDE(i, n) a[i] = v;
}

__global__ void k_fill_u64(unsigned long long* __restrict__ a, int64_t from, int64_t to, unsigned long long v) {
    GRID_STRIDE(i, to - from) a[from + i] = v;
}

// ---- connected components --------------------------------------------------------------
// labT / labF hold node codes (row i -> i, column j -> m + j); -1 for nodes out of the graph
__global__ void k_cc_init(const unsigned char* __restrict__ aliveT, const unsigned char* __restrict__ aliveF,
                          int64_t m, int64_t n, int* __restrict__ lab) {
    GRID_STRIDE(v, m + n) lab[v] = (v < m ? aliveT[v] : aliveF[v - m]) ? static_cast<int>(v) : -1;
}

// min over every alive edge, both ends; `changed` is set when a label drops
__global__ void k_cc_hook(const int64_t* __restrict__ rp, const int* __restrict__ rc, int64_t m,
                          int* __restrict__ lab, int* __restrict__ changed) {
    GRID_STRIDE(i, m) {
        const int li = lab[i];
        if (li < 0) continue;
        int best = li;
        for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
            const int64_t vj = m + rc[e];
            const int lj = lab[vj];
            if (lj < 0) continue;
            if (lj < best) best = lj;
            if (li < lj) {
                if (atomicMin(&lab[vj], li) > li) *changed = 1;
            }
        }
        if (best < li) {
            if (atomicMin(&lab[i], best) > best) *changed = 1;
        }
    }
}

// pointer jumping: lab[v] <- lab[lab[v]] until it stops dropping (labels only decrease and
// stay inside the component, so the walk ends)
__global__ void k_cc_jump(int64_t total, int* __restrict__ lab, int* __restrict__ changed) {
    GRID_STRIDE(v, total) {
        int l = lab[v];
        if (l < 0) continue;
        int nl = lab[l];
        bool moved = false;
        while (nl >= 0 && nl < l) {
            l = nl;
            nl = lab[l];
            moved = true;
        }
        if (moved) {
            if (atomicMin(&lab[v], l) > l) *changed = 1;
        }
    }
}

// sizes per root code; the giant as the maximum of (size, -code) packed in 64 bits
__global__ void k_cc_sizes(const int* __restrict__ lab, int64_t total, int* __restrict__ size) {
    GRID_STRIDE(v, total) {
        const int l = lab[v];
        if (l >= 0) atomicAdd(&size[l], 1);
    }
}

__global__ void k_cc_giant(const int* __restrict__ lab, const int* __restrict__ size, int64_t total,
                           unsigned long long* __restrict__ best, int* __restrict__ ncomp) {
    GRID_STRIDE(v, total) {
        if (lab[v] == static_cast<int>(v)) {
            atomicAdd(ncomp, 1);
            const unsigned long long key = (static_cast<unsigned long long>(size[v]) << 32) |
                                           static_cast<unsigned long long>(0x7FFFFFFF - static_cast<int>(v));
            atomicMax(best, key);
        }
    }
}

// nodes of the giant (count) and keys (code, index) of every other alive node
__global__ void k_spoke_keys(const int* __restrict__ lab, int64_t from, int64_t cnt, int giant,
                             unsigned long long* __restrict__ keys, int* __restrict__ nkeys, int* __restrict__ ngiant) {
    GRID_STRIDE(i, cnt) {
        const int l = lab[from + i];
        if (l < 0) continue;
        if (l == giant) {
            atomicAdd(ngiant, 1);
        } else {
            const int slot = atomicAdd(nkeys, 1);
            keys[slot] = (static_cast<unsigned long long>(l) << 32) | static_cast<unsigned long long>(i);
        }
    }
}

__global__ void k_spoke_assign(const unsigned long long* __restrict__ keys, int64_t cnt, int64_t lo,
                               int* __restrict__ pi, unsigned char* __restrict__ alive) {
    GRID_STRIDE(r, cnt) {
        const int v = static_cast<int>(keys[r] & 0xFFFFFFFFull);
        pi[v] = static_cast<int>(lo + r);
        alive[v] = 0;
    }
}

// the final giant: ids in ascending index order
__global__ void k_alive_flags(const unsigned char* __restrict__ alive, int64_t cnt, int* __restrict__ flag) {
    GRID_STRIDE(v, cnt) flag[v] = alive[v] ? 1 : 0;
}

__global__ void k_final_assign(const unsigned char* __restrict__ alive, const int64_t* __restrict__ rank,
                               int64_t cnt, int64_t lo, int* __restrict__ pi) {
    GRID_STRIDE(v, cnt) if (alive[v]) pi[v] = static_cast<int>(lo + rank[v]);
}

// ---- validation of a device CSR ---------------------------------------------------------
// pass 1: rowptr[0] = 0, rowptr[m] = nnz, monotone (so every entry index lies in [0, nnz))
__global__ void k_check_rowptr(const int64_t* __restrict__ rowptr, int64_t m, int64_t nnz, int* __restrict__ bad) {
    GRID_STRIDE(i, m) {
        if (rowptr[i + 1] < rowptr[i]) atomicOr(bad, 1);
        if (i == 0 && (rowptr[0] != 0 || rowptr[m] != nnz)) atomicOr(bad, 1);
    }
}

// pass 2 (only after pass 1): columns in [0, n), strictly increasing per row; finite values
__global__ void k_check_entries(const int64_t* __restrict__ rowptr, const int* __restrict__ col,
                                const double* __restrict__ val, int64_t m, int64_t n, int* __restrict__ bad) {
    GRID_STRIDE(i, m) {
        for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
            const int c = col[e];
            if (c < 0 || c >= n || (e > rowptr[i] && c <= col[e - 1])) atomicOr(bad, 2);
            if (val && !isfinite(val[e])) atomicOr(bad, 4);
        }
    }
}

#undef GRID_STRIDE

// ---- host helpers ----------------------------------------------------------------------
struct DevBuf {
    std::vector<void*> ptrs;
    template <typename T>
    T* get(size_t count) {
        void* p = nullptr;
        if (hipMalloc(&p, std::max<size_t>(count, 1) * sizeof(T)) != hipSuccess) return nullptr;
        ptrs.push_back(p);
        return static_cast<T*>(p);
    }
    ~DevBuf() {
        for (void* p : ptrs) hipFree(p);
    }
};

struct Scan {
    int64_t* sums = nullptr;
    int64_t cap = 0;
};

// out[0..n] = exclusive prefix of in[0..n) plus base (out[n] = base + total)
void scan_ints(const int* in, int64_t n, int64_t base, int64_t* out, Scan& sc, hipStream_t st) {
    const int64_t nb = std::max<int64_t>(1, (n + kScanBlock - 1) / kScanBlock);
    hipLaunchKernelGGL(k_scan_block_sums, dim3(static_cast<unsigned>(nb)), dim3(kThreads), 0, st, in, n, sc.sums);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(kThreads), 0, st, sc.sums, nb);
    hipLaunchKernelGGL(k_scan_apply, dim3(static_cast<unsigned>(nb)), dim3(kThreads), 0, st, in, n, sc.sums, base,
                       out);
}

// ascending sort of keys[0..n) (scratch: keys must hold the next power of two >= n)
void sort_keys(unsigned long long* keys, int64_t n, hipStream_t st) {
    if (n <= 1) return;
    int64_t p2 = 1;
    while (p2 < n) p2 <<= 1;
    if (p2 > n)
        hipLaunchKernelGGL(k_fill_u64, dim3(grid_of(p2 - n)), dim3(kThreads), 0, st, keys, n, p2, ~0ull);
    const unsigned lb = static_cast<unsigned>((p2 + 4095) / 4096);
    for (int64_t k = 2; k <= p2; k <<= 1) {
        int64_t j = k >> 1;
        for (; j >= 2048; j >>= 1)
            hipLaunchKernelGGL(k_bitonic_global, dim3(grid_of(p2)), dim3(kThreads), 0, st, keys, p2, j, k);
        hipLaunchKernelGGL(k_bitonic_local, dim3(lb), dim3(1024), 0, st, keys, p2, k, j);
    }
}

int64_t pow2_at_least(int64_t n) {
    int64_t p = 1;
    while (p < n) p <<= 1;
    return p;
}

}  // namespace

int validate_csr_gpu(int64_t m, int64_t n, int64_t nnz, const int64_t* rowptr, const int32_t* col,
                     const double* val, hipStream_t st) {
    if (m <= 0 || n <= 0 || m > INT32_MAX || n > INT32_MAX || m + n > INT32_MAX || nnz < 0) {
        set_error("m, n must be in [1, 2^31) with m + n < 2^31, nnz >= 0");
        return FASTPI_EINVAL;
    }
    if (!rowptr || (nnz > 0 && !col)) {
        set_error("null CSR pointer");
        return FASTPI_EINVAL;
    }
    int* bad = nullptr;
    if (hipHostMalloc(reinterpret_cast<void**>(&bad), sizeof(int)) != hipSuccess) {
        set_error("pinned allocation failed");
        return FASTPI_ENOMEM;
    }
    int* dbad = nullptr;
    if (hipMalloc(reinterpret_cast<void**>(&dbad), sizeof(int)) != hipSuccess) {
        hipHostFree(bad);
        set_error("device allocation failed");
        return FASTPI_ENOMEM;
    }
    int rc = FASTPI_OK;
    auto read = [&]() {
        return hipMemcpyAsync(bad, dbad, sizeof(int), hipMemcpyDeviceToHost, st) == hipSuccess &&
               hipStreamSynchronize(st) == hipSuccess;
    };
    launch_fill_i32(dbad, 1, 0, st);
    hipLaunchKernelGGL(k_check_rowptr, dim3(grid_of(m)), dim3(kThreads), 0, st, rowptr, m, nnz, dbad);
    if (!read()) {
        set_error("GPU validation failed");
        rc = FASTPI_EHIP;
    } else if (*bad) {
        set_error("rowptr must start at 0, end at nnz and be monotone");
        rc = FASTPI_ESHAPE;
    } else {
        hipLaunchKernelGGL(k_check_entries, dim3(grid_of(m)), dim3(kThreads), 0, st, rowptr, col, val, m, n, dbad);
        if (!read()) {
            set_error("GPU validation failed");
            rc = FASTPI_EHIP;
        } else if (*bad & 2) {
            set_error("column index out of range or not strictly increasing within a row");
            rc = FASTPI_ESHAPE;
        } else if (*bad & 4) {
            set_error("non-finite value");
            rc = FASTPI_ENONFINITE;
        }
    }
    hipFree(dbad);
    hipHostFree(bad);
    return rc;
}

int reorder_pattern_gpu(int64_t m, int64_t n, const int64_t* rowptr, const int32_t* col, const double* val,
                        int64_t nnz, double k, hipStream_t st, ReorderOut& out) {
    if (!(k > 0.0 && k < 1.0)) {
        set_error("k must lie in (0, 1)");
        return FASTPI_EINVAL;
    }
    auto hip_fail = [](const char* what) {
        set_error(std::string("GPU reordering: ") + what);
        return FASTPI_EHIP;
    };
    DevBuf db;
    const int64_t total = m + n;
    const int64_t side = std::max(m, n);
    int* cnt = db.get<int>(side + 1);
    int64_t* rp = db.get<int64_t>(m + 1);
    int64_t* cp = db.get<int64_t>(n + 1);
    int* ccnt = db.get<int>(n);
    int* cpos = db.get<int>(n);
    int* rc = db.get<int>(nnz);
    int* cr = db.get<int>(nnz);
    unsigned char* aliveT = db.get<unsigned char>(m);
    unsigned char* aliveF = db.get<unsigned char>(n);
    int* degT = db.get<int>(m);
    int* degF = db.get<int>(n);
    int* histT = db.get<int>(n + 1);   // row degrees are at most n
    int* histF = db.get<int>(m + 1);
    int* flag = db.get<int>(side);
    int64_t* rank = db.get<int64_t>(side + 1);
    int64_t* thr = db.get<int64_t>(2);
    int* lab = db.get<int>(total);
    int* size = db.get<int>(total);
    int* piT = db.get<int>(m);
    int* piF = db.get<int>(n);
    unsigned long long* keys = db.get<unsigned long long>(pow2_at_least(side));
    int* words = db.get<int>(8);   // [0] key count, [1] giant nodes, [2] changed, [3] components
    unsigned long long* best = db.get<unsigned long long>(1);
    Scan sc;
    sc.cap = (side + kScanBlock - 1) / kScanBlock + 1;
    sc.sums = db.get<int64_t>(sc.cap + 1);
    for (void* p : db.ptrs)
        if (!p) {
            set_error("GPU reordering: device allocation failed");
            return FASTPI_ENOMEM;
        }
    int* hwords = nullptr;
    if (hipHostMalloc(reinterpret_cast<void**>(&hwords), 8 * sizeof(int)) != hipSuccess)
        return hip_fail("pinned allocation failed");
    struct HostFree {
        int* p;
        ~HostFree() { hipHostFree(p); }
    } hf{hwords};
    unsigned long long* hbest = nullptr;
    if (hipHostMalloc(reinterpret_cast<void**>(&hbest), sizeof(unsigned long long)) != hipSuccess)
        return hip_fail("pinned allocation failed");
    struct HostFree64 {
        unsigned long long* p;
        ~HostFree64() { hipHostFree(p); }
    } hf64{hbest};
    auto sync = [&]() { return hipStreamSynchronize(st) == hipSuccess; };
    auto read_words = [&]() -> bool {
        return hipMemcpyAsync(hwords, words, 8 * sizeof(int), hipMemcpyDeviceToHost, st) == hipSuccess && sync();
    };

    // graph without stored zeros: CSR, then CSC (column cursors start at the column offsets)
    hipLaunchKernelGGL(k_row_keep, dim3(grid_of(m)), dim3(kThreads), 0, st, rowptr, val, m, cnt);
    scan_ints(cnt, m, 0, rp, sc, st);
    launch_fill_i32(ccnt, n, 0, st);
    hipLaunchKernelGGL(k_row_fill, dim3(grid_of(m)), dim3(kThreads), 0, st, rowptr, col, val, m, rp, rc, ccnt);
    scan_ints(ccnt, n, 0, cp, sc, st);
    {
        std::vector<int64_t> hcp(static_cast<size_t>(n) + 1);
        if (hipMemcpyAsync(hcp.data(), cp, (n + 1) * sizeof(int64_t), hipMemcpyDeviceToHost, st) != hipSuccess ||
            !sync())
            return hip_fail("copy failed");
        std::vector<int> hpos(static_cast<size_t>(n));
        for (int64_t j = 0; j < n; ++j) hpos[j] = static_cast<int>(hcp[j]);
        if (hipMemcpyAsync(cpos, hpos.data(), n * sizeof(int), hipMemcpyHostToDevice, st) != hipSuccess)
            return hip_fail("copy failed");
        out.nnz_edges = hcp[n];
        hipLaunchKernelGGL(k_col_fill, dim3(grid_of(m)), dim3(kThreads), 0, st, rp, rc, m, cpos, cr);
        if (!sync()) return hip_fail("graph build failed");
    }
    hipLaunchKernelGGL(k_fill_u8, dim3(grid_of(m)), dim3(kThreads), 0, st, aliveT, m, static_cast<unsigned char>(1));
    hipLaunchKernelGGL(k_fill_u8, dim3(grid_of(n)), dim3(kThreads), 0, st, aliveF, n, static_cast<unsigned char>(1));
    launch_fill_i32(piT, m, -1, st);
    launch_fill_i32(piF, n, -1, st);

    // hubs of one side from its degrees and histogram (maxdeg: the other side's size)
    auto take_hubs = [&](int64_t cntv, int64_t maxdeg, const int* deg, const int* hist, int64_t h, int64_t& hi,
                         int* pi, unsigned char* alive) -> bool {
        if (h <= 0) return true;
        hipLaunchKernelGGL(k_hub_threshold, dim3(1), dim3(1024), 0, st, hist, maxdeg, h, thr);
        hipLaunchKernelGGL(k_eq_flags, dim3(grid_of(cntv)), dim3(kThreads), 0, st, deg, cntv, thr, flag);
        scan_ints(flag, cntv, 0, rank, sc, st);
        launch_fill_i32(words, 8, 0, st);
        hipLaunchKernelGGL(k_hub_keys, dim3(grid_of(cntv)), dim3(kThreads), 0, st, deg, cntv, thr, rank, keys,
                           words);
        // exactly h keys, or the ids below would come from unwritten slots
        if (!read_words() || hwords[0] != h) return false;
        sort_keys(keys, h, st);
        hipLaunchKernelGGL(k_hub_assign, dim3(grid_of(h)), dim3(kThreads), 0, st, keys, h, hi, pi, alive);
        hi -= h;
        return true;
    };
    // the non-giant nodes of one side, sorted by (component code, index); returns their codes
    auto take_spokes = [&](int64_t from, int64_t cntv, int giant, int64_t& lo, int* pi, unsigned char* alive,
                           std::vector<int>& codes, int64_t& ngiant) -> bool {
        launch_fill_i32(words, 8, 0, st);
        hipLaunchKernelGGL(k_spoke_keys, dim3(grid_of(cntv)), dim3(kThreads), 0, st, lab, from, cntv, giant, keys,
                           words, words + 1);
        if (!read_words()) return false;
        const int64_t nk = hwords[0];
        ngiant = hwords[1];
        codes.assign(static_cast<size_t>(nk), 0);
        if (nk == 0) return true;
        sort_keys(keys, nk, st);
        hipLaunchKernelGGL(k_spoke_assign, dim3(grid_of(nk)), dim3(kThreads), 0, st, keys, nk, lo, pi, alive);
        std::vector<unsigned long long> hk(static_cast<size_t>(nk));
        if (hipMemcpyAsync(hk.data(), keys, nk * sizeof(unsigned long long), hipMemcpyDeviceToHost, st) !=
                hipSuccess ||
            !sync())
            return false;
        for (int64_t r = 0; r < nk; ++r) codes[r] = static_cast<int>(hk[r] >> 32);
        lo += nk;
        return true;
    };

    out.blocks.clear();
    int64_t nT = m, nF = n, loT = 0, loF = 0, hiT = m - 1, hiF = n - 1, iters = 0;
    while (true) {
        ++iters;
        const int64_t mh = std::min(target_rank(k, nT), nT), nh = std::min(target_rank(k, nF), nF);
        // 1. degrees of both sides in the current graph
        launch_fill_i32(histT, n + 1, 0, st);
        launch_fill_i32(histF, m + 1, 0, st);
        hipLaunchKernelGGL(k_degrees, dim3(grid_of(m)), dim3(kThreads), 0, st, rp, rc, m, aliveT, aliveF, degT,
                           histT);
        hipLaunchKernelGGL(k_degrees, dim3(grid_of(n)), dim3(kThreads), 0, st, cp, cr, n, aliveF, aliveT, degF,
                           histF);
        // 2. hubs take the highest free ids
        if (!take_hubs(m, n, degT, histT, mh, hiT, piT, aliveT) || !take_hubs(n, m, degF, histF, nh, hiF, piF, aliveF))
            return hip_fail("hub selection failed");
        // 3. components of the rest
        hipLaunchKernelGGL(k_cc_init, dim3(grid_of(total)), dim3(kThreads), 0, st, aliveT, aliveF, m, n, lab);
        for (int pass = 0;; ++pass) {
            launch_fill_i32(words, 8, 0, st);
            hipLaunchKernelGGL(k_cc_hook, dim3(grid_of(m)), dim3(kThreads), 0, st, rp, rc, m, lab, words + 2);
            hipLaunchKernelGGL(k_cc_jump, dim3(grid_of(total)), dim3(kThreads), 0, st, total, lab, words + 2);
            if (!read_words()) return hip_fail("component labelling failed");
            if (hwords[2] == 0) break;
            if (pass > 4 * (total + 1)) return hip_fail("component labelling did not settle");
        }
        // 4. giant: most nodes, the smallest code on ties
        launch_fill_i32(size, total, 0, st);
        launch_fill_i32(words, 8, 0, st);
        hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(kThreads), 0, st, best, static_cast<int64_t>(0),
                           static_cast<int64_t>(1), 0ull);
        hipLaunchKernelGGL(k_cc_sizes, dim3(grid_of(total)), dim3(kThreads), 0, st, lab, total, size);
        hipLaunchKernelGGL(k_cc_giant, dim3(grid_of(total)), dim3(kThreads), 0, st, lab, size, total, best, words + 3);
        if (hipMemcpyAsync(hbest, best, sizeof(unsigned long long), hipMemcpyDeviceToHost, st) != hipSuccess ||
            !read_words())
            return hip_fail("giant selection failed");
        if (hwords[3] == 0) {   // nothing left after the hubs
            nT = nF = 0;
            break;
        }
        const int giant = 0x7FFFFFFF - static_cast<int>(*hbest & 0xFFFFFFFFull);
        std::vector<int> codesT, codesF;
        int64_t gT = 0, gF = 0;
        const int64_t lo0T = loT, lo0F = loF;
        if (!take_spokes(0, m, giant, loT, piT, aliveT, codesT, gT) ||
            !take_spokes(m, n, giant, loF, piF, aliveF, codesF, gF))
            return hip_fail("spoke assignment failed");
        // blocks in component order: merge the two sorted code lists
        {
            size_t a = 0, b = 0;
            int64_t r0 = lo0T, c0 = lo0F;
            while (a < codesT.size() || b < codesF.size()) {
                const int c = (b >= codesF.size() || (a < codesT.size() && codesT[a] <= codesF[b])) ? codesT[a]
                                                                                                   : codesF[b];
                int64_t nr = 0, nc = 0;
                while (a < codesT.size() && codesT[a] == c) ++a, ++nr;
                while (b < codesF.size() && codesF[b] == c) ++b, ++nc;
                out.blocks.push_back({r0, c0, nr, nc});
                r0 += nr;
                c0 += nc;
            }
        }
        nT = gT;
        nF = gF;
        if (gT < mh || gF < nh || gT + gF == 0) break;
    }
    // the last giant: ascending ids
    if (nT > 0 || nF > 0) {
        out.blocks.push_back({loT, loF, nT, nF});
        hipLaunchKernelGGL(k_alive_flags, dim3(grid_of(m)), dim3(kThreads), 0, st, aliveT, m, flag);
        scan_ints(flag, m, 0, rank, sc, st);
        hipLaunchKernelGGL(k_final_assign, dim3(grid_of(m)), dim3(kThreads), 0, st, aliveT, rank, m, loT, piT);
        hipLaunchKernelGGL(k_alive_flags, dim3(grid_of(n)), dim3(kThreads), 0, st, aliveF, n, flag);
        scan_ints(flag, n, 0, rank, sc, st);
        hipLaunchKernelGGL(k_final_assign, dim3(grid_of(n)), dim3(kThreads), 0, st, aliveF, rank, n, loF, piF);
        loT += nT;
        loF += nF;
    }
    if (loT != hiT + 1 || loF != hiF + 1) {
        set_error("internal: GPU reordering ids do not meet");
        return FASTPI_EINTERNAL;
    }
    out.piT.assign(static_cast<size_t>(m), -1);
    out.piF.assign(static_cast<size_t>(n), -1);
    if (hipMemcpyAsync(out.piT.data(), piT, m * sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipMemcpyAsync(out.piF.data(), piF, n * sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess || !sync())
        return hip_fail("copy of the permutation failed");
    if (hipGetLastError() != hipSuccess) return hip_fail("kernel launch failed");
    out.m1 = loT;
    out.n1 = loF;
    out.m2 = m - loT;
    out.n2 = n - loF;
    out.iterations = iters;
    return FASTPI_OK;
}

}  // namespace fastpi
