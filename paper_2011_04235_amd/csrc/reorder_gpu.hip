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
//  3. connected components of what remains, by lock-free union-find that always hooks the
//     larger root under the smaller: node codes are row i -> i and column j -> m + j, and
//     every node ends with the smallest code of its component. That code is the component's seed in the scan order (rows by
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

// One wave (64 lanes) per node: the node index of this wave, uniform across its lanes.
#define WAVE_NODE(v, cnt)                                                                                    \
    const int lane = threadIdx.x % 64;                                                                    \
    const int64_t v = static_cast<int64_t>(blockIdx.x) * (kThreads / 64) +                             \
                      __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x / 64));                  \
    if (v >= (cnt)) return;

__device__ inline int wave_sum_i(int x) {
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    return x;
}

__device__ inline int wave_min_i(int x) {
    for (int off = 32; off > 0; off >>= 1) x = min(x, __shfl_xor(x, off, 64));
    return x;
}

// one atomic per wave: the lanes with `take` get consecutive slots of *counter (every lane of
// the wave must call this)
__device__ inline int wave_slot(bool take, int* counter) {
    const unsigned long long mask = __ballot(take);
    const int lane = threadIdx.x % 64;
    int base = 0;
    if (mask) {
        const int leader = __ffsll(static_cast<long long>(mask)) - 1;
        if (lane == leader) base = atomicAdd(counter, __popcll(mask));
        base = __shfl(base, leader, 64);
    }
    return base + __popcll(mask & ((1ull << lane) - 1ull));
}

unsigned wave_grid(int64_t nodes) {
    return static_cast<unsigned>(std::max<int64_t>(1, (nodes + kThreads / 64 - 1) / (kThreads / 64)));
}

// ---- graph build -----------------------------------------------------------------------
// nonzero-valued entries per row (all entries when val is null); one wave per row
__global__ __launch_bounds__(kThreads) void k_row_keep(const int64_t* __restrict__ rowptr,
                                                       const double* __restrict__ val, int64_t m,
                                                       int* __restrict__ cnt) {
    WAVE_NODE(i, m)
    int c = 0;
    for (int64_t e = rowptr[i] + lane; e < rowptr[i + 1]; e += 64) c += (val == nullptr || val[e] != 0.0) ? 1 : 0;
    c = wave_sum_i(c);
    if (lane == 0) cnt[i] = c;
}

// kept entries in order (ballot prefix inside each chunk of 64), column counts on the side
__global__ __launch_bounds__(kThreads) void k_row_fill(const int64_t* __restrict__ rowptr,
                                                       const int* __restrict__ col,
                                                       const double* __restrict__ val, int64_t m,
                                                       const int64_t* __restrict__ rp, int* __restrict__ rc,
                                                       int* __restrict__ ccnt) {
    WAVE_NODE(i, m)
    int64_t base = rp[i];
    const int64_t end = rowptr[i + 1];
    for (int64_t e0 = rowptr[i]; e0 < end; e0 += 64) {
        const int64_t e = e0 + lane;
        const bool keep = e < end && (val == nullptr || val[e] != 0.0);
        const unsigned long long mask = __ballot(keep);
        if (keep) {
            const int pos = __popcll(mask & ((1ull << lane) - 1ull));
            const int c = col[e];
            rc[base + pos] = c;
            atomicAdd(&ccnt[c], 1);
        }
        base += __popcll(mask);
    }
}

// CSC from the kept CSR; the order inside a column is immaterial (degrees and components
// do not depend on it)
__global__ __launch_bounds__(kThreads) void k_col_fill(const int64_t* __restrict__ rp, const int* __restrict__ rc,
                                                       int64_t m, int* __restrict__ cpos, int* __restrict__ cr) {
    WAVE_NODE(i, m)
    for (int64_t e = rp[i] + lane; e < rp[i + 1]; e += 64) {
        const int slot = atomicAdd(&cpos[rc[e]], 1);
        cr[slot] = static_cast<int>(i);
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
// A node with at most kLight edges is handled by one thread; heavier nodes (listed once) by
// one wave each, lanes striding over the edges (hub-like nodes have thousands).
constexpr int64_t kLight = 64;

__device__ inline void put_degree(int64_t v, int d, int* deg, int* hist, int* dmax) {
    deg[v] = d;
    atomicAdd(&hist[d], 1);
    atomicMax(dmax, d);
}

__global__ __launch_bounds__(kThreads) void k_degrees(const int64_t* __restrict__ ptr, const int* __restrict__ idx,
                                                      int64_t cnt, const unsigned char* __restrict__ alive_self,
                                                      const unsigned char* __restrict__ alive_other,
                                                      int* __restrict__ deg, int* __restrict__ hist,
                                                      int* __restrict__ dmax) {
    GRID_STRIDE(v, cnt) {
        if (!alive_self[v]) {
            deg[v] = -1;
            continue;
        }
        const int64_t b = ptr[v], e1 = ptr[v + 1];
        if (e1 - b > kLight) continue;   // heavy: k_degrees_heavy
        int d = 0;
        for (int64_t e = b; e < e1; ++e) d += alive_other[idx[e]];
        put_degree(v, d, deg, hist, dmax);
    }
}

__global__ __launch_bounds__(kThreads) void k_degrees_heavy(const int64_t* __restrict__ ptr,
                                                            const int* __restrict__ idx,
                                                            const int* __restrict__ heavy, int64_t nheavy,
                                                            const unsigned char* __restrict__ alive_self,
                                                            const unsigned char* __restrict__ alive_other,
                                                            int* __restrict__ deg, int* __restrict__ hist,
                                                            int* __restrict__ dmax) {
    WAVE_NODE(h, nheavy)
    const int64_t v = heavy[h];
    if (!alive_self[v]) return;   // deg[v] = -1 was written by k_degrees
    int d = 0;
    for (int64_t e = ptr[v] + lane; e < ptr[v + 1]; e += 64) d += alive_other[idx[e]];
    d = wave_sum_i(d);
    if (lane == 0) put_degree(v, d, deg, hist, dmax);
}

// One workgroup: the threshold degree D with count(deg > D) < h <= count(deg >= D), written
// as out[0] = D, out[1] = h - count(deg > D) (nodes of degree D to take, lowest index first).
__global__ __launch_bounds__(1024) void k_hub_threshold(const int* __restrict__ hist, const int* __restrict__ dmax,
                                                        int64_t h, int64_t* __restrict__ out) {
    __shared__ int64_t s[1024];
    const int64_t bins = static_cast<int64_t>(*dmax) + 1;   // every bin above the largest degree is empty
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
        const bool hub = d >= 0 && (d > D || (d == D && eqrank[v] < take));
        const int slot = wave_slot(hub, nkeys);
        if (hub)
            keys[slot] = (static_cast<unsigned long long>(0x7FFFFFFF - d) << 32) | static_cast<unsigned long long>(v);
    }
}

// hub r (in key order) takes id hi - r and leaves the graph; slots still holding the
// all-ones filler (fewer keys than expected) are skipped, and the final id check reports it
__global__ void k_hub_assign(const unsigned long long* __restrict__ keys, int64_t h, int64_t hi, int64_t cnt,
                             int* __restrict__ pi, unsigned char* __restrict__ alive) {
    GRID_STRIDE(r, h) {
        const unsigned long long key = keys[r];
        const int64_t v = static_cast<int64_t>(key & 0xFFFFFFFFull);
        if (key == ~0ull || v >= cnt) continue;
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

// the whole sort of at most 4096 keys in one workgroup
__global__ __launch_bounds__(1024) void k_bitonic_small(unsigned long long* __restrict__ a, int64_t n) {
    __shared__ unsigned long long s[4096];
    for (int t = threadIdx.x; t < n; t += 1024) s[t] = a[t];
    __syncthreads();
    for (int k = 2; k <= n; k <<= 1)
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int t = threadIdx.x; t < n; t += 1024) {
                const int l = t ^ j;
                if (l > t) {
                    const bool up = (t & k) == 0;
                    const unsigned long long x = s[t], y = s[l];
                    if ((x > y) == up) {
                        s[t] = y;
                        s[l] = x;
                    }
                }
            }
            __syncthreads();
        }
    for (int t = threadIdx.x; t < n; t += 1024) a[t] = s[t];
}

__global__ void k_copy_u64(const unsigned long long* __restrict__ src, int64_t n,
                           unsigned long long* __restrict__ dst) {
    GRID_STRIDE(i, n) dst[i] = src[i];
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

// ---- union-find ------------------------------------------------------------------------
// p[v] <= v always: a root is only ever hooked under a smaller root, so the root of every
// set is its smallest code, whatever the order of the unions. find() halves the path it
// walks (benign races: every write moves a node to one of its ancestors).
// Parent reads and writes go to the device-coherent level (relaxed atomics at agent
// scope): plain loads may be served from a compute unit's own cache, which does not see
// the hooks other compute units make during the launch.
__device__ inline int uf_load(const int* p, int v) {
    return __hip_atomic_load(p + v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline void uf_store(int* p, int v, int x) {
    __hip_atomic_store(p + v, x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline int uf_find(int* p, int v) {
    int par = uf_load(p, v);
    if (par != v) {
        int prev = v, next;
        while (par > (next = uf_load(p, par))) {
            uf_store(p, prev, next);
            prev = par;
            par = next;
        }
    }
    return par;
}

__device__ inline void uf_unite(int* p, int a, int b) {
    int ra = uf_find(p, a), rb = uf_find(p, b);
    while (ra != rb) {
        if (ra > rb) {
            const int t = ra;
            ra = rb;
            rb = t;
        }
        // hook the larger root rb under ra; if rb stopped being a root, climb and retry
        const int old = atomicCAS(&p[rb], rb, ra);
        if (old == rb) break;
        rb = uf_find(p, old);
        ra = uf_find(p, ra);
    }
}

__global__ __launch_bounds__(kThreads) void k_uf_hook(const int64_t* __restrict__ rp, const int* __restrict__ rc,
                                                      int64_t m, int* p) {
    GRID_STRIDE(i, m) {
        const int64_t b = rp[i], e1 = rp[i + 1];
        if (e1 - b > kLight || p[i] < 0) continue;   // heavy rows: k_uf_hook_heavy
        for (int64_t e = b; e < e1; ++e) {
            const int vj = static_cast<int>(m + rc[e]);
            if (p[vj] >= 0) uf_unite(p, static_cast<int>(i), vj);
        }
    }
}

__global__ __launch_bounds__(kThreads) void k_uf_hook_heavy(const int64_t* __restrict__ rp, const int* __restrict__ rc,
                                                            int64_t m, const int* __restrict__ heavy, int64_t nheavy,
                                                            int* p) {
    WAVE_NODE(h, nheavy)
    const int64_t i = heavy[h];
    if (p[i] < 0) return;
    for (int64_t e = rp[i] + lane; e < rp[i + 1]; e += 64) {
        const int vj = static_cast<int>(m + rc[e]);
        if (p[vj] >= 0) uf_unite(p, static_cast<int>(i), vj);
    }
}

// every alive node points at its root (after all unions). The walk only reads: a halving
// store here could overwrite a node already set to its root with an older ancestor, and the
// node would end outside its component's count. The only stores are roots.
__global__ void k_uf_compress(int64_t total, int* p) {
    GRID_STRIDE(v, total) {
        int r = uf_load(p, static_cast<int>(v));
        if (r < 0) continue;
        for (int nx = uf_load(p, r); nx != r; nx = uf_load(p, r)) r = nx;
        uf_store(p, static_cast<int>(v), r);
    }
}

// sizes per root code; the giant as the maximum of (size, -code) packed in 64 bits
// most nodes share the giant's label: the lanes of a wave with equal labels add together
__global__ __launch_bounds__(kThreads) void k_cc_sizes(const int* __restrict__ lab, int64_t total,
                                                       int* __restrict__ size) {
    const int lane = threadIdx.x % 64;
    // the loop bound is uniform across the workgroup, so every lane joins every ballot
    for (int64_t base = static_cast<int64_t>(blockIdx.x) * blockDim.x; base < total;
         base += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int64_t v = base + threadIdx.x;
        const int l = v < total ? lab[v] : -1;
        bool pending = l >= 0;
        while (true) {
            const unsigned long long act = __ballot(pending);
            if (!act) break;
            const int leader = __ffsll(static_cast<long long>(act)) - 1;
            const int ll = __shfl(l, leader, 64);
            const bool mine = pending && l == ll;
            const unsigned long long same = __ballot(mine);
            if (lane == leader) atomicAdd(&size[ll], __popcll(same));
            if (mine) pending = false;
        }
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
__global__ void k_spoke_keys(const int* __restrict__ lab, int64_t from, int64_t cnt,
                             const unsigned long long* __restrict__ best, unsigned long long* __restrict__ keys,
                             int* __restrict__ nkeys, int* __restrict__ ngiant) {
    const int giant = 0x7FFFFFFF - static_cast<int>(*best & 0xFFFFFFFFull);
    GRID_STRIDE(i, cnt) {
        const int l = lab[from + i];
        const bool in_giant = l >= 0 && l == giant;
        const bool spoke = l >= 0 && l != giant;
        wave_slot(in_giant, ngiant);
        const int slot = wave_slot(spoke, nkeys);
        if (spoke) keys[slot] = (static_cast<unsigned long long>(l) << 32) | static_cast<unsigned long long>(i);
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
__global__ __launch_bounds__(kThreads) void k_check_entries(const int64_t* __restrict__ rowptr,
                                                             const int* __restrict__ col,
                                                             const double* __restrict__ val, int64_t m, int64_t n,
                                                             int* __restrict__ bad) {
    WAVE_NODE(i, m)
    int flags = 0;
    for (int64_t e = rowptr[i] + lane; e < rowptr[i + 1]; e += 64) {
        const int c = col[e];
        if (c < 0 || c >= n || (e > rowptr[i] && c <= col[e - 1])) flags |= 2;
        if (val && !isfinite(val[e])) flags |= 4;
    }
    if (__any(flags & 2) && lane == 0) atomicOr(bad, 2);
    if (__any(flags & 4) && lane == 0) atomicOr(bad, 4);
}

#undef GRID_STRIDE
#undef WAVE_NODE

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
    if (p2 <= 4096) {
        hipLaunchKernelGGL(k_bitonic_small, dim3(1), dim3(1024), 0, st, keys, p2);
        return;
    }
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
        hipLaunchKernelGGL(k_check_entries, dim3(wave_grid(m)), dim3(kThreads), 0, st, rowptr, col, val, m, n, dbad);
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
    unsigned long long* keysT = db.get<unsigned long long>(pow2_at_least(m));
    unsigned long long* keysF = db.get<unsigned long long>(pow2_at_least(n));
    unsigned long long* logT = db.get<unsigned long long>(m);   // sorted spoke keys of every iteration
    unsigned long long* logF = db.get<unsigned long long>(n);
    // [0] row keys, [1] row giant nodes, [3] components, [4] column keys, [5] column giant nodes,
    // [6] [7] row and column hub keys
    int* words = db.get<int>(8);
    int* dmax = db.get<int>(2);   // largest degree of the rows, of the columns
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

    int *heavyT = nullptr, *heavyF = nullptr;
    int64_t nheavyT = 0, nheavyF = 0;
    // graph without stored zeros: CSR, then CSC (column cursors start at the column offsets)
    hipLaunchKernelGGL(k_row_keep, dim3(wave_grid(m)), dim3(kThreads), 0, st, rowptr, val, m, cnt);
    scan_ints(cnt, m, 0, rp, sc, st);
    launch_fill_i32(ccnt, n, 0, st);
    hipLaunchKernelGGL(k_row_fill, dim3(wave_grid(m)), dim3(kThreads), 0, st, rowptr, col, val, m, rp, rc, ccnt);
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
        hipLaunchKernelGGL(k_col_fill, dim3(wave_grid(m)), dim3(kThreads), 0, st, rp, rc, m, cpos, cr);
        // nodes with more than kLight edges go to the one-wave-per-node kernels
        std::vector<int64_t> hrp(static_cast<size_t>(m) + 1);
        if (hipMemcpyAsync(hrp.data(), rp, (m + 1) * sizeof(int64_t), hipMemcpyDeviceToHost, st) != hipSuccess ||
            !sync())
            return hip_fail("graph build failed");
        std::vector<int> hT, hF;
        for (int64_t i = 0; i < m; ++i)
            if (hrp[i + 1] - hrp[i] > kLight) hT.push_back(static_cast<int>(i));
        for (int64_t j = 0; j < n; ++j)
            if (hcp[j + 1] - hcp[j] > kLight) hF.push_back(static_cast<int>(j));
        nheavyT = static_cast<int64_t>(hT.size());
        nheavyF = static_cast<int64_t>(hF.size());
        heavyT = db.get<int>(nheavyT);
        heavyF = db.get<int>(nheavyF);
        if (!heavyT || !heavyF) {
            set_error("GPU reordering: device allocation failed");
            return FASTPI_ENOMEM;
        }
        if ((nheavyT && hipMemcpyAsync(heavyT, hT.data(), nheavyT * sizeof(int), hipMemcpyHostToDevice, st) !=
                            hipSuccess) ||
            (nheavyF && hipMemcpyAsync(heavyF, hF.data(), nheavyF * sizeof(int), hipMemcpyHostToDevice, st) !=
                            hipSuccess) ||
            !sync())
            return hip_fail("graph build failed");
    }
    hipLaunchKernelGGL(k_fill_u8, dim3(grid_of(m)), dim3(kThreads), 0, st, aliveT, m, static_cast<unsigned char>(1));
    hipLaunchKernelGGL(k_fill_u8, dim3(grid_of(n)), dim3(kThreads), 0, st, aliveF, n, static_cast<unsigned char>(1));
    launch_fill_i32(piT, m, -1, st);
    launch_fill_i32(piF, n, -1, st);

    // hubs of one side from its degrees and histogram (maxdeg: the other side's size); the key
    // slots start as all-ones so that a short count cannot hand out stale indices
    auto take_hubs = [&](int64_t cntv, const int* dm, const int* deg, const int* hist, int64_t h, int64_t& hi,
                         int* pi, unsigned char* alive, unsigned long long* keys, int* nkeys) {
        if (h <= 0) return;
        hipLaunchKernelGGL(k_fill_u64, dim3(grid_of(h)), dim3(kThreads), 0, st, keys, static_cast<int64_t>(0), h,
                           ~0ull);
        hipLaunchKernelGGL(k_hub_threshold, dim3(1), dim3(1024), 0, st, hist, dm, h, thr);
        hipLaunchKernelGGL(k_eq_flags, dim3(grid_of(cntv)), dim3(kThreads), 0, st, deg, cntv, thr, flag);
        scan_ints(flag, cntv, 0, rank, sc, st);
        hipLaunchKernelGGL(k_hub_keys, dim3(grid_of(cntv)), dim3(kThreads), 0, st, deg, cntv, thr, rank, keys,
                           nkeys);
        sort_keys(keys, h, st);
        hipLaunchKernelGGL(k_hub_assign, dim3(grid_of(h)), dim3(kThreads), 0, st, keys, h, hi, cntv, pi, alive);
        hi -= h;
    };

    out.blocks.clear();
    struct Peel {
        int64_t loT, loF, offT, offF, nkT, nkF;   // ids and log offsets of one iteration's spokes
    };
    std::vector<Peel> peels;
    int64_t nT = m, nF = n, loT = 0, loF = 0, hiT = m - 1, hiF = n - 1, iters = 0;
    while (true) {
        ++iters;
        const int64_t mh = std::min(target_rank(k, nT), nT), nh = std::min(target_rank(k, nF), nF);
        // 1. degrees of both sides in the current graph
        launch_fill_i32(histT, n + 1, 0, st);
        launch_fill_i32(histF, m + 1, 0, st);
        launch_fill_i32(words, 8, 0, st);
        launch_fill_i32(dmax, 2, 0, st);
        hipLaunchKernelGGL(k_degrees, dim3(grid_of(m)), dim3(kThreads), 0, st, rp, rc, m, aliveT, aliveF, degT,
                           histT, dmax);
        if (nheavyT)
            hipLaunchKernelGGL(k_degrees_heavy, dim3(wave_grid(nheavyT)), dim3(kThreads), 0, st, rp, rc, heavyT,
                               nheavyT, aliveT, aliveF, degT, histT, dmax);
        hipLaunchKernelGGL(k_degrees, dim3(grid_of(n)), dim3(kThreads), 0, st, cp, cr, n, aliveF, aliveT, degF,
                           histF, dmax + 1);
        if (nheavyF)
            hipLaunchKernelGGL(k_degrees_heavy, dim3(wave_grid(nheavyF)), dim3(kThreads), 0, st, cp, cr, heavyF,
                               nheavyF, aliveF, aliveT, degF, histF, dmax + 1);
        // 2. hubs take the highest free ids
        take_hubs(m, dmax, degT, histT, mh, hiT, piT, aliveT, keysT, words + 6);
        take_hubs(n, dmax + 1, degF, histF, nh, hiF, piF, aliveF, keysF, words + 7);
        // 3. components of the rest: union-find over the alive edges, then full compression
        hipLaunchKernelGGL(k_cc_init, dim3(grid_of(total)), dim3(kThreads), 0, st, aliveT, aliveF, m, n, lab);
        hipLaunchKernelGGL(k_uf_hook, dim3(grid_of(m)), dim3(kThreads), 0, st, rp, rc, m, lab);
        if (nheavyT)
            hipLaunchKernelGGL(k_uf_hook_heavy, dim3(wave_grid(nheavyT)), dim3(kThreads), 0, st, rp, rc, m, heavyT,
                               nheavyT, lab);
        hipLaunchKernelGGL(k_uf_compress, dim3(grid_of(total)), dim3(kThreads), 0, st, total, lab);
        // 4. giant (most nodes, the smallest code on ties) and the spoke keys of both sides
        launch_fill_i32(size, total, 0, st);
        hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(kThreads), 0, st, best, static_cast<int64_t>(0),
                           static_cast<int64_t>(1), 0ull);
        hipLaunchKernelGGL(k_cc_sizes, dim3(grid_of(total)), dim3(kThreads), 0, st, lab, total, size);
        hipLaunchKernelGGL(k_cc_giant, dim3(grid_of(total)), dim3(kThreads), 0, st, lab, size, total, best, words + 3);
        hipLaunchKernelGGL(k_spoke_keys, dim3(grid_of(m)), dim3(kThreads), 0, st, lab, static_cast<int64_t>(0), m,
                           best, keysT, words, words + 1);
        hipLaunchKernelGGL(k_spoke_keys, dim3(grid_of(n)), dim3(kThreads), 0, st, lab, m, n, best, keysF, words + 4,
                           words + 5);
        if (!read_words()) return hip_fail("component counts failed");
        if (hwords[3] == 0) {   // nothing left after the hubs
            nT = nF = 0;
            break;
        }
        const int64_t nkT = hwords[0], gT = hwords[1], nkF = hwords[4], gF = hwords[5];
        // every node left after the hubs is in the giant or in a spoke
        if (nkT + gT != nT - mh || nkF + gF != nF - nh) return hip_fail("component counts do not add up");
        Peel pl{loT, loF, 0, 0, nkT, nkF};
        pl.offT = peels.empty() ? 0 : peels.back().offT + peels.back().nkT;
        pl.offF = peels.empty() ? 0 : peels.back().offF + peels.back().nkF;
        if (nkT > 0) {
            sort_keys(keysT, nkT, st);
            hipLaunchKernelGGL(k_spoke_assign, dim3(grid_of(nkT)), dim3(kThreads), 0, st, keysT, nkT, loT, piT,
                               aliveT);
            hipLaunchKernelGGL(k_copy_u64, dim3(grid_of(nkT)), dim3(kThreads), 0, st, keysT, nkT, logT + pl.offT);
        }
        if (nkF > 0) {
            sort_keys(keysF, nkF, st);
            hipLaunchKernelGGL(k_spoke_assign, dim3(grid_of(nkF)), dim3(kThreads), 0, st, keysF, nkF, loF, piF,
                               aliveF);
            hipLaunchKernelGGL(k_copy_u64, dim3(grid_of(nkF)), dim3(kThreads), 0, st, keysF, nkF, logF + pl.offF);
        }
        peels.push_back(pl);
        loT += nkT;
        loF += nkF;
        nT = gT;
        nF = gF;
        if (gT < mh || gF < nh || gT + gF == 0) break;
    }
    // blocks of every iteration, in component order: merge its two sorted code lists
    {
        const int64_t totT = peels.empty() ? 0 : peels.back().offT + peels.back().nkT;
        const int64_t totF = peels.empty() ? 0 : peels.back().offF + peels.back().nkF;
        std::vector<unsigned long long> hT(static_cast<size_t>(totT)), hF(static_cast<size_t>(totF));
        if ((totT > 0 && hipMemcpyAsync(hT.data(), logT, totT * sizeof(unsigned long long), hipMemcpyDeviceToHost,
                                        st) != hipSuccess) ||
            (totF > 0 && hipMemcpyAsync(hF.data(), logF, totF * sizeof(unsigned long long), hipMemcpyDeviceToHost,
                                        st) != hipSuccess) ||
            !sync())
            return hip_fail("copy of the component log failed");
        for (const Peel& pl : peels) {
            int64_t a = 0, b = 0, r0 = pl.loT, c0 = pl.loF;
            auto codeT = [&](int64_t x) { return static_cast<int64_t>(hT[pl.offT + x] >> 32); };
            auto codeF = [&](int64_t x) { return static_cast<int64_t>(hF[pl.offF + x] >> 32); };
            while (a < pl.nkT || b < pl.nkF) {
                const int64_t c = (b >= pl.nkF || (a < pl.nkT && codeT(a) <= codeF(b))) ? codeT(a) : codeF(b);
                int64_t nr = 0, nc = 0;
                while (a < pl.nkT && codeT(a) == c) ++a, ++nr;
                while (b < pl.nkF && codeF(b) == c) ++b, ++nc;
                out.blocks.push_back({r0, c0, nr, nc});
                r0 += nr;
                c0 += nc;
            }
        }
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
