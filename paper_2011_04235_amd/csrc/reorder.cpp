// Hub-and-spoke matrix reordering on the host (Section 3.2, Algorithm 2).
//
// The feature matrix is a bipartite graph (Definition 1). Every iteration takes the
// ceil(k|V_T|) instance hubs and ceil(k|V_F|) feature hubs of the current graph, gives them
// the highest free ids, finds the connected components of the remainder by breadth-first
// search, gives the non-giant components the lowest free ids, and continues on the giant
// component until it has fewer instance nodes than this iteration's instance-hub count or
// fewer feature nodes than its feature-hub count. The tie-break rules are listed in
// fastpi.h; the result is a pure function of the pattern and k.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>

#include "host_internal.h"

namespace fastpi {

int64_t target_rank(double alpha, int64_t x) {
    double v = std::ceil(alpha * static_cast<double>(x));
    return v > 0 ? static_cast<int64_t>(v) : 0;
}

int validate_csr(int64_t m, int64_t n, const int64_t* rowptr, const int32_t* col,
                 const double* val) {
    if (m <= 0 || n <= 0 || n > INT32_MAX || m > INT32_MAX) {
        set_error("m and n must be in [1, 2^31)");
        return FASTPI_EINVAL;
    }
    if (!rowptr || (!col && rowptr[m] > 0)) {
        set_error("null CSR pointer");
        return FASTPI_EINVAL;
    }
    if (rowptr[0] != 0) {
        set_error("rowptr[0] must be 0");
        return FASTPI_ESHAPE;
    }
    for (int64_t i = 0; i < m; ++i) {
        if (rowptr[i + 1] < rowptr[i]) {
            set_error("rowptr is not monotone at row " + std::to_string(i));
            return FASTPI_ESHAPE;
        }
        for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
            if (col[e] < 0 || col[e] >= n) {
                set_error("column index out of range in row " + std::to_string(i));
                return FASTPI_ESHAPE;
            }
            if (e > rowptr[i] && col[e] <= col[e - 1]) {
                set_error("columns not strictly increasing in row " + std::to_string(i));
                return FASTPI_ESHAPE;
            }
            if (val && !std::isfinite(val[e])) {
                set_error("non-finite value in row " + std::to_string(i));
                return FASTPI_ENONFINITE;
            }
        }
    }
    return FASTPI_OK;
}

namespace {

// hub count ceil(k * count) in double, clamped to count
int64_t hub_count(double k, int64_t count) {
    int64_t h = target_rank(k, count);
    return std::min(h, count);
}

}  // namespace

int reorder_pattern(int64_t m, int64_t n, const int64_t* rowptr, const int32_t* col,
                    const double* val, double k, ReorderOut& out) {
    if (!(k > 0.0 && k < 1.0)) {
        set_error("k must lie in (0, 1)");
        return FASTPI_EINVAL;
    }
    // adjacency in both directions, stored zeros removed
    std::vector<int64_t> rp(m + 1, 0);
    std::vector<int32_t> rc;
    rc.reserve(static_cast<size_t>(rowptr[m]));
    for (int64_t i = 0; i < m; ++i) {
        for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e)
            if (!val || val[e] != 0.0) rc.push_back(col[e]);
        rp[i + 1] = static_cast<int64_t>(rc.size());
    }
    const int64_t E = static_cast<int64_t>(rc.size());
    std::vector<int64_t> cp(n + 1, 0);
    for (int64_t e = 0; e < E; ++e) cp[rc[e] + 1]++;
    for (int64_t j = 0; j < n; ++j) cp[j + 1] += cp[j];
    std::vector<int32_t> cr(E);
    {
        std::vector<int64_t> fill(cp.begin(), cp.end() - 1);
        for (int64_t i = 0; i < m; ++i)
            for (int64_t e = rp[i]; e < rp[i + 1]; ++e) cr[fill[rc[e]]++] = static_cast<int32_t>(i);
    }

    out.piT.assign(m, -1);
    out.piF.assign(n, -1);
    out.blocks.clear();
    out.nnz_edges = E;
    std::vector<uint8_t> aliveT(m, 1), aliveF(n, 1);
    std::vector<int32_t> curT(m), curF(n);   // alive nodes, ascending
    std::iota(curT.begin(), curT.end(), 0);
    std::iota(curF.begin(), curF.end(), 0);
    int64_t loT = 0, loF = 0, hiT = m - 1, hiF = n - 1;
    std::vector<int32_t> degT(m, 0), degF(n, 0);
    std::vector<int32_t> compT(m, -1), compF(n, -1);
    std::vector<int32_t> queue;                 // encoded node: instance i -> i, feature j -> m + j
    queue.reserve(static_cast<size_t>(m + n));
    int64_t iters = 0;

    // per-component member lists (rebuilt every iteration)
    std::vector<int64_t> comp_first;            // start offset in members arrays
    std::vector<int32_t> memT, memF;
    std::vector<int64_t> offT, offF;

    while (true) {
        ++iters;
        const int64_t nT = static_cast<int64_t>(curT.size());
        const int64_t nF = static_cast<int64_t>(curF.size());
        const int64_t mh = hub_count(k, nT), nh = hub_count(k, nF);
        for (int32_t i : curT) {
            int32_t d = 0;
            for (int64_t e = rp[i]; e < rp[i + 1]; ++e) d += aliveF[rc[e]];
            degT[i] = d;
        }
        for (int32_t j : curF) {
            int32_t d = 0;
            for (int64_t e = cp[j]; e < cp[j + 1]; ++e) d += aliveT[cr[e]];
            degF[j] = d;
        }
        auto by_degree = [](const std::vector<int32_t>& deg) {
            return [&deg](int32_t a, int32_t b) {
                return deg[a] != deg[b] ? deg[a] > deg[b] : a < b;
            };
        };
        std::vector<int32_t> hubsT(curT), hubsF(curF);
        std::partial_sort(hubsT.begin(), hubsT.begin() + mh, hubsT.end(), by_degree(degT));
        std::partial_sort(hubsF.begin(), hubsF.begin() + nh, hubsF.end(), by_degree(degF));
        for (int64_t h = 0; h < mh; ++h) {
            out.piT[hubsT[h]] = static_cast<int32_t>(hiT--);
            aliveT[hubsT[h]] = 0;
        }
        for (int64_t h = 0; h < nh; ++h) {
            out.piF[hubsF[h]] = static_cast<int32_t>(hiF--);
            aliveF[hubsF[h]] = 0;
        }

        // breadth-first search over the remaining graph
        int32_t ncomp = 0;
        std::vector<int64_t> size;
        std::vector<int32_t> cntT, cntF;
        memT.clear();
        memF.clear();
        std::vector<std::vector<int32_t>> listsT, listsF;
        auto bfs = [&](int64_t seed) {
            const int32_t c = ncomp++;
            listsT.emplace_back();
            listsF.emplace_back();
            auto& LT = listsT.back();
            auto& LF = listsF.back();
            queue.clear();
            queue.push_back(static_cast<int32_t>(seed));
            if (seed < m) compT[seed] = c; else compF[seed - m] = c;
            for (size_t qh = 0; qh < queue.size(); ++qh) {
                const int64_t v = queue[qh];
                if (v < m) {
                    LT.push_back(static_cast<int32_t>(v));
                    for (int64_t e = rp[v]; e < rp[v + 1]; ++e) {
                        const int32_t j = rc[e];
                        if (aliveF[j] && compF[j] < 0) {
                            compF[j] = c;
                            queue.push_back(static_cast<int32_t>(m + j));
                        }
                    }
                } else {
                    const int64_t j = v - m;
                    LF.push_back(static_cast<int32_t>(j));
                    for (int64_t e = cp[j]; e < cp[j + 1]; ++e) {
                        const int32_t i = cr[e];
                        if (aliveT[i] && compT[i] < 0) {
                            compT[i] = c;
                            queue.push_back(i);
                        }
                    }
                }
            }
            size.push_back(static_cast<int64_t>(LT.size() + LF.size()));
        };
        for (int32_t i : curT)
            if (aliveT[i] && compT[i] < 0) bfs(i);
        for (int32_t j : curF)
            if (aliveF[j] && compF[j] < 0) bfs(m + j);
        if (ncomp == 0) {
            curT.clear();
            curF.clear();
            break;
        }
        int32_t giant = 0;
        for (int32_t c = 1; c < ncomp; ++c)
            if (size[c] > size[giant]) giant = c;
        for (int32_t c = 0; c < ncomp; ++c) {
            auto& LT = listsT[c];
            auto& LF = listsF[c];
            if (c == giant) continue;
            std::sort(LT.begin(), LT.end());
            std::sort(LF.begin(), LF.end());
            out.blocks.push_back({loT, loF, static_cast<int64_t>(LT.size()),
                                  static_cast<int64_t>(LF.size())});
            for (int32_t i : LT) {
                out.piT[i] = static_cast<int32_t>(loT++);
                aliveT[i] = 0;
            }
            for (int32_t j : LF) {
                out.piF[j] = static_cast<int32_t>(loF++);
                aliveF[j] = 0;
            }
        }
        // reset component marks of the giant, which becomes the next graph
        auto& GT = listsT[giant];
        auto& GF = listsF[giant];
        std::sort(GT.begin(), GT.end());
        std::sort(GF.begin(), GF.end());
        for (int32_t i : GT) compT[i] = -1;
        for (int32_t j : GF) compF[j] = -1;
        for (int32_t c = 0; c < ncomp; ++c) {
            if (c == giant) continue;
            for (int32_t i : listsT[c]) compT[i] = -1;
            for (int32_t j : listsF[c]) compF[j] = -1;
        }
        curT.assign(GT.begin(), GT.end());
        curF.assign(GF.begin(), GF.end());
        const int64_t gT = static_cast<int64_t>(curT.size()), gF = static_cast<int64_t>(curF.size());
        if (gT < mh || gF < nh || gT + gF == 0) break;
    }
    if (!curT.empty() || !curF.empty()) {
        out.blocks.push_back({loT, loF, static_cast<int64_t>(curT.size()),
                              static_cast<int64_t>(curF.size())});
        for (int32_t i : curT) out.piT[i] = static_cast<int32_t>(loT++);
        for (int32_t j : curF) out.piF[j] = static_cast<int32_t>(loF++);
    }
    if (loT != hiT + 1 || loF != hiF + 1) {
        set_error("internal: reordering ids do not meet");
        return FASTPI_EINTERNAL;
    }
    out.m1 = loT;
    out.n1 = loF;
    out.m2 = m - loT;
    out.n2 = n - loF;
    out.iterations = iters;
    return FASTPI_OK;
}

}  // namespace fastpi
