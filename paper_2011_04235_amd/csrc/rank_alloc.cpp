// Host arithmetic of the learned rank allocation (the learned form of Eq. 1's rank rule
// s_i = ceil(alpha n_i)): the network's inputs (standardised block features and the range
// test that decides which blocks it may speak for) and the budgeted integer allocation that
// turns its kept fractions into ranks with the alpha rule's total.
//
// Every sum runs in index order and no multiply-add is contracted, so the results are the
// same on every build and match a plain sequential reading of the rules in any language.
#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

#include "host_internal.h"

#pragma clang fp contract(off)

namespace fastpi {

void rank_inputs(int64_t n, const double* feats, const fastpi_rank_model& m, float* X, int32_t* ok) {
    for (int64_t i = 0; i < n; ++i) {
        const double* x = feats + i * kRankFeatures;
        bool in = true;
        for (int j = 0; j < kRankFeatures; ++j) {
            const double span = std::max(m.hi[j] - m.lo[j], 1e-12);
            if (!(x[j] >= m.lo[j] - m.margin * span && x[j] <= m.hi[j] + m.margin * span)) in = false;
            if (X) X[i * kRankFeatures + j] = static_cast<float>((x[j] - m.mean[j]) / m.std[j]);
        }
        if (ok) ok[i] = in ? 1 : 0;
    }
}

void rank_allocate(int64_t n, const float* f, const int64_t* q, int64_t budget, int64_t* s) {
    int64_t qsum = 0, qmax = 0;
    for (int64_t i = 0; i < n; ++i) {
        qsum += q[i];
        qmax = std::max(qmax, q[i]);
    }
    budget = std::min(budget, qsum);
    if (budget <= 0 || n == 0) {
        std::fill(s, s + n, 0);
        return;
    }
    // x_i: the predicted kept count f_i q_i (f clipped to [0, 1]), kept above zero so every
    // block can take a share
    std::vector<double> x(n);
    double xmin = 0;
    for (int64_t i = 0; i < n; ++i) {
        double fi = static_cast<double>(f[i]);
        fi = fi > 0.0 ? (fi < 1.0 ? fi : 1.0) : 0.0;   // NaN counts as 0
        x[i] = std::max(fi * static_cast<double>(q[i]), 1e-9);
        xmin = i == 0 ? x[i] : std::min(xmin, x[i]);
    }
    // largest scale c with sum_i min(c x_i, q_i) <= budget (the sum is monotone in c)
    double lo = 0.0, hi = static_cast<double>(qmax) / xmin + 1.0;
    for (int it = 0; it < 200; ++it) {
        const double mid = 0.5 * (lo + hi);
        double tot = 0.0;
        for (int64_t i = 0; i < n; ++i) tot += std::min(mid * x[i], static_cast<double>(q[i]));
        if (tot > static_cast<double>(budget)) hi = mid;
        else lo = mid;
    }
    std::vector<double> frac(n);
    int64_t used = 0;
    for (int64_t i = 0; i < n; ++i) {
        const double share = std::min(lo * x[i], static_cast<double>(q[i]));
        s[i] = static_cast<int64_t>(std::floor(share));
        frac[i] = share - static_cast<double>(s[i]);
        used += s[i];
    }
    // the units left go to the largest fractional parts (ties to the lower index)
    int64_t rest = budget - used;
    if (rest > 0) {
        std::vector<int64_t> order(n);
        std::iota(order.begin(), order.end(), 0);
        std::stable_sort(order.begin(), order.end(), [&](int64_t a, int64_t b) { return frac[a] > frac[b]; });
        for (int64_t i : order) {
            if (rest == 0) break;
            if (s[i] < q[i]) {
                ++s[i];
                --rest;
            }
        }
    }
}

}  // namespace fastpi
