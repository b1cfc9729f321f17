"""Plain Python reading of the learned rank allocation's host rules (the learned form of
Eq. 1's rank rule: the alpha rule's total s_b, shared in proportion to the predicted kept
counts), written loop by loop in IEEE double so that the library must agree bit for bit:
sums in index order, no fused multiply-add, ties to the lower index."""
from __future__ import annotations

import math

import numpy as np

N_FEATURES = 16


def inputs(F, mean, std, lo, hi, margin):
    """Standardised features rounded to float32, and the range flags: a row is in range when
    every feature lies within [lo - margin span, hi + margin span], span = max(hi - lo, 1e-12)."""
    F = np.asarray(F, np.float64).reshape(-1, N_FEATURES)
    n = F.shape[0]
    X = np.empty((n, N_FEATURES), np.float32)
    ok = np.zeros(n, bool)
    for i in range(n):
        inside = True
        for j in range(N_FEATURES):
            x = float(F[i, j])
            span = max(float(hi[j]) - float(lo[j]), 1e-12)
            if not (x >= float(lo[j]) - margin * span and x <= float(hi[j]) + margin * span):
                inside = False
            X[i, j] = np.float32((x - float(mean[j])) / float(std[j]))
        ok[i] = inside
    return X, ok


def allocate(f, q, budget):
    """Integer s_i in [0, q_i] with sum min(budget, sum q): the largest scale c with
    sum min(c x_i, q_i) <= budget (x_i = max(clip(f_i) q_i, 1e-9)) by 200 bisection steps,
    floors, then one unit each to the largest fractional parts below their cap."""
    q = [int(v) for v in q]
    n = len(q)
    budget = min(int(budget), sum(q))
    if budget <= 0 or n == 0:
        return np.zeros(n, np.int64)
    x = []
    for fi, qi in zip(f, q):
        v = float(np.float32(fi))
        v = (v if v < 1.0 else 1.0) if v > 0.0 else 0.0
        x.append(max(v * float(qi), 1e-9))
    lo, hi = 0.0, float(max(q)) / min(x) + 1.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        tot = 0.0
        for xi, qi in zip(x, q):
            tot += min(mid * xi, float(qi))
        if tot > float(budget):
            hi = mid
        else:
            lo = mid
    share = [min(lo * xi, float(qi)) for xi, qi in zip(x, q)]
    s = [int(math.floor(v)) for v in share]
    frac = [v - si for v, si in zip(share, s)]
    rest = budget - sum(s)
    for i in sorted(range(n), key=lambda i: (-frac[i], i)):
        if rest == 0:
            break
        if s[i] < q[i]:
            s[i] += 1
            rest -= 1
    return np.asarray(s, np.int64)


def plan_ranks(blocks, alpha_ranks, f_in, ok):
    """The whole allocation given the alpha rule's ranks of every block (a fresh plan's) and
    the network's outputs f_in for the in-range dense blocks (in block order): out-of-range
    blocks keep the alpha rule, in-range ones share the rest of its total."""
    blocks = np.asarray(blocks)
    dense = np.flatnonzero((blocks[:, 2] > 0) & (blocks[:, 3] > 0))
    q = np.minimum(blocks[dense, 2], blocks[dense, 3])
    a = np.asarray(alpha_ranks, np.int64)[dense]
    out = np.zeros(len(blocks), np.int64)
    s = a.copy()
    if ok.any():
        s[ok] = allocate(f_in, q[ok], int(a.sum()) - int(a[~ok].sum()))
    out[dense] = s
    return out
