"""Oracle for the learned per-block rank predictor (FP64, CPU).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Eq. 1 keeps s_i = ceil(alpha n_1i) directions of every diagonal block. For a block-diagonal
matrix the best rank-s_b approximation (Eckart-Young) instead keeps the s_b largest singular
values over all blocks together. With the total held at the alpha rule's s_b, the label of
block i is s_i* = #{sigma_ij >= tau}, tau being the s_b-th largest singular value over all
blocks; the network predicts the kept fraction f_i = s_i* / min(m_i, n_i) from 16 cheap
features of the block. This module computes those features and labels from a dense block
and its spectrum, and the FP64 forward pass, backward pass and Adam step of the 16-64-64-1
network (ReLU, ReLU, sigmoid; mean squared error on f).
"""
from __future__ import annotations

import math

import numpy as np

N_FEATURES = 16
H1 = 64
H2 = 64
N_PARAMS = H1 * N_FEATURES + H1 + H2 * H1 + H2 + H2 + 1   # 5313

FEATURE_NAMES = [
    "log rows", "log cols", "log nnz", "density", "log ||A_i||_F^2", "log max col norm^2",
    "log min col norm^2", "mean log col norm^2", "std log col norm^2", "log max row norm^2",
    "stable-rank proxy ||A_i||_F^2 / max col norm^2", "energy share of the block in A11",
    "alpha", "cols / n1", "log(1 + hub edges)", "block position / number of blocks",
]


def block_features(Ai, alpha, n1, a11_energy, hub_edges, position, nblocks):
    """The 16 features of one dense diagonal block Ai (rows x cols, rows, cols >= 1)."""
    Ai = np.asarray(Ai, dtype=np.float64)
    m, n = Ai.shape
    nnz = int(np.count_nonzero(Ai))
    fro2 = float(np.sum(Ai * Ai))
    col2 = np.sum(Ai * Ai, axis=0)
    row2 = np.sum(Ai * Ai, axis=1)
    tiny = 1e-300
    lc = np.log(np.maximum(col2, tiny))
    return np.array([
        math.log(m), math.log(n), math.log(max(nnz, 1)), nnz / (m * n),
        math.log(max(fro2, tiny)), float(lc.max()), float(lc.min()), float(lc.mean()),
        float(lc.std()), math.log(max(float(row2.max()), tiny)),
        fro2 / max(float(col2.max()), tiny), fro2 / max(a11_energy, tiny),
        alpha, n / max(n1, 1), math.log1p(hub_edges), position / max(nblocks, 1),
    ], dtype=np.float64)


def eckart_young_ranks(spectra, budget):
    """s_i* = #{sigma_ij >= tau}, tau = the budget-th largest value over all spectra
    (ties at tau are all kept, so the sum may exceed the budget by the tie count)."""
    allv = np.concatenate([np.asarray(s, float) for s in spectra]) if spectra else np.zeros(0)
    if budget <= 0 or allv.size == 0:
        return np.zeros(len(spectra), dtype=np.int64)
    budget = min(budget, allv.size)
    tau = np.sort(allv)[::-1][budget - 1]
    return np.array([int(np.sum(np.asarray(s) >= tau)) for s in spectra], dtype=np.int64)


def truncation_error2(spectra, ranks):
    """Squared Frobenius error of keeping ranks[i] leading values of every spectrum."""
    return float(sum(np.sum(np.asarray(s)[int(k):] ** 2) for s, k in zip(spectra, ranks)))


# ------------------------------------------------------------------ network ------------
def unpack(theta):
    theta = np.asarray(theta, dtype=np.float64)
    o = 0
    W1 = theta[o:o + H1 * N_FEATURES].reshape(H1, N_FEATURES); o += H1 * N_FEATURES
    b1 = theta[o:o + H1]; o += H1
    W2 = theta[o:o + H2 * H1].reshape(H2, H1); o += H2 * H1
    b2 = theta[o:o + H2]; o += H2
    W3 = theta[o:o + H2]; o += H2
    b3 = theta[o]
    return W1, b1, W2, b2, W3, b3


def init_params(seed):
    """Deterministic initialisation: U(-1/sqrt(fan_in), 1/sqrt(fan_in)) from a PCG64 stream,
    layer by layer (weights then biases)."""
    rng = np.random.default_rng(seed)
    parts = []
    for fan_in, shape in ((N_FEATURES, (H1, N_FEATURES)), (N_FEATURES, (H1,)),
                          (H1, (H2, H1)), (H1, (H2,)), (H2, (H2,)), (H2, (1,))):
        lim = 1.0 / math.sqrt(fan_in)
        parts.append(rng.uniform(-lim, lim, size=shape).ravel())
    return np.concatenate(parts)


def forward(theta, X):
    """f = sigmoid(W3 relu(W2 relu(W1 x + b1) + b2) + b3) for every row x of X."""
    W1, b1, W2, b2, W3, b3 = unpack(theta)
    z1 = X @ W1.T + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2.T + b2
    h2 = np.maximum(z2, 0.0)
    z3 = h2 @ W3 + b3
    f = 1.0 / (1.0 + np.exp(-z3))
    return f, (z1, h1, z2, h2, z3)


def loss(theta, X, y):
    f, _ = forward(theta, X)
    return float(np.mean((f - y) ** 2))


def gradient(theta, X, y):
    """Analytic gradient of the mean squared error, in the packed parameter order."""
    W1, b1, W2, b2, W3, b3 = unpack(theta)
    N = X.shape[0]
    f, (z1, h1, z2, h2, z3) = forward(theta, X)
    dz3 = (2.0 / N) * (f - y) * f * (1.0 - f)          # N
    gW3 = dz3 @ h2
    gb3 = np.sum(dz3)
    dh2 = np.outer(dz3, W3)
    dz2 = dh2 * (z2 > 0)
    gW2 = dz2.T @ h1
    gb2 = dz2.sum(axis=0)
    dh1 = dz2 @ W2
    dz1 = dh1 * (z1 > 0)
    gW1 = dz1.T @ X
    gb1 = dz1.sum(axis=0)
    return np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3, [gb3]])


def adam_step(theta, g, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba), step counted from 1; returns new (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def problem_blocks(m, n, indptr, indices, data, alpha, k=0.01):
    """Features, spectra and alpha-rule ranks of every dense diagonal block of one matrix,
    in block order (oracle reordering and LAPACK spectra)."""
    import scipy.sparse as sp

    from .fastpi import split_blocks, target_rank
    from .reorder import reorder
    A = sp.csr_matrix((np.asarray(data, float), np.asarray(indices), np.asarray(indptr)),
                      shape=(m, n))
    A.eliminate_zeros()
    A.sort_indices()
    R = reorder(m, n, A.indptr, A.indices, k)
    S = split_blocks(m, n, A.indptr, A.indices, A.data, R)
    a11 = sum(float(np.sum(b * b)) for b in S.block_dense)
    Ap = S.A_perm
    tr = np.diff(S.T.indptr)                          # hub-column entries per (new) row
    a21c = np.diff(S.A21.tocsc().indptr) if S.n1 else np.zeros(0, np.int64)
    feats, spectra, alpha_ranks, shapes = [], [], [], []
    nb = len(S.blocks)
    for Ai, b in zip(S.block_dense, S.block_index):
        r0, c0, mi, ni = (int(x) for x in S.blocks[b])
        hub = int(tr[r0:r0 + mi].sum()) + int(a21c[c0:c0 + ni].sum())
        feats.append(block_features(Ai, alpha, S.n1, a11, hub, b, nb))
        spectra.append(np.linalg.svd(Ai, compute_uv=False))
        alpha_ranks.append(min(target_rank(alpha, ni), mi, ni))
        shapes.append((mi, ni))
    del Ap
    return (np.array(feats).reshape(-1, N_FEATURES), spectra, np.array(alpha_ranks, np.int64),
            np.array(shapes, np.int64).reshape(-1, 2))
