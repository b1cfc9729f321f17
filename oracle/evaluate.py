"""Oracle of Application 1's evaluation loop: the pseudoinverse applied to a sparse label
matrix, and top-k precision on held-out rows (the accuracy experiment of Section 4).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the benchmark's
CPU-baseline leg, never by the product path.

Readings where the paper is silent:
- rank_k breaks ties between equal scores towards the lower label index;
- the P@k of a test set is the mean of the per-row values over every test row, rows
  without a positive label included (they contribute zero);
- the score of a test row x is accumulated over x's stored entries in CSR order, one
  rounded multiply and one rounded add per entry (no fused multiply-add), so that the
  integer decision rank_k is taken on scores of a fixed, stated precision and order.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .fastpi import pinv_apply


def labels_dense(m: int, L: int, indptr, indices, data=None) -> np.ndarray:
    """The m x L label matrix Y of a CSR pattern (values 1 where data is None)."""
    vals = np.ones(len(indices)) if data is None else np.asarray(data, np.float64)
    return sp.csr_matrix((vals, np.asarray(indices), np.asarray(indptr)), shape=(m, L)).toarray()


def pinv_apply_sparse(U, sigma, V, m, n, L, y_indptr, y_indices, y_data=None) -> np.ndarray:
    """Z = V Sigma^+ U^T Y for Y given as a CSR pattern (Application 1, Problem 1).
    The definition does not depend on Y's storage: Y is formed densely."""
    return pinv_apply(U, sigma, V, labels_dense(m, L, y_indptr, y_indices, y_data), m, n)


def row_scores(indptr, indices, data, Z, row: int) -> np.ndarray:
    """yhat = Z^T x for test row `row` of a CSR matrix (Application 1's score vector),
    accumulated entry by entry in storage order."""
    acc = np.zeros(Z.shape[1], dtype=np.float64)
    for e in range(int(indptr[row]), int(indptr[row + 1])):
        prod = np.float64(data[e]) * Z[int(indices[e])]   # rounded product
        acc = acc + prod                                  # rounded sum
    return acc


def rank_k(yhat: np.ndarray, k: int) -> np.ndarray:
    """The k labels with the largest scores, in descending score order; equal scores go
    to the lower label first."""
    order = np.argsort(-np.asarray(yhat, np.float64), kind="stable")
    return order[:k]


def precision_at_k(yhat: np.ndarray, positives, k: int) -> float:
    """P@k = (1/k) * (number of the k top-ranked labels that are positive)."""
    pos = set(int(x) for x in positives)
    return sum(1 for lab in rank_k(yhat, k) if int(lab) in pos) / float(k)


def topk_hits(indptr, indices, data, Z, y_indptr, y_indices, ks) -> np.ndarray:
    """hits[row, t] = number of positives among the ks[t] top-ranked labels of each row of
    a CSR test matrix; P@k of the set is hits[:, t].sum() / (rows * ks[t])."""
    rows = len(indptr) - 1
    ks = [int(k) for k in ks]
    out = np.zeros((rows, len(ks)), dtype=np.int64)
    kmax = max(ks) if ks else 0
    for i in range(rows):
        top = rank_k(row_scores(indptr, indices, data, Z, i), kmax)
        pos = set(int(x) for x in y_indices[int(y_indptr[i]):int(y_indptr[i + 1])])
        hit = np.cumsum([1 if int(lab) in pos else 0 for lab in top])
        for t, k in enumerate(ks):
            out[i, t] = int(hit[min(k, len(top)) - 1]) if k > 0 and len(top) else 0
    return out


def p_at_k(hits: np.ndarray, ks) -> np.ndarray:
    """Test-set P@k for every k from a hits table (mean over rows of the per-row value)."""
    rows = hits.shape[0]
    return np.array([hits[:, t].sum() / float(rows * k) if rows else 0.0
                     for t, k in enumerate(ks)])
