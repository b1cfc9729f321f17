"""Pins of the evaluation oracle (Application 1's regression and the P@k measure of the
accuracy experiment, Section 4) against a hand-worked example, a count-based brute force of
rank_k, closed forms of special scorers and the least-squares solution it must reach."""
import json
import os

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from synth import make_labelled_problem, small_config

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "p_at_k_example.json")


def test_worked_example_single_row():
    ex = json.load(open(GOLDEN))["single_row"]
    s = np.array(ex["scores"])
    assert oracle.rank_k(s, 6).tolist() == ex["rank_6"]
    for k, want in ex["p_at_k"].items():
        assert oracle.precision_at_k(s, ex["positives"], int(k)) == pytest.approx(want, abs=0)


def test_worked_example_test_set():
    ex = json.load(open(GOLDEN))["test_set"]
    Z = np.array(ex["Z"], dtype=np.float64)
    ip, ix, dv = np.array(ex["indptr"]), np.array(ex["indices"]), np.array(ex["data"])
    for i, want in enumerate(ex["scores"]):
        assert oracle.row_scores(ip, ix, dv, Z, i).tolist() == want
    hits = oracle.topk_hits(ip, ix, dv, Z, np.array(ex["y_indptr"]), np.array(ex["y_indices"]), ex["ks"])
    assert hits.tolist() == ex["hits"]
    assert oracle.p_at_k(hits, ex["ks"]) == pytest.approx(ex["p_at_k"], abs=1e-15)


@pytest.mark.parametrize("seed", range(6))
def test_rank_k_matches_count_definition(seed):
    """l is at position p of rank_k iff exactly p labels beat it (a higher score, or an
    equal score at a lower index); brute force over heavy ties."""
    rng = np.random.default_rng(seed)
    L = int(rng.integers(1, 40))
    s = rng.integers(-3, 4, size=L).astype(np.float64)
    beats = [sum(1 for j in range(L) if s[j] > s[l] or (s[j] == s[l] and j < l)) for l in range(L)]
    for k in range(0, L + 2):
        top = oracle.rank_k(s, k)
        want = sorted((l for l in range(L) if beats[l] < k), key=lambda l: beats[l])
        assert top.tolist() == want


def test_special_scorers():
    rng = np.random.default_rng(3)
    L = 30
    y = (rng.random(L) < 0.2).astype(np.float64)
    pos = np.flatnonzero(y)
    for k in (1, 3, 5, L):
        # a perfect scorer ranks every positive first
        assert oracle.precision_at_k(y + 0.01 * rng.random(L), pos, k) == min(len(pos), k) / k
        # the worst scorer ranks them last
        worst = max(0, k - (L - len(pos))) / k
        assert oracle.precision_at_k(-y, pos, k) == pytest.approx(worst)
    # P@L is the fraction of positive labels, whatever the scores
    assert oracle.precision_at_k(rng.standard_normal(L), pos, L) == pytest.approx(len(pos) / L)


def test_row_scores_are_exact_on_integers_and_match_the_product():
    rng = np.random.default_rng(5)
    A = sp.random(20, 15, density=0.3, random_state=5, format="csr")
    A.data = rng.integers(-8, 9, size=A.nnz).astype(np.float64)
    Z = rng.integers(-8, 9, size=(15, 7)).astype(np.float64)
    want = (A @ Z)
    for i in range(20):
        assert np.array_equal(oracle.row_scores(A.indptr, A.indices, A.data, Z, i), want[i])
    A.data = rng.standard_normal(A.nnz)
    Zf = rng.standard_normal((15, 7))
    for i in range(20):
        np.testing.assert_allclose(oracle.row_scores(A.indptr, A.indices, A.data, Zf, i),
                                   (A @ Zf)[i], rtol=1e-13, atol=1e-13)


def test_sparse_apply_at_full_rank_is_least_squares():
    """alpha = 1 on a full-column-rank A: Z = A^+ Y is the least-squares solution."""
    lp = make_labelled_problem(small_config(300, 40, 0.2, gamma=2.2, L=9, seed=21, k=0.05))
    tr = lp.train
    res = oracle.fastpi_svd(tr.m, tr.n, tr.indptr, tr.indices, tr.data, 1.0, 0.05)
    Z = oracle.pinv_apply_sparse(res.U, res.sigma, res.V, tr.m, tr.n, lp.L, tr.y_indptr, tr.y_indices)
    A = sp.csr_matrix((tr.data, tr.indices, tr.indptr), shape=(tr.m, tr.n)).toarray()
    assert np.linalg.matrix_rank(A) == tr.n
    Y = oracle.labels_dense(tr.m, lp.L, tr.y_indptr, tr.y_indices)
    Zls = np.linalg.lstsq(A, Y, rcond=None)[0]
    np.testing.assert_allclose(Z, Zls, rtol=0, atol=1e-9 * max(1.0, np.abs(Zls).max()))


def test_labelled_recipe_split_and_signal():
    """The 90/10 split partitions the rows; the planted labels are predictable (P@1 far
    above the label density), so P@k measures the regression, not noise."""
    lp = make_labelled_problem("c1")
    tr, te = lp.train, lp.test
    assert te.m == 200 and tr.m == 1800
    assert np.intersect1d(tr.rows, te.rows).size == 0
    assert np.union1d(tr.rows, te.rows).size == 2000
    for part in (tr, te):
        assert np.all(np.diff(part.y_indptr) >= 0)
        for i in range(part.m):
            row = part.y_indices[part.y_indptr[i]:part.y_indptr[i + 1]]
            assert np.all(np.diff(row) > 0) and (row.size == 0 or (row[0] >= 0 and row[-1] < lp.L))
    density = tr.y_nnz / (tr.m * lp.L)
    assert density < 0.05
    res = oracle.fastpi_svd(tr.m, tr.n, tr.indptr, tr.indices, tr.data, 0.3, 0.01)
    Z = oracle.pinv_apply_sparse(res.U, res.sigma, res.V, tr.m, tr.n, lp.L, tr.y_indptr, tr.y_indices)
    p = oracle.p_at_k(oracle.topk_hits(te.indptr, te.indices, te.data, Z, te.y_indptr, te.y_indices, [1, 3]), [1, 3])
    assert p[0] > 5 * density and p[1] > 3 * density
