"""GPU parity of Application 1's evaluation loop through the C ABI: the sparse-label apply
Z = V Sigma^+ U^T Y against the oracle (and the dense-label apply), and the top-k hit counts
of held-out rows (the P@k measure of the accuracy experiment, Section 4).

The ranking is an integer decision taken on floating-point scores, so both sides take it on
scores of the same precision and order: the oracle scores the GPU's own Z entry by entry
(one rounded multiply and add per stored entry, CSR order) and the hit counts must then be
identical. Against the oracle's own Z, P@k may differ only on rows whose k-th and (k+1)-th
scores are within the Z tolerance of each other."""
import sys

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from parity import MIXED_LS_RTOL, compare_apply, compare_svd, to_np
from synth import make_labelled_problem

pytestmark = pytest.mark.gpu
KS = [1, 3, 5]


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


class _Prob:
    """Training part in the shape the parity helpers read (dense Y)."""

    def __init__(self, part, L):
        self.m, self.n = part.m, part.n
        self.indptr, self.indices, self.data = part.indptr, part.indices, part.data
        self.Y = oracle.labels_dense(part.m, L, part.y_indptr, part.y_indices)


@pytest.fixture(scope="module")
def env():
    import torch

    import paper_2011_04235_amd as fp
    fp.load()
    return torch, fp


def dev_t(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(torch.device("cuda", 0))


def gpu_hits(torch, h, part, Z, ks):
    out = h.topk_hits(dev_t(torch, part.indptr), dev_t(torch, part.indices), dev_t(torch, part.data), Z,
                      dev_t(torch, part.y_indptr), dev_t(torch, part.y_indices), ks)
    torch.cuda.synchronize()
    return to_np(out).astype(np.int64)


def ambiguous_rows(part, Z, ks, tol):
    """Rows whose k-th and (k+1)-th largest scores are within tol (per k)."""
    out = np.zeros((part.m, len(ks)), dtype=bool)
    for i in range(part.m):
        s = np.sort(oracle.row_scores(part.indptr, part.indices, part.data, Z, i))[::-1]
        for t, k in enumerate(ks):
            if k < s.size:
                out[i, t] = s[k - 1] - s[k] <= tol
    return out


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_labelled_loop_matches_oracle(env, precision):
    torch, fp = env
    lp = make_labelled_problem("c1")
    tr, te, L = lp.train, lp.test, lp.L
    say(f"labelled 2000x500 (train {tr.m}, test {te.m}, L={L}, nnz(Y)={tr.y_nnz}) {precision}")
    plan = fp.Plan(tr.m, tr.n, tr.indptr, tr.indices, tr.data, alpha=0.3, k=0.01)
    h = fp.Handle(0, precision=precision)
    h.upload_plan(plan)
    U, S, V = h.svd(dev_t(torch, tr.indptr), dev_t(torch, tr.indices), dev_t(torch, tr.data))
    labels = fp.Labels(h, tr.m, L, tr.y_indptr, tr.y_indices)
    assert labels.nnz == tr.y_nnz
    Zs = h.apply_sparse(U, S, V, labels)
    prob = _Prob(tr, L)
    Zd = h.apply(U, S, V, dev_t(torch, prob.Y))
    h.sync()
    Zs_h, Zd_h = to_np(Zs), to_np(Zd)
    dz = float(np.linalg.norm(Zs_h - Zd_h) / np.linalg.norm(Zd_h))
    say(f"  sparse vs dense apply rel diff {dz:.2e}")
    assert dz <= (1e-13 if precision == "fp64" else 1e-5)
    ores = oracle.fastpi_svd(tr.m, tr.n, tr.indptr, tr.indices, tr.data, 0.3, 0.01)
    if precision == "fp64":
        ok, info = compare_svd(prob, to_np(U), to_np(S), to_np(V), ores)
        assert ok, info
    Zo = oracle.pinv_apply_sparse(ores.U, ores.sigma, ores.V, tr.m, tr.n, L, tr.y_indptr, tr.y_indices)
    ok, zinfo = compare_apply(prob, Zs_h, ores)
    say(f"  {zinfo}")
    assert (ok if precision == "fp64" else zinfo["ls_rel"] <= MIXED_LS_RTOL), zinfo
    # hit counts: identical to the oracle scoring the GPU's Z
    hg = gpu_hits(torch, h, te, Zs, KS)
    ho_same = oracle.topk_hits(te.indptr, te.indices, te.data, Zs_h, te.y_indptr, te.y_indices, KS)
    assert np.array_equal(hg, ho_same)
    # against the oracle's own Z: P@k equal up to near-tied rows
    ho = oracle.topk_hits(te.indptr, te.indices, te.data, Zo, te.y_indptr, te.y_indices, KS)
    tol = (1e-6 if precision == "fp64" else 1e-2) * float(np.abs(Zo).max()) * float(np.abs(te.data).max()) * 8
    amb = ambiguous_rows(te, Zo, KS, tol)
    pg, po = oracle.p_at_k(hg, KS), oracle.p_at_k(ho, KS)
    say(f"  P@{KS} gpu {np.round(pg, 4).tolist()} oracle {np.round(po, 4).tolist()} "
        f"near-tied rows {amb.sum(axis=0).tolist()}")
    diff_rows = (hg != ho)
    assert np.all(~diff_rows | amb), np.argwhere(diff_rows & ~amb)[:5]
    density = tr.y_nnz / (tr.m * L)
    assert pg[0] > 5 * density


def test_hits_equal_oracle_at_the_scoring_workload(env):
    """20000 x 2000 features (2000 test rows, 200 labels), FP64: the apply against the dense
    apply, and the hit counts exactly equal to the oracle scoring the same Z."""
    torch, fp = env
    lp = make_labelled_problem("c2")
    tr, te, L = lp.train, lp.test, lp.L
    say(f"labelled 20000x2000 (train {tr.m}, test {te.m}, L={L}, nnz(Y)={tr.y_nnz})")
    plan = fp.Plan(tr.m, tr.n, tr.indptr, tr.indices, tr.data, alpha=0.2, k=0.01)
    h = fp.Handle(0)
    h.upload_plan(plan)
    U, S, V = h.svd(dev_t(torch, tr.indptr), dev_t(torch, tr.indices), dev_t(torch, tr.data))
    labels = fp.Labels(h, tr.m, L, tr.y_indptr, tr.y_indices)
    Zs = h.apply_sparse(U, S, V, labels)
    Zd = h.apply(U, S, V, dev_t(torch, oracle.labels_dense(tr.m, L, tr.y_indptr, tr.y_indices)))
    h.sync()
    dz = float(torch.linalg.norm(Zs - Zd) / torch.linalg.norm(Zd))
    say(f"  sparse vs dense apply rel diff {dz:.2e}")
    assert dz <= 1e-12
    hg = gpu_hits(torch, h, te, Zs, [1, 3, 5, 10])
    ho = oracle.topk_hits(te.indptr, te.indices, te.data, to_np(Zs), te.y_indptr, te.y_indices, [1, 3, 5, 10])
    say(f"  P@1,3,5,10 {np.round(oracle.p_at_k(hg, [1, 3, 5, 10]), 4).tolist()}")
    assert np.array_equal(hg, ho)


@pytest.mark.parametrize("L,rows", [(3, 150), (50, 150), (64, 150), (7680, 150), (9000, 4000)])
def test_topk_ties_and_label_counts(env, L, rows):
    """Integer scores (exact, heavily tied) so the tie rule decides; L = 3 has fewer labels
    than the largest k, 64 is one full label slice, 50 and 7680 end in a partial one, and
    4000 rows of 9000 labels take two chunks of the score buffer (32M doubles). Includes rows
    without entries (all scores zero) and without positives."""
    torch, fp = env
    rng = np.random.default_rng(L)
    n = 40
    A = sp.random(rows, n, density=0.08, random_state=L, format="csr")
    A.data = rng.integers(1, 4, size=A.nnz).astype(np.float64)
    A.sort_indices()
    Z = rng.integers(-2, 3, size=(n, L)).astype(np.float64)
    Y = sp.random(rows, L, density=min(0.5, 6.0 / L), random_state=L + 1, format="csr")
    Y.sort_indices()
    ks = [1, 2, 5, 17, 64]
    say(f"ties: {rows} rows, n={n}, L={L}, ks={ks}")
    h = fp.Handle(0)
    part = type("P", (), {})()
    part.indptr, part.indices, part.data = A.indptr.astype(np.int64), A.indices.astype(np.int32), A.data
    part.y_indptr, part.y_indices = Y.indptr.astype(np.int64), Y.indices.astype(np.int32)
    hg = gpu_hits(torch, h, part, dev_t(torch, Z), ks)
    ho = oracle.topk_hits(part.indptr, part.indices, part.data, Z, part.y_indptr, part.y_indices, ks)
    assert np.array_equal(hg, ho)
    assert np.any(np.diff(A.indptr) == 0)


def test_topk_rejects_bad_arguments_and_marks_bad_rows(env):
    torch, fp = env
    h = fp.Handle(0)
    Z = dev_t(torch, np.arange(12.0).reshape(3, 4))
    ip = dev_t(torch, np.array([0, 1, 2], np.int64))
    col = dev_t(torch, np.array([2, 7], np.int32))     # row 1 names column 7 of a 3-row Z
    val = dev_t(torch, np.array([1.0, 1.0]))
    yp = dev_t(torch, np.array([0, 1, 1], np.int64))
    yc = dev_t(torch, np.array([3], np.int32))
    hits = h.topk_hits(ip, col, val, Z, yp, yc, [1, 2])
    torch.cuda.synchronize()
    assert to_np(hits).tolist() == [[1, 1], [-1, -1]]
    for bad in ([0], [65], list(range(1, 18))):
        with pytest.raises(fp.FastPIError):
            h.topk_hits(ip, col, val, Z, yp, yc, bad)


def test_labels_edge_cases(env):
    """Labels without positives give zero columns of Z; an empty label matrix gives Z = 0;
    malformed patterns are rejected on the host."""
    torch, fp = env
    lp = make_labelled_problem("c1")
    tr, L = lp.train, lp.L
    plan = fp.Plan(tr.m, tr.n, tr.indptr, tr.indices, tr.data, alpha=0.3, k=0.01)
    h = fp.Handle(0)
    h.upload_plan(plan)
    U, S, V = h.svd(dev_t(torch, tr.indptr), dev_t(torch, tr.indices), dev_t(torch, tr.data))
    # keep only the positives of labels 0..9: the other columns must come out zero
    Ydense = oracle.labels_dense(tr.m, L, tr.y_indptr, tr.y_indices)
    Ydense[:, 10:] = 0.0
    Ys = sp.csr_matrix(Ydense)
    yp, yc = Ys.indptr.astype(np.int64), Ys.indices.astype(np.int32)
    Z = to_np(h.apply_sparse(U, S, V, fp.Labels(h, tr.m, L, yp, yc)))
    h.sync()
    assert np.all(Z[:, 10:] == 0.0) and np.any(Z[:, :10] != 0.0)
    Zd = to_np(h.apply(U, S, V, dev_t(torch, Ydense)))
    h.sync()
    assert np.linalg.norm(Z - Zd) <= 1e-13 * np.linalg.norm(Zd)
    Z0 = to_np(h.apply_sparse(U, S, V, fp.Labels(h, tr.m, L, np.zeros(tr.m + 1, np.int64), np.zeros(0, np.int32))))
    h.sync()
    assert np.all(Z0 == 0.0)
    with pytest.raises(fp.FastPIError):
        fp.Labels(h, 3, 4, np.array([0, 2, 1, 3]), np.array([0, 1, 2], np.int32))
    with pytest.raises(fp.FastPIError):
        fp.Labels(h, 2, 4, np.array([0, 1, 2]), np.array([0, 4], np.int32))
    with pytest.raises(fp.FastPIError):
        fp.Labels(h, 2, 4, np.array([0, 1, 2]), np.array([0, 1], np.int32), np.array([1.0, np.nan]))


@pytest.mark.parametrize("m,n,r,L,density,weighted,seed", [
    (3000, 400, 13, 2500, 0.004, True, 1),     # two label groups, ragged column block, weights
    (5000, 300, 200, 37, 0.05, False, 2),      # few labels, many positives per label
    (700, 200, 64, 300, 0.01, False, 3),       # fewer labelled rows than one row block
])
def test_label_spmm_against_oracle(env, m, n, r, L, density, weighted, seed):
    """The sparse-label apply on random factors against the oracle's Z = V Sigma^+ U^T Y
    (dense Y), element by element, for the row-blocked label SpMM's edge shapes: label counts
    above one workgroup's 2048, r not a multiple of its 8 columns, a ragged last row block,
    unlabelled rows, weighted labels; two calls give identical bits (fixed order)."""
    torch, fp = env
    say(f"label spmm m={m} n={n} r={r} L={L} density={density} weighted={weighted}")
    rng = np.random.default_rng(seed)
    U = np.linalg.qr(rng.standard_normal((m, r)))[0]
    V = np.linalg.qr(rng.standard_normal((n, r)))[0]
    S = np.sort(rng.uniform(0.5, 3.0, r))[::-1].copy()
    Y = sp.random(m, L, density=density, format="csr", random_state=seed)
    Y.data = rng.uniform(0.5, 2.0, Y.nnz) if weighted else np.ones(Y.nnz)
    Y.sort_indices()
    Y[: m // 10] = 0.0                                   # a band of unlabelled rows
    Y.eliminate_zeros()
    yp, yc = Y.indptr.astype(np.int64), Y.indices.astype(np.int32)
    yv = Y.data.astype(np.float64) if weighted else None
    h = fp.Handle(0)
    labels = fp.Labels(h, m, L, yp, yc, yv)
    Ud, Sd, Vd = dev_t(torch, U), dev_t(torch, S), dev_t(torch, V)
    Z1 = to_np(h.apply_sparse(Ud, Sd, Vd, labels))
    Z2 = to_np(h.apply_sparse(Ud, Sd, Vd, labels))
    h.sync()
    Zo = oracle.pinv_apply_sparse(U, S, V, m, n, L, yp, yc, yv)
    err = np.max(np.abs(Z1 - Zo)) / max(np.max(np.abs(Zo)), 1e-300)
    say(f"  max err {err:.2e}")
    assert err <= 1e-12
    assert np.array_equal(Z1.view(np.uint64), Z2.view(np.uint64))


def test_label_spmm_segmented_fallback_against_oracle(env):
    """A label matrix with a row of more than 4096 positives keeps the segmented label SpMM
    (no row block can hold that row); Z against the oracle element by element, repeatable."""
    torch, fp = env
    m, n, r, L, seed = 900, 150, 24, 6000, 5
    say(f"label spmm segmented form m={m} L={L} (one row with 5000 positives)")
    rng = np.random.default_rng(seed)
    U = np.linalg.qr(rng.standard_normal((m, r)))[0]
    V = np.linalg.qr(rng.standard_normal((n, r)))[0]
    S = np.sort(rng.uniform(0.5, 3.0, r))[::-1].copy()
    Y = sp.random(m, L, density=0.002, format="lil", random_state=seed)
    Y[7, :5000] = 1.0
    Y = Y.tocsr()
    Y.data[:] = 1.0
    Y.sort_indices()
    yp, yc = Y.indptr.astype(np.int64), Y.indices.astype(np.int32)
    assert np.max(np.diff(yp)) > 4096
    h = fp.Handle(0)
    labels = fp.Labels(h, m, L, yp, yc)
    Ud, Sd, Vd = dev_t(torch, U), dev_t(torch, S), dev_t(torch, V)
    Z1 = to_np(h.apply_sparse(Ud, Sd, Vd, labels))
    Z2 = to_np(h.apply_sparse(Ud, Sd, Vd, labels))
    h.sync()
    Zo = oracle.pinv_apply_sparse(U, S, V, m, n, L, yp, yc)
    err = np.max(np.abs(Z1 - Zo)) / max(np.max(np.abs(Zo)), 1e-300)
    say(f"  max err {err:.2e}")
    assert err <= 1e-12
    assert np.array_equal(Z1.view(np.uint64), Z2.view(np.uint64))
