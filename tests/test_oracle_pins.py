"""Pins of the CPU oracle to facts the paper and the mathematics fix.

Every check here compares the oracle with something other than itself: a
hand-derived toy example, an independently written breadth-first reordering,
closed forms, the exactness of the method at alpha = 1 (Problem 1), the
Moore-Penrose conditions, Eckart-Young identities computed from an eigenvalue
routine (not the SVD the oracle calls), and dense reconstructions.
"""
import json
import math
import os
from collections import deque

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

import oracle
from oracle import fastpi as ofp
from synth import make_problem, small_config

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def csr_from_edges(m, n, edges, vals=None):
    edges = np.asarray(edges, dtype=np.int64)
    v = np.ones(len(edges)) if vals is None else np.asarray(vals, float)
    A = sp.csr_matrix((v, (edges[:, 0], edges[:, 1])), shape=(m, n))
    A.sort_indices()
    return A


# --------------------------------------------------------------------------------------
# An independent reordering: explicit BFS with a queue, written from Algorithm 2 and the
# same tie-break readings, without scipy.  Used only to pin the oracle on tiny graphs.
# --------------------------------------------------------------------------------------
def bfs_reorder(m, n, A, k):
    adjT = [list(A.indices[A.indptr[i]:A.indptr[i + 1]]) for i in range(m)]
    At = A.tocsc()
    adjF = [list(At.indices[At.indptr[j]:At.indptr[j + 1]]) for j in range(n)]
    aliveT = [True] * m
    aliveF = [True] * n
    piT = [-1] * m
    piF = [-1] * n
    lo = [0, 0]
    hi = [m - 1, n - 1]
    blocks = []
    it = 0
    while True:
        it += 1
        T = [i for i in range(m) if aliveT[i]]
        F = [j for j in range(n) if aliveF[j]]
        mh = min(len(T), math.ceil(k * len(T)))
        nh = min(len(F), math.ceil(k * len(F)))
        dT = {i: sum(1 for j in adjT[i] if aliveF[j]) for i in T}
        dF = {j: sum(1 for i in adjF[j] if aliveT[i]) for j in F}
        hT = sorted(T, key=lambda i: (-dT[i], i))[:mh]
        hF = sorted(F, key=lambda j: (-dF[j], j))[:nh]
        for i in hT:
            piT[i] = hi[0]; hi[0] -= 1; aliveT[i] = False
        for j in hF:
            piF[j] = hi[1]; hi[1] -= 1; aliveF[j] = False
        seen_T, seen_F = {}, {}
        comps = []
        seeds = [(0, i) for i in range(m) if aliveT[i]] + [(1, j) for j in range(n) if aliveF[j]]
        for side, v in seeds:
            if (seen_T if side == 0 else seen_F).get(v) is not None:
                continue
            cid = len(comps)
            cT, cF = [], []
            q = deque([(side, v)])
            (seen_T if side == 0 else seen_F)[v] = cid
            while q:
                s, u = q.popleft()
                if s == 0:
                    cT.append(u)
                    for j in adjT[u]:
                        if aliveF[j] and j not in seen_F:
                            seen_F[j] = cid; q.append((1, j))
                else:
                    cF.append(u)
                    for i in adjF[u]:
                        if aliveT[i] and i not in seen_T:
                            seen_T[i] = cid; q.append((0, i))
            comps.append((sorted(cT), sorted(cF)))
        if not comps:
            break
        sizes = [len(a) + len(b) for a, b in comps]
        g = sizes.index(max(sizes))
        for c, (cT, cF) in enumerate(comps):
            if c == g:
                continue
            blocks.append((lo[0], lo[1], len(cT), len(cF)))
            for i in cT:
                piT[i] = lo[0]; lo[0] += 1
            for j in cF:
                piF[j] = lo[1]; lo[1] += 1
        gT, gF = comps[g]
        for i in range(m):
            aliveT[i] = False
        for j in range(n):
            aliveF[j] = False
        for i in gT:
            aliveT[i] = True
        for j in gF:
            aliveF[j] = True
        if len(gT) < mh or len(gF) < nh or len(gT) + len(gF) == 0:
            break
    gT = [i for i in range(m) if aliveT[i]]
    gF = [j for j in range(n) if aliveF[j]]
    if gT or gF:
        blocks.append((lo[0], lo[1], len(gT), len(gF)))
        for i in gT:
            piT[i] = lo[0]; lo[0] += 1
        for j in gF:
            piF[j] = lo[1]; lo[1] += 1
    return np.array(piT), np.array(piF), np.array(blocks, dtype=np.int64).reshape(-1, 4), it


# ------------------------------------------------------------------ reordering pins ----
def test_toy_graph_matches_paper_ids():
    g = json.load(open(os.path.join(GOLDEN, "toy_fig2.json")))
    A = csr_from_edges(g["m"], g["n"], g["edges"])
    R = oracle.reorder(g["m"], g["n"], A.indptr, A.indices, g["k"])
    e = g["expected"]
    assert R.piT.tolist() == e["piT"]
    assert R.piF.tolist() == e["piF"]
    assert R.blocks.tolist() == e["blocks"]
    assert (R.m1, R.n1, R.m2, R.n2, R.iterations) == (e["m1"], e["n1"], e["m2"], e["n2"], e["iterations"])
    # the facts the paper states for the first iteration (ids 9 and 7, spokes lowest)
    assert R.piT[4] == g["m"] - 1 and R.piF[3] == g["n"] - 1
    assert R.blocks[0].tolist() == e["first_iteration"]["spoke_block"]


@pytest.mark.parametrize("seed", range(12))
def test_reorder_matches_independent_bfs(seed):
    rng = np.random.default_rng(100 + seed)
    m = int(rng.integers(5, 40)); n = int(rng.integers(3, 25))
    dens = rng.uniform(0.03, 0.3)
    mask = rng.random((m, n)) < dens
    A = sp.csr_matrix(mask.astype(float))
    k = float(rng.choice([0.01, 0.05, 0.1, 0.2]))
    R = oracle.reorder(m, n, A.indptr, A.indices, k)
    piT, piF, blocks, it = bfs_reorder(m, n, A, k)
    assert R.piT.tolist() == piT.tolist()
    assert R.piF.tolist() == piF.tolist()
    assert R.blocks.tolist() == blocks.tolist()
    assert R.iterations == it


def _check_reorder_invariants(m, n, A, R):
    assert sorted(R.piT.tolist()) == list(range(m))
    assert sorted(R.piF.tolist()) == list(range(n))
    assert R.blocks[:, 2].sum() == R.m1 and R.blocks[:, 3].sum() == R.n1
    C = A.tocoo()
    nr, nc = R.piT[C.row], R.piF[C.col]
    in11 = (nr < R.m1) & (nc < R.n1)
    rb = np.full(R.m1, -1); cb = np.full(R.n1, -1)
    for b, (r0, c0, mi, ni) in enumerate(R.blocks):
        rb[r0:r0 + mi] = b; cb[c0:c0 + ni] = b
    assert (rb >= 0).all() and (cb >= 0).all()
    # A11 is exactly block diagonal
    assert (rb[nr[in11]] == cb[nc[in11]]).all()
    # every block with rows and columns is connected
    for b, (r0, c0, mi, ni) in enumerate(R.blocks):
        if mi == 0 or ni == 0:
            assert mi + ni == 1 or b == len(R.blocks) - 1
            continue
        sel = in11 & (rb[np.minimum(nr, R.m1 - 1)] == b)
        Bsub = sp.coo_matrix((np.ones(sel.sum()), (nr[sel] - r0, m * 0 + nc[sel] - c0)), shape=(mi, ni))
        G = sp.bmat([[None, Bsub], [Bsub.T, None]])
        ncomp, _ = sp.csgraph.connected_components(G, directed=False)
        assert ncomp == 1


@pytest.mark.parametrize("name,cfg", [
    ("c1-like", small_config(2000, 500, 0.01, gamma=2.1, values="uniform", seed=1000)),
    ("mid", small_config(3000, 800, 0.004, gamma=1.9, seed=11)),
])
def test_reorder_invariants(name, cfg):
    p = make_problem(cfg, with_labels=False)
    A = sp.csr_matrix((p.data, p.indices, p.indptr), shape=(p.m, p.n))
    R = oracle.reorder(p.m, p.n, p.indptr, p.indices, cfg.k)
    _check_reorder_invariants(p.m, p.n, A, R)


def test_hub_counts_use_double_ceiling():
    assert oracle.target_rank(0.3, 500) == 150
    assert oracle.target_rank(0.2, 2000) == 400
    assert oracle.target_rank(0.1, 5000) == 500
    assert oracle.target_rank(0.1, 10000) == 1000
    assert oracle.hub_count(0.01, 20000) == 200 and oracle.hub_count(0.01, 2000) == 20
    assert oracle.hub_count(0.01, 1) == 1 and oracle.hub_count(0.01, 0) == 0


# ------------------------------------------------------------------ SVD-stage pins -----
def small_problem(m=120, n=40, density=0.08, seed=3, alpha=1.0, k=0.05, values="lognormal"):
    cfg = small_config(m, n, density, gamma=2.0, values=values, L=6, p_label=0.2, alpha=alpha,
                       seed=seed, k=k)
    return make_problem(cfg)


def dense(p):
    return sp.csr_matrix((p.data, p.indices, p.indptr), shape=(p.m, p.n)).toarray()


def eig_sigma(M):
    """Singular values from the symmetric eigenvalue routine, descending."""
    M = np.asarray(M)
    G = M.T @ M if M.shape[0] >= M.shape[1] else M @ M.T
    w = sla.eigh(G, eigvals_only=True)[::-1]
    return np.sqrt(np.clip(w, 0.0, None))


@pytest.mark.parametrize("seed", [1, 2, 3, 4])
def test_alpha_one_is_exact(seed):
    """Problem 1: at full rank no truncation bites, so U Sigma V^T = A and
    V Sigma^+ U^T is the Moore-Penrose inverse."""
    p = small_problem(seed=seed)
    A = dense(p)
    res = oracle.fastpi_svd(p.m, p.n, p.indptr, p.indices, p.data, 1.0, 0.05)
    Arec = (res.U * res.sigma) @ res.V.T
    assert np.abs(Arec - A).max() <= 1e-12 * np.abs(A).max()
    # singular values equal those of A (eigenvalue route, different routine)
    # (compared as squares: the eigenvalue route fixes sigma^2 to eps * sigma_1^2)
    lam = eig_sigma(A) ** 2
    assert np.abs(np.sort(res.sigma)[::-1] ** 2 - lam[:res.r]).max() <= 1e-12 * lam[0]
    # Moore-Penrose conditions
    Ap = (res.V * oracle.sigma_pinv(res.sigma, p.m, p.n)) @ res.U.T
    s = np.abs(A).max()
    assert np.abs(A @ Ap @ A - A).max() <= 1e-10 * s
    assert np.abs(Ap @ A @ Ap - Ap).max() <= 1e-10 * np.abs(Ap).max()
    assert np.abs((A @ Ap).T - A @ Ap).max() <= 1e-10
    assert np.abs((Ap @ A).T - Ap @ A).max() <= 1e-10
    # the regression solution is the least-squares one (normal equations, Cholesky)
    Z = oracle.pinv_apply(res.U, res.sigma, res.V, p.Y)
    if np.linalg.matrix_rank(A) == p.n:
        Zn = sla.cho_solve(sla.cho_factor(A.T @ A), A.T @ p.Y)
        assert np.abs(Z - Zn).max() <= 1e-8 * max(1.0, np.abs(Zn).max())


def test_alpha_one_rank_deficient_matches_dense_pinv():
    # duplicate columns make A rank deficient; the minimum-norm solution is the pinv one
    p = small_problem(m=90, n=30, density=0.1, seed=9)
    A = dense(p)
    A[:, 5] = A[:, 7]
    A[:, 11] = 0.0
    Asp = sp.csr_matrix(A)
    res = oracle.fastpi_svd(p.m, p.n, Asp.indptr, Asp.indices, Asp.data, 1.0, 0.05)
    Z = oracle.pinv_apply(res.U, res.sigma, res.V, p.Y)
    Zd = np.linalg.pinv(A) @ p.Y
    assert np.abs(Z - Zd).max() <= 1e-9 * max(1.0, np.abs(Zd).max())


def test_one_wide_and_rank_one_blocks_closed_form():
    # a 1-wide block, a rank-one block and a 2x2 block, a larger dense block that stays
    # the giant component, one hub row and one hub column touching everything
    rng = np.random.default_rng(5)
    a = rng.uniform(0.5, 2.0, 4)
    x = rng.uniform(0.5, 2.0, 3); y = rng.uniform(0.5, 2.0, 2)
    A = np.zeros((15, 9))
    A[0:4, 0] = a
    A[4:7, 1:3] = np.outer(x, y)
    A[7:9, 3:5] = [[3.0, 1.0], [1.0, 2.0]]
    A[9:14, 5:8] = rng.uniform(0.5, 2.0, (5, 3))
    A[14, :] = 1.0            # hub row
    A[:, 8] = 1.0             # hub column
    Asp = sp.csr_matrix(A)
    R = oracle.reorder(15, 9, Asp.indptr, Asp.indices, 0.05)
    S = ofp.split_blocks(15, 9, Asp.indptr, Asp.indices, Asp.data, R)
    B = ofp.block_svd(S, 1.0)
    got = [np.asarray(s) for s in B.block_sigma]
    # 1-wide: sigma = ||a||; rank one: sigma = ||x|| ||y||, 0; 2x2 symmetric: its eigenvalues
    ev = np.sort(np.linalg.eigvalsh(np.array([[3.0, 1.0], [1.0, 2.0]])))[::-1]
    want = [np.array([np.linalg.norm(a)]),
            np.array([np.linalg.norm(x) * np.linalg.norm(y), 0.0]),
            ev]
    for w in want:
        assert any(g.shape == w.shape and np.allclose(g, w, rtol=1e-13, atol=1e-13) for g in got), w
    # the spoke blocks are the first three blocks, in discovery order
    assert R.blocks[:3, 2:].tolist() == [[4, 1], [3, 2], [2, 2]]


def test_block_stage_reconstructs_a11_at_full_rank():
    p = small_problem(m=200, n=60, density=0.04, seed=21)
    R = oracle.reorder(p.m, p.n, p.indptr, p.indices, 0.05)
    S = ofp.split_blocks(p.m, p.n, p.indptr, p.indices, p.data, R)
    B = ofp.block_svd(S, 1.0)
    A11 = S.A_perm[:S.m1, :S.n1].toarray()
    rec = (B.U1.toarray() * B.sigma1) @ B.V1.toarray().T
    assert np.abs(rec - A11).max() <= 1e-12 * max(1.0, np.abs(A11).max())
    assert oracle.orthonormality_error(B.U1.toarray()) < 1e-13
    assert oracle.orthonormality_error(B.V1.toarray()) < 1e-13


@pytest.mark.parametrize("alpha", [0.2, 0.5])
def test_row_and_column_updates_are_eckart_young(alpha):
    """Each update is the best rank-s (rank-r) approximation of the formed matrix:
    the squared error equals the sum of the discarded squared singular values,
    which is taken here from an eigenvalue routine on a matrix the test forms itself."""
    p = small_problem(m=300, n=90, density=0.05, seed=31, alpha=alpha)
    R = oracle.reorder(p.m, p.n, p.indptr, p.indices, 0.05)
    S = ofp.split_blocks(p.m, p.n, p.indptr, p.indices, p.data, R)
    B = ofp.block_svd(S, alpha)
    # row update
    R2 = ofp.row_update(S, B, alpha)
    top = (B.U1.toarray() * B.sigma1) @ B.V1.toarray().T       # U1 Sigma1 V1^T
    M = np.vstack([top, S.A21.toarray()])                     # [A11_approx ; A21]
    s = R2.sigma.size
    assert s == min(oracle.target_rank(alpha, S.n1), B.sigma1.size + S.m2, S.n1)
    err2 = np.sum((M - (R2.U * R2.sigma) @ R2.V.T) ** 2)
    lam = eig_sigma(M) ** 2
    assert abs(err2 - lam[s:].sum()) <= 1e-9 * lam.sum()
    assert np.allclose(R2.sigma, np.sqrt(lam[:s]), rtol=1e-9, atol=1e-12 * np.sqrt(lam[0]))
    assert oracle.orthonormality_error(R2.U) < 1e-12
    # column update
    R3 = ofp.column_update(S, R2, alpha, p.m, p.n)
    X = np.hstack([(R2.U * R2.sigma) @ R2.V.T, S.T.toarray()])  # [U2 Sigma2 V2^T, T]
    r = R3.sigma.size
    assert r == min(oracle.target_rank(alpha, min(p.m, p.n)), s + S.n2, p.m)
    err2 = np.sum((X - (R3.U * R3.sigma) @ R3.V.T) ** 2)
    lam = eig_sigma(X) ** 2
    assert abs(err2 - lam[r:].sum()) <= 1e-9 * lam.sum()
    assert oracle.orthonormality_error(R3.U) < 1e-12
    assert oracle.orthonormality_error(R3.V) < 1e-12


def test_truncated_error_is_bounded_by_eckart_young():
    p = small_problem(m=400, n=100, density=0.03, seed=41, alpha=0.3)
    A = dense(p)
    res = oracle.fastpi_svd(p.m, p.n, p.indptr, p.indices, p.data, 0.3, 0.05)
    e = oracle.recon_error(sp.csr_matrix(A), res.U, res.sigma, res.V)
    lam = eig_sigma(A) ** 2
    e_opt = math.sqrt(lam[res.r:].sum() / lam.sum())
    assert e >= e_opt - 1e-12
    assert e <= 1.0
    # and the trace formula equals the dense Frobenius error
    ed = np.linalg.norm(A - (res.U * res.sigma) @ res.V.T) / np.linalg.norm(A)
    assert abs(e - ed) <= 1e-12


def test_sigma_pinv_threshold():
    s = np.array([2.0, 1.0, 1e-14, 0.0])
    out = oracle.sigma_pinv(s, 100, 10)
    assert out[0] == 0.5 and out[1] == 1.0 and out[2] == 0.0 and out[3] == 0.0
    tol = 100 * np.finfo(float).eps * 2.0
    s2 = np.array([2.0, tol * 1.01])
    assert oracle.sigma_pinv(s2, 100, 10)[1] > 0


# ------------------------------------------------ planted mistakes must fail a pin -----
def test_planted_mistakes_are_caught(monkeypatch):
    """A plausible slip in the oracle (dropped Sigma1 in Eq. 2, a transposed right
    factor in Eq. 3) breaks the alpha = 1 exactness pin."""
    p = small_problem(seed=2)
    A = dense(p)

    def exact(res):
        return np.abs((res.U * res.sigma) @ res.V.T - A).max() <= 1e-10 * np.abs(A).max()

    good = oracle.fastpi_svd(p.m, p.n, p.indptr, p.indices, p.data, 1.0, 0.05)
    assert exact(good)

    orig_row = ofp.row_update

    def row_without_sigma(S, B, alpha, inner=None):
        B2 = ofp.BlockStage(B.U1, np.ones_like(B.sigma1), B.V1, B.ranks, B.block_sigma)
        return orig_row(S, B2, alpha, inner)

    monkeypatch.setattr(ofp, "row_update", row_without_sigma)
    bad = ofp.fastpi_svd(p.m, p.n, p.indptr, p.indices, p.data, 1.0, 0.05)
    assert not exact(bad)
    monkeypatch.setattr(ofp, "row_update", orig_row)

    orig_col = ofp.column_update

    def col_transposed(S, R2, alpha, m, n, inner=None):
        st = orig_col(S, R2, alpha, m, n, inner)
        s = R2.sigma.size
        Vh_top = np.linalg.lstsq(R2.V, st.V[:S.n1], rcond=None)[0]
        V = np.vstack([R2.V @ Vh_top[:, ::-1], st.V[S.n1:]])
        return ofp.Stage(st.U, st.sigma, V, st.full_sigma)

    monkeypatch.setattr(ofp, "column_update", col_transposed)
    bad = ofp.fastpi_svd(p.m, p.n, p.indptr, p.indices, p.data, 1.0, 0.05)
    assert not exact(bad)


# ------------------------------------- the two metric functions every parity test uses -----
# ls_residual is Application 1's least-squares objective ||A Z - Y||_F / ||Y||_F, and
# orthonormality_error is max |Q^T Q - I| over the columns kept by the pseudoinverse
# threshold (the orthonormality claims after Eqs. 1-3 hold for those). Both are pinned to
# hand-computed values, and a planted slip in either must break its pin.

def _ls_pin(fn):
    """Integer A, Z, Y with the residual worked out by hand:
    A Z = [[1, 2], [0, 3], [4, 0]], Y = [[1, 2], [0, 5], [3, 0]], so A Z - Y has the
    entries 0, 0, 0, -2, 1, 0: ||A Z - Y||_F = sqrt(5), ||Y||_F = sqrt(1+4+25+9) = sqrt(39)."""
    A = sp.csr_matrix(np.array([[1.0, 2.0], [0.0, 3.0], [4.0, 0.0]]))
    Z = np.array([[1.0, 0.0], [0.0, 1.0]])
    Y = np.array([[1.0, 2.0], [0.0, 5.0], [3.0, 0.0]])
    ok = abs(fn(A, Z, Y) - math.sqrt(5.0 / 39.0)) <= 1e-15
    # a non-square Z: A (3x2) Z (2x3) with Z = [[1, 0, 2], [0, 1, -1]]:
    # A Z = [[1, 2, 0], [0, 3, -3], [4, 0, 8]]; Y2 = A Z + E with E = [[0, 0, 1], [0, -2, 0],
    # [0, 0, 0]] gives ||A Z - Y2||_F = sqrt(5) and ||Y2||_F^2 = 1+4+1+0+1+9+16+0+64 = 96
    Z2 = np.array([[1.0, 0.0, 2.0], [0.0, 1.0, -1.0]])
    Y2 = np.array([[1.0, 2.0, 1.0], [0.0, 1.0, -3.0], [4.0, 0.0, 8.0]])
    ok &= abs(fn(A, Z2, Y2) - math.sqrt(5.0 / 96.0)) <= 1e-15
    # at the least-squares solution the residual is Y minus its projection on range(A):
    # ||R||^2 = ||Y||^2 - ||Q^T Y||^2 with Q from a QR of A (another routine than the
    # product the function forms)
    rng = np.random.default_rng(7)
    Ad = rng.standard_normal((30, 6))
    Yd = rng.standard_normal((30, 4))
    Zd = sla.lstsq(Ad, Yd)[0]
    Q, _ = sla.qr(Ad, mode="economic")
    want = math.sqrt(max(np.sum(Yd ** 2) - np.sum((Q.T @ Yd) ** 2), 0.0) / np.sum(Yd ** 2))
    ok &= abs(fn(sp.csr_matrix(Ad), Zd, Yd) - want) <= 1e-13
    return bool(ok)


def test_ls_residual_pinned():
    assert _ls_pin(oracle.ls_residual)
    # Y = 0: the unnormalised residual norm (documented), here ||A Z||_F = sqrt(1+4+9+16)
    A = sp.csr_matrix(np.array([[1.0, 2.0], [0.0, 3.0], [4.0, 0.0]]))
    assert abs(oracle.ls_residual(A, np.eye(2), np.zeros((3, 2))) - math.sqrt(30.0)) <= 1e-15


def test_ls_residual_planted_slips_fail_the_pin():
    def by_square_norm(A, Z, Y):            # normalised by ||Y||^2 instead of ||Y||
        R = sp.csr_matrix(A) @ Z - Y
        return float(np.linalg.norm(R)) / float(np.sum(Y ** 2))

    def plus_y(A, Z, Y):                     # A Z + Y instead of A Z - Y
        R = sp.csr_matrix(A) @ Z + Y
        return float(np.linalg.norm(R)) / float(np.linalg.norm(Y))

    def max_norm(A, Z, Y):                   # largest entry instead of the Frobenius norm
        R = sp.csr_matrix(A) @ Z - Y
        return float(np.abs(R).max()) / float(np.linalg.norm(Y))

    for slip in (by_square_norm, plus_y, max_norm):
        assert not _ls_pin(slip), slip.__name__


def _orth_pin(fn):
    """A planted Q (6 x 4) with known defects:
    q1 = e1; q2 = (1 + eta) e2 (norm defect (1+eta)^2 - 1); q3 = e3 + delta e1 (off-diagonal
    defect delta < 0, norm defect delta^2); q4 = 5 e4 (defect 24) carried by a singular value
    that the pseudoinverse threshold max(m, n) eps sigma_1 drops or keeps."""
    eta, delta = 1e-3, -3e-3
    Q = np.zeros((6, 4))
    Q[0, 0] = 1.0
    Q[1, 1] = 1.0 + eta
    Q[2, 2] = 1.0
    Q[0, 2] = delta
    Q[3, 3] = 5.0
    eps = np.finfo(np.float64).eps
    m, n = 6, 1000                    # threshold 1000 eps sigma_1, set by n (not by Q's rows)
    want_kept3 = max((1 + eta) ** 2 - 1, abs(delta), delta ** 2)      # = 3e-3 (the |delta|)
    ok = True
    # sigma_4 under the threshold: column 4 is left out
    s_drop = np.array([1.0, 0.5, 0.2, 500 * eps])
    ok &= abs(fn(Q, s_drop, m, n) - want_kept3) <= 1e-15
    # sigma_4 just above it: column 4 counts, its defect 24 dominates
    s_keep = np.array([1.0, 0.5, 0.2, 1001 * eps])
    ok &= abs(fn(Q, s_keep, m, n) - 24.0) <= 1e-12
    # no sigma: every column counts
    ok &= abs(fn(Q) - 24.0) <= 1e-12
    # an exactly orthonormal Q (a Householder reflector's columns) reads ~0
    v = np.arange(1.0, 7.0)[:, None]
    H = np.eye(6) - 2.0 * (v @ v.T) / float(np.sum(v * v))
    ok &= fn(H[:, :4]) <= 4 * eps
    return bool(ok)


def test_orthonormality_error_pinned():
    assert _orth_pin(oracle.orthonormality_error)
    assert oracle.orthonormality_error(np.zeros((5, 0))) == 0.0


def test_orthonormality_error_planted_slips_fail_the_pin():
    def signed_max(Q, sigma=None, m=None, n=None):        # missing abs
        if sigma is not None:
            Q = Q[:, oracle.sigma_pinv(sigma, m or Q.shape[0], n or Q.shape[0]) > 0]
        return float(np.max(Q.T @ Q - np.eye(Q.shape[1])))

    def rows_as_n(Q, sigma=None, m=None, n=None):         # threshold from Q's rows, not n
        if sigma is not None:
            Q = Q[:, oracle.sigma_pinv(sigma, Q.shape[0], Q.shape[0]) > 0]
        return float(np.max(np.abs(Q.T @ Q - np.eye(Q.shape[1]))))

    def no_filter(Q, sigma=None, m=None, n=None):         # sigma ignored
        return float(np.max(np.abs(Q.T @ Q - np.eye(Q.shape[1]))))

    def positive_filter(Q, sigma=None, m=None, n=None):   # keeps every sigma > 0
        if sigma is not None:
            Q = Q[:, np.asarray(sigma) > 0]
        return float(np.max(np.abs(Q.T @ Q - np.eye(Q.shape[1]))))

    def offdiag_only(Q, sigma=None, m=None, n=None):      # norm defects missed
        if sigma is not None:
            Q = Q[:, oracle.sigma_pinv(sigma, m, n) > 0]
        G = Q.T @ Q
        return float(np.max(np.abs(G - np.diag(np.diag(G)))))

    for slip in (signed_max, rows_as_n, no_filter, positive_filter, offdiag_only):
        assert not _orth_pin(slip), slip.__name__


def _block_override_pin(fastpi_svd):
    """Eq. 1 with given per-block ranks: each dense block keeps min(given, m_i, n_i)
    directions, its truncation loss is the Eckart-Young one (eigenvalue route), the block
    singular values are the block's largest ones, and the later ranks follow their rules."""
    p = small_problem(m=300, n=90, density=0.05, seed=21, alpha=0.3, k=0.05)
    alpha = 0.3
    R = oracle.reorder(p.m, p.n, p.indptr, p.indices, 0.05)
    rng = np.random.default_rng(4)
    given = rng.integers(0, 6, size=len(R.blocks))
    res = fastpi_svd(p.m, p.n, p.indptr, p.indices, p.data, alpha, 0.05, block_ranks=given)
    S = ofp.split_blocks(p.m, p.n, p.indptr, p.indices, p.data, R)
    col = 0
    for Ai, b in zip(S.block_dense, S.block_index):
        mi, ni = Ai.shape
        si = min(int(given[b]), mi, ni)
        assert res.blocks.ranks[b] == si
        sig = eig_sigma(Ai)
        r0, c0 = int(S.blocks[b][0]), int(S.blocks[b][1])
        U1 = res.blocks.U1[r0:r0 + mi, col:col + si].toarray()
        V1 = res.blocks.V1[c0:c0 + ni, col:col + si].toarray()
        s1 = res.blocks.sigma1[col:col + si]
        assert np.allclose(s1, sig[:si], rtol=1e-10, atol=1e-12 * max(sig[0], 1e-300))
        loss = np.sum((Ai - (U1 * s1) @ V1.T) ** 2)
        assert abs(loss - np.sum(sig[si:] ** 2)) <= 1e-10 * np.sum(sig ** 2)
        col += si
    s_b = col
    assert res.blocks.sigma1.size == s_b
    assert res.row.sigma.size == min(ofp.target_rank(alpha, S.n1), s_b + S.m2, S.n1)
    return res


def test_block_rank_override_pinned():
    p = small_problem(m=300, n=90, density=0.05, seed=21, alpha=0.3, k=0.05)
    _block_override_pin(oracle.fastpi_svd)
    # the alpha rule's own ranks given explicitly: the same result, bit for bit
    ref = oracle.fastpi_svd(p.m, p.n, p.indptr, p.indices, p.data, 0.3, 0.05)
    same = oracle.fastpi_svd(p.m, p.n, p.indptr, p.indices, p.data, 0.3, 0.05, block_ranks=ref.blocks.ranks)
    assert np.array_equal(ref.sigma, same.sigma) and np.array_equal(ref.U, same.U)


def test_block_rank_override_planted_slip_fails_the_pin():
    """An oracle that ignores the given ranks (keeps Eq. 1's alpha rule) fails the pin."""
    def ignoring(m, n, indptr, indices, data, alpha, k=0.01, block_ranks=None):
        return oracle.fastpi_svd(m, n, indptr, indices, data, alpha, k)
    with pytest.raises(AssertionError):
        _block_override_pin(ignoring)

    def off_by_one(m, n, indptr, indices, data, alpha, k=0.01, block_ranks=None):
        return oracle.fastpi_svd(m, n, indptr, indices, data, alpha, k,
                                 block_ranks=np.asarray(block_ranks) + 1)
    with pytest.raises(AssertionError):
        _block_override_pin(off_by_one)
