"""Oracle for FastPI's low-rank SVD and pseudoinverse apply, FP64 on the CPU.

TEST INFRASTRUCTURE ONLY (see the package docstring).

FastPI truncates at three points, so its result has no closed form for alpha < 1;
the oracle therefore follows the method's steps in the paper's order, and every
"low-rank approximation" is the exact truncated SVD of the explicitly formed
intermediate matrix (the paper's "standard SVD" branch, Section 3.3.2), taken
with LAPACK through ``numpy.linalg.svd``:

1. reorder A (Algorithm 2; ``oracle.reorder``) and split it into A11, A12, A21,
   A22 (Section 3.3);
2. SVD of every diagonal block of A11, block i truncated to
   s_i = min(ceil(alpha*n_i), m_i, n_i) and concatenated in block order with no
   global re-truncation (Eq. 1);
3. row update: SVD of the formed M2 = [Sigma1 V1^T ; A21], truncated to
   s = min(ceil(alpha*n1), s_b + m2, n1), and U2 = [U1 Ut_top ; Ut_bot] (Eq. 2);
4. column update: SVD of the formed X3 = [U2 Sigma2, T] with T = [A12 ; A22],
   truncated to r = min(ceil(alpha*min(m, n)), s + n2, m), and
   V = [V2 Vt_top ; Vt_bot] (Eq. 3);
5. map U and V back to the original row and column order;
6. apply: Z = V Sigma^+ (U^T Y) (Problem 1, Application 1), where
   sigma^+_i = 1/sigma_i if sigma_i > max(m, n) * eps * sigma_1, else 0.

Readings of points the paper leaves open: the ceiling of a real product is
ceil(alpha * x) in IEEE double; Eq. 1's garbled rank sum is read as the sum of
the per-block ranks; Eq. 2 uses "s" for its input and output ranks, read as s_b
in and ceil(alpha*n1) out; the pseudoinverse threshold (not stated in the
paper) is MATLAB's documented pinv default, since the paper's experiments use
MATLAB (Section 4.1).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import scipy.sparse as sp

from .randomized import InnerSolver, rsvd_right, sign_convention, use_randomized
from .reorder import Reordering, reorder

EPS = np.finfo(np.float64).eps


def target_rank(alpha: float, x: int) -> int:
    """ceil(alpha * x) evaluated in IEEE double (Table 1: r = ceil(alpha n))."""
    return max(0, int(math.ceil(alpha * float(x))))


@dataclasses.dataclass
class Split:
    """The reordered matrix cut into its four parts (Section 3.3)."""
    m1: int
    n1: int
    m2: int
    n2: int
    blocks: np.ndarray            # int64[B, 4] (row0, col0, rows, cols)
    block_dense: list             # dense A11 blocks (only blocks with rows and cols > 0)
    block_index: list             # index into `blocks` of each dense block
    A21: sp.csr_matrix            # m2 x n1
    T: sp.csr_matrix              # m x n2, = [A12 ; A22]
    A_perm: sp.csr_matrix         # the whole reordered matrix (m x n)


def split_blocks(m, n, indptr, indices, data, R: Reordering) -> Split:
    A = sp.csr_matrix((np.asarray(data, np.float64), np.asarray(indices), np.asarray(indptr)),
                      shape=(m, n))
    A.eliminate_zeros()
    # reordered matrix: row i moves to piT[i], column j to piF[j]
    P = A.tocoo()
    Ap = sp.csr_matrix((P.data, (R.piT[P.row].astype(np.int64), R.piF[P.col].astype(np.int64))),
                       shape=(m, n))
    Ap.sort_indices()
    m1, n1 = R.m1, R.n1
    block_dense, block_index = [], []
    for b, (r0, c0, mi, ni) in enumerate(R.blocks):
        if mi > 0 and ni > 0:
            block_dense.append(Ap[r0:r0 + mi, c0:c0 + ni].toarray())
            block_index.append(b)
    A21 = Ap[m1:, :n1].tocsr()
    T = Ap[:, n1:].tocsr()
    return Split(m1, n1, m - m1, n - n1, R.blocks, block_dense, block_index, A21, T, Ap)


@dataclasses.dataclass
class BlockStage:
    U1: sp.csr_matrix      # m1 x s_b, block diagonal
    sigma1: np.ndarray     # s_b
    V1: sp.csr_matrix      # n1 x s_b, block diagonal
    ranks: np.ndarray      # s_i of every block in `blocks` (0 for empty blocks)
    block_sigma: list      # full singular value list of every dense block


def block_svd(S: Split, alpha: float, block_ranks=None) -> BlockStage:
    """Eq. 1: truncated SVD of every diagonal block, joined with bdiag. Block i keeps
    s_i = min(ceil(alpha n_i), m_i, n_i) directions, or min(block_ranks[i], m_i, n_i) when
    per-block ranks are given (one per entry of the block table, e.g. a learned allocation)."""
    if block_ranks is not None:
        block_ranks = np.asarray(block_ranks, dtype=np.int64)
        if block_ranks.shape != (len(S.blocks),) or np.any(block_ranks < 0):
            raise ValueError("block_ranks needs one non-negative rank per block")
    ranks = np.zeros(len(S.blocks), dtype=np.int64)
    urows, ucols, uvals = [], [], []
    vrows, vcols, vvals = [], [], []
    sig = []
    block_sigma = []
    col = 0
    for Ai, b in zip(S.block_dense, S.block_index):
        r0, c0, mi, ni = (int(x) for x in S.blocks[b])
        U, s, Vt = np.linalg.svd(Ai, full_matrices=False)
        block_sigma.append(s)
        want = target_rank(alpha, ni) if block_ranks is None else int(block_ranks[b])
        si = min(want, mi, ni)
        ranks[b] = si
        if si == 0:
            continue
        rr, cc = np.meshgrid(np.arange(mi), np.arange(si), indexing="ij")
        urows.append((r0 + rr).ravel()); ucols.append((col + cc).ravel()); uvals.append(U[:, :si].ravel())
        rr, cc = np.meshgrid(np.arange(ni), np.arange(si), indexing="ij")
        vrows.append((c0 + rr).ravel()); vcols.append((col + cc).ravel()); vvals.append(Vt[:si].T.ravel())
        sig.append(s[:si])
        col += si
    s_b = col
    cat = (lambda xs, dt: np.concatenate(xs).astype(dt) if xs else np.zeros(0, dt))
    U1 = sp.csr_matrix((cat(uvals, np.float64), (cat(urows, np.int64), cat(ucols, np.int64))),
                       shape=(S.m1, s_b))
    V1 = sp.csr_matrix((cat(vvals, np.float64), (cat(vrows, np.int64), cat(vcols, np.int64))),
                       shape=(S.n1, s_b))
    return BlockStage(U1, cat(sig, np.float64), V1, ranks, block_sigma)


@dataclasses.dataclass
class Stage:
    U: np.ndarray          # rows x rank
    sigma: np.ndarray      # rank
    V: np.ndarray          # cols x rank
    full_sigma: np.ndarray  # every singular value of the formed matrix (for gap checks)


def row_update(S: Split, B: BlockStage, alpha: float, inner: InnerSolver | None = None) -> Stage:
    """Eq. 2: SVD of M2 = [Sigma1 V1^T ; A21] truncated to s, U2 = [U1 Ut_top ; Ut_bot].
    With a randomized inner solver that applies (oracle.randomized), the truncated SVD of
    M2 is the randomized one (full_sigma then holds the exact spectrum for reference)."""
    s_b = B.sigma1.size
    top = (B.V1.multiply(B.sigma1[None, :])).T.toarray() if s_b else np.zeros((0, S.n1))
    M2 = np.vstack([top, S.A21.toarray()])
    if M2.size == 0:
        m = S.m1 + S.m2
        return Stage(np.zeros((m, 0)), np.zeros(0), np.zeros((S.n1, 0)), np.zeros(0))
    s = min(target_rank(alpha, S.n1), s_b + S.m2, S.n1)
    if use_randomized(inner, s, S.n1):
        Ut, sig, V2 = rsvd_right(M2, s, inner.oversample, inner.iters, inner.seed, 0)
        U2 = np.vstack([B.U1 @ Ut[:s_b], Ut[s_b:]])
        return Stage(U2, sig, V2, np.linalg.svd(M2, compute_uv=False))
    Ut, st, Vt = np.linalg.svd(M2, full_matrices=False)
    U2 = np.vstack([B.U1 @ Ut[:s_b, :s], Ut[s_b:, :s]])
    return Stage(U2, st[:s].copy(), Vt[:s].T.copy(), st)


def column_update(S: Split, R2: Stage, alpha: float, m: int, n: int,
                  inner: InnerSolver | None = None) -> Stage:
    """Eq. 3: SVD of X3 = [U2 Sigma2, T] truncated to r, V = [V2 Vt_top ; Vt_bot] (randomized
    as in row_update when the inner solver applies)."""
    s = R2.sigma.size
    r = min(target_rank(alpha, min(m, n)), s + S.n2, m)
    if use_randomized(inner, r, s + S.n2):
        sgn = sign_convention(R2.V)
        X3 = np.hstack([R2.U * (sgn * R2.sigma)[None, :], S.T.toarray()])
        Ur, sig, Vh = rsvd_right(X3, r, inner.oversample, inner.iters, inner.seed, 1)
        V = np.vstack([(R2.V * sgn[None, :]) @ Vh[:s], Vh[s:]])
        return Stage(Ur, sig, V, np.linalg.svd(X3, compute_uv=False))
    X3 = np.hstack([R2.U * R2.sigma[None, :], S.T.toarray()])
    if X3.size == 0:
        return Stage(np.zeros((m, 0)), np.zeros(0), np.zeros((n, 0)), np.zeros(0))
    Ut, st, Vt = np.linalg.svd(X3, full_matrices=False)
    Vh = Vt[:r].T
    V = np.vstack([R2.V @ Vh[:s], Vh[s:]])
    return Stage(Ut[:, :r].copy(), st[:r].copy(), V, st)


@dataclasses.dataclass
class OracleResult:
    U: np.ndarray          # m x r, original row order
    sigma: np.ndarray      # r, descending
    V: np.ndarray          # n x r, original column order
    reordering: Reordering
    split: Split
    blocks: BlockStage
    row: Stage
    col: Stage

    @property
    def r(self):
        return self.sigma.size


def fastpi_svd(m, n, indptr, indices, data, alpha, k=0.01,
               inner: InnerSolver | None = None, block_ranks=None) -> OracleResult:
    """Algorithm 1 lines 1-4, results mapped back to the original order; `inner` selects
    the truncated inner solver of the two updates (None: exact); `block_ranks` replaces
    Eq. 1's per-block ranks (one per entry of the reordering's block table), the later
    truncations keep their rules (s from n1 and the new s_b, r from min(m, n))."""
    if not (0.0 < alpha <= 1.0):
        raise ValueError("alpha must lie in (0, 1]")
    A = sp.csr_matrix((np.asarray(data, np.float64), np.asarray(indices), np.asarray(indptr)),
                      shape=(m, n))
    A.eliminate_zeros()
    A.sort_indices()
    R = reorder(m, n, A.indptr, A.indices, k)
    S = split_blocks(m, n, A.indptr, A.indices, A.data, R)
    B = block_svd(S, alpha, block_ranks)
    R2 = row_update(S, B, alpha, inner)
    R3 = column_update(S, R2, alpha, m, n, inner)
    U = R3.U[R.piT.astype(np.int64), :]
    V = R3.V[R.piF.astype(np.int64), :]
    return OracleResult(U, R3.sigma, V, R, S, B, R2, R3)


def sigma_pinv(sigma: np.ndarray, m: int, n: int) -> np.ndarray:
    """Sigma^+ with MATLAB's pinv threshold max(m, n) * eps * sigma_1."""
    if sigma.size == 0:
        return sigma.copy()
    tol = max(m, n) * EPS * float(np.max(sigma))
    out = np.zeros_like(sigma)
    keep = sigma > tol
    out[keep] = 1.0 / sigma[keep]
    return out


def pinv_apply(U, sigma, V, Y, m=None, n=None) -> np.ndarray:
    """Z = V Sigma^+ U^T Y (Problem 1 with Application 1)."""
    m = U.shape[0] if m is None else m
    n = V.shape[0] if n is None else n
    W = U.T @ Y
    W = sigma_pinv(sigma, m, n)[:, None] * W
    return V @ W


def recon_error(A: sp.spmatrix, U, sigma, V) -> float:
    """||A - U Sigma V^T||_F / ||A||_F without forming an m x n matrix:
    ||A||^2 - 2 tr(Sigma U^T A V) + tr((U^T U) Sigma (V^T V) Sigma)."""
    A = sp.csr_matrix(A)
    a2 = float(np.sum(A.data ** 2))
    AV = A @ V
    cross = float(np.sum(sigma * np.einsum("ij,ij->j", U, AV)))
    G = (U.T @ U) * sigma[None, :]
    H = (V.T @ V) * sigma[None, :]
    quad = float(np.sum(G * H.T))
    e2 = max(a2 - 2.0 * cross + quad, 0.0)
    return math.sqrt(e2 / a2) if a2 > 0 else 0.0


def ls_residual(A: sp.spmatrix, Z, Y) -> float:
    """||A Z - Y||_F / ||Y||_F (Application 1's least-squares objective)."""
    R = sp.csr_matrix(A) @ Z - Y
    ny = float(np.linalg.norm(Y))
    return float(np.linalg.norm(R)) / ny if ny > 0 else float(np.linalg.norm(R))


def orthonormality_error(Q, sigma=None, m=None, n=None) -> float:
    """max |Q^T Q - I| over the columns whose singular value is above the pinv threshold."""
    if sigma is not None:
        m = Q.shape[0] if m is None else m
        n = Q.shape[0] if n is None else n
        keep = sigma_pinv(sigma, m, n) > 0
        Q = Q[:, keep]
    if Q.shape[1] == 0:
        return 0.0
    return float(np.max(np.abs(Q.T @ Q - np.eye(Q.shape[1]))))
