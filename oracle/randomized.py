"""Oracle of the truncated inner solver for the two incremental updates (Section 3.3: for a
low target rank the paper computes the update's SVD with a randomized method with power
iterations, oversampling 5 and 11 iterations, instead of the standard SVD).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the benchmark's
CPU-baseline leg, never by the product path.

The method written out here is randomized subspace iteration for the leading right
singular subspace of a formed matrix M (Halko, Martinsson & Tropp 2011, "randomized
subspace iteration"): a Gaussian test matrix Omega (q x k, k = t + oversample) gives
Y = M^T M Omega; each of `iters` power iterations orthonormalizes Y and applies M^T M again;
the final orthonormal basis Q (q x k) gives the thin SVD of the formed M Q, whose leading t
triplets are the result: sigma, V = Q W_t, U = the left factor. In exact arithmetic the
subspace span(Y) does not depend on how Y is orthonormalized between iterations.

Omega comes from a counter-based generator, so that any implementation can draw the same
numbers: Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC 2011) with key (seed, stream),
counter (pair index low word, high word, 0, 0); its four outputs make two 53-bit uniforms
u1 in (0, 1] and u2 in [0, 1), and the Box-Muller transform gives the normals
sqrt(-2 ln u1) cos(2 pi u2) for the even element and sqrt(-2 ln u1) sin(2 pi u2) for the
odd element of the pair (elements in row-major order).

The column update's test matrix multiplies the columns of X3 = [U2 Sigma2, T], and the row
update fixes each column of U2 and V2 only up to sign; a flipped column is a different draw.
So before a randomized column update both sides fix those signs: each right singular vector
v of the row update (with its left partner) is negated unless its entry of largest magnitude
(the first such entry on ties) is positive.

Readings: the paper's frPCA normalizes with an LU factorization between power iterations;
this oracle uses a QR factorization (same subspace in exact arithmetic). The branch is
taken for an update whose target rank t satisfies t < ceil(0.3 q) (q: the order of the
update's right factor; the paper states the rule as r < ceil(0.3 n)) and t + oversample < q;
the row update draws from stream 0, the column update from stream 1.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

PHILOX_M0 = np.uint64(0xD2511F53)
PHILOX_M1 = np.uint64(0xCD9E8D57)
PHILOX_W0 = 0x9E3779B9
PHILOX_W1 = 0xBB67AE85
MASK32 = np.uint64(0xFFFFFFFF)


def philox4x32_10(ctr, key):
    """Philox4x32 with 10 rounds. ctr: four uint32 arrays of equal shape; key: two ints.
    Returns the four output words (uint32 arrays)."""
    x0, x1, x2, x3 = (np.asarray(c, dtype=np.uint64) & MASK32 for c in ctr)
    k0, k1 = int(key[0]) & 0xFFFFFFFF, int(key[1]) & 0xFFFFFFFF
    for rnd in range(10):
        if rnd > 0:
            k0 = (k0 + PHILOX_W0) & 0xFFFFFFFF
            k1 = (k1 + PHILOX_W1) & 0xFFFFFFFF
        p0 = PHILOX_M0 * x0
        p1 = PHILOX_M1 * x2
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK32
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK32
        x0, x1, x2, x3 = (hi1 ^ x1 ^ np.uint64(k0), lo1, hi0 ^ x3 ^ np.uint64(k1), lo0)
    return tuple(x.astype(np.uint32) for x in (x0, x1, x2, x3))


def gaussian(rows: int, cols: int, seed: int, stream: int) -> np.ndarray:
    """rows x cols standard normals (row-major element e uses pair e // 2)."""
    count = rows * cols
    pairs = (count + 1) // 2
    idx = np.arange(pairs, dtype=np.uint64)
    zero = np.zeros(pairs, dtype=np.uint64)
    x0, x1, x2, x3 = philox4x32_10((idx & MASK32, idx >> np.uint64(32), zero, zero), (seed, stream))
    two26, two53 = 67108864.0, 2.0 ** -53
    u1 = ((x0 >> 5).astype(np.float64) * two26 + (x1 >> 6).astype(np.float64) + 1.0) * two53
    u2 = ((x2 >> 5).astype(np.float64) * two26 + (x3 >> 6).astype(np.float64)) * two53
    rad = np.sqrt(-2.0 * np.log(u1))
    ang = 2.0 * math.pi * u2
    z = np.empty(2 * pairs, dtype=np.float64)
    z[0::2] = rad * np.cos(ang)
    z[1::2] = rad * np.sin(ang)
    return z[:count].reshape(rows, cols)


@dataclasses.dataclass(frozen=True)
class InnerSolver:
    """mode 0: exact truncated SVD everywhere; 1: randomized where t < ceil(0.3 q);
    2: randomized for every update with t + oversample < q."""
    mode: int = 0
    oversample: int = 5
    iters: int = 11
    seed: int = 0


def use_randomized(inner: InnerSolver | None, t: int, q: int) -> bool:
    if inner is None or inner.mode == 0 or t <= 0:
        return False
    if t + inner.oversample >= q:
        return False
    return inner.mode == 2 or t < int(math.ceil(0.3 * float(q)))


def sign_convention(V: np.ndarray) -> np.ndarray:
    """+1 or -1 per column: the sign that makes the column's largest-magnitude entry (the
    first on ties) positive."""
    if V.shape[0] == 0:
        return np.ones(V.shape[1])
    lead = V[np.argmax(np.abs(V), axis=0), np.arange(V.shape[1])]
    return np.where(lead < 0, -1.0, 1.0)


def rsvd_right(M: np.ndarray, t: int, oversample: int, iters: int, seed: int, stream: int):
    """Leading t singular triplets of M (p x q) by randomized subspace iteration on its
    right singular subspace. Returns (U (p x t), sigma (t), V (q x t))."""
    q = M.shape[1]
    k = min(t + oversample, q)
    omega = gaussian(q, k, seed, stream)
    Y = M.T @ (M @ omega)
    for _ in range(iters):
        Q, _ = np.linalg.qr(Y)
        Y = M.T @ (M @ Q)
    Q, _ = np.linalg.qr(Y)
    Uc, sig, Wt = np.linalg.svd(M @ Q, full_matrices=False)
    return Uc[:, :t].copy(), sig[:t].copy(), Q @ Wt[:t].T
