"""Helpers for GPU-versus-oracle parity checks.

The singular vectors of a truncated SVD are fixed only up to sign (and rotation inside
repeated singular values), so results are compared through what is unique: the singular
values, the rank-r matrix U Sigma V^T (probed with random vectors), the regression solution
Z, the reconstruction error, and the orthonormality of U and V.

Tolerances (FP64 path), derived from the arithmetic: the device path obtains the truncated
factors from FP64 Gram matrices, whose eigenvalues carry an absolute error of about
q * eps * sigma_1^2, so a singular value sigma_i carries a relative error of about
q * eps * (sigma_1 / sigma_i)^2 (q <= 10^4, sigma_1 / sigma_r <= 10^2 on these inputs gives
~2e-8 in the worst case and ~1e-12 typically); vectors near a truncation cut move by about
eps / gap, with gaps >= 1e-3 here. Hence: sigma 1e-9 relative (sigma_i >= 1e-6 sigma_1),
the rank-r product and Z 1e-8 relative, the reconstruction error 1e-10 absolute (or, near an
exact reconstruction, its square within 64 eps: the trace formula resolves e only to about
sqrt(eps) there).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

import oracle

SIGMA_RTOL = 1e-9
PRODUCT_RTOL = 1e-8
Z_RTOL = 1e-8
RECON_ATOL = 1e-10
ORTH_ATOL = 1e-10

# mixed-precision gates (stated for the mixed form): sigma 1e-5 relative, the
# reconstruction error within 1e-5 of the oracle's, the regression residual 1e-4 relative
MIXED_SIGMA_RTOL = 1e-5
MIXED_RECON_ATOL = 1e-5
MIXED_LS_RTOL = 1e-4


def to_np(t):
    return t.detach().cpu().numpy()


def sigma_rel_err(s_gpu, s_or, floor=1e-6):
    s_gpu = np.asarray(s_gpu); s_or = np.asarray(s_or)
    assert s_gpu.shape == s_or.shape, (s_gpu.shape, s_or.shape)
    if s_or.size == 0:
        return 0.0
    keep = s_or >= floor * s_or[0]
    return float(np.max(np.abs(s_gpu[keep] - s_or[keep]) / s_or[keep])) if keep.any() else 0.0


def product_rel_err(U, S, V, Uo, So, Vo, seed=0, probes=8):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((V.shape[0], probes))
    a = U @ (S[:, None] * (V.T @ X))
    b = Uo @ (So[:, None] * (Vo.T @ X))
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def vector_elementwise_err(Q, Qo, sigma_full, r, q, slack=256.0, limit=1e-6):
    """Element-wise comparison of singular vectors, column by column, up to sign: for each
    column i < r whose squared singular value is separated from its neighbours in the final
    stage's spectrum (sigma_full: every singular value of the formed X3, descending) by a
    relative gap g_i, the computed vector may move by about q eps / g_i (q: the largest core
    order), so max|q_i -/+ q_i^o| / max|q_i^o| is checked against max(1e-9, slack q eps / g_i)
    on the columns where that bound is at most `limit`. Returns (worst err/bound ratio,
    columns checked)."""
    lam = np.asarray(sigma_full, dtype=np.float64) ** 2
    if r == 0 or lam.size == 0 or lam[0] <= 0:
        return 0.0, 0
    eps = np.finfo(np.float64).eps
    worst, checked = 0.0, 0
    for i in range(r):
        nb = []
        if i > 0:
            nb.append(abs(lam[i - 1] - lam[i]))
        if i + 1 < lam.size:
            nb.append(abs(lam[i] - lam[i + 1]))
        gap = min(nb) / lam[0] if nb else 1.0
        if lam[i] < 1e-12 * lam[0] or gap <= 0:
            continue
        bound = max(1e-9, slack * q * eps / gap)
        if bound > limit:
            continue
        a, b = Q[:, i], Qo[:, i]
        j = int(np.argmax(np.abs(b)))
        sgn = 1.0 if a[j] * b[j] >= 0 else -1.0
        err = float(np.max(np.abs(sgn * a - b)) / max(np.max(np.abs(b)), 1e-300))
        worst = max(worst, err / bound)
        checked += 1
    return worst, checked


def compare_svd(prob, U, S, V, ores, sigma_rtol=SIGMA_RTOL, product_rtol=PRODUCT_RTOL,
                recon_atol=RECON_ATOL, orth_atol=ORTH_ATOL, elementwise=None):
    A = sp.csr_matrix((prob.data, prob.indices, prob.indptr), shape=(prob.m, prob.n))
    out = {}
    out["sigma"] = sigma_rel_err(S, ores.sigma)
    out["product"] = product_rel_err(U, S, V, ores.U, ores.sigma, ores.V)
    e_gpu = oracle.recon_error(A, U, S, V)
    e_or = oracle.recon_error(A, ores.U, ores.sigma, ores.V)
    out["recon"] = abs(e_gpu - e_or)
    out["recon_gpu"], out["recon_oracle"] = e_gpu, e_or
    # The trace formula gives e^2 = (||A||^2 - 2 tr(...) + tr(...)) / ||A||^2 with absolute
    # rounding of a few eps, so e itself is only known to ~sqrt(eps) when it is near 0 (an
    # exact-rank input): there the squared errors are compared instead.
    recon_ok = (out["recon"] <= recon_atol
                or abs(e_gpu * e_gpu - e_or * e_or) <= 64 * np.finfo(np.float64).eps)
    out["orthU"] = oracle.orthonormality_error(U, S, prob.m, prob.n)
    out["orthV"] = oracle.orthonormality_error(V, S, prob.m, prob.n)
    ok = (out["sigma"] <= sigma_rtol and out["product"] <= product_rtol
          and recon_ok and out["orthU"] <= orth_atol and out["orthV"] <= orth_atol)
    # element by element: U and V column by column up to sign where the spectrum's gaps fix
    # them (FP64 gates only: the mixed form's vectors carry FP32 rounding)
    if elementwise is None:
        elementwise = sigma_rtol <= SIGMA_RTOL
    if elementwise and ores.r > 0:
        q = max(ores.split.n1, ores.row.sigma.size + ores.split.n2, 1)
        wu, cu = vector_elementwise_err(U, ores.U, ores.col.full_sigma, ores.r, q)
        wv, cv = vector_elementwise_err(V, ores.V, ores.col.full_sigma, ores.r, q)
        out["vec_ratio"], out["vec_cols"] = max(wu, wv), cu + cv
        ok = ok and out["vec_ratio"] <= 1.0
    return ok, out


def compare_apply(prob, Z, ores, rtol=Z_RTOL):
    Zo = oracle.pinv_apply(ores.U, ores.sigma, ores.V, prob.Y, prob.m, prob.n)
    err = float(np.linalg.norm(Z - Zo) / max(np.linalg.norm(Zo), 1e-300))
    # element by element, relative to the largest entry
    err_max = float(np.max(np.abs(Z - Zo)) / max(np.max(np.abs(Zo)), 1e-300)) if Zo.size else 0.0
    A = sp.csr_matrix((prob.data, prob.indices, prob.indptr), shape=(prob.m, prob.n))
    ls_g = oracle.ls_residual(A, Z, prob.Y)
    ls_o = oracle.ls_residual(A, Zo, prob.Y)
    return err <= rtol and err_max <= rtol, {"Z": err, "Z_max": err_max, "ls_gpu": ls_g, "ls_oracle": ls_o,
                                             "ls_rel": abs(ls_g - ls_o) / max(ls_o, 1e-300)}
