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


def compare_svd(prob, U, S, V, ores, sigma_rtol=SIGMA_RTOL, product_rtol=PRODUCT_RTOL,
                recon_atol=RECON_ATOL, orth_atol=ORTH_ATOL):
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
    return ok, out


def compare_apply(prob, Z, ores, rtol=Z_RTOL):
    Zo = oracle.pinv_apply(ores.U, ores.sigma, ores.V, prob.Y, prob.m, prob.n)
    err = float(np.linalg.norm(Z - Zo) / max(np.linalg.norm(Zo), 1e-300))
    A = sp.csr_matrix((prob.data, prob.indices, prob.indptr), shape=(prob.m, prob.n))
    ls_g = oracle.ls_residual(A, Z, prob.Y)
    ls_o = oracle.ls_residual(A, Zo, prob.Y)
    return err <= rtol, {"Z": err, "ls_gpu": ls_g, "ls_oracle": ls_o,
                         "ls_rel": abs(ls_g - ls_o) / max(ls_o, 1e-300)}
