"""Writes tests/golden/<workload>_reference.npz: quantities of the oracle's result on a full-size
workload that a GPU test can compare without re-running the oracle (which takes minutes there).
A workload is a named configuration (c3, c5) or instance i of the 64-matrix batched workload
(c4:i, written as c4_i_reference.npz).

Only oracle/ and synth/ are called. Stored: the r singular values, the reconstruction error
||A - U S V^T||_F / ||A||_F, the least-squares residual ||A Z - Y||_F / ||Y||_F, Z at 16 seeded
rows, and, at 64 seeded rows of U and 64 seeded rows of V, the rank-r products
(U S V^T P)[rows] and (V S U^T Q)[rows] for four fixed Gaussian probe columns P (n x 4) and
Q (m x 4) drawn from a seeded generator (invariant under the sign freedom of the singular
vectors).

    python tests/golden/make_large_reference.py c3
    python tests/golden/make_large_reference.py c4:23
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from synth import CONFIGS, make_problem, sample_batch_configs  # noqa: E402

PROBE_SEED = 77


def sample_rows(count, size, seed):
    return np.sort(np.random.default_rng(seed).choice(size, size=min(count, size), replace=False))


def probes(m, n):
    g = np.random.default_rng(PROBE_SEED)
    return g.standard_normal((n, 4)), g.standard_normal((m, 4))


def workload(name):
    """(config, file stem) of a named workload or of batched-workload instance c4:i."""
    if name.startswith("c4:"):
        i = int(name.split(":")[1])
        return sample_batch_configs(64)[i], f"c4_{i}"
    return CONFIGS[name], name


def main(name):
    cfg, stem = workload(name)
    prob = make_problem(cfg)
    t0 = time.time()
    res = oracle.fastpi_svd(prob.m, prob.n, prob.indptr, prob.indices, prob.data, cfg.alpha, cfg.k)
    t1 = time.time()
    Z = oracle.pinv_apply(res.U, res.sigma, res.V, prob.Y, prob.m, prob.n)
    import scipy.sparse as sp
    A = sp.csr_matrix((prob.data, prob.indices, prob.indptr), shape=(prob.m, prob.n))
    P, Q = probes(prob.m, prob.n)
    rows_u = sample_rows(64, prob.m, PROBE_SEED + 1)
    rows_v = sample_rows(64, prob.n, PROBE_SEED + 2)
    rows_z = sample_rows(16, prob.n, PROBE_SEED + 3)
    usvp = (res.U[rows_u] * res.sigma[None, :]) @ (res.V.T @ P)
    vsuq = (res.V[rows_v] * res.sigma[None, :]) @ (res.U.T @ Q)
    out = os.path.join(HERE, f"{stem}_reference.npz")
    np.savez_compressed(out, sigma=res.sigma, recon=oracle.recon_error(A, res.U, res.sigma, res.V),
                        ls=oracle.ls_residual(A, Z, prob.Y), rows_u=rows_u, rows_v=rows_v, rows_z=rows_z,
                        usvp=usvp, vsuq=vsuq, z_rows=Z[rows_z], probe_seed=PROBE_SEED, r=res.r,
                        oracle_seconds=t1 - t0)
    print(f"{name}: r={res.r} oracle {t1 - t0:.0f} s -> {out}")


if __name__ == "__main__":
    for arg in (sys.argv[1:] or ["c3"]):
        main(arg)
