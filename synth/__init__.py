"""Seeded synthetic inputs for the FastPI hot path.

This module is shared by the CPU oracle, the tests and the benchmark. It only
draws random numbers and lays them out; it holds none of the method's
arithmetic (no reordering, no SVD, no products).

The paper measures on four multi-label text datasets (Section 4, Table 3) that
are not available here. These generators stand in for them: a sparse feature
matrix whose bipartite graph has power-law degrees on both the instance and the
feature side (the skew shown in Fig. 1), positive tf-idf-like values, and a
sparse binary label matrix (Application 1).

Recipe (every step uses one ``numpy.random.default_rng(seed)`` stream, PCG64,
in this order):

1. target nnz = round(density * m * n);
2. Chung-Lu weights w_T[i] = (i+1)^(-1/(gamma-1)), w_F[j] likewise;
3. draw (row, col) pairs i.i.d. by inverse CDF from the two weight vectors in
   rounds, keeping the first occurrence of every distinct pair in draw order,
   until `target nnz` distinct pairs exist;
4. relabel rows and columns with two seeded permutations (row permutation drawn
   first) so that index and degree are uncorrelated;
5. values in CSR order: uniform(0,1] as 1-U[0,1), or lognormal(0,1) as exp(N(0,1));
6. labels Y (m x L) i.i.d. Bernoulli(p) in {0,1}, drawn row-major in chunks.

The evaluation loop of Application 1 needs labels that the features predict, which i.i.d.
labels are not. ``make_labelled_problem`` draws, from its own stream (seed + 1):
1. the feature matrix by steps 1-5 above;
2. for each label, ``triggers`` distinct trigger features uniformly at random; the label is
   positive on every row that stores one of them;
3. each such positive is dropped with probability ``drop``;
4. ``round(noise * planted)`` positives at uniform (row, label) positions are added;
5. the rows are split by a random permutation: the first ``round(test_frac * m)`` go to the
   test set (kept in increasing row order), the rest to the training set.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = ["Config", "CONFIGS", "Problem", "make_problem", "make_csr", "make_labels",
           "sample_batch_configs", "small_config", "CsrPart", "LabelledProblem",
           "make_labelled_problem", "csr_rows"]


@dataclasses.dataclass(frozen=True)
class Config:
    name: str
    m: int
    n: int
    density: float
    gamma: float
    values: str          # "uniform" or "lognormal"
    L: int
    p_label: float
    alpha: float
    seed: int
    k: float = 0.01      # hub selection ratio (Table 3 uses 0.01 for every dataset)


CONFIGS = {
    "c1": Config("c1", 2000, 500, 0.01, 2.1, "uniform", 50, 0.05, 0.3, 1000),
    "c2": Config("c2", 20000, 2000, 0.005, 2.0, "lognormal", 200, 0.02, 0.2, 2000),
    "c3": Config("c3", 100000, 5000, 0.002, 1.9, "lognormal", 1000, 0.005, 0.1, 3000),
    "c5": Config("c5", 300000, 10000, 0.0005, 1.8, "lognormal", 2000, 0.002, 0.1, 5000),
}


def small_config(m, n, density, gamma=2.0, values="lognormal", L=8, p_label=0.1,
                 alpha=0.3, seed=0, k=0.01, name="small"):
    return Config(name, m, n, density, gamma, values, L, p_label, alpha, seed, k)


def sample_batch_configs(count=64, base_seed=4000):
    """Instances of the batched workload: m log-uniform in [5k, 50k], n log-uniform
    in [500, 4k], density U[0.001, 0.01], gamma U[1.8, 2.3], L U{100..500},
    p_label = 4/L, lognormal values, alpha 0.2; instance i uses seed base_seed+i."""
    out = []
    for i in range(count):
        rng = np.random.default_rng(base_seed + i)
        m = int(round(math.exp(rng.uniform(math.log(5000), math.log(50000)))))
        n = int(round(math.exp(rng.uniform(math.log(500), math.log(4000)))))
        density = float(rng.uniform(0.001, 0.01))
        gamma = float(rng.uniform(1.8, 2.3))
        L = int(rng.integers(100, 501))
        out.append(Config(f"b{i}", m, n, density, gamma, "lognormal", L, 4.0 / L, 0.2,
                          base_seed + i))
    return out


@dataclasses.dataclass
class Problem:
    cfg: Config
    indptr: np.ndarray   # int64[m+1]
    indices: np.ndarray  # int32[nnz], sorted and unique within each row
    data: np.ndarray     # float64[nnz]
    Y: np.ndarray | None  # float64[m, L] in {0, 1}

    @property
    def m(self):
        return self.cfg.m

    @property
    def n(self):
        return self.cfg.n

    @property
    def nnz(self):
        return int(self.indptr[-1])


def _powerlaw_weights(size, gamma):
    expo = -1.0 / (gamma - 1.0)
    return np.power(np.arange(1, size + 1, dtype=np.float64), expo)


def _draw(rng, cdf, count):
    u = rng.random(count)
    idx = np.searchsorted(cdf, u * cdf[-1], side="right")
    return np.minimum(idx, cdf.size - 1)


def make_csr(cfg: Config, rng: np.random.Generator):
    m, n = cfg.m, cfg.n
    target = int(round(cfg.density * m * n))
    target = min(target, m * n)
    cdf_T = np.cumsum(_powerlaw_weights(m, cfg.gamma))
    cdf_F = np.cumsum(_powerlaw_weights(n, cfg.gamma))
    keys = np.empty(0, dtype=np.int64)
    uniq = np.empty(0, dtype=np.int64)
    while uniq.size < target:
        need = target - uniq.size
        batch = int(need * 1.25) + 64
        rows = _draw(rng, cdf_T, batch)
        cols = _draw(rng, cdf_F, batch)
        keys = np.concatenate([keys, rows.astype(np.int64) * n + cols])
        uniq, first = np.unique(keys, return_index=True)
        # keep first occurrences in draw order
        keys = keys[np.sort(first)]
        uniq = keys
    keys = keys[:target]
    permT = rng.permutation(m)
    permF = rng.permutation(n)
    rows = permT[keys // n]
    cols = permF[keys % n]
    order = np.lexsort((cols, rows))
    rows = rows[order]
    cols = cols[order]
    indptr = np.zeros(m + 1, dtype=np.int64)
    np.add.at(indptr, rows + 1, 1)
    indptr = np.cumsum(indptr)
    indices = cols.astype(np.int32)
    if cfg.values == "uniform":
        data = 1.0 - rng.random(target)
    elif cfg.values == "lognormal":
        data = np.exp(rng.standard_normal(target))
    else:
        raise ValueError(f"unknown value distribution {cfg.values!r}")
    return indptr, indices, data.astype(np.float64)


def make_labels(cfg: Config, rng: np.random.Generator, chunk_rows=8192):
    Y = np.empty((cfg.m, cfg.L), dtype=np.float64)
    for r0 in range(0, cfg.m, chunk_rows):
        r1 = min(cfg.m, r0 + chunk_rows)
        Y[r0:r1] = (rng.random((r1 - r0, cfg.L)) < cfg.p_label)
    return Y


def make_problem(cfg: Config | str, with_labels=True) -> Problem:
    if isinstance(cfg, str):
        cfg = CONFIGS[cfg]
    rng = np.random.default_rng(cfg.seed)
    indptr, indices, data = make_csr(cfg, rng)
    Y = make_labels(cfg, rng) if with_labels else None
    return Problem(cfg, indptr, indices, data, Y)


def csr_rows(indptr, indices, data, rows):
    """The CSR of the given rows (in the given order) of a CSR matrix."""
    rows = np.asarray(rows, np.int64)
    lens = indptr[rows + 1] - indptr[rows]
    out_ptr = np.zeros(rows.size + 1, np.int64)
    np.cumsum(lens, out=out_ptr[1:])
    src = np.repeat(indptr[rows] - out_ptr[:-1], lens) + np.arange(int(out_ptr[-1]), dtype=np.int64)
    return out_ptr, indices[src], (data[src] if data is not None else None)


@dataclasses.dataclass
class CsrPart:
    """Rows of a feature matrix with their labels (CSR, values 1)."""
    m: int
    n: int
    indptr: np.ndarray
    indices: np.ndarray
    data: np.ndarray
    y_indptr: np.ndarray
    y_indices: np.ndarray
    rows: np.ndarray      # row ids in the full matrix

    @property
    def nnz(self):
        return int(self.indptr[-1])

    @property
    def y_nnz(self):
        return int(self.y_indptr[-1])


@dataclasses.dataclass
class LabelledProblem:
    cfg: Config
    L: int
    train: CsrPart
    test: CsrPart


def make_labelled_problem(cfg: Config | str, test_frac=0.1, triggers=3, drop=0.1,
                          noise=0.1) -> LabelledProblem:
    if isinstance(cfg, str):
        cfg = CONFIGS[cfg]
    rng = np.random.default_rng(cfg.seed + 1)
    indptr, indices, data = make_csr(cfg, rng)
    m, n, L = cfg.m, cfg.n, cfg.L
    # rows of every feature (CSC pattern)
    rows_of = np.repeat(np.arange(m, dtype=np.int64), np.diff(indptr))
    order = np.argsort(indices, kind="stable")
    col_ptr = np.zeros(n + 1, np.int64)
    np.cumsum(np.bincount(indices, minlength=n), out=col_ptr[1:])
    col_rows = rows_of[order]
    keys = []
    for lab in range(L):
        trig = rng.choice(n, size=min(triggers, n), replace=False)
        r = np.unique(np.concatenate([col_rows[col_ptr[j]:col_ptr[j + 1]] for j in trig]))
        keys.append(r * L + lab)
    keys = np.concatenate(keys) if keys else np.zeros(0, np.int64)
    keys = keys[rng.random(keys.size) >= drop]
    extra = rng.integers(0, m * L, size=int(round(noise * keys.size)), dtype=np.int64)
    keys = np.unique(np.concatenate([keys, extra]))
    y_rows, y_cols = keys // L, (keys % L).astype(np.int32)
    y_ptr = np.zeros(m + 1, np.int64)
    np.cumsum(np.bincount(y_rows, minlength=m), out=y_ptr[1:])
    perm = rng.permutation(m)
    nt = int(round(test_frac * m))
    parts = []
    for sel in (np.sort(perm[nt:]), np.sort(perm[:nt])):
        a_ptr, a_idx, a_val = csr_rows(indptr, indices, data, sel)
        b_ptr, b_idx, _ = csr_rows(y_ptr, y_cols, None, sel)
        parts.append(CsrPart(int(sel.size), n, a_ptr, a_idx, a_val, b_ptr, b_idx, sel))
    return LabelledProblem(cfg, L, parts[0], parts[1])
