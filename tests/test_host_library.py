"""CPU checks of the C-ABI library: it loads, exports every symbol the header declares,
and its host reordering is bit-exact with the oracle's."""
import ctypes
import json
import os
import re

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from synth import CONFIGS, make_problem, small_config

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fastpi.h")


@pytest.fixture(scope="module")
def fp():
    import paper_2011_04235_amd as fp
    fp.load()
    return fp


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(fastpi_[a-z_0-9]+)\s*\(", text)
    return sorted(set(names))


def test_library_exports_every_declared_symbol(fp):
    lib = ctypes.CDLL(fp.LIB_PATH)
    names = declared_functions()
    assert len(names) >= 18
    for name in names:
        assert hasattr(lib, name), name
    bound = {n for n, _, _ in fp.SIGNATURES}
    assert set(names) == bound, set(names) ^ bound


def test_target_rank_rule(fp):
    for a, x in [(0.3, 500), (0.2, 2000), (0.1, 5000), (0.1, 10000), (0.07, 13), (1.0, 7)]:
        assert fp.target_rank(a, x) == oracle.target_rank(a, x)


def _compare(fp, m, n, indptr, indices, data, k):
    piT, piF, blocks, info = fp.reorder(m, n, indptr, indices, data, k)
    R = oracle.reorder(m, n, indptr, indices, k)
    assert np.array_equal(piT, R.piT)
    assert np.array_equal(piF, R.piF)
    assert np.array_equal(blocks, R.blocks)
    assert (info["m1"], info["n1"], info["m2"], info["n2"], info["T_it"]) == \
        (R.m1, R.n1, R.m2, R.n2, R.iterations)


def test_toy_graph(fp):
    g = json.load(open(os.path.join(ROOT, "tests", "golden", "toy_fig2.json")))
    e = np.asarray(g["edges"])
    A = sp.csr_matrix((np.ones(len(e)), (e[:, 0], e[:, 1])), shape=(g["m"], g["n"]))
    A.sort_indices()
    piT, piF, blocks, info = fp.reorder(g["m"], g["n"], A.indptr, A.indices, A.data, g["k"])
    assert piT.tolist() == g["expected"]["piT"]
    assert piF.tolist() == g["expected"]["piF"]
    assert blocks.tolist() == g["expected"]["blocks"]


@pytest.mark.parametrize("seed", range(30))
def test_reorder_bitexact_random_small(fp, seed):
    rng = np.random.default_rng(500 + seed)
    m = int(rng.integers(1, 60)); n = int(rng.integers(1, 40))
    mask = rng.random((m, n)) < rng.uniform(0.02, 0.4)
    A = sp.csr_matrix(mask.astype(float))
    k = float(rng.choice([0.01, 0.05, 0.1, 0.3]))
    _compare(fp, m, n, A.indptr, A.indices, A.data, k)


@pytest.mark.parametrize("name", ["c1", "c2"])
def test_reorder_bitexact_configs(fp, name):
    p = make_problem(name, with_labels=False)
    _compare(fp, p.m, p.n, p.indptr, p.indices, p.data, p.cfg.k)


def test_reorder_bitexact_c3_shape(fp):
    p = make_problem(small_config(30000, 3000, 0.002, gamma=1.9, seed=77), with_labels=False)
    _compare(fp, p.m, p.n, p.indptr, p.indices, p.data, 0.01)


def test_stored_zeros_are_not_edges(fp):
    p = make_problem(small_config(300, 80, 0.05, seed=4), with_labels=False)
    data = p.data.copy()
    data[::7] = 0.0
    A = sp.csr_matrix((data, p.indices, p.indptr), shape=(p.m, p.n))
    B = A.copy()
    B.eliminate_zeros()
    a = fp.reorder(p.m, p.n, A.indptr, A.indices, A.data, 0.05)
    b = fp.reorder(p.m, p.n, B.indptr, B.indices, None, 0.05)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_plan_ranks_match_oracle(fp):
    p = make_problem("c1", with_labels=False)
    pl = fp.Plan(p.m, p.n, p.indptr, p.indices, p.data, alpha=0.3, k=0.01)
    res_blocks = oracle.reorder(p.m, p.n, p.indptr, p.indices, 0.01).blocks
    want = [min(oracle.target_rank(0.3, c), r, c) if r and c else 0 for (_, _, r, c) in res_blocks]
    assert pl.block_ranks().tolist() == want
    assert pl.s_b == sum(want)
    assert pl.s == min(oracle.target_rank(0.3, pl.n1), pl.s_b + pl.m2, pl.n1)
    assert pl.r == min(oracle.target_rank(0.3, min(p.m, p.n)), pl.s + pl.n2, p.m)


@pytest.mark.parametrize("bad", ["alpha0", "alpha_big", "k", "unsorted", "dup", "range", "nan",
                                 "rowptr"])
def test_plan_rejects_bad_input(fp, bad):
    p = make_problem(small_config(50, 20, 0.1, seed=1), with_labels=False)
    indptr, indices, data = p.indptr.copy(), p.indices.copy(), p.data.copy()
    alpha, k = 0.5, 0.05
    row = int(np.argmax(np.diff(indptr) >= 2))
    e0 = indptr[row]
    if bad == "alpha0":
        alpha = 0.0
    elif bad == "alpha_big":
        alpha = 1.5
    elif bad == "k":
        k = 1.0
    elif bad == "unsorted":
        indices[e0], indices[e0 + 1] = indices[e0 + 1], indices[e0]
    elif bad == "dup":
        indices[e0 + 1] = indices[e0]
    elif bad == "range":
        indices[e0] = 20
    elif bad == "nan":
        data[3] = np.nan
    elif bad == "rowptr":
        indptr[5] = indptr[6] + 1
    with pytest.raises(fp.FastPIError) as ei:
        fp.Plan(p.m, p.n, indptr, indices, data, alpha=alpha, k=k)
    expect = {"alpha0": "EINVAL", "alpha_big": "EINVAL", "k": "EINVAL", "unsorted": "ESHAPE",
              "dup": "ESHAPE", "range": "ESHAPE", "nan": "ENONFINITE", "rowptr": "ESHAPE"}[bad]
    assert ei.value.status == expect
