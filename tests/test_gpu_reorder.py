"""GPU reordering (Algorithm 2 on the device) through the C ABI: the permutation, the block
table and the shape report must equal the host reordering's bit for bit (itself pinned to the
oracle and the paper's toy graph in the CPU tests), on the toy graph, random small graphs,
degenerate patterns, stored zeros, the benchmark workloads up to 300000 x 10000, and a few
matrices of the batched workload; a plan built with the GPU reordering equals the host plan;
malformed device CSR input is rejected before any reordering kernel runs."""
import json
import os
import sys
import time

import numpy as np
import pytest
import scipy.sparse as sp

from synth import CONFIGS, make_problem, sample_batch_configs

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def env():
    import torch

    import paper_2011_04235_amd as fp
    fp.load()
    return torch, fp, fp.Handle(0)


def dev_t(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(torch.device("cuda", 0))


def both(torch, fp, h, m, n, indptr, indices, data, k):
    indptr = np.ascontiguousarray(indptr, np.int64)
    indices = np.ascontiguousarray(indices, np.int32)
    data = None if data is None else np.ascontiguousarray(data, np.float64)
    t0 = time.perf_counter()
    host = fp.reorder(m, n, indptr, indices, data, k=k)
    t1 = time.perf_counter()
    gpu = h.reorder(m, n, dev_t(torch, indptr), dev_t(torch, indices),
                    None if data is None else dev_t(torch, data), k=k)
    t2 = time.perf_counter()
    return host, gpu, t1 - t0, t2 - t1


def same(host, gpu):
    return (np.array_equal(host[0], gpu[0]) and np.array_equal(host[1], gpu[1])
            and np.array_equal(host[2], gpu[2]) and host[3] == gpu[3])


def test_toy_graph(env):
    torch, fp, h = env
    g = json.load(open(os.path.join(ROOT, "tests", "golden", "toy_fig2.json")))
    e = np.asarray(g["edges"])
    A = sp.csr_matrix((np.ones(len(e)), (e[:, 0], e[:, 1])), shape=(g["m"], g["n"]))
    A.sort_indices()
    host, gpu, _, _ = both(torch, fp, h, g["m"], g["n"], A.indptr, A.indices, A.data, g["k"])
    assert gpu[0].tolist() == g["expected"]["piT"] and gpu[1].tolist() == g["expected"]["piF"]
    assert gpu[2].tolist() == g["expected"]["blocks"]
    assert same(host, gpu)


@pytest.mark.parametrize("seed", range(12))
def test_random_small_graphs(env, seed):
    torch, fp, h = env
    rng = np.random.default_rng(900 + seed)
    m, n = int(rng.integers(1, 120)), int(rng.integers(1, 90))
    M = rng.random((m, n)) < rng.uniform(0.01, 0.3)
    A = sp.csr_matrix(M.astype(np.float64))
    k = float(rng.choice([0.01, 0.05, 0.1, 0.3]))
    say(f"random {m}x{n} nnz={A.nnz} k={k}")
    host, gpu, _, _ = both(torch, fp, h, m, n, A.indptr, A.indices, A.data, k)
    assert same(host, gpu)


def test_degenerate_patterns(env):
    torch, fp, h = env
    cases = {
        "empty": (50, 20, np.zeros(51), np.zeros(0), np.zeros(0)),
        "one-row": (1, 30, [0, 5], [1, 4, 9, 17, 29], np.arange(1.0, 6.0)),
        "one-column": (40, 1, np.concatenate([[0], np.cumsum(np.arange(40) % 3 == 0)]), np.zeros(14),
                       np.linspace(1, 2, 14)),
        "dense": (12, 7, np.arange(0, 85, 7), np.tile(np.arange(7), 12), np.ones(84)),
        "diagonal": (30, 30, np.arange(31), np.arange(30), np.linspace(1, 3, 30)),
    }
    for name, (m, n, ip, ix, dv) in cases.items():
        say(f"degenerate {name}")
        host, gpu, _, _ = both(torch, fp, h, m, n, ip, ix, dv, 0.1)
        assert same(host, gpu), name


def test_stored_zeros_are_not_edges(env):
    torch, fp, h = env
    p = make_problem("c1")
    data = p.data.copy()
    data[::7] = 0.0
    host, gpu, _, _ = both(torch, fp, h, p.m, p.n, p.indptr, p.indices, data, 0.01)
    assert same(host, gpu)
    nozero, gpu_nv, _, _ = both(torch, fp, h, p.m, p.n, p.indptr, p.indices, None, 0.01)
    assert same(nozero, gpu_nv)
    assert not np.array_equal(gpu[0], gpu_nv[0])


@pytest.mark.parametrize("name", ["c1", "c2", "c3", "c5"])
def test_workloads(env, name):
    torch, fp, h = env
    p = make_problem(name)
    say(f"{name} {p.m}x{p.n} nnz={p.nnz}")
    host, gpu, th, tg = both(torch, fp, h, p.m, p.n, p.indptr, p.indices, p.data, CONFIGS[name].k)
    say(f"  host {th * 1e3:.1f} ms, GPU {tg * 1e3:.1f} ms, T_it {gpu[3]['T_it']}, blocks {len(gpu[2])}")
    assert same(host, gpu)
    # the components come from concurrent unions: every repetition must give the same result
    args = (p.m, p.n, dev_t(torch, p.indptr), dev_t(torch, p.indices), dev_t(torch, p.data))
    for _ in range(3):
        assert same(host, h.reorder(*args, k=CONFIGS[name].k))


def test_batched_workload_instances(env):
    torch, fp, h = env
    for c in sample_batch_configs(64)[:6]:
        p = make_problem(c)
        host, gpu, _, _ = both(torch, fp, h, p.m, p.n, p.indptr, p.indices, p.data, c.k)
        assert same(host, gpu), c.name


def test_gpu_planned_matches_host_plan(env):
    torch, fp, h = env
    p = make_problem("c2")
    a = fp.Plan(p.m, p.n, p.indptr, p.indices, p.data, alpha=0.2, k=0.01)
    b = fp.Plan(p.m, p.n, p.indptr, p.indices, p.data, alpha=0.2, k=0.01, gpu=h)
    assert a.info == b.info
    for x, y in zip(a.permutation(), b.permutation()):
        assert np.array_equal(x, y)
    assert np.array_equal(a.blocks(), b.blocks()) and np.array_equal(a.block_ranks(), b.block_ranks())


def test_malformed_device_csr_is_rejected(env):
    torch, fp, h = env
    ok_ip, ok_ix = np.array([0, 2, 3]), np.array([0, 2, 1])
    bad = {
        "column out of range": (ok_ip, np.array([0, 5, 1])),
        "columns not increasing": (ok_ip, np.array([2, 0, 1])),
        "rowptr not monotone": (np.array([0, 3, 2]), ok_ix),
        "rowptr end": (np.array([0, 2, 2]), ok_ix),
    }
    for name, (ip, ix) in bad.items():
        say(f"rejects: {name}")
        with pytest.raises(fp.FastPIError):
            h.reorder(2, 3, dev_t(torch, ip.astype(np.int64)), dev_t(torch, ix.astype(np.int32)), None, k=0.1)
    with pytest.raises(fp.FastPIError):
        h.reorder(2, 3, dev_t(torch, ok_ip.astype(np.int64)), dev_t(torch, ok_ix.astype(np.int32)),
                  dev_t(torch, np.array([1.0, np.inf, 2.0])), k=0.1)


@pytest.mark.parametrize("name", ["c3", "c5"])
def test_large_workloads_equal_the_oracle(env, name):
    """The GPU reordering at 100000 x 5000 and 300000 x 10000 against the oracle's Algorithm 2
    directly (not through the host library): permutations, block table and split sizes bit
    for bit."""
    torch, fp, h = env
    import oracle
    cfg = CONFIGS[name]
    p = make_problem(cfg, with_labels=False)
    say(f"GPU reordering vs oracle at {name} {p.m}x{p.n}")
    gpu = h.reorder(p.m, p.n, dev_t(torch, p.indptr), dev_t(torch, p.indices), dev_t(torch, p.data), k=cfg.k)
    R = oracle.reorder(p.m, p.n, p.indptr, p.indices, cfg.k)
    assert np.array_equal(gpu[0], R.piT) and np.array_equal(gpu[1], R.piF)
    assert np.array_equal(gpu[2], R.blocks)
    split = gpu[3]
    assert (split["m1"], split["n1"], split["m2"], split["n2"], split["T_it"]) == \
        (R.m1, R.n1, R.m2, R.n2, R.iterations)
