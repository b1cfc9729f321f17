"""GPU edge cases through the C ABI: degenerate inputs of the method (empty matrix, a single
row or column, a matrix with no spoke block left, all-singleton blocks), at alpha < 1 and
alpha = 1, alone and mixed into one batch with an ordinary matrix. Each is compared with the
oracle where A is not zero; the empty matrix must give zero singular values and a zero Z
without an error."""
import sys

import numpy as np
import pytest

import oracle
from parity import compare_apply, compare_svd, to_np

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


class P:
    """Minimal problem record with the fields the parity helpers read."""

    def __init__(self, m, n, indptr, indices, data, L=3, seed=0):
        self.m, self.n = m, n
        self.indptr = np.ascontiguousarray(indptr, np.int64)
        self.indices = np.ascontiguousarray(indices, np.int32)
        self.data = np.ascontiguousarray(data, np.float64)
        self.Y = (np.random.default_rng(seed).random((m, L)) < 0.3).astype(np.float64)

    @property
    def nnz(self):
        return int(self.indptr[-1])


def cases():
    rng = np.random.default_rng(0)
    D = rng.random((12, 7)) + 0.1
    return {
        "empty-50x20": P(50, 20, np.zeros(51), np.zeros(0), np.zeros(0)),
        "one-row-1x30": P(1, 30, [0, 5], [1, 4, 9, 17, 29], np.arange(1.0, 6.0)),
        "one-column-40x1": P(40, 1, np.concatenate([[0], np.cumsum(np.arange(40) % 3 == 0)]),
                             np.zeros(14), np.linspace(1, 2, 14)),
        "dense-12x7": P(12, 7, np.arange(0, 85, 7), np.tile(np.arange(7), 12), D.ravel()),
        "diagonal-30x30": P(30, 30, np.arange(31), np.arange(30), np.linspace(1, 3, 30)),
    }


@pytest.fixture(scope="module")
def env():
    import torch

    import paper_2011_04235_amd as fp
    fp.load()
    return torch, fp


def run(fp, torch, p, alpha, h):
    dev = torch.device("cuda", 0)
    plan = fp.Plan(p.m, p.n, p.indptr, p.indices, p.data, alpha=alpha, k=0.1)
    h.upload_plan(plan)
    U, S, V = h.svd(*(torch.from_numpy(a).to(dev) for a in (p.indptr, p.indices, p.data)))
    Z = h.apply(U, S, V, torch.from_numpy(p.Y).to(dev))
    h.sync()
    return plan, to_np(U), to_np(S), to_np(V), to_np(Z)


@pytest.mark.parametrize("alpha", [0.3, 1.0])
@pytest.mark.parametrize("name", list(cases()))
def test_degenerate_inputs(env, name, alpha):
    torch, fp = env
    p = cases()[name]
    say(f"edge {name} alpha={alpha}")
    h = fp.Handle(0)
    plan, U, S, V, Z = run(fp, torch, p, alpha, h)
    ores = oracle.fastpi_svd(p.m, p.n, p.indptr, p.indices, p.data, alpha, 0.1)
    assert S.shape == (ores.r,) == (plan.r,)
    assert np.all(np.isfinite(U)) and np.all(np.isfinite(V)) and np.all(np.isfinite(Z))
    if p.nnz == 0:
        assert np.all(S == 0.0) and np.all(Z == 0.0)
        return
    ok, info = compare_svd(p, U, S, V, ores)
    say(f"  {info}")
    assert ok, info
    ok, zinfo = compare_apply(p, Z, ores)
    say(f"  {zinfo}")
    assert ok, zinfo


def test_degenerate_inputs_in_one_batch(env):
    torch, fp = env
    from synth import make_problem
    cs = cases()
    probs = [cs["empty-50x20"], cs["one-column-40x1"], make_problem("c1"), cs["dense-12x7"]]
    alphas = [0.3, 0.3, 0.3, 1.0]
    ks = [0.1, 0.1, 0.01, 0.1]
    say("batch of empty, one-column, 2000x500 and dense matrices")
    dev = torch.device("cuda", 0)
    h = fp.Handle(0)
    b = fp.Batch(h, [fp.Plan(p.m, p.n, p.indptr, p.indices, p.data, alpha=a, k=k)
                     for p, a, k in zip(probs, alphas, ks)])
    for graph in (False, True):
        b.set_graph(graph)
        out = b.svd([torch.from_numpy(p.data).to(dev) for p in probs])
        status, _ = b.sync()
        assert status == ["OK"] * len(probs), status
        for p, a, k, (U, S, V) in zip(probs, alphas, ks, out):
            U, S, V = to_np(U), to_np(S), to_np(V)
            if p.nnz == 0:
                assert np.all(S == 0.0)
                continue
            ores = oracle.fastpi_svd(p.m, p.n, p.indptr, p.indices, p.data, a, k)
            ok, info = compare_svd(p, U, S, V, ores)
            assert ok, (graph, info)
