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


def graded_problem(m=400, n=60, decades=9.0, seed=5):
    """A sparse matrix whose singular values span about `decades` orders of magnitude: a
    random sparse pattern with U(0.5, 1] values plus a full diagonal (so every column is
    used), columns scaled by 10^(-decades * j / (n - 1)) in a random column order."""
    rng = np.random.default_rng(seed)
    mask = rng.random((m, n)) < 0.08
    mask[np.arange(n), np.arange(n)] = True
    dense = np.where(mask, 0.5 + 0.5 * rng.random((m, n)), 0.0)
    scale = 10.0 ** (-decades * rng.permutation(n) / (n - 1))
    dense *= scale[None, :]
    indptr = np.concatenate([[0], np.cumsum(mask.sum(1))])
    rows, cols = np.nonzero(mask)
    return P(m, n, indptr, cols, dense[rows, cols], L=4, seed=seed)


def test_graded_spectrum_full_rank_reports_the_gram_floor(env):
    """alpha = 1 on a matrix with singular values from 1 down to ~1e-9 of the largest: the
    Gram route resolves a singular value sigma to a relative error of about q eps
    (sigma_1 / sigma)^2, so values at or below 1e-7 sigma_1 come back as exactly 0 and
    fastpi_sync reports the warning WFLOOR. The resolved values match the oracle within that
    bound, and the pseudoinverse apply restricted to the well-resolved directions
    (sigma >= 1e-3 sigma_1) matches the oracle's on the same directions."""
    torch, fp = env
    p = graded_problem()
    say("graded spectrum 400x60, alpha=1")
    h = fp.Handle(0)
    dev = torch.device("cuda", 0)
    plan = fp.Plan(p.m, p.n, p.indptr, p.indices, p.data, alpha=1.0, k=0.05)
    h.upload_plan(plan)
    Ut, St, Vt = h.svd(*(torch.from_numpy(a).to(dev) for a in (p.indptr, p.indices, p.data)))
    code = h.sync()
    U, S, V = to_np(Ut), to_np(St), to_np(Vt)
    ores = oracle.fastpi_svd(p.m, p.n, p.indptr, p.indices, p.data, 1.0, 0.05)
    so = ores.sigma
    say(f"  status {code}, oracle sigma range {so[0]:.3e} .. {so[-1]:.3e}")
    assert so[-1] < 1e-8 * so[0]            # the input does reach under the floor
    assert code == "WFLOOR"
    q = max(plan.n1, plan.s + plan.n2)
    eps = np.finfo(np.float64).eps
    bound = np.maximum(1e-9, 8.0 * q * eps * (so[0] / so) ** 2)
    resolved = bound <= 1e-2
    rel = np.abs(S - so) / so
    say(f"  resolved {int(resolved.sum())} of {so.size}; worst ratio err/bound "
        f"{np.max(rel[resolved] / bound[resolved]):.3f}")
    assert np.all(rel[resolved] <= bound[resolved])
    assert np.all(S[so <= 1e-8 * so[0]] == 0.0)   # under the floor with margin: returned as 0
    # Z on the well-resolved directions, both sides restricted the same way
    def z_restricted(U, S, V, keep):
        return V[:, keep] @ ((U[:, keep].T @ p.Y) / S[keep, None])
    keep_g, keep_o = S >= 1e-3 * S[0], so >= 1e-3 * so[0]
    assert np.array_equal(keep_g, keep_o)
    Zg, Zo = z_restricted(U, S, V, keep_g), z_restricted(ores.U, so, ores.V, keep_o)
    err = float(np.max(np.abs(Zg - Zo)) / np.max(np.abs(Zo)))
    say(f"  restricted Z max rel err {err:.2e}")
    assert err <= 1e-6


def test_graded_spectrum_truncated_above_the_floor_meets_fp64_gates(env):
    """The same graded matrix at alpha = 0.3: every kept singular value lies far above the
    floor, no warning, and the FP64 gates hold against the oracle."""
    torch, fp = env
    p = graded_problem()
    say("graded spectrum 400x60, alpha=0.3")
    h = fp.Handle(0)
    plan, U, S, V, Z = run(fp, torch, p, 0.3, h)
    assert h.sync() == "OK"
    ores = oracle.fastpi_svd(p.m, p.n, p.indptr, p.indices, p.data, 0.3, 0.1)
    ok, info = compare_svd(p, U, S, V, ores)
    say(f"  {info}")
    assert ok, info
    ok, zinfo = compare_apply(p, Z, ores)
    assert ok, zinfo


def test_sweep_cap_reports_enoconv(env):
    """max_sweeps = 1 stops every Jacobi iteration after one sweep (a bounded exit: the
    kernels return normally); fastpi_sync and fastpi_batch_sync report ENOCONV."""
    torch, fp = env
    from synth import make_problem
    p = make_problem("c1")
    say("sweep cap 1 on 2000x500")
    dev = torch.device("cuda", 0)
    h = fp.Handle(0, max_sweeps=1)
    plan = fp.Plan(p.m, p.n, p.indptr, p.indices, p.data, alpha=0.3, k=0.01)
    h.upload_plan(plan)
    h.svd(*(torch.from_numpy(a).to(dev) for a in (p.indptr, p.indices, p.data)))
    with pytest.raises(fp.FastPIError) as ei:
        h.sync()
    assert ei.value.status == "ENOCONV"
    b = fp.Batch(h, [plan])
    b.svd([torch.from_numpy(p.data).to(dev)])
    status, sweeps = b.sync()
    assert status == ["ENOCONV"], status
    # the same handle without the cap converges
    h2 = fp.Handle(0)
    h2.upload_plan(plan)
    h2.svd(*(torch.from_numpy(a).to(dev) for a in (p.indptr, p.indices, p.data)))
    assert h2.sync() == "OK"


def test_workspace_cap_reports_enomem(env):
    """A workspace cap below what the plan needs fails the upload with ENOMEM (nothing is
    launched); a cap above it works."""
    torch, fp = env
    from synth import make_problem
    p = make_problem("c1")
    say("workspace cap on 2000x500")
    plan = fp.Plan(p.m, p.n, p.indptr, p.indices, p.data, alpha=0.3, k=0.01)
    h = fp.Handle(0, max_workspace_bytes=1 << 16)
    with pytest.raises(fp.FastPIError) as ei:
        h.upload_plan(plan)
    assert ei.value.status == "ENOMEM"
    h2 = fp.Handle(0, max_workspace_bytes=1 << 32)
    h2.upload_plan(plan)
    dev = torch.device("cuda", 0)
    h2.svd(*(torch.from_numpy(a).to(dev) for a in (p.indptr, p.indices, p.data)))
    assert h2.sync() == "OK"


def test_handle_destroyed_before_its_batch(env):
    """A handle destroyed while a batch created on it is alive releases the batch's device
    resources and detaches it: later batch calls fail with EINVAL, and destroying the batch
    afterwards is safe (the order in which a garbage collector finalises the two objects
    does not matter)."""
    torch, fp = env
    import ctypes
    from synth import make_problem
    p = make_problem("c1")
    say("handle destroyed before its batch")
    lib = fp.load()
    plan = fp.Plan(p.m, p.n, p.indptr, p.indices, p.data, alpha=0.3, k=0.01)
    h = fp.Handle(0)
    b = fp.Batch(h, [plan])
    dev = torch.device("cuda", 0)
    b.svd([torch.from_numpy(p.data).to(dev)])
    assert b.sync()[0] == ["OK"]
    lib.fastpi_destroy(h._h)            # the handle goes first
    h._h = None
    st = (ctypes.c_int32 * 1)()
    assert lib.fastpi_batch_sync(b._b, st, None) == -1
    assert lib.fastpi_batch_set_tuning(b._b, ctypes.byref(fp.Tuning(32768, 4, 128, 1, 1))) == -1
    lib.fastpi_batch_destroy(b._b)      # then the batch
    b._b = None
