"""GPU tests of the batching form through the C ABI: several matrices in one persistent
block-SVD launch and batched eigensolvers, graph replay of the stage chain, schedule
variants and the autotuner.

Every input is seeded and synthetic (synth). Each case prints its name before touching the
GPU so that a failing run names the case.
"""
import sys

import numpy as np
import pytest

import oracle
from synth import make_problem, sample_batch_configs, small_config
from parity import compare_svd, to_np

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch
    return torch


@pytest.fixture(scope="module")
def fp():
    import paper_2011_04235_amd as fp
    fp.load()
    return fp


def plan_of(fp, prob, alpha):
    return fp.Plan(prob.m, prob.n, prob.indptr, prob.indices, prob.data, alpha=alpha, k=prob.cfg.k)


def dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(torch.device("cuda", 0))


def single(fp, torch, prob, alpha, precision="fp64", graph=False, tuning=None):
    """One matrix on its own handle (the per-instance path)."""
    h = fp.Handle(0, precision=precision)
    if tuning:
        h.set_tuning(**tuning)
    h.set_graph(graph)
    h.upload_plan(plan_of(fp, prob, alpha))
    U, S, V = h.svd(dev(torch, prob.indptr), dev(torch, prob.indices), dev(torch, prob.data))
    h.sync()
    return h, (U, S, V)


def same(a, b):
    return all(x.shape == y.shape and bool((x == y).all()) for x, y in zip(a, b))


SMALL = [
    ("small-a1", small_config(300, 80, 0.05, alpha=1.0, seed=7, k=0.05, L=6), 1.0),
    ("ragged", small_config(777, 131, 0.02, gamma=1.9, seed=9, k=0.02, L=5), 0.23),
    ("wide", small_config(120, 300, 0.03, gamma=2.2, seed=10, k=0.05, L=4), 0.5),
    ("c1", "c1", 0.3),
    ("tiny", small_config(40, 12, 0.2, seed=11, k=0.1, L=3), 0.5),
]


@pytest.fixture(scope="module")
def small_probs():
    return [(name, make_problem(cfg), alpha) for name, cfg, alpha in SMALL]


def test_batch_matches_oracle_and_single_runs(fp, torch, small_probs):
    say("batch of " + ",".join(n for n, _, _ in small_probs))
    h = fp.Handle(0)
    b = fp.Batch(h, [plan_of(fp, p, a) for _, p, a in small_probs])
    out = b.svd([dev(torch, p.data) for _, p, _ in small_probs])
    status, sweeps = b.sync()
    say(f"  status={status} sweeps={sweeps.tolist()}")
    assert status == ["OK"] * len(small_probs)
    rot = b.rotations()
    for (name, prob, alpha), r, sw in zip(small_probs, rot, sweeps):
        plan = plan_of(fp, prob, alpha)
        for k, q in enumerate((plan.n1, plan.s + plan.n2)):
            nb = -(-q // 16)
            # every sweep of a core checks (nb + nb % 2 - 1) rounds of ceil(nb / 2) pairs
            bound = int(sw[1 + k]) * (nb + nb % 2 - 1) * ((nb + 1) // 2)
            assert 0 <= r[k] <= bound, (name, k, r[k], bound)
    for (name, prob, alpha), (U, S, V) in zip(small_probs, out):
        ores = oracle.fastpi_svd(prob.m, prob.n, prob.indptr, prob.indices, prob.data, alpha, prob.cfg.k)
        ok, info = compare_svd(prob, to_np(U), to_np(S), to_np(V), ores)
        say(f"  {name}: {info}")
        assert ok, (name, info)
        _, ref = single(fp, torch, prob, alpha)
        assert same((U, S, V), ref), name


def test_batch_fused_rounds_equal_three_launch_rounds(fp, torch, small_probs):
    """The batched eigensolves with two launches per round equal, bitwise, those with three
    launches per round, eager and replayed from graphs (the batch's jobs have different
    rounds per sweep, so some sit out the last rounds of a sweep)."""
    say("batch: fused vs three-launch eigensolver rounds")
    vals = [dev(torch, p.data) for _, p, _ in small_probs]
    res = {}
    for fused in (0, 1):
        for graph in (False, True):
            h = fp.Handle(0)
            b = fp.Batch(h, [plan_of(fp, p, a) for _, p, a in small_probs])
            b.set_tuning(eig_fused=fused)
            b.set_graph(graph)
            for _ in range(2 if graph else 1):
                out = b.svd(vals)
                st, sweeps = b.sync()
                assert st == ["OK"] * len(small_probs)
            res[(fused, graph)] = ([tuple(t.clone() for t in o) for o in out], sweeps.tolist(),
                                   b.rotations().tolist())
    ref = res[(0, False)]
    for key, got in res.items():
        assert got[1] == ref[1] and got[2] == ref[2], key
        for o, e in zip(got[0], ref[0]):
            assert same(o, e), key


def test_batch_graph_replays_equal_eager(fp, torch, small_probs):
    say("batch graph replay")
    h = fp.Handle(0)
    b = fp.Batch(h, [plan_of(fp, p, a) for _, p, a in small_probs])
    vals = [dev(torch, p.data) for _, p, _ in small_probs]
    eager = [tuple(t.clone() for t in o) for o in b.svd(vals)]
    b.sync()
    assert b.last_graph_launches() == 0
    b.set_graph(True)
    out = b.outputs()
    for rep in range(3):
        for o in out:
            for t in o:
                t.fill_(float("nan"))
        b.svd(vals, out=out)
        st, _ = b.sync()
        assert st == ["OK"] * len(small_probs)
        assert b.last_graph_launches() >= 3
        for o, e in zip(out, eager):
            assert same(o, e), rep
        # eager work of the program between replays
        x = torch.randn(256, 256, device="cuda", dtype=torch.float64)
        (x @ x.T).sum().item()
        b.set_graph(False)
        e2 = b.svd(vals)
        b.sync()
        for o, e in zip(e2, eager):
            assert same(o, e), rep
        b.set_graph(True)


def test_single_graph_replays_and_recapture(fp, torch):
    prob = make_problem("c1")
    say("single-matrix graph replay c1")
    h, eager = single(fp, torch, prob, 0.3)
    eager = tuple(t.clone() for t in eager)
    h.set_graph(True)
    rp, ci, va = dev(torch, prob.indptr), dev(torch, prob.indices), dev(torch, prob.data)
    for rep in range(3):
        U, S, V = h.svd(rp, ci, va)      # fresh outputs: new pointers, so a new capture
        h.sync()
        assert h.last_graph_launches() >= 3
        assert same((U, S, V), eager), rep
        out = (U, S, V)
        for t in out:
            t.zero_()
        h.svd(rp, ci, va, out=out)       # same pointers: replay
        h.sync()
        assert same(out, eager), rep
        y = torch.ones(1000, device="cuda", dtype=torch.float64).cumsum(0)
        assert float(y[-1].item()) == 1000.0


def test_failing_matrix_does_not_poison_the_batch(fp, torch, small_probs):
    say("batch with a non-finite value in matrix 1")
    probs = small_probs[:3]
    h = fp.Handle(0)
    b = fp.Batch(h, [plan_of(fp, p, a) for _, p, a in probs])
    vals = [dev(torch, p.data) for _, p, _ in probs]
    vals[1][5] = float("inf")
    out = b.svd(vals)
    status, _ = b.sync()
    assert status == ["OK", "ENONFINITE", "OK"]
    for i in (0, 2):
        _, ref = single(fp, torch, probs[i][1], probs[i][2])
        assert same(out[i], ref), i


SCHEDULES = [
    dict(block_lds=16384, block_wgs_per_cu=8, gram_rows=64, inner_sweeps=2),
    dict(block_lds=57344, block_wgs_per_cu=2, gram_rows=256, inner_sweeps=1),
    dict(block_lds=4096, block_wgs_per_cu=1, gram_rows=128, inner_sweeps=1),
    dict(block_lds=32768, block_wgs_per_cu=4, gram_rows=128, inner_sweeps=1, precond=0),
    dict(block_lds=32768, block_wgs_per_cu=4, gram_rows=64, inner_sweeps=2, eig_fused=0),
]


@pytest.mark.parametrize("k", range(len(SCHEDULES)))
def test_schedules_keep_parity(fp, torch, small_probs, k):
    name, prob, alpha = small_probs[1]
    say(f"schedule {SCHEDULES[k]} on {name}")
    _, (U, S, V) = single(fp, torch, prob, alpha, tuning=SCHEDULES[k])
    ores = oracle.fastpi_svd(prob.m, prob.n, prob.indptr, prob.indices, prob.data, alpha, prob.cfg.k)
    ok, info = compare_svd(prob, to_np(U), to_np(S), to_np(V), ores)
    say(f"  {info}")
    assert ok, info


def test_invalid_schedule_is_rejected(fp, torch):
    h = fp.Handle(0)
    with pytest.raises(fp.FastPIError) as ei:
        h.set_tuning(gram_rows=96)
    assert ei.value.status == "EINVAL"


def test_autotuner_picks_and_caches_a_schedule(fp, torch, small_probs, tmp_path):
    name, prob, alpha = small_probs[3]
    say(f"autotune {name}")
    cache = tmp_path / "tuning.txt"
    h = fp.Handle(0)
    h.set_tuning_cache(cache)
    h.upload_plan(plan_of(fp, prob, alpha))
    rp, ci, va = dev(torch, prob.indptr), dev(torch, prob.indices), dev(torch, prob.data)
    report = h.autotune(rp, ci, va)
    say(f"  {report}")
    assert "chose" in report
    lines = cache.read_text().strip().splitlines()
    assert len(lines) == 1 and "|" in lines[0]
    chosen = h.get_tuning()
    # a second handle with the same cache and shape takes the stored schedule
    h2 = fp.Handle(0)
    h2.set_tuning_cache(cache)
    h2.upload_plan(plan_of(fp, prob, alpha))
    assert h2.get_tuning() == chosen
    assert "cached" in h2.autotune(rp, ci, va)
    U, S, V = h2.svd(rp, ci, va)
    h2.sync()
    ores = oracle.fastpi_svd(prob.m, prob.n, prob.indptr, prob.indices, prob.data, alpha, prob.cfg.k)
    ok, info = compare_svd(prob, to_np(U), to_np(S), to_np(V), ores)
    assert ok, info


@pytest.fixture(scope="module")
def c4_subset():
    """Six instances of the 64-matrix batched workload (the ones with the smallest n)."""
    cfgs = sorted(sample_batch_configs(64), key=lambda c: c.n)[:6]
    return [make_problem(c) for c in cfgs]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_c4_subset_batched_equals_per_matrix(fp, torch, c4_subset, precision):
    say(f"c4 subset {[p.cfg.name for p in c4_subset]} {precision}")
    h = fp.Handle(0, precision=precision)
    b = fp.Batch(h, [plan_of(fp, p, p.cfg.alpha) for p in c4_subset])
    vals = [dev(torch, p.data) for p in c4_subset]
    out = b.svd(vals)
    status, sweeps = b.sync()
    say(f"  status={status} sweeps={sweeps.tolist()}")
    assert status == ["OK"] * len(c4_subset)
    for prob, o in zip(c4_subset, out):
        _, ref = single(fp, torch, prob, prob.cfg.alpha, precision=precision)
        assert same(o, ref), prob.cfg.name
    b.set_graph(True)
    out2 = b.svd(vals)
    b.sync()
    for o, r in zip(out2, out):
        assert same(o, r)
