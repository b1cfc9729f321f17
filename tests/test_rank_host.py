"""CPU checks of the learned-rank plumbing: the library's block features equal the
oracle's, rank overrides recompute the stage ranks, the allocation keeps the budget."""
import numpy as np
import pytest

from oracle import rank as orank
from synth import make_problem, small_config


@pytest.fixture(scope="module")
def fp():
    import paper_2011_04235_amd as fp
    fp.load()
    return fp


@pytest.mark.parametrize("cfg,alpha", [("c1", 0.3),
                                       (small_config(3000, 700, 0.004, gamma=1.9, seed=21), 0.1)])
def test_library_features_match_oracle(fp, cfg, alpha):
    p = make_problem(cfg, with_labels=False)
    plan = fp.Plan(p.m, p.n, p.indptr, p.indices, p.data, alpha=alpha, k=p.cfg.k)
    got = plan.block_features(p.data)
    want, spectra, alpha_ranks, shapes = orank.problem_blocks(p.m, p.n, p.indptr, p.indices,
                                                              p.data, alpha, p.cfg.k)
    assert got.shape == want.shape
    assert np.allclose(got, want, rtol=1e-12, atol=1e-12), np.abs(got - want).max(axis=0)


def test_block_rank_override(fp):
    p = make_problem("c1", with_labels=False)
    plan = fp.Plan(p.m, p.n, p.indptr, p.indices, p.data, alpha=0.3, k=0.01)
    base = plan.block_ranks()
    blocks = plan.blocks()
    new = base.copy()
    dense = np.flatnonzero((blocks[:, 2] > 0) & (blocks[:, 3] > 0))
    new[dense[0]] = 0
    new[dense[1]] = 10 ** 6              # clamped to min(rows, cols)
    plan.set_block_ranks(new)
    got = plan.block_ranks()
    assert got[dense[0]] == 0 and got[dense[1]] == min(blocks[dense[1], 2], blocks[dense[1], 3])
    assert plan.s_b == int(got.sum())
    assert plan.s == min(fp.target_rank(0.3, plan.n1), plan.s_b + plan.m2, plan.n1)


def _ref():
    import os
    import sys
    sys.path.insert(0, os.path.dirname(__file__))
    import rank_reference
    return rank_reference


def test_rank_inputs_match_reference(fp):
    """fastpi_rank_inputs against the plain reading of the standardisation and range rules:
    identical float32 inputs and flags, rows in and out of range, a zero-span feature."""
    ref = _ref()
    rng = np.random.default_rng(4)
    F = rng.standard_normal((60, 16)) * rng.uniform(0.1, 5.0, size=16) + rng.uniform(-3, 3, size=16)
    train = F[:40]
    mean, std = train.mean(0), train.std(0)
    lo, hi = train.min(0), train.max(0)
    F[40:] = train[:20]                            # copies of training rows, then edited
    F[45, 3] = hi[3] + 0.049 * (hi[3] - lo[3])     # just inside the 5% margin
    F[46, 3] = hi[3] + 0.051 * (hi[3] - lo[3])     # just outside
    F[47, 9] = lo[9] - 0.2 * (hi[9] - lo[9])       # far below
    for margin in (0.0, 0.05):
        X, ok = fp.rank_inputs(F, mean, std, lo, hi, margin)
        Xr, okr = ref.inputs(F, mean, std, lo, hi, margin)
        assert np.array_equal(X.view(np.uint32), Xr.view(np.uint32))
        assert np.array_equal(ok, okr)
        assert ok[:40].all()
        assert ok[45] == (margin > 0) and not ok[46] and not ok[47]
    # a zero-span feature: only its exact training value is in range
    lo2, hi2 = lo.copy(), hi.copy()
    lo2[7] = hi2[7] = F[0, 7]
    X, ok = fp.rank_inputs(F[:2], mean, std, lo2, hi2, 0.05)
    Xr, okr = ref.inputs(F[:2], mean, std, lo2, hi2, 0.05)
    assert np.array_equal(ok, okr) and ok[0] and (ok[1] == (F[1, 7] == F[0, 7]))


def test_rank_inputs_reject_bad_statistics(fp):
    F = np.zeros((2, 16))
    with pytest.raises(fp.FastPIError):
        fp.rank_inputs(F, np.zeros(16), np.zeros(16), np.zeros(16), np.ones(16), 0.05)   # std 0
    with pytest.raises(fp.FastPIError):
        fp.rank_inputs(F, np.zeros(16), np.ones(16), np.zeros(16), np.ones(16), -1.0)


def test_rank_allocate_matches_reference(fp):
    """fastpi_rank_allocate against the plain reading of the budgeted allocation, bit for
    bit, over random and edge cases; the budget and the caps always hold."""
    ref = _ref()
    rng = np.random.default_rng(0)
    cases = []
    for _ in range(60):
        n = int(rng.integers(1, 80))
        q = rng.integers(0, 40, size=n)
        f = rng.random(n).astype(np.float32)
        budget = int(rng.integers(0, max(int(q.sum()), 1) + 5))
        cases.append((f, q, budget))
    q = np.array([4, 4, 4, 4])
    cases += [
        (np.zeros(0, np.float32), np.zeros(0, np.int64), 5),                   # no blocks
        (np.full(4, 0.5, np.float32), q, 0),                                   # zero budget
        (np.full(4, 0.5, np.float32), q, 100),                                 # budget above sum q
        (np.zeros(4, np.float32), q, 6),                                       # all predictions 0
        (np.full(4, 0.25, np.float32), q, 6),                                  # ties
        (np.array([2.0, -1.0, np.nan, 0.5], np.float32), q, 7),                # clipping, NaN
        (np.array([0.9, 0.9, 0.1], np.float32), np.array([3, 0, 50]), 20),    # a zero cap
    ]
    for f, q, budget in cases:
        got = fp.rank_allocate(f, q, budget)
        want = ref.allocate(f, q, budget)
        assert np.array_equal(got, want), (f, q, budget, got, want)
        assert got.sum() == min(budget, int(np.sum(q))) and (got >= 0).all() and (got <= q).all()
    # proportional where nothing saturates, remainder to the largest fraction
    assert fp.rank_allocate(np.array([0.5, 0.25, 0.25]), np.array([4, 4, 4]), 4).tolist() == [2, 1, 1]
    assert fp.rank_allocate(np.full(4, 0.25), np.array([4, 4, 4, 4]), 6).tolist() == [2, 2, 1, 1]


@pytest.mark.parametrize("cfg,alpha", [("c1", 0.3), ("c2", 0.2)])
def test_alpha_fractions_give_back_the_alpha_rule(fp, cfg, alpha):
    """Eq. 1 as a fixed point: fed the alpha rule's own kept fractions s_i / q_i at the alpha
    rule's total, the allocation returns the alpha rule's ranks."""
    p = make_problem(cfg, with_labels=False)
    plan = fp.Plan(p.m, p.n, p.indptr, p.indices, p.data, alpha=alpha, k=p.cfg.k)
    blocks = plan.blocks()
    dense = (blocks[:, 2] > 0) & (blocks[:, 3] > 0)
    s = plan.block_ranks()[dense]
    q = np.minimum(blocks[dense, 2], blocks[dense, 3])
    got = fp.rank_allocate((s / q).astype(np.float32), q, int(s.sum()))
    assert np.array_equal(got, s)


def test_initialisation_matches_oracle_definition():
    from paper_2011_04235_amd.rank_mlp import init_params
    assert np.allclose(init_params(7), orank.init_params(7), rtol=0, atol=1e-7)
