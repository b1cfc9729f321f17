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


def test_allocation_keeps_budget_and_bounds():
    from paper_2011_04235_amd.rank_mlp import RankPredictor
    rng = np.random.default_rng(0)
    for _ in range(20):
        q = rng.integers(1, 12, size=50)
        f = rng.random(50)
        budget = int(rng.integers(1, q.sum()))
        s = RankPredictor.allocate(f, q, budget)
        assert s.sum() == budget and (s >= 0).all() and (s <= q).all()
    # proportional where nothing saturates
    s = RankPredictor.allocate(np.array([0.5, 0.25, 0.25]), np.array([4, 4, 4]), 4)
    assert s.tolist() == [2, 1, 1]


def test_initialisation_matches_oracle_definition():
    from paper_2011_04235_amd.rank_mlp import init_params
    assert np.allclose(init_params(7), orank.init_params(7), rtol=0, atol=1e-7)
