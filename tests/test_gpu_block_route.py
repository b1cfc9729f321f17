"""GPU parity of the Gram route for diagonal blocks of A11 (Eq. 1): a block whose Jacobi cost
p q^2 reaches the route's threshold is solved through G = X^T X, the batched eigensolver and
W = X E. The threshold is lowered so that the route carries most or all blocks of small
workloads, which are then compared with the oracle under the FP64 gates of the path; the
block singular values themselves are held to the Gram route's own bound,
max(1e-12, 8 q eps (sigma_1 / sigma_i)^2) relative, or zero below 1e-7 sigma_1."""
import sys

import numpy as np
import pytest

import oracle
from parity import MIXED_RECON_ATOL, MIXED_SIGMA_RTOL, compare_apply, compare_svd, to_np
from synth import make_problem, small_config

pytestmark = pytest.mark.gpu
EPS = np.finfo(np.float64).eps


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def env():
    import torch

    import paper_2011_04235_amd as fp
    fp.load()
    return torch, fp


def dev_t(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(torch.device("cuda", 0))


def run(torch, fp, prob, alpha, k, route, precision="fp64", graph=False):
    plan = fp.Plan(prob.m, prob.n, prob.indptr, prob.indices, prob.data, alpha=alpha, k=k)
    h = fp.Handle(0, precision=precision)
    h.set_block_route(route)
    h.upload_plan(plan)
    h.set_graph(graph)
    U, S, V = h.svd(dev_t(torch, prob.indptr), dev_t(torch, prob.indices), dev_t(torch, prob.data))
    Z = h.apply(U, S, V, dev_t(torch, prob.Y))
    sig1 = to_np(h.stage_output(0))
    h.sync()
    return plan, h, to_np(U), to_np(S), to_np(V), to_np(Z), sig1


def check_block_sigma(plan, sig1, ores):
    """Per block, the kept singular values against the oracle's block SVD."""
    worst = 0.0
    off = 0
    ranks = plan.block_ranks()
    blocks = plan.blocks()
    dense = [i for i, b in enumerate(blocks) if b[2] > 0 and b[3] > 0]
    for bi, full in zip(dense, ores.blocks.block_sigma):
        si = int(ranks[bi])
        if si == 0:
            continue
        got, want = sig1[off:off + si], full[:si]
        off += si
        q = min(blocks[bi][2], blocks[bi][3])
        s1 = want[0]
        for g, w in zip(got, want):
            if w < 1e-7 * s1:
                assert g == 0.0 or abs(g - w) <= 1e-7 * s1
                continue
            bound = max(1e-12, 8 * q * EPS * (s1 / w) ** 2)
            err = abs(g - w) / w
            worst = max(worst, err / bound)
            assert err <= bound, (bi, g, w, bound)
    assert off == sig1.size
    return worst


CASES = [
    ("2000x500-all", "c1", 0.3, 0.01, 0.0),
    ("777x131-all", small_config(777, 131, 0.02, gamma=1.9, seed=9, k=0.02, L=5), 0.23, 0.02, 0.0),
    ("20000x2000-large", "c2", 0.2, 0.01, 1e5),
    ("20000x2000-all", "c2", 0.2, 0.01, 0.0),
]


@pytest.mark.parametrize("name,cfg,alpha,k,route", CASES, ids=[c[0] for c in CASES])
def test_gram_route_matches_oracle(env, name, cfg, alpha, k, route):
    torch, fp = env
    prob = make_problem(cfg)
    say(f"{name}: {prob.m}x{prob.n} alpha={alpha} route threshold {route:g}")
    plan, h, U, S, V, Z, sig1 = run(torch, fp, prob, alpha, k, route)
    ores = oracle.fastpi_svd(prob.m, prob.n, prob.indptr, prob.indices, prob.data, alpha, k)
    worst = check_block_sigma(plan, sig1, ores)
    say(f"  block sigma: worst error / bound {worst:.3f}")
    ok, sinfo = compare_svd(prob, U, S, V, ores)
    say(f"  {sinfo}")
    assert ok, sinfo
    ok, zinfo = compare_apply(prob, Z, ores)
    assert ok, zinfo


def test_gram_route_mixed_batch_and_graph(env):
    """Mixed precision with every block on the route within the mixed gates; a batch of two
    matrices bitwise equal to single runs; graph replays bitwise equal to eager runs."""
    torch, fp = env
    prob = make_problem("c1")
    say("2000x500 mixed, every block on the Gram route")
    _, _, U, S, V, _, _ = run(torch, fp, prob, 0.3, 0.01, 0.0, precision="mixed")
    ores = oracle.fastpi_svd(prob.m, prob.n, prob.indptr, prob.indices, prob.data, 0.3, 0.01)
    ok, sinfo = compare_svd(prob, U, S, V, ores, sigma_rtol=MIXED_SIGMA_RTOL, product_rtol=1e-4,
                            recon_atol=MIXED_RECON_ATOL, orth_atol=1e-5)
    assert ok, sinfo
    probs = [prob, make_problem(small_config(777, 131, 0.02, gamma=1.9, seed=9, k=0.02, L=5))]
    alphas, ks = [0.3, 0.23], [0.01, 0.02]
    singles = [run(torch, fp, p, a, k, 0.0)[2:5] for p, a, k in zip(probs, alphas, ks)]
    h = fp.Handle(0)
    h.set_block_route(0.0)
    b = fp.Batch(h, [fp.Plan(p.m, p.n, p.indptr, p.indices, p.data, alpha=a, k=k)
                     for p, a, k in zip(probs, alphas, ks)])
    vals = [dev_t(torch, p.data) for p in probs]
    for graph in (False, True, True):
        say(f"  batch, graph={graph}")
        b.set_graph(graph)
        out = b.svd(vals)
        status, _ = b.sync()
        assert status == ["OK", "OK"], status
        for (Ub, Sb, Vb), (Us, Ss, Vs) in zip(out, singles):
            assert np.array_equal(to_np(Sb), Ss) and np.array_equal(to_np(Ub), Us)
            assert np.array_equal(to_np(Vb), Vs)


def test_block_route_rejects_bad_cost(env):
    torch, fp = env
    h = fp.Handle(0)
    for bad in (-1.0, float("nan")):
        with pytest.raises(fp.FastPIError):
            h.set_block_route(bad)
