"""GPU parity: the HIP path, called through the C ABI, against the CPU oracle.

Every input is seeded and synthetic (synth). Each case prints its name and shape before
touching the GPU so that a failing run names the case.
"""
import sys

import numpy as np
import pytest

import oracle
from synth import make_problem, small_config
from parity import (MIXED_LS_RTOL, MIXED_RECON_ATOL, MIXED_SIGMA_RTOL, compare_apply,
                    compare_svd, sigma_rel_err, to_np)

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


def run_gpu(fp, torch, prob, alpha, precision="fp64", handle=None):
    plan = fp.Plan(prob.m, prob.n, prob.indptr, prob.indices, prob.data, alpha=alpha, k=prob.cfg.k)
    h = handle or fp.Handle(0, precision=precision)
    h.set_precision(precision)
    h.upload_plan(plan)
    dev = torch.device("cuda", 0)
    rowptr = torch.from_numpy(prob.indptr).to(dev)
    col = torch.from_numpy(prob.indices).to(dev)
    val = torch.from_numpy(prob.data).to(dev)
    U, S, V = h.svd(rowptr, col, val)
    h.sync()
    return h, plan, U, S, V


def run_oracle(prob, alpha):
    return oracle.fastpi_svd(prob.m, prob.n, prob.indptr, prob.indices, prob.data, alpha, prob.cfg.k)


# ------------------------------------------------------------------ eigensolver ---------
@pytest.mark.parametrize("q,t,rank", [(1, 1, 1), (5, 3, 5), (16, 8, 16), (17, 17, 17),
                                      (40, 10, 40), (130, 60, 130), (300, 120, 250),
                                      (513, 100, 513), (1100, 64, 1100), (2500, 200, 2500),
                                      (4500, 100, 4000)])
def test_syev_top_matches_dense_eigensolver(fp, torch, q, t, rank):
    say(f"syev_top q={q} t={t} rank={rank}")
    rng = np.random.default_rng(q * 7 + t)
    X = rng.lognormal(size=(q + 20, rank)) * (rng.random((q + 20, rank)) < 0.3)
    X = X @ rng.standard_normal((rank, q))
    G = X.T @ X
    h = fp.Handle(0)
    Gd = torch.from_numpy(G).cuda()
    vals, vecs = h.syev_top(Gd, t)
    torch.cuda.synchronize()
    vals, vecs = to_np(vals), to_np(vecs)
    w, Q = np.linalg.eigh(G)
    w, Q = w[::-1], Q[:, ::-1]
    scale = max(w[0], 1e-300)
    assert np.max(np.abs(vals - w[:t])) <= 1e-12 * scale * max(1, q / 100)
    # eigenvector check through the residual and orthonormality (unique up to sign)
    res = G @ vecs - vecs * vals[None, :]
    assert np.max(np.abs(res)) <= 1e-10 * scale
    assert np.max(np.abs(vecs.T @ vecs - np.eye(t))) <= 1e-10


@pytest.mark.parametrize("e2", [500, -300, -500])
def test_syev_top_is_scale_invariant(fp, torch, e2):
    """The eigenpairs of 2^e2 G are 2^e2 times those of G. At 2^500 and 2^-500 the pair
    solves' d^2 + 4 h^2 leaves the normal range and their rotations take the tangent form."""
    q, t = 130, 60
    say(f"syev_top q={q} t={t} scale 2^{e2}")
    rng = np.random.default_rng(5)
    X = rng.lognormal(size=(q + 20, q)) * (rng.random((q + 20, q)) < 0.3)
    G = X.T @ X
    c = 2.0 ** e2
    h = fp.Handle(0)
    vals, vecs = h.syev_top(torch.from_numpy(G * c).cuda(), t)
    torch.cuda.synchronize()
    vals, vecs = to_np(vals) / c, to_np(vecs)
    w = np.linalg.eigvalsh(G)[::-1]
    assert np.max(np.abs(vals - w[:t])) <= 1e-12 * w[0] * 1.3
    res = G @ vecs - vecs * vals[None, :]
    assert np.max(np.abs(res)) <= 1e-10 * w[0]
    assert np.max(np.abs(vecs.T @ vecs - np.eye(t))) <= 1e-10


@pytest.mark.parametrize("q,t,rows", [(1, 1, 128), (17, 9, 128), (40, 10, 64), (130, 60, 256),
                                      (513, 100, 128), (1100, 64, 64), (2500, 200, 256)])
def test_syev_top_fused_rounds_equal_three_launch_rounds(fp, torch, q, t, rows):
    """Two launches per Jacobi round (round t's column update fused with round t + 1's partial
    Grams, then the pair solves) compute bitwise what three launches per round compute: the
    same products in the same order, on two iterates."""
    say(f"syev_top fused vs three-launch rounds q={q} t={t} rows={rows}")
    rng = np.random.default_rng(q * 3 + rows)
    X = rng.lognormal(size=(q + 20, q)) * (rng.random((q + 20, q)) < 0.3)
    G = X.T @ X
    Gd = torch.from_numpy(G).cuda()
    out = []
    for fused in (0, 1):
        h = fp.Handle(0)
        h.set_tuning(gram_rows=rows, eig_fused=fused)
        assert h.get_tuning()["eig_fused"] == fused
        vals, vecs = h.syev_top(Gd, t)
        torch.cuda.synchronize()
        out.append((to_np(vals), to_np(vecs)))
    assert np.array_equal(out[0][0], out[1][0])
    assert np.array_equal(out[0][1], out[1][1])
    w = np.linalg.eigvalsh(G)[::-1]
    assert np.max(np.abs(out[1][0] - w[:t])) <= 1e-12 * w[0] * max(1, q / 100)


# ------------------------------------------------------------------ whole path ----------
SMALL = [
    ("small-a1", small_config(300, 80, 0.05, alpha=1.0, seed=7, k=0.05, L=6), 1.0),
    ("small-a03", small_config(300, 80, 0.05, alpha=0.3, seed=8, k=0.05, L=6), 0.3),
    ("ragged", small_config(777, 131, 0.02, gamma=1.9, seed=9, k=0.02, L=5), 0.23),
    ("wide", small_config(120, 300, 0.03, gamma=2.2, seed=10, k=0.05, L=4), 0.5),
    ("c1", "c1", 0.3),
]


@pytest.mark.parametrize("name,cfg,alpha", SMALL, ids=[s[0] for s in SMALL])
def test_svd_and_apply_parity(fp, torch, name, cfg, alpha):
    prob = make_problem(cfg)
    say(f"svd {name} m={prob.m} n={prob.n} nnz={prob.nnz} alpha={alpha}")
    h, plan, U, S, V = run_gpu(fp, torch, prob, alpha)
    ores = run_oracle(prob, alpha)
    assert S.shape[0] == ores.r == plan.r
    ok, info = compare_svd(prob, to_np(U), to_np(S), to_np(V), ores)
    say(f"  {info}")
    assert ok, info
    Y = torch.from_numpy(prob.Y).cuda()
    Z = h.apply(U, S, V, Y)
    torch.cuda.synchronize()
    ok, zinfo = compare_apply(prob, to_np(Z), ores)
    say(f"  {zinfo}")
    assert ok, zinfo


def test_stage_outputs_match_oracle(fp, torch):
    prob = make_problem("c1")
    say("stages c1")
    h, plan, U, S, V = run_gpu(fp, torch, prob, 0.3)
    ores = run_oracle(prob, 0.3)
    sig1 = to_np(h.stage_output(0))
    sig2 = to_np(h.stage_output(1))
    assert sig1.shape == ores.blocks.sigma1.shape
    assert np.max(np.abs(sig1 - ores.blocks.sigma1) / ores.blocks.sigma1) <= 1e-12
    assert sigma_rel_err(sig2, ores.row.sigma) <= 1e-9
    # V2 spans the oracle's subspace: compare projectors on random probes
    V2 = to_np(h.stage_output(2))
    X = np.random.default_rng(1).standard_normal((V2.shape[0], 6))
    P1 = V2 @ (V2.T @ X)
    P2 = ores.row.V @ (ores.row.V.T @ X)
    assert np.linalg.norm(P1 - P2) <= 1e-8 * np.linalg.norm(P2)


def test_c2_full_size_parity(fp, torch):
    """The benchmark workload (20000 x 2000, alpha 0.2) in the benchmark's configuration."""
    prob = make_problem("c2")
    say(f"svd c2 m={prob.m} n={prob.n} nnz={prob.nnz}")
    h, plan, U, S, V = run_gpu(fp, torch, prob, 0.2)
    ores = run_oracle(prob, 0.2)
    ok, info = compare_svd(prob, to_np(U), to_np(S), to_np(V), ores)
    say(f"  {info} sweeps={h.last_sweeps()}")
    assert ok, info
    Z = h.apply(U, S, V, torch.from_numpy(prob.Y).cuda())
    torch.cuda.synchronize()
    ok, zinfo = compare_apply(prob, to_np(Z), ores)
    say(f"  {zinfo}")
    assert ok, zinfo


def test_runs_are_bitwise_reproducible(fp, torch):
    prob = make_problem("c1")
    say("determinism c1")
    h, plan, U, S, V = run_gpu(fp, torch, prob, 0.3)
    U1, S1, V1 = U.clone(), S.clone(), V.clone()
    dev = torch.device("cuda", 0)
    U, S, V = h.svd(torch.from_numpy(prob.indptr).to(dev), torch.from_numpy(prob.indices).to(dev),
                    torch.from_numpy(prob.data).to(dev))
    h.sync()
    assert torch.equal(U, U1) and torch.equal(S, S1) and torch.equal(V, V1)


def test_nonfinite_value_is_reported(fp, torch):
    prob = make_problem(small_config(200, 50, 0.05, seed=3, k=0.05))
    say("non-finite input")
    plan = fp.Plan(prob.m, prob.n, prob.indptr, prob.indices, prob.data, alpha=0.5, k=0.05)
    h = fp.Handle(0)
    h.upload_plan(plan)
    dev = torch.device("cuda", 0)
    val = torch.from_numpy(prob.data).to(dev)
    val[3] = float("inf")
    h.svd(torch.from_numpy(prob.indptr).to(dev), torch.from_numpy(prob.indices).to(dev), val)
    with pytest.raises(fp.FastPIError) as ei:
        h.sync()
    assert ei.value.status == "ENONFINITE"


def test_c2_benchmark_form_parity(fp, torch):
    """The benchmark line's form at its full size: 20000 x 2000, alpha 0.2, mixed precision,
    the autotuned schedule and the stages replayed from graphs, against the oracle under the
    mixed-precision gates, on two replays, each bitwise equal to an eager run."""
    prob = make_problem("c2")
    say(f"benchmark form c2 m={prob.m} n={prob.n}: mixed, autotuned, graph replay")
    plan = fp.Plan(prob.m, prob.n, prob.indptr, prob.indices, prob.data, alpha=0.2, k=prob.cfg.k)
    h = fp.Handle(0, precision="mixed")
    h.upload_plan(plan)
    dev = torch.device("cuda", 0)
    args = [torch.from_numpy(x).to(dev) for x in (prob.indptr, prob.indices, prob.data)]
    U = torch.empty((plan.m, plan.r), dtype=torch.float64, device=dev)
    S = torch.empty((plan.r,), dtype=torch.float64, device=dev)
    V = torch.empty((plan.n, plan.r), dtype=torch.float64, device=dev)
    say(f"  {h.autotune(*args, out=(U, S, V)).split('chose')[-1].strip()}")
    h.svd(*args, out=(U, S, V))
    h.sync()
    eager = (to_np(U), to_np(S), to_np(V))
    ores = run_oracle(prob, 0.2)
    h.set_graph(True)
    for rep in range(2):
        h.svd(*args, out=(U, S, V))
        h.sync()
        got = (to_np(U), to_np(S), to_np(V))
        assert all(np.array_equal(x, y) for x, y in zip(got, eager)), rep
        ok, info = compare_svd(prob, *got, ores, sigma_rtol=MIXED_SIGMA_RTOL, product_rtol=1e-4,
                               recon_atol=MIXED_RECON_ATOL, orth_atol=1e-5)
        say(f"  replay {rep}: {info}")
        assert ok, info


# ------------------------------------------------------------------ mixed precision -----
MIXED = [
    ("c1", "c1", 0.3),
    ("small-a1", small_config(300, 80, 0.05, alpha=1.0, seed=7, k=0.05, L=6), 1.0),
    ("c2", "c2", 0.2),
]


@pytest.mark.parametrize("name,cfg,alpha", MIXED, ids=[s[0] for s in MIXED])
def test_mixed_precision_meets_gates(fp, torch, name, cfg, alpha):
    """FP32 block Jacobi and FP32 GEMMs with the FP64 cores: sigma within 1e-5, the
    reconstruction error within 1e-5 of the oracle's, the regression residual within 1e-4."""
    prob = make_problem(cfg)
    say(f"mixed {name} m={prob.m} n={prob.n} alpha={alpha}")
    h, plan, U, S, V = run_gpu(fp, torch, prob, alpha, precision="mixed")
    ores = run_oracle(prob, alpha)
    ok, info = compare_svd(prob, to_np(U), to_np(S), to_np(V), ores,
                           sigma_rtol=MIXED_SIGMA_RTOL, product_rtol=1e-4,
                           recon_atol=MIXED_RECON_ATOL, orth_atol=1e-5)
    say(f"  {info}")
    assert ok, info
    Z = h.apply(U, S, V, torch.from_numpy(prob.Y).cuda())
    torch.cuda.synchronize()
    _, zinfo = compare_apply(prob, to_np(Z), ores)
    say(f"  {zinfo}")
    assert zinfo["ls_rel"] <= MIXED_LS_RTOL, zinfo


def test_tolerance_option_reaches_the_eigensolvers(fp, torch):
    """The handle's tol is the cosine threshold of the eigensolvers of both cores: a loose one
    rotates fewer pairs and still meets the mixed-precision gates. One below FP32 rounding
    leaves the mixed form's FP32 block Jacobi at FP32 epsilon (a threshold it can reach)
    instead of running it into its sweep cap."""
    prob = make_problem("c1")
    ores = run_oracle(prob, 0.3)
    gates = dict(sigma_rtol=MIXED_SIGMA_RTOL, product_rtol=1e-4, recon_atol=MIXED_RECON_ATOL, orth_atol=1e-5)
    say("tolerance option c1: default")
    h0, _, _, _, _ = run_gpu(fp, torch, prob, 0.3)
    rot0 = h0.last_rotations()
    say("tolerance option c1: tol 1e-6")
    h1, _, U, S, V = run_gpu(fp, torch, prob, 0.3, handle=fp.Handle(0, tol=1e-6))
    rot1 = h1.last_rotations()
    say(f"  rotated pairs: default {rot0}, tol 1e-6 {rot1}")
    assert sum(rot1) < sum(rot0)
    ok, info = compare_svd(prob, to_np(U), to_np(S), to_np(V), ores, **gates)
    assert ok, info
    say("tolerance option c1: mixed, tol 1e-11")
    h2, _, U, S, V = run_gpu(fp, torch, prob, 0.3, precision="mixed",
                             handle=fp.Handle(0, precision="mixed", tol=1e-11))
    assert h2.last_sweeps()[0] < 60
    ok, info = compare_svd(prob, to_np(U), to_np(S), to_np(V), ores, **gates)
    assert ok, info
