"""GPU checks of the learned rank predictor: forward, gradient and Adam kernels against the
FP64 oracle, training on oracle-labelled blocks, and the gain over the alpha rule."""
import os
import sys

import numpy as np
import pytest

from oracle import rank as orank

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)


@pytest.fixture(scope="module")
def env():
    import torch

    import paper_2011_04235_amd as fp
    from paper_2011_04235_amd.rank_mlp import RankPredictor, init_params
    fp.load()
    d = np.load(os.path.join(GOLDEN, "rank_dataset.npz"))
    return torch, fp, fp.Handle(0), d, RankPredictor, init_params


def standardised(d):
    tr = d["instance"] < d["n_train"]
    X = d["X"]
    mean, std = X[tr].mean(0), X[tr].std(0)
    std = np.where(std > 0, std, 1.0)
    return ((X - mean) / std), tr


def test_forward_and_gradient_match_oracle(env):
    torch, fp, h, d, RankPredictor, init_params = env
    say("mlp forward/gradient vs oracle")
    Xs, tr = standardised(d)
    X32 = Xs[tr][:3000].astype(np.float32)
    y32 = d["y"][tr][:3000].astype(np.float32)
    theta = init_params(5)
    dev = torch.device("cuda", 0)
    Xd, yd, th = (torch.from_numpy(a).to(dev) for a in (X32, y32, theta))
    f = h.mlp_forward(Xd, th).cpu().numpy()
    g = h.mlp_gradient(Xd, yd, th).cpu().numpy()
    g2 = h.mlp_gradient(Xd, yd, th).cpu().numpy()
    fo, _ = orank.forward(theta.astype(np.float64), X32.astype(np.float64))
    go = orank.gradient(theta.astype(np.float64), X32.astype(np.float64), y32.astype(np.float64))
    assert np.max(np.abs(f - fo)) <= 2e-6
    rel = np.linalg.norm(g - go) / np.linalg.norm(go)
    say(f"  forward max err {np.max(np.abs(f - fo)):.2e}, gradient rel err {rel:.2e}")
    assert rel <= 1e-4
    assert np.array_equal(g, g2)        # fixed-order reductions: bitwise reproducible


def test_adam_step_matches_oracle(env):
    torch, fp, h, d, RankPredictor, init_params = env
    say("mlp adam vs oracle")
    rng = np.random.default_rng(3)
    theta = init_params(9)
    g = (rng.standard_normal(theta.size) * 1e-2).astype(np.float32)
    m = (rng.standard_normal(theta.size) * 1e-3).astype(np.float32)
    v = (rng.random(theta.size) * 1e-4).astype(np.float32)
    dev = torch.device("cuda", 0)
    th, gd, md, vd = (torch.from_numpy(a.copy()).to(dev) for a in (theta, g, m, v))
    h.mlp_adam(th, gd, md, vd, 7, 1e-3)
    to, mo, vo = orank.adam_step(theta.astype(np.float64), g.astype(np.float64),
                                 m.astype(np.float64), v.astype(np.float64), 7, 1e-3)
    assert np.max(np.abs(th.cpu().numpy() - to)) <= 1e-6
    assert np.max(np.abs(md.cpu().numpy() - mo)) <= 1e-8
    assert np.max(np.abs(vd.cpu().numpy() - vo)) <= 1e-9


def test_training_beats_alpha_rule_and_gains_on_held_out_matrices(env):
    """Trained on 24 matrices, judged on 8 held-out ones: the predicted kept fractions are
    closer to the Eckart-Young labels than the alpha rule's, and at the alpha rule's budget
    the learned allocation loses less of A11 (sum of discarded squared singular values)."""
    torch, fp, h, d, RankPredictor, init_params = env
    say("mlp training")
    tr = d["instance"] < d["n_train"]
    pred = RankPredictor()
    hist = pred.fit(h, d["X"][tr], d["y"][tr], epochs=600, lr=3e-3, seed=1, log_every=100)
    say(f"  training loss {hist}")
    va = ~tr
    f = pred.predict(h, d["X"][va])
    mse_mlp = float(np.mean((f - d["y"][va]) ** 2))
    mse_alpha = float(np.mean((d["s_alpha"][va] / d["q"][va] - d["y"][va]) ** 2))
    say(f"  validation MSE: network {mse_mlp:.4f}, alpha rule {mse_alpha:.4f}")
    assert mse_mlp < 0.5 * mse_alpha
    # truncation of A11 on the held-out matrices at the alpha rule's budget
    sys.path.insert(0, GOLDEN)
    from make_rank_dataset import instance_config
    from synth import make_problem
    ratios = []
    for i in range(int(d["n_train"]), int(d["instance"].max()) + 1):
        cfg = instance_config(i)
        p = make_problem(cfg, with_labels=False)
        X, spectra, s_alpha, shapes = orank.problem_blocks(p.m, p.n, p.indptr, p.indices, p.data,
                                                           cfg.alpha, cfg.k)
        q = np.minimum(shapes[:, 0], shapes[:, 1])
        s_net = fp.rank_allocate(pred.predict(h, X), q, int(s_alpha.sum()))
        e_net = orank.truncation_error2(spectra, s_net)
        e_alpha = orank.truncation_error2(spectra, s_alpha)
        e_opt = orank.truncation_error2(spectra, orank.eckart_young_ranks(spectra, int(s_alpha.sum())))
        ratios.append(e_net / e_alpha)
        say(f"  matrix {i}: A11 loss network {e_net:.4g}, alpha rule {e_alpha:.4g}, optimum {e_opt:.4g}")
    say(f"  mean loss ratio network / alpha rule: {np.mean(ratios):.3f}")
    assert np.mean(ratios) < 0.9


def test_learned_ranks_end_to_end(env):
    """The whole path with the shipped predictor's ranks (same total s_b as the alpha rule)
    on held-out matrices: reconstruction error of A (and of its A11 part) against the alpha
    rule. Reported always; the learned ranks must not make the result worse overall."""
    torch, fp, h, d, RankPredictor, init_params = env
    import scipy.sparse as sp
    sys.path.insert(0, GOLDEN)
    from make_rank_dataset import instance_config
    from synth import make_problem
    pred = RankPredictor.load(os.path.join(os.path.dirname(fp.__file__), "rank_predictor.npz"))
    dev = torch.device("cuda", 0)
    gains = []
    for i in range(int(d["n_train"]), int(d["instance"].max()) + 1):
        cfg = instance_config(i)
        p = make_problem(cfg, with_labels=False)
        say(f"end-to-end matrix {i}: {p.m}x{p.n} alpha {cfg.alpha}")
        A = sp.csr_matrix((p.data, p.indices, p.indptr), shape=(p.m, p.n))
        errs = {}
        for mode in ("alpha", "learned"):
            plan = fp.Plan(p.m, p.n, p.indptr, p.indices, p.data, alpha=cfg.alpha, k=cfg.k)
            if mode == "learned":
                blocks = plan.blocks()
                dense = (blocks[:, 2] > 0) & (blocks[:, 3] > 0)
                ranks = pred.block_ranks(h, plan, p.data)
                plan.set_block_ranks(ranks)
            h.upload_plan(plan)
            U, S, V = h.svd(torch.from_numpy(p.indptr).to(dev), torch.from_numpy(p.indices).to(dev),
                            torch.from_numpy(p.data).to(dev))
            h.sync()
            errs[mode] = oracle_recon(A, U.cpu().numpy(), S.cpu().numpy(), V.cpu().numpy())
        say(f"  recon error alpha rule {errs['alpha']:.6f}, learned {errs['learned']:.6f}")
        gains.append(errs["alpha"] - errs["learned"])
    say(f"  mean recon-error gain {np.mean(gains):.3e}")
    assert np.mean(gains) >= -1e-4


def oracle_recon(A, U, S, V):
    import oracle
    return oracle.recon_error(A, U, S, V)


def test_learned_ranks_at_scale(env):
    """The 300000 x 10000 workload (alpha 0.1): the shipped predictor's ranks against the alpha
    rule at the same total s_b, through the whole GPU path. Reported: the share of blocks the
    network ranks (the rest fall back to the alpha rule), the squared A11 truncation loss of
    both allocations (oracle block spectra) and the reconstruction error of A of both runs.
    The learned allocation must lose less of A11 and must not raise the error of A."""
    torch, fp, h, d, RankPredictor, init_params = env
    from synth import CONFIGS, make_problem
    cfg = CONFIGS["c5"]
    say("learned ranks at scale: building the 300000 x 10000 workload")
    p = make_problem("c5", with_labels=False)
    pred = RankPredictor.load(os.path.join(os.path.dirname(fp.__file__), "rank_predictor.npz"))
    dev = torch.device("cuda", 0)
    import scipy.sparse as sp
    A = sp.csr_matrix((p.data, p.indices, p.indptr), shape=(p.m, p.n))
    errs, ranks_used = {}, {}
    for mode in ("alpha", "learned"):
        plan = fp.Plan(p.m, p.n, p.indptr, p.indices, p.data, alpha=cfg.alpha, k=cfg.k)
        blocks = plan.blocks()
        dense = (blocks[:, 2] > 0) & (blocks[:, 3] > 0)
        if mode == "learned":
            X = plan.block_features(p.data)
            say(f"  network ranks {int(pred.in_range(X).sum())} of {len(X)} blocks")
            plan.set_block_ranks(pred.block_ranks(h, plan, p.data))
        ranks_used[mode] = plan.block_ranks()[dense]
        h.upload_plan(plan)
        say(f"  {mode}: s_b={plan.s_b} s={plan.s} r={plan.r}, GPU run")
        U, S, V = h.svd(torch.from_numpy(p.indptr).to(dev), torch.from_numpy(p.indices).to(dev),
                        torch.from_numpy(p.data).to(dev))
        h.sync()
        errs[mode] = oracle_recon(A, U.cpu().numpy(), S.cpu().numpy(), V.cpu().numpy())
        del U, S, V
        say(f"  {mode}: reconstruction error {errs[mode]:.8f}")
    assert ranks_used["alpha"].sum() == ranks_used["learned"].sum()
    say("  A11 block spectra (oracle)")
    X, spectra, s_alpha, shapes = orank.problem_blocks(p.m, p.n, p.indptr, p.indices, p.data, cfg.alpha, cfg.k)
    assert np.array_equal(s_alpha, ranks_used["alpha"])
    e_alpha = orank.truncation_error2(spectra, ranks_used["alpha"])
    e_net = orank.truncation_error2(spectra, ranks_used["learned"])
    e_opt = orank.truncation_error2(spectra, orank.eckart_young_ranks(spectra, int(s_alpha.sum())))
    say(f"  A11 loss: alpha rule {e_alpha:.6g}, network {e_net:.6g}, optimum {e_opt:.6g}; "
        f"recon alpha {errs['alpha']:.8f} learned {errs['learned']:.8f}")
    assert e_net < e_alpha
    assert errs["learned"] <= errs["alpha"] + 1e-4



def test_learned_ranks_match_oracle_with_same_ranks(env):
    """The whole GPU path under the shipped predictor's per-block ranks against the oracle
    run with the same per-block ranks (Eq. 1 with given s_i), on two held-out matrices, FP64
    gates (singular values, rank-r product, reconstruction error, orthonormality, Z)."""
    torch, fp, h, d, RankPredictor, init_params = env
    sys.path.insert(0, GOLDEN)
    sys.path.insert(0, os.path.dirname(__file__))
    import oracle
    from make_rank_dataset import instance_config
    from parity import compare_apply, compare_svd
    from synth import make_problem
    pred = RankPredictor.load(os.path.join(os.path.dirname(fp.__file__), "rank_predictor.npz"))
    dev = torch.device("cuda", 0)
    for i in range(int(d["n_train"]), int(d["n_train"]) + 2):
        cfg = instance_config(i)
        p = make_problem(cfg)
        say(f"learned ranks vs oracle, matrix {i}: {p.m}x{p.n} alpha {cfg.alpha}")
        plan = fp.Plan(p.m, p.n, p.indptr, p.indices, p.data, alpha=cfg.alpha, k=cfg.k)
        blocks = plan.blocks()
        dense = (blocks[:, 2] > 0) & (blocks[:, 3] > 0)
        alpha_ranks = plan.block_ranks().copy()
        plan.set_block_ranks(pred.block_ranks(h, plan, p.data))
        ranks = plan.block_ranks()
        assert not np.array_equal(ranks, alpha_ranks)
        h.upload_plan(plan)
        U, S, V = h.svd(*(torch.from_numpy(a).to(dev) for a in (p.indptr, p.indices, p.data)))
        Z = h.apply(U, S, V, torch.from_numpy(p.Y).to(dev))
        h.sync()
        ores = oracle.fastpi_svd(p.m, p.n, p.indptr, p.indices, p.data, cfg.alpha, cfg.k, block_ranks=ranks)
        assert np.array_equal(ores.blocks.ranks, ranks)
        ok, info = compare_svd(p, U.cpu().numpy(), S.cpu().numpy(), V.cpu().numpy(), ores)
        say(f"  {info}")
        assert ok, info
        okz, zinfo = compare_apply(p, Z.cpu().numpy(), ores)
        say(f"  {zinfo}")
        assert okz, zinfo


def test_plan_learned_ranks_match_reference(env):
    """fastpi_plan_learned_ranks (standardisation, range fallback, network, budgeted
    allocation inside the library) against the Python reference of the same rules fed by the
    network's outputs, on the 20000 x 2000 workload and a held-out matrix; bit-exact ranks."""
    torch, fp, h, d, RankPredictor, init_params = env
    sys.path.insert(0, GOLDEN)
    sys.path.insert(0, os.path.dirname(__file__))
    import rank_reference as ref
    from make_rank_dataset import instance_config
    from synth import CONFIGS, make_problem
    pred = RankPredictor.load(os.path.join(os.path.dirname(fp.__file__), "rank_predictor.npz"))
    dev = torch.device("cuda", 0)
    th = torch.from_numpy(pred.theta).to(dev)
    for name, cfg in (("c2", CONFIGS["c2"]), ("held-out", instance_config(int(d["n_train"])))):
        p = make_problem(cfg, with_labels=False)
        plan = fp.Plan(p.m, p.n, p.indptr, p.indices, p.data, alpha=cfg.alpha, k=cfg.k)
        got = plan.learned_ranks(h, p.data, th, pred.mean, pred.std, pred.lo, pred.hi, pred.MARGIN)
        F = plan.block_features(p.data)
        X, ok = ref.inputs(F, pred.mean, pred.std, pred.lo, pred.hi, pred.MARGIN)
        f = h.mlp_forward(torch.from_numpy(np.ascontiguousarray(X[ok])).to(dev), th).cpu().numpy()
        want = ref.plan_ranks(plan.blocks(), plan.block_ranks(), f, ok)
        say(f"  {name}: {int(ok.sum())} of {len(ok)} blocks ranked by the network, "
            f"{int(np.sum(got != plan.block_ranks()))} ranks moved")
        assert np.array_equal(got, want)
        assert got.sum() == plan.block_ranks().sum()
