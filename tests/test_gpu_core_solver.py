"""The subspace core solver of the two updates (subspace iteration with Cholesky-QR
orthonormalisation, Rayleigh-Ritz through the block Jacobi, a residual and rank check with
the Jacobi route as the fallback) through the C ABI, against the oracle: the routes it takes,
FP64 and mixed gates, agreement with the Jacobi route, the fallback on a forced failure (too
few products, and a rank-deficient core), and a batch mixing routes."""
import sys

import numpy as np
import pytest

import oracle
from parity import MIXED_RECON_ATOL, MIXED_SIGMA_RTOL, compare_apply, compare_svd, to_np

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def env():
    import torch

    import paper_2011_04235_amd as fp
    fp.load()
    return torch, fp


def run(torch, fp, prob, alpha, k, precision="fp64", **core):
    dev = torch.device("cuda", 0)
    h = fp.Handle(0, precision=precision)
    if core:
        h.set_core_solver(**core)
    plan = fp.Plan(prob.m, prob.n, prob.indptr, prob.indices, prob.data, alpha=alpha, k=k)
    h.upload_plan(plan)
    U, S, V = h.svd(*(torch.from_numpy(a).to(dev) for a in (prob.indptr, prob.indices, prob.data)))
    Z = h.apply(U, S, V, torch.from_numpy(prob.Y).to(dev))
    code = h.sync()
    return h, plan, code, to_np(U), to_np(S), to_np(V), to_np(Z)


_ORACLE = {}


def oracle_of(prob, alpha, k):
    key = (prob.cfg, alpha, k)
    if key not in _ORACLE:
        _ORACLE[key] = oracle.fastpi_svd(prob.m, prob.n, prob.indptr, prob.indices, prob.data, alpha, k)
    return _ORACLE[key]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_benchmark_shape_takes_the_subspace_route(env, precision):
    """20000 x 2000 (alpha 0.2): the row core (order 1357, t 272) goes through subspace
    iteration, the column core (order 915) stays on Jacobi; gates of the form against the
    oracle, and the FP64 result equals the all-Jacobi one to the FP64 bound."""
    torch, fp = env
    from synth import make_problem
    p = make_problem("c2")
    say(f"20000x2000 {precision}, default core solver")
    h, plan, code, U, S, V, Z = run(torch, fp, p, 0.2, 0.01, precision)
    routes = h.last_core_routes()
    say(f"  routes {routes}, sweeps {h.last_sweeps()}")
    assert code == "OK" and routes == ["subspace", "jacobi"]
    ores = oracle_of(p, 0.2, 0.01)
    if precision == "fp64":
        ok, info = compare_svd(p, U, S, V, ores)
        okz, zinfo = compare_apply(p, Z, ores)
    else:
        ok, info = compare_svd(p, U, S, V, ores, sigma_rtol=MIXED_SIGMA_RTOL, product_rtol=1e-4,
                               recon_atol=MIXED_RECON_ATOL, orth_atol=1e-5)
        okz, zinfo = True, {}
    say(f"  {info} {zinfo}")
    assert ok, info
    assert okz, zinfo
    if precision == "fp64":
        hj, _, _, Uj, Sj, Vj, Zj = run(torch, fp, p, 0.2, 0.01, precision, mode=0)
        assert hj.last_core_routes() == ["jacobi", "jacobi"]
        assert np.max(np.abs(S - Sj) / Sj) <= 1e-12
        assert float(np.linalg.norm(Z - Zj) / np.linalg.norm(Zj)) <= 1e-9


def test_precision_switch_rebuilds_the_subspace_basis(env):
    """20000 x 2000: the row core's basis is 544 columns in FP64 (k_factor 2) and 416 in the
    mixed form (k_factor_mixed 1.5). Switching one handle's precision between runs rebuilds
    the core sets; each run meets its form's gates and the FP64 runs before and after the
    mixed one are bitwise equal."""
    torch, fp = env
    from synth import make_problem
    p = make_problem("c2")
    dev = torch.device("cuda", 0)
    core = fp.Handle(0).get_core_solver()
    assert core["k_factor"] == 2.0 and core["k_factor_mixed"] == 1.5
    say("20000x2000: fp64, mixed, fp64 on one handle")
    h = fp.Handle(0, precision="fp64")
    plan = fp.Plan(p.m, p.n, p.indptr, p.indices, p.data, alpha=0.2, k=0.01)
    h.upload_plan(plan)
    args = [torch.from_numpy(a).to(dev) for a in (p.indptr, p.indices, p.data)]
    ores = oracle_of(p, 0.2, 0.01)
    outs = []
    for precision in ("fp64", "mixed", "fp64"):
        h.set_precision(precision)
        U, S, V = h.svd(*args)
        assert h.sync() == "OK"
        assert h.last_core_routes() == ["subspace", "jacobi"]
        U, S, V = to_np(U), to_np(S), to_np(V)
        if precision == "fp64":
            ok, info = compare_svd(p, U, S, V, ores)
        else:
            ok, info = compare_svd(p, U, S, V, ores, sigma_rtol=MIXED_SIGMA_RTOL, product_rtol=1e-4,
                                   recon_atol=MIXED_RECON_ATOL, orth_atol=1e-5)
        say(f"  {precision}: {info}")
        assert ok, (precision, info)
        outs.append((U, S, V))
    for a, b in zip(outs[0], outs[2]):
        assert np.array_equal(a, b)


def test_forced_subspace_on_a_small_matrix(env):
    """2000 x 500 with the route opened to small orders: the row core (order 383) takes it,
    FP64 gates against the oracle."""
    torch, fp = env
    from synth import make_problem
    p = make_problem("c1")
    say("2000x500, subspace route forced down to order 64")
    h, plan, code, U, S, V, Z = run(torch, fp, p, 0.3, 0.01, min_order=64, max_frac=1.0)
    routes = h.last_core_routes()
    say(f"  routes {routes}")
    assert routes[0] == "subspace"
    ores = oracle_of(p, 0.3, 0.01)
    ok, info = compare_svd(p, U, S, V, ores)
    okz, zinfo = compare_apply(p, Z, ores)
    say(f"  {info} {zinfo}")
    assert ok and okz, (info, zinfo)


def test_failed_check_falls_back_to_jacobi(env):
    """One product only and a tight residual tolerance: the check fails, the core is solved
    again by Jacobi (route 'subspace+jacobi'), and the result still meets the FP64 gates."""
    torch, fp = env
    from synth import make_problem
    p = make_problem("c1")
    say("2000x500, subspace route with one product (must fall back)")
    h, plan, code, U, S, V, Z = run(torch, fp, p, 0.3, 0.01, min_order=64, max_frac=1.0, iters_fp64=1,
                                    res_tol_fp64=1e-14)
    routes = h.last_core_routes()
    say(f"  routes {routes}")
    assert routes[0] == "subspace+jacobi"
    ores = oracle_of(p, 0.3, 0.01)
    ok, info = compare_svd(p, U, S, V, ores)
    okz, zinfo = compare_apply(p, Z, ores)
    assert ok and okz, (info, zinfo)


def test_rank_deficient_core_falls_back(env):
    """A matrix whose row-update Gram matrix has rank below the basis size (few hub rows, one
    block rank per block at alpha = 0.3 on narrow blocks): the Cholesky QR loses rank, the
    core falls back to Jacobi, FP64 gates hold."""
    torch, fp = env
    from synth import small_config, make_problem
    # n1 = 629, rank(M2) = 440, s = 189: a 480-column basis cannot stay independent
    p = make_problem(small_config(3000, 700, 0.002, gamma=2.3, alpha=0.3, seed=32, k=0.002, L=6))
    say("3000x700 sparse, row core of rank 440 < basis 480")
    h, plan, code, U, S, V, Z = run(torch, fp, p, 0.3, 0.002, min_order=64, max_frac=1.0, k_factor=2.5)
    routes = h.last_core_routes()
    say(f"  routes {routes} n1={plan.n1} s_b={plan.s_b} m2={plan.m2} s={plan.s}")
    assert routes[0] == "subspace+jacobi"
    ores = oracle_of(p, 0.3, 0.002)
    ok, info = compare_svd(p, U, S, V, ores)
    okz, zinfo = compare_apply(p, Z, ores)
    say(f"  {info} {zinfo}")
    assert ok and okz, (info, zinfo)


def test_batch_mixing_routes_equals_single_runs(env):
    """A batch of 20000 x 2000 (subspace row core) and 2000 x 500 (Jacobi cores): routes per
    matrix and results bitwise equal to the single runs."""
    torch, fp = env
    from synth import make_problem
    probs = [make_problem("c2"), make_problem("c1")]
    alphas = [0.2, 0.3]
    dev = torch.device("cuda", 0)
    h = fp.Handle(0)
    b = fp.Batch(h, [fp.Plan(p.m, p.n, p.indptr, p.indices, p.data, alpha=a, k=0.01)
                     for p, a in zip(probs, alphas)])
    for graph in (False, True):
        b.set_graph(graph)
        out = b.svd([torch.from_numpy(p.data).to(dev) for p in probs])
        status, _ = b.sync()
        assert status == ["OK", "OK"]
        routes = b.core_routes()
        say(f"  batch graph={graph} routes {routes}")
        assert routes == [["subspace", "jacobi"], ["jacobi", "jacobi"]]
        for p, a, (Ub, Sb, Vb) in zip(probs, alphas, out):
            _, _, _, U, S, V, _ = run(torch, fp, p, a, 0.01)
            assert np.array_equal(to_np(Sb), S) and np.array_equal(to_np(Ub), U) and np.array_equal(to_np(Vb), V)


@pytest.mark.parametrize("ta,tb", [(False, False), (True, False), (False, True), (True, True)])
@pytest.mark.parametrize("fp32", [False, True])
def test_matrix_core_product(env, ta, tb, fp32):
    """The matrix-core product against numpy on ragged shapes (edges inside a 128 x 128 tile
    and a 16-deep slice), every operand orientation, FP64 and FP32; a strided output."""
    torch, fp = env
    dev = torch.device("cuda", 0)
    h = fp.Handle(0)
    rng = np.random.default_rng(7)
    for (M, N, K) in [(1, 1, 1), (130, 70, 33), (257, 300, 129), (64, 129, 1000)]:
        A = rng.standard_normal((K, M) if ta else (M, K))
        B = rng.standard_normal((N, K) if tb else (K, N))
        ref = (A.T if ta else A) @ (B.T if tb else B)
        Cbig = torch.full((M, N + 5), 7.0, dtype=torch.float64, device=dev)
        C = h.mfma_gemm(torch.from_numpy(A).to(dev), torch.from_numpy(B).to(dev), ta=ta, tb=tb, fp32=fp32,
                        out=Cbig[:, :N])
        torch.cuda.synchronize()
        got = C.cpu().numpy()
        err = np.max(np.abs(got - ref)) / max(np.max(np.abs(ref)), 1e-300)
        tol = 1e-5 if fp32 else 1e-13
        assert err <= tol, (M, N, K, ta, tb, fp32, err)
        assert np.all(Cbig[:, N:].cpu().numpy() == 7.0)
