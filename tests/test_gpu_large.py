"""Full-size parity on the 100000 x 5000 (alpha 0.1, 1000 labels) and 300000 x 10000 (alpha
0.1, 2000 labels) workloads in the bench's launch configuration, FP64 and mixed, against
quantities of the oracle's result stored by
tests/golden/make_large_reference.py (the oracle takes minutes at this size): the singular
values, the reconstruction and least-squares errors, Z at sampled rows, and rank-r products
with fixed probe vectors at sampled rows of U and V.

Tolerances follow from the arithmetic: the cores' eigenvalues carry absolute error about
q eps sigma_1^2, so sigma_i has relative error about q eps (sigma_1 / sigma_i)^2 (q the
core order); the factor 8 covers the rounding of the Gram assembly. The mixed form uses the
gates of the scope table.
"""
import os
import sys

import numpy as np
import pytest

from synth import CONFIGS, make_problem

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
EPS = np.finfo(np.float64).eps


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


_CACHE = {}


def setup(name):
    """Problem, plan and stored reference of one workload (built once per module)."""
    if name not in _CACHE:
        import torch

        import paper_2011_04235_amd as fp
        fp.load()
        say(f"building {name}")
        ref = np.load(os.path.join(GOLDEN, f"{name}_reference.npz"))
        prob = make_problem(name)
        cfg = CONFIGS[name]
        plan = fp.Plan(prob.m, prob.n, prob.indptr, prob.indices, prob.data, alpha=cfg.alpha, k=cfg.k)
        _CACHE.clear()
        _CACHE[name] = (torch, fp, ref, prob, cfg, plan)
    return _CACHE[name]


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("name,precision", [("c3", "fp64"), ("c3", "mixed"), ("c5", "fp64"), ("c5", "mixed")])
def test_full_size(name, precision):
    torch, fp, ref, prob, cfg, plan = setup(name)
    import scipy.sparse as sp

    import oracle
    say(f"{name} {prob.m}x{prob.n} nnz={prob.nnz} alpha={cfg.alpha} {precision} (graph replay)")
    dev = torch.device("cuda", 0)
    h = fp.Handle(0, precision=precision)
    h.upload_plan(plan)
    rp, ci, va = (torch.from_numpy(a).to(dev) for a in (prob.indptr, prob.indices, prob.data))
    h.set_graph(True)
    U, S, V = h.svd(rp, ci, va)
    h.sync()
    Y = torch.from_numpy(prob.Y).to(dev)
    Z = h.apply(U, S, V, Y)
    torch.cuda.synchronize()
    say(f"  sweeps {h.last_sweeps()}")
    s = S.cpu().numpy()
    assert s.shape == ref["sigma"].shape
    sig = ref["sigma"]
    q = max(plan.n1, plan.s + plan.n2)
    keep = sig >= 1e-6 * sig[0]
    err = np.abs(s[keep] - sig[keep]) / sig[keep]
    if precision == "fp64":
        bound = np.maximum(1e-9, 8 * q * EPS * (sig[0] / sig[keep]) ** 2)
    else:
        bound = np.full(err.shape, 1e-5)
    say(f"  sigma max rel err {err.max():.2e} (bound at the cut {bound[-1]:.1e})")
    assert np.all(err <= bound)
    A = sp.csr_matrix((prob.data, prob.indices, prob.indptr), shape=(prob.m, prob.n))
    Uh, Vh = U.cpu().numpy(), V.cpu().numpy()
    say("  reconstruction error on the host")
    recon = oracle.recon_error(A, Uh, s, Vh)
    say(f"  recon {recon:.12f} oracle {float(ref['recon']):.12f}")
    assert abs(recon - float(ref["recon"])) <= (1e-10 if precision == "fp64" else 1e-5)
    g = np.random.default_rng(int(ref["probe_seed"]))
    P, Qp = g.standard_normal((prob.n, 4)), g.standard_normal((prob.m, 4))
    usvp = (Uh[ref["rows_u"]] * s[None, :]) @ (Vh.T @ P)
    vsuq = (Vh[ref["rows_v"]] * s[None, :]) @ (Uh.T @ Qp)
    e1, e2 = rel(usvp, ref["usvp"]), rel(vsuq, ref["vsuq"])
    say(f"  probe products rel err {e1:.2e} {e2:.2e}")
    tol = 1e-8 if precision == "fp64" else 1e-4
    assert e1 <= tol and e2 <= tol
    Zh = Z.cpu().numpy()
    ez = rel(Zh[ref["rows_z"]], ref["z_rows"])
    ls = oracle.ls_residual(A, Zh, prob.Y)
    say(f"  Z rows rel err {ez:.2e}; LS residual {ls:.10f} oracle {float(ref['ls']):.10f}")
    assert ez <= (1e-7 if precision == "fp64" else 1e-3)
    assert abs(ls - float(ref["ls"])) <= (1e-9 if precision == "fp64" else 1e-4) * float(ref["ls"])


C4_INSTANCES = [23, 19, 55, 0]   # the widest (7272 x 3905), the most non-zeros, a tall narrow one, the first


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batched_instances_against_stored_oracle(precision):
    """Four instances of the 64-matrix batched workload in one batch (persistent block launch,
    batched eigensolvers, graph replay), each against the oracle's stored quantities for that
    instance: singular values, reconstruction and least-squares errors, Z at sampled rows and
    the probed rank-r products."""
    import scipy.sparse as sp
    import torch

    import oracle
    import paper_2011_04235_amd as fp
    from synth import sample_batch_configs
    fp.load()
    cfgs = sample_batch_configs(64)
    probs, plans, refs = [], [], []
    for i in C4_INSTANCES:
        c = cfgs[i]
        probs.append(make_problem(c))
        plans.append(fp.Plan(c.m, c.n, probs[-1].indptr, probs[-1].indices, probs[-1].data, alpha=c.alpha, k=c.k))
        refs.append(np.load(os.path.join(GOLDEN, f"c4_{i}_reference.npz")))
    say(f"batched instances {C4_INSTANCES} {precision} (graph replay)")
    dev = torch.device("cuda", 0)
    h = fp.Handle(0, precision=precision)
    b = fp.Batch(h, plans)
    b.set_graph(True)
    out = b.svd([torch.from_numpy(p.data).to(dev) for p in probs])
    status, sweeps = b.sync()
    assert all(s in ("OK",) for s in status), status
    for i, p, plan, ref, (U, S, V) in zip(C4_INSTANCES, probs, plans, refs, out):
        Z = h.apply(U, S, V, torch.from_numpy(p.Y).to(dev))
        torch.cuda.synchronize()
        s, Uh, Vh, Zh = S.cpu().numpy(), U.cpu().numpy(), V.cpu().numpy(), Z.cpu().numpy()
        sig = ref["sigma"]
        assert s.shape == sig.shape
        q = max(plan.n1, plan.s + plan.n2)
        keep = sig >= 1e-6 * sig[0]
        err = np.abs(s[keep] - sig[keep]) / sig[keep]
        bound = (np.maximum(1e-9, 8 * q * EPS * (sig[0] / sig[keep]) ** 2) if precision == "fp64"
                 else np.full(err.shape, 1e-5))
        A = sp.csr_matrix((p.data, p.indices, p.indptr), shape=(p.m, p.n))
        recon = oracle.recon_error(A, Uh, s, Vh)
        g = np.random.default_rng(int(ref["probe_seed"]))
        P, Qp = g.standard_normal((p.n, 4)), g.standard_normal((p.m, 4))
        e1 = rel((Uh[ref["rows_u"]] * s[None, :]) @ (Vh.T @ P), ref["usvp"])
        e2 = rel((Vh[ref["rows_v"]] * s[None, :]) @ (Uh.T @ Qp), ref["vsuq"])
        ez = rel(Zh[ref["rows_z"]], ref["z_rows"])
        ls = oracle.ls_residual(A, Zh, p.Y)
        say(f"  instance {i} {p.m}x{p.n} r={plan.r}: sigma {err.max():.1e}, recon {recon:.10f} vs "
            f"{float(ref['recon']):.10f}, products {e1:.1e} {e2:.1e}, Z {ez:.1e}, LS {ls:.8f} vs {float(ref['ls']):.8f}")
        assert np.all(err <= bound)
        assert abs(recon - float(ref["recon"])) <= (1e-10 if precision == "fp64" else 1e-5)
        tol = 1e-8 if precision == "fp64" else 1e-4
        assert e1 <= tol and e2 <= tol
        assert ez <= (1e-7 if precision == "fp64" else 1e-3)
        assert abs(ls - float(ref["ls"])) <= (1e-9 if precision == "fp64" else 1e-4) * float(ref["ls"])
