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
