"""fastpi_apply_noalloc (the apply without device allocation, on the library's fixed per-GPU
scratch) against fastpi_apply through the C ABI: two calls in a row, the second smaller, both
bitwise equal to the allocating apply (same kernels, same split of U^T Y); a shape whose split
must shrink to fit the scratch, equal to the allocating apply to FP64 rounding; a shape beyond
the scratch rejected with EINVAL; mixed precision."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

SCRATCH_DOUBLES = 8 << 20


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def factors(torch, m, n, r, L, seed):
    rng = np.random.default_rng(seed)
    dev = torch.device("cuda", 0)
    U = torch.from_numpy(rng.standard_normal((m, r)) / np.sqrt(m)).to(dev)
    S = torch.from_numpy(np.sort(rng.uniform(0.1, 3.0, r))[::-1].copy()).to(dev)
    V = torch.from_numpy(rng.standard_normal((n, r)) / np.sqrt(n)).to(dev)
    Y = torch.from_numpy((rng.random((m, L)) < 0.05).astype(np.float64)).to(dev)
    return U, S, V, Y


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_noalloc_apply_equals_apply(precision):
    import torch

    import paper_2011_04235_amd as fp
    fp.load()
    h = fp.Handle(0, precision=precision)
    dev = torch.device("cuda", 0)
    # two calls in a row, the second smaller: the scratch keeps the first call's contents
    for (m, n, r, L, seed) in [(20000, 2000, 400, 200, 1), (2000, 500, 150, 50, 2)]:
        say(f"noalloc apply {precision} m={m} n={n} r={r} L={L}")
        U, S, V, Y = factors(torch, m, n, r, L, seed)
        Za = h.apply(U, S, V, Y)
        Zb = torch.full((n, L), float("nan"), dtype=torch.float64, device=dev)
        h.apply_noalloc(U, S, V, Y, out=Zb)
        torch.cuda.synchronize()
        assert torch.equal(Za, Zb)
    # a split that must shrink to fit: equal up to the summation order
    m, n, r, L = 6000, 800, 2000, 1500
    say(f"noalloc apply {precision} with fewer splits m={m} r={r} L={L}")
    U, S, V, Y = factors(torch, m, n, r, L, 3)
    Za = h.apply(U, S, V, Y)
    Zb = torch.empty((n, L), dtype=torch.float64, device=dev)
    h.apply_noalloc(U, S, V, Y, out=Zb)
    torch.cuda.synchronize()
    tol = 1e-12 if precision == "fp64" else 1e-4
    err = float((Za - Zb).abs().max() / Za.abs().max())
    say(f"  max rel diff {err:.2e}")
    assert err <= tol
    # beyond the scratch: rejected before any launch
    r, L = 2048, SCRATCH_DOUBLES // (2 * 2048) + 1
    U, S, V, Y = factors(torch, 64, 16, r, L, 4)
    Z = torch.empty((16, L), dtype=torch.float64, device=dev)
    with pytest.raises(fp.FastPIError) as ei:
        h.apply_noalloc(U, S, V, Y, out=Z)
    assert ei.value.status == "EINVAL"
    del ei
