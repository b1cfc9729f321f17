"""Pins of the randomized inner solver's oracle (the truncated SVD the paper uses for a low
target rank in the incremental updates, Section 3.3): the counter-based generator against the
published Philox4x32-10 known-answer vectors, the normal transform's distribution, exact
recovery of planted low-rank spectra, Ritz-value bounds and convergence on planted spectra,
and the branch rule."""
import math

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from synth import make_problem

# Philox4x32-10 known-answer vectors (counter words, key words, output words) published with
# the generator's reference implementation (Random123)
KAT = [
    ((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
    ((0xFFFFFFFF,) * 4, (0xFFFFFFFF,) * 2, (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
    ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
     (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)),
]


@pytest.mark.parametrize("ctr,key,want", KAT)
def test_philox_known_answers(ctr, key, want):
    out = oracle.philox4x32_10([np.array([c], dtype=np.uint64) for c in ctr], key)
    assert tuple(int(o[0]) for o in out) == want


def test_gaussian_distribution_and_streams():
    z = oracle.gaussian(500, 801, seed=3, stream=0)
    assert z.shape == (500, 801)
    n = z.size
    assert abs(z.mean()) < 5 / math.sqrt(n)
    assert abs(z.var() - 1) < 5 * math.sqrt(2 / n)
    assert abs((np.abs(z) < 1).mean() - 0.682689492) < 0.005
    assert abs((np.abs(z) < 2).mean() - 0.954499736) < 0.003
    assert abs(np.mean(z ** 3)) < 0.03 and abs(np.mean(z ** 4) - 3) < 0.05
    # row-major pairs: element e and e+1 (e even) share one counter
    flat = z.ravel()
    assert np.corrcoef(flat[0:-1:2], flat[1::2])[0, 1] == pytest.approx(0, abs=0.01)
    # another stream or seed gives other numbers; the same ones give the same numbers
    assert not np.allclose(z, oracle.gaussian(500, 801, seed=3, stream=1))
    assert not np.allclose(z, oracle.gaussian(500, 801, seed=4, stream=0))
    assert np.array_equal(z, oracle.gaussian(500, 801, seed=3, stream=0))
    # a prefix of a longer draw is the same draw
    assert np.array_equal(oracle.gaussian(7, 5, 9, 0).ravel(), oracle.gaussian(5, 7, 9, 0).ravel())


def planted(p, q, sigma, seed):
    rng = np.random.default_rng(seed)
    U, _ = np.linalg.qr(rng.standard_normal((p, len(sigma))))
    V, _ = np.linalg.qr(rng.standard_normal((q, len(sigma))))
    return (U * sigma) @ V.T, U, V


def test_low_rank_spectrum_is_recovered_exactly():
    """rank 12 < k: the sketch spans the whole row space, so every triplet is exact."""
    sigma = np.geomspace(50, 0.5, 12)
    M, U, V = planted(300, 80, sigma, 1)
    Ur, sr, Vr = oracle.rsvd_right(M, 10, 5, 0, seed=2, stream=0)
    np.testing.assert_allclose(sr, sigma[:10], rtol=1e-12)
    np.testing.assert_allclose(np.abs(np.sum(Vr * V[:, :10], axis=0)), 1, atol=1e-10)
    np.testing.assert_allclose((Ur * sr) @ Vr.T, (U[:, :10] * sigma[:10]) @ V[:, :10].T, atol=1e-10)


def test_ritz_bounds_and_convergence():
    """Slowly decaying planted spectrum: the Ritz values never exceed the true singular
    values (interlacing), and the error of the leading values falls with every extra pair
    of power iterations; at 11 iterations the leading five, whose convergence factor
    (sigma_26 / sigma_j)^(4*11+2) is below 1e-16, are exact to 1e-12."""
    sigma = 1.0 / np.arange(1, 121) ** 0.5
    M, _, _ = planted(400, 120, sigma, 5)
    errs = []
    for it in (0, 2, 4, 11):
        _, sr, _ = oracle.rsvd_right(M, 20, 5, it, seed=7, stream=0)
        assert np.all(sr <= sigma[:20] * (1 + 1e-13))
        errs.append(np.max((sigma[:20] - sr) / sigma[:20]))
    assert errs[0] > errs[1] > errs[2] > errs[3]
    _, sr, _ = oracle.rsvd_right(M, 20, 5, 11, seed=7, stream=0)
    np.testing.assert_allclose(sr[:5], sigma[:5], rtol=1e-12)


def test_branch_rule():
    S = oracle.InnerSolver
    assert not oracle.use_randomized(None, 10, 100)
    assert not oracle.use_randomized(S(0), 10, 100)
    assert oracle.use_randomized(S(1), 29, 100) and not oracle.use_randomized(S(1), 30, 100)
    assert oracle.use_randomized(S(2), 60, 100) and not oracle.use_randomized(S(2), 95, 100)
    assert not oracle.use_randomized(S(2), 0, 100)


def test_fastpi_with_randomized_updates():
    """Mode 0 is the exact method; mode 2 with 11 iterations stays within 0.1% of its
    reconstruction error on the 2000 x 500 workload, and keeps U orthonormal."""
    p = make_problem("c1")
    A = sp.csr_matrix((p.data, p.indices, p.indptr), shape=(p.m, p.n))
    ex = oracle.fastpi_svd(p.m, p.n, p.indptr, p.indices, p.data, 0.3, 0.01)
    e0 = oracle.fastpi_svd(p.m, p.n, p.indptr, p.indices, p.data, 0.3, 0.01, inner=oracle.InnerSolver(0))
    assert np.array_equal(ex.sigma, e0.sigma)
    rr = oracle.fastpi_svd(p.m, p.n, p.indptr, p.indices, p.data, 0.3, 0.01,
                           inner=oracle.InnerSolver(2, 5, 11, 1))
    re, rx = oracle.recon_error(A, rr.U, rr.sigma, rr.V), oracle.recon_error(A, ex.U, ex.sigma, ex.V)
    assert rx <= re <= rx * 1.001
    assert oracle.orthonormality_error(rr.U) < 1e-12


def test_library_branch_rule_matches_oracle():
    """The library's rule (C ABI, no GPU) against the oracle's on a grid of settings."""
    import paper_2011_04235_amd as fp
    fp.load()
    for mode in (0, 1, 2):
        for over in (0, 5, 40):
            for q in (1, 2, 10, 99, 100, 101, 383, 1357):
                for t in range(0, q + 2, max(1, q // 37)):
                    want = oracle.use_randomized(oracle.InnerSolver(mode, over), t, q)
                    assert fp.inner_applies(mode, over, t, q) == want, (mode, over, t, q)


def test_randomized_column_update_is_sign_invariant():
    """The row update fixes its singular vectors only up to sign; with the sign convention the
    randomized column update gives the same result for any choice of those signs (without
    it a flip changes the test matrix's draw against X3's columns)."""
    from oracle import fastpi as ofp
    p = make_problem("c1")
    inner = oracle.InnerSolver(2, 5, 3, 4)
    A = sp.csr_matrix((p.data, p.indices, p.indptr), shape=(p.m, p.n))
    R = oracle.reorder(p.m, p.n, A.indptr, A.indices, 0.01)
    S = ofp.split_blocks(p.m, p.n, A.indptr, A.indices, A.data, R)
    B = ofp.block_svd(S, 0.3)
    R2 = ofp.row_update(S, B, 0.3, inner)
    flip = np.where(np.arange(R2.sigma.size) % 3 == 1, -1.0, 1.0)
    R2f = ofp.Stage(R2.U * flip, R2.sigma, R2.V * flip, R2.full_sigma)
    a = ofp.column_update(S, R2, 0.3, p.m, p.n, inner)
    b = ofp.column_update(S, R2f, 0.3, p.m, p.n, inner)
    np.testing.assert_allclose(a.sigma, b.sigma, rtol=1e-12)
    np.testing.assert_allclose((a.U * a.sigma) @ a.V.T, (b.U * b.sigma) @ b.V.T, atol=1e-10)
    assert np.all(oracle.sign_convention(R2f.V * oracle.sign_convention(R2f.V)) == 1)
