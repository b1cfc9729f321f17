"""Pins of the rank-predictor oracle: finite differences, a closed-form Adam step,
Eckart-Young on the whole block-diagonal matrix, hand-computed features."""
import math

import numpy as np
import scipy.linalg as sla

from oracle import rank as orank


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(0)
    theta = orank.init_params(3)
    X = rng.standard_normal((40, orank.N_FEATURES))
    y = rng.random(40)
    g = orank.gradient(theta, X, y)
    h = 1e-6
    idx = rng.choice(orank.N_PARAMS, 60, replace=False)
    idx = np.concatenate([idx, [0, 1023, 1024, 1087, 1088, 5183, 5184, 5247, 5248, 5311, 5312]])
    for i in idx:
        e = np.zeros_like(theta); e[i] = h
        fd = (orank.loss(theta + e, X, y) - orank.loss(theta - e, X, y)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 + 1e-5 * abs(fd), (i, fd, g[i])


def test_parameter_count_and_layout():
    assert orank.N_PARAMS == 5313
    W1, b1, W2, b2, W3, b3 = orank.unpack(np.arange(orank.N_PARAMS, dtype=float))
    assert W1.shape == (64, 16) and W2.shape == (64, 64) and W3.shape == (64,)
    assert b3 == 5312 and W2[0, 0] == 1088


def test_adam_first_step_closed_form():
    # at step 1 the bias-corrected moments are g and g^2: the update is -lr g / (|g| + eps)
    theta = np.array([1.0, -2.0, 0.5]); g = np.array([0.3, -4.0, 0.0])
    t1, m, v = orank.adam_step(theta, g, np.zeros(3), np.zeros(3), 1, 0.01)
    assert np.allclose(t1, theta - 0.01 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_eckart_young_ranks_are_optimal_for_the_block_diagonal_matrix():
    rng = np.random.default_rng(1)
    blocks = [rng.lognormal(size=(rng.integers(1, 9), rng.integers(1, 6))) for _ in range(12)]
    spectra = [np.linalg.svd(b, compute_uv=False) for b in blocks]
    budget = 15
    ranks = orank.eckart_young_ranks(spectra, budget)
    assert ranks.sum() == budget
    full = sla.block_diag(*blocks)
    lam = np.sort(np.linalg.eigvalsh(full.T @ full))[::-1]
    opt = float(np.sum(np.clip(lam[budget:], 0, None)))
    assert abs(orank.truncation_error2(spectra, ranks) - opt) <= 1e-9 * max(opt, 1.0)
    # no other allocation with the same total does better
    lens = np.array([len(s) for s in spectra])
    for trial in range(50):
        alloc = np.zeros(len(spectra), dtype=int)
        for _ in range(budget):
            free = np.flatnonzero(alloc < lens)
            alloc[rng.choice(free)] += 1
        assert orank.truncation_error2(spectra, ranks) <= orank.truncation_error2(spectra, alloc) + 1e-12


def test_features_of_a_hand_block():
    A = np.array([[3.0, 1.0], [4.0, 0.0]])
    f = orank.block_features(A, 0.3, 10, 52.0, 5, 3, 12)
    want = [math.log(2), math.log(2), math.log(3), 0.75, math.log(26), math.log(25), math.log(1),
            (math.log(25) + 0.0) / 2, math.log(25) / 2, math.log(16), 26 / 25, 0.5, 0.3, 0.2,
            math.log(6), 0.25]
    assert np.allclose(f, want, rtol=0, atol=1e-12)
