"""Learned per-block rank allocation (the learned form of Eq. 1's rank rule).

Eq. 1 keeps ceil(alpha n_i) directions of every diagonal block. A 16-64-64-1 network,
trained on the GPU by the library's own forward, backward and Adam kernels, predicts from
cheap block features (fastpi_block_features) the fraction of a block's directions that the
Eckart-Young allocation at the same total budget would keep. The predictions are turned into
integer ranks with exactly the alpha rule's total s_b; blocks whose features fall outside the
training range keep the alpha rule's rank (the fallback). The standardisation, the range test
and the budgeted allocation are library calls (fastpi_rank_inputs, fastpi_rank_allocate,
fastpi_plan_learned_ranks) and the network runs in HIP kernels; this module only keeps the
parameters and the training statistics and marshals them.
"""
from __future__ import annotations

import numpy as np

from . import _lib

N_FEATURES = 16
N_PARAMS = 5313


def init_params(seed: int) -> np.ndarray:
    """U(-1/sqrt(fan_in), 1/sqrt(fan_in)) per layer, weights then biases, from one PCG64
    stream (float32)."""
    rng = np.random.default_rng(seed)
    parts = []
    for fan_in, size in ((16, 64 * 16), (16, 64), (64, 64 * 64), (64, 64), (64, 64), (64, 1)):
        lim = 1.0 / np.sqrt(fan_in)
        parts.append(rng.uniform(-lim, lim, size=size))
    return np.concatenate(parts).astype(np.float32)


class RankPredictor:
    def __init__(self, theta=None, mean=None, std=None, lo=None, hi=None):
        self.theta = None if theta is None else np.asarray(theta, np.float32)
        self.mean = mean
        self.std = std
        self.lo = lo
        self.hi = hi

    # ---------------------------------------------------------------- training ----------
    def fit(self, handle, X, y, epochs=400, lr=3e-3, seed=0, log_every=0):
        """Full-batch Adam on the mean squared error, on the handle's device."""
        torch = handle.torch
        X = np.asarray(X, np.float64)
        self.mean = X.mean(axis=0)
        self.std = np.where(X.std(axis=0) > 0, X.std(axis=0), 1.0)
        self.lo = X.min(axis=0)
        self.hi = X.max(axis=0)
        dev = handle.device
        Xd = torch.from_numpy(self._standardise(X)).to(dev)
        yd = torch.from_numpy(np.asarray(y, np.float32)).to(dev)
        th = torch.from_numpy(init_params(seed)).to(dev)
        m = torch.zeros_like(th)
        v = torch.zeros_like(th)
        g = torch.empty_like(th)
        history = []
        for step in range(1, epochs + 1):
            handle.mlp_gradient(Xd, yd, th, out=g)
            handle.mlp_adam(th, g, m, v, step, lr)
            if log_every and (step % log_every == 0 or step == epochs):
                f = handle.mlp_forward(Xd, th)
                history.append((step, float(((f - yd) ** 2).mean())))
        self.theta = th.cpu().numpy()
        return history

    MARGIN = 0.05

    def _model(self):
        return (self.mean, self.std, self.lo, self.hi, self.MARGIN)

    def _standardise(self, X):
        return _lib.rank_inputs(X, *self._model())[0]

    def predict(self, handle, X):
        torch = handle.torch
        if len(X) == 0:
            return np.zeros(0, np.float32)
        Xd = torch.from_numpy(self._standardise(X)).to(handle.device)
        th = torch.from_numpy(self.theta).to(handle.device)
        return handle.mlp_forward(Xd, th).cpu().numpy()

    def in_range(self, X):
        return _lib.rank_inputs(X, *self._model())[1]

    def block_ranks(self, handle, plan, data):
        """Ranks for every block of the plan's block table (fastpi_plan_learned_ranks):
        predictions for in-range dense blocks, the alpha rule for the others, at the alpha
        rule's total budget."""
        th = handle.torch.from_numpy(self.theta).to(handle.device)
        return plan.learned_ranks(handle, data, th, *self._model())

    def save(self, path):
        np.savez(path, theta=self.theta, mean=self.mean, std=self.std, lo=self.lo, hi=self.hi)

    @classmethod
    def load(cls, path):
        d = np.load(path)
        return cls(d["theta"], d["mean"], d["std"], d["lo"], d["hi"])
