"""Writes tests/golden/rank_dataset.npz: features and Eckart-Young labels of the dense
diagonal blocks of seeded synthetic matrices, computed by the oracle only.

Instance i (seed 100000 + i) draws m log-uniform in [2000, 12000], n log-uniform in
[300, 1500], density U[0.002, 0.01], power-law exponent U[1.8, 2.3], lognormal values and
alpha from {0.1, 0.2, 0.3}; k = 0.01. For every instance the label of block i is the kept
fraction s_i* / min(m_i, n_i) of the Eckart-Young allocation at the alpha rule's total
budget (see oracle.rank). Instances 0..23 train, 24..31 validate.
"""
import math
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import rank as orank  # noqa: E402
from synth import make_problem, small_config  # noqa: E402

N_INSTANCES = 32
N_TRAIN = 24


def instance_config(i):
    rng = np.random.default_rng(100000 + i)
    m = int(round(math.exp(rng.uniform(math.log(2000), math.log(12000)))))
    n = int(round(math.exp(rng.uniform(math.log(300), math.log(1500)))))
    density = float(rng.uniform(0.002, 0.01))
    gamma = float(rng.uniform(1.8, 2.3))
    alpha = float(rng.choice([0.1, 0.2, 0.3]))
    return small_config(m, n, density, gamma=gamma, values="lognormal", L=4, p_label=0.1,
                        alpha=alpha, seed=100000 + i, k=0.01, name=f"r{i}")


def main():
    X, Y, INST, Q, SA, SY = [], [], [], [], [], []
    for i in range(N_INSTANCES):
        cfg = instance_config(i)
        p = make_problem(cfg, with_labels=False)
        feats, spectra, alpha_ranks, shapes = orank.problem_blocks(p.m, p.n, p.indptr, p.indices,
                                                                    p.data, cfg.alpha, cfg.k)
        budget = int(alpha_ranks.sum())
        ey = orank.eckart_young_ranks(spectra, budget)
        q = np.minimum(shapes[:, 0], shapes[:, 1])
        X.append(feats)
        Y.append(ey / q)
        INST.append(np.full(len(q), i))
        Q.append(q)
        SA.append(alpha_ranks)
        SY.append(ey)
        print(f"instance {i}: {p.m}x{p.n} alpha {cfg.alpha} blocks {len(q)} budget {budget}")
    np.savez_compressed(os.path.join(HERE, "rank_dataset.npz"),
                        X=np.concatenate(X), y=np.concatenate(Y), instance=np.concatenate(INST),
                        q=np.concatenate(Q), s_alpha=np.concatenate(SA), s_ey=np.concatenate(SY),
                        n_train=N_TRAIN)


if __name__ == "__main__":
    main()
