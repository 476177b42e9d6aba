"""Writes disk2m_v_oracle_sample.npz: the oracle's V[f] at a stratified seeded
sample of the disk-2M workload's targets (the unit disk at ~2M triangles,
~12M volume nodes = targets, f = exp(-|x|^2/0.1)).

Calls only the workload generator and oracle/ (direct sums plus the local
expansions, float64).  5000 targets lie within 12 sqrt(delta_1) of the circle,
where the local part acts, and 5000 farther in; their coordinates are stored
too, so that a test can check it regenerates the same targets.  Takes a few
minutes on 8 cores:

    python tests/golden/make_disk2m_oracle_sample.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

N_NEAR = N_FAR = 5000
SEED = 2024


def sample_indices(P, delta1):
    rng = np.random.default_rng(SEED)
    near = P.geom["r"] <= 12.0 * np.sqrt(delta1)
    a = rng.choice(np.flatnonzero(near), N_NEAR, replace=False)
    b = rng.choice(np.flatnonzero(~near), N_FAR, replace=False)
    return np.sort(np.concatenate([a, b]))


def main():
    import oracle
    from workloads import config_problem
    P = config_problem(3)
    d1 = oracle.delta1_of(P)
    idx = sample_indices(P, d1)
    v = oracle.evaluate(P.subset_targets(idx), kinds="V")["V"]
    np.savez_compressed(os.path.join(HERE, "disk2m_v_oracle_sample.npz"), idx=idx, x=P.tgt_x[idx],
                        y=P.tgt_y[idx], v=v, delta1=d1, n_tgt=P.n_tgt)
    print("wrote", idx.size, "values; delta_1", d1)


if __name__ == "__main__":
    main()
