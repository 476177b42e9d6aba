"""Pins of the per-triangle quadratic jets of the volume density:

* exact for quadratic f (all six jet rows, any triangle shape);
* for a Gaussian, against its analytic jets: the gradient error falls like
  h^2 and the Hessian's like h (halving h: at least 3x and 1.6x);
* the volume potential evaluated with them approaches the one with analytic
  jets (the local part is the only consumer), at least 10x per halving of h.
"""
import copy

import numpy as np

import oracle
from oracle.volume_jets import p2_jets
from workloads.problems import disk_problem

GAUSS = ((1.0, 0.0, 0.0, np.sqrt(0.1)),)


def test_quadratic_exact():
    D = disk_problem(2000, seed=1, gauss=GAUSS)
    rng = np.random.default_rng(0)
    c = rng.standard_normal(6)
    x, y = D.src_x, D.src_y
    J = p2_jets(x, y, c[0] + c[1] * x + c[2] * y + c[3] * x * x + c[4] * x * y + c[5] * y * y)
    ex = np.stack([c[0] + c[1] * x + c[2] * y + c[3] * x * x + c[4] * x * y + c[5] * y * y,
                   c[1] + 2 * c[3] * x + c[4] * y, c[2] + c[4] * x + 2 * c[5] * y,
                   np.full(x.size, 2 * c[3]), np.full(x.size, c[4]), np.full(x.size, 2 * c[5])])
    assert np.max(np.abs(J - ex)) <= 1e-10


def test_gaussian_convergence_and_volume_potential():
    rng = np.random.default_rng(1)
    errs, vdiff = [], []
    for n in (2000, 8000):
        D = disk_problem(n, seed=1, gauss=GAUSS)
        J = p2_jets(D.src_x, D.src_y, D.f_src)
        errs.append(np.max(np.abs(J - D.jet6), axis=1))
        idx = np.sort(rng.choice(D.n_tgt, 2000, replace=False))
        S = D.subset_targets(idx)
        a = oracle.evaluate(S, kinds="V")["total"]
        S2 = copy.copy(S)
        S2.jet6 = J[:, idx]
        vdiff.append(oracle.rel_linf(oracle.evaluate(S2, kinds="V")["total"], a))
    print("jet errors (coarse, fine):", errs, "V differences:", vdiff)
    assert errs[0][0] == 0.0 and errs[1][0] == 0.0
    assert np.all(errs[0][1:3] / errs[1][1:3] >= 3.0)
    assert np.all(errs[0][3:] / errs[1][3:] >= 1.6)
    assert vdiff[1] <= vdiff[0] / 10 and vdiff[1] <= 2e-6
