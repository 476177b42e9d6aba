"""Pins of the per-triangle quadratic jets of the volume density:

* exact for quadratic f (all six jet rows, any triangle shape);
* for a Gaussian, against its analytic jets: the gradient error falls like
  h^2 and the Hessian's like h (halving h: at least 3x and 1.6x);
* the volume potential evaluated with them approaches the one with analytic
  jets (the local part is the only consumer), at least 10x per halving of h.

and of the patch jets (least squares over a triangle and its edge neighbours):
exact for quadratics on a mesh with slivers, equal to the interpolant without
neighbours, and converging on the slivers for a Gaussian.
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


# ---------------------------------------------------------------------------
# Patch jets: the least-squares quadratic over a triangle and its edge
# neighbours (the six nodes of a sliver do not fix the derivatives across it).

def _slivers(x, y):
    """Per node: True on triangles whose node spread has an axis ratio below 0.1."""
    X, Y = x.reshape(-1, 6), y.reshape(-1, 6)
    dx, dy = X - X.mean(1, keepdims=True), Y - Y.mean(1, keepdims=True)
    sxx, syy, sxy = (dx * dx).sum(1), (dy * dy).sum(1), (dx * dy).sum(1)
    rad = np.sqrt((0.5 * (sxx - syy)) ** 2 + sxy ** 2)
    l1, l2 = 0.5 * (sxx + syy) + rad, 0.5 * (sxx + syy) - rad
    return np.repeat(np.sqrt(np.maximum(l2, 0) / np.maximum(l1, 1e-300)) < 0.1, 6)


def test_patch_quadratic_exact_on_slivers():
    from oracle.volume_jets import patch_jets
    from workloads.mesh import square_mesh, triangle_neighbours
    x, y, _, info = square_mesh(3000, 5, 400)
    nbr = triangle_neighbours(info["tri"])
    rng = np.random.default_rng(2)
    c = rng.standard_normal(6)
    f = c[0] + c[1] * x + c[2] * y + c[3] * x * x + c[4] * x * y + c[5] * y * y
    J = patch_jets(x, y, f, nbr)
    ex = np.stack([f, c[1] + 2 * c[3] * x + c[4] * y, c[2] + c[4] * x + 2 * c[5] * y,
                   np.full(x.size, 2 * c[3]), np.full(x.size, c[4]), np.full(x.size, 2 * c[5])])
    assert np.all(np.isfinite(J))
    assert _slivers(x, y).sum() > 100 * 6
    assert np.max(np.abs(J - ex)) <= 1e-8


def test_patch_without_neighbours_is_the_interpolant():
    from oracle.volume_jets import patch_jets
    D = disk_problem(2000, seed=1, gauss=GAUSS)
    nbr = np.full((D.src_x.size // 6, 3), -1, np.int32)
    J = patch_jets(D.src_x, D.src_y, D.f_src, nbr)
    I = p2_jets(D.src_x, D.src_y, D.f_src)
    assert np.max(np.abs(J - I) / np.maximum(np.max(np.abs(I), axis=1, keepdims=True), 1e-300)) <= 1e-9


def test_patch_gaussian_on_slivers_converges():
    """On the split square mesh the slivers' jets are as accurate as the
    well-shaped triangles' and converge: gradient like h^2, Hessian like h."""
    from oracle.volume_jets import patch_jets
    from workloads.mesh import square_mesh, triangle_neighbours
    from workloads.problems import gauss_jets
    G = ((1.0, 0.1, -0.2, 0.3),)
    errs = []
    for n in (4000, 16000):
        x, y, _, info = square_mesh(n, 3, n // 9)
        ex = gauss_jets(x, y, G)
        J = patch_jets(x, y, ex[0], triangle_neighbours(info["tri"]))
        sl = _slivers(x, y) & np.all(np.isfinite(J), 0)
        errs.append([np.max(np.abs(J[k][sl] - ex[k][sl])) / np.max(np.abs(ex[k])) for k in range(1, 6)])
    errs = np.array(errs)
    print("sliver jet errors (coarse, fine):", errs)
    assert np.all(errs[0, :2] <= 0.02) and np.all(errs[0, 2:] <= 0.6)
    assert np.all(errs[0, :2] / errs[1, :2] >= 2.5)
    assert np.all(errs[0, 2:] / errs[1, 2:] >= 1.5)
