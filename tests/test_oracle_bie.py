"""Pins of the Dirichlet-solve oracle (double-layer representation, operator
D_int assembled from the method's evaluation at the boundary nodes):

* Gauss: D_int[1] = -1;
* the unit circle in closed form: D[cos n t] = -r^n cos(n t) / 2 inside, so
  D_int[mu] = cos(n t) has mu = -2 cos(n t), and u = r^n cos(n t) inside;
* a lobed star: u = Re((z - z0)^3) + linear recovered inside;
* every error falls with refinement of the panels (delta_1 ~ spacing^2).
"""
import numpy as np
from numpy.polynomial.legendre import leggauss

from oracle import bie
from workloads.problems import StarCurve, panel_nodes, star_params


def _circle(n_pan, q=16):
    xg, wg = leggauss(q)
    e = np.linspace(0, 2 * np.pi, n_pan + 1)
    a, b = e[:-1, None], e[1:, None]
    t = (0.5 * (a + b) + 0.5 * (b - a) * xg[None]).ravel()
    w = (0.5 * (b - a) * wg[None]).ravel()
    return np.cos(t), np.sin(t), np.cos(t), np.sin(t), w, t


def _circle_errors(n_pan):
    bx, by, nx, ny, w, t = _circle(n_pan)
    P = bie.on_boundary_problem(bx, by, nx, ny, w, 16)
    gauss = np.max(np.abs(bie.apply_interior_double_layer(P, np.ones(bx.size)) + 1.0))
    g = np.cos(3 * t)
    mu = bie.solve_dirichlet(P, g)
    rng = np.random.default_rng(0)
    th, rr = rng.uniform(0, 2 * np.pi, 100), rng.uniform(0.1, 0.95, 100)
    u = bie.double_layer_at(P, mu, rr * np.cos(th), rr * np.sin(th))
    return gauss, np.max(np.abs(mu + 2 * g)), np.max(np.abs(u - rr ** 3 * np.cos(3 * th)))


def test_circle_closed_forms_and_convergence():
    coarse = _circle_errors(16)
    fine = _circle_errors(32)
    print("circle errors (gauss, mu, u): 16 panels", coarse, "32 panels", fine)
    assert fine[0] <= 1e-9 and fine[1] <= 5e-7 and fine[2] <= 2e-6
    assert all(f <= c / 10 for f, c in zip(fine, coarse))


def test_star_harmonic_recovered():
    curve = StarCurve(**star_params(3, r=0.8))
    bx, by, bnx, bny, bw, _ = panel_nodes(curve, 24, 16)
    P = bie.on_boundary_problem(bx, by, bnx, bny, bw, 16)
    z0 = complex(0.1, -0.05)

    def uex(x, y):
        return ((x + 1j * y - z0) ** 3).real + 0.3 * x - 0.2 * y + 1.0

    mu = bie.solve_dirichlet(P, uex(bx, by))
    rng = np.random.default_rng(1)
    k = rng.integers(0, bx.size, 200)
    s = rng.uniform(0.3, 0.97, 200)
    cx, cy = np.mean(bx), np.mean(by)
    tx, ty = cx + s * (bx[k] - cx), cy + s * (by[k] - cy)
    e = np.max(np.abs(bie.double_layer_at(P, mu, tx, ty) - uex(tx, ty)))
    print("star: interior error", e)
    assert e <= 1e-4
