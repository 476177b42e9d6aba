"""Pins of the geometry oracle (local frame and density jets from Gauss-Legendre
panels) against quantities fixed independently of its formulas:

* the inverse-function / Faa di Bruno step against power-series composition
  done with numpy polynomial products (sin(log(1+xi)), asinh(xi)^2);
* the circle: closest point, distance, side and the exact frame
  kappa = 1/R, gamma3 = 0, gamma4 = 3/R^3;
* the star domains of the workloads, whose frames and density jets are built
  from the analytic curve by series reversion (a different route);
* brute force: no sample of the panel interpolants lies closer to a target
  than the closest point found.
"""
import numpy as np
import pytest
from numpy.polynomial import polynomial as Pm
from numpy.polynomial.legendre import leggauss

from oracle import geometry as G
from workloads import star_problem


def _series_derivs(c, n=5):
    """k! c_k: derivatives at 0 of the power series with coefficients c."""
    from math import factorial
    c = np.concatenate([c, np.zeros(n)])[:n]
    return np.array([factorial(k) * c[k] for k in range(n)])


def test_inverse_chain_matches_series_composition():
    # xi(u) = e^u - 1 at u = 0 (all derivatives 1); h(u) = sin u; h(u(xi)) = sin(log(1 + xi))
    lg = np.array([0.0, 1.0, -1 / 2, 1 / 3, -1 / 4])          # log(1 + xi)
    z3 = Pm.polymul(Pm.polymul(lg, lg), lg)[:5]
    z5 = Pm.polymul(Pm.polymul(z3, lg), lg)[:5]
    comp = lg - z3 / 6 + np.concatenate([z5, np.zeros(5)])[:5] / 120
    want = _series_derivs(comp)
    got = G.inverse_chain(np.array([0, 1, 1, 1, 1.0]), np.array([0, 1, 0, -1, 0.0]))
    assert np.allclose(got, want, rtol=1e-14, atol=1e-14)
    # xi(u) = sinh u, h(u) = u^2: asinh(xi)^2 = xi^2 - xi^4/3 + ...
    got = G.inverse_chain(np.array([0, 1, 0, 1, 0.0]), np.array([0, 0, 2, 0, 0.0]))
    assert np.allclose(got, [0, 0, 2, 0, -8], atol=1e-14)


def _circle_panels(R, c, n_pan, q):
    xg, _ = leggauss(q)
    e = np.linspace(0, 2 * np.pi, n_pan + 1)
    t = (0.5 * (e[:-1, None] + e[1:, None]) + 0.5 * (e[1:, None] - e[:-1, None]) * xg[None]).ravel()
    return c[0] + R * np.cos(t), c[1] + R * np.sin(t), t


def test_circle_frame_is_exact():
    R, c, q = 1.3, (0.2, -0.1), 16
    bx, by, t = _circle_panels(R, c, 24, q)
    rng = np.random.default_rng(3)
    ang = rng.uniform(0, 2 * np.pi, 400)
    rad = R * np.concatenate([rng.uniform(0.2, 0.999, 200), rng.uniform(1.001, 2.0, 200)])
    tx = np.concatenate([c[0] + rad * np.cos(ang), bx[:5]])
    ty = np.concatenate([c[1] + rad * np.sin(ang), by[:5]])
    fr = G.boundary_frame(bx, by, q, tx, ty)
    d = np.hypot(tx - c[0], ty - c[1])
    assert np.allclose(fr["r"], np.abs(R - d), rtol=0, atol=1e-13)
    assert np.allclose(fr["nx"][:-5], (tx - c[0])[:-5] / d[:-5], atol=1e-12)
    assert np.allclose(fr["ny"][:-5], (ty - c[1])[:-5] / d[:-5], atol=1e-12)
    assert np.array_equal(fr["sgn"][:-5], np.where(d[:-5] < R, 1, -1))
    assert np.all(fr["sgn"][-5:] == 0) and np.all(fr["r"][-5:] <= 1e-13)
    # higher derivatives of the interpolant carry the nodal rounding amplified
    # by P_k^(m)(+-1) ~ k^(2m) near the panel ends and by |x'|^-m (panels of
    # 0.17 here): ~1e-7 in gamma3, ~1e-5 in gamma4 -- which enter the local
    # expansions only times delta^(3/2) and delta^2
    assert np.allclose(fr["kappa"], 1 / R, atol=1e-9)
    assert np.allclose(fr["gamma3"], 0.0, atol=2e-6)
    assert np.allclose(fr["gamma4"], 3 / R ** 3, atol=2e-4)


@pytest.mark.parametrize("seed", [4, 5, 9])
def test_star_frames_and_jets_match_series_reversion(seed):
    P = star_problem(3000, seed=seed)
    near = P.info["near_mask"]
    idx = np.flatnonzero(near)[:800]
    q = P.info["q"]
    fr = G.boundary_frame(P.bnd_x, P.bnd_y, q, P.tgt_x[idx], P.tgt_y[idx])
    g = P.geom
    # the panel interpolant (16-point panels, ~95 of them round a lobed star)
    # stands in for the exact curve: positions to ~1e-14; each further
    # derivative loses about two to three digits (measured: kappa 1e-8,
    # gamma3 2e-6, gamma4 1e-4 relative); bounds with a tenfold margin
    def rel(a, b):
        return np.max(np.abs(a - b)) / np.max(np.abs(b))
    assert np.max(np.abs(fr["r"] - g["r"][idx])) <= 1e-13
    assert np.max(np.abs(fr["nx"] - g["nx"][idx])) <= 1e-10
    assert np.max(np.abs(fr["ny"] - g["ny"][idx])) <= 1e-10
    assert np.array_equal(fr["sgn"], g["sgn"][idx])
    assert rel(fr["kappa"], g["kappa"][idx]) <= 1e-7
    assert rel(fr["gamma3"], g["gamma3"][idx]) <= 2e-5
    assert rel(fr["gamma4"], g["gamma4"][idx]) <= 1e-3
    sj = G.density_jets(P.bnd_x, P.bnd_y, q, P.sigma, fr["pan"], fr["u"], 2)
    mj = G.density_jets(P.bnd_x, P.bnd_y, q, P.mu, fr["pan"], fr["u"], 4)
    for k, tol in enumerate((1e-11, 1e-9, 1e-6)):
        assert rel(sj[k], P.sigma_jet[k][idx]) <= tol, (k, rel(sj[k], P.sigma_jet[k][idx]))
    for k, tol in enumerate((1e-11, 1e-9, 1e-6, 2e-5, 1e-3)):
        assert rel(mj[k], P.mu_jet[k][idx]) <= tol, (k, rel(mj[k], P.mu_jet[k][idx]))


def test_closest_point_beats_dense_sampling():
    P = star_problem(1500, seed=4)
    q = P.info["q"]
    rng = np.random.default_rng(8)
    k = rng.integers(0, P.n_bnd, 60)
    off = rng.normal(0, 0.05, (60, 2))
    tx, ty = P.bnd_x[k] + off[:, 0], P.bnd_y[k] + off[:, 1]
    fr = G.boundary_frame(P.bnd_x, P.bnd_y, q, tx, ty)
    n_pan = P.n_bnd // q
    xg, _ = leggauss(q)
    uu = np.linspace(-1, 1, 801)
    from numpy.polynomial import legendre as L
    pts = []
    for p in range(n_pan):
        cx = L.legfit(xg, P.bnd_x[p * q:(p + 1) * q], q - 1)
        cy = L.legfit(xg, P.bnd_y[p * q:(p + 1) * q], q - 1)
        pts.append(np.stack([L.legval(uu, cx), L.legval(uu, cy)], 1))
    pts = np.concatenate(pts)
    dmin = np.min(np.hypot(pts[None, :, 0] - tx[:, None], pts[None, :, 1] - ty[:, None]), axis=1)
    assert np.all(fr["r"] <= dmin + 1e-13)
    assert np.all(dmin - fr["r"] <= 1e-5)   # the samples are 1/400 of a panel apart


def test_panel_geometry_serves_the_method_at_fp64_tolerance():
    """The whole evaluation (history + local parts of V, S, D) with frames and
    layer jets taken from the panels agrees with the one from the analytic
    curve: the layer jets are float64-grade, and the curve's fourth derivative,
    which the double layer's local part uses, is limited by the nodal
    coordinates' rounding amplified by the panel interpolant (finer panels
    amplify it more): ~1.5e-9 on this lobed star (gamma4 up to 7e3)."""
    import copy
    import oracle
    P = star_problem(1500, seed=6)
    q = P.info["q"]
    fr = G.boundary_frame(P.bnd_x, P.bnd_y, q, P.tgt_x, P.tgt_y)
    Q = copy.copy(P)
    Q.geom = {k: fr[k] for k in ("r", "nx", "ny", "kappa", "gamma3", "gamma4", "sgn")}
    Q.sigma_jet = G.density_jets(P.bnd_x, P.bnd_y, q, P.sigma, fr["pan"], fr["u"], 2)
    Q.mu_jet = G.density_jets(P.bnd_x, P.bnd_y, q, P.mu, fr["pan"], fr["u"], 4)
    a = oracle.evaluate(P, kinds="VSD")["total"]
    b = oracle.evaluate(Q, kinds="VSD")["total"]
    e = oracle.rel_linf(b, a)
    print("panel vs analytic geometry: e_inf", e)
    assert e <= 5e-9
    # without the curve's derivatives (analytic kappa, gamma3, gamma4) the rest is float64-grade
    Q.geom = dict(Q.geom, kappa=P.geom["kappa"], gamma3=P.geom["gamma3"], gamma4=P.geom["gamma4"])
    e2 = oracle.rel_linf(oracle.evaluate(Q, kinds="VSD")["total"], a)
    print("with analytic curve derivatives: e_inf", e2)
    assert e2 <= 1e-11
