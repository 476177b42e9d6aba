"""Pins of the geometry oracle (local frame and density jets from Gauss-Legendre
panels) against quantities fixed independently of its formulas:

* the inverse-function / Faa di Bruno step against power-series composition
  done with numpy polynomial products (sin(log(1+xi)), asinh(xi)^2);
* the circle: closest point, distance, side and the exact frame
  kappa = 1/R, gamma3 = 0, gamma4 = 3/R^3;
* the star domains of the workloads, whose frames and density jets are built
  from the analytic curve by series reversion (a different route);
* brute force: no sample of the panel interpolants lies closer to a target
  than the closest point found;
* the plain interpolant's curve derivatives and density jets on finely
  resolved circles (where the nodal rounding dominates them) stay within the
  rounding bound of tests/geometry_bounds.py against the exact values, and
  the evaluation with panel geometry moves from the analytic-geometry one by
  no more than the local expansions' response to those bounds.
"""
import numpy as np
import pytest
from numpy.polynomial import polynomial as Pm
from numpy.polynomial.legendre import leggauss

from oracle import geometry as G
from tests.geometry_bounds import frame_bounds, jet_bounds
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


def _local_response(P, geom, bounds):
    """Per target, the local parts' change (V, S, D at the oracle's default orders)
    when kappa, gamma3 and gamma4 each move by their bound, summed over the three."""
    import copy
    import oracle
    base = oracle.evaluate(P, kinds="VSD")["total"]
    acc = np.zeros(P.n_tgt)
    for k, name in enumerate(("kappa", "gamma3", "gamma4")):
        Q = copy.copy(P)
        Q.geom = dict(geom, **{name: geom[name] + bounds[k]})
        acc += np.abs(oracle.evaluate(Q, kinds="VSD")["total"] - base)
    return acc


def test_panel_geometry_error_is_the_rounding_bound():
    """The whole evaluation (history + local parts of V, S, D) with frames and
    layer jets taken from the panels against the one from the analytic curve.
    The layer jets and the frame's position and normal are float64-grade: with
    the analytic kappa, gamma3, gamma4 put back the two agree to 1e-11.  The
    curve derivatives of the plain interpolant carry the nodal coordinates'
    rounding amplified by the derivatives (gamma4 most, finer panels more); on
    this lobed star they stay within their rounding bound of the analytic
    values, and the evaluation moves by at most the local parts' response to
    those bounds (a bit over 1e-7 of the largest value here)."""
    import copy
    import oracle
    P = star_problem(1500, seed=6)
    q = P.info["q"]
    fr = G.boundary_frame(P.bnd_x, P.bnd_y, q, P.tgt_x, P.tgt_y)
    B = frame_bounds(P.bnd_x, P.bnd_y, q, fr["pan"], fr["u"], q)
    near = P.info["near_mask"]   # the workload's exact frames (farther targets only need r)
    for k, name in enumerate(("kappa", "gamma3", "gamma4")):
        assert np.all((np.abs(fr[name] - P.geom[name]) <= B[k])[near]), name
    Q = copy.copy(P)
    Q.geom = {k: fr[k] for k in ("r", "nx", "ny", "kappa", "gamma3", "gamma4", "sgn")}
    Q.sigma_jet = G.density_jets(P.bnd_x, P.bnd_y, q, P.sigma, fr["pan"], fr["u"], 2)
    Q.mu_jet = G.density_jets(P.bnd_x, P.bnd_y, q, P.mu, fr["pan"], fr["u"], 4)
    a = oracle.evaluate(P, kinds="VSD")["total"]
    b = oracle.evaluate(Q, kinds="VSD")["total"]
    resp = _local_response(P, P.geom, B)
    print("panel vs analytic geometry: e_inf", oracle.rel_linf(b, a), "response bound", np.max(resp) / np.max(np.abs(a)))
    assert np.all(np.abs(b - a) <= resp + 1e-11 * np.max(np.abs(a)))
    # with the analytic curve derivatives put back the rest is float64-grade
    Q.geom = dict(Q.geom, kappa=P.geom["kappa"], gamma3=P.geom["gamma3"], gamma4=P.geom["gamma4"])
    e2 = oracle.rel_linf(oracle.evaluate(Q, kinds="VSD")["total"], a)
    print("with analytic curve derivatives: e_inf", e2)
    assert e2 <= 1e-11


def _circle_xi_jets(R, tb):
    """xi-derivatives 0..4 at b = R(cos tb, sin tb) of mu = cos 3t on the circle
    of radius R: along the tangent line t = tb + asin(xi/R), and the series of
    cos(3 tb + 3 asin(xi/R)) through xi^4 gives these."""
    ca, sa = np.cos(3 * tb), np.sin(3 * tb)
    return np.stack([ca, -3 * sa / R, -9 * ca / R ** 2, 24 * sa / R ** 3, 45 * ca / R ** 4])


@pytest.mark.parametrize("R,shift,n_pan", [(3.0, 0.0, 4400), (3.0, 50.0, 4400), (1.3, 0.0, 24)])
def test_plain_interpolant_within_rounding_bound_on_circles(R, shift, n_pan):
    """On circles the exact frame is kappa = 1/R, gamma3 = 0, gamma4 = 3/R^3.
    At 4400 panels of 16 (70,400 nodes, panels 4.3e-3 long) the nodal
    coordinates' rounding dominates the interpolant's higher derivatives
    (gamma4 wrong by up to ~5e3 at the origin, ~8e4 shifted by 50); each error
    stays within the rounding bound (q ulps of the panel's largest coordinate
    per Legendre coefficient) and reaches about a third of it."""
    q = 16
    xg, _ = leggauss(q)
    e = np.linspace(0, 2 * np.pi, n_pan + 1)
    t = (0.5 * (e[:-1, None] + e[1:, None]) + 0.5 * (e[1:, None] - e[:-1, None]) * xg[None]).ravel()
    bx, by = shift + R * np.cos(t), R * np.sin(t)
    k = np.random.default_rng(0).choice(bx.size, 150, replace=False)
    tx, ty = bx[k] - 0.01 * np.cos(t[k]), by[k] - 0.01 * np.sin(t[k])
    fr = G.boundary_frame(bx, by, q, tx, ty)
    B = frame_bounds(bx, by, q, fr["pan"], fr["u"], q)
    err = np.abs(np.stack([fr["kappa"] - 1 / R, fr["gamma3"], fr["gamma4"] - 3 / R ** 3]))
    print("R", R, "shift", shift, "panels", n_pan, "max error / bound", np.max(err / B, axis=1),
          "max error", np.max(err, axis=1))
    assert np.all(err <= B)
    mu = np.cos(3 * t)
    mj = G.density_jets(bx, by, q, mu, fr["pan"], fr["u"], 4)
    Bj = jet_bounds(bx, by, q, mu, fr["pan"], fr["u"], q)
    ex = _circle_xi_jets(R, np.arctan2(ty, tx - shift))
    # derivatives 1..4 at the found closest point (the value itself also moves with b's position)
    assert np.all(np.abs(mj[1:] - ex[1:]) <= Bj[1:])
