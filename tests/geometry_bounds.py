"""Rounding bounds for frames and jets taken from Gauss-Legendre panels.

Test infrastructure (imported by the geometry tests, CPU and GPU).  The frame
of Sec. 4 (kappa, gamma3, gamma4) and the densities' xi-derivatives come from
each panel's degree q-1 interpolant.  Two computations of that interpolant
whose Legendre coefficients differ by at most dc on a panel (rounding of the
nodal values, two ways of computing the coefficients, or coefficients below
a floor set to zero) give u-derivatives that differ by at most

    |d^m/du^m (sum_k dc_k P_k)(u)| <= dc * S_m(u),   S_m(u) = sum_{k<q} |P_k^(m)(u)|,

and the frame and jets follow from those u-derivatives by a smooth map
(tangent rotation, then the inverse function of xi(u) and Faa di Bruno).
That map is linearised here by complex-step differentiation, and its
absolute Jacobian times the u-derivative bounds, doubled for the neglected
second-order terms, bounds each result per target.

Coefficient bounds used by the tests (eps = 2^-52, M = max |value| on the panel):
* nodal rounding passed through the interpolant: the coefficient of P_k is
  (2k+1)/2 sum_j w_j P_k(x_j) f_j, so a change of at most eps M / 2 in each f_j
  moves it by at most (k + 1/2) eps M <= q eps M;
* a second computation of the coefficients (the other side's own rounding):
  another q eps M;
* a floor that zeroes coefficients below 4 q eps M: at most 4 q eps M.
"""
import numpy as np
from numpy.polynomial import legendre as L

EPS = np.finfo(float).eps


def legendre_abs_sums(q, u, nmax=4):
    """S[m, i] = sum_{k<q} |P_k^(m)(u_i)|, m = 0..nmax."""
    u = np.asarray(u, float)
    S = np.zeros((nmax + 1, u.size))
    for k in range(q):
        c = np.zeros(k + 1)
        c[k] = 1.0
        d = c
        for m in range(nmax + 1):
            if d.size:
                S[m] += np.abs(L.legval(u, d))
            d = L.legder(d)
    return S


def _panel_max(vals, q, pan):
    v = np.abs(np.asarray(vals, float)).reshape(-1, q).max(axis=1)
    return v[np.asarray(pan)]


def _derivs(c, u, nmax=4):
    """[n_targets, nmax+1] u-derivatives of the Legendre series c[n_targets, q]."""
    out = np.zeros((u.size, nmax + 1))
    for i in range(u.size):
        d = c[i]
        for m in range(nmax + 1):
            out[i, m] = L.legval(u[i], d) if d.size else 0.0
            d = L.legder(d)
    return out


def _chain(dx, dy, ds=None):
    """(kappa, gamma3, gamma4) from coordinate u-derivatives, or with ds the
    density's xi-derivatives 0..4; complex-analytic in its arguments."""
    sp = np.sqrt(dx[1] * dx[1] + dy[1] * dy[1])
    tx, ty = dx[1] / sp, dy[1] / sp
    nx, ny = ty, -tx
    xi = [dx[m] * tx + dy[m] * ty for m in range(5)]
    h = ds if ds is not None else [-(dx[m] * nx + dy[m] * ny) for m in range(5)]
    x1, x2, x3, x4 = xi[1], xi[2], xi[3], xi[4]
    u1 = 1.0 / x1
    u2 = -x2 / x1 ** 3
    u3 = (3 * x2 * x2 - x1 * x3) / x1 ** 5
    u4 = (-15 * x2 ** 3 + 10 * x1 * x2 * x3 - x1 * x1 * x4) / x1 ** 7
    g1 = h[1] * u1
    g2 = h[2] * u1 ** 2 + h[1] * u2
    g3 = h[3] * u1 ** 3 + 3 * h[2] * u1 * u2 + h[1] * u3
    g4 = h[4] * u1 ** 4 + 6 * h[3] * u1 ** 2 * u2 + h[2] * (3 * u2 * u2 + 4 * u1 * u3) + h[1] * u4
    if ds is not None:
        return np.array([h[0], g1, g2, g3, g4])
    return np.array([g2, g3, g4])


def _propagate(args, bounds):
    """2 * sum_j |d out / d arg_j| * bound_j, args and bounds lists of [n] arrays."""
    n_out = _chain(*[np.stack(a) for a in args]).shape[0]
    acc = np.zeros((n_out, args[0][0].size))
    h = 1e-30
    for a in range(len(args)):
        for m in range(5):
            z = [np.stack(x).astype(complex) for x in args]
            z[a][m] = z[a][m] + 1j * h
            acc += np.abs(_chain(*z).imag / h) * bounds[a][m]
    return 2.0 * acc


def frame_bounds(node_x, node_y, q, pan, u, coef_ulps):
    """[3, n] bounds on kappa, gamma3, gamma4 for coefficient changes of at most
    coef_ulps * eps * M on each panel (M: the panel's largest coordinate)."""
    node_x = np.asarray(node_x, float)
    node_y = np.asarray(node_y, float)
    pan = np.asarray(pan)
    u = np.asarray(u, float)
    xg, _ = L.leggauss(q)
    cx = np.stack([L.legfit(xg, v, q - 1) for v in node_x.reshape(-1, q)])[pan]
    cy = np.stack([L.legfit(xg, v, q - 1) for v in node_y.reshape(-1, q)])[pan]
    dx, dy = _derivs(cx, u).T, _derivs(cy, u).T
    S = legendre_abs_sums(q, u)
    M = np.maximum(_panel_max(node_x, q, pan), _panel_max(node_y, q, pan))
    b = coef_ulps * EPS * M * S
    return _propagate([list(dx), list(dy)], [b, b])


def jet_bounds(node_x, node_y, q, dens, pan, u, coef_ulps):
    """[5, n] bounds on a density's xi-derivatives 0..4 for coefficient changes
    of at most coef_ulps * eps * M of the coordinates and of the density (each
    with its own panel maximum M)."""
    node_x = np.asarray(node_x, float)
    node_y = np.asarray(node_y, float)
    dens = np.asarray(dens, float)
    pan = np.asarray(pan)
    u = np.asarray(u, float)
    xg, _ = L.leggauss(q)
    fit = lambda v: np.stack([L.legfit(xg, w, q - 1) for w in v.reshape(-1, q)])[pan]  # noqa: E731
    dx, dy, ds = _derivs(fit(node_x), u).T, _derivs(fit(node_y), u).T, _derivs(fit(dens), u).T
    S = legendre_abs_sums(q, u)
    M = np.maximum(_panel_max(node_x, q, pan), _panel_max(node_y, q, pan))
    bxy = coef_ulps * EPS * M * S
    bs = coef_ulps * EPS * _panel_max(dens, q, pan) * S
    return _propagate([list(dx), list(dy), list(ds)], [bxy, bxy, bs])
