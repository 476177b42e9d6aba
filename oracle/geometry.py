"""Oracle: each target's local frame and the layer-density jets, computed from
a boundary given only as Gauss-Legendre panels (the frame of Sec. 4, which the
paper treats as a geometry preprocessing step outside the solver).

Test infrastructure only: plain numpy/scipy in float64, one target at a time.
Nothing here is imported by the product path.

Boundary: n_pan panels in order along the curve, counter-clockwise (interior
on the left), each holding q nodes at the Gauss-Legendre points of its own
parameter u in [-1, 1], ascending.  On a panel each coordinate (and a density)
is its degree q-1 interpolant in u, here as the Legendre series through the
q nodal values (numpy's fit of degree q-1 at q points, which interpolates).
Its derivatives are taken as they are: the high coefficients of a finely
resolved panel hold mostly the nodal values' rounding, which the derivatives
amplify (fourth derivatives most), and nothing here removes it.

Frame of a target p:
1. the nearest boundary node (lowest index on ties) gives a panel and u;
2. Newton on g(u) = (x(u) - p) . x'(u) = 0 from there; when u leaves
   [-1, 1] the search continues on the neighbouring panel from its near end;
3. b = x(u*), r = |p - b|, tangent tau = x'/|x'| (counter-clockwise),
   outward normal nu = (tau_y, -tau_x), sgn = +1 if (p - b).nu < 0 (inside),
   -1 if > 0, 0 (on the boundary) if r <= 1e-12 |x'(u*)|, the panel's own
   length scale (a target given as a node lands within rounding of the
   interpolant, not exactly on it);
4. in the tangent-line frame (xi along tau, eta along -nu) the curve is
   eta = gamma(xi): kappa, gamma3, gamma4 = gamma'', gamma''', gamma'''' at 0,
   and a density s has xi-derivatives d^k s / d xi^k at 0 -- both through the
   inverse function u(xi) of xi(u) = (x(u) - b) . tau.
"""
import numpy as np
from numpy.polynomial import legendre as L
from scipy.spatial import cKDTree

NEWTON_ITERS = 30
ON_CURVE = 1e-12   # r <= ON_CURVE |x'(u*)|: the target is on the boundary (sgn 0)


def _panel_series(vals, q):
    """Legendre coefficients of the degree q-1 interpolants of vals[n_pan, q]
    at the Gauss-Legendre points of each panel."""
    xg, _ = L.leggauss(q)
    return np.stack([L.legfit(xg, v, q - 1) for v in vals])


def _derivs(c, u, nmax):
    """[p(u), p'(u), ..., p^(nmax)(u)] of the Legendre series c."""
    out = [L.legval(u, c)]
    d = c
    for _ in range(nmax):
        d = L.legder(d)
        out.append(L.legval(u, d) if d.size else 0.0)
    return np.array(out)


def inverse_chain(xi, h):
    """d^k/dxi^k of h(u(xi)) at the base point, k = 0..4, given the u-derivatives
    xi[1..4] of xi(u) and h[0..4] of h(u) (inverse function, then Faa di Bruno)."""
    x1, x2, x3, x4 = xi[1], xi[2], xi[3], xi[4]
    u1 = 1.0 / x1
    u2 = -x2 / x1 ** 3
    u3 = (3 * x2 * x2 - x1 * x3) / x1 ** 5
    u4 = (-15 * x2 ** 3 + 10 * x1 * x2 * x3 - x1 * x1 * x4) / x1 ** 7
    g0 = h[0]
    g1 = h[1] * u1
    g2 = h[2] * u1 ** 2 + h[1] * u2
    g3 = h[3] * u1 ** 3 + 3 * h[2] * u1 * u2 + h[1] * u3
    g4 = h[4] * u1 ** 4 + 6 * h[3] * u1 ** 2 * u2 + h[2] * (3 * u2 * u2 + 4 * u1 * u3) + h[1] * u4
    return np.array([g0, g1, g2, g3, g4])


def closest_on_panels(cx, cy, tx, ty, node_x, node_y, q):
    """(panel, u*) of each target's closest point (steps 1-2 above)."""
    n_pan = cx.shape[0]
    xg, _ = L.leggauss(q)
    _, j = cKDTree(np.stack([node_x, node_y], 1)).query(np.stack([tx, ty], 1))
    pan = (j // q).astype(np.int64)
    u = xg[j % q].copy()
    for i in range(tx.size):
        pi, ui = int(pan[i]), float(u[i])
        for _ in range(NEWTON_ITERS):
            dx = _derivs(cx[pi], ui, 2)
            dy = _derivs(cy[pi], ui, 2)
            gx, gy = dx[0] - tx[i], dy[0] - ty[i]
            g = gx * dx[1] + gy * dy[1]
            gp = dx[1] ** 2 + dy[1] ** 2 + gx * dx[2] + gy * dy[2]
            un = ui - g / gp
            if un > 1.0:
                pi, ui = (pi + 1) % n_pan, -1.0
            elif un < -1.0:
                pi, ui = (pi - 1) % n_pan, 1.0
            else:
                done = abs(un - ui) <= 1e-15
                ui = un
                if done:
                    break
        pan[i], u[i] = pi, ui
    return pan, u


def boundary_frame(node_x, node_y, q, tx, ty):
    """dict(r, nx, ny, kappa, gamma3, gamma4, sgn, pan, u) for targets (tx, ty)."""
    node_x = np.asarray(node_x, float)
    node_y = np.asarray(node_y, float)
    tx = np.asarray(tx, float)
    ty = np.asarray(ty, float)
    n_pan = node_x.size // q
    cx = _panel_series(node_x.reshape(n_pan, q), q)
    cy = _panel_series(node_y.reshape(n_pan, q), q)
    pan, u = closest_on_panels(cx, cy, tx, ty, node_x, node_y, q)
    n = tx.size
    out = {k: np.zeros(n) for k in ("r", "nx", "ny", "kappa", "gamma3", "gamma4")}
    out["sgn"] = np.zeros(n, np.int8)
    for i in range(n):
        dx = _derivs(cx[pan[i]], u[i], 4)
        dy = _derivs(cy[pan[i]], u[i], 4)
        sp = np.hypot(dx[1], dy[1])
        tau = np.array([dx[1], dy[1]]) / sp
        nu = np.array([tau[1], -tau[0]])
        d = np.array([tx[i] - dx[0], ty[i] - dy[0]])
        r = np.hypot(d[0], d[1])
        xi = dx * tau[0] + dy * tau[1]
        eta = -(dx * nu[0] + dy * nu[1])
        g = inverse_chain(xi, eta)
        out["r"][i] = r
        out["nx"][i], out["ny"][i] = nu
        out["kappa"][i], out["gamma3"][i], out["gamma4"][i] = g[2], g[3], g[4]
        s = d @ nu
        out["sgn"][i] = 0 if r <= ON_CURVE * sp else (1 if s < 0 else -1)
    out["pan"] = pan
    out["u"] = u
    return out


def density_jets(node_x, node_y, q, dens, pan, u, nder):
    """[nder+1, n] xi-derivatives at each target's b of the density given at the
    nodes, b being x(u) on panel pan (as returned by boundary_frame)."""
    node_x = np.asarray(node_x, float)
    n_pan = node_x.size // q
    cx = _panel_series(node_x.reshape(n_pan, q), q)
    cy = _panel_series(np.asarray(node_y, float).reshape(n_pan, q), q)
    cs = _panel_series(np.asarray(dens, float).reshape(n_pan, q), q)
    out = np.zeros((nder + 1, len(pan)))
    for i in range(len(pan)):
        dx = _derivs(cx[pan[i]], u[i], 4)
        dy = _derivs(cy[pan[i]], u[i], 4)
        sp = np.hypot(dx[1], dy[1])
        tau = np.array([dx[1], dy[1]]) / sp
        xi = dx * tau[0] + dy * tau[1]
        out[:, i] = inverse_chain(xi, _derivs(cs[pan[i]], u[i], 4))[: nder + 1]
    return out


def jet_weights(node_x, node_y, q, pan, u, nder):
    """Weights w[k, i, j] with jets[k, i] = sum_j w[k, i, j] dens[pan[i] q + j]:
    density_jets as the linear map it is (the jets of the q unit densities of
    each target's panel), for applying it to many densities."""
    n = len(pan)
    w = np.zeros((nder + 1, n, q))
    n_pan = np.asarray(node_x).size // q
    for j in range(q):
        e = np.zeros(n_pan * q)
        e[j::q] = 1.0                       # node j of every panel
        w[:, :, j] = density_jets(node_x, node_y, q, e, pan, u, nder)
    return w
