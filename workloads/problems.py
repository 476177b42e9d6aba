"""Problem builders: sources, boundary nodes, targets, densities and jets.

Every array is float64 (sgn int8).  Geometry per target follows the local
frame of Sec. 4: b is the closest boundary point, r = |x - b|, nu_b the
outward normal at b, x = b - sgn*r*nu_b with sgn = +1 inside, 0 on, -1
outside.  In the tangent-line frame (xi along the CCW tangent, the second axis
along the inward normal) the curve is x2 = gamma(xi) with gamma''(0) = kappa
(positive for convex arcs), gamma3 = gamma'''(0), gamma4 = gamma''''(0); layer
densities are expanded as sigma(xi), mu(xi) and their xi-derivatives at b are
supplied.  Volume density jets are (f, fx, fy, fxx, fxy, fyy) in global
coordinates at the target.
"""
from dataclasses import dataclass, field
from typing import Optional

import numpy as np
from numpy.polynomial.legendre import leggauss
from scipy.spatial import cKDTree

from . import series as S
from .mesh import curve_mesh, square_mesh


@dataclass
class Problem:
    name: str
    src_x: np.ndarray
    src_y: np.ndarray
    src_w: np.ndarray
    bnd_x: np.ndarray
    bnd_y: np.ndarray
    bnd_nx: np.ndarray
    bnd_ny: np.ndarray
    bnd_w: np.ndarray
    tgt_x: np.ndarray
    tgt_y: np.ndarray
    geom: dict                      # r, nx, ny, kappa, gamma3, gamma4, sgn
    f_src: Optional[np.ndarray]     # density at volume nodes
    jet6: Optional[np.ndarray]      # (6, n_tgt)
    sigma: Optional[np.ndarray]     # (n_bnd,)
    sigma_jet: Optional[np.ndarray]  # (3, n_tgt): sigma, sigma', sigma''
    mu: Optional[np.ndarray]
    mu_jet: Optional[np.ndarray]    # (5, n_tgt): mu, mu', mu'', mu''', mu''''
    info: dict = field(default_factory=dict)

    @property
    def n_src(self):
        return self.src_x.size

    @property
    def n_bnd(self):
        return self.bnd_x.size

    @property
    def n_tgt(self):
        return self.tgt_x.size

    def subset_targets(self, idx):
        """Same sources, only targets idx (for oracle sampling)."""
        g = {k: v[idx] for k, v in self.geom.items()}
        tk = lambda a: None if a is None else a[..., idx]
        return Problem(self.name + "[sub]", self.src_x, self.src_y, self.src_w,
                       self.bnd_x, self.bnd_y, self.bnd_nx, self.bnd_ny, self.bnd_w,
                       self.tgt_x[idx], self.tgt_y[idx], g, self.f_src, tk(self.jet6),
                       self.sigma, tk(self.sigma_jet), self.mu, tk(self.mu_jet), dict(self.info))


# ----------------------------------------------------------------------------
# Curves: the paper's boundary family (Sec. 6, star-shaped Fourier curves)


class StarCurve:
    """gamma(t) = r * rho(t) * (cos s t, sin s t) + (x0, y0), rho a cosine/sine series."""

    def __init__(self, r=1.0, alpha=(1.0,), beta=(), s=1, x0=0.0, y0=0.0):
        self.r = float(r)
        self.alpha = np.asarray(alpha, float)
        self.beta = np.asarray(beta, float)  # beta[k-1] multiplies sin(k t)
        self.s = int(s)
        self.x0, self.y0 = float(x0), float(y0)
        tt = np.linspace(0, 2 * np.pi, 8193)
        d = self.deriv(tt[:-1], 1)
        sp = np.hypot(d[:, 0], d[:, 1])
        self._s_tab = np.concatenate([[0.0], np.cumsum(sp) * (2 * np.pi / 8192)])
        self._t_tab = tt
        self.length = self._s_tab[-1]
        p = self.point(tt[:-1])
        self.area = 0.5 * np.sum(p[:, 0] * d[:, 1] - p[:, 1] * d[:, 0]) * (2 * np.pi / 8192)

    def rho_series(self, t0):
        """Taylor coefficients (K+1, n) of rho(t0 + tau)."""
        t0 = np.atleast_1d(np.asarray(t0, float))
        acc = np.zeros((S.K + 1, t0.size))
        for k, a in enumerate(self.alpha):
            if a:
                c, _ = S.trig_shift_coeffs(k, t0)
                acc += a * c
        for k, b in enumerate(self.beta, start=1):
            if b:
                _, sn = S.trig_shift_coeffs(k, t0)
                acc += b * sn
        return acc

    def point_series(self, t0):
        rho = S.TS(self.rho_series(t0))
        c, sn = S.trig_shift_coeffs(self.s, np.atleast_1d(t0))
        px = rho * S.TS(c) * self.r + self.x0
        py = rho * S.TS(sn) * self.r + self.y0
        return px, py

    def deriv(self, t, k):
        px, py = self.point_series(t)
        return np.stack([px.deriv(k), py.deriv(k)], axis=1)

    def point(self, t):
        return self.deriv(t, 0)

    def t_of_s(self, s):
        return np.interp(s, self._s_tab, self._t_tab)

    def rho_derivs(self, t, n=2):
        """rho(t) and its first n derivatives by direct trig sums."""
        t = np.asarray(t, float)
        out = [np.zeros_like(t) for _ in range(n + 1)]
        for k, a in enumerate(self.alpha):
            if a:
                c, s = np.cos(k * t), np.sin(k * t)
                d = [c, -s, -c, s]
                for j in range(n + 1):
                    out[j] += a * k ** j * d[j % 4]
        for k, b in enumerate(self.beta, start=1):
            if b:
                c, s = np.cos(k * t), np.sin(k * t)
                d = [s, c, -s, -c]
                for j in range(n + 1):
                    out[j] += b * k ** j * d[j % 4]
        return out

    def point_derivs(self, t):
        """gamma, gamma', gamma'' at t (each (n, 2)) by direct evaluation."""
        r0, r1, r2 = self.rho_derivs(t, 2)
        s = self.s
        c, sn = np.cos(s * t), np.sin(s * t)
        e0 = np.stack([c, sn], 1)
        e1 = np.stack([-sn, c], 1) * s
        e2 = -e0 * s * s
        g0 = self.r * r0[:, None] * e0 + np.array([self.x0, self.y0])
        g1 = self.r * (r1[:, None] * e0 + r0[:, None] * e1)
        g2 = self.r * (r2[:, None] * e0 + 2 * r1[:, None] * e1 + r0[:, None] * e2)
        return g0, g1, g2

    def inside(self, p):
        dx = p[:, 0] - self.x0
        dy = p[:, 1] - self.y0
        th = np.arctan2(dy, dx) / self.s
        rho = self.r * self.rho_derivs(np.mod(th, 2 * np.pi), 0)[0]
        return np.hypot(dx, dy) < rho

    def closest(self, p, near=np.inf, iters=6):
        """Parameter of the closest curve point: nearest dense sample + Newton
        for points within `near` of the curve; points farther away start Newton
        from their polar angle (star-shaped curves), which lands on a stationary
        point of the distance, whose distance is >= the true one."""
        n = 16 * 1024
        tt = np.linspace(0, 2 * np.pi, n, endpoint=False)
        d, j = cKDTree(self.point(tt)).query(p, distance_upper_bound=near)
        th = np.mod(np.arctan2(p[:, 1] - self.y0, p[:, 0] - self.x0) / self.s, 2 * np.pi)
        ok = np.isfinite(d)
        t = np.where(ok, tt[np.minimum(j, n - 1)], th)
        for _ in range(iters):
            g0, d1, d2 = self.point_derivs(t)
            g = g0 - p
            num = np.sum(g * d1, 1)
            den = np.sum(d1 * d1, 1) + np.sum(g * d2, 1)
            t = t - num / den
        return np.mod(t, 2 * np.pi)


def trig_density(coef_c, coef_s):
    """Return callable g(t) and its Taylor-coefficient function."""
    coef_c = np.asarray(coef_c, float)
    coef_s = np.asarray(coef_s, float)

    def series(t0):
        t0 = np.atleast_1d(t0)
        acc = np.zeros((S.K + 1, t0.size))
        for k, a in enumerate(coef_c):
            if a:
                acc += a * S.trig_shift_coeffs(k, t0)[0]
        for k, b in enumerate(coef_s, start=1):
            if b:
                acc += b * S.trig_shift_coeffs(k, t0)[1]
        return acc

    return (lambda t: series(t)[0]), series


def curve_frame_jets(curve, t_b, dens_series):
    """Local frame quantities at b = curve(t_b) for every target.

    Returns dict(b, tau, nu, kappa, gamma3, gamma4) and a list with, for each
    density series function, its xi-derivatives [d0..d4] at b.
    """
    px, py = curve.point_series(t_b)
    bx, by = px.c[0].copy(), py.c[0].copy()
    d1x, d1y = px.c[1], py.c[1]
    sp = np.hypot(d1x, d1y)
    tx, ty = d1x / sp, d1y / sp
    nx, ny = ty, -tx  # outward for a CCW curve
    dx = px - bx
    dy = py - by
    xi = dx * tx + dy * ty
    eta = dx * (-nx) + dy * (-ny)
    tau_of_xi = xi.reversion()
    g = tau_of_xi.compose_into(eta.c)
    out = dict(bx=bx, by=by, tx=tx, ty=ty, nx=nx, ny=ny,
               kappa=g.deriv(2), gamma3=g.deriv(3), gamma4=g.deriv(4))
    dens = []
    for fs in dens_series:
        d = tau_of_xi.compose_into(fs(t_b))
        dens.append(np.stack([d.deriv(k) for k in range(S.K + 1)]))
    return out, dens


def gauss_jets(x, y, gauss):
    """f and derivatives for f = sum A exp(-|x-c|^2/s^2); gauss = [(A,cx,cy,s)]."""
    f = np.zeros_like(x)
    fx = np.zeros_like(x)
    fy = np.zeros_like(x)
    fxx = np.zeros_like(x)
    fxy = np.zeros_like(x)
    fyy = np.zeros_like(x)
    for A, cx, cy, s in gauss:
        u = x - cx
        v = y - cy
        s2 = s * s
        e = A * np.exp(-(u * u + v * v) / s2)
        f += e
        fx += e * (-2 * u / s2)
        fy += e * (-2 * v / s2)
        fxx += e * (4 * u * u / (s2 * s2) - 2 / s2)
        fyy += e * (4 * v * v / (s2 * s2) - 2 / s2)
        fxy += e * (4 * u * v / (s2 * s2))
    return np.stack([f, fx, fy, fxx, fxy, fyy])


def panel_nodes(curve, n_panels, q):
    """Gauss-Legendre panels in the curve parameter: nodes, outward normals, weights."""
    xg, wg = leggauss(q)
    edges = np.linspace(0, 2 * np.pi, n_panels + 1)
    a, b = edges[:-1, None], edges[1:, None]
    t = (0.5 * (a + b) + 0.5 * (b - a) * xg[None, :]).ravel()
    wt = (0.5 * (b - a) * wg[None, :]).ravel()
    p = curve.point(t)
    d = curve.deriv(t, 1)
    sp = np.hypot(d[:, 0], d[:, 1])
    return p[:, 0], p[:, 1], d[:, 1] / sp, -d[:, 0] / sp, wt * sp, t


def _empty():
    return np.zeros(0)


# ----------------------------------------------------------------------------
# Problem families


def star_params(seed, r=0.8):
    """Random star-shaped domain (Sec. 6 curve family): alpha0 = 1, |alpha_k|,|beta_k| <= 0.25/k."""
    rng = np.random.default_rng(seed)
    ks = np.arange(1, 7)
    alpha = np.concatenate([[1.0], rng.uniform(-0.25 / ks, 0.25 / ks)])
    beta = rng.uniform(-0.25 / ks, 0.25 / ks)
    return dict(r=r, alpha=alpha * 0.55, beta=beta * 0.55)


def disk_problem(n_tri, seed=1, gauss=((1.0, 0.0, 0.0, np.sqrt(0.1)),), name="disk"):
    """Unit disk, curved boundary elements, f = sum of Gaussians; targets = nodes."""
    curve = StarCurve(r=1.0, alpha=(1.0,))
    x, y, w, info = curve_mesh(curve, n_tri, seed)
    jet = gauss_jets(x, y, gauss)
    rr = np.hypot(x, y)
    geom = dict(r=1.0 - rr, nx=x / rr, ny=y / rr, kappa=np.ones_like(x),
                gamma3=np.zeros_like(x), gamma4=np.full_like(x, 3.0),
                sgn=np.ones(x.size, np.int8))
    info.update(kind="disk", gauss=gauss, n_tri_target=n_tri, seed=seed)
    e = _empty()
    return Problem(name, x, y, w, e, e, e, e, e, x.copy(), y.copy(), geom, jet[0].copy(), jet,
                   None, None, None, None, info)


def disk_at_targets(P, tx, ty):
    """The disk problem P with its targets replaced by (tx, ty), inside or outside
    the unit circle: exact frames of the circle and f's analytic jets there."""
    tx, ty = np.asarray(tx, float), np.asarray(ty, float)
    rr = np.hypot(tx, ty)
    geom = dict(r=np.abs(1.0 - rr), nx=tx / rr, ny=ty / rr, kappa=np.ones_like(tx),
                gamma3=np.zeros_like(tx), gamma4=np.full_like(tx, 3.0),
                sgn=np.where(rr < 1.0, 1, np.where(rr > 1.0, -1, 0)).astype(np.int8))
    return Problem(P.name + "[targets]", P.src_x, P.src_y, P.src_w, P.bnd_x, P.bnd_y, P.bnd_nx, P.bnd_ny,
                   P.bnd_w, tx.copy(), ty.copy(), geom, P.f_src, gauss_jets(tx, ty, P.info["gauss"]),
                   None, None, None, None, dict(P.info))


def square_problem(n_tri=180_000, n_split=20_000, seed=2, n_panels=250, q=20, name="square"):
    """[-1,1]^2 with slivers/degenerate triangles/gaps; f = 5 Gaussians; mu = cos(3 theta)."""
    rng = np.random.default_rng(seed)
    x, y, w, info = square_mesh(n_tri, seed, n_split)
    gauss = []
    for _ in range(5):
        s = float(np.exp(rng.uniform(np.log(0.02), np.log(0.3))))
        cx, cy = rng.uniform(-0.8, 0.8, 2)
        A = float(rng.uniform(0.5, 1.0) * rng.choice([-1.0, 1.0]))
        gauss.append((A, float(cx), float(cy), s))
    jet = gauss_jets(x, y, gauss)
    # boundary: 4 sides x n_panels Gauss-Legendre panels, CCW
    xg, wg = leggauss(q)
    edges = np.linspace(-1, 1, n_panels + 1)
    u = (0.5 * (edges[:-1, None] + edges[1:, None]) + 0.5 * (edges[1:, None] - edges[:-1, None]) * xg).ravel()
    wu = (0.5 * (edges[1:, None] - edges[:-1, None]) * wg).ravel()
    one = np.ones_like(u)
    sides = [  # (x, y, nx, ny) for bottom, right, top, left (CCW)
        (u, -one, 0 * one, -one), (one, u, one, 0 * one),
        (-u, one, 0 * one, one), (-one, -u, -one, 0 * one)]
    bx = np.concatenate([s[0] for s in sides])
    by = np.concatenate([s[1] for s in sides])
    bnx = np.concatenate([s[2] for s in sides])
    bny = np.concatenate([s[3] for s in sides])
    bw = np.concatenate([wu] * 4)
    mu = np.cos(3 * np.arctan2(by, bx))
    # geometry: nearest side
    d = np.stack([y + 1, 1 - x, 1 - y, x + 1])  # distances to bottom, right, top, left
    k = np.argmin(d, axis=0)
    r = d[k, np.arange(x.size)]
    nxs = np.array([0.0, 1.0, 0.0, -1.0])[k]
    nys = np.array([-1.0, 0.0, 1.0, 0.0])[k]
    geom = dict(r=r, nx=nxs, ny=nys, kappa=np.zeros_like(x), gamma3=np.zeros_like(x),
                gamma4=np.zeros_like(x), sgn=np.ones(x.size, np.int8))
    # second-nearest side distance (corner proximity), informational
    d_sorted = np.sort(d, axis=0)
    info.update(kind="square", gauss=gauss, r2=d_sorted[1], n_panels=n_panels, q=q)
    # mu jets along the nearest side: mu(xi) = cos(3 atan2(b + xi t))
    bxp = x + r * nxs
    byp = y + r * nys
    tx, ty = -nys, nxs  # CCW tangent
    n = x.size
    X = S.TS.const(bxp, n) + S.TS.var(n) * tx
    Y = S.TS.const(byp, n) + S.TS.var(n) * ty
    dth = (X * X + Y * Y).recip() * (bxp * ty - byp * tx)
    th = dth.integrate(0.0)
    th0 = np.arctan2(byp, bxp)
    sn, cs = S.sin_cos_shift(3 * th0, th * 3.0)
    mu_jet = np.stack([cs.deriv(kk) for kk in range(S.K + 1)])
    e = None
    return Problem(name, x, y, w, bx, by, bnx, bny, bw, x.copy(), y.copy(), geom,
                   jet[0].copy(), jet, e, e, mu, mu_jet, info)


def star_problem(n_tri, seed, kinds="VSD", name="star", n_bnd=None, r=0.8):
    """Seeded star domain (batching / serving workloads): Gaussian f, trig sigma/mu."""
    rng = np.random.default_rng(10_000 + seed)
    prm = star_params(seed, r=r)
    curve = StarCurve(**prm)
    x, y, w, info = curve_mesh(curve, n_tri, seed)
    s = float(rng.uniform(0.05, 0.3))
    c = rng.uniform(-0.2, 0.2, 2)
    gauss = [(1.0, float(c[0]), float(c[1]), s)]
    jet = gauss_jets(x, y, gauss)
    deg = int(rng.integers(1, 6))
    sc = np.concatenate([[1.0], rng.uniform(-0.5, 0.5, deg)])
    ss = rng.uniform(-0.5, 0.5, deg)
    mc = np.concatenate([[0.5], rng.uniform(-0.5, 0.5, deg)])
    ms = rng.uniform(-0.5, 0.5, deg)
    sig_f, sig_s = trig_density(sc, ss)
    mu_f, mu_s = trig_density(mc, ms)
    # boundary panels: spacing ~ a third of the volume node spacing
    dx = np.sqrt(np.sum(w) / x.size)
    if n_bnd is None:
        n_bnd = int(np.ceil(curve.length / (dx / 3.0)))
    q = 16
    npan = max(4, int(np.ceil(n_bnd / q)))
    bx, by, bnx, bny, bw, bt = panel_nodes(curve, npan, q)
    # target geometry: closest point for targets near the boundary; far ones get
    # the exact distance via the same Newton solve (cheap enough at these sizes)
    P = np.stack([x, y], 1)
    # Exact closest points (nearest dense sample + Newton) and local frames for
    # targets within 18 sqrt(delta_1) of the boundary (delta_1 = 3 sum(w)/N, the
    # experiments' rule).  Farther targets only need r > 12 sqrt(delta_1): they
    # get a lower bound of their distance (no dense sample lies within `near`,
    # so the distance exceeds near - spacing) and a placeholder frame.
    near = 18.0 * np.sqrt(3.0 * np.sum(w) / x.size)
    n_dense = 16 * 1024
    tt = np.linspace(0, 2 * np.pi, n_dense, endpoint=False)
    dense = curve.point(tt)
    spacing = np.max(np.hypot(*(np.roll(dense, -1, 0) - dense).T))
    dd, jj = cKDTree(dense).query(P, distance_upper_bound=near)
    is_near = np.isfinite(dd)
    n = x.size
    geom = dict(r=np.full(n, near - spacing), nx=np.ones(n), ny=np.zeros(n), kappa=np.zeros(n),
                gamma3=np.zeros(n), gamma4=np.zeros(n), sgn=np.ones(n, np.int8))
    sj = np.zeros((3, n))
    mj = np.zeros((5, n))
    if np.any(is_near):
        Pn = P[is_near]
        t_b = tt[jj[is_near]]
        for _ in range(6):
            g0, d1, d2 = curve.point_derivs(t_b)
            g = g0 - Pn
            t_b = t_b - np.sum(g * d1, 1) / (np.sum(d1 * d1, 1) + np.sum(g * d2, 1))
        t_b = np.mod(t_b, 2 * np.pi)
        fr, (sjn, mjn) = curve_frame_jets(curve, t_b, [sig_s, mu_s])
        geom["r"][is_near] = np.hypot(Pn[:, 0] - fr["bx"], Pn[:, 1] - fr["by"])
        for k in ("nx", "ny", "kappa", "gamma3", "gamma4"):
            geom[k][is_near] = fr[k]
        geom["sgn"][is_near] = np.where(((Pn[:, 0] - fr["bx"]) * fr["nx"] + (Pn[:, 1] - fr["by"]) * fr["ny"]) < 0,
                                        1, -1).astype(np.int8)
        sj[:, is_near] = sjn[:3]
        mj[:, is_near] = mjn
    info.update(kind="star", params=prm, gauss=gauss, seed=seed, near=near, near_mask=is_near,
                npan=npan, q=q, sigma_trig=(sc, ss), mu_trig=(mc, ms))
    sigma = sig_f(bt) if "S" in kinds else None
    mu = mu_f(bt) if "D" in kinds else None
    return Problem(name, x, y, w, bx, by, bnx, bny, bw, x.copy(), y.copy(), geom,
                   jet[0].copy() if "V" in kinds else None, jet if "V" in kinds else None,
                   sigma, sj if "S" in kinds else None, mu, mj if "D" in kinds else None, info)


def fine_boundary(problem, levels):
    """The problem's boundary with every panel split into 2^levels panels (same
    Gauss-Legendre order), densities evaluated there: the oversampled boundary
    of the dyadic refinement of the local layer parts (Sec. 4), whose slice
    kernels narrow by a factor two per level.  Returns dict(x, y, nx, ny, w,
    sigma, mu) (sigma / mu None when the problem has no such density)."""
    info = problem.info
    m = 2 ** int(levels)
    if info.get("kind") == "square":
        xg, wg = leggauss(info["q"])
        edges = np.linspace(-1, 1, info["n_panels"] * m + 1)
        u = (0.5 * (edges[:-1, None] + edges[1:, None]) + 0.5 * (edges[1:, None] - edges[:-1, None]) * xg).ravel()
        wu = (0.5 * (edges[1:, None] - edges[:-1, None]) * wg).ravel()
        one = np.ones_like(u)
        sides = [(u, -one, 0 * one, -one), (one, u, one, 0 * one),
                 (-u, one, 0 * one, one), (-one, -u, -one, 0 * one)]
        x = np.concatenate([t[0] for t in sides])
        y = np.concatenate([t[1] for t in sides])
        return dict(x=x, y=y, nx=np.concatenate([t[2] for t in sides]), ny=np.concatenate([t[3] for t in sides]),
                    w=np.concatenate([wu] * 4), sigma=None,
                    mu=np.cos(3 * np.arctan2(y, x)) if problem.mu is not None else None)
    if info.get("kind") == "star":
        curve = StarCurve(**info["params"])
        x, y, nx, ny, w, t = panel_nodes(curve, info["npan"] * m, info["q"])
        sig_f, _ = trig_density(*info["sigma_trig"])
        mu_f, _ = trig_density(*info["mu_trig"])
        return dict(x=x, y=y, nx=nx, ny=ny, w=w, sigma=sig_f(t) if problem.sigma is not None else None,
                    mu=mu_f(t) if problem.mu is not None else None)
    raise ValueError("no panel description for this problem")


def circle_layer_problem(n_bnd, tgt_xy, sigma_fn=None, mu_fn=None, radius=1.0):
    """Unit circle boundary (trapezoid nodes), given targets; densities as functions of
    the angle: sigma_fn(theta) -> (K+1,n) Taylor coefficients in the angle."""
    th = 2 * np.pi * np.arange(n_bnd) / n_bnd
    bx, by = radius * np.cos(th), radius * np.sin(th)
    bw = np.full(n_bnd, 2 * np.pi * radius / n_bnd)
    curve = StarCurve(r=radius, alpha=(1.0,))
    tx, ty = tgt_xy[:, 0], tgt_xy[:, 1]
    tb = np.mod(np.arctan2(ty, tx), 2 * np.pi)
    fns = [f for f in (sigma_fn, mu_fn) if f is not None]
    fr, dens = curve_frame_jets(curve, tb, fns)
    rr = np.hypot(tx, ty)
    r = np.abs(radius - rr)
    sgn = np.where(rr < radius, 1, np.where(rr > radius, -1, 0)).astype(np.int8)
    geom = dict(r=r, nx=fr["nx"], ny=fr["ny"], kappa=fr["kappa"], gamma3=fr["gamma3"],
                gamma4=fr["gamma4"], sgn=sgn)
    sigma = sig_jet = mu = mu_jet = None
    i = 0
    if sigma_fn is not None:
        sigma = sigma_fn(th)[0]
        sig_jet = dens[i][:3]
        i += 1
    if mu_fn is not None:
        mu = mu_fn(th)[0]
        mu_jet = dens[i]
    e = np.zeros(0)
    return Problem("circle", e, e, e, bx, by, bx / radius, by / radius, bw, tx.copy(), ty.copy(),
                   geom, None, None, sigma, sig_jet, mu, mu_jet, dict(kind="circle"))


# ----------------------------------------------------------------------------
# Named workloads (sizes of the five benchmark configurations)

def config_problem(k, scale=1.0, seed=None):
    """k = 1: disk ~2000 triangles (~12k nodes); 2: square 200k triangles with
    slivers and gaps (~1.2M nodes) and 20k boundary nodes; 3: disk ~2M
    triangles (~12M nodes).  scale shrinks triangle counts for quick runs."""
    if k == 1:
        return disk_problem(int(2000 * scale), seed=1 if seed is None else seed, name="disk-2k")
    if k == 2:
        return square_problem(int(180_000 * scale), int(20_000 * scale), seed=2 if seed is None else seed,
                              n_panels=max(4, int(250 * min(1.0, scale ** 0.5))), name="square-200k")
    if k == 3:
        return disk_problem(int(2_000_000 * scale), seed=3 if seed is None else seed, name="disk-2M")
    raise ValueError("config must be 1, 2 or 3")
