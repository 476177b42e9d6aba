"""Pins of the Dirichlet-solve oracle (double-layer representation, operator
D_int assembled from the method's evaluation at the boundary nodes):

* Gauss: D_int[1] = -1;
* the unit circle in closed form: D[cos n t] = -r^n cos(n t) / 2 inside, so
  D_int[mu] = cos(n t) has mu = -2 cos(n t), and u = r^n cos(n t) inside;
* a lobed star: u = Re((z - z0)^3) + linear recovered inside;
* every error falls with refinement of the panels (delta_1 ~ spacing^2);
* the Poisson problem -Lap u = exp(-r^2/s) on the unit disk with u = cos 3t on
  the circle, u = w(r) + r^3 cos 3t, where the radial part
  w(r) = (s/4)(2 ln(1/r) - E1(r^2/s) + E1(1/s)) has -Lap w = exp(-r^2/s),
  w(1) = 0; and V[f] = 0 on the circle for a radial f (Newton's theorem:
  outside a radial mass, V is -M ln|x| / (2 pi));
* the same source inside a lobed star, u = w(|x|) + Re((z - z0)^3): there V[f]
  on the boundary is far from zero, so the sign of the volume term in the
  boundary equation is checked too;
* the exterior Dirichlet problem (u = D[mu] + integral of mu outside): on the
  circle g = cos 3t gives mu = 2 cos 3t and u = r^-3 cos 3t; outside a lobed
  star u = Re(1/(z - z0)) + 0.3 is recovered with integral of mu = u at
  infinity = 0.3;
* the interior Neumann problem (Green's representation, boundary values of
  zero mean): on the circle g = 3 cos 3t gives u = cos 3t on it and r^3 cos 3t
  inside; with the Gaussian source on the disk and inside the star, the
  closed forms above up to their boundary mean;
* the exterior Dirichlet problem with a volume source (a Gaussian ring
  outside the unit circle), V[f] taken on the clockwise-traversed boundary:
  against the radial solution by nested adaptive quadrature plus
  r^-3 cos 3t, converging as the nodes are refined.
"""
import numpy as np
from numpy.polynomial.legendre import leggauss
from scipy.integrate import quad
from scipy.special import exp1

from oracle import bie
from workloads.mesh import curve_mesh
from workloads.problems import StarCurve, disk_problem, gauss_jets, panel_nodes, star_params


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


def _disk_poisson_errors(n_tri, n_pan, s2=0.1):
    gauss = ((1.0, 0.0, 0.0, np.sqrt(s2)),)
    D = disk_problem(n_tri, seed=1, gauss=gauss)
    bx, by, nx, ny, w, t = _circle(n_pan)
    P = bie.on_boundary_problem(bx, by, nx, ny, w, 16, src=(D.src_x, D.src_y, D.src_w))
    v_bnd = np.max(np.abs(bie.volume_at_nodes(P, D.f_src, gauss_jets(bx, by, gauss))))
    mu = bie.solve_dirichlet(P, np.cos(3 * t), D.f_src, gauss_jets(bx, by, gauss))
    rng = np.random.default_rng(0)
    th, rr = rng.uniform(0, 2 * np.pi, 150), rng.uniform(0.1, 0.95, 150)
    tx, ty = rr * np.cos(th), rr * np.sin(th)
    u = bie.solution_at(P, mu, tx, ty, D.f_src, gauss_jets(tx, ty, gauss))
    w_r = 0.25 * s2 * (2 * np.log(1 / rr) - exp1(rr * rr / s2) + exp1(1 / s2))
    return v_bnd, np.max(np.abs(u - w_r - rr ** 3 * np.cos(3 * th)))


def test_disk_poisson_closed_form_and_convergence():
    coarse = _disk_poisson_errors(2000, 48)
    fine = _disk_poisson_errors(8000, 64)
    print("disk Poisson (|V| on the circle, interior error): coarse", coarse, "fine", fine)
    assert coarse[0] <= 1e-8 and fine[0] <= 1e-9
    assert coarse[1] <= 1e-5 and fine[1] <= 1e-7 and fine[1] <= coarse[1] / 10


def test_star_poisson_recovered():
    s2 = 0.1
    gauss = ((1.0, 0.0, 0.0, np.sqrt(s2)),)
    curve = StarCurve(**star_params(3, r=0.8))
    z0 = complex(0.1, -0.05)

    def uex(x, y):
        r = np.hypot(x, y)
        return 0.25 * s2 * (2 * np.log(1 / r) - exp1(r * r / s2) + exp1(1 / s2)) + ((x + 1j * y - z0) ** 3).real

    x, y, w, _ = curve_mesh(curve, 1500, 3)
    bx, by, bnx, bny, bw, _ = panel_nodes(curve, 32, 16)
    P = bie.on_boundary_problem(bx, by, bnx, bny, bw, 16, src=(x, y, w))
    f = gauss_jets(x, y, gauss)[0]
    v_bnd = bie.volume_at_nodes(P, f, gauss_jets(bx, by, gauss))
    mu = bie.solve_dirichlet(P, uex(bx, by), f, gauss_jets(bx, by, gauss))
    rng = np.random.default_rng(1)
    k = rng.integers(0, bx.size, 150)
    s = rng.uniform(0.3, 0.97, 150)
    cx, cy = np.mean(bx), np.mean(by)
    tx, ty = cx + s * (bx[k] - cx), cy + s * (by[k] - cy)
    e = np.max(np.abs(bie.solution_at(P, mu, tx, ty, f, gauss_jets(tx, ty, gauss)) - uex(tx, ty)))
    print("star Poisson: max |V| on the boundary", np.max(np.abs(v_bnd)), "interior error", e)
    assert np.max(np.abs(v_bnd)) >= 0.01          # the volume term matters on this boundary
    assert e <= 1e-5


def _wr(r, s2=0.1):
    return 0.25 * s2 * (2 * np.log(1 / r) - exp1(r * r / s2) + exp1(1 / s2))


def _wdr(r, s2=0.1):
    """w'(r)."""
    return -(s2 / (2 * r)) * (1 - np.exp(-r * r / s2))


def _circle_ext_neu_errors(n_pan):
    bx, by, nx, ny, w, t = _circle(n_pan)
    P = bie.on_boundary_problem(bx, by, nx, ny, w, 16)
    rng = np.random.default_rng(0)
    mu = bie.solve_exterior_dirichlet(P, np.cos(3 * t))
    th, rr = rng.uniform(0, 2 * np.pi, 100), rng.uniform(1.05, 3, 100)
    ue = bie.exterior_solution_at(P, mu, rr * np.cos(th), rr * np.sin(th))
    ub = bie.solve_neumann(P, 3 * np.cos(3 * t))
    th2, rr2 = rng.uniform(0, 2 * np.pi, 100), rng.uniform(0.1, 0.95, 100)
    un = bie.neumann_solution_at(P, ub, 3 * np.cos(3 * t), rr2 * np.cos(th2), rr2 * np.sin(th2))
    return (np.max(np.abs(mu - 2 * np.cos(3 * t))), np.max(np.abs(ue - rr ** -3 * np.cos(3 * th))),
            np.max(np.abs(ub - np.cos(3 * t))), np.max(np.abs(un - rr2 ** 3 * np.cos(3 * th2))))


def test_circle_exterior_dirichlet_and_neumann_closed_forms():
    coarse = _circle_ext_neu_errors(16)
    fine = _circle_ext_neu_errors(32)
    print("circle (ext mu, ext u, neu u_b, neu u): 16 panels", coarse, "32 panels", fine)
    assert max(fine) <= 1e-6
    assert all(f <= c / 10 for f, c in zip(fine, coarse))


def test_disk_neumann_with_source():
    gauss = ((1.0, 0.0, 0.0, np.sqrt(0.1)),)
    D = disk_problem(2000, seed=1, gauss=gauss)
    bx, by, nx, ny, w, t = _circle(48)
    P = bie.on_boundary_problem(bx, by, nx, ny, w, 16, src=(D.src_x, D.src_y, D.src_w))
    g = _wdr(1.0) + 3 * np.cos(3 * t)
    ub = bie.solve_neumann(P, g, D.f_src, gauss_jets(bx, by, gauss))
    rng = np.random.default_rng(3)
    th, rr = rng.uniform(0, 2 * np.pi, 100), rng.uniform(0.1, 0.95, 100)
    tx, ty = rr * np.cos(th), rr * np.sin(th)
    u = bie.neumann_solution_at(P, ub, g, tx, ty, D.f_src, gauss_jets(tx, ty, gauss))
    e_b, e_u = np.max(np.abs(ub - np.cos(3 * t))), np.max(np.abs(u - _wr(rr) - rr ** 3 * np.cos(3 * th)))
    print("disk Neumann with source: boundary", e_b, "interior", e_u)
    assert e_b <= 2e-6 and e_u <= 5e-6


def test_star_exterior_dirichlet_and_neumann():
    gauss = ((1.0, 0.0, 0.0, np.sqrt(0.1)),)
    curve = StarCurve(**star_params(3, r=0.8))
    bx, by, bnx, bny, bw, _ = panel_nodes(curve, 32, 16)
    z0 = complex(0.1, -0.05)
    rng = np.random.default_rng(4)
    k = rng.integers(0, bx.size, 150)
    cx, cy = np.mean(bx), np.mean(by)
    # exterior: a decaying harmonic plus a constant
    P = bie.on_boundary_problem(bx, by, bnx, bny, bw, 16)
    uext = lambda x, y: (1 / (x + 1j * y - z0)).real + 0.3
    mu = bie.solve_exterior_dirichlet(P, uext(bx, by))
    s = rng.uniform(1.03, 2.5, 150)
    tx, ty = cx + s * (bx[k] - cx), cy + s * (by[k] - cy)
    e_ext = np.max(np.abs(bie.exterior_solution_at(P, mu, tx, ty) - uext(tx, ty)))
    # Neumann with the source
    x, y, w, _ = curve_mesh(curve, 1500, 3)
    P = bie.on_boundary_problem(bx, by, bnx, bny, bw, 16, src=(x, y, w))
    z = bx + 1j * by
    rb = np.abs(z)
    g = ((_wdr(rb) * bx / rb + (3 * (z - z0) ** 2).real) * bnx
         + (_wdr(rb) * by / rb - (3 * (z - z0) ** 2).imag) * bny)
    uin = lambda px, py: _wr(np.hypot(px, py)) + ((px + 1j * py - z0) ** 3).real
    f = gauss_jets(x, y, gauss)[0]
    ub = bie.solve_neumann(P, g, f, gauss_jets(bx, by, gauss))
    c = np.dot(bw, uin(bx, by)) / np.sum(bw)
    s = rng.uniform(0.3, 0.97, 150)
    tx, ty = cx + s * (bx[k] - cx), cy + s * (by[k] - cy)
    u = bie.neumann_solution_at(P, ub, g, tx, ty, f, gauss_jets(tx, ty, gauss))
    e_b, e_u = np.max(np.abs(ub - uin(bx, by) + c)), np.max(np.abs(u - uin(tx, ty) + c))
    print("star: exterior", e_ext, "integral of mu", np.dot(bw, mu), "Neumann boundary", e_b, "interior", e_u)
    assert e_ext <= 2e-4 and abs(np.dot(bw, mu) - 0.3) <= 1e-6
    assert e_b <= 1e-5 and e_u <= 1e-5


def _ring(x, y, r0=1.3, s=0.05):
    """f = exp(-(r - r0)^2 / s) and its Cartesian jets."""
    r = np.hypot(x, y)
    c, sn = x / r, y / r
    f = np.exp(-(r - r0) ** 2 / s)
    f1 = -2 * (r - r0) / s * f
    f2 = (4 * (r - r0) ** 2 / s ** 2 - 2 / s) * f
    return np.stack([f, f1 * c, f1 * sn, f2 * c * c + f1 * sn * sn / r, (f2 - f1 / r) * c * sn,
                     f2 * sn * sn + f1 * c * c / r])


def _ring_radial_solution(r, r0=1.3, s=0.05):
    """-Lap w = the ring outside the unit circle, w(1) = 0, w'(r) = -(1/r) int_1^r f t dt."""
    f = lambda t: np.exp(-(t - r0) ** 2 / s)
    inner = lambda u: quad(lambda t: f(t) * t, 1.0, u, epsabs=1e-15, epsrel=1e-13)[0]
    return -quad(lambda u: inner(u) / u, 1.0, r, epsabs=1e-14, epsrel=1e-12, limit=200)[0]


def _exterior_source_error(n_r, n_t, n_pan, R=2.6):
    xr, wr = leggauss(n_r)
    rr = 1 + (R - 1) * (xr + 1) / 2
    wr = wr * (R - 1) / 2
    th = 2 * np.pi * np.arange(n_t) / n_t
    RR, TT = np.meshgrid(rr, th, indexing="ij")
    src = ((RR * np.cos(TT)).ravel(), (RR * np.sin(TT)).ravel(), np.outer(wr * rr, np.full(n_t, 2 * np.pi / n_t)).ravel())
    f = _ring(src[0], src[1])[0]
    bx, by, nx, ny, w, t = _circle(n_pan)
    rb = bie.reversed_boundary(bx, by, nx, ny, w)
    Pcw = bie.on_boundary_problem(*rb, 16, src=src)
    vb = bie.volume_at_nodes(Pcw, f, _ring(rb[0], rb[1]))[::-1]
    P = bie.on_boundary_problem(bx, by, nx, ny, w, 16, src=src)
    mu = bie.solve_exterior_dirichlet(P, np.cos(3 * t) - vb)
    rng = np.random.default_rng(0)
    tq, rq = rng.uniform(0, 2 * np.pi, 40), rng.uniform(1.05, 2.2, 40)
    tx, ty = rq * np.cos(tq), rq * np.sin(tq)
    u = bie.volume_at(Pcw, f, _ring(tx, ty), tx, ty) + bie.exterior_solution_at(P, mu, tx, ty)
    ue = np.array([_ring_radial_solution(r) for r in rq]) + rq ** -3 * np.cos(3 * tq)
    return np.max(np.abs(vb)), np.max(np.abs(u - ue))


def test_exterior_dirichlet_with_source():
    coarse = _exterior_source_error(60, 240, 32)
    fine = _exterior_source_error(120, 480, 48)
    print("exterior with source (max |V| on the circle, error): coarse", coarse, "fine", fine)
    assert coarse[0] >= 0.1                       # the volume term matters on the boundary
    assert coarse[1] <= 2e-4 and fine[1] <= 2e-6 and fine[1] <= coarse[1] / 30


def _circle_operator(n_pan, delta, order_d=3, exact=False):
    """The oracle's D_int on the unit circle (16-node panels) at a given delta_1,
    its frames from the panels or exact (kappa = 1, gamma3 = 0, gamma4 = 3)."""
    import copy
    from oracle.potential import evaluate
    bx, by, nx, ny, w, t = _circle(n_pan)
    P = bie.on_boundary_problem(bx, by, nx, ny, w, 16)
    if exact:
        P.geom = dict(P.geom, kappa=np.ones(bx.size), gamma3=np.zeros(bx.size), gamma4=np.full(bx.size, 3.0))
    A = np.empty((bx.size, bx.size))
    for j in range(bx.size):
        e = np.zeros(bx.size)
        e[j] = 1.0
        Q = copy.copy(P)
        Q.mu, Q.mu_jet = e, bie._jets(P, e)
        A[:, j] = evaluate(Q, kinds="D", delta=delta, order_d=order_d)["D"]
    h = 2 * np.pi / bx.size
    return A, w, delta ** 1.5 / h ** 2


def _gmres_reaches(A, tol, maxiter):
    from scipy.sparse.linalg import gmres
    b = np.random.default_rng(0).standard_normal(A.shape[0])   # every frequency the panels carry
    x, _ = gmres(A, b, rtol=tol, restart=50, maxiter=maxiter)
    return np.linalg.norm(b - A @ x) / np.linalg.norm(b) <= tol


def test_operator_conditioning_grows_with_resolution():
    """Why the solves refuse boundaries resolved far finer than sqrt(delta_1).
    At a node the double layer's local part carries delta^{3/2} (kappa mu'' +
    gamma3 mu') terms with mu's derivatives from the panel interpolant: for
    the node spacing's frequency they are of size chi = delta^{3/2} kappa / h^2
    next to the jump 1/2.  On the unit circle the oracle's D_int grows in
    condition number with chi (2.4, 13, 254 at chi = 0.005, 0.05, 0.42), the
    same with exact curve derivatives as with the panels' (so the frames do
    not cause it), not at all without those terms (order_d = 2: about 2.1
    throughout), and its eigenvalues stay near -1/2 (besides -1 for the
    constants): the growth is non-normality.  GMRES(50) on a right-hand side
    holding every frequency reaches the solves' default 1e-12 at chi = 0.21
    within two cycles but not at chi = 1.7 within twenty (n = 512); the
    operator x/2 + D[x] + (w . x) of the exterior and Neumann problems fails
    already at chi = 0.59.  Smooth data converge far beyond those points; the
    device solves refuse chi above 4 and 2, where the condition numbers pass
    1e8 (1.6e8 and 9.4e7) and GMRES on every frequency reaches 1e-8 but not
    1e-10."""
    conds = []
    for d in (2e-4, 1e-3, 4e-3):
        A, _, chi = _circle_operator(16, d)
        A2, _, _ = _circle_operator(16, d, order_d=2)
        c, c2 = np.linalg.cond(A), np.linalg.cond(A2)
        ev = np.sort(np.linalg.eigvals(A).real)   # ev[0] ~ -1: the constants (D_int[1] = -1)
        print("chi %.3g: cond %.3g (order_d = 2: %.3g), eigenvalues' real parts: %.4f, then [%.3f, %.3f]"
              % (chi, c, c2, ev[0], ev[1], ev[-1]))
        conds.append(c)
        assert c2 <= 2.5
        assert abs(ev[0] + 1) <= 1e-3 and ev[1] > -0.6 and ev[-1] < -0.45
    assert conds[0] <= 3 and conds[1] >= 4 * conds[0] and conds[2] >= 10 * conds[1]
    Ae, _, _ = _circle_operator(16, 4e-3, exact=True)
    assert abs(np.linalg.cond(Ae) / conds[2] - 1) <= 0.1
    A, w, chi = _circle_operator(32, 1e-3)
    assert 0.2 <= chi <= 0.22 and _gmres_reaches(A, 1e-12, 2)
    A, w, chi = _circle_operator(32, 4e-3)
    assert 1.6 <= chi <= 1.7 and not _gmres_reaches(A, 1e-12, 20)
    A, w, chi = _circle_operator(32, 2e-3)
    Aplus = A + np.eye(w.size) + np.outer(np.ones(w.size), w)
    assert 0.58 <= chi <= 0.6 and not _gmres_reaches(Aplus, 1e-12, 20)
    A, w, chi = _circle_operator(32, 7.13e-3)
    assert 3.99 <= chi <= 4.01 and 1e8 <= np.linalg.cond(A) <= 1e9
    assert _gmres_reaches(A, 1e-8, 20) and not _gmres_reaches(A, 1e-10, 20)
    A, w, chi = _circle_operator(32, 4.49e-3)
    Aplus = A + np.eye(w.size) + np.outer(np.ones(w.size), w)
    assert 1.99 <= chi <= 2.01 and 5e7 <= np.linalg.cond(Aplus) <= 5e8
    assert _gmres_reaches(Aplus, 1e-8, 20) and not _gmres_reaches(Aplus, 1e-10, 20)
