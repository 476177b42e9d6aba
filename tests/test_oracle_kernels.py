"""Pins of the oracle's split kernel (Sec. 2, kernel splitting) against
definitions that do not go through the oracle's own code: mpmath's E1 at 50
digits, the time-integral identity of the heat kernel, a finite-difference
normal derivative, and brute-force mpmath sums on tiny inputs."""
import mpmath as mp
import numpy as np
import pytest
from scipy.integrate import quad

from oracle import direct

GAMMA = 0.57721566490153286061


def ein_mp(z):
    mp.mp.dps = 50
    z = mp.mpf(z)
    return mp.e1(z) + mp.euler + mp.log(z)


def gh_mp(d2, delta):
    """G_H[delta](d) = -log|d|/(2 pi) - E1(|d|^2/(4 delta))/(4 pi) for d != 0."""
    mp.mp.dps = 50
    d2 = mp.mpf(d2)
    return -mp.log(d2) / (4 * mp.pi) - mp.e1(d2 / (4 * mp.mpf(delta))) / (4 * mp.pi)


def test_ein_matches_library_e1_50_digits():
    z = np.concatenate([np.geomspace(1e-8, 2.0, 40), np.linspace(1.9, 3.0, 12),
                        np.geomspace(3.0, 900.0, 40)])
    got = direct.ein(z)
    ref = np.array([float(ein_mp(v)) for v in z])
    assert np.max(np.abs(got - ref) / np.abs(ref)) < 4e-15


def test_gh_origin_value_and_split_identity():
    delta = 7.853981633974483e-4
    g0 = direct.gh(0.0, delta)[0]
    assert abs(g0 - (GAMMA - np.log(4 * delta)) / (4 * np.pi)) < 1e-15
    # G_H + G_L = G for d != 0 (Sec. 2, eqs. splitting/splitting2)
    d2 = np.geomspace(1e-7, 9.0, 60)
    got = direct.gh(d2, delta)
    ref = np.array([float(gh_mp(v, delta)) for v in d2])
    assert np.max(np.abs(got - ref)) < 2e-15 * max(1.0, np.max(np.abs(ref)))


@pytest.mark.parametrize("dist", [0.0, 0.01, 0.05, 0.2, 0.7])
def test_gh_difference_is_heat_kernel_time_integral(dist):
    """G_H[d1] - G_H[d2] = int_{d1}^{d2} exp(-r^2/4t)/(4 pi t) dt (eq. eiformula)."""
    d1, d2_ = 1e-3, 3.2e-2
    lhs = direct.gh(dist * dist, d1)[0] - direct.gh(dist * dist, d2_)[0]
    rhs = quad(lambda t: np.exp(-dist * dist / (4 * t)) / (4 * np.pi * t), d1, d2_,
               epsabs=1e-16, epsrel=1e-14, limit=200)[0]
    assert abs(lhs - rhs) < 1e-14


def test_kd_is_normal_derivative_of_gh_in_source_variable():
    delta = 2e-3
    rng = np.random.default_rng(0)
    for _ in range(20):
        x = rng.uniform(-1, 1, 2)
        y = x + rng.normal(size=2) * rng.choice([0.02, 0.1, 0.5])
        th = rng.uniform(0, 2 * np.pi)
        nu = np.array([np.cos(th), np.sin(th)])
        h = 1e-4 * np.sqrt(delta)
        gp = direct.gh(np.sum((x - (y + h * nu)) ** 2), delta)[0]
        gm = direct.gh(np.sum((x - (y - h * nu)) ** 2), delta)[0]
        fd = (gp - gm) / (2 * h)
        kd = direct.kd(x[0] - y[0], x[1] - y[1], nu[0], nu[1], delta)
        assert abs(fd - kd) < 1e-7 * max(1.0, abs(kd))
    # coincident points: the smooth kernel's gradient vanishes
    assert direct.kd(0.0, 0.0, 1.0, 0.0, delta) == 0.0


def test_direct_sums_match_mpmath_brute_force_tiny():
    rng = np.random.default_rng(5)
    delta = 1e-3
    ns, nb, nt = 40, 24, 6
    sx, sy = rng.uniform(-1, 1, (2, ns))
    c = rng.normal(size=ns)
    th = np.linspace(0, 2 * np.pi, nb, endpoint=False)
    bx, by = np.cos(th), np.sin(th)
    s = rng.normal(size=nb)
    m = rng.normal(size=nb)
    tx, ty = rng.uniform(-1.2, 1.2, (2, nt))
    tx[0], ty[0] = sx[3], sy[3]          # a target on a source
    tx[1], ty[1] = bx[2], by[2]          # a target on a boundary node
    V, Sg, D = direct.history(tx, ty, sx, sy, c, bx, by, bx, by, s, m, delta)
    mp.mp.dps = 40
    for i in range(nt):
        def gh_exact(dx, dy):
            d2 = mp.mpf(dx) ** 2 + mp.mpf(dy) ** 2
            if d2 == 0:
                return (mp.euler - mp.log(4 * mp.mpf(delta))) / (4 * mp.pi)
            return gh_mp(d2, delta)
        v = mp.fsum(mp.mpf(c[j]) * gh_exact(tx[i] - sx[j], ty[i] - sy[j]) for j in range(ns))
        sv = mp.fsum(mp.mpf(s[j]) * gh_exact(tx[i] - bx[j], ty[i] - by[j]) for j in range(nb))
        dv = mp.mpf(0)
        for j in range(nb):
            dx = mp.mpf(tx[i] - bx[j])
            dy = mp.mpf(ty[i] - by[j])
            d2 = dx * dx + dy * dy
            if d2 > 0:
                dv += mp.mpf(m[j]) * (bx[j] * dx + by[j] * dy) * (1 - mp.exp(-d2 / (4 * delta))) / (2 * mp.pi * d2)
        assert abs(V[i] - float(v)) < 1e-14 * max(1, abs(float(v)))
        assert abs(Sg[i] - float(sv)) < 1e-14 * max(1, abs(float(sv)))
        assert abs(D[i] - float(dv)) < 1e-14 * max(1, abs(float(dv)))
