"""Pins of the dyadic-refinement oracle (Sec. 4, local part with arbitrary
precision) against quantities fixed independently of its formulas:

* the slice kernels are time integrals of the heat kernel (and of its source
  normal derivative) over [delta/4^j, delta/4^(j-1)], computed here by
  adaptive quadrature in t;
* the slices telescope: their sum over j = 1..J is the integral over
  [delta/4^J, delta] (used by the device kernel, which evaluates that single
  kernel);
* on a circle, the refined local parts converge to the exact local integrals
  int E1(|x-y|^2/4 delta)/(4 pi) sigma ds and
  int nu.(x-y) exp(-|x-y|^2/4 delta)/(2 pi |x-y|^2) mu ds (adaptive quadrature
  in the angle), the error falling with every level.
"""
import numpy as np
import pytest
from scipy.integrate import quad
from scipy.special import exp1

from oracle import refine
from oracle.local import double_local, single_local
from workloads.problems import circle_layer_problem, trig_density


@pytest.mark.parametrize("j", [1, 2, 3, 4])
def test_slice_kernels_are_time_integrals(j):
    delta = 2.5e-3
    a, b = delta / 4.0 ** j, delta / 4.0 ** (j - 1)
    for rho in (0.0, 1e-3, 0.02, 0.07, 0.15):
        r = np.array([rho * rho / delta])
        k_s = refine._slice_single(r, j)[0]
        if rho == 0.0:
            ref = np.log(b / a) / (4 * np.pi)   # int dt / (4 pi t)
        else:
            ref = quad(lambda t: np.exp(-rho * rho / (4 * t)) / (4 * np.pi * t), a, b, epsabs=0, epsrel=1e-13)[0]
        assert abs(k_s - ref) <= 1e-12 * max(abs(ref), 1e-30), (rho, k_s, ref)
        if rho > 0.0:
            # source at the origin with normal (0.6, 0.8), target at distance rho along (1, 1)/sqrt 2
            dx = dy = rho / np.sqrt(2.0)
            nx, ny = np.array([0.6]), np.array([0.8])
            k_d = refine._slice_double(np.array([dx]), np.array([dy]), nx, ny, np.array([rho * rho]), delta, j)[0]
            ndot = 0.6 * dx + 0.8 * dy
            ref = quad(lambda t: ndot / (2 * t) * np.exp(-rho * rho / (4 * t)) / (4 * np.pi * t), a, b,
                       epsabs=0, epsrel=1e-13)[0]
            assert abs(k_d - ref) <= 1e-11 * max(abs(ref), 1e-300), (rho, k_d, ref)


def test_slices_telescope():
    delta = 1e-3
    rho2 = np.array([0.0, 1e-8, 1e-6, 1e-4, 4e-4, 2e-3, 1e-2])
    r = rho2 / delta
    for J in (1, 2, 3, 5):
        tot = sum(refine._slice_single(r, j) for j in range(1, J + 1))
        one = np.where(r > 0, exp1(np.maximum(r, 1e-300) / 4) - exp1(np.maximum(r, 1e-300) * 4.0 ** (J - 1)),
                       np.log(4.0 ** J)) / (4 * np.pi)
        assert np.allclose(tot, one, rtol=1e-13, atol=1e-16)


def _circle_case():
    sig_f, sig_s = trig_density([1.0, 0.0, 0.0, 0.4], [0.0, 0.3])
    mu_f, mu_s = trig_density([0.5, 0.2], [0.0, 0.0, -0.3])
    delta = 1e-3
    sd = np.sqrt(delta)
    th0 = 0.7
    cs = (0.3, 1.0, 2.5)
    tgt = np.array([((1.0 - s * c * sd) * np.cos(th0), (1.0 - s * c * sd) * np.sin(th0))
                    for c in cs for s in (+1, -1)])
    P = circle_layer_problem(64, tgt, sigma_fn=sig_s, mu_fn=mu_s)
    n_f = 8192
    th = 2 * np.pi * np.arange(n_f) / n_f
    fine = dict(x=np.cos(th), y=np.sin(th), nx=np.cos(th), ny=np.sin(th), w=np.full(n_f, 2 * np.pi / n_f),
                sigma=sig_f(th), mu=mu_f(th))

    def sig(t):
        return float(np.squeeze(sig_f(np.atleast_1d(t))))

    def mu(t):
        return float(np.squeeze(mu_f(np.atleast_1d(t))))

    exact_s, exact_d = [], []
    for x, y in tgt:
        fs = lambda t: exp1(((x - np.cos(t)) ** 2 + (y - np.sin(t)) ** 2) / (4 * delta)) / (4 * np.pi) * sig(t)

        def fd(t):
            dx, dy = x - np.cos(t), y - np.sin(t)
            rho2 = dx * dx + dy * dy
            return (np.cos(t) * dx + np.sin(t) * dy) / (2 * np.pi * rho2) * np.exp(-rho2 / (4 * delta)) * mu(t)

        kw = dict(points=[th0], limit=800, epsabs=1e-15, epsrel=1e-13)
        exact_s.append(quad(fs, th0 - np.pi, th0 + np.pi, **kw)[0])
        exact_d.append(quad(fd, th0 - np.pi, th0 + np.pi, **kw)[0])
    return P, fine, delta, np.array(exact_s), np.array(exact_d)


def test_refined_local_parts_converge_to_exact_local_integrals():
    P, fine, delta, ex_s, ex_d = _circle_case()
    g = P.geom
    sj, mj = P.sigma_jet, P.mu_jet
    s_asym = single_local(delta, g["r"], g["sgn"], g["kappa"], g["gamma3"], g["gamma4"], *sj, order=3)
    d_asym = double_local(delta, g["r"], g["sgn"], g["kappa"], g["gamma3"], g["gamma4"], *mj, order=3)
    err_s = [np.abs(s_asym - ex_s)]
    err_d = [np.abs(d_asym - ex_d)]
    for J in (1, 2, 3):
        err_s.append(np.abs(s_asym + refine.layer_refinement(P, fine, J, delta, kinds="S") - ex_s))
        err_d.append(np.abs(d_asym + refine.layer_refinement(P, fine, J, delta, kinds="D") - ex_d))
    print("S errors by level", [float(e.max()) for e in err_s], "D errors", [float(e.max()) for e in err_d])
    # three levels: at least a hundredfold below the asymptotics alone, and small in absolute terms
    assert np.all(err_s[3] <= err_s[0] / 100) and np.all(err_d[3] <= err_d[0] / 100)
    assert err_s[3].max() <= 2e-10 * np.abs(ex_s).max() / 1e-2 and err_d[3].max() <= 5e-10
    # every level helps (worst target)
    for e in (err_s, err_d):
        assert all(e[k + 1].max() < e[k].max() for k in range(3))
