"""Oracle: local (small-time) parts V_L, S_L, D_L by the paper's asymptotics.

Test infrastructure only.  Plain numpy in float64, one formula per function,
terms grouped by powers of sqrt(delta) so that a truncation order can be
chosen (order = highest power of sqrt(delta) kept).

Readings of the paper (each pinned by brute-force quadrature in the tests):

* S_L (Lemma 4.1, eq. slplocO5) and D_L (Lemma 4.3, eq. dlplocO5) are used
  with the overall sign reversed.  With the kernels as defined in Sec. 2.1
  (heat kernel > 0, outward normal), S_L of a positive density is positive,
  and D_L carries the interior limit -mu/2 that the harmonic jump relation of
  Sec. 1 requires; the printed expansions (and their on-surface corollaries)
  have the opposite overall sign.
* V_L (Lemma 4.5, eq. vplocO5): the delta^{3/2} term uses (2 f_eta - kappa f),
  the form the paper's own on-boundary special case gives; the general
  formula prints (kappa f - 2 f_eta).  The delta and delta^2 terms are used as
  printed.
* The two delta^2 single-layer brackets with gamma4 and sigma'*gamma3 share
  one radial factor; it is written once.

Frame (Sec. 4): c = r / sqrt(delta); sgn = +1 inside, 0 on, -1 outside;
kappa = gamma''(0) > 0 for convex arcs; f_xi, f_eta are derivatives along the
tangent and the inward normal at the target.
"""
import numpy as np
from scipy.special import erf, erfc

SQPI = np.sqrt(np.pi)
C_FAR = 12.0   # beyond 12 sqrt(delta) the local layer parts are below 1e-14 (Sec. 2.2)


def _c(r, delta):
    return np.asarray(r, float) / np.sqrt(delta)


def volume_local(delta, r, kappa, f, f_eta, f_xixi, f_etaeta, order=4, sgn=None):
    """V_L[f] at targets inside or on the boundary (Lemma 4.5, sign reading above).

    Far targets (c > 12) inside use the interior limit delta f + delta^2 (f_xixi+f_etaeta)/2;
    far targets outside (sgn < 0) get zero: V_L is the time integral over [0, delta] of the
    heat kernel against f, which vanishes off the domain, and the kernel's mass within the
    domain is below 1e-14 there (Sec. 2.2's 12 sqrt(delta) cutoff).  Near exterior targets
    are outside the lemma (the caller rejects them).
    """
    c = _c(r, delta)
    near = c <= C_FAR
    inside = np.ones_like(c, bool) if sgn is None else np.asarray(sgn) >= 0
    E = erfc(c / 2)
    e = np.exp(-c * c / 4)
    out = np.zeros_like(c)
    if order >= 2:
        t = delta / 4 * (2 * erf(c / 2) + 2 * e * c / SQPI - c * c * E + 2) * f
        out += np.where(near, t, np.where(inside, delta * f, 0.0))
    if order >= 3:
        t = delta ** 1.5 * ((4 - 2 * c * c) * e + SQPI * c ** 3 * E) * (2 * f_eta - kappa * f) / (12 * SQPI)
        out += np.where(near, t, 0.0)
    if order >= 4:
        c4 = c ** 4
        t = delta ** 2 / 48 * (
            E * (4 * c4 * kappa * f_eta - 3 * (c4 + 4) * f_etaeta + (c4 - 12) * f_xixi - 3 * c4 * kappa ** 2 * f)
            + 2 * c * (c * c - 2) * e * (-4 * kappa * f_eta + 3 * f_etaeta - f_xixi + 3 * kappa ** 2 * f) / SQPI
            + 24 * (f_xixi + f_etaeta))
        out += np.where(near, t, np.where(inside, delta ** 2 / 2 * (f_xixi + f_etaeta), 0.0))
    return out


def single_local(delta, r, sgn, kappa, gamma3, gamma4, s0, s1, s2, order=3):
    """S_L[sigma] (Lemma 4.1 with the overall sign reversed); zero for c > 12.

    s0, s1, s2 = sigma, sigma', sigma'' at b (tangent-line parametrization).
    """
    c = _c(r, delta)
    sg = np.asarray(sgn, float)
    E = erfc(c / 2)
    e = np.exp(-c * c / 4)
    P1 = c * E - 2 * e / SQPI
    Q = 2 * (c * c - 2) * e / SQPI - c ** 3 * E
    out = np.zeros_like(c)
    if order >= 1:
        out += np.sqrt(delta) * s0 / 2 * P1
    if order >= 2:
        out += sg * delta * c * kappa * s0 / 4 * P1
    if order >= 3:
        out += delta ** 1.5 * (s0 * kappa ** 2 / 12 * (2 * c ** 3 * E - (4 * c * c + 1) * e / SQPI)
                               + s2 / 12 * Q)
    if order >= 4:
        out += delta ** 2 * sg * (c * kappa ** 3 * s0 / 16 * (3 * c ** 3 * E - (6 * c * c - 2) * e / SQPI)
                                  + c * kappa * s2 / 8 * Q
                                  + c * s0 * gamma4 / 48 * Q + c * s1 * gamma3 / 12 * Q)
    return np.where(c <= C_FAR, -out, 0.0)


def double_local(delta, r, sgn, kappa, gamma3, gamma4, m0, m1, m2, m3, m4, order=3):
    """D_L[mu] (Lemma 4.3 with the overall sign reversed); zero for c > 12.

    m0..m4 = mu and its first four derivatives at b (tangent-line parametrization).
    """
    c = _c(r, delta)
    sg = np.asarray(sgn, float)
    E = erfc(c / 2)
    e = np.exp(-c * c / 4)
    out = np.zeros_like(c)
    out += sg * m0 / 2 * E
    if order >= 1:
        out += np.sqrt(delta) * kappa * m0 / (2 * SQPI) * e
    if order >= 2:
        out += delta * sg * (3 * c * kappa ** 2 * m0 / (8 * SQPI) * e
                             + c * m2 / 4 * (2 * e / SQPI - c * E))
    A = 2 * (c * c + 1) * e / SQPI - c ** 3 * E
    B = 2 * (c * c + 4) * e / SQPI - c ** 3 * E
    if order >= 3:
        out += delta ** 1.5 * (5 * (c * c - 2) * kappa ** 3 * m0 / (16 * SQPI) * e
                               + gamma4 * m0 / (4 * SQPI) * e
                               + kappa * m2 / 4 * A + gamma3 * m1 / 12 * B)
    if order >= 4:
        out += delta ** 2 * sg * (35 * c * kappa ** 4 * m0 * (c * c - 6) / (128 * SQPI) * e
                                  + 5 * c * gamma3 ** 2 * m0 / (12 * SQPI) * e
                                  + 5 * c * kappa * gamma4 * m0 / (8 * SQPI) * e)
        out += delta ** 2 * sg * 5 * c * (kappa ** 2 * m2 / 16 * A + kappa * gamma3 * m1 / 24 * B)
        out += delta ** 2 * sg * c * m4 / 48 * (c ** 3 * E - 2 * (c * c - 2) * e / SQPI)
    return np.where(c <= C_FAR, -out, 0.0)


def rotate_jets(jet6, nx, ny):
    """(f, f_eta, f_xixi, f_etaeta) from global jets; eta = inward normal (-nu_b)."""
    f, fx, fy, fxx, fxy, fyy = jet6
    ex, ey = -nx, -ny            # inward normal
    tx, ty = -ny, nx             # tangent
    f_eta = fx * ex + fy * ey
    f_etaeta = fxx * ex * ex + 2 * fxy * ex * ey + fyy * ey * ey
    f_xixi = fxx * tx * tx + 2 * fxy * tx * ty + fyy * ty * ty
    return f, f_eta, f_xixi, f_etaeta
