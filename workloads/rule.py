"""A symmetric 6-point quadrature rule on the triangle, derived here.

The paper uses six interior nodes per triangle, exact for polynomials of
degree two (Sec. 6).  The node table it cites is not available offline, so we
derive a fully symmetric 6-point rule made of two 3-point orbits
(a, a, 1-2a) and (b, b, 1-2b) in barycentric coordinates by solving the moment
equations for every symmetric polynomial up to degree four.  The solution is
exact for all polynomials of total degree <= 4 (checked in the tests).
"""
import warnings
from functools import lru_cache
from math import factorial

import numpy as np
from scipy.optimize import fsolve


def _bary_moment(i, j, k):
    """Mean over a triangle of l1^i l2^j l3^k (l = barycentric coordinates)."""
    return 2.0 * factorial(i) * factorial(j) * factorial(k) / factorial(i + j + k + 2)


def _orbit(a):
    return np.array([[a, a, 1 - 2 * a], [a, 1 - 2 * a, a], [1 - 2 * a, a, a]])


def _residual(p):
    a, b, wa = p
    wb = 1.0 / 3.0 - wa
    pts = np.vstack([_orbit(a), _orbit(b)])
    wts = np.array([wa] * 3 + [wb] * 3)
    l1, l2, l3 = pts.T
    # Symmetric invariants e2 = sum l_i l_j, e3 = l1 l2 l3 and e2^2 generate the
    # symmetric polynomials of degree <= 4 on the simplex.
    e2 = l1 * l2 + l2 * l3 + l1 * l3
    e3 = l1 * l2 * l3
    ex_e2 = 3 * _bary_moment(1, 1, 0)
    ex_e3 = _bary_moment(1, 1, 1)
    ex_e22 = 3 * _bary_moment(2, 2, 0) + 6 * _bary_moment(2, 1, 1)
    return [wts @ e2 - ex_e2, wts @ e3 - ex_e3, wts @ (e2 * e2) - ex_e22]


@lru_cache(maxsize=1)
def six_point_rule():
    """Return (bary[6,3], weights[6]) with weights summing to 1 (times area)."""
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        sol = fsolve(_residual, [0.45, 0.09, 0.22], xtol=1e-15)
    if max(abs(v) for v in _residual(sol)) > 1e-15:
        raise RuntimeError("moment equations did not converge")
    a, b, wa = sol
    wb = 1.0 / 3.0 - wa
    if not (0 < a < 0.5 and 0 < b < 0.5 and wa > 0 and wb > 0):
        raise RuntimeError("moment solution is not an interior positive rule")
    pts = np.vstack([_orbit(a), _orbit(b)])
    wts = np.array([wa] * 3 + [wb] * 3)
    return pts, wts
