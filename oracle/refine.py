"""Oracle: dyadic refinement of the local layer parts (Sec. 4, the subsection on
computing the local part with arbitrary precision).

Test infrastructure only: plain numpy/scipy in float64, no blocking or fusion
beyond what the paper states.  Nothing here is imported by the product path.

The local part of a layer potential is the time integral of the heat layer
potential over [0, delta].  With delta* = delta / 4^J the paper writes it as

    (local part over [0, delta*])  +  sum_{j=1..J} (slice [delta/4^j, delta/4^(j-1)]),

takes the first term from the small-time asymptotics (here the same
expansions as `oracle.local`, evaluated at delta*), and the slices by direct
quadrature over the boundary.  For the single layer the slice j is the
difference kernel

    K_j(r) = (E1(4^(j-2) r) - E1(4^(j-1) r)) / (4 pi),   r = |x - y|^2 / delta,

(the time integral of exp(-|x-y|^2/4t) / (4 pi t) over the slice).  For the
double layer the same time integral of the heat kernel's normal derivative
at the source gives

    nu_y . (x - y) / (2 pi |x - y|^2) * (exp(-4^(j-2) r) - exp(-4^(j-1) r)).

The slices' kernels narrow by a factor two per level, so the boundary is
sampled finely enough for the last level: `fine` holds nodes, outward normals,
quadrature weights and the densities on that oversampled boundary.

`layer_refinement` returns the correction to ADD to the local parts at delta
(with the sign reading of `oracle.local`: S_L and D_L as pinned there), i.e.

    [S_L(delta*) - S_L(delta)] + [D_L(delta*) - D_L(delta)] + slices.
"""
import numpy as np
from scipy.spatial import cKDTree
from scipy.special import exp1

from .local import double_local, single_local

# Beyond this distance (in units of sqrt(delta)) every slice kernel is below
# 1e-17 relative to its value at the origin: E1(z) < e^-z / z, z = rho^2 / (4 delta).
R_SLICE = 12.0


def _slice_single(r, j):
    """K_j(r): time integral of the heat kernel over slice j, r = rho^2 / delta."""
    a = 4.0 ** (j - 2) * r
    b = 4.0 ** (j - 1) * r
    out = np.empty_like(r)
    small = r == 0.0
    out[small] = np.log(4.0)                     # E1(a) - E1(4a) -> ln 4 as a -> 0
    out[~small] = exp1(a[~small]) - exp1(b[~small])
    return out / (4.0 * np.pi)


def _slice_double(dx, dy, nx, ny, rho2, delta, j):
    """Time integral over slice j of the source normal derivative of the heat kernel."""
    a = 4.0 ** (j - 2) / delta
    b = 4.0 ** (j - 1) / delta
    out = np.zeros_like(rho2)
    m = rho2 > 0.0
    # exp(-a rho^2) - exp(-b rho^2) = -exp(-a rho^2) expm1(-(b - a) rho^2)
    diff = -np.exp(-a * rho2[m]) * np.expm1(-(b - a) * rho2[m])
    out[m] = (nx[m] * dx[m] + ny[m] * dy[m]) / (2.0 * np.pi * rho2[m]) * diff
    return out


def slices(tx, ty, fine, delta, J, sigma=None, mu=None):
    """sum_{j=1..J} slice j of S[sigma] and D[mu] at the targets by direct sums
    over the fine boundary nodes within R_SLICE sqrt(delta) of each target."""
    tx = np.asarray(tx, float)
    ty = np.asarray(ty, float)
    fx, fy = np.asarray(fine["x"], float), np.asarray(fine["y"], float)
    fnx, fny = np.asarray(fine["nx"], float), np.asarray(fine["ny"], float)
    fw = np.asarray(fine["w"], float)
    out = np.zeros(tx.size)
    tree = cKDTree(np.stack([fx, fy], 1))
    lists = tree.query_ball_point(np.stack([tx, ty], 1), R_SLICE * np.sqrt(delta))
    for i, nb in enumerate(lists):
        if not nb:
            continue
        k = np.asarray(nb)
        dx = tx[i] - fx[k]
        dy = ty[i] - fy[k]
        rho2 = dx * dx + dy * dy
        for j in range(1, J + 1):
            if sigma is not None:
                out[i] += np.sum(_slice_single(rho2 / delta, j) * sigma[k] * fw[k])
            if mu is not None:
                out[i] += np.sum(_slice_double(dx, dy, fnx[k], fny[k], rho2, delta, j) * mu[k] * fw[k])
    return out


def layer_refinement(problem, fine, J, delta, order_s=3, order_d=3, kinds="SD"):
    """Correction added to the local layer parts at delta (see module docstring).

    fine: dict(x, y, nx, ny, w, sigma, mu) of the oversampled boundary.
    """
    P = problem
    g = P.geom
    ds = delta / 4.0 ** J
    corr = np.zeros(P.n_tgt)
    sig = mu = None
    if "S" in kinds and P.sigma_jet is not None:
        s0, s1, s2 = P.sigma_jet
        args = (g["r"], g["sgn"], g["kappa"], g["gamma3"], g["gamma4"], s0, s1, s2)
        corr += single_local(ds, *args, order=order_s) - single_local(delta, *args, order=order_s)
        sig = np.asarray(fine["sigma"], float)
    if "D" in kinds and P.mu_jet is not None:
        m = P.mu_jet
        args = (g["r"], g["sgn"], g["kappa"], g["gamma3"], g["gamma4"], m[0], m[1], m[2], m[3], m[4])
        corr += double_local(ds, *args, order=order_d) - double_local(delta, *args, order=order_d)
        mu = np.asarray(fine["mu"], float)
    corr += slices(P.tgt_x, P.tgt_y, fine, delta, J, sigma=sig, mu=mu)
    return corr
