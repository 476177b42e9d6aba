"""Oracle entry point: the discrete target of the method, computed plainly.

Test infrastructure only (used by tests/, the smoke check and the benchmark's
CPU-baseline leg).  It shares no code with the library.

What is computed, per target x_i (Secs. 2-4):

    V(x_i) = sum_j f_j w_j G_H[d1](x_i - x_j)                 + V_L[f](x_i)
    S(x_i) = sum_j' sigma_j' wG_j' G_H[d1](x_i - y_j')         + S_L[sigma](x_i)
    D(x_i) = sum_j' mu_j' wG_j' K_D(x_i, y_j')                 + D_L[mu](x_i)

i.e. the history part (near + far history together = the split kernel G_H at
delta_1, exactly, in the limit of a vanishing history tolerance) by direct
summation, plus the local part by the asymptotic expansions.  delta_1 follows
the experiments' rule delta = 3 dx^2 with dx^2 = sum(w)/N (Sec. 6); with no
volume nodes dx is the mean boundary weight.
"""
import numpy as np

from . import direct
from .local import double_local, rotate_jets, single_local, volume_local


def delta1_of(problem, c_delta=3.0):
    if problem.n_src:
        return c_delta * float(np.sum(problem.src_w)) / problem.n_src
    return c_delta * float(np.mean(problem.bnd_w)) ** 2


def evaluate(problem, delta=None, order_v=4, order_s=3, order_d=3, kinds="VSD", c_delta=3.0):
    """Return dict with per-kind arrays (history + local) and their sum 'total'."""
    if delta is None:
        delta = delta1_of(problem, c_delta)
    g = problem.geom
    out = {"delta": delta}
    use_v = "V" in kinds and problem.f_src is not None and problem.n_src
    use_s = "S" in kinds and problem.sigma is not None
    use_d = "D" in kinds and problem.mu is not None
    c = problem.f_src * problem.src_w if use_v else None
    s = problem.sigma * problem.bnd_w if use_s else None
    m = problem.mu * problem.bnd_w if use_d else None
    vh, sh, dh = direct.history(problem.tgt_x, problem.tgt_y, problem.src_x, problem.src_y, c,
                                problem.bnd_x, problem.bnd_y, problem.bnd_nx, problem.bnd_ny,
                                s, m, delta)
    total = np.zeros(problem.n_tgt)
    if use_v:
        c_ = g["r"] / np.sqrt(delta)
        if np.any((g["sgn"] < 0) & (c_ <= 12.0)):
            raise ValueError("volume local part is defined for targets in the closed domain")
        f, fe, fxx, fee = rotate_jets(problem.jet6, g["nx"], g["ny"])
        vl = volume_local(delta, g["r"], g["kappa"], f, fe, fxx, fee, order=order_v, sgn=g["sgn"])
        out["V_hist"], out["V_loc"], out["V"] = vh, vl, vh + vl
        total += out["V"]
    if use_s:
        sj = problem.sigma_jet
        sl = single_local(delta, g["r"], g["sgn"], g["kappa"], g["gamma3"], g["gamma4"],
                          sj[0], sj[1], sj[2], order=order_s)
        out["S_hist"], out["S_loc"], out["S"] = sh, sl, sh + sl
        total += out["S"]
    if use_d:
        mj = problem.mu_jet
        dl = double_local(delta, g["r"], g["sgn"], g["kappa"], g["gamma3"], g["gamma4"],
                          mj[0], mj[1], mj[2], mj[3], mj[4], order=order_d)
        out["D_hist"], out["D_loc"], out["D"] = dh, dl, dh + dl
        total += out["D"]
    out["total"] = total
    return out


def rel_linf(a, b):
    """e_inf = max|a - b| / max|b| (Sec. 6 error measure)."""
    a = np.asarray(a, float)
    b = np.asarray(b, float)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))
