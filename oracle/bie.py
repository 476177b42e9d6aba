"""Oracle: the interior Dirichlet problem -Lap u = f in the domain, u = g on
its boundary, by the representation u = V[f] + D[mu] (Sec. 1 and the boundary
integral correction of Sec. 5, whose matrix-vector product is the layer
potential evaluated on the boundary).

Test infrastructure only: plain numpy in float64 (dense operator, direct
solve).  Nothing here is imported by the product path.

D[mu] is harmonic inside; its interior limit on the boundary is
D_int[mu] = -mu/2 + (principal value of D[mu]), so the boundary condition
u = g on the boundary is the second-kind equation D_int[mu] = g - V[f]
(f = 0: the Laplace equation).  With volume nodes present, delta_1 follows
their rule 3 sum(w)/N for every part, as in the method.  Here D_int
at a boundary node is what the method computes for a target at that node with
r = 0 and sgn = +1 (history part plus the local part's interior limit), the
density's jets at the node coming from its panel interpolant
(oracle.geometry).  The operator is linear in mu, so its matrix is assembled
column by column from unit densities and the system is solved directly.

A problem may carry the curve's exact derivatives (curvature=: a callable
giving kappa, gamma3, gamma4 at the closest points of given points) in place
of the panel interpolant's, whose higher derivatives hold the nodal
coordinates' rounding amplified; the closest point, normal and density jets
still come from the panels.
"""
import copy

import numpy as np

from . import geometry as G
from .potential import delta1_of, evaluate


class _Layer:
    """Volume nodes (optional), boundary nodes, targets with their frames and
    the densities: the fields oracle.potential.evaluate reads."""

    def __init__(self, bx, by, bnx, bny, bw, tx, ty, geom, mu=None, mu_jet=None, info=None, src=None,
                 f_src=None, jet6=None):
        e = np.zeros(0)
        self.src_x, self.src_y, self.src_w = (e, e, e) if src is None else (np.asarray(a, float) for a in src)
        self.f_src, self.jet6 = f_src, jet6
        self.sigma = self.sigma_jet = None
        self.bnd_x, self.bnd_y, self.bnd_nx, self.bnd_ny, self.bnd_w = bx, by, bnx, bny, bw
        self.tgt_x, self.tgt_y, self.geom = tx, ty, geom
        self.mu, self.mu_jet = mu, mu_jet
        self.info = info or {}

    n_src = property(lambda self: self.src_x.size)
    n_bnd = property(lambda self: self.bnd_x.size)
    n_tgt = property(lambda self: self.tgt_x.size)


def _curvature_override(geom, curvature, tx, ty):
    if curvature is not None:
        c = curvature(np.asarray(tx, float), np.asarray(ty, float))
        geom.update({k: np.asarray(c[k], float) for k in ("kappa", "gamma3", "gamma4")})
    return geom


def on_boundary_problem(bx, by, bnx, bny, bw, q, src=None, curvature=None):
    """Problem whose targets are the boundary nodes themselves, each with its
    local frame from the panels and sgn = +1 (the interior limit); src =
    (x, y, w) of the volume nodes, if any; curvature: see the module header."""
    bx, by = np.asarray(bx, float), np.asarray(by, float)
    fr = G.boundary_frame(bx, by, q, bx, by)
    geom = dict(r=np.zeros(bx.size), nx=fr["nx"], ny=fr["ny"], kappa=fr["kappa"], gamma3=fr["gamma3"],
                gamma4=fr["gamma4"], sgn=np.ones(bx.size, np.int8))
    _curvature_override(geom, curvature, bx, by)
    return _Layer(bx, by, np.asarray(bnx, float), np.asarray(bny, float), np.asarray(bw, float),
                  bx.copy(), by.copy(), geom, info=dict(q=q, pan=fr["pan"], u=fr["u"], curvature=curvature), src=src)


def _target_frames(P, tx, ty):
    """Frames of targets (tx, ty) from P's panels (with P's exact curve derivatives, if any)."""
    fr = G.boundary_frame(P.bnd_x, P.bnd_y, P.info["q"], tx, ty)
    geom = {k: fr[k] for k in ("r", "nx", "ny", "kappa", "gamma3", "gamma4", "sgn")}
    return _curvature_override(geom, P.info.get("curvature"), tx, ty), fr


def _jets(P, mu):
    """mu's jets at the targets' closest points (weights cached on P)."""
    if "jw" not in P.info:
        P.info["jw"] = G.jet_weights(P.bnd_x, P.bnd_y, P.info["q"], P.info["pan"], P.info["u"], 4)
    q = P.info["q"]
    idx = np.asarray(P.info["pan"])[:, None] * q + np.arange(q)[None, :]
    return np.einsum("kij,ij->ki", P.info["jw"], np.asarray(mu, float)[idx])


def apply_interior_double_layer(P, mu):
    """D_int[mu] at the nodes of the on-boundary problem P."""
    Q = copy.copy(P)  # same nodes and frames, this density
    Q.mu = np.asarray(mu, float)
    Q.mu_jet = _jets(P, Q.mu)
    return evaluate(Q, kinds="D")["D"]


def interior_double_layer_matrix(P):
    """Dense matrix of mu -> D_int[mu] at the nodes (column j: unit density at node j)."""
    n = P.n_bnd
    A = np.empty((n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        A[:, j] = apply_interior_double_layer(P, e)
    return A


def volume_at_nodes(P, f_src, jet6):
    """V[f] at the nodes of the on-boundary problem P (volume nodes of P; jet6:
    f and its derivatives at the nodes)."""
    Q = copy.copy(P)
    Q.f_src, Q.jet6 = np.asarray(f_src, float), np.asarray(jet6, float)
    return evaluate(Q, kinds="V")["V"]


def solve_dirichlet(P, g, f_src=None, jet6=None):
    """mu with D_int[mu] = g - V[f] at the nodes (direct solve of the assembled
    operator); f_src = None: the Laplace equation."""
    b = np.asarray(g, float)
    if f_src is not None:
        b = b - volume_at_nodes(P, f_src, jet6)
    return np.linalg.solve(interior_double_layer_matrix(P), b)


def solution_at(P, mu, tx, ty, f_src=None, jet6=None):
    """u = V[f] + D[mu] at targets (tx, ty): their frames and the density's jets
    from the panels, jet6 = f's jets at the targets (with f_src)."""
    q = P.info["q"]
    geom, fr = _target_frames(P, tx, ty)
    T = _Layer(P.bnd_x, P.bnd_y, P.bnd_nx, P.bnd_ny, P.bnd_w, np.asarray(tx, float), np.asarray(ty, float),
               geom, np.asarray(mu, float), G.density_jets(P.bnd_x, P.bnd_y, q, mu, fr["pan"], fr["u"], 4),
               src=(P.src_x, P.src_y, P.src_w), f_src=f_src, jet6=jet6)
    return evaluate(T, kinds="VD" if f_src is not None else "D", delta=delta1_of(P))["total"]


def double_layer_at(P, mu, tx, ty):
    """u = D[mu] at targets (tx, ty)."""
    return solution_at(P, mu, tx, ty)


# ---------------------------------------------------------------------------
# The exterior Dirichlet and the interior Neumann problems (Sec. 5).  Both
# lead to the operator A+[x] = x/2 + (principal value of D[x]) + (sum of
# w_j x_j), which in terms of the interior limit is D_int[x] + x + (w . x):
# * exterior Dirichlet, u = D_E[mu] outside, D_E the double layer plus the
#   integral of mu (the kernel's +1); its exterior limit on the boundary is
#   mu/2 + D[mu] + integral of mu = g (bounded solutions: no logarithmic
#   term; for growth A log|x - x0| the caller moves that term into g);
# * interior Neumann, Green's representation u = V[f] + S[du/dnu] - D[u]; on
#   the boundary u/2 + D[u] = V[f] + S[g].  That operator annihilates
#   constants (D_int[1] = -1); the added integral of u makes it invertible
#   and picks the solution whose boundary integral vanishes (the data are
#   consistent by Gauss's theorem, so the added term is zero at the solution).


def plus_operator_matrix(P):
    """Dense matrix of x -> D_int[x] + x + (w . x) at the nodes of P."""
    n = P.n_bnd
    return interior_double_layer_matrix(P) + np.eye(n) + np.outer(np.ones(n), P.bnd_w)


def single_layer_at_nodes(P, g):
    """S[g] at the nodes of the on-boundary problem P (g's jets from the panels)."""
    Q = copy.copy(P)
    Q.sigma = np.asarray(g, float)
    Q.sigma_jet = G.density_jets(P.bnd_x, P.bnd_y, P.info["q"], Q.sigma, P.info["pan"], P.info["u"], 2)
    return evaluate(Q, kinds="S")["S"]


def solve_exterior_dirichlet(P, g):
    """mu with mu/2 + D[mu] + (integral of mu) = g at the nodes."""
    return np.linalg.solve(plus_operator_matrix(P), np.asarray(g, float))


def exterior_solution_at(P, mu, tx, ty):
    """u = D[mu] + integral of mu at exterior targets (tx, ty)."""
    return solution_at(P, mu, tx, ty) + float(np.dot(P.bnd_w, mu))


def solve_neumann(P, g, f_src=None, jet6=None):
    """Boundary values u with u/2 + D[u] = V[f] + S[g] and zero boundary integral."""
    b = single_layer_at_nodes(P, g)
    if f_src is not None:
        b = b + volume_at_nodes(P, f_src, jet6)
    return np.linalg.solve(plus_operator_matrix(P), b)


def neumann_solution_at(P, ub, g, tx, ty, f_src=None, jet6=None):
    """u = V[f] + S[g] - D[ub] at interior targets (tx, ty)."""
    q = P.info["q"]
    geom, fr = _target_frames(P, tx, ty)
    mu = -np.asarray(ub, float)
    T = _Layer(P.bnd_x, P.bnd_y, P.bnd_nx, P.bnd_ny, P.bnd_w, np.asarray(tx, float), np.asarray(ty, float),
               geom, mu, G.density_jets(P.bnd_x, P.bnd_y, q, mu, fr["pan"], fr["u"], 4),
               src=(P.src_x, P.src_y, P.src_w), f_src=f_src, jet6=jet6)
    T.sigma = np.asarray(g, float)
    T.sigma_jet = G.density_jets(P.bnd_x, P.bnd_y, q, T.sigma, fr["pan"], fr["u"], 2)
    return evaluate(T, kinds="VSD" if f_src is not None else "SD", delta=delta1_of(P))["total"]


# ---------------------------------------------------------------------------
# Exterior problems with a volume source.  The volume local part needs the
# domain on the interior side of a target's frame.  Traversing the boundary
# clockwise makes the outside that side: the frames from the reversed panels
# carry the normal pointing into the curve (the exterior domain's outward
# normal), the matching curvature and sgn = +1 outside.  V[f] is then
# evaluated on the reversed boundary and enters the exterior Dirichlet
# equation as data: mu/2 + D[mu] + integral of mu = g - V[f].


def reversed_boundary(bx, by, bnx, bny, bw):
    """The same nodes traversed clockwise (panel order and node order within
    each panel reversed; Gauss-Legendre nodes are symmetric), normals flipped."""
    return (np.asarray(bx, float)[::-1], np.asarray(by, float)[::-1], -np.asarray(bnx, float)[::-1],
            -np.asarray(bny, float)[::-1], np.asarray(bw, float)[::-1])


def volume_at(P, f_src, jet6, tx, ty, delta=None):
    """V[f] at targets (tx, ty) with their frames from P's panels (P's volume
    nodes; jet6 = f's jets at the targets)."""
    geom, _ = _target_frames(P, tx, ty)
    T = _Layer(P.bnd_x, P.bnd_y, P.bnd_nx, P.bnd_ny, P.bnd_w, np.asarray(tx, float), np.asarray(ty, float), geom,
               src=(P.src_x, P.src_y, P.src_w), f_src=np.asarray(f_src, float), jet6=np.asarray(jet6, float))
    return evaluate(T, kinds="V", delta=delta1_of(P) if delta is None else delta)["V"]
