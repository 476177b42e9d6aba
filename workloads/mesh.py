"""Seeded triangulations and their volume quadrature nodes.

Meshes follow the paper's experimental setup (Sec. 6): unstructured
triangulations with six quadrature nodes per triangle, curved boundary
elements, and (Sec. 6.4) meshes made non-conforming and degenerate by random
splitting, with gaps from removed triangles.  Triangulations come from
scipy's Delaunay on jittered hexagonal lattices (the paper's mesher is not
available offline).
"""
import numpy as np
from scipy.spatial import Delaunay, cKDTree

from .rule import six_point_rule


def hex_lattice(h, box, rng, jitter=0.25):
    (x0, x1), (y0, y1) = box
    dy = h * np.sqrt(3.0) / 2.0
    ys = np.arange(y0 - h, y1 + h, dy)
    pts = []
    for i, y in enumerate(ys):
        off = 0.5 * h * (i % 2)
        xs = np.arange(x0 - h + off, x1 + h, h)
        pts.append(np.stack([xs, np.full_like(xs, y)], axis=1))
    p = np.concatenate(pts)
    p += rng.uniform(-jitter * h, jitter * h, size=p.shape)
    return p


def _p2_shape(xi, eta):
    """P2 Lagrange shape functions on the reference triangle and derivatives.

    Node order: v0 (0,0), v1 (1,0), v2 (0,1), m01, m12, m20.
    """
    l0 = 1 - xi - eta
    N = np.array([l0 * (2 * l0 - 1), xi * (2 * xi - 1), eta * (2 * eta - 1),
                  4 * l0 * xi, 4 * xi * eta, 4 * eta * l0])
    dxi = np.array([-(4 * l0 - 1), 4 * xi - 1, 0.0 * xi, 4 * (l0 - xi), 4 * eta, -4 * eta])
    deta = np.array([-(4 * l0 - 1), 0.0 * xi, 4 * eta - 1, -4 * xi, 4 * xi, 4 * (l0 - eta)])
    return N, dxi, deta


def quadrature_nodes(P, tri, curved_mid=None):
    """Six nodes per triangle.

    P: (np,2) vertices, tri: (M,3).  curved_mid: optional dict-like arrays
    (tri_index[], edge_index[], midpoint[.,2]) giving, for triangles with a
    curved boundary edge, that edge's midpoint on the curve (P2 element).
    Straight triangles use the affine map; weights = rule weight * |area|.
    Returns x (M*6,), y, w.
    """
    bary, wq = six_point_rule()
    A = P[tri[:, 0]]
    B = P[tri[:, 1]]
    C = P[tri[:, 2]]
    area = 0.5 * np.abs((B[:, 0] - A[:, 0]) * (C[:, 1] - A[:, 1])
                        - (C[:, 0] - A[:, 0]) * (B[:, 1] - A[:, 1]))
    # node = l1*A + l2*B + l3*C
    X = (bary[None, :, 0, None] * A[:, None, :] + bary[None, :, 1, None] * B[:, None, :]
         + bary[None, :, 2, None] * C[:, None, :])
    W = area[:, None] * wq[None, :]
    if curved_mid is not None and len(curved_mid[0]):
        ti, ei, mp = curved_mid
        # reference coords of the rule nodes: vertex0=A (0,0), vertex1=B (1,0), vertex2=C (0,1)
        xi = bary[:, 1]
        eta = bary[:, 2]
        N, dxi, deta = _p2_shape(xi, eta)  # (6 shape, 6 nodes)
        for e in range(3):
            sel = ei == e
            if not np.any(sel):
                continue
            t = ti[sel]
            V = np.stack([P[tri[t, 0]], P[tri[t, 1]], P[tri[t, 2]]], axis=1)  # (m,3,2)
            mids = np.stack([0.5 * (V[:, 0] + V[:, 1]), 0.5 * (V[:, 1] + V[:, 2]),
                             0.5 * (V[:, 2] + V[:, 0])], axis=1)
            mids[:, e] = mp[sel]
            nodes = np.concatenate([V, mids], axis=1)  # (m,6,2)
            X[t] = np.einsum("sq,msd->mqd", N, nodes)
            jx = np.einsum("sq,msd->mqd", dxi, nodes)
            jy = np.einsum("sq,msd->mqd", deta, nodes)
            det = jx[..., 0] * jy[..., 1] - jx[..., 1] * jy[..., 0]
            W[t] = 0.5 * wq[None, :] * np.abs(det)
    return X[..., 0].ravel(), X[..., 1].ravel(), W.ravel()


def _boundary_edges(tri, nb, closed=True):
    """Triangles owning an edge between consecutive boundary vertices 0..nb-1."""
    ti, ei, a_idx = [], [], []
    for e, (p, q) in enumerate([(0, 1), (1, 2), (2, 0)]):
        a = tri[:, p]
        b = tri[:, q]
        isb = (a < nb) & (b < nb)
        d = (b - a) % nb
        cons = isb & ((d == 1) | (d == nb - 1))
        idx = np.nonzero(cons)[0]
        lo = np.where(((b[idx] - a[idx]) % nb) == 1, a[idx], b[idx])
        ti.append(idx)
        ei.append(np.full(idx.size, e))
        a_idx.append(lo)
    return np.concatenate(ti), np.concatenate(ei), np.concatenate(a_idx)


def curve_mesh(curve, n_tri, seed, margin=0.5):
    """Triangulate the interior of a closed CCW curve.

    curve: object with .point(t) -> (n,2), .length, .t_of_s(s) (arclength
    inverse) and .inside(p) -> bool[].  Boundary vertices are placed at equal
    arclength; boundary triangles get a P2 map with the edge midpoint on the
    curve.  Returns (x, y, w, info).
    """
    rng = np.random.default_rng(seed)
    area = curve.area
    h = np.sqrt(area / (n_tri * np.sqrt(3.0) / 4.0))
    nb = max(8, int(round(curve.length / h)))
    s = (np.arange(nb) + rng.uniform(0, 1)) * (curve.length / nb)
    tb = curve.t_of_s(s)
    Pb = curve.point(tb)
    lo = Pb.min(axis=0) - h
    hi = Pb.max(axis=0) + h
    Pi = hex_lattice(h, ((lo[0], hi[0]), (lo[1], hi[1])), rng)
    Pi = Pi[curve.inside(Pi)]
    dense = curve.point(curve.t_of_s(np.linspace(0, curve.length, 16 * nb, endpoint=False)))
    # only "closer than margin*h" matters; a bounded query avoids the degenerate
    # all-equidistant search for points deep inside a circle
    dist, _ = cKDTree(dense).query(Pi, distance_upper_bound=margin * h)
    Pi = Pi[~np.isfinite(dist)]
    P = np.concatenate([Pb, Pi])
    tri = Delaunay(P).simplices
    cen = P[tri].mean(axis=1)
    tri = tri[curve.inside(cen)]
    # orient triangles counterclockwise
    A, B, C = P[tri[:, 0]], P[tri[:, 1]], P[tri[:, 2]]
    cr = (B[:, 0] - A[:, 0]) * (C[:, 1] - A[:, 1]) - (C[:, 0] - A[:, 0]) * (B[:, 1] - A[:, 1])
    neg = cr < 0
    tri[neg] = tri[neg][:, [0, 2, 1]]
    ti, ei, a = _boundary_edges(tri, nb)
    # parameter midpoint of the arc between boundary vertex a and a+1
    s_mid = (s[a] + 0.5 * curve.length / nb)
    mp = curve.point(curve.t_of_s(np.mod(s_mid, curve.length)))
    x, y, w = quadrature_nodes(P, tri, (ti, ei, mp))
    info = dict(h=h, n_tri=len(tri), n_bnd_vertices=nb, vertices=P, tri=tri)
    return x, y, w, info


def triangle_neighbours(tri):
    """[M, 3] int32: for each triangle the triangle across each of its edges
    (edge e joins vertices e and e+1), -1 where no other triangle has that
    edge (the boundary, a gap, or a nonconforming side)."""
    tri = np.asarray(tri)
    M = len(tri)
    a = tri
    b = np.roll(tri, -1, axis=1)
    lo, hi = np.minimum(a, b).ravel(), np.maximum(a, b).ravel()
    key = lo.astype(np.int64) * (int(tri.max()) + 1) + hi
    order = np.argsort(key, kind="stable")
    ks = key[order]
    out = np.full(3 * M, -1, np.int64)
    same = np.nonzero(ks[1:] == ks[:-1])[0]           # pairs of half-edges on one edge
    e0, e1 = order[same], order[same + 1]
    out[e0] = e1 // 3
    out[e1] = e0 // 3
    return out.reshape(M, 3).astype(np.int32)


def square_mesh(n_tri, seed, n_split, degenerate_frac=0.05, gap_frac=0.002):
    """Straight-sided mesh of [-1,1]^2, then random splits and gaps (Sec. 6.4).

    n_tri: triangles before splitting.  n_split triangles are each split in
    two by a line from the opposite vertex to a random point on a random
    interior side, placed at a log-uniform fraction in [1e-4, 0.5] of the
    side from one of its endpoints (a fraction degenerate_frac is put exactly
    on the endpoint, giving zero-area triangles).  Then gap_frac of all
    triangles are removed.
    """
    rng = np.random.default_rng(seed)
    h = np.sqrt(4.0 / (n_tri * np.sqrt(3.0) / 4.0))
    nside = int(round(2.0 / h))
    e = np.linspace(-1, 1, nside + 1)
    bnd = np.concatenate([
        np.stack([e[:-1], np.full(nside, -1.0)], 1),
        np.stack([np.full(nside, 1.0), e[:-1]], 1),
        np.stack([e[::-1][:-1], np.full(nside, 1.0)], 1),
        np.stack([np.full(nside, -1.0), e[::-1][:-1]], 1)])
    Pi = hex_lattice(h, ((-1, 1), (-1, 1)), rng)
    m = 0.5 * h
    Pi = Pi[(np.abs(Pi[:, 0]) < 1 - m) & (np.abs(Pi[:, 1]) < 1 - m)]
    P = np.concatenate([bnd, Pi])
    tri = Delaunay(P).simplices
    nb = len(bnd)
    # split
    M = len(tri)
    pick = rng.choice(M, size=min(n_split, M), replace=False)
    keep = np.ones(M, bool)
    keep[pick] = False
    newP = [P]
    newT = [tri[keep]]
    base = len(P)
    Tp = tri[pick]
    side = rng.integers(0, 3, size=len(pick))
    # an interior side: both endpoints boundary vertices on the same edge means boundary side
    a_i = Tp[np.arange(len(pick)), side]
    b_i = Tp[np.arange(len(pick)), (side + 1) % 3]
    o_i = Tp[np.arange(len(pick)), (side + 2) % 3]
    onb = (a_i < nb) & (b_i < nb)
    side = np.where(onb, (side + 1) % 3, side)
    a_i = Tp[np.arange(len(pick)), side]
    b_i = Tp[np.arange(len(pick)), (side + 1) % 3]
    o_i = Tp[np.arange(len(pick)), (side + 2) % 3]
    frac = np.exp(rng.uniform(np.log(1e-4), np.log(0.5), size=len(pick)))
    frac[rng.uniform(size=len(pick)) < degenerate_frac] = 0.0
    flip = rng.uniform(size=len(pick)) < 0.5
    frac = np.where(flip, 1.0 - frac, frac)
    Q = P[a_i] + frac[:, None] * (P[b_i] - P[a_i])
    qi = base + np.arange(len(pick))
    newP.append(Q)
    newT.append(np.stack([a_i, qi, o_i], 1))
    newT.append(np.stack([qi, b_i, o_i], 1))
    P = np.concatenate(newP)
    tri = np.concatenate(newT)
    # gaps
    nrem = int(round(gap_frac * len(tri)))
    if nrem:
        drop = rng.choice(len(tri), size=nrem, replace=False)
        k = np.ones(len(tri), bool)
        k[drop] = False
        tri = tri[k]
    x, y, w = quadrature_nodes(P, tri)
    A, B, C = P[tri[:, 0]], P[tri[:, 1]], P[tri[:, 2]]
    ar = 0.5 * np.abs((B[:, 0] - A[:, 0]) * (C[:, 1] - A[:, 1]) - (C[:, 0] - A[:, 0]) * (B[:, 1] - A[:, 1]))
    ed = np.stack([np.linalg.norm(B - A, axis=1), np.linalg.norm(C - B, axis=1),
                   np.linalg.norm(A - C, axis=1)], 1)
    longest = ed.max(1)
    with np.errstate(divide="ignore"):
        aspect = longest ** 2 / np.maximum(2 * ar, 1e-300)
    info = dict(h=h, n_tri=len(tri), aspect=aspect, removed_area=4.0 - ar.sum(),
                n_degenerate=int(np.sum(ar <= 1e-15)), vertices=P, tri=tri)
    return x, y, w, info
