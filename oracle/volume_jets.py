"""Oracle: the volume density's jets at the volume nodes from per-triangle
quadratic interpolants (the derivatives of f the volume local part of Sec. 4
needs, Lemma 4.1, when f is known only at the nodes of Sec. 2.2's
triangulation).

Test infrastructure only: plain numpy in float64.  Nothing here is imported
by the product path.

Each triangle carries six nodes (stored consecutively); f's quadratic
interpolant at them, written in monomials of the coordinates centred at the
nodes' mean and scaled by their extent, is differentiated at each node:
f, f_x, f_y, f_xx, f_xy, f_yy (the layout of the evaluation's jet6, value
row = the given f).

`patch_jets` fits instead the least-squares quadratic over the triangle's
nodes and those of its edge neighbours: on a sliver the six nodes lie close
to a line and do not fix the derivatives across it, while the neighbours'
nodes do.  Pinned by exactness for quadratics on the split square mesh, by
reducing to `p2_jets` without neighbours, and by h^2 / h convergence of the
slivers' gradient and Hessian for a Gaussian (tests/test_oracle_volume_jets.py).
"""
import numpy as np


def p2_jets(x, y, f):
    """[6, n] jets at the n = 6 M nodes of M triangles."""
    x, y, f = (np.asarray(a, float).reshape(-1, 6) for a in (x, y, f))
    cx, cy = x.mean(1, keepdims=True), y.mean(1, keepdims=True)
    h = np.maximum(np.ptp(x, 1), np.ptp(y, 1))[:, None]
    u, v = (x - cx) / h, (y - cy) / h
    A = np.stack([np.ones_like(u), u, v, u * u, u * v, v * v], 2)       # [M, 6 nodes, 6 monomials]
    c = np.linalg.solve(A, f[..., None])[..., 0]                        # [M, 6]
    out = np.empty((6,) + x.shape)
    out[0] = f
    out[1] = (c[:, 1:2] + 2 * c[:, 3:4] * u + c[:, 4:5] * v) / h
    out[2] = (c[:, 2:3] + c[:, 4:5] * u + 2 * c[:, 5:6] * v) / h
    out[3] = np.broadcast_to(2 * c[:, 3:4] / h ** 2, u.shape)
    out[4] = np.broadcast_to(c[:, 4:5] / h ** 2, u.shape)
    out[5] = np.broadcast_to(2 * c[:, 5:6] / h ** 2, u.shape)
    return out.reshape(6, -1)


def patch_jets(x, y, f, nbr):
    """[6, n] jets at the n = 6 M nodes of M triangles from the least-squares
    quadratic over each triangle's six nodes and the six nodes of each of its
    edge neighbours (nbr [M, 3], -1: none).  Quadratics are invariant under
    affine maps, so the fitted polynomial does not depend on the coordinates;
    they are centred at the triangle's node mean and scaled by the patch's
    extent only to keep the solve well conditioned.  A patch that determines
    no quadratic gives NaN derivatives; the value row is f itself."""
    X, Y, Fv = (np.asarray(a, float).reshape(-1, 6) for a in (x, y, f))
    nbr = np.asarray(nbr).reshape(-1, 3)
    M = len(X)
    out = np.full((6, M, 6), np.nan)
    out[0] = Fv
    for t in range(M):
        ids = [t] + [int(k) for k in nbr[t] if k >= 0]
        px, py, pf = X[ids].ravel(), Y[ids].ravel(), Fv[ids].ravel()
        cx, cy = X[t].mean(), Y[t].mean()
        h = max(np.ptp(px), np.ptp(py))
        if not h > 0:
            continue
        u, v = (px - cx) / h, (py - cy) / h
        A = np.stack([np.ones_like(u), u, v, u * u, u * v, v * v], 1)
        c, _, rank, _ = np.linalg.lstsq(A, pf, rcond=None)
        if rank < 6:
            continue
        uo, vo = (X[t] - cx) / h, (Y[t] - cy) / h
        out[1, t] = (c[1] + 2 * c[3] * uo + c[4] * vo) / h
        out[2, t] = (c[2] + c[4] * uo + 2 * c[5] * vo) / h
        out[3, t] = 2 * c[3] / h ** 2
        out[4, t] = c[4] / h ** 2
        out[5, t] = 2 * c[5] / h ** 2
    return out.reshape(6, -1)
