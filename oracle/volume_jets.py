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
