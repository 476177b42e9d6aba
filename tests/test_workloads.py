"""Input generators: the derived triangle rule and mesh/geometry sanity."""
import numpy as np

from workloads import disk_problem, square_problem, star_problem
from workloads.rule import six_point_rule


def test_six_point_rule_exact_to_degree_four():
    bary, w = six_point_rule()
    # reference triangle (0,0),(1,0),(0,1): x = l2, y = l3; int x^i y^j = i! j! / (i+j+2)!
    from math import factorial
    x, y = bary[:, 1], bary[:, 2]
    for i in range(5):
        for j in range(5 - i):
            exact = factorial(i) * factorial(j) / factorial(i + j + 2)
            assert abs(0.5 * np.sum(w * x ** i * y ** j) - exact) < 1e-15
    assert np.all(w > 0) and abs(w.sum() - 1) < 1e-15


def test_disk_mesh_area_and_geometry():
    P = disk_problem(1500, seed=3)
    assert abs(P.src_w.sum() - np.pi) < 1e-6
    assert np.all(P.geom["r"] > 0) and np.all(P.geom["sgn"] == 1)


def test_square_mesh_has_slivers_degenerates_and_gaps():
    P = square_problem(6000, 800, seed=2, n_panels=20, q=10)
    info = P.info
    assert info["n_degenerate"] > 0
    assert np.max(info["aspect"][np.isfinite(info["aspect"])]) > 1e3
    assert 0 < info["removed_area"] < 0.05
    assert abs(P.src_w.sum() + info["removed_area"] - 4.0) < 1e-9
    assert abs(P.bnd_w.sum() - 8.0) < 1e-12


def test_star_geometry_closest_point():
    P = star_problem(800, seed=4)
    g = P.geom
    m = P.info["near_mask"]
    assert m.sum() > 100
    # far targets carry a lower bound of their distance, above 12 sqrt(delta_1)
    d1 = 3 * P.src_w.sum() / P.n_src
    assert np.all(g["r"][~m] > 12 * np.sqrt(d1))
    bx = (P.tgt_x + g["sgn"] * g["r"] * g["nx"])[m]
    by = (P.tgt_y + g["sgn"] * g["r"] * g["ny"])[m]
    # b lies on the boundary: its distance to the dense boundary nodes is tiny
    from scipy.spatial import cKDTree
    d, _ = cKDTree(np.stack([P.bnd_x, P.bnd_y], 1)).query(np.stack([bx, by], 1))
    assert np.max(d) < 0.05
