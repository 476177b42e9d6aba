"""GPU parity of vp_volume_jets (per-triangle quadratic jets of the volume
density) against the oracle's interpolants, exactness for quadratics on a mesh
with slivers and degenerate triangles, and the volume potential evaluated
with the device's jets against the oracle's."""
import copy

import numpy as np
import pytest

import oracle
from oracle.volume_jets import p2_jets
from workloads.problems import disk_problem, square_problem

pytestmark = pytest.mark.gpu

GAUSS = ((1.0, 0.0, 0.0, np.sqrt(0.1)),)


def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch


def _jets(torch, x, y, f):
    from paper_2409_11998_amd import volume_jets
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    out = volume_jets(t(x), t(y), t(f))
    torch.cuda.synchronize()
    return out.cpu().numpy()


def test_disk_matches_oracle_and_volume_potential():
    torch = _gpu()
    D = disk_problem(2000, seed=1, gauss=GAUSS)
    got = _jets(torch, D.src_x, D.src_y, D.f_src)
    ref = p2_jets(D.src_x, D.src_y, D.f_src)
    e = np.max(np.abs(got - ref), axis=1) / np.max(np.abs(ref), axis=1)
    print("disk: relative difference per row", e)
    assert np.all(np.isfinite(got)) and np.all(e <= 1e-11)
    # the volume potential with these jets, device path against the oracle on sampled targets
    from workloads.device import make_plan, run, to_device
    P = copy.copy(D)
    P.jet6 = got
    dev = to_device(P)
    plan = make_plan(dev, tol=1e-10, precision=1, kinds=1)
    out = run(plan, dev, "V").cpu().numpy()
    plan.close()
    idx = np.sort(np.random.default_rng(2).choice(P.n_tgt, 3000, replace=False))
    S = P.subset_targets(idx)
    S.jet6 = ref[:, idx]
    e_v = oracle.rel_linf(out[idx], oracle.evaluate(S, kinds="V")["total"])
    print("V with device jets vs oracle with its jets:", e_v)
    assert e_v <= 1e-10


def test_quadratic_on_slivers_and_degenerate_triangles():
    torch = _gpu()
    S = square_problem(n_tri=3000, n_split=1000, seed=2, n_panels=20, q=16)
    rng = np.random.default_rng(0)
    c = rng.standard_normal(6)
    x, y = S.src_x, S.src_y
    fq = c[0] + c[1] * x + c[2] * y + c[3] * x * x + c[4] * x * y + c[5] * y * y
    ex = np.stack([fq, c[1] + 2 * c[3] * x + c[4] * y, c[2] + c[4] * x + 2 * c[5] * y,
                   np.full(x.size, 2 * c[3]), np.full(x.size, c[4]), np.full(x.size, 2 * c[5])])
    got = _jets(torch, x, y, fq)
    bad = ~np.isfinite(got[1:]).all(axis=0)
    per_tri = bad.reshape(-1, 6)
    w = S.src_w.reshape(-1, 6)
    print("triangles with NaN jets:", int(per_tri.any(1).sum()), "of", per_tri.shape[0])
    # NaN only and wholly for degenerate (zero-area, zero-weight) triangles
    assert np.all(per_tri.all(1) == per_tri.any(1))
    assert np.all(w[per_tri.any(1)] == 0.0)
    assert np.array_equal(got[0], fq)
    ok = ~bad
    e = np.max(np.abs(got[:, ok] - ex[:, ok]), axis=1)
    print("quadratic on slivers (aspect up to 1e4): max error per row", e)
    # f's rounding over the square of a sliver's thickness bounds the Hessian across it
    assert np.all(e[1:3] <= 1e-8) and np.all(e[3:] <= 1e-3)


def test_empty_and_argument_errors():
    torch = _gpu()
    from paper_2409_11998_amd import lib
    from paper_2409_11998_amd.binding import VP_ERR_ARG
    assert lib().vp_volume_jets(0, None, None, None, None, None) == 0
    assert lib().vp_volume_jets(-1, None, None, None, None, None) == VP_ERR_ARG
    assert lib().vp_volume_jets(3, None, None, None, None, None) == VP_ERR_ARG


def test_patch_jets_match_oracle_on_slivers():
    """vp_volume_jets_patch against the oracle's least-squares patch jets on the
    split square mesh (slivers, degenerate triangles, gaps), element by
    element; exact for quadratics there; without neighbours equal to
    vp_volume_jets."""
    torch = _gpu()
    from paper_2409_11998_amd import volume_jets_patch
    from oracle.volume_jets import patch_jets
    from workloads.mesh import square_mesh, triangle_neighbours
    from workloads.problems import gauss_jets
    t = lambda a, dt=torch.float64: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")
    x, y, _, info = square_mesh(3000, 5, 400)
    nbr = triangle_neighbours(info["tri"])
    f = gauss_jets(x, y, ((1.0, 0.1, -0.2, 0.3),))[0]
    got = volume_jets_patch(t(x), t(y), t(f), t(nbr, torch.int32)).cpu().numpy()
    ref = patch_jets(x, y, f, nbr)
    assert np.all(np.isfinite(ref)) and np.all(np.isfinite(got))
    e = np.max(np.abs(got - ref), axis=1) / np.max(np.abs(ref), axis=1)
    print("patch jets against the oracle, relative per row:", e)
    assert e[0] == 0.0 and np.all(e <= 1e-9)
    rng = np.random.default_rng(3)
    c = rng.standard_normal(6)
    q = c[0] + c[1] * x + c[2] * y + c[3] * x * x + c[4] * x * y + c[5] * y * y
    got = volume_jets_patch(t(x), t(y), t(q), t(nbr, torch.int32)).cpu().numpy()
    ex = np.stack([q, c[1] + 2 * c[3] * x + c[4] * y, c[2] + c[4] * x + 2 * c[5] * y,
                   np.full(x.size, 2 * c[3]), np.full(x.size, c[4]), np.full(x.size, 2 * c[5])])
    print("quadratic: max error", np.max(np.abs(got - ex)))
    assert np.max(np.abs(got - ex)) <= 1e-8
    D = disk_problem(2000, seed=1, gauss=GAUSS)
    none = np.full((D.src_x.size // 6, 3), -1, np.int32)
    got = volume_jets_patch(t(D.src_x), t(D.src_y), t(D.f_src), t(none, torch.int32)).cpu().numpy()
    ref = _jets(torch, D.src_x, D.src_y, D.f_src)
    e = np.max(np.abs(got - ref), axis=1) / np.max(np.abs(ref), axis=1)
    print("without neighbours against vp_volume_jets:", e)
    assert np.all(e <= 1e-9)


def test_patch_jets_ignore_invalid_neighbours():
    """Neighbour entries outside [0, n_tri) or naming the triangle itself count
    as none: the result equals the one with -1 there."""
    torch = _gpu()
    from paper_2409_11998_amd import volume_jets_patch
    from workloads.mesh import square_mesh, triangle_neighbours
    t = lambda a, dt=torch.float64: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")
    x, y, _, info = square_mesh(1200, 7, 150)
    nbr = triangle_neighbours(info["tri"])
    m = len(nbr)
    rng = np.random.default_rng(4)
    bad = nbr.copy()
    none = bad < 0
    junk = rng.choice(np.array([m, m + 5, -7, 2 ** 31 - 1], np.int64), size=int(none.sum()))
    bad[none] = junk.astype(np.int32)
    self_rows = rng.choice(m, 20, replace=False)
    ref_nbr = nbr.copy()
    bad[self_rows, 0] = self_rows
    ref_nbr[self_rows, 0] = -1
    f = np.sin(3 * x) * np.cos(2 * y)
    a = volume_jets_patch(t(x), t(y), t(f), t(bad, torch.int32)).cpu().numpy()
    b = volume_jets_patch(t(x), t(y), t(f), t(ref_nbr, torch.int32)).cpu().numpy()
    assert np.array_equal(np.isnan(a), np.isnan(b))
    assert np.array_equal(a[~np.isnan(a)], b[~np.isnan(b)])
    empty = torch.zeros(0, dtype=torch.float64, device="cuda")
    assert volume_jets_patch(empty, empty, empty, torch.zeros(0, dtype=torch.int32, device="cuda")).numel() == 0
