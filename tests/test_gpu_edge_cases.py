"""Edge cases of the plan/evaluate path on the GPU: no targets, one target and
ragged target counts, coincident nodes, and inputs the planner must reject."""
import copy

import numpy as np
import pytest

import oracle
from workloads import star_problem

pytestmark = pytest.mark.gpu


def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch


def test_no_targets_is_a_no_op():
    torch = _gpu()
    from workloads.device import make_plan, run, to_device
    P = star_problem(600, seed=50).subset_targets(np.arange(0))
    dev = to_device(P)
    for precision in (1, 0):
        plan = make_plan(dev, tol=1e-10 if precision else 1e-6, precision=precision, kinds=7)
        out = run(plan, dev, "VSD", out=torch.empty(0, dtype=torch.float64, device="cuda"))
        torch.cuda.synchronize()
        assert out.numel() == 0 and plan.info()["n_tgt"] == 0
        plan.close()


@pytest.mark.parametrize("n", [1, 33, 257])
def test_one_and_ragged_target_counts(n):
    """Target counts that fill no chunk, tile or workgroup evenly."""
    torch = _gpu()
    from workloads.device import make_plan, run, to_device
    P0 = star_problem(1500, seed=51)
    rng = np.random.default_rng(n)
    P = P0.subset_targets(np.sort(rng.choice(P0.n_tgt, n, replace=False)))
    ref = oracle.evaluate(P, kinds="VSD")["total"]
    dev = to_device(P)
    for precision, tol in ((1, 1e-10), (0, 1e-6)):
        plan = make_plan(dev, tol=tol, precision=precision, kinds=7)
        out = run(plan, dev, "VSD")
        torch.cuda.synchronize()
        e = oracle.rel_linf(out.cpu().numpy(), ref)
        print("n", n, "precision", precision, "e_inf", e)
        assert e <= tol
        plan.close()


def test_coincident_nodes_split_weight():
    """Duplicating volume nodes with their weight split in halves leaves the
    result unchanged once delta_1 is held fixed (c_delta scaled by N'/N, as
    delta_1 = c_delta sum(w) / N): spreading is linear in the strengths."""
    torch = _gpu()
    from workloads.device import make_plan, run, to_device
    P = star_problem(1500, seed=52)
    dup = np.arange(0, P.n_src, 7)
    Q = copy.copy(P)
    Q.src_x = np.concatenate([P.src_x, P.src_x[dup]])
    Q.src_y = np.concatenate([P.src_y, P.src_y[dup]])
    w = P.src_w.copy()
    w[dup] *= 0.5
    Q.src_w = np.concatenate([w, w[dup]])
    Q.f_src = np.concatenate([P.f_src, P.f_src[dup]])
    c_delta = 3.0 * Q.n_src / P.n_src
    res = []
    for prob, cd in ((P, 3.0), (Q, c_delta)):
        dev = to_device(prob)
        plan = make_plan(dev, tol=1e-10, precision=1, kinds=7, c_delta=cd)
        assert abs(plan.info()["delta1"] - oracle.delta1_of(P)) <= 1e-15 * oracle.delta1_of(P)
        out = run(plan, dev, "VSD")
        torch.cuda.synchronize()
        res.append(out.cpu().numpy())
        plan.close()
    e = oracle.rel_linf(res[1], res[0])
    print("coincident nodes: rel diff", e)
    assert e <= 1e-10


def test_inputs_the_planner_rejects():
    torch = _gpu()
    from paper_2409_11998_amd.binding import VP_ERR_ARG, VP_ERR_GEOMETRY, VPError
    from workloads.device import make_plan, to_device
    P = star_problem(600, seed=53)

    def expect(status, mutate):
        dev = to_device(P)
        mutate(dev)
        with pytest.raises(VPError) as ei:
            make_plan(dev, tol=1e-10, kinds=7)
        assert ei.value.status == status, ei.value

    def nan_pos(d):
        d["src_x"][3] = float("nan")

    def neg_w(d):
        d["src_w"][5] = -1.0

    def neg_bw(d):
        d["bnd_w"][2] = -1e-3

    def bad_sgn(d):
        d["geom"]["sgn"][0] = 2

    def neg_r(d):
        d["geom"]["r"][1] = -0.5

    def exterior_near(d):          # a target just outside the boundary, with the volume kind
        d["geom"]["sgn"][0] = -1
        d["geom"]["r"][0] = 1e-6

    for m in (nan_pos, neg_w, neg_bw, bad_sgn, neg_r):
        expect(VP_ERR_ARG, m)
    expect(VP_ERR_GEOMETRY, exterior_near)
