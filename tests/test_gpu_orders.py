"""GPU parity at every truncation order of the local expansions (Sec. 4:
V_L through delta^2, S_L and D_L through the delta^2 terms of Lemmas 4.3 and
4.5), device against the oracle at the same orders."""
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


@pytest.mark.parametrize("orders", [(4, 4, 4), (2, 1, 1), (0, 0, 0), (3, 2, 4)])
def test_orders_match_oracle(orders):
    torch = _gpu()
    from workloads.device import make_plan, run, to_device
    ov, os_, od = orders
    P = star_problem(1500, seed=61)
    idx = np.sort(np.random.default_rng(7).choice(P.n_tgt, 2500, replace=False))
    ref = oracle.evaluate(P.subset_targets(idx), kinds="VSD", order_v=ov, order_s=os_, order_d=od)["total"]
    dev = to_device(P)
    plan = make_plan(dev, tol=1e-10, precision=1, kinds=7, order_v=ov, order_s=os_, order_d=od)
    out = run(plan, dev, "VSD").cpu().numpy()
    plan.close()
    e = oracle.rel_linf(out[idx], ref)
    print("orders", orders, "e_inf vs oracle", e)
    assert e <= 1e-10


def test_order_four_layers_on_the_sliver_square():
    """The layers' delta^2 terms on the workload with slivers, gaps and
    targets on the boundary (D only, as in the benchmark)."""
    torch = _gpu()
    from workloads import config_problem
    from workloads.device import make_plan, run, to_device
    P = config_problem(2, scale=0.05)
    near = np.flatnonzero(np.asarray(P.geom["r"]) <= 0.05)
    idx = np.sort(np.random.default_rng(8).choice(near, min(1500, near.size), replace=False))
    ref = oracle.evaluate(P.subset_targets(idx), kinds="VD", order_d=4)["total"]
    dev = to_device(P)
    plan = make_plan(dev, tol=1e-10, precision=1, kinds=5, order_d=4)
    out = run(plan, dev, "VD").cpu().numpy()
    plan.close()
    e = oracle.rel_linf(out[idx], ref)
    print("square, order_d = 4, near-boundary targets: e_inf vs oracle", e)
    assert e <= 1e-10
