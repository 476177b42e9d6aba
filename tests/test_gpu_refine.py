"""GPU parity of the dyadic refinement of the local layer parts (vp_refine_attach /
vp_layer_refine) against the oracle's level-by-level evaluation (Sec. 4)."""
import numpy as np
import pytest

import oracle
from oracle import refine
from workloads import star_problem
from workloads.problems import fine_boundary

pytestmark = pytest.mark.gpu


def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch


def _fine_dev(torch, fine):
    return {k: (torch.as_tensor(v, dtype=torch.float64, device="cuda") if v is not None else None)
            for k, v in fine.items()}


@pytest.mark.parametrize("precision,levels,kinds", [(1, 3, "SD"), (1, 1, "VSD"), (0, 3, "VSD"), (1, 3, "D")])
def test_refined_layers_match_oracle(precision, levels, kinds):
    torch = _gpu()
    from workloads.device import make_plan, run, to_device
    P = star_problem(1500, seed=21)
    fine = fine_boundary(P, levels)
    dev = to_device(P)
    mask = (1 if "V" in kinds else 0) | (2 if "S" in kinds else 0) | (4 if "D" in kinds else 0)
    tol = 1e-10 if precision == 1 else 1e-6
    plan = make_plan(dev, tol=tol, precision=precision, kinds=mask)
    out = run(plan, dev, kinds)
    fd = _fine_dev(torch, fine)
    plan.refine_attach(levels, fd["x"], fd["y"], fd["nx"], fd["ny"], fd["w"], dev["tgt_x"], dev["tgt_y"])
    plan.layer_refine(out, sigma_jet=dev["sigma_jet"] if "S" in kinds else None,
                      fine_sigma=fd["sigma"] if "S" in kinds else None,
                      mu_jet=dev["mu_jet"] if "D" in kinds else None, fine_mu=fd["mu"] if "D" in kinds else None)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    delta = plan.info()["delta1"]
    ref = oracle.evaluate(P, kinds=kinds)["total"] + refine.layer_refinement(P, fine, levels, delta, kinds=kinds)
    corr = refine.layer_refinement(P, fine, levels, delta, kinds=kinds)
    e = oracle.rel_linf(got, ref)
    print("refined", precision, levels, kinds, "e_inf", e, "max |correction|", np.abs(corr).max(),
          "fine nodes", fine["x"].size)
    assert np.abs(corr).max() > 0          # the correction is exercised
    assert e <= tol
    plan.close()


def test_refinement_argument_errors():
    torch = _gpu()
    from paper_2409_11998_amd.binding import VP_ERR_ARG, VPError
    from workloads.device import make_plan, to_device
    P = star_problem(600, seed=22)
    dev = to_device(P)
    plan = make_plan(dev, tol=1e-10, kinds=6)
    out = torch.zeros(P.n_tgt, dtype=torch.float64, device="cuda")
    with pytest.raises(VPError) as ei:
        plan.layer_refine(out, mu_jet=dev["mu_jet"], fine_mu=dev["mu"])
    assert ei.value.status == VP_ERR_ARG          # nothing attached
    fd = _fine_dev(torch, fine_boundary(P, 2))
    with pytest.raises(VPError):
        plan.refine_attach(0, fd["x"], fd["y"], fd["nx"], fd["ny"], fd["w"], dev["tgt_x"], dev["tgt_y"])
    bad_w = fd["w"].clone()
    bad_w[3] = -1.0
    with pytest.raises(VPError):
        plan.refine_attach(2, fd["x"], fd["y"], fd["nx"], fd["ny"], bad_w, dev["tgt_x"], dev["tgt_y"])
    plan.refine_attach(2, fd["x"], fd["y"], fd["nx"], fd["ny"], fd["w"], dev["tgt_x"], dev["tgt_y"])
    with pytest.raises(VPError):                 # pairs come together
        plan.layer_refine(out, mu_jet=dev["mu_jet"])
    plan.layer_refine(out, mu_jet=dev["mu_jet"], fine_mu=fd["mu"])
    torch.cuda.synchronize()
    plan.close()
