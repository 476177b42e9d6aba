"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Float64 plans must match the oracle to 1e-10 (relative l_inf per result);
float32 plans to 1e-6 (the tolerances stated for the two precisions)."""
import numpy as np
import pytest

import oracle
from workloads import disk_problem, square_problem, star_problem

pytestmark = pytest.mark.gpu


def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch


def _run(P, which, **opts):
    torch = _gpu()
    from workloads.device import make_plan, run, to_device
    dev = to_device(P)
    plan = make_plan(dev, **opts)
    out = run(plan, dev, which)
    torch.cuda.synchronize()
    return out.cpu().numpy(), plan


def test_disk_fp64_volume_matches_oracle():
    P = disk_problem(2000, seed=1)
    got, plan = _run(P, "V", tol=1e-10, kinds=1)
    ref = oracle.evaluate(P, kinds="V")["V"]
    e = oracle.rel_linf(got, ref)
    print("disk fp64 e_inf", e, plan.info())
    assert e <= 1e-10


def test_star_fp64_all_kinds_match_oracle():
    P = star_problem(1500, seed=4)
    for kinds in ("V", "S", "D", "VSD"):
        mask = (1 if "V" in kinds else 0) | (2 if "S" in kinds else 0) | (4 if "D" in kinds else 0)
        got, plan = _run(P, kinds, tol=1e-10, kinds=mask)
        ref = oracle.evaluate(P, kinds=kinds)["total"]
        e = oracle.rel_linf(got, ref)
        print("star fp64", kinds, "e_inf", e)
        assert e <= 1e-10, (kinds, e)


def test_disk_fp32_volume_matches_oracle():
    P = disk_problem(3000, seed=5)
    got, plan = _run(P, "V", tol=1e-6, precision=0, kinds=1)
    ref = oracle.evaluate(P, kinds="V")["V"]
    e = oracle.rel_linf(got, ref)
    print("disk fp32 e_inf", e, plan.info())
    assert e <= 1e-6
