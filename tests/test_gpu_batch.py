"""Batched execution (one kernel per stage for all instances): every instance's result equals its own
single-plan result (the same kernels; only LDS atomic order may differ) and the
oracle, eagerly and on repeated graph replays with eager work in between."""
import numpy as np
import pytest

import oracle
from workloads import star_problem

pytestmark = pytest.mark.gpu


def _setup(precision, sizes, kinds="VD", seed0=40):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from workloads.device import make_batch_plans, run, to_device
    probs = [star_problem(n, seed=seed0 + i) for i, n in enumerate(sizes)]
    tol = 1e-10 if precision == 1 else 1e-6
    mask = (1 if "V" in kinds else 0) | (2 if "S" in kinds else 0) | (4 if "D" in kinds else 0)
    devs = [to_device(P) for P in probs]
    plans = make_batch_plans(devs, classes=2, tol=tol, precision=precision, kinds=mask)
    return torch, probs, devs, plans, run, mask


@pytest.mark.parametrize("precision", [1, 0])
def test_batch_matches_single_plans_and_oracle(precision):
    from paper_2409_11998_amd import Batch
    torch, probs, devs, plans, run, mask = _setup(precision, [300, 1200, 700, 2500, 450])
    batch = Batch(plans, mask)
    outs = [torch.full((P.n_tgt,), np.nan, dtype=torch.float64, device="cuda") for P in probs]
    args = [dict(f=d["f"], jet6=d["jet6"], mu=d["mu"], mu_jet=d["mu_jet"], out=o) for d, o in zip(devs, outs)]
    # the batch runs first: its plans' workspaces hold nothing of a single-plan evaluation yet
    batch.eval(args, graph=False)
    batch.stream.synchronize()
    first = [o.cpu().numpy() for o in outs]
    single = []
    for p, d in zip(plans, devs):
        single.append(run(p, d, "VD").clone())
    torch.cuda.synchronize()
    for i, (g, s1) in enumerate(zip(first, single)):
        assert oracle.rel_linf(g, s1.cpu().numpy()) <= (1e-13 if precision == 1 else 1e-6), i
    tol = 1e-10 if precision == 1 else 1e-6
    refs = [oracle.evaluate(P, kinds="VD")["total"] for P in probs]
    for rep, graph in enumerate([False, True, True, True]):
        for o in outs:
            o.fill_(np.nan)
        batch.eval(args, graph=graph)
        batch.stream.synchronize()
        # eager work between replays on the default stream
        for p, d in zip(plans[:1], devs[:1]):
            run(p, d, "VD")
        torch.cuda.synchronize()
        for i, (o, s1, ref) in enumerate(zip(outs, single, refs)):
            got = o.cpu().numpy()
            assert np.all(np.isfinite(got)), (rep, i)
            e_single = oracle.rel_linf(got, s1.cpu().numpy())
            e_oracle = oracle.rel_linf(got, ref)
            print("rep", rep, "inst", i, "batch vs single", e_single, "batch vs oracle", e_oracle,
                  "single vs oracle", oracle.rel_linf(s1.cpu().numpy(), ref))
            assert e_single <= (1e-13 if precision == 1 else 1e-6), (rep, i, e_single)
            assert e_oracle <= tol, (rep, i, e_oracle)
    # a timed call (events between the stage kinds, no graph) gives the same results
    batch.set_timing(True)
    for o in outs:
        o.fill_(np.nan)
    batch.eval(args, graph=True)
    t = batch.timing()
    batch.set_timing(False)
    print("batch stage times (ms)", t)
    assert set(t) == set(Batch.BATCH_STAGES) and all(v >= 0 for v in t.values())
    assert t["spread"] > 0 and t["interp"] > 0 and t["col_fft_mul"] > 0
    for o, s1 in zip(outs, single):
        assert oracle.rel_linf(o.cpu().numpy(), s1.cpu().numpy()) <= (1e-13 if precision == 1 else 1e-6)
    batch.close()


def test_batch_mixed_widths_run_and_mixed_precisions_are_rejected():
    """Instances may differ in spreading width (one launch per distinct width);
    they may not differ in precision."""
    from paper_2409_11998_amd import Batch, VPError
    torch, probs, devs, plans, run, mask = _setup(1, [300, 400])
    from workloads.device import make_plan
    loose = make_plan(devs[1], tol=1e-5, precision=1, kinds=mask)       # narrower kernel
    assert tuple(loose.info()["width"]) != tuple(plans[0].info()["width"])
    pair = [plans[0], loose]
    single = [run(p, d, "VD").clone() for p, d in zip(pair, devs)]
    torch.cuda.synchronize()
    batch = Batch(pair, mask)
    outs = [torch.full((P.n_tgt,), np.nan, dtype=torch.float64, device="cuda") for P in probs]
    args = [dict(f=d["f"], jet6=d["jet6"], mu=d["mu"], mu_jet=d["mu_jet"], out=o) for d, o in zip(devs, outs)]
    for graph in (False, True, True):
        batch.eval(args, graph=graph)
        batch.stream.synchronize()
        for o, s1 in zip(outs, single):
            assert oracle.rel_linf(o.cpu().numpy(), s1.cpu().numpy()) <= 1e-13
    batch.close()
    fp32 = make_plan(devs[1], tol=1e-6, precision=0, kinds=mask)
    with pytest.raises(VPError):
        Batch([plans[0], fp32], mask)
