"""Serving loop: each request's result is the same alone and in a mix of
concurrent requests (and matches the oracle); in-flight workspace never
exceeds the HBM budget; oversized and invalid requests fail alone."""
import numpy as np
import pytest

import oracle
from workloads import star_problem

pytestmark = pytest.mark.gpu

KINDS = ["V", "S", "D", "VD", "VSD", "V"]
PRECS = [1, 0, 1, 0, 1, 0]


def _problems():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from workloads.device import make_plan, to_device
    probs = [star_problem(n, seed=60 + i) for i, n in enumerate([400, 1500, 800, 2500, 600, 1100])]
    devs = [to_device(P) for P in probs]
    plans = []
    for d, k, pr in zip(devs, KINDS, PRECS):
        mask = (1 if "V" in k else 0) | (2 if "S" in k else 0) | (4 if "D" in k else 0)
        plans.append(make_plan(d, tol=1e-10 if pr == 1 else 1e-6, precision=pr, kinds=mask, no_workspace=True))
    return torch, probs, devs, plans


def _args(d, k):
    return dict(f=d["f"] if "V" in k else None, jet6=d["jet6"] if "V" in k else None,
                sigma=d["sigma"] if "S" in k else None, sigma_jet=d["sigma_jet"] if "S" in k else None,
                mu=d["mu"] if "D" in k else None, mu_jet=d["mu_jet"] if "D" in k else None)


def test_results_same_alone_and_in_the_mix():
    from paper_2409_11998_amd import Server
    torch, probs, devs, plans = _problems()
    alone = []
    for p, d, k in zip(plans, devs, KINDS):
        alone.append(p.eval(**_args(d, k)).clone())   # temporary stream-ordered workspace
    torch.cuda.synchronize()
    # a 200 ms admission window: requests submitted back to back share groups
    srv = Server(hbm_budget_bytes=2 << 30, max_in_flight=6, n_streams=4, max_wait_us=200000)
    reps = 4
    order = [i for rep in range(reps) for i in np.random.default_rng(rep).permutation(len(plans))]
    outs = [torch.full((probs[i].n_tgt,), np.nan, dtype=torch.float64, device="cuda") for i in order]
    torch.cuda.synchronize()
    tickets = [(i, srv.submit(plans[i], o, **_args(devs[i], KINDS[i]))) for i, o in zip(order, outs)]
    for (i, t), o in zip(tickets, outs):
        st, lat = srv.wait(t, timeout=120)
        assert st == 0
        got = o.cpu().numpy()
        ref_alone = alone[i].cpu().numpy()
        tol = 1e-10 if PRECS[i] == 1 else 1e-6
        assert oracle.rel_linf(got, ref_alone) <= (1e-13 if PRECS[i] == 1 else 1e-6)
        assert oracle.rel_linf(got, oracle.evaluate(probs[i], kinds=KINDS[i])["total"]) <= tol
    s = srv.stats()
    assert s["completed"] == reps * len(plans) and s["failed"] == 0
    assert s["peak_in_flight"] >= 2        # requests actually overlapped
    assert s["groups"] < s["completed"]    # some requests ran together in one group
    assert s["device_allocs"] < s["completed"]  # workspace blocks were reused
    assert s["p99_s"] >= s["p50_s"] > 0
    srv.close()


def _size_class(b):
    """The server's workspace size class: b rounded up to a multiple of 1/8 of
    the largest power of two not above it (4 KiB at least)."""
    if b <= 4096:
        return 4096
    q = 1 << (b.bit_length() - 1 - 3)
    return -(-b // q) * q


def test_budget_admission_and_rejection():
    from paper_2409_11998_amd import Server
    from paper_2409_11998_amd.binding import VP_ERR_OOM
    torch, probs, devs, plans = _problems()
    ws = [_size_class(p.info()["workspace_bytes"]) for p in plans]
    top = sorted(ws)
    budget = (top[-2] + top[-1]) // 2   # the largest never fits, two of the next ones never together
    assert max(ws) > budget >= top[-2] and top[-2] + top[-3] > budget
    srv = Server(hbm_budget_bytes=budget, max_in_flight=8, n_streams=2)
    tickets = []
    for rep in range(3):
        for i in range(len(plans)):
            o = torch.zeros(probs[i].n_tgt, dtype=torch.float64, device="cuda")
            tickets.append((i, srv.submit(plans[i], o, **_args(devs[i], KINDS[i]))))
    for i, t in tickets:
        st, _ = srv.wait(t, timeout=120)
        assert st == (VP_ERR_OOM if ws[i] > budget else 0), (i, st, ws[i], budget)
    s = srv.stats()
    assert s["peak_bytes"] <= budget and s["peak_held_bytes"] <= budget
    assert s["completed"] == len(tickets)
    assert s["rejected"] == 3 * sum(1 for w in ws if w > budget)
    assert s["deferred"] >= 1              # requests waited for room
    srv.close()


def test_invalid_request_fails_alone():
    from paper_2409_11998_amd import Server
    torch, probs, devs, plans = _problems()
    srv = Server(hbm_budget_bytes=1 << 30, max_in_flight=4, n_streams=2)
    o_bad = torch.zeros(probs[0].n_tgt, dtype=torch.float64, device="cuda")
    # plan 1 supports S only: asking it for V is an argument error reported on the ticket
    t_bad = srv.submit(plans[1], o_bad, f=devs[1]["f"], jet6=devs[1]["jet6"])
    o_ok = torch.zeros(probs[0].n_tgt, dtype=torch.float64, device="cuda")
    t_ok = srv.submit(plans[0], o_ok, **_args(devs[0], KINDS[0]))
    assert srv.wait(t_bad)[0] != 0
    assert srv.wait(t_ok)[0] == 0
    srv.close()
