"""Move a Problem to device tensors and drive the library through its binding.

Marshalling only (no arithmetic of the method): used by the GPU tests, the
smoke check and the benchmark.
"""
import numpy as np


def to_device(problem, device="cuda"):
    import torch

    def t(a, dtype=torch.float64):
        if a is None:
            return None
        return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=device)

    g = problem.geom
    d = dict(
        src_x=t(problem.src_x) if problem.n_src else None,
        src_y=t(problem.src_y) if problem.n_src else None,
        src_w=t(problem.src_w) if problem.n_src else None,
        bnd_x=t(problem.bnd_x) if problem.n_bnd else None,
        bnd_y=t(problem.bnd_y) if problem.n_bnd else None,
        bnd_nx=t(problem.bnd_nx) if problem.n_bnd else None,
        bnd_ny=t(problem.bnd_ny) if problem.n_bnd else None,
        bnd_w=t(problem.bnd_w) if problem.n_bnd else None,
        tgt_x=t(problem.tgt_x), tgt_y=t(problem.tgt_y),
        geom=dict(r=t(g["r"]), nx=t(g["nx"]), ny=t(g["ny"]), kappa=t(g["kappa"]), gamma3=t(g["gamma3"]),
                  gamma4=t(g["gamma4"]), sgn=t(g["sgn"], torch.int8)),
        f=t(problem.f_src), jet6=t(problem.jet6), sigma=t(problem.sigma), sigma_jet=t(problem.sigma_jet),
        mu=t(problem.mu), mu_jet=t(problem.mu_jet))
    return d


def make_plan(dev, **opts):
    from paper_2409_11998_amd import Plan
    return Plan(dev["src_x"], dev["src_y"], dev["src_w"], dev["bnd_x"], dev["bnd_y"], dev["bnd_nx"],
                dev["bnd_ny"], dev["bnd_w"], dev["tgt_x"], dev["tgt_y"], dev["geom"], **opts)


def run(plan, dev, kinds="VSD", out=None):
    return plan.eval(f=dev["f"] if "V" in kinds else None, jet6=dev["jet6"] if "V" in kinds else None,
                     sigma=dev["sigma"] if "S" in kinds else None,
                     sigma_jet=dev["sigma_jet"] if "S" in kinds else None,
                     mu=dev["mu"] if "D" in kinds else None, mu_jet=dev["mu_jet"] if "D" in kinds else None,
                     out=out)


def make_batch_plans(devs, autotune_sample=0, **opts):
    """Plans for a batch: one spreading width per level for all instances.

    Without autotune_sample, the width is the largest the static planner picks
    for any instance.  With autotune_sample = k > 0, k instances spread over
    the size range are planned with the measured level selection (autotune)
    and the batch takes the widest of their chosen widths.  Every instance is
    then planned at that width, which fixes its fine grids (the smallest on
    which the width meets the tolerance)."""
    order = sorted(range(len(devs)), key=lambda i: devs[i]["tgt_x"].numel())
    if autotune_sample > 0:
        pick = sorted({order[int(round(j * (len(order) - 1) / max(1, autotune_sample - 1)))]
                       for j in range(autotune_sample)})
        w = [0, 0]
        for i in pick:
            p = make_plan(devs[i], autotune=True, **opts)
            w = [max(w[l], p.info()["width"][l]) for l in range(2)]
            p.close()
    else:
        w = [0, 0]
        for d in devs:
            p = make_plan(d, **opts)
            w = [max(w[l], p.info()["width"][l]) for l in range(2)]
            p.close()
    while True:
        out, widen = [], None
        for d in devs:
            try:
                out.append(make_plan(d, spread_width=tuple(w), **opts))
            except Exception:  # this instance needs a wider kernel: widen the batch and start over
                p = make_plan(d, **opts)
                widen = [max(w[l], p.info()["width"][l]) for l in range(2)]
                p.close()
                break
        if widen is None:
            return out
        for p in out:
            p.close()
        if widen == w:
            raise RuntimeError("no common spreading width for the batch")
        w = widen
