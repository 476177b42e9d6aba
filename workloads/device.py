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


def _class_choice(devs, members, sample, opts):
    """Widths and tile edge for the instances `members` (sorted by size).

    Widths: the widest the planner picks for `sample` of them spread over the
    size range, measured (autotune) when sample > 0, else the static choice
    for every member.  Tile: the edge the measured selection chose for every
    sampled level when it chose one edge throughout, else 0 (the planner's
    static rule per level)."""
    if sample > 0:
        pick = sorted({members[int(round(j * (len(members) - 1) / max(1, sample - 1)))] for j in range(sample)})
        tune = True
    else:
        pick, tune = members, False
    w, tiles = [0, 0], set()
    for i in pick:
        p = make_plan(devs[i], autotune=tune, **opts)
        inf = p.info()
        w = [max(w[l], inf["width"][l]) for l in range(2)]
        tiles.update(inf["tile"])
        p.close()
    return w, (tiles.pop() if tune and len(tiles) == 1 else 0)


def make_batch_plans(devs, autotune_sample=0, classes=1, **opts):
    """Plans for a batch, one spreading width per level within each width class.

    The instances, sorted by target count, are cut into `classes` classes of
    about equal count.  A class's width per level is the largest the planner
    picks for its members: with autotune_sample = k > 0, for k of them spread
    over the class's size range with the measured level selection (autotune),
    else the static choice for every member; with autotune the class also
    takes the tile edge the measurements agreed on.  Every member is then
    planned at its class's width (and tile), which fixes its fine grids (the
    smallest on which the width meets the tolerance); a member that needs a
    wider kernel widens its class, which is planned again.  Returns the plans
    in the order of devs."""
    order = sorted(range(len(devs)), key=lambda i: devs[i]["tgt_x"].numel())
    classes = max(1, min(classes, len(order)))
    cut = [round(c * len(order) / classes) for c in range(classes + 1)]
    out = [None] * len(devs)
    for c in range(classes):
        members = order[cut[c]:cut[c + 1]]
        w, tile = _class_choice(devs, members, autotune_sample, opts)
        copts = dict(opts, tile=tile) if tile and "tile" not in opts else opts
        while True:
            made, widen = [], None
            for i in members:
                try:
                    made.append(make_plan(devs[i], spread_width=tuple(w), **copts))
                except Exception:  # this member needs a wider kernel: widen the class and start over
                    p = make_plan(devs[i], **copts)
                    widen = [max(w[l], p.info()["width"][l]) for l in range(2)]
                    p.close()
                    break
            if widen is None:
                break
            for p in made:
                p.close()
            if widen == w:
                raise RuntimeError("no common spreading width for a batch class")
            w = widen
        for i, p in zip(members, made):
            out[i] = p
    return out
