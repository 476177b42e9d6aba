"""Benchmark: target points/s for V[f] + D[mu] through the C ABI on one MI355X.

Workload (timed step = one vp_eval of V[f] + D[mu], all stages of the path):
  square [-1,1]^2, 200k triangles with 10% sliver splits, degenerate
  triangles and 0.2% gaps (~1.2M volume nodes = targets), f = 5 Gaussians,
  D[mu] from 20k Gauss-Legendre boundary nodes with mu = cos(3 theta),
  float64 at tolerance 1e-10.
Both precisions run on both large workloads: float32 at 1e-6 on the same
square workload (its error against the float64 result at every target and
against the oracle sample), and the unit disk with ~2M triangles (~12M nodes,
V[f]) in float64 at 1e-10 and float32 at 1e-6 (errors against the float64
result at every target and against 10^4 stored oracle values, half of them
near the circle).  The roofline fractions use the step table's algorithmic
bytes (coordinates, strengths and grids; record layouts not counted).

Prints one JSON line.  Inputs are resident in HBM before the timed region;
the timed region is bracketed by torch.cuda.synchronize().  In the timed
steps the far-history level's spread and interpolation run on a second stream
beside the near-history level's.  Per-stage times come from HIP events
recorded on the plan's stream (vp_set_timing) in a separate pass of the same
number of steps, in which every launch runs alone, in order, on that stream.  The CPU baseline is the float64
oracle (direct sums + local asymptotics) on a bounded sample of targets on
this host's cores.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "target pts/s for V[f]+D[mu] at 1e-6 FP32 vs 1e-10 FP64; p50/p99 request latency"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6   # MI355X dense float64 (vector and matrix)
STAGES = ["strengths", "spread", "row_fft", "col_fft_mul", "row_ifft", "interp", "local"]
LAUNCHES = ["strengths", "spread_nh", "spread_fh", "row_fft_nh", "row_fft_fh", "col_fft_mul_nh", "col_fft_mul_fh",
            "row_ifft_nh", "row_ifft_fh", "interp_nh", "interp_fh", "local"]
KERNELS = {"strengths": "k_strengths", "spread": "k_spread", "row_fft": "k_row_r2c", "col_fft_mul": "k_col",
           "row_ifft": "k_row_c2r", "interp": "k_interp", "local": "k_local"}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def algorithmic_bytes(info, P, kinds, b):
    """Bytes each timed launch must move at minimum: one read of each input and one write of
    each output (b = bytes of the plan's real type).  A spread node record is its packed
    support corner and node index (4 B each), two offsets and the strength it gathers (two
    more for double-layer boundary nodes); a target record likewise, plus its history value.
    The spread writes its level's grid once; the first slot also zeroes both grids."""
    n_v = P.n_src if "V" in kinds else 0
    n_b = P.n_bnd if ("S" in kinds or "D" in kinds) else 0
    dl = "D" in kinds
    out = {}
    grids = sum(F * F * b for F in info["fine"])
    out["strengths"] = grids + n_v * (16 + b) + n_b * (16 + b + (16 + 2 * b if dl else 0))
    nt = P.n_tgt
    for l, tag in enumerate(("nh", "fh")):
        F = info["fine"][l]
        M = (info["modes"][l] - 1) // 2
        half = (M + 1) * F * 2 * b
        rec = 8 + 2 * b
        out["spread_" + tag] = n_v * (rec + b) + n_b * (rec + b + (2 * b if dl else 0)) + F * F * b
        out["row_fft_" + tag] = F * F * b + half
        out["col_fft_mul_" + tag] = 2 * half + (M + 1) ** 2 * b
        out["row_ifft_" + tag] = half + F * F * b
        out["interp_" + tag] = F * F * b + nt * (8 + 2 * b) + nt * b
    # local part: every target reads r, both history values and writes its result; targets
    # within 12 sqrt(delta_1) of the boundary also read their frame and layer jets
    near = int(np.count_nonzero(np.asarray(P.geom["r"]) <= 12.0 * np.sqrt(info["delta1"])))
    loc = nt * (8 + 2 * b + 8)
    if "V" in kinds:
        loc += nt * 3 * 8 + near * (3 * 8)
    loc += near * (3 * 8 + 1 + 16)  # nx, ny, kappa, sgn, gamma3, gamma4
    if "D" in kinds:
        loc += near * 5 * 8
    if "S" in kinds:
        loc += near * 3 * 8
    out["local"] = loc
    for st in ("spread", "row_fft", "col_fft_mul", "row_ifft", "interp"):
        out[st] = out[st + "_nh"] + out[st + "_fh"]
    return out


def step_bytes(info, P, kinds, b):
    """Algorithmic bytes of each hot-path step (one read of each input, one
    write of each output),
    for the one grid channel this design spreads: a volume node brings its two
    coordinates and one strength, a double-layer boundary node its coordinates
    and three strengths (sigma w, and mu nu w for the kernel derivative), a
    single-layer-only node one strength.
      spread     (coordinates + strengths) of every node + F^2 b (the grid, written once)
      FFT chain  R2C 2 F^2 b + multiply 2 F^2 b (grid and table) + C2R 2 F^2 b = 6 F^2 b
                 (the row pass, the column pass with the multiply, the inverse row pass)
      interp     F^2 b + 3 b per target (two coordinates in, the value out)
    Record layouts, indices and tile bookkeeping of the implementation are not counted."""
    n_v = P.n_src if "V" in kinds else 0
    n_b = P.n_bnd if ("S" in kinds or "D" in kinds) else 0
    per_b = 2 * b + (3 * b if "D" in kinds else b)
    out = {}
    for l, tag in enumerate(("nh", "fh")):
        F2b = info["fine"][l] ** 2 * b
        out["spread_" + tag] = n_v * 3 * b + n_b * per_b + F2b
        out["fft_chain_" + tag] = 6 * F2b
        out["interp_" + tag] = F2b + P.n_tgt * 3 * b
    return out


def step_roofline(st, sb):
    """(key, ms, bytes, GB/s, fraction of HBM peak) per step of step_bytes; FFT chains take the
    sum of their three launches' times."""
    rows = {}
    for tag in ("nh", "fh"):
        t = {"spread_" + tag: st["spread_" + tag], "interp_" + tag: st["interp_" + tag],
             "fft_chain_" + tag: st["row_fft_" + tag] + st["col_fft_mul_" + tag] + st["row_ifft_" + tag]}
        for k, ms in t.items():
            gbs = sb[k] / (ms * 1e-3) / 1e9
            rows[k] = {"ms": round(ms, 4), "bytes": int(sb[k]), "gbs": round(gbs, 1),
                       "frac": round(gbs / HBM_PEAK_GBS, 4)}
    return rows


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("vp_device.hpp", "vp_kernels.hip", "vp_internal.hpp"):
        with open(os.path.join(ROOT, "paper_2409_11998_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profiles(kernel, workload):
    """HBM bytes per launch from committed counter summaries, if taken on the current kernels."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as fh:
            d = json.load(fh)
        e = d.get(workload, {}).get(kernel)
        if e and e.get("source_hash") == kernel_source_hash():
            return e["hbm_bytes_per_launch"]
    except Exception:
        return None
    return None


def time_steps(torch, fn, steps):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def stage_times(torch, plan, fn, steps):
    plan.set_timing(True)
    acc = {}
    for _ in range(steps):
        fn()
        t = plan.timing()
        for k, v in t.items():
            acc[k] = acc.get(k, 0.0) + v
    plan.set_timing(False)
    torch.cuda.synchronize()
    return {k: v / steps for k, v in acc.items()}


def run_leg(torch, P, kinds, tol, precision, steps, warmup, oracle_sample, seed, autotune=True, sample=None,
            reference=None, tile=0):
    """Plan (autotuned), warm up, time `steps` evaluations, then a timing pass for the stage
    times.  oracle_sample > 0: the oracle at that many seeded targets (its time is the CPU
    baseline).  sample = (idx, values): e_inf on those targets; reference: e_inf on all."""
    from workloads.device import make_plan, run, to_device
    dev = to_device(P)
    mask = (1 if "V" in kinds else 0) | (2 if "S" in kinds else 0) | (4 if "D" in kinds else 0)
    t0 = time.perf_counter()
    plan = make_plan(dev, tol=tol, precision=precision, kinds=mask, autotune=autotune,
                     **({"tile": tile} if tile else {}))
    torch.cuda.synchronize()
    plan_s = time.perf_counter() - t0
    info = plan.info()
    out = torch.empty(P.n_tgt, dtype=torch.float64, device="cuda")
    fn = lambda: run(plan, dev, kinds, out=out)
    for _ in range(warmup):
        fn()
    el = time_steps(torch, fn, steps)
    st = stage_times(torch, plan, fn, steps)
    res = dict(info=info, plan_s=plan_s, elapsed=el, stages=st)
    fn()
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    res["got"] = got
    plan.close()
    del dev, out
    if oracle_sample:
        import oracle
        from oracle import direct
        rng = np.random.default_rng(seed)
        idx = np.sort(rng.choice(P.n_tgt, size=min(oracle_sample, P.n_tgt), replace=False))
        sub = P.subset_targets(idx)
        t1 = time.perf_counter()
        ref = oracle.evaluate(sub, kinds=kinds)["total"]
        res["oracle_s"] = time.perf_counter() - t1
        res["oracle_n"] = len(idx)
        res["oracle_threads"] = direct.num_threads()
        res["oracle_sample"] = (idx, ref)
        sample = (idx, ref)
    if sample is not None:
        idx, ref = sample
        res["e_inf_sample"] = float(np.max(np.abs(got[idx] - ref)) / np.max(np.abs(ref)))
    if reference is not None:
        res["e_inf_all"] = float(np.max(np.abs(got - reference)) / np.max(np.abs(reference)))
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=30)
    ap.add_argument("--oracle-sample", type=int, default=16384,
                    help="targets of the main workload the CPU oracle evaluates (its timing is the "
                         "cpu_baseline, about 10 s on 16 cores; its values check the GPU result)")
    ap.add_argument("--no-fp32-leg", action="store_true")
    ap.add_argument("--no-disk-legs", action="store_true",
                    help="skip the 12M-node disk legs (FP64 and FP32) but keep FP32 on the square workload")
    ap.add_argument("--scale", type=float, default=1.0, help="shrink the workloads (quick runs)")
    ap.add_argument("--no-batch-leg", action="store_true")
    ap.add_argument("--no-refine-leg", action="store_true")
    ap.add_argument("--no-geometry-leg", action="store_true")
    ap.add_argument("--no-solve-leg", action="store_true")
    ap.add_argument("--solve-panels", type=int, default=256, help="panels of 16 nodes in the Dirichlet-solve leg")
    ap.add_argument("--solve-triangles", type=int, default=60000, help="triangles of the Dirichlet-solve leg's mesh")
    ap.add_argument("--refine-levels", type=int, default=3)
    ap.add_argument("--no-neumann-leg", action="store_true")
    ap.add_argument("--neumann-sizes", type=str, default="674664,1198728,2695248",
                    help="volume node counts of the paper-size interior Neumann leg")
    ap.add_argument("--no-serve-leg", action="store_true")
    ap.add_argument("--batch-instances", type=int, default=256)
    ap.add_argument("--batch-max-tri", type=float, default=2e5)
    ap.add_argument("--batch-tune-sample", type=int, default=3,
                    help="instances per width class timed by the autotuner to choose its spreading widths")
    ap.add_argument("--batch-classes", type=int, default=4,
                    help="width classes of the batch (instances cut by size, one width pair per class)")
    ap.add_argument("--serve-meshes", type=int, default=16)
    ap.add_argument("--serve-requests", type=int, default=2000, help="requests per arrival rate")
    ap.add_argument("--serve-loads", type=str, default="0.2,0.5,0.8,0.95",
                    help="arrival rates as fractions of the saturated rate")
    ap.add_argument("--tile", type=int, default=0,
                    help="headline leg: restrict the autotuner to this spreading tile edge (profiling runs, "
                         "so that every pass launches the kernels an unprofiled run picks)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="first run one device-to-device copy of this size (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(instances and requests would be placed one GPU each); got --gpus %d" % args.gpus, file=sys.stderr)
        sys.exit(2)
    # inputs of the batch and serving legs are generated in a process pool before any GPU use
    rng = np.random.default_rng(4)
    batch_specs, serve_specs = [], []
    if not args.no_batch_leg:
        tri = np.exp(rng.uniform(np.log(1e3), np.log(args.batch_max_tri), args.batch_instances)) * args.scale
        batch_specs = [(max(200, int(t)), 4000 + i, "VD") for i, t in enumerate(tri)]
    if not args.no_serve_leg:
        rs = np.random.default_rng(5)
        nodes = np.exp(rs.uniform(np.log(2e3), np.log(5e5), args.serve_meshes)) * args.scale
        serve_specs = [(max(200, int(n / 6)), 5000 + i, "VSD") for i, n in enumerate(nodes)]
    pool_probs = []
    if batch_specs or serve_specs:
        from workloads.pool import stars
        log("bench: generating %d batch and %d serving meshes" % (len(batch_specs), len(serve_specs)))
        pool_probs = stars(batch_specs + serve_specs)
    batch_probs = pool_probs[:len(batch_specs)]
    serve_probs = pool_probs[len(batch_specs):]
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a HIP device", file=sys.stderr)
        sys.exit(1)
    import paper_2409_11998_amd
    paper_2409_11998_amd.lib()
    if args.calib_copy_mib:
        n = args.calib_copy_mib * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b_ = torch.empty_like(a)
        torch.cuda.synchronize()
        b_.copy_(a)
        torch.cuda.synchronize()
        del a, b_
    from workloads import config_problem

    log("bench: generating square-200k workload")
    P = config_problem(2, scale=args.scale)
    log("bench: fp64 V+D leg, n_tgt=%d n_bnd=%d" % (P.n_tgt, P.n_bnd))
    r64 = run_leg(torch, P, "VD", 1e-10, 1, args.steps, args.warmup, args.oracle_sample, seed=20, tile=args.tile)
    value = P.n_tgt * args.steps / r64["elapsed"]
    ms = 1000.0 * r64["elapsed"] / args.steps
    alg = algorithmic_bytes(r64["info"], P, "VD", 8)
    st = r64["stages"]
    sroof = step_roofline(st, step_bytes(r64["info"], P, "VD", 8))
    dom = max(("spread_nh", "spread_fh", "interp_nh", "interp_fh"), key=lambda k: st[k])
    workload = "square-200k-slivers-gaps V+D fp64 tol1e-10"
    lvl = {"nh": 0, "fh": 1}[dom.rsplit("_", 1)[-1]]
    step = dom.rsplit("_", 1)[0]
    mma = step == "spread" and r64["info"]["spread_mma"][lvl]
    kname = ("k_spread_mma<double, %d>" % r64["info"]["width"][lvl] if mma else KERNELS[step]) + \
        " (%s level, w=%d, F=%d)" % (("near-history", "far-history")[lvl], r64["info"]["width"][lvl],
                                     r64["info"]["fine"][lvl])
    roof = {"bound": "hbm", "kernel": kname, "launch": dom, "achieved": sroof[dom]["gbs"], "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": sroof[dom]["frac"],
            "traffic": traffic_from_profiles(dom, workload),
            "algorithmic_bytes_per_launch": sroof[dom]["bytes"],
            "record_bytes_per_launch": int(alg[dom]),
            "avg_ms": round(st[dom], 4),
            "avg_ms_from": "HIP events, timing pass (each launch alone on the plan's stream)",
            "steps_frac_of_hbm": {k: v["frac"] for k, v in sroof.items()}}
    if mma:
        # the spread as rank-1 updates: useful FMAs w^2 per term (a volume node is one term,
        # a double-layer boundary node two); the matrix instructions cover the 32 x 32 window,
        # 1024 FMAs per term
        w_ = r64["info"]["width"][lvl]
        terms = P.n_src + 2 * P.n_bnd
        t_s = st[dom] * 1e-3
        roof["flops"] = {"useful_tflops": round(2.0 * terms * w_ * w_ / t_s / 1e12, 2),
                         "matrix_tflops": round(2.0 * terms * 1024 / t_s / 1e12, 2),
                         "peak_tflops": FP64_PEAK_TFLOPS}
    stages_gbs = {k: round(alg[k] / (st[k] * 1e-3) / 1e9, 1) for k in LAUNCHES if st.get(k, 0) > 0}
    cpu = None
    if args.oracle_sample:
        cpu = {"value": round(r64["oracle_n"] / r64["oracle_s"], 2), "unit": "target pts/s",
               "cores": r64["oracle_threads"], "kind": "oracle",
               "sample": "%d seeded targets of the same workload against all %d sources and %d boundary nodes"
                         % (r64["oracle_n"], P.n_src, P.n_bnd)}
    rec = {"metric": METRIC, "value": round(value, 1), "unit": "target pts/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": workload, "n_src": P.n_src, "n_bnd": P.n_bnd, "n_tgt": P.n_tgt,
                      "fine_grid": list(r64["info"]["fine"]), "modes": list(r64["info"]["modes"]),
                      "spread_width": list(r64["info"]["width"]), "tile": list(r64["info"]["tile"]), "interp_tile": list(r64["info"]["interp_tile"]),
                      "spread_mma": list(r64["info"]["spread_mma"]),
                      "autotuned": r64["info"]["autotuned"], "tol": 1e-10},
           "roofline": roof, "cpu_baseline": cpu,
           "stages_ms": {k: round(v, 4) for k, v in st.items()}, "stages_gbs_record_bytes": stages_gbs,
           "plan_s": round(r64["plan_s"], 3), "e_inf_vs_oracle_sample": r64.get("e_inf_sample")}
    if not args.no_fp32_leg:
        log("bench: fp32 V+D leg on the same workload")
        r = run_leg(torch, P, "VD", 1e-6, 0, args.steps, args.warmup, 0, seed=21,
                    sample=r64.get("oracle_sample"), reference=r64["got"])
        rec["fp32_same_workload"] = leg_summary(r, P, "VD", 4, args.steps, "square-200k-slivers-gaps V+D fp32 tol1e-6")
        rec["fp32_same_workload"]["e_inf_vs_fp64_all_targets"] = r.get("e_inf_all")
        rec["fp32_same_workload"]["e_inf_vs_oracle_sample"] = r.get("e_inf_sample")
    r64.pop("got")
    if not args.no_refine_leg:
        log("bench: dyadic refinement leg, %d levels" % args.refine_levels)
        rec["refine"] = refine_leg(torch, P, args.refine_levels, args.steps)
    if not args.no_geometry_leg:
        log("bench: geometry leg")
        rec["geometry"] = geometry_leg(torch, P, args.steps)
    if not args.no_solve_leg:
        log("bench: Dirichlet solve leg, %d panels" % args.solve_panels)
        rec["solve"] = solve_leg(torch, args.solve_panels, int(args.solve_triangles * args.scale),
                                 max(1, min(args.steps, 10)))
    if not args.no_neumann_leg:
        log("bench: interior Neumann leg at the paper's sizes")
        rec["neumann_paper"] = neumann_paper_leg(torch, [int(float(v) * args.scale) for v in
                                                         args.neumann_sizes.split(",")])
    if not args.no_fp32_leg and not args.no_disk_legs:
        log("bench: generating disk-2M workload")
        Q = config_problem(3, scale=args.scale)
        sample = disk2m_oracle_sample(Q)
        log("bench: fp64 V leg on disk-2M, n_tgt=%d" % Q.n_tgt)
        q64 = run_leg(torch, Q, "V", 1e-10, 1, args.steps, args.warmup, 0, seed=31, sample=sample)
        rec["fp64_disk2m"] = leg_summary(q64, Q, "V", 8, args.steps, "disk-2M V fp64 tol1e-10")
        rec["fp64_disk2m"]["e_inf_vs_oracle_sample"] = q64.get("e_inf_sample")
        log("bench: fp32 V leg, n_tgt=%d" % Q.n_tgt)
        r32 = run_leg(torch, Q, "V", 1e-6, 0, args.steps, args.warmup, 0, seed=30, sample=sample,
                      reference=q64["got"])
        q64.pop("got")
        rec["fp32"] = leg_summary(r32, Q, "V", 4, args.steps, "disk-2M V fp32 tol1e-6")
        rec["fp32"]["e_inf_vs_fp64_all_targets"] = r32.get("e_inf_all")
        rec["fp32"]["fp64_reference_tol"] = 1e-10
        rec["fp32"]["e_inf_vs_oracle_sample"] = r32.get("e_inf_sample")
        rec["fp32"]["oracle_sample"] = None if sample is None else "%d stored oracle values (%d within 12 sqrt(delta_1) of the circle)" % (
            sample[0].size, int(np.count_nonzero(Q.geom["r"][sample[0]] <= 12 * np.sqrt(r32["info"]["delta1"]))))
        r32.pop("got")
    if batch_probs:
        log("bench: batch leg, %d instances, %d targets" % (len(batch_probs), sum(P.n_tgt for P in batch_probs)))
        rec["batch"] = batch_leg(torch, batch_probs, args.steps, args.warmup, args.batch_tune_sample,
                                 args.batch_classes)
    if serve_probs:
        log("bench: serving leg, %d meshes" % len(serve_probs))
        loads = [float(x) for x in args.serve_loads.split(",")]
        rec["serve"] = serve_leg(torch, serve_probs, args.serve_requests, loads)
        ref_load = min(rec["serve"]["loads"], key=lambda k: abs(float(k) - 0.8))
        rec["latency_p50_s"] = rec["serve"]["loads"][ref_load]["served"]["p50_s"]
        rec["latency_p99_s"] = rec["serve"]["loads"][ref_load]["served"]["p99_s"]
        rec["latency_load"] = float(ref_load)
    print(json.dumps(rec), flush=True)


def leg_summary(r, P, kinds, b, steps, workload):
    st = r["stages"]
    sroof = step_roofline(st, step_bytes(r["info"], P, kinds, b))
    dom = max(sroof, key=lambda k: sroof[k]["ms"])
    return {"workload": workload, "n_tgt": P.n_tgt, "value": round(P.n_tgt * steps / r["elapsed"], 1),
            "unit": "target pts/s", "ms_per_step": round(1000.0 * r["elapsed"] / steps, 4),
            "fine_grid": list(r["info"]["fine"]), "spread_width": list(r["info"]["width"]),
            "tile": list(r["info"]["tile"]), "interp_tile": list(r["info"]["interp_tile"]),
            "spread_mma": list(r["info"]["spread_mma"]), "stages_ms": {k: round(v, 4) for k, v in st.items()},
            "steps_frac_of_hbm": {k: v["frac"] for k, v in sroof.items()}, "dominant_step": dom,
            "dominant_frac_of_hbm_peak": sroof[dom]["frac"], "plan_s": round(r["plan_s"], 3)}


def disk2m_oracle_sample(Q):
    """(idx, V) of the oracle at 10^4 stratified disk-2M targets, stored by
    tests/golden/make_disk2m_oracle_sample.py, if they are this workload's targets."""
    path = os.path.join(ROOT, "tests", "golden", "disk2m_v_oracle_sample.npz")
    if not os.path.exists(path):
        return None
    d = np.load(path)
    idx = d["idx"]
    if Q.n_tgt != int(d["n_tgt"]) or not (np.array_equal(Q.tgt_x[idx], d["x"]) and np.array_equal(Q.tgt_y[idx], d["y"])):
        return None
    return idx, d["v"]


def geometry_leg(torch, P, steps):
    """Local frame and double-layer jets of every target from the boundary panels
    alone (vp_boundary_frame, vp_boundary_jets) on the square workload; the
    distance and side against the exact square."""
    from paper_2409_11998_amd import boundary_frame, boundary_jets, volume_jets, volume_jets_patch
    from workloads.mesh import triangle_neighbours
    q = P.info["q"]
    f64 = torch.float64
    bx, by = (torch.as_tensor(a, dtype=f64, device="cuda") for a in (P.bnd_x, P.bnd_y))
    tx, ty = (torch.as_tensor(a, dtype=f64, device="cuda") for a in (P.tgt_x, P.tgt_y))
    mu = torch.as_tensor(P.mu, dtype=f64, device="cuda")
    fr = {}
    frame = lambda: fr.update(boundary_frame(bx, by, q, tx, ty))
    jets = lambda: boundary_jets(bx, by, q, mu, fr["pan"], fr["u"], 4)
    for _ in range(3):
        frame()
        jets()
    el_f = time_steps(torch, frame, steps)
    el_j = time_steps(torch, jets, steps)
    # f's jets at the volume nodes from the triangles' quadratic interpolants
    sx, sy, sf = (torch.as_tensor(a, dtype=f64, device="cuda") for a in (P.src_x, P.src_y, P.f_src))
    vj = lambda: volume_jets(sx, sy, sf)
    for _ in range(3):
        vj()
    el_v = time_steps(torch, vj, steps)
    J = vj().cpu().numpy()
    fin = np.all(np.isfinite(J), axis=0)
    n_tri = P.n_src // 6
    # triangles whose node spread has an axis ratio of at least 0.1 (not slivers)
    X, Y = (np.asarray(a).reshape(-1, 6) for a in (P.src_x, P.src_y))
    dxm, dym = X - X.mean(1, keepdims=True), Y - Y.mean(1, keepdims=True)
    sxx, sxy, syy = (dxm * dxm).sum(1), (dxm * dym).sum(1), (dym * dym).sum(1)
    rad = np.hypot(0.5 * (sxx - syy), sxy)
    ratio = np.sqrt(np.maximum(0.5 * (sxx + syy) - rad, 0) / np.maximum(0.5 * (sxx + syy) + rad, 1e-300))
    shaped = np.repeat(ratio >= 0.1, 6) & fin

    def rel(rows, sel=fin, J=J):
        ref = np.asarray(P.jet6)[rows]
        return float(np.max(np.abs(J[rows][:, sel] - ref[:, sel])) / np.max(np.abs(ref)))
    # the same jets from the least-squares quadratic over each triangle and its edge neighbours
    nbr = torch.as_tensor(triangle_neighbours(P.info["tri"]), dtype=torch.int32, device="cuda")
    vp_ = lambda: volume_jets_patch(sx, sy, sf, nbr)
    for _ in range(3):
        vp_()
    el_p = time_steps(torch, vp_, steps)
    Jp = vp_().cpu().numpy()
    finp = np.all(np.isfinite(Jp), axis=0)
    slivers = np.repeat(ratio < 0.1, 6) & finp
    # V[f] at the volume nodes (targets = nodes) with the device's patch jets against V[f]
    # with the Gaussians' analytic jets: what nodal f alone gives the headline workload
    from workloads.device import make_plan, to_device
    dev = to_device(P)
    plan = make_plan(dev, tol=1e-10, precision=1, kinds=1)
    v_exact = plan.eval(f=dev["f"], jet6=dev["jet6"]).cpu().numpy()
    v_patch = plan.eval(f=dev["f"], jet6=torch.as_tensor(Jp, device="cuda")).cpu().numpy()
    plan.close()
    del dev
    v_diff = float(np.max(np.abs(v_patch - v_exact)) / np.max(np.abs(v_exact)))
    r = fr["r"].cpu().numpy()
    sgn = fr["sgn"].cpu().numpy()
    return {"workload": "square-200k targets (%d) against %d boundary nodes in %d panels of %d" %
                        (P.n_tgt, P.n_bnd, P.n_bnd // q, q),
            "frame_ms": round(1e3 * el_f / steps, 4), "jets4_ms": round(1e3 * el_j / steps, 4),
            "targets_per_s": round(P.n_tgt * steps / el_f, 1),
            "max_abs_r_vs_exact": float(np.max(np.abs(r - np.asarray(P.geom["r"])))),
            # the workload labels targets on the curve (mesh nodes on the square's edges)
            # with their interior limit +1; the frame reports them as on the curve, 0
            "sgn_differs_from_exact": int(np.count_nonzero(sgn != np.asarray(P.geom["sgn"]))),
            "volume_jets_ms": round(1e3 * el_v / steps, 4), "volume_jets_triangles": n_tri,
            "volume_jets_gbs": round(432.0 * n_tri * steps / el_v / 1e9, 1),
            "volume_jets_nan_triangles": int(np.count_nonzero(~fin.reshape(-1, 6).all(1))),
            "volume_jets_rel_err_vs_analytic": {"gradient": rel([1, 2]), "hessian": rel([3, 4, 5])},
            "volume_jets_rel_err_vs_analytic_axis_ratio_ge_0.1": {"gradient": rel([1, 2], shaped),
                                                                  "hessian": rel([3, 4, 5], shaped),
                                                                  "triangles": int(shaped.sum() // 6)},
            "volume_jets_patch_ms": round(1e3 * el_p / steps, 4),
            "volume_jets_patch_nan_triangles": int(np.count_nonzero(~finp.reshape(-1, 6).all(1))),
            "volume_jets_patch_rel_err_vs_analytic": {"gradient": rel([1, 2], finp, Jp),
                                                      "hessian": rel([3, 4, 5], finp, Jp)},
            "volume_jets_patch_rel_err_vs_analytic_axis_ratio_lt_0.1": {"gradient": rel([1, 2], slivers, Jp),
                                                                       "hessian": rel([3, 4, 5], slivers, Jp),
                                                                       "triangles": int(slivers.sum() // 6)},
            "v_with_patch_jets_rel_diff_vs_analytic_jets": v_diff,
            "sgn_differs_only_on_curve": bool(np.all(np.asarray(P.geom["r"])[sgn != np.asarray(P.geom["sgn"])] <= 1e-12)
                                              and np.all(sgn[sgn != np.asarray(P.geom["sgn"])] == 0))}


def solve_leg(torch, n_pan, n_tri, steps, q=16):
    """Interior Dirichlet problem -Lap u = f inside a three-lobed star
    (vp_dirichlet_solve): f a Gaussian at the volume nodes of a curved
    triangulation, the right-hand side g - V[f] and GMRES whose product is the
    double layer at the boundary nodes, from a zero start in each timed solve;
    then u = V[f] + D[mu] at interior points against the exact solution
    w(|x|) + Re((z - z0)^3), w the radial solution of the Gaussian source.
    The interior Neumann problem with the same source and solution follows
    (vp_neumann_solve; u = V[f] + S[g] - D[u_b], exact up to a constant)."""
    from scipy.special import exp1
    from paper_2409_11998_amd import Plan, boundary_frame, boundary_jets, dirichlet_solve, neumann_solve
    from workloads.mesh import curve_mesh
    from workloads.problems import StarCurve, gauss_jets, panel_nodes, star_params
    f64 = torch.float64
    curve = StarCurve(**star_params(3, r=0.8))
    x, y, w, _ = curve_mesh(curve, n_tri, 3)
    bx, by, bnx, bny, bw, _ = panel_nodes(curve, n_pan, q)
    s2, z0 = 0.1, complex(0.1, -0.05)
    gauss = ((1.0, 0.0, 0.0, np.sqrt(s2)),)

    def uex(px, py):
        r = np.hypot(px, py)
        return 0.25 * s2 * (2 * np.log(1 / r) - exp1(r * r / s2) + exp1(1 / s2)) + ((px + 1j * py - z0) ** 3).real

    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=f64, device="cuda")
    sx, sy, sw, fs = t(x), t(y), t(w), t(gauss_jets(x, y, gauss)[0])
    dx, dy, dnx, dny, dw = (t(a) for a in (bx, by, bnx, bny, bw))
    t0 = time.perf_counter()
    fr = boundary_frame(dx, dy, q, dx, dy)
    geom = dict(r=torch.zeros_like(dx), nx=fr["nx"], ny=fr["ny"], kappa=fr["kappa"], gamma3=fr["gamma3"],
                gamma4=fr["gamma4"], sgn=torch.ones(dx.numel(), dtype=torch.int8, device="cuda"))
    plan = Plan(sx, sy, sw, dx, dy, dnx, dny, dw, dx, dy, geom, tol=1e-10, precision=1, kinds=7)
    torch.cuda.synchronize()
    plan_s = time.perf_counter() - t0
    g, jb = t(uex(bx, by)), t(gauss_jets(bx, by, gauss))
    mu = torch.zeros_like(dx)
    stat = {}

    def solve():
        mu.zero_()
        _, stat["its"], stat["res"] = dirichlet_solve(plan, q, dx, dy, fr["pan"], fr["u"], g, mu=mu, f=fs, jet6=jb)

    solve()
    el = time_steps(torch, solve, steps)
    # Neumann data: the normal derivative of the same solution
    z = bx + 1j * by
    rb = np.abs(z)
    wd = -(s2 / (2 * rb)) * (1 - np.exp(-rb * rb / s2))
    gn = t((wd * bx / rb + (3 * (z - z0) ** 2).real) * bnx + (wd * by / rb - (3 * (z - z0) ** 2).imag) * bny)
    ub = torch.zeros_like(dx)

    def solve_n():
        ub.zero_()
        _, stat["its_n"], stat["res_n"] = neumann_solve(plan, q, dx, dy, dw, fr["pan"], fr["u"], gn, ub=ub, f=fs,
                                                        jet6=jb)

    solve_n()
    el_n = time_steps(torch, solve_n, steps)
    info = plan.info()
    plan.close()
    # interior values: seeded points pulled toward the centroid from the nodes
    rng = np.random.default_rng(42)
    k = rng.integers(0, bx.size, 4096)
    s_ = rng.uniform(0.2, 0.95, 4096)
    cx, cy = np.mean(bx), np.mean(by)
    tx, ty = cx + s_ * (bx[k] - cx), cy + s_ * (by[k] - cy)
    ftx, fty = t(tx), t(ty)
    fi = boundary_frame(dx, dy, q, ftx, fty)
    gi = {kk: fi[kk] for kk in ("r", "nx", "ny", "kappa", "gamma3", "gamma4", "sgn")}
    pi = Plan(sx, sy, sw, dx, dy, dnx, dny, dw, ftx, fty, gi, tol=1e-10, precision=1, kinds=7)
    jt = t(gauss_jets(tx, ty, gauss))
    u = pi.eval(f=fs, jet6=jt, mu=mu, mu_jet=boundary_jets(dx, dy, q, mu, fi["pan"], fi["u"], 4)).cpu().numpy()
    mub = -ub
    un = pi.eval(f=fs, jet6=jt, sigma=gn, sigma_jet=boundary_jets(dx, dy, q, gn, fi["pan"], fi["u"], 2).contiguous(),
                 mu=mub, mu_jet=boundary_jets(dx, dy, q, mub, fi["pan"], fi["u"], 4)).cpu().numpy()
    pi.close()
    cmean = float(np.dot(bw, uex(bx, by)) / np.sum(bw))
    return {"workload": "three-lobed star, Gaussian source at %d volume nodes (%d curved triangles), %d panels of "
                        "%d Gauss-Legendre nodes, fp64 tol1e-10" % (x.size, n_tri, n_pan, q),
            "n_src": int(x.size), "n_nodes": int(bx.size), "delta1": info["delta1"], "fine_grid": list(info["fine"]),
            "gmres_products": stat["its"], "rel_residual": stat["res"], "solve_ms": round(1e3 * el / steps, 3),
            "solves_timed": steps, "plan_s": round(plan_s, 3), "interior_points": int(tx.size),
            "max_abs_err_interior_vs_exact": float(np.max(np.abs(u - uex(tx, ty)))),
            "neumann": {"gmres_products": stat["its_n"], "rel_residual": stat["res_n"],
                        "solve_ms": round(1e3 * el_n / steps, 3),
                        "max_abs_err_interior_vs_exact_up_to_boundary_mean":
                            float(np.max(np.abs(un - uex(tx, ty) + cmean)))}}


def neumann_paper_leg(torch, sizes, q=16, levels=3, reps=3):
    """The interior Neumann experiment of the paper's numerical section at its
    sizes: the curve with r = 1, alpha_0 = 5/6, beta_3 = 1/30, alpha_5 = 1/15,
    alpha_{6,8,10} = 1/30; u = (x-a)/((x-a)^2+(y-b)^2) + x^2/9 - y + 8 +
    exp(-5x^2), a = 1.1, b = 1.3, so -Lap u = -(2/9 + (100x^2 - 10) exp(-5x^2));
    g = nu . grad u.  History tolerance 1e-6, GMRES 1e-8, local terms up to
    O(delta) with three levels of dyadic refinement of the layer parts, as
    there; float64.  Timed from the mesh (not generated in the timed region)
    to u at every volume node: frames at the boundary nodes, the boundary
    plan, the Neumann solve, frames at the volume nodes, the evaluation plan,
    the layer jets, u = V[f] + S[g] - D[u_b], and the refinement.  Also timed
    with the plans and frames already built ("resident": the solve, the jets,
    the evaluation and the refinement).  Error as the paper defines it, about
    the value at a seeded node."""
    from paper_2409_11998_amd import Plan, boundary_frame, boundary_jets, neumann_solve
    from workloads.mesh import curve_mesh
    from workloads.problems import StarCurve, panel_nodes
    f64 = torch.float64
    curve = StarCurve(r=1.0, alpha=(5 / 6, 0, 0, 0, 0, 1 / 15, 1 / 30, 0, 1 / 30, 0, 1 / 30), beta=(0, 0, 1 / 30))
    a_, b_ = 1.1, 1.3

    def u_exact(x, y):
        return (x - a_) / ((x - a_) ** 2 + (y - b_) ** 2) + x * x / 9 - y + 8 + np.exp(-5 * x * x)

    def grad_u(x, y):
        dx, dy = x - a_, y - b_
        r4 = (dx * dx + dy * dy) ** 2
        return ((dy * dy - dx * dx) / r4 + 2 * x / 9 - 10 * x * np.exp(-5 * x * x), -2 * dx * dy / r4 - 1.0)

    def f_jets(x, y):   # f = -Lap u and its derivatives (f depends on x only)
        e = np.exp(-5 * x * x)
        z = np.zeros_like(x)
        return np.stack([-2 / 9 - (100 * x * x - 10) * e, -(300 * x - 1000 * x ** 3) * e, z,
                         -(300 - 6000 * x * x + 10000 * x ** 4) * e, z, z])

    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=f64, device="cuda")
    m = 2 ** levels
    rows = []
    for n_nodes in sizes:
        x, y, w, _ = curve_mesh(curve, int(round(n_nodes / 6)), 5)
        n_pan = int(np.ceil(2.5 * np.sqrt(x.size) / q))
        bx, by, bnx, bny, bw, _ = panel_nodes(curve, n_pan, q)
        fx, fy, fnx, fny, fw, _ = panel_nodes(curve, n_pan * m, q)
        gx, gy = grad_u(bx, by)
        g = gx * bnx + gy * bny
        gfx, gfy = grad_u(fx, fy)
        g_fine = gfx * fnx + gfy * fny
        # fine node (panel p, child c, point j) sits at u = -1 + (2c + 1 + x_j) / m of coarse panel p
        xg, _ = np.polynomial.legendre.leggauss(q)
        cc = np.arange(m)
        uf = (-1 + (2 * cc[:, None] + 1 + xg[None, :]) / m).ravel()
        pan_f = t(np.repeat(np.arange(n_pan), m * q)).to(torch.int32)
        u_f = t(np.tile(uf, n_pan))
        sx, sy, sw = t(x), t(y), t(w)
        fs, jv = t(f_jets(x, y)[0]), t(f_jets(x, y))
        jb = t(f_jets(bx, by))
        dx, dy, dnx, dny, dw, dg = (t(a) for a in (bx, by, bnx, bny, bw, g))
        ddx, ddy, ddnx, ddny, ddw, dgf = (t(a) for a in (fx, fy, fnx, fny, fw, g_fine))
        opts = dict(tol=1e-6, precision=1, kinds=7, order_v=2, order_s=2, order_d=2)
        torch.cuda.synchronize()
        st = {}

        def build():
            frb = boundary_frame(dx, dy, q, dx, dy)
            geom = dict(r=torch.zeros_like(dx), nx=frb["nx"], ny=frb["ny"], kappa=frb["kappa"],
                        gamma3=frb["gamma3"], gamma4=frb["gamma4"],
                        sgn=torch.ones(dx.numel(), dtype=torch.int8, device="cuda"))
            pb = Plan(sx, sy, sw, dx, dy, dnx, dny, dw, dx, dy, geom, **opts)
            frv = boundary_frame(dx, dy, q, sx, sy)
            gv = {k: frv[k] for k in ("r", "nx", "ny", "kappa", "gamma3", "gamma4", "sgn")}
            pv = Plan(sx, sy, sw, dx, dy, dnx, dny, dw, sx, sy, gv, **opts)
            pv.refine_attach(levels, ddx, ddy, ddnx, ddny, ddw, sx, sy)
            return frb, pb, frv, pv

        def solve(frb, pb, frv, pv):
            ub, st["its"], st["res"] = neumann_solve(pb, q, dx, dy, dw, frb["pan"], frb["u"], dg, f=fs, jet6=jb,
                                                     tol=1e-8)
            mub = -ub
            sj = boundary_jets(dx, dy, q, dg, frv["pan"], frv["u"], 2)
            mj = boundary_jets(dx, dy, q, mub, frv["pan"], frv["u"], 4)
            out = pv.eval(f=fs, jet6=jv, sigma=dg, sigma_jet=sj, mu=mub, mu_jet=mj)
            mu_fine = boundary_jets(dx, dy, q, mub, pan_f, u_f, 0)[0].contiguous()
            pv.layer_refine(out, sigma_jet=sj, fine_sigma=dgf, mu_jet=mj, fine_mu=mu_fine)
            return out

        # end to end (from the mesh): frames, plans, solve, evaluation, refinement
        t0 = time.perf_counter()
        frb, pb, frv, pv = build()
        out = solve(frb, pb, frv, pv)
        torch.cuda.synchronize()
        t_total = time.perf_counter() - t0
        for _ in range(reps):   # resident: plans and frames built
            out = solve(frb, pb, frv, pv)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            out = solve(frb, pb, frv, pv)
        torch.cuda.synchronize()
        t_res = (time.perf_counter() - t0) / reps
        info = pv.info()
        pb.close()
        pv.close()
        uc = out.cpu().numpy()
        ue = u_exact(x, y)
        c = int(np.random.default_rng(7).integers(0, x.size))
        du = (uc - uc[c]) - (ue - ue[c])
        e_inf = float(np.max(np.abs(du)) / np.max(np.abs(ue - ue[c])))
        e_2 = float(np.linalg.norm(du) / np.linalg.norm(ue - ue[c]))
        rows.append({"n_volume_nodes": int(x.size), "n_boundary_nodes": int(bx.size), "n_fine_boundary": int(fx.size),
                     "delta1": info["delta1"], "fine_grid": list(info["fine"]), "gmres_products": st["its"],
                     "rel_residual": st["res"], "end_to_end_s": round(t_total, 4),
                     "end_to_end_pts_per_s": round(x.size / t_total, 1), "resident_ms": round(1e3 * t_res, 3),
                     "resident_pts_per_s": round(x.size / t_res, 1), "e_inf": e_inf, "e_2": e_2})
        log("bench: Neumann (paper) N_V=%d end-to-end %.3f s, resident %.2f ms, e_inf %.2e" %
            (x.size, t_total, 1e3 * t_res, e_inf))
    return {"workload": "interior Neumann problem of the paper's numerical section (its curve, u, f, tolerances, "
                        "three refinement levels), float64", "rows": rows,
            "paper_one_core_pts_per_s": {"674664": 8.3e5, "1198728": 8.7e5, "2695248": 8.4e5}}


def refine_leg(torch, P, levels, steps):
    """Dyadic refinement of the local double-layer part on the square workload:
    every boundary panel split into 2^levels; time of the correction launch alone
    and of evaluation + correction, and the size of the correction (its parity
    against the oracle is a GPU test)."""
    from workloads.device import make_plan, run, to_device
    from workloads.problems import fine_boundary
    dev = to_device(P)
    plan = make_plan(dev, tol=1e-10, precision=1, kinds=5)
    delta = plan.info()["delta1"]
    fine = fine_boundary(P, levels)
    fd = {k: (torch.as_tensor(v, dtype=torch.float64, device="cuda") if v is not None else None)
          for k, v in fine.items()}
    t0 = time.perf_counter()
    plan.refine_attach(levels, fd["x"], fd["y"], fd["nx"], fd["ny"], fd["w"], dev["tgt_x"], dev["tgt_y"])
    attach_s = time.perf_counter() - t0
    out = torch.empty(P.n_tgt, dtype=torch.float64, device="cuda")
    corr_only = lambda: plan.layer_refine(out, mu_jet=dev["mu_jet"], fine_mu=fd["mu"])
    both = lambda: (run(plan, dev, "VD", out=out), corr_only())
    for _ in range(3):
        both()
    el_c = time_steps(torch, corr_only, steps)
    el_b = time_steps(torch, both, steps)
    base = run(plan, dev, "VD").cpu().numpy()
    both()
    torch.cuda.synchronize()
    corr = out.cpu().numpy() - base
    near = np.flatnonzero(np.asarray(P.geom["r"]) <= 12.0 * np.sqrt(delta))
    far = np.setdiff1d(np.arange(P.n_tgt), near)
    plan.close()
    return {"workload": "square-200k V+D fp64 tol1e-10, D_L refined", "levels": levels,
            "n_fine": int(fine["x"].size), "near_targets": int(near.size),
            "refine_ms": round(1e3 * el_c / steps, 4), "eval_plus_refine_ms": round(1e3 * el_b / steps, 4),
            "attach_s": round(attach_s, 3), "max_abs_correction": float(np.max(np.abs(corr))),
            "max_abs_correction_far_from_boundary": float(np.max(np.abs(corr[far]))) if far.size else 0.0}


def batch_leg(torch, probs, steps, warmup, tune_sample, classes):
    """Float32 V+D on many star instances: one persistent launch per stage (hipGraph)
    against the same plans launched one after another."""
    from paper_2409_11998_amd import Batch
    from workloads.device import make_batch_plans, run, to_device
    devs = [to_device(P) for P in probs]
    t0 = time.perf_counter()
    plans = make_batch_plans(devs, autotune_sample=tune_sample, classes=classes, tol=1e-6, precision=0, kinds=5)
    plan_s = time.perf_counter() - t0
    batch = Batch(plans, 5)
    outs = [torch.empty(P.n_tgt, dtype=torch.float64, device="cuda") for P in probs]
    args = [dict(f=d["f"], jet6=d["jet6"], mu=d["mu"], mu_jet=d["mu_jet"], out=o) for d, o in zip(devs, outs)]
    for _ in range(warmup):
        batch.eval(args, graph=True)
    batch.stream.synchronize()
    n_t = sum(P.n_tgt for P in probs)
    t0 = time.perf_counter()
    for _ in range(steps):
        batch.eval(args, graph=True)
    batch.stream.synchronize()
    el_b = time.perf_counter() - t0
    # stage times of the batched launch (a pass of its own: events between stages, no graph)
    batch.set_timing(True)
    stages = {}
    for _ in range(steps):
        batch.eval(args, graph=False)
        for k, v in batch.timing().items():
            stages[k] = stages.get(k, 0.0) + v / steps
    batch.set_timing(False)
    batch.stream.synchronize()
    # step-table bytes of the stages over all instances (float32: b = 4; one read of each input and
    # one write of each output), as for the single-plan legs
    b = 4
    sb = {"spread": 0, "fft": 0, "interp": 0}
    for P, p in zip(probs, plans):
        inf = p.info()
        for l in range(2):
            F2b = inf["fine"][l] ** 2 * b
            sb["spread"] += P.n_src * 3 * b + P.n_bnd * 5 * b + F2b + (2 * F2b if l == 1 else 0)
            sb["fft"] += 6 * F2b + (4 * F2b if l == 1 else 0)
            sb["interp"] += F2b + P.n_tgt * 3 * b
    fft_ms = stages["row_fft"] + stages["col_fwd_channels"] + stages["col_fft_mul"] + stages["row_ifft"]
    cells = int(sum(sum(F * F for F in p_.info()["fine"]) for p_ in plans))
    stage_frac = {"spread": sb["spread"] / (stages["spread"] * 1e-3) / 1e9 / HBM_PEAK_GBS,
                  "fft_chain": sb["fft"] / (fft_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                  "interp": sb["interp"] / (stages["interp"] * 1e-3) / 1e9 / HBM_PEAK_GBS}
    got = [o.cpu().numpy() for o in outs]
    # the same plans, one plain launch sequence each
    seq_outs = [torch.empty_like(o) for o in outs]
    for p, d, o in zip(plans, devs, seq_outs):
        run(p, d, "VD", out=o)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        for p, d, o in zip(plans, devs, seq_outs):
            run(p, d, "VD", out=o)
    torch.cuda.synchronize()
    el_s = time.perf_counter() - t0
    dev_single = max(float(np.max(np.abs(g - s.cpu().numpy())) / max(np.max(np.abs(s.cpu().numpy())), 1e-300))
                     for g, s in zip(got, seq_outs))
    sizes = [P.n_src for P in probs]
    wc = {}
    for P, p_ in zip(probs, plans):
        inf = p_.info()
        c = wc.setdefault((tuple(inf["width"]), tuple(inf["tile"])), [0, P.n_src, P.n_src])
        c[0] += 1
        c[1], c[2] = min(c[1], P.n_src), max(c[2], P.n_src)
    widths = [{"width": list(k[0]), "tile": list(k[1]), "instances": v[0], "nodes": [int(v[1]), int(v[2])]}
              for k, v in sorted(wc.items())]
    grids = sorted({tuple(p.info()["fine"]) for p in plans})
    batch.close()
    for p in plans:
        p.close()
    return {"workload": "%d star instances, triangles log-U[1e3,%g], V+D fp32 tol1e-6" % (len(probs), max(
                P.info["n_tri"] for P in probs)),
            "instances": len(probs), "n_tgt_total": n_t, "nodes_min": int(min(sizes)), "nodes_max": int(max(sizes)),
            "value": round(n_t * steps / el_b, 1), "unit": "target pts/s", "ms_per_step": round(1e3 * el_b / steps, 4),
            "sequential_value": round(n_t * steps / el_s, 1), "sequential_ms_per_step": round(1e3 * el_s / steps, 4),
            "max_rel_dev_vs_single_plans": dev_single,
            "stages_ms": {k: round(v, 4) for k, v in stages.items()},
            "steps_frac_of_hbm": {k: round(v, 4) for k, v in stage_frac.items()},
            "grid_cells_total": cells,
            "width_classes": widths, "fine_grids": [list(g) for g in grids],
            "autotune_sample_per_class": tune_sample,
            "plan_s": round(plan_s, 2)}


def serve_leg(torch, probs, n_req, loads):
    """Poisson streams of V/S/D requests (70% float32 1e-6, 30% float64 1e-10) on
    resident plans through the serving loop, at several arrival rates (fractions of
    the measured saturated rate); the same arrival stream is also served by the
    plain float64 path (every request at 1e-10, one at a time in arrival order)."""
    from paper_2409_11998_amd import Server
    from workloads.device import make_plan, to_device
    devs = [to_device(P) for P in probs]
    plans = {}
    for i, d in enumerate(devs):
        for prec, tol in ((0, 1e-6), (1, 1e-10)):
            plans[(i, prec)] = make_plan(d, tol=tol, precision=prec, kinds=7, no_workspace=True)
    fp64_plans = {i: make_plan(d, tol=1e-10, precision=1, kinds=7) for i, d in enumerate(devs)}
    rng = np.random.default_rng(55)

    def draw(n):
        out = []
        for _ in range(n):
            i = int(rng.integers(len(probs)))
            kind = "VSD"[int(rng.integers(3))]
            prec = 0 if rng.uniform() < 0.7 else 1
            out.append((i, kind, prec))
        return out

    def kw(d, kind):
        return dict(f=d["f"] if kind == "V" else None, jet6=d["jet6"] if kind == "V" else None,
                    sigma=d["sigma"] if kind == "S" else None, sigma_jet=d["sigma_jet"] if kind == "S" else None,
                    mu=d["mu"] if kind == "D" else None, mu_jet=d["mu_jet"] if kind == "D" else None)
    budget = int(0.8 * torch.cuda.mem_get_info()[0])
    # saturated rate: a request list submitted at once
    sat_reqs = draw(min(400, n_req))
    srv = Server(hbm_budget_bytes=budget, max_in_flight=64, n_streams=4)
    sat_out = [torch.empty(probs[i].n_tgt, dtype=torch.float64, device="cuda") for i, _, _ in sat_reqs]
    torch.cuda.synchronize()
    tk = [srv.submit(plans[(i, p)], o, **kw(devs[i], k)) for (i, k, p), o in zip(sat_reqs, sat_out)]
    for t in tk:
        srv.wait(t, timeout=300)
    sat = srv.stats()
    srv.close()
    del sat_out
    rate_sat = sat["completed"] / max(sat["span_s"], 1e-9)
    res = {"workload": "%d requests per load on %d seeded star meshes (nodes log-U[2e3,5e5]); kinds V/S/D "
                       "uniform; 70%% fp32 1e-6 / 30%% fp64 1e-10; Poisson arrivals" % (n_req, len(probs)),
           "saturated_req_per_s": round(rate_sat, 1), "saturated_mean_group": round(sat["mean_group"], 2),
           "hbm_budget_bytes": budget, "loads": {}}
    for load in loads:
        reqs = draw(n_req)
        lam = load * rate_sat
        arrive = np.cumsum(rng.exponential(1.0 / lam, n_req))
        n_t = sum(probs[i].n_tgt for i, _, _ in reqs)
        # served: mixed precision plans through the serving loop
        srv = Server(hbm_budget_bytes=budget, max_in_flight=64, n_streams=4)
        req_out = [torch.empty(probs[i].n_tgt, dtype=torch.float64, device="cuda") for i, _, _ in reqs]
        torch.cuda.synchronize()
        tickets = []
        t0 = time.perf_counter()
        for r, (i, k, p) in enumerate(reqs):
            while time.perf_counter() - t0 < arrive[r]:
                pass
            tickets.append(srv.submit(plans[(i, p)], req_out[r], **kw(devs[i], k)))
        for t in tickets:
            srv.wait(t, timeout=600)
        st = srv.stats()
        srv.close()
        del req_out
        # plain float64: the same arrivals, one request at a time, each synchronized
        lat = np.empty(n_req)
        outs = {i: torch.empty(P.n_tgt, dtype=torch.float64, device="cuda") for i, P in enumerate(probs)}
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for r, (i, k, p) in enumerate(reqs):
            while time.perf_counter() - t0 < arrive[r]:
                pass
            fp64_plans[i].eval(out=outs[i], **kw(devs[i], k))
            torch.cuda.synchronize()
            lat[r] = time.perf_counter() - t0 - arrive[r]
        span64 = time.perf_counter() - t0
        lat.sort()
        res["loads"]["%.2f" % load] = {
            "arrival_req_per_s": round(lam, 1),
            "served": {"p50_s": st["p50_s"], "p99_s": st["p99_s"], "max_s": st["max_s"],
                       "targets_per_s": round(st["targets_per_s"], 1), "completed": st["completed"],
                       "deferred": st["deferred"], "peak_in_flight": st["peak_in_flight"],
                       "groups": st["groups"], "mean_group": round(st["mean_group"], 2),
                       "peak_held_bytes": st["peak_held_bytes"], "device_allocs": st["device_allocs"],
                       "peak_workspace_bytes": st["peak_bytes"]},
            "plain_fp64": {"p50_s": float(lat[n_req // 2]), "p99_s": float(lat[min(n_req - 1, int(0.99 * n_req))]),
                           "max_s": float(lat[-1]), "targets_per_s": round(n_t / span64, 1)}}
    for p in list(plans.values()) + list(fp64_plans.values()):
        p.close()
    return res


if __name__ == "__main__":
    main()
