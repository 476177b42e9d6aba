"""ctypes binding of libvp.so (include/vp.h): argument marshalling only.

Device memory comes from PyTorch CUDA tensors (float64; int8 for sgn); every
step of the computation runs in the library's HIP kernels.  There is no CPU
fallback: without the built library or a HIP device the calls raise.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvp.so")

VP_FP32, VP_FP64 = 0, 1
NOALLOC_MAX_NODES = 65536   # VP_NOALLOC_MAX_NODES of include/vp.h
VP_KIND_V, VP_KIND_S, VP_KIND_D = 1, 2, 4
(VP_OK, VP_ERR_ARG, VP_ERR_OOM, VP_ERR_DEVICE, VP_ERR_GEOMETRY, VP_ERR_TOL, VP_ERR_BUSY,
 VP_ERR_INTERNAL) = range(8)
STATUS = {0: "VP_OK", 1: "VP_ERR_ARG", 2: "VP_ERR_OOM", 3: "VP_ERR_DEVICE", 4: "VP_ERR_GEOMETRY",
          5: "VP_ERR_TOL", 6: "VP_ERR_BUSY", 7: "VP_ERR_INTERNAL"}

EXPORTED = ["vp_opts_default", "vp_plan", "vp_eval", "vp_volume", "vp_layer", "vp_destroy",
            "vp_last_error", "vp_get_plan_info", "vp_set_timing", "vp_get_timing",
            "vp_batch_create", "vp_batch_eval", "vp_batch_destroy", "vp_batch_last_error",
            "vp_batch_set_timing", "vp_batch_get_timing",
            "vp_server_create", "vp_server_submit", "vp_server_poll", "vp_server_wait", "vp_server_get_stats",
            "vp_server_destroy", "vp_server_last_error", "vp_refine_attach", "vp_layer_refine",
            "vp_boundary_frame", "vp_boundary_jets", "vp_dirichlet_solve", "vp_exterior_dirichlet_solve",
            "vp_neumann_solve", "vp_volume_jets", "vp_boundary_jets_noalloc", "vp_exterior_dirichlet_solve_growth",
            "vp_add_log_growth", "vp_volume_jets_patch"]


class VPError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS.get(status, status), msg))
        self.status = status


class VPOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("precision", ctypes.c_int), ("c_delta", ctypes.c_double),
                ("delta_ratio", ctypes.c_double), ("order_v", ctypes.c_int), ("order_s", ctypes.c_int),
                ("order_d", ctypes.c_int), ("kinds", ctypes.c_int), ("fine_grid", ctypes.c_int * 2),
                ("spread_width", ctypes.c_int * 2), ("tile", ctypes.c_int), ("stream", ctypes.c_void_p),
                ("no_workspace", ctypes.c_int), ("autotune", ctypes.c_int)]


class VPLocalGeom(ctypes.Structure):
    _fields_ = [("r", ctypes.c_void_p), ("nx", ctypes.c_void_p), ("ny", ctypes.c_void_p),
                ("kappa", ctypes.c_void_p), ("gamma3", ctypes.c_void_p), ("gamma4", ctypes.c_void_p),
                ("sgn", ctypes.c_void_p)]


class VPEvalArgs(ctypes.Structure):
    _fields_ = [("f_src", ctypes.c_void_p), ("jet6", ctypes.c_void_p), ("sigma", ctypes.c_void_p),
                ("sigma_jet3", ctypes.c_void_p), ("mu", ctypes.c_void_p), ("mu_jet5", ctypes.c_void_p),
                ("out", ctypes.c_void_p)]


class VPServerOpts(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_size_t), ("max_in_flight", ctypes.c_int), ("n_streams", ctypes.c_int),
                ("max_wait_us", ctypes.c_int)]


class VPRequest(ctypes.Structure):
    _fields_ = [("plan", ctypes.c_void_p), ("f_src", ctypes.c_void_p), ("jet6", ctypes.c_void_p),
                ("sigma", ctypes.c_void_p), ("sigma_jet3", ctypes.c_void_p), ("mu", ctypes.c_void_p),
                ("mu_jet5", ctypes.c_void_p), ("out", ctypes.c_void_p)]


class VPServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64), ("rejected", ctypes.c_uint64),
                ("failed", ctypes.c_uint64), ("deferred", ctypes.c_uint64), ("peak_bytes", ctypes.c_size_t),
                ("peak_in_flight", ctypes.c_int), ("p50_s", ctypes.c_double), ("p99_s", ctypes.c_double),
                ("max_s", ctypes.c_double), ("mean_s", ctypes.c_double), ("span_s", ctypes.c_double),
                ("targets_per_s", ctypes.c_double), ("groups", ctypes.c_uint64), ("mean_group", ctypes.c_double),
                ("peak_held_bytes", ctypes.c_size_t), ("device_allocs", ctypes.c_uint64)]


class VPPlanInfo(ctypes.Structure):
    _fields_ = [("delta1", ctypes.c_double), ("delta2", ctypes.c_double), ("eps_hist", ctypes.c_double),
                ("period", ctypes.c_double * 2), ("kmax", ctypes.c_double * 2), ("trunc_L", ctypes.c_double),
                ("modes", ctypes.c_int * 2), ("fine", ctypes.c_int * 2), ("width", ctypes.c_int * 2),
                ("tile", ctypes.c_int * 2), ("spread_mma", ctypes.c_int * 2), ("precision", ctypes.c_int),
                ("n_src", ctypes.c_int64),
                ("n_bnd", ctypes.c_int64), ("n_tgt", ctypes.c_int64), ("spread_records", ctypes.c_int64 * 2),
                ("device_bytes", ctypes.c_size_t), ("workspace_bytes", ctypes.c_size_t),
                ("autotuned", ctypes.c_int), ("tune_candidates", ctypes.c_int * 2), ("level_ms", ctypes.c_double * 2),
                ("spread_terms", ctypes.c_int * 2), ("interp_terms", ctypes.c_int * 2),
                ("spread_fit_err", ctypes.c_double * 2), ("interp_fit_err", ctypes.c_double * 2),
                ("interp_tile", ctypes.c_int * 2)]


_lib = None


def lib():
    """Load libvp.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libvp.so is not built (run __graft_entry__.build() or "
                               "python paper_2409_11998_amd/build.py)")
        L = ctypes.CDLL(LIB_PATH)
        vp = ctypes.c_void_p
        i64 = ctypes.c_int64
        L.vp_opts_default.argtypes = [ctypes.POINTER(VPOpts)]
        L.vp_opts_default.restype = None
        L.vp_plan.argtypes = [ctypes.POINTER(vp), i64, vp, vp, vp, i64, vp, vp, vp, vp, vp, i64, vp, vp,
                              ctypes.POINTER(VPLocalGeom), ctypes.POINTER(VPOpts)]
        L.vp_plan.restype = ctypes.c_int
        L.vp_eval.argtypes = [vp] * 8
        L.vp_eval.restype = ctypes.c_int
        L.vp_volume.argtypes = [vp] * 4
        L.vp_volume.restype = ctypes.c_int
        L.vp_layer.argtypes = [vp] * 6
        L.vp_layer.restype = ctypes.c_int
        L.vp_refine_attach.argtypes = [vp, ctypes.c_int, ctypes.c_int64] + [vp] * 7
        L.vp_refine_attach.restype = ctypes.c_int
        L.vp_layer_refine.argtypes = [vp] * 6
        L.vp_layer_refine.restype = ctypes.c_int
        L.vp_boundary_frame.argtypes = [i64, ctypes.c_int, vp, vp, i64] + [vp] * 11 + [vp]
        L.vp_boundary_frame.restype = ctypes.c_int
        L.vp_boundary_jets.argtypes = [i64, ctypes.c_int, vp, vp, vp, i64, vp, vp, ctypes.c_int, vp, vp]
        L.vp_boundary_jets.restype = ctypes.c_int
        L.vp_boundary_jets_noalloc.argtypes = [i64, ctypes.c_int, vp, vp, vp, i64, vp, vp, ctypes.c_int, vp, vp]
        L.vp_boundary_jets_noalloc.restype = ctypes.c_int
        L.vp_dirichlet_solve.argtypes = [vp, i64, ctypes.c_int, vp, vp, vp, vp, vp, vp, vp, vp, ctypes.c_double,
                                         ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double)]
        L.vp_dirichlet_solve.restype = ctypes.c_int
        L.vp_exterior_dirichlet_solve.argtypes = [vp, i64, ctypes.c_int, vp, vp, vp, vp, vp, vp, vp, ctypes.c_double,
                                                  ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                                  ctypes.POINTER(ctypes.c_double)]
        L.vp_exterior_dirichlet_solve.restype = ctypes.c_int
        L.vp_exterior_dirichlet_solve_growth.argtypes = [vp, i64, ctypes.c_int, vp, vp, vp, vp, vp, vp,
                                                         ctypes.c_double, ctypes.c_double, ctypes.c_double, vp,
                                                         ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                                         ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double)]
        L.vp_exterior_dirichlet_solve_growth.restype = ctypes.c_int
        L.vp_add_log_growth.argtypes = [i64, vp, vp, ctypes.c_double, ctypes.c_double, ctypes.c_double, vp, vp]
        L.vp_add_log_growth.restype = ctypes.c_int
        L.vp_neumann_solve.argtypes = [vp, i64, ctypes.c_int, vp, vp, vp, vp, vp, vp, vp, vp, vp, ctypes.c_double,
                                       ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                       ctypes.POINTER(ctypes.c_double)]
        L.vp_neumann_solve.restype = ctypes.c_int
        L.vp_volume_jets.argtypes = [i64, vp, vp, vp, vp, vp]
        L.vp_volume_jets.restype = ctypes.c_int
        L.vp_volume_jets_patch.argtypes = [i64, vp, vp, vp, vp, vp, vp]
        L.vp_volume_jets_patch.restype = ctypes.c_int
        L.vp_destroy.argtypes = [vp]
        L.vp_destroy.restype = ctypes.c_int
        L.vp_last_error.argtypes = []
        L.vp_last_error.restype = ctypes.c_char_p
        L.vp_get_plan_info.argtypes = [vp, ctypes.POINTER(VPPlanInfo)]
        L.vp_get_plan_info.restype = ctypes.c_int
        L.vp_set_timing.argtypes = [vp, ctypes.c_int]
        L.vp_set_timing.restype = ctypes.c_int
        L.vp_get_timing.argtypes = [vp, ctypes.POINTER(ctypes.c_double)]
        L.vp_get_timing.restype = ctypes.c_int
        L.vp_batch_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int, ctypes.POINTER(vp), ctypes.c_int, vp]
        L.vp_batch_create.restype = ctypes.c_int
        L.vp_batch_eval.argtypes = [vp, ctypes.POINTER(VPEvalArgs), ctypes.c_int]
        L.vp_batch_eval.restype = ctypes.c_int
        L.vp_batch_destroy.argtypes = [vp]
        L.vp_batch_destroy.restype = ctypes.c_int
        L.vp_batch_set_timing.argtypes = [vp, ctypes.c_int]
        L.vp_batch_set_timing.restype = ctypes.c_int
        L.vp_batch_get_timing.argtypes = [vp, ctypes.POINTER(ctypes.c_float), ctypes.c_int]
        L.vp_batch_get_timing.restype = ctypes.c_int
        L.vp_batch_last_error.argtypes = []
        L.vp_batch_last_error.restype = ctypes.c_char_p
        L.vp_server_create.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(VPServerOpts)]
        L.vp_server_create.restype = ctypes.c_int
        L.vp_server_submit.argtypes = [vp, ctypes.POINTER(VPRequest), ctypes.POINTER(ctypes.c_uint64)]
        L.vp_server_submit.restype = ctypes.c_int
        L.vp_server_poll.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                     ctypes.POINTER(ctypes.c_double)]
        L.vp_server_poll.restype = ctypes.c_int
        L.vp_server_wait.argtypes = [vp, ctypes.c_uint64, ctypes.c_double, ctypes.POINTER(ctypes.c_int),
                                     ctypes.POINTER(ctypes.c_double)]
        L.vp_server_wait.restype = ctypes.c_int
        L.vp_server_get_stats.argtypes = [vp, ctypes.POINTER(VPServerStats)]
        L.vp_server_get_stats.restype = ctypes.c_int
        L.vp_server_destroy.argtypes = [vp]
        L.vp_server_destroy.restype = ctypes.c_int
        L.vp_server_last_error.argtypes = []
        L.vp_server_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _check(status):
    if status != 0:
        raise VPError(status, lib().vp_last_error().decode(errors="replace"))


def default_opts():
    o = VPOpts()
    lib().vp_opts_default(ctypes.byref(o))
    return o


def _ptr(t, dtype=None):
    """Device pointer of a CUDA tensor (None -> NULL)."""
    if t is None:
        return None
    import torch
    if not t.is_cuda:
        raise ValueError("expected a device (CUDA/HIP) tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    if dtype is not None and t.dtype != dtype:
        raise ValueError("expected dtype %s, got %s" % (dtype, t.dtype))
    return ctypes.c_void_p(t.data_ptr())


class Plan:
    """A plan bound to fixed nodes and targets (vp_plan); see include/vp.h."""

    def __init__(self, src_x, src_y, src_w, bnd_x=None, bnd_y=None, bnd_nx=None, bnd_ny=None, bnd_w=None,
                 tgt_x=None, tgt_y=None, geom=None, tol=1e-10, precision=VP_FP64, kinds=7, stream=None,
                 c_delta=3.0, delta_ratio=32.0, order_v=4, order_s=3, order_d=3, fine_grid=(0, 0),
                 spread_width=(0, 0), tile=0, no_workspace=False, autotune=False):
        import torch
        f64 = torch.float64
        o = default_opts()
        o.tol = tol
        o.precision = precision
        o.c_delta = c_delta
        o.delta_ratio = delta_ratio
        o.order_v, o.order_s, o.order_d = order_v, order_s, order_d
        o.kinds = kinds
        o.fine_grid[0], o.fine_grid[1] = fine_grid
        o.spread_width[0], o.spread_width[1] = spread_width
        o.tile = tile
        o.no_workspace = 1 if no_workspace else 0
        o.autotune = 1 if autotune else 0
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        o.stream = ctypes.c_void_p(stream.cuda_stream)
        n_src = 0 if src_x is None else src_x.numel()
        n_bnd = 0 if bnd_x is None else bnd_x.numel()
        n_tgt = tgt_x.numel()
        g = VPLocalGeom()
        g.r = _ptr(geom["r"], f64)
        g.nx = _ptr(geom["nx"], f64)
        g.ny = _ptr(geom["ny"], f64)
        g.kappa = _ptr(geom["kappa"], f64)
        g.gamma3 = _ptr(geom.get("gamma3"), f64)
        g.gamma4 = _ptr(geom.get("gamma4"), f64)
        g.sgn = _ptr(geom["sgn"], torch.int8)
        h = ctypes.c_void_p()
        _check(lib().vp_plan(ctypes.byref(h), n_src, _ptr(src_x, f64), _ptr(src_y, f64), _ptr(src_w, f64),
                             n_bnd, _ptr(bnd_x, f64), _ptr(bnd_y, f64), _ptr(bnd_nx, f64), _ptr(bnd_ny, f64),
                             _ptr(bnd_w, f64), n_tgt, _ptr(tgt_x, f64), _ptr(tgt_y, f64), ctypes.byref(g),
                             ctypes.byref(o)))
        self.handle = h
        self.n_src, self.n_bnd, self.n_tgt = n_src, n_bnd, n_tgt
        self.device = tgt_x.device

    def eval(self, f=None, jet6=None, sigma=None, sigma_jet=None, mu=None, mu_jet=None, out=None):
        """V[f] + S[sigma] + D[mu] at the targets (vp_eval); returns out (float64)."""
        import torch
        f64 = torch.float64
        if out is None:
            out = torch.empty(self.n_tgt, dtype=f64, device=self.device)
        _check(lib().vp_eval(self.handle, _ptr(f, f64), _ptr(jet6, f64), _ptr(sigma, f64), _ptr(sigma_jet, f64),
                             _ptr(mu, f64), _ptr(mu_jet, f64), _ptr(out, f64)))
        return out

    def volume(self, f, jet6, out=None):
        import torch
        if out is None:
            out = torch.empty(self.n_tgt, dtype=torch.float64, device=self.device)
        _check(lib().vp_volume(self.handle, _ptr(f, torch.float64), _ptr(jet6, torch.float64),
                               _ptr(out, torch.float64)))
        return out

    def layer(self, sigma=None, sigma_jet=None, mu=None, mu_jet=None, out=None):
        import torch
        f64 = torch.float64
        if out is None:
            out = torch.empty(self.n_tgt, dtype=f64, device=self.device)
        _check(lib().vp_layer(self.handle, _ptr(sigma, f64), _ptr(sigma_jet, f64), _ptr(mu, f64),
                              _ptr(mu_jet, f64), _ptr(out, f64)))
        return out

    def refine_attach(self, levels, fine_x, fine_y, fine_nx, fine_ny, fine_w, tgt_x, tgt_y):
        """Attach the oversampled boundary of the dyadic refinement (vp_refine_attach)."""
        import torch
        f64 = torch.float64
        _check(lib().vp_refine_attach(self.handle, int(levels), int(fine_x.numel()), _ptr(fine_x, f64),
                                      _ptr(fine_y, f64), _ptr(fine_nx, f64), _ptr(fine_ny, f64), _ptr(fine_w, f64),
                                      _ptr(tgt_x, f64), _ptr(tgt_y, f64)))
        self._refine_keep = (fine_x, fine_y, fine_nx, fine_ny, fine_w)

    def layer_refine(self, out, sigma_jet=None, fine_sigma=None, mu_jet=None, fine_mu=None):
        """Add the dyadic refinement of the local layer parts to out (vp_layer_refine)."""
        import torch
        f64 = torch.float64
        _check(lib().vp_layer_refine(self.handle, _ptr(sigma_jet, f64), _ptr(fine_sigma, f64), _ptr(mu_jet, f64),
                                     _ptr(fine_mu, f64), _ptr(out, f64)))
        return out

    def info(self):
        i = VPPlanInfo()
        _check(lib().vp_get_plan_info(self.handle, ctypes.byref(i)))
        return dict(delta1=i.delta1, delta2=i.delta2, eps_hist=i.eps_hist, period=tuple(i.period),
                    kmax=tuple(i.kmax), trunc_L=i.trunc_L, modes=tuple(i.modes), fine=tuple(i.fine),
                    width=tuple(i.width), tile=tuple(i.tile), spread_mma=tuple(i.spread_mma), precision=i.precision, n_src=i.n_src, n_bnd=i.n_bnd,
                    n_tgt=i.n_tgt, spread_records=tuple(i.spread_records), device_bytes=i.device_bytes,
                    workspace_bytes=i.workspace_bytes, autotuned=bool(i.autotuned),
                    tune_candidates=tuple(i.tune_candidates), level_ms=tuple(i.level_ms),
                    spread_terms=tuple(i.spread_terms), interp_terms=tuple(i.interp_terms),
                    spread_fit_err=tuple(i.spread_fit_err), interp_fit_err=tuple(i.interp_fit_err),
                    interp_tile=tuple(i.interp_tile))

    def set_timing(self, on=True):
        _check(lib().vp_set_timing(self.handle, 1 if on else 0))

    LAUNCHES = ["strengths", "spread_nh", "spread_fh", "row_fft_nh", "row_fft_fh", "col_fft_mul_nh",
                "col_fft_mul_fh", "row_ifft_nh", "row_ifft_fh", "interp_nh", "interp_fh", "local", "total"]

    def timing(self):
        """Per-launch milliseconds of the last evaluation (see vp_get_timing), plus per-stage sums."""
        a = (ctypes.c_double * 13)()
        _check(lib().vp_get_timing(self.handle, a))
        d = dict(zip(self.LAUNCHES, list(a)))
        for st in ("spread", "row_fft", "col_fft_mul", "row_ifft", "interp"):
            d[st] = d[st + "_nh"] + d[st + "_fh"]
        return d

    def close(self):
        if getattr(self, "handle", None):
            lib().vp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _bcheck(status):
    if status != 0:
        raise VPError(status, lib().vp_batch_last_error().decode(errors="replace"))


class Batch:
    """Plans executed together by one persistent kernel per stage (vp_batch_*)."""

    def __init__(self, plans, kinds, stream=None):
        import torch
        self.plans = list(plans)  # keep the plans alive
        if stream is None:
            stream = torch.cuda.Stream()
        self.stream = stream
        arr = (ctypes.c_void_p * len(self.plans))(*[p.handle for p in self.plans])
        h = ctypes.c_void_p()
        _bcheck(lib().vp_batch_create(ctypes.byref(h), len(self.plans), arr, kinds,
                                      ctypes.c_void_p(stream.cuda_stream)))
        self.handle = h
        self.kinds = kinds

    def eval(self, args, graph=True):
        """args: list of dicts with tensors f, jet6, sigma, sigma_jet, mu, mu_jet, out (per instance)."""
        import torch
        f64 = torch.float64
        n = len(self.plans)
        a = (VPEvalArgs * n)()
        for i, d in enumerate(args):
            a[i].f_src = _ptr(d.get("f"), f64)
            a[i].jet6 = _ptr(d.get("jet6"), f64)
            a[i].sigma = _ptr(d.get("sigma"), f64)
            a[i].sigma_jet3 = _ptr(d.get("sigma_jet"), f64)
            a[i].mu = _ptr(d.get("mu"), f64)
            a[i].mu_jet5 = _ptr(d.get("mu_jet"), f64)
            a[i].out = _ptr(d["out"], f64)
        _bcheck(lib().vp_batch_eval(self.handle, a, 1 if graph else 0))

    BATCH_STAGES = ("zero", "strengths", "spread", "row_fft", "col_fwd_channels", "col_fft_mul", "row_ifft",
                    "interp", "local")

    def set_timing(self, on):
        """Record stage events in later eval calls (vp_batch_set_timing; those calls run without the graph)."""
        _bcheck(lib().vp_batch_set_timing(self.handle, 1 if on else 0))

    def timing(self):
        """{stage: ms} of the last timed eval (vp_batch_get_timing)."""
        ms = (ctypes.c_float * len(self.BATCH_STAGES))()
        _bcheck(lib().vp_batch_get_timing(self.handle, ms, len(self.BATCH_STAGES)))
        return dict(zip(self.BATCH_STAGES, [float(v) for v in ms]))

    def close(self):
        if getattr(self, "handle", None):
            lib().vp_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _scheck(status):
    if status != 0:
        raise VPError(status, lib().vp_server_last_error().decode(errors="replace"))


class Server:
    """Continuous-admission serving loop (vp_server_*); requests name resident plans."""

    def __init__(self, hbm_budget_bytes, max_in_flight=8, n_streams=4, max_wait_us=0):
        o = VPServerOpts(int(hbm_budget_bytes), int(max_in_flight), int(n_streams), int(max_wait_us))
        h = ctypes.c_void_p()
        _scheck(lib().vp_server_create(ctypes.byref(h), ctypes.byref(o)))
        self.handle = h
        self._keep = {}

    def submit(self, plan, out, f=None, jet6=None, sigma=None, sigma_jet=None, mu=None, mu_jet=None):
        """Queue one evaluation (inputs must be ready on the device); returns a ticket."""
        import torch
        f64 = torch.float64
        r = VPRequest(plan.handle, _ptr(f, f64), _ptr(jet6, f64), _ptr(sigma, f64), _ptr(sigma_jet, f64),
                      _ptr(mu, f64), _ptr(mu_jet, f64), _ptr(out, f64))
        t = ctypes.c_uint64()
        _scheck(lib().vp_server_submit(self.handle, ctypes.byref(r), ctypes.byref(t)))
        self._keep[t.value] = (plan, out, f, jet6, sigma, sigma_jet, mu, mu_jet)
        return t.value

    def poll(self, ticket):
        done = ctypes.c_int()
        st = ctypes.c_int()
        lat = ctypes.c_double()
        _scheck(lib().vp_server_poll(self.handle, ticket, ctypes.byref(done), ctypes.byref(st), ctypes.byref(lat)))
        return (bool(done.value), st.value, lat.value) if done.value else (False, None, None)

    def wait(self, ticket, timeout=60.0):
        st = ctypes.c_int()
        lat = ctypes.c_double()
        _scheck(lib().vp_server_wait(self.handle, ticket, float(timeout), ctypes.byref(st), ctypes.byref(lat)))
        self._keep.pop(ticket, None)
        return st.value, lat.value

    def stats(self):
        s = VPServerStats()
        _scheck(lib().vp_server_get_stats(self.handle, ctypes.byref(s)))
        return {k: getattr(s, k) for k, _ in VPServerStats._fields_}

    def close(self):
        if getattr(self, "handle", None):
            lib().vp_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _stream(t):
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


def boundary_frame(bnd_x, bnd_y, q, tgt_x, tgt_y):
    """Local frame of each target from a boundary of Gauss-Legendre panels
    (vp_boundary_frame): dict of device tensors r, nx, ny, kappa, gamma3,
    gamma4 (float64), sgn (int8), pan (int32), u (float64)."""
    import torch
    f64 = torch.float64
    nb, n = bnd_x.numel(), tgt_x.numel()
    if q <= 0 or nb % q:
        raise ValueError("the boundary must hold whole panels of q nodes")
    dev = tgt_x.device
    out = {k: torch.empty(n, dtype=f64, device=dev) for k in ("r", "nx", "ny", "kappa", "gamma3", "gamma4", "u")}
    out["sgn"] = torch.empty(n, dtype=torch.int8, device=dev)
    out["pan"] = torch.empty(n, dtype=torch.int32, device=dev)
    _check(lib().vp_boundary_frame(nb // q, q, _ptr(bnd_x, f64), _ptr(bnd_y, f64), n, _ptr(tgt_x, f64),
                                   _ptr(tgt_y, f64), _ptr(out["r"]), _ptr(out["nx"]), _ptr(out["ny"]),
                                   _ptr(out["kappa"]), _ptr(out["gamma3"]), _ptr(out["gamma4"]), _ptr(out["sgn"]),
                                   _ptr(out["pan"]), _ptr(out["u"]), _stream(tgt_x)))
    return out


def boundary_jets(bnd_x, bnd_y, q, dens, pan, u, nder, out=None, noalloc=False):
    """d^k dens / d xi^k, k = 0..nder, at each target's closest boundary point
    (vp_boundary_jets; with noalloc, vp_boundary_jets_noalloc, which writes
    into a caller-given out and allocates nothing): device tensor
    [nder + 1, n_tgt]."""
    import torch
    f64 = torch.float64
    nb, n = bnd_x.numel(), pan.numel()
    if q <= 0 or nb % q:
        raise ValueError("the boundary must hold whole panels of q nodes")
    if out is None:
        out = torch.empty((nder + 1, n), dtype=f64, device=pan.device)
    elif tuple(out.shape) != (nder + 1, n) or out.dtype != f64 or not out.is_contiguous():
        raise ValueError("out must be a contiguous float64 tensor of shape (nder + 1, n_tgt)")
    fn = lib().vp_boundary_jets_noalloc if noalloc else lib().vp_boundary_jets
    _check(fn(nb // q, q, _ptr(bnd_x, f64), _ptr(bnd_y, f64), _ptr(dens, f64), n,
              _ptr(pan, torch.int32), _ptr(u, f64), nder, _ptr(out), _stream(pan)))
    return out


def dirichlet_solve(plan, q, bnd_x, bnd_y, pan, u, g, mu=None, tol=1e-12, max_iter=200, restart=50, f=None,
                    jet6=None):
    """mu with D_int[mu] = g - V[f] at the panel nodes (vp_dirichlet_solve);
    plan's boundary nodes and targets are the nodes (targets with r = 0,
    sgn = +1); f at the plan's volume nodes and jet6 [6, n_bnd] at the boundary
    nodes, or neither.  Returns (mu, products, relative residual)."""
    import torch
    f64 = torch.float64
    n = bnd_x.numel()
    if mu is None:
        mu = torch.zeros(n, dtype=f64, device=g.device)
    it = ctypes.c_int(0)
    res = ctypes.c_double(0.0)
    _check(lib().vp_dirichlet_solve(plan.handle, n // q, q, _ptr(bnd_x, f64), _ptr(bnd_y, f64),
                                    _ptr(pan, torch.int32), _ptr(u, f64), _ptr(g, f64), _ptr(f, f64),
                                    _ptr(jet6, f64), _ptr(mu, f64), tol,
                                    max_iter, restart, ctypes.byref(it), ctypes.byref(res)))
    return mu, it.value, res.value


def exterior_dirichlet_solve(plan, q, bnd_x, bnd_y, bnd_w, pan, u, g, mu=None, tol=1e-12, max_iter=200, restart=50):
    """mu with mu/2 + D[mu] + (integral of mu) = g at the panel nodes
    (vp_exterior_dirichlet_solve); u = D[mu] + (integral of mu) outside.
    Returns (mu, products, relative residual)."""
    import torch
    f64 = torch.float64
    n = bnd_x.numel()
    if mu is None:
        mu = torch.zeros(n, dtype=f64, device=g.device)
    it = ctypes.c_int(0)
    res = ctypes.c_double(0.0)
    _check(lib().vp_exterior_dirichlet_solve(plan.handle, n // q, q, _ptr(bnd_x, f64), _ptr(bnd_y, f64),
                                             _ptr(bnd_w, f64), _ptr(pan, torch.int32), _ptr(u, f64), _ptr(g, f64),
                                             _ptr(mu, f64), tol, max_iter, restart, ctypes.byref(it),
                                             ctypes.byref(res)))
    return mu, it.value, res.value


def exterior_dirichlet_solve_growth(plan, q, bnd_x, bnd_y, bnd_w, pan, u, g, A, x0, mu=None, tol=1e-12, max_iter=200,
                                    restart=50):
    """mu with mu/2 + D[mu] + (integral of mu) = g - A log|x' - x0| at the panel
    nodes (vp_exterior_dirichlet_solve_growth); u = D[mu] + (integral of mu) +
    A log|x - x0| outside.  x0 = (x, y).  Returns (mu, products, relative residual)."""
    import torch
    f64 = torch.float64
    n = bnd_x.numel()
    if mu is None:
        mu = torch.zeros(n, dtype=f64, device=g.device)
    it = ctypes.c_int(0)
    res = ctypes.c_double(0.0)
    _check(lib().vp_exterior_dirichlet_solve_growth(plan.handle, n // q, q, _ptr(bnd_x, f64), _ptr(bnd_y, f64),
                                                    _ptr(bnd_w, f64), _ptr(pan, torch.int32), _ptr(u, f64),
                                                    _ptr(g, f64), float(A), float(x0[0]), float(x0[1]), _ptr(mu, f64),
                                                    tol, max_iter, restart, ctypes.byref(it), ctypes.byref(res)))
    return mu, it.value, res.value


def add_log_growth(x, y, A, x0, out):
    """out += A log|(x, y) - x0| in place (vp_add_log_growth), on the current stream."""
    import torch
    f64 = torch.float64
    _check(lib().vp_add_log_growth(x.numel(), _ptr(x, f64), _ptr(y, f64), float(A), float(x0[0]), float(x0[1]),
                                   _ptr(out, f64), _stream(x)))
    return out


def neumann_solve(plan, q, bnd_x, bnd_y, bnd_w, pan, u, g, ub=None, tol=1e-12, max_iter=200, restart=50, f=None,
                  jet6=None):
    """Boundary values ub (zero boundary integral) with ub/2 + D[ub] = V[f] + S[g]
    (vp_neumann_solve); u = V[f] + S[g] - D[ub] inside.  Returns (ub, products,
    relative residual)."""
    import torch
    f64 = torch.float64
    n = bnd_x.numel()
    if ub is None:
        ub = torch.zeros(n, dtype=f64, device=g.device)
    it = ctypes.c_int(0)
    res = ctypes.c_double(0.0)
    _check(lib().vp_neumann_solve(plan.handle, n // q, q, _ptr(bnd_x, f64), _ptr(bnd_y, f64), _ptr(bnd_w, f64),
                                  _ptr(pan, torch.int32), _ptr(u, f64), _ptr(g, f64), _ptr(f, f64), _ptr(jet6, f64),
                                  _ptr(ub, f64), tol, max_iter, restart, ctypes.byref(it), ctypes.byref(res)))
    return ub, it.value, res.value


def volume_jets_patch(x, y, f, nbr):
    """As volume_jets, from the least-squares quadratic over each triangle and
    its edge neighbours (vp_volume_jets_patch); nbr [n_tri, 3] int32 device
    tensor, -1 where an edge has no neighbour.  Device tensor [6, n]."""
    import torch
    f64 = torch.float64
    n = x.numel()
    if n % 6:
        raise ValueError("the nodes must come six per triangle")
    if nbr.numel() != 3 * (n // 6):
        raise ValueError("nbr must hold three entries per triangle")
    out = torch.empty((6, n), dtype=f64, device=x.device)
    _check(lib().vp_volume_jets_patch(n // 6, _ptr(x, f64), _ptr(y, f64), _ptr(f, f64), _ptr(nbr, torch.int32),
                                      _ptr(out), _stream(x)))
    return out


def volume_jets(x, y, f):
    """f and its first and second derivatives at the volume nodes (six per
    triangle, stored consecutively) from per-triangle quadratic interpolants
    (vp_volume_jets): device tensor [6, n]."""
    import torch
    f64 = torch.float64
    n = x.numel()
    if n % 6:
        raise ValueError("the nodes must come six per triangle")
    out = torch.empty((6, n), dtype=f64, device=x.device)
    _check(lib().vp_volume_jets(n // 6, _ptr(x, f64), _ptr(y, f64), _ptr(f, f64), _ptr(out), _stream(x)))
    return out
