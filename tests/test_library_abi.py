"""The C-ABI library loads on a CPU-only host and exports every declared entry point."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "vp.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(vp_[a-z_]+)\s*\(", text)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_symbols()
    for n in ["vp_plan", "vp_volume", "vp_layer", "vp_destroy", "vp_eval"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2409_11998_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("libvp.so not built")
    L = ctypes.CDLL(binding.LIB_PATH)
    for n in declared_symbols():
        assert hasattr(L, n), n
    assert sorted(binding.EXPORTED) == sorted(declared_symbols())


def test_opts_defaults_without_device():
    from paper_2409_11998_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("libvp.so not built")
    o = binding.default_opts()
    assert o.tol == 1e-10 and o.precision == binding.VP_FP64 and o.c_delta == 3.0
    assert o.delta_ratio == 32.0 and o.kinds == 7


def test_host_side_argument_checks():
    """The binding and the library reject malformed arguments before any device
    work: these run without a GPU."""
    import torch
    from paper_2409_11998_amd import binding, boundary_frame, boundary_jets, volume_jets
    x = torch.zeros(30, dtype=torch.float64)
    with pytest.raises(ValueError):           # 30 nodes are not whole panels of 16
        boundary_frame(x, x, 16, x, x)
    with pytest.raises(ValueError):
        boundary_jets(x, x, 16, x, torch.zeros(30, dtype=torch.int32), x, 4)
    with pytest.raises(ValueError):           # nodes come six per triangle
        volume_jets(torch.zeros(7, dtype=torch.float64), x[:7], x[:7])
    with pytest.raises(ValueError):           # host tensors are refused before the call
        volume_jets(torch.zeros(12, dtype=torch.float64), x[:12], x[:12])
    L = binding.lib()
    assert L.vp_volume_jets(0, None, None, None, None, None) == binding.VP_OK
    assert L.vp_volume_jets(-1, None, None, None, None, None) == binding.VP_ERR_ARG
    assert L.vp_boundary_jets(1, 16, None, None, None, 0, None, None, 4, None, None) == binding.VP_ERR_ARG
    assert L.vp_boundary_jets(4, 40, None, None, None, 0, None, None, 4, None, None) == binding.VP_ERR_ARG
    assert L.vp_dirichlet_solve(None, 4, 16, None, None, None, None, None, None, None, None, 1e-12, 10, 10, None,
                                None) == binding.VP_ERR_ARG
    assert L.vp_neumann_solve(None, 4, 16, None, None, None, None, None, None, None, None, None, 1e-12, 10, 10, None,
                              None) == binding.VP_ERR_ARG
    assert L.vp_exterior_dirichlet_solve_growth(None, 4, 16, None, None, None, None, None, None, 1.0, 0.0, 0.0, None,
                                                1e-12, 10, 10, None, None) == binding.VP_ERR_ARG
    # the growth term: nothing to do for n = 0; negative counts, NULL arrays and
    # non-finite coefficients or centres are rejected before any launch
    inf = float("inf")
    assert L.vp_add_log_growth(0, None, None, 1.0, 0.0, 0.0, None, None) == binding.VP_OK
    assert L.vp_add_log_growth(-1, None, None, 1.0, 0.0, 0.0, None, None) == binding.VP_ERR_ARG
    assert L.vp_add_log_growth(5, None, None, 1.0, 0.0, 0.0, None, None) == binding.VP_ERR_ARG
    buf = (ctypes.c_double * 5)()
    assert L.vp_add_log_growth(5, buf, buf, inf, 0.0, 0.0, buf, None) == binding.VP_ERR_ARG
    assert L.vp_add_log_growth(5, buf, buf, 1.0, float("nan"), 0.0, buf, None) == binding.VP_ERR_ARG


def test_noalloc_limit_matches_header():
    from paper_2409_11998_amd import binding
    text = open(os.path.join(ROOT, "include", "vp.h")).read()
    m = re.search(r"#define\s+VP_NOALLOC_MAX_NODES\s+(\d+)", text)
    assert m and int(m.group(1)) == binding.NOALLOC_MAX_NODES
