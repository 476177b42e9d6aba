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
