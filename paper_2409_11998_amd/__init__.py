"""MI355X-native layer and volume potentials (heat-kernel split, Fourier history + local asymptotics).

The computation lives in libvp.so (C ABI in include/vp.h, HIP kernels for
gfx950); this package is its Python binding.
"""
from .binding import (VP_FP32, VP_FP64, VP_KIND_D, VP_KIND_S, VP_KIND_V, Batch, Plan,  # noqa: F401
                      Server, VPError, boundary_frame, boundary_jets, default_opts, dirichlet_solve,
                      exterior_dirichlet_solve, exterior_dirichlet_solve_growth, add_log_growth, lib,
                      neumann_solve, volume_jets, volume_jets_patch)

__all__ = ["Plan", "Batch", "Server", "VPError", "VP_FP32", "VP_FP64", "VP_KIND_V", "VP_KIND_S", "VP_KIND_D", "lib",
           "default_opts", "boundary_frame", "boundary_jets", "dirichlet_solve", "exterior_dirichlet_solve",
           "exterior_dirichlet_solve_growth", "add_log_growth", "neumann_solve", "volume_jets", "volume_jets_patch"]
