"""Seeded synthetic inputs for the layer/volume potential path.

This package only builds inputs: meshes, quadrature nodes and weights,
densities, and the per-target boundary geometry and density jets that the
local (small-delta) part of the method takes as given (the paper treats the
closest-point computation as a geometry preprocessing step, Sec. 2.2).  It
holds none of the method's arithmetic and is shared by the oracle, the tests
and the benchmark.
"""
from .problems import (Problem, disk_problem, square_problem, star_problem,
                       circle_layer_problem, config_problem, star_params)

__all__ = ["Problem", "disk_problem", "square_problem", "star_problem",
           "circle_layer_problem", "config_problem", "star_params"]
