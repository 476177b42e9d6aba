"""CPU float64 oracle for the layer and volume potential path.

TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check and the benchmark's
CPU-baseline leg may import, call, link or execute anything here; the library
never does, and the two share no code.  It evaluates what the method computes
(history part by direct summation of the split kernel, local part by the
paper's asymptotic expansions) plainly and slowly, and is itself pinned by
tests against closed forms, brute-force quadrature and invariants.

Parity pinned: G_H, K_D, Ein (closed forms, library E1 at 50 digits,
finite-difference normal derivative, time-integral identity), V_L/S_L/D_L
(brute-force quadrature of the local kernels on curved boundaries, residual
O(delta^{5/2})), totals (radial closed forms on the disk, Gauss's identity and
its jump, harmonic-polynomial layer potentials on the circle).
"""
from .potential import delta1_of, evaluate, rel_linf

__all__ = ["evaluate", "delta1_of", "rel_linf"]
