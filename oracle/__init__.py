"""Plain, slow CPU oracle of the single-node boundary-scheme LBM step.

TEST INFRASTRUCTURE ONLY.  Only the tests, the package smoke check and the
benchmark's CPU-baseline leg may import this package; the HIP engine never
calls it and shares no code, table or helper with it.

What it computes (Zhao & Yong, "A family of single-node second-order
boundary schemes for the lattice Boltzmann method"):

* lattice.py   velocity sets, weights and moment matrices (Appendix; D3Q19
               from the d'Humieres et al. 2002 moment polynomials).
* scheme.py    the free parameter l(gamma), the convexity band Eq. (212)
               and the coefficients of Eq. (210) / Eq. (213).
* lbm.py       one time step in the paper's order: MRT collision (Appendix,
               equilibrium Eq. (42)), advection Eq. (22b), then Eq. (213)
               on every cut link; moments, mass, momentum and the
               momentum-exchange force.
* adjoint.py   the reverse sweep of that step (a discrete adjoint derived
               here; pinned by complex-step differentiation of lbm.py).

Everything is float64 (or complex128 for complex-step checks), vectorised
over nodes with numpy and otherwise unoptimised.  Parity status of each
function is stated in its docstring; the FP32 comparison is "parity
unpinned" (the error against this oracle is reported, not asserted).
"""

from . import lattice, scheme, lbm, adjoint

__all__ = ["lattice", "scheme", "lbm", "adjoint"]
