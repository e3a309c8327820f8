"""MI355X lattice Boltzmann engine with the Zhao-Yong single-node boundary
scheme (fused pull MRT collide-stream, cut-link boundary, hand-written
adjoint).  The compute path is the HIP library built from csrc/; the Python
layer only marshals arguments.

    from paper_1712_08288_amd import binding
    sv = binding.solver_for(geom, s, precision="fp32")
"""
