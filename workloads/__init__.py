"""Seeded synthetic inputs for the lattice Boltzmann boundary-scheme engine.

This package produces the *inputs* of the method and nothing else: solid
masks, cut links with their exact wall fractions q (called gamma in the
paper's Section 2) and wall velocities phi, initial distributions drawn from
a seeded generator, and the analytic flow solutions used to measure accuracy.
It holds none of the method's arithmetic (no equilibrium, collision,
streaming or boundary rule), so both the CPU oracle and the HIP engine can
take their inputs from here without sharing any of the computation.
"""

from .velocities import VELOCITIES, opposite
from .geometry import Geometry
from . import geometry, configs, analytic, states

__all__ = ["VELOCITIES", "opposite", "Geometry", "geometry", "configs",
           "analytic", "states"]
