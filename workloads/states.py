"""Seeded initial values.

The engine and the oracle both accept either macroscopic fields (rho, u),
from which each computes its own equilibrium, or raw distributions given as
deviations from the rest state (delta f_i = f_i - w_i rho0).  The generators
below only draw numbers; they compute nothing of the method.
"""

import numpy as np


def random_fields(n_nodes, D, seed, rho_amp=1e-3, u_amp=1e-2, rho0=1.0):
    """rho ~ rho0 + U(-rho_amp, rho_amp), u ~ U(-u_amp, u_amp)^D per node."""
    rng = np.random.default_rng(seed)
    rho = rho0 + rng.uniform(-rho_amp, rho_amp, size=n_nodes)
    u = rng.uniform(-u_amp, u_amp, size=(n_nodes, D))
    return rho, u


def random_deviation(Q, n_nodes, seed, amp=1e-3):
    """Distribution deviations delta f ~ U(-amp, amp), shape (Q, N), so that
    the state has a non-equilibrium part for the collision to relax."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-amp, amp, size=(Q, n_nodes))
