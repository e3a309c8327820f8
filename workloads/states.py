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


def outlet_consistent(df, shape, velocities):
    """Copy, for every population moving in -x, the initial value of column
    nx-2 into column nx-1.  A zero-gradient outlet reads those populations
    from the neighbouring column, so an initial state given with the outflow
    x boundary must already satisfy this to be representable exactly."""
    nx, ny, nz = shape
    out = np.array(df, copy=True)
    cols = out.reshape(out.shape[0], nz, ny, nx)
    for i, e in enumerate(velocities):
        if e[0] == -1:
            cols[i, :, :, nx - 1] = cols[i, :, :, nx - 2]
    return out
