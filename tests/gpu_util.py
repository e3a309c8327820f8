"""Shared helpers of the GPU tests: running the HIP engine and the oracle on
the same seeded inputs and comparing them."""

import numpy as np

from oracle.lbm import Oracle
from workloads import states
from workloads.velocities import VELOCITIES


def require_gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU (run with -m 'not gpu' on CPU)"
    torch.cuda.set_device(0)


def rel_l2(a, b, mask=None):
    if mask is not None:
        a, b = a[..., mask], b[..., mask]
    return float(np.sqrt(((a - b) ** 2).sum() / max((b ** 2).sum(), 1e-300)))


def pair(geom, s, steps, precision="fp64", init="deviation", seed=1, amp=1e-3,
         g=None, dp=0.0, l_rule="min", b=1.0, rho0=1.0, fields=None, two_node=False):
    """Run `steps` steps on the GPU and on the oracle from the same seeded
    initial state; return (gpu deviations, oracle deviations, fluid mask,
    solver, oracle, oracle state)."""
    from paper_1712_08288_amd import binding
    Q = len(VELOCITIES[geom.lattice])
    sv = binding.solver_for(geom, s, rho0=rho0, g=g, precision=precision,
                            l_rule=l_rule, b=b, dp=dp, two_node=two_node)
    o = Oracle(geom, s, rho0=rho0, g=g, dp=dp, l_rule=l_rule, b=b, two_node=two_node)
    if init == "deviation":
        df0 = states.random_deviation(Q, geom.n_nodes, seed=seed, amp=amp)
        sv.init_deviation(df0)
        f = o.init_deviation(df0)
    elif init == "fields":
        rho, u = fields
        sv.init(rho, u)
        f = o.init_equilibrium(rho, u)
    else:
        sv.init()
        f = o.init_equilibrium()
    sv.step(steps)
    f = o.run(f, steps)
    return sv.distribution(), o.as_deviation(f), geom.solid == 0, sv, o, f
