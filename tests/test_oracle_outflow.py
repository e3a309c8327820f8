"""Pins of the oracle's zero-gradient outflow reading.

Reading (outflow x boundary of the channel workload): column x = 0 is a
solid inlet wall, and at x = nx-1 a population moving in -x, whose source
x = nx would lie outside the domain, is read from (nx-1, y - e_y, z - e_z):
the post-collision field is continued with zero x-gradient.  The paper has
no outlet, so nothing it prints fixes this; three consequences that the
definition of a zero-gradient outlet fixes on its own are checked instead:

* a uniform flow f^eq(rho0, u_in) with an inlet wall moving at u_in is an
  exact fixed point (Eq. (42) with the single-node scheme Eq. (213) is
  consistent for any l and gamma: with f = f' = f^eq the link value is
  f^eq_ibar + 6 w_i rho0 e_i.u = f^eq_i), and the outlet must not disturb it;
* an x-invariant flow is continued exactly by a zero-gradient outlet, so away
  from the inlet (beyond the one node per step its influence travels) the
  outflow run equals the same channel run periodic in x;
* mass bookkeeping per step: the collision conserves mass at every node, a
  post-collision population is either advected to a fluid node, stopped by a
  wall (and replaced by the link value of Eq. (213)) or, moving in +x at
  x = nx-1, lost through the outlet, and the outlet adds a copy of each -x
  population of column nx-1; so the mass change is (link values) - (stopped
  populations) + (outlet copies) - (outlet losses), exactly.
"""

import numpy as np
import pytest

from oracle import lattice as L
from oracle.lbm import Oracle
from workloads import configs, states
from workloads import geometry as G


def _inlet_channel(lattice, shape, u_in, inlet_plane=0.5, walls=None):
    """Column x = 0 solid with a wall plane at x = inlet_plane moving at
    (u_in, 0, 0); optional resting y walls (planes at walls[0] and walls[1]);
    zero-gradient outflow at x = nx-1."""
    nx, ny, nz = shape
    planes = []
    if walls is not None:
        planes += [G.PlaneWall(1, -1, 0, walls[0], tag=0),
                   G.PlaneWall(1, +1, ny - 1, walls[1], tag=0)]
    planes.append(G.PlaneWall(0, -1, 0, inlet_plane, tag=2, velocity=(u_in, 0.0, 0.0)))
    return G.build(lattice, shape, planes=planes, x_bc="outflow")


def _rates(lattice, tau):
    return configs.d2q9_rates(tau) if lattice == "D2Q9" else configs.d3q19_rates(tau)


@pytest.mark.parametrize("lattice,shape", [("D2Q9", (14, 7, 1)), ("D3Q19", (11, 5, 4))])
@pytest.mark.parametrize("rule,plane", [("min", 0.5), ("gamma", 0.3), ("gamma2+gamma", 0.8)])
def test_uniform_inflow_is_a_fixed_point(lattice, shape, rule, plane):
    u_in = 0.04
    geom = _inlet_channel(lattice, shape, u_in, inlet_plane=plane)
    o = Oracle(geom, _rates(lattice, 0.6), l_rule=rule, deviation=False)
    u = np.zeros((o.N, o.D))
    u[:, 0] = u_in
    f0 = o.init_equilibrium(u=u)
    f = o.run(f0, 40)
    fl = o.fluid
    assert np.all(np.isfinite(f[:, fl]))
    assert np.abs(f[:, fl] - f0[:, fl]).max() <= 2e-16


@pytest.mark.parametrize("lattice,shape,walls", [
    ("D2Q9", (16, 9, 1), (0.5, 9 - 1.5)),
    ("D2Q9", (16, 9, 1), (0.7, 9 - 1.2)),
    ("D3Q19", (12, 7, 3), (0.6, 7 - 1.35)),
])
def test_x_invariant_flow_matches_the_periodic_channel(lattice, shape, walls):
    nx, ny, nz = shape
    steps = 6
    out = _inlet_channel(lattice, shape, 0.03, walls=walls)
    per = G.build(lattice, shape, planes=[G.PlaneWall(1, -1, 0, walls[0], tag=0),
                                          G.PlaneWall(1, +1, ny - 1, walls[1], tag=0)])
    lat = L.get(lattice)
    # random deviations that depend on (i, y, z) only
    col = states.random_deviation(lat.Q, ny * nz, seed=17, amp=2e-3).reshape(lat.Q, nz, ny, 1)
    df0 = np.broadcast_to(col, (lat.Q, nz, ny, nx)).reshape(lat.Q, -1).copy()
    kw = dict(g=(2e-5, 0, 0), l_rule="gamma2", deviation=False)
    oo = Oracle(out, _rates(lattice, 0.7), **kw)
    op = Oracle(per, _rates(lattice, 0.7), **kw)
    fo = oo.run(oo.init_deviation(df0), steps)
    fp = op.run(op.init_deviation(df0), steps)
    fo = fo.reshape(lat.Q, nz, ny, nx)
    fp = fp.reshape(lat.Q, nz, ny, nx)
    keep = slice(steps + 1, nx)            # beyond the inlet's reach
    a, b = fo[..., keep], fp[..., keep]
    m = ~np.isnan(b)
    assert np.array_equal(np.isnan(a), np.isnan(b))
    assert np.abs(a[m] - b[m]).max() <= 1e-16
    # the comparison covers the outlet column itself
    assert np.all(np.isfinite(fo[:, :, 1:-1, nx - 1]))


@pytest.mark.parametrize("lattice,shape", [("D2Q9", (13, 8, 1)), ("D3Q19", (9, 5, 4))])
@pytest.mark.parametrize("rule,plane", [("min", 0.5), ("gamma", 0.35)])
def test_mass_balance_through_the_outlet(lattice, shape, rule, plane):
    """y (and z) periodic, only the inlet wall, random (not x-invariant)
    state: the per-step mass change is accounted for exactly."""
    nx = shape[0]
    geom = _inlet_channel(lattice, shape, 0.05, inlet_plane=plane)
    lat = L.get(lattice)
    o = Oracle(geom, _rates(lattice, 0.65), g=(1e-5, 2e-6, 0), l_rule=rule, deviation=False)
    f = o.init_deviation(states.random_deviation(lat.Q, o.N, seed=23, amp=3e-3))
    x = np.arange(o.N) % nx
    outlet = (x == nx - 1) & o.fluid
    ex = o.e[:, 0]
    for _ in range(6):
        m0 = o.mass(f)
        fn, fp = o.step(f)
        # Eq. (213) values of the inlet links, and the populations f'_ibar(x_f)
        # that the inlet wall stops
        xf, i, ib = o.lk_node, o.lk_dir, o.lk_opp
        c0, c1, c2, c3, c4 = o.c
        link_in = (c0 * f[i, xf] + c1 * f[ib, xf] + c2 * fp[i, xf] + c3 * fp[ib, xf]
                   + c4 * o.wall_term).sum()
        link_out = fp[ib, xf].sum()
        dup = fp[ex < 0][:, outlet].sum()
        lost = fp[ex > 0][:, outlet].sum()
        want = m0 + link_in - link_out + dup - lost
        assert abs(o.mass(fn) - want) <= 1e-13 * abs(m0)
        f = fn
