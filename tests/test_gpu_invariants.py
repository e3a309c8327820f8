"""Invariants of the step on the GPU (the oracle has the same pins):
the rest state is a fixed point for every rule and gamma, an integer
translation of a periodic problem translates the result bit for bit, and a
90-degree rotation of a D2Q9 problem with s_qx = s_qy rotates the result."""

import numpy as np
import pytest

from gpu_util import require_gpu
from workloads import configs, states
from workloads import geometry as G

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("rule", ["gamma", "1.5gamma", "2gamma", "gamma2", "gamma2+gamma", "min"])
def test_rest_state_is_exactly_preserved(rule, precision):
    from paper_1712_08288_amd import binding
    for geom, s in ((G.random_cylinders(50, 37, 3, 3.0, 6.0, seed=4), configs.d2q9_rates(0.7)),
                    (G.random_spheres(24, 18, 16, 2, 2.5, 4.0, seed=6, x_bc="pressure"),
                     configs.d3q19_rates(0.8))):
        sv = binding.solver_for(geom, s, precision=precision, l_rule=rule, b=0.9)
        sv.init()
        sv.step(70)
        df = sv.distribution()
        assert np.all(df[:, geom.solid == 0] == 0.0)
        sv.close()


def _shift(geom, dx, dy):
    """The same periodic cylinder problem translated by (dx, dy) nodes."""
    nx, ny, _ = geom.shape
    x, y, _ = geom.coords()
    newn = (x + dx) % nx + nx * ((y + dy) % ny)
    solid = np.empty_like(geom.solid)
    solid[newn] = geom.solid
    node = newn[geom.node]
    return G.Geometry(geom.lattice, geom.shape, solid, node, geom.dir, geom.q,
                      geom.wall_u, geom.tag, geom.x_bc, dict(geom.meta)), newn


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_integer_translation_is_bitwise(precision):
    from paper_1712_08288_amd import binding
    geom = G.random_cylinders(70, 45, 3, 4.0, 7.0, seed=31)
    geom2, newn = _shift(geom, 23, 11)
    s = configs.d2q9_rates(0.62)
    df0 = states.random_deviation(9, geom.n_nodes, seed=2, amp=1e-3)
    df2 = np.empty_like(df0)
    df2[:, newn] = df0
    out = []
    for g, d in ((geom, df0), (geom2, df2)):
        sv = binding.solver_for(g, s, precision=precision, g=(1e-5, 2e-6, 0), l_rule="gamma2")
        sv.init_deviation(d)
        sv.step(40)
        out.append(sv.distribution())
        sv.close()
    fl = geom.solid == 0
    assert np.array_equal(out[1][:, newn][:, fl], out[0][:, fl])


def test_quarter_turn_rotates_the_result():
    """D2Q9 with s_qx = s_qy: rotating geometry, initial state and force by
    90 degrees rotates the velocity field (to round-off: the pair form sums
    the directions in a different order after rotation)."""
    from paper_1712_08288_amd import binding
    n = 48
    geom = G.random_cylinders(n, n, 3, 3.0, 6.0, seed=9)
    e = binding.lattice_info("D2Q9")[0]
    # rotation (x, y) -> (n-1-y, x); velocities e -> (-e_y, e_x)
    rot_dir = np.array([int(np.nonzero((e[:, 0] == -e[i, 1]) & (e[:, 1] == e[i, 0]))[0][0])
                        for i in range(9)])
    x, y, _ = geom.coords()
    newn = (n - 1 - y) + n * x
    solid = np.empty_like(geom.solid)
    solid[newn] = geom.solid
    geom2 = G.Geometry("D2Q9", geom.shape, solid, newn[geom.node], rot_dir[geom.dir], geom.q,
                       geom.wall_u, geom.tag, geom.x_bc, dict(geom.meta))
    s = configs.d2q9_paper_rates(1.3)
    df0 = states.random_deviation(9, geom.n_nodes, seed=5, amp=1e-3)
    df2 = np.empty_like(df0)
    df2[rot_dir[:, None], newn[None, :]] = df0
    gvec = np.array([1e-5, 3e-6])
    res = []
    for gm, d, gg in ((geom, df0, gvec), (geom2, df2, np.array([-gvec[1], gvec[0]]))):
        sv = binding.solver_for(gm, s, g=(gg[0], gg[1], 0), l_rule="gamma")
        sv.init_deviation(d)
        sv.step(30)
        res.append(sv.moments()[1])
        sv.close()
    u, u2 = res
    fl = geom.solid == 0
    ur = np.stack([-u[:, 1], u[:, 0]], 1)
    assert np.max(np.abs(u2[newn][fl] - ur[fl])) < 1e-14 * np.max(np.abs(u[fl])) + 1e-19
