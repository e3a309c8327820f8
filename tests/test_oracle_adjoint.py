"""Pins of the oracle's reverse sweep by complex-step differentiation of the
forward oracle (derivatives exact to round-off, independent of the reverse
sweep's hand-derived formulas)."""

import numpy as np
import pytest

from oracle.adjoint import Objective, forward, reverse
from oracle.lbm import Oracle
from workloads import configs, states
from workloads import geometry as G

H = 1e-30


def _cs(make, f0, steps, obj):
    o = make()
    J, _ = forward(o, f0.astype(complex), steps, obj)
    return np.imag(J) / H


def _check(geom, s, kw, obj, steps, n_q=None, seed=0):
    rule = kw.get("l_rule", "min")
    g0 = np.asarray(kw.get("g", (0, 0, 0)), dtype=float)
    base = dict(kw)
    base.pop("g", None)
    o = Oracle(geom, s, g=g0, **base)
    df0 = states.random_deviation(o.Q, o.N, seed=seed, amp=2e-3)
    f0 = o.init_deviation(df0)
    J, st = forward(o, f0, steps, obj)
    r = reverse(o, st, obj, rule=rule)
    assert abs(J) > 0

    def make(q=None, wu=None, g=None, ss=None):
        return lambda: Oracle(geom, s if ss is None else ss,
                              g=g0 if g is None else g,
                              q=q, wall_u=wu, **base)

    rng = np.random.default_rng(seed)
    ks = np.arange(geom.n_links) if n_q is None else rng.choice(geom.n_links, n_q, replace=False)
    for k in ks:
        q = geom.q.astype(complex)
        q[k] += 1j * H
        want = _cs(make(q=q), f0, steps, obj)
        assert np.isclose(r["q"][k], want, rtol=1e-10, atol=1e-18 + 1e-10 * abs(want)), (k, r["q"][k], want)
    for a in range(o.D):
        wu = geom.wall_u.astype(complex)
        k = ks[0]
        wu[k, a] += 1j * H
        want = _cs(make(wu=wu), f0, steps, obj)
        assert np.isclose(r["wall_u"][k, a], want, rtol=1e-10, atol=1e-20)
        g = g0[: o.D].astype(complex)
        g[a] += 1j * H
        want = _cs(make(g=g), f0, steps, obj)
        assert np.isclose(r["g"][a], want, rtol=1e-10, atol=1e-20), (a, r["g"][a], want)
    for k in range(o.Q):
        ss = np.asarray(s, dtype=complex)
        ss[k] += 1j * H
        want = _cs(make(ss=ss), f0, steps, obj)
        assert np.isclose(r["s"][k], want, rtol=1e-9, atol=1e-16), (k, r["s"][k], want)
    # dot-product test on the initial state
    d = states.random_deviation(o.Q, o.N, seed=seed + 100, amp=1.0)
    d[:, ~o.fluid] = 0.0
    want = _cs(lambda: o, f0 + 1j * H * d, steps, obj)
    got = (r["lam0"] * d).sum()
    assert np.isclose(got, want, rtol=1e-10, atol=1e-18)
    return r


def test_drag_gradient_d2q9_periodic():
    geom = G.random_cylinders(22, 17, 2, 2.4, 3.6, seed=6)
    wu = np.zeros_like(geom.wall_u)
    wu[:, 0] = 0.02
    geom = geom.with_wall_u(wu)
    obj = Objective("force_x", tag=1, t0=2, t1=7)
    _check(geom, configs.d2q9_rates(0.7), dict(g=(1e-4, 2e-5, 0), l_rule="gamma2", b=0.9),
           obj, 7, n_q=12)


def test_drag_gradient_outflow_channel():
    geom = G.channel_cylinder(24, 13, 2.7, (9.3, 6.4), 0.04)
    obj = Objective("force_x", tag=1, t0=0, t1=6)
    _check(geom, configs.d2q9_rates(0.6), dict(l_rule="gamma2+gamma"), obj, 6, n_q=10)


def test_mean_ux_gradient_d3q19_seam():
    geom = G.random_spheres(10, 8, 7, 1, 1.8, 2.4, seed=4, x_bc="pressure")
    obj = Objective("mean_ux", t0=1, t1=5)
    _check(geom, configs.d3q19_rates(0.65), dict(g=(2e-5, 0, 1e-5), dp=1e-3, l_rule="gamma"),
           obj, 5, n_q=8)


def test_min_rule_gradient_away_from_the_kink():
    """l = max(0, 2g - 1) has a kink at g = 1/2; elsewhere it is smooth."""
    geom = G.random_cylinders(18, 15, 1, 3.1, 3.1, seed=2)
    keep = np.abs(geom.q - 0.5) > 1e-3
    assert keep.all()
    obj = Objective("force_x", tag=1, t0=0, t1=4)
    _check(geom, configs.d2q9_rates(0.8), dict(l_rule="min"), obj, 4, n_q=8)


def test_two_node_scheme_gradient():
    """Eq. (211): the c1 term reads the advected f_ibar(x_f, t+1)."""
    geom = G.random_cylinders(22, 17, 2, 2.4, 3.6, seed=6)
    wu = np.zeros_like(geom.wall_u)
    wu[:, 1] = 0.015
    geom = geom.with_wall_u(wu)
    obj = Objective("force_x", tag=1, t0=1, t1=6)
    _check(geom, configs.d2q9_rates(0.7),
           dict(g=(1e-4, 0, 0), l_rule="gamma2", b=0.85, two_node=True), obj, 6, n_q=12)


def test_two_node_gradient_seam_d3q19():
    geom = G.random_spheres(10, 8, 7, 1, 1.8, 2.4, seed=4, x_bc="pressure")
    obj = Objective("mean_ux", t0=0, t1=5)
    _check(geom, configs.d3q19_rates(0.65),
           dict(dp=1e-3, l_rule="gamma", two_node=True), obj, 5, n_q=8)


def test_decaying_wall_data_gradient():
    """Wall data phi(x_b, t) = phi(x_b, 0) * lambda^t (the Taylor-Green
    boundary of Section 3.2): gradients with respect to phi(x_b, 0)."""
    geom = G.random_cylinders(22, 17, 2, 2.4, 3.6, seed=6)
    wu = np.zeros_like(geom.wall_u)
    wu[:, 0] = 0.03
    wu[:, 1] = -0.01
    geom = geom.with_wall_u(wu)
    obj = Objective("force_x", tag=1, t0=1, t1=7)
    _check(geom, configs.d2q9_rates(0.7),
           dict(g=(1e-4, 0, 0), l_rule="gamma2", wall_decay=0.93), obj, 7, n_q=10)


# ----------------------------------------------------------------------------
# pressure drop between two cross-sections


def test_pressure_drop_value_is_the_plane_density_difference():
    """J at t = 0 of f = f^eq(rho, u): c_s^2 times the difference of the
    prescribed rho averaged over the fluid nodes of the two planes."""
    geom = G.random_spheres(12, 9, 8, 2, 2.0, 3.0, seed=11, x_bc="pressure")
    rng = np.random.default_rng(3)
    rho = 1.0 + rng.uniform(-1e-2, 1e-2, geom.n_nodes)
    u = rng.uniform(-1e-2, 1e-2, (geom.n_nodes, 3))
    x = np.arange(geom.n_nodes) % 12
    fl = geom.solid == 0
    for planes in [(0, -1), (3, 8), (7, 2)]:
        o = Oracle(geom, configs.d3q19_rates(0.7), dp=1e-3)
        obj = Objective("pressure_drop", t0=0, t1=1, planes=planes)
        J, _ = forward(o, o.init_equilibrium(rho=rho, u=u), 1, obj)
        a, b = planes[0] % 12, planes[1] % 12
        assert (fl & (x == a)).sum() < (x == a).sum() or (fl & (x == b)).sum() < (x == b).sum()
        want = (rho[fl & (x == a)].mean() - rho[fl & (x == b)].mean()) / 3.0
        assert abs(J - want) <= 1e-15, (planes, J, want)


def test_pressure_drop_of_the_seam_driven_channel_is_linear():
    """Steady channel flow driven by a seam jump drho: the pressure falls
    linearly by c_s^2 drho over one period, so between planes a < b the drop
    is c_s^2 drho (b - a) / nx."""
    nx, ny_mesh, drho = 8, 10, 2e-4
    geom = G.build("D2Q9", (nx, ny_mesh + 1, 1),
                   planes=[G.PlaneWall(1, -1, 0, 0.5), G.PlaneWall(1, +1, ny_mesh, ny_mesh - 0.5)],
                   x_bc="pressure")
    o = Oracle(geom, configs.d2q9_rates(0.8), dp=drho, l_rule="min")
    f = o.run(o.init_equilibrium(), 4000)
    for a, b in [(0, nx - 1), (2, 5), (1, 7)]:
        obj = Objective("pressure_drop", t0=0, t1=1, planes=(a, b))
        J = obj.value(o, 0, f, None, None)
        want = drho * (b - a) / nx / 3.0
        assert abs(J - want) < 1e-9 * want, (a, b, J, want)


def test_pressure_drop_gradient_d3q19_seam():
    geom = G.random_spheres(10, 8, 7, 1, 1.8, 2.4, seed=4, x_bc="pressure")
    obj = Objective("pressure_drop", t0=1, t1=6, planes=(2, 7))
    _check(geom, configs.d3q19_rates(0.65), dict(g=(2e-5, 0, 1e-5), dp=1e-3, l_rule="gamma2"),
           obj, 6, n_q=8)


def test_pressure_drop_gradient_outflow_channel():
    geom = G.channel_cylinder(24, 13, 2.7, (9.3, 6.4), 0.04)
    obj = Objective("pressure_drop", t0=0, t1=7, planes=(3, -1))
    _check(geom, configs.d2q9_rates(0.6), dict(l_rule="gamma2+gamma"), obj, 7, n_q=10)


def test_pressure_drop_gradient_two_node_periodic():
    geom = G.random_cylinders(22, 17, 2, 2.4, 3.6, seed=6)
    wu = np.zeros_like(geom.wall_u)
    wu[:, 0] = 0.02
    geom = geom.with_wall_u(wu)
    obj = Objective("pressure_drop", t0=2, t1=7, planes=(1, 12))
    _check(geom, configs.d2q9_rates(0.7), dict(g=(1e-4, 2e-5, 0), l_rule="gamma", two_node=True),
           obj, 7, n_q=12)
