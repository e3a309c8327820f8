"""Oracle against the paper's analytic flows: second-order convergence of the
relative L2 velocity error (Section 3: Poiseuille Eq. (52)-(53), 3D
Hagen-Poiseuille) and circular Couette flow, plus the pressure-jump seam
reproducing the equivalent body-force flow."""

import numpy as np
import pytest

from oracle.lbm import Oracle
from workloads import analytic, configs
from workloads import geometry as G


def run_steady(o, f, chunk=200, tol=1e-9, max_steps=200_000):
    u_old = o.velocity(f)
    steps = 0
    while steps < max_steps:
        f = o.run(f, chunk)
        steps += chunk
        u = o.velocity(f)
        fl = o.fluid
        du = np.nanmax(np.abs(u[:, fl] - u_old[:, fl]))
        if du <= tol * np.nanmax(np.abs(u[:, fl])):
            return f, steps
        u_old = u
    raise AssertionError("no steady state")


def poiseuille_error(ny_mesh, gamma, s_nu, rule, nu=0.03, lattice="D2Q9", two_node=False,
                     collision=None):
    """Paper Section 3.1: h = H/(N_y - 2 + 2 gamma), dt = eta h^2 with
    eta = (1/s_nu - 1/2)/(3 nu); body force G = 0.8 nu, H = 1.  In lattice
    units the force is G dt^2 / h."""
    h = 1.0 / (ny_mesh - 2 + 2 * gamma)
    eta = (1.0 / s_nu - 0.5) / (3.0 * nu)
    dt = eta * h * h
    G_lat = 0.8 * nu * dt * dt / h
    geom = G.poiseuille_channel(ny_mesh, gamma, nx=2, lattice=lattice,
                                nz=1 if lattice == "D2Q9" else 2)
    s = configs.d2q9_paper_rates(s_nu) if lattice == "D2Q9" else configs.d3q19_rates(1.0 / s_nu)
    o = Oracle(geom, s, g=(G_lat, 0, 0), l_rule=rule, two_node=two_node, collision=collision)
    x, y, z = geom.coords()
    H = geom.meta["H"]
    nu_lat = (1.0 / s_nu - 0.5) / 3.0
    U = G_lat * H * H / (8 * nu_lat)
    ua = np.zeros((o.N, o.D))
    ua[:, 0] = analytic.poiseuille_u(y.astype(float), U, geom.meta["y_lo"], H)
    f, _ = run_steady(o, o.init_equilibrium(u=ua))
    _, u = o.macroscopic(f)
    return analytic.relative_l2(u, ua, o.fluid)


def order(sizes, errs):
    return -np.polyfit(np.log(sizes), np.log(errs), 1)[0]


@pytest.mark.parametrize("rule", ["gamma", "1.5gamma", "2gamma", "gamma2",
                                  "gamma2+gamma", "min"])
@pytest.mark.parametrize("gamma", [0.25, 0.75, 1.0])
def test_poiseuille_second_order(rule, gamma):
    """Section 3.1 reports orders close to 2 for every rule, gamma and s_nu."""
    sizes = [11, 21, 41]
    errs = [poiseuille_error(n, gamma, 1.0, rule) for n in sizes]
    p = order([n - 2 + 2 * gamma for n in sizes], errs)
    assert 1.85 < p < 2.15, (errs, p)


@pytest.mark.parametrize("rule", ["gamma", "2gamma", "gamma2"])
@pytest.mark.parametrize("gamma", [0.25, 1.0])
def test_two_node_scheme_second_order(rule, gamma):
    """Eq. (211) (Remark (2)) is second order too; with l = gamma it is the
    scheme of Remark (4) attributed to Yu, Mei and Shyy."""
    sizes = [11, 21, 41]
    errs = [poiseuille_error(n, gamma, 1.0, rule, two_node=True) for n in sizes]
    p = order([n - 2 + 2 * gamma for n in sizes], errs)
    assert 1.85 < p < 2.15, (errs, p)


@pytest.mark.parametrize("s_nu", [0.5, 1.5])
def test_poiseuille_second_order_other_rates(s_nu):
    sizes = [11, 21, 41]
    errs = [poiseuille_error(n, 0.75, s_nu, "gamma2") for n in sizes]
    assert 1.8 < order([n - 0.5 for n in sizes], errs) < 2.2, errs


def test_poiseuille_half_way_bounce_back_is_small_and_second_order():
    """At gamma = 1/2 with l(1/2) = 0 the walls are half-way bounce-back,
    which is exact for plane Poiseuille flow with this forcing up to the
    rate-dependent slip; the error must be small and still second order."""
    errs = [poiseuille_error(n, 0.5, 1.0, "min") for n in (11, 21, 41)]
    assert errs[-1] < 1e-2
    assert order([10, 20, 40], errs) > 1.8


@pytest.mark.parametrize("rule", ["gamma", "min"])
def test_couette_second_order(rule):
    errs, sizes = [], [32, 48, 64]
    for n in sizes:
        w = configs.c1_couette(n)
        geom = w.geometry()
        o = Oracle(geom, w.s, l_rule=rule)
        f = o.run(o.init_equilibrium(), w.steps)
        _, u = o.macroscopic(f)
        errs.append(analytic.relative_l2(u, analytic.couette_velocity(geom),
                                         geom.solid == 0))
    p = order(sizes, errs)
    assert 1.6 < p < 2.8, (errs, p)
    assert errs[-1] < 2e-3


@pytest.mark.parametrize("lattice", ["D3Q19", "D3Q15"])
def test_hagen_poiseuille_second_order(lattice):
    """Section 3.3: pipe of radius R along x, force G, the analytic
    u = U(1 - r^2/R^2), U = G R^2/(4 nu); D3Q15 with the Section 3 rates
    (the paper's own 3D test), D3Q19 with the d'Humieres et al. rates."""
    errs, radii = [], [4.0, 8.0, 16.0]
    for R in radii:
        geom = G.pipe(R, nx=1, lattice=lattice)
        s_nu = 1.0
        nu = (1 / s_nu - 0.5) / 3
        Gf = 1e-6
        rates = configs.d3q19_rates(1 / s_nu) if lattice == "D3Q19" else configs.d3q15_paper_rates(s_nu)
        o = Oracle(geom, rates, g=(Gf, 0, 0), l_rule="gamma2")
        x, y, z = geom.coords()
        c = geom.meta["center"]
        r = np.sqrt((y - c[1]) ** 2 + (z - c[2]) ** 2)
        ua = np.zeros((o.N, 3))
        ua[:, 0] = analytic.hagen_poiseuille_u(r, Gf * R * R / (4 * nu), R)
        f, _ = run_steady(o, o.init_equilibrium(u=ua), chunk=100, tol=1e-9)
        _, u = o.macroscopic(f)
        errs.append(analytic.relative_l2(u, ua, o.fluid))
    p = order(radii, errs)
    assert 1.6 < p < 2.6, (errs, p)


def pressure_channel_error(ny_mesh, gamma=0.5, nx=4, s_nu=1.0, nu=0.03):
    h = 1.0 / (ny_mesh - 2 + 2 * gamma)
    eta = (1.0 / s_nu - 0.5) / (3.0 * nu)
    dt = eta * h * h
    G_lat = 0.8 * nu * dt * dt / h
    drho = 3.0 * nx * G_lat            # c_s^2 drho / nx = G
    geom = G.build("D2Q9", (nx, ny_mesh + 1, 1),
                   planes=[G.PlaneWall(1, -1, 0, 1 - gamma),
                           G.PlaneWall(1, +1, ny_mesh, ny_mesh - 1 + gamma)],
                   x_bc="pressure")
    o = Oracle(geom, configs.d2q9_paper_rates(s_nu), dp=drho, l_rule="gamma2")
    x, y, z = geom.coords()
    H = ny_mesh - 2 + 2 * gamma
    U = G_lat * H * H / (8 * (1.0 / s_nu - 0.5) / 3.0)
    ua = np.zeros((o.N, 2))
    ua[:, 0] = analytic.poiseuille_u(y.astype(float), U, 1 - gamma, H)
    f, _ = run_steady(o, o.init_equilibrium(u=ua))
    rho, u = o.macroscopic(f)
    rr = rho.reshape(ny_mesh + 1, nx)[ny_mesh // 2]
    slope = np.polyfit(np.arange(nx), rr, 1)[0]
    return analytic.relative_l2(u, ua, o.fluid), slope * nx / drho, u[o.fluid, 0]


def test_pressure_seam_drives_poiseuille_flow():
    """A density jump drho at the periodic x seam acts as the pressure
    gradient c_s^2 drho / nx: the channel flow converges at second order to
    the Poiseuille profile with G = c_s^2 drho / (nx rho0), the density falls
    linearly by drho over one period, and the flow runs towards +x."""
    res = [pressure_channel_error(n) for n in (11, 21, 41)]
    errs = [r[0] for r in res]
    assert 1.8 < order([10, 20, 40], errs) < 2.2, errs
    for _, slope, ux in res:
        assert abs(slope + 1.0) < 1e-3
        assert np.all(ux > 0)
