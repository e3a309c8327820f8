"""The paper's Section 3 experiments, run on the GPU through the library.

* Poiseuille flow (Section 3.1): straight walls at distance gamma from the
  nearest fluid row, body force G = 0.8 nu, H = 1, nu = 0.03,
  h = H / (N_y - 2 + 2 gamma), N_x = 2 (N_y - 1).
* Taylor-Green vortex in the disk (x - 1/2)^2 + (y - 1/2)^2 <= 1/16
  (Section 3.2): nu = 0.002, U0 = 0.05, initial and wall data from the
  analytic solution, error at T = 1 / U0.  The wall data decay as
  exp(-8 pi^2 nu t), passed to the library as a per-step factor.
* Hagen-Poiseuille flow in a pipe of radius 1/2 (Section 3.3): force
  G = 0.8 nu, nu = 0.03, D3Q15 with the Section 3 rates (or D3Q19).
* The b family of Eq. (213) near s_nu -> 2 (stability of the convex
  combination).

All use the diffusive scaling dt = eta h^2, eta = (1/s_nu - 1/2) / (3 nu),
and the paper's relative L2 error of the velocity over the fluid nodes.
Small problems leave most of the GPU idle, so each sweep runs its cases
concurrently, one solver per HIP stream; a case at steady state stops.
"""

import math
import time

import numpy as np

from workloads import analytic, configs
from workloads import geometry as G

from . import binding

NU_POISEUILLE = 0.03
NU_TAYLOR_GREEN = 0.002
U0_TAYLOR_GREEN = 0.05


def rates(lattice, s_nu, collision=None):
    if collision in ("bgk", "trt"):
        return binding.collision_rates(lattice, collision, s_nu)
    if lattice == "D2Q9":
        return configs.d2q9_paper_rates(s_nu)
    if lattice == "D3Q15":
        return configs.d3q15_paper_rates(s_nu)
    return configs.d3q19_rates(1.0 / s_nu)


def eta_of(s_nu, nu):
    return (1.0 / s_nu - 0.5) / (3.0 * nu)


class Case:
    """One run: a solver, the analytic velocity (lattice units) at the
    nodes, the fluid mask and bookkeeping for the steady-state loop."""

    def __init__(self, label, solver, ua, fluid, chunk, max_steps, fixed_steps=None):
        self.label, self.sv, self.ua, self.fluid = label, solver, ua, fluid
        self.chunk, self.max_steps, self.fixed_steps = chunk, max_steps, fixed_steps
        self.u_old = None
        self.steps = 0
        self.done = False
        self.error = None
        self.status = "running"


def _finish(case):
    _, u = case.sv.moments()
    if not np.all(np.isfinite(u[case.fluid])):
        case.status, case.error = "unstable", float("nan")
    else:
        case.error = analytic.relative_l2(u, case.ua, case.fluid)
        if case.status == "running":
            case.status = "converged" if case.fixed_steps is None else "done"
    case.done = True
    case.sv.close()


def run_cases(cases, tol=1e-9, streams=8, log=None):
    """Advance every case on its own stream until steady (relative change of
    u over one chunk below tol) or, for fixed_steps cases, to that count."""
    import torch
    pool = [torch.cuda.Stream() for _ in range(min(streams, len(cases)))]
    for k, c in enumerate(cases):
        c.sv.set_stream(pool[k % len(pool)])
    t0 = time.time()
    active = list(cases)
    while active:
        for c in active:
            n = c.chunk if c.fixed_steps is None else min(c.chunk, c.fixed_steps - c.steps)
            c.sv.step(n)
            c.steps += n
        still = []
        for c in active:
            if c.fixed_steps is not None:
                if c.steps >= c.fixed_steps:
                    _finish(c)
                else:
                    still.append(c)
                continue
            _, u = c.sv.moments()
            uf = u[c.fluid]
            if not np.all(np.isfinite(uf)):
                c.status = "unstable"
                _finish(c)
                continue
            if c.u_old is not None:
                du = np.max(np.abs(uf - c.u_old))
                if du <= tol * max(np.max(np.abs(uf)), 1e-300):
                    _finish(c)
                    continue
            if c.steps >= c.max_steps:
                c.status = "max_steps"
                _finish(c)
                continue
            c.u_old = uf.copy()
            still.append(c)
        active = still
        if log:
            log("%d/%d cases running, %.0f s" % (len(active), len(cases), time.time() - t0))
    torch.cuda.synchronize()
    return cases


def _chunk(diffusive_steps):
    return int(max(512, min(200_000, 0.02 * diffusive_steps)) // 64 * 64)


# ----------------------------------------------------------------------------
# Section 3.1


def poiseuille_case(ny_mesh, gamma, s_nu, rule, lattice="D2Q9", collision=None, b=1.0,
                    two_node=False, precision="fp64"):
    nu = NU_POISEUILLE
    h = 1.0 / (ny_mesh - 2 + 2 * gamma)
    dt = eta_of(s_nu, nu) * h * h
    g_lat = 0.8 * nu * dt * dt / h
    nz = 1 if lattice == "D2Q9" else 2
    geom = G.poiseuille_channel(ny_mesh, gamma, nx=2 * (ny_mesh - 1), lattice=lattice, nz=nz)
    sv = binding.solver_for(geom, rates(lattice, s_nu, collision), g=(g_lat, 0, 0),
                            precision=precision, l_rule=rule, b=b, two_node=two_node)
    H = geom.meta["H"]
    nu_lat = (1.0 / s_nu - 0.5) / 3.0
    U = g_lat * H * H / (8 * nu_lat)
    _, y, _ = geom.coords()
    D = 2 if lattice == "D2Q9" else 3
    ua = np.zeros((geom.n_nodes, D))
    ua[:, 0] = analytic.poiseuille_u(y.astype(float), U, geom.meta["y_lo"], H)
    sv.init(u=ua)
    diff = H * H / nu_lat
    label = dict(test="poiseuille", lattice=lattice, rule=rule, gamma=gamma, s_nu=s_nu,
                 ny=ny_mesh, h=h, collision=collision or "mrt", b=b, two_node=two_node)
    return Case(label, sv, ua, geom.solid == 0, _chunk(diff), int(6 * diff) + 10_000)


# ----------------------------------------------------------------------------
# Section 3.2


def taylor_green_velocity(xp, yp, t):
    """Analytic (u, v) in physical units at positions xp, yp and time t."""
    dec = math.exp(-8.0 * math.pi ** 2 * NU_TAYLOR_GREEN * t)
    u = -U0_TAYLOR_GREEN * np.cos(2 * np.pi * xp) * np.sin(2 * np.pi * yp) * dec
    v = U0_TAYLOR_GREEN * np.cos(2 * np.pi * yp) * np.sin(2 * np.pi * xp) * dec
    return u, v


def taylor_green_case(inv_h, s_nu, rule, b=1.0, two_node=False, precision="fp64"):
    nu = NU_TAYLOR_GREEN
    h = 1.0 / inv_h
    dt = eta_of(s_nu, nu) * h * h
    vel = dt / h                                   # physical -> lattice velocity
    pad = 2
    n = int(math.ceil(0.5 / h)) + 2 * pad + 1
    # lattice node (i, j) sits at x = 1/2 + (i - c) h; c off the grid's own
    # symmetry lines so that no node lies exactly on the circle
    c = ((n - 1) / 2.0 + 0.137, (n - 1) / 2.0 - 0.211)
    wall = G.HollowBall((c[0], c[1], 0.0), 0.25 / h, axes=(0, 1), tag=0)
    geom = G.build("D2Q9", (n, n, 1), hollows=[wall])
    # wall data at x_b = x_f - q e_i, at t = 0
    e = binding.lattice_info("D2Q9")[0]
    xf, yf, _ = geom.coords()
    xb = xf[geom.node] - geom.q * e[geom.dir, 0]
    yb = yf[geom.node] - geom.q * e[geom.dir, 1]
    ub, vb = taylor_green_velocity(0.5 + (xb - c[0]) * h, 0.5 + (yb - c[1]) * h, 0.0)
    geom = geom.with_wall_u(np.stack([ub, vb], 1) * vel)
    sv = binding.solver_for(geom, rates("D2Q9", s_nu), precision=precision, l_rule=rule,
                            b=b, two_node=two_node)
    sv.set_wall_decay(math.exp(-8.0 * math.pi ** 2 * nu * dt))
    xp, yp = 0.5 + (xf - c[0]) * h, 0.5 + (yf - c[1]) * h
    u0, v0 = taylor_green_velocity(xp, yp, 0.0)
    dp = -0.25 * U0_TAYLOR_GREEN ** 2 * (np.cos(4 * np.pi * xp) + np.cos(4 * np.pi * yp))
    rho = 1.0 + 3.0 * dp * vel * vel               # p - p0 = c_s^2 (rho - rho0)
    sv.init(rho=rho, u=np.stack([u0, v0], 1) * vel)
    T = 1.0 / U0_TAYLOR_GREEN
    steps = int(round(T / dt))
    uT, vT = taylor_green_velocity(xp, yp, steps * dt)
    ua = np.stack([uT, vT], 1) * vel
    label = dict(test="taylor_green", rule=rule, s_nu=s_nu, inv_h=inv_h, h=h, b=b,
                 two_node=two_node, steps=steps, u0_lattice=U0_TAYLOR_GREEN * vel)
    chunk = max(64, min(steps, 100_000))
    return Case(label, sv, ua, geom.solid == 0, chunk, steps, fixed_steps=steps)


# ----------------------------------------------------------------------------
# Section 3.3


def hagen_poiseuille_case(inv_h, s_nu, rule, lattice="D3Q15", b=1.0, precision="fp64"):
    nu = NU_POISEUILLE
    h = 1.0 / inv_h
    dt = eta_of(s_nu, nu) * h * h
    g_lat = 0.8 * nu * dt * dt / h
    R = 0.5 / h
    geom = G.pipe(R, nx=2, lattice=lattice)
    sv = binding.solver_for(geom, rates(lattice, s_nu), g=(g_lat, 0, 0), precision=precision,
                            l_rule=rule, b=b)
    nu_lat = (1.0 / s_nu - 0.5) / 3.0
    _, y, z = geom.coords()
    cen = geom.meta["center"]
    r = np.sqrt((y - cen[1]) ** 2 + (z - cen[2]) ** 2)
    ua = np.zeros((geom.n_nodes, 3))
    ua[:, 0] = analytic.hagen_poiseuille_u(r, g_lat * R * R / (4 * nu_lat), R)
    sv.init(u=ua)
    diff = R * R / nu_lat
    label = dict(test="hagen_poiseuille", lattice=lattice, rule=rule, s_nu=s_nu, inv_h=inv_h,
                 h=h, b=b)
    return Case(label, sv, ua, geom.solid == 0, _chunk(diff), int(6 * diff) + 10_000)


# ----------------------------------------------------------------------------


def fitted_order(hs, errs):
    hs, errs = np.asarray(hs, float), np.asarray(errs, float)
    ok = np.isfinite(errs) & (errs > 0)
    if ok.sum() < 2:
        return float("nan")
    return float(np.polyfit(np.log(hs[ok]), np.log(errs[ok]), 1)[0])


def summarize(cases, key_fields, size_field="h"):
    """Group finished cases by key_fields and fit the order over h."""
    groups = {}
    for c in cases:
        key = tuple(c.label[k] for k in key_fields)
        groups.setdefault(key, []).append(c)
    out = []
    for key, cs in sorted(groups.items(), key=lambda kv: str(kv[0])):
        cs = sorted(cs, key=lambda c: -c.label[size_field])
        hs = [c.label[size_field] for c in cs]
        errs = [c.error for c in cs]
        out.append(dict(zip(key_fields, key), h=hs, errors=errs,
                        steps=[c.steps for c in cs], status=[c.status for c in cs],
                        order=fitted_order(hs, errs)))
    return out


RULES = ["gamma", "1.5gamma", "2gamma", "gamma2", "gamma2+gamma"]
S_NUS = [0.5, 1.0, 1.5, 1.99]


def poiseuille_study(rules=RULES, gammas=(0.25, 0.75, 1.0), s_nus=S_NUS,
                     sizes=(11, 21, 41, 61, 81), tol=1e-8, log=None, max_size_by_snu=None,
                     **kw):
    """max_size_by_snu: optional {s_nu: largest N_y} (the steady state takes
    ~ H^2 / nu steps, 7e6 at N_y = 81 and s_nu = 1.99)."""
    lim = max_size_by_snu or {}
    cases = [poiseuille_case(n, g, s, r, **kw) for r in rules for g in gammas for s in s_nus
             for n in sizes if n <= lim.get(s, n)]
    run_cases(cases, tol=tol, log=log)
    return summarize(cases, ["rule", "gamma", "s_nu", "collision", "b", "two_node"])


def taylor_green_study(rules=RULES, s_nus=S_NUS, inv_hs=(40, 80, 120, 160, 200), log=None, **kw):
    cases = [taylor_green_case(n, s, r, **kw) for r in rules for s in s_nus for n in inv_hs]
    run_cases(cases, log=log)
    return summarize(cases, ["rule", "s_nu", "b", "two_node"])


def hagen_poiseuille_study(rules=RULES, s_nus=S_NUS, inv_hs=(10, 20, 40, 80), lattice="D3Q15",
                           tol=1e-8, log=None, max_size_by_snu=None, **kw):
    lim = max_size_by_snu or {}
    cases = [hagen_poiseuille_case(n, s, r, lattice=lattice, **kw) for r in rules for s in s_nus
             for n in inv_hs if n <= lim.get(s, n)]
    run_cases(cases, tol=tol, log=log)
    return summarize(cases, ["lattice", "rule", "s_nu", "b"])


def b_study(bs=(1.0, 0.9, 0.7, 0.5), s_nus=(1.99, 1.995, 1.999), rules=("gamma", "2gamma"),
            sizes=(11, 21), gamma=0.75, tol=1e-8, log=None, collision=None):
    """Eq. (213) with b < 1 near s_nu -> 2: stability and error of the
    Poiseuille test."""
    cases = [poiseuille_case(n, gamma, s, r, b=bb, collision=collision) for bb in bs
             for s in s_nus for r in rules for n in sizes]
    run_cases(cases, tol=tol, log=log)
    return summarize(cases, ["rule", "gamma", "s_nu", "collision", "b", "two_node"])
