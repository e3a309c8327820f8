"""Pins of the oracle's whole step: a brute-force loop implementation on tiny
grids, exact invariants (rest state, half-way bounce-back mass, momentum
bookkeeping, symmetry, translation) and the deviation form."""

import numpy as np
import pytest

from oracle import lattice as L
from oracle import scheme as S
from oracle.lbm import Oracle
from workloads import geometry as G
from workloads import configs, states
from workloads.velocities import opposite


# ----------------------------------------------------------------------------
# brute force: plain nested loops over nodes and directions, absolute f


def brute_step(geom, s, rho0, g, rule, b, dp, f, two_node=False):
    """One step written node by node from Eq. (22a), the Appendix MRT
    collision with Eq. (42), Eq. (22b) and Eq. (213).  f: dict node -> list."""
    lat = L.get(geom.lattice)
    Q, D = lat.Q, lat.D
    e = [tuple(int(c) for c in v) for v in lat.e]
    w = list(lat.w)
    M = lat.M.tolist()
    norm = [sum(M[k][j] ** 2 for j in range(Q)) for k in range(Q)]
    opp = [e.index(tuple(-c for c in v)) for v in e]
    nx, ny, nz = geom.shape
    fluid = [geom.solid[n] == 0 for n in range(nx * ny * nz)]
    gg = list(g)[:D] + [0.0] * (3 - D)

    fp = {}
    for n, fn_ in f.items():
        rho = sum(fn_)
        u = [sum(e[i][a] * fn_[i] for i in range(Q)) / rho0 for a in range(D)]
        uu = sum(c * c for c in u)
        feq = []
        for i in range(Q):
            eu = sum(e[i][a] * u[a] for a in range(D))
            feq.append(w[i] * (rho + rho0 * (3 * eu + 4.5 * eu * eu - 1.5 * uu)))
        m = [sum(M[k][j] * (fn_[j] - feq[j]) for j in range(Q)) for k in range(Q)]
        out = []
        for i in range(Q):
            # M^{-1} = M^T diag(1/norm) for orthogonal rows
            relax = sum(M[k][i] / norm[k] * s[k] * m[k] for k in range(Q))
            force = 3 * w[i] * rho0 * sum(e[i][a] * gg[a] for a in range(D))
            out.append(fn_[i] - relax + force)
        fp[n] = out

    links = {}
    for k in range(geom.n_links):
        links[(int(geom.node[k]), int(geom.dir[k]))] = k

    def streamed(n, i):
        x, y, z = n % nx, (n // nx) % ny, n // (nx * ny)
        ex = e[i][0]
        ey = e[i][1]
        ez = e[i][2] if D == 3 else 0
        sx = x - ex
        jump = 0.0
        if geom.x_bc == "outflow":
            sx = min(max(sx, 0), nx - 1)
        else:
            if geom.x_bc == "pressure":
                jump = w[i] * dp if sx < 0 else (-w[i] * dp if sx >= nx else 0.0)
            sx %= nx
        src = sx + nx * (((y - ey) % ny) + ny * ((z - ez) % nz))
        assert fluid[src], "pull from a solid node without a link"
        return fp[src][i] + jump

    new = {}
    for n in f:
        vals = []
        for i in range(Q):
            if (n, i) in links:
                k = links[(n, i)]
                gam = float(geom.q[k])
                l = float(S.l_of_gamma(rule, gam))
                c0 = 1 - b
                c1 = b * (1 + l - 2 * gam) / (1 + l)
                c2 = b * l / (1 + l)
                c3 = b * (2 * gam - l) / (1 + l)
                c4 = b * 2 / (1 + l)
                phi = [float(v) for v in geom.wall_u[k]]
                wall = 3 * w[i] * rho0 * sum(e[i][a] * phi[a] for a in range(D))
                ib = opp[i]
                f_ib = f[n][ib]
                if two_node and (n, ib) not in links:
                    f_ib = streamed(n, ib)      # f'_ibar(x_f + e_i, t), Eq. (211)
                vals.append(c0 * f[n][i] + c1 * f_ib + c2 * fp[n][i]
                            + c3 * fp[n][ib] + c4 * wall)
                continue
            vals.append(streamed(n, i))
        new[n] = vals
    return new


def _tiny_cases():
    yield "cyl2d", G.random_cylinders(13, 11, 2, 2.2, 3.1, seed=4), \
        configs.d2q9_rates(0.7) + np.array([0.3, 0, 0, 0.2, 0, 0.1, 0, 0, 0]), \
        (2e-4, -1e-4, 0), 0.0, "gamma2"
    box = G.build("D2Q9", (9, 8, 1),
                  balls=[G.Balls([[4.3, 3.6, 0]], [2.3], tag=1, omega=[0.01])],
                  x_bc="pressure")
    yield "seam2d", box, configs.d2q9_paper_rates(1.3, literal=True), \
        (0, 0, 0), 1e-3, "1.5gamma"
    yield "outflow2d", G.channel_cylinder(14, 9, 1.7, (6.2, 4.4), 0.03), \
        configs.d2q9_rates(0.56), (0, 0, 0), 0.0, "min"
    yield "sph3d", G.random_spheres(7, 6, 5, 1, 1.6, 1.9, seed=9, x_bc="pressure"), \
        configs.d3q19_rates(0.65), (1e-4, 0, 2e-5), 2e-3, "gamma"


@pytest.mark.parametrize("two_node", [False, True], ids=["eq210", "eq211"])
@pytest.mark.parametrize("case", list(_tiny_cases()), ids=lambda c: c[0])
def test_oracle_matches_brute_force(case, two_node):
    name, geom, s, g, dp, rule = case
    lat = L.get(geom.lattice)
    o = Oracle(geom, s, rho0=1.0, g=g, dp=dp, l_rule=rule, b=0.9, deviation=False,
               two_node=two_node)
    df = states.random_deviation(lat.Q, o.N, seed=3, amp=2e-3)
    f = o.init_deviation(df)
    fb = {n: list(f[:, n]) for n in range(o.N) if o.fluid[n]}
    for _ in range(3):
        f, _ = o.step(f)
        fb = brute_step(geom, s, 1.0, g, rule, 0.9, dp, fb, two_node=two_node)
    got = np.array([f[:, n] for n in sorted(fb)])
    want = np.array([fb[n] for n in sorted(fb)])
    assert np.all(np.isfinite(got))
    assert np.allclose(got, want, atol=1e-15, rtol=1e-13)


# ----------------------------------------------------------------------------
# invariants


@pytest.mark.parametrize("rule", S.RULES[:5] + ("min",))
def test_rest_state_is_preserved(rule):
    geom = G.random_cylinders(40, 36, 4, 3.0, 6.0, seed=21)
    o = Oracle(geom, configs.d2q9_rates(0.6), l_rule=rule, deviation=False)
    f0 = o.init_equilibrium()
    f = o.run(f0, 60)
    fl = o.fluid
    assert np.abs(f[:, fl] - f0[:, fl]).max() <= 4e-16


def test_half_way_bounce_back_box_conserves_mass():
    geom = G.closed_box(12, 10)
    assert np.all(geom.q == 0.5)
    o = Oracle(geom, configs.d2q9_rates(0.7), l_rule="min", deviation=False)
    f = o.init_deviation(states.random_deviation(9, o.N, seed=5, amp=1e-2))
    m0 = o.mass(f)
    f = o.run(f, 300)
    assert abs(o.mass(f) - m0) / m0 < 1e-14


def test_general_gamma_mass_drift_is_reported_not_zero():
    """Outside half-way bounce-back the scheme is not mass conserving: the
    per-link change c1 f_ibar + c2 f'_i - (c1 + c2) f'_ibar is nonzero."""
    geom = G.closed_box(12, 10)
    o = Oracle(geom, configs.d2q9_rates(0.7), l_rule="gamma", deviation=False)
    f = o.init_deviation(states.random_deviation(9, o.N, seed=5, amp=1e-2))
    m0 = o.mass(f)
    f = o.run(f, 300)
    assert abs(o.mass(f) - m0) / m0 > 1e-8


@pytest.mark.parametrize("g", [(0, 0, 0), (3e-5, -2e-5, 0)])
def test_momentum_bookkeeping(g):
    """Fluid momentum after a step = before + rho0 g N_f - sum of the
    momentum-exchange forces (exact per step on a periodic domain)."""
    geom = G.random_cylinders(30, 26, 3, 3.0, 5.0, seed=8)
    o = Oracle(geom, configs.d2q9_rates(0.8), g=g, l_rule="gamma2+gamma",
               deviation=False)
    geom_u = np.zeros_like(geom.wall_u)
    geom_u[:, 0] = 0.01
    o2 = Oracle(geom.with_wall_u(geom_u), configs.d2q9_rates(0.8), g=g,
                l_rule="gamma2+gamma", deviation=False)
    for oo in (o, o2):
        f = oo.init_deviation(states.random_deviation(9, oo.N, seed=2, amp=1e-3))
        for _ in range(5):
            p0 = oo.momentum(f)
            fn, fp = oo.step(f)
            p1 = oo.momentum(fn)
            force = oo.force(fp, fn).sum(0)
            want = p0 + 1.0 * np.asarray(g)[:2] * oo.fluid.sum() - force
            assert np.allclose(p1, want, atol=1e-14)
            f = fn


def test_translation_invariance():
    a = G.build("D2Q9", (24, 20, 1), balls=[G.Balls([[7.3, 8.6, 0], [17.2, 14.1, 0]], [3.4, 2.7])])
    b = G.build("D2Q9", (24, 20, 1), balls=[G.Balls([[7.3 + 5, 8.6 + 3, 0], [17.2 + 5, 14.1 + 3, 0]], [3.4, 2.7])])
    s = configs.d2q9_rates(0.7)
    oa = Oracle(a, s, g=(1e-4, 0, 0))
    ob = Oracle(b, s, g=(1e-4, 0, 0))
    fa = oa.run(oa.init_equilibrium(), 80)
    fb = ob.run(ob.init_equilibrium(), 80)
    fa = fa.reshape(9, 20, 24)
    fb = fb.reshape(9, 20, 24)
    shifted = np.roll(np.roll(fa, 3, axis=1), 5, axis=2)
    m = ~np.isnan(shifted)
    assert np.array_equal(np.isnan(shifted), np.isnan(fb))
    assert np.allclose(shifted[m], fb[m], atol=1e-18, rtol=1e-13)


def test_mirror_symmetry_d2q9():
    """Reflecting y maps the solution onto itself with u_y negated when the
    rates treat x and y alike (s_qx = s_qy)."""
    ny = 21
    c = [[8.3, 6.6, 0.0]]
    a = G.build("D2Q9", (26, ny, 1), balls=[G.Balls(c, [3.1])])
    b = G.build("D2Q9", (26, ny, 1), balls=[G.Balls([[8.3, ny - 1 - 6.6, 0.0]], [3.1])])
    s = configs.d2q9_rates(0.7)
    oa, ob = Oracle(a, s, g=(1e-4, 0, 0)), Oracle(b, s, g=(1e-4, 0, 0))
    ra, ua = oa.macroscopic(oa.run(oa.init_equilibrium(), 120))
    rb, ub = ob.macroscopic(ob.run(ob.init_equilibrium(), 120))
    ua = ua.reshape(ny, 26, 2)
    ub = ub.reshape(ny, 26, 2)[::-1]
    m = ~np.isnan(ua[..., 0])
    assert np.allclose(ua[m][:, 0], ub[m][:, 0], atol=1e-17, rtol=1e-11)
    assert np.allclose(ua[m][:, 1], -ub[m][:, 1], atol=1e-17, rtol=1e-11)


def test_deviation_form_equals_plain_form():
    w = configs.c1_couette(32, steps=600)
    geom = w.geometry()
    od = Oracle(geom, w.s, deviation=True)
    op = Oracle(geom, w.s, deviation=False)
    rd, ud = od.macroscopic(od.run(od.init_equilibrium(), w.steps))
    rp, up = op.macroscopic(op.run(op.init_equilibrium(), w.steps))
    fl = geom.solid == 0
    err = np.sqrt(((ud - up)[fl] ** 2).sum() / (up[fl] ** 2).sum())
    assert err < 1e-13
    assert np.abs(rd - rp)[fl].max() < 1e-14


def test_uncovered_solid_pull_is_rejected():
    geom = G.random_cylinders(20, 20, 1, 3.0, 4.0, seed=1)
    bad = G.Geometry(geom.lattice, geom.shape, geom.solid, geom.node[1:],
                     geom.dir[1:], geom.q[1:], geom.wall_u[1:], geom.tag[1:])
    with pytest.raises(ValueError):
        Oracle(bad, configs.d2q9_rates(0.7))


@pytest.mark.parametrize("xbc", ["periodic", "pressure", "outflow"])
def test_window_mode_matches_full_domain(xbc):
    """The sampled-window evaluation used for full-size parity equals the
    full-domain run at the window centres."""
    from oracle.lbm import sampled_step_outputs
    if xbc == "outflow":
        geom = G.channel_cylinder(40, 21, 4.3, (15.2, 10.4), 0.03)
    else:
        geom = G.build("D3Q19", (17, 14, 12),
                       balls=[G.Balls([[5.2, 6.1, 4.3], [12.6, 3.3, 8.8]], [3.1, 2.6])],
                       x_bc=xbc)
    lat = L.get(geom.lattice)
    s = configs.d3q19_rates(0.7) if lat.Q == 19 else configs.d2q9_rates(0.7)
    df0 = states.random_deviation(lat.Q, geom.n_nodes, seed=12)
    kw = dict(g=(1e-5, 2e-6, 0), dp=1e-3, l_rule="gamma2")
    o = Oracle(geom, s, **kw)
    full = o.as_deviation(o.run(o.init_deviation(df0), 3))
    fluid = np.nonzero(geom.solid == 0)[0]
    rng = np.random.default_rng(0)
    samples = np.sort(rng.choice(fluid, 12, replace=False))
    # include nodes on the x seam / outlet column
    nx = geom.shape[0]
    edge = fluid[(fluid % nx == nx - 1) | (fluid % nx == 1)][:4]
    samples = np.unique(np.concatenate([samples, edge]))
    got = sampled_step_outputs(geom, s, df0, 3, samples, **kw)
    assert np.all(np.isfinite(got))
    assert np.allclose(got, full[:, samples], atol=1e-18, rtol=1e-12)
