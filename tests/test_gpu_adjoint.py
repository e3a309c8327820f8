"""HIP adjoint against the oracle's reverse sweep and against central finite
differences of the HIP forward run (GPU).

Tolerances.  FP64 adjoint vs the oracle reverse sweep: both in double with
different summation orders; 1e-10 relative (the required figure).  Central
differences with step 1e-6 in FP64: truncation O(h^2 J''') ~ 1e-12 and
cancellation eps |J| / h ~ 1e-10 |J|, compared on links whose |dJ/dq| is
not tiny against |J|; bound 1e-6 relative (the required figure).
FP32: the forward is FP32, so its gradient differs from the FP64 one by the
FP32 forward error; reported against a 1e-3 relative bound (parity unpinned).
"""

import numpy as np
import pytest

from gpu_util import require_gpu
from oracle.adjoint import Objective, forward, reverse
from oracle.lbm import Oracle
from workloads import configs, states
from workloads import geometry as G
from workloads.velocities import VELOCITIES

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _gpu_grad(geom, s, kw, obj, steps, every, df0, precision="fp64", rates=True):
    """rates=False turns the rate gradients off; with the single-node scheme
    the reverse sweep then reads recorded velocities instead of the forward
    populations."""
    from paper_1712_08288_amd import binding
    sv = binding.solver_for(geom, s, precision=precision, g=kw.get("g"),
                            dp=kw.get("dp", 0.0), l_rule=kw.get("l_rule", "min"),
                            b=kw.get("b", 1.0), two_node=kw.get("two_node", False))
    if kw.get("wall_decay", 1.0) != 1.0:
        sv.set_wall_decay(kw["wall_decay"])
    if not rates:
        sv.set_rate_gradient(False)
    sv.init_deviation(df0)
    sv.set_objective(obj.kind, obj.tag, obj.t0, obj.t1, planes=obj.planes)
    sv.run_checkpointed(steps, every)
    J = sv.objective()
    sv.adjoint()
    gr = sv.grad()
    gr["lam0"] = sv.get_adjoint()
    return sv, J, gr


def _moving_channel():
    """D3Q19 channel whose wall rows give waves of more than 64 cut links
    (the links past the 64th of a wave take the direct path) and moving walls
    (non-zero wall-velocity gradients)."""
    geom = G.poiseuille_channel(9, 0.7, nx=24, lattice="D3Q19", nz=5)
    return geom.with_wall_u(np.tile([0.02, 0.0, -0.01], (geom.n_links, 1)))


CASES = [
    ("d2q9_drag_periodic", lambda: G.random_cylinders(40, 29, 2, 3.1, 5.2, seed=6),
     lambda: configs.d2q9_rates(0.7), dict(g=(1e-4, 2e-5, 0), l_rule="gamma2", b=0.9),
     Objective("force_x", tag=1, t0=3, t1=12), 12),
    ("d2q9_drag_outflow", lambda: G.channel_cylinder(48, 25, 4.2, (16.3, 12.4), 0.04),
     lambda: configs.d2q9_rates(0.6), dict(l_rule="gamma2+gamma"),
     Objective("force_x", tag=1, t0=0, t1=10), 10),
    ("d3q19_meanux_seam", lambda: G.random_spheres(20, 14, 12, 2, 2.2, 3.4, seed=4, x_bc="pressure"),
     lambda: configs.d3q19_rates(0.65), dict(g=(2e-5, 0, 1e-5), dp=1e-3, l_rule="gamma"),
     Objective("mean_ux", t0=2, t1=8), 8),
    ("d2q9_drag_two_node", lambda: G.random_cylinders(40, 29, 2, 3.1, 5.2, seed=6),
     lambda: configs.d2q9_rates(0.7), dict(g=(1e-4, 2e-5, 0), l_rule="gamma2", b=0.9, two_node=True),
     Objective("force_x", tag=1, t0=3, t1=12), 12),
    ("d3q19_meanux_two_node_seam", lambda: G.random_spheres(20, 14, 12, 2, 2.2, 3.4, seed=4, x_bc="pressure"),
     lambda: configs.d3q19_rates(0.65), dict(dp=1e-3, l_rule="gamma", two_node=True),
     Objective("mean_ux", t0=0, t1=8), 8),
    ("d2q9_drag_decaying_walls", lambda: G.random_cylinders(40, 29, 2, 3.1, 5.2, seed=6).with_wall_u(
        np.tile([0.03, -0.01], (G.random_cylinders(40, 29, 2, 3.1, 5.2, seed=6).n_links, 1))),
     lambda: configs.d2q9_rates(0.7), dict(g=(1e-4, 0, 0), l_rule="gamma2", wall_decay=0.95),
     Objective("force_x", tag=1, t0=2, t1=12), 12),
    ("d3q15_meanux_seam", lambda: G.random_spheres(20, 14, 12, 2, 2.2, 3.4, seed=4, x_bc="pressure",
                                                    lattice="D3Q15"),
     lambda: configs.d3q15_paper_rates(1.3), dict(g=(2e-5, 1e-5, 0), dp=1e-3, l_rule="gamma2"),
     Objective("mean_ux", t0=1, t1=8), 8),
    ("d3q19_meanux_channel_many_links", _moving_channel,
     lambda: configs.d3q19_rates(0.8), dict(g=(1e-5, 0, 2e-6), l_rule="gamma2", b=0.95),
     Objective("mean_ux", t0=1, t1=7), 7),
    ("d3q19_meanux_no_links", lambda: G.build("D3Q19", (24, 10, 6)),
     lambda: configs.d3q19_rates(0.75), dict(g=(3e-5, -1e-5, 2e-5)),
     Objective("mean_ux", t0=0, t1=6), 6),
    ("d3q15_drag_periodic_two_node", lambda: G.random_spheres(18, 15, 13, 2, 2.4, 3.6, seed=11,
                                                              lattice="D3Q15"),
     lambda: configs.d3q15_paper_rates(1.1), dict(g=(3e-5, 0, 0), l_rule="1.5gamma", b=0.95,
                                                   two_node=True),
     Objective("force_x", tag=1, t0=2, t1=9), 9),
    ("d3q19_pdrop_seam", lambda: G.random_spheres(22, 14, 12, 2, 2.2, 3.4, seed=4, x_bc="pressure"),
     lambda: configs.d3q19_rates(0.7), dict(dp=1e-3, l_rule="min"),
     Objective("pressure_drop", t0=1, t1=9, planes=(0, -1)), 9),
    ("d3q19_pdrop_seam_rows", lambda: G.random_spheres(64, 9, 8, 2, 2.2, 3.4, seed=14, x_bc="pressure"),
     lambda: configs.d3q19_rates(0.65), dict(g=(1e-5, 0, 0), dp=1e-3, l_rule="gamma2"),
     Objective("pressure_drop", t0=0, t1=7, planes=(5, 40)), 7),
    ("d3q19_meanux_rows256_seam", lambda: G.random_spheres(256, 8, 8, 6, 1.6, 2.9, seed=19,
                                                           x_bc="pressure"),
     lambda: configs.d3q19_rates(0.7), dict(dp=1e-3, g=(1e-5, 0, 2e-6), l_rule="gamma2"),
     Objective("mean_ux", t0=2, t1=20), 20),
    ("d2q9_pdrop_outflow", lambda: G.channel_cylinder(48, 25, 4.2, (16.3, 12.4), 0.04),
     lambda: configs.d2q9_rates(0.6), dict(l_rule="gamma2+gamma"),
     Objective("pressure_drop", t0=2, t1=10, planes=(3, -1)), 10),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_adjoint_matches_oracle_reverse(case):
    name, mk_geom, mk_s, kw, obj, steps = case
    geom, s = mk_geom(), mk_s()
    print("case", name, flush=True)
    Q = len(VELOCITIES[geom.lattice])
    df0 = states.random_deviation(Q, geom.n_nodes, seed=3, amp=2e-3)
    if geom.x_bc == "outflow":
        df0 = states.outlet_consistent(df0, geom.shape, VELOCITIES[geom.lattice])
    base = dict(kw)
    g0 = base.pop("g", None)
    o = Oracle(geom, s, g=g0, **base)
    J_o, st = forward(o, o.init_deviation(df0), steps, obj)
    r = reverse(o, st, obj)
    sv, J, gr = _gpu_grad(geom, s, kw, obj, steps, 4, df0)
    assert abs(J - J_o) <= 1e-12 * abs(J_o) + 1e-18
    fl = geom.solid == 0
    for key in ("q", "wall_u", "g"):
        a, b = gr[key], r[key]
        assert a.shape == b.shape, key
        if b.size == 0:      # no cut links
            continue
        scale = max(np.abs(b).max(), 1e-300)
        assert np.abs(a - b).max() <= 1e-10 * scale, (key, np.abs(a - b).max(), scale)
    # dJ/ds is exactly zero when no wall breaks the momentum balance (the
    # case without links): an absolute floor far below any real gradient
    ds_scale = np.abs(r["s"]).max()
    assert np.abs(gr["s"] - r["s"]).max() <= 1e-10 * ds_scale + 1e-18
    lam_scale = np.abs(r["lam0"][:, fl]).max()
    assert np.abs(gr["lam0"][:, fl] - r["lam0"][:, fl]).max() <= 1e-10 * lam_scale
    sv.close()


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_velocity_mode_matches_oracle_reverse(case):
    """Rate gradients off: the reverse sweep reads the step records the
    forward steps wrote (velocity, link values; with Eq. (211) also the
    advected f_ibar of the next step) instead of the forward states.  Against
    the oracle's reverse sweep at 1e-10, against the state-reading sweep
    of the same run (the same arithmetic on the same values), and with every
    step recorded bit for bit against the run checkpointed every 3 steps."""
    name, mk_geom, mk_s, kw, obj, steps = case
    geom, s = mk_geom(), mk_s()
    print("case", name, flush=True)
    Q = len(VELOCITIES[geom.lattice])
    df0 = states.random_deviation(Q, geom.n_nodes, seed=3, amp=2e-3)
    if geom.x_bc == "outflow":
        df0 = states.outlet_consistent(df0, geom.shape, VELOCITIES[geom.lattice])
    base = dict(kw)
    g0 = base.pop("g", None)
    o = Oracle(geom, s, g=g0, **base)
    J_o, st = forward(o, o.init_deviation(df0), steps, obj)
    r = reverse(o, st, obj)
    sv, J, gu = _gpu_grad(geom, s, kw, obj, steps, 3, df0, rates=False)
    sv.close()
    sv, J2, gf = _gpu_grad(geom, s, kw, obj, steps, 3, df0)
    sv.close()
    assert J == J2
    # every step recorded: the link terms of up to eight steps are summed at
    # once instead of three, in the same order, so the result is the same bits
    sv, J1, g1 = _gpu_grad(geom, s, kw, obj, steps, 1, df0, rates=False)
    sv.close()
    assert J1 == J
    for key in ("q", "wall_u", "g", "lam0"):
        assert np.array_equal(g1[key], gu[key]), key
    fl = geom.solid == 0
    for key in ("q", "wall_u", "g"):
        if r[key].size == 0:
            continue
        scale = max(np.abs(r[key]).max(), 1e-300)
        assert np.abs(gu[key] - r[key]).max() <= 1e-10 * scale, key
        assert np.abs(gu[key] - gf[key]).max() <= 1e-14 * scale, key
    lam_scale = np.abs(r["lam0"][:, fl]).max()
    assert np.abs(gu["lam0"][:, fl] - r["lam0"][:, fl]).max() <= 1e-10 * lam_scale
    assert np.abs(gu["lam0"][:, fl] - gf["lam0"][:, fl]).max() <= 1e-14 * lam_scale
    assert np.all(gu["s"] == 0.0)


@pytest.mark.parametrize("case_name", ["d3q19_pdrop_seam", "d3q19_meanux_two_node_seam"])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_velocity_mode_is_independent_of_the_checkpoints(precision, case_name):
    """Records written at segment ends (checkpointed run) and by the replay
    (other steps) cover every step for any interval -- with Eq. (211) also
    the next step's f_ibar across segment ends and at the run's end -- and
    the sweep in uneven pieces equals the whole sweep, bit for bit."""
    from paper_1712_08288_amd import binding
    name, mk_geom, mk_s, kw, obj, steps = [c for c in CASES if c[0] == case_name][0]
    geom, s = mk_geom(), mk_s()
    df0 = states.random_deviation(19, geom.n_nodes, seed=6, amp=2e-3)
    out = []
    for every in (1, 2, 4, steps, steps + 3):
        sv, J, gr = _gpu_grad(geom, s, kw, obj, steps, every, df0, precision=precision, rates=False)
        out.append((J, gr))
        sv.close()
    for J, gr in out[1:]:
        assert J == out[0][0]
        for key in ("q", "wall_u", "g", "lam0"):
            assert np.array_equal(gr[key], out[0][1][key]), key
    sv = binding.solver_for(geom, s, precision=precision, g=kw.get("g"), dp=kw.get("dp", 0.0),
                            l_rule=kw.get("l_rule", "min"), b=kw.get("b", 1.0),
                            two_node=kw.get("two_node", False))
    sv.set_rate_gradient(False)
    sv.init_deviation(df0)
    sv.set_objective(obj.kind, obj.tag, obj.t0, obj.t1, planes=obj.planes)
    sv.run_checkpointed(steps, 4)
    for piece in (3, 1, 2, steps):
        sv.adjoint_step(piece)
    gr = sv.grad()
    gr["lam0"] = sv.get_adjoint()
    for key in ("q", "wall_u", "g", "lam0"):
        assert np.array_equal(gr[key], out[0][1][key]), key
    sv.close()


def test_record_only_run_needs_velocity_mode_at_the_sweep():
    """A run with one step per segment in velocity mode keeps step records
    and no snapshot: a sweep after switching the rate gradients on has no
    state to read and fails with ESTATE; a new run then sweeps normally."""
    from paper_1712_08288_amd import binding
    name, mk_geom, mk_s, kw, obj, steps = [c for c in CASES if c[0] == "d3q19_pdrop_seam"][0]
    geom, s = mk_geom(), mk_s()
    df0 = states.random_deviation(19, geom.n_nodes, seed=6, amp=2e-3)
    sv0, _, want = _gpu_grad(geom, s, kw, obj, steps, 4, df0)
    sv0.close()
    sv = binding.solver_for(geom, s, precision="fp64", dp=kw["dp"], l_rule=kw["l_rule"])
    sv.set_rate_gradient(False)
    sv.init_deviation(df0)
    sv.set_objective(obj.kind, obj.tag, obj.t0, obj.t1, planes=obj.planes)
    sv.run_checkpointed(steps, 1)
    sv.set_rate_gradient(True)
    with pytest.raises(binding.LBMError) as ex:
        sv.adjoint()
    assert ex.value.name == "ESTATE"
    sv.init_deviation(df0)
    sv.set_objective(obj.kind, obj.tag, obj.t0, obj.t1, planes=obj.planes)
    sv.run_checkpointed(steps, 1)
    sv.adjoint()
    gr = sv.grad()
    for key in ("q", "wall_u", "g", "s"):
        scale = max(np.abs(want[key]).max(), 1e-300)
        assert np.abs(gr[key] - want[key]).max() <= 1e-14 * scale, key
    sv.close()


def test_checkpoint_interval_does_not_change_the_gradient():
    name, mk_geom, mk_s, kw, obj, steps = CASES[0]
    geom, s = mk_geom(), mk_s()
    df0 = states.random_deviation(9, geom.n_nodes, seed=5, amp=2e-3)
    out = []
    for every in (1, 3, 5, steps, 10 ** 6):   # an interval past the run: one segment
        sv, J, gr = _gpu_grad(geom, s, kw, obj, steps, every, df0)
        out.append((J, gr))
        sv.close()
    for J, gr in out[1:]:
        assert J == out[0][0]
        for key in ("q", "wall_u", "g", "s", "lam0"):
            assert np.array_equal(gr[key], out[0][1][key]), key


def test_adjoint_against_central_differences():
    from paper_1712_08288_amd import binding
    name, mk_geom, mk_s, kw, obj, steps = CASES[1]
    geom, s = mk_geom(), mk_s()
    df0 = np.zeros((9, geom.n_nodes))
    sv, J, gr = _gpu_grad(geom, s, kw, obj, steps, 5, df0)
    h = 1e-6

    def J_at(q=None, wall_u=None, g=None, ss=None):
        sv.update_links(q if q is not None else geom.q,
                        wall_u if wall_u is not None else geom.wall_u)
        sv.set_parameters(ss if ss is not None else s, g if g is not None else (0, 0))
        sv.init_deviation(df0)
        sv.set_objective(obj.kind, obj.tag, obj.t0, obj.t1)
        sv.step(steps)
        return sv.objective()

    order = np.argsort(-np.abs(gr["q"]))[:6]
    for k in order:
        qp, qm = geom.q.copy(), geom.q.copy()
        qp[k] += h if geom.q[k] + h <= 1 else 0
        qm[k] -= h
        fd = (J_at(q=qp) - J_at(q=qm)) / (qp[k] - qm[k])
        assert abs(fd - gr["q"][k]) <= 1e-6 * abs(gr["q"][k]), (k, fd, gr["q"][k])
    # inflow velocity: sum over the inlet links (tag 2) of dJ/dphi_x
    inlet = geom.tag == 2
    up, um = geom.wall_u.copy(), geom.wall_u.copy()
    up[inlet, 0] += h
    um[inlet, 0] -= h
    fd = (J_at(wall_u=up) - J_at(wall_u=um)) / (2 * h)
    dui = gr["wall_u"][inlet, 0].sum()
    assert abs(fd - dui) <= 1e-6 * abs(dui), (fd, dui)
    # viscous rate s_nu (rows 7, 8 together), i.e. tau
    sp, sm = s.copy(), s.copy()
    sp[7:9] += h
    sm[7:9] -= h
    fd = (J_at(ss=sp) - J_at(ss=sm)) / (2 * h)
    dsn = gr["s"][7] + gr["s"][8]
    assert abs(fd - dsn) <= 1e-6 * abs(dsn), (fd, dsn)
    sv.close()


def test_pressure_drop_gradient_against_central_differences():
    """C3-like case (D3Q19 sphere packing, pressure seam drho = 1e-3,
    tau = 0.7): dJ/dgamma of the largest links, dJ/dg and dJ/dtau of the
    pressure drop between the first and last cross-section."""
    geom = G.random_spheres(32, 20, 18, 3, 3.0, 4.5, seed=3, x_bc="pressure")
    s = configs.d3q19_rates(0.7)
    obj = Objective("pressure_drop", t0=4, t1=16, planes=(0, -1))
    steps = 16
    df0 = np.zeros((19, geom.n_nodes))
    kw = dict(dp=1e-3, l_rule="gamma2", g=(1e-5, 0, 0))
    sv, J, gr = _gpu_grad(geom, s, kw, obj, steps, 4, df0)
    assert abs(J) > 0
    h = 1e-6
    g0 = np.array([1e-5, 0.0, 0.0])

    def J_at(q=None, g=None, ss=None):
        sv.update_links(q if q is not None else geom.q, geom.wall_u)
        sv.set_parameters(ss if ss is not None else s, g if g is not None else g0)
        sv.init_deviation(df0)
        sv.set_objective(obj.kind, 0, obj.t0, obj.t1, planes=obj.planes)
        sv.step(steps)
        return sv.objective()

    for k in np.argsort(-np.abs(gr["q"]))[:4]:
        qp, qm = geom.q.copy(), geom.q.copy()
        qp[k] += h if geom.q[k] + h <= 1 else 0
        qm[k] -= h
        fd = (J_at(q=qp) - J_at(q=qm)) / (qp[k] - qm[k])
        assert abs(fd - gr["q"][k]) <= 1e-6 * abs(gr["q"][k]), (k, fd, gr["q"][k])
    gp, gm = g0.copy(), g0.copy()
    gp[0] += h
    gm[0] -= h
    fd = (J_at(g=gp) - J_at(g=gm)) / (2 * h)
    assert abs(fd - gr["g"][0]) <= 1e-6 * abs(gr["g"][0]), (fd, gr["g"][0])
    visc = [9, 11, 13, 14, 15]
    sp, sm = s.copy(), s.copy()
    sp[visc] += h
    sm[visc] -= h
    fd = (J_at(ss=sp) - J_at(ss=sm)) / (2 * h)
    dsn = gr["s"][visc].sum()
    assert abs(fd - dsn) <= 1e-6 * abs(dsn), (fd, dsn)
    sv.close()


@pytest.mark.parametrize("rates", [True, False], ids=["states", "records"])
@pytest.mark.parametrize("case", [CASES[1], CASES[4]], ids=[CASES[1][0], CASES[4][0]])
def test_debug_poison_mode_leaves_the_adjoint_unchanged(monkeypatch, case, rates):
    """With LBM_DEBUG=1 the replayed states, the step records and every
    lambda(t) array are filled with NaN before they are written: the
    gradients and lambda(0) must be bitwise those of the normal mode (with
    the rate gradients off and the single-node scheme the sweep reads step
    records)."""
    name, mk_geom, mk_s, kw, obj, steps = case
    geom, s = mk_geom(), mk_s()
    Q = len(VELOCITIES[geom.lattice])
    df0 = states.random_deviation(Q, geom.n_nodes, seed=4, amp=2e-3)
    if geom.x_bc == "outflow":
        df0 = states.outlet_consistent(df0, geom.shape, VELOCITIES[geom.lattice])
    res = {}
    for mode in ("0", "1"):
        monkeypatch.setenv("LBM_DEBUG", mode)
        sv, J, gr = _gpu_grad(geom, s, kw, obj, steps, 3, df0, rates=rates)
        res[mode] = (J, gr)
        sv.close()
    monkeypatch.delenv("LBM_DEBUG", raising=False)
    assert res["0"][0] == res["1"][0]
    for key in ("q", "wall_u", "g", "s", "lam0"):
        assert np.array_equal(res["0"][1][key], res["1"][1][key]), key


@pytest.mark.parametrize("rates", [True, False], ids=["states", "records"])
@pytest.mark.parametrize("case", [CASES[2], [c for c in CASES if c[0] == "d3q19_meanux_rows256_seam"][0]],
                         ids=["d3q19_meanux_seam", "d3q19_meanux_rows256_seam"])
def test_fp32_adjoint_is_close_to_fp64(case, rates):
    name, mk_geom, mk_s, kw, obj, steps = case
    geom, s = mk_geom(), mk_s()
    df0 = states.random_deviation(19, geom.n_nodes, seed=3, amp=2e-3)
    sv64, J64, g64 = _gpu_grad(geom, s, kw, obj, steps, 4, df0, "fp64", rates=rates)
    sv32, J32, g32 = _gpu_grad(geom, s, kw, obj, steps, 4, df0, "fp32", rates=rates)
    assert abs(J32 - J64) <= 1e-4 * abs(J64)
    for key in ("q", "g"):
        scale = np.abs(g64[key]).max()
        assert np.abs(g32[key] - g64[key]).max() <= 1e-3 * scale, key
    sv64.close()
    sv32.close()


@pytest.mark.parametrize("dev", ["cpu", "cuda"])
def test_autograd_function_matches_adjoint(dev):
    """Leaves on the host take the host gradient path; leaves on the device
    get the per-link gradients written on the device (lbm_grad_device)."""
    import torch
    from paper_1712_08288_amd import binding
    from paper_1712_08288_amd.autograd import Problem, objective
    name, mk_geom, mk_s, kw, obj, steps = CASES[1]
    geom, s = mk_geom(), mk_s()
    sv = binding.solver_for(geom, s, l_rule=kw["l_rule"])
    prob = Problem(sv, steps=steps, every=4, objective="force_x", tag=1,
                   window=(obj.t0, obj.t1))
    q = torch.tensor(geom.q, device=dev, requires_grad=True)
    wu = torch.tensor(geom.wall_u, device=dev, requires_grad=True)
    g = torch.zeros(2, dtype=torch.float64, device=dev, requires_grad=True)
    tau = torch.tensor(1.0 / s[7], dtype=torch.float64, device=dev, requires_grad=True)
    ss = torch.cat([torch.tensor(s[:7], device=dev), (1.0 / tau).reshape(1), (1.0 / tau).reshape(1)])
    J = objective(q, wu, g, ss, prob)
    J.backward()
    sv2, J2, gr = _gpu_grad(geom, s, kw, obj, steps, 4, np.zeros((9, geom.n_nodes)))
    assert float(J) == J2
    assert q.grad.device.type == dev and wu.grad.device.type == dev
    assert np.array_equal(q.grad.cpu().numpy(), gr["q"])
    assert np.array_equal(wu.grad.cpu().numpy(), gr["wall_u"])
    dtau = -(gr["s"][7] + gr["s"][8]) / float(tau) ** 2
    assert np.isclose(float(tau.grad), dtau, rtol=1e-12)
    sv.close()
    sv2.close()


@pytest.mark.parametrize("every", [4, 1])
def test_autograd_without_rate_gradient_reads_step_records(every):
    """With s not requiring a gradient the autograd function turns the rate
    gradients off, so the sweep reads step records (every = 1: no snapshot):
    the other gradients equal those of the state-reading sweep to 1e-14."""
    import torch
    from paper_1712_08288_amd import binding
    from paper_1712_08288_amd.autograd import Problem, objective
    name, mk_geom, mk_s, kw, obj, steps = CASES[1]
    geom, s = mk_geom(), mk_s()
    sv = binding.solver_for(geom, s, l_rule=kw["l_rule"])
    prob = Problem(sv, steps=steps, every=every, objective="force_x", tag=1,
                   window=(obj.t0, obj.t1))
    q = torch.tensor(geom.q, device="cuda", requires_grad=True)
    wu = torch.tensor(geom.wall_u, device="cuda", requires_grad=True)
    g = torch.zeros(2, dtype=torch.float64, device="cuda", requires_grad=True)
    ss = torch.tensor(s, dtype=torch.float64, device="cuda")
    J = objective(q, wu, g, ss, prob)
    J.backward()
    sv2, J2, gr = _gpu_grad(geom, s, kw, obj, steps, 4, np.zeros((9, geom.n_nodes)))
    assert float(J) == J2
    for got, key in ((q.grad, "q"), (wu.grad, "wall_u"), (g.grad, "g")):
        scale = max(np.abs(gr[key]).max(), 1e-300)
        assert np.abs(got.cpu().numpy() - gr[key]).max() <= 1e-14 * scale, key
    sv.close()
    sv2.close()


def test_device_gradients_equal_host_gradients():
    """lbm_grad_device puts the per-link gradients in the caller's order on
    the device, bit for bit what lbm_grad returns on the host."""
    import torch
    name, mk_geom, mk_s, kw, obj, steps = [c for c in CASES if c[0] == "d3q19_meanux_channel_many_links"][0]
    geom, s = mk_geom(), mk_s()
    df0 = states.random_deviation(19, geom.n_nodes, seed=5, amp=1e-3)
    sv, J, gr = _gpu_grad(geom, s, kw, obj, steps, 3, df0)
    nl = geom.n_links
    dq = torch.full((nl,), float("nan"), dtype=torch.float64, device="cuda")
    du = torch.full((nl, 3), float("nan"), dtype=torch.float64, device="cuda")
    small = sv.grad_device(dq, du)
    assert np.array_equal(dq.cpu().numpy(), gr["q"])
    assert np.array_equal(du.cpu().numpy(), gr["wall_u"])
    assert np.array_equal(small["g"], gr["g"]) and np.array_equal(small["s"], gr["s"])
    assert np.abs(gr["wall_u"]).max() > 0 and np.abs(gr["q"]).max() > 0
    only = sv.grad_device(dq=dq)       # host outputs still filled, wall_u skipped
    assert np.array_equal(only["g"], gr["g"])
    sv.close()


@pytest.mark.parametrize("case", [CASES[0], CASES[4]], ids=[CASES[0][0], CASES[4][0]])
def test_reverse_sweep_in_pieces_is_bitwise_the_full_sweep(case):
    """lbm_adjoint_step: the reverse sweep in uneven pieces (crossing segment
    boundaries) gives the gradients and lambda(0) of lbm_adjoint, bit for
    bit; the remaining-step count follows the sweep."""
    name, mk_geom, mk_s, kw, obj, steps = case
    geom, s = mk_geom(), mk_s()
    Q = len(VELOCITIES[geom.lattice])
    df0 = states.random_deviation(Q, geom.n_nodes, seed=8, amp=2e-3)
    sv, J, full = _gpu_grad(geom, s, kw, obj, steps, 3, df0)
    sv.close()
    from paper_1712_08288_amd import binding
    sv = binding.solver_for(geom, s, precision="fp64", g=kw.get("g"), dp=kw.get("dp", 0.0),
                            l_rule=kw.get("l_rule", "min"), b=kw.get("b", 1.0),
                            two_node=kw.get("two_node", False))
    sv.init_deviation(df0)
    sv.set_objective(obj.kind, obj.tag, obj.t0, obj.t1)
    sv.run_checkpointed(steps, 3)
    assert sv.adjoint_remaining() == -1
    done = 0
    for piece in (2, 0, 5, 1, steps):
        sv.adjoint_step(piece)
        done = min(steps, done + piece)
        assert sv.adjoint_remaining() == steps - done
    gr = sv.grad()
    gr["lam0"] = sv.get_adjoint()
    for key in ("q", "wall_u", "g", "s", "lam0"):
        assert np.array_equal(gr[key], full[key]), key
    # a new lbm_adjoint restarts the sweep
    sv.adjoint()
    assert sv.adjoint_remaining() == 0
    assert np.array_equal(sv.grad()["q"], full["q"])
    sv.close()
