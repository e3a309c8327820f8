"""Parity at the benchmark sizes (GPU): the full domain runs on the GPU in
the launch configuration bench.py times; the oracle recomputes sampled
nodes one by one on windows around them (window mode: exact after k steps
when the window half-width exceeds k), from the same seeded non-equilibrium
initial state.  Samples include nodes with cut links and nodes on the x
seam.  Tolerances as in test_gpu_forward.py.
"""

import numpy as np
import pytest

from gpu_util import require_gpu
from oracle.lbm import sampled_step_outputs
from workloads import configs, states
from workloads.velocities import VELOCITIES

pytestmark = pytest.mark.gpu

STEPS = 3
TOL = {"fp64": 1e-12, "fp32": 3e-6}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _samples(geom, n_random=24, n_link=16, seed=0):
    rng = np.random.default_rng(seed)
    fluid = np.nonzero(geom.solid == 0)[0]
    pick = [rng.choice(fluid, n_random, replace=False)]
    if geom.n_links:
        pick.append(rng.choice(np.unique(geom.node), n_link, replace=False))
    nx = geom.shape[0]
    x = fluid % nx
    for col in (0, nx - 1):
        c = fluid[x == col]
        if len(c):
            pick.append(rng.choice(c, min(4, len(c)), replace=False))
    return np.unique(np.concatenate(pick))


def _run(w, precision, seed=17):
    from paper_1712_08288_amd import binding
    geom = w.geometry()
    Q = len(VELOCITIES[geom.lattice])
    print("workload", w.name, precision, geom.shape, "links", geom.n_links, flush=True)
    df0 = states.random_deviation(Q, geom.n_nodes, seed=seed, amp=1e-3)
    if geom.x_bc == "outflow":
        df0 = states.outlet_consistent(df0, geom.shape, VELOCITIES[geom.lattice])
    sv = binding.solver_for(geom, w.s, g=w.g, precision=precision, dp=w.dp,
                            l_rule=w.l_rule, b=w.b)
    sv.init_deviation(df0)
    sv.step(STEPS)
    got = sv.distribution()
    sv.close()
    samples = _samples(geom)
    want = sampled_step_outputs(geom, w.s, df0, STEPS, samples, g=w.g, dp=w.dp,
                                l_rule=w.l_rule, b=w.b)
    g = got[:, samples]
    err = np.sqrt(((g - want) ** 2).sum() / (want ** 2).sum())
    return err, np.isfinite(g).all()


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_c3_spheres_256(precision):
    err, finite = _run(configs.c3_spheres(), precision)
    assert finite
    assert err < TOL[precision], err


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_c2_cylinders_2048(precision):
    err, finite = _run(configs.c2_cylinders(), precision)
    assert finite
    assert err < TOL[precision], err


def test_c4_channel_1024x512():
    err, finite = _run(configs.c4_cylinder(), "fp64")
    assert finite
    assert err < TOL["fp64"], err


def test_c5_porous_384x256x256_fp32():
    err, finite = _run(configs.c5_porous(), "fp32")
    assert finite
    assert err < TOL["fp32"], err


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_c5_crop_96x64x64_parity(precision):
    """The C5 crop-sized medium (96x64x64, 5 spheres, seed 55) against the
    oracle over the whole domain."""
    from gpu_util import pair, rel_l2
    w = configs.c5_crop(steps=15)
    geom = w.geometry()
    got, want, fl, sv, o, f = pair(geom, w.s, w.steps, precision=precision, g=w.g,
                                   l_rule=w.l_rule)
    assert rel_l2(got, want, fl) < (1e-12 if precision == "fp64" else 3e-6)
    sv.close()


def test_c3_adjoint_matches_central_differences_at_full_size():
    """The benchmark workload's reverse sweep (256^3 D3Q19, FP64, checkpointed
    as bench.py runs it) against central differences of J along directions
    in g, in all link fractions q at once and in all wall velocities at once:
    directional derivatives hold at any size, so this checks the adjoint
    kernels on the real grid, wave mix and link count.  The q and wall
    directions are the gradients themselves (a strong, well-conditioned
    signal); a wrong gradient pattern changes the directional derivative the
    differences measure, so it still fails."""
    from paper_1712_08288_amd import binding
    w = configs.c3_spheres()
    geom = w.geometry()
    g0 = np.array([2e-6, 0.0, 0.0])
    steps, every = 12, 4
    sv = binding.solver_for(geom, w.s, g=g0, precision="fp64", dp=w.dp, l_rule=w.l_rule)
    print("workload", w.name, "fp64 adjoint", geom.shape, "links", geom.n_links, flush=True)

    def J_at(q=None, wall_u=None, g=None):
        sv.update_links(q if q is not None else geom.q,
                        wall_u if wall_u is not None else geom.wall_u)
        sv.set_parameters(w.s, g if g is not None else g0)
        sv.init()
        sv.set_objective("mean_ux", 0, 0, steps)
        sv.step(steps)
        return sv.objective()

    sv.init()
    sv.set_objective("mean_ux", 0, 0, steps)
    sv.run_checkpointed(steps, every)
    J = sv.objective()
    sv.adjoint()
    gr = sv.grad()
    assert abs(J - J_at()) <= 1e-14 * abs(J)
    h = 1e-7
    fd = (J_at(g=g0 + [h, 0, 0]) - J_at(g=g0 - [h, 0, 0])) / (2 * h)
    print("dJ/dg_x", fd, gr["g"][0], flush=True)
    assert abs(fd - gr["g"][0]) <= 1e-6 * abs(gr["g"][0]), (fd, gr["g"][0])
    hq = 1e-6
    dq = gr["q"] / np.abs(gr["q"]).max()
    dq[(geom.q + hq * dq > 1.0) | (geom.q - hq * dq <= 0.0)] = 0.0
    fd = (J_at(q=geom.q + hq * dq) - J_at(q=geom.q - hq * dq)) / (2 * hq)
    want = float(gr["q"] @ dq)
    print("dJ/dq along dq", fd, want, flush=True)
    assert abs(fd - want) <= 1e-6 * abs(want), (fd, want)
    du = gr["wall_u"] / np.abs(gr["wall_u"]).max()
    fd = (J_at(wall_u=geom.wall_u + hq * du) - J_at(wall_u=geom.wall_u - hq * du)) / (2 * hq)
    want = float((gr["wall_u"] * du).sum())
    print("dJ/dwall_u along du", fd, want, flush=True)
    assert abs(fd - want) <= 1e-6 * abs(want), (fd, want)
    sv.close()
    # the FP32 path bench.py times, against these FP64 gradients
    sv32 = binding.solver_for(geom, w.s, g=g0, precision="fp32", dp=w.dp, l_rule=w.l_rule)
    sv32.set_rate_gradient(False)
    sv32.init()
    sv32.set_objective("mean_ux", 0, 0, steps)
    sv32.run_checkpointed(steps, every)
    J32 = sv32.objective()
    sv32.adjoint()
    g32 = sv32.grad()
    print("fp32 vs fp64: J", abs(J32 - J) / abs(J), "dJ/dg",
          np.abs(g32["g"] - gr["g"]).max() / np.abs(gr["g"]).max(), flush=True)
    assert abs(J32 - J) <= 1e-4 * abs(J)
    for key in ("q", "wall_u", "g"):
        scale = np.abs(gr[key]).max()
        err = np.abs(g32[key] - gr[key]).max() / scale
        print("fp32 vs fp64", key, err, flush=True)
        assert err <= 1e-3, key
    sv32.close()


def test_population_arrays_beyond_4gib_fp64():
    """A porous medium of 384x256x320 nodes in FP64: each population array
    (19 x 31.5M values) is 4.78 GB, past the reach of 32-bit byte offsets.
    Sampled forward parity with the oracle after three steps, and the
    reverse sweep on step records (every step recorded) against central
    differences of J in g_x and against the sweep that reads the states."""
    from paper_1712_08288_amd import binding
    w = configs.c5_porous(384, 256, 320, n_obst=375, seed=8)
    geom = w.geometry()
    assert 19 * geom.n_nodes * 8 > (1 << 32)
    err, finite = _run(w, "fp64")
    assert finite
    assert err < TOL["fp64"], err
    steps = 3
    sv = binding.solver_for(geom, w.s, g=w.g, precision="fp64", l_rule=w.l_rule)

    def J_at(gx):
        sv.set_parameters(w.s, (gx, 0.0, 0.0))
        sv.init()
        sv.set_objective("mean_ux", 0, 0, steps)
        sv.step(steps)
        return sv.objective()

    grads = {}
    for rates in (False, True):
        sv.set_rate_gradient(rates)
        sv.set_parameters(w.s, w.g)
        sv.init()
        sv.set_objective("mean_ux", 0, 0, steps)
        sv.run_checkpointed(steps, 1)
        sv.adjoint()
        grads[rates] = sv.grad()
    gx = w.g[0]
    h = 1e-7
    fd = (J_at(gx + h) - J_at(gx - h)) / (2 * h)
    got = grads[False]["g"][0]
    print("dJ/dg_x", fd, got, flush=True)
    assert abs(fd - got) <= 1e-6 * abs(got), (fd, got)
    for key in ("q", "wall_u", "g"):
        scale = max(np.abs(grads[True][key]).max(), 1e-300)
        assert np.abs(grads[False][key] - grads[True][key]).max() <= 1e-12 * scale, key
    sv.close()
