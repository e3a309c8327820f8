"""Long oracle runs for the configured-step parity tests.

    python tests/oracle_runs.py NAME OUTDIR

runs the float64 oracle on one benchmark workload for its configured number
of steps and writes, at each checkpoint step t, OUTDIR/NAME_t.npz with the
pre-collision deviations f(., t) - w rho0 (Q, N), the velocity u (N, D) and
the objective accumulated so far.  Each file appears atomically (written
under a temporary name, then renamed), so a reader can poll for it.  The
test session starts these runs in the background when the tests that need
them are selected (tests/conftest.py), so that they overlap the other GPU
tests.  Only oracle/ and workloads/ are used.
"""

import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle.adjoint import Objective   # noqa: E402
from oracle.lbm import Oracle          # noqa: E402
from workloads import configs          # noqa: E402


def _c4():
    """Channel flow past a cylinder (1024 x 512, D2Q9, tau = 0.56, u_in = 0.05,
    zero-gradient outlet), rest start, 3000 steps; the drag on the cylinder
    (tag 1) averaged over the last 1000 steps."""
    w = configs.c4_cylinder()
    t0, t1 = w.extra["obj_window"]
    return w, Objective("force_x", tag=1, t0=t0, t1=t1), (1000, 2000, 3000)


def _c5_crop():
    """Periodic porous medium 96 x 64 x 64 (D3Q19, 5 spheres r ~ U[8, 16],
    g_x = 1e-6, tau = 0.65), rest start, 2000 steps; mean u_x over all steps."""
    w = configs.c5_crop()
    return w, Objective("mean_ux", t0=0, t1=w.steps), (500, 1000, 1500, 2000)


RUNS = {"c4_3000": _c4, "c5crop_2000": _c5_crop}


def run(name, outdir):
    w, obj, checkpoints = RUNS[name]()
    try:   # the collision's dense products use a few BLAS threads
        import threadpoolctl
        threadpoolctl.threadpool_limits(8)
    except Exception:
        pass
    geom = w.geometry()
    o = Oracle(geom, w.s, g=w.g, dp=w.dp, l_rule=w.l_rule)
    f = o.init_equilibrium()
    J = 0.0
    t_start = time.time()
    for t in range(w.steps):
        fn, fp = o.step(f)
        J += obj.value(o, t, f, fp, fn)
        f = fn
        if t + 1 in checkpoints:
            _, u = o.macroscopic(f)
            tmp = os.path.join(outdir, "%s_%d.tmp.npz" % (name, t + 1))
            np.savez(tmp, df=o.as_deviation(f), u=u, J=J, t=t + 1)
            os.replace(tmp, os.path.join(outdir, "%s_%d.npz" % (name, t + 1)))
        if (t + 1) % 100 == 0:
            print("%s: step %d of %d, %.0f s" % (name, t + 1, w.steps, time.time() - t_start),
                  flush=True)


if __name__ == "__main__":
    run(sys.argv[1], sys.argv[2])
