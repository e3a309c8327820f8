"""The five benchmark workloads and small parity cases.

Lattice units throughout: h = dt = c = 1, c_s^2 = 1/3, rho0 = 1.
Relaxation rates are listed in the row order of each lattice's moment
matrix: D2Q9 (rho, e, eps, j_x, q_x, j_y, q_y, p_xx, p_xy); D3Q19 (rho, e,
eps, j_x, q_x, j_y, q_y, j_z, q_z, 3p_xx, 3pi_xx, p_ww, pi_ww, p_xy, p_yz,
p_xz, m_x, m_y, m_z).
"""

from dataclasses import dataclass, field
from typing import Callable, Optional
import numpy as np

from . import geometry as G


def d2q9_rates(tau, s_e=1.4, s_eps=1.4, s_q=1.2):
    return np.array([0.0, s_e, s_eps, 0.0, s_q, 0.0, s_q, 1.0 / tau, 1.0 / tau])


def d2q9_paper_rates(s_nu, literal=False):
    """Rates of the paper's Section 3 for D2Q9.  The printed vector gives
    s_jy = 0.5 and s_qy = 1 (x and y treated differently); the default reading
    mirrors its D3Q15 pattern, s_j = 1 and s_q = 0.5 in both directions."""
    if literal:
        return np.array([1, 1.8, 1.2, 1, 0.5, 0.5, 1, s_nu, s_nu], dtype=np.float64)
    return np.array([1, 1.8, 1.2, 1, 0.5, 1, 0.5, s_nu, s_nu], dtype=np.float64)


def d3q15_paper_rates(s_nu):
    """Rates of the paper's Section 3 for D3Q15, in its Appendix row order
    (rho, e, eps, jx, qx, jy, qy, jz, qz, pxx, pww, pxy, pyz, pxz, mxyz)."""
    return np.array([1, 1.8, 1.2, 1, 0.5, 1, 0.5, 1, 0.5,
                     s_nu, s_nu, s_nu, s_nu, s_nu, 1.5], dtype=np.float64)


def d3q19_rates(tau):
    """d'Humieres et al. (2002) rates for D3Q19: s_e = 1.19, s_eps = s_pi =
    1.4, s_q = 1.2, s_m = 1.98, viscous rows 1/tau; conserved rows 0."""
    sn = 1.0 / tau
    return np.array([0, 1.19, 1.4, 0, 1.2, 0, 1.2, 0, 1.2,
                     sn, 1.4, sn, 1.4, sn, sn, sn, 1.98, 1.98, 1.98],
                    dtype=np.float64)


@dataclass
class Workload:
    name: str
    lattice: str
    shape: tuple
    s: np.ndarray
    steps: int
    make_geometry: Callable
    g: tuple = (0.0, 0.0, 0.0)
    rho0: float = 1.0
    x_bc: str = "periodic"
    dp: float = 0.0                 # density jump at the x seam ("pressure")
    l_rule: str = "min"
    b: float = 1.0
    precisions: tuple = ("fp64",)
    description: str = ""
    extra: dict = field(default_factory=dict)

    @property
    def n_nodes(self):
        return int(np.prod(self.shape))

    def geometry(self):
        return self.make_geometry()


def c1_couette(n=64, steps=None, u_w=None):
    """Circular Couette, D2Q9 FP64.  At n = 64: u_w = 0.01, 5000 steps.  The
    refinement runs keep tau and scale u_w with h and the step count with
    1/h^2 (diffusive scaling) so every size reaches the same physical time."""
    s = n / 64.0
    if u_w is None:
        u_w = 0.01 / s
    if steps is None:
        steps = int(round(5000 * s * s))
    return Workload(
        name="c1_couette_%d" % n, lattice="D2Q9", shape=(n, n, 1),
        s=d2q9_rates(0.8), steps=steps,
        make_geometry=lambda: G.annulus(n, u_w),
        description="D2Q9 MRT circular Couette %dx%d, %d steps" % (n, n, steps),
        extra=dict(u_w=u_w))


def c2_cylinders(nx=2048, ny=2048, n_obst=400, seed=2, steps=1000):
    return Workload(
        name="c2_cylinders_%dx%d" % (nx, ny), lattice="D2Q9", shape=(nx, ny, 1),
        s=d2q9_rates(0.6), steps=steps, g=(1e-6, 0.0, 0.0),
        make_geometry=lambda: G.random_cylinders(nx, ny, n_obst, 8.0, 24.0, seed),
        precisions=("fp64", "fp32"),
        description="D2Q9 MRT %dx%d periodic, %d random cylinders r~U[8,24], "
                    "g_x=1e-6, %d steps" % (nx, ny, n_obst, steps))


def c3_spheres(n=256, n_obst=120, seed=3, steps=500, rmin=10.0, rmax=20.0):
    return Workload(
        name="c3_spheres_%d" % n, lattice="D3Q19", shape=(n, n, n),
        s=d3q19_rates(0.7), steps=steps, x_bc="pressure", dp=1e-3,
        make_geometry=lambda: G.random_spheres(n, n, n, n_obst, rmin, rmax,
                                               seed, x_bc="pressure"),
        precisions=("fp32", "fp64"),
        description="D3Q19 MRT %d^3 random sphere packing (%d spheres, "
                    "r~U[%g,%g]), pressure-driven x (drho=1e-3), %d steps"
                    % (n, n_obst, rmin, rmax, steps))


def c3_shard(nx=256, ny=256, nz=32, n_obst=15, seed=33, steps=500):
    """One GPU's share of the 256^3 sphere packing split into eight z-slabs:
    an independent 256x256x32 packing with the full-size density (120
    spheres / 8 = 15, r~U[10,20]) and the same seam, so the step runs at a
    shard's real shape (whole x rows, 2^21 nodes).  The slab is periodic in
    z instead of exchanging halos."""
    w = c3_spheres(n=nx, n_obst=n_obst, seed=seed, steps=steps)
    w.name = "c3_shard_%dx%dx%d" % (nx, ny, nz)
    w.shape = (nx, ny, nz)
    w.make_geometry = lambda: G.random_spheres(nx, ny, nz, n_obst, 10.0, 20.0, seed,
                                               x_bc="pressure")
    w.description = ("D3Q19 MRT %dx%dx%d z-slab of sphere packing (%d spheres, r~U[10,20]), "
                     "pressure-driven x (drho=1e-3), %d steps" % (nx, ny, nz, n_obst, steps))
    return w


def c4_cylinder(nx=1024, ny=512, steps=3000, u_in=0.05, radius=20.3,
                center=(128.4, 256.2)):
    return Workload(
        name="c4_cylinder_%dx%d" % (nx, ny), lattice="D2Q9", shape=(nx, ny, 1),
        s=d2q9_rates(0.56), steps=steps, x_bc="outflow",
        make_geometry=lambda: G.channel_cylinder(nx, ny, radius, center, u_in),
        precisions=("fp64", "fp32"),
        description="D2Q9 MRT channel %dx%d, cylinder r=%g, u_in=%g, %d steps"
                    % (nx, ny, radius, u_in, steps),
        extra=dict(u_in=u_in, obj_window=(steps - 1000 if steps > 1000 else 0, steps)))


def c5_porous(nx=384, ny=256, nz=256, n_obst=300, seed=5, steps=2000):
    return Workload(
        name="c5_porous_%dx%dx%d" % (nx, ny, nz), lattice="D3Q19",
        shape=(nx, ny, nz), s=d3q19_rates(0.65), steps=steps,
        g=(1e-6, 0.0, 0.0),
        make_geometry=lambda: G.random_spheres(nx, ny, nz, n_obst, 8.0, 16.0, seed),
        precisions=("fp32",),
        description="D3Q19 MRT %dx%dx%d periodic porous medium, %d spheres "
                    "r~U[8,16], g_x=1e-6, %d steps" % (nx, ny, nz, n_obst, steps))


def c5_crop(steps=2000):
    """Independent periodic 96x64x64 medium with the full-size porosity:
    300 spheres in 384x256x256 scale to 300 * (96*64*64)/(384*256*256) ~ 4.7,
    so 5 spheres."""
    return c5_porous(96, 64, 64, n_obst=5, seed=55, steps=steps)


CONFIGS = {
    "c1": c1_couette,
    "c2": c2_cylinders,
    "c3": c3_spheres,
    "c4": c4_cylinder,
    "c5": c5_porous,
}
