"""One lattice Boltzmann time step with the single-node boundary scheme.

Paper order (Section 2 and Appendix):

1. collision, Eq. (22a):  f'_i = f_i + Omega_i with the MRT operator
   Omega = -M^{-1} S M (f - f^eq) of the Appendix, f^eq from Eq. (42) with
   c = 1, c_s^2 = 1/3:  f^eq_i = w_i {rho + rho0 [3 e_i.u + 4.5 (e_i.u)^2
   - 1.5 u.u]}, rho = sum f_i, rho0 u = sum e_i f_i.  A body force g enters
   as F_i = 3 w_i rho0 e_i.g added to f' (the paper drives two of its tests
   by a force but does not print the forcing term; this reading adds the
   first-order term and leaves the velocity definition unshifted).
2. advection, Eq. (22b):  f_i(x, t+1) = f'_i(x - e_i, t)  for every pair of
   fluid nodes; y and z periodic; x periodic, periodic with a density jump
   (+w_i drho for populations that cross from x = nx-1 to 0, -w_i drho the
   other way), or zero-gradient outflow (at x = nx-1 a population moving in
   -x is read from (nx-1, y - e_y, z - e_z)).
3. boundary, Eq. (213) (Eq. (210) when b = 1) on every cut link (x_f, i):
   f_i(x_f, t+1) = c0 f_i(x_f,t) + c1 f_ibar(x_f,t) + c2 f'_i(x_f,t)
                   + c3 f'_ibar(x_f,t) + c4 * 3 w_i rho0 e_i.phi_k
   using only values held at x_f (the time-lag approximation Eq. (29)).

State: the pre-collision f(., t) of Eq. (21) at every node, shape (Q, N);
solid nodes hold NaN so any read of them shows up in the result.  With
deviation=True the stored values are f_i - w_i rho0; every step above is
unchanged in that form (sum w_i = 1, w_i = w_ibar, c0+c1+c2+c3 = 1), only
rho gets rho0 added back on output.

The arithmetic is generic over the numpy dtype, so complex inputs give
complex-step derivatives.  Parity pins: tests/test_oracle_*.py.
"""

import numpy as np

from . import lattice as _lattice
from . import scheme as _scheme


class Oracle:
    def __init__(self, geom, s, rho0=1.0, g=None, dp=0.0, l_rule="min",
                 b=1.0, deviation=True, q=None, wall_u=None,
                 allow_nonconvex=False, nodes=None, two_node=False, collision=None,
                 wall_decay=1.0):
        """collision: None for the MRT operator of the Appendix with rates s;
        ("trt", s_plus, s_minus) for the two-relaxation-time operator and
        ("bgk", s_nu) for the single-relaxation-time one (Remark (1): the
        boundary scheme does not depend on the collision operator).  TRT
        relaxes the even and odd halves f^+- = (f_i +- f_ibar)/2 towards the
        halves of f^eq at s_plus and s_minus; BGK is s_plus = s_minus = s_nu.
        wall_decay: wall data phi(x_b, t) = phi(x_b, 0) * wall_decay**t, t
        counted in steps from the last init_* call (the Taylor-Green data of
        Section 3.2 decay this way); the step from t uses phi at t (Eq. (210)).
        two_node: use Eq. (211) (Remark (2)) instead of Eq. (210): the
        time-lagged f_ibar(x_f, t) is replaced by its advected value
        f'_ibar(x_f + e_i, t) whenever that neighbour is fluid; links whose
        neighbour x_f + e_i is solid keep Eq. (210).
        nodes: optional sorted array of global node indices to simulate (a
        window).  Pull sources outside the window read NaN, so after k steps
        exactly the nodes at least k pulls away from the window's edge are
        exact; the full domain is used when nodes is None."""
        lat = _lattice.get(geom.lattice)
        self.lat = lat
        self.Q, self.D = lat.Q, lat.D
        self.e = lat.e.astype(np.float64)
        self.w = lat.w
        self.M = lat.M
        self.Minv = lat.Minv
        self.opp = lat.opp
        self.shape = tuple(geom.shape)
        nx, ny, nz = self.shape
        self.x_bc = geom.x_bc
        self.s = np.asarray(s)
        self.rho0 = rho0
        self.g = np.zeros(self.D) if g is None else np.asarray(g)[: self.D]
        self.dp = dp
        self.deviation = deviation
        self.base = self.w * rho0 if deviation else np.zeros(self.Q)
        self.rho_base = rho0 if deviation else 0.0
        self.l_rule, self.b = l_rule, b
        self.two_node = two_node
        if collision is not None:
            if collision[0] == "bgk":
                collision = ("trt", collision[1], collision[1])
            if collision[0] != "trt" or len(collision) != 3:
                raise ValueError("collision must be None, ('bgk', s) or ('trt', s_plus, s_minus)")
        self.collision = collision
        self.wall_decay = wall_decay
        self.time = 0
        n_all = nx * ny * nz
        self.window = nodes is not None
        self.nodes = (np.arange(n_all, dtype=np.int64) if nodes is None
                      else np.asarray(nodes, dtype=np.int64))
        self.N = self.nodes.shape[0]
        self.fluid = np.asarray(geom.solid)[self.nodes] == 0
        local = np.full(n_all, self.N, dtype=np.int64) if self.window else None
        if self.window:
            local[self.nodes] = np.arange(self.N)

        # pull table: node read by direction i at node n, and the seam sign
        n = self.nodes
        x, y, z = n % nx, (n // nx) % ny, n // (nx * ny)
        self.src = np.empty((self.Q, self.N), dtype=np.int64)
        self.seam = np.zeros((self.Q, self.N))
        ez = lat.e[:, 2] if self.D == 3 else np.zeros(self.Q, np.int64)
        for i in range(self.Q):
            sx = x - lat.e[i, 0]
            if self.x_bc == "outflow":
                sx = np.clip(sx, 0, nx - 1)
            else:
                if self.x_bc == "pressure":
                    self.seam[i] = np.where(sx < 0, 1.0, np.where(sx >= nx, -1.0, 0.0))
                sx = np.mod(sx, nx)
            sy = np.mod(y - lat.e[i, 1], ny)
            sz = np.mod(z - ez[i], nz)
            src = sx + nx * (sy + ny * sz)
            self.src[i] = local[src] if self.window else src

        # cut links and their coefficients, Eq. (213)
        keep = slice(None)
        lk_node = np.asarray(geom.node, dtype=np.int64)
        if self.window:
            keep = local[lk_node] < self.N
            lk_node = local[lk_node[keep]]
        self.lk_node = lk_node
        self.lk_dir = np.asarray(geom.dir, dtype=np.int64)[keep]
        self.lk_opp = self.opp[self.lk_dir]
        self.lk_tag = np.asarray(geom.tag, dtype=np.int64)[keep]
        self.q = np.asarray(geom.q if q is None else q)[keep]
        self.wall_u = np.asarray(geom.wall_u if wall_u is None else wall_u)[keep]
        self.l = _scheme.l_of_gamma(l_rule, self.q)
        if not allow_nonconvex and not np.all(_scheme.convex(self.q, self.l)):
            raise ValueError("l(gamma) violates Eq. (212)")
        self.c = _scheme.coefficients(self.q, self.l, b)
        # bounce-back wall term 3 w_i rho0 e_i.phi (paper Eq. (26), lattice units)
        e_l = self.e[self.lk_dir]
        self.wall_term = 3.0 * self.w[self.lk_dir] * rho0 * (e_l * self.wall_u).sum(1)
        # forcing term per direction
        self.F = 3.0 * self.w * rho0 * (self.e @ self.g)
        if not self.window:
            self._check_links()
        is_link = np.zeros((self.Q, self.N), dtype=bool)
        is_link[self.lk_dir, self.lk_node] = True
        self.lk_ibar_is_link = is_link[self.lk_opp, self.lk_node]

    def _check_links(self):
        """A direction at a fluid node is a cut link exactly when the node it
        would read is solid; every link is listed once."""
        solid = ~self.fluid
        need = np.zeros((self.Q, self.N), dtype=bool)
        need[:, self.fluid] = solid[self.src[:, self.fluid]]
        have = np.zeros((self.Q, self.N), dtype=np.int64)
        np.add.at(have, (self.lk_dir, self.lk_node), 1)
        if np.any(have > 1):
            raise ValueError("duplicate cut link")
        if np.any(have.astype(bool) != need):
            raise ValueError("cut links do not match the solid mask")

    # ------------------------------------------------------------------ moments
    def density_deviation(self, f):
        """sum_i f_i (in deviation form: rho - rho0)."""
        return f.sum(0)

    def velocity(self, f):
        """u = sum_i e_i f_i / rho0, shape (D, N)."""
        return (self.e.T @ f) / self.rho0

    def equilibrium(self, rho_s, u):
        """Eq. (42) with c = 1, c_s^2 = 1/3; rho_s is the stored-form density
        (rho, or rho - rho0 in deviation form) and the result is in the same
        form."""
        eu = self.e @ u
        uu = (u * u).sum(0)
        return self.w[:, None] * (rho_s[None, :] + self.rho0 * (
            3.0 * eu + 4.5 * eu * eu - 1.5 * uu[None, :]))

    # ---------------------------------------------------------------- the step
    def collide(self, f):
        """Eq. (22a) with the MRT operator of the Appendix (or the TRT / BGK
        operator chosen at construction) plus forcing."""
        feq = self.equilibrium(self.density_deviation(f), self.velocity(f))
        if self.collision is not None:
            _, s_plus, s_minus = self.collision
            neq = f - feq
            even = 0.5 * (neq + neq[self.opp])
            odd = 0.5 * (neq - neq[self.opp])
            return f - s_plus * even - s_minus * odd + self.F[:, None]
        m_neq = self.M @ (f - feq)
        return f - self.Minv @ (self.s[:, None] * m_neq) + self.F[:, None]

    def stream(self, fp):
        """Eq. (22b) as a pull over the node table; link directions read a
        solid node here and are overwritten by the boundary scheme."""
        rows = np.arange(self.Q)[:, None]
        if self.window:     # column N stands for every node outside the window
            fp = np.concatenate([fp, np.full((self.Q, 1), np.nan, dtype=fp.dtype)], axis=1)
        fn = fp[rows, self.src]
        if self.dp != 0.0:
            fn = fn + self.seam * (self.w * self.dp)[:, None]
        return fn

    def boundary(self, f, fp, fn):
        """Eq. (213) on every cut link, from values held at x_f only
        (Eq. (211) variant: the f_ibar term from the advected value)."""
        xf, i, ib = self.lk_node, self.lk_dir, self.lk_opp
        c0, c1, c2, c3, c4 = self.c
        f_ib = f[ib, xf]
        if self.two_node:
            # f_ibar(x_f, t+1) after advection, unless (x_f, ibar) is itself
            # a cut link (x_f + e_i solid): then the single-node form
            f_ib = np.where(self.lk_ibar_is_link, f_ib, fn[ib, xf])
        fn[i, xf] = (c0 * f[i, xf] + c1 * f_ib + c2 * fp[i, xf]
                     + c3 * fp[ib, xf] + c4 * self.wall_term * self.wall_scale(self.time))
        return fn

    def wall_scale(self, t):
        return 1.0 if self.wall_decay == 1.0 else self.wall_decay ** t

    def step(self, f):
        fp = self.collide(f)
        fn = self.stream(fp)
        self.boundary(f, fp, fn)
        fn[:, ~self.fluid] = np.nan
        self.time += 1
        return fn, fp

    def run(self, f, steps, observe=None):
        """Advance `steps` steps; observe(t, f_t, fp_t, f_t+1) after each."""
        for t in range(steps):
            fn, fp = self.step(f)
            if observe is not None:
                observe(t, f, fp, fn)
            f = fn
        return f

    # ------------------------------------------------------------ set-up / out
    def init_equilibrium(self, rho=None, u=None):
        """f(x, 0) = f^eq(rho(x), u(x)) at fluid nodes (rest if omitted)."""
        rho = np.full(self.N, self.rho0) if rho is None else np.asarray(rho)
        u = np.zeros((self.N, self.D)) if u is None else np.asarray(u)
        f = self.equilibrium(rho - self.rho_base, np.asarray(u).T)
        f = f.astype(np.result_type(f, np.float64))
        f[:, ~self.fluid] = np.nan
        self.time = 0
        return f

    def init_deviation(self, df):
        """f(x, 0) given as deviations from w_i rho0, shape (Q, N)."""
        f = np.array(df, dtype=np.result_type(df, np.float64)) + (
            self.w * self.rho0 - self.base)[:, None]
        f[:, ~self.fluid] = np.nan
        self.time = 0
        return f

    def as_deviation(self, f):
        return f + (self.base - self.w * self.rho0)[:, None]

    def macroscopic(self, f):
        """(rho (N,), u (N, D)) from the pre-collision state, NaN at solids."""
        return self.rho_base + self.density_deviation(f), self.velocity(f).T

    def mass(self, f):
        return float(np.real(self.density_deviation(f)[self.fluid].sum())) + \
            self.rho_base * int(self.fluid.sum())

    def momentum(self, f):
        return (self.e.T @ f[:, self.fluid]).sum(1)

    def force(self, fp, fn, n_tags=None):
        """Momentum-exchange force on each tag during the step t -> t+1:
        sum over the tag's links of e_ibar (f'_ibar(x_f, t) + f_i(x_f, t+1)),
        with absolute (not deviation) values.  Shape (n_tags, D)."""
        xf, i, ib = self.lk_node, self.lk_dir, self.lk_opp
        val = (fp[ib, xf] + self.base[ib]) + (fn[i, xf] + self.base[i])
        contrib = self.e[ib] * val[:, None]
        nt = (int(self.lk_tag.max()) + 1 if len(self.lk_tag) else 0) if n_tags is None else n_tags
        out = np.zeros((nt, self.D), dtype=contrib.dtype)
        np.add.at(out, self.lk_tag, contrib)
        return out


def box_window(shape, node, radius):
    """Sorted global indices of the periodic box of half-width `radius`
    around `node` (clipped to the domain extent in each direction)."""
    nx, ny, nz = shape
    x, y, z = node % nx, (node // nx) % ny, node // (nx * ny)
    axes = []
    for c, n in ((x, nx), (y, ny), (z, nz)):
        r = min(radius, (n - 1) // 2)
        axes.append(np.unique(np.mod(np.arange(c - r, c + r + 1), n)))
    gx, gy, gz = np.meshgrid(*axes, indexing="ij")
    return np.unique((gx + nx * (gy + ny * gz)).ravel())


def sampled_step_outputs(geom, s, df0, steps, samples, radius=None, **kw):
    """f(x, steps) - w rho0 at the sampled global nodes, each computed on its
    own window of half-width steps + 1 from the full initial deviations df0
    (Q, N).  Returns an array (Q, len(samples))."""
    r = steps + 1 if radius is None else radius
    out = np.empty((df0.shape[0], len(samples)))
    for j, n in enumerate(samples):
        nodes = box_window(tuple(geom.shape), int(n), r)
        o = Oracle(geom, s, nodes=nodes, **kw)
        f = o.run(o.init_deviation(df0[:, nodes]), steps)
        loc = int(np.searchsorted(nodes, n))
        out[:, j] = o.as_deviation(f)[:, loc]
    return out
