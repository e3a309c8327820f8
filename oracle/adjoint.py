"""Reverse sweep (discrete adjoint) of the oracle step, and the objectives.

TEST INFRASTRUCTURE ONLY (see the package header).

The forward map of one step is the oracle's collide -> stream -> boundary
(lbm.py: Eq. (22a) with the Appendix MRT operator, Eq. (22b), Eq. (213)).
Its reverse, for lambda(t+1) = dJ/df(., t+1):

* a = lambda(t+1) + (direct objective terms on f(t+1));
* the stream part is the transposed gather: every pulled entry
  f_i(x, t+1) = f'_i(src(x, i), t) sends a_i(x) back to f'_i(src(x, i));
* every cut link (x_f, i) sends its a_i(x_f) to f'_i (times c2), f'_ibar
  (times c3), f_i (times c0) and f_ibar (times c1) at x_f -- Eq. (213);
* the collision's Jacobian, per node, is I - M^{-1} S M (I - J_eq) with
  J_eq the derivative of Eq. (42) (formed densely here), applied transposed.

Objectives: the drag (momentum-exchange force), the mean velocity and the
pressure drop between two cross-sections.

Gradients: of the coefficients of Eq. (213) through gamma (l follows the
rule), of the wall velocity phi (of phi(x_b, 0) when the wall data decay as
phi(0) * wall_decay**t), of the body force g and of the relaxation rates s.  Pinned by complex-step differentiation of the forward oracle
(tests/test_oracle_adjoint.py), which is exact to round-off because the
step is a rational function of these parameters.
"""

import numpy as np

from . import scheme as _scheme
from .lbm import Oracle


class Objective:
    """J = sum over steps t in [t0, t1) of j(t) / (t1 - t0), with
    kind "force_x": x momentum-exchange force on `tag` during step t -> t+1,
    kind "mean_ux": mean u_x over fluid nodes of f(t),
    kind "pressure_drop": p_in - p_out of f(t), where p = c_s^2 rho (the
    pressure of the incompressible model, c_s^2 = 1/3 in lattice units) and
    p_in, p_out are its means over the fluid nodes of the planes x = x_in and
    x = x_out (planes = (x_in, x_out); negative values count from nx)."""

    def __init__(self, kind, tag=0, t0=0, t1=1, planes=(0, -1)):
        self.kind, self.tag, self.t0, self.t1 = kind, tag, t0, t1
        self.planes = planes

    def weight(self, t):
        return 1.0 / (self.t1 - self.t0) if self.t0 <= t < self.t1 else 0.0

    def plane_weights(self, o):
        """Per-node weights a(x) with p_in - p_out = c_s^2 sum_x a(x) rho(x):
        1/n_in on the fluid nodes of x_in, -1/n_out on those of x_out."""
        nx = o.shape[0]
        x = o.nodes % nx
        a = np.zeros(o.N)
        for xp, sign in zip(self.planes, (1.0, -1.0)):
            sel = (x == xp % nx) & o.fluid
            if not sel.any():
                raise ValueError("plane x = %d has no fluid node" % (xp % nx))
            a[sel] += sign / sel.sum()
        return a

    def value(self, o, t, f, fp, fn):
        w = self.weight(t)
        if w == 0.0:
            return 0.0
        if self.kind == "force_x":
            nt = max(int(o.lk_tag.max()) + 1 if len(o.lk_tag) else 0, self.tag + 1)
            return w * o.force(fp, fn, n_tags=nt)[self.tag, 0]
        if self.kind == "pressure_drop":
            a = self.plane_weights(o)
            rho = o.density_deviation(f)
            return w * (a[o.fluid] * rho[o.fluid]).sum() / 3.0
        u = o.velocity(f)
        return w * u[0, o.fluid].sum() / o.fluid.sum()


def forward(o, f0, steps, obj):
    """Run the oracle from f0 at time 0 and accumulate the objective;
    returns (J, states)."""
    o.time = 0
    J = 0.0
    states = [f0]
    f = f0
    for t in range(steps):
        fn, fp = o.step(f)
        J = J + obj.value(o, t, f, fp, fn)
        states.append(fn)
        f = fn
    return J, states


def _collision_jacobian_T(o, f, mu):
    """(d f'/d f)^T mu at every node, dense per node."""
    u = o.velocity(f)                                   # (D, N)
    e, w = o.e, o.w
    eu = e @ u                                          # (Q, N)
    # c_i = 3 e_i + 9 (e_i.u) e_i - 3 u  -> (Q, D, N)
    c = 3.0 * e[:, :, None] + 9.0 * eu[:, None, :] * e[:, :, None] - 3.0 * u[None, :, :]
    Jeq = w[:, None, None] * (1.0 + np.einsum("iaN,ja->ijN", c, e))   # (Q, Q, N)
    Q = o.Q
    A = o.Minv @ (o.s[:, None] * o.M)                  # M^{-1} S M
    I = np.eye(Q)
    # J_C = I - A (I - Jeq)  per node; out_j = sum_i J_C[i, j] mu_i
    ImJ = I[:, :, None] - Jeq                           # (Q, Q, N)
    AIJ = np.einsum("ik,kjN->ijN", A, ImJ)
    JC = I[:, :, None] - AIJ
    return np.einsum("ijN,iN->jN", JC, mu)


def reverse(o, states, obj, rule=None):
    """Adjoint sweep over the recorded forward states.  Returns a dict with
    lam0 (dJ/df(., 0)) and the gradients q, wall_u, g, s."""
    steps = len(states) - 1
    Q, D, N = o.Q, o.D, o.N
    fluid = o.fluid
    xf, i, ib = o.lk_node, o.lk_dir, o.lk_opp
    c0, c1, c2, c3, c4 = o.c
    rule = rule or o.l_rule
    d0, d1, d2, d3, d4 = _scheme.coefficient_derivatives(np.real(o.q), rule, o.b)
    unit_e = 3.0 * o.w[i][:, None] * o.rho0 * o.e[i]            # (L, D)

    gq = np.zeros(len(xf))
    gphi = np.zeros((len(xf), D))
    gg = np.zeros(D)
    gs = np.zeros(Q)
    lam = np.zeros((Q, N))
    n_f = fluid.sum()
    for t in range(steps - 1, -1, -1):
        f = states[t]
        fp = o.collide(f)
        fn = states[t + 1]
        wt = obj.weight(t)
        a = lam.copy()
        dmu = np.zeros((Q, N))
        if wt and obj.kind == "force_x":
            sel = o.lk_tag == obj.tag
            ex = o.e[i[sel], 0]
            np.add.at(a, (i[sel], xf[sel]), -ex * wt)
            np.add.at(dmu, (ib[sel], xf[sel]), -ex * wt)
        a[:, ~fluid] = 0.0
        a_link = a[i, xf].copy()
        a_stream = a.copy()
        a_stream[i, xf] = 0.0
        # Eq. (211): the c1 term reads the advected f_ibar(x_f, t+1)
        defer = o.two_node & ~o.lk_ibar_is_link if o.two_node else np.zeros(len(xf), bool)
        np.add.at(a_stream, (ib[defer], xf[defer]), (c1 * a_link)[defer]
                  if np.ndim(c1) else c1 * a_link[defer])
        f_ib = np.where(defer, fn[ib, xf], f[ib, xf])
        mu = np.zeros((Q, N))
        for d in range(Q):
            np.add.at(mu[d], o.src[d, fluid], a_stream[d, fluid])
        mu[:, ~fluid] = 0.0
        mu += dmu
        direct = np.zeros((Q, N))
        np.add.at(mu, (i, xf), c2 * a_link)
        np.add.at(mu, (ib, xf), c3 * a_link)
        np.add.at(direct, (i, xf), c0 * a_link)
        np.add.at(direct, (ib, xf), np.where(defer, 0.0, c1 * a_link))
        # per-link gradients
        ws = o.wall_scale(t)
        gq += a_link * (d0 * f[i, xf] + d1 * f_ib + d2 * fp[i, xf]
                        + d3 * fp[ib, xf] + d4 * o.wall_term * ws)
        gphi += (a_link * c4 * ws)[:, None] * unit_e
        # body force and rates
        muf = np.where(fluid[None, :], mu, 0.0)
        gg += (3.0 * o.w[:, None] * o.rho0 * muf).T.sum(0) @ o.e
        feq = o.equilibrium(o.density_deviation(f), o.velocity(f))
        m_neq = o.M @ np.where(fluid[None, :], f - feq, 0.0)
        gs -= ((o.Minv.T @ muf) * m_neq).sum(1)
        # collision adjoint
        fz = np.where(fluid[None, :], f, 0.0)
        lam = _collision_jacobian_T(o, fz, muf) + direct
        if wt and obj.kind == "mean_ux":
            lam += (wt * o.e[:, 0] / (o.rho0 * n_f))[:, None]
        if wt and obj.kind == "pressure_drop":
            lam += (wt / 3.0) * obj.plane_weights(o)[None, :]
        lam[:, ~fluid] = 0.0
    return dict(lam0=lam, q=gq, wall_u=gphi, g=gg, s=gs)


def complex_step(make_oracle, f0, steps, obj, h=1e-30):
    """Return a function p -> dJ/dp for a complex perturbation built by
    make_oracle(perturbation) (complex-step differentiation)."""
    def deriv(pert):
        o = make_oracle(1j * h * pert)
        J, _ = forward(o, f0.astype(complex), steps, obj)
        return np.imag(J) / h
    return deriv
