"""Closed-form steady flows used to measure accuracy (not the method itself)."""

import numpy as np


def couette_utheta(r, u_w, r_in, r_out):
    """Circular Couette flow, inner cylinder (radius r_in) moving at u_w,
    outer (r_out) at rest: u_theta = u_w r_in (r_out^2/r - r)/(r_out^2 - r_in^2)."""
    return u_w * r_in * (r_out ** 2 / r - r) / (r_out ** 2 - r_in ** 2)


def couette_velocity(geom):
    """Analytic (u_x, u_y) at every node of an annulus geometry (N, 2)."""
    m = geom.meta
    x, y, _ = geom.coords()
    dx = x - m["center"][0]
    dy = y - m["center"][1]
    r = np.sqrt(dx * dx + dy * dy)
    with np.errstate(divide="ignore", invalid="ignore"):
        ut = couette_utheta(r, m["u_w"], m["r_in"], m["r_out"])
        ux = -ut * dy / r
        uy = ut * dx / r
    return np.stack([ux, uy], axis=1)


def poiseuille_u(y, U, y_lo, H):
    """Plane Poiseuille profile, the paper's Eq. (52), with y measured from
    the lower wall: u = 4U(1 - s)s, s = (y - y_lo)/H."""
    s = (y - y_lo) / H
    return 4.0 * U * (1.0 - s) * s


def hagen_poiseuille_u(r, U, R):
    """Pipe flow (paper, Section 3.3): u = U(1 - r^2/R^2)."""
    return U * (1.0 - (r / R) ** 2)


def relative_l2(u_num, u_ref, mask):
    """Relative L2 error of a vector field over the masked nodes, the
    paper's E_r: sqrt(sum |u - u*|^2) / sqrt(sum |u|^2)."""
    d = (u_num - u_ref)[mask]
    return float(np.sqrt((d * d).sum() / (u_ref[mask] ** 2).sum()))
