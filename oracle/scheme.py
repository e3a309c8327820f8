"""The free parameter l(gamma) and the coefficients of the boundary scheme.

Paper, Section 2:
* Eq. (210): single-node scheme, coefficients (1+l-2g)/(1+l) on the
  pre-collision f_{i-bar}(x_f, t), l/(1+l) on f'_i(x_f, t), (2g-l)/(1+l) on
  f'_{i-bar}(x_f, t) and 2/(1+l) on the bounce-back wall term
  w_i h rho0 e_i.phi / (dt c_s^2) (= 3 w_i rho0 e_i.phi in lattice units).
* Eq. (212): the convexity band max{0, 2g - 1} <= l <= 2g.
* Eq. (213): (1 - b) f_i(x_f, t) + b [right-hand side of Eq. (210)].
* Section 3 tests five rules: l = g, 1.5g, 2g, g^2, g^2 + g.  Two more are
  offered: l = 0 (nonconvex for g > 1/2, Remark (5)) and l = max(0, 2g-1),
  the lower edge of Eq. (212), the only listed rule besides l = 0 that gives
  l(1/2) = 0 and so reproduces half-way bounce-back at g = 1/2.

Pinned by: sum of the five coefficients c0..c3 = 1, convexity, the special
cases of Remarks (3)-(5), and the reduction to half-way bounce-back
(tests/test_oracle_scheme.py).  Works on real or complex gamma (complex-step
derivatives); branch decisions use the real part.
"""

import numpy as np

RULES = ("gamma", "1.5gamma", "2gamma", "gamma2", "gamma2+gamma", "zero", "min")


def l_of_gamma(rule, g):
    g = np.asarray(g)
    if rule == "gamma":
        return g * 1.0
    if rule == "1.5gamma":
        return 1.5 * g
    if rule == "2gamma":
        return 2.0 * g
    if rule == "gamma2":
        return g * g
    if rule == "gamma2+gamma":
        return g * g + g
    if rule == "zero":
        return g * 0.0
    if rule == "min":
        return np.where(np.real(2.0 * g - 1.0) > 0.0, 2.0 * g - 1.0, 0.0 * g)
    raise ValueError(rule)


def dl_dgamma(rule, g):
    g = np.asarray(g, dtype=np.float64)
    one = np.ones_like(g)
    return {"gamma": one, "1.5gamma": 1.5 * one, "2gamma": 2.0 * one,
            "gamma2": 2.0 * g, "gamma2+gamma": 2.0 * g + 1.0,
            "zero": 0.0 * one,
            "min": np.where(2.0 * g - 1.0 > 0.0, 2.0, 0.0)}[rule]


def convex(g, l):
    """Eq. (212)."""
    g = np.real(np.asarray(g))
    l = np.real(np.asarray(l))
    return (l >= np.maximum(0.0, 2.0 * g - 1.0)) & (l <= 2.0 * g)


def coefficients(g, l, b=1.0):
    """(c0, c1, c2, c3, c4) of Eq. (213); with b = 1 those of Eq. (210).

    f_i(x_f, t+1) = c0 f_i(x_f,t) + c1 f_ibar(x_f,t) + c2 f'_i(x_f,t)
                    + c3 f'_ibar(x_f,t) + c4 * 3 w_i rho0 e_i.phi(x_b,t)
    """
    g = np.asarray(g)
    l = np.asarray(l)
    c0 = (1.0 - b) + 0.0 * g
    c1 = b * (1.0 + l - 2.0 * g) / (1.0 + l)
    c2 = b * l / (1.0 + l)
    c3 = b * (2.0 * g - l) / (1.0 + l)
    c4 = b * 2.0 / (1.0 + l)
    return c0, c1, c2, c3, c4


def coefficient_derivatives(g, rule, b=1.0):
    """d c_k / d gamma along l = l(gamma) (chain rule through the rule)."""
    g = np.asarray(g, dtype=np.float64)
    l = l_of_gamma(rule, g)
    lp = dl_dgamma(rule, g)
    den = 1.0 + l
    # partial derivatives with respect to gamma (l fixed) and to l
    d1 = b * (-2.0 / den + lp * ((1.0 / den) - (1.0 + l - 2.0 * g) / den ** 2))
    d2 = b * lp * (1.0 / den - l / den ** 2)
    d3 = b * (2.0 / den + lp * (-1.0 / den - (2.0 * g - l) / den ** 2))
    d4 = b * lp * (-2.0 / den ** 2)
    return 0.0 * g, d1, d2, d3, d4
