"""Pins of the boundary-scheme coefficients (paper, Section 2)."""

import numpy as np
import pytest

from oracle import scheme as S

PAPER_RULES = ("gamma", "1.5gamma", "2gamma", "gamma2", "gamma2+gamma")
G = np.linspace(1e-6, 1.0, 2001)


@pytest.mark.parametrize("rule", S.RULES)
@pytest.mark.parametrize("b", [1.0, 0.7, 0.2])
def test_coefficients_sum_to_one(rule, b):
    c0, c1, c2, c3, c4 = S.coefficients(G, S.l_of_gamma(rule, G), b)
    assert np.allclose(c0 + c1 + c2 + c3, 1.0, atol=1e-15)


@pytest.mark.parametrize("rule", PAPER_RULES + ("min",))
def test_paper_rules_are_convex_on_unit_interval(rule):
    """Eq. (212) holds on (0, 1] for the five tested rules and max(0,2g-1);
    then every coefficient lies in [0, 1] (a convex combination)."""
    l = S.l_of_gamma(rule, G)
    assert S.convex(G, l).all()
    for c in S.coefficients(G, l, 1.0)[:4]:
        assert (c >= -1e-15).all() and (c <= 1 + 1e-15).all()


def test_l_zero_is_nonconvex_above_half():
    """Remark (5): l = 0 is the nonconvex member: c1 = 1 - 2g < 0 for g > 1/2."""
    l = S.l_of_gamma("zero", G)
    assert not S.convex(G[G > 0.5], l[G > 0.5]).any()
    assert S.convex(G[G <= 0.5], l[G <= 0.5]).all()


def test_remark_4_single_node_special_case():
    """Remark (4): with l = gamma, Eq. (210) is the scheme printed there:
    (1-g)/(1+g) f_ibar(x_f,t) + g/(1+g) [f'_i + f'_ibar] + 2/(1+g) wall."""
    c0, c1, c2, c3, c4 = S.coefficients(G, S.l_of_gamma("gamma", G), 1.0)
    assert np.allclose(c1, (1 - G) / (1 + G), atol=1e-15)
    assert np.allclose(c2, G / (1 + G), atol=1e-15)
    assert np.allclose(c3, G / (1 + G), atol=1e-15)
    assert np.allclose(c4, 2 / (1 + G), atol=1e-15)
    assert np.all(c0 == 0.0)


@pytest.mark.parametrize("rule", ["zero", "min"])
def test_half_gamma_is_half_way_bounce_back(rule):
    """Eq. (26) with x_1 = x_2 = x_f: at gamma = 1/2 and l(1/2) = 0 the scheme
    reduces to f_i(x_f, t+1) = f'_ibar(x_f, t) + 2 * wall term."""
    c0, c1, c2, c3, c4 = S.coefficients(0.5, S.l_of_gamma(rule, 0.5), 1.0)
    assert (c0, c1, c2, c3, c4) == (0.0, 0.0, 0.0, 1.0, 2.0)


@pytest.mark.parametrize("rule", PAPER_RULES)
def test_paper_rules_are_not_bounce_back_at_half(rule):
    """l(1/2) > 0 for the five tested rules, so at gamma = 1/2 they keep a
    share of f_ibar(x_f, t) and f'_i and are not half-way bounce-back."""
    c0, c1, c2, c3, c4 = S.coefficients(0.5, S.l_of_gamma(rule, 0.5), 1.0)
    assert c3 < 1.0 and c1 > 0.0 and c2 > 0.0


def test_b_one_reduces_213_to_210():
    l = S.l_of_gamma("gamma2", G)
    a = S.coefficients(G, l, 1.0)
    assert np.all(a[0] == 0.0)
    b = S.coefficients(G, l, 0.4)
    for k in range(1, 5):
        assert np.allclose(b[k], 0.4 * a[k], atol=1e-16)
    assert np.allclose(b[0], 0.6)


@pytest.mark.parametrize("rule", S.RULES)
def test_coefficient_derivatives_by_complex_step(rule):
    g = np.linspace(0.01, 0.99, 97)
    g = g[np.abs(g - 0.5) > 1e-3]       # the "min" rule has a kink at 1/2
    h = 1e-30
    cs = S.coefficients(g + 1j * h, S.l_of_gamma(rule, g + 1j * h), 0.8)
    d = S.coefficient_derivatives(g, rule, 0.8)
    for k in range(5):
        assert np.allclose(np.imag(cs[k]) / h, d[k], atol=1e-14, rtol=1e-13)
