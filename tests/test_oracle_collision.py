"""Pins of the oracle's TRT / BGK collision (Remark (1): the boundary scheme
is independent of the collision operator).

* TRT relaxes the even and odd halves of f - f^eq; every moment row of the
  Appendix matrices (and of the D3Q19 polynomials) is even or odd under
  e -> -e, so TRT equals the MRT operator whose even rows relax at s_plus
  and odd rows at s_minus.  The two oracle paths share no arithmetic (dense
  M and M^-1 against a half-sum split), so a swapped rate, a sign in the odd
  half or a wrong opposite table fails the comparison.
* Collision conserves mass and momentum.
* Poiseuille flow converges at second order with BGK and TRT under the
  single-node scheme, as it does with MRT (Section 3.1).
"""

import numpy as np
import pytest

from oracle import lattice as L
from oracle.lbm import Oracle
from test_oracle_physics import order, poiseuille_error
from workloads import geometry as G
from workloads import states


def parity_rates(lattice, s_plus, s_minus):
    lat = L.get(lattice)
    even = np.all(lat.M[:, lat.opp] == lat.M, axis=1)
    odd = np.all(lat.M[:, lat.opp] == -lat.M, axis=1)
    assert np.all(even ^ odd)
    return np.where(even, s_plus, s_minus)


def magic_minus(s_plus, magic):
    return 1.0 / (0.5 + magic / (1.0 / s_plus - 0.5))


GEOMS = {
    "D2Q9": lambda: G.random_cylinders(23, 19, 2, 2.5, 3.5, seed=3),
    "D3Q15": lambda: G.random_spheres(11, 9, 8, 1, 1.9, 2.6, seed=5, lattice="D3Q15"),
    "D3Q19": lambda: G.random_spheres(11, 9, 8, 1, 1.9, 2.6, seed=5),
}


@pytest.mark.parametrize("lattice", ["D2Q9", "D3Q15", "D3Q19"])
@pytest.mark.parametrize("s_plus,magic", [(1.3, 3 / 16), (0.7, 0.25), (1.9, 1 / 12)])
def test_trt_equals_mrt_with_parity_rates(lattice, s_plus, magic):
    geom = GEOMS[lattice]()
    s_minus = magic_minus(s_plus, magic)
    g = (2e-5, -1e-5, 3e-6)
    trt = Oracle(geom, np.zeros(len(L.get(lattice).w)), g=g, collision=("trt", s_plus, s_minus))
    mrt = Oracle(geom, parity_rates(lattice, s_plus, s_minus), g=g)
    f = trt.init_deviation(states.random_deviation(trt.Q, trt.N, seed=7, amp=1e-2))
    a, b = trt.collide(f), mrt.collide(f)
    fl = trt.fluid
    assert np.allclose(a[:, fl], b[:, fl], rtol=0, atol=1e-15)
    # a whole step including the boundary scheme
    na, _ = trt.step(f)
    nb, _ = mrt.step(f)
    assert np.allclose(na[:, fl], nb[:, fl], rtol=0, atol=1e-15)


@pytest.mark.parametrize("lattice", ["D2Q9", "D3Q15", "D3Q19"])
def test_trt_and_bgk_conserve_mass_and_momentum(lattice):
    geom = GEOMS[lattice]()
    Q = len(L.get(lattice).w)
    for col in (("trt", 1.2, 0.8), ("bgk", 1.7)):
        o = Oracle(geom, np.zeros(Q), collision=col)
        f = o.init_deviation(states.random_deviation(Q, o.N, seed=2, amp=1e-2))
        fp = o.collide(f)
        fl = o.fluid
        assert np.allclose(fp[:, fl].sum(0), f[:, fl].sum(0), rtol=0, atol=1e-15)
        assert np.allclose(o.e.T @ fp[:, fl], o.e.T @ f[:, fl], rtol=0, atol=1e-15)
        # and it relaxes: the non-equilibrium part shrinks
        feq = o.equilibrium(o.density_deviation(f), o.velocity(f))
        assert np.linalg.norm((fp - feq)[:, fl]) < np.linalg.norm((f - feq)[:, fl])


@pytest.mark.parametrize("collision", ["bgk", "trt"])
@pytest.mark.parametrize("rule,gamma", [("gamma", 0.25), ("min", 0.75), ("gamma2", 1.0)])
def test_poiseuille_second_order_other_collisions(collision, rule, gamma):
    sizes = [11, 21, 41]
    s_nu = 1.2
    col = ("bgk", s_nu) if collision == "bgk" else ("trt", s_nu, magic_minus(s_nu, 3 / 16))
    errs = [poiseuille_error(n, gamma, s_nu, rule, collision=col) for n in sizes]
    p = order([n - 2 + 2 * gamma for n in sizes], errs)
    assert 1.85 < p < 2.15, (errs, p)
