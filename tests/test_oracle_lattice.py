"""Pins of the oracle's lattice tables and equilibrium (CPU only).

The tables are checked against facts fixed outside the oracle: weight
moments of an isotropic lattice, orthogonality and the published row norms
of the moment matrices (tests/golden/lattice_norms.json), the moment
polynomials that define the printed matrices, and the published
moment-space equilibria (tests/golden/moment_equilibria.json).
"""

import json
import os

import numpy as np
import pytest

from oracle import lattice as L
from oracle.lbm import Oracle
from workloads import geometry as G
from workloads.velocities import VELOCITIES

GOLD = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("name", ["D2Q9", "D3Q15", "D3Q19"])
def test_weight_moments(name):
    lat = L.get(name)
    e = lat.e.astype(float)
    assert abs(lat.w.sum() - 1.0) < 1e-15
    assert np.abs(lat.w @ e).max() < 1e-15
    second = np.einsum("i,ia,ib->ab", lat.w, e, e)
    assert np.allclose(second, np.eye(lat.D) / 3.0, atol=1e-15)
    # fourth-order isotropy: sum w e_a e_b e_c e_d = (d_ab d_cd + d_ac d_bd + d_ad d_bc)/9
    fourth = np.einsum("i,ia,ib,ic,id->abcd", lat.w, e, e, e, e)
    I = np.eye(lat.D)
    iso = (np.einsum("ab,cd->abcd", I, I) + np.einsum("ac,bd->abcd", I, I)
           + np.einsum("ad,bc->abcd", I, I)) / 9.0
    assert np.allclose(fourth, iso, atol=1e-15)


@pytest.mark.parametrize("name", ["D2Q9", "D3Q15", "D3Q19"])
def test_moment_matrix_norms(name):
    gold = json.load(open(os.path.join(GOLD, "lattice_norms.json")))[name]
    M = L.get(name).M
    MMt = M @ M.T
    assert np.allclose(MMt, np.diag(np.diag(MMt)), atol=0)
    assert np.array_equal(np.diag(MMt), np.array(gold, dtype=float))
    # inverse equals M^T D^-1 for an orthogonal-row matrix
    assert np.allclose(L.get(name).Minv, M.T / np.diag(MMt)[None, :], atol=1e-15)


def test_d2q9_printed_matrix_is_the_moment_polynomials():
    """Paper Appendix D2Q9 M against the Lallemand-Luo polynomials."""
    lat = L.get("D2Q9")
    ex, ey = lat.e[:, 0].astype(float), lat.e[:, 1].astype(float)
    e2 = ex * ex + ey * ey
    poly = np.array([np.ones(9), 3 * e2 - 4, (9 * e2 * e2 - 21 * e2 + 8) / 2,
                     ex, (3 * e2 - 5) * ex, ey, (3 * e2 - 5) * ey,
                     ex * ex - ey * ey, ex * ey])
    assert np.array_equal(lat.M, poly)


def test_d3q15_printed_matrix_is_the_moment_polynomials():
    """Paper Appendix D3Q15 M against the d'Humieres et al. polynomials."""
    lat = L.get("D3Q15")
    ex, ey, ez = (lat.e[:, a].astype(float) for a in range(3))
    e2 = ex * ex + ey * ey + ez * ez
    poly = np.array([np.ones(15), e2 - 2, (15 * e2 * e2 - 55 * e2 + 32) / 2,
                     ex, (5 * e2 - 13) / 2 * ex, ey, (5 * e2 - 13) / 2 * ey,
                     ez, (5 * e2 - 13) / 2 * ez, 3 * ex * ex - e2,
                     ey * ey - ez * ez, ex * ey, ey * ez, ex * ez, ex * ey * ez])
    assert np.array_equal(lat.M, poly)


@pytest.mark.parametrize("name", ["D2Q9", "D3Q15", "D3Q19"])
def test_velocity_tables_agree_with_input_generators(name):
    assert np.array_equal(L.get(name).e, VELOCITIES[name])


def _basis(D, drho, u, rho0=1.0):
    j = rho0 * u
    jx, jy = j[0], j[1]
    jz = j[2] if D == 3 else 0.0 * jx
    jj = (j * j).sum(0) / rho0
    return np.array([drho, jj, jx, jy, jz, (jx * jx - jy * jy) / rho0,
                     jx * jy / rho0, (2 * jx * jx - jy * jy - jz * jz) / rho0,
                     (jy * jy - jz * jz) / rho0, jy * jz / rho0, jx * jz / rho0])


@pytest.mark.parametrize("name", ["D2Q9", "D3Q19"])
def test_equilibrium_moments_match_published(name):
    gold = np.array(json.load(open(os.path.join(GOLD, "moment_equilibria.json")))[name])
    shape = (3, 2, 1) if name == "D2Q9" else (2, 2, 2)
    o = Oracle(G.empty(name, shape), np.zeros(L.get(name).Q))
    rng = np.random.default_rng(7)
    n = o.N
    drho = rng.uniform(-0.01, 0.01, n)
    u = rng.uniform(-0.05, 0.05, (o.D, n))
    feq = o.equilibrium(drho, u)
    m = o.M @ feq
    want = gold @ _basis(o.D, drho, u)
    assert np.allclose(m, want, atol=1e-15, rtol=1e-13)


@pytest.mark.parametrize("name", ["D2Q9", "D3Q15", "D3Q19"])
def test_equilibrium_conserved_moments(name):
    lat = L.get(name)
    shape = (3, 2, 1) if lat.D == 2 else (2, 2, 2)
    o = Oracle(G.empty(name, shape), np.zeros(lat.Q), rho0=1.3)
    rng = np.random.default_rng(1)
    rho = rng.uniform(-0.01, 0.01, o.N)
    u = rng.uniform(-0.05, 0.05, (o.D, o.N))
    feq = o.equilibrium(rho, u)
    assert np.allclose(feq.sum(0), rho, atol=1e-16)
    assert np.allclose(o.e.T @ feq, 1.3 * u, atol=1e-16)
