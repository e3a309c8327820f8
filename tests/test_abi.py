"""The C-ABI library loads, exports every symbol include/lbm.h declares, and
its lattice tables agree with the oracle's and the input generators'
(no GPU needed: none of these calls touches a device)."""

import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbm.h")
PROBE_HEADER = os.path.join(ROOT, "include", "lbm_probe.h")


def _declared(path=HEADER):
    text = open(path).read()
    return sorted(set(re.findall(r"\b(lbm_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def binding():
    from paper_1712_08288_amd import binding
    return binding


def test_library_exports_every_declared_symbol(binding):
    lib = ctypes.CDLL(binding.LIB_PATH)
    names = _declared()
    probes = _declared(PROBE_HEADER)
    assert len(names) >= 25 and len(probes) >= 4
    for n in names + probes:
        assert hasattr(lib, n), n
    assert sorted(binding.EXPORTED) == names
    assert sorted(binding.EXPORTED_PROBES) == probes


@pytest.mark.parametrize("lattice", ["D2Q9", "D3Q15", "D3Q19"])
def test_lattice_tables_agree(binding, lattice):
    from oracle import lattice as L
    from workloads.velocities import VELOCITIES
    e, w, M = binding.lattice_info(lattice)
    lat = L.get(lattice)
    assert np.array_equal(e, lat.e)
    assert np.array_equal(e, VELOCITIES[lattice])
    assert np.allclose(w, lat.w, rtol=0, atol=1e-17)
    assert np.array_equal(M, lat.M)


def test_create_rejects_bad_arguments_before_touching_a_device(binding):
    lib = binding._lib
    h = ctypes.c_void_p()
    s = (ctypes.c_double * 19)(*([1.0] * 19))
    g = (ctypes.c_double * 3)(0, 0, 0)
    EINVAL = -1
    assert lib.lbm_create(ctypes.byref(h), 7, 0, 8, 8, 1, s, 1.0, g) == EINVAL
    assert lib.lbm_create(ctypes.byref(h), 0, 3, 8, 8, 1, s, 1.0, g) == EINVAL
    assert lib.lbm_create(ctypes.byref(h), 0, 0, 8, 8, 2, s, 1.0, g) == EINVAL
    assert lib.lbm_create(ctypes.byref(h), 0, 0, 0, 8, 1, s, 1.0, g) == EINVAL
    assert lib.lbm_create(ctypes.byref(h), 0, 0, 8, 8, 1, s, -1.0, g) == EINVAL
    bad = (ctypes.c_double * 19)(*([1.0] * 8 + [2.5] + [1.0] * 10))
    assert lib.lbm_create(ctypes.byref(h), 0, 0, 8, 8, 1, bad, 1.0, g) == EINVAL
    assert lib.lbm_create(ctypes.byref(h), 1, 0, 1 << 11, 1 << 11, 1 << 10, s, 1.0, g) == EINVAL
    assert not h.value


def test_lattice_info_rejects_unknown_lattice(binding):
    assert binding._lib.lbm_lattice_info(5, None, None, None, None, None) == -1


def test_create_rejects_planes_of_4gib_or_more(binding):
    """One direction plane must stay below 4 GiB (32-bit byte offsets):
    rejected at create, before any device call."""
    lib = binding._lib
    h = ctypes.c_void_p()
    s = (ctypes.c_double * 19)(*([1.0] * 19))
    g = (ctypes.c_double * 3)(0, 0, 0)
    EINVAL = -1
    assert lib.lbm_create(ctypes.byref(h), 1, 1, 1024, 1024, 1024, s, 1.0, g) == EINVAL
    assert lib.lbm_create(ctypes.byref(h), 1, 0, 1024, 1024, 512, s, 1.0, g) == EINVAL


@pytest.mark.parametrize("lattice", ["D2Q9", "D3Q15", "D3Q19"])
@pytest.mark.parametrize("kind", ["bgk", "trt"])
def test_collision_rates_follow_the_row_parity(binding, lattice, kind):
    """lbm_collision_rates (no GPU): even moment rows get s_nu, odd rows
    s_minus from (1/s_nu - 1/2)(1/s_minus - 1/2) = magic (BGK: s_nu), with
    the row parity taken from the oracle's own moment matrix."""
    from oracle import lattice as L
    lat = L.get(lattice)
    even = np.all(lat.M[:, lat.opp] == lat.M, axis=1)
    s_nu, magic = 1.3, 0.21
    got = binding.collision_rates(lattice, kind, s_nu, magic)
    s_minus = s_nu if kind == "bgk" else 1.0 / (0.5 + magic / (1.0 / s_nu - 0.5))
    assert np.allclose(got, np.where(even, s_nu, s_minus), rtol=0, atol=1e-15)
    if kind == "trt":
        assert abs((1 / s_nu - 0.5) * (1 / got[~even][0] - 0.5) - magic) < 1e-14
    with pytest.raises(binding.LBMError):
        binding.collision_rates(lattice, kind, 2.0, magic)
