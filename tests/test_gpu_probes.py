"""The measurement probes of the library move data as their headers state:
the pull-pattern probe (the step's addressing without arithmetic) writes
plane i at node x from node x - e_i of the source (periodic in every axis),
and the streaming copy copies."""

import numpy as np
import pytest

from gpu_util import require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()


@pytest.mark.parametrize("lattice,shape,precision", [
    ("D3Q19", (10, 7, 5), "fp32"), ("D3Q19", (300, 3, 2), "fp64"),
    ("D3Q15", (9, 6, 4), "fp32"), ("D2Q9", (13, 11, 1), "fp64")])
def test_pull_pattern_copy_is_the_periodic_pull(lattice, shape, precision):
    import torch
    from paper_1712_08288_amd import binding
    e, _, _ = binding.lattice_info(lattice)
    Q = e.shape[0]
    nx, ny, nz = shape
    n = nx * ny * nz
    dt = torch.float32 if precision == "fp32" else torch.float64
    rng = np.random.default_rng(7)
    src_h = rng.standard_normal((Q, n))
    src = torch.tensor(src_h, dtype=dt, device="cuda").contiguous()
    dst = torch.full_like(src, float("nan"))
    ms = binding.pull_pattern_copy(lattice, precision, dst, src, shape, reps=2)
    assert ms > 0
    got = dst.cpu().numpy().astype(np.float64)
    s3 = torch.tensor(src_h, dtype=dt).numpy().astype(np.float64).reshape(Q, nz, ny, nx)
    for i in range(Q):
        ex = int(e[i, 0]); ey = int(e[i, 1]); ez = int(e[i, 2]) if e.shape[1] == 3 else 0
        want = np.roll(s3[i], shift=(ez, ey, ex), axis=(0, 1, 2)).reshape(n)
        assert np.array_equal(got[i], want), i


@pytest.mark.parametrize("lattice,shape,precision", [
    ("D3Q19", (11, 6, 5), "fp32"), ("D2Q9", (7, 9, 1), "fp64")])
def test_adjoint_pattern_copy_reads_pull_and_push_sources(lattice, shape, precision):
    import torch
    from paper_1712_08288_amd import binding
    e, _, _ = binding.lattice_info(lattice)
    Q = e.shape[0]
    nx, ny, nz = shape
    n = nx * ny * nz
    dt = torch.float32 if precision == "fp32" else torch.float64
    rng = np.random.default_rng(8)
    f_h = rng.standard_normal((Q, n))
    l_h = rng.standard_normal((Q, n))
    f = torch.tensor(f_h, dtype=dt, device="cuda").contiguous()
    lam = torch.tensor(l_h, dtype=dt, device="cuda").contiguous()
    dst = torch.full_like(f, float("nan"))
    assert binding.adjoint_pattern_copy(lattice, precision, dst, f, lam, shape, reps=2) > 0
    got = dst.cpu()
    f3 = f.cpu().reshape(Q, nz, ny, nx)
    l3 = lam.cpu().reshape(Q, nz, ny, nx)
    for i in range(Q):
        ex = int(e[i, 0]); ey = int(e[i, 1]); ez = int(e[i, 2]) if e.shape[1] == 3 else 0
        pulled = torch.roll(f3[i], shifts=(ez, ey, ex), dims=(0, 1, 2))
        pushed = torch.roll(l3[i], shifts=(-ez, -ey, -ex), dims=(0, 1, 2))
        assert torch.equal(got[i], (pulled + pushed).reshape(n)), i


def test_pull_pattern_copy_rejects_bad_sizes():
    import torch
    from paper_1712_08288_amd import binding
    a = torch.zeros(19 * 8, device="cuda")
    with pytest.raises(binding.LBMError):
        binding.pull_pattern_copy("D2Q9", "fp32", a, a.clone(), (2, 2, 2))
    with pytest.raises(binding.LBMError):
        binding.pull_pattern_copy("D3Q19", "fp32", a, a.clone(), (0, 2, 2))


def test_stream_copy_copies():
    import torch
    from paper_1712_08288_amd import binding
    a = torch.arange(1 << 16, dtype=torch.float32, device="cuda")
    for mode in (0, 1, 2):
        b = torch.zeros_like(a)
        assert binding.stream_copy(b, a, a.numel() * 4, mode=mode, reps=2) > 0
        assert torch.equal(a, b)
