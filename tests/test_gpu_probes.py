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
    P = binding.population_elements(lattice, shape)
    idx = binding.population_index(lattice, shape)
    assert P % (Q * 2048) == 0 and idx.max() < P
    rng = np.random.default_rng(7)
    src_h = rng.standard_normal(P)
    src = torch.tensor(src_h, dtype=dt, device="cuda")
    dst = torch.full_like(src, float("nan"))
    ms = binding.pull_pattern_copy(lattice, precision, dst, src, shape, reps=2)
    assert ms > 0
    got = dst.cpu().numpy().astype(np.float64)
    s_all = torch.tensor(src_h, dtype=dt).numpy().astype(np.float64)
    s3 = s_all[idx].reshape(Q, nz, ny, nx)
    for i in range(Q):
        ex = int(e[i, 0]); ey = int(e[i, 1]); ez = int(e[i, 2]) if e.shape[1] == 3 else 0
        want = np.roll(s3[i], shift=(ez, ey, ex), axis=(0, 1, 2)).reshape(n)
        assert np.array_equal(got[idx[i]], want), i
    # the block tail past the last node is neither read nor written
    tail = np.ones(P, bool)
    tail[idx.ravel()] = False
    assert np.isnan(got[tail]).all()


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
    P = binding.population_elements(lattice, shape)
    idx = torch.from_numpy(binding.population_index(lattice, shape))
    rng = np.random.default_rng(8)
    f_h = rng.standard_normal(P)
    l_h = rng.standard_normal(P)
    f = torch.tensor(f_h, dtype=dt, device="cuda")
    lam = torch.tensor(l_h, dtype=dt, device="cuda")
    dst = torch.full_like(f, float("nan"))
    assert binding.adjoint_pattern_copy(lattice, precision, dst, f, lam, shape, reps=2) > 0
    got = dst.cpu()
    f3 = f.cpu()[idx].reshape(Q, nz, ny, nx)
    l3 = lam.cpu()[idx].reshape(Q, nz, ny, nx)
    for i in range(Q):
        ex = int(e[i, 0]); ey = int(e[i, 1]); ez = int(e[i, 2]) if e.shape[1] == 3 else 0
        pulled = torch.roll(f3[i], shifts=(ez, ey, ex), dims=(0, 1, 2))
        pushed = torch.roll(l3[i], shifts=(-ez, -ey, -ex), dims=(0, 1, 2))
        assert torch.equal(got[idx[i]], (pulled + pushed).reshape(n)), i


def test_pull_pattern_copy_rejects_bad_sizes():
    import torch
    from paper_1712_08288_amd import binding
    a = torch.zeros(19 * 2048, device="cuda")
    with pytest.raises(binding.LBMError):
        binding.pull_pattern_copy("D2Q9", "fp32", a, a.clone(), (2, 2, 2))
    with pytest.raises(binding.LBMError):
        binding.pull_pattern_copy("D3Q19", "fp32", a, a.clone(), (0, 2, 2))
    # buffers smaller than whole population blocks are refused before launch
    with pytest.raises(binding.LBMError):
        binding.pull_pattern_copy("D3Q19", "fp32", a[:19 * 8], a[:19 * 8].clone(), (2, 2, 2))


def test_stream_copy_copies():
    import torch
    from paper_1712_08288_amd import binding
    a = torch.arange(1 << 16, dtype=torch.float32, device="cuda")
    for mode in (0, 1, 2):
        b = torch.zeros_like(a)
        assert binding.stream_copy(b, a, a.numel() * 4, mode=mode, reps=2) > 0
        assert torch.equal(a, b)


@pytest.mark.parametrize("block", [64, 512])
def test_blocked_pull_pattern_copy_is_the_periodic_pull(block):
    import torch
    from paper_1712_08288_amd import binding
    lattice, shape = "D3Q19", (16, 8, 4)
    e, _, _ = binding.lattice_info(lattice)
    Q = e.shape[0]
    nx, ny, nz = shape
    n = nx * ny * nz
    idx = (np.arange(n) // block) * Q * block + np.arange(Q)[:, None] * block + np.arange(n) % block
    rng = np.random.default_rng(9)
    src_h = rng.standard_normal(Q * n)
    src = torch.tensor(src_h, dtype=torch.float64, device="cuda")
    dst = torch.full_like(src, float("nan"))
    assert binding.blocked_pull_pattern_copy(lattice, "fp64", block, dst, src, shape, reps=2) > 0
    got = dst.cpu().numpy()
    s3 = src_h[idx].reshape(Q, nz, ny, nx)
    for i in range(Q):
        want = np.roll(s3[i], shift=(int(e[i, 2]), int(e[i, 1]), int(e[i, 0])), axis=(0, 1, 2))
        assert np.array_equal(got[idx[i]], want.reshape(n)), i
    with pytest.raises(binding.LBMError):   # the block must divide the node count
        binding.blocked_pull_pattern_copy(lattice, "fp64", 1024, dst, src, shape, reps=1)


def test_aa_pattern_copy_permutes_in_place():
    import torch
    from paper_1712_08288_amd import binding
    lattice, shape = "D3Q19", (6, 5, 4)
    n = int(np.prod(shape))
    buf = torch.arange(19 * n, dtype=torch.float64, device="cuda")
    ms_even, ms_odd = binding.aa_pattern_copy(lattice, "fp64", buf, shape, reps=2)
    assert ms_even > 0 and ms_odd > 0
    # both passes move every value to exactly one place: a permutation
    assert torch.equal(torch.sort(buf.cpu()).values, torch.arange(19 * n, dtype=torch.float64))
