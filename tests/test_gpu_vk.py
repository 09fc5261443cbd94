"""GPU parity of the variable-coefficient step with a source (the paper's
own equation, Eq. 1-4) against the CPU oracle.

The kernels evaluate the oracle's expression in the same order and
precision without contraction, so every comparison is bit-for-bit, for the
Interior/Boundary split (one and several slabs), the fused z-march, the
one-thread-per-node form, every built tile shape, FP64 and FP32.  Shapes
span several tiles and z-blocks and end in ragged tails; the paper's test
case (Eq. 2, 3, 5) runs at 66^3 and in full at 512^3.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2608_11882_amd import inputs

pytestmark = pytest.mark.gpu


def note(msg):
    print("[case] " + msg, flush=True)


def gpu_vk(hc, u0, kappa, rhs, beta, steps, mode="split", parts=1):
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    u, k, f = t(u0), t(kappa), t(rhs)
    un = torch.empty_like(u)
    hc.heat_vk_step(u, un, k, f, beta, steps, mode=mode, parts=parts)
    torch.cuda.synchronize()
    return u.cpu().numpy()


def random_case(dims, seed, dtype=np.float64):
    nx, ny, nz = dims
    u0 = inputs.uniform_field(nx, ny, nz, seed=seed, dtype=dtype)
    kappa, rhs = inputs.random_coefficients(nx, ny, nz, seed=seed + 1, dtype=dtype)
    return u0, kappa, rhs


@pytest.mark.parametrize("mode", ["split", "fused", "plain"])
def test_papers_test_case_66_bitwise(gpu, mode, time_block):
    note("vk paper problem 66^3, 60 steps, mode=%s" % mode)
    pb = inputs.paper_problem(66)
    want = oracle.heat_vk(pb["u0"], pb["kappa"], pb["rhs"], pb["beta"], 60)
    got = gpu_vk(gpu, pb["u0"], pb["kappa"], pb["rhs"], pb["beta"], 60, mode=mode)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("dims", [(3, 3, 3), (5, 4, 3), (130, 9, 7), (67, 33, 41),
                                  (260, 12, 70), (1029, 6, 5), (64, 131, 36)])
@pytest.mark.parametrize("mode", ["split", "fused", "plain"])
def test_random_coefficients_bitwise(gpu, dims, mode, time_block):
    note("vk random %s mode=%s" % (dims, mode))
    u0, kappa, rhs = random_case(dims, seed=sum(dims))
    for steps in (1, 4):
        want = oracle.heat_vk(u0, kappa, rhs, 0.04, steps)
        got = gpu_vk(gpu, u0, kappa, rhs, 0.04, steps, mode=mode)
        assert np.array_equal(got, want), (dims, mode, steps)


@pytest.mark.parametrize("parts", [2, 3, 7, 16])
def test_split_into_slabs_bitwise(gpu, parts, time_block):
    dims = (70, 20, 40)
    note("vk split parts=%d %s" % (parts, dims))
    u0, kappa, rhs = random_case(dims, seed=3)
    want = oracle.heat_vk(u0, kappa, rhs, 0.035, 5)
    assert np.array_equal(gpu_vk(gpu, u0, kappa, rhs, 0.035, 5, parts=parts), want)


@pytest.mark.parametrize("mode", ["split", "fused", "plain"])
def test_f32_bitwise(gpu, mode, time_block):
    dims = (132, 37, 45)
    note("vk f32 %s mode=%s" % (dims, mode))
    u0, kappa, rhs = random_case(dims, seed=8, dtype=np.float32)
    want = oracle.heat_vk_f32(u0, kappa, rhs, 0.04, 6)
    got = gpu_vk(gpu, u0, kappa, rhs, 0.04, 6, mode=mode)
    assert got.dtype == np.float32 and np.array_equal(got, want)


def built_shapes(hc, dtype):
    lib = hc.load()
    code = hc.DTYPES[dtype]
    out = []
    for vec in (1, 2, 4):
        for wx in (1, 2, 4):
            for by in (4, 8, 16):
                for zd in (16, 32):
                    for pf in (1, 2, 3):
                        if lib.hc_heat_vk_set_tiling(code, vec, wx, by, zd, pf, 0) == 0:
                            out.append((vec, wx, by, zd, pf))
    hc.set_vk_tiling(dtype=dtype)
    return out


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_every_built_shape_bitwise(one_step, dtype):
    gpu = one_step
    shapes = built_shapes(gpu, dtype)
    assert len(shapes) >= 8
    npdt = np.float64 if dtype == "f64" else np.float32
    dims = (264, 19, 75)       # ragged in x, y and z for every shape
    u0, kappa, rhs = random_case(dims, seed=21, dtype=npdt)
    ref = oracle.heat_vk if dtype == "f64" else oracle.heat_vk_f32
    want = ref(u0, kappa, rhs, 0.04, 3)
    try:
        for shape in shapes:
            for xcd in (0, 8):
                for mode in ("split", "fused"):
                    note("vk %s shape %s xcd=%d %s" % (dtype, shape, xcd, mode))
                    gpu.set_vk_tiling(*shape, xcd=xcd, dtype=dtype)
                    got = gpu_vk(gpu, u0, kappa, rhs, 0.04, 3, mode=mode)
                    assert np.array_equal(got, want), (shape, xcd, mode)
    finally:
        gpu.set_vk_tiling(dtype=dtype)


def built_shapes2(hc, dtype):
    lib = hc.load()
    code = hc.DTYPES[dtype]
    out = []
    for vec in (1, 2, 4):
        for wx in (1, 2, 4):
            for by in (4, 8, 16):
                for zd in (16, 32):
                    for pf in (1, 2, 3):
                        if lib.hc_heat_vk2_set_tiling(code, vec, wx, by, zd, pf, 0) == 0:
                            out.append((vec, wx, by, zd, pf))
    hc.set_vk2_tiling(dtype=dtype)
    return out


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_every_built_two_step_shape_bitwise(gpu, dtype):
    saved = gpu.get_time_block()
    gpu.set_time_block(2)
    shapes = built_shapes2(gpu, dtype)
    assert len(shapes) >= 5
    npdt = np.float64 if dtype == "f64" else np.float32
    dims = (264, 19, 75)
    u0, kappa, rhs = random_case(dims, seed=23, dtype=npdt)
    ref = oracle.heat_vk if dtype == "f64" else oracle.heat_vk_f32
    want = ref(u0, kappa, rhs, 0.04, 5)
    try:
        for shape in shapes:
            for xcd in (0, 8):
                for mode in ("split", "fused"):
                    note("vk2 %s shape %s xcd=%d %s" % (dtype, shape, xcd, mode))
                    gpu.set_vk2_tiling(*shape, xcd=xcd, dtype=dtype)
                    got = gpu_vk(gpu, u0, kappa, rhs, 0.04, 5, mode=mode)
                    assert np.array_equal(got, want), (shape, xcd, mode)
    finally:
        gpu.set_vk2_tiling(dtype=dtype)
        gpu.set_time_block(saved)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_two_step_run_lengths_bitwise(gpu, dtype):
    """Runs of several z-blocks per block (kappa's four LDS planes keep
    their rotation across sub-blocks) and whole columns."""
    saved = gpu.get_time_block()
    gpu.set_time_block(2)
    npdt = np.float64 if dtype == "f64" else np.float32
    dims = (130, 21, 150)
    u0, kappa, rhs = random_case(dims, seed=37, dtype=npdt)
    ref = oracle.heat_vk if dtype == "f64" else oracle.heat_vk_f32
    want = ref(u0, kappa, rhs, 0.04, 6)
    try:
        for zrun in (1, 40, 64, 96, 1 << 20):
            for mode in ("split", "fused"):
                note("vk2 %s run of %d planes %s" % (dtype, zrun, mode))
                gpu.set_vk2_zrun(zrun, dtype=dtype)
                got = gpu_vk(gpu, u0, kappa, rhs, 0.04, 6, mode=mode)
                assert np.array_equal(got, want), (zrun, mode)
    finally:
        gpu.set_vk2_zrun(0, dtype=dtype)
        gpu.set_time_block(saved)


def test_tiling_for_reports_a_built_shape_and_odd_rows_fall_back(gpu):
    t = lambda *s: torch.zeros(*s, dtype=torch.float64, device="cuda")  # noqa: E731
    a = [t(8, 8, 512) for _ in range(4)]
    sh = gpu.vk_tiling_for(*a)
    assert sh["vec"] == 2
    b = [t(8, 8, 511) for _ in range(4)]
    assert gpu.vk_tiling_for(*b)["vec"] == 1
    u0, kappa, rhs = random_case((511, 8, 8), seed=2)
    want = oracle.heat_vk(u0, kappa, rhs, 0.04, 2)
    assert np.array_equal(gpu_vk(gpu, u0, kappa, rhs, 0.04, 2), want)


def test_constant_kappa_agrees_with_the_seven_point_kernel_within_rounding(gpu):
    n = 96
    note("vk constant kappa vs heat_step, %d^3" % n)
    u0 = inputs.sine_field(n, n, n, noise=1e-3, seed=5)
    alpha, beta = 0.5, 0.1
    got = gpu_vk(gpu, u0, np.full(u0.shape, alpha), np.zeros(u0.shape), beta, 20)
    u = torch.from_numpy(u0).cuda()
    gpu.heat_step(u, torch.empty_like(u), 2 * alpha * beta, 20)
    torch.cuda.synchronize()
    assert np.max(np.abs(got - u.cpu().numpy())) <= 1e-14


def test_degenerate_steps_and_buffers(gpu):
    u0, kappa, rhs = random_case((9, 8, 7), seed=30)
    assert np.array_equal(gpu_vk(gpu, u0, kappa, rhs, 0.04, 0), u0)
    # kappa and rhs may share one buffer
    want = oracle.heat_vk(u0, kappa, kappa, 0.01, 3)
    uu = torch.from_numpy(u0).cuda()
    kk = torch.from_numpy(kappa).cuda()
    gpu.heat_vk_step(uu, torch.empty_like(uu), kk, kk, 0.01, 3)
    torch.cuda.synchronize()
    assert np.array_equal(uu.cpu().numpy(), want)
    with pytest.raises(gpu.HeatCGError):
        gpu.heat_vk_step(uu, torch.empty_like(uu), uu, kk, 0.01, 1)       # kappa is u
    with pytest.raises(TypeError):
        b = torch.zeros(9, 8, 7, dtype=torch.bfloat16, device="cuda")
        gpu.heat_vk_step(b, b.clone(), b.clone(), b.clone(), 0.01, 1)


@pytest.mark.parametrize("mode", ["split", "fused"])
def test_papers_test_case_512_full_size(gpu, mode, time_block):
    """The configuration the variable-coefficient rate is measured on, in
    the launch shape the benchmark times; compared in full after 3 steps."""
    n, steps = inputs.VARCOEF["n"], 3
    note("vk paper problem %d^3 %d steps mode=%s, %d per pass (full size)"
         % (n, steps, mode, time_block))
    pb = inputs.paper_problem(n)
    want = oracle.heat_vk(pb["u0"], pb["kappa"], pb["rhs"], pb["beta"], steps)
    got = gpu_vk(gpu, pb["u0"], pb["kappa"], pb["rhs"], pb["beta"], steps, mode=mode)
    assert np.array_equal(got, want)
