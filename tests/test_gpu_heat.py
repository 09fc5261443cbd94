"""GPU parity of the heat sweep: the HIP kernels against the CPU oracle.

The FP64 kernels evaluate the same written expression in the same order
without contraction, so every comparison here is bit-for-bit
(np.array_equal).  Shapes span several 64 x BY tiles and several z-blocks
and end in ragged tails; the Interior/Boundary split, the fused z-march and
the one-thread-per-node form must all agree.  At the full 512^3 size the
oracle checks a short run in full, and the 1000-step run is checked against
the exact decay of a pure sine mode (a property that holds at any size).
"""
import json
import os

import numpy as np
import pytest
import torch

import oracle
from paper_2608_11882_amd import inputs

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "paper_constants.json")


def note(msg):
    print("[case] " + msg, flush=True)


def gpu_heat(hc, u0, r, steps, mode="split", parts=1, stream=None):
    u = torch.from_numpy(np.ascontiguousarray(u0)).cuda()
    un = torch.empty_like(u)
    hc.heat_step(u, un, r, steps, mode=mode, parts=parts, stream=stream)
    torch.cuda.synchronize()
    return u.cpu().numpy(), un.cpu().numpy()


def decay_factor(r, dims, modes=(1, 1, 1)):
    g = 1.0
    for n, m in zip(dims, modes):
        g -= 4.0 * r * np.sin(np.pi * m / (2.0 * (n - 1))) ** 2
    return g


@pytest.mark.parametrize("mode", ["split", "fused", "plain"])
def test_small_config_bitwise(gpu, mode, time_block):
    cfg = inputs.HEAT_SMALL
    note("heat 66^3 r=0.1 100 steps mode=%s" % mode)
    u0 = inputs.heat_small_f64(seed=cfg["seed"])
    want = oracle.heat(u0, cfg["r"], cfg["steps"])
    got, _ = gpu_heat(gpu, u0, cfg["r"], cfg["steps"], mode=mode)
    assert np.array_equal(got, want)
    # the paper's own acceptance rule holds a fortiori
    acc = json.load(open(GOLDEN))["acceptance"]
    assert np.all(np.abs(got - want) <= acc["atol"] + acc["rtol"] * np.abs(want))
    assert np.all(np.isfinite(got))


def test_small_config_pure_mode_matches_closed_form(gpu):
    n, r, steps = 66, 0.1, 100
    note("heat 66^3 pure sine mode vs G^100")
    u0 = inputs.sine_field(n, n, n)
    got, _ = gpu_heat(gpu, u0, r, steps)
    want = decay_factor(r, (n, n, n)) ** steps * u0
    assert np.max(np.abs(got - want)) <= 1e-12 * np.max(np.abs(u0))


@pytest.mark.parametrize("dims", [(67, 35, 20), (130, 9, 40), (3, 3, 3), (64, 6, 70),
                                  (200, 13, 5), (65, 66, 4), (129, 130, 37)])
@pytest.mark.parametrize("mode", ["split", "fused", "plain"])
def test_ragged_shapes_bitwise(gpu, dims, mode):
    nx, ny, nz = dims
    note("heat ragged %s mode=%s" % (dims, mode))
    u0 = inputs.uniform_field(nx, ny, nz, seed=nx * 7 + ny * 3 + nz)
    steps = 7  # odd: the result comes back from the scratch buffer
    want = oracle.heat(u0, 0.15, steps)
    got, _ = gpu_heat(gpu, u0, 0.15, steps, mode=mode)
    assert np.array_equal(got, want)


def built_shapes(dtype="f64"):
    """Every tile shape libheatcg.so accepts for one element type (probed
    through the C ABI)."""
    import paper_2608_11882_amd as hc
    lib = hc.load()
    code = hc.DTYPES[dtype]
    shapes = []
    for vec in (1, 2, 4, 8):
        for wx in (1, 2, 4):
            for by in (4, 8, 16):
                for zd in (16, 32, 64):
                    for pf in (1, 2, 3, 4):
                        if lib.hc_heat_set_tiling(code, vec, wx, by, zd, pf, 0) == 0:
                            shapes.append((vec, wx, by, zd, pf))
    hc.set_tiling(dtype=dtype)
    return shapes


def test_every_tile_shape_is_bitwise_identical(one_step):
    gpu = one_step
    dims = (150, 37, 75)   # 71 interior planes: ragged against every depth and width
    u0 = inputs.uniform_field(*dims, seed=31)
    want = oracle.heat(u0, 1.0 / 6.5, 5)
    shapes = built_shapes()
    assert len(shapes) >= 12
    try:
        for shape in shapes:
            for xcd in (0, 3, 8):
                note("heat tiling vec,wx,by,zdepth,pf=%s xcd=%d" % (shape, xcd))
                gpu.set_tiling(*shape, xcd=xcd)
                for mode in ("split", "fused"):
                    got, _ = gpu_heat(gpu, u0, 1.0 / 6.5, 5, mode=mode)
                    assert np.array_equal(got, want), (shape, xcd, mode)
    finally:
        gpu.set_tiling()


@pytest.mark.parametrize("dims", [(131, 20, 40), (257, 9, 35), (256, 17, 36), (260, 30, 34)])
def test_wide_lanes_on_ragged_and_odd_widths(one_step, dims):
    gpu = one_step
    """Two-node lanes: widths that end inside a tile, and odd widths (which
    fall back to one-node lanes)."""
    note("heat wide lanes %s" % (dims,))
    u0 = inputs.uniform_field(*dims, seed=dims[0])
    want = oracle.heat(u0, 0.16, 6)
    for shape in [(2, 1, 8, 16, 2), (2, 2, 8, 16, 2), (2, 4, 4, 16, 2)]:
        try:
            gpu.set_tiling(*shape)
            got, _ = gpu_heat(gpu, u0, 0.16, 6)
        finally:
            gpu.set_tiling()
        assert np.array_equal(got, want), shape


def test_misaligned_arrays_fall_back_to_one_node_lanes(gpu):
    dims = (130, 21, 33)
    note("heat on 8-byte aligned (not 16) views")
    u0 = inputs.uniform_field(*dims, seed=77)
    n = u0.size
    big_u = torch.zeros(n + 1, dtype=torch.float64, device="cuda")
    big_v = torch.zeros(n + 1, dtype=torch.float64, device="cuda")
    u = big_u[1:].view(dims[::-1])
    un = big_v[1:].view(dims[::-1])
    assert u.data_ptr() % 16 == 8
    u.copy_(torch.from_numpy(u0))
    gpu.heat_step(u, un, 0.1, 4)
    torch.cuda.synchronize()
    assert np.array_equal(u.cpu().numpy(), oracle.heat(u0, 0.1, 4))
    assert big_u[0].item() == 0.0 and big_v[0].item() == 0.0


@pytest.mark.parametrize("parts", [1, 2, 3, 7, 32])
def test_slab_split_bitwise(gpu, parts):
    dims = (70, 20, 50)
    note("heat parts=%d" % parts)
    u0 = inputs.uniform_field(*dims, seed=parts)
    want = oracle.heat(u0, 0.12, 6)
    got, _ = gpu_heat(gpu, u0, 0.12, 6, parts=parts)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("steps", [5, 6])
def test_nonzero_dirichlet_data_is_kept_and_scratch_contract(gpu, steps, time_block):
    """Dirichlet data need not be zero; u_new ends as the header states: its
    outermost layer is u's; with one step per pass it holds u^(steps-1) for
    even step counts and u^steps for odd ones."""
    dims = (40, 33, 21)
    note("heat nonzero boundary, %d steps, %d per pass" % (steps, time_block))
    rng = np.random.default_rng(17)
    u0 = rng.uniform(-1, 1, size=dims[::-1])
    want = oracle.heat(u0, 0.1, steps)
    got, scratch = gpu_heat(gpu, u0, 0.1, steps)
    assert np.array_equal(got, want)
    layer = np.ones(u0.shape, bool)
    layer[1:-1, 1:-1, 1:-1] = False
    assert np.array_equal(scratch[layer], u0[layer])
    if time_block == 1:
        expect_scratch = want if steps % 2 else oracle.heat(u0, 0.1, steps - 1)
        assert np.array_equal(scratch, expect_scratch)


def test_chunked_calls_compose_and_zero_steps_is_a_noop(gpu):
    dims = (90, 45, 38)
    note("heat chunked 3+4 vs 7")
    u0 = inputs.uniform_field(*dims, seed=5)
    u = torch.from_numpy(u0).cuda()
    un = torch.empty_like(u)
    gpu.heat_step(u, un, 0.14, 3)
    gpu.heat_step(u, un, 0.14, 0)
    gpu.heat_step(u, un, 0.14, 4)
    torch.cuda.synchronize()
    assert np.array_equal(u.cpu().numpy(), oracle.heat(u0, 0.14, 7))


def test_runs_on_a_side_stream(gpu):
    dims = (70, 33, 45)
    note("heat on a side stream")
    u0 = inputs.uniform_field(*dims, seed=8)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        got, _ = gpu_heat(gpu, u0, 0.1, 10, stream=s)
    assert np.array_equal(got, oracle.heat(u0, 0.1, 10))


def test_blocking_plain_entry_point(gpu):
    import ctypes
    dims = (34, 34, 34)
    note("heat through heat_step (blocking C entry point)")
    u0 = inputs.heat_small_f64(seed=3, n=34)
    u = torch.from_numpy(u0).cuda()
    un = torch.empty_like(u)
    torch.cuda.synchronize()
    rc = gpu.abi().heat_step(ctypes.c_void_p(u.data_ptr()), ctypes.c_void_p(un.data_ptr()),
                             34, 34, 34, 0.1, 9)
    assert rc == 0
    assert np.array_equal(u.cpu().numpy(), oracle.heat(u0, 0.1, 9))


def test_large_config_short_run_bitwise(gpu):
    cfg = inputs.HEAT_LARGE
    n = cfg["n"]
    note("heat 512^3 r=1/6.5 12 steps split, bitwise vs oracle")
    u0 = inputs.heat_large_f64(seed=cfg["seed"], n=n)
    want = oracle.heat(u0, cfg["r"], 12)
    got, _ = gpu_heat(gpu, u0, cfg["r"], 12)
    assert np.array_equal(got, want)


def test_large_config_full_run_pure_mode_and_max_principle(gpu):
    cfg = inputs.HEAT_LARGE
    n, r, steps = cfg["n"], cfg["r"], cfg["steps"]
    note("heat 512^3 pure sine mode 1000 steps vs G^1000")
    u0 = inputs.sine_field(n, n, n)
    got, _ = gpu_heat(gpu, u0, r, steps)
    g = decay_factor(r, (n, n, n)) ** steps
    err = np.max(np.abs(got - g * u0))
    assert err <= 4e-16 * steps * np.max(np.abs(u0)), err
    assert got.max() <= u0.max() and got.min() >= 0.0


def test_large_config_recipe_full_run_properties(gpu):
    cfg = inputs.HEAT_LARGE
    n, r, steps = cfg["n"], cfg["r"], cfg["steps"]
    note("heat 512^3 recipe 1000 steps: max principle, decay, boundary")
    u0 = inputs.heat_large_f64(seed=cfg["seed"], n=n)
    got, _ = gpu_heat(gpu, u0, r, steps)
    assert np.all(np.isfinite(got))
    assert got.min() >= 0.0 and got.max() <= u0.max()
    assert got.sum() < u0.sum()
    assert not got[0].any() and not got[-1].any() and not got[:, 0].any()
    assert not got[:, :, 0].any() and not got[:, :, -1].any() and not got[:, -1].any()
