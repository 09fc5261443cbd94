"""GPU parity of the reduced-precision heat sweeps (binary32, and bfloat16
storage with binary32 arithmetic) against the CPU oracle's binary32 and
bfloat16 steps.

Both sides evaluate the same written expression in the same order in
binary32 without contraction, and the bfloat16 rounding is round to
nearest, ties to even on both, so every comparison is bit-for-bit.  At the
full 1024^3 size the oracle checks a short run on the first and last planes
(an output plane after s steps depends only on the input planes within s of
it), and the 500-step binary32 run is checked against the exact decay of a
pure sine mode within a rigorous rounding-error bound.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2608_11882_amd import inputs

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24   # unit roundoff of binary32


def note(msg):
    print("[case] " + msg, flush=True)


def to_device(a):
    """uint16 bit patterns become a torch.bfloat16 tensor of the same bits."""
    if a.dtype == np.uint16:
        return torch.from_numpy(np.ascontiguousarray(a).view(np.int16)).cuda().view(torch.bfloat16)
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def to_host(t):
    if t.dtype == torch.bfloat16:
        return t.view(torch.int16).cpu().numpy().view(np.uint16)
    return t.cpu().numpy()


def gpu_heat(hc, u0, r, steps, mode="split", parts=1):
    u = to_device(u0)
    un = torch.empty_like(u)
    hc.heat_step(u, un, r, steps, mode=mode, parts=parts)
    torch.cuda.synchronize()
    return to_host(u)


def oracle_heat(u0, r, steps):
    return oracle.heat_bf16(u0, r, steps) if u0.dtype == np.uint16 else oracle.heat_f32(u0, r, steps)


def field(dims, seed, dtype, noise=None):
    nx, ny, nz = dims
    if noise is None:   # rough data: U[0,1] interior, rounded once
        u = inputs.uniform_field(nx, ny, nz, seed=seed)
        return u.astype(np.float32) if dtype == "f32" else inputs.to_bf16_bits(u)
    return inputs.sine_field_lowp(nx, ny, nz, noise, seed, dtype)


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
@pytest.mark.parametrize("mode", ["split", "fused", "plain"])
def test_small_config_bitwise(gpu, dtype, mode, time_block):
    cfg = inputs.HEAT_SMALL
    note("heat %s 66^3 r=0.1 100 steps mode=%s" % (dtype, mode))
    u0 = inputs.sine_field_lowp(66, 66, 66, 1e-3, cfg["seed"], dtype)
    want = oracle_heat(u0, cfg["r"], cfg["steps"])
    got = gpu_heat(gpu, u0, cfg["r"], cfg["steps"], mode=mode)
    assert got.dtype == want.dtype and np.array_equal(got, want)


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
@pytest.mark.parametrize("dims", [(67, 35, 20), (130, 9, 40), (3, 3, 3), (64, 6, 70),
                                  (1030, 13, 5), (520, 66, 37), (1024, 12, 36)])
@pytest.mark.parametrize("mode", ["split", "fused"])
def test_ragged_shapes_bitwise(gpu, dtype, dims, mode):
    """Widths that end inside a tile, widths that are not a multiple of the
    lane width (one-node fallback), and very short z-extents."""
    note("heat %s ragged %s mode=%s" % (dtype, dims, mode))
    u0 = field(dims, dims[0] * 7 + dims[1] * 3 + dims[2], dtype)
    want = oracle_heat(u0, 0.15, 7)
    assert np.array_equal(gpu_heat(gpu, u0, 0.15, 7, mode=mode), want)


def test_parts_bitwise(gpu):
    dims = (256, 20, 67)
    for dtype in ("f32", "bf16"):
        u0 = field(dims, 77, dtype)
        want = oracle_heat(u0, 0.125, 6)
        for parts in (2, 5, 32):
            note("heat %s parts=%d" % (dtype, parts))
            assert np.array_equal(gpu_heat(gpu, u0, 0.125, 6, parts=parts), want)


def built_shapes(dtype):
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


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_every_tile_shape_is_bitwise_identical(one_step, dtype):
    gpu = one_step
    dims = (2056, 37, 75)   # ragged against every width (2056 = 8 * 257) and depth
    u0 = field(dims, 31, dtype)
    want = oracle_heat(u0, 1.0 / 6.5, 5)
    shapes = built_shapes(dtype)
    assert len(shapes) >= 6
    try:
        for shape in shapes:
            for xcd in (0, 3, 8):
                note("heat %s tiling %s xcd=%d" % (dtype, shape, xcd))
                gpu.set_tiling(*shape, xcd=xcd, dtype=dtype)
                for mode in ("split", "fused"):
                    assert np.array_equal(gpu_heat(gpu, u0, 1.0 / 6.5, 5, mode=mode), want), \
                        (shape, xcd, mode)
    finally:
        gpu.set_tiling(dtype=dtype)


def test_misaligned_arrays_fall_back_bitwise(gpu):
    """Arrays that start off the lane alignment take the one-node shape."""
    dims = (64, 10, 12)
    n = dims[0] * dims[1] * dims[2]
    for dtype, tdt in (("f32", torch.float32), ("bf16", torch.bfloat16)):
        u0 = field(dims, 5, dtype)
        want = oracle_heat(u0, 0.1, 3)
        big = torch.empty(2 * n + 16, dtype=tdt, device="cuda")
        u = big[1:1 + n].view(dims[2], dims[1], dims[0])
        un = big[n + 9:2 * n + 9].view(dims[2], dims[1], dims[0])
        u.copy_(to_device(u0))
        note("heat %s misaligned" % dtype)
        gpu.heat_step(u, un, 0.1, 3)
        torch.cuda.synchronize()
        assert np.array_equal(to_host(u), want)


def test_reduced_precision_error_against_fp64_is_within_bound(gpu):
    """Max error of the binary32 sweep against the FP64 oracle on the small
    configuration, against the worst-case rounding bound: each step adds at
    most (1 + 46 r) u32 max|u| to first order (the five additions of the
    neighbour sum err by at most 16 u32 max|u| together, 6c by 6, the
    difference and the product by r 12 each with |lap| <= 12 max|u|, the
    final addition by 1) and the scheme is contractive in the max norm for
    r <= 1/6, so the errors of the steps add up without amplification."""
    cfg = inputs.HEAT_SMALL
    note("heat f32 vs f64 error bound 66^3")
    u64 = inputs.sine_field(66, 66, 66, noise=1e-3, seed=cfg["seed"])
    u32 = inputs.sine_field_lowp(66, 66, 66, 1e-3, cfg["seed"], "f32")
    ref = oracle.heat(u32.astype(np.float64), cfg["r"], cfg["steps"])
    got = gpu_heat(gpu, u32, cfg["r"], cfg["steps"]).astype(np.float64)
    m = np.max(np.abs(u64))
    bound = cfg["steps"] * (1 + 46 * cfg["r"]) * U32 * m + abs(np.float32(cfg["r"]) - cfg["r"]) \
        * cfg["steps"] * 12 * m
    err = np.max(np.abs(got - ref))
    assert err <= bound, (err, bound)
    assert np.max(np.abs(u32.astype(np.float64) - u64)) <= U32 * m


# ---- full size: 1024^3 ------------------------------------------------------------

def full_size_slab_check(hc, dtype, steps=3, planes=24):
    cfg = inputs.HEAT_PRECISION
    n, r = cfg["n"], cfg["r"]
    note("heat %s %d^3 %d steps, oracle on the first and last %d planes" % (dtype, n, steps, planes))
    u0 = inputs.sine_field_lowp(n, n, n, 1e-3, cfg["seed"], dtype)
    lo, hi = u0[:planes].copy(), u0[n - planes:].copy()
    u = to_device(u0)
    del u0
    un = torch.empty_like(u)
    hc.heat_step(u, un, r, steps)
    torch.cuda.synchronize()
    got_lo, got_hi = to_host(u[:planes - steps]), to_host(u[n - planes + steps:])
    want_lo = oracle_heat(lo, r, steps)[:planes - steps]
    want_hi = oracle_heat(hi, r, steps)[steps:]
    assert np.array_equal(got_lo, want_lo)
    assert np.array_equal(got_hi, want_hi)


def test_full_size_f32_short_run_bitwise_on_slabs(gpu):
    full_size_slab_check(gpu, "f32")


def test_full_size_bf16_short_run_bitwise_on_slabs(gpu):
    full_size_slab_check(gpu, "bf16")


def test_full_size_f32_pure_mode_500_steps_within_rounding_bound(gpu):
    cfg = inputs.HEAT_PRECISION
    n, r, steps = cfg["n"], cfg["r"], cfg["steps"]
    note("heat f32 %d^3 pure sine mode, %d steps, vs G^steps" % (n, steps))
    s = torch.sin(torch.pi * torch.from_numpy(inputs.node_coords(n))).cuda()
    s[0] = 0.0
    s[-1] = 0.0
    u64 = s[:, None, None] * s[None, :, None] * s[None, None, :]
    u = u64.float()
    del u64
    un = torch.empty_like(u)
    u0 = u.clone()
    gpu.heat_step(u, un, r, steps)
    torch.cuda.synchronize()
    del un
    r32 = float(np.float32(r))
    g = 1.0 - 3 * 4.0 * r32 * np.sin(np.pi / (2.0 * (n - 1))) ** 2
    # exact discrete result for the rounded initial field and the rounded r
    err = 0.0
    for k0 in range(0, n, 128):
        want = (g ** steps) * u0[k0:k0 + 128].double()
        err = max(err, (u[k0:k0 + 128].double() - want).abs().max().item())
    m = u0.abs().max().item()
    bound = steps * (1 + 46 * r32) * U32 * m
    note("f32 pure-mode max error %.3e (bound %.3e)" % (err, bound))
    assert err <= bound
    assert torch.isfinite(u).all().item()


def test_full_size_bf16_500_steps_keeps_the_maximum_principle(gpu):
    """bfloat16 storage at 1024^3: the smooth mode changes by less than half
    a bfloat16 ulp per step, so round-to-nearest leaves most nodes where
    they are; what must hold at any size is the discrete maximum principle
    (values stay within [min(0, min u0), max(0, max u0)]) and finiteness."""
    cfg = inputs.HEAT_PRECISION
    n, r, steps = cfg["n"], cfg["r"], cfg["steps"]
    note("heat bf16 %d^3 %d steps, maximum principle" % (n, steps))
    u0 = inputs.sine_field_lowp(n, n, n, 1e-3, cfg["seed"], "bf16")
    u = to_device(u0)
    lo = min(0.0, float(u.float().min().item()))
    hi = max(0.0, float(u.float().max().item()))
    del u0
    un = torch.empty_like(u)
    gpu.heat_step(u, un, r, steps)
    torch.cuda.synchronize()
    uf = u.float()
    assert torch.isfinite(uf).all().item()
    assert uf.min().item() >= lo and uf.max().item() <= hi


# ---- errors against the FP64 oracle, with stated bounds --------------------------------

def bf16_ulp(x):
    """ulp of a bfloat16 in the binade of x > 0 (8 significant bits)."""
    return 2.0 ** (np.floor(np.log2(x)) - 7)


def sr_noise_sum(r, steps, m=64):
    """sum over m = 0 .. steps-1 of the squared 2-norm of the free-lattice
    kernel of m steps (I + rL)^m, by Parseval: the mean over a midpoint grid
    of wavenumbers of sum_m G^(2m), G = 1 - 4r sum_i sin^2(theta_i / 2).  The
    Dirichlet kernel is bounded by the free one entry by entry (r <= 1/6, no
    negative weights), so this bounds its row norms as well."""
    th = (np.arange(m) + 0.5) / m * 2 * np.pi - np.pi
    s = np.sin(th / 2) ** 2
    g2 = (1 - 4 * r * (s[:, None, None] + s[None, :, None] + s[None, None, :])) ** 2
    return float(np.mean((1 - g2 ** steps) / (1 - g2)))


class Norms:
    """max |a - b|, ||a - b||_2 and ||b||_2 over device fields (FP64 sums,
    chunks of planes)."""

    def __init__(self, a, b):
        self.max, e2, b2 = 0.0, 0.0, 0.0
        for k0 in range(0, a.shape[0], 64):
            x = a[k0:k0 + 64].double()
            y = b[k0:k0 + 64].double()
            d = x - y
            self.max = max(self.max, d.abs().max().item())
            e2 += (d * d).sum().item()
            b2 += (y * y).sum().item()
        self.l2, self.ref_l2 = e2 ** 0.5, b2 ** 0.5


def check_precision_errors(hc, u0_64, us_64, r, steps, tag):
    """Run the binary32, bfloat16 (nearest) and bfloat16 (stochastic) sweeps
    from u0_64 rounded once, compare with us_64 = the FP64 oracle's result,
    and hold each error to its bound:

    * binary32 (rigorous): the initial rounding (u32 max|u|) plus, per step,
      (1 + 46 r) u32 max|u| (the scheme is contractive in the max norm, so
      step errors add up) plus the effect of rounding r once;
    * bfloat16, nearest (stall model): an increment below half an ulp is
      dropped, so in the worst case a node never moves; its error is then at
      most its initial rounding plus the change of the exact solution,
      max|v0 - u0| + max|u0 - uS|, plus half an ulp of the largest value for
      the nodes whose increments are resolved (the same in 2-norms);
    * bfloat16, stochastic (rigorous in expectation): the roundings are
      unbiased and independent, so E||e_S||^2 <= ||v0 - u0||^2 +
      (ulp_max / 2)^2 N sum_m ||K_m||^2 (K_m the m-step kernel), plus the
      binary32 arithmetic's share; with 10^9 nodes the realized mean square
      sits close to its expectation.
    Returns the measured errors."""
    n = u0_64.numel()
    interior = (u0_64.shape[0] - 2) * (u0_64.shape[1] - 2) * (u0_64.shape[2] - 2)
    m = u0_64.abs().max().item()
    drift = Norms(u0_64, us_64)            # ||u0 - uS||
    out = {}
    # binary32
    u = u0_64.float()
    q32 = Norms(u, u0_64)
    un = torch.empty_like(u)
    hc.heat_step(u, un, r, steps)
    torch.cuda.synchronize()
    e = Norms(u, us_64)
    r32 = float(np.float32(r))
    b32 = U32 * m + steps * (1 + 46 * r32) * U32 * m + abs(r32 - r) * steps * 12 * m
    note("%s f32: max %.3e (bound %.3e), rel-L2 %.3e" % (tag, e.max, b32, e.l2 / e.ref_l2))
    assert q32.max <= U32 * m
    assert e.max <= b32
    out["f32"] = (e.max, e.l2 / e.ref_l2)
    del u, un
    # bfloat16 input, rounded once from FP64 (to nearest, ties to even)
    v0 = torch.empty(u0_64.shape, dtype=torch.bfloat16, device=u0_64.device)
    host = u0_64.cpu().numpy() if n <= 2 ** 27 else None
    for k0 in range(0, u0_64.shape[0], 64):
        part = host[k0:k0 + 64] if host is not None else u0_64[k0:k0 + 64].cpu().numpy()
        v0[k0:k0 + 64].view(torch.int16).copy_(
            torch.from_numpy(inputs.to_bf16_bits(part).view(np.int16)))
    q16 = Norms(v0, u0_64)                 # ||v0 - u0||
    vmax = v0.float().abs().max().item()
    ulp_hi = bf16_ulp(vmax)
    f32_share = steps * (1 + 46 * r32) * U32 * vmax
    # nearest
    v = v0.clone()
    vn = torch.empty_like(v)
    hc.heat_step(v, vn, r, steps)
    torch.cuda.synchronize()
    e = Norms(v, us_64)
    bmax = q16.max + drift.max + ulp_hi / 2 + f32_share
    bl2 = (q16.l2 + drift.l2 + (ulp_hi / 2 + f32_share) * interior ** 0.5) / e.ref_l2
    note("%s bf16: max %.3e (bound %.3e), rel-L2 %.3e (bound %.3e)"
         % (tag, e.max, bmax, e.l2 / e.ref_l2, bl2))
    assert e.max <= bmax and e.l2 / e.ref_l2 <= bl2
    out["bf16"] = (e.max, e.l2 / e.ref_l2)
    # stochastic
    v.copy_(v0)
    hc.heat_step_sr(v, vn, r, steps, 2026)
    torch.cuda.synchronize()
    e = Norms(v, us_64)
    c = sr_noise_sum(r32, steps)
    rms = (q16.l2 ** 2 / interior + (ulp_hi / 2) ** 2 * c) ** 0.5 + f32_share
    bsr = rms * interior ** 0.5 / e.ref_l2
    note("%s bf16-sr: max %.3e, rel-L2 %.3e (bound %.3e, kernel sum %.3f)"
         % (tag, e.max, e.l2 / e.ref_l2, bsr, c))
    assert e.l2 / e.ref_l2 <= bsr
    out["bf16_sr"] = (e.max, e.l2 / e.ref_l2)
    return out


def test_precision_errors_on_the_256_instance(gpu):
    """The reduced-precision sweeps on a 256^3 instance of the precision
    configuration (sine mode + U[-1e-3, 1e-3] noise, r = 0.15, 500 steps)
    against the FP64 oracle run in full.  Here the smooth mode decays by 3%
    over the run, far more than a bfloat16 ulp, so nearest rounding stalls
    visibly while stochastic rounding follows."""
    cfg = inputs.HEAT_PRECISION
    r, steps = cfg["r"], cfg["steps"]
    note("precision errors 256^3 x%d against the FP64 oracle" % steps)
    u0 = inputs.sine_field(256, 256, 256, noise=1e-3, seed=cfg["seed"])
    us = oracle.heat(u0, r, steps)
    out = check_precision_errors(gpu, torch.from_numpy(u0).cuda(), torch.from_numpy(us).cuda(),
                                 r, steps, "256^3")
    assert out["bf16_sr"][1] < 0.25 * out["bf16"][1]
    # the other remedy, bfloat16 offsets from the rounded initial field
    # (evaluated in the oracle: the library has no kernel for it)
    base, off = inputs.bf16_offset_split(u0)
    widen = lambda b: (b.astype(np.uint32) << np.uint32(16)).view(np.float32).astype(np.float64)  # noqa: E731
    got = widen(base) + widen(oracle.heat_bf16_offset(base, off, r, steps))
    e = got - us
    rel = np.linalg.norm(e) / np.linalg.norm(us)
    note("256^3 bf16 offsets (oracle): max %.3e, rel-L2 %.3e" % (np.abs(e).max(), rel))
    assert rel < 0.1 * out["bf16"][1] and rel < out["bf16_sr"][1]


def test_precision_errors_on_the_full_grid(gpu):
    """The precision configuration itself: 1024^3, sine mode + noise (seed
    3), r = 0.15, 500 steps, against the FP64 oracle on the full grid (run
    as five calls of 100 steps, which compose exactly).  At this size the
    smooth mode decays by only 0.2% over the run, about as much as the
    stochastic rounding's noise floor, so both bfloat16 forms end near the
    same error."""
    cfg = inputs.HEAT_PRECISION
    n, r, steps = cfg["n"], cfg["r"], cfg["steps"]
    note("precision errors %d^3 x%d: building the FP64 input" % (n, steps))
    u0 = inputs.sine_field(n, n, n, noise=1e-3, seed=cfg["seed"])
    u0_dev = torch.from_numpy(u0).cuda()
    us = u0
    for q in range(steps // 100):
        us = oracle.heat(us, r, 100)
        note("precision errors %d^3: oracle at %d of %d steps" % (n, 100 * (q + 1), steps))
    del u0
    us_dev = torch.from_numpy(us).cuda()
    del us
    check_precision_errors(gpu, u0_dev, us_dev, r, steps, "%d^3" % n)


# ---- bfloat16 with stochastic rounding ------------------------------------------------

def gpu_heat_sr(hc, u0, r, steps, seed, step0=0, mode="split", parts=1):
    u = to_device(u0)
    un = torch.empty_like(u)
    hc.heat_step_sr(u, un, r, steps, seed, step0=step0, mode=mode, parts=parts)
    torch.cuda.synchronize()
    return to_host(u)


@pytest.mark.parametrize("mode", ["split", "fused", "plain"])
def test_sr_small_config_bitwise(gpu, mode):
    cfg = inputs.HEAT_SMALL
    note("heat bf16-sr 66^3 r=0.1 100 steps mode=%s" % mode)
    u0 = inputs.sine_field_lowp(66, 66, 66, 1e-3, cfg["seed"], "bf16")
    want = oracle.heat_bf16_sr(u0, cfg["r"], cfg["steps"], seed=20260)
    got = gpu_heat_sr(gpu, u0, cfg["r"], cfg["steps"], 20260, mode=mode)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("dims", [(67, 35, 20), (130, 9, 40), (3, 3, 3), (1030, 13, 5),
                                  (520, 66, 37), (1024, 12, 36), (12, 5, 70)])
def test_sr_ragged_shapes_bitwise(gpu, dims):
    note("heat bf16-sr ragged %s" % (dims,))
    u0 = field(dims, dims[0] + dims[1] + dims[2], "bf16")
    want = oracle.heat_bf16_sr(u0, 0.15, 7, seed=3, step0=11)
    for mode in ("split", "fused"):
        assert np.array_equal(gpu_heat_sr(gpu, u0, 0.15, 7, 3, step0=11, mode=mode), want), mode


def test_sr_every_tile_shape_parts_and_64_bit_keys(gpu):
    dims = (2056, 37, 75)
    u0 = field(dims, 32, "bf16")
    seed, step0 = 0x1234_5678_9ABC_DEF0, (1 << 33) + 5
    want = oracle.heat_bf16_sr(u0, 1.0 / 6.5, 5, seed=seed, step0=step0)
    shapes = built_shapes("bf16")
    try:
        for shape in shapes:
            note("heat bf16-sr tiling %s" % (shape,))
            gpu.set_tiling(*shape, xcd=3, dtype="bf16")
            assert np.array_equal(gpu_heat_sr(gpu, u0, 1.0 / 6.5, 5, seed, step0=step0), want), shape
    finally:
        gpu.set_tiling(dtype="bf16")
    for parts in (2, 7):
        note("heat bf16-sr parts=%d" % parts)
        assert np.array_equal(gpu_heat_sr(gpu, u0, 1.0 / 6.5, 5, seed, step0=step0, parts=parts),
                              want)


def test_sr_calls_compose_and_depend_on_seed(gpu):
    dims = (256, 20, 30)
    u0 = field(dims, 8, "bf16")
    note("heat bf16-sr composition")
    u = to_device(u0)
    un = torch.empty_like(u)
    gpu.heat_step_sr(u, un, 0.12, 4, 77, step0=0)
    gpu.heat_step_sr(u, un, 0.12, 5, 77, step0=4)
    torch.cuda.synchronize()
    whole = gpu_heat_sr(gpu, u0, 0.12, 9, 77)
    assert np.array_equal(to_host(u), whole)
    assert np.array_equal(whole, oracle.heat_bf16_sr(u0, 0.12, 9, seed=77))
    assert not np.array_equal(whole, gpu_heat_sr(gpu, u0, 0.12, 9, 78))


def test_sr_full_size_short_run_bitwise_on_slabs(gpu):
    cfg = inputs.HEAT_PRECISION
    n, r, steps, planes, seed = cfg["n"], cfg["r"], 3, 24, 99
    note("heat bf16-sr %d^3 %d steps, oracle on the first and last %d planes" % (n, steps, planes))
    u0 = inputs.sine_field_lowp(n, n, n, 1e-3, cfg["seed"], "bf16")
    lo, hi = u0[:planes].copy(), u0[n - planes:].copy()
    u = to_device(u0)
    del u0
    un = torch.empty_like(u)
    gpu.heat_step_sr(u, un, r, steps, seed)
    torch.cuda.synchronize()
    got_lo, got_hi = to_host(u[:planes - steps]), to_host(u[n - planes + steps:])
    want_lo = oracle.heat_bf16_sr(lo, r, steps, seed=seed)[:planes - steps]
    want_hi = oracle.heat_bf16_sr(hi, r, steps, seed=seed, node0=(n - planes) * n * n)[steps:]
    assert np.array_equal(got_lo, want_lo)
    assert np.array_equal(got_hi, want_hi)
