"""GPU parity of the batched heat sweep: every problem of a batch against
the oracle run on that problem alone.

A batch shares launches only; each problem's sweep is the single-problem
tile body, so every comparison is bit-for-bit (binary64, binary32 and
bfloat16 storage), for every built batch shape and grid size, with and
without the captured step graph, including replays of one graph.  At the
configuration's full size (256 problems, edges 32..192, 200 steps) the
oracle checks every problem of up to 40^3 nodes over all 200 steps and
two large problems over a short run, and the maximum principle is checked
on every problem.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2608_11882_amd import inputs

pytestmark = pytest.mark.gpu


def note(msg):
    print("[case] " + msg, flush=True)


def make_fields(dims, seed, dtype):
    rng = np.random.default_rng(seed)
    out = []
    for nx, ny, nz in dims:
        u = inputs.uniform_field(nx, ny, nz, seed=0, rng=rng)
        if dtype == "f32":
            u = u.astype(np.float32)
        elif dtype == "bf16":
            u = inputs.to_bf16_bits(u)
        out.append(u)
    return out


def to_torch(a):
    if a.dtype == np.uint16:
        return torch.from_numpy(a.view(np.int16)).view(torch.bfloat16)
    return torch.from_numpy(a)


def to_numpy(t):
    t = t.contiguous()
    if t.dtype == torch.bfloat16:
        return t.view(torch.int16).cpu().numpy().view(np.uint16)
    return t.cpu().numpy()


def oracle_run(u0, r, steps):
    if u0.dtype == np.uint16:
        return oracle.heat_bf16(u0, r, steps)
    if u0.dtype == np.float32:
        return oracle.heat_f32(u0, r, steps)
    return oracle.heat(u0, r, steps)


def run_batch(hc, batch, fields, steps, graph=True):
    u = batch.empty()
    un = batch.empty()
    for v, f in zip(batch.views(u), fields):
        v.copy_(to_torch(f).cuda())
    batch.step(u, un, steps, graph=graph)
    torch.cuda.synchronize()
    return [to_numpy(v) for v in batch.views(u)]


SMALL_DIMS = [(3, 3, 3), (40, 12, 9), (64, 6, 70), (33, 20, 17), (128, 3, 5), (24, 24, 24),
              (96, 17, 40), (8, 50, 4), (200, 9, 12), (36, 36, 33)]


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("steps", [6, 7])
@pytest.mark.parametrize("graph", [False, True])
def test_small_batch_bitwise(gpu, dtype, steps, graph, time_block):
    note("batch %s %d problems, %d steps, graph=%s" % (dtype, len(SMALL_DIMS), steps, graph))
    rs = np.linspace(0.05, 1.0 / 6.0, len(SMALL_DIMS))
    fields = make_fields(SMALL_DIMS, 11, dtype)
    batch = gpu.Batch(SMALL_DIMS, rs, dtype)
    got = run_batch(gpu, batch, fields, steps, graph)
    for p, (g, f) in enumerate(zip(got, fields)):
        assert np.array_equal(g, oracle_run(f, rs[p], steps)), (dtype, p, SMALL_DIMS[p])
    batch.close()


def test_layout_is_packed_and_aligned(gpu):
    batch = gpu.Batch(SMALL_DIMS, [0.1] * len(SMALL_DIMS), "f32")
    end = 0
    for (nx, ny, nz), off, pitch in zip(batch.dims, batch.offsets, batch.pitches):
        assert off % 16 == 0 and off >= end           # 64-byte aligned problems
        assert pitch % 4 == 0 and nx <= pitch < nx + 4  # 16-byte rows
        end = off + pitch * ny * nz
    assert batch.total >= end and batch.total - end < 16
    want = sum(4.0 * (nx * ny * nz + (nx - 2) * (ny - 2) * (nz - 2)) for nx, ny, nz in SMALL_DIMS)
    assert batch.step_bytes == want
    batch.close()


def test_every_batch_shape_class_and_grid_bitwise(gpu, time_block):
    dims = [(64, 30, 40), (127, 9, 35), (73, 40, 20), (33, 32, 32), (190, 10, 18), (3, 5, 7),
            (500, 6, 9)]
    rs = [0.1, 0.15, 0.12, 1.0 / 6.5, 0.05, 0.16, 0.11]
    lib = gpu.load()
    for dtype in ("f32", "bf16", "f64"):
        fields = make_fields(dims, 3, dtype)
        want = [oracle_run(f, r, 5) for f, r in zip(fields, rs)]
        batch = gpu.Batch(dims, rs, dtype)
        shapes = [(v, nt, z, pf) for v in (2, 4, 8) for nt in (256, 512, 1024) for z in (16, 32)
                  for pf in (1, 2, 3)
                  if lib.hc_batch_set_tiling(batch._h, v, nt, z, pf, 0, -1, 0, 0) == 0]
        assert len(shapes) >= 3
        for sh in shapes:
            settings = [(-1, 0, 0, 8), (-1, 7, 17, 3), (-1, 1024, 64, 0)]
            settings += [(c, 0, 64, 8) for c in range(5)
                         if lib.hc_batch_set_tiling(batch._h, *sh, 8, c, 0, 64) == 0]
            for cls, grid, depth, xcd in settings:
                note("batch %s shape %s class %d grid %d depth %d xcd %d"
                     % (dtype, sh, cls, grid, depth, xcd))
                batch.set_tiling(*sh, xcd=xcd, width_class=cls, grid=grid, item_depth=depth)
                got = run_batch(gpu, batch, fields, 5, graph=(grid == 7))
                for p in range(len(dims)):
                    assert np.array_equal(got[p], want[p]), (dtype, sh, cls, grid, depth, p)
        batch.close()


def test_automatic_width_classes(gpu):
    # 16-byte lanes of 4 nodes; with 512 threads class c covers 32 << c
    # nodes by 64 >> c rows: among the classes whose tile covers a whole
    # row, the one leaving the fewest idle threads, the wider one on a tie
    dims = [(30, 66, 10), (60, 34, 10), (120, 18, 10), (250, 10, 10), (500, 6, 10), (3, 9, 9),
            (30, 10, 10), (200, 66, 10), (900, 10, 10)]
    batch = gpu.Batch(dims, [0.1] * len(dims), "f32")
    batch.set_tiling(4, 512)
    assert batch.classes() == [0, 1, 2, 3, 4, 3, 3, 3, 4]
    batch.set_tiling(4, 256)                        # 256 threads have no 128-lane class
    assert batch.classes() == [0, 1, 2, 3, 3, 2, 2, 3, 3]
    batch.close()


def test_graph_replays_and_odd_widths(gpu, time_block):
    dims = [(31, 20, 20), (64, 16, 18), (45, 9, 30)]      # odd widths: padded rows
    rs = [0.1, 0.12, 0.14]
    fields = make_fields(dims, 5, "f32")
    batch = gpu.Batch(dims, rs, "f32")
    u, un = batch.empty(), batch.empty()
    for v, f in zip(batch.views(u), fields):
        v.copy_(torch.from_numpy(f).cuda())
    for rep in range(1, 4):
        note("batch graph replay %d" % rep)
        batch.step(u, un, 4, graph=True)
        torch.cuda.synchronize()
        x = torch.ones(1000, device="cuda").sum()     # unrelated work between replays
        assert x.item() == 1000.0
        for p, (v, f) in enumerate(zip(batch.views(u), fields)):
            assert np.array_equal(v.cpu().numpy(), oracle.heat_f32(f, rs[p], 4 * rep)), (rep, p)
    assert batch.get_tiling()["vec"] == 4 and batch.get_tiling()["width_class"] == -1
    batch.close()


def test_autotune_keeps_results_bitwise(gpu):
    dims = [(64, 30, 40), (128, 9, 35), (96, 40, 20)]
    rs = [0.1, 0.15, 0.12]
    fields = make_fields(dims, 9, "f32")
    batch = gpu.Batch(dims, rs, "f32")
    u = batch.empty().zero_()       # padding included, so the comparison below sees no NaN
    for v, f in zip(batch.views(u), fields):
        v.copy_(torch.from_numpy(f).cuda())
    keep = u.clone()
    note("batch autotune")
    best = batch.autotune(u, trial_steps=2)
    assert torch.equal(u, keep)                     # the tuner does not write u
    res = batch.tune_results()
    assert len(res) >= 40 and best > 0
    # the kept shape is one of the four fastest of the first round (those
    # are timed again and the fastest of the second round is kept)
    t = batch.get_tiling()
    kept = [ms for sh, ms in res if sh == t]
    assert len(kept) == 1 and kept[0] <= sorted(ms for _, ms in res)[3]
    got = run_batch(gpu, batch, fields, 6)
    for p in range(len(dims)):
        assert np.array_equal(got[p], oracle.heat_f32(fields[p], rs[p], 6))
    batch.close()


def test_full_configuration_sampled(gpu):
    cfg = inputs.BATCHED
    dims, rs, rng = inputs.batched_problems(cfg["count"], cfg["lo"], cfg["hi"], cfg["seed"],
                                            cfg["r_lo"], cfg["r_hi"])
    fields = inputs.batched_fields(dims, rng, dtype=np.float32)
    note("batch full configuration: %d problems, %d steps" % (len(dims), cfg["steps"]))
    batch = gpu.Batch(dims, rs, "f32")
    u, un = batch.empty(), batch.empty()
    for v, f in zip(batch.views(u), fields):
        v.copy_(torch.from_numpy(f).cuda())
    batch.step(u, un, cfg["steps"], graph=True)
    torch.cuda.synchronize()
    views = batch.views(u)
    sizes = [int(np.prod(d)) for d in dims]
    small = [p for p in range(len(dims)) if sizes[p] <= 40 ** 3]
    assert len(small) >= 1
    for p in small:
        assert np.array_equal(views[p].cpu().numpy(), oracle.heat_f32(fields[p], rs[p], cfg["steps"]))
    for p in range(len(dims)):
        v = views[p]
        assert torch.isfinite(v).all().item()
        assert v.min().item() >= 0.0 and v.max().item() <= fields[p].max()
    # two of the largest problems, a short run of the same batch
    big = sorted(range(len(dims)), key=lambda p: -sizes[p])[:2]
    for v, f in zip(batch.views(u), fields):
        v.copy_(torch.from_numpy(f).cuda())
    batch.step(u, un, 3, graph=False)
    torch.cuda.synchronize()
    views = batch.views(u)
    for p in big:
        assert np.array_equal(views[p].cpu().numpy(), oracle.heat_f32(fields[p], rs[p], 3))
    batch.close()
