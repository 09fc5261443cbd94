"""GPU parity of the mixed-precision CG (binary64 iterative refinement
around a binary32 inner CG) and of its binary32 operator.

The binary32 operator evaluates the oracle's expression in the same order
and precision without contraction, so it is compared bit-for-bit.  The
refinement's dot products are summed in a different order on the GPU (a
block tree) than in the oracle (compensated sums), so, as for binary64 CG,
several results are correct; what must hold:
  * the binary64 true relative residual meets the tolerance;
  * inner iterations and outer steps are close to the oracle's;
  * the error against the exact solution is within kappa(A) * tol and close
    to the oracle's;
  * runs are deterministic.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2608_11882_amd import inputs

pytestmark = pytest.mark.gpu


def note(msg):
    print("[case] " + msg, flush=True)


def eigen_kappa(nx, ny, nz):
    lam = lambda n, k: 4 * np.sin(np.pi * k / (2.0 * (n + 1))) ** 2  # noqa: E731
    lo = lam(nx, 1) + lam(ny, 1) + lam(nz, 1)
    hi = lam(nx, nx) + lam(ny, ny) + lam(nz, nz)
    return hi / lo


def gpu_lap7_f32(hc, x):
    xt = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()
    yt = torch.empty_like(xt)
    hc.lap7_apply_f32(xt, yt)
    torch.cuda.synchronize()
    return yt.cpu().numpy()


def gpu_ir(hc, b, tol, maxit, x0=None, inner_tol=0.0, work=None):
    bt = torch.from_numpy(np.ascontiguousarray(b)).cuda()
    xt = torch.zeros_like(bt) if x0 is None else torch.from_numpy(np.ascontiguousarray(x0)).cuda()
    st, it, outer, rel = hc.cg_solve_ir(bt, xt, tol, maxit, inner_tol=inner_tol, work=work)
    return st, it, outer, rel, xt.cpu().numpy()


def close_iters(it, ref_it):
    return abs(it - ref_it) <= max(5, int(0.05 * ref_it))


@pytest.mark.parametrize("dims", [(1, 1, 1), (5, 3, 2), (64, 4, 32), (70, 9, 33),
                                  (128, 130, 40), (256, 256, 16), (33, 65, 97), (260, 12, 20)])
def test_f32_operator_bitwise(gpu, dims):
    nx, ny, nz = dims
    note("lap7 f32 %s" % (dims,))
    x = inputs.manufactured_solution(nx, ny, nz, seed=nx + 2 * ny + nz).astype(np.float32)
    assert np.array_equal(gpu_lap7_f32(gpu, x), oracle.lap7_apply_f32(x))


@pytest.mark.parametrize("dims", [(48, 48, 48), (70, 33, 41), (64, 64, 96)])
def test_refinement_against_oracle(gpu, dims):
    nx, ny, nz = dims
    note("cg_ir %s tol 1e-10" % (dims,))
    xs = inputs.manufactured_solution(nx, ny, nz, seed=4)
    b = oracle.lap7_apply(xs)
    tol = 1e-10
    ref = oracle.cg_ir(b, tol, 5000)
    st, it, outer, rel, x = gpu_ir(gpu, b, tol, 5000)
    assert ref.status == 0 and st == 0
    assert rel <= tol
    assert close_iters(it, ref.iters), (it, ref.iters)
    assert abs(outer - ref.outer) <= 1, (outer, ref.outer)
    err = np.linalg.norm(x - xs) / np.linalg.norm(xs)
    err_ref = np.linalg.norm(ref.x - xs) / np.linalg.norm(xs)
    assert err <= eigen_kappa(nx, ny, nz) * tol
    assert err <= 10 * err_ref + 1e-13
    rel_cpu = np.linalg.norm(b - oracle.lap7_apply(x)) / np.linalg.norm(b)
    assert abs(rel_cpu - rel) <= 1e-3 * rel + 1e-16


def built_ir_shapes():
    import paper_2608_11882_amd as hc
    lib = hc.load()
    shapes = []
    for vec in (1, 2, 4):
        for wx in (1, 2, 4):
            for by in (4, 8, 16):
                for zd in (8, 16, 32):
                    if lib.hc_cg_ir_set_tiling(vec, wx, by, zd, 0) == 0:
                        shapes.append((vec, wx, by, zd))
    hc.set_cg_ir_tiling()
    return shapes


def test_every_f32_shape_operator_bitwise_and_refinement_converges(gpu):
    shapes = built_ir_shapes()
    assert len(shapes) >= 8
    x1 = inputs.manufactured_solution(260, 66, 40, seed=5).astype(np.float32)
    x2 = inputs.manufactured_solution(71, 9, 35, seed=6).astype(np.float32)   # odd width
    want1, want2 = oracle.lap7_apply_f32(x1), oracle.lap7_apply_f32(x2)
    b = oracle.lap7_apply(inputs.manufactured_solution(40, 38, 36, seed=7))
    ref = oracle.cg_ir(b, 1e-10, 3000)
    try:
        for shape in shapes:
            for xcd in (0, 8):
                note("cg_ir shape vec,wx,by,zdepth=%s xcd=%d" % (shape, xcd))
                gpu.set_cg_ir_tiling(*shape, xcd=xcd)
                assert np.array_equal(gpu_lap7_f32(gpu, x1), want1), (shape, xcd)
                assert np.array_equal(gpu_lap7_f32(gpu, x2), want2), (shape, xcd)
                st, it, outer, rel, _ = gpu_ir(gpu, b, 1e-10, 3000)
                assert st == 0 and rel <= 1e-10 and close_iters(it, ref.iters), (shape, xcd, it)
    finally:
        gpu.set_cg_ir_tiling()


def test_deterministic_odd_width_and_caller_workspace(gpu):
    nx, ny, nz = 37, 30, 28     # odd x-edge: one-node lanes
    note("cg_ir determinism, odd width, caller workspace")
    b = oracle.lap7_apply(inputs.manufactured_solution(nx, ny, nz, seed=9))
    a = gpu_ir(gpu, b, 1e-10, 3000)
    work = torch.empty(gpu.cg_ir_workspace_bytes(nx, ny, nz), dtype=torch.uint8, device="cuda")
    c = gpu_ir(gpu, b, 1e-10, 3000, work=work)
    assert a[0] == 0 and a[1] == c[1] and a[2] == c[2] and np.array_equal(a[4], c[4])
    ref = oracle.cg_ir(b, 1e-10, 3000)
    assert close_iters(a[1], ref.iters)


def test_degenerate_inputs_and_iteration_cap(gpu):
    note("cg_ir zero rhs, exact start, maxit")
    st, it, outer, rel, x = gpu_ir(gpu, np.zeros((8, 9, 10)), 1e-10, 10, x0=np.ones((8, 9, 10)))
    assert st == 0 and it == 0 and not x.any()
    xs = inputs.manufactured_solution(16, seed=3)
    b = oracle.lap7_apply(xs)
    st, it, outer, rel, x = gpu_ir(gpu, b, 1e-10, 100, x0=xs)
    assert st == 0 and it == 0 and outer == 0
    st, it, outer, rel, x = gpu_ir(gpu, oracle.lap7_apply(inputs.manufactured_solution(24, seed=5)),
                                   1e-10, 7)
    assert st == 1 and it == 7 and rel > 1e-10
    ref = oracle.cg_ir(oracle.lap7_apply(inputs.manufactured_solution(24, seed=5)), 1e-10, 7)
    assert ref.status == 1 and ref.iters == 7


def test_large_config_against_oracle(gpu):
    """The full-size system (256^3, seed 4, tol 1e-10) by refinement on the
    GPU and in the oracle: binary64 residual within the tolerance, inner
    iterations close to the oracle's, the same number of outer steps (within
    one), error within kappa * tol and within 10x the oracle's."""
    cfg = inputs.CG_LARGE
    n = cfg["n"]
    note("cg_ir 256^3 tol 1e-10 (full size) against the oracle")
    xs = inputs.manufactured_solution(n, seed=cfg["seed"])
    b = oracle.lap7_apply(xs)
    st, it, outer, rel, x = gpu_ir(gpu, b, cfg["tol"], cfg["maxit"])
    assert st == 0 and rel <= cfg["tol"]
    note("cg_ir 256^3: GPU %d inner iterations, %d outer; running the oracle" % (it, outer))
    ref = oracle.cg_ir(b, cfg["tol"], cfg["maxit"])
    assert ref.status == 0 and ref.relres_true <= cfg["tol"]
    assert close_iters(it, ref.iters), (it, ref.iters)
    assert abs(outer - ref.outer) <= 1, (outer, ref.outer)
    err = np.linalg.norm(x - xs) / np.linalg.norm(xs)
    err_ref = np.linalg.norm(ref.x - xs) / np.linalg.norm(xs)
    assert err <= eigen_kappa(n, n, n) * cfg["tol"]
    assert err <= 10 * err_ref + 1e-13, (err, err_ref)
    # binary64 residual of the returned x recomputed by the oracle
    rel_cpu = np.linalg.norm(b - oracle.lap7_apply(x)) / np.linalg.norm(b)
    assert abs(rel_cpu - rel) <= 1e-3 * rel
    note("cg_ir 256^3: oracle %d inner / %d outer; error %.3g (oracle %.3g)"
         % (ref.iters, ref.outer, err, err_ref))


def test_more_blocks_than_threads_against_oracle(gpu):
    """A binary32 tile of 64 x 4 nodes (256 threads) on a 200 x 100 x 40 box:
    300 blocks, so the inner solve's reductions fold two partial sums per
    thread."""
    nx, ny, nz = 200, 100, 40
    note("cg_ir %dx%dx%d with 1x1x4x16 tiles (300 blocks)" % (nx, ny, nz))
    xs = inputs.manufactured_solution(nx, ny, nz, seed=22)
    b = oracle.lap7_apply(xs)
    ref = oracle.cg_ir(b, 1e-10, 5000)
    try:
        gpu.set_cg_ir_tiling(1, 1, 4, 16, xcd=8)
        st, it, outer, rel, x = gpu_ir(gpu, b, 1e-10, 5000)
    finally:
        gpu.set_cg_ir_tiling()
    assert st == 0 and rel <= 1e-10
    assert close_iters(it, ref.iters) and abs(outer - ref.outer) <= 1, (it, outer, ref.iters)
    err = np.linalg.norm(x - xs) / np.linalg.norm(xs)
    err_ref = np.linalg.norm(ref.x - xs) / np.linalg.norm(xs)
    assert err <= 10 * err_ref + 1e-13
