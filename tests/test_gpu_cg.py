"""GPU parity of CG on the 7-point Laplacian and of its SpMV.

The SpMV evaluates the oracle's expression in the same order without
contraction, so it is compared bit-for-bit.  CG iterates depend on the
summation order of the dot products (a block tree on the GPU, compensated
sums on the CPU), so several results are correct; what must hold is:
  * the GPU's true relative residual meets the tolerance;
  * its iteration count is within max(3, 1%) of the oracle's;
  * its error against the exact solution is within the condition-number
    bound kappa(A) * tol (and, in practice, close to the oracle's);
  * exact-arithmetic facts: m-mode right-hand sides finish in m iterations;
  * the GPU run is deterministic (two runs, same bits).
"""
import numpy as np
import pytest
import scipy.fft
import torch

import oracle
from paper_2608_11882_amd import inputs

pytestmark = pytest.mark.gpu


def note(msg):
    print("[case] " + msg, flush=True)


def eigenvalues(nx, ny, nz):
    kz = np.arange(1, nz + 1)[:, None, None]
    ky = np.arange(1, ny + 1)[None, :, None]
    kx = np.arange(1, nx + 1)[None, None, :]
    return (4 * np.sin(np.pi * kx / (2.0 * (nx + 1))) ** 2
            + 4 * np.sin(np.pi * ky / (2.0 * (ny + 1))) ** 2
            + 4 * np.sin(np.pi * kz / (2.0 * (nz + 1))) ** 2)


def gpu_lap7(hc, x):
    xt = torch.from_numpy(np.ascontiguousarray(x)).cuda()
    yt = torch.empty_like(xt)
    hc.lap7_apply(xt, yt)
    torch.cuda.synchronize()
    return yt.cpu().numpy()


def gpu_cg(hc, b, tol, maxit, x0=None):
    bt = torch.from_numpy(np.ascontiguousarray(b)).cuda()
    xt = torch.zeros_like(bt) if x0 is None else torch.from_numpy(x0).cuda()
    st, it, rel = hc.cg_solve(bt, xt, tol, maxit)
    return st, it, rel, xt.cpu().numpy()


@pytest.mark.parametrize("dims", [(1, 1, 1), (5, 3, 2), (64, 4, 32), (70, 9, 33),
                                  (128, 130, 40), (256, 256, 16), (33, 65, 97)])
def test_spmv_bitwise(gpu, dims):
    nx, ny, nz = dims
    note("lap7 %s" % (dims,))
    x = inputs.manufactured_solution(nx, ny, nz, seed=nx + ny + nz)
    assert np.array_equal(gpu_lap7(gpu, x), oracle.lap7_apply(x))


@pytest.mark.parametrize("dims", [(48, 48, 48), (70, 33, 41), (64, 64, 96)])
def test_cg_against_oracle(gpu, dims):
    nx, ny, nz = dims
    note("cg %s tol 1e-10" % (dims,))
    xs = inputs.manufactured_solution(nx, ny, nz, seed=4)
    b = oracle.lap7_apply(xs)
    tol = 1e-10
    ref = oracle.cg(b, tol, 5000)
    st, it, rel, x = gpu_cg(gpu, b, tol, 5000)
    assert ref.status == 0 and st == 0
    assert rel <= tol
    assert abs(it - ref.iters) <= max(3, int(0.01 * ref.iters)), (it, ref.iters)
    lam = eigenvalues(nx, ny, nz)
    kappa = lam.max() / lam.min()
    err = np.linalg.norm(x - xs) / np.linalg.norm(xs)
    err_ref = np.linalg.norm(ref.x - xs) / np.linalg.norm(xs)
    assert err <= kappa * tol
    assert err <= 10 * err_ref + 1e-13
    # the recomputed true residual agrees with a CPU evaluation
    rel_cpu = np.linalg.norm(b - oracle.lap7_apply(x)) / np.linalg.norm(b)
    assert abs(rel_cpu - rel) <= 1e-3 * rel + 1e-16


@pytest.mark.parametrize("m", [1, 2, 4])
def test_finite_termination_on_gpu(gpu, m):
    nx, ny, nz = 66, 20, 12
    note("cg %d-mode rhs" % m)
    lam = eigenvalues(nx, ny, nz)
    rng = np.random.default_rng(50 + m)
    coef = np.zeros((nz, ny, nx))
    used = []
    while len(used) < m:
        idx = tuple(int(rng.integers(0, d)) for d in (nz, ny, nx))
        if all(abs(lam[idx] - lam[u]) > 1e-4 for u in used):
            used.append(idx)
            coef[idx] = rng.uniform(0.5, 1.5)
    b = scipy.fft.idstn(coef, type=1, norm="ortho")
    st, it, rel, _ = gpu_cg(gpu, b, 1e-10, 50)
    assert st == 0 and it == m and rel <= 1e-10


def test_deterministic_and_zero_rhs(gpu):
    n = 40
    note("cg determinism + zero rhs")
    b = oracle.lap7_apply(inputs.manufactured_solution(n, seed=9))
    a = gpu_cg(gpu, b, 1e-10, 2000)
    c = gpu_cg(gpu, b, 1e-10, 2000)
    assert a[1] == c[1] and np.array_equal(a[3], c[3])
    st, it, rel, x = gpu_cg(gpu, np.zeros((8, 9, 10)), 1e-10, 10,
                            x0=np.ones((8, 9, 10)))
    assert st == 0 and it == 0 and not x.any()


def test_maxit_exhaustion_and_resume(gpu):
    n = 32
    note("cg maxit=5 then resume")
    b = oracle.lap7_apply(inputs.manufactured_solution(n, seed=10))
    st, it, rel, x = gpu_cg(gpu, b, 1e-10, 5)
    assert st == 1 and it == 5 and rel > 1e-10
    ref = oracle.cg(b, 1e-30, 5)
    assert np.max(np.abs(x - ref.x)) <= 1e-10 * np.max(np.abs(ref.x))
    st2, it2, rel2, _ = gpu_cg(gpu, b, 1e-10, 2000, x0=x)
    assert st2 == 0 and rel2 <= 1e-10


def test_caller_workspace_and_plain_entry_point(gpu):
    import ctypes
    n = 36
    note("cg with caller workspace; cg_solve C entry point")
    b = oracle.lap7_apply(inputs.manufactured_solution(n, seed=11))
    bt = torch.from_numpy(b).cuda()
    xt = torch.zeros_like(bt)
    work = torch.empty(gpu.cg_workspace_bytes(n, n, n), dtype=torch.uint8, device="cuda")
    st, it, rel = gpu.cg_solve(bt, xt, 1e-10, 2000, work=work)
    assert st == 0 and rel <= 1e-10
    x2 = torch.zeros_like(bt)
    torch.cuda.synchronize()
    rc = gpu.abi().cg_solve(ctypes.c_void_p(bt.data_ptr()), ctypes.c_void_p(x2.data_ptr()),
                            n, 1e-10, 2000)
    assert rc == 0
    iters = ctypes.c_int(0)
    relres = ctypes.c_double(0.0)
    gpu.abi().hc_cg_last_info(ctypes.byref(iters), ctypes.byref(relres))
    assert iters.value == it and relres.value <= 1e-10
    assert torch.equal(xt, x2)


def check_against_oracle(x, it, rel, ref, xs, b, tol, kappa):
    """The acceptance rule for CG parity (several results are correct)."""
    assert ref.status == 0 and ref.relres_true <= tol
    assert rel <= tol
    assert abs(it - ref.iters) <= max(3, int(0.01 * ref.iters)), (it, ref.iters)
    err = np.linalg.norm(x - xs) / np.linalg.norm(xs)
    err_ref = np.linalg.norm(ref.x - xs) / np.linalg.norm(xs)
    assert err <= kappa * tol, (err, kappa * tol)
    assert err <= 10 * err_ref + 1e-13, (err, err_ref)
    rel_cpu = np.linalg.norm(b - oracle.lap7_apply(x)) / np.linalg.norm(b)
    assert abs(rel_cpu - rel) <= 1e-3 * rel + 1e-16
    return err, err_ref


def test_large_config_against_oracle(gpu):
    """The full-size system (256^3, x* ~ U[-1, 1] with seed 4, b = A x*, tol
    1e-10) solved on the GPU and by the oracle: same acceptance rule as the
    small boxes.  The default tile launches 2048 blocks here, so every block
    folds eight partial sums per thread when it finishes a reduction."""
    cfg = inputs.CG_LARGE
    n = cfg["n"]
    note("cg 256^3 tol 1e-10 (full size) against the oracle")
    xs = inputs.manufactured_solution(n, seed=cfg["seed"])
    b = oracle.lap7_apply(xs)
    st, it, rel, x = gpu_cg(gpu, b, cfg["tol"], cfg["maxit"])
    assert st == 0
    note("cg 256^3: GPU %d iterations, relres %.3g; running the oracle" % (it, rel))
    ref = oracle.cg(b, cfg["tol"], cfg["maxit"])
    lam = eigenvalues(n, n, n)
    err, err_ref = check_against_oracle(x, it, rel, ref, xs, b, cfg["tol"],
                                        lam.max() / lam.min())
    note("cg 256^3: oracle %d iterations; error %.3g (oracle %.3g)" % (ref.iters, err, err_ref))


def test_more_blocks_than_threads_against_oracle(gpu):
    """256 x 256 x 48 at the default tile (128 x 4 nodes, z-blocks of 16):
    384 blocks of 256 threads, so a reduction's partials are folded two per
    thread before the block tree."""
    nx, ny, nz = 256, 256, 48
    note("cg %dx%dx%d (384 blocks) against the oracle" % (nx, ny, nz))
    tl = gpu.get_cg_tiling()
    blocks = (-(-nx // (64 * tl["vec"] * tl["wx"]))) * (-(-ny // tl["by"])) * \
        (-(-nz // tl["zdepth"]))
    assert blocks > 64 * tl["wx"] * tl["by"], blocks
    xs = inputs.manufactured_solution(nx, ny, nz, seed=21)
    b = oracle.lap7_apply(xs)
    st, it, rel, x = gpu_cg(gpu, b, 1e-10, 5000)
    assert st == 0
    ref = oracle.cg(b, 1e-10, 5000)
    lam = eigenvalues(nx, ny, nz)
    check_against_oracle(x, it, rel, ref, xs, b, 1e-10, lam.max() / lam.min())


def test_misaligned_workspace_is_rejected(gpu):
    """A caller workspace must be 256-byte aligned; an offset view is
    refused before any launch (x is left as it was)."""
    n = 20
    note("cg with a misaligned caller workspace")
    b = torch.from_numpy(oracle.lap7_apply(inputs.manufactured_solution(n, seed=15))).cuda()
    work = torch.empty(gpu.cg_workspace_bytes(n, n, n) + 256, dtype=torch.uint8, device="cuda")
    assert work.data_ptr() % 256 == 0
    x = torch.full_like(b, 3.0)
    for off in (8, 128):
        with pytest.raises(gpu.HeatCGError) as e:
            gpu.cg_solve(b, x, 1e-10, 100, work=work[off:])
        assert e.value.code == -1 and "aligned" in e.value.message
        with pytest.raises(gpu.HeatCGError) as e:
            gpu.cg_solve_ir(b, x, 1e-10, 100, work=work[off:])
        assert e.value.code == -1
    torch.cuda.synchronize()
    assert bool((x == 3.0).all())
    st, it, rel = gpu.cg_solve(b, torch.zeros_like(b), 1e-10, 500, work=work[256:])
    assert st == 0 and rel <= 1e-10


def test_concurrent_solves_on_one_device(gpu):
    """Two host threads solving at once on the library's workspace: solves
    on one device are serialized, so both give the single-thread bits."""
    import threading
    note("cg from two host threads")
    bs = [oracle.lap7_apply(inputs.manufactured_solution(n, seed=16 + n)) for n in (40, 56)]
    want = [gpu_cg(gpu, b, 1e-10, 3000) for b in bs]
    out = [None, None]

    def run(q):
        torch.cuda.set_device(0)
        with torch.cuda.stream(torch.cuda.Stream()):
            out[q] = gpu_cg(gpu, bs[q], 1e-10, 3000)
            torch.cuda.synchronize()

    for _ in range(3):
        th = [threading.Thread(target=run, args=(q,)) for q in (0, 1)]
        for t in th:
            t.start()
        for t in th:
            t.join()
        for q in (0, 1):
            assert out[q][:2] == want[q][:2] and np.array_equal(out[q][3], want[q][3])


def built_cg_shapes():
    """Every CG tile shape libheatcg.so accepts (probed through the C ABI)."""
    import paper_2608_11882_amd as hc
    lib = hc.load()
    shapes = []
    for vec in (1, 2):
        for wx in (1, 2, 4):
            for by in (4, 8, 16):
                for zd in (8, 16, 32):
                    if lib.hc_cg_set_tiling(vec, wx, by, zd, 0) == 0:
                        shapes.append((vec, wx, by, zd))
    hc.set_cg_tiling()
    return shapes


def test_every_cg_shape_spmv_bitwise_and_converges(gpu):
    shapes = built_cg_shapes()
    assert len(shapes) >= 10
    x1 = inputs.manufactured_solution(130, 66, 40, seed=5)
    x2 = inputs.manufactured_solution(71, 9, 35, seed=6)   # odd width: one-node lanes
    want1, want2 = oracle.lap7_apply(x1), oracle.lap7_apply(x2)
    b = oracle.lap7_apply(inputs.manufactured_solution(40, 38, 36, seed=7))
    ref = oracle.cg(b, 1e-10, 3000)
    try:
        for shape in shapes:
            for xcd in (0, 3, 8):
                note("cg shape vec,wx,by,zdepth=%s xcd=%d" % (shape, xcd))
                gpu.set_cg_tiling(*shape, xcd=xcd)
                assert np.array_equal(gpu_lap7(gpu, x1), want1), (shape, xcd)
                assert np.array_equal(gpu_lap7(gpu, x2), want2), (shape, xcd)
                st, it, rel, _ = gpu_cg(gpu, b, 1e-10, 3000)
                assert st == 0 and rel <= 1e-10 and abs(it - ref.iters) <= 3, (shape, xcd, it)
    finally:
        gpu.set_cg_tiling()


def test_non_finite_data_is_reported(gpu):
    """A NaN in b or an infinite initial guess ends the solve with
    HC_ENONFINITE (the residual kernel's test), for plain CG and for the
    refinement; the library stays usable afterwards."""
    n = 24
    note("cg non-finite b / x0")
    b = oracle.lap7_apply(inputs.manufactured_solution(n, seed=12))
    bad = b.copy()
    bad[3, 4, 5] = np.nan
    with pytest.raises(gpu.HeatCGError) as e:
        gpu_cg(gpu, bad, 1e-10, 100)
    assert e.value.code == -7
    x0 = np.zeros_like(b)
    x0[1, 2, 3] = np.inf
    with pytest.raises(gpu.HeatCGError) as e:
        gpu_cg(gpu, b, 1e-10, 100, x0=x0)
    assert e.value.code == -7
    bt = torch.from_numpy(bad).cuda()
    with pytest.raises(gpu.HeatCGError) as e:
        gpu.cg_solve_ir(bt, torch.zeros_like(bt), 1e-10, 100)
    assert e.value.code == -7
    st, it, rel, _ = gpu_cg(gpu, b, 1e-10, 2000)
    assert st == 0 and rel <= 1e-10


@pytest.mark.parametrize("maxit", [1, 2, 3, 4, 5, 6, 7, 15, 16, 17, 33])
def test_iteration_budget_across_host_polls(gpu, maxit):
    """The host polls the device scalars every 16 iterations; a budget that
    ends just before, at or after a poll stops at exactly maxit, and the
    iterate equals the one reached by an unlimited run after as many
    iterations (the oracle's, within the summation-order tolerance).  x
    takes its steps two at a time, so odd budgets end with one step still
    waiting, which the solver applies before it returns."""
    n = 40
    note("cg maxit=%d" % maxit)
    b = oracle.lap7_apply(inputs.manufactured_solution(n, seed=13))
    st, it, rel, x = gpu_cg(gpu, b, 1e-12, maxit)
    assert st == 1 and it == maxit
    ref = oracle.cg(b, 1e-30, maxit)
    assert ref.iters == maxit
    assert np.max(np.abs(x - ref.x)) <= 1e-9 * np.max(np.abs(ref.x))


def test_restarts_after_a_residual_gap(gpu):
    """A tolerance below what binary64 can reach (1e-17) lets the recursive
    residual meet it while the true residual cannot: the solver restarts
    from its iterate three times, then reports HC_ENOTCONV before maxit.
    Every restart begins a new group of x's waiting steps, so the returned
    x must carry every step taken: its residual, computed here from the
    returned x with the oracle's operator, is at the level binary64 allows
    and is the one the solver reported."""
    n = 20
    note("cg with tol 1e-17: residual gap and restarts")
    xs = inputs.manufactured_solution(n, seed=15)
    b = oracle.lap7_apply(xs)
    maxit = 5000
    st, it, rel, x = gpu_cg(gpu, b, 1e-17, maxit)
    assert st == 1 and it < maxit
    mine = np.linalg.norm(b - oracle.lap7_apply(x)) / np.linalg.norm(b)
    assert mine < 1e-13
    assert abs(rel - mine) <= 1e-6 * mine
    assert np.max(np.abs(x - xs)) <= 1e-11 * np.max(np.abs(xs))


def test_workspace_contents_do_not_matter(gpu):
    """Partial sums and scalar slots are written before they are read: a
    caller workspace full of NaN bit patterns gives the same bits as a
    zeroed one, for plain CG and for the refinement."""
    n = 30
    note("cg with a NaN-filled workspace")
    b = torch.from_numpy(oracle.lap7_apply(inputs.manufactured_solution(n, seed=14))).cuda()
    outs = []
    for fill in (0, 0xFF):
        work = torch.full((gpu.cg_workspace_bytes(n, n, n),), fill, dtype=torch.uint8,
                          device="cuda")
        x = torch.zeros_like(b)
        st, it, rel = gpu.cg_solve(b, x, 1e-10, 2000, work=work)
        assert st == 0 and rel <= 1e-10
        outs.append((it, x.cpu()))
    assert outs[0][0] == outs[1][0] and torch.equal(outs[0][1], outs[1][1])
    outs = []
    for fill in (0, 0xFF):
        work = torch.full((gpu.cg_ir_workspace_bytes(n, n, n),), fill, dtype=torch.uint8,
                          device="cuda")
        x = torch.zeros_like(b)
        st, it, outer, rel = gpu.cg_solve_ir(b, x, 1e-10, 2000, work=work)
        assert st == 0 and rel <= 1e-10
        outs.append((it, outer, x.cpu()))
    assert outs[0][:2] == outs[1][:2] and torch.equal(outs[0][2], outs[1][2])
