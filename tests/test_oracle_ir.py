"""Pins for the mixed-precision CG oracle: binary64 iterative refinement
around a binary32 inner CG with binary64 dot products.

References that do not re-type the oracle:
* the binary32 operator against scipy's sparse Kronecker sum, exactly on
  small-integer vectors (every binary32 operation is then exact) and within
  its rounding bound on general ones;
* the binary32 dot product against an exactly rounded sum (math.fsum) of
  the exact binary64 products;
* the refined solution against the exact fast Poisson solve (orthonormal
  DST-I) within the condition-number bound of the tolerance;
* finite termination of the first inner solve on an m-mode right-hand side
  (binary32 rounding leaves a residual far below the inner tolerance);
* the refinement itself: few outer steps, and inner iterations close to the
  binary64 CG's count (a broken refinement stalls or restarts from scratch).
"""
import math

import numpy as np
import scipy.fft

import oracle
from paper_2608_11882_amd import inputs
from test_oracle_cg import eigenvalues, fast_poisson, sparse_operator

U32 = 2.0 ** -24


def test_f32_operator_exact_on_small_integers_and_bounded_otherwise():
    nx, ny, nz = 9, 7, 5
    rng = np.random.default_rng(1)
    xi = rng.integers(-1000, 1000, size=(nz, ny, nx)).astype(np.float32)
    want = (sparse_operator(nx, ny, nz) @ xi.astype(np.float64).ravel()).reshape(xi.shape)
    assert np.array_equal(oracle.lap7_apply_f32(xi).astype(np.float64), want)
    xf = rng.uniform(-1, 1, size=(nz, ny, nx)).astype(np.float32)
    want = (sparse_operator(nx, ny, nz) @ xf.astype(np.float64).ravel()).reshape(xf.shape)
    got = oracle.lap7_apply_f32(xf).astype(np.float64)
    assert np.max(np.abs(got - want)) <= 24 * U32 * np.max(np.abs(xf))


def test_f32_dot_is_nearly_exact():
    rng = np.random.default_rng(2)
    a = rng.uniform(-1, 1, size=(6, 5, 7)).astype(np.float32)
    b = rng.uniform(-1, 1, size=(6, 5, 7)).astype(np.float32)
    exact = math.fsum(float(x) * float(y) for x, y in zip(a.ravel(), b.ravel()))
    got = oracle.dot_f32(a, b)
    assert abs(got - exact) <= 4 * 2.0 ** -53 * math.fsum(abs(float(x) * float(y)) for x, y in
                                                           zip(a.ravel(), b.ravel()))


def test_refined_solution_meets_the_condition_number_bound():
    nx, ny, nz = 30, 22, 17
    xs = inputs.manufactured_solution(nx, ny, nz, seed=31)
    b = (sparse_operator(nx, ny, nz) @ xs.ravel()).reshape(xs.shape)
    tol = 1e-10
    res = oracle.cg_ir(b, tol, 5000)
    assert res.status == 0 and res.relres_true <= tol
    exact = fast_poisson(b)
    lam = eigenvalues(nx, ny, nz)
    kappa = lam.max() / lam.min()
    assert np.linalg.norm(res.x - exact) / np.linalg.norm(exact) <= kappa * tol
    # the binary64 true residual is recomputed independently here
    r = b - (sparse_operator(nx, ny, nz) @ res.x.ravel()).reshape(b.shape)
    assert abs(np.linalg.norm(r) / np.linalg.norm(b) - res.relres_true) <= 1e-3 * tol


def test_first_inner_solve_terminates_in_m_iterations():
    nx, ny, nz = 24, 20, 12
    lam = eigenvalues(nx, ny, nz)
    for m in (1, 2, 4):
        rng = np.random.default_rng(40 + m)
        coef = np.zeros((nz, ny, nx))
        used = []
        while len(used) < m:
            idx = tuple(int(rng.integers(0, d)) for d in (nz, ny, nx))
            if all(abs(lam[idx] - lam[u]) > 1e-3 for u in used):
                used.append(idx)
                coef[idx] = rng.uniform(0.5, 1.5)
        b = scipy.fft.idstn(coef, type=1, norm="ortho")
        res = oracle.cg_ir(b, 1e-10, 2000, inner_tol=1e-5)
        assert res.status == 0
        assert res.inner_iters[0] == m, (m, res.inner_iters)


def test_refinement_converges_in_few_steps_near_the_f64_iteration_count():
    n = 40
    xs = inputs.manufactured_solution(n, seed=7)
    b = oracle.lap7_apply(xs)
    ref = oracle.cg(b, 1e-10, 5000)
    res = oracle.cg_ir(b, 1e-10, 5000)
    assert res.status == 0 and res.relres_true <= 1e-10
    assert 2 <= res.outer <= 5
    assert sum(res.inner_iters) == res.iters
    assert res.iters <= 1.3 * ref.iters
    # tighter inner solves need fewer outer steps
    tight = oracle.cg_ir(b, 1e-10, 5000, inner_tol=1e-6)
    assert tight.outer <= res.outer


def test_degenerate_inputs_and_iteration_cap():
    b = np.zeros((5, 6, 7))
    res = oracle.cg_ir(b, 1e-10, 10, x0=np.ones_like(b))
    assert res.status == 0 and res.iters == 0 and not res.x.any()
    xs = inputs.manufactured_solution(12, seed=3)
    b = oracle.lap7_apply(xs)
    res = oracle.cg_ir(b, 1e-10, 100, x0=xs)        # already solved
    assert res.status == 0 and res.iters == 0
    capped = oracle.cg_ir(oracle.lap7_apply(inputs.manufactured_solution(24, seed=5)),
                          1e-10, 7)
    assert capped.status == 1 and capped.iters == 7 and capped.relres_true > 1e-10
