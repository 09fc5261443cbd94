"""Pins for the CG oracle and its 7-point operator.

References that do not re-type the oracle:
* the operator against scipy's sparse Kronecker sum of 1-D second
  differences (anisotropic box, so swapped axes fail);
* the solution against a dense direct solve and against the exact fast
  Poisson solve x = S diag(1/lambda) S b with S the orthonormal DST-I;
* finite termination: with a right-hand side in the span of m eigenvectors
  of distinct eigenvalue, CG ends in m iterations (exact arithmetic);
* the Hestenes-Stiefel monotonicity of the A-norm and 2-norm errors.

The method is the textbook CG named in the paper's CG case study (SpMV,
dot products and vector updates, Saad 2003); the relative residual is
||r|| / ||b||.
"""
import math

import numpy as np
import pytest
import scipy.fft
import scipy.sparse as sp

import oracle
from paper_2608_11882_amd import inputs


def sparse_operator(nx, ny, nz):
    def t(m):
        return sp.diags([-np.ones(m - 1), 2.0 * np.ones(m), -np.ones(m - 1)], [-1, 0, 1])
    ix, iy, iz = sp.identity(nx), sp.identity(ny), sp.identity(nz)
    return (sp.kron(sp.kron(t(nz), iy), ix) + sp.kron(sp.kron(iz, t(ny)), ix)
            + sp.kron(sp.kron(iz, iy), t(nx))).tocsr()


def eigenvalues(nx, ny, nz):
    kz = np.arange(1, nz + 1)[:, None, None]
    ky = np.arange(1, ny + 1)[None, :, None]
    kx = np.arange(1, nx + 1)[None, None, :]
    return (4 * np.sin(np.pi * kx / (2.0 * (nx + 1))) ** 2
            + 4 * np.sin(np.pi * ky / (2.0 * (ny + 1))) ** 2
            + 4 * np.sin(np.pi * kz / (2.0 * (nz + 1))) ** 2)


def fast_poisson(b):
    nz, ny, nx = b.shape
    return scipy.fft.idstn(scipy.fft.dstn(b, type=1, norm="ortho") / eigenvalues(nx, ny, nz),
                           type=1, norm="ortho")


def test_operator_matches_sparse_kronecker_sum():
    nx, ny, nz = 9, 6, 5
    x = inputs.manufactured_solution(nx, ny, nz, seed=21)
    want = (sparse_operator(nx, ny, nz) @ x.ravel()).reshape(x.shape)
    got = oracle.lap7_apply(x)
    assert np.max(np.abs(got - want)) < 1e-14


def test_operator_on_a_single_point_box():
    x = np.full((1, 1, 1), 2.5)
    assert oracle.lap7_apply(x)[0, 0, 0] == 15.0


def test_dot_is_accurate_under_cancellation():
    rng = np.random.default_rng(3)
    a = rng.uniform(-1, 1, size=(7, 5, 9)) * 10.0 ** rng.integers(-8, 9, size=(7, 5, 9))
    b = rng.uniform(-1, 1, size=a.shape)
    exact = math.fsum((a * b).ravel().tolist())
    assert abs(oracle.dot(a, b) - exact) <= 1e-15 * np.sum(np.abs(a * b))


def test_cg_matches_dense_direct_solve():
    nx, ny, nz = 6, 5, 4
    b = inputs.manufactured_solution(nx, ny, nz, seed=2)
    res = oracle.cg(b, tol=1e-13, maxit=500)
    want = np.linalg.solve(sparse_operator(nx, ny, nz).toarray(), b.ravel()).reshape(b.shape)
    assert res.status == 0
    assert np.max(np.abs(res.x - want)) < 1e-12 * np.max(np.abs(want))
    assert res.relres_true <= 1e-13 * 1.01


@pytest.mark.parametrize("m", [1, 2, 3, 5])
def test_finite_termination_in_m_iterations(m):
    """b built from m DST modes of distinct eigenvalue: CG needs exactly m steps."""
    nx, ny, nz = 7, 6, 5
    lam = eigenvalues(nx, ny, nz)
    rng = np.random.default_rng(100 + m)
    coef = np.zeros((nz, ny, nx))
    used = []
    while len(used) < m:
        idx = tuple(int(rng.integers(0, d)) for d in (nz, ny, nx))
        if all(abs(lam[idx] - lam[u]) > 1e-6 for u in used):
            used.append(idx)
            coef[idx] = rng.uniform(0.5, 1.5)
    b = scipy.fft.idstn(coef, type=1, norm="ortho")
    res = oracle.cg(b, tol=1e-11, maxit=50)
    assert res.status == 0
    assert res.iters == m
    assert np.max(np.abs(res.x - fast_poisson(b))) < 1e-10


def test_four_cubed_converges_within_distinct_eigenvalue_count():
    n = 4
    lam = np.sort(eigenvalues(n, n, n).ravel())
    distinct = 1 + int(np.sum(np.diff(lam) > 1e-9))
    b = inputs.manufactured_solution(n, seed=8)
    res = oracle.cg(b, tol=1e-13, maxit=100)
    assert res.status == 0 and res.iters <= distinct


def test_errors_decrease_monotonically_in_a_norm_and_2_norm():
    n = 10
    xs = inputs.manufactured_solution(n, seed=4)
    a = sparse_operator(n, n, n)
    b = (a @ xs.ravel()).reshape(xs.shape)
    prev_a = prev_2 = np.inf
    for k in range(1, 26):
        res = oracle.cg(b, tol=1e-30, maxit=k)
        assert res.status == 1 and res.iters == k
        e = (xs - res.x).ravel()
        ea, e2 = math.sqrt(e @ (a @ e)), np.linalg.norm(e)
        assert ea < prev_a and e2 < prev_2
        prev_a, prev_2 = ea, e2


def test_solution_matches_fast_poisson_solve_within_condition_bound():
    n = 24
    xs = inputs.manufactured_solution(n, seed=4)
    b = (sparse_operator(n, n, n) @ xs.ravel()).reshape(xs.shape)
    exact = fast_poisson(b)
    assert np.max(np.abs(exact - xs)) < 1e-12        # the RHS really is A x*
    tol = 1e-10
    res = oracle.cg(b, tol=tol, maxit=2000)
    lam = eigenvalues(n, n, n)
    kappa = lam.max() / lam.min()
    assert res.status == 0 and res.relres_true <= tol * 1.5
    assert np.linalg.norm(res.x - exact) / np.linalg.norm(exact) <= kappa * tol
    assert res.history[0] == pytest.approx(1.0) and res.history[-1] <= tol
    assert len(res.history) == res.iters + 1


def test_zero_rhs_gives_zero_solution():
    res = oracle.cg(np.zeros((4, 5, 6)), tol=1e-10, maxit=10,
                    x0=np.ones((4, 5, 6)))
    assert res.status == 0 and res.iters == 0 and not res.x.any()


def test_maxit_exhaustion_then_resume_converges():
    n = 12
    b = inputs.manufactured_solution(n, seed=6)
    first = oracle.cg(b, tol=1e-10, maxit=3)
    assert first.status == 1 and first.iters == 3
    second = oracle.cg(b, tol=1e-10, maxit=500, x0=first.x)
    assert second.status == 0 and second.relres_true <= 1.5e-10
