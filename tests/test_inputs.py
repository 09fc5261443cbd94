"""The seeded input recipes: determinism, chunking, boundary layer."""
import numpy as np

from paper_2608_11882_amd import inputs


def test_chunked_draws_equal_one_large_draw():
    nx, ny, nz = 9, 7, 6
    u = inputs.uniform_field(nx, ny, nz, seed=42, lo=-2.0, hi=3.0)
    ref = np.random.default_rng(42).uniform(-2.0, 3.0, size=(nz - 2, ny - 2, nx - 2))
    assert np.array_equal(u[1:-1, 1:-1, 1:-1], ref)


def test_boundary_layer_is_exactly_zero():
    for u in (inputs.sine_field(10, 9, 8, noise=1e-3, seed=1),
              inputs.uniform_hotspot_field(10, 9, 8, seed=2)):
        for sl in (np.s_[0], np.s_[-1], np.s_[:, 0], np.s_[:, -1], np.s_[:, :, 0], np.s_[:, :, -1]):
            assert not u[sl].any()


def test_sine_field_and_hotspot_values():
    n = 11
    u = inputs.sine_field(n, n, n)
    x = np.arange(n) / (n - 1)
    assert np.allclose(u[3, 4, 5], np.sin(np.pi * x[5]) * np.sin(np.pi * x[4]) * np.sin(np.pi * x[3]))
    h = inputs.uniform_hotspot_field(n, n, n, seed=2) - inputs.uniform_field(n, n, n, seed=2)
    assert abs(h[5, 5, 5] - 1.0) < 1e-15          # centre of the hot spot
    assert h[5, 5, 1] < h[5, 5, 3] < h[5, 5, 5]


def test_recipes_are_deterministic():
    a = inputs.heat_small_f64(seed=1, n=20)
    b = inputs.heat_small_f64(seed=1, n=20)
    c = inputs.heat_small_f64(seed=2, n=20)
    assert np.array_equal(a, b) and not np.array_equal(a, c)


def test_batched_problem_dimensions_and_rates():
    dims, rs, rng = inputs.batched_problems(count=64, seed=5)
    assert dims.shape == (64, 3) and dims.min() >= 32 and dims.max() <= 192
    assert rs.min() >= 0.05 and rs.max() <= 0.16
    fields = inputs.batched_fields(dims[:3], rng)
    assert [f.shape for f in fields] == [tuple(int(v) for v in d[::-1]) for d in dims[:3]]
