"""Pins of the oracle's bfloat16 step with stochastic rounding.

* The generator is Philox4x32-10: its known-answer vectors (distributed by
  its authors) must come out exactly.
* Stochastic rounding is exactly unbiased by construction: over all 2^16
  values of the random bits, the mean of the rounded value equals the
  binary32 input exactly, and each result is one of the two bfloat16
  neighbours of the input.
* A step's results bracket the binary32 step of the same widened field, and
  the number of round-ups matches the discarded fractions within a
  binomial bound.
* Steps compose (the counter advances with the step index) and depend on
  the seed.
* On the small sine configuration, where round-to-nearest stagnates, the
  stochastic form tracks the FP64 oracle to about one bfloat16 ulp.
"""
import json
import os

import numpy as np

import oracle
from paper_2608_11882_amd import inputs

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                      "philox4x32_10_kat.json")


def widen(bits):
    return oracle.bf16_widen(bits)


def test_philox_known_answer_vectors():
    kat = json.load(open(GOLDEN))
    for v in kat["vectors"]:
        got = oracle.philox4x32_10([int(x, 16) for x in v["ctr"]], [int(x, 16) for x in v["key"]])
        assert got == tuple(int(x, 16) for x in v["out"])


def test_sr_bits_are_uniform_and_vary_with_step_and_seed():
    bits = np.array([oracle.sr_bits(p, 7, 99) for p in range(4096)])
    counts = np.bincount(bits >> 12, minlength=16)          # top 4 bits
    chi2 = np.sum((counts - 256.0) ** 2 / 256.0)
    assert chi2 < 60.0                                      # 15 dof, far tail
    assert bits.min() >= 0 and bits.max() <= 0xFFFF
    other_step = np.array([oracle.sr_bits(p, 8, 99) for p in range(256)])
    other_seed = np.array([oracle.sr_bits(p, 7, 98) for p in range(256)])
    assert np.mean(other_step == bits[:256]) < 0.05
    assert np.mean(other_seed == bits[:256]) < 0.05


def test_rounding_is_exactly_unbiased_over_all_random_bits():
    rng = np.random.default_rng(3)
    xs = list(rng.uniform(-2, 2, size=3).astype(np.float32)) + \
        [np.float32(1.0 + 2.0 ** -9), np.float32(-3.0e-3), np.float32(0.5)]
    rho = np.arange(1 << 16)
    for x in xs:
        xb = int(np.float32(x).view(np.uint32))
        lo, up = xb >> 16, (xb >> 16) + 1
        res = np.array([oracle.bf16_sr(x, int(q)) for q in rho], dtype=np.int64)
        assert set(np.unique(res)) <= {lo, up}
        n_up = int(np.sum(res == up))
        assert n_up == (xb & 0xFFFF)       # up with probability (discarded bits) / 2^16
        mean = np.mean(widen(res.astype(np.uint16)).astype(np.float64))
        assert mean == float(x)            # exact: the average of 2^16 dyadic values


def test_step_brackets_the_binary32_step_and_rounds_up_at_the_right_rate():
    n = 40
    u0 = inputs.to_bf16_bits(inputs.uniform_field(n, n, n, seed=21))
    r = 0.13
    got = oracle.heat_bf16_sr(u0, r, 1, seed=5)
    v = oracle.heat_f32(widen(u0), r, 1)               # the binary32 step
    vb = v.view(np.uint32)
    lo = (vb >> 16).astype(np.int64)
    g = got.astype(np.int64)
    up = g == lo + 1
    assert np.all((g == lo) | up)
    frac = (vb & 0xFFFF).astype(np.float64) / 65536.0
    assert not np.any(up & (frac == 0))                 # representable values stay
    inner = np.s_[1:-1, 1:-1, 1:-1]
    mean_up, var = frac[inner].sum(), (frac[inner] * (1 - frac[inner])).sum()
    assert abs(up[inner].sum() - mean_up) <= 5 * np.sqrt(var)
    # the Dirichlet layer is never written
    assert np.array_equal(got[0], u0[0]) and np.array_equal(got[:, :, -1], u0[:, :, -1])


def test_steps_compose_and_depend_on_the_seed():
    n = 20
    u0 = inputs.to_bf16_bits(inputs.uniform_field(n, n, n, seed=4))
    a = oracle.heat_bf16_sr(u0, 0.1, 7, seed=11)
    b = oracle.heat_bf16_sr(oracle.heat_bf16_sr(u0, 0.1, 3, seed=11), 0.1, 4, seed=11, step0=3)
    assert np.array_equal(a, b)
    c = oracle.heat_bf16_sr(u0, 0.1, 7, seed=12)
    d = oracle.heat_bf16_sr(oracle.heat_bf16_sr(u0, 0.1, 3, seed=11), 0.1, 4, seed=11, step0=0)
    assert not np.array_equal(a, c)
    assert not np.array_equal(a, d)
    # r = 0: every value is representable, nothing moves
    assert np.array_equal(oracle.heat_bf16_sr(u0, 0.0, 5, seed=1), u0)


def test_stochastic_rounding_removes_the_stagnation():
    n, r, steps = 34, 0.15, 200
    u64 = inputs.sine_field(n, n, n, noise=1e-3, seed=1)
    ref = oracle.heat(u64, r, steps)
    b = inputs.to_bf16_bits(u64)
    norm = np.linalg.norm(ref)
    e_sr = np.linalg.norm(widen(oracle.heat_bf16_sr(b, r, steps, seed=2024)) - ref) / norm
    e_rne = np.linalg.norm(widen(oracle.heat_bf16(b, r, steps)) - ref) / norm
    # about one bfloat16 ulp (2^-8 relative) versus a stalled field
    assert e_sr < 2.0 ** -7
    assert e_rne > 10 * e_sr


def test_slab_with_node_offset_equals_the_whole_array():
    """node0 keys a slab's bits to its place in a larger array: the slab
    [k0, k0 + m) of a whole-array run equals the slab run with node0, away
    from the slab's cut planes (s steps reach s planes)."""
    n, k0, m, steps = 12, 5, 7, 2
    u0 = inputs.to_bf16_bits(inputs.uniform_field(n, n, n, seed=6))
    whole = oracle.heat_bf16_sr(u0, 0.1, steps, seed=9)
    part = oracle.heat_bf16_sr(u0[k0:k0 + m], 0.1, steps, seed=9, node0=k0 * n * n)
    assert np.array_equal(part[steps:m - steps], whole[k0 + steps:k0 + m - steps])
    unkeyed = oracle.heat_bf16_sr(u0[k0:k0 + m], 0.1, steps, seed=9)
    assert not np.array_equal(unkeyed[steps:m - steps], whole[k0 + steps:k0 + m - steps])
