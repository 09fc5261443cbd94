"""Seeded synthetic inputs for the heat sweep and the CG solve.

These recipes are shared by the HIP path and by the CPU oracle; they hold
none of the method's arithmetic (no stencil, no time step, no solver).  All
random draws come from ``numpy.random.default_rng(seed)`` (PCG64) in C order
over the interior nodes, plane by plane, so a chunked draw is the same
stream as one large draw.  Arrays are ``(nz, ny, nx)`` with x fastest.

Grid convention: an array edge counts every stored node including the
one-node Dirichlet layer, so a box of edge ``n`` has spacing h = 1/(n-1) and
node coordinates x_i = i h; ``n - 2`` nodes per axis are updated.  Boundary
nodes are forced to exactly 0.0 (the paper's zero Dirichlet condition, Eq. 5;
sin(pi) is not exactly 0 in floating point).
"""
from __future__ import annotations

import numpy as np


def node_coords(n: int) -> np.ndarray:
    """x_i = i / (n - 1), i = 0..n-1 (alg:heat3d: h = 1/(n-1))."""
    return np.arange(n, dtype=np.float64) / float(n - 1)


def _check_dims(nx: int, ny: int, nz: int) -> None:
    if min(nx, ny, nz) < 3:
        raise ValueError("every edge needs at least 3 nodes (one interior node)")


def sine_field(nx: int, ny: int, nz: int, modes=(1, 1, 1), noise: float = 0.0,
               seed: int | None = None, dtype=np.float64) -> np.ndarray:
    """sin(a pi x) sin(b pi y) sin(c pi z) plus optional U[-noise, noise].

    With modes (1,1,1) this is the paper's initial condition (Eq. 5).  The
    noise is drawn over the interior only, in [k][j][i] order.
    """
    _check_dims(nx, ny, nz)
    a, b, c = modes
    sx = np.sin(a * np.pi * node_coords(nx))
    sy = np.sin(b * np.pi * node_coords(ny))
    sz = np.sin(c * np.pi * node_coords(nz))
    rng = np.random.default_rng(seed) if noise else None
    out = np.zeros((nz, ny, nx), dtype=dtype)
    syx = sy[1:-1, None] * sx[None, 1:-1]
    for k in range(1, nz - 1):
        plane = sz[k] * syx
        if rng is not None:
            plane = plane + rng.uniform(-noise, noise, size=(ny - 2, nx - 2))
        out[k, 1:-1, 1:-1] = plane
    return out


def uniform_hotspot_field(nx: int, ny: int, nz: int, seed: int, sigma: float = 0.1,
                          amplitude: float = 1.0, dtype=np.float64) -> np.ndarray:
    """U[0,1] plus a Gaussian hot spot exp(-|x-c|^2 / (2 sigma^2)), c = centre."""
    _check_dims(nx, ny, nz)
    rng = np.random.default_rng(seed)
    dx2 = (node_coords(nx)[1:-1] - 0.5) ** 2
    dy2 = (node_coords(ny)[1:-1] - 0.5) ** 2
    dz2 = (node_coords(nz) - 0.5) ** 2
    dyx2 = dy2[:, None] + dx2[None, :]
    inv = 1.0 / (2.0 * sigma * sigma)
    out = np.zeros((nz, ny, nx), dtype=dtype)
    for k in range(1, nz - 1):
        noise = rng.random(size=(ny - 2, nx - 2))
        out[k, 1:-1, 1:-1] = noise + amplitude * np.exp(-(dz2[k] + dyx2) * inv)
    return out


def uniform_field(nx: int, ny: int, nz: int, seed: int, lo: float = 0.0,
                  hi: float = 1.0, dtype=np.float64, rng=None) -> np.ndarray:
    """U[lo, hi] on the interior, zero on the boundary layer."""
    _check_dims(nx, ny, nz)
    rng = np.random.default_rng(seed) if rng is None else rng
    out = np.zeros((nz, ny, nx), dtype=dtype)
    for k in range(1, nz - 1):
        out[k, 1:-1, 1:-1] = rng.uniform(lo, hi, size=(ny - 2, nx - 2))
    return out


def manufactured_solution(nx: int, ny: int | None = None, nz: int | None = None,
                          seed: int = 4) -> np.ndarray:
    """x* ~ U[-1, 1] on every unknown (the CG vectors carry no ghost layer)."""
    ny = nx if ny is None else ny
    nz = nx if nz is None else nz
    rng = np.random.default_rng(seed)
    out = np.empty((nz, ny, nx), dtype=np.float64)
    for k in range(nz):
        out[k] = rng.uniform(-1.0, 1.0, size=(ny, nx))
    return out


def batched_problems(count: int = 256, lo: int = 32, hi: int = 192, seed: int = 5,
                     r_lo: float = 0.05, r_hi: float = 0.16):
    """Many independent heat problems of uneven size.

    Returns (dims, rs, rng): dims is an int array (count, 3) of storage edges
    (nx, ny, nz), each drawn uniformly from [lo, hi]; rs holds one r per
    problem drawn from U[r_lo, r_hi]; the generator is returned positioned
    for the fields, which ``batched_fields`` then draws in problem order.
    """
    rng = np.random.default_rng(seed)
    dims = rng.integers(lo, hi + 1, size=(count, 3))
    rs = rng.uniform(r_lo, r_hi, size=count)
    return dims, rs, rng


def batched_fields(dims, rng, dtype=np.float32):
    """U[0,1] interior fields for each problem, in problem order."""
    out = []
    for nx, ny, nz in dims:
        out.append(uniform_field(int(nx), int(ny), int(nz), seed=0, dtype=dtype, rng=rng))
    return out


def to_bf16_bits(x) -> np.ndarray:
    """bfloat16 bit patterns (uint16) of float64 values, rounded once to the
    nearest bfloat16 with ties to even (no double rounding through binary32).
    Values must be finite and inside the bfloat16 normal range, or zero.

    x = m 2^e with 1/2 <= |m| < 1 (frexp); m 2^8 holds the 8 significant
    bits a bfloat16 keeps in its integer part, so rint (ties to even) of it,
    scaled back, is the rounded value -- every step exact in float64."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    m, e = np.frexp(x)
    y = np.ldexp(np.rint(np.ldexp(m, 8)), e - 8)
    ay = np.abs(y)
    if np.any((x != 0.0) & ((ay < 2.0 ** -126) | (ay > (2.0 - 2.0 ** -7) * 2.0 ** 127))) or \
            not np.all(np.isfinite(x)):
        raise ValueError("value outside the bfloat16 normal range")
    return (y.astype(np.float32).view(np.uint32) >> np.uint32(16)).astype(np.uint16)


def bf16_offset_split(u: np.ndarray):
    """A float64 field as a bfloat16 base and a bfloat16 offset: base =
    u rounded to the nearest bfloat16, offset = (u - base) rounded likewise
    (the difference is exact in float64).  Returns the two uint16 arrays."""
    u = np.ascontiguousarray(u, dtype=np.float64)
    base = to_bf16_bits(u)
    widened = (base.astype(np.uint32) << np.uint32(16)).view(np.float32).astype(np.float64)
    return base, to_bf16_bits(u - widened)


def sine_field_lowp(nx: int, ny: int, nz: int, noise: float, seed: int, dtype: str):
    """sine_field(..., noise, seed) rounded once from float64 to "f32" or
    "bf16" (bfloat16 returned as uint16 bit patterns), plane by plane."""
    if dtype not in ("f32", "bf16"):
        raise ValueError(dtype)
    _check_dims(nx, ny, nz)
    sx = np.sin(np.pi * node_coords(nx))
    sy = np.sin(np.pi * node_coords(ny))
    sz = np.sin(np.pi * node_coords(nz))
    rng = np.random.default_rng(seed)
    out = np.zeros((nz, ny, nx), dtype=np.float32 if dtype == "f32" else np.uint16)
    syx = sy[1:-1, None] * sx[None, 1:-1]
    for k in range(1, nz - 1):
        plane = sz[k] * syx
        if noise:
            plane = plane + rng.uniform(-noise, noise, size=(ny - 2, nx - 2))
        out[k, 1:-1, 1:-1] = plane.astype(np.float32) if dtype == "f32" else to_bf16_bits(plane)
    return out


# --- the paper's test case: variable coefficient and source ----------------

KAPPA_MEAN, KAPPA_AMP, KAPPA_MAX = 0.5, 0.45, 0.95   # Eq. (2), alg:heat3d


def paper_problem(n: int, dtype=np.float64) -> dict:
    """The paper's test case on an n^3 grid (Eq. 2, 3, 5 and the set-up of
    alg:heat3d): h = 1/(n-1), dt = h^2 / (12 kappa_max), beta = dt/(2 h^2);
    kappa = 0.5 + 0.45 sin(pi x) sin(pi y) sin(pi z) and
    rhs = dt (1 + cos(pi x) cos(pi y) cos(pi z)) at every node;
    u0 = sin(pi x) sin(pi y) sin(pi z) inside, 0 on the boundary layer.

    Returns dict(u0, kappa, rhs, beta, dt, h), arrays (n, n, n) of dtype
    (each value computed in float64 and rounded once)."""
    _check_dims(n, n, n)
    h = 1.0 / (n - 1)
    dt = h * h / (12.0 * KAPPA_MAX)
    beta = dt / (2.0 * h * h)
    x = node_coords(n)
    s, c = np.sin(np.pi * x), np.cos(np.pi * x)
    s2, c2 = s[:, None] * s[None, :], c[:, None] * c[None, :]
    kappa = np.empty((n, n, n), dtype=dtype)
    rhs = np.empty((n, n, n), dtype=dtype)
    u0 = np.zeros((n, n, n), dtype=dtype)
    for k in range(n):
        kappa[k] = KAPPA_MEAN + KAPPA_AMP * (s[k] * s2)
        rhs[k] = dt * (1.0 + c[k] * c2)
        if 0 < k < n - 1:
            u0[k, 1:-1, 1:-1] = (s[k] * s2)[1:-1, 1:-1]
    return dict(u0=u0, kappa=kappa, rhs=rhs, beta=beta, dt=dt, h=h)


def random_coefficients(nx: int, ny: int, nz: int, seed: int, k_lo: float = 0.05,
                        k_hi: float = KAPPA_MAX, f_amp: float = 1e-3, dtype=np.float64):
    """kappa ~ U[k_lo, k_hi] and rhs ~ U[-f_amp, f_amp] at every node (the
    boundary layer included: the update reads kappa there), drawn plane by
    plane, kappa's plane before rhs's.  Returns (kappa, rhs)."""
    _check_dims(nx, ny, nz)
    rng = np.random.default_rng(seed)
    kappa = np.empty((nz, ny, nx), dtype=dtype)
    rhs = np.empty((nz, ny, nx), dtype=dtype)
    for k in range(nz):
        kappa[k] = rng.uniform(k_lo, k_hi, size=(ny, nx))
        rhs[k] = rng.uniform(-f_amp, f_amp, size=(ny, nx))
    return kappa, rhs


# --- the configurations the library is measured and tested on -------------

def heat_small_f64(seed: int = 1, n: int = 66) -> np.ndarray:
    """64^3 interior (66^3 stored): sine initial condition + U[-1e-3, 1e-3]."""
    return sine_field(n, n, n, noise=1e-3, seed=seed)


def heat_large_f64(seed: int = 2, n: int = 512) -> np.ndarray:
    """512^3 stored: U[0,1] + central Gaussian hot spot, sigma = 0.1."""
    return uniform_hotspot_field(n, n, n, seed=seed)


HEAT_SMALL = dict(n=66, r=0.1, steps=100, seed=1)
HEAT_LARGE = dict(n=512, r=1.0 / 6.5, steps=1000, seed=2)
HEAT_PRECISION = dict(n=1024, r=0.15, steps=500, seed=3)
CG_LARGE = dict(n=256, tol=1e-10, maxit=10000, seed=4)
BATCHED = dict(count=256, lo=32, hi=192, r_lo=0.05, r_hi=0.16, steps=200, seed=5)
VARCOEF = dict(n=512, steps=500)     # the paper's test case (its runs: 500 steps)
