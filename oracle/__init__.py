"""CPU FP64 oracle for the 7-point heat update and 7-point-Laplacian CG.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
baseline leg of the benchmark may import this package.  The product library
never loads it and shares no code with it; the only thing both sides share
is the seeded input recipes, which hold none of the method's arithmetic.

The arithmetic lives in ``heatcg_oracle.c`` (plain loops, FP64, compiled
without floating-point contraction); this module only builds it and marshals
numpy arrays through ctypes.  Arrays are C-ordered ``(nz, ny, nx)``: x
fastest, z slowest, as the paper lays out ``u[k, j, i]``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "heatcg_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (OpenMP, no FP contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
               "-std=c11", "-Wall", "-shared", "-fPIC", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _configure(lib):
    dp = ctypes.POINTER(ctypes.c_double)
    L = ctypes.c_long
    lib.oracle_heat_sweep_f64.argtypes = [dp, dp, L, L, L, ctypes.c_double]
    lib.oracle_heat_sweep_f64.restype = None
    lib.oracle_heat_f64.argtypes = [dp, L, L, L, ctypes.c_double, L]
    lib.oracle_heat_f64.restype = ctypes.c_int
    lib.oracle_lap7_apply.argtypes = [dp, dp, L, L, L]
    lib.oracle_lap7_apply.restype = None
    lib.oracle_dot.argtypes = [dp, dp, L, L, L]
    lib.oracle_dot.restype = ctypes.c_double
    lib.oracle_cg.argtypes = [dp, dp, L, L, L, ctypes.c_double, L,
                              ctypes.POINTER(L), dp, dp]
    lib.oracle_cg.restype = ctypes.c_int
    lib.oracle_threads.argtypes = []
    lib.oracle_threads.restype = ctypes.c_int
    lib.oracle_set_threads.argtypes = [ctypes.c_int]
    lib.oracle_set_threads.restype = None
    lib.oracle_last_loop_seconds.argtypes = []
    lib.oracle_last_loop_seconds.restype = ctypes.c_double
    fp = ctypes.POINTER(ctypes.c_float)
    hp = ctypes.POINTER(ctypes.c_uint16)
    lib.oracle_heat_f32.argtypes = [fp, L, L, L, ctypes.c_float, L]
    lib.oracle_heat_f32.restype = ctypes.c_int
    lib.oracle_heat_bf16.argtypes = [hp, L, L, L, ctypes.c_float, L]
    lib.oracle_heat_bf16.restype = ctypes.c_int
    lib.oracle_heat_bf16_offset.argtypes = [hp, hp, L, L, L, ctypes.c_float, L]
    lib.oracle_heat_bf16_offset.restype = ctypes.c_int
    lib.oracle_bf16_round_array.argtypes = [fp, hp, L]
    lib.oracle_bf16_round_array.restype = None
    u32p = ctypes.POINTER(ctypes.c_uint32)
    U64 = ctypes.c_uint64
    lib.oracle_philox4x32_10.argtypes = [u32p, u32p, u32p]
    lib.oracle_philox4x32_10.restype = None
    lib.oracle_sr_bits.argtypes = [U64, U64, U64]
    lib.oracle_sr_bits.restype = ctypes.c_uint16
    lib.oracle_bf16_sr_from_f32.argtypes = [ctypes.c_float, ctypes.c_uint16]
    lib.oracle_bf16_sr_from_f32.restype = ctypes.c_uint16
    lib.oracle_heat_bf16_sr.argtypes = [hp, L, L, L, ctypes.c_float, L, U64, U64, U64]
    lib.oracle_lap7_apply_f32.argtypes = [fp, fp, L, L, L]
    lib.oracle_lap7_apply_f32.restype = None
    lib.oracle_dot_f32.argtypes = [fp, fp, L, L, L]
    lib.oracle_dot_f32.restype = ctypes.c_double
    LP = ctypes.POINTER(L)
    lib.oracle_cg_ir.argtypes = [dp, dp, L, L, L, ctypes.c_double, L, ctypes.c_double,
                                 ctypes.c_double, L, LP, LP, dp, LP]
    lib.oracle_cg_ir.restype = ctypes.c_int
    lib.oracle_heat_bf16_sr.restype = ctypes.c_int
    lib.oracle_heat_vk_sweep_f64.argtypes = [dp, dp, dp, dp, L, L, L, ctypes.c_double]
    lib.oracle_heat_vk_sweep_f64.restype = None
    lib.oracle_heat_vk_f64.argtypes = [dp, dp, dp, L, L, L, ctypes.c_double, L]
    lib.oracle_heat_vk_f64.restype = ctypes.c_int
    lib.oracle_heat_vk_f32.argtypes = [fp, fp, fp, L, L, L, ctypes.c_float, L]
    lib.oracle_heat_vk_f32.restype = ctypes.c_int
    return lib


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build(force=True)
    _lib = _configure(ctypes.CDLL(_LIB))
    return _lib


class using_library:
    """Temporarily route every oracle call to another build of the same
    source (used by the test that plants mistakes in the oracle)."""

    def __init__(self, path: str):
        self._path = path
        self._saved = None

    def __enter__(self):
        global _lib
        self._saved = _load()
        _lib = _configure(ctypes.CDLL(self._path))
        return self

    def __exit__(self, *exc):
        global _lib
        _lib = self._saved
        return False


def source_path() -> str:
    return _SRC


def threads() -> int:
    """OpenMP threads the oracle's loops use."""
    return int(_load().oracle_threads())


def set_threads(n: int) -> None:
    """Thread count of the oracle's parallel loops from now on."""
    _load().oracle_set_threads(int(n))


def last_loop_seconds() -> float:
    """Wall time of the step loop of the last ``heat`` call, or of the
    iteration loop of the last ``cg`` call (set-up and copies excluded)."""
    return float(_load().oracle_last_loop_seconds())


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64_c(a) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.ndim != 3:
        raise ValueError("expected a 3-D (nz, ny, nx) array")
    return a


def heat_sweep(u: np.ndarray, r: float) -> np.ndarray:
    """One explicit 7-point step (Eq. 4, kappa constant, f = 0); boundary kept."""
    u = _f64_c(u)
    out = u.copy()
    nz, ny, nx = u.shape
    _load().oracle_heat_sweep_f64(_ptr(u), _ptr(out), nx, ny, nz, float(r))
    return out


def heat(u0: np.ndarray, r: float, steps: int) -> np.ndarray:
    """``steps`` explicit steps from ``u0`` (not modified); returns u^steps."""
    u = _f64_c(u0).copy()
    nz, ny, nx = u.shape
    rc = _load().oracle_heat_f64(_ptr(u), nx, ny, nz, float(r), int(steps))
    if rc != 0:
        raise MemoryError("oracle_heat_f64 returned %d" % rc)
    return u


def heat_f32(u0: np.ndarray, r: float, steps: int) -> np.ndarray:
    """The explicit step in binary32 throughout (r rounded to binary32)."""
    u = np.ascontiguousarray(u0, dtype=np.float32).copy()
    if u.ndim != 3:
        raise ValueError("expected a 3-D (nz, ny, nx) array")
    nz, ny, nx = u.shape
    rc = _load().oracle_heat_f32(u.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                 nx, ny, nz, float(np.float32(r)), int(steps))
    if rc != 0:
        raise MemoryError("oracle_heat_f32 returned %d" % rc)
    return u


def heat_bf16(u0_bits: np.ndarray, r: float, steps: int) -> np.ndarray:
    """bfloat16 storage (uint16 bit patterns), binary32 arithmetic."""
    u = np.ascontiguousarray(u0_bits, dtype=np.uint16).copy()
    if u.ndim != 3:
        raise ValueError("expected a 3-D (nz, ny, nx) array")
    nz, ny, nx = u.shape
    rc = _load().oracle_heat_bf16(u.ctypes.data_as(ctypes.POINTER(ctypes.c_uint16)),
                                  nx, ny, nz, float(np.float32(r)), int(steps))
    if rc != 0:
        raise MemoryError("oracle_heat_bf16 returned %d" % rc)
    return u


def heat_bf16_sr(u0_bits: np.ndarray, r: float, steps: int, seed: int, step0: int = 0,
                 node0: int = 0) -> np.ndarray:
    """bfloat16 storage, binary32 arithmetic, stochastic rounding with the
    Philox4x32-10 bits of (seed, step, node); step s uses t = step0 + s.
    node0: linear index of u0_bits' first node in the array the bits are
    keyed to (a slab of planes k0.. of a larger array: k0 * nx * ny)."""
    u = np.ascontiguousarray(u0_bits, dtype=np.uint16).copy()
    if u.ndim != 3:
        raise ValueError("expected a 3-D (nz, ny, nx) array")
    nz, ny, nx = u.shape
    rc = _load().oracle_heat_bf16_sr(u.ctypes.data_as(ctypes.POINTER(ctypes.c_uint16)),
                                     nx, ny, nz, float(np.float32(r)), int(steps),
                                     int(seed) & (2 ** 64 - 1), int(step0) & (2 ** 64 - 1),
                                     int(node0))
    if rc != 0:
        raise MemoryError("oracle_heat_bf16_sr returned %d" % rc)
    return u


def heat_bf16_offset(base_bits: np.ndarray, delta_bits: np.ndarray, r: float,
                     steps: int) -> np.ndarray:
    """bfloat16 storage as offsets from a fixed bfloat16 base: returns the
    offsets after `steps` steps (the value is base + offset); see
    ``oracle_heat_bf16_offset``."""
    base = np.ascontiguousarray(base_bits, dtype=np.uint16)
    d = np.ascontiguousarray(delta_bits, dtype=np.uint16).copy()
    if base.shape != d.shape or base.ndim != 3:
        raise ValueError("expected two 3-D arrays of one shape")
    nz, ny, nx = d.shape
    hp = ctypes.POINTER(ctypes.c_uint16)
    st = _load().oracle_heat_bf16_offset(base.ctypes.data_as(hp), d.ctypes.data_as(hp), nx, ny,
                                         nz, float(np.float32(r)), int(steps))
    if st == -4:
        raise MemoryError("oracle_heat_bf16_offset: out of memory")
    return d


def philox4x32_10(ctr, key) -> tuple:
    """One Philox4x32-10 block: four 32-bit counter words, two key words."""
    c = (ctypes.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (ctypes.c_uint32 * 4)()
    _load().oracle_philox4x32_10(c, k, o)
    return tuple(o)


def sr_bits(p: int, t: int, seed: int) -> int:
    """The 16 random bits of node p at step t."""
    return int(_load().oracle_sr_bits(int(p), int(t), int(seed) & (2 ** 64 - 1)))


def bf16_sr(x: float, rho: int) -> int:
    """Stochastic rounding of one binary32 to bfloat16 with 16 bits rho."""
    return int(_load().oracle_bf16_sr_from_f32(float(np.float32(x)), int(rho)))


def bf16_round(x: np.ndarray) -> np.ndarray:
    """binary32 -> bfloat16 bit patterns, round to nearest, ties to even."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    out = np.empty(x.shape, dtype=np.uint16)
    _load().oracle_bf16_round_array(x.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                    out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint16)), x.size)
    return out


def bf16_widen(bits: np.ndarray) -> np.ndarray:
    """bfloat16 bit patterns -> binary32 (exact)."""
    return (np.asarray(bits, dtype=np.uint16).astype(np.uint32) << 16).view(np.float32)


def lap7_apply(x: np.ndarray) -> np.ndarray:
    """y = A x, A = 6 I - (face neighbours), zero Dirichlet data outside."""
    x = _f64_c(x)
    y = np.empty_like(x)
    nz, ny, nx = x.shape
    _load().oracle_lap7_apply(_ptr(x), _ptr(y), nx, ny, nz)
    return y


def dot(a: np.ndarray, b: np.ndarray) -> float:
    """Compensated dot product in a thread-count-independent order."""
    a = _f64_c(a)
    b = _f64_c(b)
    nz, ny, nx = a.shape
    return float(_load().oracle_dot(_ptr(a), _ptr(b), nx, ny, nz))


class CGResult:
    __slots__ = ("x", "status", "iters", "relres_true", "history")

    def __init__(self, x, status, iters, relres_true, history):
        self.x = x
        self.status = status
        self.iters = iters
        self.relres_true = relres_true
        self.history = history


def cg(b: np.ndarray, tol: float, maxit: int, x0: np.ndarray | None = None) -> CGResult:
    """Textbook CG on the 7-point Laplacian; see ``oracle_cg`` for statuses."""
    b = _f64_c(b)
    x = np.zeros_like(b) if x0 is None else _f64_c(x0).copy()
    nz, ny, nx = b.shape
    iters = ctypes.c_long(0)
    rel = ctypes.c_double(0.0)
    hist = np.full(int(maxit) + 1, np.nan)
    st = _load().oracle_cg(_ptr(b), _ptr(x), nx, ny, nz, float(tol), int(maxit),
                           ctypes.byref(iters), ctypes.byref(rel), _ptr(hist))
    return CGResult(x, int(st), int(iters.value), float(rel.value),
                    hist[: iters.value + 1].copy())


def lap7_apply_f32(x: np.ndarray) -> np.ndarray:
    """y = A x in binary32 (each operation rounded), zero outside the box."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    y = np.empty_like(x)
    nz, ny, nx = x.shape
    fp = ctypes.POINTER(ctypes.c_float)
    _load().oracle_lap7_apply_f32(x.ctypes.data_as(fp), y.ctypes.data_as(fp), nx, ny, nz)
    return y


def dot_f32(a: np.ndarray, b: np.ndarray) -> float:
    """a.b of binary32 arrays, accumulated in binary64."""
    a = np.ascontiguousarray(a, dtype=np.float32)
    b = np.ascontiguousarray(b, dtype=np.float32)
    if a.shape != b.shape or a.ndim != 3:
        raise ValueError("expected two 3-D arrays of one shape")
    nz, ny, nx = a.shape
    fp = ctypes.POINTER(ctypes.c_float)
    return float(_load().oracle_dot_f32(a.ctypes.data_as(fp), b.ctypes.data_as(fp), nx, ny, nz))


class IRResult:
    def __init__(self, x, status, iters, outer, relres_true, inner_iters):
        self.x = x
        self.status = status
        self.iters = iters
        self.outer = outer
        self.relres_true = relres_true
        self.inner_iters = inner_iters


def cg_ir(b: np.ndarray, tol: float, maxit: int, inner_tol: float = 1e-5,
          floor: float = 0.5, max_outer: int = 64, x0: np.ndarray | None = None) -> IRResult:
    """Binary64 iterative refinement around a binary32 inner CG; see
    ``oracle_cg_ir`` for the steps and statuses."""
    b = _f64_c(b)
    x = np.zeros_like(b) if x0 is None else _f64_c(x0).copy()
    nz, ny, nx = b.shape
    it, outer = ctypes.c_long(0), ctypes.c_long(0)
    rel = ctypes.c_double(0.0)
    hist = (ctypes.c_long * max_outer)()
    st = _load().oracle_cg_ir(_ptr(b), _ptr(x), nx, ny, nz, float(tol), int(maxit),
                              float(inner_tol), float(floor), int(max_outer),
                              ctypes.byref(it), ctypes.byref(outer), ctypes.byref(rel), hist)
    if st == -4:
        raise MemoryError("oracle_cg_ir: out of memory")
    return IRResult(x, st, it.value, outer.value, rel.value, list(hist[:outer.value]))


def _same_shape(u, *others):
    for a in others:
        if a.shape != u.shape:
            raise ValueError("kappa and rhs must have u's shape %s, got %s" % (u.shape, a.shape))


def heat_vk_sweep(u: np.ndarray, kappa: np.ndarray, rhs: np.ndarray, beta: float) -> np.ndarray:
    """One variable-coefficient step with a source (Eq. 4, flux form,
    rhs = dt f, beta = dt / (2 h^2)); boundary kept."""
    u, kappa, rhs = _f64_c(u), _f64_c(kappa), _f64_c(rhs)
    _same_shape(u, kappa, rhs)
    out = u.copy()
    nz, ny, nx = u.shape
    _load().oracle_heat_vk_sweep_f64(_ptr(u), _ptr(kappa), _ptr(rhs), _ptr(out), nx, ny, nz,
                                     float(beta))
    return out


def heat_vk(u0: np.ndarray, kappa: np.ndarray, rhs: np.ndarray, beta: float,
            steps: int) -> np.ndarray:
    """``steps`` variable-coefficient steps from ``u0`` (not modified)."""
    u, kappa, rhs = _f64_c(u0).copy(), _f64_c(kappa), _f64_c(rhs)
    _same_shape(u, kappa, rhs)
    nz, ny, nx = u.shape
    rc = _load().oracle_heat_vk_f64(_ptr(u), _ptr(kappa), _ptr(rhs), nx, ny, nz, float(beta),
                                    int(steps))
    if rc != 0:
        raise MemoryError("oracle_heat_vk_f64 returned %d" % rc)
    return u


def heat_vk_f32(u0: np.ndarray, kappa: np.ndarray, rhs: np.ndarray, beta: float,
                steps: int) -> np.ndarray:
    """The variable-coefficient step in binary32 throughout (beta rounded to
    binary32 once; kappa and rhs taken as binary32 arrays)."""
    f = lambda a: np.ascontiguousarray(a, dtype=np.float32)  # noqa: E731
    u, kappa, rhs = f(u0).copy(), f(kappa), f(rhs)
    if u.ndim != 3:
        raise ValueError("expected a 3-D (nz, ny, nx) array")
    _same_shape(u, kappa, rhs)
    nz, ny, nx = u.shape
    P = ctypes.POINTER(ctypes.c_float)
    rc = _load().oracle_heat_vk_f32(u.ctypes.data_as(P), kappa.ctypes.data_as(P),
                                    rhs.ctypes.data_as(P), nx, ny, nz, float(np.float32(beta)),
                                    int(steps))
    if rc != 0:
        raise MemoryError("oracle_heat_vk_f32 returned %d" % rc)
    return u
