"""Python binding of libheatcg.so: argument marshalling only.

Every step of the computation runs in the HIP library; this module checks
torch tensors (device, dtype, contiguity, shape), passes their data
pointers and the current torch stream through ctypes, and turns status
codes into exceptions.  There is no fallback: if the library is not built,
every entry point raises.
"""
from __future__ import annotations

import ctypes
import os

__all__ = ["HeatCGError", "load", "abi", "library_path", "heat_step", "heat_step_sr", "cg_solve",
           "cg_workspace_bytes", "lap7_apply", "copy_probe", "prof_enable",
           "prof_read", "strerror", "KERNELS", "HC_OK", "HC_ENOTCONV", "set_tiling",
           "get_tiling", "DEFAULT_TILING", "set_cg_tiling", "get_cg_tiling",
           "DEFAULT_CG_TILING", "DTYPES", "HC_F64", "HC_F32", "HC_BF16",
           "AUTO_TILING", "tiling_for", "cg_solve_ir", "cg_ir_workspace_bytes",
           "lap7_apply_f32", "set_cg_ir_tiling", "get_cg_ir_tiling", "DEFAULT_CG_IR_TILING",
           "Batch", "heat_vk_step", "set_vk_tiling", "get_vk_tiling", "vk_tiling_for",
           "set_time_block", "get_time_block", "set_tiling2", "get_tiling2", "tiling2_for",
           "set_vk2_tiling", "get_vk2_tiling", "vk2_tiling_for", "cg_solve_noalloc",
           "set_zrun2", "get_zrun2", "set_vk2_zrun", "get_vk2_zrun",
           "CG_NOALLOC_BYTES"]

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libheatcg.so")

HC_OK, HC_ENOTCONV = 0, 1
HC_F64, HC_F32, HC_BF16 = 0, 1, 2
CG_NOALLOC_BYTES = 96 << 20  # HC_CG_NOALLOC_BYTES of heatcg.h
MODES = {"split": 0, "fused": 1, "plain": 2}
KERNELS = {"heat_interior": 0, "heat_boundary": 1, "heat_fused": 2, "heat_plain": 3,
           "cg_direction": 4, "cg_update": 5, "cg_residual": 6, "lap7": 7, "copy": 8,
           "cg32_direction": 9, "cg32_update": 10, "ir_residual": 11, "ir_update": 12,
           "batch": 13, "vk_interior": 14, "vk_boundary": 15, "vk_fused": 16, "vk_plain": 17,
           "heat2_interior": 18, "heat2_boundary": 19, "heat2_fused": 20,
           "vk2_interior": 21, "vk2_boundary": 22, "vk2_fused": 23,
           "cg_update_x": 24, "cg32_update_x": 25}

_lib = None


class HeatCGError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__("heatcg error %d: %s" % (code, message))
        self.code = code
        self.message = message


def library_path() -> str:
    return _LIB_PATH


def load():
    """Load libheatcg.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise ImportError("libheatcg.so is not built (%s); run __graft_entry__.build() "
                          "or python -m paper_2608_11882_amd.build" % _LIB_PATH)
    lib = ctypes.CDLL(_LIB_PATH)
    vp, i, d, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
    ip, dp = ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double)
    llp = ctypes.POINTER(ctypes.c_longlong)
    sig = {
        "heat_step": (i, [vp, vp, i, i, i, d, i]),
        "heat_step_ex": (i, [vp, vp, i, i, i, d, i, i, i, i, vp]),
        "heat_step_streams": (i, [vp, vp, i, i, i, d, i, i, i, vp, vp]),
        "heat_step_sr": (i, [vp, vp, i, i, i, d, i, ctypes.c_uint64, ctypes.c_uint64, i, i, vp]),
        "cg_solve": (i, [vp, vp, i, d, i]),
        "cg_solve_ex": (i, [vp, vp, i, i, i, d, i, vp, sz, vp, ip, dp]),
        "cg_workspace_bytes": (sz, [i, i, i]),
        "cg_solve_noalloc": (i, [vp, vp, i, i, i, d, i, vp, ip, dp]),
        "hc_cg_last_info": (None, [ip, dp]),
        "hc_lap7_apply": (i, [vp, vp, i, i, i, vp]),
        "hc_copy_probe": (i, [vp, vp, sz, vp]),
        "hc_strerror": (ctypes.c_char_p, [i]),
        "hc_last_error_message": (ctypes.c_char_p, []),
        "hc_prof_enable": (i, [i]),
        "hc_prof_read": (i, [i, dp, llp, dp]),
        "hc_heat_set_tiling": (i, [i, i, i, i, i, i, i]),
        "hc_heat_get_tiling": (i, [i, ip, ip, ip, ip, ip, ip]),
        "hc_heat_tiling_for": (i, [i, i, vp, vp, ip, ip, ip, ip, ip, ip]),
        "hc_cg_set_tiling": (i, [i, i, i, i, i]),
        "hc_cg_ir_set_tiling": (i, [i, i, i, i, i]),
        "hc_cg_ir_get_tiling": (None, [ip, ip, ip, ip, ip]),
        "cg_solve_ir": (i, [vp, vp, i, i, i, d, i, d, vp, sz, vp, ip, ip, dp]),
        "cg_ir_workspace_bytes": (sz, [i, i, i]),
        "hc_lap7_apply_f32": (i, [vp, vp, i, i, i, vp]),
        "hc_batch_create": (i, [i, ctypes.POINTER(i), dp, i, ctypes.POINTER(vp)]),
        "hc_batch_destroy": (None, [vp]),
        "hc_batch_layout": (i, [vp, llp, ip, llp, dp]),
        "hc_batch_step": (i, [vp, vp, vp, i, i, vp]),
        "hc_batch_set_tiling": (i, [vp, i, i, i, i, i, i, i, i]),
        "hc_batch_get_tiling": (i, [vp, ip, ip, ip, ip, ip, ip, ip, ip]),
        "hc_batch_classes": (i, [vp, ip]),
        "hc_batch_autotune": (i, [vp, vp, i, vp, dp]),
        "hc_batch_tune_result": (i, [vp, i, ip, dp]),
        "hc_batch_steps_per_pass": (i, [vp]),
        "hc_cg_get_tiling": (None, [ip, ip, ip, ip, ip]),
        "heat_vk_step": (i, [vp, vp, vp, vp, i, i, i, d, i, i, i, i, vp]),
        "hc_heat_vk_set_tiling": (i, [i, i, i, i, i, i, i]),
        "hc_heat_vk_get_tiling": (i, [i, ip, ip, ip, ip, ip, ip]),
        "hc_heat_vk_tiling_for": (i, [i, i, vp, vp, vp, vp, ip, ip, ip, ip, ip, ip]),
        "hc_heat_set_time_block": (i, [i]),
        "hc_heat_get_time_block": (i, []),
        "hc_heat2_set_tiling": (i, [i, i, i, i, i, i, i]),
        "hc_heat2_get_tiling": (i, [i, ip, ip, ip, ip, ip, ip]),
        "hc_heat2_tiling_for": (i, [i, i, vp, vp, ip, ip, ip, ip, ip, ip]),
        "hc_heat2_set_zrun": (i, [i, i]),
        "hc_heat2_get_zrun": (i, [i]),
        "hc_heat_vk2_set_tiling": (i, [i, i, i, i, i, i, i]),
        "hc_heat_vk2_get_tiling": (i, [i, ip, ip, ip, ip, ip, ip]),
        "hc_heat_vk2_tiling_for": (i, [i, i, vp, vp, vp, vp, ip, ip, ip, ip, ip, ip]),
        "hc_heat_vk2_set_zrun": (i, [i, i]),
        "hc_heat_vk2_get_zrun": (i, [i]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def abi():
    """The raw ctypes library (for tests of the C ABI itself)."""
    return load()


def strerror(code: int) -> str:
    return load().hc_strerror(int(code)).decode()


def _check(code: int) -> int:
    if code < 0:
        lib = load()
        raise HeatCGError(code, "%s: %s" % (lib.hc_strerror(code).decode(),
                                            lib.hc_last_error_message().decode()))
    return code


def _stream_handle(t, stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream(t.device)
    return ctypes.c_void_p(stream.cuda_stream)


def _dtype_code(t):
    import torch
    codes = {torch.float64: HC_F64, torch.float32: HC_F32, torch.bfloat16: HC_BF16}
    if t.dtype not in codes:
        raise TypeError("unsupported dtype %s" % t.dtype)
    return codes[t.dtype]


def _require_cuda_3d(*ts):
    for t in ts:
        if not t.is_cuda:
            raise ValueError("expected a CUDA (HIP) tensor")
        if t.dim() != 3 or not t.is_contiguous():
            raise ValueError("expected a contiguous 3-D (nz, ny, nx) tensor")
        if t.shape != ts[0].shape or t.dtype != ts[0].dtype or t.device != ts[0].device:
            raise ValueError("tensors must share shape, dtype and device")


def heat_step(u, u_new, r: float, steps: int, mode: str = "split", parts: int = 1,
              stream=None, bnd_stream=None) -> None:
    """Advance ``u`` by ``steps`` explicit 7-point steps (result in ``u``).

    ``u_new`` is scratch of the same shape.  Enqueued on ``stream`` (default:
    torch's current stream); does not synchronize.  With ``bnd_stream`` (a
    torch stream, split mode only) the Boundary kernels run on it
    (heat_step_streams).
    """
    _require_cuda_3d(u, u_new)
    nz, ny, nx = u.shape
    lib = load()
    if bnd_stream is not None:
        if mode != "split":
            raise ValueError("a Boundary stream needs the split mode")
        _check(lib.heat_step_streams(ctypes.c_void_p(u.data_ptr()),
                                     ctypes.c_void_p(u_new.data_ptr()), nx, ny, nz, float(r),
                                     int(steps), _dtype_code(u), int(parts),
                                     _stream_handle(u, stream), _stream_handle(u, bnd_stream)))
        return
    _check(lib.heat_step_ex(ctypes.c_void_p(u.data_ptr()), ctypes.c_void_p(u_new.data_ptr()),
                            nx, ny, nz, float(r), int(steps), _dtype_code(u), MODES[mode],
                            int(parts), _stream_handle(u, stream)))


def heat_step_sr(u, u_new, r: float, steps: int, seed: int, step0: int = 0, mode: str = "split",
                 parts: int = 1, stream=None) -> None:
    """bfloat16 steps with stochastic rounding (torch.bfloat16 tensors): the
    random bits of node p at step step0 + s come from Philox4x32-10 keyed by
    ``seed``.  Otherwise as heat_step."""
    import torch
    _require_cuda_3d(u, u_new)
    if u.dtype != torch.bfloat16:
        raise TypeError("heat_step_sr needs torch.bfloat16 tensors")
    nz, ny, nx = u.shape
    lib = load()
    _check(lib.heat_step_sr(ctypes.c_void_p(u.data_ptr()), ctypes.c_void_p(u_new.data_ptr()),
                            nx, ny, nz, float(r), int(steps), int(seed) & (2 ** 64 - 1),
                            int(step0) & (2 ** 64 - 1), MODES[mode], int(parts),
                            _stream_handle(u, stream)))


def heat_vk_step(u, u_new, kappa, rhs, beta: float, steps: int, mode: str = "split",
                 parts: int = 1, stream=None) -> None:
    """Advance ``u`` by ``steps`` explicit steps of the variable-coefficient
    equation with a source: u_new = (u + rhs) + beta * (D_x + D_y + D_z),
    flux form, rhs = dt f, beta = dt / (2 h^2).  float64 or float32 tensors,
    all four of one shape; ``kappa`` and ``rhs`` are read only.  Enqueued on
    ``stream`` (default: torch's current stream); does not synchronize."""
    import torch
    _require_cuda_3d(u, u_new, kappa, rhs)
    if u.dtype not in (torch.float64, torch.float32):
        raise TypeError("heat_vk_step needs float64 or float32 tensors")
    nz, ny, nx = u.shape
    _check(load().heat_vk_step(ctypes.c_void_p(u.data_ptr()), ctypes.c_void_p(u_new.data_ptr()),
                               ctypes.c_void_p(kappa.data_ptr()), ctypes.c_void_p(rhs.data_ptr()),
                               nx, ny, nz, float(beta), int(steps), _dtype_code(u), MODES[mode],
                               int(parts), _stream_handle(u, stream)))


def cg_workspace_bytes(nx: int, ny: int, nz: int) -> int:
    return int(load().cg_workspace_bytes(nx, ny, nz))


def cg_solve(b, x, tol: float, maxit: int, work=None, stream=None):
    """Solve A x = b (7-point Laplacian, zero Dirichlet) in place in ``x``.

    Returns (status, iterations, true relative residual); status is 0
    (converged) or 1 (maxit reached).  Errors raise HeatCGError.
    """
    import torch
    _require_cuda_3d(b, x)
    if b.dtype != torch.float64:
        raise TypeError("cg_solve works in float64")
    nz, ny, nx = b.shape
    it = ctypes.c_int(0)
    rel = ctypes.c_double(0.0)
    wptr, wbytes = None, 0
    if work is not None:
        if not work.is_cuda or not work.is_contiguous():
            raise ValueError("work must be a contiguous CUDA tensor")
        wptr, wbytes = ctypes.c_void_p(work.data_ptr()), work.numel() * work.element_size()
    st = _check(load().cg_solve_ex(ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(x.data_ptr()),
                                   nx, ny, nz, float(tol), int(maxit), wptr, wbytes,
                                   _stream_handle(b, stream), ctypes.byref(it),
                                   ctypes.byref(rel)))
    return st, it.value, rel.value


def cg_solve_noalloc(b, x, tol: float, maxit: int, stream=None):
    """cg_solve on the library's fixed device workspace (no allocation);
    boxes whose workspace exceeds CG_NOALLOC_BYTES raise HeatCGError.

    Returns (status, iterations, true relative residual).
    """
    import torch
    _require_cuda_3d(b, x)
    if b.dtype != torch.float64:
        raise TypeError("cg_solve_noalloc works in float64")
    nz, ny, nx = b.shape
    it = ctypes.c_int(0)
    rel = ctypes.c_double(0.0)
    st = _check(load().cg_solve_noalloc(ctypes.c_void_p(b.data_ptr()),
                                        ctypes.c_void_p(x.data_ptr()), nx, ny, nz, float(tol),
                                        int(maxit), _stream_handle(b, stream), ctypes.byref(it),
                                        ctypes.byref(rel)))
    return st, it.value, rel.value


def cg_ir_workspace_bytes(nx: int, ny: int, nz: int) -> int:
    return int(load().cg_ir_workspace_bytes(nx, ny, nz))


def cg_solve_ir(b, x, tol: float, maxit: int, inner_tol: float = 0.0, work=None, stream=None):
    """Solve A x = b by binary64 iterative refinement around a binary32
    inner CG (in place in ``x``, float64 tensors).

    Returns (status, inner iterations, outer steps, true relative residual);
    status is 0 (converged) or 1 (not converged).  inner_tol <= 0 takes the
    library default.  Errors raise HeatCGError.
    """
    import torch
    _require_cuda_3d(b, x)
    if b.dtype != torch.float64:
        raise TypeError("cg_solve_ir works on float64 tensors")
    nz, ny, nx = b.shape
    it, out = ctypes.c_int(0), ctypes.c_int(0)
    rel = ctypes.c_double(0.0)
    wptr, wbytes = None, 0
    if work is not None:
        if not work.is_cuda or not work.is_contiguous():
            raise ValueError("work must be a contiguous CUDA tensor")
        wptr, wbytes = ctypes.c_void_p(work.data_ptr()), work.numel() * work.element_size()
    st = load().cg_solve_ir(ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(x.data_ptr()),
                            nx, ny, nz, float(tol), int(maxit), float(inner_tol), wptr, wbytes,
                            _stream_handle(b, stream), ctypes.byref(it), ctypes.byref(out),
                            ctypes.byref(rel))
    if st < 0:
        _check(st)
    return st, it.value, out.value, rel.value


def lap7_apply_f32(x, y, stream=None) -> None:
    """y = A x in binary32 (float32 tensors); enqueued, no sync."""
    import torch
    _require_cuda_3d(x, y)
    if x.dtype != torch.float32:
        raise TypeError("lap7_apply_f32 works in float32")
    nz, ny, nx = x.shape
    _check(load().hc_lap7_apply_f32(ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                    nx, ny, nz, _stream_handle(x, stream)))


def lap7_apply(x, y, stream=None) -> None:
    """y = A x (7-point Laplacian, zero outside); enqueued, no sync."""
    import torch
    _require_cuda_3d(x, y)
    if x.dtype != torch.float64:
        raise TypeError("lap7_apply works in float64")
    nz, ny, nx = x.shape
    _check(load().hc_lap7_apply(ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                nx, ny, nz, _stream_handle(x, stream)))


def copy_probe(src, dst, stream=None) -> None:
    """dst = src with the library's streaming copy kernel; enqueued, no sync."""
    if not (src.is_cuda and dst.is_cuda and src.is_contiguous() and dst.is_contiguous()):
        raise ValueError("expected contiguous CUDA tensors")
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes:
        raise ValueError("size mismatch")
    _check(load().hc_copy_probe(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()),
                                nbytes, _stream_handle(src, stream)))


DTYPES = {"f64": HC_F64, "f32": HC_F32, "bf16": HC_BF16}
_TILE_KEYS = ("vec", "wx", "by", "zdepth", "pf", "xcd")
# the default of every element type: the library's automatic choice per call
AUTO_TILING = dict.fromkeys(_TILE_KEYS, 0)
DEFAULT_TILING = {dt: dict(AUTO_TILING) for dt in DTYPES}


def set_tiling(vec: int | None = None, wx: int | None = None, by: int | None = None,
               zdepth: int | None = None, pf: int = 2, xcd: int = 8,
               dtype: str = "f64") -> None:
    """Tile shape of the z-marching heat kernels for one element type
    ("f64", "f32", "bf16"); with no shape given, the automatic choice.
    Results do not depend on the shape."""
    if vec is None and wx is None and by is None and zdepth is None:
        t = AUTO_TILING
    else:
        if None in (vec, wx, by, zdepth):
            raise ValueError("give vec, wx, by and zdepth, or none of them")
        t = dict(vec=vec, wx=wx, by=by, zdepth=zdepth, pf=pf, xcd=xcd)
    _check(load().hc_heat_set_tiling(DTYPES[dtype], *(int(t[k]) for k in _TILE_KEYS)))


def get_tiling(dtype: str = "f64") -> dict:
    """The setting for one element type (all zeros: automatic)."""
    v = [ctypes.c_int(0) for _ in range(6)]
    _check(load().hc_heat_get_tiling(DTYPES[dtype], *[ctypes.byref(x) for x in v]))
    return dict(zip(_TILE_KEYS, (x.value for x in v)))


def tiling_for(u, u_new=None, sr: bool = False) -> dict:
    """The tile shape heat_step (heat_step_sr with sr) would sweep these
    tensors with."""
    v = [ctypes.c_int(0) for _ in range(6)]
    un = u if u_new is None else u_new
    code = 3 if sr else _dtype_code(u)
    _check(load().hc_heat_tiling_for(code, int(u.shape[-1]),
                                     ctypes.c_void_p(u.data_ptr()),
                                     ctypes.c_void_p(un.data_ptr()),
                                     *[ctypes.byref(x) for x in v]))
    return dict(zip(_TILE_KEYS, (x.value for x in v)))


def set_time_block(steps_per_pass: int) -> None:
    """Steps per pass of the constant-coefficient z-marching sweeps (1 or
    2); results do not depend on it."""
    _check(load().hc_heat_set_time_block(int(steps_per_pass)))


def get_time_block() -> int:
    return int(load().hc_heat_get_time_block())


def set_tiling2(vec: int | None = None, wx: int | None = None, by: int | None = None,
                zdepth: int | None = None, pf: int = 2, xcd: int = 8,
                dtype: str = "f64") -> None:
    """Tile shape of the two-step sweep for one element type; with no shape
    given, the automatic choice."""
    if vec is None and wx is None and by is None and zdepth is None:
        t = AUTO_TILING
    else:
        if None in (vec, wx, by, zdepth):
            raise ValueError("give vec, wx, by and zdepth, or none of them")
        t = dict(vec=vec, wx=wx, by=by, zdepth=zdepth, pf=pf, xcd=xcd)
    _check(load().hc_heat2_set_tiling(DTYPES[dtype], *(int(t[k]) for k in _TILE_KEYS)))


def set_zrun2(planes: int = 0, dtype: str = "f64") -> None:
    """Output planes per block of the two-step sweep (0: automatic)."""
    _check(load().hc_heat2_set_zrun(DTYPES[dtype], int(planes)))


def get_zrun2(dtype: str = "f64") -> int:
    return _check(load().hc_heat2_get_zrun(DTYPES[dtype]))


def get_tiling2(dtype: str = "f64") -> dict:
    v = [ctypes.c_int(0) for _ in range(6)]
    _check(load().hc_heat2_get_tiling(DTYPES[dtype], *[ctypes.byref(x) for x in v]))
    return dict(zip(_TILE_KEYS, (x.value for x in v)))


def tiling2_for(u, u_new=None) -> dict:
    """The tile shape a two-step sweep of these tensors would run with."""
    v = [ctypes.c_int(0) for _ in range(6)]
    un = u if u_new is None else u_new
    _check(load().hc_heat2_tiling_for(_dtype_code(u), int(u.shape[-1]),
                                      ctypes.c_void_p(u.data_ptr()),
                                      ctypes.c_void_p(un.data_ptr()),
                                      *[ctypes.byref(x) for x in v]))
    return dict(zip(_TILE_KEYS, (x.value for x in v)))


def set_vk_tiling(vec: int | None = None, wx: int | None = None, by: int | None = None,
                  zdepth: int | None = None, pf: int = 2, xcd: int = 8,
                  dtype: str = "f64") -> None:
    """Tile shape of the variable-coefficient kernels ("f64" or "f32");
    with no shape given, the automatic choice."""
    if vec is None and wx is None and by is None and zdepth is None:
        t = AUTO_TILING
    else:
        if None in (vec, wx, by, zdepth):
            raise ValueError("give vec, wx, by and zdepth, or none of them")
        t = dict(vec=vec, wx=wx, by=by, zdepth=zdepth, pf=pf, xcd=xcd)
    _check(load().hc_heat_vk_set_tiling(DTYPES[dtype], *(int(t[k]) for k in _TILE_KEYS)))


def get_vk_tiling(dtype: str = "f64") -> dict:
    v = [ctypes.c_int(0) for _ in range(6)]
    _check(load().hc_heat_vk_get_tiling(DTYPES[dtype], *[ctypes.byref(x) for x in v]))
    return dict(zip(_TILE_KEYS, (x.value for x in v)))


def vk_tiling_for(u, u_new, kappa, rhs) -> dict:
    """The tile shape heat_vk_step would sweep these tensors with."""
    v = [ctypes.c_int(0) for _ in range(6)]
    ptrs = [ctypes.c_void_p(t.data_ptr()) for t in (u, u_new, kappa, rhs)]
    _check(load().hc_heat_vk_tiling_for(_dtype_code(u), int(u.shape[-1]), *ptrs,
                                        *[ctypes.byref(x) for x in v]))
    return dict(zip(_TILE_KEYS, (x.value for x in v)))


def set_vk2_tiling(vec: int | None = None, wx: int | None = None, by: int | None = None,
                   zdepth: int | None = None, pf: int = 2, xcd: int = 8,
                   dtype: str = "f64") -> None:
    """Tile shape of the two-step variable-coefficient kernels; with no
    shape given, the automatic choice."""
    if vec is None and wx is None and by is None and zdepth is None:
        t = AUTO_TILING
    else:
        if None in (vec, wx, by, zdepth):
            raise ValueError("give vec, wx, by and zdepth, or none of them")
        t = dict(vec=vec, wx=wx, by=by, zdepth=zdepth, pf=pf, xcd=xcd)
    _check(load().hc_heat_vk2_set_tiling(DTYPES[dtype], *(int(t[k]) for k in _TILE_KEYS)))


def get_vk2_tiling(dtype: str = "f64") -> dict:
    v = [ctypes.c_int(0) for _ in range(6)]
    _check(load().hc_heat_vk2_get_tiling(DTYPES[dtype], *[ctypes.byref(x) for x in v]))
    return dict(zip(_TILE_KEYS, (x.value for x in v)))


def set_vk2_zrun(planes: int = 0, dtype: str = "f64") -> None:
    """Output planes per block of the two-step variable-coefficient sweep
    (0: automatic)."""
    _check(load().hc_heat_vk2_set_zrun(DTYPES[dtype], int(planes)))


def get_vk2_zrun(dtype: str = "f64") -> int:
    return _check(load().hc_heat_vk2_get_zrun(DTYPES[dtype]))


def vk2_tiling_for(u, u_new, kappa, rhs) -> dict:
    """The tile shape a two-step variable-coefficient sweep of these tensors
    would run with."""
    v = [ctypes.c_int(0) for _ in range(6)]
    ptrs = [ctypes.c_void_p(t.data_ptr()) for t in (u, u_new, kappa, rhs)]
    _check(load().hc_heat_vk2_tiling_for(_dtype_code(u), int(u.shape[-1]), *ptrs,
                                         *[ctypes.byref(x) for x in v]))
    return dict(zip(_TILE_KEYS, (x.value for x in v)))


DEFAULT_CG_TILING = dict(vec=2, wx=1, by=4, zdepth=16, xcd=8)


def set_cg_tiling(vec: int = 2, wx: int = 1, by: int = 4, zdepth: int = 16, xcd: int = 8) -> None:
    """Tile shape of the CG kernels and of lap7_apply."""
    _check(load().hc_cg_set_tiling(int(vec), int(wx), int(by), int(zdepth), int(xcd)))


def get_cg_tiling() -> dict:
    v = [ctypes.c_int(0) for _ in range(5)]
    load().hc_cg_get_tiling(*[ctypes.byref(x) for x in v])
    return dict(zip(("vec", "wx", "by", "zdepth", "xcd"), (x.value for x in v)))


DEFAULT_CG_IR_TILING = dict(vec=4, wx=1, by=8, zdepth=32, xcd=8)


def set_cg_ir_tiling(vec: int = 4, wx: int = 1, by: int = 8, zdepth: int = 32,
                     xcd: int = 8) -> None:
    """Tile shape of the binary32 inner CG kernels and of lap7_apply_f32."""
    _check(load().hc_cg_ir_set_tiling(int(vec), int(wx), int(by), int(zdepth), int(xcd)))


def get_cg_ir_tiling() -> dict:
    v = [ctypes.c_int(0) for _ in range(5)]
    load().hc_cg_ir_get_tiling(*[ctypes.byref(x) for x in v])
    return dict(zip(("vec", "wx", "by", "zdepth", "xcd"), (x.value for x in v)))


def prof_enable(on: bool = True, every: int = 1) -> None:
    """Time every `every`-th launch of each kernel kind (off: on=False)."""
    _check(load().hc_prof_enable(int(every) if on else 0))


def prof_read(kind: str):
    """(total_ms, launches, algorithmic_bytes) for one kernel kind."""
    ms = ctypes.c_double(0.0)
    n = ctypes.c_longlong(0)
    b = ctypes.c_double(0.0)
    _check(load().hc_prof_read(KERNELS[kind], ctypes.byref(ms), ctypes.byref(n), ctypes.byref(b)))
    return ms.value, n.value, b.value


class Batch:
    """Many independent heat problems advanced together (hc_batch_*).

    ``dims``: sequence of (nx, ny, nz) storage edges; ``r``: one coefficient
    per problem; ``dtype``: "f64", "f32" or "bf16".  States live in packed
    buffers of ``total`` elements (``empty()`` allocates one, ``views(buf)``
    gives each problem's (nz, ny, nx) view, ``pack`` fills one).
    """

    _TORCH = {"f64": "float64", "f32": "float32", "bf16": "bfloat16"}

    def __init__(self, dims, r, dtype: str = "f32"):
        import numpy as np
        dims = np.ascontiguousarray(np.asarray(dims, dtype=np.int32).reshape(-1, 3))
        r = np.ascontiguousarray(np.asarray(r, dtype=np.float64).ravel())
        if len(r) != len(dims):
            raise ValueError("one r per problem")
        self.dtype = dtype
        self.dims = [tuple(int(v) for v in d) for d in dims]
        self.count = len(self.dims)
        self._h = ctypes.c_void_p(None)
        _check(load().hc_batch_create(self.count, dims.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                                      r.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                      DTYPES[dtype], ctypes.byref(self._h)))
        offs = (ctypes.c_longlong * self.count)()
        pitches = (ctypes.c_int * self.count)()
        total = ctypes.c_longlong(0)
        step_bytes = ctypes.c_double(0.0)
        _check(load().hc_batch_layout(self._h, offs, pitches, ctypes.byref(total),
                                      ctypes.byref(step_bytes)))
        self.offsets = list(offs)
        self.pitches = list(pitches)
        self.total = total.value
        self.step_bytes = step_bytes.value

    def close(self):
        if self._h:
            load().hc_batch_destroy(self._h)
            self._h = ctypes.c_void_p(None)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def empty(self, device="cuda"):
        import torch
        return torch.empty(self.total, dtype=getattr(torch, self._TORCH[self.dtype]), device=device)

    def views(self, buf):
        """Each problem's (nz, ny, nx) view of a packed buffer (rows
        ``pitch`` elements apart, so the views are strided)."""
        out = []
        for (nx, ny, nz), off, pitch in zip(self.dims, self.offsets, self.pitches):
            out.append(buf[off:off + pitch * ny * nz].view(nz, ny, pitch)[:, :, :nx])
        return out

    def step(self, u, u_new, steps: int, graph: bool = True, stream=None) -> None:
        for t in (u, u_new):
            if not t.is_cuda or not t.is_contiguous() or t.numel() < self.total:
                raise ValueError("expected contiguous CUDA buffers of %d elements" % self.total)
        _check(load().hc_batch_step(self._h, ctypes.c_void_p(u.data_ptr()),
                                    ctypes.c_void_p(u_new.data_ptr()), int(steps), int(bool(graph)),
                                    _stream_handle(u, stream)))

    _KEYS = ("vec", "threads", "zdepth", "pf", "xcd", "width_class", "grid", "item_depth")

    def set_tiling(self, vec, threads, zdepth=16, pf=2, xcd=8, width_class=-1, grid=0,
                   item_depth=0) -> None:
        _check(load().hc_batch_set_tiling(self._h, int(vec), int(threads), int(zdepth), int(pf),
                                          int(xcd), int(width_class), int(grid), int(item_depth)))

    def classes(self) -> list:
        """The tile width class (rows of 8 << c lanes) of every problem."""
        out = (ctypes.c_int * self.count)()
        _check(load().hc_batch_classes(self._h, out))
        return list(out)

    def get_tiling(self) -> dict:
        v = [ctypes.c_int(0) for _ in range(8)]
        _check(load().hc_batch_get_tiling(self._h, *[ctypes.byref(x) for x in v]))
        return dict(zip(self._KEYS, (x.value for x in v)))

    def steps_per_pass(self) -> int:
        """Steps one launch of this batch's shape advances (1 or 2)."""
        return _check(load().hc_batch_steps_per_pass(self._h))

    def autotune(self, u, trial_steps: int = 20, stream=None) -> float:
        """Time every candidate shape on copies of u, the four fastest again
        over twice the steps; keep the fastest of those.  Returns its
        milliseconds per step."""
        best = ctypes.c_double(0.0)
        _check(load().hc_batch_autotune(self._h, ctypes.c_void_p(u.data_ptr()), int(trial_steps),
                                        _stream_handle(u, stream), ctypes.byref(best)))
        return best.value

    def tune_results(self) -> list:
        lib = load()
        n = lib.hc_batch_tune_result(self._h, -1, None, None)
        out = []
        for i in range(max(n, 0)):
            sh = (ctypes.c_int * 8)()
            ms = ctypes.c_double(0.0)
            _check(lib.hc_batch_tune_result(self._h, i, sh, ctypes.byref(ms)))
            out.append((dict(zip(self._KEYS, list(sh))), ms.value))
        return out
