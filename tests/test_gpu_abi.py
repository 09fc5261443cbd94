"""The C ABI on the GPU: buffer checks against the runtime, the copy probe,
kernel timing counters."""
import ctypes

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

HC_EINVAL = -1


def note(msg):
    print("[case] " + msg, flush=True)


def test_host_memory_is_rejected(gpu):
    note("host pointer -> EINVAL")
    a = np.zeros((6, 6, 6))
    b = np.zeros((6, 6, 6))
    rc = gpu.abi().heat_step(ctypes.c_void_p(a.ctypes.data), ctypes.c_void_p(b.ctypes.data),
                             6, 6, 6, 0.1, 1)
    assert rc == HC_EINVAL
    assert "device" in gpu.abi().hc_last_error_message().decode()


def test_undersized_allocation_is_rejected(gpu):
    note("undersized hipMalloc -> EINVAL")
    hip = ctypes.CDLL("libamdhip64.so")
    p = ctypes.c_void_p()
    q = ctypes.c_void_p()
    assert hip.hipMalloc(ctypes.byref(p), ctypes.c_size_t(4096)) == 0
    assert hip.hipMalloc(ctypes.byref(q), ctypes.c_size_t(8 * 100 ** 3)) == 0
    try:
        # the runtime must report an allocation far smaller than 100^3 doubles
        base = ctypes.c_void_p()
        size = ctypes.c_size_t()
        assert hip.hipMemGetAddressRange(ctypes.byref(base), ctypes.byref(size), p) == 0
        assert size.value < 8 * 100 ** 3
        rc = gpu.abi().heat_step(p, q, 100, 100, 100, 0.1, 1)
        assert rc == HC_EINVAL
        assert "allocation" in gpu.abi().hc_last_error_message().decode()
    finally:
        hip.hipFree(p)
        hip.hipFree(q)


def test_copy_probe_copies_bitwise_and_is_timed(gpu):
    note("copy probe 64 MiB")
    src = torch.randn(8 * 1024 * 1024, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    gpu.prof_enable(True)
    gpu.copy_probe(src, dst)
    torch.cuda.synchronize()
    ms, n, nbytes = gpu.prof_read("copy")
    gpu.prof_enable(False)
    assert torch.equal(src, dst)
    assert n == 1 and ms > 0 and nbytes == 2 * src.numel() * 8


def test_heat_kernels_are_timed_per_role(one_step):
    gpu = one_step
    note("prof counters on a split run, one step per pass")
    u = torch.rand(40, 36, 70, dtype=torch.float64, device="cuda")
    un = torch.empty_like(u)
    gpu.prof_enable(True)
    gpu.heat_step(u, un, 0.1, 4)
    torch.cuda.synchronize()
    ms_i, n_i, b_i = gpu.prof_read("heat_interior")
    ms_b, n_b, b_b = gpu.prof_read("heat_boundary")
    gpu.prof_enable(False)
    assert n_i == 4 and n_b == 4 and ms_i > 0 and ms_b > 0
    # interior: reads planes 1..38, writes planes 2..37
    assert b_i == 4 * 8 * (38 * 36 * 70 + 36 * 34 * 68)


def test_two_step_kernels_are_timed_per_role(gpu):
    note("prof counters on a split run, two steps per pass")
    saved = gpu.get_time_block()
    gpu.set_time_block(2)
    try:
        u = torch.rand(40, 36, 70, dtype=torch.float64, device="cuda")
        un = torch.empty_like(u)
        gpu.prof_enable(True)
        gpu.heat_step(u, un, 0.1, 5)
        torch.cuda.synchronize()
        ms_i, n_i, b_i = gpu.prof_read("heat2_interior")
        ms_b, n_b, b_b = gpu.prof_read("heat2_boundary")
        n_1 = gpu.prof_read("heat_interior")[1]
        gpu.prof_enable(False)
    finally:
        gpu.set_time_block(saved)
    # 5 steps: two two-step passes and a last single step
    assert n_i == 2 and n_b == 2 and n_1 == 1 and ms_i > 0 and ms_b > 0
    # interior: output planes 3..36 read planes 1..38
    assert b_i == 2 * 8 * (38 * 36 * 70 + 34 * 34 * 68)
    # boundary: output planes {1, 2, 37, 38} read planes 0..4 and 35..39
    assert b_b == 2 * 8 * (10 * 36 * 70 + 4 * 34 * 68)
