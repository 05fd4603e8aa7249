"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every entry point that include/accx.h declares, validates arguments, and
refuses to compute without a device instead of falling back to the host."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "accx.h")


def _declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"ACCX_API\s+[\w\s\*]+?\b(acc[x]?_\w+)\s*\(", txt)))


def test_header_declares_entry_points():
    names = _declared()
    for must in ("acc_init", "acc_data_begin", "acc_data_end", "acc_loopnest_matmul", "acc_reduce_sum"):
        assert must in names


def test_library_exports_every_declared_symbol():
    import paper_1412_1127_amd as ax
    lib = ctypes.CDLL(ax.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    # the binding wraps every declared entry point under the same name
    assert sorted(ax.EXPORTED) == _declared()


def test_status_strings():
    import paper_1412_1127_amd as ax
    assert ax.status_string(ax.ACC_OK) == "ACC_OK"
    assert ax.status_string(ax.ACC_ERR_NOT_PRESENT) == "ACC_ERR_NOT_PRESENT"
    assert "gfx950" in ax.version()


def _no_gpu():
    import torch
    return not torch.cuda.is_available()


@pytest.mark.skipif(not _no_gpu(), reason="checks the no-device path")
def test_no_device_no_fallback():
    import paper_1412_1127_amd as ax
    with pytest.raises(ax.AccxError) as e:
        ax.acc_init(0, 0)
    assert e.value.status == ax.ACC_ERR_NO_DEVICE
    a = np.zeros(4, np.float32)
    with pytest.raises(ax.AccxError) as e:
        ax.acc_data_begin([ax.clause(ax.ACC_COPY, ax.ACC_FLOAT32, a)])
    assert e.value.status == ax.ACC_ERR_NO_DEVICE
    with pytest.raises(ax.AccxError) as e:
        ax.accx_matmul_dev(ax.ACC_FLOAT32, 256, 512, 768, 4, ax.ACC_KERNEL_PLAIN)
    assert e.value.status == ax.ACC_ERR_NO_DEVICE
    with pytest.raises(ax.AccxError) as e:
        ax.accx_reduce_sum_dev(ax.ACC_FLOAT32, 256, 4, 0.0, 512)
    assert e.value.status == ax.ACC_ERR_NO_DEVICE


def test_argument_validation_without_device():
    import paper_1412_1127_amd as ax
    for bad in [(ax.ACC_FLOAT32, 0, 0), (ax.ACC_FLOAT32, 65537, 0), (7, 16, 0),
                (ax.ACC_FLOAT32, 16, 0x4), (ax.ACC_FLOAT32, 16, 0x50), (ax.ACC_INT32, 16, ax.ACC_LIMBS(5))]:
        with pytest.raises(ax.AccxError) as e:
            ax.accx_matmul_workspace_size(*bad)
        assert e.value.status == ax.ACC_ERR_INVALID_ARG, bad
    assert ax.accx_matmul_workspace_size(ax.ACC_FLOAT32, 64, ax.ACC_KERNEL_PLAIN) == 0
    with pytest.raises(ax.AccxError) as e:
        ax.accx_reduce_workspace_size(ax.ACC_FLOAT32, -1, 0)
    assert e.value.status == ax.ACC_ERR_INVALID_ARG
    assert ax.accx_reduce_workspace_size(ax.ACC_FLOAT32, 1 << 20, 0) > 256
    assert ax.accx_reduce_workspace_size(ax.ACC_INT32, 1000, ax.ACC_REDUCE_PLAIN) == 4 * 4


def test_set_allocator_needs_both_or_neither():
    import ctypes

    import paper_1412_1127_amd as ax
    fa = ax._ALLOC_FN(lambda n, c: 0)
    assert ax._lib.accx_set_allocator(ctypes.cast(fa, ctypes.c_void_p), None, None) == ax.ACC_ERR_INVALID_ARG
    ax.accx_set_allocator(None, None)                  # back to hipMalloc: always valid


def test_gemm_shape_validation_without_device():
    import paper_1412_1127_amd as ax
    f6 = ax.ACC_KERNEL_TILED | ax.ACC_PREC_FULL6
    for bad in [(-1, 4, 4), (4, -1, 4), (4, 4, -1), (131073, 4, 4), (4, 131073, 4), (4, 4, 65537)]:
        with pytest.raises(ax.AccxError) as e:
            ax.accx_gemm_workspace_size(ax.ACC_FLOAT32, *bad, f6)
        assert e.value.status == ax.ACC_ERR_INVALID_ARG, bad
    # the square shape needs what the square entry needs, for every flag set
    for dt, fl in [(ax.ACC_FLOAT32, f6), (ax.ACC_FLOAT32, ax.ACC_KERNEL_TILED),
                   (ax.ACC_INT32, ax.ACC_KERNEL_TILED), (ax.ACC_INT32, ax.ACC_KERNEL_TILED | ax.ACC_LIMBS(2))]:
        for n in (1, 33, 1000):
            assert ax.accx_gemm_workspace_size(dt, n, n, n, fl) == ax.accx_matmul_workspace_size(dt, n, fl)
    # two packed operands: ceil(m/32) and ceil(n/32) row blocks of ceil(2k/64) units of 3 x 2 KB planes
    m, n, k = 70, 300, 129
    units = (-(-m // 32) + -(-n // 32)) * -(-2 * k // 64)
    assert ax.accx_gemm_workspace_size(ax.ACC_FLOAT32, m, n, k, f6) == units * 3 * 2048
    assert ax.accx_gemm_workspace_size(ax.ACC_FLOAT32, 0, n, k, f6) == 0
    assert ax.accx_gemm_workspace_size(ax.ACC_FLOAT32, m, n, k, ax.ACC_KERNEL_PLAIN) == 0
    # the workspace does not grow with k = 0 beyond the probe records
    off, cnt = ax.accx_gemm_probe_layout(m, n, k, ax.ACC_KERNEL_TILED)
    assert off >= units * 3 * 2048 and cnt >= 1


@pytest.mark.skipif(not _no_gpu(), reason="checks the no-device path")
def test_gemm_dev_no_device_no_fallback():
    import paper_1412_1127_amd as ax
    with pytest.raises(ax.AccxError) as e:
        ax.accx_gemm_dev(ax.ACC_FLOAT32, 4, 4, 4, 256, 4, 512, 4, 768, 4, ax.ACC_KERNEL_PLAIN)
    assert e.value.status == ax.ACC_ERR_NO_DEVICE


def test_reduce_variables_validation_without_device():
    import paper_1412_1127_amd as ax
    S, MX, OR = ax.ACC_RED_SUM, ax.ACC_RED_MAX, ax.ACC_RED_OR
    # the float32 / int32 single sum keeps the dedicated kernels' workspace
    for dt in (ax.ACC_FLOAT32, ax.ACC_INT32):
        assert ax.accx_reduce_vars_workspace_size(dt, 1 << 20, [(S, 0)]) == ax.accx_reduce_workspace_size(dt, 1 << 20)
    general = ax.accx_reduce_vars_workspace_size(ax.ACC_FLOAT64, 1 << 20, [(S, 0)])
    assert general >= 8 * 4 * 4096  # four 8-byte partials per workgroup
    assert ax.accx_reduce_vars_workspace_size(ax.ACC_FLOAT32, 10, [(S, 0), (S, 1)]) == general
    for dt, vars_, fl in [(ax.ACC_FLOAT32, [], 0), (ax.ACC_FLOAT32, [(S, 0)] * 5, 0), (ax.ACC_INT32, [(OR, 1)], 0),
                          (ax.ACC_INT32, [(OR, 0), (S, 0)], 0), (ax.ACC_FLOAT32, [(9, 0)], 0),
                          (ax.ACC_FLOAT32, [(S, 2)], 0), (ax.ACC_FLOAT32, [(MX, 0)], ax.ACC_REDUCE_PLAIN),
                          (ax.ACC_FLOAT64, [(S, 0)], ax.ACC_REDUCE_PLAIN), (7, [(S, 0)], 0)]:
        with pytest.raises(ax.AccxError) as e:
            ax.accx_reduce_vars_workspace_size(dt, 10, vars_, fl)
        assert e.value.status == ax.ACC_ERR_INVALID_ARG, (dt, vars_, fl)
    # the matmul still takes the 4-byte types only
    with pytest.raises(ax.AccxError):
        ax.accx_matmul_workspace_size(ax.ACC_FLOAT64, 16, 0)


@pytest.mark.skipif(not _no_gpu(), reason="checks the no-device path")
def test_reduce_dev_no_device_no_fallback():
    import paper_1412_1127_amd as ax
    with pytest.raises(ax.AccxError) as e:
        ax.accx_reduce_dev(ax.ACC_FLOAT64, 256, 4, [(ax.ACC_RED_MAX, 0)], [0.0], 512)
    assert e.value.status == ax.ACC_ERR_NO_DEVICE
