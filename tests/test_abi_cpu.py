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
                (ax.ACC_FLOAT32, 16, 0x4), (ax.ACC_FLOAT32, 16, 0x30), (ax.ACC_INT32, 16, ax.ACC_LIMBS(5))]:
        with pytest.raises(ax.AccxError) as e:
            ax.accx_matmul_workspace_size(*bad)
        assert e.value.status == ax.ACC_ERR_INVALID_ARG, bad
    assert ax.accx_matmul_workspace_size(ax.ACC_FLOAT32, 64, ax.ACC_KERNEL_PLAIN) == 0
    with pytest.raises(ax.AccxError) as e:
        ax.accx_reduce_workspace_size(ax.ACC_FLOAT32, -1, 0)
    assert e.value.status == ax.ACC_ERR_INVALID_ARG
    assert ax.accx_reduce_workspace_size(ax.ACC_FLOAT32, 1 << 20, 0) > 256
    assert ax.accx_reduce_workspace_size(ax.ACC_INT32, 1000, ax.ACC_REDUCE_PLAIN) == 4 * 4
