"""The tiled kernel's prepass, bit-exact against the oracle: the bf16x3
split of float32 operands and the balanced base-256 digits of int32
operands, unpacked from the documented packed layout (include/accx.h)."""
import numpy as np
import pytest

import oracle
import synth
from _util import SEED

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ax():
    import paper_1412_1127_amd as ax
    ax.acc_init(0, 0)
    yield ax
    ax.acc_shutdown()


def _unpack(buf: np.ndarray, rows: int, k: int, elem_bytes: int, planes: int) -> np.ndarray:
    """Packed bytes -> array [planes, rows, k] of raw elements (uint16 or int8)."""
    nrb = -(-rows // 32)
    kb_elems = 64 // elem_bytes
    nkb = -(-k // kb_elems)
    u = buf[:nrb * nkb * planes * 2048].reshape(nrb, nkb, planes, 4, 32, 16)
    # -> [planes, rb, r, kb, c, 16 bytes]
    u = u.transpose(2, 0, 4, 1, 3, 5).reshape(planes, nrb * 32, nkb * 64)
    dt = np.uint16 if elem_bytes == 2 else np.int8
    full = np.ascontiguousarray(u).view(dt)
    return full[:, :rows, :k], full


def _pack(ax, x: np.ndarray, rows: int, k: int, transposed: bool, planes: int):
    import torch
    dt = ax.ACC_FLOAT32 if x.dtype == np.float32 else ax.ACC_INT32
    size = ax.accx_packed_size(dt, rows, k, planes)
    out = torch.full((size,), 0x5A, dtype=torch.uint8, device="cuda")
    dx = torch.from_numpy(x).cuda()
    print("pack dtype=%s rows=%d k=%d trans=%d planes=%d" % (x.dtype, rows, k, transposed, planes), flush=True)
    ax.accx_pack_dev(dt, dx, rows, k, transposed, planes, out, size)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("rows,k", [(1, 1), (31, 33), (64, 64), (100, 257), (256, 96)])
@pytest.mark.parametrize("transposed", [False, True])
def test_bf16x3_split_bit_exact(ax, rows, k, transposed):
    x = np.concatenate([synth.uniform_pm1_f32((rows * k,), SEED, 1)[: rows * k // 2],
                        synth.normal_rowscaled_f32(1, rows * k, SEED, 2).ravel()[rows * k // 2:]])
    x = x.reshape((k, rows) if transposed else (rows, k)).astype(np.float32)
    got, full = _unpack(_pack(ax, x, rows, k, transposed, 3), rows, k, 2, 3)
    src = np.ascontiguousarray(x.T) if transposed else x
    hi, mid, lo = oracle.split_bf16x3(src)
    assert np.array_equal(got[0], hi) and np.array_equal(got[1], mid) and np.array_equal(got[2], lo)
    # zero padding past rows and k
    pad = full.copy()
    pad[:, :rows, :k] = 0
    assert not pad.any()


@pytest.mark.parametrize("planes", [1, 2, 3, 4])
@pytest.mark.parametrize("rows,k", [(1, 1), (33, 65), (64, 128), (70, 200)])
@pytest.mark.parametrize("transposed", [False, True])
def test_int8_limbs_bit_exact(ax, planes, rows, k, transposed):
    x = synth.full_range_i32((k, rows) if transposed else (rows, k), SEED, 3)
    got, full = _unpack(_pack(ax, x, rows, k, transposed, planes), rows, k, 1, planes)
    src = np.ascontiguousarray(x.T) if transposed else x
    assert np.array_equal(got, oracle.limbs_i8(src, planes))
    pad = full.copy()
    pad[:, :rows, :k] = 0
    assert not pad.any()


def test_pack_argument_errors(ax):
    with pytest.raises(ax.AccxError):
        ax.accx_packed_size(ax.ACC_FLOAT32, 8, 8, 2)
    with pytest.raises(ax.AccxError):
        ax.accx_packed_size(ax.ACC_INT32, 8, 8, 5)
    import torch
    x = torch.zeros(64, dtype=torch.float32, device="cuda")
    out = torch.zeros(16, dtype=torch.uint8, device="cuda")
    with pytest.raises(ax.AccxError) as e:
        ax.accx_pack_dev(ax.ACC_FLOAT32, x, 8, 8, False, 3, out, 16)
    assert e.value.status == ax.ACC_ERR_INVALID_ARG
