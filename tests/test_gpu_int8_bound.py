"""The int32 path at the longest sequential loop it admits (k = 65536): the
loop nest of section 1.3 with Listing 1b's int operands, whose digit-pair
sums pass 2^31 there.

2139062144 = 0x7F7F7F80 has the balanced base-256 digits (-128, -128, -128,
-128) (plus a carry of 2^32, which vanishes modulo 2^32), so every digit
product is +2^14, the largest there is, and the four-pair shift group sums
4 * 2^14 * k: 2^31 at k = 32768, 2^32 at k = 65536.  The result must still
equal the oracle modulo 2^32 bit for bit."""
import numpy as np
import pytest

import oracle
import synth
from _util import SEED

pytestmark = pytest.mark.gpu

X = 2139062144


@pytest.fixture(scope="module")
def ax():
    import paper_1412_1127_amd as ax
    ax.acc_init(0, 0)
    yield ax
    ax.acc_shutdown()


def _gemm(ax, a, b, flags):
    import torch
    m, k = a.shape
    n = b.shape[1]
    da, db = torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()
    dc = torch.full((m, n), -7, dtype=torch.int32, device="cuda")
    print("int32 gemm %dx%dx%d flags=%#x" % (m, n, k, flags), flush=True)
    ax.accx_gemm_dev(ax.ACC_INT32, m, n, k, da, k, db, n, dc, n, flags)
    torch.cuda.synchronize()
    return dc.cpu().numpy()


def _wrap32(v: int) -> int:
    v &= 0xFFFFFFFF
    return v - (1 << 32) if v >= 1 << 31 else v


def test_digits_of_x_are_all_minus_128():
    d = oracle.limbs_i8(np.array([X], dtype=np.int32), 4)
    assert list(np.asarray(d).ravel()) == [-128, -128, -128, -128]


@pytest.mark.parametrize("k", [32768, 65536])
@pytest.mark.parametrize("sign", [1, -1])
@pytest.mark.parametrize("limbs", ["forced4", "decided"])
def test_largest_digit_sums(ax, k, sign, limbs):
    m = n = 64
    a = np.full((m, k), X, dtype=np.int32)
    b = np.full((k, n), sign * X, dtype=np.int32)
    flags = ax.ACC_KERNEL_TILED | (ax.ACC_LIMBS(4) if limbs == "forced4" else 0)
    c = _gemm(ax, a, b, flags)
    ref = oracle.gemm(a, b)
    assert np.all(ref == _wrap32(k * X * sign * X))      # closed form of the constant nest
    assert np.array_equal(c, ref)


def test_full_range_k65536(ax):
    m, n, k = 64, 96, 65536
    a = synth.full_range_i32((m, k), SEED, 61)
    b = synth.full_range_i32((k, n), SEED, 62)
    assert np.array_equal(_gemm(ax, a, b, ax.ACC_KERNEL_TILED), oracle.gemm(a, b))
