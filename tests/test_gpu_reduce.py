"""Parity of the reduction(+) kernels (section 2.3; SRAD paragraph of 4.2)
with the CPU oracle, through the C ABI."""
import numpy as np
import pytest

import oracle
import synth
from _util import SEED

pytestmark = pytest.mark.gpu

KINDS = ["fast", "plain"]


@pytest.fixture(scope="module")
def ax():
    import paper_1412_1127_amd as ax
    ax.acc_init(0, 0)
    yield ax
    ax.acc_shutdown()


def _flags(ax, kind):
    return ax.ACC_REDUCE_PLAIN if kind == "plain" else ax.ACC_REDUCE_FAST


def _reduce(ax, x, init, kind, offset=0):
    import torch
    dt = ax.ACC_FLOAT32 if x.dtype == np.float32 else ax.ACC_INT32
    buf = torch.zeros(x.size + offset + 1, dtype=torch.float32 if dt == ax.ACC_FLOAT32 else torch.int32,
                      device="cuda")
    buf[offset:offset + x.size] = torch.from_numpy(x).cuda()
    res = torch.zeros(1, dtype=buf.dtype, device="cuda")
    print("reduce dtype=%s n=%d offset=%d kind=%s" % (x.dtype, x.size, offset, kind), flush=True)
    ax.accx_reduce_sum_dev(dt, buf.data_ptr() + 4 * offset, x.size, init, res, _flags(ax, kind))
    torch.cuda.synchronize()
    return res.cpu().numpy()[0]


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("n", [0, 1, 3, 4, 5, 255, 256, 257, 1000, 5792])
def test_closed_form_exact(ax, kind, n):
    # x_k = k for k = 1..n: every partial sum is an integer below 2^24, exact in any order.
    x = np.arange(1, n + 1, dtype=np.float32)
    assert _reduce(ax, x, 0.0, kind) == np.float32(n * (n + 1) // 2)
    xi = np.arange(1, n + 1, dtype=np.int32)
    assert _reduce(ax, xi, 0, kind) == oracle.sum_i32(xi)


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("offset", [0, 1, 2, 3])
@pytest.mark.parametrize("n", [7, 1 << 16, (1 << 20) + 3])
def test_uniform_parity_misaligned(ax, kind, offset, n):
    x = synth.uniform01_f32(n, SEED, synth.STREAM_X)
    ref = oracle.sum_f32(x, 1.5)  # exact: values are multiples of 2^-24
    got = float(_reduce(ax, x, 1.5, kind, offset))
    assert abs(got - ref) / abs(ref) <= 1e-5
    xi = synth.full_range_i32((n,), SEED, synth.STREAM_X)
    assert _reduce(ax, xi, -5, kind, offset) == oracle.sum_i32(xi, -5)


@pytest.mark.parametrize("kind", KINDS)
def test_empty_returns_init(ax, kind):
    assert _reduce(ax, np.zeros(0, np.float32), 2.5, kind) == np.float32(2.5)
    assert _reduce(ax, np.zeros(0, np.int32), -9, kind) == -9


def test_deterministic_and_repeatable(ax):
    x = synth.uniform_pm1_f32(((1 << 22) + 5,), SEED, 17)
    r = [_reduce(ax, x, 0.0, "fast") for _ in range(3)]
    assert r[0] == r[1] == r[2]


def test_full_size(ax):
    # 2^28 uniform[0,1) floats: the float64 serial oracle is the exact sum.
    n = 1 << 28
    x = synth.uniform01_f32(n, SEED, synth.STREAM_X)
    ref = oracle.sum_f32(x)
    for kind in KINDS:
        got = float(_reduce(ax, x, 0.0, kind))
        assert abs(got - ref) / ref <= 1e-5, (kind, got, ref)
