"""The reduction entry point that allocates nothing (accx_reduce_dev_noalloc):
its partials live in the library's static device scratch.  Through the C
ABI it must give bitwise the result of accx_reduce_dev (same kernels, same
workgroup count), on two calls in a row (the second smaller, so stale
partials of the first would show), match the CPU oracle, reject a need
beyond the scratch, and take no memory from the library's allocator."""
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


def _both(ax, dtype, x, vars_, init, flags=0):
    """(no-alloc result, workspace result) for x on the GPU."""
    import torch
    dx = torch.from_numpy(x).cuda()
    got = torch.full((len(vars_),), 77, dtype=dx.dtype, device="cuda")
    ref = torch.full((len(vars_),), 55, dtype=dx.dtype, device="cuda")
    print("noalloc reduce dtype=%d n=%d vars=%s flags=%d" % (dtype, x.size, vars_, flags), flush=True)
    ax.accx_reduce_dev_noalloc(dtype, dx, x.size, vars_, init, got, flags)
    ax.accx_reduce_dev(dtype, dx, x.size, vars_, init, ref, flags)
    torch.cuda.synchronize()
    return got.cpu().numpy(), ref.cpu().numpy()


def _rel(got, ref):
    return abs(float(got) - ref) / max(abs(ref), 1e-30)


@pytest.mark.parametrize("sizes", [((1 << 24) + 5, 1000), ((1 << 20) + 3, 3)])
def test_float32_sum_twice_smaller_second(ax, sizes):
    for k, n in enumerate(sizes):
        x = synth.uniform01_f32(n, SEED, 700 + k)
        got, ref = _both(ax, ax.ACC_FLOAT32, x, [(ax.ACC_RED_SUM, 0)], [0.25])
        assert got.tobytes() == ref.tobytes()
        assert _rel(got[0], oracle.sum_f32(x, 0.25)) <= 1e-5


def test_int32_sum_twice_smaller_second(ax):
    for k, n in enumerate([(1 << 22) + 7, 4097]):
        x = synth.full_range_i32((n,), SEED, 710 + k)
        got, ref = _both(ax, ax.ACC_INT32, x, [(ax.ACC_RED_SUM, 0)], [-5])
        assert got.tobytes() == ref.tobytes()
        assert int(got[0]) == oracle.sum_i32(x, -5)


def test_several_variables_twice_smaller_second(ax):
    # SRAD's sum and sum of squares, then max and min, over float64
    for k, (n, vars_) in enumerate([((1 << 21) + 1, [(ax.ACC_RED_SUM, 0), (ax.ACC_RED_SUM, 1)]),
                                    (777, [(ax.ACC_RED_MAX, 0), (ax.ACC_RED_MIN, 0)])]):
        x = synth.uniform_pm1_f64(n, SEED, 720 + k)
        init = [0.5, -0.5]
        got, ref = _both(ax, ax.ACC_FLOAT64, x, vars_, init)
        assert got.tobytes() == ref.tobytes()
        for v, (op, sq) in enumerate(vars_):
            want = oracle.reduce(x, {ax.ACC_RED_SUM: "sum", ax.ACC_RED_MAX: "max", ax.ACC_RED_MIN: "min"}[op],
                                 init[v], square=bool(sq))
            assert _rel(got[v], want) <= 1e-12


def test_plain_kernel_and_limit(ax):
    import torch
    for k, n in enumerate([(1 << 23), 300]):   # 2^23 = the largest plain n the scratch holds
        x = synth.uniform01_f32(n, SEED, 730 + k)
        got, ref = _both(ax, ax.ACC_FLOAT32, x, [(ax.ACC_RED_SUM, 0)], [0.0], ax.ACC_REDUCE_PLAIN)
        assert got.tobytes() == ref.tobytes()
        assert _rel(got[0], oracle.sum_f32(x, 0.0)) <= 1e-5
    dx = torch.zeros((1 << 23) + 1, dtype=torch.float32, device="cuda")
    res = torch.zeros(1, dtype=torch.float32, device="cuda")
    with pytest.raises(ax.AccxError) as ei:
        ax.accx_reduce_dev_noalloc(ax.ACC_FLOAT32, dx, dx.numel(), [(ax.ACC_RED_SUM, 0)], [0.0], res,
                                   ax.ACC_REDUCE_PLAIN)
    assert ei.value.status == ax.ACC_ERR_INVALID_ARG


def test_takes_nothing_from_the_allocator(ax):
    import torch
    talloc = ax.TorchAllocator().install()
    try:
        x = synth.uniform01_f32((1 << 20) + 9, SEED, 740)
        dx = torch.from_numpy(x).cuda()
        res = torch.zeros(1, dtype=torch.float32, device="cuda")
        for n in (x.size, 4096):
            ax.accx_reduce_dev_noalloc(ax.ACC_FLOAT32, dx, n, [(ax.ACC_RED_SUM, 0)], [0.0], res)
            torch.cuda.synchronize()
            assert _rel(res.cpu().numpy()[0], oracle.sum_f32(x[:n], 0.0)) <= 1e-5
        assert talloc.allocs == 0
    finally:
        ax.accx_set_allocator(None, None)
