"""Parity of the reduction clause with the operators +, max, min and logical
or, over float32 / int32 / float64 / int64, with one or several variables
per pass (the SRAD loop's sum and sum of squares), with the CPU oracle,
through the C ABI."""
import numpy as np
import pytest

import oracle
import synth
from _util import SEED

pytestmark = pytest.mark.gpu

DTYPES = {"f32": np.float32, "i32": np.int32, "f64": np.float64, "i64": np.int64}
SIZES = [1, 3, 1000, 65537, (1 << 20) + 3]
REL = {"f32": 1e-5, "f64": 1e-12}


@pytest.fixture(scope="module")
def ax():
    import paper_1412_1127_amd as ax
    ax.acc_init(0, 0)
    yield ax
    ax.acc_shutdown()


def _code(ax, name):
    return {"f32": ax.ACC_FLOAT32, "i32": ax.ACC_INT32, "f64": ax.ACC_FLOAT64, "i64": ax.ACC_INT64}[name]


def _op(ax, op):
    return {"sum": ax.ACC_RED_SUM, "max": ax.ACC_RED_MAX, "min": ax.ACC_RED_MIN, "or": ax.ACC_RED_OR}[op]


def _data(dt, n, stream, kind="mixed"):
    if dt == "f32":
        return synth.uniform01_f32(n, SEED, stream) if kind == "pos" else synth.uniform_pm1_f32((n,), SEED, stream)
    if dt == "f64":
        x = synth.uniform_pm1_f64(n, SEED, stream)
        return np.abs(x) if kind == "pos" else x
    if dt == "i32":
        return synth.full_range_i32((n,), SEED, stream)
    return synth.full_range_i64(n, SEED, stream)


def _run(ax, dt, x, vars_, init, offset=0):
    """Reduce x (placed `offset` elements into a device buffer) on the GPU."""
    import torch
    n = x.size
    buf = np.zeros(n + offset + 1, dtype=x.dtype)
    buf[offset:offset + n] = x
    dbuf = torch.from_numpy(buf).cuda()
    dx = dbuf[offset:offset + n]
    res = torch.full((len(vars_),), 77, dtype=dbuf.dtype, device="cuda")
    print("reduce dtype=%s n=%d vars=%s offset=%d" % (dt, n, vars_, offset), flush=True)
    ax.accx_reduce_dev(_code(ax, dt), dx, n, [(_op(ax, o), s) for o, s in vars_], init, res)
    torch.cuda.synchronize()
    return res.cpu().numpy()


def _check(dt, got, want, op):
    if dt in REL and op == "sum":
        assert abs(float(got) - want) <= REL[dt] * max(abs(want), 1e-300), (got, want)
    elif dt in REL:
        assert float(got) == want or (np.isnan(got) and np.isnan(want)), (got, want)
    else:
        assert int(got) == want, (got, want)


@pytest.mark.parametrize("dt", list(DTYPES))
@pytest.mark.parametrize("op", ["sum", "max", "min"])
@pytest.mark.parametrize("square", [False, True])
@pytest.mark.parametrize("n", SIZES)
def test_single_variable(ax, dt, op, square, n):
    x = _data(dt, n, 300 + n % 97, "pos" if op == "sum" else "mixed")
    init = 3 if op == "sum" else oracle.identity(op, DTYPES[dt])
    got = _run(ax, dt, x, [(op, square)], [init])[0]
    _check(dt, got, oracle.reduce(x, op, init=init, square=square), op)


@pytest.mark.parametrize("dt", list(DTYPES))
@pytest.mark.parametrize("offset", [1, 2, 3])
def test_unaligned_start(ax, dt, offset):
    n = 100_003
    x = _data(dt, n, 320 + offset, "pos")
    vars_ = [("sum", False), ("max", False), ("min", True)]
    got = _run(ax, dt, x, vars_, [1, -5, 10 ** 6], offset=offset)
    for g, (op, sq), init in zip(got, vars_, [1, -5, 10 ** 6]):
        _check(dt, g, oracle.reduce(x, op, init=init, square=sq), op)


@pytest.mark.parametrize("dt", ["f32", "f64"])
def test_srad_sum_and_sum_of_squares(ax, dt):
    # the SRAD statistics loop: sum and sum of squares of one image, one pass
    n = 2048 * 2048
    x = _data(dt, n, 330, "pos")
    got = _run(ax, dt, x, [("sum", False), ("sum", True)], [0, 0])
    _check(dt, got[0], oracle.reduce(x, "sum"), "sum")
    _check(dt, got[1], oracle.reduce(x, "sum", square=True), "sum")


@pytest.mark.parametrize("dt", list(DTYPES))
def test_four_variables(ax, dt):
    n = 300_001
    x = _data(dt, n, 340, "pos")
    vars_ = [("max", True), ("sum", False), ("min", False), ("sum", True)]
    inits = [0, 7, 100, -2]
    got = _run(ax, dt, x, vars_, inits)
    for g, (op, sq), init in zip(got, vars_, inits):
        _check(dt, g, oracle.reduce(x, op, init=init, square=sq), op)


@pytest.mark.parametrize("dt", list(DTYPES))
def test_logical_or_flag(ax, dt):
    n = 1 << 20
    z = np.zeros(n, DTYPES[dt])
    assert _run(ax, dt, z, [("or", False)], [0])[0] == 0
    assert _run(ax, dt, z, [("or", False)], [9])[0] == 1
    for pos in (0, 5, n // 2, n - 1):
        z2 = z.copy()
        z2[pos] = 1
        assert _run(ax, dt, z2, [("or", False)], [0])[0] == 1, pos
    f = synth.sparse_flags_i32(n, 3e-6, SEED, 350).astype(DTYPES[dt])
    assert _run(ax, dt, f, [("or", False)], [0])[0] == oracle.reduce(f, "or")


def test_logical_or_special_values(ax):
    assert _run(ax, "i64", np.array([0, 0, 1 << 40, 0], np.int64), [("or", False)], [0])[0] == 1
    assert _run(ax, "f32", np.array([-0.0, 0.0, -0.0], np.float32), [("or", False)], [0])[0] == 0
    assert _run(ax, "f64", np.array([0.0, np.nan], np.float64), [("or", False)], [0])[0] == 1


@pytest.mark.parametrize("dt", ["f32", "f64"])
def test_max_min_ignore_nan(ax, dt):
    x = _data(dt, 50_000, 360)
    x[[3, 777, 49_999]] = np.nan
    got = _run(ax, dt, x, [("max", False), ("min", False)], [-np.inf, np.inf])
    assert float(got[0]) == oracle.reduce(x, "max") and float(got[1]) == oracle.reduce(x, "min")


@pytest.mark.parametrize("dt", ["f32", "f64"])
def test_bitwise_repeatable(ax, dt):
    x = _data(dt, 3_000_001, 370, "pos")
    a = _run(ax, dt, x, [("sum", False), ("sum", True)], [0, 0])
    b = _run(ax, dt, x, [("sum", False), ("sum", True)], [0, 0])
    assert a.tobytes() == b.tobytes()


@pytest.mark.parametrize("dt", list(DTYPES))
def test_empty_input_gives_init(ax, dt):
    got = _run(ax, dt, np.zeros(0, DTYPES[dt]), [("sum", False), ("max", False)], [4, 9])
    assert got[0] == 4 and got[1] == 9
    assert _run(ax, dt, np.zeros(0, DTYPES[dt]), [("or", False)], [2])[0] == 1


@pytest.mark.parametrize("dt", ["f64", "i64"])
def test_sum_entry_takes_8_byte_types(ax, dt):
    import torch
    x = _data(dt, 123_457, 380, "pos")
    dx = torch.from_numpy(x).cuda()
    r = torch.zeros(1, dtype=dx.dtype, device="cuda")
    ax.accx_reduce_sum_dev(_code(ax, dt), dx, x.size, 5, r)
    torch.cuda.synchronize()
    _check(dt, r.cpu().numpy()[0], oracle.reduce(x, "sum", init=5), "sum")


def test_region_reduce_async_several_variables(ax):
    n = 200_000
    x = synth.uniform01_f32(n, SEED, 390)
    y = synth.full_range_i64(n, SEED, 391)
    fl = synth.sparse_flags_i32(n, 1e-5, SEED, 392)
    r = ax.acc_data_begin([ax.clause(ax.ACC_COPYIN, ax.ACC_FLOAT32, x), ax.clause(ax.ACC_COPYIN, ax.ACC_INT64, y),
                           ax.clause(ax.ACC_COPYIN, ax.ACC_INT32, fl)])
    sx = np.array([0.5, 0.0], np.float32)
    sy = np.array([oracle.identity("max", np.int64), 11], np.int64)
    sf = np.array([0], np.int32)
    ax.acc_reduce(r, ax.ACC_FLOAT32, x, n, [(ax.ACC_RED_SUM, 0), (ax.ACC_RED_SUM, 1)], sx, ax.ACC_ASYNC)
    ax.acc_reduce(r, ax.ACC_INT64, y, n, [(ax.ACC_RED_MAX, 0), (ax.ACC_RED_SUM, 0)], sy, ax.ACC_ASYNC)
    ax.acc_reduce(r, ax.ACC_INT32, fl, n, [(ax.ACC_RED_OR, 0)], sf, ax.ACC_ASYNC)
    ax.acc_data_end(r)
    assert abs(float(sx[0]) - oracle.reduce(x, "sum", init=0.5)) <= 1e-5 * oracle.reduce(x, "sum", init=0.5)
    assert abs(float(sx[1]) - oracle.reduce(x, "sum", square=True)) <= 1e-5 * oracle.reduce(x, "sum", square=True)
    assert int(sy[0]) == oracle.reduce(y, "max") and int(sy[1]) == oracle.reduce(y, "sum", init=11)
    assert int(sf[0]) == oracle.reduce(fl, "or")


def test_invalid_variable_sets(ax):
    import torch
    dx = torch.zeros(16, device="cuda")
    r = torch.zeros(4, device="cuda")
    for vars_ in ([], [(ax.ACC_RED_OR, 1)], [(ax.ACC_RED_OR, 0), (ax.ACC_RED_SUM, 0)], [(7, 0)],
                  [(ax.ACC_RED_SUM, 0)] * 5):
        with pytest.raises(ax.AccxError) as e:
            ax.accx_reduce_dev(ax.ACC_FLOAT32, dx, 16, vars_, [0] * max(1, len(vars_)), r)
        assert e.value.status == ax.ACC_ERR_INVALID_ARG
    with pytest.raises(ax.AccxError):
        ax.accx_reduce_dev(ax.ACC_FLOAT32, dx, 16, [(ax.ACC_RED_MAX, 0)], [0], r, ax.ACC_REDUCE_PLAIN)
