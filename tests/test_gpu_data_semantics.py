"""Richer data semantics of the data directive (section 1.3's data clauses
and section 2.3's host-accelerator pointer exchange): present and
present_or_* clauses with reference-counted nesting, the update directive in
both directions, and page-locked host memory for transfers that overlap
kernels of another region, through the C ABI, against the oracle."""
import ctypes

import numpy as np
import pytest

import oracle
import synth
from _util import FP32_REL_FRO_TOL, SEED, rel_fro

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ax():
    import paper_1412_1127_amd as ax
    ax.acc_init(0, 0)
    yield ax
    ax.acc_shutdown()


def _cl(ax, kind, arr, start=0, n=None):
    dt = {np.dtype(np.float32): ax.ACC_FLOAT32, np.dtype(np.int32): ax.ACC_INT32,
          np.dtype(np.float64): ax.ACC_FLOAT64, np.dtype(np.int64): ax.ACC_INT64}[arr.dtype]
    return ax.clause(kind, dt, arr, start, n)


def _mats(n, stream):
    return (synth.uniform_pm1_f32((n, n), SEED, stream), synth.uniform_pm1_f32((n, n), SEED, stream + 1),
            np.zeros((n, n), np.float32))


@pytest.mark.parametrize("outer_ends_first", [False, True])
def test_present_nesting_copies_out_at_last_release(ax, outer_ends_first):
    n = 96
    a, b, c = _mats(n, 401)
    outer = ax.acc_data_begin([_cl(ax, ax.ACC_COPYIN, a), _cl(ax, ax.ACC_COPYIN, b), _cl(ax, ax.ACC_COPY, c)])
    inner = ax.acc_data_begin([_cl(ax, ax.ACC_PRESENT, a), _cl(ax, ax.ACC_PRESENT, b), _cl(ax, ax.ACC_PRESENT, c)])
    ax.acc_loopnest_matmul(inner, ax.ACC_FLOAT32, a, b, c, n, ax.ACC_KERNEL_PLAIN)
    ax.acc_wait(inner)
    first, second = (outer, inner) if outer_ends_first else (inner, outer)
    ax.acc_data_end(first)
    assert np.all(c == 0), "copied out while another region still holds the mapping"
    assert ax.acc_is_present(c)
    ax.acc_data_end(second)
    assert not ax.acc_is_present(c) and not ax.acc_is_present(a)
    assert rel_fro(c, oracle.matmul_f32(a, b)) <= FP32_REL_FRO_TOL


def test_present_errors(ax):
    x = np.zeros(64, np.float32)
    with pytest.raises(ax.AccxError) as e:
        ax.acc_data_begin([_cl(ax, ax.ACC_PRESENT, x)])
    assert e.value.status == ax.ACC_ERR_NOT_PRESENT
    r = ax.acc_data_begin([_cl(ax, ax.ACC_COPYIN, x, 0, 32)])
    try:
        with pytest.raises(ax.AccxError) as e:   # extends past the mapping
            ax.acc_data_begin([_cl(ax, ax.ACC_PRESENT, x, 16, 32)])
        assert e.value.status == ax.ACC_ERR_NOT_PRESENT
        with pytest.raises(ax.AccxError) as e:   # partly mapped: present_or_* may not remap it
            ax.acc_data_begin([_cl(ax, ax.ACC_PRESENT_OR_COPY, x, 16, 32)])
        assert e.value.status == ax.ACC_ERR_ALREADY_PRESENT
        with pytest.raises(ax.AccxError) as e:   # same bytes, another dtype
            ax.acc_data_begin([ax.clause(ax.ACC_PRESENT, ax.ACC_INT32, x, 0, 8)])
        assert e.value.status == ax.ACC_ERR_INVALID_ARG
        inner = ax.acc_data_begin([_cl(ax, ax.ACC_PRESENT, x, 8, 8)])  # a subrange is present
        ax.acc_data_end(inner)
    finally:
        ax.acc_data_end(r)


def test_present_or_copyin_does_not_copy_a_present_range(ax):
    n = 1 << 16
    x = synth.uniform01_f32(n, SEED, 410)
    outer = ax.acc_data_begin([_cl(ax, ax.ACC_COPYIN, x)])
    ax.acc_wait(outer)
    old = x.copy()
    x[:] = 0.0                                   # host changes; the device copy keeps the old values
    inner = ax.acc_data_begin([_cl(ax, ax.ACC_PRESENT_OR_COPYIN, x)])
    s = np.zeros(1, np.float32)
    ax.acc_reduce_sum(inner, ax.ACC_FLOAT32, x, n, s)
    ax.acc_data_end(inner)
    ax.acc_data_end(outer)
    assert abs(float(s[0]) - oracle.sum_f32(old)) <= 1e-5 * oracle.sum_f32(old)
    # not mapped: present_or_copyin copies in
    y = synth.uniform01_f32(n, SEED, 411)
    r = ax.acc_data_begin([_cl(ax, ax.ACC_PRESENT_OR_COPYIN, y)])
    s[0] = 0
    ax.acc_reduce_sum(r, ax.ACC_FLOAT32, y, n, s)
    ax.acc_data_end(r)
    assert abs(float(s[0]) - oracle.sum_f32(y)) <= 1e-5 * oracle.sum_f32(y)


def test_present_or_copyout_and_create_when_absent(ax):
    n = 64
    a, b, c = _mats(n, 420)
    t = np.zeros((n, n), np.float32)
    r = ax.acc_data_begin([_cl(ax, ax.ACC_PRESENT_OR_COPYIN, a), _cl(ax, ax.ACC_PRESENT_OR_COPYIN, b),
                           _cl(ax, ax.ACC_PRESENT_OR_CREATE, t), _cl(ax, ax.ACC_PRESENT_OR_COPYOUT, c)])
    ax.acc_loopnest_matmul(r, ax.ACC_FLOAT32, a, b, t, n, ax.ACC_KERNEL_PLAIN)      # t = ab
    ax.acc_loopnest_matmul(r, ax.ACC_FLOAT32, t, b, c, n, ax.ACC_KERNEL_PLAIN)      # c = (ab)b
    ax.acc_data_end(r)
    assert np.all(t == 0)                                                            # create: never copied out
    ab = oracle.matmul_f32(a, b)
    ref = oracle.matmul_f32(ab.astype(np.float32), b)
    # The device's t carries the first product's error (at most 1e-5 of
    # ||ab||), which the second product multiplies by b (at most its spectral
    # norm), on top of the second product's own 1e-5: the bound for c is
    # 1e-5 * (1 + ||ab|| ||b||_2 / ||(ab)b||), about 3e-5 for these inputs.
    tol = FP32_REL_FRO_TOL * (1.0 + np.linalg.norm(ab) * np.linalg.norm(b.astype(np.float64), 2) /
                              np.linalg.norm(ref))
    assert rel_fro(c, ref) <= tol


def test_update_device_and_host(ax):
    n = 1 << 18
    x = synth.uniform01_f32(n, SEED, 430)
    r = ax.acc_data_begin([_cl(ax, ax.ACC_COPYIN, x)])
    s = np.zeros(1, np.float32)
    ax.acc_reduce_sum(r, ax.ACC_FLOAT32, x, n, s)
    assert abs(float(s[0]) - oracle.sum_f32(x)) <= 1e-5 * oracle.sum_f32(x)
    x[1000:3000] = 1.0                                                               # host-side change ...
    ax.acc_update(r, ax.ACC_UPDATE_DEVICE, ax.ACC_FLOAT32, x, 1000, 2000)           # ... pushed for a subrange
    s[0] = 0
    ax.acc_reduce_sum(r, ax.ACC_FLOAT32, x, n, s)
    assert abs(float(s[0]) - oracle.sum_f32(x)) <= 1e-5 * oracle.sum_f32(x)
    ax.acc_data_end(r)

    m = 80
    a, b, c = _mats(m, 431)
    r = ax.acc_data_begin([_cl(ax, ax.ACC_COPYIN, a), _cl(ax, ax.ACC_COPYIN, b), _cl(ax, ax.ACC_CREATE, c)])
    ax.acc_loopnest_matmul(r, ax.ACC_FLOAT32, a, b, c, m, ax.ACC_KERNEL_TILED | ax.ACC_PREC_FULL6)
    ax.acc_update(r, ax.ACC_UPDATE_HOST, ax.ACC_FLOAT32, c, 0, m * m // 2, ax.ACC_ASYNC)   # first half of the rows
    ax.acc_wait(r)
    ref = oracle.matmul_f32(a, b)
    assert rel_fro(c[:m // 2], ref[:m // 2]) <= FP32_REL_FRO_TOL
    assert np.all(c[m // 2:] == 0)
    ax.acc_data_end(r)                                                               # create: no copyout
    with pytest.raises(ax.AccxError) as e:
        r2 = ax.acc_data_begin([_cl(ax, ax.ACC_COPYIN, a)])
        try:
            ax.acc_update(r2, ax.ACC_UPDATE_HOST, ax.ACC_FLOAT32, b, 0, 4)
        finally:
            ax.acc_data_end(r2)
    assert e.value.status == ax.ACC_ERR_NOT_PRESENT


def test_pinned_regions_on_two_streams(ax):
    # region A streams a large reduction input in while region B runs a matmul
    import torch
    n = 1 << 26
    pa = ax.accx_host_alloc(n * 4)
    try:
        x = np.ctypeslib.as_array((ctypes.c_float * n).from_address(pa))
        x[:] = synth.uniform01_f32(n, SEED, 440)
        m = 1024
        a, b, c = _mats(m, 441)
        ra = ax.acc_data_begin([_cl(ax, ax.ACC_COPYIN, x)])
        rb = ax.acc_data_begin([_cl(ax, ax.ACC_COPYIN, a), _cl(ax, ax.ACC_COPYIN, b), _cl(ax, ax.ACC_COPY, c)])
        ax.acc_loopnest_matmul(rb, ax.ACC_FLOAT32, a, b, c, m, ax.ACC_KERNEL_PLAIN)
        s = np.zeros(1, np.float32)
        ax.acc_reduce_sum(ra, ax.ACC_FLOAT32, x, n, s, ax.ACC_ASYNC)
        ax.acc_data_end(ra)
        ax.acc_data_end(rb)
        torch.cuda.synchronize()
        ref = oracle.sum_f32(x)
        assert abs(float(s[0]) - ref) <= 1e-5 * ref
        g = synth.rng(SEED, 442)
        ii, jj = g.integers(0, m, 256), g.integers(0, m, 256)
        assert rel_fro(c[ii, jj], oracle.matmul_at(a, b, ii, jj)) <= FP32_REL_FRO_TOL
    finally:
        ax.accx_host_free(pa)


def test_present_region_waits_for_the_creators_copy_in(ax):
    # The outer region copies a and b in from page-locked memory, which runs
    # asynchronously on its stream; an inner region takes them with present
    # clauses and launches the matmul at once, with no wait on the outer
    # region: its stream must still see the copied-in values.
    import torch
    n = 2048
    ptrs = [ax.accx_host_alloc(n * n * 4) for _ in range(3)]
    try:
        a, b, c = [np.ctypeslib.as_array((ctypes.c_float * (n * n)).from_address(p)).reshape(n, n) for p in ptrs]
        a[:] = synth.uniform_pm1_f32((n, n), SEED, 451)
        b[:] = synth.uniform_pm1_f32((n, n), SEED, 452)
        c[:] = 0.0
        outer = ax.acc_data_begin([_cl(ax, ax.ACC_COPYIN, a), _cl(ax, ax.ACC_COPYIN, b)])
        inner = ax.acc_data_begin([_cl(ax, ax.ACC_PRESENT, a), _cl(ax, ax.ACC_PRESENT, b),
                                   _cl(ax, ax.ACC_COPYOUT, c)])
        ax.acc_loopnest_matmul(inner, ax.ACC_FLOAT32, a, b, c, n, ax.ACC_KERNEL_TILED | ax.ACC_PREC_FULL6)
        ax.acc_data_end(inner)
        ax.acc_data_end(outer)
        torch.cuda.synchronize()
        g = synth.rng(SEED, 453)
        ii, jj = g.integers(0, n, 512), g.integers(0, n, 512)
        assert rel_fro(c[ii, jj], oracle.matmul_at(np.array(a), np.array(b), ii, jj)) <= FP32_REL_FRO_TOL
    finally:
        for p in ptrs:
            ax.accx_host_free(p)


def test_budget_counts_new_mappings_only(ax):
    x = np.zeros(1 << 20, np.float32)
    r = ax.acc_data_begin([_cl(ax, ax.ACC_COPYIN, x)])
    used = ax.acc_budget_used()
    inner = ax.acc_data_begin([_cl(ax, ax.ACC_PRESENT, x), _cl(ax, ax.ACC_PRESENT_OR_COPY, x)])
    assert ax.acc_budget_used() == used
    ax.acc_data_end(inner)
    ax.acc_data_end(r)
    assert ax.acc_budget_used() < used
