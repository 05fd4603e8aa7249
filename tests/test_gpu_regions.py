"""Data regions (copy / copyin / copyout / create over [start:n], section 1.3;
pointer exchange, section 2.3) and the ops that run inside them, through the
C ABI, against the oracle."""
import os
import subprocess
import sys

import numpy as np
import pytest

import oracle
import synth
from _util import FP32_REL_FRO_TOL, SEED, rel_fro

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def ax():
    import paper_1412_1127_amd as ax
    ax.acc_init(0, 0)
    yield ax
    ax.acc_shutdown()


def test_listing1a_data_region_copy(ax):
    # copy(a[0:LEN*LEN], b[0:LEN*LEN], c[0:LEN*LEN]) + kernels loop nest
    n = 128
    a = synth.uniform_pm1_f32((n, n), SEED, 1)
    b = synth.uniform_pm1_f32((n, n), SEED, 2)
    c = np.zeros((n, n), np.float32)
    r = ax.acc_data_begin([ax.clause(ax.ACC_COPY, ax.ACC_FLOAT32, m) for m in (a, b, c)])
    ax.acc_loopnest_matmul(r, ax.ACC_FLOAT32, a, b, c, n, ax.ACC_KERNEL_PLAIN)
    assert np.all(c == 0)  # host c changes only at region exit
    ax.acc_data_end(r)
    assert rel_fro(c, oracle.matmul_f32(a, b)) <= FP32_REL_FRO_TOL


def test_copyin_copyout_create_subarrays(ax):
    n = 64
    big_a = synth.full_range_i32((3 * n * n,), SEED, 3)
    big_b = synth.full_range_i32((n * n + 5,), SEED, 4)
    out = np.zeros(2 * n * n, np.int32)
    a_view = big_a[n * n:2 * n * n].reshape(n, n)
    b_view = big_b[5:].reshape(n, n)
    r = ax.acc_data_begin([
        ax.clause(ax.ACC_COPYIN, ax.ACC_INT32, big_a, n * n, n * n),
        ax.clause(ax.ACC_COPYIN, ax.ACC_INT32, big_b, 5, n * n),
        ax.clause(ax.ACC_COPYOUT, ax.ACC_INT32, out, n * n, n * n),
    ])
    # host addresses inside the mapped subarrays
    ax.acc_loopnest_matmul(r, ax.ACC_INT32, a_view, b_view, out[n * n:], n, ax.ACC_KERNEL_PLAIN)
    ax.acc_data_end(r)
    assert np.array_equal(out[n * n:].reshape(n, n), oracle.matmul_i32(np.ascontiguousarray(a_view),
                                                                         np.ascontiguousarray(b_view)))
    assert np.all(out[:n * n] == 0)  # outside the copyout range


def test_create_is_device_only_and_reused(ax):
    n = 32
    a = synth.uniform_pm1_f32((n, n), SEED, 5)
    b = synth.uniform_pm1_f32((n, n), SEED, 6)
    tmp = np.full((n, n), 3.0, np.float32)
    c = np.zeros((n, n), np.float32)
    r = ax.acc_data_begin([ax.clause(ax.ACC_COPYIN, ax.ACC_FLOAT32, a), ax.clause(ax.ACC_COPYIN, ax.ACC_FLOAT32, b),
                           ax.clause(ax.ACC_CREATE, ax.ACC_FLOAT32, tmp), ax.clause(ax.ACC_COPYOUT, ax.ACC_FLOAT32, c)])
    ax.acc_loopnest_matmul(r, ax.ACC_FLOAT32, a, b, tmp, n, ax.ACC_KERNEL_PLAIN)   # tmp = a b (device)
    ax.acc_loopnest_matmul(r, ax.ACC_FLOAT32, tmp, b, c, n, ax.ACC_KERNEL_PLAIN)   # c = (a b) b
    ax.acc_data_end(r)
    assert np.all(tmp == 3.0)  # create never copies back
    ab = oracle.matmul_f32(a, b).astype(np.float32)
    assert rel_fro(c, oracle.matmul_f32(ab, b)) <= 1e-5


def test_reduce_in_region_sync_and_async(ax):
    x = synth.uniform01_f32(100003, SEED, 7)
    xi = synth.int_uniform_i32((5000,), -1000, 1000, SEED, 8)
    r = ax.acc_data_begin([ax.clause(ax.ACC_COPYIN, ax.ACC_FLOAT32, x), ax.clause(ax.ACC_COPYIN, ax.ACC_INT32, xi)])
    s = np.array([0.25], np.float32)
    ax.acc_reduce_sum(r, ax.ACC_FLOAT32, x, x.size, s)
    assert abs(float(s[0]) - oracle.sum_f32(x, 0.25)) / oracle.sum_f32(x, 0.25) <= 1e-5
    si = np.array([7], np.int32)
    ax.acc_reduce_sum(r, ax.ACC_INT32, xi, xi.size, si, ax.ACC_REDUCE_PLAIN)
    assert si[0] == oracle.sum_i32(xi, 7)
    # asynchronous: results land at acc_wait
    outs = [np.array([float(k)], np.float32) for k in range(5)]
    for k, o in enumerate(outs):
        ax.acc_reduce_sum(r, ax.ACC_FLOAT32, x[k:], x.size - k, o, ax.ACC_ASYNC)
    ax.acc_wait(r)
    for k, o in enumerate(outs):
        ref = oracle.sum_f32(x[k:], float(k))
        assert abs(float(o[0]) - ref) / ref <= 1e-5
    z = np.array([4.0], np.float32)
    ax.acc_reduce_sum(r, ax.ACC_FLOAT32, x, 0, z)  # n = 0: unchanged
    assert z[0] == 4.0
    ax.acc_data_end(r)


def test_present_errors(ax):
    a = np.zeros(100, np.float32)
    other = np.zeros(100, np.float32)
    r = ax.acc_data_begin([ax.clause(ax.ACC_COPYIN, ax.ACC_FLOAT32, a, 10, 50)])
    try:
        with pytest.raises(ax.AccxError) as e:   # overlaps a[10:60]
            ax.acc_data_begin([ax.clause(ax.ACC_COPYIN, ax.ACC_FLOAT32, a, 50, 20)])
        assert e.value.status == ax.ACC_ERR_ALREADY_PRESENT
        with pytest.raises(ax.AccxError) as e:   # not mapped
            ax.acc_reduce_sum(r, ax.ACC_FLOAT32, other, 10, np.zeros(1, np.float32))
        assert e.value.status == ax.ACC_ERR_NOT_PRESENT
        with pytest.raises(ax.AccxError) as e:   # runs past the mapped end
            ax.acc_reduce_sum(r, ax.ACC_FLOAT32, a[40:], 30, np.zeros(1, np.float32))
        assert e.value.status == ax.ACC_ERR_NOT_PRESENT
        with pytest.raises(ax.AccxError) as e:   # dtype mismatch
            ax.acc_reduce_sum(r, ax.ACC_INT32, a[10:], 5, np.zeros(1, np.int32))
        assert e.value.status == ax.ACC_ERR_INVALID_ARG
        # pointer exchange
        base = ax.acc_deviceptr(a[10:])
        assert ax.acc_deviceptr(a[11:]) == base + 4
        with pytest.raises(ax.AccxError):
            ax.acc_deviceptr(a[60:])
        # a disjoint range of the same array is fine
        r2 = ax.acc_data_begin([ax.clause(ax.ACC_COPYIN, ax.ACC_FLOAT32, a, 60, 40)])
        ax.acc_data_end(r2)
    finally:
        ax.acc_data_end(r)


def test_budget_admission(ax):
    used0 = ax.acc_budget_used()
    ax.acc_shutdown()
    ax.acc_init(0, 1 << 20)  # 1 MiB
    try:
        small = np.zeros(1 << 17, np.float32)  # 512 KiB
        big = np.zeros(1 << 18, np.float32)    # 1 MiB
        r = ax.acc_data_begin([ax.clause(ax.ACC_COPYIN, ax.ACC_FLOAT32, small)])
        assert ax.acc_budget_used() == small.nbytes
        with pytest.raises(ax.AccxError) as e:
            ax.acc_data_begin([ax.clause(ax.ACC_COPYIN, ax.ACC_FLOAT32, big)])
        assert e.value.status == ax.ACC_ERR_OUT_OF_MEMORY
        ax.acc_data_end(r)
        assert ax.acc_budget_used() == 0
        r = ax.acc_data_begin([ax.clause(ax.ACC_COPYIN, ax.ACC_FLOAT32, big)])
        ax.acc_data_end(r)
    finally:
        ax.acc_shutdown()
        ax.acc_init(0, 0)
    assert used0 >= 0


FAULT_SCRIPT = r'''
import sys, numpy as np
sys.path.insert(0, %(root)r)
import paper_1412_1127_amd as ax
ax.acc_init(0, 0)
a = np.ones((8, 8), np.float32); c = np.zeros((8, 8), np.float32)
kind = %(kind)r
try:
    r = ax.acc_data_begin([ax.clause(ax.ACC_COPYIN, ax.ACC_FLOAT32, a), ax.clause(ax.ACC_COPYOUT, ax.ACC_FLOAT32, c)])
except ax.AccxError as e:
    print("BEGIN", e.status); print("USED", ax.acc_budget_used()); sys.exit(0)
try:
    ax.acc_loopnest_matmul(r, ax.ACC_FLOAT32, a, a, c, 8, ax.ACC_KERNEL_PLAIN)
    print("OP", 0)
except ax.AccxError as e:
    print("OP", e.status)
    try:
        ax.acc_loopnest_matmul(r, ax.ACC_FLOAT32, a, a, c, 8, ax.ACC_KERNEL_PLAIN)
    except ax.AccxError as e2:
        print("POISONED", e2.status)
try:
    ax.acc_data_end(r); print("END", 0)
except ax.AccxError as e:
    print("END", e.status)
print("USED", ax.acc_budget_used())
print("C", float(c.sum()))
'''


@pytest.mark.parametrize("kind,expect", [
    ("alloc:2", {"BEGIN": "-4", "USED": "0"}),
    ("copy:1", {"BEGIN": "-5", "USED": "0"}),
    ("launch:1", {"OP": "-5", "POISONED": "-5", "END": "-5", "USED": "0", "C": "0.0"}),
    ("copy:2", {"OP": "0", "END": "-5", "USED": "0"}),
])
def test_fault_injection(kind, expect):
    # Injected on the host before the HIP call: no kernel ever faults.
    env = dict(os.environ, ACCX_FAULT=kind)
    out = subprocess.run([sys.executable, "-c", FAULT_SCRIPT % {"root": ROOT, "kind": kind}], env=env,
                         capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stderr
    got = dict(line.split(None, 1) for line in out.stdout.strip().splitlines())
    for k, v in expect.items():
        assert got.get(k) == v, (kind, got)
