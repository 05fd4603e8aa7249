"""Parity of the plain loop-nest kernels (one thread per (i, j), l sequential;
Listing 1a/1b, section 1.3) with the CPU oracle, through the C ABI."""
import numpy as np
import pytest

import oracle
import synth
from _util import FP32_REL_FRO_TOL, SEED, rel_fro, sample_entries

pytestmark = pytest.mark.gpu

PLAIN_KERNELS = ["plain", "listing1b"]


@pytest.fixture(scope="module")
def ax():
    import paper_1412_1127_amd as ax
    ax.acc_init(0, 0)
    yield ax
    ax.acc_shutdown()


def _flag(ax, name):
    return {"plain": ax.ACC_KERNEL_PLAIN, "listing1b": ax.ACC_KERNEL_PLAIN_LISTING1B}[name]


def _run(ax, a, b, flags):
    import torch
    n = a.shape[0]
    dt = ax.ACC_FLOAT32 if a.dtype == np.float32 else ax.ACC_INT32
    da, db = torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()
    dc = torch.full((n, n), -7, dtype=da.dtype, device="cuda")
    print("matmul dtype=%s LEN=%d flags=%#x" % (a.dtype, n, flags), flush=True)
    ax.accx_matmul_dev(dt, da, db, dc, n, flags)
    torch.cuda.synchronize()
    return dc.cpu().numpy()


@pytest.mark.parametrize("kernel", PLAIN_KERNELS)
@pytest.mark.parametrize("n", [1, 2, 17, 64, 100, 256, 257])
def test_f32_parity(ax, kernel, n):
    a = synth.uniform_pm1_f32((n, n), SEED, synth.STREAM_A)
    b = synth.uniform_pm1_f32((n, n), SEED, synth.STREAM_B)
    c = _run(ax, a, b, _flag(ax, kernel))
    assert rel_fro(c, oracle.matmul_f32(a, b)) <= FP32_REL_FRO_TOL


@pytest.mark.parametrize("kernel", PLAIN_KERNELS)
@pytest.mark.parametrize("n", [1, 3, 64, 129, 256])
def test_i32_bit_exact_full_range(ax, kernel, n):
    a = synth.full_range_i32((n, n), SEED, synth.STREAM_A)
    b = synth.full_range_i32((n, n), SEED, synth.STREAM_B)
    assert np.array_equal(_run(ax, a, b, _flag(ax, kernel)), oracle.matmul_i32(a, b))


@pytest.mark.parametrize("kernel", PLAIN_KERNELS)
def test_identity_and_ones_exact(ax, kernel):
    n = 96
    a = synth.uniform_pm1_f32((n, n), SEED, 5)
    eye = np.eye(n, dtype=np.float32)
    assert np.array_equal(_run(ax, eye, a, _flag(ax, kernel)), a)
    one = np.ones((n, n), np.float32)
    assert np.all(_run(ax, one, one, _flag(ax, kernel)) == n)


@pytest.mark.parametrize("kernel", PLAIN_KERNELS)
def test_integer_valued_floats_equal_int_path(ax, kernel):
    n = 200
    ai = synth.int_uniform_i32((n, n), -16, 16, SEED, synth.STREAM_A)
    bi = synth.int_uniform_i32((n, n), -16, 16, SEED, synth.STREAM_B)
    cf = _run(ax, ai.astype(np.float32), bi.astype(np.float32), _flag(ax, kernel))
    ci = _run(ax, ai, bi, _flag(ax, kernel))
    assert np.array_equal(cf, ci.astype(np.float32))
    assert np.array_equal(ci, oracle.matmul_i32(ai, bi))


def test_deterministic(ax):
    n = 300
    a = synth.uniform_pm1_f32((n, n), SEED, 7)
    b = synth.uniform_pm1_f32((n, n), SEED, 8)
    c1 = _run(ax, a, b, ax.ACC_KERNEL_PLAIN)
    c2 = _run(ax, a, b, ax.ACC_KERNEL_PLAIN)
    assert np.array_equal(c1, c2)


def test_full_size_sampled(ax):
    # LEN = 4096, the plain-method-at-scale workload: sampled entries vs the oracle.
    n = 4096
    a = synth.uniform_pm1_f32((n, n), SEED, synth.STREAM_A)
    b = synth.uniform_pm1_f32((n, n), SEED, synth.STREAM_B)
    c = _run(ax, a, b, ax.ACC_KERNEL_PLAIN)
    ii, jj = sample_entries(n, 256)
    assert rel_fro(c[ii, jj], oracle.matmul_at(a, b, ii, jj)) <= FP32_REL_FRO_TOL
    ai = synth.int_uniform_i32((n, n), -16, 16, SEED, synth.STREAM_A)
    bi = synth.int_uniform_i32((n, n), -16, 16, SEED, synth.STREAM_B)
    ci = _run(ax, ai, bi, ax.ACC_KERNEL_PLAIN)
    assert np.array_equal(ci[ii, jj], oracle.matmul_at(ai, bi, ii, jj))
