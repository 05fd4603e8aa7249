"""Parity of the float32 tiled kernel on the float32 matrix cores
(ACC_PREC_F32MFMA: no split, float32 operands, float32 accumulation), the
comparator the bf16x3 modes are measured against, with the CPU oracle: the
loop nest of Listing 1a (section 1.3) on the LDS-tiled kernel of the Matrix
Multiplication paragraph of section 4.2."""
import numpy as np
import pytest

import oracle
import synth
from _util import FP32_REL_FRO_TOL, SEED, rel_fro, tile_samples

pytestmark = pytest.mark.gpu

SIZES = [1, 2, 15, 16, 17, 31, 33, 64, 100, 255, 256, 257, 300, 513, 1000]


@pytest.fixture(scope="module")
def ax():
    import paper_1412_1127_amd as ax
    ax.acc_init(0, 0)
    yield ax
    ax.acc_shutdown()


def _flags(ax, tile=None):
    return ax.ACC_KERNEL_TILED | ax.ACC_PREC_F32MFMA | (ax.TILES[tile] if tile else 0)


def _gemm(ax, a, b, flags):
    import torch
    m, k = a.shape
    n = b.shape[1]
    da, db = torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()
    dc = torch.full((m, n), float("nan"), device="cuda")
    print("f32mfma %dx%dx%d flags=%#x" % (m, n, k, flags), flush=True)
    ax.accx_gemm_dev(ax.ACC_FLOAT32, m, n, k, da, k, db, n, dc, n, flags)
    torch.cuda.synchronize()
    return dc.cpu().numpy()


@pytest.mark.parametrize("n", SIZES)
def test_square_parity(ax, n):
    a = synth.uniform_pm1_f32((n, n), SEED, synth.STREAM_A)
    b = synth.uniform_pm1_f32((n, n), SEED, synth.STREAM_B)
    err = rel_fro(_gemm(ax, a, b, _flags(ax)), oracle.matmul_f32(a, b))
    print("LEN=%d F32MFMA rel_fro=%.3g" % (n, err))
    assert err <= FP32_REL_FRO_TOL


@pytest.mark.parametrize("tile", ["256", "256x128", "128", "64"])
@pytest.mark.parametrize("shape", [(100, 257, 1000), (257, 100, 33), (513, 640, 129), (64, 64, 4096)])
def test_every_tile_rectangular(ax, tile, shape):
    m, n, k = shape
    a = synth.uniform_pm1_f32((m, k), SEED, 21)
    b = synth.uniform_pm1_f32((k, n), SEED, 22)
    err = rel_fro(_gemm(ax, a, b, _flags(ax, tile)), oracle.gemm(a, b))
    assert err <= FP32_REL_FRO_TOL, (tile, shape, err)


def test_identity_and_ones_exact(ax):
    n = 160
    a = synth.uniform_pm1_f32((n, n), SEED, 5)
    eye = np.eye(n, dtype=np.float32)
    assert np.array_equal(_gemm(ax, eye, a, _flags(ax)), a)
    assert np.array_equal(_gemm(ax, a, eye, _flags(ax)), a)
    one = np.ones((n, n), np.float32)
    assert np.all(_gemm(ax, one, one, _flags(ax)) == n)


def test_integer_valued_floats_bitwise_equal_int(ax):
    # |C| <= LEN * 256 < 2^24: every partial sum is an exact integer
    n = 512
    ai = synth.int_uniform_i32((n, n), -16, 16, SEED, synth.STREAM_A)
    bi = synth.int_uniform_i32((n, n), -16, 16, SEED, synth.STREAM_B)
    cf = _gemm(ax, ai.astype(np.float32), bi.astype(np.float32), _flags(ax))
    assert np.array_equal(cf, oracle.matmul_i32(ai, bi).astype(np.float32))


def test_len4096_uniform_and_8192_rowscaled(ax):
    n = 4096
    a = synth.uniform_pm1_f32((n, n), SEED, synth.STREAM_A)
    b = synth.uniform_pm1_f32((n, n), SEED, synth.STREAM_B)
    c = _gemm(ax, a, b, _flags(ax))
    ii, jj = tile_samples(n, n, 256, 256, 2048)
    err = rel_fro(c[ii, jj], oracle.matmul_at(a, b, ii, jj))
    print("LEN=4096 F32MFMA rel_fro=%.3g" % err, flush=True)
    assert err <= FP32_REL_FRO_TOL
    n = 8192
    a = synth.normal_rowscaled_f32(n, n, SEED, synth.STREAM_A)
    b = synth.normal_rowscaled_f32(n, n, SEED, synth.STREAM_B)
    c = _gemm(ax, a, b, _flags(ax))
    ii, jj = tile_samples(n, n, 256, 256, 4096)
    err = rel_fro(c[ii, jj], oracle.matmul_at(a, b, ii, jj))
    print("LEN=8192 row-scaled F32MFMA rel_fro=%.3g" % err)
    assert err <= FP32_REL_FRO_TOL


def test_deterministic_and_autotuned(ax):
    n = 1000
    tile, ms = ax.accx_autotune(ax.ACC_FLOAT32, n, ax.ACC_PREC_F32MFMA)
    assert tile in ax.TILES.values() and ms > 0
    a = synth.uniform_pm1_f32((n, n), SEED, 31)
    b = synth.uniform_pm1_f32((n, n), SEED, 32)
    c1 = _gemm(ax, a, b, _flags(ax))
    c2 = _gemm(ax, a, b, _flags(ax))
    assert np.array_equal(c1, c2)
    assert rel_fro(c1, oracle.matmul_f32(a, b)) <= FP32_REL_FRO_TOL
