"""Parity of the configurations the benchmark times, at their full sizes, in
the launch configuration it times them (Listing 1a's loop nest, section 1.3):

- float32 LEN=4096, uniform[-1, 1], ACC_PREC_AUTO (three-product pass, the
  float64 probe and the correction of marked tiles) on the autotuned tile
  and on the size heuristic's tile: the whole matrix against the oracle;
- int32 LEN=4096, integers in [-16, 16], the one-digit path with its max|x|
  decision on the device: the whole matrix, bit-exact;
- float32 LEN=8192, N(0, 1) x 2^U(-8, 8) per row, AUTO: 4096+ entries that
  touch every tile row and column;
- inputs whose split error is biased (every term the cheap pass drops is
  positive) at LEN=2048 and 4096, AUTO on the heuristic's tile: every tile is
  marked, every marked tile corrected, the whole result within the bound.

The biased-split cases run first, before any autotuning in this module, so
that the tile the probe and the correction use is the size heuristic's."""
import numpy as np
import pytest

import oracle
import synth
from _util import FP32_REL_FRO_TOL, SEED, rel_fro, tile_samples

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ax():
    import paper_1412_1127_amd as ax
    ax.acc_init(0, 0)
    yield ax
    ax.acc_shutdown()


def _dev_matmul(ax, a, b, flags, want_records=False):
    import torch
    n = a.shape[0]
    dt = ax.ACC_FLOAT32 if a.dtype == np.float32 else ax.ACC_INT32
    ws = torch.empty(ax.accx_matmul_workspace_size(dt, n, flags), dtype=torch.uint8, device="cuda")
    da, db = torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()
    dc = torch.full((n, n), -7, dtype=da.dtype, device="cuda")
    print("matmul dtype=%s LEN=%d flags=%#x" % (a.dtype, n, flags), flush=True)
    ax.accx_matmul_dev(dt, da, db, dc, n, flags, ws, ws.numel())
    torch.cuda.synchronize()
    recs = None
    if want_records:
        off, cnt = ax.accx_probe_layout(n, flags)
        recs = ax.probe_records(ws.cpu().numpy().tobytes()[off:], cnt)
    return dc.cpu().numpy(), recs


def _biased_split(g, shape):
    # x = h + m + l exactly, with h on the bf16 grid in [1, 1.125), m in
    # [1.5, 2) * 2^-9 and l in [1.5, 2) * 2^-18 on grids fine enough that the
    # split returns (h, m, l): every product the cheap pass drops (h*l, l*h,
    # m*m) is positive, so its error accumulates to about 2.3e-5 relative.
    h = 1.0 + g.integers(0, 16, shape) * 2.0 ** -7
    m = 2.0 ** -9 * (1.0 + g.integers(64, 128, shape) * 2.0 ** -7)
    l = 2.0 ** -18 * (1.0 + g.integers(16, 32, shape) * 2.0 ** -5)
    x = (h + m + l).astype(np.float32)
    assert np.array_equal(x.astype(np.float64), h + m + l)
    return x


@pytest.mark.parametrize("n", [2048, 4096])
def test_auto_biased_split_heuristic_tile(ax, n):
    g = synth.rng(SEED, 18)
    a, b = _biased_split(g, (n, n)), _biased_split(g, (n, n))
    flags = ax.ACC_KERNEL_TILED | ax.ACC_PREC_AUTO
    c, recs = _dev_matmul(ax, a, b, flags, want_records=True)
    ref = oracle.matmul_f32(a, b)
    err = rel_fro(c, ref)
    print("LEN=%d biased split AUTO rel_fro=%.3g, %d/%d tiles corrected" % (
        n, err, sum(r.corrected for r in recs), len(recs)), flush=True)
    # the heuristic's tile: 128 x 128 at 2048 (16 x 16 tiles), 256 x 256 at 4096
    assert len(recs) == (n // (128 if n == 2048 else 256)) ** 2
    assert all(r.corrected for r in recs)
    assert err <= FP32_REL_FRO_TOL


def test_f32_auto_len4096_heuristic_tile_whole(ax):
    n = 4096
    a = synth.uniform_pm1_f32((n, n), SEED, synth.STREAM_A)
    b = synth.uniform_pm1_f32((n, n), SEED, synth.STREAM_B)
    c, _ = _dev_matmul(ax, a, b, ax.ACC_KERNEL_TILED | ax.ACC_PREC_AUTO)
    err = rel_fro(c, oracle.matmul_f32(a, b))
    print("LEN=4096 AUTO (heuristic tile) rel_fro=%.3g" % err)
    assert err <= FP32_REL_FRO_TOL


def test_bench_step_whole_matrices(ax):
    # The benchmark's step exactly: autotune both tiles, then the float32
    # AUTO matmul and the int32 matmul with the device-side digit decision.
    n = 4096
    tf, _ = ax.accx_autotune(ax.ACC_FLOAT32, n, ax.ACC_KERNEL_TILED | ax.ACC_PREC_AUTO)
    ti, _ = ax.accx_autotune(ax.ACC_INT32, n, ax.ACC_LIMBS(1))
    print("autotuned tiles f32 %#x i32 %#x" % (tf, ti), flush=True)
    a = synth.uniform_pm1_f32((n, n), SEED, synth.STREAM_A)
    b = synth.uniform_pm1_f32((n, n), SEED, synth.STREAM_B)
    c, _ = _dev_matmul(ax, a, b, ax.ACC_KERNEL_TILED | ax.ACC_PREC_AUTO)
    err = rel_fro(c, oracle.matmul_f32(a, b))
    print("LEN=4096 AUTO (autotuned tile) rel_fro=%.3g" % err, flush=True)
    assert err <= FP32_REL_FRO_TOL
    ai = synth.int_uniform_i32((n, n), -16, 16, SEED, synth.STREAM_A)
    bi = synth.int_uniform_i32((n, n), -16, 16, SEED, synth.STREAM_B)
    ci, _ = _dev_matmul(ax, ai, bi, ax.ACC_KERNEL_TILED)
    assert np.array_equal(ci, oracle.matmul_i32(ai, bi))


def test_precision_len8192_auto_tiles_sampled(ax):
    n = 8192
    a = synth.normal_rowscaled_f32(n, n, SEED, synth.STREAM_A)
    b = synth.normal_rowscaled_f32(n, n, SEED, synth.STREAM_B)
    ii, jj = tile_samples(n, n, 256, 256, 4096)
    ref = oracle.matmul_at(a, b, ii, jj)
    for prec in ("AUTO", "FULL6"):
        c, _ = _dev_matmul(ax, a, b, ax.ACC_KERNEL_TILED | getattr(ax, "ACC_PREC_" + prec))
        err = rel_fro(c[ii, jj], ref)
        print("LEN=8192 row-scaled %s rel_fro=%.3g over %d entries" % (prec, err, ii.size), flush=True)
        assert np.isfinite(c).all()
        assert err <= FP32_REL_FRO_TOL
