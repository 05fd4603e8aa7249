"""The sampled float64 error probe behind ACC_PREC_AUTO: its float64 dot
products against the oracle, its decisions against its own rule, and the
final result against the float32 bound."""
import numpy as np
import pytest

import oracle
import synth
from _util import FP32_REL_FRO_TOL, SEED, rel_fro

pytestmark = pytest.mark.gpu
TAU = 7e-6


@pytest.fixture(scope="module")
def ax():
    import paper_1412_1127_amd as ax
    ax.acc_init(0, 0)
    yield ax
    ax.acc_shutdown()


def _auto(ax, a, b):
    import torch
    n = a.shape[0]
    flags = ax.ACC_KERNEL_TILED | ax.ACC_PREC_AUTO
    ws = torch.zeros(ax.accx_matmul_workspace_size(ax.ACC_FLOAT32, n, flags), dtype=torch.uint8, device="cuda")
    da, db = torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()
    dc = torch.empty((n, n), dtype=torch.float32, device="cuda")
    print("AUTO LEN=%d" % n, flush=True)
    ax.accx_matmul_dev(ax.ACC_FLOAT32, da, db, dc, n, flags, ws, ws.numel())
    dcc = torch.empty_like(dc)
    ax.accx_matmul_dev(ax.ACC_FLOAT32, da, db, dcc, n, ax.ACC_KERNEL_TILED | ax.ACC_PREC_CHEAP3)
    torch.cuda.synchronize()
    off, cnt = ax.accx_probe_layout(n, flags)
    raw = ws.cpu().numpy().tobytes()[off:]
    return dc.cpu().numpy(), dcc.cpu().numpy(), ax.probe_records(raw, cnt)


def _check_records(a, b, cheap, recs):
    for r in recs:
        rows, cols = list(r.rows), list(r.cols)
        ii = np.repeat(rows, len(rows))
        jj = np.tile(cols, len(rows))
        ref = oracle.matmul_at(a, b, ii, jj)
        got = np.array(list(r.ref))
        # float64 sums in another order: agree to float64 rounding
        assert np.all(np.abs(got - ref) <= 1e-12 * np.maximum(1.0, np.abs(ref).max())), (rows, cols)
        c = cheap[ii, jj].astype(np.float64)
        e2, r2 = float(np.sum((c - got) ** 2)), float(np.sum(got ** 2))
        assert abs(e2 - r.err2) <= 1e-9 * max(e2, 1e-300) + 1e-300
        assert abs(r2 - r.ref2) <= 1e-12 * r2
        assert r.corrected == int(e2 > TAU * TAU * r2 if r2 > 0 else e2 > 0)


@pytest.mark.parametrize("n", [100, 257, 1000, 2048])
def test_auto_full_precision_inputs(ax, n):
    a = synth.uniform_pm1_f32((n, n), SEED, synth.STREAM_A)
    b = synth.uniform_pm1_f32((n, n), SEED, synth.STREAM_B)
    c, cheap, recs = _auto(ax, a, b)
    _check_records(a, b, cheap, recs)
    ref = oracle.matmul_f32(a, b) if n <= 1000 else None
    if ref is not None:
        err = rel_fro(c, ref)
        print("LEN=%d AUTO rel_fro=%.3g CHEAP3=%.3g corrected %d/%d" % (
            n, err, rel_fro(cheap, ref), sum(r.corrected for r in recs), len(recs)))
        assert err <= FP32_REL_FRO_TOL


def _biased_split(g, shape):
    # x = h + m + l with h in [1, 1.125) on the bf16 grid, m in
    # [1.5, 2) * 2^-9 on its grid (below half an ulp of h) and l in
    # [1.5, 2) * 2^-18 with 6 bits (below half an ulp of m): the split returns
    # (h, m, l) exactly, and every term the three cheap products drop (h*l,
    # l*h, m*m) is positive, so the cheap error accumulates instead of
    # cancelling: 2.3e-5 relative, against 4e-8 for the six products.
    h = 1.0 + g.integers(0, 16, shape) * 2.0 ** -7
    m = 2.0 ** -9 * (1.0 + g.integers(64, 128, shape) * 2.0 ** -7)
    l = 2.0 ** -18 * (1.0 + g.integers(16, 32, shape) * 2.0 ** -5)
    x = (h + m + l).astype(np.float32)
    assert np.array_equal(x.astype(np.float64), h + m + l)   # 24 significant bits: exact
    return x


@pytest.mark.parametrize("n", [256, 300])
def test_auto_corrects_biased_split_error(ax, n):
    g = synth.rng(SEED, 8)
    a, b = _biased_split(g, (n, n)), _biased_split(g, (n, n))
    c, cheap, recs = _auto(ax, a, b)
    _check_records(a, b, cheap, recs)
    ref = oracle.matmul_f32(a, b)
    print("LEN=%d biased split: CHEAP3 rel_fro=%.3g AUTO=%.3g corrected %d/%d" % (
        n, rel_fro(cheap, ref), rel_fro(c, ref), sum(r.corrected for r in recs), len(recs)))
    assert rel_fro(cheap, ref) > 1.2e-5          # the cheap pass alone misses the bound
    assert all(r.corrected for r in recs)        # the probe marks every tile
    assert rel_fro(c, ref) <= FP32_REL_FRO_TOL   # and the correction brings it back


def test_auto_low_precision_inputs_keep_cheap(ax):
    # 8-bit significands: every input is one bf16 term, the three cheap
    # products are exact, no tile needs the correction.
    n = 700
    g = synth.rng(SEED, 5)
    a = (g.integers(-128, 128, (n, n)) * 2.0 ** -7).astype(np.float32)
    b = (g.integers(-128, 128, (n, n)) * 2.0 ** -5).astype(np.float32)
    c, cheap, recs = _auto(ax, a, b)
    _check_records(a, b, cheap, recs)
    assert not any(r.corrected for r in recs)
    assert np.array_equal(c, cheap)
    assert rel_fro(c, oracle.matmul_f32(a, b)) <= FP32_REL_FRO_TOL


def test_auto_mixed_rows(ax):
    # top half of A full-precision, bottom half 8-bit: only tiles that touch
    # the top rows need the correction.
    n = 512
    g = synth.rng(SEED, 6)
    a = synth.uniform_pm1_f32((n, n), SEED, 7)
    a[n // 2:] = (g.integers(-128, 128, (n // 2, n)) * 2.0 ** -7).astype(np.float32)
    b = (g.integers(-128, 128, (n, n)) * 2.0 ** -7).astype(np.float32)
    c, cheap, recs = _auto(ax, a, b)
    _check_records(a, b, cheap, recs)
    assert rel_fro(c, oracle.matmul_f32(a, b)) <= FP32_REL_FRO_TOL
    bottom = [r for r in recs if min(r.rows) >= n // 2]
    assert bottom and not any(r.corrected for r in bottom)
