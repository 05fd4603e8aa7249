"""Parity of the loop nest on rectangular operands with leading dimensions
(C (m x n) = A (m x k) B (k x n), the nest of section 1.3 with its trip
counts and row strides as parameters) with the CPU oracle, through the C ABI:
every kernel, ragged shapes, padded rows, empty shapes, the region form, and
the whole 512 x 4096 x 4096 row block."""
import numpy as np
import pytest

import oracle
import synth
from _util import FP32_REL_FRO_TOL, SEED, rel_fro

pytestmark = pytest.mark.gpu

SHAPES = [(1, 1, 1), (1, 300, 77), (300, 1, 77), (37, 300, 129), (200, 65, 1000), (64, 64, 1), (96, 160, 33),
          (513, 257, 640)]
F32_KERNELS = ["plain", "listing1b", "full6", "auto"]
I32_KERNELS = ["plain", "listing1b", "tiled"]
GUARD = -7


@pytest.fixture(scope="module")
def ax():
    import paper_1412_1127_amd as ax
    ax.acc_init(0, 0)
    yield ax
    ax.acc_shutdown()


def _flags(ax, kernel):
    return {"plain": ax.ACC_KERNEL_PLAIN, "listing1b": ax.ACC_KERNEL_PLAIN_LISTING1B,
            "full6": ax.ACC_KERNEL_TILED | ax.ACC_PREC_FULL6, "cheap3": ax.ACC_KERNEL_TILED | ax.ACC_PREC_CHEAP3,
            "auto": ax.ACC_KERNEL_TILED | ax.ACC_PREC_AUTO, "tiled": ax.ACC_KERNEL_TILED}[kernel]


def _inputs(m, n, k, dtype, stream0=11):
    if dtype == "f32":
        return (synth.uniform_pm1_f32((m, k), SEED, stream0), synth.uniform_pm1_f32((k, n), SEED, stream0 + 1))
    if dtype == "i32small":
        return (synth.int_uniform_i32((m, k), -16, 16, SEED, stream0),
                synth.int_uniform_i32((k, n), -16, 16, SEED, stream0 + 1))
    return synth.full_range_i32((m, k), SEED, stream0), synth.full_range_i32((k, n), SEED, stream0 + 1)


def _gemm(ax, a, b, flags, pads=(3, 5, 2), m=None, n=None, k=None):
    """Run accx_gemm_dev on device copies of a and b held in row-padded
    buffers (lda = k + pads[0], ldb = n + pads[1], ldc = n + pads[2]).  The
    padding of A and B holds poison (NaN / INT32_MIN) that a stray read would
    carry into C; C's padding must keep its guard value.  Returns C (m x n)."""
    import torch
    m = a.shape[0] if m is None else m
    k = a.shape[1] if k is None else k
    n = b.shape[1] if n is None else n
    f32 = a.dtype == np.float32
    poison = np.float32(np.nan) if f32 else np.int32(-2 ** 31)
    lda, ldb, ldc = k + pads[0], n + pads[1], n + pads[2]
    ah = np.full((max(m, 1), lda), poison, dtype=a.dtype)
    bh = np.full((max(k, 1), ldb), poison, dtype=a.dtype)
    ah[:m, :k] = a
    bh[:k, :n] = b
    da, db = torch.from_numpy(ah).cuda(), torch.from_numpy(bh).cuda()
    dc = torch.full((max(m, 1), ldc), GUARD, dtype=da.dtype, device="cuda")
    dt = ax.ACC_FLOAT32 if f32 else ax.ACC_INT32
    print("gemm dtype=%s m=%d n=%d k=%d ld=(%d,%d,%d) flags=%#x" % (a.dtype, m, n, k, lda, ldb, ldc, flags),
          flush=True)
    ax.accx_gemm_dev(dt, m, n, k, da, lda, db, ldb, dc, ldc, flags)
    torch.cuda.synchronize()
    c = dc.cpu().numpy()
    assert np.all(c[:, n:] == GUARD), "C padding written"
    if m == 0:
        assert np.all(c == GUARD)
    return c[:m, :n]


@pytest.mark.parametrize("kernel", F32_KERNELS)
@pytest.mark.parametrize("m,n,k", SHAPES)
def test_f32_parity(ax, m, n, k, kernel):
    a, b = _inputs(m, n, k, "f32")
    c = _gemm(ax, a, b, _flags(ax, kernel))
    err = rel_fro(c, oracle.gemm(a, b))
    print("m=%d n=%d k=%d %s rel_fro=%.3g" % (m, n, k, kernel, err))
    assert err <= FP32_REL_FRO_TOL


@pytest.mark.parametrize("kernel", I32_KERNELS)
@pytest.mark.parametrize("m,n,k", SHAPES)
@pytest.mark.parametrize("vals", ["i32small", "i32full"])
def test_i32_bit_exact(ax, m, n, k, kernel, vals):
    a, b = _inputs(m, n, k, vals)
    assert np.array_equal(_gemm(ax, a, b, _flags(ax, kernel)), oracle.gemm(a, b))


@pytest.mark.parametrize("tile", ["256", "256w4", "256x128", "128", "64"])
def test_forced_tiles(ax, tile):
    import paper_1412_1127_amd as pk
    m, n, k = 300, 200, 129
    a, b = _inputs(m, n, k, "f32", 21)
    fl = _flags(ax, "full6") | pk.TILES[tile]
    assert rel_fro(_gemm(ax, a, b, fl), oracle.gemm(a, b)) <= FP32_REL_FRO_TOL
    ai, bi = _inputs(m, n, k, "i32small", 23)
    assert np.array_equal(_gemm(ax, ai, bi, _flags(ax, "tiled") | ax.ACC_LIMBS(1) | pk.TILES[tile]),
                          oracle.gemm(ai, bi))


@pytest.mark.parametrize("tile", ["256", "128", "256w4", "64"])
@pytest.mark.parametrize("k", [1, 16, 32, 33, 64, 65, 96])
def test_forced_tiles_short_k(ax, tile, k):
    # bf16x3 K loops of two, four or six 16-element steps: the ends of the
    # look-ahead loops, where the read-ahead runs past the last stage; the
    # int8 tile's loop over one or two 64-element steps
    import paper_1412_1127_amd as pk
    m, n = 300, 270
    a, b = _inputs(m, n, k, "f32", 31)
    ref = oracle.gemm(a, b)
    for prec, tol in (("full6", FP32_REL_FRO_TOL), ("auto", FP32_REL_FRO_TOL), ("cheap3", 2.0 ** -12)):
        err = rel_fro(_gemm(ax, a, b, _flags(ax, prec) | pk.TILES[tile]), ref)
        assert err <= tol, (prec, err)
    ai, bi = _inputs(m, n, k, "i32small", 33)
    assert np.array_equal(_gemm(ax, ai, bi, _flags(ax, "tiled") | ax.ACC_LIMBS(1) | pk.TILES[tile]),
                          oracle.gemm(ai, bi))


@pytest.mark.parametrize("kernel", ["plain", "listing1b", "full6", "cheap3", "auto"])
def test_f32_leading_dimensions_do_not_change_the_result(ax, kernel):
    # padded rows (odd and multiple-of-4 strides) give the bits of tight rows
    m, n, k = 97, 131, 203
    a, b = _inputs(m, n, k, "f32", 31)
    tight = _gemm(ax, a, b, _flags(ax, kernel), pads=(0, 0, 0))
    for pads in [(3, 5, 2), (4, 8, 4), (1, 1, 64)]:
        assert np.array_equal(_gemm(ax, a, b, _flags(ax, kernel), pads=pads), tight)


@pytest.mark.parametrize("kernel", ["plain", "tiled"])
def test_i32_leading_dimensions_do_not_change_the_result(ax, kernel):
    m, n, k = 97, 131, 203
    a, b = _inputs(m, n, k, "i32full", 33)
    tight = _gemm(ax, a, b, _flags(ax, kernel), pads=(0, 0, 0))
    for pads in [(3, 5, 2), (4, 8, 4)]:
        assert np.array_equal(_gemm(ax, a, b, _flags(ax, kernel), pads=pads), tight)


@pytest.mark.parametrize("kernel", ["plain", "full6", "auto"])
def test_square_shape_matches_matmul_entry(ax, kernel):
    import torch
    n = 257
    a, b = _inputs(n, n, n, "f32", 41)
    da, db = torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()
    c1 = torch.empty((n, n), dtype=torch.float32, device="cuda")
    c2 = torch.empty((n, n), dtype=torch.float32, device="cuda")
    fl = _flags(ax, kernel)
    ax.accx_matmul_dev(ax.ACC_FLOAT32, da, db, c1, n, fl)
    ax.accx_gemm_dev(ax.ACC_FLOAT32, n, n, n, da, n, db, n, c2, n, fl)
    torch.cuda.synchronize()
    assert torch.equal(c1, c2)
    assert ax.accx_gemm_workspace_size(ax.ACC_FLOAT32, n, n, n, fl) == ax.accx_matmul_workspace_size(
        ax.ACC_FLOAT32, n, fl)


@pytest.mark.parametrize("kernel", ["plain", "listing1b", "full6", "auto", "tiled"])
def test_k_zero_sets_c_to_zero(ax, kernel):
    m, n = 70, 45
    for dt in (np.float32, np.int32):
        if kernel == "tiled" and dt == np.float32:
            continue
        if kernel in ("full6", "auto") and dt == np.int32:
            continue
        a = np.zeros((m, 0), dt)
        b = np.zeros((0, n), dt)
        c = _gemm(ax, a, b, _flags(ax, kernel))
        assert c.shape == (m, n) and np.all(c == 0)


@pytest.mark.parametrize("kernel", ["plain", "full6", "tiled"])
def test_empty_result_is_a_no_op(ax, kernel):
    for m, n in [(0, 5), (5, 0), (0, 0)]:
        k = 9
        dt = np.int32 if kernel == "tiled" else np.float32
        a = np.ones((m, k), dt)
        b = np.ones((k, n), dt)
        _gemm(ax, a, b, _flags(ax, kernel))  # guards checked inside


def test_region_gemm_on_padded_host_views(ax):
    m, n, k = 45, 70, 130
    lda, ldb, ldc = 133, 75, 72
    a, b = _inputs(m, n, k, "f32", 51)
    ah = np.full((m, lda), np.nan, np.float32)
    bh = np.full((k, ldb), np.nan, np.float32)
    ch = np.full((m, ldc), GUARD, np.float32)
    ah[:, :k] = a
    bh[:, :n] = b
    r = ax.acc_data_begin([ax.clause(ax.ACC_COPYIN, ax.ACC_FLOAT32, ah), ax.clause(ax.ACC_COPYIN, ax.ACC_FLOAT32, bh),
                           ax.clause(ax.ACC_COPY, ax.ACC_FLOAT32, ch)])
    ax.acc_loopnest_gemm(r, ax.ACC_FLOAT32, m, n, k, ah, lda, bh, ldb, ch, ldc, _flags(ax, "full6"))
    ax.acc_data_end(r)
    assert rel_fro(ch[:, :n], oracle.gemm(a, b)) <= FP32_REL_FRO_TOL
    assert np.all(ch[:, n:] == GUARD)


def test_region_gemm_span_must_be_mapped(ax):
    m, n, k = 8, 8, 8
    lda = 16
    ah = np.zeros((m, lda), np.float32)
    bh = np.zeros((k, n), np.float32)
    ch = np.zeros((m, n), np.float32)
    span = (m - 1) * lda + k  # elements from A's first to its last element
    r = ax.acc_data_begin([ax.clause(ax.ACC_COPYIN, ax.ACC_FLOAT32, ah, 0, span - 1),
                           ax.clause(ax.ACC_COPYIN, ax.ACC_FLOAT32, bh), ax.clause(ax.ACC_COPY, ax.ACC_FLOAT32, ch)])
    try:
        with pytest.raises(ax.AccxError) as e:
            ax.acc_loopnest_gemm(r, ax.ACC_FLOAT32, m, n, k, ah, lda, bh, n, ch, n, ax.ACC_KERNEL_PLAIN)
        assert e.value.status == ax.ACC_ERR_NOT_PRESENT
    finally:
        ax.acc_data_end(r)
    r = ax.acc_data_begin([ax.clause(ax.ACC_COPYIN, ax.ACC_FLOAT32, ah, 0, span),
                           ax.clause(ax.ACC_COPYIN, ax.ACC_FLOAT32, bh), ax.clause(ax.ACC_COPY, ax.ACC_FLOAT32, ch)])
    ax.acc_loopnest_gemm(r, ax.ACC_FLOAT32, m, n, k, ah, lda, bh, n, ch, n, ax.ACC_KERNEL_PLAIN)
    ax.acc_data_end(r)


def test_probe_records_on_rectangular_shape(ax):
    import torch
    m, n, k = 300, 700, 257
    a, b = _inputs(m, n, k, "f32", 61)
    fl = _flags(ax, "auto")
    ws = ax.accx_gemm_workspace_size(ax.ACC_FLOAT32, m, n, k, fl)
    off, cnt = ax.accx_gemm_probe_layout(m, n, k, fl)
    da, db = torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()
    dc = torch.empty((m, n), dtype=torch.float32, device="cuda")
    work = torch.zeros(ws, dtype=torch.uint8, device="cuda")
    ax.accx_gemm_dev(ax.ACC_FLOAT32, m, n, k, da, k, db, n, dc, n, fl, work, ws)
    torch.cuda.synchronize()
    assert rel_fro(dc.cpu().numpy(), oracle.gemm(a, b)) <= FP32_REL_FRO_TOL
    import ctypes
    size = ctypes.sizeof(ax.accx_probe_record)
    assert size == 608
    recs = ax.probe_records(work[off:off + cnt * size].cpu().numpy().tobytes(), cnt)
    assert len(recs) == cnt > 0
    ref = oracle.gemm(a, b)
    for r in recs:
        rows, cols = list(r.rows), list(r.cols)
        assert all(0 <= i < m for i in rows) and all(0 <= j < n for j in cols)
        want = np.array([ref[i, j] for i in rows for j in cols])
        assert np.allclose(np.array(list(r.ref)), want, rtol=1e-12, atol=1e-12)


def test_row_block_whole_block(ax):
    # one 512-row block of an 8192 x 4096 by 4096 x 4096 product (one GPU's
    # share of the LEN=4096 product over eight), against the oracle on the
    # whole block: float32 per 128 x 128 tile (no tile hides in a pooled
    # norm) and over the block, int32 bit-exact
    import torch
    m, n, k = 512, 4096, 4096
    a, b = _inputs(m, n, k, "f32", 72)
    ref = oracle.gemm(a, b)
    da, db = torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()
    for kernel in ("full6", "auto"):
        dc = torch.empty((m, n), dtype=torch.float32, device="cuda")
        print("row block m=%d n=%d k=%d %s" % (m, n, k, kernel), flush=True)
        ax.accx_gemm_dev(ax.ACC_FLOAT32, m, n, k, da, k, db, n, dc, n, _flags(ax, kernel))
        torch.cuda.synchronize()
        c = dc.cpu().numpy()
        assert rel_fro(c, ref) <= FP32_REL_FRO_TOL
        worst = max(rel_fro(c[i:i + 128, j:j + 128], ref[i:i + 128, j:j + 128])
                    for i in range(0, m, 128) for j in range(0, n, 128))
        assert worst <= FP32_REL_FRO_TOL, (kernel, worst)
    ai, bi = _inputs(m, n, k, "i32small", 74)
    refi = oracle.gemm(ai, bi)
    dai, dbi = torch.from_numpy(ai).cuda(), torch.from_numpy(bi).cuda()
    dci = torch.empty((m, n), dtype=torch.int32, device="cuda")
    ax.accx_gemm_dev(ax.ACC_INT32, m, n, k, dai, k, dbi, n, dci, n, _flags(ax, "tiled"))
    torch.cuda.synchronize()
    assert np.array_equal(dci.cpu().numpy(), refi)


@pytest.mark.parametrize("tile", [None, "256", "256w4", "128", "64"])
def test_split_k_long_inner_dimension(ax, tile):
    # few output tiles and a long K: the K loop of each tile is split over
    # several workgroups whose partial sums are added in part order
    import paper_1412_1127_amd as pk
    m, n, k = 256, 192, 8192
    a, b = _inputs(m, n, k, "f32", 81)
    fl = _flags(ax, "full6") | (pk.TILES[tile] if tile else 0)
    c1 = _gemm(ax, a, b, fl, pads=(0, 0, 0))
    assert rel_fro(c1, oracle.gemm(a, b)) <= FP32_REL_FRO_TOL
    assert np.array_equal(_gemm(ax, a, b, fl, pads=(0, 0, 0)), c1)     # same bits on every run
    ai, bi = _inputs(m, n, k, "i32small", 83)
    fi = _flags(ax, "tiled") | (pk.TILES[tile] if tile else 0)
    assert np.array_equal(_gemm(ax, ai, bi, fi), oracle.gemm(ai, bi))
    c3 = _gemm(ax, a, b, _flags(ax, "auto") | (pk.TILES[tile] if tile else 0))
    assert rel_fro(c3, oracle.gemm(a, b)) <= FP32_REL_FRO_TOL


@pytest.mark.parametrize("tile,m,n,k", [("256", 1792, 1792, 4096), ("256x128", 1536, 768, 4096),
                                         ("128", 250, 5500, 4096)])
def test_split_k_part_counts_off_the_load_group(ax, tile, m, n, k):
    # On a 256-CU GPU these shapes split K into 5, 7 and 5 parts (the 128 x
    # 128 tile fills two workgroup slots per CU: 86 ragged tiles, 5 parts):
    # the last part reads the parts back in groups of 4, 4 and 2, so the last
    # group is partly past the last part (those loads must not be added).
    # Checked on sampled rows against the oracle, and for the same bits on
    # every run.
    import torch

    import paper_1412_1127_amd as pk
    g = synth.rng(SEED, 87)
    rows = np.unique(np.concatenate([[0, m - 1], g.integers(0, m, 24)]))
    for dt in ("f32", "i32"):
        a, b = _inputs(m, n, k, "f32" if dt == "f32" else "i32small", 88)
        dtype = ax.ACC_FLOAT32 if dt == "f32" else ax.ACC_INT32
        fl = _flags(ax, "full6" if dt == "f32" else "tiled") | pk.TILES[tile]
        base = ax.accx_gemm_workspace_size(dtype, m, n, k, _flags(ax, "full6" if dt == "f32" else "tiled")
                                           | pk.TILES["64"])
        full = ax.accx_gemm_workspace_size(dtype, m, n, k, fl)
        assert full > base                                                     # this shape splits
        if torch.cuda.get_device_properties(0).multi_processor_count == 256:
            bm, bn = {"256": (256, 256), "256x128": (256, 128), "128": (128, 128)}[tile]
            tiles = -(-m // bm) * -(-n // bn)
            parts = (full - base - (256 + 4 * tiles + 255) // 256 * 256) // (tiles * bm * bn * 4)
            assert parts == {"256": 5, "256x128": 7, "128": 5}[tile], parts
        print("split K %s %s m=%d n=%d k=%d" % (tile, dt, m, n, k), flush=True)
        c1 = _gemm(ax, a, b, fl, pads=(0, 0, 0))
        ref = oracle.gemm(np.ascontiguousarray(a[rows]), b)
        if dt == "f32":
            assert rel_fro(c1[rows], ref) <= FP32_REL_FRO_TOL
        else:
            assert np.array_equal(c1[rows], ref)
        assert np.array_equal(_gemm(ax, a, b, fl, pads=(0, 0, 0)), c1)


def test_split_k_with_a_small_caller_workspace_runs_unsplit(ax):
    # a workspace that holds the operands but not the split area: no split
    import torch
    m, n, k = 128, 128, 4096
    a, b = _inputs(m, n, k, "f32", 85)
    fl = _flags(ax, "full6")
    full = ax.accx_gemm_workspace_size(ax.ACC_FLOAT32, m, n, k, fl)
    base = 2 * 4 * (-(-2 * k // 64)) * 3 * 2048                       # packed A and B^T
    assert full > base
    da, db = torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()
    c = torch.empty((m, n), device="cuda")
    w = torch.empty(base, dtype=torch.uint8, device="cuda")
    ax.accx_gemm_dev(ax.ACC_FLOAT32, m, n, k, da, k, db, n, c, n, fl, w, base)
    torch.cuda.synchronize()
    assert rel_fro(c.cpu().numpy(), oracle.gemm(a, b)) <= FP32_REL_FRO_TOL
    with pytest.raises(ax.AccxError):
        ax.accx_gemm_dev(ax.ACC_FLOAT32, m, n, k, da, k, db, n, c, n, fl, w, base - 256)
