"""Parity of the LDS-tiled matrix-core loop nest (bf16x3 for float32, int8
limbs for int32) with the CPU oracle and with the plain kernel."""
import numpy as np
import pytest

import oracle
import synth
from _util import FP32_REL_FRO_TOL, SEED, rel_fro, sample_entries

pytestmark = pytest.mark.gpu

SIZES = [1, 2, 31, 32, 33, 64, 100, 128, 255, 256, 257, 300, 513, 640, 1000]


@pytest.fixture(scope="module")
def ax():
    import paper_1412_1127_amd as ax
    ax.acc_init(0, 0)
    yield ax
    ax.acc_shutdown()


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


def _tiled(ax, prec=None):
    return ax.ACC_KERNEL_TILED | (ax.ACC_PREC_FULL6 if prec is None else prec)


@pytest.mark.parametrize("n", SIZES)
def test_f32_full6_parity(ax, n):
    a = synth.uniform_pm1_f32((n, n), SEED, synth.STREAM_A)
    b = synth.uniform_pm1_f32((n, n), SEED, synth.STREAM_B)
    c = _run(ax, a, b, _tiled(ax))
    err = rel_fro(c, oracle.matmul_f32(a, b))
    print("LEN=%d FULL6 rel_fro=%.3g" % (n, err))
    assert err <= FP32_REL_FRO_TOL


@pytest.mark.parametrize("n", [33, 256, 1000])
def test_f32_cheap3_error_is_bf16_scale(ax, n):
    # Three products drop terms of relative size ~2^-16; the error is stated,
    # not held to the float32 bound.
    a = synth.uniform_pm1_f32((n, n), SEED, synth.STREAM_A)
    b = synth.uniform_pm1_f32((n, n), SEED, synth.STREAM_B)
    err = rel_fro(_run(ax, a, b, _tiled(ax, ax.ACC_PREC_CHEAP3)), oracle.matmul_f32(a, b))
    print("LEN=%d CHEAP3 rel_fro=%.3g" % (n, err))
    assert err <= 2.0 ** -12


@pytest.mark.parametrize("n", [33, 256, 1000])
def test_f32_five_products(ax, n):
    # FULL6 without mid*mid: within the float32 bound, and between FULL6 and
    # CHEAP3 in error (the dropped term is second order: |mid*mid| <= 2^-16 |a||b|)
    a = synth.uniform_pm1_f32((n, n), SEED, synth.STREAM_A)
    b = synth.uniform_pm1_f32((n, n), SEED, synth.STREAM_B)
    ref = oracle.matmul_f32(a, b)
    e5 = rel_fro(_run(ax, a, b, _tiled(ax, ax.ACC_PREC_FIVE)), ref)
    e6 = rel_fro(_run(ax, a, b, _tiled(ax, ax.ACC_PREC_FULL6)), ref)
    e3 = rel_fro(_run(ax, a, b, _tiled(ax, ax.ACC_PREC_CHEAP3)), ref)
    print("LEN=%d FULL6 %.3g FIVE %.3g CHEAP3 %.3g" % (n, e6, e5, e3))
    assert e5 <= FP32_REL_FRO_TOL
    assert e6 <= e5 <= e3


@pytest.mark.parametrize("prec", ["FULL6", "FIVE", "CHEAP3"])
def test_identity_ones_exact(ax, prec):
    p = getattr(ax, "ACC_PREC_" + prec)
    n = 160
    a = synth.uniform_pm1_f32((n, n), SEED, 5)
    eye = np.eye(n, dtype=np.float32)
    if prec in ("FULL6", "FIVE"):   # hi + mid + lo == a exactly, and 1 * term is exact
        assert np.array_equal(_run(ax, eye, a, _tiled(ax, p)), a)
        assert np.array_equal(_run(ax, a, eye, _tiled(ax, p)), a)
    one = np.ones((n, n), np.float32)
    assert np.all(_run(ax, one, one, _tiled(ax, p)) == n)


@pytest.mark.parametrize("prec", ["FULL6", "CHEAP3"])
def test_integer_valued_floats_bitwise_equal_int(ax, prec):
    # |C| <= LEN*256 < 2^24: every partial sum is exact on every path.
    n = 512
    ai = synth.int_uniform_i32((n, n), -16, 16, SEED, synth.STREAM_A)
    bi = synth.int_uniform_i32((n, n), -16, 16, SEED, synth.STREAM_B)
    cf = _run(ax, ai.astype(np.float32), bi.astype(np.float32), _tiled(ax, getattr(ax, "ACC_PREC_" + prec)))
    assert np.array_equal(cf, oracle.matmul_i32(ai, bi).astype(np.float32))


LIMB_RANGES = {1: 127, 2: 32639, 3: 8355711, 4: None}


@pytest.mark.parametrize("limbs", [1, 2, 3, 4])
@pytest.mark.parametrize("n", [1, 33, 64, 200, 257, 512])
def test_i32_bit_exact_probe(ax, limbs, n):
    bound = LIMB_RANGES[limbs]
    if bound is None:
        a = synth.full_range_i32((n, n), SEED, synth.STREAM_A)
        b = synth.full_range_i32((n, n), SEED, synth.STREAM_B)
    else:
        a = synth.int_uniform_i32((n, n), -bound, bound, SEED, synth.STREAM_A)
        b = synth.int_uniform_i32((n, n), -bound, bound, SEED, synth.STREAM_B)
        a.flat[0] = bound  # the probe must see the extreme
    ref = oracle.matmul_i32(a, b)
    assert np.array_equal(_run(ax, a, b, ax.ACC_KERNEL_TILED), ref)          # limb count by probe
    assert np.array_equal(_run(ax, a, b, ax.ACC_KERNEL_TILED | ax.ACC_LIMBS(4)), ref)  # forced 4
    assert np.array_equal(_run(ax, a, b, ax.ACC_KERNEL_TILED | ax.ACC_LIMBS(limbs)), ref)


# The device picks the digit count from max |x|: one digit holds [-128, 127]
# (taken for |x| <= 127), two [-32896, 32639], three [-8421504, 8355711].
# One element at each side of each threshold, in A or in B, on small values
# elsewhere; 130 = two 128-row tiles of the multi-digit kernel plus a ragged one.
@pytest.mark.parametrize("v", [127, -127, 128, -128, 32639, 32640, -32896, -32897, 8355711, 8355712, -8421504,
                               -8421505, 2 ** 31 - 1, -(2 ** 31)])
@pytest.mark.parametrize("where", ["a", "b"])
def test_i32_digit_count_thresholds(ax, v, where):
    n = 130
    a = synth.int_uniform_i32((n, n), -100, 100, SEED, synth.STREAM_A)
    b = synth.int_uniform_i32((n, n), -100, 100, SEED, synth.STREAM_B)
    (a if where == "a" else b)[n - 1, 57] = v
    assert np.array_equal(_run(ax, a, b, ax.ACC_KERNEL_TILED), oracle.matmul_i32(a, b))


# More output tiles than the multi-digit kernel has workgroups (one per CU):
# every workgroup takes several tiles in turn.
@pytest.mark.parametrize("bound", [32639, 8355711, None])
def test_i32_multi_digit_many_tiles(ax, bound):
    n = 2100
    if bound is None:
        a = synth.full_range_i32((n, n), SEED, 41)
        b = synth.full_range_i32((n, n), SEED, 42)
    else:
        a = synth.int_uniform_i32((n, n), -bound, bound, SEED, 41)
        b = synth.int_uniform_i32((n, n), -bound, bound, SEED, 42)
    ref = oracle.matmul_i32(a, b)
    assert np.array_equal(_run(ax, a, b, ax.ACC_KERNEL_TILED), ref)
    if bound is not None:
        limbs = 2 if bound == 32639 else 3
        assert np.array_equal(_run(ax, a, b, ax.ACC_KERNEL_TILED | ax.ACC_LIMBS(limbs)), ref)


def test_i32_digit_decision_with_reused_and_garbage_workspace(ax):
    # the max|x| words in the workspace are never cleared: a call must not
    # read an earlier call's maxima, nor whatever a workspace held, as its own
    import torch
    n = 300
    small = [synth.int_uniform_i32((n, n), -100, 100, SEED, 61 + k) for k in range(2)]
    big = [synth.full_range_i32((n, n), SEED, 63 + k) for k in range(2)]
    mid = [synth.int_uniform_i32((n, n), -30000, 30000, SEED, 65 + k) for k in range(2)]
    nbytes = ax.accx_matmul_workspace_size(ax.ACC_INT32, n, ax.ACC_KERNEL_TILED)
    w = torch.full((nbytes,), 0xFF, dtype=torch.uint8, device="cuda")
    g = synth.rng(SEED, 67)
    for k, (a, b) in enumerate([small, big, small, mid, small, big]):
        if k == 4:
            w.copy_(torch.from_numpy(g.integers(0, 256, nbytes).astype(np.uint8)).cuda())
        da, db = torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()
        dc = torch.full((n, n), -7, dtype=torch.int32, device="cuda")
        print("int32 auto with a reused workspace, call %d" % k, flush=True)
        ax.accx_matmul_dev(ax.ACC_INT32, da, db, dc, n, ax.ACC_KERNEL_TILED, w, nbytes)
        torch.cuda.synchronize()
        assert np.array_equal(dc.cpu().numpy(), oracle.matmul_i32(a, b)), k


# On the 256 x 256 one-digit tile the automatic path is one launch that runs
# the one-digit tile or, for larger data, the multi-digit product on the same
# workgroups (more of them than one-digit tiles at these sizes, split K at
# 1100); both branches, bit-exact.
@pytest.mark.parametrize("n", [300, 1100])
@pytest.mark.parametrize("kind", ["one", "two", "full"])
def test_i32_auto_on_256_tile(ax, n, kind):
    if kind == "full":
        a, b = synth.full_range_i32((n, n), SEED, 71), synth.full_range_i32((n, n), SEED, 72)
    else:
        bound = 100 if kind == "one" else 30000
        a = synth.int_uniform_i32((n, n), -bound, bound, SEED, 71)
        b = synth.int_uniform_i32((n, n), -bound, bound, SEED, 72)
    assert np.array_equal(_run(ax, a, b, ax.ACC_KERNEL_TILED | ax.ACC_TILE_256), oracle.matmul_i32(a, b))


def test_i32_wraparound(ax):
    n = 48
    a = np.full((n, n), 2 ** 31 - 1, np.int32)
    b = np.full((n, n), -(2 ** 31), np.int32)
    a[::3] = -(2 ** 31)
    assert np.array_equal(_run(ax, a, b, ax.ACC_KERNEL_TILED), oracle.matmul_i32(a, b))


def test_deterministic(ax):
    n = 777
    a = synth.uniform_pm1_f32((n, n), SEED, 7)
    b = synth.uniform_pm1_f32((n, n), SEED, 8)
    c1 = _run(ax, a, b, _tiled(ax))
    c2 = _run(ax, a, b, _tiled(ax))
    assert np.array_equal(c1, c2)


def test_scale_4096_vs_oracle_and_plain(ax):
    # The plain-method-at-scale workload: LEN = 4096, float32 uniform[-1,1]
    # and int32 in [-16,16]; sampled entries vs the oracle, the whole matrix
    # vs the plain kernel.
    n = 4096
    a = synth.uniform_pm1_f32((n, n), SEED, synth.STREAM_A)
    b = synth.uniform_pm1_f32((n, n), SEED, synth.STREAM_B)
    ct = _run(ax, a, b, _tiled(ax))
    cp = _run(ax, a, b, ax.ACC_KERNEL_PLAIN)
    ii, jj = sample_entries(n, 512)
    ref = oracle.matmul_at(a, b, ii, jj)
    e_or, e_pl = rel_fro(ct[ii, jj], ref), rel_fro(ct, cp)
    print("LEN=4096 FULL6 rel_fro vs oracle(sampled)=%.3g vs plain=%.3g plain-vs-oracle=%.3g"
          % (e_or, e_pl, rel_fro(cp[ii, jj], ref)))
    assert e_or <= FP32_REL_FRO_TOL and e_pl <= FP32_REL_FRO_TOL
    ai = synth.int_uniform_i32((n, n), -16, 16, SEED, synth.STREAM_A)
    bi = synth.int_uniform_i32((n, n), -16, 16, SEED, synth.STREAM_B)
    ci = _run(ax, ai, bi, ax.ACC_KERNEL_TILED)
    assert np.array_equal(ci[ii, jj], oracle.matmul_at(ai, bi, ii, jj))
    assert np.array_equal(ci, _run(ax, ai, bi, ax.ACC_KERNEL_PLAIN))


def test_precision_8192_rowscaled(ax):
    # The precision workload: LEN = 8192, N(0,1) * 2^U(-8,8) per row.
    n = 8192
    a = synth.normal_rowscaled_f32(n, n, SEED, synth.STREAM_A)
    b = synth.normal_rowscaled_f32(n, n, SEED, synth.STREAM_B)
    c = _run(ax, a, b, _tiled(ax))
    ii, jj = sample_entries(n, 1024)
    err = rel_fro(c[ii, jj], oracle.matmul_at(a, b, ii, jj))
    print("LEN=8192 rowscaled FULL6 rel_fro(sampled)=%.3g" % err)
    assert err <= FP32_REL_FRO_TOL


@pytest.mark.parametrize("tile", ["256", "256x128", "128", "64", "256w4"])
@pytest.mark.parametrize("n", [100, 257, 1000])
def test_every_tile_config(ax, tile, n):
    t = ax.TILES[tile]
    a = synth.uniform_pm1_f32((n, n), SEED, synth.STREAM_A)
    b = synth.uniform_pm1_f32((n, n), SEED, synth.STREAM_B)
    c = _run(ax, a, b, _tiled(ax) | t)
    assert rel_fro(c, oracle.matmul_f32(a, b)) <= FP32_REL_FRO_TOL
    ai = synth.int_uniform_i32((n, n), -16, 16, SEED, synth.STREAM_A)
    bi = synth.int_uniform_i32((n, n), -16, 16, SEED, synth.STREAM_B)
    assert np.array_equal(_run(ax, ai, bi, ax.ACC_KERNEL_TILED | t), oracle.matmul_i32(ai, bi))


def test_autotune_then_auto_uses_it(ax, tmp_path):
    n = 640
    tile, ms = ax.accx_autotune(ax.ACC_FLOAT32, n, ax.ACC_PREC_FULL6)
    assert tile in ax.TILES.values() and ms > 0
    a = synth.uniform_pm1_f32((n, n), SEED, 1)
    b = synth.uniform_pm1_f32((n, n), SEED, 2)
    auto = _run(ax, a, b, _tiled(ax))
    forced = _run(ax, a, b, _tiled(ax) | tile)
    assert np.array_equal(auto, forced)
    ti, _ = ax.accx_autotune(ax.ACC_INT32, n, ax.ACC_LIMBS(1))
    assert ti in ax.TILES.values()
    p = tmp_path / "tune.txt"
    ax.accx_tune_save(str(p))
    lines = p.read_text().split("\n")
    assert any(l.startswith("0 6 10 ") for l in lines)
    ax.accx_tune_load(str(p))
