"""One compute region with two independent nests -- the float32 matmul of
Listing 1a (section 1.3) and a reduction(+) (section 2.3) -- through
accx_matmul_reduce_dev: the matrix is bitwise the one accx_matmul_dev
computes with the same flags, and the sum is checked against the CPU
oracle, on the co-scheduled path (the sum inside the three-product pass's
launch) and on the sequential one."""
import numpy as np
import pytest

import oracle
import synth
from _util import SEED

pytestmark = pytest.mark.gpu

SUM_REL_TOL = 1e-5   # as the reduction tests: float32 sum vs the float64 oracle


@pytest.fixture(scope="module")
def ax():
    import paper_1412_1127_amd as ax
    ax.acc_init(0, 0)
    yield ax
    ax.acc_shutdown()


def _run(ax, len_, flags, n, init=0.25, offset=0, work="library", seed_stream=3):
    """Returns (C from accx_matmul_reduce_dev, C from accx_matmul_dev, the
    sum, the sum's oracle value, the kernel names timed during the call)."""
    import torch
    a = synth.uniform_pm1_f32((len_, len_), SEED, 41)
    b = synth.uniform_pm1_f32((len_, len_), SEED, 42)
    x = synth.uniform01_f32(n, SEED, seed_stream)
    da, db = torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()
    dc = torch.full((len_, len_), float("nan"), device="cuda")
    dc0 = torch.empty((len_, len_), device="cuda")
    buf = torch.zeros(n + offset + 4, dtype=torch.float32, device="cuda")
    if n:
        buf[offset:offset + n] = torch.from_numpy(x).cuda()
    res = torch.full((1,), float("nan"), device="cuda")
    wb = ax.accx_matmul_reduce_workspace_size(len_, flags, n)
    w = None
    if work == "caller":
        w = torch.randint(0, 255, (wb,), dtype=torch.uint8, device="cuda")   # any contents
    print("matmul+reduce len=%d flags=%#x n=%d offset=%d work=%s" % (len_, flags, n, offset, work), flush=True)
    ax.accx_timing_enable(True)
    ax.accx_timing_read(reset=True)
    ax.accx_matmul_reduce_dev(da, db, dc, len_, flags, buf.data_ptr() + 4 * offset, n, init, res,
                              w, wb if w is not None else 0)
    torch.cuda.synchronize()
    names = set(ax.accx_timing_read(reset=True))
    ax.accx_timing_enable(False)
    ax.accx_matmul_dev(ax.ACC_FLOAT32, da, db, dc0, len_, flags)
    torch.cuda.synchronize()
    return dc.cpu().numpy(), dc0.cpu().numpy(), float(res.item()), oracle.sum_f32(x, init), names


def _flags(ax, prec):
    return ax.ACC_KERNEL_TILED | {"auto": ax.ACC_PREC_AUTO, "cheap3": ax.ACC_PREC_CHEAP3,
                                  "full6": ax.ACC_PREC_FULL6}[prec]


@pytest.mark.parametrize("prec", ["auto", "cheap3"])
@pytest.mark.parametrize("n", [1 << 26, (1 << 20) + 3, 5, 0])
def test_co_scheduled_matches_separate_calls(ax, prec, n):
    # LEN=4096: the 256 x 256 three-product pass, which carries the sum (n up
    # to 2^26 floats fills every K-step's loads; a ragged n leaves a tail for
    # workgroup 0; n = 5 leaves most workgroups without a vector); n = 0 has
    # no array to carry and runs the empty reduction (init) after the matmul
    c, c0, got, ref, names = _run(ax, 4096, _flags(ax, prec), n)
    if n:
        # the fused path ran: no reduction kernel of its own; its last step
        # rides in the probe's launch (AUTO) or runs alone (CHEAP3)
        assert "reduce_fast" not in names and ("reduce_final" in names) == (prec == "cheap3")
    else:
        assert got == np.float32(0.25)
    assert np.array_equal(c, c0)
    assert abs(got - ref) <= SUM_REL_TOL * abs(ref)


@pytest.mark.parametrize("len_,prec,offset", [(300, "auto", 0), (4096, "full6", 0), (4096, "auto", 1),
                                              (4096, "cheap3", 2)])
def test_sequential_when_the_pass_cannot_carry_the_sum(ax, len_, prec, offset):
    # a small matmul (64 x 64 tiles), six products, or a sum that does not
    # start on a 16-byte boundary: the two nests run one after the other
    n = (1 << 22) + 1
    c, c0, got, ref, names = _run(ax, len_, _flags(ax, prec), n, offset=offset)
    assert "reduce_fast" in names and "reduce_final" not in names
    assert np.array_equal(c, c0)
    assert abs(got - ref) <= SUM_REL_TOL * abs(ref)


def test_co_scheduled_on_a_ragged_matrix(ax):
    # LEN=4000: still one 256 x 256 tile per CU (16 x 16 tiles, the last row
    # and column of tiles ragged), so the sum rides in the pass; an odd n
    # leaves a tail of three floats
    n = (1 << 23) + 3
    c, c0, got, ref, names = _run(ax, 4000, _flags(ax, "auto"), n)
    assert "reduce_fast" not in names
    assert np.array_equal(c, c0)
    assert abs(got - ref) <= SUM_REL_TOL * abs(ref)


def test_sum_beyond_the_pass_capacity_runs_apart(ax):
    # the LEN=4096 pass carries at most 2^28 floats (two 16-byte loads per
    # thread per K-step); one vector more and the sum runs on its own
    import torch
    x = torch.ones((1 << 28) + 4, device="cuda")
    a = torch.zeros((4096, 4096), device="cuda")
    c = torch.empty_like(a)
    res = torch.empty(1, device="cuda")
    for n, fused in (((1 << 28), True), ((1 << 28) + 4, False)):
        ax.accx_timing_enable(True)
        ax.accx_timing_read(reset=True)
        ax.accx_matmul_reduce_dev(a, a, c, 4096, _flags(ax, "auto"), x, n, 0.0, res)
        torch.cuda.synchronize()
        names = set(ax.accx_timing_read(reset=True))
        ax.accx_timing_enable(False)
        assert ("reduce_fast" not in names) == fused, (n, names)
        # ones: every partial sum is exact up to the float32 spacing of the
        # total (32 at 2^28), so the result is n to that spacing
        assert abs(res.item() - n) <= 32.0, (n, res.item())
        assert not c.any().item()


def test_caller_workspace_and_repeatable(ax):
    n = (1 << 24) + 7
    fl = _flags(ax, "auto")
    c1, c0, s1, ref, _ = _run(ax, 4096, fl, n, work="caller")
    c2, _, s2, _, _ = _run(ax, 4096, fl, n, work="caller")
    assert np.array_equal(c1, c0) and np.array_equal(c2, c0)
    assert s1 == s2                                                       # same bits on every call
    assert abs(s1 - ref) <= SUM_REL_TOL * abs(ref)


def test_exact_sum_of_integers(ax):
    # x_k = k mod 16 (integers) over 2^20 elements: the total, 7864320, is
    # below 2^24, so every partial sum is an integer below 2^24 and exact in
    # any order: the co-scheduled sum equals the closed form
    import torch
    n = 1 << 20
    x = (np.arange(n) % 16).astype(np.float32)
    a = torch.zeros((4096, 4096), device="cuda")
    c = torch.empty_like(a)
    dx = torch.from_numpy(x).cuda()
    res = torch.empty(1, device="cuda")
    ax.accx_matmul_reduce_dev(a, a, c, 4096, _flags(ax, "auto"), dx, n, 0.0, res)
    torch.cuda.synchronize()
    assert res.item() == float((n // 16) * 120)
    assert not c.any().item()


def test_argument_errors(ax):
    import torch
    a = torch.zeros((64, 64), device="cuda")
    r = torch.empty(1, device="cuda")
    fl = _flags(ax, "auto")
    with pytest.raises(ax.AccxError):
        ax.accx_matmul_reduce_dev(a, a, a, 64, fl, a, -1, 0.0, r)
    with pytest.raises(ax.AccxError):
        ax.accx_matmul_reduce_dev(a, a, a, 64, fl, None, 16, 0.0, r)
    wb = ax.accx_matmul_reduce_workspace_size(64, fl, 16)
    w = torch.empty(wb, dtype=torch.uint8, device="cuda")
    with pytest.raises(ax.AccxError):
        ax.accx_matmul_reduce_dev(a, a, a, 64, fl, a, 16, 0.0, r, w, wb - 1)


def test_caller_workspace_must_be_256_byte_aligned(ax):
    # the entry points that take a caller's workspace reject one whose start
    # is not 256-byte aligned, before anything is launched
    import torch
    a = torch.zeros((256, 256), device="cuda")
    c = torch.empty_like(a)
    r = torch.empty(1, device="cuda")
    fl = _flags(ax, "auto")
    wb = ax.accx_matmul_reduce_workspace_size(256, fl, 1024)
    w = torch.empty(wb + 256, dtype=torch.uint8, device="cuda")
    assert w.data_ptr() % 256 == 0
    off = w.data_ptr() + 16
    with pytest.raises(ax.AccxError, match="256-byte"):
        ax.accx_matmul_reduce_dev(a, a, c, 256, fl, a, 1024, 0.0, r, off, wb)
    with pytest.raises(ax.AccxError, match="256-byte"):
        ax.accx_matmul_dev(ax.ACC_FLOAT32, a, a, c, 256, fl, off, wb)
    with pytest.raises(ax.AccxError, match="256-byte"):
        ax.accx_reduce_sum_dev(ax.ACC_FLOAT32, a, 1024, 0.0, r, 0, off, wb)
    # the aligned start of the same buffer works
    ax.accx_matmul_reduce_dev(a, a, c, 256, fl, a, 1024, 0.0, r, w, wb)
    torch.cuda.synchronize()
    assert r.item() == 0.0 and not c.any().item()
