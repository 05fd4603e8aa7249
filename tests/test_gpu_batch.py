"""The batched launch: many float32 loop-nest matmuls and reductions in one
graph of a packing kernel and a persistent work-queue kernel, against the
oracle, against the standalone kernels, and graph against eager."""
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


class Batch:
    """Seeded inputs on the device, the batch items, and host copies."""

    def __init__(self, ax, lens, ns, seed, tile=0, offsets=None, flags=0, gen=None):
        import torch
        self.ax = ax
        self.mats, self.reds = [], []
        items = []
        for k, n in enumerate(lens):
            if gen is not None and gen(k) is not None:
                a, b = gen(k)(n, seed, 1000 + 2 * k), gen(k)(n, seed, 1001 + 2 * k)
            else:
                a = synth.uniform_pm1_f32((n, n), seed, 1000 + 2 * k)
                b = synth.uniform_pm1_f32((n, n), seed, 1001 + 2 * k)
            da, db = torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()
            dc = torch.full((n, n), float("nan"), device="cuda")
            self.mats.append((a, b, da, db, dc, n))
            items.append(ax.batch_matmul(da, db, dc, n, tile))
        for k, n in enumerate(ns):
            off = offsets[k] if offsets else 0
            x = synth.uniform01_f32(n, seed, 5000 + k)
            buf = torch.zeros(n + off + 1, device="cuda")
            buf[off:off + n] = torch.from_numpy(x).cuda()
            res = torch.full((1,), float("nan"), device="cuda")
            init = 0.25 * k
            self.reds.append((x, buf, res, n, init))
            items.append(ax.batch_reduce(buf.data_ptr() + 4 * off, n, res, init))
        print("batch: %d matmuls, %d reductions, flags %#x" % (len(lens), len(ns), flags), flush=True)
        self.handle = ax.accx_batch_create(items, flags)

    def outputs(self):
        import torch
        torch.cuda.synchronize()
        return [m[4].cpu().numpy() for m in self.mats], [float(r[2].item()) for r in self.reds]

    def close(self):
        self.ax.accx_batch_destroy(self.handle)


def test_small_batch_parity(ax):
    g = synth.rng(SEED, 1)
    lens = [64, 100, 128, 257, 300, 511, 512, 640, 1000, 1, 33] + list(g.choice([64 * k for k in range(1, 9)], 9))
    # around the reduction's work-unit size (2^17 elements): one element
    # short, exact, one over, several units with a ragged last one
    ns = [0, 1, 5, 1000, (1 << 16) + 3, (1 << 17) - 1, 1 << 18, (1 << 18) + 1, 3 * (1 << 18) + 7]
    bt = Batch(ax, lens, ns, SEED, offsets=[0, 1, 2, 3, 1, 2, 0, 2, 3])
    ax.accx_batch_launch(bt.handle)
    cs, rs = bt.outputs()
    info = ax.accx_batch_info(bt.handle)
    print(info)
    assert info["matmuls"] == len(lens) and info["reductions"] == len(ns) and info["graph_nodes"] == 2
    for (a, b, *_r, n), c in zip(bt.mats, cs):
        assert rel_fro(c, oracle.matmul_f32(a, b)) <= FP32_REL_FRO_TOL, n
    for (x, _b, _r, n, init), got in zip(bt.reds, rs):
        ref = oracle.sum_f32(x, init)
        assert abs(got - ref) <= 1e-5 * max(abs(ref), 1e-30) or (n == 0 and got == init), (n, got, ref)
    bt.close()


def test_batch_matmul_bitwise_equals_standalone(ax):
    import torch
    lens = [96, 256, 700]
    for tile in (ax.ACC_TILE_128, ax.ACC_TILE_64):
        bt = Batch(ax, lens, [1000], SEED + 1, tile=tile)
        ax.accx_batch_launch(bt.handle)
        cs, _ = bt.outputs()
        for (a, b, da, db, dc, n), c in zip(bt.mats, cs):
            solo = torch.empty_like(dc)
            # a workspace holding just the packed operands: the standalone call
            # runs unsplit (one workgroup per tile, fixed K order), as the batch does
            base = 2 * ax.accx_packed_size(ax.ACC_FLOAT32, n, n, 3)
            w = torch.empty(base, dtype=torch.uint8, device="cuda")
            ax.accx_matmul_dev(ax.ACC_FLOAT32, da, db, solo, n, ax.ACC_KERNEL_TILED | ax.ACC_PREC_FULL6 | tile, w,
                               base)
            torch.cuda.synchronize()
            assert np.array_equal(c, solo.cpu().numpy()), (tile, n)
        bt.close()


def _biased_split(n, seed, stream):
    # x = h + m + l, each on its own bf16 grid and all positive: the three
    # products the cheap pass drops add up instead of cancelling (2.3e-5
    # relative error without the correction)
    g = synth.rng(seed, stream)
    h = 1.0 + g.integers(0, 16, (n, n)) * 2.0 ** -7
    m = 2.0 ** -9 * (1.0 + g.integers(64, 128, (n, n)) * 2.0 ** -7)
    l = 2.0 ** -18 * (1.0 + g.integers(16, 32, (n, n)) * 2.0 ** -5)
    return (h + m + l).astype(np.float32)


def _low_precision(n, seed, stream):
    # 8-bit significands: one bf16 term per input, the cheap pass is exact
    g = synth.rng(seed, stream)
    return (g.integers(-128, 128, (n, n)) * 2.0 ** -7).astype(np.float32)


def _auto_gen(k):
    return [None, _biased_split, _low_precision][k % 3]


def test_auto_batch_bitwise_equals_standalone_auto(ax):
    import torch
    lens = [96, 256, 700, 130, 512, 64]
    for tile in (ax.ACC_TILE_128, ax.ACC_TILE_64):
        bt = Batch(ax, lens, [1000], SEED + 5, tile=tile, flags=ax.ACC_BATCH_PREC_AUTO, gen=_auto_gen)
        ax.accx_batch_launch(bt.handle)
        cs, _ = bt.outputs()
        for k, ((a, b, da, db, dc, n), c) in enumerate(zip(bt.mats, cs)):
            solo = torch.empty_like(dc)
            # the packed operands and the probe records, no split area: the
            # standalone AUTO call runs unsplit, as the batch does
            flags = ax.ACC_KERNEL_TILED | ax.ACC_PREC_AUTO | tile
            off, _cnt = ax.accx_probe_layout(n, flags)
            _o, cnt64 = ax.accx_probe_layout(n, ax.ACC_KERNEL_TILED | ax.ACC_PREC_AUTO | ax.ACC_TILE_64)
            base = off + cnt64 * 608
            w = torch.empty(base, dtype=torch.uint8, device="cuda")
            ax.accx_matmul_dev(ax.ACC_FLOAT32, da, db, solo, n, flags, w, base)
            torch.cuda.synchronize()
            assert np.array_equal(c, solo.cpu().numpy()), (tile, n, k)
            assert rel_fro(c, oracle.matmul_f32(a, b)) <= FP32_REL_FRO_TOL, (tile, n, k)
        bt.close()


def test_auto_batch_corrects_and_replays(ax):
    # every third matmul has biased-split inputs (the cheap pass alone is
    # off by about 2.3e-5): only the per-tile probe and correction bring it
    # within the bound; graph replays equal the eager launch
    import torch
    g = synth.rng(SEED, 12)
    lens = [int(v) for v in g.choice([64 * k for k in range(1, 12)], 18)]
    ns = [int(v) for v in g.integers(1 << 10, 1 << 20, 6)]
    bt = Batch(ax, lens, ns, SEED + 6, flags=ax.ACC_BATCH_PREC_AUTO | ax.ACC_BATCH_AUTOTUNE, gen=_auto_gen)
    ax.accx_batch_launch_eager(bt.handle)
    ref_c, ref_r = bt.outputs()
    for k, ((a, b, *_r, n), c) in enumerate(zip(bt.mats, ref_c)):
        assert rel_fro(c, oracle.matmul_f32(a, b)) <= FP32_REL_FRO_TOL, (k, n)
    for (x, _b, _r, n, init), got in zip(bt.reds, ref_r):
        ref = oracle.sum_f32(x, init)
        assert abs(got - ref) <= 1e-5 * abs(ref), (n, got, ref)
    for rep in range(2):
        for m in bt.mats:
            m[4].fill_(float("nan"))
        (torch.randn(1 << 20, device="cuda") * 2).sum().item()
        ax.accx_batch_launch(bt.handle)
        cs, rs = bt.outputs()
        assert all(np.array_equal(x, y) for x, y in zip(cs, ref_c)), rep
        assert rs == ref_r, rep
    info = ax.accx_batch_info(bt.handle)
    assert info["mfma_flops"] == 3 * info["flops"]
    bt.close()


def test_graph_replays_equal_eager(ax):
    import torch
    g = synth.rng(SEED, 2)
    lens = list(g.choice([64 * k for k in range(1, 11)], 16))
    ns = list(g.integers(1 << 10, 1 << 20, 8))
    bt = Batch(ax, lens, ns, SEED + 2)
    ax.accx_batch_launch_eager(bt.handle)
    ref_c, ref_r = bt.outputs()
    for rep in range(3):
        for m in bt.mats:
            m[4].fill_(float("nan"))
        for r in bt.reds:
            r[2].fill_(float("nan"))
        # unrelated eager work between replays
        junk = torch.randn(1 << 20, device="cuda")
        (junk * 2).sum().item()
        ax.accx_batch_launch(bt.handle)
        cs, rs = bt.outputs()
        assert all(np.array_equal(x, y) for x, y in zip(cs, ref_c)), rep
        assert rs == ref_r, rep
    bt.close()


def test_closed_form_reductions_exact(ax):
    import torch
    ns = [1, 4, 255, 5792, 300000]
    xs = [torch.arange(1, n + 1, dtype=torch.float32, device="cuda") for n in ns[:4]]
    xs.append(torch.ones(ns[4], device="cuda"))
    res = torch.zeros(len(ns), device="cuda")
    items = [ax.batch_reduce(x, x.numel(), res[k:k + 1]) for k, x in enumerate(xs)]
    b = ax.accx_batch_create(items)
    ax.accx_batch_launch(b)
    torch.cuda.synchronize()
    got = res.cpu().numpy()
    want = [n * (n + 1) // 2 for n in ns[:4]] + [ns[4]]
    assert list(got) == [float(w) for w in want]
    ax.accx_batch_destroy(b)


def test_batch_rejects_bad_items(ax):
    import torch
    x = torch.zeros(64 * 64, device="cuda")
    with pytest.raises(ax.AccxError):
        ax.accx_batch_create([ax.batch_matmul(x, x, x, 0)])
    with pytest.raises(ax.AccxError):
        ax.accx_batch_create([ax.batch_matmul(x, x, x, 64, ax.ACC_TILE_256)])
    bad = ax.batch_reduce(x, 10, x)
    bad.dtype = ax.ACC_INT32
    with pytest.raises(ax.AccxError):
        ax.accx_batch_create([bad])
    with pytest.raises(ax.AccxError):
        ax.accx_batch_create([])


def test_batching_workload_per_item(ax):
    # The batching workload: 512 float32 matmuls, LEN uniform over
    # {64, 128, ..., 1024}, and 256 reductions, n log-uniform in [2^16, 2^24].
    # Every matmul is held to the bound on its own: the whole matrix up to
    # LEN = 512, otherwise 64+ entries touching every 64 x 64 tile row and
    # column (the finest tiling a batch runs).
    lens = synth.lens_uniform(512, [64 * k for k in range(1, 17)], SEED)
    ns = synth.log_uniform_int(256, 1 << 16, 1 << 24, SEED, synth.STREAM_X)
    bt = Batch(ax, list(lens), list(ns), SEED)
    info = ax.accx_batch_info(bt.handle)
    print(info, flush=True)
    ax.accx_batch_launch(bt.handle)
    cs, rs = bt.outputs()
    worst = 0.0
    for q, ((a, b, *_r, n), c) in enumerate(zip(bt.mats, cs)):
        assert np.isfinite(c).all(), q
        if n <= 512:
            err = rel_fro(c, oracle.matmul_f32(a, b))
        else:
            ii, jj = tile_samples(n, n, 64, 64, 64, stream=300 + q)
            err = rel_fro(c[ii, jj], oracle.matmul_at(a, b, ii, jj))
        worst = max(worst, err)
        assert err <= FP32_REL_FRO_TOL, (q, n, err)
    print("worst per-matmul rel_fro %.3g" % worst)
    for (x, _b, _r, n, init), got in zip(bt.reds, rs):
        ref = oracle.sum_f32(x, init)
        assert abs(got - ref) / ref <= 1e-5, (n, got, ref)
    bt.close()
