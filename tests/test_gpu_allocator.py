"""Device memory from the caller (accx_set_allocator; the memory-allocation
data function of section 2.3's data-clause step): region arrays, library
workspaces, batch and serving memory come from torch's caching allocator,
results still match the oracle, and every block goes back when the library
is done with it."""
import numpy as np
import pytest

import oracle
import synth
from _util import FP32_REL_FRO_TOL, SEED, rel_fro

pytestmark = pytest.mark.gpu


def test_everything_through_torch_allocator():
    import torch

    import paper_1412_1127_amd as ax
    ax.acc_init(0, 0)
    talloc = ax.TorchAllocator().install()
    try:
        # data region: copyin a, b; copyout c; AUTO tiled matmul (workspace)
        n = 700
        a = synth.uniform_pm1_f32((n, n), SEED, 601)
        b = synth.uniform_pm1_f32((n, n), SEED, 602)
        c = np.zeros((n, n), np.float32)
        r = ax.acc_data_begin([ax.clause(ax.ACC_COPYIN, ax.ACC_FLOAT32, a), ax.clause(ax.ACC_COPYIN, ax.ACC_FLOAT32, b),
                               ax.clause(ax.ACC_COPYOUT, ax.ACC_FLOAT32, c)])
        assert len(talloc.live) == 3
        ax.acc_loopnest_matmul(r, ax.ACC_FLOAT32, a, b, c, n, ax.ACC_KERNEL_TILED | ax.ACC_PREC_AUTO)
        x = a.reshape(-1)
        s = np.zeros(1, np.float32)
        ax.acc_reduce_sum(r, ax.ACC_FLOAT32, x, x.size, s)
        ax.acc_data_end(r)
        ref = oracle.matmul_f32(a, b)
        assert rel_fro(c, ref) <= FP32_REL_FRO_TOL
        assert abs(float(s[0]) - oracle.sum_f32(x)) <= 1e-5 * max(1.0, abs(oracle.sum_f32(x)))
        assert not talloc.live                          # region arrays and workspaces returned
        # device-pointer entry with a library-owned workspace
        da, db = torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()
        dc = torch.empty_like(da)
        before = talloc.allocs
        ax.accx_matmul_dev(ax.ACC_FLOAT32, da, db, dc, n, ax.ACC_KERNEL_TILED | ax.ACC_PREC_FULL6)
        torch.cuda.synchronize()
        assert talloc.allocs > before
        assert rel_fro(dc.cpu().numpy(), ref) <= FP32_REL_FRO_TOL
        # a batch
        items = [ax.batch_matmul(da, db, dc, n), ax.batch_reduce(da, n * n, dc[0, :1])]
        bh = ax.accx_batch_create(items)
        live_batch = len(talloc.live)
        ax.accx_batch_launch(bh)
        torch.cuda.synchronize()
        assert rel_fro(dc.cpu().numpy()[1:], ref[1:]) <= FP32_REL_FRO_TOL
        ax.accx_batch_destroy(bh)
        assert len(talloc.live) == live_batch - 1
        # the serving engine's block cache
        from paper_1412_1127_amd import serve
        wl = serve.make_workload(40, SEED + 7, rate=4000.0, len_hi=256, n_hi=1 << 18)
        pools = serve.Pools(wl)
        got = {}
        res = serve.run(wl, pools, slots=4, on_region_done=lambda rr, v: got.__setitem__(rr.key, v.numpy().copy()))
        assert res["completed_ok"] == len(wl.requests)
        for k, cc in got.items():
            rr = wl.regions[k]
            aa, bb = pools.inputs(rr)
            if rr.dtype == ax.ACC_INT32:
                assert np.array_equal(cc.reshape(rr.n, rr.n),
                                      oracle.matmul_i32(aa.numpy().reshape(rr.n, rr.n), bb.numpy().reshape(rr.n, rr.n)))
        ax.acc_shutdown()
        assert not talloc.live, "blocks the library did not return: %d" % len(talloc.live)
        assert talloc.allocs == talloc.frees
    finally:
        ax.accx_set_allocator(None, None)
        ax.acc_shutdown()
