"""Open-loop driver for the libaccx serving engine (accx_server_*).

Generates a seeded stream of offload-region requests, submits each at its
scheduled arrival time (open loop: a slow server does not delay later
arrivals), polls the engine between arrivals and reports latency from the
scheduled arrival to completion, so queueing delay is counted.

Workload (the serving configuration): Poisson arrivals at `rate` requests/s;
a region is a float32 or int32 matmul (probability `p_matmul`, LEN
log-uniform in [len_lo, len_hi], float32 and int32 equally likely) or a
float32 reduction (n log-uniform in [n_lo, n_hi]); each region serves
`per_region` requests on its device-resident arrays; an arrival opens a new
region while fewer than `window` are open, otherwise it goes to a random open
region that still has requests left.  Inputs are views into pinned pools of
seeded values (uniform[-1, 1] float32, integers in [-16, 16], uniform[0, 1)
float32), so host memory stays bounded.
"""
from __future__ import annotations

import dataclasses
import time

import numpy as np
import torch

import paper_1412_1127_amd as ax
import synth


@dataclasses.dataclass
class Region:
    key: int
    op: int          # ax.ACC_SERVE_MATMUL / ACC_SERVE_REDUCE
    dtype: int
    n: int
    a_off: int = 0   # offsets into the input pools
    b_off: int = 0
    requests: int = 0


@dataclasses.dataclass
class Request:
    t: float         # scheduled arrival, seconds from the start
    region: int
    first: bool
    last: bool
    init: float
    tag: int


@dataclasses.dataclass
class Workload:
    regions: dict
    requests: list
    rate: float

    def flops(self) -> float:
        return sum(2.0 * r.n ** 3 * r.requests for r in self.regions.values() if r.op == ax.ACC_SERVE_MATMUL)

    def reduce_bytes(self) -> float:
        return sum(4.0 * r.n * r.requests for r in self.regions.values() if r.op == ax.ACC_SERVE_REDUCE)


def make_workload(n_requests: int, seed: int = synth.DEFAULT_SEED, rate: float = 2000.0, p_matmul: float = 0.7,
                  len_lo: int = 128, len_hi: int = 2048, n_lo: int = 1 << 16, n_hi: int = 1 << 26,
                  per_region: int = 4, window: int = 16, pool_elems: int = 1 << 23,
                  pool01_elems: int = (1 << 26) + (1 << 24)) -> Workload:
    g = synth.rng(seed, synth.STREAM_SIZES)
    arrivals = synth.poisson_arrivals(n_requests, rate, seed)
    regions, requests, open_keys = {}, [], []
    for k, t in enumerate(arrivals):
        if len(open_keys) < window:
            key = len(regions)
            if g.random() < p_matmul:
                n = int(min(len_hi, np.floor(np.exp(g.uniform(np.log(len_lo), np.log(len_hi))))))
                dt = ax.ACC_FLOAT32 if g.random() < 0.5 else ax.ACC_INT32
                r = Region(key, ax.ACC_SERVE_MATMUL, dt, n, int(g.integers(0, pool_elems - n * n + 1)),
                           int(g.integers(0, pool_elems - n * n + 1)))
            else:
                n = int(min(n_hi, np.floor(np.exp(g.uniform(np.log(n_lo), np.log(n_hi))))))
                r = Region(key, ax.ACC_SERVE_REDUCE, ax.ACC_FLOAT32, n, int(g.integers(0, pool01_elems - n + 1)))
            regions[key] = r
            open_keys.append(key)
        else:
            key = open_keys[int(g.integers(0, len(open_keys)))]
            r = regions[key]
        first = r.requests == 0
        r.requests += 1
        last = r.requests == per_region
        if last:
            open_keys.remove(key)
        requests.append(Request(float(t), key, first, last, float(k % 7) * 0.5, k))
    # regions cut off by the end of the stream close on their final request
    last_of = {}
    for q in requests:
        last_of[q.region] = q
    for key in open_keys:
        last_of[key].last = True
    return Workload(regions, requests, rate)


class Pools:
    """Pinned host memory: seeded input pools, recycled matmul outputs and one
    result slot per reduction request."""

    def __init__(self, workload: Workload, seed: int = synth.DEFAULT_SEED, pool_elems: int = 1 << 23,
                 pool01_elems: int = (1 << 26) + (1 << 24)):
        self.f = torch.from_numpy(synth.uniform_pm1_f32((pool_elems,), seed, 21)).pin_memory()
        self.i = torch.from_numpy(synth.int_uniform_i32((pool_elems,), -16, 16, seed, 22)).pin_memory()
        self.x = torch.from_numpy(synth.uniform01_f32(pool01_elems, seed, 23)).pin_memory()
        self.results = torch.zeros(len(workload.requests), dtype=torch.float64).pin_memory()
        self.res_i = torch.zeros(len(workload.requests), dtype=torch.int32).pin_memory()
        self.res_f = torch.zeros(len(workload.requests), dtype=torch.float32).pin_memory()
        self._free = []
        self.len_hi = max([r.n for r in workload.regions.values() if r.op == ax.ACC_SERVE_MATMUL] + [1])

    def out_buffer(self) -> torch.Tensor:
        if self._free:
            return self._free.pop()
        return torch.empty(self.len_hi * self.len_hi, dtype=torch.float32).pin_memory()

    def release(self, buf: torch.Tensor) -> None:
        self._free.append(buf)

    def inputs(self, r: Region):
        if r.op == ax.ACC_SERVE_REDUCE:
            return self.x[r.a_off:r.a_off + r.n], None
        pool = self.f if r.dtype == ax.ACC_FLOAT32 else self.i
        nn = r.n * r.n
        return pool[r.a_off:r.a_off + nn], pool[r.b_off:r.b_off + nn]


def run(workload: Workload, pools: Pools, slots: int = 8, budget: int = 64 << 30, matmul_flags: int = 0,
        on_region_done=None, alone: bool = False, time_scale: float = 1.0) -> dict:
    """Serve the workload.  alone=True submits each request only after the
    previous one finished (no overlap), for comparisons.  on_region_done(region,
    output) gets each matmul region's output (a flat float32 or int32 view of
    the pinned buffer, valid during the call) when its last request completes;
    reduction results are in the returned 'reduce_results' (tag -> value)."""
    server = ax.accx_server_create(1 if alone else slots, budget)
    try:
        outbuf, pending_last = {}, {}
        lat, status = {}, {}
        reduce_results = {}
        t_base = ax.accx_server_now(server)
        wall0 = time.perf_counter()

        def handle(done):
            for tag, st, ts, tstart, tdone in done:
                q = workload.requests[tag]
                status[tag] = st
                lat[tag] = (tdone - t_base) - q.t * time_scale
                r = workload.regions[q.region]
                if r.op == ax.ACC_SERVE_REDUCE and st == ax.ACC_OK:
                    reduce_results[tag] = float(pools.res_f[tag]) if r.dtype == ax.ACC_FLOAT32 else int(pools.res_i[tag])
                if q.last and r.op == ax.ACC_SERVE_MATMUL:
                    buf = outbuf.pop(q.region)
                    if on_region_done is not None and st == ax.ACC_OK:
                        view = buf[:r.n * r.n]
                        if r.dtype == ax.ACC_INT32:
                            view = view.view(torch.int32)
                        on_region_done(r, view)
                    pools.release(buf)

        for q in workload.requests:
            r = workload.regions[q.region]
            if alone:
                ax.accx_server_drain(server)
                handle(ax.accx_server_poll(server))
            else:
                while ax.accx_server_now(server) - t_base < q.t * time_scale:
                    handle(ax.accx_server_poll(server))
            a, b = pools.inputs(r)
            if r.op == ax.ACC_SERVE_MATMUL:
                if q.region not in outbuf:
                    outbuf[q.region] = pools.out_buffer()
                c_ptr = outbuf[q.region].data_ptr()
                flags = matmul_flags
            else:
                c_ptr = (pools.res_f if r.dtype == ax.ACC_FLOAT32 else pools.res_i)[q.tag:q.tag + 1].data_ptr()
                flags = 0
            req = ax.accx_request(r.op, r.dtype, q.region, int(q.first), int(q.last), a.data_ptr(),
                                  b.data_ptr() if b is not None else None, c_ptr, r.n, q.init, flags, 0, q.tag)
            ax.accx_server_submit(server, req)
            handle(ax.accx_server_poll(server))
        ax.accx_server_drain(server)
        handle(ax.accx_server_poll(server))
        wall = time.perf_counter() - wall0
        stats = ax.accx_server_stats(server)
    finally:
        ax.accx_server_destroy(server)
    vals = np.array([lat[t] for t in sorted(lat)]) * 1e3
    ok = sum(1 for s in status.values() if s == ax.ACC_OK)
    return {
        "requests": len(workload.requests), "completed_ok": ok,
        "errors": {int(s): sum(1 for v in status.values() if v == s) for s in set(status.values()) if s != ax.ACC_OK},
        "latency_ms": {"p50": float(np.percentile(vals, 50)), "p99": float(np.percentile(vals, 99)),
                       "mean": float(vals.mean()), "max": float(vals.max())},
        "wall_s": wall, "throughput_rps": len(workload.requests) / wall,
        "matmul_tflops": workload.flops() / wall / 1e12, "reduce_gbs": workload.reduce_bytes() / wall / 1e9,
        "server": stats, "reduce_results": reduce_results,
    }
