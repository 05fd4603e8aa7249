"""Benchmark of the offload hot path on one MI355X.

One step is one pass of the whole path over the plain-method-at-scale
workload: the loop-nest matmul of Listing 1a at LEN = 4096 in float32
(uniform[-1, 1], LDS-tiled bf16x3 matrix-core kernel) and in int32
(uniform integers in [-16, 16], int8-limb matrix-core kernel with its max|x|
probe), then reduction(+) over 2^28 float32 values uniform in [0, 1), on
device-resident inputs (the data region is opened before the timed region,
as the data directive keeps arrays on the device across the kernels).

value = matmul operations of the step (2*LEN^3 for each of the two matmuls)
divided by the wall time of the step, in TFLOP/s; the reduction's time is in
the step.  Per-kernel durations come from HIP events that the library records
on the launch stream around each kernel.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_BF16_TFLOPS = 2500.0   # MI355X dense bf16 matrix peak
PEAK_INT8_TOPS = 5000.0     # MI355X dense int8 matrix peak
PEAK_HBM_GBS = 8000.0       # MI355X HBM3E
PEAK_FP32_TFLOPS = 157.3    # MI355X float32 matrix / vector peak
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")


def _args():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=50)
    p.add_argument("--warmup", type=int, default=20)
    p.add_argument("--len", type=int, default=4096)
    p.add_argument("--n-reduce", type=int, default=1 << 28)
    p.add_argument("--prec", choices=["full6", "five", "auto", "cheap3"], default="auto")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-rows", type=int, default=0,
                   help="rows of C the CPU baseline computes per matmul, scaled to the whole step "
                        "(0: all LEN rows, the whole step)")
    p.add_argument("--no-verify", action="store_true")
    p.add_argument("--tile", choices=["256", "256x128", "128", "64", "256w4"], default=None,
                   help="force the float32 tile configuration (implies --no-autotune)")
    p.add_argument("--no-autotune", action="store_true",
                   help="skip the tile autotuner before the timed region (size heuristic instead)")
    p.add_argument("--workload", choices=["scale", "small", "precision", "batch", "serve", "rowblock", "reductions",
                                          "regions"],
                   default="scale",
                   help="scale (default): the step described above; the others measure the remaining "
                        "configurations (LEN=256 plain method, LEN=8192 precision, batching, serving) and "
                        "one GPU's 512-row block of the LEN=4096 product (rowblock)")
    p.add_argument("--requests", type=int, default=2000, help="serve: number of requests")
    p.add_argument("--batch-prec", choices=["auto", "full6"], default="auto",
                   help="batch: ACC_BATCH_PREC_AUTO (three products, per-tile probe and correction) or six products")
    p.add_argument("--streams", type=int, choices=[1, 2], default=1,
                   help="scale: 2 runs the int32 matmul and the reduction on a second stream, overlapped "
                        "with the float32 matmul")
    p.add_argument("--region", choices=["fused", "separate"], default="fused",
                   help="scale, one stream: 'fused' runs the float32 matmul and the reduction as one region "
                        "(accx_matmul_reduce_dev: the sum rides in the three-product pass's launch when that "
                        "pass runs on the 256 x 256 tile); 'separate' makes one call per operation")
    p.add_argument("--ingest-counters", metavar="DIR", default=None,
                   help="write the HBM traffic summary from rocprofv3 FETCH_SIZE/WRITE_SIZE runs in DIR and exit")
    p.add_argument("--no-onbox", action="store_true",
                   help="scale: skip the on-box reference points (device copy, vendor GEMMs)")
    p.add_argument("--time-all-kernels", action="store_true",
                   help="scale: event-time every kernel inside the timed region (default: the dominant one only)")
    p.add_argument("--copy-calib", action="store_true",
                   help="also run one plain 1 GiB device copy (counter calibration under rocprofv3)")
    return p.parse_args()


def _source_hash(*names) -> str:
    h = hashlib.sha256()
    for n in names:
        with open(os.path.join(ROOT, "paper_1412_1127_amd", "csrc", n), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _traffic(kernel: str, workload: str):
    """HBM bytes per launch from the committed counter summary, if it was
    taken on the current kernel source; else None."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
        e = t[kernel][workload]
        if e.get("source_hash") != _source_hash("gemm_mfma.hip", "mfma_tile.h"):
            return None
        return float(e["fetch_bytes"]) + float(e["write_bytes"])
    except (OSError, KeyError, ValueError):
        return None


def ingest_counters(root: str, prec: str) -> int:
    """Fold two rocprofv3 counter runs of this script (FETCH_SIZE under
    root/fetch, WRITE_SIZE under root/write, csv output named after the
    directory, both with --copy-calib and precision `prec`) into
    TRAFFIC_FILE: per-dispatch KiB scaled by what the same counter reads for
    the plain 1 GiB device copy, averaged over the float32 LEN=4096 GEMM's
    dispatches.  Prints the per-kernel table as well."""
    import collections
    import csv

    def load(kind):
        per, names = collections.defaultdict(float), {}
        with open(os.path.join(root, kind, kind + "_counter_collection.csv")) as f:
            for r in csv.DictReader(f):
                per[r["Dispatch_Id"]] += float(r["Counter_Value"])
                names[r["Dispatch_Id"]] = r["Kernel_Name"]
        return per, names

    fetch, fnames = load("fetch")
    write, wnames = load("write")
    by = collections.defaultdict(lambda: ([], []))
    for d, v in fetch.items():
        by[fnames[d]][0].append(v)
    for d, v in write.items():
        by[wnames[d]][1].append(v)
    copy = [k for k in by if "copyBuffer" in k and by[k][0] and by[k][1]]
    if not copy:
        print("no device-copy dispatch found: run both passes with --copy-calib", file=sys.stderr)
        return 1
    ff, wf = 1048576.0 / by[copy[0]][0][-1], 1048576.0 / by[copy[0]][1][-1]
    print("copy calibration: FETCH_SIZE x %.4f, WRITE_SIZE x %.4f" % (ff, wf))
    print("| kernel | FETCH_SIZE raw (KiB) | WRITE_SIZE raw (KiB) | fetched (MB, scaled) | written (MB, scaled) |")
    print("|---|---|---|---|---|")
    for k, (fv, wv) in by.items():
        if fv and wv:
            fm, wm = sum(fv) / len(fv), sum(wv) / len(wv)
            name = k.replace("void ", "", 1).replace("accx::(anonymous namespace)::", "")
            depth, cut = 0, len(name)
            for i, ch in enumerate(name):                 # drop the parameter list
                depth += (ch == "<") - (ch == ">")
                if ch == "(" and depth == 0 and i > 0:
                    cut = i
                    break
            print("| `%s` | %.0f | %.0f | %.1f | %.1f |" % (name[:cut][:100], fm, wm, fm * ff * 1.024e-3,
                                                          wm * wf * 1.024e-3))
    # the float32 GEMM of the run (the counter runs fix the 256 x 256 tile,
    # so that no autotuner candidate is in them): the bf16x3 kernel of that
    # tile with the precision's product count (template argument 9)
    nprod = {"full6": 6, "five": 5, "auto": 3, "cheap3": 3}[prec]

    def targs(k):
        head = "void accx::(anonymous namespace)::gemm_packed<"
        return k[len(head):k.index(">(")].split(", ") if k.startswith(head) and ">(" in k else []

    # (last template argument: "true" for the pass that carries the
    # co-scheduled reduction, recorded under its own workload key)
    g = [k for k in by if targs(k)[:4] == ["false", "3", "256", "256"] and targs(k)[8] == str(nprod)
         and by[k][0] and by[k][1]]
    if not g or len({targs(k)[-1] for k in g}) != len(g):
        print("expected one float32 256 x 256 GEMM with %d products per kind, found %d" % (nprod, len(g)),
              file=sys.stderr)
        return 1
    cur = _source_hash("gemm_mfma.hip", "mfma_tile.h")
    try:
        with open(TRAFFIC_FILE) as f:
            old = json.load(f).get("gemm_bf16x3", {})
    except (OSError, ValueError, AttributeError):
        old = {}
    out = {"gemm_bf16x3": {k: v for k, v in old.items() if v.get("source_hash") == cur}}  # drop stale entries
    for k in g:
        fv, wv = by[k]
        fm, wm = sum(fv) / len(fv), sum(wv) / len(wv)
        key = "len4096_" + prec + ("_coreduce" if targs(k)[-1] == "true" else "")
        out["gemm_bf16x3"][key] = {
            "fetch_bytes": fm * ff * 1024, "write_bytes": wm * wf * 1024, "fetch_kib_raw": fm, "write_kib_raw": wm,
            "fetch_factor": ff, "write_factor": wf, "source_hash": cur, "kernel": k}
    with open(TRAFFIC_FILE, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out, indent=1))
    return 0


def _onbox(torch, x):
    """Reference points measured on this GPU outside the timed region, beside
    the datasheet peaks the roofline fractions use: the measured ceilings
    (library kernels doing nothing but matrix instructions, bf16 and int8,
    on every CU; a read-only stream of the 1 GiB reduction input), a plain
    device copy of that input (read + write bytes), and the vendor library's
    bf16 and float32 GEMMs at LEN=4096 (torch.matmul, hipBLASLt)."""
    import paper_1412_1127_amd as ax

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps
    out = {"datasheet": {"bf16_tflops": PEAK_BF16_TFLOPS, "int8_tops": PEAK_INT8_TOPS, "hbm_gbs": PEAK_HBM_GBS}}
    stream = torch.cuda.current_stream()
    # a ceiling is the best of three timings (the clock under load drifts)
    for name, kind in (("measured_bf16_mfma_tflops", 0), ("measured_int8_mfma_tops", 1)):
        ops = ax.accx_onbox_mfma(kind, 5000, stream)            # about 1.5 ms per launch
        timed(lambda: ax.accx_onbox_mfma(kind, 5000, stream), 3)  # clocks to their loaded state
        out[name] = max(ops / (timed(lambda: ax.accx_onbox_mfma(kind, 5000, stream), 5) * 1e-3) / 1e12
                        for _ in range(3))
    nbytes = x.numel() * x.element_size()
    out["measured_hbm_read_gbs"] = max(
        nbytes / (timed(lambda: ax.accx_onbox_read(x, nbytes, stream), 10) * 1e-3) / 1e9 for _ in range(3))
    dst = torch.empty_like(x)
    ms = timed(lambda: dst.copy_(x), 10)
    out["copy_gbs"] = 2.0 * x.numel() * x.element_size() / (ms * 1e-3) / 1e9
    del dst
    n = 4096
    for name, dt in (("vendor_bf16_gemm_tflops", torch.bfloat16), ("vendor_fp32_gemm_tflops", torch.float32)):
        a = torch.rand((n, n), device=x.device, dtype=dt)
        b = torch.rand((n, n), device=x.device, dtype=dt)
        timed(lambda: torch.matmul(a, b), 10)               # clocks to their loaded state
        out[name] = 2.0 * n ** 3 / (timed(lambda: torch.matmul(a, b), 30) * 1e-3) / 1e12
        del a, b
    return out


def _pct(v, q):
    import numpy as np
    return float(np.percentile(np.asarray(v), q)) if len(v) else None


def run_scale(args) -> int:
    import numpy as np
    import torch

    import paper_1412_1127_amd as ax
    import synth

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    n, nred = args.len, args.n_reduce
    seed = synth.DEFAULT_SEED
    prec = {"full6": ax.ACC_PREC_FULL6, "five": ax.ACC_PREC_FIVE, "auto": ax.ACC_PREC_AUTO,
            "cheap3": ax.ACC_PREC_CHEAP3}[args.prec]
    # matrix products per launch of the kernel named gemm_bf16x3 (with AUTO:
    # the cheap pass; its correction pass is gemm_bf16x3_corr)
    nprod = {"full6": 6, "five": 5, "auto": 3, "cheap3": 3}[args.prec]

    t_gen = time.time()
    a = synth.uniform_pm1_f32((n, n), seed, synth.STREAM_A)
    b = synth.uniform_pm1_f32((n, n), seed, synth.STREAM_B)
    ai = synth.int_uniform_i32((n, n), -16, 16, seed, synth.STREAM_A)
    bi = synth.int_uniform_i32((n, n), -16, 16, seed, synth.STREAM_B)
    x = synth.uniform01_f32(nred, seed, synth.STREAM_X)
    print("inputs generated in %.1f s" % (time.time() - t_gen), file=sys.stderr, flush=True)

    dev = torch.device("cuda:0")
    ax.acc_init(0, 0)
    da, db = torch.from_numpy(a).to(dev), torch.from_numpy(b).to(dev)
    dai, dbi = torch.from_numpy(ai).to(dev), torch.from_numpy(bi).to(dev)
    dx = torch.from_numpy(x).to(dev)
    dc = torch.empty((n, n), dtype=torch.float32, device=dev)
    dci = torch.empty((n, n), dtype=torch.int32, device=dev)
    dr = torch.empty(1, dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream()
    sh = stream.cuda_stream
    # Library workspaces, allocated once outside the timed region.
    f_flags = ax.ACC_KERNEL_TILED | prec | (ax.TILES[args.tile] if args.tile else 0)
    i_flags = ax.ACC_KERNEL_TILED
    wf = torch.empty(ax.accx_matmul_workspace_size(ax.ACC_FLOAT32, n, f_flags), dtype=torch.uint8, device=dev)
    wi = torch.empty(ax.accx_matmul_workspace_size(ax.ACC_INT32, n, i_flags), dtype=torch.uint8, device=dev)
    wr = torch.zeros(ax.accx_reduce_workspace_size(ax.ACC_FLOAT32, nred, 0), dtype=torch.uint8, device=dev)
    fused = args.region == "fused" and args.streams == 1
    wfr = (torch.empty(ax.accx_matmul_reduce_workspace_size(n, f_flags, nred), dtype=torch.uint8, device=dev)
           if fused else None)

    tuned = {}
    if not args.no_autotune and not args.tile:
        tuned["f32"] = ax.accx_autotune(ax.ACC_FLOAT32, n, f_flags)
        tuned["i32"] = ax.accx_autotune(ax.ACC_INT32, n, ax.ACC_LIMBS(1))
        print("autotuned tiles:", tuned, file=sys.stderr, flush=True)

    # The three operations of a step are independent: with --streams 2 the
    # int32 matmul and the reduction run on a second stream (default
    # priority), so the HBM-bound reduction and packing overlap the float32
    # matrix-core GEMM; the step ends when both streams are done.
    side = torch.cuda.Stream() if args.streams == 2 else stream
    fork, join = torch.cuda.Event(), torch.cuda.Event()

    def step():
        if fused:
            # one region: the float32 matmul nest and the reduction nest
            ax.accx_matmul_reduce_dev(da, db, dc, n, f_flags, dx, nred, 0.0, dr, wfr, wfr.numel(), sh)
            ax.accx_matmul_dev(ax.ACC_INT32, dai, dbi, dci, n, i_flags, wi, wi.numel(), sh)
            return
        if side is not stream:
            fork.record(stream)
            side.wait_event(fork)
        ax.accx_matmul_dev(ax.ACC_FLOAT32, da, db, dc, n, f_flags, wf, wf.numel(), sh)
        if side is not stream:
            # the HBM-bound reduction first: it can share CUs with the float32
            # packing and GEMM; the int32 GEMM needs LDS the float32 GEMM holds
            ax.accx_reduce_sum_dev(ax.ACC_FLOAT32, dx, nred, 0.0, dr, 0, wr, wr.numel(), side.cuda_stream)
            ax.accx_matmul_dev(ax.ACC_INT32, dai, dbi, dci, n, i_flags, wi, wi.numel(), side.cuda_stream)
        else:
            ax.accx_matmul_dev(ax.ACC_INT32, dai, dbi, dci, n, i_flags, wi, wi.numel(), sh)
            ax.accx_reduce_sum_dev(ax.ACC_FLOAT32, dx, nred, 0.0, dr, 0, wr, wr.numel(), sh)
        if side is not stream:
            join.record(side)
            stream.wait_event(join)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    print("warmup done", file=sys.stderr, flush=True)

    # Inside the timed region only the dominant kernel carries timing events
    # (each timed kernel adds two event records to the stream); the other
    # kernels' breakdown comes from extra steps after the timed region.
    ax.accx_timing_filter(None if args.time_all_kernels else ["gemm_bf16x3"])
    ax.accx_timing_enable(True)
    ax.accx_timing_read(reset=True)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        ev[k][0].record(stream)
        step()
        ev[k][1].record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ktimed = ax.accx_timing_read(reset=True)
    step_ms = [s.elapsed_time(e) for s, e in ev]
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    print("timed %d steps: %.3f ms/step" % (args.steps, ms_per_step), file=sys.stderr, flush=True)
    nb = min(args.steps, 10)                      # breakdown steps (not timed as a whole)
    ax.accx_timing_filter(None)
    for _ in range(nb):
        step()
    torch.cuda.synchronize()
    ktimes = ax.accx_timing_read(reset=True)
    # with the fused region, the three-product pass and the reduction also
    # run apart (separate calls, after the timed region), for their own
    # rooflines
    kalone = None
    if fused:
        for _ in range(nb):
            ax.accx_matmul_dev(ax.ACC_FLOAT32, da, db, dc, n, f_flags, wf, wf.numel(), sh)
            ax.accx_reduce_sum_dev(ax.ACC_FLOAT32, dx, nred, 0.0, dr, 0, wr, wr.numel(), sh)
        torch.cuda.synchronize()
        kalone = ax.accx_timing_read(reset=True)
    ax.accx_timing_enable(False)

    if args.copy_calib:
        src = torch.empty(1 << 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        src.fill_(1.0)
        dst.copy_(src)
        torch.cuda.synchronize()

    ops = 2.0 * 2.0 * n ** 3
    value = ops / (ms_per_step * 1e-3) / 1e12

    def kavg(name, kt=None):
        v = (ktimes if kt is None else kt).get(name)
        return (v[1] / v[0]) if v and v[0] else None

    g_ms = kavg("gemm_bf16x3", ktimed)
    # the int32 matmul launches a one-digit and a four-digit GEMM, one of which
    # exits at once: its cost per matmul is the sum over both
    gi_ms = ktimes["gemm_i8"][1] / nb if "gemm_i8" in ktimes else None
    # the sum rode in the three-product pass if no reduction kernel of its
    # own ran (its last step runs in the probe's launch, or with CHEAP3 in a
    # one-workgroup launch of its own)
    co_red = fused and "reduce_fast" not in ktimes
    red_ms = kavg("reduce_fast")
    g_flops = nprod * 2.0 * n ** 3
    achieved = g_flops / (g_ms * 1e-3) / 1e12 if g_ms else None
    workload = "len%d_%s%s" % (n, args.prec, "_coreduce" if co_red else "")
    roofline = {"kernel": "gemm_bf16x3", "bound": "mfma", "achieved": achieved, "peak": PEAK_BF16_TFLOPS,
                "unit": "TFLOP/s", "frac": (achieved / PEAK_BF16_TFLOPS) if achieved else None,
                "traffic": _traffic("gemm_bf16x3", workload),
                "flops_per_launch": g_flops, "avg_ms": g_ms}
    if co_red and g_ms:
        # the same launch also streamed the reduction's 4 * n_reduce bytes
        roofline["co_scheduled_reduce_bytes"] = 4.0 * nred
        roofline["co_scheduled_reduce_gbs"] = 4.0 * nred / (g_ms * 1e-3) / 1e9
        roofline["co_scheduled_reduce_frac_hbm"] = roofline["co_scheduled_reduce_gbs"] / PEAK_HBM_GBS
    if kalone:
        ga, ra = kavg("gemm_bf16x3", kalone), kavg("reduce_fast", kalone)
        roofline["apart"] = {"gemm_ms": ga, "gemm_frac": g_flops / (ga * 1e-3) / 1e12 / PEAK_BF16_TFLOPS if ga else None,
                             "reduce_ms": ra,
                             "reduce_frac_hbm": 4.0 * nred / (ra * 1e-3) / 1e9 / PEAK_HBM_GBS if ra else None,
                             "saved_ms": (ga + ra - g_ms) if (ga and ra and g_ms) else None}

    components = {}
    f32_total = sum(v[1] for k, v in ktimes.items() if "bf16x3" in k or k == "probe_f64") / nb
    components["f32_matmul"] = {"kernels_ms_per_step": f32_total, "gemm_ms": g_ms,
                                "tflops_fp32_equiv_gemm": 2.0 * n ** 3 / (g_ms * 1e-3) / 1e12 if g_ms else None,
                                "tflops_fp32_equiv_with_pack": 2.0 * n ** 3 / (f32_total * 1e-3) / 1e12,
                                "products": nprod,
                                "probe_ms": kavg("probe_f64"), "correction_ms": kavg("gemm_bf16x3_corr")}
    i_total = sum(v[1] for k, v in ktimes.items() if k in ("gemm_i8", "pack_i8")) / nb
    components["i32_matmul"] = {"kernels_ms_per_step": i_total, "gemm_ms": gi_ms,
                                "tops_int32_equiv_gemm": 2.0 * n ** 3 / (gi_ms * 1e-3) / 1e12 if gi_ms else None,
                                "frac_int8_peak_gemm": (2.0 * n ** 3 / (gi_ms * 1e-3) / 1e12 / PEAK_INT8_TOPS)
                                if gi_ms else None}
    components["reduce"] = {"ms": red_ms, "gbs": 4.0 * nred / (red_ms * 1e-3) / 1e9 if red_ms else None,
                            "frac_hbm": (4.0 * nred / (red_ms * 1e-3) / 1e9 / PEAK_HBM_GBS) if red_ms else None}
    if co_red:
        components["reduce"]["co_scheduled_in"] = "gemm_bf16x3"
        components["reduce"]["final_ms"] = kavg("reduce_final")  # None: added in the probe's launch
    components["kernels"] = {k: {"launches": v[0], "avg_ms": v[1] / v[0], "min_ms": v[2], "max_ms": v[3]}
                             for k, v in ktimes.items()}
    components["breakdown_steps"] = nb

    accuracy = {}
    if not args.no_verify:
        import oracle
        g = synth.rng(seed, 99)
        ii, jj = g.integers(0, n, 2048), g.integers(0, n, 2048)
        c = dc.cpu().numpy()
        ref = oracle.matmul_at(a, b, ii, jj)
        accuracy["f32_rel_fro_vs_oracle_sampled"] = float(np.linalg.norm(c[ii, jj] - ref) / np.linalg.norm(ref))
        dcp = torch.empty_like(dc)
        ax.accx_matmul_dev(ax.ACC_FLOAT32, da, db, dcp, n, ax.ACC_KERNEL_PLAIN, None, 0, sh)
        torch.cuda.synchronize()
        cp = dcp.cpu().numpy().astype(np.float64)
        accuracy["f32_rel_fro_vs_plain"] = float(np.linalg.norm(c - cp) / np.linalg.norm(cp))
        ci = dci.cpu().numpy()
        accuracy["i32_bit_exact_sampled"] = bool(np.array_equal(ci[ii, jj], oracle.matmul_at(ai, bi, ii, jj)))
        sref = oracle.sum_f32(x)
        accuracy["reduce_rel_err"] = abs(float(dr.item()) - sref) / sref

    onbox = None if args.no_onbox else _onbox(torch, dx)
    if onbox:
        mb = onbox["measured_bf16_mfma_tflops"]
        roofline["measured_peak"] = mb
        roofline["measured_frac"] = achieved / mb if achieved else None
        gi = components["i32_matmul"]["tops_int32_equiv_gemm"]
        components["i32_matmul"]["frac_measured_int8_gemm"] = gi / onbox["measured_int8_mfma_tops"] if gi else None
        gb = components["reduce"]["gbs"]
        components["reduce"]["frac_measured_read"] = gb / onbox["measured_hbm_read_gbs"] if gb else None

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        rows = min(args.cpu_rows, n) if args.cpu_rows > 0 else n
        t = time.perf_counter()
        oracle.matmul_rows(a, b, 0, rows)
        tf = time.perf_counter() - t
        t = time.perf_counter()
        oracle.matmul_rows(ai, bi, 0, rows)
        ti = time.perf_counter() - t
        t = time.perf_counter()
        oracle.sum_f32(x)
        tr = time.perf_counter() - t
        cpu_step_s = (tf + ti) * (n / rows) + tr
        cpu = {"value": ops / cpu_step_s / 1e12, "unit": "TFLOP/s", "cores": oracle.max_threads(), "kind": "oracle",
               "sample": ("the whole step: " if rows == n else "rows 0..%d of both matmuls, scaled by %d/%d; " %
                          (rows - 1, n, rows)) +
                         "float64 (float32 inputs) and uint64-wrapping (int32) LEN=%d matmul oracles with OpenMP, "
                         "serial float64 sum of %d values; measured %.1f s" % (n, nred, tf + ti + tr),
               "step_s_scaled": cpu_step_s}

    line = {
        "metric": "matmul TFLOP/s (% MFMA peak) at <=1e-5 rel err vs plain kernel; p50/p99 latency",
        "value": value, "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 (bf16x3 matrix cores, f32 accumulate) + int32 (int8-limb matrix cores)",
        "data": "synthetic",
        "config": {"workload": "plain method at scale: LEN=%d square row-major matmul in float32 uniform[-1,1] "
                               "and int32 uniform [-16,16], plus reduction(+) over %d float32 uniform[0,1)"
                               % (n, nred),
                   "len": n, "n_reduce": nred, "precision": args.prec, "seed": seed, "streams": args.streams,
                   "region": "fused" if fused else "separate", "reduce_co_scheduled": co_red,
                   "tiles": {k: {"tile": [t for t, v in ax.TILES.items() if v == tv][0], "tune_ms": ms}
                             for k, (tv, ms) in tuned.items()}},
        "latency_ms": {"p50": _pct(step_ms, 50), "p99": _pct(step_ms, 99),
                       "hmean": len(step_ms) / sum(1.0 / s for s in step_ms)},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "components": components,
        "accuracy": accuracy,
        "onbox": onbox,
    }
    ax.acc_shutdown()
    print(json.dumps(line))
    return 0


def _common(args, metric, value, unit, ms, config, higher=True, dtype="f32", **extra):
    line = {"metric": metric, "value": value, "unit": unit, "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": higher, "scaling": "weak",
            "vs_baseline": None, "dtype": dtype, "data": "synthetic", "config": config}
    line.update(extra)
    return line


def _event_times(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(steps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    return ts


def run_small(args) -> int:
    """LEN=256 float32, uniform[-1,1]: the plain one-thread-per-(i,j) kernel
    (and the tiled kernel beside it), per-call latency and error vs the
    float64 oracle."""
    import numpy as np
    import torch

    import oracle
    import paper_1412_1127_amd as ax
    import synth
    n = 256
    a = synth.uniform_pm1_f32((n, n), synth.DEFAULT_SEED, synth.STREAM_A)
    b = synth.uniform_pm1_f32((n, n), synth.DEFAULT_SEED, synth.STREAM_B)
    ax.acc_init(0, 0)
    da, db = torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()
    dc = torch.empty((n, n), device="cuda")
    ref = oracle.matmul_f32(a, b)
    out = {}
    for name, flags in [("plain", ax.ACC_KERNEL_PLAIN), ("listing1b", ax.ACC_KERNEL_PLAIN_LISTING1B),
                        ("tiled_full6", ax.ACC_KERNEL_TILED | ax.ACC_PREC_FULL6)]:
        ts = _event_times(lambda: ax.accx_matmul_dev(ax.ACC_FLOAT32, da, db, dc, n, flags), args.steps, args.warmup)
        c = dc.cpu().numpy()
        out[name] = {"p50_ms": float(np.percentile(ts, 50)), "p99_ms": float(np.percentile(ts, 99)),
                     "tflops_p50": 2.0 * n ** 3 / (np.percentile(ts, 50) * 1e-3) / 1e12,
                     "rel_fro_vs_oracle": float(np.linalg.norm(c - ref) / np.linalg.norm(ref))}
    ax.acc_shutdown()
    p = out["plain"]
    print(json.dumps(_common(args, "matmul TFLOP/s (plain kernel, LEN=256) and p50/p99 latency", p["tflops_p50"],
                             "TFLOP/s", p["p50_ms"],
                             {"workload": "plain method, smallest: LEN=256 float32 uniform[-1,1]", "len": n},
                             latency_ms={"p50": p["p50_ms"], "p99": p["p99_ms"]}, kernels=out)))
    return 0


def run_precision(args) -> int:
    """LEN=8192 float32, N(0,1) x 2^U(-8,8) per row: bf16x3 on matrix cores
    (six products, and the probed AUTO mode) beside the float32 plain kernel;
    relative Frobenius error vs the float64 oracle on sampled entries."""
    import numpy as np
    import torch

    import oracle
    import paper_1412_1127_amd as ax
    import synth
    n = 8192
    a = synth.normal_rowscaled_f32(n, n, synth.DEFAULT_SEED, synth.STREAM_A)
    b = synth.normal_rowscaled_f32(n, n, synth.DEFAULT_SEED, synth.STREAM_B)
    ax.acc_init(0, 0)
    da, db = torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()
    dc = torch.empty((n, n), device="cuda")
    g = synth.rng(synth.DEFAULT_SEED, 98)
    ii, jj = g.integers(0, n, 2048), g.integers(0, n, 2048)
    ref = oracle.matmul_at(a, b, ii, jj)
    ax.accx_autotune(ax.ACC_FLOAT32, n, ax.ACC_PREC_FULL6)
    ax.accx_timing_enable(True)
    out = {}
    ax.accx_autotune(ax.ACC_FLOAT32, n, ax.ACC_PREC_F32MFMA)
    for name, flags, reps in [("bf16x3_full6", ax.ACC_KERNEL_TILED | ax.ACC_PREC_FULL6, args.steps),
                              ("bf16x3_auto", ax.ACC_KERNEL_TILED | ax.ACC_PREC_AUTO, args.steps),
                              ("f32_mfma_tiled", ax.ACC_KERNEL_TILED | ax.ACC_PREC_F32MFMA, args.steps),
                              ("plain_f32", ax.ACC_KERNEL_PLAIN, 1)]:
        ax.accx_timing_read(reset=True)
        ts = _event_times(lambda: ax.accx_matmul_dev(ax.ACC_FLOAT32, da, db, dc, n, flags), reps,
                          1 if reps > 1 else 0)
        kt = ax.accx_timing_read(reset=True)
        c = dc.cpu().numpy()
        ms = float(np.median(ts))
        out[name] = {"ms": ms, "tflops_fp32_equiv": 2.0 * n ** 3 / (ms * 1e-3) / 1e12,
                     "rel_fro_vs_oracle_sampled": float(np.linalg.norm(c[ii, jj] - ref) / np.linalg.norm(ref)),
                     "kernels": {k: v[1] / v[0] for k, v in kt.items()}}
    ax.accx_timing_enable(False)
    ax.acc_shutdown()
    f = out["bf16x3_full6"]
    gm = f["kernels"].get("gemm_bf16x3")
    achieved = 6 * 2.0 * n ** 3 / (gm * 1e-3) / 1e12 if gm else None
    # the float32 tiled comparator against the float32 matrix-core peak
    fm = out["f32_mfma_tiled"]["kernels"].get("gemm_f32mm")
    out["f32_mfma_tiled"]["roofline"] = {
        "kernel": "gemm_f32mm", "bound": "mfma", "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
        "achieved": 2.0 * n ** 3 / (fm * 1e-3) / 1e12 if fm else None,
        "frac": 2.0 * n ** 3 / (fm * 1e-3) / 1e12 / PEAK_FP32_TFLOPS if fm else None}
    out["bf16x3_speedup_over_f32_mfma"] = out["f32_mfma_tiled"]["ms"] / f["ms"]
    print(json.dumps(_common(
        args, "matmul TFLOP/s (bf16x3, LEN=8192) at <=1e-5 rel err", f["tflops_fp32_equiv"], "TFLOP/s", f["ms"],
        {"workload": "precision: LEN=8192 float32 N(0,1) x 2^U(-8,8) per row", "len": n},
        roofline={"kernel": "gemm_bf16x3", "bound": "mfma", "achieved": achieved, "peak": PEAK_BF16_TFLOPS,
                  "unit": "TFLOP/s", "frac": achieved / PEAK_BF16_TFLOPS if achieved else None},
        paths=out)))
    return 0


def run_batch(args) -> int:
    """512 float32 matmuls (LEN uniform over {64, ..., 1024}) + 256 float32
    reductions (n log-uniform in [2^16, 2^24]) as one graph launch."""
    import numpy as np
    import torch

    import oracle
    import paper_1412_1127_amd as ax
    import synth
    seed = synth.DEFAULT_SEED
    lens = synth.lens_uniform(512, [64 * k for k in range(1, 17)], seed)
    ns = synth.log_uniform_int(256, 1 << 16, 1 << 24, seed, synth.STREAM_X)
    ax.acc_init(0, 0)
    items, mats, reds = [], [], []
    for k, n in enumerate(lens):
        a = synth.uniform_pm1_f32((n, n), seed, 1000 + 2 * k)
        b = synth.uniform_pm1_f32((n, n), seed, 1001 + 2 * k)
        da, db = torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()
        dc = torch.empty((n, n), device="cuda")
        mats.append((a, b, da, db, dc, int(n)))
        items.append(ax.batch_matmul(da, db, dc, int(n)))
    for k, n in enumerate(ns):
        x = synth.uniform01_f32(int(n), seed, 5000 + k)
        dx = torch.from_numpy(x).cuda()
        r = torch.empty(1, device="cuda")
        reds.append((x, dx, r))
        items.append(ax.batch_reduce(dx, int(n), r))
    t0 = time.time()
    auto = args.batch_prec == "auto"
    bh = ax.accx_batch_create(items, ax.ACC_BATCH_AUTOTUNE | (ax.ACC_BATCH_PREC_AUTO if auto else 0))
    create_s = time.time() - t0
    info = ax.accx_batch_info(bh)
    ts = _event_times(lambda: ax.accx_batch_launch(bh), args.steps, args.warmup)
    ms = float(np.median(ts))
    ax.accx_timing_enable(True)
    ax.accx_timing_read(reset=True)
    for _ in range(3):
        ax.accx_batch_launch_eager(bh)
    kt = {k: v[1] / v[0] for k, v in ax.accx_timing_read(reset=True).items()}
    ax.accx_timing_enable(False)
    # one call per item, no graph, for comparison
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for (_a, _b, da, db, dc, n) in mats:
        ax.accx_matmul_dev(ax.ACC_FLOAT32, da, db, dc, n,
                           ax.ACC_KERNEL_TILED | (ax.ACC_PREC_AUTO if auto else ax.ACC_PREC_FULL6))
    for (x, dx, r) in reds:
        ax.accx_reduce_sum_dev(ax.ACC_FLOAT32, dx, x.size, 0.0, r)
    torch.cuda.synchronize()
    per_item_ms = (time.perf_counter() - t0) * 1e3
    ax.accx_batch_launch(bh)
    torch.cuda.synchronize()
    g = synth.rng(seed, 77)
    got, ref, per_item = [], [], []
    for (a, b, _da, _db, dc, n) in mats:
        ii, jj = g.integers(0, n, 64), g.integers(0, n, 64)
        got.append(dc.cpu().numpy()[ii, jj])
        ref.append(oracle.matmul_at(a, b, ii, jj))
        per_item.append(float(np.linalg.norm(got[-1] - ref[-1]) / np.linalg.norm(ref[-1])))
    got, ref = np.concatenate(got), np.concatenate(ref)
    red_err = max(abs(float(r.item()) - oracle.sum_f32(x)) / oracle.sum_f32(x) for (x, _dx, r) in reds)
    ax.accx_batch_destroy(bh)
    ax.acc_shutdown()
    tf = info["flops"] / (ms * 1e-3) / 1e12
    mfma = info["mfma_flops"] / (ms * 1e-3) / 1e12
    print(json.dumps(_common(
        args, "batched matmul TFLOP/s (one graph launch: 512 matmuls + 256 reductions)", tf, "TFLOP/s", ms,
        {"workload": "batching: 512 float32 matmuls LEN in {64..1024} + 256 float32 reductions n in [2^16, 2^24]",
         "tile_threshold": info["tile_threshold"], "precision": args.batch_prec},
        batch=info, create_s=create_s, mfma_tflops=mfma, mfma_frac=mfma / PEAK_BF16_TFLOPS,
        reduce_gbs_if_alone=info["reduce_bytes"] / (ms * 1e-3) / 1e9, eager_kernels_ms=kt,
        one_call_per_item_ms=per_item_ms,
        accuracy={"matmul_rel_fro_sampled": float(np.linalg.norm(got - ref) / np.linalg.norm(ref)),
                  "matmul_rel_fro_max_per_item_64_samples": max(per_item),
                  "reduce_max_rel_err": red_err})))
    return 0


def run_rowblock(args) -> int:
    """One GPU's share of the LEN=4096 product split by row blocks over eight
    GPUs: C (512 x 4096) = A (512 x 4096) B (4096 x 4096), float32 on the
    bf16x3 path at the default scale workload's precision (--prec, AUTO by
    default) and int32 on the int8-limb path, through the rectangular entry
    point; error on sampled rows vs the float64 oracle.  The six-product
    GEMM on the same block is timed beside it for reference."""
    import numpy as np
    import torch

    import oracle
    import paper_1412_1127_amd as ax
    import synth
    m, n, k = 512, 4096, 4096
    seed = synth.DEFAULT_SEED
    a = synth.uniform_pm1_f32((m, k), seed, synth.STREAM_A)
    b = synth.uniform_pm1_f32((k, n), seed, synth.STREAM_B)
    ai = synth.int_uniform_i32((m, k), -16, 16, seed, synth.STREAM_A)
    bi = synth.int_uniform_i32((k, n), -16, 16, seed, synth.STREAM_B)
    ax.acc_init(0, 0)
    da, db = torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()
    dai, dbi = torch.from_numpy(ai).cuda(), torch.from_numpy(bi).cuda()
    dc = torch.empty((m, n), device="cuda")
    dci = torch.empty((m, n), dtype=torch.int32, device="cuda")
    prec = {"full6": ax.ACC_PREC_FULL6, "five": ax.ACC_PREC_FIVE, "auto": ax.ACC_PREC_AUTO,
            "cheap3": ax.ACC_PREC_CHEAP3}[args.prec]
    nprod = {"full6": 6, "five": 5, "auto": 3, "cheap3": 3}[args.prec]   # products of the dominant GEMM
    ff = ax.ACC_KERNEL_TILED | prec
    f6 = ax.ACC_KERNEL_TILED | ax.ACC_PREC_FULL6
    fi = ax.ACC_KERNEL_TILED
    tuned = {}
    if not args.no_autotune:
        tuned["f32"] = ax.accx_autotune_gemm(ax.ACC_FLOAT32, m, n, k, ff)
        tuned["i32"] = ax.accx_autotune_gemm(ax.ACC_INT32, m, n, k, ax.ACC_LIMBS(1))
        if ff != f6:
            ax.accx_autotune_gemm(ax.ACC_FLOAT32, m, n, k, f6)
    wf = torch.empty(max(ax.accx_gemm_workspace_size(ax.ACC_FLOAT32, m, n, k, ff),
                         ax.accx_gemm_workspace_size(ax.ACC_FLOAT32, m, n, k, f6)), dtype=torch.uint8, device="cuda")
    wi = torch.empty(ax.accx_gemm_workspace_size(ax.ACC_INT32, m, n, k, fi), dtype=torch.uint8, device="cuda")

    def step(fl=ff):
        ax.accx_gemm_dev(ax.ACC_FLOAT32, m, n, k, da, k, db, n, dc, n, fl, wf, wf.numel())
        ax.accx_gemm_dev(ax.ACC_INT32, m, n, k, dai, k, dbi, n, dci, n, fi, wi, wi.numel())

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # timed region: only the dominant kernel carries timing events; the
    # breakdown of the other kernels comes from extra steps afterwards
    ax.accx_timing_filter(["gemm_bf16x3"])
    ax.accx_timing_enable(True)
    ax.accx_timing_read(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    gm_t = ax.accx_timing_read(reset=True).get("gemm_bf16x3")
    ax.accx_timing_filter(None)
    nb = max(3, min(args.steps, 10))
    for _ in range(nb):
        step()
    torch.cuda.synchronize()
    kt = {kk: v[1] / v[0] for kk, v in ax.accx_timing_read(reset=True).items()}
    for _ in range(nb):
        ax.accx_gemm_dev(ax.ACC_FLOAT32, m, n, k, da, k, db, n, dc, n, f6, wf, wf.numel())
    torch.cuda.synchronize()
    kt6 = {kk: v[1] / v[0] for kk, v in ax.accx_timing_read(reset=True).items()}
    ax.accx_timing_enable(False)
    step()          # leave the --prec results in C for the accuracy check
    torch.cuda.synchronize()
    g = synth.rng(seed, 97)
    rows = np.unique(np.concatenate([[0, m - 1], g.integers(0, m, 30)]))
    ref = oracle.gemm(np.ascontiguousarray(a[rows]), b)
    refi = oracle.gemm(np.ascontiguousarray(ai[rows]), bi)
    c, ci = dc.cpu().numpy()[rows], dci.cpu().numpy()[rows]
    ax.acc_shutdown()
    ops = 2.0 * 2.0 * m * n * k
    gm = gm_t[1] / gm_t[0] if gm_t else None
    achieved = nprod * 2.0 * m * n * k / (gm * 1e-3) / 1e12 if gm else None
    gi = kt.get("gemm_i8")
    g6 = kt6.get("gemm_bf16x3")
    print(json.dumps(_common(
        args, "matmul TFLOP/s on one GPU's 512-row block of the LEN=4096 product", ops / (ms * 1e-3) / 1e12,
        "TFLOP/s", ms,
        {"workload": "row block: C (512 x 4096) = A (512 x 4096) B (4096 x 4096), float32 uniform[-1,1] and "
                     "int32 uniform [-16,16]", "m": m, "n": n, "k": k, "precision": args.prec,
         "tiles": {kk: {"tile": [t for t, v in ax.TILES.items() if v == tv][0], "tune_ms": tms}
                   for kk, (tv, tms) in tuned.items()}},
        dtype="f32 (bf16x3 matrix cores) + int32 (int8-limb matrix cores)",
        roofline={"kernel": "gemm_bf16x3", "bound": "mfma", "achieved": achieved, "peak": PEAK_BF16_TFLOPS,
                  "unit": "TFLOP/s", "frac": achieved / PEAK_BF16_TFLOPS if achieved else None,
                  "products": nprod, "avg_ms": gm},
        components={"f32_gemm_tflops_fp32_equiv": 2.0 * m * n * k / (gm * 1e-3) / 1e12 if gm else None,
                    "i32_gemm_tops": 2.0 * m * n * k / (gi * 1e-3) / 1e12 if gi else None,
                    "kernels_ms": kt,
                    "full6_gemm": {"ms": g6, "frac": 6 * 2.0 * m * n * k / (g6 * 1e-3) / 1e12 / PEAK_BF16_TFLOPS
                                   if g6 else None}},
        accuracy={"f32_rel_fro_vs_oracle_sampled_rows": float(np.linalg.norm(c - ref) / np.linalg.norm(ref)),
                  "i32_bit_exact_sampled_rows": bool(np.array_equal(ci, refi)), "rows_checked": int(rows.size)})))
    return 0


def run_reductions(args) -> int:
    """The reduction clause beyond float32 +: float64 and int64 sums, the
    SRAD statistics (sum and sum of squares of one float32 image in one
    pass), max and min together, and the logical-or flag of a sparse 0/1
    frontier; 1 GiB of input each, HBM GB/s per call vs the oracle."""
    import numpy as np
    import torch

    import oracle
    import paper_1412_1127_amd as ax
    import synth
    seed = synth.DEFAULT_SEED
    nb = 1 << 30
    cases = [
        ("f64_sum", ax.ACC_FLOAT64, lambda: synth.uniform_pm1_f64(nb // 8, seed, 31), [("sum", False)]),
        ("i64_sum", ax.ACC_INT64, lambda: synth.full_range_i64(nb // 8, seed, 32), [("sum", False)]),
        ("f32_srad_sum_sumsq", ax.ACC_FLOAT32, lambda: synth.uniform01_f32(nb // 4, seed, 33),
         [("sum", False), ("sum", True)]),
        ("f32_max_min", ax.ACC_FLOAT32, lambda: synth.uniform_pm1_f32((nb // 4,), seed, 34),
         [("max", False), ("min", False)]),
        ("i32_or_flag", ax.ACC_INT32, lambda: synth.sparse_flags_i32(nb // 4, 0.0, seed, 35), [("or", False)]),
    ]
    ops = {"sum": ax.ACC_RED_SUM, "max": ax.ACC_RED_MAX, "min": ax.ACC_RED_MIN, "or": ax.ACC_RED_OR}
    ax.acc_init(0, 0)
    out = {}
    for name, dt, gen, vars_ in cases:
        x = gen()
        dx = torch.from_numpy(x).cuda()
        res = torch.zeros(len(vars_), dtype=dx.dtype, device="cuda")
        v = [(ops[o], sq) for o, sq in vars_]
        init = [oracle.identity(o, x.dtype) for o, _ in vars_]
        ts = _event_times(lambda: ax.accx_reduce_dev(dt, dx, x.size, v, init, res), args.steps, args.warmup)
        got = res.cpu().numpy()
        ms = float(np.median(ts))
        errs = []
        for g, (o, sq), i0 in zip(got, vars_, init):
            ref = oracle.reduce(x, o, init=i0, square=sq)
            errs.append(abs(float(g) - ref) / max(abs(ref), 1e-300) if x.dtype.kind == "f" else int(int(g) != ref))
        out[name] = {"ms": ms, "gbs": nb / (ms * 1e-3) / 1e9, "frac_hbm": nb / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS,
                     "max_rel_err_or_mismatch": max(errs)}
        del dx
    ax.acc_shutdown()
    srad = out["f32_srad_sum_sumsq"]
    print(json.dumps(_common(
        args, "reduction GB/s (1 GiB per call; operators and types beyond float32 +)", srad["gbs"], "GB/s",
        srad["ms"], {"workload": "reductions: float64 / int64 sums, SRAD sum + sum of squares, max + min, "
                                 "logical-or flag; 1 GiB each", "bytes_per_call": nb},
        dtype="f32 / f64 / i32 / i64", cases=out)))
    return 0


def run_serve(args) -> int:
    """Poisson 2000 requests/s of offload-region requests through the
    serving engine; latency from scheduled arrival to completion."""
    import numpy as np

    import oracle
    import paper_1412_1127_amd as ax
    from paper_1412_1127_amd import serve
    import synth
    ax.acc_init(0, 0)
    wl = serve.make_workload(args.requests, synth.DEFAULT_SEED)
    pools = serve.Pools(wl)
    g = synth.rng(synth.DEFAULT_SEED, 4)
    picked = []
    # Entries checked per request.  From 8 entries the estimate is a ratio of
    # two 8-term sums of squares, whose maximum over a thousand requests runs
    # to 3x the true error.  The oracle runs after the timed pass.
    nsamp = 256

    def check(r, view):
        c = view.numpy().reshape(r.n, r.n)
        ii, jj = g.integers(0, r.n, nsamp), g.integers(0, r.n, nsamp)
        picked.append((r, ii, jj, c[ii, jj].copy()))
    serve.run(wl, pools, slots=8, budget=64 << 30)  # warm-up pass (kernels, block cache)
    res = serve.run(wl, pools, slots=8, budget=64 << 30, on_region_done=check)
    ax.acc_shutdown()
    errs, exact, e2, r2 = [], [], 0.0, 0.0
    for r, ii, jj, got in picked:
        a, b = pools.inputs(r)
        ref = oracle.matmul_at(a.numpy().reshape(r.n, r.n), b.numpy().reshape(r.n, r.n), ii, jj)
        if r.dtype == ax.ACC_INT32:
            exact.append(bool(np.array_equal(got, ref)))
        else:
            d = float(np.sum((got.astype(np.float64) - ref) ** 2))
            n2 = float(np.sum(np.asarray(ref, np.float64) ** 2))
            errs.append((d / n2) ** 0.5)
            e2, r2 = e2 + d, r2 + n2
    rr = res.pop("reduce_results")
    red = [abs(rr[q.tag] - oracle.sum_f32(pools.inputs(wl.regions[q.region])[0].numpy(), q.init)) /
           oracle.sum_f32(pools.inputs(wl.regions[q.region])[0].numpy(), q.init)
           for q in wl.requests[:400] if q.tag in rr]
    print(json.dumps(_common(
        args, "serving p50 latency (ms) at 2000 requests/s; p99 and throughput alongside", res["latency_ms"]["p50"],
        "ms", res["latency_ms"]["p50"],
        {"workload": "serving: Poisson 2000 req/s, 70% matmuls (LEN log-uniform [128, 2048], float32/int32), "
                     "30% reductions (n log-uniform [2^16, 2^26]), 4 requests per region, 64 GB budget",
         "requests": args.requests, "slots": 8},
        higher=False, latency_ms=res["latency_ms"], serving=res,
        accuracy={"matmul_f32_max_rel_fro_sampled": max(errs) if errs else None,
                  "matmul_f32_pooled_rel_fro_sampled": (e2 / r2) ** 0.5 if r2 else None,
                  "samples_per_request": nsamp,
                  "matmul_i32_bit_exact_sampled": all(exact), "reduce_max_rel_err": max(red) if red else None})))
    return 0


def run_regions(args) -> int:
    """The data directive around the worked example (section 1.3): a region
    with copyin(a, b) and copyout(c) for a LEN=4096 float32 matmul, from
    pageable numpy arrays and from page-locked host memory, plus the update
    directive on a subrange.  Host<->device bytes over PCIe are in every
    time here: these rates are transfer rates, not the kernel's."""
    import ctypes

    import numpy as np

    import oracle
    import paper_1412_1127_amd as ax
    import synth
    ax.acc_init(0, 0)
    n = args.len
    seed = synth.DEFAULT_SEED
    a0 = synth.uniform_pm1_f32((n, n), seed, synth.STREAM_A)
    b0 = synth.uniform_pm1_f32((n, n), seed, synth.STREAM_B)
    nbytes = n * n * 4
    flags = ax.ACC_KERNEL_TILED | ax.ACC_PREC_AUTO
    out, pinned = {}, []
    try:
        for mode in ("pageable", "pinned"):
            if mode == "pageable":
                a, b, c = a0.copy(), b0.copy(), np.zeros((n, n), np.float32)
            else:
                bufs = []
                for _ in range(3):
                    p_ = ax.accx_host_alloc(nbytes)
                    pinned.append(p_)
                    bufs.append(np.ctypeslib.as_array((ctypes.c_float * (n * n)).from_address(p_)).reshape(n, n))
                a, b, c = bufs
                a[:], b[:], c[:] = a0, b0, 0.0
            cl = [ax.clause(ax.ACC_COPYIN, ax.ACC_FLOAT32, a), ax.clause(ax.ACC_COPYIN, ax.ACC_FLOAT32, b),
                  ax.clause(ax.ACC_COPYOUT, ax.ACC_FLOAT32, c)]
            tin, tk, tout, tup = [], [], [], []
            for it in range(args.warmup + args.steps):
                t0 = time.perf_counter()
                r = ax.acc_data_begin(cl)
                ax.acc_wait(r)
                t1 = time.perf_counter()
                ax.acc_loopnest_matmul(r, ax.ACC_FLOAT32, a, b, c, n, flags)
                ax.acc_wait(r)
                t2 = time.perf_counter()
                ax.acc_update(r, ax.ACC_UPDATE_DEVICE, ax.ACC_FLOAT32, a, 0, n * n // 4)   # a quarter of a
                t3 = time.perf_counter()
                ax.acc_data_end(r)
                t4 = time.perf_counter()
                if it >= args.warmup:
                    tin.append(t1 - t0), tk.append(t2 - t1), tup.append(t3 - t2), tout.append(t4 - t3)
            g = synth.rng(seed, 99)
            ii, jj = g.integers(0, n, 1024), g.integers(0, n, 1024)
            ref = oracle.matmul_at(a0, b0, ii, jj)
            med = lambda v: float(np.median(v))
            out[mode] = {"copyin_gbs": 2 * nbytes / med(tin) / 1e9, "copyout_gbs": nbytes / med(tout) / 1e9,
                         "update_device_gbs": nbytes / 4 / med(tup) / 1e9, "matmul_ms": med(tk) * 1e3,
                         "region_ms": (med(tin) + med(tk) + med(tup) + med(tout)) * 1e3,
                         "rel_fro_vs_oracle_sampled": float(np.linalg.norm(c[ii, jj] - ref) / np.linalg.norm(ref))}
    finally:
        for p_ in pinned:
            ax.accx_host_free(p_)
        ax.acc_shutdown()
    best = out["pinned"]
    print(json.dumps(_common(
        args, "data-region host<->device GB/s (copyin, pinned host memory)", best["copyin_gbs"], "GB/s",
        best["region_ms"], {"workload": "data region around the LEN=%d float32 matmul: copyin(a, b), copyout(c), "
                                         "update device on a quarter of a" % n, "len": n},
        modes=out)))
    return 0


def main() -> int:
    args = _args()
    if args.ingest_counters:
        return ingest_counters(args.ingest_counters, args.prec)
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: every step of this offload path runs on a single device, "
              "and no multi-GPU form is built; run with --gpus 1.", file=sys.stderr)
        return 2
    return {"scale": run_scale, "small": run_small, "precision": run_precision, "batch": run_batch,
            "serve": run_serve, "rowblock": run_rowblock, "reductions": run_reductions,
            "regions": run_regions}[args.workload](args)


if __name__ == "__main__":
    sys.exit(main())
