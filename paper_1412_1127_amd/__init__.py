"""Python binding of libaccx (include/accx.h): argument marshalling only.

Every step of the hot path runs in the HIP kernels of ``libaccx.so``; this
module only converts Python arguments to the C ABI and raises ``AccxError`` on
a failing status.  The names match the C entry points.

torch is imported first so that libaccx binds to the same HIP runtime that
torch loaded: device memory and streams handed over from torch tensors are
then valid inside the library.  There is no fallback: if ``libaccx.so`` has
not been built, importing this package fails.
"""
from __future__ import annotations

import ctypes
import os

import torch  # noqa: F401  (HIP runtime shared with libaccx)

_HERE = os.path.dirname(os.path.abspath(__file__))
# ACCX_LIB: another build of the same library to load instead (the sanitizer
# test's build with AddressSanitizer / UndefinedBehaviorSanitizer host code).
LIB_PATH = os.environ.get("ACCX_LIB") or os.path.join(_HERE, "libaccx.so")

# ---- constants (mirror include/accx.h) ------------------------------------
ACC_OK = 0
ACC_ERR_INVALID_ARG = -1
ACC_ERR_NOT_PRESENT = -2
ACC_ERR_ALREADY_PRESENT = -3
ACC_ERR_OUT_OF_MEMORY = -4
ACC_ERR_DEVICE = -5
ACC_ERR_NO_DEVICE = -6

ACC_COPY, ACC_COPYIN, ACC_COPYOUT, ACC_CREATE = 0, 1, 2, 3
ACC_PRESENT, ACC_PRESENT_OR_COPY, ACC_PRESENT_OR_COPYIN, ACC_PRESENT_OR_COPYOUT, ACC_PRESENT_OR_CREATE = 4, 5, 6, 7, 8
ACC_UPDATE_HOST, ACC_UPDATE_DEVICE = 0, 1
ACC_FLOAT32, ACC_INT32, ACC_FLOAT64, ACC_INT64 = 0, 1, 2, 3
ACC_RED_SUM, ACC_RED_MAX, ACC_RED_MIN, ACC_RED_OR = 0, 1, 2, 3
ACC_MAX_REDUCE_VARS = 4

ACC_KERNEL_AUTO = 0x0
ACC_KERNEL_PLAIN = 0x1
ACC_KERNEL_PLAIN_LISTING1B = 0x2
ACC_KERNEL_TILED = 0x3
ACC_PREC_AUTO = 0x00
ACC_PREC_FULL6 = 0x10
ACC_PREC_CHEAP3 = 0x20
ACC_PREC_FIVE = 0x30
ACC_PREC_F32MFMA = 0x40
ACC_LIMBS_SHIFT = 8
ACC_ASYNC = 0x1000
ACC_REDUCE_FAST = 0x0
ACC_REDUCE_PLAIN = 0x1
ACC_TILE_SHIFT = 16
ACC_TILE_AUTO = 0x00000
ACC_TILE_256 = 0x10000
ACC_TILE_256x128 = 0x20000
ACC_TILE_128 = 0x30000
ACC_TILE_64 = 0x40000
ACC_SERVE_MATMUL = 0
ACC_SERVE_REDUCE = 1
ACC_BATCH_MATMUL = 0
ACC_BATCH_REDUCE = 1
ACC_BATCH_AUTOTUNE = 0x1
ACC_BATCH_PREC_AUTO = 0x2
ACC_TILE_256W4 = 0x50000
TILES = {"256": ACC_TILE_256, "256x128": ACC_TILE_256x128, "128": ACC_TILE_128, "64": ACC_TILE_64,
         "256w4": ACC_TILE_256W4}


def ACC_LIMBS(n: int) -> int:
    return (int(n) & 0xF) << ACC_LIMBS_SHIFT


class AccxError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__("%s: %s (%s)" % (where, status_string(status), detail))
        self.status = status


class accx_kernel_time(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 48), ("launches", ctypes.c_int64), ("total_ms", ctypes.c_double),
                ("min_ms", ctypes.c_double), ("max_ms", ctypes.c_double)]


class accx_probe_record(ctypes.Structure):
    _fields_ = [("rows", ctypes.c_int32 * 8), ("cols", ctypes.c_int32 * 8), ("ref", ctypes.c_double * 64),
                ("err2", ctypes.c_double), ("ref2", ctypes.c_double), ("corrected", ctypes.c_int32),
                ("pad", ctypes.c_int32 * 3)]


class accx_batch_item(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("dtype", ctypes.c_int32), ("a", ctypes.c_void_p), ("b", ctypes.c_void_p),
                ("c", ctypes.c_void_p), ("n", ctypes.c_int64), ("init", ctypes.c_float), ("flags", ctypes.c_uint32)]


class accx_batch_info_t(ctypes.Structure):
    _fields_ = [("units", ctypes.c_int64), ("tiles", ctypes.c_int64), ("chunks", ctypes.c_int64),
                ("tile_threshold", ctypes.c_int64), ("workgroups", ctypes.c_int32), ("matmuls", ctypes.c_int32), ("reductions", ctypes.c_int32),
                ("pad", ctypes.c_int32), ("device_bytes", ctypes.c_uint64), ("flops", ctypes.c_double),
                ("mfma_flops", ctypes.c_double), ("reduce_bytes", ctypes.c_double)]


class accx_request(ctypes.Structure):
    _fields_ = [("op", ctypes.c_int32), ("dtype", ctypes.c_int32), ("region", ctypes.c_int64),
                ("first", ctypes.c_int32), ("last", ctypes.c_int32), ("a", ctypes.c_void_p), ("b", ctypes.c_void_p),
                ("c", ctypes.c_void_p), ("n", ctypes.c_int64), ("init", ctypes.c_double), ("flags", ctypes.c_uint32),
                ("pad", ctypes.c_uint32), ("tag", ctypes.c_uint64)]


class accx_completion(ctypes.Structure):
    _fields_ = [("tag", ctypes.c_uint64), ("status", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("t_submit", ctypes.c_double), ("t_start", ctypes.c_double), ("t_done", ctypes.c_double)]


class accx_server_stats_t(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("admitted", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("rejected", ctypes.c_int64), ("regions_open", ctypes.c_int64), ("max_inflight", ctypes.c_int64),
                ("max_regions_open", ctypes.c_int64), ("budget_used", ctypes.c_uint64),
                ("budget_peak", ctypes.c_uint64), ("blocks_held", ctypes.c_uint64),
                ("blocks_held_peak", ctypes.c_uint64)]


class acc_reduce_var(ctypes.Structure):
    _fields_ = [("op", ctypes.c_int32), ("square", ctypes.c_int32)]


class acc_clause(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("dtype", ctypes.c_int32), ("host", ctypes.c_void_p),
                ("start", ctypes.c_int64), ("n", ctypes.c_int64)]


if not os.path.exists(LIB_PATH):
    raise ImportError("libaccx.so is not built (%s); run `python paper_1412_1127_amd/build.py` "
                      "or __graft_entry__.build()" % LIB_PATH)

_lib = ctypes.CDLL(LIB_PATH)

_i32, _i64, _u32, _u64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64
_vp, _sz = ctypes.c_void_p, ctypes.c_size_t

# name -> argtypes (every entry point returns acc_status unless listed below)
_SIGS = {
    "acc_init": [ctypes.c_int, _u64],
    "acc_shutdown": [],
    "acc_budget_used": [ctypes.POINTER(_u64)],
    "accx_set_allocator": [_vp, _vp, _vp],
    "acc_data_begin": [ctypes.POINTER(acc_clause), ctypes.c_int, _vp, ctypes.POINTER(_vp)],
    "acc_data_end": [_vp],
    "acc_wait": [_vp],
    "acc_deviceptr": [_vp, ctypes.POINTER(_vp)],
    "acc_update": [_vp, ctypes.c_int, ctypes.c_int, _vp, _i64, _i64, _u32],
    "acc_is_present": [_vp, _sz, ctypes.POINTER(ctypes.c_int)],
    "accx_host_alloc": [_sz, ctypes.POINTER(_vp)],
    "accx_host_free": [_vp],
    "acc_loopnest_matmul": [_vp, ctypes.c_int, _vp, _vp, _vp, _i64, _u32],
    "acc_loopnest_gemm": [_vp, ctypes.c_int, _i64, _i64, _i64, _vp, _i64, _vp, _i64, _vp, _i64, _u32],
    "acc_reduce_sum": [_vp, ctypes.c_int, _vp, _i64, _vp, _u32],
    "acc_reduce": [_vp, ctypes.c_int, _vp, _i64, ctypes.POINTER(acc_reduce_var), ctypes.c_int, _vp, _u32],
    "accx_matmul_workspace_size": [ctypes.c_int, _i64, _u32, ctypes.POINTER(_sz)],
    "accx_matmul_dev": [ctypes.c_int, _vp, _vp, _vp, _i64, _u32, _vp, _sz, _vp],
    "accx_gemm_workspace_size": [ctypes.c_int, _i64, _i64, _i64, _u32, ctypes.POINTER(_sz)],
    "accx_gemm_dev": [ctypes.c_int, _i64, _i64, _i64, _vp, _i64, _vp, _i64, _vp, _i64, _u32, _vp, _sz, _vp],
    "accx_reduce_workspace_size": [ctypes.c_int, _i64, _u32, ctypes.POINTER(_sz)],
    "accx_reduce_sum_dev": [ctypes.c_int, _vp, _i64, _vp, _vp, _u32, _vp, _sz, _vp],
    "accx_reduce_vars_workspace_size": [ctypes.c_int, _i64, ctypes.POINTER(acc_reduce_var), ctypes.c_int, _u32,
                                        ctypes.POINTER(_sz)],
    "accx_reduce_dev": [ctypes.c_int, _vp, _i64, ctypes.POINTER(acc_reduce_var), ctypes.c_int, _vp, _vp, _u32, _vp,
                        _sz, _vp],
    "accx_reduce_dev_noalloc": [ctypes.c_int, _vp, _i64, ctypes.POINTER(acc_reduce_var), ctypes.c_int, _vp, _vp,
                                _u32, _vp],
    "accx_matmul_reduce_dev": [_vp, _vp, _vp, _i64, _u32, _vp, _i64, ctypes.c_float, _vp, _vp, _sz, _vp],
    "accx_matmul_reduce_workspace_size": [_i64, _u32, _i64, ctypes.POINTER(_sz)],
    "accx_onbox_mfma": [ctypes.c_int, _i64, ctypes.POINTER(ctypes.c_double), _vp],
    "accx_onbox_read": [_vp, _i64, _vp],
    "accx_packed_size": [ctypes.c_int, _i64, _i64, ctypes.c_int, ctypes.POINTER(_sz)],
    "accx_pack_dev": [ctypes.c_int, _vp, _i64, _i64, ctypes.c_int, ctypes.c_int, _vp, _sz, _vp],
    "accx_batch_create": [ctypes.POINTER(accx_batch_item), ctypes.c_int, _u32, ctypes.POINTER(_vp)],
    "accx_batch_launch": [_vp, _vp],
    "accx_batch_launch_eager": [_vp, _vp],
    "accx_batch_info": [_vp, ctypes.POINTER(accx_batch_info_t)],
    "accx_batch_destroy": [_vp],
    "accx_server_create": [ctypes.c_int, _u64, ctypes.POINTER(_vp)],
    "accx_server_submit": [_vp, ctypes.POINTER(accx_request)],
    "accx_server_poll": [_vp, ctypes.POINTER(accx_completion), ctypes.c_int, ctypes.POINTER(ctypes.c_int)],
    "accx_server_drain": [_vp],
    "accx_server_now": [_vp, ctypes.POINTER(ctypes.c_double)],
    "accx_server_stats": [_vp, ctypes.POINTER(accx_server_stats_t)],
    "accx_server_destroy": [_vp],
    "accx_probe_layout": [_i64, _u32, ctypes.POINTER(_sz), ctypes.POINTER(ctypes.c_int)],
    "accx_gemm_probe_layout": [_i64, _i64, _i64, _u32, ctypes.POINTER(_sz), ctypes.POINTER(ctypes.c_int)],
    "accx_autotune": [ctypes.c_int, _i64, _u32, ctypes.POINTER(_u32), ctypes.POINTER(ctypes.c_double)],
    "accx_autotune_gemm": [ctypes.c_int, _i64, _i64, _i64, _u32, ctypes.POINTER(_u32),
                           ctypes.POINTER(ctypes.c_double)],
    "accx_tune_save": [ctypes.c_char_p],
    "accx_tune_load": [ctypes.c_char_p],
    "accx_timing_enable": [ctypes.c_int],
    "accx_timing_filter": [ctypes.c_char_p],
    "accx_timing_read": [_vp, ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.c_int],
}
_STRINGS = {"acc_status_string": [ctypes.c_int], "acc_last_error_string": [], "accx_version": []}

for _name, _args in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = ctypes.c_int
for _name, _args in _STRINGS.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = ctypes.c_char_p

EXPORTED = tuple(_SIGS) + tuple(_STRINGS)
FEATURES = ("plain", "tiled")


def status_string(s: int) -> str:
    return _lib.acc_status_string(int(s)).decode()


def last_error_string() -> str:
    return _lib.acc_last_error_string().decode()


def version() -> str:
    return _lib.accx_version().decode()


def _check(status: int, where: str) -> None:
    if status != ACC_OK:
        raise AccxError(status, where, last_error_string())


def _addr(p) -> int | None:
    """Address of a numpy array, torch tensor, ctypes object or plain int."""
    if p is None:
        return None
    if isinstance(p, int):
        return p
    if hasattr(p, "data_ptr"):
        return int(p.data_ptr())
    if hasattr(p, "ctypes"):
        return int(p.ctypes.data)
    return ctypes.addressof(p)


def _stream(s) -> int | None:
    if s is None:
        return None
    if isinstance(s, int):
        return s
    return int(s.cuda_stream)


# ---- entry points ----------------------------------------------------------

def acc_init(device: int = 0, hbm_budget_bytes: int = 0) -> None:
    _check(_lib.acc_init(int(device), int(hbm_budget_bytes)), "acc_init")


def acc_shutdown() -> None:
    _check(_lib.acc_shutdown(), "acc_shutdown")


def acc_budget_used() -> int:
    v = _u64(0)
    _check(_lib.acc_budget_used(ctypes.byref(v)), "acc_budget_used")
    return int(v.value)


def clause(kind: int, dtype: int, host, start: int = 0, n: int | None = None) -> acc_clause:
    """One data clause host[start:n]; n defaults to the array's size."""
    if n is None:
        n = int(host.size) - int(start)
    return acc_clause(int(kind), int(dtype), _addr(host), int(start), int(n))


def acc_data_begin(clauses, stream=None) -> int:
    arr = (acc_clause * max(1, len(clauses)))(*clauses)
    out = _vp(0)
    _check(_lib.acc_data_begin(arr, len(clauses), _stream(stream), ctypes.byref(out)), "acc_data_begin")
    return int(out.value)


def acc_data_end(region: int) -> None:
    _check(_lib.acc_data_end(region), "acc_data_end")


def acc_wait(region: int) -> None:
    _check(_lib.acc_wait(region), "acc_wait")


def acc_deviceptr(host) -> int:
    out = _vp(0)
    _check(_lib.acc_deviceptr(_addr(host), ctypes.byref(out)), "acc_deviceptr")
    return int(out.value or 0)


def acc_update(region: int, direction: int, dtype: int, host, start: int = 0, n: int | None = None,
               flags: int = 0) -> None:
    """host: numpy array (n defaults to its size - start) or an address."""
    if n is None:
        n = int(host.size) - int(start)
    _check(_lib.acc_update(region, int(direction), int(dtype), _addr(host), int(start), int(n), int(flags)),
           "acc_update")


def acc_is_present(host, nbytes: int | None = None) -> bool:
    if nbytes is None:
        nbytes = int(host.nbytes)
    out = ctypes.c_int(0)
    _check(_lib.acc_is_present(_addr(host), int(nbytes), ctypes.byref(out)), "acc_is_present")
    return bool(out.value)


_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)
_allocator_refs = []   # the callbacks stay referenced while the library may call them


def accx_set_allocator(alloc=None, free=None) -> None:
    """Device memory for the library from Python callables: alloc(nbytes) ->
    device address (int, 256-byte aligned; 0 on failure), free(address).
    Both None: back to hipMalloc / hipFree."""
    if (alloc is None) != (free is None):
        raise ValueError("give both alloc and free, or neither")
    if alloc is None:
        _check(_lib.accx_set_allocator(None, None, None), "accx_set_allocator")
        return
    fa = _ALLOC_FN(lambda nbytes, _ctx: int(alloc(int(nbytes)) or 0))
    ff = _FREE_FN(lambda ptr, _ctx: free(int(ptr)))
    _allocator_refs.append((fa, ff))
    _check(_lib.accx_set_allocator(ctypes.cast(fa, _vp), ctypes.cast(ff, _vp), None), "accx_set_allocator")


class TorchAllocator:
    """Routes the library's device allocations through torch's caching
    allocator: each block is a uint8 tensor kept alive until the library
    frees it.  `live` holds the blocks the library currently owns."""

    def __init__(self):
        self.live = {}
        self.allocs = 0
        self.frees = 0

    def alloc(self, nbytes: int) -> int:
        t = torch.empty(max(1, nbytes), dtype=torch.uint8, device="cuda")
        self.live[t.data_ptr()] = t
        self.allocs += 1
        return t.data_ptr()

    def free(self, ptr: int) -> None:
        self.live.pop(ptr)
        self.frees += 1

    def install(self) -> "TorchAllocator":
        accx_set_allocator(self.alloc, self.free)
        return self


def accx_host_alloc(nbytes: int) -> int:
    """Address of `nbytes` of page-locked host memory (free with accx_host_free)."""
    out = _vp(0)
    _check(_lib.accx_host_alloc(int(nbytes), ctypes.byref(out)), "accx_host_alloc")
    return int(out.value)


def accx_host_free(addr: int) -> None:
    _check(_lib.accx_host_free(addr), "accx_host_free")


def acc_loopnest_matmul(region: int, dtype: int, a, b, c, length: int, flags: int = 0) -> None:
    _check(_lib.acc_loopnest_matmul(region, int(dtype), _addr(a), _addr(b), _addr(c), int(length), int(flags)),
           "acc_loopnest_matmul")


def acc_loopnest_gemm(region: int, dtype: int, m: int, n: int, k: int, a, lda: int, b, ldb: int, c, ldc: int,
                      flags: int = 0) -> None:
    _check(_lib.acc_loopnest_gemm(region, int(dtype), int(m), int(n), int(k), _addr(a), int(lda), _addr(b), int(ldb),
                                  _addr(c), int(ldc), int(flags)), "acc_loopnest_gemm")


def acc_reduce_sum(region: int, dtype: int, x, n: int, inout, flags: int = 0) -> None:
    """inout: a one-element numpy array (float32 or int32) or ctypes scalar, updated in place."""
    _check(_lib.acc_reduce_sum(region, int(dtype), _addr(x), int(n), _addr(inout), int(flags)), "acc_reduce_sum")


def accx_matmul_workspace_size(dtype: int, length: int, flags: int = 0) -> int:
    v = _sz(0)
    _check(_lib.accx_matmul_workspace_size(int(dtype), int(length), int(flags), ctypes.byref(v)),
           "accx_matmul_workspace_size")
    return int(v.value)


def accx_matmul_dev(dtype: int, dA, dB, dC, length: int, flags: int = 0, work=None, work_bytes: int = 0,
                    stream=None) -> None:
    _check(_lib.accx_matmul_dev(int(dtype), _addr(dA), _addr(dB), _addr(dC), int(length), int(flags),
                                _addr(work), int(work_bytes), _stream(stream)), "accx_matmul_dev")


def accx_gemm_workspace_size(dtype: int, m: int, n: int, k: int, flags: int = 0) -> int:
    v = _sz(0)
    _check(_lib.accx_gemm_workspace_size(int(dtype), int(m), int(n), int(k), int(flags), ctypes.byref(v)),
           "accx_gemm_workspace_size")
    return int(v.value)


def accx_gemm_dev(dtype: int, m: int, n: int, k: int, dA, lda: int, dB, ldb: int, dC, ldc: int, flags: int = 0,
                  work=None, work_bytes: int = 0, stream=None) -> None:
    _check(_lib.accx_gemm_dev(int(dtype), int(m), int(n), int(k), _addr(dA), int(lda), _addr(dB), int(ldb),
                              _addr(dC), int(ldc), int(flags), _addr(work), int(work_bytes), _stream(stream)),
           "accx_gemm_dev")


def accx_reduce_workspace_size(dtype: int, n: int, flags: int = 0) -> int:
    v = _sz(0)
    _check(_lib.accx_reduce_workspace_size(int(dtype), int(n), int(flags), ctypes.byref(v)),
           "accx_reduce_workspace_size")
    return int(v.value)


_CTYPE = {ACC_FLOAT32: ctypes.c_float, ACC_INT32: ctypes.c_int32, ACC_FLOAT64: ctypes.c_double,
          ACC_INT64: ctypes.c_int64}


def _values(dtype: int, vals):
    """A host array of the element type holding `vals`."""
    ct = _CTYPE[int(dtype)]
    conv = float if dtype in (ACC_FLOAT32, ACC_FLOAT64) else int
    return (ct * len(vals))(*[conv(v) for v in vals])


def _vars(vars_):
    """[(op, square), ...] or acc_reduce_var instances -> ctypes array."""
    out = (acc_reduce_var * len(vars_))()
    for i, v in enumerate(vars_):
        out[i] = v if isinstance(v, acc_reduce_var) else acc_reduce_var(int(v[0]), int(v[1]))
    return out


def acc_reduce(region: int, dtype: int, x, n: int, vars_, inout, flags: int = 0) -> None:
    """vars_: [(op, square), ...]; inout: a numpy array of len(vars_) elements of the dtype, updated in place."""
    v = _vars(vars_)
    _check(_lib.acc_reduce(region, int(dtype), _addr(x), int(n), v, len(v), _addr(inout), int(flags)), "acc_reduce")


def accx_reduce_vars_workspace_size(dtype: int, n: int, vars_, flags: int = 0) -> int:
    v = _vars(vars_)
    out = _sz(0)
    _check(_lib.accx_reduce_vars_workspace_size(int(dtype), int(n), v, len(v), int(flags), ctypes.byref(out)),
           "accx_reduce_vars_workspace_size")
    return int(out.value)


def accx_reduce_dev(dtype: int, dX, n: int, vars_, init, dResult, flags: int = 0, work=None, work_bytes: int = 0,
                    stream=None) -> None:
    """init: Python numbers, one per variable; dResult: len(vars_) device elements of the dtype."""
    v = _vars(vars_)
    iv = _values(dtype, init)
    _check(_lib.accx_reduce_dev(int(dtype), _addr(dX), int(n), v, len(v), iv, _addr(dResult), int(flags),
                                _addr(work), int(work_bytes), _stream(stream)), "accx_reduce_dev")


def accx_onbox_mfma(kind: int, rounds: int, stream=None) -> float:
    """Enqueue the matrix-instruction-only loop (0: bf16, 1: int8); returns its operation count."""
    ops = ctypes.c_double(0.0)
    _check(_lib.accx_onbox_mfma(int(kind), int(rounds), ctypes.byref(ops), _stream(stream)), "accx_onbox_mfma")
    return float(ops.value)


def accx_onbox_read(dX, nbytes: int, stream=None) -> None:
    """Enqueue a read-only stream of nbytes at dX."""
    _check(_lib.accx_onbox_read(_addr(dX), int(nbytes), _stream(stream)), "accx_onbox_read")


def accx_reduce_dev_noalloc(dtype: int, dX, n: int, vars_, init, dResult, flags: int = 0, stream=None) -> None:
    """accx_reduce_dev with the library's static device scratch instead of a workspace (allocates nothing)."""
    v = _vars(vars_)
    iv = _values(dtype, init)
    _check(_lib.accx_reduce_dev_noalloc(int(dtype), _addr(dX), int(n), v, len(v), iv, _addr(dResult), int(flags),
                                        _stream(stream)), "accx_reduce_dev_noalloc")


def accx_reduce_sum_dev(dtype: int, dX, n: int, init, dResult, flags: int = 0, work=None, work_bytes: int = 0,
                        stream=None) -> None:
    """init: a Python number (marshalled to a host value of the dtype)."""
    iv = _CTYPE[int(dtype)](float(init) if dtype in (ACC_FLOAT32, ACC_FLOAT64) else int(init))
    _check(_lib.accx_reduce_sum_dev(int(dtype), _addr(dX), int(n), ctypes.byref(iv), _addr(dResult), int(flags),
                                    _addr(work), int(work_bytes), _stream(stream)), "accx_reduce_sum_dev")


def accx_matmul_reduce_workspace_size(len_: int, flags: int, n: int) -> int:
    v = _sz(0)
    _check(_lib.accx_matmul_reduce_workspace_size(int(len_), int(flags), int(n), ctypes.byref(v)),
           "accx_matmul_reduce_workspace_size")
    return int(v.value)


def accx_matmul_reduce_dev(dA, dB, dC, len_: int, flags: int, dX, n: int, init: float, dResult, work=None,
                           work_bytes: int = 0, stream=None) -> None:
    """float32 matmul nest and reduction(+) nest in one region (the sum may ride in the matmul's launch)."""
    _check(_lib.accx_matmul_reduce_dev(_addr(dA), _addr(dB), _addr(dC), int(len_), int(flags), _addr(dX), int(n),
                                       float(init), _addr(dResult), _addr(work), int(work_bytes), _stream(stream)),
           "accx_matmul_reduce_dev")


def accx_packed_size(dtype: int, rows: int, k: int, planes: int) -> int:
    v = _sz(0)
    _check(_lib.accx_packed_size(int(dtype), int(rows), int(k), int(planes), ctypes.byref(v)), "accx_packed_size")
    return int(v.value)


def accx_pack_dev(dtype: int, dX, rows: int, k: int, transposed: bool, planes: int, dOut, out_bytes: int,
                  stream=None) -> None:
    _check(_lib.accx_pack_dev(int(dtype), _addr(dX), int(rows), int(k), int(bool(transposed)), int(planes),
                              _addr(dOut), int(out_bytes), _stream(stream)), "accx_pack_dev")


def accx_timing_enable(on: bool = True) -> None:
    _check(_lib.accx_timing_enable(int(bool(on))), "accx_timing_enable")


def accx_timing_filter(names=None) -> None:
    """Time only the kernels in `names` (an iterable of timing names); None: all."""
    arg = None if not names else ",".join(names).encode()
    _check(_lib.accx_timing_filter(arg), "accx_timing_filter")


def accx_timing_read(reset: bool = False) -> dict:
    """{kernel name: (launches, total_ms, min_ms, max_ms)}; synchronizes on the recorded events."""
    cap = 64
    buf = (accx_kernel_time * cap)()
    n = ctypes.c_int(0)
    _check(_lib.accx_timing_read(buf, cap, ctypes.byref(n), int(bool(reset))), "accx_timing_read")
    return {buf[i].name.decode(): (int(buf[i].launches), float(buf[i].total_ms), float(buf[i].min_ms),
                                   float(buf[i].max_ms)) for i in range(min(cap, n.value))}


def accx_autotune(dtype: int, length: int, flags: int = 0):
    """Time every tile configuration for (dtype, length, flags); returns (ACC_TILE_* chosen, ms)."""
    tile = _u32(0)
    ms = ctypes.c_double(0)
    _check(_lib.accx_autotune(int(dtype), int(length), int(flags), ctypes.byref(tile), ctypes.byref(ms)),
           "accx_autotune")
    return int(tile.value), float(ms.value)


def accx_autotune_gemm(dtype: int, m: int, n: int, k: int, flags: int = 0):
    """Time every tile configuration for (dtype, m, n, k, flags); returns (ACC_TILE_* chosen, ms)."""
    tile = _u32(0)
    ms = ctypes.c_double(0)
    _check(_lib.accx_autotune_gemm(int(dtype), int(m), int(n), int(k), int(flags), ctypes.byref(tile),
                                   ctypes.byref(ms)), "accx_autotune_gemm")
    return int(tile.value), float(ms.value)


def accx_tune_save(path: str) -> None:
    _check(_lib.accx_tune_save(os.fsencode(path)), "accx_tune_save")


def accx_tune_load(path: str) -> None:
    _check(_lib.accx_tune_load(os.fsencode(path)), "accx_tune_load")


def accx_probe_layout(length: int, flags: int):
    """(byte offset of the probe records in the matmul workspace, record count)."""
    off = _sz(0)
    cnt = ctypes.c_int(0)
    _check(_lib.accx_probe_layout(int(length), int(flags), ctypes.byref(off), ctypes.byref(cnt)), "accx_probe_layout")
    return int(off.value), int(cnt.value)


def accx_gemm_probe_layout(m: int, n: int, k: int, flags: int):
    """(byte offset of the probe records in the accx_gemm_dev workspace, record count)."""
    off = _sz(0)
    cnt = ctypes.c_int(0)
    _check(_lib.accx_gemm_probe_layout(int(m), int(n), int(k), int(flags), ctypes.byref(off), ctypes.byref(cnt)),
           "accx_gemm_probe_layout")
    return int(off.value), int(cnt.value)


def probe_records(raw: bytes, count: int):
    """Decode `count` accx_probe_record structs from raw workspace bytes."""
    size = ctypes.sizeof(accx_probe_record)
    return [accx_probe_record.from_buffer_copy(raw[i * size:(i + 1) * size]) for i in range(count)]


def batch_matmul(a, b, c, length: int, tile: int = 0) -> accx_batch_item:
    """A float32 matmul item on device arrays (torch tensors or addresses)."""
    return accx_batch_item(ACC_BATCH_MATMUL, ACC_FLOAT32, _addr(a), _addr(b), _addr(c), int(length), 0.0, int(tile))


def batch_reduce(x, n: int, result, init: float = 0.0) -> accx_batch_item:
    """A float32 reduction item: result = init + sum x[0:n]."""
    return accx_batch_item(ACC_BATCH_REDUCE, ACC_FLOAT32, _addr(x), None, _addr(result), int(n), float(init), 0)


def accx_batch_create(items, flags: int = 0) -> int:
    arr = (accx_batch_item * max(1, len(items)))(*items)
    out = _vp(0)
    _check(_lib.accx_batch_create(arr, len(items), int(flags), ctypes.byref(out)), "accx_batch_create")
    return int(out.value)


def accx_batch_launch(batch: int, stream=None) -> None:
    _check(_lib.accx_batch_launch(batch, _stream(stream)), "accx_batch_launch")


def accx_batch_launch_eager(batch: int, stream=None) -> None:
    _check(_lib.accx_batch_launch_eager(batch, _stream(stream)), "accx_batch_launch_eager")


def accx_batch_info(batch: int) -> dict:
    info = accx_batch_info_t()
    _check(_lib.accx_batch_info(batch, ctypes.byref(info)), "accx_batch_info")
    d = {f: getattr(info, f) for f, _ in accx_batch_info_t._fields_}
    d["graph_nodes"] = d.pop("pad")
    return d


def accx_batch_destroy(batch: int) -> None:
    _check(_lib.accx_batch_destroy(batch), "accx_batch_destroy")


def accx_server_create(slots: int = 8, hbm_budget_bytes: int = 0) -> int:
    out = _vp(0)
    _check(_lib.accx_server_create(int(slots), int(hbm_budget_bytes), ctypes.byref(out)), "accx_server_create")
    return int(out.value)


def accx_server_submit(server: int, req: accx_request) -> None:
    _check(_lib.accx_server_submit(server, ctypes.byref(req)), "accx_server_submit")


_POLL_CAP = 1024
_poll_buf = (accx_completion * _POLL_CAP)()


def accx_server_poll(server: int):
    """Progress the server; returns the finished requests as
    (tag, status, t_submit, t_start, t_done) tuples."""
    n = ctypes.c_int(0)
    out = []
    while True:
        _check(_lib.accx_server_poll(server, _poll_buf, _POLL_CAP, ctypes.byref(n)), "accx_server_poll")
        out.extend((int(c.tag), int(c.status), c.t_submit, c.t_start, c.t_done) for c in _poll_buf[:n.value])
        if n.value < _POLL_CAP:
            return out


def accx_server_drain(server: int) -> None:
    _check(_lib.accx_server_drain(server), "accx_server_drain")


def accx_server_now(server: int) -> float:
    t = ctypes.c_double(0)
    _check(_lib.accx_server_now(server, ctypes.byref(t)), "accx_server_now")
    return float(t.value)


def accx_server_stats(server: int) -> dict:
    st = accx_server_stats_t()
    _check(_lib.accx_server_stats(server, ctypes.byref(st)), "accx_server_stats")
    return {f: int(getattr(st, f)) for f, _ in accx_server_stats_t._fields_}


def accx_server_destroy(server: int) -> None:
    _check(_lib.accx_server_destroy(server), "accx_server_destroy")
