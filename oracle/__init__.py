"""CPU oracle (numpy front end over ``oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check in
``__graft_entry__`` and by the CPU-baseline leg of ``bench.py``.  The device
library and its Python binding never import it.

Each function states the passage of the paper (IPMACC, arXiv 1412.1127) it
follows; the arithmetic itself lives in ``oracle.c`` and is documented there.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_HDR = os.path.join(_HERE, "oracle.h")
_LIB = os.path.join(_HERE, "liboracle.so")
# A prebuilt oracle library to load instead (the sanitizer test's
# AddressSanitizer / UndefinedBehaviorSanitizer build of oracle.c).
_LIB_OVERRIDE = os.environ.get("ACCX_ORACLE_LIB")

_lib = None


def build(force: bool = False) -> str:
    """Compile ``liboracle.so`` with gcc (plain C, OpenMP, no fast-math)."""
    stale = (not os.path.exists(_LIB)) or any(
        os.path.getmtime(p) > os.path.getmtime(_LIB) for p in (_SRC, _HDR))
    if force or stale:
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        L = ctypes.CDLL(_LIB_OVERRIDE or build())
        i64, i32, f64, vp = ctypes.c_int64, ctypes.c_int32, ctypes.c_double, ctypes.c_void_p
        sig = {
            "oracle_set_threads": (None, [ctypes.c_int]),
            "oracle_max_threads": (ctypes.c_int, []),
            "oracle_matmul_f32_ijl": (None, [i64, vp, vp, vp]),
            "oracle_matmul_f32": (None, [i64, vp, vp, vp]),
            "oracle_matmul_i32_ijl": (None, [i64, vp, vp, vp]),
            "oracle_matmul_i32": (None, [i64, vp, vp, vp]),
            "oracle_matmul_f32_rows": (None, [i64, i64, i64, vp, vp, vp]),
            "oracle_matmul_i32_rows": (None, [i64, i64, i64, vp, vp, vp]),
            "oracle_gemm_f32": (None, [i64, i64, i64, vp, i64, vp, i64, vp, i64]),
            "oracle_gemm_i32": (None, [i64, i64, i64, vp, i64, vp, i64, vp, i64]),
            "oracle_matmul_f32_at": (None, [i64, vp, vp, i64, vp, vp, vp]),
            "oracle_matmul_i32_at": (None, [i64, vp, vp, i64, vp, vp, vp]),
            "oracle_sum_f32": (f64, [i64, vp, f64]),
            "oracle_sum_i32": (i32, [i64, vp, i32]),
            "oracle_reduce": (None, [ctypes.c_int, ctypes.c_int, ctypes.c_int, vp, i64, vp, vp]),
            "oracle_round_bf16": (ctypes.c_uint16, [ctypes.c_float]),
            "oracle_bf16_value": (f64, [ctypes.c_uint16]),
            "oracle_split_bf16x3": (None, [i64, vp, vp, vp, vp]),
            "oracle_maxabs_i32": (i64, [i64, vp]),
            "oracle_limbs_i8": (None, [i64, vp, ctypes.c_int, vp]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _p(arr: np.ndarray):
    return arr.ctypes.data_as(ctypes.c_void_p)


def _square(a: np.ndarray, b: np.ndarray, dtype) -> int:
    a = np.asarray(a)
    if a.ndim != 2 or a.shape[0] != a.shape[1] or b.shape != a.shape:
        raise ValueError("square LEN*LEN operands of equal shape expected")
    if a.dtype != dtype or b.dtype != dtype or not (a.flags.c_contiguous and b.flags.c_contiguous):
        raise ValueError("contiguous %s operands expected" % np.dtype(dtype).name)
    return int(a.shape[0])


def set_threads(n: int) -> None:
    lib().oracle_set_threads(int(n))


def max_threads() -> int:
    return int(lib().oracle_max_threads())


def matmul_f32(a: np.ndarray, b: np.ndarray, literal_order: bool = False) -> np.ndarray:
    """Listing 1a (section 1.3) with ``sum`` in float64: C[i,j] = sum_l A[i,l] B[l,j], l ascending."""
    n = _square(a, b, np.float32)
    c = np.empty((n, n), dtype=np.float64)
    fn = lib().oracle_matmul_f32_ijl if literal_order else lib().oracle_matmul_f32
    fn(n, _p(a), _p(b), _p(c))
    return c


def matmul_i32(a: np.ndarray, b: np.ndarray, literal_order: bool = False) -> np.ndarray:
    """Listing 1b's int operands (section 1.3) with wraparound: C = (sum_l A[i,l] B[l,j]) mod 2**32."""
    n = _square(a, b, np.int32)
    c = np.empty((n, n), dtype=np.int32)
    fn = lib().oracle_matmul_i32_ijl if literal_order else lib().oracle_matmul_i32
    fn(n, _p(a), _p(b), _p(c))
    return c


def _rowmajor_ld(x: np.ndarray) -> int:
    """Leading dimension (elements) of a 2-D row-major view; rows may be padded."""
    if x.ndim != 2 or x.strides[1] != x.itemsize or x.strides[0] % x.itemsize or x.strides[0] < x.shape[1] * x.itemsize:
        raise ValueError("2-D row-major array (unit column stride) expected")
    return x.strides[0] // x.itemsize


def gemm(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Listing 1a's loop nest on rectangular operands: C (m x n) = A (m x k) B (k x n),
    float64 accumulation for float32 inputs, wraparound mod 2**32 for int32.
    A and B may be row-major views with padded rows (leading dimensions)."""
    if a.ndim != 2 or b.ndim != 2 or a.shape[1] != b.shape[0] or a.dtype != b.dtype:
        raise ValueError("A (m x k) and B (k x n) of one dtype expected")
    m, k = a.shape
    n = b.shape[1]
    lda, ldb = _rowmajor_ld(a), _rowmajor_ld(b)
    if a.dtype == np.float32:
        c = np.empty((m, n), dtype=np.float64)
        lib().oracle_gemm_f32(m, n, k, _p(a), lda, _p(b), ldb, _p(c), n)
    elif a.dtype == np.int32:
        c = np.empty((m, n), dtype=np.int32)
        lib().oracle_gemm_i32(m, n, k, _p(a), lda, _p(b), ldb, _p(c), n)
    else:
        raise ValueError("float32 or int32 operands expected")
    return c


def matmul_rows(a: np.ndarray, b: np.ndarray, row0: int, nrows: int) -> np.ndarray:
    """Rows [row0, row0+nrows) of matmul_f32 / matmul_i32 (same arithmetic)."""
    if a.dtype == np.float32:
        n = _square(a, b, np.float32)
        out = np.empty((nrows, n), dtype=np.float64)
        fn = lib().oracle_matmul_f32_rows
    else:
        n = _square(a, b, np.int32)
        out = np.empty((nrows, n), dtype=np.int32)
        fn = lib().oracle_matmul_i32_rows
    if row0 < 0 or nrows < 0 or row0 + nrows > n:
        raise IndexError("row range out of bounds")
    fn(n, int(row0), int(nrows), _p(a), _p(b), _p(out))
    return out


def matmul_at(a: np.ndarray, b: np.ndarray, ii, jj) -> np.ndarray:
    """Selected entries C[ii[s], jj[s]] of the matmul above (float64 or wrapped int32)."""
    ii = np.ascontiguousarray(ii, dtype=np.int64)
    jj = np.ascontiguousarray(jj, dtype=np.int64)
    if ii.shape != jj.shape:
        raise ValueError("index arrays differ in shape")
    n0 = int(np.asarray(a).shape[0])
    if ii.size and (ii.min() < 0 or jj.min() < 0 or ii.max() >= n0 or jj.max() >= n0):
        raise IndexError("entry index out of range")
    if a.dtype == np.float32:
        n = _square(a, b, np.float32)
        out = np.empty(ii.shape, dtype=np.float64)
        lib().oracle_matmul_f32_at(n, _p(a), _p(b), ii.size, _p(ii), _p(jj), _p(out))
    else:
        n = _square(a, b, np.int32)
        out = np.empty(ii.shape, dtype=np.int32)
        lib().oracle_matmul_i32_at(n, _p(a), _p(b), ii.size, _p(ii), _p(jj), _p(out))
    return out


def sum_f32(x: np.ndarray, init: float = 0.0) -> float:
    """reduction(+) (section 2.3; SRAD paragraph of 4.2): init + x[0] + x[1] + ..., float64, index order."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    return float(lib().oracle_sum_f32(x.size, _p(x), float(init)))


def sum_i32(x: np.ndarray, init: int = 0) -> int:
    """reduction(+) over int32 with wraparound: (init + sum x) mod 2**32 as int32."""
    x = np.ascontiguousarray(x, dtype=np.int32)
    return int(lib().oracle_sum_i32(x.size, _p(x), int(np.int32(init))))


REDUCE_OPS = {"sum": 0, "max": 1, "min": 2, "or": 3}
_RED_DTYPES = {np.dtype(np.float32): (0, np.float64), np.dtype(np.int32): (1, np.int32),
               np.dtype(np.float64): (2, np.float64), np.dtype(np.int64): (3, np.int64)}


def identity(op: str, dtype) -> float | int:
    """The value that leaves a reduction unchanged: 0 for + and logical or,
    the lowest value for max, the highest for min."""
    dt = np.dtype(dtype)
    if op in ("sum", "or"):
        return 0
    if dt.kind == "f":
        return -np.inf if op == "max" else np.inf
    info = np.iinfo(dt)
    return int(info.min) if op == "max" else int(info.max)


def reduce(x: np.ndarray, op: str, init=None, square: bool = False):
    """One reduction variable (section 2.3's reduction lowering with the
    operators +, max, min and logical or): init (op) f(x[0]) (op) f(x[1]) ...
    in index order, f(x) = x or x*x in the element type.  float32: + in
    float64; float64: + in long double; int32/int64: + and * wrap around;
    max/min ignore NaN operands; 'or' gives 1 if init or any element is
    nonzero, else 0.  Returns a Python float (float types) or int."""
    x = np.ascontiguousarray(x)
    if x.dtype not in _RED_DTYPES:
        raise ValueError("float32, int32, float64 or int64 elements expected")
    if op not in REDUCE_OPS:
        raise ValueError("op must be one of %s" % sorted(REDUCE_OPS))
    if op == "or" and square:
        raise ValueError("logical or takes the elements themselves")
    code, out_t = _RED_DTYPES[x.dtype]
    iv = np.array([identity(op, x.dtype) if init is None else init], dtype=x.dtype)
    out = np.zeros(1, dtype=out_t)
    lib().oracle_reduce(code, REDUCE_OPS[op], int(bool(square)), _p(x), x.size, _p(iv), _p(out))
    return float(out[0]) if out_t == np.float64 else int(out[0])


def round_bf16(x: float) -> int:
    """Nearest bfloat16 bit pattern of a finite float, ties to even."""
    return int(lib().oracle_round_bf16(float(np.float32(x))))


def bf16_value(h: int) -> float:
    return float(lib().oracle_bf16_value(int(h)))


def split_bf16x3(x: np.ndarray):
    """hi = RN(x), mid = RN(x - hi), lo = RN(x - hi - mid); uint16 bf16 patterns, same shape as x."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    hi = np.empty(x.shape, dtype=np.uint16)
    mid = np.empty(x.shape, dtype=np.uint16)
    lo = np.empty(x.shape, dtype=np.uint16)
    lib().oracle_split_bf16x3(x.size, _p(x), _p(hi), _p(mid), _p(lo))
    return hi, mid, lo


def maxabs_i32(x: np.ndarray) -> int:
    x = np.ascontiguousarray(x, dtype=np.int32)
    return int(lib().oracle_maxabs_i32(x.size, _p(x)))


def limbs_i8(x: np.ndarray, nl: int) -> np.ndarray:
    """Balanced base-256 digits, shape (nl,) + x.shape, digit k first."""
    if not 1 <= nl <= 4:
        raise ValueError("1..4 limbs")
    x = np.ascontiguousarray(x, dtype=np.int32)
    d = np.empty((nl,) + x.shape, dtype=np.int8)
    lib().oracle_limbs_i8(x.size, _p(x), int(nl), _p(d))
    return d
