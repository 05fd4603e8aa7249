"""Pins of the CPU oracle against facts that do not come from the oracle itself.

The paper (IPMACC, arXiv 1412.1127) prints no numeric results, so every pin is
a closed form, an invariant, a textbook special case, exact (rational or
bignum) brute force on tiny inputs, an error bound, or a hand-worked fixture
under tests/golden/.  Each is chosen so that a plausible slip in the oracle (a
dropped term, a wrong index, a transposed operand, a wrong rounding or digit
rule) fails at least one of them.
"""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
SEED = synth.DEFAULT_SEED


def _rand_f32(n, stream):
    return synth.uniform_pm1_f32((n, n), SEED, stream)


# --------------------------------------------------------------- matmul f32 --

@pytest.mark.parametrize("n", [1, 2, 7, 33, 100])
def test_identity_gives_other_operand(n):
    a = _rand_f32(n, 11)
    eye = np.eye(n, dtype=np.float32)
    assert np.array_equal(oracle.matmul_f32(eye, a), a.astype(np.float64))
    assert np.array_equal(oracle.matmul_f32(a, eye), a.astype(np.float64))
    ai = synth.full_range_i32((n, n), SEED, 12)
    eyei = np.eye(n, dtype=np.int32)
    assert np.array_equal(oracle.matmul_i32(eyei, ai), ai)
    assert np.array_equal(oracle.matmul_i32(ai, eyei), ai)


@pytest.mark.parametrize("n", [1, 5, 64, 129])
def test_all_ones_gives_len(n):
    one = np.ones((n, n), dtype=np.float32)
    assert np.all(oracle.matmul_f32(one, one) == n)
    onei = np.ones((n, n), dtype=np.int32)
    assert np.all(oracle.matmul_i32(onei, onei) == n)


def test_hand_worked_3x3():
    rows = {}
    with open(os.path.join(GOLDEN, "matmul_3x3_int.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                k, *v = line.split()
                rows[k] = np.array([int(t) for t in v]).reshape(3, 3)
    a, b, c = (rows[k] for k in "abc")
    assert np.array_equal(oracle.matmul_i32(a.astype(np.int32), b.astype(np.int32)), c)
    assert np.array_equal(oracle.matmul_f32(a.astype(np.float32), b.astype(np.float32)), c)


def _exact_product(a, b):
    n = a.shape[0]
    fa = [[Fraction(float(v)) for v in row] for row in a]
    fb = [[Fraction(float(v)) for v in row] for row in b]
    return [[sum((fa[i][l] * fb[l][j] for l in range(n)), Fraction(0)) for j in range(n)]
            for i in range(n)]


@pytest.mark.parametrize("n", [1, 2, 3, 5, 8])
def test_brute_force_rational_grid_inputs(n):
    # uniform[-1,1] inputs are multiples of 2^-23: every product is a multiple
    # of 2^-46 below 1 and every partial sum needs < 53 bits, so the float64
    # accumulation is exact and must equal the rational result.
    a, b = _rand_f32(n, 21), _rand_f32(n, 22)
    exact = _exact_product(a, b)
    c = oracle.matmul_f32(a, b)
    for i in range(n):
        for j in range(n):
            assert Fraction(float(c[i, j])) == exact[i][j]


@pytest.mark.parametrize("n", [2, 5, 8])
def test_brute_force_error_bound_arbitrary_floats(n):
    # Arbitrary floats (full 24-bit significands, mixed exponents): recursive
    # float64 summation of exact products obeys |c - s| <= gamma_n * sum|a||b|
    # with gamma_n = n u / (1 - n u), u = 2^-53.
    g = synth.rng(SEED, 23)
    a = (g.standard_normal((n, n)) * np.exp2(g.uniform(-20, 20, (n, n)))).astype(np.float32)
    b = (g.standard_normal((n, n)) * np.exp2(g.uniform(-20, 20, (n, n)))).astype(np.float32)
    exact = _exact_product(a, b)
    c = oracle.matmul_f32(a, b)
    u = 2.0 ** -53
    gamma = n * u / (1 - n * u)
    absprod = np.abs(a.astype(np.float64)) @ np.abs(b.astype(np.float64))
    for i in range(n):
        for j in range(n):
            err = abs(Fraction(float(c[i, j])) - exact[i][j])
            assert err <= Fraction(gamma * absprod[i, j] * (1 + 1e-12))


@pytest.mark.parametrize("n", [1, 3, 17, 96])
def test_loop_order_bitwise(n):
    a, b = _rand_f32(n, 31), _rand_f32(n, 32)
    assert np.array_equal(oracle.matmul_f32(a, b), oracle.matmul_f32(a, b, literal_order=True))
    ai, bi = synth.full_range_i32((n, n), SEED, 33), synth.full_range_i32((n, n), SEED, 34)
    assert np.array_equal(oracle.matmul_i32(ai, bi), oracle.matmul_i32(ai, bi, literal_order=True))


def test_transpose_identity_bitwise():
    # (AB)^T == B^T A^T: same terms in the same l order.
    n = 45
    g = synth.rng(SEED, 41)
    a = g.standard_normal((n, n)).astype(np.float32)
    b = g.standard_normal((n, n)).astype(np.float32)
    lhs = oracle.matmul_f32(a, b).T
    rhs = oracle.matmul_f32(np.ascontiguousarray(b.T), np.ascontiguousarray(a.T))
    assert np.array_equal(lhs, rhs)


def test_permutation_rows_and_columns():
    n = 37
    g = synth.rng(SEED, 42)
    perm = g.permutation(n)
    p = np.zeros((n, n), dtype=np.float32)
    p[np.arange(n), perm] = 1.0
    b = _rand_f32(n, 43)
    assert np.array_equal(oracle.matmul_f32(p, b), b[perm].astype(np.float64))
    # right multiplication by P^T permutes columns the same way
    pt = np.ascontiguousarray(p.T)
    assert np.array_equal(oracle.matmul_f32(b, pt), b[:, perm].astype(np.float64))


def test_thread_count_invariance():
    n = 77
    a, b = _rand_f32(n, 51), _rand_f32(n, 52)
    ai, bi = synth.full_range_i32((n, n), SEED, 53), synth.full_range_i32((n, n), SEED, 54)
    nt = oracle.max_threads()
    try:
        oracle.set_threads(1)
        c1, i1 = oracle.matmul_f32(a, b), oracle.matmul_i32(ai, bi)
        oracle.set_threads(max(2, nt))
        c8, i8 = oracle.matmul_f32(a, b), oracle.matmul_i32(ai, bi)
    finally:
        oracle.set_threads(nt)
    assert np.array_equal(c1, c8) and np.array_equal(i1, i8)


def test_integer_valued_floats_match_int_path():
    # Integers in [-16, 16] stored as floats: |partial sums| <= LEN * 256 < 2^53,
    # so the float64 oracle is exact and equals the int oracle.
    n = 64
    ai = synth.int_uniform_i32((n, n), -16, 16, SEED, 61)
    bi = synth.int_uniform_i32((n, n), -16, 16, SEED, 62)
    cf = oracle.matmul_f32(ai.astype(np.float32), bi.astype(np.float32))
    assert np.array_equal(cf, oracle.matmul_i32(ai, bi).astype(np.float64))


def test_sampled_entries_match_full():
    n = 53
    a, b = _rand_f32(n, 71), _rand_f32(n, 72)
    ai, bi = synth.full_range_i32((n, n), SEED, 73), synth.full_range_i32((n, n), SEED, 74)
    g = synth.rng(SEED, 75)
    ii, jj = g.integers(0, n, 40), g.integers(0, n, 40)
    assert np.array_equal(oracle.matmul_at(a, b, ii, jj), oracle.matmul_f32(a, b)[ii, jj])
    assert np.array_equal(oracle.matmul_at(ai, bi, ii, jj), oracle.matmul_i32(ai, bi)[ii, jj])
    with pytest.raises(IndexError):
        oracle.matmul_at(a, b, [n], [0])


def test_row_slices_match_full():
    n = 61
    a, b = _rand_f32(n, 76), _rand_f32(n, 77)
    ai, bi = synth.full_range_i32((n, n), SEED, 78), synth.full_range_i32((n, n), SEED, 79)
    assert np.array_equal(oracle.matmul_rows(a, b, 10, 17), oracle.matmul_f32(a, b)[10:27])
    assert np.array_equal(oracle.matmul_rows(ai, bi, 44, 17), oracle.matmul_i32(ai, bi)[44:61])
    with pytest.raises(IndexError):
        oracle.matmul_rows(a, b, 50, 20)


# ------------------------------------------------------- rectangular gemm --

@pytest.mark.parametrize("m,n,k", [(1, 1, 1), (3, 5, 2), (7, 2, 9), (4, 8, 1)])
def test_gemm_rational_brute_force(m, n, k):
    # grid-valued inputs: the float64 accumulation is exact at these sizes
    a = synth.uniform_pm1_f32((m, k), SEED, 131)
    b = synth.uniform_pm1_f32((k, n), SEED, 132)
    c = oracle.gemm(a, b)
    for i in range(m):
        for j in range(n):
            ex = sum((Fraction(float(a[i, l])) * Fraction(float(b[l, j])) for l in range(k)), Fraction(0))
            assert Fraction(float(c[i, j])) == ex


def test_gemm_square_equals_matmul():
    n = 33
    a, b = _rand_f32(n, 133), _rand_f32(n, 134)
    assert np.array_equal(oracle.gemm(a, b), oracle.matmul_f32(a, b))
    ai, bi = synth.full_range_i32((n, n), SEED, 135), synth.full_range_i32((n, n), SEED, 136)
    assert np.array_equal(oracle.gemm(ai, bi), oracle.matmul_i32(ai, bi))


def test_gemm_leading_dimensions():
    # views with padded rows give the result of their contiguous copies
    big_a = synth.uniform_pm1_f32((20, 37), SEED, 137)
    big_b = synth.uniform_pm1_f32((30, 41), SEED, 138)
    a, b = big_a[3:15, 5:29], big_b[2:26, 7:40]          # 12 x 24 and 24 x 33
    assert np.array_equal(oracle.gemm(a, b), oracle.gemm(np.ascontiguousarray(a), np.ascontiguousarray(b)))
    bia = synth.full_range_i32((20, 37), SEED, 139)
    bib = synth.full_range_i32((30, 41), SEED, 140)
    ai, bi = bia[3:15, 5:29], bib[2:26, 7:40]
    assert np.array_equal(oracle.gemm(ai, bi), oracle.gemm(np.ascontiguousarray(ai), np.ascontiguousarray(bi)))


def test_gemm_outer_product_and_transpose():
    # k = 1: C is the outer product, every entry one exact product
    a = synth.uniform_pm1_f32((9, 1), SEED, 141)
    b = synth.uniform_pm1_f32((1, 13), SEED, 142)
    assert np.array_equal(oracle.gemm(a, b), a.astype(np.float64) @ b.astype(np.float64))
    # (AB)^T == B^T A^T bitwise on rectangular shapes
    g = synth.rng(SEED, 143)
    a = g.standard_normal((6, 11)).astype(np.float32)
    b = g.standard_normal((11, 4)).astype(np.float32)
    lhs = oracle.gemm(a, b).T
    rhs = oracle.gemm(np.ascontiguousarray(b.T), np.ascontiguousarray(a.T))
    assert np.array_equal(lhs, rhs)


def test_gemm_int_associativity_rectangular():
    a = synth.full_range_i32((3, 5), SEED, 144)
    b = synth.full_range_i32((5, 2), SEED, 145)
    c = synth.full_range_i32((2, 4), SEED, 146)
    assert np.array_equal(oracle.gemm(oracle.gemm(a, b), c), oracle.gemm(a, oracle.gemm(b, c)))


# --------------------------------------------------------------- matmul i32 --

@pytest.mark.parametrize("n", [1, 2, 4, 8])
def test_int_brute_force_bignum_wraps(n):
    a = synth.full_range_i32((n, n), SEED, 81)
    b = synth.full_range_i32((n, n), SEED, 82)
    c = oracle.matmul_i32(a, b)
    for i in range(n):
        for j in range(n):
            s = sum(int(a[i, l]) * int(b[l, j]) for l in range(n)) % (1 << 32)
            s = s - (1 << 32) if s >= (1 << 31) else s
            assert int(c[i, j]) == s


def test_int_wrap_near_limits():
    n = 4
    a = np.full((n, n), 2 ** 31 - 1, dtype=np.int32)
    b = np.full((n, n), -(2 ** 31), dtype=np.int32)
    c = oracle.matmul_i32(a, b)
    s = (n * (2 ** 31 - 1) * -(2 ** 31)) % (1 << 32)
    s = s - (1 << 32) if s >= (1 << 31) else s
    assert np.all(c == s)


@pytest.mark.parametrize("n", [1, 3, 6])
def test_int_associativity(n):
    # (AB)C == A(BC) in the ring of integers mod 2^32; fails for a transposed operand.
    a, b, c = (synth.full_range_i32((n, n), SEED, 90 + k) for k in range(3))
    assert np.array_equal(oracle.matmul_i32(oracle.matmul_i32(a, b), c),
                          oracle.matmul_i32(a, oracle.matmul_i32(b, c)))


def test_int_linearity():
    n = 9
    a, b1, b2 = (synth.full_range_i32((n, n), SEED, 95 + k) for k in range(3))
    bsum = (b1.astype(np.int64) + b2.astype(np.int64)).astype(np.uint64).astype(np.uint32).view(np.int32)
    lhs = oracle.matmul_i32(a, np.ascontiguousarray(bsum))
    rhs = (oracle.matmul_i32(a, b1).astype(np.int64) + oracle.matmul_i32(a, b2).astype(np.int64))
    rhs = rhs.astype(np.uint64).astype(np.uint32).view(np.int32)
    assert np.array_equal(lhs, rhs)


# ---------------------------------------------------------------- reduction --

@pytest.mark.parametrize("n", [0, 1, 2, 1000, 5792, 100000])
def test_sum_closed_form(n):
    k = np.arange(1, n + 1)
    closed = n * (n + 1) // 2
    assert oracle.sum_i32(k.astype(np.int32)) == np.int64(closed).astype(np.uint64).astype(np.uint32).view(np.int32)
    if n < (1 << 24):
        assert oracle.sum_f32(k.astype(np.float32)) == float(closed)


def test_sum_init_and_empty():
    assert oracle.sum_f32(np.zeros(0, np.float32), 2.5) == 2.5
    assert oracle.sum_i32(np.zeros(0, np.int32), -7) == -7
    assert oracle.sum_f32(np.array([1.0, 2.0], np.float32), 0.5) == 3.5
    assert oracle.sum_i32(np.array([2 ** 31 - 1], np.int32), 1) == -(2 ** 31)


def test_sum_uniform01_is_exact():
    # values k * 2^-24: the float64 serial sum is the exact sum; math.fsum
    # returns the correctly rounded exact sum by a different algorithm.
    x = synth.uniform01_f32(1 << 20, SEED, 101)
    assert oracle.sum_f32(x) == math.fsum(x.astype(np.float64).tolist())


def test_sum_int_wraps():
    x = np.full(1000, 2 ** 31 - 1, dtype=np.int32)
    s = (1000 * (2 ** 31 - 1)) % (1 << 32)
    s = s - (1 << 32) if s >= (1 << 31) else s
    assert oracle.sum_i32(x) == s


# ---------------------------------------------------------------- bf16 split --

def _load_split_golden():
    out = []
    with open(os.path.join(GOLDEN, "bf16x3_split.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                out.append([int(t, 16) for t in line.split()])
    return out


def test_split_golden():
    for xb, h, m, l in _load_split_golden():
        x = np.array([xb], dtype=np.uint32).view(np.float32)
        hi, mid, lo = oracle.split_bf16x3(x)
        assert (int(hi[0]), int(mid[0]), int(lo[0])) == (h, m, l), hex(xb)


def _nearest_bf16_by_value(x: float) -> float:
    # Independent route: arithmetic on the value, not on bit patterns.
    if x == 0.0:
        return 0.0
    ax = abs(x)
    e = math.floor(math.log2(ax))
    if 2.0 ** e > ax:
        e -= 1
    if 2.0 ** (e + 1) <= ax:
        e += 1
    ulp = 2.0 ** (e - 7)
    k = math.floor(ax / ulp)
    lo, hi = k * ulp, (k + 1) * ulp
    if ax - lo < hi - ax:
        r = lo
    elif hi - ax < ax - lo:
        r = hi
    else:
        r = lo if k % 2 == 0 else hi
    return math.copysign(r, x)


def test_split_nearest_and_exact_sum():
    g = synth.rng(SEED, 111)
    x = np.concatenate([
        synth.uniform_pm1_f32((4000,), SEED, 112),
        synth.normal_rowscaled_f32(40, 100, SEED, 113).ravel(),
        (g.standard_normal(4000) * np.exp2(g.uniform(-60, 60, 4000))).astype(np.float32),
    ])
    hi, mid, lo = oracle.split_bf16x3(x)
    val = lambda p: (p.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    vh, vm, vl = val(hi), val(mid), val(lo)
    xd = x.astype(np.float64)
    # the three terms add up to x exactly
    assert np.array_equal(vh + vm + vl, xd)
    assert np.array_equal((vh + vm) + vl, xd)
    # hi and mid are the nearest bf16 values of x and of x - hi
    for t in range(0, x.size, 7):
        assert vh[t] == _nearest_bf16_by_value(float(xd[t]))
        assert vm[t] == _nearest_bf16_by_value(float(xd[t] - vh[t]))
    # term sizes shrink by the bf16 precision (8 significant bits)
    nz = xd != 0
    assert np.all(np.abs(vm[nz]) <= np.abs(xd[nz]) * 2.0 ** -8)
    assert np.all(np.abs(vl[nz]) <= np.abs(xd[nz]) * 2.0 ** -16)


def test_round_bf16_ties_to_even():
    # 1 + 2^-8 sits halfway between 1.0 (even) and 1 + 2^-7 (odd).
    assert oracle.round_bf16(1.0 + 2 ** -8) == 0x3F80
    assert oracle.round_bf16(1.0 + 3 * 2 ** -8) == 0x3F82
    assert oracle.round_bf16(-(1.0 + 2 ** -8)) == 0xBF80
    assert oracle.bf16_value(0x3F80) == 1.0


# --------------------------------------------------------------- int8 limbs --

def test_limbs_golden():
    with open(os.path.join(GOLDEN, "int8_limbs.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                v = [int(t) for t in line.split()]
                d = oracle.limbs_i8(np.array([v[0]], np.int32), 4)
                assert [int(t) for t in d[:, 0]] == v[1:], v[0]


@pytest.mark.parametrize("nl,bound", [(1, 127), (2, 32639), (3, 8355711), (4, None)])
def test_limbs_reconstruct(nl, bound):
    if bound is None:
        x = synth.full_range_i32((5000,), SEED, 121)
        x[:4] = [2 ** 31 - 1, -(2 ** 31), 0, -1]
    else:
        x = synth.int_uniform_i32((5000,), -bound, bound, SEED, 122)
        x[:2] = [bound, -bound]
    d = oracle.limbs_i8(x, nl).astype(np.int64)
    assert d.min() >= -128 and d.max() <= 127
    rec = sum(d[k] * (256 ** k) for k in range(nl))
    if bound is None:
        assert np.array_equal(rec.astype(np.uint64).astype(np.uint32).view(np.int32), x)
    else:
        assert np.array_equal(rec, x.astype(np.int64))


def test_maxabs():
    assert oracle.maxabs_i32(np.array([-(2 ** 31), 5], np.int32)) == 2 ** 31
    assert oracle.maxabs_i32(np.array([3, -4, 2], np.int32)) == 4
    assert oracle.maxabs_i32(np.zeros(0, np.int32)) == 0


# ------------------------------------------- reduction operators and types --

def test_reduce_int_closed_forms():
    n = 100_000
    k = np.arange(1, n + 1, dtype=np.int64)
    assert oracle.reduce(k, "sum") == n * (n + 1) // 2
    assert oracle.reduce(k, "sum", square=True) == n * (n + 1) * (2 * n + 1) // 6
    assert oracle.reduce(k, "sum", init=-5) == n * (n + 1) // 2 - 5
    assert oracle.reduce(k, "max") == n and oracle.reduce(k, "min") == 1
    assert oracle.reduce(k, "max", init=n + 7) == n + 7 and oracle.reduce(k, "min", init=-3) == -3
    k32 = k[:1000].astype(np.int32)
    assert oracle.reduce(k32, "sum", square=True) == 1000 * 1001 * 2001 // 6


def test_reduce_int_wraparound():
    # 5 * 2^30 = 2^32 + 2^30; 65536^2 = 2^32; int64: 2^62 * 4 = 2^64
    assert oracle.reduce(np.full(5, 1 << 30, np.int32), "sum") == 1 << 30
    assert oracle.reduce(np.array([65536, 3], np.int32), "sum", square=True) == 9
    assert oracle.reduce(np.full(4, 1 << 62, np.int64), "sum", init=7) == 7
    assert oracle.reduce(np.array([1 << 32], np.int64), "sum", square=True) == 0
    # bignum brute force on full-range values
    for dt, bits, stream in ((np.int32, 32, 201), (np.int64, 64, 202)):
        x = (synth.full_range_i32(500, SEED, stream) if dt == np.int32 else synth.full_range_i64(500, SEED, stream))
        for sq in (False, True):
            exact = sum(int(v) * int(v) if sq else int(v) for v in x) % (1 << bits)
            if exact >= 1 << (bits - 1):
                exact -= 1 << bits
            assert oracle.reduce(x, "sum", square=sq) == exact


def test_reduce_extremes_and_signed_order():
    x = np.array([-(1 << 63), (1 << 63) - 1, 0, -1], np.int64)
    assert oracle.reduce(x, "max") == (1 << 63) - 1 and oracle.reduce(x, "min") == -(1 << 63)
    y = synth.full_range_i32(4001, SEED, 203)
    assert oracle.reduce(y, "max") == int(max(y.tolist())) and oracle.reduce(y, "min") == int(min(y.tolist()))
    z = synth.full_range_i64(4001, SEED, 204)
    assert oracle.reduce(z, "max") == max(z.tolist()) and oracle.reduce(z, "min") == min(z.tolist())


def test_reduce_f64_sum_against_exact_sum():
    # grid values: the long-double sum of 4096 multiples of 2^-52 in [-1, 1) is exact
    x = synth.uniform_pm1_f64(4096, SEED, 205)
    assert oracle.reduce(x, "sum") == math.fsum(x.tolist())
    # arbitrary doubles: within a few units of the last place of the exact sum
    g = synth.rng(SEED, 206)
    y = g.random(100_000)
    ex = math.fsum(y.tolist())
    assert abs(oracle.reduce(y, "sum") - ex) <= 4 * 2.0 ** -52 * ex
    # squares are rounded to double first (the loop body's own arithmetic)
    ex2 = math.fsum((np.float64(v) * np.float64(v)) for v in y[:20_000])
    assert abs(oracle.reduce(y[:20_000], "sum", square=True) - ex2) <= 4 * 2.0 ** -52 * ex2


def test_reduce_f32_sum_and_squares():
    x = synth.uniform_pm1_f32((3000,), SEED, 207)
    assert oracle.reduce(x, "sum") == math.fsum(float(v) for v in x)          # grid values: exact
    sq = [float(np.float32(v) * np.float32(v)) for v in x]                       # rounded to float32
    assert oracle.reduce(x, "sum", square=True) == pytest.approx(math.fsum(sq), rel=1e-14)
    assert oracle.reduce(x, "sum", init=2.5) == 2.5 + math.fsum(float(v) for v in x)
    assert oracle.reduce(x, "max", square=True) == max(sq) and oracle.reduce(x, "min", square=True) == min(sq)
    # agrees with the pinned float32 sum
    u = synth.uniform01_f32(5000, SEED, 208)
    assert oracle.reduce(u, "sum", init=1.0) == oracle.sum_f32(u, 1.0)


def test_reduce_max_min_ignore_nan():
    x = synth.uniform_pm1_f32((1000,), SEED, 209).astype(np.float64)
    x[[0, 17, 999]] = np.nan
    assert oracle.reduce(x, "max") == np.nanmax(x) and oracle.reduce(x, "min") == np.nanmin(x)
    assert oracle.reduce(x.astype(np.float32), "max") == float(np.nanmax(x))
    allnan = np.full(5, np.nan)
    assert oracle.reduce(allnan, "max") == -np.inf           # the identity init survives
    assert math.isnan(oracle.reduce(allnan, "max", init=np.nan))
    assert oracle.reduce(allnan, "max", init=3.0) == 3.0
    assert oracle.reduce(np.array([np.nan, 2.0]), "min", init=np.nan) == 2.0


def test_reduce_logical_or():
    z = np.zeros(1000, np.int32)
    assert oracle.reduce(z, "or") == 0 and oracle.reduce(z, "or", init=5) == 1
    z[-1] = 1
    assert oracle.reduce(z, "or") == 1
    assert oracle.reduce(np.array([0, 1 << 40], np.int64), "or") == 1    # high bits only
    assert oracle.reduce(np.array([-0.0, 0.0], np.float32), "or") == 0   # -0 equals zero
    assert oracle.reduce(np.array([0.0, np.nan]), "or") == 1             # NaN is unequal to zero
    f = synth.sparse_flags_i32(100_000, 1e-4, SEED, 210)
    assert oracle.reduce(f, "or") == int(f.any())
    assert oracle.reduce(np.zeros(0, np.float64), "or", init=0.0) == 0
    with pytest.raises(ValueError):
        oracle.reduce(f, "or", square=True)


def test_reduce_empty_returns_init():
    for dt in (np.float32, np.int32, np.float64, np.int64):
        e = np.zeros(0, dt)
        for op in ("sum", "max", "min"):
            assert oracle.reduce(e, op, init=3) == 3
