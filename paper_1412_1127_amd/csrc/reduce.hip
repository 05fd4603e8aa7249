// reduction(+) lowering (section 2.3, "Replacing the dummy OpenACC kernels
// region calls"; SRAD paragraph of section 4.2): reduce across the threads of
// each workgroup on the GPU, then across workgroups.
//
// Two kernels:
//  - plain: the paper's shape.  One element per thread, a shared-memory tree
//    per workgroup, one partial per workgroup; the cross-workgroup stage is a
//    second, one-workgroup launch that adds the partials in index order.  (The
//    paper's translator copies the partials to the host for that stage; here
//    it stays on the device so that every arithmetic step runs in a kernel
//    and the call needs no host synchronisation.)
//  - fast: a pass that streams the input at HBM rate.  Each thread keeps
//    eight independent 16-byte accumulators over a grid-stride slice, a
//    wavefront reduces with cross-lane exchanges, the wavefronts of a
//    workgroup combine through LDS, and each workgroup stores one partial.
//    A second, one-workgroup launch adds the partials in index order and
//    then the initial value.  (Electing the last workgroup with an atomic
//    ticket instead saves that launch but needs a device-scope release in
//    every workgroup, an L2 write-back on gfx950: measured 18 us slower over
//    1 GiB than the two launches.)
// Both are bitwise deterministic: nothing depends on the order in which
// workgroups finish.
//
// float: float32 arithmetic throughout.  int32: unsigned 32-bit adds
// (wraparound modulo 2^32).  The other operators and element types (max,
// min, logical or; float64, int64; several variables per pass) follow the
// sum kernels below.
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace accx {
namespace {

constexpr int RT = 256;          // threads per workgroup
constexpr int RU = 8;            // 16-byte loads in flight per thread
constexpr int MAX_BLOCKS = 4096; // fast kernel: upper bound on workgroups

typedef float f4 __attribute__((ext_vector_type(4)));
typedef uint32_t u4 __attribute__((ext_vector_type(4)));

template <typename L> struct Vec;
template <> struct Vec<float> { using T = f4; };
template <> struct Vec<uint32_t> { using T = u4; };

template <typename L> __device__ inline L hsum(typename Vec<L>::T v) { return (v.x + v.y) + (v.z + v.w); }

template <typename L> __device__ inline L wave_sum(L v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = v + __shfl_xor(v, o, 64);
    return v;
}

// Sum over the 256 threads of a workgroup, fixed order; valid in thread 0.
template <typename L> __device__ inline L block_sum(L v, L *lds4)
{
    v = wave_sum(v);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) lds4[w] = v;
    __syncthreads();
    L r = 0;
    if (threadIdx.x == 0) r = (lds4[0] + lds4[1]) + (lds4[2] + lds4[3]);
    return r;
}

__device__ inline uint32_t to_bits(float v) { return __float_as_uint(v); }
__device__ inline uint32_t to_bits(uint32_t v) { return v; }
template <typename L> __device__ inline L from_bits(uint32_t b);
template <> __device__ inline float from_bits<float>(uint32_t b) { return __uint_as_float(b); }
template <> __device__ inline uint32_t from_bits<uint32_t>(uint32_t b) { return b; }

template <typename L>
__global__ __launch_bounds__(RT) void reduce_fast(const L *__restrict__ x, int64_t n, uint32_t *__restrict__ partials)
{
    using V = typename Vec<L>::T;
    __shared__ L lds4[4];

    // Aligned body of 16-byte vectors, with up to 3 leading and 3 trailing
    // scalars (x may start at any 4-byte boundary).
    const uintptr_t addr = (uintptr_t)x;
    int64_t head = (int64_t)(((16u - (unsigned)(addr & 15u)) & 15u) >> 2);
    if (head > n) head = n;
    const int64_t nvec = (n - head) >> 2;
    const int64_t tail0 = head + (nvec << 2);
    const V *__restrict__ xv = reinterpret_cast<const V *>(x + head);

    const int64_t stride = (int64_t)gridDim.x * RT;
    int64_t v = (int64_t)blockIdx.x * RT + threadIdx.x;
    V acc[RU];
#pragma unroll
    for (int u = 0; u < RU; ++u) acc[u] = (V)0;
    for (; v + (RU - 1) * stride < nvec; v += RU * stride) {
        V t[RU];
#pragma unroll
        for (int u = 0; u < RU; ++u) t[u] = __builtin_nontemporal_load(xv + v + u * stride);
#pragma unroll
        for (int u = 0; u < RU; ++u) acc[u] += t[u];
    }
    for (; v < nvec; v += stride) acc[0] += __builtin_nontemporal_load(xv + v);
    // fixed pairwise combination of the accumulators
#pragma unroll
    for (int w = RU / 2; w > 0; w >>= 1)
#pragma unroll
        for (int u = 0; u < w; ++u) acc[u] += acc[u + w];
    L s = hsum<L>(acc[0]);
    if (blockIdx.x == 0) {
        if (threadIdx.x < head) s = s + x[threadIdx.x];
        if ((int64_t)threadIdx.x < n - tail0) s = s + x[tail0 + threadIdx.x];
    }
    s = block_sum(s, lds4);
    if (threadIdx.x == 0) partials[blockIdx.x] = to_bits(s);
}

// One workgroup: result = init + (the g partials, added in index order over a
// fixed tree).
template <typename L>
__global__ __launch_bounds__(RT) void reduce_fast_final(const uint32_t *__restrict__ partials, unsigned g, L init,
                                                        L *__restrict__ result)
{
    __shared__ L lds4[4];
    L t = 0;
    for (unsigned k = threadIdx.x; k < g; k += RT) t = t + from_bits<L>(partials[k]);
    t = block_sum(t, lds4);
    if (threadIdx.x == 0) result[0] = init + t;
}

template <typename L>
__global__ __launch_bounds__(RT) void reduce_plain_blocks(const L *__restrict__ x, int64_t n, L *__restrict__ partials)
{
    __shared__ L s[RT];
    const int64_t i = (int64_t)blockIdx.x * RT + threadIdx.x;
    s[threadIdx.x] = i < n ? x[i] : (L)0;
    __syncthreads();
    for (int st = RT / 2; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) s[threadIdx.x] = s[threadIdx.x] + s[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) partials[blockIdx.x] = s[0];
}

template <typename L>
__global__ __launch_bounds__(RT) void reduce_plain_final(const L *__restrict__ partials, int64_t g, L init,
                                                         L *__restrict__ result)
{
    __shared__ L s[RT];
    L v = 0;
    for (int64_t k = threadIdx.x; k < g; k += RT) v = v + partials[k];
    s[threadIdx.x] = v;
    __syncthreads();
    for (int st = RT / 2; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) s[threadIdx.x] = s[threadIdx.x] + s[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) result[0] = init + s[0];
}

// ---- reduction variables of any operator and type --------------------------
//
// Up to four reduction variables over one array in one pass (the SRAD loop
// keeps a sum and a sum of squares of the same image): variable v combines
// f_v(x[k]) with operator op_v, where f_v(x) = x or x*x in the element type.
// Operators: + (integers wrap around), max, min (floats: a NaN operand is
// ignored, as fmax/fmin do).  Each thread folds its grid-stride slice into
// one accumulator per variable in a fixed order, the workgroup combines its
// threads in a fixed tree and stores one partial per variable, and a second,
// one-workgroup launch folds the partials in index order and then the
// initial value: result_v = init_v (op_v) (partial_0 (op_v) partial_1 ...).

template <typename E> struct Red;
template <> struct Red<float> {
    using V = f4;
    using Bits = uint32_t;
    static constexpr int W = 4;
    __device__ static float lowest() { return -__builtin_inff(); }
    __device__ static float highest() { return __builtin_inff(); }
    __device__ static float add(float a, float b) { return a + b; }
    __device__ static float mul(float a, float b) { return a * b; }
    __device__ static float max(float a, float b) { return __builtin_fmaxf(a, b); }
    __device__ static float min(float a, float b) { return __builtin_fminf(a, b); }
    __device__ static bool nonzero(float a) { return a != 0.0f; }
};
typedef double d2 __attribute__((ext_vector_type(2)));
template <> struct Red<double> {
    using V = d2;
    using Bits = uint64_t;
    static constexpr int W = 2;
    __device__ static double lowest() { return -__builtin_inf(); }
    __device__ static double highest() { return __builtin_inf(); }
    __device__ static double add(double a, double b) { return a + b; }
    __device__ static double mul(double a, double b) { return a * b; }
    __device__ static double max(double a, double b) { return __builtin_fmax(a, b); }
    __device__ static double min(double a, double b) { return __builtin_fmin(a, b); }
    __device__ static bool nonzero(double a) { return a != 0.0; }
};
typedef int32_t i4 __attribute__((ext_vector_type(4)));
template <> struct Red<int32_t> {
    using V = i4;
    using Bits = uint32_t;
    static constexpr int W = 4;
    __device__ static int32_t lowest() { return INT32_MIN; }
    __device__ static int32_t highest() { return INT32_MAX; }
    __device__ static int32_t add(int32_t a, int32_t b) { return (int32_t)((uint32_t)a + (uint32_t)b); }
    __device__ static int32_t mul(int32_t a, int32_t b) { return (int32_t)((uint32_t)a * (uint32_t)b); }
    __device__ static int32_t max(int32_t a, int32_t b) { return a > b ? a : b; }
    __device__ static int32_t min(int32_t a, int32_t b) { return a < b ? a : b; }
    __device__ static bool nonzero(int32_t a) { return a != 0; }
};
typedef int64_t l2 __attribute__((ext_vector_type(2)));
template <> struct Red<int64_t> {
    using V = l2;
    using Bits = uint64_t;
    static constexpr int W = 2;
    __device__ static int64_t lowest() { return INT64_MIN; }
    __device__ static int64_t highest() { return INT64_MAX; }
    __device__ static int64_t add(int64_t a, int64_t b) { return (int64_t)((uint64_t)a + (uint64_t)b); }
    __device__ static int64_t mul(int64_t a, int64_t b) { return (int64_t)((uint64_t)a * (uint64_t)b); }
    __device__ static int64_t max(int64_t a, int64_t b) { return a > b ? a : b; }
    __device__ static int64_t min(int64_t a, int64_t b) { return a < b ? a : b; }
    __device__ static bool nonzero(int64_t a) { return a != 0; }
};

template <typename E> __device__ inline E red_identity(int op)
{
    return op == RED_SUM ? (E)0 : op == RED_MAX ? Red<E>::lowest() : Red<E>::highest();
}

template <typename E> __device__ inline E red_apply(int op, E a, E b)
{
    return op == RED_SUM ? Red<E>::add(a, b) : op == RED_MAX ? Red<E>::max(a, b) : Red<E>::min(a, b);
}

template <typename E> __device__ inline E bits_as(uint64_t b)
{
    typename Red<E>::Bits t = (typename Red<E>::Bits)b;
    return __builtin_bit_cast(E, t);
}
template <typename E> __device__ inline uint64_t as_bits(E v)
{
    return (uint64_t)__builtin_bit_cast(typename Red<E>::Bits, v);
}

// Combine v over the workgroup in a fixed order; valid in thread 0.
template <typename E> __device__ inline E block_apply(int op, E v, E *lds4)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = red_apply<E>(op, v, __shfl_xor(v, o, 64));
    if ((threadIdx.x & 63) == 0) lds4[threadIdx.x >> 6] = v;
    __syncthreads();
    E r = v;
    if (threadIdx.x == 0) r = red_apply<E>(op, red_apply<E>(op, lds4[0], lds4[1]), red_apply<E>(op, lds4[2], lds4[3]));
    __syncthreads();
    return r;
}

// Operators fixed at compile time: SIG holds (op | square << 2) of variable v
// in bits 4v..4v+3; SIG_RUNTIME reads them from `vars` (any combination, but
// the per-element operator selection then costs more VALU work than the
// element's load: about 4.5 instead of 6.9 TB/s over 1 GiB).
constexpr uint32_t SIG_RUNTIME = 0xffffffffu;

template <typename E, int NV, uint32_t SIG>
__global__ __launch_bounds__(RT) void reduce_vars(const E *__restrict__ x, int64_t n, RedVars vars,
                                                  uint64_t *__restrict__ partials)
{
    using R = Red<E>;
    using V = typename R::V;
    constexpr int W = R::W;
    __shared__ E lds4[4];

    int op[NV], sq[NV];
    E acc[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        op[v] = SIG == SIG_RUNTIME ? vars.op[v] : (int)((SIG >> (4 * v)) & 3u);
        sq[v] = SIG == SIG_RUNTIME ? vars.square[v] : (int)((SIG >> (4 * v + 2)) & 1u);
        acc[v] = red_identity<E>(op[v]);
    }
    auto fold = [&](E t) {
#pragma unroll
        for (int v = 0; v < NV; ++v) acc[v] = red_apply<E>(op[v], acc[v], sq[v] ? R::mul(t, t) : t);
    };

    // Aligned body of 16-byte vectors, up to W-1 leading and trailing scalars.
    const uintptr_t addr = (uintptr_t)x;
    int64_t head = (int64_t)(((16u - (unsigned)(addr & 15u)) & 15u) / sizeof(E));
    if (head > n) head = n;
    const int64_t nvec = (n - head) / W;
    const int64_t tail0 = head + nvec * W;
    const V *__restrict__ xv = reinterpret_cast<const V *>(x + head);
    const int64_t stride = (int64_t)gridDim.x * RT;
    int64_t i = (int64_t)blockIdx.x * RT + threadIdx.x;
    for (; i + (RU - 1) * stride < nvec; i += RU * stride) {
        V t[RU];
#pragma unroll
        for (int u = 0; u < RU; ++u) t[u] = __builtin_nontemporal_load(xv + i + u * stride);
#pragma unroll
        for (int u = 0; u < RU; ++u)
#pragma unroll
            for (int e = 0; e < W; ++e) fold(t[u][e]);
    }
    for (; i < nvec; i += stride) {
        const V t = __builtin_nontemporal_load(xv + i);
#pragma unroll
        for (int e = 0; e < W; ++e) fold(t[e]);
    }
    if (blockIdx.x == 0) {
        if ((int64_t)threadIdx.x < head) fold(x[threadIdx.x]);
        if ((int64_t)threadIdx.x < n - tail0) fold(x[tail0 + threadIdx.x]);
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        const E b = block_apply<E>(op[v], acc[v], lds4);
        if (threadIdx.x == 0) partials[(size_t)v * gridDim.x + blockIdx.x] = as_bits<E>(b);
    }
}

// One workgroup folds the g partials of each variable in index order, then
// the initial value.
template <typename E, int NV>
__global__ __launch_bounds__(RT) void reduce_vars_final(const uint64_t *__restrict__ partials, unsigned g,
                                                        RedVars vars, E *__restrict__ result)
{
    __shared__ E lds4[4];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        const int op = vars.op[v];
        E t = red_identity<E>(op);
        for (unsigned k = threadIdx.x; k < g; k += RT) t = red_apply<E>(op, t, bits_as<E>(partials[(size_t)v * g + k]));
        t = block_apply<E>(op, t, lds4);
        if (threadIdx.x == 0) result[v] = red_apply<E>(op, bits_as<E>(vars.init[v]), t);
    }
}

// Logical or as a guarded write (the flag idiom hand-written code uses in
// place of a reduction): result = (init != 0) is stored first; then every
// thread that finds a nonzero element stores 1 (all writers store the same
// value).  A wavefront stops scanning once it sees the flag set.
template <typename E> __global__ void red_flag_init(E *result, uint64_t init_bits)
{
    if (threadIdx.x == 0) result[0] = Red<E>::nonzero(bits_as<E>(init_bits)) ? (E)1 : (E)0;
}

template <typename E>
__global__ __launch_bounds__(RT) void reduce_or_flag(const E *__restrict__ x, int64_t n, E *result)
{
    using R = Red<E>;
    using V = typename R::V;
    constexpr int W = R::W;
    using B = typename R::Bits;
    B *flag = reinterpret_cast<B *>(result);
    const B one = __builtin_bit_cast(B, (E)1);
    const uintptr_t addr = (uintptr_t)x;
    int64_t head = (int64_t)(((16u - (unsigned)(addr & 15u)) & 15u) / sizeof(E));
    if (head > n) head = n;
    const int64_t nvec = (n - head) / W;
    const int64_t tail0 = head + nvec * W;
    const V *__restrict__ xv = reinterpret_cast<const V *>(x + head);
    const int64_t stride = (int64_t)gridDim.x * RT;
    bool found = false;
    if (blockIdx.x == 0) {
        if ((int64_t)threadIdx.x < head) found |= R::nonzero(x[threadIdx.x]);
        if ((int64_t)threadIdx.x < n - tail0) found |= R::nonzero(x[tail0 + threadIdx.x]);
    }
    for (int64_t i = (int64_t)blockIdx.x * RT + threadIdx.x; i - threadIdx.x < nvec; i += RU * stride) {
        // The flag is read with this iteration's data loads and tested after
        // them (a test before the loads would add the flag's latency to every
        // iteration); a wave-uniform early exit once any thread has stored it.
        const B seen = __hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
        for (int u = 0; u < RU; ++u) {
            const int64_t j = i + u * stride;
            if (j < nvec) {
                const V t = __builtin_nontemporal_load(xv + j);
#pragma unroll
                for (int e = 0; e < W; ++e) found |= R::nonzero(t[e]);
            }
        }
        if (found) __hip_atomic_store(flag, one, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (__any(found) || __builtin_amdgcn_readfirstlane((int)(seen == one))) return;  // decided
    }
    if (found) __hip_atomic_store(flag, one, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

int64_t fast_blocks(int64_t n)
{
    const int64_t nvec = n / 4;
    int64_t want = (nvec + (int64_t)RT * RU - 1) / ((int64_t)RT * RU);
    // Three workgroups per CU: a float32 sum over 1 GiB on MI355X (both
    // launches) took 169, 155 and 158 us at 2, 3 and 4 per CU.
    int64_t cap = (int64_t)device_cu_count() * 3;
    if (cap > MAX_BLOCKS) cap = MAX_BLOCKS;
    if (want > cap) want = cap;
    return want < 1 ? 1 : want;
}

int64_t plain_blocks(int64_t n) { return n <= 0 ? 1 : (n + RT - 1) / RT; }

template <typename L>
hipError_t launch_reduce(const L *x, int64_t n, L init, L *result, void *work, bool plain, hipStream_t s)
{
    if (plain) {
        const int64_t g = plain_blocks(n);
        L *partials = static_cast<L *>(work);
        if (n > 0) {
            tmark("reduce_plain_blocks", s, true);
            hipLaunchKernelGGL(reduce_plain_blocks<L>, dim3((unsigned)g), dim3(RT), 0, s, x, n, partials);
            tmark("reduce_plain_blocks", s, false);
        }
        tmark("reduce_plain_final", s, true);
        hipLaunchKernelGGL(reduce_plain_final<L>, dim3(1), dim3(RT), 0, s, partials, n > 0 ? g : 0, init, result);
        tmark("reduce_plain_final", s, false);
    } else {
        const int64_t g = fast_blocks(n);
        uint32_t *partials = static_cast<uint32_t *>(work);
        tmark("reduce_fast", s, true);  // both launches
        hipLaunchKernelGGL(reduce_fast<L>, dim3((unsigned)g), dim3(RT), 0, s, x, n, partials);
        hipLaunchKernelGGL(reduce_fast_final<L>, dim3(1), dim3(RT), 0, s, partials, (unsigned)g, init, result);
        tmark("reduce_fast", s, false);
    }
    return hipGetLastError();
}

template <typename E, int NV, uint32_t SIG>
void launch_sig(const E *x, int64_t n, const RedVars &vars, uint64_t *partials, unsigned g, hipStream_t s)
{
    hipLaunchKernelGGL((reduce_vars<E, NV, SIG>), dim3(g), dim3(RT), 0, s, x, n, vars, partials);
}

// Compiled operator sets: one variable (+, max, min; x or x*x), and the
// pairs the paper's reduction loops use (SRAD's sum and sum of squares) or
// that come as one (max and min); anything else decodes at run time.
template <typename E, int NV>
void launch_vars_nv(const E *x, int64_t n, const RedVars &vars, E *result, uint64_t *partials, unsigned g,
                    hipStream_t s)
{
    uint32_t sig = 0;
    for (int v = 0; v < NV; ++v) sig |= (uint32_t)(vars.op[v] | (vars.square[v] ? 4 : 0)) << (4 * v);
    bool done = true;
    if constexpr (NV == 1) {
        switch (sig) {
        case 0x0: launch_sig<E, 1, 0x0>(x, n, vars, partials, g, s); break;
        case 0x1: launch_sig<E, 1, 0x1>(x, n, vars, partials, g, s); break;
        case 0x2: launch_sig<E, 1, 0x2>(x, n, vars, partials, g, s); break;
        case 0x4: launch_sig<E, 1, 0x4>(x, n, vars, partials, g, s); break;
        case 0x5: launch_sig<E, 1, 0x5>(x, n, vars, partials, g, s); break;
        case 0x6: launch_sig<E, 1, 0x6>(x, n, vars, partials, g, s); break;
        default: done = false;
        }
    } else if constexpr (NV == 2) {
        switch (sig) {
        case 0x40: launch_sig<E, 2, 0x40>(x, n, vars, partials, g, s); break;  // sum, sum of squares
        case 0x04: launch_sig<E, 2, 0x04>(x, n, vars, partials, g, s); break;  // sum of squares, sum
        case 0x21: launch_sig<E, 2, 0x21>(x, n, vars, partials, g, s); break;  // max, min
        case 0x12: launch_sig<E, 2, 0x12>(x, n, vars, partials, g, s); break;  // min, max
        default: done = false;
        }
    } else {
        done = false;
    }
    if (!done) launch_sig<E, NV, SIG_RUNTIME>(x, n, vars, partials, g, s);
    hipLaunchKernelGGL((reduce_vars_final<E, NV>), dim3(1), dim3(RT), 0, s, partials, g, vars, result);
}

template <typename E>
hipError_t launch_vars(const E *x, int64_t n, const RedVars &vars, E *result, void *work, hipStream_t s)
{
    if (vars.op[0] == RED_OR) {
        hipLaunchKernelGGL(red_flag_init<E>, dim3(1), dim3(64), 0, s, result, vars.init[0]);
        if (n > 0) {
            const int64_t g = fast_blocks(n * (int64_t)sizeof(E) / 4);
            tmark("reduce_or_flag", s, true);
            hipLaunchKernelGGL(reduce_or_flag<E>, dim3((unsigned)g), dim3(RT), 0, s, x, n, result);
            tmark("reduce_or_flag", s, false);
        }
        return hipGetLastError();
    }
    const int64_t g = fast_blocks(n * (int64_t)sizeof(E) / 4);
    uint64_t *partials = static_cast<uint64_t *>(work);
    tmark("reduce_vars", s, true);  // both launches
    switch (vars.nvars) {
    case 1: launch_vars_nv<E, 1>(x, n, vars, result, partials, (unsigned)g, s); break;
    case 2: launch_vars_nv<E, 2>(x, n, vars, result, partials, (unsigned)g, s); break;
    case 3: launch_vars_nv<E, 3>(x, n, vars, result, partials, (unsigned)g, s); break;
    case 4: launch_vars_nv<E, 4>(x, n, vars, result, partials, (unsigned)g, s); break;
    default: return hipErrorInvalidValue;
    }
    tmark("reduce_vars", s, false);
    return hipGetLastError();
}

}  // namespace

size_t reduce_vars_workspace_bytes() { return sizeof(uint64_t) * RED_MAX_VARS * MAX_BLOCKS; }

// ---- static scratch for callers that cannot allocate -----------------------
//
// The per-workgroup partials of the reductions, in a device array of fixed
// size instead of an allocated workspace.  Each GPU holds its own copy of
// the array, at its own address, for the life of the process; host code
// never passes the array's name to a kernel (on the host it is only a
// stand-in for the symbol), only the device address hipGetSymbolAddress gave
// for that device.  No call needs its contents to start at zero: every
// reduction overwrites the partials it later reads.
namespace {
static __device__ __align__(256) uint64_t scratch[NOALLOC_SCRATCH_BYTES / sizeof(uint64_t)];
constexpr int NOALLOC_MAX_DEVICES = 64;
void *scratch_ptr[NOALLOC_MAX_DEVICES];  // set once per device, never cleared
}  // namespace

hipError_t noalloc_scratch_setup(int device)
{
    if (device < 0 || device >= NOALLOC_MAX_DEVICES) return hipErrorInvalidDevice;
    if (scratch_ptr[device]) return hipSuccess;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    scratch_ptr[device] = p;
    return hipSuccess;
}

void *noalloc_scratch(int device)
{
    return device >= 0 && device < NOALLOC_MAX_DEVICES ? scratch_ptr[device] : nullptr;
}

hipError_t launch_reduce_vars(int dtype, const void *x, int64_t n, const RedVars &vars, void *result, void *work,
                              hipStream_t s)
{
    switch (dtype) {
    case 0: return launch_vars<float>(static_cast<const float *>(x), n, vars, static_cast<float *>(result), work, s);
    case 1:
        return launch_vars<int32_t>(static_cast<const int32_t *>(x), n, vars, static_cast<int32_t *>(result), work, s);
    case 2: return launch_vars<double>(static_cast<const double *>(x), n, vars, static_cast<double *>(result), work, s);
    case 3:
        return launch_vars<int64_t>(static_cast<const int64_t *>(x), n, vars, static_cast<int64_t *>(result), work, s);
    default: return hipErrorInvalidValue;
    }
}

size_t reduce_fast_workspace_bytes(int64_t) { return sizeof(uint32_t) * MAX_BLOCKS; }

size_t reduce_plain_workspace_bytes(int64_t n) { return sizeof(uint32_t) * (size_t)plain_blocks(n); }

hipError_t launch_reduce_f32(const float *x, int64_t n, float init, float *result, void *work, bool plain,
                             hipStream_t s)
{
    return launch_reduce<float>(x, n, init, result, work, plain, s);
}

hipError_t launch_reduce_final_f32(const uint32_t *partials, int g, float init, float *result, hipStream_t s)
{
    tmark("reduce_final", s, true);
    hipLaunchKernelGGL(reduce_fast_final<float>, dim3(1), dim3(RT), 0, s, partials, (unsigned)g, init, result);
    tmark("reduce_final", s, false);
    return hipGetLastError();
}

hipError_t launch_reduce_i32(const int32_t *x, int64_t n, int32_t init, int32_t *result, void *work, bool plain,
                             hipStream_t s)
{
    return launch_reduce<uint32_t>(reinterpret_cast<const uint32_t *>(x), n, (uint32_t)init,
                                   reinterpret_cast<uint32_t *>(result), work, plain, s);
}

}  // namespace accx
