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
//  - fast: one pass that streams the input at HBM rate.  Each thread keeps
//    eight independent 16-byte accumulators over a grid-stride slice, a
//    wavefront reduces with cross-lane exchanges, the wavefronts of a
//    workgroup combine through LDS, and each workgroup publishes one partial.
//    An atomic ticket elects the last workgroup to finish; it adds all
//    partials in index order, adds the initial value, writes the result and
//    resets the ticket to zero for the next call.
// Both are bitwise deterministic: which workgroup finishes last does not
// change the order in which anything is added.
//
// float: float32 arithmetic throughout.  int32: unsigned 32-bit adds
// (wraparound modulo 2^32).
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace accx {
namespace {

constexpr int RT = 256;          // threads per workgroup
constexpr int RU = 8;            // 16-byte loads in flight per thread
constexpr int MAX_BLOCKS = 4096; // fast kernel: upper bound on workgroups
constexpr size_t TICKET_BYTES = 256;

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
__global__ __launch_bounds__(RT) void reduce_fast(const L *__restrict__ x, int64_t n, L init, L *__restrict__ result,
                                                  uint32_t *__restrict__ ticket, uint32_t *__restrict__ partials)
{
    using V = typename Vec<L>::T;
    __shared__ L lds4[4];
    __shared__ int is_last;

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

    if (threadIdx.x == 0) {
        __hip_atomic_store(partials + blockIdx.x, to_bits(s), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __threadfence();
        const uint32_t prev = atomicAdd(ticket, 1u);
        is_last = (prev == gridDim.x - 1);
    }
    __syncthreads();
    if (!is_last) return;
    __threadfence();

    L t = 0;
    for (unsigned k = threadIdx.x; k < gridDim.x; k += RT)
        t = t + from_bits<L>(__hip_atomic_load(partials + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    __syncthreads();  // lds4 reuse
    t = block_sum(t, lds4);
    if (threadIdx.x == 0) {
        result[0] = init + t;
        __hip_atomic_store(ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
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

int64_t fast_blocks(int64_t n)
{
    const int64_t nvec = n / 4;
    int64_t want = (nvec + (int64_t)RT * RU - 1) / ((int64_t)RT * RU);
    // Two workgroups per CU: measured on MI355X, more resident streams lower
    // the achieved read bandwidth of this kernel.
    int64_t cap = (int64_t)device_cu_count() * 2;
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
        uint32_t *ticket = static_cast<uint32_t *>(work);
        uint32_t *partials = reinterpret_cast<uint32_t *>(static_cast<char *>(work) + TICKET_BYTES);
        tmark("reduce_fast", s, true);
        hipLaunchKernelGGL(reduce_fast<L>, dim3((unsigned)g), dim3(RT), 0, s, x, n, init, result, ticket, partials);
        tmark("reduce_fast", s, false);
    }
    return hipGetLastError();
}

}  // namespace

size_t reduce_fast_workspace_bytes(int64_t) { return TICKET_BYTES + sizeof(uint32_t) * MAX_BLOCKS; }

size_t reduce_plain_workspace_bytes(int64_t n) { return sizeof(uint32_t) * (size_t)plain_blocks(n); }

hipError_t launch_reduce_f32(const float *x, int64_t n, float init, float *result, void *work, bool plain,
                             hipStream_t s)
{
    return launch_reduce<float>(x, n, init, result, work, plain, s);
}

hipError_t launch_reduce_i32(const int32_t *x, int64_t n, int32_t init, int32_t *result, void *work, bool plain,
                             hipStream_t s)
{
    return launch_reduce<uint32_t>(reinterpret_cast<const uint32_t *>(x), n, (uint32_t)init,
                                   reinterpret_cast<uint32_t *>(result), work, plain, s);
}

}  // namespace accx
