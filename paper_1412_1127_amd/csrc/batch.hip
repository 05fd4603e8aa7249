// Batched offload: many independent loop-nest matmuls (Listing 1a,
// section 1.3) and reduction(+) clauses (section 2.3; SRAD paragraph of
// section 4.2) run as one graph of two kernels:
//
//  1. batch_pack: the bf16x3 split of every matmul operand, each operand on
//     a number of workgroups in proportion to its size (descriptor table of
//     pack jobs, and the job of each workgroup);
//  2. batch_persistent: a persistent kernel (a fixed number of workgroups per
//     CU) that pulls work units from one queue through an atomic counter:
//     either one output tile of one matmul (the same LDS-tiled matrix-core
//     tile as the standalone kernel, in the tile configuration chosen for
//     that matmul's size class) or one chunk of one reduction.  The queue
//     interleaves matmul tiles (largest matmuls first) with reduction chunks
//     so that HBM-bound and matrix-core-bound work share the CUs.
//
// A reduction's chunk partials are combined by the workgroup that finishes
// its last chunk (atomic ticket), in chunk order, so results do not depend
// on which workgroup ran what.  A matmul tile is computed by one workgroup in
// fixed K order, bitwise as by the standalone kernel in the same tile
// configuration when that one runs unsplit (no split K).  The last workgroup
// to leave resets the queue counters, so the graph can be replayed with no
// memset node.
//
// Precision: six products (FULL6), or AUTO: the three-product pass of the
// tile, then the same workgroup probes that tile in float64 (probe_tile:
// the standalone probe's samples, summed in the order of this kernel's
// 256-thread workgroups) and, if the tile is
// marked, adds the three correction products over its 64 x 64 sub-tiles --
// the standalone AUTO path's steps for that tile, done in place, so no other
// workgroup and no other launch is involved.
#include <hip/hip_runtime.h>

#include "kernels.h"
#include "mfma_tile.h"

namespace accx {
namespace {

using namespace dev;

constexpr int BT = 256;              // threads per workgroup (both kernels)
constexpr int WG_PER_CU = 2;         // persistent workgroups per CU (LDS: 2 x 72 KB)
constexpr uint32_t UNIT_RED = 0x80000000u;

// Tile variants the persistent kernels carry: T128 (first-product
// look-ahead) and T64; six products (FULL6), or three (CHEAP3) plus the
// correction products on T64 (AUTO), one kernel per precision.
#define ACCX_T128(NP, PLIST) false, 3, 128, 128, 32, 2, 2, 3, NP, PLIST, 1, 2
#define ACCX_T64(NP, PLIST) false, 3, 64, 64, 64, 2, 2, 2, NP, PLIST, 1

constexpr int cmax(int a, int b) { return a > b ? a : b; }
constexpr int LDS_MAX = cmax(cmax(gemm_lds_bytes<128, 128, 32, 3, 6, PL_FULL6>(), gemm_lds_bytes<64, 64, 64, 2, 6, PL_FULL6>()),
                             (int)sizeof(ProbeLds));
static_assert(LDS_MAX * WG_PER_CU <= 160 * 1024, "persistent kernel LDS");

// One workgroup of the pack launch: a share of one operand's chunks (the
// operand's workgroups split its chunks grid-stride among themselves).
__global__ __launch_bounds__(BT) void batch_pack(const BatchPackJob *__restrict__ jobs,
                                                 const uint32_t *__restrict__ job_of)
{
    const BatchPackJob j = jobs[job_of[blockIdx.x]];
    const int64_t id0 = (int64_t)(blockIdx.x - j.wg0) * BT + threadIdx.x, step = (int64_t)j.nwg * BT;
    if (j.trans)
        pack_bf16x3_range<true>(j.x, j.rows, j.k, j.ld, j.out, j.nrb, j.nkb, id0, step);
    else
        pack_bf16x3_range<false>(j.x, j.rows, j.k, j.ld, j.out, j.nrb, j.nkb, id0, step);
}

__device__ inline float wave_sum_f(float v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sum over the workgroup in fixed order; valid in thread 0.
__device__ inline float block_sum_f(float v, float *red4)
{
    v = wave_sum_f(v);
    if ((threadIdx.x & 63) == 0) red4[threadIdx.x >> 6] = v;
    __syncthreads();
    const float r = (threadIdx.x == 0) ? (red4[0] + red4[1]) + (red4[2] + red4[3]) : 0.0f;
    __syncthreads();
    return r;
}

typedef float f4v __attribute__((ext_vector_type(4)));

__device__ __attribute__((always_inline)) inline void reduce_chunk(const BatchRed &r, uint32_t chunk, float *red4, int *is_last)
{
    const int64_t b0 = (int64_t)chunk * r.chunk;
    const int64_t b1 = b0 + r.chunk < r.n ? b0 + r.chunk : r.n;
    const float *__restrict__ x = r.x;
    float s = 0.0f;
    if ((((uintptr_t)(x + b0)) & 15u) == 0) {
        const int64_t nv = (b1 - b0) >> 2;
        const f4v *__restrict__ xv = reinterpret_cast<const f4v *>(x + b0);
        // eight 16-byte loads in flight per thread
        f4v acc[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) acc[u] = (f4v)0;
        int64_t v = threadIdx.x;
        for (; v + 7 * BT < nv; v += 8 * BT) {
            f4v t[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) t[u] = __builtin_nontemporal_load(xv + v + u * BT);
#pragma unroll
            for (int u = 0; u < 8; ++u) acc[u] += t[u];
        }
        for (; v < nv; v += BT) acc[0] += xv[v];
#pragma unroll
        for (int w = 4; w > 0; w >>= 1)
#pragma unroll
            for (int u = 0; u < w; ++u) acc[u] += acc[u + w];
        s = (acc[0].x + acc[0].y) + (acc[0].z + acc[0].w);
        for (int64_t e = b0 + (nv << 2) + threadIdx.x; e < b1; e += BT) s += x[e];
    } else {
        for (int64_t e = b0 + threadIdx.x; e < b1; e += BT) s += x[e];
    }
    s = block_sum_f(s, red4);
    if (threadIdx.x == 0) {
        // The partial goes out as a device-scope store (through to the
        // level the XCDs share) and counts as done before the ticket; the
        // last chunk reads the partials with device-scope loads.  No fence:
        // a device-scope fence writes back and invalidates this XCD's whole
        // L2 under the matmul tiles that share it, once per chunk.
        __hip_atomic_store(r.partials + chunk, __float_as_uint(s), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        asm volatile("" ::: "memory");
        __builtin_amdgcn_s_waitcnt(vmcnt_imm<0>());
        asm volatile("" ::: "memory");
        *is_last = (atomicAdd(r.ticket, 1u) == (uint32_t)r.nchunks - 1);
    }
    __syncthreads();
    if (!*is_last) return;
    float t = 0.0f;
    for (int k = threadIdx.x; k < r.nchunks; k += BT)
        t += __uint_as_float(__hip_atomic_load(r.partials + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    t = block_sum_f(t, red4);
    if (threadIdx.x == 0) {
        *r.result = r.init + t;
        __hip_atomic_store(r.ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

template <bool AUTO>
__device__ __attribute__((always_inline)) inline void matmul_unit(const BatchMat &m, uint32_t tile, char *lds,
                                                                  double tau2)
{
    GemmArgs g{};
    g.A = m.pa;
    g.B = m.pb;
    g.C = m.c;
    g.M = g.N = g.ldc = m.len;
    g.nkb = m.nkb;
    g.nrb_a = g.nrb_b = (m.len + 31) / 32;
    g.tiles_m = m.tiles_m;
    g.tiles_n = m.tiles_n;
    const int tm = (int)(tile / (uint32_t)m.tiles_n), tn = (int)(tile % (uint32_t)m.tiles_n);
    const bool t128 = m.tile == GEMM_TILE_128;
    if constexpr (!AUTO) {
        if (t128)
            gemm_tile<ACCX_T128(6, PL_FULL6)>(g, tm, tn, lds);
        else
            gemm_tile<ACCX_T64(6, PL_FULL6)>(g, tm, tn, lds);
    } else {
        if (t128)
            gemm_tile<ACCX_T128(3, PL_CHEAP3)>(g, tm, tn, lds);
        else
            gemm_tile<ACCX_T64(3, PL_CHEAP3)>(g, tm, tn, lds);
        // This tile of C is read back only by this workgroup (probe, then the
        // correction's read-modify-write), so the barrier's workgroup-scope
        // release and acquire make it visible; a device-scope fence here
        // would write back the L2 after every tile.  The LDS stages are free
        // after the barrier too.
        __syncthreads();
        const int bt = t128 ? 128 : 64;
        if (!probe_tile<BT>(m.pa, m.pb, m.c, m.len, m.len, m.len, m.len, bt, bt, tile, tm, tn, m.nkb, tau2, nullptr,
                            *reinterpret_cast<ProbeLds *>(lds)))
            return;
        // marked: C += the three correction products, on the 64 x 64 tiles
        // inside this one (those that lie in C), as the standalone correction
        GemmArgs h = g;
        h.accumulate = 1;
        h.tiles_m = h.tiles_n = (int)((m.len + 63) / 64);
        const int sub = bt / 64;
        for (int i = 0; i < sub; ++i)
            for (int j = 0; j < sub; ++j) {
                const int sm = tm * sub + i, sn = tn * sub + j;
                if (sm >= h.tiles_m || sn >= h.tiles_n) continue;
                __syncthreads();  // the LDS stages are reused
                gemm_tile<ACCX_T64(3, PL_CORR3)>(h, sm, sn, lds);
            }
    }
}

template <bool AUTO>
__global__ __launch_bounds__(BT, WG_PER_CU) void batch_persistent(BatchQueue q)
{
    __shared__ __attribute__((aligned(1024))) char lds[LDS_MAX];
    __shared__ uint32_t cur;
    __shared__ float red4[4];
    __shared__ int is_last;
    for (;;) {
        if (threadIdx.x == 0) cur = atomicAdd(q.counter, 1u);
        __syncthreads();
        const uint32_t u = cur;
        __syncthreads();  // every thread has read `cur` before it is rewritten
        if (u >= q.nunits) break;
        const BatchUnit w = q.units[u];
        if (w.item & UNIT_RED)
            reduce_chunk(q.reds[w.item & ~UNIT_RED], w.sub, red4, &is_last);
        else
            matmul_unit<AUTO>(q.mats[w.item], w.sub, lds, q.tau2);
        __syncthreads();  // LDS and shared scalars are reused by the next unit
    }
    // The last workgroup out resets the queue for the next launch.  Only
    // device-scope atomics take part: each workgroup's last pull from the
    // counter precedes its exit count in its own program order.  No fence,
    // which would write back and invalidate this XCD's L2 under the
    // workgroups still running.
    if (threadIdx.x == 0) {
        if (atomicAdd(q.done, 1u) == gridDim.x - 1) {
            __hip_atomic_store(q.counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(q.done, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

}  // namespace

int batch_tile_supported(int tile) { return tile == GEMM_TILE_128 || tile == GEMM_TILE_64; }

int batch_workgroups() { return device_cu_count() * WG_PER_CU; }

int batch_pack_workgroups(int64_t nrb, int64_t nkb)
{
    const int64_t chunks = nrb * nkb * 128;  // pack_bf16x3_range's work items
    return (int)std::min<int64_t>(4096, std::max<int64_t>(1, (chunks + BT - 1) / BT));
}

hipError_t launch_batch_pack(const BatchPackJob *jobs, const uint32_t *job_of, int64_t nwg, hipStream_t s)
{
    if (nwg <= 0) return hipSuccess;
    tmark("batch_pack", s, true);
    hipLaunchKernelGGL(batch_pack, dim3((unsigned)nwg), dim3(BT), 0, s, jobs, job_of);
    tmark("batch_pack", s, false);
    return hipGetLastError();
}

hipError_t launch_batch_persistent(const BatchQueue &q, hipStream_t s)
{
    tmark("batch_persistent", s, true);
    if (q.auto_prec)
        hipLaunchKernelGGL(batch_persistent<true>, dim3((unsigned)batch_workgroups()), dim3(BT), 0, s, q);
    else
        hipLaunchKernelGGL(batch_persistent<false>, dim3((unsigned)batch_workgroups()), dim3(BT), 0, s, q);
    tmark("batch_persistent", s, false);
    return hipGetLastError();
}

}  // namespace accx
