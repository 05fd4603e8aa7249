// Device-side building blocks shared by the tiled matmul kernels
// (gemm_mfma.hip) and the persistent batch kernel (batch.hip): the bf16x3
// split, the packed operand layout, and the LDS-tiled matrix-core tile.
// Device functions and constants only; the kernels live in the .hip files.
//
// Packed operand layout.  An operand of R rows of K elements (A: rows of A;
// B: columns of B, i.e. rows of B^T) with P planes is cut into units of 32
// rows x 64 bytes of each plane.  Unit (rb, kb) starts at byte
// (rb*nkb + kb) * P * 2048; inside it, plane p, 16-byte chunk c (0..3) of
// row r (0..31) is at p*2048 + c*512 + r*16.  Rows >= R and elements >= K
// are zero.  The layout makes every global->LDS copy a contiguous 1 KB block
// (one direct-to-LDS dwordx4 load per wavefront) and every matrix-core
// operand fetch a conflict-free ds_read_b128 of 1 KB (lane l: row l%32,
// chunk l/32).
#pragma once

#include <hip/hip_runtime.h>

#include "kernels.h"

namespace accx {
namespace dev {


typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef int i32x16 __attribute__((ext_vector_type(16)));
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));

constexpr int PLANE_BYTES = 2048;  // 32 rows x 64 bytes

// ---------------------------------------------------------------- packing --

__device__ inline uint16_t bf16_bits(__bf16 h) { return __builtin_bit_cast(uint16_t, h); }

// x = hi + mid + lo, each term rounded to nearest even bf16 (v_cvt_pk_bf16_f32).
// x - hi and (x - hi) - mid are exact in float32.
__device__ inline void split3(float x, uint16_t &h, uint16_t &m, uint16_t &l)
{
    const __bf16 bh = (__bf16)x;
    const float r1 = x - (float)bh;
    const __bf16 bm = (__bf16)r1;
    const float r2 = r1 - (float)bm;
    h = bf16_bits(bh);
    m = bf16_bits(bm);
    l = bf16_bits((__bf16)r2);
}

// One thread per (unit, row, chunk): 8 consecutive K elements of one row.
// TRANS = false: X is R x K row-major (operand row r = X row r), element
//                (r, e) at X[r*ld + e].
// TRANS = true:  X is K x R row-major (operand row r = X column r), element
//                (e, r) at X[e*ld + r].
// Work items id0, id0 + step, ... of one operand (128 items per unit).
template <bool TRANS>
__device__ __attribute__((always_inline)) inline void pack_bf16x3_range(const float *__restrict__ X, int64_t R,
                                                                        int64_t K, int64_t ld,
                                                                        char *__restrict__ out, int64_t nrb,
                                                                        int64_t nkb, int64_t id0, int64_t step)
{
    const int64_t total = nrb * nkb * 128;
    for (int64_t id = id0; id < total; id += step) {
        const int64_t unit = id >> 7;
        const int w = (int)(id & 127);
        int r, c;
        if (TRANS) {
            r = w & 31;
            c = w >> 5;
        } else {
            r = w >> 2;
            c = w & 3;
        }
        const int64_t rb = unit / nkb, kb = unit - rb * nkb;
        const int64_t row = rb * 32 + r;
        const int64_t k0 = kb * 32 + c * 8;
        float v[8];
        if (TRANS) {
#pragma unroll
            for (int t = 0; t < 8; ++t) v[t] = (row < R && k0 + t < K) ? X[(k0 + t) * ld + row] : 0.0f;
        } else if (row < R && k0 + 8 <= K && ((ld & 3) == 0) && (((uintptr_t)X & 15u) == 0)) {
            const f32x4 *p = reinterpret_cast<const f32x4 *>(X + row * ld + k0);
            // read once: non-temporal, so that the stream keeps out of the caches
            const f32x4 a = __builtin_nontemporal_load(p), b = __builtin_nontemporal_load(p + 1);
            v[0] = a.x, v[1] = a.y, v[2] = a.z, v[3] = a.w, v[4] = b.x, v[5] = b.y, v[6] = b.z, v[7] = b.w;
        } else {
#pragma unroll
            for (int t = 0; t < 8; ++t) v[t] = (row < R && k0 + t < K) ? X[row * ld + k0 + t] : 0.0f;
        }
        u16x8 h, m, l;
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            uint16_t a, b, d;
            split3(v[t], a, b, d);
            h[t] = a;
            m[t] = b;
            l[t] = d;
        }
        char *u = out + unit * (3 * PLANE_BYTES) + c * 512 + r * 16;
        *reinterpret_cast<u16x8 *>(u) = h;
        *reinterpret_cast<u16x8 *>(u + PLANE_BYTES) = m;
        *reinterpret_cast<u16x8 *>(u + 2 * PLANE_BYTES) = l;
    }
}

// ------------------------------------------------------------------- GEMM --

// 16-byte direct global->LDS load of one wavefront: lane l reads 16 bytes at
// its own `src` and they land at dst + 16*l (dst is wavefront-uniform; M0
// holds its LDS address).  Issued as inline assembly, not through the
// compiler's builtin: for the builtin the compiler cannot tell the LDS bytes
// a load writes from those the following reads use, and waits for every
// load in flight before the first LDS read after it, i.e. for the stage just
// issued, which undoes the ring's prefetch.  The kernels order these loads
// themselves: s_waitcnt vmcnt(N) for the stage they read, then a barrier.
__device__ inline void dma16(const void *src, void *dst)
{
    const uint32_t lds = __builtin_amdgcn_readfirstlane((uint32_t)(uintptr_t)dst);
    asm volatile("global_load_lds_dwordx4 %0, off" ::"v"(src), "{m0}"(lds) : "memory");
}
// The same with the non-temporal hint, for data read once (streaming): on
// the co-scheduled reduction's loads it keeps the stream from displacing the
// GEMM operands that other tiles re-read (fused pass 0.41 -> 0.39 ms at
// LEN=4096 with 2^28 floats).
__device__ inline void dma16_nt(const void *src, void *dst)
{
    const uint32_t lds = __builtin_amdgcn_readfirstlane((uint32_t)(uintptr_t)dst);
    asm volatile("global_load_lds_dwordx4 %0, off nt" ::"v"(src), "{m0}"(lds) : "memory");
}

template <bool INT8> struct Mma;
template <> struct Mma<false> {
    using Frag = bf16x8;
    using Acc = f32x16;
    using Elem = float;
    __device__ static inline Acc run(Frag a, Frag b, Acc c)
    {
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
    }
};
template <> struct Mma<true> {
    using Frag = i32x4;
    using Acc = i32x16;
    using Elem = int;
    __device__ static inline Acc run(Frag a, Frag b, Acc c)
    {
        return __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b, c, 0, 0, 0);
    }
};

// float32 on the float32 matrix cores (v_mfma_f32_32x32x2_f32: K = 2 per
// instruction, one float of A and one of B per lane).  A fragment is the
// 16-byte chunk a lane reads from the packed layout: four consecutive k of
// one row, the lanes of the upper half one chunk further along K.  The four
// instructions of one fragment pair take its elements 0..3 in turn, so
// instruction j sums, for each row and column, k = 8q + j (lower half) and
// k = 8q + 4 + j (upper half): A and B pair the same k, and the eight k of
// the chunk pair are covered once each.
struct MmaF32 {
    using Frag = f32x4;
    using Acc = f32x16;
    using Elem = float;
    __device__ static inline Acc run(Frag a, Frag b, Acc c)
    {
        c = __builtin_amdgcn_mfma_f32_32x32x2f32(a[0], b[0], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_32x32x2f32(a[1], b[1], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_32x32x2f32(a[2], b[2], c, 0, 0, 0);
        return __builtin_amdgcn_mfma_f32_32x32x2f32(a[3], b[3], c, 0, 0, 0);
    }
};

template <bool C, typename T, typename F> struct Pick { using type = T; };
template <typename T, typename F> struct Pick<false, T, F> { using type = F; };

// Product list: entry t = (plane of A, plane of B, accumulator) in 6 bits.
constexpr uint64_t prod(int t, int p, int q, int acc)
{
    return (uint64_t)(p | (q << 2) | (acc << 4)) << (6 * t);
}
constexpr int prod_p(uint64_t L, int t) { return (int)((L >> (6 * t)) & 3); }
constexpr int prod_q(uint64_t L, int t) { return (int)((L >> (6 * t + 2)) & 3); }
constexpr int prod_acc(uint64_t L, int t) { return (int)((L >> (6 * t + 4)) & 3); }

// bf16x3: hi*hi, hi*mid, mid*hi | hi*lo, lo*hi, mid*mid
constexpr uint64_t PL_CHEAP3 = prod(0, 0, 0, 0) | prod(1, 0, 1, 0) | prod(2, 1, 0, 0);
constexpr uint64_t PL_FULL6 = PL_CHEAP3 | prod(3, 0, 2, 0) | prod(4, 2, 0, 0) | prod(5, 1, 1, 0);
constexpr uint64_t PL_CORR3 = prod(0, 0, 2, 0) | prod(1, 2, 0, 0) | prod(2, 1, 1, 0);
// FULL6 without mid*mid: |mid| <= 2^-8 |x|, so the dropped term is the
// smallest of the three second-order ones
constexpr uint64_t PL_FIVE = PL_CHEAP3 | prod(3, 0, 2, 0) | prod(4, 2, 0, 0);
// int8 limbs, accumulator = shift group k+m
constexpr uint64_t PL_L1 = prod(0, 0, 0, 0);
constexpr uint64_t PL_L2 = prod(0, 0, 0, 0) | prod(1, 0, 1, 1) | prod(2, 1, 0, 1) | prod(3, 1, 1, 2);
constexpr uint64_t PL_L3 = prod(0, 0, 0, 0) | prod(1, 0, 1, 1) | prod(2, 1, 0, 1) | prod(3, 0, 2, 2) |
                           prod(4, 1, 1, 2) | prod(5, 2, 0, 2) | prod(6, 1, 2, 3) | prod(7, 2, 1, 3);
constexpr uint64_t PL_L4 = PL_L3 | prod(8, 0, 3, 3) | prod(9, 3, 0, 3);

// Product t is the first of products 1..t to need A plane prod_p(L, t) (or B
// plane prod_q(L, t)), and that plane is not the one product 0 uses.
constexpr bool first_use_a(uint64_t L, int t)
{
    if (prod_p(L, t) == prod_p(L, 0)) return false;
    for (int u = 1; u < t; ++u)
        if (prod_p(L, u) == prod_p(L, t)) return false;
    return true;
}
constexpr bool first_use_b(uint64_t L, int t)
{
    if (prod_q(L, t) == prod_q(L, 0)) return false;
    for (int u = 1; u < t; ++u)
        if (prod_q(L, u) == prod_q(L, t)) return false;
    return true;
}

// Fragment reads of products 1..nprod-1 beyond product 0's planes.
constexpr int later_reads(uint64_t L, int nprod, int wbm, int wbn)
{
    int r = 0;
    for (int t = 1; t < nprod; ++t) r += (first_use_a(L, t) ? wbm : 0) + (first_use_b(L, t) ? wbn : 0);
    return r;
}

// Planes a product list touches: 1 + the largest plane index on either side.
constexpr int planes_used(uint64_t L, int nprod)
{
    int m = 0;
    for (int t = 0; t < nprod; ++t) {
        m = prod_p(L, t) > m ? prod_p(L, t) : m;
        m = prod_q(L, t) > m ? prod_q(L, t) : m;
    }
    return m + 1;
}

// Most parts a split-K launch cuts the K range into.
constexpr int KSPLIT_MAX = 8;

struct GemmArgs {
    const char *A;  // packed A, P planes
    const char *B;  // packed B^T, P planes
    void *C;        // M x N row-major, leading dimension ldc
    int64_t M, N, ldc;
    int64_t nkb;     // 64-byte K units per row
    int64_t nrb_a;   // 32-row blocks present in packed A
    int64_t nrb_b;   // 32-row blocks present in packed B
    int tiles_m, tiles_n;
    int accumulate;  // float: C += result instead of C = result
    const ProbeRecord *probe;  // non-null: skip tiles whose record says no correction
    int probe_shm, probe_shn;  // log2 of (probed tile) / (this tile), rows and columns
    int probe_tiles_n;         // probed tiles per row of C
    const uint64_t *decide;    // non-null: run only if limb_gate(decide, gen, expect)
    uint32_t gen;              // the call's stamp in the decide words
    int expect;
    // Split K: ksplit > 1 cuts the K range into ksplit parts (kb_count units
    // each, the last shorter); the workgroup of part `split` of tile `tile`
    // stores its partial sums to `partials`, and the last of a tile's parts to
    // finish (ticket) adds them in part order and writes C.
    int ksplit, split, tile;
    int64_t kb_count;     // 64-byte K units this workgroup runs (<= nkb)
    void *partials;       // ksplit x tiles x BM x BN 4-byte words
    uint32_t *tickets;    // one per tile: zero before the launch, left at zero
    // Co-scheduled reduction (the fused launch only, unsplit): besides its
    // tile, workgroup b adds the 16-byte vectors [b * red_per, (b + 1) *
    // red_per) of red_x (at most red_nvec) and the red_ntail (< 4) floats
    // after them if b is 0, and leaves its sum's bits in red_part[b].
    const float *red_x;
    int64_t red_nvec, red_per;
    int red_ntail;
    uint32_t *red_part;
};

// The one-digit pass leaves, per operand, a 64-bit word (stamp << 32 |
// max |x|) in which it records maxima above 127 only; the stamp is the
// call's own (a number the host draws per call, never 0).  A word with
// another stamp -- left by an earlier call, or whatever the workspace held
// -- was not written by this call and reads as 0.  The words never need
// clearing: a reader can only see this call's stamp with a maximum the call
// recorded (or, if stale contents happen to carry the same stamp, with a
// larger one, which can only ask for more digits than needed).
__device__ inline uint32_t recorded_max(uint64_t w, uint32_t stamp)
{
    return (uint32_t)(w >> 32) == stamp ? (uint32_t)w : 0u;
}

// Digits the int8 path needs for two operands with the given max |x| words:
// the fewest balanced base-256 digits that hold every value exactly (four
// hold any int32 modulo 2^32).  A max |x| up to 127 may read as zero (only
// larger maxima are recorded): the answer is one digit either way.
__device__ inline int limbs_needed(const uint64_t *maxabs2, uint32_t stamp)
{
    const uint32_t a = recorded_max(maxabs2[0], stamp), b = recorded_max(maxabs2[1], stamp);
    const uint32_t m = a > b ? a : b;
    return m <= 127u ? 1 : m <= 32639u ? 2 : m <= 8355711u ? 3 : 4;
}

// The one-digit kernels (expect = 1) run when one digit is enough; the
// multi-digit kernels (expect = 4) serve every other case.
__device__ inline bool limb_gate(const uint64_t *maxabs2, uint32_t stamp, int expect)
{
    return (limbs_needed(maxabs2, stamp) == 1) == (expect == 1);
}

// Map the linear workgroup id to an output tile.  Workgroups are dealt to
// the 8 XCDs round-robin; give each XCD a contiguous run of the grouped tile
// order so that the workgroups sharing an L2 also share A and B tiles.
__device__ inline void tile_of(int bid, int tiles_m, int tiles_n, int &tm, int &tn)
{
    const int T = tiles_m * tiles_n;
    int t = bid;
    if ((T & 7) == 0) t = (bid & 7) * (T >> 3) + (bid >> 3);
    constexpr int GM = 8;
    const int per_group = GM * tiles_n;
    const int g = t / per_group;
    const int first = g * GM;
    const int gsz = min(tiles_m - first, GM);
    const int w = t - g * per_group;
    tm = first + w % gsz;
    tn = w / gsz;
}

// The 32-bit pattern of an accumulator element, taken by value (a bit cast
// applied to a vector-element expression itself reads element 0).
__device__ inline uint32_t word_of(float v) { return __float_as_uint(v); }
__device__ inline uint32_t word_of(int v) { return (uint32_t)v; }

// s_waitcnt immediate that waits until at most N vector-memory operations of
// this wavefront are outstanding (gfx9 encoding: vmcnt[3:0] and [15:14],
// expcnt and lgkmcnt left at their maxima).
template <int N> constexpr int vmcnt_imm() { return (N & 15) | (7 << 4) | (15 << 8) | ((N >> 4) << 14); }

// One workgroup computes the BM x BN tile (tm, tn) of C with WGM x WGN
// wavefronts, staging operands in `lds` (gemm_lds_bytes bytes, 1 KB aligned).
// The K loop runs over K-steps of KBK bytes per row per plane, staged in LDS
// through an NS-deep ring: the direct-to-LDS loads of step s+NS-1 are in
// flight while step s is computed.  Every wavefront issues the same number
// of loads per step (row blocks past the operand are clamped to its last
// block; those rows of C are never stored), so the wait for step s is a
// fixed count of younger loads.  A raw s_barrier (no memory fence, which
// would wait for every load) separates the steps: each wavefront waits for
// its own loads first, and every LDS read of a step is consumed by a matrix
// instruction before the wavefront reaches the next barrier, so a buffer is
// only overwritten after all wavefronts are done reading it.
// LDS bytes the tile needs: NS stages of (BM + BN)/32 units of NPL planes.
template <int BM, int BN, int KBK, int NS, int NPROD, uint64_t PL>
constexpr int gemm_lds_bytes()
{
    return NS * (BM / 32 + BN / 32) * planes_used(PL, NPROD) * 32 * KBK;
}
// The co-scheduled reduction's 16-byte vectors per thread per K-step, and
// the LDS its ring adds to a tile of THREADS threads and NS stages.
constexpr int RED_RV = 2;
template <int THREADS, int NS> constexpr int red_lds_bytes() { return NS * THREADS * RED_RV * 16; }

//
// LAM selects the main loop: 0 plain (wait, barrier, read, compute), 1 full
// look-ahead, 2 first-product look-ahead (described at its loop below).
// Full look-ahead: each iteration waits for the NEXT stage, reads its
// operand fragments from LDS into a second register set and runs the matrix
// instructions of the current stage from registers, with the LDS reads
// spread between the matrix instructions (one read per NMFMA/NREAD of them;
// issuing the reads in bursts next to the matrix instructions measured
// several times slower on gfx950).  The LDS read latency of one step then
// hides behind the matrix work of the previous one even with a single
// wavefront per SIMD.  It costs a second fragment register set and one step
// of global-load lead (needs NS >= 3).
// F32MM: float32 operands (one plane of 4-byte elements) on the float32
// matrix cores (MmaF32) instead of bf16 planes; plain loop only.
// RED: the tile also runs the co-scheduled reduction of GemmArgs (red_*):
// each K-step issues RV 16-byte non-temporal loads per thread of its slice
// beside the step's operand loads and adds them after the next step's wait,
// so the HBM-bound sum runs in the shadow of the matrix work (first-product
// look-ahead loop, three stages); what the K loop leaves of the slice is
// added after it.
template <bool INT8, int P, int BM, int BN, int KBK, int WGM, int WGN, int NS, int NPROD, uint64_t PL, int NACC,
          int LAM = 0, bool F32MM = false, bool RED = false>
__device__ __attribute__((always_inline)) inline void gemm_tile(const GemmArgs &g, int tm, int tn, char *lds)
{
    using M = typename Pick<F32MM, MmaF32, Mma<INT8>>::type;
    static_assert(!F32MM || (!INT8 && LAM == 0 && P == 1), "float32 matrix cores: one plane, plain loop");
    using Frag = typename M::Frag;
    using Acc = typename M::Acc;
    constexpr int WAVES = WGM * WGN;
    constexpr int NPL = planes_used(PL, NPROD);        // planes staged in LDS (<= P)
    constexpr int MB = BM / 32, NB = BN / 32;          // 32-row units per tile
    constexpr int WBM = MB / WGM, WBN = NB / WGN;      // 32x32 blocks per wave
    constexpr int LUNIT = NPL * 32 * KBK;              // LDS bytes per unit per K-step
    constexpr int CPU = NPL * KBK / 32;                // 1 KB copies per unit per K-step
    constexpr int NCOPY = (MB + NB) * CPU;
    constexpr int LPW = NCOPY / WAVES;                 // loads per wave per K-step
    constexpr int STAGE = (MB + NB) * LUNIT;
    constexpr int SUB = KBK / 32;                      // matrix-core K steps per K-step
    constexpr int HALVES = 64 / KBK;                   // K-steps per 64-byte unit
    static_assert(MB % WGM == 0 && NB % WGN == 0, "tile/wave mismatch");
    static_assert(KBK == 32 || KBK == 64, "K step is 32 or 64 bytes");
    static_assert(NCOPY % WAVES == 0, "loads must divide evenly over the wavefronts");
    static_assert(NS >= 2 && LPW * (NS - 2) < 64, "vmcnt range");
    static_assert(LAM == 0 || NS >= 3, "look-ahead needs three stages");
    static_assert(LAM != 2 || (SUB == 1 && NPROD > 1), "first-product look-ahead: one matrix step per stage");
    static_assert(NS * STAGE <= 160 * 1024, "LDS");
    static_assert(NPL <= P, "product list names a plane the operand lacks");
    static_assert(!RED || (LAM == 2 && NS == 3 && !INT8), "co-scheduled reduction: first-product look-ahead, 3 stages");

    // wavefront index in a scalar register: everything derived from it
    // (copy descriptors, fragment offsets) stays out of vector registers
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int wm = wave / WGN, wn = wave % WGN;
    const int64_t ustride = (int64_t)P * PLANE_BYTES;  // bytes per packed unit
    const int64_t rb0 = (int64_t)tm * MB, cb0 = (int64_t)tn * NB;
    const int nsteps = (int)((g.ksplit > 1 ? g.kb_count : g.nkb) * HALVES);

    // Per-wave copy descriptors: global unit-row base and LDS offset.
    const char *src_base[LPW];
    int dst_off[LPW];
#pragma unroll
    for (int c = 0; c < LPW; ++c) {
        const int q = c * WAVES + wave;
        const bool isA = q < MB * CPU;
        const int qq = isA ? q : q - MB * CPU;
        const int u = qq / CPU, part = qq % CPU;
        const int p = part / (KBK / 32), piece = part % (KBK / 32);
        int64_t rb = (isA ? rb0 : cb0) + u;
        const int64_t nrb = isA ? g.nrb_a : g.nrb_b;
        if (rb >= nrb) rb = nrb - 1;
        src_base[c] = (isA ? g.A : g.B) + rb * g.nkb * ustride + p * PLANE_BYTES + piece * 1024;
        dst_off[c] = (isA ? 0 : MB * LUNIT) + u * LUNIT + p * (32 * KBK) + piece * 1024;
    }

    // Co-scheduled reduction (RED): K-step s also carries RV 16-byte vectors
    // per thread of this workgroup's slice of red_x -- vector rv0 + s * RTH *
    // RV + u * RTH + thread, u < RV -- as direct-to-LDS loads issued with the
    // step's operand loads into a ring of NS areas after the operand stages,
    // so they arrive with the stage and are waited for by the same counts.
    // A vector past the slice loads a valid dummy address (the packed A) and
    // is not added.
    constexpr int RTH = WAVES * 64, RV = RED ? RED_RV : 0, RSTAGE = RTH * RV * 16;
    constexpr int LPWR = LPW + RV;  // loads per wave per K-step
    static_assert(!RED || NS * (STAGE + RSTAGE) <= 160 * 1024, "LDS");
    static_assert(!RED || LPWR * (NS - 2) < 64, "vmcnt range");
    int64_t rv0 = 0, rv1 = 0;
    if constexpr (RED) {
        rv0 = (int64_t)blockIdx.x * g.red_per;
        rv1 = rv0 + g.red_per < g.red_nvec ? rv0 + g.red_per : g.red_nvec;
    }
    auto red_vec = [&](int step, int u) { return rv0 + (int64_t)step * (RTH * RV) + u * RTH + (int)threadIdx.x; };
    auto issue = [&](int step) {
        const int64_t kb = step / HALVES;
        const int h = step % HALVES;
        char *sbase = lds + (step % NS) * STAGE;
#pragma unroll
        for (int c = 0; c < LPW; ++c)
            dma16(src_base[c] + kb * ustride + h * (KBK * 32) + lane * 16, sbase + dst_off[c]);
        if constexpr (RED) {
            char *rbase = lds + NS * STAGE + (step % NS) * RSTAGE;
#pragma unroll
            for (int u = 0; u < RV; ++u) {
                const int64_t v = red_vec(step, u);
                const void *src = v < rv1 ? static_cast<const void *>(g.red_x + 4 * v) : static_cast<const void *>(g.A);
                dma16_nt(src, rbase + (u * RTH + wave * 64) * 16);
            }
        }
    };

    Acc acc[NACC][WBM][WBN];
#pragma unroll
    for (int a = 0; a < NACC; ++a)
#pragma unroll
        for (int i = 0; i < WBM; ++i)
#pragma unroll
            for (int j = 0; j < WBN; ++j) acc[a][i][j] = (Acc)0;

#pragma unroll
    for (int s = 0; s < NS - 1; ++s)
        if (s < nsteps) issue(s);

    if constexpr (LAM == 2) {
        // First-product look-ahead (for tiles whose registers cannot hold
        // two full fragment sets): each iteration waits for the NEXT stage
        // and reads ahead only the two planes of its first product; the
        // current stage's other planes are read at the start of the
        // iteration, behind the matrix instructions of that first product,
        // which need only the fragments read one iteration earlier.
        constexpr int PA0 = prod_p(PL, 0), PB0 = prod_q(PL, 0);
        struct P0 {
            Frag a[WBM], b[WBN];
        };
        const int off = (lane >> 5) * 512 + (lane & 31) * 16;
        auto load_p0 = [&](int step, P0 &F) {
            const char *sA = lds + (step % NS) * STAGE;
            const char *sB = sA + MB * LUNIT;
#pragma unroll
            for (int i = 0; i < WBM; ++i)
                F.a[i] = *reinterpret_cast<const Frag *>(sA + (wm * WBM + i) * LUNIT + PA0 * 32 * KBK + off);
#pragma unroll
            for (int j = 0; j < WBN; ++j)
                F.b[j] = *reinterpret_cast<const Frag *>(sB + (wn * WBN + j) * LUNIT + PB0 * 32 * KBK + off);
        };
        typedef float f4r __attribute__((ext_vector_type(4)));
        f4r racc[RV > 0 ? RV : 1];
        if constexpr (RED) {
#pragma unroll
            for (int u = 0; u < RV; ++u) racc[u] = (f4r)0;
        }
        // this thread's vectors of step s, in LDS since the wait for stage s
        // (each lane reads what its own loads wrote: no barrier involved)
        auto red_add = [&](int step) {
            const char *rbase = lds + NS * STAGE + (step % NS) * RSTAGE;
#pragma unroll
            for (int u = 0; u < RV; ++u)
                if (red_vec(step, u) < rv1)
                    racc[u] += *reinterpret_cast<const f4r *>(rbase + (u * RTH + (int)threadIdx.x) * 16);
        };
        auto pla_step = [&](int step, const P0 &cur, P0 &next) {
            if (step + 1 < nsteps) {
                if (step + NS - 2 <= nsteps - 1)
                    __builtin_amdgcn_s_waitcnt(vmcnt_imm<LPWR * (NS - 3)>());
                else
                    __builtin_amdgcn_s_waitcnt(vmcnt_imm<0>());
                asm volatile("" ::: "memory");
                __builtin_amdgcn_s_barrier();
                asm volatile("" ::: "memory");
                if (step + NS - 1 < nsteps) issue(step + NS - 1);
            }
            if constexpr (RED) red_add(step);  // stage `step` arrived before the previous wait
            // the other planes of this stage (intact until the next
            // iteration's refill), B before A and in the order the products
            // need them, so that each product waits only for its own reads
            const char *sA = lds + (step % NS) * STAGE;
            const char *sB = sA + MB * LUNIT;
            Frag fa[NPL][WBM], fb[NPL][WBN];
#pragma unroll
            for (int i = 0; i < WBM; ++i) fa[PA0][i] = cur.a[i];
#pragma unroll
            for (int j = 0; j < WBN; ++j) fb[PB0][j] = cur.b[j];
#pragma unroll
            for (int t = 1; t < NPROD; ++t) {
                if (first_use_b(PL, t)) {
#pragma unroll
                    for (int j = 0; j < WBN; ++j)
                        fb[prod_q(PL, t)][j] = *reinterpret_cast<const Frag *>(
                            sB + (wn * WBN + j) * LUNIT + prod_q(PL, t) * 32 * KBK + off);
                }
                if (first_use_a(PL, t)) {
#pragma unroll
                    for (int i = 0; i < WBM; ++i)
                        fa[prod_p(PL, t)][i] = *reinterpret_cast<const Frag *>(
                            sA + (wm * WBM + i) * LUNIT + prod_p(PL, t) * 32 * KBK + off);
                }
            }
            // Unconditional, so that reads and matrix instructions form one
            // block the scheduler can interleave: after the last step it
            // reads a stage no load is writing, and the values go unused.
            load_p0(step + 1, next);
#pragma unroll
            for (int t = 0; t < NPROD; ++t)
#pragma unroll
                for (int i = 0; i < WBM; ++i)
#pragma unroll
                    for (int j = 0; j < WBN; ++j)
                        acc[prod_acc(PL, t)][i][j] =
                            M::run(fa[prod_p(PL, t)][i], fb[prod_q(PL, t)][j], acc[prod_acc(PL, t)][i][j]);
            // Order: this stage's reads; product 0 (registers only); the
            // other products with the next stage's first-product reads spread
            // between their matrix instructions.
            constexpr int NCUR = later_reads(PL, NPROD, WBM, WBN), NNEXT = WBM + WBN;
            constexpr int NREST = (NPROD - 1) * WBM * WBN, PER = NREST / NNEXT;
            __builtin_amdgcn_sched_group_barrier(0x100, NCUR, 0);
            __builtin_amdgcn_sched_group_barrier(0x008, WBM * WBN, 0);
#pragma unroll
            for (int r = 0; r < NNEXT; ++r) {
                __builtin_amdgcn_sched_group_barrier(0x008, PER, 0);
                __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
            }
            __builtin_amdgcn_sched_group_barrier(0x008, NREST - PER * NNEXT, 0);
        };
        if (nsteps > 0) {
            if (NS - 2 <= nsteps - 1)
                __builtin_amdgcn_s_waitcnt(vmcnt_imm<LPWR * (NS - 2)>());
            else
                __builtin_amdgcn_s_waitcnt(vmcnt_imm<0>());
            asm volatile("" ::: "memory");
            __builtin_amdgcn_s_barrier();
            asm volatile("" ::: "memory");
            P0 F0, F1;
            load_p0(0, F0);
            int step = 0;
            for (; step + 1 < nsteps; step += 2) {
                pla_step(step, F0, F1);
                pla_step(step + 1, F1, F0);
            }
            if (step < nsteps) pla_step(step, F0, F1);
        }
        if constexpr (RED) {
            // what the K loop left of the slice, the tail floats, then this
            // workgroup's sum in a fixed order (lanes, wavefronts)
            const f4r *rx = reinterpret_cast<const f4r *>(g.red_x);
            for (int64_t idx = rv0 + (int64_t)nsteps * (RTH * RV) + threadIdx.x; idx < rv1; idx += RTH)
                racc[0] += __builtin_nontemporal_load(rx + idx);
            float rs = 0.0f;
#pragma unroll
            for (int u = 0; u < RV; ++u) rs += (racc[u].x + racc[u].y) + (racc[u].z + racc[u].w);
            if (blockIdx.x == 0 && (int)threadIdx.x < g.red_ntail) rs += g.red_x[g.red_nvec * 4 + threadIdx.x];
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) rs += __shfl_xor(rs, o, 64);
            __shared__ float red_w[WAVES];
            if (lane == 0) red_w[wave] = rs;
            __syncthreads();
            if (threadIdx.x == 0) {
                float t = 0.0f;
#pragma unroll
                for (int w = 0; w < WAVES; ++w) t += red_w[w];
                g.red_part[blockIdx.x] = __float_as_uint(t);
            }
        }
    } else if constexpr (LAM == 1) {
        struct FragSet {
            Frag a[SUB][NPL][WBM], b[SUB][NPL][WBN];
        };
        auto load_frags = [&](int step, FragSet &F) {
            const char *sA = lds + (step % NS) * STAGE;
            const char *sB = sA + MB * LUNIT;
#pragma unroll
            for (int s = 0; s < SUB; ++s) {
                const int off = (2 * s + (lane >> 5)) * 512 + (lane & 31) * 16;
#pragma unroll
                for (int p = 0; p < NPL; ++p) {
#pragma unroll
                    for (int i = 0; i < WBM; ++i)
                        F.a[s][p][i] = *reinterpret_cast<const Frag *>(sA + (wm * WBM + i) * LUNIT + p * 32 * KBK + off);
#pragma unroll
                    for (int j = 0; j < WBN; ++j)
                        F.b[s][p][j] = *reinterpret_cast<const Frag *>(sB + (wn * WBN + j) * LUNIT + p * 32 * KBK + off);
                }
            }
        };
        auto compute = [&](const FragSet &F) {
#pragma unroll
            for (int s = 0; s < SUB; ++s)
#pragma unroll
                for (int t = 0; t < NPROD; ++t)
#pragma unroll
                    for (int i = 0; i < WBM; ++i)
#pragma unroll
                        for (int j = 0; j < WBN; ++j)
                            acc[prod_acc(PL, t)][i][j] = M::run(F.a[s][prod_p(PL, t)][i], F.b[s][prod_q(PL, t)][j],
                                                                acc[prod_acc(PL, t)][i][j]);
        };
        // one iteration: make stage step+1 visible, refill the ring, read
        // stage step+1 into `next`, then compute stage `step` from `cur`
        auto la_step = [&](int step, const FragSet &cur, FragSet &next) {
            if (step + 1 < nsteps) {
                // younger than step+1 and issued: NS-3 stages, fewer at the tail
                if (step + NS - 2 <= nsteps - 1)
                    __builtin_amdgcn_s_waitcnt(vmcnt_imm<LPW * (NS - 3)>());
                else
                    __builtin_amdgcn_s_waitcnt(vmcnt_imm<0>());
                asm volatile("" ::: "memory");
                __builtin_amdgcn_s_barrier();
                asm volatile("" ::: "memory");
                if (step + NS - 1 < nsteps) issue(step + NS - 1);
            }
            // reads of the next stage (a stale but in-bounds stage at the end)
            // spread between the matrix instructions: 1 LDS read per 4 MFMA
            load_frags(step + 1 < nsteps ? step + 1 : step, next);
            compute(cur);
            constexpr int NREAD = SUB * NPL * (WBM + WBN);
            constexpr int NMFMA = SUB * NPROD * WBM * WBN;
#pragma unroll
            for (int q = 0; q < NREAD; ++q) {
                __builtin_amdgcn_sched_group_barrier(0x008, NMFMA / NREAD, 0);
                __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
            }
        };
        if (nsteps > 0) {
            if (NS - 2 <= nsteps - 1)
                __builtin_amdgcn_s_waitcnt(vmcnt_imm<LPW * (NS - 2)>());
            else
                __builtin_amdgcn_s_waitcnt(vmcnt_imm<0>());
            asm volatile("" ::: "memory");
            __builtin_amdgcn_s_barrier();
            asm volatile("" ::: "memory");
            FragSet F0, F1;
            load_frags(0, F0);
            int step = 0;
            for (; step + 1 < nsteps; step += 2) {
                la_step(step, F0, F1);
                la_step(step + 1, F1, F0);
            }
            if (step < nsteps) compute(F0);  // odd step count: the last stage is in F0
        }
    } else
    for (int step = 0; step < nsteps; ++step) {
        // stage `step` has landed once at most (younger stages issued) x LPW loads are outstanding
        if (step + NS - 2 < nsteps)
            __builtin_amdgcn_s_waitcnt(vmcnt_imm<LPW * (NS - 2)>());
        else
            __builtin_amdgcn_s_waitcnt(vmcnt_imm<0>());
        asm volatile("" ::: "memory");
        __builtin_amdgcn_s_barrier();
        asm volatile("" ::: "memory");
        if (step + NS - 1 < nsteps) issue(step + NS - 1);
        const char *sA = lds + (step % NS) * STAGE;
        const char *sB = sA + MB * LUNIT;
#pragma unroll
        for (int s = 0; s < SUB; ++s) {
            const int off = (2 * s + (lane >> 5)) * 512 + (lane & 31) * 16;
            Frag fa[NPL][WBM], fb[NPL][WBN];
#pragma unroll
            for (int p = 0; p < NPL; ++p) {
#pragma unroll
                for (int i = 0; i < WBM; ++i)
                    fa[p][i] = *reinterpret_cast<const Frag *>(sA + (wm * WBM + i) * LUNIT + p * 32 * KBK + off);
#pragma unroll
                for (int j = 0; j < WBN; ++j)
                    fb[p][j] = *reinterpret_cast<const Frag *>(sB + (wn * WBN + j) * LUNIT + p * 32 * KBK + off);
            }
#pragma unroll
            for (int t = 0; t < NPROD; ++t) {
#pragma unroll
                for (int i = 0; i < WBM; ++i)
#pragma unroll
                    for (int j = 0; j < WBN; ++j)
                        acc[prod_acc(PL, t)][i][j] =
                            M::run(fa[prod_p(PL, t)][i], fb[prod_q(PL, t)][j], acc[prod_acc(PL, t)][i][j]);
            }
        }
    }

    // Split K: store this part's sums (register-major: word r*64 + lane of
    // block (wave, i, j)), and let the last part to finish add all parts in
    // part order; the other parts are done.  The last part reads every
    // part's words back, its own included (the same bits it stored), QG
    // parts of a block per round of loads (the rounds, not the bytes, set
    // the time of this step: one memory round trip each); QG (4, 2 or 1) is
    // as large as the registers allow without lowering the tile's occupancy.
    if (NACC == 1 && g.ksplit > 1) {
        __shared__ int last_part;
        constexpr int BLOCKS = WAVES * WBM * WBN;
        constexpr int QG = WBM * WBN >= 8 ? 4 : WBM * WBN >= 4 ? 2 : 1;
        const int64_t tiles = (int64_t)g.tiles_m * g.tiles_n;
        uint32_t *mine = static_cast<uint32_t *>(g.partials) + ((int64_t)g.split * tiles + g.tile) * (BLOCKS * 1024);
#pragma unroll
        for (int i = 0; i < WBM; ++i)
#pragma unroll
            for (int j = 0; j < WBN; ++j) {
                uint32_t *blk = mine + ((wave * WBM + i) * WBN + j) * 1024;
#pragma unroll
                for (int r = 0; r < 16; ++r)
                    __hip_atomic_store(blk + r * 64 + lane, word_of(acc[0][i][j][r]), __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
            }
        // Device-scope stores go through to the level all XCDs share, and
        // count as done only once they are there: waiting for them (before
        // the barrier, so for every wavefront) orders them before the
        // ticket, with no fence.  A device-scope fence would also write back
        // this XCD's whole L2 (every other tile's dirty lines) and, on the
        // reading side, invalidate it: measured, those two fences cost more
        // than the parts' matrix work on a 512 x 4096 x 4096 product.  The
        // last part reads the partials with device-scope loads, which go to
        // that shared level too.
        asm volatile("" ::: "memory");
        __builtin_amdgcn_s_waitcnt(vmcnt_imm<0>());
        asm volatile("" ::: "memory");
        __syncthreads();
        if (threadIdx.x == 0) last_part = atomicAdd(g.tickets + g.tile, 1u) == (uint32_t)(g.ksplit - 1);
        __syncthreads();
        if (!last_part) return;
#pragma unroll
        for (int i = 0; i < WBM; ++i)
#pragma unroll
            for (int j = 0; j < WBN; ++j) {
                const uint32_t *blk0 = static_cast<const uint32_t *>(g.partials) +
                                       (int64_t)g.tile * (BLOCKS * 1024) + ((wave * WBM + i) * WBN + j) * 1024 + lane;
                // float: ((0 + part 0) + part 1) + ...; int: the same modulo 2^32
                float fs[16];
                uint32_t us[16];
#pragma unroll
                for (int r = 0; r < 16; ++r) fs[r] = 0.0f, us[r] = 0u;
                for (int q0 = 0; q0 < g.ksplit; q0 += QG) {
                    uint32_t w[QG][16];
#pragma unroll
                    for (int d = 0; d < QG; ++d) {
                        // a part past the last re-reads the last one, unused
                        const int q = q0 + d < g.ksplit ? q0 + d : g.ksplit - 1;
                        const uint32_t *blk = blk0 + (int64_t)q * tiles * (BLOCKS * 1024);
#pragma unroll
                        for (int r = 0; r < 16; ++r)
                            w[d][r] = __hip_atomic_load(blk + r * 64, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    }
#pragma unroll
                    for (int d = 0; d < QG; ++d) {
                        if (q0 + d >= g.ksplit) break;
#pragma unroll
                        for (int r = 0; r < 16; ++r) {
                            if (INT8)
                                us[r] += w[d][r];
                            else
                                fs[r] += __builtin_bit_cast(float, w[d][r]);
                        }
                    }
                }
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    if constexpr (INT8)
                        acc[0][i][j][r] = (int)us[r];
                    else
                        acc[0][i][j][r] = fs[r];
                }
            }
        if (threadIdx.x == 0) __hip_atomic_store(g.tickets + g.tile, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }

    // Epilogue.  32x32 accumulator layout: register r of lane l holds
    // row (r/4)*8 + (l/32)*4 + r%4, column l%32 of the block.
#pragma unroll
    for (int i = 0; i < WBM; ++i)
#pragma unroll
        for (int j = 0; j < WBN; ++j) {
            const int64_t col = ((int64_t)tn * NB + wn * WBN + j) * 32 + (lane & 31);
            const int64_t rowb = ((int64_t)tm * MB + wm * WBM + i) * 32 + (lane >> 5) * 4;
            if (col >= g.N) continue;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int64_t row = rowb + (r >> 2) * 8 + (r & 3);
                if (row >= g.M) continue;
                if (INT8) {
                    uint32_t v = 0;
#pragma unroll
                    for (int a = 0; a < NACC; ++a) v += (uint32_t)acc[a][i][j][r] << (8 * a);
                    static_cast<int32_t *>(g.C)[row * g.ldc + col] = (int32_t)v;
                } else {
                    float *cp = static_cast<float *>(g.C) + row * g.ldc + col;
                    const float v = (float)acc[0][i][j][r];
                    *cp = g.accumulate ? *cp + v : v;
                }
            }
        }
}

// 32-bit integer hash (timing operands, probe positions): the published
// xorshift-multiply "lowbias32" mixer (two multiply rounds, shifts 16, 15,
// 16).
__device__ inline uint32_t hash32(uint32_t x)
{
    x ^= x >> 16;
    x *= 0x7feb352dU;
    x ^= x >> 15;
    x *= 0x846ca68bU;
    x ^= x >> 16;
    return x;
}

// ---------------------------------------------------------- float64 probe --

constexpr int PS = PROBE_SIDE;       // sampled rows (and columns) per tile
constexpr int PROBE_PK = 1024;       // K elements per pass, at most
constexpr int PROBE_PKS = PROBE_PK + 4;  // LDS row stride (floats): rows fall in different banks
constexpr int PROBE_NW = 8;          // wavefronts of a probing workgroup, at most (one partial sum each)

// The k-th of PS consecutive positions in [0, extent), starting at a hashed
// multiple of PS (salt 0: rows, 1: columns), drawn per tile; clamped at a
// ragged edge.  (Drawn per tile, not per tile row or column: with shared
// picks every tile of a row would rest on the same sampled rows, so that one
// unrepresentative sample would pass or mark the whole row together.)  PS
// consecutive rows of a packed operand share each 128-byte line of a 16-byte
// K chunk (rows are 16 bytes apart in a unit), so the probe reads whole
// lines; rows spread over the tile would use 16 bytes of each.
__device__ inline int probe_pick(int64_t key, int k, int extent, int salt)
{
    const int blocks = (extent + PS - 1) / PS;
    const int b = (int)(hash32((uint32_t)(key * 2 + salt) * 2654435761u + 977u) % (uint32_t)blocks);
    const int v = b * PS + k;
    return v < extent ? v : extent - 1;
}

struct ProbeLds {
    float xs[2][PS][PROBE_PKS];   // [A / B^T][sample row][k in pass], exact float32
    double part[PROBE_NW][PS * PS];
    int marked;
};

// The float64 error probe of one output tile (tile index `tile` = tm *
// tiles_n + tn, bm x bn) of a cheap-pass result C (m x n, leading dimension
// ldc), by a workgroup of THREADS threads (64 to 512, a multiple of 64).  It
// takes PS consecutive rows and PS consecutive columns of the tile (hashed
// block positions), computes the PS x PS dot products in float64 from the
// exact operands (each float32 x float32 product is exact in float64),
// compares them with C, and marks the tile for correction when the sampled
// relative Frobenius error exceeds sqrt(tau2) (or the samples are all zero
// but C is not).  C must be visible to the workgroup.  Returns the decision
// in every thread; rec (nullable) receives the record.
//
// K runs in passes of PK = 2 THREADS elements: the workgroup first rebuilds
// the PS rows of A and PS rows of B^T for the pass as exact float32 in LDS
// (each thread loads four 16-byte chunks of the three planes; eight
// neighbouring lanes read one 128-byte line).  Then each thread takes 4
// consecutive K elements of the pass and half of the samples (sample rows
// 0-3 in lanes 0-31 of a wavefront, 4-7 in lanes 32-63; every sample
// column): it converts its 4 + 8 row segments to float64 once and adds the
// 32 x 4 products, in K order, to 32 float64 accumulators that it carries
// over the passes (register blocking: a product costs three eighths of a
// conversion and 1.5 bytes of LDS reads, against two and 8 for one
// accumulator per sample).  At the end a butterfly over each
// half-wavefront leaves lane l with its wavefront's sum for sample l (at
// each of five steps a lane keeps half of its sums and adds its partner's
// matching half), and the wavefront sums are added in wavefront order.  The
// order of the additions is fixed for a given THREADS.  A pass stages and
// sums only the 8-element chunks that hold elements below k (the rest of a
// pass would add exact zero products, which change no sum but the sign of a
// zero one, and no decision).  The raw plane words of the next pass are
// loaded while this pass is staged and summed (double buffering in
// registers); the barriers are raw s_barrier after an LDS-only wait, since a
// full workgroup fence would also wait for those loads.
template <int THREADS>
__device__ __attribute__((always_inline)) inline bool probe_tile(const char *__restrict__ pa,
                                                                 const char *__restrict__ pb,
                                                                 const float *__restrict__ C, int64_t m, int64_t n,
                                                                 int64_t k, int64_t ldc, int bm, int bn, int64_t tile,
                                                                 int tm, int tn, int64_t nkb, double tau2,
                                                                 ProbeRecord *__restrict__ rec, ProbeLds &L)
{
    constexpr int WAVES = THREADS / 64;
    constexpr int PK = 2 * THREADS;                   // K elements per pass (at most PROBE_PK)
    constexpr int CH = PK / 8;                        // 16-byte chunks per row per pass
    constexpr int PER = 2 * PS * CH / THREADS;        // 16-byte chunks per thread per pass
    constexpr int HS = PS * PS / 2;                   // samples per thread (half of them)
    static_assert(PS * PS == 64 && PS == 8, "8 x 8 samples, one per lane");
    static_assert(THREADS % 64 == 0 && WAVES <= PROBE_NW && PK <= PROBE_PK && PER == 4, "thread count");
    constexpr int LGKM0 = 0xF | (7 << 4) | (3 << 14);  // s_waitcnt lgkmcnt(0)
    const int64_t row0 = (int64_t)tm * bm, col0 = (int64_t)tn * bn;
    const int rext = (int)min<int64_t>(bm, m - row0), cext = (int)min<int64_t>(bn, n - col0);
    const int q = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int uh = q >> 5;                            // sample rows 4 uh .. 4 uh + 3
    const int kg = (wave * 32 + (q & 31)) * 4;        // this thread's K elements kg .. kg + 3 of a pass
    const int64_t kpad = nkb * 32;                    // elements the packed operands hold per row
    double acc[HS];                                   // acc[8 i + v]: sample (4 uh + i, v) = 32 uh + 8 i + v
#pragma unroll
    for (int z = 0; z < HS; ++z) acc[z] = 0.0;
    // chunk j of this thread: operand ab, sample row r, chunk ch of a pass
    const char *src[PER];
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        const int id = threadIdx.x + j * THREADS;
        const int r = id % PS, ab = id / (PS * CH);
        const int64_t rr = ab == 0 ? row0 + probe_pick(tile, r, rext, 0) : col0 + probe_pick(tile, r, cext, 1);
        src[j] = (ab == 0 ? pa : pb) + (rr >> 5) * nkb * (3 * PLANE_BYTES) + (rr & 31) * 16;
    }
    u32x4_t rh[PER], rm[PER], rl[PER];
    auto load = [&](int64_t k0) {
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int ch = ((threadIdx.x + j * THREADS) / PS) % CH;
            const int64_t k8 = k0 + (int64_t)ch * 8;
            const char *c = src[j] + (k8 >> 5) * (3 * PLANE_BYTES) + ((k8 & 31) >> 3) * 512;
            const bool in = k8 < kpad;
            rh[j] = in ? *reinterpret_cast<const u32x4_t *>(c) : u32x4_t{0, 0, 0, 0};
            rm[j] = in ? *reinterpret_cast<const u32x4_t *>(c + PLANE_BYTES) : u32x4_t{0, 0, 0, 0};
            rl[j] = in ? *reinterpret_cast<const u32x4_t *>(c + 2 * PLANE_BYTES) : u32x4_t{0, 0, 0, 0};
        }
    };
    load(0);
    for (int64_t k0 = 0; k0 < k; k0 += PK) {
        const int kk = (int)min<int64_t>(PK, k - k0);  // elements of this pass below k
        const int nch = (kk + 7) / 8;                       // chunks staged and read
        // stage: chunk id -> (operand, chunk in pass, sample row); row fastest;
        // hi + mid + lo of a float32 x is x itself (the two additions are exact)
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int id = threadIdx.x + j * THREADS;
            const int r = id % PS, ch = (id / PS) % CH, ab = id / (PS * CH);
            if (ch >= nch) continue;
            float x[8];
#pragma unroll
            for (int w = 0; w < 4; ++w) {
                x[2 * w] = (__uint_as_float(rh[j][w] << 16) + __uint_as_float(rm[j][w] << 16)) +
                           __uint_as_float(rl[j][w] << 16);
                x[2 * w + 1] = (__uint_as_float(rh[j][w] & 0xffff0000u) + __uint_as_float(rm[j][w] & 0xffff0000u)) +
                               __uint_as_float(rl[j][w] & 0xffff0000u);
            }
            float4 *d = reinterpret_cast<float4 *>(&L.xs[ab][r][ch * 8]);
            d[0] = make_float4(x[0], x[1], x[2], x[3]);
            d[1] = make_float4(x[4], x[5], x[6], x[7]);
        }
        __builtin_amdgcn_s_waitcnt(LGKM0);
        asm volatile("" ::: "memory");
        __builtin_amdgcn_s_barrier();
        asm volatile("" ::: "memory");
        if (k0 + PK < k) load(k0 + PK);
        // this thread's 4 K elements, when their chunk was staged (staged
        // chunks hold zeros past k)
        if (kg < nch * 8) {
            // the A segments in float64 once (16 values), then one B
            // segment at a time: each accumulator adds its 4 products in
            // K order
            double xa[4][4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float4 t4 = *reinterpret_cast<const float4 *>(&L.xs[0][4 * uh + i][kg]);
                xa[i][0] = t4.x, xa[i][1] = t4.y, xa[i][2] = t4.z, xa[i][3] = t4.w;
            }
#pragma unroll
            for (int j = 0; j < PS; ++j) {
                const float4 t4 = *reinterpret_cast<const float4 *>(&L.xs[1][j][kg]);
                const double xb[4] = {t4.x, t4.y, t4.z, t4.w};
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int e = 0; e < 4; ++e) acc[PS * i + j] = __builtin_fma(xa[i][e], xb[e], acc[PS * i + j]);
            }
        }
        // the next pass overwrites xs: every LDS read above has been consumed
        asm volatile("" ::: "memory");
        __builtin_amdgcn_s_barrier();
        asm volatile("" ::: "memory");
    }
    // butterfly over the half-wavefront: at mask o a lane keeps the half of
    // its c live sums that its lane bit o selects and adds its partner's
    // copy of that half; lane l ends with acc[0] = the wavefront's sum for
    // sample l
#pragma unroll
    for (int o = 16, c = HS; o > 0; o >>= 1, c >>= 1) {
        const bool hi = (q & o) != 0;
#pragma unroll
        for (int z = 0; z < c / 2; ++z) {
            const double keep = hi ? acc[z + c / 2] : acc[z];
            const double send = hi ? acc[z] : acc[z + c / 2];
            acc[z] = keep + __shfl_xor(send, o, 64);
        }
    }
    L.part[wave][q] = acc[0];
    __syncthreads();
    // wavefront 0, one sample per lane: compare, then sum the squares over
    // the wavefront (a fixed butterfly: every lane ends with the same sums)
    if (threadIdx.x < 64) {
        const int u = q / PS, v = q % PS;
        const int64_t row = row0 + probe_pick(tile, u, rext, 0), col = col0 + probe_pick(tile, v, cext, 1);
        double ref = L.part[0][q];
#pragma unroll
        for (int w = 1; w < WAVES; ++w) ref += L.part[w][q];
        const double c = (double)C[row * ldc + col];
        double e2 = (c - ref) * (c - ref), r2 = ref * ref;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            e2 += __shfl_xor(e2, o, 64);
            r2 += __shfl_xor(r2, o, 64);
        }
        const int marked = (r2 > 0.0) ? (e2 > tau2 * r2) : (e2 > 0.0);
        if (rec) {
            rec->ref[q] = ref;
            if (q < PS) {
                rec->rows[q] = (int32_t)(row0 + probe_pick(tile, q, rext, 0));
                rec->cols[q] = (int32_t)(col0 + probe_pick(tile, q, cext, 1));
            }
            if (q == 0) {
                rec->err2 = e2;
                rec->ref2 = r2;
                rec->corrected = marked;
                rec->pad[0] = rec->pad[1] = rec->pad[2] = 0;
            }
        }
        if (q == 0) L.marked = marked;
    }
    __syncthreads();
    return L.marked != 0;
}

}  // namespace dev
}  // namespace accx
