// Internal launch interface between the C-ABI runtime (runtime.cpp) and the
// HIP kernels (*.hip).  Not installed; the public ABI is include/accx.h.
#pragma once

#include <hip/hip_runtime_api.h>
#include <stddef.h>
#include <stdint.h>

namespace accx {

// Shape of one loop nest C (m x n) = A (m x k) B (k x n), row-major, with
// leading dimensions (elements between rows): Listing 1a is
// m = n = k = lda = ldb = ldc = LEN.
struct GemmShape {
    int64_t m, n, k, lda, ldb, ldc;
};
inline GemmShape square_shape(int64_t len) { return GemmShape{len, len, len, len, len, len}; }

// ---- plain loop nest (Listing 1a/1b): one thread per output element -------
hipError_t launch_matmul_plain_f32(const float *a, const float *b, float *c, const GemmShape &sh,
                                   bool listing1b_mapping, hipStream_t s);
hipError_t launch_matmul_plain_i32(const int32_t *a, const int32_t *b, int32_t *c, const GemmShape &sh,
                                   bool listing1b_mapping, hipStream_t s);

// ---- reduction(+) ----------------------------------------------------------
// Fast: a streaming pass that stores one partial per block, then a
// one-block launch that adds them in index order.
// Workspace: 4 bytes per block (<= 4096 blocks), any contents.
size_t reduce_fast_workspace_bytes(int64_t n);
// Plain: one element per thread and a block tree, then one block combines.
size_t reduce_plain_workspace_bytes(int64_t n);

hipError_t launch_reduce_f32(const float *x, int64_t n, float init, float *result, void *work,
                             bool plain, hipStream_t s);
hipError_t launch_reduce_i32(const int32_t *x, int64_t n, int32_t init, int32_t *result, void *work,
                             bool plain, hipStream_t s);
// result = init + the g float partials' (bits) sum, in index order over a
// fixed tree (the fast reduction's second launch).
hipError_t launch_reduce_final_f32(const uint32_t *partials, int g, float init, float *result, hipStream_t s);

// Reduction variables over one array (any operator, element type).
enum { RED_SUM = 0, RED_MAX = 1, RED_MIN = 2, RED_OR = 3, RED_MAX_VARS = 4 };
struct RedVars {
    int32_t nvars;                 // 1..4 (logical or: 1)
    int32_t op[RED_MAX_VARS];      // RED_*
    int32_t square[RED_MAX_VARS];  // 1: the variable folds x*x
    uint64_t init[RED_MAX_VARS];   // initial values as element bit patterns
};
// Workspace: RED_MAX_VARS x 4096 partial words of 8 bytes, any contents.
size_t reduce_vars_workspace_bytes();
// Static device scratch (reduce.hip) for the entry point that allocates
// nothing: NOALLOC_SCRATCH_BYTES per GPU.  noalloc_scratch_setup(device)
// takes the array's device address on `device` (which must be current) once;
// noalloc_scratch(device) returns it, or NULL before the setup.
constexpr size_t NOALLOC_SCRATCH_BYTES = 128 * 1024;
hipError_t noalloc_scratch_setup(int device);
void *noalloc_scratch(int device);
// dtype: 0 float32, 1 int32, 2 float64, 3 int64; result: nvars elements.
hipError_t launch_reduce_vars(int dtype, const void *x, int64_t n, const RedVars &vars, void *result, void *work,
                              hipStream_t s);

// ---- tiled matrix-core path (gemm_mfma.hip) --------------------------------
// Bytes of a packed operand: `rows` rows of `k_elems` elements of
// `elem_bytes` bytes, `planes` planes (units of 32 rows x 64 bytes per plane).
size_t packed_bytes(int64_t rows, int64_t k_elems, int elem_bytes, int planes);
// float32 -> hi/mid/lo bf16 planes.  trans = false: x is rows x k row-major
// (element (r, e) at x[r*ld + e]); trans = true: x is k x rows row-major
// (element (e, r) at x[e*ld + r]; packs the columns, i.e. B^T).
hipError_t launch_pack_bf16x3(const float *x, int64_t rows, int64_t k, int64_t ld, bool trans, void *out,
                              hipStream_t s);
// int32 -> `planes` balanced base-256 digit planes.
hipError_t launch_pack_i8(const int32_t *x, int64_t rows, int64_t k, int64_t ld, bool trans, int planes, void *out,
                          hipStream_t s);
// Both operands of one product in one launch: A (m x k, rows) into pa and B
// (k x n, packed as B^T) into pb, as the two calls above would; for int8,
// maxabs (nullable, int8) gets A's max |x| in word 0 and B's in word 1, as
// 64-bit words (stamp << 32 | max) that need no clearing between calls: each
// call passes a fresh nonzero stamp, and a word with another stamp reads as
// no maximum above 127 recorded.
hipError_t launch_pack_bf16x3_pair(const float *a, int64_t m, int64_t lda, const float *b, int64_t n, int64_t ldb,
                                   int64_t k, void *pa, void *pb, hipStream_t s);
// decide (optional, int8): the two max|x| words of a finished one-digit
// pass with stamp `stamp`; the launch then packs only if more than one digit
// is needed, and writes as many digit planes as are needed into units of
// four planes (`planes` is ignored).
hipError_t launch_pack_i8_pair(const int32_t *a, int64_t m, int64_t lda, const int32_t *b, int64_t n, int64_t ldb,
                               int64_t k, int planes, void *pa, void *pb, uint64_t *maxabs, hipStream_t s,
                               const uint64_t *decide = nullptr, uint32_t stamp = 0);
// C (m x n, leading dimension ldc) = sum over the product set of A-plane x
// B-plane, A and B packed with k elements per row.
// products: 6 = FULL6, 5 = FIVE (FULL6 without mid*mid), 3 = CHEAP3, -3 = the
// three products FULL6 adds to CHEAP3.  accumulate: C += instead of C =.
// tile: one of GEMM_TILE_* (0 = size heuristic).
enum { GEMM_TILE_DEFAULT = 0, GEMM_TILE_256 = 1, GEMM_TILE_256x128 = 2, GEMM_TILE_128 = 3, GEMM_TILE_64 = 4,
       GEMM_TILE_256W4 = 5, GEMM_TILE_COUNT = 6 };
// Per-tile record of the float64 error probe (layout documented in accx.h).
constexpr int PROBE_SIDE = 8;  // sampled rows and columns per tile
struct ProbeRecord {
    int32_t rows[PROBE_SIDE], cols[PROBE_SIDE];  // sampled rows and columns of the tile
    double ref[PROBE_SIDE * PROBE_SIDE];         // float64 dot products, ref[8*u + v] at (rows[u], cols[v])
    double err2, ref2;                           // sum over the samples of (C - ref)^2 and of ref^2
    int32_t corrected;                           // 1 if the tile got the three correction products
    int32_t pad[3];
};
static_assert(sizeof(ProbeRecord) == 608, "probe record layout");

// Split K (short-and-wide results that leave CUs idle): the K loop of each
// output tile runs in `parts` workgroups whose partial sums are added in
// part order by the last to finish.  work: split_k_bytes(...) bytes (tile
// tickets, then partial sums); parts <= 1 = no split.  Ignored for the
// accumulating (C +=) and multi-digit launches.
struct SplitK {
    int parts = 1;
    void *work = nullptr;
};
// The split the library uses for (tile, m, n) with nkb 64-byte K units per
// row, when the output tiles leave at least half the CUs idle: as many parts
// as fill the CUs' workgroup slots (two per CU for the 128 x 128 tile, one
// for the others), at most KSPLIT_MAX.
int split_k_parts(int tile, int64_t m, int64_t n, int64_t nkb);
size_t split_k_bytes(int tile, int64_t m, int64_t n, int parts);

// probe: non-null = skip the tiles whose record has corrected == 0.
// probe_tile: the tile configuration the records were made for (0 = `tile`);
// its tiles must contain whole tiles of this launch.
hipError_t launch_gemm_bf16x3(const void *pa, const void *pb, float *c, const GemmShape &sh, int products,
                              bool accumulate, int tile, hipStream_t s, const ProbeRecord *probe = nullptr,
                              const SplitK &sk = SplitK(), int probe_tile = 0);
// The three-product pass on the 256 x 256 tile (bitwise as
// launch_gemm_bf16x3 with products 3 and that tile, unsplit) that also sums
// the float32 array x[0, n) (16-byte aligned): one partial per workgroup in
// part[0, red_fused_parts(m, n)), for launch_reduce_final_f32.
hipError_t launch_gemm_bf16x3_red(const void *pa, const void *pb, float *c, const GemmShape &sh, const float *x,
                                  int64_t n, uint32_t *part, hipStream_t s);
int red_fused_parts(int64_t m, int64_t n);
// Floats the pass's K loop carries (beyond them, each workgroup adds the rest
// of its slice after the loop, with one load in flight per thread).
int64_t red_fused_capacity(int64_t m, int64_t n, int64_t k);
// The last step of a co-scheduled reduction: *result = init + the `parts`
// float partials (bits) in part[], added in a fixed order.  result NULL: none.
struct RedFinal {
    const uint32_t *part = nullptr;
    int parts = 0;
    float init = 0.0f;
    float *result = nullptr;
};
// Float64 probe of C per output tile of `tile`; tau: relative Frobenius
// threshold above which a tile is marked for correction.  fin: a
// reduction's last step, run by the launch's first workgroup.
hipError_t launch_probe_f64(const void *pa, const void *pb, const float *c, const GemmShape &sh, int tile, double tau,
                            ProbeRecord *rec, hipStream_t s, const RedFinal &fin = RedFinal());
// Output tiles of `tile` (0 = the heuristic's choice) over an m x n result.
int probe_tiles(int tile, int64_t m, int64_t n);
// The configuration the size heuristic picks for an m x n result.
int default_tile(int64_t m, int64_t n);
// float32 -> one plane of float32 elements in the packed layout (16 elements
// per 64-byte unit row), for the float32 matrix cores; trans as above.
hipError_t launch_pack_f32(const float *x, int64_t rows, int64_t k, int64_t ld, bool trans, void *out, hipStream_t s);
hipError_t launch_pack_f32_pair(const float *a, int64_t m, int64_t lda, const float *b, int64_t n, int64_t ldb,
                                int64_t k, void *pa, void *pb, hipStream_t s);
// C = A B on the float32 matrix cores from float32-packed operands.
hipError_t launch_gemm_f32mm(const void *pa, const void *pb, float *c, const GemmShape &sh, int tile, hipStream_t s,
                             const SplitK &sk = SplitK());
// limbs: digits per operand, also the planes per packed unit.  limbs = 1:
// the one-digit kernel on `tile`; limbs >= 2: a persistent kernel on 128 x
// 128 tiles.  decide (optional): the two max|x| words of the one-digit pass;
// the one-digit kernel then runs only if one digit is enough, and the
// multi-digit kernel (limbs = 4 units) only if more are needed, with as many
// digits as are needed.
hipError_t launch_gemm_i8(const void *pa, const void *pb, int32_t *c, const GemmShape &sh, int limbs, int tile,
                          hipStream_t s, const uint64_t *decide = nullptr, uint32_t stamp = 0,
                          const SplitK &sk = SplitK());
// The automatic int32 GEMMs after the one-digit and multi-digit passes: the
// one-digit product on `tile` (pa1, pb1) if one digit is enough, else the
// multi-digit one (pa4, pb4: units of four planes); one launch when the
// one-digit tile is 256 x 256, two otherwise.
hipError_t launch_gemm_i8_auto(const void *pa1, const void *pb1, const void *pa4, const void *pb4, int32_t *c,
                               const GemmShape &sh, int tile, hipStream_t s, const uint64_t *maxabs, uint32_t stamp,
                               const SplitK &sk = SplitK());
hipError_t launch_zero_u32(uint32_t *p, int n, hipStream_t s);

// ---- measurement kernels (onbox.hip) ---------------------------------------
// Matrix instructions only (kind 0: bf16 32x32x16, 1: int8 32x32x32) on
// every CU; *ops = the operations the launch performs.
hipError_t launch_onbox_mfma(int kind, int64_t rounds, double *ops, hipStream_t s);
// Read-only stream of `bytes` (a multiple of 16, 16-byte aligned) at x.
hipError_t launch_onbox_read(const void *x, int64_t bytes, hipStream_t s);
// n pseudo-random 32-bit words for timing runs: float32 in [-1, 1) or int32 in [-16, 16].
hipError_t launch_fill_hash(void *p, int64_t n, bool as_int, hipStream_t s);

// ---- batched launch (batch.hip) -------------------------------------------
struct BatchPackJob {   // one bf16x3 operand to pack
    const float *x;
    char *out;
    int64_t rows, k, ld, nrb, nkb;
    int32_t trans, nwg;    // nwg: the pack launch's workgroups on this operand
    uint32_t wg0, pad;     // the first of them
};
// Workgroups of the pack launch for an operand of nrb 32-row blocks and nkb
// K units: about one 8-element chunk per thread (at most 4096 workgroups).
int batch_pack_workgroups(int64_t nrb, int64_t nkb);
struct BatchMat {       // one matmul: packed operands, output, tiling
    const char *pa, *pb;
    float *c;
    int64_t len, nkb;
    int32_t tile, tiles_m, tiles_n, products;
};
struct BatchRed {       // one reduction: input, chunking, result slot
    const float *x;
    float *result;
    uint32_t *ticket;   // zero before the first launch; left at zero
    uint32_t *partials; // nchunks words
    int64_t n, chunk;
    int32_t nchunks;
    float init;
};
struct BatchUnit {      // item index (top bit set: reduction), tile or chunk
    uint32_t item, sub;
};
struct BatchQueue {
    const BatchMat *mats;
    const BatchRed *reds;
    const BatchUnit *units;
    uint32_t nunits;
    uint32_t *counter, *done;  // zero before the first launch; left at zero
    int32_t auto_prec;         // 1: three products + per-tile float64 probe + correction; 0: six products
    double tau2;               // AUTO: squared relative error bound of the probe
};
int batch_tile_supported(int tile);
int batch_workgroups();
// job_of[w]: the job of pack workgroup w (nwg workgroups in all).
hipError_t launch_batch_pack(const BatchPackJob *jobs, const uint32_t *job_of, int64_t nwg, hipStream_t s);
hipError_t launch_batch_persistent(const BatchQueue &q, hipStream_t s);

int device_cu_count();  // compute units of the current device (cached)

// Kernel timing hooks (runtime.cpp): when timing is enabled, record a HIP
// event on `s` before (begin = true) and after each kernel launch.
void tmark(const char *name, hipStream_t s, bool begin);

}  // namespace accx
