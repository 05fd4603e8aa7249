/*
 * libaccx: the data-parallel hot path of an OpenACC offload region on one
 * AMD Instinct MI355X (gfx950), behind a plain C ABI.
 *
 * Paper: A. Lashgar, A. Majidi, A. Baniasadi, "IPMACC: Open Source OpenACC
 * to CUDA/OpenCL Translator", arXiv 1412.1127.  The calls follow the paper's
 * statement of the problem:
 *
 *   - data directive with copy / copyin / copyout / create clauses over
 *     [start:n] subarrays, and the host-accelerator pointer exchange
 *     (section 1.2 "OpenACC Model", section 1.3 and Listing 1a, and the
 *     data-clause step of section 2.3);
 *   - the `kernels` + `loop independent` matrix-multiplication loop nest of
 *     the worked example, i and j parallel, l sequential (Listing 1a/1b,
 *     section 1.3), for float and int operands;
 *   - the `reduction(+)` clause lowering: a reduction across the threads of
 *     a block, then across blocks (section 2.3, "Replacing the dummy OpenACC
 *     kernels region calls"; SRAD paragraph of section 4.2).
 *
 * Conventions shared by every call:
 *   - Every call returns an acc_status; nothing throws across this ABI.
 *     acc_last_error_string() gives a thread-local message for the last
 *     failing call on the calling thread.
 *   - Element counts are int64_t; element types are 4 bytes (float, int32).
 *   - Matrices are square, row-major, LEN*LEN, element (i, j) at i*LEN + j.
 *   - int32 arithmetic wraps: results are exact modulo 2^32, read as two's
 *     complement.
 *   - float results are computed in float32 arithmetic (or on bf16 matrix
 *     cores with a three-term split, see ACC_PREC_*) and are not bitwise
 *     reproducible across kernels; each kernel is bitwise deterministic
 *     run to run.
 *   - Without a usable GPU every compute or memory call returns
 *     ACC_ERR_NO_DEVICE; there is no host fallback.
 */
#ifndef ACCX_H
#define ACCX_H

#include <stddef.h>
#include <stdint.h>

#if defined(__GNUC__)
#define ACCX_API __attribute__((visibility("default")))
#else
#define ACCX_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    ACC_OK = 0,
    ACC_ERR_INVALID_ARG = -1,     /* bad pointer, size, kind, dtype or flag */
    ACC_ERR_NOT_PRESENT = -2,     /* operand not inside a mapped host range */
    ACC_ERR_ALREADY_PRESENT = -3, /* clause overlaps a mapped host range */
    ACC_ERR_OUT_OF_MEMORY = -4,   /* HBM budget exceeded or allocation failed */
    ACC_ERR_DEVICE = -5,          /* HIP runtime or kernel launch error */
    ACC_ERR_NO_DEVICE = -6,       /* no gfx950 device, or acc_init not called */
    /* not statuses: they make every int32 a value of the type, so that any
     * int a caller passes through the ABI is well defined */
    ACC_STATUS_RANGE_MIN_ = -0x7fffffff - 1,
    ACC_STATUS_RANGE_MAX_ = 0x7fffffff
} acc_status;

/* Data clauses (section 1.3): copy = copy in at region entry and out at exit;
 * copyin = in only; copyout = out only; create = device allocation only.
 * present = the range must already be mapped (by an enclosing region): the
 * region uses that mapping.  present_or_X = present if the range is already
 * mapped, else X.  Mappings are reference counted: every clause of every
 * region that uses a mapping holds one reference, and the mapping is copied
 * out (if its creating clause was copy or copyout) and freed when the last
 * region holding a reference ends, whichever region that is. */
typedef enum {
    ACC_COPY = 0,
    ACC_COPYIN = 1,
    ACC_COPYOUT = 2,
    ACC_CREATE = 3,
    ACC_PRESENT = 4,
    ACC_PRESENT_OR_COPY = 5,
    ACC_PRESENT_OR_COPYIN = 6,
    ACC_PRESENT_OR_COPYOUT = 7,
    ACC_PRESENT_OR_CREATE = 8
} acc_clause_kind;

/* directions of acc_update */
#define ACC_UPDATE_HOST 0   /* device copy -> host (update host / self) */
#define ACC_UPDATE_DEVICE 1 /* host -> device copy (update device) */

/* Element types.  The matmul takes ACC_FLOAT32 and ACC_INT32; data clauses
 * and reductions take all four. */
typedef enum {
    ACC_FLOAT32 = 0,
    ACC_INT32 = 1,
    ACC_FLOAT64 = 2,
    ACC_INT64 = 3,
    /* not element types: they make every int32 a value of the type, so that
     * a caller's invalid dtype is a defined value the library rejects with
     * ACC_ERR_INVALID_ARG */
    ACC_DTYPE_RANGE_MIN_ = -0x7fffffff - 1,
    ACC_DTYPE_RANGE_MAX_ = 0x7fffffff
} acc_dtype;

/* One data clause: host[start : start+n) in elements of `dtype` ("[start:n]
 * means n elements from element start", section 1.3).  `host` is the base of
 * the host array, owned by the caller, alive until acc_data_end. */
typedef struct {
    int32_t kind;  /* acc_clause_kind */
    int32_t dtype; /* acc_dtype */
    void *host;
    int64_t start;
    int64_t n;
} acc_clause;

typedef struct acc_region_s *acc_region; /* opaque */

/* ---- flags for acc_loopnest_matmul / accx_matmul_dev -------------------- */
/* kernel choice (low 4 bits) */
#define ACC_KERNEL_AUTO 0x0u            /* tiled matrix-core kernel */
#define ACC_KERNEL_PLAIN 0x1u           /* one thread per (i,j), j on lanes */
#define ACC_KERNEL_PLAIN_LISTING1B 0x2u /* Listing 1b's mapping: i on x, 16x16 */
#define ACC_KERNEL_TILED 0x3u           /* LDS-tiled matrix-core kernel */
#define ACC_KERNEL_MASK 0xFu
/* float precision on the tiled kernel (bits 4..7); ignored for int32 and the
 * plain kernels.  x = hi + mid + lo, three bf16 terms per operand. */
#define ACC_PREC_AUTO 0x00u   /* cheap split + sampled float64 error probe;
                                 adds the missing products if needed */
#define ACC_PREC_FULL6 0x10u  /* 6 bf16 products: all pairs with p+q <= 2 */
#define ACC_PREC_CHEAP3 0x20u /* 3 bf16 products: pairs with p+q <= 1 */
#define ACC_PREC_FIVE 0x30u   /* 5 bf16 products: FULL6 without mid*mid
                                 (|mid*mid| <= 2^-16 |a||b|) */
#define ACC_PREC_F32MFMA 0x40u /* no split: the float32 operands themselves on the
                                  float32 matrix cores (v_mfma_f32_32x32x2_f32),
                                  float32 accumulation: the plain float32 tiled
                                  kernel the bf16x3 modes are measured against */
#define ACC_PREC_MASK 0xF0u
/* int32 on the tiled kernel: limb count (bits 8..11); 0 = probe max |x|. */
#define ACC_LIMBS_SHIFT 8
#define ACC_LIMBS_MASK 0xF00u
/* asynchronous completion (acc_reduce_sum): *inout valid after acc_wait */
#define ACC_ASYNC 0x1000u
/* tile configuration of the tiled kernel (bits 16..19).  AUTO takes the
 * autotuner's choice for the size class (see accx_autotune), else a size
 * heuristic; the others force one configuration. */
#define ACC_TILE_SHIFT 16
#define ACC_TILE_MASK 0xF0000u
#define ACC_TILE_AUTO 0x00000u
#define ACC_TILE_256 0x10000u     /* 256 x 256 output tile, 8 wavefronts */
#define ACC_TILE_256x128 0x20000u /* 256 x 128, 4 wavefronts, 2 workgroups/CU */
#define ACC_TILE_128 0x30000u     /* 128 x 128, 4 wavefronts */
#define ACC_TILE_64 0x40000u      /* 64 x 64, 4 wavefronts */
#define ACC_TILE_256W4 0x50000u   /* 256 x 256 output tile, 4 wavefronts */

/* ---- flags for acc_reduce_sum / accx_reduce_sum_dev --------------------- */
#define ACC_REDUCE_FAST 0x0u  /* streaming pass (grid-stride 16-byte loads, one partial
                                 per workgroup), then a one-workgroup launch that
                                 adds the partials in index order */
#define ACC_REDUCE_PLAIN 0x1u /* one element per thread + block tree, then a
                                 second one-block launch over the partials */

/* ---- library ------------------------------------------------------------ */

/* Select `device` (HIP ordinal) and set the HBM budget for region data and
 * library workspaces (0 = no budget beyond the device).  Must precede every
 * other call but the string and version calls.  May be called again after
 * acc_shutdown.  Errors: NO_DEVICE, INVALID_ARG (device < 0). */
ACCX_API acc_status acc_init(int device, uint64_t hbm_budget_bytes);

/* Free every region still open (no copyout) and all library memory. */
ACCX_API acc_status acc_shutdown(void);

/* Bytes currently charged against the budget (region arrays + workspaces). */
ACCX_API acc_status acc_budget_used(uint64_t *bytes_out);

/* Memory allocation, the third of the data functions that replace the data
 * clauses (section 2.3, data-clause step: pointer exchange, copy in/out and
 * memory allocation), taken from the caller: every device allocation the
 * library makes (region arrays, library-owned workspaces, autotuner scratch,
 * batch and serving memory) calls alloc(bytes, ctx) instead of hipMalloc,
 * and frees with free_(ptr, ctx).  alloc returns device memory of the current
 * device, aligned to 256 bytes, or NULL (the call then fails with
 * OUT_OF_MEMORY).  The library frees a block only after the work that uses it
 * has finished on the device.  Both NULL: back to hipMalloc / hipFree.  A
 * block always goes back to the allocator that gave it, also after a later
 * change.  The callbacks run on the thread of the library call that needs
 * them, under the library's lock: they must not call into the library.
 * Errors: INVALID_ARG (one of the two NULL). */
ACCX_API acc_status accx_set_allocator(void *(*alloc)(size_t bytes, void *ctx), void (*free_)(void *ptr, void *ctx),
                                       void *ctx);

/* ---- data regions (section 1.3, data-clause step of section 2.3) -------- */

/* Open a data region: allocate a device copy of each clause's host range and,
 * for copy and copyin, copy it host->device on the region's stream.
 * `hip_stream` = NULL: the region creates its own stream; otherwise the
 * caller's hipStream_t, which must outlive the region.  Clause ranges must
 * not overlap one another or any mapped range (ALREADY_PRESENT).  n = 0 is
 * allowed and maps nothing.  On any error nothing stays mapped.
 * Errors: INVALID_ARG, ALREADY_PRESENT, OUT_OF_MEMORY, DEVICE, NO_DEVICE. */
ACCX_API acc_status acc_data_begin(const acc_clause *clauses, int nclauses, void *hip_stream,
                          acc_region *region_out);

/* Close a region: wait for its stream, copy device->host for copy and
 * copyout, free its device memory and unmap its ranges.  Always frees, also
 * after an error; returns the first error the region met. */
ACCX_API acc_status acc_data_end(acc_region region);

/* Block until all work enqueued on the region has finished. */
ACCX_API acc_status acc_wait(acc_region region);

/* The update directive: copy host[start : start+n) (elements of dtype t)
 * between the host and its device copy, which must lie in one mapped range
 * of dtype t.  Enqueued on the region's stream, in order with its kernels
 * (the region's stream is its async queue); synchronous unless ACC_ASYNC,
 * then complete by acc_wait / acc_data_end.
 * Errors: INVALID_ARG, NOT_PRESENT, DEVICE. */
ACCX_API acc_status acc_update(acc_region region, int direction, acc_dtype t, void *host, int64_t start, int64_t n,
                               uint32_t flags);

/* *present_out = 1 if host[0 : bytes) lies inside one mapped range, else 0. */
ACCX_API acc_status acc_is_present(const void *host, size_t bytes, int *present_out);

/* Page-locked host memory (hipHostMalloc) for region arrays: copies from and
 * to it run asynchronously on the region's stream, so the transfers of one
 * region overlap the kernels of another.  Free with accx_host_free.
 * Errors: INVALID_ARG, OUT_OF_MEMORY, NO_DEVICE. */
ACCX_API acc_status accx_host_alloc(size_t bytes, void **host_out);
ACCX_API acc_status accx_host_free(void *host);

/* Host-accelerator pointer exchange (section 2.3): the device address of the
 * mapped host address `host`.  Errors: NOT_PRESENT. */
ACCX_API acc_status acc_deviceptr(const void *host, void **device_out);

/* ---- the loop nest (Listing 1a, section 1.3) ---------------------------- */

/* c[i*len+j] = sum over l of a[i*len+l] * b[l*len+j], for 0 <= i, j < len:
 * i and j parallel, l sequential.  a, b, c are HOST addresses, each of whose
 * len*len elements must lie inside one mapped range of dtype `t` (the kernel
 * reads and writes the device copies; host c changes at acc_data_end, for
 * copy/copyout).  Enqueued on the region's stream.  1 <= len <= 65536.
 * Errors: INVALID_ARG, NOT_PRESENT, OUT_OF_MEMORY (workspace), DEVICE. */
ACCX_API acc_status acc_loopnest_matmul(acc_region region, acc_dtype t, const void *a, const void *b,
                               void *c, int64_t len, uint32_t flags);

/* The same nest on rectangular operands with leading dimensions (section
 * 1.3's loop nest with the trip counts and row strides as parameters; the
 * output-parallel form of section 4.2's Matrix Multiplication paragraph):
 *   c[i*ldc + j] = sum over l < k of a[i*lda + l] * b[l*ldb + j],
 *   0 <= i < m, 0 <= j < n.
 * Row-major A (m x k), B (k x n), C (m x n); a, b, c are HOST addresses and
 * the span of each view (from its first to its last element) must lie in one
 * mapped range of dtype `t`; c's span must not overlap a's or b's.
 * 0 <= m, n <= 131072; 0 <= k <= 65536; lda >= max(1, k), ldb >= max(1, n),
 * ldc >= max(1, n), each at most 2^31.  m = 0 or n = 0 does nothing; k = 0
 * sets C to zero.  Same flags and results as acc_loopnest_matmul, which is
 * the case m = n = k = lda = ldb = ldc = len.
 * Errors: INVALID_ARG, NOT_PRESENT, OUT_OF_MEMORY (workspace), DEVICE. */
ACCX_API acc_status acc_loopnest_gemm(acc_region region, acc_dtype t, int64_t m, int64_t n, int64_t k, const void *a,
                                      int64_t lda, const void *b, int64_t ldb, void *c, int64_t ldc, uint32_t flags);

/* ---- reduction(+) (section 2.3; SRAD paragraph of section 4.2) ---------- */

/* *inout = *inout + sum of x[0..n), x a HOST address whose n elements lie in
 * one mapped range of dtype `t`; *inout is a host value of type t (float32
 * and int32 run the dedicated sum kernels; float64 and int64 the general
 * ones of acc_reduce).  n = 0 leaves *inout unchanged.  Synchronous unless ACC_ASYNC, then *inout is
 * written by the time acc_wait / acc_data_end returns.
 * Errors: INVALID_ARG, NOT_PRESENT, DEVICE. */
ACCX_API acc_status acc_reduce_sum(acc_region region, acc_dtype t, const void *x, int64_t n,
                          void *inout_result, uint32_t flags);

/* ---- reduction variables: operators, types, several per loop ------------
 * The reduction clause with the operators +, max, min and logical or
 * (section 2.3's reduction lowering; the BFS paragraph of section 4.2 names a
 * boolean "more nodes" flag, the SRAD paragraph a loop with two sum
 * variables).  Variable v of a loop over x[0..n):
 *   result_v = init_v (op) f(x[0]) (op) f(x[1]) ... , f(x) = x, or x*x when
 *   `square` is 1 (the square in the element type, as `v += t*t` computes it).
 * +: float32 and float64 add in their own type (any order: the result is
 * within rounding of the exact sum, and bitwise the same on every run);
 * int32 and int64 wrap around.  max / min: exact; a NaN element is ignored
 * (fmax / fmin).  Logical or: result = 1 if init or any element is nonzero,
 * else 0 (a variable of its own, not squared), computed as a guarded write
 * (every thread that sees a nonzero element stores 1) instead of a tree.
 * Up to ACC_MAX_REDUCE_VARS variables over the same array share one pass. */
typedef enum { ACC_RED_SUM = 0, ACC_RED_MAX = 1, ACC_RED_MIN = 2, ACC_RED_OR = 3 } acc_reduce_op;
#define ACC_MAX_REDUCE_VARS 4
typedef struct {
    int32_t op;     /* acc_reduce_op */
    int32_t square; /* 0: fold x; 1: fold x*x */
} acc_reduce_var;

/* inout: nvars HOST values of type t (initial values in, results out), x a
 * HOST address whose n elements lie in one mapped range of dtype t.  n = 0
 * leaves every value unchanged (logical or: normalised to 0 or 1).
 * Synchronous unless ACC_ASYNC, as acc_reduce_sum; ACC_REDUCE_PLAIN only for
 * one float32 / int32 sum.  Errors: INVALID_ARG, NOT_PRESENT, DEVICE. */
ACCX_API acc_status acc_reduce(acc_region region, acc_dtype t, const void *x, int64_t n, const acc_reduce_var *vars,
                               int nvars, void *inout, uint32_t flags);

/* ---- device-pointer entries (memory owned by the caller, e.g. torch) ----- */

/* Workspace bytes accx_matmul_dev needs for (t, len, flags); 0 for the plain
 * kernels.  The size depends on the tile the call will use (the autotuned
 * table, else the size heuristic): when the output tiles leave more than
 * half of the CUs idle, the K loop of each tile is split over up to eight
 * workgroups whose partial sums (a split area at the end of the workspace)
 * are added in a fixed part order by the last to finish.  A workspace that
 * holds the packed operands but not the split area still works: the call
 * then runs unsplit.  Errors: INVALID_ARG. */
ACCX_API acc_status accx_matmul_workspace_size(acc_dtype t, int64_t len, uint32_t flags, size_t *bytes_out);

/* The loop nest on device pointers dA, dB, dC (len*len elements each, 4-byte
 * aligned, dC not overlapping dA or dB), enqueued on `hip_stream` (NULL = the
 * null stream).  dWork: device workspace of at least the size above,
 * 256-byte aligned (as hipMalloc and torch allocations are), or NULL to use
 * a library-owned workspace of that stream (grown on demand).
 * Errors: INVALID_ARG, OUT_OF_MEMORY, DEVICE, NO_DEVICE. */
ACCX_API acc_status accx_matmul_dev(acc_dtype t, const void *dA, const void *dB, void *dC, int64_t len,
                           uint32_t flags, void *dWork, size_t work_bytes, void *hip_stream);

/* Workspace bytes accx_gemm_dev needs for (t, m, n, k, flags); does not
 * depend on the leading dimensions.  0 for the plain kernels and for m = 0
 * or n = 0.  Errors: INVALID_ARG. */
ACCX_API acc_status accx_gemm_workspace_size(acc_dtype t, int64_t m, int64_t n, int64_t k, uint32_t flags,
                                             size_t *bytes_out);

/* acc_loopnest_gemm's nest on device pointers (4-byte aligned; dA and dB may
 * be NULL when k = 0; dC's span must not overlap dA's or dB's), enqueued on
 * `hip_stream` (NULL = the null stream); dWork as for accx_matmul_dev.
 * Shape limits and results as acc_loopnest_gemm.
 * Errors: INVALID_ARG, OUT_OF_MEMORY, DEVICE, NO_DEVICE. */
ACCX_API acc_status accx_gemm_dev(acc_dtype t, int64_t m, int64_t n, int64_t k, const void *dA, int64_t lda,
                                  const void *dB, int64_t ldb, void *dC, int64_t ldc, uint32_t flags, void *dWork,
                                  size_t work_bytes, void *hip_stream);

/* Workspace bytes accx_reduce_sum_dev needs for (t, n, flags). */
ACCX_API acc_status accx_reduce_workspace_size(acc_dtype t, int64_t n, uint32_t flags, size_t *bytes_out);

/* dResult (device scalar of type t) = init + sum of dX[0..n), enqueued on
 * `hip_stream`.  `init` points to a HOST value of type t.  dWork as above
 * (NULL: library-owned per-stream workspace); a workspace passed in may hold
 * anything: it receives per-workgroup partial results, which every call
 * overwrites.  Calls that share a workspace must be ordered (one stream).
 * Errors: INVALID_ARG, OUT_OF_MEMORY, DEVICE, NO_DEVICE. */
ACCX_API acc_status accx_reduce_sum_dev(acc_dtype t, const void *dX, int64_t n, const void *init, void *dResult,
                               uint32_t flags, void *dWork, size_t work_bytes, void *hip_stream);

/* Workspace bytes accx_reduce_dev needs for (t, n, vars, flags). */
ACCX_API acc_status accx_reduce_vars_workspace_size(acc_dtype t, int64_t n, const acc_reduce_var *vars, int nvars,
                                                    uint32_t flags, size_t *bytes_out);

/* acc_reduce on device memory: dResult[v] (nvars device elements of type t)
 * = the variable's result; init: nvars HOST values of type t.  dX and
 * dResult aligned to the element size.  dWork as for accx_reduce_sum_dev
 * (any contents; NULL: library-owned per stream).
 * accx_reduce_sum_dev is the case of one sum variable.
 * Errors: INVALID_ARG, OUT_OF_MEMORY, DEVICE, NO_DEVICE. */
ACCX_API acc_status accx_reduce_dev(acc_dtype t, const void *dX, int64_t n, const acc_reduce_var *vars, int nvars,
                                    const void *init, void *dResult, uint32_t flags, void *dWork, size_t work_bytes,
                                    void *hip_stream);

/* One compute region holding two independent nests: the float32 loop nest
 * of Listing 1a (section 1.3) on dA, dB -> dC (len*len elements, as
 * accx_matmul_dev) and a reduction(+) nest (section 2.3) over dX[0, n)
 * into the device float *dResult = init + sum (init a HOST value).  The
 * paper's kernels construct lets one region hold several such nests; here,
 * when the matmul runs the three-product pass on the 256 x 256 tile
 * (ACC_PREC_AUTO or ACC_PREC_CHEAP3 with that tile chosen or autotuned, no
 * split K), dX is 16-byte aligned and n is at most what the pass's K loop
 * carries (2^28 floats at len = 4096: 2 x 16-byte loads per thread per
 * K-step of 16 elements), the sum is co-scheduled inside that
 * pass's launch: each workgroup streams a slice of dX beside its matrix
 * work, and the workgroups' partials are added in a fixed order by the
 * next launch (the float64 probe's with AUTO, a one-workgroup launch with
 * CHEAP3).  Otherwise the two nests run one after the other.  dC is bitwise
 * what accx_matmul_dev computes with the same flags; the sum is
 * deterministic for given (len, n, flags) but adds in another order than
 * accx_reduce_sum_dev.  Pointers 4-byte aligned, dX may be NULL when n = 0;
 * dWork: at least accx_matmul_reduce_workspace_size bytes (any contents,
 * 256-byte aligned), or NULL for the library's per-stream workspace.
 * Errors: INVALID_ARG, OUT_OF_MEMORY, DEVICE, NO_DEVICE. */
ACCX_API acc_status accx_matmul_reduce_dev(const float *dA, const float *dB, float *dC, int64_t len, uint32_t flags,
                                           const float *dX, int64_t n, float init, float *dResult, void *dWork,
                                           size_t work_bytes, void *hip_stream);
/* Workspace bytes accx_matmul_reduce_dev needs for (len, flags, n).
 * Errors: INVALID_ARG. */
ACCX_API acc_status accx_matmul_reduce_workspace_size(int64_t len, uint32_t flags, int64_t n, size_t *bytes_out);

/* accx_reduce_dev for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same arguments, kernels and results (bitwise those of accx_reduce_dev with
 * the same t, n, vars and flags), but the per-workgroup partials go to a
 * static device array of 128 KiB per GPU instead of a workspace: the call
 * allocates nothing (no hipMalloc / hipFree, no library allocation), and each
 * GPU the library runs on holds that array until the process ends.  Its
 * device address is taken once per device by acc_init.  Every call on a GPU
 * shares that GPU's array: calls that overlap on one GPU (different streams
 * or threads with no ordering between them) race and give wrong results;
 * calls ordered on one stream are safe (no contents need to start at zero;
 * each call overwrites the partials it reads).  Limit: 128 KiB of partials,
 * which holds every ACC_REDUCE_FAST reduction (any n, 1..4 variables) and
 * ACC_REDUCE_PLAIN for n <= 8388608; a larger need is INVALID_ARG.
 * (With accx_timing_enable(1) the timing facility still creates its host
 * event objects.)  Errors: INVALID_ARG, DEVICE, NO_DEVICE. */
ACCX_API acc_status accx_reduce_dev_noalloc(acc_dtype t, const void *dX, int64_t n, const acc_reduce_var *vars,
                                            int nvars, const void *init, void *dResult, uint32_t flags,
                                            void *hip_stream);

/* ---- batched launch --------------------------------------------------------
 * Many independent float32 loop-nest matmuls and reductions on device
 * pointers, run by one hipGraph of two kernels: a packing kernel for every
 * matmul operand, then a persistent kernel whose workgroups take matmul
 * output tiles and reduction chunks from one shared queue.  A matmul runs
 * 128 x 128 tiles when its LEN reaches a threshold, else 64 x 64 (or the
 * tile its flags force); ACC_BATCH_AUTOTUNE picks the threshold by timing
 * the batch itself, otherwise it is 512.  Matmuls in a batch use the
 * six-product bf16x3 split (or ACC_PREC_AUTO's steps, ACC_BATCH_PREC_AUTO);
 * a matmul's result is bitwise that of accx_matmul_dev with ACC_PREC_FULL6
 * (ACC_PREC_AUTO) and the same tile, run unsplit (a workspace without the
 * split area).  Reductions are deterministic (fixed chunking, chunk-order
 * combine). */
#define ACC_BATCH_MATMUL 0
#define ACC_BATCH_REDUCE 1
typedef struct {
    int32_t kind;  /* ACC_BATCH_MATMUL or ACC_BATCH_REDUCE */
    int32_t dtype; /* ACC_FLOAT32 */
    const void *a; /* matmul: device A (n x n); reduce: device x (n elements) */
    const void *b; /* matmul: device B (n x n); reduce: unused */
    void *c;       /* matmul: device C (n x n); reduce: device float result */
    int64_t n;     /* matmul: LEN in [1, 65536]; reduce: element count >= 0 */
    float init;    /* reduce: result = init + sum */
    uint32_t flags;/* matmul: ACC_TILE_128, ACC_TILE_64 or ACC_TILE_AUTO */
} accx_batch_item;

typedef struct accx_batch_s *accx_batch; /* opaque */

#define ACC_BATCH_AUTOTUNE 0x1u /* create: time the tile policies on this batch, keep the fastest */
#define ACC_BATCH_PREC_AUTO 0x2u /* create: matmuls take ACC_PREC_AUTO's steps per tile (the
                                    three-product pass, the float64 probe of the tile, and the
                                    correction products if the probe marks it) instead of six
                                    products; a matmul's result is then bitwise that of
                                    accx_matmul_dev with ACC_PREC_AUTO and the same tile, run
                                    unsplit */

typedef struct {
    int64_t units;        /* queue entries: matmul tiles + reduction chunks */
    int64_t tiles, chunks;
    int64_t tile_threshold; /* LEN from which un-forced matmuls take 128 x 128 tiles */
    int32_t workgroups;   /* persistent workgroups */
    int32_t matmuls, reductions;
    int32_t pad;
    uint64_t device_bytes;/* descriptors, packed operands, partials */
    double flops;         /* sum of 2 n^3 over the matmuls */
    double mfma_flops;    /* bf16 matrix-core flops of the matmuls' main pass (6 or 3 products) */
    double reduce_bytes;  /* sum of 4 n over the reductions */
} accx_batch_info_t;

/* Plan a batch: validates the items, picks tiles, allocates the device
 * workspace (charged to the budget), uploads descriptors and captures the
 * graph.  The item pointers are baked in: the same arrays are used at every
 * launch.  Errors: INVALID_ARG, OUT_OF_MEMORY, DEVICE, NO_DEVICE. */
ACCX_API acc_status accx_batch_create(const accx_batch_item *items, int nitems, uint32_t flags, accx_batch *out);
/* One hipGraphLaunch of the batch on `hip_stream`.  Launches of one batch
 * must not overlap (they share its queue and workspace). */
ACCX_API acc_status accx_batch_launch(accx_batch b, void *hip_stream);
/* The same two kernels launched directly, without the graph. */
ACCX_API acc_status accx_batch_launch_eager(accx_batch b, void *hip_stream);
ACCX_API acc_status accx_batch_info(accx_batch b, accx_batch_info_t *out);
/* Waits for the device, frees the workspace and the graph. */
ACCX_API acc_status accx_batch_destroy(accx_batch b);

/* ---- serving: continuous batching of offload-region requests -------------
 * A request is one operation of a data region (the data directive of
 * section 1.3: inputs copied in at region entry stay on the device for every
 * kernel of the region; outputs are copied out at its exit).  The server
 * keeps a FIFO of requests and `slots` HIP streams.  Progress (on submit,
 * poll and drain) retires finished requests and admits queued ones while a
 * slot is free: a region's first request is admitted when the region's
 * device footprint (arrays + workspace) fits in the server's HBM budget
 * (first requests keep arrival order; requests of open regions pass a first
 * request that waits for memory).  Requests of different regions run
 * concurrently; requests of one region keep submission order.  Host arrays
 * should be pinned (hipHostMalloc) for copies to overlap with compute.
 * Results are bitwise those of the same calls made one at a time. */
#define ACC_SERVE_MATMUL 0
#define ACC_SERVE_REDUCE 1
typedef struct {
    int32_t op;     /* ACC_SERVE_MATMUL or ACC_SERVE_REDUCE */
    int32_t dtype;  /* ACC_FLOAT32 or ACC_INT32 */
    int64_t region; /* caller's key: requests with one key share a data region */
    int32_t first;  /* 1: opens the region: device arrays allocated, inputs copied in */
    int32_t last;   /* 1: closes it: matmul c copied out, arrays freed */
    const void *a;  /* HOST matmul A (n*n) or reduction x (n); read by the first request */
    const void *b;  /* HOST matmul B (n*n); unused by reductions */
    void *c;        /* HOST matmul C (n*n), written by the last request;
                       reduction: this request's result (one element) */
    int64_t n;      /* matmul LEN; reduction element count */
    double init;    /* reduction: result = init + sum (converted to dtype) */
    uint32_t flags; /* matmul flags (ACC_KERNEL_*, ACC_PREC_*, ...); reduction flags */
    uint32_t pad;
    uint64_t tag;   /* returned in the completion */
} accx_request;

typedef struct {
    uint64_t tag;
    int32_t status; /* acc_status of the request */
    int32_t pad;
    double t_submit, t_start, t_done; /* server clock (accx_server_now), seconds */
} accx_completion;

typedef struct {
    int64_t submitted, admitted, completed, rejected;
    int64_t regions_open, max_inflight, max_regions_open;
    uint64_t budget_used, budget_peak; /* device bytes of the blocks open regions hold (now, peak) */
    uint64_t blocks_held, blocks_held_peak; /* device bytes the server holds, cached free blocks included:
                                               never above the budget when one is set */
} accx_server_stats_t;

typedef struct accx_server_s *accx_server; /* opaque */

/* slots in [1, 64]; hbm_budget_bytes = 0: no budget.  Errors: INVALID_ARG,
 * OUT_OF_MEMORY, DEVICE, NO_DEVICE. */
ACCX_API acc_status accx_server_create(int slots, uint64_t hbm_budget_bytes, accx_server *out);
/* Queue a request (validated now; a rejected request returns an error and
 * is not queued).  Requests that fail later complete with their status. */
ACCX_API acc_status accx_server_submit(accx_server s, const accx_request *r);
/* Make progress without blocking and return up to `cap` completions. */
ACCX_API acc_status accx_server_poll(accx_server s, accx_completion *out, int cap, int *n_out);
/* Block until nothing is queued or running (completions stay for poll). */
ACCX_API acc_status accx_server_drain(accx_server s);
ACCX_API acc_status accx_server_now(accx_server s, double *t_out);
ACCX_API acc_status accx_server_stats(accx_server s, accx_server_stats_t *out);
/* Drains, frees every open region, destroys the streams. */
ACCX_API acc_status accx_server_destroy(accx_server s);

/* ---- float64 error probe (ACC_PREC_AUTO) ----------------------------------
 * With ACC_PREC_AUTO the float32 tiled matmul runs the three-product split
 * first, then, per output tile of the tile configuration in use, computes 64
 * sampled entries (8 consecutive rows x 8 consecutive columns of the tile at
 * a hashed, 8-aligned position) as float64 dot products of the float32
 * inputs, compares them with the cheap result and marks the tile when the
 * sampled relative Frobenius error exceeds 7e-6 (0.7 x the 1e-5 bound; the
 * environment variable ACCX_PROBE_TAU overrides it); a correction pass on
 * 64 x 64 tiles then adds
 * the three missing products (hi*lo, lo*hi, mid*mid) inside the marked tiles
 * only.  One record per tile is left in the workspace (row-major tile order)
 * for inspection: */
typedef struct {
    int32_t rows[8], cols[8]; /* sampled rows and columns */
    double ref[64];           /* float64 dot product at (rows[u], cols[v]) in ref[8*u+v] */
    double err2, ref2;        /* sums over the samples of (C_cheap - ref)^2 and ref^2 */
    int32_t corrected;        /* 1: the tile received the correction products */
    int32_t pad[3];
} accx_probe_record;          /* 608 bytes */
/* Byte offset of the records inside the workspace of accx_matmul_dev and
 * their count, for a float32 tiled call with (len, flags), flags carrying
 * ACC_PREC_AUTO.  Errors: INVALID_ARG. */
ACCX_API acc_status accx_probe_layout(int64_t len, uint32_t flags, size_t *offset_out, int *count_out);
/* The same for accx_gemm_dev with (m, n, k, flags); m, n >= 1. */
ACCX_API acc_status accx_gemm_probe_layout(int64_t m, int64_t n, int64_t k, uint32_t flags, size_t *offset_out,
                                           int *count_out);

/* ---- autotuner ------------------------------------------------------------
 * Times every tile configuration of the tiled kernel for (t, m, n, k, and the
 * precision / limb bits of flags) on the current device, on scratch operands
 * of that shape, and records the fastest for the shape's size class (m, n
 * and k each rounded up to a power of two).  Later tiled calls with
 * ACC_TILE_AUTO in that class use it; untuned classes take a size heuristic.
 * Allocates and frees its scratch (charged to the budget while held).
 * best_tile_out: the ACC_TILE_* value chosen; ms_out: its kernel time (both
 * nullable).  accx_autotune(t, len, ...) is the square case.
 * Errors: INVALID_ARG (also m, n or k = 0), OUT_OF_MEMORY, DEVICE, NO_DEVICE. */
ACCX_API acc_status accx_autotune(acc_dtype t, int64_t len, uint32_t flags, uint32_t *best_tile_out, double *ms_out);
ACCX_API acc_status accx_autotune_gemm(acc_dtype t, int64_t m, int64_t n, int64_t k, uint32_t flags,
                                       uint32_t *best_tile_out, double *ms_out);
/* Write / read the tuned table as text, one line per entry:
 * "dtype variant class_m class_n class_k tile ms"; loading also takes
 * "dtype variant class tile ms" for a square class.
 * Errors: INVALID_ARG (I/O, format). */
ACCX_API acc_status accx_tune_save(const char *path);
ACCX_API acc_status accx_tune_load(const char *path);

/* ---- matrix-core operand packing (the prepass of the tiled kernel) -------
 * The tiled kernel reads its operands in a packed layout written by a
 * prepass: float32 -> three bf16 planes hi = RN(x), mid = RN(x - hi),
 * lo = RN(x - hi - mid) (RN = round to nearest even); int32 -> `planes`
 * balanced base-256 digit planes d_k in [-128, 127], x = sum d_k 256^k
 * (exactly for |x| within the digit range, else modulo 2^32).
 * Layout: an operand of `rows` rows of `k` elements (transposed = 0: row r of
 * the row-major rows x k array; transposed = 1: column r of the row-major
 * k x rows array) is cut into units of 32 rows x 64 bytes per plane; unit
 * (rb, kb) (rb < ceil(rows/32), kb < nkb = ceil(k * elem_bytes / 64)) starts
 * at byte (rb*nkb + kb) * planes * 2048, and inside it plane p, 16-byte chunk
 * c (0..3) of row r (0..31) is at p*2048 + c*512 + r*16.  Elements past rows
 * or k are zero.  elem_bytes = 2 (bf16) or 1 (int8). */
ACCX_API acc_status accx_packed_size(acc_dtype t, int64_t rows, int64_t k, int planes, size_t *bytes_out);
/* Pack device array dX into dOut (at least accx_packed_size bytes) on
 * `hip_stream`.  float32 needs planes = 3; int32 planes in 1..4.
 * Errors: INVALID_ARG, DEVICE, NO_DEVICE. */
ACCX_API acc_status accx_pack_dev(acc_dtype t, const void *dX, int64_t rows, int64_t k, int transposed, int planes,
                                  void *dOut, size_t out_bytes, void *hip_stream);

/* ---- kernel timing -------------------------------------------------------
 * The paper reports kernel execution time separately from launch and
 * transfer time (section 3, "Performance evaluations").  With timing on, the
 * library records a HIP event on the launch stream before and after every
 * kernel it launches; accx_timing_read synchronizes on those events and
 * returns per-kernel totals.  Off by default; costs two event records per
 * kernel when on. */
typedef struct {
    char name[48];   /* kernel name, NUL-terminated */
    int64_t launches;
    double total_ms; /* sum of event-measured durations */
    double min_ms, max_ms;
} accx_kernel_time;

ACCX_API acc_status accx_timing_enable(int on);
/* Restrict timing to the kernels named in `names` (comma-separated timing
 * names as accx_timing_read reports them, e.g. "gemm_bf16x3"); NULL or ""
 * times every kernel again.  Kernels not named get no event records.
 * Errors: INVALID_ARG (called between a kernel's two event records, i.e.
 * from another thread during a launch). */
ACCX_API acc_status accx_timing_filter(const char *names);
/* Fills up to `cap` entries, sets *n_out to the number of kernels seen;
 * reset != 0 clears the totals afterwards.  Errors: INVALID_ARG. */
ACCX_API acc_status accx_timing_read(accx_kernel_time *out, int cap, int *n_out, int reset);

/* ---- measured ceilings ----------------------------------------------------
 * The paper compares kernel times measured on its GPU (section 3,
 * "Performance evaluations").  A kernel's fraction of roofline is stated
 * against the datasheet peak; these two calls measure what this GPU reaches
 * with nothing but the bounding resource, so the fraction can also be given
 * against the measured ceiling.  Both enqueue one kernel on `hip_stream`
 * (NULL = the null stream) and allocate nothing; time them with events. */

/* Matrix instructions only: every CU runs two wavefronts per SIMD, each
 * issuing `rounds` rounds of 8 independent 32x32 matrix instructions from
 * operands in registers (kind 0: v_mfma_f32_32x32x16_bf16; kind 1:
 * v_mfma_i32_32x32x32_i8).  *ops_out = operations of the launch (2 per
 * multiply-add).  Errors: INVALID_ARG (kind not 0 or 1, rounds outside
 * [1, 2^30], ops_out NULL), DEVICE, NO_DEVICE. */
ACCX_API acc_status accx_onbox_mfma(int kind, int64_t rounds, double *ops_out, void *hip_stream);

/* Read-only stream of `bytes` of device memory at dX (16-byte aligned,
 * bytes a positive multiple of 16), three workgroups per CU.
 * Errors: INVALID_ARG, DEVICE, NO_DEVICE. */
ACCX_API acc_status accx_onbox_read(const void *dX, int64_t bytes, void *hip_stream);

/* ---- strings ------------------------------------------------------------ */
ACCX_API const char *acc_status_string(acc_status s);
ACCX_API const char *acc_last_error_string(void);
ACCX_API const char *accx_version(void);

#ifdef __cplusplus
}
#endif
#endif /* ACCX_H */
