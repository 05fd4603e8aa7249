// libaccx runtime: the C ABI of include/accx.h.
//
// Holds the present table (mapped host range -> device copy), the data
// regions with their streams, the HBM budget, library-owned workspaces and
// the dispatch from the ABI calls to the kernels.  The data-management part
// follows the paper's clause semantics (section 1.3: copy/copyin/copyout/
// create over [start:n]; section 2.3: the data functions replace the dummy
// data-clause calls with "host-accelerator pointer exchange, data copy in/out
// to/from accelerator, and memory allocation").
//
// Failure handling: no C++ exception crosses the ABI; every entry point
// returns an acc_status and leaves a thread-local message.  A device error
// inside a region poisons it: later ops on it fail fast, acc_data_end still
// frees everything and returns the first error.  For tests, ACCX_FAULT =
// "alloc:N", "copy:N" or "launch:N" makes the N-th such call (counted from
// acc_init) fail on the host, before any HIP call is made.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <set>
#include <atomic>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/accx.h"
#include "kernels.h"
#include "runtime_internal.h"

namespace {

thread_local std::string t_last_error;

acc_status fail(acc_status s, const std::string &msg)
{
    t_last_error = msg;
    return s;
}

acc_status fail_hip(hipError_t e, const char *what)
{
    return fail(ACC_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

struct Fault {
    int alloc_at = 0, copy_at = 0, launch_at = 0;
    int allocs = 0, copies = 0, launches = 0;
};

struct Entry {
    uintptr_t hbeg = 0, hend = 0;  // host byte range [hbeg, hend)
    void *dev = nullptr;
    int kind = 0, dtype = 0;       // kind: the creating clause's data movement (ACC_COPY..ACC_CREATE)
    int refs = 0;                  // region references (creating clause + present clauses)
};

struct Pending {  // an asynchronous reduction result waiting for acc_wait
    void *host_dst;
    int slot;       // first result slot
    size_t bytes;   // bytes to copy from the slots
};

struct Workspace {
    void *ptr = nullptr;
    size_t bytes = 0;
};

}  // namespace

struct acc_region_s {
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::vector<uintptr_t> keys;  // present-table keys this region holds a reference to (one per clause)
    acc_status err = ACC_OK;
    std::string err_msg;
    Workspace mm_work;            // matmul workspace
    Workspace red_work;           // fast reduction partials (any contents)
    Workspace red_plain_work;     // plain reduction partials
    Workspace red_vars_work;      // reduction-variable partials (any contents)
    void *dres = nullptr;         // device result slots (8 bytes each)
    uint64_t *hres = nullptr;     // pinned host staging for the slots
    int nslots = 0, used_slots = 0;
    std::vector<Pending> pending;
    std::vector<hipEvent_t> waits;  // events this region's stream waits on (present ranges)
};

namespace {

constexpr int kMaxSlots = 256;

std::set<accx_batch_s *> &batches();  // open batches (defined with the batch code)
void batch_release(accx_batch_s *b);
void batch_destroy_all();  // release and delete every open batch

struct State {
    std::recursive_mutex mu;
    bool init = false;
    int device = -1;
    uint64_t budget = 0;  // 0 = unlimited
    uint64_t used = 0;
    std::map<uintptr_t, Entry> present;  // key = hbeg
    std::set<acc_region_s *> regions;
    std::map<hipStream_t, Workspace> mm_ws, red_ws, red_plain_ws, red_vars_ws;  // device-pointer entries
    Fault fault;
};

State &S()
{
    static State *s = new State();  // never destroyed: safe at process exit
    return *s;
}

bool fault_hit(int &counter, int at)
{
    ++counter;
    return at > 0 && counter == at;
}

void parse_fault(Fault &f)
{
    f = Fault();
    const char *env = std::getenv("ACCX_FAULT");
    if (!env) return;
    std::string s(env);
    const size_t c = s.find(':');
    if (c == std::string::npos) return;
    const std::string kind = s.substr(0, c);
    const int n = std::atoi(s.c_str() + c + 1);
    if (kind == "alloc") f.alloc_at = n;
    if (kind == "copy") f.copy_at = n;
    if (kind == "launch") f.launch_at = n;
}

size_t elem_bytes(int t) { return (t == ACC_FLOAT64 || t == ACC_INT64) ? 8 : 4; }

// Element types of data clauses and reductions; the matmul takes the 4-byte ones.
bool valid_dtype(int t) { return t == ACC_FLOAT32 || t == ACC_INT32 || t == ACC_FLOAT64 || t == ACC_INT64; }
bool matmul_dtype(int t) { return t == ACC_FLOAT32 || t == ACC_INT32; }

// Where device memory comes from: hipMalloc, or the caller's allocator
// (accx_set_allocator).  Each block remembers the allocator that gave it,
// so that it goes back there even after the allocator has been changed.
struct Allocator {
    void *(*alloc)(size_t, void *) = nullptr;  // nullptr: hipMalloc / hipFree
    void (*free)(void *, void *) = nullptr;
    void *ctx = nullptr;
};

Allocator &user_allocator()
{
    static auto *a = new Allocator();
    return *a;
}

std::map<void *, Allocator> &user_blocks()  // blocks the caller's allocator gave
{
    static auto *m = new std::map<void *, Allocator>();
    return *m;
}

// Device memory from the current allocator, not charged to any budget.
acc_status raw_alloc(void **p, size_t bytes)
{
    *p = nullptr;
    const Allocator a = user_allocator();
    if (a.alloc) {
        void *q = a.alloc(bytes, a.ctx);
        if (!q) return fail(ACC_ERR_OUT_OF_MEMORY, "the caller's allocator returned NULL");
        if ((uintptr_t)q & 255u) {
            a.free(q, a.ctx);
            return fail(ACC_ERR_OUT_OF_MEMORY, "the caller's allocator returned memory not aligned to 256 bytes");
        }
        user_blocks()[q] = a;
        *p = q;
        return ACC_OK;
    }
    const hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        return fail(ACC_ERR_OUT_OF_MEMORY, std::string("hipMalloc: ") + hipGetErrorString(e));
    }
    return ACC_OK;
}

void raw_free(void *p)
{
    if (!p) return;
    auto &m = user_blocks();
    auto it = m.find(p);
    if (it != m.end()) {
        const Allocator a = it->second;
        m.erase(it);
        a.free(p, a.ctx);
        return;
    }
    (void)hipFree(p);
}

// Device allocation charged against the budget.
acc_status dev_alloc(void **p, size_t bytes)
{
    State &st = S();
    *p = nullptr;
    if (bytes == 0) return ACC_OK;
    if (st.budget && st.used + bytes > st.budget)
        return fail(ACC_ERR_OUT_OF_MEMORY, "HBM budget exceeded: " + std::to_string(st.used) + " used + " +
                                               std::to_string(bytes) + " requested > " +
                                               std::to_string(st.budget));
    if (fault_hit(st.fault.allocs, st.fault.alloc_at))
        return fail(ACC_ERR_OUT_OF_MEMORY, "injected allocation fault (ACCX_FAULT)");
    acc_status s = raw_alloc(p, bytes);
    if (s != ACC_OK) return s;
    st.used += bytes;
    return ACC_OK;
}

void dev_free(void *p, size_t bytes)
{
    if (!p) return;
    raw_free(p);
    State &st = S();
    st.used = st.used >= bytes ? st.used - bytes : 0;
}

acc_status ws_reserve(Workspace &w, size_t bytes, bool zero, hipStream_t stream)
{
    if (w.bytes >= bytes && w.ptr) return ACC_OK;
    if (w.ptr) {
        // the old buffer may still be in use by enqueued work
        const hipError_t e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return fail_hip(e, "hipStreamSynchronize");
        dev_free(w.ptr, w.bytes);
        w = Workspace();
    }
    void *p = nullptr;
    acc_status s = dev_alloc(&p, bytes);
    if (s != ACC_OK) return s;
    if (zero) {
        hipError_t e = hipMemsetAsync(p, 0, bytes, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        if (e != hipSuccess) {
            dev_free(p, bytes);
            return fail_hip(e, "hipMemsetAsync");
        }
    }
    w.ptr = p;
    w.bytes = bytes;
    return ACC_OK;
}

void ws_release(Workspace &w)
{
    dev_free(w.ptr, w.bytes);
    w = Workspace();
}

// Entry whose range holds [p, p + bytes), or nullptr.
Entry *lookup(const void *p, size_t bytes)
{
    State &st = S();
    const uintptr_t a = reinterpret_cast<uintptr_t>(p);
    auto it = st.present.upper_bound(a);
    if (it == st.present.begin()) return nullptr;
    --it;
    Entry &e = it->second;
    if (a < e.hbeg || a + bytes > e.hend || a + bytes < a) return nullptr;
    return &e;
}

bool overlaps_present(uintptr_t b, uintptr_t e)
{
    State &st = S();
    auto it = st.present.lower_bound(b);
    if (it != st.present.end() && it->second.hbeg < e) return true;
    if (it != st.present.begin()) {
        --it;
        if (it->second.hend > b) return true;
    }
    return false;
}

acc_status check_ready()
{
    if (!S().init) return fail(ACC_ERR_NO_DEVICE, "acc_init has not been called (or failed)");
    return ACC_OK;
}

acc_status poison(acc_region_s *r, acc_status s)
{
    if (r->err == ACC_OK) {
        r->err = s;
        r->err_msg = t_last_error;
    }
    return s;
}

// Device address for `bytes` at host address p, mapped with dtype t.
acc_status resolve(const void *p, size_t bytes, int t, const char *what, void **dev)
{
    if (!p) return fail(ACC_ERR_INVALID_ARG, std::string(what) + " is NULL");
    Entry *e = lookup(p, bytes);
    if (!e)
        return fail(ACC_ERR_NOT_PRESENT,
                    std::string(what) + " is not inside a mapped host range (or extends past its end)");
    if (e->dtype != t) return fail(ACC_ERR_INVALID_ARG, std::string(what) + " is mapped with another dtype");
    *dev = static_cast<char *>(e->dev) + (reinterpret_cast<uintptr_t>(p) - e->hbeg);
    return ACC_OK;
}

acc_status launch_fault()
{
    State &st = S();
    if (fault_hit(st.fault.launches, st.fault.launch_at))
        return fail(ACC_ERR_DEVICE, "injected launch fault (ACCX_FAULT)");
    return ACC_OK;
}

acc_status check_launch(hipError_t e, const char *what)
{
    if (e != hipSuccess) return fail_hip(e, what);
    return ACC_OK;
}

// A caller's workspace holds packed operands read by 16-byte direct-to-LDS
// loads, float64 probe records and atomic counters at offsets that are
// multiples of 256 from its start: the start must be 256-byte aligned (as
// hipMalloc and torch allocations are).
acc_status check_work_align(const void *dWork)
{
    if ((uintptr_t)dWork & 255u) return fail(ACC_ERR_INVALID_ARG, "dWork must be 256-byte aligned");
    return ACC_OK;
}

// ---- matmul dispatch ------------------------------------------------------

using accx::GemmShape;

acc_status validate_flags(uint32_t flags)
{
    const uint32_t known = ACC_KERNEL_MASK | ACC_PREC_MASK | ACC_LIMBS_MASK | ACC_ASYNC | ACC_TILE_MASK;
    if (flags & ~known) return fail(ACC_ERR_INVALID_ARG, "unknown flag bits");
    const uint32_t k = flags & ACC_KERNEL_MASK;
    if (k > ACC_KERNEL_TILED) return fail(ACC_ERR_INVALID_ARG, "unknown kernel selector");
    const uint32_t p = flags & ACC_PREC_MASK;
    if (p != ACC_PREC_AUTO && p != ACC_PREC_FULL6 && p != ACC_PREC_CHEAP3 && p != ACC_PREC_FIVE &&
        p != ACC_PREC_F32MFMA)
        return fail(ACC_ERR_INVALID_ARG, "unknown precision selector");
    const uint32_t nl = (flags & ACC_LIMBS_MASK) >> ACC_LIMBS_SHIFT;
    if (nl > 4) return fail(ACC_ERR_INVALID_ARG, "limb count must be 0 (probe) or 1..4");
    if (((flags & ACC_TILE_MASK) >> ACC_TILE_SHIFT) >= (uint32_t)accx::GEMM_TILE_COUNT)
        return fail(ACC_ERR_INVALID_ARG, "unknown tile selector");
    return ACC_OK;
}

acc_status validate_matmul(int t, int64_t len, uint32_t flags)
{
    if (!matmul_dtype(t)) return fail(ACC_ERR_INVALID_ARG, "dtype must be ACC_FLOAT32 or ACC_INT32");
    if (len < 1 || len > 65536) return fail(ACC_ERR_INVALID_ARG, "len must be in [1, 65536]");
    return validate_flags(flags);
}

constexpr int64_t kMaxMN = 131072;  // rows of A, columns of B
// Longest sequential loop.  int32 path: a digit product is at most 2^14 in
// magnitude, and shift group g (digit pairs with k+m = g) sums g+1 pairs per
// element of k (g = 3 of four digits: 4 pairs), so its int32 accumulator can
// pass 2^31 from k = 32768 on (4 * 2^14 * 2^15 = 2^31; 2^32 at k = 65536).
// Group g enters C shifted left by 8g, so only its value modulo 2^(32-8g)
// matters, and the matrix cores' integer accumulation wraps modulo 2^32
// (two's complement, no saturation): the result stays exact modulo 2^32.
// Group 0 (one pair) stays within 2^30 up to this limit.
constexpr int64_t kMaxK = 65536;
constexpr int64_t kMaxLd = (int64_t)1 << 31;

acc_status validate_gemm(int t, const GemmShape &sh, uint32_t flags)
{
    if (!matmul_dtype(t)) return fail(ACC_ERR_INVALID_ARG, "dtype must be ACC_FLOAT32 or ACC_INT32");
    if (sh.m < 0 || sh.n < 0 || sh.m > kMaxMN || sh.n > kMaxMN)
        return fail(ACC_ERR_INVALID_ARG, "m and n must be in [0, 131072]");
    if (sh.k < 0 || sh.k > kMaxK) return fail(ACC_ERR_INVALID_ARG, "k must be in [0, 65536]");
    if (sh.lda < std::max<int64_t>(1, sh.k) || sh.ldb < std::max<int64_t>(1, sh.n) ||
        sh.ldc < std::max<int64_t>(1, sh.n))
        return fail(ACC_ERR_INVALID_ARG, "leading dimensions must satisfy lda >= k, ldb >= n, ldc >= n (and >= 1)");
    if (sh.lda > kMaxLd || sh.ldb > kMaxLd || sh.ldc > kMaxLd)
        return fail(ACC_ERR_INVALID_ARG, "leading dimensions must be at most 2^31");
    return validate_flags(flags);
}

// Elements spanned by a rows x cols row-major view with leading dimension ld.
int64_t span_elems(int64_t rows, int64_t cols, int64_t ld) { return rows && cols ? (rows - 1) * ld + cols : 0; }

bool is_plain(uint32_t flags)
{
    const uint32_t k = flags & ACC_KERNEL_MASK;
    return k == ACC_KERNEL_PLAIN || k == ACC_KERNEL_PLAIN_LISTING1B;
}

constexpr size_t kMaxabsBytes = 256;  // int path: two max|x| words, padded

int flag_limbs(uint32_t flags) { return (int)((flags & ACC_LIMBS_MASK) >> ACC_LIMBS_SHIFT); }

bool is_f32mm(uint32_t flags) { return (flags & ACC_PREC_MASK) == ACC_PREC_F32MFMA; }

// Bytes per element of the packed operands the tiled kernel reads: bf16
// planes, float32 (float32 matrix cores) or int8 digits.
int kelem_bytes(int t, uint32_t flags) { return t == ACC_INT32 ? 1 : is_f32mm(flags) ? 4 : 2; }

// ACC_PREC_AUTO: relative Frobenius error a tile may show on the probe's 64
// samples and still keep the cheap (three-product) result (ACCX_PROBE_TAU
// overrides).  7e-6 = 0.7 x the 1e-5 bound of the float32 path: a tile whose
// true error is at the bound passes only if its sampled mean square falls
// below 0.49 x its expectation (for 64 independent errors a chi-square tail
// of about 1e-4), while a tile at the cheap pass's usual 4e-6 is marked only
// if its mean square exceeds 3 x its expectation, which practically never
// happens.
double probe_tau()
{
    static double tau = [] {
        const char *e = std::getenv("ACCX_PROBE_TAU");
        const double v = e ? std::atof(e) : 0.0;
        return v > 0.0 ? v : 7e-6;
    }();
    return tau;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Packed A (m rows of k) and packed B^T (n rows of k).
size_t packed_pair(const GemmShape &sh, int elem_bytes, int planes)
{
    return accx::packed_bytes(sh.m, sh.k, elem_bytes, planes) + accx::packed_bytes(sh.n, sh.k, elem_bytes, planes);
}

// Probe records live after the two packed operands; sized for the smallest
// tile so that any tile choice fits.
size_t probe_offset(const GemmShape &sh) { return align256(packed_pair(sh, 2, 3)); }
size_t probe_bytes_max(const GemmShape &sh)
{
    return (size_t)accx::probe_tiles(accx::GEMM_TILE_64, sh.m, sh.n) * sizeof(accx::ProbeRecord);
}

int resolve_tile(int t, const GemmShape &sh, uint32_t flags, int limbs);

// Split-K plan of the launch that may split (float: the first GEMM pass;
// int: the one-digit GEMM); the split area follows the other workspace parts.
struct SplitPlan {
    int tile = 0, parts = 1;
    size_t bytes = 0;
};

SplitPlan split_plan(int t, const GemmShape &sh, uint32_t flags)
{
    SplitPlan p;
    if (is_plain(flags) || sh.m == 0 || sh.n == 0 || sh.k == 0) return p;
    if (t == ACC_INT32 && flag_limbs(flags) > 1) return p;  // several digits: no split
    uint32_t f = flags;
    if (t == ACC_FLOAT32 && (flags & ACC_PREC_MASK) == ACC_PREC_AUTO) f = (flags & ~ACC_PREC_MASK) | ACC_PREC_CHEAP3;
    p.tile = resolve_tile(t, sh, f, t == ACC_INT32 ? 1 : 0);
    const int64_t nkb = (sh.k * kelem_bytes(t, flags) + 63) / 64;
    p.parts = accx::split_k_parts(p.tile, sh.m, sh.n, nkb);
    p.bytes = accx::split_k_bytes(p.tile, sh.m, sh.n, p.parts);
    return p;
}

size_t matmul_ws_base(int t, const GemmShape &sh, uint32_t flags)
{
    if (is_plain(flags) || sh.m == 0 || sh.n == 0) return 0;
    if (t == ACC_FLOAT32 && is_f32mm(flags)) return packed_pair(sh, 4, 1);
    if (t == ACC_FLOAT32 && (flags & ACC_PREC_MASK) == ACC_PREC_AUTO) return probe_offset(sh) + probe_bytes_max(sh);
    if (t == ACC_FLOAT32) return packed_pair(sh, 2, 3);
    if (flag_limbs(flags)) return kMaxabsBytes + packed_pair(sh, 1, flag_limbs(flags));
    // probe: one-digit and four-digit operands side by side
    return kMaxabsBytes + packed_pair(sh, 1, 1) + packed_pair(sh, 1, 4);
}

size_t matmul_ws_bytes(int t, const GemmShape &sh, uint32_t flags)
{
    const size_t base = matmul_ws_base(t, sh, flags);
    const SplitPlan p = split_plan(t, sh, flags);
    return p.parts > 1 ? align256(base) + p.bytes : base;
}

// ---- autotuned tile table -----------------------------------------------

int size_class(int64_t len)
{
    int c = 0;
    while ((int64_t)1 << c < len) ++c;
    return c;
}

// Variant of the kernel a tile choice applies to: float products or int limbs.
int tune_variant(int t, uint32_t flags, int limbs)
{
    if (t == ACC_FLOAT32) {
        const uint32_t p = flags & ACC_PREC_MASK;
        // AUTO is timed as its dominant kernel, the three-product pass
        if (p == ACC_PREC_F32MFMA) return 32;
        return (p == ACC_PREC_CHEAP3 || p == ACC_PREC_AUTO) ? 3 : p == ACC_PREC_FIVE ? 5 : 6;
    }
    return limbs;
}

struct TuneEntry {
    int tile;
    double ms;
};

// Key: dtype, variant (+100 per kernel family), and the size classes of m,
// n and k (each rounded up to a power of two).
using TuneKey = std::tuple<int, int, int, int, int>;

TuneKey tune_key(int t, int variant, const GemmShape &sh)
{
    return TuneKey{t, variant, size_class(sh.m), size_class(sh.n), size_class(sh.k)};
}

std::map<TuneKey, TuneEntry> &tune_table()
{
    static auto *t = new std::map<TuneKey, TuneEntry>();
    return *t;
}

int resolve_tile(int t, const GemmShape &sh, uint32_t flags, int limbs)
{
    const int forced = (int)((flags & ACC_TILE_MASK) >> ACC_TILE_SHIFT);
    if (forced) return forced;
    auto &tab = tune_table();
    auto it = tab.find(tune_key(t, tune_variant(t, flags, limbs), sh));
    return it == tab.end() ? 0 : it->second.tile;
}

// The split area if the caller's workspace holds it, else no split (a
// workspace sized before the tile table changed).
accx::SplitK split_for(int t, const GemmShape &sh, uint32_t flags, char *work, size_t work_bytes)
{
    accx::SplitK sk;
    const SplitPlan p = split_plan(t, sh, flags);
    const size_t off = align256(matmul_ws_base(t, sh, flags));
    if (p.parts > 1 && work_bytes >= off + p.bytes) {
        sk.parts = p.parts;
        sk.work = work + off;
    }
    return sk;
}

// A reduction co-scheduled with the three-product pass (see
// accx_matmul_reduce_dev): x[0, n), one partial per workgroup of the pass in
// part[0, parts), and *result = init + sum at the end (in the probe's launch
// with AUTO, else in a launch of its own after the pass).
struct CoReduce {
    const float *x;
    int64_t n;
    uint32_t *part;
    int parts;
    float init;
    float *result;
};

// The three-product pass of a float32 product, on `tile`, carrying `red`
// if given (the caller has checked that the fused launch applies).
hipError_t cheap_pass(const char *pa, const char *pbt, float *c, const GemmShape &sh, int tile, const accx::SplitK &sk,
                      const CoReduce *red, hipStream_t s)
{
    if (red) return accx::launch_gemm_bf16x3_red(pa, pbt, c, sh, red->x, red->n, red->part, s);
    return accx::launch_gemm_bf16x3(pa, pbt, c, sh, 3, false, tile, s, nullptr, sk);
}

acc_status run_tiled_f32(const float *a, const float *b, float *c, const GemmShape &sh, uint32_t flags, char *work,
                         size_t work_bytes, hipStream_t s, const CoReduce *red = nullptr)
{
    const accx::SplitK sk = split_for(ACC_FLOAT32, sh, flags, work, work_bytes);
    if (is_f32mm(flags)) {
        char *pa = work, *pbt = work + accx::packed_bytes(sh.m, sh.k, 4, 1);
        hipError_t e = accx::launch_pack_f32_pair(a, sh.m, sh.lda, b, sh.n, sh.ldb, sh.k, pa, pbt, s);
        if (e != hipSuccess) return fail_hip(e, "pack (float32) launch");
        return check_launch(
            accx::launch_gemm_f32mm(pa, pbt, c, sh, resolve_tile(ACC_FLOAT32, sh, flags, 0), s, sk),
            "gemm (float32 matrix cores) launch");
    }
    const size_t pb = accx::packed_bytes(sh.m, sh.k, 2, 3);
    char *pa = work, *pbt = work + pb;
    hipError_t e = accx::launch_pack_bf16x3_pair(a, sh.m, sh.lda, b, sh.n, sh.ldb, sh.k, pa, pbt, s);
    if (e != hipSuccess) return fail_hip(e, "pack (bf16x3) launch");
    const uint32_t prec = flags & ACC_PREC_MASK;
    if (prec == ACC_PREC_AUTO) {
        // cheap pass, float64 probe per tile, then the three missing products
        // on the tiles the probe marked (the others exit at once).  The tile
        // is made concrete here: the correction reads the probe's records in
        // the layout of this tile, which must not be left to a default that
        // each launch would resolve on its own.
        int tile = resolve_tile(ACC_FLOAT32, sh, (flags & ~ACC_PREC_MASK) | ACC_PREC_CHEAP3, 0);
        if (!tile) tile = accx::default_tile(sh.m, sh.n);
        auto *rec = reinterpret_cast<accx::ProbeRecord *>(work + probe_offset(sh));
        e = cheap_pass(pa, pbt, c, sh, tile, sk, red, s);
        accx::RedFinal fin;
        if (red) fin = accx::RedFinal{red->part, red->parts, red->init, red->result};
        if (e == hipSuccess) e = accx::launch_probe_f64(pa, pbt, c, sh, tile, probe_tau(), rec, s, fin);
        // the correction runs on 64 x 64 tiles, so a marked tile costs its
        // share of the work, not a whole pass of the big tile (128 x 128
        // correction tiles measured slower on the row-scaled LEN=8192
        // inputs: 0.89 against 0.77 ms)
        if (e == hipSuccess)
            e = accx::launch_gemm_bf16x3(pa, pbt, c, sh, -3, true, accx::GEMM_TILE_64, s, rec, accx::SplitK(), tile);
        return check_launch(e, "gemm (bf16x3, probed) launch");
    }
    const int products = (prec == ACC_PREC_CHEAP3) ? 3 : (prec == ACC_PREC_FIVE) ? 5 : 6;
    if (red) {
        e = cheap_pass(pa, pbt, c, sh, 0, sk, red, s);
        if (e == hipSuccess) e = accx::launch_reduce_final_f32(red->part, red->parts, red->init, red->result, s);
    } else
        e = accx::launch_gemm_bf16x3(pa, pbt, c, sh, products, false, resolve_tile(ACC_FLOAT32, sh, flags, 0), s,
                                     nullptr, sk);
    return check_launch(e, "gemm (bf16x3) launch");
}

// Stamp of one int32 call's max|x| words: a process-wide counter, never 0.
uint32_t next_stamp()
{
    static std::atomic<uint32_t> counter{0};
    uint32_t v;
    do {
        v = counter.fetch_add(1, std::memory_order_relaxed) + 1;
    } while (v == 0);
    return v;
}

acc_status run_tiled_i32(const int32_t *a, const int32_t *b, int32_t *c, const GemmShape &sh, uint32_t flags,
                         char *work, size_t work_bytes, hipStream_t s)
{
    const accx::SplitK sk = split_for(ACC_INT32, sh, flags, work, work_bytes);
    uint64_t *maxabs = reinterpret_cast<uint64_t *>(work);
    char *pa = work + kMaxabsBytes;
    const int nl = flag_limbs(flags);
    hipError_t e;
    if (nl == 0) {
        // Probe on the device, no host round trip: one pass writes digit 0 of
        // both operands and max|x|; the multi-digit pass and GEMM run only if
        // the maxima call for more than one digit (with as many digits as
        // they call for: two, three or four), the one-digit GEMM only if
        // they do not (each kernel reads the decision and exits at once
        // otherwise; the multi-digit kernels on small persistent grids, so
        // that their exit costs little).  The max|x| words carry this call's
        // stamp and need no clearing launch (recorded_max).
        const size_t pa1 = accx::packed_bytes(sh.m, sh.k, 1, 1), pa4 = accx::packed_bytes(sh.m, sh.k, 1, 4);
        char *p4 = pa + packed_pair(sh, 1, 1);
        const uint32_t stamp = next_stamp();
        e = accx::launch_pack_i8_pair(a, sh.m, sh.lda, b, sh.n, sh.ldb, sh.k, 1, pa, pa + pa1, maxabs, s, nullptr,
                                      stamp);
        if (e == hipSuccess)
            e = accx::launch_pack_i8_pair(a, sh.m, sh.lda, b, sh.n, sh.ldb, sh.k, 4, p4, p4 + pa4, nullptr, s, maxabs,
                                          stamp);
        if (e != hipSuccess) return fail_hip(e, "pack (int8) launch");
        e = accx::launch_gemm_i8_auto(pa, pa + pa1, p4, p4 + pa4, c, sh, resolve_tile(ACC_INT32, sh, flags, 1), s,
                                      maxabs, stamp, sk);
        return check_launch(e, "gemm (int8) launch");
    }
    const size_t pan = accx::packed_bytes(sh.m, sh.k, 1, nl);
    e = accx::launch_pack_i8_pair(a, sh.m, sh.lda, b, sh.n, sh.ldb, sh.k, nl, pa, pa + pan, nullptr, s);
    if (e != hipSuccess) return fail_hip(e, "pack (int8) launch");
    return check_launch(
        accx::launch_gemm_i8(pa, pa + pan, c, sh, nl, resolve_tile(ACC_INT32, sh, flags, nl), s, nullptr, 0, sk),
        "gemm (int8) launch");
}

acc_status run_matmul(int t, const void *a, const void *b, void *c, const GemmShape &sh, uint32_t flags, void *work,
                      size_t work_bytes, hipStream_t s)
{
    acc_status st = launch_fault();
    if (st != ACC_OK) return st;
    if (sh.m == 0 || sh.n == 0) return ACC_OK;  // empty result
    const uint32_t k = flags & ACC_KERNEL_MASK;
    if (k == ACC_KERNEL_PLAIN || k == ACC_KERNEL_PLAIN_LISTING1B) {
        const bool l1b = (k == ACC_KERNEL_PLAIN_LISTING1B);
        hipError_t e = (t == ACC_FLOAT32)
                           ? accx::launch_matmul_plain_f32(static_cast<const float *>(a),
                                                           static_cast<const float *>(b), static_cast<float *>(c), sh,
                                                           l1b, s)
                           : accx::launch_matmul_plain_i32(static_cast<const int32_t *>(a),
                                                           static_cast<const int32_t *>(b),
                                                           static_cast<int32_t *>(c), sh, l1b, s);
        return check_launch(e, "matmul (plain) launch");
    }
    if (work_bytes < matmul_ws_base(t, sh, flags)) return fail(ACC_ERR_INVALID_ARG, "workspace too small");
    if (t == ACC_FLOAT32)
        return run_tiled_f32(static_cast<const float *>(a), static_cast<const float *>(b), static_cast<float *>(c), sh,
                             flags, static_cast<char *>(work), work_bytes, s);
    return run_tiled_i32(static_cast<const int32_t *>(a), static_cast<const int32_t *>(b), static_cast<int32_t *>(c),
                         sh, flags, static_cast<char *>(work), work_bytes, s);
}

// ---- reduction dispatch ---------------------------------------------------

acc_status validate_reduce(int t, int64_t n, uint32_t flags)
{
    if (!valid_dtype(t)) return fail(ACC_ERR_INVALID_ARG, "unknown dtype");
    if (n < 0) return fail(ACC_ERR_INVALID_ARG, "n must be >= 0");
    if (flags & ~(ACC_REDUCE_PLAIN | ACC_ASYNC)) return fail(ACC_ERR_INVALID_ARG, "unknown flag bits");
    if ((flags & ACC_REDUCE_PLAIN) && !matmul_dtype(t))
        return fail(ACC_ERR_INVALID_ARG, "ACC_REDUCE_PLAIN takes float32 and int32 sums only");
    return ACC_OK;
}

// The one-variable float32/int32 sum runs on the dedicated sum kernels (fast
// or plain); every other variable set on the general kernels.
bool legacy_sum(int t, const acc_reduce_var *vars, int nvars)
{
    return matmul_dtype(t) && nvars == 1 && vars[0].op == ACC_RED_SUM && !vars[0].square;
}

acc_status validate_vars(int t, int64_t n, const acc_reduce_var *vars, int nvars, uint32_t flags)
{
    acc_status s = validate_reduce(t, n, flags & ~ACC_REDUCE_PLAIN);
    if (s != ACC_OK) return s;
    if (!vars || nvars < 1 || nvars > ACC_MAX_REDUCE_VARS)
        return fail(ACC_ERR_INVALID_ARG, "1 to 4 reduction variables expected");
    for (int v = 0; v < nvars; ++v) {
        if (vars[v].op < ACC_RED_SUM || vars[v].op > ACC_RED_OR) return fail(ACC_ERR_INVALID_ARG, "unknown operator");
        if (vars[v].square != 0 && vars[v].square != 1) return fail(ACC_ERR_INVALID_ARG, "square must be 0 or 1");
        if (vars[v].op == ACC_RED_OR && (nvars != 1 || vars[v].square))
            return fail(ACC_ERR_INVALID_ARG, "logical or is a variable of its own, over the elements themselves");
    }
    if ((flags & ACC_REDUCE_PLAIN) && !legacy_sum(t, vars, nvars))
        return fail(ACC_ERR_INVALID_ARG, "ACC_REDUCE_PLAIN takes one float32 or int32 sum");
    return ACC_OK;
}

size_t reduce_ws_bytes(int64_t n, uint32_t flags)
{
    return (flags & ACC_REDUCE_PLAIN) ? accx::reduce_plain_workspace_bytes(n) : accx::reduce_fast_workspace_bytes(n);
}

size_t vars_ws_bytes(int t, int64_t n, const acc_reduce_var *vars, int nvars, uint32_t flags)
{
    if (legacy_sum(t, vars, nvars)) return reduce_ws_bytes(n, flags);
    return accx::reduce_vars_workspace_bytes();
}

acc_status run_reduce(int t, const void *x, int64_t n, const void *init, void *dres, uint32_t flags, void *work,
                      hipStream_t s)
{
    acc_status st = launch_fault();
    if (st != ACC_OK) return st;
    const bool plain = (flags & ACC_REDUCE_PLAIN) != 0;
    hipError_t e;
    if (t == ACC_FLOAT32) {
        float iv;
        std::memcpy(&iv, init, 4);
        e = accx::launch_reduce_f32(static_cast<const float *>(x), n, iv, static_cast<float *>(dres), work, plain, s);
    } else {
        int32_t iv;
        std::memcpy(&iv, init, 4);
        e = accx::launch_reduce_i32(static_cast<const int32_t *>(x), n, iv, static_cast<int32_t *>(dres), work,
                                    plain, s);
    }
    return check_launch(e, "reduction launch");
}

// init: nvars host values of type t; dres: nvars device elements.
acc_status run_reduce_vars(int t, const void *x, int64_t n, const acc_reduce_var *vars, int nvars, const void *init,
                           void *dres, uint32_t flags, void *work, hipStream_t s)
{
    if (legacy_sum(t, vars, nvars)) return run_reduce(t, x, n, init, dres, flags, work, s);
    acc_status st = launch_fault();
    if (st != ACC_OK) return st;
    accx::RedVars rv{};
    rv.nvars = nvars;
    const size_t eb = elem_bytes(t);
    for (int v = 0; v < nvars; ++v) {
        rv.op[v] = vars[v].op;
        rv.square[v] = vars[v].square;
        std::memcpy(&rv.init[v], static_cast<const char *>(init) + v * eb, eb);
    }
    return check_launch(accx::launch_reduce_vars(t, x, n, rv, dres, work, s), "reduction launch");
}

void free_region(acc_region_s *r)
{
    State &st = S();
    // drop this region's references; a mapping goes when its last one does
    for (uintptr_t k : r->keys) {
        auto it = st.present.find(k);
        if (it == st.present.end()) continue;
        if (--it->second.refs > 0) continue;
        dev_free(it->second.dev, it->second.hend - it->second.hbeg);
        st.present.erase(it);
    }
    r->keys.clear();
    ws_release(r->mm_work);
    ws_release(r->red_work);
    ws_release(r->red_plain_work);
    ws_release(r->red_vars_work);
    if (r->dres) dev_free(r->dres, (size_t)r->nslots * 8);
    if (r->hres) (void)hipHostFree(r->hres);
    r->dres = nullptr;
    r->hres = nullptr;
    for (hipEvent_t ev : r->waits) (void)hipEventDestroy(ev);
    r->waits.clear();
    if (r->own_stream && r->stream) (void)hipStreamDestroy(r->stream);
    r->stream = nullptr;
}

acc_status finish_pending(acc_region_s *r)
{
    if (r->pending.empty()) {
        r->used_slots = 0;
        return ACC_OK;
    }
    for (const Pending &p : r->pending) std::memcpy(p.host_dst, r->hres + p.slot, p.bytes);
    r->pending.clear();
    r->used_slots = 0;
    return ACC_OK;
}

acc_status wait_region(acc_region_s *r)
{
    const hipError_t e = hipStreamSynchronize(r->stream);
    if (e != hipSuccess) return poison(r, fail_hip(e, "hipStreamSynchronize"));
    return finish_pending(r);
}


// ---- kernel timing (accx_timing_*) ----------------------------------------

struct TimingRec {
    const char *name;
    hipEvent_t start, stop;
};

struct TimingStats {
    int64_t launches = 0;
    double total = 0, mn = 1e300, mx = 0;
};

struct Timing {
    std::mutex mu;
    bool on = false;
    std::vector<std::string> only;  // record only these kernels (empty: all)
    std::vector<hipEvent_t> pool;
    std::vector<TimingRec> pending;
    int open = -1;
    std::map<std::string, TimingStats> stats;
};

Timing &TM()
{
    static Timing *t = new Timing();
    return *t;
}

hipEvent_t tm_event(Timing &t)
{
    if (!t.pool.empty()) {
        hipEvent_t e = t.pool.back();
        t.pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

void tm_collect(Timing &t)
{
    for (TimingRec &r : t.pending) {
        if (r.start && r.stop && hipEventSynchronize(r.stop) == hipSuccess) {
            float ms = 0;
            if (hipEventElapsedTime(&ms, r.start, r.stop) == hipSuccess) {
                TimingStats &st = t.stats[r.name];
                st.launches += 1;
                st.total += ms;
                st.mn = std::min(st.mn, (double)ms);
                st.mx = std::max(st.mx, (double)ms);
            }
        }
        if (r.start) t.pool.push_back(r.start);
        if (r.stop) t.pool.push_back(r.stop);
    }
    t.pending.clear();
    t.open = -1;
}

}  // namespace

thread_local bool t_capturing = false;  // no event records inside a graph capture

namespace accx {
void tmark(const char *name, hipStream_t s, bool begin)
{
    Timing &t = TM();
    if (!t.on || t_capturing) return;
    std::lock_guard<std::mutex> lk(t.mu);
    if (!t.only.empty() && std::find(t.only.begin(), t.only.end(), name) == t.only.end()) return;
    if (begin) {
        TimingRec r{name, tm_event(t), nullptr};
        if (r.start) (void)hipEventRecord(r.start, s);
        t.pending.push_back(r);
        t.open = (int)t.pending.size() - 1;
    } else if (t.open >= 0) {
        TimingRec &r = t.pending[(size_t)t.open];
        r.stop = tm_event(t);
        if (r.stop) (void)hipEventRecord(r.stop, s);
        t.open = -1;
        if (t.pending.size() > 4096) tm_collect(t);
    }
}
}  // namespace accx

// =========================================================================
extern "C" {

acc_status accx_timing_enable(int on)
{
    Timing &t = TM();
    std::lock_guard<std::mutex> lk(t.mu);
    t.on = on != 0;
    return ACC_OK;
}

acc_status accx_timing_filter(const char *names)
{
    Timing &t = TM();
    std::lock_guard<std::mutex> lk(t.mu);
    if (t.open >= 0) return fail(ACC_ERR_INVALID_ARG, "a kernel is being timed");
    t.only.clear();
    if (names) {
        std::string all(names), cur;
        for (char c : all + ",") {
            if (c == ',') {
                if (!cur.empty()) t.only.push_back(cur);
                cur.clear();
            } else {
                cur += c;
            }
        }
    }
    return ACC_OK;
}

acc_status accx_timing_read(accx_kernel_time *out, int cap, int *n_out, int reset)
{
    if (!n_out || cap < 0 || (cap > 0 && !out)) return fail(ACC_ERR_INVALID_ARG, "bad output buffer");
    Timing &t = TM();
    std::lock_guard<std::mutex> lk(t.mu);
    tm_collect(t);
    int n = 0;
    for (const auto &kv : t.stats) {
        if (n < cap) {
            accx_kernel_time &o = out[n];
            std::memset(&o, 0, sizeof o);
            std::strncpy(o.name, kv.first.c_str(), sizeof(o.name) - 1);
            o.launches = kv.second.launches;
            o.total_ms = kv.second.total;
            o.min_ms = kv.second.launches ? kv.second.mn : 0.0;
            o.max_ms = kv.second.mx;
        }
        ++n;
    }
    *n_out = n;
    if (reset) t.stats.clear();
    return ACC_OK;
}

acc_status acc_init(int device, uint64_t hbm_budget_bytes)
{
    State &st = S();
    std::lock_guard<std::recursive_mutex> lk(st.mu);
    if (device < 0) return fail(ACC_ERR_INVALID_ARG, "device must be >= 0");
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess || count == 0) {
        (void)hipGetLastError();
        return fail(ACC_ERR_NO_DEVICE, "no HIP device visible");
    }
    if (device >= count) return fail(ACC_ERR_NO_DEVICE, "device ordinal out of range");
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, device);
    if (e != hipSuccess) return fail_hip(e, "hipGetDeviceProperties");
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(ACC_ERR_NO_DEVICE, std::string("device is ") + prop.gcnArchName + ", libaccx is built for gfx950");
    e = hipSetDevice(device);
    if (e != hipSuccess) return fail_hip(e, "hipSetDevice");
    // device address of the static scratch on this device (once per device)
    e = accx::noalloc_scratch_setup(device);
    if (e != hipSuccess) return fail_hip(e, "hipGetSymbolAddress (static reduction scratch)");
    st.init = true;
    st.device = device;
    st.budget = hbm_budget_bytes;
    parse_fault(st.fault);
    return ACC_OK;
}

acc_status acc_shutdown(void)
{
    State &st = S();
    std::lock_guard<std::recursive_mutex> lk(st.mu);
    if (!st.init) return ACC_OK;
    (void)hipDeviceSynchronize();
    for (acc_region_s *r : st.regions) {
        free_region(r);
        delete r;
    }
    st.regions.clear();
    batch_destroy_all();
    for (auto *m : {&st.mm_ws, &st.red_ws, &st.red_plain_ws, &st.red_vars_ws}) {
        for (auto &kv : *m) ws_release(kv.second);
        m->clear();
    }
    st.present.clear();
    st.used = 0;
    st.init = false;
    return ACC_OK;
}

acc_status acc_budget_used(uint64_t *bytes_out)
{
    State &st = S();
    std::lock_guard<std::recursive_mutex> lk(st.mu);
    if (!bytes_out) return fail(ACC_ERR_INVALID_ARG, "bytes_out is NULL");
    *bytes_out = st.used;
    return ACC_OK;
}

acc_status accx_set_allocator(void *(*alloc)(size_t, void *), void (*free_)(void *, void *), void *ctx)
{
    State &st = S();
    std::lock_guard<std::recursive_mutex> lk(st.mu);
    if (!alloc != !free_) return fail(ACC_ERR_INVALID_ARG, "give both alloc and free, or neither");
    Allocator &a = user_allocator();
    a.alloc = alloc;
    a.free = free_;
    a.ctx = alloc ? ctx : nullptr;
    return ACC_OK;
}

acc_status acc_data_begin(const acc_clause *cl, int ncl, void *hip_stream, acc_region *out)
{
    State &st = S();
    std::lock_guard<std::recursive_mutex> lk(st.mu);
    if (!out) return fail(ACC_ERR_INVALID_ARG, "region_out is NULL");
    *out = nullptr;
    if (ncl < 0 || (ncl > 0 && !cl)) return fail(ACC_ERR_INVALID_ARG, "bad clause list");
    acc_status s = check_ready();
    if (s != ACC_OK) return s;

    // Validate every clause before touching the device.  A present clause,
    // and a present_or_* clause whose range is already mapped, takes a
    // reference to the mapping that holds it; every other clause maps a new
    // range, which must not overlap any mapped range or another new one.
    struct Plan {
        uintptr_t b, e;
        int kind;            // data movement of a new mapping
        int dtype;
        uintptr_t ref = 0;   // key of the mapping referenced, else 0
        bool fresh = false;  // maps a new range
    };
    std::vector<Plan> plan;
    uint64_t total = 0;
    for (int k = 0; k < ncl; ++k) {
        const acc_clause &c = cl[k];
        if (c.kind < ACC_COPY || c.kind > ACC_PRESENT_OR_CREATE)
            return fail(ACC_ERR_INVALID_ARG, "unknown clause kind");
        if (!valid_dtype(c.dtype)) return fail(ACC_ERR_INVALID_ARG, "unknown clause dtype");
        if (c.start < 0 || c.n < 0) return fail(ACC_ERR_INVALID_ARG, "clause start and n must be >= 0");
        if (c.n == 0) continue;
        if (!c.host) return fail(ACC_ERR_INVALID_ARG, "clause host pointer is NULL");
        if (c.n > (int64_t)(1ll << 40)) return fail(ACC_ERR_INVALID_ARG, "clause too large");
        Plan p;
        p.b = reinterpret_cast<uintptr_t>(c.host) + (uintptr_t)c.start * elem_bytes(c.dtype);
        p.e = p.b + (uintptr_t)c.n * elem_bytes(c.dtype);
        const bool present_kind = c.kind >= ACC_PRESENT;
        p.kind = c.kind >= ACC_PRESENT_OR_COPY ? c.kind - ACC_PRESENT_OR_COPY + ACC_COPY : c.kind;
        p.dtype = c.dtype;
        Entry *hold = present_kind ? lookup(reinterpret_cast<void *>(p.b), p.e - p.b) : nullptr;
        if (hold) {
            if (hold->dtype != c.dtype)
                return fail(ACC_ERR_INVALID_ARG, "clause " + std::to_string(k) + " is mapped with another dtype");
            p.ref = hold->hbeg;
        } else if (c.kind == ACC_PRESENT) {
            return fail(ACC_ERR_NOT_PRESENT, "present clause " + std::to_string(k) + " is not inside a mapped range");
        } else {
            if (overlaps_present(p.b, p.e))
                return fail(ACC_ERR_ALREADY_PRESENT, "clause " + std::to_string(k) + " overlaps a mapped host range");
            for (const Plan &q : plan)
                if (q.fresh && p.b < q.e && q.b < p.e) return fail(ACC_ERR_ALREADY_PRESENT, "clauses of one region overlap");
            p.fresh = true;
            total += p.e - p.b;
        }
        plan.push_back(p);
    }
    if (st.budget && st.used + total > st.budget)
        return fail(ACC_ERR_OUT_OF_MEMORY, "region needs " + std::to_string(total) + " bytes; budget has " +
                                               std::to_string(st.budget - std::min(st.budget, st.used)) + " left");

    acc_region_s *r = new (std::nothrow) acc_region_s();
    if (!r) return fail(ACC_ERR_OUT_OF_MEMORY, "host allocation failed");
    if (hip_stream) {
        r->stream = static_cast<hipStream_t>(hip_stream);
    } else {
        const hipError_t e = hipStreamCreateWithFlags(&r->stream, hipStreamNonBlocking);
        if (e != hipSuccess) {
            delete r;
            return fail_hip(e, "hipStreamCreate");
        }
        r->own_stream = true;
    }

    for (const Plan &p : plan) {
        if (!p.fresh) {
            // The mapping's contents are whatever the regions holding it have
            // enqueued so far (its copy-in, kernels that write it): this
            // region's stream waits for all of it before its own work.
            for (acc_region_s *h : st.regions) {
                if (h->stream == r->stream || std::find(h->keys.begin(), h->keys.end(), p.ref) == h->keys.end())
                    continue;
                hipEvent_t ev = nullptr;
                hipError_t e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
                if (e == hipSuccess) e = hipEventRecord(ev, h->stream);
                if (e == hipSuccess) e = hipStreamWaitEvent(r->stream, ev, 0);
                if (ev) r->waits.push_back(ev);
                if (e != hipSuccess) {
                    s = fail_hip(e, "ordering after the regions holding a present range");
                    const std::string msg = t_last_error;
                    (void)hipStreamSynchronize(r->stream);
                    free_region(r);
                    delete r;
                    return fail(s, msg);
                }
            }
            st.present[p.ref].refs++;
            r->keys.push_back(p.ref);
            continue;
        }
        Entry en;
        en.hbeg = p.b;
        en.hend = p.e;
        en.kind = p.kind;
        en.dtype = p.dtype;
        en.refs = 1;
        s = dev_alloc(&en.dev, en.hend - en.hbeg);
        if (s == ACC_OK && (p.kind == ACC_COPY || p.kind == ACC_COPYIN)) {
            if (fault_hit(st.fault.copies, st.fault.copy_at)) {
                s = fail(ACC_ERR_DEVICE, "injected copy fault (ACCX_FAULT)");
            } else {
                const hipError_t e = hipMemcpyAsync(en.dev, reinterpret_cast<void *>(en.hbeg), en.hend - en.hbeg,
                                                    hipMemcpyHostToDevice, r->stream);
                if (e != hipSuccess) s = fail_hip(e, "hipMemcpyAsync H2D");
            }
        }
        if (s != ACC_OK) {
            const std::string msg = t_last_error;
            if (en.dev) {
                (void)hipStreamSynchronize(r->stream);
                dev_free(en.dev, en.hend - en.hbeg);
            }
            (void)hipStreamSynchronize(r->stream);
            free_region(r);
            delete r;
            return fail(s, msg);
        }
        st.present[en.hbeg] = en;
        r->keys.push_back(en.hbeg);
    }
    st.regions.insert(r);
    *out = r;
    return ACC_OK;
}

acc_status acc_wait(acc_region r)
{
    State &st = S();
    std::lock_guard<std::recursive_mutex> lk(st.mu);
    if (!r || !st.regions.count(r)) return fail(ACC_ERR_INVALID_ARG, "unknown region");
    acc_status s = wait_region(r);
    if (s != ACC_OK) return s;
    if (r->err != ACC_OK) return fail(r->err, r->err_msg);
    return ACC_OK;
}

acc_status acc_data_end(acc_region r)
{
    State &st = S();
    std::lock_guard<std::recursive_mutex> lk(st.mu);
    if (!r || !st.regions.count(r)) return fail(ACC_ERR_INVALID_ARG, "unknown region");
    acc_status first = r->err;
    std::string first_msg = r->err_msg;
    acc_status s = wait_region(r);
    if (first == ACC_OK && s != ACC_OK) {
        first = s;
        first_msg = t_last_error;
    }
    if (first == ACC_OK) {
        // copy out the mappings whose last reference this region drops
        std::map<uintptr_t, int> held;
        for (uintptr_t k : r->keys) held[k]++;
        for (const auto &kv : held) {
            const Entry &en = st.present[kv.first];
            if (en.refs > kv.second) continue;
            if (en.kind != ACC_COPY && en.kind != ACC_COPYOUT) continue;
            if (fault_hit(st.fault.copies, st.fault.copy_at)) {
                first = ACC_ERR_DEVICE;
                first_msg = "injected copy fault (ACCX_FAULT)";
                break;
            }
            const hipError_t e = hipMemcpyAsync(reinterpret_cast<void *>(en.hbeg), en.dev, en.hend - en.hbeg,
                                                hipMemcpyDeviceToHost, r->stream);
            if (e != hipSuccess) {
                first = fail_hip(e, "hipMemcpyAsync D2H");
                first_msg = t_last_error;
                break;
            }
        }
        const hipError_t e = hipStreamSynchronize(r->stream);
        if (e != hipSuccess && first == ACC_OK) {
            first = fail_hip(e, "hipStreamSynchronize");
            first_msg = t_last_error;
        }
    }
    free_region(r);
    st.regions.erase(r);
    delete r;
    if (first != ACC_OK) return fail(first, first_msg);
    return ACC_OK;
}

acc_status acc_update(acc_region r, int direction, acc_dtype t, void *host, int64_t start, int64_t n,
                      uint32_t flags)
{
    State &st = S();
    std::lock_guard<std::recursive_mutex> lk(st.mu);
    if (!r || !st.regions.count(r)) return fail(ACC_ERR_INVALID_ARG, "unknown region");
    if (r->err != ACC_OK) return fail(r->err, "region already failed: " + r->err_msg);
    if (direction != ACC_UPDATE_HOST && direction != ACC_UPDATE_DEVICE)
        return fail(ACC_ERR_INVALID_ARG, "direction must be ACC_UPDATE_HOST or ACC_UPDATE_DEVICE");
    if (!valid_dtype(t)) return fail(ACC_ERR_INVALID_ARG, "unknown dtype");
    if (start < 0 || n < 0) return fail(ACC_ERR_INVALID_ARG, "start and n must be >= 0");
    if (flags & ~ACC_ASYNC) return fail(ACC_ERR_INVALID_ARG, "unknown flag bits");
    if (n == 0) return ACC_OK;
    if (!host) return fail(ACC_ERR_INVALID_ARG, "host is NULL");
    char *h = static_cast<char *>(host) + start * (int64_t)elem_bytes(t);
    const size_t bytes = (size_t)n * elem_bytes(t);
    void *dev;
    acc_status s = resolve(h, bytes, t, "update range", &dev);
    if (s != ACC_OK) return s;
    if (fault_hit(st.fault.copies, st.fault.copy_at)) return poison(r, fail(ACC_ERR_DEVICE, "injected copy fault (ACCX_FAULT)"));
    const hipError_t e = direction == ACC_UPDATE_HOST
                             ? hipMemcpyAsync(h, dev, bytes, hipMemcpyDeviceToHost, r->stream)
                             : hipMemcpyAsync(dev, h, bytes, hipMemcpyHostToDevice, r->stream);
    if (e != hipSuccess) return poison(r, fail_hip(e, "hipMemcpyAsync (update)"));
    if (flags & ACC_ASYNC) return ACC_OK;
    return wait_region(r);
}

acc_status acc_is_present(const void *host, size_t bytes, int *present_out)
{
    State &st = S();
    std::lock_guard<std::recursive_mutex> lk(st.mu);
    if (!present_out) return fail(ACC_ERR_INVALID_ARG, "present_out is NULL");
    *present_out = host && lookup(host, bytes ? bytes : 1) ? 1 : 0;
    return ACC_OK;
}

acc_status accx_host_alloc(size_t bytes, void **host_out)
{
    if (!host_out) return fail(ACC_ERR_INVALID_ARG, "host_out is NULL");
    *host_out = nullptr;
    acc_status s = check_ready();
    if (s != ACC_OK) return s;
    const hipError_t e = hipHostMalloc(host_out, bytes ? bytes : 1, hipHostMallocDefault);
    if (e != hipSuccess) return fail(ACC_ERR_OUT_OF_MEMORY, std::string("hipHostMalloc: ") + hipGetErrorString(e));
    return ACC_OK;
}

acc_status accx_host_free(void *host)
{
    if (!host) return ACC_OK;
    const hipError_t e = hipHostFree(host);
    if (e != hipSuccess) return fail_hip(e, "hipHostFree");
    return ACC_OK;
}

acc_status acc_deviceptr(const void *host, void **device_out)
{
    State &st = S();
    std::lock_guard<std::recursive_mutex> lk(st.mu);
    if (!device_out) return fail(ACC_ERR_INVALID_ARG, "device_out is NULL");
    *device_out = nullptr;
    Entry *e = lookup(host, 1);
    if (!e) return fail(ACC_ERR_NOT_PRESENT, "host address is not mapped");
    *device_out = static_cast<char *>(e->dev) + (reinterpret_cast<uintptr_t>(host) - e->hbeg);
    return ACC_OK;
}

namespace {
acc_status region_gemm(acc_region r, int t, const GemmShape &sh, const void *a, const void *b, void *c,
                       uint32_t flags)
{
    State &st = S();
    if (!r || !st.regions.count(r)) return fail(ACC_ERR_INVALID_ARG, "unknown region");
    if (r->err != ACC_OK) return fail(r->err, "region already failed: " + r->err_msg);
    acc_status s = validate_gemm(t, sh, flags);
    if (s != ACC_OK) return s;
    if (sh.m == 0 || sh.n == 0) return ACC_OK;
    const size_t ab = (size_t)span_elems(sh.m, sh.k, sh.lda) * 4, bb = (size_t)span_elems(sh.k, sh.n, sh.ldb) * 4;
    const size_t cb = (size_t)span_elems(sh.m, sh.n, sh.ldc) * 4;
    void *da = nullptr, *db = nullptr, *dc;
    if (ab && (s = resolve(a, ab, t, "a", &da)) != ACC_OK) return s;
    if (bb && (s = resolve(b, bb, t, "b", &db)) != ACC_OK) return s;
    if ((s = resolve(c, cb, t, "c", &dc)) != ACC_OK) return s;
    const uintptr_t ci = reinterpret_cast<uintptr_t>(c);
    const std::pair<const void *, size_t> ins[2] = {{a, ab}, {b, bb}};
    for (const auto &in : ins) {
        const uintptr_t ii = reinterpret_cast<uintptr_t>(in.first);
        if (in.second && ci < ii + in.second && ii < ci + cb) return fail(ACC_ERR_INVALID_ARG, "c overlaps an input");
    }
    const size_t wsb = matmul_ws_bytes(t, sh, flags);
    if (wsb && (s = ws_reserve(r->mm_work, wsb, false, r->stream)) != ACC_OK) return s;
    s = run_matmul(t, da, db, dc, sh, flags, r->mm_work.ptr, r->mm_work.bytes, r->stream);
    if (s != ACC_OK) return poison(r, s);
    return ACC_OK;
}
}  // namespace

acc_status acc_loopnest_matmul(acc_region r, acc_dtype t, const void *a, const void *b, void *c, int64_t len,
                               uint32_t flags)
{
    std::lock_guard<std::recursive_mutex> lk(S().mu);
    acc_status s = validate_matmul(t, len, flags);
    if (s != ACC_OK) return s;
    return region_gemm(r, t, accx::square_shape(len), a, b, c, flags);
}

acc_status acc_loopnest_gemm(acc_region r, acc_dtype t, int64_t m, int64_t n, int64_t k, const void *a, int64_t lda,
                             const void *b, int64_t ldb, void *c, int64_t ldc, uint32_t flags)
{
    std::lock_guard<std::recursive_mutex> lk(S().mu);
    return region_gemm(r, t, GemmShape{m, n, k, lda, ldb, ldc}, a, b, c, flags);
}

namespace {
// Logical or of zero elements: the variable becomes 1 if it was nonzero, else 0.
void or_of_nothing(int t, void *inout)
{
    switch (t) {
    case ACC_FLOAT32: *static_cast<float *>(inout) = *static_cast<float *>(inout) != 0.0f ? 1.0f : 0.0f; break;
    case ACC_INT32: *static_cast<int32_t *>(inout) = *static_cast<int32_t *>(inout) != 0; break;
    case ACC_FLOAT64: *static_cast<double *>(inout) = *static_cast<double *>(inout) != 0.0 ? 1.0 : 0.0; break;
    default: *static_cast<int64_t *>(inout) = *static_cast<int64_t *>(inout) != 0; break;
    }
}

acc_status region_reduce(acc_region r, int t, const void *x, int64_t n, const acc_reduce_var *vars, int nvars,
                         void *inout, uint32_t flags)
{
    State &st = S();
    if (!r || !st.regions.count(r)) return fail(ACC_ERR_INVALID_ARG, "unknown region");
    if (r->err != ACC_OK) return fail(r->err, "region already failed: " + r->err_msg);
    acc_status s = validate_vars(t, n, vars, nvars, flags);
    if (s != ACC_OK) return s;
    if (!inout) return fail(ACC_ERR_INVALID_ARG, "inout_result is NULL");
    if (n == 0) {  // nothing to fold: every variable keeps its value
        if (vars[0].op == ACC_RED_OR) or_of_nothing(t, inout);
        return ACC_OK;
    }
    const size_t eb = elem_bytes(t);
    void *dx;
    if ((s = resolve(x, (size_t)n * eb, t, "x", &dx)) != ACC_OK) return s;
    if (!r->dres) {
        if ((s = dev_alloc(&r->dres, (size_t)kMaxSlots * 8)) != ACC_OK) return s;
        r->nslots = kMaxSlots;
        const hipError_t e = hipHostMalloc(reinterpret_cast<void **>(&r->hres), (size_t)kMaxSlots * 8);
        if (e != hipSuccess) return fail_hip(e, "hipHostMalloc");
    }
    if (r->used_slots + nvars > r->nslots) {
        if ((s = wait_region(r)) != ACC_OK) return s;
    }
    const bool legacy = legacy_sum(t, vars, nvars);
    const bool plain = (flags & ACC_REDUCE_PLAIN) != 0;
    Workspace &w = !legacy ? r->red_vars_work : plain ? r->red_plain_work : r->red_work;
    if ((s = ws_reserve(w, vars_ws_bytes(t, n, vars, nvars, flags), false, r->stream)) != ACC_OK) return s;
    const int slot = r->used_slots;
    r->used_slots += nvars;
    void *dslot = static_cast<char *>(r->dres) + (size_t)slot * 8;
    s = run_reduce_vars(t, dx, n, vars, nvars, inout, dslot, flags, w.ptr, r->stream);
    if (s != ACC_OK) return poison(r, s);
    hipError_t e = hipMemcpyAsync(r->hres + slot, dslot, nvars * eb, hipMemcpyDeviceToHost, r->stream);
    if (e != hipSuccess) return poison(r, fail_hip(e, "hipMemcpyAsync D2H (result)"));
    r->pending.push_back(Pending{inout, slot, nvars * eb});
    if (flags & ACC_ASYNC) return ACC_OK;
    return wait_region(r);
}
}  // namespace

acc_status acc_reduce_sum(acc_region r, acc_dtype t, const void *x, int64_t n, void *inout, uint32_t flags)
{
    std::lock_guard<std::recursive_mutex> lk(S().mu);
    const acc_reduce_var sum{ACC_RED_SUM, 0};
    return region_reduce(r, t, x, n, &sum, 1, inout, flags);
}

acc_status acc_reduce(acc_region r, acc_dtype t, const void *x, int64_t n, const acc_reduce_var *vars, int nvars,
                      void *inout, uint32_t flags)
{
    std::lock_guard<std::recursive_mutex> lk(S().mu);
    return region_reduce(r, t, x, n, vars, nvars, inout, flags);
}

acc_status accx_matmul_workspace_size(acc_dtype t, int64_t len, uint32_t flags, size_t *bytes_out)
{
    if (!bytes_out) return fail(ACC_ERR_INVALID_ARG, "bytes_out is NULL");
    acc_status s = validate_matmul(t, len, flags);
    if (s != ACC_OK) return s;
    *bytes_out = matmul_ws_bytes(t, accx::square_shape(len), flags);
    return ACC_OK;
}

acc_status accx_gemm_workspace_size(acc_dtype t, int64_t m, int64_t n, int64_t k, uint32_t flags, size_t *bytes_out)
{
    if (!bytes_out) return fail(ACC_ERR_INVALID_ARG, "bytes_out is NULL");
    const GemmShape sh{m, n, k, std::max<int64_t>(1, k), std::max<int64_t>(1, n), std::max<int64_t>(1, n)};
    acc_status s = validate_gemm(t, sh, flags);
    if (s != ACC_OK) return s;
    *bytes_out = matmul_ws_bytes(t, sh, flags);
    return ACC_OK;
}

namespace {
acc_status dev_gemm(int t, const GemmShape &sh, const void *dA, const void *dB, void *dC, uint32_t flags, void *dWork,
                    size_t work_bytes, void *hip_stream)
{
    State &st = S();
    acc_status s = check_ready();
    if (s != ACC_OK) return s;
    if ((s = validate_gemm(t, sh, flags)) != ACC_OK) return s;
    if (flags & ACC_ASYNC) return fail(ACC_ERR_INVALID_ARG, "ACC_ASYNC applies to region calls only");
    if (sh.m == 0 || sh.n == 0) return ACC_OK;
    if ((sh.k > 0 && (!dA || !dB)) || !dC) return fail(ACC_ERR_INVALID_ARG, "NULL device pointer");
    if (((uintptr_t)dA | (uintptr_t)dB | (uintptr_t)dC) & 3u)
        return fail(ACC_ERR_INVALID_ARG, "device pointers must be 4-byte aligned");
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    const size_t need = matmul_ws_bytes(t, sh, flags);
    if (need) {
        if (dWork) {
            if ((s = check_work_align(dWork)) != ACC_OK) return s;
            // below `need` but holding the operands: runs without split K
            if (work_bytes < matmul_ws_base(t, sh, flags)) return fail(ACC_ERR_INVALID_ARG, "workspace too small");
        } else {
            Workspace &w = st.mm_ws[stream];
            if ((s = ws_reserve(w, need, false, stream)) != ACC_OK) return s;
            dWork = w.ptr;
            work_bytes = w.bytes;
        }
    }
    return run_matmul(t, dA, dB, dC, sh, flags, dWork, work_bytes, stream);
}
}  // namespace

acc_status accx_matmul_dev(acc_dtype t, const void *dA, const void *dB, void *dC, int64_t len, uint32_t flags,
                           void *dWork, size_t work_bytes, void *hip_stream)
{
    std::lock_guard<std::recursive_mutex> lk(S().mu);
    acc_status s = check_ready();
    if (s != ACC_OK) return s;
    if ((s = validate_matmul(t, len, flags)) != ACC_OK) return s;
    return dev_gemm(t, accx::square_shape(len), dA, dB, dC, flags, dWork, work_bytes, hip_stream);
}

acc_status accx_gemm_dev(acc_dtype t, int64_t m, int64_t n, int64_t k, const void *dA, int64_t lda, const void *dB,
                         int64_t ldb, void *dC, int64_t ldc, uint32_t flags, void *dWork, size_t work_bytes,
                         void *hip_stream)
{
    std::lock_guard<std::recursive_mutex> lk(S().mu);
    return dev_gemm(t, GemmShape{m, n, k, lda, ldb, ldc}, dA, dB, dC, flags, dWork, work_bytes, hip_stream);
}

acc_status accx_reduce_workspace_size(acc_dtype t, int64_t n, uint32_t flags, size_t *bytes_out)
{
    const acc_reduce_var sum{ACC_RED_SUM, 0};
    return accx_reduce_vars_workspace_size(t, n, &sum, 1, flags, bytes_out);
}

acc_status accx_reduce_vars_workspace_size(acc_dtype t, int64_t n, const acc_reduce_var *vars, int nvars,
                                           uint32_t flags, size_t *bytes_out)
{
    if (!bytes_out) return fail(ACC_ERR_INVALID_ARG, "bytes_out is NULL");
    acc_status s = validate_vars(t, n, vars, nvars, flags);
    if (s != ACC_OK) return s;
    *bytes_out = vars_ws_bytes(t, n, vars, nvars, flags);
    return ACC_OK;
}

namespace {
// Checks shared by the device-pointer reductions.
acc_status dev_reduce_args(int t, const void *dX, int64_t n, const acc_reduce_var *vars, int nvars, const void *init,
                           const void *dResult, uint32_t flags)
{
    acc_status s = check_ready();
    if (s != ACC_OK) return s;
    if ((s = validate_vars(t, n, vars, nvars, flags)) != ACC_OK) return s;
    if (flags & ACC_ASYNC) return fail(ACC_ERR_INVALID_ARG, "ACC_ASYNC applies to region calls only");
    if ((n > 0 && !dX) || !dResult || !init) return fail(ACC_ERR_INVALID_ARG, "NULL pointer");
    const uintptr_t am = elem_bytes(t) - 1;
    if (((uintptr_t)dX | (uintptr_t)dResult) & am)
        return fail(ACC_ERR_INVALID_ARG, "pointers must be aligned to the element size");
    return ACC_OK;
}

acc_status dev_reduce(int t, const void *dX, int64_t n, const acc_reduce_var *vars, int nvars, const void *init,
                      void *dResult, uint32_t flags, void *dWork, size_t work_bytes, void *hip_stream)
{
    State &st = S();
    acc_status s = dev_reduce_args(t, dX, n, vars, nvars, init, dResult, flags);
    if (s != ACC_OK) return s;
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    const bool legacy = legacy_sum(t, vars, nvars);
    const bool plain = (flags & ACC_REDUCE_PLAIN) != 0;
    const size_t need = vars_ws_bytes(t, n, vars, nvars, flags);
    if (dWork) {
        if ((s = check_work_align(dWork)) != ACC_OK) return s;
        if (work_bytes < need) return fail(ACC_ERR_INVALID_ARG, "workspace too small");
    } else {
        Workspace &w = !legacy ? st.red_vars_ws[stream] : plain ? st.red_plain_ws[stream] : st.red_ws[stream];
        if ((s = ws_reserve(w, need, false, stream)) != ACC_OK) return s;
        dWork = w.ptr;
    }
    return run_reduce_vars(t, dX, n, vars, nvars, init, dResult, flags, dWork, stream);
}
}  // namespace

acc_status accx_reduce_sum_dev(acc_dtype t, const void *dX, int64_t n, const void *init, void *dResult,
                               uint32_t flags, void *dWork, size_t work_bytes, void *hip_stream)
{
    std::lock_guard<std::recursive_mutex> lk(S().mu);
    const acc_reduce_var sum{ACC_RED_SUM, 0};
    return dev_reduce(t, dX, n, &sum, 1, init, dResult, flags, dWork, work_bytes, hip_stream);
}

acc_status accx_reduce_dev(acc_dtype t, const void *dX, int64_t n, const acc_reduce_var *vars, int nvars,
                           const void *init, void *dResult, uint32_t flags, void *dWork, size_t work_bytes,
                           void *hip_stream)
{
    std::lock_guard<std::recursive_mutex> lk(S().mu);
    return dev_reduce(t, dX, n, vars, nvars, init, dResult, flags, dWork, work_bytes, hip_stream);
}

namespace {
// A float32 matmul nest and an independent reduction(+) nest in one region:
// whether the sum rides in the three-product pass's launch (the pass runs
// unsplit on the 256 x 256 tile and x is 16-byte aligned), and where the
// workspace holds the matmul's part and the reduction's partials.
struct MatRedPlan {
    bool fused = false;
    size_t mm = 0, red_off = 0, total = 0;
    int parts = 0;
};

MatRedPlan matred_plan(const GemmShape &sh, uint32_t flags, int64_t n, const void *dX)
{
    MatRedPlan p;
    p.mm = matmul_ws_bytes(ACC_FLOAT32, sh, flags);
    p.red_off = align256(p.mm);
    p.parts = accx::red_fused_parts(sh.m, sh.n);
    p.total = p.red_off + std::max(sizeof(uint32_t) * (size_t)p.parts, accx::reduce_fast_workspace_bytes(n));
    const uint32_t prec = flags & ACC_PREC_MASK;
    if (is_plain(flags) || (prec != ACC_PREC_AUTO && prec != ACC_PREC_CHEAP3)) return p;
    if (!dX || ((uintptr_t)dX & 15u)) return p;
    // a sum larger than the pass's loads can carry runs on its own at full
    // HBM rate instead of in the pass's tail
    if (n > accx::red_fused_capacity(sh.m, sh.n, sh.k)) return p;
    int tile = resolve_tile(ACC_FLOAT32, sh, (flags & ~ACC_PREC_MASK) | ACC_PREC_CHEAP3, 0);
    if (!tile) tile = accx::default_tile(sh.m, sh.n);
    if (tile != accx::GEMM_TILE_256 || split_plan(ACC_FLOAT32, sh, flags).parts > 1) return p;
    p.fused = true;
    return p;
}
}  // namespace

acc_status accx_matmul_reduce_workspace_size(int64_t len, uint32_t flags, int64_t n, size_t *bytes_out)
{
    std::lock_guard<std::recursive_mutex> lk(S().mu);
    if (!bytes_out) return fail(ACC_ERR_INVALID_ARG, "bytes_out is NULL");
    acc_status s = validate_matmul(ACC_FLOAT32, len, flags);
    if (s != ACC_OK) return s;
    if (n < 0) return fail(ACC_ERR_INVALID_ARG, "n must be >= 0");
    *bytes_out = matred_plan(accx::square_shape(len), flags, n, nullptr).total;
    return ACC_OK;
}

acc_status accx_matmul_reduce_dev(const float *dA, const float *dB, float *dC, int64_t len, uint32_t flags,
                                  const float *dX, int64_t n, float init, float *dResult, void *dWork,
                                  size_t work_bytes, void *hip_stream)
{
    std::lock_guard<std::recursive_mutex> lk(S().mu);
    State &st = S();
    acc_status s = check_ready();
    if (s != ACC_OK) return s;
    if ((s = validate_matmul(ACC_FLOAT32, len, flags)) != ACC_OK) return s;
    if (flags & ACC_ASYNC) return fail(ACC_ERR_INVALID_ARG, "ACC_ASYNC applies to region calls only");
    if (n < 0) return fail(ACC_ERR_INVALID_ARG, "n must be >= 0");
    if (!dA || !dB || !dC || !dResult || (n > 0 && !dX)) return fail(ACC_ERR_INVALID_ARG, "NULL device pointer");
    if (((uintptr_t)dA | (uintptr_t)dB | (uintptr_t)dC | (uintptr_t)dX | (uintptr_t)dResult) & 3u)
        return fail(ACC_ERR_INVALID_ARG, "device pointers must be 4-byte aligned");
    if ((s = launch_fault()) != ACC_OK) return s;
    const GemmShape sh = accx::square_shape(len);
    const MatRedPlan p = matred_plan(sh, flags, n, n > 0 ? dX : nullptr);
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    if (dWork) {
        if ((s = check_work_align(dWork)) != ACC_OK) return s;
        if (work_bytes < p.total) return fail(ACC_ERR_INVALID_ARG, "workspace too small");
    } else {
        Workspace &w = st.mm_ws[stream];
        if ((s = ws_reserve(w, p.total, false, stream)) != ACC_OK) return s;
        dWork = w.ptr;
        work_bytes = w.bytes;
    }
    char *work = static_cast<char *>(dWork);
    if (!p.fused) {
        if ((s = run_matmul(ACC_FLOAT32, dA, dB, dC, sh, flags, work, p.mm, stream)) != ACC_OK) return s;
        return check_launch(accx::launch_reduce_f32(dX, n, init, dResult, work + p.red_off, false, stream),
                            "reduction launch");
    }
    auto *part = reinterpret_cast<uint32_t *>(work + p.red_off);
    const CoReduce red{dX, n, part, p.parts, init, dResult};
    return run_tiled_f32(dA, dB, dC, sh, flags, work, p.mm, stream, &red);
}

acc_status accx_onbox_mfma(int kind, int64_t rounds, double *ops_out, void *hip_stream)
{
    std::lock_guard<std::recursive_mutex> lk(S().mu);
    acc_status s = check_ready();
    if (s != ACC_OK) return s;
    if ((kind != 0 && kind != 1) || rounds < 1 || rounds > ((int64_t)1 << 30) || !ops_out)
        return fail(ACC_ERR_INVALID_ARG, "kind must be 0 or 1, rounds in [1, 2^30], ops_out non-NULL");
    return check_launch(accx::launch_onbox_mfma(kind, rounds, ops_out, static_cast<hipStream_t>(hip_stream)),
                        "matrix-instruction loop launch");
}

acc_status accx_onbox_read(const void *dX, int64_t bytes, void *hip_stream)
{
    std::lock_guard<std::recursive_mutex> lk(S().mu);
    acc_status s = check_ready();
    if (s != ACC_OK) return s;
    if (!dX || bytes <= 0 || (bytes & 15) || ((uintptr_t)dX & 15))
        return fail(ACC_ERR_INVALID_ARG, "dX must be 16-byte aligned and bytes a positive multiple of 16");
    return check_launch(accx::launch_onbox_read(dX, bytes, static_cast<hipStream_t>(hip_stream)),
                        "read stream launch");
}

acc_status accx_reduce_dev_noalloc(acc_dtype t, const void *dX, int64_t n, const acc_reduce_var *vars, int nvars,
                                   const void *init, void *dResult, uint32_t flags, void *hip_stream)
{
    State &st = S();
    std::lock_guard<std::recursive_mutex> lk(st.mu);
    acc_status s = dev_reduce_args(t, dX, n, vars, nvars, init, dResult, flags);
    if (s != ACC_OK) return s;
    const size_t need = vars_ws_bytes(t, n, vars, nvars, flags);
    if (need > accx::NOALLOC_SCRATCH_BYTES)
        return fail(ACC_ERR_INVALID_ARG, "the reduction needs " + std::to_string(need) +
                                             " bytes of scratch; the static scratch holds " +
                                             std::to_string(accx::NOALLOC_SCRATCH_BYTES) +
                                             " (ACC_REDUCE_PLAIN: n <= 8388608)");
    void *scratch = accx::noalloc_scratch(st.device);
    if (!scratch) return fail(ACC_ERR_DEVICE, "static reduction scratch has no device address");
    return run_reduce_vars(t, dX, n, vars, nvars, init, dResult, flags, scratch, static_cast<hipStream_t>(hip_stream));
}

namespace {
acc_status probe_layout(const GemmShape &sh, uint32_t flags, size_t *offset_out, int *count_out)
{
    if (!offset_out || !count_out) return fail(ACC_ERR_INVALID_ARG, "NULL output");
    acc_status s = validate_gemm(ACC_FLOAT32, sh, flags);
    if (s != ACC_OK) return s;
    if (is_plain(flags) || (flags & ACC_PREC_MASK) != ACC_PREC_AUTO)
        return fail(ACC_ERR_INVALID_ARG, "the probe runs only for the tiled kernel with ACC_PREC_AUTO");
    if (sh.m == 0 || sh.n == 0) return fail(ACC_ERR_INVALID_ARG, "an empty result has no probe records");
    const int tile = resolve_tile(ACC_FLOAT32, sh, (flags & ~ACC_PREC_MASK) | ACC_PREC_CHEAP3, 0);
    *offset_out = probe_offset(sh);
    *count_out = accx::probe_tiles(tile, sh.m, sh.n);
    return ACC_OK;
}
}  // namespace

acc_status accx_probe_layout(int64_t len, uint32_t flags, size_t *offset_out, int *count_out)
{
    std::lock_guard<std::recursive_mutex> lk(S().mu);
    acc_status s = validate_matmul(ACC_FLOAT32, len, flags);
    if (s != ACC_OK) return s;
    return probe_layout(accx::square_shape(len), flags, offset_out, count_out);
}

acc_status accx_gemm_probe_layout(int64_t m, int64_t n, int64_t k, uint32_t flags, size_t *offset_out, int *count_out)
{
    std::lock_guard<std::recursive_mutex> lk(S().mu);
    return probe_layout(GemmShape{m, n, k, std::max<int64_t>(1, k), std::max<int64_t>(1, n), std::max<int64_t>(1, n)},
                        flags, offset_out, count_out);
}

acc_status accx_packed_size(acc_dtype t, int64_t rows, int64_t k, int planes, size_t *bytes_out)
{
    if (!bytes_out) return fail(ACC_ERR_INVALID_ARG, "bytes_out is NULL");
    if (!matmul_dtype(t)) return fail(ACC_ERR_INVALID_ARG, "dtype must be ACC_FLOAT32 or ACC_INT32");
    if (rows < 1 || k < 1 || rows > 65536 || k > 65536) return fail(ACC_ERR_INVALID_ARG, "rows and k in [1, 65536]");
    if (t == ACC_FLOAT32 ? planes != 3 : (planes < 1 || planes > 4))
        return fail(ACC_ERR_INVALID_ARG, "planes: 3 for float32, 1..4 for int32");
    *bytes_out = accx::packed_bytes(rows, k, t == ACC_FLOAT32 ? 2 : 1, planes);
    return ACC_OK;
}

acc_status accx_pack_dev(acc_dtype t, const void *dX, int64_t rows, int64_t k, int transposed, int planes, void *dOut,
                         size_t out_bytes, void *hip_stream)
{
    State &st = S();
    std::lock_guard<std::recursive_mutex> lk(st.mu);
    acc_status s = check_ready();
    if (s != ACC_OK) return s;
    size_t need = 0;
    if ((s = accx_packed_size(t, rows, k, planes, &need)) != ACC_OK) return s;
    if (!dX || !dOut) return fail(ACC_ERR_INVALID_ARG, "NULL device pointer");
    if (out_bytes < need) return fail(ACC_ERR_INVALID_ARG, "output buffer too small");
    if ((uintptr_t)dX & 3u) return fail(ACC_ERR_INVALID_ARG, "dX must be 4-byte aligned");
    if ((uintptr_t)dOut & 15u) return fail(ACC_ERR_INVALID_ARG, "dOut must be 16-byte aligned");
    if ((s = launch_fault()) != ACC_OK) return s;
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    const hipError_t e =
        (t == ACC_FLOAT32)
            ? accx::launch_pack_bf16x3(static_cast<const float *>(dX), rows, k, transposed ? rows : k,
                                       transposed != 0, dOut, stream)
            : accx::launch_pack_i8(static_cast<const int32_t *>(dX), rows, k, transposed ? rows : k, transposed != 0,
                                   planes, dOut, stream);
    return check_launch(e, "pack launch");
}

// Time the tile configurations in `mask` (bit i = tile i) and record the
// fastest in the table of `family` (0: standalone kernels, 1: batch kernel).
}  // extern "C"

namespace {
acc_status autotune_impl(int t, const GemmShape &sh, uint32_t flags, unsigned mask, int family, int *best_out,
                         double *ms_out)
{
    acc_status s = ACC_OK;
    const int limbs = (t == ACC_INT32) ? (flag_limbs(flags) ? flag_limbs(flags) : 1) : 0;
    // one scratch input serves as A (m x k) and as B (k x n)
    const int64_t xel = std::max<int64_t>(1, std::max(sh.m * sh.k, sh.k * sh.n));
    const size_t xbytes = (size_t)xel * 4, cbytes = (size_t)std::max<int64_t>(1, sh.m * sh.n) * 4;
    const bool f32mm = t == ACC_FLOAT32 && is_f32mm(flags);
    const int eb = kelem_bytes(t, flags), planes = t == ACC_INT32 ? limbs : f32mm ? 1 : 3;
    const size_t pka = accx::packed_bytes(sh.m, sh.k, eb, planes);
    const size_t pk2b = std::max<size_t>(256, pka + accx::packed_bytes(sh.n, sh.k, eb, planes));
    // each candidate runs with the split K the library would give it
    const int64_t nkb = (sh.k * eb + 63) / 64;
    size_t splitb = 0;
    for (int tile = 1; tile < accx::GEMM_TILE_COUNT; ++tile)
        if (limbs <= 1)
            splitb = std::max(splitb, accx::split_k_bytes(tile, sh.m, sh.n, accx::split_k_parts(tile, sh.m, sh.n, nkb)));
    void *spl = nullptr;
    void *x = nullptr, *c = nullptr, *pk2 = nullptr;
    hipStream_t stream = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int best = 0;
    double best_ms = 1e300;
    hipError_t he = hipSuccess;
    if ((s = dev_alloc(&x, xbytes)) != ACC_OK) goto out;
    if ((s = dev_alloc(&c, cbytes)) != ACC_OK) goto out;
    if ((s = dev_alloc(&pk2, pk2b)) != ACC_OK) goto out;
    if (splitb && (s = dev_alloc(&spl, splitb)) != ACC_OK) goto out;
    if ((he = hipStreamCreateWithFlags(&stream, hipStreamNonBlocking)) != hipSuccess) goto hip_out;
    if ((he = hipEventCreate(&e0)) != hipSuccess || (he = hipEventCreate(&e1)) != hipSuccess) goto hip_out;
    // Operands: hashed uniform values, float in [-1, 1) or int in [-16, 16]
    // (one limb); constant operands run the matrix cores at a higher clock
    // than real data and would mislead the choice.
    if ((he = accx::launch_fill_hash(x, xel, t == ACC_INT32, stream)) != hipSuccess) goto hip_out;
    if (f32mm) {
        he = accx::launch_pack_f32(static_cast<float *>(x), sh.m, sh.k, sh.k, false, pk2, stream);
        if (he == hipSuccess)
            he = accx::launch_pack_f32(static_cast<float *>(x), sh.n, sh.k, sh.n, true, static_cast<char *>(pk2) + pka,
                                       stream);
    } else if (t == ACC_FLOAT32) {
        he = accx::launch_pack_bf16x3(static_cast<float *>(x), sh.m, sh.k, sh.k, false, pk2, stream);
        if (he == hipSuccess)
            he = accx::launch_pack_bf16x3(static_cast<float *>(x), sh.n, sh.k, sh.n, true,
                                          static_cast<char *>(pk2) + pka, stream);
    } else {
        he = accx::launch_pack_i8(static_cast<int32_t *>(x), sh.m, sh.k, sh.k, false, limbs, pk2, stream);
        if (he == hipSuccess)
            he = accx::launch_pack_i8(static_cast<int32_t *>(x), sh.n, sh.k, sh.n, true, limbs,
                                      static_cast<char *>(pk2) + pka, stream);
    }
    if (he != hipSuccess) goto hip_out;
    {
        // Round-robin over the candidates, several rounds, best per-call time
        // of each: the first rounds also bring the clocks to their loaded
        // steady state, so no candidate is timed alone on a cold device.
        const GemmShape csh{sh.m, sh.n, sh.k, sh.k, sh.n, sh.n};
        auto run = [&](int tile) {
            accx::SplitK sk;
            if (limbs <= 1) {
                sk.parts = accx::split_k_parts(tile, sh.m, sh.n, nkb);
                sk.work = spl;
            }
            if (f32mm)
                return accx::launch_gemm_f32mm(pk2, static_cast<char *>(pk2) + pka, static_cast<float *>(c), csh,
                                               tile, stream, sk);
            return (t == ACC_FLOAT32)
                       ? accx::launch_gemm_bf16x3(pk2, static_cast<char *>(pk2) + pka, static_cast<float *>(c), csh,
                                                  tune_variant(t, flags, 0), false, tile, stream, nullptr, sk)
                       : accx::launch_gemm_i8(pk2, static_cast<char *>(pk2) + pka, static_cast<int32_t *>(c), csh,
                                              limbs, tile, stream, nullptr, 0, sk);
        };
        const double work = std::max(1.0, 2.0 * (double)sh.m * (double)sh.n * (double)sh.k);
        const int reps = (int)std::max<double>(2.0, std::min<double>(50.0, 2e11 / work));
        // The clock drifts up over the first rounds: the order alternates
        // (forward, backward) so that no candidate is always timed later.
        const int rounds = 5;
        std::vector<double> per(accx::GEMM_TILE_COUNT, 1e300);
        for (int r = 0; r < rounds; ++r) {
            for (int q = 1; q < accx::GEMM_TILE_COUNT; ++q) {
                const int tile = (r & 1) ? accx::GEMM_TILE_COUNT - q : q;
                if (!(mask & (1u << tile))) continue;
                if (limbs > 1 && tile != accx::GEMM_TILE_64) continue;  // several limbs: small tile only
                if ((he = run(tile)) != hipSuccess) goto hip_out;
                if ((he = hipEventRecord(e0, stream)) != hipSuccess) goto hip_out;
                for (int k = 0; k < reps && he == hipSuccess; ++k) he = run(tile);
                if (he != hipSuccess) goto hip_out;
                if ((he = hipEventRecord(e1, stream)) != hipSuccess || (he = hipEventSynchronize(e1)) != hipSuccess)
                    goto hip_out;
                float ms = 0;
                if ((he = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) goto hip_out;
                if (r > 0) per[tile] = std::min(per[tile], (double)ms / reps);  // round 0 warms up
            }
        }
        // the fastest, except that a candidate earlier in the fixed order
        // within 2 % of it wins: tiles that differ less than the clock's
        // drift between boxes would otherwise change from run to run
        double fastest = 1e300;
        for (int tile = 1; tile < accx::GEMM_TILE_COUNT; ++tile) fastest = std::min(fastest, per[tile]);
        for (int tile = 1; tile < accx::GEMM_TILE_COUNT && fastest < 1e300; ++tile)
            if (per[tile] <= fastest * 1.02) {
                best = tile;
                best_ms = per[tile];
                break;
            }
    }
    tune_table()[tune_key(t, tune_variant(t, flags, limbs) + 100 * family, sh)] = TuneEntry{best, best_ms};
    if (best_out) *best_out = best;
    if (ms_out) *ms_out = best_ms;
    goto out;
hip_out:
    s = fail_hip(he, "autotune");
out:
    if (stream) (void)hipStreamSynchronize(stream);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (stream) (void)hipStreamDestroy(stream);
    dev_free(x, xbytes);
    dev_free(c, cbytes);
    dev_free(pk2, pk2b);
    dev_free(spl, splitb);
    return s;
}

}  // namespace

extern "C" {

acc_status accx_autotune(acc_dtype t, int64_t len, uint32_t flags, uint32_t *best_tile_out, double *ms_out)
{
    State &st = S();
    std::lock_guard<std::recursive_mutex> lk(st.mu);
    acc_status s = check_ready();
    if (s != ACC_OK) return s;
    if ((s = validate_matmul(t, len, flags)) != ACC_OK) return s;
    return accx_autotune_gemm(t, len, len, len, flags, best_tile_out, ms_out);
}

acc_status accx_autotune_gemm(acc_dtype t, int64_t m, int64_t n, int64_t k, uint32_t flags, uint32_t *best_tile_out,
                              double *ms_out)
{
    State &st = S();
    std::lock_guard<std::recursive_mutex> lk(st.mu);
    acc_status s = check_ready();
    if (s != ACC_OK) return s;
    const GemmShape sh{m, n, k, std::max<int64_t>(1, k), std::max<int64_t>(1, n), std::max<int64_t>(1, n)};
    if ((s = validate_gemm(t, sh, flags)) != ACC_OK) return s;
    if (m == 0 || n == 0 || k == 0) return fail(ACC_ERR_INVALID_ARG, "autotune needs m, n, k >= 1");
    int best = 0;
    if ((s = autotune_impl(t, sh, flags, ~0u, 0, &best, ms_out)) != ACC_OK) return s;
    if (best_tile_out) *best_tile_out = (uint32_t)best << ACC_TILE_SHIFT;
    return ACC_OK;
}

acc_status accx_tune_save(const char *path)
{
    State &st = S();
    std::lock_guard<std::recursive_mutex> lk(st.mu);
    if (!path) return fail(ACC_ERR_INVALID_ARG, "path is NULL");
    FILE *f = std::fopen(path, "w");
    if (!f) return fail(ACC_ERR_INVALID_ARG, std::string("cannot write ") + path);
    for (const auto &kv : tune_table())
        std::fprintf(f, "%d %d %d %d %d %d %.6f\n", std::get<0>(kv.first), std::get<1>(kv.first), std::get<2>(kv.first),
                     std::get<3>(kv.first), std::get<4>(kv.first), kv.second.tile, kv.second.ms);
    std::fclose(f);
    return ACC_OK;
}

acc_status accx_tune_load(const char *path)
{
    State &st = S();
    std::lock_guard<std::recursive_mutex> lk(st.mu);
    if (!path) return fail(ACC_ERR_INVALID_ARG, "path is NULL");
    FILE *f = std::fopen(path, "r");
    if (!f) return fail(ACC_ERR_INVALID_ARG, std::string("cannot read ") + path);
    // lines "dtype variant cm cn ck tile ms", or "dtype variant c tile ms"
    // for a square size class (m, n, k all in class c)
    acc_status s = ACC_OK;
    char line[256];
    while (std::fgets(line, sizeof line, f)) {
        std::vector<std::string> tok;
        for (char *p = std::strtok(line, " \t\r\n"); p; p = std::strtok(nullptr, " \t\r\n")) tok.emplace_back(p);
        if (tok.empty()) continue;
        std::vector<long> iv;
        double ms = 0;
        bool ok = tok.size() == 7 || tok.size() == 5;
        for (size_t q = 0; ok && q + 1 < tok.size(); ++q) {
            char *end = nullptr;
            iv.push_back(std::strtol(tok[q].c_str(), &end, 10));
            ok = end && *end == '\0';
        }
        if (ok) {
            char *end = nullptr;
            ms = std::strtod(tok.back().c_str(), &end);
            ok = end && *end == '\0';
        }
        if (!ok) {
            s = fail(ACC_ERR_INVALID_ARG, "malformed tune table");
            break;
        }
        const bool sq = tok.size() == 5;
        const TuneKey key{(int)iv[0], (int)iv[1], (int)iv[2], (int)iv[sq ? 2 : 3], (int)iv[sq ? 2 : 4]};
        const int tile = (int)iv[sq ? 3 : 5];
        const int cm = std::get<2>(key), cn = std::get<3>(key), ck = std::get<4>(key);
        if (!matmul_dtype(std::get<0>(key)) || tile < 1 || tile >= accx::GEMM_TILE_COUNT || cm < 0 || cm > 17 ||
            cn < 0 || cn > 17 || ck < 0 || ck > 16) {
            s = fail(ACC_ERR_INVALID_ARG, "bad tune table entry");
            break;
        }
        tune_table()[key] = TuneEntry{tile, ms};
    }
    std::fclose(f);
    return s;
}

const char *acc_status_string(acc_status s)
{
    switch (s) {
    case ACC_OK: return "ACC_OK";
    case ACC_ERR_INVALID_ARG: return "ACC_ERR_INVALID_ARG";
    case ACC_ERR_NOT_PRESENT: return "ACC_ERR_NOT_PRESENT";
    case ACC_ERR_ALREADY_PRESENT: return "ACC_ERR_ALREADY_PRESENT";
    case ACC_ERR_OUT_OF_MEMORY: return "ACC_ERR_OUT_OF_MEMORY";
    case ACC_ERR_DEVICE: return "ACC_ERR_DEVICE";
    case ACC_ERR_NO_DEVICE: return "ACC_ERR_NO_DEVICE";
    default: break;
    }
    return "unknown acc_status";
}

const char *acc_last_error_string(void) { return t_last_error.c_str(); }

const char *accx_version(void) { return "libaccx 0.1 (gfx950)"; }

}  // extern "C"

// =========================================================================
// Entry points for the serving engine (serve.cpp); see runtime_internal.h.
namespace accx {
namespace rt {
acc_status fail(acc_status s, const std::string &msg) { return ::fail(s, msg); }
acc_status fail_hip(hipError_t e, const char *what) { return ::fail_hip(e, what); }
acc_status ready() { return check_ready(); }
acc_status check_matmul(int t, int64_t len, uint32_t flags) { return validate_matmul(t, len, flags); }
acc_status check_reduce(int t, int64_t n, uint32_t flags)
{
    if (!matmul_dtype(t)) return ::fail(ACC_ERR_INVALID_ARG, "served reductions are float32 or int32 sums");
    return validate_reduce(t, n, flags);
}
size_t matmul_workspace(int t, int64_t len, uint32_t flags)
{
    return matmul_ws_bytes(t, accx::square_shape(len), flags);
}
size_t reduce_workspace(int64_t n, uint32_t flags) { return reduce_ws_bytes(n, flags); }
acc_status matmul(int t, const void *a, const void *b, void *c, int64_t len, uint32_t flags, void *work,
                  size_t work_bytes, hipStream_t s)
{
    return run_matmul(t, a, b, c, accx::square_shape(len), flags, work, work_bytes, s);
}
acc_status reduce(int t, const void *x, int64_t n, const void *init, void *result, uint32_t flags, void *work,
                  hipStream_t s)
{
    return run_reduce(t, x, n, init, result, flags, work, s);
}
std::recursive_mutex &lock() { return S().mu; }
acc_status device_alloc(void **p, size_t bytes)
{
    std::lock_guard<std::recursive_mutex> lk(S().mu);
    return raw_alloc(p, bytes);
}
void device_free(void *p)
{
    std::lock_guard<std::recursive_mutex> lk(S().mu);
    raw_free(p);
}
}  // namespace rt
}  // namespace accx

// =========================================================================
// Batched launch: plan, graph, launch.

struct accx_batch_s {
    void *dev = nullptr;  // one allocation: descriptors, queue, counters, partials, packed operands
    size_t dev_bytes = 0;
    accx::BatchQueue queue{};
    accx::BatchPackJob *jobs = nullptr;  // device
    int njobs = 0;
    uint32_t *job_of = nullptr;          // device: the job of each pack workgroup
    int64_t pack_wgs = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    accx_batch_info_t info{};
};

namespace {

constexpr int64_t kReduceChunk = 1 << 17;  // elements per reduction work unit

std::set<accx_batch_s *> &batches()
{
    static auto *b = new std::set<accx_batch_s *>();
    return *b;
}

// Tile policy of a batch: an item's forced tile, else 128 x 128 when its
// LEN is at least `threshold`, else 64 x 64.
int batch_tile(const accx_batch_item &it, int64_t threshold)
{
    const int forced = (int)((it.flags & ACC_TILE_MASK) >> ACC_TILE_SHIFT);
    if (forced) return forced;
    return it.n >= threshold ? accx::GEMM_TILE_128 : accx::GEMM_TILE_64;
}

constexpr int64_t kBatchDefaultThreshold = 512;

// Work queue for the given tiles: matmul tiles, largest matmul first, with
// the reduction chunks spread evenly through it by cumulative cost, so that
// both kinds of work are in flight throughout.
std::vector<accx::BatchUnit> batch_units(std::vector<accx::BatchMat> &mats, const std::vector<accx::BatchRed> &reds)
{
    std::vector<int> order(mats.size());
    for (size_t k = 0; k < order.size(); ++k) order[k] = (int)k;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return mats[x].len > mats[y].len; });
    std::vector<std::pair<double, accx::BatchUnit>> mu, ru;
    double mtot = 0, rtot = 0;
    for (int k : order) {
        accx::BatchMat &m = mats[k];
        const int bm = m.tile == accx::GEMM_TILE_128 ? 128 : 64;
        m.tiles_m = m.tiles_n = (int32_t)((m.len + bm - 1) / bm);
        for (int t = 0; t < m.tiles_m * m.tiles_n; ++t) {
            mu.push_back({mtot, accx::BatchUnit{(uint32_t)k, (uint32_t)t}});
            mtot += (double)bm * bm * (double)m.len;
        }
    }
    for (size_t k = 0; k < reds.size(); ++k)
        for (int32_t c = 0; c < reds[k].nchunks; ++c) {
            ru.push_back({rtot, accx::BatchUnit{(uint32_t)k | 0x80000000u, (uint32_t)c}});
            rtot += (double)std::min<int64_t>(reds[k].chunk, std::max<int64_t>(0, reds[k].n - c * reds[k].chunk));
        }
    std::vector<accx::BatchUnit> units;
    units.reserve(mu.size() + ru.size());
    size_t im = 0, ir = 0;
    while (im < mu.size() || ir < ru.size()) {
        const double fm = im < mu.size() ? (mtot > 0 ? mu[im].first / mtot : 0) : 2.0;
        const double fr = ir < ru.size() ? (rtot > 0 ? ru[ir].first / rtot : 0) : 2.0;
        if (fm <= fr)
            units.push_back(mu[im++].second);
        else
            units.push_back(ru[ir++].second);
    }
    return units;
}

void batch_destroy_all()
{
    for (accx_batch_s *b : batches()) {
        batch_release(b);
        delete b;
    }
    batches().clear();
}

void batch_release(accx_batch_s *b)
{
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->dev) dev_free(b->dev, b->dev_bytes);
    b->exec = nullptr;
    b->graph = nullptr;
    b->dev = nullptr;
}

hipError_t batch_enqueue(accx_batch_s *b, hipStream_t s)
{
    hipError_t e = accx::launch_batch_pack(b->jobs, b->job_of, b->pack_wgs, s);
    if (e == hipSuccess) e = accx::launch_batch_persistent(b->queue, s);
    return e;
}

}  // namespace

extern "C" {

acc_status accx_batch_create(const accx_batch_item *items, int nitems, uint32_t flags, accx_batch *out)
{
    State &st = S();
    std::lock_guard<std::recursive_mutex> lk(st.mu);
    if (!out) return fail(ACC_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    acc_status s = check_ready();
    if (s != ACC_OK) return s;
    if (nitems <= 0 || !items) return fail(ACC_ERR_INVALID_ARG, "empty batch");
    if (flags & ~(ACC_BATCH_AUTOTUNE | ACC_BATCH_PREC_AUTO)) return fail(ACC_ERR_INVALID_ARG, "unknown batch flag");
    const bool auto_prec = (flags & ACC_BATCH_PREC_AUTO) != 0;
    const int products = auto_prec ? 3 : 6;

    std::vector<accx::BatchMat> mats;
    std::vector<accx::BatchRed> reds;
    std::vector<int> mat_item;
    std::vector<int64_t> red_chunks;
    std::vector<size_t> pk_bytes;
    accx_batch_info_t info{};
    int64_t max_tiles = 0;  // queue bound over every tile policy (all 64 x 64)
    for (int i = 0; i < nitems; ++i) {
        const accx_batch_item &it = items[i];
        const std::string where = "item " + std::to_string(i) + ": ";
        if (it.dtype != ACC_FLOAT32) return fail(ACC_ERR_INVALID_ARG, where + "batches hold float32 items");
        if (it.kind == ACC_BATCH_MATMUL) {
            if (it.n < 1 || it.n > 65536) return fail(ACC_ERR_INVALID_ARG, where + "LEN must be in [1, 65536]");
            if (!it.a || !it.b || !it.c) return fail(ACC_ERR_INVALID_ARG, where + "NULL pointer");
            if (((uintptr_t)it.a | (uintptr_t)it.b | (uintptr_t)it.c) & 3u)
                return fail(ACC_ERR_INVALID_ARG, where + "pointers must be 4-byte aligned");
            if (it.flags & ~ACC_TILE_MASK) return fail(ACC_ERR_INVALID_ARG, where + "only tile bits allowed");
            const int forced = (int)((it.flags & ACC_TILE_MASK) >> ACC_TILE_SHIFT);
            if (forced && !accx::batch_tile_supported(forced))
                return fail(ACC_ERR_INVALID_ARG, where + "batches run ACC_TILE_128 or ACC_TILE_64");
            accx::BatchMat m{};
            m.c = static_cast<float *>(it.c);
            m.len = it.n;
            m.nkb = (it.n * 2 + 63) / 64;
            m.tile = batch_tile(it, kBatchDefaultThreshold);
            m.products = products;
            mats.push_back(m);
            mat_item.push_back(i);
            pk_bytes.push_back(accx::packed_bytes(it.n, it.n, 2, 3));
            max_tiles += ((it.n + 63) / 64) * ((it.n + 63) / 64);
            info.flops += 2.0 * (double)it.n * (double)it.n * (double)it.n;
            info.mfma_flops += products * 2.0 * (double)it.n * (double)it.n * (double)it.n;
        } else if (it.kind == ACC_BATCH_REDUCE) {
            if (it.n < 0) return fail(ACC_ERR_INVALID_ARG, where + "n must be >= 0");
            if ((it.n > 0 && !it.a) || !it.c) return fail(ACC_ERR_INVALID_ARG, where + "NULL pointer");
            if (((uintptr_t)it.a | (uintptr_t)it.c) & 3u)
                return fail(ACC_ERR_INVALID_ARG, where + "pointers must be 4-byte aligned");
            if (it.flags) return fail(ACC_ERR_INVALID_ARG, where + "reductions take no flags");
            accx::BatchRed r{};
            r.x = static_cast<const float *>(it.a);
            r.result = static_cast<float *>(it.c);
            r.n = it.n;
            r.chunk = kReduceChunk;
            r.nchunks = (int32_t)std::max<int64_t>(1, (it.n + kReduceChunk - 1) / kReduceChunk);
            r.init = it.init;
            reds.push_back(r);
            red_chunks.push_back(r.nchunks);
            info.chunks += r.nchunks;
            info.reduce_bytes += 4.0 * (double)it.n;
        } else {
            return fail(ACC_ERR_INVALID_ARG, where + "unknown kind");
        }
    }
    if (max_tiles + info.chunks >= (int64_t)0x7fffffff) return fail(ACC_ERR_INVALID_ARG, "batch too large");
    std::vector<accx::BatchUnit> units = batch_units(mats, reds);
    const size_t max_units = (size_t)(max_tiles + info.chunks);

    // Device layout.
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    size_t off = 0;
    const size_t o_mats = off;
    off = al(off + sizeof(accx::BatchMat) * std::max<size_t>(1, mats.size()));
    const size_t o_reds = off;
    off = al(off + sizeof(accx::BatchRed) * std::max<size_t>(1, reds.size()));
    const size_t o_units = off;
    off = al(off + sizeof(accx::BatchUnit) * std::max<size_t>(1, max_units));
    const size_t o_jobs = off;
    off = al(off + sizeof(accx::BatchPackJob) * std::max<size_t>(1, 2 * mats.size()));
    // pack workgroups: A and B^T of matmul k get batch_pack_workgroups each
    int64_t pack_wgs = 0;
    for (size_t k = 0; k < mats.size(); ++k)
        pack_wgs += 2 * (int64_t)accx::batch_pack_workgroups((mats[k].len + 31) / 32, mats[k].nkb);
    const size_t o_jobof = off;
    off = al(off + sizeof(uint32_t) * (size_t)std::max<int64_t>(1, pack_wgs));
    const size_t o_zero = off;  // counters, tickets, partials: zero-filled
    size_t zbytes = 256;
    for (size_t k = 0; k < reds.size(); ++k) zbytes += 4 + 4 * (size_t)reds[k].nchunks;
    off = al(off + zbytes);
    const size_t o_pack = off;
    for (size_t k = 0; k < mats.size(); ++k) off = al(off + 2 * pk_bytes[k]);

    accx_batch_s *b = new (std::nothrow) accx_batch_s();
    if (!b) return fail(ACC_ERR_OUT_OF_MEMORY, "host allocation failed");
    if ((s = dev_alloc(&b->dev, off)) != ACC_OK) {
        delete b;
        return s;
    }
    b->dev_bytes = off;
    char *base = static_cast<char *>(b->dev);
    std::vector<accx::BatchPackJob> jobs;
    std::vector<uint32_t> job_of;
    job_of.reserve((size_t)pack_wgs);
    {
        size_t p = o_pack;
        for (size_t k = 0; k < mats.size(); ++k) {
            const accx_batch_item &it = items[mat_item[k]];
            char *pa = base + p, *pb = base + p + pk_bytes[k];
            p = al(p + 2 * pk_bytes[k]);
            mats[k].pa = pa;
            mats[k].pb = pb;
            const int64_t nrb = (it.n + 31) / 32;
            const int nwg = accx::batch_pack_workgroups(nrb, mats[k].nkb);
            for (int t = 0; t < 2; ++t) {
                jobs.push_back(accx::BatchPackJob{static_cast<const float *>(t ? it.b : it.a), t ? pb : pa, it.n,
                                                  it.n, it.n, nrb, mats[k].nkb, t, nwg, (uint32_t)job_of.size(), 0});
                job_of.insert(job_of.end(), (size_t)nwg, (uint32_t)(jobs.size() - 1));
            }
        }
        uint32_t *z = reinterpret_cast<uint32_t *>(base + o_zero);
        size_t w = 64;  // counter at word 0, done at word 1
        for (size_t k = 0; k < reds.size(); ++k) {
            reds[k].ticket = z + w;
            reds[k].partials = z + w + 1;
            w += 1 + (size_t)reds[k].nchunks;
        }
        b->queue.counter = z;
        b->queue.done = z + 1;
    }
    b->queue.auto_prec = auto_prec ? 1 : 0;
    b->queue.tau2 = probe_tau() * probe_tau();
    b->queue.mats = reinterpret_cast<const accx::BatchMat *>(base + o_mats);
    b->queue.reds = reinterpret_cast<const accx::BatchRed *>(base + o_reds);
    b->queue.units = reinterpret_cast<const accx::BatchUnit *>(base + o_units);
    b->queue.nunits = (uint32_t)units.size();
    b->jobs = reinterpret_cast<accx::BatchPackJob *>(base + o_jobs);
    b->njobs = (int)jobs.size();
    b->job_of = reinterpret_cast<uint32_t *>(base + o_jobof);
    b->pack_wgs = (int64_t)job_of.size();
    if (b->pack_wgs != pack_wgs || pack_wgs >= ((int64_t)1 << 31)) {  // the layout's count, and one launch's grid
        dev_free(b->dev, b->dev_bytes);
        delete b;
        return fail(ACC_ERR_INVALID_ARG, "batch too large");
    }

    hipError_t e = hipSuccess;
    hipStream_t cs = nullptr;
    if (!mats.empty()) e = hipMemcpy(base + o_mats, mats.data(), sizeof(accx::BatchMat) * mats.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess && !reds.empty())
        e = hipMemcpy(base + o_reds, reds.data(), sizeof(accx::BatchRed) * reds.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess && !units.empty())
        e = hipMemcpy(base + o_units, units.data(), sizeof(accx::BatchUnit) * units.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess && !jobs.empty())
        e = hipMemcpy(base + o_jobs, jobs.data(), sizeof(accx::BatchPackJob) * jobs.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess && !job_of.empty())
        e = hipMemcpy(base + o_jobof, job_of.data(), sizeof(uint32_t) * job_of.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(base + o_zero, 0, zbytes);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    int64_t threshold = kBatchDefaultThreshold;
    if (e == hipSuccess && (flags & ACC_BATCH_AUTOTUNE) && !mats.empty()) {
        // Autotune the tile policy on this batch itself: pack once, then time
        // the persistent kernel under each LEN threshold between the 64 x 64
        // and 128 x 128 tiles (best of two runs after a warm-up run each).
        e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (e == hipSuccess) e = hipEventCreate(&e0);
        if (e == hipSuccess) e = hipEventCreate(&e1);
        if (e == hipSuccess) e = accx::launch_batch_pack(b->jobs, b->job_of, b->pack_wgs, cs);
        double best = 1e300;
        const int64_t cand[] = {0, 192, 320, 448, 576, 768, 65537};
        for (int64_t th : cand) {
            if (e != hipSuccess) break;
            for (size_t k = 0; k < mats.size(); ++k) mats[k].tile = batch_tile(items[mat_item[k]], th);
            std::vector<accx::BatchUnit> u = batch_units(mats, reds);
            b->queue.nunits = (uint32_t)u.size();
            e = hipMemcpy(base + o_mats, mats.data(), sizeof(accx::BatchMat) * mats.size(), hipMemcpyHostToDevice);
            if (e == hipSuccess)
                e = hipMemcpy(base + o_units, u.data(), sizeof(accx::BatchUnit) * u.size(), hipMemcpyHostToDevice);
            double t_best = 1e300;
            for (int r = 0; r < 3 && e == hipSuccess; ++r) {
                e = hipEventRecord(e0, cs);
                if (e == hipSuccess) e = accx::launch_batch_persistent(b->queue, cs);
                if (e == hipSuccess) e = hipEventRecord(e1, cs);
                if (e == hipSuccess) e = hipEventSynchronize(e1);
                float ms = 0;
                if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
                if (r > 0) t_best = std::min(t_best, (double)ms);
            }
            if (t_best < best) {
                best = t_best;
                threshold = th;
            }
        }
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        if (cs) (void)hipStreamDestroy(cs);
        cs = nullptr;
        if (e == hipSuccess) {
            for (size_t k = 0; k < mats.size(); ++k) mats[k].tile = batch_tile(items[mat_item[k]], threshold);
            units = batch_units(mats, reds);
            b->queue.nunits = (uint32_t)units.size();
            e = hipMemcpy(base + o_mats, mats.data(), sizeof(accx::BatchMat) * mats.size(), hipMemcpyHostToDevice);
            if (e == hipSuccess)
                e = hipMemcpy(base + o_units, units.data(), sizeof(accx::BatchUnit) * units.size(),
                              hipMemcpyHostToDevice);
        }
    }
    for (const accx::BatchMat &m : mats) info.tiles += (int64_t)m.tiles_m * m.tiles_n;
    // Capture the two kernels into one graph (no memset node: the kernels
    // leave every counter at zero).
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        t_capturing = true;
        hipError_t le = batch_enqueue(b, cs);
        t_capturing = false;
        e = hipStreamEndCapture(cs, &b->graph);
        if (e == hipSuccess) e = le;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
    size_t nnodes = 0;
    if (e == hipSuccess) e = hipGraphGetNodes(b->graph, nullptr, &nnodes);
    if (cs) (void)hipStreamDestroy(cs);
    if (e != hipSuccess) {
        const acc_status fs = fail_hip(e, "batch setup");
        batch_release(b);
        delete b;
        return fs;
    }
    info.units = (int64_t)units.size();
    info.tile_threshold = threshold;
    info.workgroups = accx::batch_workgroups();
    info.matmuls = (int32_t)mats.size();
    info.reductions = (int32_t)reds.size();
    info.device_bytes = off;
    info.pad = (int32_t)nnodes;
    b->info = info;
    batches().insert(b);
    *out = b;
    return ACC_OK;
}

acc_status accx_batch_launch(accx_batch b, void *hip_stream)
{
    State &st = S();
    std::lock_guard<std::recursive_mutex> lk(st.mu);
    if (!b || !batches().count(b)) return fail(ACC_ERR_INVALID_ARG, "unknown batch");
    acc_status s = launch_fault();
    if (s != ACC_OK) return s;
    const hipError_t e = hipGraphLaunch(b->exec, static_cast<hipStream_t>(hip_stream));
    if (e != hipSuccess) return fail_hip(e, "hipGraphLaunch");
    return ACC_OK;
}

acc_status accx_batch_launch_eager(accx_batch b, void *hip_stream)
{
    State &st = S();
    std::lock_guard<std::recursive_mutex> lk(st.mu);
    if (!b || !batches().count(b)) return fail(ACC_ERR_INVALID_ARG, "unknown batch");
    acc_status s = launch_fault();
    if (s != ACC_OK) return s;
    return check_launch(batch_enqueue(b, static_cast<hipStream_t>(hip_stream)), "batch launch");
}

acc_status accx_batch_info(accx_batch b, accx_batch_info_t *out)
{
    State &st = S();
    std::lock_guard<std::recursive_mutex> lk(st.mu);
    if (!b || !batches().count(b) || !out) return fail(ACC_ERR_INVALID_ARG, "unknown batch or NULL output");
    *out = b->info;
    return ACC_OK;
}

acc_status accx_batch_destroy(accx_batch b)
{
    State &st = S();
    std::lock_guard<std::recursive_mutex> lk(st.mu);
    if (!b || !batches().count(b)) return fail(ACC_ERR_INVALID_ARG, "unknown batch");
    (void)hipDeviceSynchronize();
    batch_release(b);
    batches().erase(b);
    delete b;
    return ACC_OK;
}

}  // extern "C"

namespace accx {
int device_cu_count()
{
    static int cached = 0;
    if (cached) return cached;
    int dev = 0;
    (void)hipGetDevice(&dev);
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0) v = 256;
    cached = v;
    return v;
}
}  // namespace accx
