// Internal launch interface between the C-ABI runtime (runtime.cpp) and the
// HIP kernels (*.hip).  Not installed; the public ABI is include/accx.h.
#pragma once

#include <hip/hip_runtime_api.h>
#include <stddef.h>
#include <stdint.h>

namespace accx {

// ---- plain loop nest (Listing 1a/1b): one thread per output element -------
hipError_t launch_matmul_plain_f32(const float *a, const float *b, float *c, int64_t len,
                                   bool listing1b_mapping, hipStream_t s);
hipError_t launch_matmul_plain_i32(const int32_t *a, const int32_t *b, int32_t *c, int64_t len,
                                   bool listing1b_mapping, hipStream_t s);

// ---- reduction(+) ----------------------------------------------------------
// Fast: one pass, per-block partials, last block combines them in index order.
// Workspace: [0,256) ticket word (must start at zero, left at zero),
//            [256, 256 + 4*blocks) partials.
size_t reduce_fast_workspace_bytes(int64_t n);
// Plain: one element per thread and a block tree, then one block combines.
size_t reduce_plain_workspace_bytes(int64_t n);

hipError_t launch_reduce_f32(const float *x, int64_t n, float init, float *result, void *work,
                             bool plain, hipStream_t s);
hipError_t launch_reduce_i32(const int32_t *x, int64_t n, int32_t init, int32_t *result, void *work,
                             bool plain, hipStream_t s);

int device_cu_count();  // compute units of the current device (cached)

}  // namespace accx
