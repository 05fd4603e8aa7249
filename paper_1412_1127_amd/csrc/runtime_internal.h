// Internal entry points of the runtime (runtime.cpp) used by the serving
// engine (serve.cpp).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime_api.h>

#include <mutex>
#include <string>

#include "../../include/accx.h"

namespace accx {
namespace rt {
acc_status fail(acc_status s, const std::string &msg);  // sets the thread-local message
acc_status fail_hip(hipError_t e, const char *what);
acc_status ready();                                     // NO_DEVICE unless acc_init succeeded
acc_status check_matmul(int t, int64_t len, uint32_t flags);
acc_status check_reduce(int t, int64_t n, uint32_t flags);
size_t matmul_workspace(int t, int64_t len, uint32_t flags);
size_t reduce_workspace(int64_t n, uint32_t flags);
// Enqueue on stream s; device pointers; workspace as sized above (the fast
// reduction's workspace must be zero-filled once before first use).
acc_status matmul(int t, const void *a, const void *b, void *c, int64_t len, uint32_t flags, void *work,
                  size_t work_bytes, hipStream_t s);
acc_status reduce(int t, const void *x, int64_t n, const void *init, void *result, uint32_t flags, void *work,
                  hipStream_t s);
std::recursive_mutex &lock();  // the runtime's state lock
// Device memory from the allocator in effect (accx_set_allocator, else
// hipMalloc), not charged to the library's budget; device_free returns a
// block to the allocator that gave it.
acc_status device_alloc(void **p, size_t bytes);
void device_free(void *p);
}  // namespace rt
}  // namespace accx
