// Per-device resources shared by the data-set types of libptafs: a
// stream-ordered memory pool that keeps released blocks for reuse, and a
// library stream for work that no caller stream orders (tuning changes,
// reservation, release).
#pragma once

#include <hip/hip_runtime.h>

namespace ptr {
int device_pool(int dev, hipMemPool_t *pool, hipStream_t *aux);
}  // namespace ptr
