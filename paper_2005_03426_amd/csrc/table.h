// Per-problem parameter tables of the grouped eigensolver kernels (internal).
//
// Every eigensolver kernel reads its problem's sizes and buffers from a
// device array of small structs indexed by the problem number, so one launch
// advances the same step of many independent matrices.  The table is written
// by kernels that receive the entries by value (kernel arguments), so no host
// buffer has to outlive the call and nothing is copied from pageable memory.
#pragma once
#include "common.h"

namespace mmf {

template <class T, int K>
struct TableChunk {
  T v[K];
  int32_t count;
};

template <class T, int K>
__global__ void table_set(T *dst, TableChunk<T, K> c) {
  if ((int)threadIdx.x < c.count) dst[threadIdx.x] = c.v[threadIdx.x];
}

// Writes host entries [0, count) into the device table, as many entries per
// launch as fit in ARG_BYTES of kernel arguments (under 1 KiB by default;
// large per-problem tables take up to 3840 bytes, below the 4 KiB limit).
template <class T, int ARG_BYTES = 960>
inline int table_write(T *dev, const T *host, int64_t count, hipStream_t st) {
  constexpr int K = (ARG_BYTES / (int)sizeof(T)) > 0 ? (ARG_BYTES / (int)sizeof(T)) : 1;
  for (int64_t base = 0; base < count; base += K) {
    TableChunk<T, K> c;
    c.count = (int32_t)((count - base < K) ? count - base : K);
    for (int j = 0; j < c.count; ++j) c.v[j] = host[base + j];
    hipLaunchKernelGGL((table_set<T, K>), dim3(1), dim3(64 * ((K + 63) / 64)), 0, st, dev + base, c);
    MMF_LAUNCH_CHECK();
  }
  return MMF_OK;
}

}  // namespace mmf
