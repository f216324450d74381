// Plain streaming copy: the reference point for achievable HBM bandwidth and
// for calibrating the hardware traffic counters.  Each lane keeps UNROLL
// 16-byte loads in flight before storing them (nontemporal), and workgroups
// stride over blocks of 256 * UNROLL vectors.
#include "mp_device.h"
#include "mp_internal.h"

namespace mp {

template <int UNROLL>
__global__ __launch_bounds__(256) void copy_kernel(const u32x4 *__restrict__ src,
                                                   u32x4 *__restrict__ dst,
                                                   int64_t n_vec) {
  constexpr int64_t BLK = 256 * UNROLL;
  const int64_t n_full = n_vec / BLK;
  for (int64_t blk = blockIdx.x; blk < n_full; blk += gridDim.x) {
    const int64_t base = blk * BLK + threadIdx.x;
    u32x4 v[UNROLL];
#pragma unroll
    for (int u = 0; u < UNROLL; ++u) v[u] = __builtin_nontemporal_load(src + base + u * 256);
#pragma unroll
    for (int u = 0; u < UNROLL; ++u) __builtin_nontemporal_store(v[u], dst + base + u * 256);
  }
  // tail: fewer than one block of vectors, spread over the first workgroup
  if (blockIdx.x == 0)
    for (int64_t i = n_full * BLK + threadIdx.x; i < n_vec; i += 256) dst[i] = src[i];
}

hipError_t launch_copy(const void *src, void *dst, int64_t n_bytes, int unroll,
                       int grid, hipStream_t s) {
  const int64_t n_vec = n_bytes / 16;
  if (n_vec == 0) return hipSuccess;
  if (grid <= 0) grid = device_cu_count() * 32;
  const u32x4 *a = (const u32x4 *)src;
  u32x4 *b = (u32x4 *)dst;
  switch (unroll) {
    case 1: hipLaunchKernelGGL(copy_kernel<1>, dim3(grid), dim3(256), 0, s, a, b, n_vec); break;
    case 2: hipLaunchKernelGGL(copy_kernel<2>, dim3(grid), dim3(256), 0, s, a, b, n_vec); break;
    case 4: hipLaunchKernelGGL(copy_kernel<4>, dim3(grid), dim3(256), 0, s, a, b, n_vec); break;
    case 0:
    case 8: hipLaunchKernelGGL(copy_kernel<8>, dim3(grid), dim3(256), 0, s, a, b, n_vec); break;
    default: return hipErrorNotSupported;
  }
  return hipGetLastError();
}

}  // namespace mp
