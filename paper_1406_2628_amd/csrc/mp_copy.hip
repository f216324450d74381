// Bandwidth references: the reference points for achievable HBM bandwidth and
// for calibrating the hardware traffic counters.
//   copy   each lane keeps UNROLL 16-byte loads in flight before storing them
//          (nontemporal), workgroups stride over blocks of 256 * UNROLL vectors;
//   read   the same loads, folded into one 16-byte word per wavefront;
//   write  the same stores of a fixed pattern, nothing read.
#include <type_traits>

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

// Reads n_vec vectors; wavefront w of workgroup g stores the XOR of what its
// lanes read at sink[g * 4 + w] (grid * 4 vectors).
template <int UNROLL>
__global__ __launch_bounds__(256) void read_kernel(const u32x4 *__restrict__ src,
                                                   u32x4 *__restrict__ sink, int64_t n_vec) {
  constexpr int64_t BLK = 256 * UNROLL;
  const int64_t n_full = n_vec / BLK;
  u32x4 acc = {0u, 0u, 0u, 0u};
  for (int64_t blk = blockIdx.x; blk < n_full; blk += gridDim.x) {
    const int64_t base = blk * BLK + threadIdx.x;
    u32x4 v[UNROLL];
#pragma unroll
    for (int u = 0; u < UNROLL; ++u) v[u] = __builtin_nontemporal_load(src + base + u * 256);
#pragma unroll
    for (int u = 0; u < UNROLL; ++u) acc ^= v[u];
  }
  if (blockIdx.x == 0)
    for (int64_t i = n_full * BLK + threadIdx.x; i < n_vec; i += 256) acc ^= src[i];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    acc.x ^= __shfl_xor(acc.x, o);
    acc.y ^= __shfl_xor(acc.y, o);
    acc.z ^= __shfl_xor(acc.z, o);
    acc.w ^= __shfl_xor(acc.w, o);
  }
  if ((threadIdx.x & 63) == 0) sink[(int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)] = acc;
}

// Writes n_vec vectors of the pattern {i, i, i, i} (i = vector index, low 32 bits).
template <int UNROLL>
__global__ __launch_bounds__(256) void write_kernel(u32x4 *__restrict__ dst, int64_t n_vec) {
  constexpr int64_t BLK = 256 * UNROLL;
  const int64_t n_full = n_vec / BLK;
  for (int64_t blk = blockIdx.x; blk < n_full; blk += gridDim.x) {
    const int64_t base = blk * BLK + threadIdx.x;
#pragma unroll
    for (int u = 0; u < UNROLL; ++u) {
      const uint32_t x = (uint32_t)(base + u * 256);
      const u32x4 v = {x, x, x, x};
      __builtin_nontemporal_store(v, dst + base + u * 256);
    }
  }
  if (blockIdx.x == 0)
    for (int64_t i = n_full * BLK + threadIdx.x; i < n_vec; i += 256) {
      const uint32_t x = (uint32_t)i;
      dst[i] = u32x4{x, x, x, x};
    }
}

hipError_t launch_bw_probe(int kind, const void *src, void *dst, int64_t n_bytes, int unroll,
                           int grid, hipStream_t s) {
  const int64_t n_vec = n_bytes / 16;
  if (n_vec == 0) return hipSuccess;
  if (grid <= 0) grid = device_cu_count() * 32;
  const u32x4 *a = (const u32x4 *)src;
  u32x4 *b = (u32x4 *)dst;
  auto go = [&](auto uc) {
    constexpr int U = decltype(uc)::value;
    if (kind == 0) hipLaunchKernelGGL(copy_kernel<U>, dim3(grid), dim3(256), 0, s, a, b, n_vec);
    else if (kind == 1) hipLaunchKernelGGL(read_kernel<U>, dim3(grid), dim3(256), 0, s, a, b, n_vec);
    else hipLaunchKernelGGL(write_kernel<U>, dim3(grid), dim3(256), 0, s, b, n_vec);
  };
  switch (unroll) {
    case 1: go(std::integral_constant<int, 1>()); break;
    case 2: go(std::integral_constant<int, 2>()); break;
    case 4: go(std::integral_constant<int, 4>()); break;
    case 0:
    case 8: go(std::integral_constant<int, 8>()); break;
    case 16: go(std::integral_constant<int, 16>()); break;
    default: return hipErrorNotSupported;
  }
  return hipGetLastError();
}

hipError_t launch_copy(const void *src, void *dst, int64_t n_bytes, int unroll,
                       int grid, hipStream_t s) {
  return launch_bw_probe(0, src, dst, n_bytes, unroll, grid, s);
}

}  // namespace mp
