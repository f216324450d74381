// Block sort: the first stage of the cache-efficient merge sort (section 4.2:
// sort blocks sized to on-chip memory, then merge rounds), with LDS as the
// cache.  One workgroup of 256 lanes sorts a block of 2048 keys:
//   1. every lane sorts its 8 keys in registers with an odd-even
//      transposition network that swaps only strictly greater neighbours
//      (stable);
//   2. eight rounds of Merge Path inside LDS merge runs of 8, 16, ..., 1024
//      keys pairwise: the lanes of a run pair each find their split at local
//      diagonal q * 8 (Algorithm 2) and merge 8 outputs serially, left run as
//      A so that ties keep input order (section 2.1 tie rule).
// A short last block is handled by index bounds, never by sentinel keys.
#include "mp_device.h"
#include "mp_internal.h"

namespace mp {

// in and out may be the same array (each block is read whole before it is
// written), so they are not declared __restrict__.
template <typename K, bool KV>
__global__ __launch_bounds__(256) void blocksort_kernel(const K *in, const uint32_t *vin,
                                                        K *out, uint32_t *vout, int64_t n) {
  constexpr int NT = 256, VT = 8, BS = NT * VT;
  static_assert(BS == kSortBlock, "block size");
  // two buffers; VT + 1 slack slots for the unguarded serial merge
  __shared__ K keys[2][BS + VT + 1];
  __shared__ uint32_t vals[KV ? 2 : 1][KV ? BS + VT + 1 : 1];
  const int tid = threadIdx.x;
  const int64_t base = (int64_t)blockIdx.x * BS;
  const int cnt = (int)(n - base < BS ? n - base : BS);

  for (int i = tid; i < cnt; i += NT) {
    keys[0][i] = in[base + i];
    if constexpr (KV) vals[0][i] = vin[base + i];
  }
  __syncthreads();

  // 1. per-lane stable sort of VT keys
  {
    const int c = cnt - tid * VT < 0 ? 0 : (cnt - tid * VT < VT ? cnt - tid * VT : VT);
    K k[VT];
    uint32_t v[VT];
#pragma unroll
    for (int i = 0; i < VT; ++i) {
      k[i] = keys[0][tid * VT + i];
      if constexpr (KV) v[i] = vals[0][tid * VT + i];
    }
#pragma unroll
    for (int r = 0; r < VT; ++r) {
#pragma unroll
      for (int i = r & 1; i + 1 < VT; i += 2) {
        const bool sw = (i + 1 < c) && (k[i + 1] < k[i]);
        const K lo = sw ? k[i + 1] : k[i], hi = sw ? k[i] : k[i + 1];
        k[i] = lo;
        k[i + 1] = hi;
        if constexpr (KV) {
          const uint32_t vl = sw ? v[i + 1] : v[i], vh = sw ? v[i] : v[i + 1];
          v[i] = vl;
          v[i + 1] = vh;
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < VT; ++i) {
      if (i < c) {
        keys[0][tid * VT + i] = k[i];
        if constexpr (KV) vals[0][tid * VT + i] = v[i];
      }
    }
  }
  __syncthreads();

  // 2. Merge Path rounds inside LDS
  int src = 0;
#pragma unroll 1
  for (int r = VT; r < BS; r *= 2) {
    const int lanes_per_pair = (2 * r) / VT;
    const int p = tid / lanes_per_pair, q = tid % lanes_per_pair;
    const int ps = p * 2 * r;
    const int a0 = ps < cnt ? ps : cnt;
    const int b0 = ps + r < cnt ? ps + r : cnt;
    const int e = ps + 2 * r < cnt ? ps + 2 * r : cnt;
    const int na = b0 - a0, nb = e - b0;
    const int dl = q * VT < na + nb ? q * VT : na + nb;
    const K *ks = keys[src];
    int lo, hi;
    diag_range<int>(dl, na, nb, lo, hi);
    const int a = split_search<int>(
        dl, lo, hi, [&](int i) { return ks[a0 + i]; }, [&](int j) { return ks[b0 + j]; });
    K o[VT];
    int s[VT];
    serial_merge<K, VT>(ks, a0 + a, b0 + (dl - a), b0, e, o, s);
    const int steps = na + nb - dl < VT ? na + nb - dl : VT;
#pragma unroll
    for (int i = 0; i < VT; ++i) {
      if (i < steps) {
        keys[src ^ 1][a0 + dl + i] = o[i];
        if constexpr (KV) vals[src ^ 1][a0 + dl + i] = vals[src][s[i]];
      }
    }
    __syncthreads();
    src ^= 1;
  }

  for (int i = tid; i < cnt; i += NT) {
    out[base + i] = keys[src][i];
    if constexpr (KV) vout[base + i] = vals[src][i];
  }
}

template <typename K>
hipError_t launch_blocksort(const K *in, const uint32_t *vin, K *out, uint32_t *vout,
                            int64_t n, hipStream_t s) {
  const int64_t blocks = (n + kSortBlock - 1) / kSortBlock;
  if (blocks == 0) return hipSuccess;
  if (vout)
    hipLaunchKernelGGL((blocksort_kernel<K, true>), dim3((unsigned)blocks), dim3(256), 0, s,
                       in, vin, out, vout, n);
  else
    hipLaunchKernelGGL((blocksort_kernel<K, false>), dim3((unsigned)blocks), dim3(256), 0, s,
                       in, vin, out, vout, n);
  return hipGetLastError();
}

#define MP_INSTANTIATE(K)                                                        \
  template hipError_t launch_blocksort<K>(const K *, const uint32_t *, K *,      \
                                          uint32_t *, int64_t, hipStream_t);
MP_INSTANTIATE(uint32_t)
MP_INSTANTIATE(int32_t)
MP_INSTANTIATE(uint64_t)
MP_INSTANTIATE(float)
#undef MP_INSTANTIATE

}  // namespace mp
