// Grid-level split search (Algorithm 2): one lane per diagonal, lower-bound
// binary search along the cross diagonal (Theorem 14 bounds the steps by
// ceil(log2(min(na, nb) + 1))).  Launches with few diagonals give each
// diagonal a group of lanes that cuts the interval more ways per round.
#include "mp_device.h"
#include "mp_internal.h"

namespace mp {

// The split on diagonal d by binary lifting from the aligned origin 0: x
// counts the positions known to fail Algorithm 2's test, and each power of
// two, largest first, is added when the position it reaches still fails
// (positions below lo fail by the grid's bounds and are not read; none at
// or past hi is probed; the test is monotone, Corollary 12).  A probe's A
// index depends only on the steps taken so far, so diagonals that share them
// share the probe; on diagonals that are multiples of a power of two T, every
// probe at a step of at least T also falls on a multiple of T in B.  Both
// come from the caches for neighbouring diagonals.
template <typename K>
__device__ __forceinline__ int64_t aligned_split(const K *__restrict__ A, const K *__restrict__ B,
                                                 int64_t d, int64_t lo, int64_t hi) {
  int64_t x = 0;
  if (hi <= 0) return 0;
  for (int64_t bit = (int64_t)1 << (63 - __clzll((unsigned long long)hi)); bit > 0; bit >>= 1) {
    const int64_t c = x + bit - 1;
    if (c < hi && (c < lo || !(B[d - 1 - c] < A[c]))) x += bit;
  }
  return x;
}

template <typename K>
__global__ void partition_kernel(const K *__restrict__ A, int64_t na,
                                 const K *__restrict__ B, int64_t nb,
                                 const int64_t *__restrict__ diag, int64_t tile,
                                 int64_t n_diag, int64_t *__restrict__ a_split) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n_diag) return;
  const int64_t n = na + nb;
  int64_t d = diag ? diag[k] : k * tile;
  d = d < 0 ? 0 : (d > n ? n : d);
  int64_t lo, hi;
  diag_range<int64_t>(d, na, nb, lo, hi);
  // tile boundaries k * T: the aligned search (identical splits; the A
  // probes are shared for any T, the B probes too when T is a power of
  // two); diagonals the caller lists: the plain lower-bound search
  if (!diag && tile > 0)
    a_split[k] = aligned_split(A, B, d, lo, hi);
  else
    a_split[k] = split_search<int64_t>(
        d, lo, hi, [&](int64_t i) { return A[i]; },
        [&](int64_t j) { return B[j]; });
}

// G lanes per diagonal (group_split_search); lane 0 of each group writes.
template <typename K, int G>
__global__ __launch_bounds__(256) void partition_group_kernel(
    const K *__restrict__ A, int64_t na, const K *__restrict__ B, int64_t nb,
    const int64_t *__restrict__ diag, int64_t tile, int64_t n_diag,
    int64_t *__restrict__ a_split) {
  // groups never straddle a workgroup (G divides 256), so a group exits as one
  const int64_t k = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / G;
  if (k >= n_diag) return;
  const int64_t n = na + nb;
  int64_t d = diag ? diag[k] : k * tile;
  d = d < 0 ? 0 : (d > n ? n : d);
  int64_t lo, hi;
  diag_range<int64_t>(d, na, nb, lo, hi);
  const int64_t a = group_split_search<G, int64_t>(
      d, lo, hi, [&](int64_t i) { return A[i]; }, [&](int64_t j) { return B[j]; });
  if ((threadIdx.x & (G - 1)) == 0) a_split[k] = a;
}

int g_partition_lanes = 0;

// Measured on MI355X (2^29 + 2^29 keys): groups pay while G * n_diag stays
// within 2^14 lanes (2^10 diagonals: 21.8 us with one lane, 8.2 with 16;
// 2^12: 18.4 us, 11.4 with 4; from 2^14 diagonals on one lane is fastest,
// the extra probes then cost more bandwidth than the rounds they save).
int partition_lanes(int64_t n_diag) {
  if (g_partition_lanes > 0) return g_partition_lanes;
  int g = 1;
  while (g < 16 && n_diag * (2 * g) <= ((int64_t)1 << 14)) g *= 2;
  return g;
}

template <typename K>
hipError_t launch_partition(const K *A, int64_t na, const K *B, int64_t nb,
                            const int64_t *diag, int64_t tile, int64_t n_diag,
                            int64_t *a_split, hipStream_t s) {
  if (n_diag <= 0) return hipSuccess;
  constexpr int kThreads = 256;
  const int g = partition_lanes(n_diag);
  const int64_t blocks = (n_diag * g + kThreads - 1) / kThreads;
  switch (g) {
#define MP_GROUP_CASE(G)                                                                   \
  case G:                                                                                  \
    hipLaunchKernelGGL((partition_group_kernel<K, G>), dim3((unsigned)blocks),             \
                       dim3(kThreads), 0, s, A, na, B, nb, diag, tile, n_diag, a_split);   \
    break;
    MP_GROUP_CASE(2)
    MP_GROUP_CASE(4)
    MP_GROUP_CASE(8)
    MP_GROUP_CASE(16)
    MP_GROUP_CASE(32)
    MP_GROUP_CASE(64)
#undef MP_GROUP_CASE
    default:
      hipLaunchKernelGGL(partition_kernel<K>, dim3((unsigned)blocks), dim3(kThreads), 0, s, A,
                         na, B, nb, diag, tile, n_diag, a_split);
  }
  return hipGetLastError();
}

#define MP_INSTANTIATE(K)                                                      \
  template hipError_t launch_partition<K>(const K *, int64_t, const K *,       \
                                          int64_t, const int64_t *, int64_t,   \
                                          int64_t, int64_t *, hipStream_t);
MP_INSTANTIATE(uint32_t)
MP_INSTANTIATE(int32_t)
MP_INSTANTIATE(uint64_t)
MP_INSTANTIATE(float)
#undef MP_INSTANTIATE

}  // namespace mp
