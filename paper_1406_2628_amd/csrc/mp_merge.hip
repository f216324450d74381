// Grid-level split search and the per-tile merge (Algorithms 1 and 2).
//
// launch_partition: one lane per diagonal, lower-bound binary search along
//   the cross diagonal (Algorithm 2; Theorem 14 bounds the steps by
//   ceil(log2(min(na, nb) + 1))).  Launches with few diagonals give each
//   diagonal a group of lanes that cuts the interval more ways per round.
// merge_tile_kernel: one workgroup per output tile of T = NT * VT elements.
//   The tile's A and B windows are exactly the pair cut by two consecutive
//   splits (Theorem 5); they are staged in LDS, every lane finds its own
//   split inside the tile at local diagonal lane * VT (the same search, now
//   over LDS), merges VT outputs serially, and the tile is written back with
//   coalesced stores through an LDS transpose.
#include "mp_device.h"
#include "mp_internal.h"

namespace mp {

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

// SEARCH = false: the splits of the tile's two diagonals come from a_split
// (mp_merge_split).  SEARCH = true: the workgroup finds them itself, wave 0
// on the start diagonal and wave 1 on the end diagonal at once, each probing
// 64 points per round (Theorem 14's search with a 65-way cut); this is
// Algorithm 1 with one processor per tile and needs no memory beyond the
// inputs and the output.
template <typename K, bool KV, int NT, int VT, bool SEARCH>
__global__ __launch_bounds__(NT) void merge_tile_kernel(
    const K *__restrict__ A, const uint32_t *__restrict__ Av, int64_t na,
    const K *__restrict__ B, const uint32_t *__restrict__ Bv, int64_t nb,
    K *__restrict__ S, uint32_t *__restrict__ Sv,
    const int64_t *__restrict__ a_split) {
  static_assert(!SEARCH || NT >= 128, "the in-kernel searches need two wavefronts");
  constexpr int T = NT * VT;
  // slack of VT + 1 slots: the unguarded serial merge may read up to VT
  // positions past the A window end (outputs discarded)
  __shared__ __attribute__((aligned(16))) K keys[T + VT + 1];
  __shared__ __attribute__((aligned(16))) uint32_t vals[KV ? T : 1];
  __shared__ int64_t s_a[SEARCH ? 2 : 1];
  const int tid = threadIdx.x;
  const int64_t tile = blockIdx.x;
  const int64_t n_all = na + nb;
  const int64_t d0 = tile * T;
  const int64_t d1 = d0 + T < n_all ? d0 + T : n_all;
  int64_t a0, a1;
  if constexpr (SEARCH) {
    if (tid < 128) {
      const int64_t d = tid < 64 ? d0 : d1;
      int64_t lo, hi;
      diag_range<int64_t>(d, na, nb, lo, hi);
      const int64_t a = group_split_search<64, int64_t>(
          d, lo, hi, [&](int64_t i) { return A[i]; }, [&](int64_t j) { return B[j]; });
      if ((tid & 63) == 0) s_a[tid >> 6] = a;
    }
    __syncthreads();
    a0 = s_a[0];
    a1 = s_a[1];
  } else {
    a0 = a_split[tile];
    a1 = a_split[tile + 1];
  }
  // The splits may come from the caller (mp_merge_split): a0 is kept on the
  // start diagonal inside the grid and the window width below in its valid
  // range, so every access stays in bounds whatever the split values.  For
  // true splits of sorted inputs both clamps change nothing.
  const int64_t lo0 = d0 > nb ? d0 - nb : 0, hi0 = d0 < na ? d0 : na;
  a0 = a0 < lo0 ? lo0 : (a0 > hi0 ? hi0 : a0);
  const int64_t b0 = d0 - a0;
  const int n = (int)(d1 - d0);
  int64_t wa64 = a1 - a0;
  const int64_t wa_lo = d1 - nb - a0 > 0 ? d1 - nb - a0 : 0;
  const int64_t wa_hi = na - a0 < (int64_t)n ? na - a0 : (int64_t)n;
  wa64 = wa64 < wa_lo ? wa_lo : (wa64 > wa_hi ? wa_hi : wa64);
  const int wa = (int)wa64, wb = n - wa;

  // Stage the pair (A[a0, a1), B[b0, b1)) back to back in LDS.  Each lane
  // issues all its loads into registers before its first LDS write, so they
  // are in flight together.
  {
    K rk[VT];
    uint32_t rv[KV ? VT : 1];
#pragma unroll
    for (int s = 0; s < VT; ++s) {
      const int i = tid + s * NT;
      const int64_t g = i < wa ? a0 + i : b0 + (i - wa);
      if (i < n) {
        rk[s] = (i < wa ? A : B)[g];
        if constexpr (KV) rv[s] = (i < wa ? Av : Bv)[g];
      }
    }
#pragma unroll
    for (int s = 0; s < VT; ++s) {
      const int i = tid + s * NT;
      if (i < n) {
        keys[i] = rk[s];
        if constexpr (KV) vals[i] = rv[s];
      }
    }
  }
  __syncthreads();

  // Lane split at local diagonal tid * VT, then VT serial steps.
  const int dl = tid * VT < n ? tid * VT : n;
  int lo, hi;
  diag_range<int>(dl, wa, wb, lo, hi);
  const int a = split_search<int>(
      dl, lo, hi, [&](int i) { return keys[i]; },
      [&](int j) { return keys[wa + j]; });
  const int steps = n - dl < VT ? n - dl : VT;
  K out[VT];
  int src[VT];
  serial_merge<K, VT>(keys, a, wa + dl - a, wa, n, out, src);
  uint32_t ov[VT];
  if constexpr (KV) {
#pragma unroll
    for (int i = 0; i < VT; ++i)
      if (i < steps) ov[i] = vals[src[i]];
  }
  __syncthreads();

  // Transpose through LDS so that the global stores are coalesced.
#pragma unroll
  for (int i = 0; i < VT; ++i) {
    if (i < steps) {
      keys[tid * VT + i] = out[i];
      if constexpr (KV) vals[tid * VT + i] = ov[i];
    }
  }
  __syncthreads();
  // 16-byte nontemporal stores where the tile's output is aligned (every
  // tile starts at a multiple of T keys), element stores for the rest
  constexpr int VEC = 16 / (int)sizeof(K);
  const bool vec = (((uintptr_t)(S + d0) | (KV ? (uintptr_t)(Sv + d0) : 0)) % 16) == 0;
  const int nv = vec ? n / VEC : 0;
  for (int v = tid; v < nv; v += NT)
    __builtin_nontemporal_store(reinterpret_cast<const u32x4 *>(keys)[v],
                                reinterpret_cast<u32x4 *>(S + d0) + v);
  for (int i = nv * VEC + tid; i < n; i += NT) S[d0 + i] = keys[i];
  if constexpr (KV) {
    const int nv4 = vec ? n / 4 : 0;
    for (int v = tid; v < nv4; v += NT)
      __builtin_nontemporal_store(reinterpret_cast<const u32x4 *>(vals)[v],
                                  reinterpret_cast<u32x4 *>(Sv + d0) + v);
    for (int i = nv4 * 4 + tid; i < n; i += NT) Sv[d0 + i] = vals[i];
  }
}

TileCfg default_tile_cfg(size_t key_bytes, bool kv) {
  (void)key_bytes;
  (void)kv;
  return TileCfg{256, 16};
}

template <typename K, bool KV, int NT, int VT>
static hipError_t launch_tiles_impl(const K *A, const uint32_t *Av, int64_t na,
                                    const K *B, const uint32_t *Bv, int64_t nb,
                                    K *S, uint32_t *Sv, const int64_t *a_split,
                                    hipStream_t s) {
  constexpr int64_t T = NT * VT;
  const int64_t n_tiles = (na + nb + T - 1) / T;
  if (n_tiles == 0) return hipSuccess;
  if (a_split)
    hipLaunchKernelGGL((merge_tile_kernel<K, KV, NT, VT, false>), dim3((unsigned)n_tiles),
                       dim3(NT), 0, s, A, Av, na, B, Bv, nb, S, Sv, a_split);
  else
    hipLaunchKernelGGL((merge_tile_kernel<K, KV, NT, VT, true>), dim3((unsigned)n_tiles),
                       dim3(NT), 0, s, A, Av, na, B, Bv, nb, S, Sv, nullptr);
  return hipGetLastError();
}

template <typename K>
hipError_t launch_merge_tiles(TileCfg cfg, const K *A, const uint32_t *Av,
                              int64_t na, const K *B, const uint32_t *Bv,
                              int64_t nb, K *S, uint32_t *Sv,
                              const int64_t *a_split, hipStream_t s) {
  const bool kv = Sv != nullptr;
#define MP_TILE_CASE(NT_, VT_)                                                \
  if (cfg.nt == NT_ && cfg.vt == VT_)                                         \
    return kv ? launch_tiles_impl<K, true, NT_, VT_>(A, Av, na, B, Bv, nb, S, \
                                                     Sv, a_split, s)          \
              : launch_tiles_impl<K, false, NT_, VT_>(A, Av, na, B, Bv, nb,   \
                                                      S, Sv, a_split, s);
  MP_TILE_CASE(256, 16)
  MP_TILE_CASE(256, 15)
  MP_TILE_CASE(256, 8)
  MP_TILE_CASE(128, 16)
#undef MP_TILE_CASE
  return hipErrorNotSupported;
}

#define MP_INSTANTIATE(K)                                                      \
  template hipError_t launch_partition<K>(const K *, int64_t, const K *,       \
                                          int64_t, const int64_t *, int64_t,   \
                                          int64_t, int64_t *, hipStream_t);    \
  template hipError_t launch_merge_tiles<K>(                                   \
      TileCfg, const K *, const uint32_t *, int64_t, const K *,                \
      const uint32_t *, int64_t, K *, uint32_t *, const int64_t *, hipStream_t);
MP_INSTANTIATE(uint32_t)
MP_INSTANTIATE(int32_t)
MP_INSTANTIATE(uint64_t)
MP_INSTANTIATE(float)
#undef MP_INSTANTIATE

}  // namespace mp
