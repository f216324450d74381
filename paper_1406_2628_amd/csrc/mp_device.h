// Device-side building blocks of the Merge Path kernels (gfx950, wave64).
//
// Notation follows the paper: A and B are the sorted inputs, a split on cross
// diagonal d is the pair (a, b = d - a) where the Merge Path crosses that
// diagonal.  The split is the smallest a on the diagonal for which
//     B[b-1] < A[a]                     (the path does not step right there)
// holds, with terms outside A or B counting as true; at that a the second
// condition of Algorithm 2, A[a-1] <= B[b], holds as well, and the split is
// unique (Corollary 12, Proposition 13).  Every search below is a lower-bound
// binary search for that predicate (Algorithm 2 with its search interval
// clamped to the diagonal's extent inside the grid, and floor midpoints).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mp {

// 16-byte vector of four 32-bit words (native clang vector: usable with the
// nontemporal load/store builtins and lowered to dwordx4 / b128 accesses).
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Bounds of the candidate a on diagonal d of an na x nb grid.
template <typename I>
__device__ __forceinline__ void diag_range(I d, I na, I nb, I &lo, I &hi) {
  lo = d > nb ? d - nb : 0;
  hi = d < na ? d : na;
}

// Lower-bound search for the split on diagonal d over arrays reachable
// through the accessors ga(i) (A) and gb(j) (B).  Only indices in
// [lo, hi) of A and [d-hi, d-1-lo] of B are probed.
template <typename I, typename GA, typename GB>
__device__ __forceinline__ I split_search(I d, I lo, I hi, GA ga, GB gb) {
  while (lo < hi) {
    I mid = lo + ((hi - lo) >> 1);
    if (gb(d - 1 - mid) < ga(mid))
      hi = mid;
    else
      lo = mid + 1;
  }
  return lo;
}

// Split on diagonal d restricted to the candidate interval [lo, hi), found
// by the 64 lanes of the calling wavefront (every lane returns the same
// value).  Each round probes 64 interior points and keeps the gap where the
// predicate B[d-1-a] < A[a] first turns true (it is monotone in a,
// Corollary 12).
template <typename GA, typename GB>
__device__ int64_t wave_split_search(int64_t d, int64_t lo, int64_t hi, GA ga, GB gb) {
  const int lane = threadIdx.x & 63;
  while (lo < hi) {
    const int64_t span = hi - lo;
    if (span <= 64) {
      const int64_t p = lo + lane;
      const bool pred = lane < span && (gb(d - 1 - p) < ga(p));
      const uint64_t m = __ballot(pred);
      return m ? lo + (int64_t)(__ffsll((long long)m) - 1) : hi;
    }
    const int64_t p = lo + ((int64_t)(lane + 1) * span) / 65;
    const bool pred = gb(d - 1 - p) < ga(p);
    const uint64_t m = __ballot(pred);
    if (m == 0) {
      lo = lo + ((int64_t)64 * span) / 65 + 1;
    } else {
      const int f = __ffsll((long long)m) - 1;
      const int64_t pf = lo + ((int64_t)(f + 1) * span) / 65;
      lo = f == 0 ? lo : lo + ((int64_t)f * span) / 65 + 1;
      hi = pf;
    }
  }
  return lo;
}

// The same search with G lanes per diagonal (G a power of two, 2..64): the
// group is an aligned block of G lanes of one wavefront holding the same d,
// lo and hi.  Each round its lanes probe G points that cut [lo, hi) G + 1
// ways and the group keeps the part where the predicate turns true (it is
// monotone along the diagonal, Corollary 12), so about log_{G+1} of the
// interval rounds of dependent loads replace log_2 of it.  Every lane of
// the group returns the split.
template <int G, typename I, typename GA, typename GB>
__device__ __forceinline__ I group_split_search(I d, I lo, I hi, GA ga, GB gb) {
  static_assert(G >= 2 && G <= 64 && (G & (G - 1)) == 0, "group size");
  const int lane = threadIdx.x & 63;
  const int r = lane & (G - 1);
  const int base = lane & (64 - G);  // first lane of the group
  const uint64_t gmask = G == 64 ? ~0ull : ((1ull << G) - 1);
  while (lo < hi) {
    const I span = hi - lo;
    if (span <= G) {
      // one probe per remaining candidate
      const I p = lo + r;
      const bool pred = r < span && (gb(d - 1 - p) < ga(p));
      const uint64_t m = (__ballot(pred) >> base) & gmask;
      return m ? lo + (I)(__ffsll((long long)m) - 1) : hi;
    }
    const I p = lo + ((I)(r + 1) * span) / (G + 1);
    const bool pred = gb(d - 1 - p) < ga(p);
    const uint64_t m = (__ballot(pred) >> base) & gmask;
    if (m == 0) {
      lo = lo + ((I)G * span) / (G + 1) + 1;
    } else {
      // first true probe f: the split lies after probe f - 1, at or before f
      const int f = __ffsll((long long)m) - 1;
      const I pf = lo + ((I)(f + 1) * span) / (G + 1);
      lo = f == 0 ? lo : lo + ((I)f * span) / (G + 1) + 1;
      hi = pf;
    }
  }
  return lo;
}

// Serial merge of VT outputs from a split, entirely in LDS (Lemma 1; the
// loser of each compare stays in a register so each step reads one key).
//   keys: LDS array; A keys at positions [ai, a_end), B keys at [bi, b_end).
//   ai, bi: LDS positions of the next A and B keys.
// All VT steps run without guards: a lane whose run is shorter than VT keeps
// stepping past it, and the caller discards those outputs.  Such extra steps
// only read positions below max(a_end, b_end) + VT, which the caller keeps
// inside the LDS array.
// On return out[i] holds the keys and src[i] their LDS positions.
template <typename K, int VT>
__device__ __forceinline__ void serial_merge(const K *keys, int ai, int bi,
                                             int a_end, int b_end,
                                             K (&out)[VT], int (&src)[VT]) {
  K ka = keys[ai];
  K kb = keys[bi];
#pragma unroll
  for (int i = 0; i < VT; ++i) {
    const bool take_b = (bi < b_end) && (ai >= a_end || kb < ka);
    out[i] = take_b ? kb : ka;
    const int taken = take_b ? bi : ai;
    src[i] = taken;
    // the side just taken advances to its next key, which is read next
    ai = take_b ? ai : taken + 1;
    bi = take_b ? taken + 1 : bi;
    const K nxt = keys[taken + 1];
    ka = take_b ? ka : nxt;
    kb = take_b ? nxt : kb;
  }
}

// The same merge without end tests, for a lane whose run ends at the split
// (a1, b1) of the next lane's diagonal with A[a1] and B[b1] both real keys in
// LDS.  Then every compare reads real keys and takes the right side: while
// the lane still has A keys left, B[b1] >= A[ai] (the split's condition
// A[a1-1] <= B[b1]); while it has B keys left, B[bi] < A[a1] (the condition
// B[b1-1] < A[a1]).  So no step needs to know where either input ends.
template <typename K, int VT>
__device__ __forceinline__ void serial_merge_inner(const K *keys, int ai, int bi,
                                                   K (&out)[VT], int (&src)[VT]) {
  K ka = keys[ai];
  K kb = keys[bi];
#pragma unroll
  for (int i = 0; i < VT; ++i) {
    const bool take_b = kb < ka;
    out[i] = take_b ? kb : ka;
    const int taken = take_b ? bi : ai;
    src[i] = taken;
    // the side just taken advances to its next key, which is read next
    ai = take_b ? ai : taken + 1;
    bi = take_b ? taken + 1 : bi;
    const K nxt = keys[taken + 1];
    ka = take_b ? ka : nxt;
    kb = take_b ? nxt : kb;
  }
}

// Inclusive scan of one value per lane across a workgroup of 1024 lanes
// (every lane must call it); *total receives the sum over all lanes.
// Calling it again needs a barrier first (its wave totals sit in LDS).
__device__ __forceinline__ int64_t workgroup_scan1024(int64_t v, int64_t *total) {
  __shared__ int64_t s_w[1024 / 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int64_t y = __shfl_up(v, o);
    if (lane >= o) v += y;
  }
  if (lane == 63) s_w[wave] = v;
  __syncthreads();
  int64_t before = 0, all = 0;
#pragma unroll
  for (int w = 0; w < 1024 / 64; ++w) {
    const int64_t t = s_w[w];
    before += w < wave ? t : 0;
    all += t;
  }
  *total = all;
  return v + before;
}

}  // namespace mp
