// Decoupled look-back over tiles that take their indices in the order they
// start (a ticket counter), so that every tile waited on belongs to a
// workgroup that is already running and publishes before it waits: every
// wait ends.  A bound on the number of polls backs that up.
//
// status: one zeroed word per tile.  0 = nothing published yet, else a flag
// in the top two bits and a count below.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mp {

constexpr unsigned long long kLbAggregate = 1ull << 62;  // the tile's own count
constexpr unsigned long long kLbInclusive = 2ull << 62;  // count of all tiles up to it
constexpr unsigned long long kLbValue = (1ull << 62) - 1;
constexpr unsigned kLbMaxPolls = 1u << 22;  // far beyond any real wait

// Called by the 64 lanes of one wavefront of tile `tile` with its own count
// `total` (the same in every lane).  Publishes the count, adds up the
// counts of the tiles before it, 64 per round and nearest first, back to the
// nearest one that has published its inclusive count, publishes its own
// inclusive count and returns the exclusive one.  *gave_up is set when a
// wait passed the poll bound (a correct launch never does); the returned
// offset is then too small, never too large.
__device__ __forceinline__ int64_t lookback_exclusive(unsigned long long *status, int64_t tile,
                                                      int64_t total, bool *gave_up) {
  const int lane = threadIdx.x & 63;
  int64_t excl = 0;
  *gave_up = false;
  if (tile == 0) {
    if (lane == 0) atomicExch(&status[0], kLbInclusive | (unsigned long long)total);
    return 0;
  }
  if (lane == 0) atomicExch(&status[tile], kLbAggregate | (unsigned long long)total);
  int64_t j_hi = tile - 1;
  unsigned polls = 0;
  while (true) {
    const int64_t j = j_hi - lane;
    // before tile 0: an inclusive count of 0
    const unsigned long long v = j >= 0 ? atomicAdd(&status[j], 0ull) : kLbInclusive;
    const uint64_t inc = __ballot((v & kLbInclusive) != 0);
    const uint64_t empty = __ballot(v == 0);
    const int f = inc ? __ffsll((long long)inc) - 1 : 64;  // nearest inclusive lane
    const uint64_t upto = f >= 63 ? ~0ull : ((2ull << f) - 1);  // lanes 0..f
    if (empty & upto) {
      // a tile in range has not published yet: read the window again
      if (++polls > kLbMaxPolls) {
        *gave_up = true;
        break;
      }
      continue;
    }
    unsigned long long x = lane <= f ? (v & kLbValue) : 0ull;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
    excl += (int64_t)x;
    if (f < 64) break;
    j_hi -= 64;
  }
  if (lane == 0) atomicExch(&status[tile], kLbInclusive | (unsigned long long)(excl + total));
  return excl;
}

}  // namespace mp
