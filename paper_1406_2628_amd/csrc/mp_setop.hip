// Multiset operations on two sorted inputs through the same partition: the
// output tiles of the merge are cut by splits on their diagonals (Algorithm
// 2) and each tile's pair is processed independently (Corollary 6), here
// keeping or dropping each merged key instead of writing all of them.
//
// In the stable merge the copies of a value sit together, A's m copies
// first, then B's n.  Pairing equal keys front to front:
//   - A's copy of rank k (k counted from the start of its run in A) is
//     matched when B holds more than k copies, i.e. when B[lb_B + k] equals
//     it, where lb_B, the start of the value's run in B, is exactly the
//     path's b when that A copy is taken (ties take A, so no copy of the
//     value from B precedes it);
//   - B's copy of rank k is matched when A holds more than k copies, i.e.
//     when A[ub_A - 1 - k] equals it, where ub_A is the path's a when that B
//     copy is taken (all of A's copies precede it).
// Intersection keeps matched A copies; union keeps every A copy and the
// unmatched B copies; difference keeps the unmatched A copies; symmetric
// difference keeps the unmatched copies of both.
//
// The rank of the first A (and B) copy a lane takes comes from a lower-bound
// search in the tile's LDS window; only the window's first value can have its
// run start before the window, and wave 0 finds that start in global memory
// once per tile.  Along the lane's serial merge each side then keeps where
// its current run starts, and a copy's rank is its distance from there.
//
// One pass: each tile's kept keys are compacted through LDS and written at
// the tile's output offset, found by a decoupled look-back over the tiles
// before it.  Workgroups take tiles in the order they start (a ticket
// counter), so every tile a workgroup waits on belongs to a workgroup that
// is already running; each tile publishes its own count before it waits,
// so every wait ends, and a bound on the polls backs that up.
#include <mutex>
#include <type_traits>
#include <vector>

#include "mp_device.h"
#include "mp_internal.h"
#include "mp_lookback.h"

namespace mp {

// 512 lanes per tile, each taking 25 outputs for 4-byte keys and 13 for
// 8-byte keys (about 50 KiB of LDS either way, three workgroups per CU).  An
// odd count keeps the lanes' LDS cursors, half a lane's outputs apart in
// each window, off a shared bank.
constexpr int kSetNT = 512;
template <typename K>
constexpr int kSetVT = sizeof(K) == 4 ? 25 : 13;
constexpr int kSetTMin = kSetNT * 12;  // at most the smaller tile: bounds the tile count
// keys per 16-byte chunk of the window loads and output stores
template <typename K>
constexpr int kSetCH = 16 / (int)sizeof(K);

// The chunk X[g, g + CH) of an array of lim keys.  Chunks sit on a grid
// aligned to 16 bytes in memory, so one that lies inside the array is one
// nontemporal vector load; at the array's ends (g may be negative) only the
// keys inside it are read.
template <typename K>
__device__ __forceinline__ void set_load_chunk(const K *__restrict__ X, int64_t g, int64_t lim,
                                               K (&v)[kSetCH<K>]) {
  constexpr int CH = kSetCH<K>;
  if (g >= 0 && g + CH <= lim) {
    *reinterpret_cast<u32x4 *>(v) =
        __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(X + g));
  } else {
#pragma unroll
    for (int j = 0; j < CH; ++j) v[j] = g + j >= 0 && g + j < lim ? X[g + j] : K{};
  }
}

template <typename K>
__device__ __forceinline__ bool key_eq(K x, K y) {
  return !(x < y) && !(y < x);
}

// First index i in [lo, hi) with pred(i) true (pred monotone false -> true),
// hi if none; found by the 64 lanes of the calling wavefront, 64 probes per
// round.  Every lane returns the result.
template <typename P>
__device__ int64_t wave_first_true(int64_t lo, int64_t hi, P pred) {
  const int lane = threadIdx.x & 63;
  while (lo < hi) {
    const int64_t span = hi - lo;
    if (span <= 64) {
      const uint64_t m = __ballot(lane < span && pred(lo + lane));
      return m ? lo + (int64_t)(__ffsll((long long)m) - 1) : hi;
    }
    const int64_t p = lo + ((int64_t)(lane + 1) * span) / 65;
    const uint64_t m = __ballot(pred(p));
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

// Start of the run of keys equal to X[p] (p > 0), by the 64 lanes of the
// calling wavefront: one round over the 64 keys before p, then, for a
// longer run, the 64-way search over everything before them.
template <typename K>
__device__ int64_t run_start(const K *X, int64_t p) {
  const int lane = threadIdx.x & 63;
  const K v = X[p];
  const int64_t q = p - 1 - lane;
  const uint64_t smaller = __ballot(q < 0 || X[q] < v);
  if (smaller) return p - (__ffsll((long long)smaller) - 1);  // lane f: X[p-1-f] < v
  return wave_first_true(0, p - 64, [&](int64_t i) { return !(X[i] < v); });
}

// OP: 0 intersection, 1 union, 2 difference, 3 symmetric difference.
// status: n_tiles zeroed words; ticket: a zeroed counter; *count: zeroed,
// receives the output length (-1 if a wait ever gave up, which a correct
// launch never does).  cap: the slots of S.  Sorted inputs never keep more
// than cap keys, but unsorted ones can: their splits need not increase from
// tile to tile, so the tiles' pairs may overlap and together keep more keys
// than either input holds.  Every store is therefore bounded by cap, and the
// count is clamped to it.
template <typename K, int OP>
__global__ __launch_bounds__(kSetNT) void setop_tile_kernel(
    const K *__restrict__ A, int64_t na, const K *__restrict__ B, int64_t nb,
    const int64_t *__restrict__ a_split, unsigned long long *__restrict__ status,
    unsigned long long *__restrict__ ticket, int64_t n_tiles, int64_t *__restrict__ count,
    K *__restrict__ S, int64_t cap) {
  constexpr int NT = kSetNT, VT = kSetVT<K>, T = NT * VT;
  constexpr int CH = kSetCH<K>;
  // both windows' chunks (at most T + 4 CH - 4 keys) and the slack the walk
  // reads past the end of B's window
  __shared__ __align__(16) K keys[T + 4 * CH + VT + 1];
  __shared__ int s_cnt[NT / 64];
  __shared__ int64_t s_lb[2], s_tile, s_excl;
  const int tid = threadIdx.x;
  if (tid == 0) s_tile = (int64_t)atomicAdd(ticket, 1ull);
  __syncthreads();
  const int64_t tile = s_tile;
  const int64_t N = na + nb;
  const int64_t d0 = tile * T;
  const int64_t d1 = d0 + T < N ? d0 + T : N;
  const int n = (int)(d1 - d0);
  // the tile's pair (splits from the grid search; the clamps keep every
  // access in bounds as in the merge's per-tile kernel)
  const int64_t lo0 = d0 > nb ? d0 - nb : 0, hi0 = d0 < na ? d0 : na;
  int64_t a0 = a_split[tile];
  a0 = a0 < lo0 ? lo0 : (a0 > hi0 ? hi0 : a0);
  const int64_t b0 = d0 - a0;
  int64_t wa64 = a_split[tile + 1] - a0;
  const int64_t wa_lo = d1 - nb - a0 > 0 ? d1 - nb - a0 : 0;
  const int64_t wa_hi = na - a0 < (int64_t)n ? na - a0 : (int64_t)n;
  wa64 = wa64 < wa_lo ? wa_lo : (wa64 > wa_hi ? wa_hi : wa64);
  const int wa = (int)wa64, wb = n - wa;
  // the pair in LDS, read in 16-byte chunks on a grid aligned in memory and
  // stored whole: A's chunks from position 0 and B's after them, so A[a0]
  // sits at oa and B[b0] at ob, and the windows end at ae and be.  Each lane
  // issues all its chunk loads into registers before the first LDS write,
  // so they are in flight together.
  constexpr int PV = (T / CH + 4 + NT - 1) / NT;  // ca + cb <= T / CH + 3
  const int sa = (int)(((uintptr_t)(A + a0) / sizeof(K)) & (CH - 1));
  const int sb = (int)(((uintptr_t)(B + b0) / sizeof(K)) & (CH - 1));
  const int ca = (sa + wa + CH - 1) / CH, cb = (sb + wb + CH - 1) / CH;
  const int oa = sa, ob = ca * CH + sb, ae = oa + wa, be = ob + wb;
  K stage[PV][CH];
#pragma unroll
  for (int k = 0; k < PV; ++k) {
    const int c = tid + k * NT;
    if (c < ca + cb) {
      const bool fb = c >= ca;
      const int64_t g = fb ? b0 - sb + (int64_t)(c - ca) * CH : a0 - sa + (int64_t)c * CH;
      set_load_chunk<K>(fb ? B : A, g, fb ? nb : na, stage[k]);
    }
  }
  // run starts of the window's first A and first B value (global search only
  // when the run reaches back past the window)
  if (tid < 64) {
    int64_t lbA = a0, lbB = b0;
    if (wa > 0 && a0 > 0) lbA = run_start(A, a0);
    if (wb > 0 && b0 > 0) lbB = run_start(B, b0);
    if (tid == 0) {
      s_lb[0] = lbA;
      s_lb[1] = lbB;
    }
  }
#pragma unroll
  for (int k = 0; k < PV; ++k) {
    const int c = tid + k * NT;
    if (c < ca + cb)
      *reinterpret_cast<u32x4 *>(keys + c * CH) = *reinterpret_cast<const u32x4 *>(stage[k]);
  }
  __syncthreads();

  // this lane's split at local diagonal tid * VT
  const int dl = tid * VT < n ? tid * VT : n;
  int lo, hi;
  diag_range<int>(dl, wa, wb, lo, hi);
  const int a = split_search<int>(
      dl, lo, hi, [&](int i) { return keys[oa + i]; }, [&](int j) { return keys[ob + j]; });
  int ai = oa + a, bi = ob + dl - a;  // LDS positions
  const int steps = n - dl < VT ? n - dl : VT;
  // ranks of the first A and B copies this lane takes
  int64_t kA = 0, kB = 0;
  // (a search only when the key before it in the window is equal)
  if (ai < ae) {
    const K v = keys[ai];
    if (ai > oa && key_eq(keys[ai - 1], v)) {
      int l = oa, h = ai - 1;  // first position in [oa, ai - 1] holding v
      while (l < h) {
        const int m = (l + h) >> 1;
        if (keys[m] < v) l = m + 1; else h = m;
      }
      kA = l > oa ? ai - l : (a0 + (ai - oa)) - s_lb[0];
    } else {
      kA = ai > oa ? 0 : a0 - s_lb[0];
    }
  }
  if (bi < be) {
    const K v = keys[bi];
    if (bi > ob && key_eq(keys[bi - 1], v)) {
      int l = ob, h = bi - 1;
      while (l < h) {
        const int m = (l + h) >> 1;
        if (keys[m] < v) l = m + 1; else h = m;
      }
      kB = l > ob ? bi - l : (b0 + (bi - ob)) - s_lb[1];
    } else {
      kB = bi > ob ? 0 : b0 - s_lb[1];
    }
  }

  // The walk.  sA / sB: the LDS position where the run of the next A / B
  // copy starts, so a copy taken at position p has rank p - sA (or p - sB).
  // The lane's first runs may start far before the window: their starts are
  // placed at most 2^30 back, and a partner lookup through such a run adds
  // the exact rest (xA / xB) while the start is still the first one.  A
  // partner inside the window is one LDS read; one outside it takes the
  // exact index and a global read.  When a copy is taken, the key after it
  // on its side says whether the next copy continues the run.  The loser of
  // each compare stays in a register (ka / kb).
  const int kA0s = (int)(kA < (1 << 30) ? kA : (1 << 30));
  const int kB0s = (int)(kB < (1 << 30) ? kB : (1 << 30));
  const int64_t xA = kA - kA0s, xB = kB - kB0s;
  const int sA0 = ai - kA0s, sB0 = bi - kB0s;
  int sA = sA0, sB = sB0;
  K ka = keys[ai], kb = keys[bi];
  K out[VT];
  uint32_t keep = 0;
  // all VT steps run: a lane whose run is shorter keeps stepping past it
  // (LDS reads stay below be + VT + 1, global reads inside the arrays);
  // the outputs past its run are masked off after the walk
#pragma unroll
  for (int s = 0; s < VT; ++s) {
    const bool tb = (bi < be) && (ai >= ae || kb < ka);
    const K v = tb ? kb : ka;
    const int pos = tb ? bi : ai;
    const int st = tb ? sB : sA;
    const int r = pos - st;
    // partner: an A copy's is B[b + rank] (b = the path's b, where the run
    // starts in B); a B copy's is A[a - 1 - rank] (a = the path's a, where
    // the run ends in A).  As LDS positions: bi + r, inside B's window when
    // below be, and ai - 1 - r, inside A's when at least oa; one unsigned
    // compare against [oa, be) tells both.
    const int idx = tb ? ai - 1 - r : bi + r;
    const bool in_win = (unsigned)(idx - oa) < (unsigned)(be - oa);
    bool m = key_eq(keys[in_win ? idx : 0], v);
    if (!in_win) {
      const int64_t r64 = r + (tb ? (st == sB0 ? xB : 0) : (st == sA0 ? xA : 0));
      const int64_t q = tb ? a0 + (ai - oa) - 1 - r64 : b0 + (bi - ob) + r64;
      const bool in_range = tb ? q >= 0 : q < nb;
      m = in_range && key_eq(tb ? A[q] : B[q], v);
    }
    out[s] = v;
    const bool kept = tb ? (OP == 1 || OP == 3) && !m : OP == 1 || (OP == 0 ? m : !m);
    keep = kept ? keep | (1u << s) : keep;
    // an empty asm that reads and writes keep in a VGPR: it pins the update
    // to this step instead of letting every step's decision stay live in
    // scalar registers until the end of the walk
    asm volatile("" : "+v"(keep));
    const int p1 = pos + 1;
    const K nxt = keys[p1];
    const int st1 = key_eq(nxt, v) ? st : p1;
    ai = tb ? ai : p1;
    bi = tb ? p1 : bi;
    ka = tb ? ka : nxt;
    kb = tb ? nxt : kb;
    sA = tb ? sA : st1;
    sB = tb ? st1 : sB;
  }
  keep &= steps >= 32 ? ~0u : (1u << steps) - 1u;

  // prefix of the lanes' kept counts: a shuffle scan inside each wavefront,
  // then the wavefront totals through LDS
  const int c = __popc(keep);
  const int lane = tid & 63, wave = tid >> 6;
  int incl = c;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(incl, o);
    if (lane >= o) incl += y;
  }
  if (lane == 63) s_cnt[wave] = incl;
  __syncthreads();
  int total = 0;
#pragma unroll
  for (int w = 0; w < NT / 64; ++w) {
    const int t = s_cnt[w];
    incl += w < wave ? t : 0;
    total += t;
  }
  // output offset: publish this tile's count and look back over the tiles
  // before it (wave 0)
  if (tid < 64) {
    bool gave_up;
    const int64_t excl = lookback_exclusive(status, tile, total, &gave_up);
    if (tid == 0) {
      s_excl = excl;
      const int64_t end = excl + total < cap ? excl + total : cap;
      if (gave_up) atomicExch((unsigned long long *)count, ~0ull);
      else if (tile == n_tiles - 1)
        atomicCAS((unsigned long long *)count, 0ull, (unsigned long long)end);
    }
  }
  // compact through LDS (the windows are no longer read) from position so,
  // where the output's 16-byte grid in memory falls, then store whole
  // chunks as one vector each (element stores for the parts of the end
  // chunks that belong to this tile)
  __syncthreads();
  const int64_t base = s_excl;
  const int so = (int)(((uintptr_t)(S + base) / sizeof(K)) & (CH - 1));
  int pos = so + incl - c;
#pragma unroll
  for (int s = 0; s < VT; ++s)
    if ((keep >> s) & 1u) keys[pos++] = out[s];
  __syncthreads();
  const int64_t room = cap - base;  // slots of S left from this tile's offset
  const int lim = room < (int64_t)total ? (room > 0 ? (int)room : 0) : total;
  if (lim > 0) {
    const int nc = (so + lim + CH - 1) / CH;
    for (int ci = tid; ci < nc; ci += NT) {
      const int w0 = ci * CH - so;  // tile position of the chunk's first key
      if (w0 >= 0 && w0 + CH <= lim) {
        __builtin_nontemporal_store(*reinterpret_cast<const u32x4 *>(keys + ci * CH),
                                    reinterpret_cast<u32x4 *>(S + (base + w0)));
      } else {
#pragma unroll
        for (int j = 0; j < CH; ++j)
          if (w0 + j >= 0 && w0 + j < lim) S[base + w0 + j] = keys[ci * CH + j];
      }
    }
  }
}

// Zero the look-back state: tile status words, the ticket counter and the
// output count.
__global__ void setop_init_kernel(unsigned long long *__restrict__ status, int64_t n_tiles,
                                  unsigned long long *__restrict__ ticket,
                                  int64_t *__restrict__ count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n_tiles) status[i] = 0;
  if (i == 0) {
    *ticket = 0;
    *count = 0;
  }
}

int64_t setop_tiles(int64_t n) { return (n + kSetTMin - 1) / kSetTMin; }

// Fixed device scratch of the allocation-free entry point (mp_set_op_noalloc):
// the splits, tile status words and ticket counter of one call, sized for
// na + nb up to kSetScratchKeys.  Each GPU the library runs on holds its own
// copy until the process ends.  In host code `scratch` names a host-side
// stand-in; its device address comes from hipGetSymbolAddress, once per
// device, and only that address is ever passed to a kernel.
static __device__ __align__(256) int64_t scratch[kSetScratchWords];

hipError_t setop_scratch_ptr(int64_t **out) {
  static std::mutex mu;
  static std::vector<int64_t *> per_device;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lock(mu);
  if ((int)per_device.size() <= dev) per_device.resize(dev + 1, nullptr);
  if (!per_device[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    per_device[dev] = (int64_t *)p;
  }
  *out = per_device[dev];
  return hipSuccess;
}

template <typename K>
hipError_t launch_set_op(int op, const K *A, int64_t na, const K *B, int64_t nb, K *S,
                         int64_t cap, int64_t *count, int64_t *ws, hipStream_t s) {
  constexpr int T = kSetNT * kSetVT<K>;
  const int64_t n_tiles = (na + nb + T - 1) / T;  // at most setop_tiles(na + nb)
  int64_t *splits = ws;
  unsigned long long *status = (unsigned long long *)(ws + (n_tiles + 1));
  unsigned long long *ticket = status + n_tiles;
  hipLaunchKernelGGL(setop_init_kernel, dim3((unsigned)((n_tiles + 256) / 256)), dim3(256), 0, s,
                     status, n_tiles, ticket, count);
  if (n_tiles == 0) return hipGetLastError();  // empty inputs: the count is 0
  hipError_t e = launch_partition<K>(A, na, B, nb, nullptr, T, n_tiles + 1, splits, s);
  if (e != hipSuccess) return e;
  auto run = [&](auto opc) {
    constexpr int OP = decltype(opc)::value;
    hipLaunchKernelGGL((setop_tile_kernel<K, OP>), dim3((unsigned)n_tiles), dim3(kSetNT), 0, s, A,
                       na, B, nb, splits, status, ticket, n_tiles, count, S, cap);
  };
  switch (op) {
    case 0: run(std::integral_constant<int, 0>()); break;
    case 1: run(std::integral_constant<int, 1>()); break;
    case 2: run(std::integral_constant<int, 2>()); break;
    case 3: run(std::integral_constant<int, 3>()); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

#define MP_INSTANTIATE(K)                                                               \
  template hipError_t launch_set_op<K>(int, const K *, int64_t, const K *, int64_t, K *, \
                                       int64_t, int64_t *, int64_t *, hipStream_t);
MP_INSTANTIATE(uint32_t)
MP_INSTANTIATE(int32_t)
MP_INSTANTIATE(uint64_t)
MP_INSTANTIATE(float)
#undef MP_INSTANTIATE

}  // namespace mp
