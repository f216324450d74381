// Inner join of two sorted inputs through the merge partition: every pair
// (i, j) with A[i] equal to B[j], ordered by i, then j.  The paper names
// database joins among the uses of the merge (introduction); here the merge
// path does the work twice.
//
// 1. Ranks (join_rank_kernel).  The merge's output tiles are cut by
//    Algorithm 2 on their diagonals and each tile's pair is walked in LDS as
//    in the merge (Theorem 17 for the lanes' splits, Lemma 1 for the walk).
//    When the walk takes A[i] its column b is the first B position whose key
//    is not below A[i] (ties take A first), so B's copies of A[i] are
//    B[b, b + c).  The walk records b per A key in LDS; then the first key
//    of every run of equal A keys reads c off the B window (a gallop in
//    LDS), and only the one value whose B run reaches past the window's end
//    continues in global memory.  Each A key gets lo[i] = b and c[i] = c,
//    written by consecutive lanes for consecutive keys.
// 2. Offsets: an exclusive scan of c over A gives each A key the position of
//    its first pair, and the total, which goes to *count.  The rank tiles
//    already add their counts into the scan's block sums.
// 3. Pairs (join_emit_kernel), balanced whatever the duplicates: output p
//    belongs to the last A key i with off[i] <= p.  That is again a merge:
//    of off[] (non-decreasing) with the output indices 0, 1, 2, ..., ties
//    taking off[] first, and output p then lies in the rows of key i at
//    column p - off[i].  So the emission is cut like a Merge Path merge of
//    those two sequences: tiles of E items of the combined grid (keys and
//    pairs together) split by Algorithm 2.  Inside a tile, consecutive lanes
//    take consecutive outputs and find their key by a search over the
//    tile's offsets in LDS, so the pairs are stored coalesced.  The number
//    of tiles is only known on the device (it depends on the count), so a
//    grid of resident workgroups walks them.
#include <stdint.h>

#include "mp_device.h"
#include "mp_internal.h"

namespace mp {

namespace {

constexpr int kJoinNT = 256, kJoinVT = 8, kJoinT = kJoinNT * kJoinVT;   // rank tiles
constexpr int kEmitNT = 256, kEmitE = 2048;                               // emission tiles
constexpr int kEmitG = 8, kEmitCB = 31;  // emission splits: lanes per boundary, tiles per chunk
constexpr int kScanPer = 4;                                              // keys per scan lane
constexpr int64_t kScanBlock = 1024 * kScanPer;

template <typename K>
__device__ __forceinline__ bool key_equal(K x, K y) {
  return !(x < y) && !(y < x);
}

// The chunk X[g, g + CH) of an array of lim keys.  Chunks sit on a grid
// aligned to 16 bytes in memory, so one that lies inside the array is one
// nontemporal vector load; at the array's ends (g may be negative) only the
// keys inside it are read.
template <typename K>
__device__ __forceinline__ void join_load_chunk(const K *__restrict__ X, int64_t g, int64_t lim,
                                                K (&v)[16 / sizeof(K)]) {
  constexpr int CH = 16 / (int)sizeof(K);
  if (g >= 0 && g + CH <= lim) {
    *reinterpret_cast<u32x4 *>(v) =
        __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(X + g));
  } else {
#pragma unroll
    for (int j = 0; j < CH; ++j) v[j] = g + j >= 0 && g + j < lim ? X[g + j] : K{};
  }
}

// First index in [lo, hi) of B whose key is above v (hi if none); B is
// sorted.  Galloping from lo, then a binary search, so a short run costs
// few probes.
template <typename K>
__device__ int64_t upper_from(const K *__restrict__ B, int64_t lo, int64_t hi, K v) {
  int64_t step = 1, base = lo;
  while (base + step <= hi && !(v < B[base + step - 1])) {
    base += step;
    step <<= 1;
  }
  int64_t l = base, h = base + step - 1 < hi ? base + step - 1 : hi;
  while (l < h) {
    const int64_t m = l + ((h - l) >> 1);
    if (v < B[m]) h = m; else l = m + 1;
  }
  return l;
}

// Phase 1: per A key, its first column in B and the length of its B run.
template <typename K>
__global__ __launch_bounds__(kJoinNT) void join_rank_kernel(
    const K *__restrict__ A, int64_t na, const K *__restrict__ B, int64_t nb,
    const int64_t *__restrict__ a_split, int64_t n_tiles, int64_t *__restrict__ lo_out,
    int64_t *__restrict__ cnt_out, int64_t *__restrict__ bsum) {
  constexpr int NT = kJoinNT, VT = kJoinVT, T = kJoinT;
  constexpr int CH = 16 / (int)sizeof(K);
  // both windows' chunks (at most T + 4 CH - 4 keys) and the slack the walk
  // reads past the end of B's window
  __shared__ __align__(16) K keys[T + 4 * CH + VT + 1];
  __shared__ int32_t s_lo[T];   // per A key of the window: first B column, from b0
  // per A key of the window: for the first key of a run of equal keys (a
  // head), -(c + 2) with c the B run length of its value in the window (-1:
  // past it); for any other key, the index of its head
  __shared__ int32_t s_cnt[T];
  __shared__ int32_t s_wmax[NT / 64];
  __shared__ int64_t s_big;     // the B run length of the value that goes past it
  __shared__ int64_t s_part[2][NT / 64];
  const int tid = threadIdx.x;
  const int64_t tile = blockIdx.x;
  const int64_t N = na + nb;
  const int64_t d0 = tile * T;
  const int64_t d1 = d0 + T < N ? d0 + T : N;
  const int n = (int)(d1 - d0);
  // the tile's pair, clamped as in the merge so every access stays in bounds
  const int64_t lo0 = d0 > nb ? d0 - nb : 0, hi0 = d0 < na ? d0 : na;
  int64_t a0 = a_split[tile];
  a0 = a0 < lo0 ? lo0 : (a0 > hi0 ? hi0 : a0);
  const int64_t b0 = d0 - a0;
  int64_t wa64 = a_split[tile + 1] - a0;
  const int64_t wa_lo = d1 - nb - a0 > 0 ? d1 - nb - a0 : 0;
  const int64_t wa_hi = na - a0 < (int64_t)n ? na - a0 : (int64_t)n;
  wa64 = wa64 < wa_lo ? wa_lo : (wa64 > wa_hi ? wa_hi : wa64);
  const int wa = (int)wa64, wb = n - wa;
  const int64_t b1 = b0 + wb;  // first B key after the window
  // 16-byte chunks on a grid aligned in memory, stored whole into LDS: A's
  // from position 0 and B's after them, so A[a0] sits at oa and B[b0] at
  // ob, and the windows end at ae and be
  const int sa = (int)(((uintptr_t)(A + a0) / sizeof(K)) & (CH - 1));
  const int sb = (int)(((uintptr_t)(B + b0) / sizeof(K)) & (CH - 1));
  const int ca = (sa + wa + CH - 1) / CH, cb = (sb + wb + CH - 1) / CH;
  const int oa = sa, ob = ca * CH + sb, ae = oa + wa, be = ob + wb;
  {
    constexpr int PV = (T / CH + 4 + NT - 1) / NT;  // ca + cb <= T / CH + 3
    K r[PV][CH];
#pragma unroll
    for (int k = 0; k < PV; ++k) {
      const int c = tid + k * NT;
      if (c < ca + cb) {
        const bool fb = c >= ca;
        const int64_t g = fb ? b0 - sb + (int64_t)(c - ca) * CH : a0 - sa + (int64_t)c * CH;
        join_load_chunk<K>(fb ? B : A, g, fb ? nb : na, r[k]);
      }
    }
#pragma unroll
    for (int k = 0; k < PV; ++k) {
      const int c = tid + k * NT;
      if (c < ca + cb)
        *reinterpret_cast<u32x4 *>(keys + c * CH) = *reinterpret_cast<const u32x4 *>(r[k]);
    }
  }
  if (tid == 0) s_big = 0;
  __syncthreads();
  // the walk: each A key's first B column (ties take A, so every B key
  // before it is smaller).  All VT steps run: past the lane's own outputs
  // the walk follows the same path as the next lane and records the same
  // columns, and past the tile's end it takes nothing from A (LDS reads stay
  // below be + VT + 1).
  {
    const int dl = tid * VT < n ? tid * VT : n;
    int lo, hi;
    diag_range<int>(dl, wa, wb, lo, hi);
    const int a = split_search<int>(
        dl, lo, hi, [&](int i) { return keys[oa + i]; }, [&](int j) { return keys[ob + j]; });
    int ai = oa + a, bi = ob + (dl - a);
    K ka = keys[ai], kb = keys[bi];
#pragma unroll
    for (int s = 0; s < VT; ++s) {
      const bool take_b = (bi < be) && (ai >= ae || kb < ka);
      if (!take_b && ai < ae) s_lo[ai - oa] = bi - ob;
      const int taken = take_b ? bi : ai;
      ai = take_b ? ai : taken + 1;
      bi = take_b ? taken + 1 : bi;
      const K nxt = keys[taken + 1];
      ka = take_b ? ka : nxt;
      kb = take_b ? nxt : kb;
    }
  }
  // each A key's head (the first key of its run of equal keys in the
  // window) by a segmented max-scan: lane t takes keys [t VT, t VT + VT),
  // keeps the last head it has seen, and adds the last head of the lanes
  // before it (a wavefront scan, then the wavefronts' maxima through LDS)
  const int i0 = tid * VT;
  int hd[VT];
  {
    int run = -1;
    K prev = i0 > 0 && i0 <= wa ? keys[oa + i0 - 1] : K{};
#pragma unroll
    for (int j = 0; j < VT; ++j) {
      const int i = i0 + j;
      const K v = keys[oa + i];
      const bool head = i < wa && (i == 0 || !key_equal(prev, v));
      run = head ? i : run;
      hd[j] = run;
      prev = v;
    }
    const int lane = tid & 63;
    int incl = run;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int y = __shfl_up(incl, o);
      incl = lane >= o && y > incl ? y : incl;
    }
    const int before = __shfl_up(incl, 1);
    if (lane == 63) s_wmax[tid >> 6] = incl;
    __syncthreads();
    int carry = lane > 0 ? before : -1;
    for (int w = 0; w < (tid >> 6); ++w) carry = s_wmax[w] > carry ? s_wmax[w] : carry;
#pragma unroll
    for (int j = 0; j < VT; ++j) hd[j] = hd[j] > carry ? hd[j] : carry;
  }
  // non-heads record their head's index
#pragma unroll
  for (int j = 0; j < VT; ++j)
    if (i0 + j < wa && hd[j] != i0 + j) s_cnt[i0 + j] = hd[j];
  // run heads: the length of the B run of their value, galloping in the
  // window from the first column; only the value equal to the window's last
  // B key can go on past it
  for (int i = tid; i < wa; i += NT) {
    const K v = keys[oa + i];
    if (i > 0 && key_equal(keys[oa + i - 1], v)) continue;
    const int j0 = ob + (s_lo[i] < 0 ? 0 : (s_lo[i] > wb ? wb : s_lo[i]));
    int l = j0;
    if (j0 < be && key_equal(keys[j0], v)) {
      int base = j0, step = 1;
      while (base + step < be && key_equal(keys[base + step], v)) {
        base += step;
        step <<= 1;
      }
      int lo2 = base + 1, hi2 = base + step < be ? base + step : be;
      while (lo2 < hi2) {
        const int m = (lo2 + hi2) >> 1;
        if (key_equal(keys[m], v)) lo2 = m + 1; else hi2 = m;
      }
      l = lo2;
    }
    int c = l - j0;
    if (l == be && b1 < nb && key_equal(B[b1], v)) {
      s_big = c + (upper_from(B, b1, nb, v) - b1);
      c = -1;
    }
    s_cnt[i] = -(c + 2);
  }
  __syncthreads();
  // every A key of the window: its column, and its run head's count.  The
  // counts also add up per scan block of A: a window of at most T keys
  // touches at most two blocks, blk0 and the next, which starts at key
  // i_split of the window.
  const int64_t blk0 = a0 / kScanBlock;
  const int64_t next_blk = (blk0 + 1) * kScanBlock - a0;
  const int i_split = next_blk < wa ? (int)next_blk : wa;
  int64_t part_all = 0, part1 = 0;
  for (int i = tid; i < wa; i += NT) {
    const int e = s_cnt[i];
    const int c = -s_cnt[e >= 0 ? e : i] - 2;  // a non-head reads its head's entry
    const int rl = s_lo[i] < 0 ? 0 : (s_lo[i] > wb ? wb : s_lo[i]);
    lo_out[a0 + i] = b0 + rl;
    const int64_t cv = c >= 0 ? (int64_t)c : s_big;
    cnt_out[a0 + i] = cv;
    part_all += cv;
    part1 += i >= i_split ? cv : 0;
  }
  int64_t part0 = part_all - part1;
  // A keys between this window and the next tile's, which no tile visits
  // (none for sorted inputs, whose splits increase), get no pairs; so every
  // count is defined without clearing all of them first
  if (tile + 1 < n_tiles) {
    const int64_t lo0n = d1 > nb ? d1 - nb : 0, hi0n = d1 < na ? d1 : na;
    int64_t a0n = a_split[tile + 1];
    a0n = a0n < lo0n ? lo0n : (a0n > hi0n ? hi0n : a0n);
    for (int64_t i = a0 + wa + tid; i < a0n; i += NT) cnt_out[i] = 0;
  }
  // the two partial block sums over the workgroup, added into the scan's
  // block sums (zeroed before this kernel; one atomic per touched block, at
  // addresses of their own).  Every nonzero count left in cnt_out was added
  // by the tile that wrote it, so a block sum is never below its counts'
  // sum and the offsets stay non-decreasing even for unsorted inputs.
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    part0 += __shfl_xor(part0, o);
    part1 += __shfl_xor(part1, o);
  }
  if ((tid & 63) == 0) {
    s_part[0][tid >> 6] = part0;
    s_part[1][tid >> 6] = part1;
  }
  __syncthreads();
  if (tid == 0) {
    int64_t p0 = 0, p1 = 0;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) {
      p0 += s_part[0][w];
      p1 += s_part[1][w];
    }
    if (p0 != 0) atomicAdd((unsigned long long *)&bsum[blk0], (unsigned long long)p0);
    if (p1 != 0) atomicAdd((unsigned long long *)&bsum[blk0 + 1], (unsigned long long)p1);
  }
}

// Zeroes the scan's block sums, which the rank tiles add into.
__global__ void join_zero_kernel(int64_t *__restrict__ p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

// Phase 2a is in the rank kernel: each tile adds its counts into the sums
// of the blocks of kScanBlock A keys it touches.
// Phase 2b (one workgroup): block sums to exclusive block offsets; the
// grand total goes to *count.
__global__ __launch_bounds__(1024) void join_scan_blocks_kernel(int64_t *__restrict__ bsum,
                                                                int64_t n_blocks,
                                                                int64_t *__restrict__ total_out,
                                                                int64_t *__restrict__ count) {
  int64_t carry = 0;
  for (int64_t b0 = 0; b0 < n_blocks; b0 += 1024) {
    const int64_t b = b0 + threadIdx.x;
    const int64_t v = b < n_blocks ? bsum[b] : 0;
    int64_t total;
    const int64_t incl = workgroup_scan1024(v, &total);
    __syncthreads();
    if (b < n_blocks) bsum[b] = carry + incl - v;
    carry += total;
  }
  if (threadIdx.x == 0) {
    *total_out = carry;
    *count = carry;
  }
}

// Phase 2c: counts to exclusive offsets, in place.
__global__ __launch_bounds__(1024) void join_scan_apply_kernel(int64_t *__restrict__ cnt, int64_t n,
                                                               const int64_t *__restrict__ bsum) {
  const int64_t k0 = (int64_t)blockIdx.x * kScanBlock + (int64_t)threadIdx.x * kScanPer;
  int64_t c[kScanPer], sum = 0;
#pragma unroll
  for (int i = 0; i < kScanPer; ++i) {
    c[i] = k0 + i < n ? cnt[k0 + i] : 0;
    sum += c[i];
  }
  int64_t total;
  int64_t t = workgroup_scan1024(sum, &total) - sum + bsum[blockIdx.x];
#pragma unroll
  for (int i = 0; i < kScanPer; ++i) {
    if (k0 + i < n) cnt[k0 + i] = t;
    t += c[i];
  }
}

// Phase 3: the pairs.  off[0..na) offsets, off[na] the total (ws), lo[]
// the first B column of every A key.  Each resident workgroup takes a
// contiguous range of the tiles of the combined grid (na keys + total
// pairs).  It finds the splits on its tiles' boundaries up front, kEmitCB + 1
// at a time with kEmitG lanes each, so the searches' dependent loads overlap
// one another instead of starting every tile.
__global__ __launch_bounds__(kEmitNT) void join_emit_kernel(const int64_t *__restrict__ off,
                                                            const int64_t *__restrict__ lo_col,
                                                            int64_t na, int64_t *__restrict__ I,
                                                            int64_t *__restrict__ J, int64_t cap) {
  constexpr int NT = kEmitNT, E = kEmitE, G = kEmitG, CB = kEmitCB;
  static_assert((CB + 1) * G <= NT, "one group of lanes per boundary of a chunk");
  // off and lo of keys [a0 - 1, a1) (slot 0 is the key before the tile)
  __shared__ int64_t s_off[E + 2], s_lo[E + 2];
  __shared__ int64_t s_bnd[CB + 1];  // splits on the chunk's boundaries
  const int tid = threadIdx.x;
  const int64_t total = off[na];
  const int64_t N = na + total;  // items of the combined grid
  // A tile starting at item d0 emits outputs from d0 - na on, so tiles with
  // d0 >= cap + na hold no output below cap: the walk stops before them
  // (the work stays bounded by the caller's room, whatever the count).
  const int64_t n_all = (N + E - 1) / E, n_room = (cap + na + E - 1) / E;
  const int64_t n_tiles = n_all < n_room ? n_all : n_room;
  const int64_t t_begin = n_tiles * blockIdx.x / gridDim.x;
  const int64_t t_end = n_tiles * (blockIdx.x + 1) / gridDim.x;
  for (int64_t c0 = t_begin; c0 < t_end; c0 += CB) {
    const int64_t c1 = c0 + CB < t_end ? c0 + CB : t_end;
    // the split on diagonal d: off entries among the first d items (ties
    // take off first: output p comes after every key with off <= p); a
    // group of G lanes per boundary c0 .. c1
    const int g = tid / G;
    if (g <= c1 - c0) {
      const int64_t d = (c0 + g) * E < N ? (c0 + g) * E : N;
      int64_t l, h;
      diag_range<int64_t>(d, na, total, l, h);
      const int64_t a = group_split_search<G, int64_t>(
          d, l, h, [&](int64_t i) { return off[i]; }, [&](int64_t j) { return j; });
      if (tid % G == 0) s_bnd[g] = a;
    }
    __syncthreads();
    // off and lo of tile t's keys, loaded into registers one tile ahead so
    // that the loads overlap the previous tile's stores
    constexpr int PR = (E + 1 + NT - 1) / NT;
    int64_t r_off[PR], r_lo[PR];
    auto fetch = [&](int64_t t) {
      const int64_t a0 = s_bnd[t - c0];
      const int wa = (int)(s_bnd[t - c0 + 1] - a0);
#pragma unroll
      for (int k = 0; k < PR; ++k) {
        const int i = tid + k * NT;
        const int64_t key = a0 - 1 + i;
        r_off[k] = i <= wa && key >= 0 ? off[key] : 0;
        r_lo[k] = i <= wa && key >= 0 ? lo_col[key] : 0;
      }
    };
    fetch(c0);
    for (int64_t t = c0; t < c1; ++t) {
      const int64_t d0 = t * E;
      const int64_t d1 = d0 + E < N ? d0 + E : N;
      const int64_t a0 = s_bnd[t - c0], a1 = s_bnd[t - c0 + 1];
      const int64_t p0 = d0 - a0;  // first output of the tile
      const int wa = (int)(a1 - a0);
      const int n_out = (int)(d1 - d0) - wa;  // outputs p0 .. p0 + n_out - 1
#pragma unroll
      for (int k = 0; k < PR; ++k) {
        const int i = tid + k * NT;
        if (i <= wa) {
          s_off[i] = r_off[k];
          s_lo[i] = r_lo[k];
        }
      }
      __syncthreads();
      if (t + 1 < c1) fetch(t + 1);
      // output p belongs to the last key with off <= p: slot 0 (key a0 - 1)
      // has off <= p0, slots 1 .. wa are the tile's keys
      for (int q = tid; q < n_out; q += NT) {
        const int64_t p = p0 + q;
        int l = 0, r = wa;  // last slot in [0, wa] with s_off <= p
        while (l < r) {
          const int m = (l + r + 1) >> 1;
          if (s_off[m] <= p) l = m; else r = m - 1;
        }
        if (p < cap) {
          I[p] = a0 - 1 + l;
          J[p] = s_lo[l] + (p - s_off[l]);
        }
      }
      __syncthreads();  // the LDS windows are reused by the next tile
    }
  }
}

}  // namespace

// Workspace: first B column per A key (na), counts then offsets (na + 1),
// block sums of the scan, and the splits of the rank tiles.
int64_t join_ws_bytes(int64_t na, int64_t nb) {
  const int64_t n_blocks = (na + kScanBlock - 1) / kScanBlock;
  const int64_t n_tiles = (na + nb + kJoinT - 1) / kJoinT;
  return 8 * (na + (na + 1) + n_blocks + (n_tiles + 1));
}

template <typename K>
hipError_t launch_join(const K *A, int64_t na, const K *B, int64_t nb, int64_t *I, int64_t *J,
                       int64_t cap, int64_t *count, int64_t *ws, hipStream_t s) {
  const int64_t n_blocks = (na + kScanBlock - 1) / kScanBlock;
  const int64_t n_tiles = (na + nb + kJoinT - 1) / kJoinT;
  int64_t *lo = ws, *off = lo + na, *bsum = off + (na + 1), *splits = bsum + n_blocks;
  hipError_t e = hipSuccess;
  if (n_blocks > 0)
    hipLaunchKernelGGL(join_zero_kernel, dim3((unsigned)((n_blocks + 255) / 256)), dim3(256), 0, s,
                       bsum, n_blocks);
  if (n_tiles > 0) {
    e = launch_partition<K>(A, na, B, nb, nullptr, kJoinT, n_tiles + 1, splits, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((join_rank_kernel<K>), dim3((unsigned)n_tiles), dim3(kJoinNT), 0, s, A, na,
                       B, nb, splits, n_tiles, lo, off, bsum);
  }
  // (with no A keys the scan still writes the zero total)
  hipLaunchKernelGGL(join_scan_blocks_kernel, dim3(1), dim3(1024), 0, s, bsum, n_blocks, off + na,
                     count);
  if (n_blocks > 0)
    hipLaunchKernelGGL(join_scan_apply_kernel, dim3((unsigned)n_blocks), dim3(1024), 0, s, off, na,
                       bsum);
  if (na > 0 && cap > 0) {
    // resident workgroups (four per CU: 33 KB of LDS each) walk contiguous
    // ranges of the emission tiles
    const int grid = 4 * device_cu_count();
    hipLaunchKernelGGL(join_emit_kernel, dim3((unsigned)grid), dim3(kEmitNT), 0, s, off, lo, na, I,
                       J, cap);
  }
  return hipGetLastError();
}

#define MP_INSTANTIATE(K)                                                                    \
  template hipError_t launch_join<K>(const K *, int64_t, const K *, int64_t, int64_t *,      \
                                     int64_t *, int64_t, int64_t *, int64_t *, hipStream_t);
MP_INSTANTIATE(uint32_t)
MP_INSTANTIATE(int32_t)
MP_INSTANTIATE(uint64_t)
MP_INSTANTIATE(float)
#undef MP_INSTANTIATE

}  // namespace mp
