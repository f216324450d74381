// Per-tile merge: Algorithm 1 with one workgroup per output tile.
//
// Step 1 (tile_splits_kernel): the split on every tile boundary diagonal
// k * T is found by Algorithm 2 (one lane, or a group of lanes cutting the
// interval more ways per round, per diagonal; Theorem 14 bounds the rounds).
// Step 2 (merge_tile_kernel): each workgroup takes the pair that its two
// splits cut out of A and B (Theorem 5: it merges to exactly the tile's
// range of S), stages it in LDS with 16-byte loads, finds every lane's split
// at local diagonal lane * VT inside it (Theorem 17), merges VT outputs per
// lane in registers (Lemma 1; ties take A) and writes the tile through an
// LDS transpose with 16-byte stores.
//
// The splits travel from step 1 to step 2 inside S itself: tile k's pair
// (a0, b0, a1, b1) is written into the first 32 bytes of tile k's own output
// range, which no other tile reads or writes; tile k's workgroup reads them
// before it stores anything there.  So the merge needs no memory beyond its
// inputs and output, and concurrent calls on different streams share
// nothing.  A last tile shorter than 32 bytes gets no header; its end split
// is the end of the grid (or of its run pair), and its start split is found
// by stepping the path backwards from there (fewer than 8 steps).
//
// Layouts: kSingle merges (A, B); kRuns is one round of merge sort over X:
// pair k is (X[2wk, 2wk+w), X[2wk+w, 2wk+2w)) clipped to n, left run as A
// (stable), and tiles (a power of two dividing 2w) never cross a pair end,
// so every tile is again one plain pair of ranges of X.  kBatch is a batch
// of independent pairs given by CSR offsets (Corollary 6 pair by pair),
// merged as one merge of the concatenated inputs in (pair, key) order: its
// tiles of T outputs cross pair ends, each is one contiguous window of A and
// of B, and a lane whose outputs cross a pair end switches pairs there.  Its
// splits and the pair of each tile's first output go to the caller's
// workspace (a batch has one, and a tile can be shorter than a header only
// at the very end).
#pragma once

#include "mp_device.h"
#include "mp_internal.h"

namespace mp {

enum TileKind { kTileSingle = 0, kTileRuns = 1, kTileBatch = 2 };
enum TileSrc { kTileHeader = 0, kTileSplitArray = 1, kTileSearch = 2 };

template <typename K>
struct TileArgs {
  const K *A, *B;           // kTileRuns: both are X
  const uint32_t *Av, *Bv;  // values (key-value merges only)
  K *S;
  uint32_t *Sv;
  int64_t NA, NB;           // lengths of A and B (kTileRuns: n and n)
  int64_t N;                // outputs (kTileSingle: NA + NB; kTileRuns: n)
  int lw;                   // kTileRuns: log2 of the run width
  const int64_t *a_split;   // kTileSplitArray: the splits of the tiles
  int64_t n_tiles;
  // kTileBatch
  const int64_t *a_off, *b_off;  // CSR offsets of the pairs (n_pairs + 1)
  int64_t n_pairs;
  int64_t *split_out;       // the splits step 1 writes (n_tiles + 1; workspace)
  int32_t *tile_pair;       // pair holding each tile's first output (workspace)
};

// Pair k of a batch with its offsets kept inside the arrays and
// non-decreasing (no-ops for valid offsets): A[a0, a1) and B[b0, b1).
template <typename K>
__device__ __forceinline__ void batch_pair(const TileArgs<K> &P, int64_t k, int64_t &a0,
                                           int64_t &a1, int64_t &b0, int64_t &b1) {
  auto clamp = [](int64_t v, int64_t lo, int64_t hi) { return v < lo ? lo : (v > hi ? hi : v); };
  a0 = clamp(P.a_off[k], 0, P.NA);
  a1 = clamp(P.a_off[k + 1], a0, P.NA);
  b0 = clamp(P.b_off[k], 0, P.NB);
  b1 = clamp(P.b_off[k + 1], b0, P.NB);
}

// ---- a batch as one merge of its concatenations ---------------------------
// With pair k owning A[a_off(k), a_off(k+1)), B[b_off(k), b_off(k+1)) and
// the outputs [o(k), o(k+1)), o(k) = a_off(k) + b_off(k), the batch is one
// merge of the concatenated A and B in the order (pair, key): the split on a
// global diagonal D inside pair p is (a_off(p) + a, b_off(p) + D - o(p) - a)
// with a the split of pair p on its own diagonal D - o(p), and A + B counts
// add up to D again.  So the batch is cut into tiles of T outputs like a
// single merge, each tile one contiguous window of A and of B, and only a
// lane whose outputs cross a pair end needs to know more.

// Offsets of pair k's start, kept inside the arrays (no-ops when valid).
template <typename K>
__device__ __forceinline__ int64_t batch_a_at(const TileArgs<K> &P, int64_t k) {
  const int64_t v = P.a_off[k];
  return v < 0 ? 0 : (v > P.NA ? P.NA : v);
}
template <typename K>
__device__ __forceinline__ int64_t batch_b_at(const TileArgs<K> &P, int64_t k) {
  const int64_t v = P.b_off[k];
  return v < 0 ? 0 : (v > P.NB ? P.NB : v);
}

// The pair holding global output D, searched from pair p (o(p) <= D): the
// last k in [p, n_pairs) with o(k) <= D, galloping from p then bisecting
// (one probe when D lies in pair p).
template <typename K>
__device__ __forceinline__ int64_t batch_pair_of(const TileArgs<K> &P, int64_t p, int64_t D) {
  int64_t step = 1;
  while (p + step < P.n_pairs && batch_a_at(P, p + step) + batch_b_at(P, p + step) <= D) {
    p += step;
    step <<= 1;
  }
  int64_t lo = p + 1, hi = p + step < P.n_pairs ? p + step : P.n_pairs;
  while (lo < hi) {
    const int64_t mid = lo + ((hi - lo) >> 1);
    if (batch_a_at(P, mid) + batch_b_at(P, mid) <= D) lo = mid + 1;
    else hi = mid;
  }
  return lo - 1;
}

// Pair holding the first output of every tile: each nonempty pair k writes
// itself for the tiles that start inside [o(k), o(k+1)).
template <typename K>
__global__ __launch_bounds__(256) void batch_bound_kernel(TileArgs<K> P, int64_t T) {
  const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (k >= P.n_pairs) return;
  int64_t a0, a1, b0, b1;
  batch_pair(P, k, a0, a1, b0, b1);
  const int64_t o0 = a0 + b0, o1 = a1 + b1;
  const int64_t t_end = (o1 + T - 1) / T < P.n_tiles ? (o1 + T - 1) / T : P.n_tiles;
  for (int64_t t = (o0 + T - 1) / T; t < t_end; ++t) P.tile_pair[t] = (int32_t)k;
}

// Header bytes at the start of each tile's range of S.
constexpr int kTileHdrBytes = 32;

template <typename K>
__device__ __forceinline__ void put_tile_hdr(K *S, int64_t d, int slot, int64_t a, int64_t b) {
  uint32_t *w = reinterpret_cast<uint32_t *>(S + d) + 4 * slot;
  const u32x4 v = {(uint32_t)a, (uint32_t)((uint64_t)a >> 32), (uint32_t)b,
                   (uint32_t)((uint64_t)b >> 32)};
  if (((uintptr_t)w % 16) == 0) {
    *reinterpret_cast<u32x4 *>(w) = v;  // one 16-byte store (S aligned)
  } else {
    w[0] = v.x;
    w[1] = v.y;
    w[2] = v.z;
    w[3] = v.w;
  }
}

template <typename K>
__device__ __forceinline__ int64_t tile_bytes(const TileArgs<K> &P, int64_t T, int64_t t) {
  const int64_t r = P.N - t * T;
  return (r < T ? r : T) * (int64_t)sizeof(K);
}

// Run pair of output d in a merge-sort round: its first output P0 and the
// ranges [P0, aE) (left run, A) and [aE, bE) (right run, B) of X.
__device__ __forceinline__ void run_pair(int64_t d, int64_t n, int lw, int64_t &P0, int64_t &aE,
                                         int64_t &bE) {
  const int64_t w = (int64_t)1 << lw;
  P0 = (d >> (lw + 1)) << (lw + 1);
  aE = P0 + w < n ? P0 + w : n;
  bE = P0 + 2 * w < n ? P0 + 2 * w : n;
}

// Step 1.  Boundary k = 0 .. n_tiles (diagonal min(k * T, N)); G lanes per
// boundary.  Writes the split as tile k's start and tile k - 1's end.
template <typename K, int KIND, int G>
__global__ __launch_bounds__(256) void tile_splits_kernel(TileArgs<K> P, int64_t T) {
  const int64_t k = ((int64_t)blockIdx.x * 256 + threadIdx.x) / G;
  auto search = [&](int64_t d, int64_t lo, int64_t hi, auto ga, auto gb) -> int64_t {
    if constexpr (G == 1) return split_search<int64_t>(d, lo, hi, ga, gb);
    else return group_split_search<G, int64_t>(d, lo, hi, ga, gb);
  };
  if constexpr (KIND == kTileBatch) {
    // boundary k: the global split on diagonal min(kT, N), found in the
    // pair holding output kT
    if (k > P.n_tiles) return;  // a group exits as one
    const int64_t D = k * T < P.N ? k * T : P.N;
    int64_t a = P.NA;
    if (D < P.N) {
      int64_t pk = P.tile_pair[k];
      pk = pk < 0 ? 0 : (pk >= P.n_pairs ? P.n_pairs - 1 : pk);
      int64_t a0, a1, b0, b1;
      batch_pair(P, pk, a0, a1, b0, b1);
      const int64_t size = (a1 - a0) + (b1 - b0);
      int64_t dl = D - (a0 + b0);
      dl = dl < 0 ? 0 : (dl > size ? size : dl);
      int64_t lo, hi;
      diag_range<int64_t>(dl, a1 - a0, b1 - b0, lo, hi);
      const K *A = P.A + a0, *B = P.B + b0;
      a = a0 + search(dl, lo, hi, [&](int64_t i) { return A[i]; }, [&](int64_t q) { return B[q]; });
    }
    if constexpr (G > 1) {
      if ((threadIdx.x & (G - 1)) != 0) return;
    }
    P.split_out[k] = a;
    return;
  } else {
  if (k > P.n_tiles) return;  // a group exits as one (G divides 256)
  const int64_t N = P.N;
  const int64_t D = k * T < N ? k * T : N;
  int64_t sa, sb, ea, eb;  // start of tile k, end of tile k - 1
  if constexpr (KIND == kTileSingle) {
    int64_t lo, hi;
    diag_range<int64_t>(D, P.NA, P.NB, lo, hi);
    const K *A = P.A, *B = P.B;
    sa = search(D, lo, hi, [&](int64_t i) { return A[i]; }, [&](int64_t j) { return B[j]; });
    sb = D - sa;
    ea = sa;
    eb = sb;
  } else {
    const K *X = P.A;
    const int64_t w = (int64_t)1 << P.lw;
    int64_t P0, aE, bE;
    if (D == N) {
      // end of the last pair
      run_pair(N - 1, N, P.lw, P0, aE, bE);
      sa = ea = aE;
      sb = eb = bE;
    } else {
      run_pair(D, N, P.lw, P0, aE, bE);
      const int64_t dl = D - P0;
      int64_t lo, hi;
      diag_range<int64_t>(dl, aE - P0, bE - aE, lo, hi);
      const int64_t a = search(dl, lo, hi, [&](int64_t i) { return X[P0 + i]; },
                               [&](int64_t j) { return X[aE + j]; });
      sa = P0 + a;
      sb = aE + (dl - a);
      if (D == P0 && D > 0) {
        // tile k - 1 ends its own pair: that pair's two run ends
        ea = P0 - w;
        eb = P0;
      } else {
        ea = sa;
        eb = sb;
      }
    }
  }
  if constexpr (G > 1) {
    if ((threadIdx.x & (G - 1)) != 0) return;
  }
  if (k < P.n_tiles && tile_bytes(P, T, k) >= kTileHdrBytes) put_tile_hdr(P.S, k * T, 0, sa, sb);
  if (k > 0 && tile_bytes(P, T, k - 1) >= kTileHdrBytes) put_tile_hdr(P.S, (k - 1) * T, 1, ea, eb);
  }
}

// Chunk of CH elements at src + g: one vector access when the chunk lies
// inside the array (lim elements), element loads for the part inside else.
// Vector loads are nontemporal: every window is read once, in long streams.
template <typename T, int CH>
__device__ __forceinline__ void tile_load_chunk(const T *__restrict__ src, int64_t g, int64_t lim,
                                                T (&v)[CH]) {
  typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
  if (g + CH <= lim) {
    if constexpr (CH * sizeof(T) == 16) {
      const u32x4 *p = reinterpret_cast<const u32x4 *>(src + g);
      *reinterpret_cast<u32x4 *>(v) = __builtin_nontemporal_load(p);
    } else if constexpr (CH * sizeof(T) == 8) {
      const u32x2 *p = reinterpret_cast<const u32x2 *>(src + g);
      *reinterpret_cast<u32x2 *>(v) = __builtin_nontemporal_load(p);
    } else {
#pragma unroll
      for (int i = 0; i < CH; ++i) v[i] = src[g + i];
    }
  } else {
#pragma unroll
    for (int i = 0; i < CH; ++i) v[i] = g + i < lim ? src[g + i] : T{};
  }
}

template <typename T, int CH>
__device__ __forceinline__ void tile_put_chunk(T *lds, const T (&v)[CH]) {
  if constexpr (CH * sizeof(T) == 16) {
    *reinterpret_cast<u32x4 *>(lds) = *reinterpret_cast<const u32x4 *>(v);
  } else if constexpr (CH * sizeof(T) == 8) {
    *reinterpret_cast<uint2 *>(lds) = *reinterpret_cast<const uint2 *>(v);
  } else {
#pragma unroll
    for (int i = 0; i < CH; ++i) lds[i] = v[i];
  }
}

// LDS of one tile: keys (and values) of both windows, in chunks, plus the
// slack the unguarded tail of the serial merge may read.
template <typename K, bool KV, int NT, int VT, bool VLOAD>
struct TileLds {
  static constexpr int T = NT * VT;
  static constexpr int CH = VLOAD ? 16 / (int)sizeof(K) : 1;
  static constexpr int N_KEYS = T + 4 * CH + VT + 1;
  static constexpr int N_VALS = KV ? T + 4 * CH : 1;
  static constexpr size_t bytes = (size_t)N_KEYS * sizeof(K) + (size_t)N_VALS * 4;
};
// Tile shapes needing more than 96 KB of LDS are not built.
template <typename K, bool KV, int NT, int VT>
constexpr bool tile_shape_fits() {
  return TileLds<K, KV, NT, VT, true>::bytes <= 96 * 1024;
}

// Tile of workgroup b among G.  Workgroups are dealt to the 8 XCDs in turn
// (b mod 8), each XCD with its own L2; this bijection gives XCD x one
// contiguous range of tiles, so each XCD streams its own stretch of A, B and
// S (measured: 0.698 against about 0.74 ms for the 2^28 + 2^28 u32 tile
// merge, together with nontemporal window loads).
__device__ __forceinline__ int64_t tile_of_block(int64_t b, int64_t G) {
  const int64_t q = G >> 3, r = G & 7, x = b & 7, i = b >> 3;
  return x * q + (x < r ? x : r) + i;
}

// Serial merge of VT outputs of a batch tile for a lane whose outputs cross
// the end of its pair.  A pair's part of the tile is the merge of its parts
// of the two windows; where the lane's part ends (seg, the outputs left in
// it, reaches 0) next(cur, ...) moves it to the part holding tile output cur,
// which starts where the finished parts ended, and returns that part's LDS
// positions, limits and length.  Outputs at or past the tile's end n are
// discarded by the caller.
template <typename K, int VT, typename Next>
__device__ __forceinline__ void merge_lane_parts(const K *keys, int ai, int bi, int a_end,
                                                 int b_end, int seg, int cur, int n, Next next,
                                                 K (&out)[VT]) {
  K ka = keys[ai];
  K kb = keys[bi];
#pragma unroll
  for (int i = 0; i < VT; ++i) {
    if (seg <= 0 && cur < n) {
      next(cur, ai, bi, a_end, b_end, seg);
      ka = keys[ai];
      kb = keys[bi];
    }
    const bool take_b = (bi < b_end) && (ai >= a_end || kb < ka);
    out[i] = take_b ? kb : ka;
    const int taken = take_b ? bi : ai;
    ai = take_b ? ai : taken + 1;
    bi = take_b ? taken + 1 : bi;
    const K nxt = keys[taken + 1];
    ka = take_b ? ka : nxt;
    kb = take_b ? nxt : kb;
    --seg;
    ++cur;
  }
}

// A batch tile keeps the starts of its pairs relative to its windows in LDS
// when it spans fewer than kPairTab of them (else lanes look pairs up in
// global memory).
constexpr int kPairTab = 256;

// Step 2.  One workgroup per tile.
template <typename K, bool KV, int NT, int VT, int KIND, int SRC, bool VLOAD>
__global__ __launch_bounds__(NT) void merge_tile_kernel(TileArgs<K> P) {
  using L = TileLds<K, KV, NT, VT, VLOAD>;
  constexpr int T = L::T, CH = L::CH;
  __shared__ __attribute__((aligned(16))) K keys[L::N_KEYS];
  __shared__ __attribute__((aligned(16))) uint32_t vals[L::N_VALS];
  // kTileBatch: window-relative starts of the tile's pairs
  __shared__ int32_t tab_a[KIND == kTileBatch ? kPairTab : 1];
  __shared__ int32_t tab_b[KIND == kTileBatch ? kPairTab : 1];
  const int tid = threadIdx.x;
  const int64_t tile = tile_of_block(blockIdx.x, gridDim.x);
  const int64_t N = P.N, NA = P.NA, NB = P.NB;
  // output range of the tile, and for a header-less tile the pair it ends
  // ([alo, ia) of A and [blo, ib) of B)
  const int64_t d0 = tile * T;
  const int n = (int)(N - d0 < T ? N - d0 : T);
  int64_t alo = 0, blo = 0, ia = NA, ib = NB;
  if constexpr (KIND == kTileRuns) {
    int64_t P0, aE, bE;
    run_pair(d0, N, P.lw, P0, aE, bE);
    alo = P0;
    blo = aE;
    ia = aE;
    ib = bE;
  }

  // ---- the tile's pair --------------------------------------------------
  int64_t a0, b0, a1;
  // kTileBatch: the pairs holding the tile's first output (pf) and the next
  // tile's (pn); the table covers pairs pf .. pn + 1 (cnt entries)
  int64_t pf = 0, cnt = 0;
  if constexpr (KIND == kTileBatch) {
    pf = P.tile_pair[tile];
    int64_t pn = tile + 1 < P.n_tiles ? (int64_t)P.tile_pair[tile + 1] : P.n_pairs - 1;
    pf = pf < 0 ? 0 : (pf >= P.n_pairs ? P.n_pairs - 1 : pf);
    pn = pn < pf ? pf : (pn >= P.n_pairs ? P.n_pairs - 1 : pn);
    cnt = pn + 2 - pf;
  }
  const bool use_tab = KIND == kTileBatch && cnt <= kPairTab;
  if constexpr (SRC == kTileSearch) {
    // one launch for a merge whose tiles all run at once: the tile finds its
    // own two splits (Algorithm 1's first step), wavefront 0 on its start
    // diagonal and wavefront 1 on its end diagonal, each by a 64-way search
    // in global memory (single pairs only)
    static_assert(KIND == kTileSingle && NT >= 128, "two wavefronts per single-pair tile");
    __shared__ int64_t s_ends[2];
    const int w = tid >> 6;
    if (w < 2) {
      const int64_t d = d0 + (w == 0 ? 0 : n);
      int64_t lo, hi;
      diag_range<int64_t>(d, NA, NB, lo, hi);
      const int64_t a = wave_split_search(
          d, lo, hi, [&](int64_t i) { return P.A[i]; }, [&](int64_t j) { return P.B[j]; });
      if ((tid & 63) == 0) s_ends[w] = a;
    }
    __syncthreads();
    a0 = s_ends[0];
    b0 = d0 - a0;
    a1 = s_ends[1];
  } else if constexpr (SRC == kTileSplitArray) {
    // the caller's splits: a0 kept on the start diagonal inside the grid and
    // the A count in its valid range, whatever the values (for the true
    // splits of sorted inputs both clamps change nothing)
    a0 = P.a_split[tile];
    a1 = P.a_split[tile + 1];
    const int64_t lo0 = d0 > NB ? d0 - NB : 0, hi0 = d0 < NA ? d0 : NA;
    a0 = a0 < lo0 ? lo0 : (a0 > hi0 ? hi0 : a0);
    b0 = d0 - a0;
  } else if ((int64_t)n * (int64_t)sizeof(K) >= kTileHdrBytes) {
    const uint32_t *h = reinterpret_cast<const uint32_t *>(P.S + d0);
    a0 = (int64_t)(((uint64_t)h[1] << 32) | h[0]);
    b0 = (int64_t)(((uint64_t)h[3] << 32) | h[2]);
    a1 = (int64_t)(((uint64_t)h[5] << 32) | h[4]);
  } else {
    // last tile (of the grid or of a run pair), shorter than a
    // header: from that end step the path back n times; each step takes the
    // larger of the two keys before the cursor, B on ties (ties went to A
    // forwards)
    a1 = ia;
    for (int s = 0; s < n; ++s) {
      const bool ta = ia > alo && (ib <= blo || P.B[ib - 1] < P.A[ia - 1]);
      if (ta) --ia; else --ib;
    }
    a0 = ia;
    b0 = ib;
  }
  // keep every access inside the arrays (no-ops for consistent pairs)
  a0 = a0 < 0 ? 0 : (a0 > NA ? NA : a0);
  b0 = b0 < 0 ? 0 : (b0 > NB ? NB : b0);
  int64_t wa64 = a1 - a0;
  const int64_t wa_hi = NA - a0 < (int64_t)n ? NA - a0 : (int64_t)n;
  const int64_t wa_lo0 = (int64_t)n - (NB - b0);
  const int64_t wa_lo = wa_lo0 > 0 ? wa_lo0 : 0;
  wa64 = wa64 < wa_lo ? wa_lo : wa64;
  wa64 = wa64 > wa_hi ? wa_hi : wa64;
  const int wa = (int)wa64;
  const int wb0 = n - wa;
  const int wb = (int64_t)wb0 <= NB - b0 ? wb0 : (int)(NB - b0);

  // ---- stage the pair in LDS --------------------------------------------
  // A's chunks first (from the chunk holding A[a0]), then B's; every lane
  // issues all its loads before its first LDS write.
  const int sa = (int)(a0 & (CH - 1)), sb = (int)(b0 & (CH - 1));
  const int ca = (sa + wa + CH - 1) / CH, cb = (sb + wb + CH - 1) / CH;
  const int64_t abase = a0 - sa, bbase = b0 - sb;
  const int pa = sa, pb = ca * CH + sb;  // LDS positions of A[a0] and B[b0]
  int64_t lp = 0, lp_a = 0, lp_b = 0, lp_a1 = 0, lp_b1 = 0;  // kTileBatch: lane's pair
  {
    constexpr int PV = (T / CH + 4 + NT - 1) / NT;
    K rk[PV][CH];
    uint32_t rv[KV ? PV : 1][CH];
#pragma unroll
    for (int k = 0; k < PV; ++k) {
      const int c = tid + k * NT;
      if (c < ca + cb) {
        const bool fb = c >= ca;
        const int64_t g = fb ? bbase + (int64_t)(c - ca) * CH : abase + (int64_t)c * CH;
        const int64_t lim = fb ? NB : NA;
        tile_load_chunk<K, CH>(fb ? P.B : P.A, g, lim, rk[k]);
        if constexpr (KV) tile_load_chunk<uint32_t, CH>(fb ? P.Bv : P.Av, g, lim, rv[k]);
      }
    }
    // kTileBatch: the pair starts for the table (their loads go out with
    // the window loads), else the lane's own pair from global memory
    constexpr int TPL = KIND == kTileBatch ? (kPairTab + NT - 1) / NT : 1;
    int64_t ta[TPL], tb[TPL];
    if constexpr (KIND == kTileBatch) {
      if (use_tab) {
#pragma unroll
        for (int k = 0; k < TPL; ++k) {
          const int i = tid + k * NT;
          if (i < cnt) {
            ta[k] = batch_a_at(P, pf + i);
            tb[k] = batch_b_at(P, pf + i);
          }
        }
      } else {
        const int dl0 = tid * VT < n ? tid * VT : n;
        lp = pf;
        lp_a = batch_a_at(P, pf);
        lp_b = batch_b_at(P, pf);
        lp_a1 = batch_a_at(P, pf + 1);
        lp_b1 = batch_b_at(P, pf + 1);
        if (dl0 < n && lp_a1 + lp_b1 <= d0 + dl0) {
          lp = batch_pair_of(P, pf, d0 + dl0);
          lp_a = batch_a_at(P, lp);
          lp_b = batch_b_at(P, lp);
          lp_a1 = batch_a_at(P, lp + 1);
          lp_b1 = batch_b_at(P, lp + 1);
        }
      }
    }
#pragma unroll
    for (int k = 0; k < PV; ++k) {
      const int c = tid + k * NT;
      if (c < ca + cb) {
        tile_put_chunk<K, CH>(keys + c * CH, rk[k]);
        if constexpr (KV) tile_put_chunk<uint32_t, CH>(vals + c * CH, rv[k]);
      }
    }
    if constexpr (KIND == kTileBatch) {
      if (use_tab) {
        // starts relative to the windows, kept inside them (a pair that
        // starts before the tile reads as 0, one after it as its end)
#pragma unroll
        for (int k = 0; k < TPL; ++k) {
          const int i = tid + k * NT;
          if (i < cnt) {
            const int64_t ra = ta[k] - a0, rb = tb[k] - b0;
            tab_a[i] = (int32_t)(ra < 0 ? 0 : (ra > wa ? wa : ra));
            tab_b[i] = (int32_t)(rb < 0 ? 0 : (rb > wb ? wb : rb));
          }
        }
      }
    }
  }
  __syncthreads();

  // ---- lane split and serial merge ---------------------------------------
  const int dl = tid * VT < n ? tid * VT : n;
  const int steps = n - dl < VT ? n - dl : VT;
  K out[VT];
  int src[VT];
  if constexpr (KIND == kTileBatch) {
    // the lane's pair's parts of the windows (LDS offsets from pa and pb)
    // and its split there: the pair's part of the tile is the merge of
    // those parts (Theorem 5)
    auto cl = [](int64_t v, int64_t lo_, int64_t hi_) {
      return (int)(v < lo_ ? lo_ : (v > hi_ ? hi_ : v));
    };
    int pa_lo, pa_hi, pb_lo, pb_hi, seg;
    int ti = 0;  // table entry of the lane's pair
    if (use_tab) {
      // last entry (before the final one) whose pair starts at or before dl
      int lo_ = 0, hi_ = (int)cnt - 1;
      while (lo_ + 1 < hi_) {
        const int mid = (lo_ + hi_) >> 1;
        if (tab_a[mid] + tab_b[mid] <= dl) lo_ = mid; else hi_ = mid;
      }
      ti = lo_;
      pa_lo = tab_a[ti];
      pb_lo = tab_b[ti];
      pa_hi = tab_a[ti + 1] > pa_lo ? tab_a[ti + 1] : pa_lo;
      pb_hi = tab_b[ti + 1] > pb_lo ? tab_b[ti + 1] : pb_lo;
      seg = tab_a[ti + 1] + tab_b[ti + 1] - dl;
    } else {
      pa_lo = cl(lp_a - a0, 0, wa);
      pa_hi = cl(lp_a1 - a0, pa_lo, wa);
      pb_lo = cl(lp_b - b0, 0, wb);
      pb_hi = cl(lp_b1 - b0, pb_lo, wb);
      seg = cl(lp_a1 + lp_b1 - (d0 + dl), -1, T + 1);
    }
    const int na_p = pa_hi - pa_lo, nb_p = pb_hi - pb_lo;
    int dlp = dl - (pa_lo + pb_lo < dl ? pa_lo + pb_lo : dl);
    dlp = dlp < na_p + nb_p ? dlp : na_p + nb_p;
    int lo, hi;
    diag_range<int>(dlp, na_p, nb_p, lo, hi);
    const int a = split_search<int>(
        dlp, lo, hi, [&](int i) { return keys[pa + pa_lo + i]; },
        [&](int j) { return keys[pb + pb_lo + j]; });
    const int ai = pa + pa_lo + a, bi = pb + pb_lo + (dlp - a);
    if (seg >= steps) {
      serial_merge<K, VT>(keys, ai, bi, pa + pa_hi, pb + pb_hi, out, src);
    } else if (use_tab) {
      merge_lane_parts<K, VT>(
          keys, ai, bi, pa + pa_hi, pb + pb_hi, seg, dl, n,
          [&](int cur, int &ai_, int &bi_, int &ae, int &be, int &sg) {
            while (ti + 2 < cnt && tab_a[ti + 1] + tab_b[ti + 1] <= cur) ++ti;
            const int a_lo = tab_a[ti], b_lo = tab_b[ti];
            ai_ = pa + a_lo;
            bi_ = pb + b_lo;
            ae = pa + (tab_a[ti + 1] > a_lo ? tab_a[ti + 1] : a_lo);
            be = pb + (tab_b[ti + 1] > b_lo ? tab_b[ti + 1] : b_lo);
            sg = tab_a[ti + 1] + tab_b[ti + 1] - cur;
          },
          out);
    } else {
      merge_lane_parts<K, VT>(
          keys, ai, bi, pa + pa_hi, pb + pb_hi, seg, dl, n,
          [&](int cur, int &ai_, int &bi_, int &ae, int &be, int &sg) {
            lp = batch_pair_of(P, lp, d0 + cur);
            const int64_t ga = batch_a_at(P, lp), gb = batch_b_at(P, lp);
            const int64_t ga1 = batch_a_at(P, lp + 1), gb1 = batch_b_at(P, lp + 1);
            ai_ = pa + cl(ga - a0, 0, wa);
            bi_ = pb + cl(gb - b0, 0, wb);
            ae = pa + cl(ga1 - a0, ai_ - pa, wa);
            be = pb + cl(gb1 - b0, bi_ - pb, wb);
            sg = cl(ga1 + gb1 - (d0 + cur), -1, T + 1);
          },
          out);
    }
  } else {
    int lo, hi;
    diag_range<int>(dl, wa, wb, lo, hi);
    const int a = split_search<int>(
        dl, lo, hi, [&](int i) { return keys[pa + i]; }, [&](int j) { return keys[pb + j]; });
    serial_merge<K, VT>(keys, pa + a, pb + (dl - a), pa + wa, pb + wb, out, src);
  }
  uint32_t ov[KV ? VT : 1];
  if constexpr (KV) {
    // (past a short lane's run, src may point beyond the staged values)
#pragma unroll
    for (int i = 0; i < VT; ++i) ov[i] = i < steps ? vals[src[i]] : 0u;
  }
  __syncthreads();

  // ---- LDS transpose and coalesced stores --------------------------------
  constexpr int RUN_BYTES = VT * (int)sizeof(K);
  if (RUN_BYTES % 16 == 0 && n == T) {
#pragma unroll
    for (int i = 0; i < VT; i += 16 / (int)sizeof(K))
      *reinterpret_cast<u32x4 *>(keys + tid * VT + i) = *reinterpret_cast<const u32x4 *>(out + i);
  } else {
#pragma unroll
    for (int i = 0; i < VT; ++i)
      if (i < steps) keys[tid * VT + i] = out[i];
  }
  if constexpr (KV) {
    if ((VT * 4) % 16 == 0 && n == T) {
#pragma unroll
      for (int i = 0; i < VT; i += 4)
        *reinterpret_cast<u32x4 *>(vals + tid * VT + i) = *reinterpret_cast<const u32x4 *>(ov + i);
    } else {
#pragma unroll
      for (int i = 0; i < VT; ++i)
        if (i < steps) vals[tid * VT + i] = ov[i];
    }
  }
  __syncthreads();
  constexpr int VEC = 16 / (int)sizeof(K);
  K *S = P.S + d0;
  const bool vs = ((uintptr_t)S % 16) == 0;
  const int nv = vs ? n / VEC : 0;
  if (n == T && vs) {
    constexpr int KVN = T / VEC, NK = (KVN + NT - 1) / NT;
#pragma unroll
    for (int j = 0; j < NK; ++j) {
      const int v = tid + j * NT;
      if (KVN % NT == 0 || v < KVN)
        __builtin_nontemporal_store(reinterpret_cast<const u32x4 *>(keys)[v],
                                    reinterpret_cast<u32x4 *>(S) + v);
    }
  } else {
    for (int v = tid; v < nv; v += NT)
      __builtin_nontemporal_store(reinterpret_cast<const u32x4 *>(keys)[v],
                                  reinterpret_cast<u32x4 *>(S) + v);
    for (int i = nv * VEC + tid; i < n; i += NT) S[i] = keys[i];
  }
  if constexpr (KV) {
    uint32_t *Sv = P.Sv + d0;
    const int nv4 = ((uintptr_t)Sv % 16) == 0 ? n / 4 : 0;
    for (int v = tid; v < nv4; v += NT)
      __builtin_nontemporal_store(reinterpret_cast<const u32x4 *>(vals)[v],
                                  reinterpret_cast<u32x4 *>(Sv) + v);
    for (int i = nv4 * 4 + tid; i < n; i += NT) Sv[i] = vals[i];
  }
}

// ---- launchers ------------------------------------------------------------

template <typename K, int KIND>
static hipError_t launch_tile_splits(const TileArgs<K> &P, int64_t T, hipStream_t s) {
  // boundaries 0 .. n_tiles
  const int64_t n_b = P.n_tiles + 1;
  const int g = partition_lanes(n_b);
  const int64_t blocks = (n_b * g + 255) / 256;
  switch (g) {
#define MP_SPLITS_CASE(G)                                                                  \
  case G:                                                                                  \
    hipLaunchKernelGGL((tile_splits_kernel<K, KIND, G>), dim3((unsigned)blocks), dim3(256), \
                       0, s, P, T);                                                        \
    break;
    MP_SPLITS_CASE(1)
    MP_SPLITS_CASE(2)
    MP_SPLITS_CASE(4)
    MP_SPLITS_CASE(8)
    MP_SPLITS_CASE(16)
    MP_SPLITS_CASE(32)
    MP_SPLITS_CASE(64)
#undef MP_SPLITS_CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename K, bool KV, int NT, int VT, int KIND, int SRC>
static hipError_t launch_tiles_shape(TileArgs<K> P, bool vload, hipStream_t s) {
  if constexpr (!tile_shape_fits<K, KV, NT, VT>()) {
    return hipErrorNotSupported;
  } else {
    constexpr int64_t T = (int64_t)NT * VT;
    P.n_tiles = (P.N + T - 1) / T;
    if (P.n_tiles == 0) return hipSuccess;
    if constexpr (KIND == kTileBatch) {
      // workspace: the splits (n_tiles + 1 int64), then the pair of every
      // tile's first output (n_tiles int32)
      P.a_split = P.split_out;
      P.tile_pair = reinterpret_cast<int32_t *>(P.split_out + P.n_tiles + 1);
      KernelTimer timer("batch_tiles", s);
      hipLaunchKernelGGL((batch_bound_kernel<K>), dim3((unsigned)((P.n_pairs + 255) / 256)), dim3(256),
                         0, s, P, T);
      const hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
    if constexpr (SRC == kTileHeader || KIND == kTileBatch) {
      KernelTimer timer("tile_splits", s);
      const hipError_t e = launch_tile_splits<K, KIND>(P, T, s);
      if (e != hipSuccess) return e;
    }
    KernelTimer timer("tile_merge", s);
    if (vload)
      hipLaunchKernelGGL((merge_tile_kernel<K, KV, NT, VT, KIND, SRC, true>),
                         dim3((unsigned)P.n_tiles), dim3(NT), 0, s, P);
    else
      hipLaunchKernelGGL((merge_tile_kernel<K, KV, NT, VT, KIND, SRC, false>),
                         dim3((unsigned)P.n_tiles), dim3(NT), 0, s, P);
    return hipGetLastError();
  }
}

template <typename K, int KIND, int SRC>
static hipError_t launch_tiles_any(TileCfg cfg, const TileArgs<K> &P, bool vload, hipStream_t s) {
  // (merges on given splits and batches carry keys only)
  constexpr bool KV_OK = SRC == kTileHeader && KIND != kTileBatch;
  static_assert(SRC != kTileSearch, "the one-launch path has its own dispatch");
  const bool kv = KV_OK && P.Sv != nullptr;
#define MP_TILE_CASE(NT_, VT_)                                                             \
  if (cfg.nt == NT_ && cfg.vt == VT_) {                                                    \
    if constexpr (KV_OK)                                                                   \
      if (kv) return launch_tiles_shape<K, true, NT_, VT_, KIND, SRC>(P, vload, s);        \
    return launch_tiles_shape<K, false, NT_, VT_, KIND, SRC>(P, vload, s);                 \
  }
  MP_TILE_CASE(1024, 16)
  MP_TILE_CASE(1024, 8)
  MP_TILE_CASE(512, 16)
  MP_TILE_CASE(512, 12)
  MP_TILE_CASE(256, 16)
  MP_TILE_CASE(256, 15)
  MP_TILE_CASE(256, 8)
  MP_TILE_CASE(128, 16)
#undef MP_TILE_CASE
  return hipErrorNotSupported;
}

static inline bool tile_aligned16(const void *p) { return ((uintptr_t)p % 16) == 0; }

// A merge small enough that all its tiles run at once (at most two per
// compute unit) on one of the small built-in shapes takes one launch: each
// tile searches its own splits, so no split kernel runs before it.
template <typename K, bool KV>
static hipError_t launch_tiles_search(TileCfg cfg, TileArgs<K> P, bool vload, hipStream_t s) {
#define MP_SEARCH_CASE(NT_, VT_)                                                           \
  if (cfg.nt == NT_ && cfg.vt == VT_) {                                                    \
    P.n_tiles = (P.N + NT_ * VT_ - 1) / (NT_ * VT_);                                       \
    KernelTimer timer("tile_merge", s);                                                    \
    if (vload)                                                                             \
      hipLaunchKernelGGL((merge_tile_kernel<K, KV, NT_, VT_, kTileSingle, kTileSearch, true>), \
                         dim3((unsigned)P.n_tiles), dim3(NT_), 0, s, P);                    \
    else                                                                                   \
      hipLaunchKernelGGL((merge_tile_kernel<K, KV, NT_, VT_, kTileSingle, kTileSearch, false>), \
                         dim3((unsigned)P.n_tiles), dim3(NT_), 0, s, P);                    \
    return hipGetLastError();                                                              \
  }
  MP_SEARCH_CASE(256, 16)
  MP_SEARCH_CASE(256, 8)
#undef MP_SEARCH_CASE
  return hipErrorNotSupported;
}

template <typename K>
hipError_t launch_merge_tiles(TileCfg cfg, const K *A, const uint32_t *Av, int64_t na,
                              const K *B, const uint32_t *Bv, int64_t nb, K *S, uint32_t *Sv,
                              hipStream_t s) {
  TileArgs<K> P{};
  P.A = A; P.B = B; P.Av = Av; P.Bv = Bv; P.S = S; P.Sv = Sv;
  P.NA = na; P.NB = nb; P.N = na + nb;
  const bool kv = Sv != nullptr;
  const bool vload = tile_aligned16(A) && tile_aligned16(B) &&
                     (!kv || (tile_aligned16(Av) && tile_aligned16(Bv)));
  const int64_t T = (int64_t)cfg.nt * cfg.vt;
  const bool small_shape = cfg.nt == 256 && (cfg.vt == 16 || cfg.vt == 8);
  if (small_shape && P.N > 0 && (P.N + T - 1) / T <= 2 * (int64_t)device_cu_count())
    return kv ? launch_tiles_search<K, true>(cfg, P, vload, s)
              : launch_tiles_search<K, false>(cfg, P, vload, s);
  return launch_tiles_any<K, kTileSingle, kTileHeader>(cfg, P, vload, s);
}

template <typename K>
hipError_t launch_merge_tiles_split(TileCfg cfg, const K *A, int64_t na, const K *B, int64_t nb,
                                    K *S, const int64_t *a_split, hipStream_t s) {
  TileArgs<K> P{};
  P.A = A; P.B = B; P.S = S;
  P.NA = na; P.NB = nb; P.N = na + nb;
  P.a_split = a_split;
  const bool vload = tile_aligned16(A) && tile_aligned16(B);
  return launch_tiles_any<K, kTileSingle, kTileSplitArray>(cfg, P, vload, s);
}

template <typename K>
hipError_t launch_merge_batched_tiles(TileCfg cfg, const K *A, const int64_t *a_off, const K *B,
                                      const int64_t *b_off, int64_t n_pairs, int64_t total_a,
                                      int64_t total_b, K *S, void *ws, hipStream_t s) {
  if ((int64_t)cfg.nt * cfg.vt < kBatchMinTile) return hipErrorNotSupported;
  TileArgs<K> P{};
  P.A = A; P.B = B; P.S = S;
  P.NA = total_a; P.NB = total_b; P.N = total_a + total_b;
  P.a_off = a_off; P.b_off = b_off; P.n_pairs = n_pairs;
  P.split_out = reinterpret_cast<int64_t *>(ws);
  const bool vload = tile_aligned16(A) && tile_aligned16(B);
  return launch_tiles_any<K, kTileBatch, kTileSplitArray>(cfg, P, vload, s);
}

template <typename K>
hipError_t launch_sort_round_tiles(TileCfg cfg, const K *X, const uint32_t *Xv, K *Y,
                                   uint32_t *Yv, int64_t n, int lw, hipStream_t s) {
  TileArgs<K> P{};
  P.A = X; P.B = X; P.Av = Xv; P.Bv = Xv; P.S = Y; P.Sv = Yv;
  P.NA = n; P.NB = n; P.N = n;
  P.lw = lw;
  const bool kv = Yv != nullptr;
  const bool vload = tile_aligned16(X) && (!kv || tile_aligned16(Xv));
  return launch_tiles_any<K, kTileRuns, kTileHeader>(cfg, P, vload, s);
}

}  // namespace mp

#define MP_TILE_INSTANTIATE(K)                                                               \
  namespace mp {                                                                             \
  template hipError_t launch_merge_tiles<K>(TileCfg, const K *, const uint32_t *, int64_t,   \
                                            const K *, const uint32_t *, int64_t, K *,       \
                                            uint32_t *, hipStream_t);                        \
  template hipError_t launch_merge_tiles_split<K>(TileCfg, const K *, int64_t, const K *,    \
                                                  int64_t, K *, const int64_t *,             \
                                                  hipStream_t);                              \
  template hipError_t launch_sort_round_tiles<K>(TileCfg, const K *, const uint32_t *, K *,  \
                                                 uint32_t *, int64_t, int, hipStream_t);     \
  template hipError_t launch_merge_batched_tiles<K>(TileCfg, const K *, const int64_t *,     \
                                                    const K *, const int64_t *, int64_t,     \
                                                    int64_t, int64_t, K *, void *,           \
                                                    hipStream_t);                            \
  }
