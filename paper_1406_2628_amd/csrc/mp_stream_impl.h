// Persistent merge over a global output index: one kernel for a single merge,
// for batches of independent merges and for the rounds of merge sort.
//
// Each workgroup walks a contiguous run of output tiles (Corollary 7: equal
// tiles balance the work).  This is the segmented parallel merge of section 4
// (Algorithm 3) with LDS in the role of the cache: the workgroup keeps its
// current split (a_cur, b_cur); a tile of n <= T outputs uses at most n keys
// of A and n keys of B (Lemma 16), so windows of n keys each always suffice;
// every lane finds its split at local diagonal lane * VT inside the windows
// (Theorem 17) and merges VT outputs serially; the tile's end split becomes
// the next tile's start.  Only the first split of each workgroup is searched
// in global memory, by one wavefront probing 64 points per round (Theorem
// 14's search with a 65-way cut).
//
// Pairs.  A batch is a list of independent pairs (A_k, B_k) laid end to end:
// A' = A_0 A_1 ..., B' = B_0 B_1 ...; pair k's merge belongs at output offset
// out(k) = a_off(k) + b_off(k) (Corollary 6 applied pair by pair).  Ordering
// keys by (pair, key) makes A' and B' sorted and their merge the
// concatenation of the pair merges, so the same Merge Path machinery applies
// to the global output index.  The kernel realises the (pair, key) order
// without storing pair ids: a split on global diagonal D lies inside pair
// k = pair_of_out(D) (the last pair with out(k) <= D), and restricting the
// search interval to that pair makes every probe compare two keys of the
// same pair; a lane whose outputs cross a pair end switches to the next pair
// there.  Three pair layouts share the kernel:
//   kSingle    one pair (A, B): plain merge;
//   kRuns      merge-sort round over X: pair k = (X[2wk, 2wk+w), X[2wk+w,
//              2wk+2w)) clipped to n, left run as A (section 1, section 3);
//   kExplicit  CSR offsets a_off[], b_off[] (batched merge), cached in LDS.
//
// Speculative windows.  Loading n keys of each input per tile would fetch
// every key twice.  Instead the next tile's windows are sized from what the
// current tile consumed plus a margin M, capped by the full extents.  The
// end split found inside these windows is exact unless it lands on a
// truncated window edge; then the full windows are loaded and the tile is
// searched again, so the output never depends on the prediction.  (Every
// probe reads true keys, so the lower-bound search returns the true split
// whenever it lies strictly inside the probed range; otherwise it can only
// return a range end, and a range end that is a truncated edge is rejected.)
// The next tile's windows are fetched into registers as soon as the end
// split is known, overlapping their latency with this tile's merge.
// By default the windows are not predicted from the A/B mix (which heavy
// runs of equal keys upset) but bracketed by probes of the split two tiles
// ahead (see the lookahead probes below); the mix prediction plus a margin
// remains for a workgroup's first tile and as an option.
#pragma once

#include <mutex>
#include <type_traits>
#include <vector>

#include "mp_device.h"
#include "mp_internal.h"

namespace mp {

enum PairKind { kSingle = 0, kRuns = 1, kExplicit = 2 };

template <typename K>
struct PairArgs {
  const K *A, *B;          // kRuns: both are the source X
  const uint32_t *Av, *Bv; // values (KV only)
  K *S;
  uint32_t *Sv;
  int64_t NA, NB;          // lengths of A' and B'
  int64_t n_tiles;
  int margin;              // 0: lookahead windows, > 0: predicted + margin, < 0: full
  int lw;                  // kRuns: log2 of the run width
  const int64_t *a_off, *b_off;  // kExplicit
  int64_t n_pairs;
  unsigned long long *stats;     // optional: [tiles, window reloads, workgroups]
  unsigned long long *checksum;  // no-store launches: sum of S[i] * (i + 1) added here
};

// Value of the first active lane (wave-uniform).
__device__ __forceinline__ int64_t first_lane64(int64_t v) {
  const uint64_t u = (uint64_t)v;
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)u);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(u >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Chunk of CH consecutive elements at src + g, loaded with one vector access.
template <typename T, int CH>
__device__ __forceinline__ void load_chunk_full(const T *__restrict__ src, int64_t g,
                                                T (&v)[CH]) {
  if constexpr (CH * sizeof(T) == 16) {
    *reinterpret_cast<u32x4 *>(v) = *reinterpret_cast<const u32x4 *>(src + g);
  } else if constexpr (CH * sizeof(T) == 8) {
    *reinterpret_cast<uint2 *>(v) = *reinterpret_cast<const uint2 *>(src + g);
  } else {
#pragma unroll
    for (int i = 0; i < CH; ++i) v[i] = src[g + i];
  }
}

// The first cnt (< CH) elements of a chunk that crosses the array end.
template <typename T, int CH>
__device__ __forceinline__ void load_chunk_part(const T *__restrict__ src, int64_t g,
                                                int cnt, T (&v)[CH]) {
#pragma unroll
  for (int i = 0; i < CH; ++i)
    if (i < cnt) v[i] = src[g + i];
}

template <typename T, int CH>
__device__ __forceinline__ void store_chunk_lds(T *lds, const T (&v)[CH]) {
  if constexpr (CH * sizeof(T) == 16) {
    *reinterpret_cast<u32x4 *>(lds) = *reinterpret_cast<const u32x4 *>(v);
  } else if constexpr (CH * sizeof(T) == 8) {
    *reinterpret_cast<uint2 *>(lds) = *reinterpret_cast<const uint2 *>(v);
  } else {
#pragma unroll
    for (int i = 0; i < CH; ++i) lds[i] = v[i];
  }
}

// One tile's windows over A' and B'.  A' keys from a_base (aligned to CH) sit
// at LDS 0, B' keys from b_base at LDS OB; the split (a_cur, b_cur) is at
// offsets sa, sb.
//   wa, wb   full extents: keys of A' and B' this tile could use (<= n)
//   la, lb   loaded extents (la <= wa, lb <= wb)
//   ca, cb   chunks covering [0, sa + la) and [0, sb + lb)
//   fa, fb   chunks lying wholly inside A' / B' (vector-loadable)
struct Window {
  int64_t a_base, b_base;
  int n, wa, wb, la, lb, sa, sb, ca, cb, fa, fb;
};

template <int CH>
__device__ __forceinline__ Window make_window(int64_t a_cur, int64_t b_cur,
                                              int64_t NA, int64_t NB, int n,
                                              int pa, int pb) {
  Window w;
  w.n = n;
  w.wa = (int)(NA - a_cur < n ? NA - a_cur : n);
  w.wb = (int)(NB - b_cur < n ? NB - b_cur : n);
  w.la = w.wa < pa ? w.wa : pa;
  w.lb = w.wb < pb ? w.wb : pb;
  w.a_base = a_cur & ~(int64_t)(CH - 1);
  w.b_base = b_cur & ~(int64_t)(CH - 1);
  w.sa = (int)(a_cur - w.a_base);
  w.sb = (int)(b_cur - w.b_base);
  w.ca = (w.sa + w.la + CH - 1) / CH;
  w.cb = (w.sb + w.lb + CH - 1) / CH;
  const int64_t fa = (NA - w.a_base) / CH, fb = (NB - w.b_base) / CH;
  w.fa = fa < w.ca ? (int)fa : w.ca;
  w.fb = fb < w.cb ? (int)fb : w.cb;
  return w;
}

// STORE = false: the diagnostic run that keeps the merged outputs in
// registers (the paper's runs that write to a local register): no output
// stage and no stores; each lane adds S[i] * (i + 1) over its outputs (keys
// as unsigned bits, modulo 2^64), one atomic per wavefront at the end.
template <typename K, bool KV, int NT, int VT, int KIND, bool VECTOR, bool STORE = true>
__global__ __launch_bounds__(NT) void merge_pairs_kernel(PairArgs<K> args) {
  constexpr int T = NT * VT;
  constexpr int VEC = 16 / (int)sizeof(K);
  constexpr int CH = VECTOR ? VEC : 1;        // elements per staged chunk
  constexpr int OB = T + VEC;                 // LDS offset of the B window
  // B window end (<= OB + T + VEC - 1) plus VT slots read by the unguarded
  // serial merge past a window end
  constexpr int LDS_N = OB + T + VEC + VT + 1;
  constexpr int MAX_MARGIN = T / 16;
  // chunks of speculative windows: (T + 2 * margin) keys plus alignment
  constexpr int PV = ((T + 2 * MAX_MARGIN) / CH + 4 + NT - 1) / NT;
  constexpr int TP = KIND == kExplicit ? 128 : 1;  // cached pair offsets
  __shared__ __attribute__((aligned(16))) K keys[LDS_N];
  __shared__ __attribute__((aligned(16))) uint32_t vals[KV ? LDS_N : 1];
  __shared__ int64_t t_a[TP + 1], t_b[TP + 1];  // a_off / b_off of pairs [tk, tk + TP]
  __shared__ int64_t s_split, s_kf, s_kl, s_kf2, s_kl2, s_tk, s_pq_D, s_pq_lo;
  __shared__ int s_pq_span;
  __shared__ int s_end, s_valid, s_inner, s_pa, s_pb, s_rearm;

  const PairArgs<K> &P = args;
  const int tid = threadIdx.x;
  const int64_t NA = P.NA, NB = P.NB, N = NA + NB;
  // Balanced contiguous tile range of this workgroup (Corollary 7).
  const int64_t g = blockIdx.x, G = gridDim.x;
  const int64_t t_begin = g * P.n_tiles / G;
  const int64_t t_end = (g + 1) * P.n_tiles / G;
  if (t_begin >= t_end) return;
  // margin == 0: windows sized by the lookahead probes below; > 0: sized by
  // the predicted end split plus this margin; < 0: full windows
  const bool speculate = P.margin >= 0;
  // (batches keep the prediction: their pair bookkeeping is heavier per
  // tile and their reloads are rare)
  const bool lookahead = KIND != kExplicit && P.margin == 0;
  const int M0 = P.margin > 0 ? P.margin : 64 + T / 32;
  const int M = M0 > MAX_MARGIN ? MAX_MARGIN : M0;

  // ---- addressing of A' and B' -------------------------------------------
  auto a_addr = [&](int64_t i) -> int64_t {
    if constexpr (KIND == kRuns) return i + ((i >> P.lw) << P.lw);
    else return i;
  };
  auto b_addr = [&](int64_t j) -> int64_t {
    if constexpr (KIND == kRuns) return ((int64_t)1 << P.lw) + j + ((j >> P.lw) << P.lw);
    else return j;
  };

  // ---- pair structure ----------------------------------------------------
  const int64_t n_pairs = KIND == kSingle   ? 1
                          : KIND == kRuns   ? (N + ((int64_t)2 << P.lw) - 1) >> (P.lw + 1)
                                            : P.n_pairs;
  // kExplicit: first pair held in the LDS table (negative until it is loaded,
  // which sends every lookup to global memory)
  int64_t tk = -((int64_t)1 << 62);
  auto aoff = [&](int64_t k) -> int64_t {
    if constexpr (KIND == kSingle) return k == 0 ? 0 : NA;
    else if constexpr (KIND == kRuns) { const int64_t v = k << P.lw; return v < NA ? v : NA; }
    else return (uint64_t)(k - tk) <= (uint64_t)TP ? t_a[k - tk] : P.a_off[k];
  };
  auto boff = [&](int64_t k) -> int64_t {
    if constexpr (KIND == kSingle) return k == 0 ? 0 : NB;
    else if constexpr (KIND == kRuns) { const int64_t v = k << P.lw; return v < NB ? v : NB; }
    else return (uint64_t)(k - tk) <= (uint64_t)TP ? t_b[k - tk] : P.b_off[k];
  };
  // End of the A' / B' keys a window of a tile inside pair k may hold.  A
  // merge-sort round never crosses a pair end inside a tile, so its windows
  // stop at the pair's ends and stay contiguous in the source array.
  auto end_a = [&](int64_t k) -> int64_t {
    if constexpr (KIND == kRuns) return aoff(k + 1);
    else return NA;
  };
  auto end_b = [&](int64_t k) -> int64_t {
    if constexpr (KIND == kRuns) return boff(k + 1);
    else return NB;
  };
  // Last pair k in [klo, khi] with out(k) <= D (out(klo) <= D is required).
  auto pair_of_out = [&](int64_t D, int64_t klo, int64_t khi) -> int64_t {
    if constexpr (KIND == kSingle) return 0;
    else if constexpr (KIND == kRuns) {
      const int64_t k = D >> (P.lw + 1);
      return k < n_pairs - 1 ? k : n_pairs - 1;
    } else {
      // gallop from klo (the answer is usually klo or just past it), then
      // finish with a binary search
      int64_t step = 1;
      while (klo + step <= khi && aoff(klo + step) + boff(klo + step) <= D) {
        klo += step;
        step <<= 1;
      }
      khi = klo + step - 1 < khi ? klo + step - 1 : khi;
      while (klo < khi) {
        const int64_t mid = klo + ((khi - klo + 1) >> 1);
        if (aoff(mid) + boff(mid) <= D) klo = mid; else khi = mid - 1;
      }
      return klo;
    }
  };
  // Candidate interval (global A' index) of the split on global diagonal D
  // inside pair k, intersected with a_cur <= a <= a_cur + la and
  // b_cur <= D - a <= b_cur + lb.
  auto pair_range = [&](int64_t D, int64_t k, int64_t a_cur, int64_t b_cur, int la,
                        int lb, int64_t &lo, int64_t &hi) {
    const int64_t ak = aoff(k), bk = boff(k), ak1 = aoff(k + 1), bk1 = boff(k + 1);
    const int64_t dk = D - ak - bk;
    lo = ak + (dk > bk1 - bk ? dk - (bk1 - bk) : 0);
    hi = ak + (dk < ak1 - ak ? dk : ak1 - ak);
    const int64_t lo2 = D - (b_cur + lb), hi2 = D - b_cur;
    lo = lo > a_cur ? lo : a_cur;
    lo = lo > lo2 ? lo : lo2;
    hi = hi < a_cur + la ? hi : a_cur + la;
    hi = hi < hi2 ? hi : hi2;
  };

  // ---- window staging ----------------------------------------------------
  auto load_chunk = [&](const Window &w, int c, K (&kc)[CH], uint32_t (&vc)[CH]) {
    const bool from_b = c >= w.ca;
    const int cc = from_b ? c - w.ca : c;
    const int64_t gi = (from_b ? w.b_base : w.a_base) + (int64_t)cc * CH;
    const int64_t mi = from_b ? b_addr(gi) : a_addr(gi);
    const K *src = from_b ? P.B : P.A;
    const uint32_t *vsrc = from_b ? P.Bv : P.Av;
    if (cc < (from_b ? w.fb : w.fa)) {
      load_chunk_full<K, CH>(src, mi, kc);
      if constexpr (KV) load_chunk_full<uint32_t, CH>(vsrc, mi, vc);
    } else {
      const int cnt = (int)((from_b ? NB : NA) - gi);
      load_chunk_part<K, CH>(src, mi, cnt, kc);
      if constexpr (KV) load_chunk_part<uint32_t, CH>(vsrc, mi, cnt, vc);
    }
  };
  auto put_chunk = [&](const Window &w, int c, const K (&kc)[CH], const uint32_t (&vc)[CH]) {
    const int pos = c >= w.ca ? OB + (c - w.ca) * CH : c * CH;
    store_chunk_lds<K, CH>(keys + pos, kc);
    if constexpr (KV) store_chunk_lds<uint32_t, CH>(vals + pos, vc);
  };
  auto load_now = [&](const Window &w) {
    for (int c = tid; c < w.ca + w.cb; c += NT) {
      K kc[CH];
      uint32_t vc[CH];
      load_chunk(w, c, kc, vc);
      put_chunk(w, c, kc, vc);
    }
  };
  K pk[PV][CH];
  uint32_t pv[KV ? PV : 1][CH];
  // Windows made of whole chunks (every window away from the array ends,
  // and for sort rounds away from the pair ends): both windows are contiguous
  // in memory, so chunk c sits at c * CH elements from one of two per-window
  // bases and no chunk needs 64-bit index arithmetic or a tail test.
  auto whole_chunks = [&](const Window &w) { return w.fa >= w.ca && w.fb >= w.cb; };
  auto prefetch = [&](const Window &w) {
    const bool fast = whole_chunks(w);
    // fast windows: chunk c of A' at ka0 + c * CH, of B' at kb0 + c * CH
    const int64_t xa = a_addr(w.a_base), xb = b_addr(w.b_base) - (int64_t)w.ca * CH;
    const K *ka0 = P.A + xa;
    const K *kb0 = P.B + xb;
    const uint32_t *va0 = KV ? P.Av + xa : nullptr;
    const uint32_t *vb0 = KV ? P.Bv + xb : nullptr;
#pragma unroll
    for (int k = 0; k < PV; ++k) {
      const int c = tid + k * NT;
      if (c < w.ca + w.cb) {
        if (fast) {
          const bool from_b = c >= w.ca;
          const uint32_t e = (uint32_t)c * CH;
          load_chunk_full<K, CH>(from_b ? kb0 : ka0, e, pk[k]);
          if constexpr (KV) load_chunk_full<uint32_t, CH>(from_b ? vb0 : va0, e, pv[k]);
        } else {
          if constexpr (KV) load_chunk(w, c, pk[k], pv[k]);
          else load_chunk(w, c, pk[k], pv[0]);
        }
      }
    }
  };
  auto commit = [&](const Window &w) {
    const bool fast = whole_chunks(w);
    const int shift_b = OB - w.ca * CH;  // LDS position of chunk c >= ca, minus c * CH
#pragma unroll
    for (int k = 0; k < PV; ++k) {
      const int c = tid + k * NT;
      if (c < w.ca + w.cb) {
        if (fast) {
          const int pos = c * CH + (c >= w.ca ? shift_b : 0);
          store_chunk_lds<K, CH>(keys + pos, pk[k]);
          if constexpr (KV) store_chunk_lds<uint32_t, CH>(vals + pos, pv[k]);
        } else {
          if constexpr (KV) put_chunk(w, c, pk[k], pv[k]);
          else put_chunk(w, c, pk[k], pv[0]);
        }
      }
    }
  };
  auto load_table = [&](int64_t k0) {  // kExplicit: pairs [k0, k0 + TP]
    for (int i = tid; i <= TP; i += NT) {
      const int64_t k = k0 + i <= n_pairs ? k0 + i : n_pairs;
      t_a[i] = P.a_off[k];
      t_b[i] = P.b_off[k];
    }
  };

  // ---- searches inside the windows ---------------------------------------
  int64_t a_cur = 0, b_cur = 0, d0 = 0;
  // Window-local split on global diagonal D, pair searched in [kf, kl].
  auto local_split = [&](const Window &w, int64_t D, int64_t kf, int64_t kl, int la, int lb,
                         int64_t &k_out) -> int {
    if constexpr (KIND == kSingle) {
      // one pair: the window bounds are the whole interval
      k_out = 0;
      const int dl = (int)(D - a_cur - b_cur);
      int lo, hi;
      diag_range<int>(dl, la, lb, lo, hi);
      const K *ka = keys + w.sa;
      const K *kb = keys + OB + w.sb;
      const int a = split_search<int>(
          dl, lo, hi, [&](int i) { return ka[i]; }, [&](int j) { return kb[j]; });
      return a < la ? a : la;
    }
    const int64_t k = pair_of_out(D, kf, kl);
    k_out = k;
    int64_t lo, hi;
    pair_range(D, k, a_cur, b_cur, la, lb, lo, hi);
    const K *ka = keys + w.sa;
    const K *kb = keys + OB + w.sb;
    const int dl = (int)(D - a_cur - b_cur);
    int a = split_search<int>(dl, (int)(lo - a_cur), (int)(hi - a_cur),
                              [&](int i) { return ka[i]; }, [&](int j) { return kb[j]; });
    // An empty interval (only for a lane parked on the tile's last diagonal
    // at a pair end, whose outputs are discarded) returns its low end; keep
    // the position inside the windows.
    a = a < la ? a : la;
    a = a > dl - lb ? a : dl - lb;
    return a > 0 ? a : 0;
  };
  // Lane 0 searches the tile's end diagonal in step with the other lanes'
  // own searches (its own split, at local diagonal 0, is known) and the
  // result is recorded here (see record_end): end split r inside pair k, the
  // window-edge test, the next tile's pair range and the next windows' sizes.
  auto end_record = [&](const Window &w, int64_t k, int r, int64_t kt, bool have,
                        int64_t b_lo, int64_t b_hi, int64_t b_D) {
    const int64_t D = d0 + w.n;
    int64_t lo, hi, tlo, thi;
    pair_range(D, k, a_cur, b_cur, w.la, w.lb, lo, hi);
    pair_range(D, k, a_cur, b_cur, w.wa, w.wb, tlo, thi);
    const int64_t ra = a_cur + r;
    s_end = r;
    // The end split lies strictly inside the loaded windows and before the
    // ends of the tile's pair: every lane's merge compares real keys of its
    // own pair only and needs no end tests.
    s_inner = r < w.la && w.n - r < w.lb && ra < aoff(kt + 1) && D - ra < boff(kt + 1);
    s_valid = lo <= hi && (ra < hi || hi == thi) && (ra > lo || lo == tlo);
    s_kf2 = k;
    const int64_t d1 = D + T < N ? D + T : N;
    s_kl2 = d1 > D ? pair_of_out(d1 - 1, k, n_pairs - 1) : k;
    // Window sizes for the next tile: predict its end split and add the
    // margin.  Inside the same pair the path keeps this tile's A/B mix; a new
    // pair starts from its own A fraction.  With a lookahead bracket
    // [b_lo, b_hi] of that split the windows instead reach just past both
    // ends of the bracket (the keys at the split itself included), and a
    // bracket the prediction would not have covered keeps the probes going.
    // The pair's candidate interval caps both windows exactly.
    s_rearm = 0;
    if (d1 > D) {
      const int64_t k1 = pair_of_out(d1, s_kl2, n_pairs - 1);
      const int64_t ak = aoff(k1), bk = boff(k1), ak1 = aoff(k1 + 1), bk1 = boff(k1 + 1);
      const int64_t dk = d1 - ak - bk;
      const int64_t lo1 = ak + (dk > bk1 - bk ? dk - (bk1 - bk) : 0);
      const int64_t hi1 = ak + (dk < ak1 - ak ? dk : ak1 - ak);
      const int64_t a_nx = ra, b_nx = D - ra;
      int64_t ap;
      const int64_t ok = ak + bk;  // output offset where pair k1 starts
      if (k1 == k && D - (ok > d0 ? ok : d0) >= T / 2) {
        // keep the A/B mix pair k showed inside this tile
        const int64_t from_d = ok > d0 ? ok : d0, from_a = ok > d0 ? ak : a_cur;
        const int n1 = (int)(d1 - D);
        ap = a_nx + (int64_t)((float)(ra - from_a) * (float)n1 / (float)(D - from_d));
      } else {
        const int64_t sk = (ak1 - ak) + (bk1 - bk);
        ap = ak + (sk > 0 ? (int64_t)((double)dk * (double)(ak1 - ak) / (double)sk) : 0);
      }
      const int64_t alo = lo1 > a_nx ? lo1 : a_nx;
      const int64_t ahi = hi1 < a_nx + (d1 - D) ? hi1 : a_nx + (d1 - D);
      ap = ap < alo ? alo : (ap > ahi ? ahi : ap);
      int64_t pa = ap - a_nx + M, pb = (d1 - ap) - b_nx + M;
      if (have && b_D == d1) {
        const int64_t qa = b_hi - a_nx + 1, qb = (d1 - b_lo) - b_nx + 1;
        s_rearm = qa > pa || qb > pb;
        pa = qa;
        pb = qb;
      }
      s_pa = (int)(pa < hi1 - a_nx ? pa : hi1 - a_nx);
      s_pb = (int)(pb < (d1 - lo1) - b_nx ? pb : (d1 - lo1) - b_nx);
    }
  };

  // ---- lookahead probes (wave 0) -----------------------------------------
  // Once a tile's end split is known, wave 0 probes 64 evenly spaced points
  // of the interval that must hold the split two tiles further on (Theorem
  // 14's search cut 65 ways, one step of it).  The loads have a whole tile to
  // arrive; the ballot one tile later brackets that split to 1/65 of the
  // interval, which sizes those windows so that they always hold it.  The
  // probed keys lie inside windows fetched soon after.  Probing costs a few
  // percent where the A/B mix is steady, so it runs only for PROBE_RUN tiles
  // after a window reload, extended while the brackets show that the
  // prediction would have missed (long runs of equal keys).
  // Only the probed keys stay in registers; the probe's diagonal and
  // interval wait in LDS (written by lane 0, read after a barrier).
  K pq_a{}, pq_b{};  // this lane's probe keys
  auto probe_point = [](int64_t lo, int span, int i) {
    return lo + ((int64_t)(i + 1) * span) / 65;
  };
  // Probe the split on diagonal D, knowing the split (a_b, b_b) on diagonal
  // a_b + b_b <= D and a pair k_from <= the pair of D.
  auto probe_issue = [&](int64_t D, int64_t k_from, int64_t a_b, int64_t b_b) {
    const int64_t k = pair_of_out(D, k_from, n_pairs - 1);
    const int span_d = (int)(D - a_b - b_b);
    int64_t lo, hi;
    pair_range(D, k, a_b, b_b, span_d, span_d, lo, hi);
    const int span = hi > lo ? (int)(hi - lo) : 0;
    if (tid == 0) {
      s_pq_D = D;
      s_pq_lo = lo;
      s_pq_span = span;
    }
    if (span > 0) {
      const int64_t pt = probe_point(lo, span, tid);
      pq_a = P.A[a_addr(pt)];
      pq_b = P.B[b_addr(D - 1 - pt)];
    }
  };
  // Bracket [b_lo, b_hi] of the pending probe's split on diagonal b_D (all
  // 64 lanes of wave 0); false when no probe is pending.
  auto probe_bracket = [&](int64_t &b_lo, int64_t &b_hi, int64_t &b_D) -> bool {
    b_D = s_pq_D;
    if (b_D < 0) return false;
    const int64_t lo = s_pq_lo;
    const int span = s_pq_span;
    b_lo = lo;
    b_hi = lo + span;
    if (span > 0) {
      const uint64_t m = __ballot(pq_b < pq_a);
      if (m == 0) {
        b_lo = probe_point(lo, span, 63) + 1;
      } else {
        const int f = __ffsll((long long)m) - 1;
        b_hi = probe_point(lo, span, f);
        if (f > 0) b_lo = probe_point(lo, span, f - 1) + 1;
      }
    }
    return true;
  };

  // ---- prologue: this workgroup's first split ----------------------------
  d0 = t_begin * T;
  if (tid < 64) {
    const int64_t d = d0 < N ? d0 : N;
    const int64_t k = pair_of_out(d, 0, n_pairs - 1);
    // candidate interval of the split inside pair k
    const int64_t ak = aoff(k), bk = boff(k), ak1 = aoff(k + 1), bk1 = boff(k + 1);
    const int64_t dk = d - ak - bk;
    int64_t lo = ak + (dk > bk1 - bk ? dk - (bk1 - bk) : 0);
    int64_t hi = ak + (dk < ak1 - ak ? dk : ak1 - ak);
    // no-ops for valid offsets; keep malformed ones inside the grid
    int64_t glo, ghi;
    diag_range<int64_t>(d, NA, NB, glo, ghi);
    lo = lo < glo ? glo : (lo > ghi ? ghi : lo);
    hi = hi < lo ? lo : (hi > ghi ? ghi : hi);
    const int64_t a = wave_split_search(
        d, lo, hi, [&](int64_t i) { return P.A[a_addr(i)]; },
        [&](int64_t j) { return P.B[b_addr(j)]; });
    if (tid == 0) {
      s_split = a;
      s_kf = k;
      const int64_t d1 = d0 + T < N ? d0 + T : N;
      s_kl = pair_of_out(d1 > d ? d1 - 1 : d, k, n_pairs - 1);
    }
  }
  __syncthreads();
  a_cur = s_split;
  b_cur = d0 - a_cur;
  int64_t kf = s_kf, kl = s_kl;
  if constexpr (KIND == kExplicit) {
    tk = kf;
    load_table(tk);
  }
  const int n0 = (int)(N - d0 < T ? N - d0 : T);
  Window w = make_window<CH>(a_cur, b_cur, end_a(kf), end_b(kf), n0, n0, n0);
  load_now(w);
  __syncthreads();
  if (tid == 0) s_pq_D = -1;
  __syncthreads();
  constexpr int PROBE_RUN = 128;
  int probe_left = 0;  // tiles that still issue probes (uniform)

  // Lane 0's end split (r, k) into end_record.  Single merges and sort
  // rounds run it on all of wave 0 with lane 0's values made uniform, which
  // keeps its arithmetic in scalar registers; batches keep it on lane 0,
  // where their pair lookups stay vector loads.
  auto record_end = [&](int r, int64_t k) {
    if constexpr (KIND == kExplicit) {
      if (tid == 0) end_record(w, k, r, kf, false, 0, 0, -1);
    } else if (tid < 64) {
      int64_t b_lo = 0, b_hi = 0, b_D = -1;
      const bool have = probe_bracket(b_lo, b_hi, b_D);
      const int r0 = __builtin_amdgcn_readfirstlane(r);
      end_record(w, first_lane64(k), r0, kf, have, b_lo, b_hi, b_D);
    }
  };

  unsigned long long n_reload = 0;
  unsigned long long ck = 0;  // STORE = false: this lane's checksum
  for (int64_t t = t_begin; t < t_end; ++t) {
    d0 = t * T;
    const int n = w.n;
    const int dl = tid * VT < n ? tid * VT : n;
    // Lane 0's own split is the window start; it searches the end diagonal.
    const int64_t dq = tid == 0 ? d0 + n : d0 + dl;
    const int64_t kq_lo = tid == 0 ? kl : kf, kq_hi = tid == 0 ? n_pairs - 1 : kl;
    int64_t k_q;
    int r_q = local_split(w, dq, kq_lo, kq_hi, w.la, w.lb, k_q);
    record_end(r_q, k_q);
    __syncthreads();
    const bool reloaded = !s_valid;
    if (!s_valid) {
      // The split left the speculative windows: load the full ones (exact).
      ++n_reload;
      w = make_window<CH>(a_cur, b_cur, end_a(kf), end_b(kf), n, n, n);
      load_now(w);
      __syncthreads();
      r_q = local_split(w, dq, kq_lo, kq_hi, w.la, w.lb, k_q);
      record_end(r_q, k_q);
      __syncthreads();
    }
    if (lookahead) {
      if (reloaded || s_rearm) probe_left = PROBE_RUN;
      else if (probe_left > 0) --probe_left;
    }
    const int a_own = tid == 0 ? 0 : r_q;
    const int64_t k_own = tid == 0 ? kf : k_q;
    const int a_end = s_end;
    const bool inner = s_inner;
    const int64_t a_next = a_cur + a_end, b_next = b_cur + (n - a_end);
    const int64_t kf_next = s_kf2, kl_next = s_kl2;

    // Probe the end split of the tile after next (its start, this tile's
    // end split, is now known).
    if (lookahead && tid < 64) {
      if (probe_left > 0 && t + 2 < t_end) {
        const int64_t D3 = d0 + 3 * T < N ? d0 + 3 * T : N;
        probe_issue(D3, kf_next, a_next, b_next);
      } else if (tid == 0) {
        s_pq_D = -1;
      }
    }

    // Fetch the next tile's windows while this tile is merged.
    Window wn = w;
    const bool more = t + 1 < t_end;
    if (more) {
      const int64_t d1 = d0 + T;
      const int n1 = (int)(N - d1 < T ? N - d1 : T);
      const int pa = speculate ? s_pa : n1;
      const int pb = speculate ? s_pb : n1;
      wn = make_window<CH>(a_next, b_next, end_a(kf_next), end_b(kf_next), n1, pa, pb);
      if (speculate) prefetch(wn);
    }

    // Serial merge of this lane's VT outputs.
    K out[VT];
    int src[VT];
    {
      const int64_t ak1 = aoff(k_own + 1), bk1 = boff(k_own + 1);
      const int64_t D = d0 + dl;
      auto clip_a = [&](int64_t e) { const int64_t l = e - a_cur; return w.sa + (int)(l < w.la ? l : w.la); };
      auto clip_b = [&](int64_t e) { const int64_t l = e - b_cur; return OB + w.sb + (int)(l < w.lb ? l : w.lb); };
      int ai = w.sa + a_own, bi = OB + w.sb + (dl - a_own);
      // Run pairs span 2w outputs (w at least one sorted block) and start at
      // multiples of 2w, and sort tiles are powers of two no larger than two
      // blocks (the host enforces it), so a run pair never ends inside a tile.  Batches cross
      // pair ends often: they always take the pair-tracking loop below.
      if (KIND == kSingle || KIND == kRuns) {
        if (inner) serial_merge_inner<K, VT>(keys, ai, bi, out, src);
        else serial_merge<K, VT>(keys, ai, bi, clip_a(ak1), clip_b(bk1), out, src);
      } else {
        // this lane's outputs cross the end of its pair
        // pair end as a tile-local output index (capped past this lane's run)
        auto local_end = [&](int64_t e) {
          const int64_t l = e - d0;
          return (int)(l < dl + VT + 1 ? l : dl + VT + 1);
        };
        int64_t k = k_own;
        int oe = local_end(ak1 + bk1);
        int a_e = clip_a(ak1), b_e = clip_b(bk1);
        K ka = keys[ai], kb = keys[bi];
#pragma unroll
        for (int i = 0; i < VT; ++i) {
          if (dl + i == oe && k + 1 < n_pairs) {
            k = pair_of_out(D + i, k + 1, kl > k + 1 ? kl : k + 1);
            const int64_t a2 = aoff(k + 1), b2 = boff(k + 1);
            oe = local_end(a2 + b2);
            a_e = clip_a(a2);
            b_e = clip_b(b2);
          }
          const bool take_b = (bi < b_e) && (ai >= a_e || kb < ka);
          out[i] = take_b ? kb : ka;
          src[i] = take_b ? bi : ai;
          ai += take_b ? 0 : 1;
          bi += take_b ? 1 : 0;
          const K nxt = keys[take_b ? bi : ai];
          ka = take_b ? ka : nxt;
          kb = take_b ? nxt : kb;
        }
      }
    }
    const int steps = n - dl < VT ? n - dl : VT;
    uint32_t ov[VT];
    if constexpr (KV) {
#pragma unroll
      for (int i = 0; i < VT; ++i) ov[i] = vals[src[i]];
    }
    __syncthreads();

    if constexpr (!STORE) {
      typedef typename std::conditional<sizeof(K) == 8, uint64_t, uint32_t>::type Bits;
#pragma unroll
      for (int i = 0; i < VT; ++i)
        if (i < steps)
          ck += (unsigned long long)__builtin_bit_cast(Bits, out[i]) *
                (unsigned long long)(d0 + dl + i + 1);
    } else {
    bool staged = false;
    // full tile: each lane's VT outputs with the widest LDS store that
    // divides its run (16 or 8 bytes)
    constexpr int RUN_BYTES = VT * (int)sizeof(K);
    constexpr int SW = RUN_BYTES % 16 == 0 ? 16 : (RUN_BYTES % 8 == 0 ? 8 : 0);
    if constexpr (SW != 0) {
      if (n == T) {
        constexpr int PER = SW / (int)sizeof(K);
#pragma unroll
        for (int i = 0; i < VT; i += PER) {
          if constexpr (SW == 16)
            *reinterpret_cast<u32x4 *>(keys + tid * VT + i) =
                *reinterpret_cast<const u32x4 *>(out + i);
          else
            *reinterpret_cast<uint2 *>(keys + tid * VT + i) =
                *reinterpret_cast<const uint2 *>(out + i);
        }
        if constexpr (KV) {
#pragma unroll
          for (int i = 0; i < VT; ++i) vals[tid * VT + i] = ov[i];
        }
        staged = true;
      }
    }
    if (!staged) {
#pragma unroll
      for (int i = 0; i < VT; ++i) {
        if (i < steps) {
          keys[tid * VT + i] = out[i];
          if constexpr (KV) vals[tid * VT + i] = ov[i];
        }
      }
    }
    __syncthreads();

    K *S = P.S;
    uint32_t *Sv = P.Sv;
    if constexpr (VECTOR) {
      const int nvec = n / VEC;
      u32x4 *vdst = reinterpret_cast<u32x4 *>(S + d0);
      const u32x4 *vsrc = reinterpret_cast<const u32x4 *>(keys);
      if (n == T) {
        // full tile: a fixed count of vectors per lane, all LDS reads issued
        // before the first store
        constexpr int KVN = T / VEC, NK = (KVN + NT - 1) / NT;
#pragma unroll
        for (int j = 0; j < NK; ++j) {
          const int v = tid + j * NT;
          if (KVN % NT == 0 || v < KVN) __builtin_nontemporal_store(vsrc[v], vdst + v);
        }
      } else {
        for (int v = tid; v < nvec; v += NT) __builtin_nontemporal_store(vsrc[v], vdst + v);
        for (int i = nvec * VEC + tid; i < n; i += NT) S[d0 + i] = keys[i];
      }
      if constexpr (KV) {
        const int nv4 = n / 4;
        u32x4 *vd = reinterpret_cast<u32x4 *>(Sv + d0);
        const u32x4 *vs = reinterpret_cast<const u32x4 *>(vals);
        for (int v = tid; v < nv4; v += NT) __builtin_nontemporal_store(vs[v], vd + v);
        for (int i = nv4 * 4 + tid; i < n; i += NT) Sv[d0 + i] = vals[i];
      }
    } else {
      for (int i = tid; i < n; i += NT) {
        S[d0 + i] = keys[i];
        if constexpr (KV) Sv[d0 + i] = vals[i];
      }
    }
    __syncthreads();
    }  // STORE

    if (more) {
      if (speculate) commit(wn);
      else load_now(wn);
      if constexpr (KIND == kExplicit) {
        // slide the cached offsets when the next tile's pairs leave them
        if (kl_next + 1 > tk + TP || kf_next < tk) {
          tk = kf_next;
          load_table(tk);
        }
      }
      __syncthreads();
    }
    a_cur = a_next;
    b_cur = b_next;
    kf = kf_next;
    kl = kl_next;
    w = wn;
  }
  if constexpr (!STORE) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) ck += __shfl_xor(ck, o);
    if ((tid & 63) == 0) atomicAdd(P.checksum, ck);
  }
  if (P.stats && tid == 0) {
    atomicAdd(&P.stats[0], (unsigned long long)(t_end - t_begin));
    atomicAdd(&P.stats[1], n_reload);
    atomicAdd(&P.stats[2], 1ull);
  }
}

template <typename K, bool KV, int NT, int VT, int KIND, bool STORE = true>
static hipError_t launch_pairs_impl(int grid, bool vec, PairArgs<K> args, hipStream_t s) {
  constexpr int64_t T = NT * VT;
  args.n_tiles = (args.NA + args.NB + T - 1) / T;
  args.stats = stats_device_ptr();
  if (args.n_tiles == 0) return hipSuccess;
  if (grid <= 0) {
    // one full wave of resident workgroups (occupancy queried once per
    // device and kernel; the answer is the same for every device of one
    // kind, but a process may mix kinds)
    static std::mutex mu;
    static std::vector<int> per_cu;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = 0;
    int occ = 0;
    {
      std::lock_guard<std::mutex> lock(mu);
      if ((int)per_cu.size() <= dev) per_cu.resize(dev + 1, 0);
      occ = per_cu[dev];
    }
    if (occ == 0) {
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
              &occ, merge_pairs_kernel<K, KV, NT, VT, KIND, true, STORE>, NT, 0) != hipSuccess ||
          occ <= 0)
        occ = 1;
      std::lock_guard<std::mutex> lock(mu);
      per_cu[dev] = occ;
    }
    grid = occ * device_cu_count();
  }
  g_last_pairs_grid = grid;
  const int64_t G = grid < args.n_tiles ? grid : args.n_tiles;
  if (vec)
    hipLaunchKernelGGL((merge_pairs_kernel<K, KV, NT, VT, KIND, true, STORE>), dim3((unsigned)G),
                       dim3(NT), 0, s, args);
  else
    hipLaunchKernelGGL((merge_pairs_kernel<K, KV, NT, VT, KIND, false, STORE>), dim3((unsigned)G),
                       dim3(NT), 0, s, args);
  return hipGetLastError();
}

template <typename K, int KIND>
static hipError_t launch_pairs(StreamCfg cfg, bool vec, const PairArgs<K> &args,
                               hipStream_t s) {
  const bool kv = args.Sv != nullptr;
#define MP_PAIRS_CASE(NT_, VT_)                                                    \
  if (cfg.nt == NT_ && cfg.vt == VT_)                                              \
    return kv ? launch_pairs_impl<K, true, NT_, VT_, KIND>(cfg.grid, vec, args, s) \
              : launch_pairs_impl<K, false, NT_, VT_, KIND>(cfg.grid, vec, args, s);
  MP_PAIRS_CASE(256, 16)
  MP_PAIRS_CASE(256, 8)
  MP_PAIRS_CASE(256, 12)
  MP_PAIRS_CASE(256, 14)
  MP_PAIRS_CASE(256, 18)
  MP_PAIRS_CASE(128, 16)
  MP_PAIRS_CASE(512, 8)
  MP_PAIRS_CASE(192, 24)
  // 8192-key tiles: for 4-byte keys only (8-byte keys with values would need
  // 192 KB of LDS); the sort rounds of uniform keys gain 3% with them
  if constexpr (sizeof(K) == 4) { MP_PAIRS_CASE(512, 16) }
#undef MP_PAIRS_CASE
  return hipErrorNotSupported;
}

static bool aligned16(const void *p) { return ((uintptr_t)p % 16) == 0; }

template <typename K>
hipError_t launch_merge_stream(StreamCfg cfg, const K *A, const uint32_t *Av,
                               int64_t na, const K *B, const uint32_t *Bv,
                               int64_t nb, K *S, uint32_t *Sv, hipStream_t s) {
  PairArgs<K> a{};
  a.A = A; a.B = B; a.Av = Av; a.Bv = Bv; a.S = S; a.Sv = Sv;
  a.NA = na; a.NB = nb; a.margin = cfg.margin;
  const bool kv = Sv != nullptr;
  const bool vec = aligned16(A) && aligned16(B) && aligned16(S) &&
                   (!kv || (aligned16(Sv) && aligned16(Av) && aligned16(Bv)));
  return launch_pairs<K, kSingle>(cfg, vec, a, s);
}

// No-store merge (see merge_pairs_kernel): keys only, the merge's built-in
// 192 x 24 tiles or 256 x 16.
template <typename K>
hipError_t launch_merge_checksum(StreamCfg cfg, const K *A, int64_t na, const K *B, int64_t nb,
                                 unsigned long long *checksum, hipStream_t s) {
  PairArgs<K> a{};
  a.A = A; a.B = B;
  a.NA = na; a.NB = nb; a.margin = cfg.margin;
  a.checksum = checksum;
  const bool vec = aligned16(A) && aligned16(B);
  if (cfg.nt == 256 && cfg.vt == 16)
    return launch_pairs_impl<K, false, 256, 16, kSingle, false>(cfg.grid, vec, a, s);
  if (cfg.nt == 192 && cfg.vt == 24)
    return launch_pairs_impl<K, false, 192, 24, kSingle, false>(cfg.grid, vec, a, s);
  return hipErrorNotSupported;
}

template <typename K>
hipError_t launch_merge_batched(StreamCfg cfg, const K *A, const int64_t *a_off,
                                const K *B, const int64_t *b_off, int64_t n_pairs,
                                int64_t total_a, int64_t total_b, K *S, hipStream_t s) {
  PairArgs<K> a{};
  a.A = A; a.B = B; a.S = S;
  a.NA = total_a; a.NB = total_b; a.margin = cfg.margin;
  a.a_off = a_off; a.b_off = b_off; a.n_pairs = n_pairs;
  const bool vec = aligned16(A) && aligned16(B) && aligned16(S);
  return launch_pairs<K, kExplicit>(cfg, vec, a, s);
}

template <typename K>
hipError_t launch_sort_round(StreamCfg cfg, const K *X, const uint32_t *Xv, K *Y,
                             uint32_t *Yv, int64_t n, int lw, hipStream_t s) {
  PairArgs<K> a{};
  const int64_t w = (int64_t)1 << lw;
  const int64_t q = n >> (lw + 1), r = n - (q << (lw + 1));
  a.A = X; a.B = X; a.Av = Xv; a.Bv = Xv; a.S = Y; a.Sv = Yv;
  a.NA = q * w + (r < w ? r : w);
  a.NB = n - a.NA;
  a.margin = cfg.margin;
  a.lw = lw;
  const bool kv = Yv != nullptr;
  // run starts are multiples of w (>= 16 keys here), so CH-aligned chunks
  // never straddle two runs
  const bool vec = aligned16(X) && aligned16(Y) && (!kv || (aligned16(Xv) && aligned16(Yv))) &&
                   w * (int64_t)sizeof(K) % 16 == 0;
  return launch_pairs<K, kRuns>(cfg, vec, a, s);
}

}  // namespace mp

// Each mp_stream_<key>.hip instantiates the launchers for one key type (one
// translation unit per key type keeps the build parallel).
#define MP_STREAM_INSTANTIATE(K)                                                         \
  namespace mp {                                                                         \
  template hipError_t launch_merge_stream<K>(StreamCfg, const K *, const uint32_t *,     \
                                             int64_t, const K *, const uint32_t *,       \
                                             int64_t, K *, uint32_t *, hipStream_t);     \
  template hipError_t launch_merge_checksum<K>(StreamCfg, const K *, int64_t, const K *, \
                                               int64_t, unsigned long long *, hipStream_t); \
  template hipError_t launch_merge_batched<K>(StreamCfg, const K *, const int64_t *,     \
                                              const K *, const int64_t *, int64_t,       \
                                              int64_t, int64_t, K *, hipStream_t);       \
  template hipError_t launch_sort_round<K>(StreamCfg, const K *, const uint32_t *, K *,  \
                                           uint32_t *, int64_t, int, hipStream_t);       \
  }
