// Persistent merge: each workgroup walks a contiguous run of output tiles.
//
// This is the segmented parallel merge of section 4 (Algorithm 3) mapped to a
// GPU workgroup, with LDS in the role of the cache.  The workgroup keeps its
// current split (a_cur, b_cur).  For a tile of n <= T outputs the path uses
// at most n keys of A and n keys of B (Lemma 16), so windows of n keys each
// always suffice; every lane then finds its split at local diagonal lane * VT
// inside the windows (Theorem 17) and merges VT outputs serially, and the
// tile's end split becomes the next tile's start.  Only the first split of
// each workgroup is searched in global memory, by one wavefront probing 64
// points of the diagonal per round (Theorem 14's search with a 65-way cut).
//
// Speculative windows.  Loading n keys of each input per tile would fetch
// every key twice.  Instead the next tile's windows are sized from what the
// current tile consumed (ca of A, cb of B) plus a margin M: la = ca + M and
// lb = cb + M, capped by the full extents.  The end split found inside these
// windows is exact unless it lands on a truncated window edge; in that case
// the full windows are loaded and the tile is searched again, so the output
// never depends on the prediction.  (Why the edge test suffices: every probe
// of the search reads true keys, so the lower-bound search returns the true
// split whenever it lies strictly inside the probed range; if it lies
// outside, the search can only return a range end, and a range end that is a
// truncated window edge is rejected.)
//
// The next tile's windows are fetched into registers right after the end
// split is known, so their latency overlaps this tile's merge and stores.
#include "mp_device.h"
#include "mp_internal.h"

namespace mp {

// Split on diagonal d by the 64 lanes of the calling wavefront; every lane
// returns the same value.  Each round probes 64 interior points of the
// candidate interval and keeps the gap where the predicate B[d-1-a] < A[a]
// first turns true (it is monotone in a, Corollary 12).
template <typename K>
__device__ int64_t wave_split_search(const K *__restrict__ A, int64_t na,
                                     const K *__restrict__ B, int64_t nb,
                                     int64_t d) {
  const int lane = threadIdx.x & 63;
  int64_t lo, hi;
  diag_range<int64_t>(d, na, nb, lo, hi);
  while (lo < hi) {
    const int64_t span = hi - lo;
    if (span <= 64) {
      const int64_t p = lo + lane;
      const bool pred = lane < span && (B[d - 1 - p] < A[p]);
      const uint64_t m = __ballot(pred);
      return m ? lo + (int64_t)(__ffsll((long long)m) - 1) : hi;
    }
    const int64_t p = lo + ((int64_t)(lane + 1) * span) / 65;
    const bool pred = B[d - 1 - p] < A[p];
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

// One tile's windows.  A keys from a_base (aligned to CH) sit at LDS 0, B keys
// from b_base at LDS OB; the split (a_cur, b_cur) is at offsets sa, sb.
//   wa, wb   full extents: keys of A and B this tile could use (<= n)
//   la, lb   loaded extents (la <= wa, lb <= wb)
//   ca, cb   chunks covering [0, sa + la) and [0, sb + lb)
//   fa, fb   chunks lying wholly inside their array (vector-loadable)
struct Window {
  int64_t a_base, b_base;
  int n, wa, wb, la, lb, sa, sb, ca, cb, fa, fb;
};

template <int CH>
__device__ __forceinline__ Window make_window(int64_t a_cur, int64_t b_cur,
                                              int64_t na, int64_t nb, int n,
                                              int pa, int pb) {
  Window w;
  w.n = n;
  w.wa = (int)(na - a_cur < n ? na - a_cur : n);
  w.wb = (int)(nb - b_cur < n ? nb - b_cur : n);
  w.la = w.wa < pa ? w.wa : pa;
  w.lb = w.wb < pb ? w.wb : pb;
  w.a_base = a_cur & ~(int64_t)(CH - 1);
  w.b_base = b_cur & ~(int64_t)(CH - 1);
  w.sa = (int)(a_cur - w.a_base);
  w.sb = (int)(b_cur - w.b_base);
  w.ca = (w.sa + w.la + CH - 1) / CH;
  w.cb = (w.sb + w.lb + CH - 1) / CH;
  const int64_t fa = (na - w.a_base) / CH, fb = (nb - w.b_base) / CH;
  w.fa = fa < w.ca ? (int)fa : w.ca;
  w.fb = fb < w.cb ? (int)fb : w.cb;
  return w;
}

// Global index, array and LDS position of chunk c of window w.
template <int CH, int OB>
__device__ __forceinline__ void chunk_place(const Window &w, int c, bool &from_b,
                                            int64_t &g, int &pos, int &valid) {
  from_b = c >= w.ca;
  const int cc = from_b ? c - w.ca : c;
  g = (from_b ? w.b_base : w.a_base) + (int64_t)cc * CH;
  pos = (from_b ? OB : 0) + cc * CH;
  valid = cc < (from_b ? w.fb : w.fa) ? CH : -1;  // -1: partial chunk
}

template <typename K, bool KV, int NT, int VT, bool VECTOR>
__global__ __launch_bounds__(NT) void merge_stream_kernel(
    const K *__restrict__ A, const uint32_t *__restrict__ Av, int64_t na,
    const K *__restrict__ B, const uint32_t *__restrict__ Bv, int64_t nb,
    K *__restrict__ S, uint32_t *__restrict__ Sv, int64_t n_tiles, int margin) {
  constexpr int T = NT * VT;
  constexpr int VEC = 16 / (int)sizeof(K);
  constexpr int CH = VECTOR ? VEC : 1;        // elements per staged chunk
  constexpr int OB = T + VEC;                 // LDS offset of the B window
  // B window end (<= OB + T + VEC - 1) plus VT slots read by the unguarded
  // serial merge past a window end
  constexpr int LDS_N = OB + T + VEC + VT + 1;
  constexpr int MAX_MARGIN = T / 8;
  // chunks of speculative windows: (T + 2 * margin) keys plus alignment
  constexpr int PV = ((T + 2 * MAX_MARGIN) / CH + 4 + NT - 1) / NT;
  __shared__ __attribute__((aligned(16))) K keys[LDS_N];
  __shared__ __attribute__((aligned(16))) uint32_t vals[KV ? LDS_N : 1];
  __shared__ int64_t s_split;
  __shared__ int s_end, s_valid;

  const int tid = threadIdx.x;
  const int64_t n_all = na + nb;
  // Balanced contiguous tile range of this workgroup (Corollary 7).
  const int64_t g = blockIdx.x, G = gridDim.x;
  const int64_t t_begin = g * n_tiles / G;
  const int64_t t_end = (g + 1) * n_tiles / G;
  if (t_begin >= t_end) return;
  // margin < 0: always load full windows; otherwise at most T / 8
  const bool speculate = margin >= 0;
  const int M = margin > MAX_MARGIN ? MAX_MARGIN : margin;

  auto load_chunk = [&](const Window &w, int c, K (&kc)[CH], uint32_t (&vc)[CH]) {
    bool from_b;
    int64_t gi;
    int pos, valid;
    chunk_place<CH, OB>(w, c, from_b, gi, pos, valid);
    const K *src = from_b ? B : A;
    const uint32_t *vsrc = from_b ? Bv : Av;
    if (valid > 0) {
      load_chunk_full<K, CH>(src, gi, kc);
      if constexpr (KV) load_chunk_full<uint32_t, CH>(vsrc, gi, vc);
    } else {
      const int cnt = (int)((from_b ? nb : na) - gi);
      load_chunk_part<K, CH>(src, gi, cnt, kc);
      if constexpr (KV) load_chunk_part<uint32_t, CH>(vsrc, gi, cnt, vc);
    }
  };
  auto put_chunk = [&](const Window &w, int c, const K (&kc)[CH], const uint32_t (&vc)[CH]) {
    const int pos = c >= w.ca ? OB + (c - w.ca) * CH : c * CH;
    store_chunk_lds<K, CH>(keys + pos, kc);
    if constexpr (KV) store_chunk_lds<uint32_t, CH>(vals + pos, vc);
  };
  // Load every chunk of window w straight into LDS (prologue and fallback).
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
  auto prefetch = [&](const Window &w) {
#pragma unroll
    for (int k = 0; k < PV; ++k) {
      const int c = tid + k * NT;
      if (c < w.ca + w.cb) {
        if constexpr (KV) load_chunk(w, c, pk[k], pv[k]);
        else load_chunk(w, c, pk[k], pv[0]);
      }
    }
  };
  auto commit = [&](const Window &w) {
#pragma unroll
    for (int k = 0; k < PV; ++k) {
      const int c = tid + k * NT;
      if (c < w.ca + w.cb) {
        if constexpr (KV) put_chunk(w, c, pk[k], pv[k]);
        else put_chunk(w, c, pk[k], pv[0]);
      }
    }
  };
  // Lower-bound split search on local diagonal dl inside the loaded windows.
  auto local_search = [&](const Window &w, int dl) {
    int lo, hi;
    diag_range<int>(dl, w.la, w.lb, lo, hi);
    const K *ka = keys + w.sa;
    const K *kb = keys + OB + w.sb;
    return split_search<int>(
        dl, lo, hi, [&](int i) { return ka[i]; }, [&](int j) { return kb[j]; });
  };
  // End split of the tile plus the window-edge test (lane 0 only).
  auto end_search = [&](const Window &w) {
    int lo, hi;
    diag_range<int>(w.n, w.la, w.lb, lo, hi);
    const int r = local_search(w, w.n);
    int tlo, thi;  // bounds over the full extents
    diag_range<int>(w.n, w.wa, w.wb, tlo, thi);
    s_end = r;
    s_valid = lo <= hi && (r < hi || hi == thi) && (r > lo || lo == tlo);
  };

  if (tid < 64) {
    const int64_t d = t_begin * T < n_all ? t_begin * T : n_all;
    const int64_t a = wave_split_search<K>(A, na, B, nb, d);
    if (tid == 0) s_split = a;
  }
  __syncthreads();
  int64_t a_cur = s_split;
  int64_t b_cur = t_begin * T - a_cur;
  const int n0 = (int)(n_all - t_begin * T < T ? n_all - t_begin * T : T);
  Window w = make_window<CH>(a_cur, b_cur, na, nb, n0, n0, n0);
  load_now(w);
  __syncthreads();

  for (int64_t t = t_begin; t < t_end; ++t) {
    const int64_t d0 = t * T;
    const int n = w.n;
    const int dl = tid * VT < n ? tid * VT : n;
    if (tid == 0) end_search(w);
    int a_own = local_search(w, dl);
    __syncthreads();
    if (!s_valid) {
      // The split left the speculative windows: load the full ones (exact).
      w = make_window<CH>(a_cur, b_cur, na, nb, n, n, n);
      load_now(w);
      __syncthreads();
      if (tid == 0) end_search(w);
      a_own = local_search(w, dl);
      __syncthreads();
    }
    const int a_end = s_end;
    const int64_t a_next = a_cur + a_end, b_next = b_cur + (n - a_end);

    // Fetch the next tile's windows while this tile is merged.
    Window wn = w;
    const bool more = t + 1 < t_end;
    if (more) {
      const int64_t d1 = d0 + T;
      const int n1 = (int)(n_all - d1 < T ? n_all - d1 : T);
      const int pa = speculate ? a_end + M : n1;
      const int pb = speculate ? (n - a_end) + M : n1;
      wn = make_window<CH>(a_next, b_next, na, nb, n1, pa, pb);
      // register prefetch holds speculative windows only; full windows are
      // loaded at commit time
      if (speculate) prefetch(wn);
    }

    K out[VT];
    int src[VT];
    serial_merge<K, VT>(keys, w.sa + a_own, OB + w.sb + (dl - a_own), w.sa + w.la,
                        OB + w.sb + w.lb, out, src);
    const int steps = n - dl < VT ? n - dl : VT;
    uint32_t ov[VT];
    if constexpr (KV) {
#pragma unroll
      for (int i = 0; i < VT; ++i) ov[i] = vals[src[i]];
    }
    __syncthreads();

    bool staged = false;
    if constexpr ((VT * sizeof(K)) % 16 == 0) {
      if (n == T) {
        // full tile: each lane's VT outputs as 16-byte LDS stores
#pragma unroll
        for (int i = 0; i < VT; i += VEC)
          *reinterpret_cast<u32x4 *>(keys + tid * VT + i) =
              *reinterpret_cast<const u32x4 *>(out + i);
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

    if constexpr (VECTOR) {
      const int nvec = n / VEC;
      u32x4 *vdst = reinterpret_cast<u32x4 *>(S + d0);
      const u32x4 *vsrc = reinterpret_cast<const u32x4 *>(keys);
      for (int v = tid; v < nvec; v += NT) __builtin_nontemporal_store(vsrc[v], vdst + v);
      for (int i = nvec * VEC + tid; i < n; i += NT) S[d0 + i] = keys[i];
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

    if (more) {
      if (speculate) commit(wn);
      else load_now(wn);
      __syncthreads();
    }
    a_cur = a_next;
    b_cur = b_next;
    w = wn;
  }
}

template <typename K, bool KV, int NT, int VT>
static hipError_t launch_stream_impl(int grid, int margin, bool vec, const K *A,
                                     const uint32_t *Av, int64_t na, const K *B,
                                     const uint32_t *Bv, int64_t nb, K *S,
                                     uint32_t *Sv, hipStream_t s) {
  constexpr int64_t T = NT * VT;
  const int64_t n_tiles = (na + nb + T - 1) / T;
  if (n_tiles == 0) return hipSuccess;
  if (grid <= 0) {
    // one full wave of resident workgroups
    static int per_cu = 0;
    if (per_cu == 0) {
      int occ = 0;
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
              &occ, merge_stream_kernel<K, KV, NT, VT, true>, NT, 0) != hipSuccess ||
          occ <= 0)
        occ = 1;
      per_cu = occ;
    }
    grid = per_cu * device_cu_count();
  }
  if (margin == 0) margin = 64 + (int)(T / 16);  // default prediction margin
  const int64_t G = grid < n_tiles ? grid : n_tiles;
  if (vec)
    hipLaunchKernelGGL((merge_stream_kernel<K, KV, NT, VT, true>), dim3((unsigned)G),
                       dim3(NT), 0, s, A, Av, na, B, Bv, nb, S, Sv, n_tiles, margin);
  else
    hipLaunchKernelGGL((merge_stream_kernel<K, KV, NT, VT, false>), dim3((unsigned)G),
                       dim3(NT), 0, s, A, Av, na, B, Bv, nb, S, Sv, n_tiles, margin);
  return hipGetLastError();
}

template <typename K>
hipError_t launch_merge_stream(StreamCfg cfg, const K *A, const uint32_t *Av,
                               int64_t na, const K *B, const uint32_t *Bv,
                               int64_t nb, K *S, uint32_t *Sv, hipStream_t s) {
  const bool kv = Sv != nullptr;
  // 16-byte paths need 16-byte aligned base pointers.
  const bool vec = ((uintptr_t)A % 16 == 0) && ((uintptr_t)B % 16 == 0) &&
                   ((uintptr_t)S % 16 == 0) &&
                   (!kv || ((uintptr_t)Sv % 16 == 0 && (uintptr_t)Av % 16 == 0 &&
                            (uintptr_t)Bv % 16 == 0));
#define MP_STREAM_CASE(NT_, VT_)                                                 \
  if (cfg.nt == NT_ && cfg.vt == VT_)                                            \
    return kv ? launch_stream_impl<K, true, NT_, VT_>(cfg.grid, cfg.margin, vec, \
                                                      A, Av, na, B, Bv, nb, S,   \
                                                      Sv, s)                     \
              : launch_stream_impl<K, false, NT_, VT_>(cfg.grid, cfg.margin, vec,\
                                                       A, Av, na, B, Bv, nb, S,  \
                                                       Sv, s);
  MP_STREAM_CASE(256, 16)
  MP_STREAM_CASE(256, 8)
  MP_STREAM_CASE(256, 12)
  MP_STREAM_CASE(128, 16)
  MP_STREAM_CASE(512, 8)
#undef MP_STREAM_CASE
  return hipErrorNotSupported;
}

#define MP_INSTANTIATE(K)                                                       \
  template hipError_t launch_merge_stream<K>(StreamCfg, const K *,              \
                                             const uint32_t *, int64_t,         \
                                             const K *, const uint32_t *,       \
                                             int64_t, K *, uint32_t *, hipStream_t);
MP_INSTANTIATE(uint32_t)
MP_INSTANTIATE(int32_t)
MP_INSTANTIATE(uint64_t)
MP_INSTANTIATE(float)
#undef MP_INSTANTIATE

}  // namespace mp
