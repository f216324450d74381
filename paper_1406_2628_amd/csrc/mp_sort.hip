// Block sort: the first stage of the cache-efficient merge sort (section 4.2:
// sort blocks sized to on-chip memory, then merge rounds), with LDS as the
// cache.  One workgroup of NT lanes sorts a block of NT * VT keys (VT = 16,
// or 32 for 4-byte keys without values):
//   1. every lane sorts its VT keys in registers with Batcher's odd-even
//      merge network.  Where the order of equal keys can be seen (values
//      travel with the keys, or float keys, whose +0 and -0 compare equal),
//      the network orders (key, position) pairs, which makes it stable;
//   2. rounds of Merge Path inside LDS merge runs of VT, 2 VT, ..., NT VT / 2
//      keys pairwise: the lanes of a run pair each find their split at local
//      diagonal q * VT (Algorithm 2) and merge VT outputs serially, left run
//      as A so that ties keep input order (section 2.1 tie rule).  Outputs
//      go to registers, and after a barrier back to the same LDS positions,
//      so one LDS copy of the block suffices.
// The block sits in LDS with one padding slot per 128 bytes (lds_pos) to keep
// the lanes' strided accesses on distinct banks.
// A short last block pads only the registers of its last lane (with the
// largest key, ordered after every real key) and is bounded by index
// everywhere else.
#include <type_traits>

#include "mp_device.h"
#include "mp_internal.h"

namespace mp {

template <typename K>
__device__ __forceinline__ K key_max() {
  if constexpr (std::is_same<K, float>::value) return __builtin_huge_valf();
  else if constexpr (std::is_same<K, int32_t>::value) return (int32_t)0x7fffffff;
  else return ~(K)0;
}

// Batcher's odd-even merge sort on N (a power of two) register slots, as a
// compile-time sequence of compare-exchanges ce(i, j), i < j.
template <int N, typename CE>
__device__ __forceinline__ void oddeven_merge_sort(CE ce) {
#pragma unroll
  for (int p = 1; p < N; p <<= 1)
#pragma unroll
    for (int k = p; k >= 1; k >>= 1)
#pragma unroll
      for (int j = k % p; j + k < N; j += 2 * k)
#pragma unroll
        for (int i = 0; i < k; ++i)
          if (i + j + k < N && (i + j) / (2 * p) == (i + j + k) / (2 * p)) ce(i + j, i + j + k);
}

// LDS slot of element i of a block: one padding element after every 128
// bytes.  Lane runs start VT keys apart and their search probes and merge
// reads start at multiples of 8 keys, which without padding fall into a few
// of the 32 four-byte banks; with it they spread over all of them.  A lane's
// run (VT keys: 64 or 128 bytes for 4-byte keys, 128 for 8-byte keys) never
// crosses a padding slot.
template <typename T>
__host__ __device__ constexpr int lds_pos(int i) {
  return i + (i >> (sizeof(T) == 8 ? 4 : 5));
}

// in and out may be the same array (each block is read whole before it is
// written), so they are not declared __restrict__.  vec: all four arrays are
// 16-byte aligned (full blocks then move as 16-byte vectors).
template <typename K, bool KV, int NT, int VT>
__global__ __launch_bounds__(NT) void blocksort_kernel(const K *in, const uint32_t *vin,
                                                       K *out, uint32_t *vout, int64_t n,
                                                       int vec) {
  constexpr int BS = NT * VT;
  constexpr int VEC = 16 / (int)sizeof(K);
  constexpr bool STABLE = KV || std::is_floating_point<K>::value;
  // VT + 1 slack slots for the unguarded steps of the serial merge
  constexpr int SLOTS = BS + VT + 1;
  __shared__ K keys[lds_pos<K>(SLOTS - 1) + 1];
  __shared__ uint32_t vals[KV ? lds_pos<uint32_t>(SLOTS - 1) + 1 : 1];
  auto key_at = [&](int i) -> K { return keys[lds_pos<K>(i)]; };
  const int tid = threadIdx.x;
  const int64_t base = (int64_t)blockIdx.x * BS;
  const int cnt = (int)(n - base < BS ? n - base : BS);
  const bool full_vec = vec && cnt == BS;

  // A 16-byte chunk, and a lane's run of VT keys, never crosses a padding
  // slot (rows hold whole chunks and whole runs), so each is contiguous in LDS
  // from the slot of its first element.
  if (full_vec) {
    const u32x4 *src = reinterpret_cast<const u32x4 *>(in + base);
#pragma unroll
    for (int j = 0; j < BS / VEC / NT; ++j) {
      const int v = tid + j * NT;
      K t[VEC];
      *reinterpret_cast<u32x4 *>(t) = src[v];
      const int p = lds_pos<K>(v * VEC);
#pragma unroll
      for (int e = 0; e < VEC; ++e) keys[p + e] = t[e];
    }
    if constexpr (KV) {
      const u32x4 *vs = reinterpret_cast<const u32x4 *>(vin + base);
#pragma unroll
      for (int j = 0; j < BS / 4 / NT; ++j) {
        const int v = tid + j * NT;
        uint32_t t[4];
        *reinterpret_cast<u32x4 *>(t) = vs[v];
        const int p = lds_pos<uint32_t>(v * 4);
#pragma unroll
        for (int e = 0; e < 4; ++e) vals[p + e] = t[e];
      }
    }
  } else {
    for (int i = tid; i < cnt; i += NT) {
      keys[lds_pos<K>(i)] = in[base + i];
      if constexpr (KV) vals[lds_pos<uint32_t>(i)] = vin[base + i];
    }
  }
  __syncthreads();

  // 1. per-lane sort of VT keys
  {
    const int own = tid * VT;
    const int c = cnt - own < 0 ? 0 : (cnt - own < VT ? cnt - own : VT);
    const int po = lds_pos<K>(own);
    K k[VT];
#pragma unroll
    for (int i = 0; i < VT; ++i) k[i] = i < c ? keys[po + i] : key_max<K>();
    if constexpr (STABLE) {
      int ix[VT];
#pragma unroll
      for (int i = 0; i < VT; ++i) ix[i] = i;
      oddeven_merge_sort<VT>([&](int a, int b) {
        const bool sw = k[b] < k[a] || (!(k[a] < k[b]) && ix[b] < ix[a]);
        const K ka = k[a], kb = k[b];
        const int ia = ix[a], ib = ix[b];
        k[a] = sw ? kb : ka;
        k[b] = sw ? ka : kb;
        ix[a] = sw ? ib : ia;
        ix[b] = sw ? ia : ib;
      });
      // padding sorts after every real key (largest key, later position), so
      // slots [0, c) hold the c real keys
      if constexpr (KV) {
        const int pv = lds_pos<uint32_t>(own);
        uint32_t v[VT];
#pragma unroll
        for (int i = 0; i < VT; ++i) v[i] = vals[pv + ix[i]];
#pragma unroll
        for (int i = 0; i < VT; ++i)
          if (i < c) vals[pv + i] = v[i];
      }
    } else {
      // integer keys alone: equal keys are indistinguishable, and a padding
      // key equal to a real one has the same bits
      oddeven_merge_sort<VT>([&](int a, int b) {
        const K ka = k[a], kb = k[b];
        k[a] = kb < ka ? kb : ka;
        k[b] = kb < ka ? ka : kb;
      });
    }
#pragma unroll
    for (int i = 0; i < VT; ++i)
      if (i < c) keys[po + i] = k[i];
  }
  __syncthreads();

  // 2. Merge Path rounds inside LDS
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
    int lo, hi;
    diag_range<int>(dl, na, nb, lo, hi);
    const int a = split_search<int>(
        dl, lo, hi, [&](int i) { return key_at(a0 + i); }, [&](int j) { return key_at(b0 + j); });
    // serial merge of VT outputs (Lemma 1), A run [a0, b0), B run [b0, e);
    // steps past the pair's end only read slots below e + VT
    K o[VT];
    int s[VT];
    {
      int ai = a0 + a, bi = b0 + (dl - a);
      K ka = key_at(ai), kb = key_at(bi);
#pragma unroll
      for (int i = 0; i < VT; ++i) {
        const bool take_b = (bi < e) && (ai >= b0 || kb < ka);
        o[i] = take_b ? kb : ka;
        const int taken = take_b ? bi : ai;
        s[i] = taken;
        ai = take_b ? ai : taken + 1;
        bi = take_b ? taken + 1 : bi;
        const K nxt = key_at(taken + 1);
        ka = take_b ? ka : nxt;
        kb = take_b ? nxt : kb;
      }
    }
    uint32_t ov[KV ? VT : 1];
    if constexpr (KV) {
#pragma unroll
      for (int i = 0; i < VT; ++i) ov[i] = vals[lds_pos<uint32_t>(s[i])];
    }
    const int steps = na + nb - dl < VT ? na + nb - dl : VT;
    __syncthreads();
    // outputs a0 + dl + [0, VT) are a lane run: contiguous slots
    const int at = a0 + dl, pk = lds_pos<K>(at);
#pragma unroll
    for (int i = 0; i < VT; ++i)
      if (i < steps) keys[pk + i] = o[i];
    if constexpr (KV) {
      const int pv = lds_pos<uint32_t>(at);
#pragma unroll
      for (int i = 0; i < VT; ++i)
        if (i < steps) vals[pv + i] = ov[i];
    }
    __syncthreads();
  }

  if (full_vec) {
    u32x4 *dst = reinterpret_cast<u32x4 *>(out + base);
#pragma unroll
    for (int j = 0; j < BS / VEC / NT; ++j) {
      const int v = tid + j * NT;
      const int p = lds_pos<K>(v * VEC);
      K t[VEC];
#pragma unroll
      for (int e = 0; e < VEC; ++e) t[e] = keys[p + e];
      __builtin_nontemporal_store(*reinterpret_cast<const u32x4 *>(t), dst + v);
    }
    if constexpr (KV) {
      u32x4 *vd = reinterpret_cast<u32x4 *>(vout + base);
#pragma unroll
      for (int j = 0; j < BS / 4 / NT; ++j) {
        const int v = tid + j * NT;
        const int p = lds_pos<uint32_t>(v * 4);
        uint32_t t[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) t[e] = vals[p + e];
        __builtin_nontemporal_store(*reinterpret_cast<const u32x4 *>(t), vd + v);
      }
    }
  } else {
    for (int i = tid; i < cnt; i += NT) {
      out[base + i] = keys[lds_pos<K>(i)];
      if constexpr (KV) vout[base + i] = vals[lds_pos<uint32_t>(i)];
    }
  }
}

// Larger blocks leave fewer merge rounds in HBM (each reads and writes every
// key once) for one more round in LDS each.  4-byte keys: 16384-key blocks
// (512 lanes x 32 keys, 68 KB of LDS; with values 1024 x 16, 135 KB).
// 8-byte keys: 8192 (70 KB, 104 KB with values; 16384 would not fit with
// values).
int sort_block_log2(size_t key_bytes, bool kv) {
  (void)kv;
  return key_bytes == 8 ? 13 : 14;
}

template <typename K, bool KV, int NT, int VT = 16>
hipError_t launch_blocksort_nt(const K *in, const uint32_t *vin, K *out, uint32_t *vout,
                               int64_t n, hipStream_t s) {
  constexpr int64_t BS = NT * VT;
  const int64_t blocks = (n + BS - 1) / BS;
  if (blocks == 0) return hipSuccess;
  auto a16 = [](const void *p) { return ((uintptr_t)p % 16) == 0; };
  const int vec = a16(in) && a16(out) && (!KV || (a16(vin) && a16(vout)));
  hipLaunchKernelGGL((blocksort_kernel<K, KV, NT, VT>), dim3((unsigned)blocks), dim3(NT), 0, s, in,
                     vin, out, vout, n, vec);
  return hipGetLastError();
}

template <typename K>
hipError_t launch_blocksort(const K *in, const uint32_t *vin, K *out, uint32_t *vout,
                            int64_t n, int log2_block, hipStream_t s) {
  const bool kv = vout != nullptr;
  switch (log2_block) {
    case 12:
      return kv ? launch_blocksort_nt<K, true, 256>(in, vin, out, vout, n, s)
                : launch_blocksort_nt<K, false, 256>(in, vin, out, vout, n, s);
    case 13:
      return kv ? launch_blocksort_nt<K, true, 512>(in, vin, out, vout, n, s)
                : launch_blocksort_nt<K, false, 512>(in, vin, out, vout, n, s);
    case 14:
      // 16384 keys of 8 bytes would need 128 KB (with values, more than a
      // workgroup's LDS); 4-byte keys alone go 32 to a lane (one LDS round
      // fewer, 12-15% faster than 16 per lane), with values 16 (32 measured
      // 7% slower: 169 registers, one workgroup per CU)
      if constexpr (sizeof(K) == 8) return hipErrorInvalidValue;
      else if (kv) return launch_blocksort_nt<K, true, 1024>(in, vin, out, vout, n, s);
      else return launch_blocksort_nt<K, false, 512, 32>(in, vin, out, vout, n, s);
    default:
      return hipErrorInvalidValue;
  }
}

#define MP_INSTANTIATE(K)                                                        \
  template hipError_t launch_blocksort<K>(const K *, const uint32_t *, K *,      \
                                          uint32_t *, int64_t, int, hipStream_t);
MP_INSTANTIATE(uint32_t)
MP_INSTANTIATE(int32_t)
MP_INSTANTIATE(uint64_t)
MP_INSTANTIATE(float)
#undef MP_INSTANTIATE

}  // namespace mp
