// C ABI layer: host-side argument validation, dtype dispatch and launches.
// Validation never touches device memory, so every argument error is
// reported before any work is enqueued.
#include <algorithm>
#include <mutex>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>
#include <vector>

#include "mp_internal.h"

namespace mp {
namespace {

thread_local char g_err[512] = "";

mp_status fail(mp_status st, const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
  return st;
}

mp_status hip_fail(hipError_t e, const char *what) {
  return fail(MP_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

bool is_key(mp_dtype t) {
  return t == MP_U32 || t == MP_I32 || t == MP_U64 || t == MP_F32;
}
bool is_val32(mp_dtype t) { return t == MP_U32 || t == MP_I32 || t == MP_F32; }

struct Range {
  uintptr_t lo, hi;
};
Range span(const void *p, int64_t n, size_t es) {
  const uintptr_t b = (uintptr_t)p;
  return Range{b, b + (uintptr_t)n * es};
}
bool overlaps(Range x, Range y) {
  return x.lo < x.hi && y.lo < y.hi && x.lo < y.hi && y.lo < x.hi;
}

mp_status check_array(const void *p, int64_t n, size_t es, const char *name) {
  if (n < 0) return fail(MP_ERR_INVALID_ARG, "%s: negative size %lld", name, (long long)n);
  if (n > 0 && p == nullptr) return fail(MP_ERR_INVALID_ARG, "%s: NULL pointer with size %lld", name, (long long)n);
  if (n > 0 && ((uintptr_t)p % es) != 0) return fail(MP_ERR_INVALID_ARG, "%s: pointer not aligned to %zu bytes", name, es);
  return MP_OK;
}

enum Op { kOpMerge = 0, kOpBatched = 1, kOpSort = 2, kNumOps = 3 };

// Built-in variant per operation (chosen from measurements on MI355X):
// merges and sort rounds per tile with the tile picked from the size (nt = vt
// = 0), batches persistent.
const mp_config kDefaultConfig[kNumOps] = {
    {1, 0, 0, 0, 0},     // merge
    {1, 0, 0, 0, 0},     // batched
    {1, 0, 0, 0, 0},     // sort rounds
};
// Batches too large for 32-bit pair and tile indices stay on the persistent
// kernel in the built-in configuration.
const mp_config kBatchedPersistent = {2, 256, 16, 0, 0};
// The persistent shape the no-store diagnostic uses when the merge is not
// set to a persistent shape that has a no-store variant.
const mp_config kChecksumConfig = {2, 192, 24, 0, 0};
mp_config g_config[kNumOps] = {kDefaultConfig[0], kDefaultConfig[1], kDefaultConfig[2]};
// Whether g_config[op] was chosen (mp_set_config or the autotuner) rather
// than being the built-in choice.
bool g_config_chosen[kNumOps] = {false, false, false};

mp_config current_config(Op op) { return g_config[op]; }

int op_index(const char *name) {
  if (!name) return -1;
  if (!strcmp(name, "merge")) return kOpMerge;
  if (!strcmp(name, "batched")) return kOpBatched;
  if (!strcmp(name, "sort")) return kOpSort;
  return -1;
}

}  // namespace

int g_last_pairs_grid = 0;

mp_status set_error(mp_status st, const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
  return st;
}

// Largest tile of the key's ladder that still leaves at least two tiles per
// compute unit (smaller tiles only for small merges).  The ladders keep a
// tile's LDS at or under 72 KB: 16384 keys of 4 bytes (1024 x 16), 8192 of
// 8 bytes (1024 x 8) or of 4 bytes with values (512 x 16: 3-5% faster than
// 1024 x 8), 6144 of 8 bytes with values (512 x 12: 1.11 against 1.17 ms
// for 2^27 + 2^27 u64 keys with values at 256 x 16).
TileCfg auto_tile_cfg(size_t key_bytes, bool kv, int64_t n) {
  static const TileCfg k4[] = {{1024, 16}, {512, 16}, {256, 16}, {256, 8}};
  static const TileCfg k4v[] = {{512, 16}, {256, 16}, {256, 8}};
  static const TileCfg k8[] = {{1024, 8}, {256, 16}, {256, 8}};
  static const TileCfg k8v[] = {{512, 12}, {256, 16}, {256, 8}};
  const TileCfg *lad = key_bytes == 8 ? (kv ? k8v : k8) : (kv ? k4v : k4);
  const int len = key_bytes == 8 ? 3 : (kv ? 3 : 4);
  const int64_t want = 2 * (int64_t)device_cu_count();
  for (int i = 0; i < len; ++i)
    if (n / ((int64_t)lad[i].nt * lad[i].vt) >= want) return lad[i];
  return lad[len - 1];
}

int device_cu_count() {
  static std::mutex mu;
  static std::vector<int> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  std::lock_guard<std::mutex> lock(mu);
  if ((int)cache.size() <= dev) cache.resize(dev + 1, 0);
  if (cache[dev] == 0) {
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0)
      n = 256;
    cache[dev] = n;
  }
  return cache[dev];
}

}  // namespace mp

using namespace mp;

extern "C" {

const char *mp_last_error(void) { return g_err; }

int mp_version(void) { return 100; }

mp_status mp_partition(mp_dtype kt, const void *A, int64_t na, const void *B,
                       int64_t nb, const int64_t *diag, int64_t n_diag,
                       int64_t *a_split, void *stream) {
  if (!is_key(kt)) return fail(MP_ERR_UNSUPPORTED, "mp_partition: unsupported key dtype %d", (int)kt);
  const size_t es = dtype_size(kt);
  mp_status st;
  if ((st = check_array(A, na, es, "A")) != MP_OK) return st;
  if ((st = check_array(B, nb, es, "B")) != MP_OK) return st;
  if ((st = check_array(diag, n_diag, 8, "diag")) != MP_OK) return st;
  if ((st = check_array(a_split, n_diag, 8, "a_split")) != MP_OK) return st;
  const Range out = span(a_split, n_diag, 8);
  if (overlaps(out, span(A, na, es)) || overlaps(out, span(B, nb, es)) ||
      overlaps(out, span(diag, n_diag, 8)))
    return fail(MP_ERR_OVERLAP, "mp_partition: a_split overlaps an input");
  if (n_diag == 0) return MP_OK;
  hipError_t e = hipSuccess;
  dispatch_key(kt, [&](auto k) {
    using K = decltype(k);
    KernelTimer timer("partition", (hipStream_t)stream);
    e = launch_partition<K>((const K *)A, na, (const K *)B, nb, diag, 0, n_diag,
                            a_split, (hipStream_t)stream);
  });
  return e == hipSuccess ? MP_OK : hip_fail(e, "mp_partition launch");
}

static mp_status merge_common(const char *fn, mp_dtype kt, mp_dtype vt,
                              const void *Ak, const void *Av, int64_t na,
                              const void *Bk, const void *Bv, int64_t nb,
                              void *Sk, void *Sv, void *stream) {
  if (!is_key(kt)) return fail(MP_ERR_UNSUPPORTED, "%s: unsupported key dtype %d", fn, (int)kt);
  const bool kv = vt != MP_NONE;
  if (kv && !is_val32(vt)) return fail(MP_ERR_UNSUPPORTED, "%s: unsupported value dtype %d", fn, (int)vt);
  const size_t es = dtype_size(kt);
  mp_status st;
  if ((st = check_array(Ak, na, es, "A")) != MP_OK) return st;
  if ((st = check_array(Bk, nb, es, "B")) != MP_OK) return st;
  if (na > INT64_MAX - nb) return fail(MP_ERR_INVALID_ARG, "%s: na + nb overflows", fn);
  const int64_t n = na + nb;
  if ((st = check_array(Sk, n, es, "S")) != MP_OK) return st;
  const Range rs = span(Sk, n, es);
  if (overlaps(rs, span(Ak, na, es)) || overlaps(rs, span(Bk, nb, es)))
    return fail(MP_ERR_OVERLAP, "%s: output keys overlap an input", fn);
  if (kv) {
    if ((st = check_array(Av, na, 4, "Av")) != MP_OK) return st;
    if ((st = check_array(Bv, nb, 4, "Bv")) != MP_OK) return st;
    if ((st = check_array(Sv, n, 4, "Sv")) != MP_OK) return st;
    const Range rv = span(Sv, n, 4);
    if (overlaps(rv, span(Av, na, 4)) || overlaps(rv, span(Bv, nb, 4)) ||
        overlaps(rv, span(Ak, na, es)) || overlaps(rv, span(Bk, nb, es)) ||
        overlaps(rv, rs) || overlaps(rs, span(Av, na, 4)) ||
        overlaps(rs, span(Bv, nb, 4)))
      return fail(MP_ERR_OVERLAP, "%s: an output overlaps an input or the other output", fn);
  }
  if (n == 0) return MP_OK;

  hipStream_t s = (hipStream_t)stream;
  const mp_config cfg = current_config(kOpMerge);
  hipError_t e = hipSuccess;
  if (cfg.mode == 1) {
    // split search on the tile diagonals, then one workgroup per tile
    const TileCfg tc = cfg.nt > 0 ? TileCfg{cfg.nt, cfg.vt} : auto_tile_cfg(es, kv, n);
    dispatch_key(kt, [&](auto k) {
      using K = decltype(k);
      KernelTimer timer("merge_tiles", s);
      e = launch_merge_tiles<K>(tc, (const K *)Ak, (const uint32_t *)Av, na,
                                (const K *)Bk, (const uint32_t *)Bv, nb, (K *)Sk,
                                kv ? (uint32_t *)Sv : nullptr, s);
    });
  } else {
    const StreamCfg sc{cfg.nt, cfg.vt, cfg.grid, cfg.margin};
    dispatch_key(kt, [&](auto k) {
      using K = decltype(k);
      KernelTimer timer("merge_stream", s);
      e = launch_merge_stream<K>(sc, (const K *)Ak, (const uint32_t *)Av, na,
                                 (const K *)Bk, (const uint32_t *)Bv, nb, (K *)Sk,
                                 kv ? (uint32_t *)Sv : nullptr, s);
    });
  }
  if (e == hipErrorNotSupported)
    return fail(MP_ERR_UNSUPPORTED, "%s: configuration mode=%d nt=%d vt=%d not compiled in",
                fn, cfg.mode, cfg.nt, cfg.vt);
  return e == hipSuccess ? MP_OK : hip_fail(e, "merge launch");
}

mp_status mp_merge(mp_dtype kt, const void *A, int64_t na, const void *B,
                   int64_t nb, void *S, void *stream) {
  return merge_common("mp_merge", kt, MP_NONE, A, nullptr, na, B, nullptr, nb, S,
                      nullptr, stream);
}

size_t mp_set_op_workspace_bytes(int64_t na, int64_t nb) {
  if (na < 0 || nb < 0 || na > INT64_MAX - nb) return 0;
  return (size_t)(3 * (setop_tiles(na + nb) + 1)) * sizeof(int64_t);
}

static mp_status set_op_common(const char *fn, int32_t op, mp_dtype kt, const void *A, int64_t na,
                               const void *B, int64_t nb, void *S, int64_t *count, void *ws,
                               size_t ws_bytes, bool noalloc, void *stream) {
  if (op < 0 || op > 3) return fail(MP_ERR_INVALID_ARG, "%s: op must be 0, 1, 2 or 3", fn);
  if (!is_key(kt)) return fail(MP_ERR_UNSUPPORTED, "%s: unsupported key dtype %d", fn, (int)kt);
  const size_t es = dtype_size(kt);
  mp_status st;
  if ((st = check_array(A, na, es, "A")) != MP_OK) return st;
  if ((st = check_array(B, nb, es, "B")) != MP_OK) return st;
  if (na > INT64_MAX - nb) return fail(MP_ERR_INVALID_ARG, "%s: na + nb overflows", fn);
  if (!count || (uintptr_t)count % 8)
    return fail(MP_ERR_INVALID_ARG, "%s: count must be an 8-byte aligned device pointer", fn);
  // largest possible output: every key of A (intersection, difference) or of both
  const int64_t cap = (op == 0 || op == 2) ? na : na + nb;
  if ((st = check_array(S, cap, es, "S")) != MP_OK) return st;
  const size_t need = mp_set_op_workspace_bytes(na, nb);
  if (noalloc) {
    if (need > (size_t)kSetScratchWords * sizeof(int64_t))
      return fail(MP_ERR_UNSUPPORTED,
                  "%s: na + nb = %lld exceeds the %lld keys the fixed scratch serves", fn,
                  (long long)(na + nb), (long long)kSetScratchKeys);
    ws = nullptr;  // set below from the device scratch
  } else {
    if (!ws || ws_bytes < need)
      return fail(MP_ERR_WORKSPACE, "%s: workspace of %zu bytes needed, %zu given", fn, need, ws_bytes);
    if ((uintptr_t)ws % 8) return fail(MP_ERR_INVALID_ARG, "%s: workspace not 8-byte aligned", fn);
  }
  const Range rs = span(S, cap, es), rc = span(count, 1, 8);
  const Range ra = span(A, na, es), rb = span(B, nb, es);
  const Range rw = noalloc ? Range{0, 0} : span(ws, (int64_t)need, 1);
  if (overlaps(rs, ra) || overlaps(rs, rb) || overlaps(rs, rw) || overlaps(rs, rc) ||
      overlaps(rw, ra) || overlaps(rw, rb) || overlaps(rw, rc) || overlaps(rc, ra) ||
      overlaps(rc, rb))
    return fail(MP_ERR_OVERLAP, "%s: S, count, workspace and the inputs must not overlap", fn);
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = hipSuccess;
  if (noalloc) {
    int64_t *p = nullptr;
    e = setop_scratch_ptr(&p);
    if (e != hipSuccess) return hip_fail(e, "mp_set_op_noalloc: scratch address");
    ws = p;
  }
  dispatch_key(kt, [&](auto k) {
    using K = decltype(k);
    KernelTimer timer("set_op", s);
    e = launch_set_op<K>(op, (const K *)A, na, (const K *)B, nb, (K *)S, cap, count,
                         (int64_t *)ws, s);
  });
  return e == hipSuccess ? MP_OK : hip_fail(e, "set operation launch");
}

mp_status mp_set_op(int32_t op, mp_dtype kt, const void *A, int64_t na, const void *B, int64_t nb,
                    void *S, int64_t *count, void *ws, size_t ws_bytes, void *stream) {
  return set_op_common("mp_set_op", op, kt, A, na, B, nb, S, count, ws, ws_bytes, false, stream);
}

mp_status mp_set_op_noalloc(int32_t op, mp_dtype kt, const void *A, int64_t na, const void *B,
                            int64_t nb, void *S, int64_t *count, void *stream) {
  return set_op_common("mp_set_op_noalloc", op, kt, A, na, B, nb, S, count, nullptr, 0, true,
                       stream);
}

size_t mp_join_workspace_bytes(int64_t na, int64_t nb) {
  if (na < 0 || nb < 0 || na > INT64_MAX - nb) return 0;
  return (size_t)join_ws_bytes(na, nb);
}

mp_status mp_join(mp_dtype kt, const void *A, int64_t na, const void *B, int64_t nb, int64_t *I,
                  int64_t *J, int64_t cap, int64_t *count, void *ws, size_t ws_bytes,
                  void *stream) {
  const char *fn = "mp_join";
  if (!is_key(kt)) return fail(MP_ERR_UNSUPPORTED, "%s: unsupported key dtype %d", fn, (int)kt);
  const size_t es = dtype_size(kt);
  mp_status st;
  if ((st = check_array(A, na, es, "A")) != MP_OK) return st;
  if ((st = check_array(B, nb, es, "B")) != MP_OK) return st;
  if (na > INT64_MAX - nb) return fail(MP_ERR_INVALID_ARG, "%s: na + nb overflows", fn);
  if (cap < 0) return fail(MP_ERR_INVALID_ARG, "%s: negative cap", fn);
  if ((st = check_array(I, cap, 8, "I")) != MP_OK) return st;
  if ((st = check_array(J, cap, 8, "J")) != MP_OK) return st;
  if (!count || (uintptr_t)count % 8)
    return fail(MP_ERR_INVALID_ARG, "%s: count must be an 8-byte aligned device pointer", fn);
  const size_t need = mp_join_workspace_bytes(na, nb);
  if (!ws || ws_bytes < need)
    return fail(MP_ERR_WORKSPACE, "%s: workspace of %zu bytes needed, %zu given", fn, need, ws_bytes);
  if ((uintptr_t)ws % 8) return fail(MP_ERR_INVALID_ARG, "%s: workspace not 8-byte aligned", fn);
  const Range ri = span(I, cap, 8), rj = span(J, cap, 8), rc = span(count, 1, 8);
  const Range rw = span(ws, (int64_t)need, 1), ra = span(A, na, es), rb = span(B, nb, es);
  const Range outs[] = {ri, rj, rc, rw};
  for (int x = 0; x < 4; ++x) {
    if (overlaps(outs[x], ra) || overlaps(outs[x], rb))
      return fail(MP_ERR_OVERLAP, "%s: an output or the workspace overlaps an input", fn);
    for (int y = x + 1; y < 4; ++y)
      if (overlaps(outs[x], outs[y]))
        return fail(MP_ERR_OVERLAP, "%s: I, J, count and the workspace must not overlap", fn);
  }
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = hipSuccess;
  dispatch_key(kt, [&](auto k) {
    using K = decltype(k);
    KernelTimer timer("join", s);
    e = launch_join<K>((const K *)A, na, (const K *)B, nb, I, J, cap, count, (int64_t *)ws, s);
  });
  return e == hipSuccess ? MP_OK : hip_fail(e, "mp_join launch");
}

mp_status mp_merge_split(mp_dtype kt, const void *A, int64_t na, const void *B, int64_t nb,
                         const int64_t *a_split, int32_t tile, void *S, void *stream) {
  const char *fn = "mp_merge_split";
  if (!is_key(kt)) return fail(MP_ERR_UNSUPPORTED, "%s: unsupported key dtype %d", fn, (int)kt);
  TileCfg tc{0, 0};
  if (tile == 16384) tc = {1024, 16};
  else if (tile == 8192) tc = {512, 16};
  else if (tile == 4096) tc = {256, 16};
  else if (tile == 3840) tc = {256, 15};
  else if (tile == 2048) tc = {256, 8};
  else return fail(MP_ERR_UNSUPPORTED, "%s: tile must be 2048, 3840, 4096, 8192 or 16384", fn);
  const size_t es = dtype_size(kt);
  mp_status st;
  if ((st = check_array(A, na, es, "A")) != MP_OK) return st;
  if ((st = check_array(B, nb, es, "B")) != MP_OK) return st;
  if (na > INT64_MAX - nb) return fail(MP_ERR_INVALID_ARG, "%s: na + nb overflows", fn);
  const int64_t n = na + nb;
  const int64_t n_tiles = (n + tile - 1) / tile;
  if ((st = check_array(S, n, es, "S")) != MP_OK) return st;
  if (n > 0 && (st = check_array(a_split, n_tiles + 1, 8, "a_split")) != MP_OK) return st;
  const Range rs = span(S, n, es);
  if (overlaps(rs, span(A, na, es)) || overlaps(rs, span(B, nb, es)) ||
      overlaps(rs, span(a_split, n_tiles + 1, 8)))
    return fail(MP_ERR_OVERLAP, "%s: S overlaps an input", fn);
  if (n == 0) return MP_OK;
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = hipSuccess;
  dispatch_key(kt, [&](auto k) {
    using K = decltype(k);
    KernelTimer timer("merge_tiles", s);
    e = launch_merge_tiles_split<K>(tc, (const K *)A, na, (const K *)B, nb, (K *)S, a_split, s);
  });
  if (e == hipErrorNotSupported)
    return fail(MP_ERR_UNSUPPORTED, "%s: tile %d is not built for this key type", fn, tile);
  return e == hipSuccess ? MP_OK : hip_fail(e, "mp_merge_split launch");
}

mp_status mp_merge_checksum(mp_dtype kt, const void *A, int64_t na, const void *B, int64_t nb,
                            uint64_t *checksum, void *stream) {
  const char *fn = "mp_merge_checksum";
  if (!is_key(kt)) return fail(MP_ERR_UNSUPPORTED, "%s: unsupported key dtype %d", fn, (int)kt);
  const size_t es = dtype_size(kt);
  mp_status st;
  if ((st = check_array(A, na, es, "A")) != MP_OK) return st;
  if ((st = check_array(B, nb, es, "B")) != MP_OK) return st;
  if (na > INT64_MAX - nb) return fail(MP_ERR_INVALID_ARG, "%s: na + nb overflows", fn);
  if (!checksum || (uintptr_t)checksum % 8)
    return fail(MP_ERR_INVALID_ARG, "%s: checksum must be an 8-byte aligned device pointer", fn);
  const Range rc = span(checksum, 1, 8);
  if (overlaps(rc, span(A, na, es)) || overlaps(rc, span(B, nb, es)))
    return fail(MP_ERR_OVERLAP, "%s: checksum overlaps an input", fn);
  if (na + nb == 0) return MP_OK;
  mp_config cfg = current_config(kOpMerge);
  // the persistent kernel with the merge's tile when it has a no-store
  // variant, else 192 x 24
  if (cfg.mode != 2 || !((cfg.nt == 192 && cfg.vt == 24) || (cfg.nt == 256 && cfg.vt == 16))) {
    cfg = kChecksumConfig;
  }
  const StreamCfg sc{cfg.nt, cfg.vt, cfg.grid, cfg.margin};
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = hipSuccess;
  dispatch_key(kt, [&](auto k) {
    using K = decltype(k);
    KernelTimer timer("merge_checksum", s);
    e = launch_merge_checksum<K>(sc, (const K *)A, na, (const K *)B, nb,
                                 (unsigned long long *)checksum, s);
  });
  return e == hipSuccess ? MP_OK : hip_fail(e, "mp_merge_checksum launch");
}

mp_status mp_merge_kv(mp_dtype kt, mp_dtype vt, const void *Ak, const void *Av,
                      int64_t na, const void *Bk, const void *Bv, int64_t nb,
                      void *Sk, void *Sv, void *stream) {
  if (vt == MP_NONE) return fail(MP_ERR_INVALID_ARG, "mp_merge_kv: value dtype is MP_NONE");
  return merge_common("mp_merge_kv", kt, vt, Ak, Av, na, Bk, Bv, nb, Sk, Sv, stream);
}

mp_status mp_set_config(const char *op, const mp_config *cfg) {
  const int i = op_index(op);
  if (i < 0) return fail(MP_ERR_INVALID_ARG, "mp_set_config: unknown operation");
  if (!cfg) {
    g_config[i] = kDefaultConfig[i];
    g_config_chosen[i] = false;
    return MP_OK;
  }
  // mode 1 takes nt = vt = 0 for the tile picked from each call's size
  const bool auto_tile = cfg->mode == 1 && cfg->nt == 0 && cfg->vt == 0;
  if ((cfg->mode != 1 && cfg->mode != 2) || cfg->grid < 0 ||
      (!auto_tile && (cfg->nt <= 0 || cfg->vt <= 0)))
    return fail(MP_ERR_INVALID_ARG, "mp_set_config: invalid configuration");
  if (cfg->mode == 1 && i == kOpBatched && !auto_tile &&
      (int64_t)cfg->nt * cfg->vt < kBatchMinTile)
    return fail(MP_ERR_UNSUPPORTED, "mp_set_config: per-tile batches need tiles of at least %lld",
                (long long)kBatchMinTile);
  if (i == kOpSort && !auto_tile) {
    // merge rounds rely on tiles that divide every run pair (2w >= 2 blocks;
    // persistent rounds as built assume the smallest block of 4096)
    const int64_t t = (int64_t)cfg->nt * cfg->vt;
    const int64_t lim = cfg->mode == 1 ? (int64_t)2 << 13 : (int64_t)2 << kSortBlockMinLog2;
    if ((t & (t - 1)) != 0 || t > lim)
      return fail(MP_ERR_UNSUPPORTED, "mp_set_config: sort tiles must be a power of two <= %lld",
                  (long long)lim);
  }
  g_config[i] = *cfg;
  g_config_chosen[i] = true;
  return MP_OK;
}

mp_status mp_copy(const void *src, void *dst, int64_t n_bytes, int32_t unroll,
                  int32_t grid, void *stream) {
  if (n_bytes < 0 || n_bytes % 16) return fail(MP_ERR_INVALID_ARG, "mp_copy: n_bytes must be a non-negative multiple of 16");
  if (n_bytes == 0) return MP_OK;
  if (!src || !dst || ((uintptr_t)src % 16) || ((uintptr_t)dst % 16))
    return fail(MP_ERR_INVALID_ARG, "mp_copy: pointers must be non-NULL and 16-byte aligned");
  if (overlaps(span(src, n_bytes, 1), span(dst, n_bytes, 1)))
    return fail(MP_ERR_OVERLAP, "mp_copy: ranges overlap");
  KernelTimer timer("copy", (hipStream_t)stream);
  if (grid < 0) return fail(MP_ERR_INVALID_ARG, "mp_copy: negative grid");
  hipError_t e = launch_copy(src, dst, n_bytes, unroll, grid, (hipStream_t)stream);
  if (e == hipErrorNotSupported) return fail(MP_ERR_UNSUPPORTED, "mp_copy: unroll %d not provided", unroll);
  return e == hipSuccess ? MP_OK : hip_fail(e, "mp_copy launch");
}

mp_status mp_bw_probe(int32_t kind, const void *src, void *dst, int64_t n_bytes, int32_t unroll,
                      int32_t grid, void *stream) {
  const char *fn = "mp_bw_probe";
  if (kind < 0 || kind > 2) return fail(MP_ERR_INVALID_ARG, "%s: kind must be 0, 1 or 2", fn);
  if (n_bytes < 0 || n_bytes % 16)
    return fail(MP_ERR_INVALID_ARG, "%s: n_bytes must be a non-negative multiple of 16", fn);
  if (grid < 0) return fail(MP_ERR_INVALID_ARG, "%s: negative grid", fn);
  if (n_bytes == 0) return MP_OK;
  const int g = grid > 0 ? grid : device_cu_count() * 32;
  const bool need_src = kind != 2;
  if ((need_src && (!src || (uintptr_t)src % 16)) || !dst || (uintptr_t)dst % 16)
    return fail(MP_ERR_INVALID_ARG, "%s: pointers must be non-NULL and 16-byte aligned", fn);
  // the read probe's sink holds one 16-byte word per wavefront
  const int64_t dst_bytes = kind == 1 ? (int64_t)g * 4 * 16 : n_bytes;
  if (need_src && overlaps(span(src, n_bytes, 1), span(dst, dst_bytes, 1)))
    return fail(MP_ERR_OVERLAP, "%s: ranges overlap", fn);
  KernelTimer timer("bw_probe", (hipStream_t)stream);
  hipError_t e = launch_bw_probe(kind, src, dst, n_bytes, unroll, g, (hipStream_t)stream);
  if (e == hipErrorNotSupported) return fail(MP_ERR_UNSUPPORTED, "%s: unroll %d not provided", fn, unroll);
  return e == hipSuccess ? MP_OK : hip_fail(e, "mp_bw_probe launch");
}

size_t mp_merge_batched_workspace_bytes(mp_dtype kt, int64_t n_pairs, int64_t total) {
  (void)kt;
  if (n_pairs < 0 || total < 0) return 0;
  return (size_t)batch_tile_ws_bytes(total);
}

mp_status mp_merge_batched(mp_dtype kt, const void *A, const int64_t *a_off,
                           const void *B, const int64_t *b_off, int64_t n_pairs,
                           int64_t total_a, int64_t total_b, void *S, void *ws,
                           size_t ws_bytes, void *stream) {
  const char *fn = "mp_merge_batched";
  if (!is_key(kt)) return fail(MP_ERR_UNSUPPORTED, "%s: unsupported key dtype %d", fn, (int)kt);
  if (n_pairs < 0) return fail(MP_ERR_INVALID_ARG, "%s: negative pair count", fn);
  const size_t es = dtype_size(kt);
  mp_status st;
  if ((st = check_array(A, total_a, es, "A")) != MP_OK) return st;
  if ((st = check_array(B, total_b, es, "B")) != MP_OK) return st;
  if (total_a > INT64_MAX - total_b) return fail(MP_ERR_INVALID_ARG, "%s: total overflows", fn);
  const int64_t n = total_a + total_b;
  if (n_pairs == 0 && n != 0)
    return fail(MP_ERR_INVALID_ARG, "%s: keys given but no pairs", fn);
  if ((st = check_array(a_off, n_pairs ? n_pairs + 1 : 0, 8, "a_off")) != MP_OK) return st;
  if ((st = check_array(b_off, n_pairs ? n_pairs + 1 : 0, 8, "b_off")) != MP_OK) return st;
  if ((st = check_array(S, n, es, "S")) != MP_OK) return st;
  const Range rs = span(S, n, es);
  if (overlaps(rs, span(A, total_a, es)) || overlaps(rs, span(B, total_b, es)) ||
      overlaps(rs, span(a_off, n_pairs + 1, 8)) || overlaps(rs, span(b_off, n_pairs + 1, 8)))
    return fail(MP_ERR_OVERLAP, "%s: output overlaps an input", fn);
  if (n == 0) return MP_OK;
  mp_config cfg = current_config(kOpBatched);
  TileCfg tc{cfg.nt, cfg.vt};
  // batch tiles index pairs and tiles with 32-bit integers
  const bool tiles_fit = n_pairs < INT32_MAX && (n + kBatchMinTile - 1) / kBatchMinTile < INT32_MAX;
  if (cfg.mode == 1 && cfg.nt == 0) {
    // built-in: 4096-key tiles (256 x 16 measured best from pairs of 64 to
    // 5000 keys), or the persistent kernel past the 32-bit indices
    if (!tiles_fit) cfg = kBatchedPersistent;
    else tc = TileCfg{256, 16};
  }
  if (cfg.mode == 1 && !tiles_fit)
    return fail(MP_ERR_UNSUPPORTED, "%s: batch tiles take fewer than 2^31 - 1 pairs", fn);
  if (cfg.mode == 1) {
    const size_t need = mp_merge_batched_workspace_bytes(kt, n_pairs, n);
    if (!ws || ws_bytes < need)
      return fail(MP_ERR_WORKSPACE, "%s: workspace of %zu bytes needed, %zu given", fn, need, ws_bytes);
    if ((uintptr_t)ws % 8) return fail(MP_ERR_INVALID_ARG, "%s: workspace not 8-byte aligned", fn);
    const Range rw = span(ws, (int64_t)need, 1);
    if (overlaps(rw, rs) || overlaps(rw, span(A, total_a, es)) || overlaps(rw, span(B, total_b, es)) ||
        overlaps(rw, span(a_off, n_pairs + 1, 8)) || overlaps(rw, span(b_off, n_pairs + 1, 8)))
      return fail(MP_ERR_OVERLAP, "%s: workspace overlaps an input or the output", fn);
  }
  const StreamCfg sc{cfg.nt, cfg.vt, cfg.grid, cfg.margin};
  hipStream_t s = (hipStream_t)stream;
  const std::vector<uint64_t> key = {
      1, (uint64_t)kt, (uint64_t)(uintptr_t)A, (uint64_t)(uintptr_t)a_off,
      (uint64_t)(uintptr_t)B, (uint64_t)(uintptr_t)b_off, (uint64_t)n_pairs,
      (uint64_t)total_a, (uint64_t)total_b, (uint64_t)(uintptr_t)S,
      (uint64_t)cfg.mode, (uint64_t)tc.nt, (uint64_t)tc.vt, (uint64_t)cfg.grid,
      (uint64_t)(uint32_t)cfg.margin, (uint64_t)(uintptr_t)ws};
  hipError_t e = run_maybe_graph(key, s, [&](hipStream_t st) {
    hipError_t ee = hipSuccess;
    dispatch_key(kt, [&](auto k) {
      using K = decltype(k);
      KernelTimer timer("merge_batched", st);
      if (cfg.mode == 1)
        ee = launch_merge_batched_tiles<K>(tc, (const K *)A, a_off, (const K *)B, b_off, n_pairs,
                                           total_a, total_b, (K *)S, ws, st);
      else
        ee = launch_merge_batched<K>(sc, (const K *)A, a_off, (const K *)B, b_off, n_pairs,
                                     total_a, total_b, (K *)S, st);
    });
    return ee;
  });
  if (e == hipErrorNotSupported)
    return fail(MP_ERR_UNSUPPORTED, "%s: configuration nt=%d vt=%d not compiled in", fn, cfg.nt, cfg.vt);
  return e == hipSuccess ? MP_OK : hip_fail(e, "mp_merge_batched launch");
}

// Workspace of mp_sort: a second buffer for keys (256-byte aligned) and, with
// values, one for values; merge rounds ping-pong between it and the caller's
// arrays.
static size_t sort_ws_keys_bytes(size_t es, int64_t n) {
  return ((size_t)n * es + 255) & ~(size_t)255;
}

int64_t mp_sort_block_keys(mp_dtype kt, mp_dtype vt) {
  const size_t es = dtype_size(kt);
  if (es == 0 || (vt != MP_NONE && !is_val32(vt))) return 0;
  return (int64_t)1 << sort_block_log2(es, vt != MP_NONE);
}

size_t mp_sort_workspace_bytes(mp_dtype kt, mp_dtype vt, int64_t n) {
  const size_t es = dtype_size(kt);
  if (es == 0 || n <= 0 || (vt != MP_NONE && !is_val32(vt))) return 0;
  return sort_ws_keys_bytes(es, n) + (vt != MP_NONE ? (size_t)n * 4 : 0);
}

mp_status mp_sort(mp_dtype kt, mp_dtype vt, void *keys, void *vals, int64_t n,
                  void *ws, size_t ws_bytes, void *stream) {
  const char *fn = "mp_sort";
  if (!is_key(kt)) return fail(MP_ERR_UNSUPPORTED, "%s: unsupported key dtype %d", fn, (int)kt);
  const bool kv = vt != MP_NONE;
  if (kv && !is_val32(vt)) return fail(MP_ERR_UNSUPPORTED, "%s: unsupported value dtype %d", fn, (int)vt);
  const size_t es = dtype_size(kt);
  mp_status st;
  if ((st = check_array(keys, n, es, "keys")) != MP_OK) return st;
  if (kv && (st = check_array(vals, n, 4, "vals")) != MP_OK) return st;
  if (!kv && vals) return fail(MP_ERR_INVALID_ARG, "%s: values given with value dtype MP_NONE", fn);
  if (n <= 1) return MP_OK;
  const size_t need = mp_sort_workspace_bytes(kt, vt, n);
  if (!ws || ws_bytes < need)
    return fail(MP_ERR_WORKSPACE, "%s: workspace of %zu bytes needed, %zu given", fn, need, ws_bytes);
  if ((uintptr_t)ws % 16) return fail(MP_ERR_INVALID_ARG, "%s: workspace not 16-byte aligned", fn);
  const Range rw = span(ws, (int64_t)need, 1);
  if (overlaps(rw, span(keys, n, es)) || (kv && overlaps(rw, span(vals, n, 4))) ||
      (kv && overlaps(span(keys, n, es), span(vals, n, 4))))
    return fail(MP_ERR_OVERLAP, "%s: workspace, keys and values must not overlap", fn);

  const mp_config cfg = current_config(kOpSort);
  const StreamCfg sc{cfg.nt, cfg.vt, cfg.grid, cfg.margin};
  hipStream_t s = (hipStream_t)stream;
  const int lb = sort_block_log2(es, kv);
  const TileCfg tc = cfg.nt > 0 ? TileCfg{cfg.nt, cfg.vt} : auto_tile_cfg(es, kv, n);
  if (cfg.mode == 1 && (int64_t)tc.nt * tc.vt > ((int64_t)2 << lb))
    return fail(MP_ERR_UNSUPPORTED, "%s: tile %d x %d does not divide a run pair of %lld keys", fn,
                tc.nt, tc.vt, (long long)((int64_t)2 << lb));
  int rounds = 0;
  for (int64_t w = (int64_t)1 << lb; w < n; w <<= 1) ++rounds;
  const std::vector<uint64_t> key = {
      2, (uint64_t)kt, (uint64_t)vt, (uint64_t)(uintptr_t)keys, (uint64_t)(uintptr_t)vals,
      (uint64_t)n, (uint64_t)(uintptr_t)ws, (uint64_t)cfg.nt, (uint64_t)cfg.vt,
      (uint64_t)cfg.grid, (uint64_t)(uint32_t)cfg.margin};
  hipError_t e = run_maybe_graph(key, s, [&](hipStream_t st) {
    hipError_t ee = hipSuccess;
    dispatch_key(kt, [&](auto k) {
      using K = decltype(k);
      K *kb[2] = {(K *)keys, (K *)ws};
      uint32_t *vb[2] = {(uint32_t *)vals,
                         kv ? (uint32_t *)((char *)ws + sort_ws_keys_bytes(es, n)) : nullptr};
      // Choose where the sorted blocks land so that the last round writes the
      // caller's arrays.
      int cur = rounds % 2;
      {
        KernelTimer timer("blocksort", st);
        ee = launch_blocksort<K>((const K *)keys, (const uint32_t *)vals, kb[cur], vb[cur], n, lb,
                                 st);
      }
      for (int lw = lb; ee == hipSuccess && ((int64_t)1 << lw) < n; ++lw) {
        KernelTimer timer("sort_round", st);
        if (cfg.mode == 1)
          ee = launch_sort_round_tiles<K>(tc, kb[cur], vb[cur], kb[cur ^ 1], vb[cur ^ 1], n, lw, st);
        else
          ee = launch_sort_round<K>(sc, kb[cur], vb[cur], kb[cur ^ 1], vb[cur ^ 1], n, lw, st);
        cur ^= 1;
      }
    });
    return ee;
  });
  if (e == hipErrorNotSupported)
    return fail(MP_ERR_UNSUPPORTED, "%s: configuration nt=%d vt=%d not compiled in", fn, cfg.nt, cfg.vt);
  return e == hipSuccess ? MP_OK : hip_fail(e, "mp_sort launch");
}

}  // extern "C"

// ---- autotuner ---------------------------------------------------------------
//
// Times every compiled persistent variant of an operation on the caller's
// inputs (HIP events on the caller's stream; one warm-up call, then the
// median of `reps` calls), installs the fastest with mp_set_config and
// returns it.  `setup`, when given, runs untimed before every call (the sort
// restores its unsorted input).

static const int kTuneShapes[][2] = {{192, 24}, {256, 16}, {256, 18}, {256, 14}, {256, 12},
                                     {256, 8},  {128, 16}, {512, 8},   {512, 16}};
// per-tile shapes (merge and sort)
static const int kTuneTileShapes[][2] = {{1024, 16}, {1024, 8}, {512, 16}, {512, 12},
                                         {256, 16},  {256, 8}};

template <typename Run, typename Setup>
static mp_status autotune(Op op, int reps, hipStream_t s, Run run, Setup setup, mp_config *best) {
  if (reps < 1 || reps > 1000) return fail(MP_ERR_INVALID_ARG, "autotune: reps must be in [1, 1000]");
  const mp_config saved = g_config[op];
  const bool saved_chosen = g_config_chosen[op];
  g_config_chosen[op] = true;  // candidates apply as set, built-in rules aside
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    g_config_chosen[op] = saved_chosen;
    return fail(MP_ERR_HIP, "autotune: event creation failed");
  }
  float best_ms = 0.f;
  bool have = false;
  mp_status st = MP_OK;
  // Median time of config c (negative: the variant is not compiled).
  auto time_config = [&](const mp_config &c) -> float {
    g_config[op] = c;
    std::vector<float> ts;
    for (int r = 0; r <= reps && st == MP_OK; ++r) {
      setup();
      if (hipEventRecord(e0, s) != hipSuccess) { st = fail(MP_ERR_HIP, "autotune: event"); break; }
      const mp_status rs = run();
      if (rs == MP_ERR_UNSUPPORTED) break;
      if (rs != MP_OK) { st = rs; break; }
      float ms = 0.f;
      if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
          hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
        st = fail(MP_ERR_HIP, "autotune: timing");
        break;
      }
      if (r > 0) ts.push_back(ms);
    }
    if (st != MP_OK || ts.empty()) return -1.f;
    std::sort(ts.begin(), ts.end());
    return ts[ts.size() / 2];
  };
  auto consider = [&](const mp_config &c, float ms) {
    if (ms >= 0.f && (!have || ms < best_ms)) {
      best_ms = ms;
      *best = c;
      have = true;
    }
  };
  const int cus = device_cu_count();
  {
    for (const auto &shape : kTuneTileShapes) {
      const mp_config c{1, shape[0], shape[1], 0, 0};
      if (op == kOpSort) {
        const int64_t t = (int64_t)c.nt * c.vt;
        if ((t & (t - 1)) != 0) continue;
      }
      consider(c, time_config(c));
      if (st != MP_OK) break;
    }
  }
  for (const auto &shape : kTuneShapes) {
    if (st != MP_OK) break;
    mp_config c{2, shape[0], shape[1], 0, 0};
    if (op == kOpSort) {
      const int64_t t = (int64_t)c.nt * c.vt;
      if ((t & (t - 1)) != 0 || t > (2 << kSortBlockMinLog2)) continue;
    }
    g_last_pairs_grid = 0;
    const float ms = time_config(c);
    if (st != MP_OK) break;
    consider(c, ms);
    // One workgroup fewer per compute unit than the occupancy query allows:
    // a persistent grid that does not fit at once leaves a second round of
    // workgroups running alone at the end.
    const int g0 = g_last_pairs_grid;
    if (ms >= 0.f && cus > 0 && g0 >= 2 * cus) {
      const mp_config c1{2, shape[0], shape[1], g0 - cus, 0};
      consider(c1, time_config(c1));
      if (st != MP_OK) break;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != MP_OK || !have) {
    g_config[op] = saved;
    g_config_chosen[op] = saved_chosen;
    return st != MP_OK ? st : fail(MP_ERR_UNSUPPORTED, "autotune: no variant ran");
  }
  g_config[op] = *best;
  return MP_OK;
}

extern "C" {

mp_status mp_autotune_merge(mp_dtype kt, mp_dtype vt, const void *Ak, const void *Av,
                            int64_t na, const void *Bk, const void *Bv, int64_t nb, void *Sk,
                            void *Sv, int reps, mp_config *best, void *stream) {
  if (!best) return fail(MP_ERR_INVALID_ARG, "mp_autotune_merge: NULL result");
  auto run = [&]() {
    return vt == MP_NONE ? mp_merge(kt, Ak, na, Bk, nb, Sk, stream)
                         : mp_merge_kv(kt, vt, Ak, Av, na, Bk, Bv, nb, Sk, Sv, stream);
  };
  return autotune(kOpMerge, reps, (hipStream_t)stream, run, [] {}, best);
}

mp_status mp_autotune_batched(mp_dtype kt, const void *A, const int64_t *a_off, const void *B,
                              const int64_t *b_off, int64_t n_pairs, int64_t total_a,
                              int64_t total_b, void *S, int reps, mp_config *best, void *stream) {
  if (!best) return fail(MP_ERR_INVALID_ARG, "mp_autotune_batched: NULL result");
  // the per-tile candidates need a workspace: one for the whole tuning run
  // (a set-up call, not the merge itself)
  const size_t need = mp_merge_batched_workspace_bytes(kt, n_pairs, total_a + total_b);
  void *ws = nullptr;
  if (need > 0) {
    const hipError_t e = hipMalloc(&ws, need);
    if (e != hipSuccess) return hip_fail(e, "mp_autotune_batched: workspace");
  }
  auto run = [&]() {
    return mp_merge_batched(kt, A, a_off, B, b_off, n_pairs, total_a, total_b, S, ws, need,
                            stream);
  };
  const mp_status st = autotune(kOpBatched, reps, (hipStream_t)stream, run, [] {}, best);
  if (ws) {
    (void)hipStreamSynchronize((hipStream_t)stream);
    (void)hipFree(ws);
  }
  return st;
}

mp_status mp_autotune_sort(mp_dtype kt, mp_dtype vt, const void *keys_in, const void *vals_in,
                           void *keys, void *vals, int64_t n, void *ws, size_t ws_bytes, int reps,
                           mp_config *best, void *stream) {
  if (!best) return fail(MP_ERR_INVALID_ARG, "mp_autotune_sort: NULL result");
  const size_t es = dtype_size(kt);
  if (es == 0 || n < 0 || (n > 0 && (!keys_in || !keys)) || (vt != MP_NONE && n > 0 && (!vals_in || !vals)))
    return fail(MP_ERR_INVALID_ARG, "mp_autotune_sort: bad arguments");
  if (overlaps(span(keys_in, n, es), span(keys, n, es)))
    return fail(MP_ERR_OVERLAP, "mp_autotune_sort: source and work keys overlap");
  hipStream_t s = (hipStream_t)stream;
  hipError_t copy_err = hipSuccess;
  auto setup = [&]() {
    if (copy_err == hipSuccess && n > 0)
      copy_err = hipMemcpyAsync(keys, keys_in, (size_t)n * es, hipMemcpyDeviceToDevice, s);
    if (copy_err == hipSuccess && n > 0 && vt != MP_NONE)
      copy_err = hipMemcpyAsync(vals, vals_in, (size_t)n * 4, hipMemcpyDeviceToDevice, s);
  };
  auto run = [&]() {
    if (copy_err != hipSuccess) return hip_fail(copy_err, "mp_autotune_sort: restoring input");
    return mp_sort(kt, vt, keys, vals, n, ws, ws_bytes, stream);
  };
  return autotune(kOpSort, reps, s, run, setup, best);
}

mp_status mp_partition_lanes(int32_t lanes) {
  if (lanes < 0 || lanes > 64 || (lanes & (lanes - 1)) != 0)
    return fail(MP_ERR_INVALID_ARG, "mp_partition_lanes: lanes must be 0 or a power of two <= 64");
  g_partition_lanes = lanes;
  return MP_OK;
}

mp_status mp_get_config(const char *op, mp_config *cfg) {
  const int i = op_index(op);
  if (i < 0 || !cfg) return fail(MP_ERR_INVALID_ARG, "mp_get_config: unknown operation or NULL");
  *cfg = g_config[i];
  return MP_OK;
}

}  // extern "C"
