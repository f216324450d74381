// Host-side internal interface between the C ABI layer and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <functional>
#include <vector>

#include "mergepath.h"

namespace mp {

// Calls f(K{}) with a value of the key type named by kt; returns false for
// an unknown dtype.
template <typename F>
bool dispatch_key(mp_dtype kt, F &&f) {
  switch (kt) {
    case MP_U32: f(uint32_t{}); return true;
    case MP_I32: f(int32_t{}); return true;
    case MP_U64: f(uint64_t{}); return true;
    case MP_F32: f(float{}); return true;
    default: return false;
  }
}

inline size_t dtype_size(mp_dtype t) {
  switch (t) {
    case MP_U32: case MP_I32: case MP_F32: return 4;
    case MP_U64: return 8;
    default: return 0;
  }
}

// Tile geometry of the per-tile merge: NT lanes x VT outputs per lane.
struct TileCfg {
  int nt;
  int vt;
};

// Lanes that search one diagonal together: g_partition_lanes when set (a
// power of two, 1..64), else chosen from the number of diagonals so that
// small launches still fill the device.
extern int g_partition_lanes;
int partition_lanes(int64_t n_diag);

// Grid-level split search on explicit diagonals (diag != nullptr) or on the
// equispaced diagonals k * tile clamped to na + nb (diag == nullptr).
template <typename K>
hipError_t launch_partition(const K *A, int64_t na, const K *B, int64_t nb,
                            const int64_t *diag, int64_t tile, int64_t n_diag,
                            int64_t *a_split, hipStream_t s);

// Per-tile merge (Algorithm 1) of T = nt * vt outputs per workgroup: the
// splits of every tile boundary are found first and handed to each tile in
// the first 32 bytes of its own range of S, then one workgroup per tile
// merges its pair.  Av/Bv/Sv may be null (keys only).  hipErrorNotSupported
// for a shape that is not built for the key type.
template <typename K>
hipError_t launch_merge_tiles(TileCfg cfg, const K *A, const uint32_t *Av,
                              int64_t na, const K *B, const uint32_t *Bv,
                              int64_t nb, K *S, uint32_t *Sv, hipStream_t s);

// The tile merge on the caller's splits of the tile diagonals (keys only).
template <typename K>
hipError_t launch_merge_tiles_split(TileCfg cfg, const K *A, int64_t na, const K *B,
                                    int64_t nb, K *S, const int64_t *a_split, hipStream_t s);

// One merge-sort round through the per-tile merge: runs of width 2^lw in X
// merged pairwise into Y; the tile (a power of two) must divide 2^(lw+1).
template <typename K>
hipError_t launch_sort_round_tiles(TileCfg cfg, const K *X, const uint32_t *Xv, K *Y,
                                   uint32_t *Yv, int64_t n, int lw, hipStream_t s);

// Batch of independent pairs through the per-tile merge, merged as one merge
// of the concatenated inputs in (pair, key) order (keys only; tiles of at
// least kBatchMinTile outputs).  ws: batch_tile_ws_bytes(total) bytes,
// 8-byte aligned: the splits of the tile boundaries (int64 each) and the pair
// holding each tile's first output (int32 each).
constexpr int64_t kBatchMinTile = 2048;
inline int64_t batch_tile_ws_bytes(int64_t total) {
  const int64_t tiles = (total + kBatchMinTile - 1) / kBatchMinTile;
  return 8 * (tiles + 1) + 4 * tiles;
}
template <typename K>
hipError_t launch_merge_batched_tiles(TileCfg cfg, const K *A, const int64_t *a_off, const K *B,
                                      const int64_t *b_off, int64_t n_pairs, int64_t total_a,
                                      int64_t total_b, K *S, void *ws, hipStream_t s);

// Built-in per-tile shape for n outputs of a key size, with or without
// values: the largest tile that still gives every compute unit a few tiles.
TileCfg auto_tile_cfg(size_t key_bytes, bool kv, int64_t n);

// Persistent merge: nt lanes x vt outputs per tile, `grid` workgroups each
// walking a contiguous run of tiles (0 = one full wave of resident groups).
struct StreamCfg {
  int nt;
  int vt;
  int grid;
  int margin;  // window margin: 0 = adaptive (prediction, then lookahead probes),
               // > 0 = prediction with this margin only, < 0 = full windows
};

template <typename K>
hipError_t launch_merge_stream(StreamCfg cfg, const K *A, const uint32_t *Av,
                               int64_t na, const K *B, const uint32_t *Bv,
                               int64_t nb, K *S, uint32_t *Sv, hipStream_t s);

// Persistent merge that stores nothing: adds sum of S[i] * (i + 1) (keys as
// unsigned bits, modulo 2^64) to *checksum.  Tiles 192 x 24 or 256 x 16.
template <typename K>
hipError_t launch_merge_checksum(StreamCfg cfg, const K *A, int64_t na, const K *B, int64_t nb,
                                 unsigned long long *checksum, hipStream_t s);

// Multiset operation (0 intersection, 1 union, 2 difference, 3 symmetric
// difference) of sorted A and B into S (cap slots; no store beyond them);
// *count (device) receives the output length.  ws: 3 * (setop_tiles(na + nb)
// + 1) int64 of device workspace (setop_tiles bounds the tile count of every
// key type).
int64_t setop_tiles(int64_t n);
// The allocation-free variant's fixed scratch: kSetScratchWords int64 per
// device (4 MiB), enough for na + nb up to kSetScratchKeys.
constexpr int64_t kSetScratchWords = (int64_t)1 << 19;
constexpr int64_t kSetScratchKeys = (kSetScratchWords / 3 - 1) * (512 * 12);
// Device address of this device's scratch (looked up once per device).
hipError_t setop_scratch_ptr(int64_t **out);
template <typename K>
hipError_t launch_set_op(int op, const K *A, int64_t na, const K *B, int64_t nb, K *S,
                         int64_t cap, int64_t *count, int64_t *ws, hipStream_t s);

// Inner join of sorted A and B: every (i, j) with A[i] == B[j], ordered by
// i then j; the first cap pairs go to I and J, the total to *count (device).
// ws: join_ws_bytes(na, nb) bytes, 8-byte aligned.
int64_t join_ws_bytes(int64_t na, int64_t nb);
template <typename K>
hipError_t launch_join(const K *A, int64_t na, const K *B, int64_t nb, int64_t *I, int64_t *J,
                       int64_t cap, int64_t *count, int64_t *ws, hipStream_t s);

// Batched merge of CSR-concatenated pairs (persistent, one launch).
template <typename K>
hipError_t launch_merge_batched(StreamCfg cfg, const K *A, const int64_t *a_off,
                                const K *B, const int64_t *b_off, int64_t n_pairs,
                                int64_t total_a, int64_t total_b, K *S, hipStream_t s);

// One merge-sort round: runs of width 2^lw in X merged pairwise into Y.
template <typename K>
hipError_t launch_sort_round(StreamCfg cfg, const K *X, const uint32_t *Xv, K *Y,
                             uint32_t *Yv, int64_t n, int lw, hipStream_t s);

// Stable sort of each block of 2^log2_block keys (in place allowed:
// in == out).  One workgroup of 2^log2_block / 16 lanes per block;
// log2_block is kSortBlockMinLog2 .. kSortBlockMaxLog2.
constexpr int kSortBlockMinLog2 = 12;
constexpr int kSortBlockMaxLog2 = 14;
// Block size the sort uses for a key size, with or without 32-bit values.
int sort_block_log2(size_t key_bytes, bool kv);
template <typename K>
hipError_t launch_blocksort(const K *in, const uint32_t *vin, K *out, uint32_t *vout,
                            int64_t n, int log2_block, hipStream_t s);

// Plain 16-byte streaming copy (bandwidth reference).
hipError_t launch_copy(const void *src, void *dst, int64_t n_bytes, int unroll,
                       int grid, hipStream_t s);
// Bandwidth probes: kind 0 copy, 1 read only (per-wavefront XOR to dst,
// grid * 4 vectors), 2 write only (to dst).
hipError_t launch_bw_probe(int kind, const void *src, void *dst, int64_t n_bytes, int unroll,
                           int grid, hipStream_t s);

// Number of compute units of the current device (cached per device).
int device_cu_count();

// Workgroup count the last persistent merge launch chose before clipping to
// its tile count (the autotuner derives grid candidates from it).
extern int g_last_pairs_grid;

// Brackets one kernel launch with HIP events on its stream while timing is
// enabled (mp_timing_enable); does nothing otherwise.
class KernelTimer {
 public:
  KernelTimer(const char *name, hipStream_t s);
  ~KernelTimer();

 private:
  const char *name_;
  hipStream_t s_;
  hipEvent_t start_ = nullptr;
};

// Graph mode (mp_graph_enable): issue(stream) is recorded once per key into a
// hipGraph and replayed on s; otherwise issue(s) runs directly.
bool graph_mode();
hipError_t run_maybe_graph(std::vector<uint64_t> key, hipStream_t s,
                           const std::function<hipError_t(hipStream_t)> &issue);

// Record the message returned by mp_last_error() (this thread) and return st.
mp_status set_error(mp_status st, const char *fmt, ...);

// Device counters [tiles, window reloads, workgroups] of the persistent kernels while
// timing is enabled, nullptr otherwise.
unsigned long long *stats_device_ptr();


}  // namespace mp
