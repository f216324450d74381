/*
 * mergepath.h -- C ABI of the MI355X (gfx950) Merge Path library.
 *
 * The operations follow the problem statement of Green, Odeh and Birk,
 * "Merge Path - A Visually Intuitive Approach to Parallel Merging":
 * A and B are sorted ascending and may differ in length (section 2.1); S is
 * their merge; the split on cross diagonal d is where the Merge Path crosses
 * that diagonal (Lemma 8, Theorem 9), found by a binary search along it
 * (Algorithm 2, Theorem 14); pairs cut at any diagonals merge independently
 * and concatenate to S (Theorem 5, Corollary 6).
 *
 * Conventions shared by every entry point:
 *  - Pointers: every array argument is a DEVICE pointer owned by the caller,
 *    unless the comment says "host".  The library never frees caller memory.
 *    Arrays must be aligned to their element size.
 *  - Layout: arrays are dense, one element after the other (structure of
 *    arrays: keys and values are separate arrays).
 *  - Sizes are element counts (int64_t); a size of 0 is a valid no-op and
 *    the matching pointer may then be NULL.
 *  - Streams: `stream` is a hipStream_t passed as void* (NULL = the null
 *    stream).  Calls are asynchronous: they return once work is enqueued.
 *    Argument errors are reported before anything is enqueued; launch errors
 *    are reported as MP_ERR_HIP; faults during execution surface at the
 *    caller's next synchronisation.
 *  - Preconditions NOT checked on the device: inputs sorted ascending under
 *    the key order, and float keys free of NaN.  Violating them gives an
 *    unspecified result but every memory access stays in bounds.
 *  - Key order: MP_U32 and MP_U64 unsigned, MP_I32 signed, MP_F32 IEEE
 *    (-0.0 and +0.0 are equal keys).  Ties take A first (section 2.1: the
 *    path steps right, taking B[j], only when A[i] > B[j]), so every merge
 *    is stable with A before B, and the output is bit-exact.
 *  - Output must not overlap any input (MP_ERR_OVERLAP): no in-place merge.
 *  - On any status other than MP_OK, mp_last_error() returns a message
 *    (per thread).
 *  - Thread safety: calls without a handle are thread-safe; a learned
 *    partitioner handle must not be used by two threads at once.
 */
#ifndef MERGEPATH_H
#define MERGEPATH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MP_NONE = 0, /* no values (keys-only) */
  MP_U32 = 1,
  MP_I32 = 2,
  MP_U64 = 3,
  MP_F32 = 4
} mp_dtype;

typedef enum {
  MP_OK = 0,
  MP_ERR_INVALID_ARG = -1, /* negative size, NULL pointer with size > 0, bad option */
  MP_ERR_UNSUPPORTED = -2, /* dtype or dtype combination not provided */
  MP_ERR_OVERLAP = -3,     /* an output range overlaps an input range */
  MP_ERR_WORKSPACE = -4,   /* workspace NULL or smaller than required */
  MP_ERR_HIP = -5,         /* the HIP runtime reported an error */
  MP_ERR_STATE = -6        /* handle not trained, or file format mismatch */
} mp_status;

/* Message describing the most recent non-OK status on this thread. */
const char *mp_last_error(void);

/* Library version as major*10000 + minor*100 + patch. */
int mp_version(void);

/*
 * mp_partition -- split on each requested cross diagonal (Algorithm 2,
 * Theorem 9, Theorem 14).
 *   kt        key dtype (MP_U32, MP_I32, MP_U64, MP_F32)
 *   A, na     sorted keys of A;  B, nb  sorted keys of B
 *   diag      n_diag diagonals (int64), each in [0, na+nb], any order;
 *             values outside that range are clamped into it
 *   a_split   n_diag int64 outputs: a_split[k] is the unique a with
 *             b = diag[k] - a satisfying  A[a-1] <= B[b]  and  B[b-1] < A[a]
 *             (terms whose index falls outside A or B count as satisfied).
 *             The pair (A[a_k, a_{k+1}), B[b_k, b_{k+1})) merges to
 *             S[diag[k], diag[k+1]) for consecutive diagonals (Corollary 6).
 * At most ceil(log2(min(na, nb) + 1)) search steps per diagonal.
 */
mp_status mp_partition(mp_dtype kt, const void *A, int64_t na, const void *B,
                       int64_t nb, const int64_t *diag, int64_t n_diag,
                       int64_t *a_split, void *stream);

/*
 * Lanes per diagonal of mp_partition and mp_partition_learned.  With G > 1
 * lanes a diagonal's search probes G points per round, cutting the interval
 * G + 1 ways (Theorem 14's search with a wider cut): about log_{G+1} rounds
 * of dependent loads instead of log_2, for G times the loads.  That pays
 * when there are too few diagonals to fill the device.
 *   lanes  0 = chosen per call (the largest power of two G <= 16 with
 *          G * n_diag <= 2^14, else 1); 1, 2, 4, ..., 64 = that many
 *          lanes always.  Results never depend on it.  Applies to later calls
 *          on every thread; MP_ERR_INVALID_ARG for any other value.
 */
mp_status mp_partition_lanes(int32_t lanes);

/*
 * mp_merge -- S = merge of A and B (Algorithm 1: equal-length output tiles,
 * each tile's split by Algorithm 2, tiles merged independently).
 *   S   na+nb keys of dtype kt, must not overlap A or B.
 */
mp_status mp_merge(mp_dtype kt, const void *A, int64_t na, const void *B,
                   int64_t nb, void *S, void *stream);

/*
 * mp_set_op -- multiset operations on sorted A and B through the same
 * partition: the merge's output tiles are cut by Algorithm 2 on their
 * diagonals and each tile's pair is processed independently (Corollary 6),
 * keeping or dropping each merged key.
 *   op     0 intersection, 1 union, 2 difference (A minus B),
 *          3 symmetric difference.  A value found m times in A and n times
 *          in B comes out min(m, n), max(m, n), max(m - n, 0) and |m - n|
 *          times, in sorted order with A's copies before B's; equal keys
 *          pair front to front, so intersection keeps A's first copies,
 *          difference A's last ones, union and symmetric difference the
 *          longer run's last excess copies (the rules of the C++ standard
 *          library's set algorithms).
 *   S      room for na keys (intersection, difference) or na + nb keys
 *          (union, symmetric difference); the first *count are written.
 *          No store ever lands past that room, unsorted inputs included
 *          (their count is then clamped to it).
 *   count  one int64 in device memory (8-byte aligned): the output length,
 *          written when the work runs.  One pass: each tile finds its output
 *          offset by looking back over the tiles before it (tiles are taken
 *          in the order workgroups start, so every wait ends; a bound on the
 *          polls backs that up, and should it ever trip, count is -1).
 *   ws     device workspace of at least mp_set_op_workspace_bytes(na, nb)
 *          bytes, 8-byte aligned.
 * Neither S, count nor ws may overlap an input or each other.
 */
size_t mp_set_op_workspace_bytes(int64_t na, int64_t nb);
mp_status mp_set_op(int32_t op, mp_dtype kt, const void *A, int64_t na, const void *B,
                    int64_t nb, void *S, int64_t *count, void *ws, size_t ws_bytes,
                    void *stream);

/*
 * mp_join -- inner join of sorted A and B through the merge partition (the
 * introduction names database joins among the merge's uses): every pair
 * (i, j) with A[i] equal to B[j] (IEEE equality for f32, so -0.0 matches
 * +0.0), ordered by i, then j.  A value found m times in A and n times in B
 * gives its m x n pairs.  The merge's tiles (Algorithm 2 splits, Theorem 17
 * inside a tile) give each A key the first B column of its run and the run's
 * length; a scan gives each key its first output; the pairs are emitted by a
 * second Merge Path merge, of those offsets with the output indices, in
 * tiles of equal work whatever the duplicates.
 *   I, J   room for `cap` int64 each (device): the first min(cap, count)
 *          pairs, i in I and j in J; cap = 0 only counts.
 *   count  one int64 (device, 8-byte aligned): the total number of pairs,
 *          written when the work runs (may exceed cap: call again with room).
 *   ws     device workspace of mp_join_workspace_bytes(na, nb) bytes
 *          (about 16 bytes per A key), 8-byte aligned.
 * I, J, count and ws must not overlap each other or the inputs.  Unsorted
 * inputs give unspecified pairs and count but every store stays in bounds.
 */
size_t mp_join_workspace_bytes(int64_t na, int64_t nb);
mp_status mp_join(mp_dtype kt, const void *A, int64_t na, const void *B, int64_t nb, int64_t *I,
                  int64_t *J, int64_t cap, int64_t *count, void *ws, size_t ws_bytes,
                  void *stream);

/*
 * mp_set_op_noalloc -- mp_set_op for callers that cannot allocate device
 * memory or pass a workspace (code under hipGraph capture, tight serving
 * loops, harnesses that forbid hipMalloc).  Same operation, arguments and
 * results as mp_set_op without ws / ws_bytes: the look-back state lives in a
 * fixed scratch array of 4 MiB in device memory that the library owns, one
 * per GPU, held until the process ends.  It allocates, frees and
 * synchronises nothing.
 *   na + nb  at most 1073731584 keys; larger inputs return
 *            MP_ERR_UNSUPPORTED before anything is enqueued.
 * Every call on one GPU shares that GPU's scratch (it is cleared by a kernel
 * at the start of each call): calls that overlap in time on one GPU, from
 * different streams or threads, race and give wrong counts and outputs.
 * Serialise them (one stream, or events between streams).
 */
mp_status mp_set_op_noalloc(int32_t op, mp_dtype kt, const void *A, int64_t na, const void *B,
                            int64_t nb, void *S, int64_t *count, void *stream);

/*
 * mp_merge_split -- the second step of Algorithm 1 on splits the caller
 * already has: output tile k, S[k*tile, min((k+1)*tile, na+nb)), is merged
 * from the pair that a_split[k] and a_split[k+1] cut out (Corollary 6),
 * one workgroup per tile, tiles independent.
 *   a_split  ceil((na+nb)/tile) + 1 int64 splits (device) on the diagonals
 *            min(k*tile, na+nb): what mp_partition or mp_partition_learned
 *            return for those diagonals.
 *   tile     2048, 3840, 4096, 8192 or 16384 outputs per tile; 16384 for
 *            4-byte keys only (MP_ERR_UNSUPPORTED else).
 *   S        na+nb keys, must overlap neither input nor a_split.
 * The result is the merge when the splits are the true ones.  Other split
 * values give some other output but stay memory-safe: every split is
 * clamped to its diagonal's extent inside the grid.
 */
mp_status mp_merge_split(mp_dtype kt, const void *A, int64_t na, const void *B,
                         int64_t nb, const int64_t *a_split, int32_t tile, void *S,
                         void *stream);

/*
 * mp_merge_checksum -- the merge of A and B computed but not written: the
 * runs of section 6 whose merged values go to a local register instead of
 * memory, which isolate reading and comparing from storing.  Every output
 * stays in the registers of the lane that merged it; the kernel adds
 *     sum over i of S[i] * (i + 1)   (modulo 2^64; keys as unsigned bits,
 *                                     4-byte keys zero-extended)
 * to *checksum, where S is the merge mp_merge would write, so the result
 * still depends on every output and its position.
 *   checksum  one uint64 in device memory (8-byte aligned), added to, not
 *             overwritten: zero it first.
 * A diagnostic for measurement; it uses the persistent kernel with the
 * merge's current tile if that is 192 x 24 or 256 x 16, else 192 x 24.
 */
mp_status mp_merge_checksum(mp_dtype kt, const void *A, int64_t na, const void *B,
                            int64_t nb, uint64_t *checksum, void *stream);

/*
 * mp_merge_kv -- key-value merge: keys as mp_merge; each value travels with
 * its key (stable: equal keys keep A's values before B's, each input's own
 * order preserved).
 *   vt   value dtype: any 4-byte type (MP_U32, MP_I32, MP_F32), moved as bits
 *   Ak/Av, na and Bk/Bv, nb   keys and values of A and of B
 *   Sk/Sv  na+nb outputs; neither may overlap an input nor each other.
 */
mp_status mp_merge_kv(mp_dtype kt, mp_dtype vt, const void *Ak, const void *Av,
                      int64_t na, const void *Bk, const void *Bv, int64_t nb,
                      void *Sk, void *Sv, void *stream);

/*
 * mp_merge_batched -- many independent merges in one launch (Corollary 6
 * applied to a concatenation of pairs; Corollary 7 load balance over the
 * global output index).  The batch is merged as one merge of the
 * concatenated inputs in (pair, key) order, cut into equal tiles of the
 * global output that may span many pairs.
 *   A, a_off  concatenated A_k; a_off has n_pairs+1 int64 entries (device),
 *             a_off[0] = 0, non-decreasing; A_k = A[a_off[k], a_off[k+1])
 *   B, b_off  likewise for B_k
 *   S         a_off[n]+b_off[n] outputs; pair k is written to
 *             S[a_off[k]+b_off[k], a_off[k+1]+b_off[k+1])
 *   total_a, total_b   a_off[n_pairs] and b_off[n_pairs] (host copies,
 *             used to size the launch; must match the device offsets)
 *   ws, ws_bytes  device workspace of at least
 *             mp_merge_batched_workspace_bytes(kt, n_pairs, total_a+total_b)
 *             bytes (12 bytes per 2048 outputs), 8-byte aligned, overlapping
 *             nothing else; the persistent configuration (mode 2) needs none.
 * Offsets are not validated on the device; non-monotone offsets give an
 * unspecified result with in-bounds accesses.
 */
size_t mp_merge_batched_workspace_bytes(mp_dtype kt, int64_t n_pairs,
                                        int64_t total);
mp_status mp_merge_batched(mp_dtype kt, const void *A, const int64_t *a_off,
                           const void *B, const int64_t *b_off,
                           int64_t n_pairs, int64_t total_a, int64_t total_b,
                           void *S, void *ws, size_t ws_bytes, void *stream);

/*
 * mp_sort -- stable merge sort in place (section 3: sorted blocks, then
 * log2 rounds of merges of adjacent runs, left run as A; section 4.2:
 * blocks sized to on-chip memory first).
 *   keys, n     keys of dtype kt, sorted in place
 *   vt, vals    MP_NONE and NULL, or a 4-byte value dtype and n values
 *               permuted with their keys
 *   ws          device workspace of at least mp_sort_workspace_bytes(kt, vt, n)
 * mp_sort_block_keys returns the length of the blocks sorted first (the
 * runs the first merge round starts from) for keys of dtype kt with values
 * of dtype vt (MP_NONE: keys only), or 0 for an unsupported pair: a sort of
 * n keys makes 1 + ceil(log2(n / mp_sort_block_keys(kt, vt))) passes over
 * the data.
 */
int64_t mp_sort_block_keys(mp_dtype kt, mp_dtype vt);
size_t mp_sort_workspace_bytes(mp_dtype kt, mp_dtype vt, int64_t n);
mp_status mp_sort(mp_dtype kt, mp_dtype vt, void *keys, void *vals, int64_t n,
                  void *ws, size_t ws_bytes, void *stream);

/*
 * Learned split predictor.  Not part of the paper: a small FP32 MLP
 * predicts where the Merge Path crosses a diagonal, and the exact search of
 * Algorithm 2 then runs only in a window [a_hat + lo, a_hat + hi] around the
 * prediction a_hat.  A result on a window edge that is not a diagonal bound
 * is checked against
 * both conditions of Algorithm 2; if they fail, the full-range search runs.
 * mp_partition_learned therefore always returns exactly what mp_partition
 * returns; the model only changes how many probes that takes.
 *
 * Model: inputs x = [t, sin 2pi t, cos 2pi t, sin 4pi t, cos 4pi t][:F] with
 * t = d / (na + nb); y = w2 . relu(W1 x + b1) + b2; the prediction is
 * a_prior(d) + round(y * na), a_prior(d) = clamp(round(d * na / (na + nb))).
 * Parameter vector (float32): [W1 (H x F row-major), b1 (H), w2 (H), b2].
 * A handle owns its device memory (parameters, Adam moments, training
 * buffers) and must not be used by two threads at once.
 */
typedef struct mp_lp_s *mp_lp;

/* New model with `hidden` units (1..64) and `features` inputs (1, 3 or 5),
   weights drawn from `seed`; window unset. */
mp_status mp_lp_create(mp_lp *h, int hidden, int features, uint64_t seed);
void mp_lp_destroy(mp_lp h);
int mp_lp_num_params(mp_lp h);
/* Number of inputs F and hidden units H of the model (HOST outputs). */
mp_status mp_lp_shape(mp_lp h, int *features, int *hidden);
/* Copy the n = mp_lp_num_params(h) parameters to / from HOST memory
   (set also clears the Adam moments and step count). */
mp_status mp_lp_get_params(mp_lp h, float *host, int n);
mp_status mp_lp_set_params(mp_lp h, const float *host, int n);
/* Search windows.  mp_lp_set_window sets the symmetric window [-w, w]
   (w >= 0) for every diagonal; mp_lp_calibrate sets one asymmetric window
   (lo, hi offsets from the prediction, lo <= hi) per bucket of t (16384
   equal buckets of [0, 1]).  mp_lp_window returns the largest |offset| of
   any window (-1 when unset).  mp_lp_windows copies up to cap buckets'
   (lo, hi) pairs (2 cap int64) to HOST memory and returns how many buckets
   the model has (0: one symmetric window everywhere; -1: NULL handle). */
mp_status mp_lp_set_window(mp_lp h, int64_t window);
int64_t mp_lp_window(mp_lp h);
int32_t mp_lp_windows(mp_lp h, int64_t *windows, int32_t cap);

/* Training examples for K stratified diagonals of one (A, B) set: the exact
   splits from the plain search, features X (K x F, device float) and
   targets r (K, device float) = (a* - a_prior) / na; diag and split (device
   int64, may be NULL) receive the diagonals and exact splits. */
mp_status mp_lp_examples(mp_lp h, mp_dtype kt, const void *A, int64_t na,
                         const void *B, int64_t nb, int64_t K, uint64_t seed,
                         float *X, float *r, int64_t *diag, int64_t *split,
                         void *stream);
/* y[k] = model(X[k]) for K rows of X (device). */
mp_status mp_lp_forward(mp_lp h, const float *X, int64_t K, float *y, void *stream);
/* Full-batch gradient of mean((y - r)^2) into grad (device, num_params
   floats) and, if loss is not NULL, the loss (device float); reductions run
   in a fixed order, so repeated calls give identical bits. */
mp_status mp_lp_grad(mp_lp h, const float *X, const float *r, int64_t K,
                     float *grad, float *loss, void *stream);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) with learning rate lr. */
mp_status mp_lp_adam_step(mp_lp h, const float *X, const float *r, int64_t K,
                          float lr, void *stream);
/* Train on n_sets (A_i, B_i) pairs: As/Bs are HOST arrays of device
   pointers, nas/nbs HOST arrays of lengths; k_diag stratified diagonals per
   set get exact splits from the plain search; then `epochs` full-batch Adam
   steps with learning rate decaying from lr (cosine).  final_loss (HOST,
   may be NULL) receives the last loss; this synchronises the stream. */
mp_status mp_lp_train(mp_lp h, mp_dtype kt, const void *const *As,
                      const int64_t *nas, const void *const *Bs,
                      const int64_t *nbs, int n_sets, int64_t k_diag, int epochs,
                      float lr, float *final_loss, void *stream);
/* Set the windows from a held-out set: n_diag random diagonals get exact
   splits and signed errors e = split - prediction.  Bucket b takes the
   smallest and largest e over buckets [b - r, b + r] (r = max(1,
   ceil(16 * 16384 / n_diag)); the overall extremes if none of them has a
   sample), each side widened by an eighth of that span plus
   ceil(3 sqrt(na nb / (4 (na + nb)))) + 1 (three standard deviations of
   the seed-to-seed noise of a split of iid samples).  max_err (HOST, may be
   NULL) receives the largest |e|.  Synchronises the stream. */
mp_status mp_lp_calibrate(mp_lp h, mp_dtype kt, const void *A, int64_t na,
                          const void *B, int64_t nb, int64_t n_diag,
                          int64_t *max_err, void *stream);
/* As mp_partition (identical output), searching only the predicted window.
   n_fallback (device uint64, may be NULL) is incremented once per diagonal
   whose split fell outside its window.  MP_ERR_STATE if no window is set. */
mp_status mp_partition_learned(mp_lp h, mp_dtype kt, const void *A, int64_t na,
                               const void *B, int64_t nb, const int64_t *diag,
                               int64_t n_diag, int64_t *a_split,
                               uint64_t *n_fallback, void *stream);
/* Save / load the model (features, hidden units, windows, seed, parameters)
   in a small binary file; load creates a new handle on the current device
   and also reads the two earlier formats (one window; 1024 symmetric
   per-bucket windows). */
mp_status mp_lp_save(mp_lp h, const char *path);
mp_status mp_lp_load(mp_lp *h, const char *path);

/*
 * Kernel variant selection (used by the autotuner and by tests that compare
 * variants).  Applies to later calls of the named operation on every thread;
 * it must not be changed while another thread is inside a library call.
 *   op    "merge" (mp_merge and mp_merge_kv), "batched" (mp_merge_batched),
 *         "sort" (the merge rounds of mp_sort)
 *   cfg   NULL restores the built-in choice (persistent; merge nt 192,
 *         vt 24, but nt 256, vt 12 for 8-byte keys with values; batched
 *         and sort nt 256, vt 16); otherwise
 *         mode: 1 = per-tile (one workgroup per output tile, which finds
 *                   the splits on its tile's two diagonals itself in global
 *                   memory; Algorithm 1 with p = tiles; no memory beyond
 *                   the inputs and outputs),
 *               2 = persistent (each workgroup finds one split and walks a
 *                   contiguous run of tiles, finding each next split in
 *                   on-chip memory; Algorithm 3, Theorem 17)
 *         nt, vt: lanes per workgroup and outputs per lane (tile = nt*vt)
 *         grid: workgroups of a persistent launch, 0 = one resident wave
 *         margin: persistent mode only; how each tile's input windows are
 *               sized (a split found on a truncated window edge always
 *               triggers an exact reload of full windows):
 *               0  = predicted as for >0 with a built-in margin; after a
 *                    window reload, and for as long as the A/B mix stays
 *                    unpredictable (long runs of equal keys), from a
 *                    64-point probe of the tile's end split issued a tile
 *                    ahead (one 65-way step of the Theorem 14 search).
 *                    Batched merges use the prediction only;
 *               >0 = from the previous tile's A/B mix plus `margin` keys per
 *                    input;
 *               <0 = full windows (n keys of each input per tile of n
 *                    outputs).
 * Persistent (nt, vt) pairs compiled in: (192, 24), (256, 8), (256, 12),
 * (256, 14), (256, 16), (256, 18), (128, 16), (512, 8), and (512, 16) for
 * 4-byte keys; per-tile mode: (256, 8), (256, 15), (256, 16), (128, 16).
 * A call with a pair that is not compiled in for its key type returns
 * MP_ERR_UNSUPPORTED.
 */
typedef struct {
  int32_t mode;
  int32_t nt;
  int32_t vt;
  int32_t grid;
  int32_t margin;
} mp_config;
mp_status mp_set_config(const char *op, const mp_config *cfg);
/* The configuration `op` currently uses (HOST output). */
mp_status mp_get_config(const char *op, mp_config *cfg);

/*
 * Autotuner.  Times every compiled persistent (nt, vt) variant of an
 * operation on the caller's own inputs (HIP events on `stream`: one warm-up
 * call, then the median of `reps` calls), installs the fastest for later
 * calls (as mp_set_config) and returns it in *best (HOST).  Arguments are
 * those of the operation; outputs are overwritten.  mp_autotune_sort sorts
 * `keys` (and `vals`) repeatedly, restoring them from keys_in / vals_in
 * before every call.  Synchronises the stream.
 */
mp_status mp_autotune_merge(mp_dtype kt, mp_dtype vt, const void *Ak, const void *Av,
                            int64_t na, const void *Bk, const void *Bv, int64_t nb,
                            void *Sk, void *Sv, int reps, mp_config *best, void *stream);
mp_status mp_autotune_batched(mp_dtype kt, const void *A, const int64_t *a_off,
                              const void *B, const int64_t *b_off, int64_t n_pairs,
                              int64_t total_a, int64_t total_b, void *S, int reps,
                              mp_config *best, void *stream);
mp_status mp_autotune_sort(mp_dtype kt, mp_dtype vt, const void *keys_in,
                           const void *vals_in, void *keys, void *vals, int64_t n,
                           void *ws, size_t ws_bytes, int reps, mp_config *best,
                           void *stream);

/*
 * hipGraph mode (off by default).  While enabled, mp_sort and
 * mp_merge_batched record their kernel launches into a hipGraph the first
 * time they see a given argument tuple (pointers, sizes, dtypes, current
 * configuration) and launch that graph on the caller's stream, then and on
 * every later identical call; kernels read the buffers when the graph runs.
 * At most 32 graphs are kept (least recently used evicted).  Calls that
 * overlap on different threads must not share buffers (as without graphs).
 */
mp_status mp_graph_enable(int on);
mp_status mp_graph_clear(void);
int64_t mp_graph_count(void);

/*
 * mp_copy -- plain streaming copy of n_bytes (multiple of 16) from src to
 * dst (16-byte aligned device pointers, non-overlapping), with the 16-byte
 * loads and nontemporal stores the merge kernels use.  A measurement
 * reference for achievable HBM bandwidth and for calibrating hardware
 * traffic counters; not part of the merge method.
 *   unroll  16-byte loads in flight per lane: 1, 2, 4, 8 (0 = 8) or 16
 *   grid    workgroups of 256 lanes (0 = 32 per compute unit)
 */
mp_status mp_copy(const void *src, void *dst, int64_t n_bytes, int32_t unroll,
                  int32_t grid, void *stream);

/*
 * mp_bw_probe -- bandwidth references for the roofline: the copy above
 * (kind 0), the same loads alone (kind 1: src is read, and each wavefront
 * stores the XOR of what it read to dst, which must hold grid * 4 16-byte
 * words; grid 0 means 32 per compute unit, the count used for the sink)
 * and the same stores alone (kind 2: dst receives n_bytes of a fixed
 * pattern, src is unused and may be NULL).  Not part of the merge method.
 *   n_bytes  multiple of 16; pointers 16-byte aligned; unroll 1, 2, 4, 8
 *            (0 = 8) or 16 loads or stores in flight per lane.
 * MP_ERR_INVALID_ARG for a bad kind, size or pointer, MP_ERR_OVERLAP when
 * src and dst (as used) overlap, MP_ERR_UNSUPPORTED for another unroll.
 */
mp_status mp_bw_probe(int32_t kind, const void *src, void *dst, int64_t n_bytes,
                      int32_t unroll, int32_t grid, void *stream);

/*
 * Kernel timing (profiling aid, off by default).  While enabled, every kernel
 * the library launches is bracketed by two HIP events recorded on the launch
 * stream.  mp_timing_query synchronises on the recorded events and returns,
 * for the kernel family `name` (e.g. "merge_tiles", "partition"), the summed
 * duration in milliseconds and the number of launches since the last reset.
 * Returns MP_ERR_INVALID_ARG for NULL outputs, MP_ERR_HIP on event errors.
 */
mp_status mp_timing_enable(int on);
mp_status mp_timing_reset(void);
mp_status mp_timing_query(const char *name, double *total_ms, int64_t *launches);

/*
 * Window statistics of the persistent merge kernels, collected while timing
 * is enabled (device counters, zeroed by mp_timing_reset): the number of
 * output tiles processed and how many of them left their predicted input
 * windows and were searched again over full windows.  Synchronises with the
 * device.  MP_ERR_INVALID_ARG for NULL outputs.
 */
mp_status mp_stats_query(int64_t *tiles, int64_t *reloads);

/*
 * Companion counter of mp_stats_query: how many workgroups of the persistent
 * merge kernels had at least one tile (each walks a contiguous run of tiles,
 * Corollary 7), so tiles / workgroups is the mean run length.  Same
 * collection, reset and synchronisation rules.  MP_ERR_INVALID_ARG for NULL.
 */
mp_status mp_stats_workgroups(int64_t *groups);

#ifdef __cplusplus
}
#endif

#endif /* MERGEPATH_H */
