/*
 * Merge Path oracle: TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, obviously correct, single-threaded C written from the paper
 * (Green, Odeh, Birk: "Merge Path - A Visually Intuitive Approach to Parallel
 * Merging").  It shares no code, header or constant with the GPU library, and
 * only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * load it.  The GPU product path never calls it.
 *
 * Every function computes the plain definition of what the GPU path reaches:
 *   - merge:      the sequential merge that walks the Merge Path
 *                 (section 2.1, construction; Lemma 1);
 *   - partition:  the point where the Merge Path crosses cross diagonal d
 *                 (Lemma 8, Theorem 9): the number of A elements among the
 *                 first d merged outputs;
 *   - sort:       bottom-up merge sort, log2 N rounds of pairwise merges
 *                 (section 1; section 3, parallel merge sort);
 *   - batched:    independent merges of many (A_k, B_k) pairs written back to
 *                 back (Corollary 6 applied pair by pair);
 *   - set ops:    the multiset intersection, union, difference and symmetric
 *                 difference walked like the merge (matched equal heads);
 *   - join:       every equal-key pair (i, j), by a nested loop.
 *
 * Key types: u32 and u64 compare unsigned, i32 signed, f32 with IEEE '<'/'>'
 * (so -0.0 and +0.0 tie, and the tie rule decides which bit pattern is output).
 * Values are opaque 4-byte words carried with their key.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* The path's step rule (section 2.1): step right, taking B[j], iff A[i] > B[j].
 * Overridable only so that a test can build a deliberately wrong oracle and
 * show that the pins reject it. */
#ifndef ORACLE_TAKE_B
#define ORACLE_TAKE_B(a, b) ((a) > (b))
#endif

/*
 * Sequential merge along the Merge Path (section 2.1): standing at (i, j),
 * if A[i] > B[j] the path steps right and emits B[j]; otherwise it steps down
 * and emits A[i].  At the right or bottom edge only one direction remains.
 * Ties therefore emit A first.  src[k] (optional) receives the position of
 * S[k] in the concatenation A ++ B.
 */
#define DEFINE_MERGE(T, NAME)                                                  \
  void oracle_merge_##NAME(const T *A, int64_t na, const T *B, int64_t nb,     \
                           T *S, int64_t *src) {                               \
    int64_t i = 0, j = 0;                                                      \
    for (int64_t k = 0; k < na + nb; ++k) {                                    \
      int take_b;                                                              \
      if (i == na)                                                             \
        take_b = 1;                                                            \
      else if (j == nb)                                                        \
        take_b = 0;                                                            \
      else                                                                     \
        take_b = ORACLE_TAKE_B(A[i], B[j]);                                    \
      if (take_b) {                                                            \
        S[k] = B[j];                                                           \
        if (src) src[k] = na + j;                                              \
        ++j;                                                                   \
      } else {                                                                 \
        S[k] = A[i];                                                           \
        if (src) src[k] = i;                                                   \
        ++i;                                                                   \
      }                                                                        \
    }                                                                          \
  }

/* Key-value merge: the key merge above, each value travelling with its key. */
#define DEFINE_MERGE_KV(T, NAME)                                               \
  int oracle_merge_kv_##NAME(const T *Ak, const uint32_t *Av, int64_t na,      \
                             const T *Bk, const uint32_t *Bv, int64_t nb,      \
                             T *Sk, uint32_t *Sv) {                            \
    int64_t n = na + nb;                                                       \
    int64_t *src = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t)); \
    if (!src) return -1;                                                       \
    oracle_merge_##NAME(Ak, na, Bk, nb, Sk, src);                              \
    for (int64_t k = 0; k < n; ++k)                                            \
      Sv[k] = src[k] < na ? Av[src[k]] : Bv[src[k] - na];                      \
    free(src);                                                                 \
    return 0;                                                                  \
  }

/*
 * Split on cross diagonal d (Lemma 8, Theorem 9): the k-th point of the Merge
 * Path lies on the k-th cross diagonal, so the path crosses diagonal d after
 * exactly d merge steps; the split is how many of those d steps took A.
 * Diagonals may come in any order; each must lie in [0, na + nb].
 */
typedef struct {
  int64_t d;
  int64_t idx;
} diag_item;

static int cmp_diag(const void *x, const void *y) {
  const diag_item *p = (const diag_item *)x, *q = (const diag_item *)y;
  if (p->d != q->d) return p->d < q->d ? -1 : 1;
  return p->idx < q->idx ? -1 : (p->idx > q->idx);
}

#define DEFINE_PARTITION(T, NAME)                                              \
  int oracle_partition_##NAME(const T *A, int64_t na, const T *B, int64_t nb,  \
                              const int64_t *diag, int64_t n_diag,             \
                              int64_t *a_split) {                              \
    diag_item *items =                                                         \
        (diag_item *)malloc((size_t)(n_diag > 0 ? n_diag : 1) * sizeof(diag_item)); \
    if (!items) return -1;                                                     \
    for (int64_t t = 0; t < n_diag; ++t) {                                     \
      if (diag[t] < 0 || diag[t] > na + nb) {                                  \
        free(items);                                                           \
        return -2;                                                             \
      }                                                                        \
      items[t].d = diag[t];                                                    \
      items[t].idx = t;                                                        \
    }                                                                          \
    qsort(items, (size_t)n_diag, sizeof(diag_item), cmp_diag);                 \
    int64_t i = 0, j = 0, t = 0;                                               \
    for (int64_t k = 0; k <= na + nb; ++k) {                                   \
      while (t < n_diag && items[t].d == k) a_split[items[t++].idx] = i;       \
      if (k == na + nb) break;                                                 \
      int take_b;                                                              \
      if (i == na)                                                             \
        take_b = 1;                                                            \
      else if (j == nb)                                                        \
        take_b = 0;                                                            \
      else                                                                     \
        take_b = ORACLE_TAKE_B(A[i], B[j]);                                    \
      if (take_b)                                                              \
        ++j;                                                                   \
      else                                                                     \
        ++i;                                                                   \
    }                                                                          \
    free(items);                                                               \
    return 0;                                                                  \
  }

/*
 * Bottom-up merge sort: round r merges adjacent sorted runs of width 2^r,
 * the left run as A and the right run as B, so equal keys keep their input
 * order (stable).  A trailing run without a partner is copied through.
 * vals may be NULL.
 */
#define DEFINE_SORT(T, NAME)                                                   \
  int oracle_sort_##NAME(T *keys, uint32_t *vals, int64_t n) {                 \
    if (n <= 1) return 0;                                                      \
    T *tk = (T *)malloc((size_t)n * sizeof(T));                                \
    uint32_t *tv = vals ? (uint32_t *)malloc((size_t)n * sizeof(uint32_t)) : NULL; \
    int64_t *src = (int64_t *)malloc((size_t)n * sizeof(int64_t));             \
    if (!tk || !src || (vals && !tv)) {                                        \
      free(tk); free(tv); free(src);                                           \
      return -1;                                                               \
    }                                                                          \
    T *ik = keys, *ok = tk;                                                    \
    uint32_t *iv = vals, *ov = tv;                                             \
    for (int64_t w = 1; w < n; w *= 2) {                                       \
      for (int64_t lo = 0; lo < n; lo += 2 * w) {                              \
        int64_t mid = lo + w < n ? lo + w : n;                                 \
        int64_t hi = lo + 2 * w < n ? lo + 2 * w : n;                          \
        oracle_merge_##NAME(ik + lo, mid - lo, ik + mid, hi - mid, ok + lo, src); \
        if (vals)                                                              \
          for (int64_t k = 0; k < hi - lo; ++k) ov[lo + k] = iv[lo + src[k]];  \
      }                                                                        \
      T *sk = ik; ik = ok; ok = sk;                                            \
      uint32_t *sv = iv; iv = ov; ov = sv;                                     \
    }                                                                          \
    if (ik != keys) {                                                          \
      memcpy(keys, ik, (size_t)n * sizeof(T));                                 \
      if (vals) memcpy(vals, iv, (size_t)n * sizeof(uint32_t));                \
    }                                                                          \
    free(tk); free(tv); free(src);                                             \
    return 0;                                                                  \
  }

/*
 * Batched merge: pair k is (A[a_off[k], a_off[k+1]), B[b_off[k], b_off[k+1]));
 * its merge is written to S starting at a_off[k] + b_off[k].
 */
#define DEFINE_BATCHED(T, NAME)                                                \
  int oracle_merge_batched_##NAME(const T *A, const int64_t *a_off,            \
                                  const T *B, const int64_t *b_off,            \
                                  int64_t n_pairs, T *S) {                     \
    for (int64_t k = 0; k < n_pairs; ++k) {                                    \
      int64_t na = a_off[k + 1] - a_off[k], nb = b_off[k + 1] - b_off[k];      \
      if (na < 0 || nb < 0) return -2;                                         \
      oracle_merge_##NAME(A + a_off[k], na, B + b_off[k], nb,                  \
                          S + a_off[k] + b_off[k], NULL);                      \
    }                                                                          \
    return 0;                                                                  \
  }

/*
 * Multiset operations on sorted inputs, walked like the merge (op 0 =
 * intersection, 1 = union, 2 = difference A minus B, 3 = symmetric
 * difference).  Standing at (i, j): the smaller head is unmatched and moves
 * on alone; equal heads are a matched pair and both move on.  Union keeps
 * every unmatched head and one key (A's) of each matched pair; intersection
 * keeps A's key of each matched pair; difference keeps unmatched A heads;
 * symmetric difference keeps every unmatched head.  So a value found m
 * times in A and n times in B comes out min(m, n), max(m, n), max(m - n, 0)
 * and |m - n| times, A's copies before B's.  Returns the output count.
 */
#define DEFINE_SETOP(T, NAME)                                                  \
  int64_t oracle_set_op_##NAME(int op, const T *A, int64_t na, const T *B,     \
                               int64_t nb, T *S) {                             \
    int64_t i = 0, j = 0, k = 0;                                               \
    while (i < na || j < nb) {                                                 \
      if (j == nb || (i < na && A[i] < B[j])) {                                \
        if (op != 0) S[k++] = A[i];                                            \
        ++i;                                                                   \
      } else if (i == na || B[j] < A[i]) {                                     \
        if (op == 1 || op == 3) S[k++] = B[j];                                 \
        ++j;                                                                   \
      } else {                                                                 \
        if (op == 0 || op == 1) S[k++] = A[i];                                 \
        ++i;                                                                   \
        ++j;                                                                   \
      }                                                                        \
    }                                                                          \
    return k;                                                                  \
  }

/*
 * Inner join (the database join the introduction names as a use of the
 * merge): every pair (i, j) with A[i] equal to B[j], by its definition, a
 * nested loop over A then B, so the pairs come out ordered by i, then j.
 * Equality is IEEE equality for floats (-0.0 equals +0.0).  The first `cap`
 * pairs are written to I[] and J[]; returns the number of pairs.  (The
 * equality test is overridable only so that a test can plant a mistake.)
 */
#ifndef ORACLE_JOIN_EQ
#define ORACLE_JOIN_EQ(a, b) ((a) == (b))
#endif
#define DEFINE_JOIN(T, NAME)                                                   \
  int64_t oracle_join_##NAME(const T *A, int64_t na, const T *B, int64_t nb,   \
                             int64_t *I, int64_t *J, int64_t cap) {            \
    int64_t k = 0;                                                             \
    for (int64_t i = 0; i < na; ++i)                                           \
      for (int64_t j = 0; j < nb; ++j)                                         \
        if (ORACLE_JOIN_EQ(A[i], B[j])) {                                      \
          if (k < cap) {                                                       \
            I[k] = i;                                                          \
            J[k] = j;                                                          \
          }                                                                    \
          ++k;                                                                 \
        }                                                                      \
    return k;                                                                  \
  }

#define DEFINE_ALL(T, NAME)                                                    \
  DEFINE_MERGE(T, NAME)                                                        \
  DEFINE_MERGE_KV(T, NAME)                                                     \
  DEFINE_PARTITION(T, NAME)                                                    \
  DEFINE_SORT(T, NAME)                                                         \
  DEFINE_BATCHED(T, NAME)                                                      \
  DEFINE_SETOP(T, NAME)                                                        \
  DEFINE_JOIN(T, NAME)

DEFINE_ALL(uint32_t, u32)
DEFINE_ALL(int32_t, i32)
DEFINE_ALL(uint64_t, u64)
DEFINE_ALL(float, f32)
