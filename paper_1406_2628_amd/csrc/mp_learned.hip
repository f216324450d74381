// Learned split predictor: a small MLP that predicts where the Merge Path
// crosses each diagonal, followed by an exact search in a bounded window.
//
// The paper's split search (Algorithm 2, Theorem 14) needs up to
// ceil(log2(min(na, nb) + 1)) dependent probes per diagonal.  Here an MLP
// predicts the split a_hat; the exact lower-bound search then runs only on
// [a_hat - w, a_hat + w] clipped to the diagonal.  The result is certified
// by the search itself: a lower-bound search over true keys returns the
// unique split whenever it lies strictly inside the probed interval (the
// predicate B[d-1-a] < A[a] is monotone, Corollary 12).  Only a result on a
// window edge that is not also a diagonal bound needs the two conditions of
// Algorithm 2 checked explicitly (two more probes); if they fail, the plain
// full-range search runs (the fallback), so the output is always identical
// to mp_partition.
//
// Model (F inputs, H hidden units, FP32):
//   x = [t, sin 2 pi t, cos 2 pi t, sin 4 pi t, cos 4 pi t][:F],  t = d / (na + nb)
//   y = w2 . relu(W1 x + b1) + b2
//   a_hat = a_prior(d) + round(y * na),  a_prior(d) = clamp(round(d na / N))
// Parameters: [W1 (H x F, row-major), b1 (H), w2 (H), b2].  Training
// minimises the mean squared error of y against (a* - a_prior) / na over
// exact splits a* produced by the binary search itself; gradients are
// reduced in a fixed order (deterministic), and Adam updates the weights.
//
// Windows.  The model's error is far from uniform along the diagonals (it
// peaks where the key distribution has a kink: a narrow cluster, a run of
// equal keys) and, where the smooth model misses such a kink, it is biased
// to one side.  So calibration keeps, per bucket of t = d / N (kLpBuckets
// equal buckets), an asymmetric window [a_hat + lo, a_hat + hi]: the
// smallest and largest signed error a* - a_hat seen in the bucket and its
// neighbours, widened by an eighth of that span and by three standard
// deviations of the seed-to-seed noise of a split.  A diagonal searches only
// its bucket's window; a split beyond it is caught by the certificate below
// and found by the fallback, so the output never depends on the windows.
#include <math.h>
#include <algorithm>
#include <mutex>
#include <stdio.h>
#include <string.h>
#include <string>
#include <type_traits>
#include <vector>

#include "mp_device.h"
#include "mp_internal.h"

namespace mp {

constexpr int kLpMaxHidden = 64;
constexpr int kLpMaxFeatures = 5;
constexpr int kLpMaxParams = kLpMaxHidden * kLpMaxFeatures + 2 * kLpMaxHidden + 1;
constexpr int kLpBuckets = 16384;  // window buckets of t = d / N
constexpr int kLpOldBuckets = 1024;  // buckets of the symmetric windows of format 2
static_assert(kLpBuckets % kLpOldBuckets == 0, "format 2 buckets must nest");

// Bucket of diagonal d in [0, N] (N = na + nb): floor(d K / (N + 1)), exact
// for N < 2^49 (any pair that fits in device memory).
__host__ __device__ inline int lp_bucket(int64_t d, int64_t N) {
  const int64_t b = N > 0 ? (d * kLpBuckets) / (N + 1) : 0;
  return (int)(b < 0 ? 0 : (b >= kLpBuckets ? kLpBuckets - 1 : b));
}

__host__ __device__ inline int lp_num_params(int F, int H) { return H * F + 2 * H + 1; }

// Inputs of the model for diagonal d of an na x nb grid.
__device__ __forceinline__ void lp_features(int64_t d, int64_t na, int64_t nb, int F,
                                            float *x) {
  const float t = (float)((double)d / (double)(na + nb));
  const float two_pi = 6.28318530717958647692f;
  x[0] = t;
  if (F >= 3) {
    x[1] = sinf(two_pi * t);
    x[2] = cosf(two_pi * t);
  }
  if (F >= 5) {
    x[3] = sinf(2.0f * two_pi * t);
    x[4] = cosf(2.0f * two_pi * t);
  }
}

// Proportional prior: the split if both inputs were spread evenly.
__device__ __forceinline__ int64_t lp_prior(int64_t d, int64_t na, int64_t nb) {
  int64_t lo, hi;
  diag_range<int64_t>(d, na, nb, lo, hi);
  const int64_t n = na + nb;
  int64_t a = n > 0 ? (int64_t)llrint((double)d * (double)na / (double)n) : 0;
  return a < lo ? lo : (a > hi ? hi : a);
}

// y = w2 . relu(W1 x + b1) + b2 with parameters in p (any address space).
// FC, HC > 0 fix the shape at compile time (F = FC, H = HC; the loops then
// unroll and constant-offset reads of a kernel-argument pointer become
// scalar loads); the operations and their order are the same either way, so
// both give the same bits.
template <int FC = 0, int HC = 0, typename PP>
__device__ __forceinline__ float lp_forward(const PP &p, const float *x, int F_, int H_) {
  const int F = FC > 0 ? FC : F_, H = HC > 0 ? HC : H_;
  const int ob1 = H * F, ow2 = ob1 + H, ob2 = ow2 + H;
  float y = p[ob2];
  for (int j = 0; j < H; ++j) {
    float z = p[ob1 + j];
    for (int f = 0; f < F; ++f) z = fmaf(p[j * F + f], x[f], z);
    y = fmaf(p[ow2 + j], z > 0.f ? z : 0.f, y);
  }
  return y;
}

// Prediction for diagonal d clipped to the diagonal [dlo, dhi]: the point
// both calibration and search put their windows around.  A prediction that
// is not finite (or absurdly large) adds nothing to the prior.
template <int FC = 0, int HC = 0, typename PP>
__device__ __forceinline__ int64_t lp_predict(const PP &p, int64_t d, int64_t na, int64_t nb,
                                              int F, int H, int64_t dlo, int64_t dhi) {
  float x[kLpMaxFeatures];
  lp_features(d, na, nb, FC > 0 ? FC : F, x);
  const float ys = lp_forward<FC, HC>(p, x, F, H) * (float)na;
  const int64_t a = lp_prior(d, na, nb) +
                    (isfinite(ys) && fabsf(ys) < 4.0e18f ? (int64_t)llrintf(ys) : 0);
  return a < dlo ? dlo : (a > dhi ? dhi : a);
}

// a_hat + off clipped to [dlo, dhi], without overflow for any offset
// (dlo <= a_hat <= dhi).
__device__ __forceinline__ int64_t lp_edge(int64_t ahat, int64_t off, int64_t dlo, int64_t dhi) {
  return off <= dlo - ahat ? dlo : (off >= dhi - ahat ? dhi : ahat + off);
}

// ---- training kernels -------------------------------------------------------

// Features and targets of K training diagonals of one set.
__global__ void lp_examples_kernel(const int64_t *__restrict__ diag,
                                   const int64_t *__restrict__ split, int64_t K,
                                   int64_t na, int64_t nb, int F, float *__restrict__ X,
                                   float *__restrict__ r) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= K) return;
  float x[kLpMaxFeatures];
  lp_features(diag[k], na, nb, F, x);
  for (int f = 0; f < F; ++f) X[k * F + f] = x[f];
  r[k] = na > 0 ? (float)((double)(split[k] - lp_prior(diag[k], na, nb)) / (double)na) : 0.f;
}

// Stratified diagonals: d_j = floor((j + u_j) N / K), u_j from a
// counter-based hash (SplitMix64 finaliser) of (seed, j).
__device__ __forceinline__ uint64_t lp_mix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__global__ void lp_diagonals_kernel(int64_t *__restrict__ diag, int64_t K, int64_t n,
                                    uint64_t seed) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= K) return;
  const double u = (double)(lp_mix64(seed * 0x100000001B3ull + (uint64_t)j) >> 11) *
                   (1.0 / 9007199254740992.0);
  int64_t d = (int64_t)(((double)j + u) * (double)n / (double)K);
  diag[j] = d < 0 ? 0 : (d > n ? n : d);
}

// Per-block partial gradients of the mean squared error (deterministic:
// every reduction runs in a fixed order).  grad_part[block][p].
__global__ __launch_bounds__(256) void lp_grad_kernel(const float *__restrict__ params,
                                                      const float *__restrict__ X,
                                                      const float *__restrict__ r,
                                                      int64_t K, int F, int H,
                                                      float *__restrict__ grad_part,
                                                      float *__restrict__ loss_part) {
  __shared__ float sp[kLpMaxParams];
  __shared__ float wsum[4][kLpMaxParams + 1];
  const int P = lp_num_params(F, H);
  for (int i = threadIdx.x; i < P; i += blockDim.x) sp[i] = params[i];
  __syncthreads();
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool live = k < K;
  float x[kLpMaxFeatures] = {0.f, 0.f, 0.f, 0.f, 0.f};
  if (live)
    for (int f = 0; f < F; ++f) x[f] = X[k * F + f];
  const int ob1 = H * F, ow2 = ob1 + H, ob2 = ow2 + H;
  float z[kLpMaxHidden];
  float y = sp[ob2];
  for (int j = 0; j < H; ++j) {
    float zz = sp[ob1 + j];
    for (int f = 0; f < F; ++f) zz = fmaf(sp[j * F + f], x[f], zz);
    z[j] = zz;
    y = fmaf(sp[ow2 + j], zz > 0.f ? zz : 0.f, y);
  }
  const float e = live ? y - r[k] : 0.f;
  const float gy = 2.0f * e / (float)K;  // dL/dy for this sample
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  // one parameter at a time: this sample's contribution, summed over the wave
  auto wave_sum = [&](float v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
  };
  for (int p = 0; p <= P; ++p) {
    float v;
    if (p == P) {
      v = live ? e * e : 0.f;  // loss numerator
    } else if (p < ob1) {
      const int j = p / F, f = p - j * F;
      v = z[j] > 0.f ? gy * sp[ow2 + j] * x[f] : 0.f;
    } else if (p < ow2) {
      const int j = p - ob1;
      v = z[j] > 0.f ? gy * sp[ow2 + j] : 0.f;
    } else if (p < ob2) {
      const int j = p - ow2;
      v = gy * (z[j] > 0.f ? z[j] : 0.f);
    } else {
      v = gy;
    }
    v = wave_sum(v);
    if (lane == 0) wsum[wv][p] = v;
  }
  __syncthreads();
  const int nw = (blockDim.x + 63) >> 6;
  for (int p = threadIdx.x; p <= P; p += blockDim.x) {
    float s = 0.f;
    for (int w = 0; w < nw; ++w) s += wsum[w][p];
    if (p == P) loss_part[blockIdx.x] = s;
    else grad_part[(int64_t)blockIdx.x * P + p] = s;
  }
}

// Sum the block partials in block order, then (lr > 0) one Adam step.
__global__ void lp_adam_kernel(float *__restrict__ params, float *__restrict__ m,
                               float *__restrict__ v, const float *__restrict__ grad_part,
                               const float *__restrict__ loss_part, int n_blocks, int P,
                               float lr, float beta1, float beta2, float eps, int step,
                               float *__restrict__ grad_out, float *__restrict__ loss_out,
                               int64_t K) {
  const int p = threadIdx.x;
  if (p == 0 && loss_out) {
    float s = 0.f;
    for (int b = 0; b < n_blocks; ++b) s += loss_part[b];
    *loss_out = s / (float)K;
  }
  if (p >= P) return;
  float g = 0.f;
  for (int b = 0; b < n_blocks; ++b) g += grad_part[(int64_t)b * P + p];
  if (grad_out) grad_out[p] = g;
  if (lr <= 0.f) return;
  const float mm = beta1 * m[p] + (1.f - beta1) * g;
  const float vv = beta2 * v[p] + (1.f - beta2) * g * g;
  m[p] = mm;
  v[p] = vv;
  const float mh = mm / (1.f - powf(beta1, (float)step));
  const float vh = vv / (1.f - powf(beta2, (float)step));
  params[p] -= lr * mh / (sqrtf(vh) + eps);
}

__global__ void lp_forward_kernel(const float *__restrict__ params, const float *__restrict__ X,
                                  int64_t K, int F, int H, float *__restrict__ y) {
  __shared__ float sp[kLpMaxParams];
  const int P = lp_num_params(F, H);
  for (int i = threadIdx.x; i < P; i += blockDim.x) sp[i] = params[i];
  __syncthreads();
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= K) return;
  float x[kLpMaxFeatures];
  for (int f = 0; f < F; ++f) x[f] = X[k * F + f];
  y[k] = lp_forward(sp, x, F, H);
}

// Largest |a_hat - a*| over a set of diagonals, overall (max_err[0]) and per
// window bucket (max_err[1 + b]).
// Signed calibration errors e = a* - a_hat.  err[0]: the largest |e|; per
// bucket b, err[1 + b] the smallest and err[1 + kLpBuckets + b] the largest
// e, each stored as e with its sign bit flipped so that unsigned atomics
// order them as signed values (the caller fills the minima with all ones
// and the maxima with zeros).
__device__ __forceinline__ unsigned long long lp_ordered(int64_t e) {
  return (unsigned long long)e ^ (1ull << 63);
}

__global__ void lp_error_kernel(const float *__restrict__ params, const int64_t *__restrict__ diag,
                                const int64_t *__restrict__ split, int64_t K, int64_t na,
                                int64_t nb, int F, int H, unsigned long long *__restrict__ err) {
  __shared__ float sp[kLpMaxParams];
  const int P = lp_num_params(F, H);
  for (int i = threadIdx.x; i < P; i += blockDim.x) sp[i] = params[i];
  __syncthreads();
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= K) return;
  const int64_t d = diag[k];
  int64_t dlo, dhi;
  diag_range<int64_t>(d, na, nb, dlo, dhi);
  const int64_t e = split[k] - lp_predict(sp, d, na, nb, F, H, dlo, dhi);
  const int b = lp_bucket(d, na + nb);
  atomicMax(err, (unsigned long long)(e < 0 ? -e : e));
  atomicMin(err + 1 + b, lp_ordered(e));
  atomicMax(err + 1 + kLpBuckets + b, lp_ordered(e));
}

// ---- inference: predicted window + exact search + certificate ------------

// windows: kLpBuckets (lo, hi) offset pairs (device), or NULL for the
// symmetric window [-window, window] on every diagonal.  G lanes per
// diagonal (G = 1: split_search; G > 1: group_split_search, every lane of
// the group evaluating the same model and lane 0 writing).  FC, HC > 0: a
// model of that shape compiled in, its weights read straight from
// `params` (scalar loads, no LDS staging or barrier); 0: any shape, weights
// staged in LDS.
template <typename K, int G, int FC, int HC>
__global__ __launch_bounds__(256) void learned_partition_kernel(
    const float *__restrict__ params, int F, int H, int64_t window,
    const int64_t *__restrict__ windows, const K *__restrict__ A, int64_t na,
    const K *__restrict__ B, int64_t nb, const int64_t *__restrict__ diag, int64_t n_diag,
    int64_t *__restrict__ a_split, unsigned long long *__restrict__ n_fallback) {
  __shared__ float sp[FC > 0 ? 1 : kLpMaxParams];
  if constexpr (FC == 0) {
    const int P = lp_num_params(F, H);
    for (int i = threadIdx.x; i < P; i += blockDim.x) sp[i] = params[i];
    __syncthreads();
  }
  // groups never straddle a workgroup (G divides 256), so a group exits as one
  const int64_t k = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / G;
  if (k >= n_diag) return;
  const int64_t n = na + nb;
  int64_t d = diag[k];
  d = d < 0 ? 0 : (d > n ? n : d);
  int64_t dlo, dhi;
  diag_range<int64_t>(d, na, nb, dlo, dhi);
  // the window offsets depend on d alone: their load overlaps the model
  int64_t wlo = -window, whi = window;
  if (windows) {
    const int b = lp_bucket(d, n);
    wlo = windows[2 * b];
    whi = windows[2 * b + 1];
  }
  int64_t ahat;
  if constexpr (FC > 0) ahat = lp_predict<FC, HC>(params, d, na, nb, F, H, dlo, dhi);
  else ahat = lp_predict(sp, d, na, nb, F, H, dlo, dhi);
  // wlo <= whi, so lo <= hi
  const int64_t lo = lp_edge(ahat, wlo, dlo, dhi);
  const int64_t hi = lp_edge(ahat, whi, dlo, dhi);
  auto ga = [&](int64_t i) { return A[i]; };
  auto gb = [&](int64_t j) { return B[j]; };
  auto search = [&](int64_t l, int64_t h) -> int64_t {
    if constexpr (G == 1) return split_search<int64_t>(d, l, h, ga, gb);
    else return group_split_search<G, int64_t>(d, l, h, ga, gb);
  };
  int64_t a = search(lo, hi);
  // Certificate, needed only on a window edge that is not a diagonal bound:
  // at a == hi the predicate B[d-1-a] < A[a] was never probed; at a == lo
  // its failure at a - 1 was never probed.
  bool ok = true;
  if (a == hi && hi < dhi) ok = B[d - 1 - a] < A[a];
  if (ok && a == lo && lo > dlo) ok = !(B[d - a] < A[a - 1]);
  const bool first = (threadIdx.x & (G - 1)) == 0;
  if (!ok) {
    a = search(dlo, dhi);
    if (n_fallback && first) atomicAdd(n_fallback, 1ull);
  }
  if (first) a_split[k] = a;
}

// ---- host side ----------------------------------------------------------------

struct LpBuf {
  void *p = nullptr;
  size_t size = 0;
  hipError_t ensure(size_t bytes) {
    if (size >= bytes) return hipSuccess;
    if (p) (void)hipFree(p);
    p = nullptr;
    size = 0;
    hipError_t e = hipMalloc(&p, bytes);
    if (e == hipSuccess) size = bytes;
    return e;
  }
  ~LpBuf() {
    if (p) (void)hipFree(p);
  }
};

}  // namespace mp

struct mp_lp_s {
  int F = 5, H = 32;
  int device = 0;
  uint64_t seed = 0;
  int64_t window = -1;  // largest |offset| of any window; < 0: not calibrated
  // kLpBuckets (lo, hi) offset pairs, or empty ([-window, window] everywhere)
  std::vector<int64_t> windows;
  int64_t *d_windows = nullptr;  // device copy of `windows`
  int64_t step = 0;     // Adam steps taken
  float *params = nullptr, *m = nullptr, *v = nullptr;  // device
  mp::LpBuf X, r, diag, split, gpart, lpart, misc;
  ~mp_lp_s() {
    if (d_windows) (void)hipFree(d_windows);
    if (params) (void)hipFree(params);
    if (m) (void)hipFree(m);
    if (v) (void)hipFree(v);
  }
};

namespace mp {
namespace {

mp_status lp_fail(mp_status st, const char *msg) { return set_error(st, "%s", msg); }
mp_status lp_hip(hipError_t e, const char *what) {
  return set_error(MP_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

// Deterministic host-side initialisation: SplitMix64 stream -> Box-Muller.
struct HostRng {
  uint64_t s;
  uint64_t next() {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  }
  double uniform() { return ((next() >> 11) + 0.5) * (1.0 / 9007199254740992.0); }
  double normal() {
    const double u1 = uniform(), u2 = uniform();
    return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
  }
};

std::vector<float> lp_init_params(int F, int H, uint64_t seed) {
  HostRng g{seed};
  std::vector<float> p(lp_num_params(F, H));
  for (int i = 0; i < H * F; ++i) p[i] = (float)(2.0 * g.normal());       // W1
  for (int j = 0; j < H; ++j) p[H * F + j] = (float)g.normal();          // b1
  for (int j = 0; j < H; ++j) p[H * F + H + j] = (float)(0.05 * g.normal());  // w2
  p[H * F + 2 * H] = 0.f;                                                 // b2
  return p;
}

// One full-batch gradient (and optionally an Adam step) over X, r.
mp_status lp_step(mp_lp h, const float *X, const float *r, int64_t K, float lr, float *grad_out,
                  float *loss_out, hipStream_t s) {
  const int P = lp_num_params(h->F, h->H);
  const int64_t nblk = (K + 255) / 256;
  if (nblk > (1 << 22)) return lp_fail(MP_ERR_INVALID_ARG, "too many training examples");
  hipError_t e = h->gpart.ensure((size_t)nblk * P * sizeof(float));
  if (e == hipSuccess) e = h->lpart.ensure((size_t)nblk * sizeof(float));
  if (e != hipSuccess) return lp_hip(e, "training buffers");
  hipLaunchKernelGGL(lp_grad_kernel, dim3((unsigned)nblk), dim3(256), 0, s, h->params, X, r, K,
                     h->F, h->H, (float *)h->gpart.p, (float *)h->lpart.p);
  if (lr > 0.f) h->step += 1;
  hipLaunchKernelGGL(lp_adam_kernel, dim3(1), dim3(kLpMaxParams < 512 ? 512 : kLpMaxParams), 0, s,
                     h->params, h->m, h->v, (const float *)h->gpart.p, (const float *)h->lpart.p,
                     (int)nblk, P, lr, 0.9f, 0.999f, 1e-8f, (int)(h->step > 0 ? h->step : 1),
                     grad_out, loss_out, K);
  e = hipGetLastError();
  return e == hipSuccess ? MP_OK : lp_hip(e, "training launch");
}

// Exact splits of K stratified diagonals of one (A, B) set into h->diag/h->split.
mp_status lp_exact_splits(mp_lp h, mp_dtype kt, const void *A, int64_t na, const void *B,
                          int64_t nb, int64_t K, uint64_t seed, int64_t offset, hipStream_t s) {
  hipError_t e = hipSuccess;
  int64_t *dg = (int64_t *)h->diag.p + offset, *sp = (int64_t *)h->split.p + offset;
  hipLaunchKernelGGL(lp_diagonals_kernel, dim3((unsigned)((K + 255) / 256)), dim3(256), 0, s, dg,
                     K, na + nb, seed);
  dispatch_key(kt, [&](auto k) {
    using KT = decltype(k);
    e = launch_partition<KT>((const KT *)A, na, (const KT *)B, nb, dg, 0, K, sp, s);
  });
  if (e == hipSuccess) e = hipGetLastError();
  return e == hipSuccess ? MP_OK : lp_hip(e, "exact splits");
}

bool lp_valid_key(mp_dtype t) { return t == MP_U32 || t == MP_I32 || t == MP_U64 || t == MP_F32; }

// Install per-bucket windows (w: kLpBuckets (lo, hi) pairs with lo <= hi),
// or, for an empty w, the window [-one, one] everywhere.
mp_status lp_install_windows(mp_lp h, const std::vector<int64_t> &w, int64_t one) {
  if (w.empty()) {
    h->windows.clear();
    h->window = one;
    return MP_OK;
  }
  if (!h->d_windows) {
    hipError_t e = hipMalloc(&h->d_windows, 2 * kLpBuckets * sizeof(int64_t));
    if (e != hipSuccess) {
      h->d_windows = nullptr;
      return lp_hip(e, "window table");
    }
  }
  hipError_t e = hipMemcpy(h->d_windows, w.data(), 2 * kLpBuckets * sizeof(int64_t),
                           hipMemcpyHostToDevice);
  if (e != hipSuccess) return lp_hip(e, "window table");
  h->windows = w;
  int64_t m = 0;
  for (int64_t x : w) m = std::max(m, x < 0 ? -x : x);
  h->window = m;
  return MP_OK;
}

}  // namespace
}  // namespace mp

using namespace mp;

extern "C" {

mp_status mp_lp_create(mp_lp *out, int hidden, int features, uint64_t seed) {
  if (!out) return lp_fail(MP_ERR_INVALID_ARG, "mp_lp_create: NULL handle pointer");
  *out = nullptr;
  if (hidden < 1 || hidden > kLpMaxHidden)
    return lp_fail(MP_ERR_INVALID_ARG, "mp_lp_create: hidden units must be in [1, 64]");
  if (features != 1 && features != 3 && features != 5)
    return lp_fail(MP_ERR_INVALID_ARG, "mp_lp_create: features must be 1, 3 or 5");
  mp_lp h = new mp_lp_s();
  h->F = features;
  h->H = hidden;
  h->seed = seed;
  const int P = lp_num_params(features, hidden);
  hipError_t e = hipGetDevice(&h->device);
  if (e == hipSuccess) e = hipMalloc(&h->params, P * sizeof(float));
  if (e == hipSuccess) e = hipMalloc(&h->m, P * sizeof(float));
  if (e == hipSuccess) e = hipMalloc(&h->v, P * sizeof(float));
  if (e == hipSuccess) e = hipMemset(h->m, 0, P * sizeof(float));
  if (e == hipSuccess) e = hipMemset(h->v, 0, P * sizeof(float));
  if (e == hipSuccess) {
    const std::vector<float> p = lp_init_params(features, hidden, seed);
    e = hipMemcpy(h->params, p.data(), P * sizeof(float), hipMemcpyHostToDevice);
  }
  if (e != hipSuccess) {
    delete h;
    return lp_hip(e, "mp_lp_create");
  }
  *out = h;
  return MP_OK;
}

void mp_lp_destroy(mp_lp h) { delete h; }

int mp_lp_num_params(mp_lp h) { return h ? lp_num_params(h->F, h->H) : 0; }

mp_status mp_lp_shape(mp_lp h, int *features, int *hidden) {
  if (!h || !features || !hidden) return lp_fail(MP_ERR_INVALID_ARG, "mp_lp_shape: bad arguments");
  *features = h->F;
  *hidden = h->H;
  return MP_OK;
}

mp_status mp_lp_get_params(mp_lp h, float *host, int n) {
  if (!h || !host || n != lp_num_params(h->F, h->H))
    return lp_fail(MP_ERR_INVALID_ARG, "mp_lp_get_params: bad handle, buffer or count");
  hipError_t e = hipMemcpy(host, h->params, n * sizeof(float), hipMemcpyDeviceToHost);
  return e == hipSuccess ? MP_OK : lp_hip(e, "mp_lp_get_params");
}

mp_status mp_lp_set_params(mp_lp h, const float *host, int n) {
  if (!h || !host || n != lp_num_params(h->F, h->H))
    return lp_fail(MP_ERR_INVALID_ARG, "mp_lp_set_params: bad handle, buffer or count");
  hipError_t e = hipMemcpy(h->params, host, n * sizeof(float), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(h->m, 0, n * sizeof(float));
  if (e == hipSuccess) e = hipMemset(h->v, 0, n * sizeof(float));
  h->step = 0;
  return e == hipSuccess ? MP_OK : lp_hip(e, "mp_lp_set_params");
}

mp_status mp_lp_set_window(mp_lp h, int64_t window) {
  if (!h || window < 0) return lp_fail(MP_ERR_INVALID_ARG, "mp_lp_set_window: bad handle or window");
  return lp_install_windows(h, {}, window);
}

int64_t mp_lp_window(mp_lp h) { return h ? h->window : -1; }

int32_t mp_lp_windows(mp_lp h, int64_t *windows, int32_t cap) {
  if (!h) return -1;
  const int32_t n = (int32_t)(h->windows.size() / 2);
  if (windows)
    for (int32_t i = 0; i < 2 * cap && i < 2 * n; ++i) windows[i] = h->windows[i];
  return n;
}

mp_status mp_lp_forward(mp_lp h, const float *X, int64_t K, float *y, void *stream) {
  if (!h || K < 0 || (K > 0 && (!X || !y))) return lp_fail(MP_ERR_INVALID_ARG, "mp_lp_forward: bad arguments");
  if (K == 0) return MP_OK;
  hipLaunchKernelGGL(lp_forward_kernel, dim3((unsigned)((K + 255) / 256)), dim3(256), 0,
                     (hipStream_t)stream, h->params, X, K, h->F, h->H, y);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? MP_OK : lp_hip(e, "mp_lp_forward");
}

mp_status mp_lp_grad(mp_lp h, const float *X, const float *r, int64_t K, float *grad,
                     float *loss, void *stream) {
  if (!h || K <= 0 || !X || !r || !grad) return lp_fail(MP_ERR_INVALID_ARG, "mp_lp_grad: bad arguments");
  return lp_step(h, X, r, K, 0.f, grad, loss, (hipStream_t)stream);
}

mp_status mp_lp_adam_step(mp_lp h, const float *X, const float *r, int64_t K, float lr,
                          void *stream) {
  if (!h || K <= 0 || !X || !r || !(lr > 0.f)) return lp_fail(MP_ERR_INVALID_ARG, "mp_lp_adam_step: bad arguments");
  return lp_step(h, X, r, K, lr, nullptr, nullptr, (hipStream_t)stream);
}

mp_status mp_lp_examples(mp_lp h, mp_dtype kt, const void *A, int64_t na, const void *B,
                         int64_t nb, int64_t K, uint64_t seed, float *X, float *r,
                         int64_t *diag, int64_t *split, void *stream) {
  if (!h || !lp_valid_key(kt) || na < 0 || nb < 0 || K <= 0 || !X || !r || (na && !A) || (nb && !B))
    return lp_fail(MP_ERR_INVALID_ARG, "mp_lp_examples: bad arguments");
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = h->diag.ensure(K * 8);
  if (e == hipSuccess) e = h->split.ensure(K * 8);
  if (e != hipSuccess) return lp_hip(e, "mp_lp_examples buffers");
  mp_status st = lp_exact_splits(h, kt, A, na, B, nb, K, seed, 0, s);
  if (st != MP_OK) return st;
  hipLaunchKernelGGL(lp_examples_kernel, dim3((unsigned)((K + 255) / 256)), dim3(256), 0, s,
                     (const int64_t *)h->diag.p, (const int64_t *)h->split.p, K, na, nb, h->F, X, r);
  if (diag) e = hipMemcpyAsync(diag, h->diag.p, K * 8, hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess && split) e = hipMemcpyAsync(split, h->split.p, K * 8, hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess) e = hipGetLastError();
  return e == hipSuccess ? MP_OK : lp_hip(e, "mp_lp_examples");
}

mp_status mp_lp_train(mp_lp h, mp_dtype kt, const void *const *As, const int64_t *nas,
                      const void *const *Bs, const int64_t *nbs, int n_sets, int64_t k_diag,
                      int epochs, float lr, float *final_loss, void *stream) {
  if (!h || !lp_valid_key(kt) || n_sets <= 0 || !As || !Bs || !nas || !nbs || k_diag <= 0 ||
      epochs <= 0 || !(lr > 0.f))
    return lp_fail(MP_ERR_INVALID_ARG, "mp_lp_train: bad arguments");
  for (int i = 0; i < n_sets; ++i)
    if (nas[i] < 0 || nbs[i] < 0 || (nas[i] && !As[i]) || (nbs[i] && !Bs[i]))
      return lp_fail(MP_ERR_INVALID_ARG, "mp_lp_train: bad training set");
  hipStream_t s = (hipStream_t)stream;
  const int64_t K = k_diag * n_sets;
  const int F = h->F;
  hipError_t e = h->X.ensure(K * F * sizeof(float));
  if (e == hipSuccess) e = h->r.ensure(K * sizeof(float));
  if (e == hipSuccess) e = h->diag.ensure(K * 8);
  if (e == hipSuccess) e = h->split.ensure(K * 8);
  if (e != hipSuccess) return lp_hip(e, "mp_lp_train buffers");
  // exact splits from the plain search, then examples
  for (int i = 0; i < n_sets; ++i) {
    const int64_t off = (int64_t)i * k_diag;
    mp_status st = lp_exact_splits(h, kt, As[i], nas[i], Bs[i], nbs[i], k_diag,
                                   h->seed * 1315423911ull + (uint64_t)i + 1, off, s);
    if (st != MP_OK) return st;
    hipLaunchKernelGGL(lp_examples_kernel, dim3((unsigned)((k_diag + 255) / 256)), dim3(256), 0, s,
                       (const int64_t *)h->diag.p + off, (const int64_t *)h->split.p + off, k_diag,
                       nas[i], nbs[i], F, (float *)h->X.p + off * F, (float *)h->r.p + off);
  }
  // cosine-decayed Adam over the full batch
  for (int ep = 0; ep < epochs; ++ep) {
    const float lr_t = 1e-5f + 0.5f * lr * (1.0f + cosf(3.14159265f * (float)ep / (float)epochs));
    mp_status st = lp_step(h, (const float *)h->X.p, (const float *)h->r.p, K, lr_t, nullptr,
                           nullptr, s);
    if (st != MP_OK) return st;
  }
  if (final_loss) {
    e = h->misc.ensure(64 * sizeof(float) + kLpMaxParams * sizeof(float));
    if (e != hipSuccess) return lp_hip(e, "mp_lp_train");
    mp_status st = lp_step(h, (const float *)h->X.p, (const float *)h->r.p, K, 0.f,
                           (float *)h->misc.p + 64, (float *)h->misc.p, s);
    if (st != MP_OK) return st;
    e = hipMemcpyAsync(final_loss, h->misc.p, sizeof(float), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return lp_hip(e, "mp_lp_train");
  }
  return MP_OK;
}

mp_status mp_lp_calibrate(mp_lp h, mp_dtype kt, const void *A, int64_t na, const void *B,
                          int64_t nb, int64_t n_diag, int64_t *max_err, void *stream) {
  if (!h || !lp_valid_key(kt) || na < 0 || nb < 0 || n_diag <= 0 || (na && !A) || (nb && !B))
    return lp_fail(MP_ERR_INVALID_ARG, "mp_lp_calibrate: bad arguments");
  hipStream_t s = (hipStream_t)stream;
  const size_t n_err = 1 + 2 * (size_t)kLpBuckets;
  hipError_t e = h->diag.ensure(n_diag * 8);
  if (e == hipSuccess) e = h->split.ensure(n_diag * 8);
  if (e == hipSuccess) e = h->misc.ensure(n_err * sizeof(unsigned long long));
  if (e != hipSuccess) return lp_hip(e, "mp_lp_calibrate buffers");
  mp_status st = lp_exact_splits(h, kt, A, na, B, nb, n_diag, h->seed ^ 0xC0FFEEull, 0, s);
  if (st != MP_OK) return st;
  unsigned long long *derr = (unsigned long long *)h->misc.p;
  e = hipMemsetAsync(derr, 0, sizeof(unsigned long long), s);
  if (e == hipSuccess) e = hipMemsetAsync(derr + 1, 0xff, kLpBuckets * sizeof(unsigned long long), s);
  if (e == hipSuccess)
    e = hipMemsetAsync(derr + 1 + kLpBuckets, 0, kLpBuckets * sizeof(unsigned long long), s);
  if (e != hipSuccess) return lp_hip(e, "mp_lp_calibrate");
  hipLaunchKernelGGL(lp_error_kernel, dim3((unsigned)((n_diag + 255) / 256)), dim3(256), 0, s,
                     h->params, (const int64_t *)h->diag.p, (const int64_t *)h->split.p, n_diag,
                     na, nb, h->F, h->H, derr);
  std::vector<unsigned long long> he(n_err);
  e = hipMemcpyAsync(he.data(), derr, n_err * sizeof(unsigned long long), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return lp_hip(e, "mp_lp_calibrate");
  auto signed_of = [](unsigned long long u) { return (int64_t)(u ^ (1ull << 63)); };
  const unsigned long long kEmpty = ~0ull;  // a minimum slot no sample reached
  // Overall extremes, for buckets without samples nearby.
  int64_t all_lo = 0, all_hi = 0;
  bool any = false;
  for (int b = 0; b < kLpBuckets; ++b) {
    if (he[1 + b] == kEmpty) continue;
    const int64_t lo = signed_of(he[1 + b]), hi = signed_of(he[1 + kLpBuckets + b]);
    all_lo = any ? std::min(all_lo, lo) : lo;
    all_hi = any ? std::max(all_hi, hi) : hi;
    any = true;
  }
  // Neighbourhood of a bucket: itself and r buckets on each side, r chosen
  // so that it holds about 16 samples or more (r = 1 at 16 samples per
  // bucket).
  const int64_t r64 = (16 * (int64_t)kLpBuckets + n_diag - 1) / n_diag;
  const int r = (int)std::min<int64_t>(std::max<int64_t>(r64, 1), kLpBuckets);
  // Seed-to-seed noise of a split: for two iid samples the number of A keys
  // among the first d keys of the merge is hypergeometric, with variance at
  // most na nb / (4 (na + nb)).
  const double sigma = na + nb > 0 ? sqrt((double)na * (double)nb / (4.0 * (double)(na + nb))) : 0.0;
  const int64_t noise = (int64_t)ceil(3.0 * sigma) + 1;
  // Extremes over [b - r, b + r] for every b in O(kLpBuckets) (van Herk /
  // Gil-Werman: running extremes inside blocks of 2r + 1, from the left and
  // from the right); an empty bucket holds the neutral value.
  const int64_t kNone = INT64_MAX;  // neutral for the minimum; -kNone for the maximum
  auto sliding = [&](std::vector<int64_t> v, bool is_max) {
    const int K = kLpBuckets, m = 2 * r + 1;
    auto pick = [&](int64_t a, int64_t b) { return is_max ? std::max(a, b) : std::min(a, b); };
    // pre/suf: extremes from the start of i's block to i / from i to the
    // end of its block; p0/s0: from bucket 0 to i / from i to the last.
    std::vector<int64_t> pre(K), suf(K), p0(K), s0(K), out(K);
    for (int i = 0; i < K; ++i) {
      pre[i] = (i % m == 0) ? v[i] : pick(pre[i - 1], v[i]);
      p0[i] = i == 0 ? v[i] : pick(p0[i - 1], v[i]);
    }
    for (int i = K - 1; i >= 0; --i) {
      suf[i] = (i % m == m - 1 || i == K - 1) ? v[i] : pick(suf[i + 1], v[i]);
      s0[i] = i == K - 1 ? v[i] : pick(s0[i + 1], v[i]);
    }
    for (int b = 0; b < K; ++b) {
      const int l = b - r, h = b + r;
      if (l <= 0)
        out[b] = p0[h < K - 1 ? h : K - 1];
      else if (h >= K - 1)
        out[b] = s0[l];
      else
        out[b] = pick(suf[l], pre[h]);  // [l, h] spans one block or two adjacent ones
    }
    return out;
  };
  std::vector<int64_t> bmin(kLpBuckets), bmax(kLpBuckets);
  for (int b = 0; b < kLpBuckets; ++b) {
    const bool has = he[1 + b] != kEmpty;
    bmin[b] = has ? signed_of(he[1 + b]) : kNone;
    bmax[b] = has ? signed_of(he[1 + kLpBuckets + b]) : -kNone;
  }
  const std::vector<int64_t> nmin = sliding(bmin, false), nmax = sliding(bmax, true);
  std::vector<int64_t> w(2 * (size_t)kLpBuckets);
  for (int b = 0; b < kLpBuckets; ++b) {
    const bool seen = nmin[b] != kNone;
    const int64_t lo = seen ? nmin[b] : all_lo, hi = seen ? nmax[b] : all_hi;
    const int64_t pad = (hi - lo) / 8 + noise;
    w[2 * b] = lo - pad;
    w[2 * b + 1] = hi + pad;
  }
  if (max_err) *max_err = (int64_t)he[0];
  return lp_install_windows(h, w, 0);
}

mp_status mp_partition_learned(mp_lp h, mp_dtype kt, const void *A, int64_t na, const void *B,
                               int64_t nb, const int64_t *diag, int64_t n_diag, int64_t *a_split,
                               uint64_t *n_fallback, void *stream) {
  if (!h) return lp_fail(MP_ERR_INVALID_ARG, "mp_partition_learned: NULL handle");
  if (h->window < 0) return lp_fail(MP_ERR_STATE, "mp_partition_learned: window not set (calibrate first)");
  if (!lp_valid_key(kt)) return lp_fail(MP_ERR_UNSUPPORTED, "mp_partition_learned: unsupported key dtype");
  if (na < 0 || nb < 0 || n_diag < 0 || (na && !A) || (nb && !B) || (n_diag && (!diag || !a_split)))
    return lp_fail(MP_ERR_INVALID_ARG, "mp_partition_learned: bad arguments");
  if (n_diag == 0) return MP_OK;
  hipStream_t s = (hipStream_t)stream;
  KernelTimer timer("partition_learned", s);
  const int g = partition_lanes(n_diag);
  const unsigned blocks = (unsigned)((n_diag * g + 255) / 256);
  dispatch_key(kt, [&](auto k) {
    using KT = decltype(k);
    const int64_t *wt = h->windows.empty() ? nullptr : (const int64_t *)h->d_windows;
    auto go = [&](auto kernel) {
      hipLaunchKernelGGL(kernel, dim3(blocks), dim3(256), 0, s, (const float *)h->params, h->F,
                         h->H, h->window, wt, (const KT *)A, na, (const KT *)B, nb, diag, n_diag,
                         a_split, (unsigned long long *)n_fallback);
    };
    // the default model shape (5 inputs, 32 hidden units) is compiled in
    auto by_shape = [&](auto gc) {
      constexpr int G = decltype(gc)::value;
      if (h->F == 5 && h->H == 32) go(learned_partition_kernel<KT, G, 5, 32>);
      else go(learned_partition_kernel<KT, G, 0, 0>);
    };
    switch (g) {
      case 2: by_shape(std::integral_constant<int, 2>()); break;
      case 4: by_shape(std::integral_constant<int, 4>()); break;
      case 8: by_shape(std::integral_constant<int, 8>()); break;
      case 16: by_shape(std::integral_constant<int, 16>()); break;
      case 32: by_shape(std::integral_constant<int, 32>()); break;
      case 64: by_shape(std::integral_constant<int, 64>()); break;
      default: by_shape(std::integral_constant<int, 1>());
    }
  });
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? MP_OK : lp_hip(e, "mp_partition_learned launch");
}

// File format (little endian): "MPLP" magic, u32 version, i32 F, i32 H,
// i64 window, u64 seed, then F*H + 2H + 1 float32 parameters; version 3
// appends i32 n and n (lo, hi) i64 offset pairs (n = 0 or kLpBuckets).
// Older files still load: version 1 has one window, version 2 appends i32 n
// and n i64 symmetric windows over kLpOldBuckets buckets (each covers
// kLpBuckets / kLpOldBuckets of today's buckets exactly, since both divide
// [0, N] the same way).
mp_status mp_lp_save(mp_lp h, const char *path) {
  if (!h || !path) return lp_fail(MP_ERR_INVALID_ARG, "mp_lp_save: bad arguments");
  const int P = lp_num_params(h->F, h->H);
  std::vector<float> p(P);
  hipError_t e = hipMemcpy(p.data(), h->params, P * sizeof(float), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return lp_hip(e, "mp_lp_save");
  FILE *f = fopen(path, "wb");
  if (!f) return lp_fail(MP_ERR_INVALID_ARG, "mp_lp_save: cannot open file");
  const uint32_t ver = 3;
  const int32_t nw = (int32_t)(h->windows.size() / 2);
  bool ok = fwrite("MPLP", 1, 4, f) == 4 && fwrite(&ver, 4, 1, f) == 1 &&
            fwrite(&h->F, 4, 1, f) == 1 && fwrite(&h->H, 4, 1, f) == 1 &&
            fwrite(&h->window, 8, 1, f) == 1 && fwrite(&h->seed, 8, 1, f) == 1 &&
            fwrite(p.data(), sizeof(float), P, f) == (size_t)P && fwrite(&nw, 4, 1, f) == 1 &&
            (nw == 0 || fwrite(h->windows.data(), 8, 2 * (size_t)nw, f) == 2 * (size_t)nw);
  ok = (fclose(f) == 0) && ok;
  return ok ? MP_OK : lp_fail(MP_ERR_INVALID_ARG, "mp_lp_save: write failed");
}

mp_status mp_lp_load(mp_lp *out, const char *path) {
  if (!out || !path) return lp_fail(MP_ERR_INVALID_ARG, "mp_lp_load: bad arguments");
  *out = nullptr;
  FILE *f = fopen(path, "rb");
  if (!f) return lp_fail(MP_ERR_INVALID_ARG, "mp_lp_load: cannot open file");
  char magic[4];
  uint32_t ver = 0;
  int F = 0, H = 0;
  int64_t window = -1;
  uint64_t seed = 0;
  bool ok = fread(magic, 1, 4, f) == 4 && !memcmp(magic, "MPLP", 4) && fread(&ver, 4, 1, f) == 1 &&
            (ver >= 1 && ver <= 3) && fread(&F, 4, 1, f) == 1 && fread(&H, 4, 1, f) == 1 &&
            fread(&window, 8, 1, f) == 1 && fread(&seed, 8, 1, f) == 1 &&
            (F == 1 || F == 3 || F == 5) && H >= 1 && H <= kLpMaxHidden;
  std::vector<float> p;
  std::vector<int64_t> wt;
  if (ok) {
    p.resize(lp_num_params(F, H));
    ok = fread(p.data(), sizeof(float), p.size(), f) == p.size();
  }
  int32_t nw = 0;
  if (ok && ver >= 2) ok = fread(&nw, 4, 1, f) == 1;
  if (ok && ver == 2 && nw != 0) {
    std::vector<int64_t> old(kLpOldBuckets);
    ok = nw == kLpOldBuckets && fread(old.data(), 8, old.size(), f) == old.size();
    for (size_t i = 0; ok && i < old.size(); ++i) ok = old[i] >= 0;
    if (ok) {
      constexpr int rep = kLpBuckets / kLpOldBuckets;
      wt.resize(2 * (size_t)kLpBuckets);
      for (int b = 0; b < kLpBuckets; ++b) {
        wt[2 * b] = -old[b / rep];
        wt[2 * b + 1] = old[b / rep];
      }
    }
  }
  if (ok && ver == 3 && nw != 0) {
    wt.resize(2 * (size_t)kLpBuckets);
    ok = nw == kLpBuckets && fread(wt.data(), 8, wt.size(), f) == wt.size();
    for (int b = 0; ok && b < kLpBuckets; ++b) ok = wt[2 * b] <= wt[2 * b + 1];
  }
  fclose(f);
  if (!ok) return lp_fail(MP_ERR_STATE, "mp_lp_load: not a model file of this format");
  mp_lp h = nullptr;
  mp_status st = mp_lp_create(&h, H, F, seed);
  if (st != MP_OK) return st;
  st = mp_lp_set_params(h, p.data(), (int)p.size());
  if (st != MP_OK) {
    mp_lp_destroy(h);
    return st;
  }
  st = lp_install_windows(h, wt, window);
  if (st != MP_OK) {
    mp_lp_destroy(h);
    return st;
  }
  *out = h;
  return MP_OK;
}

}  // extern "C"
