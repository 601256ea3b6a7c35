// gfx950 kernels of the sFFT4.0 hot path.
//
//   fold_kernel        HashToBins part 1 (Sec. 2.4, Lemma 1): permuted gather
//                      x[sigma (t - T) mod N], window G_t, alias t -> t mod B.
//   bucket_fft_kernel  HashToBins part 2: B-point DFT with the 1/N factor.
//   recover_kernel     one iteration loop per signal (Sec. 3.1-3.2):
//                      subtraction, detection, multiscale location,
//                      verification, median estimation (Eq. 14), dedupe,
//                      accumulation, and the final top-K.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace sfft {

template <typename R>
struct alignas(2 * sizeof(R)) cplx {
  R re, im;
};

template <typename R>
__device__ __forceinline__ cplx<R> cmul(cplx<R> a, cplx<R> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename R>
__device__ __forceinline__ cplx<R> cadd(cplx<R> a, cplx<R> b) {
  return {a.re + b.re, a.im + b.im};
}
template <typename R>
__device__ __forceinline__ cplx<R> csub(cplx<R> a, cplx<R> b) {
  return {a.re - b.re, a.im - b.im};
}
template <typename R>
__device__ __forceinline__ cplx<R> cscale(cplx<R> a, R s) {
  return {a.re * s, a.im * s};
}

// exp(sign * 2 pi i p / N) for an exact phase index p in [0, N).  Shifting p
// to the top of a 32-bit word gives the phase as a signed fixed-point
// fraction of a turn, so the argument handed to sincospi lies in [-1, 1).
__device__ __forceinline__ cplx<float> expi_index(uint32_t p, uint32_t logN, float sign) {
  const int32_t ps = int32_t(p << (32 - logN));
  const float x = float(ps) * 0x1p-30f;  // 2 p / N, reduced to [-1, 1)
  float s, c;
  sincospif(x, &s, &c);
  return {c, sign * s};
}
__device__ __forceinline__ cplx<double> expi_index_d(uint32_t p, uint32_t logN, double sign) {
  const int32_t ps = int32_t(p << (32 - logN));
  const double x = double(ps) * 0x1p-30;
  double s, c;
  sincospi(x, &s, &c);
  return {c, sign * s};
}
template <typename R>
__device__ __forceinline__ cplx<R> expi(uint32_t p, uint32_t logN, R sign);
template <>
__device__ __forceinline__ cplx<float> expi<float>(uint32_t p, uint32_t logN, float sign) {
  return expi_index(p, logN, sign);
}
template <>
__device__ __forceinline__ cplx<double> expi<double>(uint32_t p, uint32_t logN, double sign) {
  return expi_index_d(p, logN, sign);
}

// ------------------------------------------------------------------------
// Sample loaders.
// ------------------------------------------------------------------------
struct LoadC64 {
  using R = float;
  static constexpr bool kScaled = false;
  static __device__ __forceinline__ cplx<float> load(const void* x, uint32_t i) {
    return reinterpret_cast<const cplx<float>*>(x)[i];
  }
};
struct LoadC128 {
  using R = double;
  static constexpr bool kScaled = false;
  static __device__ __forceinline__ cplx<double> load(const void* x, uint32_t i) {
    return reinterpret_cast<const cplx<double>*>(x)[i];
  }
};
struct LoadF16 {
  using R = float;
  static constexpr bool kScaled = true;
  typedef _Float16 h2 __attribute__((ext_vector_type(2)));
  static __device__ __forceinline__ cplx<float> load(const void* x, uint32_t i) {
    const h2 v = reinterpret_cast<const h2*>(x)[i];
    return {float(v.x), float(v.y)};
  }
};

// ------------------------------------------------------------------------
// Fold: y_j[b] = sum_{|t| <= h, t = b mod B} G_t x[sigma (t - T_j) mod N].
// One thread owns one bucket b and walks its taps t = t_first + k B; the
// sample index advances by sigma B mod N per tap.  All index arithmetic is
// uint32 with wrap-around, exact because N divides 2^32.
// ------------------------------------------------------------------------
template <typename R, bool KAHAN>
struct Acc {
  R re = 0, im = 0, cre = 0, cim = 0;
  __device__ __forceinline__ void add(R g, cplx<R> s) {
    if (KAHAN) {
      R yr = g * s.re - cre;
      R tr = re + yr;
      cre = (tr - re) - yr;
      re = tr;
      R yi = g * s.im - cim;
      R ti = im + yi;
      cim = (ti - im) - yi;
      im = ti;
    } else {
      re += g * s.re;
      im += g * s.im;
    }
  }
};

template <class Ld, bool KAHAN>
__global__ __launch_bounds__(kFoldTile) void fold_kernel(const SignalDesc* __restrict__ sigs,
                                                         const FoldTile* __restrict__ tiles) {
  using R = typename Ld::R;
  const FoldTile tl = tiles[blockIdx.x];
  const SignalDesc* sd = sigs + tl.sig;
  const PlanDesc* pd = sd->plan;
  const IterDesc* it = pd->iters + tl.m;
  const uint32_t B = it->B;
  const uint32_t b = tl.b0 + threadIdx.x;
  if (b >= B) return;
  const uint32_t nmask = pd->N - 1;
  const int32_t h = int32_t(it->h);
  const uint32_t T = it->T[tl.j];
  const uint32_t sigma = it->sigma;
  const R* __restrict__ G = reinterpret_cast<const R*>(pd->window) + it->win_off;
  const void* x = sd->x;
  // first tap t = b (mod B) with t >= -h; B <= w guarantees t_first <= h
  const int32_t tf = -h + int32_t((b + uint32_t(h)) & (B - 1));
  const uint32_t ntaps = uint32_t(h - tf) / B + 1;
  uint32_t idx = (sigma * (uint32_t(tf) - T)) & nmask;
  const uint32_t step = (sigma * B) & nmask;
  Acc<R, KAHAN> acc;
  int32_t t = tf;
  uint32_t k = 0;
  constexpr int U = 8;
  for (; k + U <= ntaps; k += U) {
    cplx<R> s[U];
    R g[U];
#pragma unroll
    for (int q = 0; q < U; ++q) {
      s[q] = Ld::load(x, idx);
      const int32_t tt = t + q * int32_t(B);
      g[q] = G[tt < 0 ? -tt : tt];
      idx = (idx + step) & nmask;
    }
#pragma unroll
    for (int q = 0; q < U; ++q) acc.add(g[q], s[q]);
    t += U * int32_t(B);
  }
  for (; k < ntaps; ++k) {
    const cplx<R> s = Ld::load(x, idx);
    acc.add(G[t < 0 ? -t : t], s);
    idx = (idx + step) & nmask;
    t += int32_t(B);
  }
  cplx<R> out{acc.re, acc.im};
  if (Ld::kScaled) out = cscale(out, R(sd->scale));
  cplx<R>* Y = reinterpret_cast<cplx<R>*>(sd->y) + it->y_off + size_t(tl.j) * B;
  Y[b] = out;
}

// ------------------------------------------------------------------------
// Bucket DFT: yhat_j[i] = (1/N) sum_b y_j[b] exp(-2 pi i i b / B), in place.
// Radix-2 decimation in time on an LDS copy (bit-reversed load).
// ------------------------------------------------------------------------
template <typename R>
__global__ __launch_bounds__(256) void bucket_fft_kernel(const SignalDesc* __restrict__ sigs,
                                                         const RoundItem* __restrict__ items) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  cplx<R>* X = reinterpret_cast<cplx<R>*>(smem_raw);
  const RoundItem itm = items[blockIdx.x];
  const SignalDesc* sd = sigs + itm.sig;
  const PlanDesc* pd = sd->plan;
  const IterDesc* it = pd->iters + itm.m;
  const uint32_t B = it->B, logB = it->logB;
  cplx<R>* Y = reinterpret_cast<cplx<R>*>(sd->y) + it->y_off + size_t(itm.j) * B;
  const cplx<R>* tw = reinterpret_cast<const cplx<R>*>(pd->twiddle) + it->tw_off;
  for (uint32_t b = threadIdx.x; b < B; b += blockDim.x) X[__brev(b) >> (32 - logB)] = Y[b];
  __syncthreads();
  for (uint32_t s = 1; s <= logB; ++s) {
    const uint32_t half = 1u << (s - 1);
    for (uint32_t k = threadIdx.x; k < B / 2; k += blockDim.x) {
      const uint32_t pos = k & (half - 1);
      const uint32_t i0 = ((k >> (s - 1)) << s) + pos, i1 = i0 + half;
      const cplx<R> w = tw[pos << (logB - s)];
      const cplx<R> a = X[i0], c = cmul(w, X[i1]);
      X[i0] = cadd(a, c);
      X[i1] = csub(a, c);
    }
    __syncthreads();
  }
  const R inv = R(1) / R(pd->N);
  for (uint32_t i = threadIdx.x; i < B; i += blockDim.x) Y[i] = cscale(X[i], inv);
}

// ------------------------------------------------------------------------
// Workgroup primitives of the recovery kernel (1024 threads).
// ------------------------------------------------------------------------
constexpr int kRecThreads = 1024;
constexpr uint32_t kNone = 0xFFFFFFFFu;

struct K128 {
  uint64_t hi, lo;
};
__device__ __forceinline__ bool key_less(uint64_t a, uint64_t b) { return a < b; }
__device__ __forceinline__ bool key_less(const K128& a, const K128& b) {
  return a.hi < b.hi || (a.hi == b.hi && a.lo < b.lo);
}

// Ascending bitonic sort of n (a power of two) keys by the whole block.
template <typename Key>
__device__ void block_bitonic_sort(Key* keys, uint32_t n) {
  for (uint32_t k = 2; k <= n; k <<= 1) {
    for (uint32_t j = k >> 1; j > 0; j >>= 1) {
      for (uint32_t p = threadIdx.x; p < n / 2; p += blockDim.x) {
        const uint32_t lo = p & (j - 1);
        const uint32_t i = ((p - lo) << 1) + lo, ixj = i + j;
        const Key a = keys[i], b = keys[ixj];
        const bool up = (i & k) == 0;
        if (up ? key_less(b, a) : key_less(a, b)) {
          keys[i] = b;
          keys[ixj] = a;
        }
      }
      __syncthreads();
    }
  }
}

// In-place exclusive prefix sum of a[0..n) by the whole block; returns the total.
__device__ uint32_t block_scan_exclusive(uint32_t* a, uint32_t n, uint32_t* sh) {
  const uint32_t T = blockDim.x, tid = threadIdx.x;
  const uint32_t chunk = (n + T - 1) / T;
  const uint32_t lo = min(n, tid * chunk), hi = min(n, lo + chunk);
  uint32_t s = 0;
  for (uint32_t i = lo; i < hi; ++i) s += a[i];
  sh[tid] = s;
  __syncthreads();
  for (uint32_t off = 1; off < T; off <<= 1) {
    const uint32_t v = tid >= off ? sh[tid - off] : 0u;
    __syncthreads();
    sh[tid] += v;
    __syncthreads();
  }
  const uint32_t total = sh[T - 1];
  uint32_t run = tid ? sh[tid - 1] : 0u;
  for (uint32_t i = lo; i < hi; ++i) {
    const uint32_t v = a[i];
    a[i] = run;
    run += v;
  }
  __syncthreads();
  return total;
}

template <typename V>
__device__ V block_reduce_max(V v, V* sh) {
  for (int off = 32; off > 0; off >>= 1) {
    V o = __shfl_xor(v, off, 64);
    v = v > o ? v : o;
  }
  const uint32_t wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  V r = sh[0];
  for (uint32_t w = 1; w < blockDim.x / 64; ++w) r = r > sh[w] ? r : sh[w];
  __syncthreads();
  return r;
}

__device__ uint32_t block_reduce_sum(uint32_t v, uint32_t* sh) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const uint32_t wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  uint32_t r = 0;
  for (uint32_t w = 0; w < blockDim.x / 64; ++w) r += sh[w];
  __syncthreads();
  return r;
}

__device__ __forceinline__ int64_t floor_div(int64_t a, int64_t b) {  // b > 0
  return a >= 0 ? a / b : -((-a + b - 1) / b);
}

// Lower bound in an ascending uint32 array.
__device__ __forceinline__ uint32_t lower_bound_u32(const uint32_t* a, uint32_t n, uint32_t v) {
  uint32_t lo = 0, hi = n;
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    if (a[mid] < v) lo = mid + 1; else hi = mid;
  }
  return lo;
}
__device__ __forceinline__ uint32_t lower_bound_u64(const uint64_t* a, uint32_t n, uint64_t v) {
  uint32_t lo = 0, hi = n;
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    if (a[mid] < v) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// Circular distance between two binary angles (2^64 = one turn).
__device__ __forceinline__ uint64_t angle_dist(uint64_t a, uint64_t b) {
  const uint64_t d = a - b;
  const uint64_t e = b - a;
  return d < e ? d : e;
}

// theta_j = arg(yhat_0 conj(yhat_j)) (Eq. 15-16, sign read so that theta_j =
// 2 pi (tau_j u mod N) / N) as a binary angle.
template <typename R>
__device__ __forceinline__ uint64_t theta_bin(cplx<R> y0, cplx<R> yj, bool fp64) {
  double turns;
  if (fp64 || sizeof(R) == 8) {
    const double zr = double(y0.re) * double(yj.re) + double(y0.im) * double(yj.im);
    const double zi = double(y0.im) * double(yj.re) - double(y0.re) * double(yj.im);
    turns = atan2(zi, zr) * 0.15915494309189533577;  // 1 / (2 pi)
  } else {
    const float zr = float(y0.re) * float(yj.re) + float(y0.im) * float(yj.im);
    const float zi = float(y0.im) * float(yj.re) - float(y0.re) * float(yj.im);
    turns = double(atan2f(zi, zr) * 0.159154943f);
  }
  if (turns < 0.0) turns += 1.0;
  const double t64 = turns * 18446744073709551616.0;
  if (!(t64 < 18446744073709551616.0)) return 0;
  return uint64_t(t64);
}

// Phase of position p seen through multiplier tau: (p tau mod N) / N turns.
__device__ __forceinline__ uint64_t pos_angle(uint64_t p, uint64_t tau, uint32_t logN) {
  return ((p * tau) & ((uint64_t(1) << logN) - 1)) << (64 - logN);
}

// Multiscale location (Sec. 3.2) of the lone coefficient of bucket i and its
// verification.  Returns kNone if rejected, else u; *dist = |iL - u|_N.
template <typename R>
__device__ uint32_t locate_bucket(const PlanDesc* pd, const IterDesc* it, const cplx<R>* Y, uint32_t i,
                                  uint32_t* dist) {
  const uint32_t B = it->B, L = it->L, R_ = it->R, logN = pd->logN, nmask = pd->N - 1;
  const bool fp64 = pd->fp64_phase != 0;
  const cplx<R> y0 = Y[i];
  const uint32_t l = pd->l, logM2 = 1 + pd->logl + logN;
  const uint64_t m2mask = (uint64_t(1) << logM2) - 1;
  const uint32_t sh = 64 - logM2;
  const uint32_t den_shift = 1 + pd->logqd + pd->logl;
  const int64_t qd = int64_t(1) << pd->logqd, qn = pd->qn;
  int64_t a = int64_t(i) * L - int64_t(L / 2) - int64_t(it->e);
  uint32_t u = 0;
  for (uint32_t j = 1; j <= R_; ++j) {
    const uint64_t th = theta_bin(y0, Y[size_t(j) * B + i], fp64);
    const uint64_t len = it->len[j], tau = it->tau[j];
    if (j < R_) {
      // block step: centre of block b is a + (b + 1/2) len / l; its phase is
      // ((2 l a + (2b+1) len) tau mod 2lN) / 2lN turns
      const uint64_t A = uint64_t(int64_t(2 * l) * a);
      uint32_t best_b = 0;
      uint64_t best_d = ~uint64_t(0);
      for (uint32_t b = 0; b < l; ++b) {
        const uint64_t num = ((A + uint64_t(2 * b + 1) * len) * tau) & m2mask;
        const uint64_t d = angle_dist(num << sh, th);
        if (d < best_d) {
          best_d = d;
          best_b = b;
        }
      }
      // new region starts q/2 blocks before the chosen block (floor)
      const int64_t num = (2 * int64_t(best_b) * qd - qn) * int64_t(len);
      a += num >> den_shift;
    } else {
      // last step: the single position of the region closest in phase
      int64_t best_c = a;
      uint64_t best_d = ~uint64_t(0);
      for (uint64_t c = 0; c < len; ++c) {
        const uint64_t d = angle_dist(pos_angle(uint64_t(a + int64_t(c)), tau, logN), th);
        if (d < best_d) {
          best_d = d;
          best_c = a + int64_t(c);
        }
      }
      u = uint32_t(uint64_t(best_c) & nmask);
    }
  }
  // verification: within reach of the bucket centre, and every round's
  // phase within pi / l of the located position (Eq. 18)
  const uint32_t d1 = (i * L - u) & nmask;
  const uint32_t dd = min(d1, pd->N - d1);
  if (dd > it->D) return kNone;
  const uint64_t tol = uint64_t(1) << (63 - pd->logl);
  for (uint32_t j = 1; j <= R_; ++j) {
    const uint64_t th = theta_bin(y0, Y[size_t(j) * B + i], fp64);
    if (angle_dist(pos_angle(u, it->tau[j], logN), th) > tol) return kNone;
  }
  *dist = dd;
  return u;
}

// Median of n values (mean of the two middle values when n is even).
template <typename R>
__device__ R median_small(R* v, uint32_t n) {
  for (uint32_t a = 1; a < n; ++a) {
    const R x = v[a];
    uint32_t b = a;
    while (b > 0 && v[b - 1] > x) {
      v[b] = v[b - 1];
      --b;
    }
    v[b] = x;
  }
  return (n & 1) ? v[n / 2] : (v[n / 2 - 1] + v[n / 2]) * R(0.5);
}

template <typename R>
__device__ __forceinline__ uint64_t real_bits(R v);
template <>
__device__ __forceinline__ uint64_t real_bits<float>(float v) {
  return uint64_t(__float_as_uint(v));
}
template <>
__device__ __forceinline__ uint64_t real_bits<double>(double v) {
  return uint64_t(__double_as_longlong(v));
}
template <typename R>
__device__ __forceinline__ R real_from_bits(uint64_t v);
template <>
__device__ __forceinline__ float real_from_bits<float>(uint64_t v) {
  return __uint_as_float(uint32_t(v));
}
template <>
__device__ __forceinline__ double real_from_bits<double>(uint64_t v) {
  return __longlong_as_double(int64_t(v));
}

// Top-K key: descending magnitude, ties to the smaller frequency.
template <typename R>
struct TopKey;
template <>
struct TopKey<float> {
  using T = uint64_t;
  static __device__ __forceinline__ T make(float mag2, uint32_t f) {
    return (uint64_t(~__float_as_uint(mag2)) << 32) | f;
  }
  static __device__ __forceinline__ T none() { return ~uint64_t(0); }
};
template <>
struct TopKey<double> {
  using T = K128;
  static __device__ __forceinline__ T make(double mag2, uint32_t f) {
    return K128{~uint64_t(__double_as_longlong(mag2)), uint64_t(f)};
  }
  static __device__ __forceinline__ T none() { return K128{~uint64_t(0), ~uint64_t(0)}; }
};
__device__ __forceinline__ bool key_eq(uint64_t a, uint64_t b) { return a == b; }
__device__ __forceinline__ bool key_eq(const K128& a, const K128& b) { return a.hi == b.hi && a.lo == b.lo; }

template <typename R>
__global__ __launch_bounds__(kRecThreads) void recover_kernel(const SignalDesc* __restrict__ sigs) {
  __shared__ uint32_t sh_scan[kRecThreads];
  __shared__ R sh_red[kRecThreads / 64];
  __shared__ uint32_t sh_ured[kRecThreads / 64];
  const uint32_t tid = threadIdx.x, NT = blockDim.x;
  const SignalDesc* sd = sigs + blockIdx.x;
  const PlanDesc* pd = sd->plan;
  unsigned char* ws = reinterpret_cast<unsigned char*>(sd->ws);
  cplx<R>* Yall = reinterpret_cast<cplx<R>*>(sd->y);
  uint32_t* recf[2] = {reinterpret_cast<uint32_t*>(ws + pd->off_recf0), reinterpret_cast<uint32_t*>(ws + pd->off_recf1)};
  cplx<R>* recv[2] = {reinterpret_cast<cplx<R>*>(ws + pd->off_recv0), reinterpret_cast<cplx<R>*>(ws + pd->off_recv1)};
  uint32_t* cand_u = reinterpret_cast<uint32_t*>(ws + pd->off_candu);
  uint32_t* cand_d = reinterpret_cast<uint32_t*>(ws + pd->off_candd);
  cplx<R>* cand_v = reinterpret_cast<cplx<R>*>(ws + pd->off_candv);
  uint32_t* pairs = reinterpret_cast<uint32_t*>(ws + pd->off_pairs);
  uint32_t* cnt = reinterpret_cast<uint32_t*>(ws + pd->off_cnt);
  uint32_t* start = reinterpret_cast<uint32_t*>(ws + pd->off_start);
  uint64_t* keys = reinterpret_cast<uint64_t*>(ws + pd->off_keys);
  R* p0 = reinterpret_cast<R*>(ws + pd->off_p0);
  const uint32_t N = pd->N, nmask = N - 1, logN = pd->logN;
  uint32_t nrec = 0, cur = 0;
  bool overflow = false;

  for (uint32_t m = 0; m < pd->M && !overflow; ++m) {
    const IterDesc* it = pd->iters + m;
    const uint32_t B = it->B, L = it->L, D = it->D, R1 = it->R + 1;
    cplx<R>* Y = Yall + it->y_off;
    const R* ghat = reinterpret_cast<const R*>(pd->ghat) + it->ghat_off;
    const uint32_t sigma = it->sigma;

    // ---- subtraction of the coefficients recovered so far (Sec. 3.1) ----
    if (nrec > 0) {
      for (uint32_t i = tid; i < B; i += NT) cnt[i] = 0;
      __syncthreads();
      for (uint32_t k = tid; k < nrec; k += NT) {
        const int64_t u = int64_t((sigma * recf[cur][k]) & nmask);
        const int64_t lo = -floor_div(int64_t(D) - u, L), hi = floor_div(u + int64_t(D), L);
        for (int64_t i = lo; i <= hi; ++i) atomicAdd(&cnt[uint32_t(i) & (B - 1)], 1u);
      }
      __syncthreads();
      for (uint32_t i = tid; i < B; i += NT) start[i] = cnt[i];
      __syncthreads();
      block_scan_exclusive(start, B, sh_scan);
      for (uint32_t i = tid; i < B; i += NT) cnt[i] = 0;
      __syncthreads();
      for (uint32_t k = tid; k < nrec; k += NT) {
        const int64_t u = int64_t((sigma * recf[cur][k]) & nmask);
        const int64_t lo = -floor_div(int64_t(D) - u, L), hi = floor_div(u + int64_t(D), L);
        for (int64_t i = lo; i <= hi; ++i) {
          const uint32_t ii = uint32_t(i) & (B - 1);
          pairs[start[ii] + atomicAdd(&cnt[ii], 1u)] = k;
        }
      }
      __syncthreads();
      for (uint32_t i = tid; i < B; i += NT) {
        const uint32_t n = cnt[i], s0 = start[i];
        // entries in ascending index (= ascending frequency) order
        for (uint32_t a = 1; a < n; ++a) {
          const uint32_t v = pairs[s0 + a];
          uint32_t b = a;
          while (b > 0 && pairs[s0 + b - 1] > v) {
            pairs[s0 + b] = pairs[s0 + b - 1];
            --b;
          }
          pairs[s0 + b] = v;
        }
        for (uint32_t q = 0; q < n; ++q) {
          const uint32_t k = pairs[s0 + q];
          const uint32_t u = (sigma * recf[cur][k]) & nmask;
          const uint32_t d1 = (i * L - u) & nmask;
          const uint32_t dd = min(d1, N - d1);
          const cplx<R> vg = cscale(recv[cur][k], ghat[dd]);
          for (uint32_t j = 0; j < R1; ++j) {
            const uint32_t p = (it->T[j] * u) & nmask;
            cplx<R>& y = Y[size_t(j) * B + i];
            y = csub(y, cmul(vg, expi<R>(p, logN, R(-1))));
          }
        }
      }
      __syncthreads();
    }

    // ---- singleton detection ----
    R mx = 0;
    for (uint32_t i = tid; i < B; i += NT) {
      const cplx<R> y0 = Y[i];
      const R p = y0.re * y0.re + y0.im * y0.im;
      p0[i] = p;
      keys[i] = real_bits<R>(p);
      mx = p > mx ? p : mx;
      const R m0 = sqrt(p);
      uint32_t cons = 1;
      for (uint32_t j = 1; j < R1; ++j) {
        const cplx<R> yj = Y[size_t(j) * B + i];
        const R mj = sqrt(yj.re * yj.re + yj.im * yj.im);
        if (fabs(mj - m0) > R(pd->rho) * m0) cons = 0;
      }
      cand_u[i] = cons;
    }
    mx = block_reduce_max(mx, sh_red);
    block_bitonic_sort(keys, B);
    const R med = (real_from_bits<R>(keys[B / 2 - 1]) + real_from_bits<R>(keys[B / 2])) * R(0.5);
    const R nu = med / R(0.69314718055994530942);
    const R thr_noise = R(2.0 * it->log_B) * nu;
    const R thr_floor = R(pd->eta * pd->eta) * mx;
    const R thr = thr_noise > thr_floor ? thr_noise : thr_floor;
    __syncthreads();

    // ---- location, verification, median estimation ----
    for (uint32_t i = tid; i < B; i += NT) {
      uint32_t uo = kNone;
      const R p = p0[i];
      if (cand_u[i] && p >= thr && p > R(0)) {
        uint32_t dd = 0;
        const uint32_t u = locate_bucket<R>(pd, it, Y, i, &dd);
        const R g = u != kNone ? ghat[dd] : R(0);
        if (u != kNone && g != R(0)) {
          R er[kMaxRounds], ei[kMaxRounds];
          for (uint32_t j = 0; j < R1; ++j) {
            const uint32_t ph = (it->T[j] * u) & nmask;
            const cplx<R> e = cmul(Y[size_t(j) * B + i], expi<R>(ph, logN, R(1)));
            er[j] = e.re / g;
            ei[j] = e.im / g;
          }
          cand_v[i] = cplx<R>{median_small(er, R1), median_small(ei, R1)};
          cand_d[i] = dd;
          uo = u;
        }
      }
      cand_u[i] = uo;
    }
    __syncthreads();

    // ---- dedupe: one candidate per position, nearest bucket centre wins ----
    for (uint32_t i = tid; i < B; i += NT) {
      const uint32_t u = cand_u[i];
      uint32_t keep = 0;
      if (u != kNone) {
        keep = 1;
        const uint32_t d = cand_d[i];
        for (uint32_t dd = 1; dd <= it->reach && keep; ++dd) {
          const uint32_t nb[2] = {(i - dd) & (B - 1), (i + dd) & (B - 1)};
          for (int s = 0; s < 2; ++s) {
            const uint32_t i2 = nb[s];
            if (i2 != i && cand_u[i2] == u && (cand_d[i2] < d || (cand_d[i2] == d && i2 < i))) keep = 0;
          }
        }
      }
      cnt[i] = keep;
      start[i] = keep;
    }
    __syncthreads();
    const uint32_t nsurv = block_scan_exclusive(cnt, B, sh_scan);
    uint32_t npow = 1;
    while (npow < nsurv) npow <<= 1;
    for (uint32_t i = tid; i < B; i += NT) {
      if (start[i]) {
        const uint32_t f = (it->sigma_inv * cand_u[i]) & nmask;
        keys[cnt[i]] = (uint64_t(f) << 32) | i;
      }
    }
    for (uint32_t c = nsurv + tid; c < npow; c += NT) keys[c] = ~uint64_t(0);
    __syncthreads();
    if (nsurv > 1) block_bitonic_sort(keys, npow);

    // ---- accumulate into the sorted store: rec[f] += v (Sec. 3.1 step 5) ----
    const uint32_t* of = recf[cur];
    const cplx<R>* ov = recv[cur];
    uint32_t* nf = recf[cur ^ 1];
    cplx<R>* nv = recv[cur ^ 1];
    for (uint32_t c = tid; c < nsurv; c += NT) {
      const uint32_t f = uint32_t(keys[c] >> 32);
      const uint32_t pos = lower_bound_u32(of, nrec, f);
      pairs[c] = (pos < nrec && of[pos] == f) ? 0u : 1u;
    }
    __syncthreads();
    const uint32_t nnew = block_scan_exclusive(pairs, nsurv, sh_scan);
    if (nrec + nnew > pd->rec_cap) {
      overflow = true;
      break;
    }
    for (uint32_t k = tid; k < nrec; k += NT) {
      const uint32_t f = of[k];
      const uint32_t r = lower_bound_u64(keys, nsurv, uint64_t(f) << 32);
      const uint32_t newbefore = r < nsurv ? pairs[r] : nnew;
      cplx<R> v = ov[k];
      if (r < nsurv && uint32_t(keys[r] >> 32) == f) v = cadd(v, cand_v[uint32_t(keys[r])]);
      nf[k + newbefore] = f;
      nv[k + newbefore] = v;
    }
    for (uint32_t c = tid; c < nsurv; c += NT) {
      const uint32_t f = uint32_t(keys[c] >> 32);
      const uint32_t pos = lower_bound_u32(of, nrec, f);
      if (!(pos < nrec && of[pos] == f)) {
        nf[pos + pairs[c]] = f;
        nv[pos + pairs[c]] = cand_v[uint32_t(keys[c])];
      }
    }
    __syncthreads();
    nrec += nnew;
    cur ^= 1;
  }

  if (overflow) {
    if (tid == 0) *sd->count = -1;
    return;
  }

  // ---- top-K by magnitude, ties to the smaller frequency; output sorted by f ----
  using Key = typename TopKey<R>::T;
  Key* tk = reinterpret_cast<Key*>(keys);
  uint32_t npow = 1;
  while (npow < nrec) npow <<= 1;
  uint32_t nz = 0;
  for (uint32_t k = tid; k < npow; k += NT) {
    if (k < nrec) {
      const cplx<R> v = recv[cur][k];
      const R mag2 = v.re * v.re + v.im * v.im;
      tk[k] = mag2 != R(0) ? TopKey<R>::make(mag2, recf[cur][k]) : TopKey<R>::none();
      nz += mag2 != R(0);
    } else {
      tk[k] = TopKey<R>::none();
    }
  }
  nz = block_reduce_sum(nz, sh_ured);
  __syncthreads();
  if (npow > 1) block_bitonic_sort(tk, npow);
  const uint32_t Kp = min(pd->K, nz);
  if (Kp == 0) {
    if (tid == 0) *sd->count = 0;
    return;
  }
  const Key kth = tk[Kp - 1];
  __syncthreads();
  for (uint32_t k = tid; k < nrec; k += NT) {
    const cplx<R> v = recv[cur][k];
    const R mag2 = v.re * v.re + v.im * v.im;
    const Key key = TopKey<R>::make(mag2, recf[cur][k]);
    pairs[k] = (mag2 != R(0) && (key_less(key, kth) || key_eq(key, kth))) ? 1u : 0u;
  }
  __syncthreads();
  block_scan_exclusive(pairs, nrec, sh_scan);
  cplx<R>* outv = reinterpret_cast<cplx<R>*>(sd->val);
  for (uint32_t k = tid; k < nrec; k += NT) {
    const cplx<R> v = recv[cur][k];
    const R mag2 = v.re * v.re + v.im * v.im;
    const Key key = TopKey<R>::make(mag2, recf[cur][k]);
    if (mag2 != R(0) && (key_less(key, kth) || key_eq(key, kth))) {
      sd->idx[pairs[k]] = int64_t(recf[cur][k]);
      outv[pairs[k]] = v;
    }
  }
  if (tid == 0) *sd->count = int64_t(Kp);
}

// ------------------------------------------------------------------------
// Launchers.
// ------------------------------------------------------------------------
int launch_fold(int dtype, int kahan, const SignalDesc* d_sigs, const FoldTile* d_tiles, uint32_t ntiles,
                void* stream) {
  if (ntiles == 0) return hipSuccess;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  dim3 grid(ntiles), block(kFoldTile);
  if (dtype == SFFT_C128) {
    if (kahan) hipLaunchKernelGGL((fold_kernel<LoadC128, true>), grid, block, 0, s, d_sigs, d_tiles);
    else hipLaunchKernelGGL((fold_kernel<LoadC128, false>), grid, block, 0, s, d_sigs, d_tiles);
  } else if (dtype == SFFT_F16X2_SCALED) {
    if (kahan) hipLaunchKernelGGL((fold_kernel<LoadF16, true>), grid, block, 0, s, d_sigs, d_tiles);
    else hipLaunchKernelGGL((fold_kernel<LoadF16, false>), grid, block, 0, s, d_sigs, d_tiles);
  } else {
    if (kahan) hipLaunchKernelGGL((fold_kernel<LoadC64, true>), grid, block, 0, s, d_sigs, d_tiles);
    else hipLaunchKernelGGL((fold_kernel<LoadC64, false>), grid, block, 0, s, d_sigs, d_tiles);
  }
  return hipGetLastError();
}

int launch_bucket_fft(int dtype, const SignalDesc* d_sigs, const RoundItem* d_items, uint32_t nitems, uint32_t max_B,
                      void* stream) {
  if (nitems == 0) return hipSuccess;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  dim3 grid(nitems), block(256);
  if (dtype == SFFT_C128) {
    hipLaunchKernelGGL(bucket_fft_kernel<double>, grid, block, size_t(max_B) * 16, s, d_sigs, d_items);
  } else {
    hipLaunchKernelGGL(bucket_fft_kernel<float>, grid, block, size_t(max_B) * 8, s, d_sigs, d_items);
  }
  return hipGetLastError();
}

int launch_recover(int dtype, const SignalDesc* d_sigs, uint32_t nsig, void* stream) {
  if (nsig == 0) return hipSuccess;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  dim3 grid(nsig), block(kRecThreads);
  if (dtype == SFFT_C128) {
    hipLaunchKernelGGL(recover_kernel<double>, grid, block, 0, s, d_sigs);
  } else {
    hipLaunchKernelGGL(recover_kernel<float>, grid, block, 0, s, d_sigs);
  }
  return hipGetLastError();
}

}  // namespace sfft
