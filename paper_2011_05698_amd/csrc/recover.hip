// Reconstruction of one signal (Sec. 3.1-3.2), one workgroup per signal,
// iterations in order:
//   subtraction of the coefficients recovered so far (Sec. 3.1, steps 2-3),
//   singleton detection, multiscale location (Eq. 15-19) and verification,
//   median estimation (Eq. 14 per round), dedupe, accumulation
//   rec[f] += v (step 5); finally the K largest coefficients.
// Per-bucket work is one thread per bucket.  No private (scratch) arrays:
// per-bucket round values live in registers through compile-time-indexed
// sorting networks.  Counting of (coefficient, bucket) pairs uses LDS atomics.
#include "device_common.h"

namespace sfft {

constexpr int kRecThreads = 256;
constexpr int kLdsBytes = 32768;    // one buffer, reused phase by phase
constexpr uint32_t kNone = 0xFFFFFFFFu;
constexpr int kRegRounds = 16;      // rounds whose estimates are sorted in registers

struct K128 {
  uint64_t hi, lo;
};
__device__ __forceinline__ bool key_less(uint32_t a, uint32_t b) { return a < b; }
__device__ __forceinline__ bool key_less(uint64_t a, uint64_t b) { return a < b; }
__device__ __forceinline__ bool key_less(const K128& a, const K128& b) {
  return a.hi < b.hi || (a.hi == b.hi && a.lo < b.lo);
}

// Ascending bitonic sort of n keys (n a power of two) by the whole block.
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
    const V o = __shfl_xor(v, off, 64);
    v = v > o ? v : o;
  }
  if (threadIdx.x % 64 == 0) sh[threadIdx.x / 64] = v;
  __syncthreads();
  V r = sh[0];
  for (uint32_t w = 1; w < blockDim.x / 64; ++w) r = r > sh[w] ? r : sh[w];
  __syncthreads();
  return r;
}

__device__ uint32_t block_reduce_sum(uint32_t v, uint32_t* sh) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  if (threadIdx.x % 64 == 0) sh[threadIdx.x / 64] = v;
  __syncthreads();
  uint32_t r = 0;
  for (uint32_t w = 0; w < blockDim.x / 64; ++w) r += sh[w];
  __syncthreads();
  return r;
}

__device__ __forceinline__ int64_t floor_div(int64_t a, int64_t b) {  // b > 0
  return a >= 0 ? a / b : -((-a + b - 1) / b);
}

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
  const uint64_t d = a - b, e = b - a;
  return d < e ? d : e;
}

// theta_j = arg(yhat_0 conj(yhat_j)), the two-round phase difference of
// Eq. 15-16 (sign read so that theta_j = 2 pi (tau_j u mod N) / N for a lone
// coefficient at permuted position u), as a binary angle.
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
  if (!(t64 < 18446744073709551616.0) || !(t64 >= 0.0)) return 0;
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
      // block step: the centre of block b is a + (b + 1/2) len / l; its phase
      // is ((2 l a + (2b+1) len) tau mod 2lN) / 2lN turns
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
      // the new region starts q/2 blocks before the chosen block (floor)
      a += ((2 * int64_t(best_b) * qd - qn) * int64_t(len)) >> den_shift;
    } else {
      // last step: the position of the region closest in phase
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
  // phase within pi / l of the located position (the Eq. 18 bound)
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

// Round-j estimate of the coefficient at permuted position u in bucket i
// (Eq. 14): yhat_j[i] exp(+2 pi i T_j u / N) / Ghat.
template <typename R>
__device__ __forceinline__ cplx<R> round_estimate(const cplx<R>* Y, uint32_t B, uint32_t i, uint32_t j,
                                                   uint32_t Tj, uint32_t u, uint32_t nmask, uint32_t logN, R g) {
  const cplx<R> e = cmul(Y[size_t(j) * B + i], expi<R>((Tj * u) & nmask, logN, R(1)));
  return {e.re / g, e.im / g};
}

template <typename R>
__device__ __forceinline__ void cswap(R& a, R& b) {
  const bool s = b < a;
  const R lo = s ? b : a, hi = s ? a : b;
  a = lo;
  b = hi;
}

// Bitonic network on a register array of kRegRounds values (compile-time indices).
template <typename R>
__device__ __forceinline__ void sort_regs(R (&v)[kRegRounds]) {
#pragma unroll
  for (int k = 2; k <= kRegRounds; k <<= 1)
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1)
#pragma unroll
      for (int i = 0; i < kRegRounds; ++i) {
        const int ixj = i ^ j;
        if (ixj > i) {
          if ((i & k) == 0) cswap(v[i], v[ixj]);
          else cswap(v[ixj], v[i]);
        }
      }
}

template <typename R>
__device__ __forceinline__ R pick_median(const R (&v)[kRegRounds], uint32_t n) {
  const uint32_t lo = (n - 1) / 2, hi = n / 2;
  R a = 0, b = 0;
#pragma unroll
  for (int q = 0; q < kRegRounds; ++q) {
    if (uint32_t(q) == lo) a = v[q];
    if (uint32_t(q) == hi) b = v[q];
  }
  return (a + b) * R(0.5);
}

// Median over the R+1 rounds, real and imaginary parts separately; the mean
// of the two middle values for an even count.
template <typename R>
__device__ cplx<R> median_estimate(const cplx<R>* Y, const IterDesc* it, uint32_t i, uint32_t u, uint32_t nmask,
                                   uint32_t logN, R g) {
  const uint32_t B = it->B, n = it->R + 1;
  if (n <= uint32_t(kRegRounds)) {
    R vr[kRegRounds], vi[kRegRounds];
#pragma unroll
    for (int j = 0; j < kRegRounds; ++j) {
      if (uint32_t(j) < n) {
        const cplx<R> e = round_estimate(Y, B, i, uint32_t(j), it->T[j], u, nmask, logN, g);
        vr[j] = e.re;
        vi[j] = e.im;
      } else {
        vr[j] = R(INFINITY);
        vi[j] = R(INFINITY);
      }
    }
    sort_regs(vr);
    sort_regs(vi);
    return {pick_median(vr, n), pick_median(vi, n)};
  }
  // more rounds than registers: order statistics by counting ranks
  const uint32_t lo = (n - 1) / 2, hi = n / 2;
  R lr = 0, hr = 0, li = 0, hi_ = 0;
  for (uint32_t a = 0; a < n; ++a) {
    const cplx<R> ea = round_estimate(Y, B, i, a, it->T[a], u, nmask, logN, g);
    uint32_t ltr = 0, ler = 0, lti = 0, lei = 0;
    for (uint32_t b = 0; b < n; ++b) {
      const cplx<R> eb = round_estimate(Y, B, i, b, it->T[b], u, nmask, logN, g);
      ltr += eb.re < ea.re;
      ler += eb.re <= ea.re;
      lti += eb.im < ea.im;
      lei += eb.im <= ea.im;
    }
    if (ltr <= lo && lo < ler) lr = ea.re;
    if (ltr <= hi && hi < ler) hr = ea.re;
    if (lti <= lo && lo < lei) li = ea.im;
    if (lti <= hi && hi < lei) hi_ = ea.im;
  }
  return {(lr + hr) * R(0.5), (li + hi_) * R(0.5)};
}

template <typename R>
struct RealKey;
template <>
struct RealKey<float> {  // order of non-negative floats = order of their bits
  using T = uint32_t;
  static __device__ __forceinline__ T bits(float v) { return __float_as_uint(v); }
  static __device__ __forceinline__ float value(T b) { return __uint_as_float(b); }
};
template <>
struct RealKey<double> {
  using T = uint64_t;
  static __device__ __forceinline__ T bits(double v) { return uint64_t(__double_as_longlong(v)); }
  static __device__ __forceinline__ double value(T b) { return __longlong_as_double(int64_t(b)); }
};

// Top-K key: descending magnitude, ties to the smaller frequency.  The store
// is sorted by frequency, so its index breaks ties the same way and names
// the entry directly.
template <typename R>
struct TopKey;
template <>
struct TopKey<float> {
  using T = uint64_t;
  static __device__ __forceinline__ T make(float mag2, uint32_t k) {
    return (uint64_t(~__float_as_uint(mag2)) << 32) | k;
  }
  static __device__ __forceinline__ T none() { return ~uint64_t(0); }
  static __device__ __forceinline__ uint32_t index(T key) { return uint32_t(key); }
};
template <>
struct TopKey<double> {
  using T = K128;
  static __device__ __forceinline__ T make(double mag2, uint32_t k) {
    return K128{~uint64_t(__double_as_longlong(mag2)), uint64_t(k)};
  }
  static __device__ __forceinline__ T none() { return K128{~uint64_t(0), ~uint64_t(0)}; }
  static __device__ __forceinline__ uint32_t index(T key) { return uint32_t(key.lo); }
};

template <typename R>
__global__ __launch_bounds__(kRecThreads) void recover_kernel(SigArg arg) {
  __shared__ __attribute__((aligned(16))) unsigned char lds_buf[kLdsBytes];
  __shared__ uint32_t sh_scan[kRecThreads];
  __shared__ R sh_red[kRecThreads / 64];
  __shared__ uint32_t sh_ured[kRecThreads / 64];
  uint32_t* lds32 = reinterpret_cast<uint32_t*>(lds_buf);
  using RK = RealKey<R>;
  typename RK::T* ldskey = reinterpret_cast<typename RK::T*>(lds_buf);

  const uint32_t tid = threadIdx.x, NT = blockDim.x;
  const SignalDesc sd = load_signal(arg, blockIdx.x);
  const PlanDesc* pd = sd.plan;
  unsigned char* ws = reinterpret_cast<unsigned char*>(sd.ws);
  cplx<R>* Yall = reinterpret_cast<cplx<R>*>(sd.y);
  uint32_t* const recf0 = reinterpret_cast<uint32_t*>(ws + pd->off_recf0);
  uint32_t* const recf1 = reinterpret_cast<uint32_t*>(ws + pd->off_recf1);
  cplx<R>* const recv0 = reinterpret_cast<cplx<R>*>(ws + pd->off_recv0);
  cplx<R>* const recv1 = reinterpret_cast<cplx<R>*>(ws + pd->off_recv1);
  uint32_t* cand_u = reinterpret_cast<uint32_t*>(ws + pd->off_candu);
  uint32_t* cand_d = reinterpret_cast<uint32_t*>(ws + pd->off_candd);
  cplx<R>* cand_v = reinterpret_cast<cplx<R>*>(ws + pd->off_candv);
  uint32_t* pairs = reinterpret_cast<uint32_t*>(ws + pd->off_pairs);
  uint32_t* kflag = reinterpret_cast<uint32_t*>(ws + pd->off_cnt);
  uint64_t* keys = reinterpret_cast<uint64_t*>(ws + pd->off_keys);
  R* p0 = reinterpret_cast<R*>(ws + pd->off_p0);
  const uint32_t N = pd->N, nmask = N - 1, logN = pd->logN;
  uint32_t nrec = 0, cur = 0;
  bool overflow = false;

  for (uint32_t m = 0; m < pd->M; ++m) {
    const IterDesc* it = pd->iters + m;
    const uint32_t B = it->B, L = it->L, D = it->D, R1 = it->R + 1;
    cplx<R>* Y = Yall + it->y_off;
    const R* ghat = reinterpret_cast<const R*>(pd->ghat) + it->ghat_off;
    const uint32_t sigma = it->sigma;
    const uint32_t* of = cur ? recf1 : recf0;
    const cplx<R>* ov = cur ? recv1 : recv0;
    uint32_t* nf = cur ? recf0 : recf1;
    cplx<R>* nv = cur ? recv0 : recv1;

    // ---- subtraction of the coefficients recovered so far ----
    if (nrec > 0) {
      uint32_t* end = lds32;  // per-bucket counts, then list ends
      for (uint32_t i = tid; i < B; i += NT) end[i] = 0;
      __syncthreads();
      for (uint32_t k = tid; k < nrec; k += NT) {
        const int64_t u = int64_t((sigma * of[k]) & nmask);
        const int64_t lo = -floor_div(int64_t(D) - u, L), hi = floor_div(u + int64_t(D), L);
        for (int64_t i = lo; i <= hi; ++i) atomicAdd(&end[uint32_t(i) & (B - 1)], 1u);
      }
      __syncthreads();
      block_scan_exclusive(end, B, sh_scan);
      for (uint32_t k = tid; k < nrec; k += NT) {
        const int64_t u = int64_t((sigma * of[k]) & nmask);
        const int64_t lo = -floor_div(int64_t(D) - u, L), hi = floor_div(u + int64_t(D), L);
        for (int64_t i = lo; i <= hi; ++i) pairs[atomicAdd(&end[uint32_t(i) & (B - 1)], 1u)] = k;
      }
      __syncthreads();
      for (uint32_t i = tid; i < B; i += NT) {
        const uint32_t s0 = i ? end[i - 1] : 0u, e0 = end[i];
        for (uint32_t a = s0 + 1; a < e0; ++a) {  // entries in frequency order
          const uint32_t v = pairs[a];
          uint32_t b = a;
          while (b > s0 && pairs[b - 1] > v) {
            pairs[b] = pairs[b - 1];
            --b;
          }
          pairs[b] = v;
        }
        if (e0 == s0) continue;
        for (uint32_t j = 0; j < R1; ++j) {
          cplx<R> acc{0, 0};
          for (uint32_t q = s0; q < e0; ++q) {
            const uint32_t k = pairs[q];
            const uint32_t u = (sigma * of[k]) & nmask;
            const uint32_t d1 = (i * L - u) & nmask;
            const cplx<R> vg = cscale(ov[k], ghat[min(d1, N - d1)]);
            acc = cadd(acc, cmul(vg, expi<R>((it->T[j] * u) & nmask, logN, R(-1))));
          }
          Y[size_t(j) * B + i] = csub(Y[size_t(j) * B + i], acc);
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
      ldskey[i] = RK::bits(p);
      mx = p > mx ? p : mx;
      const R m0 = sqrt(p);
      uint32_t cons = 1;
      for (uint32_t j = 1; j < R1; ++j) {
        const cplx<R> yj = Y[size_t(j) * B + i];
        if (fabs(sqrt(yj.re * yj.re + yj.im * yj.im) - m0) > R(pd->rho) * m0) cons = 0;
      }
      cand_u[i] = cons;
    }
    mx = block_reduce_max(mx, sh_red);
    block_bitonic_sort(ldskey, B);
    const R med = (RK::value(ldskey[B / 2 - 1]) + RK::value(ldskey[B / 2])) * R(0.5);
    const R thr_noise = R(2.0 * it->log_B) * (med / R(0.69314718055994530942));
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
          cand_v[i] = median_estimate<R>(Y, it, i, u, nmask, logN, g);
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
        for (uint32_t dd = 1; dd <= it->reach; ++dd) {
          const uint32_t i1 = (i - dd) & (B - 1), i2 = (i + dd) & (B - 1);
          if (i1 != i && cand_u[i1] == u && (cand_d[i1] < d || (cand_d[i1] == d && i1 < i))) keep = 0;
          if (i2 != i && cand_u[i2] == u && (cand_d[i2] < d || (cand_d[i2] == d && i2 < i))) keep = 0;
        }
      }
      lds32[i] = keep;
      kflag[i] = keep;
    }
    __syncthreads();
    const uint32_t nsurv = block_scan_exclusive(lds32, B, sh_scan);
    uint32_t npow = 1;
    while (npow < nsurv) npow <<= 1;
    for (uint32_t i = tid; i < B; i += NT) {
      if (kflag[i]) {
        const uint32_t f = (it->sigma_inv * cand_u[i]) & nmask;
        keys[lds32[i]] = (uint64_t(f) << 32) | i;
      }
    }
    for (uint32_t c = nsurv + tid; c < npow; c += NT) keys[c] = ~uint64_t(0);
    __syncthreads();
    if (nsurv > 1) block_bitonic_sort(keys, npow);

    // ---- accumulate into the frequency-sorted store: rec[f] += v ----
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
    cur ^= 1u;
  }

  if (overflow) {
    if (tid == 0) *sd.count = -1;
    return;
  }

  // ---- top-K by magnitude, ties to the smaller frequency; output by frequency ----
  const uint32_t* rf = cur ? recf1 : recf0;
  const cplx<R>* rv = cur ? recv1 : recv0;
  using TK = TopKey<R>;
  typename TK::T* tk = reinterpret_cast<typename TK::T*>(keys);
  uint32_t npow = 1;
  while (npow < nrec) npow <<= 1;
  uint32_t nz = 0;
  for (uint32_t k = tid; k < npow; k += NT) {
    if (k < nrec) {
      const cplx<R> v = rv[k];
      const R mag2 = v.re * v.re + v.im * v.im;
      tk[k] = mag2 != R(0) ? TK::make(mag2, k) : TK::none();
      nz += mag2 != R(0) ? 1u : 0u;
      pairs[k] = 0;
    } else {
      tk[k] = TK::none();
    }
  }
  nz = block_reduce_sum(nz, sh_ured);
  if (npow > 1) block_bitonic_sort(tk, npow);
  const uint32_t Kp = min(pd->K, nz);
  for (uint32_t c = tid; c < Kp; c += NT) pairs[TK::index(tk[c])] = 1u;
  __syncthreads();
  const uint32_t nsel = block_scan_exclusive(pairs, nrec, sh_scan);  // == Kp: indices are unique
  cplx<R>* outv = reinterpret_cast<cplx<R>*>(sd.val);
  for (uint32_t k = tid; k < nrec; k += NT) {
    const uint32_t slot = pairs[k];
    const uint32_t next = k + 1 < nrec ? pairs[k + 1] : nsel;
    if (next != slot) {  // selected
      sd.idx[slot] = int64_t(rf[k]);
      outv[slot] = rv[k];
    }
  }
  if (tid == 0) *sd.count = int64_t(nsel);
}

int launch_recover(int dtype, const SigArg& sig, uint32_t nsig, void* stream) {
  if (nsig == 0) return hipSuccess;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  dim3 grid(nsig), block(kRecThreads);
  if (dtype == SFFT_C128) {
    hipLaunchKernelGGL(recover_kernel<double>, grid, block, 0, s, sig);
  } else {
    hipLaunchKernelGGL(recover_kernel<float>, grid, block, 0, s, sig);
  }
  return hipGetLastError();
}

}  // namespace sfft
