// Reconstruction of one signal (Sec. 3.1-3.2), one workgroup per signal,
// iterations in order:
//   subtraction of the coefficients recovered so far (Sec. 3.1, steps 2-3),
//   singleton detection, multiscale location (Eq. 15-19) and verification,
//   median estimation (Eq. 14 per round), dedupe, accumulation
//   rec[f] += v (step 5); finally the K largest coefficients.
// Under the vote over loops (SFFT_COMBINE_VOTE) no loop subtracts; a store
// entry keeps one estimate per loop that located it, and the entries that at
// least half of the loops located take the median of their estimates.
// One thread per bucket for the per-bucket work.  The recovered store is an
// append-only array with an open-addressing hash index on the frequency, so an
// iteration's survivors go straight in; every sum that depends on the store's
// order (per-bucket subtraction, top-K) is taken in frequency order, so results
// are bit-reproducible.  No private (scratch) arrays; wave-level scans and an
// LDS radix select keep the number of workgroup barriers low.
#include "device_common.h"

namespace sfft {

constexpr int kRecThreads = 256;    // 4 waves; the radix select assumes >= 256
constexpr int kWaves = kRecThreads / 64;
constexpr int kLdsBytes = 75776;    // one buffer, reused phase by phase; two workgroups still fit a CU
constexpr uint32_t kNone = 0xFFFFFFFFu;
constexpr int kRegRounds = 16;      // rounds whose estimates are sorted in registers
constexpr int kVgBatch = 4;         // entries whose loads a thread issues together
constexpr int kMaxRoundsPerPass = 4; // rounds the subtraction handles in one pass when LDS allows

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

// ---- cross-lane moves within a wavefront (DPP) ----
// dpp_move<CTRL, ROW_MASK, BANK_MASK>(old, v) returns v of the lane that CTRL
// selects, 0 where that lane is outside the row, and `old` in rows or banks
// masked off.  No LDS traffic and no waits: a fixed sequence of these gives
// reductions and scans whose order of operations is fixed.
constexpr int kDppXor1 = 0xB1;        // quad_perm [1,0,3,2]
constexpr int kDppXor2 = 0x4E;        // quad_perm [2,3,0,1]
constexpr int kDppShr1 = 0x111, kDppShr2 = 0x112, kDppShr3 = 0x113, kDppShr4 = 0x114, kDppShr8 = 0x118;
constexpr int kDppMirror = 0x140;     // lane 15 - i of the row
constexpr int kDppHalfMirror = 0x141; // lane 7 - i of the half row
constexpr int kDppBcast15 = 0x142;    // lane 15 of the previous row
constexpr int kDppBcast31 = 0x143;    // lane 31

template <int CTRL, int RM = 0xF, int BM = 0xF, typename T>
__device__ __forceinline__ T dpp_move(T old, T v) {
  static_assert(sizeof(T) == 4 || sizeof(T) == 8, "32- or 64-bit values");
  if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(T, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, old), __builtin_bit_cast(int, v),
                                                              CTRL, RM, BM, true));
  } else {
    const uint64_t o = __builtin_bit_cast(uint64_t, old), x = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = uint32_t(__builtin_amdgcn_update_dpp(int(uint32_t(o)), int(uint32_t(x)), CTRL, RM, BM, true));
    const uint32_t hi =
        uint32_t(__builtin_amdgcn_update_dpp(int(uint32_t(o >> 32)), int(uint32_t(x >> 32)), CTRL, RM, BM, true));
    return __builtin_bit_cast(T, (uint64_t(hi) << 32) | lo);
  }
}

// Sum over aligned teams of S lanes (S a power of two <= 64, uniform).  The
// team's sum is in its last lane (in every lane of the team for S <= 16).
template <typename T>
__device__ __forceinline__ T team_sum(T v, uint32_t S) {
  if (S >= 2) v = v + dpp_move<kDppXor1>(T(0), v);
  if (S >= 4) v = v + dpp_move<kDppXor2>(T(0), v);
  if (S >= 8) v = v + dpp_move<kDppHalfMirror>(T(0), v);
  if (S >= 16) v = v + dpp_move<kDppMirror>(T(0), v);
  if (S >= 32) v = v + dpp_move<kDppBcast15, 0xA>(T(0), v);
  if (S >= 64) v = v + dpp_move<kDppBcast31, 0xC>(T(0), v);
  return v;
}

// Max / min over the wavefront; the result is in lane 63.
template <typename T>
__device__ __forceinline__ T wave_max(T v) {
  T o;
  o = dpp_move<kDppXor1>(v, v); v = o > v ? o : v;
  o = dpp_move<kDppXor2>(v, v); v = o > v ? o : v;
  o = dpp_move<kDppHalfMirror>(v, v); v = o > v ? o : v;
  o = dpp_move<kDppMirror>(v, v); v = o > v ? o : v;
  o = dpp_move<kDppBcast15, 0xA>(v, v); v = o > v ? o : v;
  o = dpp_move<kDppBcast31, 0xC>(v, v); v = o > v ? o : v;
  return v;
}
template <typename T>
__device__ __forceinline__ T wave_min(T v) {
  T o;
  o = dpp_move<kDppXor1>(v, v); v = o < v ? o : v;
  o = dpp_move<kDppXor2>(v, v); v = o < v ? o : v;
  o = dpp_move<kDppHalfMirror>(v, v); v = o < v ? o : v;
  o = dpp_move<kDppMirror>(v, v); v = o < v ? o : v;
  o = dpp_move<kDppBcast15, 0xA>(v, v); v = o < v ? o : v;
  o = dpp_move<kDppBcast31, 0xC>(v, v); v = o < v ? o : v;
  return v;
}

// Inclusive prefix sum over the wavefront: row-local prefix from shifts by
// 1, 2, 3, then 4 and 8, then the row totals through lanes 15 and 31.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
  uint32_t s = v + dpp_move<kDppShr1>(0u, v);
  s = s + dpp_move<kDppShr2>(0u, v);
  s = s + dpp_move<kDppShr3>(0u, v);
  s = s + dpp_move<kDppShr4, 0xF, 0xE>(0u, s);
  s = s + dpp_move<kDppShr8, 0xF, 0xC>(0u, s);
  s = s + dpp_move<kDppBcast15, 0xA>(0u, s);
  s = s + dpp_move<kDppBcast31, 0xC>(0u, s);
  return s;
}

// Exclusive prefix of one value per thread across the block; *total gets the sum.
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t* wsum, uint32_t* total) {
  const uint32_t incl = wave_incl_scan(v);
  const uint32_t wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 63) wsum[wave] = incl;
  __syncthreads();
  uint32_t before = 0, tot = 0;
  for (uint32_t w = 0; w < blockDim.x / 64; ++w) {
    const uint32_t s = wsum[w];
    before += w < wave ? s : 0u;
    tot += s;
  }
  __syncthreads();
  *total = tot;
  return before + incl - v;
}

// In-place exclusive prefix sum of a[0..n) (contiguous chunk per thread); returns the total.
__device__ uint32_t block_scan_array(uint32_t* a, uint32_t n, uint32_t* wsum) {
  const uint32_t chunk = (n + blockDim.x - 1) / blockDim.x;
  const uint32_t lo = min(n, threadIdx.x * chunk), hi = min(n, lo + chunk);
  uint32_t s = 0;
  for (uint32_t i = lo; i < hi; ++i) s += a[i];
  uint32_t total;
  uint32_t run = block_excl_scan(s, wsum, &total);
  for (uint32_t i = lo; i < hi; ++i) {
    const uint32_t v = a[i];
    a[i] = run;
    run += v;
  }
  __syncthreads();
  return total;
}

template <typename V>
__device__ V block_max(V v, V* sh) {
  v = wave_max(v);
  if ((threadIdx.x & 63) == 63) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  V r = sh[0];
  for (uint32_t w = 1; w < blockDim.x / 64; ++w) r = r > sh[w] ? r : sh[w];
  __syncthreads();
  return r;
}

template <typename V>
__device__ V block_min(V v, V* sh) {
  v = wave_min(v);
  if ((threadIdx.x & 63) == 63) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  V r = sh[0];
  for (uint32_t w = 1; w < blockDim.x / 64; ++w) r = sh[w] < r ? sh[w] : r;
  __syncthreads();
  return r;
}

__device__ uint32_t block_sum(uint32_t v, uint32_t* sh) {
  v = team_sum(v, 64u);
  if ((threadIdx.x & 63) == 63) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  uint32_t r = 0;
  for (uint32_t w = 0; w < blockDim.x / 64; ++w) r += sh[w];
  __syncthreads();
  return r;
}

// The k-th smallest (0-based) of n unsigned keys, by most-significant-digit
// radix selection (8-bit digits); the block must have at least 256 threads.
template <typename K>
__device__ K block_select(const K* keys, uint32_t n, uint32_t k, uint32_t* hist, uint32_t* wsum, uint32_t* sel) {
  K prefix = 0, mask = 0;
  uint32_t r = k;
  for (int shift = int(sizeof(K) * 8) - 8; shift >= 0; shift -= 8) {
    if (threadIdx.x < 256) hist[threadIdx.x] = 0;
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) {
      const K key = keys[i];
      if ((key & mask) == prefix) atomicAdd(&hist[uint32_t(key >> shift) & 255u], 1u);
    }
    __syncthreads();
    const uint32_t c = threadIdx.x < 256 ? hist[threadIdx.x] : 0u;
    uint32_t total;
    const uint32_t before = block_excl_scan(c, wsum, &total);
    if (threadIdx.x < 256 && before <= r && r < before + c) {
      sel[0] = threadIdx.x;
      sel[1] = r - before;
    }
    __syncthreads();
    const uint32_t d = sel[0];
    r = sel[1];
    __syncthreads();
    prefix |= K(d) << shift;
    mask |= K(255) << shift;
  }
  return prefix;
}

// The run of sorted store entries that reach one bucket.
struct RunBounds {
  uint32_t first, count;
};

// Block-wide copy of a descriptor (a multiple of 4 bytes) into LDS.
__device__ __forceinline__ void copy_words(void* dst, const void* src, size_t bytes) {
  for (uint32_t w = threadIdx.x; w < bytes / 4; w += blockDim.x)
    reinterpret_cast<uint32_t*>(dst)[w] = reinterpret_cast<const uint32_t*>(src)[w];
}

// First bucket i0 = ceil((u - D) / L) whose centre i0 L is within D of u
// (possibly -1; taken mod B by the caller).  L is a power of two, so the
// floor of the signed quotient is an arithmetic shift.
__device__ __forceinline__ int64_t first_bucket(uint32_t u, uint32_t D, uint32_t logL) {
  return -((int64_t(D) - int64_t(u)) >> logL);
}

// Hash index of the recovered store: frequency -> entry, linear probing.
// Keys are read with L1-bypassing atomic loads (slots are claimed by atomics).
__device__ __forceinline__ uint32_t hslot(uint32_t f, uint32_t logh) { return (f * 0x9E3779B1u) >> (32 - logh); }
__device__ __forceinline__ uint32_t hkey(const uint32_t* hk, uint32_t h) {
  return __hip_atomic_load(hk + h, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ uint32_t ht_find(const uint32_t* hk, const uint32_t* hi, uint32_t f, uint32_t logh) {
  const uint32_t m = (1u << logh) - 1;
  uint32_t h = hslot(f, logh);
  for (uint32_t probe = 0; probe <= m; ++probe) {
    const uint32_t k = hkey(hk, h);
    if (k == f) return hi[h];
    if (k == kNone) return kNone;
    h = (h + 1) & m;
  }
  return kNone;
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
  if (pd->location == SFFT_LOCATE_DIRECT) {
    // two rounds, tau_1 = 1: theta_1 = 2 pi u / N; the nearest position,
    // halves rounded up (floor(2 theta N) + 1) / 2 on the binary angle
    const uint64_t th = theta_bin(y0, Y[size_t(B) + i], fp64);
    u = uint32_t(((th >> (63 - logN)) + 1) >> 1) & nmask;
  }
  for (uint32_t j = 1; j <= R_ && pd->location != SFFT_LOCATE_DIRECT; ++j) {
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

// Bitonic network on a register array of NR values (compile-time indices).
template <int NR, typename R>
__device__ __forceinline__ void sort_regs(R (&v)[NR]) {
#pragma unroll
  for (int k = 2; k <= NR; k <<= 1)
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1)
#pragma unroll
      for (int i = 0; i < NR; ++i) {
        const int ixj = i ^ j;
        if (ixj > i) {
          if ((i & k) == 0) cswap(v[i], v[ixj]);
          else cswap(v[ixj], v[i]);
        }
      }
}

template <int NR, typename R>
__device__ __forceinline__ R pick_median(const R (&v)[NR], uint32_t n) {
  const uint32_t lo = (n - 1) / 2, hi = n / 2;
  R a = 0, b = 0;
#pragma unroll
  for (int q = 0; q < NR; ++q) {
    if (uint32_t(q) == lo) a = v[q];
    if (uint32_t(q) == hi) b = v[q];
  }
  return (a + b) * R(0.5);
}

// Median over the R+1 rounds, real and imaginary parts separately; the mean
// of the two middle values for an even count.
// The R+1 round estimates sorted in registers (a network of NR >= R+1).
template <int NR, typename R>
__device__ __forceinline__ cplx<R> median_in_regs(const cplx<R>* Y, const IterDesc* it, uint32_t i, uint32_t u,
                                                  uint32_t nmask, uint32_t logN, R g, uint32_t n) {
  R vr[NR], vi[NR];
#pragma unroll
  for (int j = 0; j < NR; ++j) {
    if (uint32_t(j) < n) {
      const cplx<R> e = round_estimate(Y, it->B, i, uint32_t(j), it->T[j], u, nmask, logN, g);
      vr[j] = e.re;
      vi[j] = e.im;
    } else {
      vr[j] = R(INFINITY);
      vi[j] = R(INFINITY);
    }
  }
  sort_regs<NR>(vr);
  sort_regs<NR>(vi);
  return {pick_median<NR>(vr, n), pick_median<NR>(vi, n)};
}

// Median over the R+1 rounds, real and imaginary parts separately; the mean
// of the two middle values for an even count.
template <typename R>
__device__ cplx<R> median_estimate(const cplx<R>* Y, const IterDesc* it, uint32_t i, uint32_t u, uint32_t nmask,
                                   uint32_t logN, R g) {
  const uint32_t B = it->B, n = it->R + 1;
  if (n <= 8u) return median_in_regs<8>(Y, it, i, u, nmask, logN, g, n);
  if (n <= uint32_t(kRegRounds)) return median_in_regs<kRegRounds>(Y, it, i, u, nmask, logN, g, n);
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
struct TopKey<float> {  // descending magnitude, then ascending frequency
  using T = uint64_t;
  static __device__ __forceinline__ T make(float mag2, uint32_t f) {
    return (uint64_t(~__float_as_uint(mag2)) << 32) | f;
  }
  static __device__ __forceinline__ T none() { return ~uint64_t(0); }
  static __device__ __forceinline__ uint32_t freq(T key) { return uint32_t(key); }
  static __device__ __forceinline__ T by_freq(uint32_t f) { return uint64_t(f); }
  static __device__ __forceinline__ uint32_t freq_of_sorted(T key) { return uint32_t(key); }
};
template <>
struct TopKey<double> {
  using T = K128;
  static __device__ __forceinline__ T make(double mag2, uint32_t f) {
    return K128{~uint64_t(__double_as_longlong(mag2)), uint64_t(f)};
  }
  static __device__ __forceinline__ T none() { return K128{~uint64_t(0), ~uint64_t(0)}; }
  static __device__ __forceinline__ uint32_t freq(T key) { return uint32_t(key.lo); }
  static __device__ __forceinline__ T by_freq(uint32_t f) { return K128{uint64_t(f), 0}; }
  static __device__ __forceinline__ uint32_t freq_of_sorted(T key) { return uint32_t(key.hi); }
};

// Median of the real (IM = false) or imaginary parts of n loop estimates
// (mean of the two middle values for an even n), by rank: the value whose
// rank, ties broken by position, is floor((n-1)/2) and the one of rank
// floor(n/2).  n <= 64; one thread.
template <typename R, bool IM>
__device__ R loop_median(const cplx<R>* vs, uint32_t n) {
  R lo = R(0), hi = R(0);
  for (uint32_t a = 0; a < n; ++a) {
    const R x = IM ? vs[a].im : vs[a].re;
    uint32_t rank = 0;
    for (uint32_t b = 0; b < n; ++b) {
      const R y = IM ? vs[b].im : vs[b].re;
      rank += (y < x || (y == x && b < a)) ? 1u : 0u;
    }
    if (rank == (n - 1) / 2) lo = x;
    if (rank == n / 2) hi = x;
  }
  return (n & 1u) ? lo : (lo + hi) * R(0.5);
}

template <typename R>
__global__ __launch_bounds__(kRecThreads) void recover_kernel(SigArg arg) {
  __shared__ __attribute__((aligned(16))) unsigned char lds_buf[kLdsBytes];
  __shared__ uint32_t hist[256];
  __shared__ uint32_t wsum[kWaves];
  __shared__ uint32_t sel[2];
  __shared__ uint32_t nrec_sh;
  __shared__ R sh_red[kWaves];
  __shared__ uint64_t sh_u64[kWaves];
  // the plan and the current iteration's descriptors, read in every phase
  __shared__ PlanDesc sh_pd;
  __shared__ IterDesc sh_it;
  using RK = RealKey<R>;

  const uint32_t tid = threadIdx.x, NT = blockDim.x;
  const SignalDesc sd = load_signal(arg, blockIdx.x);
  copy_words(&sh_pd, sd.plan, sizeof(PlanDesc));
  __syncthreads();
  const PlanDesc* pd = &sh_pd;
  unsigned char* ws = reinterpret_cast<unsigned char*>(sd.ws);
  cplx<R>* Yall = reinterpret_cast<cplx<R>*>(sd.y);
  uint32_t* rf = reinterpret_cast<uint32_t*>(ws + pd->off_recf);
  cplx<R>* rv = reinterpret_cast<cplx<R>*>(ws + pd->off_recv);
  uint32_t* hk = reinterpret_cast<uint32_t*>(ws + pd->off_htkey);
  uint32_t* hi = reinterpret_cast<uint32_t*>(ws + pd->off_htidx);
  uint32_t* g_cand_u = reinterpret_cast<uint32_t*>(ws + pd->off_candu);
  uint32_t* g_cand_d = reinterpret_cast<uint32_t*>(ws + pd->off_candd);
  cplx<R>* g_cand_v = reinterpret_cast<cplx<R>*>(ws + pd->off_candv);
  uint64_t* gkeys = reinterpret_cast<uint64_t*>(ws + pd->off_keys);
  R* g_p0 = reinterpret_cast<R*>(ws + pd->off_p0);
  const uint32_t N = pd->N, nmask = N - 1, logN = pd->logN, logh = pd->log_hcap;
  const uint32_t hmask = (1u << logh) - 1;
  const bool vote = pd->combine == SFFT_COMBINE_VOTE;
  uint32_t* nvote = reinterpret_cast<uint32_t*>(ws + pd->off_nvote);
  cplx<R>* votes = reinterpret_cast<cplx<R>*>(ws + pd->off_votes);

  // empty store and hash index
  for (uint32_t h = tid; h <= hmask; h += NT) hk[h] = kNone;
  if (tid == 0) nrec_sh = 0;
  __threadfence();
  __syncthreads();
  uint32_t nrec = 0;

  for (uint32_t m = 0; m < pd->M; ++m) {
    copy_words(&sh_it, pd->iters + m, sizeof(IterDesc));
    __syncthreads();
    const IterDesc* it = &sh_it;
    const uint32_t B = it->B, L = it->L, D = it->D, R1 = it->R + 1;
    const R* ghat = reinterpret_cast<const R*>(pd->ghat) + it->ghat_off;
    const uint32_t sigma = it->sigma;

    // The vote (SFFT_COMBINE_VOTE) subtracts nothing: every loop sees the
    // whole signal.
    const uint32_t nsub = vote ? 0u : nrec;

    // ---- LDS plan of the iteration ----
    // The iteration's bucket block ((R+1) x B values) and the per-bucket
    // arrays are staged in LDS when they fit beside the scratch that the
    // subtraction and the detection need; otherwise they stay in the
    // workspace.  The subtraction then updates the staged block in place and
    // every later phase reads it from LDS.
    uint32_t npow = 1, logc = 0;
    while (npow < nsub) {
      npow <<= 1;
      ++logc;
    }
    const uint32_t nslot = it->reach + 1;  // buckets a coefficient can reach
    // subtraction scratch: cell ends, sorted keys, values (over the scattered
    // keys), window weights per (entry, reachable bucket), one round's
    // value x phase per entry, one round's sums per bucket
    constexpr uint32_t CB = uint32_t(sizeof(cplx<R>));
    const uint32_t o_sk = (npow * 4u + 15u) & ~15u;
    const uint32_t o_sv = (o_sk + nsub * 8u + 15u) & ~15u;
    const uint32_t o_gq = (o_sv + nsub * CB + 15u) & ~15u;
    const uint32_t o_w = (o_gq + nsub * nslot * uint32_t(sizeof(R)) + 15u) & ~15u;
    // then per bucket the bounds of its run, and (bucket values in the
    // workspace) the sums of the rounds of one pass; rp rounds share a pass
    auto sub_bytes = [&](uint32_t rp, bool staged) -> uint32_t {
      if (nsub == 0) return 0u;
      const uint32_t orun = (o_w + nsub * CB * rp + 15u) & ~15u;
      return orun + B * 8u + (staged ? 0u : B * CB * rp);
    };
    const uint32_t det_need = B * uint32_t(sizeof(typename RK::T));
    const uint32_t ys_bytes = (R1 * B * uint32_t(sizeof(cplx<R>)) + 15u) & ~15u;
    const uint32_t pb_bytes = ((B * uint32_t(sizeof(R)) + 15u) & ~15u) + 2u * ((B * 4u + 15u) & ~15u) +
                              B * uint32_t(sizeof(cplx<R>));
    auto fits = [&](uint32_t rp, bool staged, bool pbs) -> bool {
      const uint32_t sub = sub_bytes(rp, staged);
      return (staged ? ys_bytes : 0u) + (pbs ? pb_bytes : 0u) + (sub > det_need ? sub : det_need) <=
             uint32_t(kLdsBytes);
    };
    const bool y_lds = fits(1, true, false);
    const bool pb_lds_plan = fits(1, y_lds, true);
    uint32_t rp = 1;  // more rounds per pass only where the LDS plan above still holds
    while (rp < uint32_t(kMaxRoundsPerPass) && fits(rp * 2, y_lds, pb_lds_plan)) rp *= 2;
    const uint32_t o_run = (o_w + nsub * CB * rp + 15u) & ~15u;
    const uint32_t o_ys = o_run + B * 8u;
    const uint32_t sub_need = sub_bytes(rp, y_lds);
    const uint32_t scr_need = sub_need > det_need ? sub_need : det_need;
    const uint32_t pb_at = y_lds ? ys_bytes : 0u;
    const bool pb_lds = pb_lds_plan;
    const uint32_t scr_at = (pb_at + (pb_lds ? pb_bytes : 0u) + 15u) & ~15u;
    unsigned char* scr = lds_buf + scr_at;
    const uint32_t scr_bytes = uint32_t(kLdsBytes) - scr_at;
    cplx<R>* const Yg = Yall + it->y_off;
    cplx<R>* const Y = y_lds ? reinterpret_cast<cplx<R>*>(lds_buf) : Yg;
    R* const p0 = pb_lds ? reinterpret_cast<R*>(lds_buf + pb_at) : g_p0;
    uint32_t* const cand_u = pb_lds ? reinterpret_cast<uint32_t*>(lds_buf + pb_at + ((B * uint32_t(sizeof(R)) + 15u) & ~15u))
                                    : g_cand_u;
    uint32_t* const cand_d = pb_lds ? cand_u + ((B + 3u) & ~3u) : g_cand_d;
    cplx<R>* const cand_v = pb_lds ? reinterpret_cast<cplx<R>*>(cand_d + ((B + 3u) & ~3u)) : g_cand_v;
    typename RK::T* const ldskey = reinterpret_cast<typename RK::T*>(scr);
    if (y_lds) {
      for (uint32_t e = tid; e < R1 * B; e += NT) Y[e] = Yg[e];
      __syncthreads();
    }

    // ---- subtraction of the coefficients recovered so far ----
    // Sorted by its permuted frequency u = sigma f mod N, the store lists the
    // coefficients that leak into bucket i (circular distance |iL - u| <= D)
    // as one circular run.  The sort is a counting sort on the top bits of u
    // (about one entry per cell) followed by exact ranks inside each cell;
    // the cell ends locate any run in O(1).  Then, round by round: every
    // entry's value times its phase exp(-2 pi i T_j u / N) is formed once,
    // evenly over the threads; a team of lanes per bucket adds window weight
    // times that value over the bucket's run, closed by a fixed sequence of
    // cross-lane adds; and the round's sums are taken off the bucket values
    // in one pass.  The order of every sum depends only on the recovered set.
    if (nsub > 0) {
      const uint32_t cshift = logN - logc;  // npow <= rec_cap < N
      const bool in_lds = sub_need <= scr_bytes;
      unsigned char* base = in_lds ? scr : reinterpret_cast<unsigned char*>(gkeys);
      uint32_t* cend = reinterpret_cast<uint32_t*>(base);  // cell counts, then cell ends
      uint64_t* sk = reinterpret_cast<uint64_t*>(base + o_sk);
      uint64_t* tmp = reinterpret_cast<uint64_t*>(base + o_sv);  // scattered keys, then values
      cplx<R>* sv = reinterpret_cast<cplx<R>*>(base + o_sv);
      R* gq = reinterpret_cast<R*>(base + o_gq);
      cplx<R>* w = reinterpret_cast<cplx<R>*>(base + o_w);
      RunBounds* run = reinterpret_cast<RunBounds*>(base + o_run);
      cplx<R>* ysub = reinterpret_cast<cplx<R>*>(base + o_ys);
      for (uint32_t c = tid; c < npow; c += NT) cend[c] = 0;
      __syncthreads();
      for (uint32_t k = tid; k < nsub; k += NT) atomicAdd(&cend[((sigma * rf[k]) & nmask) >> cshift], 1u);
      __syncthreads();
      block_scan_array(cend, npow, wsum);  // cend[c] = start of cell c
      for (uint32_t k = tid; k < nsub; k += NT) {
        const uint32_t u = (sigma * rf[k]) & nmask;
        tmp[atomicAdd(&cend[u >> cshift], 1u)] = (uint64_t(u) << 32) | k;  // cend[c] ends as the end of cell c
      }
      __syncthreads();
      for (uint32_t p = tid; p < nsub; p += NT) {  // exact rank inside the cell
        const uint64_t key = tmp[p];
        const uint32_t c = uint32_t(key >> 32) >> cshift;
        const uint32_t c0 = c ? cend[c - 1] : 0u, c1 = cend[c];
        uint32_t r = 0;
        for (uint32_t p2 = c0; p2 < c1; ++p2) r += tmp[p2] < key ? 1u : 0u;
        sk[c0 + r] = key;
      }
      __syncthreads();
      // number of sorted entries whose u is below x (x <= N)
      auto lower = [&](uint32_t x) -> uint32_t {
        if (x >= N) return nsub;
        const uint32_t c = x >> cshift;
        uint32_t q = c ? cend[c - 1] : 0u;
        const uint32_t c1 = cend[c];
        while (q < c1 && uint32_t(sk[q] >> 32) < x) ++q;
        return q;
      };
      // values in sorted order and the window weight of each bucket an entry
      // reaches (slot r: bucket i0(u) + r, i0 = ceil((u - D) / L)); a thread
      // issues the loads of kVgBatch entries together
      for (uint32_t qb = 0; qb < nsub; qb += kVgBatch * NT) {
        uint64_t key[kVgBatch];
        cplx<R> val[kVgBatch];
#pragma unroll
        for (int e = 0; e < kVgBatch; ++e) {
          const uint32_t q = qb + uint32_t(e) * NT + tid;
          key[e] = q < nsub ? sk[q] : 0;
        }
#pragma unroll
        for (int e = 0; e < kVgBatch; ++e) {
          const uint32_t q = qb + uint32_t(e) * NT + tid;
          val[e] = q < nsub ? rv[uint32_t(key[e])] : cplx<R>{0, 0};
        }
#pragma unroll
        for (int e = 0; e < kVgBatch; ++e) {
          const uint32_t q = qb + uint32_t(e) * NT + tid;
          if (q < nsub) {
            const uint32_t u = uint32_t(key[e] >> 32);
            const int64_t i0 = first_bucket(u, D, it->logL);
            sv[q] = val[e];
            for (uint32_t r = 0; r < nslot; ++r) {
              const int64_t dist = (i0 + int64_t(r)) * int64_t(L) - int64_t(u);
              const int64_t ad = dist < 0 ? -dist : dist;
              gq[q * nslot + r] = ad <= int64_t(D) ? ghat[ad] : R(0);
            }
          }
        }
      }
      __syncthreads();
      // every bucket's run: its first entry and its length (the same in every round)
      const uint32_t span = 2 * D + 1;  // < N
      for (uint32_t i = tid; i < B; i += NT) {
        const uint32_t a = (i * L - D) & nmask;  // first u of the run
        const uint64_t stop = uint64_t(a) + span;
        const uint32_t q0 = lower(a);
        const uint32_t cnt = stop <= N ? lower(uint32_t(stop)) - q0 : nsub - q0 + lower(uint32_t(stop - N));
        run[i] = RunBounds{q0, cnt};
      }
      __syncthreads();
      // team size: enough lanes to cover the mean run, as many as let one
      // pass take all buckets (at least 1, at most 64)
      const double mean_run = double(nsub) * double(2 * D + 1) / double(N);
      uint32_t S = 1;
      while (S < 64 && double(S) < mean_run && S * 2u * B <= NT) S <<= 1;
      const uint32_t team = tid / S, lane = tid & (S - 1), nteams = NT / S;
      for (uint32_t j0 = 0; j0 < R1; j0 += rp) {
        const uint32_t nj = min(rp, R1 - j0);
        for (uint32_t q = tid; q < nsub; q += NT) {
          const uint32_t u = uint32_t(sk[q] >> 32);
          const cplx<R> v = sv[q];
          for (uint32_t r = 0; r < nj; ++r)
            w[q * rp + r] = cmul(v, expi<R>((it->T[j0 + r] * u) & nmask, logN, R(-1)));
        }
        __syncthreads();
        for (uint32_t base_i = 0; base_i < B; base_i += nteams) {  // uniform trip count per wave
          const uint32_t i = base_i + team;
          cplx<R> acc[kMaxRoundsPerPass];
#pragma unroll
          for (int r = 0; r < kMaxRoundsPerPass; ++r) acc[r] = cplx<R>{0, 0};
          if (i < B) {
            const RunBounds rb = run[i];
            const uint32_t q0 = rb.first, cnt = rb.count;
            for (uint32_t v = lane; v < cnt; v += S) {
              uint32_t q = q0 + v;
              q = q >= nsub ? q - nsub : q;
              const uint32_t u = uint32_t(sk[q] >> 32);
              const uint32_t slot = (i - uint32_t(first_bucket(u, D, it->logL))) & (B - 1);
              const R g = gq[q * nslot + slot];
#pragma unroll
              for (int r = 0; r < kMaxRoundsPerPass; ++r)
                if (uint32_t(r) < nj) acc[r] = cadd(acc[r], cscale(w[q * rp + uint32_t(r)], g));
            }
          }
#pragma unroll
          for (int r = 0; r < kMaxRoundsPerPass; ++r) {
            if (uint32_t(r) < nj) {  // uniform; the team's sums land in its last lane
              acc[r].re = team_sum(acc[r].re, S);
              acc[r].im = team_sum(acc[r].im, S);
            }
          }
          if (i < B && lane == S - 1) {
#pragma unroll
            for (int r = 0; r < kMaxRoundsPerPass; ++r) {
              if (uint32_t(r) < nj) {
                cplx<R>* yp = Y + size_t(j0 + uint32_t(r)) * B + i;
                if (y_lds) *yp = csub(*yp, acc[r]);  // staged block: in place
                else ysub[size_t(r) * B + i] = acc[r];
              }
            }
          }
        }
        __syncthreads();
        if (y_lds) continue;
        // bucket values in the workspace: take the pass's sums off, loads batched
        for (uint32_t r = 0; r < nj; ++r) {
          cplx<R>* Yj = Y + size_t(j0 + r) * B;
          const cplx<R>* sj = ysub + size_t(r) * B;
          for (uint32_t ib = 0; ib < B; ib += kVgBatch * NT) {
            cplx<R> yv[kVgBatch];
#pragma unroll
            for (int e = 0; e < kVgBatch; ++e) {
              const uint32_t i = ib + uint32_t(e) * NT + tid;
              if (i < B) yv[e] = Yj[i];
            }
#pragma unroll
            for (int e = 0; e < kVgBatch; ++e) {
              const uint32_t i = ib + uint32_t(e) * NT + tid;
              if (i < B) Yj[i] = csub(yv[e], sj[i]);
            }
          }
        }
        __syncthreads();
      }
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
    mx = block_max(mx, sh_red);
    // median of the B powers: the two middle order statistics
    const typename RK::T ka = block_select(ldskey, B, B / 2 - 1, hist, wsum, sel);
    uint32_t le = 0;
    typename RK::T above = ~typename RK::T(0);
    for (uint32_t i = tid; i < B; i += NT) {
      const typename RK::T kk = ldskey[i];
      le += kk <= ka ? 1u : 0u;
      if (kk > ka && kk < above) above = kk;
    }
    le = block_sum(le, wsum);
    const typename RK::T kb = le >= B / 2 + 1 ? ka : block_min(above, reinterpret_cast<typename RK::T*>(sh_u64));
    const R med = (RK::value(ka) + RK::value(kb)) * R(0.5);
    const R thr_noise = R(2.0 * it->log_B) * (med / R(0.69314718055994530942));
    const R thr_floor = R(pd->eta * pd->eta) * mx;
    const R thr = thr_noise > thr_floor ? thr_noise : thr_floor;

    // ---- location, verification, median estimation ----
    // The buckets that pass the screen are listed first (in bucket order, a
    // contiguous chunk per thread), so that the long location chains run on
    // full wavefronts instead of on the few lanes whose bucket is active.
    uint32_t* act = reinterpret_cast<uint32_t*>(scr);  // the median keys are no longer needed
    uint32_t nact;
    {
      const uint32_t chunk = (B + NT - 1) / NT;
      const uint32_t lo = min(B, tid * chunk), hi = min(B, lo + chunk);
      uint32_t mine = 0;
      for (uint32_t i = lo; i < hi; ++i) {
        const R p = p0[i];
        mine += (cand_u[i] && p >= thr && p > R(0)) ? 1u : 0u;
      }
      uint32_t at = block_excl_scan(mine, wsum, &nact);
      for (uint32_t i = lo; i < hi; ++i) {
        const R p = p0[i];
        if (cand_u[i] && p >= thr && p > R(0)) act[at++] = i;
      }
      __syncthreads();
      for (uint32_t i = lo; i < hi; ++i) cand_u[i] = kNone;
      __syncthreads();
    }
    for (uint32_t a = tid; a < nact; a += NT) {
      const uint32_t i = act[a];
      uint32_t dd = 0;
      const uint32_t u = locate_bucket<R>(pd, it, Y, i, &dd);
      const R g = u != kNone ? ghat[dd] : R(0);
      if (u != kNone && g != R(0)) {
        cand_v[i] = median_estimate<R>(Y, it, i, u, nmask, logN, g);
        cand_d[i] = dd;
        cand_u[i] = u;
      }
    }
    __syncthreads();

    // ---- dedupe (nearest bucket centre wins) and rec[f] += v ----
    for (uint32_t i = tid; i < B; i += NT) {
      const uint32_t u = cand_u[i];
      if (u == kNone) continue;
      const uint32_t d = cand_d[i];
      bool keep = true;
      for (uint32_t dd = 1; dd <= it->reach; ++dd) {
        const uint32_t i1 = (i - dd) & (B - 1), i2 = (i + dd) & (B - 1);
        if (i1 != i && cand_u[i1] == u && (cand_d[i1] < d || (cand_d[i1] == d && i1 < i))) keep = false;
        if (i2 != i && cand_u[i2] == u && (cand_d[i2] < d || (cand_d[i2] == d && i2 < i))) keep = false;
      }
      if (!keep) continue;
      const uint32_t f = (it->sigma_inv * u) & nmask;
      const cplx<R> v = cand_v[i];
      uint32_t h = hslot(f, logh);
      for (uint32_t probe = 0; probe <= hmask; ++probe) {
        const uint32_t k = hkey(hk, h);
        if (k == f) {  // seen in an earlier iteration
          const uint32_t e = hi[h];
          if (vote) {  // one estimate per loop (f is unique within a loop): at most M per entry
            const uint32_t c = nvote[e];
            if (c < pd->M) {
              votes[size_t(e) * pd->M + c] = v;
              nvote[e] = c + 1;
            }
          } else {
            rv[e] = cadd(rv[e], v);
          }
          break;
        }
        if (k == kNone) {
          const uint32_t prev = atomicCAS(hk + h, kNone, f);
          if (prev == kNone) {
            const uint32_t e = atomicAdd(&nrec_sh, 1u);
            rf[e] = f;
            rv[e] = v;
            if (vote) {
              nvote[e] = 1;
              votes[size_t(e) * pd->M] = v;
            }
            hi[h] = e;
            break;
          }
        }
        h = (h + 1) & hmask;
      }
    }
    __syncthreads();
    nrec = nrec_sh;
    __syncthreads();
  }

  // ---- the vote over loops: keep f when at least half of the loops located it ----
  if (vote) {
    for (uint32_t e = tid; e < nrec; e += NT) {
      const uint32_t n = nvote[e];
      const cplx<R>* vs = votes + size_t(e) * pd->M;
      rv[e] = 2u * n >= pd->M ? cplx<R>{loop_median<R, false>(vs, n), loop_median<R, true>(vs, n)} : cplx<R>{0, 0};
    }
    __syncthreads();
  }

  // ---- top-K by magnitude, ties to the smaller frequency; output by frequency ----
  using TK = TopKey<R>;
  uint32_t npow = 1;
  while (npow < nrec) npow <<= 1;
  const bool in_lds = npow * sizeof(typename TK::T) <= uint32_t(kLdsBytes);
  typename TK::T* tk = in_lds ? reinterpret_cast<typename TK::T*>(lds_buf) : reinterpret_cast<typename TK::T*>(gkeys);
  uint32_t nz = 0;
  for (uint32_t k = tid; k < npow; k += NT) {
    if (k < nrec) {
      const cplx<R> v = rv[k];
      const R mag2 = v.re * v.re + v.im * v.im;
      tk[k] = mag2 != R(0) ? TK::make(mag2, rf[k]) : TK::none();
      nz += mag2 != R(0) ? 1u : 0u;
    } else {
      tk[k] = TK::none();
    }
  }
  nz = block_sum(nz, wsum);
  if (npow > 1) block_bitonic_sort(tk, npow);
  const uint32_t Kp = min(pd->K, nz);
  // the selected frequencies, sorted ascending
  uint32_t kpow = 1;
  while (kpow < Kp) kpow <<= 1;
  for (uint32_t c = tid; c < kpow; c += NT) {  // each thread rewrites only its own slots
    const typename TK::T key = c < Kp ? TK::by_freq(TK::freq(tk[c])) : TK::none();
    tk[c] = key;
  }
  __syncthreads();
  if (kpow > 1) block_bitonic_sort(tk, kpow);
  cplx<R>* outv = reinterpret_cast<cplx<R>*>(sd.val);
  for (uint32_t c = tid; c < Kp; c += NT) {
    const uint32_t f = TK::freq_of_sorted(tk[c]);
    const uint32_t e = ht_find(hk, hi, f, logh);
    sd.idx[c] = int64_t(f);
    outv[c] = e != kNone ? rv[e] : cplx<R>{0, 0};
  }
  if (tid == 0) *sd.count = int64_t(Kp);
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
