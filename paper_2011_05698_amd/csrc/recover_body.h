// Reconstruction of one signal (Sec. 3.1-3.2), one workgroup per signal,
// iterations in order:
//   subtraction of the coefficients recovered so far (Sec. 3.1, steps 2-3),
//   singleton detection, multiscale location (Eq. 15-19) and verification,
//   median estimation (Eq. 14 per round), accumulation
//   rec[f] += v (step 5); finally the K largest coefficients.
// Under the vote over loops (SFFT_COMBINE_VOTE) no loop subtracts; a store
// entry keeps one estimate per loop that located it, and the entries that at
// least half of the loops located take the median of their estimates.
//
// Work per iteration, in the order the decisions need it:
//   1. the store, read once from memory, is sorted by its permuted frequency
//      u = sigma f mod N (a counting sort on the top bits of u); the
//      coefficients that leak into bucket i are then one circular run of
//      that order;
//   2. round 0 of every bucket, minus its run's contributions;
//   3. the detection threshold from round 0 alone (median and maximum of
//      |yhat_0|^2): only buckets above it can be detected, so
//   4. rounds 1..R are formed (bucket values minus their runs) for those
//      candidate buckets only;
//   5. per candidate, the round-to-round magnitude test; the candidates that
//      pass it form a compact list, and per (listed candidate, round) the
//      phase difference theta_j as a binary angle;
//   6. per listed candidate: location, verification and the median
//      estimate, from values and angles already in LDS;
//   7. accumulation: a located position is looked up in the sorted store
//      (no hash index), existing entries are updated, new ones appended.
// Every sum over the store is taken in u order by a team of lanes closed by a
// fixed cross-lane butterfly, so results are bit-reproducible: repeated runs,
// batches and single calls agree.  The arrays of an iteration live in LDS
// while it has room and in the signal's work area otherwise.
#pragma once

#include "device_common.h"

namespace sfft {

// Two workgroup shapes run the same code: 256 threads with 77 KiB of LDS
// (two workgroups per compute unit: batches of more signals than compute
// units), and 512 threads with 152 KiB (one per compute unit: fewer signals).
// Every sum over the store is split over lanes the same way in both (team
// sizes are chosen for 256 threads), so both give the same bits.
constexpr int kRecThreads = 256;    // 4 waves; the radix select assumes >= 256
constexpr int kRecThreadsWide = 512;
constexpr int kWaves = kRecThreads / 64;
constexpr uint32_t kLdsBytes = kRecoverLdsBytes;
constexpr uint32_t kLdsBytesWide = 155648;
constexpr uint32_t kNone = 0xFFFFFFFFu;
constexpr int kRegRounds = 8;       // rounds whose estimates are sorted in registers
constexpr int kBatch = 4;           // independent loads a thread issues together
constexpr int kBatchY = 8;          // ... for the candidates' bucket values

struct K128 {
  uint64_t hi, lo;
};
__device__ __forceinline__ bool key_less(uint32_t a, uint32_t b) { return a < b; }
__device__ __forceinline__ bool key_less(uint64_t a, uint64_t b) { return a < b; }
__device__ __forceinline__ bool key_less(const K128& a, const K128& b) {
  return a.hi < b.hi || (a.hi == b.hi && a.lo < b.lo);
}

// Ascending bitonic sort of n keys (n a power of two) with a 32-bit payload
// that moves with its key, by the whole block.
template <typename Key>
__device__ void block_bitonic_sort(Key* keys, uint32_t* pay, uint32_t n) {
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
          const uint32_t t = pay[i];
          pay[i] = pay[ixj];
          pay[ixj] = t;
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

__device__ uint32_t block_sum(uint32_t v, uint32_t* sh) {
  v = team_sum(v, 64u);
  if ((threadIdx.x & 63) == 63) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  uint32_t r = 0;
  for (uint32_t w = 0; w < blockDim.x / 64; ++w) r += sh[w];
  __syncthreads();
  return r;
}

// The k-th smallest (0-based) of n unsigned keys, and the next one in order
// (the (k+1)-th; equal to the k-th when that value repeats), by most-
// significant-digit radix selection with 8-bit digits.  Per digit: the
// keys that match the prefix so far add into a histogram, and wave 0 alone
// scans it, picks the digit that holds rank k and clears the other
// histogram for the next digit: two barriers per digit.  hist holds 2 x 256
// counters and must be zero on entry; it is zero again on return.
template <typename K>
__device__ void block_select2(const K* keys, uint32_t n, uint32_t k, uint32_t* hist, uint32_t* sel,
                              uint32_t* wsum, K* red, K* out_k, K* out_k1) {
  K prefix = 0, mask = 0;
  uint32_t r = k;
  int cur = 0;
  for (int shift = int(sizeof(K) * 8) - 8; shift >= 0; shift -= 8) {
    uint32_t* h = hist + cur * 256;
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) {
      const K key = keys[i];
      if ((key & mask) == prefix) atomicAdd(&h[uint32_t(key >> shift) & 255u], 1u);
    }
    __syncthreads();
    if (threadIdx.x < 64) {
      const uint32_t l = threadIdx.x;
      const uint32_t c0 = h[4 * l], c1 = h[4 * l + 1], c2 = h[4 * l + 2], c3 = h[4 * l + 3];
      const uint32_t tot = c0 + c1 + c2 + c3;
      const uint32_t before = wave_incl_scan(tot) - tot;
      if (before <= r && r < before + tot) {
        uint32_t b = before, d = 4 * l;
        if (r >= b + c0) { b += c0; ++d;
          if (r >= b + c1) { b += c1; ++d;
            if (r >= b + c2) { b += c2; ++d; } } }
        sel[0] = d;
        sel[1] = r - b;
      }
      uint32_t* other = hist + (cur ^ 1) * 256;
      other[4 * l] = 0; other[4 * l + 1] = 0; other[4 * l + 2] = 0; other[4 * l + 3] = 0;
    }
    __syncthreads();
    prefix |= K(sel[0]) << shift;
    mask |= K(255) << shift;
    r = sel[1];
    cur ^= 1;
  }
  // the k-th is `prefix`; the (k+1)-th is the same value if more than k+1
  // keys are <= it, else the smallest key above it
  uint32_t le = 0;
  K above = ~K(0);
  for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) {
    const K key = keys[i];
    le += key <= prefix ? 1u : 0u;
    if (key > prefix && key < above) above = key;
  }
  le = team_sum(le, 64u);
  above = wave_min(above);
  if ((threadIdx.x & 63) == 63) {
    wsum[threadIdx.x >> 6] = le;
    red[threadIdx.x >> 6] = above;
  }
  // the histogram used by the last digit is cleared for the next call
  if (threadIdx.x < 256) hist[(cur ^ 1) * 256 + threadIdx.x] = 0;
  __syncthreads();
  uint32_t tle = 0;
  K ab = ~K(0);
  for (uint32_t w = 0; w < blockDim.x / 64; ++w) {
    tle += wsum[w];
    ab = red[w] < ab ? red[w] : ab;
  }
  __syncthreads();
  *out_k = prefix;
  *out_k1 = tle >= k + 2 ? prefix : ab;
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

// Work area of one iteration: a stack over the workgroup's LDS buffer that
// places an array in the signal's work region (at its own offset there)
// once LDS has no room left.  Every thread computes the same layout.
struct Arena {
  unsigned char* lds;
  unsigned char* glob;
  uint32_t lds_top;
  uint64_t glob_top;
  uint32_t lds_cap;  // bytes of the LDS buffer
  struct Mark {
    uint32_t l;
    uint64_t g;
  };
  __device__ Mark mark() const { return Mark{lds_top, glob_top}; }
  __device__ void release(Mark m) {
    lds_top = m.l;
    glob_top = m.g;
  }
  template <typename T>
  __device__ T* take(uint64_t count) {
    const uint64_t bytes = (count * sizeof(T) + 15) & ~uint64_t(15);
    if (uint64_t(lds_top) + bytes <= lds_cap) {
      T* p = reinterpret_cast<T*>(lds + lds_top);
      lds_top += uint32_t(bytes);
      return p;
    }
    T* p = reinterpret_cast<T*>(glob + glob_top);
    glob_top += bytes;
    return p;
  }
};

// ---- binary angles: one turn = 2^32 (uint32_t) or 2^64 (uint64_t) ----
template <typename A>
__device__ __forceinline__ A angle_dist(A a, A b) {
  const A d = a - b, e = b - a;
  return d < e ? d : e;
}

// theta_j = arg(yhat_0 conj(yhat_j)), the two-round phase difference of
// Eq. 15-16 (sign read so that theta_j = 2 pi (tau_j u mod N) / N for a lone
// coefficient at permuted position u), as a binary angle: the angle in
// turns, times 2^32 or 2^64, truncated.
template <typename A, typename R>
__device__ __forceinline__ A theta_bin(cplx<R> y0, cplx<R> yj, bool fp64) {
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
  constexpr double kTurn = sizeof(A) == 8 ? 18446744073709551616.0 : 4294967296.0;
  const double t = turns * kTurn;
  if (!(t < kTurn) || !(t >= 0.0)) return 0;
  return A(t);
}

// Index k < n of the angle first + k step nearest to t (the smallest index on
// a tie), with four independent running minima (k = 0, 1, 2, 3 mod 4) so
// that the comparisons of consecutive candidates do not wait on each other.
template <typename A>
__device__ __forceinline__ uint32_t argmin_progression(A first, A step, uint32_t n, A t) {
  A bd[4] = {~A(0), ~A(0), ~A(0), ~A(0)};
  uint32_t bk[4] = {0, 1, 2, 3};
  A cur[4] = {first, first + step, first + 2 * step, first + 3 * step};
  const A step4 = 4 * step;
  uint32_t k = 0;
  for (; k + 4 <= n; k += 4) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const A d = angle_dist(cur[r], t);
      if (d < bd[r]) {
        bd[r] = d;
        bk[r] = k + uint32_t(r);
      }
      cur[r] += step4;
    }
  }
#pragma unroll
  for (int r = 0; r < 3; ++r) {  // the n mod 4 remaining candidates
    if (k + uint32_t(r) < n) {
      const A d = angle_dist(cur[r], t);
      if (d < bd[r]) {
        bd[r] = d;
        bk[r] = k + uint32_t(r);
      }
    }
  }
  A best_d = bd[0];
  uint32_t best_k = bk[0];
#pragma unroll
  for (int r = 1; r < 4; ++r) {
    if (bd[r] < best_d || (bd[r] == best_d && bk[r] < best_k)) {
      best_d = bd[r];
      best_k = bk[r];
    }
  }
  return best_k;
}

// Multiscale location (Sec. 3.2) of the lone coefficient of a candidate
// bucket i, from its binary angles th(j), j = 1..R, and its verification.
// Returns kNone if rejected, else u; *dist = |iL - u|_N.
//   block step: the centre of block b of the region [a, a + len) is
//     a + (b + 1/2) len / l, whose phase is ((2 l a + (2b+1) len) tau mod 2lN)
//     / 2lN turns: an exact integer fraction that grows by 2 len tau per
//     block; the nearest block wins (the smaller on a tie) and the region
//     restarts q/2 blocks before it (floor);
//   last step: the position of the region nearest in phase (the smaller on
//     a tie);
//   verification: bucket i is the home bucket of u (u in [iL - L/2,
//     iL + L/2)), and every round's phase is within pi / l of the located
//     position (the Eq. 18 bound).
// A = uint32_t needs 2lN <= 2^32 (block-centre phases exact in 32 bits).
template <typename A, typename TH>
__device__ uint32_t locate_bucket(const PlanDesc* pd, const IterDesc* it, uint32_t i, TH th, uint32_t* dist) {
  constexpr uint32_t kBits = sizeof(A) * 8;
  const uint32_t L = it->L, R_ = it->R, logN = pd->logN, nmask = pd->N - 1;
  const uint32_t l = pd->l, logM2 = 1 + pd->logl + logN;
  const uint64_t m2mask = (uint64_t(1) << logM2) - 1;
  const uint32_t den_shift = 1 + pd->logqd + pd->logl;
  const int64_t qd = int64_t(1) << pd->logqd, qn = pd->qn;
  int64_t a = int64_t(i) * L - int64_t(L / 2) - int64_t(it->e);
  uint32_t u = 0;
  if (pd->location == SFFT_LOCATE_DIRECT) {
    // two rounds, tau_1 = 1: theta_1 = 2 pi u / N; the nearest position,
    // halves rounded up: (floor(2 theta N) + 1) / 2 on the binary angle
    u = uint32_t(((uint64_t(th(1)) >> (kBits - 1 - logN)) + 1) >> 1) & nmask;
  } else {
    for (uint32_t j = 1; j <= R_; ++j) {
      const A t = th(j);
      const uint64_t len = it->len[j], tau = it->tau[j];
      if (j < R_) {
        const uint64_t base = ((uint64_t(int64_t(2 * l) * a) + len) * tau) & m2mask;
        const A step = A(((2 * len * tau) & m2mask) << (kBits - logM2));
        const uint32_t best_b = argmin_progression<A>(A(base << (kBits - logM2)), step, l, t);
        a += ((2 * int64_t(best_b) * qd - qn) * int64_t(len)) >> den_shift;
      } else {
        const A step = A((tau & nmask) << (kBits - logN));
        const A first = A(((uint64_t(a) * tau) & nmask) << (kBits - logN));
        const int64_t best_c = a + int64_t(argmin_progression<A>(first, step, uint32_t(len), t));
        u = uint32_t(uint64_t(best_c) & nmask);
      }
    }
  }
  // home bucket of u: the range [iL - L/2, iL + L/2) holds it (Lemma 1, Eq. 14)
  if ((((u + L / 2) & nmask) >> it->logL) != i) return kNone;
  const uint32_t d1 = (i * L - u) & nmask;
  const uint32_t dd = min(d1, pd->N - d1);
  const A tol = A(1) << (kBits - 1 - pd->logl);
  for (uint32_t j = 1; j <= R_; ++j) {
    const A pos = A((uint64_t((u * it->tau[j]) & nmask)) << (kBits - logN));
    if (angle_dist(pos, th(j)) > tol) return kNone;
  }
  *dist = dd;
  return u;
}

// Round-j estimate of the coefficient at permuted position u (Eq. 14) before
// the division by Ghat: yhat_j exp(+2 pi i T_j u / N).  Dividing every
// round by the same Ghat does not change which rounds are the middle ones,
// so the median is divided once, afterwards.
template <typename R>
__device__ __forceinline__ cplx<R> round_estimate(cplx<R> y, uint32_t Tj, uint32_t u, uint32_t nmask, uint32_t logN) {
  return cmul(y, expi<R>((Tj * u) & nmask, logN, R(1)));
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
// of the two middle values for an even count.  yv(j) gives round j's value.
template <int NR, typename R, typename YV>
__device__ __forceinline__ cplx<R> median_in_regs(YV yv, const IterDesc* it, uint32_t u, uint32_t nmask,
                                                  uint32_t logN, uint32_t n) {
  R vr[NR], vi[NR];
#pragma unroll
  for (int j = 0; j < NR; ++j) {
    if (uint32_t(j) < n) {
      const cplx<R> e = round_estimate<R>(yv(uint32_t(j)), it->T[j], u, nmask, logN);
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

template <typename R, typename YV>
__device__ cplx<R> median_estimate(YV yv, const IterDesc* it, uint32_t u, uint32_t nmask, uint32_t logN) {
  const uint32_t n = it->R + 1;
  if (n <= uint32_t(kRegRounds)) return median_in_regs<kRegRounds, R>(yv, it, u, nmask, logN, n);
  // more rounds than registers: order statistics by counting ranks
  const uint32_t lo = (n - 1) / 2, hi = n / 2;
  R lr = 0, hr = 0, li = 0, hi_ = 0;
  for (uint32_t a = 0; a < n; ++a) {
    const cplx<R> ea = round_estimate<R>(yv(a), it->T[a], u, nmask, logN);
    uint32_t ltr = 0, ler = 0, lti = 0, lei = 0;
    for (uint32_t b = 0; b < n; ++b) {
      const cplx<R> eb = round_estimate<R>(yv(b), it->T[b], u, nmask, logN);
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

// Top-K key: descending magnitude, ties to the smaller frequency; then the
// selected keys again by ascending frequency.
template <typename R>
struct TopKey;
template <>
struct TopKey<float> {
  using T = uint64_t;
  static __device__ __forceinline__ T make(float mag2, uint32_t f) {
    return (uint64_t(~__float_as_uint(mag2)) << 32) | f;
  }
  static __device__ __forceinline__ T none() { return ~uint64_t(0); }
  static __device__ __forceinline__ uint32_t freq(T key) { return uint32_t(key); }
  static __device__ __forceinline__ T by_freq(uint32_t f) { return uint64_t(f); }
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

// Per candidate: the round-to-round magnitude test of the detection rule
// over rounds 1..R.  A candidate that passes it is appended to good (in no
// particular order: every later step writes per candidate, so the order
// changes no result); the location of a failed candidate is never taken.
// One thread per candidate, its rounds' values read in batches of kBatch.
template <typename R, int NT>
__device__ void consistency(const cplx<R>* y0, const uint16_t* cand, const cplx<R>* rows, uint32_t ncand, uint32_t R_,
                            R rho, uint16_t* good, uint32_t* ngood) {
  for (uint32_t c = threadIdx.x; c < ncand; c += NT) {
    const cplx<R> a = y0[cand[c]];
    const R m0 = sqrt(a.re * a.re + a.im * a.im);
    bool fail = false;
    for (uint32_t j0 = 0; j0 < R_; j0 += kBatch) {
      cplx<R> b[kBatch];
#pragma unroll
      for (int e = 0; e < kBatch; ++e)
        if (j0 + uint32_t(e) < R_) b[e] = rows[(j0 + uint32_t(e)) * ncand + c];
#pragma unroll
      for (int e = 0; e < kBatch; ++e)
        if (j0 + uint32_t(e) < R_ && fabs(sqrt(b[e].re * b[e].re + b[e].im * b[e].im) - m0) > rho * m0) fail = true;
    }
    if (!fail) good[atomicAdd(ngood, 1u)] = uint16_t(c);
  }
}

// theta_j of every round of the candidates that passed, as binary angles.
template <typename A, typename R, int NT>
__device__ void angles(const cplx<R>* y0, const uint16_t* cand, const cplx<R>* rows, uint32_t ncand, uint32_t R_,
                       bool fp64, const uint16_t* good, uint32_t ngood, A* th) {
  for (uint32_t k = threadIdx.x; k < ngood; k += NT) {
    const uint32_t c = good[k];
    const cplx<R> a = y0[cand[c]];
    for (uint32_t j0 = 0; j0 < R_; j0 += kBatch) {
      cplx<R> b[kBatch];
#pragma unroll
      for (int e = 0; e < kBatch; ++e)
        if (j0 + uint32_t(e) < R_) b[e] = rows[(j0 + uint32_t(e)) * ncand + c];
#pragma unroll
      for (int e = 0; e < kBatch; ++e)
        if (j0 + uint32_t(e) < R_) th[(j0 + uint32_t(e)) * ncand + c] = theta_bin<A>(a, b[e], fp64);
    }
  }
}

template <typename A, typename R, int NT>
__device__ void locate_candidates(const PlanDesc* pd, const IterDesc* it, const R* ghat, const cplx<R>* y0,
                                  const uint16_t* cand, const cplx<R>* rows, const A* th, const uint16_t* good,
                                  uint32_t ngood, uint32_t ncand, uint32_t* cu, cplx<R>* cval) {
  const uint32_t nmask = pd->N - 1, logN = pd->logN;
  for (uint32_t k = threadIdx.x; k < ngood; k += NT) {
    const uint32_t c = good[k];
    const uint32_t i = cand[c];
    uint32_t dd = 0;
    const uint32_t u = locate_bucket<A>(pd, it, i, [&](uint32_t j) { return th[(j - 1) * ncand + c]; }, &dd);
    if (u == kNone) continue;
    const R g = ghat[dd];
    const cplx<R> yi = y0[i];
    const cplx<R> med =
        median_estimate<R>([&](uint32_t j) { return j == 0 ? yi : rows[(j - 1) * ncand + c]; }, it, u, nmask, logN);
    if (g == R(0)) continue;
    cval[c] = cplx<R>{med.re / g, med.im / g};
    cu[c] = u;
  }
}

// LDS state of one signal's recovery.  The fused batch kernel gives its other
// work items (fold tiles, bucket DFTs) the same buffer.
template <typename R, int NT = kRecThreads, uint32_t LDS = kLdsBytes>
struct RecoverShared {
  static constexpr int kThreads = NT;
  static constexpr uint32_t kBuf = LDS;
  unsigned char buf[LDS] __attribute__((aligned(16)));
  uint32_t hist[2 * 256];
  uint32_t wsum[NT / 64];
  uint32_t sel[2];
  uint32_t nrec;
  uint32_t ncand;  // candidate buckets of the iteration
  uint32_t ngood;  // candidates that passed the round-to-round test
  R red[NT / 64];
  typename RealKey<R>::T key[NT / 64];
  // the plan and the current iteration's descriptors, read in every phase
  PlanDesc pd;
  IterDesc it;
};

// The whole reconstruction of one signal by the calling workgroup (Sh::kThreads
// threads).  Everything it keeps in LDS lives in sh.
template <typename R, typename Sh>
__device__ void recover_signal(const SignalDesc& sd, Sh& sh) {
  static_assert(Sh::kThreads >= 256 && Sh::kThreads % 64 == 0, "the radix select and the histograms take 256 threads");
  unsigned char* lds_buf = sh.buf;
  uint32_t* hist = sh.hist;
  uint32_t* wsum = sh.wsum;
  uint32_t* sel = sh.sel;
  uint32_t& nrec_sh = sh.nrec;
  R* sh_red = sh.red;
  typename RealKey<R>::T* sh_key = sh.key;
  PlanDesc& sh_pd = sh.pd;
  IterDesc& sh_it = sh.it;
  using RK = RealKey<R>;
  using KT = typename RK::T;

  const uint32_t tid = threadIdx.x, NT = Sh::kThreads;
  copy_words(&sh_pd, sd.plan, sizeof(PlanDesc));
  if (tid < 256) {
    hist[tid] = 0;
    hist[256 + tid] = 0;
  }
  if (tid == 0) nrec_sh = 0;
  __syncthreads();
  const PlanDesc* pd = &sh_pd;
  unsigned char* ws = reinterpret_cast<unsigned char*>(sd.ws);
  cplx<R>* Yall = reinterpret_cast<cplx<R>*>(sd.y);
  uint32_t* rf = reinterpret_cast<uint32_t*>(ws + pd->off_recf);
  cplx<R>* rv = reinterpret_cast<cplx<R>*>(ws + pd->off_recv);
  unsigned char* gwork = ws + pd->off_work;
  const uint32_t N = pd->N, nmask = N - 1, logN = pd->logN;
  const bool vote = pd->combine == SFFT_COMBINE_VOTE;
  const bool fp64 = pd->fp64_phase != 0;
  // location in 32-bit binary angles when the block-centre phases are exact there
  const bool ang32 = sizeof(R) == 4 && 1 + pd->logl + logN <= 32;
  uint32_t* nvote = reinterpret_cast<uint32_t*>(ws + pd->off_nvote);
  cplx<R>* votes = reinterpret_cast<cplx<R>*>(ws + pd->off_votes);
  uint32_t nrec = 0;

  // The descriptor of iteration m + 1 is read into registers (one word per
  // thread) while iteration m runs, and stored to LDS when m + 1 starts.
  constexpr uint32_t kDescWords = uint32_t(sizeof(IterDesc) / 4);
  static_assert(sizeof(IterDesc) % 4 == 0 && kDescWords <= uint32_t(Sh::kThreads), "one descriptor word per thread");
  uint32_t desc_word = tid < kDescWords ? reinterpret_cast<const uint32_t*>(pd->iters)[tid] : 0u;
  for (uint32_t m = 0; m < pd->M; ++m) {
    if (tid < kDescWords) reinterpret_cast<uint32_t*>(&sh_it)[tid] = desc_word;
    __syncthreads();
    if (m + 1 < pd->M && tid < kDescWords) desc_word = reinterpret_cast<const uint32_t*>(pd->iters + m + 1)[tid];
    const IterDesc* it = &sh_it;
    const uint32_t B = it->B, L = it->L, D = it->D, R_ = it->R;
    const R* ghat = reinterpret_cast<const R*>(pd->ghat) + it->ghat_off;
    const uint32_t sigma = it->sigma;
    const cplx<R>* Yg = Yall + it->y_off;  // this iteration's (R+1) x B bucket block
    const uint32_t nst = nrec;             // store entries when the iteration starts
    const bool subtract = !vote && nst > 0;
    const uint32_t nslot = it->reach + 1;  // buckets a coefficient can reach
    Arena ar{lds_buf, gwork, 0u, 0ull, Sh::kBuf};

    // ---- 1. the store sorted by permuted frequency, and round 0 ----
    // Cells of the top bits of u hold about one entry each; exact ranks
    // inside a cell finish the sort, and the cell ends locate any u in O(1).
    // The store and round 0 of the bucket values are read in one pass, and
    // the window weights the subtraction needs are gathered while the cells
    // are counted.
    uint32_t npow = 1, logc = 0;
    while (npow < nst) {
      npow <<= 1;
      ++logc;
    }
    const uint32_t cshift = logN - logc;  // npow <= rec_cap < N
    uint32_t* cend = nullptr;
    uint64_t* sk = nullptr;
    cplx<R>* sv = nullptr;
    if (nst > 0) {
      cend = ar.take<uint32_t>(npow);
      sk = ar.take<uint64_t>(nst);
      sv = ar.take<cplx<R>>(nst);
    }
    cplx<R>* y0 = ar.take<cplx<R>>(B);
    R* gw = nullptr;                      // window weight per (entry, reachable bucket), by entry index
    RunBounds* run = nullptr;
    cplx<R>* w0 = nullptr;                // v exp(-2 pi i T_0 u / N) per sorted entry
    if (subtract) {
      gw = ar.take<R>(uint64_t(nst) * nslot);
      run = ar.take<RunBounds>(B);
      w0 = ar.take<cplx<R>>(nst);
    }
    const auto mk_det = ar.mark();
    KT* pk = ar.take<KT>(B);  // |round 0|^2 as order-preserving keys (detection only)
    const auto mk_tmp = ar.mark();
    uint32_t* raw_u = nst > 0 ? ar.take<uint32_t>(nst) : nullptr;
    cplx<R>* raw_v = nst > 0 ? ar.take<cplx<R>>(nst) : nullptr;
    uint64_t* tmp = nst > 0 ? ar.take<uint64_t>(nst) : nullptr;
    for (uint32_t c = tid; c < npow && nst > 0; c += NT) cend[c] = 0;
    {
      const uint32_t nload = max(B, nst);
      for (uint32_t i0 = 0; i0 < nload; i0 += kBatch * NT) {
        cplx<R> y[kBatch], v[kBatch];
        uint32_t f[kBatch];
#pragma unroll
        for (int e = 0; e < kBatch; ++e) {
          const uint32_t i = i0 + uint32_t(e) * NT + tid;
          if (i < B) y[e] = Yg[i];
          if (i < nst) {
            f[e] = rf[i];
            v[e] = rv[i];
          }
        }
#pragma unroll
        for (int e = 0; e < kBatch; ++e) {
          const uint32_t i = i0 + uint32_t(e) * NT + tid;
          if (i < B) {
            y0[i] = y[e];
            if (!subtract) pk[i] = RK::bits(y[e].re * y[e].re + y[e].im * y[e].im);
          }
          if (i < nst) {
            raw_u[i] = (sigma * f[e]) & nmask;
            raw_v[i] = v[e];
          }
        }
      }
    }
    __syncthreads();
    if (nst > 0) {
      for (uint32_t k = tid; k < nst; k += NT) atomicAdd(&cend[raw_u[k] >> cshift], 1u);
      if (subtract) {
        // window weight of each bucket an entry reaches (slot r: bucket
        // i0(u) + r, i0 = ceil((u - D) / L)), at gw[k * nslot + r]
        auto weight = [&](uint32_t u, uint32_t r) -> R {
          const int64_t dist = (first_bucket(u, D, it->logL) + int64_t(r)) * int64_t(L) - int64_t(u);
          const int64_t ad = dist < 0 ? -dist : dist;
          return ad <= int64_t(D) ? ghat[ad] : R(0);
        };
        if (nslot <= 2) {
          // both slots of kBatch entries per thread in flight together
          for (uint32_t k0 = 0; k0 < nst; k0 += kBatch * NT) {
            R g0[kBatch], g1[kBatch];
#pragma unroll
            for (int e = 0; e < kBatch; ++e) {
              const uint32_t k = k0 + uint32_t(e) * NT + tid;
              g0[e] = g1[e] = R(0);
              if (k < nst) {
                const uint32_t u = raw_u[k];
                g0[e] = weight(u, 0);
                if (nslot == 2) g1[e] = weight(u, 1);
              }
            }
#pragma unroll
            for (int e = 0; e < kBatch; ++e) {
              const uint32_t k = k0 + uint32_t(e) * NT + tid;
              if (k < nst) {
                gw[k * nslot] = g0[e];
                if (nslot == 2) gw[k * nslot + 1] = g1[e];
              }
            }
          }
        } else {
          for (uint32_t k = tid; k < nst; k += NT) {
            const uint32_t u = raw_u[k];
            for (uint32_t r = 0; r < nslot; ++r) gw[k * nslot + r] = weight(u, r);
          }
        }
      }
      __syncthreads();
      block_scan_array(cend, npow, wsum);  // cend[c] = start of cell c
      for (uint32_t k = tid; k < nst; k += NT) {
        const uint32_t u = raw_u[k];
        tmp[atomicAdd(&cend[u >> cshift], 1u)] = (uint64_t(u) << 32) | k;  // cend[c] ends as the end of cell c
      }
      __syncthreads();
      for (uint32_t p = tid; p < nst; p += NT) {  // exact rank inside the cell
        const uint64_t key = tmp[p];
        const uint32_t c = uint32_t(key >> 32) >> cshift;
        const uint32_t c0 = c ? cend[c - 1] : 0u, c1 = cend[c];
        uint32_t r = 0;
        for (uint32_t p2 = c0; p2 < c1; ++p2) r += tmp[p2] < key ? 1u : 0u;
        const uint32_t q = c0 + r, k = uint32_t(key);
        sk[q] = key;
        const cplx<R> v = raw_v[k];
        sv[q] = v;
        if (subtract) {
          // round 0's value x phase, once per entry
          w0[q] = cmul(v, expi<R>((it->T[0] * uint32_t(key >> 32)) & nmask, logN, R(-1)));
        }
      }
      __syncthreads();
    }
    ar.release(mk_tmp);
    // number of sorted entries whose u is below x (x <= N)
    auto lower = [&](uint32_t x) -> uint32_t {
      if (x >= N) return nst;
      const uint32_t c = x >> cshift;
      uint32_t q = c ? cend[c - 1] : 0u;
      const uint32_t c1 = cend[c];
      while (q < c1 && uint32_t(sk[q] >> 32) < x) ++q;
      return q;
    };

    // ---- 2. round 0 of every bucket, minus the store's contributions ----
    uint32_t S = 1;  // lanes per bucket in the run sums
    if (subtract) {
      // every bucket's run: its first entry and its length (the same in every round)
      const uint32_t span = 2 * D + 1;  // < N
      for (uint32_t i = tid; i < B; i += NT) {
        const uint32_t a = (i * L - D) & nmask;  // first u of the run
        const uint64_t stop = uint64_t(a) + span;
        const uint32_t q0 = lower(a);
        const uint32_t cnt = stop <= N ? lower(uint32_t(stop)) - q0 : nst - q0 + lower(uint32_t(stop - N));
        run[i] = RunBounds{q0, cnt};
      }
      __syncthreads();
      // team size: enough lanes to cover the mean run, as many as let one
      // pass of 256 threads take all buckets (S B <= 256; at least 1, at
      // most 64): the same in both workgroup shapes
      const double mean_run = double(nst) * double(2 * D + 1) / double(N);
      while (S < 64 && double(S) < mean_run && S * 2u * B <= 2u * uint32_t(kRecThreads)) S <<= 1;
    }
    // The sum over bucket i's run of Ghat x v exp(-2 pi i T_j u / N), by the
    // S lanes of a team: lane-strided partial sums closed by a fixed butterfly.
    // wq, when given, holds v exp(-2 pi i T_j u / N) per sorted entry.
    auto run_sum = [&](uint32_t i, uint32_t Tj, const cplx<R>* wq, uint32_t lane, uint32_t S_) -> cplx<R> {
      cplx<R> acc{0, 0};
      const RunBounds rb = run[i];
      for (uint32_t v = lane; v < rb.count; v += S_) {
        uint32_t q = rb.first + v;
        q = q >= nst ? q - nst : q;
        const uint64_t key = sk[q];
        const uint32_t u = uint32_t(key >> 32);
        const uint32_t slot = (i - uint32_t(first_bucket(u, D, it->logL))) & (B - 1);
        const R g = gw[uint32_t(key) * nslot + slot];
        const cplx<R> w = wq ? wq[q] : cmul(sv[q], expi<R>((Tj * u) & nmask, logN, R(-1)));
        acc = cadd(acc, cscale(w, g));
      }
      return acc;
    };
    if (subtract) {
      const uint32_t team = tid / S, lane = tid & (S - 1), nteams = NT / S;
      for (uint32_t base_i = 0; base_i < B; base_i += nteams) {  // uniform trip count per wave
        const uint32_t i = base_i + team;
        cplx<R> acc = i < B ? run_sum(i, it->T[0], w0, lane, S) : cplx<R>{0, 0};
        acc.re = team_sum(acc.re, S);
        acc.im = team_sum(acc.im, S);
        if (i < B && lane == S - 1) {
          const cplx<R> v = csub(y0[i], acc);
          y0[i] = v;
          pk[i] = RK::bits(v.re * v.re + v.im * v.im);
        }
      }
      __syncthreads();
    }

    // ---- 3. detection threshold from round 0 ----
    // The median of the B powers (the two middle order statistics) and the
    // largest: by counting ranks for a few buckets, else by radix selection.
    KT ka, kb, kmax;
    if (B <= 128) {  // B is a power of two >= 16
      if (tid < B) {
        const KT k = pk[tid];
        uint32_t lt = 0, le = 0;
        for (uint32_t b0 = 0; b0 < B; b0 += 16) {
          KT o[16];
#pragma unroll
          for (int r = 0; r < 16; ++r) o[r] = pk[b0 + uint32_t(r)];
#pragma unroll
          for (int r = 0; r < 16; ++r) {
            lt += o[r] < k ? 1u : 0u;
            le += o[r] <= k ? 1u : 0u;
          }
        }
        const uint32_t r = B / 2 - 1;
        if (lt <= r && r < le) sh_key[0] = k;
        if (lt <= r + 1 && r + 1 < le) sh_key[1] = k;
        if (le == B) sh_key[2] = k;
      }
      __syncthreads();
      ka = sh_key[0];
      kb = sh_key[1];
      kmax = sh_key[2];
    } else {
      KT mk = 0;
      for (uint32_t i = tid; i < B; i += NT) mk = pk[i] > mk ? pk[i] : mk;
      kmax = block_max(mk, sh_key);
      block_select2(pk, B, B / 2 - 1, hist, sel, wsum, sh_key, &ka, &kb);
    }
    const R mx = RK::value(kmax);
    const R med = (RK::value(ka) + RK::value(kb)) * R(0.5);
    const R thr_noise = R(2.0 * it->log_B) * (med / R(0.69314718055994530942));
    const R thr_floor = R(pd->eta * pd->eta) * mx;
    const R thr = thr_noise > thr_floor ? thr_noise : thr_floor;
    if (tid == 0) sh.ncand = 0;
    __syncthreads();  // sh_key is read before it is written again
    ar.release(mk_det);

    // ---- 4. candidate buckets (above the threshold), appended in no
    // particular order: every later step writes per candidate, so the order
    // changes no result ----
    uint16_t* cand = ar.take<uint16_t>(B);  // bucket indices (B <= 16384)
    for (uint32_t i = tid; i < B; i += NT) {
      const cplx<R> v = y0[i];
      const R p = v.re * v.re + v.im * v.im;
      if (p >= thr && p > R(0)) cand[atomicAdd(&sh.ncand, 1u)] = uint16_t(i);
    }
    __syncthreads();
    const uint32_t ncand = sh.ncand;
    uint16_t* good = ar.take<uint16_t>(ncand);  // candidates that pass the round-to-round test
    if (tid == 0) sh.ngood = 0;  // read after the barrier that ends step 5
    cplx<R>* rows = ar.take<cplx<R>>(uint64_t(R_) * ncand);  // round j of candidate c at (j-1) ncand + c

    // ---- 5. rounds 1..R of the candidates, minus the store's contributions ----
    const uint32_t nitems = R_ * ncand;
    if (!subtract) {
      // one thread per candidate: its rounds' bucket values, kBatchY loads in flight
      for (uint32_t c = tid; c < ncand; c += NT) {
        const uint32_t i = cand[c];
        for (uint32_t j0 = 0; j0 < R_; j0 += kBatchY) {
          cplx<R> v[kBatchY];
#pragma unroll
          for (int e = 0; e < kBatchY; ++e)
            if (j0 + uint32_t(e) < R_) v[e] = Yg[size_t(j0 + uint32_t(e) + 1) * B + i];
#pragma unroll
          for (int e = 0; e < kBatchY; ++e)
            if (j0 + uint32_t(e) < R_) rows[(j0 + uint32_t(e)) * ncand + c] = v[e];
        }
      }
    } else {
      const double mean_run = double(nst) * double(2 * D + 1) / double(N);
      uint32_t S2 = 1;
      while (S2 < 64 && double(S2) < mean_run && S2 * 2u * nitems <= uint32_t(kRecThreads)) S2 <<= 1;
      const uint32_t team = tid / S2, lane = tid & (S2 - 1), nteams = NT / S2;
      for (uint32_t base_q = 0; base_q < nitems; base_q += nteams) {  // uniform trip count per wave
        const uint32_t q = base_q + team;
        cplx<R> acc{0, 0}, yv{0, 0};
        if (q < nitems) {
          const uint32_t j = 1 + q / ncand;
          const uint32_t i = cand[q - (j - 1) * ncand];
          if (lane == S2 - 1) yv = Yg[size_t(j) * B + i];  // in flight during the run sum
          acc = run_sum(i, it->T[j], nullptr, lane, S2);
        }
        acc.re = team_sum(acc.re, S2);
        acc.im = team_sum(acc.im, S2);
        if (q < nitems && lane == S2 - 1) rows[q] = csub(yv, acc);
      }
    }
    __syncthreads();

    // ---- 6. the round-to-round test, then phase differences ----
    // ---- 7. location, verification, median estimation ----
    cplx<R>* cval;  // estimates of the located candidates
    uint32_t* cu;   // located position per candidate, or kNone
    consistency<R, Sh::kThreads>(y0, cand, rows, ncand, R_, R(pd->rho), good, &sh.ngood);
    __syncthreads();
    const uint32_t ngood = sh.ngood;
    if (ang32) {
      uint32_t* th = ar.take<uint32_t>(nitems);
      cval = ar.take<cplx<R>>(ncand);
      cu = ar.take<uint32_t>(ncand);
      for (uint32_t c = tid; c < ncand; c += NT) cu[c] = kNone;
      angles<uint32_t, R, Sh::kThreads>(y0, cand, rows, ncand, R_, fp64, good, ngood, th);
      __syncthreads();
      locate_candidates<uint32_t, R, Sh::kThreads>(pd, it, ghat, y0, cand, rows, th, good, ngood, ncand, cu, cval);
    } else {
      uint64_t* th = ar.take<uint64_t>(nitems);
      cval = ar.take<cplx<R>>(ncand);
      cu = ar.take<uint32_t>(ncand);
      for (uint32_t c = tid; c < ncand; c += NT) cu[c] = kNone;
      angles<uint64_t, R, Sh::kThreads>(y0, cand, rows, ncand, R_, fp64, good, ngood, th);
      __syncthreads();
      locate_candidates<uint64_t, R, Sh::kThreads>(pd, it, ghat, y0, cand, rows, th, good, ngood, ncand, cu, cval);
    }
    __syncthreads();

    // ---- 8. rec[f] += v ----
    // Verification keeps a position only in its home bucket, so each located
    // position is one candidate.
    for (uint32_t c = tid; c < ncand; c += NT) {
      const uint32_t u = cu[c];
      if (u == kNone) continue;
      const uint32_t f = (it->sigma_inv * u) & nmask;
      const cplx<R> v = cval[c];
      // is f in the store?  The store sorted by u under this iteration's sigma
      // holds it at the position of u, if anywhere.
      uint32_t q = kNone;
      if (nst > 0) {
        const uint32_t p = lower(u);
        if (p < nst && uint32_t(sk[p] >> 32) == u) q = p;
      }
      if (q != kNone) {
        const uint32_t e = uint32_t(sk[q]);
        if (vote) {  // one estimate per loop (f is unique within a loop): at most M per entry
          const uint32_t cn = nvote[e];
          if (cn < pd->M) {
            votes[size_t(e) * pd->M + cn] = v;
            nvote[e] = cn + 1;
          }
        } else {
          rv[e] = cadd(sv[q], v);
        }
      } else {
        const uint32_t e = atomicAdd(&nrec_sh, 1u);
        rf[e] = f;
        rv[e] = v;
        if (vote) {
          nvote[e] = 1;
          votes[size_t(e) * pd->M] = v;
        }
      }
    }
    __syncthreads();
    nrec = nrec_sh;
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
  Arena ar{lds_buf, gwork, 0u, 0ull, Sh::kBuf};
  typename TK::T* tk = ar.take<typename TK::T>(npow);
  uint32_t* tp = ar.take<uint32_t>(npow);  // store entry of each key
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
    tp[k] = k;
  }
  nz = block_sum(nz, wsum);
  if (npow > 1) block_bitonic_sort(tk, tp, npow);
  const uint32_t Kp = min(pd->K, nz);
  // the selected frequencies, sorted ascending (payloads follow their keys)
  uint32_t kpow = 1;
  while (kpow < Kp) kpow <<= 1;
  for (uint32_t c = tid; c < kpow; c += NT) {  // each thread rewrites only its own slots
    const typename TK::T key = c < Kp ? TK::by_freq(TK::freq(tk[c])) : TK::none();
    tk[c] = key;
  }
  __syncthreads();
  if (kpow > 1) block_bitonic_sort(tk, tp, kpow);
  cplx<R>* outv = reinterpret_cast<cplx<R>*>(sd.val);
  for (uint32_t c = tid; c < Kp; c += NT) {
    const uint32_t e = tp[c];
    sd.idx[c] = int64_t(rf[e]);
    outv[c] = rv[e];
  }
  if (tid == 0) *sd.count = int64_t(Kp);
}

}  // namespace sfft
