// HashToBins, part 1 (Sec. 2.4, Lemma 1): permuted gather x[sigma (t - T) mod N]
// (Eq. 7), window G_t (Eq. 10) and aliasing t -> t mod B (Eq. 11):
//   y_j[b] = sum_{|t| <= h, t = b mod B} G_t x[sigma (t - T_j) mod N].
// One thread owns one (round j, bucket b) item of an iteration and walks its
// taps t = t_first + k B; the sample index advances by sigma B mod N per tap.
// Index arithmetic is uint32 with wrap-around, exact because N divides 2^32.
// Taps are fetched U at a time (predicated at the end) so that U independent
// gathers are in flight per thread.
//
// Rounds of one iteration share sigma, so tap t of round j reads the sample
// of tap t - d_j of round 0, d_j = T_j - T_0 mod N: when the offsets of
// rounds 0..nu-1 step by less than w, their windows tile one interval of
// round-0 taps, [-h - d_{nu-1}, h].  A union tile (fold_union) walks that
// interval once per round-0 bucket b and adds each sample into every round
// whose window holds it (round j's bucket is b + d_j mod B), so a sample
// is gathered once for all of those rounds instead of once per round.  Each
// round still takes its taps in increasing t with the same arithmetic, so
// its sum is bit for bit the one-round tile's.
#pragma once

#include "device_common.h"

namespace sfft {

struct LoadC64 {
  using R = float;
  static constexpr bool kScaled = false;
  static __device__ __forceinline__ cplx<float> load(const void* x, uint64_t i) {
    return reinterpret_cast<const cplx<float>*>(x)[i];
  }
  typedef float f4 __attribute__((ext_vector_type(4)));
  // elements i and i + 1 in one 16-byte load (x + i 16-byte aligned)
  static __device__ __forceinline__ void load2(const void* x, uint64_t i, cplx<float>* v) {
    const f4 q = *reinterpret_cast<const f4*>(reinterpret_cast<const cplx<float>*>(x) + i);
    v[0] = {q.x, q.y};
    v[1] = {q.z, q.w};
  }
};
struct LoadC128 {
  using R = double;
  static constexpr bool kScaled = false;
  static __device__ __forceinline__ cplx<double> load(const void* x, uint64_t i) {
    return reinterpret_cast<const cplx<double>*>(x)[i];
  }
};
struct LoadF16 {
  using R = float;
  static constexpr bool kScaled = true;
  typedef _Float16 h2 __attribute__((ext_vector_type(2)));
  typedef _Float16 h4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ cplx<float> load(const void* x, uint64_t i) {
    const h2 v = reinterpret_cast<const h2*>(x)[i];
    return {float(v.x), float(v.y)};
  }
  typedef _Float16 h8 __attribute__((ext_vector_type(8)));
  // elements i and i + 1 in one 8-byte load (x + i 8-byte aligned)
  static __device__ __forceinline__ void load2(const void* x, uint64_t i, cplx<float>* v) {
    const h4 q = *reinterpret_cast<const h4*>(reinterpret_cast<const h2*>(x) + i);
    v[0] = {float(q.x), float(q.y)};
    v[1] = {float(q.z), float(q.w)};
  }
  // elements i .. i + 3 in one 16-byte load (x + i 16-byte aligned)
  static __device__ __forceinline__ void load4(const void* x, uint64_t i, cplx<float>* v) {
    const h8 q = *reinterpret_cast<const h8*>(reinterpret_cast<const h2*>(x) + i);
    v[0] = {float(q[0]), float(q[1])};
    v[1] = {float(q[2]), float(q[3])};
    v[2] = {float(q[4]), float(q[5])};
    v[3] = {float(q[6]), float(q[7])};
  }
};

template <typename R, bool KAHAN>
struct Acc {
  R re = 0, im = 0, cre = 0, cim = 0;
  __device__ __forceinline__ void add(R g, cplx<R> s) {
    if (KAHAN) {  // compensated summation (Kahan)
      const R yr = g * s.re - cre;
      const R tr = re + yr;
      cre = (tr - re) - yr;
      re = tr;
      const R yi = g * s.im - cim;
      const R ti = im + yi;
      cim = (ti - im) - yi;
      im = ti;
    } else {
      re += g * s.re;
      im += g * s.im;
    }
  }
};

// Union tile of rounds 0..NU-1 of iteration m: thread threadIdx.x takes the
// round-0 bucket b = i0 + threadIdx.x and writes bucket b + d_j mod B of
// each round j < NU.
template <class Ld, bool KAHAN, int U, int NU>
__device__ __forceinline__ void fold_union(const SignalDesc& sd, uint32_t m, uint32_t i0) {
  using R = typename Ld::R;
  const PlanDesc* pd = sd.plan;
  const IterDesc* it = pd->iters + m;
  const uint32_t B = it->B;
  const uint32_t b = i0 + threadIdx.x;
  if (b >= B) return;
  const uint32_t nmask = pd->N - 1;
  const int32_t h = int32_t(it->h);
  const uint32_t T0 = it->T[0];
  const uint32_t sigma = it->sigma;
  const R* __restrict__ G = reinterpret_cast<const R*>(pd->window) + it->win_off;
  int32_t d[NU];  // d_j = T_j - T_0 mod N, ascending, d_{NU-1} + w <= N (host-checked)
#pragma unroll
  for (int j = 0; j < NU; ++j) d[j] = int32_t((it->T[j] - T0) & nmask);
  // first round-0 tap t0 = b (mod B) with t0 >= lo; the interval is longer than B
  const int32_t lo = -h - d[NU - 1];
  const int32_t tf = lo + int32_t((b - uint32_t(lo)) & (B - 1));
  const uint32_t ntaps = uint32_t(h - tf) / B + 1;
  uint32_t idx = (sigma * (uint32_t(tf) - T0)) & nmask;
  const uint32_t step = (sigma * B) & nmask;
  Acc<R, KAHAN> acc[NU];
  int32_t t0 = tf;
  for (uint32_t k0 = 0; k0 < ntaps; k0 += U) {
    cplx<R> s[U];
    R g[U][NU];
#pragma unroll
    for (int q = 0; q < U; ++q) {
      s[q] = k0 + q < ntaps ? Ld::load(sd.x, idx) : cplx<R>{0, 0};
#pragma unroll
      for (int j = 0; j < NU; ++j) {
        const int32_t t = t0 + d[j];
        g[q][j] = (k0 + q < ntaps && t >= -h && t <= h) ? G[t < 0 ? -t : t] : R(0);
      }
      idx = (idx + step) & nmask;
      t0 += int32_t(B);
    }
    // round j's taps in increasing t; taps outside its window are not added
    // (a one-round tile adds exact zeros there, which leave a sum unchanged)
    int32_t tq = t0 - int32_t(U) * int32_t(B);
#pragma unroll
    for (int q = 0; q < U; ++q) {
#pragma unroll
      for (int j = 0; j < NU; ++j) {
        const int32_t t = tq + d[j];
        if (k0 + q < ntaps && t >= -h && t <= h) acc[j].add(g[q][j], s[q]);
      }
      tq += int32_t(B);
    }
  }
  cplx<R>* Y = reinterpret_cast<cplx<R>*>(sd.y) + it->y_off;
#pragma unroll
  for (int j = 0; j < NU; ++j) {
    cplx<R> out{acc[j].re, acc[j].im};
    if (Ld::kScaled) out = cscale(out, R(sd.scale));
    Y[(uint32_t(j) << it->logB) + ((b + uint32_t(d[j])) & (B - 1))] = out;
  }
}

// One fold tile of one signal (not a union tile): thread threadIdx.x takes
// item tl.i0 + threadIdx.x.
template <class Ld, bool KAHAN, int U>
__device__ __forceinline__ void fold_tile(const SignalDesc& sd, const FoldTile& tl) {
  using R = typename Ld::R;
  const PlanDesc* pd = sd.plan;
  const IterDesc* it = pd->iters + fold_tile_iter(tl.m);
  const uint32_t B = it->B, logB = it->logB;
  const uint32_t item = tl.i0 + threadIdx.x;
  if (item >= ((it->R + 1) << logB)) return;
  const uint32_t j = item >> logB, b = item & (B - 1);
  const uint32_t nmask = pd->N - 1;
  const int32_t h = int32_t(it->h);
  const uint32_t T = it->T[j];
  const uint32_t sigma = it->sigma;
  const R* __restrict__ G = reinterpret_cast<const R*>(pd->window) + it->win_off;
  // first tap t = b (mod B) with t >= -h; B <= w guarantees t_first <= h
  const int32_t tf = -h + int32_t((b + uint32_t(h)) & (B - 1));
  const uint32_t ntaps = uint32_t(h - tf) / B + 1;
  uint32_t idx = (sigma * (uint32_t(tf) - T)) & nmask;
  const uint32_t step = (sigma * B) & nmask;
  Acc<R, KAHAN> acc;
  int32_t t = tf;
  for (uint32_t k0 = 0; k0 < ntaps; k0 += U) {
    cplx<R> s[U];
    R g[U];
#pragma unroll
    for (int q = 0; q < U; ++q) {
      if (k0 + q < ntaps) {
        s[q] = Ld::load(sd.x, idx);
        g[q] = G[t < 0 ? -t : t];
      } else {
        s[q] = cplx<R>{0, 0};
        g[q] = R(0);
      }
      idx = (idx + step) & nmask;
      t += int32_t(B);
    }
#pragma unroll
    for (int q = 0; q < U; ++q)
      if (!KAHAN || k0 + q < ntaps) acc.add(g[q], s[q]);  // padded taps add exact zeros
  }
  cplx<R> out{acc.re, acc.im};
  if (Ld::kScaled) out = cscale(out, R(sd.scale));
  cplx<R>* Y = reinterpret_cast<cplx<R>*>(sd.y) + it->y_off;
  Y[item] = out;  // item = j * B + b: row j of the iteration's (R+1) x B block
}

// Any per-signal fold tile: a union tile of its round count, or a one-round tile.
template <class Ld, bool KAHAN, int U>
__device__ __forceinline__ void fold_tile_any(const SignalDesc& sd, const FoldTile& tl) {
  const uint32_t nu = fold_tile_rounds(tl.m), m = fold_tile_iter(tl.m);
  if (nu == 2) fold_union<Ld, KAHAN, U, 2>(sd, m, tl.i0);
  else if (nu == 3) fold_union<Ld, KAHAN, U, 3>(sd, m, tl.i0);
  else if (nu >= 4) fold_union<Ld, KAHAN, U, 4>(sd, m, tl.i0);
  else fold_tile<Ld, KAHAN, U>(sd, tl);
}

// Position-major batch: the signals share one plan and sample c of signal s
// sits at x_s + c * ld with x_s = x_0 + s, so for a given tap the signals of
// a workgroup are adjacent elements of one row.  Lanes are signals (P = 1)
// or runs of P adjacent signals (P = 2: one 16-byte load of two complex64
// samples, or 8 bytes of two FP16 pairs; P = 4, FP16 pairs only: one
// 16-byte load of four), so that a load instruction moves P times the
// bytes, and each wave walks the taps of kIlvItems / 4 items:
// index, tap weight and loop bounds are wave-uniform (scalar), every gather
// is one contiguous row segment, and the sum for each (item, signal) takes
// the taps in the same order and arithmetic as fold_kernel, whatever P.
// The kIlvItems x 64 P results are transposed through LDS so that each
// signal's consecutive items are written as one contiguous run.
// LDS of one position-major fold tile: the results, and the destination of
// each signal's run.
template <typename R, int P = 1>
struct IlvShared {
  cplx<R> tile[kIlvItems][kIlvSigs * P + 1];
  cplx<R>* ys[kIlvSigs * P];
};

// One position-major fold tile (kIlvItems items x the 64 P signals from
// group tl.sig on, groups of kIlvSigs) by a workgroup of 256 threads.  P > 1
// takes x_0 aligned to P elements and ld and the signal count multiples of
// P, so that each lane's run is P live signals or none (host-checked).
template <class Ld, bool KAHAN, int U, int P = 1>
__device__ __forceinline__ void fold_tile_ilv(const SignalDesc* __restrict__ table, uint32_t nsig, const FoldTile& tl,
                                              IlvShared<typename Ld::R, P>& sh) {
  using R = typename Ld::R;
  static_assert(P == 1 || P == 2 || P == 4, "one, two or four signals per lane");
  constexpr int kPerWave = kIlvItems / 4;
  constexpr uint32_t kSigs = kIlvSigs * P;
  auto& tile = sh.tile;
  auto& ys = sh.ys;
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const uint32_t s0 = tl.sig * kIlvSigs, s = s0 + lane * P;
  const bool live = s < nsig;
  const SignalDesc& head = table[s0];
  const PlanDesc* pd = head.plan;
  const IterDesc* it = pd->iters + tl.m;
  const uint64_t ld = head.ld;
  const char* xs = live ? reinterpret_cast<const char*>(table[s].x) : nullptr;
  R scale[P];
#pragma unroll
  for (int p = 0; p < P; ++p) {
    scale[p] = live ? R(table[s + p].scale) : R(0);
    if (wave == 0) ys[lane * P + p] = live ? reinterpret_cast<cplx<R>*>(table[s + p].y) + it->y_off : nullptr;
  }
  const uint32_t B = it->B, logB = it->logB;
  const uint32_t nmask = pd->N - 1;
  const int32_t h = int32_t(it->h);
  const uint32_t sigma = it->sigma;
  const uint32_t step = (sigma * B) & nmask;
  const R* __restrict__ G = reinterpret_cast<const R*>(pd->window) + it->win_off;
  for (int q = 0; q < kPerWave; ++q) {
    const uint32_t item = tl.i0 + wave * kPerWave + q;
    const uint32_t j = item >> logB, b = item & (B - 1);
    const uint32_t T = it->T[j];
    const int32_t tf = -h + int32_t((b + uint32_t(h)) & (B - 1));
    const uint32_t ntaps = uint32_t(h - tf) / B + 1;
    uint32_t idx = (sigma * (uint32_t(tf) - T)) & nmask;
    Acc<R, KAHAN> acc[P];
    int32_t t = tf;
    for (uint32_t k0 = 0; k0 < ntaps; k0 += U) {
      cplx<R> v[U][P];
      R g[U];
#pragma unroll
      for (int r = 0; r < U; ++r) {
        if (k0 + r < ntaps && live) {
          if constexpr (P == 4) Ld::load4(xs, uint64_t(idx) * ld, v[r]);
          else if constexpr (P == 2) Ld::load2(xs, uint64_t(idx) * ld, v[r]);
          else v[r][0] = Ld::load(xs, uint64_t(idx) * ld);
        } else {
#pragma unroll
          for (int p = 0; p < P; ++p) v[r][p] = cplx<R>{0, 0};
        }
        g[r] = k0 + r < ntaps ? G[t < 0 ? -t : t] : R(0);
        idx = (idx + step) & nmask;
        t += int32_t(B);
      }
#pragma unroll
      for (int r = 0; r < U; ++r)
        if (!KAHAN || k0 + r < ntaps) {
#pragma unroll
          for (int p = 0; p < P; ++p) acc[p].add(g[r], v[r][p]);
        }
    }
#pragma unroll
    for (int p = 0; p < P; ++p) {
      cplx<R> out{acc[p].re, acc[p].im};
      if (Ld::kScaled) out = cscale(out, scale[p]);
      tile[wave * kPerWave + q][lane * P + p] = out;
    }
  }
  __syncthreads();
  // each group of kIlvItems lanes writes one signal's run of items
  for (uint32_t e = threadIdx.x; e < uint32_t(kIlvItems) * kSigs; e += 256) {
    const uint32_t sl = e / kIlvItems, il = e % kIlvItems;
    if (s0 + sl < nsig) ys[sl][tl.i0 + il] = tile[il][sl];
  }
}

}  // namespace sfft
