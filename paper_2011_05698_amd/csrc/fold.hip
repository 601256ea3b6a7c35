// HashToBins, part 1 (Sec. 2.4, Lemma 1): permuted gather x[sigma (t - T) mod N]
// (Eq. 7), window G_t (Eq. 10) and aliasing t -> t mod B (Eq. 11):
//   y_j[b] = sum_{|t| <= h, t = b mod B} G_t x[sigma (t - T_j) mod N].
// One thread owns one bucket b and walks its taps t = t_first + k B; the
// sample index advances by sigma B mod N per tap.  Index arithmetic is uint32
// with wrap-around, exact because N divides 2^32.
#include "device_common.h"

namespace sfft {

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

template <class Ld, bool KAHAN>
__global__ __launch_bounds__(kFoldTile) void fold_kernel(SigArg arg, const FoldTile* __restrict__ tiles) {
  using R = typename Ld::R;
  const FoldTile tl = tiles[blockIdx.x];
  const SignalDesc sd = load_signal(arg, tl.sig);
  const PlanDesc* pd = sd.plan;
  const IterDesc* it = pd->iters + tl.m;
  const uint32_t B = it->B;
  const uint32_t b = tl.b0 + threadIdx.x;
  if (b >= B) return;
  const uint32_t nmask = pd->N - 1;
  const int32_t h = int32_t(it->h);
  const uint32_t T = it->T[tl.j];
  const uint32_t sigma = it->sigma;
  const R* __restrict__ G = reinterpret_cast<const R*>(pd->window) + it->win_off;
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
      s[q] = Ld::load(sd.x, idx);
      const int32_t tt = t + q * int32_t(B);
      g[q] = G[tt < 0 ? -tt : tt];
      idx = (idx + step) & nmask;
    }
#pragma unroll
    for (int q = 0; q < U; ++q) acc.add(g[q], s[q]);
    t += U * int32_t(B);
  }
  for (; k < ntaps; ++k) {
    const cplx<R> s = Ld::load(sd.x, idx);
    acc.add(G[t < 0 ? -t : t], s);
    idx = (idx + step) & nmask;
    t += int32_t(B);
  }
  cplx<R> out{acc.re, acc.im};
  if (Ld::kScaled) out = cscale(out, R(sd.scale));
  cplx<R>* Y = reinterpret_cast<cplx<R>*>(sd.y) + it->y_off + size_t(tl.j) * B;
  Y[b] = out;
}

int launch_fold(int dtype, int kahan, const SigArg& sig, const FoldTile* d_tiles, uint32_t ntiles, void* stream) {
  if (ntiles == 0) return hipSuccess;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  dim3 grid(ntiles), block(kFoldTile);
  if (dtype == SFFT_C128) {
    if (kahan) hipLaunchKernelGGL((fold_kernel<LoadC128, true>), grid, block, 0, s, sig, d_tiles);
    else hipLaunchKernelGGL((fold_kernel<LoadC128, false>), grid, block, 0, s, sig, d_tiles);
  } else if (dtype == SFFT_F16X2_SCALED) {
    if (kahan) hipLaunchKernelGGL((fold_kernel<LoadF16, true>), grid, block, 0, s, sig, d_tiles);
    else hipLaunchKernelGGL((fold_kernel<LoadF16, false>), grid, block, 0, s, sig, d_tiles);
  } else {
    if (kahan) hipLaunchKernelGGL((fold_kernel<LoadC64, true>), grid, block, 0, s, sig, d_tiles);
    else hipLaunchKernelGGL((fold_kernel<LoadC64, false>), grid, block, 0, s, sig, d_tiles);
  }
  return hipGetLastError();
}

}  // namespace sfft
