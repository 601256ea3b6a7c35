// Device-side helpers shared by the gfx950 kernels.
#pragma once

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
// fraction of a turn, ps / 2^32; sincospi takes 2 p / N = ps / 2^31 in [-1, 1).
template <typename R>
__device__ __forceinline__ cplx<R> expi(uint32_t p, uint32_t logN, R sign);
template <>
__device__ __forceinline__ cplx<float> expi<float>(uint32_t p, uint32_t logN, float sign) {
  const int32_t ps = int32_t(p << (32 - logN));
  float s, c;
  sincospif(float(ps) * 0x1p-31f, &s, &c);
  return {c, sign * s};
}
template <>
__device__ __forceinline__ cplx<double> expi<double>(uint32_t p, uint32_t logN, double sign) {
  const int32_t ps = int32_t(p << (32 - logN));
  double s, c;
  sincospi(double(ps) * 0x1p-31, &s, &c);
  return {c, sign * s};
}

__device__ __forceinline__ SignalDesc load_signal(const SigArg& a, uint32_t s) {
  return a.table ? a.table[s] : a.one;
}

}  // namespace sfft
