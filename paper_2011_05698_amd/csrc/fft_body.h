// HashToBins, part 2: the B-point DFT of each folded round with the 1/N
// factor that makes yhat[i] equal the filtered permuted spectrum at iL
// (Eq. 12-13):  yhat_j[i] = (1/N) sum_b y_j[b] exp(-2 pi i i b / B), in place.
// Radix-2 decimation in time on an LDS copy (bit-reversed load).
#pragma once

#include "device_common.h"

namespace sfft {

// The B-point DFT with its 1/N factor of n rounds in place, in LDS buffer X
// (n B points); row(g) is round g's array and inv(g) its 1/N.  Radix-2
// decimation in time on a bit-reversed copy.  Stages s and s + 1 go in one
// pass: four points b + p + {0, 1, 2, 3} half (b a multiple of 4 half,
// p < half) take stage s's butterflies (0, 1) and (2, 3) with twiddle p,
// then stage s + 1's (0, 2) and (1, 3) with twiddles p and p + half: the same
// butterflies as two radix-2 passes, with half the barriers and LDS round
// trips.  An odd log B ends with one radix-2 pass.  Ends with the rounds
// written back; no barrier after the write-back.
template <typename R, class Row, class Inv>
__device__ __forceinline__ void fft_rounds(cplx<R>* X, uint32_t n, uint32_t B, uint32_t logB, const cplx<R>* tw,
                                           Row row, Inv inv) {
  const uint32_t total = n << logB, half_total = total >> 1;
  for (uint32_t e = threadIdx.x; e < total; e += blockDim.x) {
    const uint32_t g = e >> logB, b = e & (B - 1);
    X[(g << logB) + (__brev(b) >> (32 - logB))] = row(g)[b];
  }
  __syncthreads();
  // Stages s and s + 1 in one pass: four points b + p + {0, 1, 2, 3} half
  // (b a multiple of 4 half, p < half) take stage s's butterflies (0, 1) and
  // (2, 3) with twiddle p, then stage s + 1's (0, 2) and (1, 3) with
  // twiddles p and p + half: the same butterflies as two radix-2 passes,
  // with half the barriers and LDS round trips.  An odd log B ends with one
  // radix-2 pass.
  uint32_t s = 1;
  for (; s + 1 <= logB; s += 2) {
    const uint32_t half = 1u << (s - 1);
    const uint32_t quarter_total = total >> 2;
    for (uint32_t k = threadIdx.x; k < quarter_total; k += blockDim.x) {
      const uint32_t p = k & (half - 1);
      const uint32_t i0 = ((k >> (s - 1)) << (s + 1)) + p;  // B is a multiple of 4 half: groups never straddle rounds
      const uint32_t i1 = i0 + half, i2 = i0 + 2 * half, i3 = i0 + 3 * half;
      const cplx<R> w1 = tw[p << (logB - s)];
      const cplx<R> w2a = tw[p << (logB - s - 1)], w2b = tw[(p + half) << (logB - s - 1)];
      const cplx<R> x0 = X[i0], x1 = X[i1], x2 = X[i2], x3 = X[i3];
      const cplx<R> c1 = cmul(w1, x1), c3 = cmul(w1, x3);
      const cplx<R> y0 = cadd(x0, c1), y1 = csub(x0, c1), y2 = cadd(x2, c3), y3 = csub(x2, c3);
      const cplx<R> d2 = cmul(w2a, y2), d3 = cmul(w2b, y3);
      X[i0] = cadd(y0, d2);
      X[i2] = csub(y0, d2);
      X[i1] = cadd(y1, d3);
      X[i3] = csub(y1, d3);
    }
    __syncthreads();
  }
  if (s == logB) {
    const uint32_t half = 1u << (s - 1);
    for (uint32_t k = threadIdx.x; k < half_total; k += blockDim.x) {
      const uint32_t pos = k & (half - 1);
      const uint32_t i0 = ((k >> (s - 1)) << s) + pos, i1 = i0 + half;
      const cplx<R> w = tw[pos << (logB - s)];
      const cplx<R> a = X[i0], c = cmul(w, X[i1]);
      X[i0] = cadd(a, c);
      X[i1] = csub(a, c);
    }
    __syncthreads();
  }
  for (uint32_t e = threadIdx.x; e < total; e += blockDim.x) {
    const uint32_t g = e >> logB, i = e & (B - 1);
    row(g)[i] = cscale(X[e], inv(g));
  }
}

}  // namespace sfft
