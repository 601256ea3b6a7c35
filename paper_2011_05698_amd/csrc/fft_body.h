// HashToBins, part 2: the B-point DFT of each folded round with the 1/N
// factor that makes yhat[i] equal the filtered permuted spectrum at iL
// (Eq. 12-13):  yhat_j[i] = (1/N) sum_b y_j[b] exp(-2 pi i i b / B), in place.
// Radix-2 decimation in time on an LDS copy (bit-reversed load).
#pragma once

#include "device_common.h"

namespace sfft {

// Stages s .. s + 3 of the radix-2 decimation in time in one pass over the
// LDS buffer X of `total` points: a thread takes sixteen points
// b + p + m half (b a multiple of 16 half, p < half, m < 16) into registers
// and applies the four stages' butterflies to them, stage s + t pairing m
// and m + 2^t (bit t of m clear) with the twiddle of the pair's offset
// p + (m mod 2^t) half in its block of 2^(s+t) points.  The same butterflies
// as four radix-2 passes, with a quarter of the barriers and LDS round trips.
template <typename R>
__device__ __forceinline__ void dit_pass16(cplx<R>* X, uint32_t total, uint32_t s, uint32_t logB, const cplx<R>* tw) {
  const uint32_t half = 1u << (s - 1);
  for (uint32_t k = threadIdx.x; k < (total >> 4); k += blockDim.x) {
    const uint32_t p = k & (half - 1);
    const uint32_t i0 = ((k >> (s - 1)) << (s + 3)) + p;  // 16 half divides B: groups never straddle rounds
    cplx<R> x[16];
#pragma unroll
    for (int m = 0; m < 16; ++m) x[m] = X[i0 + uint32_t(m) * half];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
#pragma unroll
      for (int m = 0; m < 16; ++m) {
        if (m & (1 << t)) continue;
        const uint32_t o = p + uint32_t(m & ((1 << t) - 1)) * half;
        const cplx<R> c = cmul(tw[o << (logB - s - uint32_t(t))], x[m + (1 << t)]);
        x[m + (1 << t)] = csub(x[m], c);
        x[m] = cadd(x[m], c);
      }
    }
#pragma unroll
    for (int m = 0; m < 16; ++m) X[i0 + uint32_t(m) * half] = x[m];
  }
}

// The B-point DFT with its 1/N factor of n rounds in place, in LDS buffer X
// (n B points); row(g) is round g's array and inv(g) its 1/N.  Radix-2
// decimation in time on a bit-reversed copy: four stages per pass while
// they last and the rounds hold a sixteen-point group per thread
// (dit_pass16; PASS16 = false leaves it out, and its sixteen registers per
// point group with it), then two: four points b + p + {0, 1, 2, 3} half
// (b a multiple of 4 half, p < half) take stage s's butterflies (0, 1) and
// (2, 3) with twiddle p, then stage s + 1's (0, 2) and (1, 3) with twiddles p
// and p + half.  A last odd stage takes one radix-2 pass.  Ends with the
// rounds written back; no barrier after the write-back.
template <typename R, bool PASS16 = true, class Row, class Inv>
__device__ __forceinline__ void fft_rounds(cplx<R>* X, uint32_t n, uint32_t B, uint32_t logB, const cplx<R>* tw,
                                           Row row, Inv inv) {
  const uint32_t total = n << logB, half_total = total >> 1;
  for (uint32_t e = threadIdx.x; e < total; e += blockDim.x) {
    const uint32_t g = e >> logB, b = e & (B - 1);
    X[(g << logB) + (__brev(b) >> (32 - logB))] = row(g)[b];
  }
  __syncthreads();
  // four stages per pass while there are at least as many sixteen-point
  // groups as threads (else two: fewer threads would wait idle)
  uint32_t s = 1;
  for (; PASS16 && s + 3 <= logB && (total >> 4) >= blockDim.x; s += 4) {
    dit_pass16<R>(X, total, s, logB, tw);
    __syncthreads();
  }
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
