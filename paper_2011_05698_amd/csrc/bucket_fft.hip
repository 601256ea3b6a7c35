// HashToBins, part 2: the B-point DFT of each folded round with the 1/N
// factor that makes yhat[i] equal the filtered permuted spectrum at iL
// (Eq. 12-13):  yhat_j[i] = (1/N) sum_b y_j[b] exp(-2 pi i i b / B), in place.
// Radix-2 decimation in time on an LDS copy (bit-reversed load).
#include "device_common.h"

namespace sfft {

// A workgroup takes a group of rounds with the same B (one round when B is
// large, up to kFftGroupPoints points of several rounds, of one or several
// signals, when it is small).  Rounds of different plans may share a group:
// the twiddles exp(-2 pi i k / B) depend on B only; 1/N is per round.
template <typename R>
__global__ __launch_bounds__(256) void bucket_fft_kernel(SigArg arg, const RoundItem* __restrict__ items,
                                                         const FftGroup* __restrict__ groups) {
  HIP_DYNAMIC_SHARED(double2, smem_raw)  // 16-byte aligned dynamic LDS
  constexpr uint32_t kMaxRoundsPerGroup = kFftGroupPoints / 16;  // B >= 16
  __shared__ cplx<R>* sh_y[kMaxRoundsPerGroup];
  __shared__ R sh_inv[kMaxRoundsPerGroup];
  cplx<R>* X = reinterpret_cast<cplx<R>*>(smem_raw);
  const FftGroup grp = groups[blockIdx.x];
  const RoundItem first = items[grp.first];
  const SignalDesc sd0 = load_signal(arg, first.sig);
  const IterDesc* it0 = sd0.plan->iters + first.m;
  const uint32_t B = it0->B, logB = it0->logB, n = grp.count;
  const cplx<R>* tw = reinterpret_cast<const cplx<R>*>(sd0.plan->twiddle) + it0->tw_off;
  for (uint32_t g = threadIdx.x; g < n; g += blockDim.x) {
    const RoundItem itm = items[grp.first + g];
    const SignalDesc sd = load_signal(arg, itm.sig);
    const IterDesc* it = sd.plan->iters + itm.m;
    sh_y[g] = reinterpret_cast<cplx<R>*>(sd.y) + it->y_off + size_t(itm.j) * B;
    sh_inv[g] = R(1) / R(sd.plan->N);
  }
  __syncthreads();
  const uint32_t total = n << logB, half_total = total >> 1;
  for (uint32_t e = threadIdx.x; e < total; e += blockDim.x) {
    const uint32_t g = e >> logB, b = e & (B - 1);
    X[(g << logB) + (__brev(b) >> (32 - logB))] = sh_y[g][b];
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
    sh_y[g][i] = cscale(X[e], sh_inv[g]);
  }
}

int launch_bucket_fft(int dtype, const SigArg& sig, const RoundItem* d_items, const FftGroup* d_groups,
                      uint32_t ngroups, uint32_t max_points, void* stream) {
  if (ngroups == 0) return hipSuccess;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  dim3 grid(ngroups), block(256);
  // up to 128 KiB of dynamic LDS (gfx950 gives a workgroup 160 KiB)
  if (dtype == SFFT_C128) {
    const size_t lds = size_t(max_points) * 16;
    if (lds > 65536) {
      const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&bucket_fft_kernel<double>),
                                               hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(bucket_fft_kernel<double>, grid, block, lds, s, sig, d_items, d_groups);
  } else {
    const size_t lds = size_t(max_points) * 8;
    if (lds > 65536) {
      const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&bucket_fft_kernel<float>),
                                               hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(bucket_fft_kernel<float>, grid, block, lds, s, sig, d_items, d_groups);
  }
  return hipGetLastError();
}

}  // namespace sfft
