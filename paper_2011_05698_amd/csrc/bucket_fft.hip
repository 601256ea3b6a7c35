// HashToBins, part 2: the B-point DFT of each folded round with the 1/N
// factor that makes yhat[i] equal the filtered permuted spectrum at iL
// (Eq. 12-13):  yhat_j[i] = (1/N) sum_b y_j[b] exp(-2 pi i i b / B), in place.
// Radix-2 decimation in time on an LDS copy (bit-reversed load).
#include "device_common.h"

namespace sfft {

template <typename R>
__global__ __launch_bounds__(256) void bucket_fft_kernel(SigArg arg, const RoundItem* __restrict__ items) {
  HIP_DYNAMIC_SHARED(double2, smem_raw)  // 16-byte aligned dynamic LDS
  cplx<R>* X = reinterpret_cast<cplx<R>*>(smem_raw);
  const RoundItem itm = items[blockIdx.x];
  const SignalDesc sd = load_signal(arg, itm.sig);
  const PlanDesc* pd = sd.plan;
  const IterDesc* it = pd->iters + itm.m;
  const uint32_t B = it->B, logB = it->logB;
  cplx<R>* Y = reinterpret_cast<cplx<R>*>(sd.y) + it->y_off + size_t(itm.j) * B;
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

int launch_bucket_fft(int dtype, const SigArg& sig, const RoundItem* d_items, uint32_t nitems, uint32_t max_B,
                      void* stream) {
  if (nitems == 0) return hipSuccess;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  dim3 grid(nitems), block(256);
  // up to 128 KiB of dynamic LDS (gfx950 gives a workgroup 160 KiB)
  if (dtype == SFFT_C128) {
    const size_t lds = size_t(max_B) * 16;
    if (lds > 65536) {
      const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&bucket_fft_kernel<double>),
                                               hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(bucket_fft_kernel<double>, grid, block, lds, s, sig, d_items);
  } else {
    const size_t lds = size_t(max_B) * 8;
    if (lds > 65536) {
      const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&bucket_fft_kernel<float>),
                                               hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(bucket_fft_kernel<float>, grid, block, lds, s, sig, d_items);
  }
  return hipGetLastError();
}

}  // namespace sfft
