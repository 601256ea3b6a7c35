// Stage kernel of the bucket DFT: one workgroup per group of rounds with the
// same B (device body in fft_body.h).
#include "fft_body.h"

namespace sfft {

// A workgroup takes a group of rounds with the same B (one round when B is
// large, up to 1024..4096 points (kFftGroupPoints by default) of several rounds, of one or several
// signals, when it is small).  Rounds of different plans may share a group:
// the twiddles exp(-2 pi i k / B) depend on B only; 1/N is per round.
template <typename R>
__global__ __launch_bounds__(256) void bucket_fft_kernel(SigArg arg, const RoundItem* __restrict__ items,
                                                         const FftGroup* __restrict__ groups) {
  HIP_DYNAMIC_SHARED(double2, smem_raw)  // 16-byte aligned dynamic LDS
  constexpr uint32_t kMaxRoundsPerGroup = kMaxFftGroupPoints / 16;  // B >= 16
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
  fft_rounds<R>(X, n, B, logB, tw, [&](uint32_t g) { return sh_y[g]; }, [&](uint32_t g) { return sh_inv[g]; });
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
