// Stage kernel of the bucket DFT: one workgroup per group of rounds with the
// same B (device body in fft_body.h).
#include "fft_body.h"
#include "fft_wave.h"

namespace sfft {

// A workgroup takes a group of rounds with the same B: one round (or a few)
// when B is above the wave path's size, a few chunks of 64 / L1 rounds per
// wave below it, of one or several signals.  Rounds of different plans may
// share a group: the twiddles exp(-2 pi i k / B) depend on B only; 1/N is
// per round.  Two kernels, for the register budgets of the two paths: the
// LDS pass (few registers, many workgroups per CU) for the groups
// [0, nlds), the in-register wave path for the rest.
template <typename R>
struct GroupRows {
  cplx<R>* y[kMaxFftGroupPoints / 16];  // B >= 16
  R inv[kMaxFftGroupPoints / 16];
};

// The rows of the group's rounds into LDS; returns the group's first round.
template <typename R>
__device__ RoundItem load_group(const SigArg& arg, const RoundItem* __restrict__ items, const FftGroup& grp,
                                GroupRows<R>& rows) {
  for (uint32_t g = threadIdx.x; g < grp.count; g += blockDim.x) {
    const RoundItem itm = items[grp.first + g];
    const SignalDesc sd = load_signal(arg, itm.sig);
    const IterDesc* it = sd.plan->iters + itm.m;
    rows.y[g] = reinterpret_cast<cplx<R>*>(sd.y) + it->y_off + size_t(itm.j) * it->B;
    rows.inv[g] = R(1) / R(sd.plan->N);
  }
  return items[grp.first];
}

constexpr uint32_t kFftLdsMaxThreads = 1024;

template <typename R, bool PASS16>
__global__ __launch_bounds__(kFftLdsMaxThreads) void bucket_fft_lds_kernel(SigArg arg, const RoundItem* __restrict__ items,
                                                                           const FftGroup* __restrict__ groups,
                                                                           uint32_t first_group) {
  HIP_DYNAMIC_SHARED(double2, smem_raw)  // 16-byte aligned dynamic LDS
  __shared__ GroupRows<R> rows;
  const FftGroup grp = groups[first_group + blockIdx.x];
  const RoundItem first = load_group(arg, items, grp, rows);
  const SignalDesc sd0 = load_signal(arg, first.sig);
  const IterDesc* it0 = sd0.plan->iters + first.m;
  const cplx<R>* tw = reinterpret_cast<const cplx<R>*>(sd0.plan->twiddle) + it0->tw_off;
  __syncthreads();
  fft_rounds<R, PASS16>(reinterpret_cast<cplx<R>*>(smem_raw), grp.count, it0->B, it0->logB, tw,
                [&](uint32_t g) { return rows.y[g]; }, [&](uint32_t g) { return rows.inv[g]; });
}

template <typename R>
__global__ __launch_bounds__(256, 2) void bucket_fft_wave_kernel(SigArg arg, const RoundItem* __restrict__ items,
                                                                 const FftGroup* __restrict__ groups,
                                                                 uint32_t first_group) {
  HIP_DYNAMIC_SHARED(double2, smem_raw)
  __shared__ GroupRows<R> rows;
  cplx<R>* X = reinterpret_cast<cplx<R>*>(smem_raw);
  const FftGroup grp = groups[first_group + blockIdx.x];
  const RoundItem first = load_group(arg, items, grp, rows);
  const SignalDesc sd0 = load_signal(arg, first.sig);
  const IterDesc* it0 = sd0.plan->iters + first.m;
  const uint32_t B = it0->B;
  const cplx<R>* tw = reinterpret_cast<const cplx<R>*>(sd0.plan->twiddle) + it0->tw_off;
  for (uint32_t k = threadIdx.x; k < B / 2; k += blockDim.x) X[k] = tw[k];  // twiddles, then the wave tiles
  __syncthreads();
  wave_fft_rounds<R>(grp.count, it0->logB, [&](uint32_t g) { return rows.y[g]; },
                     [&](uint32_t g) { return rows.inv[g]; }, X + B / 2, X);
}

template <typename R>
static int launch_t(const SigArg& sig, const RoundItem* d_items, const FftGroup* d_groups, const FftGroups& fg,
                    hipStream_t s) {
  constexpr size_t CB = sizeof(cplx<R>);
  // LDS groups [0, n16) hold a sixteen-point butterfly group per thread of
  // a 1024-thread workgroup and take four stages per pass; the others
  // [n16, nlds) take two, in a kernel with the registers of that pass alone,
  // one thread per radix-2^2 butterfly group of the largest group's points
  // (256 to 1024 threads)
  const uint32_t bounds[3] = {0u, fg.n16, fg.nlds};
  for (int k = 0; k < 2; ++k) {
    const uint32_t g0 = bounds[k], g1 = bounds[k + 1];
    if (g1 <= g0) continue;
    const uint32_t pts = k == 0 ? fg.max_points : fg.max_points_rest;
    const size_t lds = size_t(pts) * CB;
    const void* fn = k == 0 ? reinterpret_cast<const void*>(&bucket_fft_lds_kernel<R, true>)
                            : reinterpret_cast<const void*>(&bucket_fft_lds_kernel<R, false>);
    if (lds > 65536) {
      const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
      if (e != hipSuccess) return e;
    }
    const uint32_t threads = k == 0 ? kFftLdsMaxThreads : std::min(kFftLdsMaxThreads, std::max(256u, pts / 4));
    if (k == 0)
      hipLaunchKernelGGL((bucket_fft_lds_kernel<R, true>), dim3(g1 - g0), dim3(threads), lds, s, sig, d_items,
                         d_groups, g0);
    else
      hipLaunchKernelGGL((bucket_fft_lds_kernel<R, false>), dim3(g1 - g0), dim3(threads), lds, s, sig, d_items,
                         d_groups, g0);
  }
  if (fg.ngroups > fg.nlds) {
    // the largest need of the sizes up to the largest present (a smaller B
    // can need more: 2^6 points take 18,688 bytes of complex64, 2^7 points
    // 18,944, 2^4 points 10,304 and 2^5 points 10,368); at most 75,776 bytes
    uint32_t elems = 0;
    for (uint32_t l = 4; l <= fg.wave_logB; ++l) elems = max(elems, wave_fft_lds_elems(l, kFftWaves));
    const size_t lds = size_t(elems) * CB;
    if (lds > 65536) {
      const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&bucket_fft_wave_kernel<R>),
                                               hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(bucket_fft_wave_kernel<R>, dim3(fg.ngroups - fg.nlds), dim3(kFftWaves * 64), lds, s, sig,
                       d_items, d_groups, fg.nlds);
  }
  return hipGetLastError();
}

int launch_bucket_fft(int dtype, const SigArg& sig, const RoundItem* d_items, const FftGroup* d_groups,
                      const FftGroups& fg, void* stream) {
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  return dtype == SFFT_C128 ? launch_t<double>(sig, d_items, d_groups, fg, s)
                            : launch_t<float>(sig, d_items, d_groups, fg, s);
}

}  // namespace sfft
