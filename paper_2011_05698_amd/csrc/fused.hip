// The batch as one persistent launch (the batching form of the method): the
// workgroups of a single kernel take work items from a queue, in an order in
// which every item's inputs come from items taken before it:
//   * fold tile: the permuted gather, window and fold of one tile of one
//     signal (or of a group of 64 signals in a position-major batch), as in
//     the fold stage kernels (fold_body.h);
//   * finish: the bucket DFT of every round of one signal (the LDS pass of
//     fft_body.h), then its recovery (recover_body.h), once every fold tile
//     of its signal (or group) is done.
// A finish item waits on a per-group counter of completed fold tiles.  The
// items it waits for were taken earlier by workgroups that are running and
// never wait on later items, so every wait ends; a wait that has not ended
// after a bounded number of polls gives up and marks the signal's count -2
// instead of hanging.  Recovery (latency-bound, one workgroup per signal)
// of the early signals then overlaps the gather (bandwidth-bound) of the
// later ones.  The fold and the recovery compute every sum as the stage
// kernels do, in the same order; the bucket DFT takes the LDS pass for
// every B, where the stage kernel takes the in-register wave path up to
// 2048 points (fft_wave.h): bucket values agree to rounding, not bit for bit.
#include "fft_body.h"
#include "fold_body.h"
#include "recover_body.h"

namespace sfft {

constexpr int kFusedUnroll = 24;              // taps in flight per thread in fold tiles
constexpr uint32_t kSpinLimit = 1u << 22;     // polls (s_sleep 8 each, ~0.5 us) before a wait gives up

// Zeroes the queue head, the error count and the per-group counters.
__global__ void fused_reset_kernel(uint32_t* ctl, uint32_t n) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) ctl[i] = 0u;
}

// The B-point DFTs (with 1/N) of every round of every iteration of one
// signal, in place, as many rounds per LDS pass as fit.
template <typename R>
__device__ void signal_dfts(const SignalDesc& sd, unsigned char* lds, uint32_t lds_bytes) {
  const PlanDesc* pd = sd.plan;
  cplx<R>* X = reinterpret_cast<cplx<R>*>(lds);
  const uint32_t cap = lds_bytes / uint32_t(sizeof(cplx<R>));
  const R inv = R(1) / R(pd->N);
  const uint32_t M = pd->M;
  for (uint32_t m = 0; m < M; ++m) {
    const IterDesc* it = pd->iters + m;
    const uint32_t B = it->B, logB = it->logB, R1 = it->R + 1;
    const cplx<R>* tw = reinterpret_cast<const cplx<R>*>(pd->twiddle) + it->tw_off;
    cplx<R>* Y = reinterpret_cast<cplx<R>*>(sd.y) + it->y_off;
    const uint32_t per = max(1u, min(R1, cap >> logB));
    for (uint32_t j0 = 0; j0 < R1; j0 += per) {
      const uint32_t n = min(per, R1 - j0);
      fft_rounds<R>(X, n, B, logB, tw, [&](uint32_t g) { return Y + size_t(j0 + g) * B; },
                    [&](uint32_t) { return inv; });
      __syncthreads();  // X is refilled by the next pass
    }
  }
}

template <typename R, class Ld, bool KAHAN, bool PM>
__global__ __launch_bounds__(kRecThreads, 2) void fused_kernel(FusedArgs a) {
  static_assert(sizeof(IlvShared<R>) <= kLdsBytes, "a position-major fold tile fits the recovery's LDS");
  __shared__ RecoverShared<R> sh;
  __shared__ uint32_t item_sh, ok_sh;
  const uint32_t tid = threadIdx.x;
  uint32_t* head = a.ctl;
  uint32_t* err = a.ctl + 1;
  uint32_t* done = a.ctl + 2;
  for (;;) {
    if (tid == 0) item_sh = atomicAdd(head, 1u);
    __syncthreads();
    const uint32_t q = item_sh;
    if (q >= a.nitems) break;  // uniform: every wave leaves once the queue is drained
    const FusedItem f = a.items[q];
    if (f.kind == kFusedFold) {
      const FoldTile tl{f.grp, f.m, f.i0};
      if (PM) fold_tile_ilv<Ld, KAHAN, kFusedUnroll>(a.table, a.nsig, tl, *reinterpret_cast<IlvShared<R>*>(sh.buf));
      else fold_tile_any<Ld, KAHAN, kFusedUnroll>(a.table[f.grp], tl);
      __threadfence();  // this thread's bucket values, visible device-wide
      __syncthreads();
      if (tid == 0) atomicAdd(done + f.grp, 1u);
    } else {
      const uint32_t s = f.grp, g = PM ? s / uint32_t(kIlvSigs) : s;
      if (tid == 0) {
        uint32_t spins = 0, ok = 1u;
        while (__hip_atomic_load(done + g, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < a.need[g]) {
          __builtin_amdgcn_s_sleep(8);
          if (++spins == kSpinLimit) {
            ok = 0u;
            atomicAdd(err, 1u);
            break;
          }
        }
        ok_sh = ok;
      }
      __syncthreads();
      __threadfence();  // acquire: the bucket values other workgroups wrote
      const SignalDesc sd = a.table[s];
      if (!ok_sh) {
        if (tid == 0) *sd.count = -2;
      } else {
        signal_dfts<R>(sd, sh.buf, kLdsBytes);
        recover_signal<R>(sd, sh);
      }
    }
    __syncthreads();  // sh and item_sh are reused by the next item
  }
}

template <typename R, class Ld, bool KAHAN>
static void launch_fused_t(bool pm, uint32_t grid, hipStream_t s, const FusedArgs& a) {
  if (pm) hipLaunchKernelGGL((fused_kernel<R, Ld, KAHAN, true>), dim3(grid), dim3(kRecThreads), 0, s, a);
  else hipLaunchKernelGGL((fused_kernel<R, Ld, KAHAN, false>), dim3(grid), dim3(kRecThreads), 0, s, a);
}

int launch_fused(int dtype, int kahan, bool position_major, uint32_t grid, uint32_t nctl, const FusedArgs& a,
                 void* stream) {
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(fused_reset_kernel, dim3(1), dim3(256), 0, s, a.ctl, nctl);
  if (dtype == SFFT_C128) {
    if (kahan) launch_fused_t<double, LoadC128, true>(position_major, grid, s, a);
    else launch_fused_t<double, LoadC128, false>(position_major, grid, s, a);
  } else if (dtype == SFFT_F16X2_SCALED) {
    if (kahan) launch_fused_t<float, LoadF16, true>(position_major, grid, s, a);
    else launch_fused_t<float, LoadF16, false>(position_major, grid, s, a);
  } else {
    if (kahan) launch_fused_t<float, LoadC64, true>(position_major, grid, s, a);
    else launch_fused_t<float, LoadC64, false>(position_major, grid, s, a);
  }
  return hipGetLastError();
}

}  // namespace sfft
