// The recovery stage kernel: one workgroup per signal runs recover_signal
// (recover_body.h) on the bucket values the fold and the bucket DFT wrote.
#include "recover_body.h"

namespace sfft {

template <typename R>
__global__ __launch_bounds__(kRecThreads, 2) void recover_kernel(SigArg arg) {
  __shared__ RecoverShared<R> sh;
  recover_signal<R>(load_signal(arg, blockIdx.x), sh);
}

int launch_recover(int dtype, const SigArg& sig, uint32_t nsig, void* stream) {
  if (nsig == 0) return hipSuccess;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  dim3 grid(nsig), block(kRecThreads);
  if (dtype == SFFT_C128) {
    hipLaunchKernelGGL(recover_kernel<double>, grid, block, 0, s, sig);
  } else {
    hipLaunchKernelGGL(recover_kernel<float>, grid, block, 0, s, sig);
  }
  return hipGetLastError();
}

}  // namespace sfft
