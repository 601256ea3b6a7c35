// The recovery stage kernel: one workgroup per signal runs recover_signal
// (recover_body.h) on the bucket values the fold and the bucket DFT wrote.
// A batch of more signals than the device has compute units takes the
// 256-thread shape, two workgroups per compute unit; a smaller batch (a
// single signal among them) takes the 512-thread shape with twice the LDS,
// one workgroup per compute unit.  Both give the same bits.
#include "recover_body.h"

namespace sfft {

template <typename R>
__global__ __launch_bounds__(kRecThreads, 2) void recover_kernel(SigArg arg) {
  __shared__ RecoverShared<R> sh;
  recover_signal<R>(load_signal(arg, blockIdx.x), sh);
}

template <typename R>
__global__ __launch_bounds__(kRecThreadsWide, 2) void recover_wide_kernel(SigArg arg) {
  __shared__ RecoverShared<R, kRecThreadsWide, kLdsBytesWide> sh;
  recover_signal<R>(load_signal(arg, blockIdx.x), sh);
}

// Compute units of the current device (read once per device).
static int device_cus() {
  constexpr int kMaxDev = 64;
  static int cus[kMaxDev] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDev) return 0;
  if (cus[dev] == 0) {
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && n > 0) cus[dev] = n;
  }
  return cus[dev];
}

int launch_recover(int dtype, const SigArg& sig, uint32_t nsig, void* stream) {
  if (nsig == 0) return hipSuccess;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const bool wide = nsig <= uint32_t(device_cus());
  dim3 grid(nsig), block(wide ? kRecThreadsWide : kRecThreads);
  if (dtype == SFFT_C128) {
    if (wide) hipLaunchKernelGGL(recover_wide_kernel<double>, grid, block, 0, s, sig);
    else hipLaunchKernelGGL(recover_kernel<double>, grid, block, 0, s, sig);
  } else {
    if (wide) hipLaunchKernelGGL(recover_wide_kernel<float>, grid, block, 0, s, sig);
    else hipLaunchKernelGGL(recover_kernel<float>, grid, block, 0, s, sig);
  }
  return hipGetLastError();
}

}  // namespace sfft
