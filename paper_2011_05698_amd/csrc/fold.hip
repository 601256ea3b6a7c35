// Stage kernels of the fold: one workgroup per tile (device bodies in fold_body.h).
#include "fold_body.h"

namespace sfft {

template <class Ld, bool KAHAN, int U>
__global__ __launch_bounds__(kFoldTile) void fold_kernel(SigArg arg, const FoldTile* __restrict__ tiles) {
  const FoldTile tl = tiles[blockIdx.x];
  fold_tile<Ld, KAHAN, U>(load_signal(arg, tl.sig), tl);
}

template <class Ld, bool KAHAN, int U>
__global__ __launch_bounds__(256) void fold_interleaved_kernel(const SignalDesc* __restrict__ table, uint32_t nsig,
                                                               const FoldTile* __restrict__ tiles) {
  __shared__ IlvShared<typename Ld::R> sh;
  fold_tile_ilv<Ld, KAHAN, U>(table, nsig, tiles[blockIdx.x], sh);
}

int fold_lds_bytes(int wg_per_cu) {
  // 160 KiB of LDS per CU; reserving just over 1/(n+1) of it caps residency at n
  if (wg_per_cu <= 0) return 0;
  const int per = 163840 / (wg_per_cu + 1) + 1024;
  return per > 65536 ? 65536 : per;
}

template <class Ld, bool KAHAN>
static void launch_u(int unroll, dim3 grid, dim3 block, size_t lds, hipStream_t s, const SigArg& sig,
                     const FoldTile* d_tiles) {
  if (unroll >= 24) hipLaunchKernelGGL((fold_kernel<Ld, KAHAN, 24>), grid, block, lds, s, sig, d_tiles);
  else if (unroll >= 16) hipLaunchKernelGGL((fold_kernel<Ld, KAHAN, 16>), grid, block, lds, s, sig, d_tiles);
  else hipLaunchKernelGGL((fold_kernel<Ld, KAHAN, 8>), grid, block, lds, s, sig, d_tiles);
}

int launch_fold(int dtype, int kahan, const FoldConfig& cfg, const SigArg& sig, const FoldTile* d_tiles,
                uint32_t ntiles, void* stream) {
  if (ntiles == 0) return hipSuccess;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const dim3 grid(ntiles), block(kFoldTile);
  const size_t lds = size_t(fold_lds_bytes(cfg.wg_per_cu));
  if (dtype == SFFT_C128) {
    if (kahan) launch_u<LoadC128, true>(cfg.unroll, grid, block, lds, s, sig, d_tiles);
    else launch_u<LoadC128, false>(cfg.unroll, grid, block, lds, s, sig, d_tiles);
  } else if (dtype == SFFT_F16X2_SCALED) {
    if (kahan) launch_u<LoadF16, true>(cfg.unroll, grid, block, lds, s, sig, d_tiles);
    else launch_u<LoadF16, false>(cfg.unroll, grid, block, lds, s, sig, d_tiles);
  } else {
    if (kahan) launch_u<LoadC64, true>(cfg.unroll, grid, block, lds, s, sig, d_tiles);
    else launch_u<LoadC64, false>(cfg.unroll, grid, block, lds, s, sig, d_tiles);
  }
  return hipGetLastError();
}

template <class Ld, bool KAHAN>
static void launch_ilv_u(int unroll, dim3 grid, hipStream_t s, const SignalDesc* table, uint32_t nsig,
                         const FoldTile* d_tiles) {
  const dim3 block(256);
  if (unroll >= 24) hipLaunchKernelGGL((fold_interleaved_kernel<Ld, KAHAN, 24>), grid, block, 0, s, table, nsig, d_tiles);
  else if (unroll >= 16) hipLaunchKernelGGL((fold_interleaved_kernel<Ld, KAHAN, 16>), grid, block, 0, s, table, nsig, d_tiles);
  else hipLaunchKernelGGL((fold_interleaved_kernel<Ld, KAHAN, 8>), grid, block, 0, s, table, nsig, d_tiles);
}

int launch_fold_interleaved(int dtype, int kahan, int unroll, const SignalDesc* table, uint32_t nsig,
                            const FoldTile* d_tiles, uint32_t ntiles, void* stream) {
  if (ntiles == 0 || nsig == 0) return hipSuccess;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const dim3 grid(ntiles);
  if (dtype == SFFT_C128) {
    if (kahan) launch_ilv_u<LoadC128, true>(unroll, grid, s, table, nsig, d_tiles);
    else launch_ilv_u<LoadC128, false>(unroll, grid, s, table, nsig, d_tiles);
  } else if (dtype == SFFT_F16X2_SCALED) {
    if (kahan) launch_ilv_u<LoadF16, true>(unroll, grid, s, table, nsig, d_tiles);
    else launch_ilv_u<LoadF16, false>(unroll, grid, s, table, nsig, d_tiles);
  } else {
    if (kahan) launch_ilv_u<LoadC64, true>(unroll, grid, s, table, nsig, d_tiles);
    else launch_ilv_u<LoadC64, false>(unroll, grid, s, table, nsig, d_tiles);
  }
  return hipGetLastError();
}

}  // namespace sfft
