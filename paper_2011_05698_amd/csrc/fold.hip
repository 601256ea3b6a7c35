// Stage kernels of the fold: one workgroup per tile (device bodies in
// fold_body.h); union tiles and one-round tiles in kernels of their own.
#include <type_traits>

#include "fold_body.h"

namespace sfft {

template <class Ld, bool KAHAN, int U>
__global__ __launch_bounds__(kFoldTile) void fold_kernel(SigArg arg, const FoldTile* __restrict__ tiles) {
  const FoldTile tl = tiles[blockIdx.x];
  fold_tile<Ld, KAHAN, U>(load_signal(arg, tl.sig), tl);
}

template <class Ld, bool KAHAN, int U, int NU>
__global__ __launch_bounds__(kFoldTile) void fold_union_kernel(SigArg arg, const FoldTile* __restrict__ tiles) {
  const FoldTile tl = tiles[blockIdx.x];
  fold_union<Ld, KAHAN, U, NU>(load_signal(arg, tl.sig), fold_tile_iter(tl.m), tl.i0);
}

// P > 1: workgroup k takes tiles P k .. P k + P - 1, the same items of signal
// groups g .. g + P - 1 (g a multiple of P: the tile list puts a block's
// groups innermost and the host checks that their count is a multiple of P).
template <class Ld, bool KAHAN, int U, int P>
__global__ __launch_bounds__(256) void fold_interleaved_kernel(const SignalDesc* __restrict__ table, uint32_t nsig,
                                                               const FoldTile* __restrict__ tiles) {
  __shared__ IlvShared<typename Ld::R, P> sh;
  fold_tile_ilv<Ld, KAHAN, U, P>(table, nsig, tiles[P * blockIdx.x], sh);
}

int fold_lds_bytes(int wg_per_cu) {
  // 160 KiB of LDS per CU; reserving just over 1/(n+1) of it caps residency at n
  if (wg_per_cu <= 0) return 0;
  const int per = 163840 / (wg_per_cu + 1) + 1024;
  return per > 65536 ? 65536 : per;
}

template <class Ld, bool KAHAN, int U>
static void launch_one(uint32_t nu, uint32_t n, size_t lds, hipStream_t s, const SigArg& sig, const FoldTile* t) {
  const dim3 grid(n), block(kFoldTile);
  if (nu == 2) hipLaunchKernelGGL((fold_union_kernel<Ld, KAHAN, U, 2>), grid, block, lds, s, sig, t);
  else if (nu == 3) hipLaunchKernelGGL((fold_union_kernel<Ld, KAHAN, U, 3>), grid, block, lds, s, sig, t);
  else if (nu == 4) hipLaunchKernelGGL((fold_union_kernel<Ld, KAHAN, U, 4>), grid, block, lds, s, sig, t);
  else hipLaunchKernelGGL((fold_kernel<Ld, KAHAN, U>), grid, block, lds, s, sig, t);
}

template <class Ld, bool KAHAN>
static void launch_u(int unroll, uint32_t nu, uint32_t n, size_t lds, hipStream_t s, const SigArg& sig,
                     const FoldTile* t) {
  if (unroll >= 24) launch_one<Ld, KAHAN, 24>(nu, n, lds, s, sig, t);
  else if (unroll >= 16) launch_one<Ld, KAHAN, 16>(nu, n, lds, s, sig, t);
  else launch_one<Ld, KAHAN, 8>(nu, n, lds, s, sig, t);
}

int launch_fold(int dtype, int kahan, const FoldConfig& cfg, const SigArg& sig, const FoldTile* d_tiles,
                uint32_t ntiles, const FoldSplit& split, void* stream) {
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const size_t lds = size_t(fold_lds_bytes(cfg.wg_per_cu));
  uint32_t at = 0;
  for (uint32_t k = 0; k <= kMaxUnionRounds - 1; ++k) {
    // union tiles of k + 2 rounds, then (k = kMaxUnionRounds - 1) the one-round tiles
    const uint32_t nu = k < kMaxUnionRounds - 1 ? k + 2 : 1;
    const uint32_t n = k < kMaxUnionRounds - 1 ? split.nunion[k] : ntiles - at;
    if (n == 0) continue;
    const FoldTile* t = d_tiles + at;
    at += n;
    if (dtype == SFFT_C128) {
      if (kahan) launch_u<LoadC128, true>(cfg.unroll, nu, n, lds, s, sig, t);
      else launch_u<LoadC128, false>(cfg.unroll, nu, n, lds, s, sig, t);
    } else if (dtype == SFFT_F16X2_SCALED) {
      if (kahan) launch_u<LoadF16, true>(cfg.unroll, nu, n, lds, s, sig, t);
      else launch_u<LoadF16, false>(cfg.unroll, nu, n, lds, s, sig, t);
    } else {
      if (kahan) launch_u<LoadC64, true>(cfg.unroll, nu, n, lds, s, sig, t);
      else launch_u<LoadC64, false>(cfg.unroll, nu, n, lds, s, sig, t);
    }
  }
  return hipGetLastError();
}

template <class Ld, bool KAHAN, int P>
static void launch_ilv_u(int unroll, dim3 grid, hipStream_t s, const SignalDesc* table, uint32_t nsig,
                         const FoldTile* d_tiles) {
  const dim3 block(256);
  if (unroll >= 24) hipLaunchKernelGGL((fold_interleaved_kernel<Ld, KAHAN, 24, P>), grid, block, 0, s, table, nsig, d_tiles);
  else if (unroll >= 16) hipLaunchKernelGGL((fold_interleaved_kernel<Ld, KAHAN, 16, P>), grid, block, 0, s, table, nsig, d_tiles);
  else hipLaunchKernelGGL((fold_interleaved_kernel<Ld, KAHAN, 8, P>), grid, block, 0, s, table, nsig, d_tiles);
}

template <class Ld, bool KAHAN>
static void launch_ilv_p(int lanes, uint32_t ntiles, hipStream_t s, int unroll, const SignalDesc* table,
                         uint32_t nsig, const FoldTile* d_tiles) {
  if constexpr (std::is_same<Ld, LoadF16>::value) {
    if (lanes == 4) return launch_ilv_u<Ld, KAHAN, 4>(unroll, dim3(ntiles / 4), s, table, nsig, d_tiles);
  }
  if (lanes == 2) launch_ilv_u<Ld, KAHAN, 2>(unroll, dim3(ntiles / 2), s, table, nsig, d_tiles);
  else launch_ilv_u<Ld, KAHAN, 1>(unroll, dim3(ntiles), s, table, nsig, d_tiles);
}

int launch_fold_interleaved(int dtype, int kahan, int unroll, int lanes, const SignalDesc* table, uint32_t nsig,
                            const FoldTile* d_tiles, uint32_t ntiles, void* stream) {
  if (ntiles == 0 || nsig == 0) return hipSuccess;
  const uint32_t ngroups = (nsig + uint32_t(kIlvSigs) - 1) / uint32_t(kIlvSigs);
  const int most = dtype == SFFT_C128 ? 1 : dtype == SFFT_F16X2_SCALED ? 4 : 2;
  if ((lanes != 1 && lanes != 2 && lanes != 4) || lanes > most || ngroups % uint32_t(lanes) != 0 ||
      nsig % uint32_t(lanes) != 0)
    return hipErrorInvalidValue;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (dtype == SFFT_C128) {
    if (kahan) launch_ilv_u<LoadC128, true, 1>(unroll, dim3(ntiles), s, table, nsig, d_tiles);
    else launch_ilv_u<LoadC128, false, 1>(unroll, dim3(ntiles), s, table, nsig, d_tiles);
  } else if (dtype == SFFT_F16X2_SCALED) {
    if (kahan) launch_ilv_p<LoadF16, true>(lanes, ntiles, s, unroll, table, nsig, d_tiles);
    else launch_ilv_p<LoadF16, false>(lanes, ntiles, s, unroll, table, nsig, d_tiles);
  } else {
    if (kahan) launch_ilv_p<LoadC64, true>(lanes, ntiles, s, unroll, table, nsig, d_tiles);
    else launch_ilv_p<LoadC64, false>(lanes, ntiles, s, unroll, table, nsig, d_tiles);
  }
  return hipGetLastError();
}

}  // namespace sfft
