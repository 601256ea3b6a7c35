// The B-point DFT with its 1/N factor (Eq. 12-13 reading) for 16 <= B <= 2048,
// one wavefront per chunk of rounds, with the data in registers.
//
// B = R1 x L1 with R1 = 2^floor(log2 B / 2) and L1 = B / R1 (= R1 or 2 R1,
// at most 64): a round spans L1 lanes, so a wave holds 64 / L1 rounds.
// Writing n = L1 n1 + n2 and k = k1 + R1 k2 (Cooley-Tukey):
//   pass 1: lane n2 holds x[L1 n1 + n2], n1 < R1 (coalesced loads), and
//           takes their R1-point DFT in registers (radix 2, unrolled);
//           then the twiddle W_B^{n2 k1};
//   LDS:    the R1 x L1 results go through a padded LDS tile of the wave
//           (row stride L1 + 1, or L1 + 2 when L1 = 2 R1, so that the lanes
//           of a read do not share banks);
//   pass 2: each k1 takes the L1-point DFT over n2: when L1 = R1 one lane
//           does it in registers; when L1 = 2 R1 two neighbouring lanes
//           each do the R1-point DFT of the even or the odd n2, and a DPP
//           exchange between the two lanes closes the last radix-2 stage;
//   stores: lane k1 writes k = k1 + R1 k2, so consecutive lanes write
//           consecutive buckets.
// The roots inside the in-register DFTs (orders up to 64) are compile-time
// constants; the twiddles W_B^{n2 k1} between the passes come from an LDS
// copy of the plan's table of B/2 values exp(-2 pi i j / B) (the other half
// by W_B^{j + B/2} = -W_B^j).
#pragma once

#include "device_common.h"

namespace sfft {

// B <= 2048 (32 values per lane); complex128 up to 512 so that four wave
// tiles and the twiddles fit in 78,848 bytes of LDS
template <typename R>
__host__ __device__ constexpr uint32_t wave_fft_max_logB() {
  return sizeof(R) == 8 ? kWaveFftMaxLogB64 : kWaveFftMaxLogB32;
}

template <typename R>
__device__ __forceinline__ cplx<R> tw_at(const cplx<R>* tw, uint32_t j, uint32_t B) {
  const uint32_t half = B >> 1;
  const cplx<R> w = tw[j < half ? j : j - half];
  return j < half ? w : cplx<R>{-w.re, -w.im};
}

template <int C>
__device__ __forceinline__ constexpr int bitrev_c(int i) {
  int r = 0;
  for (int b = 0; b < C; ++b) r |= ((i >> b) & 1) << (C - 1 - b);
  return r;
}

// cos(2 pi k / 64) for k = 0..16, correctly rounded to double
__device__ constexpr double kCos64[17] = {1.0,
                                          0.9951847266721969,
                                          0.9807852804032304,
                                          0.9569403357322088,
                                          0.9238795325112867,
                                          0.881921264348355,
                                          0.8314696123025452,
                                          0.773010453362737,
                                          0.7071067811865476,
                                          0.6343932841636455,
                                          0.5555702330196022,
                                          0.47139673682599764,
                                          0.3826834323650898,
                                          0.2902846772544624,
                                          0.19509032201612828,
                                          0.0980171403295606,
                                          0.0};

// x W_64^K (K < 64) with the root exp(-2 pi i K / 64) known at compile time:
// its quadrant by symmetry, and no multiplication for 1 and -i.
template <typename R, int K>
__device__ __forceinline__ cplx<R> mul_w64(cplx<R> x) {
  static_assert(K >= 0 && K < 64, "root index");
  if constexpr (K == 0) {
    return x;
  } else if constexpr (K == 16) {
    return cplx<R>{x.im, -x.re};
  } else {
    constexpr double c = K <= 16 ? kCos64[K] : K <= 32 ? -kCos64[32 - K] : K <= 48 ? -kCos64[K - 32] : kCos64[64 - K];
    constexpr double s = K <= 16 ? -kCos64[16 - K] : K <= 32 ? -kCos64[K - 16] : K <= 48 ? kCos64[48 - K] : kCos64[K - 48];
    return cmul(x, cplx<R>{R(c), R(s)});
  }
}

// One radix-2 stage of span H of an in-register DFT of 2^C points, from
// position P of every butterfly group on; twiddle W_{2H}^P = W_64^{32 P / H}.
template <typename R, int C, int H, int P = 0>
__device__ __forceinline__ void lane_dft_stage(cplx<R> (&v)[1 << C]) {
  if constexpr (P < H) {
#pragma unroll
    for (int k = 0; k < (1 << C); k += 2 * H) {
      const cplx<R> a = v[k + P], b = mul_w64<R, P * (32 / H)>(v[k + P + H]);
      v[k + P] = cadd(a, b);
      v[k + P + H] = csub(a, b);
    }
    lane_dft_stage<R, C, H, P + 1>(v);
  }
}

template <typename R, int C, int H = 1>
__device__ __forceinline__ void lane_dft_stages(cplx<R> (&v)[1 << C]) {
  if constexpr (H < (1 << C)) {
    lane_dft_stage<R, C, H>(v);
    lane_dft_stages<R, C, 2 * H>(v);
  }
}

// v[k] W_64^{k S} for every k, where `on`; left as is elsewhere.
template <typename R, int N, int S, int K = 0>
__device__ __forceinline__ void mul_w64_ramp(cplx<R> (&v)[N], bool on) {
  if constexpr (K < N) {
    const cplx<R> t = mul_w64<R, (K * S) % 64>(v[K]);
    v[K].re = on ? t.re : v[K].re;  // selects of scalars: a select of the
    v[K].im = on ? t.im : v[K].im;  // structs would keep v in scratch
    mul_w64_ramp<R, N, S, K + 1>(v, on);
  }
}

// In-register forward DFT of 2^C points (C <= 5), natural order in and
// out: a compile-time bit-reversal, then radix-2 stages with compile-time
// twiddles.
template <typename R, int C>
__device__ __forceinline__ void lane_dft(cplx<R> (&v)[1 << C]) {
  constexpr int N = 1 << C;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    const int j = bitrev_c<C>(i);
    if (j > i) {
      const cplx<R> t = v[i];
      v[i] = v[j];
      v[j] = t;
    }
  }
  lane_dft_stages<R, C>(v);
}

// The value of lane ^ 1 (DPP quad permutation [1, 0, 3, 2]).
template <typename R>
__device__ __forceinline__ R dpp_xor1(R x) {
  if constexpr (sizeof(R) == 4) {
    return __builtin_bit_cast(R, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), 0xB1, 0xF, 0xF, false));
  } else {
    const uint64_t u = __builtin_bit_cast(uint64_t, x);
    const uint32_t lo = uint32_t(__builtin_amdgcn_update_dpp(0, int(uint32_t(u)), 0xB1, 0xF, 0xF, false));
    const uint32_t hi = uint32_t(__builtin_amdgcn_update_dpp(0, int(uint32_t(u >> 32)), 0xB1, 0xF, 0xF, false));
    return __builtin_bit_cast(R, (uint64_t(hi) << 32) | lo);
  }
}

// Row stride of a wave tile, in values: L1 + 1 when L1 = R1, L1 + 2 when
// L1 = 2 R1.  Pass 2 reads column pairs (2m + h) of rows k1 across the lane
// pairs (k1, h): with an odd stride the rows of k1 and k1 + 1 fall on the
// banks that h = 1 reads, with L1 + 2 they do not.
__host__ __device__ constexpr uint32_t wave_fft_tile_stride(uint32_t logB) {
  return (1u << (logB - logB / 2)) + 1u + (logB & 1u);
}

// LDS a wave needs for rounds of 2^logB points: its tile (64 / L1 rounds of
// R1 rows).
__host__ __device__ constexpr uint32_t wave_fft_tile_elems(uint32_t logB) {
  return (64u >> (logB - logB / 2)) * (1u << (logB / 2)) * wave_fft_tile_stride(logB);
}

// One chunk of up to 64 / L1 rounds of B = 2^(2C + E) points (E = 0 or 1)
// by the calling wave.  row(r) is round r's array (r < nr), inv(r) its 1/N;
// tile is this wave's LDS tile, tw the LDS twiddle table.
template <typename R, int C, int E, class Row, class Inv>
__device__ __forceinline__ void wave_fft_chunk(uint32_t nr, Row row, Inv inv, cplx<R>* tile, const cplx<R>* tw) {
  constexpr uint32_t R1 = 1u << C, L1 = R1 << E, B = R1 * L1, LPK = 1u << E;
  constexpr uint32_t S = wave_fft_tile_stride(2 * C + E);
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t r = lane / L1, q = lane % L1;  // round slot, index within the round
  const bool live = r < nr;
  cplx<R>* T = tile + r * R1 * S;
  cplx<R> v[R1];
  // pass 1: lane n2 = q takes x[L1 n1 + n2]
  if (live) {
    const cplx<R>* x = row(r);
#pragma unroll
    for (uint32_t n1 = 0; n1 < R1; ++n1) v[n1] = x[L1 * n1 + q];
  }
  lane_dft<R, C>(v);
#pragma unroll
  for (uint32_t k1 = 1; k1 < R1; ++k1) v[k1] = cmul(v[k1], tw_at(tw, q * k1, B));
  if (live) {
#pragma unroll
    for (uint32_t k1 = 0; k1 < R1; ++k1) T[k1 * S + q] = v[k1];
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  // pass 2: lane q = LPK k1 + h takes n2 = LPK m + h, m < R1
  const uint32_t k1 = q / LPK, h = q % LPK;
  if (live) {
#pragma unroll
    for (uint32_t m = 0; m < R1; ++m) v[m] = T[k1 * S + LPK * m + h];
  }
  lane_dft<R, C>(v);  // R1-point DFT over m
  if constexpr (E == 1) {
    // the last radix-2 stage across the lane pair: Z[k1 + R1 (k2 + R1 s)] =
    // even[k2] + (-1)^s W_{L1}^{k2} odd[k2]; lane h = s keeps output half s
    mul_w64_ramp<R, int(R1), 64 / int(L1)>(v, h == 1);  // odd half: W_L1^{k2}
#pragma unroll
    for (uint32_t k2 = 0; k2 < R1; ++k2) {
      const cplx<R> o{dpp_xor1(v[k2].re), dpp_xor1(v[k2].im)};
      const cplx<R> sum = cadd(v[k2], o), dif = csub(o, v[k2]);
      v[k2].re = h == 0 ? sum.re : dif.re;
      v[k2].im = h == 0 ? sum.im : dif.im;
    }
  }
  if (live) {
    cplx<R>* y = row(r);
    const R s = inv(r);
#pragma unroll
    for (uint32_t k2 = 0; k2 < R1; ++k2) y[k1 + R1 * (k2 + R1 * h)] = cscale(v[k2], s);
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The calling wave's chunks of n rounds of B = 2^(2C + E) points: the
// waves of the block take chunks of 64 / L1 rounds in turn.
template <typename R, int C, int E, class Row, class Inv>
__device__ void wave_fft_loop(uint32_t n, Row row, Inv inv, cplx<R>* tiles, const cplx<R>* tw) {
  constexpr uint32_t logB = 2 * C + E, rpw = 64u >> (C + E);
  const uint32_t wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
  cplx<R>* tile = tiles + wave * wave_fft_tile_elems(logB);
  for (uint32_t r0 = wave * rpw; r0 < n; r0 += nwaves * rpw) {
    wave_fft_chunk<R, C, E>(
        min(rpw, n - r0), [&](uint32_t r) { return row(r0 + r); }, [&](uint32_t r) { return inv(r0 + r); }, tile, tw);
  }
}

// n rounds of B = 2^logB points (16 <= B <= 2048) by the whole block.  tw
// is an LDS copy of the B/2 twiddles; tiles holds blockDim.x / 64 wave
// tiles of wave_fft_tile_elems(logB).
template <typename R, class Row, class Inv>
__device__ void wave_fft_rounds(uint32_t n, uint32_t logB, Row row, Inv inv, cplx<R>* tiles, const cplx<R>* tw) {
  constexpr uint32_t kMax = wave_fft_max_logB<R>();
  switch (logB) {
    case 4: wave_fft_loop<R, 2, 0>(n, row, inv, tiles, tw); break;
    case 5: wave_fft_loop<R, 2, 1>(n, row, inv, tiles, tw); break;
    case 6: wave_fft_loop<R, 3, 0>(n, row, inv, tiles, tw); break;
    case 7: wave_fft_loop<R, 3, 1>(n, row, inv, tiles, tw); break;
    case 8: wave_fft_loop<R, 4, 0>(n, row, inv, tiles, tw); break;
    case 9: wave_fft_loop<R, 4, 1>(n, row, inv, tiles, tw); break;
    case 10: if constexpr (kMax >= 10) wave_fft_loop<R, 5, 0>(n, row, inv, tiles, tw); break;
    case 11: if constexpr (kMax >= 11) wave_fft_loop<R, 5, 1>(n, row, inv, tiles, tw); break;
    default: break;
  }
}

}  // namespace sfft

namespace sfft {

// LDS of wave_fft_rounds for rounds of 2^logB points and `waves` waves:
// the B/2 twiddles, then one tile per wave.
__host__ __device__ constexpr uint32_t wave_fft_lds_elems(uint32_t logB, uint32_t waves) {
  return (1u << (logB - 1)) + waves * wave_fft_tile_elems(logB);
}

}  // namespace sfft
