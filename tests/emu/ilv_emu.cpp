// Runs the position-major fold body (fold_tile_ilv in fold_body.h, the code
// the GPU kernel runs) on the CPU through the emulation layer of hip_emu.h,
// for one plan and nsig seeded signals stored as X[c, s] (row stride ld),
// and checks it against the per-signal fold:
//   * reference: each signal copied to a contiguous buffer and folded by
//     one-round tiles (fold_tile) with 8 taps in flight;
//   * the position-major tile list (interleaved_tiles) with one signal per
//     lane, 8, 16 and 24 taps in flight;
//   * the same with two, then four, adjacent signals per lane (one
//     workgroup per two or four tiles), where the library allows that form:
//     two for complex64, two or four for FP16 pairs, with ld, the signal
//     count and the number of signal groups multiples of it.
// Every bucket array must equal the reference bit for bit and every item
// must be written.  X, the descriptor table, the plan tables, each signal's
// bucket array and the workgroup's LDS sit against an inaccessible guard
// page: past the end in guard mode 0, before the start in mode 1; an access
// outside a buffer stops the program (exit status 86).
//
// usage: ilv_emu N K B w loops l q delta seed dtype kahan guard_mode nsig ld
// dtype: 0 complex64, 1 complex128, 2 FP16 pairs with per-signal scales.
// Prints "ILV OK tiles <n> lanes <1|2|4>" and exits 0, or names the first
// mismatch and exits 1.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <type_traits>
#include <vector>

#include "fold_body.h"
#include "guarded.h"
#include "internal.h"

namespace sfft {
// host helpers of the C ABI that plan.cpp calls
void set_last_error(const std::string&) {}
void alloc_trial_begin() {}
bool alloc_should_fail() { return false; }
}  // namespace sfft

using namespace sfft;
using emu::galloc;
using emu::guard_init;
using emu::guard_mode;

namespace {

// SplitMix64: the samples, uniform in [-1, 1) per component
uint64_t mix(uint64_t& s) {
  uint64_t z = (s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
double uniform(uint64_t& s) { return double(mix(s) >> 11) * 0x1p-52 - 1.0; }

template <class Ld, bool KAHAN>
int run(const HostPlan& hp, uint64_t seed, uint32_t nsig, uint32_t ld) {
  using R = typename Ld::R;
  constexpr bool kF16 = std::is_same<Ld, LoadF16>::value;
  constexpr size_t es = kF16 ? sizeof(LoadF16::h2) : sizeof(cplx<R>);
  const size_t M = hp.iters.size();
  const uint64_t N = uint64_t(hp.N);
  auto* iters = static_cast<IterDesc*>(galloc(sizeof(IterDesc) * M, "iteration descriptors"));
  size_t nwin = 0;
  for (auto& it : hp.iters) nwin += it.G->size();
  auto* win = static_cast<R*>(galloc(nwin * sizeof(R), "window table"));
  size_t wi = 0;
  for (size_t m = 0; m < M; ++m) {
    iters[m] = hp.iters[m].d;
    for (double g : *hp.iters[m].G) win[wi++] = R(g);
  }
  auto* pd = static_cast<PlanDesc*>(galloc(sizeof(PlanDesc), "plan descriptor"));
  *pd = hp.desc;
  pd->iters = iters;
  pd->window = win;
  pd->ghat = nullptr;
  pd->twiddle = nullptr;

  // X[c, s] in the storage form; columns nsig .. ld - 1 hold samples too
  // (never read into a live signal's sums)
  auto* X = static_cast<unsigned char*>(galloc(N * ld * es, "position-major signals"));
  uint64_t st = seed;
  for (uint64_t e = 0; e < N * ld; ++e) {
    if constexpr (kF16) {
      auto* h = reinterpret_cast<LoadF16::h2*>(X) + e;
      h->x = _Float16(float(uniform(st)));
      h->y = _Float16(float(uniform(st)));
    } else {
      reinterpret_cast<cplx<R>*>(X)[e] = cplx<R>{R(uniform(st)), R(uniform(st))};
    }
  }
  const uint64_t ny = pd->y_total;
  std::vector<cplx<R>*> y(nsig);
  std::vector<std::vector<cplx<R>>> ref(nsig, std::vector<cplx<R>>(ny));
  auto* table = static_cast<SignalDesc*>(galloc(sizeof(SignalDesc) * nsig, "descriptor table"));
  for (uint32_t s = 0; s < nsig; ++s) {
    y[s] = static_cast<cplx<R>*>(galloc(ny * sizeof(cplx<R>), "bucket values"));
    SignalDesc& sd = table[s];
    std::memset(&sd, 0, sizeof sd);
    sd.plan = pd;
    sd.x = X + s * es;
    sd.y = y[s];
    sd.scale = kF16 ? 0.5f + 0.01f * float(s) : 1.0f;
    sd.ld = ld;
  }

  // reference: each signal contiguous, one-round tiles of the per-signal fold
  {
    auto* xc = static_cast<unsigned char*>(galloc(N * es, "contiguous signal"));
    for (uint32_t s = 0; s < nsig; ++s) {
      for (uint64_t c = 0; c < N; ++c) std::memcpy(xc + c * es, X + (c * ld + s) * es, es);
      SignalDesc sd = table[s];
      sd.x = xc;
      sd.ld = 0;
      std::memset(static_cast<void*>(y[s]), 0xFF, ny * sizeof(cplx<R>));
      for (size_t m = 0; m < M; ++m) {
        const uint32_t n = (hp.iters[m].d.R + 1) * hp.iters[m].d.B;
        for (uint32_t i0 = 0; i0 < n; i0 += kFoldTile) {
          blockDim = EmuDim3{uint32_t(kFoldTile), 1, 1};
          for (uint32_t t = 0; t < uint32_t(kFoldTile); ++t) {
            threadIdx = EmuDim3{t, 0, 0};
            fold_tile<Ld, KAHAN, 8>(sd, FoldTile{s, uint32_t(m), i0});
          }
        }
      }
      std::memcpy(static_cast<void*>(ref[s].data()), y[s], ny * sizeof(cplx<R>));
    }
  }

  const uint32_t ngroups = (nsig + kIlvSigs - 1) / kIlvSigs;
  std::vector<FoldTile> tiles;
  interleaved_tiles(hp, ngroups, tiles);
  auto* d_tiles = static_cast<FoldTile*>(galloc(sizeof(FoldTile) * tiles.size(), "tile list"));
  std::memcpy(d_tiles, tiles.data(), sizeof(FoldTile) * tiles.size());
  // the library's test for L signals per lane
  int lanes = 1;
  const int most = std::is_same<Ld, LoadC128>::value ? 1 : kF16 ? 4 : 2;
  for (int L : {4, 2})
    if (L <= most && ngroups % uint32_t(L) == 0 && nsig % uint32_t(L) == 0 && ld % uint32_t(L) == 0 &&
        reinterpret_cast<uintptr_t>(X) % (uint64_t(L) * es) == 0) {
      lanes = L;
      break;
    }

  auto check = [&](const char* what) -> bool {
    cplx<R> ones;
    std::memset(static_cast<void*>(&ones), 0xFF, sizeof ones);
    for (uint32_t s = 0; s < nsig; ++s)
      for (uint64_t i = 0; i < ny; ++i) {
        if (std::memcmp(&y[s][i], &ones, sizeof ones) == 0) {
          std::printf("%s left signal %u item %llu unwritten\n", what, s, (unsigned long long)i);
          return false;
        }
        if (std::memcmp(&y[s][i], &ref[s][i], sizeof(cplx<R>)) != 0) {
          std::printf("%s differs at signal %u item %llu: (%.17g, %.17g) vs (%.17g, %.17g)\n", what, s,
                      (unsigned long long)i, double(y[s][i].re), double(y[s][i].im), double(ref[s][i].re),
                      double(ref[s][i].im));
          return false;
        }
      }
    return true;
  };
  auto launch = [&](auto u, auto p) -> bool {
    constexpr int U = decltype(u)::value, P = decltype(p)::value;
    for (uint32_t s = 0; s < nsig; ++s) std::memset(static_cast<void*>(y[s]), 0xFF, ny * sizeof(cplx<R>));
    auto* sh = static_cast<IlvShared<R, P>*>(galloc(sizeof(IlvShared<R, P>), "workgroup LDS"));
    const uint32_t nblk = uint32_t(tiles.size()) / P;
    for (uint32_t k = 0; k < nblk; ++k)
      emu_run_block(256, k, [&] { fold_tile_ilv<Ld, KAHAN, U, P>(table, nsig, d_tiles[P * k], *sh); });
    char what[64];
    std::snprintf(what, sizeof what, "position-major, %d per lane, %d taps", P, U);
    return check(what);
  };
  using one = std::integral_constant<int, 1>;
  using two = std::integral_constant<int, 2>;
  using four = std::integral_constant<int, 4>;
  if (!launch(std::integral_constant<int, 8>{}, one{})) return 1;
  if (!launch(std::integral_constant<int, 16>{}, one{})) return 1;
  if (!launch(std::integral_constant<int, 24>{}, one{})) return 1;
  if constexpr (!std::is_same<Ld, LoadC128>::value) {
    if (lanes >= 2) {
      if (!launch(std::integral_constant<int, 8>{}, two{})) return 1;
      if (!launch(std::integral_constant<int, 16>{}, two{})) return 1;
      if (!launch(std::integral_constant<int, 24>{}, two{})) return 1;
    }
  }
  if constexpr (kF16) {
    if (lanes == 4) {
      if (!launch(std::integral_constant<int, 8>{}, four{})) return 1;
      if (!launch(std::integral_constant<int, 16>{}, four{})) return 1;
      if (!launch(std::integral_constant<int, 24>{}, four{})) return 1;
    }
  }
  std::printf("ILV OK tiles %zu lanes %d\n", tiles.size(), lanes);
  return 0;
}

}  // namespace

int main(int argc, char** argv) {
  if (argc != 15) {
    std::fprintf(stderr, "usage: %s N K B w loops l q delta seed dtype kahan guard_mode nsig ld\n", argv[0]);
    return 2;
  }
  guard_init();
  const int64_t N = std::atoll(argv[1]), K = std::atoll(argv[2]), B = std::atoll(argv[3]), w = std::atoll(argv[4]);
  const int32_t loops = std::atoi(argv[5]), l = std::atoi(argv[6]);
  const double q = std::atof(argv[7]), delta = std::atof(argv[8]);
  const uint64_t seed = std::strtoull(argv[9], nullptr, 10);
  const int32_t dtype = std::atoi(argv[10]), kahan = std::atoi(argv[11]);
  guard_mode() = std::atoi(argv[12]);
  const uint32_t nsig = uint32_t(std::atoi(argv[13])), ld = uint32_t(std::atoi(argv[14]));
  if (nsig < 1 || ld < nsig) {
    std::fprintf(stderr, "need 1 <= nsig <= ld\n");
    return 2;
  }
  sfft_options opt{};
  opt.delta = delta;
  opt.seed = seed;
  opt.dtype = dtype;
  opt.kahan = kahan;
  opt.b_min = 16;
  opt.eta = 1e-4;
  opt.rho = 0.25;
  HostPlan hp;
  std::string err;
  if (build_host_plan(hp, N, K, B, w, loops, l, q, opt, &err) != SFFT_OK) {
    std::fprintf(stderr, "plan: %s\n", err.c_str());
    return 2;
  }
  layout_workspace(hp);
  if (dtype == SFFT_C128)
    return kahan ? run<LoadC128, true>(hp, seed, nsig, ld) : run<LoadC128, false>(hp, seed, nsig, ld);
  if (dtype == SFFT_F16X2_SCALED)
    return kahan ? run<LoadF16, true>(hp, seed, nsig, ld) : run<LoadF16, false>(hp, seed, nsig, ld);
  return kahan ? run<LoadC64, true>(hp, seed, nsig, ld) : run<LoadC64, false>(hp, seed, nsig, ld);
}
