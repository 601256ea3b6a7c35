// Runs the per-signal fold bodies (fold_body.h, the code the GPU kernels
// run) on the CPU through the emulation layer of hip_emu.h, for one plan and
// one seeded signal, and checks that the union tiles change no bit:
//   * reference: every (round, bucket) item of every iteration through
//     one-round tiles (fold_tile) with 8 taps in flight;
//   * the same with 16 and 24 taps in flight;
//   * the tile list the library launches (build_work_lists, union tiles
//     included) through fold_tile_any, with 8, 16 and 24 taps in flight.
// Every bucket array must equal the reference bit for bit, and every item
// must be written.  Every buffer the fold reads or writes (signal, plan and
// iteration descriptors, window table, bucket values) sits against an
// inaccessible guard page: past its end in guard mode 0, before its start in
// mode 1; an access outside a buffer stops the program (exit status 86).
//
// usage: fold_emu N K B w loops l q delta seed dtype kahan guard_mode
// dtype: 0 complex64, 1 complex128, 2 FP16 pairs with a scale.
// Prints "FOLD OK tiles <n> union <u> items <i>" and exits 0, or names the
// first mismatch and exits 1.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
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

// SplitMix64: the signal's samples, uniform in [-1, 1) per component
uint64_t mix(uint64_t& s) {
  uint64_t z = (s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
double uniform(uint64_t& s) { return double(mix(s) >> 11) * 0x1p-52 - 1.0; }

// A fold tile has no barrier, wave move or shared memory: its threads run
// one after another on the calling thread.
template <typename F>
void run_tile(F&& body) {
  blockDim = EmuDim3{uint32_t(kFoldTile), 1, 1};
  blockIdx = EmuDim3{0, 0, 0};
  for (uint32_t t = 0; t < uint32_t(kFoldTile); ++t) {
    threadIdx = EmuDim3{t, 0, 0};
    body();
  }
}

template <class Ld, bool KAHAN>
int run(const HostPlan& hp, uint64_t seed) {
  using R = typename Ld::R;
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

  // the signal in its storage form
  void* x = nullptr;
  float scale = 1.0f;
  uint64_t st = seed;
  if (std::is_same<Ld, LoadF16>::value) {
    auto* h = static_cast<LoadF16::h2*>(galloc(N * sizeof(LoadF16::h2), "signal"));
    for (uint64_t i = 0; i < N; ++i) {
      h[i].x = _Float16(float(uniform(st)));
      h[i].y = _Float16(float(uniform(st)));
    }
    scale = 0.75f;
    x = h;
  } else {
    auto* c = static_cast<cplx<R>*>(galloc(N * sizeof(cplx<R>), "signal"));
    for (uint64_t i = 0; i < N; ++i) c[i] = cplx<R>{R(uniform(st)), R(uniform(st))};
    x = c;
  }

  const uint64_t ny = pd->y_total;
  auto* y = static_cast<cplx<R>*>(galloc(ny * sizeof(cplx<R>), "bucket values"));
  std::vector<cplx<R>> ref(ny);
  SignalDesc sd{};
  sd.plan = pd;
  sd.x = x;
  sd.y = y;
  sd.scale = scale;

  // the library's per-signal tile list (union tiles where the plan has them)
  std::vector<FoldTile> tiles;
  std::vector<RoundItem> items;
  build_work_lists(hp, 0, tiles, items);
  uint32_t nunion = 0;
  for (const FoldTile& t : tiles) nunion += fold_tile_rounds(t.m) >= 2 ? 1u : 0u;

  auto one_round = [&](auto u) {
    constexpr int U = decltype(u)::value;
    for (size_t m = 0; m < M; ++m) {
      const uint32_t n = (hp.iters[m].d.R + 1) * hp.iters[m].d.B;
      for (uint32_t i0 = 0; i0 < n; i0 += kFoldTile)
        run_tile([&] { fold_tile<Ld, KAHAN, U>(sd, FoldTile{0, uint32_t(m), i0}); });
    }
  };
  auto listed = [&](auto u) {
    constexpr int U = decltype(u)::value;
    for (const FoldTile& t : tiles) run_tile([&] { fold_tile_any<Ld, KAHAN, U>(sd, t); });
  };
  // every item written: the array starts as all-ones bytes (a NaN pattern)
  auto fill = [&] { std::memset(static_cast<void*>(y), 0xFF, ny * sizeof(cplx<R>)); };
  auto unwritten = [&]() -> uint64_t {
    cplx<R> ones;
    std::memset(static_cast<void*>(&ones), 0xFF, sizeof ones);
    for (uint64_t i = 0; i < ny; ++i)
      if (std::memcmp(&y[i], &ones, sizeof ones) == 0) return i;
    return ny;
  };

  fill();
  one_round(std::integral_constant<int, 8>{});
  if (uint64_t u = unwritten(); u != ny) {
    std::printf("reference left item %llu unwritten\n", (unsigned long long)u);
    return 1;
  }
  std::memcpy(static_cast<void*>(ref.data()), y, ny * sizeof(cplx<R>));

  auto compare = [&](const char* what) -> bool {
    if (uint64_t u = unwritten(); u != ny) {
      std::printf("%s left item %llu unwritten\n", what, (unsigned long long)u);
      return false;
    }
    for (uint64_t i = 0; i < ny; ++i)
      if (std::memcmp(&y[i], &ref[i], sizeof(cplx<R>)) != 0) {
        std::printf("%s differs at item %llu: (%.17g, %.17g) vs (%.17g, %.17g)\n", what, (unsigned long long)i,
                    double(y[i].re), double(y[i].im), double(ref[i].re), double(ref[i].im));
        return false;
      }
    return true;
  };
  fill();
  one_round(std::integral_constant<int, 16>{});
  if (!compare("one-round tiles, 16 taps")) return 1;
  fill();
  one_round(std::integral_constant<int, 24>{});
  if (!compare("one-round tiles, 24 taps")) return 1;
  fill();
  listed(std::integral_constant<int, 8>{});
  if (!compare("tile list, 8 taps")) return 1;
  fill();
  listed(std::integral_constant<int, 16>{});
  if (!compare("tile list, 16 taps")) return 1;
  fill();
  listed(std::integral_constant<int, 24>{});
  if (!compare("tile list, 24 taps")) return 1;
  std::printf("FOLD OK tiles %zu union %u items %llu\n", tiles.size(), nunion, (unsigned long long)ny);
  return 0;
}

}  // namespace

int main(int argc, char** argv) {
  if (argc != 13) {
    std::fprintf(stderr, "usage: %s N K B w loops l q delta seed dtype kahan guard_mode\n", argv[0]);
    return 2;
  }
  guard_init();
  const int64_t N = std::atoll(argv[1]), K = std::atoll(argv[2]), B = std::atoll(argv[3]), w = std::atoll(argv[4]);
  const int32_t loops = std::atoi(argv[5]), l = std::atoi(argv[6]);
  const double q = std::atof(argv[7]), delta = std::atof(argv[8]);
  const uint64_t seed = std::strtoull(argv[9], nullptr, 10);
  const int32_t dtype = std::atoi(argv[10]), kahan = std::atoi(argv[11]);
  guard_mode() = std::atoi(argv[12]);
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
  if (dtype == SFFT_C128) return kahan ? run<LoadC128, true>(hp, seed) : run<LoadC128, false>(hp, seed);
  if (dtype == SFFT_F16X2_SCALED) return kahan ? run<LoadF16, true>(hp, seed) : run<LoadF16, false>(hp, seed);
  return kahan ? run<LoadC64, true>(hp, seed) : run<LoadC64, false>(hp, seed);
}
