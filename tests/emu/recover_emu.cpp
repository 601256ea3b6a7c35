// Runs the recovery kernel body (recover_body.h, the code the GPU kernels
// run) on the CPU through the emulation layer of hip_emu.h, in both
// workgroup shapes (256 and 512 threads, which must give the same bits; exit
// status 4 if they do not), for one signal
// whose bucket values are given, with every buffer the kernel reads or
// writes placed against an inaccessible guard page.  An access past the end
// (guard mode 0) or before the start (guard mode 1) of any buffer stops the
// program with a message naming the buffer and the distance, and exit
// status 86.
//
// Input file (little-endian): int64 N, K, B, w; int32 loops, l; double q,
// delta; uint64 seed; int32 dtype, location, combine, guard_mode; int64 ny;
// then ny complex values as (double re, double im): the bucket values of
// every round of every iteration, iteration after iteration, round after
// round, B values each (the plan's y layout).
// Output file: int64 count, then count entries of (int64 f, double re,
// double im).
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "guarded.h"
#include "internal.h"
#include "recover_body.h"

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

template <typename T>
void rd(FILE* f, T* v, size_t n = 1) {
  if (std::fread(v, sizeof(T), n, f) != n) {
    std::fprintf(stderr, "short input\n");
    std::exit(2);
  }
}

template <typename R>
int run(HostPlan& hp, const std::vector<double>& y_in, FILE* out) {
  const size_t M = hp.iters.size();
  auto* iters = static_cast<IterDesc*>(galloc(sizeof(IterDesc) * M, "iteration descriptors"));
  size_t nwin = 0, nghat = 0, ntw = 0;
  for (auto& it : hp.iters) {
    nwin += it.G->size();
    nghat += it.Ghat->size();
    ntw += it.d.B / 2;
  }
  auto* win = static_cast<R*>(galloc(nwin * sizeof(R), "window table"));
  auto* ghat = static_cast<R*>(galloc(nghat * sizeof(R), "window spectrum table"));
  auto* tw = static_cast<R*>(galloc(ntw * 2 * sizeof(R), "twiddle table"));
  size_t wi = 0, gi = 0;
  for (size_t m = 0; m < M; ++m) {
    iters[m] = hp.iters[m].d;
    for (double g : *hp.iters[m].G) win[wi++] = R(g);
    for (double g : *hp.iters[m].Ghat) ghat[gi++] = R(g);
  }
  auto* pd = static_cast<PlanDesc*>(galloc(sizeof(PlanDesc), "plan descriptor"));
  *pd = hp.desc;
  pd->iters = iters;
  pd->window = win;
  pd->ghat = ghat;
  pd->twiddle = tw;
  if (y_in.size() != 2 * size_t(pd->y_total)) {
    std::fprintf(stderr, "expected %llu bucket values, got %zu\n", (unsigned long long)pd->y_total, y_in.size() / 2);
    return 2;
  }
  auto* y = static_cast<cplx<R>*>(galloc(pd->y_total * sizeof(cplx<R>), "bucket values"));
  for (size_t i = 0; i < pd->y_total; ++i) y[i] = cplx<R>{R(y_in[2 * i]), R(y_in[2 * i + 1])};
  void* ws = galloc(pd->ws_bytes, "signal workspace");
  auto* idx = static_cast<int64_t*>(galloc(sizeof(int64_t) * pd->K, "output frequencies"));
  auto* val = static_cast<cplx<R>*>(galloc(sizeof(cplx<R>) * pd->K, "output values"));
  auto* count = static_cast<int64_t*>(galloc(sizeof(int64_t), "output count"));
  auto* sh = static_cast<RecoverShared<R>*>(galloc(sizeof(RecoverShared<R>), "workgroup LDS"));
  SignalDesc sd{};
  sd.plan = pd;
  sd.x = nullptr;
  sd.ws = ws;
  sd.y = y;
  sd.idx = idx;
  sd.val = val;
  sd.count = count;
  sd.scale = 1.0f;
  sd.ld = 0;
  emu_run_block(kRecThreads, 0, [&] { recover_signal<R>(sd, *sh); });
  const int64_t c = *count;
  if (c < 0 || c > int64_t(pd->K)) {
    std::fprintf(stderr, "EMU: count %lld outside [0, K]\n", (long long)c);
    return 3;
  }
  // the 512-thread shape (twice the LDS) on the same buckets: the same bits
  using Wide = RecoverShared<R, kRecThreadsWide, kLdsBytesWide>;
  auto* shw = static_cast<Wide*>(galloc(sizeof(Wide), "workgroup LDS (512 threads)"));
  auto* idx_w = static_cast<int64_t*>(galloc(sizeof(int64_t) * pd->K, "output frequencies (512 threads)"));
  auto* val_w = static_cast<cplx<R>*>(galloc(sizeof(cplx<R>) * pd->K, "output values (512 threads)"));
  auto* count_w = static_cast<int64_t*>(galloc(sizeof(int64_t), "output count (512 threads)"));
  SignalDesc sdw = sd;
  sdw.idx = idx_w;
  sdw.val = val_w;
  sdw.count = count_w;
  emu_run_block(kRecThreadsWide, 0, [&] { recover_signal<R>(sdw, *shw); });
  if (*count_w != c || std::memcmp(idx_w, idx, sizeof(int64_t) * size_t(c)) != 0 ||
      std::memcmp(static_cast<const void*>(val_w), static_cast<const void*>(val), sizeof(cplx<R>) * size_t(c)) != 0) {
    std::fprintf(stderr, "EMU: the 512-thread shape differs (count %lld against %lld)\n", (long long)*count_w,
                 (long long)c);
    return 4;
  }
  std::fwrite(&c, sizeof c, 1, out);
  for (int64_t k = 0; k < c; ++k) {
    const double re = double(val[k].re), im = double(val[k].im);
    std::fwrite(&idx[k], sizeof(int64_t), 1, out);
    std::fwrite(&re, sizeof re, 1, out);
    std::fwrite(&im, sizeof im, 1, out);
  }
  std::printf("EMU OK count %lld\n", (long long)c);
  return 0;
}

}  // namespace

int main(int argc, char** argv) {
  if (argc != 3) {
    std::fprintf(stderr, "usage: %s input output\n", argv[0]);
    return 2;
  }
  guard_init();
  FILE* f = std::fopen(argv[1], "rb");
  if (!f) return 2;
  int64_t N, K, B, w, ny;
  int32_t loops, l, dtype, location, combine, mode;
  double q, delta;
  uint64_t seed;
  rd(f, &N), rd(f, &K), rd(f, &B), rd(f, &w);
  rd(f, &loops), rd(f, &l);
  rd(f, &q), rd(f, &delta);
  rd(f, &seed);
  rd(f, &dtype), rd(f, &location), rd(f, &combine), rd(f, &mode);
  rd(f, &ny);
  std::vector<double> y(2 * size_t(ny));
  rd(f, y.data(), y.size());
  std::fclose(f);
  guard_mode() = mode;
  sfft_options opt{};
  opt.delta = delta;
  opt.seed = seed;
  opt.dtype = dtype;
  opt.kahan = 0;
  opt.b_min = 16;
  opt.combine = combine;
  opt.eta = 1e-4;
  opt.rho = 0.25;
  opt.flags = 0;
  opt.location = uint32_t(location);
  HostPlan hp;
  std::string err;
  if (build_host_plan(hp, N, K, B, w, loops, l, q, opt, &err) != SFFT_OK) {
    std::fprintf(stderr, "plan: %s\n", err.c_str());
    return 2;
  }
  layout_workspace(hp);
  FILE* out = std::fopen(argv[2], "wb");
  if (!out) return 2;
  const int rc = dtype == SFFT_C128 ? run<double>(hp, y, out) : run<float>(hp, y, out);
  std::fclose(out);
  return rc;
}
