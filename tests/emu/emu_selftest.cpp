// Checks of the CPU emulation itself (tests/test_cpu_emulation.py runs it):
//   fault-after  a write one element past a guarded buffer  -> exit 86
//   fault-before a write one element before a guarded buffer (guard mode 1) -> exit 86
//   diverge      one lane of a wave skips a DPP move         -> exit 87
//   dpp          the kernel's DPP reductions and scan (team_sum for every
//                team size, wave_max, wave_min, wave_incl_scan) over a
//                block, against their definitions computed sequentially -> exit 0
#include <cstdio>
#include <cstring>
#include <string>

#include "guarded.h"
#include "internal.h"
#include "recover_body.h"

using namespace sfft;

static int dpp_check() {
  constexpr unsigned n = 256;
  std::vector<uint32_t> in(n), sums[7], mx(n), mn(n), scan(n);
  for (auto& v : sums) v.resize(n);
  for (unsigned t = 0; t < n; ++t) in[t] = (t * 2654435761u) >> 20;  // arbitrary, below 2^12
  emu_run_block(n, 0, [&] {
    const unsigned t = threadIdx.x;
    for (int k = 0; k <= 6; ++k) sums[k][t] = team_sum(in[t], 1u << k);
    mx[t] = wave_max(in[t]);
    mn[t] = wave_min(in[t]);
    scan[t] = wave_incl_scan(in[t]);
  });
  int bad = 0;
  for (unsigned t = 0; t < n; ++t) {
    for (int k = 0; k <= 6; ++k) {
      const unsigned S = 1u << k, t0 = t & ~(S - 1);
      uint32_t want = 0;
      for (unsigned u = t0; u < t0 + S; ++u) want += in[u];
      // the team's sum is in its last lane (and in every lane for S <= 16)
      if ((t == t0 + S - 1 || S <= 16) && sums[k][t] != want) ++bad;
    }
    const unsigned w0 = t & ~63u;
    uint32_t m1 = 0, m2 = ~0u, s = 0;
    for (unsigned u = w0; u < w0 + 64; ++u) {
      m1 = in[u] > m1 ? in[u] : m1;
      m2 = in[u] < m2 ? in[u] : m2;
    }
    for (unsigned u = w0; u <= t; ++u) s += in[u];
    if ((t & 63) == 63 && (mx[t] != m1 || mn[t] != m2)) ++bad;
    if (scan[t] != s) ++bad;
  }
  std::printf("dpp: %d mismatches\n", bad);
  return bad ? 1 : 0;
}

int main(int argc, char** argv) {
  const std::string what = argc > 1 ? argv[1] : "";
  emu::guard_init();
  if (what == "fault-after" || what == "fault-before") {
    emu::guard_mode() = what == "fault-after" ? 0 : 1;
    float* buf = static_cast<float*>(emu::galloc(100 * sizeof(float), "self-test buffer"));
    emu_run_block(64, 0, [&] {
      const int i = what == "fault-after" ? 99 + int(threadIdx.x == 63) : -int(threadIdx.x == 63);
      buf[i] = 1.0f;
    });
    std::printf("no fault\n");
    return 0;
  }
  if (what == "diverge") {
    emu_run_block(64, 0, [&] {
      if (threadIdx.x != 5) (void)team_sum(1u, 2u);
    });
    std::printf("no divergence reported\n");
    return 0;
  }
  if (what == "dpp") return dpp_check();
  std::fprintf(stderr, "usage: %s fault-after|fault-before|diverge|dpp\n", argv[0]);
  return 2;
}
