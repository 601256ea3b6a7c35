// Host-side checks of the C ABI, built with AddressSanitizer and
// UndefinedBehaviorSanitizer on the host code (tests/test_failure_paths.py
// builds and runs it; no GPU is touched).  It drives the calls that need no
// device: host-only plans over a spread of shapes and plan options, plan and
// iteration introspection into buffers sized from the reported facts,
// parameter validation, and the SFFT_FAIL_ALLOC allocation-failure sweep of
// sfft_plan, including the device allocation of a full plan, which fails by
// injection before any HIP call.  The sanitizers report any out-of-bounds
// access, use after free, undefined behaviour or leak; the exit status is
// the number of failed expectations.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "sfft.h"

static int g_failures = 0;

#define EXPECT(cond)                                                         \
  do {                                                                       \
    if (!(cond)) {                                                           \
      std::fprintf(stderr, "%s:%d: expectation failed: %s (%s)\n", __FILE__, \
                   __LINE__, #cond, sfft_last_error());                      \
      ++g_failures;                                                          \
    }                                                                        \
  } while (0)

struct Shape {
  int64_t N, K, B, w;
  int32_t loops, l;
  double q, delta;
  int32_t dtype, location, combine;
};

static void introspect(sfft_plan_t p, int32_t loops) {
  sfft_plan_info info;
  EXPECT(sfft_get_plan_info(p, &info) == SFFT_OK);
  EXPECT(info.loops == loops && info.samples > 0 && info.yhat_elems > 0);
  for (int32_t m = 0; m < loops; ++m) {
    sfft_iter_info it;
    EXPECT(sfft_get_iter_info(p, m, &it) == SFFT_OK);
    std::vector<double> win(size_t(it.h + 1)), ghat(size_t(it.L / 2 + it.e + 1));
    EXPECT(sfft_plan_dump_tables(p, m, win.data(), ghat.data()) == SFFT_OK);
    EXPECT(win[0] == double(it.L));
  }
  sfft_iter_info it;
  EXPECT(sfft_get_iter_info(p, loops, &it) == SFFT_ERR_PARAM);
  EXPECT(sfft_get_iter_info(p, -1, &it) == SFFT_ERR_PARAM);
  EXPECT(sfft_plan_dump_tables(p, loops, nullptr, nullptr) == SFFT_ERR_PARAM);
}

static sfft_status make(const Shape& s, uint32_t flags, sfft_plan_t* out) {
  sfft_options o;
  sfft_default_options(&o);
  o.delta = s.delta;
  o.seed = 12345;
  o.dtype = s.dtype;
  o.location = uint32_t(s.location);
  o.combine = s.combine;
  o.flags = flags;
  return sfft_plan(out, s.N, s.K, s.B, s.w, s.loops, s.l, s.q, &o);
}

int main() {
  const Shape shapes[] = {
      {1 << 14, 50, 512, 7169, 8, 16, 1.0, 1e-8, SFFT_C128, SFFT_LOCATE_MULTISCALE, SFFT_COMBINE_SUM},
      {1 << 14, 50, 512, 7169, 8, 4, 0.25, 1e-8, SFFT_C64, SFFT_LOCATE_MULTISCALE, SFFT_COMBINE_SUM},
      {1 << 16, 200, 2048, 32769, 7, 16, 1.0, 1e-6, SFFT_C64, SFFT_LOCATE_MULTISCALE, SFFT_COMBINE_VOTE},
      {1 << 16, 300, 2048, 32769, 10, 16, 1.0, 1e-6, SFFT_F16X2_SCALED, SFFT_LOCATE_DIRECT, SFFT_COMBINE_SUM},
      {64, 1, 16, 33, 3, 16, 1.0, 1e-6, SFFT_C64, SFFT_LOCATE_MULTISCALE, SFFT_COMBINE_SUM},
      {1 << 20, 1000, 8192, 163841, 12, 2, 0.5, 1e-6, SFFT_C64, SFFT_LOCATE_MULTISCALE, SFFT_COMBINE_SUM},
  };
  unsetenv("SFFT_FAIL_ALLOC");
  for (const Shape& s : shapes) {
    sfft_plan_t p = nullptr;
    EXPECT(make(s, SFFT_PLAN_HOST_ONLY, &p) == SFFT_OK);
    if (p) {
      introspect(p, s.loops);
      // a host-only plan cannot execute: a state error, reported synchronously
      EXPECT(sfft_execute(p, nullptr, 1.0f, nullptr, nullptr, nullptr, nullptr) == SFFT_ERR_STATE);
      EXPECT(sfft_destroy(p) == SFFT_OK);
    }
  }

  // parameter validation: every rejected call leaves *out NULL
  const Shape bad[] = {
      {1000, 10, 64, 641, 4, 16, 1.0, 1e-6, SFFT_C64, 0, 0},          // N not a power of two
      {1 << 12, 10, 48, 641, 4, 16, 1.0, 1e-6, SFFT_C64, 0, 0},       // B not a power of two
      {1 << 12, 100, 64, 641, 4, 16, 1.0, 1e-6, SFFT_C64, 0, 0},      // K > B
      {1 << 12, 10, 64, 32, 4, 16, 1.0, 1e-6, SFFT_C64, 0, 0},        // w < B
      {1 << 12, 10, 64, 641, 0, 16, 1.0, 1e-6, SFFT_C64, 0, 0},       // loops < 1
      {1 << 12, 10, 64, 641, 4, 2, 4.0, 1e-6, SFFT_C64, 0, 0},        // l <= q + 1
      {1 << 12, 10, 64, 641, 4, 16, 0.3, 1e-6, SFFT_C64, 0, 0},       // q not dyadic
      {1 << 12, 10, 64, 641, 4, 16, 1.0, 0.5, SFFT_C64, 0, 0},        // delta out of range
      {1 << 12, 10, 64, 641, 4, 16, 1.0, 1e-6, 7, 0, 0},              // unknown dtype
      {1 << 12, 10, 64, 641, 4, 16, 1.0, 1e-6, SFFT_C64, 5, 0},       // unknown location
      {1 << 12, 10, 64, 641, 4, 16, 1.0, 1e-6, SFFT_C64, 0, 9},       // unknown combine
  };
  for (const Shape& s : bad) {
    sfft_plan_t p = reinterpret_cast<sfft_plan_t>(&g_failures);
    EXPECT(make(s, SFFT_PLAN_HOST_ONLY, &p) == SFFT_ERR_PARAM);
    EXPECT(p == nullptr);
  }
  EXPECT(sfft_plan(nullptr, 1 << 12, 10, 64, 641, 4, 16, 1.0, nullptr) == SFFT_ERR_PARAM);

  // allocation failures: the plan object (1), then each iteration's host
  // tables (2 .. loops + 1), then the device memory of a full plan
  // (loops + 2); every failing call returns SFFT_ERR_ALLOC with *out NULL
  // and keeps nothing (LeakSanitizer checks at exit)
  for (const Shape& s : shapes) {
    char buf[16];
    for (int n = 1; n <= s.loops + 1; ++n) {
      std::snprintf(buf, sizeof buf, "%d", n);
      setenv("SFFT_FAIL_ALLOC", buf, 1);
      sfft_plan_t p = nullptr;
      EXPECT(make(s, SFFT_PLAN_HOST_ONLY, &p) == SFFT_ERR_ALLOC);
      EXPECT(p == nullptr);
    }
    std::snprintf(buf, sizeof buf, "%d", s.loops + 2);
    setenv("SFFT_FAIL_ALLOC", buf, 1);
    sfft_plan_t p = nullptr;
    EXPECT(make(s, SFFT_PLAN_HOST_ONLY, &p) == SFFT_OK);  // a host-only plan has no device allocation
    if (p) EXPECT(sfft_destroy(p) == SFFT_OK);
    p = nullptr;
    EXPECT(make(s, 0, &p) == SFFT_ERR_ALLOC);            // the device allocation, injected
    EXPECT(p == nullptr);
    EXPECT(std::strstr(sfft_last_error(), "hipMalloc(plan)") != nullptr);
  }
  unsetenv("SFFT_FAIL_ALLOC");
  EXPECT(std::strcmp(sfft_status_string(SFFT_ERR_ALLOC), "allocation failed") == 0);
  EXPECT(sfft_destroy(nullptr) == SFFT_OK);
  EXPECT(sfft_batch_destroy(nullptr) == SFFT_OK);
  std::printf("abi_host_check: %d failed expectations\n", g_failures);
  return g_failures;
}
