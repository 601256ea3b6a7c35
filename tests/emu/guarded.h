// Guarded host allocations for the CPU emulation tests: every buffer sits
// against an inaccessible page, after its end (mode 0) or before its start
// (mode 1), and a fault handler names the buffer an access hit and exits
// with status 86.
#pragma once

#include <signal.h>
#include <sys/mman.h>
#include <unistd.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

namespace emu {

struct Region {
  unsigned char *lo, *hi, *user;
  size_t n;
  const char* name;
};
inline std::vector<Region>& regions() {
  static std::vector<Region> r;
  return r;
}
inline int& guard_mode() {
  static int m = 0;
  return m;
}
inline size_t& page() {
  static size_t p = 4096;
  return p;
}

inline void on_fault(int, siginfo_t* si, void*) {
  unsigned char* a = static_cast<unsigned char*>(si->si_addr);
  char msg[256];
  int len = 0;
  for (const Region& r : regions()) {
    if (a >= r.lo && a < r.hi) {
      const long off = long(a - r.user);
      len = std::snprintf(msg, sizeof msg, "EMU FAULT: access at byte %ld of %s (%zu bytes)\n", off, r.name, r.n);
      break;
    }
  }
  if (len == 0) len = std::snprintf(msg, sizeof msg, "EMU FAULT: access at %p, outside every buffer\n", (void*)a);
  if (write(2, msg, size_t(len)) < 0) {
  }
  _exit(86);
}

inline void guard_init() {
  page() = size_t(sysconf(_SC_PAGESIZE));
  struct sigaction sa {};
  sa.sa_sigaction = on_fault;
  sa.sa_flags = SA_SIGINFO;
  sigaction(SIGSEGV, &sa, nullptr);
  sigaction(SIGBUS, &sa, nullptr);
}

// n bytes (rounded up to 16) against a guard page.  Filled with 0xFF bytes,
// so that a read of memory never written yields NaN or huge integers
// rather than zeros.
inline void* galloc(size_t n, const char* name) {
  const size_t pg = page();
  const size_t nn = ((n ? n : 1) + 15) & ~size_t(15);
  const size_t body = (nn + pg - 1) / pg * pg;
  void* m = mmap(nullptr, body + 2 * pg, PROT_READ | PROT_WRITE, MAP_PRIVATE | MAP_ANONYMOUS, -1, 0);
  if (m == MAP_FAILED) {
    std::perror("mmap");
    std::exit(2);
  }
  unsigned char* base = static_cast<unsigned char*>(m);
  mprotect(base, pg, PROT_NONE);
  mprotect(base + pg + body, pg, PROT_NONE);
  unsigned char* p = guard_mode() == 0 ? base + pg + body - nn : base + pg;
  std::memset(p, 0xFF, nn);
  regions().push_back(Region{base, base + body + 2 * pg, p, n, name});
  return p;
}

}  // namespace emu
