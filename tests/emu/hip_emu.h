// CPU emulation of the subset of HIP device code that the recovery kernel
// body (recover_body.h) uses, for tests that run it on the host.
//
// A workgroup is emulated by one std::thread per work item.  __syncthreads
// is a barrier over the whole group.  Cross-lane (DPP) moves are emulated
// per wavefront of 64 threads: every lane publishes its value, the wave
// meets at a barrier, each lane reads the lane its control selects (with
// the row and bank masks and bound control of the instruction), and the
// wave meets again.  Such a move therefore requires all 64 lanes of the
// wave to execute it, as the kernel's wave-uniform loops do; a lane that
// skipped it would leave the others waiting, and the barrier reports that
// as a fault instead of hanging (see EmuBarrier).
//
// Memory: the host passes plain host pointers; LDS is a host object shared
// by the group's threads.  Atomics are host atomics on the same addresses.
// Transcendentals are the host library's (accuracy differs from the GPU's
// in the last bits, which moves no decision of a well-separated case).
#pragma once

#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <thread>
#include <type_traits>
#include <vector>

#define __device__
#define __host__
#define __global__
#define __forceinline__ inline
#define __noinline__
#define __launch_bounds__(...)
#define __restrict__ __restrict

struct EmuDim3 {
  unsigned x = 0, y = 0, z = 0;
};
inline thread_local EmuDim3 threadIdx, blockIdx;
inline EmuDim3 blockDim, gridDim;

// A reusable barrier over n threads.  A wait that has not been released
// after a generous time (60 s, or EMU_BARRIER_TIMEOUT_S) means that some
// thread of the group never reaches this barrier (a divergent barrier or
// wave move): the emulation reports it and exits with status 87.
class EmuBarrier {
 public:
  explicit EmuBarrier(unsigned n = 0) : n_(n) {}
  void reset(unsigned n) {
    n_ = n;
    count_ = 0;
    gen_ = 0;
  }
  void wait(const char* what) {
    std::unique_lock<std::mutex> lk(m_);
    const uint64_t g = gen_;
    if (++count_ == n_) {
      count_ = 0;
      ++gen_;
      cv_.notify_all();
      return;
    }
    static const long limit = [] {
      const char* e = std::getenv("EMU_BARRIER_TIMEOUT_S");
      return e ? std::atol(e) : 60L;
    }();
    if (!cv_.wait_for(lk, std::chrono::seconds(limit), [&] { return gen_ != g; })) {
      std::fprintf(stderr, "EMU: %s barrier not reached by every thread (%u of %u arrived)\n", what, count_, n_);
      std::fflush(stderr);
      std::_Exit(87);
    }
  }

 private:
  std::mutex m_;
  std::condition_variable cv_;
  unsigned n_ = 0, count_ = 0;
  uint64_t gen_ = 0;
};

struct EmuWave {
  EmuBarrier bar{64};
  uint32_t slot[64];
};

struct EmuBlock {
  explicit EmuBlock(unsigned n) : block(n), waves((n + 63) / 64) {}
  EmuBarrier block;
  std::vector<EmuWave> waves;
};
inline thread_local EmuBlock* emu_block = nullptr;

inline void __syncthreads() { emu_block->block.wait("workgroup"); }
inline void __threadfence() { std::atomic_thread_fence(std::memory_order_seq_cst); }

// v of the lane that the DPP control selects (quad_perm, row shifts and
// rotations, row mirrors, row broadcasts of lanes 15 and 31); invalid
// source lanes give 0 with bound control, else leave `old`; lanes whose row
// or bank is masked off keep `old`.
inline int emu_update_dpp(int old, int src, int ctrl, int row_mask, int bank_mask, bool bound_ctrl) {
  EmuWave& w = emu_block->waves[threadIdx.x / 64];
  const int lane = int(threadIdx.x & 63);
  w.slot[lane] = uint32_t(src);
  w.bar.wait("wavefront (DPP)");
  int sl = -1;
  const int r = lane & 15;
  if (ctrl >= 0 && ctrl <= 0xFF) {
    sl = (lane & ~3) | ((ctrl >> (2 * (lane & 3))) & 3);
  } else if (ctrl >= 0x101 && ctrl <= 0x10F) {  // row_shl: lane reads lane + n of its row
    const int n = ctrl & 15;
    sl = r + n < 16 ? lane + n : -1;
  } else if (ctrl >= 0x111 && ctrl <= 0x11F) {  // row_shr: lane reads lane - n of its row
    const int n = ctrl & 15;
    sl = r >= n ? lane - n : -1;
  } else if (ctrl >= 0x121 && ctrl <= 0x12F) {  // row_ror: rotate right within the row
    const int n = ctrl & 15;
    sl = (lane & ~15) | ((r - n) & 15);
  } else if (ctrl == 0x140) {  // row_mirror
    sl = (lane & ~15) | (15 - r);
  } else if (ctrl == 0x141) {  // row_half_mirror
    sl = (lane & ~7) | (7 - (lane & 7));
  } else if (ctrl == 0x142) {  // row_bcast:15: lane 15 of the previous row
    const int row = lane >> 4;
    sl = row > 0 ? row * 16 - 1 : -1;
  } else if (ctrl == 0x143) {  // row_bcast:31: lane 31 to rows 2 and 3
    sl = lane >= 32 ? 31 : -1;
  } else {
    std::fprintf(stderr, "EMU: DPP control 0x%x not emulated\n", ctrl);
    std::_Exit(88);
  }
  const bool write = ((row_mask >> (lane >> 4)) & 1) && ((bank_mask >> ((lane >> 2) & 3)) & 1);
  int out = old;
  if (write) out = sl >= 0 ? int(w.slot[sl]) : (bound_ctrl ? 0 : old);
  w.bar.wait("wavefront (DPP)");
  return out;
}
#define __builtin_amdgcn_update_dpp(old, src, ctrl, rm, bm, bc) emu_update_dpp((old), (src), (ctrl), (rm), (bm), (bc))
#define __builtin_amdgcn_wave_barrier() emu_block->waves[threadIdx.x / 64].bar.wait("wavefront")
#define __builtin_amdgcn_fence(...) std::atomic_thread_fence(std::memory_order_seq_cst)
#define __builtin_amdgcn_s_sleep(n) std::this_thread::yield()
// the kernels apply it to wave-uniform values only, where it is the identity
#define __builtin_amdgcn_readfirstlane(v) (v)

template <typename T>
inline T atomicAdd(T* p, T v) {
  return __atomic_fetch_add(p, v, __ATOMIC_SEQ_CST);
}

inline uint32_t __float_as_uint(float v) { return __builtin_bit_cast(uint32_t, v); }
inline float __uint_as_float(uint32_t v) { return __builtin_bit_cast(float, v); }
inline long long __double_as_longlong(double v) { return __builtin_bit_cast(long long, v); }
inline double __longlong_as_double(long long v) { return __builtin_bit_cast(double, v); }

inline void sincospif(float x, float* s, float* c) {
  const long double a = 3.141592653589793238462643383279502884L * (long double)x;
  *s = float(std::sin(a));
  *c = float(std::cos(a));
}
inline void sincospi(double x, double* s, double* c) {
  const long double a = 3.141592653589793238462643383279502884L * (long double)x;
  *s = double(std::sin(a));
  *c = double(std::cos(a));
}
using std::atan2;

using std::fabs;
using std::sqrt;

template <typename A, typename B>
inline std::common_type_t<A, B> min(A a, B b) {
  using C = std::common_type_t<A, B>;
  return C(b) < C(a) ? C(b) : C(a);
}
template <typename A, typename B>
inline std::common_type_t<A, B> max(A a, B b) {
  using C = std::common_type_t<A, B>;
  return C(a) < C(b) ? C(b) : C(a);
}

// Runs body() as one workgroup of n threads (block index bid).
template <typename F>
inline void emu_run_block(unsigned n, unsigned bid, F&& body) {
  EmuBlock blk(n);
  blockDim = EmuDim3{n, 1, 1};
  std::vector<std::thread> th;
  th.reserve(n);
  for (unsigned t = 0; t < n; ++t)
    th.emplace_back([&, t] {
      threadIdx = EmuDim3{t, 0, 0};
      blockIdx = EmuDim3{bid, 0, 0};
      emu_block = &blk;
      body();
    });
  for (auto& x : th) x.join();
}
