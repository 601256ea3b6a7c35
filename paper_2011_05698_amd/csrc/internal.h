// Internal layout shared by the host plan code and the gfx950 kernels.
#pragma once

#include <cstddef>
#include <cstdint>
#include <memory>
#include <string>
#include <vector>

#include "sfft.h"

namespace sfft {

constexpr int kMaxRounds = 48;      // R + 1 <= kMaxRounds (reference round + location steps)
constexpr int kMaxLoops = 64;
constexpr int kMaxBucketsF32 = 16384;  // the bucket DFT holds B values in LDS: 128 KiB
constexpr int kMaxBucketsF64 = 8192;   // 128 KiB of complex128

// One iteration of the method, as the kernels read it (plain data, device copy).
struct IterDesc {
  uint32_t B, logB, L, logL;
  uint32_t w, h, e, D;            // D = L/2 + e: reach of a coefficient from a bucket centre
  uint32_t R;                     // location steps; the iteration has R + 1 rounds
  uint32_t reach;                 // floor(2D / L): bucket distance of two views of one position
  uint32_t sigma, sigma_inv;      // odd scaling and its inverse mod N
  uint32_t tau0, pad0;
  uint32_t T[kMaxRounds];         // round offsets: T_0 = tau0, T_j = tau0 + tau_j mod N
  uint32_t tau[kMaxRounds];       // location multipliers (index 0 unused)
  uint32_t len[kMaxRounds];       // location region lengths (index 0 unused)
  uint64_t win_off;               // element offset of G_0..G_h in the window table
  uint64_t ghat_off;              // element offset of Ghat_0..Ghat_D in the spectrum table
  uint64_t tw_off;                // complex-element offset of B/2 twiddles exp(-2 pi i k / B)
  uint64_t y_off;                 // complex-element offset of the (R+1) x B bucket block
  double log_B;                   // ln(B)
};

// A plan as the kernels read it.
struct PlanDesc {
  uint32_t N, logN, K, M;
  uint32_t l, logl;               // multiscale parameter (power of two)
  int32_t qn;                     // extension q = qn / 2^logqd
  uint32_t logqd;
  uint32_t dtype, kahan;
  uint32_t rec_cap;               // capacity of the recovered-coefficient store
  uint32_t Bmax;                  // largest B_m
  uint32_t sort_cap;              // power of two >= max(rec_cap, Bmax)
  uint32_t fp64_phase;            // take location phases in FP64 (N >= 2^24)
  uint32_t Rmax;                  // largest R_m
  uint32_t max_slots;             // largest reach_m + 1
  uint32_t location;              // sfft_location of every iteration
  uint32_t combine;               // sfft_combine
  uint64_t y_total;               // complex elements of bucket values per signal
  uint64_t ws_bytes;              // workspace bytes per signal
  // byte offsets inside one signal's workspace
  uint64_t off_y, off_recf, off_recv;
  uint64_t off_work, work_bytes;  // the recovery's arrays that do not fit in LDS
  uint64_t off_nvote, off_votes;  // vote: loops that located each store entry, and their estimates
  double eta, rho;
  const IterDesc* iters;          // device array of M descriptors
  const void* window;             // float or double table
  const void* ghat;               // float or double table
  const void* twiddle;            // float2 or double2 table
};

// One signal of a batch (device copy).
struct SignalDesc {
  const PlanDesc* plan;
  const void* x;
  void* ws;
  void* y;                         // bucket values (R+1) x B per iteration; normally ws + off_y
  int64_t* idx;
  void* val;
  int64_t* count;
  float scale;
  uint32_t ld;                     // position-major batches: elements between samples c and c+1 (0: contiguous)
};

// How the stage kernels receive signal descriptors: a batch table in device
// memory (uploaded by the host), or one descriptor by value in the kernel
// arguments for single-signal calls.
struct SigArg {
  const SignalDesc* table;  // batch descriptor table, or nullptr
  SignalDesc one;           // the signal of a single-signal call
};

// Work items of the stage kernels.
struct FoldTile {                  // fold items [i0, i0 + kFoldTile) of iteration m; item = j * B_m + b
  uint32_t sig;
  uint32_t m;                      // iteration in the low 16 bits; a union tile's round count above
  uint32_t i0;
};
// A union tile gathers rounds 0..nu-1 of an iteration together (nu >= 2):
// its items are the round-0 buckets [i0, i0 + kFoldTile), and each thread
// writes its bucket's value in every one of those rounds (fold_body.h).
constexpr uint32_t kMaxUnionRounds = 4;
constexpr uint32_t fold_tile_iter(uint32_t m) { return m & 0xFFFFu; }
constexpr uint32_t fold_tile_rounds(uint32_t m) { return m >> 16; }
constexpr uint32_t fold_tile_code(uint32_t m, uint32_t nu) { return m | (nu << 16); }
struct RoundItem {                 // one (signal, iteration, round)
  uint32_t sig;
  uint16_t m, j;
};
struct FftGroup {                  // round items [first, first + count), all with the same B
  uint32_t first, count;
};
constexpr uint32_t kFftGroupPoints = 2048;     // points one bucket-DFT workgroup takes when B is small (default)
constexpr uint32_t kMaxFftGroupPoints = 4096;  // ... at most (the autotuner's choices)
// Largest log2 B of the bucket DFT's in-register wave path (fft_wave.h), by
// real type; rounds above it take the LDS pass (fft_body.h).
constexpr uint32_t kWaveFftMaxLogB32 = 11, kWaveFftMaxLogB64 = 9;
constexpr uint32_t kFftWaves = 4;             // waves of a bucket-DFT workgroup
// The bucket-DFT groups of a plan or batch, largest B first: [0, nlds)
// take the LDS pass, [nlds, ngroups) the wave path (rounds of at most
// 2^wave_logB points).  Of the LDS groups, [0, n16) hold at least
// kFft16Points points (at most max_points) and take four radix-2 stages per
// pass; [n16, nlds) hold fewer (at most max_points_rest).
constexpr uint32_t kFft16Points = 16384;  // a sixteen-point group per thread of 1024
struct FftGroups {
  uint32_t ngroups = 0, nlds = 0, n16 = 0, max_points = 0, max_points_rest = 0, wave_logB = 0;
};

// ------------------------------------------------------------------ host --
struct IterHost {
  IterDesc d;
  double s_t, s_f, d_delta;
  // G_0..G_h and Ghat_0..Ghat_D: they depend on N, L, h and delta only, so
  // plans (and iterations) with the same values share one copy
  std::shared_ptr<const std::vector<double>> G, Ghat;
  std::vector<uint8_t> kinds;     // 0 block step, 1 enumeration (index 0 unused)
};

struct HostPlan {
  int64_t N, K, B, w;
  int loops, l;
  int64_t qn, qd;                 // q = qn / qd, qd a power of two
  double q, delta, eta, rho;
  uint64_t seed;
  int dtype, kahan, b_min;
  uint32_t flags;
  std::vector<IterHost> iters;
  PlanDesc desc;                  // filled with host-side sizes; device pointers set on upload
  int64_t samples;
};

// Builds the host part of a plan.  Returns SFFT_OK or an error with *err set.
sfft_status build_host_plan(HostPlan& hp, int64_t N, int64_t K, int64_t B, int64_t w, int32_t loops,
                            int32_t l, double q, const sfft_options& opt, std::string* err);

// Workspace layout of one signal (fills the off_* fields of desc).
void layout_workspace(HostPlan& hp);

// Rounds 0..nu-1 of iteration d that a per-signal fold gathers in one union
// tile: the leading rounds whose offsets d_j = T_j - T_0 mod N ascend in
// steps shorter than w (so their windows cover one interval of round-0 taps
// without a gap), at most kMaxUnionRounds, with d_{nu-1} + w <= N; 1 when
// B is below a fold tile or no round overlaps round 0.
uint32_t union_rounds(const IterDesc& d, uint32_t N);

struct FoldSplit;
// Appends the work lists of signal `sig` of a per-signal launch: its fold
// tiles (union tiles included) and its (iteration, round) bucket-DFT items.
void build_work_lists(const HostPlan& hp, uint32_t sig, std::vector<FoldTile>& tiles, std::vector<RoundItem>& items);
// Orders per-signal fold tiles for the stage launches (FoldSplit) and counts
// the union tiles of each round count.
FoldSplit order_for_stages(std::vector<FoldTile>& tiles);
// The fold tiles of a position-major batch of ngroups signal groups.
void interleaved_tiles(const HostPlan& hp, uint32_t ngroups, std::vector<FoldTile>& tiles);

// Bytes of the recovery's work area (arrays of one iteration that do not fit
// in LDS, or the final top-K keys), for any iteration of the plan: every
// array at its largest size, each rounded up to 16 bytes.  cb and rb are the
// sizes of one complex and one real value.
inline uint64_t recover_work_bytes(const PlanDesc& pd, uint64_t cb, uint64_t rb) {
  const uint64_t a = 16 * 24;
  const uint64_t rc = pd.rec_cap, bm = pd.Bmax, sc = pd.sort_cap;
  const uint64_t store = sc * 4 + rc * (8 + cb) + rc * (4 + cb + 8);  // cells, keys, values; sort temporaries
  const uint64_t bucket = bm * (cb + 4) + bm * 8 + bm * 8;           // round 0, located u; runs; power keys
  const uint64_t cand = bm * (4 + 4) + uint64_t(pd.Rmax) * bm * (cb + 8) + bm * cb;  // lists, rows, angles, values
  const uint64_t iter = a + store + rc * pd.max_slots * rb + bucket + cand;
  const uint64_t topk = a + sc * (16 + 4);
  return iter > topk ? iter : topk;
}

void set_last_error(const std::string& s);

// Allocation-failure injection, for tests of the error paths.  Every host or
// device allocation the library makes while building a plan or a batch first
// asks alloc_should_fail(); when the environment variable SFFT_FAIL_ALLOC
// holds a positive integer n, the n-th such allocation of a public call
// (counted from the call's start, on the calling thread) fails as if memory
// were exhausted, and the call returns SFFT_ERR_ALLOC after releasing
// everything it had taken.  Unset or 0: never.
void alloc_trial_begin();
bool alloc_should_fail();

// Stage launchers (kernels.hip).  Each returns hipSuccess or the launch error.
// All signals of one launch share dtype and the Kahan setting.
constexpr int kFoldTile = 256;      // (round, bucket) items per fold work item (one thread each)

// Launch shape of the fold: taps in flight per thread, and a cap on resident
// workgroups per CU (enforced through an LDS reservation) that bounds how many
// signals are gathered at once, so a signal's lines stay in the last-level
// cache between the rounds and iterations that touch them again.
struct FoldConfig {
  int unroll;        // 8, 16 or 24
  int wg_per_cu;     // 0: no cap; else 2..8
  int lanes = 0;     // position-major: signals per lane (1, 2 or 4); 0: as many as the bound input allows
};
int fold_lds_bytes(int wg_per_cu);
constexpr int kIlvItems = 16;      // (round, bucket) items per position-major fold workgroup
constexpr int kIlvSigs = 64;       // signals per position-major fold workgroup, one per lane
// The per-signal stage launches take the union tiles first, by round count
// (nunion[k] tiles uniting k + 2 rounds, each count in its own launch), then
// the one-round tiles: each kernel keeps the registers of its own loop.
struct FoldSplit {
  uint32_t nunion[kMaxUnionRounds - 1] = {};
};
int launch_fold(int dtype, int kahan, const FoldConfig& cfg, const SigArg& sig, const FoldTile* d_tiles,
                uint32_t ntiles, const FoldSplit& split, void* stream);
// Position-major batch (one plan; sample c of signal s at table[s].x + c * ld,
// with table[s].x = table[0].x + s): tiles of kIlvItems items x kIlvSigs
// signals, FoldTile.sig = index of the signal group, a block's groups
// innermost.  lanes: adjacent signals per lane (1; 2 for complex64 and FP16
// pairs; 4 for FP16 pairs), one workgroup per `lanes` tiles; the caller
// checks that x_0 is aligned to `lanes` elements and that ld is a multiple
// of it (nsig and the group count are checked here).
int launch_fold_interleaved(int dtype, int kahan, int unroll, int lanes, const SignalDesc* table, uint32_t nsig,
                            const FoldTile* d_tiles, uint32_t ntiles, void* stream);
int launch_bucket_fft(int dtype, const SigArg& sig, const RoundItem* d_items, const FftGroup* d_groups,
                      const FftGroups& fg, void* stream);
int launch_recover(int dtype, const SigArg& sig, uint32_t nsig, void* stream);

// LDS the recovery of one signal works in (with its few static arrays, two
// workgroups fit a compute unit's 160 KiB).  The fused batch kernel uses the
// same buffer for its fold tiles and bucket DFTs, so it takes plans whose
// largest round (B_m complex values) fits in it.
constexpr uint32_t kRecoverLdsBytes = 78848;

// The batch as one persistent launch (fused.hip): work items in dependency
// order.  kind kFusedFold: fold tile {grp, m, i0} (grp = signal, or signal
// group of kIlvSigs in a position-major batch); kind kFusedFinish: bucket
// DFTs and recovery of signal grp, after need[group] fold tiles of its group
// are done.
constexpr uint32_t kFusedFold = 0, kFusedFinish = 1;
struct FusedItem {
  uint32_t kind, grp, m, i0;
};
struct FusedArgs {
  const SignalDesc* table;  // the batch's descriptor table
  uint32_t nsig;
  uint32_t nitems;
  const FusedItem* items;
  uint32_t* ctl;            // [0] queue head, [1] waits that gave up, [2 + g] fold tiles of group g done
  const uint32_t* need;     // fold tiles of each group
};
// Zeroes ctl[0 .. nctl) with a small kernel, then launches the persistent
// kernel with `grid` workgroups on `stream`.
int launch_fused(int dtype, int kahan, bool position_major, uint32_t grid, uint32_t nctl, const FusedArgs& a,
                 void* stream);

}  // namespace sfft
