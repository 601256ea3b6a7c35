// C ABI of the library: plan objects, batches, stage sequencing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "internal.h"

using namespace sfft;

namespace sfft {

static thread_local std::string g_last_error;
void set_last_error(const std::string& s) { g_last_error = s; }

static thread_local long t_alloc_count = 0;
void alloc_trial_begin() { t_alloc_count = 0; }
bool alloc_should_fail() {
  const long k = ++t_alloc_count;
  const char* s = std::getenv("SFFT_FAIL_ALLOC");
  if (!s || !*s) return false;
  char* end = nullptr;
  const long n = std::strtol(s, &end, 10);
  return end != s && n > 0 && n == k;
}

// Device allocation through the failure-injection point.
static hipError_t dev_malloc(void** p, size_t bytes) {
  if (alloc_should_fail()) {
    *p = nullptr;
    return hipErrorOutOfMemory;
  }
  return hipMalloc(p, bytes);
}

// Device copies of a plan's tables (window, window spectrum, twiddles), in
// one allocation shared by the plans on the same device and in the same
// precision whose iterations hold the same host tables (the host plan code
// gives plans with equal N, L, h and delta one copy of those) and the same
// B: a batch of plans that differ only in their seeds reads one set of
// tables.  Freed with the last plan that holds it.  A live entry's host
// tables are held by the plans that hold the entry, so their addresses
// cannot be reused while the entry lives.
struct DevTables {
  unsigned char* mem = nullptr;
  ~DevTables() {
    if (mem) (void)hipFree(mem);
  }
};
struct DevTablesKey {
  int dev, dtype;
  std::vector<const void*> tables;  // G and Ghat of each iteration
  std::vector<uint32_t> B;
  bool operator<(const DevTablesKey& o) const {
    return std::tie(dev, dtype, tables, B) < std::tie(o.dev, o.dtype, o.tables, o.B);
  }
};
static std::mutex g_dev_tables_mu;
static std::map<DevTablesKey, std::weak_ptr<DevTables>> g_dev_tables;

}  // namespace sfft

// Workspace of sfft_execute_noalloc: one static array per device, held until
// the process ends.  Host code never passes the array's name to a kernel (on
// the host it is only a stand-in for the symbol); it takes the device address
// from hipGetSymbolAddress once per device and uses that address.
namespace sfft {
constexpr size_t kScratchBytes = size_t(16) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
constexpr int kMaxDevices = 64;
static std::once_flag g_scratch_once[kMaxDevices];
static void* g_scratch_ptr[kMaxDevices];
static hipError_t g_scratch_err[kMaxDevices];

// Device address of the current device's scratch array (nullptr and *err on failure).
static void* scratch_address(hipError_t* err) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    *err = e != hipSuccess ? e : hipErrorInvalidDevice;
    return nullptr;
  }
  std::call_once(g_scratch_once[dev], [dev] {
    void* ptr = nullptr;
    g_scratch_err[dev] = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    g_scratch_ptr[dev] = g_scratch_err[dev] == hipSuccess ? ptr : nullptr;
  });
  *err = g_scratch_err[dev];
  return g_scratch_ptr[dev];
}
}  // namespace sfft

struct sfft_plan_s {
  HostPlan hp;
  bool on_device = false;
  unsigned char* d_mem = nullptr;   // descriptors, work lists, one-signal workspace
  std::shared_ptr<sfft::DevTables> tables;  // window, window spectrum and twiddles (shared)
  PlanDesc* d_plan = nullptr;
  FoldTile* d_tiles = nullptr;
  RoundItem* d_items = nullptr;
  FftGroup* d_groups = nullptr;
  unsigned char* d_ws = nullptr;
  uint32_t ntiles = 0, nitems = 0;
  FftGroups fft;
  FoldSplit split;
  FoldConfig fold{8, 0};
};

struct sfft_batch_s {
  std::vector<sfft_plan_t> plans;
  int dtype = 0, kahan = 0;
  unsigned char* d_mem = nullptr;
  SignalDesc* d_sigs = nullptr;
  FoldTile* d_tiles = nullptr;
  RoundItem* d_items = nullptr;
  FftGroup* d_groups = nullptr;
  unsigned char* d_ws = nullptr;
  std::vector<uint64_t> ws_off;
  uint32_t ntiles = 0, nitems = 0, max_B = 0;
  FftGroups fft;
  FoldSplit split;                  // per-signal tiles: union tiles first (order_for_stages)
  std::vector<SignalDesc> bound;    // host copy of the uploaded descriptor table
  bool has_binding = false;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipStream_t capture_stream = nullptr;
  hipEvent_t replayed = nullptr;    // recorded on the caller's stream after each graph replay
  bool replay_recorded = false;
  FoldConfig fold{8, 0};
  bool interleaved = false;         // one plan, position-major signals (sfft_batch_create_interleaved)
  uint32_t ngroups = 0;             // interleaved: signal groups of kIlvSigs
  int lanes_max = 1;                // interleaved: most signals per fold lane the bound input allows
  // bucket-DFT grouping: round items (host copy) cut into groups of at most fft_group_points points
  std::vector<RoundItem> h_items;
  uint32_t fft_group_points = kFftGroupPoints;
  // the fused persistent launch (fused.hip)
  int mode = SFFT_BATCH_STAGES;
  bool fused_ok = false;            // every plan's largest round fits the fused kernel's LDS
  uint32_t fused_chunk = 1;         // counter groups per chunk of the item order
  std::vector<std::vector<FoldTile>> group_tiles;  // fold tiles of each counter group, in launch order
  FusedItem* d_fitems = nullptr;
  uint32_t nfitems = 0;
  uint32_t* d_ctl = nullptr;        // queue head, waits that gave up, per-group counters
  uint32_t* d_need = nullptr;
  uint32_t nfgroups = 0;            // counter groups: signals, or signal groups (position-major)
  uint32_t fused_grid = 0;
  float step_ms = 0.f;              // the autotuner's time of the chosen configuration
};

namespace {

sfft_status fail(sfft_status s, const std::string& msg) {
  set_last_error(msg);
  return s;
}

sfft_status hip_fail(hipError_t e, const char* what) {
  return fail(e == hipErrorOutOfMemory ? SFFT_ERR_ALLOC : SFFT_ERR_LAUNCH,
              std::string(what) + ": " + hipGetErrorString(e));
}

uint64_t align256(uint64_t v) { return (v + 255) & ~uint64_t(255); }

// Orders round items by B (largest first, stable) and cuts them into
// bucket-DFT workgroups of equal B: rounds above the wave path's size take
// groups of at most `points` points (one round at least); wave-path rounds
// take groups of `points` points, but at least one chunk per wave of the
// workgroup (64 / L1 rounds each, L1 = 2^ceil(log2 B / 2)), so that no wave
// of it idles.
template <class BOf>
void group_rounds(std::vector<RoundItem>& items, BOf b_of, int dtype, std::vector<FftGroup>& groups,
                  FftGroups& fg, uint32_t points = kFftGroupPoints) {
  std::stable_sort(items.begin(), items.end(),
                   [&](const RoundItem& x, const RoundItem& y) { return b_of(x) > b_of(y); });
  const uint32_t wmax = dtype == SFFT_C128 ? kWaveFftMaxLogB64 : kWaveFftMaxLogB32;
  groups.clear();
  fg = FftGroups{};
  for (uint32_t a = 0; a < uint32_t(items.size());) {
    const uint32_t B = b_of(items[a]);
    uint32_t logB = 0;
    while ((1u << logB) < B) ++logB;
    uint32_t cap = std::max<uint32_t>(1u, points / B);
    if (logB <= wmax) {
      cap = std::max(cap, kFftWaves * (64u >> (logB - logB / 2)));
      fg.wave_logB = std::max(fg.wave_logB, logB);
    } else {
      fg.nlds = uint32_t(groups.size()) + 1;
    }
    uint32_t c = 1;
    while (a + c < uint32_t(items.size()) && c < cap && b_of(items[a + c]) == B) ++c;
    groups.push_back(FftGroup{a, c});
    if (logB > wmax) {
      // groups come largest B first, so the ones of kFft16Points or more lead
      if (c * B >= kFft16Points && fg.n16 == uint32_t(groups.size()) - 1) {
        fg.n16 = uint32_t(groups.size());
        fg.max_points = std::max(fg.max_points, c * B);
      } else {
        fg.max_points_rest = std::max(fg.max_points_rest, c * B);
      }
    }
    a += c;
  }
  fg.ngroups = uint32_t(groups.size());
}

bool valid_fold(const sfft_fold_config* c) {
  return c && (c->unroll == 8 || c->unroll == 16 || c->unroll == 24) && c->wg_per_cu >= 0 && c->wg_per_cu <= 8 &&
         c->wg_per_cu != 1;
}

// Uploads tables and descriptors of a plan and allocates its one-signal workspace.
sfft_status upload_plan(sfft_plan_t p) {
  HostPlan& hp = p->hp;
  const bool f64 = hp.dtype == SFFT_C128;
  const uint64_t rs = f64 ? 8 : 4;
  uint64_t nwin = 0, nghat = 0, ntw = 0;
  for (auto& it : hp.iters) {
    nwin += it.G->size();
    nghat += it.Ghat->size();
    ntw += it.d.B / 2;
  }
  std::vector<FoldTile> tiles;
  std::vector<RoundItem> items;
  build_work_lists(hp, 0, tiles, items);
  p->split = order_for_stages(tiles);
  std::vector<FftGroup> groups;
  group_rounds(items, [&](const RoundItem& r) { return hp.iters[r.m].d.B; }, hp.dtype, groups, p->fft);
  p->ntiles = uint32_t(tiles.size());
  p->nitems = uint32_t(items.size());

  uint64_t off = 0;
  auto take = [&](uint64_t bytes) {
    uint64_t o = off;
    off += align256(bytes);
    return o;
  };
  const uint64_t o_plan = take(sizeof(PlanDesc));
  const uint64_t o_iters = take(sizeof(IterDesc) * hp.iters.size());
  const uint64_t o_tiles = take(sizeof(FoldTile) * tiles.size());
  const uint64_t o_items = take(sizeof(RoundItem) * items.size());
  const uint64_t o_groups = take(sizeof(FftGroup) * groups.size());
  const uint64_t o_ws = take(hp.desc.ws_bytes);

  hipError_t e = dev_malloc(reinterpret_cast<void**>(&p->d_mem), off);
  if (e != hipSuccess) {
    p->d_mem = nullptr;
    return hip_fail(e, "hipMalloc(plan)");
  }
  // the tables: a live copy of the same ones on this device, or a new one
  uint64_t toff = 0;
  auto ttake = [&](uint64_t bytes) {
    uint64_t o = toff;
    toff += align256(bytes);
    return o;
  };
  const uint64_t o_win = ttake(nwin * rs);
  const uint64_t o_ghat = ttake(nghat * rs);
  const uint64_t o_tw = ttake(ntw * 2 * rs);
  DevTablesKey key{0, hp.dtype, {}, {}};
  e = hipGetDevice(&key.dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  for (auto& it : hp.iters) {
    key.tables.push_back(it.G.get());
    key.tables.push_back(it.Ghat.get());
    key.B.push_back(it.d.B);
  }
  {
    std::lock_guard<std::mutex> lk(g_dev_tables_mu);
    auto hit = g_dev_tables.find(key);
    if (hit != g_dev_tables.end()) p->tables = hit->second.lock();
  }
  if (!p->tables) {
    auto t = std::make_shared<DevTables>();
    e = dev_malloc(reinterpret_cast<void**>(&t->mem), toff);
    if (e != hipSuccess) {
      t->mem = nullptr;
      return hip_fail(e, "hipMalloc(plan tables)");
    }
    std::vector<unsigned char> th(toff, 0);
    uint64_t wi = 0, gi = 0, ti = 0;
    for (auto& it : hp.iters) {
      for (double g : *it.G) {
        if (f64) reinterpret_cast<double*>(th.data() + o_win)[wi++] = g;
        else reinterpret_cast<float*>(th.data() + o_win)[wi++] = float(g);
      }
      for (double g : *it.Ghat) {
        if (f64) reinterpret_cast<double*>(th.data() + o_ghat)[gi++] = g;
        else reinterpret_cast<float*>(th.data() + o_ghat)[gi++] = float(g);
      }
      const uint32_t B = it.d.B;
      for (uint32_t k = 0; k < B / 2; ++k) {
        // exp(-2 pi i k / B)
        const double a = -2.0 * 3.14159265358979323846 * double(k) / double(B);
        if (f64) {
          reinterpret_cast<double*>(th.data() + o_tw)[2 * ti] = std::cos(a);
          reinterpret_cast<double*>(th.data() + o_tw)[2 * ti + 1] = std::sin(a);
        } else {
          reinterpret_cast<float*>(th.data() + o_tw)[2 * ti] = float(std::cos(a));
          reinterpret_cast<float*>(th.data() + o_tw)[2 * ti + 1] = float(std::sin(a));
        }
        ++ti;
      }
    }
    e = hipMemcpy(t->mem, th.data(), toff, hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy(plan tables)");
    std::lock_guard<std::mutex> lk(g_dev_tables_mu);
    for (auto i = g_dev_tables.begin(); i != g_dev_tables.end();)  // entries of tables no plan holds
      i = i->second.expired() ? g_dev_tables.erase(i) : std::next(i);
    auto& slot = g_dev_tables[key];
    if (auto live = slot.lock()) {
      p->tables = std::move(live);  // another thread uploaded the same tables first
    } else {
      slot = t;
      p->tables = std::move(t);
    }
  }
  std::vector<unsigned char> host(o_ws, 0);  // everything before the workspace
  for (size_t m = 0; m < hp.iters.size(); ++m)
    std::memcpy(host.data() + o_iters + m * sizeof(IterDesc), &hp.iters[m].d, sizeof(IterDesc));
  PlanDesc pd = hp.desc;
  pd.iters = reinterpret_cast<const IterDesc*>(p->d_mem + o_iters);
  pd.window = p->tables->mem + o_win;
  pd.ghat = p->tables->mem + o_ghat;
  pd.twiddle = p->tables->mem + o_tw;
  hp.desc = pd;
  std::memcpy(host.data() + o_plan, &pd, sizeof(PlanDesc));
  std::memcpy(host.data() + o_tiles, tiles.data(), sizeof(FoldTile) * tiles.size());
  std::memcpy(host.data() + o_items, items.data(), sizeof(RoundItem) * items.size());
  std::memcpy(host.data() + o_groups, groups.data(), sizeof(FftGroup) * groups.size());
  e = hipMemcpy(p->d_mem, host.data(), o_ws, hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpy(plan descriptors)");
  p->d_plan = reinterpret_cast<PlanDesc*>(p->d_mem + o_plan);
  p->d_tiles = reinterpret_cast<FoldTile*>(p->d_mem + o_tiles);
  p->d_items = reinterpret_cast<RoundItem*>(p->d_mem + o_items);
  p->d_groups = reinterpret_cast<FftGroup*>(p->d_mem + o_groups);
  p->d_ws = p->d_mem + o_ws;
  p->on_device = true;
  return SFFT_OK;
}

sfft_status check_plan(sfft_plan_t p) {
  if (!p) return fail(SFFT_ERR_PARAM, "null plan");
  if (!p->on_device) return fail(SFFT_ERR_STATE, "plan was built with SFFT_PLAN_HOST_ONLY");
  return SFFT_OK;
}

SigArg single(const SignalDesc& sd) {
  SigArg a;
  a.table = nullptr;
  a.one = sd;
  return a;
}

SignalDesc make_signal(sfft_plan_t p, const void* d_x, float scale, void* y, int64_t* d_idx, void* d_val,
                       int64_t* d_count) {
  SignalDesc sd{};
  sd.plan = p->d_plan;
  sd.x = d_x;
  sd.ws = p->d_ws;
  sd.y = y ? y : p->d_ws + p->hp.desc.off_y;
  sd.idx = d_idx;
  sd.val = d_val;
  sd.count = d_count;
  sd.scale = scale;
  return sd;
}

uint32_t max_B(const HostPlan& hp) {
  uint32_t b = 0;
  for (auto& it : hp.iters) b = std::max(b, it.d.B);
  return b;
}

sfft_status run_hash(sfft_plan_t p, const SigArg& a, hipStream_t s) {
  int e = launch_fold(p->hp.dtype, p->hp.kahan, p->fold, a, p->d_tiles, p->ntiles, p->split, s);
  if (e != hipSuccess) return hip_fail(hipError_t(e), "fold launch");
  e = launch_bucket_fft(p->hp.dtype, a, p->d_items, p->d_groups, p->fft, s);
  if (e != hipSuccess) return hip_fail(hipError_t(e), "bucket FFT launch");
  return SFFT_OK;
}

int launch_batch_fold(const sfft_batch_s* b, const FoldConfig& cfg, hipStream_t s);

SigArg table_arg(const sfft_batch_s* b) {
  SigArg a;
  std::memset(&a, 0, sizeof(a));
  a.table = b->d_sigs;
  return a;
}

// The fused launch's work items: per chunk of `chunk` counter groups, every
// fold tile of the chunk's groups, then the finish item of each of their
// signals.
void build_fused_items(const sfft_batch_s* b, uint32_t chunk, std::vector<FusedItem>& out) {
  out.clear();
  const uint32_t nsig = uint32_t(b->plans.size());
  for (uint32_t g0 = 0; g0 < b->nfgroups; g0 += chunk) {
    const uint32_t g1 = std::min(b->nfgroups, g0 + chunk);
    for (uint32_t g = g0; g < g1; ++g)
      for (const FoldTile& t : b->group_tiles[g]) out.push_back(FusedItem{kFusedFold, t.sig, t.m, t.i0});
    const uint32_t s0 = b->interleaved ? g0 * kIlvSigs : g0;
    const uint32_t s1 = std::min(nsig, b->interleaved ? g1 * kIlvSigs : g1);
    for (uint32_t s = s0; s < s1; ++s) out.push_back(FusedItem{kFusedFinish, s, 0, 0});
  }
}

FusedArgs fused_args(const sfft_batch_s* b) {
  FusedArgs a;
  a.table = b->d_sigs;
  a.nsig = uint32_t(b->plans.size());
  a.nitems = b->nfitems;
  a.items = b->d_fitems;
  a.ctl = b->d_ctl;
  a.need = b->d_need;
  return a;
}

int launch_batch_fused(const sfft_batch_s* b, hipStream_t s) {
  return launch_fused(b->dtype, b->kahan, b->interleaved, b->fused_grid, 2 + b->nfgroups, fused_args(b), s);
}

// Cuts the round items into bucket-DFT groups of at most `points` points and
// uploads them (synchronously).
sfft_status regroup_fft(sfft_batch_s* b, uint32_t points) {
  std::vector<RoundItem> items = b->h_items;
  std::vector<FftGroup> groups;
  FftGroups fg;
  group_rounds(items, [&](const RoundItem& r) { return b->plans[r.sig]->hp.iters[r.m].d.B; }, b->dtype, groups, fg,
               points);
  hipError_t e = hipMemcpy(b->d_items, items.data(), sizeof(RoundItem) * items.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(b->d_groups, groups.data(), sizeof(FftGroup) * groups.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "bucket-DFT groups upload");
  b->fft = fg;
  b->fft_group_points = points;
  return SFFT_OK;
}

// Signals per lane of the position-major fold: the shape's count, or as many
// as the bound input allows (0), never more than it allows.
int fold_lanes(const sfft_batch_s* b, const FoldConfig& cfg) {
  return cfg.lanes == 0 ? b->lanes_max : std::min(cfg.lanes, b->lanes_max);
}

int launch_batch_fold(const sfft_batch_s* b, const FoldConfig& cfg, hipStream_t s) {
  if (b->interleaved)
    return launch_fold_interleaved(b->dtype, b->kahan, cfg.unroll, fold_lanes(b, cfg), b->d_sigs,
                                   uint32_t(b->plans.size()), b->d_tiles, b->ntiles, s);
  return launch_fold(b->dtype, b->kahan, cfg, table_arg(b), b->d_tiles, b->ntiles, b->split, s);
}

}  // namespace

extern "C" {

void sfft_default_options(sfft_options* opt) {
  if (!opt) return;
  std::memset(opt, 0, sizeof(*opt));
  opt->delta = 1e-6;
  opt->seed = 0;
  opt->dtype = SFFT_C64;
  opt->kahan = 0;
  opt->b_min = 16;
  opt->eta = 1e-4;
  opt->rho = 0.25;
  opt->flags = 0;
}

const char* sfft_status_string(sfft_status s) {
  switch (s) {
    case SFFT_OK: return "ok";
    case SFFT_ERR_PARAM: return "invalid parameter";
    case SFFT_ERR_UNSUPPORTED: return "unsupported configuration";
    case SFFT_ERR_ALLOC: return "allocation failed";
    case SFFT_ERR_LAUNCH: return "launch failed";
    case SFFT_ERR_CAPACITY: return "capacity exceeded";
    case SFFT_ERR_STATE: return "invalid state";
  }
  return "unknown status";
}

const char* sfft_last_error(void) { return g_last_error.c_str(); }

sfft_status sfft_plan(sfft_plan_t* out, int64_t N, int64_t K, int64_t B, int64_t w, int32_t loops,
                      int32_t multiscale, double extension, const sfft_options* opt) {
  if (!out) return fail(SFFT_ERR_PARAM, "out is NULL");
  *out = nullptr;
  sfft_options o;
  sfft_default_options(&o);
  if (opt) o = *opt;
  alloc_trial_begin();
  sfft_plan_t p = alloc_should_fail() ? nullptr : new (std::nothrow) sfft_plan_s();
  if (!p) return fail(SFFT_ERR_ALLOC, "host allocation of the plan failed");
  std::string err;
  sfft_status st;
  try {
    st = build_host_plan(p->hp, N, K, B, w, loops, multiscale, extension, o, &err);
  } catch (const std::bad_alloc&) {
    st = SFFT_ERR_ALLOC;
    err = "host allocation failed while building the plan";
  }
  if (st != SFFT_OK) {
    delete p;
    return fail(st, err);
  }
  if (!(o.flags & SFFT_PLAN_HOST_ONLY)) {
    try {
      st = upload_plan(p);
    } catch (const std::bad_alloc&) {
      st = fail(SFFT_ERR_ALLOC, "host allocation failed while uploading the plan");
    }
    if (st != SFFT_OK) {
      if (p->d_mem) (void)hipFree(p->d_mem);
      delete p;
      return st;
    }
  }
  *out = p;
  return SFFT_OK;
}

sfft_status sfft_destroy(sfft_plan_t p) {
  if (!p) return SFFT_OK;
  if (p->d_mem) (void)hipFree(p->d_mem);
  delete p;
  return SFFT_OK;
}

sfft_status sfft_get_plan_info(sfft_plan_t p, sfft_plan_info* info) {
  if (!p || !info) return fail(SFFT_ERR_PARAM, "null argument");
  const HostPlan& hp = p->hp;
  std::memset(info, 0, sizeof(*info));
  info->N = hp.N; info->K = hp.K; info->B = hp.B; info->w = hp.w;
  info->loops = hp.loops; info->multiscale = hp.l;
  info->extension = hp.q; info->delta = hp.delta;
  info->dtype = hp.dtype; info->kahan = hp.kahan;
  info->samples = hp.samples;
  info->yhat_elems = int64_t(hp.desc.y_total);
  info->rec_capacity = hp.desc.rec_cap;
  info->workspace_bytes = int64_t(hp.desc.ws_bytes);
  info->seed = hp.seed;
  return SFFT_OK;
}

sfft_status sfft_get_iter_info(sfft_plan_t p, int32_t m, sfft_iter_info* info) {
  if (!p || !info) return fail(SFFT_ERR_PARAM, "null argument");
  if (m < 0 || m >= p->hp.loops) return fail(SFFT_ERR_PARAM, "iteration index out of range");
  const IterHost& it = p->hp.iters[m];
  std::memset(info, 0, sizeof(*info));
  info->B = it.d.B; info->L = it.d.L; info->w = it.d.w; info->h = it.d.h; info->e = it.d.e; info->R = it.d.R;
  info->d_delta = it.d_delta;
  info->sigma = it.d.sigma; info->sigma_inv = it.d.sigma_inv; info->tau0 = it.d.tau0;
  info->y_offset = int64_t(it.d.y_off);
  for (uint32_t j = 0; j <= it.d.R; ++j) {
    info->T[j] = it.d.T[j];
    info->tau[j] = it.d.tau[j];
    info->len[j] = it.d.len[j];
  }
  info->last_kind = p->hp.desc.location == SFFT_LOCATE_DIRECT ? 2 : 1;
  return SFFT_OK;
}

sfft_status sfft_plan_dump_tables(sfft_plan_t p, int32_t m, double* h_window, double* h_ghat) {
  if (!p) return fail(SFFT_ERR_PARAM, "null plan");
  if (m < 0 || m >= p->hp.loops) return fail(SFFT_ERR_PARAM, "iteration index out of range");
  const IterHost& it = p->hp.iters[m];
  if (h_window) std::memcpy(h_window, it.G->data(), it.G->size() * sizeof(double));
  if (h_ghat) std::memcpy(h_ghat, it.Ghat->data(), it.Ghat->size() * sizeof(double));
  return SFFT_OK;
}

sfft_status sfft_execute(sfft_plan_t p, const void* d_x, float scale, int64_t* d_idx, void* d_val, int64_t* d_count,
                         void* stream) {
  sfft_status st = check_plan(p);
  if (st != SFFT_OK) return st;
  if (!d_x || !d_idx || !d_val || !d_count) return fail(SFFT_ERR_PARAM, "null buffer");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const SigArg a = single(make_signal(p, d_x, scale, nullptr, d_idx, d_val, d_count));
  st = run_hash(p, a, s);
  if (st != SFFT_OK) return st;
  int e = launch_recover(p->hp.dtype, a, 1, s);
  if (e != hipSuccess) return hip_fail(hipError_t(e), "recover launch");
  return SFFT_OK;
}

sfft_status sfft_execute_noalloc(sfft_plan_t p, const void* d_x, float scale, int64_t* d_idx, void* d_val,
                                 int64_t* d_count, void* stream) {
  sfft_status st = check_plan(p);
  if (st != SFFT_OK) return st;
  if (!d_x || !d_idx || !d_val || !d_count) return fail(SFFT_ERR_PARAM, "null buffer");
  if (p->hp.desc.ws_bytes > kScratchBytes)
    return fail(SFFT_ERR_CAPACITY, "plan workspace of " + std::to_string(p->hp.desc.ws_bytes) +
                                       " bytes exceeds the static scratch of " + std::to_string(kScratchBytes) +
                                       " bytes");
  hipError_t e = hipSuccess;
  unsigned char* ws = static_cast<unsigned char*>(scratch_address(&e));
  if (!ws) return hip_fail(e, "hipGetSymbolAddress(scratch)");
  // every workspace word the kernels read is written first in the same call
  // (bucket values by the fold and the DFT, the store and its index by the
  // recovery's own initialization), so nothing is cleared here
  SignalDesc sd = make_signal(p, d_x, scale, nullptr, d_idx, d_val, d_count);
  sd.ws = ws;
  sd.y = ws + p->hp.desc.off_y;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const SigArg a = single(sd);
  st = run_hash(p, a, s);
  if (st != SFFT_OK) return st;
  int le = launch_recover(p->hp.dtype, a, 1, s);
  if (le != hipSuccess) return hip_fail(hipError_t(le), "recover launch");
  return SFFT_OK;
}

sfft_status sfft_hash_to_bins(sfft_plan_t p, const void* d_x, float scale, void* d_yhat, void* stream) {
  sfft_status st = check_plan(p);
  if (st != SFFT_OK) return st;
  if (!d_x || !d_yhat) return fail(SFFT_ERR_PARAM, "null buffer");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  return run_hash(p, single(make_signal(p, d_x, scale, d_yhat, nullptr, nullptr, nullptr)), s);
}

sfft_status sfft_recover(sfft_plan_t p, const void* d_yhat, int64_t* d_idx, void* d_val, int64_t* d_count,
                         void* stream) {
  sfft_status st = check_plan(p);
  if (st != SFFT_OK) return st;
  if (!d_yhat || !d_idx || !d_val || !d_count) return fail(SFFT_ERR_PARAM, "null buffer");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const uint64_t bytes = p->hp.desc.y_total * (p->hp.dtype == SFFT_C128 ? 16 : 8);
  hipError_t e = hipMemcpyAsync(p->d_ws + p->hp.desc.off_y, d_yhat, bytes, hipMemcpyDeviceToDevice, s);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(yhat)");
  int le = launch_recover(p->hp.dtype, single(make_signal(p, nullptr, 1.0f, nullptr, d_idx, d_val, d_count)), 1, s);
  if (le != hipSuccess) return hip_fail(hipError_t(le), "recover launch");
  return SFFT_OK;
}

sfft_status create_batch_impl(sfft_batch_t* out, const sfft_plan_t* h_plans, int32_t n, bool interleaved) {
  if (!out || !h_plans || n < 1) return fail(SFFT_ERR_PARAM, "need at least one plan");
  *out = nullptr;
  for (int32_t s = 0; s < n; ++s) {
    sfft_status st = check_plan(h_plans[s]);
    if (st != SFFT_OK) return st;
    if (h_plans[s]->hp.dtype != h_plans[0]->hp.dtype || h_plans[s]->hp.kahan != h_plans[0]->hp.kahan)
      return fail(SFFT_ERR_PARAM, "all plans of a batch must share dtype and kahan");
  }
  sfft_batch_t b = alloc_should_fail() ? nullptr : new (std::nothrow) sfft_batch_s();
  if (!b) return fail(SFFT_ERR_ALLOC, "host allocation of the batch failed");
  struct Guard {  // releases the half-built batch if a host container throws
    sfft_batch_t b;
    ~Guard() { delete b; }
  } guard{b};
  b->plans.assign(h_plans, h_plans + n);
  b->dtype = h_plans[0]->hp.dtype;
  b->kahan = h_plans[0]->hp.kahan;
  b->fold = h_plans[0]->fold;
  b->interleaved = interleaved;
  std::vector<FoldTile> tiles;
  std::vector<RoundItem> items;
  uint64_t ws = 0;
  const uint32_t cb = b->dtype == SFFT_C128 ? 16u : 8u;
  b->fused_ok = true;
  for (int32_t s = 0; s < n; ++s) {
    const HostPlan& hp = h_plans[s]->hp;
    const size_t t0 = tiles.size();
    build_work_lists(hp, uint32_t(s), tiles, items);
    if (!interleaved) b->group_tiles.emplace_back(tiles.begin() + t0, tiles.end());
    b->ws_off.push_back(ws);
    ws += align256(hp.desc.ws_bytes);
    b->max_B = std::max(b->max_B, max_B(hp));
    if (uint64_t(max_B(hp)) * cb > kRecoverLdsBytes) b->fused_ok = false;
  }
  if (interleaved) {
    b->ngroups = uint32_t((n + kIlvSigs - 1) / kIlvSigs);
    tiles.clear();
    interleaved_tiles(h_plans[0]->hp, b->ngroups, tiles);
    b->group_tiles.resize(b->ngroups);
    for (const FoldTile& t : tiles) b->group_tiles[t.sig].push_back(t);
  } else {
    b->split = order_for_stages(tiles);  // group_tiles keep each signal's own order for the fused launch
  }
  b->nfgroups = uint32_t(b->group_tiles.size());
  b->h_items = items;
  std::vector<FftGroup> groups;
  group_rounds(items, [&](const RoundItem& r) { return h_plans[r.sig]->hp.iters[r.m].d.B; }, b->dtype, groups,
               b->fft);
  b->ntiles = uint32_t(tiles.size());
  b->nitems = uint32_t(items.size());
  // the fused launch: one chunk per signal group (position-major) or per 32 signals
  b->fused_chunk = interleaved ? 1u : std::min<uint32_t>(32u, uint32_t(n));
  std::vector<FusedItem> fitems;
  build_fused_items(b, b->fused_chunk, fitems);
  b->nfitems = uint32_t(fitems.size());
  std::vector<uint32_t> need(b->nfgroups);
  for (uint32_t g = 0; g < b->nfgroups; ++g) need[g] = uint32_t(b->group_tiles[g].size());
  int dev = 0, ncu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return hip_fail(e, "device attributes");
  b->fused_grid = uint32_t(std::max(1, ncu)) * 2u;  // two workgroups of the fused kernel fit a compute unit
  const uint64_t o_sigs = 0;
  const uint64_t o_tiles = align256(sizeof(SignalDesc) * n);
  const uint64_t o_items = o_tiles + align256(sizeof(FoldTile) * tiles.size());
  const uint64_t o_groups = o_items + align256(sizeof(RoundItem) * items.size());
  // room for the smallest grouping (one round per group)
  const uint64_t o_fitems = o_groups + align256(sizeof(FftGroup) * items.size());
  const uint64_t o_ctl = o_fitems + align256(sizeof(FusedItem) * fitems.size());
  const uint64_t o_need = o_ctl + align256(sizeof(uint32_t) * (2 + b->nfgroups));
  const uint64_t o_ws = o_need + align256(sizeof(uint32_t) * b->nfgroups);
  e = dev_malloc(reinterpret_cast<void**>(&b->d_mem), o_ws + ws);
  if (e != hipSuccess) return hip_fail(e, "hipMalloc(batch)");
  b->d_sigs = reinterpret_cast<SignalDesc*>(b->d_mem + o_sigs);
  b->d_tiles = reinterpret_cast<FoldTile*>(b->d_mem + o_tiles);
  b->d_items = reinterpret_cast<RoundItem*>(b->d_mem + o_items);
  b->d_groups = reinterpret_cast<FftGroup*>(b->d_mem + o_groups);
  b->d_fitems = reinterpret_cast<FusedItem*>(b->d_mem + o_fitems);
  b->d_ctl = reinterpret_cast<uint32_t*>(b->d_mem + o_ctl);
  b->d_need = reinterpret_cast<uint32_t*>(b->d_mem + o_need);
  b->d_ws = b->d_mem + o_ws;
  e = hipMemcpy(b->d_tiles, tiles.data(), sizeof(FoldTile) * tiles.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(b->d_items, items.data(), sizeof(RoundItem) * items.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(b->d_groups, groups.data(), sizeof(FftGroup) * groups.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(b->d_fitems, fitems.data(), sizeof(FusedItem) * fitems.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(b->d_need, need.data(), sizeof(uint32_t) * need.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->capture_stream, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->replayed, hipEventDisableTiming);
  if (e != hipSuccess) {
    if (b->capture_stream) (void)hipStreamDestroy(b->capture_stream);
    (void)hipFree(b->d_mem);
    return hip_fail(e, "batch setup");
  }
  guard.b = nullptr;
  *out = b;
  return SFFT_OK;
}

// Host containers of the work lists may throw on exhaustion; nothing throws
// across the ABI.
sfft_status create_batch(sfft_batch_t* out, const sfft_plan_t* h_plans, int32_t n, bool interleaved) {
  alloc_trial_begin();
  try {
    return create_batch_impl(out, h_plans, n, interleaved);
  } catch (const std::bad_alloc&) {
    return fail(SFFT_ERR_ALLOC, "host allocation failed while building the batch");
  }
}

sfft_status sfft_batch_create(sfft_batch_t* out, const sfft_plan_t* h_plans, int32_t n) {
  return create_batch(out, h_plans, n, false);
}

// Uploads the descriptor table when the buffers changed, captures the three
// stages into the batch graph when there is none, and replays it on `stream`.
sfft_status bind_and_replay(sfft_batch_t b, const std::vector<SignalDesc>& sig, hipStream_t s) {
  const size_t n = sig.size();
  const bool same = b->has_binding && std::memcmp(sig.data(), b->bound.data(), sizeof(SignalDesc) * n) == 0;
  if (!same) {
    // new buffers: wait for this batch's work in flight, then upload the table
    hipError_t e = hipStreamSynchronize(s);
    if (e == hipSuccess) e = hipMemcpy(b->d_sigs, sig.data(), sizeof(SignalDesc) * n, hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "batch descriptor upload");
    b->bound = sig;
    b->has_binding = true;
  }
  if (!b->exec) {  // first execute, or the launch shape changed: capture the three stages
    hipStream_t cs = b->capture_stream;
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
    const SigArg a = table_arg(b);
    int le;
    if (b->mode == SFFT_BATCH_FUSED) {
      le = launch_batch_fused(b, cs);
    } else {
      le = launch_batch_fold(b, b->fold, cs);
      if (le == hipSuccess) le = launch_bucket_fft(b->dtype, a, b->d_items, b->d_groups, b->fft, cs);
      if (le == hipSuccess) le = launch_recover(b->dtype, a, uint32_t(n), cs);
    }
    hipGraph_t g = nullptr;
    hipError_t ee = hipStreamEndCapture(cs, &g);
    if (le != hipSuccess) return hip_fail(hipError_t(le), "batch capture launch");
    if (ee != hipSuccess) return hip_fail(ee, "hipStreamEndCapture");
    b->graph = g;
    ee = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
    if (ee != hipSuccess) {
      b->exec = nullptr;
      return hip_fail(ee, "hipGraphInstantiate");
    }
  }
  hipError_t e = hipGraphLaunch(b->exec, s);
  if (e == hipSuccess) e = hipEventRecord(b->replayed, s);
  if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
  b->replay_recorded = true;
  return SFFT_OK;
}

sfft_status sfft_execute_batch(sfft_batch_t b, const void* const* h_x, const float* h_scale, int64_t* const* h_idx,
                               void* const* h_val, int64_t* d_count, void* stream) {
  if (!b || !h_x || !h_idx || !h_val || !d_count) return fail(SFFT_ERR_PARAM, "null argument");
  if (b->interleaved) return fail(SFFT_ERR_STATE, "position-major batch: use sfft_execute_interleaved");
  const size_t n = b->plans.size();
  std::vector<SignalDesc> sig(n);
  for (size_t i = 0; i < n; ++i) {
    if (!h_x[i] || !h_idx[i] || !h_val[i]) return fail(SFFT_ERR_PARAM, "null signal buffer");
    sfft_plan_t p = b->plans[i];
    SignalDesc& sd = sig[i];
    sd.plan = p->d_plan;
    sd.x = h_x[i];
    sd.ws = b->d_ws + b->ws_off[i];
    sd.y = b->d_ws + b->ws_off[i] + p->hp.desc.off_y;
    sd.idx = h_idx[i];
    sd.val = h_val[i];
    sd.count = d_count + i;
    sd.scale = h_scale ? h_scale[i] : 1.0f;
    sd.ld = 0;
  }
  return bind_and_replay(b, sig, reinterpret_cast<hipStream_t>(stream));
}

sfft_status sfft_batch_create_interleaved(sfft_batch_t* out, sfft_plan_t plan, int32_t nsig) {
  if (!out || nsig < 1) return fail(SFFT_ERR_PARAM, "need a plan and at least one signal");
  std::vector<sfft_plan_t> plans(size_t(nsig), plan);
  return create_batch(out, plans.data(), nsig, true);
}

static sfft_status drop_graph(sfft_batch_t b);

sfft_status sfft_execute_interleaved(sfft_batch_t b, const void* d_x, int64_t ld, const float* h_scale,
                                     int64_t* d_idx, void* d_val, int64_t* d_count, void* stream) {
  if (!b || !d_x || !d_idx || !d_val || !d_count) return fail(SFFT_ERR_PARAM, "null argument");
  if (!b->interleaved) return fail(SFFT_ERR_STATE, "not a position-major batch: use sfft_execute_batch");
  const size_t n = b->plans.size();
  if (ld < int64_t(n) || ld > int64_t(UINT32_MAX)) return fail(SFFT_ERR_PARAM, "ld must satisfy nsig <= ld < 2^32");
  sfft_plan_t p = b->plans[0];
  const uint64_t es = b->dtype == SFFT_C128 ? 16 : b->dtype == SFFT_F16X2_SCALED ? 4 : 8;  // input element
  const uint64_t vs = b->dtype == SFFT_C128 ? 16 : 8;                                      // output value
  const uint64_t K = p->hp.desc.K;
  std::vector<SignalDesc> sig(n);
  for (size_t i = 0; i < n; ++i) {
    SignalDesc& sd = sig[i];
    sd.plan = p->d_plan;
    sd.x = reinterpret_cast<const unsigned char*>(d_x) + i * es;
    sd.ws = b->d_ws + b->ws_off[i];
    sd.y = b->d_ws + b->ws_off[i] + p->hp.desc.off_y;
    sd.idx = d_idx + i * K;
    sd.val = reinterpret_cast<unsigned char*>(d_val) + i * K * vs;
    sd.count = d_count + i;
    sd.scale = h_scale ? h_scale[i] : 1.0f;
    sd.ld = uint32_t(ld);
  }
  // L adjacent signals per fold lane where each lane's run is one aligned
  // load of L live signals: L = 2 for complex64, 2 or 4 for FP16 pairs (the
  // fold shape picks up to this many); a change captures the graph again
  int lanes_max = 1;
  for (int L : {4, 2}) {
    const int most = b->dtype == SFFT_C128 ? 1 : b->dtype == SFFT_F16X2_SCALED ? 4 : 2;
    if (L <= most && b->ngroups % uint32_t(L) == 0 && n % size_t(L) == 0 && ld % L == 0 &&
        reinterpret_cast<uintptr_t>(d_x) % (uint64_t(L) * es) == 0) {
      lanes_max = L;
      break;
    }
  }
  if (lanes_max != b->lanes_max) {
    const sfft_status st = drop_graph(b);
    if (st != SFFT_OK) return st;
    b->lanes_max = lanes_max;
  }
  return bind_and_replay(b, sig, reinterpret_cast<hipStream_t>(stream));
}

// Drops the batch's captured graph once its last replay has ended (an event on
// the caller's stream); the next execute captures again.
static sfft_status drop_graph(sfft_batch_t b) {
  if (!b->exec && !b->graph) return SFFT_OK;
  const hipError_t e = b->replay_recorded ? hipEventSynchronize(b->replayed) : hipSuccess;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
  if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
  return SFFT_OK;
}

sfft_status sfft_batch_launch_stage(sfft_batch_t b, int32_t stage, void* stream) {
  if (!b) return fail(SFFT_ERR_PARAM, "null batch");
  if (!b->has_binding) return fail(SFFT_ERR_STATE, "no buffers bound: execute the batch first");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  int e;
  const SigArg a = table_arg(b);
  switch (stage) {
    case 0: e = launch_batch_fold(b, b->fold, s); break;
    case 1: e = launch_bucket_fft(b->dtype, a, b->d_items, b->d_groups, b->fft, s); break;
    case 2: e = launch_recover(b->dtype, a, uint32_t(b->plans.size()), s); break;
    case 3:
      if (!b->fused_ok) return fail(SFFT_ERR_UNSUPPORTED, "a round of this batch does not fit the fused kernel's LDS");
      e = launch_batch_fused(b, s);
      break;
    default: return fail(SFFT_ERR_PARAM, "stage must be 0, 1, 2 or 3");
  }
  if (e != hipSuccess) return hip_fail(hipError_t(e), "stage launch");
  return SFFT_OK;
}

sfft_status sfft_plan_set_fold_config(sfft_plan_t p, const sfft_fold_config* cfg) {
  if (!p || !valid_fold(cfg)) return fail(SFFT_ERR_PARAM, "invalid fold configuration");
  p->fold = FoldConfig{cfg->unroll, cfg->wg_per_cu};
  return SFFT_OK;
}

sfft_status sfft_batch_set_fold_config(sfft_batch_t b, const sfft_fold_config* cfg) {
  if (!b || !valid_fold(cfg)) return fail(SFFT_ERR_PARAM, "invalid fold configuration");
  b->fold = FoldConfig{cfg->unroll, cfg->wg_per_cu, b->fold.lanes};
  return drop_graph(b);
}

sfft_status sfft_batch_get_tuning(sfft_batch_t b, sfft_batch_tuning* t) {
  if (!b || !t) return fail(SFFT_ERR_PARAM, "null argument");
  std::memset(t, 0, sizeof(*t));
  t->mode = b->mode;
  t->fused_chunk = int32_t(b->fused_chunk);
  t->fold_unroll = b->fold.unroll;
  t->fold_wg_per_cu = b->fold.wg_per_cu;
  t->fft_group_points = int32_t(b->fft_group_points);
  t->fused_available = b->fused_ok ? 1 : 0;
  t->step_ms = double(b->step_ms);
  t->fold_lanes = !b->interleaved ? 1 : b->has_binding ? fold_lanes(b, b->fold) : b->fold.lanes;
  return SFFT_OK;
}

sfft_status sfft_batch_set_tuning(sfft_batch_t b, const sfft_batch_tuning* t) {
  if (!b || !t) return fail(SFFT_ERR_PARAM, "null argument");
  const sfft_fold_config fc{t->fold_unroll, t->fold_wg_per_cu, 0.0};
  if (!valid_fold(&fc)) return fail(SFFT_ERR_PARAM, "invalid fold configuration");
  if (t->mode != SFFT_BATCH_STAGES && t->mode != SFFT_BATCH_FUSED) return fail(SFFT_ERR_PARAM, "invalid mode");
  if (t->mode == SFFT_BATCH_FUSED && !b->fused_ok)
    return fail(SFFT_ERR_UNSUPPORTED, "a round of this batch does not fit the fused kernel's LDS");
  if (t->mode == SFFT_BATCH_FUSED && (t->fused_chunk < 1 || uint32_t(t->fused_chunk) > b->nfgroups))
    return fail(SFFT_ERR_PARAM, "fused_chunk must be in 1 .. the number of signals (or groups of 64)");
  if (t->fft_group_points != 1024 && t->fft_group_points != 2048 && t->fft_group_points != 4096)
    return fail(SFFT_ERR_PARAM, "fft_group_points must be 1024, 2048 or 4096");
  if (t->fold_lanes != 0 && t->fold_lanes != 1 && t->fold_lanes != 2 && t->fold_lanes != 4)
    return fail(SFFT_ERR_PARAM, "fold_lanes must be 0, 1, 2 or 4");
  sfft_status st = drop_graph(b);  // the device lists below are read by the last replay
  if (st != SFFT_OK) return st;
  if (uint32_t(t->fft_group_points) != b->fft_group_points) {
    st = regroup_fft(b, uint32_t(t->fft_group_points));
    if (st != SFFT_OK) return st;
  }
  if (t->mode == SFFT_BATCH_FUSED && uint32_t(t->fused_chunk) != b->fused_chunk) {
    std::vector<FusedItem> items;
    build_fused_items(b, uint32_t(t->fused_chunk), items);
    const hipError_t e = hipMemcpy(b->d_fitems, items.data(), sizeof(FusedItem) * items.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "fused items upload");
    b->fused_chunk = uint32_t(t->fused_chunk);
  }
  b->mode = t->mode;
  b->fold = FoldConfig{t->fold_unroll, t->fold_wg_per_cu, t->fold_lanes};
  return SFFT_OK;
}

}  // extern "C"

namespace {

// Choices of the autotuner, per batch shape, for the life of the process.
std::mutex g_tune_mu;
struct TuneChoice {
  sfft_batch_tuning tuning;
  double fold_ms;  // the winning fold shape's mean time when it was chosen
};
std::map<std::string, TuneChoice> g_tune_cache;

std::string tuning_key(const sfft_batch_s* b) {
  const std::string layout = b->interleaved ? "pm" + std::to_string(b->lanes_max) : std::string("ps");
  std::string k = std::to_string(b->dtype) + "/" + std::to_string(b->kahan) + "/" + layout + "/" +
                  std::to_string(b->plans.size());
  uint64_t h = 1469598103934665603ull;  // FNV-1a over every plan's shape
  for (const sfft_plan_t p : b->plans) {
    const uint64_t v[6] = {uint64_t(p->hp.N), uint64_t(p->hp.B), uint64_t(p->hp.w), uint64_t(p->hp.loops),
                           uint64_t(p->hp.l), uint64_t(p->hp.desc.combine)};
    for (uint64_t x : v)
      for (int i = 0; i < 8; ++i) h = (h ^ ((x >> (8 * i)) & 255u)) * 1099511628211ull;
  }
  return k + "/" + std::to_string(h);
}

// Mean time of `reps` launches of fn() on s (one warm-up first); negative on a launch error.
template <class F>
float time_launches(F fn, hipStream_t s, hipEvent_t e0, hipEvent_t e1, int reps, int* err) {
  int le = fn();
  float total = 0.f;
  for (int r = 0; r < reps && le == hipSuccess; ++r) {
    (void)hipEventRecord(e0, s);
    le = fn();
    (void)hipEventRecord(e1, s);
    if (hipEventSynchronize(e1) != hipSuccess) le = hipErrorLaunchFailure;
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    total += ms;
  }
  *err = le;
  return total / float(reps);
}

}  // namespace

extern "C" {

sfft_status sfft_batch_autotune(sfft_batch_t b, void* stream, sfft_fold_config* best) {
  if (!b) return fail(SFFT_ERR_PARAM, "null batch");
  if (!b->has_binding) return fail(SFFT_ERR_STATE, "no buffers bound: execute the batch first");
  const std::string key = tuning_key(b);
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto hit = g_tune_cache.find(key);
    if (hit != g_tune_cache.end()) {
      sfft_status st = sfft_batch_set_tuning(b, &hit->second.tuning);
      if (st != SFFT_OK) return st;
      b->step_ms = float(hit->second.tuning.step_ms);
      if (best) *best = sfft_fold_config{b->fold.unroll, b->fold.wg_per_cu, hit->second.fold_ms};
      return SFFT_OK;
    }
  }
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  sfft_status st = drop_graph(b);
  if (st != SFFT_OK) return st;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return fail(SFFT_ERR_LAUNCH, "hipEventCreate");
  int err = hipSuccess;
  const SigArg a = table_arg(b);
  // 1. fold launch shape: taps in flight x residency cap (per-signal layout)
  //    or x signals per lane (position-major: 1, 2 or 4, as the input allows)
  const int unrolls[3] = {8, 16, 24};
  const int caps[5] = {0, 2, 3, 4, 6};
  const int lanes[3] = {1, 2, 4};
  const int ncaps = b->interleaved ? (b->lanes_max == 4 ? 3 : b->lanes_max) : 5;
  FoldConfig win = b->fold;
  float fold_ms = 1e30f;
  for (int ui = 0; ui < 3 && err == hipSuccess; ++ui)
    for (int ci = 0; ci < ncaps && err == hipSuccess; ++ci) {
      const FoldConfig c = b->interleaved ? FoldConfig{unrolls[ui], 0, lanes[ci]} : FoldConfig{unrolls[ui], caps[ci]};
      const float ms = time_launches([&] { return launch_batch_fold(b, c, s); }, s, e0, e1, 3, &err);
      if (err == hipSuccess && ms < fold_ms) {
        fold_ms = ms;
        win = c;
      }
    }
  b->fold = win;
  // 2. bucket-DFT workgroup size
  uint32_t fft_win = b->fft_group_points;
  float fft_ms = 1e30f;
  for (uint32_t pts : {1024u, 2048u, 4096u}) {
    if (err != hipSuccess) break;
    st = regroup_fft(b, pts);
    if (st != SFFT_OK) break;
    const float ms = time_launches(
        [&] { return launch_bucket_fft(b->dtype, a, b->d_items, b->d_groups, b->fft, s); }, s, e0, e1, 3,
        &err);
    if (err == hipSuccess && ms < fft_ms) {
      fft_ms = ms;
      fft_win = pts;
    }
  }
  if (st == SFFT_OK && err == hipSuccess) st = regroup_fft(b, fft_win);
  // 3. the whole step: the three stage launches against the fused launch at
  //    several chunk sizes
  sfft_batch_tuning tw{};
  tw.mode = SFFT_BATCH_STAGES;
  tw.fold_unroll = win.unroll;
  tw.fold_wg_per_cu = win.wg_per_cu;
  tw.fold_lanes = win.lanes;
  tw.fft_group_points = int32_t(fft_win);
  tw.fused_chunk = int32_t(b->fused_chunk);
  float step = 1e30f;
  if (st == SFFT_OK && err == hipSuccess) {
    step = time_launches(
        [&] {
          int le = launch_batch_fold(b, b->fold, s);
          if (le == hipSuccess) le = launch_bucket_fft(b->dtype, a, b->d_items, b->d_groups, b->fft, s);
          if (le == hipSuccess) le = launch_recover(b->dtype, a, uint32_t(b->plans.size()), s);
          return le;
        },
        s, e0, e1, 3, &err);
  }
  if (b->fused_ok && st == SFFT_OK && err == hipSuccess) {
    const uint32_t base = b->interleaved ? 1u : 16u;
    for (uint32_t ch : {base, 2 * base, 4 * base, 8 * base}) {
      if (ch > b->nfgroups || err != hipSuccess || st != SFFT_OK) break;
      sfft_batch_tuning t = tw;
      t.mode = SFFT_BATCH_FUSED;
      t.fused_chunk = int32_t(ch);
      st = sfft_batch_set_tuning(b, &t);
      if (st != SFFT_OK) break;
      const float ms = time_launches([&] { return launch_batch_fused(b, s); }, s, e0, e1, 3, &err);
      if (err == hipSuccess && ms < step) {
        step = ms;
        tw = t;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (err != hipSuccess) return hip_fail(hipError_t(err), "autotune launch");
  if (st != SFFT_OK) return st;
  tw.step_ms = double(step);
  st = sfft_batch_set_tuning(b, &tw);
  if (st != SFFT_OK) return st;
  b->step_ms = step;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[key] = TuneChoice{tw, double(fold_ms)};
  }
  if (best) *best = sfft_fold_config{win.unroll, win.wg_per_cu, double(fold_ms)};
  return SFFT_OK;
}

sfft_status sfft_batch_destroy(sfft_batch_t b) {
  if (!b) return SFFT_OK;
  if (b->replay_recorded) (void)hipEventSynchronize(b->replayed);  // the last replay reads this memory
  if (b->replayed) (void)hipEventDestroy(b->replayed);
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->capture_stream) (void)hipStreamDestroy(b->capture_stream);
  if (b->d_mem) (void)hipFree(b->d_mem);
  delete b;
  return SFFT_OK;
}

}  // extern "C"
