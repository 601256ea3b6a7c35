// Host side of a plan: parameter rules, flat window, exact window spectrum,
// location schedule and per-iteration random draws (all FP64 / integer).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <iterator>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <tuple>

#include "internal.h"

namespace sfft {

namespace {

constexpr double kPi = 3.14159265358979323846;

bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }

int ilog2(uint64_t v) {
  int r = 0;
  while ((1ull << r) < v) ++r;
  return r;
}

// SplitMix64 (Steele, Lea, Flood 2014): state advances by the golden
// gamma; the output is the state passed through two multiply/xor-shift
// mixing rounds.
struct SplitMix64 {
  uint64_t s;
  uint64_t next() {
    s += 0x9E3779B97F4A7C15ull;
    uint64_t z = s;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  }
};

// Inverse of an odd number modulo 2^64 by Newton's iteration
// x <- x (2 - a x); each step doubles the number of correct low bits.
uint64_t odd_inverse(uint64_t a) {
  uint64_t x = a;  // correct to 3 bits: a * a = 1 mod 8 for odd a
  for (int i = 0; i < 6; ++i) x *= 2 - a * x;
  return x;
}

// erfc^{-1}(y) for 0 < y < 1 by Newton's method on erfc.
double erfc_inv(double y) {
  double z = std::sqrt(-std::log(y));
  for (int it = 0; it < 100; ++it) {
    double f = std::erfc(z) - y;
    double df = -2.0 / std::sqrt(kPi) * std::exp(-z * z);
    double step = f / df;
    z -= step;
    if (std::fabs(step) <= 1e-16 * std::fabs(z)) break;
  }
  return z;
}

// Flat window of Sec. 2.3: G_t = H_t g_t with H the inverse DFT (Eq. 2
// normalisation) of a width-L boxcar whose edge bins weigh 1/2,
// H_t = sin(pi L t / N) cot(pi t / N), H_0 = L, and g a Gaussian that has
// fallen to delta at |t| = h.
struct Window {
  double s_t, s_f, d_delta;
  std::vector<double> G;
};
Window make_window(int64_t N, int64_t L, int64_t h, double delta) {
  Window wd;
  wd.s_t = double(h) / std::sqrt(2.0 * std::log(1.0 / delta));
  wd.G.assign(h + 1, 0.0);
  wd.G[0] = double(L);
  for (int64_t t = 1; t <= h; ++t) {
    int64_t lt = (L * t) % (2 * N);                 // sin(pi L t / N), argument reduced exactly
    double s = std::sin(kPi * double(lt) / double(N));
    double a = kPi * double(t) / double(N);
    double g = std::exp(-double(t) * double(t) / (2.0 * wd.s_t * wd.s_t));
    wd.G[t] = s * (std::cos(a) / std::sin(a)) * g;
  }
  wd.s_f = double(N) / (2.0 * kPi * wd.s_t);
  wd.d_delta = std::sqrt(2.0) * wd.s_f * erfc_inv(2.0 * delta);
  return wd;
}

// Ghat_k = (1/N) (G_0 + 2 sum_{t=1..h} G_t cos(2 pi (k t mod N) / N)), the
// DFT of the real, even window, for k = 0..D.  The phase k t mod N is exact;
// cos(2 pi p / N) comes from two tables (high and low bits of p) joined by
// the angle-addition formula.  Work is split over k across host threads.
std::vector<double> make_spectrum(const std::vector<double>& G, int64_t N, int64_t D) {
  const int64_t h = int64_t(G.size()) - 1;
  const int n = ilog2(uint64_t(N));
  const int lo_bits = n / 2;
  const int64_t nlo = int64_t(1) << lo_bits, nhi = N >> lo_bits;
  std::vector<double> chi(nhi), shi(nhi), clo(nlo), slo(nlo);
  for (int64_t i = 0; i < nhi; ++i) {
    double a = 2.0 * kPi * double(i << lo_bits) / double(N);
    chi[i] = std::cos(a);
    shi[i] = std::sin(a);
  }
  for (int64_t i = 0; i < nlo; ++i) {
    double a = 2.0 * kPi * double(i) / double(N);
    clo[i] = std::cos(a);
    slo[i] = std::sin(a);
  }
  std::vector<double> Ghat(D + 1, 0.0);
  const uint64_t mask = uint64_t(N) - 1, lmask = uint64_t(nlo) - 1;
  auto work = [&](int64_t k0, int64_t k1) {
    for (int64_t k = k0; k < k1; ++k) {
      double acc = 0.0;
      uint64_t p = 0;
      for (int64_t t = 1; t <= h; ++t) {
        p = (p + uint64_t(k)) & mask;
        uint64_t hi = p >> lo_bits, lo = p & lmask;
        double c = chi[hi] * clo[lo] - shi[hi] * slo[lo];
        acc += G[t] * c;
      }
      Ghat[k] = (G[0] + 2.0 * acc) / double(N);
    }
  };
  int64_t cost = (D + 1) * h;
  unsigned nt = cost > (int64_t(1) << 22) ? std::max(1u, std::min(16u, std::thread::hardware_concurrency())) : 1u;
  if (nt == 1) {
    work(0, D + 1);
    return Ghat;
  }
  std::vector<std::thread> th;
  int64_t chunk = (D + 1 + nt - 1) / nt;
  for (unsigned i = 0; i < nt; ++i) {
    int64_t a = int64_t(i) * chunk, b = std::min<int64_t>(D + 1, a + chunk);
    if (a < b) th.emplace_back(work, a, b);
  }
  for (auto& t : th) t.join();
  return Ghat;
}

// The tables of the live plans, by (N, L, h, delta) for the window and
// (N, L, h, delta, D) for its spectrum: a plan holds its tables, and a later
// plan with the same values takes the same copy (tables of plans that are
// gone are computed again).  Two threads that miss on the same key at once
// both compute it; the first to insert wins.
struct TableKey {
  int64_t N, L, h, D;
  uint64_t delta_bits;
  bool operator<(const TableKey& o) const {
    return std::tie(N, L, h, D, delta_bits) < std::tie(o.N, o.L, o.h, o.D, o.delta_bits);
  }
};
struct WindowEntry {
  double s_t, s_f, d_delta;
  std::weak_ptr<const std::vector<double>> G;
};
std::mutex g_tables_mu;
std::map<TableKey, WindowEntry> g_windows;
std::map<TableKey, std::weak_ptr<const std::vector<double>>> g_spectra;

uint64_t bits_of(double v) {
  uint64_t b;
  std::memcpy(&b, &v, sizeof b);
  return b;
}

void window_tables(IterHost& it, int64_t N, double delta) {
  const TableKey key{N, int64_t(it.d.L), int64_t(it.d.h), -1, bits_of(delta)};
  {
    std::lock_guard<std::mutex> lk(g_tables_mu);
    auto hit = g_windows.find(key);
    if (hit != g_windows.end()) {
      if (auto G = hit->second.G.lock()) {
        it.s_t = hit->second.s_t;
        it.s_f = hit->second.s_f;
        it.d_delta = hit->second.d_delta;
        it.G = std::move(G);
        return;
      }
    }
  }
  Window wd = make_window(N, it.d.L, it.d.h, delta);
  auto G = std::make_shared<const std::vector<double>>(std::move(wd.G));
  std::lock_guard<std::mutex> lk(g_tables_mu);
  for (auto i = g_windows.begin(); i != g_windows.end();)  // entries of tables no plan holds
    i = i->second.G.expired() ? g_windows.erase(i) : std::next(i);
  WindowEntry& e = g_windows[key];
  if (auto live = e.G.lock()) {
    G = std::move(live);  // another thread inserted it first
  } else {
    e = WindowEntry{wd.s_t, wd.s_f, wd.d_delta, G};
  }
  it.s_t = e.s_t;
  it.s_f = e.s_f;
  it.d_delta = e.d_delta;
  it.G = std::move(G);
}

void spectrum_table(IterHost& it, int64_t N, double delta) {
  const TableKey key{N, int64_t(it.d.L), int64_t(it.d.h), int64_t(it.d.D), bits_of(delta)};
  {
    std::lock_guard<std::mutex> lk(g_tables_mu);
    auto hit = g_spectra.find(key);
    if (hit != g_spectra.end()) {
      if (auto S = hit->second.lock()) {
        it.Ghat = std::move(S);
        return;
      }
    }
  }
  auto S = std::make_shared<const std::vector<double>>(make_spectrum(*it.G, N, it.d.D));
  std::lock_guard<std::mutex> lk(g_tables_mu);
  for (auto i = g_spectra.begin(); i != g_spectra.end();)
    i = i->second.expired() ? g_spectra.erase(i) : std::next(i);
  auto& e = g_spectra[key];
  if (auto live = e.lock()) S = std::move(live);
  else e = S;
  it.Ghat = std::move(S);
}

}  // namespace

sfft_status build_host_plan(HostPlan& hp, int64_t N, int64_t K, int64_t B, int64_t w, int32_t loops,
                            int32_t l, double q, const sfft_options& opt, std::string* err) {
  auto bad = [&](sfft_status s, const std::string& m) {
    *err = m;
    return s;
  };
  if (!is_pow2(N) || N < 16 || N > (int64_t(1) << 30)) return bad(SFFT_ERR_PARAM, "N must be a power of two in [2^4, 2^30]");
  if (!is_pow2(B) || B < 16 || B > N / 4) return bad(SFFT_ERR_PARAM, "B must be a power of two with 16 <= B <= N/4");
  if (K < 1 || K > B) return bad(SFFT_ERR_PARAM, "K must satisfy 1 <= K <= B");
  if (w < B || w > N - 1) return bad(SFFT_ERR_PARAM, "w must satisfy B <= w <= N-1");
  if (loops < 1 || loops > kMaxLoops) return bad(SFFT_ERR_PARAM, "loops must be in [1, 64]");
  if (!is_pow2(l) || l < 2 || l > 1024) return bad(SFFT_ERR_PARAM, "multiscale l must be a power of two in [2, 1024]");
  if (!(q > 0.0) || !std::isfinite(q)) return bad(SFFT_ERR_PARAM, "extension q must be > 0");
  double qs = q * 65536.0;
  if (qs != std::floor(qs) || qs > 1e9) return bad(SFFT_ERR_PARAM, "extension q must be a dyadic rational (q * 2^16 integer)");
  if (!(double(l) > q + 1.0)) return bad(SFFT_ERR_PARAM, "the location region must shrink: need l > q + 1");
  if (!(opt.delta > 0.0 && opt.delta < 0.1)) return bad(SFFT_ERR_PARAM, "delta must be in (0, 0.1)");
  if (opt.dtype < 0 || opt.dtype > 2) return bad(SFFT_ERR_PARAM, "unknown dtype");
  if (!is_pow2(opt.b_min) || opt.b_min < 16 || opt.b_min > B) return bad(SFFT_ERR_PARAM, "b_min must be a power of two with 16 <= b_min <= B");
  if (!(opt.eta >= 0.0 && opt.eta < 1.0) || !(opt.rho > 0.0)) return bad(SFFT_ERR_PARAM, "need 0 <= eta < 1 and rho > 0");
  if (opt.location != SFFT_LOCATE_MULTISCALE && opt.location != SFFT_LOCATE_DIRECT)
    return bad(SFFT_ERR_PARAM, "unknown location method");
  const bool direct = opt.location == SFFT_LOCATE_DIRECT;
  if (opt.combine != SFFT_COMBINE_SUM && opt.combine != SFFT_COMBINE_VOTE)
    return bad(SFFT_ERR_PARAM, "unknown combine method");
  const bool vote = opt.combine == SFFT_COMBINE_VOTE;
  const int64_t bmax = opt.dtype == SFFT_C128 ? kMaxBucketsF64 : kMaxBucketsF32;
  if (B > bmax) return bad(SFFT_ERR_UNSUPPORTED, "B above the bucket-FFT limit of this dtype");

  // q = qn / qd with qd a power of two
  int64_t qd = 1, qn = 0;
  while (true) {
    double v = q * double(qd);
    if (v == std::floor(v)) {
      qn = int64_t(v);
      break;
    }
    qd *= 2;
  }
  if (w % 2 == 0) w += 1;

  hp.N = N; hp.K = K; hp.B = B; hp.w = w; hp.loops = loops; hp.l = l;
  hp.qn = qn; hp.qd = qd; hp.q = q; hp.delta = opt.delta; hp.eta = opt.eta; hp.rho = opt.rho;
  hp.seed = opt.seed; hp.dtype = opt.dtype; hp.kahan = opt.kahan ? 1 : 0; hp.b_min = opt.b_min;
  hp.flags = opt.flags;
  hp.iters.clear();
  hp.samples = 0;

  SplitMix64 rng{opt.seed};
  const uint32_t nmask = uint32_t(N - 1);
  uint64_t y_off = 0, win_off = 0, ghat_off = 0, tw_off = 0;
  for (int m = 0; m < loops; ++m) {
    if (alloc_should_fail()) throw std::bad_alloc();  // this iteration's host tables
    IterHost it{};
    IterDesc& d = it.d;
    // The vote keeps B and w in every loop; the iterative method halves B.
    int64_t Bm = vote ? B : std::max<int64_t>(B >> m, opt.b_min);
    int64_t Lm = N / Bm;
    int64_t wm = ((w * Bm) / B) | 1;
    d.B = uint32_t(Bm); d.logB = uint32_t(ilog2(Bm)); d.L = uint32_t(Lm); d.logL = uint32_t(ilog2(Lm));
    d.w = uint32_t(wm); d.h = uint32_t((wm - 1) / 2);
    window_tables(it, N, opt.delta);
    int64_t e = int64_t(std::ceil(it.d_delta));
    if (e > N / 2 - Lm) return bad(SFFT_ERR_PARAM, "window transition wider than the signal allows (w too small for B)");
    d.e = uint32_t(e);
    d.D = uint32_t(Lm / 2 + e);
    d.reach = uint32_t((2 * int64_t(d.D)) / Lm);
    d.log_B = std::log(double(Bm));

    // Location schedule (Sec. 3.2): extended first region, shrink by (1+q)/l.
    // The two-round location has a single step with tau = 1.
    it.kinds.assign(1, 0);
    int64_t len = Lm + 2 * e;
    int R = 0;
    d.tau[0] = 0; d.len[0] = 0;
    if (direct) {
      R = 1;
      d.len[1] = uint32_t(len);
      d.tau[1] = 1;
      it.kinds.push_back(2);
    }
    while (!direct) {
      ++R;
      if (R >= kMaxRounds) return bad(SFFT_ERR_UNSUPPORTED, "location needs more than 47 steps for these (l, q)");
      int64_t num = (qd + qn) * len, den = qd * int64_t(l);
      int64_t nxt = (num + den - 1) / den + 1;
      d.len[R] = uint32_t(len);
      d.tau[R] = uint32_t(N / len);
      if (len <= l || nxt >= len) {
        it.kinds.push_back(1);
        break;
      }
      it.kinds.push_back(0);
      len = nxt;
    }
    d.R = uint32_t(R);

    uint64_t sigma = 2 * (rng.next() % uint64_t(N / 2)) + 1;
    uint64_t tau0 = rng.next() % uint64_t(N);
    d.sigma = uint32_t(sigma);
    d.sigma_inv = uint32_t(odd_inverse(sigma) & nmask);
    d.tau0 = uint32_t(tau0);
    d.T[0] = uint32_t(tau0);
    for (int j = 1; j <= R; ++j) d.T[j] = uint32_t((tau0 + d.tau[j]) & nmask);

    spectrum_table(it, N, opt.delta);

    d.win_off = win_off;  win_off += d.h + 1;
    d.ghat_off = ghat_off; ghat_off += d.D + 1;
    d.tw_off = tw_off;    tw_off += Bm / 2;
    d.y_off = y_off;      y_off += uint64_t(R + 1) * uint64_t(Bm);
    hp.samples += int64_t(R + 1) * wm;
    hp.iters.push_back(std::move(it));
  }

  PlanDesc& pd = hp.desc;
  std::memset(&pd, 0, sizeof(pd));
  pd.location = opt.location;
  pd.combine = uint32_t(opt.combine);
  pd.N = uint32_t(N); pd.logN = uint32_t(ilog2(N)); pd.K = uint32_t(K); pd.M = uint32_t(loops);
  pd.l = uint32_t(l); pd.logl = uint32_t(ilog2(l));
  pd.qn = int32_t(qn); pd.logqd = uint32_t(ilog2(qd));
  pd.dtype = uint32_t(opt.dtype); pd.kahan = uint32_t(hp.kahan);
  uint64_t cap = 0, bm = 0;
  for (auto& it : hp.iters) {
    cap += it.d.B;
    bm = std::max<uint64_t>(bm, it.d.B);
  }
  pd.rec_cap = uint32_t(cap);
  pd.Bmax = uint32_t(bm);
  uint64_t sc = 1;
  while (sc < std::max(cap, bm)) sc <<= 1;
  pd.sort_cap = uint32_t(sc);
  pd.fp64_phase = N >= (int64_t(1) << 24) ? 1u : 0u;
  for (auto& it : hp.iters) {
    pd.Rmax = std::max(pd.Rmax, it.d.R);
    pd.max_slots = std::max(pd.max_slots, it.d.reach + 1);
  }
  pd.y_total = y_off;
  pd.eta = opt.eta;
  pd.rho = opt.rho;
  layout_workspace(hp);
  return SFFT_OK;
}

void layout_workspace(HostPlan& hp) {
  PlanDesc& pd = hp.desc;
  const uint64_t rs = hp.dtype == SFFT_C128 ? 8 : 4;  // real size
  uint64_t off = 0;
  auto take = [&](uint64_t bytes) {
    uint64_t o = off;
    off += (bytes + 255) & ~uint64_t(255);
    return o;
  };
  pd.off_y = take(pd.y_total * 2 * rs);
  pd.off_recf = take(uint64_t(pd.rec_cap) * 4);
  pd.off_recv = take(uint64_t(pd.rec_cap) * 2 * rs);
  pd.work_bytes = recover_work_bytes(pd, 2 * rs, rs);
  pd.off_work = take(pd.work_bytes);
  const bool vote = pd.combine == SFFT_COMBINE_VOTE;
  pd.off_nvote = take(vote ? uint64_t(pd.rec_cap) * 4 : 0);
  pd.off_votes = take(vote ? uint64_t(pd.rec_cap) * pd.M * 2 * rs : 0);
  pd.ws_bytes = off;
}

uint32_t union_rounds(const IterDesc& d, uint32_t N) {
  if (d.B < uint32_t(kFoldTile)) return 1;
  const uint64_t w = d.w;
  uint32_t nu = 1;
  uint64_t prev = 0;
  for (uint32_t j = 1; j <= d.R && nu < kMaxUnionRounds; ++j) {
    const uint64_t dj = (d.T[j] - d.T[0]) & (N - 1);
    if (dj < prev || dj - prev >= w || dj + w > N) break;
    prev = dj;
    ++nu;
  }
  return nu;
}

// Work lists of one signal, signal-major: the fold covers the (R_m+1) x B_m
// (round, bucket) items of every iteration in tiles of kFoldTile items.
// When B_m >= kFoldTile, the rounds whose windows overlap round 0's go into
// union tiles (union_rounds), which gather each sample once for all of them,
// and the tiles go out in chunks of 8 bucket blocks: for each round j, the
// blocks of round j that gather the same positions as the chunk's round-0
// blocks (bucket b + (T_j - T_0) mod B), so that tiles 8 dispatches apart
// (the same XCD) share the cache lines they gather.
void build_work_lists(const HostPlan& hp, uint32_t sig, std::vector<FoldTile>& tiles, std::vector<RoundItem>& items) {
  for (int m = 0; m < hp.loops; ++m) {
    const IterDesc& d = hp.iters[m].d;
    for (uint32_t j = 0; j <= d.R; ++j) items.push_back(RoundItem{sig, uint16_t(m), uint16_t(j)});
    if (d.B < uint32_t(kFoldTile)) {
      const uint32_t n = (d.R + 1) * d.B;
      for (uint32_t i0 = 0; i0 < n; i0 += kFoldTile) tiles.push_back(FoldTile{sig, uint32_t(m), i0});
      continue;
    }
    const uint32_t nu = union_rounds(d, uint32_t(hp.N));
    const uint32_t nb = d.B / kFoldTile;  // B and kFoldTile are powers of two
    for (uint32_t c0 = 0; c0 < nb; c0 += 8) {
      if (nu > 1)
        for (uint32_t blk = c0; blk < c0 + 8 && blk < nb; ++blk)
          tiles.push_back(FoldTile{sig, fold_tile_code(uint32_t(m), nu), blk * kFoldTile});
      for (uint32_t j = nu > 1 ? nu : 0; j <= d.R; ++j) {
        const uint32_t shift = ((d.T[j] - d.T[0]) & (d.B - 1)) / kFoldTile;  // B divides N and 2^32
        for (uint32_t blk = c0; blk < c0 + 8 && blk < nb; ++blk)
          tiles.push_back(FoldTile{sig, uint32_t(m), j * d.B + ((blk + shift) % nb) * kFoldTile});
      }
    }
  }
}

// Orders per-signal fold tiles for the stage launches: union tiles first, by
// round count, then the one-round tiles, each class in its original order.
FoldSplit order_for_stages(std::vector<FoldTile>& tiles) {
  auto cls = [](const FoldTile& t) {
    const uint32_t nu = fold_tile_rounds(t.m);
    return nu >= 2 ? nu - 2 : kMaxUnionRounds - 1;
  };
  std::stable_sort(tiles.begin(), tiles.end(), [&](const FoldTile& a, const FoldTile& b) { return cls(a) < cls(b); });
  FoldSplit sp;
  for (const FoldTile& t : tiles)
    if (cls(t) < kMaxUnionRounds - 1) ++sp.nunion[cls(t)];
  return sp;
}

// Position-major fold tiles (iteration, block of kIlvItems items, signal
// group), in an order that keeps a gathered row in the L2 of its XCD for the
// other rounds that need it: bucket b of round 0 and bucket
// b + (T_j - T_0) mod B of round j gather the same residue class of
// positions, over windows that overlap when tau_j < w, so the tiles of all
// rounds for a block of round-0 buckets go out together, signal groups
// innermost.  Workgroups go to the 8 XCDs in turn, so with 8 groups each
// group keeps to one XCD.  A fold workgroup that takes two or four adjacent
// groups (two or four signals per lane) covers fewer XCDs per tile, so runs
// of kBlockRun blocks interleave round by round: with 8 groups the
// workgroups of a block and group still meet the same XCD in every round.
// Every (round, bucket block, group) tile appears once.
void interleaved_tiles(const HostPlan& hp, uint32_t ngroups, std::vector<FoldTile>& tiles) {
  constexpr uint32_t kBlockRun = 4;
  for (int m = 0; m < hp.loops; ++m) {
    const IterDesc& d = hp.iters[m].d;
    const uint32_t nb = d.B / kIlvItems;  // B >= 16 = kIlvItems
    for (uint32_t blk0 = 0; blk0 < nb; blk0 += kBlockRun)
      for (uint32_t j = 0; j <= d.R; ++j) {
        const uint32_t shift = ((d.T[j] - d.T[0]) & (d.B - 1)) / kIlvItems;  // B divides N and 2^32
        for (uint32_t blk = blk0; blk < std::min(blk0 + kBlockRun, nb); ++blk) {
          const uint32_t i0 = j * d.B + ((blk + shift) % nb) * kIlvItems;
          for (uint32_t g = 0; g < ngroups; ++g) tiles.push_back(FoldTile{g, uint32_t(m), i0});
        }
      }
  }
}

}  // namespace sfft
