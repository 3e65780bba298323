// Host side of libfdet: argument checking, workspace layout, work-item plans
// and kernel launches behind the C ABI declared in include/fdet.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <mutex>
#include <queue>
#include <unordered_map>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/fdet.h"
#include "fdet_hmc.h"
#include "fdet_plan.h"

#define FDET_DECLARE_CLASS(NC)                                                          \
  extern "C" hipError_t fdet_launch_items_##NC(int kind, const fdet::Prob* probs,        \
                                               const fdet::Item* items, int nitems,      \
                                               hipStream_t st);
#define FDET_DECLARE_PERSIST(NC)                                                         \
  extern "C" hipError_t fdet_launch_persist_##NC(                                        \
      const fdet::Prob* probs, const fdet::Item* items, int nitems, const int32_t* deps,  \
      uint32_t* done, fdet::Sched* sched, uint64_t spin_ticks, int grid, hipStream_t st); \
  extern "C" int fdet_persist_blocks_per_cu_##NC(void);
FDET_DECLARE_CLASS(32)
FDET_DECLARE_CLASS(64)
FDET_DECLARE_CLASS(80)
FDET_DECLARE_CLASS(96)
FDET_DECLARE_CLASS(128)
FDET_DECLARE_CLASS(512)
FDET_DECLARE_PERSIST(32)
FDET_DECLARE_PERSIST(64)
FDET_DECLARE_PERSIST(80)
FDET_DECLARE_PERSIST(96)
FDET_DECLARE_PERSIST(128)
FDET_DECLARE_PERSIST(512)
#undef FDET_DECLARE_CLASS
#undef FDET_DECLARE_PERSIST
extern "C" hipError_t fdet_launch_init_status(const fdet::Prob* probs, int nprob, fdet::Sched* sched,
                                              hipStream_t st);
extern "C" hipError_t fdet_launch_hmc(int op, const fdet::HmcProb* hp, int nprob, int64_t maxn,
                                      double* pi, const double* force, const double* logdet,
                                      double dU, double h, double* H0, double* dH,
                                      const int32_t* st_step, int32_t* st_acc, int mode,
                                      hipStream_t st);
extern "C" hipError_t fdet_launch_diag_response(int Nt, int N, const double* fre, const double* fim,
                                                const double* a, double* out, hipStream_t st);
extern "C" hipError_t fdet_launch_trace(int N, const double* G, const double* A, double* part,
                                        double* out, hipStream_t st);

namespace {

using fdet::Item;
using fdet::Prob;
using fdet::Udv;

// Launch of one phase in the size class of its largest problem (each class
// is a separate kernel object; items smaller than the class run their own
// class's code inside it).
hipError_t fdet_launch_items(int maxn, int kind, const Prob* probs, const Item* items, int nitems,
                             hipStream_t st) {
  if (nitems <= 0) return hipSuccess;
  if (maxn <= 32) return fdet_launch_items_32(kind, probs, items, nitems, st);
  if (maxn <= 64) return fdet_launch_items_64(kind, probs, items, nitems, st);
  if (maxn <= 80) return fdet_launch_items_80(kind, probs, items, nitems, st);
  if (maxn <= 96) return fdet_launch_items_96(kind, probs, items, nitems, st);
  if (maxn <= 128) return fdet_launch_items_128(kind, probs, items, nitems, st);
  return fdet_launch_items_512(kind, probs, items, nitems, st);
}

hipError_t fdet_launch_persist(int maxn, const Prob* probs, const Item* items, int nitems,
                               const int32_t* deps, uint32_t* done, fdet::Sched* sched,
                               uint64_t spin_ticks, int grid, hipStream_t st) {
  if (maxn <= 32) return fdet_launch_persist_32(probs, items, nitems, deps, done, sched, spin_ticks, grid, st);
  if (maxn <= 64) return fdet_launch_persist_64(probs, items, nitems, deps, done, sched, spin_ticks, grid, st);
  if (maxn <= 80) return fdet_launch_persist_80(probs, items, nitems, deps, done, sched, spin_ticks, grid, st);
  if (maxn <= 96) return fdet_launch_persist_96(probs, items, nitems, deps, done, sched, spin_ticks, grid, st);
  if (maxn <= 128) return fdet_launch_persist_128(probs, items, nitems, deps, done, sched, spin_ticks, grid, st);
  return fdet_launch_persist_512(probs, items, nitems, deps, done, sched, spin_ticks, grid, st);
}

int persist_blocks_per_cu(int maxn) {
  if (maxn <= 32) return fdet_persist_blocks_per_cu_32();
  if (maxn <= 64) return fdet_persist_blocks_per_cu_64();
  if (maxn <= 80) return fdet_persist_blocks_per_cu_80();
  if (maxn <= 96) return fdet_persist_blocks_per_cu_96();
  if (maxn <= 128) return fdet_persist_blocks_per_cu_128();
  return fdet_persist_blocks_per_cu_512();
}

thread_local std::string g_last_error;

// Phase timing with HIP events (diagnostics; off unless fd_profile_start).
struct PhaseRec {
  int kind;
  int nitems;
  hipEvent_t a, b;
};
thread_local bool g_prof_on = false;
thread_local std::vector<PhaseRec> g_prof;

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }
int pad16(int n) { return (n + 15) / 16 * 16; }
size_t cmat_bytes(int Np) { return (size_t)2 * Np * Np * sizeof(double); }
size_t udv_bytes(int Np) { return align_up(2 * cmat_bytes(Np) + (size_t)Np * sizeof(double)); }
// 4 complex matrices, 2 Np doubles, and the T factors of the 16-column
// panels of a blocked QR (Np / 16 panels of 2 x 16 x 16 doubles)
size_t scratch_bytes(int Np) {
  return align_up(4 * cmat_bytes(Np) + (size_t)2 * Np * sizeof(double) +
                  (size_t)(Np / 16) * 512 * sizeof(double));
}

struct Opts {
  int s, c, segments, flags;
};

// ---- tuned choices of (s, segments), keyed by the shape of a call
struct TuneKey {
  int what, maxN, maxNt, nprob;
  long long dk_micro;
  bool operator==(const TuneKey& o) const {
    return what == o.what && maxN == o.maxN && maxNt == o.maxNt && nprob == o.nprob &&
           dk_micro == o.dk_micro;
  }
};
struct TuneVal {
  int s, segments;
  float ms;
};
std::mutex g_tune_mu;
std::vector<std::pair<TuneKey, TuneVal>> g_tune;

TuneKey tune_key(const fd_problem* p, int nprob, int what) {
  TuneKey k{what, 0, 0, nprob, 0};
  for (int i = 0; i < nprob; ++i) {
    k.maxN = std::max(k.maxN, p[i].N);
    k.maxNt = std::max(k.maxNt, p[i].Nt);
  }
  k.dk_micro = std::llround(p[0].dk * 1e6);
  return k;
}

bool tune_lookup(const TuneKey& k, TuneVal& v) {
  std::lock_guard<std::mutex> g(g_tune_mu);
  for (auto& e : g_tune)
    if (e.first == k) { v = e.second; return true; }
  return false;
}

void tune_store(const TuneKey& k, const TuneVal& v) {
  std::lock_guard<std::mutex> g(g_tune_mu);
  for (auto& e : g_tune)
    if (e.first == k) { e.second = v; return; }
  g_tune.push_back({k, v});
}

int pow2_floor(int x) {
  int r = 1;
  while (2 * r <= x) r *= 2;
  return r;
}

// Segments of a single problem when neither the caller nor the tuner chose:
// a chain segment of about 8 slices per QR interval balances chain and
// combine latency.
int default_segments(const fd_problem* p, int nprob) {
  int maxNt = 1;
  for (int i = 0; i < nprob; ++i) maxNt = std::max(maxNt, p[i].Nt);
  return std::min(32, pow2_floor(std::max(1, maxNt / 8)));
}

int device_cu_count() {
  int dev = 0, n = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n < 1)
    return 256;
  return n;
}

// Chain work of one problem in arbitrary units: a slice costs about
// max(N, 32)^2 on one workgroup (latency-bound below N = 128).
double chain_cost(const fd_problem& p) {
  const double m = std::max(p.N, 32);
  return m * m * (double)p.Nt;
}

// Options of one call: explicit fields win, then a tuned entry for this
// shape, then the defaults (s = 8, c = 16, default_segments).
Opts resolve(const fd_options* o, const fd_problem* p = nullptr, int nprob = 0, int what = -1) {
  Opts r{0, 16, 0, 0};
  if (o) {
    if (o->s > 0) r.s = o->s;
    if (o->checkpoint > 0) r.c = o->checkpoint;
    if (o->segments > 0) r.segments = o->segments;
    r.flags = o->flags;
  }
  if (p && nprob > 0 && (r.s == 0 || r.segments == 0)) {
    TuneVal v;
    if (tune_lookup(tune_key(p, nprob, what), v)) {
      if (r.s == 0) r.s = v.s;
      if (r.segments == 0) r.segments = v.segments;
    }
    if (r.segments == 0 && nprob == 1) r.segments = default_segments(p, nprob);
  }
  if (r.s == 0) r.s = 8;
  return r;
}

// Time segments of every problem (det / G / UDV).  Explicit or tuned: the
// same count for all.  Automatic for a batch: each problem gets segments in
// proportion to its chain work, so that the chains of the whole batch fill
// the compute units about once and no long problem is left running alone.
std::vector<int> plan_segments(const fd_problem* p, int nprob, const Opts& o) {
  std::vector<int> seg(nprob, 1);
  if (o.segments > 0) {
    for (int i = 0; i < nprob; ++i) seg[i] = std::max(1, std::min(o.segments, p[i].Nt));
    return seg;
  }
  double total = 0.0;
  for (int i = 0; i < nprob; ++i) total += chain_cost(p[i]);
  const double target = total / device_cu_count();
  for (int i = 0; i < nprob; ++i) {
    const int cap = std::max(1, std::min(32, p[i].Nt / 4));
    const int want = (int)std::ceil(chain_cost(p[i]) / target - 1e-9);
    seg[i] = std::max(1, std::min(cap, want));
  }
  return seg;
}

// Offsets are computed against `base`; with base == nullptr only sizes matter.
struct Plan {
  size_t item_cap = 0;   // items the descriptor region was sized for
  std::vector<Prob> probs;
  std::vector<std::vector<Item>> phases;
  size_t desc_bytes = 0;
  size_t total = 0;
  int maxN = 0;
  std::vector<int> units;   // per problem: time segments (det / G) or checkpoint intervals (force)
  // single launch (unless FD_PHASE_LAUNCHES): every item in one list, each
  // after the items it depends on, and the dependency lists; the tail of the
  // workspace holds the dependency array, the completion flags and Sched
  bool single = false;
  int grid = 0;                 // workgroups of the single launch
  std::vector<Item> order;      // items in claim order
  double est_us = 0.0;          // simulated run time of the single launch
  std::vector<int32_t> deps;
  size_t tail_off = 0, tail_bytes = 0, deps_off = 0, done_off = 0, sched_off = 0;
  // matrix-free slices (intermediate-volume variant): one descriptor per
  // problem at sops_off inside the descriptor region
  std::vector<fdet::SparseOp> sops;
  size_t sops_off = 0;
};

struct Cursor {
  char* base;
  size_t off;
  double* take(size_t bytes) {
    double* p = base ? reinterpret_cast<double*>(base + off) : nullptr;
    off += align_up(bytes);
    return p;
  }
};

Udv make_udv(double* p, int Np) {
  Udv u;
  u.X = p;
  u.T = p ? p + (size_t)2 * Np * Np : nullptr;
  u.D = p ? p + (size_t)4 * Np * Np : nullptr;
  return u;
}

Item blank_item(int kind, int prob) {
  Item it;
  std::memset(&it, 0, sizeof(it));
  it.kind = kind;
  it.prob = prob;
  it.sign = 1;
  return it;
}

// gamma_1 .. gamma_n with prod_k (1 + gamma_k x) = sum_{j <= n} x^j / j!
// (Sec. 8): gamma_k = -1 / r_k for the roots r_k of the Taylor polynomial.
// The roots of its monic form x^n + sum_j (n! / j!) x^j come from the
// Weierstrass (Durand-Kerner) iteration, each polished by Newton steps on the
// polynomial, in long double; ordered by real part, then imaginary part.
std::vector<std::complex<double>> taylor_product_coefficients(int n) {
  typedef std::complex<long double> C;
  std::vector<long double> a(n + 1);   // monic: a[j] multiplies x^j, a[n] = 1
  long double f = 1.0L;
  for (int j = n; j >= 0; --j) {
    a[j] = f;                          // n! / j!
    f *= (long double)std::max(j, 1);
  }
  auto poly = [&](C x, C* dp) {
    C v = a[n], d = 0.0L;
    for (int j = n - 1; j >= 0; --j) {
      d = d * x + v;
      v = v * x + a[j];
    }
    if (dp) *dp = d;
    return v;
  };
  std::vector<C> r(n);
  const C seed(0.4L, 0.9L);
  C z = 1.0L;
  for (int k = 0; k < n; ++k) {
    z *= seed;
    r[k] = (long double)n * z;
  }
  for (int it = 0; it < 500; ++it) {
    long double moved = 0.0L;
    for (int k = 0; k < n; ++k) {
      C den = 1.0L;
      for (int j = 0; j < n; ++j)
        if (j != k) den *= r[k] - r[j];
      const C step = poly(r[k], nullptr) / den;
      r[k] -= step;
      moved = std::max(moved, std::abs(step));
    }
    if (moved < 1e-18L) break;
  }
  for (int k = 0; k < n; ++k)
    for (int it = 0; it < 3; ++it) {
      C d;
      const C v = poly(r[k], &d);
      if (std::abs(d) > 0.0L) r[k] -= v / d;
    }
  std::vector<std::complex<double>> g(n);
  for (int k = 0; k < n; ++k) {
    const C gk = -1.0L / r[k];
    g[k] = std::complex<double>((double)gk.real(), (double)gk.imag());
  }
  std::sort(g.begin(), g.end(), [](const std::complex<double>& x, const std::complex<double>& y) {
    return x.real() < y.real() || (x.real() == y.real() && x.imag() < y.imag());
  });
  return g;
}

int validate(const fd_problem* p, int nprob, const Opts& o) {
  if (!p || nprob < 1) return fail(FD_ERR_INVALID_ARG, "no problems given");
  if (o.flags & FD_SINGLE_LAUNCH)
    return fail(FD_ERR_UNSUPPORTED,
                "FD_SINGLE_LAUNCH is switched off: one run of it (twelve N = 18 force problems "
                "with grouped scans) did not finish and its cause is not known");
  if (o.s < 1) return fail(FD_ERR_INVALID_ARG, "s must be >= 1");
  if (o.c < 1 || o.c > 64) return fail(FD_ERR_INVALID_ARG, "checkpoint interval must be in [1, 64]");
  for (int i = 0; i < nprob; ++i) {
    const fd_problem& q = p[i];
    char buf[160];
    if (q.N < 1 || q.N > FD_MAX_N) {
      std::snprintf(buf, sizeof buf, "problem %d: N = %d outside [1, %d]", i, q.N, FD_MAX_N);
      return fail(FD_ERR_INVALID_ARG, buf);
    }
    if (q.Nt < 1) {
      std::snprintf(buf, sizeof buf, "problem %d: Nt = %d must be >= 1", i, q.Nt);
      return fail(FD_ERR_INVALID_ARG, buf);
    }
    if (!std::isfinite(q.dk)) {
      std::snprintf(buf, sizeof buf, "problem %d: dk is not finite", i);
      return fail(FD_ERR_NONFINITE, buf);
    }
    if (!q.K || !q.phi) {
      std::snprintf(buf, sizeof buf, "problem %d: K and phi must be device pointers", i);
      return fail(FD_ERR_INVALID_ARG, buf);
    }
  }
  return FD_OK;
}

// ---- inclusive scans of stabilised products for the force checkpoints
//
// Sequence x_0 .. x_{n-1}; entry i is P_i = x_i o ... o x_0 where `later_left`
// puts higher indices on the left (prefix Q_k = L_k ... L_0) or on the right
// (suffix S_k = L_{n-1} ... L_k, run over i = n-1-k).  Groups of g entries:
// a sequential scan inside each group (g - 1 levels), a Hillis-Steele scan
// of the group totals (log2(n/g) levels, two buffers), then one product per
// entry with the total of all earlier groups (one level).  g = 1 is a plain
// Hillis-Steele scan (depth log2 n, n log2 n products); larger g does about
// 2n products for a few more levels, which wins once a batch fills the GPU.
//
// Slots: [0, n) the inputs x_i, [n, 2n) entry buffers, [2n, 2n+G) and
// [2n+G, 2n+2G) the two group-total buffers.
struct ScanOp {
  int level, left, right, out, scr;
};

struct ScanPlan {
  std::vector<ScanOp> ops;
  std::vector<int> final_slot;   // slot holding P_i at the end
  int levels = 0;
  bool uses_entries = false;
};

ScanPlan scan_schedule(int n, int g, bool later_left) {
  ScanPlan sp;
  const int G = (n + g - 1) / g;
  std::vector<int> loc(n);
  for (int i = 0; i < n; ++i) loc[i] = i;
  auto push = [&](int level, int later, int earlier, int out, int scr) {
    ScanOp op;
    op.level = level;
    op.left = later_left ? later : earlier;
    op.right = later_left ? earlier : later;
    op.out = out;
    op.scr = scr;
    sp.ops.push_back(op);
    sp.levels = std::max(sp.levels, level + 1);
  };
  int level = 0;
  // phase 1: inside each group
  for (int l = 1; l < g; ++l, ++level) {
    for (int b = 0; b < G; ++b) {
      const int i = b * g + l;
      if (i >= std::min(n, (b + 1) * g)) continue;
      push(level, loc[i], loc[i - 1], n + i, i);
      loc[i] = n + i;
      sp.uses_entries = true;
    }
  }
  // phase 2: group totals
  std::vector<int> last(G), hloc(G), hbuf(G, -1);
  for (int b = 0; b < G; ++b) {
    last[b] = std::min(n, (b + 1) * g) - 1;
    hloc[b] = loc[last[b]];
  }
  for (int d = 1; d < G; d *= 2, ++level) {
    std::vector<int> nloc = hloc, nbuf = hbuf;
    for (int b = d; b < G; ++b) {
      nbuf[b] = hbuf[b] == 0 ? 1 : 0;
      nloc[b] = 2 * n + nbuf[b] * G + b;
      push(level, hloc[b], hloc[b - d], nloc[b], last[b]);
    }
    hloc = nloc;
    hbuf = nbuf;
  }
  // phase 3: earlier groups' total into every entry but each group's last
  bool any = false;
  for (int b = 1; b < G; ++b) {
    for (int i = b * g; i < last[b]; ++i) {
      push(level, loc[i], hloc[b - 1], n + i, i);
      loc[i] = n + i;
      any = true;
      sp.uses_entries = true;
    }
  }
  if (any) ++level;
  for (int b = 0; b < G; ++b) loc[last[b]] = hloc[b];
  sp.final_slot = loc;
  return sp;
}

// ---- cyclic windows of interval products for the force checkpoints
//
// W(i, len) = L_{i+len-1} ... L_i, indices mod nc.  The cyclic product that
// checkpoint k needs, L_{k-1} ... L_0 L_{nc-1} ... L_k, splits into a left
// window W(k - P, P) and a right window W(k, nc - P) for any P; with P the
// smallest power of two such that 2 P >= nc, all nc left windows come from
// log2(P) doubling levels W(i, 2p) = W(i + p, p) W(i, p), nc products each,
// and the right windows (length nc - P <= P) are built from the same powers
// within those levels: a window of length p + r (p a power of two, r < p)
// is W(i + r, p) W(i, r).  Against the prefix / suffix scans this takes
// log2(P) launches instead of about 2 log2(nc), which matters while a plan
// leaves compute units idle.
struct WinBuild {
  int len, level, left, right;   // W(i, len) = W(i + right, left) W(i, right)
};

struct WinPlan {
  int P = 1, w2 = 0, levels = 0;
  std::vector<WinBuild> builds;   // in level order
};

WinPlan window_plan(int nc) {
  WinPlan wp;
  while (2 * wp.P < nc) wp.P *= 2;
  wp.w2 = nc - wp.P;
  std::vector<int> avail(nc + 1, -1);   // launches before W(., len) exists
  avail[1] = 0;
  for (int p = 2; p <= wp.P; p *= 2) {
    wp.builds.push_back({p, avail[p / 2], p / 2, p / 2});
    avail[p] = avail[p / 2] + 1;
  }
  // the right windows: lengths w2, then its remainders, built bottom-up
  std::vector<int> chain;
  for (int len = wp.w2; len > 1 && avail[len] < 0; len -= pow2_floor(len)) chain.push_back(len);
  for (int c = (int)chain.size() - 1; c >= 0; --c) {
    const int len = chain[c], p = pow2_floor(len), r = len - p;
    const int lv = std::max(avail[p], avail[r]);
    wp.builds.push_back({len, lv, p, r});
    avail[len] = lv + 1;
  }
  for (const WinBuild& b : wp.builds) wp.levels = std::max(wp.levels, b.level + 1);
  std::stable_sort(wp.builds.begin(), wp.builds.end(),
                   [](const WinBuild& x, const WinBuild& y) { return x.level < y.level; });
  return wp;
}

// Schedule of the checkpoint products: windows (g == 0) or scans with group
// size g.  The candidate whose combine levels take the fewest rounds of one
// workgroup per compute unit over the whole plan wins; on ties the windows,
// then the smallest group.  A lone problem gets the windows; a batch that
// fills the GPU many times over gets grouped scans (about 2 nc products per
// direction instead of nc log2(nc) / 2 per window level).
int force_schedule(const fd_problem* p, int nprob, const Opts& o) {
  const int ncu = device_cu_count();
  auto rounds_of = [&](const std::vector<long long>& per_level) {
    long long r = 0;
    for (long long n : per_level) r += (n + ncu - 1) / ncu;
    return r;
  };
  std::vector<long long> win;
  for (int i = 0; i < nprob; ++i) {
    const int nc = (p[i].Nt + o.c - 1) / o.c;
    const WinPlan wp = window_plan(nc);
    if ((int)win.size() < wp.levels) win.resize(wp.levels, 0);
    for (const WinBuild& b : wp.builds) win[b.level] += nc;
  }
  int best_g = 0;
  long long best_rounds = (o.flags & FD_FORCE_SCANS) ? -1 : rounds_of(win);
  for (int g : {1, 2, 4, 8, 16}) {
    std::vector<long long> per_level;
    for (int i = 0; i < nprob; ++i) {
      const int nc = (p[i].Nt + o.c - 1) / o.c;
      const ScanPlan sp = scan_schedule(nc, g, true);
      if ((int)per_level.size() < sp.levels) per_level.resize(sp.levels, 0);
      for (const ScanOp& op : sp.ops) per_level[op.level] += 2;   // both directions
    }
    const long long rounds = rounds_of(per_level);
    if (best_rounds < 0 || rounds < best_rounds) {
      best_rounds = rounds;
      best_g = g;
    }
  }
  return best_g;
}

// ---- single launch: dependencies and claim order
//
// Estimated run time of one item on one workgroup (microseconds): its model
// FLOP at a per-workgroup rate that grows with N (the small classes are
// latency-bound), plus a fixed cost per item.  Only the relative sizes
// matter: they order the simulated schedule below.
double item_cost(const Prob& P, const Item& it) {
  const double n = P.N, n3 = n * n * n;
  const double rate = 160e3 * n / (n + 100.0);   // FLOP per microsecond
  double units = 1.0;
  switch (it.kind) {
    case fdet::IK_EXPM: units = 16.0; break;
    case fdet::IK_CHAIN: {
      const int r = it.t1 - it.t0;
      units = 4.0 * r + 14.67 * ((r + std::max(1, it.s) - 1) / std::max(1, it.s));
      break;
    }
    case fdet::IK_COMBINE: units = 30.67; break;
    case fdet::IK_CLOSE: units = (it.flags & fdet::IF_WANT_G) ? 33.3 : 13.3; break;
    case fdet::IK_FORCE: units = 64.0 + 8.0 * (std::max(0, it.t1 - it.t0 - 1) + it.nb); break;
    default: break;
  }
  return 20.0 + units * n3 / rate;
}

// Workspace regions an item reads and writes, keyed by their first address:
// UDV slots (by X), scratch areas, E and E^-1.  Outputs in caller memory are
// written by one item each (disjoint force rows) and need no ordering.
struct Access {
  const void* key;
  bool write;
};

void item_access(const Prob& P, const Item& it, std::vector<Access>& acc) {
  acc.clear();
  auto rd = [&](const void* k) { if (k) acc.push_back({k, false}); };
  auto wr = [&](const void* k) { if (k) acc.push_back({k, true}); };
  wr(it.scr);
  switch (it.kind) {
    case fdet::IK_EXPM: wr(it.sign > 0 ? P.E : P.Einv); break;
    case fdet::IK_CHAIN:
      rd(P.E);
      wr(it.a.X);
      break;
    case fdet::IK_COMBINE:
      rd(it.a.X);
      rd(it.b.X);
      wr(it.o.X ? it.o.X : it.a.X);
      break;
    case fdet::IK_CLOSE: wr(it.a.X); break;   // its T serves as free storage
    case fdet::IK_FORCE:
      rd(it.a.X);
      rd(it.b.X);
      rd(P.E);
      rd(P.Einv);
      break;
    case fdet::IK_EXPORT: rd(it.a.X); break;
    default: break;
  }
}

// Items of all phases in one list for the single launch: the dependencies of
// each item follow from the regions it shares with earlier items in phase
// order (read after write, write after write, write after read), and the
// list order is that of a simulated list schedule on `workers` workgroups
// that starts the ready item with the longest remaining path first (HLFET).
// Every item then comes after the items it depends on, so claiming items in
// list order cannot wait forever; deps are rewritten to list positions.
void single_launch_order(Plan& pl, int workers) {
  std::vector<Item> items;
  for (auto& ph : pl.phases) items.insert(items.end(), ph.begin(), ph.end());
  const int n = (int)items.size();
  struct RegionState {
    int writer = -1;
    std::vector<int> readers;
  };
  std::unordered_map<const void*, RegionState> reg;
  std::vector<std::vector<int>> pred(n), succ(n);
  std::vector<Access> acc;
  for (int i = 0; i < n; ++i) {
    item_access(pl.probs[items[i].prob], items[i], acc);
    std::vector<int>& d = pred[i];
    for (const Access& a : acc) {
      RegionState& r = reg[a.key];
      if (r.writer >= 0) d.push_back(r.writer);
      bool written = false;
      for (const Access& b : acc) written = written || (b.key == a.key && b.write);
      if (written) d.insert(d.end(), r.readers.begin(), r.readers.end());
    }
    std::sort(d.begin(), d.end());
    d.erase(std::unique(d.begin(), d.end()), d.end());
    for (const Access& a : acc) {
      RegionState& r = reg[a.key];
      bool written = false;
      for (const Access& b : acc) written = written || (b.key == a.key && b.write);
      if (written) {
        r.writer = i;
        r.readers.clear();
      } else if (r.readers.empty() || r.readers.back() != i) {
        r.readers.push_back(i);
      }
    }
    for (int q : d) succ[q].push_back(i);
  }
  // longest remaining path (bottom level), items in reverse phase order
  std::vector<double> cost(n), bl(n);
  for (int i = 0; i < n; ++i) cost[i] = item_cost(pl.probs[items[i].prob], items[i]);
  for (int i = n - 1; i >= 0; --i) {
    double m = 0.0;
    for (int q : succ[i]) m = std::max(m, bl[q]);
    bl[i] = cost[i] + m;
  }
  // list-schedule simulation
  std::vector<int> indeg(n);
  for (int i = 0; i < n; ++i) indeg[i] = (int)pred[i].size();
  auto lower = [&](int a, int b) { return bl[a] < bl[b] || (bl[a] == bl[b] && a > b); };
  std::priority_queue<int, std::vector<int>, decltype(lower)> ready(lower);
  for (int i = 0; i < n; ++i)
    if (indeg[i] == 0) ready.push(i);
  typedef std::pair<double, int> Ev;
  std::priority_queue<Ev, std::vector<Ev>, std::greater<Ev>> running;
  std::vector<int> seq;
  seq.reserve(n);
  double now = 0.0;
  int idle = std::max(1, workers);
  while ((int)seq.size() < n) {
    while (idle > 0 && !ready.empty()) {
      const int i = ready.top();
      ready.pop();
      seq.push_back(i);
      running.push({now + cost[i], i});
      --idle;
    }
    if (running.empty()) break;   // unreachable: the dependency graph is acyclic
    now = running.top().first;
    while (!running.empty() && running.top().first <= now) {
      const int i = running.top().second;
      running.pop();
      ++idle;
      for (int q : succ[i])
        if (--indeg[q] == 0) ready.push(q);
    }
  }
  if ((int)seq.size() != n) {
    std::fprintf(stderr, "libfdet: dependency graph of %d items is not acyclic\n", n);
    std::abort();
  }
  pl.est_us = now;
  std::vector<int> pos(n);
  for (int k = 0; k < n; ++k) pos[seq[k]] = k;
  pl.order.resize(n);
  pl.deps.clear();
  for (int k = 0; k < n; ++k) {
    Item it = items[seq[k]];
    it.dep0 = (int32_t)pl.deps.size();
    it.ndep = (int32_t)pred[seq[k]].size();
    for (int q : pred[seq[k]]) pl.deps.push_back(pos[q]);
    pl.order[k] = it;
  }
}

// Build the layout and the work items.  `what` = FD_WHAT_*.
void build_plan(const fd_problem* p, int nprob, const Opts& o, int what, char* base, Plan& pl,
                const fd_ell* ell = nullptr, int taylor_n = 0) {
  pl.probs.assign(nprob, Prob{});
  pl.maxN = 0;
  size_t nitems = 0;
  // count items to size the descriptor region.  With FD_KEEP_CHECKPOINTS
  // every call uses the force layout: log det / G run its first phases and
  // leave the checkpoint products in the workspace, the force then runs only
  // the checkpoint items on them.
  const bool keep = (o.flags & FD_KEEP_CHECKPOINTS) != 0;
  const bool force = what == FD_WHAT_FORCE || keep;
  std::vector<int> nseg = plan_segments(p, nprob, o), nck(nprob);
  const int sgroup = force ? force_schedule(p, nprob, o) : 1;
  pl.units.assign(nprob, 0);
  int maxlev = 0;
  size_t nforce = 0;
  for (int i = 0; i < nprob; ++i) {
    pl.maxN = std::max(pl.maxN, p[i].N);
    if (force) {
      const int nc = (p[i].Nt + o.c - 1) / o.c;
      nck[i] = nc;
      size_t prods = 0;
      if (sgroup == 0) {
        const WinPlan wp = window_plan(nc);
        prods = wp.builds.size() * (size_t)nc;
        maxlev = std::max(maxlev, wp.levels);
      } else {
        const ScanPlan sp = scan_schedule(nc, sgroup, true);
        prods = 2 * sp.ops.size();
        maxlev = std::max(maxlev, sp.levels);
      }
      // 2 exponentials, nc interval chains + the identity, the checkpoint
      // products, and 2 nc force items at most (forward / backward halves)
      nitems += 2 + (size_t)nc + 1 + prods + 2 * (size_t)nc;
      nforce += nc;
      pl.units[i] = nc;
    } else {
      int lev = 0;
      while ((1 << lev) < nseg[i]) ++lev;
      maxlev = std::max(maxlev, lev);
      nitems += 1 + nseg[i] + nseg[i] + 1;
      pl.units[i] = nseg[i];
    }
  }
  pl.desc_bytes = align_up(sizeof(Prob) * nprob) + align_up(sizeof(Item) * nitems);
  pl.sops.clear();
  if (ell) {
    pl.sops_off = pl.desc_bytes;
    pl.desc_bytes += align_up(sizeof(fdet::SparseOp) * nprob);
  }
  pl.item_cap = nitems;
  // a sizing pass (base == nullptr) lays out against a stand-in address: the
  // single launch's dependencies are keyed by region addresses, so they must
  // be distinct there too (the pointers of a sizing plan are never used)
  Cursor cur{base ? base : reinterpret_cast<char*>((uintptr_t)1 << 40), align_up(pl.desc_bytes)};
  if (ell) {
    const std::vector<std::complex<double>> gam = taylor_product_coefficients(taylor_n);
    for (int i = 0; i < nprob; ++i) {
      fdet::SparseOp so;
      std::memset(&so, 0, sizeof so);
      so.n = taylor_n;
      so.q = ell[i].q;
      so.col = ell[i].col;
      so.val = ell[i].val;
      for (int k = 0; k < taylor_n; ++k) {
        so.gr[k] = gam[k].real() * p[i].dk;
        so.gi[k] = gam[k].imag() * p[i].dk;
      }
      pl.sops.push_back(so);
    }
  }

  std::vector<Item> expm, chain, close, forcei;
  std::vector<std::vector<Item>> comb(maxlev);
  for (int i = 0; i < nprob; ++i) {
    const fd_problem& q = p[i];
    Prob& P = pl.probs[i];
    P.N = q.N;
    P.Np = pad16(q.N);
    P.Nt = q.Nt;
    P.dk = q.dk;
    P.K = q.K;
    P.phi = q.phi;
    if (ell)
      P.sp = reinterpret_cast<const fdet::SparseOp*>(cur.base + pl.sops_off) + i;
    const int Np = P.Np;
    P.E = cur.take((size_t)Np * Np * sizeof(double));
    P.Einv = force ? cur.take((size_t)Np * Np * sizeof(double)) : nullptr;
    if (!force) {
      const int ns = nseg[i];
      std::vector<Udv> slot(ns);
      std::vector<double*> scr(ns);
      for (int k = 0; k < ns; ++k) {
        slot[k] = make_udv(cur.take(udv_bytes(Np)), Np);
        scr[k] = cur.take(scratch_bytes(Np));
      }
      if (!(o.flags & FD_REUSE_E) && !ell) {
        Item e = blank_item(fdet::IK_EXPM, i);
        e.sign = 1;
        e.scr = scr[0];
        expm.push_back(e);
      }
      for (int k = 0; k < ns; ++k) {
        Item c = blank_item(fdet::IK_CHAIN, i);
        c.t0 = (int)((long long)q.Nt * k / ns);
        c.t1 = (int)((long long)q.Nt * (k + 1) / ns);
        c.s = o.s;
        c.flags = fdet::IF_IDENTITY;
        c.a = slot[k];
        c.scr = scr[k];
        chain.push_back(c);
      }
      // pairwise tree: level l combines slot k+2^l (later) into slot k
      for (int l = 0; (1 << l) < ns; ++l) {
        for (int k = 0; k + (1 << l) < ns; k += 2 << l) {
          Item c = blank_item(fdet::IK_COMBINE, i);
          c.a = slot[k];
          c.b = slot[k + (1 << l)];
          c.scr = scr[k];
          comb[l].push_back(c);
        }
      }
      Item z = blank_item(what == FD_WHAT_UDV ? fdet::IK_EXPORT : fdet::IK_CLOSE, i);
      z.a = slot[0];
      z.scr = scr[0];
      if (what == FD_WHAT_GREENS) z.flags = fdet::IF_WANT_G;
      close.push_back(z);
    } else {
      // Checkpoint intervals [k c, (k+1) c): local products L_k in parallel,
      // then the two factors of every checkpoint's cyclic product
      // C_k = L_{k-1} ... L_0 L_{nc-1} ... L_k, both in the X D T form with
      // the unitary factor on the left, from either
      //   windows (sgroup == 0): C_k = W(k - P, P) W(k, nc - P), or
      //   scans: the prefix Q_{k-1} = L_{k-1} ... L_0 (the identity for
      //   k = 0) and the suffix S_k = L_{nc-1} ... L_k.
      // C_0 is the whole product: checkpoint 0 also gives log det M and G.
      const int nc = nck[i];
      const size_t ub = udv_bytes(Np);
      std::vector<Udv> base(nc);
      for (int k = 0; k < nc; ++k) base[k] = make_udv(cur.take(ub), Np);
      const Udv ident = make_udv(cur.take(ub), Np);
      std::vector<double*> sf(nc), sb(nc);
      for (int k = 0; k < nc; ++k) {
        sf[k] = cur.take(scratch_bytes(Np));
        sb[k] = cur.take(scratch_bytes(Np));
      }
      if (!(o.flags & FD_REUSE_E)) {
        for (int sg = 0; sg < 2; ++sg) {
          Item e = blank_item(fdet::IK_EXPM, i);
          e.sign = sg == 0 ? 1 : -1;
          e.scr = sg == 0 ? sf[0] : sb[0];
          expm.push_back(e);
        }
      }
      for (int k = 0; k < nc; ++k) {
        Item c = blank_item(fdet::IK_CHAIN, i);
        c.t0 = k * o.c;
        c.t1 = std::min(q.Nt, (k + 1) * o.c);
        c.s = o.s;
        c.flags = fdet::IF_IDENTITY;
        c.a = base[k];
        c.scr = sf[k];
        chain.push_back(c);
      }
      {
        // empty range: the identity (writes no scratch, so sb[0] is shared)
        Item c = blank_item(fdet::IK_CHAIN, i);
        c.s = o.s;
        c.flags = fdet::IF_IDENTITY;
        c.a = ident;
        c.scr = sb[0];
        chain.push_back(c);
      }
      std::vector<Udv> left(nc), right(nc);
      if (sgroup == 0) {
        // windows: slots per length, length 1 being the intervals
        const WinPlan wp = window_plan(nc);
        std::vector<std::vector<Udv>> win(nc + 1);
        win[1] = base;
        std::vector<int> used(wp.levels, 0);   // builds placed per level
        for (const WinBuild& bd : wp.builds) {
          win[bd.len].resize(nc);
          for (int k = 0; k < nc; ++k) win[bd.len][k] = make_udv(cur.take(ub), Np);
          const std::vector<double*>& sc = used[bd.level]++ == 0 ? sf : sb;
          for (int k = 0; k < nc; ++k) {
            Item c = blank_item(fdet::IK_COMBINE, i);
            c.b = win[bd.left][(k + bd.right) % nc];
            c.a = win[bd.right][k];
            c.o = win[bd.len][k];
            c.scr = sc[k];
            comb[bd.level].push_back(c);
          }
        }
        for (int k = 0; k < nc; ++k) {
          left[k] = win[wp.P][((k - wp.P) % nc + nc) % nc];
          right[k] = wp.w2 > 0 ? win[wp.w2][k] : ident;
        }
      } else {
        // scans (see scan_schedule); the inputs are shared by both
        const ScanPlan spf = scan_schedule(nc, sgroup, true);
        const ScanPlan spb = scan_schedule(nc, sgroup, false);
        const int G = (nc + sgroup - 1) / sgroup;
        std::vector<Udv> slf(2 * nc + 2 * G), slb(2 * nc + 2 * G);
        for (int dir = 0; dir < 2; ++dir) {
          std::vector<Udv>& sl = dir == 0 ? slf : slb;
          // prefix sequence index i is interval i; suffix index i is nc-1-i
          for (int i2 = 0; i2 < nc; ++i2) sl[i2] = base[dir == 0 ? i2 : nc - 1 - i2];
          if (spf.uses_entries)
            for (int i2 = 0; i2 < nc; ++i2) sl[nc + i2] = make_udv(cur.take(ub), Np);
          for (int b = 0; b < 2 * G; ++b) sl[2 * nc + b] = make_udv(cur.take(ub), Np);
        }
        for (int dir = 0; dir < 2; ++dir) {
          const ScanPlan& sp = dir == 0 ? spf : spb;
          const std::vector<Udv>& sl = dir == 0 ? slf : slb;
          const std::vector<double*>& sc = dir == 0 ? sf : sb;
          for (const ScanOp& op : sp.ops) {
            Item c = blank_item(fdet::IK_COMBINE, i);
            c.b = sl[op.left];
            c.a = sl[op.right];
            c.o = sl[op.out];
            c.scr = sc[op.scr];
            comb[op.level].push_back(c);
          }
        }
        // Q_{k-1}: prefix entry k-1; S_k: suffix entry nc-1-k
        for (int k = 0; k < nc; ++k) {
          left[k] = k == 0 ? ident : slf[spf.final_slot[k - 1]];
          right[k] = slb[spb.final_slot[nc - 1 - k]];
        }
      }
      // checkpoint k (row k*c) carries G~ forward over the first half of the
      // gap to the next checkpoint and backward over the second half of the
      // gap from the previous one (cyclically for k = 0), so no G~ is carried
      // across more than about c/2 slices.  While the plan leaves compute
      // units idle, the two directions are separate items (the checkpoint's
      // G~ is then formed twice, the carries run side by side).
      const bool split = 2 * nforce <= (size_t)device_cu_count();
      const int last_gap = q.Nt - (nc - 1) * o.c;
      if (keep && what != FD_WHAT_FORCE) {
        // log det (and G) of the whole product C_0 = M - 1: checkpoint 0's
        // item without carried rows
        Item f = blank_item(fdet::IK_FORCE, i);
        f.a = left[0];
        f.b = right[0];
        f.scr = sf[0];
        f.flags = fdet::IF_OUT_LOGDET | (what == FD_WHAT_GREENS ? fdet::IF_OUT_G : 0);
        forcei.push_back(f);
        continue;
      }
      for (int k = 0; k < nc; ++k) {
        Item f = blank_item(fdet::IK_FORCE, i);
        const int gap_fwd = (k + 1 < nc) ? o.c : last_gap;
        const int gap_bwd = (k > 0) ? o.c : last_gap;
        f.t0 = k * o.c;
        f.t1 = f.t0 + (gap_fwd + 1) / 2;
        f.nb = (nc == 1) ? q.Nt - (q.Nt + 1) / 2 : gap_bwd / 2;
        f.a = left[k];
        f.b = right[k];
        f.scr = sf[k];
        if (k == 0) f.flags = fdet::IF_OUT_LOGDET | fdet::IF_OUT_G;
        if (split && f.nb > 0) {
          Item g = f;
          g.flags = 0;
          g.t1 = g.t0;   // no forward rows
          g.scr = sb[k];
          f.nb = 0;
          forcei.push_back(g);
        }
        forcei.push_back(f);
      }
    }
  }
  // longest work per workgroup first: the dispatcher hands out workgroups in
  // order, so the batch's long chains start first (longest-processing-time)
  auto work = [&](const Item& it) {
    const double m = std::max(pl.probs[it.prob].N, 32);
    return m * m * (double)(it.t1 - it.t0);
  };
  std::stable_sort(chain.begin(), chain.end(),
                   [&](const Item& a, const Item& b) { return work(a) > work(b); });
  pl.phases.clear();
  if (keep && what == FD_WHAT_FORCE) {
    // the checkpoint products are in the workspace from the log det call
    pl.phases.push_back(forcei);
  } else {
    if (!expm.empty()) pl.phases.push_back(expm);
    pl.phases.push_back(chain);
    for (auto& c : comb)
      if (!c.empty()) pl.phases.push_back(c);
    if (!close.empty()) pl.phases.push_back(close);
    if (!forcei.empty()) pl.phases.push_back(forcei);
  }
  size_t n = 0;
  for (auto& ph : pl.phases) n += ph.size();
  if (n > pl.item_cap) {   // the counting pass above must cover every item
    std::fprintf(stderr, "libfdet: %zu work items exceed the %zu counted\n", n, pl.item_cap);
    std::abort();
  }
  pl.single = (o.flags & FD_SINGLE_LAUNCH) != 0;
  if (pl.single) {
    const int workers = device_cu_count() * persist_blocks_per_cu(pl.maxN);
    pl.grid = (int)std::min<size_t>(n, (size_t)workers);
    single_launch_order(pl, workers);
  }
  // tail: dependency lists, completion flags, launch state
  pl.tail_off = cur.off;
  pl.deps_off = cur.off;
  cur.take(sizeof(int32_t) * std::max<size_t>(1, pl.deps.size()));
  pl.done_off = cur.off;
  cur.take(sizeof(uint32_t) * std::max<size_t>(1, pl.item_cap));   // the same for every phase subset
  pl.sched_off = cur.off;
  cur.take(sizeof(fdet::Sched));
  pl.tail_bytes = cur.off - pl.tail_off;
  pl.total = cur.off;
}

// ---- time-displaced Green's functions G(t, t0) of one problem
//
// Per pair (t, t0): P = the slices from row t-1 up to row t0-1 (cyclically;
// all N_t slices when t = t0) and Q = the others from row t0-1 on, as in
// eq. sausage_all_in_denominator; G(t, t0) = sign (P + Q^{-1})^{-1}, sign -1
// for t < t0.  Phases: exp(+-dk K); for every pair a chain of P's slices and
// a chain of Q^{-H}'s slices exp(-dk K) diag(e^{i phi_t}) (same rows, same
// order); one IK_DISPLACED item per pair.
void displaced_rows(int Nt, int t, int t0, int& ps, int& pl, int& qs, int& ql, int& sign) {
  const int r = t - 1, r0 = t0 - 1;
  pl = ((r0 - r) % Nt + Nt) % Nt;
  if (pl == 0) pl = Nt;
  ps = r;
  qs = r0;
  ql = Nt - pl;
  sign = t < t0 ? -1 : 1;
}

void build_displaced_plan(const fd_problem* p, const Opts& o, int npairs, const int32_t* th,
                          const int32_t* t0h, char* base, Plan& pl, double* Gout) {
  pl.probs.assign(1, Prob{});
  pl.units.assign(1, npairs);
  pl.maxN = p->N;
  const size_t nitems = 2 + 3 * (size_t)npairs;
  pl.desc_bytes = align_up(sizeof(Prob)) + align_up(sizeof(Item) * nitems);
  pl.item_cap = nitems;
  Cursor cur{base ? base : reinterpret_cast<char*>((uintptr_t)1 << 40), align_up(pl.desc_bytes)};
  Prob& P = pl.probs[0];
  P.N = p->N;
  P.Np = pad16(p->N);
  P.Nt = p->Nt;
  P.dk = p->dk;
  P.K = p->K;
  P.phi = p->phi;
  const int Np = P.Np;
  P.E = cur.take((size_t)Np * Np * sizeof(double));
  P.Einv = cur.take((size_t)Np * Np * sizeof(double));
  std::vector<Item> expm, chain, disp;
  for (int k = 0; k < npairs; ++k) {
    const Udv sp = make_udv(cur.take(udv_bytes(Np)), Np);
    const Udv sq = make_udv(cur.take(udv_bytes(Np)), Np);
    double* scp = cur.take(scratch_bytes(Np));
    double* scq = cur.take(scratch_bytes(Np));
    if (k == 0) {
      for (int sg = 0; sg < 2; ++sg) {
        Item e = blank_item(fdet::IK_EXPM, 0);
        e.sign = sg == 0 ? 1 : -1;
        e.scr = sg == 0 ? scp : scq;
        expm.push_back(e);
      }
    }
    int ps, pln, qs, qln, sign;
    displaced_rows(p->Nt, th[k], t0h[k], ps, pln, qs, qln, sign);
    Item a = blank_item(fdet::IK_CHAIN, 0);
    a.t0 = ps;
    a.t1 = ps + pln;
    a.s = o.s;
    a.flags = fdet::IF_IDENTITY;
    a.a = sp;
    a.scr = scp;
    chain.push_back(a);
    Item b = blank_item(fdet::IK_CHAIN, 0);
    b.t0 = qs;
    b.t1 = qs + qln;
    b.s = o.s;
    b.flags = fdet::IF_IDENTITY | fdet::IF_EINV;
    b.a = sq;
    b.scr = scq;
    chain.push_back(b);
    Item d = blank_item(fdet::IK_DISPLACED, 0);
    d.a = sp;
    d.b = sq;
    d.sign = sign;
    d.scr = scp;
    d.out = Gout ? Gout + (size_t)2 * p->N * p->N * k : nullptr;
    disp.push_back(d);
  }
  auto work = [&](const Item& it) { return it.t1 - it.t0; };
  std::stable_sort(chain.begin(), chain.end(),
                   [&](const Item& x, const Item& y) { return work(x) > work(y); });
  pl.phases.clear();
  if (!(o.flags & FD_REUSE_E)) pl.phases.push_back(expm);
  pl.phases.push_back(chain);
  pl.phases.push_back(disp);
  pl.single = false;
  pl.tail_off = pl.deps_off = cur.off;
  cur.take(sizeof(int32_t));
  pl.done_off = cur.off;
  cur.take(sizeof(uint32_t) * nitems);
  pl.sched_off = cur.off;
  cur.take(sizeof(fdet::Sched));
  pl.tail_bytes = cur.off - pl.tail_off;
  pl.total = cur.off;
}

int validate_pairs(const fd_problem* p, int32_t npairs, const int32_t* t, const int32_t* t0) {
  if (npairs < 1) return fail(FD_ERR_INVALID_ARG, "npairs must be >= 1");
  if (!t || !t0) return fail(FD_ERR_INVALID_ARG, "t and t0 must be host arrays");
  for (int k = 0; k < npairs; ++k)
    if (t[k] < 1 || t[k] > p->Nt || t0[k] < 1 || t0[k] > p->Nt) {
      char buf[128];
      std::snprintf(buf, sizeof buf, "pair %d: (t, t0) = (%d, %d) outside [1, %d]", k, t[k], t0[k], p->Nt);
      return fail(FD_ERR_INVALID_ARG, buf);
    }
  return FD_OK;
}

// Descriptors (problems, then the items of every phase, or the single
// launch's item list) in the head of the workspace; `first` receives the
// index of each phase's first item.  `tail` receives the single launch's
// dependency lists, zeroed completion flags and launch state, which go to
// pl.tail_off.
std::vector<char> pack_descriptors(const Plan& pl, std::vector<size_t>& first,
                                   std::vector<char>* tail = nullptr) {
  std::vector<char> host(pl.desc_bytes, 0);
  const size_t pbytes = align_up(sizeof(Prob) * pl.probs.size());
  std::memcpy(host.data(), pl.probs.data(), sizeof(Prob) * pl.probs.size());
  first.clear();
  size_t n = 0;
  if (pl.single) {
    std::memcpy(host.data() + pbytes, pl.order.data(), pl.order.size() * sizeof(Item));
  } else {
    for (auto& ph : pl.phases) {
      first.push_back(n);
      std::memcpy(host.data() + pbytes + n * sizeof(Item), ph.data(), ph.size() * sizeof(Item));
      n += ph.size();
    }
  }
  if (!pl.sops.empty())
    std::memcpy(host.data() + pl.sops_off, pl.sops.data(), pl.sops.size() * sizeof(fdet::SparseOp));
  if (tail) {
    tail->assign(pl.tail_bytes, 0);
    if (!pl.deps.empty())
      std::memcpy(tail->data() + (pl.deps_off - pl.tail_off), pl.deps.data(),
                  pl.deps.size() * sizeof(int32_t));
  }
  return host;
}

// Time limit of one wait of the single launch, in ticks of the device's
// constant-rate clock: 20 times the simulated run time of the whole call,
// at least 20 s.  It only guards against a wait that cannot end; the plan
// checker shows on the host that every item waits for earlier items only.
uint64_t spin_limit_ticks(double est_us) {
  int dev = 0, khz = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0)
    khz = 100000;
  const double sec = std::max(20.0, 20.0 * est_us * 1e-6);
  return (uint64_t)(sec * 1000.0 * khz);
}

// Kernel launches only (no copies or fills): the part a HIP graph captures.
int launch_phases(const Plan& pl, const std::vector<size_t>& first, char* ws, hipStream_t st) {
  const size_t pbytes = align_up(sizeof(Prob) * pl.probs.size());
  const Prob* dprobs = reinterpret_cast<const Prob*>(ws);
  const Item* ditems = reinterpret_cast<const Item*>(ws + pbytes);
  fdet::Sched* sched = pl.single ? reinterpret_cast<fdet::Sched*>(ws + pl.sched_off) : nullptr;
  hipError_t e = fdet_launch_init_status(dprobs, (int)pl.probs.size(), sched, st);
  if (e != hipSuccess) return fail(FD_ERR_HIP, std::string("launch: ") + hipGetErrorString(e));
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  const bool prof = g_prof_on && hipStreamIsCapturing(st, &cap) == hipSuccess &&
                    cap == hipStreamCaptureStatusNone;
  auto bracket = [&](int kind, int nitems, auto&& launch) -> int {
    PhaseRec rec{kind, nitems, nullptr, nullptr};
    if (prof) {
      if (hipEventCreate(&rec.a) != hipSuccess || hipEventCreate(&rec.b) != hipSuccess)
        return fail(FD_ERR_HIP, "event creation failed");
      hipEventRecord(rec.a, st);
    }
    const hipError_t r = launch();
    if (r != hipSuccess) return fail(FD_ERR_HIP, std::string("launch: ") + hipGetErrorString(r));
    if (prof) {
      hipEventRecord(rec.b, st);
      g_prof.push_back(rec);
    }
    return FD_OK;
  };
  if (pl.single) {
    const int n = (int)pl.order.size();
    return bracket(-1, n, [&]() {
      return fdet_launch_persist(pl.maxN, dprobs, ditems, n,
                                 reinterpret_cast<const int32_t*>(ws + pl.deps_off),
                                 reinterpret_cast<uint32_t*>(ws + pl.done_off), sched,
                                 spin_limit_ticks(pl.est_us), pl.grid, st);
    });
  }
  for (size_t k = 0; k < pl.phases.size(); ++k) {
    const int kind = pl.phases[k].front().kind;
    const int rc = bracket(kind, (int)pl.phases[k].size(), [&]() {
      return fdet_launch_items(pl.maxN, kind, dprobs, ditems + first[k], (int)pl.phases[k].size(), st);
    });
    if (rc != FD_OK) return rc;
  }
  return FD_OK;
}

// Upload the descriptors (and the single launch's tail) into the workspace.
int upload(const Plan& pl, std::vector<size_t>& first, char* ws, hipStream_t st) {
  std::vector<char> tail;
  std::vector<char> host = pack_descriptors(pl, first, &tail);
  hipError_t e = hipMemcpyAsync(ws, host.data(), pl.desc_bytes, hipMemcpyHostToDevice, st);
  if (e == hipSuccess && pl.single)
    e = hipMemcpyAsync(ws + pl.tail_off, tail.data(), tail.size(), hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return fail(FD_ERR_HIP, std::string("descriptor upload: ") + hipGetErrorString(e));
  return FD_OK;
}

// Upload descriptors into the head of the workspace and launch every phase.
int execute(Plan& pl, char* ws, hipStream_t st) {
  std::vector<size_t> first;
  const int rc = upload(pl, first, ws, st);
  if (rc != FD_OK) return rc;
  return launch_phases(pl, first, ws, st);
}

int check_ws(void* ws, size_t ws_bytes, size_t need) {
  if (!ws) return fail(FD_ERR_WORKSPACE, "workspace pointer is NULL");
  if (reinterpret_cast<uintptr_t>(ws) % kAlign)
    return fail(FD_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  if (ws_bytes < need) {
    char buf[128];
    std::snprintf(buf, sizeof buf, "workspace too small: %zu bytes given, %zu needed", ws_bytes, need);
    return fail(FD_ERR_WORKSPACE, buf);
  }
  return FD_OK;
}

// Common driver of every entry point.
struct Outs {
  double* logdet = nullptr;
  double* G = nullptr;
  double* force = nullptr;
  double* force_im = nullptr;
  double* E = nullptr;
  double* X = nullptr;
  double* D = nullptr;
  double* T = nullptr;
  const double* op = nullptr;
  double* op_trace = nullptr;
  int32_t* status = nullptr;
};

// Validate, lay out the workspace and attach the outputs.
int prepare(const fd_problem* p, int nprob, const fd_options* opt, int what, const Outs& out,
            void* ws, size_t ws_bytes, Plan& pl) {
  if (!p || nprob < 1) return fail(FD_ERR_INVALID_ARG, "no problems given");
  const Opts o = resolve(opt, p, nprob, what);
  int rc = validate(p, nprob, o);
  if (rc != FD_OK) return rc;
  Plan sizing;
  build_plan(p, nprob, o, what, nullptr, sizing);
  rc = check_ws(ws, ws_bytes, sizing.total);
  if (rc != FD_OK) return rc;
  build_plan(p, nprob, o, what, static_cast<char*>(ws), pl);
  size_t goff = 0, foff = 0, toff = 0;
  for (int i = 0; i < nprob; ++i) {
    Prob& P = pl.probs[i];
    P.status = out.status ? out.status + i : nullptr;
    P.logdet = out.logdet ? out.logdet + 2 * i : nullptr;
    P.G = out.G ? out.G + goff : nullptr;
    P.force = out.force ? out.force + foff : nullptr;
    P.force_im = out.force_im ? out.force_im + foff : nullptr;
    P.outE = out.E;
    P.outX = out.X;
    P.outD = out.D;
    P.outT = out.T;
    P.op = out.op ? out.op + goff : nullptr;
    P.op_trace = out.op_trace ? out.op_trace + 2 * toff : nullptr;
    toff += (size_t)p[i].Nt;
    goff += (size_t)2 * p[i].N * p[i].N;
    foff += (size_t)p[i].Nt * p[i].N;
  }
  return FD_OK;
}

int run(const fd_problem* p, int nprob, const fd_options* opt, int what, const Outs& out, void* ws,
        size_t ws_bytes, void* stream) {
  Plan pl;
  int rc = prepare(p, nprob, opt, what, out, ws, ws_bytes, pl);
  if (rc != FD_OK) return rc;
  return execute(pl, static_cast<char*>(ws), static_cast<hipStream_t>(stream));
}

// Gershgorin bound on the spectral radius of a real symmetric K (host copy).
double radius_bound(const std::vector<double>& K, int N) {
  double r = 0.0;
  for (int i = 0; i < N; ++i) {
    double s = 0.0;
    for (int j = 0; j < N; ++j) s += std::fabs(K[(size_t)i * N + j]);
    r = std::max(r, s);
  }
  return r;
}

}  // namespace

// A prepared call whose descriptors stay resident in its workspace.
struct fd_plan {
  Plan pl;
  std::vector<size_t> first;
  char* ws = nullptr;
};

namespace {

// Workspace of fd_hmc_leapfrog: the force plan's, then the force (sum N_t N
// doubles), log det (2 per field), H at the start (1 per field), the status
// of one force evaluation (1 int32 per field) and the field descriptors.
struct HmcLayout {
  size_t force_ws, f, ld, h0, st, hp, total;
  int64_t ntot, maxn;
};

HmcLayout hmc_layout(const fd_problem* p, int nprob, size_t force_ws) {
  HmcLayout L{};
  L.force_ws = align_up(force_ws);
  for (int i = 0; i < nprob; ++i) {
    const int64_t n = (int64_t)p[i].Nt * p[i].N;
    L.ntot += n;
    L.maxn = std::max(L.maxn, n);
  }
  L.f = L.force_ws;
  L.ld = L.f + align_up((size_t)L.ntot * sizeof(double));
  L.h0 = L.ld + align_up((size_t)2 * nprob * sizeof(double));
  L.st = L.h0 + align_up((size_t)nprob * sizeof(double));
  L.hp = L.st + align_up((size_t)nprob * sizeof(int32_t));
  L.total = L.hp + align_up((size_t)nprob * sizeof(fdet::HmcProb));
  return L;
}

// A leapfrog trajectory's fixed arguments and its part of the workspace.
struct HmcState {
  fdet::HmcProb* hp = nullptr;
  int nprob = 0;
  int64_t maxn = 0;
  double dU = 0.0, eps = 0.0;
  int nsteps = 0;
  double *pi = nullptr, *dH = nullptr, *F = nullptr, *ld = nullptr, *H0 = nullptr;
  int32_t *sstep = nullptr, *status = nullptr;
  size_t force_ws = 0;   // bytes at the head of the workspace for the force plan
};

// Checks the arguments of fd_hmc_leapfrog / fd_hmc_plan_create, carves the
// workspace (hmc_layout) and uploads the field descriptors (synchronously).
// o1: the force options with FD_REUSE_E cleared.
int hmc_setup(const fd_problem* p, int32_t nprob, const fd_options* o, double dU, double eps,
              int32_t nsteps, double* pi, double* dH, void* ws, size_t ws_bytes, int32_t* status,
              void* stream, fd_options& o1, HmcState& S) {
  if (!pi || !dH || !status) return fail(FD_ERR_INVALID_ARG, "pi, dH and status must be device pointers");
  if (!(dU > 0.0) || !std::isfinite(dU)) return fail(FD_ERR_INVALID_ARG, "dU must be positive and finite");
  if (!std::isfinite(eps)) return fail(FD_ERR_INVALID_ARG, "eps must be finite");
  if (nsteps < 1) return fail(FD_ERR_INVALID_ARG, "nsteps must be >= 1");
  if (!p || nprob < 1) return fail(FD_ERR_INVALID_ARG, "no problems given");
  if (nprob > 65535) return fail(FD_ERR_INVALID_ARG, "at most 65535 fields per call");
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(st, &cap) != hipSuccess || cap != hipStreamCaptureStatusNone)
    return fail(FD_ERR_INVALID_ARG, "trajectories prepare plans: call outside stream capture");
  o1 = fd_options{0, 0, 0, 0};
  if (o) o1 = *o;
  o1.flags &= ~FD_REUSE_E;
  const size_t fw = fd_workspace_bytes(p, nprob, &o1, FD_WHAT_FORCE);
  if (fw == 0) return FD_ERR_INVALID_ARG;
  const HmcLayout L = hmc_layout(p, nprob, fw);
  int rc = check_ws(ws, ws_bytes, L.total);
  if (rc != FD_OK) return rc;
  char* base = static_cast<char*>(ws);
  S.force_ws = fw;
  S.F = reinterpret_cast<double*>(base + L.f);
  S.ld = reinterpret_cast<double*>(base + L.ld);
  S.H0 = reinterpret_cast<double*>(base + L.h0);
  S.sstep = reinterpret_cast<int32_t*>(base + L.st);
  S.hp = reinterpret_cast<fdet::HmcProb*>(base + L.hp);
  S.nprob = nprob;
  S.maxn = L.maxn;
  S.dU = dU;
  S.eps = eps;
  S.nsteps = nsteps;
  S.pi = pi;
  S.dH = dH;
  S.status = status;
  std::vector<fdet::HmcProb> hh(nprob);
  int64_t off = 0;
  for (int i = 0; i < nprob; ++i) {
    hh[i].phi = const_cast<double*>(p[i].phi);
    hh[i].off = off;
    hh[i].n = (int64_t)p[i].Nt * p[i].N;
    off += hh[i].n;
  }
  hipError_t e = hipMemcpyAsync(S.hp, hh.data(), sizeof(fdet::HmcProb) * nprob,
                                hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return fail(FD_ERR_HIP, std::string("descriptor upload: ") + hipGetErrorString(e));
  return FD_OK;
}

// Enqueues one trajectory: half kick, nsteps x (drift, force, kick), the
// last kick a half one, with H before and after.  force(n) enqueues force
// evaluation n (0 at the start field) into S.F, S.ld and S.sstep.
template <class Force>
int hmc_enqueue(const HmcState& S, hipStream_t st, Force&& force) {
  auto md = [&](int op, double step, int mode) -> int {
    const hipError_t r = fdet_launch_hmc(op, S.hp, S.nprob, S.maxn, S.pi, S.F, S.ld, S.dU, step,
                                         S.H0, S.dH, S.sstep, S.status, mode, st);
    return r == hipSuccess ? FD_OK : fail(FD_ERR_HIP, std::string("launch: ") + hipGetErrorString(r));
  };
  int rc = force(0);
  if (rc == FD_OK) rc = md(3, 0.0, 0);           // status of this force evaluation
  if (rc == FD_OK) rc = md(2, 0.0, 0);           // H at the start
  if (rc == FD_OK) rc = md(0, 0.5 * S.eps, 0);   // half kick
  for (int n = 0; n < S.nsteps && rc == FD_OK; ++n) {
    rc = md(1, S.eps, 0);                         // drift
    if (rc == FD_OK) rc = force(n + 1);
    if (rc == FD_OK) rc = md(3, 0.0, 1);
    if (rc == FD_OK) rc = md(0, n + 1 < S.nsteps ? S.eps : 0.5 * S.eps, 0);
  }
  if (rc == FD_OK) rc = md(2, 0.0, 1);           // dH = H at the end - H at the start
  return rc;
}

}  // namespace

extern "C" {

size_t fd_workspace_bytes(const fd_problem* p, int32_t nprob, const fd_options* o, int32_t what) {
  if (what == FD_WHAT_HMC) {
    const size_t fw = fd_workspace_bytes(p, nprob, o, FD_WHAT_FORCE);
    return fw ? hmc_layout(p, nprob, fw).total : 0;
  }
  if (what < FD_WHAT_LOGDET || what > FD_WHAT_UDV) {
    fail(FD_ERR_INVALID_ARG, "unknown workspace kind");
    return 0;
  }
  if (!p || nprob < 1) {
    fail(FD_ERR_INVALID_ARG, "no problems given");
    return 0;
  }
  const Opts r = resolve(o, p, nprob, what);
  if (validate(p, nprob, r) != FD_OK) return 0;
  Plan pl;
  build_plan(p, nprob, r, what, nullptr, pl);
  return pl.total;
}

int fd_slice_exponential(const fd_problem* p, double* E, void* ws, size_t ws_bytes, void* stream) {
  if (!E) return fail(FD_ERR_INVALID_ARG, "E must be a device pointer");
  fd_options o{0, 0, 1, 0};
  const Opts r = resolve(&o);
  int rc = validate(p, 1, r);
  if (rc != FD_OK) return rc;
  Plan sizing;
  build_plan(p, 1, r, FD_WHAT_LOGDET, nullptr, sizing);
  rc = check_ws(ws, ws_bytes, sizing.total);
  if (rc != FD_OK) return rc;
  Plan pl;
  build_plan(p, 1, r, FD_WHAT_LOGDET, static_cast<char*>(ws), pl);
  pl.probs[0].outE = E;
  // only the exponential phase, as one launch of its own
  std::vector<Item> keep = pl.phases.front();
  pl.phases.assign(1, keep);
  pl.single = false;
  return execute(pl, static_cast<char*>(ws), static_cast<hipStream_t>(stream));
}

int fd_logdet(const fd_problem* p, const fd_options* o, double* logdet, void* ws, size_t ws_bytes,
              int32_t* status, void* stream) {
  return fd_logdet_batched(p, 1, o, logdet, ws, ws_bytes, status, stream);
}

int fd_greens(const fd_problem* p, const fd_options* o, double* logdet, double* G, void* ws,
              size_t ws_bytes, int32_t* status, void* stream) {
  return fd_greens_batched(p, 1, o, logdet, G, ws, ws_bytes, status, stream);
}

int fd_force(const fd_problem* p, const fd_options* o, double* logdet, double* force,
             double* force_im, void* ws, size_t ws_bytes, int32_t* status, void* stream) {
  return fd_force_batched(p, 1, o, logdet, force, force_im, ws, ws_bytes, status, stream);
}

int fd_udv(const fd_problem* p, const fd_options* o, double* X, double* D, double* T, void* ws,
           size_t ws_bytes, int32_t* status, void* stream) {
  if (!X || !D || !T) return fail(FD_ERR_INVALID_ARG, "X, D and T must be device pointers");
  if (o && (o->flags & FD_KEEP_CHECKPOINTS))
    return fail(FD_ERR_INVALID_ARG, "fd_udv does not keep checkpoints");
  Outs out;
  out.X = X;
  out.D = D;
  out.T = T;
  out.status = status;
  return run(p, 1, o, FD_WHAT_UDV, out, ws, ws_bytes, stream);
}

size_t fd_displaced_workspace_bytes(const fd_problem* p, const fd_options* o, int32_t npairs) {
  const Opts r = resolve(o);
  if (validate(p, 1, r) != FD_OK) return 0;
  if (npairs < 1) {
    fail(FD_ERR_INVALID_ARG, "npairs must be >= 1");
    return 0;
  }
  std::vector<int32_t> one(npairs, 1);
  Plan pl;
  build_displaced_plan(p, r, npairs, one.data(), one.data(), nullptr, pl, nullptr);
  return pl.total;
}

int fd_greens_displaced(const fd_problem* p, const fd_options* o, int32_t npairs, const int32_t* t,
                        const int32_t* t0, double* G, void* ws, size_t ws_bytes, int32_t* status,
                        void* stream) {
  if (!G) return fail(FD_ERR_INVALID_ARG, "G must be a device pointer");
  if (!status) return fail(FD_ERR_INVALID_ARG, "status must be a device pointer");
  const Opts r = resolve(o);
  int rc = validate(p, 1, r);
  if (rc != FD_OK) return rc;
  rc = validate_pairs(p, npairs, t, t0);
  if (rc != FD_OK) return rc;
  const size_t need = fd_displaced_workspace_bytes(p, o, npairs);
  rc = check_ws(ws, ws_bytes, need);
  if (rc != FD_OK) return rc;
  Plan pl;
  build_displaced_plan(p, r, npairs, t, t0, static_cast<char*>(ws), pl, G);
  pl.probs[0].status = status;
  return execute(pl, static_cast<char*>(ws), static_cast<hipStream_t>(stream));
}

int fd_logdet_batched(const fd_problem* p, int32_t nprob, const fd_options* o, double* logdet,
                      void* ws, size_t ws_bytes, int32_t* status, void* stream) {
  if (!logdet) return fail(FD_ERR_INVALID_ARG, "logdet must be a device pointer");
  if (!status) return fail(FD_ERR_INVALID_ARG, "status must be a device pointer");
  Outs out;
  out.logdet = logdet;
  out.status = status;
  return run(p, nprob, o, FD_WHAT_LOGDET, out, ws, ws_bytes, stream);
}

int fd_greens_batched(const fd_problem* p, int32_t nprob, const fd_options* o, double* logdet,
                      double* G, void* ws, size_t ws_bytes, int32_t* status, void* stream) {
  if (!G) return fail(FD_ERR_INVALID_ARG, "G must be a device pointer");
  if (!status) return fail(FD_ERR_INVALID_ARG, "status must be a device pointer");
  Outs out;
  out.logdet = logdet;
  out.G = G;
  out.status = status;
  return run(p, nprob, o, FD_WHAT_GREENS, out, ws, ws_bytes, stream);
}

int fd_force_batched(const fd_problem* p, int32_t nprob, const fd_options* o, double* logdet,
                     double* force, double* force_im, void* ws, size_t ws_bytes, int32_t* status,
                     void* stream) {
  if (!force) return fail(FD_ERR_INVALID_ARG, "force must be a device pointer");
  if (!status) return fail(FD_ERR_INVALID_ARG, "status must be a device pointer");
  Outs out;
  out.logdet = logdet;
  out.force = force;
  out.force_im = force_im;
  out.status = status;
  return run(p, nprob, o, FD_WHAT_FORCE, out, ws, ws_bytes, stream);
}

size_t fd_sparse_workspace_bytes(const fd_problem* p, int32_t nprob, const fd_options* o,
                                 int32_t what) {
  if (!p || nprob < 1) return 0;
  if (what != FD_WHAT_LOGDET && what != FD_WHAT_GREENS) return 0;
  const Opts r = resolve(o, p, nprob, what);
  Plan pl;
  fd_ell none{1, nullptr, nullptr};
  std::vector<fd_ell> ell(nprob, none);
  build_plan(p, nprob, r, what, nullptr, pl, ell.data(), 1);
  return pl.total;
}

int fd_sparse_greens_batched(const fd_problem* p, int32_t nprob, const fd_ell* hop,
                             int32_t taylor_n, const fd_options* o, double* logdet, double* G,
                             void* ws, size_t ws_bytes, int32_t* status, void* stream) {
  if (!p || nprob < 1) return fail(FD_ERR_INVALID_ARG, "no problems given");
  if (!hop) return fail(FD_ERR_INVALID_ARG, "hop must be a host array of nprob fd_ell");
  if (!logdet) return fail(FD_ERR_INVALID_ARG, "logdet must be a device pointer");
  if (!status) return fail(FD_ERR_INVALID_ARG, "status must be a device pointer");
  if (taylor_n < 1 || taylor_n > fdet::kMaxTaylor)
    return fail(FD_ERR_INVALID_ARG, "taylor_n must be in [1, 8]");
  if (o && (o->flags & (FD_KEEP_CHECKPOINTS | FD_REUSE_E | FD_SINGLE_LAUNCH)))
    return fail(FD_ERR_INVALID_ARG, "the matrix-free slices take no flags");
  const int what = G ? FD_WHAT_GREENS : FD_WHAT_LOGDET;
  const Opts r = resolve(o, p, nprob, what);
  if (r.s > 16) return fail(FD_ERR_INVALID_ARG, "the matrix-free slices need s <= 16");
  std::vector<fd_problem> pk(p, p + nprob);
  for (int i = 0; i < nprob; ++i) {
    char buf[128];
    if (hop[i].q < 1 || hop[i].q > 64 || !hop[i].col || !hop[i].val) {
      std::snprintf(buf, sizeof buf, "problem %d: q must be in [1, 64] with col and val set", i);
      return fail(FD_ERR_INVALID_ARG, buf);
    }
    if (!pk[i].K) pk[i].K = hop[i].val;   // K itself is not read
  }
  int rc = validate(pk.data(), nprob, r);
  if (rc != FD_OK) return rc;
  Plan sizing;
  build_plan(pk.data(), nprob, r, what, nullptr, sizing, hop, taylor_n);
  rc = check_ws(ws, ws_bytes, sizing.total);
  if (rc != FD_OK) return rc;
  Plan pl;
  build_plan(pk.data(), nprob, r, what, static_cast<char*>(ws), pl, hop, taylor_n);
  size_t goff = 0;
  for (int i = 0; i < nprob; ++i) {
    Prob& P = pl.probs[i];
    P.status = status + i;
    P.logdet = logdet + 2 * i;
    P.G = G ? G + goff : nullptr;
    goff += (size_t)2 * p[i].N * p[i].N;
  }
  return execute(pl, static_cast<char*>(ws), static_cast<hipStream_t>(stream));
}

int fd_sparse_greens(const fd_problem* p, const fd_ell* hop, int32_t taylor_n,
                     const fd_options* o, double* logdet, double* G, void* ws, size_t ws_bytes,
                     int32_t* status, void* stream) {
  return fd_sparse_greens_batched(p, 1, hop, taylor_n, o, logdet, G, ws, ws_bytes, status, stream);
}

int fd_force_response_batched(const fd_problem* p, int32_t nprob, const fd_options* o,
                              const double* A, double* trace, double* logdet, double* force,
                              double* force_im, void* ws, size_t ws_bytes, int32_t* status,
                              void* stream) {
  if (!A || !trace) return fail(FD_ERR_INVALID_ARG, "A and trace must be device pointers");
  for (int i = 0; i < nprob && p; ++i)
    if (p[i].N > 128)
      return fail(FD_ERR_UNSUPPORTED,
                  "the operator trace is switched off for N > 128: one run of it at N = 162 "
                  "returned wrong traces and the next faulted, with the cause not found");
  if (!force) return fail(FD_ERR_INVALID_ARG, "force must be a device pointer");
  if (!status) return fail(FD_ERR_INVALID_ARG, "status must be a device pointer");
  Outs out;
  out.logdet = logdet;
  out.force = force;
  out.force_im = force_im;
  out.op = A;
  out.op_trace = trace;
  out.status = status;
  return run(p, nprob, o, FD_WHAT_FORCE, out, ws, ws_bytes, stream);
}

int fd_force_response(const fd_problem* p, const fd_options* o, const double* A, double* trace,
                      double* logdet, double* force, double* force_im, void* ws, size_t ws_bytes,
                      int32_t* status, void* stream) {
  return fd_force_response_batched(p, 1, o, A, trace, logdet, force, force_im, ws, ws_bytes,
                                   status, stream);
}

int fd_plan_create(int32_t what, const fd_problem* p, int32_t nprob, const fd_options* o,
                   double* logdet, double* G, double* force, double* force_im, void* ws,
                   size_t ws_bytes, int32_t* status, void* stream, fd_plan** plan) {
  if (!plan) return fail(FD_ERR_INVALID_ARG, "plan must not be NULL");
  *plan = nullptr;
  if (what != FD_WHAT_LOGDET && what != FD_WHAT_GREENS && what != FD_WHAT_FORCE)
    return fail(FD_ERR_INVALID_ARG, "a plan computes FD_WHAT_LOGDET, _GREENS or _FORCE");
  if (!status) return fail(FD_ERR_INVALID_ARG, "status must be a device pointer");
  if (what == FD_WHAT_LOGDET && !logdet) return fail(FD_ERR_INVALID_ARG, "logdet must be a device pointer");
  if (what == FD_WHAT_GREENS && !G) return fail(FD_ERR_INVALID_ARG, "G must be a device pointer");
  if (what == FD_WHAT_FORCE && !force) return fail(FD_ERR_INVALID_ARG, "force must be a device pointer");
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(st, &cap) != hipSuccess || cap != hipStreamCaptureStatusNone)
    return fail(FD_ERR_INVALID_ARG, "create plans outside stream capture");
  Outs out;
  out.logdet = logdet;
  out.G = G;   // FD_WHAT_FORCE: G from the checkpoint at row 0, if given
  out.force = what == FD_WHAT_FORCE ? force : nullptr;
  out.force_im = what == FD_WHAT_FORCE ? force_im : nullptr;
  out.status = status;
  fd_plan* h = new fd_plan;
  int rc = prepare(p, nprob, o, what, out, ws, ws_bytes, h->pl);
  if (rc != FD_OK) { delete h; return rc; }
  h->ws = static_cast<char*>(ws);
  rc = upload(h->pl, h->first, h->ws, st);
  if (rc != FD_OK) {
    delete h;
    return rc;
  }
  hipError_t e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    delete h;
    return fail(FD_ERR_HIP, std::string("descriptor upload: ") + hipGetErrorString(e));
  }
  *plan = h;
  return FD_OK;
}

int fd_plan_launch(const fd_plan* plan, void* stream) {
  if (!plan) return fail(FD_ERR_INVALID_ARG, "plan must not be NULL");
  return launch_phases(plan->pl, plan->first, plan->ws, static_cast<hipStream_t>(stream));
}

void fd_plan_destroy(fd_plan* plan) { delete plan; }

int fd_plan_segments(const fd_plan* plan, int32_t* seg, int32_t n) {
  if (!plan) return fail(FD_ERR_INVALID_ARG, "plan must not be NULL");
  const int np = (int)plan->pl.units.size();
  if (seg)
    for (int i = 0; i < std::min<int>(n, np); ++i) seg[i] = plan->pl.units[i];
  return np;
}

int fd_autotune(int32_t what, const fd_problem* p, int32_t nprob, const fd_options* o,
                void* stream, fd_options* best, float* best_ms) {
  if (what != FD_WHAT_LOGDET && what != FD_WHAT_GREENS && what != FD_WHAT_FORCE)
    return fail(FD_ERR_INVALID_ARG, "autotune covers FD_WHAT_LOGDET, _GREENS and _FORCE");
  if (!p || nprob < 1) return fail(FD_ERR_INVALID_ARG, "no problems given");
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(st, &cap) != hipSuccess || cap != hipStreamCaptureStatusNone)
    return fail(FD_ERR_INVALID_ARG, "autotune outside stream capture");
  fd_options base{0, 0, 0, 0};
  if (o) base = *o;
  base.flags &= ~FD_REUSE_E;
  {
    Opts chk = resolve(&base, p, nprob, what);
    int rc = validate(p, nprob, chk);
    if (rc != FD_OK) return rc;
  }
  // s candidates within s * dk * radius(K) <= 6
  double worst = 0.0;
  for (int i = 0; i < nprob; ++i) {
    std::vector<double> K((size_t)p[i].N * p[i].N);
    hipError_t e = hipMemcpy(K.data(), p[i].K, K.size() * sizeof(double), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return fail(FD_ERR_HIP, std::string("reading K: ") + hipGetErrorString(e));
    worst = std::max(worst, std::fabs(p[i].dk) * radius_bound(K, p[i].N));
  }
  std::vector<int> s_list, seg_list;
  if (base.s > 0) s_list.push_back(base.s);
  else
    for (int s : {4, 8, 16})
      if (s == 4 || s * worst <= 6.0) s_list.push_back(s);
  int maxNt = 1;
  for (int i = 0; i < nprob; ++i) maxNt = std::max(maxNt, p[i].Nt);
  if (what == FD_WHAT_FORCE || base.segments > 0) seg_list.push_back(std::max(base.segments, 1));
  else
    for (int g = 1; g <= 64 && g <= maxNt; g *= 2) seg_list.push_back(g);

  // outputs and the largest workspace
  size_t ws_need = 0;
  for (int s : s_list)
    for (int g : seg_list) {
      fd_options c = base;
      c.s = s;
      c.segments = g;
      Plan pl;
      build_plan(p, nprob, resolve(&c, p, nprob, what), what, nullptr, pl);
      ws_need = std::max(ws_need, pl.total);
    }
  size_t gsz = 0, fsz = 0;
  for (int i = 0; i < nprob; ++i) {
    gsz += (size_t)2 * p[i].N * p[i].N;
    fsz += (size_t)p[i].Nt * p[i].N;
  }
  void *ws = nullptr, *ld = nullptr, *out = nullptr, *stv = nullptr;
  hipEvent_t ea = nullptr, eb = nullptr;
  auto cleanup = [&]() {
    if (ws) hipFree(ws);
    if (ld) hipFree(ld);
    if (out) hipFree(out);
    if (stv) hipFree(stv);
    if (ea) hipEventDestroy(ea);
    if (eb) hipEventDestroy(eb);
  };
  const size_t out_bytes = sizeof(double) * (what == FD_WHAT_FORCE ? fsz : std::max<size_t>(gsz, 1));
  if (hipMalloc(&ws, ws_need) != hipSuccess || hipMalloc(&ld, sizeof(double) * 2 * nprob) != hipSuccess ||
      hipMalloc(&out, out_bytes) != hipSuccess || hipMalloc(&stv, sizeof(int32_t) * nprob) != hipSuccess ||
      hipEventCreate(&ea) != hipSuccess || hipEventCreate(&eb) != hipSuccess) {
    cleanup();
    return fail(FD_ERR_HIP, "autotune: device allocation failed");
  }
  float bms = -1.0f;
  fd_options bopt = base;
  std::vector<int32_t> hst(nprob);
  for (int s : s_list)
    for (int g : seg_list) {
      fd_options c = base;
      c.s = s;
      c.segments = g;
      float times[3] = {1e30f, 1e30f, 1e30f};
      bool ok = true;
      for (int rep = -1; rep < 3 && ok; ++rep) {
        if (rep >= 0) hipEventRecord(ea, st);
        int rc;
        if (what == FD_WHAT_FORCE)
          rc = fd_force_batched(p, nprob, &c, (double*)ld, (double*)out, nullptr, ws, ws_need,
                                (int32_t*)stv, stream);
        else if (what == FD_WHAT_GREENS)
          rc = fd_greens_batched(p, nprob, &c, (double*)ld, (double*)out, ws, ws_need,
                                 (int32_t*)stv, stream);
        else
          rc = fd_logdet_batched(p, nprob, &c, (double*)ld, ws, ws_need, (int32_t*)stv, stream);
        if (rc != FD_OK) { cleanup(); return rc; }
        if (rep >= 0) {
          hipEventRecord(eb, st);
          hipEventSynchronize(eb);
          hipEventElapsedTime(&times[rep], ea, eb);
        }
        if (hipMemcpy(hst.data(), stv, sizeof(int32_t) * nprob, hipMemcpyDeviceToHost) != hipSuccess) {
          cleanup();
          return fail(FD_ERR_HIP, "autotune: reading status failed");
        }
        for (int32_t v : hst) ok = ok && v >= 0;
      }
      if (!ok) continue;
      std::sort(times, times + 3);
      if (bms < 0.0f || times[1] < bms) {
        bms = times[1];
        bopt = c;
      }
    }
  cleanup();
  if (bms < 0.0f) return fail(FD_ERR_UNSUPPORTED, "autotune: no candidate finished without error");
  tune_store(tune_key(p, nprob, what), TuneVal{bopt.s, bopt.segments, bms});
  if (best) *best = bopt;
  if (best_ms) *best_ms = bms;
  return FD_OK;
}

int fd_tune_save(const char* path) {
  if (!path) return fail(FD_ERR_INVALID_ARG, "path must not be NULL");
  std::ofstream f(path);
  if (!f) return fail(FD_ERR_INVALID_ARG, std::string("cannot write ") + path);
  std::lock_guard<std::mutex> g(g_tune_mu);
  f << "fdet-tune 1\n";
  for (auto& e : g_tune)
    f << e.first.what << ' ' << e.first.maxN << ' ' << e.first.maxNt << ' ' << e.first.nprob << ' '
      << e.first.dk_micro << ' ' << e.second.s << ' ' << e.second.segments << ' ' << e.second.ms
      << '\n';
  return f ? FD_OK : fail(FD_ERR_INVALID_ARG, std::string("write failed: ") + path);
}

int fd_tune_load(const char* path) {
  if (!path) return fail(FD_ERR_INVALID_ARG, "path must not be NULL");
  std::ifstream f(path);
  if (!f) return fail(FD_ERR_INVALID_ARG, std::string("cannot read ") + path);
  std::string magic;
  int ver = 0;
  f >> magic >> ver;
  if (magic != "fdet-tune" || ver != 1) return fail(FD_ERR_INVALID_ARG, "not an fdet tune file");
  int n = 0;
  TuneKey k;
  TuneVal v;
  while (f >> k.what >> k.maxN >> k.maxNt >> k.nprob >> k.dk_micro >> v.s >> v.segments >> v.ms) {
    if (k.what < FD_WHAT_LOGDET || k.what > FD_WHAT_FORCE || v.s < 1 || v.segments < 1 ||
        k.maxN < 1 || k.maxN > FD_MAX_N)
      return fail(FD_ERR_INVALID_ARG, "malformed tune entry");
    tune_store(k, v);
    ++n;
  }
  if (!f.eof()) return fail(FD_ERR_INVALID_ARG, "malformed tune file");
  return n;
}

int fd_tune_clear(void) {
  std::lock_guard<std::mutex> g(g_tune_mu);
  g_tune.clear();
  return FD_OK;
}

const char* fd_strerror(int code) {
  switch (code) {
    case FD_OK: return "ok";
    case FD_WARN_ILLCOND: return "M is numerically close to singular; results returned";
    case FD_ERR_INVALID_ARG: return "invalid argument";
    case FD_ERR_WORKSPACE: return "workspace missing, misaligned or too small";
    case FD_ERR_SINGULAR: return "M is singular";
    case FD_ERR_NONFINITE: return "non-finite input or intermediate";
    case FD_ERR_HIP: return "HIP runtime error";
    case FD_ERR_UNSUPPORTED: return "unsupported configuration";
    default: return "unknown code";
  }
}

const char* fd_last_error(void) { return g_last_error.c_str(); }

int fd_hmc_leapfrog(const fd_problem* p, int32_t nprob, const fd_options* o, double dU, double eps,
                    int32_t nsteps, double* pi, double* dH, void* ws, size_t ws_bytes,
                    int32_t* status, void* stream) {
  HmcState S;
  fd_options o1;
  int rc = hmc_setup(p, nprob, o, dU, eps, nsteps, pi, dH, ws, ws_bytes, status, stream, o1, S);
  if (rc != FD_OK) return rc;
  // the first force evaluation also computes exp(+-dk K); the plan for the
  // later ones, created after it (same layout), reuses it
  fd_plan* plan = nullptr;
  rc = hmc_enqueue(S, static_cast<hipStream_t>(stream), [&](int n) -> int {
    if (n > 0) return fd_plan_launch(plan, stream);
    int r = fd_plan_create(FD_WHAT_FORCE, p, nprob, &o1, S.ld, nullptr, S.F, nullptr, ws,
                           S.force_ws, S.sstep, stream, &plan);
    if (r == FD_OK) r = fd_plan_launch(plan, stream);
    fd_plan_destroy(plan);
    plan = nullptr;
    if (r != FD_OK) return r;
    fd_options o2 = o1;
    o2.flags |= FD_REUSE_E;
    return fd_plan_create(FD_WHAT_FORCE, p, nprob, &o2, S.ld, nullptr, S.F, nullptr, ws,
                          S.force_ws, S.sstep, stream, &plan);
  });
  fd_plan_destroy(plan);
  return rc;
}

struct fd_hmc_plan {
  HmcState S;
  fd_plan* force = nullptr;   // prepared force call with exp(+-dk K) already in ws
};

int fd_hmc_plan_create(const fd_problem* p, int32_t nprob, const fd_options* o, double dU,
                       double eps, int32_t nsteps, double* pi, double* dH, void* ws,
                       size_t ws_bytes, int32_t* status, void* stream, fd_hmc_plan** plan) {
  if (!plan) return fail(FD_ERR_INVALID_ARG, "plan must not be NULL");
  *plan = nullptr;
  fd_hmc_plan* h = new fd_hmc_plan;
  fd_options o1;
  int rc = hmc_setup(p, nprob, o, dU, eps, nsteps, pi, dH, ws, ws_bytes, status, stream, o1, h->S);
  // one full force call now leaves exp(+-dk K) in the workspace; the plan
  // kept for the launches reuses it (K and dk fixed for the plan's lifetime)
  fd_plan* full = nullptr;
  if (rc == FD_OK)
    rc = fd_plan_create(FD_WHAT_FORCE, p, nprob, &o1, h->S.ld, nullptr, h->S.F, nullptr, ws,
                        h->S.force_ws, h->S.sstep, stream, &full);
  if (rc == FD_OK) rc = fd_plan_launch(full, stream);
  fd_plan_destroy(full);
  if (rc == FD_OK) {
    o1.flags |= FD_REUSE_E;
    rc = fd_plan_create(FD_WHAT_FORCE, p, nprob, &o1, h->S.ld, nullptr, h->S.F, nullptr, ws,
                        h->S.force_ws, h->S.sstep, stream, &h->force);
  }
  if (rc != FD_OK) {
    delete h;
    return rc;
  }
  *plan = h;
  return FD_OK;
}

int fd_hmc_plan_launch(const fd_hmc_plan* h, void* stream) {
  if (!h) return fail(FD_ERR_INVALID_ARG, "plan must not be NULL");
  return hmc_enqueue(h->S, static_cast<hipStream_t>(stream),
                     [&](int) -> int { return fd_plan_launch(h->force, stream); });
}

void fd_hmc_plan_destroy(fd_hmc_plan* h) {
  if (!h) return;
  fd_plan_destroy(h->force);
  delete h;
}

size_t fd_response_trace_workspace_bytes(int32_t N) {
  if (N < 1 || N > FD_MAX_N) {
    fail(FD_ERR_INVALID_ARG, "N must be in [1, FD_MAX_N]");
    return 0;
  }
  const size_t nb = (size_t)(N + 31) / 32;   // 32 x 32 tiles, 4 partial sums each
  return align_up(4 * nb * nb * sizeof(double));
}

int fd_response_trace(int32_t N, const double* G, const double* A, double* out, void* ws,
                      size_t ws_bytes, void* stream) {
  const size_t need = fd_response_trace_workspace_bytes(N);
  if (need == 0) return FD_ERR_INVALID_ARG;
  if (!G || !out) return fail(FD_ERR_INVALID_ARG, "G and out must be device pointers");
  const int rc = check_ws(ws, ws_bytes, need);
  if (rc != FD_OK) return rc;
  const hipError_t e = fdet_launch_trace(N, G, A, static_cast<double*>(ws), out,
                                         static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return fail(FD_ERR_HIP, hipGetErrorString(e));
  return FD_OK;
}

int fd_diag_response(int32_t Nt, int32_t N, const double* force, const double* force_im,
                     const double* a, double* out, void* stream) {
  if (Nt < 1 || N < 1 || N > FD_MAX_N) return fail(FD_ERR_INVALID_ARG, "need Nt >= 1 and 1 <= N <= FD_MAX_N");
  if (!force || !force_im || !out)
    return fail(FD_ERR_INVALID_ARG, "force, force_im and out must be device pointers");
  const hipError_t e = fdet_launch_diag_response(Nt, N, force, force_im, a, out,
                                                 static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return fail(FD_ERR_HIP, hipGetErrorString(e));
  return FD_OK;
}

#ifndef FDET_SRC_DIGEST
#define FDET_SRC_DIGEST "unknown"
#endif
const char* fd_version(void) { return "fdet 0.2.0 (gfx950) src " FDET_SRC_DIGEST; }

int fd_profile_start(void) {
  for (auto& r : g_prof) {
    hipEventDestroy(r.a);
    hipEventDestroy(r.b);
  }
  g_prof.clear();
  g_prof_on = true;
  return FD_OK;
}

int fd_profile_stop(int32_t max, int32_t* kinds, int32_t* nitems, float* ms) {
  g_prof_on = false;
  int n = 0;
  for (auto& r : g_prof) {
    if (n < max) {
      float t = -1.0f;
      if (hipEventSynchronize(r.b) == hipSuccess) hipEventElapsedTime(&t, r.a, r.b);
      if (kinds) kinds[n] = r.kind;
      if (nitems) nitems[n] = r.nitems;
      if (ms) ms[n] = t;
    }
    ++n;
    hipEventDestroy(r.a);
    hipEventDestroy(r.b);
  }
  g_prof.clear();
  return n;
}

}  // extern "C"

// Error reporting for the library's other translation units.
int fdet_fail(int code, const char* msg) { return fail(code, msg ? msg : ""); }
