// Host side of libfdet: argument checking, workspace layout, work-item plans
// and kernel launches behind the C ABI declared in include/fdet.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/fdet.h"
#include "fdet_plan.h"

extern "C" hipError_t fdet_launch_items(int maxn, int kind, const fdet::Prob* probs,
                                        const fdet::Item* items, int nitems, hipStream_t st);
extern "C" hipError_t fdet_launch_init_status(const fdet::Prob* probs, int nprob, hipStream_t st);

namespace {

using fdet::Item;
using fdet::Prob;
using fdet::Udv;

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
size_t scratch_bytes(int Np) { return align_up(4 * cmat_bytes(Np) + (size_t)2 * Np * sizeof(double)); }

struct Opts {
  int s, c, segments, flags;
};

Opts resolve(const fd_options* o) {
  Opts r{8, 16, 0, 0};
  if (o) {
    if (o->s > 0) r.s = o->s;
    if (o->checkpoint > 0) r.c = o->checkpoint;
    if (o->segments > 0) r.segments = o->segments;
    r.flags = o->flags;
  }
  return r;
}

// Number of independent time segments of one problem (det / G / UDV).
int segments_for(const fd_problem& p, const Opts& o) {
  int nseg = o.segments > 0 ? o.segments : 1;
  nseg = std::min(nseg, p.Nt);
  return std::max(nseg, 1);
}

// Offsets are computed against `base`; with base == nullptr only sizes matter.
struct Plan {
  std::vector<Prob> probs;
  std::vector<std::vector<Item>> phases;
  size_t desc_bytes = 0;
  size_t total = 0;
  int maxN = 0;
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

int validate(const fd_problem* p, int nprob, const Opts& o) {
  if (!p || nprob < 1) return fail(FD_ERR_INVALID_ARG, "no problems given");
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

// Build the layout and the work items.  `what` = FD_WHAT_*.
void build_plan(const fd_problem* p, int nprob, const Opts& o, int what, char* base, Plan& pl) {
  pl.probs.assign(nprob, Prob{});
  pl.maxN = 0;
  size_t nitems = 0;
  // count items to size the descriptor region
  const bool force = what == FD_WHAT_FORCE;
  std::vector<int> nseg(nprob), nck(nprob);
  int maxlev = 0;
  for (int i = 0; i < nprob; ++i) {
    pl.maxN = std::max(pl.maxN, p[i].N);
    if (force) {
      nck[i] = (p[i].Nt + o.c - 1) / o.c;
      nitems += 2 + 2 + 1 + nck[i];
    } else {
      nseg[i] = segments_for(p[i], o);
      int lev = 0;
      while ((1 << lev) < nseg[i]) ++lev;
      maxlev = std::max(maxlev, lev);
      nitems += 1 + nseg[i] + nseg[i] + 1;
    }
  }
  pl.desc_bytes = align_up(sizeof(Prob) * nprob) + align_up(sizeof(Item) * nitems);
  Cursor cur{base, align_up(pl.desc_bytes)};

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
      if (!(o.flags & FD_REUSE_E)) {
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
        c.c = o.c;
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
      const int nc = nck[i];
      const size_t ub = udv_bytes(Np);
      double* pre = cur.take(ub * nc);
      double* suf = cur.take(ub * nc);
      Udv st[2];
      double* cs[2];
      for (int k = 0; k < 2; ++k) {
        st[k] = make_udv(cur.take(ub), Np);
        cs[k] = cur.take(scratch_bytes(Np));
      }
      std::vector<double*> fs(nc);
      for (int k = 0; k < nc; ++k) fs[k] = cur.take(scratch_bytes(Np));
      if (!(o.flags & FD_REUSE_E)) {
        for (int sg = 0; sg < 2; ++sg) {
          Item e = blank_item(fdet::IK_EXPM, i);
          e.sign = sg == 0 ? 1 : -1;
          e.scr = cs[sg];
          expm.push_back(e);
        }
      }
      for (int k = 0; k < 2; ++k) {
        Item c = blank_item(fdet::IK_CHAIN, i);
        c.t0 = 0;
        c.t1 = q.Nt;
        c.s = o.s;
        c.c = o.c;
        c.flags = fdet::IF_IDENTITY | fdet::IF_CKPT | (k == 1 ? fdet::IF_ADJOINT : 0);
        c.a = st[k];
        c.ck = k == 0 ? pre : suf;
        c.ckstride = (int64_t)(ub / sizeof(double));
        c.scr = cs[k];
        chain.push_back(c);
      }
      // log det of the whole product from the prefix chain's final state
      {
        Item z = blank_item(fdet::IK_CLOSE, i);
        z.a = st[0];
        z.scr = cs[0];
        close.push_back(z);
      }
      // checkpoint k (row k*c) carries G~ forward over the first half of the
      // gap to the next checkpoint and backward over the second half of the
      // gap from the previous one (cyclically for k = 0), so no G~ is carried
      // across more than about c/2 slices
      const int last_gap = q.Nt - (nc - 1) * o.c;
      for (int k = 0; k < nc; ++k) {
        Item f = blank_item(fdet::IK_FORCE, i);
        const int gap_fwd = (k + 1 < nc) ? o.c : last_gap;
        const int gap_bwd = (k > 0) ? o.c : last_gap;
        f.t0 = k * o.c;
        f.t1 = f.t0 + (gap_fwd + 1) / 2;
        f.nb = (nc == 1) ? q.Nt - (q.Nt + 1) / 2 : gap_bwd / 2;
        f.a = make_udv(pre ? (double*)((char*)pre + ub * k) : nullptr, Np);
        f.b = make_udv(suf ? (double*)((char*)suf + ub * k) : nullptr, Np);
        f.scr = fs[k];
        forcei.push_back(f);
      }
    }
  }
  pl.phases.clear();
  if (!expm.empty()) pl.phases.push_back(expm);
  pl.phases.push_back(chain);
  for (auto& c : comb)
    if (!c.empty()) pl.phases.push_back(c);
  if (!close.empty()) pl.phases.push_back(close);
  if (!forcei.empty()) pl.phases.push_back(forcei);
  pl.total = cur.off;
}

// Upload descriptors into the head of the workspace and launch every phase.
int execute(Plan& pl, char* ws, hipStream_t st) {
  std::vector<char> host(pl.desc_bytes, 0);
  const size_t pbytes = align_up(sizeof(Prob) * pl.probs.size());
  std::memcpy(host.data(), pl.probs.data(), sizeof(Prob) * pl.probs.size());
  std::vector<size_t> first;
  size_t n = 0;
  for (auto& ph : pl.phases) {
    first.push_back(n);
    std::memcpy(host.data() + pbytes + n * sizeof(Item), ph.data(), ph.size() * sizeof(Item));
    n += ph.size();
  }
  hipError_t e = hipMemcpyAsync(ws, host.data(), pl.desc_bytes, hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return fail(FD_ERR_HIP, std::string("descriptor upload: ") + hipGetErrorString(e));
  const Prob* dprobs = reinterpret_cast<const Prob*>(ws);
  const Item* ditems = reinterpret_cast<const Item*>(ws + pbytes);
  e = fdet_launch_init_status(dprobs, (int)pl.probs.size(), st);
  if (e != hipSuccess) return fail(FD_ERR_HIP, std::string("launch: ") + hipGetErrorString(e));
  for (size_t k = 0; k < pl.phases.size(); ++k) {
    const int kind = pl.phases[k].front().kind;
    PhaseRec rec{kind, (int)pl.phases[k].size(), nullptr, nullptr};
    if (g_prof_on) {
      if (hipEventCreate(&rec.a) != hipSuccess || hipEventCreate(&rec.b) != hipSuccess)
        return fail(FD_ERR_HIP, "event creation failed");
      hipEventRecord(rec.a, st);
    }
    e = fdet_launch_items(pl.maxN, kind, dprobs, ditems + first[k], (int)pl.phases[k].size(), st);
    if (e != hipSuccess) return fail(FD_ERR_HIP, std::string("launch: ") + hipGetErrorString(e));
    if (g_prof_on) {
      hipEventRecord(rec.b, st);
      g_prof.push_back(rec);
    }
  }
  return FD_OK;
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
  int32_t* status = nullptr;
};

int run(const fd_problem* p, int nprob, const fd_options* opt, int what, const Outs& out, void* ws,
        size_t ws_bytes, void* stream) {
  const Opts o = resolve(opt);
  int rc = validate(p, nprob, o);
  if (rc != FD_OK) return rc;
  Plan sizing;
  build_plan(p, nprob, o, what, nullptr, sizing);
  rc = check_ws(ws, ws_bytes, sizing.total);
  if (rc != FD_OK) return rc;
  Plan pl;
  build_plan(p, nprob, o, what, static_cast<char*>(ws), pl);
  size_t goff = 0, foff = 0;
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
    goff += (size_t)2 * p[i].N * p[i].N;
    foff += (size_t)p[i].Nt * p[i].N;
  }
  return execute(pl, static_cast<char*>(ws), static_cast<hipStream_t>(stream));
}

}  // namespace

extern "C" {

size_t fd_workspace_bytes(const fd_problem* p, int32_t nprob, const fd_options* o, int32_t what) {
  const Opts r = resolve(o);
  if (what < FD_WHAT_LOGDET || what > FD_WHAT_UDV) {
    fail(FD_ERR_INVALID_ARG, "unknown workspace kind");
    return 0;
  }
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
  // only the exponential phase
  std::vector<Item> keep = pl.phases.front();
  pl.phases.assign(1, keep);
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
  Outs out;
  out.X = X;
  out.D = D;
  out.T = T;
  out.status = status;
  return run(p, 1, o, FD_WHAT_UDV, out, ws, ws_bytes, stream);
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

const char* fd_version(void) { return "fdet 0.1.0 (gfx950)"; }

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
