// Host-only check of the work-item planner (no GPU): the host side of the
// library is compiled with the kernel launchers stubbed out, plans are built
// against a fake workspace base for named shapes and for random batches of
// every kind, and every launch is checked: items of one launch share no
// scratch and never write a slot another item of it reads; every workspace
// pointer an item carries (E, E^-1, UDV slots, scratch) lies inside the
// workspace that fd_workspace_bytes sizes; slice ranges stay inside [0, N_t].
// Prints one line per plan and "bad <count>" last; exits nonzero on a finding.
#include "../paper_2604_02130_amd/csrc/fdet_abi.cpp"
#include <set>
#include <random>
#include <map>
extern "C" hipError_t fdet_launch_items_32(int, const fdet::Prob*, const fdet::Item*, int, hipStream_t) { return hipSuccess; }
extern "C" hipError_t fdet_launch_items_64(int, const fdet::Prob*, const fdet::Item*, int, hipStream_t) { return hipSuccess; }
extern "C" hipError_t fdet_launch_items_80(int, const fdet::Prob*, const fdet::Item*, int, hipStream_t) { return hipSuccess; }
extern "C" hipError_t fdet_launch_items_96(int, const fdet::Prob*, const fdet::Item*, int, hipStream_t) { return hipSuccess; }
extern "C" hipError_t fdet_launch_items_128(int, const fdet::Prob*, const fdet::Item*, int, hipStream_t) { return hipSuccess; }
extern "C" hipError_t fdet_launch_items_512(int, const fdet::Prob*, const fdet::Item*, int, hipStream_t) { return hipSuccess; }
extern "C" hipError_t fdet_launch_init_status(const fdet::Prob*, int, fdet::Sched*, hipStream_t) { return hipSuccess; }
extern "C" hipError_t fdet_launch_persist_32(const fdet::Prob*, const fdet::Item*, int, const int32_t*, uint32_t*, fdet::Sched*, uint64_t, int, hipStream_t) { return hipSuccess; }
extern "C" int fdet_persist_blocks_per_cu_32(void) { return 1; }
extern "C" hipError_t fdet_launch_persist_64(const fdet::Prob*, const fdet::Item*, int, const int32_t*, uint32_t*, fdet::Sched*, uint64_t, int, hipStream_t) { return hipSuccess; }
extern "C" int fdet_persist_blocks_per_cu_64(void) { return 1; }
extern "C" hipError_t fdet_launch_persist_80(const fdet::Prob*, const fdet::Item*, int, const int32_t*, uint32_t*, fdet::Sched*, uint64_t, int, hipStream_t) { return hipSuccess; }
extern "C" int fdet_persist_blocks_per_cu_80(void) { return 1; }
extern "C" hipError_t fdet_launch_persist_96(const fdet::Prob*, const fdet::Item*, int, const int32_t*, uint32_t*, fdet::Sched*, uint64_t, int, hipStream_t) { return hipSuccess; }
extern "C" int fdet_persist_blocks_per_cu_96(void) { return 1; }
extern "C" hipError_t fdet_launch_persist_128(const fdet::Prob*, const fdet::Item*, int, const int32_t*, uint32_t*, fdet::Sched*, uint64_t, int, hipStream_t) { return hipSuccess; }
extern "C" int fdet_persist_blocks_per_cu_128(void) { return 1; }
extern "C" hipError_t fdet_launch_persist_512(const fdet::Prob*, const fdet::Item*, int, const int32_t*, uint32_t*, fdet::Sched*, uint64_t, int, hipStream_t) { return hipSuccess; }
extern "C" int fdet_persist_blocks_per_cu_512(void) { return 1; }

extern "C" hipError_t fdet_launch_trace(int, const double*, const double*, double*, double*, hipStream_t) { return hipSuccess; }
extern "C" hipError_t fdet_launch_diag_response(int, int, const double*, const double*, const double*, double*, hipStream_t) { return hipSuccess; }
extern "C" hipError_t fdet_launch_hmc(int, const fdet::HmcProb*, int, int64_t, double*, const double*, const double*, double, double, double*, double*, const int32_t*, int32_t*, int, hipStream_t) { return hipSuccess; }

static int check(const char* name, std::vector<fd_problem> p, fd_options oo, int what, bool verbose) {
  Opts o = resolve(&oo, p.data(), (int)p.size(), what);
  // the single-launch planner (switched off in the library's entry points)
  // is built and checked on every plan here, on the host only
  o.flags |= FD_SINGLE_LAUNCH;
  Plan pl;
  build_plan(p.data(), (int)p.size(), o, what, (char*)0x10000000, pl);
  Plan sizing;
  build_plan(p.data(), (int)p.size(), o, what, nullptr, sizing);
  int bad = 0;
  // every workspace pointer of every item stays inside [base + desc, base + total)
  {
    const char* lo = (const char*)0x10000000 + align_up(pl.desc_bytes);
    const char* hi = (const char*)0x10000000 + pl.total;
    auto in = [&](const void* p, size_t bytes) { return (const char*)p >= lo && (const char*)p + bytes <= hi; };
    for (auto& P : pl.probs) {
      const size_t eb = (size_t)P.Np * P.Np * sizeof(double);
      if (!in(P.E, eb)) { printf(" [E out]"); bad++; }
      if (P.Einv && !in(P.Einv, eb)) { printf(" [Einv out]"); bad++; }
    }
    for (auto& ph : pl.phases) for (auto& it : ph) {
      const Prob& P = pl.probs[it.prob];
      const size_t ub = (size_t)4 * P.Np * P.Np * sizeof(double) + (size_t)P.Np * sizeof(double);
      for (const Udv* u : {&it.a, &it.b, &it.o}) {
        if (!u->X) continue;
        if (!in(u->X, ub) || u->T != u->X + (size_t)2 * P.Np * P.Np || u->D != u->X + (size_t)4 * P.Np * P.Np) { printf(" [udv out]"); bad++; }
      }
      if (it.scr && !in(it.scr, scratch_bytes(P.Np))) { printf(" [scr out]"); bad++; }
      if (it.t0 < 0 || it.t1 < it.t0 || it.t1 > P.Nt || it.nb < 0 || it.nb > P.Nt) { printf(" [rows out]"); bad++; }
      if (it.kind != fdet::IK_EXPM && it.kind != fdet::IK_EXPORT && it.kind != fdet::IK_CLOSE && !it.scr) { printf(" [no scr]"); bad++; }
    }
    if (pl.total > sizing.total) { printf(" [total > sized]"); bad++; }
    if (fd_workspace_bytes(p.data(), (int)p.size(), &oo, what) == 0) { printf(" [sizing failed]"); bad++; }
  }
  if (what == FD_WHAT_FORCE) printf("%s: schedule g=%d ", name, force_schedule(p.data(), (int)p.size(), o));
  else printf("%s: ", name);
  printf("phases:");
  for (auto& ph : pl.phases) {
    printf(" %s%zu", ph.empty() ? "?" : (const char*[]){"E","C","M","Z","F","X"}[ph[0].kind], ph.size());
    std::map<double*, int> scr, wr;
    std::set<double*> rd;
    for (auto& it : ph) {
      if (it.scr && ++scr[it.scr] > 1 && !(it.kind == fdet::IK_CHAIN && it.t0 == it.t1)) { printf(" [shared scr]"); bad++; }
      if (it.kind == fdet::IK_COMBINE) {
        double* w = it.o.X ? it.o.X : it.a.X;
        if (++wr[w] > 1) { printf(" [double write]"); bad++; }
        rd.insert(it.a.X); rd.insert(it.b.X);
      } else if (it.kind == fdet::IK_CHAIN) {
        if (++wr[it.a.X] > 1) { printf(" [double write chain]"); bad++; }
      } else if (it.kind == fdet::IK_FORCE || it.kind == fdet::IK_CLOSE) {
        rd.insert(it.a.X); if (it.b.X) rd.insert(it.b.X);
      }
    }
    if (ph[0].kind == fdet::IK_COMBINE) {
      std::map<double*, int> writer;
      for (size_t x = 0; x < ph.size(); ++x) writer[ph[x].o.X ? ph[x].o.X : ph[x].a.X] = (int)x;
      for (size_t x = 0; x < ph.size(); ++x)
        for (double* r : {ph[x].a.X, ph[x].b.X})
          if (writer.count(r) && writer[r] != (int)x) { printf(" [write/read race]"); bad++; }
    }
    if (ph[0].kind == fdet::IK_FORCE && verbose) {
      int nl = 0;
      for (auto& it : ph) if (it.flags & fdet::IF_OUT_LOGDET) nl++;
      printf(" (logdet items %d)", nl);
    }
  }
  // single launch: the claim list holds every item once, each after the
  // items it waits for, and any two items that touch one workspace region
  // with at least one writing it are ordered by the waits (one reaches the
  // other).  The region rules here are restated from the kernels: scratch is
  // written by its item; E / E^-1 written by the exponential and read by
  // chains and force items; a chain writes its slot; a combine reads both
  // operands and writes its result slot; a close writes the slot it closes
  // (its T is free storage); a force item reads its two factors.
  if (pl.single) {
    size_t total = 0;
    for (auto& ph : pl.phases) total += ph.size();
    const int n = (int)pl.order.size();
    if ((size_t)n != total) { printf(" [order size]"); bad++; }
    for (int k = 0; k < n; ++k) {
      const Item& it = pl.order[k];
      if (it.dep0 < 0 || it.ndep < 0 || (size_t)(it.dep0 + it.ndep) > pl.deps.size()) { printf(" [dep range]"); bad++; continue; }
      for (int d = 0; d < it.ndep; ++d)
        if (pl.deps[it.dep0 + d] < 0 || pl.deps[it.dep0 + d] >= k) { printf(" [dep not earlier]"); bad++; }
    }
    if (pl.grid < 1 || pl.grid > n) { printf(" [grid]"); bad++; }
    // reachability over the claim list (bitsets)
    const int words = (n + 63) / 64;
    std::vector<uint64_t> reach((size_t)n * words, 0);
    for (int k = 0; k < n; ++k) {
      uint64_t* rk = &reach[(size_t)k * words];
      const Item& it = pl.order[k];
      for (int d = 0; d < it.ndep; ++d) {
        const int q = pl.deps[it.dep0 + d];
        if (q < 0 || q >= k) continue;
        const uint64_t* rq = &reach[(size_t)q * words];
        for (int w = 0; w < words; ++w) rk[w] |= rq[w];
        rk[q / 64] |= 1ull << (q % 64);
      }
    }
    auto regions = [&](const Item& it, std::vector<std::pair<const void*, bool>>& r) {
      const Prob& P = pl.probs[it.prob];
      r.clear();
      if (it.scr && !(it.kind == fdet::IK_CHAIN && it.t0 == it.t1)) r.push_back({it.scr, true});
      if (it.kind == fdet::IK_EXPM) r.push_back({it.sign > 0 ? (const void*)P.E : (const void*)P.Einv, true});
      if (it.kind == fdet::IK_CHAIN) { r.push_back({P.E, false}); r.push_back({it.a.X, true}); }
      if (it.kind == fdet::IK_COMBINE) { r.push_back({it.a.X, false}); r.push_back({it.b.X, false}); r.push_back({it.o.X ? it.o.X : it.a.X, true}); }
      if (it.kind == fdet::IK_CLOSE) r.push_back({it.a.X, true});
      if (it.kind == fdet::IK_FORCE) { r.push_back({it.a.X, false}); r.push_back({it.b.X, false}); r.push_back({P.E, false}); if (P.Einv) r.push_back({P.Einv, false}); }
      if (it.kind == fdet::IK_EXPORT) r.push_back({it.a.X, false});
    };
    std::map<const void*, std::vector<std::pair<int, bool>>> users;
    std::vector<std::pair<const void*, bool>> r;
    for (int k = 0; k < n; ++k) {
      regions(pl.order[k], r);
      for (auto& x : r) users[x.first].push_back({k, x.second});
    }
    long long unordered = 0;
    for (auto& u : users) {
      auto& v = u.second;
      for (size_t a = 0; a < v.size(); ++a)
        for (size_t b = a + 1; b < v.size(); ++b) {
          if (!v[a].second && !v[b].second) continue;
          int i = v[a].first, j = v[b].first;
          if (i == j) continue;
          if (i > j) std::swap(i, j);
          if (!((reach[(size_t)j * words + i / 64] >> (i % 64)) & 1ull)) unordered++;
        }
    }
    if (unordered) { printf(" [unordered conflicts %lld]", unordered); bad++; }
    if (verbose) printf(" single: %d items, %zu waits, grid %d", n, pl.deps.size(), pl.grid);
  }
  printf("  %s\n", bad ? "BAD" : "ok");
  return bad;
}

int main() {
  static double dummy[8];
  auto prob = [&](int N, int Nt, double dk) { fd_problem q; q.N = N; q.Nt = Nt; q.dk = dk; q.K = dummy; q.phi = dummy; return q; };
  int bad = 0;
  fd_options o{}; 
  o = fd_options{8, 16, 0, 0};
  bad += check("force_L8 (N128 Nt256 c16)", {prob(128, 256, 0.125)}, o, FD_WHAT_FORCE, true);
  std::vector<fd_problem> hmc(32, prob(512, 512, 0.125));
  o = fd_options{16, 16, 0, 0};
  bad += check("hmc 32x(N512 Nt512 c16)", hmc, o, FD_WHAT_FORCE, true);
  bad += check("L16 test 2x", std::vector<fd_problem>(2, prob(512, 512, 0.125)), o, FD_WHAT_FORCE, true);
  for (int nt : {300, 301, 256}) {
    o = fd_options{4, 1, 0, 0};
    char nm[64]; snprintf(nm, 64, "grouped Nt=%d c=1", nt);
    bad += check(nm, {prob(8, nt, 0.1)}, o, FD_WHAT_FORCE, true);
    o.flags = FD_FORCE_SCANS;
    snprintf(nm, 64, "grouped Nt=%d c=1 SCANS", nt);
    bad += check(nm, {prob(8, nt, 0.1)}, o, FD_WHAT_FORCE, true);
  }
  o = fd_options{4, 1, 0, 0};
  bad += check("6x100 c=1", std::vector<fd_problem>(6, prob(8, 100, 0.1)), o, FD_WHAT_FORCE, true);
  for (int nt = 1; nt <= 70; ++nt) for (int c : {1, 3, 8, 16}) {
    o = fd_options{4, c, 0, 0};
    char nm[64]; snprintf(nm, 64, "Nt=%d c=%d", nt, c);
    bad += check(nm, {prob(18, nt, 0.1)}, o, FD_WHAT_FORCE, false);
    o.flags = FD_FORCE_SCANS;
    bad += check(nm, {prob(18, nt, 0.1)}, o, FD_WHAT_FORCE, false);
  }
  for (int ns_nt : {1, 2, 3, 5, 8, 13, 16, 40, 100, 256}) for (int s : {1, 4, 8}) {
    o = fd_options{s, 1, 0, 0};
    char nm[64]; snprintf(nm, 64, "det N72 Nt=%d s=%d", ns_nt, s);
    bad += check(nm, {prob(72, ns_nt, 0.1)}, o, FD_WHAT_LOGDET, false);
    bad += check(nm, std::vector<fd_problem>(7, prob(40, ns_nt, 0.1)), o, FD_WHAT_GREENS, false);
  }
  // FD_KEEP_CHECKPOINTS: the force call's items read only workspace slots
  // that the log det call's items write (same layout), and E / E^-1
  for (int nt : {16, 90, 256}) for (int c : {4, 16}) for (int sc : {0, (int)FD_FORCE_SCANS}) {
    fd_options ok{4, c, 0, FD_KEEP_CHECKPOINTS | sc};
    std::vector<fd_problem> v = {prob(72, nt, 0.1), prob(18, nt / 2 + 1, 0.1)};
    Opts oo = resolve(&ok, v.data(), 2, FD_WHAT_FORCE);
    Plan fw, bw;
    build_plan(v.data(), 2, oo, FD_WHAT_LOGDET, (char*)0x10000000, fw);
    build_plan(v.data(), 2, oo, FD_WHAT_FORCE, (char*)0x10000000, bw);
    std::set<const void*> written;
    for (auto& ph : fw.phases) for (auto& it : ph) {
      if (it.kind == fdet::IK_CHAIN) written.insert(it.a.X);
      if (it.kind == fdet::IK_COMBINE) written.insert(it.o.X ? it.o.X : it.a.X);
      if (it.kind == fdet::IK_EXPM) written.insert(it.sign > 0 ? (const void*)fw.probs[it.prob].E : (const void*)fw.probs[it.prob].Einv);
    }
    int b = 0;
    if (bw.phases.size() != 1 || bw.total != fw.total) b++;
    for (auto& it : bw.phases.front()) {
      if (it.kind != fdet::IK_FORCE) b++;
      if (!written.count(it.a.X) || !written.count(it.b.X)) b++;
      if (!written.count(bw.probs[it.prob].E) || !written.count(bw.probs[it.prob].Einv)) b++;
    }
    printf("keep Nt=%d c=%d scans=%d: %zu forward phases, %zu force items %s\n", nt, c, sc ? 1 : 0,
           fw.phases.size(), bw.phases.front().size(), b ? "BAD" : "ok");
    bad += b;
  }
  // the product-form Taylor coefficients: prod_k (1 + gamma_k x) multiplied
  // out must give the coefficients 1 / j! of the degree-n Taylor polynomial
  for (int n = 1; n <= fdet::kMaxTaylor; ++n) {
    const std::vector<std::complex<double>> g = taylor_product_coefficients(n);
    std::vector<std::complex<double>> c(n + 1, 0.0);
    c[0] = 1.0;
    for (int k = 0; k < n; ++k)
      for (int j = k + 1; j >= 1; --j) c[j] += g[k] * c[j - 1];
    double err = 0.0, fact = 1.0;
    for (int j = 0; j <= n; ++j) {
      if (j > 0) fact *= j;
      err = std::max(err, std::abs(c[j] - 1.0 / fact));
    }
    const int b = (int)g.size() != n || !(err < 1e-13);
    printf("taylor n=%d: max coefficient error %.2e %s\n", n, err, b ? "BAD" : "ok");
    bad += b;
  }
  // matrix-free slices: no exponential phase, one SparseOp per problem inside
  // the descriptor region carrying gamma_k dk, chunks short enough for the
  // phase staging (ns N <= Np^2)
  for (int nt : {1, 7, 64, 300}) for (int s : {1, 5, 16}) {
    std::vector<fd_problem> v = {prob(72, nt, 0.1), prob(8, nt + 3, 0.2), prob(512, nt, 0.125)};
    fd_options oo{s, 0, 0, 0};
    int32_t cols[1] = {0};
    double vals[1] = {0.0};
    std::vector<fd_ell> h(3, fd_ell{3, cols, vals});
    Opts r = resolve(&oo, v.data(), 3, FD_WHAT_GREENS);
    Plan pl, sz;
    build_plan(v.data(), 3, r, FD_WHAT_GREENS, (char*)0x10000000, pl, h.data(), 4);
    build_plan(v.data(), 3, r, FD_WHAT_GREENS, nullptr, sz, h.data(), 4);
    std::vector<size_t> first;
    std::vector<char> host = pack_descriptors(pl, first);
    int b = 0;
    if (pl.total != sz.total || pl.sops.size() != 3) b++;
    const std::vector<std::complex<double>> g = taylor_product_coefficients(4);
    for (int i = 0; i < 3; ++i) {
      const char* at = (const char*)pl.probs[i].sp;
      if (at != (const char*)0x10000000 + pl.sops_off + i * sizeof(fdet::SparseOp)) b++;
      if (pl.sops_off + 3 * sizeof(fdet::SparseOp) > pl.desc_bytes) b++;
      fdet::SparseOp so;
      std::memcpy(&so, host.data() + pl.sops_off + i * sizeof(fdet::SparseOp), sizeof so);
      if (so.n != 4 || so.q != 3 || so.col != cols || so.val != vals) b++;
      for (int k = 0; k < 4; ++k)
        if (so.gr[k] != g[k].real() * v[i].dk || so.gi[k] != g[k].imag() * v[i].dk) b++;
    }
    for (auto& ph : pl.phases) for (auto& it : ph) {
      if (it.kind == fdet::IK_EXPM) b++;
      const int Np = pl.probs[it.prob].Np;
      if (it.kind == fdet::IK_CHAIN && (long)std::min(it.s, it.t1 - it.t0) * pl.probs[it.prob].N > (long)Np * Np) b++;
    }
    printf("sparse Nt=%d s=%d: %zu phases %s\n", nt, s, pl.phases.size(), b ? "BAD" : "ok");
    bad += b;
  }
  // random batches of every kind
  {
    std::mt19937 g(12345);
    auto U = [&](int a, int b) { return std::uniform_int_distribution<int>(a, b)(g); };
    int nrun = 0;
    for (int trial = 0; trial < 400; ++trial) {
      const int nprob = U(1, 12);
      std::vector<fd_problem> ps;
      const int big = U(0, 3) == 0;
      for (int i = 0; i < nprob; ++i) ps.push_back(prob(big ? U(1, 512) : U(1, 128), U(1, 300), 0.05));
      const int what = U(0, 3);
      fd_options oo{std::vector<int>{1, 2, 4, 8, 16}[U(0, 4)], U(1, 32), U(0, 1) ? 0 : U(1, 40), U(0, 3) == 0 ? FD_FORCE_SCANS : 0};
      char nm[64]; snprintf(nm, 64, "fuzz %d what=%d nprob=%d", trial, what, nprob);
      const int b = check(nm, ps, oo, what, false);
      bad += b;
      ++nrun;
    }
    printf("fuzz runs %d\n", nrun);
  }
  printf("bad %d\n", bad);
  return bad != 0;
}
