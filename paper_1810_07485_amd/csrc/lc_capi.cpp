// lc_capi.cpp -- engine and C ABI of the loop-cluster library (host side).
//
// A chain owns its world lines (double-buffered spins and kept-operator
// lists on the device).  An engine (a chain run alone, or a batch) queues one
// sweep of its chains as a fixed sequence of kernel launches over flat index
// spaces (lc_kernels.hip), optionally captured once as a HIP graph.  The
// large per-sweep scratch (operators, parent words, loop records) lives in an
// arena shared by every engine on the same stream and allocator: sweeps on
// one stream run one after another, so the arena is sized for the largest
// engine instead of the sum, and a buffer that moves invalidates the graphs
// captured with it (generation counter).  The host reads back one small record per sweep: the exact integer
// statistics and an overflow flag.  On overflow the scratch or the chain
// buffers grow and the same sweep is run again; its random numbers are
// addressed by (seed, sweep, entity), so the replay is bit-identical.
#include "lc.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "lc_kernels.h"
#include "lc_static.h"

using lc::ChainDesc;
using lc::ChainDyn;

typedef unsigned __int128 u128;

namespace {

constexpr int kDefaultGrid = 8192;  // 256 CUs x 32 workgroups: latency-bound loops
constexpr int kRing = 64;           // sweeps per host synchronisation
constexpr int kAccWords = LC_ACC_WORDS;

// LC_VERBOSE=1 in the environment traces scratch growth and failed
// allocations on stderr.
bool verbose() {
  static const bool v = [] {
    const char* e = std::getenv("LC_VERBOSE");
    return e && *e && *e != '0';
  }();
  return v;
}

struct Mem {
  lc_alloc a{};
  bool user = false;
  hipStream_t s = nullptr;
  void* get(size_t bytes) const {
    if (bytes < 8) bytes = 8;
    void* p = nullptr;
    if (user)
      p = a.alloc(bytes, s, a.ctx);
    else if (hipMalloc(&p, bytes) != hipSuccess)
      p = nullptr;
    if (!p && verbose()) std::fprintf(stderr, "[lc] allocation of %zu bytes failed\n", bytes);
    return p;
  }
  void put(void* p, size_t bytes) const {
    if (!p) return;
    if (bytes < 8) bytes = 8;
    if (user)
      a.free(p, bytes, s, a.ctx);
    else
      (void)hipFree(p);
  }
  bool same(const Mem& o) const {
    return user == o.user && s == o.s &&
           (!user || (a.alloc == o.a.alloc && a.free == o.a.free && a.ctx == o.a.ctx));
  }
};

template <class T>
struct DBuf {
  T* p = nullptr;
  size_t n = 0;
  bool ensure(const Mem& m, size_t want, bool keep = false, hipStream_t s = nullptr) {
    if (want <= n && p) return true;
    T* q = static_cast<T*>(m.get(want * sizeof(T)));
    if (!q) return false;
    if (keep && p && n) {
      if (hipMemcpyAsync(q, p, n * sizeof(T), hipMemcpyDeviceToDevice, s) != hipSuccess ||
          hipStreamSynchronize(s) != hipSuccess) {
        m.put(q, want * sizeof(T));
        return false;
      }
    }
    release(m);
    p = q;
    n = want;
    return true;
  }
  void release(const Mem& m) {
    m.put(p, n * sizeof(T));
    p = nullptr;
    n = 0;
  }
};

// Poisson window rule (library host code): 2^w windows per bond with
// w the smallest w >= 0 such that beta / 2^w <= 8; per window the count of
// candidates of a rate-1/2 process is Poisson with mean mu = beta / 2^(w+1);
// T[i] = floor(P(n <= i) 2^64), last entry 2^64 - 1.
int window_rule(double beta, int* w_out, double* mu_out, uint64_t* T, int* K) {
  if (!(beta > 0.0) || !std::isfinite(beta) || beta > 8.0 * 4294967296.0) return LC_EINVAL;
  int w = 0;
  while (beta > std::ldexp(8.0, w)) ++w;
  const double mu = std::ldexp(beta, -w - 1);
  double term = std::exp(-mu);
  double cdf = term;
  double before = -1.0;
  int k = 0;
  for (; k < lc::kMaxTable; ++k) {
    if (k > 0) {
      const double num = term * mu;
      term = num / static_cast<double>(k);
      const double next = cdf + term;
      cdf = next;
    }
    if (cdf >= 1.0 || k == lc::kMaxTable - 1 || cdf == before) {
      T[k] = ~uint64_t(0);
      break;
    }
    T[k] = static_cast<uint64_t>(cdf * 18446744073709551616.0);
    before = cdf;
  }
  *w_out = w;
  *mu_out = mu;
  *K = k + 1;
  return LC_OK;
}

struct Accum {
  int64_t n = 0;
  u128 ops = 0, m2 = 0, ma2 = 0, n02 = 0, len2 = 0, clusters = 0;
};

// Per-sweep scratch shared by the engines of one stream and allocator.
struct Arena {
  Mem mem;
  int refs = 0;
  uint64_t gen = 1;   // bumped whenever a buffer is reallocated
  uint64_t runs = 0;  // bumped by every group of sweeps (export validity)
  std::mutex mu;      // one engine at a time
  DBuf<int64_t> opstart, kflat, parent, rcnt, xedge, frag;
  DBuf<uint64_t> optime;
  DBuf<uint8_t> optype;
  DBuf<uint32_t> accmask;
  DBuf<unsigned long long> acc, bacc;
  int64_t op_cap = 0, node_cap = 0, root_cap = 0, xcap = 0, fcap = 0;

  void release_all() {
    opstart.release(mem);
    kflat.release(mem);
    parent.release(mem);
    rcnt.release(mem);
    xedge.release(mem);
    frag.release(mem);
    optime.release(mem);
    optype.release(mem);
    accmask.release(mem);
    acc.release(mem);
    bacc.release(mem);
    op_cap = node_cap = root_cap = xcap = fcap = 0;
    ++gen;
  }
  // grow b to hold want elements; a move bumps the generation
  template <class T>
  bool grow(DBuf<T>& b, size_t want) {
    if (want <= b.n && b.p) return true;
    if (verbose())
      std::fprintf(stderr, "[lc] arena %p: buffer %zu -> %zu bytes (total before %.3f GB)\n",
                   static_cast<void*>(this), b.n * sizeof(T), want * sizeof(T), bytes() / 1e9);
    b.release(mem);
    ++gen;
    return b.ensure(mem, want);
  }
  double bytes() const {
    return 8.0 * (opstart.n + kflat.n + parent.n + rcnt.n + xedge.n + frag.n + optime.n + acc.n +
                  bacc.n) +
           static_cast<double>(optype.n) + 4.0 * accmask.n;
  }
};

std::mutex g_arena_mu;
std::vector<Arena*> g_arenas;

Arena* arena_get(const Mem& m) {
  std::lock_guard<std::mutex> g(g_arena_mu);
  for (Arena* a : g_arenas)
    if (a->mem.same(m)) {
      ++a->refs;
      return a;
    }
  Arena* a = new (std::nothrow) Arena();
  if (!a) return nullptr;
  a->mem = m;
  a->refs = 1;
  g_arenas.push_back(a);
  return a;
}

void arena_put(Arena* a) {
  if (!a) return;
  std::lock_guard<std::mutex> g(g_arena_mu);
  if (--a->refs > 0) return;
  g_arenas.erase(std::find(g_arenas.begin(), g_arenas.end(), a));
  (void)hipStreamSynchronize(a->mem.s);
  a->release_all();
  delete a;
}

}  // namespace

struct Engine;

struct lc_chain {
  int64_t L = 0;
  int two_s = 1;
  double beta = 0;
  uint64_t seed = 0;
  int w = 0;
  double mu = 0;
  uint64_t T[lc::kMaxTable] = {};
  int K = 0;
  int64_t n_sites = 0, n_bonds = 0, nwin = 0, nbn = 0;
  int tile_j = 1, tile_k = 1, tile_shrink = 0;  // linking tile (spins x windows)
  int tile_kmax = 0, tile_target = 0;            // tile shape preference (0: default)
  int flip_rule = LC_FLIP_LABEL;
  int64_t ntj = 1, ntk = 1;
  Mem mem;
  hipStream_t stream = nullptr;
  DBuf<uint8_t> s0[2];
  DBuf<int64_t> kstart[2];
  DBuf<uint64_t> ktime[2];
  DBuf<int64_t> perm;
  int64_t kept_cap = 0;
  int64_t n_kept = 0;  // host mirror of the current kept count
  int cur = 0;
  uint32_t sweep = 0;
  Accum acc;
  lc_sweep_stats last{};
  bool has_last = false;
  Engine* own = nullptr;     // engine used when run alone
  lc_batch* batch = nullptr; // batch membership
  Engine* last_engine = nullptr;
  int last_index = 0;
  uint64_t last_run = 0;  // arena run that holds this chain's last sweep
};

struct Engine {
  Mem mem;
  hipStream_t stream = nullptr;
  Arena* ar = nullptr;  // shared per-sweep scratch
  std::vector<lc_chain*> chains;
  bool dirty = true;
  int grid = kDefaultGrid;
  bool use_graph = true;
  // per-chain small arrays
  DBuf<ChainDesc> descs;
  DBuf<int64_t> win_bases, site_bases, spin_bases, op_bases, node_bases;
  DBuf<ChainDyn> dyn;
  DBuf<int64_t> totals, scan_tmp, bn_bases, grp_tile_base;
  DBuf<int> grp_chain;
  DBuf<unsigned long long> dyncnt;
  std::vector<LcTileGroup> groups;
  DBuf<uint64_t> stats;
  DBuf<uint32_t> flags, ring_ctr;
  DBuf<unsigned long long> ring;
  int64_t nwin = 0, nsites = 0, nspins = 0, sum_nbn = 0, sum_xe = 0, sum_fe = 0;
  bool any_split = false;
  hipGraphExec_t gexec = nullptr;
  bool graph_ok = false;
  uint64_t graph_gen = 0;  // arena generation the graph was captured with
  std::vector<unsigned long long> hring;
  // per-phase timing (HIP events between the kernels of each sweep)
  bool profiling = false;
  std::vector<hipEvent_t> ev;
  std::vector<double> ph_ms;
  int64_t ph_sweeps = 0;

  void drop_events() {
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    ev.clear();
  }

  void drop_graph() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    gexec = nullptr;
    graph_ok = false;
  }
  void release_all() {
    drop_graph();
    drop_events();
    descs.release(mem);
    win_bases.release(mem);
    site_bases.release(mem);
    spin_bases.release(mem);
    op_bases.release(mem);
    node_bases.release(mem);
    dyn.release(mem);
    totals.release(mem);
    scan_tmp.release(mem);
    bn_bases.release(mem);
    grp_tile_base.release(mem);
    grp_chain.release(mem);
    dyncnt.release(mem);
    stats.release(mem);
    flags.release(mem);
    ring_ctr.release(mem);
    ring.release(mem);
    arena_put(ar);
    ar = nullptr;
  }
};

struct lc_batch {
  Engine eng;
  bool owns_stream = false;
};

namespace {

int hip_err(hipError_t e) { return e == hipSuccess ? LC_OK : LC_EDEVICE; }

ChainDesc make_desc(const lc_chain* c, int64_t win_base, int64_t site_base, int64_t spin_base,
                    int64_t bnode_base) {
  ChainDesc d;
  std::memset(&d, 0, sizeof(d));
  d.seed = c->seed;
  d.L = c->L;
  d.n_sites = c->n_sites;
  d.n_bonds = c->n_bonds;
  d.nbn = c->nbn;
  d.win_base = win_base;
  d.site_base = site_base;
  d.spin_base = spin_base;
  d.bnode_base = bnode_base;
  d.kept_cap = c->kept_cap;
  for (int q = 0; q < 2; ++q) {
    d.s0[q] = c->s0[q].p;
    d.kstart[q] = c->kstart[q].p;
    d.ktime[q] = c->ktime[q].p;
  }
  d.perm = c->perm.p;
  d.two_s = c->two_s;
  d.w = c->w;
  d.K = c->K;
  d.sweep = c->sweep;
  d.cur = c->cur;
  d.tile_j = c->tile_j;
  d.flip_rule = c->flip_rule;
  d.tile_k = c->tile_k;
  d.ntj = c->ntj;
  std::memcpy(d.T, c->T, sizeof(d.T));
  return d;
}

// Edges between linking tiles and open fragments per operator: with tiles of
// 64 spins x 4 windows about one operator in twelve has an edge leaving its
// tile at S = 1/2; split-spin tiles span few spins (2S bonds wide at each
// side) and about half of their operators do.  Grown on overflow from the
// exact counts of the sweep.
double cross_per_op(int two_s) { return two_s == 1 ? 0.12 : 0.7; }
double frags_per_op(int two_s) { return two_s == 1 ? 0.12 : 0.7; }

// Initial kept-operator capacity per buffer: about 0.3 off-diagonal
// operators per bond and unit beta at low temperature; grown on overflow.
int64_t kept_initial(int64_t n_bonds, double beta) {
  return static_cast<int64_t>(0.36 * static_cast<double>(n_bonds) * beta) + 1024;
}

// Operator capacity of the next sweep.  Operators = kept + accepted
// <= kept + candidates (candidates ~ Poisson(beta N_b / 2)); and on average
// <N> = beta (N_b / 4 - E) <= beta (N_b / 4 + L S (S + 1)), because each
// sub-bond term is bounded below by -S(S+1) / (2S)^2.  The smaller of the two
// plus six standard deviations; a sweep that still overflows is replayed.
double ops_bound(double n_kept, double n_bonds, double L, int two_s, double beta) {
  const double cand = 0.5 * n_bonds * beta;
  const double S = 0.5 * two_s;
  const double mean_max = beta * (0.25 * n_bonds + L * S * (S + 1.0));
  const double b = std::min(n_kept + cand, mean_max);
  return b + 6.0 * std::sqrt(b + 1.0) + 1024.0;
}

int64_t ops_estimate(const lc_chain* c) {
  return static_cast<int64_t>(ops_bound(static_cast<double>(c->n_kept),
                                        static_cast<double>(c->n_bonds),
                                        static_cast<double>(c->L), c->two_s, c->beta));
}

// Arena capacity for ops operators, nodes loop-graph nodes, xe edges between
// tiles and fe fragments of an engine with nbn boundary nodes; loop records
// and root counts follow the items (fragments and boundary nodes).
int ensure_scratch(Arena& A, int64_t ops, int64_t nodes, int64_t xe, int64_t fe, int64_t nbn) {
  // A buffer that has to grow takes the need plus 1/16, and at least a
  // quarter more than it had: every move invalidates the graphs of all
  // engines sharing the arena, so slowly rising demand (chains still
  // equilibrating) must not move it on every call.
  auto target = [](int64_t need, int64_t cap) { return std::max(need + need / 16, cap + cap / 4); };
  if (A.op_cap < ops) {
    ops = target(ops, A.op_cap);
    A.op_cap = 0;
    if (!(A.grow(A.optime, ops) && A.grow(A.optype, ops))) return LC_ENOMEM;
    A.op_cap = ops;
  }
  if (A.node_cap < nodes) {
    nodes = target(nodes, A.node_cap);
    A.node_cap = 0;
    if (!A.grow(A.parent, nodes)) return LC_ENOMEM;
    A.node_cap = nodes;
  }
  if (A.xcap < xe) {
    xe = target(xe, A.xcap);
    A.xcap = 0;
    if (!A.grow(A.xedge, 2 * static_cast<size_t>(xe))) return LC_ENOMEM;
    A.xcap = xe;
  }
  if (A.fcap < fe) {
    fe = target(fe, A.fcap);
    A.fcap = 0;
    if (!A.grow(A.frag, 4 * static_cast<size_t>(fe))) return LC_ENOMEM;
    A.fcap = fe;
  }
  const int64_t items = A.fcap + nbn;
  if (A.root_cap < items) {
    const int64_t roots = target(items, A.root_cap);
    A.root_cap = 0;
    if (!A.grow(A.acc, kAccWords * static_cast<size_t>(roots))) return LC_ENOMEM;
    A.root_cap = roots;
  }
  if (!A.grow(A.rcnt, static_cast<size_t>(items / 4096 + 2))) return LC_ENOMEM;
  return LC_OK;
}

// Linking tile of a chain: spins x windows with at most LC_TILE_THREADS
// (subspin, window) walkers and LC_TILE_BONDS owned bonds, sized for about
// 1,500 operators at S = 1/2 and 1,400 for split spins by the density bound
// rho (the split-spin density is below it: about 1,300 in practice;
// LC_TILE_OPS and LC_TILE_OPS_SPLIT are the hard limits: a tile beyond one
// makes the sweep replay with tiles half as large, tile_shrink).  S = 1/2
// tiles are up to 8 windows tall: a site crosses a window boundary once, a
// tile side on about half of its events.  Split-spin tiles are one window
// tall: 2S bonds wide at each side, they need all the spins they can get.
// lc_set_tile overrides both (measured on the MI355X: 8 windows and 1,400
// were the fastest of the shapes tried at the benchmark sizes).
void choose_tile(lc_chain* c) {
  const int ts = c->two_s;
  const int64_t W = int64_t(1) << c->w;
  const double win_tau = c->beta / static_cast<double>(W);
  // operators per sub-bond and unit imaginary time: about ln 2 for S = 1/2,
  // the bound (N_b/4 + L S(S+1)) / N_b otherwise
  const double rho = ts == 1 ? 0.72 : (ts + 1.0) / (2.0 * ts);
  const double per_spin_window = std::max(rho * ts * ts * win_tau, 1e-9);
  const double base = c->tile_target > 0 ? c->tile_target : (ts == 1 ? 1500.0 : 1400.0);
  const double target = base / static_cast<double>(int64_t(1) << c->tile_shrink);
  int64_t tk = std::min<int64_t>(W, c->tile_kmax > 0 ? c->tile_kmax : (ts == 1 ? 8 : 1));
  // split spins: the walk's event lists hold 2 (2S) runs per walker, at most
  // 2 LC_TILE_BONDS runs: (2S)^2 bonds per spin times the windows
  while (tk > 1 && ts > 1 && ts * ts * tk > LC_TILE_BONDS) tk >>= 1;
  while (tk > 1 && per_spin_window * static_cast<double>(tk) > target) tk >>= 1;
  int64_t tj = static_cast<int64_t>(target / (per_spin_window * static_cast<double>(tk)));
  tj = std::min<int64_t>(tj, LC_TILE_THREADS / (ts * tk));
  tj = std::min<int64_t>(tj, LC_TILE_BONDS / (ts * ts * (ts > 1 ? tk : 1)));
  tj = std::min<int64_t>(tj, c->L);
  tj = std::max<int64_t>(tj, 1);
  c->tile_j = static_cast<int>(tj);
  c->tile_k = static_cast<int>(tk);
  c->ntj = (c->L + tj - 1) / tj;
  c->ntk = (W + tk - 1) / tk;
}

int layout(Engine& E) {
  const int n = static_cast<int>(E.chains.size());
  std::vector<ChainDesc> h(n);
  std::vector<int64_t> wb(n), sb(n), pb(n), bb(n), tb;
  std::vector<int> gc;
  int64_t nwin = 0, nsites = 0, nspins = 0, nbn = 0, ops = 0, xe = 0, fe = 0;
  bool split = false;
  for (int i = 0; i < n; ++i) {
    lc_chain* c = E.chains[i];
    choose_tile(c);
    h[i] = make_desc(c, nwin, nsites, nspins, nbn);
    wb[i] = nwin;
    sb[i] = nsites;
    pb[i] = nspins;
    bb[i] = nbn;
    nwin += c->nwin;
    nsites += c->n_sites;
    nspins += c->L;
    nbn += c->nbn;
    const int64_t o = ops_estimate(c);
    ops += o;
    xe += static_cast<int64_t>(cross_per_op(c->two_s) * static_cast<double>(o)) + 4096;
    fe += static_cast<int64_t>(frags_per_op(c->two_s) * static_cast<double>(o)) + 4096;
    split = split || c->two_s > 1;
  }
  // one tile group per spin length present
  E.groups.clear();
  for (int ts = 1; ts <= LC_MAX_TS; ++ts) {
    LcTileGroup g{ts, 0, static_cast<int>(gc.size()), 0};
    for (int i = 0; i < n; ++i) {
      const lc_chain* c = E.chains[i];
      if (c->two_s != ts) continue;
      gc.push_back(i);
      tb.push_back(g.ntiles);
      g.ntiles += c->ntj * c->ntk;
      g.nchain += 1;
    }
    if (g.nchain) E.groups.push_back(g);
  }
  const Mem& m = E.mem;
  const size_t nc = static_cast<size_t>(std::max(n, 1));
  bool ok = E.descs.ensure(m, nc) && E.win_bases.ensure(m, nc) && E.site_bases.ensure(m, nc) &&
            E.spin_bases.ensure(m, nc) && E.op_bases.ensure(m, nc) && E.node_bases.ensure(m, nc) &&
            E.bn_bases.ensure(m, nc) && E.grp_chain.ensure(m, nc) && E.grp_tile_base.ensure(m, nc) &&
            E.dyncnt.ensure(m, 4) &&
            E.dyn.ensure(m, nc) && E.totals.ensure(m, 2) && E.scan_tmp.ensure(m, LC_SCAN_BLOCKS + 1) &&
            E.stats.ensure(m, nc * lc::ST_WORDS * (1 + LC_STAT_STRIPES)) && E.flags.ensure(m, 2) && E.ring_ctr.ensure(m, 2) &&
            E.ring.ensure(m, static_cast<size_t>(kRing) * (nc * lc::ST_WORDS + 1));
  if (!ok) return LC_ENOMEM;
  Arena& A = *E.ar;
  ok = A.grow(A.opstart, static_cast<size_t>(nwin) + 1) && A.grow(A.kflat, static_cast<size_t>(nwin) + 1) &&
       A.grow(A.accmask, static_cast<size_t>(std::max<int64_t>(nwin, 1))) &&
       A.grow(A.bacc, static_cast<size_t>(std::max<int64_t>(nsites, 1)));
  if (!ok) return LC_ENOMEM;
  int rc = ensure_scratch(A, ops, nbn + 2 * ops, xe, fe, nbn);
  if (rc != LC_OK) return rc;
  E.nwin = nwin;
  E.nsites = nsites;
  E.nspins = nspins;
  E.sum_nbn = nbn;
  E.sum_xe = xe;
  E.sum_fe = fe;
  E.any_split = split;
  if (n > 0) {
    hipStream_t s = E.stream;
    if (hipMemcpyAsync(E.descs.p, h.data(), n * sizeof(ChainDesc), hipMemcpyHostToDevice, s) ||
        hipMemcpyAsync(E.win_bases.p, wb.data(), n * sizeof(int64_t), hipMemcpyHostToDevice, s) ||
        hipMemcpyAsync(E.site_bases.p, sb.data(), n * sizeof(int64_t), hipMemcpyHostToDevice, s) ||
        hipMemcpyAsync(E.spin_bases.p, pb.data(), n * sizeof(int64_t), hipMemcpyHostToDevice, s) ||
        hipMemcpyAsync(E.bn_bases.p, bb.data(), n * sizeof(int64_t), hipMemcpyHostToDevice, s) ||
        hipMemcpyAsync(E.grp_chain.p, gc.data(), n * sizeof(int), hipMemcpyHostToDevice, s) ||
        hipMemcpyAsync(E.grp_tile_base.p, tb.data(), n * sizeof(int64_t), hipMemcpyHostToDevice, s) ||
        hipStreamSynchronize(s))
      return LC_EDEVICE;
  }
  for (int i = 0; i < n; ++i) {
    E.chains[i]->last_engine = nullptr;
  }
  E.hring.assign(static_cast<size_t>(kRing) * (nc * lc::ST_WORDS + 1), 0);
  E.drop_graph();
  E.dirty = false;
  return LC_OK;
}

// Grow the arena, if needed, to the engine's current per-sweep bound
// (kept + candidates per chain, from the host mirror of the kept counts) and
// to at least the given counts.
int ensure_capacity(Engine& E, int64_t at_least_ops, int64_t at_least_xe = 0, int64_t at_least_fe = 0) {
  int64_t ops = 0, xe = 0, fe = 0;
  for (lc_chain* c : E.chains) {
    const int64_t o = ops_estimate(c);
    ops += o;
    xe += static_cast<int64_t>(cross_per_op(c->two_s) * static_cast<double>(o)) + 4096;
    fe += static_cast<int64_t>(frags_per_op(c->two_s) * static_cast<double>(o)) + 4096;
  }
  ops = std::max(ops, at_least_ops);
  xe = std::max(xe, at_least_xe);
  fe = std::max(fe, at_least_fe);
  return ensure_scratch(*E.ar, ops, E.sum_nbn + 2 * ops, xe, fe, E.sum_nbn);
}

LcSweepArgs sweep_args(Engine& E) {
  LcSweepArgs A;
  A.descs = E.descs.p;
  A.win_bases = E.win_bases.p;
  A.site_bases = E.site_bases.p;
  A.spin_bases = E.spin_bases.p;
  A.nchain = static_cast<int>(E.chains.size());
  A.any_split = E.any_split ? 1 : 0;
  A.bn_bases = E.bn_bases.p;
  A.nwin = E.nwin;
  A.nsites = E.nsites;
  A.nspins = E.nspins;
  A.nbn = E.sum_nbn;
  A.ngroups = static_cast<int>(E.groups.size());
  for (int g = 0; g < A.ngroups; ++g) A.groups[g] = E.groups[g];
  A.grp_chain = E.grp_chain.p;
  A.grp_tile_base = E.grp_tile_base.p;
  A.grid_blocks = E.grid;
  const Arena& R = *E.ar;
  A.opstart = R.opstart.p;
  A.accmask = R.accmask.p;
  A.kflat = R.kflat.p;
  A.optime = R.optime.p;
  A.optype = R.optype.p;
  A.parent = R.parent.p;
  A.xedge = R.xedge.p;
  A.frag = R.frag.p;
  A.xcap = R.xcap;
  A.fcap = R.fcap;
  A.dyncnt = E.dyncnt.p;
  A.acc = R.acc.p;
  A.bacc = R.bacc.p;
  A.root_cap = R.root_cap;
  A.rcnt = R.rcnt.p;
  A.op_cap = R.op_cap;
  A.node_cap = R.node_cap;
  A.dyn = E.dyn.p;
  A.op_bases = E.op_bases.p;
  A.node_bases = E.node_bases.p;
  A.totals = E.totals.p;
  A.scan_tmp = E.scan_tmp.p;
  A.stats = E.stats.p;
  A.flags = E.flags.p;
  A.ring = E.ring.p;
  A.ring_ctr = E.ring_ctr.p;
  A.ring_cap = kRing;
  A.events = E.profiling ? reinterpret_cast<void**>(E.ev.data()) : nullptr;
  return A;
}

int launch_one(Engine& E) {
  if (E.profiling) {
    if (E.ev.empty()) {
      E.ev.resize(LC_PH_COUNT + 1);
      for (auto& e : E.ev)
        if (hipEventCreate(&e) != hipSuccess) return LC_EDEVICE;
    }
    return hip_err(lc_launch_sweep(sweep_args(E), E.stream));
  }
  if (E.use_graph) {
    if (E.graph_ok && E.graph_gen != E.ar->gen) E.drop_graph();
    if (!E.graph_ok) {
      hipGraph_t g = nullptr;
      if (hipStreamBeginCapture(E.stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return LC_EDEVICE;
      const hipError_t le = lc_launch_sweep(sweep_args(E), E.stream);
      const hipError_t ce = hipStreamEndCapture(E.stream, &g);
      if (le != hipSuccess || ce != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return LC_EDEVICE;
      }
      const hipError_t ie = hipGraphInstantiate(&E.gexec, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (ie != hipSuccess) return LC_EDEVICE;
      E.graph_ok = true;
      E.graph_gen = E.ar->gen;
    }
    return hip_err(hipGraphLaunch(E.gexec, E.stream));
  }
  return hip_err(lc_launch_sweep(sweep_args(E), E.stream));
}

void apply_record(lc_chain* c, const unsigned long long* st, bool accumulate) {
  lc_sweep_stats& s = c->last;
  s.sweep = c->sweep;
  s.n_cand = static_cast<int64_t>(st[lc::ST_CAND]);
  s.n_acc = static_cast<int64_t>(st[lc::ST_ACC]);
  s.n_ops = static_cast<int64_t>(st[lc::ST_OPS]);
  s.n_kept_in = static_cast<int64_t>(st[lc::ST_KEPT_IN]);
  s.n_kept_out = static_cast<int64_t>(st[lc::ST_KEPT_OUT]);
  s.n_nodes = static_cast<int64_t>(st[lc::ST_NODES]);
  s.n_clusters = static_cast<int64_t>(st[lc::ST_CLUSTERS]);
  s.sum_m2 = st[lc::ST_M2];
  s.sum_n0sq = st[lc::ST_N0SQ];
  s.sum_size2_lo = st[lc::ST_SIZE2_LO];
  s.sum_size2_hi = st[lc::ST_SIZE2_HI];
  s.sum_len2_lo = st[lc::ST_LEN2_LO];
  s.sum_len2_hi = st[lc::ST_LEN2_HI];
  s.m_after = static_cast<int64_t>(st[lc::ST_MAFTER]);
  s.max_size = static_cast<int64_t>(st[lc::ST_MAXSIZE]);
  c->has_last = true;
  c->n_kept = s.n_kept_out;
  c->cur ^= 1;
  c->sweep += 1;
  if (accumulate) {
    Accum& a = c->acc;
    a.n += 1;
    a.ops += static_cast<u128>(s.n_ops);
    a.m2 += static_cast<u128>(s.sum_m2);
    a.ma2 += static_cast<u128>(static_cast<uint64_t>(s.m_after * s.m_after));
    a.n02 += static_cast<u128>(s.sum_n0sq);
    a.len2 += (static_cast<u128>(s.sum_len2_hi) << 64) | s.sum_len2_lo;
    a.clusters += static_cast<u128>(s.n_clusters);
  }
}

// Grow chain kept buffers (both halves, keeping the current content).
int grow_kept(lc_chain* c, int64_t need) {
  const int64_t cap = std::max<int64_t>(need + need / 4 + 1024, c->kept_cap);
  for (int q = 0; q < 2; ++q)
    if (!c->ktime[q].ensure(c->mem, static_cast<size_t>(cap), q == c->cur, c->stream)) return LC_ENOMEM;
  c->kept_cap = cap;
  if (c->own) c->own->dirty = true;
  if (c->batch) c->batch->eng.dirty = true;
  return LC_OK;
}

int run_engine(Engine& E, int64_t n_sweeps, int accumulate) {
  if (n_sweeps < 0) return LC_EINVAL;
  if (E.chains.empty() || n_sweeps == 0) return LC_OK;
  std::lock_guard<std::mutex> hold(E.ar->mu);
  Arena& R = *E.ar;
  int rc;
  if (E.dirty && (rc = layout(E)) != LC_OK) return rc;
  if ((rc = ensure_capacity(E, 0)) != LC_OK) return rc;
  const int nch = static_cast<int>(E.chains.size());
  const int64_t rec = static_cast<int64_t>(nch) * lc::ST_WORDS + 1;
  int64_t done = 0;
  int stuck = 0;
  while (done < n_sweeps) {
    const int chunk =
        E.profiling ? 1 : static_cast<int>(std::min<int64_t>(n_sweeps - done, kRing));
    if (hip_err(lc_launch_fill_u64(E.ring_ctr.p, 1, 0, E.stream)) != LC_OK) return LC_EDEVICE;
    for (int q = 0; q < chunk; ++q)
      if ((rc = launch_one(E)) != LC_OK) return rc;
    if (hipMemcpyAsync(E.hring.data(), E.ring.p, chunk * rec * sizeof(unsigned long long),
                       hipMemcpyDeviceToHost, E.stream) != hipSuccess ||
        hipStreamSynchronize(E.stream) != hipSuccess)
      return LC_EDEVICE;
    int ok = 0;
    uint32_t bad = 0;
    for (; ok < chunk; ++ok) {
      const unsigned long long* r = E.hring.data() + ok * rec;
      bad = static_cast<uint32_t>(r[rec - 1]);
      if (bad) break;
      for (int i = 0; i < nch; ++i) apply_record(E.chains[i], r + i * lc::ST_WORDS, accumulate != 0);
    }
    done += ok;
    ++R.runs;
    if (E.profiling && ok) {
      if (E.ph_ms.size() != LC_PH_COUNT) E.ph_ms.assign(LC_PH_COUNT, 0.0);
      for (int p = 0; p < LC_PH_COUNT; ++p) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, E.ev[p], E.ev[p + 1]) != hipSuccess) return LC_EDEVICE;
        E.ph_ms[p] += ms;
      }
      E.ph_sweeps += 1;
    }
    for (int i = 0; i < nch; ++i) {
      lc_chain* c = E.chains[i];
      c->last_engine = &E;
      c->last_index = i;
      c->last_run = R.runs;
      // descriptors held by the chain's other engine are now stale
      if (ok && c->own && c->own != &E) c->own->dirty = true;
    }
    if (!bad) {
      stuck = 0;
      continue;
    }
    // a sweep did not fit: grow and run it again
    if (bad & LC_FLAG_SYM) return LC_ESTATE;
    if (bad & LC_FLAG_GRAPH) {
      std::fprintf(stderr, "[lc] internal error: inconsistent loop graph (flags %#x)\n", bad);
      return LC_EDEVICE;
    }
    if (++stuck > 16) return LC_ENOMEM;
    for (int i = 0; i < nch; ++i) E.chains[i]->last_engine = nullptr;
    const unsigned long long* r = E.hring.data() + ok * rec;
    if (verbose()) std::fprintf(stderr, "[lc] sweep replayed: flags %#x\n", bad);
    if (bad & LC_FLAG_TILE) {
      for (lc_chain* c : E.chains) c->tile_shrink = std::min(c->tile_shrink + 1, 10);
    }
    int64_t tot[2] = {0, 0};
    unsigned long long dc[2] = {0, 0};
    if (bad & (LC_FLAG_OPS | LC_FLAG_NODES)) {
      if (hipMemcpy(tot, E.totals.p, sizeof(tot), hipMemcpyDeviceToHost) != hipSuccess)
        return LC_EDEVICE;
    }
    if (bad & (LC_FLAG_XEDGE | LC_FLAG_FRAG)) {
      if (hipMemcpy(dc, E.dyncnt.p, sizeof(dc), hipMemcpyDeviceToHost) != hipSuccess)
        return LC_EDEVICE;
    }
    if (bad & (LC_FLAG_OPS | LC_FLAG_NODES | LC_FLAG_XEDGE | LC_FLAG_FRAG | LC_FLAG_ROOTS)) {
      // the totals are exact; grow to them plus a margin, or to the
      // per-sweep bound of the current kept counts (the arena may already
      // be larger, sized by another engine)
      const int64_t x = static_cast<int64_t>(dc[0]), f = static_cast<int64_t>(dc[1]);
      if ((rc = ensure_capacity(E, tot[0] + tot[0] / 8 + 4096, x + x / 8 + 4096, f + f / 8 + 4096)) != LC_OK)
        return rc;
    }
    if (bad & LC_FLAG_KEPT) {
      for (int i = 0; i < nch; ++i) {
        const int64_t need = static_cast<int64_t>(r[i * lc::ST_WORDS + lc::ST_KEPT_OUT]);
        if (need > E.chains[i]->kept_cap && (rc = grow_kept(E.chains[i], need)) != LC_OK) return rc;
      }
    }
    E.dirty = true;
    if ((rc = layout(E)) != LC_OK) return rc;
  }
  return LC_OK;
}

int validate(int64_t L, double S, double beta, int* two_s) {
  if (L < 4 || (L & 1) || L >= (int64_t(1) << 32)) return LC_EINVAL;
  if (!std::isfinite(S)) return LC_EINVAL;
  const double ts = 2.0 * S;
  const int t = static_cast<int>(std::lround(ts));
  if (std::fabs(ts - t) > 1e-12 || t < 1 || t > 8) return LC_EINVAL;
  // bond and spin indices are 32-bit counter words of the Philox draws
  if (static_cast<int64_t>(t) * t * L >= (int64_t(1) << 32)) return LC_EINVAL;
  if (!(beta > 0.0) || !std::isfinite(beta) || beta > 8.0 * 4294967296.0) return LC_EINVAL;
  *two_s = t;
  return LC_OK;
}

// Bytes of one chain alone: its state and the scratch it needs of an arena.
void footprint_parts(int64_t L, int two_s, double beta, double* state_b, double* scratch_b) {
  int w, K;
  double mu;
  uint64_t T[lc::kMaxTable];
  (void)window_rule(beta, &w, &mu, T, &K);
  const double n_sites = static_cast<double>(two_s) * L;
  const double n_bonds = static_cast<double>(two_s) * two_s * L;
  const double nwin = n_bonds * std::ldexp(1.0, w);
  const double nbn = two_s == 1 ? n_sites : 2 * n_sites;
  const double kept = static_cast<double>(kept_initial(static_cast<int64_t>(n_bonds), beta));
  const double ops = ops_bound(kept, n_bonds, static_cast<double>(L), two_s, beta);
  const double nodes = nbn + 2 * ops;
  const double xe = cross_per_op(two_s) * ops + 4096, fe = frags_per_op(two_s) * ops + 4096;
  // spins, kept-operator window scans and times (both halves), permutation
  *state_b = 2 * n_sites + 2 * 8 * (nwin + 1) + 2 * 8 * kept + 8 * n_sites + 65536;
  // window scans, operators (time + type), parent words, edges between
  // tiles (16 B), fragments (32 B), loop records (one per item), boundary
  // records
  *scratch_b = 2 * 8 * (nwin + 1) + 4 * nwin + 9 * ops + nodes * 8 + 16 * xe + 32 * fe +
               (fe + nbn) * (8 * kAccWords) + 8 * n_sites + (1 << 20);
}

size_t footprint_bytes(int64_t L, int two_s, double beta) {
  double st, sc;
  footprint_parts(L, two_s, beta, &st, &sc);
  return static_cast<size_t>(st + sc);
}

}  // namespace

// ------------------------------------------------------------------------
// Scratch of one sweep of one chain carved from the static device array.
namespace {

struct Carver {
  unsigned char* base;
  size_t cap, used = 0;
  template <class T>
  T* take(size_t n) {
    used = (used + 255) & ~size_t(255);
    T* p = reinterpret_cast<T*>(base + used);
    used += (n ? n : 1) * sizeof(T);
    return p;
  }
};

// Carve the scratch of one sweep of c; false if it does not fit.
bool carve_static(lc_chain* c, unsigned char* base, size_t cap, LcSweepArgs* A) {
  Carver K{base, cap};
  const int64_t ops = ops_estimate(c);
  const int64_t nodes = c->nbn + 2 * ops;
  const int64_t xe = static_cast<int64_t>(cross_per_op(c->two_s) * static_cast<double>(ops)) + 4096;
  const int64_t fe = static_cast<int64_t>(frags_per_op(c->two_s) * static_cast<double>(ops)) + 4096;
  const int64_t items = fe + c->nbn;
  std::memset(A, 0, sizeof(*A));
  A->descs = K.take<ChainDesc>(1);
  A->win_bases = K.take<int64_t>(1);
  A->site_bases = K.take<int64_t>(1);
  A->spin_bases = K.take<int64_t>(1);
  A->bn_bases = K.take<int64_t>(1);
  A->op_bases = K.take<int64_t>(1);
  A->node_bases = K.take<int64_t>(1);
  A->grp_chain = K.take<int>(1);
  A->grp_tile_base = K.take<int64_t>(1);
  A->dyn = K.take<ChainDyn>(1);
  A->totals = K.take<int64_t>(2);
  A->scan_tmp = K.take<int64_t>(LC_SCAN_BLOCKS + 1);
  A->stats = K.take<uint64_t>(lc::ST_WORDS * (1 + LC_STAT_STRIPES));
  A->flags = K.take<uint32_t>(2);
  A->ring = K.take<unsigned long long>(lc::ST_WORDS + 1);
  A->ring_ctr = K.take<uint32_t>(2);
  A->dyncnt = K.take<unsigned long long>(4);
  A->opstart = K.take<int64_t>(c->nwin + 1);
  A->accmask = K.take<uint32_t>(c->nwin);
  A->kflat = K.take<int64_t>(c->nwin + 1);
  A->optime = K.take<uint64_t>(ops);
  A->optype = K.take<uint8_t>(ops);
  A->parent = K.take<int64_t>(nodes);
  A->xedge = K.take<int64_t>(2 * xe);
  A->frag = K.take<int64_t>(4 * fe);
  A->acc = K.take<unsigned long long>(kAccWords * items);
  A->bacc = K.take<unsigned long long>(c->n_sites);
  A->rcnt = K.take<int64_t>(items / 4096 + 2);
  if (K.used > K.cap) return false;
  A->nchain = 1;
  A->any_split = c->two_s > 1 ? 1 : 0;
  A->nwin = c->nwin;
  A->nsites = c->n_sites;
  A->nspins = c->L;
  A->nbn = c->nbn;
  A->grid_blocks = kDefaultGrid;
  A->ngroups = 1;
  A->groups[0] = LcTileGroup{c->two_s, 1, 0, c->ntj * c->ntk};
  A->op_cap = ops;
  A->node_cap = nodes;
  A->root_cap = items;
  A->xcap = xe;
  A->fcap = fe;
  A->ring_cap = 1;
  A->events = nullptr;
  return true;
}

}  // namespace

extern "C" {

const char* lc_strerror(int code) {
  switch (code) {
    case LC_OK: return "ok";
    case LC_EINVAL: return "invalid argument";
    case LC_ENOMEM: return "out of device memory";
    case LC_ETOOLARGE: return "footprint exceeds device memory";
    case LC_ECAPACITY: return "caller buffer too small";
    case LC_EDEVICE: return "HIP runtime error";
    case LC_ESTATE: return "invalid state for this call";
    default: return "unknown error";
  }
}

int lc_debug_philox(uint64_t seed, const uint32_t ctr[4], uint32_t out[4]) {
  if (!ctr || !out) return LC_EINVAL;
  const lc::u32x4 r = lc::philox10(seed, ctr[0], ctr[1], ctr[2], ctr[3]);
  out[0] = r.x;
  out[1] = r.y;
  out[2] = r.z;
  out[3] = r.w;
  return LC_OK;
}

int lc_debug_work(const lc_chain* c, int64_t* n_cross, int64_t* n_frags) {
  if (!c || !n_cross || !n_frags) return LC_EINVAL;
  if (!c->own || !c->has_last || c->last_engine != c->own) return LC_ESTATE;
  unsigned long long d[2] = {0, 0};
  if (hipMemcpy(d, c->own->dyncnt.p, sizeof(d), hipMemcpyDeviceToHost) != hipSuccess) return LC_EDEVICE;
  *n_cross = static_cast<int64_t>(d[0]);
  *n_frags = static_cast<int64_t>(d[1]);
  return LC_OK;
}

int lc_debug_window_table(double beta, int* w, double* mu, uint64_t* T, int* K) {
  if (!w || !mu || !T || !K) return LC_EINVAL;
  return window_rule(beta, w, mu, T, K);
}

int lc_footprint(int64_t L, double S, double beta, size_t* bytes) {
  int two_s;
  if (!bytes) return LC_EINVAL;
  const int rc = validate(L, S, beta, &two_s);
  if (rc != LC_OK) return rc;
  *bytes = footprint_bytes(L, two_s, beta);
  return LC_OK;
}

int lc_footprint_parts(int64_t L, double S, double beta, size_t* state, size_t* scratch) {
  int two_s;
  if (!state || !scratch) return LC_EINVAL;
  const int rc = validate(L, S, beta, &two_s);
  if (rc != LC_OK) return rc;
  double st, sc;
  footprint_parts(L, two_s, beta, &st, &sc);
  *state = static_cast<size_t>(st);
  *scratch = static_cast<size_t>(sc);
  return LC_OK;
}

int lc_init_lattice(int64_t L, double S, double beta, uint64_t seed, const lc_alloc* alloc,
                    void* hip_stream, lc_chain** out) {
  if (!out) return LC_EINVAL;
  *out = nullptr;
  int two_s, rc;
  if ((rc = validate(L, S, beta, &two_s)) != LC_OK) return rc;
  if (alloc && (!alloc->alloc || !alloc->free)) return LC_EINVAL;
  size_t fb = footprint_bytes(L, two_s, beta), freeb = 0, totalb = 0;
  if (hipMemGetInfo(&freeb, &totalb) != hipSuccess) return LC_EDEVICE;
  if (fb > totalb) return LC_ETOOLARGE;
  lc_chain* c = new (std::nothrow) lc_chain();
  if (!c) return LC_ENOMEM;
  c->L = L;
  c->two_s = two_s;
  c->beta = beta;
  c->seed = seed;
  (void)window_rule(beta, &c->w, &c->mu, c->T, &c->K);
  c->n_sites = static_cast<int64_t>(two_s) * L;
  c->n_bonds = static_cast<int64_t>(two_s) * two_s * L;
  c->nwin = c->n_bonds << c->w;
  c->nbn = two_s == 1 ? c->n_sites : 2 * c->n_sites;
  c->stream = static_cast<hipStream_t>(hip_stream);
  c->mem.s = c->stream;
  if (alloc) {
    c->mem.a = *alloc;
    c->mem.user = true;
  }
  const int64_t kcap = kept_initial(c->n_bonds, beta);
  bool ok = true;
  for (int q = 0; q < 2; ++q)
    ok = ok && c->s0[q].ensure(c->mem, c->n_sites) &&
         c->kstart[q].ensure(c->mem, static_cast<size_t>(c->nwin) + 1) &&
         c->ktime[q].ensure(c->mem, static_cast<size_t>(kcap));
  ok = ok && c->perm.ensure(c->mem, c->n_sites);
  if (!ok) {
    lc_free(c);
    return LC_ENOMEM;
  }
  c->kept_cap = kcap;
  // initial configuration on the device
  ChainDesc d = make_desc(c, 0, 0, 0, 0);
  ChainDesc* dd = static_cast<ChainDesc*>(c->mem.get(sizeof(ChainDesc)));
  if (!dd) {
    lc_free(c);
    return LC_ENOMEM;
  }
  rc = LC_OK;
  if (hipMemcpyAsync(dd, &d, sizeof(d), hipMemcpyHostToDevice, c->stream) != hipSuccess ||
      lc_launch_init_chain(dd, std::max(c->n_sites, c->nwin + 1), c->stream) != hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess)
    rc = LC_EDEVICE;
  c->mem.put(dd, sizeof(ChainDesc));
  if (rc != LC_OK) {
    lc_free(c);
    return rc;
  }
  *out = c;
  return LC_OK;
}

static Engine* own_engine(lc_chain* c) {
  if (!c->own) {
    c->own = new (std::nothrow) Engine();
    if (!c->own) return nullptr;
    c->own->mem = c->mem;
    c->own->stream = c->stream;
    c->own->ar = arena_get(c->mem);
    if (!c->own->ar) {
      delete c->own;
      c->own = nullptr;
      return nullptr;
    }
    c->own->chains.push_back(c);
    // graph capture needs a stream other than the legacy null stream
    c->own->use_graph = c->stream != nullptr;
  }
  return c->own;
}

int lc_capacity(const lc_chain* c, int64_t* kept_cap, size_t* scratch) {
  if (!c || !kept_cap || !scratch) return LC_EINVAL;
  *kept_cap = c->kept_cap;
  *scratch = c->own && c->own->ar ? static_cast<size_t>(c->own->ar->bytes()) : 0;
  return LC_OK;
}

int lc_set_schedule(lc_chain* c, int grid_blocks, int use_graph) {
  if (!c || grid_blocks < 0) return LC_EINVAL;
  Engine* E = own_engine(c);
  if (!E) return LC_ENOMEM;
  E->grid = grid_blocks > 0 ? grid_blocks : kDefaultGrid;
  E->use_graph = use_graph && c->stream != nullptr;
  E->drop_graph();
  return LC_OK;
}

// Time trial sweeps per candidate grid (graph replay when the stream allows
// capture), keep the fastest.
static int autotune(Engine& E, const int* grids, int n, int trials, int* best, double* ms) {
  if (!grids || n < 1 || trials < 1) return LC_EINVAL;
  for (int i = 0; i < n; ++i)
    if (grids[i] <= 0) return LC_EINVAL;
  const bool graph = E.stream != nullptr;
  double best_ms = 0.0;
  int bg = E.grid, rc;
  for (int i = 0; i < n; ++i) {
    E.grid = grids[i];
    E.use_graph = graph;
    E.drop_graph();
    if ((rc = run_engine(E, 1, 0)) != LC_OK) return rc;  // warm-up, capture
    const auto t0 = std::chrono::steady_clock::now();
    if ((rc = run_engine(E, trials, 0)) != LC_OK) return rc;
    const auto t1 = std::chrono::steady_clock::now();
    const double per = std::chrono::duration<double, std::milli>(t1 - t0).count() / trials;
    if (i == 0 || per < best_ms) {
      best_ms = per;
      bg = grids[i];
    }
  }
  E.grid = bg;
  E.drop_graph();
  if (best) *best = bg;
  if (ms) *ms = best_ms;
  return LC_OK;
}

// Every tile shape with every grid: the fastest pair is kept.
static int autotune_tiles(Engine& E, const int* windows, const int* targets, int n_shapes,
                          const int* grids, int n_grids, int trials, int* best_shape, int* best_grid,
                          double* ms) {
  if (!windows || !targets || n_shapes < 1) return LC_EINVAL;
  for (int i = 0; i < n_shapes; ++i) {
    const bool pow2 = windows[i] > 0 && (windows[i] & (windows[i] - 1)) == 0;
    if ((windows[i] != 0 && (!pow2 || windows[i] > 16)) ||
        (targets[i] != 0 && (targets[i] < 64 || targets[i] > LC_TILE_OPS)))
      return LC_EINVAL;
  }
  double best_ms = 0.0;
  int bs = 0, bg = E.grid, rc;
  for (int i = 0; i < n_shapes; ++i) {
    for (lc_chain* c : E.chains) {
      c->tile_kmax = windows[i];
      c->tile_target = targets[i];
      c->tile_shrink = 0;
    }
    E.dirty = true;
    int g = 0;
    double t = 0.0;
    if ((rc = autotune(E, grids, n_grids, trials, &g, &t)) != LC_OK) return rc;
    if (i == 0 || t < best_ms) {
      best_ms = t;
      bs = i;
      bg = g;
    }
  }
  for (lc_chain* c : E.chains) {
    c->tile_kmax = windows[bs];
    c->tile_target = targets[bs];
    c->tile_shrink = 0;
  }
  E.dirty = true;
  E.grid = bg;
  E.drop_graph();
  if (best_shape) *best_shape = bs;
  if (best_grid) *best_grid = bg;
  if (ms) *ms = best_ms;
  return LC_OK;
}

int lc_autotune_tiles(lc_chain* c, const int* windows, const int* targets, int n_shapes,
                      const int* grids, int n_grids, int trial_sweeps, int* best_shape,
                      int* best_grid, double* ms_per_sweep) {
  if (!c) return LC_EINVAL;
  if (c->batch) return LC_ESTATE;
  Engine* E = own_engine(c);
  if (!E) return LC_ENOMEM;
  return autotune_tiles(*E, windows, targets, n_shapes, grids, n_grids, trial_sweeps, best_shape,
                        best_grid, ms_per_sweep);
}

int lc_batch_autotune_tiles(lc_batch* b, const int* windows, const int* targets, int n_shapes,
                            const int* grids, int n_grids, int trial_sweeps, int* best_shape,
                            int* best_grid, double* ms_per_sweep) {
  if (!b) return LC_EINVAL;
  for (lc_chain* c : b->eng.chains)
    if (c->stream != b->eng.stream && hipStreamSynchronize(c->stream) != hipSuccess) return LC_EDEVICE;
  return autotune_tiles(b->eng, windows, targets, n_shapes, grids, n_grids, trial_sweeps,
                        best_shape, best_grid, ms_per_sweep);
}

int lc_autotune(lc_chain* c, const int* grids, int n_grids, int trial_sweeps, int* best_grid,
                double* ms_per_sweep) {
  if (!c) return LC_EINVAL;
  if (c->batch) return LC_ESTATE;
  Engine* E = own_engine(c);
  if (!E) return LC_ENOMEM;
  return autotune(*E, grids, n_grids, trial_sweeps, best_grid, ms_per_sweep);
}

int lc_batch_autotune(lc_batch* b, const int* grids, int n_grids, int trial_sweeps, int* best_grid,
                      double* ms_per_sweep) {
  if (!b) return LC_EINVAL;
  for (lc_chain* c : b->eng.chains)
    if (c->stream != b->eng.stream && hipStreamSynchronize(c->stream) != hipSuccess) return LC_EDEVICE;
  return autotune(b->eng, grids, n_grids, trial_sweeps, best_grid, ms_per_sweep);
}

int lc_update(lc_chain* c, int64_t n_sweeps, int accumulate) {
  if (!c || n_sweeps < 0) return LC_EINVAL;
  if (c->batch) return LC_ESTATE;
  Engine* E = own_engine(c);
  if (!E) return LC_ENOMEM;
  return run_engine(*E, n_sweeps, accumulate);
}

// Sweeps of one chain with all per-sweep scratch carved from the library's
// static device array (lc_static.hip): no allocation anywhere in the call.
int lc_update_noalloc(lc_chain* c, int64_t n_sweeps, int accumulate) {
  if (!c || n_sweeps < 0) return LC_EINVAL;
  if (c->batch) return LC_ESTATE;
  if (n_sweeps == 0) return LC_OK;
  size_t cap = 0;
  unsigned char* base = static_cast<unsigned char*>(lc_static_scratch(&cap));
  if (!base) return LC_EDEVICE;
  hipStream_t s = c->stream;
  int64_t done = 0;
  int retries = 0;
  while (done < n_sweeps) {
    choose_tile(c);
    LcSweepArgs A;
    if (!carve_static(c, base, cap, &A)) return LC_ETOOLARGE;
    const ChainDesc d = make_desc(c, 0, 0, 0, 0);
    const int64_t zero = 0;
    const int gc = 0;
    unsigned long long rec[lc::ST_WORDS + 1];
    if (hipMemcpyAsync(A.descs, &d, sizeof(d), hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(const_cast<int64_t*>(A.win_bases), &zero, 8, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(const_cast<int64_t*>(A.site_bases), &zero, 8, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(const_cast<int64_t*>(A.spin_bases), &zero, 8, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(const_cast<int64_t*>(A.bn_bases), &zero, 8, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(const_cast<int64_t*>(A.grp_tile_base), &zero, 8, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(const_cast<int*>(A.grp_chain), &gc, sizeof(int), hipMemcpyHostToDevice, s) != hipSuccess ||
        lc_launch_fill_u64(A.ring_ctr, 1, 0, s) != hipSuccess ||
        lc_launch_sweep(A, s) != hipSuccess ||
        hipMemcpyAsync(rec, A.ring, sizeof(rec), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return LC_EDEVICE;
    const uint32_t bad = static_cast<uint32_t>(rec[lc::ST_WORDS]);
    if (!bad) {
      apply_record(c, rec, accumulate != 0);
      ++done;
      retries = 0;
      continue;
    }
    // the sweep was discarded: the chain is unchanged
    if (bad & LC_FLAG_SYM) return LC_ESTATE;
    if (bad & LC_FLAG_GRAPH) return LC_EDEVICE;
    if ((bad & ~LC_FLAG_TILE) || ++retries > 10) return LC_ETOOLARGE;  // cannot grow
    c->tile_shrink = std::min(c->tile_shrink + 1, 10);
  }
  // the chain's own engine holds descriptors of an older sweep; the arena
  // holds no operators or labels of these sweeps
  if (c->own) c->own->dirty = true;
  c->last_engine = nullptr;
  return LC_OK;
}

int lc_set_tile(lc_chain* c, int max_windows, int target_ops) {
  if (!c) return LC_EINVAL;
  const bool pow2 = max_windows > 0 && (max_windows & (max_windows - 1)) == 0;
  if (max_windows != 0 && (!pow2 || max_windows > 16)) return LC_EINVAL;
  if (target_ops != 0 && (target_ops < 64 || target_ops > LC_TILE_OPS)) return LC_EINVAL;
  c->tile_kmax = max_windows;
  c->tile_target = target_ops;
  c->tile_shrink = 0;
  if (c->own) c->own->dirty = true;
  if (c->batch) c->batch->eng.dirty = true;
  return LC_OK;
}

int lc_set_flip_rule(lc_chain* c, int rule) {
  if (!c || (rule != LC_FLIP_LABEL && rule != LC_FLIP_VOTE)) return LC_EINVAL;
  c->flip_rule = rule;
  if (c->own) c->own->dirty = true;
  if (c->batch) c->batch->eng.dirty = true;
  return LC_OK;
}

int lc_measure(const lc_chain* c, lc_measurement* out) {
  if (!c || !out) return LC_EINVAL;
  std::memset(out, 0, sizeof(*out));
  const Accum& a = c->acc;
  out->n_sweeps = a.n;
  if (a.n == 0) return LC_OK;
  const double n = static_cast<double>(a.n), L = static_cast<double>(c->L), b = c->beta;
  const double nb = static_cast<double>(c->n_bonds);
  out->mean_ops = static_cast<double>(a.ops) / n;
  out->mean_clusters = static_cast<double>(a.clusters) / n;
  out->e = nb / (4.0 * L) - out->mean_ops / (b * L);
  out->chi_u = b / (4.0 * L) * (static_cast<double>(a.m2) / n);
  out->chi_u_plain = b / (4.0 * L) * (static_cast<double>(a.ma2) / n);
  out->s_pi = (static_cast<double>(a.n02) / n) / (4.0 * L);
  out->chi_s = b / (4.0 * L) * (static_cast<double>(a.len2) / 18446744073709551616.0 / n);
  return LC_OK;
}

int lc_last_sweep(const lc_chain* c, lc_sweep_stats* out) {
  if (!c || !out) return LC_EINVAL;
  if (!c->has_last) return LC_ESTATE;
  *out = c->last;
  return LC_OK;
}

int lc_reset_measurements(lc_chain* c) {
  if (!c) return LC_EINVAL;
  c->acc = Accum();
  return LC_OK;
}

int lc_export_state(const lc_chain* c, uint8_t* s0, int64_t* bond_off, uint64_t* times,
                    int64_t* n_kept, int64_t* sweep) {
  if (!c || !n_kept) return LC_EINVAL;
  const int64_t have = *n_kept;
  *n_kept = c->n_kept;
  if (sweep) *sweep = c->sweep;
  if (times && have < c->n_kept) return LC_ECAPACITY;  // before any copy starts
  hipStream_t s = c->stream;
  if (s0 && hipMemcpyAsync(s0, c->s0[c->cur].p, c->n_sites, hipMemcpyDeviceToHost, s) != hipSuccess)
    return LC_EDEVICE;
  if (bond_off) {
    std::vector<int64_t> ks(static_cast<size_t>(c->nwin) + 1);
    if (hipMemcpyAsync(ks.data(), c->kstart[c->cur].p, ks.size() * sizeof(int64_t),
                       hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return LC_EDEVICE;
    for (int64_t b = 0; b <= c->n_bonds; ++b) bond_off[b] = ks[b << c->w];
  }
  if (times) {
    if (c->n_kept && hipMemcpyAsync(times, c->ktime[c->cur].p, c->n_kept * sizeof(uint64_t),
                                    hipMemcpyDeviceToHost, s) != hipSuccess)
      return LC_EDEVICE;
  }
  return hip_err(hipStreamSynchronize(s));
}

int lc_import_state(lc_chain* c, const uint8_t* s0, const int64_t* bond_off, const uint64_t* times,
                    int64_t sweep) {
  if (!c || !s0 || !bond_off || sweep < 0 || sweep > 0xFFFFFFFFll) return LC_EINVAL;
  if (bond_off[0] != 0) return LC_EINVAL;
  for (int64_t b = 0; b < c->n_bonds; ++b)
    if (bond_off[b + 1] < bond_off[b]) return LC_EINVAL;
  const int64_t n = bond_off[c->n_bonds];
  if (n > 0 && !times) return LC_EINVAL;
  for (int64_t b = 0; b < c->n_bonds; ++b)
    for (int64_t i = bond_off[b] + 1; i < bond_off[b + 1]; ++i)
      if (times[i] < times[i - 1]) return LC_EINVAL;
  for (int64_t x = 0; x < c->n_sites; ++x)
    if (s0[x] > 1) return LC_EINVAL;
  int rc;
  if (n > c->kept_cap && (rc = grow_kept(c, n)) != LC_OK) return rc;
  // kept operators per window, exclusive scan
  std::vector<int64_t> ks(static_cast<size_t>(c->nwin) + 1, 0);
  const int64_t W = int64_t(1) << c->w;
  for (int64_t b = 0; b < c->n_bonds; ++b)
    for (int64_t i = bond_off[b]; i < bond_off[b + 1]; ++i) {
      const int64_t k = c->w == 0 ? 0 : static_cast<int64_t>(times[i] >> (64 - c->w));
      ks[b * W + k + 1] += 1;
    }
  for (size_t i = 1; i < ks.size(); ++i) ks[i] += ks[i - 1];
  hipStream_t s = c->stream;
  if (hipMemcpyAsync(c->s0[c->cur].p, s0, c->n_sites, hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemcpyAsync(c->kstart[c->cur].p, ks.data(), ks.size() * sizeof(int64_t),
                     hipMemcpyHostToDevice, s) != hipSuccess ||
      (n > 0 && hipMemcpyAsync(c->ktime[c->cur].p, times, n * sizeof(uint64_t),
                               hipMemcpyHostToDevice, s) != hipSuccess) ||
      hipStreamSynchronize(s) != hipSuccess)
    return LC_EDEVICE;
  c->n_kept = n;
  c->sweep = static_cast<uint32_t>(sweep);
  c->has_last = false;
  c->last_engine = nullptr;
  if (c->own) c->own->dirty = true;
  if (c->batch) c->batch->eng.dirty = true;
  return LC_OK;
}

// Operator and node ranges of a chain's most recent sweep, still held in the
// arena only if no other sweep has run there since (caller holds the lock).
static int last_ranges(const lc_chain* c, ChainDyn* d, int64_t* win_base) {
  const Engine* E = c->last_engine;
  if (!E || !c->has_last || E->ar->runs != c->last_run) return LC_ESTATE;
  if (hipMemcpy(d, E->dyn.p + c->last_index, sizeof(ChainDyn), hipMemcpyDeviceToHost) != hipSuccess)
    return LC_EDEVICE;
  int64_t wb = 0;
  for (int i = 0; i < c->last_index; ++i) wb += E->chains[i]->nwin;
  *win_base = wb;
  return LC_OK;
}

int lc_export_ops(const lc_chain* c, int64_t* op_bond, uint64_t* op_time, uint8_t* op_type0,
                  uint8_t* op_type1, int64_t* n_ops) {
  if (!c || !n_ops) return LC_EINVAL;
  if (!c->last_engine) return LC_ESTATE;
  std::lock_guard<std::mutex> hold(c->last_engine->ar->mu);
  ChainDyn d;
  int64_t wb;
  int rc = last_ranges(c, &d, &wb);
  if (rc != LC_OK) return rc;
  const int64_t have = *n_ops;
  *n_ops = d.n_ops;
  if (!op_bond && !op_time && !op_type0 && !op_type1) return LC_OK;
  if (have < d.n_ops) return LC_ECAPACITY;
  const Arena* E = c->last_engine->ar;
  std::vector<uint8_t> ty(static_cast<size_t>(std::max<int64_t>(d.n_ops, 1)));
  if (op_time && d.n_ops &&
      hipMemcpy(op_time, E->optime.p + d.op_base, d.n_ops * sizeof(uint64_t), hipMemcpyDeviceToHost) !=
          hipSuccess)
    return LC_EDEVICE;
  if (d.n_ops &&
      hipMemcpy(ty.data(), E->optype.p + d.op_base, d.n_ops, hipMemcpyDeviceToHost) != hipSuccess)
    return LC_EDEVICE;
  for (int64_t q = 0; q < d.n_ops; ++q) {
    if (op_type0) op_type0[q] = (ty[q] >> 1) & 1;
    if (op_type1) op_type1[q] = ty[q] & 1;
  }
  if (op_bond) {
    const int64_t W = int64_t(1) << c->w;
    std::vector<int64_t> os(static_cast<size_t>(c->n_bonds) + 1);
    for (int64_t b = 0; b <= c->n_bonds; ++b)
      if (hipMemcpy(&os[b], E->opstart.p + wb + b * W, sizeof(int64_t), hipMemcpyDeviceToHost) !=
          hipSuccess)
        return LC_EDEVICE;
    for (int64_t b = 0; b < c->n_bonds; ++b)
      for (int64_t q = os[b]; q < os[b + 1]; ++q) op_bond[q - d.op_base] = b;
  }
  return LC_OK;
}

int lc_export_labels(const lc_chain* c, int64_t* labels, int64_t* n_nodes) {
  if (!c || !n_nodes) return LC_EINVAL;
  if (!c->last_engine) return LC_ESTATE;
  std::lock_guard<std::mutex> hold(c->last_engine->ar->mu);
  ChainDyn d;
  int64_t wb;
  int rc = last_ranges(c, &d, &wb);
  if (rc != LC_OK) return rc;
  const int64_t have = *n_nodes;
  *n_nodes = d.n_nodes;
  if (!labels) return LC_OK;
  if (have < d.n_nodes) return LC_ECAPACITY;
  if (hipMemcpy(labels, c->last_engine->ar->parent.p + d.node_base, d.n_nodes * sizeof(int64_t),
                hipMemcpyDeviceToHost) != hipSuccess)
    return LC_EDEVICE;
  // parent words after a sweep: a node of a loop finished inside its
  // linking tile holds a code naming the loop's smallest node; a node
  // holding another negative word (a loop code) is the smallest node of its
  // loop; any other node's parent p is that smallest node or a node whose
  // own word is it (non-negative) or a code (p is it).  Words are read from
  // the copy before any is rewritten.
  std::vector<int64_t> w(labels, labels + d.n_nodes);
  for (int64_t v = 0; v < d.n_nodes; ++v) {
    const int64_t p = w[v];
    if (lc::is_closed_word(p)) {
      const int64_t r = lc::closed_rep(p) - d.node_base;
      if (r < 0 || r >= d.n_nodes) return LC_EDEVICE;  // not a node of this chain
      labels[v] = r;
    } else if (p < 0) {
      labels[v] = v;
    } else {
      const int64_t pl = p - d.node_base;
      if (pl < 0 || pl >= d.n_nodes) return LC_EDEVICE;  // not a node of this chain
      const int64_t pp = w[pl];
      labels[v] = (pp >= 0 ? pp : p) - d.node_base;
    }
  }
  return LC_OK;
}

int lc_slice_tables(const lc_chain* c, int n_slices, int64_t* bottom, int64_t* top,
                    int64_t* op_labels, int64_t* n_ops) {
  if (!c || !n_ops) return LC_EINVAL;
  if (!c->last_engine) return LC_ESTATE;
  Arena* R = c->last_engine->ar;
  std::lock_guard<std::mutex> hold(R->mu);
  ChainDyn d;
  int64_t wb;
  int rc = last_ranges(c, &d, &wb);
  if (rc != LC_OK) return rc;
  const int64_t W = int64_t(1) << c->w;
  if (n_slices < 1 || n_slices > W) return LC_EINVAL;
  const int64_t have = *n_ops;
  *n_ops = d.n_ops;
  if (!bottom && !top && !op_labels) return LC_OK;
  if (!bottom || !top || !op_labels) return LC_EINVAL;
  if (have < d.n_ops) return LC_ECAPACITY;
  const int64_t ns = c->n_sites, G = n_slices;
  const int64_t n = 2 * ns * G + 2 * d.n_ops;
  int64_t* par = static_cast<int64_t*>(c->mem.get(static_cast<size_t>(n) * sizeof(int64_t)));
  uint32_t* fl = static_cast<uint32_t*>(c->mem.get(8));
  if (!par || !fl) {
    c->mem.put(par, static_cast<size_t>(n) * sizeof(int64_t));
    c->mem.put(fl, 8);
    return LC_ENOMEM;
  }
  LcSliceArgs A;
  A.L = c->L;
  A.n_sites = ns;
  A.two_s = c->two_s;
  A.w = c->w;
  A.win_base = wb;
  A.op_base = d.op_base;
  A.n_ops = d.n_ops;
  A.opstart = R->opstart.p;
  A.optime = R->optime.p;
  A.n_slices = G;
  A.parent = par;
  A.flags = fl;
  std::vector<int64_t> h(static_cast<size_t>(n));
  uint32_t bad = 0;
  hipStream_t s = c->stream;
  rc = LC_OK;
  if (lc_launch_fill_u64(fl, 1, 0, s) != hipSuccess || lc_launch_slices(A, s) != hipSuccess ||
      hipMemcpyAsync(h.data(), par, static_cast<size_t>(n) * sizeof(int64_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipMemcpyAsync(&bad, fl, sizeof(bad), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    rc = LC_EDEVICE;
  c->mem.put(par, static_cast<size_t>(n) * sizeof(int64_t));
  c->mem.put(fl, 8);
  if (rc != LC_OK) return rc;
  if (bad) return LC_EDEVICE;
  for (int64_t p = 0; p < G; ++p)
    for (int64_t x = 0; x < ns; ++x) {
      bottom[p * ns + x] = h[2 * ns * p + x];
      top[p * ns + x] = h[2 * ns * p + ns + x];
    }
  for (int64_t i = 0; i < 2 * d.n_ops; ++i) op_labels[i] = h[2 * ns * G + i];
  return LC_OK;
}

int lc_fourier_last(const lc_chain* c, lc_fourier* out) {
  if (!c || !out) return LC_EINVAL;
  if (!c->last_engine) return LC_ESTATE;
  Arena* R = c->last_engine->ar;
  std::lock_guard<std::mutex> hold(R->mu);
  ChainDyn d;
  int64_t wb;
  int rc = last_ranges(c, &d, &wb);
  if (rc != LC_OK) return rc;
  LcFourierArgs A;
  A.L = c->L;
  A.n_sites = c->n_sites;
  A.n_bonds = c->n_bonds;
  A.two_s = c->two_s;
  A.w = c->w;
  A.win_base = wb;
  A.op_base = d.op_base;
  A.node_base = d.node_base;
  A.nbn = c->nbn;
  A.n_nodes = d.n_nodes;
  A.beta = c->beta;
  A.opstart = R->opstart.p;
  A.optime = R->optime.p;
  A.parent = R->parent.p;
  const size_t idx_bytes = static_cast<size_t>(d.n_nodes + 1) * sizeof(int64_t);
  const size_t scan_bytes = (LC_SCAN_BLOCKS + 1) * sizeof(int64_t);
  A.loopidx = static_cast<int64_t*>(c->mem.get(idx_bytes));
  A.scan_tmp = static_cast<int64_t*>(c->mem.get(scan_bytes));
  A.out = static_cast<double*>(c->mem.get(4 * sizeof(double)));
  A.acc = nullptr;
  hipStream_t s = c->stream;
  int64_t n_loops = 0;
  double sums[4] = {0, 0, 0, 0};
  size_t acc_bytes = 0;
  rc = LC_OK;
  if (!A.loopidx || !A.scan_tmp || !A.out) {
    rc = LC_ENOMEM;
  } else if (lc_launch_fourier_index(A, s) != hipSuccess ||
             hipMemcpyAsync(&n_loops, A.loopidx + d.n_nodes, sizeof(n_loops), hipMemcpyDeviceToHost, s) != hipSuccess ||
             hipStreamSynchronize(s) != hipSuccess) {
    rc = LC_EDEVICE;
  } else if (n_loops < 1 || n_loops > d.n_nodes) {
    rc = LC_EDEVICE;  // every loop has a smallest node: an inconsistent forest
  } else {
    acc_bytes = static_cast<size_t>(n_loops) * 7 * sizeof(double);
    A.acc = static_cast<double*>(c->mem.get(acc_bytes));
    if (!A.acc)
      rc = LC_ENOMEM;
    else if (lc_launch_fourier_sums(A, n_loops, s) != hipSuccess ||
             hipMemcpyAsync(sums, A.out, sizeof(sums), hipMemcpyDeviceToHost, s) != hipSuccess ||
             hipStreamSynchronize(s) != hipSuccess)
      rc = LC_EDEVICE;
  }
  c->mem.put(A.acc, acc_bytes);
  c->mem.put(A.out, 4 * sizeof(double));
  c->mem.put(A.scan_tmp, scan_bytes);
  c->mem.put(A.loopidx, idx_bytes);
  if (rc != LC_OK) return rc;
  const double L = static_cast<double>(c->L), beta = c->beta;
  const double w = 2.0 * 3.14159265358979323846 / beta;  // i w Q was summed
  out->chi_pi = sums[0] / (4.0 * beta * L);
  out->chi_pi_q1 = sums[1] / (4.0 * beta * L);
  out->chi_pi_w1 = sums[2] / (w * w) / (4.0 * beta * L);
  out->s_pi_q1 = sums[3] / (4.0 * L);
  out->n_loops = n_loops;
  return LC_OK;
}

int lc_export_perm(const lc_chain* c, int64_t* perm, int64_t* n) {
  if (!c || !n) return LC_EINVAL;
  const int64_t have = *n;
  *n = c->two_s > 1 ? c->n_sites : 0;
  if (!perm || c->two_s == 1) return LC_OK;
  if (!c->has_last) return LC_ESTATE;
  if (have < c->n_sites) return LC_ECAPACITY;
  return hip_err(hipMemcpy(perm, c->perm.p, c->n_sites * sizeof(int64_t), hipMemcpyDeviceToHost));
}

void lc_free(lc_chain* c) {
  if (!c) return;
  if (c->batch) (void)lc_batch_remove(c->batch, c);
  if (c->own) {
    c->own->release_all();
    delete c->own;
  }
  for (int q = 0; q < 2; ++q) {
    c->s0[q].release(c->mem);
    c->kstart[q].release(c->mem);
    c->ktime[q].release(c->mem);
  }
  c->perm.release(c->mem);
  delete c;
}

int lc_batch_create(const lc_alloc* alloc, void* hip_stream, lc_batch** out) {
  if (!out) return LC_EINVAL;
  *out = nullptr;
  if (alloc && (!alloc->alloc || !alloc->free)) return LC_EINVAL;
  lc_batch* b = new (std::nothrow) lc_batch();
  if (!b) return LC_ENOMEM;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  if (!s) {
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
      delete b;
      return LC_EDEVICE;
    }
    b->owns_stream = true;
  }
  b->eng.stream = s;
  b->eng.mem.s = s;
  if (alloc) {
    b->eng.mem.a = *alloc;
    b->eng.mem.user = true;
  }
  b->eng.ar = arena_get(b->eng.mem);
  if (!b->eng.ar) {
    if (b->owns_stream) (void)hipStreamDestroy(s);
    delete b;
    return LC_ENOMEM;
  }
  *out = b;
  return LC_OK;
}

int lc_batch_add(lc_batch* b, lc_chain* c) {
  if (!b || !c) return LC_EINVAL;
  if (c->batch) return LC_ESTATE;
  b->eng.chains.push_back(c);
  c->batch = b;
  b->eng.dirty = true;
  return LC_OK;
}

int lc_batch_remove(lc_batch* b, lc_chain* c) {
  if (!b || !c) return LC_EINVAL;
  auto& v = b->eng.chains;
  auto it = std::find(v.begin(), v.end(), c);
  if (it == v.end()) return LC_EINVAL;
  // wait for queued work before the chain leaves
  (void)hipStreamSynchronize(b->eng.stream);
  v.erase(it);
  c->batch = nullptr;
  if (c->own) c->own->dirty = true;
  if (c->last_engine == &b->eng) c->last_engine = nullptr;
  for (lc_chain* o : v)
    if (o->last_engine == &b->eng) o->last_engine = nullptr;
  b->eng.dirty = true;
  return LC_OK;
}

int lc_batch_size(const lc_batch* b, int* n) {
  if (!b || !n) return LC_EINVAL;
  *n = static_cast<int>(b->eng.chains.size());
  return LC_OK;
}

int lc_batch_update(lc_batch* b, int64_t n_sweeps, int accumulate) {
  if (!b || n_sweeps < 0) return LC_EINVAL;
  // member chains may have been driven alone or on other streams before
  for (lc_chain* c : b->eng.chains)
    if (c->stream != b->eng.stream && hipStreamSynchronize(c->stream) != hipSuccess) return LC_EDEVICE;
  return run_engine(b->eng, n_sweeps, accumulate);
}

int lc_batch_scratch_bytes(const lc_batch* b, size_t* bytes) {
  if (!b || !bytes) return LC_EINVAL;
  *bytes = b->eng.ar ? static_cast<size_t>(b->eng.ar->bytes()) : 0;
  return LC_OK;
}

int lc_batch_set_schedule(lc_batch* b, int grid_blocks, int use_graph) {
  if (!b || grid_blocks < 0) return LC_EINVAL;
  b->eng.grid = grid_blocks > 0 ? grid_blocks : kDefaultGrid;
  b->eng.use_graph = use_graph != 0;
  b->eng.drop_graph();
  return LC_OK;
}

static const char* const kPhaseNames[LC_PH_COUNT] = {
    "setup",    "gen_count", "scan_ops",     "gen_write", "link_tiles", "link_cross", "compress",
    "roots",    "accum",     "cluster_sums", "flip",      "scan_kept",  "compact"};

int lc_phase_count(void) { return LC_PH_COUNT; }

const char* lc_phase_name(int phase) {
  return (phase >= 0 && phase < LC_PH_COUNT) ? kPhaseNames[phase] : nullptr;
}

static int set_profiling(Engine* E, int on) {
  E->profiling = on != 0;
  E->ph_ms.assign(LC_PH_COUNT, 0.0);
  E->ph_sweeps = 0;
  if (!E->profiling) E->drop_events();
  return LC_OK;
}

static int get_profile(const Engine* E, double* ms, int n, int64_t* sweeps) {
  if (!ms || n < 0) return LC_EINVAL;
  for (int p = 0; p < n && p < LC_PH_COUNT; ++p)
    ms[p] = p < static_cast<int>(E->ph_ms.size()) ? E->ph_ms[p] : 0.0;
  if (sweeps) *sweeps = E->ph_sweeps;
  return LC_OK;
}

int lc_set_profiling(lc_chain* c, int on) {
  if (!c) return LC_EINVAL;
  Engine* E = own_engine(c);
  if (!E) return LC_ENOMEM;
  return set_profiling(E, on);
}

int lc_profile(const lc_chain* c, double* ms, int n, int64_t* sweeps) {
  if (!c || !c->own) return LC_EINVAL;
  return get_profile(c->own, ms, n, sweeps);
}

int lc_batch_set_profiling(lc_batch* b, int on) {
  if (!b) return LC_EINVAL;
  return set_profiling(&b->eng, on);
}

int lc_batch_profile(const lc_batch* b, double* ms, int n, int64_t* sweeps) {
  if (!b) return LC_EINVAL;
  return get_profile(&b->eng, ms, n, sweeps);
}

void lc_batch_free(lc_batch* b) {
  if (!b) return;
  (void)hipStreamSynchronize(b->eng.stream);
  for (lc_chain* c : b->eng.chains) {
    c->batch = nullptr;
    if (c->last_engine == &b->eng) c->last_engine = nullptr;
  }
  b->eng.chains.clear();
  b->eng.release_all();
  if (b->owns_stream) (void)hipStreamDestroy(b->eng.stream);
  delete b;
}

}  // extern "C"
