// C-ABI host layer: argument checks, workspaces, pair scheduling, stage order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/ace.h"
#include "ace_internal.h"

namespace ace {

struct EventRecorder {
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  uint32_t mask = ~0u;  // classes that are bracketed
  struct Mark { int cls; size_t a, b; };
  std::vector<Mark> marks;
  std::vector<size_t> open[KC_COUNT];
  double total_ms[KC_COUNT] = {0};
  double total_units[KC_COUNT] = {0};
  int64_t count[KC_COUNT] = {0};
  std::vector<double> mark_units;
  hipEvent_t next() {
    if (used == pool.size()) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      pool.push_back(e);
    }
    return pool[used++];
  }
};

void rec_begin(EventRecorder* r, int cls, hipStream_t s) {
  if (!r || !((r->mask >> cls) & 1u)) return;
  const size_t idx = r->used;
  hipEvent_t e = r->next();
  if (!e) return;
  (void)hipEventRecord(e, s);
  r->open[cls].push_back(idx);
}

void rec_end(EventRecorder* r, int cls, hipStream_t s, double units) {
  if (!r || !((r->mask >> cls) & 1u) || r->open[cls].empty()) return;
  const size_t idx = r->used;
  hipEvent_t e = r->next();
  if (!e) return;
  (void)hipEventRecord(e, s);
  r->marks.push_back({cls, r->open[cls].back(), idx});
  r->mark_units.push_back(units);
  r->open[cls].pop_back();
}

// Collect finished marks into the per-class totals (synchronizes the stream).
static void rec_collect(EventRecorder* r, hipStream_t s) {
  if (!r || r->marks.empty()) return;
  (void)hipStreamSynchronize(s);
  for (size_t q = 0; q < r->marks.size(); ++q) {
    const auto& m = r->marks[q];
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r->pool[m.a], r->pool[m.b]) == hipSuccess) {
      r->total_ms[m.cls] += ms;
      r->total_units[m.cls] += r->mark_units[q];
      r->count[m.cls] += 1;
    }
  }
  r->marks.clear();
  r->mark_units.clear();
  bool any_open = false;
  for (int c = 0; c < KC_COUNT; ++c) any_open |= !r->open[c].empty();
  if (!any_open) r->used = 0;
}

struct Buf {
  void* p = nullptr;
  size_t bytes = 0;
};

}  // namespace ace

using namespace ace;

struct ScheduleKey {
  int64_t npairs;
  int norb;
  uint64_t hash;
  bool operator<(const ScheduleKey& o) const {
    if (npairs != o.npairs) return npairs < o.npairs;
    if (norb != o.norb) return norb < o.norb;
    return hash < o.hash;
  }
};

struct Schedule {
  std::vector<Pack> packs;             // all rounds concatenated
  std::vector<int64_t> pidx;           // pair index of each pack half (-1 if none)
  struct Launch { int first, second, npairs; };
  std::vector<Launch> launches;  // (first pack, pack count, pair count) per launch
  std::vector<int> round_first, round_count;  // packs of each conflict-free round
  int max_launch = 0;
  // owner-computes W: packs of consecutive pairs in input order, their pair
  // indices, and per orbital k the adjacency entries (pair index, partner)
  // adj[2 * a], adj[2 * a + 1] for a in [adj_ptr[k], adj_ptr[k + 1])
  std::vector<Pack> opacks;
  std::vector<int64_t> opidx;
  std::vector<int32_t> adj_ptr, adj;
  // the order the owners run in: a reverse Cuthill-McKee order of the pair
  // graph, so that the owners in flight together are neighbours and read the
  // same partner rows and spectra; each owner's entries follow it too
  std::vector<int32_t> operm;
};

struct ace_ctx {
  hipStream_t stream = nullptr;
  int device = 0;
  std::string err;
  size_t ws_total = 0, ws_cap = 0;
  uint64_t ws_gen = 0;  // bumped whenever a workspace is reallocated
  std::map<std::string, Buf> bufs;
  std::map<int, Buf> twiddles;       // key: N*2 + prec
  std::map<int, PairShape> shapes;   // key: N*2 + prec
  std::map<int, int> max_packs;      // key: N*2 + prec
  // Schedules are shared: a call holds its own references, so trimming the
  // cache while a batched call builds the schedules of its other systems
  // never frees one that is still in use.
  std::map<ScheduleKey, std::shared_ptr<const Schedule>> schedules;
  EventRecorder rec;
  bool profiling = false;
  bool owner_order = true;  // owners dispatched in the schedule's order (ACE_OWNER_ORDER=0: index order)
  EventRecorder* R() { return profiling ? &rec : nullptr; }
  // batched form
  hipStream_t bstream = nullptr;
  hipEvent_t bev_in = nullptr, bev_out = nullptr;
  // branches of the batched tails (default priority), with their fork/join events
  static constexpr int kTailBranches = 4;
  hipStream_t bbr[kTailBranches] = {};
  hipEvent_t bev_fork = nullptr, bev_join[kTailBranches] = {};
  std::map<uint64_t, hipGraphExec_t> graphs;
  std::vector<uint64_t> graph_order;
  int b_txv = 16, b_plan = 0, b_bpc = 8, b_layout = 3;
  size_t owner_max = size_t(96) << 30;  // resident spectra budget of the owner-computes path
};

static int fail(ace_ctx* c, int code, const char* fmt, ...) {
  char msg[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(msg, sizeof msg, fmt, ap);
  va_end(ap);
  if (c) c->err = msg;
  return code;
}

#define HIPCHK(ctx, expr)                                                                       \
  do {                                                                                          \
    hipError_t e__ = (expr);                                                                    \
    if (e__ != hipSuccess)                                                                      \
      return fail(ctx, ACE_E_HIP, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e__), __FILE__, \
                  __LINE__);                                                                    \
  } while (0)

// Grow-only named workspace buffer.
static int ws_get(ace_ctx* c, const char* name, size_t bytes, void** out) {
  Buf& b = c->bufs[name];
  if (b.bytes < bytes) {
    if (b.p) {
      (void)hipStreamSynchronize(c->stream);
      (void)hipFree(b.p);
      c->ws_total -= b.bytes;
      b.p = nullptr;
      b.bytes = 0;
    }
    if (c->ws_cap && c->ws_total + bytes > c->ws_cap)
      return fail(c, ACE_E_NOMEM, "workspace '%s' of %zu bytes exceeds ACE_WORKSPACE_MAX", name, bytes);
    if (hipMalloc(&b.p, bytes) != hipSuccess) {
      b.p = nullptr;
      return fail(c, ACE_E_NOMEM, "hipMalloc of %zu bytes for '%s' failed", bytes, name);
    }
    b.bytes = bytes;
    c->ws_total += bytes;
    ++c->ws_gen;
  }
  *out = b.p;
  return ACE_OK;
}

#define WS(ctx, name, bytes, ptr)                                   \
  do {                                                              \
    int rc__ = ws_get(ctx, name, bytes, (void**)&(ptr));            \
    if (rc__ != ACE_OK) return rc__;                                \
  } while (0)

static int check_grid(ace_ctx* c, const ace_grid* g, int norb) {
  if (!g) return fail(c, ACE_E_ARG, "grid is NULL");
  if (norb < 1 || norb > 512) return fail(c, ACE_E_ARG, "norb=%d outside [1, 512]", norb);
  for (int d = 0; d < 3; ++d)
    if (!(g->L[d] > 0.0) || !std::isfinite(g->L[d])) return fail(c, ACE_E_ARG, "box edge L[%d] must be > 0", d);
  if (g->n[0] != g->n[1] || g->n[1] != g->n[2])
    return fail(c, ACE_E_UNSUPPORTED, "only cubic grids are supported (got %d x %d x %d)", g->n[0], g->n[1], g->n[2]);
  if (!pair_supported(g->n[0]))
    return fail(c, ACE_E_UNSUPPORTED, "grid size %d not supported (use 8,12,16,24,32,48,64,80,96,100,108,120,160)",
                g->n[0]);
  return ACE_OK;
}

static int64_t grid_size(const ace_grid* g) { return int64_t(g->n[0]) * g->n[1] * g->n[2]; }
static double grid_dv(const ace_grid* g) { return g->L[0] * g->L[1] * g->L[2] / double(grid_size(g)); }

static int twiddles(ace_ctx* c, int N, int prec, const void** out) {
  const int key = N * 2 + prec;
  auto it = c->twiddles.find(key);
  if (it == c->twiddles.end()) {
    std::vector<double> d(2 * N);
    std::vector<float> f(2 * N);
    for (int m = 0; m < N; ++m) {
      const long double a = -2.0L * 3.141592653589793238462643383279502884L * (long double)m / (long double)N;
      d[2 * m] = (double)cosl(a);
      d[2 * m + 1] = (double)sinl(a);
      f[2 * m] = (float)cosl(a);
      f[2 * m + 1] = (float)sinl(a);
    }
    Buf b;
    b.bytes = prec == 0 ? d.size() * sizeof(double) : f.size() * sizeof(float);
    HIPCHK(c, hipMalloc(&b.p, b.bytes));
    HIPCHK(c, hipMemcpy(b.p, prec == 0 ? (const void*)d.data() : (const void*)f.data(), b.bytes,
                        hipMemcpyHostToDevice));
    it = c->twiddles.emplace(key, b).first;
  }
  *out = it->second.p;
  return ACE_OK;
}

static PairShape shape_for(ace_ctx* c, int prec, int N) {
  auto it = c->shapes.find(N * 2 + prec);
  if (it != c->shapes.end()) return it->second;
  return pair_default_shape(prec, N);
}

static int max_packs_for(ace_ctx* c, int prec, int N) {
  auto it = c->max_packs.find(N * 2 + prec);
  if (it != c->max_packs.end()) return it->second;
  return 64;
}

// Split the pair list into conflict-free rounds (no orbital twice in a round):
// greedy maximal matchings, each round scanning the remaining pairs in order
// of decreasing endpoint degree so that the busiest orbitals are served first.
static void make_schedule(const std::vector<int32_t>& pr, int64_t npairs, int norb, int max_packs, Schedule& S) {
  std::vector<int64_t> rem(npairs);
  for (int64_t p = 0; p < npairs; ++p) rem[p] = p;
  std::vector<int> deg(norb), used(norb, -1);
  std::vector<int64_t> next, order;
  int round = 0;
  while (!rem.empty()) {
    std::fill(deg.begin(), deg.end(), 0);
    for (int64_t p : rem) {
      deg[pr[2 * p]]++;
      if (pr[2 * p] != pr[2 * p + 1]) deg[pr[2 * p + 1]]++;
    }
    // counting sort by decreasing deg[i] + deg[j] (stable)
    int maxk = 0;
    for (int64_t p : rem) maxk = std::max(maxk, deg[pr[2 * p]] + deg[pr[2 * p + 1]]);
    std::vector<int64_t> cnt(maxk + 2, 0);
    for (int64_t p : rem) cnt[maxk - (deg[pr[2 * p]] + deg[pr[2 * p + 1]]) + 1]++;
    for (int k = 1; k < maxk + 2; ++k) cnt[k] += cnt[k - 1];
    order.assign(rem.size(), 0);
    for (int64_t p : rem) order[cnt[maxk - (deg[pr[2 * p]] + deg[pr[2 * p + 1]])]++] = p;
    next.clear();
    std::vector<int64_t> sel;
    for (int64_t p : order) {
      const int i = pr[2 * p], j = pr[2 * p + 1];
      if (used[i] != round && used[j] != round) {
        used[i] = used[j] = round;
        sel.push_back(p);
      } else {
        next.push_back(p);
      }
    }
    std::sort(sel.begin(), sel.end());  // keep each round in pair order
    const int first = int(S.packs.size());
    for (size_t q = 0; q < sel.size(); q += 2) {
      Pack pk;
      pk.ia = pr[2 * sel[q]];
      pk.ja = pr[2 * sel[q] + 1];
      if (q + 1 < sel.size()) {
        pk.ib = pr[2 * sel[q + 1]];
        pk.jb = pr[2 * sel[q + 1] + 1];
      } else {
        pk.ib = -1;
        pk.jb = -1;
      }
      S.packs.push_back(pk);
      S.pidx.push_back(sel[q]);
      S.pidx.push_back(q + 1 < sel.size() ? sel[q + 1] : -1);
    }
    const int np = int(S.packs.size()) - first;
    S.round_first.push_back(first);
    S.round_count.push_back(np);
    for (int off = 0; off < np; off += max_packs) {
      const int cntp = std::min(max_packs, np - off);
      int npr = 0;
      for (int q = first + off; q < first + off + cntp; ++q) npr += S.packs[q].jb >= 0 ? 2 : 1;
      S.launches.push_back({first + off, cntp, npr});
      S.max_launch = std::max(S.max_launch, cntp);
    }
    rem.swap(next);
    ++round;
  }
}

// Validate a host copy of a pair list and return its (cached) schedule.
// Reverse Cuthill-McKee order of the orbitals over the pair graph: breadth
// first from a vertex of least degree, neighbours in order of increasing
// degree (then index), each component in turn, the whole order reversed.
static std::vector<int32_t> rcm_order(int n, const std::vector<int32_t>& adj_ptr, const std::vector<int32_t>& adj) {
  std::vector<int> deg(size_t(n), 0);
  for (int k = 0; k < n; ++k)
    for (int a = adj_ptr[size_t(k)]; a < adj_ptr[size_t(k) + 1]; ++a)
      if (adj[size_t(2 * a + 1)] != k) ++deg[size_t(k)];
  std::vector<char> seen(size_t(n), 0);
  std::vector<int32_t> order;
  order.reserve(size_t(n));
  std::vector<int32_t> nb;
  while (int(order.size()) < n) {
    int s = -1;
    for (int k = 0; k < n; ++k)
      if (!seen[size_t(k)] && (s < 0 || deg[size_t(k)] < deg[size_t(s)])) s = k;
    seen[size_t(s)] = 1;
    size_t head = order.size();
    order.push_back(s);
    while (head < order.size()) {
      const int v = order[head++];
      nb.clear();
      for (int a = adj_ptr[size_t(v)]; a < adj_ptr[size_t(v) + 1]; ++a) {
        const int j = adj[size_t(2 * a + 1)];
        if (!seen[size_t(j)]) {
          seen[size_t(j)] = 1;
          nb.push_back(j);
        }
      }
      std::sort(nb.begin(), nb.end(), [&](int x, int y) {
        return deg[size_t(x)] != deg[size_t(y)] ? deg[size_t(x)] < deg[size_t(y)] : x < y;
      });
      order.insert(order.end(), nb.begin(), nb.end());
    }
  }
  std::reverse(order.begin(), order.end());
  return order;
}

static void make_owner_schedule(const std::vector<int32_t>& pr, int64_t npairs, int norb, Schedule& S) {
  const int64_t npk = (npairs + 1) / 2;
  S.opacks.resize(size_t(npk));
  S.opidx.assign(size_t(2 * npk), -1);
  for (int64_t p = 0; p < npk; ++p) {
    Pack& pk = S.opacks[size_t(p)];
    pk.ia = pr[4 * p];
    pk.ja = pr[4 * p + 1];
    S.opidx[size_t(2 * p)] = 2 * p;
    if (2 * p + 1 < npairs) {
      pk.ib = pr[4 * p + 2];
      pk.jb = pr[4 * p + 3];
      S.opidx[size_t(2 * p + 1)] = 2 * p + 1;
    } else {
      pk.ib = -1;
      pk.jb = -1;
    }
  }
  std::vector<int32_t> deg(size_t(norb) + 1, 0);
  for (int64_t t = 0; t < npairs; ++t) {
    ++deg[size_t(pr[2 * t])];
    if (pr[2 * t + 1] != pr[2 * t]) ++deg[size_t(pr[2 * t + 1])];
  }
  S.adj_ptr.assign(size_t(norb) + 1, 0);
  for (int k = 0; k < norb; ++k) S.adj_ptr[size_t(k) + 1] = S.adj_ptr[size_t(k)] + deg[size_t(k)];
  S.adj.assign(size_t(2) * S.adj_ptr[size_t(norb)], 0);
  std::vector<int32_t> fill(S.adj_ptr.begin(), S.adj_ptr.end() - 1);
  for (int64_t t = 0; t < npairs; ++t) {
    const int i = pr[2 * t], j = pr[2 * t + 1];
    int32_t a = fill[size_t(i)]++;
    S.adj[size_t(2 * a)] = int32_t(t);
    S.adj[size_t(2 * a + 1)] = j;
    if (j != i) {
      a = fill[size_t(j)]++;
      S.adj[size_t(2 * a)] = int32_t(t);
      S.adj[size_t(2 * a + 1)] = i;
    }
  }
  // the owners' order, and each owner's entries by their partner's place in it
  S.operm = rcm_order(norb, S.adj_ptr, S.adj);
  std::vector<int32_t> rank(static_cast<size_t>(norb));
  for (int p = 0; p < norb; ++p) rank[size_t(S.operm[size_t(p)])] = p;
  std::vector<std::pair<int32_t, int32_t>> ent;
  for (int k = 0; k < norb; ++k) {
    const int a0 = S.adj_ptr[size_t(k)], a1 = S.adj_ptr[size_t(k) + 1];
    ent.clear();
    for (int a = a0; a < a1; ++a) ent.emplace_back(S.adj[size_t(2 * a)], S.adj[size_t(2 * a + 1)]);
    std::stable_sort(ent.begin(), ent.end(), [&](const std::pair<int32_t, int32_t>& x,
                                                 const std::pair<int32_t, int32_t>& y) {
      return rank[size_t(x.second)] < rank[size_t(y.second)];
    });
    for (int a = a0; a < a1; ++a) {
      S.adj[size_t(2 * a)] = ent[size_t(a - a0)].first;
      S.adj[size_t(2 * a + 1)] = ent[size_t(a - a0)].second;
    }
  }
}


static int schedule_for(ace_ctx* c, const std::vector<int32_t>& pr, int64_t npairs, int norb, int max_packs,
                        std::shared_ptr<const Schedule>* out) {
  uint64_t h = 1469598103934665603ull;
  std::vector<uint8_t> seen(size_t(norb) * norb, 0);
  for (int64_t p = 0; p < npairs; ++p) {
    const int i = pr[2 * p], j = pr[2 * p + 1];
    if (i < 0 || j < i || j >= norb)
      return fail(c, ACE_E_ARG, "pair %lld = (%d, %d) not 0 <= i <= j < norb", (long long)p, i, j);
    if (seen[size_t(i) * norb + j]) return fail(c, ACE_E_ARG, "pair (%d, %d) listed twice", i, j);
    seen[size_t(i) * norb + j] = 1;
    h = (h ^ uint64_t(uint32_t(i) * 65599u + uint32_t(j))) * 1099511628211ull;
  }
  ScheduleKey key{npairs, norb, h ^ (uint64_t(max_packs) << 40)};
  auto sit = c->schedules.find(key);
  if (sit == c->schedules.end()) {
    if (c->schedules.size() > 64) c->schedules.clear();
    auto S = std::make_shared<Schedule>();
    make_schedule(pr, npairs, norb, max_packs, *S);
    make_owner_schedule(pr, npairs, norb, *S);
    sit = c->schedules.emplace(key, std::move(S)).first;
  }
  *out = sit->second;
  return ACE_OK;
}

extern "C" {

const char* ace_version(void) { return "libace 0.1 (gfx950)"; }

static int scratch_on_device(ace_ctx* c, double** out);

int ace_create(ace_ctx** out, void* stream) {
  if (!out) return ACE_E_ARG;
  ace_ctx* c = new ace_ctx();
  c->stream = (hipStream_t)stream;
  // Without a visible device the context still validates arguments; the
  // first HIP call then reports ACE_E_HIP.
  if (hipGetDevice(&c->device) != hipSuccess) c->device = -1;
  // the allocation-free entry point's scratch address on this device, looked
  // up at set-up; a failure here is reported by that entry point's first call
  if (c->device >= 0) {
    double* sp = nullptr;
    if (scratch_on_device(c, &sp) != ACE_OK) c->err.clear();
  }
  if (const char* cap = getenv("ACE_WORKSPACE_MAX")) c->ws_cap = (size_t)strtoull(cap, nullptr, 10);
  if (const char* om = getenv("ACE_OWNER_SPECTRA_MAX")) c->owner_max = (size_t)strtoull(om, nullptr, 10);
  if (const char* oo = getenv("ACE_OWNER_ORDER")) c->owner_order = std::atoi(oo) != 0;
  *out = c;
  return ACE_OK;
}

int ace_destroy(ace_ctx* c) {
  if (!c) return ACE_OK;
  (void)hipStreamSynchronize(c->stream);
  for (auto& kv : c->bufs)
    if (kv.second.p) (void)hipFree(kv.second.p);
  for (auto& kv : c->twiddles)
    if (kv.second.p) (void)hipFree(kv.second.p);
  for (auto e : c->rec.pool) (void)hipEventDestroy(e);
  for (auto& kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
  if (c->bev_in) (void)hipEventDestroy(c->bev_in);
  if (c->bev_out) (void)hipEventDestroy(c->bev_out);
  if (c->bev_fork) (void)hipEventDestroy(c->bev_fork);
  for (int b = 0; b < ace_ctx::kTailBranches; ++b) {
    if (c->bev_join[b]) (void)hipEventDestroy(c->bev_join[b]);
    if (c->bbr[b]) (void)hipStreamDestroy(c->bbr[b]);
  }
  if (c->bstream) (void)hipStreamDestroy(c->bstream);
  delete c;
  return ACE_OK;
}

int ace_release_workspace(ace_ctx* c) {
  if (!c) return ACE_E_ARG;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (c->bstream) HIPCHK(c, hipStreamSynchronize(c->bstream));
  for (int b = 0; b < ace_ctx::kTailBranches; ++b)
    if (c->bbr[b]) HIPCHK(c, hipStreamSynchronize(c->bbr[b]));
  for (auto& kv : c->bufs)
    if (kv.second.p) (void)hipFree(kv.second.p);
  c->bufs.clear();
  c->ws_total = 0;
  // captured graphs hold workspace pointers
  for (auto& kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
  c->graphs.clear();
  c->graph_order.clear();
  ++c->ws_gen;
  return ACE_OK;
}

const char* ace_last_error(const ace_ctx* c) { return c ? c->err.c_str() : "null context"; }

int ace_set_stream(ace_ctx* c, void* stream) {
  if (!c) return ACE_E_ARG;
  c->stream = (hipStream_t)stream;
  return ACE_OK;
}

int ace_profile_enable(ace_ctx* c, int enable) {
  if (!c) return ACE_E_ARG;
  if (!enable) rec_collect(&c->rec, c->stream);
  c->profiling = enable != 0;
  return ACE_OK;
}

int ace_profile_classes(ace_ctx* c, unsigned mask) {
  if (!c) return ACE_E_ARG;
  if (mask >> KC_COUNT) return fail(c, ACE_E_ARG, "profile class mask 0x%x names classes beyond %d", mask, KC_COUNT - 1);
  rec_collect(&c->rec, c->stream);
  c->rec.mask = mask;
  return ACE_OK;
}

int ace_profile_read(ace_ctx* c, int cls, int64_t* launches, double* total_ms, double* units, int reset) {
  if (!c || cls < 0 || cls >= KC_COUNT) return fail(c, ACE_E_ARG, "bad profile class %d", cls);
  rec_collect(&c->rec, c->stream);
  if (launches) *launches = c->rec.count[cls];
  if (total_ms) *total_ms = c->rec.total_ms[cls];
  if (units) *units = c->rec.total_units[cls];
  if (reset) {
    c->rec.count[cls] = 0;
    c->rec.total_ms[cls] = 0.0;
    c->rec.total_units[cls] = 0.0;
  }
  return ACE_OK;
}

int ace_set_pair_shape(ace_ctx* c, int prec, int n, int fused, int max_packs) {
  if (!c || (prec != 0 && prec != 1) || !pair_supported(n) || max_packs < 1 || fused < 0 || fused > 3)
    return fail(c, ACE_E_ARG, "bad pair shape");
  PairShape sh = pair_default_shape(prec, n);
  sh.fused_xy = (fused >= 2 && fused <= 3 && pair_r2c_fits(prec, n)) ? fused
                : (fused == 1 && pair_fused_fits(prec, n)) ? 1 : 0;
  c->shapes[n * 2 + prec] = sh;
  c->max_packs[n * 2 + prec] = max_packs;
  c->schedules.clear();
  return ACE_OK;
}

int ace_get_pair_shape(ace_ctx* c, int prec, int n, int* fused, int* max_packs) {
  if (!c || (prec != 0 && prec != 1) || !pair_supported(n)) return fail(c, ACE_E_ARG, "bad pair shape query");
  PairShape sh = shape_for(c, prec, n);
  if (fused) *fused = sh.fused_xy;
  if (max_packs) *max_packs = max_packs_for(c, prec, n);
  return ACE_OK;
}

// ------------------------------------------------------------------ (a) localize
// Loewdin step on the columns `pivots`: U = A_C (A_C^T A_C)^-1/2 into U
// (nullable) and phi_k = sum_i psi_i U_ik.  AC, X, G, Z are norb x norb
// workspaces, dev one double.
static int lowdin(ace_ctx* c, int norb, int64_t ng, const double* psi, const int32_t* pivots, double* AC, double* X,
                  double* G, double* Z, double* dev, double* phi, double* U) {
  hipStream_t s = c->stream;
  // Loewdin rotation U = A_C (A_C^T A_C)^-1/2 = polar factor of A_C, by the
  // Newton-Schulz iteration X <- X (3 I - X^T X) / 2 from X = A_C scaled so
  // that every singular value is at most 1 (max row sum of |A_C^T A_C|).
  launch_gather_cols(psi, norb, ng, pivots, AC, s);
  HIPCHK(c, hipMemcpyAsync(X, AC, size_t(norb) * norb * sizeof(double), hipMemcpyDeviceToDevice, s));
  HIPCHK(c, gemm_ls(0, true, false, X, norb, X, norb, G, norb, norb, norb, norb, 1.0, s, nullptr));
  launch_scale_inf(X, G, norb, s);
  // Each iteration forms G = X^T X, which also measures max|X^T X - I|; it is
  // read back every second iteration from the fourth on.  Once below 1e-11,
  // two more iterations (the first reusing that G) take the quadratically
  // converging iterate to rounding.
  int converged_at = -1;
  for (int it = 0; it < 200; ++it) {
    HIPCHK(c, gemm_ls(0, true, false, X, norb, X, norb, G, norb, norb, norb, norb, 1.0, s, nullptr));
    if (it >= 4 && it % 2 == 0) {
      launch_dev_identity(G, norb, dev, s);
      double h = 0.0;
      HIPCHK(c, hipMemcpyAsync(&h, dev, sizeof(double), hipMemcpyDeviceToHost, s));
      HIPCHK(c, hipStreamSynchronize(s));
      if (!std::isfinite(h)) return fail(c, ACE_E_NONFINITE, "non-finite Loewdin iteration (singular A_C?)");
      if (h < 1e-11) {
        converged_at = it;
        break;
      }
    }
    HIPCHK(c, gemm_ls(0, false, false, X, norb, G, norb, Z, norb, norb, norb, norb, 1.0, s, nullptr));
    launch_ns_combine(X, Z, X, int64_t(norb) * norb, s);
  }
  if (converged_at < 0) return fail(c, ACE_E_NONFINITE, "Loewdin polar iteration did not converge");
  for (int j = 0; j < 2; ++j) {
    if (j > 0) HIPCHK(c, gemm_ls(0, true, false, X, norb, X, norb, G, norb, norb, norb, norb, 1.0, s, nullptr));
    HIPCHK(c, gemm_ls(0, false, false, X, norb, G, norb, Z, norb, norb, norb, norb, 1.0, s, nullptr));
    launch_ns_combine(X, Z, X, int64_t(norb) * norb, s);
  }
  // phi_k = sum_i psi_i U_ik
  HIPCHK(c, gemm_ls(0, true, false, X, norb, psi, ng, phi, ng, norb, norb, ng, 1.0, s, c->R()));
  if (U) HIPCHK(c, hipMemcpyAsync(U, X, size_t(norb) * norb * sizeof(double), hipMemcpyDeviceToDevice, s));
  return ACE_OK;
}

int ace_localize(ace_ctx* c, const ace_grid* g, int norb, const double* psi, double* phi, int32_t* pivots,
                 double* U) {
  if (!c) return ACE_E_ARG;
  int rc = check_grid(c, g, norb);
  if (rc) return rc;
  if (!psi || !phi || !pivots) return fail(c, ACE_E_ARG, "psi, phi and pivots must be non-NULL");
  const int64_t ng = grid_size(g);
  if (ng < norb) return fail(c, ACE_E_ARG, "grid smaller than the number of orbitals");
  hipStream_t s = c->stream;
  rec_begin(c->R(), ST_LOCALIZE, s);
  double *res, *pv, *Q, *q, *AC, *X, *G, *Z, *dev, *Ub, *pres, *Apool, *tvals, *tmax, *Lc;
  int64_t *pi, *pcnt;
  int32_t* pool;
  unsigned* hist;
  int* iv;  // [0] k, [1] stop, [2] pool size
  const int nblk_full = qrcp_blocks(ng);
  // candidate pool size (measured: 3072 columns at 128 and 256 orbitals
  // localize 4.1 -> 3.5 and 14.5 -> 14.3 ms against 2048, fewer redraws)
  const int pmax = std::max(3072, 12 * norb);
  const int nblk_pool = qrcp_blocks(pmax);
  const int64_t rchunk = std::min<int64_t>(ng, 65536);  // refresh chunk (grid columns)
  const int nbp = pool_blocks(ng);
  WS(c, "res", ng * sizeof(double), res);
  // block candidates: 8 per block of the full sweep, 1 per block of the pool steps
  // (the pool steps double buffer their block candidates)
  const size_t ncand = std::max<size_t>(size_t(nblk_full) * 8, 2 * size_t(qrcp_pool_blocks(pmax)));
  WS(c, "pv", ncand * sizeof(double), pv);
  WS(c, "pi", ncand * sizeof(int64_t), pi);
  WS(c, "Q", size_t(norb) * norb * sizeof(double), Q);
  WS(c, "q", size_t(norb) * sizeof(double), q);
  WS(c, "AC", size_t(norb) * norb * sizeof(double), AC);
  WS(c, "X", size_t(norb) * norb * sizeof(double), X);
  WS(c, "G", size_t(norb) * norb * sizeof(double), G);
  WS(c, "Z", size_t(norb) * norb * sizeof(double), Z);
  WS(c, "U", size_t(norb) * norb * sizeof(double), Ub);
  WS(c, "scal", 64 * sizeof(double), dev);
  WS(c, "pres", size_t(pmax) * sizeof(double), pres);
  WS(c, "pool", size_t(pmax) * sizeof(int32_t), pool);
  WS(c, "Apool", size_t(pmax) * norb * sizeof(double), Apool);
  WS(c, "hist", size_t(1 << 14) * sizeof(unsigned), hist);
  WS(c, "pcnt", size_t(nbp) * sizeof(int64_t), pcnt);
  WS(c, "tmax", size_t(nbp) * sizeof(double), tmax);
  WS(c, "tvals", 8 * sizeof(double), tvals);
  WS(c, "ivals", 64, iv);
  WS(c, "Lref", size_t(norb) * rchunk * sizeof(double), Lc);
  double* Tpool;
  WS(c, "Tpool", size_t(pmax) * norb * sizeof(double), Tpool);

  // Greedy QRCP.  A compact pool of the columns with the largest residual
  // bounds is searched step by step; a pick is certified against t_out, the
  // largest bound outside the pool, and when certification fails the bounds
  // of all columns are recomputed exactly from the picked directions and a
  // new pool is drawn.  Residual norms only decrease, so every stored bound
  // stays valid until it is recomputed.
  launch_colnorm(psi, norb, ng, res, s);
  HIPCHK(c, hipMemsetAsync(iv, 0, 64, s));
  // algorithmic bytes of one pool step per pool column: R read and written, residual read and written
  const double qbytes_pool = double(2 * norb + 2) * sizeof(double);
  int k = 0, kref = 0;  // kref: directions already folded into res
  for (int refresh = 0; k < norb; ++refresh) {
    if (k > kref) {
      // bounds: res = |a_r|^2 - |Q_k a_r|^2, downdated by the directions
      // picked since the last refresh only; then retire the pivots
      if (k - kref <= 128) {
        // one launch: the projections' squares are summed on the MFMA tile
        HIPCHK(c, refresh_bounds(Q + size_t(kref) * norb, norb, psi, ng, k - kref, norb, ng, res, s));
      } else {
        for (int64_t r0 = 0; r0 < ng; r0 += rchunk) {
          const int64_t w = std::min(rchunk, ng - r0);
          HIPCHK(c, gemm_ls(0, false, false, Q + size_t(kref) * norb, norb, psi + r0, ng, Lc, w, k - kref, norb, w,
                            1.0, s, nullptr));
          launch_refresh_res(Lc, k - kref, w, res + r0, res + r0, s);
        }
      }
      launch_retire(pivots, k, res, s);
      kref = k;
    }
    bool use_pool = refresh < 16;
    int np = 0;
    if (use_pool) {
      HIPCHK(c, hipMemsetAsync(hist, 0, size_t(1 << 14) * sizeof(unsigned), s));
      launch_pool_build(res, ng, pmax, hist, tvals, pcnt, tmax, iv + 2, tvals + 1, s);
      HIPCHK(c, hipMemcpyAsync(&np, iv + 2, sizeof(int), hipMemcpyDeviceToHost, s));
      HIPCHK(c, hipStreamSynchronize(s));
      use_pool = np > 0 && np <= pmax;
    }
    HIPCHK(c, hipMemsetAsync(iv + 1, 0, sizeof(int), s));  // clear stop
    if (use_pool) {
      launch_pool_write(res, ng, tvals, pcnt, pool, pres, s);
      launch_pool_gather(psi, norb, ng, pool, np, Apool, s);
      // the pool holds explicit residual columns R = (I - Q^T Q) A_pool:
      // project out the k directions already taken, twice for accuracy
      if (k > 0)
        for (int pass = 0; pass < 2; ++pass) {
          HIPCHK(c, gemm_ls(0, false, false, Q, norb, Apool, np, Lc, np, k, norb, np, 1.0, s, nullptr));
          HIPCHK(c, gemm_ls(0, true, false, Q, norb, Lc, np, Tpool, np, norb, k, np, -1.0, s, nullptr));
          launch_add_inplace(Apool, Tpool, int64_t(norb) * np, s);
        }
      launch_qrcp_update_r(Apool, norb, np, nullptr, pres, pv, pi, iv + 1, s);
      // one launch per step (selection repeated in every block, then the
      // update), the block candidates alternating between two halves of pv/pi;
      // steps are queued in batches, and since a batch after a certification
      // failure would only hold no-op launches the flag is checked between them
      const int nbp = qrcp_pool_blocks(np);
      int par = 0;
      for (int kk = k; kk < norb;) {
        const int kend = std::min(norb, kk + 24);
        for (; kk < kend; ++kk) {
          double* pvi = pv + size_t(par) * nbp;
          int64_t* pii = pi + size_t(par) * nbp;
          if (kk + 1 < norb) {
            rec_begin(c->R(), KC_QRCP, s);
            launch_qrcp_step_r(Apool, norb, np, iv, pvi, pii, Q, pres, pivots, pool, tvals + 1, iv + 1,
                               pv + size_t(1 - par) * nbp, pi + size_t(1 - par) * nbp, s);
            rec_end(c->R(), KC_QRCP, s, qbytes_pool * double(np));
            par ^= 1;
          } else {
            launch_qrcp_select_r(Apool, norb, np, iv, pvi, pii, Q, pres, pivots, q, pool, tvals + 1, iv + 1, s);
          }
        }
        if (kk < norb) {
          int hs = 0;
          HIPCHK(c, hipMemcpyAsync(&hs, iv + 1, sizeof(int), hipMemcpyDeviceToHost, s));
          HIPCHK(c, hipStreamSynchronize(s));
          if (hs) break;
        }
      }
    } else {
      // the whole grid is the pool: no certification needed
      launch_qrcp_update(psi, norb, ng, nullptr, res, pv, pi, iv + 1, s);
      const double qbytes = double(norb + 2) * double(ng) * sizeof(double);
      for (int kk = k; kk < norb; ++kk) {
        launch_qrcp_select(psi, norb, ng, iv, pv, pi, nblk_full, Q, res, pivots, q, nullptr, nullptr, iv + 1, s);
        if (kk + 1 < norb) {
          rec_begin(c->R(), KC_QRCP, s);
          launch_qrcp_update(psi, norb, ng, q, res, pv, pi, iv + 1, s);
          rec_end(c->R(), KC_QRCP, s, qbytes);
        }
      }
    }
    HIPCHK(c, hipGetLastError());
    int hk[2] = {0, 0};
    HIPCHK(c, hipMemcpyAsync(hk, iv, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    if (!use_pool && hk[0] < norb)
      return fail(c, ACE_E_NONFINITE, "pivot search stalled at step %d (degenerate orbitals?)", hk[0]);
    if (hk[0] <= k && refresh > 0 && !use_pool)
      return fail(c, ACE_E_NONFINITE, "pivot search made no progress at step %d", k);
    k = hk[0];
  }
  HIPCHK(c, hipGetLastError());
  rc = lowdin(c, norb, ng, psi, pivots, AC, X, G, Z, dev, phi, U);
  if (rc) return rc;
  rec_end(c->R(), ST_LOCALIZE, s);
  HIPCHK(c, hipGetLastError());
  return ACE_OK;
}

int ace_localize_pivots(ace_ctx* c, const ace_grid* g, int norb, const double* psi, const int32_t* pivots,
                        double* phi, double* U) {
  if (!c) return ACE_E_ARG;
  int rc = check_grid(c, g, norb);
  if (rc) return rc;
  if (!psi || !phi || !pivots) return fail(c, ACE_E_ARG, "psi, phi and pivots must be non-NULL");
  const int64_t ng = grid_size(g);
  if (ng < norb) return fail(c, ACE_E_ARG, "grid smaller than the number of orbitals");
  hipStream_t s = c->stream;
  // the columns are read by a gather kernel: check them on the host first
  std::vector<int32_t> hp(static_cast<size_t>(norb));
  HIPCHK(c, hipMemcpyAsync(hp.data(), pivots, size_t(norb) * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipStreamSynchronize(s));
  std::vector<int32_t> sorted(hp);
  std::sort(sorted.begin(), sorted.end());
  if (sorted.front() < 0 || int64_t(sorted.back()) >= ng)
    return fail(c, ACE_E_ARG, "pivot outside [0, %lld)", (long long)ng);
  if (std::adjacent_find(sorted.begin(), sorted.end()) != sorted.end())
    return fail(c, ACE_E_ARG, "repeated pivot column");
  rec_begin(c->R(), ST_LOCALIZE, s);
  double *AC, *X, *G, *Z, *dev;
  WS(c, "AC", size_t(norb) * norb * sizeof(double), AC);
  WS(c, "X", size_t(norb) * norb * sizeof(double), X);
  WS(c, "G", size_t(norb) * norb * sizeof(double), G);
  WS(c, "Z", size_t(norb) * norb * sizeof(double), Z);
  WS(c, "scal", 64 * sizeof(double), dev);
  rc = lowdin(c, norb, ng, psi, pivots, AC, X, G, Z, dev, phi, U);
  if (rc) return rc;
  rec_end(c->R(), ST_LOCALIZE, s);
  HIPCHK(c, hipGetLastError());
  return ACE_OK;
}

// ------------------------------------------------------------------ (a) across MD steps
int ace_localize_step(ace_ctx* c, const ace_grid* g, int norb, const double* psi, int32_t* pivots, double cond_max,
                      double* phi, double* U, ace_step_info* info) {
  if (!c) return ACE_E_ARG;
  int rc = check_grid(c, g, norb);
  if (rc) return rc;
  if (!psi || !phi || !pivots || !info) return fail(c, ACE_E_ARG, "psi, pivots, phi and info must be non-NULL");
  if (!(cond_max >= 1.0)) return fail(c, ACE_E_ARG, "cond_max must be >= 1");
  const int64_t ng = grid_size(g);
  if (ng < norb) return fail(c, ACE_E_ARG, "grid smaller than the number of orbitals");
  hipStream_t s = c->stream;
  std::vector<int32_t> hp(static_cast<size_t>(norb));
  HIPCHK(c, hipMemcpyAsync(hp.data(), pivots, size_t(norb) * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipStreamSynchronize(s));
  std::vector<int32_t> sorted(hp);
  std::sort(sorted.begin(), sorted.end());
  if (sorted.front() < 0 || int64_t(sorted.back()) >= ng)
    return fail(c, ACE_E_ARG, "pivot outside [0, %lld)", (long long)ng);
  if (std::adjacent_find(sorted.begin(), sorted.end()) != sorted.end())
    return fail(c, ACE_E_ARG, "repeated pivot column");
  // Quality of the previous columns on this step's orbitals: the Cholesky
  // factor of A_C^T A_C taken in pivot order is R^T of the QR factorization
  // of A_C, so (max_k R_kk / min_k R_kk)^2 is the diagonal ratio greedy
  // pivoting keeps small, and a lower bound on the condition number.
  double *AC, *G, *tinv;
  int* dinfo;
  WS(c, "AC", size_t(norb) * norb * sizeof(double), AC);
  WS(c, "G", size_t(norb) * norb * sizeof(double), G);
  WS(c, "tinv", 64 * 64 * sizeof(double), tinv);
  WS(c, "info", 64, dinfo);
  launch_gather_cols(psi, norb, ng, pivots, AC, s);
  HIPCHK(c, gemm_ls(0, true, false, AC, norb, AC, norb, G, norb, norb, norb, norb, 1.0, s, nullptr));
  launch_zero(dinfo, sizeof(int), s);
  launch_cholesky(G, norb, dinfo, tinv, s);
  std::vector<double> hg(size_t(norb) * norb);
  int hinfo = 0;
  HIPCHK(c, hipMemcpyAsync(hg.data(), G, hg.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipMemcpyAsync(&hinfo, dinfo, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipStreamSynchronize(s));
  double dmax = 0.0, dmin = INFINITY;
  for (int k = 0; k < norb; ++k) {
    const double d = hg[size_t(k) * norb + k];
    dmax = std::max(dmax, d);
    dmin = std::min(dmin, d);
  }
  const double cond = (hinfo == 0 && dmin > 0.0 && std::isfinite(dmax)) ? (dmax / dmin) * (dmax / dmin) : INFINITY;
  info->gram_cond = cond;
  info->pairs_added = info->pairs_removed = 0;
  if (cond <= cond_max) {
    info->reused_columns = 1;
    double *X, *Z, *dev;
    WS(c, "X", size_t(norb) * norb * sizeof(double), X);
    WS(c, "Z", size_t(norb) * norb * sizeof(double), Z);
    WS(c, "scal", 64 * sizeof(double), dev);
    rc = lowdin(c, norb, ng, psi, pivots, AC, X, G, Z, dev, phi, U);
    if (rc != ACE_E_NONFINITE) return rc;
    c->err.clear();  // the polar iteration failed on these columns: fresh SCDM below
  }
  info->reused_columns = 0;
  return ace_localize(c, g, norb, psi, phi, pivots, U);
}

// ------------------------------------------------------------------ (b) pairlist
static int pairlist_core(ace_ctx* c, const ace_grid* g, int norb, const double* phi, double rho_cut,
                         int64_t capacity, int32_t* pairs, double* overlap, int64_t* npairs);

int ace_pairlist(ace_ctx* c, const ace_grid* g, int norb, const double* phi, double rho_cut, int64_t capacity,
                 int32_t* pairs, double* overlap, int64_t* npairs) {
  if (!c) return ACE_E_ARG;
  int rc = check_grid(c, g, norb);
  if (rc) return rc;
  return pairlist_core(c, g, norb, phi, rho_cut, capacity, pairs, overlap, npairs);
}

// O = dV |A| |A|^T over the rows of A (norb of them), compacted at rho_cut.
static int pairlist_core(ace_ctx* c, const ace_grid* g, int norb, const double* phi, double rho_cut,
                         int64_t capacity, int32_t* pairs, double* overlap, int64_t* npairs) {
  if (!phi || !pairs || !npairs) return fail(c, ACE_E_ARG, "phi, pairs and npairs must be non-NULL");
  if (capacity < 0) return fail(c, ACE_E_ARG, "negative capacity");
  if (!std::isfinite(rho_cut)) return fail(c, ACE_E_ARG, "rho_cut must be finite");
  const int64_t ng = grid_size(g);
  hipStream_t s = c->stream;
  rec_begin(c->R(), ST_PAIRLIST, s);
  double *part, *O;
  int64_t* cnt;
  int64_t kchunk;
  const int64_t nsplit = gemm_nt_nsplit(norb, norb, ng, &kchunk);
  WS(c, "mpart", size_t(nsplit) * norb * norb * sizeof(double), part);
  WS(c, "O", size_t(norb) * norb * sizeof(double), O);
  WS(c, "cnt", 64, cnt);
  HIPCHK(c, gemm_nt(0, 1, phi, ng, phi, ng, norb, norb, ng, grid_dv(g), part, O, s, c->R(), true));
  launch_compact_pairs(O, norb, rho_cut, capacity, pairs, overlap, cnt, s);
  int64_t h = 0;
  HIPCHK(c, hipMemcpyAsync(&h, cnt, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  rec_end(c->R(), ST_PAIRLIST, s);
  HIPCHK(c, hipStreamSynchronize(s));
  *npairs = h;
  if (h > capacity) return fail(c, ACE_E_CAPACITY, "%lld pairs kept but capacity is %lld", (long long)h,
                                (long long)capacity);
  return ACE_OK;
}

// The screening with the kept count left in device memory and no host
// synchronization, for callers that queue the screening and the build without
// waiting (graph capture after a first call has grown the workspaces).
int ace_pairlist_device(ace_ctx* c, const ace_grid* g, int norb, const double* phi, double rho_cut,
                        int64_t capacity, int32_t* pairs, double* overlap, int64_t* npairs_dev) {
  if (!c) return ACE_E_ARG;
  int rc = check_grid(c, g, norb);
  if (rc) return rc;
  if (!phi || !pairs || !npairs_dev) return fail(c, ACE_E_ARG, "phi, pairs and npairs must be non-NULL");
  if (capacity < 0) return fail(c, ACE_E_ARG, "negative capacity");
  if (!std::isfinite(rho_cut)) return fail(c, ACE_E_ARG, "rho_cut must be finite");
  const int64_t ng = grid_size(g);
  hipStream_t s = c->stream;
  double *part, *O;
  int64_t kchunk;
  const int64_t nsplit = gemm_nt_nsplit(norb, norb, ng, &kchunk);
  WS(c, "mpart", size_t(nsplit) * norb * norb * sizeof(double), part);
  WS(c, "O", size_t(norb) * norb * sizeof(double), O);
  HIPCHK(c, gemm_nt(0, 1, phi, ng, phi, ng, norb, norb, ng, grid_dv(g), part, O, s, nullptr, true));
  launch_compact_pairs(O, norb, rho_cut, capacity, pairs, overlap, npairs_dev, s);
  HIPCHK(c, hipGetLastError());
  return ACE_OK;
}

// Re-screening at the next MD step against the previous step's list.  With
// the previous step's columns kept (ace_localize_step), orbital k of this
// step continues orbital k of the last one, so the two lists compare pair by
// pair: the call reports how many pairs crossed rho_cut in each direction.
// An unchanged list is bitwise the previous one, and the build then finds
// the list's schedule in the context's cache.
int ace_pairlist_step(ace_ctx* c, const ace_grid* g, int norb, const double* phi, double rho_cut,
                      const int32_t* prev_pairs, int64_t nprev, int64_t capacity, int32_t* pairs, double* overlap,
                      int64_t* npairs, ace_step_info* info) {
  if (!c) return ACE_E_ARG;
  if (!info || (nprev > 0 && !prev_pairs) || nprev < 0)
    return fail(c, ACE_E_ARG, "info must be non-NULL and prev_pairs hold nprev >= 0 pairs");
  if (nprev > int64_t(norb) * (norb + 1) / 2) return fail(c, ACE_E_ARG, "nprev above norb (norb + 1) / 2");
  hipStream_t s = c->stream;
  std::vector<int32_t> hprev(size_t(2 * nprev));
  if (nprev > 0) {
    HIPCHK(c, hipMemcpyAsync(hprev.data(), prev_pairs, hprev.size() * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
  }
  for (int64_t t = 0; t < nprev; ++t) {
    const int32_t i = hprev[size_t(2 * t)], j = hprev[size_t(2 * t + 1)];
    if (i < 0 || j < i || j >= norb) return fail(c, ACE_E_ARG, "previous pair %lld = (%d, %d) out of range",
                                                 (long long)t, i, j);
    if (t > 0) {
      const int32_t pi = hprev[size_t(2 * t - 2)], pj = hprev[size_t(2 * t - 1)];
      if (i < pi || (i == pi && j <= pj)) return fail(c, ACE_E_ARG, "previous pairs not sorted by (i, j)");
    }
  }
  int rc = ace_pairlist(c, g, norb, phi, rho_cut, capacity, pairs, overlap, npairs);
  if (rc) return rc;
  const int64_t n = *npairs;
  std::vector<int32_t> hnew(size_t(2 * n));
  if (n > 0) {
    HIPCHK(c, hipMemcpyAsync(hnew.data(), pairs, hnew.size() * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
  }
  // merge of two lists sorted by (i, j)
  int64_t a = 0, b = 0, added = 0, removed = 0;
  auto key = [](const std::vector<int32_t>& v, int64_t t) {
    return (int64_t(v[size_t(2 * t)]) << 32) | uint32_t(v[size_t(2 * t + 1)]);
  };
  while (a < nprev || b < n) {
    if (b >= n || (a < nprev && key(hprev, a) < key(hnew, b))) { ++removed; ++a; }
    else if (a >= nprev || key(hnew, b) < key(hprev, a)) { ++added; ++b; }
    else { ++a; ++b; }
  }
  info->pairs_added = added;
  info->pairs_removed = removed;
  return ACE_OK;
}

// ------------------------------------------------------------------ (c)-(e) build
static int build_impl(ace_ctx* c, const ace_grid* g, int norb, const double* phi, const int32_t* pairs,
                      int64_t npairs, int kernel, double omega, int prec, double* xi, double* Mout, double* Wout,
                      double* ex, double* pair_energy);

int ace_build(ace_ctx* c, const ace_grid* g, int norb, const double* phi, const int32_t* pairs, int64_t npairs,
              int kernel, double omega, int prec, double* xi, double* Mout, double* Wout, double* ex,
              double* pair_energy) {
  if (!c) return ACE_E_ARG;
  if (!xi) return fail(c, ACE_E_ARG, "xi must be non-NULL");
  return build_impl(c, g, norb, phi, pairs, npairs, kernel, omega, prec, xi, Mout, Wout, ex, pair_energy);
}

int ace_pair_energies(ace_ctx* c, const ace_grid* g, int norb, const double* phi, const int32_t* pairs,
                      int64_t npairs, int kernel, double omega, int prec, double* e) {
  if (!c) return ACE_E_ARG;
  if (!e) return fail(c, ACE_E_ARG, "e must be non-NULL");
  return build_impl(c, g, norb, phi, pairs, npairs, kernel, omega, prec, nullptr, nullptr, nullptr, nullptr, e);
}

static int build_impl(ace_ctx* c, const ace_grid* g, int norb, const double* phi, const int32_t* pairs,
                      int64_t npairs, int kernel, double omega, int prec, double* xi, double* Mout, double* Wout,
                      double* ex, double* pair_energy) {
  int rc = check_grid(c, g, norb);
  if (rc) return rc;
  if (!phi || !pairs) return fail(c, ACE_E_ARG, "phi and pairs must be non-NULL");
  if (kernel != ACE_KERNEL_COULOMB && kernel != ACE_KERNEL_ERFC) return fail(c, ACE_E_ARG, "unknown kernel %d", kernel);
  if (kernel == ACE_KERNEL_ERFC && !(omega > 0.0)) return fail(c, ACE_E_ARG, "omega must be > 0 for erfc");
  if (prec != ACE_FP64 && prec != ACE_FP32) return fail(c, ACE_E_ARG, "unknown precision %d", prec);
  const int64_t maxp = int64_t(norb) * (norb + 1) / 2;
  if (npairs < 1 || npairs > maxp) return fail(c, ACE_E_ARG, "npairs=%lld outside [1, %lld]", (long long)npairs,
                                               (long long)maxp);
  const int N = g->n[0];
  const int64_t ng = grid_size(g);
  const double dV = grid_dv(g);
  hipStream_t s = c->stream;
  EventRecorder* R = c->R();

  for (auto& o : c->rec.open) o.clear();
  // pair list to the host for validation and scheduling
  std::vector<int32_t> pr(size_t(2 * npairs));
  HIPCHK(c, hipMemcpyAsync(pr.data(), pairs, pr.size() * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipStreamSynchronize(s));
  const int mp = max_packs_for(c, prec, N);
  std::shared_ptr<const Schedule> Sp;
  rc = schedule_for(c, pr, npairs, norb, mp, &Sp);
  if (rc) return rc;
  const Schedule& S = *Sp;
  const int npk = int(S.packs.size());
  rec_begin(R, ST_BUILD, s);

  const size_t es = prec == 0 ? sizeof(double) : sizeof(float);
  const PairShape sh = shape_for(c, prec, N);
  // owner-computes W when every pair's half spectrum fits the budget
  const int64_t onpk = int64_t(S.opacks.size());
  const size_t slot_bytes = size_t(N) * N * (N / 2 + 1) * 2 * es;
  // ... and when the spectra, beyond what the workspace already holds, take
  // at most 60% of the free device memory (a fuller device slows down)
  bool owner = sh.fused_xy == 3 && pair_r2c_fits(prec, N) && size_t(2 * onpk) * slot_bytes <= c->owner_max;
  if (owner) {
    const size_t need = size_t(2 * onpk) * slot_bytes;
    auto it = c->bufs.find("spec");
    const size_t have = it == c->bufs.end() ? 0 : it->second.bytes;
    size_t freeb = 0, totb = 0;
    if (need > have && hipMemGetInfo(&freeb, &totb) == hipSuccess)
      owner = double(need) <= 0.6 * double(freeb + have);
  }
  const int nblk = owner ? pair_owner_ntile(prec, N) : pair_energy_blocks(N, sh);
  void *W, *spec, *phiw;
  Pack* dpk;
  int64_t* dpidx;
  int32_t *dadjp = nullptr, *dadj = nullptr, *doperm = nullptr;
  double *epart = nullptr, *part, *Mraw, *Lb, *Li, *scal;
  void* vtab = nullptr;
  int* info;
  // W lives in the workspace, or directly in the caller's FP64 output when no
  // projectors follow (exact exchange)
  if (xi || (Wout && prec == 1)) WS(c, "W", size_t(norb) * ng * es, W);
  else W = Wout;
  if (owner) {
    WS(c, "spec", size_t(2 * onpk) * slot_bytes, spec);
    WS(c, "packs", size_t(onpk) * sizeof(Pack), dpk);
    WS(c, "pidx", size_t(onpk) * 2 * sizeof(int64_t), dpidx);
    WS(c, "adjp", S.adj_ptr.size() * sizeof(int32_t), dadjp);
    WS(c, "adj", std::max<size_t>(S.adj.size(), 2) * sizeof(int32_t), dadj);
    WS(c, "operm", size_t(norb) * sizeof(int32_t), doperm);
    if (pair_energy) WS(c, "epart", size_t(onpk) * nblk * 2 * sizeof(double), epart);
    WS(c, "vtab", size_t(N / 2 + 1) * (N / 2 + 1) * (N / 2 + 1) * es, vtab);
  } else {
    WS(c, "spec", size_t(S.max_launch) * pair_spec_elems(prec, N, sh) * 2 * es, spec);
    WS(c, "packs", size_t(npk) * sizeof(Pack), dpk);
    WS(c, "pidx", size_t(npk) * 2 * sizeof(int64_t), dpidx);
    if (pair_energy) WS(c, "epart", size_t(S.max_launch) * nblk * 2 * sizeof(double), epart);
  }
  int64_t kchunk;
  const int64_t nsplit = gemm_nt_nsplit(norb, norb, ng, &kchunk);
  WS(c, "mpart", size_t(nsplit) * norb * norb * sizeof(double), part);
  WS(c, "Mraw", size_t(norb) * norb * sizeof(double), Mraw);
  WS(c, "Lc", size_t(norb) * norb * sizeof(double), Lb);
  WS(c, "Linv", size_t(norb) * norb * sizeof(double), Li);
  WS(c, "scal", 64 * sizeof(double), scal);
  WS(c, "info", 64, info);
  double* tinv;
  WS(c, "tinv", 64 * 64 * sizeof(double), tinv);
  if (prec == 1) WS(c, "phi32", size_t(norb) * ng * sizeof(float), phiw);
  else phiw = (void*)phi;
  const void* tw;
  rc = twiddles(c, N, prec, &tw);
  if (rc) return rc;

  if (owner) {
    HIPCHK(c, hipMemcpyAsync(dpk, S.opacks.data(), size_t(onpk) * sizeof(Pack), hipMemcpyHostToDevice, s));
    HIPCHK(c, hipMemcpyAsync(dpidx, S.opidx.data(), size_t(onpk) * 2 * sizeof(int64_t), hipMemcpyHostToDevice, s));
    HIPCHK(c, hipMemcpyAsync(dadjp, S.adj_ptr.data(), S.adj_ptr.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
    if (!S.adj.empty())
      HIPCHK(c, hipMemcpyAsync(dadj, S.adj.data(), S.adj.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
    HIPCHK(c, hipMemcpyAsync(doperm, S.operm.data(), size_t(norb) * sizeof(int32_t), hipMemcpyHostToDevice, s));
  } else {
    HIPCHK(c, hipMemcpyAsync(dpk, S.packs.data(), size_t(npk) * sizeof(Pack), hipMemcpyHostToDevice, s));
    HIPCHK(c, hipMemcpyAsync(dpidx, S.pidx.data(), size_t(npk) * 2 * sizeof(int64_t), hipMemcpyHostToDevice, s));
  }
  if (prec == 1) launch_d2f(phi, (float*)phiw, int64_t(norb) * ng, s);
  if (W && !owner) HIPCHK(c, hipMemsetAsync(W, 0, size_t(norb) * ng * es, s));  // the owner path writes every row

  KernelParams kp;
  kp.kind = kernel;
  kp.omega = omega;
  kp.inv_ng = 1.0 / double(ng);
  for (int d = 0; d < 3; ++d) kp.g[d] = 2.0 * 3.141592653589793238462643383279502884 / g->L[d];

  // (c) pair Poisson solves, round by round
  rec_begin(R, ST_PAIRS, s);
  if (owner) {
    HIPCHK(c, launch_vtable(prec, N, kp, vtab, s));
    HIPCHK(c, pair_owner(prec, N, phiw, spec, dpk, int(onpk), int(npairs), dadjp, dadj, c->owner_order ? doperm : nullptr,
                         norb, int64_t(S.adj.size() / 2), W, epart, tw, kp, vtab, 1 << 30, s, R));
    if (pair_energy) launch_pair_energy(epart, int(onpk), nblk, dpk, dpidx, dV, pair_energy, s);
  } else {
    for (const auto& L : S.launches) {
      HIPCHK(c, pair_round(prec, N, sh, phiw, spec, dpk + L.first, L.second, L.npairs, W, epart, tw, kp, s, R));
      if (pair_energy)
        launch_pair_energy(epart, L.second, nblk, dpk + L.first, dpidx + 2 * L.first, dV, pair_energy, s);
    }
  }
  rec_end(R, ST_PAIRS, s);
  if (!xi && !Wout) {  // energies only
    rec_end(R, ST_BUILD, s);
    HIPCHK(c, hipGetLastError());
    return ACE_OK;
  }

  // W is an output of step (c) whatever the factorization below reports
  if (Wout && W != Wout) {
    if (prec == 0)
      HIPCHK(c, hipMemcpyAsync(Wout, W, size_t(norb) * ng * sizeof(double), hipMemcpyDeviceToDevice, s));
    else
      launch_f2d((const float*)W, Wout, int64_t(norb) * ng, s);
  }

  // (d) M = dV Phi W^T, symmetrize, -M = L L^T
  rec_begin(R, ST_TAIL, s);
  HIPCHK(c, gemm_nt(prec, 0, phiw, ng, W, ng, norb, norb, ng, dV, part, Mraw, s, R));
  launch_symmetrize(Mraw, norb, Mout, Lb, ex ? ex : scal, scal + 1, s);
  if (!xi) {  // exact exchange: W, M and E_x only
    rec_end(R, ST_TAIL, s);
    rec_end(R, ST_BUILD, s);
    HIPCHK(c, hipGetLastError());
    return ACE_OK;
  }
  launch_zero(info, sizeof(int), s);
  launch_chol_inv(Lb, norb, info, Li, tinv, s);
  // (e) xi = L^-1 W; the factorization's status is read once, after it (on
  // failure the outputs are unspecified)
  HIPCHK(c, gemm_ls(prec, false, true, Li, norb, W, ng, xi, ng, norb, norb, ng, 1.0, s, R));
  rec_end(R, ST_TAIL, s);
  rec_end(R, ST_BUILD, s);
  int hinfo = 0;
  HIPCHK(c, hipMemcpyAsync(&hinfo, info, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipStreamSynchronize(s));
  if (hinfo > 0) return fail(c, ACE_E_NOT_PD, "-M is not positive definite (Cholesky column %d)", hinfo - 1);
  if (hinfo < 0) return fail(c, ACE_E_NONFINITE, "non-finite value in M (Cholesky column %d)", -hinfo - 1);
  HIPCHK(c, hipGetLastError());
  return ACE_OK;
}

int ace_exact_exchange(ace_ctx* c, const ace_grid* g, int norb, const double* psi, int kernel, double omega,
                       int prec, double* W, double* Mout, double* ex) {
  if (!c) return ACE_E_ARG;
  int rc = check_grid(c, g, norb);
  if (rc) return rc;
  if (!psi || !W) return fail(c, ACE_E_ARG, "psi and W must be non-NULL");
  if (kernel != ACE_KERNEL_COULOMB && kernel != ACE_KERNEL_ERFC) return fail(c, ACE_E_ARG, "unknown kernel %d", kernel);
  if (kernel == ACE_KERNEL_ERFC && !(omega > 0.0)) return fail(c, ACE_E_ARG, "omega must be > 0 for erfc");
  if (prec != ACE_FP64 && prec != ACE_FP32) return fail(c, ACE_E_ARG, "unknown precision %d", prec);
  // every pair i <= j, sorted by (i, j)
  const int64_t np = int64_t(norb) * (norb + 1) / 2;
  std::vector<int32_t> hp(size_t(2 * np));
  size_t q = 0;
  for (int i = 0; i < norb; ++i)
    for (int j = i; j < norb; ++j) {
      hp[q++] = i;
      hp[q++] = j;
    }
  int32_t* dp;
  WS(c, "allpairs", hp.size() * sizeof(int32_t), dp);
  HIPCHK(c, hipMemcpyAsync(dp, hp.data(), hp.size() * sizeof(int32_t), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return build_impl(c, g, norb, psi, dp, np, kernel, omega, prec, nullptr, Mout, W, ex, nullptr);
}

// ------------------------------------------------------------------ apply
// y = V_ACE x from the coefficients cb = dV xi x^T; with ex, also -sum cb^2
static int apply_impl(ace_ctx* c, const ace_grid* g, int norb, const double* xi, int nvec, const double* x, double* y,
                      double* ex) {
  if (!c) return ACE_E_ARG;
  int rc = check_grid(c, g, norb);
  if (rc) return rc;
  if (!xi || !x || !y) return fail(c, ACE_E_ARG, "xi, x and y must be non-NULL");
  if (nvec < 1) return fail(c, ACE_E_ARG, "nvec must be >= 1");
  const int64_t ng = grid_size(g);
  hipStream_t s = c->stream;
  double *part, *cb;
  int64_t kchunk;
  const int64_t nsplit = gemm_nt_nsplit(norb, nvec, ng, &kchunk);
  WS(c, "apart", size_t(nsplit) * norb * nvec * sizeof(double), part);
  WS(c, "coef", size_t(norb) * nvec * sizeof(double), cb);
  HIPCHK(c, gemm_nt(0, 0, xi, ng, x, ng, norb, nvec, ng, grid_dv(g), part, cb, s, c->R()));
  HIPCHK(c, gemm_ls(0, true, false, cb, nvec, xi, ng, y, ng, nvec, norb, ng, -1.0, s, c->R()));
  if (ex) launch_neg_sumsq(cb, int64_t(norb) * nvec, ex, s);
  HIPCHK(c, hipGetLastError());
  return ACE_OK;
}

int ace_apply(ace_ctx* c, const ace_grid* g, int norb, const double* xi, int nvec, const double* x, double* y) {
  return apply_impl(c, g, norb, xi, nvec, x, y, nullptr);
}

int ace_apply_energy(ace_ctx* c, const ace_grid* g, int norb, const double* xi, int nvec, const double* x, double* y,
                     double* ex) {
  if (c && !ex) return fail(c, ACE_E_ARG, "ex must be non-NULL");
  return apply_impl(c, g, norb, xi, nvec, x, y, ex);
}


// ------------------------------------------------------------------ allocation-free application
// The fixed device scratch of ace_apply_energy_noalloc: the split-K partial
// sums of the coefficients c = dV xi x^T (at most kNoAllocPart doubles; the
// split count is capped to fit) followed by c itself (at most 512 x 512).
// One copy per device for the life of the process; every call on a device
// shares it, so calls that overlap on one device race.
constexpr int64_t kNoAllocPart = int64_t(4) << 20;  // 32 MiB of partial sums
constexpr int64_t kNoAllocCoef = int64_t(512) * 512;
static __device__ __align__(256) double scratch[kNoAllocPart + kNoAllocCoef];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

// Device address of the scratch array on the current device, looked up once
// per device (the array's name is only a host-side stand-in).
static int scratch_on_device(ace_ctx* c, double** out) {
  int dev = -1;
  HIPCHK(c, hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(c, ACE_E_UNSUPPORTED, "device %d beyond %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    HIPCHK(c, hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(c, ACE_E_HIP, "no device address for the scratch array on device %d", dev);
    g_scratch_ptr[dev] = p;
  }
  *out = static_cast<double*>(g_scratch_ptr[dev]);
  return ACE_OK;
}

int ace_apply_energy_noalloc(ace_ctx* c, const ace_grid* g, int norb, const double* xi, int nvec, const double* x,
                             double* y, double* ex) {
  if (!c) return ACE_E_ARG;
  int rc = check_grid(c, g, norb);
  if (rc) return rc;
  if (!xi || !x || !y || !ex) return fail(c, ACE_E_ARG, "xi, x, y and ex must be non-NULL");
  if (nvec < 1 || nvec > 512) return fail(c, ACE_E_ARG, "nvec=%d outside [1, 512] (fixed scratch)", nvec);
  double* base = nullptr;
  rc = scratch_on_device(c, &base);
  if (rc) return rc;
  const int64_t ng = grid_size(g);
  const int64_t mn = int64_t(norb) * nvec;
  const int64_t max_split = std::max<int64_t>(1, std::min<int64_t>(512, kNoAllocPart / mn));
  int64_t kchunk;
  // the split count gemm_nt will use (the largest of its cases), within the cap
  const int64_t nsplit = gemm_nt_nsplit(norb, nvec, ng, &kchunk, true, max_split);
  if (nsplit * mn > kNoAllocPart || mn > kNoAllocCoef)
    return fail(c, ACE_E_CAPACITY, "norb x nvec = %lld needs %lld partial sums, scratch holds %lld", (long long)mn,
                (long long)(nsplit * mn), (long long)kNoAllocPart);
  double* part = base;
  double* cb = base + kNoAllocPart;
  hipStream_t s = c->stream;
  // every partial tile and every coefficient is written before it is read:
  // nothing in the scratch needs clearing between calls
  HIPCHK(c, gemm_nt(0, 0, xi, ng, x, ng, norb, nvec, ng, grid_dv(g), part, cb, s, nullptr, false, max_split));
  HIPCHK(c, gemm_ls(0, true, false, cb, nvec, xi, ng, y, ng, nvec, norb, ng, -1.0, s, nullptr));
  launch_neg_sumsq(cb, mn, ex, s);
  HIPCHK(c, hipGetLastError());
  return ACE_OK;
}


// ------------------------------------------------------------------ complex orbitals, k-points
int ace_build_kpoints(ace_ctx* c, const ace_grid* g, int norb, int nk, const double* kvec, const double* u,
                      const int32_t* pairs, int64_t npairs, int kernel, double omega, double* xi, double* Mout,
                      double* Wout, double* ex) {
  if (!c) return ACE_E_ARG;
  int rc = check_grid(c, g, norb);
  if (rc) return rc;
  if (nk < 1 || int64_t(nk) * norb > 2048) return fail(c, ACE_E_ARG, "nk=%d: need 1 <= nk and nk * norb <= 2048", nk);
  if (!kvec || !u || !pairs || !xi) return fail(c, ACE_E_ARG, "kvec, u, pairs and xi must be non-NULL");
  for (int q = 0; q < 3 * nk; ++q)
    if (!std::isfinite(kvec[q])) return fail(c, ACE_E_ARG, "non-finite k-point coordinate");
  if (kernel != ACE_KERNEL_COULOMB && kernel != ACE_KERNEL_ERFC) return fail(c, ACE_E_ARG, "unknown kernel %d", kernel);
  if (kernel == ACE_KERNEL_ERFC && !(omega > 0.0)) return fail(c, ACE_E_ARG, "omega must be > 0 for erfc");
  const int ntot = nk * norb;
  const int64_t maxp = int64_t(ntot) * (ntot + 1) / 2;
  if (npairs < 1 || npairs > maxp) return fail(c, ACE_E_ARG, "npairs=%lld outside [1, %lld]", (long long)npairs,
                                               (long long)maxp);
  const int N = g->n[0];
  const int64_t ng = grid_size(g);
  const double dV = grid_dv(g);
  hipStream_t s = c->stream;
  std::vector<int32_t> pr(size_t(2 * npairs));
  HIPCHK(c, hipMemcpyAsync(pr.data(), pairs, pr.size() * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipStreamSynchronize(s));
  std::shared_ptr<const Schedule> Sp;
  rc = schedule_for(c, pr, npairs, ntot, 16, &Sp);
  if (rc) return rc;
  const Schedule& S = *Sp;
  // one slot per pair of every pack, launches in the schedule's order
  std::vector<KPair> slots(2 * S.packs.size());
  for (size_t p = 0; p < S.packs.size(); ++p) {
    const Pack& pk = S.packs[p];
    for (int h = 0; h < 2; ++h) {
      KPair& kq = slots[2 * p + h];
      kq.a = h ? pk.ib : pk.ia;
      kq.b = h ? pk.jb : pk.ja;
      for (int d = 0; d < 3; ++d)
        kq.d[d] = kq.b < 0 ? 0.0 : kvec[3 * (kq.b / norb) + d] - kvec[3 * (kq.a / norb) + d];
    }
  }
  const void* tw;
  rc = twiddles(c, N, 0, &tw);
  if (rc) return rc;
  const size_t cbytes = size_t(ntot) * ng * 2 * sizeof(double);  // one complex array of every orbital
  KPair* dslots;
  double *spec, *W, *Wm, *Mre, *Mim, *part, *negM, *Lr, *Li, *X2;
  int* info;
  int64_t kchunk;
  const int64_t nsplit = gemm_nt_nsplit(norb, norb, 2 * ng, &kchunk);
  WS(c, "kslots", slots.size() * sizeof(KPair), dslots);
  WS(c, "kspec", size_t(2 * S.max_launch) * ng * 2 * sizeof(double), spec);
  if (Wout) W = Wout; else WS(c, "kW", cbytes, W);
  WS(c, "kWm", cbytes, Wm);
  WS(c, "kMre", size_t(nk) * norb * norb * sizeof(double), Mre);
  WS(c, "kMim", size_t(nk) * norb * norb * sizeof(double), Mim);
  WS(c, "mpart", size_t(nsplit) * norb * norb * sizeof(double), part);
  WS(c, "knegM", size_t(nk) * norb * norb * 2 * sizeof(double), negM);
  WS(c, "kLr", size_t(nk) * norb * norb * sizeof(double), Lr);
  WS(c, "kLi", size_t(nk) * norb * norb * sizeof(double), Li);
  WS(c, "kX2", size_t(norb) * ng * 2 * sizeof(double), X2);
  WS(c, "kinfo", size_t(nk) * sizeof(int) + 64, info);
  HIPCHK(c, hipMemcpyAsync(dslots, slots.data(), slots.size() * sizeof(KPair), hipMemcpyHostToDevice, s));
  launch_zero(W, cbytes, s);
  KernelParams kp;
  kp.kind = kernel;
  kp.omega = omega;
  kp.inv_ng = 1.0 / double(ng);
  for (int d = 0; d < 3; ++d) kp.g[d] = 2.0 * 3.141592653589793238462643383279502884 / g->L[d];
  // (c) pair potentials and W, launch by launch (each conflict-free)
  for (const Schedule::Launch& l : S.launches)
    HIPCHK(c, kpair_round(N, u, spec, dslots + 2 * size_t(l.first), 2 * l.second, W, tw, kp, 1.0 / nk, s));
  // (d) per k-point M = dV U^H W from real products over the interleaved rows
  launch_times_minus_i(W, Wm, int64_t(ntot) * ng, s);
  for (int q = 0; q < nk; ++q) {
    const size_t ro = size_t(q) * norb * ng * 2;
    const size_t mo = size_t(q) * norb * norb;
    HIPCHK(c, gemm_nt(0, 0, u + ro, 2 * ng, W + ro, 2 * ng, norb, norb, 2 * ng, dV, part, Mre + mo, s, nullptr));
    HIPCHK(c, gemm_nt(0, 0, u + ro, 2 * ng, Wm + ro, 2 * ng, norb, norb, 2 * ng, dV, part, Mim + mo, s, nullptr));
  }
  launch_hermitize(Mre, Mim, norb, nk, Mout, negM, s);
  if (ex) launch_trace_avg(Mre, norb, nk, ex, s);
  // -M = L L^H per k-point
  launch_zero(info, size_t(nk) * sizeof(int), s);
  launch_chol_c(negM, norb, nk, info, s);
  std::vector<int> hinfo(static_cast<size_t>(nk));
  HIPCHK(c, hipMemcpyAsync(hinfo.data(), info, size_t(nk) * sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipStreamSynchronize(s));
  for (int q = 0; q < nk; ++q) {
    if (hinfo[size_t(q)] > 0)
      return fail(c, ACE_E_NOT_PD, "-M of k-point %d is not positive definite (Cholesky column %d)", q,
                  hinfo[size_t(q)] - 1);
    if (hinfo[size_t(q)] < 0)
      return fail(c, ACE_E_NONFINITE, "non-finite value in M of k-point %d (column %d)", q, -hinfo[size_t(q)] - 1);
  }
  // (e) xi = conj(L)^-1 W = Re(L^-1) W + Im(L^-1) (-i W), per k-point
  launch_trinv_c(negM, norb, nk, Lr, Li, s);
  for (int q = 0; q < nk; ++q) {
    const size_t ro = size_t(q) * norb * ng * 2;
    const size_t mo = size_t(q) * norb * norb;
    HIPCHK(c, gemm_ls(0, false, true, Lr + mo, norb, W + ro, 2 * ng, xi + ro, 2 * ng, norb, norb, 2 * ng, 1.0, s,
                      nullptr));
    HIPCHK(c, gemm_ls(0, false, true, Li + mo, norb, Wm + ro, 2 * ng, X2, 2 * ng, norb, norb, 2 * ng, 1.0, s,
                      nullptr));
    launch_add_inplace(xi + ro, X2, int64_t(norb) * ng * 2, s);
  }
  HIPCHK(c, hipGetLastError());
  return ACE_OK;
}

int ace_pairlist_kpoints(ace_ctx* c, const ace_grid* g, int ntot, const double* u, double rho_cut, int64_t capacity,
                         int32_t* pairs, double* overlap, int64_t* npairs) {
  if (!c) return ACE_E_ARG;
  if (!g) return fail(c, ACE_E_ARG, "grid is NULL");
  if (ntot < 1 || ntot > 2048) return fail(c, ACE_E_ARG, "ntot=%d outside [1, 2048]", ntot);
  if (!u) return fail(c, ACE_E_ARG, "u must be non-NULL");
  int rc = check_grid(c, g, 1);
  if (rc) return rc;
  const int64_t ng = grid_size(g);
  double* mag;
  WS(c, "kabs", size_t(ntot) * ng * sizeof(double), mag);
  launch_cabs(u, mag, int64_t(ntot) * ng, c->stream);
  return pairlist_core(c, g, ntot, mag, rho_cut, capacity, pairs, overlap, npairs);
}


// ------------------------------------------------------------------ batched form
int ace_set_batched_shape(ace_ctx* c, int txv, int plan_variant, int blocks_per_cu, int layout) {
  if (!c || (txv != 8 && txv != 16) || (plan_variant != 0 && plan_variant != 1) || blocks_per_cu < 1 ||
      blocks_per_cu > 32 || (layout != 0 && layout != 2 && layout != 3))
    return fail(c, ACE_E_ARG, "bad batched shape");
  c->b_txv = txv;
  c->b_plan = plan_variant;
  c->b_bpc = blocks_per_cu;
  c->b_layout = layout;
  return ACE_OK;
}

int ace_build_batched(ace_ctx* c, int nsys, ace_system* sys, int prec, int mode) {
  if (!c) return ACE_E_ARG;
  if (nsys < 1 || nsys > 4096 || !sys) return fail(c, ACE_E_ARG, "nsys=%d outside [1, 4096]", nsys);
  if (prec != ACE_FP64 && prec != ACE_FP32) return fail(c, ACE_E_ARG, "unknown precision %d", prec);
  if (mode < 0 || mode > 2) return fail(c, ACE_E_ARG, "unknown batched mode %d", mode);
  for (int q = 0; q < nsys; ++q) {
    ace_system& y = sys[q];
    int rc = check_grid(c, &y.grid, y.norb);
    if (rc) return fail(c, rc, "system %d: %s", q, c->err.c_str());
    if (!batched_supported(y.grid.n[0]))
      return fail(c, ACE_E_UNSUPPORTED, "system %d: batched grids are 16, 24, 32, 48, 64, 80 or 96", q);
    if (!y.phi || !y.pairs || !y.xi) return fail(c, ACE_E_ARG, "system %d: phi, pairs and xi must be non-NULL", q);
    if (y.kernel != ACE_KERNEL_COULOMB && y.kernel != ACE_KERNEL_ERFC)
      return fail(c, ACE_E_ARG, "system %d: unknown kernel", q);
    if (y.kernel == ACE_KERNEL_ERFC && !(y.omega > 0.0)) return fail(c, ACE_E_ARG, "system %d: omega must be > 0", q);
    const int64_t maxp = int64_t(y.norb) * (y.norb + 1) / 2;
    if (y.npairs < 1 || y.npairs > maxp) return fail(c, ACE_E_ARG, "system %d: npairs outside [1, %lld]", q,
                                                     (long long)maxp);
    y.status = ACE_OK;
    y.fail_column = -1;
  }
  hipStream_t us = c->stream;
  if (!c->bstream) {
    HIPCHK(c, hipStreamCreateWithFlags(&c->bstream, hipStreamNonBlocking));
    HIPCHK(c, hipEventCreateWithFlags(&c->bev_in, hipEventDisableTiming));
    HIPCHK(c, hipEventCreateWithFlags(&c->bev_out, hipEventDisableTiming));
    HIPCHK(c, hipEventCreateWithFlags(&c->bev_fork, hipEventDisableTiming));
    for (int b = 0; b < ace_ctx::kTailBranches; ++b) {
      HIPCHK(c, hipStreamCreateWithFlags(&c->bbr[b], hipStreamNonBlocking));
      HIPCHK(c, hipEventCreateWithFlags(&c->bev_join[b], hipEventDisableTiming));
    }
  }
  hipStream_t bs = c->bstream;
  // pair lists to the host, schedules
  std::vector<std::vector<int32_t>> prs(nsys);
  for (int q = 0; q < nsys; ++q) {
    prs[q].resize(size_t(2 * sys[q].npairs));
    HIPCHK(c, hipMemcpyAsync(prs[q].data(), sys[q].pairs, prs[q].size() * sizeof(int32_t), hipMemcpyDeviceToHost,
                             us));
  }
  HIPCHK(c, hipStreamSynchronize(us));
  std::vector<std::shared_ptr<const Schedule>> sch(static_cast<size_t>(nsys));
  uint64_t key = 1469598103934665603ull;
  auto mix = [&key](uint64_t v) { key = (key ^ v) * 1099511628211ull; };
  mix(uint64_t(prec)); mix(uint64_t(mode)); mix(uint64_t(c->b_txv)); mix(uint64_t(c->b_plan)); mix(uint64_t(c->b_bpc));
  mix(uint64_t(c->b_layout));
  int nrounds = 0;
  for (int q = 0; q < nsys; ++q) {
    int rc = schedule_for(c, prs[q], sys[q].npairs, sys[q].norb, 1 << 30, &sch[q]);
    if (rc) return fail(c, rc, "system %d: %s", q, c->err.c_str());
    nrounds = std::max(nrounds, int(sch[q]->round_first.size()));
    const ace_system& y = sys[q];
    mix(uint64_t(uintptr_t(y.phi))); mix(uint64_t(uintptr_t(y.xi))); mix(uint64_t(uintptr_t(y.M)));
    mix(uint64_t(uintptr_t(y.ex))); mix(uint64_t(y.norb)); mix(uint64_t(y.grid.n[0])); mix(uint64_t(y.kernel));
    uint64_t ob, lb[3];
    std::memcpy(&ob, &y.omega, 8);
    std::memcpy(lb, y.grid.L, 24);
    mix(ob); mix(lb[0]); mix(lb[1]); mix(lb[2]);
    mix(uint64_t(sch[q]->packs.size()));
    for (const Pack& pk : sch[q]->packs) mix(uint64_t(uint32_t(pk.ia)) << 32 | uint32_t(pk.ja) ^ uint64_t(uint32_t(pk.jb)) << 16);
  }
  const size_t es = prec == 0 ? sizeof(double) : sizeof(float);
  // segments: (grid size, super-round) with the packs of that size in that round
  std::vector<int> sizes;
  for (int q = 0; q < nsys; ++q) sizes.push_back(sys[q].grid.n[0]);
  std::sort(sizes.begin(), sizes.end());
  sizes.erase(std::unique(sizes.begin(), sizes.end()), sizes.end());
  // Owner layout (graph and eager launches): the spectra of all pairs of the
  // sizes that take it stay resident, within the same budget as a single
  // build (the persistent launch keeps the rounds).
  std::vector<char> size_owner(sizes.size(), 0);
  size_t owner_bytes = 0;
  if (c->b_layout == 3 && mode != 1) {
    for (size_t a = 0; a < sizes.size(); ++a) {
      const int n = sizes[a];
      if (!batched_r2c_fits(prec, n)) continue;
      size_owner[a] = 1;
      const size_t slot_bytes = size_t(n) * n * (n / 2 + 1) * 2 * es;
      for (int q = 0; q < nsys; ++q)
        if (sys[q].grid.n[0] == n) owner_bytes += sch[q]->opacks.size() * 2 * slot_bytes;
    }
    bool fits = owner_bytes <= c->owner_max;
    if (fits && owner_bytes > 0) {
      auto it = c->bufs.find("bspec");
      const size_t have = it == c->bufs.end() ? 0 : it->second.bytes;
      size_t freeb = 0, totb = 0;
      if (owner_bytes > have && hipMemGetInfo(&freeb, &totb) == hipSuccess)
        fits = double(owner_bytes) <= 0.6 * double(freeb + have);
    }
    if (!fits) {
      std::fill(size_owner.begin(), size_owner.end(), 0);
      owner_bytes = 0;
    }
  }
  for (char o : size_owner) mix(uint64_t(o));
  std::vector<BRound> segs;
  std::vector<int> seg_n;
  std::vector<BPack> bp;
  std::vector<int64_t> starts;
  std::vector<int64_t> bp_off;  // spec offset of each pack (bytes, within its segment)
  std::vector<char> bp_owner;   // the pack belongs to an owner segment (offset within the owner region)
  size_t spec_bytes = 0;
  std::vector<char> seg_r2c;
  // owner segments: one per grid size, all packs of its systems
  struct OwnerSeg { int n, pack0, npacks, own0, nown; int64_t items; size_t spec_off; };
  std::vector<OwnerSeg> osegs;
  std::vector<BOwner> hown;
  std::vector<int64_t> own_adjp_off;     // offset of each system's adjacency offsets in the table
  std::vector<int32_t> hadjp, hadj, hoperm;
  size_t owner_off = 0;
  for (size_t a = 0; a < sizes.size(); ++a) {
    if (!size_owner[a]) continue;
    const int n = sizes[a];
    const size_t pack_bytes = 2 * size_t(n) * n * (n / 2 + 1) * 2 * es;
    OwnerSeg os{n, int(bp.size()), 0, int(hown.size()), 0, 0, owner_off};
    for (int q = 0; q < nsys; ++q) {
      if (sys[q].grid.n[0] != n) continue;
      const Schedule& S = *sch[q];
      const int32_t slot0 = int32_t(2 * (bp.size() - size_t(os.pack0)));
      for (const Pack& pk : S.opacks) {
        BPack b{};
        b.sys = q;
        b.pk = pk;
        bp.push_back(b);
        bp_off.push_back(int64_t(owner_off));
        bp_owner.push_back(1);
        owner_off += pack_bytes;
      }
      BOwner o{};
      o.sys = q;
      o.norb = sys[q].norb;
      o.orb0 = os.items / n;
      own_adjp_off.push_back(int64_t(hadjp.size()));
      hoperm.insert(hoperm.end(), S.operm.begin(), S.operm.end());
      const int32_t e0 = int32_t(hadj.size() / 2);
      for (int32_t v : S.adj_ptr) hadjp.push_back(v + e0);
      for (size_t e = 0; e < S.adj.size(); e += 2) {
        hadj.push_back(S.adj[e] + slot0);
        hadj.push_back(S.adj[e + 1]);
      }
      hown.push_back(o);
      os.items += int64_t(sys[q].norb) * n;
    }
    os.npacks = int(bp.size()) - os.pack0;
    os.nown = int(hown.size()) - os.own0;
    if (int64_t(hadj.size()) > int64_t(0x7fffffff)) return fail(c, ACE_E_CAPACITY, "batched adjacency too large");
    osegs.push_back(os);
  }
  for (size_t a = 0; a < sizes.size(); ++a) {
    if (size_owner[a]) continue;
    const int n = sizes[a];
    const int64_t ngn = int64_t(n) * n * n;
    const bool r2c = c->b_layout >= 2 && batched_r2c_fits(prec, n);
    // complex spectrum values per pack: two half spectra (real-to-complex) or one full field
    const int64_t pack_elems = r2c ? 2 * int64_t(n) * n * (n / 2 + 1) : ngn;
    for (int r = 0; r < nrounds; ++r) {
      BRound sg{};
      sg.pack0 = int(bp.size());
      size_t off = 0;
      for (int q = 0; q < nsys; ++q) {
        if (sys[q].grid.n[0] != n || r >= int(sch[q]->round_first.size())) continue;
        const Schedule& S = *sch[q];
        for (int k = 0; k < S.round_count[r]; ++k) {
          BPack b{};
          b.sys = q;
          b.pk = S.packs[S.round_first[r] + k];
          bp.push_back(b);
          bp_off.push_back(int64_t(off));
          bp_owner.push_back(0);
          off += size_t(pack_elems) * 2 * es;
        }
      }
      sg.npacks = int(bp.size()) - sg.pack0;
      if (sg.npacks == 0) continue;
      spec_bytes = std::max(spec_bytes, off);
      for (int p = 0; p < 5; ++p) {
        sg.start_off[p] = int64_t(starts.size());
        int64_t acc = 0;
        for (int k = 0; k < sg.npacks; ++k) {
          starts.push_back(acc);
          if (!r2c) acc += batched_phase_items(n, p, c->b_txv);
          else if (p < 3) acc += (bp[sg.pack0 + k].pk.jb >= 0 ? 2 : 1) * batched_r2c_slot_items(n, p, mode == 1);
        }
        starts.push_back(acc);
        sg.nitems[p] = acc;
      }
      segs.push_back(sg);
      seg_n.push_back(n);
      seg_r2c.push_back(r2c ? 1 : 0);
    }
  }
  // workspaces
  int64_t w_total = 0, m_total = 0;
  std::vector<int64_t> w_off(nsys), m_off(nsys);
  int max_norb = 0;
  int64_t max_nsplit = 1;
  for (int q = 0; q < nsys; ++q) {
    const int64_t ng = grid_size(&sys[q].grid);
    w_off[q] = w_total;
    w_total += int64_t(sys[q].norb) * ng;
    m_off[q] = m_total;
    m_total += int64_t(sys[q].norb) * sys[q].norb;
    max_norb = std::max(max_norb, sys[q].norb);
    int64_t kc;
    max_nsplit = std::max(max_nsplit, gemm_nt_nsplit(sys[q].norb, sys[q].norb, ng, &kc));
  }
  char *bW, *bphi = nullptr, *bspec;
  double *part, *Mraw, *Lb, *Li, *exs;
  int* infos;
  BSys* dsys;
  BPack* dbp;
  BRound* dsegs;
  int64_t* dstarts;
  WS(c, "bW", size_t(w_total) * es, bW);
  if (prec == 1) WS(c, "bphi32", size_t(w_total) * es, bphi);
  // the owner region follows the (reused) round region
  const size_t owner_base = (spec_bytes + 255) / 256 * 256;
  WS(c, "bspec", std::max<size_t>(owner_base + owner_off, 256), bspec);
  // v(G) tables of the systems in the owner layout
  std::vector<int64_t> vt_off(nsys, -1);
  int64_t vt_total = 0;
  for (size_t a = 0; a < sizes.size(); ++a) {
    if (!size_owner[a]) continue;
    for (int q = 0; q < nsys; ++q) {
      const int n = sys[q].grid.n[0];
      if (n != sizes[a]) continue;
      vt_off[q] = vt_total;
      vt_total += (int64_t(n / 2 + 1) * (n / 2 + 1) * (n / 2 + 1) * int64_t(es) + 255) / 256 * 256;
    }
  }
  char* bvt = nullptr;
  if (vt_total > 0) WS(c, "bvtab", size_t(vt_total), bvt);
  BOwner* dbown = nullptr;
  int32_t *dbadjp = nullptr, *dbadj = nullptr, *dboperm = nullptr;
  if (!osegs.empty()) {
    WS(c, "bown", std::max<size_t>(hown.size(), 1) * sizeof(BOwner), dbown);
    WS(c, "badjp", std::max<size_t>(hadjp.size(), 1) * sizeof(int32_t), dbadjp);
    WS(c, "badj", std::max<size_t>(hadj.size(), 2) * sizeof(int32_t), dbadj);
    WS(c, "boperm", std::max<size_t>(hoperm.size(), 1) * sizeof(int32_t), dboperm);
    // the owners of each system run in its schedule's order, as in the single build
    for (size_t q = 0, off = 0; q < hown.size(); off += size_t(hown[q].norb), ++q) {
      hown[q].adj_ptr = dbadjp + own_adjp_off[q];
      hown[q].operm = c->owner_order ? dboperm + off : nullptr;
    }
  }
  // per-branch scratch of the tails (the branches run concurrently)
  constexpr int NBR = ace_ctx::kTailBranches;
  const size_t part_elems = size_t(max_nsplit) * max_norb * max_norb, mat_elems = size_t(max_norb) * max_norb;
  WS(c, "bmpart", NBR * part_elems * sizeof(double), part);
  WS(c, "bMraw", NBR * mat_elems * sizeof(double), Mraw);
  WS(c, "bLc", NBR * mat_elems * sizeof(double), Lb);
  WS(c, "bLinv", NBR * mat_elems * sizeof(double), Li);
  WS(c, "bex", size_t(nsys) * 2 * sizeof(double), exs);
  WS(c, "binfo", size_t(nsys) * sizeof(int), infos);
  double* btinv;
  WS(c, "btinv", NBR * 64 * 64 * sizeof(double), btinv);
  WS(c, "bsys", size_t(nsys) * sizeof(BSys), dsys);
  WS(c, "bpacks", std::max<size_t>(bp.size(), 1) * sizeof(BPack), dbp);
  WS(c, "bsegs", std::max<size_t>(segs.size(), 1) * sizeof(BRound), dsegs);
  WS(c, "bstarts", std::max<size_t>(starts.size(), 1) * sizeof(int64_t), dstarts);
  // descriptor tables
  std::vector<BSys> hs(nsys);
  for (int q = 0; q < nsys; ++q) {
    const ace_system& y = sys[q];
    const void* tw;
    int rc = twiddles(c, y.grid.n[0], prec, &tw);
    if (rc) return rc;
    BSys& b = hs[q];
    b.N = y.grid.n[0];
    b.kind = y.kernel;
    b.omega = y.omega;
    b.inv_ng = 1.0 / double(grid_size(&y.grid));
    for (int d = 0; d < 3; ++d) b.g[d] = 2.0 * 3.141592653589793238462643383279502884 / y.grid.L[d];
    b.phi = prec == 0 ? (const void*)y.phi : (const void*)(bphi + size_t(w_off[q]) * es);
    b.W = bW + size_t(w_off[q]) * es;
    b.tw = tw;
    b.vt = vt_off[q] >= 0 ? (const void*)(bvt + vt_off[q]) : nullptr;
  }
  for (size_t k = 0; k < bp.size(); ++k) bp[k].spec = bspec + (bp_owner[k] ? owner_base : 0) + bp_off[k];
  // a captured graph holds raw workspace pointers: any reallocation retires it
  mix(c->ws_gen);
  mix(uint64_t(uintptr_t(bW))); mix(uint64_t(uintptr_t(bspec))); mix(uint64_t(uintptr_t(part)));
  mix(uint64_t(uintptr_t(bvt)));
  HIPCHK(c, hipMemcpyAsync(dsys, hs.data(), hs.size() * sizeof(BSys), hipMemcpyHostToDevice, us));
  if (!bp.empty()) HIPCHK(c, hipMemcpyAsync(dbp, bp.data(), bp.size() * sizeof(BPack), hipMemcpyHostToDevice, us));
  if (!segs.empty())
    HIPCHK(c, hipMemcpyAsync(dsegs, segs.data(), segs.size() * sizeof(BRound), hipMemcpyHostToDevice, us));
  if (!starts.empty())
    HIPCHK(c, hipMemcpyAsync(dstarts, starts.data(), starts.size() * sizeof(int64_t), hipMemcpyHostToDevice, us));
  if (!osegs.empty()) {
    HIPCHK(c, hipMemcpyAsync(dbown, hown.data(), hown.size() * sizeof(BOwner), hipMemcpyHostToDevice, us));
    HIPCHK(c, hipMemcpyAsync(dbadjp, hadjp.data(), hadjp.size() * sizeof(int32_t), hipMemcpyHostToDevice, us));
    if (!hadj.empty())
      HIPCHK(c, hipMemcpyAsync(dbadj, hadj.data(), hadj.size() * sizeof(int32_t), hipMemcpyHostToDevice, us));
    if (!hoperm.empty())
      HIPCHK(c, hipMemcpyAsync(dboperm, hoperm.data(), hoperm.size() * sizeof(int32_t), hipMemcpyHostToDevice, us));
  }
  HIPCHK(c, hipStreamSynchronize(us));

  // the whole build, in stream order on the private stream
  auto enqueue = [&](hipStream_t s) -> int {
    // the owner kernels write every row of W once; the rounds accumulate
    if (!segs.empty()) launch_zero(bW, size_t(w_total) * es, s);
    launch_zero(infos, size_t(nsys) * sizeof(int), s);
    if (prec == 1)
      for (int q = 0; q < nsys; ++q)
        launch_d2f(sys[q].phi, (float*)(bphi + size_t(w_off[q]) * es), int64_t(sys[q].norb) * grid_size(&sys[q].grid),
                   s);
    for (size_t a = 0; a < segs.size();) {
      size_t b = a;
      while (b < segs.size() && seg_n[b] == seg_n[a]) ++b;
      hipError_t e = batched_segments(prec, seg_n[a], mode == 1 ? 1 : 0, c->b_txv, c->b_plan, c->b_bpc, int(b - a),
                                      segs.data() + a, dsegs + a, dsys, dbp, dstarts, seg_r2c[a] != 0, s);
      if (e != hipSuccess) return fail(c, ACE_E_HIP, "batched pair launch failed: %s", hipGetErrorString(e));
      a = b;
    }
    for (int q = 0; q < nsys; ++q) {
      if (vt_off[q] < 0) continue;
      const BSys& b = hs[q];
      KernelParams kp;
      kp.kind = b.kind;
      kp.omega = b.omega;
      kp.inv_ng = b.inv_ng;
      for (int d = 0; d < 3; ++d) kp.g[d] = b.g[d];
      hipError_t e = launch_vtable(prec, b.N, kp, bvt + vt_off[q], s);
      if (e != hipSuccess) return fail(c, ACE_E_HIP, "batched v(G) table launch failed: %s", hipGetErrorString(e));
    }
    for (const OwnerSeg& os : osegs) {
      hipError_t e = batched_owner(prec, os.n, c->b_plan, 2 * os.npacks, os.nown, os.items, dsys, dbp + os.pack0,
                                   dbown + os.own0, dbadj, bspec + owner_base + os.spec_off, s);
      if (e != hipSuccess) return fail(c, ACE_E_HIP, "batched owner launch failed: %s", hipGetErrorString(e));
    }
    // the per-system tails (M, Cholesky, L^-1, xi) on NBR branches forked
    // from s and joined back, each with its own scratch: the small
    // latency-bound kernels of one system overlap the GEMMs of another
    // (captured as parallel graph branches in graph mode)
    HIPCHK(c, hipEventRecord(c->bev_fork, s));
    for (int b = 0; b < NBR; ++b) HIPCHK(c, hipStreamWaitEvent(c->bbr[b], c->bev_fork, 0));
    for (int q = 0; q < nsys; ++q) {
      const int br = q % NBR;
      hipStream_t sb = c->bbr[br];
      double* bpart = part + br * part_elems;
      double* bM = Mraw + br * mat_elems;
      double* bL = Lb + br * mat_elems;
      double* bLi = Li + br * mat_elems;
      double* btv = btinv + br * 64 * 64;
      const ace_system& y = sys[q];
      const int n = y.norb;
      const int64_t ng = grid_size(&y.grid);
      const void* W = bW + size_t(w_off[q]) * es;
      const void* ph = prec == 0 ? (const void*)y.phi : (const void*)(bphi + size_t(w_off[q]) * es);
      hipError_t e = gemm_nt(prec, 0, ph, ng, W, ng, n, n, ng, grid_dv(&y.grid), bpart, bM, sb, nullptr);
      if (e != hipSuccess) return fail(c, ACE_E_HIP, "batched M launch failed: %s", hipGetErrorString(e));
      launch_symmetrize(bM, n, y.M, bL, y.ex ? y.ex : exs + 2 * q, exs + 2 * q + 1, sb);
      launch_chol_inv(bL, n, infos + q, bLi, btv, sb);
      e = gemm_ls(prec, false, true, bLi, n, W, ng, y.xi, ng, n, n, ng, 1.0, sb, nullptr);
      if (e != hipSuccess) return fail(c, ACE_E_HIP, "batched projector launch failed: %s", hipGetErrorString(e));
    }
    for (int b = 0; b < NBR; ++b) {
      HIPCHK(c, hipEventRecord(c->bev_join[b], c->bbr[b]));
      HIPCHK(c, hipStreamWaitEvent(s, c->bev_join[b], 0));
    }
    return ACE_OK;
  };

  HIPCHK(c, hipEventRecord(c->bev_in, us));
  HIPCHK(c, hipStreamWaitEvent(bs, c->bev_in, 0));
  if (mode == 0) {
    auto git = c->graphs.find(key);
    if (git == c->graphs.end()) {
      hipGraph_t graph;
      HIPCHK(c, hipStreamBeginCapture(bs, hipStreamCaptureModeThreadLocal));
      const int rc = enqueue(bs);
      hipError_t ee = hipStreamEndCapture(bs, &graph);
      if (rc) {
        if (ee == hipSuccess) (void)hipGraphDestroy(graph);
        return rc;
      }
      if (ee != hipSuccess) return fail(c, ACE_E_HIP, "graph capture failed: %s", hipGetErrorString(ee));
      hipGraphExec_t exec;
      ee = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (ee != hipSuccess) return fail(c, ACE_E_HIP, "graph instantiation failed: %s", hipGetErrorString(ee));
      if (c->graphs.size() >= 8) {
        (void)hipGraphExecDestroy(c->graphs[c->graph_order.front()]);
        c->graphs.erase(c->graph_order.front());
        c->graph_order.erase(c->graph_order.begin());
      }
      git = c->graphs.emplace(key, exec).first;
      c->graph_order.push_back(key);
    }
    HIPCHK(c, hipGraphLaunch(git->second, bs));
  } else {
    const int rc = enqueue(bs);
    if (rc) return rc;
  }
  std::vector<int> hinfo(nsys, 0);
  HIPCHK(c, hipMemcpyAsync(hinfo.data(), infos, size_t(nsys) * sizeof(int), hipMemcpyDeviceToHost, bs));
  HIPCHK(c, hipEventRecord(c->bev_out, bs));
  HIPCHK(c, hipStreamWaitEvent(us, c->bev_out, 0));
  HIPCHK(c, hipStreamSynchronize(bs));
  HIPCHK(c, hipGetLastError());
  int bad = 0;
  for (int q = 0; q < nsys; ++q) {
    if (hinfo[q] > 0) { sys[q].status = ACE_E_NOT_PD; sys[q].fail_column = hinfo[q] - 1; ++bad; }
    else if (hinfo[q] < 0) { sys[q].status = ACE_E_NONFINITE; sys[q].fail_column = -hinfo[q] - 1; ++bad; }
  }
  if (bad) return fail(c, ACE_E_NOT_PD, "%d of %d systems failed the Cholesky factorization (see status)", bad, nsys);
  return ACE_OK;
}


// ------------------------------------------------------------------ learned screener
static int features_impl(ace_ctx* c, const ace_grid* g, int norb, const double* phi, const int32_t* pairs,
                         int64_t np, float* feats, int stride, double** O_out) {
  const int n = g->n[0];
  const int64_t ng = grid_size(g);
  hipStream_t s = c->stream;
  double *pz, *py, *px, *cen, *spr, *O, *P, *part;
  // the overlap integrals run over the grid subsampled by the stride
  const int m = n / stride;
  const int64_t ngs = int64_t(m) * m * m;
  const double dVs = grid_dv(g) * double(stride) * stride * stride;
  const double* phis = phi;
  if (stride > 1) {
    double* sub;
    WS(c, "f_sub", size_t(norb) * ngs * sizeof(double), sub);
    launch_subsample(phi, norb, n, stride, sub, s);
    phis = sub;
  }
  int64_t kchunk;
  const int64_t nsplit = gemm_nt_nsplit(norb, norb, ngs, &kchunk);
  WS(c, "f_pz", size_t(norb) * n * sizeof(double), pz);
  WS(c, "f_py", size_t(norb) * n * n * sizeof(double), py);
  WS(c, "f_px", size_t(norb) * n * n * sizeof(double), px);
  WS(c, "f_cen", size_t(norb) * 3 * sizeof(double), cen);
  WS(c, "f_spr", size_t(norb) * sizeof(double), spr);
  WS(c, "O", size_t(norb) * norb * sizeof(double), O);
  WS(c, "f_P", size_t(norb) * norb * sizeof(double), P);
  WS(c, "mpart", size_t(nsplit) * norb * norb * sizeof(double), part);
  launch_marginals(phi, norb, n, pz, py, px, s);
  launch_centroids(pz, py, px, norb, n, g->L[0], grid_dv(g), cen, spr, s);
  HIPCHK(c, gemm_nt(0, 1, phis, ngs, phis, ngs, norb, norb, ngs, dVs, part, O, s, nullptr, true));
  HIPCHK(c, gemm_nt(0, 2, phis, ngs, phis, ngs, norb, norb, ngs, dVs, part, P, s, nullptr, true));
  (void)ng;
  launch_pair_features(pairs, np, norb, cen, spr, O, P, g->L[0], feats, s);
  HIPCHK(c, hipGetLastError());
  if (O_out) *O_out = O;
  return ACE_OK;
}

int ace_pair_features(ace_ctx* c, const ace_grid* g, int norb, const double* phi, const int32_t* pairs, int64_t npairs,
                      float* feats, int stride) {
  if (!c) return ACE_E_ARG;
  int rc = check_grid(c, g, norb);
  if (rc) return rc;
  if (g->L[0] != g->L[1] || g->L[1] != g->L[2]) return fail(c, ACE_E_UNSUPPORTED, "features need a cubic box");
  if (!phi || !feats) return fail(c, ACE_E_ARG, "phi and feats must be non-NULL");
  if (stride < 1 || g->n[0] % stride != 0) return fail(c, ACE_E_ARG, "stride must be >= 1 and divide the grid size");
  const int64_t all = int64_t(norb) * (norb + 1) / 2;
  if (pairs ? (npairs < 1 || npairs > all) : (npairs != all))
    return fail(c, ACE_E_ARG, "npairs must be in [1, %lld] (or exactly %lld with pairs == NULL)", (long long)all,
                (long long)all);
  return features_impl(c, g, norb, phi, pairs, npairs, feats, stride, nullptr);
}

int ace_mlp_init(ace_ctx* c, float* model, uint64_t seed) {
  if (!c || !model) return fail(c, ACE_E_ARG, "model must be non-NULL");
  launch_mlp_init(model, seed, c->stream);
  HIPCHK(c, hipGetLastError());
  return ACE_OK;
}

int ace_mlp_fit_norm(ace_ctx* c, float* model, const float* x, const float* t, int64_t n) {
  if (!c || !model || !x || !t || n < 2) return fail(c, ACE_E_ARG, "model, x, t non-NULL and n >= 2 required");
  double* part;
  WS(c, "m_stats", size_t(stats_blocks(n)) * 22 * sizeof(double), part);
  launch_mlp_stats(x, t, n, part, model, c->stream);
  HIPCHK(c, hipGetLastError());
  return ACE_OK;
}

int ace_mlp_forward(ace_ctx* c, const float* model, const float* x, int64_t n, int clamp, float* y) {
  if (!c || !model || !x || !y || n < 1) return fail(c, ACE_E_ARG, "model, x, y non-NULL and n >= 1 required");
  launch_mlp_forward(model, x, n, clamp, y, c->stream);
  HIPCHK(c, hipGetLastError());
  return ACE_OK;
}

int ace_mlp_grad(ace_ctx* c, const float* model, const float* x, const float* t, int64_t n, float* grad, float* loss) {
  if (!c || !model || !x || !t || !grad || n < 1 || n > (1 << 30))
    return fail(c, ACE_E_ARG, "model, x, t, grad non-NULL and 1 <= n <= 2^30 required");
  const int nb = mlp_grad_blocks(int(n));
  float *gp, *lp;
  WS(c, "m_gpart", size_t(nb) * ACE_MLP_NPARAM * sizeof(float), gp);
  WS(c, "m_lpart", size_t(nb) * sizeof(float), lp);
  launch_mlp_grad_partial(model, x, t, n, 0, 1, 0, int(n), gp, lp, c->stream);
  launch_mlp_reduce(gp, lp, nb, grad, loss, c->stream);
  HIPCHK(c, hipGetLastError());
  return ACE_OK;
}

static uint64_t mix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

int ace_mlp_train(ace_ctx* c, float* model, float* adam_m, float* adam_v, const float* x, const float* t, int64_t n,
                  const ace_mlp_hparams* hp, float* loss_curve) {
  if (!c || !model || !adam_m || !adam_v || !x || !t || !hp || n < 1)
    return fail(c, ACE_E_ARG, "model, Adam state, x, t and hparams must be non-NULL, n >= 1");
  if (hp->batch < 1 || hp->batch > (1 << 20) || hp->epochs < 1 || !(hp->lr > 0))
    return fail(c, ACE_E_ARG, "batch in [1, 2^20], epochs >= 1 and lr > 0 required");
  hipStream_t s = c->stream;
  const int bsz_max = int(std::min<int64_t>(hp->batch, n));
  const int nb = mlp_grad_blocks(bsz_max);
  float *gp, *lp;
  WS(c, "m_gpart", size_t(nb) * ACE_MLP_NPARAM * sizeof(float), gp);
  WS(c, "m_lpart", size_t(nb) * sizeof(float), lp);
  if (loss_curve) launch_zero(loss_curve, size_t(hp->epochs) * sizeof(float), s);
  // a permutation of the samples per epoch: k -> (off + k * stride) mod n with gcd(stride, n) = 1
  auto gcd = [](uint64_t a, uint64_t b) { while (b) { uint64_t r = a % b; a = b; b = r; } return a; };
  uint64_t stride = (uint64_t(double(n) * 0.6180339887498949) | 1ull) % uint64_t(n);
  if (stride == 0) stride = 1;
  while (gcd(stride, uint64_t(n)) != 1) stride = (stride + 2) % uint64_t(n) ? (stride + 2) % uint64_t(n) : 1;
  int step = hp->step0;
  for (int e = 0; e < hp->epochs; ++e) {
    const int64_t off = int64_t(mix64(hp->seed * 1000003ull + uint64_t(e)) % uint64_t(n));
    for (int64_t b0 = 0; b0 < n; b0 += hp->batch) {
      const int bsz = int(std::min<int64_t>(hp->batch, n - b0));
      launch_mlp_grad_partial(model, x, t, n, off, int64_t(stride), b0, bsz, gp, lp, s);
      launch_mlp_adam(gp, lp, mlp_grad_blocks(bsz), model, adam_m, adam_v, ++step, hp->lr, hp->beta1, hp->beta2,
                      hp->eps, loss_curve ? loss_curve + e : nullptr, s);
    }
  }
  HIPCHK(c, hipGetLastError());
  return ACE_OK;
}

// The screener's training and inference under one state array: the model
// (ACE_MLP_NMODEL floats) followed by the Adam moments (2 x ACE_MLP_NPARAM).
int ace_screener_train(ace_ctx* c, const float* feats, const float* target, int64_t n, const ace_mlp_hparams* hp,
                       float* state) {
  if (!c) return ACE_E_ARG;
  if (!state) return fail(c, ACE_E_ARG, "state must be non-NULL");
  return ace_mlp_train(c, state, state + ACE_MLP_NMODEL, state + ACE_MLP_NMODEL + ACE_MLP_NPARAM, feats, target, n,
                       hp, nullptr);
}

int ace_screener_predict(ace_ctx* c, const float* state, const float* feats, int64_t n, float* pred) {
  return ace_mlp_forward(c, state, feats, n, 1, pred);
}

int ace_screen_learned(ace_ctx* c, const ace_grid* g, int norb, const double* phi, const float* model,
                       double budget, double rho_cut_fallback, double ood_tol, int64_t capacity, int32_t* pairs,
                       int64_t* npairs, int* used_fallback, int stride) {
  if (!c) return ACE_E_ARG;
  int rc = check_grid(c, g, norb);
  if (rc) return rc;
  if (g->L[0] != g->L[1] || g->L[1] != g->L[2]) return fail(c, ACE_E_UNSUPPORTED, "screening needs a cubic box");
  if (!phi || !model || !pairs || !npairs) return fail(c, ACE_E_ARG, "phi, model, pairs and npairs must be non-NULL");
  if (!(budget >= 0) || !std::isfinite(rho_cut_fallback) || !(ood_tol >= 0) || capacity < 0)
    return fail(c, ACE_E_ARG, "budget >= 0, finite rho_cut, ood_tol >= 0 and capacity >= 0 required");
  if (stride < 1 || g->n[0] % stride != 0) return fail(c, ACE_E_ARG, "stride must be >= 1 and divide the grid size");
  hipStream_t s = c->stream;
  const int64_t np = int64_t(norb) * (norb + 1) / 2;
  float *f, *pred;
  uint8_t* keep;
  double *tau, *O;
  int* ood;
  int64_t* cnt;
  WS(c, "s_feats", size_t(np) * 5 * sizeof(float), f);
  WS(c, "s_pred", size_t(np) * sizeof(float), pred);
  WS(c, "s_keep", size_t(np), keep);
  WS(c, "s_tau", 64, tau);
  WS(c, "s_ood", 64, ood);
  WS(c, "cnt", 64, cnt);
  float* bq;
  double* bw;
  WS(c, "s_bq", size_t(np) * sizeof(float), bq);
  WS(c, "s_bw", size_t(np) * sizeof(double), bw);
  rc = features_impl(c, g, norb, phi, nullptr, np, f, stride, &O);
  if (rc) return rc;
  launch_mlp_forward(model, f, np, 1, pred, s);
  HIPCHK(c, hipMemsetAsync(ood, 0, sizeof(int), s));
  launch_select(pred, f, np, norb, model, budget, O, rho_cut_fallback, float(ood_tol), ood, tau, keep, capacity, pairs,
                cnt, bq, bw, s);
  int64_t h = 0;
  int hood = 0;
  HIPCHK(c, hipMemcpyAsync(&h, cnt, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipMemcpyAsync(&hood, ood, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipStreamSynchronize(s));
  if (used_fallback) *used_fallback = hood > 0 ? 1 : 0;
  // the fallback is the screening criterion itself: with subsampled features
  // it is redone on the full grid
  if (hood > 0 && stride > 1) return ace_pairlist(c, g, norb, phi, rho_cut_fallback, capacity, pairs, nullptr, npairs);
  *npairs = h;
  if (h > capacity) return fail(c, ACE_E_CAPACITY, "%lld pairs kept but capacity is %lld", (long long)h,
                                (long long)capacity);
  return ACE_OK;
}

// One screening call for both rules, selected by the record.
int ace_screen(ace_ctx* c, const ace_grid* g, int norb, const double* phi, const ace_screen_spec* sc, int64_t capacity,
               int32_t* pairs, double* overlap, int64_t* npairs, int* used_fallback) {
  if (!c) return ACE_E_ARG;
  if (!sc) return fail(c, ACE_E_ARG, "screen record is NULL");
  if (used_fallback) *used_fallback = 0;
  if (sc->mode == 0) return ace_pairlist(c, g, norb, phi, sc->rho_cut, capacity, pairs, overlap, npairs);
  if (sc->mode != 1) return fail(c, ACE_E_ARG, "unknown screening mode %d", sc->mode);
  if (overlap) return fail(c, ACE_E_ARG, "the learned rule returns no overlaps (pass NULL)");
  return ace_screen_learned(c, g, norb, phi, sc->model, sc->ex_budget, sc->rho_cut, sc->ood_tol, capacity, pairs,
                            npairs, used_fallback, sc->stride);
}

}  // extern "C"
