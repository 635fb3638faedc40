// Host side of the C ABI: validation, the sweep planner, workspace layout and the
// entry points declared in include/aaqaoa.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <set>
#include <string>
#include <utility>
#include <vector>

#include "aaq_launch.h"
#include "aaqaoa.h"

using namespace aaq;

namespace {

thread_local std::string g_err;

aaq_status fail(aaq_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

#define HIPCHK(call)                                                                          \
  do {                                                                                        \
    hipError_t e_ = (call);                                                                   \
    if (e_ != hipSuccess) return fail(AAQ_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

size_t align_up(size_t x, size_t a = 256) { return (x + a - 1) / a * a; }

}  // namespace

// the error message of the library's other translation units (aaq_orbits.cpp)
aaq_status aaq::set_error(aaq_status s, const std::string& msg) { return fail(s, msg); }

aaq::LaunchEvents& aaq::launch_events() {
  static thread_local LaunchEvents e;
  return e;
}

namespace {

// ------------------------------------------------------------------ optional per-kernel timing
// When enabled, launches are bracketed by HIP events on the launching stream and the
// elapsed times are accumulated per kernel class with the algorithmic bytes moved.
enum KClass { KC_SWEEP1 = 0, KC_SWEEP2 = 1, KC_TABLES = 2, KC_REDUCE = 3, KC_ZZPASS = 4, KC_UNITS = 5, KC_N = 6 };
const char* kc_name[KC_N] = {"sweep_1state", "sweep_2state", "tables", "reduce", "zz_pass", "units"};
struct Pending {
  int cls;
  hipEvent_t a, b;
  double bytes;
};
std::mutex g_tmu;
bool g_timing = false;
uint32_t g_tclasses = (1u << KC_N) - 1;  // the classes timed while timing is on
std::vector<Pending> g_pending;
// timing-only events (no system-scope fence), created when timing is switched on and
// reused, so a timed region creates none; guarded by g_tmu
std::vector<hipEvent_t> g_evpool;
constexpr size_t kEventPool = 2048;
bool take_event(hipEvent_t* e) {
  if (!g_evpool.empty()) {
    *e = g_evpool.back();
    g_evpool.pop_back();
    return true;
  }
  return hipEventCreateWithFlags(e, hipEventDisableSystemFence) == hipSuccess;
}
double g_tot_ms[KC_N], g_tot_bytes[KC_N];
long long g_launches[KC_N];

struct TimedLaunch {
  bool on;
  Pending pe;
  hipStream_t st;
  TimedLaunch(int cls, double bytes, hipStream_t s) : on(false), st(s) {
    std::lock_guard<std::mutex> lk(g_tmu);
    if (!g_timing || !((g_tclasses >> cls) & 1u)) return;
    // kernels recorded into a graph carry no dispatch events: no timing while capturing
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;
    pe.cls = cls;
    pe.bytes = bytes;
    // timing-only events: no system-scope fence (no cache writeback and invalidation
    // between the measured kernels); aaq_timing_read reads them after the caller has
    // synchronised with the work
    if (!take_event(&pe.a)) return;
    if (!take_event(&pe.b)) {
      g_evpool.push_back(pe.a);
      return;
    }
    // the launches between here and done() take the events into their dispatches
    aaq::LaunchEvents& le = aaq::launch_events();
    le.start = pe.a;
    le.stop = pe.b;
    le.used = false;
    on = true;
  }
  void done() {
    if (!on) return;
    aaq::LaunchEvents& le = aaq::launch_events();
    if (!le.used) {  // nothing was launched: an empty interval
      (void)hipEventRecord(pe.a, st);
      (void)hipEventRecord(pe.b, st);
    }
    le = aaq::LaunchEvents{};
    std::lock_guard<std::mutex> lk(g_tmu);
    g_pending.push_back(pe);
    on = false;
  }
  ~TimedLaunch() {  // an error return before done(): drop the events
    if (!on) return;
    aaq::launch_events() = aaq::LaunchEvents{};
    (void)hipStreamSynchronize(st);
    (void)hipEventDestroy(pe.a);
    (void)hipEventDestroy(pe.b);
  }
  TimedLaunch(const TimedLaunch&) = delete;
  TimedLaunch& operator=(const TimedLaunch&) = delete;
};

// ------------------------------------------------------------------ launch tuning
int device_cus() {
  static int cached = 0;
  if (!cached) {
    int dev = 0, cu = 256;
    if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev);
    cached = cu > 0 ? cu : 256;
  }
  return cached;
}

// ------------------------------------------------------------------ validation
aaq_status validate_problem(const aaq_problem* pr) {
  if (!pr) return fail(AAQ_ERR_INVALID_ARG, "problem is NULL");
  if (pr->n < 1 || pr->n > AAQ_MAX_N) return fail(AAQ_ERR_INVALID_ARG, "n must be in [1, 34]");
  const int n = pr->n, m = pr->num_edges;
  if (m < 0) return fail(AAQ_ERR_GRAPH, "num_edges < 0");
  if (m > 0 && !pr->edges) return fail(AAQ_ERR_INVALID_ARG, "edges is NULL");
  std::set<std::pair<int, int>> seen;
  for (int e = 0; e < m; ++e) {
    int u = pr->edges[2 * e], v = pr->edges[2 * e + 1];
    if (u < 0 || u >= n || v < 0 || v >= n) return fail(AAQ_ERR_GRAPH, "edge " + std::to_string(e) + " has a vertex out of range");
    if (u == v) return fail(AAQ_ERR_GRAPH, "edge " + std::to_string(e) + " is a self-loop");
    if (!seen.insert({std::min(u, v), std::max(u, v)}).second)
      return fail(AAQ_ERR_GRAPH, "edge " + std::to_string(e) + " is a duplicate");
  }
  if (pr->edge_weight) {
    long long wsum = 0;
    for (int e = 0; e < m; ++e) {
      if (pr->edge_weight[e] < 1) return fail(AAQ_ERR_GRAPH, "edge " + std::to_string(e) + " has a weight < 1");
      wsum += pr->edge_weight[e];
    }
    if (wsum > AAQ_MAX_COST) return fail(AAQ_ERR_UNSUPPORTED, "total edge weight exceeds AAQ_MAX_COST (561)");
  }
  const int k = pr->num_orbits;
  if (m == 0) {
    if (k != 0) return fail(AAQ_ERR_ORBITS, "a graph without edges has no edge orbits");
    return AAQ_OK;
  }
  if (k < 1 || k > m) return fail(AAQ_ERR_ORBITS, "num_orbits must be in [1, |E|]");
  if (!pr->orbit_rep || !pr->orbit_size) return fail(AAQ_ERR_INVALID_ARG, "orbit_rep / orbit_size is NULL");
  long long tot = 0;
  std::set<int> reps;
  for (int o = 0; o < k; ++o) {
    if (pr->orbit_rep[o] < 0 || pr->orbit_rep[o] >= m) return fail(AAQ_ERR_ORBITS, "orbit representative is not an edge index");
    if (!reps.insert(pr->orbit_rep[o]).second) return fail(AAQ_ERR_ORBITS, "two orbits share a representative");
    if (pr->orbit_size[o] < 1) return fail(AAQ_ERR_ORBITS, "orbit size < 1");
    tot += pr->orbit_size[o];
  }
  if (tot != m) return fail(AAQ_ERR_ORBITS, "orbit sizes do not sum to |E|");
  if (pr->edge_orbit) {
    std::vector<int> cnt(k, 0);
    for (int e = 0; e < m; ++e) {
      int o = pr->edge_orbit[e];
      if (o < 0 || o >= k) return fail(AAQ_ERR_ORBITS, "edge_orbit entry out of range");
      cnt[o]++;
    }
    for (int o = 0; o < k; ++o) {
      if (cnt[o] != pr->orbit_size[o]) return fail(AAQ_ERR_ORBITS, "orbit size disagrees with edge_orbit");
      if (pr->edge_orbit[pr->orbit_rep[o]] != o) return fail(AAQ_ERR_ORBITS, "representative is not in its orbit");
    }
    if (pr->edge_weight)
      for (int e = 0; e < m; ++e)
        if (pr->edge_weight[e] != pr->edge_weight[pr->orbit_rep[pr->edge_orbit[e]]])
          return fail(AAQ_ERR_ORBITS, "edge " + std::to_string(e) + " has another weight than its orbit's representative");
  }
  return AAQ_OK;
}

aaq_status validate_p(int p) {
  if (p < 1 || p > AAQ_MAX_P) return fail(AAQ_ERR_INVALID_ARG, "p must be in [1, 64]");
  return AAQ_OK;
}

aaq_status validate_params(int p, const double* g, const double* b) {
  if (!g || !b) return fail(AAQ_ERR_INVALID_ARG, "gamma / beta is NULL");
  for (int l = 0; l < p; ++l)
    if (!std::isfinite(g[l]) || !std::isfinite(b[l])) return fail(AAQ_ERR_PARAMS, "non-finite gamma or beta");
  return AAQ_OK;
}

// ------------------------------------------------------------------ graph block
int edge_weight(const aaq_problem* pr, int e) { return pr->edge_weight ? pr->edge_weight[e] : 1; }

// the largest cut value sum_e w_e (the phase tables hold C = 0 .. this)
int total_weight(const aaq_problem* pr) {
  int w = 0;
  for (int e = 0; e < pr->num_edges; ++e) w += edge_weight(pr, e);
  return w;
}

bool is_weighted(const aaq_problem* pr) {
  for (int e = 0; e < pr->num_edges; ++e)
    if (edge_weight(pr, e) != 1) return true;
  return false;
}

GraphDev make_graph(const aaq_problem* pr) {
  GraphDev g;
  std::memset(&g, 0, sizeof(g));
  g.n = pr->n;
  g.m = pr->num_edges;
  g.cmax = total_weight(pr);
  g.weighted = is_weighted(pr);
  for (int e = 0; e < pr->num_edges; ++e) {
    int u = pr->edges[2 * e], v = pr->edges[2 * e + 1];
    g.adj[u] |= 1ull << v;
    g.adj[v] |= 1ull << u;
    g.deg[u]++;
    g.deg[v]++;
  }
  for (int v = 0; v < kAdjPad; ++v) g.adj32[v] = (uint32_t)g.adj[v];
  return g;
}

std::vector<int4> make_terms(const aaq_problem* pr, aaq_observable obs) {
  std::vector<int4> t;
  if (obs == AAQ_OBS_HC) {
    for (int e = 0; e < pr->num_edges; ++e)
      t.push_back(make_int4(pr->edges[2 * e], pr->edges[2 * e + 1], edge_weight(pr, e), 0));
  } else {
    for (int o = 0; o < pr->num_orbits; ++o) {
      int e = pr->orbit_rep[o];
      t.push_back(make_int4(pr->edges[2 * e], pr->edges[2 * e + 1], pr->orbit_size[o] * edge_weight(pr, e), 0));
    }
  }
  return t;
}

// Appends to `ext` (which starts with the plain term list) the term lists of set s
// sorted for its load and phase arrangements (see SetSpec::toff).
void add_term_lists(SetSpec& s, int L, const std::vector<int4>& terms, std::vector<int4>& ext, bool cost = false) {
  const int na = geo_na(L);
  for (int ki = 0; ki < 2; ++ki) {
    const int b0 = geo_b0(ki == 0 ? na - 1 : na - 2, L);
    int regbit[64];
    for (int v = 0; v < 64; ++v) regbit[v] = -1;
    for (int b = 0; b < kRegBits; ++b)
      if (s.pos[b0 + b] != kDummy) regbit[s.pos[b0 + b]] = b;
    std::vector<int4> grp[6];
    for (const int4& t : terms) {
      const int ri = regbit[t.x], rj = regbit[t.y];
      if (ri < 0 && rj < 0)
        grp[0].push_back(t);
      else if (ri >= 0 && rj >= 0)
        grp[5].push_back(make_int4(t.x, t.y, t.z, ri | (rj << 4)));
      else
        grp[1 + (ri >= 0 ? ri : rj)].push_back(t);
    }
    (cost ? s.coff : s.toff)[ki] = (uint16_t)ext.size();
    for (int g = 0; g < 6; ++g) {
      (cost ? s.ccnt : s.tcnt)[ki][g] = (uint16_t)grp[g].size();
      ext.insert(ext.end(), grp[g].begin(), grp[g].end());
    }
  }
}

// plain term list followed by every set's sorted lists (the device term array); with
// `cost` (the weighted cut's terms) also every set's sorted cost-term lists
std::vector<int4> term_array_of(const std::vector<int4>& terms, int L, std::vector<SetSpec>& sets,
                                const std::vector<int4>* cost = nullptr) {
  std::vector<int4> ext = terms;
  for (SetSpec& s : sets) add_term_lists(s, L, terms, ext);
  if (cost)
    for (SetSpec& s : sets) add_term_lists(s, L, *cost, ext, true);
  return ext;
}
std::vector<int4> term_array(const aaq_problem* pr, aaq_observable obs, int L, std::vector<SetSpec>& sets) {
  if (!is_weighted(pr)) return term_array_of(make_terms(pr, obs), L, sets);
  const std::vector<int4> cost = make_terms(pr, AAQ_OBS_HC);
  return term_array_of(make_terms(pr, obs), L, sets, &cost);
}

// ------------------------------------------------------------------ sweep planner
// Split the n qubits into k tile sets.  Set 0 is a contiguous block of L global bits
// (its low a_0 bits mixed); every later set mixes a_s <= L - 5 qubits and fills its
// tile with the lowest remaining global bits, so that every tile holds global bits
// 0..4 (>= 256 contiguous bytes per access).  k is the smallest possible, sizes as
// even as the caps allow.
// Register layouts ("arrangements"): arrangement k keeps tile bits
// [geo_b0(k, L), geo_b0(k, L) + 4) in registers (L = 13: b0 = 0, 4, 8, 9; L = 12:
// 0, 4, 8; L = 10: 0, 4, 6).

// Load arrangement, mixer route, active-qubit mask and register offsets of a set.
// Every set loads and stores with the top tile bits in registers (the last
// arrangement; the element offsets of its registers are tabulated).  Set 0 mixes
// through every arrangement; the later sets hold only tile bits >= 5 active and skip
// arrangement 0.
void finish_set(SetSpec& s, int L, bool first) {
  const int last = geo_na(L) - 1, b0 = geo_b0(last, L);
  s.kl = (uint8_t)last;
  s.route = first ? ROUTE_FULL : ROUTE_HIGH;
  s.gact = 0;
  for (int j = 0; j < 16; ++j)
    if (((s.act >> j) & 1u) && s.pos[j] != kDummy) s.gact |= 1ull << s.pos[j];
  for (int r = 0; r < 16; ++r) {
    uint64_t o = 0;
    for (int b = 0; b < kRegBits; ++b)
      if (((r >> b) & 1) && s.pos[b0 + b] != kDummy) o |= 1ull << s.pos[b0 + b];
    s.roff[r] = o;
  }
  // runs of thread bits at the load and phase arrangements (see SetSpec::trun)
  const int na = geo_na(L), lb = L - kRegBits;
  s.tr64 = 0;
  for (int ki = 0; ki < 2; ++ki) {
    const int bk = geo_b0(ki == 0 ? na - 1 : na - 2, L);
    int nr = 0, rs[16], rw[16], rd[16];
    for (int i = 0; i < lb; ++i) {
      const int tb = i < bk ? i : i + kRegBits;
      const int d = s.pos[tb];
      if (d == kDummy) continue;
      if (nr > 0 && rs[nr - 1] + rw[nr - 1] == i && rd[nr - 1] + rw[nr - 1] == d) {
        rw[nr - 1]++;
      } else {
        rs[nr] = i;
        rw[nr] = 1;
        rd[nr] = d;
        ++nr;
      }
      if (d >= 32) s.tr64 = 1;
    }
    // a set the planner builds holds the five lowest bits, one run of other qubits and
    // at most one block of far qubits (make_sets): at most four runs
    if (nr > kMaxRuns) std::abort();
    for (int i = 0; i < kMaxRuns; ++i)
      s.trun[ki][i] = i < nr ? (uint32_t)rs[i] | ((uint32_t)rw[i] << 8) | ((uint32_t)rd[i] << 16) : 0u;
  }
}

constexpr int kFarQubit = 26;  // first qubit spread over the sets by make_sets (see there)

std::vector<SetSpec> make_sets(int n, int L) {
  std::vector<SetSpec> sets;
  if (n <= L) {
    SetSpec s;
    std::memset(&s, 0, sizeof(s));
    for (int j = 0; j < 16; ++j) s.pos[j] = (j < n) ? (uint8_t)j : kDummy;
    s.act = (1u << n) - 1u;
    s.dummy = ((1u << L) - 1u) & ~s.act;
    s.fixmask = 0;
    s.ntiles = 1;
    finish_set(s, L, true);
    sets.push_back(s);
    return sets;
  }
  const int cap_rest = L - kMinContig;
  int k = 1 + (n - L + cap_rest - 1) / cap_rest;
  std::vector<int> a(k);
  a[0] = L;
  for (int s = 1; s < k; ++s) a[s] = cap_rest;
  int tot = L + (k - 1) * cap_rest;
  while (tot > n) {  // shave the largest set (set 0 first on ties) keeping a_0 >= 5
    int best = -1;
    for (int s = 0; s < k; ++s) {
      if (s == 0 && a[0] <= kMinContig) continue;
      if (a[s] <= 1) continue;
      if (best < 0 || a[s] > a[best]) best = s;
    }
    a[best]--;
    tot--;
  }
  // Active qubits of the sets.  Set 0 takes the lowest a[0].  Qubits from kFarQubit up
  // (byte strides of 512 MiB and more in a complex64 state) are split into consecutive
  // blocks over the later sets, as evenly as possible, the last set (which also holds
  // qubit n-1, its top tile bit) taking the smallest; the other qubits fill the rest of each
  // set in order.  A tile spans 2^m address ranges that far apart when it holds m such
  // qubits (twice as many with the mirrored registers of the half state), and the compute
  // unit's first-level address translation cache misses once they are many: at n = 34 the
  // plain sweep of the set holding qubits 26..33 missed on 11 % of its lookups and ran 20 %
  // slower than the set-0 sweep; with the blocks spread the misses are 0.1 % and the two
  // sweeps take about the same time.
  std::vector<std::vector<int>> act_of(k);
  for (int i = 0; i < a[0]; ++i) act_of[0].push_back(i);
  {
    const int h = k - 1, f0 = std::max(a[0], kFarQubit), f = std::max(0, n - f0);
    // the last set, whose mirrored registers double its pages, takes the smallest block
    std::vector<int> blk(h, 0);
    blk[h - 1] = std::max(f > 0 ? 1 : 0, f / h);
    const int rest = f - blk[h - 1];
    for (int s = 0; s + 1 < h; ++s) blk[s] = rest / (h - 1) + (s < rest % (h - 1) ? 1 : 0);
    int near = a[0], far = f0;
    for (int s = 1; s < k; ++s) {
      const int nn = a[s] - blk[s - 1];
      if (nn < 0) std::abort();  // a block never exceeds its set (f <= 36 < k - 1 sets of >= 5)
      for (int i = 0; i < nn; ++i) act_of[s].push_back(near++);
      for (int i = 0; i < blk[s - 1]; ++i) act_of[s].push_back(far++);
    }
    if (near != std::min(n, f0) || far != std::max(n, f0)) std::abort();
  }
  for (int s = 0; s < k; ++s) {
    SetSpec S;
    std::memset(&S, 0, sizeof(S));
    const std::vector<int>& active = act_of[s];
    std::vector<int> bits;
    if (s == 0) {
      for (int j = 0; j < L; ++j) bits.push_back(j);
    } else {
      std::set<int> act(active.begin(), active.end());
      bits = active;
      for (int gbit = 0; (int)bits.size() < L; ++gbit)
        if (!act.count(gbit)) bits.push_back(gbit);
      std::sort(bits.begin(), bits.end());
    }
    uint64_t tilemask = 0;
    for (int j = 0; j < L; ++j) {
      S.pos[j] = (uint8_t)bits[j];
      tilemask |= 1ull << bits[j];
      if (std::find(active.begin(), active.end(), bits[j]) != active.end()) S.act |= 1u << j;
    }
    for (int j = L; j < 16; ++j) S.pos[j] = kDummy;
    S.dummy = 0;
    const uint64_t all = (n >= 64) ? ~0ull : ((1ull << n) - 1ull);
    S.fixmask = all & ~tilemask;
    S.ntiles = 1u << (n - L);
    finish_set(S, L, s == 0);
    sets.push_back(S);
  }
  return sets;
}

// ------------------------------------------------------------------ tile size choice
// Tile sizes (log2 amplitudes per workgroup tile) with compiled sweep kernels: 12
// (256-thread workgroups) and 13 (512 threads).  Built-in rule: the fewest tile sets
// (= sweeps per layer); on ties the 12-bit tile, whose workgroups are smaller (more of
// them resident per compute unit) and whose mixer needs one LDS transpose fewer.
int sets_for(int n, int L) { return (int)make_sets(n, L).size(); }
int auto_tile_bits(int n) {
  if (n <= 12) return 12;
  return sets_for(n, 12) <= sets_for(n, 13) ? 12 : 13;
}
bool sweep_tile_ok(int L) { return L == 12 || L == 13; }
std::mutex g_tune_mu;
std::map<std::tuple<int, int, int>, int> g_tune;  // (n, complex128, gradient) -> tile bits
int chosen_tile_bits(int n, bool dbl, bool grad) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_tune.find(std::make_tuple(n, (int)dbl, (int)grad));
  return it == g_tune.end() ? auto_tile_bits(n) : it->second;
}

// Set of forward sweep i.  Positions i = 0, k-1, 2(k-1), ... are the layer boundaries
// (plus the first and the last sweep): such a sweep mixes the end of one layer and the
// start of the next (or the first / last part of the circuit) on one set.  With k >= 3
// they alternate between sets 1 and 2, and the k-2 sweeps between two of them mix the
// other sets (0, 3, ..., k-1), each once: every layer then visits every set exactly once,
// and set 0, whose twelve- or thirteen-qubit mixer needs the most work and transposes,
// only ever gets a plain sweep (one mixer, no phase).  With k = 2 the boundaries
// alternate between sets 1 and 0.
int zig(int i, int k) {
  if (k == 1) return 0;
  const int seg = i / (k - 1), pos = i % (k - 1);
  if (k == 2) return (seg % 2 == 0) ? 1 : 0;
  if (pos == 0) return (seg % 2 == 0) ? 1 : 2;
  return pos == 1 ? 0 : pos + 1;  // plain sweeps: sets 0, 3, 4, ..., k-1
}

SweepProg blank() {
  SweepProg s;
  std::memset(&s, 0, sizeof(s));
  s.pre_layer = s.mid_layer = s.mixA_layer = s.mixB_layer = -1;
  return s;
}

// Forward (and, with grad, backward) sweep programs.
//  multi-set (k >= 2): zig-zag over the sets; each layer boundary (phase) sits inside
//  a sweep that finishes layer l's mixing on its set, applies the next phase and starts
//  layer l+1 on the same set, so p layers take p(k-1)+1 sweeps.  The last forward sweep
//  evaluates h(z) and, for gradients, creates lambda = h psi and undoes the last mixer
//  part on both states; the backward sweeps mirror the forward ones.
//  single set (k == 1): the whole state is one tile; a sweep strings together
//  [ops, mixer, ops, mixer] and the program is the plain gate sequence.
std::vector<SweepProg> build_progs(int k, int p, bool grad, uint8_t energy_ops, bool store_final, bool ckpt = false) {
  std::vector<SweepProg> out;
  if (k == 1) {
    struct Step {
      bool mix;
      uint8_t ops;
      int layer;
      int dir;
      bool grad;
    };
    std::vector<Step> st;
    for (int l = 0; l < p; ++l) {
      st.push_back({false, OP_PHASE, l, 0, false});
      st.push_back({true, 0, l, +1, false});
    }
    st.push_back({false, energy_ops, -1, 0, false});
    if (grad) {
      for (int l = p - 1; l >= 0; --l) {
        st.push_back({true, 0, l, -1, true});
        st.push_back({false, (uint8_t)(l > 0 ? (OP_GRADG | OP_UNPHASE) : OP_GRADG), l, 0, false});
      }
    }
    bool lam = false;
    for (size_t i = 0; i < st.size(); i += 4) {
      SweepProg s = blank();
      s.set = 0;
      const bool first = i == 0, last = i + 4 >= st.size();
      s.flags = first ? F_INIT : (uint8_t)(F_LOAD_PSI | (lam ? (F_LOAD_LAM | F_LAM_LIVE) : 0));
      for (size_t j = i; j < std::min(st.size(), i + 4); ++j) {
        const Step& x = st[j];
        const int slot = (int)(j - i);
        if (slot == 0) {
          s.pre_ops = x.ops;
          s.pre_layer = (int8_t)x.layer;
        } else if (slot == 1) {
          s.mixA_layer = (int8_t)x.layer;
          s.mixA_dir = (int8_t)x.dir;
          s.mixA_grad = x.grad;
        } else if (slot == 2) {
          s.mid_ops = x.ops;
          s.mid_layer = (int8_t)x.layer;
        } else {
          s.mixB_layer = (int8_t)x.layer;
          s.mixB_dir = (int8_t)x.dir;
          s.mixB_grad = x.grad;
        }
        if (!x.mix && (x.ops & OP_ENERGY) && grad) {
          s.flags |= F_MAKE_LAM;
          lam = true;
        }
      }
      if (!last) s.flags |= F_STORE_PSI | (lam ? F_STORE_LAM : 0);
      if (last && store_final) s.flags |= F_STORE_PSI;
      out.push_back(s);
    }
    return out;
  }
  const int F = p * (k - 1) + 1;
  for (int i = 0; i < F; ++i) {
    SweepProg s = blank();
    s.set = (int8_t)zig(i, k);
    if (i == 0) {
      s.flags = F_INIT | F_STORE_PSI;
      s.pre_ops = OP_PHASE;
      s.pre_layer = 0;
      s.mixA_layer = 0;
      s.mixA_dir = 1;
    } else if (i < F - 1) {
      s.flags = F_LOAD_PSI | F_STORE_PSI;
      s.mixA_layer = (int8_t)((i - 1) / (k - 1));
      s.mixA_dir = 1;
      if (i % (k - 1) == 0) {
        const int l = i / (k - 1);
        s.mid_ops = OP_PHASE;
        s.mid_layer = (int8_t)l;
        s.mixB_layer = (int8_t)l;
        s.mixB_dir = 1;
      }
    } else {
      s.flags = F_LOAD_PSI;
      s.mixA_layer = (int8_t)(p - 1);
      s.mixA_dir = 1;
      s.mid_ops = energy_ops;
      if (grad) {
        s.flags |= F_MAKE_LAM | F_STORE_LAM;
        s.mixB_layer = (int8_t)(p - 1);
        s.mixB_dir = -1;
        s.mixB_grad = 1;
      }
      if (store_final) s.flags |= F_STORE_PSI;
    }
    out.push_back(s);
  }
  if (grad) {
    for (int i = F - 2; i >= 0; --i) {
      SweepProg s = blank();
      s.set = (int8_t)zig(i, k);
      s.flags = F_LOAD_PSI | F_LOAD_LAM | F_LAM_LIVE | F_STORE_PSI | F_STORE_LAM;
      if (i == 0) {
        s.flags = F_LOAD_PSI | F_LOAD_LAM | F_LAM_LIVE;
        s.mixA_layer = 0;
        s.mixA_dir = -1;
        s.mixA_grad = 1;
        s.mid_ops = OP_GRADG;
        s.mid_layer = 0;
      } else if (i % (k - 1) == 0) {
        const int l = i / (k - 1);
        s.mixA_layer = (int8_t)l;
        s.mixA_dir = -1;
        s.mixA_grad = 1;
        s.mid_ops = OP_GRADG | OP_UNPHASE;
        s.mid_layer = (int8_t)l;
        s.mixB_layer = (int8_t)(l - 1);
        s.mixB_dir = -1;
        s.mixB_grad = 1;
      } else {
        s.mixA_layer = (int8_t)((i - 1) / (k - 1));
        s.mixA_dir = -1;
        s.mixA_grad = 1;
      }
      out.push_back(s);
    }
  }
  if (ckpt && grad) {
    // forward-state checkpoints: forward sweep i (< F - 1) stores psi into buffer i and
    // sweep i + 1 reads it; backward sweep i reads psi from buffer i and stores only
    // lambda, since the state before it is already in buffer i - 1
    for (int i = 0; i < F; ++i) {
      out[i].ld_buf = (uint8_t)(i > 0 ? i - 1 : 0);
      out[i].st_buf = (uint8_t)i;
    }
    for (int j = F; j < (int)out.size(); ++j) {
      const int i = F - 2 - (j - F);
      out[j].ld_buf = (uint8_t)i;
      out[j].flags &= (uint8_t)~F_STORE_PSI;
    }
  }
  return out;
}

// number of psi buffers a program reads or writes
int prog_buffers(const std::vector<SweepProg>& progs) {
  int nb = 1;
  for (const SweepProg& s : progs) {
    if (s.flags & F_LOAD_PSI) nb = std::max(nb, s.ld_buf + 1);
    if (s.flags & F_STORE_PSI) nb = std::max(nb, s.st_buf + 1);
  }
  return nb;
}

bool needs_two_states(const SweepProg& s) {
  return (s.flags & (F_LAM_LIVE | F_MAKE_LAM | F_LOAD_LAM)) != 0;
}

// ------------------------------------------------------------------ single-instance layout
struct Layout {
  size_t graph = 0, terms = 0, params = 0, src = 0, srcb = 0, progs = 0, sets = 0, upload_end = 0;
  size_t tab = 0, scales = 0, partial = 0, zzpart = 0, stage = 0, out = 0, total = 0;
  int nsweep = 0, nslot = 0, ntiles = 0, nout = 0, nsrc = 0, T = 0;
};

constexpr int kZZBlocks = 1024;

struct Single {
  int n, p, T, cmax, L, k, nbuf;
  bool dbl, grad;
  bool weighted = false;  // integer edge weights: the sweeps cut from the per-set cost-term lists
  bool half = false;      // half state (spin-flip symmetry): 2^(n-1) stored amplitudes
  aaq_aggregation agg;
  std::vector<SetSpec> sets;
  std::vector<int4> terms;  // plain term list, then the per-set sorted lists
  std::vector<SweepProg> progs;
  std::vector<RedSrcHost> src;
  std::vector<int32_t> srcb;
  std::vector<int> grids;
  Layout lay;
};

// The global spin-flip symmetry of MaxCut QAOA: |+>, the cut phase (C(~z) = C(z)) and the
// mixer commute with flipping every bit, and so do h and lambda = h psi, so every buffer the
// sweeps touch (sigma psi(z ^ F), lambda) takes equal values at z and ~z.  The half state
// keeps the indices below 2^(n-1); each sweep runs the tiles below ntiles / 2.  Sets other
// than the last hold bit n-1 as the top tile-id bit, so those tiles lie in the stored half;
// the last set holds bit n-1 as its top tile bit (a register bit at the load arrangement),
// and the registers with that bit set read and write the mirrored index 2^n - 1 - index,
// which is the complement tile's stored element.  Every stored amplitude is then touched
// once per sweep, and every sum counts one of each equal pair.
std::atomic<bool> g_half_state{true};

// whether the sets of an n-qubit program at tile size L can sweep the half state
bool sets_half_ok(const std::vector<SetSpec>& sets, int n, int L, bool dbl) {
  if (!g_half_state || sets.size() < 2) return false;
  // The sweeps address a stored state with 32-bit buffer offsets when its 2^(n-1)
  // amplitudes span at most 4 GiB; the mirrored offsets of that path are formed over the
  // full index range, so it needs 2^n amplitudes within 4 GiB.  Larger states take 64-bit
  // addresses, mirrored offsets included.  Only the size in between (2^n amplitudes above
  // 4 GiB, their half within it: n = 30 in complex64) keeps the full state.
  const uint64_t amp = dbl ? 16u : 8u;
  const bool full32 = (((uint64_t)1 << n) * amp) <= ((uint64_t)1 << 32);
  const bool half64 = (((uint64_t)1 << (n - 1)) * amp) > ((uint64_t)1 << 32);
  if (!full32 && !half64) return false;
  const SetSpec& last = sets.back();
  const int b0l = geo_b0(geo_na(L) - 1, L);
  if (last.pos[L - 1] != n - 1 || b0l + kRegBits != L) return false;
  for (size_t i = 0; i + 1 < sets.size(); ++i)  // bit n-1 is the top tile-id bit
    if (!((sets[i].fixmask >> (n - 1)) & 1u)) return false;
  return true;
}
bool half_state_ok(const Single& S, aaq_aggregation agg, bool keep_state) {
  if (S.k < 2 || agg == AAQ_AGG_PASS_PER_TERM || keep_state) return false;
  return sets_half_ok(S.sets, S.n, S.L, S.dbl);
}

// the last set's mirrored registers (those whose index has bit n-1 set)
void mark_mirror(std::vector<SetSpec>& sets, int n, int L) {
  SetSpec& last = sets.back();
  const int b0l = geo_b0(geo_na(L) - 1, L);
  last.mirror = 0;
  for (int r = 0; r < (1 << kRegBits); ++r)
    if ((last.roff[r] >> (n - 1)) & 1u) last.mirror |= (uint16_t)(1u << r);
  last.tmax = 0;
  for (int j = 0; j < b0l; ++j)
    if (last.pos[j] != kDummy) last.tmax |= (uint64_t)1 << last.pos[j];
  last.mfull = ((uint64_t)1 << n) - 1;
}
void mark_mirror(Single& S) { mark_mirror(S.sets, S.n, S.L); }

// grids: persistent workgroups per sweep (empty: one per tile, the upper bound used for
// sizing); partial sums are laid out [sweep][slot][tile] with a tile-count stride.
aaq_status plan_single(const aaq_problem* pr, int p, bool grad, aaq_observable obs, aaq_aggregation agg,
                       aaq_precision prec, int tile, Single& S, bool with_grids = false, bool ckpt = false,
                       bool keep_state = false, bool allow_half = true) {
  if (obs != AAQ_OBS_HC && obs != AAQ_OBS_HRED) return fail(AAQ_ERR_INVALID_ARG, "bad observable");
  if (agg != AAQ_AGG_FUSED && agg != AAQ_AGG_PER_TERM && agg != AAQ_AGG_PASS_PER_TERM)
    return fail(AAQ_ERR_INVALID_ARG, "bad aggregation");
  if (prec != AAQ_PREC_C64 && prec != AAQ_PREC_C128) return fail(AAQ_ERR_INVALID_ARG, "bad precision");
  if (grad && agg != AAQ_AGG_FUSED) return fail(AAQ_ERR_UNSUPPORTED, "gradients use fused aggregation");
  S.n = pr->n;
  S.p = p;
  S.dbl = prec == AAQ_PREC_C128;
  S.grad = grad;
  S.agg = agg;
  S.T = (obs == AAQ_OBS_HC) ? pr->num_edges : pr->num_orbits;
  S.cmax = total_weight(pr);
  S.weighted = is_weighted(pr);
  S.L = tile;
  S.sets = make_sets(S.n, S.L);
  S.terms = term_array(pr, obs, S.L, S.sets);
  S.k = (int)S.sets.size();
  uint8_t eops = OP_ENERGY | (agg == AAQ_AGG_PER_TERM ? OP_PERTERM : 0);
  S.progs = build_progs(S.k, p, grad, eops, agg == AAQ_AGG_PASS_PER_TERM || keep_state, ckpt && grad && S.k >= 2);
  S.nbuf = prog_buffers(S.progs);
  if (S.nbuf > kMaxCkpt) return fail(AAQ_ERR_UNSUPPORTED, "too many checkpoint states for this depth (max 32)");
  S.half = allow_half && half_state_ok(S, agg, keep_state);
  if (S.half) mark_mirror(S);
  Layout& L = S.lay;
  L.nsweep = (int)S.progs.size();
  L.T = S.T;
  L.nslot = SLOT_TERMS + (agg == AAQ_AGG_PER_TERM ? S.T : 0);
  L.ntiles = (int)S.sets[0].ntiles >> (S.half ? 1 : 0);
  const bool zzp = agg == AAQ_AGG_PASS_PER_TERM;
  // with the half state every sum covers one of each pair (z, ~z) of equal terms
  const double hs = S.half ? 2.0 : 1.0;
  L.nout = 2 + 2 * p + ((agg != AAQ_AGG_FUSED) ? S.T : 0);
  // reduction sources
  std::vector<std::vector<RedSrcHost>> per(L.nout);
  auto part_off = [&](int sw, int slot) { return (int64_t)(sw * L.nslot + slot) * L.ntiles; };
  S.grids.assign(L.nsweep, L.ntiles);
  for (int sw = 0; sw < L.nsweep; ++sw) {
    const SweepProg& s = S.progs[sw];
    const int np = S.grids[sw];
    auto add = [&](int o, int slot, double scale) { per[o].push_back({part_off(sw, slot), np, o, hs * scale}); };
    if ((s.pre_ops | s.mid_ops) & OP_ENERGY) {
      add(0, SLOT_E, 1.0);
      add(1, SLOT_NORM, 1.0);
      if (agg == AAQ_AGG_PER_TERM)
        for (int t = 0; t < S.T; ++t) add(2 + 2 * p + t, SLOT_TERMS + t, 1.0);
    }
    if (s.pre_ops & OP_GRADG) add(2 + s.pre_layer, SLOT_GPRE, 2.0);
    if (s.mid_ops & OP_GRADG) add(2 + s.mid_layer, SLOT_GMID, 2.0);
    if (s.mixA_grad) add(2 + p + s.mixA_layer, SLOT_BA, 2.0);
    if (s.mixB_grad) add(2 + p + s.mixB_layer, SLOT_BB, 2.0);
  }
  size_t off = 0;
  L.graph = off;
  off = align_up(off + sizeof(GraphDev));
  L.terms = off;
  off = align_up(off + sizeof(int4) * std::max<size_t>(S.terms.size(), 1));
  L.params = off;
  off = align_up(off + sizeof(double) * 2 * p);
  // the zz-pass partial area starts after the sweep partials
  const int64_t sweep_part = (int64_t)L.nsweep * L.nslot * L.ntiles;
  if (zzp)
    for (int t = 0; t < S.T; ++t) per[2 + 2 * p + t].push_back({sweep_part + (int64_t)t * kZZBlocks, kZZBlocks, 2 + 2 * p + t, 1.0});
  S.src.clear();
  S.srcb.assign(L.nout + 1, 0);
  for (int o = 0; o < L.nout; ++o) {
    S.srcb[o] = (int32_t)S.src.size();
    for (auto& x : per[o]) S.src.push_back(x);
  }
  S.srcb[L.nout] = (int32_t)S.src.size();
  L.nsrc = (int)S.src.size();
  L.src = off;
  off = align_up(off + sizeof(RedSrcHost) * std::max(L.nsrc, 1));
  L.srcb = off;
  off = align_up(off + sizeof(int32_t) * (L.nout + 1));
  L.progs = off;
  off = align_up(off + sizeof(SweepProg) * L.nsweep);
  L.sets = off;
  off = align_up(off + sizeof(SetSpec) * S.sets.size());
  L.upload_end = off;
  const size_t amp = S.dbl ? 16 : 8;
  L.tab = off;
  off = align_up(off + amp * (size_t)p * (S.cmax + 1));
  L.scales = off;
  off = align_up(off + sizeof(SwScale) * (L.nsweep + 1));
  L.partial = off;
  off = align_up(off + sizeof(double) * (size_t)(sweep_part + (zzp ? (int64_t)S.T * kZZBlocks : 0)));
  L.stage = off;
  off = align_up(off + sizeof(double) * (size_t)L.nout * kReduceChunks);
  L.out = off;
  off = align_up(off + sizeof(double) * L.nout);
  L.total = off;
  return AAQ_OK;
}

// the inputs that determine a single-instance host plan
struct PlanKey {
  std::vector<int32_t> v;
  bool operator==(const PlanKey& o) const { return v == o.v; }
};
PlanKey plan_key(const aaq_problem* pr, int p, bool grad, aaq_observable obs, aaq_aggregation agg, aaq_precision prec,
                 int tile, bool ckpt, bool keep_state) {
  PlanKey k;
  k.v = {pr->n, pr->num_edges, pr->num_orbits, p, (int)grad, (int)obs, (int)agg, (int)prec, tile, (int)ckpt,
         pr->edge_orbit ? 1 : 0, (int)keep_state, (int)g_half_state.load()};
  k.v.insert(k.v.end(), pr->edges, pr->edges + 2 * pr->num_edges);
  if (pr->num_orbits > 0) {
    k.v.insert(k.v.end(), pr->orbit_rep, pr->orbit_rep + pr->num_orbits);
    k.v.insert(k.v.end(), pr->orbit_size, pr->orbit_size + pr->num_orbits);
  }
  for (int e = 0; e < pr->num_edges; ++e) k.v.push_back(edge_weight(pr, e));
  return k;
}

// per-thread pinned host buffer for the argument upload and the result download; it
// grows as needed and is kept for the life of the process
unsigned char* pinned_staging(size_t bytes) {
  thread_local unsigned char* buf = nullptr;
  thread_local size_t cap = 0;
  if (bytes > cap) {
    if (buf) (void)hipHostFree(buf);
    buf = nullptr;
    cap = 0;
    const size_t want = std::max(align_up(bytes, 4096), (size_t)65536);
    if (hipHostMalloc((void**)&buf, want, hipHostMallocDefault) != hipSuccess) return nullptr;
    cap = want;
  }
  return buf;
}

// the same role in ordinary host memory, for calls that must not allocate pinned memory;
// it grows on the host heap as needed and is kept for the life of the thread
unsigned char* pageable_staging(size_t bytes) {
  thread_local std::vector<unsigned char> buf;
  if (buf.size() < bytes) buf.resize(std::max(align_up(bytes, 4096), (size_t)65536));
  return buf.data();
}

// checks the caller's buffers against a host plan
aaq_status check_buffers(const Single& S, bool grad, void* d_state, size_t state_bytes, void* d_lam, size_t lam_bytes,
                         void* d_ws, size_t ws_bytes) {
  const size_t need_state = ((size_t)1 << (S.n - (S.half ? 1 : 0))) * (S.dbl ? 16 : 8);
  if (!d_state) return fail(AAQ_ERR_INVALID_ARG, "d_state is NULL");
  if (state_bytes < need_state * S.nbuf)
    return fail(AAQ_ERR_BUFFER, S.nbuf > 1 ? "checkpoint buffer smaller than the forward states it holds"
                                           : "state buffer smaller than 2^n amplitudes");
  if (grad) {
    if (!d_lam) return fail(AAQ_ERR_INVALID_ARG, "d_lambda is NULL");
    if (lam_bytes < need_state) return fail(AAQ_ERR_BUFFER, "lambda buffer smaller than 2^n amplitudes");
  }
  if (!d_ws) return fail(AAQ_ERR_INVALID_ARG, "workspace is NULL");
  if (ws_bytes < S.lay.total) return fail(AAQ_ERR_BUFFER, "workspace too small (need " + std::to_string(S.lay.total) + " bytes)");
  return AAQ_OK;
}

// the parameter-independent part of the upload block (graph, terms, reduction sources,
// sweep programs, tile sets) into the staging area `up`
void stage_static(const Single& S, const aaq_problem* pr, aaq_observable obs, unsigned char* up) {
  const Layout& L = S.lay;
  std::memset(up, 0, L.upload_end);
  GraphDev g = make_graph(pr);
  g.T = S.T;
  g.h_is_cut = obs == AAQ_OBS_HC && !g.weighted;
  std::memcpy(up + L.graph, &g, sizeof(g));
  if (!S.terms.empty()) std::memcpy(up + L.terms, S.terms.data(), sizeof(int4) * S.terms.size());
  if (!S.src.empty()) std::memcpy(up + L.src, S.src.data(), sizeof(RedSrcHost) * S.src.size());
  std::memcpy(up + L.srcb, S.srcb.data(), sizeof(int32_t) * S.srcb.size());
  std::memcpy(up + L.progs, S.progs.data(), sizeof(SweepProg) * S.progs.size());
  std::memcpy(up + L.sets, S.sets.data(), sizeof(SetSpec) * S.sets.size());
}

// One evaluation on the device, asynchronous on `hs`: phase tables from the device
// parameters, the sweeps, the pass-per-term <ZZ> passes, and the fixed-order reduction
// into d_out (energy, norm, dgamma[p], dbeta[p], then per-term sums).  The workspace
// holds the uploaded static block.
aaq_status launch_eval(const Single& S, bool grad, void* d_state, void* d_lam, unsigned char* ws, const double* d_gamma,
                       const double* d_beta, double* d_out, hipStream_t hs) {
  const Layout& L = S.lay;
  const int p = S.p;
  const int nst = S.n - (S.half ? 1 : 0);  // stored amplitudes per state: 2^nst
  const size_t need_state = ((size_t)1 << nst) * (S.dbl ? 16 : 8);
  const bool weighted = S.weighted;
  const aaq_aggregation agg = S.agg;
  {
    TimedLaunch tl(KC_TABLES, 0.0, hs);
    HIPCHK(launch_tables(d_gamma, d_beta, p, S.cmax, ws + L.tab, (const SweepProg*)(ws + L.progs), L.nsweep,
                         (const SetSpec*)(ws + L.sets), (int)S.sets.size(), (SwScale*)(ws + L.scales), S.dbl, hs));
    tl.done();
  }
  for (int sw = 0; sw < L.nsweep; ++sw) {
    LaunchSweep A;
    A.psi = d_state;
    A.lam = grad ? d_lam : nullptr;
    A.g = (const GraphDev*)(ws + L.graph);
    A.terms = (const int4*)(ws + L.terms);
    A.tab = ws + L.tab;
    A.scale = (const SwScale*)(ws + L.scales) + sw;
    A.partial = (double*)(ws + L.partial) + (size_t)sw * L.nslot * L.ntiles;
    A.nslot = L.nslot;
    A.T = S.T;
    A.cmax = S.cmax;
    A.amp = std::exp2(-0.5 * S.n);
    A.N = (uint64_t)1 << nst;
    A.set = S.sets[S.progs[sw].set];
    A.prog = S.progs[sw];
    A.two_states = needs_two_states(S.progs[sw]);
    A.weighted = weighted;  // the weighted copies of the specialised shapes
    A.half = S.half;
    // non-temporal loads unless the whole evaluation is one state that fits the 256 MB
    // last-level cache (in-place energy sweeps then reuse it from sweep to sweep)
    A.nt = grad || need_state > ((size_t)256 << 20);
    const SweepProg& pg = S.progs[sw];
    const int moves = !!(pg.flags & F_LOAD_PSI) + !!(pg.flags & F_LOAD_LAM) + !!(pg.flags & F_STORE_PSI) +
                      !!(pg.flags & F_STORE_LAM);
    TimedLaunch tl(A.two_states ? KC_SWEEP2 : KC_SWEEP1, (double)moves * (double)need_state, hs);
    HIPCHK(launch_sweep(A, S.dbl, S.L, hs));
    tl.done();
  }
  if (agg == AAQ_AGG_PASS_PER_TERM) {
    double* zp = (double*)(ws + L.partial) + (size_t)L.nsweep * L.nslot * L.ntiles;
    for (int t = 0; t < S.T; ++t) {
      TimedLaunch tl(KC_ZZPASS, (double)need_state, hs);
      HIPCHK(launch_zz_pass(d_state, (uint64_t)1 << S.n, S.terms[t].x, S.terms[t].y,
                            &((const SwScale*)(ws + L.scales) + L.nsweep)->s_pre,
                            &((const SwScale*)(ws + L.scales) + L.nsweep)->F_pre, zp + (size_t)t * kZZBlocks, kZZBlocks,
                            S.dbl, hs));
      tl.done();
    }
  }
  {
    TimedLaunch tl(KC_REDUCE, 0.0, hs);
    HIPCHK(launch_reduce((const double*)(ws + L.partial), ws + L.src, (const int32_t*)(ws + L.srcb),
                         (double*)(ws + L.stage), d_out, L.nout, hs));
    tl.done();
  }
  return AAQ_OK;
}

aaq_status run_single(const aaq_problem* pr, int p, const double* gamma, const double* beta, aaq_observable obs,
                      aaq_aggregation agg, aaq_precision prec, bool grad, void* d_state, size_t state_bytes,
                      void* d_lam, size_t lam_bytes, void* d_ws, size_t ws_bytes, void* stream, std::vector<double>& res,
                      int tile = 0, bool ckpt = false, bool keep_state = false, Single* plan_out = nullptr,
                      bool pageable = false) {
  aaq_status st = validate_problem(pr);
  if (st) return st;
  if ((st = validate_p(p))) return st;
  if ((st = validate_params(p, gamma, beta))) return st;
  if (!tile) tile = chosen_tile_bits(pr->n, prec == AAQ_PREC_C128, grad);
  // the host plan of the last call on this thread is reused when the instance and the
  // shape of the call are the same (repeated evaluations at new parameters)
  thread_local PlanKey last_key;
  thread_local Single last_plan;
  thread_local bool have_last = false;
  PlanKey key = plan_key(pr, p, grad, obs, agg, prec, tile, ckpt, keep_state);
  if (!have_last || !(key == last_key)) {
    have_last = false;
    if ((st = plan_single(pr, p, grad, obs, agg, prec, tile, last_plan, true, ckpt, keep_state))) return st;
    last_key = std::move(key);
    have_last = true;
  }
  const Single& S = last_plan;
  if ((st = check_buffers(S, grad, d_state, state_bytes, d_lam, lam_bytes, d_ws, ws_bytes))) return st;
  const Layout& L = S.lay;
  hipStream_t hs = (hipStream_t)stream;
  unsigned char* ws = (unsigned char*)d_ws;
  // host staging of everything that is uploaded (pinned, reused: the copies are
  // asynchronous, and the call ends with a stream synchronisation)
  unsigned char* up = pageable ? pageable_staging(L.upload_end + sizeof(double) * L.nout)
                               : pinned_staging(L.upload_end + sizeof(double) * L.nout);
  if (!up) return fail(AAQ_ERR_HIP, "hipHostMalloc of the staging buffer failed");
  stage_static(S, pr, obs, up);
  std::memcpy(up + L.params, gamma, sizeof(double) * p);
  std::memcpy(up + L.params + sizeof(double) * p, beta, sizeof(double) * p);
  HIPCHK(hipMemcpyAsync(ws, up, L.upload_end, hipMemcpyHostToDevice, hs));
  const double* dparams = (const double*)(ws + L.params);
  if ((st = launch_eval(S, grad, d_state, d_lam, ws, dparams, dparams + p, (double*)(ws + L.out), hs))) return st;
  const std::vector<int4>& terms = S.terms;
  double* down = (double*)(up + L.upload_end);
  HIPCHK(hipMemcpyAsync(down, ws + L.out, sizeof(double) * L.nout, hipMemcpyDeviceToHost, hs));
  HIPCHK(hipStreamSynchronize(hs));
  res.assign(down, down + L.nout);
  if (agg != AAQ_AGG_FUSED) {
    // energy from the per-term <ZZ>: sum_t (w_t/2)(1 - <ZZ>_t)
    double e = 0.0;
    for (int t = 0; t < S.T; ++t) e += 0.5 * terms[t].z * (1.0 - res[2 + 2 * p + t]);
    res[0] = e;
  }
  if (plan_out) *plan_out = S;
  return AAQ_OK;
}

// ------------------------------------------------------------------ final-state sampling
constexpr int kSampleBlockBits = 13;  // CDF blocks of 2^13 bitstrings

int sample_block_bits(int n) { return std::min(n, kSampleBlockBits); }

// sub-block sums: one FP64 sum per 64 bitstrings (per block when a block is smaller)
size_t sample_sub_count(int n) { return (size_t)1 << (n - std::min(sample_block_bits(n), 6)); }

size_t sample_extra_bytes(int n) {
  const size_t nb = (size_t)1 << (n - sample_block_bits(n));
  return align_up(sizeof(double) * nb) * 2 + align_up(sizeof(double) * 2) + align_up(sizeof(double) * sample_sub_count(n));
}

aaq_status run_sample(const aaq_problem* pr, int p, const double* gamma, const double* beta, aaq_precision prec,
                      int shots, const double* d_uniform, void* d_state, size_t state_bytes, void* d_ws, size_t ws_bytes,
                      void* stream, uint64_t* d_samples, int32_t* d_cuts, double* best_out, double* mean_out) {
  aaq_status st = validate_problem(pr);
  if (st) return st;
  if (pr->num_edges == 0) return fail(AAQ_ERR_UNSUPPORTED, "a graph without edges has nothing to sample for");
  if (shots < 1) return fail(AAQ_ERR_INVALID_ARG, "num_shots must be >= 1");
  if (!d_uniform || !d_samples || !d_cuts) return fail(AAQ_ERR_INVALID_ARG, "d_uniform / d_samples / d_cuts is NULL");
  const size_t extra = sample_extra_bytes(pr->n);
  if (ws_bytes < extra) return fail(AAQ_ERR_BUFFER, "workspace too small for sampling");
  // the forward pass keeps the final state; its own workspace is everything before the
  // sampling area at the end of the caller's workspace
  std::vector<double> res;
  Single S;
  if ((st = run_single(pr, p, gamma, beta, AAQ_OBS_HC, AAQ_AGG_FUSED, prec, false, d_state, state_bytes, nullptr, 0,
                       d_ws, ws_bytes - extra, stream, res, 0, false, true, &S)))
    return st;
  hipStream_t hs = (hipStream_t)stream;
  unsigned char* ws = (unsigned char*)d_ws;
  // sampling area right after the forward pass's layout: [block sums][cumulative sums][best, mean]
  unsigned char* sw = ws + S.lay.total;
  const int lb = sample_block_bits(S.n);
  const size_t nb = (size_t)1 << (S.n - lb);
  double* bsum = (double*)sw;
  double* cum = (double*)(sw + align_up(sizeof(double) * nb));
  double* stats = (double*)(sw + 2 * align_up(sizeof(double) * nb));
  double* ssum = (double*)(sw + 2 * align_up(sizeof(double) * nb) + align_up(sizeof(double) * 2));
  const SwScale* fin = (const SwScale*)(ws + S.lay.scales) + S.lay.nsweep;
  HIPCHK(launch_sample(d_state, S.n, lb, bsum, cum, ssum, &fin->F_pre, d_uniform, shots, (const GraphDev*)(ws + S.lay.graph),
                       (const int4*)(ws + S.lay.terms), d_samples, d_cuts, stats, S.dbl, hs));
  double h[2];
  HIPCHK(hipMemcpyAsync(h, stats, sizeof(h), hipMemcpyDeviceToHost, hs));
  HIPCHK(hipStreamSynchronize(hs));
  if (best_out) *best_out = h[0];
  if (mean_out) *mean_out = h[1];
  return AAQ_OK;
}

}  // namespace

aaq_status aaq::validate_call(const aaq_problem* prob, int p, const double* gamma, const double* beta) {
  aaq_status st = validate_problem(prob);
  if (st) return st;
  if ((st = validate_p(p))) return st;
  return validate_params(p, gamma, beta);
}

aaq_status aaq::energy_grad_pageable(const aaq_problem* prob, int p, const double* gamma, const double* beta,
                                     aaq_observable obs, aaq_precision prec, void* d_state, size_t state_bytes,
                                     void* d_lambda, size_t lambda_bytes, void* d_ws, size_t ws_bytes, void* stream,
                                     double* energy_out, double* dgamma_out, double* dbeta_out, double* norm_out) {
  if (!energy_out || !dgamma_out || !dbeta_out) return fail(AAQ_ERR_INVALID_ARG, "output pointer is NULL");
  std::vector<double> res;
  aaq_status s = run_single(prob, p, gamma, beta, obs, AAQ_AGG_FUSED, prec, true, d_state, state_bytes, d_lambda,
                            lambda_bytes, d_ws, ws_bytes, stream, res, 0, false, false, nullptr, true);
  if (s) return s;
  *energy_out = res[0];
  if (norm_out) *norm_out = res[1];
  for (int l = 0; l < p; ++l) {
    dgamma_out[l] = res[2 + l];
    dbeta_out[l] = res[2 + p + l];
  }
  return AAQ_OK;
}


// ====================================================================== plans
struct aaq_plan {
  int count = 0, p = 0;
  bool grad = false, dbl = false;
  aaq_plan_opts opts;
  unsigned char* ws = nullptr;
  size_t ws_bytes = 0;
  size_t units_off = 0, progs_off = 0, counter_off = 0;
  int tabmax = 1;
  // units whose state fits one tile: one persistent launch per tile size
  struct Small {
    int L;
    size_t order_off;  // device int32 list of unit indices, largest n first
    int count, blocks, counter;
  };
  std::vector<Small> small;
  // larger units: batched sweeps, one group per (tile size, tile-set count)
  struct Group {
    int L;
    size_t list_off;   // device int32 list of unit indices
    size_t wgmap_off;  // device int2 (unit, tile) of each workgroup of the group's sweep steps
    int nlist, max_tiles, nsweep, wg_count;
    std::vector<SweepProg> progs;  // the group's common program (for launch shapes)
    std::vector<uint8_t> routes;   // route of the set of each step
    bool weighted = false;         // some unit has edge weights (run-time sweep path)
  };
  std::vector<Group> groups;
  // the small-unit launches (one per tile size) run on streams of their own, forked from
  // and joined to the caller's stream, when more than one launch sequence exists
  static constexpr int kMaxAux = 3;
  hipStream_t aux[kMaxAux] = {};
  hipEvent_t ev_fork = nullptr, ev_join[kMaxAux] = {};
  int naux = 0;
  // captured graph
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
  const double* g_params = nullptr;
  double* g_out = nullptr;
  hipStream_t g_stream = nullptr;
};

namespace {

constexpr int kUnitTiles[3] = {10, 12, 13};  // tile sizes of the persistent unit kernel
constexpr int kMaxUnitTile = 13;
constexpr int kNumCounters = 4;

struct PlanLayout {
  size_t units = 0, progs = 0, order = 0, counter = 0, lists = 0, graphs = 0, wgmap = 0, total = 0;
  std::vector<UnitDesc> ud;
  std::vector<SweepProg> progs_v;
  std::vector<std::pair<int, std::vector<int32_t>>> small;        // (tile bits, units)
  std::vector<std::pair<int, std::vector<int32_t>>> group_units;  // (tile bits, units of one tile-set count)
  std::vector<unsigned char> blob;  // graphs + terms (uploaded), offsets relative to `graphs`
};

// tile size of a unit under the plan options
int unit_tile_bits(int n, const aaq_plan_opts& o) {
  const int max_small = o.max_small_n > 0 ? o.max_small_n : kMaxUnitTile;
  if (n > max_small && n <= kMaxUnitTile) return 12;  // more than one 12-bit tile: batched sweep steps
  if (n <= kMaxUnitTile) {
    const int lo = std::max(n, o.min_tile_bits_small > 0 ? o.min_tile_bits_small : kUnitTiles[0]);
    for (int L : kUnitTiles)
      if (L >= lo) return L;
    return kMaxUnitTile;
  }
  return o.tile_bits_large > 0 ? o.tile_bits_large : auto_tile_bits(n);
}

aaq_status check_opts(const aaq_plan_opts& o) {
  if (o.prec != AAQ_PREC_C64 && o.prec != AAQ_PREC_C128) return fail(AAQ_ERR_INVALID_ARG, "bad precision");
  if (o.tile_bits_large != 0 && !sweep_tile_ok(o.tile_bits_large))
    return fail(AAQ_ERR_INVALID_ARG, "tile_bits_large must be 0, 12 or 13");
  if (o.min_tile_bits_small < 0 || o.min_tile_bits_small > kMaxUnitTile)
    return fail(AAQ_ERR_INVALID_ARG, "min_tile_bits_small must be in 0..13");
  if (o.workgroups < 0) return fail(AAQ_ERR_INVALID_ARG, "workgroups must be >= 0");
  if (o.single_launch != 0 && o.single_launch != 1) return fail(AAQ_ERR_INVALID_ARG, "single_launch must be 0 or 1");
  if (o.small_streams != 0 && o.small_streams != 1) return fail(AAQ_ERR_INVALID_ARG, "small_streams must be 0 or 1");
  if (o.max_small_n != 0 && o.max_small_n != 12 && o.max_small_n != 13)
    return fail(AAQ_ERR_INVALID_ARG, "max_small_n must be 0, 12 or 13");
  return AAQ_OK;
}

// unit_terms: when given, unit i observes the weighted term list unit_terms[i] (vertex
// pairs of its own graph) instead of the problem's H_C / H_red terms; its problem then
// carries no orbit list (internal units of the light-cone evaluation).
aaq_status plan_layout(const aaq_problem* probs, int count, int p, aaq_observable obs, bool grad, const aaq_plan_opts& o,
                       PlanLayout& PL, const std::vector<std::vector<int4>>* unit_terms = nullptr) {
  if (!probs || count < 1) return fail(AAQ_ERR_INVALID_ARG, "probs is NULL or count < 1");
  aaq_status st = validate_p(p);
  if (st) return st;
  if ((st = check_opts(o))) return st;
  if (obs != AAQ_OBS_HC && obs != AAQ_OBS_HRED) return fail(AAQ_ERR_INVALID_ARG, "bad observable");
  const bool dbl = o.prec == AAQ_PREC_C128;
  const size_t amp = dbl ? 16 : 8;
  if (!unit_terms) {
    for (int i = 0; i < count; ++i) {
      if ((st = validate_problem(&probs[i]))) {
        g_err = "unit " + std::to_string(i) + ": " + g_err;
        return st;
      }
    }
  }
  // shared graph blocks: identical instance arrays (at the same tile size) are stored once
  struct GraphEntry {
    int64_t goff, toff;
    std::vector<SetSpec> sets;
    bool half;  // the unit sweeps the half state (its last set's mirrored registers marked)
  };
  std::map<std::tuple<const int32_t*, int, int, const int32_t*, const int32_t*, const int32_t*, int>, GraphEntry> gmap;
  // 13-qubit units join the batched sweep steps (two 12-bit tiles) when the plan runs such
  // steps for larger units anyway, unless the options say otherwise
  aaq_plan_opts oe = o;
  if (oe.max_small_n == 0) {
    bool any_large = false;
    for (int i = 0; i < count; ++i) any_large = any_large || probs[i].n > kMaxUnitTile;
    oe.max_small_n = (any_large && !o.single_launch) ? 12 : kMaxUnitTile;
  }
  PL.ud.assign(count, UnitDesc{});
  PL.blob.clear();
  std::vector<std::vector<SweepProg>> progs(count);
  for (int i = 0; i < count; ++i) {
    const aaq_problem* pr = &probs[i];
    UnitDesc& D = PL.ud[i];
    std::memset(&D, 0, sizeof(D));
    D.n = pr->n;
    D.p = p;
    D.row = i;
    D.T = unit_terms ? (int)(*unit_terms)[i].size() : (obs == AAQ_OBS_HC) ? pr->num_edges : pr->num_orbits;
    D.cmax = total_weight(pr);
    D.L = unit_tile_bits(pr->n, oe);
    auto key = std::make_tuple(pr->edges, pr->n, pr->num_edges, pr->orbit_rep, pr->orbit_size, pr->edge_weight, (int)D.L);
    auto it = unit_terms ? gmap.end() : gmap.find(key);
    if (it == gmap.end()) {
      GraphDev g = make_graph(pr);
      g.T = D.T;
      g.h_is_cut = !unit_terms && obs == AAQ_OBS_HC && !g.weighted;
      std::vector<SetSpec> sets = make_sets(pr->n, D.L);
      std::vector<int4> t;
      if (!unit_terms) {
        t = term_array(pr, obs, D.L, sets);
      } else {
        const std::vector<int4> cost = make_terms(pr, AAQ_OBS_HC);
        t = term_array_of((*unit_terms)[i], D.L, sets, g.weighted ? &cost : nullptr);
      }
      int64_t goff = (int64_t)PL.blob.size();
      PL.blob.resize(align_up(PL.blob.size() + sizeof(GraphDev)));
      std::memcpy(PL.blob.data() + goff, &g, sizeof(g));
      int64_t toff = (int64_t)PL.blob.size();
      PL.blob.resize(align_up(PL.blob.size() + sizeof(int4) * std::max<size_t>(t.size(), 1)));
      if (!t.empty()) std::memcpy(PL.blob.data() + toff, t.data(), sizeof(int4) * t.size());
      if (unit_terms) std::get<0>(key) = (const int32_t*)(intptr_t)(-1 - i);  // never shared
      // units swept as batched steps store and sweep the half state when their sets allow
      const bool half = pr->n > D.L && !o.single_launch && sets_half_ok(sets, pr->n, D.L, dbl);
      if (half) mark_mirror(sets, pr->n, D.L);
      it = gmap.emplace(key, GraphEntry{goff, toff, sets, half}).first;
    }
    D.graph_off = it->second.goff;  // relative to the graph area; fixed up below
    D.terms_off = it->second.toff;
    const std::vector<SetSpec>& sets = it->second.sets;
    D.half = it->second.half ? 1 : 0;
    D.nsets = (int)sets.size();
    for (int s = 0; s < D.nsets; ++s) D.sets[s] = sets[s];
    // units swept as batched steps keep their forward states (checkpoints, at most
    // kMaxCkpt of them): the backward steps then read psi and store lambda alone
    const bool ckpt = grad && D.n > D.L && !o.single_launch && p * (D.nsets - 1) <= kMaxCkpt;
    progs[i] = build_progs(D.nsets, p, grad, OP_ENERGY, false, ckpt);
    D.nsweep = (int)progs[i].size();
  }
  // offsets
  size_t off = 0;
  PL.units = off;
  off = align_up(off + sizeof(UnitDesc) * count);
  PL.progs_v.clear();
  for (int i = 0; i < count; ++i) {
    PL.ud[i].prog_off = (int32_t)PL.progs_v.size();
    PL.progs_v.insert(PL.progs_v.end(), progs[i].begin(), progs[i].end());
  }
  PL.progs = off;
  off = align_up(off + sizeof(SweepProg) * PL.progs_v.size());
  PL.order = off;
  off = align_up(off + sizeof(int32_t) * count);
  PL.counter = off;
  off = align_up(off + sizeof(int32_t) * kNumCounters);
  PL.lists = off;
  off = align_up(off + sizeof(int32_t) * count);
  // the batched sweeps' workgroup map: (unit, tile) of every tile of every unit that runs
  // as batched sweep steps (n above its tile size, not in the single-launch mode)
  PL.wgmap = off;
  size_t big_tiles = 0;
  for (int i = 0; i < count; ++i)
    if (PL.ud[i].n > PL.ud[i].L && !o.single_launch)
      big_tiles += ((size_t)1 << (PL.ud[i].n - PL.ud[i].L)) >> PL.ud[i].half;
  off = align_up(off + sizeof(int2) * big_tiles);
  PL.graphs = off;
  off = align_up(off + PL.blob.size());
  for (int i = 0; i < count; ++i) {
    PL.ud[i].graph_off += (int64_t)PL.graphs;
    PL.ud[i].terms_off += (int64_t)PL.graphs;
  }
  for (int i = 0; i < count; ++i) {
    UnitDesc& D = PL.ud[i];
    D.tab_off = (int64_t)off;
    off = align_up(off + amp * (size_t)p * (D.cmax + 1) + sizeof(SwScale) * (D.nsweep + 1));
  }
  std::map<std::pair<int, int>, std::vector<int32_t>> by_group;  // (tile bits, sets)
  std::map<int, std::vector<int32_t>> by_small;                  // tile bits
  for (int i = 0; i < count; ++i) {
    UnitDesc& D = PL.ud[i];
    if (D.n > D.L) {
      const size_t sbytes = amp * ((size_t)1 << (D.n - D.half));  // the stored amplitudes
      const int nb = prog_buffers(progs[i]);
      D.state_off = (int64_t)off;
      D.lam_off = grad ? (int64_t)(off + sbytes * nb) : -1;
      off = align_up(off + sbytes * (nb + (grad ? 1 : 0)));
      D.ntiles = (int32_t)((1u << (D.n - D.L)) >> D.half);  // tiles swept per step
      D.part_off = (int64_t)off;
      off = align_up(off + sizeof(double) * 6 * (size_t)D.nsweep * D.ntiles);
      if (o.single_launch)  // swept tile by tile by one workgroup of the persistent kernel
        by_small[D.L].push_back(i);
      else
        by_group[std::make_pair((int)D.L, D.nsets)].push_back(i);
    } else {
      D.state_off = -1;
      D.lam_off = -1;
      D.ntiles = 1;
      D.part_off = -1;
      by_small[D.L].push_back(i);
    }
  }
  PL.total = off;
  PL.small.clear();
  for (auto& kv : by_small) {
    std::vector<int32_t> v = kv.second;
    if (o.sort_units) std::stable_sort(v.begin(), v.end(), [&](int a, int b) { return PL.ud[a].n > PL.ud[b].n; });
    PL.small.emplace_back(kv.first, v);
  }
  PL.group_units.clear();
  for (auto& kv : by_group) PL.group_units.emplace_back(kv.first.first, kv.second);
  return AAQ_OK;
}

aaq_status plan_create_impl(const aaq_problem* probs, int count, int p, aaq_observable obs, int with_grad,
                            const aaq_plan_opts* opts, void* d_ws, size_t ws_bytes, void* stream, aaq_plan** out,
                            const std::vector<std::vector<int4>>* unit_terms);

aaq_status plan_launch(aaq_plan* P, const double* d_params, double* d_out, hipStream_t hs) {
  LaunchUnits U;
  U.units = (const UnitDesc*)(P->ws + P->units_off);
  U.progs = (const SweepProg*)(P->ws + P->progs_off);
  U.order = nullptr;
  U.ws = P->ws;
  U.params = d_params;
  U.out = d_out;
  U.counter = (int32_t*)(P->ws + P->counter_off);
  U.count = P->count;
  U.out_stride = 2 + 2 * P->p;
  U.tabmax = P->tabmax;
  U.psi_io = nullptr;
  {
    TimedLaunch tl(KC_TABLES, 0.0, hs);
    HIPCHK(launch_plan_tables(U, P->p, P->dbl, hs));  // every unit; also resets the counters
    tl.done();
  }
  // the persistent small-unit kernels (one per tile size, each with its own work counter)
  // and the chain of batched sweep steps touch disjoint units: the small-unit launches run
  // on one auxiliary stream beside the chain, or with small_streams each on its own
  const bool fork = P->naux > 0;
  if (fork) {
    HIPCHK(hipEventRecord(P->ev_fork, hs));
    for (int i = 0; i < P->naux; ++i) HIPCHK(hipStreamWaitEvent(P->aux[i], P->ev_fork, 0));
  }
  for (size_t i = 0; i < P->small.size(); ++i) {
    const auto& sc = P->small[i];
    const int ai = std::min((int)i, P->naux - 1);
    hipStream_t su = fork ? P->aux[ai] : hs;
    LaunchUnits V = U;
    V.order = (const int32_t*)(P->ws + sc.order_off);
    V.counter = (int32_t*)(P->ws + P->counter_off) + sc.counter;
    V.count = sc.count;
    TimedLaunch tl(KC_UNITS, 0.0, su);
    HIPCHK(launch_units(V, P->grad, P->dbl, sc.L, sc.blocks, su));
    tl.done();
  }
  if (fork)
    for (int i = 0; i < P->naux; ++i) HIPCHK(hipEventRecord(P->ev_join[i], P->aux[i]));
  for (const auto& Gp : P->groups) {
    LaunchBatch B;
    B.units = U.units;
    B.progs = U.progs;
    B.list = (const int32_t*)(P->ws + Gp.list_off);
    B.wgmap = (const int2*)(P->ws + Gp.wgmap_off);
    B.wg_count = Gp.wg_count;
    B.ws = P->ws;
    B.nlist = Gp.nlist;
    B.max_tiles = Gp.max_tiles;
    B.tabmax = P->tabmax;
    for (int s = 0; s < Gp.nsweep; ++s) {
      const SweepProg& pg = Gp.progs[s];
      B.step = s;
      B.route = Gp.routes[s];
      B.two_states = P->grad && needs_two_states(pg);
      B.energy = ((pg.pre_ops | pg.mid_ops) & OP_ENERGY) != 0;
      // the specialised shapes for unweighted groups (weighted costs take the run-time path)
      B.kind = Gp.weighted ? SK_GENERIC : sweep_kind(pg);
      TimedLaunch tl(B.two_states ? KC_SWEEP2 : KC_SWEEP1, 0.0, hs);
      HIPCHK(launch_bsweep(B, P->dbl, Gp.L, hs));
      tl.done();
    }
    TimedLaunch tl(KC_REDUCE, 0.0, hs);
    HIPCHK(launch_bsweep_out(B, d_out, 2 + 2 * P->p, P->grad, P->dbl, hs));
    tl.done();
  }
  if (fork)
    for (int i = 0; i < P->naux; ++i) HIPCHK(hipStreamWaitEvent(hs, P->ev_join[i], 0));
  return AAQ_OK;
}

}  // namespace

// ====================================================================== C ABI
extern "C" {

const char* aaq_status_string(aaq_status s) {
  switch (s) {
    case AAQ_OK: return "ok";
    case AAQ_ERR_INVALID_ARG: return "invalid argument";
    case AAQ_ERR_GRAPH: return "invalid graph";
    case AAQ_ERR_ORBITS: return "invalid edge orbits";
    case AAQ_ERR_PARAMS: return "invalid parameters";
    case AAQ_ERR_BUFFER: return "buffer too small";
    case AAQ_ERR_UNSUPPORTED: return "unsupported";
    case AAQ_ERR_HIP: return "HIP error";
  }
  return "unknown status";
}

const char* aaq_last_error_message(void) { return g_err.c_str(); }

const char* aaq_version(void) { return "aaqaoa 0.1 gfx950"; }

aaq_status aaq_validate(const aaq_problem* prob, int p) {
  aaq_status s = validate_problem(prob);
  if (s) return s;
  return validate_p(p);
}

aaq_status aaq_state_bytes(const aaq_problem* prob, aaq_precision prec, size_t* bytes) {
  aaq_status s = validate_problem(prob);
  if (s) return s;
  if (!bytes) return fail(AAQ_ERR_INVALID_ARG, "bytes is NULL");
  if (prec != AAQ_PREC_C64 && prec != AAQ_PREC_C128) return fail(AAQ_ERR_INVALID_ARG, "bad precision");
  *bytes = ((size_t)1 << prob->n) * (prec == AAQ_PREC_C128 ? 16 : 8);
  return AAQ_OK;
}

aaq_status aaq_workspace_size(const aaq_problem* prob, int p, int with_grad, aaq_observable obs, aaq_aggregation agg,
                              aaq_precision prec, size_t* bytes) {
  aaq_status s = validate_problem(prob);
  if (s) return s;
  if ((s = validate_p(p))) return s;
  if (!bytes) return fail(AAQ_ERR_INVALID_ARG, "bytes is NULL");
  size_t mx = 0;
  for (int tile : {12, 13})  // any tile choice and either state mode fits
    for (bool half : {true, false}) {
      Single S;
      if ((s = plan_single(prob, p, with_grad != 0, obs, agg, prec, tile, S, false, false, false, half))) return s;
      mx = std::max(mx, S.lay.total);
    }
  *bytes = mx;
  return AAQ_OK;
}

aaq_status aaq_energy(const aaq_problem* prob, int p, const double* gamma, const double* beta, aaq_observable obs,
                      aaq_aggregation agg, aaq_precision prec, void* d_state, size_t state_bytes, void* d_ws,
                      size_t ws_bytes, void* stream, double* energy_out, double* zz_out, double* norm_out) {
  if (!energy_out) return fail(AAQ_ERR_INVALID_ARG, "energy_out is NULL");
  std::vector<double> res;
  aaq_status s = run_single(prob, p, gamma, beta, obs, agg, prec, false, d_state, state_bytes, nullptr, 0, d_ws, ws_bytes,
                            stream, res);
  if (s) return s;
  *energy_out = res[0];
  if (norm_out) *norm_out = res[1];
  if (zz_out && agg != AAQ_AGG_FUSED) {
    const int T = (obs == AAQ_OBS_HC) ? prob->num_edges : prob->num_orbits;
    for (int t = 0; t < T; ++t) zz_out[t] = res[2 + 2 * p + t];
  }
  return AAQ_OK;
}

aaq_status aaq_energy_grad(const aaq_problem* prob, int p, const double* gamma, const double* beta, aaq_observable obs,
                           aaq_precision prec, void* d_state, size_t state_bytes, void* d_lambda, size_t lambda_bytes,
                           void* d_ws, size_t ws_bytes, void* stream, double* energy_out, double* dgamma_out,
                           double* dbeta_out, double* norm_out) {
  if (!energy_out || !dgamma_out || !dbeta_out) return fail(AAQ_ERR_INVALID_ARG, "output pointer is NULL");
  std::vector<double> res;
  aaq_status s = run_single(prob, p, gamma, beta, obs, AAQ_AGG_FUSED, prec, true, d_state, state_bytes, d_lambda,
                            lambda_bytes, d_ws, ws_bytes, stream, res);
  if (s) return s;
  *energy_out = res[0];
  if (norm_out) *norm_out = res[1];
  for (int l = 0; l < p; ++l) {
    dgamma_out[l] = res[2 + l];
    dbeta_out[l] = res[2 + p + l];
  }
  return AAQ_OK;
}

aaq_status aaq_checkpoint_bytes(const aaq_problem* prob, int p, aaq_precision prec, size_t* bytes) {
  aaq_status s = validate_problem(prob);
  if (s) return s;
  if ((s = validate_p(p))) return s;
  if (!bytes) return fail(AAQ_ERR_INVALID_ARG, "bytes is NULL");
  size_t mx = 0;
  for (int tile : {12, 13}) {  // any tile choice fits
    Single S;
    if ((s = plan_single(prob, p, true, AAQ_OBS_HC, AAQ_AGG_FUSED, prec, tile, S, false, true))) return s;
    mx = std::max(mx, (size_t)S.nbuf * ((size_t)1 << prob->n) * (prec == AAQ_PREC_C128 ? 16 : 8));
  }
  *bytes = mx;
  return AAQ_OK;
}

aaq_status aaq_energy_grad_checkpointed(const aaq_problem* prob, int p, const double* gamma, const double* beta,
                                        aaq_observable obs, aaq_precision prec, void* d_ckpt, size_t ckpt_bytes,
                                        void* d_lambda, size_t lambda_bytes, void* d_ws, size_t ws_bytes, void* stream,
                                        double* energy_out, double* dgamma_out, double* dbeta_out, double* norm_out) {
  if (!energy_out || !dgamma_out || !dbeta_out) return fail(AAQ_ERR_INVALID_ARG, "output pointer is NULL");
  std::vector<double> res;
  aaq_status s = run_single(prob, p, gamma, beta, obs, AAQ_AGG_FUSED, prec, true, d_ckpt, ckpt_bytes, d_lambda,
                            lambda_bytes, d_ws, ws_bytes, stream, res, 0, true);
  if (s) return s;
  *energy_out = res[0];
  if (norm_out) *norm_out = res[1];
  for (int l = 0; l < p; ++l) {
    dgamma_out[l] = res[2 + l];
    dbeta_out[l] = res[2 + p + l];
  }
  return AAQ_OK;
}

// ---------------------------------------------------------------- resident evaluator
}  // extern "C"

struct aaq_resident {
  Single S;
  bool grad = false;
  void* d_state = nullptr;
  void* d_lam = nullptr;
  unsigned char* ws = nullptr;
};

namespace {
aaq_status resident_plan(const aaq_problem* prob, int p, aaq_observable obs, int with_grad, int checkpoint,
                         aaq_precision prec, Single& S) {
  aaq_status s = validate_problem(prob);
  if (s) return s;
  if ((s = validate_p(p))) return s;
  const bool grad = with_grad != 0;
  const int tile = chosen_tile_bits(prob->n, prec == AAQ_PREC_C128, grad);
  return plan_single(prob, p, grad, obs, AAQ_AGG_FUSED, prec, tile, S, true, checkpoint != 0 && grad);
}
}  // namespace

extern "C" {

aaq_status aaq_resident_workspace_size(const aaq_problem* prob, int p, aaq_observable obs, int with_grad, int checkpoint,
                                       aaq_precision prec, size_t* ws_bytes, size_t* state_bytes) {
  if (!ws_bytes || !state_bytes) return fail(AAQ_ERR_INVALID_ARG, "ws_bytes / state_bytes is NULL");
  Single S;
  aaq_status s = resident_plan(prob, p, obs, with_grad, checkpoint, prec, S);
  if (s) return s;
  *ws_bytes = S.lay.total;
  *state_bytes = (size_t)S.nbuf * ((size_t)1 << S.n) * (S.dbl ? 16 : 8);
  return AAQ_OK;
}

aaq_status aaq_resident_create(const aaq_problem* prob, int p, aaq_observable obs, int with_grad, int checkpoint,
                               aaq_precision prec, void* d_state, size_t state_bytes, void* d_lambda,
                               size_t lambda_bytes, void* d_ws, size_t ws_bytes, void* stream, aaq_resident** out) {
  if (!out) return fail(AAQ_ERR_INVALID_ARG, "out is NULL");
  auto R = std::make_unique<aaq_resident>();
  aaq_status s = resident_plan(prob, p, obs, with_grad, checkpoint, prec, R->S);
  if (s) return s;
  R->grad = with_grad != 0;
  if ((s = check_buffers(R->S, R->grad, d_state, state_bytes, d_lambda, lambda_bytes, d_ws, ws_bytes))) return s;
  R->d_state = d_state;
  R->d_lam = R->grad ? d_lambda : nullptr;
  R->ws = (unsigned char*)d_ws;
  // the static block goes up once; the copy completes before the staging area is reused
  const Layout& L = R->S.lay;
  unsigned char* up = pinned_staging(L.upload_end);
  if (!up) return fail(AAQ_ERR_HIP, "hipHostMalloc of the staging buffer failed");
  stage_static(R->S, prob, obs, up);
  hipStream_t hs = (hipStream_t)stream;
  HIPCHK(hipMemcpyAsync(R->ws, up, L.upload_end, hipMemcpyHostToDevice, hs));
  HIPCHK(hipStreamSynchronize(hs));
  *out = R.release();
  return AAQ_OK;
}

aaq_status aaq_resident_execute(aaq_resident* r, const double* d_params, double* d_out, void* stream) {
  if (!r) return fail(AAQ_ERR_INVALID_ARG, "evaluator is NULL");
  if (!d_params || !d_out) return fail(AAQ_ERR_INVALID_ARG, "d_params / d_out is NULL");
  return launch_eval(r->S, r->grad, r->d_state, r->d_lam, r->ws, d_params, d_params + r->S.p, d_out,
                     (hipStream_t)stream);
}

void aaq_resident_destroy(aaq_resident* r) { delete r; }

void aaq_set_half_state(int enable) { g_half_state = enable != 0; }
int aaq_get_half_state(void) { return g_half_state ? 1 : 0; }

aaq_status aaq_sample_workspace_size(const aaq_problem* prob, int p, aaq_precision prec, size_t* bytes) {
  aaq_status s = validate_problem(prob);
  if (s) return s;
  if ((s = validate_p(p))) return s;
  if (!bytes) return fail(AAQ_ERR_INVALID_ARG, "bytes is NULL");
  size_t mx = 0;
  for (int tile : {12, 13}) {
    Single S;
    if ((s = plan_single(prob, p, false, AAQ_OBS_HC, AAQ_AGG_FUSED, prec, tile, S, false, false, true))) return s;
    mx = std::max(mx, S.lay.total);
  }
  *bytes = mx + sample_extra_bytes(prob->n);
  return AAQ_OK;
}

aaq_status aaq_sample(const aaq_problem* prob, int p, const double* gamma, const double* beta, aaq_precision prec,
                      int num_shots, const double* d_uniform, void* d_state, size_t state_bytes, void* d_ws,
                      size_t ws_bytes, void* stream, uint64_t* d_samples, int32_t* d_cuts, double* best_cut_out,
                      double* mean_cut_out) {
  return run_sample(prob, p, gamma, beta, prec, num_shots, d_uniform, d_state, state_bytes, d_ws, ws_bytes, stream,
                    d_samples, d_cuts, best_cut_out, mean_cut_out);
}

aaq_status aaq_cut_values_layout(const aaq_problem* prob, aaq_observable obs, int set_index, int arrangement,
                                 aaq_precision prec, void* d_ws, size_t ws_bytes, int32_t* d_out, void* stream) {
  aaq_status s = validate_problem(prob);
  if (s) return s;
  if (!d_out || !d_ws) return fail(AAQ_ERR_INVALID_ARG, "d_out / d_ws is NULL");
  if (obs != AAQ_OBS_HC && obs != AAQ_OBS_HRED) return fail(AAQ_ERR_INVALID_ARG, "bad observable");
  if (prec != AAQ_PREC_C64 && prec != AAQ_PREC_C128) return fail(AAQ_ERR_INVALID_ARG, "bad precision");
  const bool dbl = prec == AAQ_PREC_C128;
  const int tile = auto_tile_bits(prob->n);
  std::vector<SetSpec> sets = make_sets(prob->n, tile);
  if (set_index < 0 || set_index >= (int)sets.size()) return fail(AAQ_ERR_INVALID_ARG, "set_index out of range");
  if (arrangement != 0 && arrangement != 1) return fail(AAQ_ERR_INVALID_ARG, "arrangement must be 0 or 1");
  const int T = (obs == AAQ_OBS_HC) ? prob->num_edges : prob->num_orbits;
  std::vector<int4> terms = term_array(prob, obs, tile, sets);
  const size_t need = align_up(sizeof(GraphDev)) + sizeof(int4) * std::max<size_t>(terms.size(), 1);
  if (ws_bytes < need) return fail(AAQ_ERR_BUFFER, "workspace too small for the graph block and term lists");
  std::vector<unsigned char> up(need, 0);
  GraphDev g = make_graph(prob);
  g.T = T;
  g.h_is_cut = obs == AAQ_OBS_HC && !g.weighted;
  std::memcpy(up.data(), &g, sizeof(g));
  if (!terms.empty()) std::memcpy(up.data() + align_up(sizeof(GraphDev)), terms.data(), sizeof(int4) * terms.size());
  hipStream_t hs = (hipStream_t)stream;
  unsigned char* ws = (unsigned char*)d_ws;
  HIPCHK(hipMemcpyAsync(ws, up.data(), need, hipMemcpyHostToDevice, hs));
  HIPCHK(launch_cuts((const GraphDev*)ws, (const int4*)(ws + align_up(sizeof(GraphDev))), T, g.h_is_cut ? 0 : 1,
                     sets[set_index], arrangement, d_out, dbl, tile, hs));
  HIPCHK(hipStreamSynchronize(hs));
  return AAQ_OK;
}

aaq_status aaq_cut_values(const aaq_problem* prob, aaq_observable obs, void* d_ws, size_t ws_bytes, int32_t* d_out,
                          void* stream) {
  return aaq_cut_values_layout(prob, obs, 0, 0, AAQ_PREC_C64, d_ws, ws_bytes, d_out, stream);
}

int aaq_num_sets(int n, aaq_precision prec) {
  if (n < 1 || n > AAQ_MAX_N) return 0;
  (void)prec;
  return sets_for(n, auto_tile_bits(n));
}

void aaq_plan_default_opts(aaq_plan_opts* o) {
  if (!o) return;
  o->use_graph = 1;
  o->workgroups = 0;
  o->sort_units = 1;
  o->prec = AAQ_PREC_C64;
  o->tile_bits_large = 0;
  o->min_tile_bits_small = 0;
  o->single_launch = 0;
  o->small_streams = 0;
  o->max_small_n = 0;
}

aaq_status aaq_plan_workspace_size(const aaq_problem* probs, int count, int p, aaq_observable obs, int with_grad,
                                   const aaq_plan_opts* opts, size_t* bytes) {
  if (!bytes) return fail(AAQ_ERR_INVALID_ARG, "bytes is NULL");
  aaq_plan_opts o;
  aaq_plan_default_opts(&o);
  if (opts) o = *opts;
  PlanLayout PL;
  aaq_status s = plan_layout(probs, count, p, obs, with_grad != 0, o, PL);
  if (s) return s;
  *bytes = PL.total;
  return AAQ_OK;
}

aaq_status aaq_plan_create(const aaq_problem* probs, int count, int p, aaq_observable obs, int with_grad,
                           const aaq_plan_opts* opts, void* d_ws, size_t ws_bytes, void* stream, aaq_plan** out) {
  return plan_create_impl(probs, count, p, obs, with_grad, opts, d_ws, ws_bytes, stream, out, nullptr);
}

}  // extern "C"

namespace {
aaq_status plan_create_impl(const aaq_problem* probs, int count, int p, aaq_observable obs, int with_grad,
                            const aaq_plan_opts* opts, void* d_ws, size_t ws_bytes, void* stream, aaq_plan** out,
                            const std::vector<std::vector<int4>>* unit_terms) {
  if (!out) return fail(AAQ_ERR_INVALID_ARG, "out is NULL");
  aaq_plan_opts o;
  aaq_plan_default_opts(&o);
  if (opts) o = *opts;
  PlanLayout PL;
  aaq_status s = plan_layout(probs, count, p, obs, with_grad != 0, o, PL, unit_terms);
  if (s) return s;
  if (!d_ws) return fail(AAQ_ERR_INVALID_ARG, "workspace is NULL");
  if (ws_bytes < PL.total) return fail(AAQ_ERR_BUFFER, "workspace too small (need " + std::to_string(PL.total) + " bytes)");
  hipStream_t hs = (hipStream_t)stream;
  unsigned char* ws = (unsigned char*)d_ws;
  std::vector<unsigned char> up(PL.graphs + PL.blob.size(), 0);
  std::memcpy(up.data() + PL.units, PL.ud.data(), sizeof(UnitDesc) * count);
  if (!PL.progs_v.empty()) std::memcpy(up.data() + PL.progs, PL.progs_v.data(), sizeof(SweepProg) * PL.progs_v.size());
  aaq_plan* P = new aaq_plan();
  {
    size_t so = PL.order;
    int ci = 0;
    for (auto& sm : PL.small) {
      std::memcpy(up.data() + so, sm.second.data(), sizeof(int32_t) * sm.second.size());
      aaq_plan::Small c;
      c.L = sm.first;
      c.order_off = so;
      c.count = (int)sm.second.size();
      c.counter = ci++;
      const int auto_blocks = 2 * device_cus() * (1 << (kMaxUnitTile - c.L));
      c.blocks = std::min(c.count, o.workgroups > 0 ? o.workgroups : auto_blocks);
      P->small.push_back(c);
      so += sizeof(int32_t) * sm.second.size();
    }
    size_t lo = PL.lists, wo = PL.wgmap;
    for (auto& gl : PL.group_units) {
      const std::vector<int32_t>& units = gl.second;
      std::memcpy(up.data() + lo, units.data(), sizeof(int32_t) * units.size());
      aaq_plan::Group Gp;
      Gp.L = gl.first;
      Gp.list_off = lo;
      lo += sizeof(int32_t) * units.size();
      Gp.nlist = (int)units.size();
      Gp.max_tiles = 0;
      for (int u : units) Gp.max_tiles = std::max(Gp.max_tiles, (int)PL.ud[u].ntiles);
      // one workgroup per tile of the group's units, no idle ones for the smaller units
      Gp.wgmap_off = wo;
      Gp.wg_count = 0;
      for (int u : units) {
        int2* m = reinterpret_cast<int2*>(up.data() + wo) + Gp.wg_count;
        for (int t = 0; t < PL.ud[u].ntiles; ++t) m[t] = make_int2(u, t);
        Gp.wg_count += PL.ud[u].ntiles;
      }
      wo += sizeof(int2) * (size_t)Gp.wg_count;
      const UnitDesc& D0 = PL.ud[units[0]];
      Gp.nsweep = D0.nsweep;
      Gp.progs.assign(PL.progs_v.begin() + D0.prog_off, PL.progs_v.begin() + D0.prog_off + D0.nsweep);
      for (const SweepProg& pg : Gp.progs) Gp.routes.push_back(D0.sets[pg.set].route);
      for (int u : units) Gp.weighted = Gp.weighted || is_weighted(&probs[u]);
      P->groups.push_back(Gp);
    }
  }
  if (!PL.blob.empty()) std::memcpy(up.data() + PL.graphs, PL.blob.data(), PL.blob.size());
  hipError_t e = hipMemcpyAsync(ws, up.data(), up.size(), hipMemcpyHostToDevice, hs);
  if (e == hipSuccess) e = hipStreamSynchronize(hs);
  if (e != hipSuccess) {
    delete P;
    return fail(AAQ_ERR_HIP, std::string("plan upload: ") + hipGetErrorString(e));
  }
  P->count = count;
  P->p = p;
  P->grad = with_grad != 0;
  P->dbl = o.prec == AAQ_PREC_C128;
  P->opts = o;
  P->ws = ws;
  P->ws_bytes = ws_bytes;
  P->units_off = PL.units;
  P->progs_off = PL.progs;
  P->counter_off = PL.counter;
  for (int i = 0; i < count; ++i) P->tabmax = std::max(P->tabmax, PL.ud[i].cmax + 1);
  // fork / join of the small-unit launches (default-priority streams): one auxiliary
  // stream beside the chain of batched sweep steps, or with small_streams one per launch
  const int nsmall = (int)P->small.size();
  const bool chain = !P->groups.empty();
  if (o.small_streams && nsmall + (chain ? 1 : 0) >= 2 && nsmall <= aaq_plan::kMaxAux)
    P->naux = nsmall;
  else if (nsmall > 0 && chain)
    P->naux = 1;
  if (P->naux > 0) {
    e = hipEventCreateWithFlags(&P->ev_fork, hipEventDisableTiming);
    for (int i = 0; i < P->naux && e == hipSuccess; ++i) {
      e = hipStreamCreateWithFlags(&P->aux[i], hipStreamNonBlocking);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&P->ev_join[i], hipEventDisableTiming);
    }
    if (e != hipSuccess) {
      aaq_plan_destroy(P);
      return fail(AAQ_ERR_HIP, std::string("plan stream / events: ") + hipGetErrorString(e));
    }
  }
  *out = P;
  return AAQ_OK;
}
}  // namespace

extern "C" {

aaq_status aaq_plan_execute(aaq_plan* P, const double* d_params, double* d_out, void* stream) {
  if (!P || !d_params || !d_out) return fail(AAQ_ERR_INVALID_ARG, "plan / d_params / d_out is NULL");
  hipStream_t hs = (hipStream_t)stream;
  if (!P->opts.use_graph || hs == nullptr) return plan_launch(P, d_params, d_out, hs);
  if (!P->exec || P->g_params != d_params || P->g_out != d_out || P->g_stream != hs) {
    if (P->exec) {
      (void)hipGraphExecDestroy(P->exec);
      P->exec = nullptr;
    }
    if (P->graph) {
      (void)hipGraphDestroy(P->graph);
      P->graph = nullptr;
    }
    HIPCHK(hipStreamBeginCapture(hs, hipStreamCaptureModeThreadLocal));
    aaq_status s = plan_launch(P, d_params, d_out, hs);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(hs, &g);
    if (s) {
      if (g) (void)hipGraphDestroy(g);
      return s;
    }
    if (e != hipSuccess) return fail(AAQ_ERR_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    P->graph = g;
    HIPCHK(hipGraphInstantiate(&P->exec, g, nullptr, nullptr, 0));
    P->g_params = d_params;
    P->g_out = d_out;
    P->g_stream = hs;
  }
  HIPCHK(hipGraphLaunch(P->exec, hs));
  return AAQ_OK;
}

// ====================================================================== light cones
}  // extern "C"

// <Z_i Z_j> of the depth-p ansatz depends only on the subgraph induced by the vertices
// within distance p of {i, j}: conjugating Z_i Z_j by the layers from the last one back,
// every cost gate on an edge that does not touch the current support commutes with it,
// so the support grows by one neighbourhood per layer (the paper's reverse causal cone).
// Each observable term (every edge with weight 1 for H_C; one representative per edge
// orbit, weighted by the orbit size, for H_red) is evaluated on its own cone as one unit
// of a batched plan; the energy and gradient are the sums over the units.
struct aaq_lightcone {
  aaq_plan* plan = nullptr;
  int count = 0, p = 0;
  bool grad = false;
  unsigned char* ws = nullptr;
  size_t params_off = 0, rows_off = 0;
  std::vector<std::vector<int32_t>> edges;  // owned edge lists of the units
  std::vector<std::vector<int32_t>> weights;  // owned edge weights of the units (empty: unweighted)
  std::vector<aaq_problem> probs;
  bool use_graph = true;
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
  const double* g_params = nullptr;
  double* g_out = nullptr;
  hipStream_t g_stream = nullptr;
};

namespace {

struct Cones {
  std::vector<int> n;                       // qubits of each unit
  std::vector<std::vector<int32_t>> edges;  // relabelled edge list of each unit
  std::vector<std::vector<int32_t>> weights;  // its edge weights (empty when the instance is unweighted)
  std::vector<std::vector<int4>> terms;     // the unit's single weighted term
};

aaq_status build_cones(const aaq_problem* pr, int p, aaq_observable obs, Cones& C) {
  aaq_status st = validate_problem(pr);
  if (st) return st;
  if ((st = validate_p(p))) return st;
  if (obs != AAQ_OBS_HC && obs != AAQ_OBS_HRED) return fail(AAQ_ERR_INVALID_ARG, "bad observable");
  if (pr->num_edges == 0) return fail(AAQ_ERR_UNSUPPORTED, "a graph without edges has no observable terms");
  const int n = pr->n, m = pr->num_edges;
  std::vector<std::vector<int>> nb(n);
  for (int e = 0; e < m; ++e) {
    nb[pr->edges[2 * e]].push_back(pr->edges[2 * e + 1]);
    nb[pr->edges[2 * e + 1]].push_back(pr->edges[2 * e]);
  }
  for (const int4& t : make_terms(pr, obs)) {
    std::vector<int> dist(n, -1), q{t.x, t.y};
    dist[t.x] = dist[t.y] = 0;
    for (size_t h = 0; h < q.size(); ++h) {  // breadth-first search to depth p
      const int v = q[h];
      if (dist[v] == p) continue;
      for (int w : nb[v])
        if (dist[w] < 0) {
          dist[w] = dist[v] + 1;
          q.push_back(w);
        }
    }
    std::vector<int> idx(n, -1);
    int k = 0;
    for (int v = 0; v < n; ++v)
      if (dist[v] >= 0) idx[v] = k++;
    std::vector<int32_t> es, ws;
    for (int e = 0; e < m; ++e) {
      const int u = idx[pr->edges[2 * e]], v = idx[pr->edges[2 * e + 1]];
      if (u >= 0 && v >= 0) {
        es.push_back(u);
        es.push_back(v);
        if (pr->edge_weight) ws.push_back(pr->edge_weight[e]);
      }
    }
    C.n.push_back(k);
    C.edges.push_back(std::move(es));
    C.weights.push_back(std::move(ws));
    C.terms.push_back({make_int4(idx[t.x], idx[t.y], t.z, 0)});
  }
  return AAQ_OK;
}

std::vector<aaq_problem> cone_problems(const Cones& C) {
  std::vector<aaq_problem> v(C.n.size());
  for (size_t i = 0; i < v.size(); ++i) {
    std::memset(&v[i], 0, sizeof(aaq_problem));
    v[i].n = C.n[i];
    v[i].num_edges = (int32_t)(C.edges[i].size() / 2);
    v[i].edges = C.edges[i].data();
    v[i].edge_weight = C.weights[i].empty() ? nullptr : C.weights[i].data();
  }
  return v;
}

size_t lc_extra_bytes(int count, int p) {
  return align_up(sizeof(double) * (size_t)count * 2 * p) + align_up(sizeof(double) * (size_t)count * (2 + 2 * p));
}

aaq_status lc_launch(aaq_lightcone* LC, const double* d_params, double* d_out, hipStream_t hs) {
  double* uparams = (double*)(LC->ws + LC->params_off);
  double* rows = (double*)(LC->ws + LC->rows_off);
  HIPCHK(launch_lc_bcast(d_params, 2 * LC->p, uparams, LC->count, hs));
  aaq_status st = plan_launch(LC->plan, uparams, rows, hs);
  if (st) return st;
  HIPCHK(launch_lc_sum(rows, LC->count, 2 + 2 * LC->p, d_out, hs));
  return AAQ_OK;
}

}  // namespace

extern "C" {

aaq_status aaq_lightcone_info(const aaq_problem* prob, int p, aaq_observable obs, int* units, int* max_qubits,
                              double* amplitudes) {
  Cones C;
  aaq_status st = build_cones(prob, p, obs, C);
  if (st) return st;
  int mx = 0;
  double amp = 0.0;
  for (int k : C.n) {
    mx = std::max(mx, k);
    amp += std::ldexp(1.0, k);
  }
  if (units) *units = (int)C.n.size();
  if (max_qubits) *max_qubits = mx;
  if (amplitudes) *amplitudes = amp;
  return AAQ_OK;
}

aaq_status aaq_lightcone_workspace_size(const aaq_problem* prob, int p, aaq_observable obs, int with_grad,
                                        const aaq_plan_opts* opts, size_t* bytes) {
  if (!bytes) return fail(AAQ_ERR_INVALID_ARG, "bytes is NULL");
  Cones C;
  aaq_status st = build_cones(prob, p, obs, C);
  if (st) return st;
  aaq_plan_opts o;
  aaq_plan_default_opts(&o);
  if (opts) o = *opts;
  std::vector<aaq_problem> probs = cone_problems(C);
  PlanLayout PL;
  if ((st = plan_layout(probs.data(), (int)probs.size(), p, obs, with_grad != 0, o, PL, &C.terms))) return st;
  *bytes = align_up(PL.total) + lc_extra_bytes((int)probs.size(), p);
  return AAQ_OK;
}

aaq_status aaq_lightcone_create(const aaq_problem* prob, int p, aaq_observable obs, int with_grad,
                                const aaq_plan_opts* opts, void* d_ws, size_t ws_bytes, void* stream,
                                aaq_lightcone** out) {
  if (!out) return fail(AAQ_ERR_INVALID_ARG, "out is NULL");
  if (!d_ws) return fail(AAQ_ERR_INVALID_ARG, "workspace is NULL");
  auto LC = std::make_unique<aaq_lightcone>();
  Cones C;
  aaq_status st = build_cones(prob, p, obs, C);
  if (st) return st;
  aaq_plan_opts o;
  aaq_plan_default_opts(&o);
  if (opts) o = *opts;
  LC->edges = C.edges;  // owned copies: the unit problems point into these
  LC->weights = C.weights;
  LC->probs = cone_problems(C);
  for (size_t i = 0; i < LC->probs.size(); ++i) {
    LC->probs[i].edges = LC->edges[i].data();
    LC->probs[i].edge_weight = LC->weights[i].empty() ? nullptr : LC->weights[i].data();
  }
  LC->count = (int)LC->probs.size();
  LC->p = p;
  LC->grad = with_grad != 0;
  LC->use_graph = o.use_graph != 0;
  PlanLayout PL;
  if ((st = plan_layout(LC->probs.data(), LC->count, p, obs, LC->grad, o, PL, &C.terms))) return st;
  const size_t plan_bytes = align_up(PL.total);
  const size_t need = plan_bytes + lc_extra_bytes(LC->count, p);
  if (ws_bytes < need) return fail(AAQ_ERR_BUFFER, "workspace too small (need " + std::to_string(need) + " bytes)");
  LC->ws = (unsigned char*)d_ws;
  LC->params_off = plan_bytes;
  LC->rows_off = plan_bytes + align_up(sizeof(double) * (size_t)LC->count * 2 * p);
  aaq_plan_opts po = o;
  po.use_graph = 0;  // the light-cone handle captures its own graph around the plan
  if ((st = plan_create_impl(LC->probs.data(), LC->count, p, obs, with_grad, &po, d_ws, plan_bytes, stream, &LC->plan,
                             &C.terms)))
    return st;
  *out = LC.release();
  return AAQ_OK;
}

aaq_status aaq_lightcone_execute(aaq_lightcone* LC, const double* d_params, double* d_out, void* stream) {
  if (!LC || !d_params || !d_out) return fail(AAQ_ERR_INVALID_ARG, "handle / d_params / d_out is NULL");
  hipStream_t hs = (hipStream_t)stream;
  if (!LC->use_graph || hs == nullptr) return lc_launch(LC, d_params, d_out, hs);
  if (!LC->exec || LC->g_params != d_params || LC->g_out != d_out || LC->g_stream != hs) {
    if (LC->exec) {
      (void)hipGraphExecDestroy(LC->exec);
      LC->exec = nullptr;
    }
    if (LC->graph) {
      (void)hipGraphDestroy(LC->graph);
      LC->graph = nullptr;
    }
    HIPCHK(hipStreamBeginCapture(hs, hipStreamCaptureModeThreadLocal));
    aaq_status s = lc_launch(LC, d_params, d_out, hs);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(hs, &g);
    if (s) {
      if (g) (void)hipGraphDestroy(g);
      return s;
    }
    if (e != hipSuccess) return fail(AAQ_ERR_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    LC->graph = g;
    HIPCHK(hipGraphInstantiate(&LC->exec, g, nullptr, nullptr, 0));
    LC->g_params = d_params;
    LC->g_out = d_out;
    LC->g_stream = hs;
  }
  HIPCHK(hipGraphLaunch(LC->exec, hs));
  return AAQ_OK;
}

void aaq_lightcone_destroy(aaq_lightcone* LC) {
  if (!LC) return;
  if (LC->exec) (void)hipGraphExecDestroy(LC->exec);
  if (LC->graph) (void)hipGraphDestroy(LC->graph);
  aaq_plan_destroy(LC->plan);
  delete LC;
}

// ====================================================================== tuning
aaq_status aaq_set_tile_bits(int n, aaq_precision prec, int with_grad, int tile_bits) {
  if (n < 1 || n > AAQ_MAX_N) return fail(AAQ_ERR_INVALID_ARG, "n out of range");
  if (prec != AAQ_PREC_C64 && prec != AAQ_PREC_C128) return fail(AAQ_ERR_INVALID_ARG, "bad precision");
  if (tile_bits != 0 && !sweep_tile_ok(tile_bits)) return fail(AAQ_ERR_INVALID_ARG, "tile_bits must be 0, 12 or 13");
  std::lock_guard<std::mutex> lk(g_tune_mu);
  const auto key = std::make_tuple(n, (int)(prec == AAQ_PREC_C128), (int)(with_grad != 0));
  if (tile_bits == 0)
    g_tune.erase(key);
  else
    g_tune[key] = tile_bits;
  return AAQ_OK;
}

int aaq_get_tile_bits(int n, aaq_precision prec, int with_grad) {
  if (n < 1 || n > AAQ_MAX_N) return 0;
  return chosen_tile_bits(n, prec == AAQ_PREC_C128, with_grad != 0);
}

aaq_status aaq_autotune(const aaq_problem* prob, int p, int with_grad, aaq_observable obs, aaq_precision prec,
                        void* d_state, size_t state_bytes, void* d_lambda, size_t lambda_bytes, void* d_ws,
                        size_t ws_bytes, void* stream, int reps, int* best_tile_bits, double* ms_per_call) {
  aaq_status s = validate_problem(prob);
  if (s) return s;
  if ((s = validate_p(p))) return s;
  if (reps < 1) return fail(AAQ_ERR_INVALID_ARG, "reps must be >= 1");
  std::vector<double> gamma(p), beta(p), res;
  for (int l = 0; l < p; ++l) {
    gamma[l] = 0.4 + 0.1 * l;
    beta[l] = 0.3 - 0.02 * l;
  }
  const bool grad = with_grad != 0;
  const aaq_aggregation agg = AAQ_AGG_FUSED;
  const int cand[2] = {12, 13};
  double best = 0.0;
  int bestL = 0;
  for (int c = 0; c < 2; ++c) {
    const int L = cand[c];
    auto one = [&]() {
      return run_single(prob, p, gamma.data(), beta.data(), obs, agg, prec, grad, d_state, state_bytes, d_lambda,
                        lambda_bytes, d_ws, ws_bytes, stream, res, L);
    };
    if ((s = one())) return s;  // warm-up (and argument checks)
    const auto t0 = std::chrono::steady_clock::now();
    for (int r = 0; r < reps; ++r)
      if ((s = one())) return s;
    const double ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count() / reps;
    if (ms_per_call) ms_per_call[c] = ms;
    if (bestL == 0 || ms < best) {
      best = ms;
      bestL = L;
    }
  }
  if ((s = aaq_set_tile_bits(prob->n, prec, with_grad, bestL))) return s;
  if (best_tile_bits) *best_tile_bits = bestL;
  return AAQ_OK;
}

aaq_status aaq_plan_autotune(const aaq_problem* probs, int count, int p, aaq_observable obs, int with_grad,
                             const aaq_plan_opts* base, void* d_ws, size_t ws_bytes, const double* d_params,
                             double* d_out, void* stream, int reps, aaq_plan_opts* best, double* best_ms) {
  if (!probs || count < 1 || !best) return fail(AAQ_ERR_INVALID_ARG, "probs / best is NULL or count < 1");
  if (!d_ws || !d_params || !d_out) return fail(AAQ_ERR_INVALID_ARG, "d_ws / d_params / d_out is NULL");
  if (reps < 1) return fail(AAQ_ERR_INVALID_ARG, "reps must be >= 1");
  aaq_plan_opts b0;
  aaq_plan_default_opts(&b0);
  if (base) b0 = *base;
  bool any_large = false, any_small = false, any_tiny = false, any_13 = false;
  for (int i = 0; i < count; ++i) {
    if (probs[i].n > kMaxUnitTile) any_large = true;
    else any_small = true;
    if (probs[i].n <= 12) any_tiny = true;
    if (probs[i].n == kMaxUnitTile) any_13 = true;
  }
  std::vector<int> larges = any_large ? std::vector<int>{12, 13} : std::vector<int>{b0.tile_bits_large};
  std::vector<int> smalls = any_tiny ? std::vector<int>{10, 12, 13} : std::vector<int>{b0.min_tile_bits_small};
  std::vector<int> wgs = any_small ? std::vector<int>{0, device_cus(), 4 * device_cus()} : std::vector<int>{b0.workgroups};
  std::vector<int> singles = any_large ? std::vector<int>{0, 1} : std::vector<int>{b0.single_launch};
  std::vector<int> streams = any_small ? std::vector<int>{0, 1} : std::vector<int>{b0.small_streams};
  std::vector<int> maxsmall = (any_13 && any_large) ? std::vector<int>{13, 12} : std::vector<int>{b0.max_small_n};
  hipStream_t hs = (hipStream_t)stream;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIPCHK(hipEventCreate(&e0));
  hipError_t he = hipEventCreate(&e1);
  if (he != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(AAQ_ERR_HIP, std::string("hipEventCreate: ") + hipGetErrorString(he));
  }
  aaq_status st = AAQ_OK;
  double bms = -1.0;
  aaq_plan_opts bo = b0;
  for (int ms : maxsmall)
  for (int ss : streams)
  for (int sl : singles)
  for (int tl : larges)
    for (int ts : smalls)
      for (int wg : wgs) {
        aaq_plan_opts o = b0;
        o.tile_bits_large = tl;
        o.min_tile_bits_small = ts;
        o.workgroups = wg;
        o.single_launch = sl;
        o.small_streams = ss;
        o.max_small_n = ms;
        size_t need = 0;
        if ((st = aaq_plan_workspace_size(probs, count, p, obs, with_grad, &o, &need))) goto done;
        if (need > ws_bytes) continue;  // this candidate does not fit the caller's workspace
        aaq_plan* P = nullptr;
        if ((st = aaq_plan_create(probs, count, p, obs, with_grad, &o, d_ws, ws_bytes, stream, &P))) goto done;
        float ms = 0.0f;
        st = aaq_plan_execute(P, d_params, d_out, stream);  // warm-up (captures the graph)
        if (!st) {
          hipError_t e = hipEventRecord(e0, hs);
          for (int r = 0; r < reps && !st && e == hipSuccess; ++r) st = aaq_plan_execute(P, d_params, d_out, stream);
          if (e == hipSuccess) e = hipEventRecord(e1, hs);
          if (e == hipSuccess) e = hipEventSynchronize(e1);
          if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
          if (!st && e != hipSuccess) st = fail(AAQ_ERR_HIP, std::string("tuning events: ") + hipGetErrorString(e));
        }
        aaq_plan_destroy(P);
        if (st) goto done;
        const double per = ms / reps;
        if (bms < 0.0 || per < bms) {
          bms = per;
          bo = o;
        }
      }
  if (bms < 0.0) st = fail(AAQ_ERR_BUFFER, "no candidate configuration fits the workspace");
done:
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st) return st;
  *best = bo;
  if (best_ms) *best_ms = bms;
  return AAQ_OK;
}

aaq_status aaq_timing_enable(int on) {
  std::lock_guard<std::mutex> lk(g_tmu);
  g_timing = on != 0;
  if (g_timing) {
    while (g_evpool.size() < kEventPool) {
      hipEvent_t e;
      if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) break;
      g_evpool.push_back(e);
    }
  }
  return AAQ_OK;
}

aaq_status aaq_timing_classes(int mask) {
  if (mask < 0 || mask >= (1 << KC_N)) return fail(AAQ_ERR_INVALID_ARG, "timing class mask out of range");
  std::lock_guard<std::mutex> lk(g_tmu);
  g_tclasses = (uint32_t)mask;
  return AAQ_OK;
}

aaq_status aaq_timing_read(aaq_kernel_timing* out, int max, int* count, int reset) {
  if (!count || (max > 0 && !out)) return fail(AAQ_ERR_INVALID_ARG, "NULL output");
  std::lock_guard<std::mutex> lk(g_tmu);
  for (auto& pe : g_pending) {
    float ms = 0.f;
    HIPCHK(hipEventSynchronize(pe.b));
    HIPCHK(hipEventElapsedTime(&ms, pe.a, pe.b));
    g_tot_ms[pe.cls] += ms;
    g_tot_bytes[pe.cls] += pe.bytes;
    g_launches[pe.cls] += 1;
    for (hipEvent_t e : {pe.a, pe.b}) {
      if (g_timing && g_evpool.size() < kEventPool)
        g_evpool.push_back(e);
      else
        (void)hipEventDestroy(e);
    }
  }
  g_pending.clear();
  if (!g_timing) {
    for (hipEvent_t e : g_evpool) (void)hipEventDestroy(e);
    g_evpool.clear();
  }
  int k = 0;
  for (int c = 0; c < KC_N; ++c) {
    if (!g_launches[c]) continue;
    if (k < max) {
      std::snprintf(out[k].name, sizeof(out[k].name), "%s", kc_name[c]);
      out[k].launches = g_launches[c];
      out[k].total_ms = g_tot_ms[c];
      out[k].bytes = g_tot_bytes[c];
    }
    ++k;
  }
  *count = k;
  if (reset)
    for (int c = 0; c < KC_N; ++c) g_tot_ms[c] = g_tot_bytes[c] = 0.0, g_launches[c] = 0;
  return AAQ_OK;
}

void aaq_plan_destroy(aaq_plan* P) {
  if (!P) return;
  if (P->exec) (void)hipGraphExecDestroy(P->exec);
  if (P->graph) (void)hipGraphDestroy(P->graph);
  for (int i = 0; i < aaq_plan::kMaxAux; ++i) {
    if (P->aux[i]) {
      (void)hipStreamSynchronize(P->aux[i]);
      (void)hipStreamDestroy(P->aux[i]);
    }
    if (P->ev_join[i]) (void)hipEventDestroy(P->ev_join[i]);
  }
  if (P->ev_fork) (void)hipEventDestroy(P->ev_fork);
  delete P;
}

}  // extern "C"
