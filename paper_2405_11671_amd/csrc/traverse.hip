// Level loops for BFS and min-label connectivity over edgeMap (paper Table
// algs-list; BFS emits unvisited neighbours, Section 3.2), the public
// edgeMap entry point, and the direction / load-balance choice made before
// every edgeMap call from |U|, sum(deg(U)) and m (Section 6.3: num_edges and
// degree decide the sparse/dense cutoff).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>
#include <vector>

#include "internal.h"

namespace byo {

// ---------------------------------------------------------------- variant choice

static bool is_pull(int v) { return v == BYO_V_PULL_THREAD || v == BYO_V_PULL_WAVE; }

int heuristic_variant(const byo_opts &o, const level_features &f, bool allow_pull) {
  return heuristic_rule(f.k, f.degsum, f.m, f.max_deg, f.cv, o.dense_divisor, o.t_wave, o.t_block, allow_pull,
                        f.frontier_max_deg);
}

int choose_variant(const byo_opts &o, const level_features &f, bool allow_pull) {
  if (o.selector == BYO_SEL_FIXED) {
    int v = o.fixed_variant;
    if (v < 0 || v >= BYO_NUM_VARIANTS) v = BYO_V_PUSH_EDGE;
    if (!allow_pull && is_pull(v)) v = BYO_V_PUSH_EDGE;
    return v;
  }
  return heuristic_variant(o, f, allow_pull);
}

// Variant for this level: the learned selector's choice from this level's
// features, else the fixed / threshold rule.
static int pick(const byo_opts &o, const level_features &f, bool use_mlp) {
  if (use_mlp) {
    int v = selector_pick_cpu(f, true);
    if (v >= 0 && v < BYO_NUM_VARIANTS) return v;
  }
  return choose_variant(o, f, true);
}

// ---------------------------------------------------------------- small kernels

__global__ void bfs_init_kernel(int32_t *parent, int32_t *depth, const int32_t *srcs, int64_t nsrc, int32_t *ids,
                                byo_counters *ctr) {
  if (blockIdx.x == 0 && threadIdx.x < BYO_COUNTER_SLOTS) {
    ctr[threadIdx.x].count = 0;
    ctr[threadIdx.x].degsum = 0;
    ctr[threadIdx.x].aux0 = 0;
    ctr[threadIdx.x].aux1 = 0;
    ctr[threadIdx.x].maxdeg = 0;
  }
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nsrc) {
    int32_t s = srcs[i];
    parent[s] = s;
    depth[s] = 0;
    ids[i] = s;
  }
}

__global__ void bfs_visited_sources_kernel(uint64_t *visited, const int32_t *srcs, int64_t nsrc) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nsrc) atomicOr((unsigned long long *)&visited[srcs[i] >> 6], 1ull << (srcs[i] & 63));
}

// visited starts as {src} plus every degree-0 vertex (never reachable from
// another vertex) plus the bits past n, so the pull direction can skip whole
// 64-vertex words once their reachable members are visited.
__global__ void bfs_visited_init_kernel(uint64_t *__restrict__ visited, const uint64_t *__restrict__ zero_bits,
                                        int64_t n, int64_t words, int32_t src) {
  for (int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; w < words; w += (int64_t)gridDim.x * blockDim.x) {
    uint64_t x = zero_bits[w];
    if (w == words - 1 && (n & 63)) x |= ~0ull << (n & 63);
    if (src >= 0 && w == (int64_t)(src >> 6)) x |= 1ull << (src & 63);
    visited[w] = x;
  }
}

// Single-source start in two launches: every parent and depth to -1 and the
// visited bitmap as bfs_visited_init_kernel sets it (src included) ...
__global__ void bfs_reset_kernel(int32_t *__restrict__ parent, int32_t *__restrict__ depth,
                                 uint64_t *__restrict__ visited, const uint64_t *__restrict__ zero_bits, int64_t n,
                                 int64_t words, int32_t src) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    parent[i] = -1;
    depth[i] = -1;
    if (i < words) {
      uint64_t x = zero_bits[i];
      if (i == words - 1 && (n & 63)) x |= ~0ull << (n & 63);
      if (i == (int64_t)(src >> 6)) x |= 1ull << (src & 63);
      visited[i] = x;
    }
  }
}

// ... then the source's parent and depth, the first frontier list {src}, its
// degree scan (0, deg) and, in counter slot `stats`, its degree sum and
// largest degree; the other counter slots cleared.
__global__ void bfs_single_init_kernel(int32_t *__restrict__ parent, int32_t *__restrict__ depth, int32_t src,
                                       const int32_t *__restrict__ deg, int32_t *__restrict__ ids,
                                       long long *__restrict__ scan, byo_counters *ctr, int stats) {
  const int t = threadIdx.x;
  if (t < BYO_COUNTER_SLOTS) {
    const unsigned long long d = t == stats ? (unsigned long long)deg[src] : 0ull;
    ctr[t].count = 0;
    ctr[t].degsum = d;
    ctr[t].aux0 = 0;
    ctr[t].aux1 = 0;
    ctr[t].maxdeg = d;
  }
  if (t == 0) {
    parent[src] = src;
    depth[src] = 0;
    ids[0] = src;
    scan[0] = 0;
    scan[1] = (long long)deg[src];
  }
}

__global__ void set_tail_kernel(uint64_t *bits, int64_t n, int64_t words) {
  if (threadIdx.x == 0 && (n & 63)) bits[words - 1] |= (~0ull << (n & 63));
}

__global__ void iota_kernel(int32_t *p, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = (int32_t)i;
}

__global__ void zero_counters_kernel(byo_counters *ctr) {
  if (threadIdx.x < BYO_COUNTER_SLOTS) {
    ctr[threadIdx.x].count = 0;
    ctr[threadIdx.x].degsum = 0;
    ctr[threadIdx.x].aux0 = 0;
    ctr[threadIdx.x].aux1 = 0;
    ctr[threadIdx.x].maxdeg = 0;
  }
}

// The first frontier's statistics into one counter slot (read back once):
// the degree sum from the frontier scan, the largest degree by a max over the
// sources.
__global__ void src_stats_kernel(const int32_t *__restrict__ ids, int64_t k, const int32_t *__restrict__ deg,
                                 const long long *__restrict__ scan_total, byo_counters *slot) {
  unsigned long long mx = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < k; i += (int64_t)gridDim.x * blockDim.x) {
    const unsigned long long d = (unsigned long long)deg[ids[i]];
    mx = d > mx ? d : mx;
  }
  mx = wave_max(mx);
  if (lane_id() == 0 && mx) atomicMax(&slot->maxdeg, mx);
  if (blockIdx.x == 0 && threadIdx.x == 0) slot->degsum = (unsigned long long)*scan_total;
}

// The largest degree in a frontier as its level reported it; a level whose
// kernels do not track it leaves 0 beside a nonzero degree sum: not known.
static int64_t frontier_max(const byo_counters &c) {
  return (c.maxdeg == 0 && c.degsum > 0) ? -1 : (int64_t)c.maxdeg;
}

static byo_status read_slot(byo_graph *g, int slot, hipStream_t s, byo_counters *out) {
  return sync_read(s, g->ws.ctr + slot, out, sizeof(byo_counters));
}

static level_features features(const byo_graph *g, int64_t k, int64_t degsum, int64_t unvisited, int64_t level,
                               bool dense_in) {
  level_features f;
  f.n = g->n;
  f.m = g->m;
  f.k = k;
  f.degsum = degsum;
  f.unvisited = unvisited;
  f.max_deg = g->max_deg;
  f.level = level;
  f.cv = g->cv_deg;
  f.dense_in = dense_in;
  return f;
}

// Optional per-level record (byo_trace_enable): events around one level.
struct level_timer {
  hipStream_t s;
  hipEvent_t a = nullptr, b = nullptr;
  explicit level_timer(hipStream_t st) : s(st) {
    if (!trace_on()) return;
    a = event_get();
    b = event_get();
    if (a) (void)hipEventRecord(a, s);
  }
  void stop() {
    if (b) (void)hipEventRecord(b, s);
  }
  void record(int algo, const byo_graph *g, const level_features &f, int variant, int64_t out_count,
              int64_t out_degsum) {
    if (!a || !b) return;
    float ms = 0.f;
    (void)hipEventSynchronize(b);
    (void)hipEventElapsedTime(&ms, a, b);
    byo_level_record r;
    std::memset(&r, 0, sizeof(r));
    r.algo = algo;
    r.level = (int32_t)f.level;
    r.variant = variant;
    r.dense_in = f.dense_in ? 1 : 0;
    r.n = g->n;
    r.m = g->m;
    r.k = f.k;
    r.degsum = f.degsum;
    r.unvisited = f.unvisited;
    r.out_count = out_count;
    r.out_degsum = out_degsum;
    r.max_deg = g->max_deg;
    r.max_deg_u = (int32_t)f.frontier_max_deg;
    r.cv = g->cv_deg;
    r.ms = ms;
    trace_push(r);
  }
  ~level_timer() {
    event_put(a);
    event_put(b);
  }
};

// Frontier held in the workspace: ids[cur] and/or bits[cur].
struct frontier {
  int cur = 0;
  bool sparse = false, dense = false;
  int64_t k = 0, degsum = 0;
  int64_t maxdeg = -1;  // largest degree in the frontier (-1: not known)
};

static byo_status make_sparse(byo_graph *g, frontier &fr, hipStream_t s) {
  if (fr.sparse) return BYO_OK;
  byo_workspace &w = g->ws;
  BYO_TRY(bitmap_to_ids(w.bits[fr.cur], w.words, g->n, w.ids[fr.cur], w.partial, w.partial_cap,
                        (unsigned long long *)w.misc, s));
  fr.sparse = true;
  return BYO_OK;
}

static byo_status make_dense(byo_graph *g, frontier &fr, hipStream_t s) {
  if (fr.dense) return BYO_OK;
  byo_workspace &w = g->ws;
  BYO_TRY(ids_to_bitmap(w.ids[fr.cur], fr.k, w.bits[fr.cur], w.words, s));
  fr.dense = true;
  return BYO_OK;
}

// A container that leaves out optional functions of the graph API (Section
// 4.2; the configurations of Table api-components-avg). Without degree() the
// run sees only degrees it has mapped: the graph's degree array is swapped,
// for the run, for the buffer that the mapped degrees of each frontier go to,
// and the frontier's degree sum comes from that map. Without num_edges() m is
// summed over the vertices whenever a level needs it.
struct api_scope {
  byo_graph *g;
  uint32_t omit;
  int32_t *saved = nullptr;
  api_scope(byo_graph *gr, int32_t om) : g(gr), omit((uint32_t)om) {}
  api_scope(const api_scope &) = delete;
  api_scope &operator=(const api_scope &) = delete;
  byo_status begin(hipStream_t s) {
    if (!(omit & BYO_API_NO_DEGREE)) return BYO_OK;
    int32_t *mdeg = nullptr;
    BYO_TRY(api_degree_buffer(g, s, &mdeg));
    saved = g->deg;
    g->deg = mdeg;
    return BYO_OK;
  }
  ~api_scope() {
    if (saved) g->deg = saved;
  }
  // at a level's start: the frontier's degree sum and m as the container
  // provides them
  byo_status level(frontier &fr, hipStream_t s, int64_t *m) {
    if (omit & BYO_API_NO_DEGREE) {
      byo_workspace &w = g->ws;
      BYO_TRY(api_frontier_degrees(g, omit, fr.sparse ? w.ids[fr.cur] : nullptr,
                                   fr.sparse ? nullptr : w.bits[fr.cur], fr.k, s, &fr.degsum));
    }
    return api_num_edges(g, omit, g->deg, s, m);
  }
};

}  // namespace byo

using namespace byo;

extern "C" {

}  // extern "C"

namespace byo {

byo_status bfs_sources_init(byo_graph *g, const int32_t *d_srcs, int64_t ns, int32_t *parent, int32_t *depth,
                            hipStream_t s) {
  byo_workspace &w = g->ws;
  bfs_visited_init_kernel<<<(unsigned)std::min<int64_t>((w.words + 255) / 256, 4096), 256, 0, s>>>(
      w.visited, g->zero_bits, g->n, w.words, -1);
  bfs_visited_sources_kernel<<<(unsigned)((ns + 255) / 256), 256, 0, s>>>(w.visited, d_srcs, ns);
  bfs_init_kernel<<<(unsigned)((ns + 255) / 256), 256, 0, s>>>(parent, depth, d_srcs, ns, w.ids[0], w.ctr);
  BYO_HIP(hipGetLastError());
  return BYO_OK;
}

// BFS from a set of distinct sources (a single source, or one per graph of a
// batch laid out as a disjoint union).
byo_status bfs_run(byo_graph *g, const int32_t *srcs, int64_t ns, int32_t *d_depth, int32_t *d_parent,
                   const byo_opts &o, hipStream_t s, byo_run_stats *stats) {
  BYO_TRY(ws_ensure_traversal(g));
  byo_workspace &w = g->ws;
  int64_t n = g->n;
  api_scope api(g, o.api_omit);
  BYO_TRY(api.begin(s));
  BYO_CHECK(ns >= 1 && ns <= n, BYO_EINVAL, "bad source count");
  BYO_CHECK(!o.compressed || o.api_omit == 0, BYO_EINVAL, "byte-coded lists run with the full container API");
  if (o.compressed) BYO_TRY(cz_ensure(g, s, nullptr));
  // slot BYO_COUNTER_SLOTS - 1 receives the first frontier's statistics: it
  // is next written by level 3 and cleared by level 1
  if (ns == 1) {
    bfs_reset_kernel<<<(unsigned)std::min<int64_t>((n + 255) / 256, 8192), 256, 0, s>>>(
        d_parent, d_depth, w.visited, g->zero_bits, n, w.words, srcs[0]);
    bfs_single_init_kernel<<<1, 64, 0, s>>>(d_parent, d_depth, srcs[0], g->deg, w.ids[0], w.scan, w.ctr,
                                            BYO_COUNTER_SLOTS - 1);
    BYO_HIP(hipGetLastError());
  } else {
    BYO_TRY(fill_i32(d_parent, n, -1, s));
    BYO_TRY(fill_i32(d_depth, n, -1, s));
    // sources staged through the spare frontier list
    BYO_HIP(hipMemcpyAsync(w.ids[1], srcs, sizeof(int32_t) * (size_t)ns, hipMemcpyHostToDevice, s));
    bfs_visited_init_kernel<<<(unsigned)std::min<int64_t>((w.words + 255) / 256, 4096), 256, 0, s>>>(
        w.visited, g->zero_bits, n, w.words, srcs[0]);
    bfs_visited_sources_kernel<<<(unsigned)((ns + 255) / 256), 256, 0, s>>>(w.visited, w.ids[1], ns);
    bfs_init_kernel<<<(unsigned)((ns + 255) / 256), 256, 0, s>>>(d_parent, d_depth, w.ids[1], ns, w.ids[0], w.ctr);
    BYO_HIP(hipGetLastError());
    BYO_TRY(frontier_degree_scan(g, w.ids[0], ns, w.scan, w.partial, w.partial_cap, s));
    src_stats_kernel<<<(unsigned)std::min<int64_t>((ns + 255) / 256, 1024), 256, 0, s>>>(
        w.ids[0], ns, g->deg, w.scan + ns, w.ctr + (BYO_COUNTER_SLOTS - 1));
    BYO_HIP(hipGetLastError());
  }
  long long dsum = 0;
  bool use_mlp = o.selector == BYO_SEL_MLP && selector_ready();
  byo_counters c0;
  BYO_TRY(read_slot(g, BYO_COUNTER_SLOTS - 1, s, &c0));
  dsum = (long long)c0.degsum;

  byo_run_stats st;
  std::memset(&st, 0, sizeof(st));
  frontier fr;
  fr.cur = 0;
  fr.sparse = true;
  fr.k = ns;
  fr.degsum = dsum;
  fr.maxdeg = frontier_max(c0);
  // without degree() each frontier's degree sum is mapped at its level
  const bool mapped_deg = (o.api_omit & BYO_API_NO_DEGREE) != 0;
  int64_t reached = ns, edges = mapped_deg ? 0 : dsum;
  int64_t cap = o.max_levels > 0 ? o.max_levels : n + 1;
  bfs_state bs{d_parent, d_depth, w.visited, 0};
  int32_t level = 0;
  while (true) {
    if (level >= cap) {
      if (stats) *stats = st;
      return fail(BYO_ELIMIT, "BFS level cap reached");
    }
    const int64_t dl_edges = std::min<int64_t>(std::max<int64_t>(16 * (int64_t)o.small_frontier, 65536),
                                               BYO_DLOOP_QCAP);
    if (o.small_frontier > 0 && o.api_omit == 0 && !o.compressed && fr.k <= o.small_frontier &&
        fr.k <= BYO_DLOOP_QCAP &&
        fr.degsum <= dl_edges && bfs_small_loop_usable(g)) {
      // run levels on the device while the frontier stays small
      BYO_TRY(make_sparse(g, fr, s));
      small_loop_out r;
      int32_t budget = (int32_t)std::min<int64_t>(cap - level, 1 << 20);
      BYO_TRY(bfs_small_loop(g, w.ids[fr.cur], fr.k, fr.degsum, level, budget, o.small_frontier, dl_edges, d_parent,
                             d_depth, w.visited, w.ids[1 - fr.cur], s, &r));
      level += r.levels;
      st.device_levels += r.levels;
      st.variant_count[BYO_V_PUSH_BUCKET] += r.levels;
      reached += r.reached;
      edges += r.edges;
      if (r.empty) break;
      fr.cur = r.side == 0 ? 1 - fr.cur : fr.cur;
      fr.sparse = true;
      fr.dense = false;
      fr.k = r.count;
      fr.degsum = r.degsum;
      fr.maxdeg = -1;  // the device loop does not report it
      zero_counters_kernel<<<1, 64, 0, s>>>(w.ctr);  // ring slots were not advanced on the device
      BYO_HIP(hipGetLastError());
      if (level >= cap) {
        if (stats) *stats = st;
        return fail(BYO_ELIMIT, "BFS level cap reached");
      }
      continue;
    }
    int64_t m_seen = g->m;
    if (o.api_omit) {
      BYO_TRY(api.level(fr, s, &m_seen));
      if (mapped_deg) edges += fr.degsum;
    }
    level_features f = features(g, fr.k, fr.degsum, n - reached, level, fr.dense && !fr.sparse);
    f.m = m_seen;
    f.frontier_max_deg = mapped_deg ? -1 : fr.maxdeg;
    int v = pick(o, f, use_mlp);
    if (o.api_omit) v = api_variant((uint32_t)o.api_omit, v, true);
    if (o.compressed) v = cz_variant(v);
    int nxt = 1 - fr.cur;
    level_io io;
    std::memset(&io, 0, sizeof(io));
    io.in_count = fr.k;
    io.ctr = w.ctr + (level % BYO_COUNTER_SLOTS);
    io.ctr_clear = w.ctr + ((level + 2) % BYO_COUNTER_SLOTS);
    level_timer lt(s);
    if (is_pull(v)) {
      BYO_TRY(make_dense(g, fr, s));
      io.in_bits = w.bits[fr.cur];
      io.out_bits = w.bits[nxt];
    } else {
      BYO_TRY(make_sparse(g, fr, s));
      io.in_ids = w.ids[fr.cur];
      io.out_ids = w.ids[nxt];
    }
    bs.level = level;
    if (o.compressed)
      BYO_TRY(cz_bfs_level(g, v, bs, io, s, fr.degsum));
    else
      BYO_TRY(bfs_level(g, v, bs, io, o, s, fr.degsum));
    lt.stop();
    st.variant_count[v]++;
    byo_counters c;
    BYO_TRY(read_slot(g, level % BYO_COUNTER_SLOTS, s, &c));
    lt.record(BYO_ALGO_BFS, g, f, v, (int64_t)c.count, (int64_t)c.degsum);
    ++level;
    if (c.count == 0) break;
    reached += (int64_t)c.count;
    if (!mapped_deg) edges += (int64_t)c.degsum;
    fr.cur = nxt;
    fr.sparse = !is_pull(v);
    fr.dense = is_pull(v);
    fr.k = (int64_t)c.count;
    fr.degsum = (int64_t)c.degsum;
    fr.maxdeg = frontier_max(c);
  }
  st.levels = level;
  st.reached = reached;
  st.edges = edges;
  if (stats) *stats = st;
  return BYO_OK;
}

}  // namespace byo

extern "C" {

byo_status byo_bfs(byo_graph *g, int64_t src, int32_t *d_depth, int32_t *d_parent, const byo_opts *opts,
                   void *stream, byo_run_stats *stats) {
  BYO_CHECK(g && d_depth && d_parent, BYO_EINVAL, "null argument");
  BYO_CHECK(src >= 0 && src < g->n, BYO_EINVAL, "source out of range");
  byo_opts o;
  byo_opts_default(&o);
  if (opts) o = *opts;
  std::vector<int32_t> srcs(1, (int32_t)src);
  // persistent = 2: the whole search in one persistent launch, the one the
  // batch runs (direction by the threshold rule on the device)
  if (o.persistent == 2 && o.api_omit == 0 && !o.compressed && !o.use_graph && bfs_persistent_usable(g))
    return bfs_persistent_run(g, srcs.data(), 1, d_depth, d_parent, o, (hipStream_t)stream, stats);
  if (o.use_graph && o.api_omit == 0 && !o.compressed) return bfs_graph_run(g, srcs, d_depth, d_parent, o, (hipStream_t)stream, stats);
  return bfs_run(g, srcs.data(), (int64_t)srcs.size(), d_depth, d_parent, o, (hipStream_t)stream, stats);
}

byo_status byo_cc(byo_graph *g, int32_t *d_label, const byo_opts *opts, void *stream, byo_run_stats *stats) {
  BYO_CHECK(g && d_label, BYO_EINVAL, "null argument");
  byo_opts o;
  byo_opts_default(&o);
  if (opts) o = *opts;
  hipStream_t s = (hipStream_t)stream;
  int64_t n = g->n;
  byo_run_stats st;
  std::memset(&st, 0, sizeof(st));
  if (n == 0) {
    if (stats) *stats = st;
    return BYO_OK;
  }
  BYO_CHECK(!o.compressed || o.api_omit == 0, BYO_EINVAL, "byte-coded lists run with the full container API");
  if (o.tiled && o.api_omit == 0 && !o.compressed && tiles_wanted(g)) return cc_tiled_run(g, d_label, o, s, stats);
  BYO_TRY(ws_ensure_traversal(g));
  if (o.compressed) BYO_TRY(cz_ensure(g, s, nullptr));
  byo_workspace &w = g->ws;
  api_scope api(g, o.api_omit);
  BYO_TRY(api.begin(s));
  iota_kernel<<<(unsigned)std::min<int64_t>((n + 255) / 256, 8192), 256, 0, s>>>(d_label, n);
  zero_counters_kernel<<<1, 64, 0, s>>>(w.ctr);
  BYO_HIP(hipGetLastError());
  // every vertex starts in the frontier
  BYO_TRY(fill_u64(w.bits[0], w.words, ~0ull, s));
  if (n & 63) {
    // clear bits >= n: the frontier bitmap never holds them
    uint64_t last = ~0ull >> (64 - (n & 63));
    BYO_HIP(hipMemcpyAsync(w.bits[0] + (w.words - 1), &last, sizeof(last), hipMemcpyHostToDevice, s));
    BYO_HIP(hipStreamSynchronize(s));
  }
  frontier fr;
  fr.cur = 0;
  fr.dense = true;
  fr.k = n;
  fr.degsum = g->m;
  fr.maxdeg = g->max_deg;
  int64_t cap = o.max_levels > 0 ? o.max_levels : n + 1;
  int32_t round = 0;
  bool use_mlp = o.selector == BYO_SEL_MLP && selector_ready();
  while (true) {
    if (round >= cap) {
      if (stats) *stats = st;
      return fail(BYO_ELIMIT, "connectivity round cap reached");
    }
    int64_t m_seen = g->m;
    if (o.api_omit) {
      BYO_TRY(api.level(fr, s, &m_seen));
      // the first frontier holds every vertex: its degree sum is m
      if (round == 0 && !(o.api_omit & BYO_API_NO_DEGREE)) fr.degsum = m_seen;
    }
    level_features f = features(g, fr.k, fr.degsum, n, round, fr.dense && !fr.sparse);
    f.m = m_seen;
    f.frontier_max_deg = (o.api_omit & BYO_API_NO_DEGREE) ? -1 : fr.maxdeg;
    int v = pick(o, f, use_mlp);
    if (o.api_omit) v = api_variant((uint32_t)o.api_omit, v, false);
    if (o.compressed) v = cz_variant(v);
    int nxt = 1 - fr.cur;
    level_io io;
    std::memset(&io, 0, sizeof(io));
    io.in_count = fr.k;
    io.ctr = w.ctr + (round % BYO_COUNTER_SLOTS);
    io.ctr_clear = w.ctr + ((round + 2) % BYO_COUNTER_SLOTS);
    io.out_bits = w.bits[nxt];
    bool shortcut = o.cc_shortcut != 0;
    level_timer lt(s);
    if (is_pull(v)) {
      BYO_TRY(make_dense(g, fr, s));
      io.in_bits = w.bits[fr.cur];
    } else {
      BYO_TRY(make_sparse(g, fr, s));
      io.in_ids = w.ids[fr.cur];
      io.out_ids = shortcut ? nullptr : w.ids[nxt];
    }
    if (o.compressed)
      BYO_TRY(cz_cc_level(g, v, d_label, io, s, fr.degsum));
    else
      BYO_TRY(cc_level(g, v, d_label, io, o, s, fr.degsum));
    if (shortcut) BYO_TRY(cc_shortcut(g, d_label, w.bits[nxt], io.ctr, s));
    lt.stop();
    st.variant_count[v]++;
    byo_counters c;
    BYO_TRY(read_slot(g, round % BYO_COUNTER_SLOTS, s, &c));
    lt.record(BYO_ALGO_CC, g, f, v, (int64_t)c.count, (int64_t)c.degsum);
    ++round;
    if (c.count == 0) break;
    fr.cur = nxt;
    fr.dense = true;
    fr.sparse = !is_pull(v) && !shortcut;
    fr.k = (int64_t)c.count;
    fr.degsum = (int64_t)c.degsum;
    fr.maxdeg = frontier_max(c);
  }
  st.levels = round;
  if (stats) *stats = st;
  return BYO_OK;
}

byo_status byo_edge_map(byo_graph *g, byo_vset *U, byo_edge_fn F, const void *F_state, byo_vset *out,
                        int32_t variant, const byo_opts *opts, void *stream, int32_t *variant_used) {
  BYO_CHECK(g && U && out && F_state, BYO_EINVAL, "null argument");
  BYO_CHECK(U->g == g && out->g == g, BYO_EINVAL, "subsets belong to another graph");
  BYO_CHECK(U != out, BYO_EINVAL, "input and output subsets must differ");
  BYO_CHECK(variant < BYO_NUM_VARIANTS, BYO_EINVAL, "unknown variant");
  byo_opts o;
  byo_opts_default(&o);
  if (opts) o = *opts;
  hipStream_t s = (hipStream_t)stream;
  BYO_TRY(ws_ensure_traversal(g));
  byo_workspace &w = g->ws;
  if (F == BYO_F_PR_ACC) {
    BYO_CHECK(U->count == g->n, BYO_EINVAL, "PR_ACC needs the full vertex set as input");
    const byo_pr_fn *pf = (const byo_pr_fn *)F_state;
    BYO_TRY(pr_accumulate(g, pf->contrib, pf->acc, s));
    BYO_TRY(byo_vset_fill(out, stream));
    if (variant_used) *variant_used = BYO_V_PULL_WAVE;
    return BYO_OK;
  }
  BYO_CHECK(F == BYO_F_BFS || F == BYO_F_CC_MIN, BYO_EINVAL, "unknown edge function");
  // input degree sum (needed by the selector and the edge-balanced variant)
  if (!U->sparse_valid) {
    BYO_TRY(bitmap_to_ids(U->bits, U->words, U->n, U->ids, w.partial, w.partial_cap, U->d_tmp, s));
    U->sparse_valid = true;
  }
  long long degsum = 0;
  if (U->count > 0) {
    BYO_TRY(frontier_degree_scan(g, U->ids, U->count, w.scan, w.partial, w.partial_cap, s));
    BYO_TRY(sync_read(s, w.scan + U->count, &degsum, sizeof(degsum)));
  }
  level_features f = features(g, U->count, degsum, g->n, 0, false);
  int v = variant >= 0 ? variant : choose_variant(o, f, true);
  if (is_pull(v) && !U->dense_valid) {
    BYO_TRY(ids_to_bitmap(U->ids, U->count, U->bits, U->words, s));
    U->dense_valid = true;
  }
  zero_counters_kernel<<<1, 64, 0, s>>>(w.ctr);
  BYO_HIP(hipGetLastError());
  level_io io;
  std::memset(&io, 0, sizeof(io));
  io.in_ids = U->ids;
  io.in_bits = U->bits;
  io.in_count = U->count;
  io.ctr = w.ctr;
  io.ctr_clear = nullptr;
  io.out_bits = out->bits;
  io.out_ids = is_pull(v) ? nullptr : out->ids;
  if (F == BYO_F_BFS) {
    const byo_bfs_fn *bf = (const byo_bfs_fn *)F_state;
    BYO_CHECK(bf->parent && bf->depth && bf->visited, BYO_EINVAL, "BFS state has a null array");
    bfs_state bs{bf->parent, bf->depth, bf->visited, bf->level};
    if (!is_pull(v)) {
      // push fills the dense output too, so both forms are valid afterwards
      BYO_TRY(bitmap_clear(out->bits, out->words, s));
    }
    BYO_TRY(bfs_level(g, v, bs, io, o, s, degsum));
  } else {
    const byo_cc_fn *cf = (const byo_cc_fn *)F_state;
    BYO_CHECK(cf->label, BYO_EINVAL, "label array is null");
    BYO_TRY(cc_level(g, v, cf->label, io, o, s, degsum));
  }
  byo_counters c;
  BYO_TRY(read_slot(g, 0, s, &c));
  out->count = (int64_t)c.count;
  out->dense_valid = true;
  out->sparse_valid = !is_pull(v);
  if (variant_used) *variant_used = v;
  return BYO_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- selector training data

namespace byo {

static void push_trial(int algo, const byo_graph *g, const level_features &f, int v, float ms, int64_t oc,
                       int64_t od) {
  byo_level_record r;
  std::memset(&r, 0, sizeof(r));
  r.algo = algo;
  r.level = (int32_t)f.level;
  r.variant = v;
  r.dense_in = f.dense_in ? 1 : 0;
  r.n = g->n;
  r.m = g->m;
  r.k = f.k;
  r.degsum = f.degsum;
  r.unvisited = f.unvisited;
  r.out_count = oc;
  r.out_degsum = od;
  r.max_deg = g->max_deg;
  r.max_deg_u = (int32_t)f.frontier_max_deg;
  r.cv = g->cv_deg;
  r.ms = ms;
  trace_push(r);
}

// Time every variant of each level from the same saved state, record one row
// per (level, variant), then advance with the fastest variant.
static byo_status collect(byo_graph *g, int algo, int64_t src, int repeats, int32_t *d_out, const byo_opts &o0,
                          hipStream_t s) {
  BYO_TRY(ws_ensure_traversal(g));
  byo_workspace &w = g->ws;
  int64_t n = g->n;
  byo_opts o = o0;
  o.selector = BYO_SEL_FIXED;
  bool bfs = algo == BYO_ALGO_BFS;
  int32_t *parent = nullptr, *save_a = nullptr, *save_b = nullptr;
  uint64_t *save_vis = nullptr;
  hipEvent_t ea = nullptr, eb = nullptr;
  auto cleanup = [&]() {
    if (parent) (void)hipFree(parent);
    if (save_a) (void)hipFree(save_a);
    if (save_b) (void)hipFree(save_b);
    if (save_vis) (void)hipFree(save_vis);
    if (ea) (void)hipEventDestroy(ea);
    if (eb) (void)hipEventDestroy(eb);
  };
  struct guard {
    std::function<void()> f;
    ~guard() { f(); }
  } gd{cleanup};
  BYO_HIP(hipEventCreate(&ea));
  BYO_HIP(hipEventCreate(&eb));
  size_t ib = sizeof(int32_t) * (size_t)std::max<int64_t>(n, 1);
  BYO_HIP(hipMalloc(&save_a, ib));
  BYO_HIP(hipMalloc(&save_b, ib));
  BYO_HIP(hipMalloc(&save_vis, sizeof(uint64_t) * (size_t)std::max<int64_t>(w.words, 1)));
  frontier fr;
  int64_t reached = 0;
  if (bfs) {
    BYO_CHECK(src >= 0 && src < n, BYO_EINVAL, "source out of range");
    BYO_HIP(hipMalloc(&parent, ib));
    int32_t s32 = (int32_t)src;
    BYO_TRY(fill_i32(parent, n, -1, s));
    BYO_TRY(fill_i32(d_out, n, -1, s));
    BYO_HIP(hipMemcpyAsync(w.ids[1], &s32, sizeof(int32_t), hipMemcpyHostToDevice, s));
    bfs_visited_init_kernel<<<(unsigned)std::min<int64_t>((w.words + 255) / 256, 4096), 256, 0, s>>>(
        w.visited, g->zero_bits, n, w.words, s32);
    bfs_init_kernel<<<1, 256, 0, s>>>(parent, d_out, w.ids[1], 1, w.ids[0], w.ctr);
    int32_t d0 = 0;
    BYO_TRY(sync_read(s, g->deg + src, &d0, sizeof(d0)));
    fr.sparse = true;
    fr.k = 1;
    fr.degsum = d0;
    fr.maxdeg = d0;
    reached = 1;
  } else {
    if (n == 0) return BYO_OK;
    iota_kernel<<<(unsigned)std::min<int64_t>((n + 255) / 256, 8192), 256, 0, s>>>(d_out, n);
    zero_counters_kernel<<<1, 64, 0, s>>>(w.ctr);
    BYO_TRY(fill_u64(w.bits[0], w.words, ~0ull, s));
    if (n & 63) {
      uint64_t last = ~0ull >> (64 - (n & 63));
      BYO_HIP(hipMemcpyAsync(w.bits[0] + (w.words - 1), &last, sizeof(last), hipMemcpyHostToDevice, s));
      BYO_HIP(hipStreamSynchronize(s));
    }
    fr.dense = true;
    fr.k = n;
    fr.degsum = g->m;
    fr.maxdeg = g->max_deg;
  }
  int64_t cap = o.max_levels > 0 ? o.max_levels : n + 1;
  for (int32_t level = 0; level < cap; ++level) {
    level_features f = features(g, fr.k, fr.degsum, bfs ? n - reached : n, level, fr.dense && !fr.sparse);
    f.frontier_max_deg = fr.maxdeg;
    // save the state a level modifies
    BYO_HIP(hipMemcpyAsync(save_a, d_out, ib, hipMemcpyDeviceToDevice, s));
    if (bfs) {
      BYO_HIP(hipMemcpyAsync(save_b, parent, ib, hipMemcpyDeviceToDevice, s));
      BYO_HIP(hipMemcpyAsync(save_vis, w.visited, sizeof(uint64_t) * w.words, hipMemcpyDeviceToDevice, s));
    }
    frontier saved = fr;
    int best = -1;
    float best_ms = 0.f;
    byo_counters c;
    std::memset(&c, 0, sizeof(c));
    for (int pass = 0; pass <= BYO_NUM_VARIANTS; ++pass) {
      // passes 0..K-1 time each variant; the last pass re-runs the fastest to advance
      bool final_pass = pass == BYO_NUM_VARIANTS;
      int v = final_pass ? best : pass;
      int reps = final_pass ? 1 : std::max(1, repeats);
      float vbest = 0.f;
      for (int r = 0; r < reps; ++r) {
        BYO_HIP(hipMemcpyAsync(d_out, save_a, ib, hipMemcpyDeviceToDevice, s));
        if (bfs) {
          BYO_HIP(hipMemcpyAsync(parent, save_b, ib, hipMemcpyDeviceToDevice, s));
          BYO_HIP(hipMemcpyAsync(w.visited, save_vis, sizeof(uint64_t) * w.words, hipMemcpyDeviceToDevice, s));
        }
        fr = saved;
        zero_counters_kernel<<<1, 64, 0, s>>>(w.ctr);
        int nxt = 1 - fr.cur;
        level_io io;
        std::memset(&io, 0, sizeof(io));
        io.in_count = fr.k;
        io.ctr = w.ctr;
        BYO_HIP(hipEventRecord(ea, s));
        if (bfs) {
          if (is_pull(v)) {
            BYO_TRY(make_dense(g, fr, s));
            io.in_bits = w.bits[fr.cur];
            io.out_bits = w.bits[nxt];
          } else {
            BYO_TRY(make_sparse(g, fr, s));
            io.in_ids = w.ids[fr.cur];
            io.out_ids = w.ids[nxt];
          }
          bfs_state bs{parent, d_out, w.visited, level};
          BYO_TRY(bfs_level(g, v, bs, io, o, s, fr.degsum));
        } else {
          io.out_bits = w.bits[nxt];
          if (is_pull(v)) {
            BYO_TRY(make_dense(g, fr, s));
            io.in_bits = w.bits[fr.cur];
          } else {
            BYO_TRY(make_sparse(g, fr, s));
            io.in_ids = w.ids[fr.cur];
          }
          BYO_TRY(cc_level(g, v, d_out, io, o, s, fr.degsum));
          if (o.cc_shortcut) BYO_TRY(cc_shortcut(g, d_out, w.bits[nxt], io.ctr, s));
        }
        BYO_HIP(hipEventRecord(eb, s));
        BYO_TRY(read_slot(g, 0, s, &c));
        float ms = 0.f;
        BYO_HIP(hipEventSynchronize(eb));  // the counters can arrive before the event completes
        BYO_HIP(hipEventElapsedTime(&ms, ea, eb));
        if (r == 0 || ms < vbest) vbest = ms;
      }
      if (final_pass) break;
      push_trial(algo, g, f, v, vbest, (int64_t)c.count, (int64_t)c.degsum);
      if (best < 0 || vbest < best_ms) {
        best = v;
        best_ms = vbest;
      }
    }
    if (c.count == 0) break;
    reached += (int64_t)c.count;
    fr.cur = 1 - fr.cur;
    if (bfs) {
      fr.sparse = !is_pull(best);
      fr.dense = is_pull(best);
    } else {
      fr.dense = true;
      fr.sparse = false;
    }
    fr.k = (int64_t)c.count;
    fr.degsum = (int64_t)c.degsum;
    fr.maxdeg = frontier_max(c);
  }
  BYO_HIP(hipStreamSynchronize(s));
  return BYO_OK;
}

}  // namespace byo

extern "C" byo_status byo_selector_collect(byo_graph *g, int32_t algo, int64_t src, int32_t repeats, int32_t *d_out,
                                           const byo_opts *opts, void *stream) {
  BYO_CHECK(g && d_out, BYO_EINVAL, "null argument");
  BYO_CHECK(algo == BYO_ALGO_BFS || algo == BYO_ALGO_CC, BYO_EINVAL, "collection supports BFS and CC");
  byo_opts o;
  byo_opts_default(&o);
  if (opts) o = *opts;
  return collect(g, algo, src, repeats, d_out, o, (hipStream_t)stream);
}
