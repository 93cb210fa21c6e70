// BFS with every per-level decision on the device, so a run of levels can be
// captured once into a hipGraph and replayed with one host sync per replay.
//
// A level is a fixed launch sequence (grids fixed at capture time):
//   gm_select    one block: counts the level just finished, stops on an empty
//                frontier or at the level cap, and picks push or pull with the
//                threshold rule (dense iff |U| + sum(deg U) > m / div), or with
//                the learned selector evaluated on the device (BYO_SEL_MLP);
//   gm_prepush   push only: zero the output bitmap and, after a pull level,
//                turn the input bitmap into an ID list;
//   gm_push      degree-bucketed push from the list (thread per vertex,
//                wavefront for lists longer than t_wave); output list + bitmap;
//   gm_pull      wavefront-per-word early-exit pull; output bitmap;
// every kernel after the select returns at once unless it was chosen. Buffers
// alternate with level parity, so an even number of levels is replayable.
// Clears are kernels, never memset nodes.
#include <algorithm>
#include <cstring>

#include "internal.h"
#include "selector_dev.h"

namespace byo {

enum { GM_NONE = 0, GM_PUSH = 1, GM_PUSH_COMPACT = 2, GM_PULL = 3 };

// each field on its own 128-byte line (every workgroup adds into count and
// degsum; device-scope atomics on one line serialise)
struct gm_counters {
  unsigned long long count;
  unsigned long long pad0_[BYO_LINE_U64 - 1];
  unsigned long long degsum;
  unsigned long long pad1_[BYO_LINE_U64 - 1];
  unsigned long long list_valid;  // the frontier exists as an ID list
  unsigned long long pad2_[BYO_LINE_U64 - 1];
  unsigned long long cursor;      // append cursor used when compacting this frontier
  unsigned long long pad3_[BYO_LINE_U64 - 1];
};
static_assert(2 * sizeof(gm_counters) <= 1024, "two counter sets fit between misc + 1024 and the state at + 2048");

struct gm_state {
  int32_t sel, prev_sel;
  int32_t level;                  // index of the level being run
  int32_t done, limit, pad;
  unsigned long long reached, edges;
  unsigned long long push_levels, pull_levels;
};

constexpr int GM_BLOCK = 256;
constexpr int GM_GRID = 2048;

// One block of 64 threads. With learned weights (wts non-null) the block
// evaluates the selector network on the level's features, as the host-driven
// loop does from its counters, and a pull variant choice means pull; without
// them, or if a prediction is not finite, the threshold rule decides.
__global__ void __launch_bounds__(64) gm_select_kernel(gm_counters *__restrict__ cin, gm_counters *__restrict__ cout,
                                                       gm_state *__restrict__ st, int64_t n, int64_t m, int32_t div,
                                                       int32_t cap, const float *__restrict__ wts, int64_t max_deg,
                                                       double cv) {
  __shared__ int go, pull;
  __shared__ float raw[SEL_F];
  if (threadIdx.x == 0) {
    go = 0;
    if (st->prev_sel != GM_NONE) st->level += 1;
    st->prev_sel = GM_NONE;
    st->sel = GM_NONE;
    if (!st->done) {
      const unsigned long long k = cin->count, ds = cin->degsum;
      if (k == 0) {
        st->done = 1;
      } else if (st->level >= cap) {
        st->done = 1;
        st->limit = 1;
      } else {
        st->reached += k;
        st->edges += ds;
        go = 1;
        pull = (long long)(k + ds) > m / (div > 0 ? div : 20);
        if (wts)
          selector_features((double)k, (double)ds, (double)(n - (int64_t)st->reached), (double)n, (double)m,
                            (double)max_deg, cv, cin->list_valid ? 0.0 : 1.0, raw);
      }
    }
  }
  __syncthreads();
  if (!go) return;  // uniform over the block
  if (wts) {
    const int v = sel_pick_block(wts, raw, true, nullptr);
    if (threadIdx.x == 0 && v >= 0) pull = v == BYO_V_PULL_THREAD || v == BYO_V_PULL_WAVE;
  }
  if (threadIdx.x != 0) return;
  const int sel = pull ? GM_PULL : (cin->list_valid ? GM_PUSH : GM_PUSH_COMPACT);
  st->sel = sel;
  st->prev_sel = sel;
  if (pull) st->pull_levels += 1; else st->push_levels += 1;
  cin->cursor = 0;
  cout->count = 0;
  cout->degsum = 0;
  cout->cursor = 0;
  cout->list_valid = pull ? 0ull : 1ull;
}

__global__ void __launch_bounds__(GM_BLOCK) gm_prepush_kernel(const gm_state *__restrict__ st,
                                                              gm_counters *__restrict__ cin,
                                                              const uint64_t *__restrict__ in_bits,
                                                              int32_t *__restrict__ in_ids,
                                                              uint64_t *__restrict__ out_bits, int64_t words,
                                                              int64_t n) {
  int sel = st->sel;
  if (sel != GM_PUSH && sel != GM_PUSH_COMPACT) return;
  for (int64_t w = (int64_t)blockIdx.x * GM_BLOCK + threadIdx.x; w < words; w += (int64_t)gridDim.x * GM_BLOCK)
    out_bits[w] = 0ull;
  if (sel != GM_PUSH_COMPACT) return;
  // input bitmap -> ID list (order is irrelevant to push); one atomic per wavefront-word group
  for (int64_t w = (int64_t)blockIdx.x * GM_BLOCK + threadIdx.x; w - threadIdx.x < words;
       w += (int64_t)gridDim.x * GM_BLOCK) {
    uint64_t x = w < words ? in_bits[w] : 0ull;
    if (w == words - 1 && (n & 63)) x &= ~0ull >> (64 - (n & 63));
    unsigned c = (unsigned)__popcll(x);
    unsigned inc = c;
    for (int o = 1; o < BYO_WAVE; o <<= 1) {
      unsigned t = __shfl_up(inc, o);
      if (lane_id() >= o) inc += t;
    }
    unsigned tot = (unsigned)read_lane_i32((int32_t)inc, BYO_WAVE - 1);
    unsigned long long base = 0;
    if (lane_id() == 0 && tot) base = atomicAdd(&cin->cursor, (unsigned long long)tot);
    base = read_lane_u64(base, 0);
    unsigned long long pos = base + inc - c;
    while (x) {
      int b = __ffsll((long long)x) - 1;
      in_ids[pos++] = (int32_t)(w * 64 + b);
      x &= x - 1;
    }
  }
}

__global__ void __launch_bounds__(GM_BLOCK) gm_push_kernel(const gm_state *__restrict__ st,
                                                           const gm_counters *__restrict__ cin,
                                                           gm_counters *__restrict__ cout,
                                                           const int64_t *__restrict__ off,
                                                           const int32_t *__restrict__ nbr,
                                                           const int32_t *__restrict__ deg,
                                                           const int32_t *__restrict__ in_ids,
                                                           int32_t *__restrict__ out_ids,
                                                           uint64_t *__restrict__ out_bits,
                                                           int32_t *__restrict__ parent, int32_t *__restrict__ depth,
                                                           uint64_t *__restrict__ visited, int32_t t_wave) {
  int sel = st->sel;
  if (sel != GM_PUSH && sel != GM_PUSH_COMPACT) return;
  const int64_t k = (int64_t)cin->count;
  const int32_t nd = st->level + 1;
  unsigned long long degsum = 0;
  auto claim = [&](int32_t u, int32_t v) -> bool {
    uint64_t bit = 1ull << (v & 63);
    if (visited[v >> 6] & bit) return false;
    if (atomicCAS(&parent[v], -1, u) != -1) return false;
    depth[v] = nd;
    atomicOr((unsigned long long *)&visited[v >> 6], (unsigned long long)bit);
    atomicOr((unsigned long long *)&out_bits[v >> 6], (unsigned long long)bit);
    return true;
  };
  for (int64_t base = (int64_t)blockIdx.x * GM_BLOCK; base < k; base += (int64_t)gridDim.x * GM_BLOCK) {
    int64_t i = base + threadIdx.x;
    int32_t u = -1;
    int64_t b = 0, e = 0;
    if (i < k) {
      u = in_ids[i];
      b = off[u];
      e = off[u + 1];
    }
    bool wide = u >= 0 && e - b > t_wave;
    if (u >= 0 && !wide) {
      for (int64_t x = b; x < e; ++x) {
        int32_t v = nbr[x];
        bool ok = claim(u, v);
        wave_append(ok, v, out_ids, &cout->count);
        if (ok) degsum += (unsigned long long)deg[v];
      }
    }
    uint64_t wm = __ballot(wide);
    while (wm) {
      int l = __ffsll((long long)wm) - 1;
      wm &= wm - 1;
      int32_t wu = read_lane_i32(u, l);
      int64_t wb = (int64_t)read_lane_u64((uint64_t)b, l), we = (int64_t)read_lane_u64((uint64_t)e, l);
      for (int64_t x = wb + lane_id(); x - lane_id() < we; x += BYO_WAVE) {
        bool ok = false;
        int32_t v = 0;
        if (x < we) {
          v = nbr[x];
          ok = claim(wu, v);
        }
        wave_append(ok, v, out_ids, &cout->count);
        if (ok) degsum += (unsigned long long)deg[v];
      }
    }
  }
  unsigned long long t = block_sum<unsigned long long, GM_BLOCK>(degsum);
  if (threadIdx.x == 0 && t) atomicAdd(&cout->degsum, t);
}

__global__ void __launch_bounds__(GM_BLOCK) gm_pull_kernel(const gm_state *__restrict__ st,
                                                           gm_counters *__restrict__ cout,
                                                           const int64_t *__restrict__ off,
                                                           const int32_t *__restrict__ nbr,
                                                           const int32_t *__restrict__ deg, int64_t n, int64_t words,
                                                           const uint64_t *__restrict__ in_bits,
                                                           uint64_t *__restrict__ out_bits,
                                                           int32_t *__restrict__ parent, int32_t *__restrict__ depth,
                                                           uint64_t *__restrict__ visited, int32_t t_wave) {
  if (st->sel != GM_PULL) return;
  const int32_t nd = st->level + 1;
  unsigned long long degsum = 0, count = 0;
  const int64_t nw = (int64_t)gridDim.x * (GM_BLOCK / BYO_WAVE);
  for (int64_t w = (int64_t)xcd_block(blockIdx.x, gridDim.x) * (GM_BLOCK / BYO_WAVE) + threadIdx.x / BYO_WAVE;
       w < words; w += nw) {
    uint64_t vis = visited[w];
    if (vis == ~0ull) {
      if (lane_id() == 0) out_bits[w] = 0ull;
      continue;
    }
    int64_t v = w * 64 + lane_id();
    bool cand = v < n && !((vis >> lane_id()) & 1ull);
    int32_t par = -1;
    int64_t beg = 0, end = 0;
    if (cand) {
      beg = off[v];
      end = off[v + 1];
      int64_t lim = end - beg > t_wave ? beg + t_wave : end;
      for (int64_t e = beg; e < lim; ++e) {
        int32_t u = nbr[e];
        if (test_bit(in_bits, u)) {
          par = u;
          break;
        }
      }
    }
    uint64_t pm = __ballot(cand && par < 0 && end - beg > t_wave);
    while (pm) {
      int l = __ffsll((long long)pm) - 1;
      pm &= pm - 1;
      int64_t lb = (int64_t)read_lane_u64((uint64_t)(beg + t_wave), l);
      int64_t le = (int64_t)read_lane_u64((uint64_t)end, l);
      for (int64_t base = lb; base < le; base += BYO_WAVE) {
        int64_t e = base + lane_id();
        int32_t u = e < le ? nbr[e] : 0;
        uint64_t hm = __ballot(e < le && test_bit(in_bits, u));
        if (hm) {
          int32_t pu = read_lane_i32(u, __ffsll((long long)hm) - 1);
          if (lane_id() == l) par = pu;
          break;
        }
      }
    }
    bool found = par >= 0;
    if (found) {
      parent[v] = par;
      depth[v] = nd;
      degsum += (unsigned long long)deg[v];
    }
    uint64_t msk = __ballot(found);
    if (lane_id() == 0) {
      out_bits[w] = msk;
      if (msk) {
        visited[w] = vis | msk;
        count += (unsigned long long)__popcll(msk);
      }
    }
  }
  unsigned long long t = block_sum<unsigned long long, GM_BLOCK>(degsum);
  unsigned long long c = block_sum<unsigned long long, GM_BLOCK>(count);
  if (threadIdx.x == 0) {
    if (t) atomicAdd(&cout->degsum, t);
    if (c) atomicAdd(&cout->count, c);
  }
}

__global__ void gm_init_kernel(gm_counters *c0, gm_counters *c1, gm_state *st, unsigned long long k0,
                               const long long *degsum0) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  c0->count = k0;
  c0->degsum = (unsigned long long)*degsum0;
  c0->list_valid = 1;
  c0->cursor = 0;
  c1->count = c1->degsum = c1->list_valid = c1->cursor = 0;
  st->sel = st->prev_sel = GM_NONE;
  st->level = st->done = st->limit = st->pad = 0;
  st->reached = st->edges = st->push_levels = st->pull_levels = 0;
}

// Instantiated graph of `levels` levels for one (graph, output buffers, options) combination.
struct gm_graph {
  hipGraphExec_t exec = nullptr;
  hipStream_t cap = nullptr;
  int32_t *parent = nullptr, *depth = nullptr;
  int levels = 0, div = 0, cap_levels = 0, t_wave = 0;
  const float *wts = nullptr;  // selector weights baked into the captured select kernels
  uint64_t wver = 0;
};

void gm_release(byo_workspace &w) {
  if (!w.gmode) return;
  gm_graph *gg = (gm_graph *)w.gmode;
  if (gg->exec) (void)hipGraphExecDestroy(gg->exec);
  if (gg->cap) (void)hipStreamDestroy(gg->cap);
  delete gg;
  w.gmode = nullptr;
}

static byo_status enqueue_level(byo_graph *g, int parity, int32_t *parent, int32_t *depth, gm_counters *ctr,
                                gm_state *st, int div, int cap_levels, int t_wave, const float *wts, hipStream_t s) {
  byo_workspace &w = g->ws;
  int a = parity, b = 1 - parity;
  gm_select_kernel<<<1, 64, 0, s>>>(ctr + a, ctr + b, st, g->n, g->m, div, cap_levels, wts, g->max_deg, g->cv_deg);
  gm_prepush_kernel<<<GM_GRID, GM_BLOCK, 0, s>>>(st, ctr + a, w.bits[a], w.ids[a], w.bits[b], w.words, g->n);
  gm_push_kernel<<<GM_GRID, GM_BLOCK, 0, s>>>(st, ctr + a, ctr + b, g->off, g->nbr, g->deg, w.ids[a], w.ids[b],
                                              w.bits[b], parent, depth, w.visited, t_wave);
  gm_pull_kernel<<<GM_GRID, GM_BLOCK, 0, s>>>(st, ctr + b, g->off, g->nbr, g->deg, g->n, w.words, w.bits[a],
                                              w.bits[b], parent, depth, w.visited, t_wave);
  BYO_HIP(hipGetLastError());
  return BYO_OK;
}

// BFS from distinct sources with device-side level control, replaying a
// captured graph of `levels` levels until the device reports completion.
byo_status bfs_graph_run(byo_graph *g, const std::vector<int32_t> &srcs, int32_t *d_depth, int32_t *d_parent,
                         const byo_opts &o, hipStream_t s, byo_run_stats *stats) {
  BYO_TRY(ws_ensure_traversal(g));
  byo_workspace &w = g->ws;
  int64_t n = g->n, ns = (int64_t)srcs.size();
  BYO_CHECK(ns >= 1 && ns <= n, BYO_EINVAL, "bad source count");
  gm_counters *ctr = (gm_counters *)((char *)w.misc + 1024);
  gm_state *st = (gm_state *)((char *)w.misc + 2048);
  int div = o.dense_divisor > 0 ? o.dense_divisor : 20;
  int tw = o.t_wave > 0 ? o.t_wave : 32;
  int cap_levels = (int)std::min<int64_t>(o.max_levels > 0 ? o.max_levels : n + 1, 2147483647LL);
  const int K = 16;  // levels per replay (even: buffer parity returns to 0)
  // initial frontier: sources as list (ids[0]) and bitmap (bits[0])
  BYO_TRY(fill_i32(d_parent, n, -1, s));
  BYO_TRY(fill_i32(d_depth, n, -1, s));
  BYO_HIP(hipMemcpyAsync(w.ids[0], srcs.data(), sizeof(int32_t) * (size_t)ns, hipMemcpyHostToDevice, s));
  BYO_TRY(bfs_sources_init(g, w.ids[0], ns, d_parent, d_depth, s));
  BYO_TRY(ids_to_bitmap(w.ids[0], ns, w.bits[0], w.words, s));
  BYO_TRY(frontier_degree_scan(g, w.ids[0], ns, w.scan, w.partial, w.partial_cap, s));
  gm_init_kernel<<<1, 64, 0, s>>>(ctr, ctr + 1, st, (unsigned long long)ns, w.scan + ns);
  BYO_HIP(hipGetLastError());
  // learned choice on the device when asked for and weights are installed
  uint64_t wver = 0;
  const float *wts = o.selector == BYO_SEL_MLP ? selector_device_weights(&wver) : nullptr;
  // (re)capture when the outputs, options or selector weights changed
  gm_graph *gg = (gm_graph *)w.gmode;
  if (!gg || gg->parent != d_parent || gg->depth != d_depth || gg->div != div || gg->cap_levels != cap_levels ||
      gg->t_wave != tw || gg->wts != wts || (wts && gg->wver != wver)) {
    gm_release(w);
    gg = new gm_graph();
    w.gmode = gg;
    BYO_HIP(hipStreamCreateWithFlags(&gg->cap, hipStreamNonBlocking));
    BYO_HIP(hipStreamBeginCapture(gg->cap, hipStreamCaptureModeThreadLocal));
    byo_status cs = BYO_OK;
    for (int L = 0; L < K && cs == BYO_OK; ++L) cs = enqueue_level(g, L & 1, d_parent, d_depth, ctr, st, div,
                                                                   cap_levels, tw, wts, gg->cap);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(gg->cap, &graph);
    if (cs != BYO_OK) return cs;
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture", __FILE__, __LINE__);
    e = hipGraphInstantiate(&gg->exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate", __FILE__, __LINE__);
    gg->parent = d_parent;
    gg->depth = d_depth;
    gg->div = div;
    gg->cap_levels = cap_levels;
    gg->t_wave = tw;
    gg->wts = wts;
    gg->wver = wver;
    gg->levels = K;
  }
  gm_state h;
  while (true) {
    BYO_HIP(hipGraphLaunch(gg->exec, s));
    BYO_TRY(sync_read(s, st, &h, sizeof(h)));
    if (h.done) break;
  }
  byo_run_stats r;
  std::memset(&r, 0, sizeof(r));
  r.levels = h.level + (h.prev_sel != GM_NONE ? 1 : 0);
  r.device_levels = r.levels;
  r.variant_count[BYO_V_PUSH_BUCKET] = (int64_t)h.push_levels;
  r.variant_count[BYO_V_PULL_WAVE] = (int64_t)h.pull_levels;
  r.reached = (int64_t)h.reached;
  r.edges = (int64_t)h.edges;
  if (stats) *stats = r;
  if (h.limit) return fail(BYO_ELIMIT, "BFS level cap reached");
  return BYO_OK;
}

}  // namespace byo
