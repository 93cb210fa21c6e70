// Approximate densest subgraph (Table algs-list, substructure problems):
// peeling rounds. S starts as every vertex; each round measures |S| and
// |E(S)| (half the sum of the degrees inside S), keeps the best density seen,
// and removes every vertex of S with fewer than 2 (1 + eps) |E(S)| / |S|
// neighbours in S: a mark pass on the round's degrees, then a push that
// takes the removed vertices off their surviving neighbours' degrees. The
// best set is within 2 (1 + eps) of the densest; the rounds are
// deterministic, and the threshold test uses the same FP64 expression as the
// host computes, so the result is exact against a sequential run.
#include <algorithm>
#include <cstring>

#include "internal.h"

namespace byo {

namespace {

constexpr int DS_BLOCK = 256;
constexpr int32_t DS_WAVE_MIN = 32;

__global__ void ds_init_kernel(const int32_t *__restrict__ deg, int64_t n, int32_t *dS, uint8_t *alive) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    dS[v] = deg[v];
    alive[v] = 1;
  }
}

// |S| into ctr->count, the sum of degrees inside S into ctr->degsum
__global__ void __launch_bounds__(DS_BLOCK) ds_count_kernel(const int32_t *__restrict__ dS,
                                                            const uint8_t *__restrict__ alive, int64_t n,
                                                            byo_counters *ctr) {
  unsigned long long s = 0, e2 = 0;
  for (int64_t v = (int64_t)blockIdx.x * DS_BLOCK + threadIdx.x; v < n; v += (int64_t)gridDim.x * DS_BLOCK)
    if (alive[v]) {
      ++s;
      e2 += (unsigned long long)dS[v];
    }
  const unsigned long long ts = block_sum<unsigned long long, DS_BLOCK>(s);
  const unsigned long long te = block_sum<unsigned long long, DS_BLOCK>(e2);
  if (threadIdx.x == 0) {
    if (ts) atomicAdd(&ctr->count, ts);
    if (te) atomicAdd(&ctr->degsum, te);
  }
}

// the vertices of S below the threshold leave S (listed in out, count in
// ctr->aux0); decided on the round's degrees, before any decrement
__global__ void __launch_bounds__(DS_BLOCK) ds_mark_kernel(const int32_t *__restrict__ dS, uint8_t *alive, int64_t n,
                                                           double thr, int32_t *out, byo_counters *ctr) {
  for (int64_t base = (int64_t)blockIdx.x * DS_BLOCK; base < n; base += (int64_t)gridDim.x * DS_BLOCK) {
    const int64_t v = base + threadIdx.x;
    const bool drop = v < n && alive[v] && (double)dS[v] < thr;
    if (drop) alive[v] = 0;
    wave_append(drop, (int32_t)v, out, &ctr->aux0);
  }
}

// every removed vertex is taken off its surviving neighbours' degrees; with a
// list longer than DS_WAVE_MIN the wavefront shares it
__global__ void __launch_bounds__(DS_BLOCK) ds_peel_kernel(const int64_t *__restrict__ off,
                                                           const int32_t *__restrict__ nbr,
                                                           const int32_t *__restrict__ ids, int64_t k,
                                                           const uint8_t *__restrict__ alive, int32_t *dS) {
  for (int64_t base = (int64_t)blockIdx.x * DS_BLOCK; base < k; base += (int64_t)gridDim.x * DS_BLOCK) {
    const int64_t i = base + threadIdx.x;
    int64_t beg = 0, end = 0;
    if (i < k) {
      const int32_t v = ids[i];
      beg = off[v];
      end = off[v + 1];
    }
    const bool coop = end - beg > DS_WAVE_MIN;
    if (i < k && !coop)
      for (int64_t e = beg; e < end; ++e) {
        const int32_t u = nbr[e];
        if (alive[u]) atomicSub(&dS[u], 1);
      }
    uint64_t pm = __ballot(i < k && coop);
    while (pm) {
      const int l = __ffsll((long long)pm) - 1;
      pm &= pm - 1;
      const int64_t lb = (int64_t)read_lane_u64((uint64_t)beg, l), le = (int64_t)read_lane_u64((uint64_t)end, l);
      for (int64_t e = lb + lane_id(); e < le; e += BYO_WAVE) {
        const int32_t u = nbr[e];
        if (alive[u]) atomicSub(&dS[u], 1);
      }
    }
  }
}

__global__ void ds_reset_kernel(byo_counters *ctr) {
  if (threadIdx.x == 0) {
    ctr->count = 0;
    ctr->degsum = 0;
    ctr->aux0 = 0;
    ctr->aux1 = 0;
  }
}

unsigned ds_grid(int64_t count, int64_t per, int64_t cap) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>((count + per - 1) / per, cap));
}

}  // namespace

}  // namespace byo

using namespace byo;

extern "C" byo_status byo_densest(byo_graph *g, double eps, uint8_t *d_in_best, int64_t *best_edges,
                                  int64_t *best_vertices, const byo_opts *opts, void *stream, byo_run_stats *stats) {
  BYO_CHECK(g && best_edges && best_vertices, BYO_EINVAL, "null argument");
  BYO_CHECK(eps >= 0.0 && eps < 1e6, BYO_EINVAL, "eps outside [0, 1e6)");
  byo_opts o;
  byo_opts_default(&o);
  if (opts) o = *opts;
  hipStream_t s = (hipStream_t)stream;
  const int64_t n = g->n;
  byo_run_stats st;
  std::memset(&st, 0, sizeof(st));
  *best_edges = 0;
  *best_vertices = n > 0 ? n : 1;
  if (n == 0) {
    if (stats) *stats = st;
    return BYO_OK;
  }
  BYO_TRY(ws_ensure_traversal(g));
  byo_workspace &w = g->ws;
  if (!w.ds_deg) BYO_HIP(hipMalloc(&w.ds_deg, sizeof(int32_t) * (size_t)n));
  if (!w.ds_alive) BYO_HIP(hipMalloc(&w.ds_alive, (size_t)n));
  int32_t *dS = w.ds_deg;
  uint8_t *alive = w.ds_alive;
  ds_init_kernel<<<ds_grid(n, 256, 8192), 256, 0, s>>>(g->deg, n, dS, alive);
  BYO_HIP(hipGetLastError());
  if (d_in_best) BYO_HIP(hipMemcpyAsync(d_in_best, alive, (size_t)n, hipMemcpyDeviceToDevice, s));
  const int64_t cap = o.max_levels > 0 ? o.max_levels : n + 1;
  byo_counters *c = w.ctr;
  int64_t S = n;
  int32_t rounds = 0;
  while (S > 0) {
    if (rounds >= cap) {
      if (stats) *stats = st;
      return fail(BYO_ELIMIT, "densest-subgraph round cap reached");
    }
    ds_reset_kernel<<<1, 64, 0, s>>>(c);
    ds_count_kernel<<<ds_grid(n, DS_BLOCK, 4096), DS_BLOCK, 0, s>>>(dS, alive, n, c);
    BYO_HIP(hipGetLastError());
    byo_counters h;
    BYO_TRY(sync_read(s, c, &h, sizeof(h)));
    S = (int64_t)h.count;
    const int64_t E = (int64_t)(h.degsum / 2);
    ++rounds;
    if (S == 0) break;
    // E / S > best, compared exactly
    if ((__int128)E * (__int128)(*best_vertices) > (__int128)(*best_edges) * (__int128)S) {
      *best_edges = E;
      *best_vertices = S;
      if (d_in_best) BYO_HIP(hipMemcpyAsync(d_in_best, alive, (size_t)n, hipMemcpyDeviceToDevice, s));
    }
    if (E == 0) break;
    const double thr = 2.0 * (1.0 + eps) * ((double)E / (double)S);
    ds_reset_kernel<<<1, 64, 0, s>>>(c);
    ds_mark_kernel<<<ds_grid(n, DS_BLOCK, 4096), DS_BLOCK, 0, s>>>(dS, alive, n, thr, w.ids[0], c);
    BYO_HIP(hipGetLastError());
    BYO_TRY(sync_read(s, c, &h, sizeof(h)));
    const int64_t k = (int64_t)h.aux0;
    if (k == 0) break;  // a round that removes nothing leaves S as it is
    ds_peel_kernel<<<ds_grid(k, DS_BLOCK, 16384), DS_BLOCK, 0, s>>>(g->off, g->nbr, w.ids[0], k, alive, dS);
    BYO_HIP(hipGetLastError());
    st.variant_count[BYO_V_PUSH_WAVE]++;
    S -= k;
  }
  BYO_HIP(hipStreamSynchronize(s));
  st.levels = rounds;
  st.reached = n;
  if (stats) *stats = st;
  return BYO_OK;
}
