// k-core decomposition (Table algs-list, substructure problems): the
// coreness of every vertex, the largest k such that the vertex belongs to the
// k-core (the maximal subgraph in which every vertex keeps at least k
// neighbours). Peeling, level-synchronous on the GPU:
//  - at a new k, the alive vertices with remaining degree <= k form the
//    frontier (one pass also finds the least remaining degree, so k jumps
//    straight to the next value that removes something);
//  - a sub-round removes the frontier (coreness k) with one edgeMap push: each
//    alive neighbour loses one remaining degree (atomic), and one that drops
//    from k + 1 to k joins the next frontier; sub-rounds repeat at the same k
//    until the frontier is empty.
// The push is edge-balanced when the frontier's degree sum is large: runs of
// KC_RUN consecutive edges of the frontier's concatenated lists per lane, so
// hubs (peeled late, in small frontiers) spread over the grid; a frontier
// with a small degree sum and no long list is removed one vertex per lane.
#include <algorithm>
#include <climits>
#include <cstring>

#include "internal.h"

namespace byo {

namespace {

constexpr int KC_BLOCK = 256;
constexpr int KC_RUN = 16;
// frontiers with a smaller degree sum take the lane kernel (the edge-balanced
// one costs a degree scan, 3 launches, per sub-round)
constexpr int64_t KC_EDGE_MIN = 1 << 15;
constexpr int64_t KC_LANE_MAX = 16;  // ... and no vertex of more neighbours than this (each decrement waits on an atomic)

// block maximum of v into *dst (atomic); every thread calls it
__device__ __forceinline__ void kc_block_max(unsigned long long v, unsigned long long *dst) {
  v = wave_max(v);
  __shared__ unsigned long long wm[KC_BLOCK / BYO_WAVE];
  __syncthreads();
  if (lane_id() == 0) wm[threadIdx.x / BYO_WAVE] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long b = wm[0];
    for (int i = 1; i < KC_BLOCK / BYO_WAVE; ++i) b = wm[i] > b ? wm[i] : b;
    if (b) atomicMax(dst, b);
  }
}

// remaining degree = degree, coreness unknown (-1: alive)
__global__ void kc_init_kernel(const int32_t *__restrict__ deg, int64_t n, int32_t *dcur, int32_t *core) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    dcur[v] = deg[v];
    core[v] = -1;
  }
}

// least remaining degree over alive vertices (ctr->aux1, as unsigned min) and
// their count (ctr->aux0)
__global__ void __launch_bounds__(KC_BLOCK) kc_min_kernel(const int32_t *__restrict__ dcur,
                                                          const int32_t *__restrict__ core, int64_t n,
                                                          byo_counters *ctr) {
  unsigned long long alive = 0, mn = ULLONG_MAX;
  for (int64_t v = (int64_t)blockIdx.x * KC_BLOCK + threadIdx.x; v < n; v += (int64_t)gridDim.x * KC_BLOCK)
    if (core[v] < 0) {
      ++alive;
      const unsigned long long d = (unsigned long long)dcur[v];
      mn = d < mn ? d : mn;
    }
  const unsigned long long a = block_sum<unsigned long long, KC_BLOCK>(alive);
  // block minimum through the wavefront minima
  unsigned long long m = mn;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const unsigned long long t = __shfl_xor(m, o);
    m = t < m ? t : m;
  }
  __shared__ unsigned long long wm[KC_BLOCK / BYO_WAVE];
  if (lane_id() == 0) wm[threadIdx.x / BYO_WAVE] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long b = wm[0];
    for (int i = 1; i < KC_BLOCK / BYO_WAVE; ++i) b = wm[i] < b ? wm[i] : b;
    if (a) atomicAdd(&ctr->aux0, a);
    if (b != ULLONG_MAX) atomicMin(&ctr->aux1, b);
  }
}

// frontier = alive vertices with remaining degree <= k (count, degree sum)
__global__ void __launch_bounds__(KC_BLOCK) kc_collect_kernel(const int32_t *__restrict__ dcur,
                                                              const int32_t *__restrict__ core,
                                                              const int32_t *__restrict__ deg, int64_t n, int32_t k,
                                                              int32_t *out, byo_counters *ctr) {
  unsigned long long degsum = 0, dmax = 0;
  for (int64_t base = (int64_t)blockIdx.x * KC_BLOCK; base < n; base += (int64_t)gridDim.x * KC_BLOCK) {
    const int64_t v = base + threadIdx.x;
    const bool take = v < n && core[v] < 0 && dcur[v] <= k;
    wave_append(take, (int32_t)v, out, &ctr->count);
    if (take) {
      degsum += (unsigned long long)deg[v];
      dmax = (unsigned long long)deg[v] > dmax ? (unsigned long long)deg[v] : dmax;
    }
  }
  const unsigned long long t = block_sum<unsigned long long, KC_BLOCK>(degsum);
  if (threadIdx.x == 0 && t) atomicAdd(&ctr->degsum, t);
  kc_block_max(dmax, &ctr->aux0);
}

// coreness k for the frontier (before any list is scanned)
__global__ void kc_mark_kernel(const int32_t *__restrict__ ids, int64_t kf, int32_t k, int32_t *core) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < kf; i += (int64_t)gridDim.x * blockDim.x)
    core[ids[i]] = k;
}

// last i in [0, kf) with scan[i] <= e
__device__ __forceinline__ int64_t kc_last_le(const long long *__restrict__ scan, int64_t kf, long long e) {
  int64_t lo = 0, hi = kf - 1;
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) >> 1;
    if (scan[mid] <= e) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Removal push, edge-balanced: every alive neighbour u of a frontier vertex
// loses one remaining degree; u joins the next frontier when it drops from
// k + 1 to k. The frontier's coreness is already written, so frontier
// vertices are not alive here.
__global__ void __launch_bounds__(KC_BLOCK) kc_peel_kernel(const int64_t *__restrict__ off,
                                                           const int32_t *__restrict__ nbr,
                                                           const int32_t *__restrict__ deg,
                                                           const int32_t *__restrict__ ids, int64_t kf,
                                                           const long long *__restrict__ scan, int32_t k,
                                                           int32_t *dcur, const int32_t *core, int32_t *out,
                                                           byo_counters *ctr, byo_counters *ctr_clear) {
  unsigned long long degsum = 0, dmax = 0;
  const long long total = scan[kf];
  const int64_t nthreads = (int64_t)gridDim.x * KC_BLOCK;
  // uniform trip count per workgroup: the emission ballots see every lane
  for (int64_t c0 = (int64_t)blockIdx.x * KC_BLOCK; c0 * KC_RUN < total; c0 += nthreads) {
    const int64_t c = c0 + threadIdx.x;
    const long long e0 = c * KC_RUN, e1 = e0 + KC_RUN < total ? e0 + KC_RUN : total;
    int64_t i = 0, base = 0;
    long long iend = 0;
    if (e0 < total) {
      i = kc_last_le(scan, kf, e0);
      const int32_t v = ids[i];
      base = off[v] - scan[i];
      iend = scan[i + 1];
    }
    for (long long e = e0; e < e0 + KC_RUN; ++e) {  // same trip count in every lane
      bool joins = false;
      int32_t u = 0;
      if (e < e1) {
        while (e >= iend) {
          ++i;
          const int32_t v = ids[i];
          base = off[v] - scan[i];
          iend = scan[i + 1];
        }
        u = nbr[base + e];
        if (core[u] < 0) joins = atomicSub(&dcur[u], 1) == k + 1;
      }
      wave_append(joins, u, out, &ctr->count);
      if (joins) {
        degsum += (unsigned long long)deg[u];
        dmax = (unsigned long long)deg[u] > dmax ? (unsigned long long)deg[u] : dmax;
      }
    }
  }
  const unsigned long long t = block_sum<unsigned long long, KC_BLOCK>(degsum);
  kc_block_max(dmax, &ctr->aux0);
  if (threadIdx.x == 0) {
    if (t) atomicAdd(&ctr->degsum, t);
    if (blockIdx.x == 0 && ctr_clear) {
      ctr_clear->count = 0;
      ctr_clear->degsum = 0;
      ctr_clear->aux0 = 0;
      ctr_clear->aux1 = ULLONG_MAX;
    }
  }
}

// Removal push, one lane per frontier vertex (a container without a parallel
// map): the lane walks its whole list.
__global__ void __launch_bounds__(KC_BLOCK) kc_peel_lane_kernel(const int64_t *__restrict__ off,
                                                                const int32_t *__restrict__ nbr,
                                                                const int32_t *__restrict__ deg,
                                                                const int32_t *__restrict__ ids, int64_t kf, int32_t k,
                                                                int32_t *dcur, const int32_t *core, int32_t *out,
                                                                byo_counters *ctr, byo_counters *ctr_clear) {
  unsigned long long degsum = 0, dmax = 0;
  for (int64_t i = (int64_t)blockIdx.x * KC_BLOCK + threadIdx.x; i - threadIdx.x < kf;
       i += (int64_t)gridDim.x * KC_BLOCK) {
    if (i < kf) {
      const int32_t v = ids[i];
      const int64_t end = off[v + 1];
      for (int64_t e = off[v]; e < end; ++e) {
        const int32_t u = nbr[e];
        const bool joins = core[u] < 0 && atomicSub(&dcur[u], 1) == k + 1;
        wave_append(joins, u, out, &ctr->count);
        if (joins) {
          degsum += (unsigned long long)deg[u];
          dmax = (unsigned long long)deg[u] > dmax ? (unsigned long long)deg[u] : dmax;
        }
      }
    }
  }
  const unsigned long long t = block_sum<unsigned long long, KC_BLOCK>(degsum);
  kc_block_max(dmax, &ctr->aux0);
  if (threadIdx.x == 0) {
    if (t) atomicAdd(&ctr->degsum, t);
    if (blockIdx.x == 0 && ctr_clear) {
      ctr_clear->count = 0;
      ctr_clear->degsum = 0;
      ctr_clear->aux0 = 0;
      ctr_clear->aux1 = ULLONG_MAX;
    }
  }
}

__global__ void kc_reset_kernel(byo_counters *ctr) {
  if (threadIdx.x < BYO_COUNTER_SLOTS) {
    ctr[threadIdx.x].count = 0;
    ctr[threadIdx.x].degsum = 0;
    ctr[threadIdx.x].aux0 = 0;
    ctr[threadIdx.x].aux1 = ULLONG_MAX;
  }
}

unsigned kc_grid(int64_t count, int64_t per, int64_t cap) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>((count + per - 1) / per, cap));
}

}  // namespace

}  // namespace byo

using namespace byo;

extern "C" byo_status byo_kcore(byo_graph *g, int32_t *d_core, const byo_opts *opts, void *stream,
                                byo_run_stats *stats) {
  BYO_CHECK(g && d_core, BYO_EINVAL, "null argument");
  byo_opts o;
  byo_opts_default(&o);
  if (opts) o = *opts;
  hipStream_t s = (hipStream_t)stream;
  const int64_t n = g->n;
  byo_run_stats st;
  std::memset(&st, 0, sizeof(st));
  if (n == 0) {
    if (stats) *stats = st;
    return BYO_OK;
  }
  BYO_TRY(ws_ensure_traversal(g));
  byo_workspace &w = g->ws;
  // remaining degrees, kept with the workspace
  if (!w.kc_dcur) BYO_HIP(hipMalloc(&w.kc_dcur, sizeof(int32_t) * (size_t)n));
  int32_t *dcur = w.kc_dcur;
  // Container-API ablation (Table api-components-avg): without degree() the
  // run starts from every list counted by a map, and uses those counts where
  // it needs degrees; without a parallel map a lane removes one vertex.
  const uint32_t omit = (uint32_t)o.api_omit;
  const bool par_map = !(omit & BYO_API_NO_PAR_MAP);
  const int32_t *degs = g->deg;
  if (omit & BYO_API_NO_DEGREE) {
    int32_t *mdeg = nullptr;
    BYO_TRY(api_map_degrees(g, omit, s, &mdeg));
    degs = mdeg;
  }
  kc_init_kernel<<<kc_grid(n, 256, 8192), 256, 0, s>>>(degs, n, dcur, d_core);
  kc_reset_kernel<<<1, 64, 0, s>>>(w.ctr);
  BYO_HIP(hipGetLastError());
  const int64_t cap = o.max_levels > 0 ? o.max_levels : INT64_MAX;
  int64_t remaining = n, k = -1, kf = 0, fdeg = 0, fmax = 0, edges = 0;
  int64_t slot = 0;  // counter slot of the next kernel that emits
  int cur = 0;
  int32_t rounds = 0;
  auto read = [&](int64_t sl, byo_counters *c) -> byo_status {
    BYO_HIP(hipMemcpyAsync(w.h_ctr + (sl % BYO_COUNTER_SLOTS), w.ctr + (sl % BYO_COUNTER_SLOTS), sizeof(byo_counters),
                           hipMemcpyDeviceToHost, s));
    BYO_HIP(hipStreamSynchronize(s));
    *c = w.h_ctr[sl % BYO_COUNTER_SLOTS];
    return BYO_OK;
  };
  while (remaining > 0) {
    if (kf == 0) {
      // next k: the least remaining degree among alive vertices (at least k + 1)
      byo_counters c;
      byo_counters *cs = w.ctr + (slot % BYO_COUNTER_SLOTS);
      kc_reset_kernel<<<1, 64, 0, s>>>(w.ctr);
      kc_min_kernel<<<kc_grid(n, KC_BLOCK, 4096), KC_BLOCK, 0, s>>>(dcur, d_core, n, cs);
      BYO_HIP(hipGetLastError());
      BYO_TRY(read(slot, &c));
      remaining = (int64_t)c.aux0;
      if (remaining == 0) break;
      k = std::max<int64_t>(k + 1, (int64_t)c.aux1);
      kc_reset_kernel<<<1, 64, 0, s>>>(w.ctr);
      kc_collect_kernel<<<kc_grid(n, KC_BLOCK, 4096), KC_BLOCK, 0, s>>>(dcur, d_core, degs, n, (int32_t)k,
                                                                         w.ids[cur], w.ctr + (slot % BYO_COUNTER_SLOTS));
      BYO_HIP(hipGetLastError());
      BYO_TRY(read(slot, &c));
      ++slot;
      kf = (int64_t)c.count;
      fdeg = (int64_t)c.degsum;
      fmax = (int64_t)c.aux0;
    }
    if (rounds >= cap) {
      if (stats) *stats = st;
      return fail(BYO_ELIMIT, "k-core round cap reached");
    }
    // remove the frontier at coreness k
    kc_mark_kernel<<<kc_grid(kf, 256, 8192), 256, 0, s>>>(w.ids[cur], kf, (int32_t)k, d_core);
    byo_counters *cs = w.ctr + (slot % BYO_COUNTER_SLOTS);
    const bool balanced = par_map && (fdeg >= KC_EDGE_MIN || fmax > KC_LANE_MAX);
    if (balanced) {
      BYO_TRY(scan_degrees(degs, w.ids[cur], kf, w.scan, w.partial, w.partial_cap, s));
      kc_peel_kernel<<<kc_grid((fdeg + KC_RUN - 1) / KC_RUN, KC_BLOCK, 16384), KC_BLOCK, 0, s>>>(
          g->off, g->nbr, degs, w.ids[cur], kf, w.scan, (int32_t)k, dcur, d_core, w.ids[1 - cur], cs,
          w.ctr + ((slot + 2) % BYO_COUNTER_SLOTS));
    } else {
      kc_peel_lane_kernel<<<kc_grid(kf, KC_BLOCK, 16384), KC_BLOCK, 0, s>>>(
          g->off, g->nbr, degs, w.ids[cur], kf, (int32_t)k, dcur, d_core, w.ids[1 - cur], cs,
          w.ctr + ((slot + 2) % BYO_COUNTER_SLOTS));
    }
    BYO_HIP(hipGetLastError());
    byo_counters c;
    BYO_TRY(read(slot, &c));
    ++slot;
    ++rounds;
    st.variant_count[balanced ? BYO_V_PUSH_EDGE : BYO_V_PUSH_THREAD]++;
    edges += fdeg;
    remaining -= kf;
    cur = 1 - cur;
    kf = (int64_t)c.count;
    fdeg = (int64_t)c.degsum;
    fmax = (int64_t)c.aux0;
  }
  st.levels = rounds;
  st.reached = n;
  st.edges = edges;
  if (stats) *stats = st;
  return BYO_OK;
}
