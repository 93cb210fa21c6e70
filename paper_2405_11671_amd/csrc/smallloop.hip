// Device-resident BFS levels for small frontiers. High-diameter graphs (road
// networks, lattices) spend thousands of levels with a few thousand frontier
// vertices each; there a host round trip per level (launch, counter copy,
// sync) costs more than the level itself. One workgroup of 1024 threads runs
// consecutive push levels on its own, with the frontier double-buffered in
// LDS and mirrored to global memory, and `__syncthreads()` as the level
// barrier. It returns to the host when the frontier is empty, when the next
// frontier (or its edge count) exceeds the caps -- the full-GPU kernels take
// over from the global copy -- or after max_levels levels, so the host keeps
// its level cap and statistics. Every wait is a workgroup barrier that all
// threads reach, so the kernel always finishes.
#include "internal.h"

namespace byo {

constexpr int SL_THREADS = 1024;
constexpr int SL_QCAP = 8192;      // LDS queue capacity per side (vertices)

struct small_loop_result {
  int32_t levels;                  // levels completed (each emitted a non-empty frontier, or the last one empty)
  int32_t side;                    // which global buffer holds the final frontier (0 = out0, 1 = out1)
  int32_t empty;                   // 1 if the final frontier is empty (BFS finished)
  int32_t pad;
  unsigned long long count;        // size of the final frontier
  unsigned long long degsum;       // sum of its degrees
  unsigned long long reached;      // vertices emitted over all levels run
  unsigned long long edges;        // sum of their degrees
};

__global__ void __launch_bounds__(SL_THREADS) bfs_small_loop_kernel(
    const int64_t *__restrict__ off, const int32_t *__restrict__ nbr, const int32_t *__restrict__ deg,
    int32_t *__restrict__ parent, int32_t *__restrict__ depth, uint64_t *__restrict__ visited,
    const int32_t *__restrict__ in_ids, int32_t k0, int32_t level0, int32_t max_levels, int32_t cap_count,
    long long cap_edges, int32_t *__restrict__ out0, int32_t *__restrict__ out1, small_loop_result *__restrict__ res) {
  __shared__ int32_t q[2][SL_QCAP];
  __shared__ unsigned s_cnt[2];
  const int t = threadIdx.x;
  for (int i = t; i < k0; i += SL_THREADS) q[0][i] = in_ids[i];
  if (t == 0) {
    s_cnt[0] = (unsigned)k0;
    s_cnt[1] = 0;
  }
  __syncthreads();
  int cur = 0;
  unsigned long long reached = 0, edges = 0, last_ds = 0;
  int levels = 0;
  int empty = 0, side = 0;
  unsigned k = (unsigned)k0;
  for (int L = 0; L < max_levels; ++L) {
    int nx = 1 - cur;
    int32_t *gout = (L & 1) ? out1 : out0;
    int32_t newdepth = level0 + L + 1;
    unsigned long long mydeg = 0;
    // thread-per-vertex for short lists; wavefront-cooperative for long ones
    for (unsigned base = 0; base < k; base += SL_THREADS) {
      unsigned i = base + t;
      int32_t u = -1;
      int64_t b = 0, e = 0;
      if (i < k) {
        u = q[cur][i];
        b = off[u];
        e = off[u + 1];
      }
      bool wide = u >= 0 && e - b > 32;
      if (u >= 0 && !wide) {
        for (int64_t x = b; x < e; ++x) {
          int32_t v = nbr[x];
          uint64_t bit = 1ull << (v & 63);
          if (visited[v >> 6] & bit) continue;
          if (atomicCAS(&parent[v], -1, u) != -1) continue;
          depth[v] = newdepth;
          atomicOr((unsigned long long *)&visited[v >> 6], (unsigned long long)bit);
          unsigned pos = atomicAdd(&s_cnt[nx], 1u);
          if (pos < SL_QCAP) q[nx][pos] = v;
          gout[pos] = v;
          mydeg += (unsigned long long)deg[v];
        }
      }
      uint64_t wm = __ballot(wide);
      while (wm) {
        int l = __ffsll((long long)wm) - 1;
        wm &= wm - 1;
        int32_t wu = read_lane_i32(u, l);
        int64_t wb = (int64_t)read_lane_u64((uint64_t)b, l), we = (int64_t)read_lane_u64((uint64_t)e, l);
        for (int64_t x = wb + lane_id(); x < we; x += BYO_WAVE) {
          int32_t v = nbr[x];
          uint64_t bit = 1ull << (v & 63);
          if (visited[v >> 6] & bit) continue;
          if (atomicCAS(&parent[v], -1, wu) != -1) continue;
          depth[v] = newdepth;
          atomicOr((unsigned long long *)&visited[v >> 6], (unsigned long long)bit);
          unsigned pos = atomicAdd(&s_cnt[nx], 1u);
          if (pos < SL_QCAP) q[nx][pos] = v;
          gout[pos] = v;
          mydeg += (unsigned long long)deg[v];
        }
      }
    }
    unsigned long long ds = block_sum<unsigned long long, SL_THREADS>(mydeg);
    __syncthreads();
    unsigned kn = s_cnt[nx];
    levels = L + 1;
    side = L & 1;
    reached += kn;
    edges += ds;
    last_ds = ds;
    if (kn == 0) {
      empty = 1;
      k = 0;
      break;
    }
    k = kn;
    if ((int)kn > cap_count || (long long)ds > cap_edges || kn > (unsigned)SL_QCAP) break;
    __syncthreads();
    if (t == 0) s_cnt[cur] = 0;  // becomes the next level's output counter
    __syncthreads();
    cur = nx;
  }
  if (t == 0) {
    res->levels = levels;
    res->side = side;
    res->empty = empty;
    res->count = k;
    res->degsum = empty ? 0ull : last_ds;
    res->reached = reached;
    res->edges = edges;
  }
}

byo_status bfs_small_loop(byo_graph *g, const int32_t *in_ids, int64_t k, int32_t level, int32_t max_levels,
                          int32_t cap_count, int64_t cap_edges, int32_t *parent, int32_t *depth, uint64_t *visited,
                          int32_t *out0, int32_t *out1, void *d_res, hipStream_t s, small_loop_out *out) {
  BYO_CHECK(k >= 1 && k <= SL_QCAP, BYO_EINVAL, "small-frontier loop needs 1 <= |U| <= queue capacity");
  if (cap_count > SL_QCAP) cap_count = SL_QCAP;
  {
    ktimer_scope kt(BYO_K_SMALL_LOOP, s);
    bfs_small_loop_kernel<<<1, SL_THREADS, 0, s>>>(g->off, g->nbr, g->deg, parent, depth, visited, in_ids, (int32_t)k,
                                                   level, max_levels, cap_count, cap_edges, out0, out1,
                                                   (small_loop_result *)d_res);
  }
  BYO_HIP(hipGetLastError());
  small_loop_result r;
  BYO_TRY(sync_read(s, d_res, &r, sizeof(r)));
  out->levels = r.levels;
  out->side = r.side;
  out->empty = r.empty != 0;
  out->count = (int64_t)r.count;
  out->degsum = (int64_t)r.degsum;
  out->reached = (int64_t)r.reached;
  out->edges = (int64_t)r.edges;
  return BYO_OK;
}

}  // namespace byo
