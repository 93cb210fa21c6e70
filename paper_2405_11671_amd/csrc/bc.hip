// Single-source betweenness (Table algs-list, shortest-path problems): the
// dependency of the source s on every vertex, delta(v) = sum over targets t of
// sigma_st(v) / sigma_st (Brandes' dependency), from edgeMap passes:
//  - forward: a level-synchronous BFS that also counts shortest paths,
//    sigma(v) = sum of sigma(u) over neighbours u one level closer. Push (a
//    vertex is claimed by the CAS of its depth; every frontier neighbour then
//    adds its count, FP64 atomics) or pull (an unvisited vertex sums the counts
//    of its frontier neighbours), chosen per level by the sparse/dense cutoff.
//    Each level's vertices are appended to one order array, so the levels
//    stay available for the backward pass;
//  - backward: from the deepest level up, one pull per level over that
//    level's vertices: delta(v) = sigma(v) * sum over children w (neighbours
//    one level deeper) of coef(w), coef(w) = (1 + delta(w)) / sigma(w).
// Path counts are integers, exact in FP64 below 2^53, so their summation
// order does not matter there. The backward sums run in a fixed order in the
// lane and wavefront kernels; the edge-balanced one (the default, for skewed
// levels) adds per-run partials with FP64 atomics, so its rounding order
// varies from run to run.
#include <algorithm>
#include <cstring>
#include <vector>

#include "internal.h"

namespace byo {

namespace {

constexpr int BC_BLOCK = 256;
constexpr int32_t BC_WAVE_MIN = 32;  // lists longer than this are shared by the wavefront
constexpr int BC_ILP = 8;            // neighbours whose loads a lane issues together

// sum over e in [beg, end) of val[nbr[e]] where keep(nbr[e]), ascending, with
// BC_ILP neighbour loads, then their probes, then their values in flight
template <typename Keep>
__device__ __forceinline__ double bc_lane_sum(const int32_t *__restrict__ nbr, int64_t beg, int64_t end,
                                              const double *__restrict__ val, Keep keep) {
  double s = 0.0;
  for (int64_t e = beg; e < end; e += BC_ILP) {
    int32_t u[BC_ILP];
    bool k[BC_ILP];
    double x[BC_ILP];
#pragma unroll
    for (int j = 0; j < BC_ILP; ++j) u[j] = e + j < end ? nbr[e + j] : -1;
#pragma unroll
    for (int j = 0; j < BC_ILP; ++j) k[j] = u[j] >= 0 && keep(u[j]);
#pragma unroll
    for (int j = 0; j < BC_ILP; ++j) x[j] = k[j] ? val[u[j]] : 0.0;
#pragma unroll
    for (int j = 0; j < BC_ILP; ++j) s += x[j];
  }
  return s;
}

// the same over a list shared by the wavefront: lane l takes entries l, l+64,
// ... four at a time; the partial sums are reduced by the caller
template <typename Keep>
__device__ __forceinline__ double bc_wave_part(const int32_t *__restrict__ nbr, int64_t beg, int64_t end,
                                               const double *__restrict__ val, Keep keep) {
  double s = 0.0;
  for (int64_t e0 = beg + lane_id(); e0 < end; e0 += 4 * BYO_WAVE) {
    int32_t u[4];
    bool k[4];
    double x[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) u[j] = e0 + j * BYO_WAVE < end ? nbr[e0 + j * BYO_WAVE] : -1;
#pragma unroll
    for (int j = 0; j < 4; ++j) k[j] = u[j] >= 0 && keep(u[j]);
#pragma unroll
    for (int j = 0; j < 4; ++j) x[j] = k[j] ? val[u[j]] : 0.0;
#pragma unroll
    for (int j = 0; j < 4; ++j) s += x[j];
  }
  return s;
}

struct BcFwd {
  const int64_t *__restrict__ off;
  const int32_t *__restrict__ nbr;
  const int32_t *__restrict__ deg;
  const int32_t *__restrict__ in_ids;   // frontier (level L), k entries
  const uint64_t *__restrict__ in_bits;
  int64_t k, n, words;
  int32_t *depth;
  double *sigma;
  uint64_t *visited;
  int32_t *out_ids;                     // level L + 1 is appended here
  uint64_t *out_bits;
  byo_counters *ctr, *ctr_clear;
  int32_t level;                        // L
};

__device__ __forceinline__ void bc_finish(byo_counters *ctr, byo_counters *ctr_clear, unsigned long long degsum) {
  const unsigned long long t = block_sum<unsigned long long, BC_BLOCK>(degsum);
  if (threadIdx.x == 0) {
    if (t) atomicAdd(&ctr->degsum, t);
    if (blockIdx.x == 0 && ctr_clear) {
      ctr_clear->count = 0;
      ctr_clear->degsum = 0;
      ctr_clear->aux0 = 0;
      ctr_clear->aux1 = 0;
    }
  }
}

// u's count reaches neighbour v: claim v for level L+1 if unvisited, then add
// when v is at level L+1 (claimed now or earlier in this level)
__device__ __forceinline__ bool bc_relax(const BcFwd &a, int32_t v, double su) {
  int32_t d = a.depth[v];
  bool claimed = false;
  if (d == -1) {
    const int32_t old = atomicCAS(&a.depth[v], -1, a.level + 1);
    claimed = old == -1;
    d = claimed ? a.level + 1 : old;
  }
  if (d == a.level + 1) atomicAdd(&a.sigma[v], su);
  return claimed;
}

__device__ __forceinline__ void bc_emit(const BcFwd &a, bool claimed, int32_t v, unsigned long long &degsum) {
  wave_append(claimed, v, a.out_ids, &a.ctr->count);
  if (claimed) {
    atomicOr((unsigned long long *)&a.visited[v >> 6], 1ull << (v & 63));
    atomicOr((unsigned long long *)&a.out_bits[v >> 6], 1ull << (v & 63));
    degsum += (unsigned long long)a.deg[v];
  }
}

// Push: lane per frontier vertex; with WAVE a list longer than BC_WAVE_MIN is
// relaxed by the whole wavefront, 64 neighbours at a time.
template <bool WAVE>
__global__ void __launch_bounds__(BC_BLOCK) bc_push_kernel(BcFwd a) {
  unsigned long long degsum = 0;
  for (int64_t base = (int64_t)blockIdx.x * BC_BLOCK; base < a.k; base += (int64_t)gridDim.x * BC_BLOCK) {
    const int64_t i = base + threadIdx.x;
    int32_t u = 0;
    int64_t beg = 0, end = 0;
    double su = 0.0;
    if (i < a.k) {
      u = a.in_ids[i];
      beg = a.off[u];
      end = a.off[u + 1];
      su = a.sigma[u];
    }
    const bool coop = WAVE && end - beg > BC_WAVE_MIN;
    if (!coop)
      for (int64_t e = beg; e < end; e += BC_ILP) {
        // BC_ILP neighbours and their depths in flight, then the claims and adds
        int32_t v[BC_ILP], d[BC_ILP];
        bool claimed[BC_ILP];
#pragma unroll
        for (int j = 0; j < BC_ILP; ++j) v[j] = e + j < end ? a.nbr[e + j] : -1;
#pragma unroll
        for (int j = 0; j < BC_ILP; ++j) d[j] = v[j] >= 0 ? a.depth[v[j]] : -2;
#pragma unroll
        for (int j = 0; j < BC_ILP; ++j) {
          claimed[j] = false;
          if (d[j] == -1) {
            const int32_t old = atomicCAS(&a.depth[v[j]], -1, a.level + 1);
            claimed[j] = old == -1;
            d[j] = claimed[j] ? a.level + 1 : old;
          }
        }
#pragma unroll
        for (int j = 0; j < BC_ILP; ++j)
          if (d[j] == a.level + 1) atomicAdd(&a.sigma[v[j]], su);
#pragma unroll
        for (int j = 0; j < BC_ILP; ++j) bc_emit(a, claimed[j], v[j], degsum);
      }
    if (WAVE) {
      uint64_t pm = __ballot(coop);
      while (pm) {
        const int l = __ffsll((long long)pm) - 1;
        pm &= pm - 1;
        const int64_t lb = (int64_t)read_lane_u64((uint64_t)beg, l), le = (int64_t)read_lane_u64((uint64_t)end, l);
        const double sl = __shfl(su, l);
        for (int64_t e0 = lb; e0 < le; e0 += BYO_WAVE) {
          const int64_t e = e0 + lane_id();
          bool claimed = false;
          int32_t v = 0;
          if (e < le) {
            v = a.nbr[e];
            claimed = bc_relax(a, v, sl);
          }
          bc_emit(a, claimed, v, degsum);
        }
      }
    }
  }
  bc_finish(a.ctr, a.ctr_clear, degsum);
}

// Pull: a wavefront per 64-vertex word; an unvisited vertex sums the counts
// of its frontier neighbours (all of them: no early exit). With WAVE a list
// longer than BC_WAVE_MIN is summed by the wavefront.
template <bool WAVE>
__global__ void __launch_bounds__(BC_BLOCK) bc_pull_kernel(BcFwd a) {
  unsigned long long degsum = 0;
  const int64_t nwaves = (int64_t)gridDim.x * (BC_BLOCK / BYO_WAVE);
  for (int64_t w = (int64_t)xcd_block(blockIdx.x, gridDim.x) * (BC_BLOCK / BYO_WAVE) + threadIdx.x / BYO_WAVE;
       w < a.words; w += nwaves) {
    const uint64_t vis = a.visited[w];
    if (vis == ~0ull) {
      if (lane_id() == 0) a.out_bits[w] = 0ull;
      continue;
    }
    const int64_t v64 = w * 64 + lane_id();
    const bool cand = v64 < a.n && !((vis >> lane_id()) & 1ull);
    int64_t beg = 0, end = 0;
    double s = 0.0;
    if (cand) {
      beg = a.off[v64];
      end = a.off[v64 + 1];
    }
    const bool coop = WAVE && end - beg > BC_WAVE_MIN;
    auto in_u = [&](int32_t u) { return ((a.in_bits[u >> 6] >> (u & 63)) & 1ull) != 0; };
    if (cand && !coop) s = bc_lane_sum(a.nbr, beg, end, a.sigma, in_u);
    if (WAVE) {
      uint64_t pm = __ballot(cand && coop);
      while (pm) {
        const int l = __ffsll((long long)pm) - 1;
        pm &= pm - 1;
        const int64_t lb = (int64_t)read_lane_u64((uint64_t)beg, l), le = (int64_t)read_lane_u64((uint64_t)end, l);
        double part = wave_sum(bc_wave_part(a.nbr, lb, le, a.sigma, in_u));
        if (lane_id() == l) s = part;
      }
    }
    const bool found = s > 0.0;
    if (found) {
      a.depth[v64] = a.level + 1;
      a.sigma[v64] = s;
      degsum += (unsigned long long)a.deg[v64];
    }
    const uint64_t m = __ballot(found);
    unsigned long long b = 0;
    if (lane_id() == 0) {
      a.out_bits[w] = m;
      if (m) {
        a.visited[w] = vis | m;
        b = atomicAdd(&a.ctr->count, (unsigned long long)__popcll(m));
      }
    }
    b = read_lane_u64(b, 0);
    if (found) a.out_ids[b + __popcll(m & lanemask_lt())] = (int32_t)v64;
  }
  bc_finish(a.ctr, a.ctr_clear, degsum);
}

// Backward pass over one level's vertices ids[0..k): delta(v) = sigma(v) *
// sum of coef(w) over neighbours w at level L + 1 (ascending, or lane-strided
// then reduced for long lists), coef(v) = (1 + delta(v)) / sigma(v).
template <bool WAVE>
__global__ void __launch_bounds__(BC_BLOCK) bc_back_kernel(const int64_t *__restrict__ off,
                                                           const int32_t *__restrict__ nbr,
                                                           const int32_t *__restrict__ ids, int64_t k,
                                                           const int32_t *__restrict__ depth,
                                                           const double *__restrict__ sigma, double *__restrict__ coef,
                                                           double *__restrict__ delta, int32_t level) {
  for (int64_t base = (int64_t)blockIdx.x * BC_BLOCK; base < k; base += (int64_t)gridDim.x * BC_BLOCK) {
    const int64_t i = base + threadIdx.x;
    int32_t v = 0;
    int64_t beg = 0, end = 0;
    if (i < k) {
      v = ids[i];
      beg = off[v];
      end = off[v + 1];
    }
    const bool coop = WAVE && end - beg > BC_WAVE_MIN;
    auto child = [&](int32_t w) { return depth[w] == level + 1; };
    double acc = 0.0;
    if (i < k && !coop) acc = bc_lane_sum(nbr, beg, end, coef, child);
    if (WAVE) {
      uint64_t pm = __ballot(i < k && coop);
      while (pm) {
        const int l = __ffsll((long long)pm) - 1;
        pm &= pm - 1;
        const int64_t lb = (int64_t)read_lane_u64((uint64_t)beg, l), le = (int64_t)read_lane_u64((uint64_t)end, l);
        const double part = wave_sum(bc_wave_part(nbr, lb, le, coef, child));
        if (lane_id() == l) acc = part;
      }
    }
    if (i < k) {
      const double sv = sigma[v];
      const double dv = sv * acc;
      delta[v] = dv;
      coef[v] = (1.0 + dv) / sv;
    }
  }
}

// last i in [0, k) with scan[i] <= e (scan nondecreasing, scan[0] = 0 <= e)
__device__ __forceinline__ int64_t bc_last_le(const long long *__restrict__ scan, int64_t k, long long e) {
  int64_t lo = 0, hi = k - 1;
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) >> 1;
    if (scan[mid] <= e) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

constexpr int BC_RUN = 16;  // consecutive edges per lane in the edge-balanced passes
// below this degree sum a level takes the lane/wavefront forms: the
// edge-balanced passes cost a degree scan (3 launches) per level, which
// dominates on long chains of small levels (lattices)
constexpr int64_t BC_EDGE_MIN = 1 << 15;

// Edge-balanced push: the frontier's lists, concatenated (scan = exclusive
// scan of their degrees, scan[k] = total), in runs of BC_RUN edges per lane.
__global__ void __launch_bounds__(BC_BLOCK) bc_push_edges_kernel(BcFwd a, const long long *__restrict__ scan) {
  unsigned long long degsum = 0;
  const long long total = scan[a.k];  // the grid was sized from the host's copy
  const int64_t nthreads = (int64_t)gridDim.x * BC_BLOCK;
  for (int64_t c = (int64_t)blockIdx.x * BC_BLOCK + threadIdx.x; c * BC_RUN < total; c += nthreads) {
    const long long e0 = c * BC_RUN, e1 = e0 + BC_RUN < total ? e0 + BC_RUN : total;
    int64_t i = bc_last_le(scan, a.k, e0);
    int32_t u = a.in_ids[i];
    double su = a.sigma[u];
    long long iend = scan[i + 1];
    int64_t base = a.off[u] - scan[i];
    for (long long e = e0; e < e1; ++e) {
      while (e >= iend) {  // next frontier vertex with edges
        ++i;
        u = a.in_ids[i];
        su = a.sigma[u];
        base = a.off[u] - scan[i];
        iend = scan[i + 1];
      }
      const int32_t v = a.nbr[base + e];
      bc_emit(a, bc_relax(a, v, su), v, degsum);
    }
  }
  bc_finish(a.ctr, a.ctr_clear, degsum);
}

// Edge-balanced backward pass over one level's vertices ids[0..k): each run of
// BC_RUN edges adds, per vertex it touches, the coef of the children it meets
// into acc[v] (acc = delta, zero until the level is finished).
__global__ void __launch_bounds__(BC_BLOCK) bc_back_edges_kernel(const int64_t *__restrict__ off,
                                                                 const int32_t *__restrict__ nbr,
                                                                 const int32_t *__restrict__ ids, int64_t k,
                                                                 const long long *__restrict__ scan,
                                                                 const int32_t *__restrict__ depth,
                                                                 const double *__restrict__ coef, double *acc,
                                                                 int32_t level) {
  const long long total = scan[k];
  const int64_t nthreads = (int64_t)gridDim.x * BC_BLOCK;
  for (int64_t c = (int64_t)blockIdx.x * BC_BLOCK + threadIdx.x; c * BC_RUN < total; c += nthreads) {
    const long long e0 = c * BC_RUN, e1 = e0 + BC_RUN < total ? e0 + BC_RUN : total;
    int64_t i = bc_last_le(scan, k, e0);
    int32_t v = ids[i];
    long long iend = scan[i + 1];
    int64_t base = off[v] - scan[i];
    double part = 0.0;
    for (long long e = e0; e < e1; e += 4) {
      int32_t w[4];
      int32_t owner[4];
      bool kid[4];
      double x[4];
      // resolve the owners first (usually one), then the four loads in flight
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        owner[j] = -1;
        w[j] = -1;
        if (e + j < e1) {
          while (e + j >= iend) {
            if (part != 0.0) atomicAdd(&acc[v], part);
            part = 0.0;
            ++i;
            v = ids[i];
            base = off[v] - scan[i];
            iend = scan[i + 1];
          }
          owner[j] = v;
          w[j] = nbr[base + e + j];
        }
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) kid[j] = w[j] >= 0 && depth[w[j]] == level + 1;
#pragma unroll
      for (int j = 0; j < 4; ++j) x[j] = kid[j] ? coef[w[j]] : 0.0;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        if (owner[j] >= 0 && owner[j] != v) {
          // an earlier entry of this group belongs to an earlier vertex
          if (x[j] != 0.0) atomicAdd(&acc[owner[j]], x[j]);
        } else {
          part += x[j];
        }
      }
    }
    if (part != 0.0) atomicAdd(&acc[v], part);
  }
}

// delta(v) = sigma(v) * acc(v); coef(v) = (1 + delta(v)) / sigma(v)
__global__ void bc_back_finish_kernel(const int32_t *__restrict__ ids, int64_t k, const double *__restrict__ sigma,
                                      double *delta, double *__restrict__ coef) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < k; i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t v = ids[i];
    const double sv = sigma[v];
    const double dv = sv * delta[v];
    delta[v] = dv;
    coef[v] = (1.0 + dv) / sv;
  }
}

__global__ void bc_init_kernel(int32_t *depth, double *sigma, double *delta, uint64_t *visited,
                               const uint64_t *__restrict__ zero_bits, int64_t n, int64_t words, int32_t src,
                               int32_t *order, byo_counters *ctr) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n || i < words;
       i += (int64_t)gridDim.x * blockDim.x) {
    if (i < n) {
      depth[i] = i == src ? 0 : -1;
      sigma[i] = i == src ? 1.0 : 0.0;
      delta[i] = 0.0;
    }
    if (i < words) {
      // degree-0 vertices other than the source can never be reached
      uint64_t z = zero_bits[i];
      if ((src >> 6) == i) z &= ~(1ull << (src & 63));
      visited[i] = z | ((src >> 6) == i ? 1ull << (src & 63) : 0ull);
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    order[0] = src;
    for (int j = 0; j < BYO_COUNTER_SLOTS; ++j) {
      ctr[j].count = 0;
      ctr[j].degsum = 0;
      ctr[j].aux0 = 0;
      ctr[j].aux1 = 0;
    }
  }
}

__global__ void bc_src_bit_kernel(uint64_t *bits, int64_t words, int32_t src) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += (int64_t)gridDim.x * blockDim.x)
    bits[i] = (src >> 6) == i ? 1ull << (src & 63) : 0ull;
}

unsigned bc_grid(int64_t count, int64_t per, int64_t cap) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>((count + per - 1) / per, cap));
}

byo_status bc_buffers(byo_graph *g) {
  byo_workspace &w = g->ws;
  if (w.bc_order) return BYO_OK;
  const size_t n1 = (size_t)std::max<int64_t>(g->n, 1);
  BYO_HIP(hipMalloc(&w.bc_coef, sizeof(double) * n1));
  BYO_HIP(hipMalloc(&w.bc_sigma, sizeof(double) * n1));
  BYO_HIP(hipMalloc(&w.bc_depth, sizeof(int32_t) * n1));
  BYO_HIP(hipMalloc(&w.bc_order, sizeof(int32_t) * n1));
  return BYO_OK;
}

}  // namespace

}  // namespace byo

using namespace byo;

extern "C" byo_status byo_bc(byo_graph *g, int64_t src, double *d_delta, double *d_sigma, int32_t *d_depth,
                             const byo_opts *opts, void *stream, byo_run_stats *stats) {
  BYO_CHECK(g && d_delta, BYO_EINVAL, "null argument");
  BYO_CHECK(src >= 0 && src < g->n, BYO_EINVAL, "source out of range");
  byo_opts o;
  byo_opts_default(&o);
  if (opts) o = *opts;
  hipStream_t s = (hipStream_t)stream;
  BYO_TRY(ws_ensure_traversal(g));
  BYO_TRY(bc_buffers(g));
  byo_workspace &w = g->ws;
  // Container-API ablation (Table api-components-avg): without degree() each
  // level's frontier degrees are mapped (they size the cutoff and the
  // edge-balanced passes); without num_edges() m is summed at every level;
  // without a parallel map only the lane forms run. BC has no early exit.
  const uint32_t omit = (uint32_t)o.api_omit;
  const bool mapped = (omit & BYO_API_NO_DEGREE) != 0;
  const int32_t *degs = g->deg;
  if (mapped) BYO_TRY(api_degree_buffer(g, s, (int32_t **)&degs));
  const int64_t n = g->n, words = w.words;
  double *sigma = d_sigma ? d_sigma : w.bc_sigma;
  int32_t *depth = d_depth ? d_depth : w.bc_depth;
  bc_init_kernel<<<bc_grid(std::max(n, words), 256, 8192), 256, 0, s>>>(depth, sigma, d_delta, w.visited,
                                                                        g->zero_bits, n, words, (int32_t)src,
                                                                        w.bc_order, w.ctr);
  bc_src_bit_kernel<<<bc_grid(words, 256, 4096), 256, 0, s>>>(w.bits[0], words, (int32_t)src);
  BYO_HIP(hipGetLastError());
  int32_t src_deg = 0;
  if (!mapped) BYO_TRY(sync_read(s, g->deg + src, &src_deg, sizeof(src_deg)));

  byo_run_stats st;
  std::memset(&st, 0, sizeof(st));
  const int64_t cap = o.max_levels > 0 ? o.max_levels : n + 1;
  std::vector<int64_t> lo(1, 0), cnt(1, 1), dsum(1, src_deg);  // level L: order[lo[L], lo[L] + cnt[L])
  int64_t k = 1, degsum = src_deg, reached = 1, edges = src_deg;
  // fixed PUSH_* / PULL_* variants pin the forward kernel and the backward
  // pass's kind (lane or wavefront-shared lists); otherwise pushes and the
  // backward pass are edge-balanced on levels with a large degree sum
  const bool fixed = o.selector == BYO_SEL_FIXED || (omit & BYO_API_NO_PAR_MAP);
  const int fixed_variant = (omit & BYO_API_NO_PAR_MAP) ? BYO_V_PUSH_THREAD : o.fixed_variant;
  const bool fixed_edges = fixed && (fixed_variant == BYO_V_PUSH_EDGE || fixed_variant == BYO_V_PUSH_BUCKET);
  int cur = 0;
  int32_t L = 0;
  while (true) {
    if (L >= cap) {
      if (stats) *stats = st;
      return fail(BYO_ELIMIT, "betweenness level cap reached");
    }
    int64_t m_seen = g->m;
    if (mapped) {
      BYO_TRY(api_frontier_degrees(g, omit, w.bc_order + lo[L], nullptr, k, s, &degsum));
      dsum[L] = degsum;
      edges += degsum;
    }
    if (omit & BYO_API_NO_NUM_EDGES) BYO_TRY(api_num_edges(g, omit, degs, s, &m_seen));
    bool pull;
    bool wave = true, edges_push = fixed_edges || (!fixed && degsum >= BC_EDGE_MIN);
    const int64_t div = o.dense_divisor > 0 ? o.dense_divisor : 20;
    if (fixed && !(omit & BYO_API_NO_PAR_MAP)) {
      pull = fixed_variant == BYO_V_PULL_THREAD || fixed_variant == BYO_V_PULL_WAVE;
      wave = fixed_variant != BYO_V_PUSH_THREAD && fixed_variant != BYO_V_PULL_THREAD;
    } else {
      // the sparse/dense cutoff: dense when |U| + sum deg(U) > m / divisor
      pull = k + degsum > m_seen / div;
      if (omit & BYO_API_NO_PAR_MAP) wave = false;
    }
    BcFwd a;
    a.off = g->off;
    a.nbr = g->nbr;
    a.deg = degs;  // (stale without degree(): the next level maps its own sum)
    a.in_ids = w.bc_order + lo[L];
    a.in_bits = w.bits[cur];
    a.k = k;
    a.n = n;
    a.words = words;
    a.depth = depth;
    a.sigma = sigma;
    a.visited = w.visited;
    a.out_ids = w.bc_order + lo[L] + k;
    a.out_bits = w.bits[1 - cur];
    a.ctr = w.ctr + (L % BYO_COUNTER_SLOTS);
    a.ctr_clear = w.ctr + ((L + 2) % BYO_COUNTER_SLOTS);
    a.level = L;
    if (pull) {
      if (wave)
        bc_pull_kernel<true><<<bc_grid(words, 4, 4096), BC_BLOCK, 0, s>>>(a);
      else
        bc_pull_kernel<false><<<bc_grid(words, 4, 4096), BC_BLOCK, 0, s>>>(a);
      st.variant_count[wave ? BYO_V_PULL_WAVE : BYO_V_PULL_THREAD]++;
    } else {
      // the output bitmap is written by atomics: clear it first
      BYO_TRY(bitmap_clear(a.out_bits, words, s));
      if (edges_push) {
        BYO_TRY(scan_degrees(degs, a.in_ids, k, w.scan, w.partial, w.partial_cap, s));
        bc_push_edges_kernel<<<bc_grid((degsum + BC_RUN - 1) / BC_RUN, BC_BLOCK, 16384), BC_BLOCK, 0, s>>>(
            a, w.scan);
        st.variant_count[BYO_V_PUSH_EDGE]++;
      } else {
        if (wave)
          bc_push_kernel<true><<<bc_grid(k, BC_BLOCK, 16384), BC_BLOCK, 0, s>>>(a);
        else
          bc_push_kernel<false><<<bc_grid(k, BC_BLOCK, 16384), BC_BLOCK, 0, s>>>(a);
        st.variant_count[wave ? BYO_V_PUSH_WAVE : BYO_V_PUSH_THREAD]++;
      }
    }
    BYO_HIP(hipGetLastError());
    byo_counters c;
    BYO_HIP(hipMemcpyAsync(w.h_ctr + (L % BYO_COUNTER_SLOTS), a.ctr, sizeof(byo_counters), hipMemcpyDeviceToHost, s));
    BYO_HIP(hipStreamSynchronize(s));
    c = w.h_ctr[L % BYO_COUNTER_SLOTS];
    ++L;
    if (c.count == 0) break;
    lo.push_back(lo[L - 1] + k);
    cnt.push_back((int64_t)c.count);
    dsum.push_back((int64_t)c.degsum);
    k = (int64_t)c.count;
    degsum = (int64_t)c.degsum;  // mapped again at the next level's start without degree()
    reached += k;
    if (!mapped) edges += degsum;
    cur = 1 - cur;
  }
  // backward, deepest level first; the source (level 0) keeps delta = 0
  const int32_t deepest = (int32_t)lo.size() - 1;
  for (int32_t l = deepest; l >= 1; --l) {
    const int32_t *ids = w.bc_order + lo[l];
    if (fixed_edges || (!fixed && dsum[l] >= BC_EDGE_MIN)) {
      // edge-balanced: sums into delta (still 0 on this level), then finished
      BYO_TRY(scan_degrees(degs, ids, cnt[l], w.scan, w.partial, w.partial_cap, s));
      bc_back_edges_kernel<<<bc_grid((dsum[l] + BC_RUN - 1) / BC_RUN, BC_BLOCK, 16384), BC_BLOCK, 0, s>>>(
          g->off, g->nbr, ids, cnt[l], w.scan, depth, w.bc_coef, d_delta, l);
      bc_back_finish_kernel<<<bc_grid(cnt[l], 256, 16384), 256, 0, s>>>(ids, cnt[l], sigma, d_delta, w.bc_coef);
    } else if (fixed_variant == BYO_V_PUSH_THREAD || fixed_variant == BYO_V_PULL_THREAD) {
      bc_back_kernel<false><<<bc_grid(cnt[l], BC_BLOCK, 16384), BC_BLOCK, 0, s>>>(
          g->off, g->nbr, ids, cnt[l], depth, sigma, w.bc_coef, d_delta, l);
    } else {
      bc_back_kernel<true><<<bc_grid(cnt[l], BC_BLOCK, 16384), BC_BLOCK, 0, s>>>(
          g->off, g->nbr, ids, cnt[l], depth, sigma, w.bc_coef, d_delta, l);
    }
    BYO_HIP(hipGetLastError());
  }
  st.levels = L;
  st.reached = reached;
  st.edges = edges;
  if (stats) *stats = st;
  return BYO_OK;
}
