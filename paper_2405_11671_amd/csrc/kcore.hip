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
//
// The same peeling also runs in one persistent cooperative launch
// (`persistent`, the default where cooperative launches work): every phase
// below is separated from the next by a grid barrier, and every workgroup
// takes the same decisions from the totals the previous phase left.
//  - min: the alive count and least remaining degree, one pass over the
//    vertices; k jumps to max(k + 1, least);
//  - collect: the alive vertices with remaining degree <= k get coreness k and
//    form the frontier;
//  - sub-rounds at k, each a removal push over the frontier held as work
//    items (one per KC_RUN entries of a member's list), one item per lane, so
//    hubs and leaves spread over the grid alike with no scan of the
//    frontier's degrees. A neighbour dropping from k + 1 to k gets coreness k
//    at once and its items join the next frontier; it takes no further part
//    in the removal (only the drop k + 1 -> k is a join, so each vertex joins
//    once), so the sets are those of the host-driven loop.
#include <algorithm>
#include <climits>
#include <cstring>

#include "gridsync.h"
#include "internal.h"

namespace byo {

namespace {

constexpr int KC_BLOCK = 256;
constexpr int KC_RUN = 16;
// frontiers with a smaller degree sum take the lane kernel (the edge-balanced
// one costs a degree scan, 3 launches, per sub-round)
constexpr int64_t KC_EDGE_MIN = 1 << 15;
constexpr int64_t KC_LANE_MAX = 16;  // ... and no vertex of more neighbours than this (one run per lane)
static_assert(KC_LANE_MAX <= KC_RUN, "a lane-path list fits one run");

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

// One lane's share of a removal push: neighbours u[j] of the frontier's
// concatenated lists at positions e0 + j < e1 (at most KC_RUN), with every
// neighbour load, every liveness read and every decrement issued before the
// first result is used, so a lane waits about one round trip per run instead
// of one per edge. joins[j]: u[j] dropped from k + 1 to k (only one decrement
// sees that, so each vertex joins once).
__device__ __forceinline__ void kc_decrement_run(const int64_t *__restrict__ off, const int32_t *__restrict__ nbr,
                                                 const int32_t *__restrict__ ids, int64_t kf,
                                                 const long long *__restrict__ scan, long long e0, long long e1,
                                                 int32_t k, int32_t *dcur, const int32_t *core, int32_t (&u)[KC_RUN],
                                                 bool (&joins)[KC_RUN]) {
  int64_t i = 0, base = 0;
  long long iend = 0;
  if (e0 < e1) {
    i = kc_last_le(scan, kf, e0);
    base = off[ids[i]] - scan[i];
    iend = scan[i + 1];
  }
#pragma unroll
  for (int j = 0; j < KC_RUN; ++j) {
    const long long e = e0 + j;
    u[j] = 0;
    if (e < e1) {
      while (e >= iend) {
        ++i;
        base = off[ids[i]] - scan[i];
        iend = scan[i + 1];
      }
      u[j] = nbr[base + e];
    }
  }
  int32_t cr[KC_RUN];
#pragma unroll
  for (int j = 0; j < KC_RUN; ++j) cr[j] = e0 + j < e1 ? core[u[j]] : 0;
  int32_t old[KC_RUN];
#pragma unroll
  for (int j = 0; j < KC_RUN; ++j) old[j] = (e0 + j < e1 && cr[j] < 0) ? atomicSub(&dcur[u[j]], 1) : 0;
#pragma unroll
  for (int j = 0; j < KC_RUN; ++j) joins[j] = e0 + j < e1 && cr[j] < 0 && old[j] == k + 1;
}

// The same for the first KC_RUN neighbours from list position p of one vertex
// whose list ends at `end`.
__device__ __forceinline__ void kc_decrement_list(const int32_t *__restrict__ nbr, int64_t p, int64_t end, int32_t k,
                                                  int32_t *dcur, const int32_t *core, int32_t (&u)[KC_RUN],
                                                  bool (&joins)[KC_RUN]) {
#pragma unroll
  for (int j = 0; j < KC_RUN; ++j) u[j] = p + j < end ? nbr[p + j] : 0;
  int32_t cr[KC_RUN];
#pragma unroll
  for (int j = 0; j < KC_RUN; ++j) cr[j] = p + j < end ? core[u[j]] : 0;
  int32_t old[KC_RUN];
#pragma unroll
  for (int j = 0; j < KC_RUN; ++j) old[j] = (p + j < end && cr[j] < 0) ? atomicSub(&dcur[u[j]], 1) : 0;
#pragma unroll
  for (int j = 0; j < KC_RUN; ++j) joins[j] = p + j < end && cr[j] < 0 && old[j] == k + 1;
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
    int32_t u[KC_RUN];
    bool joins[KC_RUN];
    kc_decrement_run(off, nbr, ids, kf, scan, e0, e1, k, dcur, core, u, joins);
#pragma unroll
    for (int j = 0; j < KC_RUN; ++j) {
      wave_append(joins[j], u[j], out, &ctr->count);
      if (joins[j]) {
        degsum += (unsigned long long)deg[u[j]];
        dmax = (unsigned long long)deg[u[j]] > dmax ? (unsigned long long)deg[u[j]] : dmax;
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
      for (int64_t p = off[v]; p < end; p += KC_RUN) {
        int32_t u[KC_RUN];
        bool joins[KC_RUN];
        kc_decrement_list(nbr, p, end, k, dcur, core, u, joins);
#pragma unroll
        for (int j = 0; j < KC_RUN; ++j) {
          wave_append(joins[j], u[j], out, &ctr->count);
          if (joins[j]) {
            degsum += (unsigned long long)deg[u[j]];
            dmax = (unsigned long long)deg[u[j]] > dmax ? (unsigned long long)deg[u[j]] : dmax;
          }
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

// ---------------------------------------------------------------- persistent form

constexpr int KP_THREADS = 512;
// one workgroup per CU (256 on the chip): the kernel's registers allow no
// more, and capping them for two or three per CU spilled and ran slower
// (42.8 and 70.5 ms against 37.0 ms at RMAT-22)
constexpr int KP_PER_CU = 1;
constexpr int KP_MAX_BLOCKS = 4096;
constexpr unsigned KP_SPIN_LIMIT = 1u << 22;
constexpr int KP_ILP = 4;                    // vertices per thread in flight in the passes over all vertices
constexpr int KP_SMALL = 4;                  // items a lane stages in LDS at once (lists up to 64 entries)
constexpr int KP_STAGE = 5120;               // LDS staging of a workgroup's items

// A frontier is held as work items, one per KC_RUN consecutive entries of a
// member's list (vertex << 32 | run index): the removal push takes one item
// per lane, so every list, hub or leaf, is spread over ceil(deg / KC_RUN)
// lanes without a scan of the frontier's degrees.
__host__ __device__ inline int64_t kp_items(int64_t d) { return (d + KC_RUN - 1) / KC_RUN; }

// Same-address atomics from every workgroup serialise (tens of microseconds
// per phase with hundreds of workgroups), so a phase's totals go through per-workgroup
// records instead: each workgroup writes its own, and after the barrier every
// workgroup reduces all of them to the same values. Only the append cursor of
// the next frontier's items is an atomic, taken about once per workgroup.
struct kp_rec {
  unsigned long long a, b, c;  // min phase: alive count, least degree; else vertices, degree sum, largest degree
};

// The item cursor of phase p is cursor[p % 4]; phase p clears
// cursor[(p + 2) % 4], so two barriers separate a clear from both the read
// (in the phase after its use) and the next use.
struct kp_ctl {
  grid_sync sync;
  unsigned long long cursor[4 * 16];  // 128 bytes apart
  kp_rec rec[2][KP_MAX_BLOCKS];       // by phase parity
};

struct kp_result {
  int32_t rounds, limit, fail, pad;
  unsigned long long edges;
};

// workgroup minimum (MIN = true) or maximum, valid in every thread
template <bool MIN>
__device__ __forceinline__ unsigned long long kp_block_ext(unsigned long long v) {
  __shared__ unsigned long long wm[KP_THREADS / BYO_WAVE];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const unsigned long long t = __shfl_xor(v, o);
    v = MIN ? (t < v ? t : v) : (t > v ? t : v);
  }
  __syncthreads();
  if (lane_id() == 0) wm[threadIdx.x / BYO_WAVE] = v;
  __syncthreads();
  unsigned long long r = wm[0];
#pragma unroll
  for (int i = 1; i < KP_THREADS / BYO_WAVE; ++i) r = MIN ? (wm[i] < r ? wm[i] : r) : (wm[i] > r ? wm[i] : r);
  return r;
}

// wavefront inclusive scan of v; *total = the wavefront's sum
__device__ __forceinline__ int32_t kp_wave_scan(int32_t v, int32_t *total) {
  int32_t x = v;
#pragma unroll
  for (int o = 1; o < BYO_WAVE; o <<= 1) {
    const int32_t y = __shfl_up(x, o);
    if (lane_id() >= o) x += y;
  }
  *total = __shfl(x, BYO_WAVE - 1);
  return x;
}

// Workgroup-staged item appends. A wavefront reserves its lanes' small item
// counts (lists of at most KP_SMALL * KC_RUN entries) in LDS with one LDS
// atomic; reservations are consecutive, and one that would pass the end of
// the staging buffer goes to the list itself instead, as do the items of
// longer lists (one cursor atomic per wavefront). `vend` is the end of the
// last reservation that fitted: below it every staged slot is written.
struct kp_stager {
  uint64_t *buf;
  unsigned *n, *vend;
  unsigned long long *base;
  uint64_t *out;
  unsigned long long *cursor;
  __device__ __forceinline__ void reserve_write(int32_t cnt, int32_t pos_incl, int32_t tot, bool global,
                                                const int32_t *v, const int32_t *ci, int R) {
    unsigned long long b = 0;
    bool to_list = global;
    if (!global) {
      unsigned bl = 0;
      if (lane_id() == 0) {
        bl = atomicAdd(n, (unsigned)tot);
        if (bl + (unsigned)tot <= (unsigned)KP_STAGE) atomicMax(vend, bl + (unsigned)tot);
      }
      bl = (unsigned)__shfl((int)bl, 0);
      to_list = bl + (unsigned)tot > (unsigned)KP_STAGE;
      b = bl;
    }
    if (to_list) {
      unsigned long long g = 0;
      if (lane_id() == 0) g = atomicAdd(cursor, (unsigned long long)tot);
      b = (unsigned long long)__shfl((long long)g, 0);
    }
    uint64_t *dst = to_list ? out : buf;
    unsigned long long q = b + (unsigned long long)(pos_incl - cnt);
    for (int r = 0; r < R; ++r)
      for (int32_t j = 0; j < ci[r]; ++j) dst[q++] = ((uint64_t)(uint32_t)v[r] << 32) | (uint32_t)j;
  }
  // the items of v[r] (degree d[r]) where pred[r]; every lane of the
  // wavefront calls it (convergent code)
  template <int R>
  __device__ __forceinline__ void add(const bool (&pred)[R], const int32_t (&v)[R], const int32_t (&d)[R]) {
    int32_t sc[R], bc[R], st = 0, bt = 0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int32_t ci = pred[r] ? (int32_t)kp_items(d[r]) : 0;
      sc[r] = ci <= KP_SMALL ? ci : 0;
      bc[r] = ci - sc[r];
      st += sc[r];
      bt += bc[r];
    }
    int32_t tot;
    int32_t x = kp_wave_scan(st, &tot);
    if (tot) reserve_write(st, x, tot, false, v, sc, R);
    x = kp_wave_scan(bt, &tot);
    if (tot) reserve_write(bt, x, tot, true, v, bc, R);
  }
  __device__ __forceinline__ void flush() {
    __syncthreads();
    const unsigned cnt = *vend;
    if (threadIdx.x == 0 && cnt) *base = atomicAdd(cursor, (unsigned long long)cnt);
    __syncthreads();
    const unsigned long long b0 = *base;
    for (unsigned i = threadIdx.x; i < cnt; i += KP_THREADS) out[b0 + i] = buf[i];
    __syncthreads();
    if (threadIdx.x == 0) *n = *vend = 0;
    __syncthreads();
  }
  // between loop iterations: flush a buffer more than half full
  __device__ __forceinline__ void maybe_flush() {
    __syncthreads();
    if (*n > (unsigned)(KP_STAGE / 2)) flush();
  }
};

__global__ void __launch_bounds__(KP_THREADS) kcore_persistent_kernel(
    const int64_t *__restrict__ off, const int32_t *__restrict__ nbr, const int32_t *__restrict__ deg, int64_t n,
    int32_t *dcur, int32_t *core, uint64_t *items0, uint64_t *items1, kp_ctl *c, int32_t cap,
    kp_result *res) {
  __shared__ uint64_t s_buf[KP_STAGE];
  __shared__ unsigned s_n, s_vend;
  __shared__ unsigned long long s_base;
  const unsigned G = gridDim.x;
  const int64_t nth = (int64_t)G * KP_THREADS;
  const int64_t tid = (int64_t)blockIdx.x * KP_THREADS + threadIdx.x;
  uint64_t *items[2] = {items0, items1};
  if (threadIdx.x == 0) s_n = s_vend = 0;
  __syncthreads();
  unsigned p = 0;  // phase index
  bool ok = true;
  // every phase ends here: clear the cursor two phases ahead, then the barrier
  auto end_phase = [&]() -> bool {
    if (blockIdx.x == 0 && threadIdx.x == 0)
      __hip_atomic_store(&c->cursor[((p + 2) & 3) * 16], 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    ++p;
    return grid_barrier(&c->sync, G, KP_SPIN_LIMIT);
  };
  auto cursor_now = [&]() { return &c->cursor[(p & 3) * 16]; };
  auto prev_count = [&]() -> int64_t { return (int64_t)ld_rlx64(&c->cursor[((p - 1) & 3) * 16]); };
  // this workgroup's record for the phase, and every workgroup's reduction
  // of the previous phase's records: sum of a, min (MIN) or max of c, sum of b
  auto put = [&](unsigned long long a, unsigned long long b, unsigned long long cc) {
    if (threadIdx.x == 0) c->rec[p & 1][blockIdx.x] = kp_rec{a, b, cc};
  };
  auto reduce = [&](bool is_min, unsigned long long *a, unsigned long long *b, unsigned long long *cc) {
    const kp_rec *r = c->rec[(p - 1) & 1];
    unsigned long long x = 0, y = 0, z = is_min ? ULLONG_MAX : 0ull;
    for (unsigned j = threadIdx.x; j < G; j += KP_THREADS) {
      const kp_rec q = r[j];
      x += q.a;
      y += q.b;
      z = is_min ? (q.c < z ? q.c : z) : (q.c > z ? q.c : z);
    }
    *a = block_sum<unsigned long long, KP_THREADS>(x);
    *b = block_sum<unsigned long long, KP_THREADS>(y);
    *cc = is_min ? kp_block_ext<true>(z) : kp_block_ext<false>(z);
  };
  int64_t k = -1;
  int32_t rounds = 0;
  unsigned long long edges = 0;
  bool limit = false;
  int cur = 0;
  while (ok) {
    // min: alive count and least remaining degree
    {
      unsigned long long alive = 0, mn = ULLONG_MAX;
      for (int64_t v0 = tid; v0 < n; v0 += nth * KP_ILP) {
        int32_t cr[KP_ILP], dc[KP_ILP];
#pragma unroll
        for (int j = 0; j < KP_ILP; ++j) {
          const int64_t v = v0 + j * nth;
          cr[j] = v < n ? core[v] : 0;
          dc[j] = v < n ? dcur[v] : 0;
        }
#pragma unroll
        for (int j = 0; j < KP_ILP; ++j)
          if (cr[j] < 0) {
            ++alive;
            mn = (unsigned long long)dc[j] < mn ? (unsigned long long)dc[j] : mn;
          }
      }
      alive = block_sum<unsigned long long, KP_THREADS>(alive);
      mn = kp_block_ext<true>(mn);
      put(alive, 0, mn);
    }
    if (!(ok = end_phase())) break;
    unsigned long long alive, unused, least;
    reduce(true, &alive, &unused, &least);
    if (alive == 0) break;
    k = (int64_t)least > k + 1 ? (int64_t)least : k + 1;
    // collect: the alive vertices with remaining degree <= k get coreness k
    // and their items form the frontier
    int64_t kv, fmax;
    long long fdeg;
    {
      kp_stager stg{s_buf, &s_n, &s_vend, &s_base, items[cur], cursor_now()};
      unsigned long long cnt = 0, degsum = 0, dmax = 0;
      for (int64_t base = (int64_t)blockIdx.x * KP_THREADS; base < n; base += nth * KP_ILP) {  // uniform
        bool take[KP_ILP];
        int32_t cr[KP_ILP], dc[KP_ILP];
#pragma unroll
        for (int j = 0; j < KP_ILP; ++j) {
          const int64_t v = base + j * nth + threadIdx.x;
          cr[j] = v < n ? core[v] : 0;
          dc[j] = v < n ? dcur[v] : 0;
        }
        int32_t vv[KP_ILP], dd[KP_ILP];
#pragma unroll
        for (int j = 0; j < KP_ILP; ++j) {
          const int64_t v = base + j * nth + threadIdx.x;
          take[j] = v < n && cr[j] < 0 && dc[j] <= k;
          vv[j] = (int32_t)v;
          dd[j] = 0;
          if (take[j]) {
            core[v] = (int32_t)k;
            dd[j] = deg[v];
            ++cnt;
            degsum += (unsigned long long)dd[j];
            dmax = (unsigned long long)dd[j] > dmax ? (unsigned long long)dd[j] : dmax;
          }
        }
        stg.add(take, vv, dd);
        stg.maybe_flush();
      }
      stg.flush();
      cnt = block_sum<unsigned long long, KP_THREADS>(cnt);
      degsum = block_sum<unsigned long long, KP_THREADS>(degsum);
      dmax = kp_block_ext<false>(dmax);
      put(cnt, degsum, dmax);
    }
    if (!(ok = end_phase())) break;
    int64_t kf = prev_count();
    {
      unsigned long long a, b, cc;
      reduce(false, &a, &b, &cc);
      kv = (int64_t)a;
      fdeg = (long long)b;
      fmax = (int64_t)cc;
    }
    (void)fmax;
    while (kv > 0) {
      if (rounds >= cap) {
        limit = true;
        break;
      }
      // removal push at coreness k: one item per lane
      const uint64_t *fr = items[cur];
      kp_stager stg{s_buf, &s_n, &s_vend, &s_base, items[1 - cur], cursor_now()};
      unsigned long long cnt = 0, degsum = 0, dmax = 0;
      for (int64_t i = tid; i - (int64_t)threadIdx.x < kf; i += nth) {  // uniform per workgroup
        int64_t p0 = 0, end = 0;
        if (i < kf) {
          const uint64_t it = fr[i];
          const int32_t v = (int32_t)(it >> 32);
          p0 = off[v] + (int64_t)(uint32_t)it * KC_RUN;
          const int64_t e = off[v + 1];
          end = p0 + KC_RUN < e ? p0 + KC_RUN : e;
        }
        int32_t u[KC_RUN];
        bool joins[KC_RUN];
        kc_decrement_list(nbr, p0, end, (int32_t)k, dcur, core, u, joins);
        int32_t dd[KC_RUN];
#pragma unroll
        for (int j = 0; j < KC_RUN; ++j) dd[j] = joins[j] ? deg[u[j]] : 0;
#pragma unroll
        for (int j = 0; j < KC_RUN; ++j)
          if (joins[j]) {
            core[u[j]] = (int32_t)k;
            ++cnt;
            degsum += (unsigned long long)dd[j];
            dmax = (unsigned long long)dd[j] > dmax ? (unsigned long long)dd[j] : dmax;
          }
        stg.add(joins, u, dd);
        stg.maybe_flush();
      }
      stg.flush();
      cnt = block_sum<unsigned long long, KP_THREADS>(cnt);
      degsum = block_sum<unsigned long long, KP_THREADS>(degsum);
      dmax = kp_block_ext<false>(dmax);
      put(cnt, degsum, dmax);
      if (!(ok = end_phase())) break;
      ++rounds;
      edges += (unsigned long long)fdeg;
      cur = 1 - cur;
      kf = prev_count();
      unsigned long long a, b, cc;
      reduce(false, &a, &b, &cc);
      kv = (int64_t)a;
      fdeg = (long long)b;
    }
    if (limit) break;
  }
  if (!ok) {
    if (threadIdx.x == 0) res->fail = 1;
    return;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    res->rounds = rounds;
    res->limit = limit ? 1 : 0;
    res->edges = edges;
  }
}

}  // namespace

struct kp_ws {
  kp_ctl *ctl = nullptr;
  kp_result *res = nullptr;
  uint64_t *items[2] = {nullptr, nullptr};  // frontier items, n + ceil(m / KC_RUN) each
  int nblocks = 0;
  bool checked = false, usable = false;
};

void kp_release(void *p) {
  kp_ws *d = (kp_ws *)p;
  if (!d) return;
  if (d->ctl) (void)hipFree(d->ctl);
  if (d->res) (void)hipFree(d->res);
  for (uint64_t *q : d->items)
    if (q) (void)hipFree(q);
  delete d;
}

static byo_status kp_ensure(byo_graph *g, kp_ws **out) {
  byo_workspace &w = g->ws;
  if (!w.kcp) w.kcp = new kp_ws();
  kp_ws *d = (kp_ws *)w.kcp;
  *out = d;
  if (d->checked) return BYO_OK;
  d->checked = true;
  int dev = 0, coop = 0, cus = 0, per_cu = 0;
  BYO_HIP(hipGetDevice(&dev));
  BYO_HIP(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev));
  BYO_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  BYO_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kcore_persistent_kernel, KP_THREADS, 0));
  if (!coop || cus <= 0 || per_cu <= 0) return BYO_OK;  // not usable: the host-driven loop runs instead
  d->nblocks = std::min(cus * std::min(per_cu, KP_PER_CU), KP_MAX_BLOCKS);
  BYO_HIP(hipMalloc(&d->ctl, sizeof(kp_ctl)));
  BYO_HIP(hipMalloc(&d->res, sizeof(kp_result)));
  // a frontier's items: at most one per vertex plus one per KC_RUN entries
  const size_t cap = (size_t)(g->n + (g->m + KC_RUN - 1) / KC_RUN);
  for (uint64_t *&q : d->items) BYO_HIP(hipMalloc(&q, sizeof(uint64_t) * std::max<size_t>(cap, 1)));
  d->usable = true;
  return BYO_OK;
}

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
  kp_ws *kp = nullptr;
  if (o.persistent && omit == 0) BYO_TRY(kp_ensure(g, &kp));
  if (kp && kp->usable) {
    BYO_HIP(hipMemsetAsync(kp->ctl, 0, sizeof(kp_ctl), s));
    BYO_HIP(hipMemsetAsync(kp->res, 0, sizeof(kp_result), s));
    const int32_t cap32 = (int32_t)std::min<int64_t>(o.max_levels > 0 ? o.max_levels : INT32_MAX, INT32_MAX);
    void *args[] = {(void *)&g->off, (void *)&g->nbr, (void *)&degs, (void *)&n, (void *)&dcur, (void *)&d_core,
                    (void *)&kp->items[0], (void *)&kp->items[1], (void *)&kp->ctl, (void *)&cap32,
                    (void *)&kp->res};
    BYO_HIP(hipLaunchCooperativeKernel((const void *)kcore_persistent_kernel, dim3((unsigned)kp->nblocks),
                                       dim3(KP_THREADS), args, 0, s));
    kp_result r;
    BYO_TRY(sync_read(s, kp->res, &r, sizeof(r)));
    BYO_CHECK(!r.fail, BYO_EHIP, "persistent k-core: a grid barrier wait timed out");
    st.levels = r.rounds;
    st.device_levels = r.rounds;
    st.variant_count[BYO_V_PUSH_EDGE] = r.rounds;  // every sub-round pushes over list runs
    st.reached = n;
    st.edges = (int64_t)r.edges;
    if (stats) *stats = st;
    if (r.limit) return fail(BYO_ELIMIT, "k-core round cap reached");
    return BYO_OK;
  }
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
      kc_min_kernel<<<kc_grid(n, KC_BLOCK, 1024), KC_BLOCK, 0, s>>>(dcur, d_core, n, cs);
      BYO_HIP(hipGetLastError());
      BYO_TRY(read(slot, &c));
      remaining = (int64_t)c.aux0;
      if (remaining == 0) break;
      k = std::max<int64_t>(k + 1, (int64_t)c.aux1);
      kc_reset_kernel<<<1, 64, 0, s>>>(w.ctr);
      kc_collect_kernel<<<kc_grid(n, KC_BLOCK, 1024), KC_BLOCK, 0, s>>>(dcur, d_core, degs, n, (int32_t)k,
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
