// edgeMap(G, U, F) kernels (paper Section 3.2 "EdgeMap") for the BFS and
// min-label functors, in the schedules the paper's GraphContainer API names
// (Section 4.2): serial map_neighbors per frontier vertex (PUSH_THREAD),
// parallel_map_neighbors over one vertex's list (PUSH_WAVE, PUSH_BUCKET's
// wavefront and workgroup tiers, PUSH_EDGE's edge-balanced slices), and the
// dense direction with map_neighbors_early_exit (PULL_THREAD) and
// parallel_map_neighbors_early_exit (PULL_WAVE).
//
// Every kernel writes its per-level totals (vertices emitted, sum of their
// degrees) into one counter slot and zeroes the slot two levels ahead, so the
// level loop never needs a memset between levels.
#include <algorithm>

#include "edgemap_dev.h"

namespace byo {

// ---------------------------------------------------------------- pull scans

// min(best, label[u] for u in nbr[beg, lim) with bit u set in `bits`).
__device__ __forceinline__ int32_t min_member_label(const int32_t *__restrict__ nbr, const uint64_t *__restrict__ bits,
                                                    const int32_t *label, int64_t beg, int64_t lim,
                                                    int32_t best) {
  for (int64_t e = beg; e < lim; e += PULL_ILP) {
    int32_t u[PULL_ILP];
    uint64_t w[PULL_ILP];
    int32_t l[PULL_ILP];
#pragma unroll
    for (int j = 0; j < PULL_ILP; ++j) u[j] = (e + j < lim) ? nbr[e + j] : -1;
#pragma unroll
    for (int j = 0; j < PULL_ILP; ++j) w[j] = u[j] >= 0 ? bits[u[j] >> 6] : 0ull;
#pragma unroll
    for (int j = 0; j < PULL_ILP; ++j) l[j] = ((w[j] >> (u[j] & 63)) & 1ull) ? label[u[j]] : best;
#pragma unroll
    for (int j = 0; j < PULL_ILP; ++j) best = l[j] < best ? l[j] : best;
  }
  return best;
}

// ---------------------------------------------------------------- emission

__device__ __forceinline__ void wave_count(bool pred, unsigned long long *count) {
  uint64_t m = __ballot(pred);
  if (m == 0) return;
  if (lane_id() == __ffsll((long long)m) - 1) atomicAdd(count, (unsigned long long)__popcll(m));
}

// ---------------------------------------------------------------- push kernels

template <typename F>
__global__ void __launch_bounds__(EM_BLOCK) push_thread_kernel(LevelArgs a, F f) {
  unsigned long long degsum = 0, count = 0, maxdeg = 0;
  for (int64_t i = (int64_t)blockIdx.x * EM_BLOCK + threadIdx.x; i - threadIdx.x < a.k;
       i += (int64_t)gridDim.x * EM_BLOCK) {
    if (i < a.k) {
      int32_t u = a.in_ids[i];
      int32_t su = f.src_value(u);
      int64_t end = a.off[u + 1];
      for (int64_t e = a.off[u]; e < end; ++e) {
        int32_t v = a.nbr[e];
        bool ok = f.update(u, su, v, a.out_bits);
        emit<F>(a, ok, v, degsum, count, maxdeg);
      }
    }
  }
  finish_level<EM_BLOCK>(a, degsum, count, maxdeg);
}

template <typename F>
__global__ void __launch_bounds__(EM_BLOCK) push_wave_kernel(LevelArgs a, F f) {
  unsigned long long degsum = 0, count = 0, maxdeg = 0;
  int64_t wave = ((int64_t)blockIdx.x * EM_BLOCK + threadIdx.x) / BYO_WAVE;
  int64_t nwaves = (int64_t)gridDim.x * (EM_BLOCK / BYO_WAVE);
  for (int64_t i = wave; i < a.k; i += nwaves) {
    int32_t u = a.in_ids[i];
    int32_t su = f.src_value(u);
    int64_t beg = a.off[u], end = a.off[u + 1];
    for (int64_t e = beg + lane_id(); e - lane_id() < end; e += BYO_WAVE) {
      bool ok = false;
      int32_t v = 0;
      if (e < end) {
        v = a.nbr[e];
        ok = f.update(u, su, v, a.out_bits);
      }
      emit<F>(a, ok, v, degsum, count, maxdeg);
    }
  }
  finish_level<EM_BLOCK>(a, degsum, count, maxdeg);
}

// Degree-bucketed push: in each chunk of EM_BLOCK frontier vertices, those
// with degree >= t_block are expanded by the whole workgroup, those with
// t_wave <= degree < t_block by their wavefront, the rest by their own thread.
template <typename F>
__global__ void __launch_bounds__(EM_BLOCK) push_bucket_kernel(LevelArgs a, F f) {
  __shared__ int32_t s_u[EM_BLOCK];
  __shared__ int32_t s_su[EM_BLOCK];
  __shared__ int s_nbig;
  unsigned long long degsum = 0, count = 0, maxdeg = 0;
  for (int64_t c0 = (int64_t)blockIdx.x * EM_BLOCK; c0 < a.k; c0 += (int64_t)gridDim.x * EM_BLOCK) {
    int64_t i = c0 + threadIdx.x;
    int32_t u = -1, su = 0, d = 0;
    if (i < a.k) {
      u = a.in_ids[i];
      d = a.deg[u];
      su = f.src_value(u);
    }
    if (threadIdx.x == 0) s_nbig = 0;
    __syncthreads();
    if (d >= a.t_block) {
      int slot = atomicAdd(&s_nbig, 1);
      s_u[slot] = u;
      s_su[slot] = su;
    }
    __syncthreads();
    int nbig = s_nbig;
    for (int j = 0; j < nbig; ++j) {
      int32_t bu = s_u[j], bsu = s_su[j];
      int64_t beg = a.off[bu], end = a.off[bu + 1];
      for (int64_t e = beg + threadIdx.x; e - threadIdx.x < end; e += EM_BLOCK) {
        bool ok = false;
        int32_t v = 0;
        if (e < end) {
          v = a.nbr[e];
          ok = f.update(bu, bsu, v, a.out_bits);
        }
        emit<F>(a, ok, v, degsum, count, maxdeg);
      }
    }
    uint64_t wm = __ballot(d >= a.t_wave && d < a.t_block);
    while (wm) {
      int l = __ffsll((long long)wm) - 1;
      wm &= wm - 1;
      int32_t wu = read_lane_i32(u, l), wsu = read_lane_i32(su, l);
      int64_t beg = a.off[wu], end = a.off[wu + 1];
      for (int64_t e = beg + lane_id(); e - lane_id() < end; e += BYO_WAVE) {
        bool ok = false;
        int32_t v = 0;
        if (e < end) {
          v = a.nbr[e];
          ok = f.update(wu, wsu, v, a.out_bits);
        }
        emit<F>(a, ok, v, degsum, count, maxdeg);
      }
    }
    if (u >= 0 && d < a.t_wave) {
      int64_t beg = a.off[u], end = beg + d;
      for (int64_t e = beg; e < end; ++e) {
        int32_t v = a.nbr[e];
        bool ok = f.update(u, su, v, a.out_bits);
        emit<F>(a, ok, v, degsum, count, maxdeg);
      }
    }
    __syncthreads();
  }
  finish_level<EM_BLOCK>(a, degsum, count, maxdeg);
}

// Edge-balanced push: workgroup b owns edges [b*TILE, (b+1)*TILE) of the
// concatenated neighbour lists of U. The frontier entry owning edge e is the
// last i with scan[i] <= e (zero-degree entries are skipped by construction).
constexpr int PE_ITEMS = 4;
constexpr int PE_TILE = EM_BLOCK * PE_ITEMS;
constexpr int PE_SEG = PE_TILE + 1;

__device__ __forceinline__ int64_t last_le(const long long *scan, int64_t lo, int64_t hi, long long e) {
  // largest i in [lo, hi] with scan[i] <= e, given scan[lo] <= e
  while (lo < hi) {
    int64_t mid = (lo + hi + 1) >> 1;
    if (scan[mid] <= e) lo = mid; else hi = mid - 1;
  }
  return lo;
}

constexpr int PE_STAGE = 3072;   // LDS staging for emitted vertices (flushed with one atomic)

template <typename F>
__global__ void __launch_bounds__(EM_BLOCK) push_edge_kernel(LevelArgs a, F f) {
  __shared__ long long s_scan[PE_SEG];
  __shared__ long long s_base[PE_SEG];
  __shared__ int32_t s_u[PE_SEG];
  __shared__ int32_t s_su[PE_SEG];
  __shared__ int32_t s_out[PE_STAGE];
  __shared__ int64_t s_lo, s_hi;
  __shared__ unsigned s_cnt;
  __shared__ unsigned long long s_dst;
  unsigned long long degsum = 0, count = 0, maxdeg = 0;
  const long long total = a.scan[a.k] < a.total ? a.scan[a.k] : a.total;  // never past the real edge count
  const long long ntiles = (total + PE_TILE - 1) / PE_TILE;
  if (threadIdx.x == 0) s_cnt = 0;
  auto flush = [&]() {
    __syncthreads();
    if (threadIdx.x == 0) s_dst = s_cnt ? atomicAdd(&a.ctr->count, (unsigned long long)s_cnt) : 0ull;
    __syncthreads();
    unsigned c = s_cnt;
    for (unsigned i = threadIdx.x; i < c; i += EM_BLOCK) a.out_ids[s_dst + i] = s_out[i];
    __syncthreads();
    if (threadIdx.x == 0) s_cnt = 0;
    __syncthreads();
  };
  for (long long tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    long long t0 = tile * PE_TILE;
    long long t1 = t0 + PE_TILE < total ? t0 + PE_TILE : total;
    __syncthreads();
    if (threadIdx.x == 0) {
      s_lo = last_le(a.scan, 0, a.k - 1, t0);
      s_hi = last_le(a.scan, s_lo, a.k - 1, t1 - 1);
    }
    __syncthreads();
    int64_t lo = s_lo, hi = s_hi;
    int64_t seg = hi - lo + 1;
    bool in_lds = seg <= PE_SEG;
    if (in_lds) {
      for (int64_t j = threadIdx.x; j < seg; j += EM_BLOCK) {
        int32_t u = a.in_ids[lo + j];
        long long sc = a.scan[lo + j];
        s_scan[j] = sc;
        s_base[j] = a.off[u] - sc;
        s_u[j] = u;
        s_su[j] = f.src_value(u);
      }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < PE_ITEMS; ++it) {
      long long e = t0 + it * EM_BLOCK + threadIdx.x;
      bool ok = false;
      int32_t v = 0;
      if (e < t1) {
        int32_t u, su;
        long long pos;
        if (in_lds) {
          int64_t j = last_le(s_scan, 0, seg - 1, e);
          u = s_u[j];
          su = s_su[j];
          pos = s_base[j] + e;
        } else {
          int64_t i = last_le(a.scan, lo, hi, e);
          u = a.in_ids[i];
          su = f.src_value(u);
          pos = a.off[u] + (e - a.scan[i]);
        }
        v = a.nbr[pos];
        ok = f.update(u, su, v, a.out_bits);
      }
      if (ok) {
        if (a.out_ids) s_out[atomicAdd(&s_cnt, 1u)] = v;
        else ++count;
        if (!F::kDenseFromUpdate && a.out_bits)
          atomicOr((unsigned long long *)&a.out_bits[v >> 6], 1ull << (v & 63));
        tally_degree((unsigned long long)a.deg[v], degsum, maxdeg);
      }
    }
    if (a.out_ids) {
      __syncthreads();
      if (s_cnt > PE_STAGE - PE_TILE) flush();
    }
  }
  if (a.out_ids) flush();
  finish_level<EM_BLOCK>(a, degsum, count, maxdeg);
}

// ---------------------------------------------------------------- pull kernels (BFS)

// One wavefront per 64-vertex bitmap word; lane = bit. Only unvisited
// vertices scan their lists, and stop at the first neighbour in U (unless
// no_early_exit, for the lists the lane scans by itself). The
// wavefront owns its word of `visited` and the output bitmap, so no atomics.
template <bool WAVE_ASSIST>
__global__ void __launch_bounds__(EM_BLOCK) bfs_pull_kernel(LevelArgs a, BfsF f) {
  unsigned long long degsum = 0, count = 0, maxdeg = 0;
  const int64_t nwaves_total = (int64_t)gridDim.x * (EM_BLOCK / BYO_WAVE);
  int64_t w = (int64_t)xcd_block(blockIdx.x, gridDim.x) * (EM_BLOCK / BYO_WAVE) + threadIdx.x / BYO_WAVE;
  for (; w < a.words; w += nwaves_total) {
    uint64_t vis = f.visited[w];
    if (vis == ~0ull) {
      if (lane_id() == 0) a.out_bits[w] = 0ull;
      continue;
    }
    int32_t v = (int32_t)(w * 64 + lane_id());
    bool cand = (w * 64 + lane_id() < a.n) && !((vis >> lane_id()) & 1ull);
    bool found = false;
    int32_t par = -1;
    int64_t beg = 0, end = 0;
    if (cand) {
      beg = a.off[v];
      end = a.off[v + 1];
      // a list longer than t_wave goes to the wavefront's cooperative
      // early-exit scan; the others use the serial scan, which reads the
      // whole list when the container has no early-exit map
      const bool coop = WAVE_ASSIST && end - beg > a.t_wave;
      int64_t lim = coop ? beg + a.t_wave : end;
      par = first_member(a.nbr, a.in_bits, beg, lim, a.no_early_exit != 0 && !coop);
      found = par >= 0;
    }
    if (WAVE_ASSIST) {
      uint64_t pm = __ballot(cand && !found && end - beg > a.t_wave);
      while (pm) {
        int l = __ffsll((long long)pm) - 1;
        pm &= pm - 1;
        int64_t lb = (int64_t)read_lane_u64((uint64_t)(beg + a.t_wave), l);
        int64_t le = (int64_t)read_lane_u64((uint64_t)end, l);
        bool done = false;
        for (int64_t base = lb; base < le && !done; base += 4 * BYO_WAVE) {
          int32_t u[4];
          bool hit[4];
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            int64_t e = base + j * BYO_WAVE + lane_id();
            u[j] = e < le ? a.nbr[e] : 0;
          }
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            int64_t e = base + j * BYO_WAVE + lane_id();
            hit[j] = e < le && test_bit(a.in_bits, u[j]);
          }
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            uint64_t hm = __ballot(hit[j]);
            if (hm && !done) {
              int32_t pu = read_lane_i32(u[j], __ffsll((long long)hm) - 1);
              if (lane_id() == l) {
                par = pu;
                found = true;
              }
              done = true;
            }
          }
        }
      }
    }
    if (found) {
      f.parent[v] = par;
      f.depth[v] = f.newdepth;
      tally_degree((unsigned long long)a.deg[v], degsum, maxdeg);
    }
    uint64_t m = __ballot(found);
    if (lane_id() == 0) {
      a.out_bits[w] = m;
      if (m) {
        f.visited[w] = vis | m;
        count += (unsigned long long)__popcll(m);
      }
    }
    if (a.out_ids) {
      // ascending within the word; order across words is arbitrary
      if (m) {
        unsigned long long base = 0;
        if (lane_id() == 0) base = atomicAdd(&a.ctr->aux0, (unsigned long long)__popcll(m));
        base = read_lane_u64(base, 0);
        if (found) a.out_ids[base + __popcll(m & lanemask_lt())] = v;
      }
    }
  }
  finish_level<EM_BLOCK>(a, degsum, count, maxdeg);
}

// ---------------------------------------------------------------- pull kernel (min-label)

// Every vertex takes the minimum label over its neighbours in U (no early
// exit: the minimum needs all of them). Long lists are reduced by the
// wavefront when WAVE_ASSIST.
template <bool WAVE_ASSIST>
__global__ void __launch_bounds__(EM_BLOCK) cc_pull_kernel(LevelArgs a, CcF f) {
  unsigned long long degsum = 0, count = 0, maxdeg = 0;
  const int64_t nwaves_total = (int64_t)gridDim.x * (EM_BLOCK / BYO_WAVE);
  int64_t w = (int64_t)xcd_block(blockIdx.x, gridDim.x) * (EM_BLOCK / BYO_WAVE) + threadIdx.x / BYO_WAVE;
  for (; w < a.words; w += nwaves_total) {
    int64_t v64 = w * 64 + lane_id();
    bool valid = v64 < a.n;
    int32_t v = (int32_t)v64;
    int32_t lv = valid ? f.label[v] : 0;
    int32_t best = lv;
    int64_t beg = 0, end = 0;
    if (valid) {
      beg = a.off[v];
      end = a.off[v + 1];
      int64_t lim = WAVE_ASSIST ? (end - beg > a.t_wave ? beg + a.t_wave : end) : end;
      best = min_member_label(a.nbr, a.in_bits, f.label, beg, lim, best);
    }
    if (WAVE_ASSIST) {
      uint64_t pm = __ballot(valid && end - beg > a.t_wave);
      while (pm) {
        int l = __ffsll((long long)pm) - 1;
        pm &= pm - 1;
        int64_t lb = (int64_t)read_lane_u64((uint64_t)(beg + a.t_wave), l);
        int64_t le = (int64_t)read_lane_u64((uint64_t)end, l);
        int32_t mn = 0x7fffffff;
        for (int64_t e = lb + lane_id(); e < le; e += BYO_WAVE) {
          int32_t u = a.nbr[e];
          if (test_bit(a.in_bits, u)) {
            int32_t lu = f.label[u];
            mn = lu < mn ? lu : mn;
          }
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
          int32_t t = __shfl_xor(mn, o);
          mn = t < mn ? t : mn;
        }
        if (lane_id() == l) best = mn < best ? mn : best;
      }
    }
    bool changed = valid && best < lv;
    if (changed) {
      atomicMin(&f.label[v], best);
      tally_degree((unsigned long long)a.deg[v], degsum, maxdeg);
    }
    uint64_t m = __ballot(changed);
    if (lane_id() == 0) {
      a.out_bits[w] = m;
      count += (unsigned long long)__popcll(m);
    }
  }
  finish_level<EM_BLOCK>(a, degsum, count, maxdeg);
}

// Pointer jumping: label[v] <- label[label[v]] until it stops decreasing.
// Labels stay IDs of same-component vertices no larger than before, so the
// min-label fixed point is unchanged. Changed vertices join the output set.
__global__ void __launch_bounds__(EM_BLOCK) cc_shortcut_kernel(int32_t *label, const int32_t *__restrict__ deg,
                                                               int64_t n, int64_t words, uint64_t *out_bits,
                                                               byo_counters *ctr) {
  unsigned long long degsum = 0, count = 0, maxdeg = 0;
  const int64_t nwaves_total = (int64_t)gridDim.x * (EM_BLOCK / BYO_WAVE);
  int64_t w = (int64_t)xcd_block(blockIdx.x, gridDim.x) * (EM_BLOCK / BYO_WAVE) + threadIdx.x / BYO_WAVE;
  for (; w < words; w += nwaves_total) {
    int64_t v64 = w * 64 + lane_id();
    bool changed = false;
    if (v64 < n) {
      int32_t v = (int32_t)v64;
      int32_t l0 = label[v], l = l0;
      while (true) {
        int32_t l2 = label[l];
        if (l2 >= l) break;
        l = l2;
      }
      if (l < l0) {
        atomicMin(&label[v], l);
        changed = true;
      }
    }
    uint64_t m = __ballot(changed);
    if (m) {
      uint64_t old = out_bits[w];
      uint64_t fresh = m & ~old;
      if (changed && ((fresh >> lane_id()) & 1ull)) tally_degree((unsigned long long)deg[v64], degsum, maxdeg);
      if (lane_id() == 0) {
        out_bits[w] = old | m;
        count += (unsigned long long)__popcll(fresh);
      }
    }
  }
  unsigned long long t = block_sum<unsigned long long, EM_BLOCK>(degsum);
  unsigned long long c = block_sum<unsigned long long, EM_BLOCK>(count);
  unsigned long long mx = block_max_u64<EM_BLOCK>(maxdeg);
  if (threadIdx.x == 0) {
    if (t) atomicAdd(&ctr->degsum, t);
    if (c) atomicAdd(&ctr->count, c);
    if (mx) atomicMax(&ctr->maxdeg, mx);
  }
}

// ---------------------------------------------------------------- dispatch

static unsigned capped(int64_t blocks, int64_t cap) {
  if (blocks < 1) blocks = 1;
  return (unsigned)(blocks > cap ? cap : blocks);
}

template <typename F>
static byo_status launch_push(int variant, const LevelArgs &a, const F &f, hipStream_t s) {
  if (a.k == 0) {
    // still clear the future slot
    LevelArgs z = a;
    push_thread_kernel<F><<<1, EM_BLOCK, 0, s>>>(z, f);
    BYO_HIP(hipGetLastError());
    return BYO_OK;
  }
  switch (variant) {
    case BYO_V_PUSH_THREAD:
      push_thread_kernel<F><<<capped((a.k + EM_BLOCK - 1) / EM_BLOCK, 16384), EM_BLOCK, 0, s>>>(a, f);
      break;
    case BYO_V_PUSH_WAVE:
      push_wave_kernel<F><<<capped((a.k + 3) / 4, 16384), EM_BLOCK, 0, s>>>(a, f);
      break;
    case BYO_V_PUSH_BUCKET:
      push_bucket_kernel<F><<<capped((a.k + EM_BLOCK - 1) / EM_BLOCK, 16384), EM_BLOCK, 0, s>>>(a, f);
      break;
    case BYO_V_PUSH_EDGE: {
      int64_t tiles = (a.total + PE_TILE - 1) / PE_TILE;
      push_edge_kernel<F><<<capped(tiles, 2048), EM_BLOCK, 0, s>>>(a, f);
      break;
    }
    default:
      return fail(BYO_EINVAL, "not a push variant");
  }
  BYO_HIP(hipGetLastError());
  return BYO_OK;
}

static LevelArgs make_args(const byo_graph *g, const level_io &io, const byo_opts &o) {
  LevelArgs a;
  a.off = g->off;
  a.nbr = g->nbr;
  a.deg = g->deg;
  a.in_ids = io.in_ids;
  a.in_bits = io.in_bits;
  a.scan = g->ws.scan;
  a.k = io.in_count;
  a.n = g->n;
  a.words = (g->n + 63) / 64;
  a.total = 0;
  a.out_ids = io.out_ids;
  a.out_bits = io.out_bits;
  a.ctr = io.ctr;
  a.ctr_clear = io.ctr_clear;
  a.t_wave = o.t_wave > 0 ? o.t_wave : 32;
  a.t_block = o.t_block > 0 ? o.t_block : 4096;
  if (a.t_block < a.t_wave) a.t_block = a.t_wave;
  a.no_early_exit = (o.api_omit & BYO_API_NO_EARLY_EXIT) ? 1 : 0;
  return a;
}

// dense kernels loop over words with a grid of at most 16 workgroups per CU
static unsigned pull_grid(int64_t words) { return capped((words + 3) / 4, 4096); }

// Read back scan[k] (sum of frontier degrees) for the edge-balanced variant.
static byo_status edge_total(byo_graph *g, const level_io &io, hipStream_t s, long long *total) {
  BYO_TRY(frontier_degree_scan(g, io.in_ids, io.in_count, g->ws.scan, g->ws.partial, g->ws.partial_cap, s));
  return sync_read(s, g->ws.scan + io.in_count, total, sizeof(long long));
}

byo_status bfs_level(byo_graph *g, int variant, const bfs_state &st, const level_io &io, const byo_opts &o,
                     hipStream_t s, long long known_total) {
  LevelArgs a = make_args(g, io, o);
  BfsF f{st.parent, st.depth, st.visited, st.level + 1};
  if (variant == BYO_V_PULL_THREAD || variant == BYO_V_PULL_WAVE) {
    BYO_CHECK(io.in_bits && io.out_bits, BYO_EINVAL, "pull needs dense input and output");
    if (a.words == 0) return BYO_OK;
    ktimer_scope kt(BYO_K_BFS_PULL, s);
    if (variant == BYO_V_PULL_THREAD)
      bfs_pull_kernel<false><<<pull_grid(a.words), EM_BLOCK, 0, s>>>(a, f);
    else
      bfs_pull_kernel<true><<<pull_grid(a.words), EM_BLOCK, 0, s>>>(a, f);
    BYO_HIP(hipGetLastError());
    return BYO_OK;
  }
  BYO_CHECK(io.in_ids || io.in_count == 0, BYO_EINVAL, "push needs a sparse input");
  if (variant == BYO_V_PUSH_EDGE && a.k > 0) {
    if (known_total >= 0) {
      BYO_TRY(frontier_degree_scan(g, io.in_ids, io.in_count, g->ws.scan, g->ws.partial, g->ws.partial_cap, s));
      a.total = known_total;
    } else {
      BYO_TRY(edge_total(g, io, s, &a.total));
    }
    if (a.total == 0) variant = BYO_V_PUSH_THREAD;
  }
  ktimer_scope kt(BYO_K_BFS_PUSH, s);
  return launch_push(variant, a, f, s);
}

byo_status cc_level(byo_graph *g, int variant, int32_t *label, const level_io &io, const byo_opts &o,
                    hipStream_t s, long long known_total) {
  LevelArgs a = make_args(g, io, o);
  CcF f{label};
  BYO_CHECK(io.out_bits, BYO_EINVAL, "min-label edgeMap needs a dense output");
  if (variant == BYO_V_PULL_THREAD || variant == BYO_V_PULL_WAVE) {
    BYO_CHECK(io.in_bits, BYO_EINVAL, "pull needs dense input");
    if (a.words == 0) return BYO_OK;
    ktimer_scope kt(BYO_K_CC_PULL, s);
    if (variant == BYO_V_PULL_THREAD)
      cc_pull_kernel<false><<<pull_grid(a.words), EM_BLOCK, 0, s>>>(a, f);
    else
      cc_pull_kernel<true><<<pull_grid(a.words), EM_BLOCK, 0, s>>>(a, f);
    BYO_HIP(hipGetLastError());
    return BYO_OK;
  }
  BYO_CHECK(io.in_ids || io.in_count == 0, BYO_EINVAL, "push needs a sparse input");
  BYO_TRY(bitmap_clear(io.out_bits, a.words, s));
  if (variant == BYO_V_PUSH_EDGE && a.k > 0) {
    if (known_total >= 0) {
      BYO_TRY(frontier_degree_scan(g, io.in_ids, io.in_count, g->ws.scan, g->ws.partial, g->ws.partial_cap, s));
      a.total = known_total;
    } else {
      BYO_TRY(edge_total(g, io, s, &a.total));
    }
    if (a.total == 0) variant = BYO_V_PUSH_THREAD;
  }
  ktimer_scope kt(BYO_K_CC_PUSH, s);
  return launch_push(variant, a, f, s);
}

byo_status cc_shortcut(byo_graph *g, int32_t *label, uint64_t *out_bits, byo_counters *ctr, hipStream_t s) {
  int64_t words = (g->n + 63) / 64;
  if (words == 0) return BYO_OK;
  ktimer_scope kt(BYO_K_CC_SHORTCUT, s);
  cc_shortcut_kernel<<<pull_grid(words), EM_BLOCK, 0, s>>>(label, g->deg, g->n, words, out_bits, ctr);
  BYO_HIP(hipGetLastError());
  return BYO_OK;
}

// ---------------------------------------------------------------- multi-source push (bit-parallel)

// Multi-source BFS push: the frontier bits of u (one bit per source) that v
// has not seen yet are OR-ed into visit[v]; v is emitted once per level by
// whoever first sets its bit in `touched`.
template <int W>
struct MsF {
  const uint64_t *front;
  const uint64_t *seen;
  uint64_t *visit;
  static constexpr bool kDenseFromUpdate = true;
  __device__ __forceinline__ int32_t src_value(int32_t u) const { return u; }
  __device__ __forceinline__ bool update(int32_t u, int32_t /*su*/, int32_t v, uint64_t *touched) const {
    bool any = false;
#pragma unroll
    for (int w = 0; w < W; ++w) {
      uint64_t fb = front[(int64_t)u * W + w];
      if (!fb) continue;
      uint64_t nb = fb & ~seen[(int64_t)v * W + w];
      if (nb) {
        atomicOr((unsigned long long *)&visit[(int64_t)v * W + w], (unsigned long long)nb);
        any = true;
      }
    }
    if (!any) return false;
    uint64_t bit = 1ull << (v & 63);
    unsigned long long prev = atomicOr((unsigned long long *)&touched[v >> 6], (unsigned long long)bit);
    return !(prev & bit);
  }
};

template <int W>
static byo_status ms_push_w(byo_graph *g, int variant, const ms_state &ms, const level_io &io, const byo_opts &o,
                            hipStream_t s, long long known_total) {
  LevelArgs a = make_args(g, io, o);
  MsF<W> f{ms.front, ms.seen, ms.visit};
  if (variant == BYO_V_PUSH_EDGE && a.k > 0) {
    BYO_TRY(frontier_degree_scan(g, io.in_ids, io.in_count, g->ws.scan, g->ws.partial, g->ws.partial_cap, s));
    a.total = known_total;
    if (a.total == 0) variant = BYO_V_PUSH_THREAD;
  }
  ktimer_scope kt(BYO_K_MSBFS_PUSH, s);
  return launch_push(variant, a, f, s);
}

byo_status ms_push_level(byo_graph *g, int variant, const ms_state &ms, const level_io &io, const byo_opts &o,
                         hipStream_t s, long long known_total) {
  BYO_CHECK(io.out_bits && io.out_ids, BYO_EINVAL, "multi-source push needs touched list and bitmap");
  BYO_CHECK(variant >= 0 && variant <= BYO_V_PUSH_EDGE, BYO_EINVAL, "multi-source push needs a push variant");
  switch (ms.W) {
    case 1: return ms_push_w<1>(g, variant, ms, io, o, s, known_total);
    case 2: return ms_push_w<2>(g, variant, ms, io, o, s, known_total);
    case 3: return ms_push_w<3>(g, variant, ms, io, o, s, known_total);
    case 4: return ms_push_w<4>(g, variant, ms, io, o, s, known_total);
    default: return fail(BYO_EINVAL, "1 to 4 source words");
  }
}

}  // namespace byo
