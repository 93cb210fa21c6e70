// BFS in one persistent launch: a cooperative kernel runs every level of a
// BFS from a set of sources, with a grid barrier between levels, and returns
// when the frontier is empty. The batch of many graphs (batch.hip, one source
// per graph of the disjoint union) runs it by default: its union frontier
// grows over a few heavy levels and then trails off over many small ones,
// where a host-driven level loop pays a launch and a counter read-back per
// level.
//
// The launch also starts the search: every parent and depth to -1, the
// visited bitmap to the vertices of degree zero (and the bits past n), the
// frontier bitmaps clear; then, after a grid barrier, the sources, their
// bitmap bits and the first level's counters; so a search is one launch and
// one read-back of its totals.
//
// A level, identical in every workgroup:
//  - reads the frontier's size and degree sum (written by the level before),
//    and picks the direction with the threshold rule: dense pull iff
//    |U| + sum(deg U) > m / dense_divisor;
//  - push: edge-balanced over tiles of frontier vertices whose degree
//    prefix a workgroup builds in LDS: a list of up to PB_EB vertices is one
//    tile shared by the whole grid, a longer one a tile per workgroup, and
//    the bitmap a pull level leaves is ranked by a workgroup scan over words
//    interleaved between the workgroups; eight neighbours in flight per
//    lane; a CAS on parent[v] claims v (lane groups per vertex remain for a
//    degree sum beyond 32 bits);
//  - pull: a wavefront per 64-vertex word of the visited bitmap, words
//    already all visited skipped; each unvisited vertex scans its list until
//    a neighbour in the frontier bitmap (the lane the first t_wave entries,
//    eight loads in flight, the wavefront the rest of a longer list), the
//    first one found being its parent;
//  - either way the new vertices go to the next bitmap (three rotate, so the
//    one two levels back is cleared during this level); a push level also
//    writes them to the next ID list, staged in LDS and reserved with one
//    atomic per workgroup, while a push level after a pull reads its
//    frontier from the bitmap, so pull levels write no list;
//  - the size and degree sum of the next frontier are summed per workgroup
//    and added with one atomic each; counter slots rotate like the bitmaps.
// The depths, the reached set and its size are those of any BFS; parents are
// a valid BFS tree.
#include <algorithm>
#include <cstring>

#include "edgemap_dev.h"
#include "gridsync.h"
#include "internal.h"

namespace byo {

constexpr int PB_THREADS = 512;
constexpr int PB_STAGE = 4096;          // LDS staging of one workgroup's new vertices per level
// workgroups per compute unit in the launch: one (256 on the chip) keeps the
// grid barrier cheap for the many small levels of a batch; two were 5% slower
// there and 4% faster on a single RMAT-22 search
constexpr int PB_PER_CU = 1;
constexpr unsigned PB_SPIN_LIMIT = 1u << 22;
constexpr int PB_SLOT = 16;             // counter slots 128 bytes apart
constexpr int PB_EB = 2048;             // frontier lists up to this long are pushed edge-balanced over the grid

struct pb_ctl {
  grid_sync sync;
  unsigned long long cnt[3 * PB_SLOT];   // frontier size per level mod 3 (also the next list's append cursor)
  unsigned long long dsum[3 * PB_SLOT];  // its degree sum
};

struct pb_result {
  int32_t levels, limit, fail, pad;
  unsigned long long reached, edges, push_levels, pull_levels;
};

struct pb_ws {
  uint64_t *bits2 = nullptr;  // third frontier bitmap (the workspace holds two)
  pb_ctl *ctl = nullptr;
  pb_result *res = nullptr;
  int nblocks = 0;
  bool checked = false, usable = false;
  bool reset = true;  // the grid barrier's counters need clearing (first use, or after a failed wait)
};

// up to this many sources travel in the launch's arguments; more are copied
// to the device first
constexpr int PB_ARG_SRCS = 64;
struct pb_srcs {
  int32_t v[PB_ARG_SRCS];
};

__global__ void __launch_bounds__(PB_THREADS) bfs_persistent_kernel(
    const int64_t *__restrict__ off, const int32_t *__restrict__ nbr, const int32_t *__restrict__ deg, int64_t n,
    int64_t m, int32_t div, int32_t t_wave, int32_t *__restrict__ parent, int32_t *__restrict__ depth,
    uint64_t *__restrict__ visited, int64_t words, uint64_t *__restrict__ b0, uint64_t *__restrict__ b1,
    uint64_t *__restrict__ b2, int32_t *__restrict__ q0, int32_t *__restrict__ q1, pb_ctl *__restrict__ c,
    int32_t max_levels, pb_result *__restrict__ res, const uint64_t *__restrict__ zero_bits, pb_srcs sarg,
    const int32_t *__restrict__ sdev, int64_t ns) {
  __shared__ int32_t stage[PB_STAGE];
  __shared__ unsigned s_cnt;
  __shared__ unsigned long long s_base;
  // edge-balanced push of a short frontier list: the list's degree prefix,
  // each entry's offset from list position to neighbour index, and its vertex
  __shared__ uint32_t s_pre[PB_EB + 1];
  __shared__ int64_t s_shift[PB_EB];
  __shared__ int32_t s_u[PB_EB];
  __shared__ uint32_t s_wsum[PB_THREADS / BYO_WAVE];
  const unsigned nblocks = gridDim.x;
  const int t = threadIdx.x;
  const int64_t cutoff = m / (div > 0 ? div : 20);
  const int64_t tw = t_wave > 0 ? t_wave : 32;
  unsigned long long push_levels = 0, pull_levels = 0, reached = 0, edges = 0;
  int L = 0, limit = 0;
  {
    // start: parents and depths -1, visited = vertices of degree zero and
    // the bits past n, the first two frontier bitmaps clear (the third is
    // cleared during level 0)
    const int64_t gt = (int64_t)blockIdx.x * PB_THREADS + t, gs = (int64_t)nblocks * PB_THREADS;
    for (int64_t i = gt; i < n; i += gs) {
      parent[i] = -1;
      depth[i] = -1;
    }
    for (int64_t w = gt; w < words; w += gs) {
      uint64_t x = zero_bits[w];
      if (w == words - 1 && (n & 63)) x |= ~0ull << (n & 63);
      visited[w] = x;
      b0[w] = 0ull;
      b1[w] = 0ull;
    }
    if (!grid_barrier(&c->sync, nblocks, PB_SPIN_LIMIT)) ns = 0;
    // then the sources (workgroup 0): parent = itself, depth 0, the first
    // list and bitmap, and the first level's counters (the other two slots
    // clear)
    if (blockIdx.x == 0 && ns > 0) {
      unsigned long long dsum = 0;
      for (int64_t i = t; i < ns; i += PB_THREADS) {
        const int32_t sv = ns <= PB_ARG_SRCS ? sarg.v[i] : sdev[i];
        parent[sv] = sv;
        depth[sv] = 0;
        q0[i] = sv;
        atomicOr((unsigned long long *)&visited[sv >> 6], 1ull << (sv & 63));
        atomicOr((unsigned long long *)&b0[sv >> 6], 1ull << (sv & 63));
        dsum += (unsigned long long)deg[sv];
      }
      dsum = block_sum<unsigned long long, PB_THREADS>(dsum);
      if (t < 3) {
        c->cnt[t * PB_SLOT] = t == 0 ? (unsigned long long)ns : 0ull;
        c->dsum[t * PB_SLOT] = t == 0 ? dsum : 0ull;
      }
    }
    if (ns == 0 || !grid_barrier(&c->sync, nblocks, PB_SPIN_LIMIT)) L = -1;
  }
  bool prev_pull = false;  // level 0 pushes from the sources' list (its bitmap is set too)
  for (; L >= 0; ++L) {
    const unsigned long long k = ld_rlx64(&c->cnt[(L % 3) * PB_SLOT]);
    const unsigned long long ds = ld_rlx64(&c->dsum[(L % 3) * PB_SLOT]);
    reached += k;
    edges += ds;
    if (k == 0) break;
    if (L >= max_levels) {
      limit = 1;
      break;
    }
    uint64_t *bin = L % 3 == 0 ? b0 : (L % 3 == 1 ? b1 : b2);
    uint64_t *bout = L % 3 == 0 ? b1 : (L % 3 == 1 ? b2 : b0);
    uint64_t *bclr = L % 3 == 0 ? b2 : (L % 3 == 1 ? b0 : b1);
    const int32_t *qin = (L & 1) ? q1 : q0;
    int32_t *qout = (L & 1) ? q0 : q1;
    const int nx = (L + 1) % 3, cl = (L + 2) % 3;
    // the slot and bitmap of two levels back were last read before the
    // previous barrier: clear them for the level after this one
    if (blockIdx.x == 0 && t == 0) {
      __hip_atomic_store(&c->cnt[cl * PB_SLOT], 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&c->dsum[cl * PB_SLOT], 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    for (int64_t w = (int64_t)blockIdx.x * PB_THREADS + t; w < words; w += (int64_t)nblocks * PB_THREADS) bclr[w] = 0ull;
    if (t == 0) s_cnt = 0;
    __syncthreads();
    const int32_t nd = L + 1;
    unsigned long long mydeg = 0, mycount = 0;
    auto emit = [&](int32_t v) {
      const unsigned pos = atomicAdd(&s_cnt, 1u);
      if (pos < (unsigned)PB_STAGE) {
        stage[pos] = v;
      } else {
        const unsigned long long gp = atomicAdd(&c->cnt[nx * PB_SLOT], 1ull);
        qout[gp] = v;
      }
      mydeg += (unsigned long long)deg[v];
    };
    const bool pull = (int64_t)(k + ds) > cutoff;
    if (pull) {
      ++pull_levels;
      const int64_t nwaves = (int64_t)nblocks * (PB_THREADS / BYO_WAVE);
      for (int64_t w = (int64_t)blockIdx.x * (PB_THREADS / BYO_WAVE) + t / BYO_WAVE; w < words; w += nwaves) {
        const uint64_t vis = visited[w];
        if (vis == ~0ull) continue;  // every vertex of the word visited (bits past n are set)
        const int64_t v = w * 64 + lane_id();
        const bool cand = !((vis >> lane_id()) & 1ull);
        int32_t par = -1;
        int64_t b = 0, e = 0;
        if (cand) {
          b = off[v];
          e = off[v + 1];
          // the first t_wave entries by the lane (PULL_ILP loads in flight),
          // the rest of a long list by the whole wavefront
          par = first_member(nbr, bin, b, e - b > tw ? b + tw : e);
        }
        uint64_t pm = __ballot(cand && par < 0 && e - b > tw);
        while (pm) {
          const int l = __ffsll((long long)pm) - 1;
          pm &= pm - 1;
          const int64_t lb = (int64_t)read_lane_u64((uint64_t)(b + tw), l);
          const int64_t le = (int64_t)read_lane_u64((uint64_t)e, l);
          for (int64_t x0 = lb; x0 < le; x0 += 4 * BYO_WAVE) {
            int32_t u[4];
            bool hit[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
              const int64_t x = x0 + j * BYO_WAVE + lane_id();
              u[j] = x < le ? nbr[x] : 0;
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) {
              const int64_t x = x0 + j * BYO_WAVE + lane_id();
              hit[j] = x < le && ((bin[u[j] >> 6] >> (u[j] & 63)) & 1ull);
            }
            int32_t pu = -1;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
              const uint64_t hm = __ballot(hit[j]);
              if (hm && pu < 0) pu = read_lane_i32(u[j], __ffsll((long long)hm) - 1);
            }
            if (pu >= 0) {
              if (lane_id() == l) par = pu;
              break;
            }
          }
        }
        const bool found = par >= 0;
        const uint64_t mask = __ballot(found);
        if (mask == 0) continue;
        if (lane_id() == 0) {
          visited[w] = vis | mask;  // one wavefront owns word w in a pull level
          bout[w] = mask;
          mycount += (unsigned long long)__popcll(mask);
        }
        if (found) {
          parent[v] = par;
          depth[v] = nd;
          mydeg += (unsigned long long)deg[v];
        }
      }
    } else {
      ++push_levels;
      // a lane that won v's CAS on parent[v] sets its depth and its visited
      // and output bits; the CASes of a batch are all issued before any result
      // is used, so a lane waits about one round trip per batch, not per edge
      auto won = [&](int32_t v) {
        const unsigned long long bit = 1ull << (v & 63);
        depth[v] = nd;
        atomicOr((unsigned long long *)&visited[v >> 6], bit);
        atomicOr((unsigned long long *)&bout[v >> 6], bit);
        emit(v);
      };
      // a wavefront's lanes take list positions lb + lane, lb + lane + 64, ...
      // of u's list, four rounds in flight per step
      auto wave_list = [&](int32_t wu, int64_t wb, int64_t we) {
        for (int64_t x0 = wb + lane_id(); x0 - lane_id() < we; x0 += 4 * BYO_WAVE) {
          int32_t v[4];
          bool tried[4];
          int32_t old[4];
#pragma unroll
          for (int j = 0; j < 4; ++j) v[j] = x0 + j * BYO_WAVE < we ? nbr[x0 + j * BYO_WAVE] : -1;
#pragma unroll
          for (int j = 0; j < 4; ++j) tried[j] = v[j] >= 0 && !((visited[v[j] >> 6] >> (v[j] & 63)) & 1ull);
#pragma unroll
          for (int j = 0; j < 4; ++j) old[j] = tried[j] ? atomicCAS(&parent[v[j]], -1, wu) : 0;
#pragma unroll
          for (int j = 0; j < 4; ++j)
            if (tried[j] && old[j] == -1) won(v[j]);
        }
      };
      // Edge-balanced push, in tiles of frontier vertices whose degree prefix
      // a workgroup builds in LDS; eight edges in flight per lane.
      //  - A list of at most PB_EB vertices is one tile that every workgroup
      //    builds and whose edges the whole grid shares (a hub among a few
      //    vertices would otherwise leave one wavefront walking its list).
      //  - A longer list is cut into tiles of ceil(k / workgroups) vertices
      //    (at most PB_EB), one workgroup per tile, which shares the tile's
      //    edges among its own lanes.
      //  - After a pull level the frontier is a bitmap: a workgroup takes 512
      //    of its words, interleaved with the other workgroups' words, ranks
      //    their set bits with a workgroup scan, and pushes them in tiles of up
      //    to PB_EB.
      const unsigned long long nthreads = (unsigned long long)nblocks * PB_THREADS;
      constexpr int PER = PB_EB / PB_THREADS;
      // exclusive scan over the workgroup (every thread calls it); *total = sum
      auto bscan = [&](uint32_t val, uint32_t *total) {
        __syncthreads();  // s_wsum's previous readers are done
        uint32_t x = val;
#pragma unroll
        for (int o = 1; o < BYO_WAVE; o <<= 1) {
          const uint32_t y = __shfl_up(x, o);
          if (lane_id() >= o) x += y;
        }
        if (lane_id() == BYO_WAVE - 1) s_wsum[t / BYO_WAVE] = x;
        __syncthreads();
        uint32_t run = x - val, tot = 0;
#pragma unroll
        for (int w = 0; w < PB_THREADS / BYO_WAVE; ++w) {
          if (w < t / BYO_WAVE) run += s_wsum[w];
          tot += s_wsum[w];
        }
        *total = tot;
        return run;
      };
      // one tile of cnt vertices, from qin[lo ...] or (in_lds) from s_u; its
      // edges e = ebase + lane, + estride, ... of the tile's degree prefix
      auto eb_tile = [&](unsigned long long cnt, bool in_lds, unsigned long long lo, unsigned long long ebase,
                         unsigned long long estride) {
        int32_t ul[PER];
        int64_t bl[PER];
        uint32_t dl[PER], tsum = 0;
#pragma unroll
        for (int j = 0; j < PER; ++j) {
          const unsigned long long i = (unsigned long long)t * PER + j;
          ul[j] = i < cnt ? (in_lds ? s_u[i] : qin[lo + i]) : -1;
        }
#pragma unroll
        for (int j = 0; j < PER; ++j) {
          bl[j] = ul[j] >= 0 ? off[ul[j]] : 0;
          dl[j] = ul[j] >= 0 ? (uint32_t)deg[ul[j]] : 0u;
          tsum += dl[j];
        }
        uint32_t total;
        uint32_t run = bscan(tsum, &total);
        // each thread rewrites only the positions it read
#pragma unroll
        for (int j = 0; j < PER; ++j) {
          const unsigned long long i = (unsigned long long)t * PER + j;
          if (i < cnt) {
            s_pre[i] = run;
            s_shift[i] = bl[j] - (int64_t)run;
            s_u[i] = ul[j];
          }
          run += dl[j];
        }
        __syncthreads();
        const int kk = (int)cnt;
        // the tile position holding edge e: the last i with s_pre[i] <= e
        // (its degree is not zero, as s_pre[i + 1] > e)
        auto find = [&](uint32_t e) {
          int a = 0, b = kk;
          while (b - a > 1) {
            const int mid = (a + b) >> 1;
            if (s_pre[mid] <= e) a = mid;
            else b = mid;
          }
          return a;
        };
        for (unsigned long long e0 = ebase + t; e0 < total; e0 += 8 * estride) {
          int32_t v[8], su[8];
          uint64_t vw[8];
          bool tried[8];
          int32_t old[8];
#pragma unroll
          for (int j = 0; j < 8; ++j) {
            const unsigned long long e = e0 + j * estride;
            su[j] = -1;
            v[j] = -1;
            if (e < total) {
              const int i = find((uint32_t)e);
              su[j] = s_u[i];
              v[j] = nbr[(int64_t)e + s_shift[i]];
            }
          }
#pragma unroll
          for (int j = 0; j < 8; ++j) vw[j] = v[j] >= 0 ? visited[v[j] >> 6] : ~0ull;
#pragma unroll
          for (int j = 0; j < 8; ++j) {
            tried[j] = v[j] >= 0 && !((vw[j] >> (v[j] & 63)) & 1ull);
            old[j] = tried[j] ? atomicCAS(&parent[v[j]], -1, su[j]) : 0;
          }
#pragma unroll
          for (int j = 0; j < 8; ++j)
            if (tried[j] && old[j] == -1) won(v[j]);
        }
        // the next tile rewrites the prefix and the vertices
        __syncthreads();
      };
      if (!prev_pull && ds < (1ull << 32)) {
        const bool whole = k <= (unsigned long long)PB_EB;
        const unsigned long long T =
            whole ? k : std::min<unsigned long long>(PB_EB, (k + nblocks - 1) / nblocks);
        const unsigned long long tstep = whole ? k : T * nblocks;
        for (unsigned long long lo = whole ? 0ull : (unsigned long long)blockIdx.x * T; lo < k; lo += tstep)
          eb_tile(std::min<unsigned long long>(T, k - lo), false, lo,
                  whole ? (unsigned long long)blockIdx.x * PB_THREADS : 0ull,
                  whole ? nthreads : (unsigned long long)PB_THREADS);
      } else if (prev_pull && ds < (1ull << 32)) {
        // word p0 + t * workgroups + workgroup: every workgroup samples the
        // whole vertex range, so dense stretches of the bitmap are shared
        for (unsigned long long p0 = 0; p0 < (unsigned long long)words; p0 += nthreads) {
          const unsigned long long w = p0 + (unsigned long long)t * nblocks + blockIdx.x;
          const uint64_t word = w < (unsigned long long)words ? bin[w] : 0ull;
          const uint32_t pc = (uint32_t)__popcll(word);
          uint32_t tot;
          const uint32_t r0 = bscan(pc, &tot);
          for (uint32_t plo = 0; plo < tot; plo += PB_EB) {
            // this thread's set bits whose rank falls in [plo, plo + PB_EB)
            if (pc && r0 + pc > plo && r0 < plo + PB_EB) {
              uint64_t x = word;
              uint32_t r = r0;
              while (x) {
                const int b = __ffsll((long long)x) - 1;
                x &= x - 1;
                if (r >= plo && r < plo + PB_EB) s_u[r - plo] = (int32_t)(w * 64 + b);
                ++r;
              }
            }
            __syncthreads();
            eb_tile(std::min<uint32_t>(PB_EB, tot - plo), true, 0ull, 0ull, (unsigned long long)PB_THREADS);
          }
        }
      } else {
        // a degree sum of 2^32 or more (beyond the tiles' 32-bit prefixes): a
        // frontier list is walked by groups of g lanes per vertex, g a power
        // of two sized from the level's mean degree (about four entries per
        // lane), raised to a whole wavefront when the list has no more vertices
        // than the grid has wavefronts; the bitmap left by a pull level is
        // walked a lane per vertex
        unsigned g = 1;
        if (!prev_pull) {
          if (k * BYO_WAVE <= nthreads) {
            g = BYO_WAVE;
          } else {
            while (g < (unsigned)BYO_WAVE && (unsigned long long)g * 4 * k < ds && (unsigned long long)g * 2 * k <= nthreads) g *= 2;
          }
        }
        const unsigned sub = (unsigned)t & (g - 1);
        const unsigned long long items = prev_pull ? (unsigned long long)words * BYO_WAVE : k;
        for (unsigned long long base = (unsigned long long)blockIdx.x * PB_THREADS; base < items * g; base += nthreads) {
          const unsigned long long i = (base + t) / g;
          int32_t u = -1;
          int64_t b = 0, e = 0;
          if (prev_pull) {
            if (i < items && ((bin[i >> 6] >> (i & 63)) & 1ull)) u = (int32_t)i;
          } else if (i < k) {
            u = qin[i];
          }
          if (u >= 0) {
            b = off[u];
            e = off[u + 1];
          }
          const bool wide = u >= 0 && e - b > (int64_t)g * tw;
          if (u >= 0 && !wide) {
            // lane sub of the group takes entries b + sub, b + sub + g, ...:
            // eight entries, their visited words and their CASes in flight per step
            for (int64_t x0 = b + sub; x0 - sub < e; x0 += 8 * (int64_t)g) {
              int32_t v[8];
              uint64_t vw[8];
              bool tried[8];
              int32_t old[8];
  #pragma unroll
              for (int j = 0; j < 8; ++j) v[j] = x0 + j * (int64_t)g < e ? nbr[x0 + j * (int64_t)g] : -1;
  #pragma unroll
              for (int j = 0; j < 8; ++j) vw[j] = v[j] >= 0 ? visited[v[j] >> 6] : ~0ull;
  #pragma unroll
              for (int j = 0; j < 8; ++j) {
                tried[j] = v[j] >= 0 && !((vw[j] >> (v[j] & 63)) & 1ull);
                old[j] = tried[j] ? atomicCAS(&parent[v[j]], -1, u) : 0;
              }
  #pragma unroll
              for (int j = 0; j < 8; ++j)
                if (tried[j] && old[j] == -1) won(v[j]);
            }
          }
          // a list longer than g * t_wave is walked by the whole wavefront;
          // the lanes of one group hold the same vertex, so only its first
          // lane raises the ballot
          uint64_t wm = __ballot(wide && sub == 0);
          while (wm) {
            const int l = __ffsll((long long)wm) - 1;
            wm &= wm - 1;
            const int32_t wu = read_lane_i32(u, l);
            const int64_t wb = (int64_t)read_lane_u64((uint64_t)b, l), we = (int64_t)read_lane_u64((uint64_t)e, l);
            wave_list(wu, wb, we);
          }
        }
      }
    }
    // flush the stage with one reservation; add this workgroup's degree sum
    const unsigned long long bdeg = block_sum<unsigned long long, PB_THREADS>(mydeg);
    const unsigned long long bcount = block_sum<unsigned long long, PB_THREADS>(mycount);
    __syncthreads();
    const unsigned staged = s_cnt < (unsigned)PB_STAGE ? s_cnt : (unsigned)PB_STAGE;
    if (t == 0) {
      // a push level's count is its list's append cursor; a pull level adds its count
      s_base = staged ? atomicAdd(&c->cnt[nx * PB_SLOT], (unsigned long long)staged) : 0ull;
      if (bcount) atomicAdd(&c->cnt[nx * PB_SLOT], bcount);
      if (bdeg) atomicAdd(&c->dsum[nx * PB_SLOT], bdeg);
    }
    __syncthreads();
    for (unsigned j = t; j < staged; j += PB_THREADS) qout[s_base + j] = stage[j];
    prev_pull = pull;
    if (!grid_barrier(&c->sync, nblocks, PB_SPIN_LIMIT)) break;
  }
  if (blockIdx.x == 0 && t == 0) {
    res->levels = L < 0 ? 0 : L;
    res->limit = limit;
    res->fail = ld_rlx(&c->sync.fail[0]) ? 1 : 0;
    res->reached = reached;
    res->edges = edges;
    res->push_levels = push_levels;
    res->pull_levels = pull_levels;
  }
}

void pb_release(void *p) {
  pb_ws *d = (pb_ws *)p;
  if (!d) return;
  void *x[] = {d->bits2, d->ctl, d->res};
  for (void *y : x)
    if (y) (void)hipFree(y);
  delete d;
}

static byo_status pb_ensure(byo_graph *g, pb_ws **out) {
  byo_workspace &w = g->ws;
  if (!w.pbfs) w.pbfs = new pb_ws();
  pb_ws *d = (pb_ws *)w.pbfs;
  *out = d;
  if (d->checked) return BYO_OK;
  d->checked = true;
  int dev = 0, coop = 0, cus = 0, per_cu = 0;
  BYO_HIP(hipGetDevice(&dev));
  BYO_HIP(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev));
  BYO_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  BYO_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, bfs_persistent_kernel, PB_THREADS, 0));
  if (!coop || cus <= 0 || per_cu <= 0) return BYO_OK;  // not usable: the host-driven loop runs instead
  d->nblocks = cus * std::min(per_cu, PB_PER_CU);
  BYO_HIP(hipMalloc(&d->bits2, sizeof(uint64_t) * (size_t)std::max<int64_t>(g->ws.words, 1)));
  BYO_HIP(hipMalloc(&d->ctl, sizeof(pb_ctl)));
  BYO_HIP(hipMalloc(&d->res, sizeof(pb_result)));
  d->usable = true;
  return BYO_OK;
}

bool bfs_persistent_usable(byo_graph *g) {
  if (ws_ensure_traversal(g) != BYO_OK) return false;
  pb_ws *d = nullptr;
  if (pb_ensure(g, &d) != BYO_OK) return false;
  return d->usable;
}

byo_status bfs_persistent_run(byo_graph *g, const int32_t *srcs, int64_t ns, int32_t *d_depth, int32_t *d_parent,
                              const byo_opts &o, hipStream_t s, byo_run_stats *stats) {
  BYO_TRY(ws_ensure_traversal(g));
  pb_ws *d = nullptr;
  BYO_TRY(pb_ensure(g, &d));
  BYO_CHECK(d->usable, BYO_ESTATE, "cooperative launch not available for the persistent BFS");
  byo_workspace &w = g->ws;
  const int64_t n = g->n;
  BYO_CHECK(ns >= 1 && ns <= n, BYO_EINVAL, "bad source count");
  // up to PB_ARG_SRCS sources travel in the arguments, more through ids[1]
  pb_srcs sarg;
  std::memset(&sarg, 0, sizeof(sarg));
  const int32_t *sdev = nullptr;
  if (ns <= PB_ARG_SRCS) {
    std::memcpy(sarg.v, srcs, sizeof(int32_t) * (size_t)ns);
  } else {
    BYO_HIP(hipMemcpyAsync(w.ids[1], srcs, sizeof(int32_t) * (size_t)ns, hipMemcpyHostToDevice, s));
    sdev = w.ids[1];
  }
  if (d->reset) {
    BYO_HIP(hipMemsetAsync(d->ctl, 0, sizeof(pb_ctl), s));
    d->reset = false;
  }
  const int64_t m = g->m, words = w.words;
  const int32_t div = o.dense_divisor > 0 ? o.dense_divisor : 20;
  const int32_t tw = o.t_wave > 0 ? o.t_wave : 32;
  const int32_t cap = (int32_t)std::min<int64_t>(o.max_levels > 0 ? o.max_levels : n + 1, 2147483647LL);
  void *args[] = {(void *)&g->off, (void *)&g->nbr, (void *)&g->deg, (void *)&n, (void *)&m, (void *)&div,
                  (void *)&tw, (void *)&d_parent, (void *)&d_depth, (void *)&w.visited, (void *)&words,
                  (void *)&w.bits[0], (void *)&w.bits[1], (void *)&d->bits2, (void *)&w.ids[0], (void *)&w.ids[1],
                  (void *)&d->ctl, (void *)&cap, (void *)&d->res, (void *)&g->zero_bits, (void *)&sarg,
                  (void *)&sdev, (void *)&ns};
  {
    ktimer_scope kt(BYO_K_SMALL_LOOP, s);
    BYO_HIP(hipLaunchCooperativeKernel((const void *)bfs_persistent_kernel, dim3((unsigned)d->nblocks),
                                       dim3(PB_THREADS), args, 0, s));
  }
  pb_result r;
  BYO_TRY(sync_read(s, d->res, &r, sizeof(r)));
  // a failed wait leaves the barrier's counters mid-count
  if (r.fail) d->reset = true;
  BYO_CHECK(!r.fail, BYO_EHIP, "persistent BFS: a grid barrier wait timed out");
  if (stats) {
    std::memset(stats, 0, sizeof(*stats));
    stats->levels = r.levels;
    stats->device_levels = stats->levels;
    stats->variant_count[BYO_V_PUSH_BUCKET] = (int64_t)r.push_levels;
    stats->variant_count[BYO_V_PULL_THREAD] = (int64_t)r.pull_levels;
    stats->reached = (int64_t)r.reached;
    stats->edges = (int64_t)r.edges;
  }
  if (r.limit) return fail(BYO_ELIMIT, "BFS level cap reached");
  return BYO_OK;
}

}  // namespace byo
