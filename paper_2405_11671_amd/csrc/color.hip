// Graph colouring (Table algs-list, covering problems): the greedy colouring
// in a priority order (ascending priority, ties by vertex ID), where each
// vertex in turn takes the smallest colour no earlier neighbour holds. On the
// GPU it runs in rounds: an uncoloured vertex whose earlier neighbours are all
// coloured takes the smallest colour missing among them; one with an
// uncoloured earlier neighbour waits. Colours are final and depend only on
// earlier vertices, so rounds update in place and the result equals the
// sequential greedy colouring.
#include <algorithm>
#include <cstring>

#include "internal.h"

namespace byo {

namespace {

constexpr int CO_BLOCK = 256;
constexpr int32_t CO_WAVE_MIN = 32;   // lists longer than this are scanned by the wavefront
constexpr int32_t CO_WAVE_COLORS = 64 * BYO_WAVE;  // colours a wavefront's LDS bitmap holds

__device__ __forceinline__ bool co_before(uint64_t pu, int32_t u, uint64_t pv, int32_t v) {
  return pu < pv || (pu == pv && u < v);
}

// does an earlier neighbour of v (list [beg, end)) hold colour c? (one lane)
__device__ bool co_lane_holds(const int32_t *__restrict__ nbr, const uint64_t *__restrict__ prio,
                              const int32_t *color, int64_t beg, int64_t end, int32_t v, uint64_t pv, int32_t c) {
  for (int64_t e = beg; e < end; ++e) {
    const int32_t u = nbr[e];
    if (co_before(prio[u], u, pv, v) && color[u] == c) return true;
  }
  return false;
}

template <bool WAVE>
__global__ void __launch_bounds__(CO_BLOCK) co_round_kernel(const int64_t *__restrict__ off,
                                                            const int32_t *__restrict__ nbr,
                                                            const uint64_t *__restrict__ prio,
                                                            const int32_t *__restrict__ ids, int64_t k,
                                                            int32_t *color, int32_t *out, byo_counters *ctr,
                                                            byo_counters *ctr_clear) {
  __shared__ unsigned long long used[CO_BLOCK / BYO_WAVE][BYO_WAVE];
  unsigned long long *row = used[threadIdx.x / BYO_WAVE];
  for (int64_t base = (int64_t)blockIdx.x * CO_BLOCK; base < k; base += (int64_t)gridDim.x * CO_BLOCK) {
    const int64_t i = base + threadIdx.x;
    int32_t v = 0;
    int64_t beg = 0, end = 0;
    uint64_t pv = 0;
    if (i < k) {
      v = ids[i];
      beg = off[v];
      end = off[v + 1];
      pv = prio[v];
    }
    const bool coop = WAVE && end - beg > CO_WAVE_MIN;
    bool wait = false;
    int32_t col = -1;
    if (i < k && !coop) {
      uint64_t mask = 0;  // colours 0..63 held by earlier neighbours
      for (int64_t e = beg; e < end && !wait; ++e) {
        const int32_t u = nbr[e];
        if (!co_before(prio[u], u, pv, v)) continue;
        const int32_t c = color[u];
        wait = c < 0;
        if (c >= 0 && c < 64) mask |= 1ull << c;
      }
      if (!wait) {
        if (~mask) {
          col = __ffsll((long long)~mask) - 1;
        } else {
          int32_t c = 64;
          while (co_lane_holds(nbr, prio, color, beg, end, v, pv, c)) ++c;
          col = c;
        }
      }
    }
    if (WAVE) {
      uint64_t pm = __ballot(i < k && coop);
      while (pm) {
        const int l = __ffsll((long long)pm) - 1;
        pm &= pm - 1;
        const int64_t lb = (int64_t)read_lane_u64((uint64_t)beg, l), le = (int64_t)read_lane_u64((uint64_t)end, l);
        const int32_t vl = read_lane_i32(v, l);
        const uint64_t pl = read_lane_u64(pv, l);
        row[lane_id()] = 0ull;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        bool any_wait = false;
        for (int64_t e0 = lb; e0 < le && !any_wait; e0 += BYO_WAVE) {
          const int64_t e = e0 + lane_id();
          int32_t c = -2;  // -2: not an earlier neighbour
          if (e < le) {
            const int32_t u = nbr[e];
            if (co_before(prio[u], u, pl, vl)) c = color[u];
          }
          any_wait = __ballot(c == -1) != 0;
          if (c >= 0 && c < CO_WAVE_COLORS) atomicOr(&row[c >> 6], 1ull << (c & 63));
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        __builtin_amdgcn_wave_barrier();
        int32_t cl = -1;
        if (!any_wait) {
          const uint64_t free_bits = ~row[lane_id()];
          const uint64_t lanes = __ballot(free_bits != 0);
          if (lanes) {
            const int lf = __ffsll((long long)lanes) - 1;
            const uint64_t fb = read_lane_u64(free_bits, lf);
            cl = lf * 64 + (__ffsll((long long)fb) - 1);
          } else {
            // every colour below CO_WAVE_COLORS is taken: test larger ones in turn
            int32_t c = CO_WAVE_COLORS;
            while (true) {
              bool held = false;
              for (int64_t e = lb + lane_id(); e < le; e += BYO_WAVE) {
                const int32_t u = nbr[e];
                if (co_before(prio[u], u, pl, vl) && color[u] == c) held = true;
              }
              if (!__ballot(held)) break;
              ++c;
            }
            cl = c;
          }
        }
        __builtin_amdgcn_wave_barrier();
        if (lane_id() == l) {
          wait = any_wait;
          col = cl;
        }
      }
    }
    if (i < k && !wait) color[v] = col;
    wave_append(i < k && wait, v, out, &ctr->count);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0 && ctr_clear) {
    ctr_clear->count = 0;
    ctr_clear->degsum = 0;
    ctr_clear->aux0 = 0;
    ctr_clear->aux1 = 0;
  }
}

__global__ void co_init_kernel(int64_t n, int32_t *color, int32_t *ids, byo_counters *ctr) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    color[v] = -1;
    ids[v] = (int32_t)v;
  }
  if (blockIdx.x == 0 && threadIdx.x < BYO_COUNTER_SLOTS) {
    ctr[threadIdx.x].count = 0;
    ctr[threadIdx.x].degsum = 0;
    ctr[threadIdx.x].aux0 = 0;
    ctr[threadIdx.x].aux1 = 0;
  }
}

unsigned co_grid(int64_t count, int64_t per, int64_t cap) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>((count + per - 1) / per, cap));
}

}  // namespace

}  // namespace byo

using namespace byo;

extern "C" byo_status byo_coloring(byo_graph *g, const uint64_t *d_prio, int32_t *d_color, const byo_opts *opts,
                                   void *stream, byo_run_stats *stats) {
  BYO_CHECK(g && d_prio && d_color, BYO_EINVAL, "null argument");
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
  co_init_kernel<<<co_grid(n, 256, 8192), 256, 0, s>>>(n, d_color, w.ids[0], w.ctr);
  BYO_HIP(hipGetLastError());
  const bool wave = !(o.selector == BYO_SEL_FIXED && (o.fixed_variant == BYO_V_PUSH_THREAD ||
                                                      o.fixed_variant == BYO_V_PULL_THREAD));
  const int64_t cap = o.max_levels > 0 ? o.max_levels : n + 1;
  int64_t k = n;
  int cur = 0;
  int32_t round = 0;
  while (k > 0) {
    if (round >= cap) {
      if (stats) *stats = st;
      return fail(BYO_ELIMIT, "colouring round cap reached");
    }
    byo_counters *c = w.ctr + (round % BYO_COUNTER_SLOTS);
    byo_counters *cc = w.ctr + ((round + 2) % BYO_COUNTER_SLOTS);
    if (wave)
      co_round_kernel<true><<<co_grid(k, CO_BLOCK, 16384), CO_BLOCK, 0, s>>>(g->off, g->nbr, d_prio, w.ids[cur], k,
                                                                             d_color, w.ids[1 - cur], c, cc);
    else
      co_round_kernel<false><<<co_grid(k, CO_BLOCK, 16384), CO_BLOCK, 0, s>>>(g->off, g->nbr, d_prio, w.ids[cur], k,
                                                                              d_color, w.ids[1 - cur], c, cc);
    BYO_HIP(hipGetLastError());
    BYO_HIP(hipMemcpyAsync(w.h_ctr + (round % BYO_COUNTER_SLOTS), c, sizeof(byo_counters), hipMemcpyDeviceToHost, s));
    BYO_HIP(hipStreamSynchronize(s));
    k = (int64_t)w.h_ctr[round % BYO_COUNTER_SLOTS].count;
    st.variant_count[wave ? BYO_V_PULL_WAVE : BYO_V_PULL_THREAD]++;
    ++round;
    cur = 1 - cur;
  }
  st.levels = round;
  st.reached = n;
  if (stats) *stats = st;
  return BYO_OK;
}
