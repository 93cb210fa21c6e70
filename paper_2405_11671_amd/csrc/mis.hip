// Maximal independent set (Table algs-list, covering problems): the greedy
// MIS in a priority order (ascending priority, ties by vertex ID), computed in
// rounds on the GPU. In a round every undecided vertex v looks at the
// neighbours that come before it in the order: if one of them is in the set, v
// is out; if all of them are out, v is in; otherwise v waits. Decisions are
// final and depend only on earlier vertices, so each round updates the status
// in place and the result equals the sequential greedy one.
#include <algorithm>
#include <cstring>

#include "internal.h"

namespace byo {

namespace {

constexpr int MIS_BLOCK = 256;
constexpr int32_t MIS_WAVE_MIN = 32;  // lists longer than this are scanned by the wavefront
constexpr uint8_t MIS_UNDECIDED = 0, MIS_IN = 1, MIS_OUT = 2;

__device__ __forceinline__ bool mis_before(uint64_t pu, int32_t u, uint64_t pv, int32_t v) {
  return pu < pv || (pu == pv && u < v);
}

// One round over the undecided vertices ids[0..k); those still undecided are
// appended to out (count in ctr->count).
template <bool WAVE>
__global__ void __launch_bounds__(MIS_BLOCK) mis_round_kernel(const int64_t *__restrict__ off,
                                                              const int32_t *__restrict__ nbr,
                                                              const uint64_t *__restrict__ prio,
                                                              const int32_t *__restrict__ ids, int64_t k,
                                                              uint8_t *status, int32_t *out, byo_counters *ctr,
                                                              byo_counters *ctr_clear) {
  for (int64_t base = (int64_t)blockIdx.x * MIS_BLOCK; base < k; base += (int64_t)gridDim.x * MIS_BLOCK) {
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
    const bool coop = WAVE && end - beg > MIS_WAVE_MIN;
    bool in_nb = false, blocked = false;
    if (i < k && !coop)
      for (int64_t e = beg; e < end && !in_nb; ++e) {
        const int32_t u = nbr[e];
        if (!mis_before(prio[u], u, pv, v)) continue;
        const uint8_t su = status[u];
        in_nb = su == MIS_IN;
        blocked |= su == MIS_UNDECIDED;
      }
    if (WAVE) {
      uint64_t pm = __ballot(i < k && coop);
      while (pm) {
        const int l = __ffsll((long long)pm) - 1;
        pm &= pm - 1;
        const int64_t lb = (int64_t)read_lane_u64((uint64_t)beg, l), le = (int64_t)read_lane_u64((uint64_t)end, l);
        const int32_t vl = read_lane_i32(v, l);
        const uint64_t pl = read_lane_u64(pv, l);
        bool any_in = false, any_wait = false;
        for (int64_t e0 = lb; e0 < le && !any_in; e0 += BYO_WAVE) {
          const int64_t e = e0 + lane_id();
          uint8_t su = MIS_OUT;
          if (e < le) {
            const int32_t u = nbr[e];
            if (mis_before(prio[u], u, pl, vl)) su = status[u];
          }
          any_in = __ballot(su == MIS_IN) != 0;
          any_wait |= __ballot(su == MIS_UNDECIDED) != 0;
        }
        if (lane_id() == l) {
          in_nb = any_in;
          blocked = any_wait;
        }
      }
    }
    bool wait = false;
    if (i < k) {
      if (in_nb) status[v] = MIS_OUT;
      else if (!blocked) status[v] = MIS_IN;
      else wait = true;
    }
    wave_append(wait, v, out, &ctr->count);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0 && ctr_clear) {
    ctr_clear->count = 0;
    ctr_clear->degsum = 0;
    ctr_clear->aux0 = 0;
    ctr_clear->aux1 = 0;
  }
}

__global__ void mis_init_kernel(int64_t n, uint8_t *status, int32_t *ids, byo_counters *ctr) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    status[v] = MIS_UNDECIDED;
    ids[v] = (int32_t)v;
  }
  if (blockIdx.x == 0 && threadIdx.x < BYO_COUNTER_SLOTS) {
    ctr[threadIdx.x].count = 0;
    ctr[threadIdx.x].degsum = 0;
    ctr[threadIdx.x].aux0 = 0;
    ctr[threadIdx.x].aux1 = 0;
  }
}

// membership from the status: 1 in the set, 0 out
__global__ void mis_finish_kernel(int64_t n, uint8_t *status) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
    status[v] = status[v] == MIS_IN ? 1 : 0;
}

unsigned mis_grid(int64_t count, int64_t per, int64_t cap) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>((count + per - 1) / per, cap));
}

}  // namespace

}  // namespace byo

using namespace byo;

extern "C" byo_status byo_mis(byo_graph *g, const uint64_t *d_prio, uint8_t *d_in_set, const byo_opts *opts,
                              void *stream, byo_run_stats *stats) {
  BYO_CHECK(g && d_prio && d_in_set, BYO_EINVAL, "null argument");
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
  // d_in_set doubles as the status array until the last pass
  mis_init_kernel<<<mis_grid(n, 256, 8192), 256, 0, s>>>(n, d_in_set, w.ids[0], w.ctr);
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
      return fail(BYO_ELIMIT, "independent-set round cap reached");
    }
    byo_counters *c = w.ctr + (round % BYO_COUNTER_SLOTS);
    byo_counters *cc = w.ctr + ((round + 2) % BYO_COUNTER_SLOTS);
    if (wave)
      mis_round_kernel<true><<<mis_grid(k, MIS_BLOCK, 16384), MIS_BLOCK, 0, s>>>(g->off, g->nbr, d_prio, w.ids[cur], k,
                                                                                 d_in_set, w.ids[1 - cur], c, cc);
    else
      mis_round_kernel<false><<<mis_grid(k, MIS_BLOCK, 16384), MIS_BLOCK, 0, s>>>(
          g->off, g->nbr, d_prio, w.ids[cur], k, d_in_set, w.ids[1 - cur], c, cc);
    BYO_HIP(hipGetLastError());
    BYO_HIP(hipMemcpyAsync(w.h_ctr + (round % BYO_COUNTER_SLOTS), c, sizeof(byo_counters), hipMemcpyDeviceToHost, s));
    BYO_HIP(hipStreamSynchronize(s));
    k = (int64_t)w.h_ctr[round % BYO_COUNTER_SLOTS].count;
    st.variant_count[wave ? BYO_V_PULL_WAVE : BYO_V_PULL_THREAD]++;
    ++round;
    cur = 1 - cur;
  }
  mis_finish_kernel<<<mis_grid(n, 256, 8192), 256, 0, s>>>(n, d_in_set);
  BYO_HIP(hipGetLastError());
  st.levels = round;
  st.reached = n;
  if (stats) *stats = st;
  return BYO_OK;
}
