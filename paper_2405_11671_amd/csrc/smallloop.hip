// Device-resident BFS levels for small frontiers. High-diameter graphs (road
// networks, lattices) spend thousands of levels with a few thousand frontier
// vertices each; there the host round trip of a level (launch, counter copy,
// sync) costs more than the level itself. One persistent kernel runs
// consecutive push levels with a grid barrier between them:
//  - a cooperative launch of 64 workgroups (eight per XCD), so every
//    workgroup is resident and the barrier cannot wait on one that never
//    started; on a 4096^2 lattice (8,191 levels) 256 workgroups took 17.4 us
//    a level, 64 took 14.6 us, 32 took 13.7 us (the host loop: 24.7 us);
//  - a two-level barrier: eight group counters (workgroup b in group b % 8,
//    which is also its XCD under round-robin placement), each on its own cache
//    line, then one top counter and a generation word. Every wait is bounded:
//    a wait that exceeds its budget sets a failure flag and every workgroup
//    leaves at its next barrier, so the kernel always finishes;
//  - the next frontier goes to eight sub-queues (one per group), each
//    workgroup staging its vertices in LDS and reserving space with one atomic
//    per level;
//  - the loop stops when the frontier is empty, when it (or its degree sum)
//    exceeds the caps, or after max_levels levels; the last frontier is
//    copied to one contiguous list for the host loop to take over.
#include <algorithm>
#include <cstring>

#include "gridsync.h"
#include "internal.h"

namespace byo {

constexpr int DL_THREADS = 256;
constexpr int DL_GROUPS = 8;
constexpr int DL_PAD = 32;             // counters 128 bytes apart
constexpr int DL_STAGE = 2048;         // LDS staging of one workgroup's outputs per level
constexpr int DL_MAX_BLOCKS = 64;      // workgroups in the loop (8 per XCD); fewer barrier arrivals per level
constexpr unsigned DL_SPIN_LIMIT = 1u << 21;
constexpr int64_t DL_QCAP = BYO_DLOOP_QCAP;  // entries per sub-queue (and the edge cap per level)

struct small_loop_result {
  int32_t levels;                  // levels completed
  int32_t side;                    // always 0: the final frontier is in out0
  int32_t empty;                   // 1 if the final frontier is empty (BFS finished)
  int32_t fail;                    // 1 if a barrier wait exceeded its budget
  unsigned long long count;        // size of the final frontier
  unsigned long long degsum;       // sum of its degrees
  unsigned long long reached;      // vertices emitted over all levels run
  unsigned long long edges;        // sum of their degrees
};

struct dl_ctl {
  grid_sync sync;
  unsigned qcount[3][DL_GROUPS * DL_PAD];              // per level mod 3, per group
  unsigned long long qdeg[3][DL_GROUPS * DL_PAD / 2];  // degree sums, same layout (8 bytes each)
};

struct dl_ws {
  int32_t *q[2] = {nullptr, nullptr};  // [DL_GROUPS][DL_QCAP] each
  dl_ctl *ctl = nullptr;
  small_loop_result *res = nullptr;
  int nblocks = 0;
  bool checked = false, usable = false;
};

__global__ void __launch_bounds__(DL_THREADS) bfs_device_loop_kernel(
    const int64_t *__restrict__ off, const int32_t *__restrict__ nbr, const int32_t *__restrict__ deg,
    int32_t *__restrict__ parent, int32_t *__restrict__ depth, uint64_t *__restrict__ visited,
    const int32_t *__restrict__ in_ids, int32_t k0, int32_t level0, int32_t max_levels, int64_t cap_count,
    int64_t cap_edges, int32_t *__restrict__ q0, int32_t *__restrict__ q1, dl_ctl *__restrict__ c,
    int32_t *__restrict__ out0, small_loop_result *__restrict__ res) {
  __shared__ int32_t stage[DL_STAGE];
  __shared__ unsigned s_cnt, s_base;
  __shared__ unsigned s_pre[DL_GROUPS + 1];
  const unsigned nblocks = gridDim.x;
  const int t = threadIdx.x;
  const unsigned grp = blockIdx.x % DL_GROUPS;
  unsigned long long reached = 0, edges = 0, last_deg = 0;
  unsigned long long kcur = (unsigned long long)k0;
  int levels = 0, empty = 0;
  for (int L = 0; L < max_levels; ++L) {
    const int p = L % 3, p1 = (L + 1) % 3, p2 = (L + 2) % 3;
    int32_t *qin = (L & 1) ? q1 : q0;
    int32_t *qout = (L & 1) ? q0 : q1;
    // input layout: level 0 reads in_ids, later levels the eight sub-queues
    if (t <= DL_GROUPS) {
      unsigned cnt = 0;
      if (t < DL_GROUPS) cnt = L == 0 ? (t == 0 ? (unsigned)k0 : 0u) : ld_rlx(&c->qcount[p][t * DL_PAD]);
      s_pre[t] = cnt;
    }
    if (t == 0) s_cnt = 0;
    // clear the counters this level's successor will write (consumed two levels ago)
    if (blockIdx.x == 0 && t < DL_GROUPS) {
      c->qcount[p2][t * DL_PAD] = 0u;
      c->qdeg[p2][t * DL_PAD / 2] = 0ull;
    }
    __syncthreads();
    if (t == 0) {
      unsigned acc = 0;
      for (int i = 0; i <= DL_GROUPS; ++i) {
        unsigned x = s_pre[i];
        s_pre[i] = acc;
        acc += (i < DL_GROUPS) ? x : 0u;
      }
    }
    __syncthreads();
    const unsigned K = s_pre[DL_GROUPS];
    const int32_t newdepth = level0 + L + 1;
    unsigned long long mydeg = 0;
    const unsigned stride = nblocks * DL_THREADS;
    for (unsigned base = blockIdx.x * DL_THREADS; base < K; base += stride) {
      const unsigned i = base + t;
      int32_t u = -1;
      int64_t b = 0, e = 0;
      if (i < K) {
        if (L == 0) {
          u = in_ids[i];
        } else {
          int gq = 0;
          while (gq + 1 < DL_GROUPS && s_pre[gq + 1] <= i) ++gq;
          u = qin[(int64_t)gq * DL_QCAP + (i - s_pre[gq])];
        }
        b = off[u];
        e = off[u + 1];
      }
      const bool wide = u >= 0 && e - b > 32;
      // emit v: LDS stage, or straight to this group's sub-queue when the stage is full
      auto emit = [&](int32_t v) {
        unsigned pos = atomicAdd(&s_cnt, 1u);
        if (pos < DL_STAGE) {
          stage[pos] = v;
        } else {
          unsigned gp = atomicAdd(&c->qcount[p1][grp * DL_PAD], 1u);
          qout[(int64_t)grp * DL_QCAP + gp] = v;
        }
        mydeg += (unsigned long long)deg[v];
      };
      if (u >= 0 && !wide) {
        for (int64_t x = b; x < e; ++x) {
          const int32_t v = nbr[x];
          const uint64_t bit = 1ull << (v & 63);
          if (visited[v >> 6] & bit) continue;
          if (atomicCAS(&parent[v], -1, u) != -1) continue;
          depth[v] = newdepth;
          atomicOr((unsigned long long *)&visited[v >> 6], (unsigned long long)bit);
          emit(v);
        }
      }
      uint64_t wm = __ballot(wide);
      while (wm) {
        const int l = __ffsll((long long)wm) - 1;
        wm &= wm - 1;
        const int32_t wu = read_lane_i32(u, l);
        const int64_t wb = (int64_t)read_lane_u64((uint64_t)b, l), we = (int64_t)read_lane_u64((uint64_t)e, l);
        for (int64_t x = wb + lane_id(); x < we; x += BYO_WAVE) {
          const int32_t v = nbr[x];
          const uint64_t bit = 1ull << (v & 63);
          if (visited[v >> 6] & bit) continue;
          if (atomicCAS(&parent[v], -1, wu) != -1) continue;
          depth[v] = newdepth;
          atomicOr((unsigned long long *)&visited[v >> 6], (unsigned long long)bit);
          emit(v);
        }
      }
    }
    // flush the stage with one reservation; add this workgroup's degree sum
    const unsigned long long bdeg = block_sum<unsigned long long, DL_THREADS>(mydeg);
    __syncthreads();
    const unsigned staged = s_cnt < (unsigned)DL_STAGE ? s_cnt : (unsigned)DL_STAGE;
    if (t == 0) {
      s_base = staged ? atomicAdd(&c->qcount[p1][grp * DL_PAD], staged) : 0u;
      if (bdeg) atomicAdd(&c->qdeg[p1][grp * DL_PAD / 2], bdeg);
    }
    __syncthreads();
    for (unsigned j = t; j < staged; j += DL_THREADS) qout[(int64_t)grp * DL_QCAP + s_base + j] = stage[j];
    if (!grid_barrier(&c->sync, nblocks, DL_SPIN_LIMIT)) break;
    // every workgroup reads the same totals and takes the same decision
    unsigned long long kn = 0, dn = 0;
    for (int gq = 0; gq < DL_GROUPS; ++gq) {
      kn += ld_rlx(&c->qcount[p1][gq * DL_PAD]);
      dn += ld_rlx64(&c->qdeg[p1][gq * DL_PAD / 2]);
    }
    levels = L + 1;
    reached += kn;
    edges += dn;
    last_deg = dn;
    kcur = kn;
    if (kn == 0) {
      empty = 1;
      break;
    }
    if ((int64_t)kn > cap_count || (int64_t)dn > cap_edges) break;
  }
  // hand the last frontier back as one list (levels run >= 1 here unless a barrier failed)
  const int Lf = levels;
  if (!empty && Lf > 0 && !ld_rlx(&c->sync.fail[0])) {
    const int p = Lf % 3;
    int32_t *qin = (Lf & 1) ? q1 : q0;
    unsigned pre[DL_GROUPS + 1];
    pre[0] = 0;
    for (int gq = 0; gq < DL_GROUPS; ++gq) pre[gq + 1] = pre[gq] + ld_rlx(&c->qcount[p][gq * DL_PAD]);
    for (unsigned i = blockIdx.x * DL_THREADS + t; i < pre[DL_GROUPS]; i += nblocks * DL_THREADS) {
      int gq = 0;
      while (gq + 1 < DL_GROUPS && pre[gq + 1] <= i) ++gq;
      out0[i] = qin[(int64_t)gq * DL_QCAP + (i - pre[gq])];
    }
  }
  if (blockIdx.x == 0 && t == 0) {
    res->levels = levels;
    res->side = 0;
    res->empty = empty;
    res->fail = ld_rlx(&c->sync.fail[0]) ? 1 : 0;
    res->count = empty ? 0ull : kcur;
    res->degsum = empty ? 0ull : last_deg;
    res->reached = reached;
    res->edges = edges;
  }
}

void dl_release(byo_workspace &w) {
  if (!w.dloop) return;
  dl_ws *d = (dl_ws *)w.dloop;
  void *p[] = {d->q[0], d->q[1], d->ctl, d->res};
  for (void *x : p)
    if (x) (void)hipFree(x);
  delete d;
  w.dloop = nullptr;
}

static byo_status dl_ensure(byo_graph *g, dl_ws **out) {
  byo_workspace &w = g->ws;
  if (!w.dloop) w.dloop = new dl_ws();
  dl_ws *d = (dl_ws *)w.dloop;
  *out = d;
  if (d->checked) return BYO_OK;
  d->checked = true;
  int dev = 0, coop = 0, cus = 0, per_cu = 0;
  BYO_HIP(hipGetDevice(&dev));
  BYO_HIP(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev));
  BYO_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  BYO_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, bfs_device_loop_kernel, DL_THREADS, 0));
  if (!coop || cus <= 0 || per_cu <= 0) return BYO_OK;  // not usable: the host loop runs every level
  d->nblocks = std::min(cus, DL_MAX_BLOCKS);
  BYO_HIP(hipMalloc(&d->q[0], sizeof(int32_t) * DL_GROUPS * DL_QCAP));
  BYO_HIP(hipMalloc(&d->q[1], sizeof(int32_t) * DL_GROUPS * DL_QCAP));
  BYO_HIP(hipMalloc(&d->ctl, sizeof(dl_ctl)));
  BYO_HIP(hipMalloc(&d->res, sizeof(small_loop_result)));
  d->usable = true;
  return BYO_OK;
}

bool bfs_small_loop_usable(byo_graph *g) {
  dl_ws *d = nullptr;
  if (dl_ensure(g, &d) != BYO_OK) return false;
  return d->usable;
}

byo_status bfs_small_loop(byo_graph *g, const int32_t *in_ids, int64_t k, int64_t in_degsum, int32_t level,
                          int32_t max_levels, int64_t cap_count, int64_t cap_edges, int32_t *parent, int32_t *depth,
                          uint64_t *visited, int32_t *out, hipStream_t s, small_loop_out *res_out) {
  dl_ws *d = nullptr;
  BYO_TRY(dl_ensure(g, &d));
  BYO_CHECK(d->usable, BYO_ESTATE, "cooperative launch not available for the device-resident loop");
  // every level's output fits a sub-queue: a level runs only when its input's
  // degree sum is within the edge cap, and the outputs are at most that sum
  cap_edges = std::min<int64_t>(cap_edges, DL_QCAP);
  cap_count = std::min<int64_t>(cap_count, DL_QCAP);
  BYO_CHECK(k >= 1 && k <= cap_count, BYO_EINVAL, "device-resident loop needs 1 <= |U| <= its frontier cap");
  BYO_CHECK(in_degsum >= 0 && in_degsum <= cap_edges, BYO_EINVAL, "device-resident loop: frontier degree sum too large");
  BYO_CHECK(max_levels >= 1, BYO_EINVAL, "device-resident loop needs a level budget");
  BYO_HIP(hipMemsetAsync(d->ctl, 0, sizeof(dl_ctl), s));
  const int32_t k0 = (int32_t)k;
  void *args[] = {(void *)&g->off, (void *)&g->nbr, (void *)&g->deg, (void *)&parent, (void *)&depth,
                  (void *)&visited, (void *)&in_ids, (void *)&k0, (void *)&level, (void *)&max_levels,
                  (void *)&cap_count, (void *)&cap_edges, (void *)&d->q[0], (void *)&d->q[1], (void *)&d->ctl,
                  (void *)&out, (void *)&d->res};
  {
    ktimer_scope kt(BYO_K_SMALL_LOOP, s);
    BYO_HIP(hipLaunchCooperativeKernel((const void *)bfs_device_loop_kernel, dim3((unsigned)d->nblocks),
                                       dim3(DL_THREADS), args, 0, s));
  }
  small_loop_result r;
  BYO_TRY(sync_read(s, d->res, &r, sizeof(r)));
  BYO_CHECK(!r.fail, BYO_EHIP, "device-resident loop: a grid barrier wait timed out");
  res_out->levels = r.levels;
  res_out->side = r.side;
  res_out->empty = r.empty != 0;
  res_out->count = (int64_t)r.count;
  res_out->degsum = (int64_t)r.degsum;
  res_out->reached = (int64_t)r.reached;
  res_out->edges = (int64_t)r.edges;
  return BYO_OK;
}

}  // namespace byo
