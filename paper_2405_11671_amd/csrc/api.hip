// Container-API ablation (Section 4.2 defines the GraphContainer API, Table
// api-components-avg measures configurations that leave optional functions
// out). Without degree() the framework obtains a degree by mapping over the
// vertex's neighbours and counting them; without num_edges() it sums the
// degrees over all vertices whenever it needs m. The maps below read every
// neighbour and count the valid ids (u >= 0), so the count is not folded into
// the row bounds: they cost what the container would cost the framework.
//
// With the container's parallel map the count of one list is spread like the
// traversal's own parallel maps: a lane counts a list of up to AP_LANE
// entries, the wavefront one of up to AP_CHUNK, and longer lists are queued
// for a pass over AP_CHUNK-entry chunks spread across the GPU. Without it
// every list is counted by one lane.
#include "internal.h"

namespace byo {

namespace {

constexpr int AP_THREADS = 256;
constexpr int64_t AP_LANE = 32;
constexpr int64_t AP_CHUNK = 4096;
constexpr int64_t AP_MAX_BLOCKS = 1024;  // one atomic per workgroup into the sums
constexpr int AP_ILP = 8;

unsigned ap_blocks(int64_t count) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>((count + AP_THREADS - 1) / AP_THREADS, AP_MAX_BLOCKS));
}

// entries of nbr[beg, end) counted by one lane
__device__ __forceinline__ int32_t lane_count(const int32_t *__restrict__ nbr, int64_t beg, int64_t end) {
  int32_t c = 0;
  for (int64_t e = beg; e < end; e += AP_ILP) {
    int32_t u[AP_ILP];
#pragma unroll
    for (int j = 0; j < AP_ILP; ++j) u[j] = e + j < end ? nbr[e + j] : -1;
#pragma unroll
    for (int j = 0; j < AP_ILP; ++j) c += u[j] >= 0;
  }
  return c;
}

// entries of nbr[beg, end) counted by `width` lanes from lane offset `lane`
__device__ __forceinline__ int32_t strided_count(const int32_t *__restrict__ nbr, int64_t beg, int64_t end, int lane,
                                                 int width) {
  int32_t c = 0;
  for (int64_t e = beg + lane; e < end; e += (int64_t)AP_ILP / 2 * width) {
    int32_t u[AP_ILP / 2];
#pragma unroll
    for (int j = 0; j < AP_ILP / 2; ++j) u[j] = e + (int64_t)j * width < end ? nbr[e + (int64_t)j * width] : -1;
#pragma unroll
    for (int j = 0; j < AP_ILP / 2; ++j) c += u[j] >= 0;
  }
  return c;
}

// The degrees of a vertex set (ids[0..k), else the set bits of bits, else
// every vertex) into mdeg, and their sum into aux[0]. PAR: lists longer than
// AP_CHUNK get mdeg 0 here and go to heavy[] (count in aux[1]) for the chunk
// pass.
template <bool PAR>
__global__ void __launch_bounds__(AP_THREADS) ap_degree_kernel(const int64_t *__restrict__ off,
                                                               const int32_t *__restrict__ nbr,
                                                               const int32_t *__restrict__ ids,
                                                               const uint64_t *__restrict__ bits, int64_t k,
                                                               int64_t n, int32_t *mdeg, int32_t *heavy,
                                                               unsigned long long *aux) {
  unsigned long long acc = 0;
  const int64_t range = ids ? k : n;
  // uniform trip count per workgroup: every lane reaches the wavefront scans
  for (int64_t base = (int64_t)blockIdx.x * AP_THREADS; base < range; base += (int64_t)gridDim.x * AP_THREADS) {
    const int64_t i = base + threadIdx.x;
    int64_t u = -1;
    if (i < range) {
      if (ids) u = ids[i];
      else if (!bits || ((bits[i >> 6] >> (i & 63)) & 1ull)) u = i;
    }
    int64_t beg = 0, end = 0;
    if (u >= 0) {
      beg = off[u];
      end = off[u + 1];
    }
    const bool lane = u >= 0 && (!PAR || end - beg <= AP_LANE);
    int32_t d = lane ? lane_count(nbr, beg, end) : 0;
    if (PAR) {
      const bool chunked = u >= 0 && end - beg > AP_CHUNK;
      uint64_t pm = __ballot(u >= 0 && !lane && !chunked);
      while (pm) {
        const int l = __ffsll((long long)pm) - 1;
        pm &= pm - 1;
        const int64_t lb = (int64_t)read_lane_u64((uint64_t)beg, l);
        const int64_t le = (int64_t)read_lane_u64((uint64_t)end, l);
        const int32_t c = wave_sum(strided_count(nbr, lb, le, lane_id(), BYO_WAVE));
        if (lane_id() == l) d = c;
      }
      wave_append(chunked, (int32_t)u, heavy, aux + 1);
    }
    if (u >= 0) {
      mdeg[u] = d;
      acc += (unsigned long long)d;
    }
  }
  const unsigned long long t = block_sum<unsigned long long, AP_THREADS>(acc);
  if (threadIdx.x == 0 && t) atomicAdd(aux, t);
}

// One workgroup: pre[h] = chunks of the queued lists before h, aux[2] = all
// chunks.
__global__ void __launch_bounds__(AP_THREADS) ap_chunk_scan_kernel(const int64_t *__restrict__ off,
                                                                   const int32_t *__restrict__ heavy,
                                                                   int64_t *__restrict__ pre,
                                                                   unsigned long long *aux) {
  __shared__ int64_t sh[AP_THREADS];
  const int64_t nh = (int64_t)aux[1];
  int64_t carry = 0;
  for (int64_t base = 0; base < nh; base += AP_THREADS) {
    const int64_t h = base + threadIdx.x;
    int64_t c = 0;
    if (h < nh) {
      const int32_t u = heavy[h];
      c = (off[u + 1] - off[u] + AP_CHUNK - 1) / AP_CHUNK;
    }
    sh[threadIdx.x] = c;
    __syncthreads();
    for (int d = 1; d < AP_THREADS; d <<= 1) {
      const int64_t t = threadIdx.x >= (unsigned)d ? sh[threadIdx.x - d] : 0;
      __syncthreads();
      sh[threadIdx.x] += t;
      __syncthreads();
    }
    if (h < nh) pre[h] = carry + sh[threadIdx.x] - c;
    carry += sh[AP_THREADS - 1];
    __syncthreads();
  }
  if (threadIdx.x == 0) aux[2] = (unsigned long long)carry;
}

// The queued long lists' chunks, one per wavefront and step: chunk t belongs
// to the last list h with pre[h] <= t; its count goes to mdeg[u] and the sum.
__global__ void __launch_bounds__(AP_THREADS) ap_heavy_kernel(const int64_t *__restrict__ off,
                                                              const int32_t *__restrict__ nbr,
                                                              const int32_t *__restrict__ heavy,
                                                              const int64_t *__restrict__ pre, int32_t *mdeg,
                                                              unsigned long long *aux) {
  const int64_t nh = (int64_t)aux[1], total = (int64_t)aux[2];
  const int64_t nwaves = (int64_t)gridDim.x * (AP_THREADS / BYO_WAVE);
  unsigned long long acc = 0;
  for (int64_t t = (int64_t)blockIdx.x * (AP_THREADS / BYO_WAVE) + threadIdx.x / BYO_WAVE; t < total; t += nwaves) {
    int64_t lo = 0, hi = nh - 1;  // pre[lo] <= t throughout (pre[0] = 0)
    while (lo < hi) {
      const int64_t mid = (lo + hi + 1) >> 1;
      if (pre[mid] <= t) lo = mid;
      else hi = mid - 1;
    }
    const int32_t u = heavy[lo];
    const int64_t beg = off[u], end = off[u + 1];
    const int64_t cb = beg + (t - pre[lo]) * AP_CHUNK, ce = cb + AP_CHUNK < end ? cb + AP_CHUNK : end;
    const int32_t cnt = wave_sum(strided_count(nbr, cb, ce, lane_id(), BYO_WAVE));
    if (lane_id() == 0) {
      atomicAdd(&mdeg[u], cnt);
      acc += (unsigned long long)cnt;
    }
  }
  const unsigned long long s = block_sum<unsigned long long, AP_THREADS>(acc);
  if (threadIdx.x == 0 && s) atomicAdd(aux, s);
}

// m as the sum of degree() over all vertices
__global__ void __launch_bounds__(AP_THREADS) ap_degree_sum_kernel(const int32_t *__restrict__ deg, int64_t n,
                                                                   unsigned long long *sum) {
  unsigned long long acc = 0;
  for (int64_t v = (int64_t)blockIdx.x * AP_THREADS + threadIdx.x; v < n; v += (int64_t)gridDim.x * AP_THREADS)
    acc += (unsigned long long)deg[v];
  const unsigned long long t = block_sum<unsigned long long, AP_THREADS>(acc);
  if (threadIdx.x == 0 && t) atomicAdd(sum, t);
}

__global__ void ap_zero_aux_kernel(unsigned long long *aux) {
  if (threadIdx.x < 4) aux[threadIdx.x] = 0ull;
}

byo_status ap_buffers(byo_graph *g, hipStream_t s) {
  byo_workspace &w = g->ws;
  if (w.api_deg) return BYO_OK;
  const int64_t n1 = std::max<int64_t>(g->n, 1);
  BYO_HIP(hipMalloc(&w.api_heavy, sizeof(int32_t) * (size_t)(g->m / AP_CHUNK + 1)));
  BYO_HIP(hipMalloc(&w.api_pre, sizeof(int64_t) * (size_t)(g->m / AP_CHUNK + 1)));
  BYO_HIP(hipMalloc(&w.api_aux, 4 * sizeof(unsigned long long)));
  BYO_HIP(hipMalloc(&w.api_deg, sizeof(int32_t) * (size_t)n1));
  // entries not yet mapped read as 0, never as stale memory
  return fill_i32(w.api_deg, n1, 0, s);
}

// mdeg for the set (see ap_degree_kernel), the sum left in aux[0]
byo_status ap_map(byo_graph *g, uint32_t omit, const int32_t *ids, const uint64_t *bits, int64_t k, hipStream_t s) {
  BYO_TRY(ap_buffers(g, s));
  byo_workspace &w = g->ws;
  const int64_t range = ids ? k : g->n;
  ap_zero_aux_kernel<<<1, 64, 0, s>>>(w.api_aux);
  if (omit & BYO_API_NO_PAR_MAP) {
    ap_degree_kernel<false><<<ap_blocks(range), AP_THREADS, 0, s>>>(g->off, g->nbr, ids, bits, k, g->n, w.api_deg,
                                                                     w.api_heavy, w.api_aux);
  } else {
    ap_degree_kernel<true><<<ap_blocks(range), AP_THREADS, 0, s>>>(g->off, g->nbr, ids, bits, k, g->n, w.api_deg,
                                                                    w.api_heavy, w.api_aux);
    ap_chunk_scan_kernel<<<1, AP_THREADS, 0, s>>>(g->off, w.api_heavy, w.api_pre, w.api_aux);
    ap_heavy_kernel<<<(unsigned)AP_MAX_BLOCKS, AP_THREADS, 0, s>>>(g->off, g->nbr, w.api_heavy, w.api_pre, w.api_deg,
                                                                   w.api_aux);
  }
  BYO_HIP(hipGetLastError());
  return BYO_OK;
}

}  // namespace

byo_status api_degree_buffer(byo_graph *g, hipStream_t s, int32_t **out) {
  BYO_TRY(ap_buffers(g, s));
  *out = g->ws.api_deg;
  return BYO_OK;
}

byo_status api_frontier_degrees(byo_graph *g, uint32_t omit, const int32_t *ids, const uint64_t *bits, int64_t k,
                                hipStream_t s, int64_t *degsum) {
  BYO_CHECK(ids || bits, BYO_EINVAL, "frontier needs ids or a bitmap");
  BYO_TRY(ap_map(g, omit, ids, bits, k, s));
  unsigned long long h = 0;
  BYO_TRY(sync_read(s, g->ws.api_aux, &h, sizeof(h)));
  *degsum = (int64_t)h;
  return BYO_OK;
}

byo_status api_map_degrees(byo_graph *g, uint32_t omit, hipStream_t s, int32_t **mdeg) {
  BYO_TRY(ap_map(g, omit, nullptr, nullptr, 0, s));
  *mdeg = g->ws.api_deg;
  return BYO_OK;
}

byo_status api_num_edges(byo_graph *g, uint32_t omit, const int32_t *deg, hipStream_t s, int64_t *m) {
  if (!(omit & BYO_API_NO_NUM_EDGES)) {
    *m = g->m;
    return BYO_OK;
  }
  if (omit & BYO_API_NO_DEGREE) {
    // every degree by mapping
    BYO_TRY(ap_map(g, omit, nullptr, nullptr, 0, s));
  } else {
    BYO_TRY(ap_buffers(g, s));
    ap_zero_aux_kernel<<<1, 64, 0, s>>>(g->ws.api_aux);
    ap_degree_sum_kernel<<<ap_blocks(g->n), AP_THREADS, 0, s>>>(deg, g->n, g->ws.api_aux);
    BYO_HIP(hipGetLastError());
  }
  unsigned long long h = 0;
  BYO_TRY(sync_read(s, g->ws.api_aux, &h, sizeof(h)));
  *m = (int64_t)h;
  return BYO_OK;
}

int api_variant(uint32_t omit, int v, bool early_exit_pull) {
  // the wavefront-cooperative pull is the parallel early-exit map for BFS and
  // the parallel map (a min over the whole list) for connectivity
  const uint32_t coop = early_exit_pull ? BYO_API_NO_PAR_EARLY_EXIT : BYO_API_NO_PAR_MAP;
  if (v == BYO_V_PULL_WAVE) return (omit & coop) ? BYO_V_PULL_THREAD : v;
  if (v == BYO_V_PULL_THREAD) return v;
  // push over one vertex's list by a wavefront, workgroup or edge range is
  // the parallel map
  return (omit & BYO_API_NO_PAR_MAP) ? BYO_V_PUSH_THREAD : v;
}

}  // namespace byo
