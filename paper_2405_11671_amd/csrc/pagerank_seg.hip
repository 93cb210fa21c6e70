// Cache-blocked PageRank pull (option pr_blocked). The gather contrib[u] over
// u in N(v) is split by source segment: segment s holds the neighbours u with
// u >> SEG_SHIFT == s, so a pass over segment s reads only a 2 MiB slice of
// contrib, which stays resident in every XCD's L2 (measured on RMAT-22: 94% L2
// hits against 52% for the single-pass pull). Both versions issue one L2
// request per gathered edge, and that request rate (about 1.2e11/s measured
// for either) bounds them, so blocking changes time only by a few percent; it
// is kept as an option, the single-pass pull is the default.
//
// Each segment keeps its own CSR (int32 offsets, int32 neighbours). A pass
// runs one wavefront per 64 rows: rows with at most t_wave entries in the
// segment are summed by their lane (8 independent gathers per step), longer
// ones by the whole wavefront, and rows above SEG_LONG entries by a workgroup
// of their own. Partial sums accumulate over segments in ascending order
// (acc, touched only where the row has entries in the segment), and the last
// pass applies p' = base + d * acc and writes the next contributions. Every
// summation order is fixed, so results are deterministic. Used when the
// contribution array exceeds one L2 and the segment count stays small (the
// per-segment offsets cost 4 bytes per vertex per segment per step).
#include <algorithm>
#include <vector>

#include "internal.h"

namespace byo {

constexpr int SEG_SHIFT = 19;     // 2^19 vertices = 2 MiB of FP32 contributions per segment
constexpr int SEG_LONG = 4096;    // segment entries above which a row gets its own workgroup
constexpr int SEG_BLOCK = 256;
constexpr int SEG_ILP = 8;
constexpr int SEG_MAX = 16;       // beyond this the offsets outweigh the saved fetches

struct pr_seg {
  int S = 0;
  int64_t n = 0;
  int32_t *seg_off = nullptr;     // [S][n + 1]
  int32_t *seg_nbr = nullptr;     // [m], segment s at [seg_start[s], seg_start[s + 1])
  int32_t *long_rows = nullptr;   // per segment, the rows with more than SEG_LONG entries
  float *acc = nullptr;           // [n]
  float *dpart = nullptr;         // dangling partials (max of init and last-pass block counts)
  std::vector<int64_t> seg_start; // S + 1
  std::vector<int64_t> long_start; // S + 1
  int64_t dpart_cap = 0;
};

bool pr_seg_wanted(const byo_graph *g) {
  int64_t S = (g->n + (1ll << SEG_SHIFT) - 1) >> SEG_SHIFT;
  return g->n > (1ll << 20) && S <= SEG_MAX && g->m >= 8 * g->n;
}

void pr_seg_release(byo_workspace &w) {
  if (!w.prseg) return;
  pr_seg *p = (pr_seg *)w.prseg;
  void *d[] = {p->seg_off, p->seg_nbr, p->long_rows, p->acc, p->dpart};
  for (void *x : d)
    if (x) (void)hipFree(x);
  delete p;
  w.prseg = nullptr;
}

__device__ __forceinline__ int64_t lower_bound_row(const int32_t *__restrict__ nbr, int64_t lo, int64_t hi, int32_t key) {
  while (lo < hi) {
    int64_t mid = (lo + hi) >> 1;
    if (nbr[mid] < key) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// cnt[s][v] = number of neighbours of v in segment s (rows are sorted, so each
// segment's part of a row is contiguous); cnt[s][n] = 0.
__global__ void seg_count_kernel(const int64_t *__restrict__ off, const int32_t *__restrict__ nbr, int64_t n, int S,
                                 int32_t *__restrict__ cnt) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v <= n; v += (int64_t)gridDim.x * blockDim.x) {
    if (v == n) {
      for (int s = 0; s < S; ++s) cnt[(int64_t)s * (n + 1) + n] = 0;
      continue;
    }
    int64_t prev = off[v], end = off[v + 1];
    for (int s = 0; s < S; ++s) {
      int64_t b = (s == S - 1) ? end : lower_bound_row(nbr, prev, end, (int32_t)((int64_t)(s + 1) << SEG_SHIFT));
      cnt[(int64_t)s * (n + 1) + v] = (int32_t)(b - prev);
      prev = b;
    }
  }
}

// Copy each row's segment parts to their segment CSRs.
__global__ void seg_scatter_kernel(const int64_t *__restrict__ off, const int32_t *__restrict__ nbr, int64_t n, int S,
                                   const int32_t *__restrict__ seg_off, const int64_t *__restrict__ seg_start,
                                   int32_t *__restrict__ seg_nbr) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    int64_t prev = off[v], end = off[v + 1];
    for (int s = 0; s < S; ++s) {
      int64_t b = (s == S - 1) ? end : lower_bound_row(nbr, prev, end, (int32_t)((int64_t)(s + 1) << SEG_SHIFT));
      int64_t dst = seg_start[s] + seg_off[(int64_t)s * (n + 1) + v];
      for (int64_t e = prev; e < b; ++e) seg_nbr[dst + (e - prev)] = nbr[e];
      prev = b;
    }
  }
}

// In-place exclusive scan of int32 values (block totals through `partial`).
constexpr int SC_THREADS = 256, SC_ITEMS = 8, SC_TILE = SC_THREADS * SC_ITEMS;

__global__ void __launch_bounds__(SC_THREADS) scan_i32_reduce_kernel(const int32_t *__restrict__ a, int64_t count,
                                                                     long long *__restrict__ partial) {
  int64_t i0 = (int64_t)blockIdx.x * SC_TILE;
  long long c = 0;
  for (int j = 0; j < SC_ITEMS; ++j) {
    int64_t i = i0 + j * SC_THREADS + threadIdx.x;
    if (i < count) c += a[i];
  }
  long long t = block_sum<long long, SC_THREADS>(c);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

__global__ void __launch_bounds__(SC_THREADS) scan_i32_partials_kernel(long long *__restrict__ partial, int64_t nb) {
  __shared__ long long ws[SC_THREADS / BYO_WAVE];
  long long carry = 0;
  for (int64_t base = 0; base < nb; base += SC_THREADS) {
    int64_t i = base + threadIdx.x;
    long long v = i < nb ? partial[i] : 0;
    long long inc = v;
    for (int o = 1; o < BYO_WAVE; o <<= 1) {
      long long t = __shfl_up(inc, o);
      if (lane_id() >= o) inc += t;
    }
    __syncthreads();
    if (lane_id() == BYO_WAVE - 1) ws[threadIdx.x / BYO_WAVE] = inc;
    __syncthreads();
    long long before = 0, all = 0;
    for (int w = 0; w < SC_THREADS / BYO_WAVE; ++w) {
      if (w < (int)(threadIdx.x / BYO_WAVE)) before += ws[w];
      all += ws[w];
    }
    if (i < nb) partial[i] = carry + before + inc - v;
    carry += all;
  }
  if (threadIdx.x == 0) partial[nb] = carry;
}

__global__ void __launch_bounds__(SC_THREADS) scan_i32_write_kernel(int32_t *__restrict__ a, int64_t count,
                                                                    const long long *__restrict__ partial) {
  __shared__ long long ws[SC_THREADS / BYO_WAVE];
  int64_t i0 = (int64_t)blockIdx.x * SC_TILE + (int64_t)threadIdx.x * SC_ITEMS;
  int32_t v[SC_ITEMS];
  long long c = 0;
  for (int j = 0; j < SC_ITEMS; ++j) {
    v[j] = (i0 + j < count) ? a[i0 + j] : 0;
    c += v[j];
  }
  long long inc = c;
  for (int o = 1; o < BYO_WAVE; o <<= 1) {
    long long t = __shfl_up(inc, o);
    if (lane_id() >= o) inc += t;
  }
  if (lane_id() == BYO_WAVE - 1) ws[threadIdx.x / BYO_WAVE] = inc;
  __syncthreads();
  long long before = 0;
  for (int w = 0; w < (int)(threadIdx.x / BYO_WAVE); ++w) before += ws[w];
  long long pos = partial[blockIdx.x] + before + inc - c;
  for (int j = 0; j < SC_ITEMS; ++j) {
    if (i0 + j < count) a[i0 + j] = (int32_t)pos;
    pos += v[j];
  }
}

static byo_status scan_i32(int32_t *a, int64_t count, long long *partial, int64_t cap, hipStream_t s,
                           long long *h_total) {
  int64_t nb = std::max<int64_t>(1, (count + SC_TILE - 1) / SC_TILE);
  BYO_CHECK(nb + 1 <= cap, BYO_EINVAL, "scan scratch too small");
  scan_i32_reduce_kernel<<<(unsigned)nb, SC_THREADS, 0, s>>>(a, count, partial);
  scan_i32_partials_kernel<<<1, SC_THREADS, 0, s>>>(partial, nb);
  scan_i32_write_kernel<<<(unsigned)nb, SC_THREADS, 0, s>>>(a, count, partial);
  BYO_HIP(hipGetLastError());
  if (h_total) BYO_TRY(sync_read(s, partial + nb, h_total, sizeof(long long)));
  return BYO_OK;
}

byo_status pr_seg_ensure(byo_graph *g, hipStream_t s) {
  byo_workspace &w = g->ws;
  if (w.prseg) return BYO_OK;
  int64_t n = g->n;
  int S = (int)((n + (1ll << SEG_SHIFT) - 1) >> SEG_SHIFT);
  pr_seg *p = new pr_seg();
  w.prseg = p;
  p->S = S;
  p->n = n;
  BYO_HIP(hipMalloc(&p->seg_off, sizeof(int32_t) * (size_t)S * (n + 1)));
  BYO_HIP(hipMalloc(&p->seg_nbr, sizeof(int32_t) * (size_t)std::max<int64_t>(g->m, 1)));
  BYO_HIP(hipMalloc(&p->acc, sizeof(float) * (size_t)n));
  unsigned gb = (unsigned)std::min<int64_t>((n + 256) / 256 + 1, 8192);
  seg_count_kernel<<<gb, 256, 0, s>>>(g->off, g->nbr, n, S, p->seg_off);
  BYO_HIP(hipGetLastError());
  p->seg_start.assign(S + 1, 0);
  for (int k = 0; k < S; ++k) {
    long long tot = 0;
    BYO_TRY(scan_i32(p->seg_off + (int64_t)k * (n + 1), n + 1, w.partial, w.partial_cap, s, &tot));
    p->seg_start[k + 1] = p->seg_start[k] + tot;
  }
  BYO_CHECK(p->seg_start[S] == g->m, BYO_EINVAL, "segment split lost edges");
  int64_t *d_start = nullptr;
  BYO_HIP(hipMalloc(&d_start, sizeof(int64_t) * (S + 1)));
  BYO_HIP(hipMemcpyAsync(d_start, p->seg_start.data(), sizeof(int64_t) * (S + 1), hipMemcpyHostToDevice, s));
  seg_scatter_kernel<<<gb, 256, 0, s>>>(g->off, g->nbr, n, S, p->seg_off, d_start, p->seg_nbr);
  BYO_HIP(hipGetLastError());
  // long rows per segment, found on the host from the segment offsets
  std::vector<int32_t> ho((size_t)S * (n + 1));
  BYO_HIP(hipMemcpyAsync(ho.data(), p->seg_off, sizeof(int32_t) * ho.size(), hipMemcpyDeviceToHost, s));
  BYO_HIP(hipStreamSynchronize(s));
  (void)hipFree(d_start);
  std::vector<int32_t> lr;
  p->long_start.assign(S + 1, 0);
  for (int k = 0; k < S; ++k) {
    const int32_t *o = ho.data() + (size_t)k * (n + 1);
    for (int64_t v = 0; v < n; ++v)
      if (o[v + 1] - o[v] > SEG_LONG) lr.push_back((int32_t)v);
    p->long_start[k + 1] = (int64_t)lr.size();
  }
  BYO_HIP(hipMalloc(&p->long_rows, sizeof(int32_t) * std::max<size_t>(lr.size(), 1)));
  if (!lr.empty())
    BYO_HIP(hipMemcpy(p->long_rows, lr.data(), sizeof(int32_t) * lr.size(), hipMemcpyHostToDevice));
  int64_t most_long = 0;
  for (int k = 0; k < S; ++k) most_long = std::max(most_long, p->long_start[k + 1] - p->long_start[k]);
  p->dpart_cap = std::max<int64_t>(1, (w.words + 3) / 4) + most_long;
  BYO_HIP(hipMalloc(&p->dpart, sizeof(float) * (size_t)p->dpart_cap));
  return BYO_OK;
}

__global__ void __launch_bounds__(SEG_BLOCK) pr_base_kernel(const float *__restrict__ dpart, int64_t nparts,
                                                            double damping, int64_t n, float *__restrict__ base) {
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < nparts; i += SEG_BLOCK) s += (double)dpart[i];
  double t = block_sum<double, SEG_BLOCK>(s);
  if (threadIdx.x == 0) base[0] = (float)((1.0 - damping) / (double)n + damping * t / (double)n);
}

// Blocks [0, nlong): one long row each. Blocks [nlong, ...): one wavefront per
// 64 consecutive rows. dpart gets one dangling partial per block (last pass).
template <bool FIRST, bool LAST>
__global__ void __launch_bounds__(SEG_BLOCK) pr_seg_kernel(const int32_t *__restrict__ long_rows, int32_t nlong,
                                                           const int32_t *__restrict__ soff,
                                                           const int32_t *__restrict__ snbr, int64_t n,
                                                           const float *__restrict__ contrib, float *__restrict__ acc,
                                                           const int32_t *__restrict__ deg,
                                                           const float *__restrict__ base, float damping,
                                                           float *__restrict__ contrib_next, float *__restrict__ out,
                                                           float *__restrict__ dpart, int32_t t_wave) {
  float dang = 0.0f;
  auto finish = [&](int64_t v, float sum, bool has) {
    if (!LAST) {
      if (FIRST) acc[v] = sum;
      else if (has) acc[v] += sum;
    } else {
      float tot = FIRST ? sum : (acc[v] + sum);
      float r = base[0] + damping * tot;
      int32_t d = deg[v];
      if (contrib_next) contrib_next[v] = d > 0 ? r / (float)d : 0.0f;
      if (out) out[v] = r;
      if (d == 0) dang += r;
    }
  };
  if ((int32_t)blockIdx.x < nlong) {
    int64_t v = long_rows[blockIdx.x];
    int64_t e0 = soff[v], e1 = soff[v + 1];
    float sum = 0.0f;
    for (int64_t e = e0 + threadIdx.x; e < e1; e += 4 * SEG_BLOCK) {
      float c[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) c[j] = (e + j * SEG_BLOCK < e1) ? contrib[snbr[e + j * SEG_BLOCK]] : 0.0f;
#pragma unroll
      for (int j = 0; j < 4; ++j) sum += c[j];
    }
    float t = block_sum<float, SEG_BLOCK>(sum);
    if (threadIdx.x == 0) finish(v, t, true);
  } else {
    int64_t lb = xcd_block(blockIdx.x - nlong, gridDim.x - nlong);
    int64_t v = (lb * (SEG_BLOCK / BYO_WAVE) + threadIdx.x / BYO_WAVE) * 64 + lane_id();
    bool valid = v < n;
    int64_t beg = 0, end = 0;
    float sum = 0.0f;
    if (valid) {
      beg = soff[v];
      end = soff[v + 1];
      if (end - beg <= t_wave) {
        for (int64_t e = beg; e < end; e += SEG_ILP) {
          float c[SEG_ILP];
#pragma unroll
          for (int j = 0; j < SEG_ILP; ++j) c[j] = (e + j < end) ? contrib[snbr[e + j]] : 0.0f;
#pragma unroll
          for (int j = 0; j < SEG_ILP; ++j) sum += c[j];
        }
      }
    }
    int64_t len = end - beg;
    uint64_t pm = __ballot(valid && len > t_wave && len <= SEG_LONG);
    while (pm) {
      int l = __ffsll((long long)pm) - 1;
      pm &= pm - 1;
      int64_t lo = (int64_t)read_lane_u64((uint64_t)beg, l);
      int64_t hi = (int64_t)read_lane_u64((uint64_t)end, l);
      float part = 0.0f;
      for (int64_t e = lo + lane_id(); e < hi; e += 4 * BYO_WAVE) {
        float c[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) c[j] = (e + j * BYO_WAVE < hi) ? contrib[snbr[e + j * BYO_WAVE]] : 0.0f;
#pragma unroll
        for (int j = 0; j < 4; ++j) part += c[j];
      }
      part = wave_sum(part);
      if (lane_id() == l) sum = part;
    }
    if (valid && len <= SEG_LONG) finish(v, sum, len > 0);
  }
  if (LAST) {
    float t = block_sum<float, SEG_BLOCK>(dang);
    if (threadIdx.x == 0) dpart[blockIdx.x] = t;
  }
}

template <bool FIRST, bool LAST>
static void launch_seg(const pr_seg *p, int k, const float *contrib, const int32_t *deg, const float *base,
                       float damping, float *contrib_next, float *out, int32_t t_wave, hipStream_t s,
                       int64_t *nblocks) {
  int32_t nlong = (int32_t)(p->long_start[k + 1] - p->long_start[k]);
  int64_t words = (p->n + 63) / 64;
  int64_t nb = nlong + std::max<int64_t>(1, (words + 3) / 4);
  pr_seg_kernel<FIRST, LAST><<<(unsigned)nb, SEG_BLOCK, 0, s>>>(
      p->long_rows + p->long_start[k], nlong, p->seg_off + (int64_t)k * (p->n + 1), p->seg_nbr + p->seg_start[k],
      p->n, contrib, p->acc, deg, base, damping, contrib_next, out, p->dpart, t_wave);
  *nblocks = nb;
}

// One PageRank step over the segment passes. dpart holds `nparts` dangling
// partials of the previous step; afterwards it holds those of this step.
byo_status pr_seg_step(byo_graph *g, const float *contrib, float damping, float *contrib_next, float *out,
                       int64_t nparts, hipStream_t s, int64_t *nparts_out) {
  pr_seg *p = (pr_seg *)g->ws.prseg;
  pr_base_kernel<<<1, SEG_BLOCK, 0, s>>>(p->dpart, nparts, (double)damping, g->n, g->ws.base);
  ktimer_scope kt(BYO_K_PR_PULL, s);
  int S = p->S;
  int32_t tw = 32;
  int64_t nb = 0;
  for (int k = 0; k < S; ++k) {
    bool first = k == 0, last = k == S - 1;
    if (first && last)
      launch_seg<true, true>(p, k, contrib, g->deg, g->ws.base, damping, contrib_next, out, tw, s, &nb);
    else if (first)
      launch_seg<true, false>(p, k, contrib, g->deg, g->ws.base, damping, contrib_next, out, tw, s, &nb);
    else if (last)
      launch_seg<false, true>(p, k, contrib, g->deg, g->ws.base, damping, contrib_next, out, tw, s, &nb);
    else
      launch_seg<false, false>(p, k, contrib, g->deg, g->ws.base, damping, contrib_next, out, tw, s, &nb);
  }
  BYO_HIP(hipGetLastError());
  *nparts_out = nb;
  return BYO_OK;
}

float *pr_seg_dpart(byo_graph *g) { return ((pr_seg *)g->ws.prseg)->dpart; }

}  // namespace byo
