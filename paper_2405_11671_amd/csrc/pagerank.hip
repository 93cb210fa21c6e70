// PageRank (paper Table algs-list, "Eigenvector" category) as repeated dense
// pull edgeMaps with the apply step fused in. FP32 storage and arithmetic.
//
// One step: p'[v] = (1-d)/n + d * (sum over u in N(v) of p[u]/deg(u) + D/n),
// D = sum of p over degree-0 vertices. The kernel keeps contrib[u] =
// p[u]/deg(u) (0 for degree 0) instead of p, so the gather reads one float per
// edge, and writes p only after the last step.
//
// Summation order is fixed (no float atomics), so results are deterministic:
//  - rows with degree <= t_wave: one lane, ascending (FP64 accumulation above
//    PR_LANE_F32 terms);
//  - t_wave < degree <= HEAVY: the wavefront, lane-strided partial sums and a
//    butterfly reduction;
//  - degree > HEAVY: HEAVY-edge chunks reduced by one workgroup each in a
//    separate kernel, then the owning lane adds the chunk sums in order.
#include <algorithm>
#include <cstring>
#include <vector>

#include "cz_dev.h"
#include "internal.h"

namespace byo {

constexpr int PR_BLOCK = 256;
constexpr int64_t PR_HEAVY = 4096;   // chunk length and heavy-row threshold
constexpr int PR_ILP = 8;
constexpr int64_t PR_LANE_F32 = 256;  // longest row one lane sums in FP32

static int64_t pr_blocks(int64_t words) { return std::max<int64_t>(1, (words + 3) / 4); }

__global__ void pr_heavy_mark_kernel(const int32_t *__restrict__ deg, int64_t n, int32_t *__restrict__ list,
                                     unsigned long long *__restrict__ count) {
  int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool heavy = v < n && deg[v] > PR_HEAVY;
  wave_append(heavy, (int32_t)v, list, count);
}

__global__ void pr_row_chunk_kernel(int32_t *row_chunk0, int64_t n) {
  int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n) row_chunk0[v] = -1;
}

__global__ void pr_gather_extents_kernel(const int64_t *__restrict__ off, const int32_t *__restrict__ rows,
                                         int64_t k, int64_t *__restrict__ ext) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < k) {
    ext[2 * i] = off[rows[i]];
    ext[2 * i + 1] = off[rows[i] + 1];
  }
}

__global__ void pr_scatter_first_kernel(const int32_t *__restrict__ rows, const int32_t *__restrict__ first,
                                        int64_t k, int32_t *__restrict__ row_chunk0) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < k) row_chunk0[rows[i]] = first[i];
}

__global__ void fill_f32_kernel(float *p, int64_t n, float value) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = value;
}

// Initial contributions from p = 1/n, and dangling partial sums per block.
__global__ void __launch_bounds__(PR_BLOCK) pr_init_kernel(const int32_t *__restrict__ deg, int64_t n, int64_t words,
                                                           float *__restrict__ contrib, float *__restrict__ dpart) {
  int64_t lb = xcd_block(blockIdx.x, gridDim.x);
  int64_t v = lb * PR_BLOCK + threadIdx.x;
  float p0 = 1.0f / (float)n;
  float dang = 0.0f;
  if (v < n) {
    int32_t d = deg[v];
    contrib[v] = d > 0 ? p0 / (float)d : 0.0f;
    if (d == 0) dang = p0;
  }
  float t = block_sum<float, PR_BLOCK>(dang);
  if (threadIdx.x == 0) dpart[lb] = t;
}

// Heavy-row chunk sums; block 0 also folds the dangling partials into the
// step constant base = (1-d)/n + d*D/n (accumulated in double, fixed order).
__global__ void __launch_bounds__(PR_BLOCK) pr_chunk_kernel(const int32_t *__restrict__ nbr,
                                                            const float *__restrict__ contrib,
                                                            const int64_t *__restrict__ chunk_beg,
                                                            const int64_t *__restrict__ chunk_end, int64_t nchunks,
                                                            float *__restrict__ chunk_sum,
                                                            const float *__restrict__ dpart, int64_t nparts, double damping,
                                                            int64_t n, float *__restrict__ base, int do_base) {
  if (blockIdx.x < nchunks) {
    int64_t beg = chunk_beg[blockIdx.x], end = chunk_end[blockIdx.x];
    float s = 0.0f;
    for (int64_t e = beg + threadIdx.x; e < end; e += PR_BLOCK) s += contrib[nbr[e]];
    float t = block_sum<float, PR_BLOCK>(s);
    if (threadIdx.x == 0) chunk_sum[blockIdx.x] = t;
  }
  if (do_base && blockIdx.x == 0) {
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < nparts; i += PR_BLOCK) s += (double)dpart[i];
    double t = block_sum<double, PR_BLOCK>(s);
    if (threadIdx.x == 0) base[0] = (float)((1.0 - damping) / (double)n + damping * t / (double)n);
  }
}

// MODE 0: one PageRank step. MODE 1: plain accumulation acc[v] = sum contrib[u].
// deg, when given, divides in place of the row length (a mapped degree).
template <int MODE>
__global__ void __launch_bounds__(PR_BLOCK) pr_pull_kernel(const int64_t *__restrict__ off, const int32_t *__restrict__ nbr,
                                                           const int32_t *__restrict__ deg, int64_t n, int64_t words,
                                                           const float *__restrict__ contrib,
                                                           const int32_t *__restrict__ row_chunk0,
                                                           const float *__restrict__ chunk_sum,
                                                           const float *__restrict__ base, float damping,
                                                           float *__restrict__ contrib_next, float *__restrict__ dpart,
                                                           float *__restrict__ out, int32_t t_wave) {
  int64_t lb = xcd_block(blockIdx.x, gridDim.x);
  int64_t w = lb * (PR_BLOCK / BYO_WAVE) + threadIdx.x / BYO_WAVE;
  int64_t v64 = w * 64 + lane_id();
  bool valid = v64 < n;
  int32_t v = (int32_t)v64;
  int64_t beg = 0, end = 0;
  int32_t d = 0;
  float s = 0.0f;
  if (valid) {
    beg = off[v];
    end = off[v + 1];
    d = (int32_t)(end - beg);
    if (d <= t_wave && d <= PR_LANE_F32) {
      // ascending order, PR_ILP independent gathers per step
      for (int64_t e = beg; e < end; e += PR_ILP) {
        float c[PR_ILP];
#pragma unroll
        for (int j = 0; j < PR_ILP; ++j) c[j] = (e + j < end) ? contrib[nbr[e + j]] : 0.0f;
#pragma unroll
        for (int j = 0; j < PR_ILP; ++j) s += c[j];
      }
    } else if (d <= t_wave) {
      // a long row summed by one lane (t_wave raised, or no parallel map):
      // an FP32 running sum of 10^4..10^5 terms drifts by up to d ulps, so
      // this one accumulates in FP64
      double sd = 0.0;
      for (int64_t e = beg; e < end; e += PR_ILP) {
        float c[PR_ILP];
#pragma unroll
        for (int j = 0; j < PR_ILP; ++j) c[j] = (e + j < end) ? contrib[nbr[e + j]] : 0.0f;
#pragma unroll
        for (int j = 0; j < PR_ILP; ++j) sd += (double)c[j];
      }
      s = (float)sd;
    } else if (d > PR_HEAVY) {
      int32_t c0 = row_chunk0[v];
      int32_t nc = (int32_t)((d + PR_HEAVY - 1) / PR_HEAVY);
      for (int32_t c = 0; c < nc; ++c) s += chunk_sum[c0 + c];
    }
  }
  uint64_t pm = __ballot(valid && d > t_wave && d <= PR_HEAVY);
  while (pm) {
    int l = __ffsll((long long)pm) - 1;
    pm &= pm - 1;
    int64_t lb2 = (int64_t)read_lane_u64((uint64_t)beg, l);
    int64_t le = (int64_t)read_lane_u64((uint64_t)end, l);
    float part = 0.0f;
    for (int64_t e = lb2 + lane_id(); e < le; e += 4 * BYO_WAVE) {
      float c[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) c[j] = (e + j * BYO_WAVE < le) ? contrib[nbr[e + j * BYO_WAVE]] : 0.0f;
#pragma unroll
      for (int j = 0; j < 4; ++j) part += c[j];
    }
    part = wave_sum(part);
    if (lane_id() == l) s = part;
  }
  if (MODE == 1) {
    if (valid) out[v] = s;
    return;
  }
  float r = base[0] + damping * s;
  float dang = 0.0f;
  if (valid) {
    if (deg) d = deg[v];  // a degree the container reports by mapping
    if (contrib_next) contrib_next[v] = d > 0 ? r / (float)d : 0.0f;
    if (d == 0) dang = r;
    if (out) out[v] = r;
  }
  float t = block_sum<float, PR_BLOCK>(dang);
  if (threadIdx.x == 0) dpart[lb] = t;
}

// One PageRank step over the byte-coded lists: a lane sums its row's first
// block in order; the further blocks of long rows are summed by the
// wavefront, one block per lane, then reduced. The rest is pr_pull_kernel's
// step (same base, contributions, dangling partials).
__global__ void __launch_bounds__(PR_BLOCK) pr_cz_pull_kernel(const int64_t *__restrict__ coff,
                                                              const uint8_t *__restrict__ bytes,
                                                              const int32_t *__restrict__ deg, int64_t n,
                                                              const float *__restrict__ contrib,
                                                              const float *__restrict__ base, float damping,
                                                              float *__restrict__ contrib_next,
                                                              float *__restrict__ dpart, float *__restrict__ out) {
  int64_t lb = xcd_block(blockIdx.x, gridDim.x);
  int64_t w = lb * (PR_BLOCK / BYO_WAVE) + threadIdx.x / BYO_WAVE;
  int64_t v64 = w * 64 + lane_id();
  bool valid = v64 < n;
  int32_t v = (int32_t)v64;
  int32_t d = 0;
  int64_t r = 0;
  if (valid) {
    d = deg[v];
    r = coff[v];
  }
  const int32_t nb = cz_nblocks(d);
  // the batch's gathers are issued together, then added in order
  auto add = [&](const int32_t *u, float &acc) {
    float c[CZ_BATCH];
#pragma unroll
    for (int t = 0; t < CZ_BATCH; ++t) c[t] = u[t] >= 0 ? contrib[u[t]] : 0.0f;
#pragma unroll
    for (int t = 0; t < CZ_BATCH; ++t) acc += c[t];
    return false;
  };
  float s = 0.0f;
  if (nb > 0) cz_block_batches<false>(bytes, r, v, d, nb, 0, [&](const int32_t *u) { return add(u, s); });
  // blocks after the first: one per lane, lane-serial, then reduced
  uint64_t pm = __ballot(nb > 1);
  while (pm) {
    const int l = __ffsll((long long)pm) - 1;
    pm &= pm - 1;
    const int32_t vl = read_lane_i32(v, l), dl = read_lane_i32(d, l);
    const int64_t rl = (int64_t)read_lane_u64((uint64_t)r, l);
    const int32_t nbl = cz_nblocks(dl);
    float part = 0.0f;
    for (int32_t j = 1 + lane_id(); j < nbl; j += BYO_WAVE)
      cz_block_batches<false>(bytes, rl, vl, dl, nbl, j, [&](const int32_t *u) { return add(u, part); });
    part = wave_sum(part);
    if (lane_id() == l) s += part;
  }
  float rv = base[0] + damping * s;
  float dang = 0.0f;
  if (valid) {
    if (contrib_next) contrib_next[v] = d > 0 ? rv / (float)d : 0.0f;
    if (d == 0) dang = rv;
    if (out) out[v] = rv;
  }
  float t = block_sum<float, PR_BLOCK>(dang);
  if (threadIdx.x == 0) dpart[lb] = t;
}

byo_status ws_ensure_pagerank(byo_graph *g, hipStream_t s) {
  BYO_TRY(ws_ensure_traversal(g));
  byo_workspace &w = g->ws;
  if (w.contrib[0]) return BYO_OK;
  int64_t n = g->n;
  size_t fb = sizeof(float) * (size_t)std::max<int64_t>(n, 1);
  int64_t nb = pr_blocks(w.words);
  BYO_HIP(hipMalloc(&w.contrib[0], fb));
  BYO_HIP(hipMalloc(&w.contrib[1], fb));
  BYO_HIP(hipMalloc(&w.dpart, sizeof(float) * (size_t)nb));
  BYO_HIP(hipMalloc(&w.base, sizeof(float) * 4));
  BYO_HIP(hipMalloc(&w.row_chunk0, sizeof(int32_t) * (size_t)std::max<int64_t>(n, 1)));
  w.pr_dpart_blocks = (int32_t)nb;
  // heavy rows -> chunk table (built once per graph)
  int64_t nheavy = 0;
  if (n > 0 && g->max_deg > PR_HEAVY) {
    unsigned long long *cnt = (unsigned long long *)w.misc;
    BYO_HIP(hipMemsetAsync(cnt, 0, sizeof(unsigned long long), s));
    pr_heavy_mark_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(g->deg, n, w.ids[0], cnt);
    BYO_HIP(hipGetLastError());
    unsigned long long hc = 0;
    BYO_TRY(sync_read(s, cnt, &hc, sizeof(hc)));
    nheavy = (int64_t)hc;
  }
  std::vector<int32_t> rows((size_t)nheavy);
  if (nheavy > 0) {
    BYO_HIP(hipMemcpyAsync(rows.data(), w.ids[0], sizeof(int32_t) * (size_t)nheavy, hipMemcpyDeviceToHost, s));
    BYO_HIP(hipStreamSynchronize(s));
    std::sort(rows.begin(), rows.end());
  }
  pr_row_chunk_kernel<<<(unsigned)std::max<int64_t>(1, (n + 255) / 256), 256, 0, s>>>(w.row_chunk0, n);
  BYO_HIP(hipGetLastError());
  std::vector<int64_t> beg, end;
  std::vector<int32_t> first((size_t)nheavy);
  if (nheavy > 0) {
    // row extents of the heavy rows, gathered on the device in one pass
    int32_t *d_rows = nullptr;
    int64_t *d_ext = nullptr;
    BYO_HIP(hipMalloc(&d_rows, sizeof(int32_t) * (size_t)nheavy));
    BYO_HIP(hipMalloc(&d_ext, 2 * sizeof(int64_t) * (size_t)nheavy));
    BYO_HIP(hipMemcpyAsync(d_rows, rows.data(), sizeof(int32_t) * (size_t)nheavy, hipMemcpyHostToDevice, s));
    pr_gather_extents_kernel<<<(unsigned)((nheavy + 255) / 256), 256, 0, s>>>(g->off, d_rows, nheavy, d_ext);
    std::vector<int64_t> ext(2 * (size_t)nheavy);
    BYO_HIP(hipMemcpyAsync(ext.data(), d_ext, 2 * sizeof(int64_t) * (size_t)nheavy, hipMemcpyDeviceToHost, s));
    BYO_HIP(hipStreamSynchronize(s));
    for (int64_t i = 0; i < nheavy; ++i) {
      first[i] = (int32_t)beg.size();
      for (int64_t e = ext[2 * i]; e < ext[2 * i + 1]; e += PR_HEAVY) {
        beg.push_back(e);
        end.push_back(std::min(e + PR_HEAVY, ext[2 * i + 1]));
      }
    }
    int32_t *d_first = nullptr;
    BYO_HIP(hipMalloc(&d_first, sizeof(int32_t) * (size_t)nheavy));
    BYO_HIP(hipMemcpyAsync(d_first, first.data(), sizeof(int32_t) * (size_t)nheavy, hipMemcpyHostToDevice, s));
    pr_scatter_first_kernel<<<(unsigned)((nheavy + 255) / 256), 256, 0, s>>>(d_rows, d_first, nheavy, w.row_chunk0);
    BYO_HIP(hipGetLastError());
    BYO_HIP(hipStreamSynchronize(s));
    (void)hipFree(d_rows);
    (void)hipFree(d_ext);
    (void)hipFree(d_first);
  }
  w.nchunks = (int64_t)beg.size();
  int64_t nc = std::max<int64_t>(w.nchunks, 1);
  BYO_HIP(hipMalloc(&w.chunk_beg, sizeof(int64_t) * (size_t)nc));
  BYO_HIP(hipMalloc(&w.chunk_row, sizeof(int64_t) * (size_t)nc));  // holds chunk ends
  BYO_HIP(hipMalloc(&w.chunk_sum, sizeof(float) * (size_t)nc));
  if (w.nchunks > 0) {
    BYO_HIP(hipMemcpy(w.chunk_beg, beg.data(), sizeof(int64_t) * beg.size(), hipMemcpyHostToDevice));
    BYO_HIP(hipMemcpy(w.chunk_row, end.data(), sizeof(int64_t) * end.size(), hipMemcpyHostToDevice));
  }
  return BYO_OK;
}

byo_status pr_accumulate(byo_graph *g, const float *contrib, float *acc, hipStream_t s) {
  BYO_TRY(ws_ensure_pagerank(g, s));
  byo_workspace &w = g->ws;
  if (g->n == 0) return BYO_OK;
  if (w.nchunks > 0) {
    pr_chunk_kernel<<<(unsigned)w.nchunks, PR_BLOCK, 0, s>>>(g->nbr, contrib, w.chunk_beg, w.chunk_row, w.nchunks,
                                                             w.chunk_sum, w.dpart, 0, 0.0, g->n, w.base, 0);
  }
  pr_pull_kernel<1><<<(unsigned)pr_blocks(w.words), PR_BLOCK, 0, s>>>(
      g->off, g->nbr, nullptr, g->n, w.words, contrib, w.row_chunk0, w.chunk_sum, w.base, 1.0f, nullptr, w.dpart,
      acc, 32);
  BYO_HIP(hipGetLastError());
  return BYO_OK;
}

}  // namespace byo

using namespace byo;

extern "C" byo_status byo_pagerank(byo_graph *g, double damping, int32_t iters, float *d_rank, const byo_opts *opts,
                                   void *stream, byo_run_stats *stats) {
  BYO_CHECK(g && d_rank, BYO_EINVAL, "null argument");
  BYO_CHECK(iters >= 0, BYO_EINVAL, "iters < 0");
  BYO_CHECK(damping >= 0.0 && damping <= 1.0, BYO_EINVAL, "damping outside [0, 1]");
  byo_opts o;
  byo_opts_default(&o);
  if (opts) o = *opts;
  hipStream_t s = (hipStream_t)stream;
  int64_t n = g->n;
  if (stats) {
    std::memset(stats, 0, sizeof(*stats));
    stats->levels = iters;
    stats->variant_count[BYO_V_PULL_WAVE] = iters;
  }
  if (n == 0) return BYO_OK;
  BYO_TRY(ws_ensure_pagerank(g, s));
  byo_workspace &w = g->ws;
  int64_t nb = pr_blocks(w.words);
  int32_t tw = o.t_wave > 0 ? o.t_wave : 32;
  // Container-API ablation (Table api-components-avg): without degree() every
  // step maps each vertex's list to count it; without a parallel map every
  // list is summed by one lane.
  const uint32_t omit = (uint32_t)o.api_omit;
  BYO_CHECK(!o.compressed || omit == 0, BYO_EINVAL, "byte-coded lists run with the full container API");
  const bool par_map = !(omit & BYO_API_NO_PAR_MAP);
  int32_t *mdeg = nullptr;
  if (omit & BYO_API_NO_DEGREE) BYO_TRY(api_map_degrees(g, omit, s, &mdeg));
  if (!par_map) tw = INT32_MAX;
  const bool tiled = o.pr_blocked != 0 && omit == 0 && !o.compressed && tiles_wanted(g);
  if (!tiled) {  // the tiled path starts from the layout's own degrees below
    pr_init_kernel<<<(unsigned)nb, PR_BLOCK, 0, s>>>(mdeg ? mdeg : g->deg, n, w.words, w.contrib[0], w.dpart);
    BYO_HIP(hipGetLastError());
  }
  if (iters == 0) {
    // a zero-step run returns the initial vector p = 1/n
    fill_f32_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(d_rank, n, 1.0f / (float)n);
    BYO_HIP(hipGetLastError());
    return BYO_OK;
  }
  if (o.compressed) {
    const byo_cz *cz = nullptr;
    BYO_TRY(cz_ensure(g, s, &cz));
    int c = 0;
    for (int32_t t = 0; t < iters; ++t) {
      bool last = t + 1 == iters;
      {
        ktimer_scope kc(BYO_K_PR_CHUNK, s);  // the step constant only
        pr_chunk_kernel<<<1, PR_BLOCK, 0, s>>>(g->nbr, w.contrib[c], w.chunk_beg, w.chunk_row, 0, w.chunk_sum,
                                                w.dpart, nb, damping, n, w.base, 1);
      }
      ktimer_scope kp(BYO_K_PR_PULL, s);
      pr_cz_pull_kernel<<<(unsigned)nb, PR_BLOCK, 0, s>>>(cz->coff, cz->bytes, g->deg, n, w.contrib[c], w.base,
                                                          (float)damping, last ? nullptr : w.contrib[1 - c], w.dpart,
                                                          last ? d_rank : nullptr);
      BYO_HIP(hipGetLastError());
      c = 1 - c;
    }
    return BYO_OK;
  }
  if (tiled) {
    byo_tiles *tl = nullptr;
    BYO_TRY(tiles_ensure(g, pr_tile_shift(g, o.pr_blocked), s, &tl));
    // the tiled step runs in the layout's relabelled vertex order
    pr_init_kernel<<<(unsigned)nb, PR_BLOCK, 0, s>>>(tl->rdeg, n, w.words, w.contrib[0], w.dpart);
    BYO_HIP(hipGetLastError());
    // The degree-0 vertices receive nothing, so each holds the step constant
    // after every step (1/n before the first): the dangling mass D is their
    // count times it, and the constants follow on the host, in double.
    const double nd = (double)n, n0 = (double)g->isolated;
    double p_iso = 1.0 / nd;
    int c = 0;
    for (int32_t t = 0; t < iters; ++t) {
      bool last = t + 1 == iters;
      const double bs = (1.0 - damping) / nd + damping * (n0 * p_iso) / nd;
      BYO_TRY(pr_tile_step(g, tl, w.contrib[c], (float)bs, (float)damping, last ? nullptr : w.contrib[1 - c],
                           last ? d_rank : nullptr, s));
      p_iso = bs;
      c = 1 - c;
    }
    return BYO_OK;
  }
  int cur = 0;
  for (int32_t t = 0; t < iters; ++t) {
    bool last = t + 1 == iters;
    // the degree of every vertex, mapped again at each step
    if (mdeg && t > 0) BYO_TRY(api_map_degrees(g, omit, s, &mdeg));
    {
      // without a parallel map only the step constant is computed here
      const int64_t nch = par_map ? w.nchunks : 0;
      ktimer_scope kc(BYO_K_PR_CHUNK, s);
      pr_chunk_kernel<<<(unsigned)std::max<int64_t>(nch, 1), PR_BLOCK, 0, s>>>(
        g->nbr, w.contrib[cur], w.chunk_beg, w.chunk_row, nch, w.chunk_sum, w.dpart, nb, damping, n, w.base, 1);
    }
    ktimer_scope kp(BYO_K_PR_PULL, s);
    pr_pull_kernel<0><<<(unsigned)nb, PR_BLOCK, 0, s>>>(g->off, g->nbr, mdeg, n, w.words, w.contrib[cur],
                                                        w.row_chunk0, w.chunk_sum, w.base, (float)damping,
                                                        last ? nullptr : w.contrib[1 - cur], w.dpart,
                                                        last ? d_rank : nullptr, tw);
    BYO_HIP(hipGetLastError());
    cur = 1 - cur;
  }
  return BYO_OK;
}
