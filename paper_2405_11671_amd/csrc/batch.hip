// Batched execution over many graphs: the graphs are laid out back to back as
// one CSR (a disjoint union, vertex IDs shifted by each graph's offset), so a
// BFS from one source per graph, or one connectivity run, traverses every
// graph in the same launches (for BFS, by default, in one persistent launch
// that runs every level: persistent.hip). Per-graph results are exactly those of separate
// runs because no edge crosses between graphs; uneven sizes are balanced by
// the edgeMap schedules themselves (edge-balanced push, word-per-wave pull).
#include <algorithm>
#include <cstring>
#include <vector>

#include "internal.h"

struct byo_batch {
  int32_t count = 0;
  std::vector<int64_t> voff;    // vertex offsets, count + 1
  int64_t *d_voff = nullptr;
  byo_graph *g = nullptr;
};

namespace byo {

// Rewrite global IDs (parents or labels) to local IDs of the owning graph.
__global__ void localize_kernel(int32_t *__restrict__ ids, int64_t n, const int64_t *__restrict__ voff, int32_t count) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    int32_t x = ids[v];
    if (x < 0) continue;
    int lo = 0, hi = count - 1;  // last graph whose offset <= v
    while (lo < hi) {
      int mid = (lo + hi + 1) >> 1;
      if (voff[mid] <= v) lo = mid; else hi = mid - 1;
    }
    ids[v] = (int32_t)(x - voff[lo]);
  }
}

static byo_status localize(byo_batch *b, int32_t *ids, hipStream_t s) {
  int64_t n = b->voff.back();
  if (n == 0) return BYO_OK;
  localize_kernel<<<(unsigned)std::min<int64_t>((n + 255) / 256, 4096), 256, 0, s>>>(ids, n, b->d_voff, b->count);
  BYO_HIP(hipGetLastError());
  return BYO_OK;
}

}  // namespace byo

using namespace byo;

extern "C" {

byo_status byo_batch_create(int32_t count, const int64_t *const *h_offs, const int32_t *const *h_nbrs,
                            const int64_t *ns, void *stream, byo_batch **out) {
  BYO_CHECK(out && h_offs && h_nbrs && ns, BYO_EINVAL, "null argument");
  BYO_CHECK(count >= 1, BYO_EINVAL, "empty batch");
  std::vector<int64_t> voff((size_t)count + 1, 0), eoff((size_t)count + 1, 0);
  for (int32_t i = 0; i < count; ++i) {
    BYO_CHECK(ns[i] >= 1 && h_offs[i], BYO_EINVAL, "every graph needs n >= 1 and offsets");
    BYO_CHECK(h_offs[i][0] == 0, BYO_EINVAL, "offsets must start at 0");
    voff[i + 1] = voff[i] + ns[i];
    eoff[i + 1] = eoff[i] + h_offs[i][ns[i]];
  }
  BYO_CHECK(voff[count] < 2147483647LL, BYO_EINVAL, "total vertex count must fit int32");
  int64_t N = voff[count], M = eoff[count];
  std::vector<int64_t> off((size_t)N + 1);
  std::vector<int32_t> nbr((size_t)std::max<int64_t>(M, 1));
  for (int32_t i = 0; i < count; ++i) {
    const int64_t *o = h_offs[i];
    const int32_t *nb = h_nbrs[i];
    for (int64_t v = 0; v < ns[i]; ++v) off[voff[i] + v] = eoff[i] + o[v];
    for (int64_t e = 0; e < o[ns[i]]; ++e) {
      BYO_CHECK(nb && nb[e] >= 0 && nb[e] < ns[i], BYO_EINVAL,
                "graph " + std::to_string(i) + " has a neighbour outside [0, n)");
      nbr[eoff[i] + e] = (int32_t)(nb[e] + voff[i]);
    }
  }
  off[N] = M;
  byo_batch *b = new byo_batch();
  b->count = count;
  b->voff = voff;
  byo_status st = byo_graph_from_csr(off.data(), nbr.data(), N, M, BYO_HOST_INPUT, stream, &b->g);
  if (st != BYO_OK) {
    delete b;
    return st;
  }
  hipError_t e = hipMalloc(&b->d_voff, sizeof(int64_t) * voff.size());
  if (e == hipSuccess)
    e = hipMemcpy(b->d_voff, voff.data(), sizeof(int64_t) * voff.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    byo_graph_destroy(b->g);
    delete b;
    return hip_fail(e, "batch offsets", __FILE__, __LINE__);
  }
  *out = b;
  return BYO_OK;
}

void byo_batch_destroy(byo_batch *b) {
  if (!b) return;
  byo_graph_destroy(b->g);
  if (b->d_voff) (void)hipFree(b->d_voff);
  delete b;
}

byo_status byo_batch_info(const byo_batch *b, int64_t *total_n, int64_t *total_m) {
  BYO_CHECK(b, BYO_EINVAL, "null batch");
  if (total_n) *total_n = b->g->n;
  if (total_m) *total_m = b->g->m;
  return BYO_OK;
}

byo_status byo_batch_vertex_offset(const byo_batch *b, int32_t i, int64_t *out) {
  BYO_CHECK(b && out, BYO_EINVAL, "null argument");
  BYO_CHECK(i >= 0 && i <= b->count, BYO_EINVAL, "graph index out of range");
  *out = b->voff[i];
  return BYO_OK;
}

byo_status byo_batch_bfs(byo_batch *b, const int64_t *h_srcs, int32_t *d_depth, int32_t *d_parent,
                         const byo_opts *opts, void *stream, byo_run_stats *stats) {
  BYO_CHECK(b && h_srcs && d_depth && d_parent, BYO_EINVAL, "null argument");
  byo_opts o;
  byo_opts_default(&o);
  if (opts) o = *opts;
  std::vector<int32_t> srcs((size_t)b->count);
  for (int32_t i = 0; i < b->count; ++i) {
    BYO_CHECK(h_srcs[i] >= 0 && h_srcs[i] < b->voff[i + 1] - b->voff[i], BYO_EINVAL,
              "source of graph " + std::to_string(i) + " out of range");
    srcs[i] = (int32_t)(h_srcs[i] + b->voff[i]);
  }
  hipStream_t s = (hipStream_t)stream;
  const bool plain = o.api_omit == 0 && !o.compressed;
  if (o.use_graph && plain)
    BYO_TRY(bfs_graph_run(b->g, srcs, d_depth, d_parent, o, s, stats));
  else if (o.persistent && plain && bfs_persistent_usable(b->g))
    BYO_TRY(bfs_persistent_run(b->g, srcs.data(), (int64_t)srcs.size(), d_depth, d_parent, o, s, stats));
  else
    BYO_TRY(bfs_run(b->g, srcs.data(), (int64_t)srcs.size(), d_depth, d_parent, o, s, stats));
  return localize(b, d_parent, s);
}

byo_status byo_batch_cc(byo_batch *b, int32_t *d_label, const byo_opts *opts, void *stream, byo_run_stats *stats) {
  BYO_CHECK(b && d_label, BYO_EINVAL, "null argument");
  BYO_TRY(byo_cc(b->g, d_label, opts, stream, stats));
  return localize(b, d_label, (hipStream_t)stream);
}

}  // extern "C"
