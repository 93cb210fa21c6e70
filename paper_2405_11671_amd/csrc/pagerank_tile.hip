// PageRank step over the degree-ordered destination-tile layout (tiles.hip;
// option pr_blocked = 1, or 12..14 for tiles of 2^value vertices). Same step
// as the pull kernel,
//   p'[v] = (1-d)/n + d * (sum over u in N(v) of contrib[u] + D/n),
// run in the layout's vertex order (contributions and degrees relabelled),
// with p written in the caller's order.
//
// Sums: LDS atomics on 64-bit fixed point within a chunk, chunk partials
// written densely and added by the apply kernel, which also forms p', the
// next contributions and the dangling partial sums. Integer sums are exact,
// so the result is the same whatever order the atomics land in.
#include <algorithm>

#include "internal.h"

namespace byo {

constexpr int PT_THREADS = 1024;
constexpr int PT_ILP = 16;
constexpr int PT_APPLY = 256;

int pr_tile_shift(int32_t opt) { return (opt >= 12 && opt <= 14) ? opt : BYO_TILE_SHIFT; }

// Contributions are summed as unsigned 64-bit fixed point with 61 fraction
// bits. Every contribution is p[u]/deg(u) <= 1 and a row's total is
// at most the sum of p (1 up to rounding), so sums stay below 2^63 with room
// to spare; integer addition is exact, so the sums do not depend on the order
// of the LDS atomics and every run gives the same bits. A contribution loses
// at most 2^-61 in the conversion (below 2^-38 only; larger ones are exact).
__device__ __forceinline__ unsigned long long to_fixed(float x) {
  return (unsigned long long)(x * 0x1p61f);
}

// One workgroup per chunk: LDS sums for the chunk's tile, then a dense write
// of them to the chunk's partial row. Workgroup 0 also folds the dangling
// partials of the previous apply (or of the initialisation) into
// base = (1-d)/n + d*D/n, in double and in a fixed order.
template <int SHIFT>
__global__ void __launch_bounds__(PT_THREADS) pr_tile_kernel(const uint32_t *__restrict__ ent,
                                                             const int32_t *__restrict__ anchor,
                                                             const int64_t *__restrict__ cbeg,
                                                             const float *__restrict__ contrib,
                                                             unsigned long long *__restrict__ partial,
                                                             const float *__restrict__ dpart, int64_t nparts,
                                                             double damping, int64_t n, float *__restrict__ base) {
  constexpr int B = 1 << SHIFT;
  __shared__ unsigned long long acc[B + 1];  // slot B takes the padding entries
  const int t = threadIdx.x;
  const int64_t c = blockIdx.x;
  for (int i = t; i <= B; i += PT_THREADS) acc[i] = 0ull;
  if (c == 0) {
    double s = 0.0;
    for (int64_t i = t; i < nparts; i += PT_THREADS) s += (double)dpart[i];
    double tot = block_sum<double, PT_THREADS>(s);
    if (t == 0) base[0] = (float)((1.0 - damping) / (double)n + damping * tot / (double)n);
  }
  __syncthreads();
  const int64_t beg = cbeg[c], end = cbeg[c + 1];
  // Lane-consecutive entries per load, so a wavefront's gathers cover a
  // narrow source range; PT_ILP independent loads in flight per thread.
  // Indices past the chunk end are clamped to its first entry (a chunk is
  // never empty) and their sums skipped, so the loads stay unconditional and
  // issue back to back.
  for (int64_t e0 = beg + t; e0 < end; e0 += (int64_t)PT_THREADS * PT_ILP) {
    int32_t u[PT_ILP];
    uint32_t d[PT_ILP];
    float x[PT_ILP];
#pragma unroll
    for (int j = 0; j < PT_ILP; ++j) {
      int64_t i = e0 + (int64_t)j * PT_THREADS;
      i = i < end ? i : beg;
      tile_entry(ent, anchor, i, u[j], d[j]);
    }
#pragma unroll
    for (int j = 0; j < PT_ILP; ++j) x[j] = contrib[u[j]];
#pragma unroll
    for (int j = 0; j < PT_ILP; ++j)
      if (e0 + (int64_t)j * PT_THREADS < end) atomicAdd(&acc[d[j]], to_fixed(x[j]));
  }
  __syncthreads();
  unsigned long long *out = partial + (c << SHIFT);
  for (int i = t; i < B; i += PT_THREADS) out[i] = acc[i];
}

// p'[w] = base + d * (sum of the chunk partials of w's tile), w relabelled;
// next contributions and dangling partials per workgroup in relabelled
// order, the optional output in the caller's order.
template <int SHIFT>
__global__ void __launch_bounds__(PT_APPLY) pr_tile_apply_kernel(const unsigned long long *__restrict__ partial,
                                                                 const int32_t *__restrict__ bfirst,
                                                                 const int32_t *__restrict__ rdeg,
                                                                 const int32_t *__restrict__ orig, int64_t n,
                                                                 const float *__restrict__ base, float damping,
                                                                 float *__restrict__ contrib_next,
                                                                 float *__restrict__ dpart, float *__restrict__ out) {
  const int64_t w = (int64_t)blockIdx.x * PT_APPLY + threadIdx.x;
  float dang = 0.0f;
  if (w < n) {
    const int64_t b = w >> SHIFT, l = w & ((1 << SHIFT) - 1);
    const int32_t c0 = bfirst[b], c1 = bfirst[b + 1];
    const unsigned long long *pp = partial + l;
    unsigned long long q = 0ull;
    int32_t c = c0;
    // the tiles of the highest-degree vertices have many chunks: 8 loads in flight
    for (; c + 8 <= c1; c += 8) {
      unsigned long long x[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) x[j] = pp[(int64_t)(c + j) << SHIFT];
#pragma unroll
      for (int j = 0; j < 8; ++j) q += x[j];
    }
    for (; c < c1; ++c) q += pp[(int64_t)c << SHIFT];
    float sum = (float)((double)q * 0x1p-61);
    float r = base[0] + damping * sum;
    int32_t d = rdeg[w];
    if (contrib_next) contrib_next[w] = d > 0 ? r / (float)d : 0.0f;
    if (d == 0) dang = r;
    if (out) out[orig[w]] = r;
  }
  float t = block_sum<float, PT_APPLY>(dang);
  if (threadIdx.x == 0) dpart[blockIdx.x] = t;
}



int64_t pr_tile_parts(const byo_graph *g) { return (g->n + PT_APPLY - 1) / PT_APPLY; }

template <int SHIFT>
static void launch_step(const byo_tiles *p, const byo_graph *g, const float *contrib, float damping, float *contrib_next,
                        float *out, float *dpart, float *base, int64_t nparts, hipStream_t s) {
  {
    ktimer_scope kt(BYO_K_PR_PULL, s);
    pr_tile_kernel<SHIFT><<<(unsigned)p->nchunks, PT_THREADS, 0, s>>>(
        p->ent, p->anchor, p->cbeg, contrib, (unsigned long long *)p->partial, dpart, nparts, (double)damping, g->n,
        base);
  }
  ktimer_scope ka(BYO_K_PR_CHUNK, s);
  pr_tile_apply_kernel<SHIFT><<<(unsigned)pr_tile_parts(g), PT_APPLY, 0, s>>>(
      (const unsigned long long *)p->partial, p->bfirst, p->rdeg, p->orig, g->n, base, damping, contrib_next, dpart,
      out);
}

// One step in relabelled order: contrib indexed by relabelled vertex
// (initialised from the layout's degrees), dpart holds the previous step's
// dangling partials on entry (pr_tile_parts(g) of them) and this step's on
// return; out (nullable) receives p' in the caller's order.
byo_status pr_tile_step(byo_graph *g, const float *contrib, float damping, float *contrib_next, float *out,
                        hipStream_t s) {
  byo_tiles *p = g->ws.tiles;
  BYO_CHECK(p, BYO_ESTATE, "tile layout not built");
  BYO_TRY(tiles_partial(p, sizeof(unsigned long long) << p->shift));
  byo_workspace &w = g->ws;
  BYO_CHECK(p->nchunks > 0, BYO_ESTATE, "tile layout without entries");
  int64_t nparts = pr_tile_parts(g);
  switch (p->shift) {
    case 12: launch_step<12>(p, g, contrib, damping, contrib_next, out, w.dpart, w.base, nparts, s); break;
    case 13: launch_step<13>(p, g, contrib, damping, contrib_next, out, w.dpart, w.base, nparts, s); break;
    default: launch_step<14>(p, g, contrib, damping, contrib_next, out, w.dpart, w.base, nparts, s); break;
  }
  BYO_HIP(hipGetLastError());
  return BYO_OK;
}

}  // namespace byo
