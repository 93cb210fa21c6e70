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
constexpr int PT_AV = 4;

int pr_tile_shift(const byo_graph *g, int32_t opt) { return (opt >= 12 && opt <= 14) ? opt : tiles_auto_shift(g); }

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
  // issue back to back. The loop is software-pipelined: the entry words of
  // the next round are requested before this round's gathers are consumed,
  // so the entry latency overlaps the gather latency. A wavefront's 64 lanes
  // read one whole group (chunks are whole groups), so the group index is
  // uniform and the anchor a scalar load.
  constexpr int64_t STEP = (int64_t)PT_THREADS * PT_ILP;
  uint32_t wd[PT_ILP];
  int32_t an[PT_ILP];
  auto fetch = [&](int64_t f0) {
#pragma unroll
    for (int j = 0; j < PT_ILP; ++j) {
      int64_t i = f0 + (int64_t)j * PT_THREADS;
      i = i < end ? i : beg;
      wd[j] = ent[i];
      an[j] = anchor[__builtin_amdgcn_readfirstlane((int32_t)(i >> 6))];
    }
  };
  int64_t e0 = beg + t;
  fetch(e0);
  for (; e0 < end; e0 += STEP) {
    uint32_t d[PT_ILP];
    float x[PT_ILP];
#pragma unroll
    for (int j = 0; j < PT_ILP; ++j) {
      d[j] = wd[j] >> 16;
      x[j] = contrib[an[j] + (int32_t)(wd[j] & 0xffffu)];
    }
    fetch(e0 + STEP);
#pragma unroll
    for (int j = 0; j < PT_ILP; ++j)
      if (e0 + (int64_t)j * PT_THREADS < end) atomicAdd(&acc[d[j]], to_fixed(x[j]));
  }
  __syncthreads();
  unsigned long long *out = partial + (c << SHIFT);
  for (int i = t; i < B; i += PT_THREADS) out[i] = acc[i];
}

// p'[w] = base + d * (sum of the chunk partials of w's tile), w relabelled;
// next contributions and one dangling partial per workgroup in relabelled
// order, the optional output in the caller's order. The workgroup's plan
// word (tiles.hip) picks one of two shapes:
//  - 1024 vertices of a tile with few chunks: a thread takes PT_AV vertices
//    PT_APPLY apart and issues all their loads before using any, so a
//    wavefront pays the memory latency once for several vertices;
//  - 64 vertices of a tile with many chunks (the highest-degree
//    destinations, over 100 chunks at RMAT-22): four lanes per vertex each
//    add every fourth chunk, then LDS combines them, so those tiles' long
//    sums are spread over many workgroups instead of setting the kernel's
//    length.
template <int SHIFT>
__global__ void __launch_bounds__(PT_APPLY) pr_tile_apply_kernel(const unsigned long long *__restrict__ partial,
                                                                 const int32_t *__restrict__ bfirst,
                                                                 const int32_t *__restrict__ aplan,
                                                                 const int32_t *__restrict__ rdeg,
                                                                 const int32_t *__restrict__ orig, int64_t n,
                                                                 const float *__restrict__ base, float damping,
                                                                 float *__restrict__ contrib_next,
                                                                 float *__restrict__ dpart, float *__restrict__ out) {
  static_assert(((1 << SHIFT) % (PT_APPLY * PT_AV)) == 0, "a workgroup's vertices must share a tile");
  static_assert(PT_APPLY == 256, "the many-chunk shape is 64 vertices x 4 lanes");
  __shared__ unsigned long long red[4][64];
  const int32_t pl = aplan[blockIdx.x];
  const int64_t first = (int64_t)(pl & ~1);
  const int64_t b = first >> SHIFT;
  const int32_t c0 = bfirst[b], c1 = bfirst[b + 1];
  const float bs = base[0];
  constexpr int64_t MASK = (1 << SHIFT) - 1;
  float dang = 0.0f;
  if ((pl & 1) == 0) {
    // partial rows hold all 2^SHIFT slots of the tile, so the loads of
    // vertices past n (in the last tile) stay inside the row
    const int64_t w0 = first + threadIdx.x;
    const unsigned long long *pp = partial + (w0 & MASK);
    int32_t dg[PT_AV];
#pragma unroll
    for (int j = 0; j < PT_AV; ++j) {
      const int64_t w = w0 + (int64_t)j * PT_APPLY;
      dg[j] = w < n ? rdeg[w] : 0;
    }
    unsigned long long q[PT_AV];
#pragma unroll
    for (int j = 0; j < PT_AV; ++j) q[j] = 0ull;
    int32_t c = c0;
    for (; c + 2 <= c1; c += 2) {
      unsigned long long x[2 * PT_AV];
#pragma unroll
      for (int k = 0; k < 2; ++k)
#pragma unroll
        for (int j = 0; j < PT_AV; ++j) x[k * PT_AV + j] = pp[((int64_t)(c + k) << SHIFT) + j * PT_APPLY];
#pragma unroll
      for (int k = 0; k < 2; ++k)
#pragma unroll
        for (int j = 0; j < PT_AV; ++j) q[j] += x[k * PT_AV + j];
    }
    if (c < c1) {
#pragma unroll
      for (int j = 0; j < PT_AV; ++j) q[j] += pp[((int64_t)c << SHIFT) + j * PT_APPLY];
    }
#pragma unroll
    for (int j = 0; j < PT_AV; ++j) {
      const int64_t w = w0 + (int64_t)j * PT_APPLY;
      if (w < n) {
        const float r = bs + damping * (float)((double)q[j] * 0x1p-61);
        if (contrib_next) contrib_next[w] = dg[j] > 0 ? r / (float)dg[j] : 0.0f;
        if (dg[j] == 0) dang += r;
        if (out) out[orig[w]] = r;
      }
    }
  } else {
    const int v = threadIdx.x & 63, sl = threadIdx.x >> 6;
    const int64_t w = first + v;
    const unsigned long long *pp = partial + (w & MASK);
    unsigned long long q = 0ull;
    int32_t c = c0 + sl;
    for (; c + 28 < c1; c += 32) {  // eight chunks per round, four apart
      unsigned long long x[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) x[k] = pp[(int64_t)(c + 4 * k) << SHIFT];
#pragma unroll
      for (int k = 0; k < 8; ++k) q += x[k];
    }
    for (; c < c1; c += 4) q += pp[(int64_t)c << SHIFT];
    red[sl][v] = q;
    __syncthreads();
    if (sl == 0 && w < n) {
      q = red[0][v] + red[1][v] + red[2][v] + red[3][v];
      const int32_t dg = rdeg[w];
      const float r = bs + damping * (float)((double)q * 0x1p-61);
      if (contrib_next) contrib_next[w] = dg > 0 ? r / (float)dg : 0.0f;
      if (dg == 0) dang = r;
      if (out) out[orig[w]] = r;
    }
  }
  float t = block_sum<float, PT_APPLY>(dang);
  if (threadIdx.x == 0) dpart[blockIdx.x] = t;
}


template <int SHIFT>
static void launch_step(const byo_tiles *p, const byo_graph *g, const float *contrib, float damping, float *contrib_next,
                        float *out, const float *dpart_in, int64_t nparts_in, float *base, hipStream_t s) {
  {
    ktimer_scope kt(BYO_K_PR_PULL, s);
    pr_tile_kernel<SHIFT><<<(unsigned)p->nchunks, PT_THREADS, 0, s>>>(
        p->ent, p->anchor, p->cbeg, contrib, (unsigned long long *)p->partial, dpart_in, nparts_in, (double)damping,
        g->n, base);
  }
  ktimer_scope ka(BYO_K_PR_CHUNK, s);
  pr_tile_apply_kernel<SHIFT><<<(unsigned)p->napply, PT_APPLY, 0, s>>>(
      (const unsigned long long *)p->partial, p->bfirst, p->aplan, p->rdeg, p->orig, g->n, base, damping,
      contrib_next, p->adpart, out);
}

// One step in relabelled order: contrib indexed by relabelled vertex
// (initialised from the layout's degrees); dpart_in holds the nparts_in
// dangling partials of the previous step (the layout's adpart) or of the
// initialisation; this step's go to the layout's adpart (napply of them).
// out (nullable) receives p' in the caller's order.
byo_status pr_tile_step(byo_graph *g, byo_tiles *p, const float *contrib, float damping, float *contrib_next,
                        float *out, const float *dpart_in, int64_t nparts_in, hipStream_t s) {
  BYO_CHECK(p, BYO_ESTATE, "tile layout not built");
  BYO_TRY(tiles_partial(p, sizeof(unsigned long long) << p->shift));
  BYO_CHECK(p->nchunks > 0 && p->napply > 0, BYO_ESTATE, "tile layout without entries");
  BYO_CHECK(dpart_in && nparts_in >= 0, BYO_EINVAL, "dangling partials missing");
  byo_workspace &w = g->ws;
  switch (p->shift) {
    case 12: launch_step<12>(p, g, contrib, damping, contrib_next, out, dpart_in, nparts_in, w.base, s); break;
    case 13: launch_step<13>(p, g, contrib, damping, contrib_next, out, dpart_in, nparts_in, w.base, s); break;
    default: launch_step<14>(p, g, contrib, damping, contrib_next, out, dpart_in, nparts_in, w.base, s); break;
  }
  BYO_HIP(hipGetLastError());
  return BYO_OK;
}

}  // namespace byo
