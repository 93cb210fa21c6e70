// PageRank step over the degree-ordered destination-tile layout (tiles.hip;
// option pr_blocked = 1, or 12..14 for tiles of 2^value vertices). Same step
// as the pull kernel,
//   p'[v] = (1-d)/n + d * (sum over u in N(v) of contrib[u] + D/n),
// run in the layout's vertex order (contributions and degrees relabelled),
// with p written in the caller's order.
//
// The step constant base = (1-d)/n + d*D/n comes from the host. D, the mass
// on degree-0 vertices, needs no reduction: such a vertex has an empty list,
// so it receives nothing and its rank after every step is that step's base
// (1/n before the first), and D is the number of degree-0 vertices times it.
//
// Sums: LDS atomics on 64-bit fixed point within a chunk. A tile cut into one
// chunk finishes its vertices in the same workgroup (p', next contribution,
// output); a tile cut into several writes chunk partials that the apply
// kernel adds. Integer sums are exact, so the result is the same whatever
// order the atomics land in, and the same in either path.
#include <algorithm>

#include "internal.h"

namespace byo {

constexpr int PT_THREADS = 1024;
constexpr int PT_ILP = 12;
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

// One workgroup per chunk: LDS sums for the chunk's tile. A chunk that is
// its tile's only one then forms p', the next contributions and the optional
// output of the tile's vertices; otherwise it writes its sums densely to its
// partial row for the apply kernel.
template <int SHIFT>
__global__ void __launch_bounds__(PT_THREADS) pr_tile_kernel(const uint32_t *__restrict__ ent,
                                                             const int32_t *__restrict__ anchor,
                                                             const int64_t *__restrict__ cbeg,
                                                             const int32_t *__restrict__ cblk,
                                                             const int32_t *__restrict__ bfirst,
                                                             const float *__restrict__ contrib,
                                                             unsigned long long *__restrict__ partial,
                                                             const int32_t *__restrict__ rdeg,
                                                             const int32_t *__restrict__ orig, int64_t n, float bs,
                                                             float damping, float *__restrict__ contrib_next,
                                                             float *__restrict__ out) {
  constexpr int B = 1 << SHIFT;
  __shared__ unsigned long long acc[B + 1];  // slot B takes the padding entries
  const int t = threadIdx.x;
  const int64_t c = blockIdx.x;
  for (int i = t; i <= B; i += PT_THREADS) acc[i] = 0ull;
  __syncthreads();
  const int64_t beg = cbeg[c], end = cbeg[c + 1];
  // Lane-consecutive entries per load, so a wavefront's gathers cover a
  // narrow source range; PT_ILP independent loads in flight per thread.
  // Indices past the chunk end are clamped to its first entry (a chunk is
  // never empty) and their sums skipped, so the loads stay unconditional and
  // issue back to back. The loop is software-pipelined: the entry words of
  // the next round are requested before this round's gathers are consumed,
  // so the entry latency overlaps the gather latency. Entry words are read
  // once per step, so they are loaded non-temporally and leave the caches to
  // the contributions. A wavefront's 64 lanes read one whole group (chunks
  // are whole groups), so the group index is uniform and the anchor a scalar
  // load.
  constexpr int64_t STEP = (int64_t)PT_THREADS * PT_ILP;
  uint32_t wd[PT_ILP];
  int32_t an[PT_ILP];
  auto fetch = [&](int64_t f0) {
#pragma unroll
    for (int j = 0; j < PT_ILP; ++j) {
      int64_t i = f0 + (int64_t)j * PT_THREADS;
      i = i < end ? i : beg;
      wd[j] = __builtin_nontemporal_load(&ent[i]);
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
  const int32_t b = cblk[c];
  if (bfirst[b + 1] - bfirst[b] == 1) {
    const int64_t w0 = (int64_t)b << SHIFT;
    for (int i = t; i < B; i += PT_THREADS) {
      const int64_t w = w0 + i;
      if (w < n) {
        const float r = bs + damping * (float)((double)acc[i] * 0x1p-61);
        const int32_t dg = rdeg[w];
        if (contrib_next) contrib_next[w] = dg > 0 ? r / (float)dg : 0.0f;
        if (out) out[orig[w]] = r;
      }
    }
    return;
  }
  unsigned long long *row = partial + (c << SHIFT);
  for (int i = t; i < B; i += PT_THREADS) row[i] = acc[i];
}

// p'[w] = base + d * (sum of the chunk partials of w's tile), w relabelled,
// for the tiles cut into several chunks; next contributions in relabelled
// order, the optional output in the caller's order. The workgroup's plan
// word (tiles.hip) picks one of two shapes:
//  - 1024 vertices of a tile with a few chunks: a thread takes PT_AV
//    vertices PT_APPLY apart and issues all their loads before using any, so
//    a wavefront pays the memory latency once for several vertices;
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
                                                                 float bs, float damping,
                                                                 float *__restrict__ contrib_next,
                                                                 float *__restrict__ out) {
  static_assert(((1 << SHIFT) % (PT_APPLY * PT_AV)) == 0, "a workgroup's vertices must share a tile");
  static_assert(PT_APPLY == 256, "the many-chunk shape is 64 vertices x 4 lanes");
  __shared__ unsigned long long red[4][64];
  const int32_t pl = aplan[blockIdx.x];
  const int64_t first = (int64_t)(pl & ~1);
  const int64_t b = first >> SHIFT;
  const int32_t c0 = bfirst[b], c1 = bfirst[b + 1];
  constexpr int64_t MASK = (1 << SHIFT) - 1;
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
      if (out) out[orig[w]] = r;
    }
  }
}

// Vertices of the tiles without entries (all of degree 0, the last ones in
// the layout's order) hold the step constant: written to the output only.
__global__ void pr_tile_tail_kernel(const int32_t *__restrict__ orig, int64_t w0, int64_t n, float bs,
                                    float *__restrict__ out) {
  for (int64_t w = w0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; w < n; w += (int64_t)gridDim.x * blockDim.x)
    out[orig[w]] = bs;
}

template <int SHIFT>
static void launch_step(const byo_tiles *p, const byo_graph *g, const float *contrib, float bs, float damping,
                        float *contrib_next, float *out, hipStream_t s) {
  {
    ktimer_scope kt(BYO_K_PR_PULL, s);
    pr_tile_kernel<SHIFT><<<(unsigned)p->nchunks, PT_THREADS, 0, s>>>(
        p->ent, p->anchor, p->cbeg, p->cblk, p->bfirst, contrib, (unsigned long long *)p->partial, p->rdeg, p->orig,
        g->n, bs, damping, contrib_next, out);
  }
  if (p->napply == 0 && !(out && p->wtail < g->n)) return;
  ktimer_scope ka(BYO_K_PR_CHUNK, s);
  if (p->napply > 0)
    pr_tile_apply_kernel<SHIFT><<<(unsigned)p->napply, PT_APPLY, 0, s>>>(
        (const unsigned long long *)p->partial, p->bfirst, p->aplan, p->rdeg, p->orig, g->n, bs, damping,
        contrib_next, out);
  if (out && p->wtail < g->n)
    pr_tile_tail_kernel<<<(unsigned)std::min<int64_t>((g->n - p->wtail + 255) / 256, 2048), 256, 0, s>>>(
        p->orig, p->wtail, g->n, bs, out);
}

// One step in relabelled order: contrib indexed by relabelled vertex
// (initialised from the layout's degrees), bs = the step constant
// (1-d)/n + d*D/n. out (nullable) receives p' in the caller's order.
byo_status pr_tile_step(byo_graph *g, byo_tiles *p, const float *contrib, float bs, float damping,
                        float *contrib_next, float *out, hipStream_t s) {
  BYO_CHECK(p, BYO_ESTATE, "tile layout not built");
  BYO_TRY(tiles_partial(p, sizeof(unsigned long long) << p->shift));
  BYO_CHECK(p->nchunks > 0, BYO_ESTATE, "tile layout without entries");
  switch (p->shift) {
    case 12: launch_step<12>(p, g, contrib, bs, damping, contrib_next, out, s); break;
    case 13: launch_step<13>(p, g, contrib, bs, damping, contrib_next, out, s); break;
    default: launch_step<14>(p, g, contrib, bs, damping, contrib_next, out, s); break;
  }
  BYO_HIP(hipGetLastError());
  return BYO_OK;
}

}  // namespace byo
