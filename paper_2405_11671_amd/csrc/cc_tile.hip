// Connectivity (minimum-ID labels) over the degree-ordered tile layout
// (tiles.hip; option tiled = 1). Label propagation: every round each vertex
// whose label changed in the round before offers its label to its
// neighbours, a vertex keeps the smallest label offered, and a
// pointer-jumping pass then replaces label x by the label of vertex x when
// smaller. Labels only decrease and are always IDs of vertices in the same
// component, so the fixed point is the minimum ID of each component whatever
// the schedule.
//
// The round runs in the layout's vertex order, but label values are original
// IDs, so the minimum taken is the minimum original ID. A workgroup takes a
// chunk of a destination tile, keeps the tile's minima in LDS (atomic min is
// order-free) and skips entries whose source is not active. A tile cut into
// one chunk is finished by that chunk's workgroup; for the others the apply
// pass takes the minimum over the tile's chunks.
#include <algorithm>
#include <climits>
#include <cstring>

#include "internal.h"

namespace byo {

constexpr int CT_THREADS = 1024;
constexpr int CT_ILP = 16;
constexpr int CT_APPLY = 256;

// Lower lab[w] to m, the smallest label offered to w this round, and hook
// the vertex w's old label named; true if lab[w] changed. Every lane of the
// wavefront calls it (w >= n: nothing); the caller ORs the changed lanes into
// the next active bitmap.
__device__ __forceinline__ bool cc_lower(int64_t w, int64_t n, int32_t m, const int32_t *__restrict__ rlabel,
                                         int32_t *__restrict__ lab, uint64_t *__restrict__ abits_next) {
  if (w >= n) return false;
  const int32_t old = lab[w];
  if (m >= old) return false;
  atomicMin(&lab[w], m);
  // Hooking: the vertex whose ID w carried as its label is in w's component
  // too, so it may take m as well; it becomes active when it drops. Labels
  // only decrease and stay IDs of the component, so the result (the smallest
  // ID of each component) is unchanged; fewer rounds reach it.
  const int32_t h = rlabel[old];
  // (read first: most labels name a few roots, and once a root holds m its
  // hooks would only queue on the same address)
  if (h != w && m < lab[h] && m < atomicMin(&lab[h], m))
    atomicOr((unsigned long long *)&abits_next[h >> 6], 1ull << (h & 63));
  return true;
}

// the changed lanes of a wavefront (first vertex w0, a multiple of 64) into
// the next active bitmap; returns how many
__device__ __forceinline__ unsigned long long cc_mark(bool changed, int64_t w0, int64_t n,
                                                      uint64_t *__restrict__ abits_next) {
  const uint64_t am = __ballot(changed);
  if (lane_id() == 0 && w0 < n && am) {
    atomicOr((unsigned long long *)&abits_next[w0 >> 6], (unsigned long long)am);
    return (unsigned long long)__popcll(am);
  }
  return 0ull;
}

template <int SHIFT, bool ALL>
__global__ void __launch_bounds__(CT_THREADS) cc_tile_kernel(const uint32_t *__restrict__ ent,
                                                             const int32_t *__restrict__ anchor,
                                                             const int64_t *__restrict__ cbeg,
                                                             const int32_t *__restrict__ cblk,
                                                             const int32_t *__restrict__ bfirst,
                                                             const int32_t *__restrict__ rlabel,
                                                             int32_t *__restrict__ lab,
                                                             const uint64_t *__restrict__ abits,
                                                             uint64_t *__restrict__ abits_next, int64_t n,
                                                             byo_counters *__restrict__ ctr,
                                                             int32_t *__restrict__ partial,
                                                             uint32_t *__restrict__ cflag) {
  constexpr int B = 1 << SHIFT;
  __shared__ int32_t acc[B + 1];  // slot B takes the padding entries
  __shared__ int s_any;
  const int t = threadIdx.x;
  const int64_t c = blockIdx.x;
  const int64_t tile = cblk[c];
  const bool single = bfirst[tile + 1] - bfirst[tile] == 1;
  for (int i = t; i <= B; i += CT_THREADS) acc[i] = INT_MAX;
  if (t == 0) s_any = 0;
  __syncthreads();
  const int64_t beg = cbeg[c], end = cbeg[c + 1];
  int mine = 0;
  // Software-pipelined like the PageRank tile pass: the next round's entry
  // words are requested before this round's bitmap and label gathers are
  // consumed. A wavefront reads one whole group, so the anchor index is
  // uniform (a scalar load); indices past the chunk end are clamped. Entry
  // words are read once per round and loaded non-temporally, leaving the
  // caches to the labels (0.269 -> 0.265 ms a pass at RMAT-22). With ALL
  // (every vertex active, the first round) the active bitmap is not read
  // (0.269 -> 0.258 ms; both 0.249 ms).
  constexpr int64_t STEP = (int64_t)CT_THREADS * CT_ILP;
  uint32_t wd[CT_ILP];
  int32_t an[CT_ILP];
  auto fetch = [&](int64_t f0) {
#pragma unroll
    for (int j = 0; j < CT_ILP; ++j) {
      int64_t i = f0 + (int64_t)j * CT_THREADS;
      i = i < end ? i : beg;  // a chunk is never empty
      wd[j] = __builtin_nontemporal_load(&ent[i]);
      an[j] = anchor[__builtin_amdgcn_readfirstlane((int32_t)(i >> 6))];
    }
  };
  int64_t e0 = beg + t;
  fetch(e0);
  for (; e0 < end; e0 += STEP) {
    int32_t u[CT_ILP];
    uint32_t d[CT_ILP];
    uint64_t ab[CT_ILP];
#pragma unroll
    for (int j = 0; j < CT_ILP; ++j) {
      d[j] = wd[j] >> 16;
      u[j] = an[j] + (int32_t)(wd[j] & 0xffffu);
    }
#pragma unroll
    for (int j = 0; j < CT_ILP; ++j) ab[j] = ALL ? ~0ull : abits[u[j] >> 6];
    fetch(e0 + STEP);
    bool ok[CT_ILP];
    bool some = false;
#pragma unroll
    for (int j = 0; j < CT_ILP; ++j) {
      ok[j] = e0 + (int64_t)j * CT_THREADS < end && ((ab[j] >> (u[j] & 63)) & 1ull);
      some |= ok[j];
    }
    if (__any(some)) {
      int32_t x[CT_ILP];
#pragma unroll
      for (int j = 0; j < CT_ILP; ++j) x[j] = lab[ok[j] ? u[j] : 0];
#pragma unroll
      for (int j = 0; j < CT_ILP; ++j)
        if (ok[j]) {
          atomicMin(&acc[d[j]], x[j]);
          mine = 1;
        }
    }
  }
  if (mine) s_any = 1;  // every writer stores the same value
  __syncthreads();
  const int any = s_any;
  if (!single) {
    if (any) {
      int32_t *out = partial + (c << SHIFT);
      for (int i = t; i < B; i += CT_THREADS) out[i] = acc[i];
    }
    if (t == 0) cflag[c] = any ? 1u : 0u;
    return;
  }
  if (!any) return;  // nothing offered to the tile
  unsigned long long count = 0;
  for (int l = t; l < B; l += CT_THREADS) {
    const int64_t w = (tile << SHIFT) + l;
    const bool changed = cc_lower(w, n, acc[l], rlabel, lab, abits_next);
    count += cc_mark(changed, w - lane_id(), n, abits_next);
  }
  const unsigned long long tc = block_sum<unsigned long long, CT_THREADS>(count);
  if (threadIdx.x == 0 && tc) atomicAdd(&ctr->count, tc);
}

// The tiles cut into several chunks, in pieces of the layout's apply plan (a
// word: first vertex, bit 0 set for a 64-vertex piece of a many-chunk tile,
// else 1024 vertices): the smallest label offered to w over its tile's
// chunks lowers lab[w] (cc_lower).
template <int SHIFT>
__global__ void __launch_bounds__(CT_APPLY) cc_tile_apply_kernel(const int32_t *__restrict__ partial,
                                                                 const uint32_t *__restrict__ cflag,
                                                                 const int32_t *__restrict__ bfirst,
                                                                 const int32_t *__restrict__ plan,
                                                                 const int32_t *__restrict__ rlabel,
                                                                 int32_t *__restrict__ lab,
                                                                 uint64_t *__restrict__ abits_next, int64_t n,
                                                                 byo_counters *__restrict__ ctr) {
  constexpr int B = 1 << SHIFT;
  const int32_t piece = plan[blockIdx.x];
  const int64_t v0 = piece & ~1;
  const int64_t v1 = std::min<int64_t>(v0 + ((piece & 1) ? 64 : 1024), n);
  unsigned long long count = 0;
  for (int64_t base = v0; base < v1; base += CT_APPLY) {  // uniform per workgroup
    const int64_t w = base + threadIdx.x;
    int32_t m = INT_MAX;
    if (w < v1) {
      const int64_t b = w >> SHIFT, l = w & (B - 1);
      const int32_t *pl = partial + l;
      const int32_t c1 = bfirst[b + 1];
      int32_t c = bfirst[b];
      for (; c + 8 <= c1; c += 8) {
        uint32_t f[8];
        int32_t x[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) f[j] = cflag[c + j];
        if (!(f[0] | f[1] | f[2] | f[3] | f[4] | f[5] | f[6] | f[7])) continue;
#pragma unroll
        for (int j = 0; j < 8; ++j) x[j] = pl[(int64_t)(c + j) << SHIFT];
#pragma unroll
        for (int j = 0; j < 8; ++j) m = (f[j] && x[j] < m) ? x[j] : m;
      }
      for (; c < c1; ++c)
        if (cflag[c]) m = min(m, pl[(int64_t)c << SHIFT]);
    }
    const bool changed = cc_lower(w < v1 ? w : n, n, m, rlabel, lab, abits_next);
    // a wavefront past a 64-vertex piece marks nothing (no lane changed)
    count += cc_mark(changed, w - lane_id(), n, abits_next);
  }
  unsigned long long tc = block_sum<unsigned long long, CT_APPLY>(count);
  if (threadIdx.x == 0 && tc) atomicAdd(&ctr->count, tc);
}

// Pointer jumping: label x of w becomes the label of vertex x when smaller
// (x is an original ID; rlabel maps it to the layout's order). Reads of
// labels being lowered by other threads see either value; both are IDs in
// the component, so any interleaving is sound. Vertices it lowers join the
// next round's frontier; the count covers only bits not already set, so it
// stays equal to the frontier bitmap's population.
__global__ void __launch_bounds__(CT_APPLY) cc_tile_jump_kernel(int32_t *__restrict__ lab,
                                                                const int32_t *__restrict__ rlabel,
                                                                uint64_t *__restrict__ abits_next, int64_t n,
                                                                byo_counters *__restrict__ ctr) {
  unsigned long long count = 0;
  for (int64_t base = (int64_t)blockIdx.x * CT_APPLY; base < n; base += (int64_t)gridDim.x * CT_APPLY) {
    const int64_t w = base + threadIdx.x;
    // a vertex already marked this round is counted once: only fresh bits count
    const uint64_t oldw = w < n ? abits_next[w >> 6] : 0ull;
    bool fresh = false;
    if (w < n) {
      int32_t x = lab[w];
      int32_t y = lab[rlabel[x]];
      if (y < x) {
        lab[w] = y;
        fresh = !((oldw >> (w & 63)) & 1ull);
      }
    }
    const uint64_t am = __ballot(fresh);
    if (lane_id() == 0 && w < n && am) {
      abits_next[w >> 6] = oldw | am;
      count += (unsigned long long)__popcll(am);
    }
  }
  unsigned long long tc = block_sum<unsigned long long, CT_APPLY>(count);
  if (threadIdx.x == 0 && tc) atomicAdd(&ctr->count, tc);
}

__global__ void cc_tile_init_kernel(const int32_t *__restrict__ orig, int64_t n, int32_t *__restrict__ lab,
                                    uint64_t *__restrict__ abits) {
  int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (w < n) lab[w] = orig[w];
  int64_t words = (n + 63) / 64;
  if (w < words) abits[w] = (w + 1) * 64 <= n ? ~0ull : (~0ull >> (64 - (n & 63)));
}

__global__ void cc_tile_out_kernel(const int32_t *__restrict__ lab, const int32_t *__restrict__ orig, int64_t n,
                                   int32_t *__restrict__ out) {
  int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (w < n) out[orig[w]] = lab[w];
}

static unsigned apply_grid(int64_t n) {
  return (unsigned)std::min<int64_t>(std::max<int64_t>(1, (n + CT_APPLY - 1) / CT_APPLY), 2048);
}

template <int SHIFT>
static void cc_tile_pass(const byo_tiles *t, int32_t *lab, const uint64_t *abits, uint64_t *abits_next,
                         byo_counters *ctr, int64_t n, bool all, hipStream_t s) {
  ktimer_scope kt(BYO_K_CC_PULL, s);
  // the passes OR their bits in (a hooked vertex may sit in another wavefront's word)
  (void)fill_u64(abits_next, (n + 63) / 64, 0ull, s);
  // the first round has every vertex active: its kernel skips the bitmap
  auto kern = all ? cc_tile_kernel<SHIFT, true> : cc_tile_kernel<SHIFT, false>;
  kern<<<(unsigned)t->nchunks, CT_THREADS, 0, s>>>(t->ent, t->anchor, t->cbeg, t->cblk, t->bfirst, t->rlabel, lab,
                                                   abits, abits_next, n, ctr, (int32_t *)t->partial, t->cflag);
  if (t->napply > 0)
    cc_tile_apply_kernel<SHIFT><<<(unsigned)t->napply, CT_APPLY, 0, s>>>(
        (const int32_t *)t->partial, t->cflag, t->bfirst, t->aplan, t->rlabel, lab, abits_next, n, ctr);
}

// Rounds in the layout's order, direction-optimising: a push over the
// relabelled CSR (the push kernels with the atomic-min functor) while the
// changed vertices number at most n / div, the sparse/dense rule at average
// degree, else a pass over the tiles; each round ends with the
// pointer-jumping pass when enabled.
byo_status cc_tiled_run(byo_graph *g, int32_t *d_label, const byo_opts &o, hipStream_t s, byo_run_stats *stats) {
  BYO_TRY(ws_ensure_traversal(g));
  byo_tiles *t = nullptr;
  BYO_TRY(tiles_ensure(g, (o.tile_shift >= 12 && o.tile_shift <= 14) ? o.tile_shift : tiles_auto_shift(g), s, &t));
  BYO_TRY(tiles_partial(t, sizeof(int32_t) << t->shift));
  BYO_TRY(tiles_scratch(t));
  byo_workspace &w = g->ws;
  const int64_t n = g->n, words = (n + 63) / 64;
  int32_t *lab = t->scratch;
  cc_tile_init_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(t->orig, n, lab, w.bits[0]);
  BYO_HIP(hipGetLastError());
  byo_graph rg = tiles_view(g, t);
  const int64_t div = o.dense_divisor > 0 ? o.dense_divisor : 20;
  byo_run_stats st;
  std::memset(&st, 0, sizeof(st));
  int64_t cap = o.max_levels > 0 ? o.max_levels : n + 1;
  int64_t acount = n;
  int cur = 0;
  int32_t round = 0;
  while (true) {
    if (round >= cap) {
      if (stats) *stats = st;
      return fail(BYO_ELIMIT, "connectivity round cap reached");
    }
    byo_counters *ctr = w.ctr;
    BYO_HIP(hipMemsetAsync(ctr, 0, sizeof(byo_counters), s));
    uint64_t *an = w.bits[1 - cur];
    const bool push = acount <= n / div;
    if (push) {
      BYO_TRY(bitmap_to_ids(w.bits[cur], words, n, w.ids[cur], w.partial, w.partial_cap,
                            (unsigned long long *)w.misc, s));
      level_io io;
      std::memset(&io, 0, sizeof(io));
      io.in_ids = w.ids[cur];
      io.in_count = acount;
      io.out_bits = an;
      io.ctr = ctr;
      BYO_TRY(cc_level(&rg, BYO_V_PUSH_EDGE, lab, io, o, s, -1));  // -1: the push measures its edge total
    } else {
      switch (t->shift) {
        case 13: cc_tile_pass<13>(t, lab, w.bits[cur], an, ctr, n, acount >= n, s); break;
        case 14: cc_tile_pass<14>(t, lab, w.bits[cur], an, ctr, n, acount >= n, s); break;
        default: cc_tile_pass<12>(t, lab, w.bits[cur], an, ctr, n, acount >= n, s); break;
      }
    }
    if (o.cc_shortcut) {
      ktimer_scope kt(BYO_K_CC_SHORTCUT, s);
      cc_tile_jump_kernel<<<apply_grid(n), CT_APPLY, 0, s>>>(lab, t->rlabel, an, n, ctr);
    }
    BYO_HIP(hipGetLastError());
    byo_counters c;
    BYO_TRY(sync_read(s, ctr, &c, sizeof(c)));
    st.variant_count[push ? BYO_V_PUSH_EDGE : BYO_V_PULL_WAVE]++;
    ++round;
    cur = 1 - cur;
    acount = (int64_t)c.count;
    if (c.count == 0) break;
  }
  cc_tile_out_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(lab, t->orig, n, d_label);
  BYO_HIP(hipGetLastError());
  st.levels = round;
  if (stats) *stats = st;
  return BYO_OK;
}

}  // namespace byo
