// Degree-ordered destination-tile layout of the edge set, shared by the
// tiled PageRank step, the tiled multi-source BFS level and the tiled
// connectivity round. Built on the device once per graph (and tile size) on
// first use, kept with the graph.
//
// Dense pull levels gather a per-vertex value (a contribution, a frontier
// mask) for every edge at a random address; one L2 request per edge bounds
// them. In this layout:
//  - vertices are relabelled by descending degree (ties by ID), so the
//    sources that occur in many tiles share cache lines and the isolated
//    vertices come last;
//  - entries (u, v) are grouped by the tile of v (2^shift consecutive
//    relabelled vertices) and ordered by relabelled u inside a tile;
//  - each tile is cut into chunks of about equal entry count (about 512
//    chunks over the graph), one workgroup each.
// A workgroup keeps its tile's accumulators in LDS; its lanes read
// consecutive entries, whose sources are close together, so a wavefront's
// gathers fall in few cache lines. An entry is one 32-bit word: a 16-bit
// offset of its source from its 64-entry group's anchor (the base of the
// 2^16-aligned source window the group lies in) and its 16-bit tile-local
// destination; a wavefront's load is one group, so the anchor is one scalar
// load.
#include <cstring>

#include <algorithm>
#include <vector>

#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>

#include "internal.h"

namespace byo {

bool tiles_wanted(const byo_graph *g) { return g->n >= (1ll << 16) && g->m >= 4 * g->n && g->m > 0; }

static void tiles_free(byo_tiles *p) {
  void *d[] = {p->ent, p->anchor, p->rdeg, p->orig, p->cbeg, p->bfirst, p->cblk, p->cflag, p->rlabel,
               p->scratch, p->partial, p->roff, p->rnbr, p->aplan};
  for (void *x : d)
    if (x) (void)hipFree(x);
  delete p;
}

void tiles_release(byo_workspace &w) {
  for (auto &t : w.tiles) {
    if (t) tiles_free(t);
    t = nullptr;
  }
}

int tiles_auto_shift(const byo_graph *g) {
  int lg = 0;
  while (lg < 62 && ((int64_t)1 << lg) < g->n) ++lg;
  return std::min(14, std::max(12, lg - 10));
}

// Device construction of the tile layout, all on the caller's stream:
//  1. stable radix sort of the vertices by descending degree (ties keep ID
//     order): orig, then rlabel and rdeg by scatter;
//  2. roff = exclusive scan of rdeg; row[p], the relabelled row of CSR slot p,
//     is a max-scan of the row starts;
//  3. one pass over the slots writes the relabelled CSR and, per entry, the
//     destination tile (key) and (source << 16 | tile-local destination);
//  4. a stable radix sort by tile keeps the sources ascending inside a tile;
//  5. packing: a group never crosses a 2^16-aligned source window, so its
//     anchor is the window base, and a (tile, window) segment is cut into
//     plain 64-entry groups, the last one padded. Segments come from a scan
//     of "segment starts here" flags, group offsets from a scan of the
//     per-segment group counts; every entry is then placed independently.
namespace {

constexpr int TL_THREADS = 256;

unsigned tl_blocks(int64_t count) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>((count + TL_THREADS - 1) / TL_THREADS, 1 << 16));
}

__global__ void tl_degkey_kernel(const int32_t *__restrict__ deg, int64_t n, int64_t max_deg, uint32_t *key,
                                 int32_t *idx) {
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    key[v] = (uint32_t)(max_deg - deg[v]);
    idx[v] = (int32_t)v;
  }
}

__global__ void tl_label_kernel(const int32_t *__restrict__ orig, const int32_t *__restrict__ deg, int64_t n,
                                int32_t *rlabel, int32_t *rdeg) {
  for (int64_t w = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; w < n; w += (int64_t)gridDim.x * blockDim.x) {
    const int32_t v = orig[w];
    rlabel[v] = (int32_t)w;
    rdeg[w] = deg[v];
  }
}

// rowmark[roff[w]] = w for every non-empty row (rowmark zeroed before); the
// running maximum of rowmark is then the row of each slot.
__global__ void tl_rowmark_kernel(const int64_t *__restrict__ roff, const int32_t *__restrict__ rdeg, int64_t n,
                                  int32_t *rowmark) {
  for (int64_t w = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; w < n; w += (int64_t)gridDim.x * blockDim.x)
    if (rdeg[w] > 0) rowmark[roff[w]] = (int32_t)w;
}

__global__ void tl_entries_kernel(const int64_t *__restrict__ off, const int32_t *__restrict__ nbr,
                                  const int32_t *__restrict__ orig, const int32_t *__restrict__ rlabel,
                                  const int64_t *__restrict__ roff, const int32_t *__restrict__ row, int64_t m,
                                  int shift, int32_t *rnbr, uint32_t *key, uint64_t *val) {
  const uint32_t mask = (1u << shift) - 1;
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < m; p += (int64_t)gridDim.x * blockDim.x) {
    const int32_t w = row[p];
    const int32_t x = rlabel[nbr[off[orig[w]] + (p - roff[w])]];
    rnbr[p] = x;
    key[p] = (uint32_t)x >> shift;
    val[p] = ((uint64_t)(uint32_t)w << 16) | ((uint32_t)x & mask);
  }
}

// first entry of every tile b in [0, nblk] (m for tiles past the last entry)
__global__ void tl_tile_off_kernel(const uint32_t *__restrict__ key, int64_t m, int64_t nblk, int64_t *tile_off) {
  const int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (b > nblk) return;
  int64_t lo = 0, hi = m;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if ((int64_t)key[mid] < b) lo = mid + 1;
    else hi = mid;
  }
  tile_off[b] = lo;
}

// a segment (same tile, same 2^16 source window) starts at p
__global__ void tl_segflag_kernel(const uint32_t *__restrict__ key, const uint64_t *__restrict__ val, int64_t m,
                                  uint32_t *flag) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < m; p += (int64_t)gridDim.x * blockDim.x)
    flag[p] = p == 0 || key[p] != key[p - 1] || (val[p] >> 32) != (val[p - 1] >> 32);
}

// segid is the inclusive count of segment starts, so segment segid[p] - 1
// holds p; segbeg[nseg] = m closes the last one.
__global__ void tl_segbeg_kernel(const uint32_t *__restrict__ flag, const int64_t *__restrict__ segid, int64_t m,
                                 int64_t *segbeg) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < m; p += (int64_t)gridDim.x * blockDim.x) {
    if (flag[p]) segbeg[segid[p] - 1] = p;
    if (p == m - 1) segbeg[segid[p]] = m;
  }
}

__global__ void tl_segroups_kernel(const int64_t *__restrict__ segbeg, int64_t nseg, int64_t *ngroups) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i <= nseg; i += (int64_t)gridDim.x * blockDim.x)
    ngroups[i] = i < nseg ? (segbeg[i + 1] - segbeg[i] + 63) / 64 : 0;
}

// ent was filled with padding; every real entry goes to its segment's groups
// at its offset in the segment, and a group's first entry writes the anchor.
__global__ void tl_place_kernel(const uint64_t *__restrict__ val, const int64_t *__restrict__ segid,
                                const int64_t *__restrict__ segbeg, const int64_t *__restrict__ gbefore, int64_t m,
                                uint32_t *ent, int32_t *anchor) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < m; p += (int64_t)gridDim.x * blockDim.x) {
    const int64_t sg = segid[p] - 1, l = p - segbeg[sg], q = gbefore[sg] * 64 + l;
    const uint64_t x = val[p];
    const uint32_t w = (uint32_t)(x >> 16), base = w & ~0xffffu;
    ent[q] = (w - base) | ((uint32_t)(x & 0xffffu) << 16);
    if ((l & 63) == 0) anchor[q >> 6] = (int32_t)base;
  }
}

// first group of every tile b in [0, nblk]
__global__ void tl_tile_groups_kernel(const int64_t *__restrict__ tile_off, const int64_t *__restrict__ segid,
                                      const int64_t *__restrict__ gbefore, int64_t m, int64_t nblk, int64_t nseg,
                                      int64_t *tgrp) {
  const int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (b > nblk) return;
  const int64_t p = tile_off[b];
  tgrp[b] = p >= m ? gbefore[nseg] : gbefore[segid[p] - 1];
}

// device buffers of one build, freed on every exit once the stream's queued
// work is done
struct tl_tmp {
  hipStream_t s;
  std::vector<void *> v;
  explicit tl_tmp(hipStream_t st) : s(st) {}
  template <class T>
  byo_status get(T **p, size_t count) {
    *p = nullptr;
    BYO_HIP(hipMalloc((void **)p, sizeof(T) * std::max<size_t>(count, 1)));
    v.push_back(*p);
    return BYO_OK;
  }
  ~tl_tmp() {
    (void)hipStreamSynchronize(s);
    for (void *x : v) (void)hipFree(x);
  }
};

int bits_for(int64_t x) {  // bits needed to hold 0 .. x
  int b = 1;
  while (b < 63 && (x >> b) != 0) ++b;
  return b;
}

}  // namespace

static byo_status tiles_build(const byo_graph *g, byo_tiles *p, hipStream_t s) {
  const int64_t n = p->n, m = p->m, nblk = p->nblk;
  const int shift = p->shift;
  tl_tmp tmp(s);
  uint32_t *vkey = nullptr, *vkey2 = nullptr, *ka = nullptr, *kb = nullptr;
  int32_t *vidx = nullptr;
  uint64_t *va = nullptr, *vb = nullptr;
  BYO_TRY(tmp.get(&vkey, (size_t)n));
  BYO_TRY(tmp.get(&vkey2, (size_t)n));
  BYO_TRY(tmp.get(&vidx, (size_t)n));
  BYO_TRY(tmp.get(&ka, (size_t)m));
  BYO_TRY(tmp.get(&kb, (size_t)m));
  BYO_TRY(tmp.get(&va, (size_t)m));
  BYO_TRY(tmp.get(&vb, (size_t)m));
  BYO_HIP(hipMalloc(&p->orig, sizeof(int32_t) * (size_t)n));
  BYO_HIP(hipMalloc(&p->rlabel, sizeof(int32_t) * (size_t)n));
  BYO_HIP(hipMalloc(&p->rdeg, sizeof(int32_t) * (size_t)n));
  BYO_HIP(hipMalloc(&p->roff, sizeof(int64_t) * (size_t)(n + 1)));
  BYO_HIP(hipMalloc(&p->rnbr, sizeof(int32_t) * (size_t)m));
  int32_t *rowmark = (int32_t *)ka, *row = (int32_t *)kb;
  int64_t *segid = (int64_t *)va;
  const unsigned dbits = (unsigned)bits_for(g->max_deg), tbits = (unsigned)bits_for(nblk - 1);
  // one temporary buffer, as large as the largest library call needs
  size_t q[6] = {0, 0, 0, 0, 0, 0};
  BYO_HIP(rocprim::radix_sort_pairs(nullptr, q[0], vkey, vkey2, vidx, p->orig, (size_t)n, 0u, dbits, s));
  BYO_HIP(rocprim::exclusive_scan(nullptr, q[1], p->rdeg, p->roff, (long long)0, (size_t)n,
                                  rocprim::plus<long long>(), s));
  BYO_HIP(rocprim::inclusive_scan(nullptr, q[2], rowmark, row, (size_t)m, rocprim::maximum<int32_t>(), s));
  BYO_HIP(rocprim::radix_sort_pairs(nullptr, q[3], ka, kb, va, vb, (size_t)m, 0u, tbits, s));
  BYO_HIP(rocprim::inclusive_scan(nullptr, q[4], ka, segid, (size_t)m, rocprim::plus<long long>(), s));
  BYO_HIP(rocprim::exclusive_scan(nullptr, q[5], segid, segid, (long long)0, (size_t)m + 1,
                                  rocprim::plus<long long>(), s));
  size_t qmax = *std::max_element(q, q + 6);
  void *ts = nullptr;
  BYO_TRY(tmp.get((uint8_t **)&ts, qmax));
  // 1. relabel by descending degree
  tl_degkey_kernel<<<tl_blocks(n), TL_THREADS, 0, s>>>(g->deg, n, g->max_deg, vkey, vidx);
  BYO_HIP(hipGetLastError());
  BYO_HIP(rocprim::radix_sort_pairs(ts, qmax, vkey, vkey2, vidx, p->orig, (size_t)n, 0u, dbits, s));
  tl_label_kernel<<<tl_blocks(n), TL_THREADS, 0, s>>>(p->orig, g->deg, n, p->rlabel, p->rdeg);
  BYO_HIP(hipGetLastError());
  // 2. relabelled row offsets and the row of every slot
  BYO_HIP(rocprim::exclusive_scan(ts, qmax, p->rdeg, p->roff, (long long)0, (size_t)n, rocprim::plus<long long>(),
                                  s));
  BYO_TRY(fill_u64((uint64_t *)(p->roff + n), 1, (uint64_t)m, s));
  BYO_HIP(hipMemsetAsync(rowmark, 0, sizeof(int32_t) * (size_t)m, s));
  tl_rowmark_kernel<<<tl_blocks(n), TL_THREADS, 0, s>>>(p->roff, p->rdeg, n, rowmark);
  BYO_HIP(hipGetLastError());
  BYO_HIP(rocprim::inclusive_scan(ts, qmax, rowmark, row, (size_t)m, rocprim::maximum<int32_t>(), s));
  // 3. relabelled CSR, tile keys and packed (source, destination) values
  tl_entries_kernel<<<tl_blocks(m), TL_THREADS, 0, s>>>(g->off, g->nbr, p->orig, p->rlabel, p->roff, row, m, shift,
                                                        p->rnbr, ka, va);
  BYO_HIP(hipGetLastError());
  // 4. group by tile, sources still ascending inside a tile
  BYO_HIP(rocprim::radix_sort_pairs(ts, qmax, ka, kb, va, vb, (size_t)m, 0u, tbits, s));
  int64_t *tile_off = nullptr, *tgrp = nullptr;
  BYO_TRY(tmp.get(&tile_off, (size_t)nblk + 1));
  BYO_TRY(tmp.get(&tgrp, (size_t)nblk + 1));
  tl_tile_off_kernel<<<tl_blocks(nblk + 1), TL_THREADS, 0, s>>>(kb, m, nblk, tile_off);
  BYO_HIP(hipGetLastError());
  // 5. segments and their groups
  uint32_t *flag = ka;
  tl_segflag_kernel<<<tl_blocks(m), TL_THREADS, 0, s>>>(kb, vb, m, flag);
  BYO_HIP(hipGetLastError());
  BYO_HIP(rocprim::inclusive_scan(ts, qmax, flag, segid, (size_t)m, rocprim::plus<long long>(), s));
  int64_t nseg = 0;
  BYO_TRY(sync_read(s, segid + (m - 1), &nseg, sizeof(nseg)));
  int64_t *segbeg = nullptr, *ngrp = nullptr, *gbefore = nullptr;
  BYO_TRY(tmp.get(&segbeg, (size_t)nseg + 1));
  BYO_TRY(tmp.get(&ngrp, (size_t)nseg + 1));
  BYO_TRY(tmp.get(&gbefore, (size_t)nseg + 1));
  tl_segbeg_kernel<<<tl_blocks(m), TL_THREADS, 0, s>>>(flag, segid, m, segbeg);
  BYO_HIP(hipGetLastError());
  tl_segroups_kernel<<<tl_blocks(nseg + 1), TL_THREADS, 0, s>>>(segbeg, nseg, ngrp);
  BYO_HIP(hipGetLastError());
  BYO_HIP(rocprim::exclusive_scan(ts, qmax, ngrp, gbefore, (long long)0, (size_t)nseg + 1,
                                  rocprim::plus<long long>(), s));
  tl_tile_groups_kernel<<<tl_blocks(nblk + 1), TL_THREADS, 0, s>>>(tile_off, segid, gbefore, m, nblk, nseg, tgrp);
  BYO_HIP(hipGetLastError());
  std::vector<int64_t> ptile((size_t)nblk + 1);
  BYO_TRY(sync_read(s, tgrp, ptile.data(), sizeof(int64_t) * ptile.size()));
  const int64_t ngroups = ptile[(size_t)nblk];
  BYO_CHECK(ngroups < ((int64_t)1 << 31), BYO_EINVAL, "too many entry groups");
  for (auto &x : ptile) x *= 64;
  const int64_t mp = ngroups * 64;
  p->mp = mp;
  BYO_HIP(hipMalloc(&p->ent, sizeof(uint32_t) * (size_t)std::max<int64_t>(mp, 1)));
  BYO_HIP(hipMalloc(&p->anchor, sizeof(int32_t) * (size_t)std::max<int64_t>(ngroups, 1)));
  // padding points at the dummy slot 2^shift, one past the tile
  BYO_TRY(fill_i32((int32_t *)p->ent, mp, (int32_t)((1u << shift) << 16), s));
  tl_place_kernel<<<tl_blocks(m), TL_THREADS, 0, s>>>(vb, segid, segbeg, gbefore, m, p->ent, p->anchor);
  BYO_HIP(hipGetLastError());
  // chunks: about 512 over the whole entry set, each tile cut into equal
  // pieces of whole groups
  const int64_t target = std::max<int64_t>(1 << 16, (mp + 511) / 512);
  std::vector<int64_t> cbeg;
  std::vector<int32_t> bfirst((size_t)nblk + 1), cblk;
  for (int64_t b = 0; b < nblk; ++b) {
    bfirst[(size_t)b] = (int32_t)cbeg.size();
    int64_t lo = ptile[(size_t)b], groups = (ptile[(size_t)b + 1] - lo) / 64;
    if (groups == 0) continue;
    int64_t k = (groups * 64 + target - 1) / target;
    for (int64_t i = 0; i < k; ++i) {
      cbeg.push_back(lo + 64 * (groups * i / k));
      cblk.push_back((int32_t)b);
    }
  }
  bfirst[(size_t)nblk] = (int32_t)cbeg.size();
  p->nchunks = (int64_t)cbeg.size();
  cbeg.push_back(mp);
  BYO_HIP(hipMalloc(&p->cbeg, sizeof(int64_t) * cbeg.size()));
  BYO_HIP(hipMalloc(&p->bfirst, sizeof(int32_t) * bfirst.size()));
  BYO_HIP(hipMalloc(&p->cblk, sizeof(int32_t) * (size_t)std::max<int64_t>(p->nchunks, 1)));
  BYO_HIP(hipMalloc(&p->cflag, sizeof(uint32_t) * (size_t)std::max<int64_t>(p->nchunks, 1)));
  BYO_HIP(hipMemcpyAsync(p->cbeg, cbeg.data(), sizeof(int64_t) * cbeg.size(), hipMemcpyHostToDevice, s));
  BYO_HIP(hipMemcpyAsync(p->bfirst, bfirst.data(), sizeof(int32_t) * bfirst.size(), hipMemcpyHostToDevice, s));
  BYO_HIP(hipMemcpyAsync(p->cblk, cblk.data(), sizeof(int32_t) * cblk.size(), hipMemcpyHostToDevice, s));
  // PageRank apply plan, over the tiles cut into several chunks (a tile of
  // one chunk is finished by its chunk's workgroup): a tile with more than 8
  // chunks (the highest-degree destinations) gets 64-vertex workgroups so
  // that its many chunk sums are spread over many workgroups; the others get
  // 1024-vertex workgroups
  std::vector<int32_t> plan;
  int64_t btail = nblk;  // tiles from btail on have no entries
  while (btail > 0 && bfirst[(size_t)btail] == bfirst[(size_t)btail - 1]) --btail;
  p->wtail = std::min<int64_t>(n, btail << shift);
  for (int64_t b = 0; b < nblk; ++b) {
    const int64_t k = bfirst[(size_t)b + 1] - bfirst[(size_t)b];
    if (k <= 1) continue;
    const int64_t v0 = b << shift, v1 = std::min<int64_t>(n, (b + 1) << shift);
    for (int64_t v = v0; v < v1; v += k > 8 ? 64 : 1024) plan.push_back((int32_t)v | (k > 8 ? 1 : 0));
  }
  p->napply = (int64_t)plan.size();
  BYO_HIP(hipMalloc(&p->aplan, sizeof(int32_t) * std::max<size_t>(plan.size(), 1)));
  if (!plan.empty())
    BYO_HIP(hipMemcpyAsync(p->aplan, plan.data(), sizeof(int32_t) * plan.size(), hipMemcpyHostToDevice, s));
  // the temporaries and the host vectors must outlive the queued work
  BYO_HIP(hipStreamSynchronize(s));
  return BYO_OK;
}

byo_status tiles_ensure(byo_graph *g, int shift, hipStream_t s, byo_tiles **out) {
  byo_workspace &w = g->ws;
  BYO_CHECK(shift >= 12 && shift <= 14, BYO_EINVAL, "tile size must be 2^12 .. 2^14");
  byo_tiles *&slot = w.tiles[shift - 12];
  if (slot) {
    *out = slot;
    return BYO_OK;
  }
  BYO_CHECK(tiles_wanted(g), BYO_EINVAL, "graph too small or too sparse for the tile layout");
  BYO_CHECK(g->n <= ((int64_t)1 << 31) - 1, BYO_EINVAL, "graph too large for the tile layout");
  byo_tiles *p = new byo_tiles();
  p->shift = shift;
  p->n = g->n;
  p->m = g->m;
  p->nblk = (g->n + (1ll << shift) - 1) >> shift;
  const byo_status st = tiles_build(g, p, s);
  if (st != BYO_OK) {
    (void)hipStreamSynchronize(s);
    tiles_free(p);
    return st;
  }
  slot = p;
  *out = p;
  return BYO_OK;
}

byo_graph tiles_view(const byo_graph *g, const byo_tiles *t) {
  byo_graph r = *g;
  r.off = t->roff;
  r.nbr = t->rnbr;
  r.deg = t->rdeg;
  return r;
}

byo_status tiles_scratch(byo_tiles *t) {
  if (!t->scratch) BYO_HIP(hipMalloc(&t->scratch, sizeof(int32_t) * (size_t)t->n));
  return BYO_OK;
}

byo_status tiles_partial(byo_tiles *t, size_t bytes_per_chunk) {
  size_t need = bytes_per_chunk * (size_t)std::max<int64_t>(t->nchunks, 1);
  if (t->partial_bytes >= need) return BYO_OK;
  if (t->partial) (void)hipFree(t->partial);
  t->partial = nullptr;
  t->partial_bytes = 0;
  BYO_HIP(hipMalloc(&t->partial, need));
  t->partial_bytes = need;
  return BYO_OK;
}

}  // namespace byo
