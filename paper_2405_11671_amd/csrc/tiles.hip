// Degree-ordered destination-tile layout of the edge set, shared by the
// tiled PageRank step and the tiled multi-source BFS level. Built once per
// graph (and tile size) on first use, kept with the graph.
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
// offset of its source from its 64-entry group's anchor and its 16-bit
// tile-local destination; a wavefront's load is one group, so the anchor is
// one scalar load.
#include <algorithm>
#include <thread>
#include <vector>

#include "internal.h"

namespace byo {

bool tiles_wanted(const byo_graph *g) { return g->n >= (1ll << 16) && g->m >= 4 * g->n && g->m > 0; }

void tiles_release(byo_workspace &w) {
  if (!w.tiles) return;
  byo_tiles *p = w.tiles;
  void *d[] = {p->ent, p->anchor, p->rdeg, p->orig, p->cbeg, p->bfirst, p->cblk, p->cflag, p->rlabel,
               p->scratch, p->partial, p->roff, p->rnbr};
  for (void *x : d)
    if (x) (void)hipFree(x);
  delete p;
  w.tiles = nullptr;
}

// Host construction of the tile layout. The relabelling is a counting sort
// by degree, descending, stable in ID. Relabelled rows are then split into
// contiguous ranges of about equal entry count, one per thread; each thread
// counts its entries per tile, the counts become per-thread write cursors
// (tile-major, thread order inside a tile), and each thread copies its
// entries in relabelled row order, so every tile is ordered by source.
static void build_tiles_host(const std::vector<int64_t> &off, const std::vector<int32_t> &nbr, int64_t n, int shift,
                             std::vector<int32_t> &esrc, std::vector<uint16_t> &edst, std::vector<int64_t> &tile_off,
                             std::vector<int32_t> &rdeg, std::vector<int32_t> &orig, std::vector<int32_t> &label) {
  const int64_t m = off[n];
  int64_t max_deg = 0;
  for (int64_t v = 0; v < n; ++v) max_deg = std::max(max_deg, off[v + 1] - off[v]);
  const int64_t nblk = (n + (1ll << shift) - 1) >> shift;
  const uint32_t mask = (1u << shift) - 1;
  // relabel: label[v] = position of v in (degree desc, ID asc) order
  std::vector<int64_t> start((size_t)max_deg + 2, 0);
  for (int64_t v = 0; v < n; ++v) start[(size_t)(max_deg - (off[v + 1] - off[v]))]++;
  int64_t acc = 0;
  for (auto &x : start) {
    int64_t c = x;
    x = acc;
    acc += c;
  }
  label.resize((size_t)n);
  orig.resize((size_t)n);
  rdeg.resize((size_t)n);
  for (int64_t v = 0; v < n; ++v) {
    int32_t d = (int32_t)(off[v + 1] - off[v]);
    int64_t w = start[(size_t)(max_deg - d)]++;
    label[v] = (int32_t)w;
    orig[w] = (int32_t)v;
    rdeg[w] = d;
  }
  unsigned T = std::max(1u, std::min(32u, std::thread::hardware_concurrency()));
  if (m < (1 << 20)) T = 1;
  // relabelled row ranges of about m / T entries each (degrees descend, so
  // the prefix of rdeg is walked once)
  std::vector<int64_t> row0(T + 1, n);
  row0[0] = 0;
  {
    int64_t sum = 0;
    unsigned t = 1;
    for (int64_t w = 0; w < n && t < T; ++w) {
      while (t < T && sum >= m * (int64_t)t / (int64_t)T) row0[t++] = w;
      sum += rdeg[w];
    }
  }
  std::vector<std::vector<int64_t>> cnt(T, std::vector<int64_t>((size_t)nblk, 0));
  auto run = [&](auto fn) {
    std::vector<std::thread> th;
    for (unsigned t = 0; t < T; ++t) th.emplace_back(fn, t);
    for (auto &x : th) x.join();
  };
  run([&](unsigned t) {
    std::vector<int64_t> &c = cnt[t];
    for (int64_t w = row0[t]; w < row0[t + 1]; ++w) {
      int64_t u = orig[w];
      for (int64_t e = off[u]; e < off[u + 1]; ++e) c[(size_t)(label[nbr[e]] >> shift)]++;
    }
  });
  tile_off.assign((size_t)nblk + 1, 0);
  for (int64_t b = 0; b < nblk; ++b) {
    int64_t s = 0;
    for (unsigned t = 0; t < T; ++t) s += cnt[t][b];
    tile_off[b + 1] = tile_off[b] + s;
  }
  for (int64_t b = 0; b < nblk; ++b) {
    int64_t pos = tile_off[b];
    for (unsigned t = 0; t < T; ++t) {
      int64_t c = cnt[t][b];
      cnt[t][b] = pos;
      pos += c;
    }
  }
  esrc.resize((size_t)m);
  edst.resize((size_t)m);
  run([&](unsigned t) {
    std::vector<int64_t> &cur = cnt[t];
    for (int64_t w = row0[t]; w < row0[t + 1]; ++w) {
      int64_t u = orig[w];
      for (int64_t e = off[u]; e < off[u + 1]; ++e) {
        int32_t x = label[nbr[e]];
        int64_t p = cur[(size_t)(x >> shift)]++;
        esrc[p] = (int32_t)w;
        edst[p] = (uint16_t)((uint32_t)x & mask);
      }
    }
  });
}

byo_status tiles_ensure(byo_graph *g, int shift, hipStream_t s) {
  byo_workspace &w = g->ws;
  BYO_CHECK(shift >= 12 && shift <= 14, BYO_EINVAL, "tile size must be 2^12 .. 2^14");
  if (w.tiles && w.tiles->shift == shift) return BYO_OK;
  tiles_release(w);
  const int64_t n = g->n, m = g->m;
  BYO_CHECK(tiles_wanted(g), BYO_EINVAL, "graph too small or too sparse for the tile layout");
  BYO_CHECK(n <= ((int64_t)1 << 31) - 1, BYO_EINVAL, "graph too large for the tile layout");
  std::vector<int64_t> off((size_t)n + 1);
  std::vector<int32_t> nbr((size_t)m);
  BYO_HIP(hipMemcpyAsync(off.data(), g->off, sizeof(int64_t) * (size_t)(n + 1), hipMemcpyDeviceToHost, s));
  BYO_HIP(hipMemcpyAsync(nbr.data(), g->nbr, sizeof(int32_t) * (size_t)m, hipMemcpyDeviceToHost, s));
  BYO_HIP(hipStreamSynchronize(s));
  std::vector<int32_t> esrc, rdeg, orig, label;
  std::vector<uint16_t> edst;
  std::vector<int64_t> tile_off;
  build_tiles_host(off, nbr, n, shift, esrc, edst, tile_off, rdeg, orig, label);
  const int64_t nblk = (int64_t)tile_off.size() - 1;
  // Pack each tile into 64-entry groups. A group holds up to 64 consecutive
  // entries whose sources lie within 2^16 of the first (the group's anchor);
  // the rest of a group that cannot take the next entry is padding pointing
  // at the dummy slot 2^shift. Each entry is one word: its source's 16-bit
  // offset from the anchor and its 16-bit tile-local destination.
  const uint32_t dummy = 1u << shift;
  unsigned T = std::max(1u, std::min(32u, std::thread::hardware_concurrency()));
  if (m < (1 << 20)) T = 1;
  std::vector<int64_t> b0(T + 1, nblk);  // tile ranges of about m / T entries
  b0[0] = 0;
  for (unsigned t = 1; t < T; ++t)
    b0[t] = std::upper_bound(tile_off.begin(), tile_off.end(), m * (int64_t)t / (int64_t)T) - tile_off.begin() - 1;
  for (unsigned t = 1; t <= T; ++t) b0[t] = std::max(b0[t], b0[t - 1]);
  auto run = [&](auto fn) {
    std::vector<std::thread> th;
    for (unsigned t = 0; t < T; ++t) th.emplace_back(fn, t);
    for (auto &x : th) x.join();
  };
  // end of the group that starts at entry i of a tile ending at hi
  auto group_end = [&](int64_t i, int64_t hi) {
    const int64_t lim = std::min(hi, i + 64);
    const int32_t a = esrc[(size_t)i];
    int64_t j = i + 1;
    while (j < lim && (int64_t)esrc[(size_t)j] - a <= 65535) ++j;
    return j;
  };
  std::vector<int64_t> ngrp((size_t)nblk, 0);
  run([&](unsigned t) {
    for (int64_t b = b0[t]; b < b0[t + 1]; ++b)
      for (int64_t i = tile_off[b]; i < tile_off[b + 1]; i = group_end(i, tile_off[b + 1])) ngrp[(size_t)b]++;
  });
  std::vector<int64_t> ptile((size_t)nblk + 1, 0);
  for (int64_t b = 0; b < nblk; ++b) ptile[b + 1] = ptile[b] + 64 * ngrp[(size_t)b];
  const int64_t mp = ptile[nblk], ngroups = mp / 64;
  BYO_CHECK(ngroups < ((int64_t)1 << 31), BYO_EINVAL, "too many entry groups");
  std::vector<uint32_t> ent((size_t)mp);
  std::vector<int32_t> anchor((size_t)ngroups);
  run([&](unsigned t) {
    for (int64_t b = b0[t]; b < b0[t + 1]; ++b) {
      int64_t q = ptile[b];
      for (int64_t i = tile_off[b], hi = tile_off[b + 1]; i < hi;) {
        const int64_t j = group_end(i, hi);
        const int32_t a = esrc[(size_t)i];
        anchor[(size_t)(q / 64)] = a;
        for (int64_t r = 0; r < 64; ++r) {
          const int64_t x = i + r;
          ent[(size_t)(q + r)] = x < j ? ((uint32_t)(esrc[(size_t)x] - a) | ((uint32_t)edst[(size_t)x] << 16))
                                       : (dummy << 16);
        }
        q += 64;
        i = j;
      }
    }
  });
  std::vector<int32_t>().swap(esrc);
  std::vector<uint16_t>().swap(edst);
  // chunks: about 512 over the whole entry set, each tile cut into equal
  // pieces of whole groups
  const int64_t target = std::max<int64_t>(1 << 16, (mp + 511) / 512);
  std::vector<int64_t> cbeg;
  std::vector<int32_t> bfirst((size_t)nblk + 1), cblk;
  for (int64_t b = 0; b < nblk; ++b) {
    bfirst[b] = (int32_t)cbeg.size();
    int64_t lo = ptile[b], groups = (ptile[b + 1] - lo) / 64;
    if (groups == 0) continue;
    int64_t k = (groups * 64 + target - 1) / target;
    for (int64_t i = 0; i < k; ++i) {
      cbeg.push_back(lo + 64 * (groups * i / k));
      cblk.push_back((int32_t)b);
    }
  }
  bfirst[nblk] = (int32_t)cbeg.size();
  const int64_t nchunks = (int64_t)cbeg.size();
  cbeg.push_back(mp);

  byo_tiles *p = new byo_tiles();
  p->shift = shift;
  p->n = n;
  p->m = m;
  p->mp = mp;
  p->nblk = nblk;
  p->nchunks = nchunks;
  p->h_label = std::move(label);
  w.tiles = p;
  BYO_HIP(hipMalloc(&p->ent, sizeof(uint32_t) * (size_t)mp));
  BYO_HIP(hipMalloc(&p->anchor, sizeof(int32_t) * (size_t)ngroups));
  BYO_HIP(hipMalloc(&p->rdeg, sizeof(int32_t) * (size_t)n));
  BYO_HIP(hipMalloc(&p->orig, sizeof(int32_t) * (size_t)n));
  BYO_HIP(hipMalloc(&p->cbeg, sizeof(int64_t) * cbeg.size()));
  BYO_HIP(hipMalloc(&p->bfirst, sizeof(int32_t) * bfirst.size()));
  BYO_HIP(hipMalloc(&p->cblk, sizeof(int32_t) * (size_t)nchunks));
  BYO_HIP(hipMalloc(&p->cflag, sizeof(uint32_t) * (size_t)nchunks));
  BYO_HIP(hipMalloc(&p->rlabel, sizeof(int32_t) * (size_t)n));
  BYO_HIP(hipMemcpy(p->ent, ent.data(), sizeof(uint32_t) * (size_t)mp, hipMemcpyHostToDevice));
  BYO_HIP(hipMemcpy(p->anchor, anchor.data(), sizeof(int32_t) * (size_t)ngroups, hipMemcpyHostToDevice));
  BYO_HIP(hipMemcpy(p->rdeg, rdeg.data(), sizeof(int32_t) * (size_t)n, hipMemcpyHostToDevice));
  BYO_HIP(hipMemcpy(p->orig, orig.data(), sizeof(int32_t) * (size_t)n, hipMemcpyHostToDevice));
  BYO_HIP(hipMemcpy(p->cbeg, cbeg.data(), sizeof(int64_t) * cbeg.size(), hipMemcpyHostToDevice));
  BYO_HIP(hipMemcpy(p->bfirst, bfirst.data(), sizeof(int32_t) * bfirst.size(), hipMemcpyHostToDevice));
  BYO_HIP(hipMemcpy(p->cblk, cblk.data(), sizeof(int32_t) * (size_t)nchunks, hipMemcpyHostToDevice));
  BYO_HIP(hipMemcpy(p->rlabel, p->h_label.data(), sizeof(int32_t) * (size_t)n, hipMemcpyHostToDevice));
  // the CSR in relabelled IDs (row w = row orig[w], neighbours relabelled), for
  // push levels that run in the layout's order
  {
    std::vector<int64_t> roff((size_t)n + 1, 0);
    for (int64_t x = 0; x < n; ++x) roff[(size_t)x + 1] = roff[(size_t)x] + rdeg[(size_t)x];
    std::vector<int32_t> rnbr((size_t)m);
    const std::vector<int32_t> &lab = p->h_label;
    std::vector<int64_t> r0(T + 1, n);  // relabelled row ranges of about m / T entries
    r0[0] = 0;
    for (unsigned t = 1; t < T; ++t)
      r0[t] = std::lower_bound(roff.begin(), roff.end(), m * (int64_t)t / (int64_t)T) - roff.begin();
    for (unsigned t = 1; t <= T; ++t) r0[t] = std::max(r0[t], r0[t - 1]);
    run([&](unsigned t) {
      for (int64_t x = r0[t]; x < r0[t + 1]; ++x) {
        const int64_t u = orig[(size_t)x], o = off[(size_t)u], d = off[(size_t)u + 1] - o;
        for (int64_t i = 0; i < d; ++i) rnbr[(size_t)(roff[(size_t)x] + i)] = lab[(size_t)nbr[(size_t)(o + i)]];
      }
    });
    BYO_HIP(hipMalloc(&p->roff, sizeof(int64_t) * (size_t)(n + 1)));
    BYO_HIP(hipMalloc(&p->rnbr, sizeof(int32_t) * (size_t)m));
    BYO_HIP(hipMemcpy(p->roff, roff.data(), sizeof(int64_t) * (size_t)(n + 1), hipMemcpyHostToDevice));
    BYO_HIP(hipMemcpy(p->rnbr, rnbr.data(), sizeof(int32_t) * (size_t)m, hipMemcpyHostToDevice));
  }
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
