// Byte-coded CSR container (the compressed graphs of Section 2: difference
// encoding with byte codes, here in blocks of CZ_BLOCK neighbours so blocks
// decode independently; the format is in cz_dev.h and byo.h) and the BFS and
// min-label edgeMap levels that decode it inside the traversal kernels.
//
// Build (once per graph, on the device): blocks per vertex, their byte sizes,
// two scans to place every block, one write pass. The degree array stays with
// the graph (degree metadata is kept at framework level, Section 4.3).
//
// Levels: a lane decodes whole lists (THREAD) or only its list's first block
// while the wavefront decodes the further blocks of long lists, one block per
// lane (WAVE); the block-parallel push spreads the frontier's blocks over the
// grid (EDGE); the pull keeps the first frontier neighbour in ascending order.
#include <algorithm>
#include <cstring>
#include <vector>

#include <rocprim/device/device_scan.hpp>

#include "cz_dev.h"
#include "edgemap_dev.h"

namespace byo {

namespace {

constexpr int CZ_THREADS = 256;

unsigned cz_grid(int64_t count, int64_t cap = 65536) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>((count + CZ_THREADS - 1) / CZ_THREADS, cap));
}

// ---------------------------------------------------------------- build

__device__ __forceinline__ int32_t cz_vlen(uint32_t x) {
  return x < (1u << 7) ? 1 : x < (1u << 14) ? 2 : x < (1u << 21) ? 3 : x < (1u << 28) ? 4 : 5;
}

__device__ __forceinline__ uint32_t cz_zigzag(int32_t x) { return ((uint32_t)x << 1) ^ (uint32_t)(x >> 31); }

// nbk[v] = blocks of v's list; nbk[n] = 0
__global__ void cz_nblk_kernel(const int32_t *__restrict__ deg, int64_t n, int64_t *__restrict__ nbk) {
  for (int64_t v = (int64_t)blockIdx.x * CZ_THREADS + threadIdx.x; v <= n; v += (int64_t)gridDim.x * CZ_THREADS)
    nbk[v] = v < n ? (int64_t)((deg[v] + CZ_BLOCK - 1) / CZ_BLOCK) : 0;
}

// blkv[first block of v] = v (blkv zero elsewhere; a max-scan then names the
// vertex of every block)
__global__ void cz_mark_kernel(const int32_t *__restrict__ deg, const int64_t *__restrict__ bbase, int64_t n,
                               int32_t *__restrict__ blkv) {
  for (int64_t v = (int64_t)blockIdx.x * CZ_THREADS + threadIdx.x; v < n; v += (int64_t)gridDim.x * CZ_THREADS)
    if (deg[v] > 0) blkv[bbase[v]] = (int32_t)v;
}

// bytes of every block; sz[nblk] = 0
__global__ void cz_size_kernel(const int64_t *__restrict__ off, const int32_t *__restrict__ nbr,
                               const int32_t *__restrict__ deg, const int64_t *__restrict__ bbase,
                               const int32_t *__restrict__ blkv, int64_t nblk, int64_t *__restrict__ sz) {
  for (int64_t b = (int64_t)blockIdx.x * CZ_THREADS + threadIdx.x; b <= nblk; b += (int64_t)gridDim.x * CZ_THREADS) {
    if (b == nblk) {
      sz[b] = 0;
      continue;
    }
    const int32_t v = blkv[b];
    const int64_t j = b - bbase[v];
    const int64_t e0 = off[v] + j * CZ_BLOCK;
    const int64_t e1 = std::min<int64_t>(e0 + CZ_BLOCK, off[v] + deg[v]);
    int32_t prev = nbr[e0];
    int64_t s = cz_vlen(cz_zigzag(prev - v));
    for (int64_t e = e0 + 1; e < e1; ++e) {
      const int32_t u = nbr[e];
      s += cz_vlen((uint32_t)(u - prev));
      prev = u;
    }
    sz[b] = s;
  }
}

// bytes of every list: offset table plus blocks; reg[n] = 0
__global__ void cz_region_kernel(const int64_t *__restrict__ bbase, const int64_t *__restrict__ pos, int64_t n,
                                 int64_t *__restrict__ reg) {
  for (int64_t v = (int64_t)blockIdx.x * CZ_THREADS + threadIdx.x; v <= n; v += (int64_t)gridDim.x * CZ_THREADS) {
    if (v == n) {
      reg[v] = 0;
      continue;
    }
    const int64_t nb = bbase[v + 1] - bbase[v];
    reg[v] = (nb > 0 ? 4 * (nb - 1) : 0) + pos[bbase[v + 1]] - pos[bbase[v]];
  }
}

__device__ __forceinline__ int64_t cz_put(uint8_t *__restrict__ out, int64_t p, uint32_t x) {
  while (x >= 0x80u) {
    out[p++] = (uint8_t)(x | 0x80u);
    x >>= 7;
  }
  out[p++] = (uint8_t)x;
  return p;
}

// every block's bytes, and its entry in its list's offset table
__global__ void cz_write_kernel(const int64_t *__restrict__ off, const int32_t *__restrict__ nbr,
                                const int32_t *__restrict__ deg, const int64_t *__restrict__ bbase,
                                const int32_t *__restrict__ blkv, const int64_t *__restrict__ pos,
                                const int64_t *__restrict__ coff, int64_t nblk, uint8_t *__restrict__ out) {
  for (int64_t b = (int64_t)blockIdx.x * CZ_THREADS + threadIdx.x; b < nblk; b += (int64_t)gridDim.x * CZ_THREADS) {
    const int32_t v = blkv[b];
    const int64_t b0 = bbase[v], nb = bbase[v + 1] - b0, j = b - b0;
    const int64_t rel = 4 * (nb - 1) + pos[b] - pos[b0];  // from the list's start
    if (j > 0) {
      uint8_t *t = out + coff[v] + 4 * (j - 1);
      t[0] = (uint8_t)rel;
      t[1] = (uint8_t)(rel >> 8);
      t[2] = (uint8_t)(rel >> 16);
      t[3] = (uint8_t)(rel >> 24);
    }
    const int64_t e0 = off[v] + j * CZ_BLOCK;
    const int64_t e1 = std::min<int64_t>(e0 + CZ_BLOCK, off[v] + deg[v]);
    int64_t p = coff[v] + rel;
    int32_t prev = nbr[e0];
    p = cz_put(out, p, cz_zigzag(prev - v));
    for (int64_t e = e0 + 1; e < e1; ++e) {
      const int32_t u = nbr[e];
      p = cz_put(out, p, (uint32_t)(u - prev));
      prev = u;
    }
  }
}

__global__ void cz_decode_kernel(const int64_t *__restrict__ coff, const uint8_t *__restrict__ bytes, int32_t v,
                                 int32_t d, int32_t *__restrict__ out) {
  const int32_t nb = cz_nblocks(d);
  const int32_t j = (int32_t)(blockIdx.x * CZ_THREADS + threadIdx.x);
  if (j >= nb) return;
  int32_t i = j * CZ_BLOCK;
  cz_block_for<false>(bytes, coff[v], v, d, nb, j, [&](int32_t u) {
    out[i++] = u;
    return false;
  });
}

struct cz_tmp {
  hipStream_t s;
  std::vector<void *> v;
  explicit cz_tmp(hipStream_t st) : s(st) {}
  template <class T>
  byo_status get(T **p, size_t count) {
    *p = nullptr;
    BYO_HIP(hipMalloc((void **)p, sizeof(T) * std::max<size_t>(count, 1)));
    v.push_back(*p);
    return BYO_OK;
  }
  ~cz_tmp() {
    (void)hipStreamSynchronize(s);
    for (void *x : v) (void)hipFree(x);
  }
};

byo_status cz_build(const byo_graph *g, byo_cz *z, hipStream_t s) {
  const int64_t n = g->n;
  cz_tmp tmp(s);
  int64_t *nbk = nullptr, *bbase = nullptr, *reg = nullptr;
  BYO_TRY(tmp.get(&nbk, (size_t)n + 1));
  BYO_TRY(tmp.get(&bbase, (size_t)n + 1));
  BYO_TRY(tmp.get(&reg, (size_t)n + 1));
  BYO_HIP(hipMalloc(&z->coff, sizeof(int64_t) * (size_t)(n + 1)));
  cz_nblk_kernel<<<cz_grid(n + 1), CZ_THREADS, 0, s>>>(g->deg, n, nbk);
  BYO_HIP(hipGetLastError());
  size_t q = 0;
  BYO_HIP(rocprim::exclusive_scan(nullptr, q, nbk, bbase, (int64_t)0, (size_t)n + 1, rocprim::plus<int64_t>(), s));
  void *ts = nullptr;
  BYO_TRY(tmp.get((uint8_t **)&ts, q));
  BYO_HIP(rocprim::exclusive_scan(ts, q, nbk, bbase, (int64_t)0, (size_t)n + 1, rocprim::plus<int64_t>(), s));
  int64_t nblk = 0;
  BYO_TRY(sync_read(s, bbase + n, &nblk, sizeof(nblk)));
  int32_t *blkv = nullptr, *blkv2 = nullptr;
  int64_t *sz = nullptr, *pos = nullptr;
  BYO_TRY(tmp.get(&blkv, (size_t)nblk));
  BYO_TRY(tmp.get(&blkv2, (size_t)nblk));
  BYO_TRY(tmp.get(&sz, (size_t)nblk + 1));
  BYO_TRY(tmp.get(&pos, (size_t)nblk + 1));
  if (nblk > 0) {
    BYO_TRY(fill_i32(blkv, nblk, 0, s));
    cz_mark_kernel<<<cz_grid(n), CZ_THREADS, 0, s>>>(g->deg, bbase, n, blkv);
    BYO_HIP(hipGetLastError());
    size_t q2 = 0;
    BYO_HIP(rocprim::inclusive_scan(nullptr, q2, blkv, blkv2, (size_t)nblk, rocprim::maximum<int32_t>(), s));
    void *ts2 = nullptr;
    BYO_TRY(tmp.get((uint8_t **)&ts2, q2));
    BYO_HIP(rocprim::inclusive_scan(ts2, q2, blkv, blkv2, (size_t)nblk, rocprim::maximum<int32_t>(), s));
  }
  cz_size_kernel<<<cz_grid(nblk + 1), CZ_THREADS, 0, s>>>(g->off, g->nbr, g->deg, bbase, blkv2, nblk, sz);
  BYO_HIP(hipGetLastError());
  size_t q3 = 0;
  BYO_HIP(rocprim::exclusive_scan(nullptr, q3, sz, pos, (int64_t)0, (size_t)nblk + 1, rocprim::plus<int64_t>(), s));
  void *ts3 = nullptr;
  BYO_TRY(tmp.get((uint8_t **)&ts3, q3));
  BYO_HIP(rocprim::exclusive_scan(ts3, q3, sz, pos, (int64_t)0, (size_t)nblk + 1, rocprim::plus<int64_t>(), s));
  cz_region_kernel<<<cz_grid(n + 1), CZ_THREADS, 0, s>>>(bbase, pos, n, reg);
  BYO_HIP(hipGetLastError());
  size_t q4 = 0;
  BYO_HIP(rocprim::exclusive_scan(nullptr, q4, reg, z->coff, (int64_t)0, (size_t)n + 1, rocprim::plus<int64_t>(),
                                  s));
  void *ts4 = nullptr;
  BYO_TRY(tmp.get((uint8_t **)&ts4, q4));
  BYO_HIP(rocprim::exclusive_scan(ts4, q4, reg, z->coff, (int64_t)0, (size_t)n + 1, rocprim::plus<int64_t>(), s));
  BYO_TRY(sync_read(s, z->coff + n, &z->nbytes, sizeof(z->nbytes)));
  // the stream ends on a 4-byte boundary plus CZ_PAD readable bytes
  const int64_t alloc = ((z->nbytes + 3) / 4) * 4 + CZ_PAD;
  BYO_HIP(hipMalloc(&z->bytes, (size_t)alloc));
  BYO_HIP(hipMemsetAsync(z->bytes, 0, (size_t)alloc, s));
  cz_write_kernel<<<cz_grid(nblk), CZ_THREADS, 0, s>>>(g->off, g->nbr, g->deg, bbase, blkv2, pos, z->coff, nblk,
                                                       z->bytes);
  BYO_HIP(hipGetLastError());
  // buffers of the block-parallel push
  BYO_HIP(hipMalloc(&z->fpre, sizeof(long long) * (size_t)(n + 1)));
  z->fpart_cap = scan_partials_needed(n);
  BYO_HIP(hipMalloc(&z->fpart, sizeof(long long) * (size_t)z->fpart_cap));
  BYO_HIP(hipStreamSynchronize(s));
  return BYO_OK;
}

// ---------------------------------------------------------------- levels

LevelArgs cz_args(const byo_graph *g, const level_io &io) {
  LevelArgs a;
  std::memset(&a, 0, sizeof(a));
  a.off = g->off;
  a.nbr = g->nbr;
  a.deg = g->deg;
  a.in_ids = io.in_ids;
  a.in_bits = io.in_bits;
  a.k = io.in_count;
  a.n = g->n;
  a.words = (g->n + 63) / 64;
  a.out_ids = io.out_ids;
  a.out_bits = io.out_bits;
  a.ctr = io.ctr;
  a.ctr_clear = io.ctr_clear;
  return a;
}

struct CzArgs {
  const int64_t *__restrict__ coff;
  const uint8_t *__restrict__ bytes;
};

// Push: lane i expands frontier vertex in_ids[i]; with WAVE its list's
// blocks after the first are decoded by the whole wavefront, one per lane.
template <bool WAVE, typename F>
__global__ void __launch_bounds__(EM_BLOCK) cz_push_kernel(LevelArgs a, CzArgs z, F f) {
  __shared__ int32_t lds[EM_BLOCK / BYO_WAVE][BYO_WAVE];
  int32_t *row = lds[threadIdx.x / BYO_WAVE];
  unsigned long long degsum = 0, count = 0, maxdeg = 0;
  // uniform trip count per workgroup: every lane reaches the wavefront part
  for (int64_t base = (int64_t)blockIdx.x * EM_BLOCK; base < a.k; base += (int64_t)gridDim.x * EM_BLOCK) {
    const int64_t i = base + threadIdx.x;
    const bool valid = i < a.k;
    int32_t u = 0, d = 0, su = 0;
    int64_t r = 0;
    if (valid) {
      u = a.in_ids[i];
      d = a.deg[u];
      su = f.src_value(u);
      r = z.coff[u];
    }
    const int32_t nb = cz_nblocks(d);
    const int32_t own = WAVE ? (nb < 1 ? nb : 1) : nb;
    for (int32_t j = 0; j < own; ++j)
      cz_block_for<false>(z.bytes, r, u, d, nb, j, [&](int32_t v) {
        emit<F>(a, f.update(u, su, v, a.out_bits), v, degsum, count, maxdeg);
        return false;
      });
    if (WAVE) {
      uint64_t pm = __ballot(valid && nb > 1);
      while (pm) {
        const int l = __ffsll((long long)pm) - 1;
        pm &= pm - 1;
        const int32_t ul = read_lane_i32(u, l), dl = read_lane_i32(d, l), sul = read_lane_i32(su, l);
        const int64_t rl = (int64_t)read_lane_u64((uint64_t)r, l);
        const int64_t el = z.coff[ul + 1];
        const int32_t nbl = cz_nblocks(dl);
        for (int32_t j = 1; j < nbl; ++j) {
          const int32_t v = cz_wave_block(z.bytes, rl, el, ul, dl, nbl, j, row);
          emit<F>(a, v >= 0 && f.update(ul, sul, v, a.out_bits), v, degsum, count, maxdeg);
        }
      }
    }
  }
  finish_level<EM_BLOCK>(a, degsum, count, maxdeg);
}

// BFS pull: one wavefront per 64-vertex bitmap word; an unvisited lane
// decodes its list until the first neighbour in U. With WAVE a list of
// several blocks gets its blocks after the first from the wavefront, 64 at a
// time; the lowest block holding a member gives the parent.
template <bool WAVE>
__global__ void __launch_bounds__(EM_BLOCK) cz_bfs_pull_kernel(LevelArgs a, CzArgs z, BfsF f) {
  __shared__ int32_t lds[EM_BLOCK / BYO_WAVE][BYO_WAVE];
  int32_t *row = lds[threadIdx.x / BYO_WAVE];
  unsigned long long degsum = 0, count = 0, maxdeg = 0;
  const int64_t nwaves_total = (int64_t)gridDim.x * (EM_BLOCK / BYO_WAVE);
  int64_t w = (int64_t)xcd_block(blockIdx.x, gridDim.x) * (EM_BLOCK / BYO_WAVE) + threadIdx.x / BYO_WAVE;
  for (; w < a.words; w += nwaves_total) {
    const uint64_t vis = f.visited[w];
    if (vis == ~0ull) {
      if (lane_id() == 0) a.out_bits[w] = 0ull;
      continue;
    }
    const int32_t v = (int32_t)(w * 64 + lane_id());
    const bool cand = (w * 64 + lane_id() < a.n) && !((vis >> lane_id()) & 1ull);
    int32_t par = -1, d = 0;
    int64_t r = 0;
    if (cand) {
      d = a.deg[v];
      r = z.coff[v];
    }
    const int32_t nb = cz_nblocks(d);
    const int32_t own = WAVE ? (nb < 1 ? nb : 1) : nb;
    auto first_in_u = [&](const int32_t *u, int32_t &hit) {
      uint64_t wd[CZ_BATCH];
#pragma unroll
      for (int t = 0; t < CZ_BATCH; ++t) wd[t] = u[t] >= 0 ? a.in_bits[u[t] >> 6] : 0ull;
#pragma unroll
      for (int t = 0; t < CZ_BATCH; ++t)
        if (hit < 0 && ((wd[t] >> (u[t] & 63)) & 1ull)) hit = u[t];
      return hit >= 0;
    };
    for (int32_t j = 0; j < own; ++j)
      if (cz_block_batches<true>(z.bytes, r, v, d, nb, j, [&](const int32_t *u) { return first_in_u(u, par); }))
        break;
    bool found = par >= 0;
    if (WAVE) {
      uint64_t pm = __ballot(cand && !found && nb > 1);
      while (pm) {
        const int l = __ffsll((long long)pm) - 1;
        pm &= pm - 1;
        const int32_t vl = read_lane_i32(v, l), dl = read_lane_i32(d, l);
        const int64_t rl = (int64_t)read_lane_u64((uint64_t)r, l);
        const int64_t el = z.coff[vl + 1];
        const int32_t nbl = cz_nblocks(dl);
        bool done = false;
        for (int32_t j = 1; j < nbl && !done; ++j) {
          // block j decoded by the wavefront; its lowest member is the parent
          const int32_t u = cz_wave_block(z.bytes, rl, el, vl, dl, nbl, j, row);
          const int32_t hitu = u >= 0 && test_bit(a.in_bits, u) ? u : -1;
          const uint64_t hm = __ballot(hitu >= 0);
          if (hm) {
            const int32_t pu = read_lane_i32(hitu, __ffsll((long long)hm) - 1);
            if (lane_id() == l) {
              par = pu;
              found = true;
            }
            done = true;
          }
        }
      }
    }
    if (found) {
      f.parent[v] = par;
      f.depth[v] = f.newdepth;
      tally_degree((unsigned long long)a.deg[v], degsum, maxdeg);
    }
    const uint64_t m = __ballot(found);
    if (lane_id() == 0) {
      a.out_bits[w] = m;
      if (m) {
        f.visited[w] = vis | m;
        count += (unsigned long long)__popcll(m);
      }
    }
    if (a.out_ids && m) {
      unsigned long long b = 0;
      if (lane_id() == 0) b = atomicAdd(&a.ctr->aux0, (unsigned long long)__popcll(m));
      b = read_lane_u64(b, 0);
      if (found) a.out_ids[b + __popcll(m & lanemask_lt())] = v;
    }
  }
  finish_level<EM_BLOCK>(a, degsum, count, maxdeg);
}

// Min-label pull: every vertex takes the least label over its neighbours in U.
template <bool WAVE>
__global__ void __launch_bounds__(EM_BLOCK) cz_cc_pull_kernel(LevelArgs a, CzArgs z, CcF f) {
  unsigned long long degsum = 0, count = 0, maxdeg = 0;
  const int64_t nwaves_total = (int64_t)gridDim.x * (EM_BLOCK / BYO_WAVE);
  int64_t w = (int64_t)xcd_block(blockIdx.x, gridDim.x) * (EM_BLOCK / BYO_WAVE) + threadIdx.x / BYO_WAVE;
  for (; w < a.words; w += nwaves_total) {
    const int64_t v64 = w * 64 + lane_id();
    const bool valid = v64 < a.n;
    const int32_t v = (int32_t)v64;
    const int32_t lv = valid ? f.label[v] : 0;
    int32_t best = lv, d = 0;
    int64_t r = 0;
    if (valid) {
      d = a.deg[v];
      r = z.coff[v];
    }
    const int32_t nb = cz_nblocks(d);
    const int32_t own = WAVE ? (nb < 1 ? nb : 1) : nb;
    // least label over the batch's members of U into m
    auto take = [&](const int32_t *u, int32_t &m) {
      uint64_t wd[CZ_BATCH];
      int32_t l[CZ_BATCH];
#pragma unroll
      for (int t = 0; t < CZ_BATCH; ++t) wd[t] = u[t] >= 0 ? a.in_bits[u[t] >> 6] : 0ull;
#pragma unroll
      for (int t = 0; t < CZ_BATCH; ++t) l[t] = ((wd[t] >> (u[t] & 63)) & 1ull) ? f.label[u[t]] : 0x7fffffff;
#pragma unroll
      for (int t = 0; t < CZ_BATCH; ++t) m = l[t] < m ? l[t] : m;
      return false;
    };
    for (int32_t j = 0; j < own; ++j)
      cz_block_batches<false>(z.bytes, r, v, d, nb, j, [&](const int32_t *u) { return take(u, best); });
    if (WAVE) {
      // blocks after the first: one per lane, lane-serial
      uint64_t pm = __ballot(valid && nb > 1);
      while (pm) {
        const int l = __ffsll((long long)pm) - 1;
        pm &= pm - 1;
        const int32_t vl = read_lane_i32(v, l), dl = read_lane_i32(d, l);
        const int64_t rl = (int64_t)read_lane_u64((uint64_t)r, l);
        const int32_t nbl = cz_nblocks(dl);
        int32_t mn = 0x7fffffff;
        for (int32_t j = 1 + lane_id(); j < nbl; j += BYO_WAVE)
          cz_block_batches<false>(z.bytes, rl, vl, dl, nbl, j, [&](const int32_t *u) { return take(u, mn); });
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
          const int32_t t = __shfl_xor(mn, o);
          mn = t < mn ? t : mn;
        }
        if (lane_id() == l) best = mn < best ? mn : best;
      }
    }
    const bool changed = valid && best < lv;
    if (changed) {
      atomicMin(&f.label[v], best);
      tally_degree((unsigned long long)a.deg[v], degsum, maxdeg);
    }
    const uint64_t m = __ballot(changed);
    if (lane_id() == 0) {
      a.out_bits[w] = m;
      count += (unsigned long long)__popcll(m);
    }
  }
  finish_level<EM_BLOCK>(a, degsum, count, maxdeg);
}

// Block-parallel push (the edge-balanced push of the byte-coded lists): the
// frontier's blocks are numbered through fpre (exclusive scan of blocks per
// frontier vertex, fpre[k] = all) and every lane of the grid decodes whole
// blocks, so one long list spreads over as many lanes as it has blocks.
template <typename F>
__global__ void __launch_bounds__(EM_BLOCK) cz_push_blocks_kernel(LevelArgs a, CzArgs z,
                                                                  const long long *__restrict__ fpre, F f) {
  __shared__ int32_t lds[EM_BLOCK / BYO_WAVE][BYO_WAVE];
  int32_t *row = lds[threadIdx.x / BYO_WAVE];
  unsigned long long degsum = 0, count = 0, maxdeg = 0;
  const int64_t total = fpre[a.k];
  // Lane l of wavefront gw takes blocks gw + nw * (l + 64 t): consecutive
  // blocks (one long list) land in different wavefronts. A block of more than
  // CZ_WAVE_MIN neighbours is decoded by the whole wavefront instead.
  const int64_t nw = (int64_t)gridDim.x * (EM_BLOCK / BYO_WAVE);
  const int64_t gw = (int64_t)blockIdx.x * (EM_BLOCK / BYO_WAVE) + threadIdx.x / BYO_WAVE;
  for (int64_t t0 = 0; gw + nw * t0 < total; t0 += BYO_WAVE) {  // uniform per wavefront
    const int64_t b = gw + nw * (t0 + lane_id());
    int32_t u = 0, d = 0, su = 0, j = 0, c = 0;
    int64_t r = 0;
    if (b < total) {
      int64_t lo = 0, hi = a.k - 1;  // last i with fpre[i] <= b
      while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if (fpre[mid] <= b) lo = mid;
        else hi = mid - 1;
      }
      u = a.in_ids[lo];
      d = a.deg[u];
      su = f.src_value(u);
      r = z.coff[u];
      j = (int32_t)(b - fpre[lo]);
      c = d - j * CZ_BLOCK < CZ_BLOCK ? d - j * CZ_BLOCK : CZ_BLOCK;
    }
    const bool wide = c > CZ_WAVE_MIN;
    if (c > 0 && !wide)
      cz_block_for<false>(z.bytes, r, u, d, cz_nblocks(d), j, [&](int32_t v) {
        emit<F>(a, f.update(u, su, v, a.out_bits), v, degsum, count, maxdeg);
        return false;
      });
    uint64_t pm = __ballot(wide);
    while (pm) {
      const int l = __ffsll((long long)pm) - 1;
      pm &= pm - 1;
      const int32_t ul = read_lane_i32(u, l), dl = read_lane_i32(d, l), sul = read_lane_i32(su, l);
      const int32_t jl = read_lane_i32(j, l);
      const int64_t rl = (int64_t)read_lane_u64((uint64_t)r, l);
      const int32_t v = cz_wave_block(z.bytes, rl, z.coff[ul + 1], ul, dl, cz_nblocks(dl), jl, row);
      emit<F>(a, v >= 0 && f.update(ul, sul, v, a.out_bits), v, degsum, count, maxdeg);
    }
  }
  finish_level<EM_BLOCK>(a, degsum, count, maxdeg);
}

unsigned cz_pull_grid(int64_t words) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>((words + 3) / 4, 4096)); }

// variant: BYO_V_PUSH_THREAD, BYO_V_PUSH_WAVE or BYO_V_PUSH_EDGE (blocks);
// known_total: the frontier's degree sum (sizes the block-parallel grid)
template <typename F>
byo_status cz_launch_push(int variant, const byo_cz *cz, const LevelArgs &a, const CzArgs &z, const F &f,
                          long long known_total, hipStream_t s) {
  if (variant == BYO_V_PUSH_EDGE && a.k > 0) {
    BYO_TRY(scan_degree_units(a.deg, a.in_ids, a.k, CZ_BLOCK, cz->fpre, cz->fpart, cz->fpart_cap, s));
    // at most k + degsum / 64 blocks; about 16 per wavefront
    const int64_t bound = a.k + std::max<long long>(known_total, 0) / CZ_BLOCK;
    const int64_t per = 16 * (EM_BLOCK / BYO_WAVE);
    const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>((bound + per - 1) / per, 16384));
    cz_push_blocks_kernel<F><<<grid, EM_BLOCK, 0, s>>>(a, z, cz->fpre, f);
    BYO_HIP(hipGetLastError());
    return BYO_OK;
  }
  const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>((a.k + EM_BLOCK - 1) / EM_BLOCK, 16384));
  if (variant == BYO_V_PUSH_WAVE)
    cz_push_kernel<true, F><<<grid, EM_BLOCK, 0, s>>>(a, z, f);
  else
    cz_push_kernel<false, F><<<grid, EM_BLOCK, 0, s>>>(a, z, f);
  BYO_HIP(hipGetLastError());
  return BYO_OK;
}

}  // namespace

int cz_variant(int v) {
  // the bucketed push has no byte-coded form: its wavefront and workgroup
  // tiers become the wavefront push
  return v == BYO_V_PUSH_BUCKET ? BYO_V_PUSH_WAVE : v;
}

byo_status cz_ensure(byo_graph *g, hipStream_t s, const byo_cz **out) {
  byo_workspace &w = g->ws;
  if (!w.cz) {
    byo_cz *z = new byo_cz();
    byo_status st = cz_build(g, z, s);
    if (st != BYO_OK) {
      cz_free(z);
      return st;
    }
    w.cz = z;
  }
  if (out) *out = w.cz;
  return BYO_OK;
}

void cz_free(byo_cz *z) {
  if (!z) return;
  if (z->coff) (void)hipFree(z->coff);
  if (z->bytes) (void)hipFree(z->bytes);
  if (z->fpre) (void)hipFree(z->fpre);
  if (z->fpart) (void)hipFree(z->fpart);
  delete z;
}

byo_status cz_bfs_level(byo_graph *g, int variant, const bfs_state &st, const level_io &io, hipStream_t s,
                        long long known_total) {
  const byo_cz *cz = nullptr;
  BYO_TRY(cz_ensure(g, s, &cz));
  LevelArgs a = cz_args(g, io);
  const CzArgs z{cz->coff, cz->bytes};
  BfsF f{st.parent, st.depth, st.visited, st.level + 1};
  if (variant == BYO_V_PULL_THREAD || variant == BYO_V_PULL_WAVE) {
    BYO_CHECK(io.in_bits && io.out_bits, BYO_EINVAL, "pull needs dense input and output");
    if (a.words == 0) return BYO_OK;
    ktimer_scope kt(BYO_K_BFS_PULL, s);
    if (variant == BYO_V_PULL_THREAD)
      cz_bfs_pull_kernel<false><<<cz_pull_grid(a.words), EM_BLOCK, 0, s>>>(a, z, f);
    else
      cz_bfs_pull_kernel<true><<<cz_pull_grid(a.words), EM_BLOCK, 0, s>>>(a, z, f);
    BYO_HIP(hipGetLastError());
    return BYO_OK;
  }
  BYO_CHECK(io.in_ids || io.in_count == 0, BYO_EINVAL, "push needs a sparse input");
  ktimer_scope kt(BYO_K_BFS_PUSH, s);
  return cz_launch_push(variant, cz, a, z, f, known_total, s);
}

byo_status cz_cc_level(byo_graph *g, int variant, int32_t *label, const level_io &io, hipStream_t s,
                       long long known_total) {
  const byo_cz *cz = nullptr;
  BYO_TRY(cz_ensure(g, s, &cz));
  LevelArgs a = cz_args(g, io);
  const CzArgs z{cz->coff, cz->bytes};
  CcF f{label};
  BYO_CHECK(io.out_bits, BYO_EINVAL, "min-label edgeMap needs a dense output");
  if (variant == BYO_V_PULL_THREAD || variant == BYO_V_PULL_WAVE) {
    BYO_CHECK(io.in_bits, BYO_EINVAL, "pull needs dense input");
    if (a.words == 0) return BYO_OK;
    ktimer_scope kt(BYO_K_CC_PULL, s);
    if (variant == BYO_V_PULL_THREAD)
      cz_cc_pull_kernel<false><<<cz_pull_grid(a.words), EM_BLOCK, 0, s>>>(a, z, f);
    else
      cz_cc_pull_kernel<true><<<cz_pull_grid(a.words), EM_BLOCK, 0, s>>>(a, z, f);
    BYO_HIP(hipGetLastError());
    return BYO_OK;
  }
  BYO_CHECK(io.in_ids || io.in_count == 0, BYO_EINVAL, "push needs a sparse input");
  BYO_TRY(bitmap_clear(io.out_bits, a.words, s));
  ktimer_scope kt(BYO_K_CC_PUSH, s);
  return cz_launch_push(variant, cz, a, z, f, known_total, s);
}

}  // namespace byo

using namespace byo;

extern "C" {

byo_status byo_cz_build(byo_graph *g, void *stream) {
  BYO_CHECK(g, BYO_EINVAL, "null graph");
  return cz_ensure(g, (hipStream_t)stream, nullptr);
}

byo_status byo_cz_bytes(const byo_graph *g, int64_t *nbytes) {
  BYO_CHECK(g && nbytes, BYO_EINVAL, "null argument");
  BYO_CHECK(g->ws.cz, BYO_EINVAL, "no byte-coded lists: call byo_cz_build first");
  *nbytes = g->ws.cz->nbytes;
  return BYO_OK;
}

byo_status byo_cz_copy(const byo_graph *g, int64_t *h_off, uint8_t *h_bytes) {
  BYO_CHECK(g && h_off && (h_bytes || !g->ws.cz || g->ws.cz->nbytes == 0), BYO_EINVAL, "null argument");
  BYO_CHECK(g->ws.cz, BYO_EINVAL, "no byte-coded lists: call byo_cz_build first");
  const byo_cz *z = g->ws.cz;
  BYO_HIP(hipMemcpy(h_off, z->coff, sizeof(int64_t) * (size_t)(g->n + 1), hipMemcpyDeviceToHost));
  if (z->nbytes > 0) BYO_HIP(hipMemcpy(h_bytes, z->bytes, (size_t)z->nbytes, hipMemcpyDeviceToHost));
  return BYO_OK;
}

byo_status byo_cz_decode(byo_graph *g, int64_t v, int32_t *d_out, void *stream) {
  BYO_CHECK(g && d_out, BYO_EINVAL, "null argument");
  BYO_CHECK(v >= 0 && v < g->n, BYO_EINVAL, "vertex out of range");
  hipStream_t s = (hipStream_t)stream;
  const byo_cz *cz = nullptr;
  BYO_TRY(cz_ensure(g, s, &cz));
  int32_t d = 0;
  BYO_TRY(sync_read(s, g->deg + v, &d, sizeof(d)));
  if (d == 0) return BYO_OK;
  cz_decode_kernel<<<cz_grid(cz_nblocks(d)), CZ_THREADS, 0, s>>>(cz->coff, cz->bytes, (int32_t)v, d, d_out);
  BYO_HIP(hipGetLastError());
  return BYO_OK;
}

}  // extern "C"
