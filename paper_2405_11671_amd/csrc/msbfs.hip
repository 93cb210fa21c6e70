// Multi-source BFS: up to 256 breadth-first searches in one traversal, one
// bit per source in W <= 4 u64 words per vertex (the bit-parallel scheme of
// Then et al., "The More the Merrier: Efficient Multi-Source Graph
// Traversal", VLDB 2014). Each level is one edgeMap whose frontier value is a
// source mask instead of a single bit: push ORs the frontier mask of u into
// v, pull ORs the masks of v's neighbours and stops early once v has seen
// every source (the early-exit map of the paper's Section 4.2).
//
// Depths are written vertex-major (depth[v * k + j]) so the bytes a vertex
// gains in one level share its 256-byte row.
#include <algorithm>
#include <cstring>
#include <vector>

#include "internal.h"

namespace byo {

constexpr int MS_BLOCK = 256;
constexpr int MS_ILP = 4;
// the run's tallies, (vertex, source) pairs reached at word 0 and edges over
// them at MS_TALLY_EDGES, on separate lines (every workgroup adds into both)
constexpr int MS_TALLY_EDGES = BYO_LINE_U64;
constexpr int MS_TALLY_WORDS = 2 * BYO_LINE_U64;

// Depth bytes of the sources newly seen by v (bits of nb; sv = the sources
// seen before). When rows are 16-byte aligned (k a multiple of 16) each group
// of 16 sources with a new bit is one 16-byte store: built from 255 (the
// fill) when no source of the group was seen before, else from the group's
// current bytes, all of whose loads are issued before the first is used.
// Otherwise one byte store per new source.
template <int W>
__device__ __forceinline__ void write_depths(uint8_t *__restrict__ depth, int64_t v, int32_t k, const uint64_t *nb,
                                             const uint64_t *sv, uint8_t d) {
  uint8_t *row = depth + v * k;
  if ((k & 15) == 0 && ((uintptr_t)depth & 15) == 0) {
    constexpr int G = 4 * W;
    const uint32_t splat = 0x01010101u * d;
    uint4 *p = (uint4 *)row;
    uint4 val[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
      uint32_t bits = (uint32_t)(nb[g >> 2] >> (16 * (g & 3))) & 0xFFFFu;
      uint32_t old = (uint32_t)(sv[g >> 2] >> (16 * (g & 3))) & 0xFFFFu;
      if (bits && bits != 0xFFFFu && old) val[g] = p[g];
    }
#pragma unroll
    for (int g = 0; g < G; ++g) {
      uint32_t bits = (uint32_t)(nb[g >> 2] >> (16 * (g & 3))) & 0xFFFFu;
      uint32_t old = (uint32_t)(sv[g >> 2] >> (16 * (g & 3))) & 0xFFFFu;
      if (!bits) continue;
      uint4 x;
      if (bits == 0xFFFFu) {
        x.x = x.y = x.z = x.w = splat;
      } else {
        if (old) {
          x = val[g];
        } else {
          x.x = x.y = x.z = x.w = 0xFFFFFFFFu;
        }
        uint32_t c[4] = {x.x, x.y, x.z, x.w};
        while (bits) {
          int j = __ffs(bits) - 1;
          bits &= bits - 1;
          uint32_t sh = 8u * (uint32_t)(j & 3);
          c[j >> 2] = (c[j >> 2] & ~(0xFFu << sh)) | ((uint32_t)d << sh);
        }
        x.x = c[0];
        x.y = c[1];
        x.z = c[2];
        x.w = c[3];
      }
      p[g] = x;
    }
    return;
  }
#pragma unroll
  for (int w = 0; w < W; ++w) {
    uint64_t x = nb[w];
    while (x) {
      int j = __ffsll((long long)x) - 1;
      row[w * 64 + j] = d;
      x &= x - 1;
    }
  }
}

__device__ __forceinline__ uint64_t shfl_u64(uint64_t v, int src) {
  uint32_t lo = (uint32_t)__shfl((int)(uint32_t)v, src);
  uint32_t hi = (uint32_t)__shfl((int)(uint32_t)(v >> 32), src);
  return ((uint64_t)hi << 32) | lo;
}

// Wavefront-cooperative form of write_depths, called by every lane of the
// wavefront with its own vertex's row index, new bits nb (all zero when the
// vertex gained nothing) and previously seen bits sv. Rows are written four at
// a time, sixteen lanes per row and one 16-source group per lane, so a store
// instruction covers four 256-byte rows instead of 64 scattered 16-byte
// pieces. Needs k a multiple of 16 (k <= 256) and a 16-byte aligned array.
template <int W>
__device__ void write_depths_wave(uint8_t *__restrict__ depth, int32_t k, int64_t row, const uint64_t *nb,
                                  const uint64_t *sv, uint8_t d) {
  bool mine = false;
#pragma unroll
  for (int w = 0; w < W; ++w) mine |= nb[w] != 0;
  const uint64_t anym = __ballot(mine);
  if (!anym) return;
  const int lane = lane_id(), g = lane & 15, q = lane >> 4;
  const uint32_t splat = 0x01010101u * d;
  for (int r = 0; r < 16; ++r) {
    if (!((anym >> (4 * r)) & 0xFull)) continue;  // none of these four rows gained anything
    const int sl = 4 * r + q;
    uint64_t nw = 0, so = 0;
#pragma unroll
    for (int w = 0; w < W; ++w) {
      const uint64_t a = shfl_u64(nb[w], sl), b = shfl_u64(sv[w], sl);
      if ((g >> 2) == w) {
        nw = a;
        so = b;
      }
    }
    const int64_t rw = (int64_t)shfl_u64((uint64_t)row, sl);
    uint32_t bits = (uint32_t)(nw >> (16 * (g & 3))) & 0xFFFFu;
    if (!bits || 16 * g >= k) continue;
    const uint32_t old = (uint32_t)(so >> (16 * (g & 3))) & 0xFFFFu;
    uint4 *p = (uint4 *)(depth + rw * k + 16 * g);
    uint4 x;
    if (bits == 0xFFFFu) {
      x.x = x.y = x.z = x.w = splat;
    } else {
      if (old) {
        x = *p;
      } else {
        x.x = x.y = x.z = x.w = 0xFFFFFFFFu;
      }
      uint32_t c[4] = {x.x, x.y, x.z, x.w};
      while (bits) {
        int j = __ffs(bits) - 1;
        bits &= bits - 1;
        uint32_t sh = 8u * (uint32_t)(j & 3);
        c[j >> 2] = (c[j >> 2] & ~(0xFFu << sh)) | ((uint32_t)d << sh);
      }
      x.x = c[0];
      x.y = c[1];
      x.z = c[2];
      x.w = c[3];
    }
    *p = x;
  }
}

// Dense level: every vertex that has not seen all sources ORs its
// neighbours' frontier masks (serial with ILP for short lists, wavefront-
// parallel beyond t_wave), stopping once its mask is full.
template <int W>
__global__ void __launch_bounds__(MS_BLOCK) ms_pull_kernel(const int64_t *__restrict__ off, const int32_t *__restrict__ nbr,
                                                           const int32_t *__restrict__ deg, int64_t n,
                                                           const uint64_t *__restrict__ front, uint64_t *__restrict__ seen,
                                                           uint64_t *__restrict__ next, uint8_t *__restrict__ depth,
                                                           int32_t k, uint8_t newdepth, uint64_t *__restrict__ active_bits,
                                                           byo_counters *__restrict__ ctr, int32_t t_wave) {
  uint64_t full[W];
#pragma unroll
  for (int w = 0; w < W; ++w) {
    int bits = k - 64 * w;
    full[w] = bits >= 64 ? ~0ull : (bits <= 0 ? 0ull : (~0ull >> (64 - bits)));
  }
  unsigned long long degsum = 0, count = 0;
  const int64_t stride = (int64_t)gridDim.x * MS_BLOCK;
  for (int64_t base = (int64_t)xcd_block(blockIdx.x, gridDim.x) * MS_BLOCK; base < n; base += stride) {
    int64_t v = base + threadIdx.x;
    bool valid = v < n;
    uint64_t sv[W], acc[W];
    bool need = false;
    int64_t beg = 0, end = 0;
#pragma unroll
    for (int w = 0; w < W; ++w) {
      sv[w] = valid ? seen[v * W + w] : full[w];
      acc[w] = 0;
      need |= sv[w] != full[w];
    }
    if (need) {
      beg = off[v];
      end = off[v + 1];
      int64_t lim = end - beg > t_wave ? beg + t_wave : end;
      for (int64_t e = beg; e < lim; e += MS_ILP) {
        int32_t u[MS_ILP];
#pragma unroll
        for (int j = 0; j < MS_ILP; ++j) u[j] = (e + j < lim) ? nbr[e + j] : -1;
#pragma unroll
        for (int j = 0; j < MS_ILP; ++j)
#pragma unroll
          for (int w = 0; w < W; ++w) acc[w] |= u[j] >= 0 ? front[(int64_t)u[j] * W + w] : 0ull;
        bool done = true;
#pragma unroll
        for (int w = 0; w < W; ++w) done &= (acc[w] | sv[w]) == full[w];
        if (done) {
          end = lim;  // no wavefront pass needed
          break;
        }
      }
    }
    // wavefront pass over the rest of long lists
    uint64_t pm = __ballot(need && end - beg > t_wave);
    while (pm) {
      int l = __ffsll((long long)pm) - 1;
      pm &= pm - 1;
      int64_t lo = (int64_t)read_lane_u64((uint64_t)(beg + t_wave), l);
      int64_t hi = (int64_t)read_lane_u64((uint64_t)end, l);
      uint64_t have[W], got[W];
#pragma unroll
      for (int w = 0; w < W; ++w) {
        have[w] = read_lane_u64(sv[w] | acc[w], l);
        got[w] = 0;
      }
      for (int64_t b2 = lo; b2 < hi; b2 += BYO_WAVE) {
        int64_t e = b2 + lane_id();
        int32_t u = e < hi ? nbr[e] : -1;
#pragma unroll
        for (int w = 0; w < W; ++w) {
          uint64_t x = u >= 0 ? front[(int64_t)u * W + w] : 0ull;
#pragma unroll
          for (int o = 32; o > 0; o >>= 1) x |= __shfl_xor(x, o);
          got[w] |= x;
        }
        bool done = true;
#pragma unroll
        for (int w = 0; w < W; ++w) done &= (got[w] | have[w]) == full[w];
        if (done) break;
      }
      if (lane_id() == l) {
#pragma unroll
        for (int w = 0; w < W; ++w) acc[w] |= got[w];
      }
    }
    bool any = false;
    uint64_t nb[W];
#pragma unroll
    for (int w = 0; w < W; ++w) {
      nb[w] = acc[w] & ~sv[w];
      any |= nb[w] != 0;
    }
    if (any) {
#pragma unroll
      for (int w = 0; w < W; ++w) {
        next[v * W + w] = nb[w];
        seen[v * W + w] = sv[w] | nb[w];
      }
      write_depths<W>(depth, v, k, nb, sv, newdepth);
      degsum += (unsigned long long)deg[v];
    }
    // 64 consecutive vertices per wavefront: one bitmap word, no atomics
    uint64_t am = __ballot(any);
    if (lane_id() == 0 && v < n) {
      active_bits[v >> 6] = am;
      count += (unsigned long long)__popcll(am);
    }
  }
  unsigned long long t = block_sum<unsigned long long, MS_BLOCK>(degsum);
  unsigned long long c = block_sum<unsigned long long, MS_BLOCK>(count);
  if (threadIdx.x == 0) {
    if (t) atomicAdd(&ctr->degsum, t);
    if (c) atomicAdd(&ctr->count, c);
  }
}

// Zero the frontier words of the vertices whose bit is set in `bits`.
template <int W>
__global__ void ms_clear_bits_kernel(const uint64_t *__restrict__ bits, int64_t n, uint64_t *__restrict__ front) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    if ((bits[v >> 6] >> (v & 63)) & 1ull) {
#pragma unroll
      for (int w = 0; w < W; ++w) front[v * W + w] = 0ull;
    }
  }
}

// After a push level: fold visit[v] into seen/next for every touched v.
template <int W>
__global__ void __launch_bounds__(MS_BLOCK) ms_finish_kernel(const int32_t *__restrict__ touched,
                                                             const byo_counters *__restrict__ tctr,
                                                             const int32_t *__restrict__ deg, uint64_t *__restrict__ visit,
                                                             uint64_t *__restrict__ seen, uint64_t *__restrict__ next,
                                                             uint64_t *__restrict__ touched_bits,
                                                             uint8_t *__restrict__ depth, int32_t k, uint8_t newdepth,
                                                             int32_t *__restrict__ active, byo_counters *__restrict__ ctr) {
  int64_t cnt = (int64_t)tctr->count;
  unsigned long long degsum = 0;
  for (int64_t base = (int64_t)blockIdx.x * MS_BLOCK; base < cnt; base += (int64_t)gridDim.x * MS_BLOCK) {
    int64_t i = base + threadIdx.x;
    bool any = false;
    int32_t v = 0;
    if (i < cnt) {
      v = touched[i];
      uint64_t nb[W], sv[W];
#pragma unroll
      for (int w = 0; w < W; ++w) {
        uint64_t x = visit[(int64_t)v * W + w];
        visit[(int64_t)v * W + w] = 0ull;
        sv[w] = seen[(int64_t)v * W + w];
        nb[w] = x & ~sv[w];
        any |= nb[w] != 0;
        if (nb[w]) {
          seen[(int64_t)v * W + w] = sv[w] | nb[w];
          next[(int64_t)v * W + w] = nb[w];
        }
      }
      if (any) {
        write_depths<W>(depth, v, k, nb, sv, newdepth);
        degsum += (unsigned long long)deg[v];
      }
      atomicAnd((unsigned long long *)&touched_bits[v >> 6], ~(1ull << (v & 63)));
    }
    wave_append(any, v, active, &ctr->count);
  }
  unsigned long long t = block_sum<unsigned long long, MS_BLOCK>(degsum);
  if (threadIdx.x == 0 && t) atomicAdd(&ctr->degsum, t);
}

// Zero the frontier words of the vertices in `list` (keeps the spare buffer all-zero).
template <int W>
__global__ void ms_clear_kernel(const int32_t *__restrict__ list, int64_t cnt, uint64_t *__restrict__ front) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < cnt) {
    int32_t u = list[i];
#pragma unroll
    for (int w = 0; w < W; ++w) front[(int64_t)u * W + w] = 0ull;
  }
}

__global__ void ms_init_kernel(const int32_t *__restrict__ srcs, int32_t k, int32_t W, uint64_t *seen, uint64_t *front,
                               uint8_t *depth) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < k) {
    int64_t s = srcs[j];
    unsigned long long bit = 1ull << (j & 63);
    atomicOr((unsigned long long *)&seen[s * W + (j >> 6)], bit);
    atomicOr((unsigned long long *)&front[s * W + (j >> 6)], bit);
    depth[s * k + j] = 0;
  }
}

// reached = sum of popcount(seen[v]); edges = sum of deg(v) * popcount(seen[v]).
__global__ void __launch_bounds__(MS_BLOCK) ms_tally_kernel(const uint64_t *__restrict__ seen, int32_t W,
                                                            const int32_t *__restrict__ deg, int64_t n,
                                                            unsigned long long *__restrict__ out) {
  unsigned long long r = 0, e = 0;
  for (int64_t v = (int64_t)blockIdx.x * MS_BLOCK + threadIdx.x; v < n; v += (int64_t)gridDim.x * MS_BLOCK) {
    unsigned long long c = 0;
    for (int w = 0; w < W; ++w) c += __popcll(seen[v * W + w]);
    r += c;
    e += c * (unsigned long long)deg[v];
  }
  unsigned long long tr = block_sum<unsigned long long, MS_BLOCK>(r);
  unsigned long long te = block_sum<unsigned long long, MS_BLOCK>(e);
  if (threadIdx.x == 0) {
    atomicAdd(&out[0], tr);
    atomicAdd(&out[MS_TALLY_EDGES], te);
  }
}

__global__ void u8_fill_kernel(uint8_t *p, int64_t count, uint8_t value) {
  int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 16;
  int64_t stride = (int64_t)gridDim.x * blockDim.x * 16;
  uint4 val;
  uint32_t x = value * 0x01010101u;
  val.x = val.y = val.z = val.w = x;
  for (; i < count; i += stride) {
    if (i + 16 <= count && ((uintptr_t)(p + i) & 15) == 0) {
      *(uint4 *)(p + i) = val;
    } else {
      for (int64_t j = i; j < i + 16 && j < count; ++j) p[j] = value;
    }
  }
}

// ---------------------------------------------------------------- tiled levels
//
// With the degree-ordered tile layout (tiles.hip) every level is one pass
// over the entries in relabelled vertex order. A workgroup takes a chunk of a
// destination tile of 2^12 vertices, holds their W-word masks in LDS (128 KiB
// at W = 4) and, for every entry whose source is in the frontier and whose
// destination has not seen every source, ORs the source's frontier mask into
// the destination's (LDS atomics; OR is order-free). The apply pass ORs a
// vertex's chunk results, keeps the bits not seen before, and writes seen,
// the next frontier, the frontier and "full" bitmaps, and the depths (in the
// caller's vertex order).
constexpr int MT_THREADS = 1024;
constexpr int MT_ILP = 8;
constexpr int MT_SHIFT = 12;

// W-word mask of vertex u, in 16-byte loads where the words allow.
template <int W>
__device__ __forceinline__ void load_mask(const uint64_t *__restrict__ m, int64_t u, uint64_t *x) {
  const uint64_t *p = m + u * W;
  if constexpr (W == 4) {
    ulonglong2 a = *(const ulonglong2 *)p, b = *(const ulonglong2 *)(p + 2);
    x[0] = a.x;
    x[1] = a.y;
    x[2] = b.x;
    x[3] = b.y;
  } else if constexpr (W == 2) {
    ulonglong2 a = *(const ulonglong2 *)p;
    x[0] = a.x;
    x[1] = a.y;
  } else {
#pragma unroll
    for (int w = 0; w < W; ++w) x[w] = p[w];
  }
}

// Where the level's results land: seen and the next frontier masks, the next
// active and the "full" bitmaps, the depths (null while they come from the
// level history), the counters.
struct ms_fin_args {
  uint64_t *seen, *front_next, *abits_next, *fbits;
  const int32_t *rdeg, *orig;
  uint8_t *depth;
  int32_t k;
  uint8_t newdepth;
  int64_t n;
};

// per-workgroup level tallies: next frontier size and degree sum, (vertex,
// source) pairs reached and edges over them
struct ms_tallies {
  unsigned long long degsum = 0, count = 0, pairs = 0, edges = 0;
};

// One level's end for 64 consecutive vertices, one per lane of the wavefront
// (v of lane 0 a multiple of 64): a = the sources that reached v this level
// (already ORed over the chunks), now_full = v had seen every source before
// (lanes past n pass true). Keeps the bits not seen before, writes seen, the
// next frontier, the depths, and the words of the next active and the full
// bitmaps (when `owned`: the wavefront's word belongs to the caller).
template <int W>
__device__ __forceinline__ void ms_finish_word(const ms_fin_args &f, int64_t v, bool now_full, const uint64_t *a,
                                               const uint64_t *full, bool vec_depth,
                                               bool owned, ms_tallies &tl) {
  bool any = false;
  uint64_t nb[W], sv[W];
#pragma unroll
  for (int w = 0; w < W; ++w) nb[w] = sv[w] = 0ull;
  int64_t row = 0;
  if (v < f.n && !now_full) {
    bool got = false;
#pragma unroll
    for (int w = 0; w < W; ++w) got |= a[w] != 0;
    if (got) {  // else nothing reached v and its full bit stays clear
      now_full = true;
#pragma unroll
      for (int w = 0; w < W; ++w) {
        sv[w] = f.seen[v * W + w];
        nb[w] = a[w] & ~sv[w];
        any |= nb[w] != 0;
        now_full &= (sv[w] | nb[w]) == full[w];
      }
    }
    if (any) {
#pragma unroll
      for (int w = 0; w < W; ++w) {
        f.seen[v * W + w] = sv[w] | nb[w];
        f.front_next[v * W + w] = nb[w];
      }
      row = f.orig[v];
      tl.degsum += (unsigned long long)f.rdeg[v];
      unsigned long long pc = 0;
#pragma unroll
      for (int w = 0; w < W; ++w) pc += (unsigned long long)__popcll(nb[w]);
      tl.pairs += pc;
      tl.edges += pc * (unsigned long long)f.rdeg[v];
    } else {
#pragma unroll
      for (int w = 0; w < W; ++w) nb[w] = 0ull;
    }
  }
  if (!f.depth) {
    // depths of this level come from the level history later
  } else if (vec_depth) {
    write_depths_wave<W>(f.depth, f.k, row, nb, sv, f.newdepth);  // every lane of the wavefront
  } else if (any) {
    write_depths<W>(f.depth, row, f.k, nb, sv, f.newdepth);
  }
  const uint64_t am = __ballot(any);
  const uint64_t fm = __ballot(now_full);  // vertices past n count as full
  if (lane_id() == 0 && v < f.n && owned) {
    f.abits_next[v >> 6] = am;
    f.fbits[v >> 6] = fm;
    tl.count += (unsigned long long)__popcll(am);
  }
}

template <int W>
__device__ __forceinline__ void ms_full_words(int32_t k, uint64_t *full) {
#pragma unroll
  for (int w = 0; w < W; ++w) {
    const int bits = k - 64 * w;
    full[w] = bits >= 64 ? ~0ull : (bits <= 0 ? 0ull : (~0ull >> (64 - bits)));
  }
}

// the workgroup's tallies into the level counters (one atomic each)
template <int BLOCK>
__device__ __forceinline__ void ms_add_tallies(const ms_tallies &tl, byo_counters *ctr,
                                               unsigned long long *tally) {
  const unsigned long long ts = block_sum<unsigned long long, BLOCK>(tl.degsum);
  const unsigned long long tc = block_sum<unsigned long long, BLOCK>(tl.count);
  const unsigned long long tp = block_sum<unsigned long long, BLOCK>(tl.pairs);
  const unsigned long long te = block_sum<unsigned long long, BLOCK>(tl.edges);
  if (threadIdx.x == 0) {
    if (ts) atomicAdd(&ctr->degsum, ts);
    if (tc) atomicAdd(&ctr->count, tc);
    if (tp) atomicAdd(&tally[0], tp);
    if (te) atomicAdd(&tally[MS_TALLY_EDGES], te);
  }
}

// A tile cut into one chunk is finished by that chunk's workgroup (its
// accumulators are the tile's whole result); the chunk results of a tile cut
// into several go to `partial` for the apply pass.
// an entry word read once per pass: loaded non-temporally
__device__ __forceinline__ void tile_entry_nt(const uint32_t *__restrict__ ent, const int32_t *__restrict__ anchor,
                                              int64_t e, int32_t &src, uint32_t &dst) {
  const uint32_t x = __builtin_nontemporal_load(&ent[e]);
  const int32_t g = __builtin_amdgcn_readfirstlane((int32_t)(e >> 6));
  dst = x >> 16;
  src = anchor[g] + (int32_t)(x & 0xffffu);
}

template <int W>
__global__ void __launch_bounds__(MT_THREADS) ms_tile_kernel(const uint32_t *__restrict__ ent,
                                                             const int32_t *__restrict__ anchor,
                                                             const int64_t *__restrict__ cbeg,
                                                             const int32_t *__restrict__ cblk,
                                                             const uint64_t *__restrict__ front,
                                                             const uint64_t *__restrict__ abits,
                                                             int64_t words, const int32_t *__restrict__ bfirst,
                                                             ms_fin_args f, byo_counters *__restrict__ ctr,
                                                             unsigned long long *__restrict__ tally,
                                                             uint64_t *__restrict__ partial,
                                                             uint32_t *__restrict__ cflag) {
  constexpr int B = 1 << MT_SHIFT;
  __shared__ uint64_t acc[B * W];
  __shared__ uint64_t need[B / 64 + 1];  // word B / 64 (padding entries) stays 0
  __shared__ int s_any, s_need;
  const uint64_t *__restrict__ fbits = f.fbits;
  const int t = threadIdx.x;
  const int64_t c = blockIdx.x;
  const int64_t tile = cblk[c];
  const bool single = bfirst[tile + 1] - bfirst[tile] == 1;
  if (t == 0) {
    s_any = 0;
    s_need = 0;
  }
  __syncthreads();
  if (t <= B / 64) {
    int64_t wd = (tile << (MT_SHIFT - 6)) + t;
    const uint64_t x = (t < B / 64 && wd < words) ? ~fbits[wd] : 0ull;
    need[t] = x;
    if (x) s_need = 1;  // every writer stores the same value
  }
  __syncthreads();
  // a tile whose vertices have all seen every source has nothing to gain:
  // the workgroup leaves without streaming its entries
  if (!s_need) {
    if (!single) {
      if (t == 0) cflag[c] = 0u;
    } else if (t < B / 64) {
      const int64_t wd = (tile << (MT_SHIFT - 6)) + t;
      if (wd < words) f.abits_next[wd] = 0ull;
    }
    return;
  }
  for (int i = t; i < B * W; i += MT_THREADS) acc[i] = 0ull;
  __syncthreads();
  const int64_t beg = cbeg[c], end = cbeg[c + 1];
  int mine = 0;
  // the next iteration's entries are loaded while this iteration's bitmap and
  // mask gathers are in flight
  int32_t un[MT_ILP];
  uint32_t dn[MT_ILP];
#pragma unroll
  for (int j = 0; j < MT_ILP; ++j) {
    int64_t i = beg + t + (int64_t)j * MT_THREADS;
    i = i < end ? i : beg;  // a chunk is never empty
    tile_entry_nt(ent, anchor, i, un[j], dn[j]);
  }
  for (int64_t e0 = beg + t; e0 < end; e0 += (int64_t)MT_THREADS * MT_ILP) {
    int32_t u[MT_ILP];
    uint32_t d[MT_ILP];
    uint64_t ab[MT_ILP];
#pragma unroll
    for (int j = 0; j < MT_ILP; ++j) {
      u[j] = un[j];
      d[j] = dn[j];
    }
#pragma unroll
    for (int j = 0; j < MT_ILP; ++j) ab[j] = abits[u[j] >> 6];
    const int64_t e1 = e0 + (int64_t)MT_THREADS * MT_ILP;
#pragma unroll
    for (int j = 0; j < MT_ILP; ++j) {
      int64_t i = e1 + (int64_t)j * MT_THREADS;
      i = i < end ? i : beg;
      tile_entry_nt(ent, anchor, i, un[j], dn[j]);
    }
    bool ok[MT_ILP];
    bool some = false;
#pragma unroll
    for (int j = 0; j < MT_ILP; ++j) {
      ok[j] = e0 + (int64_t)j * MT_THREADS < end && ((ab[j] >> (u[j] & 63)) & 1ull) &&
              ((need[d[j] >> 6] >> (d[j] & 63)) & 1ull);
      some |= ok[j];
    }
    // sparse levels: most wavefronts have no active entry and load no masks;
    // otherwise inactive lanes read vertex 0's mask (one shared line)
    if (__any(some)) {
      uint64_t x[MT_ILP][W];
#pragma unroll
      for (int j = 0; j < MT_ILP; ++j) load_mask<W>(front, ok[j] ? (int64_t)u[j] : 0, x[j]);
#pragma unroll
      for (int j = 0; j < MT_ILP; ++j)
#pragma unroll
        for (int w = 0; w < W; ++w)
          if (ok[j] && x[j][w]) {
            atomicOr((unsigned long long *)&acc[d[j] * W + w], (unsigned long long)x[j][w]);
            mine = 1;
          }
    }
  }
  if (mine) s_any = 1;  // every writer stores the same value
  __syncthreads();
  const int any = s_any;
  if (!single) {
    if (any) {
      uint64_t *out = partial + ((c * B) * W);
      for (int i = t; i < B * W; i += MT_THREADS) out[i] = acc[i];
    }
    if (t == 0) cflag[c] = any ? 1u : 0u;
    return;
  }
  if (!any) {  // nothing reached the tile: no next-frontier vertex, the full bits stand
    if (t < B / 64) {
      const int64_t wd = (tile << (MT_SHIFT - 6)) + t;
      if (wd < words) f.abits_next[wd] = 0ull;
    }
    return;
  }
  uint64_t full[W];
  ms_full_words<W>(f.k, full);
  const bool vec_depth = (f.k & 15) == 0 && ((uintptr_t)f.depth & 15) == 0;
  ms_tallies tl;
  for (int l = t; l < B; l += MT_THREADS) {
    const int64_t v = (tile << MT_SHIFT) + l;
    const bool now_full = v >= f.n || !((need[l >> 6] >> (l & 63)) & 1ull);
    uint64_t a[W];
#pragma unroll
    for (int w = 0; w < W; ++w) a[w] = acc[l * W + w];
    ms_finish_word<W>(f, v, now_full, a, full, vec_depth, true, tl);
  }
  ms_add_tallies<MT_THREADS>(tl, ctr, tally);
}

// The apply pass: the vertices of the tiles cut into several chunks, in
// pieces of the tile layout's apply plan (a word: first vertex, bit 0 set for
// a 64-vertex piece of a many-chunk tile, else 1024 vertices), ORing each
// vertex's chunk results; then, in the workgroups past the plan, the
// next-active words of the trailing tiles without entries (cleared: nothing
// reaches a vertex without neighbours).
template <int W>
__global__ void __launch_bounds__(MS_BLOCK) ms_tile_apply_kernel(
    const uint64_t *__restrict__ partial, const uint32_t *__restrict__ cflag, const int32_t *__restrict__ bfirst,
    const int32_t *__restrict__ plan, int64_t nplan, int64_t wtail, ms_fin_args f, byo_counters *__restrict__ ctr,
    unsigned long long *__restrict__ tally) {
  constexpr int B = 1 << MT_SHIFT;
  if ((int64_t)blockIdx.x >= nplan) {
    const int64_t words = (f.n + 63) / 64;
    for (int64_t wd = (wtail >> 6) + ((int64_t)blockIdx.x - nplan) * MS_BLOCK + threadIdx.x; wd < words;
         wd += ((int64_t)gridDim.x - nplan) * MS_BLOCK)
      f.abits_next[wd] = 0ull;
    return;
  }
  uint64_t full[W];
  ms_full_words<W>(f.k, full);
  const bool vec_depth = (f.k & 15) == 0 && ((uintptr_t)f.depth & 15) == 0;
  const int32_t piece = plan[blockIdx.x];
  const int64_t v0 = piece & ~1;
  const int64_t v1 = v0 + ((piece & 1) ? 64 : 1024);
  ms_tallies tl;
  for (int64_t base = v0; base < v1; base += MS_BLOCK) {
    const int64_t v = base + threadIdx.x;
    const bool valid = v < v1 && v < f.n;
    bool now_full = true;
    uint64_t a[W];
#pragma unroll
    for (int w = 0; w < W; ++w) a[w] = 0ull;
    if (valid) {
      now_full = (f.fbits[v >> 6] >> (v & 63)) & 1ull;
      if (!now_full) {
        const int64_t b = v >> MT_SHIFT, l = v & (B - 1);
        // hub tiles have many chunks: eight chunk results in flight; results of
        // chunks that produced nothing this level are stale and masked out
        const int32_t c1 = bfirst[b + 1];
        const uint64_t *pl = partial + (int64_t)l * W;
        int32_t c = bfirst[b];
        for (; c + 8 <= c1; c += 8) {
          uint32_t fl[8];
#pragma unroll
          for (int j = 0; j < 8; ++j) fl[j] = cflag[c + j];
          if (!(fl[0] | fl[1] | fl[2] | fl[3] | fl[4] | fl[5] | fl[6] | fl[7])) continue;
          uint64_t x[8][W];
#pragma unroll
          for (int j = 0; j < 8; ++j)
#pragma unroll
            for (int w = 0; w < W; ++w) x[j][w] = pl[((int64_t)(c + j) * B) * W + w];
#pragma unroll
          for (int j = 0; j < 8; ++j)
#pragma unroll
            for (int w = 0; w < W; ++w) a[w] |= fl[j] ? x[j][w] : 0ull;
        }
        for (; c < c1; ++c) {
          if (!cflag[c]) continue;
#pragma unroll
          for (int w = 0; w < W; ++w) a[w] |= pl[((int64_t)c * B) * W + w];
        }
      }
    }
    // every lane calls it; a wavefront past a 64-vertex piece owns no word
    ms_finish_word<W>(f, v, now_full, a, full, vec_depth, v - (int64_t)lane_id() < v1, tl);
  }
  ms_add_tallies<MS_BLOCK>(tl, ctr, tally);
}

// Sources, in one workgroup (k <= 256 threads): the source vertices' frontier
// records are cleared (the slot may hold an earlier run's masks), then seen
// and frontier bits at the relabelled vertex and its active bitmap bit. Depth
// 0 comes from the level history. The tallies (reached (vertex, source)
// pairs, and the degrees summed over them) start from the k sources and are
// added to level by level.
__global__ void __launch_bounds__(256) ms_tile_init_kernel(const int32_t *__restrict__ srcs,
                                                           const int32_t *__restrict__ rlabel, int32_t k, int32_t W,
                                                           uint64_t *seen, uint64_t *front, uint64_t *abits,
                                                           const int32_t *__restrict__ rdeg,
                                                           unsigned long long *__restrict__ tally) {
  const int j = threadIdx.x;
  const int64_t r = j < k ? (int64_t)rlabel[srcs[j]] : 0;
  // (source, source) pairs and their degrees start the reached and edge tallies
  const unsigned long long e = block_sum<unsigned long long, 256>(j < k ? (unsigned long long)rdeg[r] : 0ull);
  if (j == 0) {
    atomicAdd(&tally[0], (unsigned long long)k);
    atomicAdd(&tally[MS_TALLY_EDGES], e);
  }
  if (j < k)
    for (int w = 0; w < W; ++w) front[r * W + w] = 0ull;
  __syncthreads();
  if (j < k) {
    const unsigned long long bit = 1ull << (j & 63);
    atomicOr((unsigned long long *)&seen[r * W + (j >> 6)], bit);
    atomicOr((unsigned long long *)&front[r * W + (j >> 6)], bit);
    atomicOr((unsigned long long *)&abits[r >> 6], 1ull << (r & 63));
  }
}

// Depth rows from the level history: level l's frontier masks f[l] (valid
// where the active bitmap a[l] has the vertex) hold the sources first seen at
// depth l; sources never seen keep 255. One thread per (relabelled vertex w,
// 64-source word), so a wavefront covers 64 / W vertices: per level one load
// of their shared active word and one contiguous load of their mask words,
// all levels in flight. A word's 64 bits become 64 depth bytes four at a time
// (a 4-bit mask times 0x00204081 puts bit j at bit 8j), and the thread writes
// its 64 bytes of row orig[w] (the caller's order).
constexpr int MS_HIST = 16;
struct ms_hist_args {
  const uint64_t *f[MS_HIST];
  const uint64_t *a[MS_HIST];
};

template <int W>
__global__ void __launch_bounds__(256) ms_depth_flush_kernel(ms_hist_args h, int32_t L,
                                                             const int32_t *__restrict__ orig, int64_t n, int32_t k,
                                                             uint8_t *__restrict__ depth) {
  const bool vec = (k & 15) == 0 && ((uintptr_t)depth & 15) == 0;
  // full 256-byte rows: a wavefront's 16 rows go through LDS so that each
  // store instruction writes four whole rows
  __shared__ uint4 tr[256 / BYO_WAVE][16 * 16];
  const bool rows = W == 4 && k == 256 && vec;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i - lane_id() < n * W;
       i += (int64_t)gridDim.x * blockDim.x) {  // uniform per wavefront
    const bool live = i < n * W;
    const int64_t w = live ? i / W : 0;
    const int word = (int)(i - w * W);
    const uint64_t bit = 1ull << (w & 63);
    uint64_t act[MS_HIST], fm[MS_HIST];
#pragma unroll
    for (int l = 0; l < MS_HIST; ++l) act[l] = l < L ? h.a[l][w >> 6] : 0ull;
#pragma unroll
    for (int l = 0; l < MS_HIST; ++l) fm[l] = (live && (act[l] & bit)) ? h.f[l][i] : 0ull;
    uint32_t c[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) c[q] = 0xFFFFFFFFu;
#pragma unroll
    for (int l = 0; l < MS_HIST; ++l) {
      const uint64_t m = fm[l];
      if (!m) continue;
      const uint32_t ls = 0x01010101u * (uint32_t)l;
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const uint32_t b4 = (uint32_t)(m >> (4 * q)) & 0xFu;
        const uint32_t bm = ((b4 * 0x00204081u) & 0x01010101u) * 0xFFu;
        c[q] = (c[q] & ~bm) | (ls & bm);
      }
    }
    if (rows) {
      uint4 *t = tr[threadIdx.x / BYO_WAVE];
      const int lane = lane_id();
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4)
        t[lane * 4 + s4] = make_uint4(c[4 * s4], c[4 * s4 + 1], c[4 * s4 + 2], c[4 * s4 + 3]);
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      const int64_t w0 = (i - lane) / W;  // the wavefront's first vertex
#pragma unroll
      for (int st = 0; st < 4; ++st) {
        const int vr = 4 * st + (lane >> 4);  // vertex of the wavefront this lane stores
        const int64_t wv = w0 + vr;
        if (wv < n) {
          // row vr's 16-byte group (lane & 15) is piece s4 = (lane & 3) of lane 4 vr + (lane & 15) / 4
          const uint4 x = t[(4 * vr + ((lane & 15) >> 2)) * 4 + (lane & 3)];
          *(uint4 *)(depth + (int64_t)orig[wv] * 256 + 16 * (lane & 15)) = x;
        }
      }
      __builtin_amdgcn_wave_barrier();
      continue;
    }
    if (!live) continue;
    uint8_t *row = depth + (int64_t)orig[w] * k + 64 * word;
    if (vec && 64 * word + 64 <= k) {
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4)
        ((uint4 *)row)[s4] = make_uint4(c[4 * s4], c[4 * s4 + 1], c[4 * s4 + 2], c[4 * s4 + 3]);
    } else {
      for (int j = 0; j < 64 && 64 * word + j < k; ++j) row[j] = (uint8_t)(c[j >> 2] >> (8 * (j & 3)));
    }
  }
}

template <int W>
static void launch_pull(const byo_graph *g, const uint64_t *front, uint64_t *seen, uint64_t *next, uint8_t *depth,
                        int32_t k, uint8_t nd, uint64_t *abits, byo_counters *ctr, int32_t tw, hipStream_t s) {
  unsigned nb = (unsigned)std::min<int64_t>(std::max<int64_t>(1, (g->n + MS_BLOCK - 1) / MS_BLOCK), 4096);
  ms_pull_kernel<W><<<nb, MS_BLOCK, 0, s>>>(g->off, g->nbr, g->deg, g->n, front, seen, next, depth, k, nd, abits,
                                            ctr, tw);
}

template <int W>
static void launch_clear_bits(const uint64_t *bits, int64_t n, uint64_t *front, hipStream_t s) {
  unsigned nb = (unsigned)std::min<int64_t>(std::max<int64_t>(1, (n + 255) / 256), 4096);
  ms_clear_bits_kernel<W><<<nb, 256, 0, s>>>(bits, n, front);
}

template <int W>
static void launch_finish(const byo_graph *g, const int32_t *touched, const byo_counters *tctr, uint64_t *visit,
                          uint64_t *seen, uint64_t *next, uint64_t *tbits, uint8_t *depth, int32_t k, uint8_t nd,
                          int32_t *active, byo_counters *ctr, int64_t bound, hipStream_t s) {
  unsigned nb = (unsigned)std::min<int64_t>(std::max<int64_t>(1, (bound + MS_BLOCK - 1) / MS_BLOCK), 16384);
  ms_finish_kernel<W><<<nb, MS_BLOCK, 0, s>>>(touched, tctr, g->deg, visit, seen, next, tbits, depth, k, nd, active,
                                              ctr);
}

template <int W>
static void launch_clear(const int32_t *list, int64_t cnt, uint64_t *front, hipStream_t s) {
  if (cnt <= 0) return;
  ms_clear_kernel<W><<<(unsigned)((cnt + 255) / 256), 256, 0, s>>>(list, cnt, front);
}

struct ms_ws {
  int64_t n = -1;
  int W = 0;
  uint64_t *seen = nullptr, *front[2] = {nullptr, nullptr}, *visit = nullptr, *tbits = nullptr;
  uint64_t *abits[2] = {nullptr, nullptr};
  uint64_t *fbits = nullptr;  // tiled levels: vertices that have seen every source
  int32_t *touched = nullptr, *active[2] = {nullptr, nullptr}, *srcs = nullptr;
  byo_counters *ctr = nullptr;
  unsigned long long *tally = nullptr;
  // Tiled runs keep each level's frontier masks and active bitmap (slots 0
  // and 1 are front[] and abits[], the rest allocated on first use) and build
  // the depths from them in one pass.
  int nhist = 0;
  uint64_t *hfront[MS_HIST] = {}, *habits[MS_HIST] = {};
  // visit and the touched bits are back to zero after a completed tiled run
  bool tiled_clean = false;
};

static void ms_free(ms_ws &m) {
  void *p[] = {m.seen, m.front[0], m.front[1], m.visit, m.tbits, m.touched, m.active[0], m.active[1], m.srcs,
               m.ctr, m.tally, m.abits[0], m.abits[1], m.fbits};
  for (void *x : p)
    if (x) (void)hipFree(x);
  for (int i = 2; i < m.nhist; ++i) {
    if (m.hfront[i]) (void)hipFree(m.hfront[i]);
    if (m.habits[i]) (void)hipFree(m.habits[i]);
  }
  m = ms_ws();
}

constexpr int MS_MAX_LEVELS = 255;

void ms_release(byo_workspace &w) {
  if (!w.ms) return;
  ms_free(*(ms_ws *)w.ms);
  delete (ms_ws *)w.ms;
  w.ms = nullptr;
}


// After a push level in the layout's order: fold visit[v] into seen and the
// next frontier for every touched v, write depths in the caller's order, set
// the frontier and "full" bitmaps, clear the touched bits, count.
template <int W>
__global__ void __launch_bounds__(MS_BLOCK) ms_tile_finish_kernel(
    const int32_t *__restrict__ touched, const byo_counters *__restrict__ tctr, const int32_t *__restrict__ rdeg,
    const int32_t *__restrict__ orig, uint64_t *__restrict__ visit, uint64_t *__restrict__ seen,
    uint64_t *__restrict__ front_next, uint64_t *__restrict__ touched_bits, uint64_t *__restrict__ abits_next,
    uint64_t *__restrict__ fbits, uint8_t *__restrict__ depth, int32_t k, uint8_t newdepth,
    byo_counters *__restrict__ ctr, unsigned long long *__restrict__ tally) {
  uint64_t full[W];
#pragma unroll
  for (int w = 0; w < W; ++w) {
    int bits = k - 64 * w;
    full[w] = bits >= 64 ? ~0ull : (bits <= 0 ? 0ull : (~0ull >> (64 - bits)));
  }
  const int64_t cnt = (int64_t)tctr->count;
  unsigned long long degsum = 0, count = 0, pairs = 0, edges = 0;
  for (int64_t i = (int64_t)blockIdx.x * MS_BLOCK + threadIdx.x; i < cnt; i += (int64_t)gridDim.x * MS_BLOCK) {
    const int32_t v = touched[i];
    uint64_t nb[W], sv[W];
    bool any = false, now_full = true;
#pragma unroll
    for (int w = 0; w < W; ++w) {
      const uint64_t x = visit[(int64_t)v * W + w];
      visit[(int64_t)v * W + w] = 0ull;
      sv[w] = seen[(int64_t)v * W + w];
      nb[w] = x & ~sv[w];
      any |= nb[w] != 0;
      now_full &= (sv[w] | nb[w]) == full[w];
    }
    const uint64_t bit = 1ull << (v & 63);
    if (any) {
#pragma unroll
      for (int w = 0; w < W; ++w) {
        seen[(int64_t)v * W + w] = sv[w] | nb[w];
        front_next[(int64_t)v * W + w] = nb[w];
      }
      if (depth) write_depths<W>(depth, orig[v], k, nb, sv, newdepth);
      degsum += (unsigned long long)rdeg[v];
      count += 1;
      unsigned long long pc = 0;
#pragma unroll
      for (int w = 0; w < W; ++w) pc += (unsigned long long)__popcll(nb[w]);
      pairs += pc;
      edges += pc * (unsigned long long)rdeg[v];
      atomicOr((unsigned long long *)&abits_next[v >> 6], (unsigned long long)bit);
      if (now_full) atomicOr((unsigned long long *)&fbits[v >> 6], (unsigned long long)bit);
    }
    atomicAnd((unsigned long long *)&touched_bits[v >> 6], ~(unsigned long long)bit);
  }
  const unsigned long long ts = block_sum<unsigned long long, MS_BLOCK>(degsum);
  const unsigned long long tc = block_sum<unsigned long long, MS_BLOCK>(count);
  const unsigned long long tp = block_sum<unsigned long long, MS_BLOCK>(pairs);
  const unsigned long long te = block_sum<unsigned long long, MS_BLOCK>(edges);
  if (threadIdx.x == 0) {
    if (ts) atomicAdd(&ctr->degsum, ts);
    if (tc) atomicAdd(&ctr->count, tc);
    if (tp) atomicAdd(&tally[0], tp);
    if (te) atomicAdd(&tally[MS_TALLY_EDGES], te);
  }
}

// Level buffers of a tiled level: the current and next frontier masks and
// active bitmaps (history slots), the active list buffer, and the depth array
// (null while the depths come from the history).
struct ms_level_bufs {
  uint64_t *front_cur, *front_next, *abits_cur, *abits_next;
  int32_t *active;
  uint8_t *depth;
};

template <int W>
static byo_status launch_tile_push(byo_graph *g, const byo_tiles *t, ms_ws &mw, const ms_level_bufs &lb,
                                   int64_t acount, long long adeg, int32_t k, uint8_t nd, byo_counters *tctr,
                                   byo_counters *ctr, const byo_opts &o, hipStream_t s) {
  const int64_t n = g->n, words = (n + 63) / 64;
  byo_workspace &w = g->ws;
  // active list from the frontier bitmap, then push over the relabelled CSR
  BYO_TRY(bitmap_to_ids(lb.abits_cur, words, n, lb.active, w.partial, w.partial_cap, (unsigned long long *)w.misc,
                        s));
  byo_graph rg = tiles_view(g, t);
  level_io io;
  std::memset(&io, 0, sizeof(io));
  io.in_ids = lb.active;
  io.in_count = acount;
  io.out_ids = mw.touched;
  io.out_bits = mw.tbits;
  io.ctr = tctr;
  ms_state ms{W, lb.front_cur, mw.seen, mw.visit};
  BYO_TRY(ms_push_level(&rg, BYO_V_PUSH_EDGE, ms, io, o, s, adeg));
  BYO_TRY(fill_u64(lb.abits_next, words, 0ull, s));
  {
    ktimer_scope kt(BYO_K_MSBFS_FINISH, s);
    const unsigned nb = (unsigned)std::min<int64_t>(std::max<int64_t>(1, (adeg + MS_BLOCK - 1) / MS_BLOCK), 2048);
    ms_tile_finish_kernel<W><<<nb, MS_BLOCK, 0, s>>>(mw.touched, tctr, t->rdeg, t->orig, mw.visit, mw.seen,
                                                     lb.front_next, mw.tbits, lb.abits_next, mw.fbits, lb.depth, k,
                                                     nd, ctr, mw.tally);
  }
  BYO_HIP(hipGetLastError());
  return BYO_OK;
}

template <int W>
static void launch_tile_level(const byo_tiles *t, ms_ws &mw, const ms_level_bufs &lb, int32_t k, uint8_t nd,
                              int64_t n, byo_counters *ctr, hipStream_t s) {
  int64_t words = (n + 63) / 64;
  const ms_fin_args f{mw.seen, lb.front_next, lb.abits_next, mw.fbits, t->rdeg, t->orig, lb.depth, k, nd, n};
  {
    ktimer_scope kt(BYO_K_MSBFS_PULL, s);
    ms_tile_kernel<W><<<(unsigned)t->nchunks, MT_THREADS, 0, s>>>(t->ent, t->anchor, t->cbeg, t->cblk, lb.front_cur,
                                                                 lb.abits_cur, words, t->bfirst, f, ctr, mw.tally,
                                                                 (uint64_t *)t->partial, t->cflag);
  }
  // the plan's pieces, then enough workgroups for the words of the trailing
  // tiles without entries (wtail is then a tile boundary; wtail == n: none)
  const int64_t tail_words = t->wtail < n ? words - (t->wtail >> 6) : 0;
  const int64_t tail_blocks = std::min<int64_t>((tail_words + MS_BLOCK - 1) / MS_BLOCK, 256);
  const int64_t grid = t->napply + tail_blocks;
  if (grid == 0) return;
  ktimer_scope kt(BYO_K_MSBFS_FINISH, s);
  ms_tile_apply_kernel<W><<<(unsigned)grid, MS_BLOCK, 0, s>>>((const uint64_t *)t->partial, t->cflag, t->bfirst,
                                                              t->aplan, t->napply, t->wtail, f, ctr, mw.tally);
}

// History slots for the tiled levels: as many as fit in a quarter of the free
// device memory, at most MS_HIST (two always exist).
static byo_status ms_hist_ensure(ms_ws &mw, int64_t n, int W) {
  if (mw.nhist > 0) return BYO_OK;
  const size_t words = (size_t)std::max<int64_t>((n + 63) / 64, 1);
  const size_t per = sizeof(uint64_t) * ((size_t)n * W + words);
  size_t fr = 0, tot = 0;
  BYO_HIP(hipMemGetInfo(&fr, &tot));
  int H = 2;
  while (H < MS_HIST && (size_t)(H - 1) * per <= fr / 4) ++H;
  mw.hfront[0] = mw.front[0];
  mw.hfront[1] = mw.front[1];
  mw.habits[0] = mw.abits[0];
  mw.habits[1] = mw.abits[1];
  mw.nhist = 2;
  for (int i = 2; i < H; ++i) {
    BYO_HIP(hipMalloc(&mw.hfront[i], sizeof(uint64_t) * (size_t)n * W));
    BYO_HIP(hipMalloc(&mw.habits[i], sizeof(uint64_t) * words));
    mw.nhist = i + 1;
  }
  return BYO_OK;
}

static void launch_depth_flush(const ms_ws &mw, int32_t L, const byo_tiles *t, int64_t n, int32_t k, int W,
                               uint8_t *depth, hipStream_t s) {
  ms_hist_args h;
  for (int i = 0; i < MS_HIST; ++i) {
    h.f[i] = i < mw.nhist ? mw.hfront[i] : nullptr;
    h.a[i] = i < mw.nhist ? mw.habits[i] : nullptr;
  }
  const int64_t total = n * (int64_t)W;
  const unsigned nb = (unsigned)std::min<int64_t>(std::max<int64_t>(1, (total + 255) / 256), 65536);
  ktimer_scope kt(BYO_K_MSBFS_FINISH, s);
  switch (W) {
    case 1: ms_depth_flush_kernel<1><<<nb, 256, 0, s>>>(h, L, t->orig, n, k, depth); break;
    case 2: ms_depth_flush_kernel<2><<<nb, 256, 0, s>>>(h, L, t->orig, n, k, depth); break;
    case 3: ms_depth_flush_kernel<3><<<nb, 256, 0, s>>>(h, L, t->orig, n, k, depth); break;
    default: ms_depth_flush_kernel<4><<<nb, 256, 0, s>>>(h, L, t->orig, n, k, depth); break;
  }
}

// Levels in the layout's vertex order, direction-optimising like the CSR
// path: a push over the relabelled CSR while |U| + sum(deg U) <= m / div,
// else a pass over the tiles. Level l's frontier masks and active bitmap go
// to history slot l; the depth rows are built from the slots in one pass at
// the end, or just before a level would need a slot beyond the last. Levels
// after that alternate between the last two slots and write their depths
// directly. The caller has zeroed seen, the full bitmap and the counters
// (and visit and the touched bits unless a tiled run left them zero).
static byo_status ms_tiled_run(byo_graph *g, ms_ws &mw, int32_t k, int W,
                               uint8_t *d_depth, const byo_opts &o, hipStream_t s, byo_run_stats *stats) {
  byo_tiles *t = nullptr;
  BYO_TRY(tiles_ensure(g, MT_SHIFT, s, &t));
  BYO_TRY(tiles_partial(t, sizeof(uint64_t) * (size_t)W << MT_SHIFT));
  const int64_t n = g->n, words = (n + 63) / 64;
  BYO_CHECK(o.ms_history == 0 || (o.ms_history >= 2 && o.ms_history <= MS_HIST), BYO_EINVAL,
            "ms_history must be 0 or 2 .. 16");
  BYO_TRY(ms_hist_ensure(mw, n, W));
  const int H = o.ms_history ? std::min(o.ms_history, mw.nhist) : mw.nhist;
  auto slot = [H](int l) { return l < H ? l : (H - 2) + ((l - H) & 1); };
  BYO_HIP(hipMemsetAsync(mw.habits[0], 0, sizeof(uint64_t) * (size_t)words, s));
  ms_tile_init_kernel<<<1, 256, 0, s>>>(mw.srcs, t->rlabel, k, W, mw.seen, mw.hfront[0], mw.habits[0], t->rdeg,
                                        mw.tally);
  BYO_HIP(hipGetLastError());
  // first frontier: the distinct sources (from the frontier bitmap) and their
  // degree sum
  int64_t acount = 0;
  long long adeg = 0;
  {
    unsigned long long cnt = 0;
    BYO_TRY(bitmap_to_ids(mw.habits[0], words, n, mw.active[0], g->ws.partial, g->ws.partial_cap,
                          (unsigned long long *)g->ws.misc, s));
    BYO_TRY(sync_read(s, g->ws.misc, &cnt, sizeof(cnt)));
    acount = (int64_t)cnt;
    byo_graph rg = tiles_view(g, t);
    BYO_TRY(frontier_degree_scan(&rg, mw.active[0], acount, g->ws.scan, g->ws.partial, g->ws.partial_cap, s));
    BYO_TRY(sync_read(s, g->ws.scan + acount, &adeg, sizeof(adeg)));
  }
  const int64_t div = o.dense_divisor > 0 ? o.dense_divisor : 20;
  byo_run_stats st;
  std::memset(&st, 0, sizeof(st));
  int level = 0;
  bool flushed = false;
  while (acount > 0) {
    if (level + 1 >= MS_MAX_LEVELS) {
      if (stats) *stats = st;
      return fail(BYO_ELIMIT, "a distance reached 255 (depths are uint8)");
    }
    if (level + 1 == H) {  // the next level needs a slot the history still uses
      launch_depth_flush(mw, H, t, n, k, W, d_depth, s);
      BYO_HIP(hipGetLastError());
      flushed = true;
    }
    const uint8_t nd = (uint8_t)(level + 1);
    const int cs = slot(level), ns = slot(level + 1);
    const ms_level_bufs lb{mw.hfront[cs], mw.hfront[ns], mw.habits[cs], mw.habits[ns], mw.active[level & 1],
                           flushed ? d_depth : nullptr};
    byo_counters *tctr = mw.ctr + 2 * level, *ctr = mw.ctr + 2 * level + 1;
    const bool fixed_pull = o.fixed_variant == BYO_V_PULL_THREAD || o.fixed_variant == BYO_V_PULL_WAVE;
    const bool push = o.selector == BYO_SEL_FIXED ? !fixed_pull : acount + adeg <= g->m / div;
    if (push) {
      switch (W) {
        case 1: BYO_TRY(launch_tile_push<1>(g, t, mw, lb, acount, adeg, k, nd, tctr, ctr, o, s)); break;
        case 2: BYO_TRY(launch_tile_push<2>(g, t, mw, lb, acount, adeg, k, nd, tctr, ctr, o, s)); break;
        case 3: BYO_TRY(launch_tile_push<3>(g, t, mw, lb, acount, adeg, k, nd, tctr, ctr, o, s)); break;
        default: BYO_TRY(launch_tile_push<4>(g, t, mw, lb, acount, adeg, k, nd, tctr, ctr, o, s)); break;
      }
    } else {
      switch (W) {
        case 1: launch_tile_level<1>(t, mw, lb, k, nd, n, ctr, s); break;
        case 2: launch_tile_level<2>(t, mw, lb, k, nd, n, ctr, s); break;
        case 3: launch_tile_level<3>(t, mw, lb, k, nd, n, ctr, s); break;
        default: launch_tile_level<4>(t, mw, lb, k, nd, n, ctr, s); break;
      }
    }
    BYO_HIP(hipGetLastError());
    byo_counters c;
    BYO_TRY(sync_read(s, ctr, &c, sizeof(c)));
    st.variant_count[push ? BYO_V_PUSH_EDGE : BYO_V_PULL_WAVE]++;
    ++level;
    acount = (int64_t)c.count;
    adeg = (long long)c.degsum;
  }
  // levels 0 .. level are in slots 0 .. level (the last one empty)
  if (!flushed) launch_depth_flush(mw, level + 1, t, n, k, W, d_depth, s);
  unsigned long long tl[MS_TALLY_WORDS] = {};
  BYO_TRY(sync_read(s, mw.tally, tl, sizeof(tl)));
  st.levels = level;
  st.reached = (int64_t)tl[0];
  st.edges = (int64_t)tl[MS_TALLY_EDGES];
  if (stats) *stats = st;
  mw.tiled_clean = true;
  return BYO_OK;
}
}  // namespace byo

using namespace byo;

extern "C" byo_status byo_msbfs(byo_graph *g, const int64_t *h_srcs, int32_t k, uint8_t *d_depth,
                                const byo_opts *opts, void *stream, byo_run_stats *stats) {
  BYO_CHECK(g && h_srcs && d_depth, BYO_EINVAL, "null argument");
  BYO_CHECK(k >= 1 && k <= 256, BYO_EINVAL, "k must be in [1, 256]");
  for (int32_t j = 0; j < k; ++j)
    BYO_CHECK(h_srcs[j] >= 0 && h_srcs[j] < g->n, BYO_EINVAL, "source out of range");
  byo_opts o;
  byo_opts_default(&o);
  if (opts) o = *opts;
  hipStream_t s = (hipStream_t)stream;
  BYO_TRY(ws_ensure_traversal(g));
  int64_t n = g->n, words = (n + 63) / 64;
  int W = (k + 63) / 64;
  // workspace on the graph, sized for the widest W seen so far
  if (!g->ws.ms) g->ws.ms = new ms_ws();
  ms_ws &mw = *(ms_ws *)g->ws.ms;
  if (mw.n != n || mw.W != W) {
    ms_free(mw);
    size_t vb = sizeof(uint64_t) * (size_t)n * W;
    BYO_HIP(hipMalloc(&mw.seen, vb));
    BYO_HIP(hipMalloc(&mw.front[0], vb));
    BYO_HIP(hipMalloc(&mw.front[1], vb));
    BYO_HIP(hipMalloc(&mw.visit, vb));
    BYO_HIP(hipMalloc(&mw.tbits, sizeof(uint64_t) * (size_t)std::max<int64_t>(words, 1)));
    BYO_HIP(hipMalloc(&mw.abits[0], sizeof(uint64_t) * (size_t)std::max<int64_t>(words, 1)));
    BYO_HIP(hipMalloc(&mw.abits[1], sizeof(uint64_t) * (size_t)std::max<int64_t>(words, 1)));
    BYO_HIP(hipMalloc(&mw.fbits, sizeof(uint64_t) * (size_t)std::max<int64_t>(words, 1)));
    BYO_HIP(hipMalloc(&mw.touched, sizeof(int32_t) * (size_t)n));
    BYO_HIP(hipMalloc(&mw.active[0], sizeof(int32_t) * (size_t)n));
    BYO_HIP(hipMalloc(&mw.active[1], sizeof(int32_t) * (size_t)n));
    BYO_HIP(hipMalloc(&mw.srcs, sizeof(int32_t) * 256));
    BYO_HIP(hipMalloc(&mw.ctr, sizeof(byo_counters) * 2 * (MS_MAX_LEVELS + 1)));
    BYO_HIP(hipMalloc(&mw.tally, sizeof(unsigned long long) * MS_TALLY_WORDS));
    mw.n = n;
    mw.W = W;
  }
  size_t vb = sizeof(uint64_t) * (size_t)n * W;
  std::vector<int32_t> hs(k);
  for (int32_t j = 0; j < k; ++j) hs[j] = (int32_t)h_srcs[j];
  BYO_HIP(hipMemcpyAsync(mw.srcs, hs.data(), sizeof(int32_t) * k, hipMemcpyHostToDevice, s));
  if (o.tiled && tiles_wanted(g)) {
    // the frontier slots need no clearing and the depth rows are written whole
    BYO_HIP(hipMemsetAsync(mw.seen, 0, vb, s));
    if (!mw.tiled_clean) {
      BYO_HIP(hipMemsetAsync(mw.visit, 0, vb, s));
      BYO_HIP(hipMemsetAsync(mw.tbits, 0, sizeof(uint64_t) * (size_t)std::max<int64_t>(words, 1), s));
    }
    BYO_HIP(hipMemsetAsync(mw.fbits, 0, sizeof(uint64_t) * (size_t)std::max<int64_t>(words, 1), s));
    BYO_HIP(hipMemsetAsync(mw.ctr, 0, sizeof(byo_counters) * 2 * (MS_MAX_LEVELS + 1), s));
    BYO_HIP(hipMemsetAsync(mw.tally, 0, sizeof(unsigned long long) * MS_TALLY_WORDS, s));
    mw.tiled_clean = false;
    byo_status r = ms_tiled_run(g, mw, k, W, d_depth, o, s, stats);
    // the copy of hs must stay alive until the stream has read it
    if (r != BYO_OK) (void)hipStreamSynchronize(s);
    return r;
  }
  mw.tiled_clean = false;
  BYO_HIP(hipMemsetAsync(mw.seen, 0, vb, s));
  BYO_HIP(hipMemsetAsync(mw.front[0], 0, vb, s));
  BYO_HIP(hipMemsetAsync(mw.front[1], 0, vb, s));
  BYO_HIP(hipMemsetAsync(mw.visit, 0, vb, s));
  BYO_HIP(hipMemsetAsync(mw.tbits, 0, sizeof(uint64_t) * (size_t)std::max<int64_t>(words, 1), s));
  BYO_HIP(hipMemsetAsync(mw.fbits, 0, sizeof(uint64_t) * (size_t)std::max<int64_t>(words, 1), s));
  BYO_HIP(hipMemsetAsync(mw.ctr, 0, sizeof(byo_counters) * 2 * (MS_MAX_LEVELS + 1), s));
  BYO_HIP(hipMemsetAsync(mw.tally, 0, sizeof(unsigned long long) * MS_TALLY_WORDS, s));
  {
    int64_t total = n * (int64_t)k;
    unsigned nb = (unsigned)std::min<int64_t>(std::max<int64_t>(1, (total / 16 + 255) / 256), 65536);
    u8_fill_kernel<<<nb, 256, 0, s>>>(d_depth, total, 255);
  }
  ms_init_kernel<<<1, 256, 0, s>>>(mw.srcs, k, W, mw.seen, mw.front[0], d_depth);
  // first active list: the distinct sources
  std::vector<int32_t> act(hs);
  std::sort(act.begin(), act.end());
  act.erase(std::unique(act.begin(), act.end()), act.end());
  BYO_HIP(hipMemcpyAsync(mw.active[0], act.data(), sizeof(int32_t) * act.size(), hipMemcpyHostToDevice, s));
  int64_t acount = (int64_t)act.size();
  long long adeg = 0;
  BYO_TRY(frontier_degree_scan(g, mw.active[0], acount, g->ws.scan, g->ws.partial, g->ws.partial_cap, s));
  BYO_TRY(sync_read(s, g->ws.scan + acount, &adeg, sizeof(adeg)));
  BYO_HIP(hipGetLastError());

  byo_run_stats st;
  std::memset(&st, 0, sizeof(st));
  int cur = 0;
  int level = 0;
  bool as_list = true;  // is the current active set held as a list (else as a bitmap)?
  int32_t tw = o.t_wave > 0 ? o.t_wave : 32;
  int64_t div = o.dense_divisor > 0 ? o.dense_divisor : 20;
  while (acount > 0) {
    if (level + 1 >= MS_MAX_LEVELS) {
      if (stats) *stats = st;
      return fail(BYO_ELIMIT, "a distance reached 255 (depths are uint8)");
    }
    uint8_t nd = (uint8_t)(level + 1);
    byo_counters *tctr = mw.ctr + 2 * level, *actr = mw.ctr + 2 * level + 1;
    int variant;
    if (o.selector == BYO_SEL_FIXED)
      variant = o.fixed_variant;
    else
      variant = (acount + adeg > g->m / div) ? BYO_V_PULL_WAVE : BYO_V_PUSH_EDGE;
    bool pull = variant == BYO_V_PULL_THREAD || variant == BYO_V_PULL_WAVE;
    int nx = 1 - cur;
    if (pull) {
      ktimer_scope kt(BYO_K_MSBFS_PULL, s);
      switch (W) {
        case 1: launch_pull<1>(g, mw.front[cur], mw.seen, mw.front[nx], d_depth, k, nd, mw.abits[nx], actr, tw, s); break;
        case 2: launch_pull<2>(g, mw.front[cur], mw.seen, mw.front[nx], d_depth, k, nd, mw.abits[nx], actr, tw, s); break;
        case 3: launch_pull<3>(g, mw.front[cur], mw.seen, mw.front[nx], d_depth, k, nd, mw.abits[nx], actr, tw, s); break;
        default: launch_pull<4>(g, mw.front[cur], mw.seen, mw.front[nx], d_depth, k, nd, mw.abits[nx], actr, tw, s); break;
      }
      BYO_HIP(hipGetLastError());
    } else {
      if (!as_list) {
        BYO_TRY(bitmap_to_ids(mw.abits[cur], words, n, mw.active[cur], g->ws.partial, g->ws.partial_cap,
                              (unsigned long long *)g->ws.misc, s));
        as_list = true;
      }
      level_io io;
      std::memset(&io, 0, sizeof(io));
      io.in_ids = mw.active[cur];
      io.in_count = acount;
      io.out_ids = mw.touched;
      io.out_bits = mw.tbits;
      io.ctr = tctr;
      io.ctr_clear = nullptr;
      ms_state ms{W, mw.front[cur], mw.seen, mw.visit};
      BYO_TRY(ms_push_level(g, variant, ms, io, o, s, adeg));
      ktimer_scope kt(BYO_K_MSBFS_FINISH, s);
      switch (W) {
        case 1: launch_finish<1>(g, mw.touched, tctr, mw.visit, mw.seen, mw.front[nx], mw.tbits, d_depth, k, nd, mw.active[nx], actr, adeg, s); break;
        case 2: launch_finish<2>(g, mw.touched, tctr, mw.visit, mw.seen, mw.front[nx], mw.tbits, d_depth, k, nd, mw.active[nx], actr, adeg, s); break;
        case 3: launch_finish<3>(g, mw.touched, tctr, mw.visit, mw.seen, mw.front[nx], mw.tbits, d_depth, k, nd, mw.active[nx], actr, adeg, s); break;
        default: launch_finish<4>(g, mw.touched, tctr, mw.visit, mw.seen, mw.front[nx], mw.tbits, d_depth, k, nd, mw.active[nx], actr, adeg, s); break;
      }
      BYO_HIP(hipGetLastError());
    }
    // the consumed frontier buffer must be all-zero before it is reused as output
    if (as_list) {
      switch (W) {
        case 1: launch_clear<1>(mw.active[cur], acount, mw.front[cur], s); break;
        case 2: launch_clear<2>(mw.active[cur], acount, mw.front[cur], s); break;
        case 3: launch_clear<3>(mw.active[cur], acount, mw.front[cur], s); break;
        default: launch_clear<4>(mw.active[cur], acount, mw.front[cur], s); break;
      }
    } else {
      switch (W) {
        case 1: launch_clear_bits<1>(mw.abits[cur], n, mw.front[cur], s); break;
        case 2: launch_clear_bits<2>(mw.abits[cur], n, mw.front[cur], s); break;
        case 3: launch_clear_bits<3>(mw.abits[cur], n, mw.front[cur], s); break;
        default: launch_clear_bits<4>(mw.abits[cur], n, mw.front[cur], s); break;
      }
    }
    BYO_HIP(hipGetLastError());
    byo_counters c;
    BYO_TRY(sync_read(s, actr, &c, sizeof(c)));
    st.variant_count[pull ? BYO_V_PULL_WAVE : variant]++;
    ++level;
    acount = (int64_t)c.count;
    adeg = (long long)c.degsum;
    as_list = !pull;
    cur = nx;
  }
  ms_tally_kernel<<<(unsigned)std::min<int64_t>(std::max<int64_t>(1, (n + 255) / 256), 4096), MS_BLOCK, 0, s>>>(
      mw.seen, W, g->deg, n, mw.tally);
  unsigned long long tl[MS_TALLY_WORDS] = {};
  BYO_TRY(sync_read(s, mw.tally, tl, sizeof(tl)));
  st.levels = level;
  st.reached = (int64_t)tl[0];
  st.edges = (int64_t)tl[MS_TALLY_EDGES];
  if (stats) *stats = st;
  return BYO_OK;
}
