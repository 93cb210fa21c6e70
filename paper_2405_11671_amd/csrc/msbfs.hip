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

template <int W>
__device__ __forceinline__ void write_depths(uint8_t *__restrict__ depth, int64_t v, int32_t k, const uint64_t *nb,
                                             uint8_t d) {
#pragma unroll
  for (int w = 0; w < W; ++w) {
    uint64_t x = nb[w];
    while (x) {
      int j = __ffsll((long long)x) - 1;
      depth[v * k + w * 64 + j] = d;
      x &= x - 1;
    }
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
      write_depths<W>(depth, v, k, nb, newdepth);
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
      uint64_t nb[W];
#pragma unroll
      for (int w = 0; w < W; ++w) {
        uint64_t x = visit[(int64_t)v * W + w];
        visit[(int64_t)v * W + w] = 0ull;
        uint64_t sv = seen[(int64_t)v * W + w];
        nb[w] = x & ~sv;
        any |= nb[w] != 0;
        if (nb[w]) {
          seen[(int64_t)v * W + w] = sv | nb[w];
          next[(int64_t)v * W + w] = nb[w];
        }
      }
      if (any) {
        write_depths<W>(depth, v, k, nb, newdepth);
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
    atomicAdd(&out[1], te);
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
  int32_t *touched = nullptr, *active[2] = {nullptr, nullptr}, *srcs = nullptr;
  byo_counters *ctr = nullptr;
  unsigned long long *tally = nullptr;
};

static void ms_free(ms_ws &m) {
  void *p[] = {m.seen, m.front[0], m.front[1], m.visit, m.tbits, m.touched, m.active[0], m.active[1], m.srcs,
               m.ctr, m.tally, m.abits[0], m.abits[1]};
  for (void *x : p)
    if (x) (void)hipFree(x);
  m = ms_ws();
}

constexpr int MS_MAX_LEVELS = 255;

void ms_release(byo_workspace &w) {
  if (!w.ms) return;
  ms_free(*(ms_ws *)w.ms);
  delete (ms_ws *)w.ms;
  w.ms = nullptr;
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
    BYO_HIP(hipMalloc(&mw.touched, sizeof(int32_t) * (size_t)n));
    BYO_HIP(hipMalloc(&mw.active[0], sizeof(int32_t) * (size_t)n));
    BYO_HIP(hipMalloc(&mw.active[1], sizeof(int32_t) * (size_t)n));
    BYO_HIP(hipMalloc(&mw.srcs, sizeof(int32_t) * 256));
    BYO_HIP(hipMalloc(&mw.ctr, sizeof(byo_counters) * 2 * (MS_MAX_LEVELS + 1)));
    BYO_HIP(hipMalloc(&mw.tally, sizeof(unsigned long long) * 2));
    mw.n = n;
    mw.W = W;
  }
  size_t vb = sizeof(uint64_t) * (size_t)n * W;
  BYO_HIP(hipMemsetAsync(mw.seen, 0, vb, s));
  BYO_HIP(hipMemsetAsync(mw.front[0], 0, vb, s));
  BYO_HIP(hipMemsetAsync(mw.front[1], 0, vb, s));
  BYO_HIP(hipMemsetAsync(mw.visit, 0, vb, s));
  BYO_HIP(hipMemsetAsync(mw.tbits, 0, sizeof(uint64_t) * (size_t)std::max<int64_t>(words, 1), s));
  BYO_HIP(hipMemsetAsync(mw.ctr, 0, sizeof(byo_counters) * 2 * (MS_MAX_LEVELS + 1), s));
  BYO_HIP(hipMemsetAsync(mw.tally, 0, sizeof(unsigned long long) * 2, s));
  {
    int64_t total = n * (int64_t)k;
    unsigned nb = (unsigned)std::min<int64_t>(std::max<int64_t>(1, (total / 16 + 255) / 256), 65536);
    u8_fill_kernel<<<nb, 256, 0, s>>>(d_depth, total, 255);
  }
  std::vector<int32_t> hs(k);
  for (int32_t j = 0; j < k; ++j) hs[j] = (int32_t)h_srcs[j];
  BYO_HIP(hipMemcpyAsync(mw.srcs, hs.data(), sizeof(int32_t) * k, hipMemcpyHostToDevice, s));
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
  unsigned long long tl[2] = {0, 0};
  BYO_TRY(sync_read(s, mw.tally, tl, sizeof(tl)));
  st.levels = level;
  st.reached = (int64_t)tl[0];
  st.edges = (int64_t)tl[1];
  if (stats) *stats = st;
  return BYO_OK;
}
