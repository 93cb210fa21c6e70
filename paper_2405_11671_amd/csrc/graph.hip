// GraphContainer over a static CSR (paper Section 4.2) and the framework-level
// degree metadata the paper keeps when a container lacks it (Section 4.3).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <thread>
#include <vector>

#include "internal.h"

namespace byo {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

byo_status fail(byo_status st, const std::string &msg) {
  g_last_error = msg;
  return st;
}

byo_status hip_fail(hipError_t e, const char *what, const char *file, int line) {
  g_last_error = std::string(what) + " failed: " + hipGetErrorString(e) + " (" + file + ":" +
                 std::to_string(line) + ")";
  return (e == hipErrorOutOfMemory) ? BYO_ENOMEM : BYO_EHIP;
}

// Small reads (level counters, counts) go through a pinned staging buffer of
// the calling host thread, allocated on its first read and kept for the
// thread's life (64 KiB; not freed at exit, when the runtime may be gone): a
// copy into pageable memory would be staged by the runtime, which costs time
// on every level of a level loop.
constexpr size_t SYNC_STAGE_BYTES = 1 << 16;
static thread_local void *g_stage = nullptr;

// Calls made inside a no_alloc_scope (noalloc.hip) must not allocate: their
// reads go straight to the caller's memory (a pageable copy), and level
// records and kernel timers, which take events from a pool, are off.
static thread_local int g_noalloc = 0;
bool noalloc_active() { return g_noalloc > 0; }
no_alloc_scope::no_alloc_scope() { ++g_noalloc; }
no_alloc_scope::~no_alloc_scope() { --g_noalloc; }

byo_status sync_read(hipStream_t s, const void *d_src, void *h_dst, size_t bytes) {
  if (bytes <= SYNC_STAGE_BYTES && !noalloc_active()) {
    if (!g_stage) BYO_HIP(hipHostMalloc(&g_stage, SYNC_STAGE_BYTES, hipHostMallocDefault));
    BYO_HIP(hipMemcpyAsync(g_stage, d_src, bytes, hipMemcpyDeviceToHost, s));
    BYO_HIP(hipStreamSynchronize(s));
    std::memcpy(h_dst, g_stage, bytes);
    return BYO_OK;
  }
  BYO_HIP(hipMemcpyAsync(h_dst, d_src, bytes, hipMemcpyDeviceToHost, s));
  BYO_HIP(hipStreamSynchronize(s));
  return BYO_OK;
}

// ---------------------------------------------------------------- kernels

// deg[v] = off[v+1] - off[v]; zero_bits = bitmap of degree-0 vertices;
// out = {max degree, number of degree-0 vertices, sum of squared degrees}.
__global__ void __launch_bounds__(256) degree_stats_kernel(const int64_t *__restrict__ off, int64_t n,
                                                           int32_t *__restrict__ deg, uint64_t *__restrict__ zero_bits,
                                                           unsigned long long *__restrict__ out) {
  unsigned long long mx = 0, iso = 0, sq = 0;
  for (int64_t base = (int64_t)blockIdx.x * 256; base < n; base += (int64_t)gridDim.x * 256) {
    int64_t v = base + threadIdx.x;
    unsigned long long d = 0;
    bool z = false;
    if (v < n) {
      d = (unsigned long long)(off[v + 1] - off[v]);
      deg[v] = (int32_t)d;
      z = d == 0;
    }
    uint64_t zm = __ballot(z);
    if (lane_id() == 0 && v < n) zero_bits[v >> 6] = zm;
    mx = d > mx ? d : mx;
    iso += z;
    sq += d * d;
  }
  __shared__ unsigned long long smx[4];
  mx = wave_max(mx);
  if (lane_id() == 0) smx[threadIdx.x / 64] = mx;
  unsigned long long tiso = block_sum<unsigned long long, 256>(iso);
  unsigned long long tsq = block_sum<unsigned long long, 256>(sq);
  if (threadIdx.x == 0) {
    unsigned long long m4 = smx[0];
    for (int i = 1; i < 4; ++i) m4 = smx[i] > m4 ? smx[i] : m4;
    atomicMax(&out[0], m4);
    if (tiso) atomicAdd(&out[1], tiso);
    atomicAdd(&out[2], tsq);
  }
}

// Offsets: off[0] == 0, off[n] == m, non-decreasing.
__global__ void validate_offsets_kernel(const int64_t *__restrict__ off, int64_t n, int64_t m,
                                        unsigned long long *__restrict__ bad) {
  int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v > n) return;
  bool ok = true;
  int64_t o = off[v];
  if (v == 0 && o != 0) ok = false;
  if (v == n && o != m) ok = false;
  if (o < 0 || o > m) ok = false;
  if (v < n && off[v + 1] < o) ok = false;
  if (!ok) atomicAdd(bad, 1ull);
}

// Rows (one wavefront per row): entries in [0, n), strictly increasing, no
// self-loop, and (if symmetric) v appears in the row of each neighbour u.
__global__ void validate_rows_kernel(const int64_t *__restrict__ off, const int32_t *__restrict__ nbr, int64_t n,
                                     int check_sym, unsigned long long *__restrict__ bad) {
  int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / BYO_WAVE;
  int64_t nwaves = (int64_t)gridDim.x * blockDim.x / BYO_WAVE;
  unsigned long long errs = 0;
  for (int64_t v = wave; v < n; v += nwaves) {
    int64_t beg = off[v], end = off[v + 1];
    for (int64_t e = beg + lane_id(); e < end; e += BYO_WAVE) {
      int32_t u = nbr[e];
      if (u < 0 || u >= n || u == v) { ++errs; continue; }
      if (e > beg && nbr[e - 1] >= u) ++errs;
      if (check_sym) {
        int64_t lo = off[u], hi = off[u + 1];
        while (lo < hi) {
          int64_t mid = (lo + hi) >> 1;
          if (nbr[mid] < (int32_t)v) lo = mid + 1; else hi = mid;
        }
        if (lo >= off[u + 1] || nbr[lo] != (int32_t)v) ++errs;
      }
    }
  }
  errs = wave_sum(errs);
  if (lane_id() == 0 && errs) atomicAdd(bad, errs);
}

__global__ void fill_i32_kernel(int32_t *p, int64_t count, int32_t value) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < count; i += stride) p[i] = value;
}

__global__ void fill_u64_kernel(uint64_t *p, int64_t count, uint64_t value) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < count; i += stride) p[i] = value;
}

static unsigned grid_for(int64_t count, int block, int64_t cap = 65536) {
  int64_t g = (count + block - 1) / block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned)g;
}

byo_status fill_i32(int32_t *p, int64_t count, int32_t value, hipStream_t s) {
  if (count <= 0) return BYO_OK;
  fill_i32_kernel<<<grid_for(count, 256, 8192), 256, 0, s>>>(p, count, value);
  BYO_HIP(hipGetLastError());
  return BYO_OK;
}

byo_status fill_u64(uint64_t *p, int64_t count, uint64_t value, hipStream_t s) {
  if (count <= 0) return BYO_OK;
  fill_u64_kernel<<<grid_for(count, 256, 8192), 256, 0, s>>>(p, count, value);
  BYO_HIP(hipGetLastError());
  return BYO_OK;
}

// ---------------------------------------------------------------- workspace

void ws_free(byo_workspace &w) {
  void *dev[] = {w.visited, w.bits[0], w.bits[1], w.ids[0], w.ids[1], w.scan, w.partial, w.ctr, w.misc,
                 w.contrib[0], w.contrib[1], w.dpart, w.base, w.heavy_rows, w.chunk_row, w.chunk_beg,
                 w.row_chunk0, w.chunk_sum, w.api_deg, w.api_heavy, w.api_pre, w.api_aux,
                 w.bc_coef, w.bc_sigma, w.bc_depth, w.bc_order, w.kc_dcur, w.ds_deg, w.ds_alive};
  for (void *p : dev)
    if (p) (void)hipFree(p);
  if (w.h_ctr) (void)hipHostFree(w.h_ctr);
  ms_release(w);
  tiles_release(w);
  cz_free(w.cz);
  gm_release(w);
  dl_release(w);
  pb_release(w.pbfs);
  kp_release(w.kcp);
  w = byo_workspace();
}

byo_status ws_ensure_traversal(byo_graph *g) {
  byo_workspace &w = g->ws;
  if (w.visited) return BYO_OK;
  int64_t n = g->n;
  int64_t words = (n + 63) / 64;
  w.n = n;
  w.words = words;
  size_t wb = sizeof(uint64_t) * (size_t)std::max<int64_t>(words, 1);
  size_t ib = sizeof(int32_t) * (size_t)std::max<int64_t>(n, 1);
  int64_t pcap = std::max<int64_t>(compaction_blocks(words), (n + 1 + 2047) / 2048) + 2;
  BYO_HIP(hipMalloc(&w.visited, wb));
  BYO_HIP(hipMalloc(&w.bits[0], wb));
  BYO_HIP(hipMalloc(&w.bits[1], wb));
  BYO_HIP(hipMalloc(&w.ids[0], ib));
  BYO_HIP(hipMalloc(&w.ids[1], ib));
  BYO_HIP(hipMalloc(&w.scan, sizeof(long long) * (size_t)(n + 2)));
  BYO_HIP(hipMalloc(&w.partial, sizeof(long long) * (size_t)pcap));
  w.partial_cap = pcap;
  BYO_HIP(hipMalloc(&w.ctr, sizeof(byo_counters) * BYO_COUNTER_SLOTS));
  BYO_HIP(hipMalloc(&w.misc, 4096));
  BYO_HIP(hipHostMalloc(&w.h_ctr, sizeof(byo_counters) * BYO_COUNTER_SLOTS, hipHostMallocDefault));
  return BYO_OK;
}

// statistics from degree_stats_kernel's {max degree, degree-0 count, sum of
// squared degrees}
void set_degree_stats(byo_graph *g, const unsigned long long *h) {
  g->max_deg = (int64_t)h[0];
  g->isolated = (int64_t)h[1];
  g->mean_deg = 0.0;
  g->cv_deg = 0.0;
  if (g->n > 0) {
    g->mean_deg = (double)g->m / (double)g->n;
    double ex2 = (double)h[2] / (double)g->n;
    double var = std::max(0.0, ex2 - g->mean_deg * g->mean_deg);
    g->cv_deg = g->mean_deg > 0 ? std::sqrt(var) / g->mean_deg : 0.0;
  }
}

byo_status graph_refresh_stats(byo_graph *g, unsigned long long *d_tmp, hipStream_t s) {
  BYO_HIP(hipMemsetAsync(d_tmp, 0, sizeof(unsigned long long) * 8, s));
  if (g->n > 0) {
    degree_stats_kernel<<<grid_for(g->n, 256, 2048), 256, 0, s>>>(g->off, g->n, g->deg, g->zero_bits, d_tmp);
    BYO_HIP(hipGetLastError());
  }
  unsigned long long h[3] = {0, 0, 0};
  BYO_TRY(sync_read(s, d_tmp, h, sizeof(h)));
  set_degree_stats(g, h);
  return BYO_OK;
}

}  // namespace byo

using namespace byo;

// ---------------------------------------------------------------- C ABI

extern "C" {

const char *byo_last_error(void) { return g_last_error.c_str(); }

const char *byo_version(void) { return "byo-mi355x 0.1 (gfx950)"; }

void byo_opts_default(byo_opts *o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->selector = BYO_SEL_HEURISTIC;
  o->fixed_variant = BYO_V_PUSH_EDGE;
  o->dense_divisor = 20;
  o->t_wave = 32;
  o->t_block = 4096;
  o->max_levels = 0;
  o->cc_shortcut = 1;
  o->small_frontier = 0;
  o->pr_blocked = 1;   // the tile layout wherever the graph qualifies (n >= 2^16, m >= 4n)
  o->use_graph = 0;
  o->tiled = 1;
  o->persistent = 1;
}

byo_status byo_csr_from_pairs(const int32_t *src, const int32_t *dst, int64_t npairs, int64_t n, int64_t *off,
                              int32_t *nbr, int64_t *m_out) {
  BYO_CHECK(n >= 0 && n < 2147483647LL, BYO_EINVAL, "n must be in [0, 2^31-1)");
  BYO_CHECK(npairs >= 0, BYO_EINVAL, "npairs < 0");
  BYO_CHECK(off && m_out && (npairs == 0 || (src && dst && nbr)), BYO_EINVAL, "null pointer");
  for (int64_t i = 0; i < npairs; ++i)
    if (src[i] < 0 || src[i] >= n || dst[i] < 0 || dst[i] >= n)
      return fail(BYO_EINVAL, "pair " + std::to_string(i) + " has an endpoint outside [0, n)");
  unsigned T = std::max(1u, std::min(32u, std::thread::hardware_concurrency()));
  // per-thread histograms cost 8 * n bytes each: keep them under about 2 GiB
  int64_t hist_cap = std::max<int64_t>(1, (int64_t(2) << 30) / (8 * std::max<int64_t>(n, 1)));
  if ((int64_t)T > hist_cap) T = (unsigned)hist_cap;
  // 1. per-thread degree histograms over the pair ranges
  std::vector<std::vector<int64_t>> cnt(T);
  auto range = [&](unsigned t, int64_t total) {
    return std::make_pair(total * t / T, total * (t + 1) / T);
  };
  {
    std::vector<std::thread> th;
    for (unsigned t = 0; t < T; ++t)
      th.emplace_back([&, t] {
        cnt[t].assign((size_t)n, 0);
        auto r = range(t, npairs);
        for (int64_t i = r.first; i < r.second; ++i) {
          if (src[i] == dst[i]) continue;
          ++cnt[t][src[i]];
          ++cnt[t][dst[i]];
        }
      });
    for (auto &x : th) x.join();
  }
  // 2. row starts with duplicates; per-thread cursors (thread t writes after t-1)
  std::vector<int64_t> start((size_t)n + 1, 0);
  for (int64_t v = 0; v < n; ++v) {
    int64_t s = start[v];
    for (unsigned t = 0; t < T; ++t) {
      int64_t c = cnt[t][v];
      cnt[t][v] = s;
      s += c;
    }
    start[v + 1] = s;
  }
  // 3. scatter both directions into nbr (raw rows, capacity 2 * npairs)
  {
    std::vector<std::thread> th;
    for (unsigned t = 0; t < T; ++t)
      th.emplace_back([&, t] {
        auto r = range(t, npairs);
        auto &cur = cnt[t];
        for (int64_t i = r.first; i < r.second; ++i) {
          int32_t a = src[i], b = dst[i];
          if (a == b) continue;
          nbr[cur[a]++] = b;
          nbr[cur[b]++] = a;
        }
      });
    for (auto &x : th) x.join();
  }
  cnt.clear();
  cnt.shrink_to_fit();
  // 4. sort + unique each row in place; record unique lengths
  std::vector<int64_t> ulen((size_t)n, 0);
  {
    std::vector<std::thread> th;
    for (unsigned t = 0; t < T; ++t)
      th.emplace_back([&, t] {
        for (int64_t v = t; v < n; v += T) {
          int32_t *b = nbr + start[v], *e = nbr + start[v + 1];
          std::sort(b, e);
          ulen[v] = std::unique(b, e) - b;
        }
      });
    for (auto &x : th) x.join();
  }
  // 5. compact rows to the front (sequential, in order: reads never trail writes)
  int64_t pos = 0;
  for (int64_t v = 0; v < n; ++v) {
    off[v] = pos;
    if (pos != start[v]) std::memmove(nbr + pos, nbr + start[v], sizeof(int32_t) * (size_t)ulen[v]);
    pos += ulen[v];
  }
  off[n] = pos;
  *m_out = pos;
  return BYO_OK;
}

byo_status byo_graph_from_csr(const int64_t *off, const int32_t *nbr, int64_t n, int64_t m, uint32_t flags,
                              void *stream, byo_graph **out) {
  BYO_CHECK(out, BYO_EINVAL, "out is null");
  BYO_CHECK(n >= 0 && n < 2147483647LL, BYO_EINVAL, "n must be in [0, 2^31-1)");
  BYO_CHECK(m >= 0, BYO_EINVAL, "m < 0");
  BYO_CHECK(off && (m == 0 || nbr), BYO_EINVAL, "null CSR pointer");
  int modes = !!(flags & BYO_HOST_INPUT) + !!(flags & BYO_DEVICE_COPY) + !!(flags & BYO_DEVICE_BORROW);
  BYO_CHECK(modes == 1, BYO_EINVAL, "exactly one of HOST_INPUT, DEVICE_COPY, DEVICE_BORROW");
  hipStream_t s = (hipStream_t)stream;
  if (flags & BYO_HOST_INPUT) {
    BYO_CHECK(off[0] == 0 && off[n] == m, BYO_EINVAL, "host offsets must start at 0 and end at m");
  }
  byo_graph *g = new byo_graph();
  g->n = n;
  g->m = m;
  BYO_HIP(hipGetDevice(&g->device));
  auto cleanup = [&](byo_status st) {
    if (g->owns_csr) {
      if (g->off) (void)hipFree(g->off);
      if (g->nbr) (void)hipFree(g->nbr);
    }
    if (g->deg) (void)hipFree(g->deg);
    if (g->zero_bits) (void)hipFree(g->zero_bits);
    delete g;
    return st;
  };
  if (flags & BYO_DEVICE_BORROW) {
    g->off = const_cast<int64_t *>(off);
    g->nbr = const_cast<int32_t *>(nbr);
  } else {
    g->owns_csr = true;
    hipMemcpyKind kind = (flags & BYO_HOST_INPUT) ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
    hipError_t e = hipMalloc(&g->off, sizeof(int64_t) * (size_t)(n + 1));
    if (e == hipSuccess) e = hipMalloc(&g->nbr, sizeof(int32_t) * (size_t)std::max<int64_t>(m, 1));
    if (e == hipSuccess) e = hipMemcpyAsync(g->off, off, sizeof(int64_t) * (size_t)(n + 1), kind, s);
    if (e == hipSuccess && m > 0) e = hipMemcpyAsync(g->nbr, nbr, sizeof(int32_t) * (size_t)m, kind, s);
    if (e != hipSuccess) return cleanup(hip_fail(e, "CSR upload", __FILE__, __LINE__));
  }
  hipError_t e = hipMalloc(&g->deg, sizeof(int32_t) * (size_t)std::max<int64_t>(n, 1));
  if (e != hipSuccess) return cleanup(hip_fail(e, "hipMalloc(deg)", __FILE__, __LINE__));
  unsigned long long *d_tmp = nullptr;
  e = hipMalloc(&d_tmp, sizeof(unsigned long long) * 8);
  if (e != hipSuccess) return cleanup(hip_fail(e, "hipMalloc(tmp)", __FILE__, __LINE__));
  unsigned long long h_tmp[8] = {0};
  auto done = [&](byo_status st) {
    (void)hipFree(d_tmp);
    return st == BYO_OK ? st : cleanup(st);
  };
  e = hipMemsetAsync(d_tmp, 0, sizeof(unsigned long long) * 8, s);
  if (e != hipSuccess) return done(hip_fail(e, "hipMemsetAsync", __FILE__, __LINE__));
  if (flags & BYO_VALIDATE) {
    validate_offsets_kernel<<<grid_for(n + 1, 256, 1 << 30), 256, 0, s>>>(g->off, n, m, d_tmp + 3);
    e = hipMemcpyAsync(h_tmp, d_tmp, sizeof(h_tmp), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return done(hip_fail(e, "validate offsets", __FILE__, __LINE__));
    if (h_tmp[3]) return done(fail(BYO_EINVAL, "CSR offsets malformed (" + std::to_string(h_tmp[3]) + " bad)"));
    if (n > 0) validate_rows_kernel<<<grid_for(n * BYO_WAVE, 256, 16384), 256, 0, s>>>(g->off, g->nbr, n, 1, d_tmp + 4);
  }
  e = hipMalloc(&g->zero_bits, sizeof(uint64_t) * (size_t)std::max<int64_t>((n + 63) / 64, 1));
  if (e != hipSuccess) return done(hip_fail(e, "hipMalloc(zero_bits)", __FILE__, __LINE__));
  if (n > 0) degree_stats_kernel<<<grid_for(n, 256, 2048), 256, 0, s>>>(g->off, n, g->deg, g->zero_bits, d_tmp);
  e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpyAsync(h_tmp, d_tmp, sizeof(h_tmp), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return done(hip_fail(e, "graph stats", __FILE__, __LINE__));
  if ((flags & BYO_VALIDATE) && h_tmp[4])
    return done(fail(BYO_EINVAL, "CSR rows malformed: " + std::to_string(h_tmp[4]) +
                                     " entries out of range, unsorted, repeated, self-loops or asymmetric"));
  set_degree_stats(g, h_tmp);
  g->nbr_cap = m;
  *out = g;
  return done(BYO_OK);
}

void byo_graph_destroy(byo_graph *g) {
  if (!g) return;
  (void)hipDeviceSynchronize();
  ws_free(g->ws);
  if (g->owns_csr) {
    if (g->off) (void)hipFree(g->off);
    if (g->nbr) (void)hipFree(g->nbr);
  }
  if (g->deg) (void)hipFree(g->deg);
  if (g->zero_bits) (void)hipFree(g->zero_bits);
  if (g->spare_off) (void)hipFree(g->spare_off);
  if (g->spare_nbr) (void)hipFree(g->spare_nbr);
  upd_free(g->upd);
  delete g;
}

int64_t byo_num_vertices(const byo_graph *g) {
  if (!g) { set_error("null graph"); return -1; }
  return g->n;
}
int64_t byo_num_edges(const byo_graph *g) {
  if (!g) { set_error("null graph"); return -1; }
  return g->m;
}

byo_status byo_degree(const byo_graph *g, int64_t v, int64_t *out) {
  BYO_CHECK(g && out, BYO_EINVAL, "null argument");
  BYO_CHECK(v >= 0 && v < g->n, BYO_EINVAL, "vertex out of range");
  int32_t d = 0;
  BYO_HIP(hipMemcpy(&d, g->deg + v, sizeof(int32_t), hipMemcpyDeviceToHost));
  *out = d;
  return BYO_OK;
}

byo_status byo_get_neighbors(const byo_graph *g, int64_t v, int32_t *h_buf, int64_t cap, int64_t *count) {
  BYO_CHECK(g && count && (cap == 0 || h_buf), BYO_EINVAL, "null argument");
  BYO_CHECK(v >= 0 && v < g->n, BYO_EINVAL, "vertex out of range");
  int64_t se[2];
  BYO_HIP(hipMemcpy(se, g->off + v, sizeof(se), hipMemcpyDeviceToHost));
  int64_t d = se[1] - se[0];
  int64_t k = std::min(d, cap);
  if (k > 0) BYO_HIP(hipMemcpy(h_buf, g->nbr + se[0], sizeof(int32_t) * (size_t)k, hipMemcpyDeviceToHost));
  *count = d;
  return BYO_OK;
}

byo_status byo_graph_arrays(const byo_graph *g, const int64_t **d_off, const int32_t **d_nbr,
                            const int32_t **d_deg) {
  BYO_CHECK(g, BYO_EINVAL, "null graph");
  if (d_off) *d_off = g->off;
  if (d_nbr) *d_nbr = g->nbr;
  if (d_deg) *d_deg = g->deg;
  return BYO_OK;
}

byo_status byo_graph_copy(const byo_graph *g, int64_t *h_off, int32_t *h_nbr) {
  BYO_CHECK(g && h_off && (g->m == 0 || h_nbr), BYO_EINVAL, "null argument");
  BYO_HIP(hipDeviceSynchronize());
  BYO_HIP(hipMemcpy(h_off, g->off, sizeof(int64_t) * (size_t)(g->n + 1), hipMemcpyDeviceToHost));
  if (g->m > 0) BYO_HIP(hipMemcpy(h_nbr, g->nbr, sizeof(int32_t) * (size_t)g->m, hipMemcpyDeviceToHost));
  return BYO_OK;
}

byo_status byo_graph_stats(const byo_graph *g, int64_t *max_deg, int64_t *isolated, double *mean, double *cv) {
  BYO_CHECK(g, BYO_EINVAL, "null graph");
  if (max_deg) *max_deg = g->max_deg;
  if (isolated) *isolated = g->isolated;
  if (mean) *mean = g->mean_deg;
  if (cv) *cv = g->cv_deg;
  return BYO_OK;
}

}  // extern "C"
