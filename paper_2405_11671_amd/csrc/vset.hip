// vertexSubset (paper Section 3.2 "VertexSubsets"): a sparse ID list or a
// dense bit array (the bit array replaces GBBS's bool array, Section 4.4),
// with conversions. Dense -> sparse compaction is a three-pass scan
// (per-block popcount, scan of block totals, per-block write) that emits IDs
// in ascending order without any sort (Section 4.4 drops the extra sorts).
#include <algorithm>

#include "internal.h"

namespace byo {

// Compaction geometry: 256 threads x 4 words = 1024 words (65536 vertices) per block.
constexpr int CB_THREADS = 256;
constexpr int CB_WPT = 4;
constexpr int CB_WORDS = CB_THREADS * CB_WPT;

int64_t compaction_blocks(int64_t words) { return std::max<int64_t>(1, (words + CB_WORDS - 1) / CB_WORDS); }

// Block-wide exclusive scan for 256 threads; returns the exclusive prefix and
// the block total in *total. All threads must call it.
template <typename T>
__device__ __forceinline__ T block_exclusive_scan_256(T v, T *total) {
  __shared__ T wsum[CB_THREADS / BYO_WAVE];
  T inc = v;
#pragma unroll
  for (int o = 1; o < BYO_WAVE; o <<= 1) {
    T t = __shfl_up(inc, o);
    if (lane_id() >= o) inc += t;
  }
  int w = threadIdx.x / BYO_WAVE;
  __syncthreads();
  if (lane_id() == BYO_WAVE - 1) wsum[w] = inc;
  __syncthreads();
  T before = 0, all = 0;
#pragma unroll
  for (int i = 0; i < CB_THREADS / BYO_WAVE; ++i) {
    if (i < w) before += wsum[i];
    all += wsum[i];
  }
  *total = all;
  return before + inc - v;
}

__device__ __forceinline__ uint64_t masked_word(const uint64_t *bits, int64_t w, int64_t words, int64_t n) {
  if (w >= words) return 0ull;
  uint64_t b = bits[w];
  if (w == words - 1 && (n & 63)) b &= (~0ull >> (64 - (n & 63)));
  return b;
}

__global__ void __launch_bounds__(CB_THREADS) compact_count_kernel(const uint64_t *__restrict__ bits, int64_t words,
                                                                   int64_t n, long long *__restrict__ partial) {
  int64_t w0 = (int64_t)blockIdx.x * CB_WORDS + threadIdx.x * CB_WPT;
  long long c = 0;
#pragma unroll
  for (int j = 0; j < CB_WPT; ++j) c += __popcll(masked_word(bits, w0 + j, words, n));
  long long t = block_sum<long long, CB_THREADS>(c);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

// Exclusive scan of partial[0..nb) in place by one block; total to *count (and partial[nb]).
__global__ void __launch_bounds__(CB_THREADS) scan_partials_kernel(long long *__restrict__ partial, int64_t nb,
                                                                   unsigned long long *__restrict__ count) {
  long long carry = 0;
  for (int64_t base = 0; base < nb; base += CB_THREADS) {
    int64_t i = base + threadIdx.x;
    long long v = (i < nb) ? partial[i] : 0;
    long long tot;
    long long ex = block_exclusive_scan_256(v, &tot);
    if (i < nb) partial[i] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) {
    partial[nb] = carry;
    if (count) *count = (unsigned long long)carry;
  }
}

__global__ void __launch_bounds__(CB_THREADS) compact_write_kernel(const uint64_t *__restrict__ bits, int64_t words,
                                                                   int64_t n, const long long *__restrict__ partial,
                                                                   int32_t *__restrict__ ids) {
  int64_t w0 = (int64_t)blockIdx.x * CB_WORDS + threadIdx.x * CB_WPT;
  uint64_t b[CB_WPT];
  long long c = 0;
#pragma unroll
  for (int j = 0; j < CB_WPT; ++j) {
    b[j] = masked_word(bits, w0 + j, words, n);
    c += __popcll(b[j]);
  }
  long long tot;
  long long pos = partial[blockIdx.x] + block_exclusive_scan_256(c, &tot);
#pragma unroll
  for (int j = 0; j < CB_WPT; ++j) {
    uint64_t x = b[j];
    while (x) {
      int bit = __ffsll((long long)x) - 1;
      ids[pos++] = (int32_t)((w0 + j) * 64 + bit);
      x &= x - 1;
    }
  }
}

byo_status bitmap_to_ids(const uint64_t *bits, int64_t words, int64_t n, int32_t *ids, long long *partial,
                         int64_t partial_cap, unsigned long long *d_count, hipStream_t s) {
  int64_t nb = compaction_blocks(words);
  BYO_CHECK(nb + 1 <= partial_cap, BYO_EINVAL, "compaction scratch too small");
  ktimer_scope kt(BYO_K_COMPACT, s);
  compact_count_kernel<<<(unsigned)nb, CB_THREADS, 0, s>>>(bits, words, n, partial);
  scan_partials_kernel<<<1, CB_THREADS, 0, s>>>(partial, nb, d_count);
  compact_write_kernel<<<(unsigned)nb, CB_THREADS, 0, s>>>(bits, words, n, partial, ids);
  BYO_HIP(hipGetLastError());
  return BYO_OK;
}

__global__ void ids_to_bitmap_kernel(const int32_t *__restrict__ ids, int64_t k, uint64_t *__restrict__ bits) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < k) {
    int32_t v = ids[i];
    atomicOr((unsigned long long *)&bits[v >> 6], 1ull << (v & 63));
  }
}

byo_status bitmap_clear(uint64_t *bits, int64_t words, hipStream_t s) { return fill_u64(bits, words, 0ull, s); }

byo_status ids_to_bitmap(const int32_t *ids, int64_t k, uint64_t *bits, int64_t words, hipStream_t s) {
  BYO_TRY(bitmap_clear(bits, words, s));
  if (k > 0) ids_to_bitmap_kernel<<<(unsigned)((k + 255) / 256), 256, 0, s>>>(ids, k, bits);
  BYO_HIP(hipGetLastError());
  return BYO_OK;
}

// ---------------------------------------------------------------- frontier degree scan

constexpr int DS_ITEMS = 8;
constexpr int DS_TILE = CB_THREADS * DS_ITEMS;  // 2048 frontier entries per block

// units of a list of d entries: d itself (per = 1), or its blocks of `per`
__device__ __forceinline__ long long deg_units(int32_t d, int32_t per) {
  return per == 1 ? (long long)d : (long long)((d + per - 1) / per);
}

__global__ void __launch_bounds__(CB_THREADS) deg_scan_reduce_kernel(const int32_t *__restrict__ ids, int64_t k,
                                                                     const int32_t *__restrict__ deg, int32_t per,
                                                                     long long *__restrict__ partial) {
  int64_t i0 = (int64_t)blockIdx.x * DS_TILE;
  long long c = 0;
#pragma unroll
  for (int j = 0; j < DS_ITEMS; ++j) {
    int64_t i = i0 + j * CB_THREADS + threadIdx.x;
    if (i < k) c += deg_units(deg[ids[i]], per);
  }
  long long t = block_sum<long long, CB_THREADS>(c);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

__global__ void __launch_bounds__(CB_THREADS) deg_scan_write_kernel(const int32_t *__restrict__ ids, int64_t k,
                                                                    const int32_t *__restrict__ deg, int32_t per,
                                                                    const long long *__restrict__ partial,
                                                                    int64_t nb, long long *__restrict__ scan) {
  // each thread owns DS_ITEMS consecutive entries
  int64_t i0 = (int64_t)blockIdx.x * DS_TILE + (int64_t)threadIdx.x * DS_ITEMS;
  long long d[DS_ITEMS];
  long long c = 0;
#pragma unroll
  for (int j = 0; j < DS_ITEMS; ++j) {
    d[j] = (i0 + j < k) ? deg_units(deg[ids[i0 + j]], per) : 0;
    c += d[j];
  }
  long long tot;
  long long pos = partial[blockIdx.x] + block_exclusive_scan_256(c, &tot);
#pragma unroll
  for (int j = 0; j < DS_ITEMS; ++j) {
    if (i0 + j < k) scan[i0 + j] = pos;
    pos += d[j];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) scan[k] = partial[nb];
}

// The same for a frontier of at most DS_TILE entries: one workgroup, one launch.
__global__ void __launch_bounds__(CB_THREADS) deg_scan_single_kernel(const int32_t *__restrict__ ids, int64_t k,
                                                                     const int32_t *__restrict__ deg, int32_t per,
                                                                     long long *__restrict__ scan) {
  const int64_t i0 = (int64_t)threadIdx.x * DS_ITEMS;
  long long d[DS_ITEMS];
  long long c = 0;
#pragma unroll
  for (int j = 0; j < DS_ITEMS; ++j) {
    d[j] = (i0 + j < k) ? deg_units(deg[ids[i0 + j]], per) : 0;
    c += d[j];
  }
  long long tot;
  long long pos = block_exclusive_scan_256(c, &tot);
#pragma unroll
  for (int j = 0; j < DS_ITEMS; ++j) {
    if (i0 + j < k) scan[i0 + j] = pos;
    pos += d[j];
  }
  if (threadIdx.x == 0) scan[k] = tot;
}

int64_t scan_partials_needed(int64_t k) { return std::max<int64_t>(1, (k + DS_TILE - 1) / DS_TILE) + 1; }

byo_status scan_degree_units(const int32_t *deg, const int32_t *ids, int64_t k, int32_t per, long long *scan,
                             long long *partial, int64_t partial_cap, hipStream_t s) {
  BYO_CHECK(per >= 1, BYO_EINVAL, "bad unit size");
  if (k <= DS_TILE) {
    deg_scan_single_kernel<<<1, CB_THREADS, 0, s>>>(ids, k, deg, per, scan);
    BYO_HIP(hipGetLastError());
    return BYO_OK;
  }
  int64_t nb = std::max<int64_t>(1, (k + DS_TILE - 1) / DS_TILE);
  BYO_CHECK(nb + 1 <= partial_cap, BYO_EINVAL, "scan scratch too small");
  deg_scan_reduce_kernel<<<(unsigned)nb, CB_THREADS, 0, s>>>(ids, k, deg, per, partial);
  scan_partials_kernel<<<1, CB_THREADS, 0, s>>>(partial, nb, nullptr);
  deg_scan_write_kernel<<<(unsigned)nb, CB_THREADS, 0, s>>>(ids, k, deg, per, partial, nb, scan);
  BYO_HIP(hipGetLastError());
  return BYO_OK;
}

byo_status scan_degrees(const int32_t *deg, const int32_t *ids, int64_t k, long long *scan, long long *partial,
                        int64_t partial_cap, hipStream_t s) {
  return scan_degree_units(deg, ids, k, 1, scan, partial, partial_cap, s);
}

byo_status frontier_degree_scan(const byo_graph *g, const int32_t *ids, int64_t k, long long *scan,
                                long long *partial, int64_t partial_cap, hipStream_t s) {
  return scan_degrees(g->deg, ids, k, scan, partial, partial_cap, s);
}

__global__ void ids_range_check_kernel(const int32_t *__restrict__ ids, int64_t k, int64_t n,
                                       unsigned long long *__restrict__ bad) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < k && (ids[i] < 0 || ids[i] >= n)) atomicAdd(bad, 1ull);
}

__global__ void bitmap_mask_tail_kernel(uint64_t *bits, int64_t words, int64_t n) {
  if (threadIdx.x == 0 && (n & 63)) bits[words - 1] &= (~0ull >> (64 - (n & 63)));
}

}  // namespace byo

using namespace byo;

// ---------------------------------------------------------------- C ABI

extern "C" {

byo_status byo_vset_create(const byo_graph *g, byo_vset **out) {
  BYO_CHECK(g && out, BYO_EINVAL, "null argument");
  byo_vset *s = new byo_vset();
  s->g = g;
  s->n = g->n;
  s->words = (g->n + 63) / 64;
  size_t wb = sizeof(uint64_t) * (size_t)std::max<int64_t>(s->words, 1);
  size_t ib = sizeof(int32_t) * (size_t)std::max<int64_t>(s->n, 1);
  hipError_t e = hipMalloc(&s->ids, ib);
  if (e == hipSuccess) e = hipMalloc(&s->bits, wb);
  if (e == hipSuccess) e = hipMalloc(&s->d_tmp, sizeof(unsigned long long) * 4);
  if (e != hipSuccess) {
    if (s->ids) (void)hipFree(s->ids);
    if (s->bits) (void)hipFree(s->bits);
    delete s;
    return hip_fail(e, "vset allocation", __FILE__, __LINE__);
  }
  s->sparse_valid = true;  // empty list
  s->count = 0;
  *out = s;
  return BYO_OK;
}

void byo_vset_destroy(byo_vset *s) {
  if (!s) return;
  (void)hipDeviceSynchronize();
  if (s->ids) (void)hipFree(s->ids);
  if (s->bits) (void)hipFree(s->bits);
  if (s->d_tmp) (void)hipFree(s->d_tmp);
  delete s;
}

byo_status byo_vset_from_ids(byo_vset *s, const int32_t *d_ids, int64_t k, void *stream) {
  BYO_CHECK(s && (k == 0 || d_ids), BYO_EINVAL, "null argument");
  BYO_CHECK(k >= 0 && k <= s->n, BYO_EINVAL, "k out of range");
  hipStream_t st = (hipStream_t)stream;
  if (k > 0) {
    BYO_HIP(hipMemcpyAsync(s->ids, d_ids, sizeof(int32_t) * (size_t)k, hipMemcpyDeviceToDevice, st));
    BYO_HIP(hipMemsetAsync(s->d_tmp, 0, sizeof(unsigned long long), st));
    ids_range_check_kernel<<<(unsigned)((k + 255) / 256), 256, 0, st>>>(s->ids, k, s->n, s->d_tmp);
    BYO_HIP(hipGetLastError());
    unsigned long long bad = 0;
    BYO_TRY(sync_read(st, s->d_tmp, &bad, sizeof(bad)));
    BYO_CHECK(bad == 0, BYO_EINVAL, "vertex IDs outside [0, n)");
  }
  s->count = k;
  s->sparse_valid = true;
  s->dense_valid = false;
  return BYO_OK;
}

byo_status byo_vset_from_bitmap(byo_vset *s, const uint64_t *d_bits, void *stream) {
  BYO_CHECK(s && d_bits, BYO_EINVAL, "null argument");
  hipStream_t st = (hipStream_t)stream;
  if (s->words > 0) {
    BYO_HIP(hipMemcpyAsync(s->bits, d_bits, sizeof(uint64_t) * (size_t)s->words, hipMemcpyDeviceToDevice, st));
    bitmap_mask_tail_kernel<<<1, 64, 0, st>>>(s->bits, s->words, s->n);
    BYO_HIP(hipGetLastError());
  }
  // count via the compaction's first two passes
  byo_graph *g = const_cast<byo_graph *>(s->g);
  BYO_TRY(ws_ensure_traversal(g));
  BYO_TRY(bitmap_to_ids(s->bits, s->words, s->n, s->ids, g->ws.partial, g->ws.partial_cap, s->d_tmp, st));
  unsigned long long c = 0;
  BYO_TRY(sync_read(st, s->d_tmp, &c, sizeof(c)));
  s->count = (int64_t)c;
  s->dense_valid = true;
  s->sparse_valid = true;
  return BYO_OK;
}

byo_status byo_vset_fill(byo_vset *s, void *stream) {
  BYO_CHECK(s, BYO_EINVAL, "null argument");
  hipStream_t st = (hipStream_t)stream;
  BYO_TRY(fill_u64(s->bits, s->words, ~0ull, st));
  if (s->words > 0) bitmap_mask_tail_kernel<<<1, 64, 0, st>>>(s->bits, s->words, s->n);
  BYO_HIP(hipGetLastError());
  s->count = s->n;
  s->dense_valid = true;
  s->sparse_valid = false;
  return BYO_OK;
}

byo_status byo_vset_size(byo_vset *s, int64_t *out, void *stream) {
  (void)stream;
  BYO_CHECK(s && out, BYO_EINVAL, "null argument");
  *out = s->count;
  return BYO_OK;
}

byo_status byo_vset_to_ids(byo_vset *s, int32_t *d_ids, int64_t cap, int64_t *k, void *stream) {
  BYO_CHECK(s && k && (cap == 0 || d_ids), BYO_EINVAL, "null argument");
  BYO_CHECK(cap >= s->count, BYO_EINVAL, "capacity smaller than the subset");
  hipStream_t st = (hipStream_t)stream;
  byo_graph *g = const_cast<byo_graph *>(s->g);
  BYO_TRY(ws_ensure_traversal(g));
  // ascending order: go through the dense form
  if (!s->dense_valid) {
    BYO_TRY(ids_to_bitmap(s->ids, s->count, s->bits, s->words, st));
    s->dense_valid = true;
  }
  BYO_TRY(bitmap_to_ids(s->bits, s->words, s->n, s->ids, g->ws.partial, g->ws.partial_cap, s->d_tmp, st));
  s->sparse_valid = true;
  if (s->count > 0)
    BYO_HIP(hipMemcpyAsync(d_ids, s->ids, sizeof(int32_t) * (size_t)s->count, hipMemcpyDeviceToDevice, st));
  BYO_HIP(hipStreamSynchronize(st));
  *k = s->count;
  return BYO_OK;
}

byo_status byo_vset_to_bitmap(byo_vset *s, uint64_t *d_bits, void *stream) {
  BYO_CHECK(s && d_bits, BYO_EINVAL, "null argument");
  hipStream_t st = (hipStream_t)stream;
  if (!s->dense_valid) {
    BYO_TRY(ids_to_bitmap(s->ids, s->count, s->bits, s->words, st));
    s->dense_valid = true;
  }
  if (s->words > 0)
    BYO_HIP(hipMemcpyAsync(d_bits, s->bits, sizeof(uint64_t) * (size_t)s->words, hipMemcpyDeviceToDevice, st));
  return BYO_OK;
}

}  // extern "C"
