// Batch edge updates of the CSR container, and the three batch forms.
//
// The paper's dynamic containers take batches of edge insertions and
// deletions: at set level insert_batch / delete_batch, at container level
// insert_sorted_batch / delete_sorted_batch, the framework sorting the batch
// first because most batch-update algorithms want it sorted (Section 4.1,
// "Translating graph batch-update API into the set API"; Section 4.2,
// "Required functionality for updates"). It prepares a batch in one of three
// forms: a global sort, a semisort (equal sources together), or a semisort
// whose groups are each sorted by target.
//
// Reading of the batch: each pair (u, v) with u != v names the undirected
// edge {u, v}, so both directions change together and the container stays
// symmetric and simple; self-pairs change nothing; repeated pairs act once.
//
// The container here is the packed CSR that every traversal reads, so a
// batch is applied as a merge into a second pair of arrays:
//  1. keys (u << 32) | v for both directions of every pair, self-pairs as a
//     sentinel that sorts last, radix-sorted (the global-sort form);
//  2. a key is kept if it is the first of its run and, for an insert, not yet
//     an edge (for a delete, an edge): a binary search in its row;
//  3. the kept keys K are compacted by a scan (sorted, unique);
//  4. kr[u] = number of keys of K with source below u, by binary search, and
//     the new offsets off'[u] = off[u] + kr[u] (insert) or - kr[u] (delete);
//  5. every old entry moves to its new place, shifted by the keys of K in
//     its row that precede it (dropped if it is one, for a delete), and for
//     an insert every key of K goes to its place among its row's old entries.
// Rows stay sorted, so the result is the set union (difference) and every
// kernel of the library reads it as before. The arrays the update wrote
// become the graph's; the previous ones are kept for the next update.
#include <algorithm>
#include <vector>

#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>

#include "internal.h"

namespace byo {
namespace {

constexpr int UP_THREADS = 256;
constexpr int UP_SLICE = 2048;           // old entries per workgroup of the move kernel
constexpr int UP_ROWS = UP_SLICE + 1;    // row offsets staged in LDS per slice
constexpr uint64_t UP_NONE = ~0ull;      // self-pair / out-of-range sentinel key

unsigned up_blocks(int64_t count, int64_t cap = 1 << 16) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>((count + UP_THREADS - 1) / UP_THREADS, cap));
}

int up_bits(int64_t x) {  // bits needed to hold 0 .. x
  int b = 1;
  while (b < 62 && (x >> b) != 0) ++b;
  return b;
}

__device__ __forceinline__ uint64_t up_key(int64_t u, int64_t v) { return ((uint64_t)u << 32) | (uint64_t)v; }

// first index in [lo, hi) of a sorted key array whose key is >= x
__device__ __forceinline__ int64_t up_lower(const uint64_t *__restrict__ a, int64_t lo, int64_t hi, uint64_t x) {
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (a[mid] < x) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// first index in [lo, hi) of a sorted neighbour list whose value is >= x
__device__ __forceinline__ int64_t up_lower_nbr(const int32_t *__restrict__ a, int64_t lo, int64_t hi, int32_t x) {
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (a[mid] < x) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// Both directions of every pair as keys; self-pairs and pairs naming a
// vertex outside [0, n) become the sentinel, and the latter set *bad.
__global__ void up_keys_kernel(const int32_t *__restrict__ src, const int32_t *__restrict__ dst, int64_t k, int64_t n,
                               uint64_t *__restrict__ keys, unsigned int *__restrict__ bad) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < k; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t s = src[i], d = dst[i];
    const bool out = s < 0 || s >= n || d < 0 || d >= n;
    if (__any(out) && lane_id() == 0) atomicOr(bad, 1u);
    const bool skip = out || s == d;
    keys[2 * i] = skip ? UP_NONE : up_key(s, d);
    keys[2 * i + 1] = skip ? UP_NONE : up_key(d, s);
  }
}

// flag[i] = 1 for the first key of each run of equal keys that is not the
// sentinel and whose presence in the graph equals want_present; flag[cnt] = 0
// so that the exclusive scan's last element is the total.
__global__ void up_flag_kernel(const uint64_t *__restrict__ keys, int64_t cnt, const int64_t *__restrict__ off,
                               const int32_t *__restrict__ nbr, int want_present, uint32_t *__restrict__ flag) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= cnt; i += (int64_t)gridDim.x * blockDim.x) {
    uint32_t keep = 0;
    if (i < cnt) {
      const uint64_t x = keys[i];
      if (x != UP_NONE && (i == 0 || keys[i - 1] != x)) {
        const int64_t u = (int64_t)(x >> 32);
        const int32_t v = (int32_t)(x & 0xffffffffu);
        const int64_t b = off[u], e = off[u + 1];
        const int64_t p = up_lower_nbr(nbr, b, e, v);
        const int present = p < e && nbr[p] == v;
        keep = present == want_present;
      }
    }
    flag[i] = keep;
  }
}

__global__ void up_compact_kernel(const uint64_t *__restrict__ keys, const uint32_t *__restrict__ flag,
                                  const int64_t *__restrict__ pos, int64_t cnt, uint64_t *__restrict__ K) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += (int64_t)gridDim.x * blockDim.x)
    if (flag[i]) K[pos[i]] = keys[i];
}

// kr[u] = keys of K with source below u (u in [0, n]); the new offsets.
__global__ void up_rows_kernel(const uint64_t *__restrict__ K, int64_t kc, const int64_t *__restrict__ off, int64_t n,
                               int64_t sign, int64_t *__restrict__ kr, int64_t *__restrict__ off2) {
  for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u <= n; u += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = up_lower(K, 0, kc, (uint64_t)u << 32);
    kr[u] = r;
    off2[u] = off[u] + sign * r;
  }
}

// Old entries to their new places. A workgroup takes UP_SLICE consecutive
// entries; the row of each is the last row whose offset is <= its index,
// searched among the slice's row offsets staged in LDS (or in global memory
// when the slice spans more rows than that, i.e. many empty rows).
template <bool INSERT>
__global__ void __launch_bounds__(UP_THREADS) up_move_kernel(const int64_t *__restrict__ off,
                                                             const int32_t *__restrict__ nbr, int64_t n, int64_t m,
                                                             const uint64_t *__restrict__ K,
                                                             const int64_t *__restrict__ kr,
                                                             int32_t *__restrict__ nbr2) {
  __shared__ int64_t soff[UP_ROWS];
  __shared__ int64_t sr[2];
  const int64_t i0 = (int64_t)blockIdx.x * UP_SLICE;
  if (i0 >= m) return;
  const int64_t i1 = std::min<int64_t>(m, i0 + UP_SLICE);
  if (threadIdx.x == 0) {
    // r0 = the row holding entry i0: the last r with off[r] <= i0
    int64_t lo = 0, hi = n;  // invariant: off[lo] <= i0, answer in [lo, hi)
    while (hi - lo > 1) {
      const int64_t mid = (lo + hi) >> 1;
      if (off[mid] <= i0) lo = mid;
      else hi = mid;
    }
    sr[0] = lo;
  }
  __syncthreads();
  const int64_t r0 = sr[0];
  const int64_t nr = std::min<int64_t>(UP_ROWS, n + 1 - r0);
  for (int64_t j = threadIdx.x; j < nr; j += UP_THREADS) soff[j] = off[r0 + j];
  __syncthreads();
  // the staged offsets cover the slice when the last staged offset lies past it
  const bool staged = soff[nr - 1] >= i1;
  for (int64_t i = i0 + threadIdx.x; i < i1; i += UP_THREADS) {
    int64_t u;
    if (staged) {
      int64_t lo = 0, hi = nr - 1;
      while (hi - lo > 1) {
        const int64_t mid = (lo + hi) >> 1;
        if (soff[mid] <= i) lo = mid;
        else hi = mid;
      }
      u = r0 + lo;
    } else {
      int64_t lo = r0, hi = n;
      while (hi - lo > 1) {
        const int64_t mid = (lo + hi) >> 1;
        if (off[mid] <= i) lo = mid;
        else hi = mid;
      }
      u = lo;
    }
    const int32_t v = nbr[i];
    const int64_t a = kr[u], b = kr[u + 1];
    const int64_t j = i - off[u];
    if (INSERT) {
      const int64_t before = a == b ? 0 : up_lower(K, a, b, up_key(u, v)) - a;
      nbr2[off[u] + a + j + before] = v;
    } else {
      if (a == b) {
        nbr2[off[u] - a + j] = v;
      } else {
        const uint64_t x = up_key(u, v);
        const int64_t p = up_lower(K, a, b, x);
        if (p < b && K[p] == x) continue;  // deleted
        nbr2[off[u] - a + j - (p - a)] = v;
      }
    }
  }
}

// Inserted keys to their places among their rows' old entries.
__global__ void up_place_kernel(const uint64_t *__restrict__ K, int64_t kc, const int64_t *__restrict__ off,
                                const int32_t *__restrict__ nbr, const int64_t *__restrict__ kr,
                                int32_t *__restrict__ nbr2) {
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < kc; q += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t x = K[q];
    const int64_t u = (int64_t)(x >> 32);
    const int32_t v = (int32_t)(x & 0xffffffffu);
    const int64_t b = off[u];
    const int64_t lt = up_lower_nbr(nbr, b, off[u + 1], v) - b;
    nbr2[b + kr[u] + (q - kr[u]) + lt] = v;
  }
}

// Per-graph buffers of the update path, grown on demand and kept.
struct upd_ws {
  int64_t key_cap = 0;
  uint64_t *keys = nullptr, *sorted = nullptr, *K = nullptr;
  uint32_t *flag = nullptr;
  int64_t *pos = nullptr;
  int64_t *kr = nullptr;      // [n + 1]
  void *tmp = nullptr;
  size_t tmp_bytes = 0;
  unsigned long long *small = nullptr;  // [8]: bad-ID flag, graph statistics
};

byo_status upd_reserve(byo_graph *g, int64_t nkeys, hipStream_t s, upd_ws **out) {
  upd_ws *w = (upd_ws *)g->upd;
  if (!w) {
    w = new upd_ws();
    g->upd = w;
  }
  if (!w->kr) {
    BYO_HIP(hipMalloc(&w->kr, sizeof(int64_t) * (size_t)(g->n + 1)));
    BYO_HIP(hipMalloc(&w->small, sizeof(unsigned long long) * 8));
  }
  if (w->key_cap < nkeys) {
    const int64_t cap = std::max<int64_t>(nkeys, 1024);
    void *old[] = {w->keys, w->sorted, w->K, w->flag, w->pos};
    for (void *p : old)
      if (p) (void)hipFree(p);
    w->keys = w->sorted = w->K = nullptr;
    w->flag = nullptr;
    w->pos = nullptr;
    w->key_cap = 0;
    BYO_HIP(hipMalloc(&w->keys, sizeof(uint64_t) * (size_t)cap));
    BYO_HIP(hipMalloc(&w->sorted, sizeof(uint64_t) * (size_t)cap));
    BYO_HIP(hipMalloc(&w->K, sizeof(uint64_t) * (size_t)cap));
    BYO_HIP(hipMalloc(&w->flag, sizeof(uint32_t) * (size_t)(cap + 1)));
    BYO_HIP(hipMalloc(&w->pos, sizeof(int64_t) * (size_t)(cap + 1)));
    w->key_cap = cap;
  }
  size_t q0 = 0, q1 = 0;
  BYO_HIP(rocprim::radix_sort_keys(nullptr, q0, w->keys, w->sorted, (size_t)w->key_cap, 0u, 64u, s));
  BYO_HIP(rocprim::exclusive_scan(nullptr, q1, w->flag, w->pos, (int64_t)0, (size_t)w->key_cap + 1,
                                  rocprim::plus<int64_t>(), s));
  const size_t need = std::max(q0, q1);
  if (w->tmp_bytes < need) {
    if (w->tmp) (void)hipFree(w->tmp);
    w->tmp = nullptr;
    w->tmp_bytes = 0;
    BYO_HIP(hipMalloc(&w->tmp, need));
    w->tmp_bytes = need;
  }
  *out = w;
  return BYO_OK;
}

byo_status apply_batch(byo_graph *g, const int32_t *d_src, const int32_t *d_dst, int64_t k, bool insert,
                       hipStream_t s, int64_t *changed) {
  BYO_CHECK(g && (k == 0 || (d_src && d_dst)), BYO_EINVAL, "null argument");
  BYO_CHECK(k >= 0 && k <= ((int64_t)1 << 40), BYO_EINVAL, "batch size out of range");
  const int64_t n = g->n, m = g->m;
  if (k == 0 || n == 0) {
    BYO_CHECK(k == 0, BYO_EINVAL, "batch names a vertex outside [0, n)");
    if (changed) *changed = 0;
    return BYO_OK;
  }
  const int64_t cnt = 2 * k;
  upd_ws *w = nullptr;
  BYO_TRY(upd_reserve(g, cnt, s, &w));
  BYO_HIP(hipMemsetAsync(w->small, 0, sizeof(unsigned long long) * 8, s));
  up_keys_kernel<<<up_blocks(k), UP_THREADS, 0, s>>>(d_src, d_dst, k, n, w->keys, (unsigned int *)w->small);
  BYO_HIP(hipGetLastError());
  size_t tb = w->tmp_bytes;
  const unsigned end_bit = (unsigned)std::min(64, 32 + up_bits(n - 1));
  BYO_HIP(rocprim::radix_sort_keys(w->tmp, tb, w->keys, w->sorted, (size_t)cnt, 0u, end_bit, s));
  up_flag_kernel<<<up_blocks(cnt + 1), UP_THREADS, 0, s>>>(w->sorted, cnt, g->off, g->nbr, insert ? 0 : 1, w->flag);
  BYO_HIP(hipGetLastError());
  tb = w->tmp_bytes;
  BYO_HIP(rocprim::exclusive_scan(w->tmp, tb, w->flag, w->pos, (int64_t)0, (size_t)cnt + 1,
                                  rocprim::plus<int64_t>(), s));
  up_compact_kernel<<<up_blocks(cnt), UP_THREADS, 0, s>>>(w->sorted, w->flag, w->pos, cnt, w->K);
  BYO_HIP(hipGetLastError());
  unsigned int bad = 0;
  int64_t kc = 0;
  BYO_TRY(sync_read(s, w->small, &bad, sizeof(bad)));
  BYO_CHECK(bad == 0, BYO_EINVAL, "batch names a vertex outside [0, n)");
  BYO_TRY(sync_read(s, w->pos + cnt, &kc, sizeof(kc)));
  if (changed) *changed = kc;
  if (kc == 0) return BYO_OK;
  const int64_t m2 = insert ? m + kc : m - kc;
  BYO_CHECK(m2 < ((int64_t)1 << 40), BYO_EINVAL, "graph too large");
  // the arrays this update writes: the spares, grown if needed
  if (!g->spare_off) BYO_HIP(hipMalloc(&g->spare_off, sizeof(int64_t) * (size_t)(n + 1)));
  if (g->spare_cap < std::max<int64_t>(m2, 1)) {
    if (g->spare_nbr) (void)hipFree(g->spare_nbr);
    g->spare_nbr = nullptr;
    g->spare_cap = 0;
    const int64_t cap = std::max<int64_t>(m2 + m2 / 8, 1024);
    BYO_HIP(hipMalloc(&g->spare_nbr, sizeof(int32_t) * (size_t)cap));
    g->spare_cap = cap;
  }
  up_rows_kernel<<<up_blocks(n + 1), UP_THREADS, 0, s>>>(w->K, kc, g->off, n, insert ? 1 : -1, w->kr, g->spare_off);
  BYO_HIP(hipGetLastError());
  if (m > 0) {
    const unsigned nb = (unsigned)((m + UP_SLICE - 1) / UP_SLICE);
    if (insert)
      up_move_kernel<true><<<nb, UP_THREADS, 0, s>>>(g->off, g->nbr, n, m, w->K, w->kr, g->spare_nbr);
    else
      up_move_kernel<false><<<nb, UP_THREADS, 0, s>>>(g->off, g->nbr, n, m, w->K, w->kr, g->spare_nbr);
    BYO_HIP(hipGetLastError());
  }
  if (insert) {
    up_place_kernel<<<up_blocks(kc), UP_THREADS, 0, s>>>(w->K, kc, g->off, g->nbr, w->kr, g->spare_nbr);
    BYO_HIP(hipGetLastError());
  }
  // the written arrays become the graph's; owned previous ones become spares
  int64_t *old_off = g->off;
  int32_t *old_nbr = g->nbr;
  const int64_t old_cap = g->nbr_cap;
  g->off = g->spare_off;
  g->nbr = g->spare_nbr;
  g->nbr_cap = g->spare_cap;
  g->m = m2;
  if (g->owns_csr) {
    g->spare_off = old_off;
    g->spare_nbr = old_nbr;
    g->spare_cap = old_cap;
  } else {
    g->spare_off = nullptr;
    g->spare_nbr = nullptr;
    g->spare_cap = 0;
    g->owns_csr = true;
  }
  // everything derived from the old structure is rebuilt on next use
  BYO_HIP(hipStreamSynchronize(s));
  ws_free(g->ws);
  return graph_refresh_stats(g, w->small, s);
}

// per-call buffers of byo_batch_order, freed once the stream's work is done
struct order_tmp {
  hipStream_t s;
  std::vector<void *> v;
  explicit order_tmp(hipStream_t st) : s(st) {}
  template <class T>
  byo_status get(T **p, size_t count) {
    *p = nullptr;
    BYO_HIP(hipMalloc((void **)p, sizeof(T) * std::max<size_t>(count, 1)));
    v.push_back(*p);
    return BYO_OK;
  }
  ~order_tmp() {
    (void)hipStreamSynchronize(s);
    for (void *x : v) (void)hipFree(x);
  }
};

__global__ void ord_check_kernel(const int32_t *__restrict__ src, const int32_t *__restrict__ dst, int64_t k,
                                 int64_t n, unsigned int *__restrict__ bad) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < k; i += (int64_t)gridDim.x * blockDim.x) {
    const bool out = src[i] < 0 || src[i] >= n || dst[i] < 0 || dst[i] >= n;
    if (__any(out) && lane_id() == 0) atomicOr(bad, 1u);
  }
}

__global__ void ord_join_kernel(const int32_t *__restrict__ src, const int32_t *__restrict__ dst, int64_t k,
                                uint64_t *__restrict__ keys) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < k; i += (int64_t)gridDim.x * blockDim.x)
    keys[i] = up_key(src[i], dst[i]);
}

__global__ void ord_split_kernel(const uint64_t *__restrict__ keys, int64_t k, int32_t *__restrict__ src,
                                 int32_t *__restrict__ dst) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < k; i += (int64_t)gridDim.x * blockDim.x) {
    src[i] = (int32_t)(keys[i] >> 32);
    dst[i] = (int32_t)(keys[i] & 0xffffffffu);
  }
}

}  // namespace

void upd_free(void *p) {
  upd_ws *w = (upd_ws *)p;
  if (!w) return;
  void *d[] = {w->keys, w->sorted, w->K, w->flag, w->pos, w->kr, w->tmp, w->small};
  for (void *x : d)
    if (x) (void)hipFree(x);
  delete w;
}

}  // namespace byo

using namespace byo;

extern "C" {

byo_status byo_graph_insert_batch(byo_graph *g, const int32_t *d_src, const int32_t *d_dst, int64_t k, void *stream,
                                  int64_t *changed) {
  return apply_batch(g, d_src, d_dst, k, true, (hipStream_t)stream, changed);
}

byo_status byo_graph_delete_batch(byo_graph *g, const int32_t *d_src, const int32_t *d_dst, int64_t k, void *stream,
                                  int64_t *changed) {
  return apply_batch(g, d_src, d_dst, k, false, (hipStream_t)stream, changed);
}

byo_status byo_batch_order(const int32_t *d_src, const int32_t *d_dst, int64_t k, int64_t n, int32_t form,
                           int32_t *d_out_src, int32_t *d_out_dst, void *stream) {
  BYO_CHECK(d_src && d_dst && d_out_src && d_out_dst, BYO_EINVAL, "null argument");
  BYO_CHECK(k >= 0 && n >= 0 && n < 2147483647LL, BYO_EINVAL, "size out of range");
  BYO_CHECK(form == BYO_FORM_SORT || form == BYO_FORM_SEMISORT || form == BYO_FORM_GROUPED_SORT, BYO_EINVAL,
            "unknown batch form");
  if (k == 0) return BYO_OK;
  hipStream_t s = (hipStream_t)stream;
  order_tmp tmp(s);
  unsigned int *bad = nullptr;
  BYO_TRY(tmp.get(&bad, 1));
  BYO_HIP(hipMemsetAsync(bad, 0, sizeof(unsigned int), s));
  ord_check_kernel<<<up_blocks(k), UP_THREADS, 0, s>>>(d_src, d_dst, k, n, bad);
  BYO_HIP(hipGetLastError());
  unsigned int h_bad = 0;
  BYO_TRY(sync_read(s, bad, &h_bad, sizeof(h_bad)));
  BYO_CHECK(h_bad == 0, BYO_EINVAL, "batch names a vertex outside [0, n)");
  const unsigned vb = (unsigned)up_bits(std::max<int64_t>(n - 1, 1));
  if (form == BYO_FORM_SORT) {
    // ascending (source, target): one radix sort of the joined keys
    uint64_t *ka = nullptr, *kb = nullptr;
    BYO_TRY(tmp.get(&ka, (size_t)k));
    BYO_TRY(tmp.get(&kb, (size_t)k));
    ord_join_kernel<<<up_blocks(k), UP_THREADS, 0, s>>>(d_src, d_dst, k, ka);
    BYO_HIP(hipGetLastError());
    size_t q = 0;
    BYO_HIP(rocprim::radix_sort_keys(nullptr, q, ka, kb, (size_t)k, 0u, 32u + vb, s));
    void *ts = nullptr;
    BYO_TRY(tmp.get((uint8_t **)&ts, q));
    BYO_HIP(rocprim::radix_sort_keys(ts, q, ka, kb, (size_t)k, 0u, 32u + vb, s));
    ord_split_kernel<<<up_blocks(k), UP_THREADS, 0, s>>>(kb, k, d_out_src, d_out_dst);
    BYO_HIP(hipGetLastError());
    return BYO_OK;
  }
  // Semisort: a stable radix sort on the source's bits alone puts equal
  // sources together (a pair keeps its input position inside its group; the
  // groups come out by source as a side effect). The grouped form first
  // orders the pairs by target, so that the stable grouping pass leaves each
  // group sorted by target.
  const uint32_t *ks = (const uint32_t *)d_src;
  const int32_t *vs = d_dst;
  size_t q = 0;
  BYO_HIP(rocprim::radix_sort_pairs(nullptr, q, (const uint32_t *)d_src, (uint32_t *)d_out_src, d_dst, d_out_dst,
                                    (size_t)k, 0u, vb, s));
  void *ts = nullptr;
  BYO_TRY(tmp.get((uint8_t **)&ts, q));
  if (form == BYO_FORM_GROUPED_SORT) {
    uint32_t *t_dst = nullptr;
    int32_t *t_src = nullptr;
    BYO_TRY(tmp.get(&t_dst, (size_t)k));
    BYO_TRY(tmp.get(&t_src, (size_t)k));
    BYO_HIP(rocprim::radix_sort_pairs(ts, q, (const uint32_t *)d_dst, t_dst, d_src, t_src, (size_t)k, 0u, vb, s));
    ks = (const uint32_t *)t_src;
    vs = (const int32_t *)t_dst;
    BYO_HIP(rocprim::radix_sort_pairs(ts, q, ks, (uint32_t *)d_out_src, vs, d_out_dst, (size_t)k, 0u, vb, s));
    return BYO_OK;
  }
  BYO_HIP(rocprim::radix_sort_pairs(ts, q, ks, (uint32_t *)d_out_src, vs, d_out_dst, (size_t)k, 0u, vb, s));
  return BYO_OK;
}

}  // extern "C"
