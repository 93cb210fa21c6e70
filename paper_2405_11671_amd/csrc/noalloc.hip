// BFS that allocates nothing: the same level loop and kernels as byo_bfs,
// with every per-run buffer (visited and frontier bitmaps, frontier lists,
// frontier degree scan, compaction partials, level counters, flags) carved
// out of one file-scope device array instead of the graph's lazily allocated
// workspace.
//
// The array lives in the library's code object, so every device the library
// runs on holds its own copy from module load until the process ends. Host
// code never passes the array's name to a kernel or a copy: the name is a
// host-side stand-in. Its device address is looked up once per device with
// hipGetSymbolAddress, with that device current, and only that address is
// used.
#include <cstring>
#include <mutex>

#include "internal.h"

namespace byo {
namespace {

constexpr size_t na_align(size_t x) { return (x + 255) & ~(size_t)255; }

constexpr int64_t NA_MAX_N = BYO_NOALLOC_MAX_N;
constexpr int64_t NA_WORDS = (NA_MAX_N + 63) / 64;
constexpr size_t NA_BITMAP = na_align(sizeof(uint64_t) * NA_WORDS);       // visited, bits[0], bits[1]
constexpr size_t NA_IDS = na_align(sizeof(int32_t) * NA_MAX_N);            // ids[0], ids[1]
constexpr size_t NA_SCAN = na_align(sizeof(long long) * (NA_MAX_N + 2));   // frontier degree scan
constexpr size_t NA_PARTIAL = 64 * 1024;                                   // scan / compaction block partials
constexpr size_t NA_CTR = na_align(sizeof(byo_counters) * BYO_COUNTER_SLOTS);
constexpr size_t NA_MISC = 4096;
constexpr size_t NA_BYTES = 3 * NA_BITMAP + 2 * NA_IDS + NA_SCAN + NA_PARTIAL + NA_CTR + NA_MISC;

}  // namespace

// The scratch array (about 34 MiB for 2^21 vertices).
static __device__ __align__(256) unsigned char scratch[NA_BYTES];

namespace {

constexpr int NA_MAX_DEVICES = 64;
std::mutex na_mu;
unsigned char *na_ptr[NA_MAX_DEVICES] = {};

// Device address of this device's copy of the scratch array, looked up on the
// first call made with `dev` current.
byo_status na_scratch(int dev, unsigned char **out) {
  BYO_CHECK(dev >= 0 && dev < NA_MAX_DEVICES, BYO_EINVAL, "device index out of range for the no-alloc BFS");
  std::lock_guard<std::mutex> lk(na_mu);
  if (!na_ptr[dev]) {
    void *p = nullptr;
    BYO_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    BYO_CHECK(p != nullptr, BYO_EHIP, "no device address for the no-alloc scratch array");
    na_ptr[dev] = (unsigned char *)p;
  }
  *out = na_ptr[dev];
  return BYO_OK;
}

// The workspace fields the host-driven BFS loop uses, laid over the scratch.
void na_layout(unsigned char *base, int64_t n, byo_workspace &w) {
  const int64_t words = (n + 63) / 64;
  size_t at = 0;
  auto take = [&](size_t bytes) {
    unsigned char *p = base + at;
    at += bytes;
    return p;
  };
  w.n = n;
  w.words = words;
  w.visited = (uint64_t *)take(NA_BITMAP);
  w.bits[0] = (uint64_t *)take(NA_BITMAP);
  w.bits[1] = (uint64_t *)take(NA_BITMAP);
  w.ids[0] = (int32_t *)take(NA_IDS);
  w.ids[1] = (int32_t *)take(NA_IDS);
  w.scan = (long long *)take(NA_SCAN);
  w.partial = (long long *)take(NA_PARTIAL);
  w.partial_cap = (int64_t)(NA_PARTIAL / sizeof(long long));
  w.ctr = (byo_counters *)take(NA_CTR);
  w.misc = (int32_t *)take(NA_MISC);
}

bool same_ptrs(const byo_workspace &a, const byo_workspace &b) {
  const void *x[] = {a.visited, a.bits[0], a.bits[1], a.ids[0], a.ids[1], a.scan, a.partial, a.ctr, a.h_ctr,
                     a.misc, a.api_deg, a.api_heavy, a.api_pre, a.api_aux, a.contrib[0], a.contrib[1], a.dpart,
                     a.base, a.heavy_rows, a.chunk_row, a.chunk_beg, a.row_chunk0, a.chunk_sum, a.ms, a.tiles[0],
                     a.tiles[1], a.tiles[2], a.cz, a.bc_coef, a.bc_sigma, a.bc_depth, a.bc_order, a.kc_dcur,
                     a.ds_deg, a.ds_alive, a.gmode, a.dloop};
  const void *y[] = {b.visited, b.bits[0], b.bits[1], b.ids[0], b.ids[1], b.scan, b.partial, b.ctr, b.h_ctr,
                     b.misc, b.api_deg, b.api_heavy, b.api_pre, b.api_aux, b.contrib[0], b.contrib[1], b.dpart,
                     b.base, b.heavy_rows, b.chunk_row, b.chunk_beg, b.row_chunk0, b.chunk_sum, b.ms, b.tiles[0],
                     b.tiles[1], b.tiles[2], b.cz, b.bc_coef, b.bc_sigma, b.bc_depth, b.bc_order, b.kc_dcur,
                     b.ds_deg, b.ds_alive, b.gmode, b.dloop};
  static_assert(sizeof(x) == sizeof(y), "field lists differ");
  return std::memcmp(x, y, sizeof(x)) == 0 && a.partial_cap == b.partial_cap;
}

}  // namespace
}  // namespace byo

using namespace byo;

extern "C" byo_status byo_bfs_noalloc(byo_graph *g, int64_t src, int32_t *d_depth, int32_t *d_parent,
                                      const byo_opts *opts, void *stream, byo_run_stats *stats) {
  BYO_CHECK(g && d_depth && d_parent, BYO_EINVAL, "null argument");
  BYO_CHECK(src >= 0 && src < g->n, BYO_EINVAL, "source out of range");
  BYO_CHECK(g->n <= NA_MAX_N, BYO_EINVAL,
            "graph has more vertices than the no-alloc BFS scratch holds (BYO_NOALLOC_MAX_N)");
  byo_opts o;
  byo_opts_default(&o);
  if (opts) o = *opts;
  BYO_CHECK(o.use_graph == 0 && o.small_frontier == 0 && o.compressed == 0 && o.api_omit == 0, BYO_EINVAL,
            "the no-alloc BFS runs the host-driven CSR loop: use_graph, small_frontier, compressed and "
            "api_omit must be 0");
  int dev = -1;
  BYO_HIP(hipGetDevice(&dev));
  BYO_CHECK(dev == g->device, BYO_EINVAL, "the graph lives on another device than the current one");
  unsigned char *base = nullptr;
  BYO_TRY(na_scratch(dev, &base));
  BYO_CHECK(compaction_blocks((g->n + 63) / 64) + 2 <= (int64_t)(NA_PARTIAL / sizeof(long long)) &&
                (g->n + 1 + 2047) / 2048 + 2 <= (int64_t)(NA_PARTIAL / sizeof(long long)),
            BYO_EINVAL, "no-alloc BFS partials too small for this graph");
  // A view of the graph: same CSR, degrees and statistics, a workspace over
  // the scratch. Counter read-backs land in host memory on this stack.
  byo_graph view = *g;
  view.ws = byo_workspace();
  na_layout(base, g->n, view.ws);
  byo_counters h_ctr[BYO_COUNTER_SLOTS];
  view.ws.h_ctr = h_ctr;
  const byo_workspace before = view.ws;
  byo_status st;
  {
    no_alloc_scope guard;
    const int32_t s0 = (int32_t)src;
    st = bfs_run(&view, &s0, 1, d_depth, d_parent, o, (hipStream_t)stream, stats);
  }
  // the view must still point only at the scratch: anything the loop had
  // allocated into it would be a defect, reported rather than leaked silently
  if (!same_ptrs(before, view.ws)) return fail(BYO_ESTATE, "internal error: the no-alloc BFS allocated a buffer");
  return st;
}
