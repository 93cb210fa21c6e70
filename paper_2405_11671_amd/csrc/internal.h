// Internal declarations shared by the library's HIP sources (not installed).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>

#include <string>
#include <vector>

#include "byo.h"
#include "byo_trace.h"
#include "byo_selector.h"

// ---------------------------------------------------------------- errors

namespace byo {

void set_error(const std::string &msg);
byo_status fail(byo_status st, const std::string &msg);
byo_status hip_fail(hipError_t e, const char *what, const char *file, int line);

}  // namespace byo

#define BYO_HIP(call)                                                        \
  do {                                                                       \
    hipError_t _e = (call);                                                  \
    if (_e != hipSuccess) return byo::hip_fail(_e, #call, __FILE__, __LINE__); \
  } while (0)

#define BYO_CHECK(cond, st, msg)            \
  do {                                      \
    if (!(cond)) return byo::fail((st), (msg)); \
  } while (0)

#define BYO_TRY(expr)                      \
  do {                                     \
    byo_status _s = (expr);                \
    if (_s != BYO_OK) return _s;           \
  } while (0)

// ---------------------------------------------------------------- device helpers

#define BYO_WAVE 64
#define BYO_NUM_XCD 8

namespace byo {

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

__device__ __forceinline__ uint64_t lanemask_lt() {
  return (lane_id() == 0) ? 0ull : (~0ull >> (64 - lane_id()));
}

// Uniform read of lane `src`'s value (v_readlane; independent of EXEC).
__device__ __forceinline__ uint64_t read_lane_u64(uint64_t v, int src) {
  uint32_t lo = __builtin_amdgcn_readlane((uint32_t)v, src);
  uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(v >> 32), src);
  return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ int32_t read_lane_i32(int32_t v, int src) {
  return (int32_t)__builtin_amdgcn_readlane((uint32_t)v, src);
}

// Wavefront-aggregated append: every active lane with `pred` writes `val`
// into out[] at a slot reserved with one atomic per wavefront. Safe in
// divergent code (ballot and readlane act on the active lanes only).
__device__ __forceinline__ void wave_append(bool pred, int32_t val, int32_t *out,
                                            unsigned long long *count) {
  uint64_t m = __ballot(pred);
  if (m == 0) return;
  int leader = __ffsll((long long)m) - 1;
  unsigned long long base = 0;
  if (lane_id() == leader) base = atomicAdd(count, (unsigned long long)__popcll(m));
  base = read_lane_u64(base, leader);
  if (pred) out[base + __popcll(m & lanemask_lt())] = val;
}

// Hardware places workgroup b on XCD b % 8. Remap so that each XCD receives
// one contiguous range of logical block indices (its L2 then holds one range).
__device__ __forceinline__ uint32_t xcd_block(uint32_t bid, uint32_t nblocks) {
  uint32_t per = nblocks / BYO_NUM_XCD, rem = nblocks % BYO_NUM_XCD;
  uint32_t x = bid % BYO_NUM_XCD, i = bid / BYO_NUM_XCD;
  return (x < rem ? x * (per + 1) : rem * (per + 1) + (x - rem) * per) + i;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

template <typename T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    T w = __shfl_xor(v, o);
    v = w > v ? w : v;
  }
  return v;
}

// Block-wide sum; result valid in every thread. All threads must call it.
template <typename T, int BLOCK>
__device__ __forceinline__ T block_sum(T v) {
  __shared__ T part[BLOCK / BYO_WAVE];
  v = wave_sum(v);
  __syncthreads();
  if (lane_id() == 0) part[threadIdx.x / BYO_WAVE] = v;
  __syncthreads();
  T r = 0;
#pragma unroll
  for (int i = 0; i < BLOCK / BYO_WAVE; ++i) r += part[i];
  return r;
}

__device__ __forceinline__ bool test_bit(const uint64_t *bits, int64_t v) {
  return (bits[v >> 6] >> (v & 63)) & 1ull;
}

}  // namespace byo

// ---------------------------------------------------------------- objects

// Per-level counters written by edgeMap kernels (ring of slots, see edgemap).
// Every workgroup of a level adds into them, and device-scope atomics on one
// 128-byte line serialise with each other, so each counter has a line of its
// own (together on one line they cost single-source BFS a quarter of its
// rate at RMAT-22).
constexpr int BYO_LINE_U64 = 16;  // 64-bit words per 128-byte line
struct byo_counters {
  unsigned long long count;   // vertices emitted
  unsigned long long pad0_[BYO_LINE_U64 - 1];
  unsigned long long degsum;  // sum of their degrees
  unsigned long long pad1_[BYO_LINE_U64 - 1];
  unsigned long long aux0;    // variant-specific (e.g. edges inspected)
  unsigned long long pad2_[BYO_LINE_U64 - 1];
  unsigned long long aux1;
  unsigned long long pad3_[BYO_LINE_U64 - 1];
  unsigned long long maxdeg;  // largest degree among them (edgeMap levels)
  unsigned long long pad4_[BYO_LINE_U64 - 1];
};
#define BYO_COUNTER_SLOTS 4

namespace byo {
struct byo_tiles;
}

namespace byo {
// byte-coded neighbour lists (cz.hip): coff[v] = byte offset of v's list
struct byo_cz {
  int64_t *coff = nullptr;   // [n + 1]
  uint8_t *bytes = nullptr;  // [coff[n]], padded
  int64_t nbytes = 0;
  long long *fpre = nullptr;   // [n + 1] exclusive scan of the frontier's blocks (block-parallel push)
  long long *fpart = nullptr;  // [scan_partials_needed(n)] that scan's block partials
  int64_t fpart_cap = 0;
};
}  // namespace byo

struct byo_workspace {
  int64_t n = 0;
  int64_t words = 0;
  uint64_t *visited = nullptr;       // [words]
  uint64_t *bits[2] = {nullptr, nullptr};  // frontier bitmaps
  int32_t *ids[2] = {nullptr, nullptr};    // frontier ID lists
  long long *scan = nullptr;         // [n + 1] exclusive scans over frontier degrees
  long long *partial = nullptr;      // block partials for scans / compaction
  int64_t partial_cap = 0;
  byo_counters *ctr = nullptr;       // [BYO_COUNTER_SLOTS]
  byo_counters *h_ctr = nullptr;     // pinned host mirror
  int32_t *misc = nullptr;           // small device scratch (flags)
  int32_t *api_deg = nullptr;        // [n] degrees counted by mapping (container-API ablation, api.hip)
  int32_t *api_heavy = nullptr;      // [m / 4096 + 1] lists counted in chunks
  int64_t *api_pre = nullptr;        // [m / 4096 + 1] chunks before each of those lists
  unsigned long long *api_aux = nullptr;  // [4] degree sum, chunked lists, chunks
  // PageRank
  float *contrib[2] = {nullptr, nullptr};
  float *dpart = nullptr;            // dangling partial sums
  float *base = nullptr;             // per-iteration constant term
  int64_t *heavy_rows = nullptr;     // rows split into chunks
  int64_t *chunk_row = nullptr;      // per chunk: row
  int64_t *chunk_beg = nullptr;      // per chunk: first edge
  int32_t *row_chunk0 = nullptr;     // per vertex: first chunk index (or -1)
  float *chunk_sum = nullptr;
  int64_t nchunks = -1;
  int32_t pr_dpart_blocks = 0;
  void *ms = nullptr;                // multi-source BFS buffers (msbfs.hip)
  // degree-ordered destination-tile layouts, one per tile size 2^12 .. 2^14 (tiles.hip)
  byo::byo_tiles *tiles[3] = {nullptr, nullptr, nullptr};
  byo::byo_cz *cz = nullptr;           // byte-coded lists, built on first use
  double *bc_coef = nullptr;           // [n] betweenness: (1 + delta) / sigma per vertex
  double *bc_sigma = nullptr;          // [n] path counts when the caller passes none
  int32_t *bc_depth = nullptr;         // [n] depths when the caller passes none
  int32_t *bc_order = nullptr;         // [n] vertices level by level
  int32_t *kc_dcur = nullptr;          // [n] k-core: remaining degrees
  int32_t *ds_deg = nullptr;           // [n] densest subgraph: degrees inside S
  uint8_t *ds_alive = nullptr;         // [n] densest subgraph: membership of S
  void *gmode = nullptr;             // captured level graph (graphmode.hip)
  void *dloop = nullptr;             // device-resident level loop buffers (smallloop.hip)
  void *pbfs = nullptr;              // persistent-launch BFS buffers (persistent.hip)
  void *kcp = nullptr;               // persistent-launch k-core buffers (kcore.hip)
};

struct byo_graph {
  int64_t n = 0, m = 0;
  int64_t *off = nullptr;
  int32_t *nbr = nullptr;
  int32_t *deg = nullptr;
  uint64_t *zero_bits = nullptr;   // bitmap of degree-0 vertices
  bool owns_csr = false;
  int device = 0;
  int64_t max_deg = 0, isolated = 0;
  double mean_deg = 0.0, cv_deg = 0.0;
  byo_workspace ws;
  // batch updates (update.hip): an update writes the new CSR into the spare
  // arrays and swaps them in; the previous arrays, when the graph owns them,
  // become the spares of the next update
  int64_t nbr_cap = 0;             // entries the current nbr array holds
  int64_t *spare_off = nullptr;    // [n + 1]
  int32_t *spare_nbr = nullptr;    // [spare_cap]
  int64_t spare_cap = 0;
  void *upd = nullptr;             // the update path's buffers
};

// vertexSubset: which representations are current is tracked by flags.
struct byo_vset {
  const byo_graph *g = nullptr;
  int64_t n = 0, words = 0;
  int32_t *ids = nullptr;      // [n]
  uint64_t *bits = nullptr;    // [words]
  bool sparse_valid = false;
  bool dense_valid = false;
  int64_t count = 0;           // |U| (always known on the host)
  unsigned long long *d_tmp = nullptr;
};

// ---------------------------------------------------------------- internal API

namespace byo {

byo_status ws_ensure_traversal(byo_graph *g);
// degree array, degree-0 bitmap and statistics (max degree, isolated count,
// mean, coefficient of variation) from the current offsets; d_tmp: 8 device
// words of scratch. Syncs (graph.hip).
byo_status graph_refresh_stats(byo_graph *g, unsigned long long *d_tmp, hipStream_t s);
// buffers of the batch-update path (update.hip)
void upd_free(void *p);
byo_status ws_ensure_pagerank(byo_graph *g, hipStream_t s);
void ws_free(byo_workspace &ws);
void ms_release(byo_workspace &ws);
// Degree-ordered destination-tile layout (tiles.hip): vertices relabelled by
// descending degree; entries grouped by tile of 2^shift relabelled
// destinations, ascending relabelled source inside a tile; tiles cut into
// chunks of about equal size.
struct byo_tiles {
  int shift = 0;
  int64_t n = 0, m = 0, mp = 0, nblk = 0, nchunks = 0;
  // mp entries in 64-entry groups (a group's sources lie in one 2^16-aligned
  // window, whose base is the group's anchor; unused places are padding
  // with destination 2^shift, a slot no vertex uses). Entry e: source = anchor[e / 64] + (ent[e] & 0xffff),
  // tile-local destination = ent[e] >> 16; sources ascend inside a tile.
  uint32_t *ent = nullptr;    // [mp]
  int32_t *anchor = nullptr;  // [mp / 64]
  int32_t *rdeg = nullptr;    // [n] degree by relabelled vertex
  int32_t *orig = nullptr;    // [n] original ID of each relabelled vertex
  int64_t *cbeg = nullptr;    // [nchunks + 1] entry range of each chunk (whole groups, never straddles tiles)
  int32_t *bfirst = nullptr;  // [nblk + 1] first chunk of each tile
  int32_t *cblk = nullptr;    // [nchunks] tile of each chunk
  uint32_t *cflag = nullptr;  // [nchunks] per-level "chunk produced something" flags
  int32_t *rlabel = nullptr;  // [n] relabelled ID of each original vertex
  int32_t *scratch = nullptr; // [n] per-vertex work array (tiles_scratch)
  int64_t *roff = nullptr;    // [n + 1] CSR in relabelled IDs: row w is row orig[w]
  int32_t *rnbr = nullptr;    // [m] its neighbours, relabelled
  void *partial = nullptr;    // chunk results, sized by the user (tiles_partial)
  size_t partial_bytes = 0;
  // PageRank apply plan over the tiles cut into several chunks: one word per
  // apply workgroup, its first relabelled vertex with bit 0 set for a
  // many-chunk tile (64 vertices, chunk sums split four ways) and clear
  // otherwise (1024 vertices).
  int32_t *aplan = nullptr;   // [napply]
  int64_t napply = 0;
  int64_t wtail = 0;          // first relabelled vertex of the trailing tiles without entries (n if none)
};
// Relabelled source and tile-local destination of entry e. The caller's
// wavefront reads one whole group (e / 64 is the same in every lane), so the
// anchor is fetched once, through the scalar unit.
__device__ __forceinline__ void tile_entry(const uint32_t *__restrict__ ent, const int32_t *__restrict__ anchor,
                                           int64_t e, int32_t &src, uint32_t &dst) {
  const uint32_t x = ent[e];
  const int32_t g = __builtin_amdgcn_readfirstlane((int32_t)(e >> 6));
  dst = x >> 16;
  src = anchor[g] + (int32_t)(x & 0xffffu);
}
bool tiles_wanted(const byo_graph *g);  // n >= 2^16 and m >= 4n
// The layout with tiles of 2^shift vertices (12 .. 14), built on first use
// and kept with the graph next to the layouts of other tile sizes.
byo_status tiles_ensure(byo_graph *g, int shift, hipStream_t s, byo_tiles **out);
// Tile size for passes that may choose: 2^12 up to n = 2^22, 2^13 up to
// 2^23, 2^14 beyond (larger graphs re-read fewer contribution lines with
// fewer, larger tiles).
int tiles_auto_shift(const byo_graph *g);
byo_status tiles_partial(byo_tiles *t, size_t bytes_per_chunk);
byo_status tiles_scratch(byo_tiles *t);
// The layout's relabelled CSR seen as a graph, for the CSR push kernels: same
// sizes and statistics, shares g's workspace; never destroyed or grown.
byo_graph tiles_view(const byo_graph *g, const byo_tiles *t);
// connectivity over the tile layout (cc_tile.hip)
byo_status cc_tiled_run(byo_graph *g, int32_t *d_label, const byo_opts &o, hipStream_t s, byo_run_stats *stats);
void tiles_release(byo_workspace &w);
// tiled PageRank step (pagerank_tile.hip); opt = byo_opts::pr_blocked
int pr_tile_shift(const byo_graph *g, int32_t opt);
// bs = the step constant (1-d)/n + d*D/n
byo_status pr_tile_step(byo_graph *g, byo_tiles *p, const float *contrib, float bs, float damping,
                        float *contrib_next, float *out, hipStream_t s);

// container-API ablation (api.hip): degree / num_edges obtained without the
// container's degree() / num_edges(), and the variants the parallel-map
// capabilities allow
byo_status api_degree_buffer(byo_graph *g, hipStream_t s, int32_t **out);
// Degrees of the frontier (ids[0..k), or the set bits of bits when ids is
// null) by mapping, into the degree buffer; their sum in *degsum. The maps
// are parallel unless omit has BYO_API_NO_PAR_MAP.
byo_status api_frontier_degrees(byo_graph *g, uint32_t omit, const int32_t *ids, const uint64_t *bits, int64_t k,
                                hipStream_t s, int64_t *degsum);
// m: g->m, or without num_edges() the sum of deg (of mapped degrees without
// degree())
byo_status api_num_edges(byo_graph *g, uint32_t omit, const int32_t *deg, hipStream_t s, int64_t *m);
// every vertex's degree by mapping, into the degree buffer (no host wait)
byo_status api_map_degrees(byo_graph *g, uint32_t omit, hipStream_t s, int32_t **mdeg);
// the variant the container's functions allow in place of v (BFS pulls exit early)
int api_variant(uint32_t omit, int v, bool early_exit_pull);

// byte-coded CSR (cz.hip): built once per graph on first use and kept with it
byo_status cz_ensure(byo_graph *g, hipStream_t s, const byo_cz **out);
void cz_free(byo_cz *z);
// the form a variant takes over byte-coded lists (the bucketed push becomes
// the wavefront push; the others keep their kind)
int cz_variant(int v);

// conversions (vset.hip)
byo_status bitmap_clear(uint64_t *bits, int64_t words, hipStream_t s);
byo_status ids_to_bitmap(const int32_t *ids, int64_t k, uint64_t *bits, int64_t words, hipStream_t s);
// Ascending compaction of a bitmap into ids; writes the count to d_count.
byo_status bitmap_to_ids(const uint64_t *bits, int64_t words, int64_t n, int32_t *ids,
                         long long *partial, int64_t partial_cap, unsigned long long *d_count,
                         hipStream_t s);
int64_t compaction_blocks(int64_t words);
byo_status fill_i32(int32_t *p, int64_t count, int32_t value, hipStream_t s);
byo_status fill_u64(uint64_t *p, int64_t count, uint64_t value, hipStream_t s);
byo_status sync_read(hipStream_t s, const void *d_src, void *h_dst, size_t bytes);
// While one of these is alive on a thread, the library's helpers on that
// thread allocate nothing: sync_read copies into pageable caller memory and
// the optional level records and kernel timers stay off (graph.hip).
struct no_alloc_scope {
  no_alloc_scope();
  ~no_alloc_scope();
  no_alloc_scope(const no_alloc_scope &) = delete;
  no_alloc_scope &operator=(const no_alloc_scope &) = delete;
};
bool noalloc_active();

// exclusive scan of ceil(deg(ids[i]) / per) (per = 1: the degrees themselves);
// partial needs scan_partials_needed(k) entries
byo_status scan_degree_units(const int32_t *deg, const int32_t *ids, int64_t k, int32_t per, long long *scan,
                             long long *partial, int64_t partial_cap, hipStream_t s);
int64_t scan_partials_needed(int64_t k);
// the same over an explicit degree array
byo_status scan_degrees(const int32_t *deg, const int32_t *ids, int64_t k, long long *scan, long long *partial,
                        int64_t partial_cap, hipStream_t s);
// exclusive scan of frontier degrees: scan[i] = sum_{j<i} deg(ids[j]); scan[k] = total
byo_status frontier_degree_scan(const byo_graph *g, const int32_t *ids, int64_t k, long long *scan,
                                long long *partial, int64_t partial_cap, hipStream_t s);

struct level_io {
  // input frontier
  const int32_t *in_ids;
  const uint64_t *in_bits;
  int64_t in_count;
  // output frontier
  int32_t *out_ids;       // may be null for dense-only output
  uint64_t *out_bits;     // may be null for sparse-only output
  byo_counters *ctr;      // this level's counter slot
  byo_counters *ctr_clear;  // slot to zero for a later level (may be null)
};

struct bfs_state {
  int32_t *parent;
  int32_t *depth;
  uint64_t *visited;
  int32_t level;
};

// One BFS edgeMap level with the given variant. Push variants need in_ids
// (and the degree scan for PUSH_EDGE in g->ws.scan); pull variants need
// in_bits and produce dense output (out_bits) only.
// known_total: sum of deg(U) if the caller knows it (skips a read-back), else -1.
byo_status bfs_level(byo_graph *g, int variant, const bfs_state &st, const level_io &io,
                     const byo_opts &o, hipStream_t s, long long known_total = -1);
byo_status cc_level(byo_graph *g, int variant, int32_t *label, const level_io &io, const byo_opts &o,
                    hipStream_t s, long long known_total = -1);
// the same levels over the byte-coded lists (variants as cz_variant maps them)
// known_total: the frontier's degree sum (sizes the block-parallel push)
byo_status cz_bfs_level(byo_graph *g, int variant, const bfs_state &st, const level_io &io, hipStream_t s,
                        long long known_total);
byo_status cz_cc_level(byo_graph *g, int variant, int32_t *label, const level_io &io, hipStream_t s,
                       long long known_total);
// acc[v] = sum over u in N(v) of contrib[u] (pagerank.hip)
byo_status pr_accumulate(byo_graph *g, const float *contrib, float *acc, hipStream_t s);
byo_status cc_shortcut(byo_graph *g, int32_t *label, uint64_t *out_bits, byo_counters *ctr, hipStream_t s);

// multi-source BFS state: per vertex W words of source bits
struct ms_state {
  int W;
  const uint64_t *front;  // current frontier bits [n][W]
  const uint64_t *seen;   // [n][W]
  uint64_t *visit;        // push accumulation [n][W] (all zero between levels)
};
byo_status ms_push_level(byo_graph *g, int variant, const ms_state &ms, const level_io &io, const byo_opts &o,
                         hipStream_t s, long long known_total);

// tracing (trace.hip)
bool trace_on();
bool ktimer_on();
hipEvent_t event_get();
void event_put(hipEvent_t e);
void trace_push(const byo_level_record &r);
// HIP events around the launches made while the scope is alive (if enabled).
struct ktimer_scope {
  int family;
  hipStream_t s;
  hipEvent_t a = nullptr, b = nullptr;
  ktimer_scope(int fam, hipStream_t st);
  ~ktimer_scope();
};

// ---------------------------------------------------------------- variant choice

// Threshold rule (host and device): dense pull iff |U| + sum(deg(U)) > m / div
// (the sparse/dense cutoff of Section 6.3); sparse pushes are edge-balanced on
// skewed graphs or heavy frontiers, wavefront-per-vertex for high average
// degree, thread-per-vertex otherwise.
// max_deg is the graph's largest degree (pulls scan the lists of unvisited
// vertices); frontier_max_deg, when known (>= 0), the largest degree in U,
// which sets how long a push's longest list is.
__host__ __device__ inline int heuristic_rule(int64_t k, int64_t degsum, int64_t m, int64_t max_deg, double cv,
                                              int div, int t_wave, int t_block, bool allow_pull,
                                              int64_t frontier_max_deg = -1) {
  if (div <= 0) div = 20;
  if (t_wave <= 0) t_wave = 32;
  if (t_block <= 0) t_block = 4096;
  if (allow_pull && k + degsum > m / div)
    return (cv > 1.0 || max_deg > 4 * (int64_t)t_wave) ? BYO_V_PULL_WAVE : BYO_V_PULL_THREAD;
  double avg = k > 0 ? (double)degsum / (double)k : 0.0;
  if (frontier_max_deg >= 0) {
    // The lists' own lengths: a wavefront takes 64 entries per round and a
    // thread one, each round waiting on its claims, so a list longer than 8
    // wavefront rounds goes to the edge-balanced push, and one lane per list
    // only when every list is at most 8 long.
    if (frontier_max_deg > 8 * BYO_WAVE || degsum >= 65536) return BYO_V_PUSH_EDGE;
    return frontier_max_deg <= 8 ? BYO_V_PUSH_THREAD : BYO_V_PUSH_WAVE;
  }
  // only the graph's largest degree known: it bounds the lists from above
  if (max_deg >= t_block || degsum >= 65536) return BYO_V_PUSH_EDGE;
  if (avg >= t_wave) return BYO_V_PUSH_WAVE;
  return BYO_V_PUSH_THREAD;
}

// Raw selector features of a level (host and device; see byo_selector.h).
__host__ __device__ inline void selector_features(double k, double degsum, double unvisited, double n, double m,
                                                  double max_deg, double cv, double dense_in, float *f) {
  f[0] = (float)log2(1.0 + k);
  f[1] = (float)log2(1.0 + degsum);
  f[2] = (float)log2(1.0 + unvisited);
  f[3] = (float)log2(1.0 + n);
  f[4] = (float)log2(1.0 + m);
  f[5] = (float)((k + degsum) / (m + 1.0));
  f[6] = (float)(k / (n + 1.0));
  f[7] = (float)log2(1.0 + max_deg);
  f[8] = (float)cv;
  f[9] = (float)log2(1.0 + degsum / (k + 1.0));
  f[10] = (float)(unvisited / (n + 1.0));
  f[11] = (float)dense_in;
}

// variant choice (selector.hip)
struct level_features {
  int64_t n, m, k, degsum, unvisited, max_deg, level;
  double cv;
  bool dense_in;
  int64_t frontier_max_deg = -1;  // largest degree in U (-1: not known)
};
int choose_variant(const byo_opts &o, const level_features &f, bool allow_pull);

// device-resident small-frontier BFS levels (smallloop.hip)
struct small_loop_out {
  int32_t levels = 0, side = 0;
  bool empty = false;
  int64_t count = 0, degsum = 0, reached = 0, edges = 0;
};
constexpr int64_t BYO_DLOOP_QCAP = 1 << 17;  // frontier and per-level edge cap of the device-resident loop
bool bfs_small_loop_usable(byo_graph *g);
byo_status bfs_small_loop(byo_graph *g, const int32_t *in_ids, int64_t k, int64_t in_degsum, int32_t level,
                          int32_t max_levels, int64_t cap_count, int64_t cap_edges, int32_t *parent, int32_t *depth,
                          uint64_t *visited, int32_t *out, hipStream_t s, small_loop_out *res_out);
void dl_release(byo_workspace &w);

// BFS with device-side level control replayed from a hipGraph (graphmode.hip)
byo_status bfs_graph_run(byo_graph *g, const std::vector<int32_t> &srcs, int32_t *d_depth, int32_t *d_parent,
                         const byo_opts &o, hipStream_t s, byo_run_stats *stats);
void gm_release(byo_workspace &w);
// parent/depth/visited set up for BFS from d_srcs (distinct), traverse.hip
byo_status bfs_sources_init(byo_graph *g, const int32_t *d_srcs, int64_t ns, int32_t *parent, int32_t *depth,
                            hipStream_t s);

// BFS from distinct sources in one persistent cooperative launch
// (persistent.hip); usable when the device supports cooperative launches
bool bfs_persistent_usable(byo_graph *g);
byo_status bfs_persistent_run(byo_graph *g, const int32_t *srcs, int64_t ns, int32_t *d_depth, int32_t *d_parent,
                              const byo_opts &o, hipStream_t s, byo_run_stats *stats);
void pb_release(void *p);
void kp_release(void *p);

// BFS from distinct sources (traverse.hip)
byo_status bfs_run(byo_graph *g, const int32_t *srcs, int64_t ns, int32_t *d_depth, int32_t *d_parent,
                   const byo_opts &o, hipStream_t s, byo_run_stats *stats);
int heuristic_variant(const byo_opts &o, const level_features &f, bool allow_pull);
// learned selector (selector.hip)
bool selector_ready();
// Device copy of the installed weights (params, mu, sd) on the current
// device, or null; *version changes whenever weights are set or cleared.
const float *selector_device_weights(uint64_t *version);
// Learned choice for one level, computed on the host from the level's
// features (the host-driven loop holds them already); -1 if no weights are
// installed or the prediction is not finite.
int selector_pick_cpu(const level_features &f, bool allow_pull);

}  // namespace byo
