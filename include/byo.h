/*
 * byo.h -- C ABI of the MI355X (gfx950) edgeMap traversal library.
 *
 * The library implements the read path of the paper's graph-container API
 * (BYO, arXiv 2405.11671): a GraphContainer over a static CSR
 * (num_vertices, num_edges, degree, map_neighbors and its early-exit and
 * parallel variants; Section 4.2), the Ligra/GBBS vertexSubset (sparse ID list
 * or dense bit array; Section 3.2 "VertexSubsets" and the bit-array change of
 * Section 4.4), and edgeMap(G, U, F) (Section 3.2 "EdgeMap"), plus the
 * algorithms the paper evaluates on top of it that reduce to edgeMap: BFS,
 * connectivity and PageRank (Table algs-list, Section 6.2).
 *
 * Conventions shared by every entry point:
 *  - Vertex IDs are int32 (n < 2^31); CSR offsets are int64.
 *  - "d_" pointers are device (HBM) pointers, "h_" pointers host pointers.
 *    Device buffers passed in stay owned by the caller; the library owns what
 *    it allocates and frees it in the matching destroy call.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream). Calls
 *    enqueue their kernels on it. Calls that return a host scalar computed on
 *    the device synchronise that stream before returning.
 *  - Calls on one graph object share its workspace: issue them from one host
 *    thread on one stream (concurrent calls on the same graph race).
 *  - Every call returns a byo_status. On error nothing is written to the
 *    out-parameters and byo_last_error() describes the failure (thread-local).
 *    Nothing in the library ever falls back to host computation.
 */
#ifndef BYO_H_
#define BYO_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  BYO_OK = 0,
  BYO_EINVAL = -1,   /* bad argument or malformed input */
  BYO_ENOMEM = -2,   /* device or host allocation failed */
  BYO_EHIP = -3,     /* a HIP runtime call failed */
  BYO_ELIMIT = -4,   /* level / round cap reached before convergence */
  BYO_ESTATE = -5    /* object in the wrong state (e.g. no selector weights) */
} byo_status;

typedef struct byo_graph byo_graph;   /* opaque CSR GraphContainer on one device */
typedef struct byo_vset byo_vset;     /* opaque vertexSubset (sparse list and/or dense bitmap) */
typedef struct byo_batch byo_batch;   /* opaque batch of graphs run in one launch sequence */

/* ------------------------------------------------------------------------
 * edgeMap variants. The paper's API study (Section 6.3, Table
 * api-components-avg) shows that which map variants a container offers
 * changes only running time; here every variant computes the same result and
 * only the schedule differs.
 *   PUSH_*: sparse input (ID list), apply F from each u in U to N(u)
 *           ("map_neighbors" / "parallel_map_neighbors", Section 4.2).
 *   PULL_*: dense input (bitmap), each candidate v scans N(v) for members of
 *           U and stops at the first hit where F allows it
 *           ("map_neighbors_early_exit" / "parallel_map_neighbors_early_exit").
 * ---------------------------------------------------------------------- */
typedef enum {
  BYO_V_PUSH_THREAD = 0,  /* one thread per frontier vertex, serial map */
  BYO_V_PUSH_WAVE = 1,    /* one 64-lane wavefront per frontier vertex */
  BYO_V_PUSH_BUCKET = 2,  /* degree-bucketed: thread / wavefront / workgroup per vertex */
  BYO_V_PUSH_EDGE = 3,    /* edge-balanced: equal slices of sum(deg(U)) per workgroup */
  BYO_V_PULL_THREAD = 4,  /* one thread per vertex, serial early-exit map */
  BYO_V_PULL_WAVE = 5,    /* thread first, then wavefront-parallel early-exit map for long lists */
  BYO_NUM_VARIANTS = 6
} byo_variant;

typedef enum {
  BYO_SEL_HEURISTIC = 0,  /* dense pull iff |U| + sum(deg(U)) > m / dense_divisor (Section 6.3) */
  BYO_SEL_MLP = 1,        /* learned selector (weights from byo_selector_set); heuristic if none */
  BYO_SEL_FIXED = 2       /* always fixed_variant */
} byo_selector_mode;

/* Options; fill with byo_opts_default() and override fields. */
typedef struct byo_opts {
  int32_t selector;       /* byo_selector_mode (default HEURISTIC) */
  int32_t fixed_variant;  /* byo_variant used with BYO_SEL_FIXED (default PUSH_EDGE) */
  int32_t dense_divisor;  /* heuristic cutoff divisor (default 20) */
  int32_t t_wave;         /* PUSH_BUCKET / PULL_WAVE: degree >= t_wave goes to a wavefront (default 32) */
  int32_t t_block;        /* PUSH_BUCKET: degree >= t_block goes to a workgroup (default 4096) */
  int32_t max_levels;     /* BFS level / CC round cap; 0 = n + 1 */
  int32_t cc_shortcut;    /* CC: pointer-jumping pass after each round (default 1) */
  int32_t small_frontier; /* BFS: frontiers of at most this many vertices (and at most
                             max(16 x this, 2^16) edges, capped at 2^17) run in the
                             device-resident loop: one cooperative kernel of 64
                             workgroups, grid barriers between levels (0 = off; default 0) */
  int32_t pr_blocked;     /* PageRank layout: 0 = pull over the CSR; 1 (default) = entries
                             regrouped by destination tile of degree-ordered vertices, exact
                             fixed-point sums in LDS, tiles of 2^12 vertices up to n = 2^22,
                             2^13 up to 2^23, 2^14 beyond; 12..14 = tiles of 2^value. The
                             tiled layout is used when n >= 2^16 and m >= 4n (else the pull);
                             it is built on the device on first use (about 8 bytes per entry
                             plus 24 per vertex of device memory) and kept with the graph,
                             one layout per tile size. */
  int32_t use_graph;      /* BFS: 1 = device-side level control replayed from a captured
                             hipGraph (push or pull chosen on the device: the threshold
                             rule, or with selector = BYO_SEL_MLP the learned network
                             evaluated there), 0 = host loop (default) */
  int32_t tiled;          /* multi-source BFS and connectivity: 1 (default) = dense levels /
                             rounds over the degree-ordered tile layout (the kind PageRank's
                             pr_blocked uses; multi-source BFS always with tiles of 2^12
                             vertices) when n >= 2^16 and m >= 4n, else over the CSR; 0 = over
                             the CSR with the selected variants */
  int32_t tile_shift;     /* connectivity with tiled = 1: tiles of 2^value vertices (12..14);
                             0 = chosen from n as for pr_blocked = 1 (default) */
  int32_t api_omit;       /* container-API ablation: BYO_API_NO_* bits of container functions
                             BFS, connectivity and PageRank may not use; 0 = the whole API
                             (default) */
  int32_t ms_history;     /* multi-source BFS with tiled = 1: levels whose frontier masks are kept
                             for building the depth rows in one pass (2..16; later levels write
                             depths directly); 0 = as many as fit in a quarter of the free device
                             memory, at most 16 (default). Each kept level costs 8 * W * n bytes
                             (W = ceil(k / 64)) plus n / 8. */
  int32_t compressed;     /* 1: BFS, connectivity and PageRank read the byte-coded lists
                             (byo_cz_build; built on first use) through the host-driven level loop:
                             push by thread, wavefront (also for PUSH_BUCKET) or blocks spread over
                             the grid (PUSH_EDGE), pull by thread or wavefront, PageRank's pull over
                             the lists.
                             With api_omit != 0: BYO_EINVAL. 0 = the CSR (default) */
  int32_t persistent;     /* byo_batch_bfs and byo_kcore: 1 (default) = the whole traversal in
                             one persistent cooperative launch with grid barriers between its
                             phases (the batch's levels take their direction by the threshold
                             rule on the device; k-core's sub-rounds their removal scheme by
                             the same frontier tests as the host loop); where cooperative
                             launches are not supported, and for k-core with api_omit != 0,
                             the host loop runs instead. 0 = the host-driven loop (for the
                             batch also hipGraph levels with use_graph = 1). 2 = as 1, and
                             byo_bfs too runs its search in that one launch (direction by the
                             threshold rule: selector, small_frontier and per-level traces do
                             not apply; not with use_graph, compressed or api_omit) */
} byo_opts;

/* Container functions a traversal can be denied (Section 4.2 defines the
 * GraphContainer API: map_neighbors and num_vertices required; num_edges,
 * degree, early-exit and parallel maps optional; Table api-components-avg
 * measures configurations that leave them out). Results never change; only
 * the work does:
 *  - NO_DEGREE: every degree the framework needs (frontier degree sums for
 *    the sparse/dense cutoff, degree bucketing, edge-balanced offsets,
 *    PageRank's division) is counted by mapping over the vertex's
 *    neighbours: once per frontier vertex per level, and for every vertex at
 *    every PageRank step;
 *  - NO_NUM_EDGES: m for the cutoff is recomputed at every level, as the
 *    sum of the degrees (by mapping, without degree);
 *  - NO_EARLY_EXIT: a BFS pull lane scans its whole list (the first frontier
 *    neighbour found is still the parent); lists handed to the wavefront's
 *    cooperative scan keep the parallel early exit unless that is left out
 *    too;
 *  - NO_PAR_MAP: a vertex's neighbours are mapped by one thread: push by a
 *    thread per frontier vertex, connectivity's pull and PageRank's rows by
 *    one lane each (no wavefront-assisted rows, no chunks);
 *  - NO_PAR_EARLY_EXIT: no wavefront-cooperative early-exit BFS pull.
 * With any bit set, BFS and connectivity run the host-driven CSR level loop
 * (no device-resident small-frontier loop, no hipGraph capture, no tiled
 * connectivity) and PageRank the CSR pull (no tiled step). The multi-source
 * BFS ignores it. */
enum {
  BYO_API_NO_DEGREE = 1,
  BYO_API_NO_NUM_EDGES = 2,
  BYO_API_NO_EARLY_EXIT = 4,
  BYO_API_NO_PAR_MAP = 8,
  BYO_API_NO_PAR_EARLY_EXIT = 16
};

/* Per-call statistics (optional out-parameter; pass NULL to skip). */
typedef struct byo_run_stats {
  int32_t levels;                          /* BFS levels / CC rounds / PR iterations executed */
  int32_t device_levels;                   /* of those, levels run in the device-resident loop */
  int64_t variant_count[BYO_NUM_VARIANTS]; /* edgeMap calls per variant */
  int64_t reached;                         /* BFS: vertices reached; CC: components */
  int64_t edges;                           /* BFS: sum of degrees of reached vertices */
} byo_run_stats;

/* Status string of the last failing call on this thread ("" if none). */
const char *byo_last_error(void);
/* Library version string. */
const char *byo_version(void);
void byo_opts_default(byo_opts *opts);

/* ------------------------------------------------------------------------
 * CSR construction (host). From raw pairs (src[i], dst[i]) over n vertices:
 * add both directions, drop self-pairs, sort each row and drop repeats
 * (the paper's graphs are symmetrised, simple and unweighted, Section 6.2).
 * Caller allocates h_off (n + 1 entries) and h_nbr (capacity 2 * npairs);
 * *m_out receives the number of directed entries written. Uses host threads.
 * ---------------------------------------------------------------------- */
byo_status byo_csr_from_pairs(const int32_t *h_src, const int32_t *h_dst, int64_t npairs, int64_t n,
                              int64_t *h_off, int32_t *h_nbr, int64_t *m_out);

/* ------------------------------------------------------------------------
 * GraphContainer (Section 4.2). CSR: offsets off[n + 1] (int64, off[0] = 0,
 * non-decreasing, off[n] = m), neighbours nbr[m] (int32, each row strictly
 * increasing, no self-loops, undirected = every (u, v) has (v, u)).
 * Flags choose where off/nbr live and whether they are copied or borrowed.
 * With BYO_VALIDATE the structure is checked on the device and
 * BYO_EINVAL is returned if any rule above fails.
 * ---------------------------------------------------------------------- */
#define BYO_HOST_INPUT 0x1u     /* off/nbr are host pointers: copied to the device */
#define BYO_DEVICE_COPY 0x2u    /* off/nbr are device pointers: copied */
#define BYO_DEVICE_BORROW 0x4u  /* off/nbr are device pointers: used in place; caller keeps them alive */
#define BYO_VALIDATE 0x8u       /* check the CSR rules (including symmetry) on the device */

byo_status byo_graph_from_csr(const int64_t *off, const int32_t *nbr, int64_t n, int64_t m, uint32_t flags,
                              void *stream, byo_graph **out);
void byo_graph_destroy(byo_graph *g);
/* n and m; -1 for a null graph, with the message in byo_last_error. */
int64_t byo_num_vertices(const byo_graph *g);        /* n (required API) */
int64_t byo_num_edges(const byo_graph *g);           /* m = directed entries (optional API) */
byo_status byo_degree(const byo_graph *g, int64_t v, int64_t *out);  /* |N(v)|, syncs */
/* getNeighbors expressed with map (Table gbbs-byo-translation): copies up to cap
 * neighbours of v, ascending, into h_buf; *count = |N(v)|. Syncs. */
byo_status byo_get_neighbors(const byo_graph *g, int64_t v, int32_t *h_buf, int64_t cap, int64_t *count);
/* Device pointers to the CSR arrays and the int32 degree array deg[n]. */
byo_status byo_graph_arrays(const byo_graph *g, const int64_t **d_off, const int32_t **d_nbr,
                            const int32_t **d_deg);
/* Host copies of the CSR: h_off (n + 1 int64) and h_nbr (m int32), caller
 * owned (after batch updates, the updated container). Waits for the device. */
byo_status byo_graph_copy(const byo_graph *g, int64_t *h_off, int32_t *h_nbr);
/* Degree statistics computed at creation (and after each batch update): max
 * degree, number of isolated vertices, mean and coefficient of variation of
 * the degree. */
byo_status byo_graph_stats(const byo_graph *g, int64_t *max_deg, int64_t *isolated, double *mean,
                           double *cv);

/* ------------------------------------------------------------------------
 * Batch updates (Section 4.1, "Translating graph batch-update API into the
 * set API", and Section 4.2, "Required functionality for updates": the
 * container's insert_sorted_batch / delete_sorted_batch, the framework
 * sorting the batch first).
 *
 * A batch is k pairs (d_src[i], d_dst[i]) in device memory (int32; caller
 * owned, only read). Each pair with src != dst names the undirected edge
 * {src, dst}: both directions are inserted or deleted together, so the
 * container stays symmetric and simple. Self-pairs change nothing and
 * repeated pairs act once; inserting an existing edge or deleting a missing
 * one changes nothing. The graph is updated in place as seen by the caller:
 * the CSR arrays (byo_graph_arrays), m, the degree array and the statistics
 * are those of the new edge set afterwards, rows still strictly increasing.
 * Derived structures (tile layouts, byte-coded lists, captured level graphs,
 * traversal workspace) are dropped and rebuilt on next use. A graph created
 * with BYO_DEVICE_BORROW stops using the caller's arrays at its first update
 * (they are left untouched). *changed (nullable) receives the number of
 * directed entries added or removed (twice the undirected edges).
 * Errors: BYO_EINVAL (and the graph unchanged) if a pair names a vertex
 * outside [0, n) or k < 0; BYO_ENOMEM if the new arrays do not fit.
 * Syncs `stream`. Cost: the batch's sort plus one pass over the CSR (the rows
 * shift in the packed arrays), about 8 bytes per entry moved.
 * ---------------------------------------------------------------------- */
byo_status byo_graph_insert_batch(byo_graph *g, const int32_t *d_src, const int32_t *d_dst, int64_t k,
                                  void *stream, int64_t *changed);
byo_status byo_graph_delete_batch(byo_graph *g, const int32_t *d_src, const int32_t *d_dst, int64_t k,
                                  void *stream, int64_t *changed);

/* The three forms in which the framework can hand a batch to a container
 * (Section 4.1). Each output holds the input's pairs, each as often:
 *  - BYO_FORM_SORT: ascending (src, dst), the global sort;
 *  - BYO_FORM_SEMISORT: the pairs of one source next to each other (here the
 *    groups come out in ascending source order and a group keeps its pairs'
 *    input order; other containers may accept any group order);
 *  - BYO_FORM_GROUPED_SORT: grouped by source, each group ascending by dst.
 * IDs must lie in [0, n) (else BYO_EINVAL); n < 2^31. Outputs are device
 * arrays of k int32 the caller owns, distinct from the inputs; every pointer
 * must be non-null, also for k = 0. Syncs. */
typedef enum { BYO_FORM_SORT = 0, BYO_FORM_SEMISORT = 1, BYO_FORM_GROUPED_SORT = 2 } byo_batch_form;
byo_status byo_batch_order(const int32_t *d_src, const int32_t *d_dst, int64_t k, int64_t n, int32_t form,
                           int32_t *d_out_src, int32_t *d_out_dst, void *stream);

/* ------------------------------------------------------------------------
 * Byte-coded CSR: the compressed container of Section 2 ("compressed
 * graphs": each sorted list stored by difference encoding with byte codes),
 * in the blocked form that lets blocks decode independently. Kept with the
 * graph next to the CSR; BFS, connectivity and PageRank decode it inside
 * their kernels when byo_opts.compressed = 1.
 *
 * Format. Vertex v's list (degree d = deg[v], neighbours u_0 < ... < u_{d-1})
 * starts at byte off[v] of the stream; off[n] = total bytes. It holds
 * nb = ceil(d / 64) blocks, block j being u_{64j} .. u_{min(d, 64j+64)-1}:
 *  - if nb > 1, first nb - 1 little-endian uint32: the byte offset, from
 *    off[v], of blocks 1 .. nb - 1;
 *  - then the blocks in order. A block's first neighbour u is stored as
 *    zigzag(u - v) (zigzag(x) = 2x for x >= 0, -2x - 1 for x < 0), every
 *    further one as its gap to the previous neighbour (>= 1);
 *  - each stored value is a byte code: 7 bits per byte, low group first,
 *    bit 7 set on every byte but the last.
 * Degree-0 vertices take no bytes.
 * ---------------------------------------------------------------------- */
/* Build the byte-coded lists on the device (once per graph; later calls
 * return at once). Syncs. */
byo_status byo_cz_build(byo_graph *g, void *stream);
/* Size of the byte stream; BYO_EINVAL before byo_cz_build. */
byo_status byo_cz_bytes(const byo_graph *g, int64_t *nbytes);
/* Copy the offsets (n + 1 int64) and the stream (byo_cz_bytes bytes) to
 * host buffers the caller owns. Syncs. BYO_EINVAL before byo_cz_build. */
byo_status byo_cz_copy(const byo_graph *g, int64_t *h_off, uint8_t *h_bytes);
/* Decode v's list on the device into d_out[0 .. deg(v)) (device buffer the
 * caller owns), ascending. Builds the lists if needed. */
byo_status byo_cz_decode(byo_graph *g, int64_t v, int32_t *d_out, void *stream);

/* ------------------------------------------------------------------------
 * vertexSubset (Section 3.2): sparse (IDs) or dense (bit array u64[ceil(n/64)],
 * bit v%64 of word v/64; Section 4.4 replaces the bool array with this).
 * ---------------------------------------------------------------------- */
byo_status byo_vset_create(const byo_graph *g, byo_vset **out);   /* empty subset */
void byo_vset_destroy(byo_vset *s);
/* Replace the contents with k distinct IDs from device memory (each < n). */
byo_status byo_vset_from_ids(byo_vset *s, const int32_t *d_ids, int64_t k, void *stream);
/* Replace the contents with a device bitmap of ceil(n/64) words (bits >= n ignored). */
byo_status byo_vset_from_bitmap(byo_vset *s, const uint64_t *d_bits, void *stream);
byo_status byo_vset_fill(byo_vset *s, void *stream);              /* all n vertices */
byo_status byo_vset_size(byo_vset *s, int64_t *out, void *stream); /* |s|, syncs */
/* Write the members in ascending order to d_ids (capacity cap); *k = |s|.
 * BYO_EINVAL if cap < |s|. Syncs. */
byo_status byo_vset_to_ids(byo_vset *s, int32_t *d_ids, int64_t cap, int64_t *k, void *stream);
/* Write the dense form (ceil(n/64) words, bits >= n zero) to d_bits. */
byo_status byo_vset_to_bitmap(byo_vset *s, uint64_t *d_bits, void *stream);

/* ------------------------------------------------------------------------
 * edgeMap(G, U, F) (Section 3.2): apply F to edges out of U and return in
 * `out` the targets F accepts. F is a closed set of functors whose state is
 * device memory:
 *   BYO_F_BFS:    state byo_bfs_fn. For u in U, v in N(u) with parent[v] == -1:
 *                 set parent[v] = u (any such u), depth[v] = level + 1, emit v,
 *                 and set bit v of `visited`. Requires: visited bit v is set
 *                 iff parent[v] != -1, with bits >= n set in the last word.
 *   BYO_F_CC_MIN: state byo_cc_fn. For u in U, v in N(u): label[v] =
 *                 min(label[v], label[u]); emit v if its label decreased.
 *   BYO_F_PR_ACC: state byo_pr_fn. acc[v] = sum over u in N(v) and U of
 *                 contrib[u] (every v; FP32; U must be the full set).
 * `variant` < 0 lets opts->selector choose; otherwise the given variant runs
 * (PR_ACC ignores it). *variant_used (nullable) receives the choice.
 * ---------------------------------------------------------------------- */
typedef enum { BYO_F_BFS = 0, BYO_F_CC_MIN = 1, BYO_F_PR_ACC = 2 } byo_edge_fn;
typedef struct { int32_t *parent; int32_t *depth; uint64_t *visited; int32_t level; } byo_bfs_fn;
typedef struct { int32_t *label; } byo_cc_fn;
typedef struct { const float *contrib; float *acc; } byo_pr_fn;

byo_status byo_edge_map(byo_graph *g, byo_vset *U, byo_edge_fn F, const void *F_state, byo_vset *out,
                        int32_t variant, const byo_opts *opts, void *stream, int32_t *variant_used);

/* ------------------------------------------------------------------------
 * Algorithms (Table algs-list). Outputs are caller-owned device arrays of n.
 * ---------------------------------------------------------------------- */
/* BFS from src: depth[v] = hop distance (-1 unreached), parent[v] = a
 * neighbour at depth - 1 (parent[src] = src, -1 unreached). */
byo_status byo_bfs(byo_graph *g, int64_t src, int32_t *d_depth, int32_t *d_parent, const byo_opts *opts,
                   void *stream, byo_run_stats *stats);
/* BFS for callers that cannot allocate: code recorded under stream capture,
 * tight serving loops and harnesses that forbid hipMalloc. Same result
 * conventions, level loop and kernels as byo_bfs (host-driven CSR levels,
 * selector as opts chooses), but it allocates no device or pinned host
 * memory and does not touch the graph's lazily allocated workspace: every
 * per-run buffer (visited and frontier bitmaps, frontier lists, the frontier
 * degree scan, block partials, level counters) lives in one device array of
 * the library's, about 34 MiB, that each device the library runs on keeps
 * until the process ends. Limits and errors:
 *  - n must be at most BYO_NOALLOC_MAX_N (2^21), else BYO_EINVAL;
 *  - opts (nullable) must leave use_graph, small_frontier, compressed and
 *    api_omit at 0 (those paths allocate), else BYO_EINVAL;
 *  - the graph must live on the current device, else BYO_EINVAL;
 *  - level records and kernel timers are not kept for this call.
 * Every call on one device shares that device's array, and the array keeps
 * the last call's contents (each call re-initialises what it reads): calls
 * that overlap on one device, from several streams or threads, race and give
 * wrong results. The call reads a few counters back per level, so it
 * synchronises `stream` like byo_bfs. */
#define BYO_NOALLOC_MAX_N (1 << 21)
byo_status byo_bfs_noalloc(byo_graph *g, int64_t src, int32_t *d_depth, int32_t *d_parent, const byo_opts *opts,
                           void *stream, byo_run_stats *stats);
/* Connectivity by min-label propagation over edgeMap: label[v] = smallest
 * vertex ID in v's component. With tiled = 1, dense rounds run over the tile
 * layout, and a vertex whose label drops also lowers the vertex its old label
 * named (hooking); cc_shortcut adds pointer jumping. Any path gives the same
 * labels. */
byo_status byo_cc(byo_graph *g, int32_t *d_label, const byo_opts *opts, void *stream, byo_run_stats *stats);
/* Single-source betweenness (Table algs-list, shortest-path problems): the
 * dependency of src on every vertex, delta[v] = sum over targets t of
 * sigma_st(v) / sigma_st, where sigma_st counts shortest src-t paths and
 * sigma_st(v) those through v (Brandes' dependency; delta[src] = 0, and 0 for
 * vertices src does not reach). sigma[v] = number of shortest src-v paths
 * (integers, exact in FP64 below 2^53; 0 when unreachable); depth[v] = hop
 * distance (-1 when unreachable).
 * Forward: level-synchronous BFS that counts paths, push or pull per level by
 * the sparse/dense cutoff (|U| + sum deg(U) > m / dense_divisor);
 * selector = BYO_SEL_FIXED forces push (PUSH_*) or pull (PULL_*), the
 * *_THREAD variants without wavefront-shared lists. Backward: one pull per
 * level, deepest first. d_delta: device FP64 [n]; d_sigma (FP64 [n]) and
 * d_depth (int32 [n]) are device buffers or NULL. Returns when done (it reads
 * each level's size back). BYO_ELIMIT if max_levels is reached. stats:
 * levels, reached, edges (sum of the frontiers' degrees), variants used. */
byo_status byo_bc(byo_graph *g, int64_t src, double *d_delta, double *d_sigma, int32_t *d_depth,
                  const byo_opts *opts, void *stream, byo_run_stats *stats);

/* k-core decomposition (Table algs-list, substructure problems): d_core[v] =
 * the coreness of v, the largest k such that v belongs to the k-core (the
 * maximal subgraph in which every vertex keeps at least k neighbours); 0 for
 * isolated vertices. Peeling: at each k, the alive vertices with remaining
 * degree <= k are removed in push sub-rounds (edge-balanced when the
 * frontier's degree sum is at least 2^15 or a list is longer than 16, else
 * one vertex per lane) until
 * none is left, k then jumping to the least remaining degree. d_core: device int32
 * [n]. Returns when done: with opts->persistent (default) every phase runs in
 * one cooperative launch, else the host loop reads each sub-round's size
 * back. BYO_ELIMIT if max_levels sub-rounds do not finish; BYO_EHIP if a
 * grid barrier wait of the persistent launch times out. stats: levels =
 * sub-rounds, edges = sum of the removed vertices' degrees. */
byo_status byo_kcore(byo_graph *g, int32_t *d_core, const byo_opts *opts, void *stream, byo_run_stats *stats);

/* Maximal independent set (Table algs-list, covering problems): the greedy
 * MIS in priority order, the vertices taken in ascending (d_prio[v], v) order,
 * each joining unless a neighbour joined before it. The caller supplies the
 * order (e.g. seeded random 64-bit priorities), so the result is unique for
 * it. Rounds: an undecided vertex is out once an earlier neighbour is in, in
 * once every earlier neighbour is out. d_prio: device uint64 [n];
 * d_in_set: device uint8 [n], 1 = in the set. selector = BYO_SEL_FIXED with
 * a *_THREAD variant scans every list by one lane, else lists longer than 32
 * are shared by the wavefront. Returns when done; BYO_ELIMIT if max_levels
 * rounds do not finish. stats: levels = rounds. */
byo_status byo_mis(byo_graph *g, const uint64_t *d_prio, uint8_t *d_in_set, const byo_opts *opts, void *stream,
                   byo_run_stats *stats);

/* Approximate densest subgraph (Table algs-list, substructure problems):
 * peeling rounds. S starts as every vertex; each round records |S| and
 * |E(S)| and removes every vertex of S with fewer than
 * 2 (1 + eps) |E(S)| / |S| neighbours in S (that test in FP64, exactly as
 * written); the rounds stop when S is empty or edgeless, or when a round
 * removes nothing. *best_edges and
 * *best_vertices = |E(S)| and |S| of the densest S seen (0 and n when no round
 * has an edge), within 2 (1 + eps) of the densest subgraph; d_in_best (device
 * uint8 [n] or NULL) = its membership. eps in [0, 1e6). Returns when done;
 * BYO_ELIMIT if max_levels rounds do not finish. stats: levels = rounds. */
byo_status byo_densest(byo_graph *g, double eps, uint8_t *d_in_best, int64_t *best_edges, int64_t *best_vertices,
                       const byo_opts *opts, void *stream, byo_run_stats *stats);

/* Graph colouring (Table algs-list, covering problems): the greedy colouring
 * in priority order, the vertices taken in ascending (d_prio[v], v) order,
 * each taking the smallest colour (0, 1, ...) no earlier neighbour holds;
 * unique for the order. Rounds: an uncoloured vertex whose earlier neighbours
 * are all coloured takes the least colour missing among them. d_prio: device
 * uint64 [n]; d_color: device int32 [n]. Variants and limits as byo_mis.
 * stats: levels = rounds. */
byo_status byo_coloring(byo_graph *g, const uint64_t *d_prio, int32_t *d_color, const byo_opts *opts, void *stream,
                        byo_run_stats *stats);

/* PageRank, FP32, `iters` steps from 1/n: p'[v] = (1-d)/n + d * (sum over
 * u in N(v) of p[u]/deg(u) + D/n), D = mass on degree-0 vertices. */
byo_status byo_pagerank(byo_graph *g, double damping, int32_t iters, float *d_rank, const byo_opts *opts,
                        void *stream, byo_run_stats *stats);
/* Multi-source BFS from k <= 256 sources, 64 sources per u64 word.
 * d_depth is vertex-major uint8: depth[v * k + j] = hop distance from
 * h_srcs[j] (255 = unreached). BYO_ELIMIT if a distance reaches 255; the
 * contents of d_depth are then unspecified. With tiled = 1 the rows are built
 * from kept per-level frontier masks (see ms_history). */
byo_status byo_msbfs(byo_graph *g, const int64_t *h_srcs, int32_t k, uint8_t *d_depth, const byo_opts *opts,
                     void *stream, byo_run_stats *stats);

/* ------------------------------------------------------------------------
 * Batched execution over many graphs (host CSRs): the graphs are laid out
 * back to back in one device CSR (a disjoint union) and traversed together,
 * so uneven sizes share every launch.
 * ---------------------------------------------------------------------- */
byo_status byo_batch_create(int32_t count, const int64_t *const *h_offs, const int32_t *const *h_nbrs,
                            const int64_t *ns, void *stream, byo_batch **out);
void byo_batch_destroy(byo_batch *b);
byo_status byo_batch_info(const byo_batch *b, int64_t *total_n, int64_t *total_m);
/* Vertex offset of graph i in the concatenated numbering (i in [0, count]). */
byo_status byo_batch_vertex_offset(const byo_batch *b, int32_t i, int64_t *out);
/* BFS in every graph at once: h_srcs[i] is the source of graph i (local ID).
 * Outputs are concatenated: entries [voff(i), voff(i+1)) belong to graph i,
 * parent IDs are local to their graph. d_depth and d_parent: device int32
 * [total_n], caller-owned. Each graph's depths are those of its own BFS
 * (edgeMap levels, Section 3.2) and its parents a valid BFS tree. With
 * opts->persistent (default) the whole search is one cooperative launch that
 * also resets the outputs and places the sources, and the call returns after
 * one read-back of its totals. Errors: BYO_EINVAL for a null argument or a
 * source outside its graph (nothing is launched), BYO_ELIMIT if max_levels
 * levels do not finish the search, BYO_EHIP if a grid barrier wait of the
 * persistent launch times out (the next call resets the barrier). */
byo_status byo_batch_bfs(byo_batch *b, const int64_t *h_srcs, int32_t *d_depth, int32_t *d_parent,
                         const byo_opts *opts, void *stream, byo_run_stats *stats);
/* Connectivity in every graph at once; labels are local IDs. */
byo_status byo_batch_cc(byo_batch *b, int32_t *d_label, const byo_opts *opts, void *stream,
                        byo_run_stats *stats);

#ifdef __cplusplus
}
#endif
#endif /* BYO_H_ */
