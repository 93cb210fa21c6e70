/*
 * CPU ORACLE -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, single-threaded definitions of what the GPU traversal path
 * computes. Only the test suite, the smoke check and the benchmark's CPU
 * baseline leg may load this file's library; the product library never does,
 * and the two share no code (this file includes nothing from the package).
 *
 * Graph model (paper Section 3, "Graphs" and "Graph representations"): an
 * undirected unweighted graph on vertices 0..n-1; an undirected edge (u, v)
 * appears as v in the neighbour set of u and u in the neighbour set of v. The
 * paper's evaluated graphs are symmetrised, unweighted and simple (Section 6.2,
 * graph-size table), so self-pairs are dropped and repeated pairs collapse.
 * Each neighbour set is kept as a sorted growable array (the "sequence of sets"
 * representation of Section 3.1), built directly from the raw pairs.
 *
 * Algorithms (paper Table "algs-list": BFS, Connectivity, PageRank): the paper
 * names them and defers their details to GBBS, so each function computes the
 * plain definition of the result:
 *   - BFS: hop distance from the source via a FIFO queue, plus the discovering
 *     vertex as parent (any BFS parent is valid; the checker below accepts any).
 *   - CC: every vertex labelled with the smallest vertex ID in its component.
 *   - PageRank: T power-iteration steps in FP64 with uniform teleport and the
 *     mass of zero-degree vertices spread uniformly.
 *   - Single-source betweenness (BC): the dependency of the source on every
 *     vertex, delta_s(v) = sum over targets t of sigma_st(v) / sigma_st, where
 *     sigma_st counts shortest s-t paths and sigma_st(v) those through v. Two
 *     forms: the definition summed pair by pair (tiny graphs, to pin the
 *     other), and Brandes' recurrence over the BFS levels.
 *   - MIS: the greedy maximal independent set in a given priority order
 *     (lower priority value first, ties by vertex ID): scan the vertices in
 *     that order and take each one none of whose neighbours was taken.
 *   - Colouring: the greedy colouring in the same kind of priority order: each
 *     vertex in turn takes the smallest colour no earlier neighbour holds.
 *   - Approximate densest subgraph: peeling rounds. S starts as all vertices;
 *     each round records the density |E(S)| / |S| and removes every vertex of
 *     S with fewer than 2 (1 + eps) |E(S)| / |S| neighbours in S; the best
 *     recorded density is the answer (within 2 (1 + eps) of the densest);
 *     the rounds stop when S is empty, has no edge left, or a round removes
 *     nothing (possible when eps = 0 and S is regular).
 *   - Low-diameter decomposition (Miller, Peng and Xu's shifted clustering):
 *     given shifts delta (the exponential draws are an input), vertex v joins
 *     the centre u minimising dist(u, v) - delta[u], ties to the smaller u.
 *     Two forms: that definition pair by pair (small graphs) and one
 *     shifted-start Dijkstra over the unweighted graph.
 *   - k-core: the coreness of every vertex, the largest k such that the vertex
 *     belongs to the k-core (the maximal subgraph whose vertices all keep at
 *     least k neighbours in it). Two forms: the definition, one deletion
 *     fixpoint per k (small graphs, to pin the other), and peeling the vertex
 *     of least remaining degree first with degree buckets.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  int64_t n;
  int64_t m;        /* directed entries = sum of degrees */
  int64_t *len;     /* neighbour-set sizes */
  int64_t *cap;
  int32_t **nb;     /* sorted, unique neighbour sets */
} oracle_graph;

static int push(oracle_graph *g, int64_t u, int32_t v) {
  if (g->len[u] == g->cap[u]) {
    int64_t nc = g->cap[u] ? 2 * g->cap[u] : 4;
    int32_t *p = (int32_t *)realloc(g->nb[u], sizeof(int32_t) * (size_t)nc);
    if (!p) return -1;
    g->nb[u] = p;
    g->cap[u] = nc;
  }
  g->nb[u][g->len[u]++] = v;
  return 0;
}

static int cmp_i32(const void *a, const void *b) {
  int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
  return (x > y) - (x < y);
}

void oracle_graph_free(oracle_graph *g) {
  if (!g) return;
  if (g->nb)
    for (int64_t v = 0; v < g->n; ++v) free(g->nb[v]);
  free(g->nb); free(g->len); free(g->cap); free(g);
}

/* Build neighbour sets from raw pairs: add both directions, skip u == v, then
 * sort every set and drop repeats. Returns NULL on bad input or no memory. */
oracle_graph *oracle_graph_new(int64_t n, int64_t npairs, const int32_t *a, const int32_t *b) {
  if (n < 0 || npairs < 0) return NULL;
  oracle_graph *g = (oracle_graph *)calloc(1, sizeof(oracle_graph));
  if (!g) return NULL;
  g->n = n;
  g->len = (int64_t *)calloc((size_t)(n + 1), sizeof(int64_t));
  g->cap = (int64_t *)calloc((size_t)(n + 1), sizeof(int64_t));
  g->nb = (int32_t **)calloc((size_t)(n + 1), sizeof(int32_t *));
  if (!g->len || !g->cap || !g->nb) { oracle_graph_free(g); return NULL; }
  for (int64_t i = 0; i < npairs; ++i) {
    int64_t u = a[i], v = b[i];
    if (u < 0 || v < 0 || u >= n || v >= n) { oracle_graph_free(g); return NULL; }
    if (u == v) continue;
    if (push(g, u, (int32_t)v) || push(g, v, (int32_t)u)) { oracle_graph_free(g); return NULL; }
  }
  g->m = 0;
  for (int64_t v = 0; v < n; ++v) {
    if (g->len[v] > 1) qsort(g->nb[v], (size_t)g->len[v], sizeof(int32_t), cmp_i32);
    int64_t w = 0;
    for (int64_t i = 0; i < g->len[v]; ++i)
      if (w == 0 || g->nb[v][i] != g->nb[v][w - 1]) g->nb[v][w++] = g->nb[v][i];
    g->len[v] = w;
    g->m += w;
  }
  return g;
}

int64_t oracle_num_vertices(const oracle_graph *g) { return g->n; }
int64_t oracle_num_edges(const oracle_graph *g) { return g->m; }
int64_t oracle_degree(const oracle_graph *g, int64_t v) { return (v >= 0 && v < g->n) ? g->len[v] : -1; }

/* Copy the neighbour set of v into out (up to cap); returns its size. */
int64_t oracle_neighbors(const oracle_graph *g, int64_t v, int32_t *out, int64_t cap) {
  if (v < 0 || v >= g->n) return -1;
  int64_t k = g->len[v] < cap ? g->len[v] : cap;
  if (k > 0) memcpy(out, g->nb[v], sizeof(int32_t) * (size_t)k);
  return g->len[v];
}

/* Write every neighbour set back to back with the running count before each
 * (used by tests to compare container contents; off has n + 1 entries). */
void oracle_export(const oracle_graph *g, int64_t *off, int32_t *nbr) {
  int64_t pos = 0;
  for (int64_t v = 0; v < g->n; ++v) {
    off[v] = pos;
    for (int64_t i = 0; i < g->len[v]; ++i) nbr[pos++] = g->nb[v][i];
  }
  off[g->n] = pos;
}

/* Breadth-first search: depth = hop distance (-1 unreachable), parent = the
 * vertex whose neighbour scan first reached it (src is its own parent). */
int oracle_bfs(const oracle_graph *g, int64_t src, int32_t *depth, int32_t *parent) {
  if (src < 0 || src >= g->n) return -1;
  int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * (size_t)(g->n > 0 ? g->n : 1));
  if (!queue) return -2;
  for (int64_t v = 0; v < g->n; ++v) { depth[v] = -1; parent[v] = -1; }
  int64_t head = 0, tail = 0;
  depth[src] = 0; parent[src] = (int32_t)src;
  queue[tail++] = (int32_t)src;
  while (head < tail) {
    int32_t u = queue[head++];
    for (int64_t i = 0; i < g->len[u]; ++i) {
      int32_t v = g->nb[u][i];
      if (depth[v] == -1) {
        depth[v] = depth[u] + 1;
        parent[v] = u;
        queue[tail++] = v;
      }
    }
  }
  free(queue);
  return 0;
}

/* Connected components: scan vertices in increasing ID order; an unlabelled
 * vertex is the smallest ID of its component, so a BFS from it labels the
 * whole component with its ID. */
int oracle_cc(const oracle_graph *g, int32_t *label) {
  int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * (size_t)(g->n > 0 ? g->n : 1));
  if (!queue) return -2;
  for (int64_t v = 0; v < g->n; ++v) label[v] = -1;
  for (int64_t s = 0; s < g->n; ++s) {
    if (label[s] != -1) continue;
    int64_t head = 0, tail = 0;
    label[s] = (int32_t)s;
    queue[tail++] = (int32_t)s;
    while (head < tail) {
      int32_t u = queue[head++];
      for (int64_t i = 0; i < g->len[u]; ++i) {
        int32_t v = g->nb[u][i];
        if (label[v] == -1) { label[v] = (int32_t)s; queue[tail++] = v; }
      }
    }
  }
  free(queue);
  return 0;
}

/*
 * PageRank, T steps, FP64. Start from p = 1/n. One step:
 *   D     = sum of p[u] over vertices with degree 0,
 *   p'[v] = (1 - d)/n + d * ( sum over neighbours u of v of p[u]/deg(u)  +  D/n ).
 * Sums run sequentially in ascending neighbour order. No convergence test.
 */
int oracle_pagerank(const oracle_graph *g, double d, int32_t T, double *rank) {
  int64_t n = g->n;
  if (n == 0) return 0;
  if (T < 0) return -1;
  double *next = (double *)malloc(sizeof(double) * (size_t)n);
  if (!next) return -2;
  for (int64_t v = 0; v < n; ++v) rank[v] = 1.0 / (double)n;
  for (int32_t t = 0; t < T; ++t) {
    double D = 0.0;
    for (int64_t u = 0; u < n; ++u)
      if (g->len[u] == 0) D += rank[u];
    for (int64_t v = 0; v < n; ++v) {
      double s = 0.0;
      for (int64_t i = 0; i < g->len[v]; ++i) {
        int32_t u = g->nb[v][i];
        s += rank[u] / (double)g->len[u];
      }
      next[v] = (1.0 - d) / (double)n + d * (s + D / (double)n);
    }
    memcpy(rank, next, sizeof(double) * (size_t)n);
  }
  free(next);
  return 0;
}

/* Multi-source BFS as k independent BFS runs. depth is vertex-major:
 * depth[v * k + j] = hop distance from srcs[j], 255 when unreachable.
 * Returns -3 if some finite distance does not fit below 255. */
int oracle_msbfs(const oracle_graph *g, const int64_t *srcs, int32_t k, uint8_t *depth) {
  int64_t n = g->n;
  int32_t *dd = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  int32_t *pp = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  if (!dd || !pp) { free(dd); free(pp); return -2; }
  int rc = 0;
  for (int32_t j = 0; j < k && rc == 0; ++j) {
    rc = oracle_bfs(g, srcs[j], dd, pp);
    for (int64_t v = 0; v < n && rc == 0; ++v) {
      if (dd[v] >= 255) rc = -3;
      depth[v * k + j] = (uint8_t)(dd[v] < 0 ? 255 : dd[v]);
    }
  }
  free(dd); free(pp);
  return rc;
}

/*
 * Check a BFS result (depth, parent) for source src against this graph:
 * depth must equal the true hop distances exactly; parent[src] == src; every
 * other reached v has parent p with (p, v) an edge and depth[p] == depth[v]-1;
 * unreached vertices have depth == parent == -1. Returns the number of
 * violations (0 = valid), -2 on no memory.
 */
int64_t oracle_check_bfs(const oracle_graph *g, int64_t src, const int32_t *depth, const int32_t *parent) {
  int64_t n = g->n, bad = 0;
  int32_t *dd = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  int32_t *pp = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  if (!dd || !pp) { free(dd); free(pp); return -2; }
  if (oracle_bfs(g, src, dd, pp) != 0) { free(dd); free(pp); return -1; }
  for (int64_t v = 0; v < n; ++v) {
    if (depth[v] != dd[v]) { ++bad; continue; }
    if (dd[v] < 0) { bad += (parent[v] != -1); continue; }
    if (v == src) { bad += (parent[v] != (int32_t)src); continue; }
    int32_t p = parent[v];
    if (p < 0 || p >= n || dd[p] != dd[v] - 1) { ++bad; continue; }
    /* (p, v) must be an edge: binary search in the sorted set of v */
    int64_t lo = 0, hi = g->len[v];
    while (lo < hi) {
      int64_t mid = (lo + hi) / 2;
      if (g->nb[v][mid] < p) lo = mid + 1; else hi = mid;
    }
    if (lo >= g->len[v] || g->nb[v][lo] != p) ++bad;
  }
  free(dd); free(pp);
  return bad;
}

/* BFS from src: hop distances (-1 unreachable) and shortest-path counts
 * sigma (1 at src, 0 unreachable), FP64 (exact integers below 2^53). When
 * order is given it receives the vertices in visiting order (nondecreasing
 * distance) and the function returns how many. */
static int64_t bfs_paths(const oracle_graph *g, int64_t src, int32_t *dist, double *sigma, int32_t *order) {
  int32_t *queue = order ? order : (int32_t *)malloc(sizeof(int32_t) * (size_t)(g->n > 0 ? g->n : 1));
  if (!queue) return -2;
  for (int64_t v = 0; v < g->n; ++v) { dist[v] = -1; sigma[v] = 0.0; }
  int64_t head = 0, tail = 0;
  dist[src] = 0;
  sigma[src] = 1.0;
  queue[tail++] = (int32_t)src;
  while (head < tail) {
    int32_t u = queue[head++];
    for (int64_t i = 0; i < g->len[u]; ++i) {
      int32_t v = g->nb[u][i];
      if (dist[v] == -1) { dist[v] = dist[u] + 1; queue[tail++] = v; }
      if (dist[v] == dist[u] + 1) sigma[v] += sigma[u];
    }
  }
  if (!order) free(queue);
  return tail;
}

/* The definition, pair by pair: v lies on a shortest s-t path iff
 * d(s,v) + d(v,t) = d(s,t), and then sigma_st(v) = sigma_sv * sigma_vt. One BFS
 * from every vertex: O(n (n + m)), for small graphs only. delta[s] = 0 and
 * delta[v] = 0 for v unreachable from s. */
int oracle_bc_definition(const oracle_graph *g, int64_t s, double *delta) {
  int64_t n = g->n;
  if (s < 0 || s >= n) return -1;
  int32_t *ds = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  int32_t *dv = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  double *ss = (double *)malloc(sizeof(double) * (size_t)n);
  double *sv = (double *)malloc(sizeof(double) * (size_t)n);
  if (!ds || !dv || !ss || !sv) { free(ds); free(dv); free(ss); free(sv); return -2; }
  bfs_paths(g, s, ds, ss, NULL);
  for (int64_t v = 0; v < n; ++v) {
    delta[v] = 0.0;
    if (v == s || ds[v] < 0) continue;
    bfs_paths(g, v, dv, sv, NULL);
    double sum = 0.0;
    for (int64_t t = 0; t < n; ++t) {
      if (t == s || t == v || ds[t] < 0 || dv[t] < 0) continue;
      if (ds[v] + dv[t] == ds[t]) sum += ss[v] * sv[t] / ss[t];
    }
    delta[v] = sum;
  }
  free(ds); free(dv); free(ss); free(sv);
  return 0;
}

/* Brandes' recurrence: with P(w) the neighbours of w one level closer to s,
 * delta(v) = sum over w with v in P(w) of sigma(v) / sigma(w) * (1 + delta(w)),
 * accumulated over the vertices in reverse visiting order; delta[s] = 0.
 * Also returns sigma (path counts) and the hop distances. */
int oracle_bc(const oracle_graph *g, int64_t s, double *sigma, double *delta, int32_t *dist) {
  int64_t n = g->n;
  if (s < 0 || s >= n) return -1;
  int32_t *order = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  if (!order) return -2;
  int64_t cnt = bfs_paths(g, s, dist, sigma, order);
  for (int64_t v = 0; v < n; ++v) delta[v] = 0.0;
  for (int64_t i = cnt - 1; i >= 0; --i) {
    int32_t w = order[i];
    for (int64_t j = 0; j < g->len[w]; ++j) {
      int32_t v = g->nb[w][j];
      if (dist[v] == dist[w] - 1) delta[v] += sigma[v] / sigma[w] * (1.0 + delta[w]);
    }
  }
  delta[s] = 0.0;
  free(order);
  return 0;
}

/* The definition: for k = 0, 1, 2, ... delete vertices with fewer than k
 * remaining neighbours until none is left to delete; what survives is the
 * k-core, and core[v] is the last k whose core still holds v. O(maxdeg * m)
 * with a full pass per deletion round: small graphs only. */
int oracle_kcore_definition(const oracle_graph *g, int32_t *core) {
  int64_t n = g->n;
  uint8_t *in = (uint8_t *)malloc((size_t)(n > 0 ? n : 1));
  int64_t *d = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  if (!in || !d) { free(in); free(d); return -2; }
  for (int64_t v = 0; v < n; ++v) core[v] = 0;
  for (int64_t k = 1;; ++k) {
    for (int64_t v = 0; v < n; ++v) in[v] = 1;
    int changed = 1;
    while (changed) {
      changed = 0;
      for (int64_t v = 0; v < n; ++v) {
        if (!in[v]) continue;
        int64_t c = 0;
        for (int64_t i = 0; i < g->len[v]; ++i) c += in[g->nb[v][i]];
        d[v] = c;
      }
      for (int64_t v = 0; v < n; ++v)
        if (in[v] && d[v] < k) { in[v] = 0; changed = 1; }
    }
    int64_t left = 0;
    for (int64_t v = 0; v < n; ++v)
      if (in[v]) { core[v] = (int32_t)k; ++left; }
    if (left == 0) break;
  }
  free(in);
  free(d);
  return 0;
}

/* Peeling: repeatedly remove a vertex of least remaining degree; its
 * coreness is the largest such least degree seen so far. Degree buckets
 * (doubly linked lists) make each step O(1) amortised: O(n + m) total. */
int oracle_kcore(const oracle_graph *g, int32_t *core) {
  int64_t n = g->n, maxd = 0;
  for (int64_t v = 0; v < n; ++v) maxd = g->len[v] > maxd ? g->len[v] : maxd;
  int64_t *deg = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  int64_t *head = (int64_t *)malloc(sizeof(int64_t) * (size_t)(maxd + 1));
  int64_t *next = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  int64_t *prev = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  uint8_t *gone = (uint8_t *)calloc((size_t)(n > 0 ? n : 1), 1);
  if (!deg || !head || !next || !prev || !gone) {
    free(deg); free(head); free(next); free(prev); free(gone);
    return -2;
  }
  for (int64_t b = 0; b <= maxd; ++b) head[b] = -1;
  for (int64_t v = 0; v < n; ++v) {  /* push v onto bucket deg[v] */
    deg[v] = g->len[v];
    prev[v] = -1;
    next[v] = head[deg[v]];
    if (head[deg[v]] >= 0) prev[head[deg[v]]] = v;
    head[deg[v]] = v;
  }
  int64_t k = 0, b = 0;
  for (int64_t done = 0; done < n; ++done) {
    while (head[b] < 0) ++b;   /* least nonempty bucket; a removal lowers degrees by at most 1 */
    int64_t v = head[b];
    head[b] = next[v];
    if (next[v] >= 0) prev[next[v]] = -1;
    gone[v] = 1;
    if (b > k) k = b;
    core[v] = (int32_t)k;
    for (int64_t i = 0; i < g->len[v]; ++i) {
      int64_t u = g->nb[v][i];
      if (gone[u]) continue;
      /* move u from bucket deg[u] to deg[u] - 1 */
      if (prev[u] >= 0) next[prev[u]] = next[u]; else head[deg[u]] = next[u];
      if (next[u] >= 0) prev[next[u]] = prev[u];
      --deg[u];
      prev[u] = -1;
      next[u] = head[deg[u]];
      if (head[deg[u]] >= 0) prev[head[deg[u]]] = u;
      head[deg[u]] = u;
    }
    if (b > 0) --b;            /* a neighbour may now sit one bucket lower */
  }
  free(deg); free(head); free(next); free(prev); free(gone);
  return 0;
}

/* Greedy maximal independent set in priority order: the vertices sorted by
 * (prio, id) ascending are visited in turn, and a vertex joins the set when
 * no neighbour has joined before it. in_set[v] = 1 if v joined, else 0. */
static const uint64_t *g_mis_prio;
static int cmp_mis(const void *a, const void *b) {
  int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
  if (g_mis_prio[x] != g_mis_prio[y]) return g_mis_prio[x] < g_mis_prio[y] ? -1 : 1;
  return x < y ? -1 : (x > y);
}
int oracle_mis(const oracle_graph *g, const uint64_t *prio, uint8_t *in_set) {
  int64_t n = g->n;
  int32_t *order = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  if (!order) return -2;
  for (int64_t v = 0; v < n; ++v) { order[v] = (int32_t)v; in_set[v] = 0; }
  g_mis_prio = prio;
  qsort(order, (size_t)n, sizeof(int32_t), cmp_mis);
  for (int64_t i = 0; i < n; ++i) {
    int32_t v = order[i];
    int taken = 0;
    for (int64_t j = 0; j < g->len[v] && !taken; ++j) taken = in_set[g->nb[v][j]];
    in_set[v] = taken ? 0 : 1;
  }
  free(order);
  return 0;
}

/* Greedy colouring in priority order: vertices sorted by (prio, id) ascending
 * take, in turn, the smallest colour (0, 1, ...) that no neighbour coloured
 * before them holds. color[v] >= 0. */
int oracle_coloring(const oracle_graph *g, const uint64_t *prio, int32_t *color) {
  int64_t n = g->n, maxd = 0;
  for (int64_t v = 0; v < n; ++v) maxd = g->len[v] > maxd ? g->len[v] : maxd;
  int32_t *order = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  int64_t *seen = (int64_t *)malloc(sizeof(int64_t) * (size_t)(maxd + 2));
  if (!order || !seen) { free(order); free(seen); return -2; }
  for (int64_t v = 0; v < n; ++v) { order[v] = (int32_t)v; color[v] = -1; }
  for (int64_t c = 0; c < maxd + 2; ++c) seen[c] = -1;
  g_mis_prio = prio;
  qsort(order, (size_t)n, sizeof(int32_t), cmp_mis);
  for (int64_t i = 0; i < n; ++i) {
    int32_t v = order[i];
    for (int64_t j = 0; j < g->len[v]; ++j) {
      int32_t c = color[g->nb[v][j]];
      if (c >= 0) seen[c] = v;   /* colour c is taken around v */
    }
    int32_t c = 0;
    while (seen[c] == v) ++c;
    color[v] = c;
  }
  free(order);
  free(seen);
  return 0;
}

/* Approximate densest subgraph by peeling rounds (see the header). Returns
 * the number of rounds; best_e / best_v = the best density seen (|E(S)| and
 * |S| of that round); in_best[v] = 1 for the vertices of that S. The removal
 * test is computed in FP64 exactly as written: (double)deg_S(v) <
 * 2.0 * (1.0 + eps) * ((double)E / (double)S). */
int64_t oracle_densest(const oracle_graph *g, double eps, int64_t *best_e, int64_t *best_v, uint8_t *in_best) {
  int64_t n = g->n;
  uint8_t *in = (uint8_t *)malloc((size_t)(n > 0 ? n : 1));
  uint8_t *drop = (uint8_t *)malloc((size_t)(n > 0 ? n : 1));
  int64_t *d = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  if (!in || !drop || !d) { free(in); free(drop); free(d); return -2; }
  for (int64_t v = 0; v < n; ++v) { in[v] = 1; in_best[v] = 1; d[v] = g->len[v]; }
  *best_e = 0;
  *best_v = n > 0 ? n : 1;
  int64_t rounds = 0, S = n;
  while (S > 0) {
    int64_t E2 = 0;
    for (int64_t v = 0; v < n; ++v)
      if (in[v]) E2 += d[v];
    const int64_t E = E2 / 2;
    ++rounds;
    /* E / S > best_e / best_v, compared exactly */
    if ((__int128)E * (__int128)(*best_v) > (__int128)(*best_e) * (__int128)S) {
      *best_e = E;
      *best_v = S;
      for (int64_t v = 0; v < n; ++v) in_best[v] = in[v];
    }
    if (E == 0) break;  /* no edge left: nothing would fall below the threshold 0 */
    const double thr = 2.0 * (1.0 + eps) * ((double)E / (double)S);
    int64_t dropped = 0;
    for (int64_t v = 0; v < n; ++v) {
      drop[v] = in[v] && (double)d[v] < thr;
      dropped += drop[v];
    }
    if (dropped == 0) break;  /* a round that removes nothing leaves S as it is */
    for (int64_t v = 0; v < n; ++v) {
      if (!drop[v]) continue;
      in[v] = 0;
      --S;
      for (int64_t i = 0; i < g->len[v]; ++i) {
        int32_t u = g->nb[v][i];
        if (in[u] || drop[u]) --d[u];
      }
    }
  }
  free(in); free(drop); free(d);
  return rounds;
}

/* Low-diameter decomposition, the definition: for every v, the u in v's
 * component minimising dist(u, v) - delta[u] (ties: smaller u); one BFS per
 * u, O(n (n + m)). cluster[v] = that u. */
int oracle_ldd_definition(const oracle_graph *g, const double *delta, int32_t *cluster) {
  int64_t n = g->n;
  int32_t *dist = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  double *sig = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
  double *best = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
  if (!dist || !sig || !best) { free(dist); free(sig); free(best); return -2; }
  for (int64_t v = 0; v < n; ++v) { cluster[v] = -1; best[v] = 0.0; }
  for (int64_t u = 0; u < n; ++u) {
    bfs_paths(g, u, dist, sig, NULL);
    for (int64_t v = 0; v < n; ++v) {
      if (dist[v] < 0) continue;
      double key = (double)dist[v] - delta[u];
      if (cluster[v] < 0 || key < best[v]) { best[v] = key; cluster[v] = (int32_t)u; }
      /* u ascends, so an equal key keeps the smaller centre already there */
    }
  }
  free(dist); free(sig); free(best);
  return 0;
}

/* The same clustering by one Dijkstra: every vertex u enters as its own
 * centre at hop 0; settling v in order of (key, centre) gives each neighbour w
 * the candidate (hop(v) + 1, centre(v)), so each vertex is settled with its
 * least (dist(u, v) - delta[u], u): the predecessor of v on a shortest path
 * from v's best centre has that same centre as its own best. Binary heap,
 * O((n + m) log n). */
/* a candidate: v reached from centre at hop distance dist; its key is
 * (double)dist - delta[centre], computed as in the definition */
typedef struct { int32_t dist; int32_t centre; int32_t v; } ldd_item;
static const double *g_ldd_delta;
static int ldd_less(const ldd_item *a, const ldd_item *b) {
  double ka = (double)a->dist - g_ldd_delta[a->centre], kb = (double)b->dist - g_ldd_delta[b->centre];
  if (ka != kb) return ka < kb;
  return a->centre < b->centre;
}
int oracle_ldd(const oracle_graph *g, const double *delta, int32_t *cluster) {
  int64_t n = g->n, cap = n + g->m + 1, size = 0;
  ldd_item *heap = (ldd_item *)malloc(sizeof(ldd_item) * (size_t)cap);
  uint8_t *done = (uint8_t *)calloc((size_t)(n > 0 ? n : 1), 1);
  if (!heap || !done) { free(heap); free(done); return -2; }
  g_ldd_delta = delta;
  #define LDD_PUSH(D, C, V) do {                                               \
    int64_t i_ = size++;                                                       \
    heap[i_].dist = (D); heap[i_].centre = (C); heap[i_].v = (V);              \
    while (i_ > 0 && ldd_less(&heap[i_], &heap[(i_ - 1) / 2])) {               \
      ldd_item t_ = heap[i_]; heap[i_] = heap[(i_ - 1) / 2]; heap[(i_ - 1) / 2] = t_; \
      i_ = (i_ - 1) / 2;                                                       \
    }                                                                          \
  } while (0)
  for (int64_t v = 0; v < n; ++v) { cluster[v] = -1; LDD_PUSH(0, (int32_t)v, (int32_t)v); }
  while (size > 0) {
    ldd_item top = heap[0];
    heap[0] = heap[--size];
    for (int64_t i = 0;;) {  /* sift down */
      int64_t l = 2 * i + 1, r = l + 1, m = i;
      if (l < size && ldd_less(&heap[l], &heap[m])) m = l;
      if (r < size && ldd_less(&heap[r], &heap[m])) m = r;
      if (m == i) break;
      ldd_item t = heap[i]; heap[i] = heap[m]; heap[m] = t;
      i = m;
    }
    if (done[top.v]) continue;
    done[top.v] = 1;
    cluster[top.v] = top.centre;
    for (int64_t i = 0; i < g->len[top.v]; ++i) {
      int32_t w = g->nb[top.v][i];
      if (!done[w]) LDD_PUSH(top.dist + 1, top.centre, w);
    }
  }
  #undef LDD_PUSH
  free(heap); free(done);
  return 0;
}
