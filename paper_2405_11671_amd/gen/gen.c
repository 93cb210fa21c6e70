/*
 * Seeded synthetic graph inputs.
 *
 * This module only draws raw vertex pairs (and source vertices); it holds none
 * of the traversal arithmetic. Both the HIP path (which builds its CSR from
 * these pairs) and the CPU oracle (which builds adjacency lists from the same
 * pairs) consume its output.
 *
 * Random numbers come from SplitMix64 (Steele, Lea and Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014) used as a counter-based
 * generator: draw i of stream s under seed k is the SplitMix64 output mixer
 * applied to (state(k, s) + (i + 1) * golden_gamma). Every draw is therefore a
 * pure function of (seed, stream, index), so generation is parallel and
 * reproducible regardless of thread count.
 *
 * Graph shapes follow the paper's synthetic inputs (Section 6.2, dataset list):
 * Erdos-Renyi uniform pairs, Graph500-style RMAT/Kronecker recursive quadrant
 * sampling with probabilities (a, b, c, d), and a road-like 2D lattice with a
 * fraction of its edges removed.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define GOLDEN_GAMMA 0x9e3779b97f4a7c15ULL

enum { STREAM_ER = 1, STREAM_RMAT = 2, STREAM_PERM = 3, STREAM_GRID_DEL = 4,
       STREAM_SOURCES = 5, STREAM_PARAMS = 6 };

static inline uint64_t sm64_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}

/* Draw `i` of stream `stream` under `seed`. */
uint64_t byogen_draw(uint64_t seed, uint64_t stream, uint64_t i) {
  uint64_t base = sm64_mix(seed * GOLDEN_GAMMA + stream * 0xd1b54a32d192ed03ULL + 0x632be59bd9b4e019ULL);
  return sm64_mix(base + (i + 1) * GOLDEN_GAMMA);
}

/* Uniform double in [0, 1) from the top 53 bits. */
static inline double to_unit(uint64_t r) { return (double)(r >> 11) * (1.0 / 9007199254740992.0); }

/* Uniform integer in [0, bound) by multiply-high (Lemire); bias < bound / 2^64. */
static inline uint64_t to_range(uint64_t r, uint64_t bound) {
  return (uint64_t)(((unsigned __int128)r * bound) >> 64);
}

double byogen_unit(uint64_t seed, uint64_t stream, uint64_t i) { return to_unit(byogen_draw(seed, stream, i)); }

/* Erdos-Renyi: npairs independent uniform (u, v) pairs over [0, n). */
int byogen_er(uint64_t seed, int64_t n, int64_t npairs, int32_t *src, int32_t *dst) {
  if (n <= 0 || n > 2147483647LL || npairs < 0) return -1;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < npairs; ++i) {
    src[i] = (int32_t)to_range(byogen_draw(seed, STREAM_ER, 2 * (uint64_t)i), (uint64_t)n);
    dst[i] = (int32_t)to_range(byogen_draw(seed, STREAM_ER, 2 * (uint64_t)i + 1), (uint64_t)n);
  }
  return 0;
}

/* Seeded Fisher-Yates permutation of [0, n). */
static void make_perm(uint64_t seed, int64_t n, int32_t *perm) {
  for (int64_t i = 0; i < n; ++i) perm[i] = (int32_t)i;
  for (int64_t i = n - 1; i > 0; --i) {
    int64_t j = (int64_t)to_range(byogen_draw(seed, STREAM_PERM, (uint64_t)i), (uint64_t)(i + 1));
    int32_t t = perm[i]; perm[i] = perm[j]; perm[j] = t;
  }
}

/*
 * RMAT / Kronecker sampling: every pair descends `scale` levels of the
 * adjacency matrix, picking quadrant (0,0) with probability a, (0,1) with b,
 * (1,0) with c and (1,1) with d = 1 - a - b - c. With `permute` set the vertex
 * IDs are relabelled by a seeded random permutation, as Graph500 does.
 */
int byogen_rmat(uint64_t seed, int scale, int64_t npairs, double a, double b, double c,
                int permute, int32_t *src, int32_t *dst) {
  if (scale < 1 || scale > 30 || npairs < 0) return -1;
  const double ab = a + b, abc = a + b + c;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < npairs; ++i) {
    uint32_t u = 0, v = 0;
    for (int l = 0; l < scale; ++l) {
      double p = to_unit(byogen_draw(seed, STREAM_RMAT, (uint64_t)i * (uint64_t)scale + (uint64_t)l));
      uint32_t row = p >= ab;                          /* quadrants c, d */
      uint32_t col = (p >= a && p < ab) || p >= abc;   /* quadrants b, d */
      u = (u << 1) | row;
      v = (v << 1) | col;
    }
    src[i] = (int32_t)u;
    dst[i] = (int32_t)v;
  }
  if (permute) {
    int64_t n = (int64_t)1 << scale;
    int32_t *perm = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    if (!perm) return -2;
    make_perm(seed, n, perm);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < npairs; ++i) {
      src[i] = perm[src[i]];
      dst[i] = perm[dst[i]];
    }
    free(perm);
  }
  return 0;
}

/* Number of lattice edges of a rows x cols 4-neighbour grid. */
int64_t byogen_grid_edges(int64_t rows, int64_t cols) {
  return rows * (cols - 1) + (rows - 1) * cols;
}

/*
 * rows x cols lattice, vertex (r, c) = r * cols + c. Edge index e enumerates
 * horizontal edges first (row-major), then vertical ones. Exactly `ndel`
 * distinct edges are deleted, chosen uniformly without replacement by a seeded
 * partial Fisher-Yates shuffle; the survivors are written in index order.
 * Returns the number of pairs written.
 */
int64_t byogen_grid(uint64_t seed, int64_t rows, int64_t cols, int64_t ndel, int32_t *src, int32_t *dst) {
  if (rows < 1 || cols < 1 || rows * cols > 2147483647LL) return -1;
  int64_t E = byogen_grid_edges(rows, cols);
  if (ndel < 0 || ndel > E) return -1;
  uint8_t *dead = (uint8_t *)calloc((size_t)(E > 0 ? E : 1), 1);
  int32_t *idx = (int32_t *)malloc(sizeof(int32_t) * (size_t)(E > 0 ? E : 1));
  if (!dead || !idx) { free(dead); free(idx); return -2; }
  for (int64_t e = 0; e < E; ++e) idx[e] = (int32_t)e;
  for (int64_t i = 0; i < ndel; ++i) {
    int64_t j = i + (int64_t)to_range(byogen_draw(seed, STREAM_GRID_DEL, (uint64_t)i), (uint64_t)(E - i));
    int32_t t = idx[i]; idx[i] = idx[j]; idx[j] = t;
    dead[idx[i]] = 1;
  }
  free(idx);
  int64_t h = rows * (cols - 1), w = 0;
  for (int64_t e = 0; e < E; ++e) {
    if (dead[e]) continue;
    int64_t u, v;
    if (e < h) {
      int64_t r = e / (cols - 1), c = e % (cols - 1);
      u = r * cols + c; v = u + 1;
    } else {
      int64_t f = e - h, r = f / cols, c = f % cols;
      u = r * cols + c; v = u + cols;
    }
    src[w] = (int32_t)u; dst[w] = (int32_t)v; ++w;
  }
  free(dead);
  return w;
}

/*
 * k distinct sources drawn uniformly among vertices that have at least one
 * pair with a different endpoint (non-isolated). Returns how many were found
 * (fewer than k only when there are fewer non-isolated vertices).
 */
int64_t byogen_pick_sources(uint64_t seed, int64_t n, int64_t npairs, const int32_t *src,
                            const int32_t *dst, int64_t k, int64_t *out) {
  if (n <= 0) return 0;
  uint8_t *has = (uint8_t *)calloc((size_t)n, 1);
  uint8_t *taken = (uint8_t *)calloc((size_t)n, 1);
  if (!has || !taken) { free(has); free(taken); return -2; }
  int64_t live = 0;
  for (int64_t i = 0; i < npairs; ++i) {
    if (src[i] == dst[i]) continue;
    if (!has[src[i]]) { has[src[i]] = 1; ++live; }
    if (!has[dst[i]]) { has[dst[i]] = 1; ++live; }
  }
  if (k > live) k = live;
  int64_t got = 0;
  for (uint64_t t = 0; got < k; ++t) {
    int64_t cand = (int64_t)to_range(byogen_draw(seed, STREAM_SOURCES, t), (uint64_t)n);
    if (has[cand] && !taken[cand]) { taken[cand] = 1; out[got++] = cand; }
  }
  free(has); free(taken);
  return got;
}
