/*
 * byo_trace.h -- tracing hooks of the edgeMap library.
 *
 * Two process-wide recorders, both off by default:
 *  - per-level records: one row per edgeMap level of BFS / connectivity /
 *    multi-source BFS (input size, sum of input degrees, chosen variant, output
 *    size and the level's device time from HIP events). They feed the learned
 *    selector's training data and the benchmark's breakdowns. The paper's
 *    protocol times whole runs (Section 6.2, "3 trials plus a warm-up"); this
 *    adds the per-level view the variant selector needs.
 *  - kernel timers: HIP events around every launch of selected kernel families
 *    on the stream that launches them; totals per family.
 * Both add host work (and per-level records add one event wait per level, which
 * the level loop already pays), so timed runs leave them off unless they
 * measure with them on purpose. Not thread-safe against concurrent reconfiguration.
 */
#ifndef BYO_TRACE_H_
#define BYO_TRACE_H_

#include <stdint.h>

#include "byo.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef enum { BYO_ALGO_BFS = 0, BYO_ALGO_CC = 1, BYO_ALGO_MSBFS = 2, BYO_ALGO_BATCH_BFS = 3 } byo_algo;

typedef struct byo_level_record {
  int32_t algo;       /* byo_algo */
  int32_t level;      /* level / round index */
  int32_t variant;    /* byo_variant that ran */
  int32_t dense_in;   /* 1 if the input frontier existed only as a bitmap */
  int64_t n, m;       /* graph size */
  int64_t k;          /* |U| */
  int64_t degsum;     /* sum of deg(U) */
  int64_t unvisited;  /* BFS: vertices not yet reached; CC: n */
  int64_t out_count;  /* |output| */
  int64_t out_degsum; /* sum of deg(output) */
  int64_t max_deg;    /* graph maximum degree */
  double cv;          /* graph degree coefficient of variation */
  float ms;           /* device time of the level, conversions included */
  int32_t max_deg_u;  /* largest degree in U (-1 when the level loop does not know it) */
} byo_level_record;

byo_status byo_trace_enable(int32_t on);
/* Copy up to cap records to out (host) and remove them; *count = copied. */
byo_status byo_trace_read(byo_level_record *out, int64_t cap, int64_t *count);
byo_status byo_trace_pending(int64_t *count);

/* Kernel families timed by the kernel timers. The dense pass of each
 * algorithm counts under *_PULL whether it runs over the CSR or over the tile
 * layout: BYO_K_PR_PULL is the pull kernel or the tile kernel of a PageRank
 * step, BYO_K_PR_CHUNK its heavy-row chunk kernel or tile apply kernel;
 * BYO_K_MSBFS_FINISH the fold after a multi-source push or the tile apply;
 * BYO_K_CC_PULL the pull or the tile pass (tile kernel + apply). */
typedef enum {
  BYO_K_BFS_PUSH = 0, BYO_K_BFS_PULL = 1, BYO_K_CC_PUSH = 2, BYO_K_CC_PULL = 3,
  BYO_K_PR_PULL = 4, BYO_K_PR_CHUNK = 5, BYO_K_MSBFS_PUSH = 6, BYO_K_MSBFS_PULL = 7,
  BYO_K_COMPACT = 8, BYO_K_CC_SHORTCUT = 9, BYO_K_MSBFS_FINISH = 10, BYO_K_SMALL_LOOP = 11,
  BYO_K_MLP = 12, BYO_K_COUNT = 16
} byo_kernel_family;

byo_status byo_ktimer_enable(int32_t on);
/* Families that record while timing is on: bit f for family f (default all).
 * Each timed launch records two events on its stream, which costs host time
 * where the host waits on the device between launches (level loops). */
byo_status byo_ktimer_select(uint32_t mask);
byo_status byo_ktimer_reset(void);
/* Launch count and summed device milliseconds of one family (waits for its events). */
byo_status byo_ktimer_read(int32_t family, int64_t *launches, double *total_ms);

#ifdef __cplusplus
}
#endif
#endif /* BYO_TRACE_H_ */
