// Device pieces shared by the edgeMap kernels over the CSR (edgemap.hip) and
// over the byte-coded CSR (cz.hip): per-level arguments, the BFS and min-label
// functors, and output emission with the per-level counters.
#pragma once

#include "internal.h"

namespace byo {

constexpr int EM_BLOCK = 256;

struct LevelArgs {
  const int64_t *__restrict__ off;
  const int32_t *__restrict__ nbr;
  const int32_t *__restrict__ deg;
  const int32_t *__restrict__ in_ids;
  const uint64_t *__restrict__ in_bits;
  const long long *__restrict__ scan;   // PUSH_EDGE: frontier degree scan
  int64_t k;                            // |U|
  int64_t n, words;
  long long total;                      // PUSH_EDGE: sum of deg(U)
  int32_t *out_ids;                     // sparse output (nullable)
  uint64_t *out_bits;                   // dense output (nullable)
  byo_counters *ctr;
  byo_counters *ctr_clear;
  int32_t t_wave, t_block;
  int32_t no_early_exit;                // pulls scan whole lists (container without early-exit maps)
};

// Serial early-exit scans issue PULL_ILP independent neighbour loads (and
// bitmap probes) per step instead of one dependent chain per neighbour.
constexpr int PULL_ILP = 8;

// First u in nbr[beg, lim) (ascending) whose bit is set in `bits`, else -1.
__device__ __forceinline__ int32_t first_member(const int32_t *__restrict__ nbr, const uint64_t *__restrict__ bits,
                                                int64_t beg, int64_t lim, bool scan_all = false) {
  int32_t first = -1;
  for (int64_t e = beg; e < lim; e += PULL_ILP) {
    int32_t u[PULL_ILP];
    uint64_t w[PULL_ILP];
#pragma unroll
    for (int j = 0; j < PULL_ILP; ++j) u[j] = (e + j < lim) ? nbr[e + j] : -1;
#pragma unroll
    for (int j = 0; j < PULL_ILP; ++j) w[j] = u[j] >= 0 ? bits[u[j] >> 6] : 0ull;
#pragma unroll
    for (int j = 0; j < PULL_ILP; ++j)
      if (first < 0 && ((w[j] >> (u[j] & 63)) & 1ull)) first = u[j];
    if (first >= 0 && !scan_all) return first;  // early exit
  }
  return first;
}

// ---------------------------------------------------------------- functors

// BFS: a vertex is claimed by the first successful CAS of its parent from -1.
struct BfsF {
  int32_t *parent;
  int32_t *depth;
  uint64_t *visited;
  int32_t newdepth;
  static constexpr bool kDenseFromUpdate = false;
  __device__ __forceinline__ int32_t src_value(int32_t u) const { return u; }
  __device__ __forceinline__ bool update(int32_t u, int32_t /*su*/, int32_t v, uint64_t * /*out_bits*/) const {
    uint64_t bit = 1ull << (v & 63);
    if (visited[v >> 6] & bit) return false;
    if (atomicCAS(&parent[v], -1, u) != -1) return false;
    depth[v] = newdepth;
    atomicOr((unsigned long long *)&visited[v >> 6], (unsigned long long)bit);
    return true;
  }
};

// Min-label: lower label[v] to label[u]; a vertex is emitted once per call,
// by whoever first sets its bit in the output bitmap.
struct CcF {
  int32_t *label;
  static constexpr bool kDenseFromUpdate = true;
  __device__ __forceinline__ int32_t src_value(int32_t u) const { return label[u]; }
  __device__ __forceinline__ bool update(int32_t /*u*/, int32_t lu, int32_t v, uint64_t *out_bits) const {
    if (lu >= label[v]) return false;
    int32_t old = atomicMin(&label[v], lu);
    if (lu >= old) return false;
    uint64_t bit = 1ull << (v & 63);
    unsigned long long prev = atomicOr((unsigned long long *)&out_bits[v >> 6], (unsigned long long)bit);
    return !(prev & bit);
  }
};

// ---------------------------------------------------------------- emission

// Emit v if pred. With a sparse output the wavefront reserves slots with one
// atomic; otherwise the count stays in a register (`count`) and is added once
// per workgroup in finish_level: same-address atomics from every wavefront of
// a large grid serialise and would dominate the level.
// The degree of an emitted vertex goes into the level's degree sum and its
// largest degree (the frontier statistics of the next level).
__device__ __forceinline__ void tally_degree(unsigned long long d, unsigned long long &degsum,
                                             unsigned long long &maxdeg) {
  degsum += d;
  maxdeg = d > maxdeg ? d : maxdeg;
}

template <typename F>
__device__ __forceinline__ void emit(const LevelArgs &a, bool pred, int32_t v, unsigned long long &degsum,
                                     unsigned long long &count, unsigned long long &maxdeg) {
  if (a.out_ids)
    wave_append(pred, v, a.out_ids, &a.ctr->count);
  else
    count += pred ? 1ull : 0ull;
  if (pred) {
    if (!F::kDenseFromUpdate && a.out_bits)
      atomicOr((unsigned long long *)&a.out_bits[v >> 6], 1ull << (v & 63));
    tally_degree((unsigned long long)a.deg[v], degsum, maxdeg);
  }
}

// Block maximum; result valid in every thread. All threads must call it.
template <int BLOCK>
__device__ __forceinline__ unsigned long long block_max_u64(unsigned long long v) {
  __shared__ unsigned long long part[BLOCK / BYO_WAVE];
  v = wave_max(v);
  __syncthreads();
  if (lane_id() == 0) part[threadIdx.x / BYO_WAVE] = v;
  __syncthreads();
  unsigned long long r = 0;
#pragma unroll
  for (int i = 0; i < BLOCK / BYO_WAVE; ++i) r = part[i] > r ? part[i] : r;
  return r;
}

template <int BLOCK>
__device__ __forceinline__ void finish_level(const LevelArgs &a, unsigned long long degsum, unsigned long long count,
                                             unsigned long long maxdeg) {
  unsigned long long t = block_sum<unsigned long long, BLOCK>(degsum);
  unsigned long long c = block_sum<unsigned long long, BLOCK>(count);
  unsigned long long mx = block_max_u64<BLOCK>(maxdeg);
  if (threadIdx.x == 0) {
    if (t) atomicAdd(&a.ctr->degsum, t);
    if (c) atomicAdd(&a.ctr->count, c);
    if (mx) atomicMax(&a.ctr->maxdeg, mx);
    if (blockIdx.x == 0 && a.ctr_clear) {
      a.ctr_clear->count = 0;
      a.ctr_clear->degsum = 0;
      a.ctr_clear->aux0 = 0;
      a.ctr_clear->aux1 = 0;
      a.ctr_clear->maxdeg = 0;
    }
  }
}

}  // namespace byo
