// Byte-coded CSR, device side: a sequential reader of byte codes and the
// decoding of one block of a neighbour list. The format (declared with
// byo_cz_build in byo.h) stores each sorted list as blocks of CZ_BLOCK
// neighbours; a block's first neighbour is its signed difference from the
// source vertex (zig-zag mapped), the others their gap to the previous
// neighbour, each as a base-128 byte code, low group first, bit 7 marking
// "more bytes follow" (the paper's difference encoding with byte codes, in
// the blocked form that lets blocks decode independently). A list of nb > 1
// blocks starts with nb - 1 little-endian 32-bit offsets, from the start of
// the list, of blocks 1 .. nb - 1.
#pragma once

#include "internal.h"

namespace byo {

constexpr int32_t CZ_BLOCK = 64;
constexpr int64_t CZ_PAD = 64;  // readable bytes past the stream's end (the reader's look-ahead)
constexpr int32_t CZ_WAVE_MIN = 16;  // a block of more neighbours is worth the whole wavefront's decode

// Reads a byte stream front to back through aligned 32-bit loads issued
// four at a time: the group being consumed (g*) and the next group (n*),
// already in flight, so a lane waits on memory about once per 16 bytes
// rather than once per word. Reads at most 36 bytes past the last byte it
// returns (the stream is padded by CZ_PAD).
struct cz_reader {
  const uint32_t *w;  // next group to load
  uint32_t g0, g1, g2, g3, n0, n1, n2, n3;
  int gi;             // words of g* not yet taken
  uint64_t buf;
  int nb;             // valid bits in buf
  __device__ __forceinline__ void init(const uint8_t *base, int64_t pos) {
    const uint64_t a = (uint64_t)(base + pos);
    w = (const uint32_t *)(a & ~3ull);
    g0 = w[0], g1 = w[1], g2 = w[2], g3 = w[3];
    n0 = w[4], n1 = w[5], n2 = w[6], n3 = w[7];
    w += 8;
    gi = 4;
    const int sh = (int)(a & 3ull) * 8;
    buf = (uint64_t)take() >> sh;
    nb = 32 - sh;
  }
  __device__ __forceinline__ uint32_t take() {
    if (gi == 0) {
      g0 = n0, g1 = n1, g2 = n2, g3 = n3;
      n0 = w[0], n1 = w[1], n2 = w[2], n3 = w[3];
      w += 4;
      gi = 4;
    }
    const uint32_t x = g0;
    g0 = g1, g1 = g2, g2 = g3;
    --gi;
    return x;
  }
  __device__ __forceinline__ uint32_t varint() {
    uint32_t x = 0;
    int s = 0;
    while (true) {
      if (nb < 8) {
        buf |= (uint64_t)take() << nb;
        nb += 32;
      }
      const uint32_t b = (uint32_t)buf & 0xffu;
      buf >>= 8;
      nb -= 8;
      x |= (b & 0x7fu) << s;
      if (!(b & 0x80u)) return x;
      s += 7;
    }
  }
};

__device__ __forceinline__ int32_t cz_unzigzag(uint32_t z) { return (int32_t)(z >> 1) ^ -(int32_t)(z & 1u); }

__host__ __device__ __forceinline__ int32_t cz_nblocks(int32_t d) { return (d + CZ_BLOCK - 1) / CZ_BLOCK; }

// byte position of block j of the list that starts at r and has nb blocks
__device__ __forceinline__ int64_t cz_block_pos(const uint8_t *__restrict__ bytes, int64_t r, int32_t nb, int32_t j) {
  if (j == 0) return r + 4 * (int64_t)(nb - 1);
  const uint8_t *p = bytes + r + 4 * (int64_t)(j - 1);
  return r + (int64_t)((uint32_t)p[0] | ((uint32_t)p[1] << 8) | ((uint32_t)p[2] << 16) | ((uint32_t)p[3] << 24));
}

constexpr int CZ_BATCH = 8;

// Calls fn(u) with the neighbours of v in block j decoded CZ_BATCH at a time
// (u[t] = -1 past the block's end), ascending, so the caller can issue the
// batch's loads together. With EXIT the scan stops after the first batch for
// which fn returns true (and returns true).
template <bool EXIT, typename Fn>
__device__ __forceinline__ bool cz_block_batches(const uint8_t *__restrict__ bytes, int64_t r, int32_t v, int32_t d,
                                                 int32_t nb, int32_t j, Fn &&fn) {
  cz_reader rd;
  rd.init(bytes, cz_block_pos(bytes, r, nb, j));
  const int32_t c = d - j * CZ_BLOCK < CZ_BLOCK ? d - j * CZ_BLOCK : CZ_BLOCK;
  int32_t prev = v + cz_unzigzag(rd.varint());
  for (int32_t i0 = 0; i0 < c; i0 += CZ_BATCH) {
    int32_t u[CZ_BATCH];
#pragma unroll
    for (int t = 0; t < CZ_BATCH; ++t) {
      if (i0 + t < c) {
        if (i0 + t > 0) prev += (int32_t)rd.varint();
        u[t] = prev;
      } else {
        u[t] = -1;
      }
    }
    if (fn(u) && EXIT) return true;
  }
  return false;
}

// Calls fn(u) for the neighbours of v in block j, ascending. With EXIT the
// scan stops at the first u for which fn returns true (and returns true).
template <bool EXIT, typename Fn>
__device__ __forceinline__ bool cz_block_for(const uint8_t *__restrict__ bytes, int64_t r, int32_t v, int32_t d,
                                             int32_t nb, int32_t j, Fn &&fn) {
  cz_reader rd;
  rd.init(bytes, cz_block_pos(bytes, r, nb, j));
  const int32_t c = d - j * CZ_BLOCK < CZ_BLOCK ? d - j * CZ_BLOCK : CZ_BLOCK;
  int32_t u = v + cz_unzigzag(rd.varint());
  if (fn(u) && EXIT) return true;
  for (int32_t i = 1; i < c; ++i) {
    u += (int32_t)rd.varint();
    if (fn(u) && EXIT) return true;
  }
  return false;
}

// ---------------------------------------------------------------- wavefront decode

__device__ __forceinline__ int32_t cz_wave_incl_scan(int32_t x) {
#pragma unroll
  for (int d = 1; d < BYO_WAVE; d <<= 1) {
    const int32_t y = __shfl_up(x, d);
    if (lane_id() >= d) x += y;
  }
  return x;
}

// The whole wavefront decodes block j of a list (starting at byte r, ending
// before byte rend, nb blocks, degree d, source v) at once: lane i returns the
// block's i-th neighbour, or -1 past its end. Every lane calls it with the
// same arguments; lds is this wavefront's 64-entry LDS row.
//
// Each lane loads one aligned dword of the block's bytes; a byte with bit 7
// clear ends a value. A lane assembles the values ending in its dword from an
// 8-byte window (the previous lane's dword and its own: a value has at most 5
// bytes), places them by the wavefront's prefix count of value ends, and a
// prefix sum over the lanes turns the gaps into neighbour ids. A block longer
// than the 256 bytes one pass covers takes a second pass from its first
// undecoded value.
__device__ __forceinline__ int32_t cz_wave_block(const uint8_t *__restrict__ bytes, int64_t r, int64_t rend, int32_t v,
                                                 int32_t d, int32_t nb, int32_t j, int32_t *lds) {
  const int lane = lane_id();
  const int64_t start = cz_block_pos(bytes, r, nb, j);
  const int64_t end = j + 1 < nb ? cz_block_pos(bytes, r, nb, j + 1) : rend;
  const int32_t c = d - j * CZ_BLOCK < CZ_BLOCK ? d - j * CZ_BLOCK : CZ_BLOCK;
  int64_t from = start;  // first byte of this pass (a value boundary)
  int32_t done = 0;      // values placed so far
  while (done < c) {
    const int64_t a0 = from & ~3ll;
    const int64_t wp = a0 + 4 * (int64_t)lane;
    const uint32_t x = wp < end ? *(const uint32_t *)(bytes + wp) : 0u;
    uint32_t tm = 0, bm = 0;  // value ends, and bytes before `from`, in this dword
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int64_t p = wp + k;
      if (p < from) bm |= 1u << k;
      else if (p < end && !((x >> (8 * k)) & 0x80u)) tm |= 1u << k;
    }
    bm |= tm;
    const uint32_t xp = __shfl_up(x, 1);
    uint32_t bmp = __shfl_up(bm, 1);
    if (lane == 0) bmp = 0xfu;  // the bytes before a0 precede `from`
    const uint64_t win = (uint64_t)xp | ((uint64_t)x << 32);
    const uint32_t wb = bmp | (bm << 4);
    const int32_t cnt = __popc(tm);
    const int32_t pre = cz_wave_incl_scan(cnt) - cnt;
    int32_t rank = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if ((tm >> k) & 1u) {
        const int q = 4 + k;
        const uint32_t below = wb & ((1u << q) - 1u);
        const int s0 = below ? 32 - __clz(below) : 0;  // first byte of the value
        uint32_t val = 0;
        for (int t = s0; t <= q; ++t) val |= (uint32_t)((win >> (8 * t)) & 0x7fu) << (7 * (t - s0));
        const int32_t idx = done + pre + rank;
        if (idx < c) lds[idx] = (int32_t)val;
        ++rank;
      }
    }
    const int32_t total = __shfl(pre + cnt, BYO_WAVE - 1);
    done += total;
    if (done < c) {
      // next pass starts after the last value end of this one
      const uint64_t lanes = __ballot(tm != 0);
      const int ll = 63 - __clzll((long long)lanes);
      const uint32_t tml = (uint32_t)__shfl((int32_t)tm, ll);
      from = a0 + 4 * (int64_t)ll + (31 - __clz(tml)) + 1;
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  const int32_t raw = lane < c ? lds[lane] : 0;
  const int32_t x0 = lane == 0 ? v + cz_unzigzag((uint32_t)raw) : raw;
  const int32_t u = cz_wave_incl_scan(x0);
  // the row is read again only after every lane has its value
  __builtin_amdgcn_wave_barrier();
  return lane < c ? u : -1;
}

}  // namespace byo
