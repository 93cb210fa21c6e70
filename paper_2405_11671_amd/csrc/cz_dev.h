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
constexpr int64_t CZ_PAD = 8;  // readable bytes past the stream's end

// Reads a byte stream front to back through aligned 32-bit loads (one load
// per four bytes instead of one per byte); may read up to 7 bytes past the
// last byte it returns.
struct cz_reader {
  const uint32_t *w;
  uint64_t buf;
  int nb;  // valid bits in buf
  __device__ __forceinline__ void init(const uint8_t *base, int64_t pos) {
    const uint64_t a = (uint64_t)(base + pos);
    w = (const uint32_t *)(a & ~3ull);
    const int sh = (int)(a & 3ull) * 8;
    buf = (uint64_t)(*w++) >> sh;
    nb = 32 - sh;
  }
  __device__ __forceinline__ uint32_t varint() {
    uint32_t x = 0;
    int s = 0;
    while (true) {
      if (nb < 8) {
        buf |= (uint64_t)(*w++) << nb;
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

}  // namespace byo
