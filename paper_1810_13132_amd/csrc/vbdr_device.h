// Device-side primitives of the VBDR hot path (gfx950).  Internal header of
// libvbdr.so.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vbdr {

typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr int kBins = 33;     // register values 0..32
constexpr uint32_t kSat = 255; // DR saturation value (InitDR with z = 8)

// MurmurHash3_x86_32 of one 4-byte little-endian key: H(x, 2^32, A)
// (Sec. 4.1 leaves the hash family open; this is the chosen member).
__device__ __forceinline__ uint32_t mm3(uint32_t x, uint32_t seed) {
  uint32_t k = x * 0xcc9e2d51u;
  k = (k << 15) | (k >> 17);
  k *= 0x1b873593u;
  uint32_t h = seed ^ k;
  h = (h << 13) | (h >> 19);
  h = h * 5u + 0xe6546b64u;
  h ^= 4u;
  h ^= h >> 16;
  h *= 0x85ebca6bu;
  h ^= h >> 13;
  h *= 0xc2b2ae35u;
  h ^= h >> 16;
  return h;
}

// MurmurHash3_x86_32 split for many seeds over one key: mm3_key(x) is the
// seed-independent block mix, mm3_seeded(mm3_key(x), A) == mm3(x, A).
__device__ __forceinline__ uint32_t mm3_key(uint32_t x) {
  uint32_t k = x * 0xcc9e2d51u;
  k = (k << 15) | (k >> 17);
  return k * 0x1b873593u;
}
__device__ __forceinline__ uint32_t mm3_seeded(uint32_t kmix, uint32_t seed) {
  uint32_t h = seed ^ kmix;
  h = (h << 13) | (h >> 19);
  h = h * 5u + 0xe6546b64u;
  h ^= 4u;
  h ^= h >> 16;
  h *= 0x85ebca6bu;
  h ^= h >> 13;
  h *= 0xc2b2ae35u;
  h ^= h >> 16;
  return h;
}

// H(x, m, A) for m < 2^32: the top 32 bits of the 64-bit product h * m.
__device__ __forceinline__ uint32_t reduce_m(uint32_t h, uint32_t m) { return __umulhi(h, m); }

// (vidx, LBP1) of a bip (Alg. 4/7/9): vidx = left b bits of H(bip, 2^32, A1);
// LBP1 = 1 + leading zeros of the remaining 32-b bits, 33-b when they are all
// zero (the sentinel bit 1 << (b-1) caps the count).
__device__ __forceinline__ void bip_map(uint32_t bip, uint32_t A1, uint32_t b, uint32_t& vidx, uint32_t& rho) {
  uint32_t h = mm3(bip, A1);
  vidx = h >> (32 - b);
  rho = __clz((h << b) | (1u << (b - 1))) + 1;
}

// ---- byte-wise (SWAR) operations on four one-byte DRs held in a uint32 ----

// Saturating increment of every byte (SlideDR): bytes below 255 gain 1.
__host__ __device__ __forceinline__ uint32_t swar_sat_inc(uint32_t x) {
  const uint32_t t = ~x;  // a byte of t is zero exactly where x holds 255
  const uint32_t not_sat = (((t & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | t) & 0x80808080u;
  return x + (not_sat >> 7);
}

// 0xFF in byte j for each set bit j of a 4-bit mask.
__host__ __device__ __forceinline__ uint32_t swar_nibble_to_bytes(uint32_t f4) {
  return ((f4 * 0x00204081u) & 0x01010101u) * 0xFFu;
}

// Bias for swar_le_mask: each byte value v sits in its own 16-bit lane, where
// v + (255 - thr) carries into bit 8 exactly when v > thr.
__host__ __device__ __forceinline__ uint32_t swar_gt_bias(uint32_t thr) { return (0xFFu - thr) * 0x00010001u; }

// 0xFF in every byte whose value is <= thr (thr < 255).
__host__ __device__ __forceinline__ uint32_t swar_le_mask(uint32_t v, uint32_t bias) {
  const uint32_t even = ((((v & 0x00FF00FFu) + bias) >> 8) & 0x00010001u);
  const uint32_t odd = ((((v >> 8) & 0x00FF00FFu) + bias) & 0x01000100u);
  return ((even | odd) ^ 0x01010101u) * 0xFFu;
}

// Bit 7 of every byte whose value is below c, for 1 <= c <= 128 (cc = c in
// every byte): (x | 0x80) - c cannot borrow across bytes, and its bit 7 is
// set exactly when (x & 0x7F) >= c; a byte is below c when neither that bit
// nor its own bit 7 is set.  Four operations against the eight or so of
// swar_le_mask, for windows of k <= 128 slices (active DR: DR < k).
__host__ __device__ __forceinline__ uint32_t swar_lt_bit7(uint32_t x, uint32_t cc) {
  const uint32_t t = (x | 0x80808080u) - cc;
  return ~(x | t) & 0x80808080u;
}

// Four register bytes (<= 32) -> four nibbles min(r, 15), byte j -> bits 4j..4j+3.
__host__ __device__ __forceinline__ uint32_t swar_pack_nibbles(uint32_t r) {
  const uint32_t ge15 = ((r + 0x71717171u) & 0x80808080u) >> 7;  // 1 where r >= 15
  const uint32_t c = (r & ~(ge15 * 0xFFu)) | (ge15 * 0x0Fu);
  const uint32_t t = (c | (c >> 4)) & 0x00FF00FFu;
  return (t & 0xFFu) | ((t >> 8) & 0xFF00u);
}

// HyperLogLog alpha_q (Flajolet et al. 2007).
__device__ __forceinline__ double hll_alpha(double q) {
  if (q == 16.0) return 0.673;
  if (q == 32.0) return 0.697;
  if (q == 64.0) return 0.709;
  return 0.7213 / (1.0 + 1.079 / q);
}

// HyperLogLog estimate of q registers whose harmonic sum is U * 2^-32 and of
// which V are zero; linear counting when the raw estimate is <= 2.5 q.
// Each FP64 operation rounds once (no contraction) so that results are
// reproducible across compilers.
__device__ __forceinline__ double hll_estimate(uint64_t U, uint64_t V, double q) {
#pragma clang fp contract(off)
  double S = (double)U * 0x1p-32;
  double E = hll_alpha(q) * q * q / S;
  if (E <= 2.5 * q && V > 0) E = q * log(q / (double)V);
  return E;
}

// ---- per-item bodies shared by the single-sketch and the batched kernels ----

// Scan one pair (Alg. 7 / Alg. 9 with the hashing of Alg. 4 and getPhyIdx of
// Alg. 3).  Fast layout: set bit pidx of bsLBP1 bit-plane LBP1-1 with a
// device-scope atomic OR; small layout: store 0 into DR[LBP1] of BDR pidx.
// TEST: read first and skip an update that is already made.
template <bool FAST, bool TEST>
__device__ __forceinline__ void scan_pair(uint32_t aip, uint32_t bip, const uint32_t* s1, uint32_t b, uint32_t A1,
                                          uint32_t m, uint8_t* dr, uint64_t mstride, uint32_t* seen,
                                          uint64_t wstride) {
  uint32_t vidx, rho;
  bip_map(bip, A1, b, vidx, rho);
  const uint32_t pidx = reduce_m(mm3(aip, s1[vidx]), m);
  if constexpr (FAST) {
    uint32_t* w = seen + (uint64_t)(rho - 1) * wstride + (pidx >> 5);
    const uint32_t bit = 1u << (pidx & 31);
    if (!TEST || !(*w & bit)) atomicOr(w, bit);
  } else {
    uint8_t* d = dr + (uint64_t)(rho - 1) * mstride + pidx;
    if (!TEST || *d != 0) *d = 0;
  }
}

// scan_pair for N pairs at once (valid where ok[v]): the state words of all N
// are located first and, with TEST, read together, so that the N random reads
// overlap instead of each waiting for the one before.
template <bool FAST, bool TEST, int N>
__device__ __forceinline__ void scan_pairs(const u32x2* p, const bool* ok, const uint32_t* s1, uint32_t b, uint32_t A1,
                                           uint32_t m, uint8_t* dr, uint64_t mstride, uint32_t* seen,
                                           uint64_t wstride) {
  uint64_t off[N];
  uint32_t bit[N];
#pragma unroll
  for (int v = 0; v < N; ++v) {
    off[v] = 0;
    bit[v] = 0;
    if (ok[v]) {
      uint32_t vidx, rho;
      bip_map(p[v].y, A1, b, vidx, rho);
      const uint32_t pidx = reduce_m(mm3(p[v].x, s1[vidx]), m);
      off[v] = FAST ? (uint64_t)(rho - 1) * wstride + (pidx >> 5) : (uint64_t)(rho - 1) * mstride + pidx;
      bit[v] = 1u << (pidx & 31);
    }
  }
  uint32_t cur[N];
#pragma unroll
  for (int v = 0; v < N; ++v) cur[v] = TEST && ok[v] ? (FAST ? seen[off[v]] : (uint32_t)dr[off[v]]) : (FAST ? 0u : 1u);
#pragma unroll
  for (int v = 0; v < N; ++v) {
    if (!ok[v]) continue;
    if constexpr (FAST) {
      if (!(cur[v] & bit[v])) atomicOr(seen + off[v], bit[v]);
    } else {
      if (cur[v] != 0) dr[off[v]] = 0;
    }
  }
}

// Advance 16 consecutive BDRs starting at `base` (a multiple of 16), planes
// visited from LBP1 = L down to 1 with a one-plane prefetch.  Fast layout
// (Alg. 6): slide every DR, zero the DR of the slice's highest LBP1, clear
// bsLBP1.  Small layout (Alg. 8): slide every DR, the window's register read
// before the slide.  Register (Alg. 2): the largest LBP1 whose DR is active,
// DR <= k-1 at the moment the window is read.  R receives the 16 registers
// (byte j of R[w] = BDR base + 4w + j); they are also stored to reg and reg4.
// With 16 BDRs per thread, the two threads sharing a bsLBP1 word are
// adjacent lanes of one wave and both consume it before the even one clears it.
// With `preg` (small layout), also the PCSA run of each BDR, the number of
// consecutive active DRs from LBP1 1 (the lowest inactive LBP1 minus 1),
// stored to preg; P receives the 16 runs like R.
template <bool FAST>
__device__ __forceinline__ void advance_group(uint8_t* dr, uint64_t mstride, uint32_t* seen, uint64_t wstride,
                                              uint8_t* reg, uint8_t* reg4, uint64_t base, uint32_t L,
                                              uint32_t gt_bias, uint32_t R[4], uint8_t* preg = nullptr,
                                              uint32_t* P = nullptr) {
  uint32_t M[4] = {0, 0, 0, 0}, Q[4];
  R[0] = R[1] = R[2] = R[3] = 0;
  Q[0] = Q[1] = Q[2] = Q[3] = L * 0x01010101u;
  uint32_t folded = 0;
  u32x4 dn = *reinterpret_cast<const u32x4*>(dr + (uint64_t)(L - 1) * mstride + base);
  uint32_t sn = 0;
  if constexpr (FAST) sn = seen[(uint64_t)(L - 1) * wstride + (base >> 5)];
  for (int i = (int)L; i >= 1; --i) {
    const u32x4 d = dn;
    const uint32_t s = sn;
    if (i > 1) {
      dn = *reinterpret_cast<const u32x4*>(dr + (uint64_t)(i - 2) * mstride + base);
      if constexpr (FAST) sn = seen[(uint64_t)(i - 2) * wstride + (base >> 5)];
    }
    uint32_t fold = 0;
    if constexpr (FAST) {
      const uint32_t bits = (s >> (base & 31)) & 0xFFFFu;
      fold = bits & ~folded;  // only the slice's highest LBP1 is recorded
      folded |= bits;
    }
    // 16 DRs at 255 with no record this slice stay 255 and none is active:
    // nothing to compute or store (decided from the loaded bytes)
    if ((d[0] & d[1] & d[2] & d[3]) == ~0u && fold == 0u) {
      if (!FAST && preg)
#pragma unroll
        for (int w = 0; w < 4; ++w) Q[w] = (uint32_t)(i - 1) * 0x01010101u;
      continue;
    }
    u32x4 nd;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      const uint32_t x = d[w];
      uint32_t y = swar_sat_inc(x);                                                // SlideDR
      if constexpr (FAST) y &= ~swar_nibble_to_bytes((fold >> (4 * w)) & 0xFu);  // SetDR
      const uint32_t act = swar_le_mask(FAST ? y : x, gt_bias);                   // IsActiveDR
      R[w] |= act & ~M[w] & ((uint32_t)i * 0x01010101u);
      M[w] |= act;
      if (!FAST && preg) Q[w] = (Q[w] & act) | (~act & ((uint32_t)(i - 1) * 0x01010101u));
      nd[w] = y;
    }
    if ((nd[0] ^ d[0]) | (nd[1] ^ d[1]) | (nd[2] ^ d[2]) | (nd[3] ^ d[3]))  // saturated, unset DRs stay 255
      *reinterpret_cast<u32x4*>(dr + (uint64_t)(i - 1) * mstride + base) = nd;
  }
  if (!FAST && preg) {
    *reinterpret_cast<u32x4*>(preg + base) = u32x4{Q[0], Q[1], Q[2], Q[3]};
#pragma unroll
    for (int w = 0; w < 4; ++w) P[w] = Q[w];
  }
  if constexpr (FAST) {
    if ((base & 31) == 0)
      for (uint32_t i = 0; i < L; ++i) seen[(uint64_t)i * wstride + (base >> 5)] = 0;
  }
  *reinterpret_cast<u32x4*>(reg + base) = u32x4{R[0], R[1], R[2], R[3]};
  uint64_t nib = 0;
#pragma unroll
  for (int w = 0; w < 4; ++w) nib |= (uint64_t)swar_pack_nibbles(R[w]) << (16 * w);
  *reinterpret_cast<uint64_t*>(reg4 + base / 2) = nib;
}

// Advance 32 consecutive BDRs starting at `base` (a multiple of 32) as
// advance_group does, with the slice's LBP1 bits of those BDRs also given as
// one word per plane, pm[(i - 1) * pm_stride] bit j <-> BDR base + j (the
// deferred scan records of the tile, gathered in LDS).  Small layout: a set
// bit means DR[i] was set to 0 during the slice (Alg. 9), so it is zeroed
// before the slide.  Fast layout: the bits join bsLBP1 (Alg. 7) and the
// slice's highest LBP1 is set after the slide (Alg. 6).  use_seen: the
// bsLBP1 bit-planes in memory may hold bits too (fast layout); they are
// read and cleared.  dn0, dn1: the 32 DRs of plane L, loaded by the caller
// (so that the load can be issued early).  R receives the 32 registers, byte j
// of R[w] = BDR base + 4w + j; they are also stored to reg and reg4.
template <bool FAST>
__device__ __forceinline__ void advance_group32(uint8_t* dr, uint64_t mstride, uint32_t* seen, uint64_t wstride,
                                                uint8_t* reg, uint8_t* reg4, uint64_t base, uint32_t L,
                                                uint32_t gt_bias, const uint32_t* pm, uint32_t pm_stride,
                                                bool use_seen, u32x4 dn0, u32x4 dn1, uint32_t R[8],
                                                uint8_t* preg = nullptr, uint32_t* P = nullptr,
                                                uint32_t* satw = nullptr, uint32_t sat_in = 0u, uint32_t kk = 0u) {
  uint32_t M[8], Q[8];
#pragma unroll
  for (int w = 0; w < 8; ++w) {
    M[w] = R[w] = 0;
    Q[w] = L * 0x01010101u;
  }
  uint32_t folded = 0;
  uint32_t sn = 0;
  if (FAST && use_seen) sn = seen[(uint64_t)(L - 1) * wstride + (base >> 5)];
  // Loads run ahead of the plane being processed: plane i-2's load is issued
  // before plane i's work.  The buffers rotate by copies, so the compiler
  // waits for that load at the end of the step; about one plane is in flight
  // while a plane is processed.  Deeper lookahead (three planes in fixed
  // registers, bounded buffer loads and stores) measured the same time: the
  // sweep is bound by its streams, not by this latency.
  // Bit r-1 of sat_in: the 32 DR[r] were all 255 after the last advance and
  // nothing but the advance has written DRs since; with no record of this
  // slice in that plane they are 255 now and stay 255, so they are neither
  // loaded nor stored.
  const u32x4 ff = {~0u, ~0u, ~0u, ~0u};
  auto skip = [&](int r) -> bool { return ((sat_in >> (r - 1)) & 1u) && pm[(uint32_t)(r - 1) * pm_stride] == 0u; };
  u32x4 nn0 = ff, nn1 = ff;
  if (L >= 2 && !skip((int)L - 1)) {
    const uint8_t* nx = dr + (uint64_t)(L - 2) * mstride + base;
    nn0 = *reinterpret_cast<const u32x4*>(nx);
    nn1 = *reinterpret_cast<const u32x4*>(nx + 16);
  }
  uint32_t sat_out = 0;
  for (int i = (int)L; i >= 1; --i) {
    const u32x4 d0 = dn0, d1 = dn1;
    const uint32_t s = sn;
    dn0 = nn0, dn1 = nn1;
    if (i > 2) {
      if (skip(i - 2)) {
        nn0 = ff, nn1 = ff;
      } else {
        const uint8_t* nx = dr + (uint64_t)(i - 3) * mstride + base;
        nn0 = *reinterpret_cast<const u32x4*>(nx);
        nn1 = *reinterpret_cast<const u32x4*>(nx + 16);
      }
    }
    if (i > 1 && FAST && use_seen) sn = seen[(uint64_t)(i - 2) * wstride + (base >> 5)];
    const uint32_t bits = s | pm[(uint32_t)(i - 1) * pm_stride];
    uint32_t fold = 0;
    if constexpr (FAST) {
      fold = bits & ~folded;  // only the slice's highest LBP1 is recorded
      folded |= bits;
    }
    // 32 DRs at 255 with no record this slice stay 255, none is active and
    // nothing is stored: the SWAR work below is skipped, by whole waves for
    // most of the high planes.  Decided from the loaded bytes, so it holds
    // whether or not the saturation masks were trusted.
    if (bits == 0u && (d0[0] & d0[1] & d0[2] & d0[3] & d1[0] & d1[1] & d1[2] & d1[3]) == ~0u) {
      sat_out |= 1u << (i - 1);
      if (!FAST && preg)
#pragma unroll
        for (int w = 0; w < 8; ++w) Q[w] = (uint32_t)(i - 1) * 0x01010101u;  // no active DR: the run restarts below
      continue;
    }
    u32x4 nd0, nd1;
    if (kk) {  // k <= 128: the active test on bit 7; M holds bit-7 flags of the BDRs whose register is found
#pragma unroll
      for (int w = 0; w < 8; ++w) {
        uint32_t x = w < 4 ? d0[w] : d1[w - 4];
        if constexpr (!FAST) x &= ~swar_nibble_to_bytes((bits >> (4 * w)) & 0xFu);  // SetDR of the slice
        uint32_t y = swar_sat_inc(x);                                                // SlideDR
        if constexpr (FAST) y &= ~swar_nibble_to_bytes((fold >> (4 * w)) & 0xFu);   // SetDR
        const uint32_t a7 = swar_lt_bit7(FAST ? y : x, kk);                          // IsActiveDR
        R[w] += ((a7 & ~M[w]) >> 7) * (uint32_t)i;  // bytes still 0 take i: no carry between bytes
        M[w] |= a7;
        if (!FAST && preg) {
          const uint32_t act = (a7 >> 7) * 0xFFu;
          Q[w] = (Q[w] & act) | (~act & ((uint32_t)(i - 1) * 0x01010101u));
        }
        if (w < 4) nd0[w] = y; else nd1[w - 4] = y;
      }
    } else {
#pragma unroll
      for (int w = 0; w < 8; ++w) {
        uint32_t x = w < 4 ? d0[w] : d1[w - 4];
        if constexpr (!FAST) x &= ~swar_nibble_to_bytes((bits >> (4 * w)) & 0xFu);  // SetDR of the slice
        uint32_t y = swar_sat_inc(x);                                                // SlideDR
        if constexpr (FAST) y &= ~swar_nibble_to_bytes((fold >> (4 * w)) & 0xFu);   // SetDR
        const uint32_t act = swar_le_mask(FAST ? y : x, gt_bias);                    // IsActiveDR
        R[w] |= act & ~M[w] & ((uint32_t)i * 0x01010101u);
        M[w] |= act;
        if (!FAST && preg) Q[w] = (Q[w] & act) | (~act & ((uint32_t)(i - 1) * 0x01010101u));
        if (w < 4) nd0[w] = y; else nd1[w - 4] = y;
      }
    }
    // a saturated DR that was not set this slice stays 255: vectors that did not
    // change are not written back (most of the high planes, whose DRs are rarely set)
    uint8_t* out = dr + (uint64_t)(i - 1) * mstride + base;
    if ((nd0[0] ^ d0[0]) | (nd0[1] ^ d0[1]) | (nd0[2] ^ d0[2]) | (nd0[3] ^ d0[3])) *reinterpret_cast<u32x4*>(out) = nd0;
    if ((nd1[0] ^ d1[0]) | (nd1[1] ^ d1[1]) | (nd1[2] ^ d1[2]) | (nd1[3] ^ d1[3]))
      *reinterpret_cast<u32x4*>(out + 16) = nd1;
    if ((nd0[0] & nd0[1] & nd0[2] & nd0[3] & nd1[0] & nd1[1] & nd1[2] & nd1[3]) == ~0u) sat_out |= 1u << (i - 1);
  }
  if (satw) *satw = sat_out;  // always: sat_in is 0 when the stored masks were stale
  if (FAST && use_seen)
    for (uint32_t i = 0; i < L; ++i) seen[(uint64_t)i * wstride + (base >> 5)] = 0;
  *reinterpret_cast<u32x4*>(reg + base) = u32x4{R[0], R[1], R[2], R[3]};
  *reinterpret_cast<u32x4*>(reg + base + 16) = u32x4{R[4], R[5], R[6], R[7]};
  if (!FAST && preg) {
    *reinterpret_cast<u32x4*>(preg + base) = u32x4{Q[0], Q[1], Q[2], Q[3]};
    *reinterpret_cast<u32x4*>(preg + base + 16) = u32x4{Q[4], Q[5], Q[6], Q[7]};
#pragma unroll
    for (int w = 0; w < 8; ++w) P[w] = Q[w];
  }
  u32x4 nib;
#pragma unroll
  for (int q = 0; q < 4; ++q) nib[q] = swar_pack_nibbles(R[2 * q]) | (swar_pack_nibbles(R[2 * q + 1]) << 16);
  *reinterpret_cast<u32x4*>(reg4 + base / 2) = nib;
}

// Sum of the four bytes of x when it is below 256.
__device__ __forceinline__ uint32_t byte_sum(uint32_t x) { return (x * 0x01010101u) >> 24; }

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
  uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const uint32_t olo = __shfl_xor(lo, off), ohi = __shfl_xor(hi, off);
    const uint64_t s = ((uint64_t)hi << 32 | lo) + ((uint64_t)ohi << 32 | olo);
    lo = (uint32_t)s, hi = (uint32_t)(s >> 32);
  }
  return (uint64_t)hi << 32 | lo;
}

// Noise-removed estimate (m E_s - g E_m) / (m - g), each operation rounded once.
__device__ __forceinline__ double noise_removed(double Es, double Em, double m, double g) {
#pragma clang fp contract(off)
  return (m * Es - g * Em) / (m - g);
}

// E_m: the HyperLogLog estimate over all m registers from their histogram.
__device__ __forceinline__ double pool_estimate(const unsigned long long* hist, double m) {
  uint64_t U = 0;
  for (int r = 0; r < kBins; ++r) U += (uint64_t)hist[r] << (32 - r);
  return hll_estimate(U, hist[0], m);
}

// Exact harmonic sum U = sum 2^(32-R) and zero count V of one host's g
// registers (getPhyIdx of Alg. 3, register gathers of Alg. 5), summed over
// the wave; kmix = mm3_key(aip).  Every lane returns the totals.  The
// registers are read from their nibble copy reg4, half the bytes of reg, so
// that a larger share of a big pool stays in each XCD's L2; a nibble of 15
// stands for 15 and more and is read again from reg.
template <int UNROLL>
__device__ __forceinline__ void host_harmonic(uint32_t kmix, const uint32_t* s1, uint32_t g, uint32_t m,
                                              const uint8_t* reg4, const uint8_t* reg, int lane, uint64_t& U,
                                              uint32_t& V) {
  U = 0;
  V = 0;
  for (uint32_t i0 = lane; i0 < g; i0 += 64 * UNROLL) {
    uint32_t p[UNROLL], r[UNROLL];
#pragma unroll
    for (int u = 0; u < UNROLL; ++u) {
      const uint32_t i = i0 + 64u * u;
      p[u] = i < g ? reduce_m(mm3_seeded(kmix, s1[i]), m) : 0u;
      r[u] = i < g ? ((uint32_t)reg4[p[u] >> 1] >> ((p[u] & 1u) << 2)) & 0xFu : 255u;
    }
#pragma unroll
    for (int u = 0; u < UNROLL; ++u)
      if (r[u] == 15u) r[u] = reg[p[u]];
#pragma unroll
    for (int u = 0; u < UNROLL; ++u)
      if (r[u] != 255u) {
        U += 1ull << (32 - r[u]);
        V += r[u] == 0;
      }
  }
  U = wave_sum_u64(U);
  V = (uint32_t)wave_sum_u64(V);
}

}  // namespace vbdr
