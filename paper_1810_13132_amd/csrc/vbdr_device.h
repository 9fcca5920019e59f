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

}  // namespace vbdr
