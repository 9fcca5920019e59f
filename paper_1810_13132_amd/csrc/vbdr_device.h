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
