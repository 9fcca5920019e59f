// libvbdr.so: gfx950 kernels and C ABI of the VBDR sliding-window host
// cardinality estimator (arXiv:1810.13132).  The ABI is documented in
// include/vbdr.h.
//
// Device layout of a sketch (m BDRs, L = 33 - b LBP1 values):
//   dr    L planes of mstride bytes: plane r-1 holds DR[r] of every BDR, so
//         an advance streams each plane contiguously and a scan update of
//         LBP1 r touches plane r-1 only (most updates hit the small planes
//         r = 1, 2, 3, which stay cache resident);
//   seen  (fast layout) L bit-planes of wstride words: bit p of plane r-1 is
//         the bsLBP1 bit r of BDR p for the open slice (Alg. 7);
//   reg   mstride bytes, the register of each BDR for the last closed window;
//   hist  33 uint64, histogram of reg over the m BDRs;
//   s1    g uint32, the virtual-index seeds s1[i] = H(i, 2^32, A0) (Alg. 3).
// mstride is m rounded up to a multiple of 4096; padding BDRs are never
// scanned (pidx < m), keep DR = 255 and register 0, and are not counted.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "vbdr_internal.h"

using namespace vbdr;

// Pools from 2^24 BDRs take the LDS-tiled estimate by default (measured at
// m = 2^26, g = 1024: tiled 1.65 ms, partitioned 2.39 ms; at m = 2^24,
// g = 2048: tiled 0.60 ms, partitioned 0.80 ms).  Below, the partitioned
// gather's per-XCD ranges are at most 512 KB and stay in the L2s.
constexpr uint64_t kTileDefaultMinM = 1ull << 24;

static vbdr_tuning default_tuning(int layout, uint64_t m) {
  vbdr_tuning t;
  t.scan_test_first = layout == VBDR_LAYOUT_FAST ? 1 : 2;
  t.scan_blocks_per_cu = 16;
  t.est_blocks_per_cu = 64;
  t.scan_binned = 2;  // measured: the direct scan is as fast or faster at 2^26 pairs per slice
  t.est_binned = m >= kTileDefaultMinM ? 3 : 2;
  t.est_parts = 8;
  t.est_bin_hosts = 0;
  t.est_bin_cap = 0;
  t.scan_defer = 1;
  return t;
}

namespace {
thread_local std::string g_err;
}  // namespace

namespace {
// allocations left before the one vbdr_test_fail_alloc makes fail; -1: none fails
std::atomic<int64_t> g_allocs_before_failure{-1};
}  // namespace

hipError_t vbdr_malloc_bytes(void** p, size_t bytes) {
  int64_t left = g_allocs_before_failure.load();
  while (left >= 0 && !g_allocs_before_failure.compare_exchange_weak(left, left - 1)) {
  }
  if (left == 0) {
    *p = nullptr;
    return hipErrorOutOfMemory;
  }
  return hipMalloc(p, bytes);
}

extern "C" int vbdr_test_fail_alloc(int64_t after) {
  g_allocs_before_failure.store(after < 0 ? -1 : after);
  return VBDR_OK;
}

int vbdr_fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

namespace {

// ----------------------------------------------------------------- init

__global__ void k_fill_u32(uint32_t* __restrict__ p, uint64_t n, uint32_t v) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void k_seeds(uint32_t* __restrict__ s1, uint32_t g, uint32_t A0) {
  uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < g) s1[i] = mm3(i, A0);
}

__global__ void k_hist_reset(unsigned long long* __restrict__ hist, unsigned long long first,
                             unsigned long long* __restrict__ psum) {
  if (threadIdx.x < kBins) hist[threadIdx.x] = threadIdx.x == 0 ? first : 0ull;
  if (psum && threadIdx.x == 0) *psum = 0;
}

// Adds the PCSA runs P[0..n) (four per word) of a thread to the pool's sum.
template <int N>
__device__ __forceinline__ void add_pcsa_sum(const uint32_t* P, unsigned long long* psum) {
  uint32_t t = 0;
#pragma unroll
  for (int w = 0; w < N; ++w) t += byte_sum(P[w]);
  const uint64_t s = wave_sum_u64(t);
  if ((threadIdx.x & 63) == 0 && s) atomicAdd(psum, (unsigned long long)s);
}

// ----------------------------------------------------------------- scan
// One pair per lane per step, kScanUnroll independent loads in flight; the
// pair stream is read once (non-temporal).  Fast layout: atomic OR of the
// LBP1 bit (Alg. 7, bsLBP1[LBP1] = 1).  Small layout: byte store DR = 0
// (Alg. 9, SetDR).  Both updates are idempotent, so pair order and repeats
// do not matter (Sec. 4.2).  TEST: read first and skip updates already made.

constexpr int kScanBlock = 256;
constexpr int kScanUnroll = 8;

template <bool FAST, bool STAGE, bool TEST>
__global__ __launch_bounds__(kScanBlock) void k_scan(const u32x2* __restrict__ pairs, uint64_t n,
                                                     const uint32_t* __restrict__ s1g, uint32_t g, uint32_t b,
                                                     uint32_t A1, uint32_t m, uint8_t* __restrict__ dr,
                                                     uint64_t mstride, uint32_t* __restrict__ seen, uint64_t wstride) {
  extern __shared__ uint32_t s1_lds[];
  const uint32_t* s1 = s1g;
  if constexpr (STAGE) {
    for (uint32_t i = threadIdx.x; i < g; i += kScanBlock) s1_lds[i] = s1g[i];
    __syncthreads();
    s1 = s1_lds;
  }
  const uint64_t step = (uint64_t)gridDim.x * kScanBlock * kScanUnroll;
  for (uint64_t base = (uint64_t)blockIdx.x * kScanBlock * kScanUnroll + threadIdx.x; base < n; base += step) {
    u32x2 p[kScanUnroll];
#pragma unroll
    for (int u = 0; u < kScanUnroll; ++u) {
      const uint64_t i = base + (uint64_t)u * kScanBlock;
      p[u] = i < n ? __builtin_nontemporal_load(pairs + i) : u32x2{0u, 0u};
    }
    // hash every pair first, then issue all test reads, then the updates, so
    // that each lane keeps kScanUnroll random accesses in flight
    uint64_t off[kScanUnroll];
    uint32_t bit[kScanUnroll];
    bool ok[kScanUnroll];
#pragma unroll
    for (int u = 0; u < kScanUnroll; ++u) {
      ok[u] = base + (uint64_t)u * kScanBlock < n;
      uint32_t vidx, rho;
      bip_map(p[u].y, A1, b, vidx, rho);
      const uint32_t pidx = reduce_m(mm3(p[u].x, s1[ok[u] ? vidx : 0u]), m);
      if constexpr (FAST) {
        off[u] = (uint64_t)(rho - 1) * wstride + (pidx >> 5);
        bit[u] = 1u << (pidx & 31);
      } else {
        off[u] = (uint64_t)(rho - 1) * mstride + pidx;
      }
    }
    uint32_t cur[kScanUnroll];
#pragma unroll
    for (int u = 0; u < kScanUnroll; ++u) {
      if constexpr (TEST) cur[u] = ok[u] ? (FAST ? seen[off[u]] : (uint32_t)dr[off[u]]) : 0u;
    }
#pragma unroll
    for (int u = 0; u < kScanUnroll; ++u) {
      if (!ok[u]) continue;
      if constexpr (FAST) {
        if (!TEST || !(cur[u] & bit[u])) atomicOr(seen + off[u], bit[u]);
      } else {
        if (!TEST || cur[u] != 0) dr[off[u]] = 0;
      }
    }
  }
}

// ---------------------------------------------------- scan, XCD-binned
// For large pools the direct scan is bound by random accesses that miss
// every L2.  Pass 1 streams the pairs, hashes each once and writes a 4-byte
// record (pidx << 5 | LBP1-1) into one of 8 bins by pool range (the top
// bits of the getPhyIdx hash, as in the partitioned estimate); a block stages
// its records in LDS sorted by bin so that each bin receives one contiguous
// run.  Pass 2 runs bin x on the workgroups dispatched to XCD x (b mod 8), so
// the test-and-set traffic of a pool range stays in one L2.  A record that
// finds its bin full is applied directly in pass 1, so any skew is correct.

constexpr int kBinBlock = 256;
constexpr int kBinPerThread = 16;
constexpr int kBinTile = kBinBlock * kBinPerThread;

__global__ void k_bin_reset(uint32_t* __restrict__ fill) {
  if (threadIdx.x < 8) fill[threadIdx.x] = 0;
}

template <bool FAST, bool STAGE, bool TEST>
__global__ __launch_bounds__(kBinBlock) void k_scan_bin(const u32x2* __restrict__ pairs, uint64_t n,
                                                        const uint32_t* __restrict__ s1g, uint32_t g, uint32_t b,
                                                        uint32_t A1, uint32_t m, uint32_t* __restrict__ bins,
                                                        uint32_t* __restrict__ fill, uint8_t* __restrict__ dr,
                                                        uint64_t mstride, uint32_t* __restrict__ seen,
                                                        uint64_t wstride) {
  extern __shared__ uint32_t s1_lds[];
  __shared__ uint32_t rec_lds[kBinTile];
  __shared__ uint32_t cnt[8], start[9], base[8];
  const uint32_t* s1 = s1g;
  if constexpr (STAGE) {
    for (uint32_t i = threadIdx.x; i < g; i += kBinBlock) s1_lds[i] = s1g[i];
    s1 = s1_lds;
  }
  for (uint64_t tile = (uint64_t)blockIdx.x * kBinTile; tile < n; tile += (uint64_t)gridDim.x * kBinTile) {
    if (threadIdx.x < 8) cnt[threadIdx.x] = 0;
    __syncthreads();
    uint32_t rec[kBinPerThread], slot[kBinPerThread];
    u32x2 p[kBinPerThread];
#pragma unroll
    for (int u = 0; u < kBinPerThread; ++u) {
      const uint64_t i = tile + (uint64_t)u * kBinBlock + threadIdx.x;
      p[u] = i < n ? __builtin_nontemporal_load(pairs + i) : u32x2{0u, 0u};
    }
#pragma unroll
    for (int u = 0; u < kBinPerThread; ++u) {
      const uint64_t i = tile + (uint64_t)u * kBinBlock + threadIdx.x;
      slot[u] = 0xFFFFFFFFu;
      if (i < n) {
        uint32_t vidx, rho;
        bip_map(p[u].y, A1, b, vidx, rho);
        const uint32_t hh = mm3(p[u].x, s1[vidx]);
        rec[u] = (reduce_m(hh, m) << 5) | (rho - 1);
        const uint32_t x = hh >> 29;
        slot[u] = (x << 24) | atomicAdd(&cnt[x], 1u);  // rank within the bin (< 2^13)
      }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      start[0] = 0;
      for (int x = 0; x < 8; ++x) start[x + 1] = start[x] + cnt[x];
    }
    if (threadIdx.x < 8) base[threadIdx.x] = atomicAdd(&fill[threadIdx.x], cnt[threadIdx.x]);
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kBinPerThread; ++u)
      if (slot[u] != 0xFFFFFFFFu) rec_lds[start[slot[u] >> 24] + (slot[u] & 0xFFFFFFu)] = rec[u];
    __syncthreads();
    const uint32_t total = start[8];
    for (uint32_t j = threadIdx.x; j < total; j += kBinBlock) {
      uint32_t x = 0;
      while (j >= start[x + 1]) ++x;
      const uint32_t r = rec_lds[j];
      const uint32_t pos = base[x] + (j - start[x]);
      if (pos < kBinCap) {
        bins[(uint64_t)x * kBinCap + pos] = r;
      } else {  // bin full: apply the update here
        const uint32_t pidx = r >> 5, plane = r & 31u;
        if constexpr (FAST) {
          uint32_t* w = seen + (uint64_t)plane * wstride + (pidx >> 5);
          const uint32_t bit = 1u << (pidx & 31);
          if (!TEST || !(*w & bit)) atomicOr(w, bit);
        } else {
          uint8_t* d = dr + (uint64_t)plane * mstride + pidx;
          if (!TEST || *d != 0) *d = 0;
        }
      }
    }
    __syncthreads();
  }
}

template <bool FAST, bool TEST>
__global__ __launch_bounds__(kScanBlock) void k_scan_apply(const uint32_t* __restrict__ bins,
                                                           const uint32_t* __restrict__ fill, uint8_t* __restrict__ dr,
                                                           uint64_t mstride, uint32_t* __restrict__ seen,
                                                           uint64_t wstride) {
  const uint32_t x = blockIdx.x & 7u;  // workgroups are dispatched round-robin over the 8 XCDs
  const uint32_t per = gridDim.x >> 3;
  const uint32_t count = fill[x] < kBinCap ? fill[x] : kBinCap;
  const uint32_t* rx = bins + (uint64_t)x * kBinCap;
  for (uint32_t j0 = (blockIdx.x >> 3) * kScanBlock * kScanUnroll + threadIdx.x; j0 < count;
       j0 += per * kScanBlock * kScanUnroll) {
    uint32_t r[kScanUnroll];
#pragma unroll
    for (int u = 0; u < kScanUnroll; ++u) {
      const uint32_t j = j0 + u * kScanBlock;
      r[u] = j < count ? __builtin_nontemporal_load(rx + j) : 0u;
    }
#pragma unroll
    for (int u = 0; u < kScanUnroll; ++u) {
      if (j0 + u * kScanBlock >= count) continue;  // every 32-bit value is a valid record
      const uint32_t pidx = r[u] >> 5, plane = r[u] & 31u;
      if constexpr (FAST) {
        uint32_t* w = seen + (uint64_t)plane * wstride + (pidx >> 5);
        const uint32_t bit = 1u << (pidx & 31);
        if (!TEST || !(*w & bit)) atomicOr(w, bit);
      } else {
        uint8_t* d = dr + (uint64_t)plane * mstride + pidx;
        if (!TEST || *d != 0) *d = 0;
      }
    }
  }
}

// -------------------------------------------------------------- advance
// One thread per 16 consecutive BDRs; planes visited from LBP1 = L down to 1.
// Fast layout (Alg. 6): slide every DR, then zero the DR of the highest LBP1
// whose bsLBP1 bit is set, and clear bsLBP1.  Small layout (Alg. 8): slide
// every DR; the window's register is read before the slide.  Register of a
// BDR: the largest LBP1 whose DR is active (Alg. 2), i.e. DR <= k-1 at the
// moment the window is read.  Each block histograms its registers in LDS.

constexpr int kAdvBlock = 256;
constexpr int kAdvBpt = 16;
static_assert(kPad % (kAdvBlock * kAdvBpt) == 0, "plane padding must cover whole advance blocks");

template <bool FAST>
__global__ __launch_bounds__(kAdvBlock) void k_advance(uint8_t* __restrict__ dr, uint64_t mstride,
                                                       uint32_t* __restrict__ seen, uint64_t wstride,
                                                       uint8_t* __restrict__ reg, uint8_t* __restrict__ reg4,
                                                       uint64_t m, uint32_t L, uint32_t thr,
                                                       unsigned long long* __restrict__ hist,
                                                       uint8_t* __restrict__ preg,
                                                       unsigned long long* __restrict__ psum) {
  __shared__ uint32_t lh[kAdvBlock / 64][kBins];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane < kBins) lh[wave][lane] = 0;
  __syncthreads();
  const uint64_t base = ((uint64_t)blockIdx.x * kAdvBlock + threadIdx.x) * kAdvBpt;
  uint32_t R[4], P[4];
  advance_group<FAST>(dr, mstride, seen, wstride, reg, reg4, base, L, swar_gt_bias(thr), R, preg, P);
  if (!FAST && preg) add_pcsa_sum<4>(P, psum);  // padding BDRs have run 0
#pragma unroll
  for (int j = 0; j < kAdvBpt; ++j)
    if (base + j < m) atomicAdd(&lh[wave][(R[j >> 2] >> (8 * (j & 3))) & 0xFFu], 1u);
  __syncthreads();
  if (threadIdx.x < kBins) {
    uint32_t c = 0;
    for (int w = 0; w < kAdvBlock / 64; ++w) c += lh[w][threadIdx.x];
    if (c) atomicAdd(hist + threadIdx.x, (unsigned long long)c);
  }
}

// ------------------------------------------- scan + advance, deferred apply
// For large pools every scan update is a random access that misses every
// cache.  Deferred: the scan only computes each pair's record
// (pidx << 5 | LBP1-1), sorts a chunk of kDeferChunk records by tile of
// kDeferTile BDRs in LDS and appends each tile's share to that tile's record
// run with one atomic per (chunk, tile).  The advance that closes the slice
// runs one workgroup per tile: it ORs the tile's records into per-plane bit
// words in LDS and applies them while it streams the tile's DRs, which it
// reads and writes anyway.  Records beyond a run's capacity are applied by the
// scan itself, as the direct scan would (fast layout: the last word of
// `fill` then tells the advance to read the bsLBP1 planes too).  Updates are
// idempotent (Sec. 4.2), so deferring them to the close of the slice leaves
// the closed state unchanged.

constexpr int kDeferBlock = 1024;
constexpr int kHistCopies = 4;  // register histograms per wave in the deferred advances (a power of two)
constexpr int kDeferPer = 32;
constexpr uint32_t kDeferChunk = kDeferBlock * kDeferPer;
constexpr uint32_t kDeferWords = kDeferTile / 32;  // bit words per plane of a tile
static_assert(kDeferTile == kDeferBlock * 32, "one thread advances 32 BDRs of a tile");
static_assert((kDeferSlots * kDeferTile) % 4 == 0, "record runs start 16-byte aligned");
static_assert(kPad % 32 == 0, "tiles of the deferred advance start on whole bit words");

// Exclusive prefix sums of a[0..n) into out[0..n) by one workgroup of
// BLOCK threads, n <= 4 * BLOCK; wsum holds BLOCK / 64 words.
template <int BLOCK = kDeferBlock>
__device__ void block_exclusive_scan(const uint32_t* a, uint32_t* out, uint32_t n, uint32_t* wsum) {
  const uint32_t per = (n + BLOCK - 1) / BLOCK;
  const uint32_t lo = threadIdx.x * per;
  uint32_t v[4] = {0, 0, 0, 0}, sum = 0;
#pragma unroll
  for (uint32_t j = 0; j < 4; ++j)
    if (j < per && lo + j < n) sum += (v[j] = a[lo + j]);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t inc = sum;  // inclusive scan over the wave
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t t = __shfl_up(inc, d);
    if (lane >= d) inc += t;
  }
  if (lane == 63) wsum[wave] = inc;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t run = 0;
    for (int w = 0; w < BLOCK / 64; ++w) {
      const uint32_t t = wsum[w];
      wsum[w] = run;
      run += t;
    }
  }
  __syncthreads();
  uint32_t off = wsum[wave] + inc - sum;
#pragma unroll
  for (uint32_t j = 0; j < 4; ++j)
    if (j < per && lo + j < n) {
      out[lo + j] = off;
      off += v[j];
    }
  __syncthreads();
}

// Apply one record to the pool: fast layout, set the bsLBP1 bit; small
// layout, SetDR; packed layout (bits != nullptr), clear the DR's z bits.
template <bool FAST>
__device__ __forceinline__ void apply_record(uint32_t rec, uint8_t* dr, uint64_t mstride, uint32_t* seen,
                                             uint64_t wstride, uint32_t* bits, uint32_t z) {
  const uint32_t pidx = rec >> 5, plane = rec & 31u;
  if constexpr (FAST) {
    atomicOr(seen + (uint64_t)plane * wstride + (pidx >> 5), 1u << (pidx & 31));
  } else if (bits) {
    for (uint32_t b = 0; b < z; ++b)
      atomicAnd(bits + ((uint64_t)plane * z + b) * wstride + (pidx >> 5), ~(1u << (pidx & 31)));
  } else {
    dr[(uint64_t)plane * mstride + pidx] = 0;
  }
}

// One chunk of kDeferChunk pairs from c0 on: records (pidx << 5 | LBP1-1),
// counted and ranked per tile in LDS, sorted by tile, appended to the tile
// runs (one 64-bit atomic per (chunk, tile)); records past a run's capacity
// are applied directly and flag the direct update.  LDS: cnt[tiles],
// start[tiles], sorted[kDeferChunk]; s1 points to LDS when staged.
template <bool FAST>
__device__ __forceinline__ void scan_defer_chunk(const u32x2* __restrict__ pairs, uint64_t n, uint64_t c0,
                                                 const uint32_t* s1, uint32_t b, uint32_t A1, uint32_t m,
                                                 uint32_t tiles, uint32_t cap, uint32_t* __restrict__ recs,
                                                 unsigned long long* __restrict__ fill, uint8_t* __restrict__ dr,
                                                 uint64_t mstride, uint32_t* __restrict__ seen, uint64_t wstride,
                                                 uint32_t Lc, uint32_t* __restrict__ bits, uint32_t z, uint32_t* lds,
                                                 uint32_t* wsum) {
  uint32_t* cnt = lds;
  uint32_t* start = lds + tiles;
  uint32_t* sorted = lds + 2 * tiles;
  for (uint32_t t = threadIdx.x; t < tiles; t += kDeferBlock) cnt[t] = 0;
  __syncthreads();
  // records and their ranks within the tile (< kDeferChunk, 16 bits each)
  uint32_t rec[kDeferPer], rank[kDeferPer / 2];
#pragma unroll
  for (int u0 = 0; u0 < kDeferPer; u0 += 8) {
    u32x2 p[8];
#pragma unroll
    for (int v = 0; v < 8; ++v) {
      const uint64_t i = c0 + (uint64_t)(u0 + v) * kDeferBlock + threadIdx.x;
      p[v] = i < n ? __builtin_nontemporal_load(pairs + i) : u32x2{0u, 0u};
    }
#pragma unroll
    for (int v = 0; v < 8; ++v) {
      const int u = u0 + v;
      const uint64_t i = c0 + (uint64_t)u * kDeferBlock + threadIdx.x;
      uint32_t r = 0;
      if (i < n) {
        uint32_t vidx, rho;
        bip_map(p[v].y, A1, b, vidx, rho);
        const uint32_t pidx = reduce_m(mm3(p[v].x, s1[vidx]), m);
        rec[u] = (pidx << 5) | ((rho < Lc ? rho : Lc) - 1);  // LBP1 above Lc is recorded at Lc
        r = atomicAdd(&cnt[pidx / kDeferTile], 1u);
      }
      if (u & 1) rank[u >> 1] |= r << 16;
      else rank[u >> 1] = r;
    }
  }
  __syncthreads();
  block_exclusive_scan(cnt, start, tiles, wsum);
  // one run segment per (chunk, tile); cnt[t] becomes the segment's run offset
  for (uint32_t t = threadIdx.x; t < tiles; t += kDeferBlock) {
    const uint32_t c = cnt[t];
    if (c) {
      const unsigned long long at = atomicAdd(fill + t, (unsigned long long)c);
      cnt[t] = at < cap ? (uint32_t)at : cap;
    }
  }
#pragma unroll
  for (int u = 0; u < kDeferPer; ++u) {
    const uint64_t i = c0 + (uint64_t)u * kDeferBlock + threadIdx.x;
    if (i < n) sorted[start[(rec[u] >> 5) / kDeferTile] + ((rank[u >> 1] >> (16 * (u & 1))) & 0xFFFFu)] = rec[u];
  }
  __syncthreads();
  const uint32_t total = n - c0 < kDeferChunk ? (uint32_t)(n - c0) : kDeferChunk;
  bool direct = false;
  for (uint32_t j = threadIdx.x; j < total; j += kDeferBlock) {
    const uint32_t r = sorted[j];
    const uint32_t t = (r >> 5) / kDeferTile;
    const uint32_t pos = cnt[t] + (j - start[t]);
    if (pos < cap) {
      recs[(uint64_t)t * cap + pos] = r;
    } else {
      apply_record<FAST>(r, dr, mstride, seen, wstride, bits, z);
      direct = true;
    }
  }
  if (direct) fill[tiles] = 1ull;  // fast: the advance reads bsLBP1; small: its saturation masks are stale
  __syncthreads();
}

// LDS: cnt[tiles], start[tiles], sorted[kDeferChunk], then s1 if staged.
template <bool FAST, bool STAGE>
__global__ __launch_bounds__(kDeferBlock) void k_scan_defer(const u32x2* __restrict__ pairs, uint64_t n,
                                                            const uint32_t* __restrict__ s1g, uint32_t g, int stage,
                                                            uint32_t b, uint32_t A1, uint32_t m, uint32_t tiles,
                                                            uint32_t cap, uint32_t* __restrict__ recs,
                                                            unsigned long long* __restrict__ fill,
                                                            uint8_t* __restrict__ dr, uint64_t mstride,
                                                            uint32_t* __restrict__ seen, uint64_t wstride,
                                                            uint32_t Lc, uint32_t* __restrict__ bits, uint32_t z) {
  extern __shared__ uint32_t lds[];
  __shared__ uint32_t wsum[kDeferBlock / 64];
  // the seeds from LDS when staged (a pointer that may point to either makes
  // every seed read a flat load, waited for one at a time)
  uint32_t* s1l = lds + 2 * tiles + kDeferChunk;
  if (STAGE)
    for (uint32_t i = threadIdx.x; i < g; i += kDeferBlock) s1l[i] = s1g[i];
  (void)stage;
  for (uint64_t c0 = (uint64_t)blockIdx.x * kDeferChunk; c0 < n; c0 += (uint64_t)gridDim.x * kDeferChunk)
    scan_defer_chunk<FAST>(pairs, n, c0, STAGE ? s1l : s1g, b, A1, m, tiles, cap, recs, fill, dr, mstride, seen,
                           wstride, Lc, bits, z, lds, wsum);
}

// OR a tile's n records into its LDS bit-planes (plane LBP1-1, bit = BDR in
// the tile).  The run starts 16-byte aligned (its capacity is a multiple of
// 4), so each thread loads quads of records, four quads at a time, before the
// LDS atomics: one load per record, waited for one at a time, left the
// advance bound by load latency.
__device__ __forceinline__ void records_to_planes(const uint32_t* __restrict__ r, uint32_t n, uint32_t* pm) {
  for (uint32_t q0 = threadIdx.x; 4 * q0 < n; q0 += 4 * kDeferBlock) {
    u32x4 v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const uint32_t q = q0 + (uint32_t)u * kDeferBlock;
      v[u] = 4 * q < n ? *reinterpret_cast<const u32x4*>(r + 4 * q) : u32x4{0u, 0u, 0u, 0u};
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const uint32_t q = q0 + (uint32_t)u * kDeferBlock;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        if (4 * q + e < n) {
          const uint32_t rec = v[u][e];
          const uint32_t p = (rec >> 5) & (kDeferTile - 1);
          atomicOr(&pm[(rec & 31u) * kDeferWords + (p >> 5)], 1u << (p & 31));
        }
      }
    }
  }
}

// The deferred advance of one tile by one workgroup: the tile's records
// become L planes of kDeferWords bit words in LDS (pm), then every thread
// slides 32 BDRs; lh holds the wave register histograms.
template <bool FAST>
__device__ __forceinline__ void advance_defer_tile(uint32_t tile, uint8_t* __restrict__ dr, uint64_t mstride,
                                                   uint32_t* __restrict__ seen, uint64_t wstride,
                                                   uint8_t* __restrict__ reg, uint8_t* __restrict__ reg4, uint64_t m,
                                                   uint32_t L, uint32_t thr, unsigned long long* __restrict__ hist,
                                                   const uint32_t* __restrict__ recs,
                                                   unsigned long long* __restrict__ fill, uint32_t cap,
                                                   uint32_t tiles, uint8_t* __restrict__ preg,
                                                   unsigned long long* __restrict__ psum, uint32_t* __restrict__ sat,
                                                   uint32_t* pm, uint32_t (*lh)[kHistCopies][kBins]) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (uint32_t i = threadIdx.x; i < L * kDeferWords; i += kDeferBlock) pm[i] = 0;
  for (int i = lane; i < kHistCopies * kBins; i += 64) (&lh[wave][0][0])[i] = 0;
  const unsigned long long f = fill[tile];
  const uint32_t n = f < cap ? (uint32_t)f : cap;
  const bool use_seen = FAST && fill[tiles] != 0;
  // the saturation masks hold only if no DR changed outside the advance since the last one
  const bool sat_ok = sat != nullptr && fill[tiles] == 0;
  // the top plane's load goes out before the record phase
  const uint64_t base = (uint64_t)tile * kDeferTile + (uint64_t)threadIdx.x * 32;
  const bool live = base < mstride;
  u32x4 top0 = {0u, 0u, 0u, 0u}, top1 = {0u, 0u, 0u, 0u};
  if (live) {
    const uint8_t* top = dr + (uint64_t)(L - 1) * mstride + base;
    top0 = *reinterpret_cast<const u32x4*>(top);
    top1 = *reinterpret_cast<const u32x4*>(top + 16);
  }
  __syncthreads();
  if (threadIdx.x == 0) fill[tile] = 0;  // every thread has read it
  const uint32_t* r = recs + (uint64_t)tile * cap;
  records_to_planes(r, n, pm);
  __syncthreads();
  uint32_t P[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  if (live) {
    uint32_t R[8];
    uint32_t* satw = sat ? sat + (base >> 5) : nullptr;
    // windows of k <= 128 slices take the bit-7 active test (swar_lt_bit7)
    const uint32_t kk = thr < 128u ? (thr + 1u) * 0x01010101u : 0u;
    advance_group32<FAST>(dr, mstride, seen, wstride, reg, reg4, base, L, swar_gt_bias(thr), pm + threadIdx.x,
                          kDeferWords, use_seen, top0, top1, R, preg, P, satw, sat_ok ? *satw : 0u, kk);
#pragma unroll
    for (int j = 0; j < 32; ++j)
      if (base + j < m) atomicAdd(&lh[wave][lane & (kHistCopies - 1)][(R[j >> 2] >> (8 * (j & 3))) & 0xFFu], 1u);
  }
  if (!FAST && preg) add_pcsa_sum<8>(P, psum);  // every lane of the wave takes part
  __syncthreads();
  if (threadIdx.x < kBins) {
    uint32_t c = 0;
    for (int w = 0; w < kDeferBlock / 64; ++w)
      for (int q = 0; q < kHistCopies; ++q) c += lh[w][q][threadIdx.x];
    if (c) atomicAdd(hist + threadIdx.x, (unsigned long long)c);
  }
}

// One workgroup per tile; LDS: L planes of kDeferWords bit words.
template <bool FAST>
__global__ __launch_bounds__(kDeferBlock) void k_advance_defer(uint8_t* __restrict__ dr, uint64_t mstride,
                                                               uint32_t* __restrict__ seen, uint64_t wstride,
                                                               uint8_t* __restrict__ reg, uint8_t* __restrict__ reg4,
                                                               uint64_t m, uint32_t L, uint32_t thr,
                                                               unsigned long long* __restrict__ hist,
                                                               const uint32_t* __restrict__ recs,
                                                               unsigned long long* __restrict__ fill, uint32_t cap,
                                                               uint32_t tiles, uint8_t* __restrict__ preg,
                                                               unsigned long long* __restrict__ psum,
                                                               uint32_t* __restrict__ sat) {
  extern __shared__ uint32_t pm[];
  // four copies of each wave's register histogram (lane & 3): registers crowd a
  // few values, and lanes adding to one LDS word are served one at a time
  __shared__ uint32_t lh[kDeferBlock / 64][kHistCopies][kBins];
  advance_defer_tile<FAST>(blockIdx.x, dr, mstride, seen, wstride, reg, reg4, m, L, thr, hist, recs, fill, cap, tiles,
                           preg, psum, sat, pm, lh);
}

// ------------------------------------------- batches: members with record runs
// Batch members whose pools take deferred scans (2^22..2^26 BDRs) are scanned
// and advanced by these two kernels instead of the batch's direct-update
// ones: every deferred member's chunks of kDeferChunk pairs in one persistent
// launch (items strided over the grid), then every member's tiles in one
// launch (one workgroup per tile).  Inputs come from the device table.

// Last member s whose first item is <= item (members without items share
// their successor's first item).
__device__ __forceinline__ uint32_t defer_member(const uint32_t* first, uint32_t S, uint32_t item) {
  uint32_t lo = 0, hi = S - 1;
  while (lo < hi) {
    const uint32_t mid = (lo + hi + 1) >> 1;
    if (first[mid] <= item) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// LDS: cnt[max tiles], start[max tiles], sorted[kDeferChunk].
__global__ __launch_bounds__(kDeferBlock) void k_batch_scan_defer(const DeferItem* __restrict__ it,
                                                                  const DeferHdr* __restrict__ hdr, uint32_t S) {
  extern __shared__ uint32_t lds[];
  __shared__ uint32_t wsum[kDeferBlock / 64];
  __shared__ uint32_t first[kMaxDeferMembers];
  for (uint32_t s = threadIdx.x; s < S; s += kDeferBlock) first[s] = it[s].scan_item0;
  __syncthreads();
  const uint32_t total = hdr->scan_total;
  for (uint32_t item = blockIdx.x; item < total; item += gridDim.x) {
    const DeferItem& D = it[defer_member(first, S, item)];
    const uint64_t c0 = (uint64_t)(item - D.scan_item0) * kDeferChunk;
    const u32x2* pairs = reinterpret_cast<const u32x2*>(D.pairs);
    if (D.layout == VBDR_LAYOUT_FAST)
      scan_defer_chunk<true>(pairs, D.n_pairs, c0, D.s1, D.b, D.A1, (uint32_t)D.m, D.tiles, D.cap, D.recs, D.fill,
                             D.dr, D.mstride, D.seen, D.wstride, D.L, nullptr, 0u, lds, wsum);
    else
      scan_defer_chunk<false>(pairs, D.n_pairs, c0, D.s1, D.b, D.A1, (uint32_t)D.m, D.tiles, D.cap, D.recs, D.fill,
                              D.dr, D.mstride, D.seen, D.wstride, D.L, nullptr, 0u, lds, wsum);
  }
}

// One workgroup per tile of every member; LDS: max L planes of kDeferWords words.
__global__ __launch_bounds__(kDeferBlock) void k_batch_advance_defer(const DeferItem* __restrict__ it, uint32_t S) {
  extern __shared__ uint32_t pm[];
  __shared__ uint32_t lh[kDeferBlock / 64][kHistCopies][kBins];
  __shared__ uint32_t first[kMaxDeferMembers];
  for (uint32_t s = threadIdx.x; s < S; s += kDeferBlock) first[s] = it[s].adv_item0;
  __syncthreads();
  const DeferItem& D = it[defer_member(first, S, blockIdx.x)];
  const uint32_t tile = blockIdx.x - D.adv_item0;
  if (D.layout == VBDR_LAYOUT_FAST)
    advance_defer_tile<true>(tile, D.dr, D.mstride, D.seen, D.wstride, D.reg, D.reg4, D.m, D.L, D.thr, D.hist, D.recs,
                             D.fill, D.cap, D.tiles, nullptr, nullptr, D.sat, pm, lh);
  else
    advance_defer_tile<false>(tile, D.dr, D.mstride, D.seen, D.wstride, D.reg, D.reg4, D.m, D.L, D.thr, D.hist,
                              D.recs, D.fill, D.cap, D.tiles, nullptr, nullptr, D.sat, pm, lh);
}

// After every tile has read it: clear each member's direct-update flag.
__global__ void k_batch_defer_flag(const DeferItem* __restrict__ it, uint32_t S) {
  for (uint32_t s = threadIdx.x; s < S; s += blockDim.x) it[s].fill[it[s].tiles] = 0ull;
}

// Packed layout (Table 1's recorder sizes): DR r of BDR p is a z-bit counter
// stored bit-sliced, bit b in bit-plane (r - 1) z + b at word p / 32, so one
// 32-bit word holds one bit of 32 BDRs and every DR operation is a handful of
// bitwise operations on z words.  One workgroup per tile, as k_advance_defer:
// the tile's records become per-plane bit words in LDS, then thread t sweeps
// word t of every plane from LBP1 Lc down to 1: SetDR of the slice's records
// (clear z bits), the window read (value < k, compared from the top bit down;
// Alg. 2 takes the highest active LBP1), SlideDR (saturating increment by a
// ripple carry; all-ones saturates).
__global__ __launch_bounds__(kDeferBlock) void k_advance_packed(uint32_t* __restrict__ bits, uint64_t wstride,
                                                                uint32_t z, uint32_t Lc, uint32_t k,
                                                                uint8_t* __restrict__ reg, uint8_t* __restrict__ reg4,
                                                                uint64_t m, unsigned long long* __restrict__ hist,
                                                                const uint32_t* __restrict__ recs,
                                                                unsigned long long* __restrict__ fill, uint32_t cap,
                                                                uint32_t tiles, uint32_t* __restrict__ sat) {
  extern __shared__ uint32_t pm[];
  // four copies of each wave's register histogram (lane & 3): registers crowd a
  // few values, and lanes adding to one LDS word are served one at a time
  __shared__ uint32_t lh[kDeferBlock / 64][kHistCopies][kBins];
  const uint32_t tile = blockIdx.x;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (uint32_t i = threadIdx.x; i < Lc * kDeferWords; i += kDeferBlock) pm[i] = 0;
  for (int i = lane; i < kHistCopies * kBins; i += 64) (&lh[wave][0][0])[i] = 0;
  const unsigned long long f = fill[tile];
  const uint32_t n = f < cap ? (uint32_t)f : cap;
  // the saturation masks hold only if no DR changed outside the advance since the last one
  const bool sat_ok = sat != nullptr && fill[tiles] == 0;
  __syncthreads();
  if (threadIdx.x == 0) fill[tile] = 0;  // every thread has read it
  const uint32_t* r = recs + (uint64_t)tile * cap;
  records_to_planes(r, n, pm);
  __syncthreads();
  const uint64_t w = (uint64_t)tile * kDeferWords + threadIdx.x;
  if (w < wstride) {
    uint32_t R[8] = {0, 0, 0, 0, 0, 0, 0, 0}, done = 0;
    // bit rr-1: the 32 DR[rr] were all 2^z - 1 after the last advance; with no
    // record of this slice they still are and stay so: not loaded, not stored
    const uint32_t sat_in = sat_ok ? sat[w] : 0u;
    uint32_t sat_out = 0;
    auto skip = [&](int rr) -> bool {
      return ((sat_in >> (rr - 1)) & 1u) && pm[(uint32_t)(rr - 1) * kDeferWords + threadIdx.x] == 0u;
    };
    uint32_t dn[8];  // the next recorder's words load while this one is processed
    const bool skip_top = skip((int)Lc);
#pragma unroll
    for (int b = 0; b < 8; ++b)
      dn[b] = (uint32_t)b < z ? (skip_top ? ~0u : bits[((uint64_t)(Lc - 1) * z + b) * wstride + w]) : 0u;
    for (int rr = (int)Lc; rr >= 1; --rr) {
      const uint64_t pb = (uint64_t)(rr - 1) * z;
      uint32_t d[8], o[8];  // o: the words as loaded
#pragma unroll
      for (int b = 0; b < 8; ++b) d[b] = o[b] = dn[b];
      if (rr > 1) {
        const bool sk = skip(rr - 1);
#pragma unroll
        for (int b = 0; b < 8; ++b) dn[b] = (uint32_t)b < z ? (sk ? ~0u : bits[(pb - z + b) * wstride + w]) : 0u;
      }
      const uint32_t set = pm[(uint32_t)(rr - 1) * kDeferWords + threadIdx.x];
      {  // 32 DRs at 2^z - 1 (>= k: inactive) with no record stay so and are not stored
        uint32_t all = ~0u;
#pragma unroll
        for (int b = 0; b < 8; ++b)
          if ((uint32_t)b < z) all &= d[b];
        if (set == 0u && all == ~0u) {
          sat_out |= 1u << (rr - 1);
          continue;
        }
      }
#pragma unroll
      for (int b = 0; b < 8; ++b) d[b] &= ~set;  // SetDR (Alg. 9) of the slice
      uint32_t lt = 0, eq = ~0u;                   // IsActiveDR: value < k
#pragma unroll
      for (int b = 7; b >= 0; --b) {
        if ((uint32_t)b >= z) continue;
        if ((k >> b) & 1u) {
          lt |= eq & ~d[b];
          eq &= d[b];
        } else {
          eq &= ~d[b];
        }
      }
      const uint32_t newly = lt & ~done;  // Alg. 2: the highest active LBP1
      done |= lt;
#pragma unroll
      for (int q = 0; q < 8; ++q) R[q] |= swar_nibble_to_bytes((newly >> (4 * q)) & 0xFu) & ((uint32_t)rr * 0x01010101u);
      uint32_t full = ~0u;  // SlideDR: saturating increment
#pragma unroll
      for (int b = 0; b < 8; ++b)
        if ((uint32_t)b < z) full &= d[b];
      uint32_t carry = ~full;
#pragma unroll
      for (int b = 0; b < 8; ++b) {
        if ((uint32_t)b >= z) continue;
        const uint32_t t = d[b] & carry;
        d[b] ^= carry;
        carry = t;
        if (d[b] != o[b]) bits[(pb + b) * wstride + w] = d[b];  // saturated, unset words stay as they are
      }
      uint32_t all = ~0u;
#pragma unroll
      for (int b = 0; b < 8; ++b)
        if ((uint32_t)b < z) all &= d[b];
      if (all == ~0u) sat_out |= 1u << (rr - 1);
    }
    if (sat) sat[w] = sat_out;
    const uint64_t base = w * 32;
    *reinterpret_cast<u32x4*>(reg + base) = u32x4{R[0], R[1], R[2], R[3]};
    *reinterpret_cast<u32x4*>(reg + base + 16) = u32x4{R[4], R[5], R[6], R[7]};
    u32x4 nib;
#pragma unroll
    for (int q = 0; q < 4; ++q) nib[q] = swar_pack_nibbles(R[2 * q]) | (swar_pack_nibbles(R[2 * q + 1]) << 16);
    *reinterpret_cast<u32x4*>(reg4 + base / 2) = nib;
#pragma unroll
    for (int j = 0; j < 32; ++j)
      if (base + j < m) atomicAdd(&lh[wave][lane & (kHistCopies - 1)][(R[j >> 2] >> (8 * (j & 3))) & 0xFFu], 1u);
  }
  __syncthreads();
  if (threadIdx.x < kBins) {
    uint32_t c = 0;
    for (int v = 0; v < kDeferBlock / 64; ++v)
      for (int q = 0; q < kHistCopies; ++q) c += lh[v][q][threadIdx.x];
    if (c) atomicAdd(hist + threadIdx.x, (unsigned long long)c);
  }
}

// Apply the pending records of every tile to the pool (before a state export
// or a switch to direct scans): one workgroup per tile.
template <bool FAST>
__global__ __launch_bounds__(256) void k_defer_flush(const uint32_t* __restrict__ recs,
                                                     unsigned long long* __restrict__ fill, uint32_t cap,
                                                     uint32_t tiles, uint8_t* __restrict__ dr, uint64_t mstride,
                                                     uint32_t* __restrict__ seen, uint64_t wstride,
                                                     uint32_t* __restrict__ bits, uint32_t z) {
  const uint32_t tile = blockIdx.x;
  const unsigned long long f = fill[tile];
  const uint32_t n = f < cap ? (uint32_t)f : cap;
  for (uint32_t j = threadIdx.x; j < n; j += 256)
    apply_record<FAST>(recs[(uint64_t)tile * cap + j], dr, mstride, seen, wstride, bits, z);
  __syncthreads();
  if (threadIdx.x == 0) {
    fill[tile] = 0;
    if (n) fill[tiles] = 1ull;
  }
}

// Clear the direct-update flag after the advance (all tiles have read it), or
// set it when bsLBP1 planes may hold bits the records do not know of.
__global__ void k_defer_flag(unsigned long long* __restrict__ fill, uint32_t tiles, unsigned long long v) {
  if (threadIdx.x == 0) fill[tiles] = v;
}

// ------------------------------------------------------------- estimate
// One wave per host: each lane hashes g/64 virtual indices (getPhyIdx,
// Alg. 3), gathers their registers (Alg. 5) and accumulates the exact
// harmonic sum U = sum 2^(32-R) and the zero count V; a wave reduction and an
// FP64 epilogue give E_s, and with the pool estimate E_m the noise-removed
// (m E_s - g E_m) / (m - g), clamped at 0.

constexpr int kEstBlock = 256;
constexpr int kEstWaves = kEstBlock / 64;

constexpr int kEstUnroll = 8;  // gathers in flight per lane

template <bool STAGE, bool EXTRA>
__global__ __launch_bounds__(kEstBlock) void k_estimate(const uint32_t* __restrict__ hosts, uint64_t nh,
                                                        const uint32_t* __restrict__ s1g, uint32_t g, uint32_t m,
                                                        const uint8_t* __restrict__ reg,
                                                        const unsigned long long* __restrict__ hist,
                                                        float* __restrict__ out, double* __restrict__ raw,
                                                        uint32_t* __restrict__ hout) {
  extern __shared__ uint32_t s1_lds[];
  __shared__ double em_sh;
  __shared__ uint32_t lh[kEstWaves][kBins];
  const uint32_t* s1 = s1g;
  if constexpr (STAGE) {
    for (uint32_t i = threadIdx.x; i < g; i += kEstBlock) s1_lds[i] = s1g[i];
    s1 = s1_lds;
  }
  if (threadIdx.x == 0) {
    uint64_t U = 0;
    for (int r = 0; r < kBins; ++r) U += (uint64_t)hist[r] << (32 - r);
    em_sh = hll_estimate(U, hist[0], (double)m);
  }
  __syncthreads();
  const double Em = em_sh;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (uint64_t h = (uint64_t)blockIdx.x * kEstWaves + wave; h < nh; h += (uint64_t)gridDim.x * kEstWaves) {
    const uint32_t kmix = mm3_key(hosts[h]);  // seed-independent half of H(aip, m, s1[i])
    if constexpr (EXTRA) {
      if (lane < kBins) lh[wave][lane] = 0;
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
    }
    uint64_t U = 0;
    uint32_t V = 0;
    for (uint32_t i0 = lane; i0 < g; i0 += 64 * kEstUnroll) {
      uint32_t r[kEstUnroll];
#pragma unroll
      for (int u = 0; u < kEstUnroll; ++u) {
        const uint32_t i = i0 + 64u * u;
        r[u] = i < g ? (uint32_t)reg[reduce_m(mm3_seeded(kmix, s1[i]), m)] : 255u;
      }
#pragma unroll
      for (int u = 0; u < kEstUnroll; ++u) {
        if (r[u] != 255u) {
          U += 1ull << (32 - r[u]);
          V += r[u] == 0;
          if constexpr (EXTRA) atomicAdd(&lh[wave][r[u]], 1u);
        }
      }
    }
    U = wave_sum_u64(U);
    V = (uint32_t)wave_sum_u64(V);
    if (lane == 0) {
      const double Es = hll_estimate(U, V, (double)g);
      const double n = noise_removed(Es, Em, (double)m, (double)g);
      out[h] = (float)(n > 0.0 ? n : 0.0);
      if (EXTRA && raw) raw[h] = Es;
    }
    if constexpr (EXTRA) {
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      __builtin_amdgcn_wave_barrier();
      if (hout && lane < kBins) hout[h * kBins + lane] = lh[wave][lane];
      __builtin_amdgcn_wave_barrier();
    }
  }
}

// ------------------------------------------- estimate, XCD-partitioned
// The register array of a large pool does not fit one XCD's L2, so direct
// gathers pull a whole line from the memory side per byte used.  Here the
// pool is split into `parts` contiguous ranges by the top bits of the
// getPhyIdx hash; workgroup b (dispatched to XCD b mod 8) hashes every
// (host, i) but gathers only those landing in range b mod parts, from the
// nibble copy of the registers, whose range share stays L2 resident.  The
// per-range partial sums are combined by k_estimate_final.  The sums are
// exact integers, so the result equals the direct kernel's bit for bit.

// The gathers of one host that land in pool range x: all elements hashed
// first, then every taken gather issued before any use, so that a wave keeps
// kEstUnroll gathers in flight.  GUARD: g is not a multiple of 64 * kEstUnroll.
template <bool GUARD, bool HIST>
__device__ __forceinline__ void part_gathers(uint32_t kmix, const uint32_t* s1, uint32_t g, uint32_t m,
                                             const uint8_t* reg, const uint8_t* reg4, uint32_t part_shift,
                                             uint32_t x, int lane, uint64_t& U, uint32_t& V, uint32_t* lh) {
  for (uint32_t i0 = lane; i0 < g; i0 += 64 * kEstUnroll) {
    uint32_t p[kEstUnroll];
    bool take[kEstUnroll];
#pragma unroll
    for (int u = 0; u < kEstUnroll; ++u) {
      const uint32_t i = i0 + 64u * u;
      const bool in = !GUARD || i < g;
      const uint32_t hh = in ? mm3_seeded(kmix, s1[i]) : 0u;
      take[u] = in && (hh >> part_shift) == x;
      p[u] = reduce_m(hh, m);
    }
    uint32_t nb[kEstUnroll];
#pragma unroll
    for (int u = 0; u < kEstUnroll; ++u) nb[u] = take[u] ? (uint32_t)reg4[p[u] >> 1] : 0u;
#pragma unroll
    for (int u = 0; u < kEstUnroll; ++u) {
      if (take[u]) {
        const uint32_t nib = (nb[u] >> ((p[u] & 1u) << 2)) & 15u;
        const uint32_t r = nib < 15u ? nib : (uint32_t)reg[p[u]];
        U += 1ull << (32 - r);
        V += r == 0;
        if constexpr (HIST) atomicAdd(&lh[r], 1u);
      }
    }
  }
}

template <bool STAGE, bool HIST>
__global__ __launch_bounds__(kEstBlock) void k_estimate_part(const uint32_t* __restrict__ hosts, uint32_t nh,
                                                             const uint32_t* __restrict__ s1g, uint32_t g, uint32_t m,
                                                             const uint8_t* __restrict__ reg,
                                                             const uint8_t* __restrict__ reg4, uint32_t parts,
                                                             uint32_t part_shift,
                                                             unsigned long long* __restrict__ part_u,
                                                             uint32_t* __restrict__ part_v, uint32_t pstride,
                                                             uint32_t* __restrict__ hout) {
  extern __shared__ uint32_t s1_lds[];
  __shared__ uint32_t lh[kEstWaves][kBins];
  const uint32_t* s1 = s1g;
  if constexpr (STAGE) {
    for (uint32_t i = threadIdx.x; i < g; i += kEstBlock) s1_lds[i] = s1g[i];
    __syncthreads();
    s1 = s1_lds;
  }
  const uint32_t x = blockIdx.x % parts;
  const uint32_t tiles = gridDim.x / parts;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (uint32_t h = (blockIdx.x / parts) * kEstWaves + wave; h < nh; h += tiles * kEstWaves) {
    const uint32_t kmix = mm3_key(hosts[h]);
    if constexpr (HIST) {
      if (lane < kBins) lh[wave][lane] = 0;
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
    }
    uint64_t U = 0;
    uint32_t V = 0;
    if (g % (64u * kEstUnroll) == 0)
      part_gathers<false, HIST>(kmix, s1, g, m, reg, reg4, part_shift, x, lane, U, V, lh[wave]);
    else
      part_gathers<true, HIST>(kmix, s1, g, m, reg, reg4, part_shift, x, lane, U, V, lh[wave]);
    if constexpr (HIST) {
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      __builtin_amdgcn_wave_barrier();
      if (lane < kBins) hout[((uint64_t)x * kLearnChunk + h) * kBins + lane] = lh[wave][lane];
      __builtin_amdgcn_wave_barrier();
    } else {
      U = wave_sum_u64(U);
      V = (uint32_t)wave_sum_u64(V);
      if (lane == 0) {
        part_u[(uint64_t)x * pstride + h] = U;
        part_v[(uint64_t)x * pstride + h] = V;
      }
    }
  }
}

__global__ __launch_bounds__(256) void k_estimate_final(uint32_t nh, uint32_t g, uint32_t m, uint32_t parts,
                                                        const unsigned long long* __restrict__ hist,
                                                        const unsigned long long* __restrict__ part_u,
                                                        const uint32_t* __restrict__ part_v, uint32_t pstride,
                                                        const unsigned long long* __restrict__ ovf_u,
                                                        const uint32_t* __restrict__ ovf_v, float* __restrict__ out) {
  __shared__ double em_sh;
  if (threadIdx.x == 0) {
    uint64_t U = 0;
    for (int r = 0; r < kBins; ++r) U += (uint64_t)hist[r] << (32 - r);
    em_sh = hll_estimate(U, hist[0], (double)m);
  }
  __syncthreads();
  const uint32_t h = blockIdx.x * 256 + threadIdx.x;
  if (h >= nh) return;
  uint64_t U = 0, V = 0;
  for (uint32_t x = 0; x < parts; ++x) {
    U += part_u[(uint64_t)x * pstride + h];
    V += part_v[(uint64_t)x * pstride + h];
  }
  if (ovf_u) {
    U += ovf_u[h];
    V += ovf_v[h];
  }
  const double Es = hll_estimate(U, V, (double)g);
  const double n = noise_removed(Es, em_sh, (double)m, (double)g);
  out[h] = (float)(n > 0.0 ? n : 0.0);
}

// ------------------------------------------------ estimate, XCD-binned
// The partitioned estimate hashes every (host, i) on all 8 XCDs.  Binned
// instead: pass 1 hashes each (host, i) once and appends its pidx to the run
// of (host, range x), the slot taken from a per-wave LDS counter; pass 2 runs
// range x on the workgroups of XCD x and gathers from the L2-resident nibble
// registers.  Entries beyond a run's capacity are gathered directly in pass 1
// and kept as a per-host overflow sum, so every (host, i) is counted exactly
// once.  (Non-temporal stores and loads of the runs were measured 1.5x slower:
// the runs' partial lines then leave L2 before they are complete.)
// GUARD: g is not a multiple of 64 * kBinRows.  POW2: m = 2^(32 - mshift), so
// that H(x, m, A) is a shift of the hash instead of a high multiply.
constexpr int kBinRows = 4;  // hash rows per wave in flight in pass 1

template <bool GUARD, bool POW2>
__global__ __launch_bounds__(kEstBlock) void k_est_bin(const uint32_t* __restrict__ hosts, uint32_t nh,
                                                       const uint32_t* __restrict__ s1g, uint32_t g, uint32_t m,
                                                       uint32_t mshift, const uint8_t* __restrict__ reg, uint32_t cap,
                                                       uint32_t hc, uint32_t* __restrict__ slots,
                                                       uint32_t* __restrict__ cnt, unsigned long long* __restrict__ ovf_u,
                                                       uint32_t* __restrict__ ovf_v) {
  extern __shared__ uint32_t s1_lds[];
  __shared__ uint32_t run_len[kEstWaves][8];
  for (uint32_t i = threadIdx.x; i < g; i += kEstBlock) s1_lds[i] = s1g[i];
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  uint32_t* len = run_len[wave];
  for (uint32_t h = blockIdx.x * kEstWaves + wave; h < nh; h += gridDim.x * kEstWaves) {
    const uint32_t kmix = mm3_key(hosts[h]);
    const uint32_t hbase = h * 8u * cap;
    if (lane < 8) len[lane] = 0;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    uint64_t oU = 0;
    uint32_t oV = 0;
    for (uint32_t i0 = lane; i0 < g; i0 += 64 * kBinRows) {
      uint32_t p[kBinRows], x[kBinRows], slot[kBinRows];
#pragma unroll
      for (int u = 0; u < kBinRows; ++u) {
        const uint32_t i = i0 + 64u * u;
        const uint32_t hh = !GUARD || i < g ? mm3_seeded(kmix, s1_lds[i]) : 0u;
        x[u] = hh >> 29;
        p[u] = POW2 ? hh >> mshift : reduce_m(hh, m);
      }
#pragma unroll
      for (int u = 0; u < kBinRows; ++u) slot[u] = !GUARD || i0 + 64u * u < g ? atomicAdd(&len[x[u]], 1u) : ~0u;
#pragma unroll
      for (int u = 0; u < kBinRows; ++u) {
        if (slot[u] < cap) {
          // run (h, x) starts at (8 h + x) cap; byte offsets < 4 * 8 * hc * cap <= 2^29
          const uint32_t off = (hbase + __umul24(x[u], cap) + slot[u]) * 4u;
          *reinterpret_cast<uint32_t*>(reinterpret_cast<char*>(slots) + off) = p[u];
        } else if (slot[u] != ~0u) {
          const uint32_t r = reg[p[u]];
          oU += 1ull << (32 - r);
          oV += r == 0;
        }
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
    if (lane < 8) {
      const uint32_t n = len[lane];
      cnt[(uint64_t)lane * hc + h] = n < cap ? n : cap;
    }
    __builtin_amdgcn_wave_barrier();
    oU = wave_sum_u64(oU);
    oV = (uint32_t)wave_sum_u64(oV);
    if (lane == 0) {
      ovf_u[h] = oU;
      ovf_v[h] = oV;
    }
  }
}

// Pass 2: a wave takes four hosts, sixteen lanes each.
constexpr int kGatherRows = 4;

__global__ __launch_bounds__(kEstBlock) void k_est_gather(uint32_t nh, const uint8_t* __restrict__ reg,
                                                          const uint8_t* __restrict__ reg4, uint32_t cap, uint32_t hc,
                                                          const uint32_t* __restrict__ slots,
                                                          const uint32_t* __restrict__ cnt,
                                                          unsigned long long* __restrict__ part_u,
                                                          uint32_t* __restrict__ part_v) {
  const uint32_t x = blockIdx.x & 7u;  // workgroups are dispatched round-robin over the 8 XCDs
  const uint32_t tiles = gridDim.x >> 3;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const uint32_t q = (uint32_t)lane >> 4, ql = (uint32_t)lane & 15u;
  for (uint32_t h0 = ((blockIdx.x >> 3) * kEstWaves + wave) * 4; h0 < nh; h0 += tiles * kEstWaves * 4) {
    const uint32_t h = h0 + q;
    const uint32_t n = h < nh ? cnt[(uint64_t)x * hc + h] : 0u;
    const uint32_t* run = slots + ((uint64_t)h * 8 + x) * cap;
    uint64_t U = 0;
    uint32_t V = 0;
    for (uint32_t j0 = ql; j0 < n; j0 += 16 * kGatherRows) {
      uint32_t p[kGatherRows], nb[kGatherRows];
#pragma unroll
      for (int u = 0; u < kGatherRows; ++u)
        p[u] = j0 + 16u * u < n ? run[j0 + 16u * u] : 0u;
#pragma unroll
      for (int u = 0; u < kGatherRows; ++u) nb[u] = j0 + 16u * u < n ? (uint32_t)reg4[p[u] >> 1] : 0u;
#pragma unroll
      for (int u = 0; u < kGatherRows; ++u) {
        if (j0 + 16u * u < n) {
          const uint32_t nib = (nb[u] >> ((p[u] & 1u) << 2)) & 15u;
          const uint32_t r = nib < 15u ? nib : (uint32_t)reg[p[u]];
          U += 1ull << (32 - r);
          V += r == 0;
        }
      }
    }
    // sum over the sixteen lanes of each host
#pragma unroll
    for (int d = 1; d < 16; d <<= 1) {
      U += __shfl_xor(U, d, 16);
      V += __shfl_xor(V, d, 16);
    }
    if (ql == 0 && h < nh) {
      part_u[(uint64_t)x * kPartChunk + h] = U;
      part_v[(uint64_t)x * kPartChunk + h] = V;
    }
  }
}

// ------------------------------------------- LogLog and PCSA on the pool
// The pool serves other estimators than HyperLogLog (the text after Alg. 5,
// Sec. 5).  One wave per host gathers the host's g values -- registers for
// LogLog (Alg. 5's literal sum), PCSA runs for PCSA -- and sums them; E_s =
// c_g * g * 2^(S/g) with c = alpha_g (LogLog) or 1/0.77351 (PCSA), E_m the
// same over the pool, then the noise removal of the HyperLogLog path.
__global__ __launch_bounds__(kEstBlock) void k_estimate_sum(const uint32_t* __restrict__ hosts, uint64_t nh,
                                                            const uint32_t* __restrict__ s1, uint32_t g, uint32_t m,
                                                            const uint8_t* __restrict__ val, double cg, double Em,
                                                            float* __restrict__ out, double* __restrict__ raw) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (uint64_t h = (uint64_t)blockIdx.x * kEstWaves + wave; h < nh; h += (uint64_t)gridDim.x * kEstWaves) {
    const uint32_t kmix = mm3_key(hosts[h]);
    uint32_t S = 0;
    for (uint32_t i0 = lane; i0 < g; i0 += 64 * 4) {
      uint32_t v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const uint32_t i = i0 + 64u * u;
        v[u] = i < g ? (uint32_t)val[reduce_m(mm3_seeded(kmix, s1[i]), m)] : 0u;
      }
      S += v[0] + v[1] + v[2] + v[3];
    }
    S = (uint32_t)wave_sum_u64(S);
    if (lane == 0) {
#pragma clang fp contract(off)
      const double Es = cg * (double)g * exp2((double)S / (double)g);
      const double n = noise_removed(Es, Em, (double)m, (double)g);
      out[h] = (float)(n > 0.0 ? n : 0.0);
      if (raw) raw[h] = Es;
    }
  }
}

// ------------------------------------------------- per-slice max-LBP1 map
// Fast layout only.  The open slice's LBP1 record is split between the
// bsLBP1 bit-planes and, with deferred scans, the pending records of each
// tile; export folds both into one byte per BDR (the highest LBP1), one
// workgroup per tile of kDeferTile BDRs, 32 BDRs per thread.
__global__ __launch_bounds__(kDeferBlock) void k_now_export(const uint32_t* __restrict__ seen, uint64_t wstride,
                                                            uint64_t mstride, uint64_t m, uint32_t L,
                                                            const uint32_t* __restrict__ recs,
                                                            const unsigned long long* __restrict__ fill, uint32_t cap,
                                                            uint8_t* __restrict__ now) {
  extern __shared__ uint32_t pm[];
  const uint32_t tile = blockIdx.x;
  for (uint32_t i = threadIdx.x; i < L * kDeferWords; i += kDeferBlock) pm[i] = 0;
  __syncthreads();
  if (recs) {
    const unsigned long long f = fill[tile];
    const uint32_t n = f < cap ? (uint32_t)f : cap;
    records_to_planes(recs + (uint64_t)tile * cap, n, pm);
  }
  __syncthreads();
  const uint64_t base = (uint64_t)tile * kDeferTile + (uint64_t)threadIdx.x * 32;
  if (base >= m) return;
  uint32_t R[8] = {0, 0, 0, 0, 0, 0, 0, 0}, done = 0;
  for (int i = (int)L; i >= 1; --i) {
    const uint32_t bits = pm[(uint32_t)(i - 1) * kDeferWords + threadIdx.x] | seen[(uint64_t)(i - 1) * wstride + (base >> 5)];
    const uint32_t fold = bits & ~done;
    done |= bits;
#pragma unroll
    for (int w = 0; w < 8; ++w) R[w] |= swar_nibble_to_bytes((fold >> (4 * w)) & 0xFu) & ((uint32_t)i * 0x01010101u);
  }
  if (base + 32 <= m) {
    *reinterpret_cast<u32x4*>(now + base) = u32x4{R[0], R[1], R[2], R[3]};
    *reinterpret_cast<u32x4*>(now + base + 16) = u32x4{R[4], R[5], R[6], R[7]};
  } else {
    for (uint32_t j = 0; base + j < m; ++j) now[base + j] = (uint8_t)(R[j >> 2] >> (8 * (j & 3)));
  }
}

// The open slice's record becomes `now`: bit-plane word w of plane r-1 gets
// bit j set exactly when now[32 w + j] == r (values outside 1..L set nothing).
__global__ __launch_bounds__(256) void k_now_import(const uint8_t* __restrict__ now, uint64_t m, uint32_t L,
                                                    uint32_t* __restrict__ seen, uint64_t wstride) {
  const uint64_t w = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  if (w >= wstride) return;
  uint32_t v[32];
#pragma unroll
  for (int j = 0; j < 32; ++j) v[j] = 32 * w + j < m ? now[32 * w + j] : 0u;
  for (uint32_t r = 1; r <= L; ++r) {
    uint32_t word = 0;
#pragma unroll
    for (int j = 0; j < 32; ++j) word |= (uint32_t)(v[j] == r) << j;
    seen[(uint64_t)(r - 1) * wstride + w] = word;
  }
}

__global__ void k_now_max(const uint8_t* __restrict__ a, const uint8_t* __restrict__ b, uint8_t* __restrict__ out,
                          uint64_t n) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
    const uint8_t x = a[i], y = b[i];
    out[i] = x > y ? x : y;
  }
}

// ------------------------------------------------ super-point selection
// Hosts whose estimate reaches the threshold, compacted per wave: a ballot
// gives each selected lane its rank, one atomic per wave reserves the run.
__global__ void k_select_reset(uint32_t* __restrict__ count) {
  if (threadIdx.x == 0) *count = 0;
}

__global__ __launch_bounds__(256) void k_select(const float* __restrict__ est, const uint32_t* __restrict__ hosts,
                                                uint32_t n, float thr, uint32_t* __restrict__ out_hosts,
                                                float* __restrict__ out_est, uint32_t cap,
                                                uint32_t* __restrict__ count) {
  const int lane = threadIdx.x & 63;
  const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
  for (uint32_t i0 = blockIdx.x * 256 + (threadIdx.x & ~63u); i0 < n; i0 += gridDim.x * 256) {
    const uint32_t i = i0 + lane;
    const float e = i < n ? est[i] : 0.0f;
    const bool take = i < n && e >= thr;
    const uint64_t mask = __ballot(take);
    if (!mask) continue;
    uint32_t base = 0;
    if (lane == 0) base = atomicAdd(count, (uint32_t)__popcll(mask));
    base = __shfl(base, 0);
    const uint32_t at = base + (uint32_t)__popcll(mask & below);
    if (take && at < cap) {
      out_hosts[at] = hosts[i];
      out_est[at] = e;
    }
  }
}

// ------------------------------------------------ estimate, LDS-tiled
// The partitioned and binned estimates both stop at the L2's rate of random
// 1-byte gathers.  Tiled: the pool's nibble registers are cut into nt <= 256
// tiles of TR = 2^shift registers (at most 128 KiB of nibbles), one per
// workgroup, held in LDS.  Per block of B hosts:
//   pass 1 hashes every (host, i) once and appends a record of the
//          register's offset in its tile and the host's slot in its
//          sub-block of 2048 (tile_rec) to the run of (sub-block, tile),
//          sorted by tile in LDS as in the deferred scan;
//   pass 2 runs tile t on one workgroup: it loads the tile into LDS once and,
//          sub-block by sub-block, gathers the runs' registers from LDS into
//          per-host sums (U + V << 48, exact integers) and writes them out;
//   pass 3 adds a host's nt partial sums (and any run overflow) and applies
//          the FP64 epilogue of the other estimates.
// Every gather is an LDS read; memory sees only streaming records and sums.
constexpr uint32_t kTileSlotBits = 11;
constexpr uint32_t kTileSub = 1u << kTileSlotBits;  // hosts per sub-block
// A record: bit 31 the nibble of the register's byte (offset & 1), bits
// 17..28 the host's slot in its sub-block plus one (12 bits), bits 0..16 the
// byte (offset >> 1; tiles hold at most 2^18 registers), bits 29..30 zero,
// so that record >> 29 is the nibble's bit shift.  Padding is the record 0
// (slot field 0, offset 0): pass 2 gathers it like any record, into an
// accumulator that is never read, and its bounded loads return it past the
// end of a run.
constexpr uint32_t kTilePad = 0u;
__device__ __forceinline__ uint32_t tile_rec(uint32_t off, uint32_t slot) {
  return (off << 31) | ((slot + 1u) << 17) | (off >> 1);
}
__device__ __forceinline__ uint32_t tile_rec_acc(uint32_t rec) { return (rec >> 17) & 0xFFFu; }  // slot + 1; 0 for padding
__device__ __forceinline__ uint32_t tile_rec_slot(uint32_t rec) { return tile_rec_acc(rec) - 1u; }
__device__ __forceinline__ uint32_t tile_rec_off(uint32_t rec) { return ((rec & 0x1FFFFu) << 1) | (rec >> 31); }
constexpr uint32_t kBufferRsrcWord3 = 0x00020000u;  // raw buffer resource, gfx9 family
constexpr uint32_t kTileMaxShift = 18;    // 2^18 registers = 128 KiB of nibbles
constexpr int kTileBinLog = 10;
constexpr int kTileBinBlock = 1 << kTileBinLog;  // pass 1 workgroup
constexpr int kTilePer = 16;              // (host, i) pairs per thread and chunk of pass 1
constexpr uint32_t kTileChunk = kTileBinBlock * kTilePer;

__host__ __device__ __forceinline__ uint32_t tile_chunk_hosts(uint32_t lg) {
  const uint32_t h = kTileChunk >> lg;
  return h < 64u ? h : 64u;
}

// LDS bytes of pass 1 (layout at the kernel).
inline size_t tile_bin_lds(uint32_t nt, uint32_t capb, uint32_t g) {
  return ((size_t)(nt + 1) * (((capb + 4) & ~3u) | 4u) + (size_t)nt + 1 + 64 + g) * 4;
}

__device__ __forceinline__ unsigned long long sum_term(uint32_t r) {
  return (1ull << (32 - r)) | (r == 0 ? (1ull << 48) : 0ull);
}

// A (tile, host) sum U + V << 48 in 32 bits, from U in units of 2^18 (Us)
// and the zero count V: V << 27 | Us.  Exact while Us < 2^27 and V <= 30;
// otherwise the sum goes to the host's overflow sum and the entry is 0.
__device__ __forceinline__ uint32_t pack_part32(uint32_t Us, uint32_t V, unsigned long long* ovf_h) {
  if (V <= 30 && Us < (1u << 27)) return V << 27 | Us;
  atomicAdd(ovf_h, ((unsigned long long)Us << 18) + ((unsigned long long)V << 48));
  return 0u;
}

// The same sum in 16 bits: Us itself when V < 4 and the part of Us that
// the nonzero registers add (Us - V 2^14, a zero register adding 2^14) is
// below 2^14 - 1, so that Us >> 14 = V; otherwise the entry is 0 and the
// whole sum goes to the overflow sum.  Used when registers 0..2 are rare in
// the pool (tile_part_narrow), where it halves the partial-sum traffic.
__device__ __forceinline__ uint32_t pack_part16(uint32_t Us, uint32_t V, unsigned long long* ovf_h) {
  if (V < 4u && Us - (V << 14) < 0x3FFFu) return Us;
  atomicAdd(ovf_h, ((unsigned long long)Us << 18) + ((unsigned long long)V << 48));
  return 0u;
}
// 16-bit per-tile sums when fewer than m/64 registers of the pool are 0, 1
// or 2 (few escapes); pass 2 and pass 3 decide alike from the histogram.
__device__ __forceinline__ bool tile_part_narrow(const unsigned long long* hist, uint64_t m) {
  return 64ull * (hist[0] + hist[1] + hist[2]) < m;
}

// Zeroes a block's run lengths and overflow sums (as 32-bit words).
__global__ void k_est_tile_clear(uint32_t* __restrict__ a, uint64_t na, uint32_t* __restrict__ b, uint64_t nb) {
  for (uint64_t q = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; q < na + nb; q += (uint64_t)gridDim.x * blockDim.x) {
    if (q < na)
      a[q] = 0u;
    else
      b[q - na] = 0u;
  }
}

// Pass 1.  A chunk is hpc = min(kTileChunk / g, 64) consecutive hosts of one
// sub-block.  Each (host, i) is hashed once and appended to the LDS bucket of
// its tile (capb entries; an entry beyond it is gathered directly into the
// host's overflow sum).  Then each wave reserves the places of its own
// buckets in the runs of (sub-block, tile), one atomic per bucket, and copies
// them out (wave 0 first computes the next chunk's host keys).  All chunks of
// a sub-block run on one XCD (workgroup b on XCD b % 8), so that the partly
// written lines at the ends of a run's segments merge in that XCD's L2.
// Pairs past the chunk's end count into a spare tile nt, and entries beyond
// a bucket's capacity go to a spare last slot, so that the append is
// branch-free.  LDS: bucket[nt + 1][capb + 1], cnt[nt + 1], kmix[64], s1[g].
// POW2: m = 2^(32 - mshift), so H(x, m, A) is the hash shifted right (the
// multiply-shift map of a power of two) instead of a high multiply.
template <bool POW2>
__global__ __launch_bounds__(kTileBinBlock) __attribute__((amdgpu_waves_per_eu(4))) void k_est_tile_bin(
    const uint32_t* __restrict__ hosts, uint32_t nh, const uint32_t* __restrict__ s1g, uint32_t g, uint32_t lg,
    uint32_t m, uint32_t mshift, uint32_t shift, uint32_t nt, uint32_t capb, uint32_t cap,
    uint32_t* __restrict__ recs, uint32_t* __restrict__ fill, const uint8_t* __restrict__ reg,
    unsigned long long* __restrict__ ovf) {
  extern __shared__ uint32_t lds[];
  const uint32_t hpc = tile_chunk_hosts(lg);  // divides kTileSub
  // room for the spare slot; rows 16-byte aligned, 4 mod 8 words apart so that rows start on different banks
  const uint32_t bstride = ((capb + 4) & ~3u) | 4u;
  uint32_t* bucket = lds;
  uint32_t* cnt = bucket + (nt + 1) * bstride;
  uint32_t* kmix = cnt + nt + 1;
  uint32_t* s1l = kmix + 64;
  const uint32_t wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const uint32_t tmask = (1u << shift) - 1;
  const uint32_t xcd = blockIdx.x & 7, per_xcd = gridDim.x >> 3;  // the grid is a multiple of 8
  const uint32_t cps = kTileSub / hpc, nsb = (nh + kTileSub - 1) / kTileSub;
  // first host of the k-th chunk of this XCD (sub-blocks xcd, xcd + 8, ...), ~0u past the end
  auto chunk_start = [&](uint32_t k) -> uint32_t {
    const uint32_t sb = xcd + 8 * (k / cps);
    if (sb >= nsb) return ~0u;
    const uint32_t c0 = sb * kTileSub + (k % cps) * hpc;
    return c0 < nh ? c0 : ~0u;
  };
  auto host_of = [&](uint32_t c0) -> bool { return c0 != ~0u && lane < hpc && c0 + lane < nh; };
  uint32_t k = blockIdx.x >> 3;
  uint32_t c0 = chunk_start(k);
  for (uint32_t i = threadIdx.x; i < g; i += kTileBinBlock) s1l[i] = s1g[i];
  for (uint32_t t = threadIdx.x; t <= nt; t += kTileBinBlock) cnt[t] = 0;
  if (wave == 0) kmix[lane] = host_of(c0) ? mm3_key(hosts[c0 + lane]) : 0u;
  __syncthreads();
  while (c0 != ~0u) {
    const uint32_t c0n = chunk_start(k + per_xcd);
    uint32_t hnext = 0;
    if (wave == 0 && host_of(c0n)) hnext = hosts[c0n + lane];
    const uint32_t sb = c0 / kTileSub, slot0 = c0 & (kTileSub - 1);
    unsigned long long* ovf_sb = ovf + (uint64_t)sb * kTileSub;
    const uint32_t npairs = (nh - c0 < hpc ? nh - c0 : hpc) << lg;
    // pair u of a thread: index (u * kTileBinBlock + tx) of the chunk, host index >> lg, i = index mod g.
    // tx is opaque to the compiler so that the LDS addresses are formed here, not kept live across chunks.
    uint32_t tx = threadIdx.x;
    asm volatile("" : "+v"(tx));
    uint32_t pv[kTilePer], qv[kTilePer];
    auto pool_index = [&](uint32_t h) -> uint32_t { return POW2 ? h >> mshift : reduce_m(h, m); };
    const bool whole = npairs == kTileChunk;  // a full chunk: no pair is padding
    bool full = false;
    if (lg == kTileBinLog && whole) {
      // g = kTileBinBlock: pair u of every lane is (host u of the chunk,
      // virtual index tx), so the host keys are uniform and sit in registers
      const uint32_t sv = s1l[tx];
      uint32_t km[kTilePer];
#pragma unroll
      for (int u = 0; u < kTilePer; ++u) km[u] = kmix[u];
#pragma unroll
      for (int u = 0; u < kTilePer; ++u) pv[u] = pool_index(mm3_seeded(km[u], sv));
#pragma unroll
      for (int u = 0; u < kTilePer; ++u) qv[u] = atomicAdd(&cnt[pv[u] >> shift], 1u);
#pragma unroll
      for (int u = 0; u < kTilePer; ++u) {
        const uint32_t p = pv[u];
        bucket[__umul24(p >> shift, bstride) + (qv[u] < capb ? qv[u] : capb)] = tile_rec(p & tmask, slot0 + (uint32_t)u);
        full |= qv[u] >= capb;
      }
    } else {
      if (lg <= kTileBinLog) {  // one seed per thread; hosts (tx >> lg) + u * (kTileBinBlock >> lg)
        const uint32_t sv = s1l[tx & (g - 1)];
        const uint32_t* kp = kmix + (tx >> lg);
        const uint32_t kst = kTileBinBlock >> lg;
#pragma unroll
        for (int u = 0; u < kTilePer; ++u) {  // branch-free: kmix is zero past the chunk's hosts
          const uint32_t p = pool_index(mm3_seeded(kp[(u * kst) & 63u], sv));
          pv[u] = whole || (uint32_t)u * kTileBinBlock + tx < npairs ? p : ~0u;
        }
      } else {  // one host for g / kTileBinBlock consecutive u
        const uint32_t gw = g >> kTileBinLog, hs = lg - kTileBinLog;
#pragma unroll
        for (int u = 0; u < kTilePer; ++u) {
          const uint32_t p =
              pool_index(mm3_seeded(kmix[(uint32_t)u >> hs], s1l[(((uint32_t)u & (gw - 1)) << kTileBinLog) + tx]));
          pv[u] = whole || (uint32_t)u * kTileBinBlock + tx < npairs ? p : ~0u;
        }
      }
#pragma unroll
      for (int u = 0; u < kTilePer; ++u) qv[u] = atomicAdd(&cnt[pv[u] != ~0u ? pv[u] >> shift : nt], 1u);
#pragma unroll
      for (int u = 0; u < kTilePer; ++u) {
        const uint32_t p = pv[u], hl = ((uint32_t)u * kTileBinBlock + tx) >> lg;
        const uint32_t t = p != ~0u ? p >> shift : nt;
        bucket[__umul24(t, bstride) + (qv[u] < capb ? qv[u] : capb)] = tile_rec(p & tmask, slot0 + hl);
        full |= p != ~0u && qv[u] >= capb;
      }
    }
    if (full) {  // rare: entries beyond a bucket's capacity are gathered directly
#pragma unroll
      for (int u = 0; u < kTilePer; ++u)
        if (pv[u] != ~0u && qv[u] >= capb)
          atomicAdd(ovf_sb + slot0 + (((uint32_t)u * kTileBinBlock + tx) >> lg), sum_term(reg[pv[u]]));
    }
    __syncthreads();
    {  // every wave reserves the run places of its own bpw buckets (lane j:
       // bucket t0 + j, one atomic) and copies them out, 16 lanes per bucket
       // and four records (16 bytes) per lane, the tail quad padded; no
       // barrier between reservation and copy, so one wave's atomics wait
       // while others copy
      const uint32_t bpw = (nt + 15) >> 4, t0 = wave * bpw;  // nt <= 256
      uint32_t c_l = 0, b_l = 0;
      if (lane < bpw && t0 + lane < nt) {
        const uint32_t t = t0 + lane, c = cnt[t];
        c_l = c < capb ? c : capb;
        cnt[t] = 0;
        if (c_l) b_l = atomicAdd(&fill[sb * nt + t], (c_l + 3u) & ~3u);  // whole quads
      }
      if (wave == 0) kmix[lane] = host_of(c0n) ? mm3_key(hnext) : 0u;  // before this wave's stores
      const uint32_t ql = lane & 15;
      for (uint32_t j0 = 0; j0 < bpw; j0 += 4) {
        const uint32_t j = j0 + (lane >> 4), t = t0 + j;
        const uint32_t c = (uint32_t)__shfl((int)c_l, (int)j), b0 = (uint32_t)__shfl((int)b_l, (int)j);  // 0 past the wave's buckets
        uint32_t* run = recs + ((uint64_t)sb * nt + t) * cap;
        for (uint32_t i = 4 * ql; i < c; i += 64) {
          uint4 v = *reinterpret_cast<const uint4*>(bucket + t * bstride + i);
          if (i + 1 >= c) v.y = kTilePad;
          if (i + 2 >= c) v.z = kTilePad;
          if (i + 3 >= c) v.w = kTilePad;
          if (b0 + i < cap) {  // cap and b0 are multiples of 4: the quad fits whole
            *reinterpret_cast<uint4*>(run + b0 + i) = v;
          } else {  // run full: gather directly
            const uint32_t r4[4] = {v.x, v.y, v.z, v.w};
            for (int e = 0; e < 4; ++e)
              if (r4[e] != kTilePad)
                atomicAdd(ovf_sb + tile_rec_slot(r4[e]), sum_term(reg[((uint64_t)t << shift) + tile_rec_off(r4[e])]));
          }
        }
      }
    }
    __syncthreads();
    k += per_xcd;
    c0 = c0n;
  }
}

// Pass 2: one workgroup per tile.  LDS (dynamic, tile_gather_lds): the
// tile's TR/2 nibble bytes at address 0, then two buffers of per-host sums
// and zero counts: 152 KiB for tiles of 2^18.  A
// host's sum over one tile and sub-block is kept in 32 bits, exactly: the
// nibble path's registers r < 15 add 2^(32-r) = 2^18 * 2^(14-r), and at most
// g <= 8192 records add at most 2^13 * 2^14 < 2^32 in units of 2^18.  Zero
// registers are counted apart, two hosts' 16-bit counts to a word (at most g
// per host).  Registers of 15 and more add 2^14 >> 15 = 0 here and go to the
// host's 64-bit overflow sum instead, through the tile's list of wide
// records (wide, gathered by k_est_tile_wide after this pass), so that no
// global load here waits behind the prefetched runs; a record past the
// list's capacity is gathered at once.  Every record, padding included,
// takes the same branch-free steps (a byte read, a nibble extract, one LDS
// add); zero and wide registers take a branch that a wave skips unless one
// of its lanes holds one.  Runs are prefetched two sub-blocks ahead.
constexpr uint32_t kTileAccU = kTileSub + 1, kTileAccV = kTileSub / 2;
inline size_t tile_gather_lds(uint32_t shift) { return ((size_t)1 << shift) / 2 + 8 * (size_t)(kTileAccU + kTileAccV) + 16; }
constexpr uint64_t kTileWideTotal = 1ull << 24;  // wide-list entries over all tiles (8 bytes each)
template <int PRE>
__global__ __launch_bounds__(kDeferBlock) void k_est_tile_gather(const uint8_t* __restrict__ reg4,
                                                                 const uint8_t* __restrict__ reg, uint64_t mstride,
                                                                 uint32_t shift, uint32_t nt, uint32_t nsb,
                                                                 uint32_t cap, const uint32_t* __restrict__ recs,
                                                                 const uint32_t* __restrict__ fill,
                                                                 uint32_t* __restrict__ part, uint32_t B,
                                                                 unsigned long long* __restrict__ ovf,
                                                                 uint2* __restrict__ wide, uint32_t wcap,
                                                                 uint32_t* __restrict__ wcnt,
                                                                 const unsigned long long* __restrict__ hist,
                                                                 uint64_t m) {
  extern __shared__ uint32_t tile_w[];
  const bool narrow = tile_part_narrow(hist, m);  // 16-bit sums
  // per-host sums in units of 2^18 (host slot s at s + 1; 0 takes the
  // padding) and zero counts, double-buffered (one barrier per sub-block)
  uint32_t* accu2 = tile_w + (1u << shift) / 8;
  uint32_t* accv2 = accu2 + 2 * kTileAccU;
  uint32_t* wide_n = accv2 + 2 * kTileAccV;  // entries in this tile's wide list
  for (uint32_t q = threadIdx.x; q < 2 * (kTileAccU + kTileAccV) + 1; q += kDeferBlock) accu2[q] = 0;
  const uint32_t t = blockIdx.x;
  wide += (uint64_t)t * wcap;
  const uint64_t tbase = (uint64_t)t << shift;
  const uint64_t nbytes = ((tbase + (1ull << shift) < mstride ? tbase + (1ull << shift) : mstride) - tbase) / 2;
  const uint32_t* src = reinterpret_cast<const uint32_t*>(reg4 + tbase / 2);
  for (uint64_t q = threadIdx.x; q < nbytes / 4; q += kDeferBlock) tile_w[q] = src[q];
  const uint8_t* tl = reinterpret_cast<const uint8_t*>(tile_w);
  // run lengths of this tile's sub-blocks (at most 256) held in registers:
  // lane l of every wave keeps sub-blocks l, l + 64, l + 128, l + 192, read
  // with readlane, so no step waits for a length load before its gathers
  const uint32_t lane = threadIdx.x & 63;
  uint32_t fr[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const uint32_t sb = 64u * q + lane;
    const uint32_t f = sb < nsb ? fill[sb * nt + t] : 0u;
    fr[q] = f < cap ? f : cap;
  }
  auto run_len = [&](uint32_t sb) -> uint32_t {  // four reads of lanes and a scalar select: no temporary VGPR
    const int l = (int)(sb & 63);
    const uint32_t a = (uint32_t)__builtin_amdgcn_readlane((int)fr[0], l), b = (uint32_t)__builtin_amdgcn_readlane((int)fr[1], l),
                   c = (uint32_t)__builtin_amdgcn_readlane((int)fr[2], l), d = (uint32_t)__builtin_amdgcn_readlane((int)fr[3], l);
    const uint32_t q = sb >> 6;
    return q == 0 ? a : q == 1 ? b : q == 2 ? c : d;
  };
  // the first PRE * kDeferBlock records of every run (all of it, for runs of
  // the expected length) are loaded two sub-blocks ahead, as whole quads: quad
  // threadIdx.x + q * kDeferBlock of the run (runs hold whole quads).  One
  // 16-byte load per quad instead of four 4-byte loads: pass 2 -3 % at g =
  // 1024, -16 % at g = 2048.
  static_assert(PRE % 4 == 0, "the prefetch holds whole quads");
  constexpr int PQ = PRE / 4;
  // three buffers of prefetched quads, each in fixed registers: sub-block
  // sbk is gathered from one while the next two sub-blocks' runs load into
  // the others (a rotation by copies would wait for the loads just issued)
  u32x4 ra[PQ], rb[PQ], rc[PQ];
  // bounded buffer loads, without branches (so that a use waits only for
  // its own loads): quads past a run's length, and the runs of sub-blocks
  // past the last, read as padding (0)
  auto load_run = [&](uint32_t sb, u32x4(&dst)[PQ]) __attribute__((always_inline)) {
    const bool in = sb < nsb;
    const uint32_t len = in ? run_len(sb) : 0u;
    const uint32_t* r = recs + ((uint64_t)(in ? sb : 0u) * nt + t) * cap;
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<uint32_t*>(r), (short)0, (int)(len * 4), (int)kBufferRsrcWord3);
#pragma unroll
    for (int q = 0; q < PQ; ++q) {
      const auto v = __builtin_amdgcn_raw_buffer_load_b128(rs, (int)(16 * (threadIdx.x + q * kDeferBlock)), 0, 0);
      dst[q] = u32x4{v[0], v[1], v[2], v[3]};
    }
  };
  // gathers sub-block sbk from cur, then starts the load of sub-block sbk + 2 into nxt2
  auto sub_block = [&](uint32_t sbk, u32x4(&cur)[PQ], u32x4(&nxt2)[PQ]) __attribute__((always_inline)) {
    uint32_t* accu = accu2 + (sbk & 1) * kTileAccU;
    uint32_t* accv = accv2 + (sbk & 1) * kTileAccV;
    unsigned long long* ovf_sb = ovf + (uint64_t)sbk * kTileSub;
    const uint32_t n = run_len(sbk);
    // one record: the register's term 2^(14-r) added to its host (0 for
    // r >= 15), given the byte that holds its nibble; returns the nibble
    auto gather = [&](uint32_t rec, uint32_t byte) -> uint32_t {
      const uint32_t nib = __builtin_amdgcn_ubfe(byte, rec >> 29, 4);
      atomicAdd(&accu[tile_rec_acc(rec)], 0x4000u >> nib);
      return nib;
    };
    // zero count of a record's host (nib == 0), or its wide register (nib
    // == 15) put on the wide list; padding is skipped
    auto rare = [&](uint32_t rec, uint32_t nib) {
      if (rec == kTilePad) return;
      const uint32_t q = tile_rec_slot(rec);
      if (nib == 0) {
        atomicAdd(&accv[q >> 1], 1u << ((q & 1u) << 4));
      } else if (nib == 15) {
        const uint32_t at = atomicAdd(wide_n, 1u);
        if (at < wcap)
          wide[at] = make_uint2(sbk, rec);
        else
          atomicAdd(ovf_sb + q, sum_term(reg[tbase + tile_rec_off(rec)]));
      }
    };
    load_run(sbk + 2, nxt2);
    if (sbk == 0) __syncthreads();  // the tile and the zeroed accumulators
    const uint32_t* run = recs + ((uint64_t)sbk * nt + t) * cap;
    // a prefetched quad slot that holds only padding in every lane of the
    // wave (runs average 8 records per thread of PRE) is skipped as a whole
    const uint32_t wave0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)(threadIdx.x & ~63u));
#pragma unroll
    for (int q = 0; q < PQ; ++q) {
      if (4 * (wave0 + (uint32_t)q * kDeferBlock) >= n) break;
      const uint32_t r4[4] = {cur[q][0], cur[q][1], cur[q][2], cur[q][3]};
      uint32_t by[4], nib[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) by[e] = tl[r4[e] & 0x1FFFFu];  // the four reads issue before any add
#pragma unroll
      for (int e = 0; e < 4; ++e) nib[e] = gather(r4[e], by[e]);
      bool any = false;
#pragma unroll
      for (int e = 0; e < 4; ++e) any |= nib[e] == 0u || nib[e] == 15u;
      if (__builtin_amdgcn_ballot_w64(any)) {
#pragma unroll
        for (int e = 0; e < 4; ++e) rare(r4[e], nib[e]);
      }
    }
    for (uint32_t j = threadIdx.x + PRE * kDeferBlock; j < n; j += kDeferBlock) {  // runs longer than expected
      const uint32_t rec = run[j];
      rare(rec, gather(rec, tl[rec & 0x1FFFFu]));
    }
    __syncthreads();
    {  // thread w packs hosts 2w and 2w + 1 (one zero-count word) and clears
       // them for the sub-block two on, after the next barrier (the spare
       // slot is never read)
      static_assert(kDeferBlock == kTileSub / 2, "one zero-count word per thread");
      const uint32_t w = threadIdx.x, v = accv[w], h = sbk * kTileSub + 2 * w;
      if (narrow) {
        const uint32_t lo = pack_part16(accu[2 * w + 1], v & 0xFFFFu, ovf + h),
                       hi = pack_part16(accu[2 * w + 2], v >> 16, ovf + h + 1);
        *reinterpret_cast<uint32_t*>(reinterpret_cast<uint16_t*>(part) + (uint64_t)t * B + h) = lo | hi << 16;
      } else {
        uint2 pr;
        pr.x = pack_part32(accu[2 * w + 1], v & 0xFFFFu, ovf + h);
        pr.y = pack_part32(accu[2 * w + 2], v >> 16, ovf + h + 1);
        *reinterpret_cast<uint2*>(part + (uint64_t)t * B + h) = pr;
      }
      accu[2 * w + 1] = 0, accu[2 * w + 2] = 0, accv[w] = 0;
    }
  };
  load_run(0, ra);
  load_run(1, rb);
  for (uint32_t sbk = 0; sbk < nsb; sbk += 3) {
    sub_block(sbk, ra, rc);
    if (sbk + 1 < nsb) sub_block(sbk + 1, rb, ra);
    if (sbk + 2 < nsb) sub_block(sbk + 2, rc, rb);
  }
  __syncthreads();
  if (threadIdx.x == 0) wcnt[t] = *wide_n < wcap ? *wide_n : wcap;
}

// After pass 2: the registers of 15 and more that pass 2 listed, read from
// the byte array and added to their hosts' overflow sums.  Grid (x, nt).
__global__ __launch_bounds__(256) void k_est_tile_wide(const uint2* __restrict__ wide, uint32_t wcap,
                                                       const uint32_t* __restrict__ wcnt,
                                                       const uint8_t* __restrict__ reg, uint32_t shift,
                                                       unsigned long long* __restrict__ ovf) {
  const uint32_t t = blockIdx.y, n = wcnt[t];
  const uint2* w = wide + (uint64_t)t * wcap;
  for (uint32_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
    const uint2 e = w[i];
    atomicAdd(ovf + (uint64_t)e.x * kTileSub + tile_rec_slot(e.y),
              sum_term(reg[((uint64_t)t << shift) + tile_rec_off(e.y)]));
  }
}

// Pass 3: one thread per host of the block.
__global__ __launch_bounds__(256) void k_est_tile_final(uint32_t nh, uint32_t g, uint32_t m, uint32_t nt, uint32_t B,
                                                        const unsigned long long* __restrict__ hist,
                                                        const uint32_t* __restrict__ part,
                                                        const unsigned long long* __restrict__ ovf,
                                                        float* __restrict__ out) {
  __shared__ double em_sh;
  if (threadIdx.x == 0) em_sh = pool_estimate(hist, (double)m);
  __syncthreads();
  const uint32_t h = blockIdx.x * 256 + threadIdx.x;
  if (h >= nh) return;
  unsigned long long U = 0, V = 0;
  const unsigned long long o = ovf[h];
  U = o & ((1ull << 48) - 1);
  V = o >> 48;
  unsigned long long Us = 0;  // in units of 2^18
  uint32_t t = 0;
  if (tile_part_narrow(hist, m)) {  // 16-bit sums: the entry is Us, and V = Us >> 14 (pack_part16)
    const uint16_t* p16 = reinterpret_cast<const uint16_t*>(part);
    for (; t + 8 <= nt; t += 8) {
      uint32_t v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = p16[(uint64_t)(t + u) * B + h];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        Us += v[u];
        V += v[u] >> 14;
      }
    }
    for (; t < nt; ++t) {
      const uint32_t v = p16[(uint64_t)t * B + h];
      Us += v;
      V += v >> 14;
    }
  } else {
    for (; t + 8 <= nt; t += 8) {
      uint32_t v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = part[(uint64_t)(t + u) * B + h];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        Us += v[u] & ((1u << 27) - 1);
        V += v[u] >> 27;
      }
    }
    for (; t < nt; ++t) {
      const uint32_t v = part[(uint64_t)t * B + h];
      Us += v & ((1u << 27) - 1);
      V += v >> 27;
    }
  }
  U += Us << 18;
  const double Es = hll_estimate(U, V, (double)g);
  const double n = noise_removed(Es, em_sh, (double)m, (double)g);
  out[h] = (float)(n > 0.0 ? n : 0.0);
}

// Nibble copy of the registers (after a state import).
__global__ void k_pack_reg4(const uint8_t* __restrict__ reg, uint8_t* __restrict__ reg4, uint64_t nbytes4) {
  for (uint64_t q = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; q < nbytes4; q += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t a = reg[2 * q], b = reg[2 * q + 1];
    reg4[q] = (uint8_t)((a < 15u ? a : 15u) | ((b < 15u ? b : 15u) << 4));
  }
}

// ------------------------------------------------------------- helpers


uint32_t grid_cap(const vbdr_sketch* sk, uint64_t want, uint32_t per_cu) {
  const uint64_t cap = (uint64_t)sk->n_cu * per_cu;
  if (want < 1) want = 1;
  return (uint32_t)(want < cap ? want : cap);
}

// LogLog constant alpha_q of Durand and Flajolet (2003),
// (Gamma(-1/q) (1 - 2^(1/q)) / ln 2)^-q.  With x = 1/q, y = x ln 2,
// |Gamma(-x)| = Gamma(1-x)/x and 2^x - 1 = y (1 + z), z = sum_k>=1 y^k/(k+1)!:
// alpha_q = exp(-q (ln Gamma(1-x) + ln(1+z))), free of cancellation for the
// large q of a pool.  q >= 16.
double loglog_alpha(double q) {
  const double x = 1.0 / q, y = x * std::log(2.0);
  double z = 0.0, term = 1.0;
  for (int k = 1; k <= 10; ++k) {
    term *= y / (double)(k + 1);
    z += term;
  }
  return std::exp(-q * (std::lgamma(1.0 - x) + std::log1p(z)));
}

uint64_t splitmix64_first(uint64_t state) {
  uint64_t z = state + 0x9e3779b97f4a7c15ull;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

int init_state(vbdr_sketch* sk, hipStream_t st) {
  const uint32_t fill_grid = grid_cap(sk, (sk->L * sk->mstride / 4 + 255) / 256, 32);
  if (sk->dr) {
    hipLaunchKernelGGL(k_fill_u32, dim3(fill_grid), dim3(256), 0, st, reinterpret_cast<uint32_t*>(sk->dr),
                       (uint64_t)sk->L * sk->mstride / 4, 0xFFFFFFFFu);  // InitDR: 255 in every byte
    VBDR_LAUNCHED("k_fill_u32(dr)");
  } else {
    hipLaunchKernelGGL(k_fill_u32, dim3(fill_grid), dim3(256), 0, st, sk->bits,
                       (uint64_t)sk->Lc * sk->z * sk->wstride, 0xFFFFFFFFu);  // InitDR: 2^z - 1 in every DR
    VBDR_LAUNCHED("k_fill_u32(bits)");
  }
  hipLaunchKernelGGL(k_fill_u32, dim3(fill_grid), dim3(256), 0, st, reinterpret_cast<uint32_t*>(sk->reg),
                     sk->mstride / 4, 0u);
  VBDR_LAUNCHED("k_fill_u32(reg)");
  hipLaunchKernelGGL(k_fill_u32, dim3(fill_grid), dim3(256), 0, st, reinterpret_cast<uint32_t*>(sk->reg4),
                     sk->mstride / 8, 0u);
  VBDR_LAUNCHED("k_fill_u32(reg4)");
  if (sk->seen) {
    hipLaunchKernelGGL(k_fill_u32, dim3(fill_grid), dim3(256), 0, st, sk->seen, (uint64_t)sk->L * sk->wstride, 0u);
    VBDR_LAUNCHED("k_fill_u32(seen)");
  }
  hipLaunchKernelGGL(k_hist_reset, dim3(1), dim3(64), 0, st, sk->hist, (unsigned long long)sk->m,
                     (unsigned long long*)nullptr);
  VBDR_LAUNCHED("k_hist_reset");
  if (sk->def_fill) {
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(256), 0, st, reinterpret_cast<uint32_t*>(sk->def_fill),
                       (uint64_t)(sk->def_tiles + 1) * 2, 0u);
    VBDR_LAUNCHED("k_fill_u32(def_fill)");
  }
  if (sk->sat) {  // no plane known saturated: the first advance reads every DR
    hipLaunchKernelGGL(k_fill_u32, dim3(fill_grid), dim3(256), 0, st, sk->sat, sk->wstride, 0u);
    VBDR_LAUNCHED("k_fill_u32(sat)");
  }
  return VBDR_OK;
}

// Apply pending deferred records to the pool (stream-ordered).
int defer_flush(vbdr_sketch* sk, hipStream_t st) {
  if (!sk->def_rec) return VBDR_OK;
  auto kern = sk->layout == VBDR_LAYOUT_FAST ? k_defer_flush<true> : k_defer_flush<false>;
  hipLaunchKernelGGL(kern, dim3(sk->def_tiles), dim3(256), 0, st, sk->def_rec, sk->def_fill, sk->def_cap,
                     sk->def_tiles, sk->dr, sk->mstride, sk->seen, sk->wstride, sk->bits, sk->z);
  VBDR_LAUNCHED("k_defer_flush");
  return VBDR_OK;
}

}  // namespace

void vbdr_defer_member(const vbdr_sketch* sk, DeferItem* d) {
  std::memset(d, 0, sizeof(*d));
  d->s1 = sk->s1, d->dr = sk->dr, d->seen = sk->seen, d->reg = sk->reg, d->reg4 = sk->reg4, d->hist = sk->hist;
  d->recs = sk->def_rec, d->fill = sk->def_fill, d->sat = sk->sat;
  d->mstride = sk->mstride, d->wstride = sk->wstride, d->m = sk->m;
  d->b = sk->b, d->A1 = sk->A1, d->tiles = sk->def_tiles, d->cap = sk->def_cap, d->L = sk->L, d->thr = sk->k - 1;
  d->layout = (uint32_t)sk->layout;
}

uint32_t vbdr_defer_chunk_pairs() { return kDeferChunk; }

int vbdr_launch_batch_defer(const DeferItem* items_dev, const DeferHdr* hdr_dev, uint32_t S, uint32_t max_tiles,
                            uint32_t max_L, uint32_t adv_total, uint32_t grid, int phase, hipStream_t st) {
  if (S == 0) return VBDR_OK;
  if (S > kMaxDeferMembers) return vbdr_fail(VBDR_EINVAL, "more than %u members with record runs", kMaxDeferMembers);
  if (phase == 0) {
    hipLaunchKernelGGL(k_batch_scan_defer, dim3(grid), dim3(kDeferBlock), (size_t)(2 * max_tiles + kDeferChunk) * 4,
                       st, items_dev, hdr_dev, S);
    VBDR_LAUNCHED("k_batch_scan_defer");
  } else {
    hipLaunchKernelGGL(k_batch_advance_defer, dim3(adv_total), dim3(kDeferBlock), (size_t)max_L * kDeferWords * 4, st,
                       items_dev, S);
    VBDR_LAUNCHED("k_batch_advance_defer");
    hipLaunchKernelGGL(k_batch_defer_flag, dim3(1), dim3(256), 0, st, items_dev, S);
    VBDR_LAUNCHED("k_batch_defer_flag");
  }
  return VBDR_OK;
}

int vbdr_check_device(const vbdr_sketch* sk) {
  int cur = -1;
  VBDR_HIP(hipGetDevice(&cur));
  if (cur != sk->device)
    return vbdr_fail(VBDR_EINVAL, "sketch lives on device %d but device %d is current", sk->device, cur);
  return VBDR_OK;
}

int vbdr_hist_pass(vbdr_sketch* sk, const uint32_t* hosts_dev, uint32_t nh, hipStream_t st) {
  if (nh == 0) return VBDR_OK;
  if (nh > kLearnChunk) return vbdr_fail(VBDR_EINVAL, "histogram pass of %u hosts exceeds %u", nh, kLearnChunk);
  const bool stage = sk->g <= kStageMaxG;
  const size_t lds = stage ? (size_t)sk->g * 4 : 0;
  if (sk->parts > 1) {
    const uint32_t parts = (uint32_t)sk->parts, shift = parts == 8 ? 29u : 30u;
    const uint64_t want = (nh + kEstWaves - 1) / kEstWaves;
    const uint64_t cap = (uint64_t)sk->n_cu * sk->tune.est_blocks_per_cu / parts;
    const uint32_t tiles = (uint32_t)(want < cap ? want : (cap ? cap : 1));
    auto kern = stage ? k_estimate_part<true, true> : k_estimate_part<false, true>;
    hipLaunchKernelGGL(kern, dim3(tiles * parts), dim3(kEstBlock), lds, st, hosts_dev, nh, sk->s1, sk->g,
                       (uint32_t)sk->m, sk->reg, sk->reg4, parts, shift, sk->part_u, sk->part_v, kPartChunk,
                       sk->hist_ws);
    VBDR_LAUNCHED("k_estimate_part(hist)");
  } else {
    const uint32_t grid = grid_cap(sk, (nh + kEstWaves - 1) / kEstWaves, sk->tune.est_blocks_per_cu);
    auto kern = stage ? k_estimate<true, true> : k_estimate<false, true>;
    hipLaunchKernelGGL(kern, dim3(grid), dim3(kEstBlock), lds, st, hosts_dev, (uint64_t)nh, sk->s1, sk->g,
                       (uint32_t)sk->m, sk->reg, sk->hist, sk->est_ws, nullptr, sk->hist_ws);
    VBDR_LAUNCHED("k_estimate(hist)");
  }
  return VBDR_OK;
}

// ================================================================= C ABI

extern "C" {

const char* vbdr_last_error(void) { return g_err.c_str(); }

}  // extern "C"

namespace {

// Deferred scans need the LDS of k_scan_defer: two words per tile plus the
// sorted chunk (s1 goes to LDS only if it fits beside them).
size_t defer_scan_lds(uint32_t tiles) { return (size_t)(2 * tiles + kDeferChunk) * 4; }

// Hosts per block of the tiled estimate under the current tuning: the
// default block (tl_B), or est_bin_hosts rounded down to whole sub-blocks.
uint32_t tiled_block_hosts(const vbdr_sketch* sk) {
  uint32_t B = sk->tl_B;
  if (sk->tune.est_bin_hosts && sk->tune.est_bin_hosts < B)
    B = sk->tune.est_bin_hosts < kTileSub ? kTileSub : sk->tune.est_bin_hosts / kTileSub * kTileSub;
  return B;
}

// Workspaces of the LDS-tiled estimate (records, run lengths, partial and
// overflow sums of one block of hosts, wide-register lists), once the
// variant is selected, sized for the tuning's block: a smaller est_bin_hosts
// gives a smaller workspace (the buffers are reallocated when it changes).
int alloc_tiled(vbdr_sketch* sk) {
  if (!sk->tl_ok) return VBDR_OK;
  const uint32_t Bw = tiled_block_hosts(sk);
  if (sk->tl_rec && sk->tl_Balloc == Bw) return VBDR_OK;
  if (sk->tl_rec) {  // another block size: the old buffers go first (no kernel may still use them)
    if (int rc = vbdr_check_device(sk)) return rc;
    VBDR_HIP(hipDeviceSynchronize());
    const uint64_t nsb0 = sk->tl_Balloc / kTileSub;
    sk->bytes -= nsb0 * sk->tl_nt * sk->tl_cap * 4 + nsb0 * sk->tl_nt * 4 + (uint64_t)sk->tl_nt * sk->tl_Balloc * 4 +
                 (uint64_t)sk->tl_Balloc * 8 + (uint64_t)sk->tl_nt * sk->tl_wcap * 8 + (uint64_t)sk->tl_nt * 4;
    for (void* q : {(void*)sk->tl_rec, (void*)sk->tl_fill, (void*)sk->tl_part, (void*)sk->tl_ovf, (void*)sk->tl_wide})
      (void)hipFree(q);
    sk->tl_rec = nullptr, sk->tl_fill = nullptr, sk->tl_part = nullptr, sk->tl_ovf = nullptr, sk->tl_wide = nullptr;
    sk->tl_Balloc = 0;
  }
  const uint64_t nsb = Bw / kTileSub;
  const uint64_t rec_b = nsb * sk->tl_nt * sk->tl_cap * 4, fill_b = nsb * sk->tl_nt * 4;
  const uint64_t part_b = (uint64_t)sk->tl_nt * Bw * 4, ovf_b = (uint64_t)Bw * 8;
  // wide lists: [nt][tl_wcap] entries, then nt counts
  sk->tl_wcap = (uint32_t)(kTileWideTotal / sk->tl_nt);
  const uint64_t wide_b = (uint64_t)sk->tl_nt * sk->tl_wcap * 8 + (uint64_t)sk->tl_nt * 4;
  if (vbdr_malloc(&sk->tl_rec, rec_b) != hipSuccess || vbdr_malloc(&sk->tl_fill, fill_b) != hipSuccess ||
      vbdr_malloc(&sk->tl_part, part_b) != hipSuccess || vbdr_malloc(&sk->tl_ovf, ovf_b) != hipSuccess ||
      vbdr_malloc(&sk->tl_wide, wide_b) != hipSuccess) {
    (void)hipGetLastError();
    for (void* q : {(void*)sk->tl_rec, (void*)sk->tl_fill, (void*)sk->tl_part, (void*)sk->tl_ovf, (void*)sk->tl_wide})
      if (q) (void)hipFree(q);
    sk->tl_rec = nullptr, sk->tl_fill = nullptr, sk->tl_part = nullptr, sk->tl_ovf = nullptr, sk->tl_wide = nullptr;
    return vbdr_fail(VBDR_ENOMEM, "allocation of the tiled-estimate workspace failed");
  }
  sk->bytes += rec_b + fill_b + part_b + ovf_b + wide_b;
  sk->tl_Balloc = Bw;
  return VBDR_OK;
}

// lean: no estimate workspaces (sketches of a batch); defer_ok: the record
// runs of deferred scans all the same (lean batch members with large pools).
int create_sketch(uint64_t m, uint32_t g, uint32_t k, uint64_t hash_seed, int layout, bool lean, bool defer_ok,
                  uint32_t Lc, vbdr_sketch** out) {
  if (!out) return vbdr_fail(VBDR_EINVAL, "out is NULL");
  *out = nullptr;
  if (g < 2 || g > 65536u || (g & (g - 1))) return vbdr_fail(VBDR_EINVAL, "g=%u must be a power of two in [2, 65536]", g);
  if (m <= g || m >= (1ull << 32)) return vbdr_fail(VBDR_EINVAL, "m=%llu must satisfy g < m < 2^32", (unsigned long long)m);
  if (k < 1 || k > 254) return vbdr_fail(VBDR_EINVAL, "k=%u must be in [1, 254]", k);
  if (layout != VBDR_LAYOUT_FAST && layout != VBDR_LAYOUT_SMALL && layout != VBDR_LAYOUT_PACKED)
    return vbdr_fail(VBDR_EINVAL, "unknown layout %d", layout);
  uint32_t b0 = 0;
  while ((1u << b0) < g) b0++;
  if (layout == VBDR_LAYOUT_PACKED) {
    if (lean) return vbdr_fail(VBDR_EINVAL, "the packed layout needs deferred scans");
    if (Lc < 1 || Lc > 33 - b0) return vbdr_fail(VBDR_EINVAL, "Lc=%u must be in [1, %u]", Lc, 33 - b0);
    if (m > kPackedMaxM) return vbdr_fail(VBDR_EINVAL, "the packed layout holds at most 2^26 BDRs");
  }
  vbdr_sketch* sk = new (std::nothrow) vbdr_sketch();
  if (!sk) return vbdr_fail(VBDR_ENOMEM, "host allocation failed");
  std::memset(sk, 0, sizeof(*sk));
  int rc = VBDR_OK;
  do {
    if (hipGetDevice(&sk->device) != hipSuccess) { rc = vbdr_fail(VBDR_EHIP, "hipGetDevice failed"); break; }
    if (hipDeviceGetAttribute(&sk->n_cu, hipDeviceAttributeMultiprocessorCount, sk->device) != hipSuccess) {
      rc = vbdr_fail(VBDR_EHIP, "hipDeviceGetAttribute failed");
      break;
    }
    int lds_max = 0;
    if (hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, sk->device) != hipSuccess) {
      rc = vbdr_fail(VBDR_EHIP, "hipDeviceGetAttribute failed");
      break;
    }
    sk->m = m, sk->g = g, sk->k = k, sk->layout = layout, sk->lean = lean;
    sk->tune = default_tuning(layout, m);
    while ((1u << sk->b) < g) sk->b++;
    sk->L = 33 - sk->b;
    const uint64_t x = splitmix64_first(hash_seed);
    sk->A0 = (uint32_t)x, sk->A1 = (uint32_t)(x >> 32);
    sk->mstride = (m + kPad - 1) / kPad * kPad;
    sk->wstride = sk->mstride / 32;
    sk->Lc = sk->L, sk->z = 8;
    if (layout == VBDR_LAYOUT_PACKED) {
      sk->Lc = Lc;
      sk->z = 1;
      while (((1u << sk->z) - 1) < k) sk->z++;  // 2^z - 1 >= k: a DR that left the window stays inactive
    }
    const uint64_t dr_bytes = layout == VBDR_LAYOUT_PACKED ? 0 : (uint64_t)sk->L * sk->mstride;
    const uint64_t bits_bytes = layout == VBDR_LAYOUT_PACKED ? (uint64_t)sk->Lc * sk->z * sk->wstride * 4 : 0;
    const uint64_t seen_bytes = layout == VBDR_LAYOUT_FAST ? (uint64_t)sk->L * sk->wstride * 4 : 0;
    // The partitioned estimate pays off once the registers outgrow one XCD's L2.
    const int xcds = sk->n_cu / (int)kCusPerXcd;
    sk->parts = (m >= kPartMinM && xcds >= 8) ? 8 : (m >= kPartMinM && xcds >= 4) ? 4 : 1;
    const uint64_t part_bytes = sk->parts > 1 ? (uint64_t)sk->parts * kPartChunk * (8 + 4) : 0;
    // the binned scan needs 8 XCDs and pidx < 2^27 to pack its records
    const uint64_t bin_bytes =
        (!lean && layout != VBDR_LAYOUT_PACKED && sk->parts == 8 && m <= kBinMaxM) ? 8ull * kBinCap * 4 : 0;
    // deferred scan records: kDeferSlots per BDR, for 2^22 <= m and 2^26 tile-rounded BDRs at most
    uint64_t def_bytes = 0;
    if ((!lean || defer_ok) && (m >= kPartMinM || layout == VBDR_LAYOUT_PACKED) && sk->mstride <= (1ull << 26)) {
      const uint32_t tiles = (uint32_t)((sk->mstride + kDeferTile - 1) / kDeferTile);
      if (defer_scan_lds(tiles) + 1024 <= (size_t)lds_max && (size_t)(33 - 1) * kDeferWords * 4 + 4096 <= (size_t)lds_max) {
        sk->def_tiles = tiles;
        sk->def_cap = kDeferSlots * kDeferTile;
        def_bytes = (uint64_t)tiles * sk->def_cap * 4 + (uint64_t)(tiles + 1) * 8;
      }
    }
    if (layout == VBDR_LAYOUT_PACKED && !def_bytes) {
      rc = vbdr_fail(VBDR_EINVAL, "the packed layout needs %zu bytes of LDS per workgroup", defer_scan_lds(1));
      break;
    }
    // binned estimate: runs of g/8 + g/16 + 32 slots per (range, host), <= 512 MiB of runs
    uint64_t est_bytes = 0;
    if (!lean && sk->parts == 8 && g >= 64 && g <= kStageMaxG) {
      sk->est_cap = g / 8 + g / 16 + 32;
      uint64_t hc = (512ull << 20) / (8ull * sk->est_cap * 4);
      hc = hc < kPartChunk ? hc : kPartChunk;
      sk->est_hc = (uint32_t)(hc / 64 * 64);
      est_bytes = 8ull * sk->est_hc * sk->est_cap * 4 + 8ull * sk->est_hc * 4 + (uint64_t)sk->est_hc * 12;
    }
    if ((dr_bytes && vbdr_malloc(&sk->dr, dr_bytes) != hipSuccess) ||
        (bits_bytes && vbdr_malloc(&sk->bits, bits_bytes) != hipSuccess) || vbdr_malloc(&sk->reg, sk->mstride) != hipSuccess ||
        vbdr_malloc(&sk->reg4, sk->mstride / 2) != hipSuccess ||
        vbdr_malloc(&sk->hist, 64 * sizeof(unsigned long long)) != hipSuccess ||
        vbdr_malloc(&sk->s1, (uint64_t)g * 4) != hipSuccess ||
        (seen_bytes && vbdr_malloc(&sk->seen, seen_bytes) != hipSuccess) ||
        (part_bytes && vbdr_malloc(&sk->part_u, (uint64_t)sk->parts * kPartChunk * 8) != hipSuccess) ||
        (part_bytes && vbdr_malloc(&sk->part_v, (uint64_t)sk->parts * kPartChunk * 4) != hipSuccess) ||
        vbdr_malloc(&sk->hist_ws, (uint64_t)sk->parts * kLearnChunk * kBins * 4) != hipSuccess ||
        vbdr_malloc(&sk->est_ws, (uint64_t)kLearnChunk * 4) != hipSuccess ||

        (def_bytes && vbdr_malloc(&sk->def_rec, (uint64_t)sk->def_tiles * sk->def_cap * 4) != hipSuccess) ||
        (def_bytes && vbdr_malloc(&sk->def_fill, (uint64_t)(sk->def_tiles + 1) * 8) != hipSuccess) ||
        (def_bytes && vbdr_malloc(&sk->sat, sk->wstride * 4) != hipSuccess)) {
      (void)hipGetLastError();
      rc = vbdr_fail(VBDR_ENOMEM, "device allocation of %llu bytes failed",
                (unsigned long long)(dr_bytes + seen_bytes + sk->mstride * 3 / 2 + part_bytes));
      break;
    }
    sk->state_only = dr_bytes + bits_bytes + seen_bytes + sk->mstride * 3 / 2 + 64 * sizeof(unsigned long long) +
                     (uint64_t)g * 4 + (sk->sat ? sk->wstride * 4 : 0);
    sk->bytes = sk->state_only + part_bytes + (uint64_t)sk->parts * kLearnChunk * kBins * 4 + (uint64_t)kLearnChunk * 4 +
                def_bytes;
    sk->bin_ok = bin_bytes != 0;  // allocated when the variant is selected (vbdr_sketch_set_tuning)
    sk->est_ok = est_bytes != 0;
    if (!lean && m >= kPartMinM && sk->mstride <= (1ull << 26) && g >= 64 && g <= kStageMaxG) {
      uint32_t sh = 12;
      while ((1ull << sh) * 256 < sk->mstride) sh++;
      const uint32_t nt = (uint32_t)((sk->mstride + (1ull << sh) - 1) >> sh);
      // hosts per block: 2^29 (host, i) pairs, at most 2^19 hosts (about 2.3 GB of records at most);
      // fewer, larger blocks measured faster (line rate: 2^17 hosts 1.58 ms, 2^18 1.49 ms, 2^19 1.45 ms)
      uint64_t B = (1ull << 29) / g;
      B = B < (1ull << 19) ? B : (1ull << 19);
      B = B / kTileSub * kTileSub;
      uint32_t lg = 0;
      while ((1u << lg) < g) lg++;
      // bucket of a (chunk, tile): Eb entries expected, room for Eb + 4 sqrt(Eb) + 4
      const double Eb = (double)(tile_chunk_hosts(lg) << lg) * (double)(1ull << sh) / (double)m;
      const uint32_t capb = ((uint32_t)(Eb + 4.0 * std::sqrt(Eb) + 4.0) + 3u) & ~3u;
      const size_t lds1 = tile_bin_lds(nt, capb, g);
      const size_t lds2 = tile_gather_lds(sh);  // the tile and two accumulator buffers
      if (sh <= kTileMaxShift && B >= kTileSub && lds1 + 1024 <= (size_t)lds_max && lds2 <= (size_t)lds_max) {
        const double E = (double)kTileSub * g * (double)(1ull << sh) / (double)m;
        sk->tl_ok = true;
        sk->tl_shift = sh, sk->tl_nt = nt, sk->tl_B = (uint32_t)B, sk->tl_capb = capb;
        sk->tl_cap = ((uint32_t)(E + 6.0 * std::sqrt(E) + 64.0) + 3u) & ~3u;  // runs hold whole quads
      }
    }
    if (sk->tune.est_binned == 3 && (rc = alloc_tiled(sk)) != VBDR_OK) break;
    hipStream_t st = nullptr;
    if ((rc = init_state(sk, st)) != VBDR_OK) break;
    hipLaunchKernelGGL(k_seeds, dim3((g + 255) / 256), dim3(256), 0, st, sk->s1, g, sk->A0);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(st) != hipSuccess) {
      rc = vbdr_fail(VBDR_EHIP, "sketch initialisation failed");
      break;
    }
  } while (0);
  if (rc != VBDR_OK) {
    vbdr_sketch_destroy(sk);
    return rc;
  }
  *out = sk;
  return VBDR_OK;
}

}  // namespace

namespace {

// The XCD-partitioned estimate: hosts in chunks of pstride, per-range partial
// sums in part_u / part_v ([parts][pstride] each), then the FP64 epilogue.
int estimate_partitioned(vbdr_sketch* sk, const uint32_t* hosts_dev, uint64_t n_hosts, float* out_dev,
                         unsigned long long* part_u, uint32_t* part_v, uint32_t pstride, hipStream_t st) {
  const bool stage = sk->g <= kStageMaxG;
  const size_t lds = stage ? (size_t)sk->g * 4 : 0;
  const uint32_t parts = (uint32_t)(sk->parts == 8 ? sk->tune.est_parts : sk->parts);
  const uint32_t shift = parts == 8 ? 29u : 30u;
  auto kern = stage ? k_estimate_part<true, false> : k_estimate_part<false, false>;
  for (uint64_t c = 0; c < n_hosts; c += pstride) {
    const uint32_t nh = (uint32_t)(n_hosts - c < pstride ? n_hosts - c : pstride);
    const uint64_t want = (nh + kEstWaves - 1) / kEstWaves;
    const uint64_t cap = (uint64_t)sk->n_cu * sk->tune.est_blocks_per_cu / parts;
    const uint32_t tiles = (uint32_t)(want < cap ? want : (cap ? cap : 1));
    hipLaunchKernelGGL(kern, dim3(tiles * parts), dim3(kEstBlock), lds, st, hosts_dev + c, nh, sk->s1, sk->g,
                       (uint32_t)sk->m, sk->reg, sk->reg4, parts, shift, part_u, part_v, pstride, nullptr);
    VBDR_LAUNCHED("k_estimate_part");
    hipLaunchKernelGGL(k_estimate_final, dim3((nh + 255) / 256), dim3(256), 0, st, nh, sk->g, (uint32_t)sk->m, parts,
                       sk->hist, part_u, part_v, pstride, (const unsigned long long*)nullptr, (const uint32_t*)nullptr,
                       out_dev + c);
    VBDR_LAUNCHED("k_estimate_final");
  }
  return VBDR_OK;
}

// The direct estimate: one wave per host gathers from the whole register
// array; optional raw E_s and per-host histograms.
int estimate_direct(vbdr_sketch* sk, const uint32_t* hosts_dev, uint64_t n_hosts, float* out_dev, double* raw_es_dev,
                    uint32_t* hist_dev, hipStream_t st) {
  const bool stage = sk->g <= kStageMaxG;
  const bool extra = raw_es_dev || hist_dev;
  const size_t lds = stage ? (size_t)sk->g * 4 : 0;
  const uint32_t grid = grid_cap(sk, (n_hosts + kEstWaves - 1) / kEstWaves, sk->tune.est_blocks_per_cu);
  auto kern = stage ? (extra ? k_estimate<true, true> : k_estimate<true, false>)
                    : (extra ? k_estimate<false, true> : k_estimate<false, false>);
  hipLaunchKernelGGL(kern, dim3(grid), dim3(kEstBlock), lds, st, hosts_dev, n_hosts, sk->s1, sk->g, (uint32_t)sk->m,
                     sk->reg, sk->hist, out_dev, raw_es_dev, hist_dev);
  VBDR_LAUNCHED("k_estimate");
  return VBDR_OK;
}

}  // namespace

int vbdr_sketch_create_lean(uint64_t m, uint32_t g, uint32_t k, uint64_t hash_seed, int layout, bool defer,
                            vbdr_sketch** out) {
  if (layout == VBDR_LAYOUT_PACKED) return vbdr_fail(VBDR_EINVAL, "batches hold fast and small layouts only");
  return create_sketch(m, g, k, hash_seed, layout, true, defer, 0, out);
}

extern "C" {

int vbdr_sketch_create_layout(uint64_t m, uint32_t g, uint32_t k, uint64_t hash_seed, int layout, vbdr_sketch** out) {
  if (layout == VBDR_LAYOUT_PACKED) return vbdr_fail(VBDR_EINVAL, "create a packed sketch with vbdr_sketch_create_packed");
  return create_sketch(m, g, k, hash_seed, layout, false, false, 0, out);
}

int vbdr_sketch_create_packed(uint64_t m, uint32_t g, uint32_t k, uint64_t hash_seed, uint32_t Lc, vbdr_sketch** out) {
  return create_sketch(m, g, k, hash_seed, VBDR_LAYOUT_PACKED, false, false, Lc, out);
}

int vbdr_sketch_create(uint64_t m, uint32_t g, uint32_t k, uint64_t hash_seed, vbdr_sketch** out) {
  return vbdr_sketch_create_layout(m, g, k, hash_seed, VBDR_LAYOUT_FAST, out);
}

void vbdr_sketch_destroy(vbdr_sketch* sk) {
  if (!sk) return;
  int prev = -1;
  (void)hipGetDevice(&prev);
  if (prev != sk->device) (void)hipSetDevice(sk->device);
  (void)hipDeviceSynchronize();
  if (sk->dr) (void)hipFree(sk->dr);
  if (sk->bits) (void)hipFree(sk->bits);
  if (sk->seen) (void)hipFree(sk->seen);
  if (sk->reg) (void)hipFree(sk->reg);
  if (sk->hist) (void)hipFree(sk->hist);
  if (sk->s1) (void)hipFree(sk->s1);
  if (sk->reg4) (void)hipFree(sk->reg4);
  if (sk->part_u) (void)hipFree(sk->part_u);
  if (sk->part_v) (void)hipFree(sk->part_v);
  if (sk->hist_ws) (void)hipFree(sk->hist_ws);
  if (sk->est_ws) (void)hipFree(sk->est_ws);
  if (sk->bins) (void)hipFree(sk->bins);
  if (sk->bin_fill) (void)hipFree(sk->bin_fill);
  if (sk->est_slots) (void)hipFree(sk->est_slots);
  if (sk->est_cnt) (void)hipFree(sk->est_cnt);
  if (sk->ovf_u) (void)hipFree(sk->ovf_u);
  if (sk->ovf_v) (void)hipFree(sk->ovf_v);
  if (sk->def_rec) (void)hipFree(sk->def_rec);
  if (sk->def_fill) (void)hipFree(sk->def_fill);
  if (sk->sat) (void)hipFree(sk->sat);
  if (sk->preg) (void)hipFree(sk->preg);
  if (sk->tl_rec) (void)hipFree(sk->tl_rec);
  if (sk->tl_fill) (void)hipFree(sk->tl_fill);
  if (sk->tl_part) (void)hipFree(sk->tl_part);
  if (sk->tl_ovf) (void)hipFree(sk->tl_ovf);
  if (sk->tl_wide) (void)hipFree(sk->tl_wide);
  if (sk->psum) (void)hipFree(sk->psum);
  if (prev >= 0 && prev != sk->device) (void)hipSetDevice(prev);
  delete sk;
}

int vbdr_sketch_set_tuning(vbdr_sketch* sk, const vbdr_tuning* tuning) {
  if (!sk || !tuning) return vbdr_fail(VBDR_EINVAL, "NULL argument");
  if (tuning->scan_test_first < 0 || tuning->scan_test_first > 2) return vbdr_fail(VBDR_EINVAL, "scan_test_first must be 0, 1 or 2");
  if (tuning->scan_binned < 0 || tuning->scan_binned > 2) return vbdr_fail(VBDR_EINVAL, "scan_binned must be 0, 1 or 2");
  if (tuning->est_binned < 0 || tuning->est_binned > 3) return vbdr_fail(VBDR_EINVAL, "est_binned must be 0..3");
  if (tuning->est_parts != 0 && tuning->est_parts != 4 && tuning->est_parts != 8)
    return vbdr_fail(VBDR_EINVAL, "est_parts must be 0, 4 or 8");
  if (tuning->scan_blocks_per_cu > 64 || tuning->est_blocks_per_cu > 64)
    return vbdr_fail(VBDR_EINVAL, "blocks per CU must be at most 64");
  if (tuning->scan_defer < 0 || tuning->scan_defer > 2) return vbdr_fail(VBDR_EINVAL, "scan_defer must be 0, 1 or 2");
  if (sk->layout == VBDR_LAYOUT_PACKED && tuning->scan_defer == 2)
    return vbdr_fail(VBDR_EINVAL, "the packed layout always defers its scans");
  const int old_defer = sk->tune.scan_defer;
  sk->tune = default_tuning(sk->layout, sk->m);
  if (tuning->scan_test_first) sk->tune.scan_test_first = tuning->scan_test_first;
  if (tuning->scan_blocks_per_cu) sk->tune.scan_blocks_per_cu = tuning->scan_blocks_per_cu;
  if (tuning->est_blocks_per_cu) sk->tune.est_blocks_per_cu = tuning->est_blocks_per_cu;
  if (tuning->scan_binned) sk->tune.scan_binned = tuning->scan_binned;
  if (tuning->est_binned) sk->tune.est_binned = tuning->est_binned;
  if (tuning->est_parts) sk->tune.est_parts = tuning->est_parts;
  if (tuning->est_bin_hosts) sk->tune.est_bin_hosts = tuning->est_bin_hosts;
  if (tuning->est_bin_cap) sk->tune.est_bin_cap = tuning->est_bin_cap;
  if (tuning->scan_defer) sk->tune.scan_defer = tuning->scan_defer;
  // workspaces of the binned variants, on first selection
  if (sk->tune.scan_binned == 1 && sk->bin_ok && !sk->bins) {
    if (vbdr_malloc(&sk->bins, 8ull * kBinCap * 4) != hipSuccess || vbdr_malloc(&sk->bin_fill, 64) != hipSuccess) {
      (void)hipGetLastError();
      if (sk->bins) (void)hipFree(sk->bins);
      sk->bins = nullptr;
      return vbdr_fail(VBDR_ENOMEM, "allocation of the binned-scan workspace failed");
    }
    sk->bytes += 8ull * kBinCap * 4 + 64;
  }
  if (sk->tune.est_binned == 1 && sk->est_ok && !sk->est_slots) {
    const uint64_t slots = 8ull * sk->est_hc * sk->est_cap * 4, cnt = 8ull * sk->est_hc * 4;
    if (vbdr_malloc(&sk->est_slots, slots) != hipSuccess || vbdr_malloc(&sk->est_cnt, cnt) != hipSuccess ||
        vbdr_malloc(&sk->ovf_u, (uint64_t)sk->est_hc * 8) != hipSuccess ||
        vbdr_malloc(&sk->ovf_v, (uint64_t)sk->est_hc * 4) != hipSuccess) {
      (void)hipGetLastError();
      for (void* q : {(void*)sk->est_slots, (void*)sk->est_cnt, (void*)sk->ovf_u, (void*)sk->ovf_v})
        if (q) (void)hipFree(q);
      sk->est_slots = nullptr, sk->est_cnt = nullptr, sk->ovf_u = nullptr, sk->ovf_v = nullptr;
      return vbdr_fail(VBDR_ENOMEM, "allocation of the binned-estimate workspace failed");
    }
    sk->bytes += slots + cnt + (uint64_t)sk->est_hc * 12;
  }
  if (sk->tune.est_binned == 3)
    if (int rc = alloc_tiled(sk)) return rc;
  if (sk->def_rec && sk->tune.scan_defer != old_defer) {
    // pending records go to the pool; the bsLBP1 planes may now hold bits
    if (int rc = vbdr_check_device(sk)) return rc;
    VBDR_HIP(hipDeviceSynchronize());
    if (int rc = defer_flush(sk, nullptr)) return rc;
    hipLaunchKernelGGL(k_defer_flag, dim3(1), dim3(64), 0, nullptr, sk->def_fill, sk->def_tiles, 1ull);
    VBDR_LAUNCHED("k_defer_flag");
    VBDR_HIP(hipDeviceSynchronize());
  }
  return VBDR_OK;
}

int vbdr_sketch_get_tuning(const vbdr_sketch* sk, vbdr_tuning* tuning) {
  if (!sk || !tuning) return vbdr_fail(VBDR_EINVAL, "NULL argument");
  *tuning = sk->tune;
  return VBDR_OK;
}

int vbdr_sketch_info(const vbdr_sketch* sk, vbdr_info* out) {
  if (!sk || !out) return vbdr_fail(VBDR_EINVAL, "NULL argument");
  out->m = sk->m, out->g = sk->g, out->b = sk->b, out->L = sk->L, out->k = sk->k;
  out->layout = sk->layout, out->A0 = sk->A0, out->A1 = sk->A1, out->t = sk->t;
  out->state_bytes = sk->bytes;
  out->est_parts = sk->parts;
  out->scan_deferred = sk->def_rec && (sk->tune.scan_defer == 1 || sk->layout == VBDR_LAYOUT_PACKED);
  out->Lc = sk->Lc;
  out->dr_bits = sk->z;
  out->est_tiled = sk->tl_rec != nullptr && sk->tune.est_binned == 3;
  out->window_state_bytes = sk->state_only;
  out->workspace_bytes = sk->bytes - sk->state_only;
  return VBDR_OK;
}

int vbdr_scan_slice(vbdr_sketch* sk, const uint32_t* pairs_dev, uint64_t n, void* stream) {
  if (!sk) return vbdr_fail(VBDR_EINVAL, "sketch is NULL");
  if (n == 0) return VBDR_OK;
  if (!pairs_dev) return vbdr_fail(VBDR_EINVAL, "pairs_dev is NULL");
  if (reinterpret_cast<uintptr_t>(pairs_dev) & 7u) return vbdr_fail(VBDR_EINVAL, "pairs_dev must be 8-byte aligned");
  if (n >= (1ull << 40)) return vbdr_fail(VBDR_EINVAL, "n=%llu too large", (unsigned long long)n);
  if (int rc = vbdr_check_device(sk)) return rc;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const bool stage = sk->g <= kStageMaxG;
  const size_t lds = stage ? (size_t)sk->g * 4 : 0;
  const uint32_t grid =
      grid_cap(sk, (n + kScanBlock * kScanUnroll - 1) / (kScanBlock * kScanUnroll), sk->tune.scan_blocks_per_cu);
  const u32x2* p = reinterpret_cast<const u32x2*>(pairs_dev);
  const uint32_t m32 = (uint32_t)sk->m;
  const bool test = sk->tune.scan_test_first == 1;
  if (sk->def_rec && (sk->tune.scan_defer == 1 || sk->layout == VBDR_LAYOUT_PACKED)) {
    const size_t base_lds = defer_scan_lds(sk->def_tiles);
    int lds_max = 0;
    VBDR_HIP(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, sk->device));
    const int stage_s1 = base_lds + (size_t)sk->g * 4 + 1024 <= (size_t)lds_max;
    const uint32_t dgrid = grid_cap(sk, (n + kDeferChunk - 1) / kDeferChunk, 1);
    auto kern = sk->layout == VBDR_LAYOUT_FAST ? (stage_s1 ? k_scan_defer<true, true> : k_scan_defer<true, false>)
                                               : (stage_s1 ? k_scan_defer<false, true> : k_scan_defer<false, false>);
    hipLaunchKernelGGL(kern, dim3(dgrid), dim3(kDeferBlock), base_lds + (stage_s1 ? (size_t)sk->g * 4 : 0), st, p, n,
                       sk->s1, sk->g, stage_s1, sk->b, sk->A1, m32, sk->def_tiles, sk->def_cap, sk->def_rec,
                       sk->def_fill, sk->dr, sk->mstride, sk->seen, sk->wstride, sk->Lc, sk->bits, sk->z);
    VBDR_LAUNCHED("k_scan_defer");
    return VBDR_OK;
  }
  if (sk->bins && sk->tune.scan_binned == 1) {
    decltype(&k_scan_bin<true, true, true>) bin;
    decltype(&k_scan_apply<true, true>) apply;
    if (sk->layout == VBDR_LAYOUT_FAST) {
      bin = stage ? (test ? k_scan_bin<true, true, true> : k_scan_bin<true, true, false>)
                  : (test ? k_scan_bin<true, false, true> : k_scan_bin<true, false, false>);
      apply = test ? k_scan_apply<true, true> : k_scan_apply<true, false>;
    } else {
      bin = stage ? (test ? k_scan_bin<false, true, true> : k_scan_bin<false, true, false>)
                  : (test ? k_scan_bin<false, false, true> : k_scan_bin<false, false, false>);
      apply = test ? k_scan_apply<false, true> : k_scan_apply<false, false>;
    }
    const uint32_t apply_grid = 8u * (uint32_t)(sk->n_cu / 8) * sk->tune.scan_blocks_per_cu;
    for (uint64_t c = 0; c < n; c += kBinChunk) {
      const uint64_t nc = n - c < kBinChunk ? n - c : kBinChunk;
      hipLaunchKernelGGL(k_bin_reset, dim3(1), dim3(64), 0, st, sk->bin_fill);
      VBDR_LAUNCHED("k_bin_reset");
      const uint32_t grid = grid_cap(sk, (nc + kBinTile - 1) / kBinTile, 4);
      hipLaunchKernelGGL(bin, dim3(grid), dim3(kBinBlock), lds, st, p + c, nc, sk->s1, sk->g, sk->b, sk->A1, m32,
                         sk->bins, sk->bin_fill, sk->dr, sk->mstride, sk->seen, sk->wstride);
      VBDR_LAUNCHED("k_scan_bin");
      hipLaunchKernelGGL(apply, dim3(apply_grid), dim3(kScanBlock), 0, st, sk->bins, sk->bin_fill, sk->dr, sk->mstride,
                         sk->seen, sk->wstride);
      VBDR_LAUNCHED("k_scan_apply");
    }
    return VBDR_OK;
  }
  decltype(&k_scan<true, true, true>) kern;
  if (sk->layout == VBDR_LAYOUT_FAST)
    kern = stage ? (test ? k_scan<true, true, true> : k_scan<true, true, false>)
                 : (test ? k_scan<true, false, true> : k_scan<true, false, false>);
  else
    kern = stage ? (test ? k_scan<false, true, true> : k_scan<false, true, false>)
                 : (test ? k_scan<false, false, true> : k_scan<false, false, false>);
  hipLaunchKernelGGL(kern, dim3(grid), dim3(kScanBlock), lds, st, p, n, sk->s1, sk->g, sk->b, sk->A1, m32, sk->dr,
                     sk->mstride, sk->seen, sk->wstride);
  VBDR_LAUNCHED("k_scan");
  return VBDR_OK;
}

int vbdr_advance_slice(vbdr_sketch* sk, void* stream) {
  if (!sk) return vbdr_fail(VBDR_EINVAL, "sketch is NULL");
  if (int rc = vbdr_check_device(sk)) return rc;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(k_hist_reset, dim3(1), dim3(64), 0, st, sk->hist, 0ull, sk->psum);
  VBDR_LAUNCHED("k_hist_reset");
  if (sk->preg) sk->pcsa_valid = true;  // written by the launch below
  if (sk->layout == VBDR_LAYOUT_PACKED) {
    hipLaunchKernelGGL(k_advance_packed, dim3(sk->def_tiles), dim3(kDeferBlock), (size_t)sk->Lc * kDeferWords * 4, st,
                       sk->bits, sk->wstride, sk->z, sk->Lc, sk->k, sk->reg, sk->reg4, sk->m, sk->hist, sk->def_rec,
                       sk->def_fill, sk->def_cap, sk->def_tiles, sk->sat);
    VBDR_LAUNCHED("k_advance_packed");
    hipLaunchKernelGGL(k_defer_flag, dim3(1), dim3(64), 0, st, sk->def_fill, sk->def_tiles, 0ull);
    VBDR_LAUNCHED("k_defer_flag");
    sk->t++;
    return VBDR_OK;
  }
  if (sk->def_rec && sk->tune.scan_defer == 1) {
    auto kern = sk->layout == VBDR_LAYOUT_FAST ? k_advance_defer<true> : k_advance_defer<false>;
    hipLaunchKernelGGL(kern, dim3(sk->def_tiles), dim3(kDeferBlock), (size_t)sk->L * kDeferWords * 4, st, sk->dr,
                       sk->mstride, sk->seen, sk->wstride, sk->reg, sk->reg4, sk->m, sk->L, sk->k - 1, sk->hist,
                       sk->def_rec, sk->def_fill, sk->def_cap, sk->def_tiles, sk->preg, sk->psum, sk->sat);
    VBDR_LAUNCHED("k_advance_defer");
    hipLaunchKernelGGL(k_defer_flag, dim3(1), dim3(64), 0, st, sk->def_fill, sk->def_tiles, 0ull);
    VBDR_LAUNCHED("k_defer_flag");
    sk->t++;
    return VBDR_OK;
  }
  const uint32_t grid = (uint32_t)(sk->mstride / (kAdvBlock * kAdvBpt));
  auto kern = sk->layout == VBDR_LAYOUT_FAST ? k_advance<true> : k_advance<false>;
  hipLaunchKernelGGL(kern, dim3(grid), dim3(kAdvBlock), 0, st, sk->dr, sk->mstride, sk->seen, sk->wstride, sk->reg,
                     sk->reg4, sk->m, sk->L, sk->k - 1, sk->hist, sk->preg, sk->psum);
  VBDR_LAUNCHED("k_advance");
  sk->t++;
  return VBDR_OK;
}

int vbdr_estimate_ex(vbdr_sketch* sk, const uint32_t* hosts_dev, uint64_t n_hosts, float* out_dev, double* raw_es_dev,
                     uint32_t* hist_dev, void* stream) {
  if (!sk) return vbdr_fail(VBDR_EINVAL, "sketch is NULL");
  if (n_hosts == 0) return VBDR_OK;
  if (!hosts_dev || !out_dev) return vbdr_fail(VBDR_EINVAL, "hosts_dev and out_dev must not be NULL");
  if (n_hosts >= (1ull << 40)) return vbdr_fail(VBDR_EINVAL, "n_hosts too large");
  if (int rc = vbdr_check_device(sk)) return rc;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const bool extra = raw_es_dev || hist_dev;
  if (sk->tl_rec && sk->tune.est_binned == 3 && !extra && n_hosts < (1ull << 32)) {
    uint32_t B = sk->tl_Balloc;  // the block the workspace holds (tiled_block_hosts of the tuning)
    {  // blocks of equal size (whole sub-blocks): no small last block (line rate: 2^19 + 102,494 hosts 1.85 ms,
       // 2 x 313,391 1.81 ms)
      const uint64_t nblk = (n_hosts + B - 1) / B, even = (n_hosts + nblk - 1) / nblk;
      const uint64_t Be = (even + kTileSub - 1) / kTileSub * kTileSub;
      if (Be < B) B = (uint32_t)Be;
    }
    const uint32_t nt = sk->tl_nt, g = sk->g;
    uint32_t cap = sk->tune.est_bin_cap && sk->tune.est_bin_cap < sk->tl_cap ? sk->tune.est_bin_cap : sk->tl_cap;
    cap = cap < 4u ? 4u : cap & ~3u;  // runs hold whole quads of records
    uint32_t lg = 0;
    while ((1u << lg) < g) lg++;
    // a bucket never needs more room than the run it is copied to
    const uint32_t hpc = tile_chunk_hosts(lg), capb = sk->tl_capb < cap ? sk->tl_capb : cap;
    const size_t lds1 = tile_bin_lds(nt, capb, g);  // fits: checked at creation
    for (uint64_t c = 0; c < n_hosts; c += B) {
      const uint32_t nh = (uint32_t)(n_hosts - c < B ? n_hosts - c : B);
      const uint32_t nsb = (nh + kTileSub - 1) / kTileSub;
      if (nsb > 256) return vbdr_fail(VBDR_EINVAL, "tiled estimate: more than 256 sub-blocks in a block");  // pass 2 holds 256 run lengths
      hipLaunchKernelGGL(k_est_tile_clear, dim3(grid_cap(sk, ((uint64_t)nsb * nt + 2ull * nh + 255) / 256, 4)),
                         dim3(256), 0, st, sk->tl_fill, (uint64_t)nsb * nt, reinterpret_cast<uint32_t*>(sk->tl_ovf),
                         (uint64_t)nh * 2);
      VBDR_LAUNCHED("k_est_tile_clear");
      // eight workgroups (one per XCD) per unit of per_xcd; an XCD owns every eighth sub-block
      const uint64_t xcd_chunks = (uint64_t)((nsb + 7) / 8) * (kTileSub / hpc);
      const uint32_t per_xcd = grid_cap(sk, xcd_chunks * 8, 1) / 8;  // one workgroup per CU (LDS)
      const bool pow2 = (sk->m & (sk->m - 1)) == 0;
      uint32_t mshift = 32;
      while (pow2 && (1ull << (32 - mshift)) < sk->m) --mshift;
      hipLaunchKernelGGL(pow2 ? k_est_tile_bin<true> : k_est_tile_bin<false>, dim3(8 * (per_xcd ? per_xcd : 1)),
                         dim3(kTileBinBlock), lds1, st, hosts_dev + c, nh, sk->s1, g, lg, (uint32_t)sk->m, mshift,
                         sk->tl_shift, nt, capb, cap, sk->tl_rec, sk->tl_fill, sk->reg, sk->tl_ovf);
      VBDR_LAUNCHED("k_est_tile_bin");
      // prefetch depth: the whole run when runs are near their expected length
      const auto gather = cap <= 12u * kDeferBlock ? k_est_tile_gather<12> : k_est_tile_gather<20>;
      hipLaunchKernelGGL(gather, dim3(nt), dim3(kDeferBlock), tile_gather_lds(sk->tl_shift), st, sk->reg4,
                         sk->reg, sk->mstride, sk->tl_shift, nt, nsb, cap, sk->tl_rec, sk->tl_fill, sk->tl_part, B,
                         sk->tl_ovf, sk->tl_wide, sk->tl_wcap,
                         reinterpret_cast<uint32_t*>(sk->tl_wide + (uint64_t)nt * sk->tl_wcap), sk->hist, sk->m);
      VBDR_LAUNCHED("k_est_tile_gather");
      hipLaunchKernelGGL(k_est_tile_wide, dim3(8, nt), dim3(256), 0, st, sk->tl_wide, sk->tl_wcap,
                         reinterpret_cast<const uint32_t*>(sk->tl_wide + (uint64_t)nt * sk->tl_wcap), sk->reg,
                         sk->tl_shift, sk->tl_ovf);
      VBDR_LAUNCHED("k_est_tile_wide");
      hipLaunchKernelGGL(k_est_tile_final, dim3((nh + 255) / 256), dim3(256), 0, st, nh, g, (uint32_t)sk->m, nt, B,
                         sk->hist, sk->tl_part, sk->tl_ovf, out_dev + c);
      VBDR_LAUNCHED("k_est_tile_final");
    }
    return VBDR_OK;
  }
  if (sk->est_slots && sk->tune.est_binned == 1 && !extra) {
    const uint32_t hc = sk->est_hc;
    const uint32_t cap = sk->tune.est_bin_cap && sk->tune.est_bin_cap < sk->est_cap ? sk->tune.est_bin_cap : sk->est_cap;
    const uint32_t step = sk->tune.est_bin_hosts && sk->tune.est_bin_hosts < hc ? sk->tune.est_bin_hosts : hc;
    for (uint64_t c = 0; c < n_hosts; c += step) {
      const uint32_t nh = (uint32_t)(n_hosts - c < step ? n_hosts - c : step);
      const uint32_t bgrid = grid_cap(sk, (nh + kEstWaves - 1) / kEstWaves, sk->tune.est_blocks_per_cu);
      const bool guard = sk->g % (64u * kBinRows) != 0, pow2 = (sk->m & (sk->m - 1)) == 0;
      uint32_t mshift = 32;
      while (pow2 && (1ull << (32 - mshift)) < sk->m) --mshift;
      auto bin = guard ? (pow2 ? k_est_bin<true, true> : k_est_bin<true, false>)
                       : (pow2 ? k_est_bin<false, true> : k_est_bin<false, false>);
      hipLaunchKernelGGL(bin, dim3(bgrid), dim3(kEstBlock), (size_t)sk->g * 4, st, hosts_dev + c, nh, sk->s1, sk->g,
                         (uint32_t)sk->m, mshift, sk->reg, cap, hc, sk->est_slots, sk->est_cnt, sk->ovf_u, sk->ovf_v);
      VBDR_LAUNCHED("k_est_bin");
      const uint64_t want = (nh + 4 * kEstWaves - 1) / (4 * kEstWaves);
      const uint64_t capb = (uint64_t)sk->n_cu * sk->tune.est_blocks_per_cu / 8;
      const uint32_t tiles = (uint32_t)(want < capb ? want : (capb ? capb : 1));
      hipLaunchKernelGGL(k_est_gather, dim3(tiles * 8), dim3(kEstBlock), 0, st, nh, sk->reg, sk->reg4, cap, hc,
                         sk->est_slots, sk->est_cnt, sk->part_u, sk->part_v);
      VBDR_LAUNCHED("k_est_gather");
      hipLaunchKernelGGL(k_estimate_final, dim3((nh + 255) / 256), dim3(256), 0, st, nh, sk->g, (uint32_t)sk->m, 8u,
                         sk->hist, sk->part_u, sk->part_v, kPartChunk, sk->ovf_u, sk->ovf_v, out_dev + c);
      VBDR_LAUNCHED("k_estimate_final");
    }
    return VBDR_OK;
  }
  if (sk->parts > 1 && !extra)
    return estimate_partitioned(sk, hosts_dev, n_hosts, out_dev, sk->part_u, sk->part_v, kPartChunk, st);
  return estimate_direct(sk, hosts_dev, n_hosts, out_dev, raw_es_dev, hist_dev, st);
}

int vbdr_estimate(vbdr_sketch* sk, const uint32_t* hosts_dev, uint64_t n_hosts, float* out_dev, void* stream) {
  return vbdr_estimate_ex(sk, hosts_dev, n_hosts, out_dev, nullptr, nullptr, stream);
}

}  // extern "C"

// ------------------------------------------------ estimate without allocation
// The partitioned estimate's per-range partial sums for callers that cannot
// allocate: [8 ranges][kNoAllocHosts] 64-bit harmonic sums, then
// [8 ranges][kNoAllocHosts] 32-bit zero counts, in a static device array
// that every device holds at its own address until the process ends.  Host
// code never passes the array's name to a kernel: it takes the device
// address from hipGetSymbolAddress, once per device.
constexpr uint32_t kNoAllocHosts = 1u << 16;
constexpr uint64_t kNoAllocBytes = 8ull * kNoAllocHosts * (8 + 4);  // 6 MiB
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices];  // device address of `scratch` on each device, once looked up

// Device address of the static scratch on `device`, which must be current.
int scratch_address(int device, void** out) {
  if (device < 0 || device >= kMaxDevices) return vbdr_fail(VBDR_EINVAL, "device %d out of range", device);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      return vbdr_fail(VBDR_EHIP, "hipGetSymbolAddress of the static scratch failed on device %d: %s", device,
                       hipGetErrorString(e));
    }
    g_scratch_dev[device] = p;
  }
  *out = g_scratch_dev[device];
  return VBDR_OK;
}
}  // namespace

extern "C" {

int vbdr_estimate_noalloc(vbdr_sketch* sk, const uint32_t* hosts_dev, uint64_t n_hosts, float* out_dev, void* stream) {
  if (!sk) return vbdr_fail(VBDR_EINVAL, "sketch is NULL");
  if (n_hosts == 0) return VBDR_OK;
  if (!hosts_dev || !out_dev) return vbdr_fail(VBDR_EINVAL, "hosts_dev and out_dev must not be NULL");
  if (n_hosts >= (1ull << 40)) return vbdr_fail(VBDR_EINVAL, "n_hosts too large");
  if (int rc = vbdr_check_device(sk)) return rc;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (sk->parts <= 1) return estimate_direct(sk, hosts_dev, n_hosts, out_dev, nullptr, nullptr, st);
  const uint32_t parts = (uint32_t)(sk->parts == 8 ? sk->tune.est_parts : sk->parts);
  if ((uint64_t)parts * kNoAllocHosts * (8 + 4) > kNoAllocBytes)
    return vbdr_fail(VBDR_EINVAL, "%u pool ranges need more than the %llu bytes of static scratch", parts,
                     (unsigned long long)kNoAllocBytes);
  void* base = nullptr;
  if (int rc = scratch_address(sk->device, &base)) return rc;
  auto* part_u = static_cast<unsigned long long*>(base);
  auto* part_v = reinterpret_cast<uint32_t*>(static_cast<unsigned char*>(base) + 8ull * kNoAllocHosts * 8);
  return estimate_partitioned(sk, hosts_dev, n_hosts, out_dev, part_u, part_v, kNoAllocHosts, st);
}

int vbdr_enable_pcsa(vbdr_sketch* sk, int on) {
  if (!sk) return vbdr_fail(VBDR_EINVAL, "sketch is NULL");
  if (sk->layout != VBDR_LAYOUT_SMALL) return vbdr_fail(VBDR_EINVAL, "PCSA runs need the small layout");
  if (int rc = vbdr_check_device(sk)) return rc;
  VBDR_HIP(hipDeviceSynchronize());
  if (on && !sk->preg) {
    if (vbdr_malloc(&sk->preg, sk->mstride) != hipSuccess || vbdr_malloc(&sk->psum, 8) != hipSuccess) {
      (void)hipGetLastError();
      if (sk->preg) (void)hipFree(sk->preg);
      if (sk->psum) (void)hipFree(sk->psum);
      sk->preg = nullptr, sk->psum = nullptr;
      return vbdr_fail(VBDR_ENOMEM, "device allocation of %llu bytes failed", (unsigned long long)sk->mstride + 8);
    }
    sk->bytes += sk->mstride + 8;
    sk->state_only += sk->mstride + 8;
  } else if (!on && sk->preg) {
    (void)hipFree(sk->preg);
    (void)hipFree(sk->psum);
    sk->preg = nullptr, sk->psum = nullptr;
    sk->bytes -= sk->mstride + 8;
    sk->state_only -= sk->mstride + 8;
  }
  sk->pcsa_valid = false;
  return VBDR_OK;
}

int vbdr_estimate_kind(vbdr_sketch* sk, const uint32_t* hosts_dev, uint64_t n_hosts, int kind, float* out_dev,
                       double* raw_es_dev, void* stream) {
  if (!sk) return vbdr_fail(VBDR_EINVAL, "sketch is NULL");
  if (kind == VBDR_EST_HLL) return vbdr_estimate_ex(sk, hosts_dev, n_hosts, out_dev, raw_es_dev, nullptr, stream);
  if (kind != VBDR_EST_LOGLOG && kind != VBDR_EST_PCSA) return vbdr_fail(VBDR_EINVAL, "unknown estimator %d", kind);
  if (kind == VBDR_EST_PCSA && !sk->pcsa_valid)
    return vbdr_fail(VBDR_ESTATE, "no PCSA runs: enable them (small layout), then advance a slice");
  if (n_hosts == 0) return VBDR_OK;
  if (!hosts_dev || !out_dev) return vbdr_fail(VBDR_EINVAL, "hosts_dev and out_dev must not be NULL");
  if (int rc = vbdr_check_device(sk)) return rc;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  // the pool's sum of values: registers from the histogram, PCSA runs from the advance's sum
  double pool_sum = 0.0;
  if (kind == VBDR_EST_LOGLOG) {
    uint64_t hist[kBins];
    VBDR_HIP(hipMemcpyAsync(hist, sk->hist, sizeof(hist), hipMemcpyDeviceToHost, st));
    VBDR_HIP(hipStreamSynchronize(st));
    uint64_t s = 0;
    for (int r = 0; r < kBins; ++r) s += hist[r] * (uint64_t)r;
    pool_sum = (double)s;
  } else {
    unsigned long long s = 0;
    VBDR_HIP(hipMemcpyAsync(&s, sk->psum, sizeof(s), hipMemcpyDeviceToHost, st));
    VBDR_HIP(hipStreamSynchronize(st));
    pool_sum = (double)s;
  }
  const double q = (double)sk->m, g = (double)sk->g;
  const double cg = kind == VBDR_EST_LOGLOG ? loglog_alpha(g) : 1.0 / 0.77351;
  const double cm = kind == VBDR_EST_LOGLOG ? loglog_alpha(q) : 1.0 / 0.77351;
  const double Em = cm * q * std::exp2(pool_sum / q);
  const uint32_t grid = grid_cap(sk, (n_hosts + kEstWaves - 1) / kEstWaves, sk->tune.est_blocks_per_cu);
  hipLaunchKernelGGL(k_estimate_sum, dim3(grid), dim3(kEstBlock), 0, st, hosts_dev, n_hosts, sk->s1, sk->g,
                     (uint32_t)sk->m, kind == VBDR_EST_LOGLOG ? sk->reg : sk->preg, cg, Em, out_dev, raw_es_dev);
  VBDR_LAUNCHED("k_estimate_sum");
  return VBDR_OK;
}

int vbdr_export_pcsa(vbdr_sketch* sk, uint8_t* preg_host, void* stream) {
  if (!sk || !preg_host) return vbdr_fail(VBDR_EINVAL, "NULL argument");
  if (!sk->pcsa_valid) return vbdr_fail(VBDR_ESTATE, "no PCSA runs: enable them (small layout), then advance a slice");
  if (int rc = vbdr_check_device(sk)) return rc;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  VBDR_HIP(hipStreamSynchronize(st));
  VBDR_HIP(hipMemcpy(preg_host, sk->preg, sk->m, hipMemcpyDeviceToHost));
  return VBDR_OK;
}

int vbdr_export_now(vbdr_sketch* sk, uint8_t* now_dev, void* stream) {
  if (!sk || !now_dev) return vbdr_fail(VBDR_EINVAL, "NULL argument");
  if (sk->layout != VBDR_LAYOUT_FAST) return vbdr_fail(VBDR_EINVAL, "max-LBP1 maps need the fast layout");
  if (int rc = vbdr_check_device(sk)) return rc;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const uint32_t tiles = (uint32_t)((sk->mstride + kDeferTile - 1) / kDeferTile);
  hipLaunchKernelGGL(k_now_export, dim3(tiles), dim3(kDeferBlock), (size_t)sk->L * kDeferWords * 4, st, sk->seen,
                     sk->wstride, sk->mstride, sk->m, sk->L, sk->def_rec, sk->def_fill, sk->def_cap, now_dev);
  VBDR_LAUNCHED("k_now_export");
  return VBDR_OK;
}

int vbdr_import_now(vbdr_sketch* sk, const uint8_t* now_dev, void* stream) {
  if (!sk || !now_dev) return vbdr_fail(VBDR_EINVAL, "NULL argument");
  if (sk->layout != VBDR_LAYOUT_FAST) return vbdr_fail(VBDR_EINVAL, "max-LBP1 maps need the fast layout");
  if (int rc = vbdr_check_device(sk)) return rc;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (sk->def_fill) {  // pending records are replaced; the advance must read the bit-planes
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(256), 0, st, reinterpret_cast<uint32_t*>(sk->def_fill),
                       (uint64_t)sk->def_tiles * 2, 0u);
    VBDR_LAUNCHED("k_fill_u32(def_fill)");
    hipLaunchKernelGGL(k_defer_flag, dim3(1), dim3(64), 0, st, sk->def_fill, sk->def_tiles, 1ull);
    VBDR_LAUNCHED("k_defer_flag");
  }
  hipLaunchKernelGGL(k_now_import, dim3((uint32_t)((sk->wstride + 255) / 256)), dim3(256), 0, st, now_dev, sk->m,
                     sk->L, sk->seen, sk->wstride);
  VBDR_LAUNCHED("k_now_import");
  return VBDR_OK;
}

int vbdr_now_max(const uint8_t* a_dev, const uint8_t* b_dev, uint8_t* out_dev, uint64_t n, void* stream) {
  if (n == 0) return VBDR_OK;
  if (!a_dev || !b_dev || !out_dev) return vbdr_fail(VBDR_EINVAL, "NULL argument");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const uint64_t want = (n + 255) / 256;
  hipLaunchKernelGGL(k_now_max, dim3((uint32_t)(want < 8192 ? want : 8192)), dim3(256), 0, st, a_dev, b_dev, out_dev, n);
  VBDR_LAUNCHED("k_now_max");
  return VBDR_OK;
}

int vbdr_select_hosts(const float* est_dev, const uint32_t* hosts_dev, uint64_t n, float threshold,
                      uint32_t* out_hosts_dev, float* out_est_dev, uint64_t cap, uint32_t* count_dev, void* stream) {
  if (!count_dev) return vbdr_fail(VBDR_EINVAL, "count_dev is NULL");
  if (n >= (1ull << 32)) return vbdr_fail(VBDR_EINVAL, "n=%llu must be below 2^32", (unsigned long long)n);
  if (n && (!est_dev || !hosts_dev)) return vbdr_fail(VBDR_EINVAL, "est_dev and hosts_dev must not be NULL");
  if (cap && (!out_hosts_dev || !out_est_dev)) return vbdr_fail(VBDR_EINVAL, "output arrays must not be NULL");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(k_select_reset, dim3(1), dim3(64), 0, st, count_dev);
  VBDR_LAUNCHED("k_select_reset");
  if (n == 0) return VBDR_OK;
  int dev = 0, n_cu = 0;
  VBDR_HIP(hipGetDevice(&dev));
  VBDR_HIP(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev));
  const uint64_t want = (n + 255) / 256, capb = (uint64_t)n_cu * 8;
  const uint32_t c32 = cap < 0xFFFFFFFFull ? (uint32_t)cap : 0xFFFFFFFFu;
  hipLaunchKernelGGL(k_select, dim3((uint32_t)(want < capb ? want : capb)), dim3(256), 0, st, est_dev, hosts_dev,
                     (uint32_t)n, threshold, out_hosts_dev, out_est_dev, c32, count_dev);
  VBDR_LAUNCHED("k_select");
  return VBDR_OK;
}

int vbdr_export_state(vbdr_sketch* sk, uint8_t* dr_host, uint32_t* bs_host, uint8_t* reg_host, uint64_t* hist_host,
                      void* stream) {
  if (!sk) return vbdr_fail(VBDR_EINVAL, "sketch is NULL");
  if (int rc = vbdr_check_device(sk)) return rc;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (int rc = defer_flush(sk, st)) return rc;  // the open slice's deferred records join the state
  VBDR_HIP(hipStreamSynchronize(st));
  const uint64_t m = sk->m, L = sk->L;
  if (dr_host && sk->dr) {
    std::vector<uint8_t> plane(m);
    for (uint64_t i = 0; i < L; ++i) {
      VBDR_HIP(hipMemcpy(plane.data(), sk->dr + i * sk->mstride, m, hipMemcpyDeviceToHost));
      for (uint64_t p = 0; p < m; ++p) dr_host[p * L + i] = plane[p];
    }
  } else if (dr_host) {  // packed: z bit-planes per recorder, recorders above Lc never set
    const uint8_t sat = (uint8_t)((1u << sk->z) - 1);
    std::vector<uint32_t> bp((uint64_t)sk->z * sk->wstride);
    for (uint64_t i = 0; i < L; ++i) {
      if (i >= sk->Lc) {
        for (uint64_t p = 0; p < m; ++p) dr_host[p * L + i] = sat;
        continue;
      }
      VBDR_HIP(hipMemcpy(bp.data(), sk->bits + i * sk->z * sk->wstride, bp.size() * 4, hipMemcpyDeviceToHost));
      for (uint64_t p = 0; p < m; ++p) {
        uint32_t v = 0;
        for (uint32_t b = 0; b < sk->z; ++b) v |= ((bp[b * sk->wstride + (p >> 5)] >> (p & 31)) & 1u) << b;
        dr_host[p * L + i] = (uint8_t)v;
      }
    }
  }
  if (bs_host) {
    std::memset(bs_host, 0, m * sizeof(uint32_t));
    if (sk->seen) {
      std::vector<uint32_t> plane(sk->wstride);
      for (uint64_t i = 0; i < L; ++i) {
        VBDR_HIP(hipMemcpy(plane.data(), sk->seen + i * sk->wstride, sk->wstride * 4, hipMemcpyDeviceToHost));
        for (uint64_t p = 0; p < m; ++p) bs_host[p] |= ((plane[p >> 5] >> (p & 31)) & 1u) << i;
      }
    }
  }
  if (reg_host) VBDR_HIP(hipMemcpy(reg_host, sk->reg, m, hipMemcpyDeviceToHost));
  if (hist_host) VBDR_HIP(hipMemcpy(hist_host, sk->hist, kBins * sizeof(uint64_t), hipMemcpyDeviceToHost));
  return VBDR_OK;
}

int vbdr_import_state(vbdr_sketch* sk, const uint8_t* dr_host, const uint32_t* bs_host, const uint8_t* reg_host,
                      const uint64_t* hist_host, uint64_t t, void* stream) {
  if (!sk) return vbdr_fail(VBDR_EINVAL, "sketch is NULL");
  if (!dr_host || !reg_host || !hist_host) return vbdr_fail(VBDR_EINVAL, "dr_host, reg_host and hist_host are required");
  if (bs_host && !sk->seen) {
    for (uint64_t p = 0; p < sk->m; ++p)
      if (bs_host[p]) return vbdr_fail(VBDR_EINVAL, "small-layout sketch cannot hold bsLBP1 bits");
  }
  uint64_t total = 0;
  for (int r = 0; r < kBins; ++r) total += hist_host[r];
  if (total != sk->m) return vbdr_fail(VBDR_EINVAL, "histogram does not sum to m");
  const uint64_t m = sk->m, L = sk->L;
  std::vector<uint64_t> reg_hist(kBins, 0);
  for (uint64_t p = 0; p < m; ++p) {
    if (reg_host[p] > sk->Lc)
      return vbdr_fail(VBDR_EINVAL, "register %u of BDR %llu exceeds %u", reg_host[p], (unsigned long long)p, sk->Lc);
    reg_hist[reg_host[p]]++;
  }
  for (int r = 0; r < kBins; ++r)  // the estimates read both (the tiled one picks its sum width from hist[0])
    if (reg_hist[r] != hist_host[r]) return vbdr_fail(VBDR_EINVAL, "histogram does not match the registers at %d", r);
  if (bs_host)
    for (uint64_t p = 0; p < m; ++p)
      if (L < 32 && (bs_host[p] >> L)) return vbdr_fail(VBDR_EINVAL, "bsLBP1 of BDR %llu has bits above L", (unsigned long long)p);
  if (int rc = vbdr_check_device(sk)) return rc;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  VBDR_HIP(hipStreamSynchronize(st));
  if (sk->dr) {
    std::vector<uint8_t> plane(sk->mstride, (uint8_t)kSat);
    for (uint64_t i = 0; i < L; ++i) {
      for (uint64_t p = 0; p < m; ++p) plane[p] = dr_host[p * L + i];
      VBDR_HIP(hipMemcpy(sk->dr + i * sk->mstride, plane.data(), sk->mstride, hipMemcpyHostToDevice));
    }
  } else {  // packed: values capped at 2^z - 1, recorders above Lc dropped, padding at 2^z - 1
    const uint32_t sat = (1u << sk->z) - 1;
    std::vector<uint32_t> bp((uint64_t)sk->z * sk->wstride);
    for (uint64_t i = 0; i < sk->Lc; ++i) {
      std::fill(bp.begin(), bp.end(), ~0u);
      for (uint64_t p = 0; p < m; ++p) {
        const uint32_t v = dr_host[p * L + i] < sat ? dr_host[p * L + i] : sat;
        for (uint32_t b = 0; b < sk->z; ++b)
          if (!((v >> b) & 1u)) bp[b * sk->wstride + (p >> 5)] &= ~(1u << (p & 31));
      }
      VBDR_HIP(hipMemcpy(sk->bits + i * sk->z * sk->wstride, bp.data(), bp.size() * 4, hipMemcpyHostToDevice));
    }
  }
  if (sk->seen) {
    std::vector<uint32_t> plane(sk->wstride);
    for (uint64_t i = 0; i < L; ++i) {
      std::fill(plane.begin(), plane.end(), 0u);
      if (bs_host)
        for (uint64_t p = 0; p < m; ++p) plane[p >> 5] |= ((bs_host[p] >> i) & 1u) << (p & 31);
      VBDR_HIP(hipMemcpy(sk->seen + i * sk->wstride, plane.data(), sk->wstride * 4, hipMemcpyHostToDevice));
    }
  }
  {
    std::vector<uint8_t> r(sk->mstride, 0);
    std::memcpy(r.data(), reg_host, m);
    VBDR_HIP(hipMemcpy(sk->reg, r.data(), sk->mstride, hipMemcpyHostToDevice));
  }
  VBDR_HIP(hipMemcpy(sk->hist, hist_host, kBins * sizeof(uint64_t), hipMemcpyHostToDevice));
  if (sk->def_fill) {  // drop pending records; the imported bsLBP1 bits must be read by the advance
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(256), 0, nullptr, reinterpret_cast<uint32_t*>(sk->def_fill),
                       (uint64_t)(sk->def_tiles + 1) * 2, 0u);
    VBDR_LAUNCHED("k_fill_u32(def_fill)");
    hipLaunchKernelGGL(k_defer_flag, dim3(1), dim3(64), 0, nullptr, sk->def_fill, sk->def_tiles, 1ull);
    VBDR_LAUNCHED("k_defer_flag");
  }
  hipLaunchKernelGGL(k_pack_reg4, dim3(grid_cap(sk, (sk->mstride / 2 + 255) / 256, 8)), dim3(256), 0, nullptr, sk->reg,
                     sk->reg4, sk->mstride / 2);
  VBDR_LAUNCHED("k_pack_reg4");
  VBDR_HIP(hipStreamSynchronize(nullptr));
  sk->t = t;
  sk->pcsa_valid = false;  // PCSA runs are not part of the canonical state: valid again after an advance
  return VBDR_OK;
}

}  // extern "C"
