// Host-side internals shared by the translation units of libvbdr.so.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "vbdr.h"
#include "vbdr_device.h"

constexpr uint64_t kPad = 4096;             // BDR padding granule of a plane
constexpr uint32_t kStageMaxG = 8192;       // s1 staged in LDS up to 32 KiB
constexpr uint32_t kCusPerXcd = 32;         // gfx950: 8 XCDs x 32 CUs
constexpr uint64_t kPartMinM = 1ull << 22;  // pools whose registers outgrow one XCD's L2
constexpr uint32_t kPartChunk = 1u << 20;   // hosts per partitioned-estimate pass
constexpr uint32_t kLearnChunk = 1u << 15;  // hosts per histogram pass of the learned estimate
constexpr uint64_t kBinMaxM = 1ull << 27;   // binned scan records pack (pidx << 5) | (LBP1 - 1)
constexpr uint32_t kBinChunk = 1u << 24;    // pairs per binned-scan pass (records stay cache resident)
constexpr uint32_t kBinCap = kBinChunk / 8 + kBinChunk / 32 + 65536;  // records per bin per pass
constexpr uint32_t kDeferTile = 1u << 15;   // BDRs per deferred-apply tile (one advance workgroup)
constexpr uint32_t kDeferSlots = 2;         // record slots per BDR per slice before the direct fallback

struct vbdr_sketch {
  int device;
  int n_cu;
  uint64_t m;
  uint32_t g, b, L, k;
  int layout;
  uint32_t A0, A1;
  uint64_t t;
  uint64_t mstride, wstride;
  uint8_t* dr;                    // byte DRs, plane-major (fast and small layouts)
  uint32_t* bits;                 // packed layout: bit-plane (r-1)*z + b holds bit b of DR r, 32 BDRs a word
  uint32_t z, Lc;                 // packed layout: bits per DR, recorders per BDR (else 8 and L)
  uint32_t* seen;
  uint8_t* reg;
  unsigned long long* hist;
  uint32_t* s1;
  uint8_t* reg4;               // registers as nibbles, min(reg, 15); 15 = read reg
  int parts;                   // XCD partitions of the estimate (1 = direct gather)
  unsigned long long* part_u;  // [parts][kPartChunk] partial harmonic sums
  uint32_t* part_v;            // [parts][kPartChunk] partial zero counts
  uint32_t* hist_ws;           // [parts][kLearnChunk][33] per-host (partial) histograms
  float* est_ws;               // [kLearnChunk] plain estimates of a histogram pass
  uint32_t* bins;              // [parts][kBinCap] binned scan records (large pools)
  uint32_t* bin_fill;          // [parts] records written per bin
  uint32_t* est_slots;         // [8][est_hc][est_cap] binned-estimate pidx runs
  uint32_t* est_cnt;           // [8][est_hc] run lengths
  unsigned long long* ovf_u;   // [est_hc] overflow partial sums
  uint32_t* ovf_v;             // [est_hc]
  uint32_t est_cap, est_hc;
  bool bin_ok, est_ok;            // the binned scan / estimate workspaces may be allocated (on request)
  bool tl_ok;                     // the LDS-tiled estimate fits this pool (workspaces on request)
  uint32_t tl_shift, tl_nt, tl_B, tl_cap;  // tile = 2^tl_shift registers; tiles; hosts per block; records per run
  uint32_t tl_capb;               // entries per LDS bucket of a (chunk, tile) in the first pass
  uint32_t* tl_rec;               // [B / 2048][nt][cap] records of a block
  uint32_t* tl_fill;              // [B / 2048][nt] run lengths
  uint32_t* tl_part;              // [nt][B] per-tile sums of a block's hosts, packed (exact or moved to tl_ovf)
  unsigned long long* tl_ovf;     // [B] sums of run overflows
  uint2* tl_wide;                 // [nt][tl_wcap] records of registers >= 15 found by pass 2, then [nt] counts
  uint32_t tl_wcap;
  uint32_t tl_Balloc;             // hosts per block the record, run-length and sum buffers hold (<= tl_B)
  uint32_t* def_rec;              // [def_tiles][def_cap] deferred scan records (pidx << 5 | LBP1-1)
  uint32_t* sat;                  // deferred scans: [wstride] bit r-1 = DR[r] of all 32 BDRs saturated (255, or 2^z - 1)
  unsigned long long* def_fill;   // [def_tiles + 1] records per tile; the last word flags direct updates
  uint32_t def_tiles, def_cap;
  bool lean;                      // no optional workspaces (sketches owned by a batch)
  uint8_t* preg;                  // small layout, on request: PCSA run of each BDR, last closed window
  unsigned long long* psum;       // sum of preg over the pool
  bool pcsa_valid;                // preg was written by an advance since it was enabled
  uint64_t bytes;                 // device bytes held: the window state plus every workspace
  uint64_t state_only;            // of which the window state: DRs, bsLBP1, registers, masks, seeds, PCSA runs
  vbdr_tuning tune;
};

// vbdr_sketch_create_layout without the optional large-pool workspaces;
// with defer, pools of 2^22..2^26 BDRs keep the record runs of deferred scans.
int vbdr_sketch_create_lean(uint64_t m, uint32_t g, uint32_t k, uint64_t hash_seed, int layout, bool defer,
                            vbdr_sketch** out);

// A batch member whose scans defer their updates, as the batch's deferred
// scan and advance kernels read it from device memory.  pairs, n_pairs and
// scan_item0 change every step; the rest is the sketch's.
constexpr uint32_t kMaxDeferMembers = 256;
struct DeferItem {
  const uint32_t* pairs;
  uint64_t n_pairs;
  const uint32_t* s1;
  uint8_t* dr;
  uint32_t* seen;
  uint8_t* reg;
  uint8_t* reg4;
  unsigned long long* hist;
  uint32_t* recs;
  unsigned long long* fill;
  uint32_t* sat;
  uint64_t mstride, wstride, m;
  uint32_t b, A1, tiles, cap, L, thr, layout;
  uint32_t scan_item0;  // first scan item (chunk) of the member this step
  uint32_t adv_item0;   // first advance item (tile) of the member
  uint32_t pad;
};
struct DeferHdr {
  uint32_t scan_total;  // scan items of the step
  uint32_t pad[3];
};

// The sketch's fields of its DeferItem (pairs, n_pairs and the item offsets zero).
void vbdr_defer_member(const vbdr_sketch* sk, DeferItem* d);
// Pairs per scan item of a deferred member.
uint32_t vbdr_defer_chunk_pairs();
// Phase 0: the deferred members' scans (grid workgroups over hdr->scan_total
// items); phase 1: their advances (adv_total tiles) and the flag reset.
int vbdr_launch_batch_defer(const DeferItem* items_dev, const DeferHdr* hdr_dev, uint32_t S, uint32_t max_tiles,
                            uint32_t max_L, uint32_t adv_total, uint32_t grid, int phase, hipStream_t st);

constexpr uint64_t kPackedMaxM = 1ull << 26;  // packed pools: records' tiles must fit the deferred scan's LDS

// Records the calling thread's error message and returns code.
int vbdr_fail(int code, const char* fmt, ...);

// hipMalloc for every device allocation of the library, so that
// vbdr_test_fail_alloc can make a chosen one fail.
hipError_t vbdr_malloc_bytes(void** p, size_t bytes);
template <class T>
inline hipError_t vbdr_malloc(T** p, size_t bytes) {
  return vbdr_malloc_bytes(reinterpret_cast<void**>(p), bytes);
}

#define VBDR_HIP(call)                                                                         \
  do {                                                                                         \
    hipError_t e_ = (call);                                                                    \
    if (e_ != hipSuccess) return vbdr_fail(VBDR_EHIP, "%s: %s", #call, hipGetErrorString(e_)); \
  } while (0)

#define VBDR_LAUNCHED(name)                                                                         \
  do {                                                                                              \
    hipError_t e_ = hipGetLastError();                                                              \
    if (e_ != hipSuccess) return vbdr_fail(VBDR_EHIP, "launch of %s: %s", name, hipGetErrorString(e_)); \
  } while (0)

// VBDR_EINVAL unless the sketch's device is current.
int vbdr_check_device(const vbdr_sketch* sk);

// Register histograms of nh <= kLearnChunk hosts into sk->hist_ws: with
// sk->parts == 1 one full histogram per host ([h][33]); otherwise one partial
// histogram per XCD range ([x][h][33]), to be summed over x.
int vbdr_hist_pass(vbdr_sketch* sk, const uint32_t* hosts_dev, uint32_t nh, hipStream_t st);
