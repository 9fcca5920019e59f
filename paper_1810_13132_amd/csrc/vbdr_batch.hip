// Many independent sketches (uneven streams, pools, windows, g, layouts)
// advanced per slice by three persistent work-queue kernels -- scan, advance,
// estimate -- that pull (sketch, tile) items from device counters.  Members
// with pools of 2^22..2^26 BDRs instead write sorted record runs in their scan
// and apply them in their advance, as a single sketch does (two more kernels
// over all such members, in vbdr.hip).  Each sketch's per-slice inputs live in
// a device descriptor table refreshed by one host-to-device copy per step, so
// the kernel sequence is captured once into a hipGraph and replayed.  Every
// block leaves its loop when the queue is drained, so a launch always
// completes.
#include <hip/hip_runtime.h>

#include <cstring>
#include <new>
#include <vector>

#include "vbdr_internal.h"

using namespace vbdr;

namespace {

constexpr uint32_t kMaxBatch = 256;
constexpr int kBBlock = 256;
constexpr uint32_t kAdvTile = 256 * 16;  // BDRs per advance item (one block of 16-BDR groups)

struct BatchDesc {
  uint8_t* dr;
  uint32_t* seen;
  uint8_t* reg;
  uint8_t* reg4;
  unsigned long long* hist;
  const uint32_t* s1;
  uint64_t mstride, wstride;
  uint32_t m, g, b, L, k, layout, A1, test;
  const uint32_t* pairs;  // per step
  uint64_t n_pairs;
  const uint32_t* hosts;
  uint64_t n_hosts;
  float* out;
  uint32_t scan_item0, adv_item0, est_item0, pad;
};

struct BatchHdr {
  uint32_t scan_total, adv_total, est_total, pad0;
  uint32_t counter[3];  // reset to 0 by every step's table upload
  uint32_t pad1;
};

__device__ __forceinline__ uint32_t find_sketch(const uint32_t* starts, uint32_t S, uint32_t item) {
  uint32_t lo = 0, hi = S - 1;  // last s with starts[s] <= item
  while (lo < hi) {
    const uint32_t mid = (lo + hi + 1) >> 1;
    if (starts[mid] <= item) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Next work item of a queue, shared by the whole block.
__device__ __forceinline__ uint32_t next_item(uint32_t* counter, uint32_t* sh) {
  __syncthreads();
  if (threadIdx.x == 0) *sh = atomicAdd(counter, 1u);
  __syncthreads();
  return *sh;
}

__global__ __launch_bounds__(kBBlock) void k_batch_scan(const BatchDesc* __restrict__ d, BatchHdr* __restrict__ hdr,
                                                        uint32_t S, uint32_t tile) {
  __shared__ uint32_t starts[kMaxBatch];
  __shared__ uint32_t cur;
  for (uint32_t s = threadIdx.x; s < S; s += kBBlock) starts[s] = d[s].scan_item0;
  const uint32_t total = hdr->scan_total;
  for (;;) {
    const uint32_t item = next_item(&hdr->counter[0], &cur);
    if (item >= total) break;
    const uint32_t s = find_sketch(starts, S, item);
    const BatchDesc& D = d[s];
    const uint64_t lo = (uint64_t)(item - starts[s]) * tile;
    const uint64_t hi = lo + tile < D.n_pairs ? lo + tile : D.n_pairs;
    const u32x2* pairs = reinterpret_cast<const u32x2*>(D.pairs);
    constexpr int kPer = 8;  // pairs per thread at a time: their loads and state reads overlap
    for (uint64_t i0 = lo + threadIdx.x; i0 < hi; i0 += (uint64_t)kPer * kBBlock) {
      u32x2 p[kPer];
      bool ok[kPer];
#pragma unroll
      for (int v = 0; v < kPer; ++v) {
        const uint64_t i = i0 + (uint64_t)v * kBBlock;
        ok[v] = i < hi;
        p[v] = ok[v] ? __builtin_nontemporal_load(pairs + i) : u32x2{0u, 0u};
      }
      if (D.layout == VBDR_LAYOUT_FAST) {
        if (D.test) scan_pairs<true, true, kPer>(p, ok, D.s1, D.b, D.A1, D.m, D.dr, D.mstride, D.seen, D.wstride);
        else scan_pairs<true, false, kPer>(p, ok, D.s1, D.b, D.A1, D.m, D.dr, D.mstride, D.seen, D.wstride);
      } else {
        if (D.test) scan_pairs<false, true, kPer>(p, ok, D.s1, D.b, D.A1, D.m, D.dr, D.mstride, D.seen, D.wstride);
        else scan_pairs<false, false, kPer>(p, ok, D.s1, D.b, D.A1, D.m, D.dr, D.mstride, D.seen, D.wstride);
      }
    }
  }
}

__global__ void k_batch_hist_reset(const BatchDesc* __restrict__ d) {
  if (threadIdx.x < kBins) d[blockIdx.x].hist[threadIdx.x] = 0ull;
}

__global__ __launch_bounds__(kBBlock) void k_batch_advance(const BatchDesc* __restrict__ d,
                                                           BatchHdr* __restrict__ hdr, uint32_t S) {
  __shared__ uint32_t starts[kMaxBatch];
  __shared__ uint32_t cur;
  // four histogram copies per wave (lane & 3): registers crowd a few values
  __shared__ uint32_t lh[kBBlock / 64][4][kBins];
  for (uint32_t s = threadIdx.x; s < S; s += kBBlock) starts[s] = d[s].adv_item0;
  const uint32_t total = hdr->adv_total;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (;;) {
    // next_item's barrier also orders the previous item's histogram read
    // before this item's reset
    const uint32_t item = next_item(&hdr->counter[1], &cur);
    if (item >= total) break;
    for (int i = lane; i < 4 * kBins; i += 64) (&lh[wave][0][0])[i] = 0;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    const uint32_t s = find_sketch(starts, S, item);
    const BatchDesc& D = d[s];
    const uint64_t base = (uint64_t)(item - starts[s]) * kAdvTile + threadIdx.x * 16u;
    uint32_t R[4];
    const uint32_t bias = swar_gt_bias(D.k - 1);
    if (D.layout == VBDR_LAYOUT_FAST)
      advance_group<true>(D.dr, D.mstride, D.seen, D.wstride, D.reg, D.reg4, base, D.L, bias, R);
    else
      advance_group<false>(D.dr, D.mstride, D.seen, D.wstride, D.reg, D.reg4, base, D.L, bias, R);
#pragma unroll
    for (int j = 0; j < 16; ++j)
      if (base + j < D.m) atomicAdd(&lh[wave][lane & 3][(R[j >> 2] >> (8 * (j & 3))) & 0xFFu], 1u);
    __syncthreads();
    if (threadIdx.x < kBins) {
      uint32_t c = 0;
      for (int w = 0; w < kBBlock / 64; ++w)
        for (int q = 0; q < 4; ++q) c += lh[w][q][threadIdx.x];
      if (c) atomicAdd(D.hist + threadIdx.x, (unsigned long long)c);
    }
  }
}

__global__ __launch_bounds__(kBBlock) void k_batch_estimate(const BatchDesc* __restrict__ d,
                                                            BatchHdr* __restrict__ hdr, uint32_t S, uint32_t tile) {
  __shared__ uint32_t starts[kMaxBatch];
  __shared__ uint32_t cur;
  __shared__ double em;
  for (uint32_t s = threadIdx.x; s < S; s += kBBlock) starts[s] = d[s].est_item0;
  const uint32_t total = hdr->est_total;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (;;) {
    const uint32_t item = next_item(&hdr->counter[2], &cur);
    if (item >= total) break;
    const uint32_t s = find_sketch(starts, S, item);
    const BatchDesc& D = d[s];
    if (threadIdx.x == 0) em = pool_estimate(D.hist, (double)D.m);
    __syncthreads();
    const double Em = em;
    const uint64_t lo = (uint64_t)(item - starts[s]) * tile;
    const uint64_t hi = lo + tile < D.n_hosts ? lo + tile : D.n_hosts;
    for (uint64_t h = lo + wave; h < hi; h += kBBlock / 64) {
      uint64_t U;
      uint32_t V;
      host_harmonic<8>(mm3_key(D.hosts[h]), D.s1, D.g, D.m, D.reg4, D.reg, lane, U, V);
      if (lane == 0) {
        const double Es = hll_estimate(U, V, (double)D.g);
        const double n = noise_removed(Es, Em, (double)D.m, (double)D.g);
        D.out[h] = (float)(n > 0.0 ? n : 0.0);
      }
    }
  }
}

}  // namespace

struct vbdr_batch {
  int device;
  int n_cu;
  uint32_t S;
  std::vector<vbdr_sketch*> sk;
  BatchDesc* desc_dev;
  BatchHdr* hdr_dev;
  uint8_t* staging[2];  // pinned: descriptors then header
  hipEvent_t staged[2];
  int next;
  hipStream_t st;       // batch-owned stream (graphs cannot capture the null stream)
  hipEvent_t ev_in, ev_out;
  hipGraph_t graph;
  hipGraphExec_t exec;
  vbdr_batch_tuning tune;
  // members with deferred scans: index in the deferred table, or ~0u
  std::vector<uint32_t> defer_of;
  uint32_t n_defer, defer_max_tiles, defer_max_L, defer_tiles;
  // learned estimators by member (NULL: plain), owned by the caller
  std::vector<const vbdr_mlp*> mlp;
};

namespace {

// Device table: [S] BatchDesc, BatchHdr, [n_defer] DeferItem, DeferHdr.
size_t table_bytes(uint32_t S, uint32_t n_defer) {
  return sizeof(BatchDesc) * S + sizeof(BatchHdr) + sizeof(DeferItem) * n_defer + sizeof(DeferHdr);
}
DeferItem* defer_items(uint8_t* table, uint32_t S) {
  return reinterpret_cast<DeferItem*>(table + sizeof(BatchDesc) * S + sizeof(BatchHdr));
}
DeferHdr* defer_hdr(uint8_t* table, uint32_t S, uint32_t n_defer) {
  return reinterpret_cast<DeferHdr*>(table + sizeof(BatchDesc) * S + sizeof(BatchHdr) + sizeof(DeferItem) * n_defer);
}

int launch_step_kernels(vbdr_batch* bt) {
  const uint32_t grid = (uint32_t)bt->n_cu * bt->tune.blocks_per_cu;
  hipLaunchKernelGGL(k_batch_scan, dim3(grid), dim3(kBBlock), 0, bt->st, bt->desc_dev, bt->hdr_dev, bt->S,
                     bt->tune.scan_tile);
  VBDR_LAUNCHED("k_batch_scan");
  uint8_t* table = reinterpret_cast<uint8_t*>(bt->desc_dev);
  DeferItem* ditems = defer_items(table, bt->S);
  DeferHdr* dhdr = defer_hdr(table, bt->S, bt->n_defer);
  if (int rc = vbdr_launch_batch_defer(ditems, dhdr, bt->n_defer, bt->defer_max_tiles, bt->defer_max_L,
                                       bt->defer_tiles, (uint32_t)bt->n_cu, 0, bt->st))
    return rc;
  hipLaunchKernelGGL(k_batch_hist_reset, dim3(bt->S), dim3(64), 0, bt->st, bt->desc_dev);
  VBDR_LAUNCHED("k_batch_hist_reset");
  hipLaunchKernelGGL(k_batch_advance, dim3(grid), dim3(kBBlock), 0, bt->st, bt->desc_dev, bt->hdr_dev, bt->S);
  VBDR_LAUNCHED("k_batch_advance");
  if (int rc = vbdr_launch_batch_defer(ditems, dhdr, bt->n_defer, bt->defer_max_tiles, bt->defer_max_L,
                                       bt->defer_tiles, (uint32_t)bt->n_cu, 1, bt->st))
    return rc;
  hipLaunchKernelGGL(k_batch_estimate, dim3(grid), dim3(kBBlock), 0, bt->st, bt->desc_dev, bt->hdr_dev, bt->S,
                     bt->tune.est_tile);
  VBDR_LAUNCHED("k_batch_estimate");
  return VBDR_OK;
}

void drop_graph(vbdr_batch* bt) {
  if (bt->exec) (void)hipGraphExecDestroy(bt->exec);
  if (bt->graph) (void)hipGraphDestroy(bt->graph);
  bt->exec = nullptr;
  bt->graph = nullptr;
}

}  // namespace

extern "C" {

int vbdr_batch_create(uint32_t n_sketches, const vbdr_batch_params* params, vbdr_batch** out) {
  if (!out || !params) return vbdr_fail(VBDR_EINVAL, "NULL argument");
  *out = nullptr;
  if (n_sketches < 1 || n_sketches > kMaxBatch) return vbdr_fail(VBDR_EINVAL, "1..%u sketches per batch", kMaxBatch);
  vbdr_batch* bt = new (std::nothrow) vbdr_batch();
  if (!bt) return vbdr_fail(VBDR_ENOMEM, "host allocation failed");
  bt->S = n_sketches;
  bt->tune.scan_tile = 8192;
  bt->tune.est_tile = 64;
  bt->tune.blocks_per_cu = 8;
  bt->tune.use_graph = 1;
  int rc = VBDR_OK;
  do {
    if (hipGetDevice(&bt->device) != hipSuccess ||
        hipDeviceGetAttribute(&bt->n_cu, hipDeviceAttributeMultiprocessorCount, bt->device) != hipSuccess) {
      rc = vbdr_fail(VBDR_EHIP, "device query failed");
      break;
    }
    for (uint32_t i = 0; i < n_sketches; ++i) {
      vbdr_sketch* s = nullptr;
      const vbdr_batch_params& p = params[i];
      if ((rc = vbdr_sketch_create_lean(p.m, p.g, p.k, p.hash_seed, p.layout, true, &s)) != VBDR_OK) break;
      bt->sk.push_back(s);
      // members with record runs scan and advance through the deferred kernels
      bt->mlp.push_back(nullptr);
      if (s->def_rec) {
        bt->defer_of.push_back(bt->n_defer++);
        bt->defer_max_tiles = bt->defer_max_tiles > s->def_tiles ? bt->defer_max_tiles : s->def_tiles;
        bt->defer_max_L = bt->defer_max_L > s->L ? bt->defer_max_L : s->L;
        bt->defer_tiles += s->def_tiles;
      } else {
        bt->defer_of.push_back(~0u);
      }
    }
    if (rc != VBDR_OK) break;
    const size_t tb = table_bytes(n_sketches, bt->n_defer);
    if (vbdr_malloc(&bt->desc_dev, tb) != hipSuccess || hipHostMalloc(&bt->staging[0], tb) != hipSuccess ||
        hipHostMalloc(&bt->staging[1], tb) != hipSuccess) {
      rc = vbdr_fail(VBDR_ENOMEM, "batch table allocation failed");
      break;
    }
    bt->hdr_dev = reinterpret_cast<BatchHdr*>(reinterpret_cast<uint8_t*>(bt->desc_dev) + sizeof(BatchDesc) * n_sketches);
    if (hipStreamCreateWithFlags(&bt->st, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&bt->ev_in, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&bt->ev_out, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&bt->staged[0], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&bt->staged[1], hipEventDisableTiming) != hipSuccess) {
      rc = vbdr_fail(VBDR_EHIP, "stream or event creation failed");
      break;
    }
  } while (0);
  if (rc != VBDR_OK) {
    vbdr_batch_destroy(bt);
    return rc;
  }
  *out = bt;
  return VBDR_OK;
}

void vbdr_batch_destroy(vbdr_batch* bt) {
  if (!bt) return;
  (void)hipDeviceSynchronize();
  drop_graph(bt);
  for (vbdr_sketch* s : bt->sk) vbdr_sketch_destroy(s);
  if (bt->desc_dev) (void)hipFree(bt->desc_dev);
  for (int i = 0; i < 2; ++i) {
    if (bt->staging[i]) (void)hipHostFree(bt->staging[i]);
    if (bt->staged[i]) (void)hipEventDestroy(bt->staged[i]);
  }
  if (bt->ev_in) (void)hipEventDestroy(bt->ev_in);
  if (bt->ev_out) (void)hipEventDestroy(bt->ev_out);
  if (bt->st) (void)hipStreamDestroy(bt->st);
  delete bt;
}

int vbdr_batch_set_mlp(vbdr_batch* bt, uint32_t i, const vbdr_mlp* mlp) {
  if (!bt || i >= bt->S) return vbdr_fail(VBDR_EINVAL, "no sketch %u in this batch", i);
  VBDR_HIP(hipStreamSynchronize(bt->st));  // steps already enqueued keep the estimator they were given
  bt->mlp[i] = mlp;
  return VBDR_OK;
}

vbdr_sketch* vbdr_batch_sketch(vbdr_batch* bt, uint32_t i) {
  if (!bt || i >= bt->S) {
    vbdr_fail(VBDR_EINVAL, "no sketch %u in this batch", i);
    return nullptr;
  }
  return bt->sk[i];
}

int vbdr_batch_set_tuning(vbdr_batch* bt, const vbdr_batch_tuning* t) {
  if (!bt || !t) return vbdr_fail(VBDR_EINVAL, "NULL argument");
  if (t->scan_tile < 256 || t->scan_tile > (1u << 22) || t->est_tile < 4 || t->est_tile > (1u << 16) ||
      t->blocks_per_cu < 1 || t->blocks_per_cu > 32 || t->use_graph < 0 || t->use_graph > 1)
    return vbdr_fail(VBDR_EINVAL, "tuning out of range");
  if (std::memcmp(t, &bt->tune, sizeof(*t)) != 0) {
    VBDR_HIP(hipStreamSynchronize(bt->st));
    drop_graph(bt);  // launch shapes are baked into the captured graph
    bt->tune = *t;
  }
  return VBDR_OK;
}

int vbdr_batch_get_tuning(const vbdr_batch* bt, vbdr_batch_tuning* t) {
  if (!bt || !t) return vbdr_fail(VBDR_EINVAL, "NULL argument");
  *t = bt->tune;
  return VBDR_OK;
}

int vbdr_batch_step(vbdr_batch* bt, const uint32_t* const* pairs_dev, const uint64_t* n_pairs,
                    const uint32_t* const* hosts_dev, const uint64_t* n_hosts, float* const* out_dev, void* stream) {
  if (!bt || !pairs_dev || !n_pairs || !hosts_dev || !n_hosts || !out_dev) return vbdr_fail(VBDR_EINVAL, "NULL argument");
  int cur = -1;
  VBDR_HIP(hipGetDevice(&cur));
  if (cur != bt->device) return vbdr_fail(VBDR_EINVAL, "batch lives on device %d", bt->device);
  const uint32_t S = bt->S;
  uint64_t scan_total = 0, adv_total = 0, est_total = 0;
  for (uint32_t s = 0; s < S; ++s) {
    if (n_pairs[s] && (!pairs_dev[s] || (reinterpret_cast<uintptr_t>(pairs_dev[s]) & 7u)))
      return vbdr_fail(VBDR_EINVAL, "sketch %u: pairs must be non-NULL and 8-byte aligned", s);
    if (n_hosts[s] && (!hosts_dev[s] || !out_dev[s])) return vbdr_fail(VBDR_EINVAL, "sketch %u: NULL hosts or out", s);
    scan_total += (n_pairs[s] + bt->tune.scan_tile - 1) / bt->tune.scan_tile;
    adv_total += bt->sk[s]->mstride / kAdvTile;
    est_total += (n_hosts[s] + bt->tune.est_tile - 1) / bt->tune.est_tile;
  }
  if (scan_total >= (1ull << 31) || adv_total >= (1ull << 31) || est_total >= (1ull << 31))
    return vbdr_fail(VBDR_EINVAL, "too many work items in one step");
  // fill a pinned staging table (wait until its previous upload has run)
  const int buf = bt->next;
  bt->next ^= 1;
  VBDR_HIP(hipEventSynchronize(bt->staged[buf]));
  BatchDesc* desc = reinterpret_cast<BatchDesc*>(bt->staging[buf]);
  BatchHdr* hdr = reinterpret_cast<BatchHdr*>(bt->staging[buf] + sizeof(BatchDesc) * S);
  DeferItem* ditems = defer_items(bt->staging[buf], S);
  DeferHdr* dhdr = defer_hdr(bt->staging[buf], S, bt->n_defer);
  const uint32_t chunk = vbdr_defer_chunk_pairs();
  uint32_t si = 0, ai = 0, ei = 0, dsi = 0, dai = 0;
  for (uint32_t s = 0; s < S; ++s) {
    const vbdr_sketch* k = bt->sk[s];
    const uint32_t di = bt->defer_of[s];
    if (di != ~0u) {  // scanned and advanced by the deferred kernels: no items in the direct ones
      DeferItem& I = ditems[di];
      vbdr_defer_member(k, &I);
      I.pairs = pairs_dev[s], I.n_pairs = n_pairs[s];
      I.scan_item0 = dsi, I.adv_item0 = dai;
      dsi += (uint32_t)((n_pairs[s] + chunk - 1) / chunk);
      dai += k->def_tiles;
    }
    BatchDesc& D = desc[s];
    D.dr = k->dr, D.seen = k->seen, D.reg = k->reg, D.reg4 = k->reg4, D.hist = k->hist, D.s1 = k->s1;
    D.mstride = k->mstride, D.wstride = k->wstride;
    D.m = (uint32_t)k->m, D.g = k->g, D.b = k->b, D.L = k->L, D.k = k->k, D.layout = (uint32_t)k->layout;
    D.A1 = k->A1, D.test = k->tune.scan_test_first == 1;
    D.pairs = pairs_dev[s], D.n_pairs = n_pairs[s];
    D.hosts = hosts_dev[s], D.n_hosts = n_hosts[s], D.out = out_dev[s];
    D.scan_item0 = si, D.adv_item0 = ai, D.est_item0 = ei, D.pad = 0;
    // members with a learned estimator are estimated after the step's kernels
    const uint64_t n_plain = bt->mlp[s] ? 0 : n_hosts[s];
    if (di == ~0u) {
      si += (uint32_t)((n_pairs[s] + bt->tune.scan_tile - 1) / bt->tune.scan_tile);
      ai += (uint32_t)(k->mstride / kAdvTile);
    }
    ei += (uint32_t)((n_plain + bt->tune.est_tile - 1) / bt->tune.est_tile);
  }
  std::memset(hdr, 0, sizeof(*hdr));
  hdr->scan_total = si, hdr->adv_total = ai, hdr->est_total = ei;
  std::memset(dhdr, 0, sizeof(*dhdr));
  dhdr->scan_total = dsi;
  // order after the caller's stream, run on the batch stream, order the caller after it
  hipStream_t user = reinterpret_cast<hipStream_t>(stream);
  VBDR_HIP(hipEventRecord(bt->ev_in, user));
  VBDR_HIP(hipStreamWaitEvent(bt->st, bt->ev_in, 0));
  VBDR_HIP(hipMemcpyAsync(bt->desc_dev, bt->staging[buf], table_bytes(S, bt->n_defer), hipMemcpyHostToDevice, bt->st));
  VBDR_HIP(hipEventRecord(bt->staged[buf], bt->st));
  if (bt->tune.use_graph) {
    if (!bt->exec) {
      VBDR_HIP(hipStreamBeginCapture(bt->st, hipStreamCaptureModeThreadLocal));
      const int rc = launch_step_kernels(bt);
      hipGraph_t g = nullptr;
      const hipError_t e = hipStreamEndCapture(bt->st, &g);
      if (rc != VBDR_OK) return rc;
      if (e != hipSuccess) return vbdr_fail(VBDR_EHIP, "graph capture failed: %s", hipGetErrorString(e));
      bt->graph = g;
      VBDR_HIP(hipGraphInstantiate(&bt->exec, bt->graph, nullptr, nullptr, 0));
    }
    VBDR_HIP(hipGraphLaunch(bt->exec, bt->st));
  } else if (int rc = launch_step_kernels(bt)) {
    return rc;
  }
  for (uint32_t s = 0; s < S; ++s)
    if (bt->mlp[s] && n_hosts[s])
      if (int rc = vbdr_estimate_learned(bt->sk[s], bt->mlp[s], hosts_dev[s], n_hosts[s], out_dev[s], nullptr, bt->st))
        return rc;
  VBDR_HIP(hipEventRecord(bt->ev_out, bt->st));
  VBDR_HIP(hipStreamWaitEvent(user, bt->ev_out, 0));
  for (vbdr_sketch* k : bt->sk) k->t++;
  return VBDR_OK;
}

}  // extern "C"
