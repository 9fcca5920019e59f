/*
 * vbdr.h -- C ABI of libvbdr.so, the gfx950 (MI355X) implementation of the
 * VBDR sliding-window host-cardinality estimator of J. Xu, "Cardinalities
 * estimation under sliding time window by sharing HyperLogLog Counter"
 * (arXiv:1810.13132).
 *
 * Model.  Traffic arrives as (aip, bip) IP pairs in time slices (Sec. 2.1,
 * Sec. 2.3).  A sketch holds a pool BDRP of m bit distance recorders (BDRs,
 * Sec. 3); every host aip owns a virtual vector of g = 2^b of them chosen by
 * getPhyIdx (Alg. 3).  Each BDR keeps one distance recorder (DR) per LBP1
 * value r = 1..L, L = 33 - b: the number of slices since r was last recorded
 * there, one byte, saturating at 255 (Sec. 3, DR operations).  The window
 * W(t, k) is the k most recently closed slices.
 *
 * Calling sequence per slice:  vbdr_scan_slice()*  ->  vbdr_advance_slice()
 * ->  vbdr_estimate().  Scans of one slice may be split over any number of
 * calls; their result does not depend on pair order or on repeated pairs.
 *
 * Three layouts (Sec. 4.2, Table 1):
 *   VBDR_LAYOUT_FAST  -- the scan records each pair's LBP1 as one bit of a
 *                        per-slice bit string (bsLBP1, Alg. 7) with an
 *                        atomic OR; the advance folds the highest bit into
 *                        the DRs (Alg. 6).  More memory, fastest scan.
 *   VBDR_LAYOUT_SMALL -- the scan zeroes the DR of the pair's LBP1 directly
 *                        (Alg. 9, a plain byte store); the advance slides
 *                        every DR (Alg. 8).
 *   VBDR_LAYOUT_PACKED -- the small layout with Table 1's recorder sizes:
 *                        z = ceil(log2(k+1))-bit DRs (bit-sliced, saturating
 *                        at 2^z - 1 >= k) and Lc recorders per BDR, LBP1
 *                        values above Lc recorded at Lc, so its registers
 *                        are min(register, Lc).  Least memory.  Pools of at
 *                        most 2^26 BDRs; scans always go through records.
 * The fast and small layouts give identical registers and estimates; the
 * packed layout gives identical ones when Lc = L = 33 - b.
 *
 * Hashing (the paper leaves H(x, N, A) open): H(x, N, A) is
 * MurmurHash3_x86_32 of the 4-byte little-endian x with seed A, mapped to
 * [0, N) as (h * N) >> 32.  A0 and A1 are the low and high 32-bit halves of
 * the first SplitMix64 output from state hash_seed.
 *
 * Memory and streams.  A sketch owns its device memory (allocated in
 * vbdr_sketch_create on the device current at that time).  Every other
 * device pointer belongs to the caller and must stay valid until the work
 * enqueued on `stream` finishes.  `stream` is a hipStream_t (NULL = the
 * default stream); all device work of a call is enqueued on it without any
 * host synchronisation, except where a function says "synchronous".  The
 * calls of one sketch must be made from the device it was created on, and a
 * sketch is not thread-safe.  scan_slice, advance_slice and the estimate
 * calls allocate no memory.
 *
 * Errors.  Every int-returning function returns VBDR_OK (0) or a negative
 * vbdr_status; vbdr_last_error() then describes the last failure of the
 * calling thread.  On error no device work has been enqueued unless the
 * status is VBDR_EHIP (a HIP call failed; the sketch may be unusable).
 */
#ifndef VBDR_H
#define VBDR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define VBDR_NBINS 33 /* register values 0..32 */

typedef struct vbdr_sketch vbdr_sketch;

enum vbdr_layout { VBDR_LAYOUT_FAST = 0, VBDR_LAYOUT_SMALL = 1, VBDR_LAYOUT_PACKED = 2 };

enum vbdr_status {
    VBDR_OK = 0,
    VBDR_EINVAL = -1, /* bad argument (range, NULL, alignment, wrong device) */
    VBDR_ENOMEM = -2, /* a device allocation failed (create, enable_pcsa, set_tuning) */
    VBDR_EHIP = -3,   /* a HIP runtime call or kernel launch failed */
    VBDR_ESTATE = -4  /* call not valid in the sketch's current state */
};

typedef struct vbdr_info {
    uint64_t m;           /* BDRs in the pool */
    uint32_t g, b, L, k;  /* g = 2^b recorders per host, L = 33 - b, window k */
    int32_t layout;       /* enum vbdr_layout */
    uint32_t A0, A1;      /* hash seeds derived from hash_seed */
    uint64_t t;           /* slices closed so far */
    uint64_t state_bytes; /* device bytes held by the sketch: window_state_bytes + workspace_bytes */
    int32_t est_parts;    /* pool ranges of the estimate's XCD-partitioned gathers (1 = direct) */
    int32_t scan_deferred; /* 1 when scans defer their updates to the advance (scan_defer = 1) */
    uint32_t Lc;          /* recorders per BDR (L except for the packed layout) */
    uint32_t dr_bits;     /* bits per DR: 8, or z for the packed layout */
    int32_t est_tiled;    /* 1 when plain estimates take the LDS-tiled path (est_binned = 3, eligible pool) */
    uint64_t window_state_bytes; /* the window's state: DRs (byte planes or packed bit-planes), bsLBP1
                                    bit-planes, registers (bytes and nibbles), saturation masks, pool
                                    histogram, seeds, PCSA runs (Sec. 4.2 Table 1 counts the DRs) */
    uint64_t workspace_bytes;    /* scratch of the hot path: deferred scan records, estimate workspaces */
} vbdr_info;

/*
 * Create a sketch: pool of m BDRs (BDRP, Sec. 4.1), g = 2^b recorders per
 * host (power of two, 2 <= g <= 65536), g < m < 2^32, window of 1 <= k <= 254
 * slices, hash seed as above.  Slice 0 is open; every DR holds its initial
 * value 255 (InitDR), every register is 0.  vbdr_sketch_create uses the fast
 * layout.  *out receives the handle (owned by the caller; free with
 * vbdr_sketch_destroy).  Synchronous.
 */
int vbdr_sketch_create(uint64_t m, uint32_t g, uint32_t k, uint64_t hash_seed, vbdr_sketch **out);
int vbdr_sketch_create_layout(uint64_t m, uint32_t g, uint32_t k, uint64_t hash_seed, int layout,
                              vbdr_sketch **out);
/* The packed layout with Lc recorders per BDR (1 <= Lc <= 33 - b), m <= 2^26. */
int vbdr_sketch_create_packed(uint64_t m, uint32_t g, uint32_t k, uint64_t hash_seed, uint32_t Lc,
                              vbdr_sketch **out);

/* Free a sketch and its device memory after synchronising the device.  NULL is a no-op. */
void vbdr_sketch_destroy(vbdr_sketch *sk);

/*
 * Scan n pairs into the open slice (Alg. 7 for the fast layout, Alg. 9 for
 * the small one, with the pair hashing of Alg. 4 and getPhyIdx of Alg. 3).
 * pairs_dev: device array of 2n uint32, interleaved aip0, bip0, aip1, bip1,
 * ..., 8-byte aligned; read only.  n = 0 is a no-op (pairs_dev may be NULL).
 */
int vbdr_scan_slice(vbdr_sketch *sk, const uint32_t *pairs_dev, uint64_t n, void *stream);

/*
 * Close the open slice and open the next (Alg. 6 or Alg. 8 over every BDR),
 * then derive each BDR's register for the window of the k most recently
 * closed slices (Alg. 2) and the pool's register histogram.
 */
int vbdr_advance_slice(vbdr_sketch *sk, void *stream);

/*
 * Estimate |OP(aip, t, k)| (Definition 1) over the window of the k most
 * recently closed slices for n_hosts hosts: each host's g registers
 * (Alg. 5, taken as a histogram) give the HyperLogLog estimate E_s of its
 * virtual vector, E_m is the same estimate over the whole pool, and the
 * sharing noise is removed as (m E_s - g E_m) / (m - g), clamped at 0.
 * Computed in FP64, stored as FP32 (round to nearest).  Before the first
 * advance every estimate is 0.
 * hosts_dev: device array of n_hosts uint32 addresses; out_dev: device
 * array of n_hosts float.  n_hosts = 0 is a no-op.  The estimate's
 * workspaces belong to the sketch: two estimates of one sketch must not run
 * concurrently (order them on one stream or with events); an estimate may
 * run beside the next slice's scan, which touches none of its buffers.
 */
int vbdr_estimate(vbdr_sketch *sk, const uint32_t *hosts_dev, uint64_t n_hosts, float *out_dev, void *stream);

/*
 * vbdr_estimate plus optional per-host outputs: raw_es_dev (n_hosts double,
 * the un-corrected E_s) and hist_dev (n_hosts x 33 uint32, the histogram of
 * the host's g register values).  Either may be NULL.
 */
int vbdr_estimate_ex(vbdr_sketch *sk, const uint32_t *hosts_dev, uint64_t n_hosts, float *out_dev,
                     double *raw_es_dev, uint32_t *hist_dev, void *stream);

/*
 * vbdr_estimate for callers that cannot allocate device memory or touch the
 * sketch's estimate workspaces: code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc.  Same arguments and the same
 * results as vbdr_estimate, bit for bit.  Pools of 2^22 BDRs and more take
 * the XCD-partitioned estimate with its per-range partial sums in a static
 * device array of the library (6 MiB; each device the library runs on holds
 * its own until the process ends), 65536 hosts per pass; smaller pools take
 * the direct estimate, which needs no scratch memory.  The array's device
 * address is looked up on the first call on each device; no call allocates.
 * Every call on one device shares that device's array: two calls that
 * overlap in time on one device (any sketches, any streams) race and give
 * wrong results, so order them.  Nothing needs clearing between calls
 * (every partial sum a pass reads is written by that pass).  n_hosts < 2^40.
 */
int vbdr_estimate_noalloc(vbdr_sketch *sk, const uint32_t *hosts_dev, uint64_t n_hosts, float *out_dev,
                          void *stream);

/*
 * Other estimators on the same pool: the text after Alg. 5 (Sec. 4.1) and
 * Sec. 5 name PCSA and LogLog as users of the recorder pool.
 *   VBDR_EST_HLL     the HyperLogLog estimate of vbdr_estimate;
 *   VBDR_EST_LOGLOG  LogLog (Durand and Flajolet 2003) over the same
 *                    registers: E_s = alpha_g g 2^(S/g), S the host's
 *                    literal sum of Alg. 5, alpha_q = (Gamma(-1/q)
 *                    (1 - 2^(1/q)) / ln 2)^-q;
 *   VBDR_EST_PCSA    PCSA (Flajolet and Martin 1985): a recorder vector read
 *                    as the bitmap of the LBP1 values active in the window,
 *                    R = the number of consecutive active DRs from LBP1 1,
 *                    E_s = g / 0.77351 2^(S/g) with S the host's sum of R.
 *                    Small layout only (it records every LBP1 of a slice);
 *                    the runs are kept from the advance after
 *                    vbdr_enable_pcsa(sk, 1) on, at m more bytes of state.
 * E_m is the same estimator over the pool; the sharing noise is removed
 * with (m E_s - g E_m)/(m - g), clamped at 0, FP64 then FP32, as for
 * HyperLogLog.  raw_es_dev (n_hosts double, nullable) receives E_s.
 * vbdr_estimate_kind reads the pool's sums on the host (it synchronises
 * with `stream`).  VBDR_ESTATE for PCSA before runs exist.
 * vbdr_export_pcsa copies the m PCSA runs of the last closed window to host
 * memory (synchronous).  vbdr_enable_pcsa(sk, 0) frees the runs.
 */
enum vbdr_estimator { VBDR_EST_HLL = 0, VBDR_EST_LOGLOG = 1, VBDR_EST_PCSA = 2 };
int vbdr_enable_pcsa(vbdr_sketch *sk, int on);
int vbdr_estimate_kind(vbdr_sketch *sk, const uint32_t *hosts_dev, uint64_t n_hosts, int kind, float *out_dev,
                       double *raw_es_dev, void *stream);
int vbdr_export_pcsa(vbdr_sketch *sk, uint8_t *preg_host, void *stream);

/*
 * Super-point (superspreader) detection over the sliding window, the use the
 * paper motivates for per-host cardinalities (Sec. 1, Sec. 2.3): the hosts
 * whose estimate is at least `threshold`.  est_dev and hosts_dev are device
 * arrays of n entries (the output and input of an estimate call), n < 2^32.
 * The selected hosts and their estimates go to out_hosts_dev and out_est_dev
 * (device arrays of cap entries) in unspecified order; *count_dev (one device
 * uint32) receives the number of hosts selected, which may exceed cap: then
 * only cap of them are written.  Stream-ordered, no synchronisation.  NaN
 * estimates are never selected.
 */
int vbdr_select_hosts(const float *est_dev, const uint32_t *hosts_dev, uint64_t n, float threshold,
                      uint32_t *out_hosts_dev, float *out_est_dev, uint64_t cap, uint32_t *count_dev, void *stream);

/*
 * Per-slice max-LBP1 map, for data parallelism over one slice's pairs (fast
 * layout).  The fast layout keeps of a slice only the highest LBP1 seen per
 * BDR (Alg. 6), i.e. the serial layout's nowLBP1 (Alg. 1, Alg. 4).  Sketches
 * with identical state (replicas) that scan disjoint shares of a slice can
 * therefore export their maps, combine them with an element-wise MAX (on
 * several GPUs: an all-reduce of m bytes), import the combined map, and
 * advance: every replica then holds the state one sketch would after
 * scanning all the pairs.
 *   vbdr_export_now: now_dev[p] (m bytes, device) = highest LBP1 of the open
 *     slice at BDR p, 0 if none.  The open slice is unchanged.
 *   vbdr_import_now: the open slice's LBP1 record becomes exactly now_dev
 *     (entries 0..L); earlier scans of the slice are replaced.
 *   vbdr_now_max: out_dev[i] = max(a_dev[i], b_dev[i]) for n bytes (out may
 *     alias a or b); the reduction operator of the exchange.
 * VBDR_EINVAL for a small-layout sketch (it records every LBP1 of a slice,
 * which a MAX does not combine).  Stream-ordered.
 */
int vbdr_export_now(vbdr_sketch *sk, uint8_t *now_dev, void *stream);
int vbdr_import_now(vbdr_sketch *sk, const uint8_t *now_dev, void *stream);
int vbdr_now_max(const uint8_t *a_dev, const uint8_t *b_dev, uint8_t *out_dev, uint64_t n, void *stream);

/* Parameters and slice counter of a sketch.  Host only, no device work. */
int vbdr_sketch_info(const vbdr_sketch *sk, vbdr_info *out);

/*
 * Launch shape and kernel variant of a sketch's hot-path calls.  None of
 * these changes any result, only speed.  Zero fields mean "default".
 *   scan_test_first    1: the scan reads the bit or DR first and skips the
 *                      update when it is already made; 2: always update
 *                      (default: the variant measured faster for the layout);
 *   scan_blocks_per_cu workgroups per compute unit of the scan (1..64);
 *   est_blocks_per_cu  workgroups per compute unit of the estimate (1..64);
 *   scan_binned        1: pools of 2^22..2^27 BDRs scan in two passes, the
 *                      pairs first binned by pool range so that each XCD
 *                      updates only its own range; 2: always scan directly
 *                      (default: 2);
 *   est_binned         for pools of 2^22 BDRs and more: 1 = hash every
 *                      (host, i) once and bin the gathers by XCD range;
 *                      2 = hash on every XCD and gather only the own range;
 *                      3 = hash every (host, i) once into runs per tile of
 *                      at most 2^18 registers, gather every register from a
 *                      tile held in LDS, add per-tile sums (pools of at most
 *                      2^26 BDRs, 64 <= g <= 8192; elsewhere 3 acts as 2)
 *                      (default: 3 for pools of 2^24 BDRs and more, else 2);
 *   est_parts          pool ranges of the XCD-partitioned estimate, 8 (one
 *                      per XCD, default) or 4 (two XCDs per range: half the
 *                      hashing, twice the cache footprint per XCD);
 *   est_bin_hosts      hosts per pass of the binned estimate (its gather
 *                      runs take about 4*g bytes per host; default: as many
 *                      as the run buffer holds); for the tiled estimate,
 *                      hosts per block, rounded down to a multiple of 2048
 *                      (at least 2048, at most the default min(2^29/g, 2^19)),
 *                      and its workspace is sized for that block (about
 *                      4.3 g + 4 nt bytes per host of the block; this call
 *                      reallocates it): a memory budget, at some speed;
 *   est_bin_cap        slots per run of the binned (per host and range) or
 *                      tiled (per 2048 hosts and tile) estimate, at most the
 *                      default; entries beyond it are gathered directly by
 *                      the first pass;
 *   scan_defer         for pools of 2^22..2^27 BDRs: 1 = the scan only
 *                      writes each pair's (pidx, LBP1) record, sorted by
 *                      tile of 2^15 BDRs, and the advance applies the records
 *                      from LDS while it streams the tile (default); 2 = the
 *                      scan updates the pool itself (direct or binned).
 *                      Up to 2 records per BDR per slice are deferred; the
 *                      rest are applied by the scan.  The sketch state seen
 *                      through vbdr_export_state is the same either way.
 */
typedef struct vbdr_tuning {
    int32_t scan_test_first;
    uint32_t scan_blocks_per_cu;
    uint32_t est_blocks_per_cu;
    int32_t scan_binned;
    int32_t est_binned;
    int32_t est_parts;
    uint32_t est_bin_hosts;
    uint32_t est_bin_cap;
    int32_t scan_defer;
} vbdr_tuning;
int vbdr_sketch_set_tuning(vbdr_sketch *sk, const vbdr_tuning *tuning);
int vbdr_sketch_get_tuning(const vbdr_sketch *sk, vbdr_tuning *tuning);

/*
 * Copy the sketch state to host memory in canonical form (synchronous:
 * waits for `stream`).  Any pointer may be NULL.
 *   dr_host   m*L bytes, dr_host[p*L + (r-1)] = DR of LBP1 r in BDR p;
 *   bs_host   m uint32, the open slice's bsLBP1 of BDR p, bit r-1 <-> r
 *             (all zero for the small layout);
 *   reg_host  m bytes, register of BDR p for the last closed window;
 *   hist_host 33 uint64, histogram of reg over the pool.
 * Packed layout: DR values are 0..2^z - 1 and recorders above Lc read
 * 2^z - 1 (they are never set).
 */
int vbdr_export_state(vbdr_sketch *sk, uint8_t *dr_host, uint32_t *bs_host, uint8_t *reg_host,
                      uint64_t *hist_host, void *stream);

/*
 * Load a canonical state (same layout as vbdr_export_state; dr_host, reg_host
 * and hist_host required, bs_host may be NULL = all zero) and the slice
 * counter t into a sketch with the same parameters, for checkpoint/resume.
 * Packed layout: DR values are capped at 2^z - 1 (every value >= k is
 * inactive alike) and recorders above Lc are ignored.  Synchronous.
 * VBDR_EINVAL when a register exceeds the recorders, when hist_host does
 * not sum to m or is not the histogram of reg_host, or when bs_host has
 * bits a small-layout sketch cannot hold.
 */
int vbdr_import_state(vbdr_sketch *sk, const uint8_t *dr_host, const uint32_t *bs_host, const uint8_t *reg_host,
                      const uint64_t *hist_host, uint64_t t, void *stream);

/* Message of the calling thread's last error ("" if none).  Valid until the next call. */
const char *vbdr_last_error(void);

/*
 * Testing aid for the out-of-memory paths: the library's device allocation
 * that comes after `after` more successful ones fails as if the device were
 * full, so the call that needed it returns VBDR_ENOMEM; after < 0 cancels.
 * Process-wide (one counter for every thread and device).  Returns VBDR_OK.
 */
int vbdr_test_fail_alloc(int64_t after);

/* ------------------------------------------------------------------------
 * Learned estimator (an addition beside the paper's estimate, not from it).
 *
 * Features of a host (VBDR_MLP_IN = 67, float):
 *   [0..32]  hist[r] / g, the host's register histogram (the per-register
 *            values Alg. 5 sums, taken as a histogram);
 *   [33..65] pool_hist[r] / m, the pool's register histogram;
 *   [66]     ln(g / m).
 * Network: 67 -> 64 -> 64 -> 1 with GELU (exact erf form), output y
 * estimating ln(1 + n), so n_hat = exp(y) - 1 clamped at 0.
 * Parameters (VBDR_MLP_PARAMS = 8577 float, in this order):
 *   W1 [64][67] row-major, b1 [64], W2 [64][64], b2 [64], w3 [64], b3 [1].
 * Inference rounds the inputs, W1, W2, w3 and the first hidden layer to
 * bfloat16 (round to nearest even) and accumulates in float32 on the matrix
 * cores; the learned estimate is replaced by the plain vbdr_estimate value
 * for hosts whose features leave the envelope [env_lo, env_hi] or whose
 * output is not finite.
 * ---------------------------------------------------------------------- */
#define VBDR_MLP_IN 67
#define VBDR_MLP_PARAMS 8577

typedef struct vbdr_mlp vbdr_mlp;
typedef struct vbdr_trainer vbdr_trainer;

/* Upload a network (params_host: VBDR_MLP_PARAMS floats, host memory, copied).
 * env_lo / env_hi: VBDR_MLP_IN floats each, or both NULL for no envelope.
 * The network lives on the current device.  Synchronous. */
int vbdr_mlp_create(const float *params_host, const float *env_lo, const float *env_hi, vbdr_mlp **out);
void vbdr_mlp_destroy(vbdr_mlp *mlp); /* NULL-safe; synchronises the device */

/* Where the plain estimate (Alg. 5 with the noise removed) is at least
 * `threshold`, vbdr_estimate_learned keeps it and flags the host 2: for
 * counts large enough that sharing noise no longer dominates the plain
 * estimate, which a network trained on log counts does not match.
 * threshold > 0; INFINITY (the default) turns the rule off.  The network
 * must be on the current device; VBDR_EINVAL otherwise.  Synchronous. */
int vbdr_mlp_set_plain_above(vbdr_mlp *mlp, float threshold);

/* Features (n_hosts x 67 float, row-major, device) of the given hosts for the
 * last closed window, from the same register gathers as vbdr_estimate. */
int vbdr_features(vbdr_sketch *sk, const uint32_t *hosts_dev, uint64_t n_hosts, float *feats_dev, void *stream);

/* Learned estimate of n_hosts hosts into out_dev (float); used_fallback_dev
 * (n_hosts bytes, nullable) receives 1 where the plain estimate was used
 * because a feature left the training envelope (or the output was not
 * finite), 2 where it was kept as a large count (vbdr_mlp_set_plain_above),
 * else 0. */
int vbdr_estimate_learned(vbdr_sketch *sk, const vbdr_mlp *mlp, const uint32_t *hosts_dev, uint64_t n_hosts,
                          float *out_dev, uint8_t *used_fallback_dev, void *stream);

/* Float32 training state (parameters, Adam moments, gradient buffer) on the
 * current device, initialised from params_host; Adam with beta1 0.9, beta2
 * 0.999, eps 1e-8 and learning rate lr. */
int vbdr_trainer_create(const float *params_host, float lr, vbdr_trainer **out);
void vbdr_trainer_destroy(vbdr_trainer *tr); /* NULL-safe; synchronises the device */
int vbdr_trainer_set_lr(vbdr_trainer *tr, float lr);

/* One Adam step on the mean squared error of y against targets over a batch:
 * feats_dev (n x 67 float), targets_dev (n float, ln(1 + n) of each sample).
 * loss_dev (nullable, 1 float) has the batch loss ADDED to it. */
int vbdr_trainer_step(vbdr_trainer *tr, const float *feats_dev, const float *targets_dev, uint64_t n, float *loss_dev,
                      void *stream);

/* The batch-mean-loss gradient at the current parameters, ADDED into
 * grads_out_dev (VBDR_MLP_PARAMS float, device); no update. */
int vbdr_trainer_grad(vbdr_trainer *tr, const float *feats_dev, const float *targets_dev, uint64_t n,
                      float *grads_out_dev, float *loss_dev, void *stream);

/* Copy the float32 parameters to host memory (synchronous on stream). */
int vbdr_trainer_params(vbdr_trainer *tr, float *params_host, void *stream);

/* ------------------------------------------------------------------------
 * Batches: many independent sketches (e.g. one per edge router), each with
 * its own pool size, g, k, seed and layout, stepped together.  One step =
 * for every sketch, scan its slice, close it, estimate its host list --
 * vbdr_scan_slice + vbdr_advance_slice + vbdr_estimate semantics per sketch,
 * run as three persistent work-queue kernels over all sketches, captured once
 * into a HIP graph and replayed.  At most 256 sketches per batch.
 * ---------------------------------------------------------------------- */
typedef struct vbdr_batch vbdr_batch;

typedef struct vbdr_batch_params {
    uint64_t m;
    uint32_t g, k;
    uint64_t hash_seed;
    int32_t layout;
} vbdr_batch_params;

/* Launch shape of a batch step (no effect on results):
 *   scan_tile      pairs per scan work item (256 .. 2^22);
 *   est_tile       hosts per estimate work item (4 .. 2^16);
 *   blocks_per_cu  workgroups per compute unit of each persistent kernel (1..32);
 *   use_graph      1 = capture the kernel sequence once and replay it. */
typedef struct vbdr_batch_tuning {
    uint32_t scan_tile;
    uint32_t est_tile;
    uint32_t blocks_per_cu;
    int32_t use_graph;
} vbdr_batch_tuning;

/* Create n_sketches (1..256) sketches described by params[n_sketches] on the
 * current device.  Synchronous. */
int vbdr_batch_create(uint32_t n_sketches, const vbdr_batch_params *params, vbdr_batch **out);
void vbdr_batch_destroy(vbdr_batch *bt); /* NULL-safe; also frees its sketches */

/* Borrowed handle of sketch i (for export, estimate_ex, learned estimates);
 * owned by the batch.  NULL (and vbdr_last_error set) if i is out of range. */
vbdr_sketch *vbdr_batch_sketch(vbdr_batch *bt, uint32_t i);

/* Learned estimates for member i from the next step on (vbdr_estimate_learned
 * semantics: the plain estimate where features leave the model's envelope);
 * mlp = NULL returns the member to plain estimates.  The model stays the
 * caller's and must outlive the steps that use it; it must live on the
 * batch's device.  The member's learned estimate runs after the step's
 * persistent kernels, on the batch's stream.  Waits for steps in flight. */
int vbdr_batch_set_mlp(vbdr_batch *bt, uint32_t i, const vbdr_mlp *mlp);

int vbdr_batch_set_tuning(vbdr_batch *bt, const vbdr_batch_tuning *tuning);
int vbdr_batch_get_tuning(const vbdr_batch *bt, vbdr_batch_tuning *tuning);

/* One step.  Host arrays of n_sketches entries: pairs_dev[i] (2*n_pairs[i]
 * uint32, device, 8-byte aligned), hosts_dev[i] (n_hosts[i] uint32, device)
 * and out_dev[i] (n_hosts[i] float, device).  Work is ordered after earlier
 * work on `stream`, and later work on `stream` is ordered after it; it runs
 * on a stream the batch owns.  The host arrays may be reused on return. */
int vbdr_batch_step(vbdr_batch *bt, const uint32_t *const *pairs_dev, const uint64_t *n_pairs,
                    const uint32_t *const *hosts_dev, const uint64_t *n_hosts, float *const *out_dev, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* VBDR_H */
