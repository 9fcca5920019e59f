/*
 * vbdr_oracle.c -- TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT PATH.
 *
 * A plain, slow, single-threaded CPU reference of the VBDR method of
 * J. Xu, "Cardinalities estimation under sliding time window by sharing
 * HyperLogLog Counter" (arXiv:1810.13132).  Only the test suite, the smoke
 * check and the CPU-baseline leg of the benchmark may load this library.
 * It shares no code, header or table with the HIP library.
 *
 * Every routine computes what the paper defines, written for clarity rather
 * than speed: the pool index of a virtual recorder is rehashed on every
 * call, a register is found by looking at every recorder of its BDR, and
 * the scan records one pair at a time.  Integer state is exact; estimates
 * are FP64.
 *
 * Readings of the paper taken here (the paper is silent or garbled):
 *  - The pool size is called m (the paper reuses the letter z for it and for
 *    the recorder width).  A distance recorder (DR) is one byte, z = 8, so
 *    InitDR stores 255 and SlideDR saturates at 255 (Sec. 3 defines SlideDR
 *    with a bound that would let a z-bit counter wrap; saturation is the only
 *    reading under which an old LBP1 never turns active again).
 *  - The recorder vector covers every LBP1 value the hash can produce,
 *    L = 33 - b values (1..L), instead of ceil(log2(n/g)) values; no clamp.
 *  - LBP1 of an all-zero (32-b)-bit suffix is (32-b)+1, the HyperLogLog
 *    convention.
 *  - H(x, N, A) is MurmurHash3_x86_32 of the 4-byte little-endian x with
 *    seed A, reduced to [0, N) by the multiply-shift map (h * N) >> 32; for
 *    N = 2^32 this is the hash itself.  The bip hash uses seed A1 and the
 *    virtual-index seeds use A0 (Alg. 3, Alg. 4).  A0 and A1 are the low and
 *    high halves of one SplitMix64 output drawn from the user's hash seed.
 *  - Serial layout: nowLBP1 is cleared after each end-of-slice update.
 *  - Fast GPU layout (Alg. 6): the slice's LBP1 is the highest set bit of
 *    bsLBP1 (bit r-1 records LBP1 = r), and an empty slice sets no DR.
 *  - Small GPU layout (Alg. 8/9): the close of slice t and the beginning of
 *    slice t+1 are the same moment; the registers of the closed window are
 *    read (Alg. 2, dr < k) and then every DR slides for the next slice.
 *  - Estimation (Alg. 5 and the HyperLogLog estimator it points to): the
 *    register histogram of a host's g recorders gives the harmonic sum; the
 *    HyperLogLog constants alpha_q and its small-range (linear counting)
 *    correction apply; the noise of pool sharing is removed with
 *    n = (m*E_s - g*E_m)/(m - g), E_m being the same estimator over the whole
 *    pool.  The result is clamped at 0 and rounded to FP32.
 *  - Other estimators on the same pool (the text after Alg. 5 in Sec. 4.1,
 *    and Sec. 5, name PCSA and LogLog as users of the pool): LogLog
 *    (Durand and Flajolet 2003) takes
 *    the same registers, E = alpha_q q 2^(S/q) with S the literal sum of
 *    Alg. 5 and alpha_q = (Gamma(-1/q) (1 - 2^(1/q)) / ln 2)^-q; PCSA
 *    (Flajolet and Martin 1985) reads each recorder vector as the bitmap of
 *    the LBP1 values seen in the window (a DR per bit: only the small layout
 *    records every LBP1 of a slice), R = the number of consecutive active
 *    DRs from LBP1 1, E = (q / 0.77351) 2^(S/q) with S the sum of R.  Both
 *    remove the sharing noise with the same (m*E_s - g*E_m)/(m - g).
 *  - Packed layout (Table 1's gsmall: log2(n/g) DRs of log2(k+1) bits): the
 *    small layout with z = ceil(log2(k+1))-bit DRs, InitDR and saturation at
 *    2^z - 1 (>= k, so a DR that left the window stays inactive), and Lc
 *    recorders per BDR with LBP1 values above Lc recorded at Lc, so that a
 *    register is min(register, Lc) of the full layout.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define VBDRO_SERIAL 0
#define VBDRO_GFAST 1
#define VBDRO_GSMALL 2
#define VBDRO_GPACKED 3 /* small layout with z-bit DRs and Lc recorders (Table 1's gsmall) */

#define DR_BITS 8u
#define DR_INIT 255u /* InitDR: 2^z - 1 with z = 8 */
#define NBINS 33u    /* register values 0..32 */

/* ------------------------------------------------------------------ */
/* Hash primitives                                                     */
/* ------------------------------------------------------------------ */

static uint32_t rotl32(uint32_t x, int r) { return (x << r) | (x >> (32 - r)); }

/* MurmurHash3_x86_32 (A. Appleby, public domain), written from its
 * published description: 4-byte blocks mixed with two odd constants and
 * rotations, a tail block, the length, then the final avalanche. */
uint32_t vbdro_murmur3_32(const uint8_t *data, uint64_t len, uint32_t seed)
{
    const uint32_t c1 = 0xcc9e2d51u, c2 = 0x1b873593u;
    uint32_t h = seed;
    uint64_t nblocks = len / 4;
    for (uint64_t i = 0; i < nblocks; i++) {
        uint32_t k = (uint32_t)data[4 * i] | ((uint32_t)data[4 * i + 1] << 8) |
                     ((uint32_t)data[4 * i + 2] << 16) | ((uint32_t)data[4 * i + 3] << 24);
        k *= c1;
        k = rotl32(k, 15);
        k *= c2;
        h ^= k;
        h = rotl32(h, 13);
        h = h * 5u + 0xe6546b64u;
    }
    const uint8_t *tail = data + 4 * nblocks;
    uint32_t k1 = 0;
    switch (len & 3) {
    case 3:
        k1 ^= (uint32_t)tail[2] << 16; /* fall through */
    case 2:
        k1 ^= (uint32_t)tail[1] << 8; /* fall through */
    case 1:
        k1 ^= (uint32_t)tail[0];
        k1 *= c1;
        k1 = rotl32(k1, 15);
        k1 *= c2;
        h ^= k1;
    }
    h ^= (uint32_t)len;
    h ^= h >> 16;
    h *= 0x85ebca6bu;
    h ^= h >> 13;
    h *= 0xc2b2ae35u;
    h ^= h >> 16;
    return h;
}

/* H(x, N, A) of Sec. 4.1: a seeded random hash of x into [0, N). */
uint32_t vbdro_H(uint32_t x, uint64_t N, uint32_t A)
{
    uint8_t key[4] = {(uint8_t)x, (uint8_t)(x >> 8), (uint8_t)(x >> 16), (uint8_t)(x >> 24)};
    uint32_t h = vbdro_murmur3_32(key, 4, A);
    return (uint32_t)(((uint64_t)h * N) >> 32);
}

/* SplitMix64 (Steele, Lea, Flood 2014): one output from state *s. */
uint64_t vbdro_splitmix64(uint64_t *s)
{
    uint64_t z = (*s += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

/* LBP1 of the (32-b)-bit string held in the top bits of w (Sec. 3, the
 * HyperLogLog rho): the position, counted from 1 at the left, of the
 * leftmost 1 bit; (32-b)+1 when all 32-b bits are 0. */
uint32_t vbdro_lbp1(uint32_t w, uint32_t b)
{
    uint32_t width = 32 - b;
    for (uint32_t pos = 1; pos <= width; pos++)
        if ((w >> (32 - pos)) & 1u)
            return pos;
    return width + 1;
}

/* ------------------------------------------------------------------ */
/* Sketch state                                                        */
/* ------------------------------------------------------------------ */

typedef struct {
    uint64_t m;       /* BDRs in the pool BDRP */
    uint32_t g, b, L; /* g = 2^b recorders per host; L = 33-b LBP1 values */
    uint32_t k;       /* window length in slices */
    uint32_t Lc;      /* recorders kept per BDR: L, or the packed layout's cap (LBP1 clamped to it) */
    uint32_t sat;     /* InitDR value and saturation bound: 255, or 2^z - 1 for z-bit DRs */
    int layout;
    uint32_t A0, A1;
    uint8_t *drv;     /* DRV of BDR p at drv[p*(L+1) + i], i = 1..L */
    uint8_t *now;     /* serial: nowLBP1 per BDR */
    uint32_t *bs;     /* fast GPU layout: bsLBP1 per BDR, bit r-1 <-> LBP1 r */
    uint8_t *reg;     /* register of each BDR over the last closed window */
    uint8_t *preg;    /* small layout: PCSA run of each BDR over the last closed window */
    uint64_t pool_hist[NBINS];
    uint64_t t;       /* closed slices */
} vbdro_sketch;

static int is_pow2(uint64_t x) { return x && !(x & (x - 1)); }

static vbdro_sketch *create(uint64_t m, uint32_t g, uint32_t k, uint64_t hash_seed, int layout, uint32_t Lc)
{
    if (!is_pow2(g) || g < 2 || g > 65536u || m <= g || m >= (1ull << 32) || k < 1 || k > 254 ||
        layout < VBDRO_SERIAL || layout > VBDRO_GPACKED)
        return NULL;
    vbdro_sketch *s = (vbdro_sketch *)calloc(1, sizeof(*s));
    if (!s)
        return NULL;
    s->m = m;
    s->g = g;
    s->b = 0;
    while ((1u << s->b) < g)
        s->b++;
    s->L = 33 - s->b;
    s->k = k;
    s->layout = layout;
    s->Lc = s->L;
    s->sat = DR_INIT;
    if (layout == VBDRO_GPACKED) {
        /* z = ceil(log2(k+1)) bits: 2^z - 1 >= k, so a DR that left the
         * window stays inactive at the saturation value */
        uint32_t z = 1;
        while (((1u << z) - 1) < k)
            z++;
        if (Lc < 1 || Lc > s->L) {
            free(s);
            return NULL;
        }
        s->Lc = Lc;
        s->sat = (1u << z) - 1;
    }
    uint64_t st = hash_seed;
    uint64_t x = vbdro_splitmix64(&st);
    s->A0 = (uint32_t)x;
    s->A1 = (uint32_t)(x >> 32);
    s->drv = (uint8_t *)malloc(m * (s->L + 1));
    s->reg = (uint8_t *)calloc(m, 1);
    if (layout == VBDRO_SERIAL)
        s->now = (uint8_t *)calloc(m, 1);
    if (layout == VBDRO_GFAST)
        s->bs = (uint32_t *)calloc(m, sizeof(uint32_t));
    if (layout >= VBDRO_GSMALL)
        s->preg = (uint8_t *)calloc(m, 1);
    if (!s->drv || !s->reg || (layout == VBDRO_SERIAL && !s->now) || (layout == VBDRO_GFAST && !s->bs) ||
        (layout >= VBDRO_GSMALL && !s->preg)) {
        free(s->drv), free(s->reg), free(s->now), free(s->bs), free(s->preg), free(s);
        return NULL;
    }
    for (uint64_t p = 0; p < m; p++)
        for (uint32_t i = 0; i <= s->L; i++)
            s->drv[p * (s->L + 1) + i] = (uint8_t)s->sat; /* InitDR */
    s->pool_hist[0] = m;
    s->t = 0;
    return s;
}

vbdro_sketch *vbdro_create(uint64_t m, uint32_t g, uint32_t k, uint64_t hash_seed, int layout)
{
    if (layout == VBDRO_GPACKED)
        return NULL;
    return create(m, g, k, hash_seed, layout, 0);
}

/* The packed layout: the small layout's algorithms (Alg. 8, 9) on z-bit DRs
 * and Lc recorders per BDR, LBP1 values above Lc recorded at Lc. */
vbdro_sketch *vbdro_create_packed(uint64_t m, uint32_t g, uint32_t k, uint64_t hash_seed, uint32_t Lc)
{
    return create(m, g, k, hash_seed, VBDRO_GPACKED, Lc);
}

void vbdro_destroy(vbdro_sketch *s)
{
    if (!s)
        return;
    free(s->drv), free(s->reg), free(s->now), free(s->bs), free(s->preg), free(s);
}

/* Distance recorders (Sec. 3).  A recorder holds how many slices ago its
 * LBP1 was last seen: 0 in the slice that sets it, one more for every slice
 * that closes, held at the saturation value.  It counts as active (the LBP1
 * lies in the window of the last k slices) while it is below k. */
static int dr_active(const vbdro_sketch *s, uint8_t dr) { return dr < s->k; }
static uint8_t dr_aged(const vbdro_sketch *s, uint8_t dr) { return dr < s->sat ? (uint8_t)(dr + 1) : dr; }

/* The recorders of BDR p, indexed by LBP1 (entry 0 unused). */
static uint8_t *recorders(vbdro_sketch *s, uint64_t p) { return s->drv + p * (s->L + 1); }

/* Where virtual recorder i of host aip lives in the pool (Sec. 4.1): the
 * index i, hashed with A0, is the seed under which aip is hashed into
 * [0, m).  Recomputed on every call, as plain as it can be. */
static uint32_t phy_idx(uint64_t m, uint32_t A0, uint32_t aip, uint32_t i)
{
    uint32_t seed = vbdro_H(i, 1ull << 32, A0);
    return vbdro_H(aip, m, seed);
}

uint32_t vbdro_phy_idx(const vbdro_sketch *s, uint32_t aip, uint32_t i)
{
    return phy_idx(s->m, s->A0, aip, i);
}

/* The BDR a pair touches and the LBP1 it records (Sec. 4.1).  One hash of
 * bip under A1 gives both: its top b bits name one of the host's g virtual
 * recorders, and the LBP1 is the 1-based rank of the leftmost 1 among its
 * other 32-b bits, 33-b when they are all 0.  Moving those bits to the top
 * and putting a 1 just below them turns that into one leading-zero count
 * (b >= 1, as g >= 2). */
static void pair_target(const vbdro_sketch *s, uint32_t aip, uint32_t bip, uint32_t *pidx, uint32_t *rho)
{
    uint32_t h = vbdro_H(bip, 1ull << 32, s->A1);
    uint32_t virt = h >> (32 - s->b);
    uint32_t rest = (h << s->b) | (1u << (s->b - 1));
    *rho = (uint32_t)__builtin_clz(rest) + 1;
    *pidx = phy_idx(s->m, s->A0, aip, virt);
}

void vbdro_pair_map(const vbdro_sketch *s, const uint32_t *pairs, uint64_t n, uint32_t *pidx, uint8_t *rho)
{
    for (uint64_t j = 0; j < n; j++) {
        uint32_t p, r;
        pair_target(s, pairs[2 * j], pairs[2 * j + 1], &p, &r);
        pidx[j] = p;
        rho[j] = (uint8_t)r;
    }
}

/* The same mapping without a pool, for pools too large to hold here. */
int vbdro_map_pairs(uint64_t m, uint32_t g, uint64_t hash_seed, const uint32_t *pairs, uint64_t n, uint32_t *pidx,
                    uint8_t *rho)
{
    if (!is_pow2(g) || g < 2 || g > 65536u || m <= g || m >= (1ull << 32))
        return -1;
    vbdro_sketch s;
    memset(&s, 0, sizeof(s));
    s.m = m, s.g = g;
    while ((1u << s.b) < g)
        s.b++;
    s.L = 33 - s.b;
    uint64_t st = hash_seed, x = vbdro_splitmix64(&st);
    s.A0 = (uint32_t)x, s.A1 = (uint32_t)(x >> 32);
    vbdro_pair_map(&s, pairs, n, pidx, rho);
    return 0;
}

/* Record the pairs of the open slice, one at a time (Sec. 3 and 4.1-4.2).
 * What is kept until the slice closes depends on the layout: the largest
 * LBP1 per BDR (serial), a bitmap of the LBP1 values seen (fast GPU
 * layout), or the recorder of each LBP1 seen, zeroed at once (small GPU
 * layouts; the packed one keeps Lc recorders, higher LBP1 values landing
 * on recorder Lc). */
void vbdro_scan(vbdro_sketch *s, const uint32_t *pairs, uint64_t n)
{
    for (uint64_t j = 0; j < n; j++) {
        uint32_t p, r;
        pair_target(s, pairs[2 * j], pairs[2 * j + 1], &p, &r);
        switch (s->layout) {
        case VBDRO_SERIAL:
            if (r > s->now[p])
                s->now[p] = (uint8_t)r;
            break;
        case VBDRO_GFAST:
            s->bs[p] |= 1u << (r - 1);
            break;
        default:
            recorders(s, p)[r < s->Lc ? r : s->Lc] = 0;
        }
    }
}

/* The register of BDR p over the window (Sec. 3): the largest LBP1 whose
 * recorder is active, 0 if none is. */
static uint32_t window_register(vbdro_sketch *s, uint64_t p)
{
    const uint8_t *v = recorders(s, p);
    uint32_t reg = 0;
    for (uint32_t r = 1; r <= s->Lc; r++)
        if (dr_active(s, v[r]))
            reg = r;
    return reg;
}

/* The PCSA reading of BDR p (the recorders as a bitmap of the LBP1 values
 * seen in the window): how many LBP1 values from 1 up are all active. */
static uint32_t pcsa_run(vbdro_sketch *s, uint64_t p)
{
    const uint8_t *v = recorders(s, p);
    uint32_t run = 0;
    while (run < s->Lc && dr_active(s, v[run + 1]))
        run++;
    return run;
}

/* Close the open slice.  In the serial and fast layouts every recorder ages
 * by one slice and then the slice's own largest LBP1 (the kept maximum, or
 * the highest bit of the bitmap) is recorded at 0, after which the window
 * is read.  The small layouts zeroed their recorders during the scan, so
 * the closing window is read first and the ageing for the next slice
 * comes after it (Sec. 4.2).  Then the pool's register histogram. */
void vbdro_advance(vbdro_sketch *s)
{
    for (uint64_t p = 0; p < s->m; p++) {
        uint8_t *v = recorders(s, p);
        if (s->layout == VBDRO_SERIAL || s->layout == VBDRO_GFAST) {
            uint32_t top;
            if (s->layout == VBDRO_SERIAL) {
                top = s->now[p];
                s->now[p] = 0;
            } else {
                top = s->bs[p] ? 32u - (uint32_t)__builtin_clz(s->bs[p]) : 0u;
                s->bs[p] = 0;
            }
            for (uint32_t r = 1; r <= s->L; r++)
                v[r] = dr_aged(s, v[r]);
            if (top > 0)
                v[top] = 0;
            s->reg[p] = (uint8_t)window_register(s, p);
        } else {
            s->reg[p] = (uint8_t)window_register(s, p);
            s->preg[p] = (uint8_t)pcsa_run(s, p);
            for (uint32_t r = 1; r <= s->L; r++)
                v[r] = dr_aged(s, v[r]);
        }
    }
    memset(s->pool_hist, 0, sizeof(s->pool_hist));
    for (uint64_t p = 0; p < s->m; p++)
        s->pool_hist[s->reg[p]]++;
    s->t++;
}

/* HyperLogLog bias constant alpha_q (Flajolet et al. 2007). */
double vbdro_alpha(double q)
{
    if (q == 16.0)
        return 0.673;
    if (q == 32.0)
        return 0.697;
    if (q == 64.0)
        return 0.709;
    return 0.7213 / (1.0 + 1.079 / q);
}

/* HyperLogLog estimate of q registers given their histogram hist[0..32]:
 * E = alpha_q q^2 / sum_j 2^-M_j, replaced by linear counting q ln(q/V) when
 * E <= 2.5 q and V = hist[0] > 0.  The harmonic sum is formed exactly as the
 * integer U = sum_r hist[r] 2^(32-r) (sum_j 2^-M_j = U 2^-32); q < 2^32. */
double vbdro_hll_from_hist(const uint64_t *hist, double q)
{
    uint64_t U = 0;
    for (uint32_t r = 0; r < NBINS; r++)
        U += hist[r] << (32 - r);
    double S = (double)U * 0x1p-32;
    double E = vbdro_alpha(q) * q * q / S;
    if (E <= 2.5 * q && hist[0] > 0)
        E = q * log(q / (double)hist[0]);
    return E;
}

/* Alg. 5 getSumLBP1, generalised from the sum of LBP1 values to their
 * histogram, then the noise-removed estimate, for a pool of m registers
 * reg[] whose histogram is pool_hist.  hist_out (n*33, nullable) receives
 * each host's histogram; raw_es (nullable) its E_s. */
static void estimate_hosts(uint64_t m, uint32_t g, uint32_t A0, const uint8_t *reg, const uint64_t *pool_hist,
                           const uint32_t *hosts, uint64_t n, float *out, double *raw_es, uint32_t *hist_out)
{
    double Em = vbdro_hll_from_hist(pool_hist, (double)m);
    for (uint64_t h = 0; h < n; h++) {
        uint64_t hist[NBINS];
        memset(hist, 0, sizeof(hist));
        for (uint32_t i = 0; i < g; i++) {
            uint32_t pidx = phy_idx(m, A0, hosts[h], i);
            hist[reg[pidx]]++; /* the BDR's register at the close */
        }
        double Es = vbdro_hll_from_hist(hist, (double)g);
        double nh = ((double)m * Es - (double)g * Em) / ((double)m - (double)g);
        out[h] = (float)(nh > 0.0 ? nh : 0.0);
        if (raw_es)
            raw_es[h] = Es;
        if (hist_out)
            for (uint32_t r = 0; r < NBINS; r++)
                hist_out[h * NBINS + r] = (uint32_t)hist[r];
    }
}

void vbdro_estimate(vbdro_sketch *s, const uint32_t *hosts, uint64_t n, float *out, double *raw_es,
                    uint32_t *hist_out)
{
    estimate_hosts(s->m, s->g, s->A0, s->reg, s->pool_hist, hosts, n, out, raw_es, hist_out);
}

/* The same estimate over a register array given by the caller (m entries,
 * each 0..32), for pools whose window state is computed another way (the
 * closed form of the recorders).  -1 for bad parameters. */
int vbdro_estimate_registers(uint64_t m, uint32_t g, uint64_t hash_seed, const uint8_t *reg, const uint32_t *hosts,
                             uint64_t n, float *out, double *raw_es, uint32_t *hist_out)
{
    if (!is_pow2(g) || g < 2 || g > 65536u || m <= g || m >= (1ull << 32))
        return -1;
    uint64_t pool_hist[NBINS];
    memset(pool_hist, 0, sizeof(pool_hist));
    for (uint64_t p = 0; p < m; p++) {
        if (reg[p] >= NBINS)
            return -1;
        pool_hist[reg[p]]++;
    }
    uint64_t st = hash_seed;
    uint32_t A0 = (uint32_t)vbdro_splitmix64(&st);
    estimate_hosts(m, g, A0, reg, pool_hist, hosts, n, out, raw_es, hist_out);
    return 0;
}

/* LogLog constant alpha_q of Durand and Flajolet (2003),
 * (Gamma(-1/q) (1 - 2^(1/q)) / ln 2)^-q.  With x = 1/q and y = x ln 2,
 * |Gamma(-x)| = Gamma(1-x)/x and 2^x - 1 = y (1 + z), z = sum_k>=1 y^k/(k+1)!,
 * so alpha_q = exp(-q (ln Gamma(1-x) + ln(1+z))): no term cancels, which a
 * pool of 2^24 and more registers needs.  q >= 16 (y < 0.05: ten terms of z
 * leave an error below 1e-20). */
double vbdro_loglog_alpha(double q)
{
    double x = 1.0 / q, y = x * log(2.0), z = 0.0, term = 1.0;
    for (int k = 1; k <= 10; k++) {
        term *= y / (double)(k + 1);
        z += term;
    }
    return exp(-q * (lgamma(1.0 - x) + log1p(z)));
}

/* Estimators on the sum S of q per-recorder values: LogLog over registers
 * (kind 1), PCSA over PCSA runs (kind 2). */
static double sum_estimate(int kind, double S, double q)
{
    if (kind == 1)
        return vbdro_loglog_alpha(q) * q * pow(2.0, S / q);
    return q / 0.77351 * pow(2.0, S / q);
}

/* Noise-removed LogLog (kind 1) or PCSA (kind 2) estimates of n hosts;
 * raw_es (nullable) receives each E_s.  -1 for PCSA without a small-layout
 * pool or for an unknown kind. */
int vbdro_estimate_kind(vbdro_sketch *s, const uint32_t *hosts, uint64_t n, int kind, float *out, double *raw_es)
{
    if (kind != 1 && !(kind == 2 && s->layout >= VBDRO_GSMALL))
        return -1;
    const uint8_t *val = kind == 1 ? s->reg : s->preg;
    uint64_t pool = 0;
    for (uint64_t p = 0; p < s->m; p++)
        pool += val[p];
    double Em = sum_estimate(kind, (double)pool, (double)s->m);
    for (uint64_t h = 0; h < n; h++) {
        uint64_t S = 0;
        for (uint32_t i = 0; i < s->g; i++)
            S += val[vbdro_phy_idx(s, hosts[h], i)];
        double Es = sum_estimate(kind, (double)S, (double)s->g);
        double nh = ((double)s->m * Es - (double)s->g * Em) / ((double)s->m - (double)s->g);
        out[h] = (float)(nh > 0.0 ? nh : 0.0);
        if (raw_es)
            raw_es[h] = Es;
    }
    return 0;
}

/* PCSA runs of the last closed window (small layout), else -1. */
int vbdro_get_preg(const vbdro_sketch *s, uint8_t *out)
{
    if (!s->preg)
        return -1;
    memcpy(out, s->preg, s->m);
    return 0;
}

/* Literal Alg. 5: the sum of the g LBP1 values of a host. */
uint64_t vbdro_sum_lbp1(vbdro_sketch *s, uint32_t aip)
{
    uint64_t sum = 0;
    for (uint32_t i = 0; i < s->g; i++)
        sum += s->reg[vbdro_phy_idx(s, aip, i)];
    return sum;
}

/* ------------------------------------------------------------------ */
/* Introspection for tests                                             */
/* ------------------------------------------------------------------ */

/* out[0..10] = m, g, b, L, k, layout, A0, A1, t, Lc, saturation value */
void vbdro_params(const vbdro_sketch *s, uint64_t *out)
{
    out[0] = s->m, out[1] = s->g, out[2] = s->b, out[3] = s->L, out[4] = s->k;
    out[5] = (uint64_t)s->layout, out[6] = s->A0, out[7] = s->A1, out[8] = s->t;
    out[9] = s->Lc, out[10] = s->sat;
}

/* Canonical state: dr[p*L + (i-1)] = DRV[i] of BDR p; bs[p] (fast layout)
 * and now[p] (serial layout) when the sketch has them; reg[p]; hist[33].
 * Any output pointer may be NULL. */
void vbdro_get_state(const vbdro_sketch *s, uint8_t *dr, uint32_t *bs, uint8_t *now, uint8_t *reg,
                     uint64_t *hist)
{
    for (uint64_t p = 0; p < s->m; p++) {
        if (dr)
            for (uint32_t i = 1; i <= s->L; i++)
                dr[p * s->L + (i - 1)] = s->drv[p * (s->L + 1) + i];
        if (bs)
            bs[p] = s->bs ? s->bs[p] : 0u;
        if (now)
            now[p] = s->now ? s->now[p] : 0u;
        if (reg)
            reg[p] = s->reg[p];
    }
    if (hist)
        memcpy(hist, s->pool_hist, sizeof(s->pool_hist));
}

/* ------------------------------------------------------------------ */
/* Closed-form window state                                            */
/* ------------------------------------------------------------------ */

/* The pool's state from the slice of each (BDR, LBP1)'s last record, the
 * quantity Sec. 3's DR counts from: last[p*L + r-1] = 1 + that slice, 0 if
 * LBP1 r was never recorded at BDR p.  A DR holds base - last, saturated at
 * sat (base = t for the fast layout, whose fold sets the DR after the
 * slide; t + 1 for the small layout, whose slide follows the read), and the
 * register (Alg. 2) is the largest LBP1 whose last record falls in the
 * window, last >= lo.  With cap < L the packed layout's recorders: LBP1
 * values cap..L share recorder cap, recorders above cap read sat.
 * dr (m*L, nullable) and reg (m) receive the canonical state. */
void vbdro_replay_state(const uint16_t *last, uint64_t m, uint32_t L, uint32_t cap, uint32_t sat, uint32_t base,
                        uint32_t lo, uint8_t *dr, uint8_t *reg)
{
    for (uint64_t p = 0; p < m; p++) {
        const uint16_t *row = last + p * L;
        uint32_t top = 0;
        for (uint32_t r = 1; r <= L; r++) {
            uint32_t s = 0;
            if (r < cap) {
                s = row[r - 1];
            } else if (r == cap) {
                for (uint32_t q = cap; q <= L; q++) /* the merged recorder: the latest record */
                    if (row[q - 1] > s)
                        s = row[q - 1];
            }
            if (s > 0 && s >= lo)
                top = r;
            if (dr) {
                uint32_t v = sat;
                if (s > 0 && base - s < sat)
                    v = base - s;
                dr[p * L + (r - 1)] = (uint8_t)v;
            }
        }
        reg[p] = (uint8_t)top;
    }
}
