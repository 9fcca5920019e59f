/*
 * synth.c -- seeded synthetic IP-pair streams for the sliding-window
 * host-cardinality workloads.  Input generation only: nothing here hashes,
 * maps or counts the way the estimator does.
 *
 * Model of one stream (all draws counter-based, so any slice can be
 * regenerated on its own):
 *   - hosts h = 0..H-1 with distinct pseudo-random 32-bit addresses aip[h]
 *     (a keyed bijection of h);
 *   - host h owns n[h] opposite hosts; n[h] ~ Zipf(s) on 1..nmax (inverse
 *     CDF), or a log-uniform draw on [lo, hi] for the planted heavy hosts;
 *   - member j of host h in slice t has address
 *         bip = mix(seed, h, j, floor((t + phase[h,j]) / churn))
 *     with phase uniform on 0..churn-1, so 1/churn of every host's
 *     opposite set is replaced at each slice boundary;
 *   - a slice holds exactly N pairs: units (h, j) are drawn with
 *     P(h) proportional to n[h] and j uniform (one uniform draw over the
 *     concatenated memberships), each repeated Poisson(lambda) times
 *     (units drawing 0 copies emit nothing), the run cut at N pairs and
 *     then permuted by a keyed Feistel bijection of [0, N).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    uint64_t seed;
    uint32_t H;          /* hosts */
    double zipf_s;       /* Zipf exponent of the background hosts */
    uint32_t nmax;       /* Zipf support 1..nmax */
    uint64_t N;          /* pairs per slice */
    uint32_t churn;      /* 1/churn of each opposite set replaced per slice */
    double lambda;       /* mean copies per unit */
    uint32_t n_heavy;    /* planted heavy hosts (hosts 0..n_heavy-1) */
    double heavy_lo, heavy_hi; /* their opposite-set sizes, log-uniform */
    /* derived */
    uint32_t *aip;       /* H */
    uint32_t *n;         /* H */
    uint64_t *cum;       /* H+1 prefix sums of n */
} synth_stream;

/* SplitMix64 finaliser as a counter-based mixer. */
static inline uint64_t fmix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}
static inline uint64_t rnd3(uint64_t key, uint64_t a, uint64_t b)
{
    return fmix64(fmix64(key + 0x9e3779b97f4a7c15ull * (a + 1)) ^ (b * 0xd1b54a32d192ed03ull + 0x8cb92ba72f3d8dd7ull));
}
static inline double u01(uint64_t r) { return (double)(r >> 11) * 0x1p-53; }

/* keyed bijection of 32-bit values: xorshift-multiply rounds, each invertible */
static inline uint32_t perm32(uint32_t x, uint64_t key)
{
    uint32_t k0 = (uint32_t)key, k1 = (uint32_t)(key >> 32);
    x ^= k0;
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    x ^= k1;
    x *= 0x9e3779b1u;
    x ^= x >> 13;
    return x;
}

void synth_destroy(synth_stream *s)
{
    if (!s)
        return;
    free(s->aip), free(s->n), free(s->cum), free(s);
}

synth_stream *synth_create(uint64_t seed, uint32_t H, double zipf_s, uint32_t nmax, uint64_t N, uint32_t churn,
                           double lambda, uint32_t n_heavy, double heavy_lo, double heavy_hi)
{
    if (H == 0 || nmax == 0 || churn == 0 || n_heavy > H || lambda <= 0)
        return NULL;
    synth_stream *s = (synth_stream *)calloc(1, sizeof(*s));
    if (!s)
        return NULL;
    s->seed = seed, s->H = H, s->zipf_s = zipf_s, s->nmax = nmax, s->N = N, s->churn = churn;
    s->lambda = lambda, s->n_heavy = n_heavy, s->heavy_lo = heavy_lo, s->heavy_hi = heavy_hi;
    s->aip = (uint32_t *)malloc(sizeof(uint32_t) * H);
    s->n = (uint32_t *)malloc(sizeof(uint32_t) * H);
    s->cum = (uint64_t *)malloc(sizeof(uint64_t) * ((uint64_t)H + 1));
    double *cdf = (double *)malloc(sizeof(double) * nmax);
    if (!s->aip || !s->n || !s->cum || !cdf) {
        free(cdf);
        synth_destroy(s);
        return NULL;
    }
    double tot = 0;
    for (uint32_t v = 1; v <= nmax; v++) {
        tot += pow((double)v, -zipf_s);
        cdf[v - 1] = tot;
    }
    uint64_t akey = fmix64(seed ^ 0xa11ce5eedull);
#pragma omp parallel for schedule(static)
    for (int64_t h = 0; h < (int64_t)H; h++) {
        s->aip[h] = perm32((uint32_t)h, akey);
        double u = u01(rnd3(seed, 0x512eull, (uint64_t)h));
        uint32_t nh;
        if ((uint32_t)h < n_heavy) {
            nh = (uint32_t)floor(exp(log(heavy_lo) + u * (log(heavy_hi) - log(heavy_lo))));
        } else {
            double target = u * tot;
            uint32_t lo = 0, hi = nmax - 1; /* first v with cdf[v] >= target */
            while (lo < hi) {
                uint32_t mid = lo + (hi - lo) / 2;
                if (cdf[mid] >= target)
                    hi = mid;
                else
                    lo = mid + 1;
            }
            nh = lo + 1;
        }
        s->n[h] = nh < 1 ? 1 : nh;
    }
    free(cdf);
    s->cum[0] = 0;
    for (uint32_t h = 0; h < H; h++)
        s->cum[h + 1] = s->cum[h] + s->n[h];
    return s;
}

void synth_hosts(const synth_stream *s, uint32_t *aip, uint32_t *n)
{
    if (aip)
        memcpy(aip, s->aip, sizeof(uint32_t) * s->H);
    if (n)
        memcpy(n, s->n, sizeof(uint32_t) * s->H);
}

/* address of member j of host h in slice t */
static inline uint32_t member(const synth_stream *s, uint32_t h, uint64_t j, uint64_t t)
{
    uint64_t key = rnd3(s->seed ^ 0xb1b1b1b1ull, h, j);
    uint64_t phase = key % s->churn;
    uint64_t epoch = (t + phase) / s->churn;
    return (uint32_t)rnd3(key, epoch, 0x0b0bull);
}

uint32_t synth_member(const synth_stream *s, uint32_t h, uint64_t j, uint64_t t) { return member(s, h, j, t); }

static inline uint32_t poisson(double lambda, double u)
{
    double p = exp(-lambda), F = p;
    uint32_t k = 0;
    while (u > F && k < 1000) {
        k++;
        p *= lambda / k;
        F += p;
    }
    return k;
}

/* Feistel bijection on [0, 2^(2*half)), cycle-walked into [0, N). */
static inline uint64_t feistel(uint64_t x, uint32_t half, uint64_t key)
{
    uint64_t mask = (1ull << half) - 1;
    uint64_t L = x >> half, R = x & mask;
    for (int r = 0; r < 4; r++) {
        uint64_t F = fmix64(R ^ (key + (uint64_t)r * 0x9e3779b97f4a7c15ull)) & mask;
        uint64_t nL = R, nR = L ^ F;
        L = nL, R = nR;
    }
    return (L << half) | R;
}
static inline uint64_t shuffle_pos(uint64_t i, uint64_t N, uint32_t half, uint64_t key)
{
    uint64_t y = feistel(i, half, key);
    while (y >= N)
        y = feistel(y, half, key);
    return y;
}

/* Emit slice t: pairs[2i], pairs[2i+1] = (aip, bip); hidx[i] = host index
 * (nullable); host_pairs[h] += pairs of host h in the slice (nullable).
 * Returns the number of pairs written (N). */
uint64_t synth_slice(const synth_stream *s, uint64_t t, uint32_t *pairs, uint32_t *hidx, uint32_t *host_pairs)
{
    const uint64_t N = s->N;
    if (N == 0)
        return 0;
    const uint64_t total = s->cum[s->H];
    const uint64_t ukey = rnd3(s->seed ^ 0x5117ceull, t, 0);
    /* pass 1: copies per unit, in blocks until N pairs are covered */
    uint64_t cap = (uint64_t)(N / s->lambda * 1.25) + 1024;
    uint32_t *copies = NULL;
    uint64_t *off = NULL;
    uint64_t U = 0;
    for (;;) {
        copies = (uint32_t *)realloc(copies, sizeof(uint32_t) * cap);
        off = (uint64_t *)realloc(off, sizeof(uint64_t) * (cap + 1));
#pragma omp parallel for schedule(static)
        for (int64_t u = 0; u < (int64_t)cap; u++)
            copies[u] = poisson(s->lambda, u01(rnd3(ukey, (uint64_t)u, 1)));
        off[0] = 0;
        for (uint64_t u = 0; u < cap; u++)
            off[u + 1] = off[u] + copies[u];
        if (off[cap] >= N) {
            U = 0;
            while (off[U + 1] < N)
                U++;
            U++; /* units 0..U-1 cover N pairs */
            break;
        }
        cap *= 2;
    }
    uint32_t bits = 1;
    while ((1ull << bits) < N)
        bits++;
    uint32_t half = (bits + 1) / 2;
    uint64_t pkey = rnd3(s->seed ^ 0x5f0ffull, t, 2);
#pragma omp parallel for schedule(dynamic, 4096)
    for (int64_t u = 0; u < (int64_t)U; u++) {
        uint64_t X = (uint64_t)(u01(rnd3(ukey, (uint64_t)u, 2)) * (double)total);
        if (X >= total)
            X = total - 1;
        uint32_t lo = 0, hi = s->H - 1; /* host with cum[h] <= X < cum[h+1] */
        while (lo < hi) {
            uint32_t mid = lo + (hi - lo + 1) / 2;
            if (s->cum[mid] <= X)
                lo = mid;
            else
                hi = mid - 1;
        }
        uint32_t h = lo;
        uint64_t j = X - s->cum[h];
        uint32_t a = s->aip[h], bip = member(s, h, j, t);
        for (uint64_t c = off[u]; c < off[u + 1] && c < N; c++) {
            uint64_t pos = shuffle_pos(c, N, half, pkey);
            pairs[2 * pos] = a;
            pairs[2 * pos + 1] = bip;
            if (hidx)
                hidx[pos] = h;
        }
        if (host_pairs) {
            uint64_t e = off[u + 1] < N ? off[u + 1] : N;
            uint32_t cnt = (uint32_t)(e - off[u]);
            if (cnt) {
#pragma omp atomic
                host_pairs[h] += cnt;
            }
        }
    }
    free(copies);
    free(off);
    return N;
}
