/*
 * Seeded synthetic graph-stream generators.
 *
 * Input generation only: nothing in this file computes any part of the
 * triangle-counting method.  Both the device library and the CPU oracle are
 * fed from the arrays written here.
 *
 * Randomness: a counter-based generator (MurmurHash3's 64-bit finaliser
 * applied to a seeded counter), so every draw is a pure function of
 * (seed, stream, index) and the output does not depend on the thread count.
 *
 * Graphs follow the paper's problem statement (Section II): a sequence of
 * undirected simple edges (u, v) with u != v and no repeated unordered pair;
 * the stream position of an edge is its array index.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#include <omp.h>

static inline uint64_t fmix64(uint64_t z) {
    z ^= z >> 33;
    z *= 0xff51afd7ed558ccdULL;
    z ^= z >> 33;
    z *= 0xc4ceb9fe1a85ec53ULL;
    z ^= z >> 33;
    return z;
}

/* draw number `i` of stream `stream` under `seed` */
static inline uint64_t crng(uint64_t seed, uint64_t stream, uint64_t i) {
    uint64_t base = fmix64(seed ^ fmix64(stream + 0x632be59bd9b4e019ULL));
    return fmix64(base + (i + 1) * 0x9e3779b97f4a7c15ULL);
}

static inline double u01(uint64_t r) { return (double)(r >> 11) * (1.0 / 9007199254740992.0); }

/* uniform integer in [0, n) by multiply-high on the top 32 bits (n < 2^32) */
static inline uint32_t below(uint64_t r, uint32_t n) {
    return (uint32_t)(((r >> 32) * (uint64_t)n) >> 32);
}

static inline uint64_t canon(uint32_t a, uint32_t b) {
    uint32_t lo = a < b ? a : b, hi = a < b ? b : a;
    return ((uint64_t)lo << 32) | hi;
}

/* ---------------- sequential open-addressing set of canonical pairs ------- */
typedef struct { uint64_t *slot; uint64_t mask; } pairset;

static int ps_init(pairset *s, uint64_t want) {
    uint64_t cap = 1024;
    while (cap < 2 * want) cap <<= 1;
    s->slot = (uint64_t *)calloc(cap, sizeof(uint64_t));
    s->mask = cap - 1;
    return s->slot ? 0 : -1;
}
/* returns 1 if inserted, 0 if already present; stored value is key+1 */
static int ps_insert(pairset *s, uint64_t key) {
    uint64_t k = key + 1, h = fmix64(key) & s->mask;
    for (;;) {
        uint64_t cur = s->slot[h];
        if (cur == 0) { s->slot[h] = k; return 1; }
        if (cur == k) return 0;
        h = (h + 1) & s->mask;
    }
}
static void ps_free(pairset *s) { free(s->slot); s->slot = NULL; }

/* Fisher-Yates shuffle of pairs with the counter generator */
static void shuffle_pairs(uint32_t *edges, uint64_t E, uint64_t order_seed) {
    if (E < 2) return;
    for (uint64_t i = E - 1; i > 0; --i) {
        uint64_t r = crng(order_seed, 7, i);
        uint64_t j = (uint64_t)(((unsigned __int128)r * (i + 1)) >> 64);
        uint32_t a = edges[2 * i], b = edges[2 * i + 1];
        edges[2 * i] = edges[2 * j];
        edges[2 * i + 1] = edges[2 * j + 1];
        edges[2 * j] = a;
        edges[2 * j + 1] = b;
    }
}

/* Erdos-Renyi G(n, M): M distinct uniform unordered pairs, then shuffled. */
int synth_er(uint32_t n, uint64_t M, uint64_t seed, uint64_t order_seed, uint32_t *edges) {
    if (n < 2 || M > (uint64_t)n * (n - 1) / 2) return -1;
    pairset s;
    if (ps_init(&s, M)) return -2;
    uint64_t kept = 0, i = 0;
    while (kept < M) {
        uint64_t r = crng(seed, 1, i++);
        uint32_t a = below(r, n), b = below(r << 32, n);
        if (a == b) continue;
        if (!ps_insert(&s, canon(a, b))) continue;
        edges[2 * kept] = a;
        edges[2 * kept + 1] = b;
        ++kept;
    }
    ps_free(&s);
    shuffle_pairs(edges, M, order_seed);
    return 0;
}

/*
 * Chung-Lu: endpoints drawn independently with probability proportional to
 * `weight` (given as a cumulative array cum[0..n], cum[0] = 0).  Self-loops and
 * repeats are rejected until E distinct pairs are kept, in draw order; the
 * result is then shuffled with order_seed.
 */
static inline uint32_t pick(const double *cum, uint32_t n, double x) {
    uint32_t lo = 0, hi = n; /* find largest i with cum[i] <= x */
    while (hi - lo > 1) {
        uint32_t mid = lo + (hi - lo) / 2;
        if (cum[mid] <= x) lo = mid; else hi = mid;
    }
    return lo;
}

int synth_chung_lu(uint32_t n, uint64_t E, const double *cum, uint64_t seed, uint64_t order_seed,
                   uint32_t *edges) {
    if (n < 2) return -1;
    pairset s;
    if (ps_init(&s, E)) return -2;
    const double total = cum[n];
    const uint64_t batch = 1 << 20;
    uint32_t *cand = (uint32_t *)malloc(sizeof(uint32_t) * 2 * batch);
    if (!cand) { ps_free(&s); return -2; }
    uint64_t kept = 0, base = 0, tries = 0;
    while (kept < E) {
        #pragma omp parallel for schedule(static)
        for (int64_t j = 0; j < (int64_t)batch; ++j) {
            uint64_t i = base + (uint64_t)j;
            cand[2 * j] = pick(cum, n, u01(crng(seed, 2, i)) * total);
            cand[2 * j + 1] = pick(cum, n, u01(crng(seed, 3, i)) * total);
        }
        for (uint64_t j = 0; j < batch && kept < E; ++j) {
            uint32_t a = cand[2 * j], b = cand[2 * j + 1];
            if (a == b || !ps_insert(&s, canon(a, b))) continue;
            edges[2 * kept] = a;
            edges[2 * kept + 1] = b;
            ++kept;
        }
        base += batch;
        if (++tries > 4096) { free(cand); ps_free(&s); return -3; } /* graph too dense */
    }
    free(cand);
    ps_free(&s);
    shuffle_pairs(edges, E, order_seed);
    return 0;
}

/*
 * R-MAT (Chakrabarti, Zhan, Faloutsos 2004): 2^scale * edge_factor draws, each
 * choosing one quadrant per level with probabilities (a, b, c, 1-a-b-c).  No
 * noise and no vertex permutation.  Self-loops are dropped; of repeated
 * unordered pairs only the first draw is kept; the kept draws stay in
 * generation order.  Returns the number of kept edges (written to `edges`,
 * which must hold 2 * 2^scale * edge_factor entries), or a negative error.
 */
int64_t synth_rmat(uint32_t scale, uint32_t edge_factor, double a, double b, double c,
                   uint64_t seed, uint32_t *edges) {
    if (scale < 1 || scale > 31) return -1;
    const uint64_t D = ((uint64_t)1 << scale) * edge_factor;
    const uint32_t ta = (uint32_t)(a * 4294967296.0), tb = (uint32_t)((a + b) * 4294967296.0),
                   tc = (uint32_t)((a + b + c) * 4294967296.0);
    /* 1) draws */
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < (int64_t)D; ++i) {
        uint32_t u = 0, v = 0;
        uint64_t r = 0;
        for (uint32_t lvl = 0; lvl < scale; ++lvl) {
            if ((lvl & 1) == 0) r = crng(seed, 4 + lvl / 2, (uint64_t)i);
            uint32_t x = (uint32_t)(r >> ((lvl & 1) ? 32 : 0));
            uint32_t bu, bv;
            if (x < ta) { bu = 0; bv = 0; }
            else if (x < tb) { bu = 0; bv = 1; }
            else if (x < tc) { bu = 1; bv = 0; }
            else { bu = 1; bv = 1; }
            u = (u << 1) | bu;
            v = (v << 1) | bv;
        }
        edges[2 * i] = u;
        edges[2 * i + 1] = v;
    }
    /* 2) first occurrence of each canonical pair: table of (key+1, min index) */
    uint64_t cap = 1024;
    while (cap < 2 * D) cap <<= 1;
    uint64_t *keys = (uint64_t *)calloc(cap, sizeof(uint64_t));
    uint64_t *first = (uint64_t *)malloc(cap * sizeof(uint64_t));
    uint8_t *keep = (uint8_t *)malloc(D);
    if (!keys || !first || !keep) { free(keys); free(first); free(keep); return -2; }
    const uint64_t mask = cap - 1;
    #pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < (int64_t)cap; ++s) first[s] = UINT64_MAX;
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < (int64_t)D; ++i) {
        uint32_t u = edges[2 * i], v = edges[2 * i + 1];
        if (u == v) continue;
        uint64_t key = canon(u, v), k1 = key + 1, h = fmix64(key) & mask;
        for (;;) {
            uint64_t cur = __atomic_load_n(&keys[h], __ATOMIC_ACQUIRE);
            if (cur == 0) {
                uint64_t expect = 0;
                if (__atomic_compare_exchange_n(&keys[h], &expect, k1, 0, __ATOMIC_ACQ_REL,
                                                __ATOMIC_ACQUIRE)) break;
                cur = expect;
            }
            if (cur == k1) break;
            h = (h + 1) & mask;
        }
        uint64_t old = __atomic_load_n(&first[h], __ATOMIC_RELAXED);
        while ((uint64_t)i < old &&
               !__atomic_compare_exchange_n(&first[h], &old, (uint64_t)i, 0, __ATOMIC_RELAXED,
                                            __ATOMIC_RELAXED)) {
        }
    }
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < (int64_t)D; ++i) {
        uint32_t u = edges[2 * i], v = edges[2 * i + 1];
        keep[i] = 0;
        if (u == v) continue;
        uint64_t key = canon(u, v), k1 = key + 1, h = fmix64(key) & mask;
        while (keys[h] != k1) h = (h + 1) & mask;
        keep[i] = (first[h] == (uint64_t)i);
    }
    free(keys);
    free(first);
    /* 3) stable compaction */
    uint64_t out = 0;
    for (uint64_t i = 0; i < D; ++i) {
        if (!keep[i]) continue;
        edges[2 * out] = edges[2 * i];
        edges[2 * out + 1] = edges[2 * i + 1];
        ++out;
    }
    free(keep);
    return (int64_t)out;
}

/* uniform doubles in [0,1) for host-side samplers (sizes, arrivals) */
void synth_uniform(uint64_t seed, uint64_t stream, uint64_t count, double *out) {
    for (uint64_t i = 0; i < count; ++i) out[i] = u01(crng(seed, stream, i));
}

/* raw 64-bit draws (used to derive per-job or per-replica seeds) */
void synth_u64(uint64_t seed, uint64_t stream, uint64_t count, uint64_t *out) {
    for (uint64_t i = 0; i < count; ++i) out[i] = crng(seed, stream, i);
}
