/*
 * CPU oracle for REPT (Wang et al., "REPT: A Streaming Algorithm of Approximating Global and
 * Local Triangle Counts in Parallel", arXiv:1811.09136).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, single-threaded statement of what
 * the device path must compute.  It shares no code, header, table or helper with the device
 * library; only the test suite, the smoke check and the bench's CPU-baseline leg use it.
 *
 * Conventions (the readings of the paper this oracle fixes):
 *  - processors, groups and slots are 0-based: processor i belongs to group k = i / m and
 *    owns slot j = i % m of that group's hash h_k : E -> [0, m) (Algorithm 2 uses this
 *    floor/modulo mapping; Algorithm 1 is its one-group case);
 *  - edges are undirected: h_k hashes the unordered pair (min, max);
 *  - when a group has fewer than m processors (c < m, or the last group when m does not
 *    divide c), an edge whose slot has no processor is stored by no processor of that group;
 *  - an edge is counted before it is inserted (Algorithm 1: UpdateTriangleCNT precedes the
 *    insertion), so N_u^(i) at time t holds only edges that arrived strictly earlier;
 *  - counters are 64-bit integers.
 *
 * Hash family.  Section III-A asks for a uniform map with P(h(e)=i, h(e')=i') = 1/m^2; the
 * variance of Theorem 3 also uses the joint behaviour of the first two edges of two triangles
 * (up to four edges), so this oracle uses a 4-wise independent family: a degree-3 polynomial
 * over the prime field GF(p), p = 2^61 - 1 (Carter and Wegman 1979; Wegman and Carter 1981).
 * For group k the coefficients a_0..a_3 are SplitMix64 outputs 4k..4k+3 of the user seed
 * (Steele, Lea, Flood, OOPSLA 2014), each shifted right by 3 and reduced mod p.  The edge
 * key is x = lo * 2^32 + hi (lo = min(u,v), hi = max(u,v); x < p for ids below 2^29),
 * h = a_3 x^3 + a_2 x^2 + a_1 x + a_0 mod p, and slot = floor(h * m / 2^61).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <pthread.h>

#define OR_OK 0
#define OR_EINVAL (-1)
#define OR_ERANGE (-2)
#define OR_ESELFLOOP (-3)
#define OR_EDUP (-4)
#define OR_ENOMEM (-5)
#define OR_ENOTSUP (-7)

/* ------------------------------------------------------------------ hash ---------------- */

/* SplitMix64: the state advances by the golden gamma, the output is the state mixed by two
 * xor-shift-multiply rounds and a final xor-shift (Steele, Lea, Flood 2014). */
static uint64_t splitmix64_next(uint64_t *state) {
    uint64_t z = (*state += 0x9e3779b97f4a7c15ULL);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

uint64_t oracle_splitmix64(uint64_t seed, uint64_t index) {
    uint64_t s = seed, r = 0;
    for (uint64_t i = 0; i <= index; ++i) r = splitmix64_next(&s);
    return r;
}

#define P61 ((((uint64_t)1) << 61) - 1)

/* group k's coefficients (a_0, a_1, a_2, a_3), written to params[4k .. 4k+3] */
void oracle_hash_params(uint64_t seed, uint32_t G, uint64_t *params) {
    uint64_t s = seed;
    for (uint32_t i = 0; i < 4 * G; ++i) params[i] = (splitmix64_next(&s) >> 3) % P61;
}

uint32_t oracle_slot(const uint64_t *a, uint32_t m, uint32_t u, uint32_t v) {
    const unsigned __int128 p = P61;
    const uint64_t lo = u < v ? u : v, hi = u < v ? v : u;
    const unsigned __int128 x = (unsigned __int128)((lo << 32) | hi) % p;
    /* a_3 x^3 + a_2 x^2 + a_1 x + a_0 in GF(p), each power formed explicitly */
    const unsigned __int128 x2 = (x * x) % p, x3 = (x2 * x) % p;
    const unsigned __int128 h = (a[3] * x3 % p + a[2] * x2 % p + a[1] * x % p + a[0]) % p;
    return (uint32_t)((h * m) >> 61);
}

/* slots of every edge for every group: out[k*E + t] = h_k(edge t) */
void oracle_slots(uint64_t seed, uint32_t m, uint32_t G, const uint32_t *edges, uint64_t E,
                  uint32_t *out) {
    uint64_t *params = (uint64_t *)malloc(sizeof(uint64_t) * 4 * (G ? G : 1));
    if (!params) return;
    oracle_hash_params(seed, G, params);
    for (uint32_t k = 0; k < G; ++k)
        for (uint64_t t = 0; t < E; ++t)
            out[(uint64_t)k * E + t] = oracle_slot(params + 4 * k, m, edges[2 * t], edges[2 * t + 1]);
    free(params);
}

/* ------------------------------------------------------------------ edge set ------------ */

typedef struct {
    uint64_t *key; /* canonical pair + 1; 0 = empty */
    uint64_t *val;
    uint64_t mask, count;
} edgeset;

static uint64_t mix(uint64_t x) {
    x ^= x >> 31;
    x *= 0x7fb5d329728ea185ULL;
    x ^= x >> 27;
    x *= 0x81dadef4bc2dd44dULL;
    x ^= x >> 33;
    return x;
}

static int es_init(edgeset *s, uint64_t expect) {
    uint64_t cap = 16;
    while (cap < 2 * expect + 2) cap <<= 1;
    s->key = (uint64_t *)calloc(cap, sizeof(uint64_t));
    s->val = (uint64_t *)calloc(cap, sizeof(uint64_t));
    s->mask = cap - 1;
    s->count = 0;
    return (s->key && s->val) ? 0 : -1;
}
static void es_free(edgeset *s) {
    free(s->key);
    free(s->val);
    s->key = s->val = NULL;
}
static uint64_t pairkey(uint32_t u, uint32_t v) {
    uint64_t lo = u < v ? u : v, hi = u < v ? v : u;
    return (lo << 32) | hi;
}
/* 1 if inserted, 0 if present */
static int es_put(edgeset *s, uint64_t k, uint64_t val) {
    uint64_t h = mix(k) & s->mask, k1 = k + 1;
    while (s->key[h]) {
        if (s->key[h] == k1) return 0;
        h = (h + 1) & s->mask;
    }
    s->key[h] = k1;
    s->val[h] = val;
    s->count++;
    return 1;
}
static int es_get(const edgeset *s, uint64_t k, uint64_t *val) {
    uint64_t h = mix(k) & s->mask, k1 = k + 1;
    while (s->key[h]) {
        if (s->key[h] == k1) {
            if (val) *val = s->val[h];
            return 1;
        }
        h = (h + 1) & s->mask;
    }
    return 0;
}

/* Section II: a simple undirected stream over nodes [0, n) */
int oracle_validate(uint32_t n, const uint32_t *edges, uint64_t E) {
    if (n > (1u << 29)) return OR_EINVAL; /* hash keys lo * 2^32 + hi must stay below 2^61 - 1 */
    for (uint64_t t = 0; t < E; ++t) {
        if (edges[2 * t] >= n || edges[2 * t + 1] >= n) return OR_ERANGE;
    }
    for (uint64_t t = 0; t < E; ++t) {
        if (edges[2 * t] == edges[2 * t + 1]) return OR_ESELFLOOP;
    }
    /* set of unordered pairs seen so far (keys only; open addressing, load <= 1/2) */
    uint64_t cap = 16;
    while (cap < 2 * E + 2) cap <<= 1;
    uint64_t *key = (uint64_t *)calloc(cap, sizeof(uint64_t));
    if (!key) return OR_ENOMEM;
    int rc = OR_OK;
    for (uint64_t t = 0; t < E && rc == OR_OK; ++t) {
        const uint64_t k1 = pairkey(edges[2 * t], edges[2 * t + 1]) + 1;
        uint64_t h = mix(k1 - 1) & (cap - 1);
        while (key[h] && key[h] != k1) h = (h + 1) & (cap - 1);
        if (key[h] == k1) rc = OR_EDUP;
        key[h] = k1;
    }
    free(key);
    return rc;
}

/* ------------------------------------------------------------------ Algorithm 1 ---------- */

/* growable adjacency list of one processor's sampled graph */
typedef struct {
    uint32_t *nbr;
    uint32_t len, cap;
} adjlist;

static int adj_push(adjlist *a, uint32_t w) {
    if (a->len == a->cap) {
        uint32_t nc = a->cap ? 2 * a->cap : 4;
        uint32_t *p = (uint32_t *)realloc(a->nbr, nc * sizeof(uint32_t));
        if (!p) return -1;
        a->nbr = p;
        a->cap = nc;
    }
    a->nbr[a->len++] = w;
    return 0;
}

/*
 * One processor's replay of Algorithm 1 (Section III-A): processor i = k*m + j, which stores the
 * edges whose slot in its group is j (slot[t] = h_k(edge t)).  The stream is replayed in order;
 * for each edge (u, v) at time t:
 *   UpdateTriangleCNT: N = N_u^(i) intersect N_v^(i); tau^(i) += |N|; tau_u^(i) += |N|;
 *                      tau_v^(i) += |N|; tau_w^(i) += 1 for each w in N;
 *   then, if h_k(u, v) == j, (u, v) joins E^(i).
 * The counter updates are applied only for t in [t0, t1) (a window of stream positions); the
 * insertions always happen, so a window's counts are the per-edge updates of that window.
 * tau^(i) is added to *glob and tau_v^(i) to loc[v].  adj: n empty-or-reusable lists (scratch).
 */
static int replay_processor(uint32_t n, uint32_t j, const uint32_t *slot, const uint32_t *edges, uint64_t E,
                            uint64_t t0, uint64_t t1, adjlist *adj, int64_t *glob, int64_t *loc) {
    uint64_t mine = 0; /* |E^(i)| at the end of the stream */
    for (uint64_t t = 0; t < E; ++t) mine += (slot[t] == j);
    edgeset Ei; /* E^(i), for membership tests */
    if (es_init(&Ei, mine)) return OR_ENOMEM;
    int rc = OR_OK;
    for (uint32_t x = 0; x < n; ++x) adj[x].len = 0;
    for (uint64_t t = 0; t < E; ++t) {
        const uint32_t u = edges[2 * t], v = edges[2 * t + 1];
        if (t >= t0 && t < t1) {
            /* N_{u,v}^(i) = N_u^(i) intersect N_v^(i): walk the smaller set, test the other */
            const adjlist *small = adj[u].len <= adj[v].len ? &adj[u] : &adj[v];
            const uint32_t other = adj[u].len <= adj[v].len ? v : u;
            int64_t cnt = 0;
            for (uint32_t q = 0; q < small->len; ++q) {
                const uint32_t w = small->nbr[q];
                if (es_get(&Ei, pairkey(other, w), NULL)) {
                    ++cnt;
                    loc[w] += 1; /* tau_w^(i) += 1 */
                }
            }
            *glob += cnt;  /* tau^(i) += |N| */
            loc[u] += cnt; /* tau_u^(i) += |N| */
            loc[v] += cnt; /* tau_v^(i) += |N| */
        }
        if (slot[t] == j) { /* h_k(u,v) selects processor i: insert into E^(i) */
            es_put(&Ei, pairkey(u, v), t);
            if (adj_push(&adj[u], v) || adj_push(&adj[v], u)) {
                rc = OR_ENOMEM;
                break;
            }
        }
    }
    es_free(&Ei);
    return rc;
}

/*
 * REPT per Algorithm 1, extended to c > m by independent groups (Section III-B): every
 * processor i = k*m + j (j < c_k) of every group k replays the stream (replay_processor).
 *
 * Outputs (accumulated, +=):
 *   global[i]                    = tau^(i)                              (c entries)
 *   local[k*n + v]               = sum over processors i of group k of tau_v^(i)   (per_proc = 0)
 *   local[i*n + v]               = tau_v^(i)                                       (per_proc = 1)
 * slot_override (optional, [G][E] uint16): replaces h_k(edge t) by slot_override[k*E + t].
 * Only processors i in [p_lo, p_hi) are replayed (processors are independent trials, Section
 * I); the others contribute nothing, so disjoint ranges sum to the full result.
 */
int oracle_rept_procs(uint32_t n, uint32_t m, uint32_t c, uint64_t seed, int per_proc,
                      const uint32_t *edges, uint64_t E, uint64_t t0, uint64_t t1,
                      const uint16_t *slot_override, uint32_t p_lo, uint32_t p_hi, int64_t *global,
                      int64_t *local) {
    if (n == 0 || m == 0 || c == 0 || !edges || !global || !local) return OR_EINVAL;
    if (t0 > t1 || t1 > E || p_lo > p_hi || p_hi > c) return OR_EINVAL;
    int rc = oracle_validate(n, edges, E);
    if (rc) return rc;
    const uint32_t G = (c + m - 1) / m;
    uint64_t *params = (uint64_t *)malloc(sizeof(uint64_t) * 4 * G);
    adjlist *adj = (adjlist *)calloc(n, sizeof(adjlist));
    uint32_t *slot = (uint32_t *)malloc(sizeof(uint32_t) * (E ? E : 1));
    if (!params || !adj || !slot) {
        free(params);
        free(adj);
        free(slot);
        return OR_ENOMEM;
    }
    oracle_hash_params(seed, G, params);

    for (uint32_t k = 0; k < G && rc == OR_OK; ++k) {
        const uint32_t ck = (k + 1 < G) ? m : c - (G - 1) * m; /* processors in group k */
        if (k * m + ck <= p_lo || k * m >= p_hi) continue;  /* no processor of this group asked */
        for (uint64_t t = 0; t < E; ++t) {
            slot[t] = slot_override ? slot_override[(uint64_t)k * E + t]
                                    : oracle_slot(params + 4 * k, m, edges[2 * t], edges[2 * t + 1]);
        }
        for (uint32_t j = 0; j < ck && rc == OR_OK; ++j) {
            const uint32_t i = k * m + j;
            if (i < p_lo || i >= p_hi) continue;
            rc = replay_processor(n, j, slot, edges, E, t0, t1, adj, global + i,
                                  local + (uint64_t)(per_proc ? i : k) * n);
        }
    }
    for (uint32_t x = 0; x < n; ++x) free(adj[x].nbr);
    free(adj);
    free(slot);
    free(params);
    return rc;
}

/*
 * The same replay with the processors spread over `threads` host threads (processors are
 * independent trials, Section I, so the order in which they run does not matter).  The stream
 * is validated once and every group's slots are computed once, shared by the threads; each
 * thread replays whole processors with its own lists and, for group sums, its own local rows,
 * which are added at the end.  Outputs and arguments as oracle_rept_procs (processors
 * [p_lo, p_hi), accumulated, +=), without slot_override.
 */
typedef struct {
    uint32_t n, m, end, G, per_proc; /* processors next .. end - 1 are replayed */
    const uint32_t *edges;
    uint64_t E, t0, t1;
    const uint32_t *slots; /* [G][E] */
    int64_t *global, *local;
    uint32_t next;         /* next processor to replay (shared) */
    pthread_mutex_t mu;
    int rc;
} par_job;

typedef struct {
    par_job *job;
    int64_t *rows; /* private group rows [G][n] (per_proc = 0), else NULL */
} par_worker;

typedef struct {
    const uint64_t *params;
    uint32_t m, G;
    const uint32_t *edges;
    uint64_t E, lo, hi;
    uint32_t *slots;
} slot_part;

static void *slot_range(void *arg) {
    slot_part *p = (slot_part *)arg;
    for (uint32_t k = 0; k < p->G; ++k)
        for (uint64_t t = p->lo; t < p->hi; ++t)
            p->slots[(uint64_t)k * p->E + t] = oracle_slot(p->params + 4 * k, p->m, p->edges[2 * t], p->edges[2 * t + 1]);
    return NULL;
}

static void *par_replay(void *arg) {
    par_worker *w = (par_worker *)arg;
    par_job *J = w->job;
    adjlist *adj = (adjlist *)calloc(J->n, sizeof(adjlist));
    if (!adj) {
        pthread_mutex_lock(&J->mu);
        J->rc = OR_ENOMEM;
        pthread_mutex_unlock(&J->mu);
        return NULL;
    }
    for (;;) {
        pthread_mutex_lock(&J->mu);
        const uint32_t i = J->next;
        const int stop = J->rc != OR_OK || i >= J->end;
        if (!stop) J->next = i + 1;
        pthread_mutex_unlock(&J->mu);
        if (stop) break;
        const uint32_t k = i / J->m, j = i % J->m;
        int64_t g = 0;
        int64_t *loc = J->per_proc ? J->local + (uint64_t)i * J->n : w->rows + (uint64_t)k * J->n;
        const int rc = replay_processor(J->n, j, J->slots + (uint64_t)k * J->E, J->edges, J->E, J->t0, J->t1, adj,
                                        &g, loc);
        pthread_mutex_lock(&J->mu);
        J->global[i] += g; /* each processor's own entry */
        if (rc != OR_OK) J->rc = rc;
        pthread_mutex_unlock(&J->mu);
    }
    for (uint32_t x = 0; x < J->n; ++x) free(adj[x].nbr);
    free(adj);
    return NULL;
}

int oracle_rept_parallel(uint32_t n, uint32_t m, uint32_t c, uint64_t seed, int per_proc, const uint32_t *edges,
                         uint64_t E, uint64_t t0, uint64_t t1, uint32_t p_lo, uint32_t p_hi, uint32_t threads,
                         int64_t *global, int64_t *local) {
    if (n == 0 || m == 0 || c == 0 || !edges || !global || !local || threads == 0) return OR_EINVAL;
    if (t0 > t1 || t1 > E || p_lo > p_hi || p_hi > c) return OR_EINVAL;
    int rc = oracle_validate(n, edges, E);
    if (rc) return rc;
    const uint32_t G = (c + m - 1) / m;
    if (threads > p_hi - p_lo) threads = p_hi - p_lo ? p_hi - p_lo : 1;
    uint64_t *params = (uint64_t *)malloc(sizeof(uint64_t) * 4 * G);
    uint32_t *slots = (uint32_t *)malloc(sizeof(uint32_t) * (uint64_t)G * (E ? E : 1));
    pthread_t *tid = (pthread_t *)calloc(threads, sizeof(pthread_t));
    par_worker *wk = (par_worker *)calloc(threads, sizeof(par_worker));
    slot_part *sp = (slot_part *)calloc(threads, sizeof(slot_part));
    if (!params || !slots || !tid || !wk || !sp) {
        rc = OR_ENOMEM;
        goto done;
    }
    oracle_hash_params(seed, G, params);
    /* every group's slots h_k(edge t), the stream split over the threads */
    for (uint32_t q = 0; q < threads; ++q) {
        sp[q] = (slot_part){params, m, G, edges, E, E * q / threads, E * (q + 1) / threads, slots};
        pthread_create(&tid[q], NULL, slot_range, &sp[q]);
    }
    for (uint32_t q = 0; q < threads; ++q) pthread_join(tid[q], NULL);

    par_job J = {n, m, p_hi, G, (uint32_t)(per_proc != 0), edges, E, t0, t1, slots, global, local, p_lo,
                 PTHREAD_MUTEX_INITIALIZER, OR_OK};
    for (uint32_t q = 0; q < threads; ++q) {
        wk[q].job = &J;
        if (!per_proc) {
            wk[q].rows = (int64_t *)calloc((uint64_t)G * n, sizeof(int64_t));
            if (!wk[q].rows) J.rc = OR_ENOMEM;
        }
    }
    if (J.rc == OR_OK) {
        for (uint32_t q = 0; q < threads; ++q) pthread_create(&tid[q], NULL, par_replay, &wk[q]);
        for (uint32_t q = 0; q < threads; ++q) pthread_join(tid[q], NULL);
    }
    rc = J.rc;
    if (rc == OR_OK && !per_proc) /* the threads' group rows, added */
        for (uint32_t q = 0; q < threads; ++q)
            for (uint64_t x = 0; x < (uint64_t)G * n; ++x) local[x] += wk[q].rows[x];
    for (uint32_t q = 0; q < threads; ++q) free(wk[q].rows);
done:
    free(params);
    free(slots);
    free(tid);
    free(wk);
    free(sp);
    return rc;
}

/* all c processors */
int oracle_rept(uint32_t n, uint32_t m, uint32_t c, uint64_t seed, int per_proc,
                const uint32_t *edges, uint64_t E, uint64_t t0, uint64_t t1,
                const uint16_t *slot_override, int64_t *global, int64_t *local) {
    return oracle_rept_procs(n, m, c, seed, per_proc, edges, E, t0, t1, slot_override, 0, c, global, local);
}

/* ------------------------------------------------------------------ per-edge form -------- */

/*
 * The per-edge update of Algorithm 1 evaluated directly from its definition, for all
 * processors at once, for the stream positions listed in `ts` (any order, no repeats).
 *
 * At time t, N_u^(i) is the set of w such that edge {u, w} arrived before t and
 * h_k({u, w}) selected processor i.  So for the edge (u, v) at time t, processor
 * i = k*m + j gains one semi-triangle for every common neighbour w of u and v (in the whole
 * stream graph) whose two edges {u, w}, {v, w} both arrived before t and both hash to slot j
 * of group k, with j < c_k.  Counts are accumulated (+=) exactly as oracle_rept does for a
 * window, so the two must agree; this form needs no replay of the stream and is what makes
 * sampled checks possible on large streams.
 *
 * The static adjacency (neighbour, arrival time) is built once per call with a counting
 * sort by vertex; each neighbour list is then searched linearly (plain, not fast).
 */
typedef struct {
    uint32_t w;
    uint32_t t;
} nbr_t;

static int cmp_nbr(const void *a, const void *b) {
    const nbr_t *x = (const nbr_t *)a, *y = (const nbr_t *)b;
    return (x->w > y->w) - (x->w < y->w);
}

int oracle_edge_updates(uint32_t n, uint32_t m, uint32_t c, uint64_t seed, int per_proc,
                        const uint32_t *edges, uint64_t E, const uint64_t *ts, uint64_t nts,
                        int64_t *global, int64_t *local) {
    if (n == 0 || m == 0 || c == 0 || !edges || !global || !local) return OR_EINVAL;
    for (uint64_t q = 0; q < nts; ++q)
        if (ts[q] >= E) return OR_EINVAL;
    int rc = oracle_validate(n, edges, E);
    if (rc) return rc;
    const uint32_t G = (c + m - 1) / m;
    uint64_t *params = (uint64_t *)malloc(sizeof(uint64_t) * 4 * G);
    uint64_t *off = (uint64_t *)calloc((uint64_t)n + 1, sizeof(uint64_t));
    uint64_t *fill = (uint64_t *)calloc((uint64_t)n, sizeof(uint64_t));
    uint8_t *need = (uint8_t *)calloc((uint64_t)n, 1);
    if (!params || !off || !fill || !need) {
        free(params);
        free(off);
        free(fill);
        free(need);
        return OR_ENOMEM;
    }
    oracle_hash_params(seed, G, params);
    /* adjacency lists only of the endpoints of the edges asked for */
    for (uint64_t q = 0; q < nts; ++q) {
        need[edges[2 * ts[q]]] = 1;
        need[edges[2 * ts[q] + 1]] = 1;
    }
    for (uint64_t t = 0; t < E; ++t) {
        const uint32_t u = edges[2 * t], v = edges[2 * t + 1];
        if (need[u]) off[u + 1]++;
        if (need[v]) off[v + 1]++;
    }
    for (uint32_t x = 0; x < n; ++x) off[x + 1] += off[x];
    nbr_t *nb = (nbr_t *)malloc(sizeof(nbr_t) * (off[n] ? off[n] : 1));
    if (!nb) {
        free(params);
        free(off);
        free(fill);
        free(need);
        return OR_ENOMEM;
    }
    for (uint64_t t = 0; t < E; ++t) {
        const uint32_t u = edges[2 * t], v = edges[2 * t + 1];
        if (need[u]) nb[off[u] + fill[u]++] = (nbr_t){v, (uint32_t)t};
        if (need[v]) nb[off[v] + fill[v]++] = (nbr_t){u, (uint32_t)t};
    }
    for (uint32_t x = 0; x < n; ++x)
        if (need[x]) qsort(nb + off[x], off[x + 1] - off[x], sizeof(nbr_t), cmp_nbr);
    free(need);

    for (uint64_t q = 0; q < nts; ++q) {
        const uint64_t t = ts[q];
        const uint32_t u = edges[2 * t], v = edges[2 * t + 1];
        /* common neighbours of u and v by a merge of the two id-sorted lists */
        uint64_t a = off[u], ae = off[u + 1], b = off[v], be = off[v + 1];
        while (a < ae && b < be) {
            if (nb[a].w < nb[b].w) {
                ++a;
            } else if (nb[a].w > nb[b].w) {
                ++b;
            } else {
                const uint32_t w = nb[a].w;
                if (nb[a].t < t && nb[b].t < t) { /* both edges arrived before t */
                    for (uint32_t k = 0; k < G; ++k) {
                        const uint32_t ck = (k + 1 < G) ? m : c - (G - 1) * m;
                        const uint32_t su = oracle_slot(params + 4 * k, m, u, w);
                        const uint32_t sv = oracle_slot(params + 4 * k, m, v, w);
                        if (su == sv && su < ck) {
                            const uint32_t i = k * m + su;
                            int64_t *loc = local + (uint64_t)(per_proc ? i : k) * n;
                            global[i] += 1;
                            loc[u] += 1;
                            loc[v] += 1;
                            loc[w] += 1;
                        }
                    }
                }
                ++a;
                ++b;
            }
        }
    }
    free(params);
    free(off);
    free(nb);
    free(fill);
    return OR_OK;
}

/* ------------------------------------------------------------------ estimators ----------- */

/*
 * Estimators for c <= m (Algorithm 1, Section III-A) and for c > m with m dividing c
 * (Section III-B, case c2 = 0):
 *   tau_hat   = m^2 / c * sum_i tau^(i)          (equals m / c1 * sum when c = c1 * m)
 *   tau_v_hat = m^2 / c * sum_i tau_v^(i)
 * evaluated as ((double)S * (double)(m*m)) / (double)c in IEEE binary64, round to nearest.
 * The sum S is exact in 64-bit integers; S >= 2^53 is refused (the conversion would round).
 * c > m with c % m != 0 (Algorithm 2) is not handled here.
 * local_rows: rows of `local` (G group sums, or c per-processor rows); all rows are summed.
 */
int oracle_estimate(uint32_t n, uint32_t m, uint32_t c, uint32_t local_rows,
                    const int64_t *global, const int64_t *local, double *tau_hat, double *tau_v_hat) {
    if (n == 0 || m == 0 || c == 0 || !global || !tau_hat) return OR_EINVAL;
    if (c > m && c % m != 0) return OR_ENOTSUP;
    const int64_t lim = (int64_t)1 << 53;
    const double scale_num = (double)((uint64_t)m * (uint64_t)m);
    const double denom = (double)c;
    int64_t S = 0;
    for (uint32_t i = 0; i < c; ++i) {
        if (global[i] < 0 || global[i] >= lim - S) return OR_ERANGE;
        S += global[i];
    }
    *tau_hat = ((double)S * scale_num) / denom;
    if (tau_v_hat && local) {
        for (uint32_t v = 0; v < n; ++v) {
            int64_t Sv = 0;
            for (uint32_t r = 0; r < local_rows; ++r) {
                const int64_t x = local[(uint64_t)r * n + v];
                if (x < 0 || x >= lim - Sv) return OR_ERANGE;
                Sv += x;
            }
            tau_v_hat[v] = ((double)Sv * scale_num) / denom;
        }
    }
    return OR_OK;
}

/* ------------------------------------------------------------------ Algorithm 2 counters -- */

/*
 * The triangle-pair counters of Section III-B, from their definition.
 *
 * eta^(i) is the number of unordered pairs of distinct semi-triangles of processor i (triangles
 * whose two earlier edges processor i stored) that share an edge which is the last edge of
 * neither.  Two distinct triangles share at most one edge, and an edge that is not the last of
 * a semi-triangle of i is one of its two earlier edges, so it is an edge g of E^(i).  With
 *   s_g = the number of semi-triangles of i in which g is one of the two earlier edges,
 * the pairs sharing g number C(s_g, 2), and eta^(i) = sum over g in E^(i) of C(s_g, 2).
 * Both triangles of such a pair contain node v only when v is an endpoint of g (otherwise they
 * would share a second edge), so eta_v^(i) = sum over the edges g of E^(i) at v of C(s_g, 2).
 *
 * Algorithm 2 as printed starts the counter of a newly stored edge g at |N| (the number of
 * semi-triangles of i whose last edge is g, call it L_g) and adds the counter's current value
 * each time g is an earlier edge of a new semi-triangle; its totals are therefore
 * sum over g of (s_g L_g + C(s_g, 2)), per processor and per endpoint.  Both readings are
 * returned (the first is the definition, which the estimator's E(eta^(i)) = eta / m^3 needs).
 *
 * Per processor i = k*m + j the stream is replayed in order to find its semi-triangles: for the
 * edge (u, v) at time t every w in N_u^(i) intersect N_v^(i) closes one, with earlier edges
 * {u, w} and {v, w}; then (u, v) joins E^(i) if h_k(u, v) = j, and L of it is |N|.  The sums
 * are taken after the whole stream.
 * Outputs (overwritten): eta_def[i], eta_lit[i] for every processor i < c; eta_v_def[v],
 * eta_v_lit[v] = sum over all processors of eta_v^(i).
 */
int oracle_rept2_eta(uint32_t n, uint32_t m, uint32_t c, uint64_t seed, const uint32_t *edges, uint64_t E,
                     int64_t *eta_def, int64_t *eta_lit, int64_t *eta_v_def, int64_t *eta_v_lit) {
    if (n == 0 || m == 0 || c == 0 || !edges || !eta_def || !eta_lit || !eta_v_def || !eta_v_lit)
        return OR_EINVAL;
    int rc = oracle_validate(n, edges, E);
    if (rc) return rc;
    const uint32_t G = (c + m - 1) / m;
    uint64_t *params = (uint64_t *)malloc(sizeof(uint64_t) * 4 * G);
    adjlist *adj = (adjlist *)calloc(n, sizeof(adjlist));
    uint32_t *slot = (uint32_t *)malloc(sizeof(uint32_t) * (E ? E : 1));
    int64_t *s_of = (int64_t *)malloc(sizeof(int64_t) * (E ? E : 1)); /* s_g, by stored index */
    int64_t *l_of = (int64_t *)malloc(sizeof(int64_t) * (E ? E : 1)); /* L_g */
    uint64_t *t_of = (uint64_t *)malloc(sizeof(uint64_t) * (E ? E : 1)); /* stream position of g */
    if (!params || !adj || !slot || !s_of || !l_of || !t_of) {
        rc = OR_ENOMEM;
        goto done;
    }
    memset(eta_def, 0, sizeof(int64_t) * c);
    memset(eta_lit, 0, sizeof(int64_t) * c);
    memset(eta_v_def, 0, sizeof(int64_t) * n);
    memset(eta_v_lit, 0, sizeof(int64_t) * n);
    oracle_hash_params(seed, G, params);
    for (uint32_t k = 0; k < G && rc == OR_OK; ++k) {
        const uint32_t ck = (k + 1 < G) ? m : c - (G - 1) * m;
        for (uint64_t t = 0; t < E; ++t) slot[t] = oracle_slot(params + 4 * k, m, edges[2 * t], edges[2 * t + 1]);
        for (uint32_t j = 0; j < ck && rc == OR_OK; ++j) {
            const uint32_t i = k * m + j;
            uint64_t mine = 0;
            for (uint64_t t = 0; t < E; ++t) mine += (slot[t] == j);
            edgeset Ei; /* E^(i): pair -> its stored index */
            if (es_init(&Ei, mine)) {
                rc = OR_ENOMEM;
                break;
            }
            uint64_t stored = 0;
            for (uint32_t x = 0; x < n; ++x) adj[x].len = 0;
            /* the semi-triangles of i, in stream order */
            for (uint64_t t = 0; t < E && rc == OR_OK; ++t) {
                const uint32_t u = edges[2 * t], v = edges[2 * t + 1];
                const adjlist *small = adj[u].len <= adj[v].len ? &adj[u] : &adj[v];
                const uint32_t other = adj[u].len <= adj[v].len ? v : u;
                int64_t closed = 0;
                for (uint32_t q = 0; q < small->len; ++q) {
                    const uint32_t w = small->nbr[q];
                    if (!es_get(&Ei, pairkey(other, w), NULL)) continue;
                    uint64_t guw = 0, gvw = 0; /* the two earlier edges of the semi-triangle (u, v, w) */
                    es_get(&Ei, pairkey(u, w), &guw);
                    es_get(&Ei, pairkey(v, w), &gvw);
                    s_of[guw] += 1;
                    s_of[gvw] += 1;
                    ++closed;
                }
                if (slot[t] == j) {
                    s_of[stored] = 0;
                    l_of[stored] = closed; /* semi-triangles of i whose last edge is (u, v) */
                    t_of[stored] = t;
                    es_put(&Ei, pairkey(u, v), stored);
                    ++stored;
                    if (adj_push(&adj[u], v) || adj_push(&adj[v], u)) rc = OR_ENOMEM;
                }
            }
            /* the sums over the stored edges of i and over their endpoints */
            for (uint64_t g = 0; g < stored && rc == OR_OK; ++g) {
                const int64_t sg = s_of[g];
                const int64_t pairs_def = sg * (sg - 1) / 2;
                const int64_t pairs_lit = sg * l_of[g] + pairs_def;
                const uint32_t gu = edges[2 * t_of[g]], gv = edges[2 * t_of[g] + 1];
                eta_def[i] += pairs_def;
                eta_lit[i] += pairs_lit;
                eta_v_def[gu] += pairs_def;
                eta_v_def[gv] += pairs_def;
                eta_v_lit[gu] += pairs_lit;
                eta_v_lit[gv] += pairs_lit;
            }
            es_free(&Ei);
        }
    }
done:
    if (adj)
        for (uint32_t x = 0; x < n; ++x) free(adj[x].nbr);
    free(adj);
    free(slot);
    free(params);
    free(s_of);
    free(l_of);
    free(t_of);
    return rc;
}

/*
 * Algorithm 2's combined estimators (Section III-B, c > m with c2 = c mod m != 0), in IEEE
 * binary64 with the operations in this order (c1 = floor(c / m), c2 = c mod m):
 *   t1  = (S1 * m) / c1                      S1: sum of tau^(i) over the first c1 m processors
 *   t2  = (S2 * m^2) / c2                    S2: sum over the last c2 processors
 *   eh  = (eta * m^3) / c                    eta: sum of eta^(i) over all processors
 *   v1  = (t1 * (m - 1)) / c1                Var(t1), tau replaced by t1
 *   v2  = (t1 * (m^2 - c2) + (2 eh) * (m - c2)) / c2
 *   tau_hat = (v2 t1 + v1 t2) / (v1 + v2), and t1 when v1 + v2 = 0 (its limit: the weight of
 *             t2 is v1, which is then 0).
 * The local estimators are the same expressions with S1_v, S2_v (the local rows of the first c1
 * groups, resp. of the last group) and eta_v.  Integer sums are exact; any sum below 0 or at or
 * above 2^53 is refused (ERANGE).  local: local_rows x n, either G group rows or c processor
 * rows (per_proc).
 */
int oracle_estimate2(uint32_t n, uint32_t m, uint32_t c, uint32_t local_rows, int per_proc,
                     const int64_t *global, const int64_t *local, int64_t eta, const int64_t *eta_v,
                     double *tau_hat, double *tau_v_hat) {
    if (n == 0 || m == 0 || c == 0 || !global || !tau_hat) return OR_EINVAL;
    const uint32_t c1 = c / m, c2 = c % m;
    if (c1 == 0 || c2 == 0) return OR_EINVAL; /* only c > m with m not dividing c */
    const int64_t lim = (int64_t)1 << 53;
    int64_t S1 = 0, S2 = 0;
    for (uint32_t i = 0; i < c; ++i) {
        int64_t *S = i < c1 * m ? &S1 : &S2;
        if (global[i] < 0 || global[i] >= lim - *S) return OR_ERANGE;
        *S += global[i];
    }
    if (eta < 0 || eta >= lim) return OR_ERANGE;
    const double dm = (double)m, dm2 = (double)((uint64_t)m * m), dm3 = (double)((uint64_t)m * m * m);
    const double dc1 = (double)c1, dc2 = (double)c2, dc = (double)c;
    const double a2 = (double)((uint64_t)m * m - c2), b2 = (double)(m - c2), dm1 = (double)(m - 1);
    {
        const double t1 = ((double)S1 * dm) / dc1, t2 = ((double)S2 * dm2) / dc2;
        const double eh = ((double)eta * dm3) / dc;
        const double v1 = (t1 * dm1) / dc1, v2 = (t1 * a2 + (2.0 * eh) * b2) / dc2;
        *tau_hat = (v1 + v2 == 0.0) ? t1 : (v2 * t1 + v1 * t2) / (v1 + v2);
    }
    if (tau_v_hat && local && eta_v) {
        const uint32_t split = per_proc ? c1 * m : c1; /* rows before the last group */
        for (uint32_t v = 0; v < n; ++v) {
            int64_t A = 0, B = 0;
            for (uint32_t r = 0; r < local_rows; ++r) {
                const int64_t x = local[(uint64_t)r * n + v];
                int64_t *S = r < split ? &A : &B;
                if (x < 0 || x >= lim - *S) return OR_ERANGE;
                *S += x;
            }
            if (eta_v[v] < 0 || eta_v[v] >= lim) return OR_ERANGE;
            const double t1 = ((double)A * dm) / dc1, t2 = ((double)B * dm2) / dc2;
            const double eh = ((double)eta_v[v] * dm3) / dc;
            const double v1 = (t1 * dm1) / dc1, v2 = (t1 * a2 + (2.0 * eh) * b2) / dc2;
            tau_v_hat[v] = (v1 + v2 == 0.0) ? t1 : (v2 * t1 + v1 * t2) / (v1 + v2);
        }
    }
    return OR_OK;
}

/* ------------------------------------------------------------------ parallel MASCOT ------ */

/*
 * Parallel MASCOT (Section III-C; MASCOT by Lim and Kang, KDD 2015): c processors, each
 * running MASCOT with edge sampling probability p = 1/m independently of the others.  For
 * every stream edge (u, v) at time t, processor i counts N = N_u^(i) intersect N_v^(i) over its
 * own sampled edges that arrived before t, adds |N| to its counter tau^(i) and to tau_u^(i),
 * tau_v^(i), and 1 to tau_w^(i) for each w in N; then it keeps (u, v) with probability p.
 * The counting step is Algorithm 1's; only the sampling differs from REPT: the processors'
 * samples overlap instead of partitioning the stream.
 *
 * The independent coin of processor i is drawn from the same hash family as REPT's groups:
 * processor i keeps edge e iff h_i(e) == 0, where h_i : E -> [0, m) has the coefficients of
 * group i (SplitMix64 outputs 4i..4i+3 of `seed`).  So P(keep) = 1/m, and different processors
 * use independent hash functions (one group each).
 * Outputs (overwritten): global[i] = tau^(i) (c entries); local[i*n + v] = tau_v^(i).
 */
int oracle_mascot(uint32_t n, uint32_t m, uint32_t c, uint64_t seed, const uint32_t *edges, uint64_t E,
                  int64_t *global, int64_t *local) {
    if (n == 0 || m == 0 || c == 0 || !edges || !global || !local) return OR_EINVAL;
    int rc = oracle_validate(n, edges, E);
    if (rc) return rc;
    uint64_t *params = (uint64_t *)malloc(sizeof(uint64_t) * 4 * c);
    adjlist *adj = (adjlist *)calloc(n, sizeof(adjlist));
    uint8_t *keep = (uint8_t *)malloc(E ? E : 1);
    if (!params || !adj || !keep) {
        rc = OR_ENOMEM;
        goto done;
    }
    memset(global, 0, sizeof(int64_t) * c);
    memset(local, 0, sizeof(int64_t) * (uint64_t)c * n);
    oracle_hash_params(seed, c, params);
    for (uint32_t i = 0; i < c && rc == OR_OK; ++i) {
        uint64_t kept = 0;
        for (uint64_t t = 0; t < E; ++t) {
            keep[t] = oracle_slot(params + 4 * i, m, edges[2 * t], edges[2 * t + 1]) == 0;
            kept += keep[t];
        }
        edgeset Si; /* the sample of processor i */
        if (es_init(&Si, kept)) {
            rc = OR_ENOMEM;
            break;
        }
        int64_t *loc = local + (uint64_t)i * n;
        for (uint32_t x = 0; x < n; ++x) adj[x].len = 0;
        for (uint64_t t = 0; t < E; ++t) {
            const uint32_t u = edges[2 * t], v = edges[2 * t + 1];
            const adjlist *small = adj[u].len <= adj[v].len ? &adj[u] : &adj[v];
            const uint32_t other = adj[u].len <= adj[v].len ? v : u;
            int64_t cnt = 0;
            for (uint32_t q = 0; q < small->len; ++q) {
                const uint32_t w = small->nbr[q];
                if (es_get(&Si, pairkey(other, w), NULL)) {
                    ++cnt;
                    loc[w] += 1;
                }
            }
            global[i] += cnt;
            loc[u] += cnt;
            loc[v] += cnt;
            if (keep[t]) {
                es_put(&Si, pairkey(u, v), t);
                if (adj_push(&adj[u], v) || adj_push(&adj[v], u)) {
                    rc = OR_ENOMEM;
                    break;
                }
            }
        }
        es_free(&Si);
    }
done:
    if (adj)
        for (uint32_t x = 0; x < n; ++x) free(adj[x].nbr);
    free(adj);
    free(keep);
    free(params);
    return rc;
}

/*
 * Parallel MASCOT's estimators: each processor's estimate is m^2 tau^(i) (MASCOT scales a
 * counted triangle by 1/p^2), and the parallel estimate is their mean,
 *   tau_hat = ((double)S * (double)(m*m)) / (double)c,   S = sum_i tau^(i),
 * and per node with S_v = sum_i tau_v^(i) (local: c rows of n); binary64, one rounding for
 * the product and one for the quotient; a sum below 0 or at or above 2^53 is ERANGE.
 */
int oracle_estimate_mascot(uint32_t n, uint32_t m, uint32_t c, const int64_t *global, const int64_t *local,
                           double *tau_hat, double *tau_v_hat) {
    if (n == 0 || m == 0 || c == 0 || !global || !tau_hat) return OR_EINVAL;
    const int64_t lim = (int64_t)1 << 53;
    const double num = (double)((uint64_t)m * m), den = (double)c;
    int64_t S = 0;
    for (uint32_t i = 0; i < c; ++i) {
        if (global[i] < 0 || global[i] >= lim - S) return OR_ERANGE;
        S += global[i];
    }
    if (tau_v_hat && local) {
        for (uint32_t v = 0; v < n; ++v) {
            int64_t Sv = 0;
            for (uint32_t i = 0; i < c; ++i) {
                const int64_t x = local[(uint64_t)i * n + v];
                if (x < 0 || x >= lim - Sv) return OR_ERANGE;
                Sv += x;
            }
            tau_v_hat[v] = ((double)Sv * num) / den;
        }
    }
    *tau_hat = ((double)S * num) / den;
    return OR_OK;
}
