// C ABI of the REPT counting library (declarations and contracts in include/rept.h).
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <condition_variable>
#include <functional>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "common.h"

namespace {

// SplitMix64 (Steele, Lea, Flood, OOPSLA 2014): Weyl-sequence state, two multiply/xor-shift
// mixing rounds.  Group k's hash coefficients a_0..a_3 are outputs 4k..4k+3 from state `seed`,
// each shifted right by 3 and reduced modulo the Mersenne prime 2^61 - 1.
struct SplitMix64 {
    uint64_t s;
    uint64_t next() {
        s += 0x9e3779b97f4a7c15ULL;
        uint64_t z = s;
        z ^= z >> 30;
        z *= 0xbf58476d1ce4e5b9ULL;
        z ^= z >> 27;
        z *= 0x94d049bb133111ebULL;
        return z ^ (z >> 31);
    }
};

// the coefficients of groups k0 .. k0 + G - 1: SplitMix64 outputs 4 k0 .. 4 (k0 + G) - 1
void group_params(uint64_t seed, uint32_t G, uint64_t* hp, uint32_t k0 = 0) {
    const uint64_t p61 = (1ull << 61) - 1;
    SplitMix64 r{seed};
    for (uint64_t q = 0; q < 4ull * k0; ++q) (void)r.next();
    for (uint32_t q = 0; q < 4 * G; ++q) {
        uint64_t v = r.next() >> 3;  // < 2^61 = p61 + 1
        hp[q] = v == p61 ? 0 : v;
    }
}

bool params_ok(const rept_params* p) {
    if (!p || p->m == 0 || p->c == 0 || p->reserved != 0) return false;
    if (p->flags & ~(REPT_LOCAL_PER_PROC | REPT_MASCOT)) return false;
    return true;
}

bool is_mascot(const rept_params* p) { return (p->flags & REPT_MASCOT) != 0; }

// hash groups: ceil(c/m) for REPT; one per processor for parallel MASCOT
uint32_t groups_of(const rept_params* p) { return is_mascot(p) ? p->c : (p->c + p->m - 1) / p->m; }

// 16-bit words per stored edge in the slot table: one slot per group (padded to 1, 2, 4, 8),
// or for parallel MASCOT one keep mask (bit k: processor k keeps the edge)
uint32_t table_stride(const rept_params* p) { return is_mascot(p) ? 1u : rept_slot_stride(groups_of(p)); }

// bytes of the slot table of a graph's stored edges
size_t table_bytes(const rept_graph* g, const rept_params* p) {
    const size_t b = (size_t)g->E * table_stride(p) * sizeof(uint16_t);
    return b < 256 ? 256 : (b + 255) & ~(size_t)255;
}

struct Shape {
    BatchHeader hdr;
};
std::mutex g_mu;
std::unordered_map<void*, Shape> g_shapes;  // prepared batch workspaces -> launch shape

bool valid_graph(const rept_graph* g) { return g && g->magic == REPT_MAGIC; }

// ---- incremental streams: host handle and the layout of the caller's buffer ---------------
constexpr uint32_t REPT_STREAM_MAGIC = 0x52535452u;
}  // namespace
struct rept_stream {
    uint32_t magic;
    rept_params params;
    uint64_t capacity, max_chunk;
    IncState st;
    IncCount base;  // parameters of the per-edge count (pointers filled per append)
    // the windowed recount: the stream in arrival order, and the regions a build of the prefix
    // and its count use (sized for `capacity` edges)
    uint32_t* eall;
    void *gpers, *gscr, *gws;
    size_t gpers_bytes, gscr_bytes, gws_bytes;
    uint32_t policy;
    uint64_t n_per_edge, n_recount;  // appends counted by each path
};
namespace {
bool valid_stream(const rept_stream* s) { return s && s->magic == REPT_STREAM_MAGIC; }

// The per-edge count of an append costs about one binary search per work item (the chunk's total
// of min(d_u, d_v) over its edges at the chunk's end); the windowed recount, a build and a count
// of the whole prefix.  On the 1M/20M power-law stream in ten appends the first took 4.4e-11 s
// per item and the second 4.5e-10 s per prefix edge, so the recount is taken when the items
// exceed 10 per prefix edge.
constexpr uint64_t kRecountItemsPerEdge = 10;

// Count the edges at times [t0, t1) of the stream appended so far by the one-shot path: build
// the prefix [0, t1) into the handle's reserved regions, then add the window's per-edge updates
// to the handle's counters (rept_count_range: a triangle belongs to the window of its last edge,
// so this equals Algorithm 1's updates of those edges).  ENOMEM if the prefix needs more than was
// reserved (the caller then counts edge by edge).
rept_status recount_window(rept_stream* h, uint64_t t0, uint64_t t1, hipStream_t s) {
    size_t pb = 0, sb = 0;
    rept_status st = rept_query_sizes(h->st.n, t1, &pb, &sb);
    if (st != REPT_OK) return st;
    if (pb > h->gpers_bytes || sb > h->gscr_bytes) return REPT_ENOMEM;
    rept_graph* g = nullptr;
    st = rept_build(h->st.n, h->eall, t1, h->gpers, h->gpers_bytes, h->gscr, h->gscr_bytes, s, &g);
    if (st != REPT_OK) return st;
    size_t wb = 0;
    st = rept_count_workspace_size(g, &h->params, &wb);
    if (st == REPT_OK && wb > h->gws_bytes) st = REPT_ENOMEM;
    if (st == REPT_OK)
        st = rept_count_range(g, &h->params, t0, t1, h->base.global, h->base.local, h->gws, h->gws_bytes, s);
    rept_destroy(g);
    return st;
}

struct IncLayout {
    size_t key[2], tim[2], off, coff, ckey_a, ckey_b, ctim_a, ctim_b, end, flags, temp, total, temp_bytes;
    size_t eall, gpers, gscr, gws, gpers_bytes, gscr_bytes, gws_bytes;
};
size_t up256(size_t x) { return (x + 255) & ~(size_t)255; }
IncLayout inc_layout(uint32_t n, uint64_t cap, uint64_t maxc) {
    IncLayout L;
    const size_t E2 = 2 * cap, C2 = 2 * maxc;
    size_t p = 0;
    for (int i = 0; i < 2; ++i) {
        L.key[i] = p; p = up256(p + 8 * E2);
        L.tim[i] = p; p = up256(p + 4 * E2);
    }
    L.off = p; p = up256(p + 4 * ((size_t)n + 1));
    L.coff = p; p = up256(p + 4 * ((size_t)n + 1));
    L.ckey_a = p; p = up256(p + 8 * C2);
    L.ckey_b = p; p = up256(p + 8 * C2);
    L.ctim_a = p; p = up256(p + 4 * C2);
    L.ctim_b = p; p = up256(p + 4 * C2);
    L.end = p; p = up256(p + 8 * C2);
    L.flags = p; p = up256(p + 8);
    L.temp_bytes = rept_inc_sort_temp_bytes(C2, 64);
    L.temp = p; p = up256(p + L.temp_bytes);
    // the windowed recount: the stream in arrival order, a built graph of up to `cap` edges with
    // its build scratch, and the slot table of its count (at most 8 groups: 16 bytes per edge)
    L.gpers_bytes = L.gscr_bytes = 0;
    if (rept_query_sizes(n, cap, &L.gpers_bytes, &L.gscr_bytes) != REPT_OK) L.temp_bytes = 0;  // reported as EDEVICE
    L.gws_bytes = up256(16 * (size_t)cap);
    L.eall = p; p = up256(p + 8 * (size_t)cap);
    L.gpers = p; p = up256(p + L.gpers_bytes);
    L.gscr = p; p = up256(p + L.gscr_bytes);
    L.gws = p; p = up256(p + L.gws_bytes);
    L.total = p;
    return L;
}
uint32_t bit_length(uint32_t x) { return x ? 32u - (uint32_t)__builtin_clz(x) : 0u; }

// Fill the launch shape for jobs of at most G_max groups, at most c_max processors and at most
// max_out entries in an apex list.
rept_status make_header(uint32_t njobs, uint32_t G_max, uint32_t gs_max, uint32_t c_max, uint32_t max_out,
                        uint64_t zero_words, bool any_zero, const rept_tuning* tu, BatchHeader* h, bool eta = false) {
    memset(h, 0, sizeof(*h));
    const uint32_t cus = rept_num_cus() ? rept_num_cus() : 256;
    uint32_t fit = 64;
    // one W chunk per unit up to 2048 entries: re-walking a unit's B lists per extra chunk
    // costs more than the occupancy a smaller table would buy (R-MAT scale 24, largest list
    // 1761, 256-thread workgroups: 322 ms at 2048, 338 at 1024, 450 at 512; 559 at 4096, one
    // workgroup per CU)
    while (fit < max_out && fit < 2048) fit <<= 1;
    const bool own_block_cap = tu && tu->block_cap, own_b_chunk = tu && tu->b_chunk;
    uint32_t block_cap = own_block_cap ? tu->block_cap : fit;
    // Lists of more than 1024 entries: one workgroup of 1024 threads per compute unit (16 waves),
    // one 2048-entry table chunk (no second walk of a unit's B lists below 2048 entries),
    // 1024-list B chunks, and units of up to 256 entries left to single wavefronts, taken 16 at a
    // time (R-MAT scale 24, longest list 1761: 198 ms with units of up to 128 entries on
    // wavefronts, 210 with up to 64; 274 with 512-thread workgroups, 1024-entry table chunks and
    // 256-list B chunks, two workgroups per compute unit; 206 with 512-list B chunks.  With the
    // four-slot heavy tables below: 179.9 ms at 128, 176.4 at 256, 175.6 at 256 with 16-unit
    // light tiles).  Shorter lists keep 256-thread workgroups (the 1M/20M power-law graph,
    // longest list 480: 5.99 ms; 8.5-10.8 with 1024 threads).
    const bool wide = !own_block_cap && block_cap >= 2048 && !(tu && tu->threads);
    const bool own_wave_cap = tu && tu->wave_cap;
    uint32_t wave_cap = own_wave_cap ? tu->wave_cap : (wide ? 256u : 64u);
    // units with long lists also have many lists to walk: bigger B chunks pay there, not on
    // shorter lists (the 1M/20M power-law graph: 6.64 ms at 128, 7.13 at 64, 7.41 at 256)
    uint32_t b_chunk = own_b_chunk ? tu->b_chunk : (wide ? 1024u : (block_cap >= 2048 ? 512u : 128u));
    const uint32_t threads = (tu && tu->threads) ? tu->threads : (wide ? 1024u : 256u);
    const uint32_t light_tile = (tu && tu->light_tile) ? tu->light_tile : (wide ? 16u : 8u);
    if (wave_cap < 8 || wave_cap > 256) return REPT_EINVAL;
    if (block_cap < 64 || block_cap > 4096) return REPT_EINVAL;
    if (b_chunk < 16 || b_chunk > 1024) return REPT_EINVAL;
    if (threads < 64 || threads > 1024 || threads % 64) return REPT_EINVAL;
    if (light_tile < 1 || light_tile > 64) return REPT_EINVAL;  // one unit per lane of a wavefront
    const uint32_t pl = tu ? tu->phase_launches : 0u;
    if (pl > 3 || (tu && tu->reserved)) return REPT_EINVAL;
    // default (0): the light phase in a launch of its own, on a second stream
    const bool split = pl != 1;
    // A light launch of its own needs no heavy team area, and a heavy launch then needs no light
    // areas.  It keeps the heavy launch's workgroup size, except with the wide shape below.
    uint32_t light_threads = threads;
    const uint32_t hist_c = c_max <= REPT_HIST_CAP ? c_max : 0;
    // the light phase's hash tables are sparser (fewer probes) where the LDS budget allows
    uint32_t light_table = 4, heavy_table = 2;
    // a light wavefront stages its lists to walk in chunks of light_b (at most wave_cap)
    uint32_t light_b = wave_cap;
    // The wide shape's light launch (units of up to 256 entries): 256-thread workgroups with
    // two-slot tables and 128-list chunks, so that three fit a CU (12 waves); four-slot tables
    // and 256-list chunks fit two (R-MAT scale 24: 169.8 against 175.9 ms; 64-list chunks 170.3)
    if (split && wide) {
        light_threads = 256;
        light_table = 2;
        light_b = wave_cap < 128 ? wave_cap : 128u;
    }
    auto heavy_lds = [&]() {  // the launch that runs the heavy phase (both phases if not split)
        return rept_count_lds(threads, wave_cap, block_cap, b_chunk, G_max, gs_max, hist_c, light_table,
                              heavy_table, light_b, eta, true, !split);
    };
    auto light_lds = [&]() {  // the light areas alone, in the launch that holds them
        return rept_count_lds(split ? light_threads : threads, wave_cap, block_cap, b_chunk, G_max, gs_max, hist_c,
                              light_table, heavy_table, light_b, eta, false, true);
    };
    // Past the 160 KB of a CU (static LDS takes a few bytes more), the light areas shrink first
    // (sparser tables, then a default wave cap halved down to 64), then the default heavy chunk
    // sizes.  A shape the caller chose is never changed: it is refused if it does not fit.
    const uint32_t cap = 160 * 1024 - 256;
    while (light_lds() > cap) {
        if (light_table == 4) {
            light_table = 2;
        } else if (!own_wave_cap && wave_cap > 64) {
            wave_cap >>= 1;
            light_b = light_b < wave_cap ? light_b : wave_cap;
        } else {
            return REPT_EINVAL;
        }
    }
    // default chunks keep two workgroups per CU where they can (down to 128 lists, 1024 entries);
    // a 1024-thread workgroup has a compute unit to itself anyway
    while (threads <= 512 && heavy_lds() > 80 * 1024 - 256 &&
           ((!own_b_chunk && b_chunk > 128) || (!own_block_cap && block_cap > 1024))) {
        if (!own_b_chunk && b_chunk > 128) b_chunk >>= 1;
        else block_cap >>= 1;
    }
    while (heavy_lds() > cap) {
        if (!own_b_chunk && b_chunk > 128) b_chunk >>= 1;
        else if (!own_block_cap && block_cap > 64) block_cap >>= 1;
        else return REPT_EINVAL;
    }
    auto resident = [&](uint32_t bytes) {  // workgroups per CU, as the default grid counts them
        uint32_t per_cu = rept_count_blocks_per_cu(threads, bytes, eta);
        if (per_cu == 0) per_cu = 1;
        return per_cu > 4 ? 4u : per_cu;
    };
    // Sparser heavy tables (four slots per key: fewer probes past the first bucket) with the wide
    // shape, where they fit and cost no resident workgroup (R-MAT scale 24, one 1024-thread
    // workgroup per CU either way: 179 against 198 ms).  Shorter lists keep two: on the 1M/20M
    // power-law graph four slots would drop REPT's default launch from four workgroups per CU to
    // three (7.04 against 5.99 ms), and where they keep the occupancy they cost MASCOT with eight
    // processors 9.8 against 8.0 ms, for 4.9 against 5.1 ms for REPT with the same m and c.
    if (wide) {
        const uint32_t per_cu2 = resident(heavy_lds());
        heavy_table = 4;
        const uint32_t lds4 = heavy_lds();
        if (lds4 > cap || resident(lds4) < per_cu2) heavy_table = 2;
    }
    const uint32_t lds = heavy_lds();
    uint32_t blocks = tu ? tu->blocks : 0;
    if (!blocks) blocks = resident(lds) * cus;
    h->njobs = njobs;
    h->wave_cap = wave_cap;
    h->block_cap = block_cap;
    h->b_chunk = b_chunk;
    h->blocks = blocks;
    h->threads = threads;
    h->light_tile = light_tile;
    h->hist_c = hist_c;
    h->G_max = G_max;
    h->gs_max = gs_max;
    h->lds_bytes = lds;
    h->light_table = light_table;
    h->heavy_table = heavy_table;
    h->light_b = light_b;
    h->any_zero = any_zero ? 1u : 0u;
    h->any_eta = eta ? 1u : 0u;
    h->zero_words = zero_words;
    h->split = split ? 1u : 0u;
    h->split_streams = (pl == 0 || pl == 3) ? 1u : 0u;
    if (h->split) {
        h->light_threads = light_threads;
        h->light_lds = light_lds();
        uint32_t per_cu = rept_count_blocks_per_cu(light_threads, h->light_lds, eta);
        if (per_cu == 0) per_cu = 1;
        if (per_cu > 8) per_cu = 8;
        h->light_blocks = (tu && tu->blocks) ? tu->blocks : per_cu * cus;
    }
    return REPT_OK;
}

rept_status make_job(const rept_job& jb, JobDev* d, uint64_t* zero_words) {
    const rept_graph* g = jb.graph;
    if (!valid_graph(g) || !params_ok(&jb.params) || !jb.global || !jb.local) return REPT_EINVAL;
    if (jb.flags & ~(REPT_JOB_ACCUMULATE | REPT_JOB_TABLE_READY)) return REPT_EINVAL;
    const uint32_t G = groups_of(&jb.params);
    if (G > REPT_GMAX || jb.params.m > 65536) return REPT_ENOTSUP;  // slots are staged as 16-bit
    if (!jb.workspace || ((uintptr_t)jb.workspace & 255u)) return REPT_EINVAL;
    if (jb.workspace_bytes < table_bytes(g, &jb.params)) return REPT_ENOMEM;
    memset(d, 0, sizeof(*d));
    d->off = g->off;
    d->nbr = g->nbr;
    d->tim = g->tim;
    d->apex = g->apex;
    d->roff = g->roff;
    d->rrec = g->rrec;
    d->rpos = g->rpos;
    d->global = jb.global;
    d->local = jb.local;
    group_params(jb.params.seed, G, d->hp);
    d->n = g->n;
    d->m = jb.params.m;
    d->c = jb.params.c;
    d->G = G;
    // processor of slot j of group k: k * pstride + j for the slots j < ck (last group: last_ck)
    if (is_mascot(&jb.params)) {
        d->ck = d->last_ck = 1;  // processor k keeps the edges with h_k(e) = 0
        d->pstride = 1;
    } else {
        d->ck = jb.params.m;
        d->last_ck = jb.params.c - (G - 1) * jb.params.m;
        d->pstride = jb.params.m;
    }
    d->per_proc = (jb.params.flags & REPT_LOCAL_PER_PROC) ? 1u : 0u;
    d->rows = d->per_proc ? jb.params.c : G;
    d->accumulate = (jb.flags & REPT_JOB_ACCUMULATE) ? 1u : 0u;
    const uint64_t t1 = jb.t1 > g->E ? g->E : jb.t1;
    if (jb.t0 > t1) return REPT_EINVAL;
    d->t0 = (uint32_t)jb.t0;
    d->t1 = (uint32_t)t1;
    const uint32_t u1 = jb.unit1 > g->num_apex ? g->num_apex : jb.unit1;
    if (jb.unit0 > u1) return REPT_EINVAL;
    d->unit0 = jb.unit0;
    d->unit1 = u1;
    d->gs = table_stride(&jb.params);
    d->mask = is_mascot(&jb.params) ? 1u : 0u;
    d->tab = (uint16_t*)jb.workspace;
    d->fill = (jb.flags & REPT_JOB_TABLE_READY) ? 0u : 1u;
    *zero_words = (uint64_t)d->c + (uint64_t)d->rows * d->n;
    return REPT_OK;
}

// One counting pass.  More than REPT_GMAX groups run as successive launches of at most that
// many (groups are independent): launch q counts groups 8q .. 8q + 7 with their own hash
// coefficients into its slice of the outputs, so the results equal one launch over all groups.
rept_status count_one(const rept_graph* graph, const rept_params* params, uint64_t t0, uint64_t t1,
                      bool accumulate, int64_t* global, int64_t* local, void* workspace, size_t workspace_bytes,
                      void* stream, const rept_tuning* tuning = nullptr) {
    if (!valid_graph(graph) || !params_ok(params) || !global || !local) return REPT_EINVAL;
    if (t0 > t1 || t1 > graph->E) return REPT_EINVAL;
    if (params->m > 65536) return REPT_ENOTSUP;
    const uint32_t G = groups_of(params), m = params->m, n = graph->n;
    const bool mascot = is_mascot(params), per_proc = (params->flags & REPT_LOCAL_PER_PROC) != 0;
    // every pass's arguments are checked (check = 0) before the first launch (check = 1)
    const uint32_t passes = (G + REPT_GMAX - 1) / REPT_GMAX;
    for (uint32_t check = 0; check < 2; ++check) {
        for (uint32_t q = 0; q < passes; ++q) {
            const uint32_t k0 = q * REPT_GMAX, Gq = (G - k0) < REPT_GMAX ? (G - k0) : REPT_GMAX;
            rept_params pp = *params;
            uint64_t goff, loff;
            if (mascot) {  // processors k0 .. k0 + Gq - 1, one group and one local row each
                pp.c = Gq;
                goff = k0;
                loff = (uint64_t)k0 * n;
            } else {  // the groups' processors k0 m .. ; the last group may be partial
                const uint64_t left = (uint64_t)params->c - (uint64_t)k0 * m;
                pp.c = (uint32_t)(left < (uint64_t)Gq * m ? left : (uint64_t)Gq * m);
                goff = (uint64_t)k0 * m;
                loff = per_proc ? (uint64_t)k0 * m * n : (uint64_t)k0 * n;
            }
            rept_job jb;
            memset(&jb, 0, sizeof(jb));
            jb.graph = graph;
            jb.params = pp;
            jb.global = global + goff;
            jb.local = local + loff;
            jb.t0 = t0;
            jb.t1 = t1;
            jb.unit0 = 0;
            jb.unit1 = UINT32_MAX;
            jb.flags = accumulate ? REPT_JOB_ACCUMULATE : 0u;
            jb.workspace = workspace;
            jb.workspace_bytes = workspace_bytes;
            JobDev dq;
            uint64_t zw = 0;
            rept_status st = make_job(jb, &dq, &zw);
            if (st != REPT_OK) return st;
            group_params(params->seed, dq.G, dq.hp, k0);  // this pass's groups of the whole seed
            BatchHeader h;
            st = make_header(1, dq.G, dq.gs, dq.c, graph->max_out, zw, !accumulate, tuning, &h);
            if (st != REPT_OK) return st;
            if (!check) continue;
            h.any_fill = 1;
            h.fill_edges = graph->E > UINT32_MAX ? UINT32_MAX : (uint32_t)graph->E;
            if (rept_launch_single(graph->ctrl, h, dq, (hipStream_t)stream) != hipSuccess) return REPT_EDEVICE;
        }
    }
    return REPT_OK;
}

}  // namespace

uint32_t rept_num_cus() {
    static int cached_dev = -1;
    static uint32_t cached = 0;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (dev != cached_dev) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
        cached = (uint32_t)v;
        cached_dev = dev;
    }
    return cached;
}

extern "C" {

uint32_t rept_local_rows(const rept_params* p) {
    if (!params_ok(p)) return 0;
    return ((p->flags & REPT_LOCAL_PER_PROC) || is_mascot(p)) ? p->c : groups_of(p);
}

rept_status rept_query_sizes(uint32_t n, uint64_t num_edges, size_t* persistent_bytes, size_t* scratch_bytes) {
    if (n == 0 || n > (1u << 29) || num_edges >= (1ull << 31) || !persistent_bytes || !scratch_bytes)
        return REPT_EINVAL;
    rept_sizes_impl(n, num_edges, persistent_bytes, scratch_bytes);
    return REPT_OK;
}

rept_status rept_build(uint32_t n, const uint32_t* edges, uint64_t num_edges, void* persistent,
                       size_t persistent_bytes, void* scratch, size_t scratch_bytes, void* stream,
                       rept_graph** out) {
    if (!out || n == 0 || n > (1u << 29) || num_edges >= (1ull << 31) || !persistent || !scratch)
        return REPT_EINVAL;
    if (num_edges > 0 && !edges) return REPT_EINVAL;
    if (((uintptr_t)edges & 7u) || ((uintptr_t)persistent & 255u) || ((uintptr_t)scratch & 255u))
        return REPT_EINVAL;
    return rept_build_impl(n, edges, num_edges, persistent, persistent_bytes, scratch, scratch_bytes,
                           (hipStream_t)stream, out);
}

rept_status rept_build_host(uint32_t n, const uint32_t* host_edges, uint64_t num_edges, void* persistent,
                            size_t persistent_bytes, void* scratch, size_t scratch_bytes, void* stream,
                            rept_graph** out) {
    if (!out || n == 0 || n > (1u << 29) || num_edges >= (1ull << 31) || !persistent || !scratch)
        return REPT_EINVAL;
    if (num_edges > 0 && !host_edges) return REPT_EINVAL;
    if (((uintptr_t)persistent & 255u) || ((uintptr_t)scratch & 255u)) return REPT_EINVAL;
    size_t pb = 0, sb = 0;
    rept_sizes_impl(n, num_edges, &pb, &sb);
    if (persistent_bytes < pb || scratch_bytes < sb) return REPT_ENOMEM;
    uint32_t* staged = (uint32_t*)((uint8_t*)persistent + rept_host_stage_offset(n, num_edges));
    if (num_edges > 0 && hipMemcpyAsync(staged, host_edges, (size_t)num_edges * 8, hipMemcpyHostToDevice,
                                        (hipStream_t)stream) != hipSuccess)
        return REPT_EDEVICE;
    return rept_build_impl(n, staged, num_edges, persistent, persistent_bytes, scratch, scratch_bytes,
                           (hipStream_t)stream, out);
}

rept_status rept_graph_get_info(const rept_graph* g, rept_graph_info* info) {
    if (!valid_graph(g) || !info) return REPT_EINVAL;
    info->n = g->n;
    info->num_edges = g->E;
    info->num_apex = g->num_apex;
    info->max_out_degree = g->max_out;
    info->oriented_work = g->work;
    info->sum_out_sq = g->sum_out_sq;
    info->num_reverse = g->num_rev;
    return REPT_OK;
}

rept_status rept_count_workspace_size(const rept_graph* graph, const rept_params* params, size_t* bytes) {
    if (!valid_graph(graph) || !params_ok(params) || !bytes) return REPT_EINVAL;
    if (params->m > 65536) return REPT_ENOTSUP;  // more than 8 groups: the table of one launch
    *bytes = table_bytes(graph, params);
    return REPT_OK;
}

rept_status rept_count(const rept_graph* graph, const rept_params* params, int64_t* global, int64_t* local,
                       void* workspace, size_t workspace_bytes, void* stream) {
    if (!valid_graph(graph)) return REPT_EINVAL;
    return count_one(graph, params, 0, graph->E, false, global, local, workspace, workspace_bytes, stream);
}

rept_status rept_count_range(const rept_graph* graph, const rept_params* params, uint64_t t0, uint64_t t1,
                             int64_t* global, int64_t* local, void* workspace, size_t workspace_bytes,
                             void* stream) {
    return count_one(graph, params, t0, t1, true, global, local, workspace, workspace_bytes, stream);
}

}  // extern "C"

// ---- the allocation-free count: the slot table in a static device array -------------------
// The array below is a host-side stand-in in host code; its device address is taken once per
// device with hipGetSymbolAddress (with that device current) and only that address is used.
static __device__ __align__(256) uint8_t scratch[REPT_NOALLOC_SCRATCH_BYTES];

namespace {
std::mutex g_scratch_mu;
void* g_scratch_ptr[64] = {};  // per device: the device address of `scratch`, once taken

// the device address of this device's `scratch`, taken on the first call on the device
rept_status scratch_for_current(void** out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return REPT_EDEVICE;
    if (dev < 0 || dev >= 64) return REPT_EDEVICE;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return REPT_EDEVICE;
        }
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return REPT_OK;
}
}  // namespace

extern "C" {

rept_status rept_count_noalloc(const rept_graph* graph, const rept_params* params, int64_t* global, int64_t* local,
                               void* stream) {
    if (!valid_graph(graph) || !params_ok(params) || !global || !local) return REPT_EINVAL;
    if (params->m > 65536) return REPT_ENOTSUP;
    if (table_bytes(graph, params) > (size_t)REPT_NOALLOC_SCRATCH_BYTES) return REPT_ENOMEM;
    void* ws = nullptr;
    const rept_status st = scratch_for_current(&ws);
    if (st != REPT_OK) return st;
    // both phases in one launch on `stream`: no second stream or event is created
    rept_tuning one{};
    one.phase_launches = 1;
    return count_one(graph, params, 0, graph->E, false, global, local, ws, (size_t)REPT_NOALLOC_SCRATCH_BYTES, stream,
                     &one);
}

namespace {

// Host workers for the estimators: started on first use and kept for the life of the process
// (idle workers wait on a condition variable), so a call pays no thread start-up.  The pool is
// never destroyed: threads still waiting at exit end with the process.
class HostPool {
   public:
    static HostPool& get() {
        static HostPool* pool = new HostPool();
        return *pool;
    }
    uint32_t threads() const { return (uint32_t)workers_.size() + 1; }
    // fn(k) for every k in [0, parts), on the workers and the calling thread; returns when all
    // parts are done.  One job runs at a time.
    void run(uint32_t parts, const std::function<void(uint32_t)>& fn) {
        std::lock_guard<std::mutex> one(call_);
        if (workers_.empty() || parts <= 1) {
            for (uint32_t k = 0; k < parts; ++k) fn(k);
            return;
        }
        {
            std::lock_guard<std::mutex> lk(mu_);
            fn_ = &fn;
            parts_ = parts;
            next_ = 0;
            active_ = (uint32_t)workers_.size();
            ++gen_;
        }
        start_.notify_all();
        for (uint32_t k; (k = next_.fetch_add(1)) < parts;) fn(k);
        std::unique_lock<std::mutex> lk(mu_);
        done_.wait(lk, [&] { return active_ == 0; });
        fn_ = nullptr;
    }

   private:
    HostPool() {
        const uint32_t hw = std::max(1u, std::thread::hardware_concurrency());
        const uint32_t total = std::min(16u, hw);
        for (uint32_t i = 1; i < total; ++i) workers_.emplace_back([this] { work(); });
    }
    void work() {
        uint64_t seen = 0;
        for (;;) {
            const std::function<void(uint32_t)>* fn;
            uint32_t parts;
            {
                std::unique_lock<std::mutex> lk(mu_);
                start_.wait(lk, [&] { return gen_ != seen; });
                seen = gen_;
                fn = fn_;
                parts = parts_;
            }
            for (uint32_t k; (k = next_.fetch_add(1)) < parts;) (*fn)(k);
            std::lock_guard<std::mutex> lk(mu_);
            if (--active_ == 0) done_.notify_one();
        }
    }
    std::vector<std::thread> workers_;
    std::mutex call_, mu_;
    std::condition_variable start_, done_;
    const std::function<void(uint32_t)>* fn_ = nullptr;
    uint32_t parts_ = 0, active_ = 0;
    std::atomic<uint32_t> next_{0};
    uint64_t gen_ = 0;
};

// The estimators' common part.  S = sum of global (exact int64), tau_hat = RN(RN(S m^2) / c);
// with `local` (rows x n, row stride n) and tau_v_hat: S_v = sum over the rows at v (exact),
// tau_v_hat[v] = RN(RN(S_v m^2) / c).  Every sum is checked before any output is written (a
// first pass over the node ranges only validates; the second writes), so an error return
// leaves tau_hat and tau_v_hat untouched.  Node ranges are independent and run on the host pool.
rept_status estimate_core(uint32_t n, const rept_params* params, const int64_t* global, const int64_t* local,
                          uint32_t rows, double* tau_hat, double* tau_v_hat) {
    if (!params_ok(params) || n == 0 || !global || !tau_hat) return REPT_EINVAL;
    const uint32_t m = params->m, c = params->c;
    if (c > m && c % m != 0 && !is_mascot(params)) return REPT_ENOTSUP;
    const int64_t limit = (int64_t)1 << 53;
    const double num = (double)((uint64_t)m * (uint64_t)m);
    const double den = (double)c;
    int64_t S = 0;
    for (uint32_t i = 0; i < c; ++i) {
        const int64_t x = global[i];
        if (x < 0 || x >= limit - S) return REPT_ERANGE;
        S += x;
    }
    double* tv = tau_v_hat;
    if (tv && local) {
        std::atomic<bool> bad{false};
        constexpr uint32_t kPart = 32768;  // nodes per part of the node range
        const uint32_t parts = (uint32_t)(((uint64_t)n + kPart - 1) / kPart);
        // write = false: only check that every node's sum is in [0, 2^53); true: write the estimates
        bool write = false;
        const std::function<void(uint32_t)> part = [&](uint32_t k) {
            const uint32_t v0 = k * kPart, v1 = std::min<uint64_t>((uint64_t)v0 + kPart, n);
            constexpr uint32_t kBlock = 4096;  // nodes per pass, kept in a stack buffer
            int64_t acc[kBlock];
            for (uint32_t b0 = v0; b0 < v1; b0 += kBlock) {
                const uint32_t b1 = std::min(v1, b0 + kBlock), nb = b1 - b0;
                bool ok = true;
                for (uint32_t i = 0; i < nb; ++i) {
                    const int64_t x = local[b0 + i];
                    ok &= x >= 0 && x < limit;
                    acc[i] = x;
                }
                for (uint32_t r = 1; r < rows; ++r) {
                    const int64_t* row = local + (uint64_t)r * n + b0;
                    for (uint32_t i = 0; i < nb; ++i) {
                        const int64_t x = row[i];
                        ok &= x >= 0 && x < limit - acc[i];
                        acc[i] += ok ? x : 0;
                    }
                }
                if (!ok) {
                    bad = true;
                    return;
                }
                if (!write) continue;
                for (uint32_t i = 0; i < nb; ++i) {
                    const double prod = (double)acc[i] * num;
                    tv[b0 + i] = prod / den;
                }
            }
        };
        HostPool::get().run(parts, part);
        if (bad) return REPT_ERANGE;
        write = true;
        HostPool::get().run(parts, part);
    }
    const double prod = (double)S * num;
    *tau_hat = prod / den;
    return REPT_OK;
}

}  // namespace

rept_status rept_estimate(uint32_t n, const rept_params* params, const int64_t* global, const int64_t* local,
                          double* tau_hat, double* tau_v_hat) {
    if (!params_ok(params)) return REPT_EINVAL;
    return estimate_core(n, params, global, local, rept_local_rows(params), tau_hat, tau_v_hat);
}

rept_status rept_estimate_sums(uint32_t n, const rept_params* params, const int64_t* global, const int64_t* sums,
                               double* tau_hat, double* tau_v_hat) {
    return estimate_core(n, params, global, sums, 1u, tau_hat, tau_v_hat);
}

rept_status rept_reduce_local(const int64_t* local, uint32_t rows, uint32_t n, int64_t* sums, void* stream) {
    if (!local || !sums || rows == 0 || n == 0) return REPT_EINVAL;
    if (((uintptr_t)local | (uintptr_t)sums) & 7u) return REPT_EINVAL;
    if (rept_launch_reduce(local, rows, n, sums, (hipStream_t)stream) != hipSuccess) return REPT_EDEVICE;
    return REPT_OK;
}

rept_status rept_count_eta_workspace_size(const rept_graph* graph, const rept_params* params, size_t* bytes) {
    if (!valid_graph(graph) || !params_ok(params) || !bytes) return REPT_EINVAL;
    if (params->m > 65536) return REPT_ENOTSUP;
    const uint32_t G = groups_of(params), Gl = G < REPT_GMAX ? G : REPT_GMAX;  // groups of one launch
    const size_t pairs = (size_t)8 * Gl * graph->E;
    *bytes = table_bytes(graph, params) + ((pairs + 255) & ~(size_t)255);
    return REPT_OK;
}

rept_status rept_count_eta(const rept_graph* graph, const rept_params* params, int64_t* global, int64_t* local,
                           int64_t* eta, int64_t* eta_v, void* workspace, size_t workspace_bytes,
                           const rept_tuning* tuning, void* stream) {
    if (!valid_graph(graph) || !params_ok(params) || !global || !local || !eta) return REPT_EINVAL;
    if (((uintptr_t)eta | (uintptr_t)eta_v) & 7u) return REPT_EINVAL;
    if (is_mascot(params)) return REPT_ENOTSUP;
    if (params->m > 65536) return REPT_ENOTSUP;
    size_t need = 0;
    rept_status st = rept_count_eta_workspace_size(graph, params, &need);
    if (st != REPT_OK) return st;
    if (!workspace || ((uintptr_t)workspace & 255u)) return REPT_EINVAL;
    if (workspace_bytes < need) return REPT_ENOMEM;
    // groups in launches of at most 8, as rept_count: launch q counts its groups' processors
    // into its slice of the outputs and adds their pair counts to eta and eta_v
    const uint32_t G = groups_of(params), m = params->m, n = graph->n, c = params->c;
    const bool per_proc = (params->flags & REPT_LOCAL_PER_PROC) != 0;
    const uint32_t passes = (G + REPT_GMAX - 1) / REPT_GMAX;
    uint32_t* pairs = (uint32_t*)((uint8_t*)workspace + table_bytes(graph, params));
    hipStream_t s = (hipStream_t)stream;
    for (uint32_t check = 0; check < 2; ++check) {
        if (check) {
            if (rept_launch_zero(eta, (uint64_t)16 * c, s) != hipSuccess) return REPT_EDEVICE;
            if (eta_v && rept_launch_zero(eta_v, (uint64_t)16 * n, s) != hipSuccess) return REPT_EDEVICE;
        }
        for (uint32_t q = 0; q < passes; ++q) {
            const uint32_t k0 = q * REPT_GMAX, Gq = (G - k0) < REPT_GMAX ? (G - k0) : REPT_GMAX;
            const uint64_t left = (uint64_t)c - (uint64_t)k0 * m;
            rept_params pp = *params;
            pp.c = (uint32_t)(left < (uint64_t)Gq * m ? left : (uint64_t)Gq * m);
            const uint64_t goff = (uint64_t)k0 * m, loff = per_proc ? (uint64_t)k0 * m * n : (uint64_t)k0 * n;
            rept_job jb;
            memset(&jb, 0, sizeof(jb));
            jb.graph = graph;
            jb.params = pp;
            jb.global = global + goff;
            jb.local = local + loff;
            jb.t0 = 0;
            jb.t1 = graph->E;
            jb.unit0 = 0;
            jb.unit1 = UINT32_MAX;
            jb.workspace = workspace;
            jb.workspace_bytes = table_bytes(graph, params);
            JobDev d;
            uint64_t zw = 0;
            st = make_job(jb, &d, &zw);
            if (st != REPT_OK) return st;
            group_params(params->seed, d.G, d.hp, k0);
            d.es = (uint32_t)graph->E;
            d.pairs = pairs;
            BatchHeader h;
            st = make_header(1, d.G, d.gs, d.c, graph->max_out, zw, true, tuning, &h, true);
            if (st != REPT_OK) return st;
            if (!check) continue;
            h.any_fill = 1;
            h.fill_edges = graph->E > UINT32_MAX ? UINT32_MAX : (uint32_t)graph->E;
            if (rept_launch_zero(pairs, (uint64_t)8 * d.G * graph->E, s) != hipSuccess) return REPT_EDEVICE;
            if (rept_launch_single(graph->ctrl, h, d, s) != hipSuccess) return REPT_EDEVICE;
            if (rept_launch_eta(graph, d, eta, eta_v, (uint32_t)goff, c, s) != hipSuccess) return REPT_EDEVICE;
        }
    }
    return REPT_OK;
}

namespace {
// Algorithm 2's combination of the two estimates (Section III-B), one value: S1, S2 the sums
// over the first c1 groups and over the last group, eta the pair count; binary64 operations in
// the stated order, t1 when both variances are zero
double combine(int64_t S1, int64_t S2, int64_t eta, uint32_t m, uint32_t c) {
    const uint32_t c1 = c / m, c2 = c % m;
    const double dm = (double)m, dm2 = (double)((uint64_t)m * m), dm3 = (double)((uint64_t)m * m * m);
    const double dc1 = (double)c1, dc2 = (double)c2, dc = (double)c;
    const double a2 = (double)((uint64_t)m * m - c2), b2 = (double)(m - c2), dm1 = (double)(m - 1);
    const double t1 = ((double)S1 * dm) / dc1, t2 = ((double)S2 * dm2) / dc2;
    const double eh = ((double)eta * dm3) / dc;
    const double v1 = (t1 * dm1) / dc1, v2 = (t1 * a2 + (2.0 * eh) * b2) / dc2;
    return (v1 + v2 == 0.0) ? t1 : (v2 * t1 + v1 * t2) / (v1 + v2);
}
}  // namespace

rept_status rept_estimate_combined(uint32_t n, const rept_params* params, const int64_t* global,
                                   const int64_t* local, int64_t eta, const int64_t* eta_v, double* tau_hat,
                                   double* tau_v_hat) {
    if (!params_ok(params) || n == 0 || !global || !tau_hat || is_mascot(params)) return REPT_EINVAL;
    const uint32_t m = params->m, c = params->c;
    if (c <= m || c % m == 0) return REPT_EINVAL;  // rept_estimate covers these
    const int64_t lim = (int64_t)1 << 53;
    const uint32_t c1 = c / m;
    int64_t S1 = 0, S2 = 0;
    for (uint32_t i = 0; i < c; ++i) {
        int64_t* S = i < c1 * m ? &S1 : &S2;
        if (global[i] < 0 || global[i] >= lim - *S) return REPT_ERANGE;
        *S += global[i];
    }
    if (eta < 0 || eta >= lim) return REPT_ERANGE;
    if (tau_v_hat && local && eta_v) {
        const bool per_proc = (params->flags & REPT_LOCAL_PER_PROC) != 0;
        const uint32_t rows = rept_local_rows(params), split = per_proc ? c1 * m : c1;
        std::atomic<bool> bad{false};
        constexpr uint32_t kPart = 32768;
        const uint32_t parts = (uint32_t)(((uint64_t)n + kPart - 1) / kPart);
        bool write = false;  // first pass: check every sum; second pass: write (no output on ERANGE)
        const std::function<void(uint32_t)> part = [&](uint32_t k) {
            const uint32_t v0 = k * kPart, v1 = std::min<uint64_t>((uint64_t)v0 + kPart, n);
            for (uint32_t v = v0; v < v1; ++v) {
                int64_t A = 0, B = 0;
                bool ok = eta_v[v] >= 0 && eta_v[v] < lim;
                for (uint32_t r = 0; r < rows; ++r) {
                    const int64_t x = local[(uint64_t)r * n + v];
                    int64_t* S = r < split ? &A : &B;
                    ok &= x >= 0 && x < lim - *S;
                    *S += ok ? x : 0;
                }
                if (!ok) {
                    bad = true;
                    return;
                }
                if (write) tau_v_hat[v] = combine(A, B, eta_v[v], m, c);
            }
        };
        HostPool::get().run(parts, part);
        if (bad) return REPT_ERANGE;
        write = true;
        HostPool::get().run(parts, part);
    }
    *tau_hat = combine(S1, S2, eta, m, c);
    return REPT_OK;
}

rept_status rept_hash_slots(const rept_params* params, const uint32_t* edges, uint64_t num_edges, uint32_t* slots,
                            void* stream) {
    if (!params_ok(params) || (num_edges && (!edges || !slots))) return REPT_EINVAL;
    if ((uintptr_t)edges & 7u) return REPT_EINVAL;
    const uint32_t G = groups_of(params);
    if (G > REPT_GMAX) return REPT_ENOTSUP;
    if (num_edges == 0) return REPT_OK;
    uint64_t hp[4 * REPT_GMAX] = {0};
    group_params(params->seed, G, hp);
    if (rept_launch_slots(hp, G, params->m, edges, num_edges, slots, (hipStream_t)stream) != hipSuccess)
        return REPT_EDEVICE;
    return REPT_OK;
}

rept_status rept_batch_workspace_size(uint32_t njobs, size_t* bytes) {
    if (!bytes || njobs == 0 || njobs > 65535) return REPT_EINVAL;
    *bytes = (sizeof(BatchHeader) + (size_t)njobs * sizeof(JobDev) + 255) & ~(size_t)255;
    return REPT_OK;
}

}  // extern "C"

namespace {
// Pinned host staging of job tables: a ring of buffers, each reused only after the copy that last
// read it has completed (an event recorded after that copy), so rept_batch_prepare needs no
// stream synchronisation.  Buffers grow on demand and are kept for the process.
struct StageSlot {
    void* buf = nullptr;
    size_t bytes = 0;
    hipEvent_t done = nullptr;
    int device = -1;
    bool pending = false;  // `done` was recorded after a copy from `buf`
};
constexpr int kStageSlots = 8;
std::mutex g_stage_mu;
StageSlot g_stage[kStageSlots];
int g_stage_next = 0;

// a slot of at least `bytes` on the current device, free to write (caller holds g_stage_mu)
rept_status stage_slot(size_t bytes, StageSlot** out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return REPT_EDEVICE;
    StageSlot& s = g_stage[g_stage_next];
    g_stage_next = (g_stage_next + 1) % kStageSlots;
    if (s.pending) {
        if (hipEventSynchronize(s.done) != hipSuccess) return REPT_EDEVICE;
        s.pending = false;
    }
    if (s.device != dev && s.done) {  // events belong to the device they were created on
        (void)hipEventDestroy(s.done);
        s.done = nullptr;
    }
    if (!s.done) {
        if (hipEventCreateWithFlags(&s.done, hipEventDisableTiming) != hipSuccess) return REPT_EDEVICE;
        s.device = dev;
    }
    if (s.bytes < bytes) {
        if (s.buf) (void)hipHostFree(s.buf);
        s.buf = nullptr;
        s.bytes = 0;
        const size_t want = (bytes + 65535) & ~(size_t)65535;
        if (hipHostMalloc(&s.buf, want, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            return REPT_ENOMEM;
        }
        s.bytes = want;
    }
    *out = &s;
    return REPT_OK;
}
}  // namespace

extern "C" {

rept_status rept_batch_prepare(const rept_job* jobs, uint32_t njobs, const rept_tuning* tuning, void* workspace,
                               size_t workspace_bytes, void* stream) {
    size_t need = 0;
    if (!jobs || !workspace || rept_batch_workspace_size(njobs, &need) != REPT_OK) return REPT_EINVAL;
    if ((uintptr_t)workspace & 255u) return REPT_EINVAL;
    if (workspace_bytes < need) return REPT_ENOMEM;
    const size_t bytes = sizeof(BatchHeader) + (size_t)njobs * sizeof(JobDev);
    std::lock_guard<std::mutex> stage_lock(g_stage_mu);
    StageSlot* slot = nullptr;
    rept_status sst = stage_slot(bytes, &slot);
    if (sst != REPT_OK) return sst;
    uint8_t* host = (uint8_t*)slot->buf;
    memset(host, 0, bytes);
    JobDev* hj = (JobDev*)(host + sizeof(BatchHeader));
    uint32_t G_max = 1, gs_max = 1, c_max = 1, max_out = 0;
    uint64_t zero_words = 0;
    bool any_zero = false, any_fill = false;
    uint64_t fill_edges = 0;
    for (uint32_t j = 0; j < njobs; ++j) {
        uint64_t zw = 0;
        rept_status st = make_job(jobs[j], &hj[j], &zw);
        if (st != REPT_OK) return st;
        G_max = hj[j].G > G_max ? hj[j].G : G_max;
        gs_max = hj[j].gs > gs_max ? hj[j].gs : gs_max;
        c_max = hj[j].c > c_max ? hj[j].c : c_max;
        max_out = jobs[j].graph->max_out > max_out ? jobs[j].graph->max_out : max_out;
        if (!hj[j].accumulate) {
            any_zero = true;
            zero_words = zw > zero_words ? zw : zero_words;
        }
        if (hj[j].fill) {
            any_fill = true;
            fill_edges = jobs[j].graph->E > fill_edges ? jobs[j].graph->E : fill_edges;
        }
    }
    BatchHeader h;
    rept_status st = make_header(njobs, G_max, gs_max, c_max, max_out, zero_words, any_zero, tuning, &h);
    if (st != REPT_OK) return st;
    h.any_fill = any_fill ? 1u : 0u;
    h.fill_edges = fill_edges > UINT32_MAX ? UINT32_MAX : (uint32_t)fill_edges;
    memcpy(host, &h, sizeof(h));
    // stream-ordered: launches enqueued on `stream` after this call see the table; the staging
    // buffer is reused only after this copy's event has completed
    hipError_t e = hipMemcpyAsync(workspace, host, bytes, hipMemcpyHostToDevice, (hipStream_t)stream);
    if (e == hipSuccess) e = hipEventRecord(slot->done, (hipStream_t)stream);
    if (e != hipSuccess) return REPT_EDEVICE;
    slot->pending = true;
    std::lock_guard<std::mutex> lk(g_mu);
    g_shapes[workspace] = Shape{h};
    return REPT_OK;
}

rept_status rept_batch_launch(void* workspace, void* stream) {
    BatchHeader h;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        auto it = g_shapes.find(workspace);
        if (it == g_shapes.end()) return REPT_EINVAL;
        h = it->second.hdr;
    }
    if (rept_launch_batch(workspace, h, (hipStream_t)stream) != hipSuccess) return REPT_EDEVICE;
    return REPT_OK;
}

rept_status rept_batch_count(const rept_job* jobs, uint32_t njobs, const rept_tuning* tuning, void* workspace,
                             size_t workspace_bytes, void* stream) {
    rept_status st = rept_batch_prepare(jobs, njobs, tuning, workspace, workspace_bytes, stream);
    if (st != REPT_OK) return st;
    return rept_batch_launch(workspace, stream);
}

rept_status rept_stream_query_sizes(uint32_t n, uint64_t capacity, uint64_t max_chunk, size_t* bytes) {
    if (n == 0 || n > (1u << 29) || capacity == 0 || capacity >= (1ull << 31) || max_chunk == 0 ||
        max_chunk > capacity || !bytes)
        return REPT_EINVAL;
    const IncLayout L = inc_layout(n, capacity, max_chunk);
    if (L.temp_bytes == 0) return REPT_EDEVICE;
    *bytes = L.total;
    return REPT_OK;
}

rept_status rept_stream_create(uint32_t n, uint64_t capacity, uint64_t max_chunk, const rept_params* params,
                               void* buffer, size_t bytes, int64_t* global, int64_t* local, void* stream,
                               rept_stream** out) {
    if (!out || !params_ok(params) || !buffer || !global || !local) return REPT_EINVAL;
    if (((uintptr_t)buffer & 255u) || (((uintptr_t)global | (uintptr_t)local) & 7u)) return REPT_EINVAL;
    size_t need = 0;
    rept_status st = rept_stream_query_sizes(n, capacity, max_chunk, &need);
    if (st != REPT_OK) return st;
    const uint32_t G = groups_of(params);
    if (G > REPT_GMAX || params->m > 65536) return REPT_ENOTSUP;
    if (bytes < need) return REPT_ENOMEM;
    const IncLayout L = inc_layout(n, capacity, max_chunk);
    uint8_t* B = (uint8_t*)buffer;
    rept_stream* h = (rept_stream*)calloc(1, sizeof(rept_stream));
    if (!h) return REPT_ENOMEM;
    h->params = *params;
    h->capacity = capacity;
    h->max_chunk = max_chunk;
    IncState& S = h->st;
    S.n = n;
    S.end_bit = 32 + (bit_length(n - 1) ? bit_length(n - 1) : 1);
    S.T = 0;
    S.cur = 0;
    for (int i = 0; i < 2; ++i) {
        S.key[i] = (uint64_t*)(B + L.key[i]);
        S.tim[i] = (uint32_t*)(B + L.tim[i]);
    }
    S.off = (uint32_t*)(B + L.off);
    S.coff = (uint32_t*)(B + L.coff);
    S.ckey_a = (uint64_t*)(B + L.ckey_a);
    S.ckey_b = (uint64_t*)(B + L.ckey_b);
    S.ctim_a = (uint32_t*)(B + L.ctim_a);
    S.ctim_b = (uint32_t*)(B + L.ctim_b);
    S.end = (uint64_t*)(B + L.end);
    S.flags = (uint32_t*)(B + L.flags);
    S.temp = B + L.temp;
    S.temp_bytes = L.temp_bytes;
    h->eall = (uint32_t*)(B + L.eall);
    h->gpers = B + L.gpers;
    h->gscr = B + L.gscr;
    h->gws = B + L.gws;
    h->gpers_bytes = L.gpers_bytes;
    h->gscr_bytes = L.gscr_bytes;
    h->gws_bytes = L.gws_bytes;
    h->policy = REPT_STREAM_AUTO;
    const uint32_t cus = rept_num_cus() ? rept_num_cus() : 256;
    S.count_blocks = 8 * cus;
    IncCount& a = h->base;
    memset(&a, 0, sizeof(a));
    a.global = global;
    a.local = local;
    a.n = n;
    a.m = params->m;
    a.c = params->c;
    a.G = G;
    if (is_mascot(params)) {
        a.ck_full = a.last_ck = 1;
        a.pstride = 1;
    } else {
        a.ck_full = params->m;
        a.last_ck = params->c - (G - 1) * params->m;
        a.pstride = params->m;
    }
    a.per_proc = (params->flags & REPT_LOCAL_PER_PROC) ? 1u : 0u;
    group_params(params->seed, G, a.hp);
    hipStream_t s = (hipStream_t)stream;
    const uint64_t rows = rept_local_rows(params);
    if (rept_launch_zero(S.off, 4 * ((uint64_t)n + 1), s) != hipSuccess ||
        rept_inc_zero64(global, params->c, s) != hipSuccess ||
        rept_inc_zero64(local, rows * n, s) != hipSuccess) {
        free(h);
        return REPT_EDEVICE;
    }
    h->magic = REPT_STREAM_MAGIC;
    *out = h;
    return REPT_OK;
}

rept_status rept_stream_append(rept_stream* h, const uint32_t* edges, uint64_t num_edges, void* stream) {
    if (!valid_stream(h)) return REPT_EINVAL;
    if (num_edges == 0) return REPT_OK;
    if (!edges || ((uintptr_t)edges & 7u)) return REPT_EINVAL;
    if (num_edges > h->max_chunk || h->st.T + num_edges > h->capacity) return REPT_ENOMEM;
    const size_t temp = rept_inc_sort_temp_bytes(2 * num_edges, h->st.end_bit);
    if (temp == 0) return REPT_EDEVICE;
    if (temp > h->st.temp_bytes) return REPT_ENOMEM;  // not expected: sized for the largest chunk
    hipStream_t s = (hipStream_t)stream;
    if (rept_inc_prepare(h->st, edges, num_edges, s) != hipSuccess) return REPT_EDEVICE;
    uint32_t flags = 0;
    if (hipMemcpyAsync(&flags, h->st.flags, sizeof(flags), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return REPT_EDEVICE;
    // the stream's own order of precedence: ids, then self-loops, then repeated pairs
    if (flags & RF_RANGE) return REPT_ERANGE;
    if (flags & RF_SELFLOOP) return REPT_ESELFLOOP;
    if (flags & RF_DUP) return REPT_EDUP;
    const uint64_t t0 = h->st.T;
    if (hipMemcpyAsync(h->eall + 2 * t0, edges, 8 * num_edges, hipMemcpyDeviceToDevice, s) != hipSuccess ||
        rept_inc_merge(h->st, num_edges, s) != hipSuccess)
        return REPT_EDEVICE;
    bool recount = h->policy == REPT_STREAM_RECOUNT;
    if (h->policy == REPT_STREAM_AUTO) {
        uint64_t items = 0;
        if (hipMemcpyAsync(&items, h->st.end + 2 * num_edges - 1, sizeof(items), hipMemcpyDeviceToHost, s) !=
                hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return REPT_EDEVICE;
        recount = items > kRecountItemsPerEdge * h->st.T;
    }
    if (recount) {
        const rept_status st = recount_window(h, t0, h->st.T, s);
        if (st == REPT_OK) {
            ++h->n_recount;
            return REPT_OK;
        }
        if (st != REPT_ENOMEM) return st;  // ENOMEM: the prefix outgrew the reserved regions
    }
    if (rept_inc_count(h->st, num_edges, h->base, s) != hipSuccess) return REPT_EDEVICE;
    ++h->n_per_edge;
    return REPT_OK;
}

rept_status rept_stream_set_policy(rept_stream* h, uint32_t policy) {
    if (!valid_stream(h) || policy > REPT_STREAM_RECOUNT) return REPT_EINVAL;
    h->policy = policy;
    return REPT_OK;
}

rept_status rept_stream_paths(const rept_stream* h, uint64_t* per_edge, uint64_t* recount) {
    if (!valid_stream(h) || !per_edge || !recount) return REPT_EINVAL;
    *per_edge = h->n_per_edge;
    *recount = h->n_recount;
    return REPT_OK;
}

rept_status rept_stream_num_edges(const rept_stream* h, uint64_t* num_edges) {
    if (!valid_stream(h) || !num_edges) return REPT_EINVAL;
    *num_edges = h->st.T;
    return REPT_OK;
}

void rept_stream_destroy(rept_stream* h) {
    if (valid_stream(h)) {
        h->magic = 0;
        free(h);
    }
}

void rept_destroy(rept_graph* graph) {
    if (valid_graph(graph)) {
        graph->magic = 0;
        free(graph);
    }
}

const char* rept_status_str(int status) {
    switch (status) {
        case REPT_OK: return "ok";
        case REPT_EINVAL: return "invalid argument";
        case REPT_ERANGE: return "value out of range";
        case REPT_ESELFLOOP: return "self-loop in stream";
        case REPT_EDUP: return "duplicate edge in stream";
        case REPT_ENOMEM: return "buffer too small";
        case REPT_EDEVICE: return "device error";
        case REPT_ENOTSUP: return "not supported";
        default: return "unknown status";
    }
}

uint32_t rept_device_cus(void) { return rept_num_cus(); }

}  // extern "C"
