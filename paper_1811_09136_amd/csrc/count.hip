// The counting pass of REPT (Algorithm 1, Section III-A; groups of Section III-B) for every
// processor at once.
//
// What is counted.  For the stream edge (u, v) arriving at time t, processor i adds
// |N_u^(i) ∩ N_v^(i)| to tau^(i), tau_u^(i) and tau_v^(i) and one to tau_w^(i) for each common
// neighbour w, where N_x^(i) holds the neighbours of x through edges processor i stored
// before t.  So every triangle {x, y, z} of the stream graph is counted exactly once per
// processor that stored its first two edges -- at the update of its last edge -- and then
// adds one to tau^(i) and one to the local counter of each of its three nodes (the
// semi-triangles of Section III; Theorem 2).
//
// How it is counted here.  The build stores each edge once, at its lower-ranked endpoint
// (the "apex" side).  A triangle a < b < w (by rank) is found exactly once: from apex a, as
// the entry w of b's list that is also in a's list.  The three arrival times give its last
// edge; the hash of its first two edges gives, per group, whether one processor stored both.
// One pass therefore serves all c processors, and a window [t0, t1) of stream updates is the
// set of triangles whose last edge arrived in the window.
//
// Kernel.  k_count is persistent and drains a device work queue over all jobs of a batch, in
// two phases: apexes with long lists one per workgroup (the list is hashed into LDS chunk by
// chunk), then apexes with short lists one per wavefront.  A team (workgroup or wavefront)
// stages a's list in an LDS hash table (W side) and the lists of a's out-neighbours b that
// are not empty (B side), then walks the concatenated b lists in windows of 64 entries: each
// entry is one global load and one LDS probe.  Hits (triangles) go to a per-wavefront LDS
// queue and are attributed in full-wave batches.  Local counts are aggregated per staged
// entry and global counts per processor in LDS before the 64-bit global atomics.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>

#include <mutex>

#include "common.h"
#include "edge_hash.h"

namespace {

constexpr uint32_t kHashMul = 0x9E3779B1u;  // table index: Fibonacci hashing of the node id
constexpr uint32_t kWalk = 4;                // windows of 64 entries walked per round
constexpr uint32_t kQueue = 64 * (kWalk + 1);  // per-wavefront hit queue: < 64 left + one round

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <bool BLOCK>
__device__ __forceinline__ void team_sync() {
    if (BLOCK) __syncthreads();
    else wave_sync();
}

__device__ __forceinline__ uint32_t lane_id() { return threadIdx.x & 63; }

// A value that is the same in every active lane, in a scalar register.  The compiler cannot
// see that a value read from LDS or exchanged between lanes is uniform; in a scalar register,
// the loops and branches on it take scalar instructions instead of exec-mask control flow.
// (Applied only where it was measured to pay: scalar registers are scarce in k_count, and
// their spills cost vector instructions.)
__device__ __forceinline__ uint32_t wave_uni(uint32_t v) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)v); }
// lane u's value (u uniform), in a scalar register
__device__ __forceinline__ uint32_t lane_val(uint32_t v, uint32_t u) {
    return (uint32_t)__builtin_amdgcn_readlane((int)v, (int)u);
}

// Inclusive prefix sum over the 64 lanes with DPP: shifts by 1, 2, 4, 8 within rows of 16
// lanes, then row 0's and row 2's last lanes broadcast into rows 1 and 3 (row_bcast:15), then
// lane 31 into rows 2 and 3 (row_bcast:31).  Lanes without a source add zero.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, false);  // row_shr:1
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, false);  // row_shr:2
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, false);  // row_shr:4
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, false);  // row_shr:8
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false);  // row_bcast:15
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false);  // row_bcast:31
    return v;
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_readlane((int)wave_incl_scan(v), 63);
}

__host__ __device__ inline uint32_t pow2_at_least(uint32_t x) {
    uint32_t p = 64;
    while (p < x) p <<= 1;
    return p;
}
__host__ __device__ inline uint32_t log2u(uint32_t p) {
    uint32_t l = 0;
    while ((1u << l) < p) ++l;
    return l;
}
__host__ __device__ inline uint32_t up16(uint32_t x) { return (x + 15u) & ~15u; }
// 16-bit slots per staged edge: G padded to 1, 2, 4 or 8 (the slot table's row width)
__host__ __device__ inline uint32_t slot_width(uint32_t G) { return G <= 1 ? 1u : (G <= 2 ? 2u : (G <= 4 ? 4u : 8u)); }

// ---- LDS layout (shared by host sizing and device carving) --------------------------------
// [per-wave misc] x nwaves, then one union region: the workgroup's heavy team area or the
// wavefronts' light team areas (the heavy phase finishes before the light phase starts).
struct Area {  // one team's staging area: W side (hash table of a's list) + B side (b lists)
    uint32_t hkey, hidx, ew, et, wslot, cntw;
    uint32_t eb, etb, bslot, cntb, bpos, epos, ewe, ebe;
    uint32_t red;  // 64 words of team scratch (scans, reductions, broadcast)
    uint32_t bytes;
};
// eta: the B side also keeps each staged pair's adjacency position (Algorithm 2's counters)
// RW: slots per staged row (the widest slot-table row of the launch's jobs: the padded group
// count, or one keep mask for parallel MASCOT); G: groups of per-entry counters
__host__ __device__ inline Area area_layout(uint32_t DW, uint32_t DB, uint32_t G, uint32_t RW, uint32_t tf, bool eta) {
    Area A;
    const uint32_t H = pow2_at_least(tf * DW);
    uint32_t p = 0;
    A.hkey = p; p = up16(p + 4 * H);
    A.hidx = p; p = up16(p + 2 * H);
    A.ew = p; p = up16(p + 4 * DW);
    A.et = p; p = up16(p + 4 * DW);
    A.wslot = p; p = up16(p + 2 * RW * DW);
    A.cntw = p; p = up16(p + 4 * G * DW);
    A.eb = p; p = up16(p + 4 * DB);
    A.etb = p; p = up16(p + 4 * DB);
    A.bslot = p; p = up16(p + 2 * RW * DB);
    A.cntb = p; p = up16(p + 4 * G * DB);
    A.bpos = p; p = up16(p + 8 * (DB + 1));  // (list offset, first item) per staged list
    A.epos = p; p = eta ? up16(p + 4 * DB) : p;  // position of the pair {a, b} in the adjacency
    // Algorithm 2's per-edge counts of the W and B entries, (s, L) packed 16 + 16 bits per group
    A.ewe = p; p = eta ? up16(p + 4 * G * DW) : p;
    A.ebe = p; p = eta ? up16(p + 4 * G * DB) : p;
    A.red = p; p = up16(p + 4 * 64);
    A.bytes = p;
    return A;
}
struct Misc {  // per wavefront
    uint32_t mark, qv, qp, hist, hits, bytes;
};
__host__ __device__ inline Misc misc_layout(uint32_t HC) {
    Misc M;
    uint32_t p = 0;
    M.mark = p; p = up16(p + 64 * kWalk);  // one byte per entry of a round
    M.qv = p; p = up16(p + 4 * kQueue);
    M.qp = p; p = up16(p + 4 * kQueue);
    M.hist = p; p = up16(p + 4 * HC);
    M.hits = p; p = up16(p + 4);  // hits drained since the histogram's last flush
    M.bytes = p;
    return M;
}
struct Layout {
    Misc misc;
    Area heavy, light;
    uint32_t union_off, total;
};
__host__ __device__ inline Layout count_layout(uint32_t nwaves, uint32_t DL, uint32_t DW, uint32_t DB,
                                               uint32_t G, uint32_t RW, uint32_t HC, uint32_t LT, uint32_t HT,
                                               uint32_t DLB, bool eta, bool heavy, bool light) {
    Layout L;
    L.misc = misc_layout(HC);
    L.heavy = area_layout(DW, DB, G, RW, HT, eta);
    L.light = area_layout(DL, DLB, G, RW, LT, eta);
    L.union_off = nwaves * L.misc.bytes;
    // a launch holds only the areas of the phases it runs
    const uint32_t hb = heavy ? L.heavy.bytes : 0u, lb = light ? nwaves * L.light.bytes : 0u;
    const uint32_t u = hb > lb ? hb : lb;
    L.total = L.union_off + u;
    return L;
}

// ---- views ---------------------------------------------------------------------------------
struct TeamView {
    uint32_t* hkey;
    uint16_t* hidx;
    uint32_t* ew;
    uint32_t* et;
    uint16_t* wslot;  // [DW][gs] slot rows of the W entries
    uint32_t* cntw;
    uint32_t* eb;
    uint32_t* etb;
    uint16_t* bslot;  // [DB][gs] slot rows of the B entries
    uint32_t* cntb;
    uint2* bpos;  // .x: offset of b's list, .y: index of its first item in the chunk's walk
    uint32_t* epos;  // adjacency position of each staged pair {a, b}
    uint32_t* ewe;   // [G][DW] pair counts (s | L << 16) of the W entries since the last flush
    uint32_t* ebe;   // [G][DB] the same for the B entries
    uint32_t* red;
    uint32_t DW, DB;
    uint32_t tf;  // hash slots per key, at least
};
__device__ inline TeamView team_view(uint8_t* base, const Area& A, uint32_t DW, uint32_t DB, uint32_t tf) {
    TeamView T;
    T.tf = tf;
    T.hkey = (uint32_t*)(base + A.hkey);
    T.hidx = (uint16_t*)(base + A.hidx);
    T.ew = (uint32_t*)(base + A.ew);
    T.et = (uint32_t*)(base + A.et);
    T.wslot = (uint16_t*)(base + A.wslot);
    T.cntw = (uint32_t*)(base + A.cntw);
    T.eb = (uint32_t*)(base + A.eb);
    T.etb = (uint32_t*)(base + A.etb);
    T.bslot = (uint16_t*)(base + A.bslot);
    T.cntb = (uint32_t*)(base + A.cntb);
    T.bpos = (uint2*)(base + A.bpos);
    T.epos = (uint32_t*)(base + A.epos);
    T.ewe = (uint32_t*)(base + A.ewe);
    T.ebe = (uint32_t*)(base + A.ebe);
    T.red = (uint32_t*)(base + A.red);
    T.DW = DW;
    T.DB = DB;
    return T;
}
struct WaveView {
    uint8_t* mark;
    uint32_t* qv;
    uint32_t* qp;
    uint32_t* hist;
    uint32_t* hits;
};
__device__ inline WaveView wave_view(uint8_t* base, const Misc& M) {
    WaveView V;
    V.mark = base + M.mark;
    V.qv = (uint32_t*)(base + M.qv);
    V.qp = (uint32_t*)(base + M.qp);
    V.hist = (uint32_t*)(base + M.hist);
    V.hits = (uint32_t*)(base + M.hits);
    return V;
}

// ---- per-job constants held while a wavefront works on that job ----------------------------
struct JobRegs {
    const uint32_t* off;
    const uint32_t* nbr;
    const uint32_t* tim;
    const uint32_t* apex;
    const uint32_t* roff;
    const uint4* rrec;
    const uint32_t* rpos;
    int64_t* global;
    int64_t* local;
    const uint16_t* tab;  // slot table of the stored edges, gs slots per edge
    uint32_t* pairs;      // Algorithm 2 pair counters [G][es][2], or null
    uint32_t n, m, c, G, gs, per_proc, t0, t1, ck, last_ck, pstride, use_hist, es, mask;
};

__device__ inline void load_job(const JobDev* __restrict__ j, uint32_t HC, JobRegs& r) {
    r.off = j->off;
    r.nbr = j->nbr;
    r.tim = j->tim;
    r.apex = j->apex;
    r.roff = j->roff;
    r.rrec = j->rrec;
    r.rpos = j->rpos;
    r.global = j->global;
    r.local = j->local;
    r.tab = j->tab;
    r.pairs = j->pairs;
    r.es = j->es;
    r.gs = j->gs;
    r.n = j->n;
    r.m = j->m;
    r.c = j->c;
    r.G = j->G;
    r.per_proc = j->per_proc;
    r.t0 = j->t0;
    r.t1 = j->t1;
    r.ck = j->ck;
    r.last_ck = j->last_ck;
    r.pstride = j->pstride;
    r.mask = j->mask;
    r.use_hist = (HC != 0 && j->c <= HC) ? 1u : 0u;
}

using rept_hash::slot_of;

__device__ __forceinline__ void add64(int64_t* p, uint64_t v) {
    atomicAdd((unsigned long long*)p, (unsigned long long)v);
}

// loads from the graph arrays (global memory: lets the compiler emit global, not flat, loads)
template <typename T>
__device__ __forceinline__ T ldg(const T* p) {
    return *(const __attribute__((address_space(1))) T*)p;
}

// Slots of the edge stored at position p for every group, 16 bits per group: groups 0-3 in
// `lo`, groups 4-7 in `hi`.  gs (1, 2, 4 or 8) is uniform over the wavefront.
__device__ __forceinline__ void load_slots(const uint16_t* tab, uint32_t gs, uint32_t p, uint64_t& lo,
                                           uint64_t& hi) {
    hi = 0;
    if (gs == 1) {
        lo = ldg(tab + p);
    } else if (gs == 2) {
        lo = ldg((const uint32_t*)tab + p);
    } else if (gs == 4) {
        lo = ldg((const uint64_t*)tab + p);
    } else {
        lo = ldg((const uint64_t*)tab + 2 * (uint64_t)p);
        hi = ldg((const uint64_t*)tab + 2 * (uint64_t)p + 1);
    }
}
// staged slot rows in LDS, in the slot table's format; GS: row width known at compile time
template <uint32_t GS>
__device__ __forceinline__ void lds_row_t(const uint16_t* rows, uint32_t i, uint64_t& lo, uint64_t& hi) {
    hi = 0;
    if (GS == 1) {
        lo = rows[i];
    } else if (GS == 2) {
        lo = ((const uint32_t*)rows)[i];
    } else if (GS == 4) {
        lo = ((const uint64_t*)rows)[i];
    } else {
        const uint4 r = ((const uint4*)rows)[i];
        lo = ((uint64_t)r.y << 32) | r.x;
        hi = ((uint64_t)r.w << 32) | r.z;
    }
}
template <uint32_t GS>
__device__ __forceinline__ void load_slots_t(const uint16_t* tab, uint32_t p, uint64_t& lo, uint64_t& hi) {
    hi = 0;
    if (GS == 1) {
        lo = ldg(tab + p);
    } else if (GS == 2) {
        lo = ldg((const uint32_t*)tab + p);
    } else if (GS == 4) {
        lo = ldg((const uint64_t*)tab + p);
    } else {
        lo = ldg((const uint64_t*)tab + 2 * (uint64_t)p);
        hi = ldg((const uint64_t*)tab + 2 * (uint64_t)p + 1);
    }
}
__device__ __forceinline__ void lds_row(const uint16_t* rows, uint32_t gs, uint32_t i, uint64_t& lo, uint64_t& hi) {
    hi = 0;
    if (gs == 1) {
        lo = rows[i];
    } else if (gs == 2) {
        lo = ((const uint32_t*)rows)[i];
    } else if (gs == 4) {
        lo = ((const uint64_t*)rows)[i];
    } else {
        lo = ((const uint64_t*)rows)[2 * i];
        hi = ((const uint64_t*)rows)[2 * i + 1];
    }
}
__device__ __forceinline__ void store_row(uint16_t* rows, uint32_t gs, uint32_t i, uint64_t lo, uint64_t hi) {
    if (gs == 1) {
        rows[i] = (uint16_t)lo;
    } else if (gs == 2) {
        ((uint32_t*)rows)[i] = (uint32_t)lo;
    } else if (gs == 4) {
        ((uint64_t*)rows)[i] = lo;
    } else {
        ((uint64_t*)rows)[2 * i] = lo;
        ((uint64_t*)rows)[2 * i + 1] = hi;
    }
}
// bit 16g + 15 set for each 16-bit field g where x and y agree (exact per field: adding 0x7fff
// to a field's low 15 bits cannot carry into the next field)
__device__ __forceinline__ uint64_t eq_fields(uint64_t x, uint64_t y) {
    constexpr uint64_t kLow15 = 0x7fff7fff7fff7fffull;
    const uint64_t z = x ^ y;
    return ~(((z & kLow15) + kLow15) | z) & ~kLow15;
}
// field bits (bit 16g + 15) of the groups g < G, in the low and high words of a row
__device__ __forceinline__ void group_masks(uint32_t G, uint64_t& lo, uint64_t& hi) {
    constexpr uint64_t kHigh = 0x8000800080008000ull;
    lo = G >= 4 ? kHigh : kHigh & ((1ull << (16 * G)) - 1ull);
    hi = G <= 4 ? 0ull : (G >= 8 ? kHigh : kHigh & ((1ull << (16 * (G - 4))) - 1ull));
}

// ---- LDS hash table of a's list: 2-slot buckets probed linearly; keys w + 1, 0 = empty.
// Slot 0 of a bucket fills before slot 1, so an empty slot ends a probe sequence.  kbits is
// log2 of the bucket count (at least the number of keys: load factor <= 1/2).
__device__ __forceinline__ void hash_insert(uint32_t* hkey, uint16_t* hidx, uint32_t kbits, uint32_t w,
                                            uint32_t i) {
    const uint32_t mask = (1u << kbits) - 1u;
    uint32_t b = (w * kHashMul) >> (32 - kbits);
    for (;;) {
        if (atomicCAS(&hkey[2 * b], 0u, w + 1u) == 0u) {
            hidx[2 * b] = (uint16_t)i;
            return;
        }
        if (atomicCAS(&hkey[2 * b + 1], 0u, w + 1u) == 0u) {
            hidx[2 * b + 1] = (uint16_t)i;
            return;
        }
        b = (b + 1u) & mask;
    }
}

// largest i in [0, cnt) with bpos[i].y <= it, given bpos[0].y <= it < bpos[cnt].y (cnt and it
// the same in every lane: the search runs in scalar registers)
__device__ __forceinline__ uint32_t find_seg(const uint2* bpos, uint32_t cnt, uint32_t it) {
    uint32_t lo = 0, hi = cnt;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (wave_uni(bpos[mid].y) <= it) lo = mid; else hi = mid;
    }
    return lo;
}

// find the job owning queue position `tile` (largest j with prefix[j] <= tile)
__device__ __forceinline__ uint32_t find_job(const JobDev* jobs, uint32_t njobs, uint32_t tile, bool heavy) {
    uint32_t lo = 0, hi = njobs;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        const uint32_t p = heavy ? jobs[mid].heavy_prefix : jobs[mid].light_prefix;
        if (p <= tile) lo = mid; else hi = mid;
    }
    return lo;
}

// exclusive scan over the team (wave: 64 lanes; block: all threads, via T.red)
template <bool BLOCK>
__device__ __forceinline__ uint32_t team_excl_scan(uint32_t v, uint32_t* red, uint32_t& total) {
    const uint32_t inc = wave_incl_scan(v);
    if (!BLOCK) {
        total = lane_val(inc, 63);
        return inc - v;
    }
    const uint32_t lane = lane_id(), wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    if (lane == 63) red[wid] = inc;
    __syncthreads();
    uint32_t pre = 0, tot = 0;
    for (uint32_t w = 0; w < nw; ++w) {
        const uint32_t x = red[w];
        if (w < wid) pre += x;
        tot += x;
    }
    __syncthreads();
    total = wave_uni(tot);
    return pre + inc - v;
}

// sum over the team, 64-bit (the per-thread parts may exceed 32 bits together).  Within a
// wavefront the part is summed with the DPP scan, which needs no LDS permutes (unlike lane
// shuffles): in one 32-bit pass if the caller knows the wavefront's sum is below 2^32
// (`narrow`), else in three pieces of 26, 26 and 12 bits, whose 64-lane sums stay below 2^32
// and so are exact in 32 bits.
template <bool BLOCK>
__device__ __forceinline__ uint64_t team_sum64(uint64_t v, uint32_t* red, bool narrow) {
    if (narrow)
        v = wave_sum((uint32_t)v);
    else
        v = (uint64_t)wave_sum((uint32_t)v & 0x3ffffffu) + ((uint64_t)wave_sum((uint32_t)(v >> 26) & 0x3ffffffu) << 26) +
            ((uint64_t)wave_sum((uint32_t)(v >> 52)) << 52);
    if (!BLOCK) return v;
    const uint32_t lane = lane_id(), wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    uint64_t* red64 = (uint64_t*)(red + 16);  // words 16..47: up to 16 wavefronts
    if (lane == 0) red64[wid] = v;
    __syncthreads();
    uint64_t t = 0;
    for (uint32_t w = 0; w < nw; ++w) t += red64[w];
    __syncthreads();
    return t;
}

// Attribute queued hits [0, qn) of this wavefront.  A hit is (B index ib, hash slot of the W
// entry k, list position p): the triangle (a, b = eb[ib], w = ew[k]) with times t_ab = etb[ib],
// t_aw = et[k], t_bw = tim[p].  Its first two edges by time decide the processor per group:
// edges at a have their slots staged; the slots of {b, w} come from the slot table.
template <uint32_t GS, bool ETA>
__device__ void drain_hits_t(const JobRegs& J, const TeamView& T, const WaveView& V, uint32_t a, uint32_t wbase,
                             uint32_t qn) {
    const uint32_t lane = lane_id();
    for (uint32_t q0 = 0; q0 < qn; q0 += 64) {
        const uint32_t q = q0 + lane;
        if (q < qn) {
            const uint32_t v = V.qv[q];
            const uint32_t ib = v & 0xffffu, k = T.hidx[v >> 16];
            const uint32_t p = V.qp[q];
            const uint32_t b = T.eb[ib], w = T.ew[k];
            const uint32_t tab = T.etb[ib], taw = T.et[k], tbw = ldg(J.tim + p);
            // slots of {b, w}, the edge at position p, loaded with its time (one latency): the
            // branch below depends on both
            uint64_t blo, bhi;
            load_slots_t<GS>(J.tab, p, blo, bhi);
            uint64_t alo, ahi, wlo, whi;
            lds_row_t<GS>(T.bslot, ib, alo, ahi);
            lds_row_t<GS>(T.wslot, k, wlo, whi);
            // which edge arrived last: 0 = {a,b}, 1 = {a,w}, 2 = {b,w} (times are distinct)
            const uint32_t last = (tab > taw && tab > tbw) ? 0u : (taw > tbw ? 1u : 2u);
            const uint32_t tl = last == 0 ? tab : (last == 1 ? taw : tbw);
            // slot rows of the first two edges; the groups where their slots agree, all at once
            const uint64_t xlo = last == 0 ? wlo : alo, xhi = last == 0 ? whi : ahi;
            const uint64_t ylo = last == 2 ? wlo : blo, yhi = last == 2 ? whi : bhi;
            if (GS == 1 && J.mask) {
                // parallel MASCOT: the processors that kept both earlier edges
                uint32_t mm = (uint32_t)(xlo & ylo) & ((1u << J.G) - 1u);
                if (!(tl >= J.t0 && tl < J.t1)) mm = 0;
                while (mm) {
                    const uint32_t g = (uint32_t)__builtin_ctz(mm);  // processor g, its own group
                    mm &= mm - 1u;
                    if (J.use_hist) atomicAdd(&V.hist[g], 1u);
                    else add64(J.global + g, 1);
                    if (J.per_proc) {
                        int64_t* row = J.local + (uint64_t)g * J.n;
                        add64(row + a, 1);
                        add64(row + b, 1);
                        add64(row + w, 1);
                    } else {
                        atomicAdd(&T.cntb[g * T.DB + ib], 1u);
                        atomicAdd(&T.cntw[g * T.DW + k], 1u);
                    }
                }
                continue;
            }
            uint64_t glo, ghi;
            group_masks(J.G, glo, ghi);
            if (!(tl >= J.t0 && tl < J.t1)) glo = ghi = 0;
            uint64_t mlo = eq_fields(xlo, ylo) & glo, mhi = GS == 8 ? eq_fields(xhi, yhi) & ghi : 0ull;
            {
                while (mlo | mhi) {
                    uint32_t g, s1;
                    if (mlo) {
                        const uint32_t bit = (uint32_t)__builtin_ctzll(mlo);
                        g = bit >> 4;
                        s1 = (uint32_t)(xlo >> (bit - 15)) & 0xffffu;
                        mlo &= mlo - 1;
                    } else {
                        const uint32_t bit = (uint32_t)__builtin_ctzll(mhi);
                        g = 4 + (bit >> 4);
                        s1 = (uint32_t)(xhi >> (bit - 15)) & 0xffffu;
                        mhi &= mhi - 1;
                    }
                    const uint32_t ck = (g + 1 < J.G) ? J.ck : J.last_ck;
                    if (s1 < ck) {
                        const uint32_t proc = g * J.pstride + s1;
                        if (J.use_hist) atomicAdd(&V.hist[proc], 1u);
                        else add64(J.global + proc, 1);
                        if (J.per_proc) {
                            int64_t* row = J.local + (uint64_t)proc * J.n;
                            add64(row + a, 1);
                            add64(row + b, 1);
                            add64(row + w, 1);
                        } else {
                            atomicAdd(&T.cntb[g * T.DB + ib], 1u);
                            atomicAdd(&T.cntw[g * T.DW + k], 1u);
                        }
                        if (ETA && J.pairs) {
                            // Algorithm 2's per-edge counts (Section III-B): the first two edges
                            // gain a non-last occurrence (s), the last edge a last-edge occurrence
                            // (L) when the same processor stores it.  {a, w} and {a, b} are staged
                            // entries, counted in LDS; {b, w} (list position p) in global memory.
                            const uint64_t llo = last == 0 ? alo : (last == 1 ? wlo : blo);
                            const uint64_t lhi = last == 0 ? ahi : (last == 1 ? whi : bhi);
                            const uint32_t sl = (uint32_t)((g < 4 ? llo >> (16 * g) : lhi >> (16 * (g - 4))) & 0xffffu);
                            const uint32_t lw = sl == s1 ? (1u << 16) : 0u;  // the last edge's L step
                            const uint32_t we = last == 1 ? lw : 1u;  // {a, w}: last (L) or not (s)
                            const uint32_t be = last == 0 ? lw : 1u;  // {a, b}
                            if (we) atomicAdd(&T.ewe[g * T.DW + k], we);
                            if (be) atomicAdd(&T.ebe[g * T.DB + ib], be);
                            uint32_t* cp = J.pairs + 2 * ((uint64_t)g * J.es + p);
                            if (last != 2) atomicAdd(cp, 1u);
                            else if (lw) atomicAdd(cp + 1, 1u);
                        }
                    }
                }
            }
        }
    }
    wave_sync();
}

// Add the wavefront's histogram of global counts to the outputs and clear it.
__device__ void flush_hist_now(const JobRegs& J, const WaveView& V) {
    const uint32_t lane = lane_id();
    wave_sync();
    for (uint32_t p = lane; p < J.c; p += 64) {
        const uint32_t v = V.hist[p];
        if (v) {
            add64(J.global + p, v);
            V.hist[p] = 0;
        }
    }
    if (lane == 0) *V.hits = 0;
    wave_sync();
}

// A histogram counter gains at most one per drained hit (a hit is one triangle, and it is a
// semi-triangle of at most one processor per group), so it cannot pass kHistFlushHits + one
// drain's hits (< 2^32) if the histogram is flushed whenever the wavefront's hits since the
// last flush reach kHistFlushHits.
constexpr uint32_t kHistFlushHits = 1u << 31;

// the drain for the job's slot-row width (uniform over the wavefront)
template <bool ETA>
__device__ __forceinline__ void drain_hits(const JobRegs& J, const TeamView& T, const WaveView& V, uint32_t a,
                                           uint32_t wbase, uint32_t qn) {
    if (J.gs == 1) drain_hits_t<1, ETA>(J, T, V, a, wbase, qn);
    else if (J.gs == 2) drain_hits_t<2, ETA>(J, T, V, a, wbase, qn);
    else if (J.gs == 4) drain_hits_t<4, ETA>(J, T, V, a, wbase, qn);
    else drain_hits_t<8, ETA>(J, T, V, a, wbase, qn);
    if (J.use_hist) {
        const uint32_t h = *V.hits + qn;  // the same LDS word in every lane: uniform
        if (h >= kHistFlushHits) {
            flush_hist_now(J, V);
        } else {
            wave_sync();
            if (lane_id() == 0) *V.hits = h;
            wave_sync();
        }
    }
}

// add packed pair counts (s | L << 16) to the stored edge at adjacency position pos, group g
__device__ __forceinline__ void flush_pair(const JobRegs& J, uint32_t g, uint32_t pos, uint32_t v) {
    uint32_t* cp = J.pairs + 2 * ((uint64_t)g * J.es + pos);
    if (v & 0xffffu) atomicAdd(cp, v & 0xffffu);
    if (v >> 16) atomicAdd(cp + 1, v >> 16);
}

// popcount of the bits of `m` below this lane
__device__ __forceinline__ uint32_t lanes_below(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Walk items [it_begin, it_end) of the staged B chunk, kWalk windows of 64 entries per round:
// item `it` is entry it - bpos[own].y of the list of b = eb[own], where own is the largest
// index with bpos[own].y <= it.  Only non-empty lists are staged, so list starts are distinct
// and a lane's owner is i0 (the owner of the round's first item) plus the number of list
// starts after the round's first item and at or before its own.  The owners, the neighbour
// loads and the first hash probes of all windows of a round are issued together.
// A hit is queued as (owner | hash slot << 16, list position).
template <bool ETA>
__device__ void walk_items(const JobRegs& J, const TeamView& T, const WaveView& V, uint32_t a, uint32_t wbase,
                           uint32_t kbits, uint32_t bn, uint32_t it_begin, uint32_t it_end) {
    constexpr uint32_t R = 64 * kWalk;
    const uint32_t lane = lane_id();
    const uint32_t bmask = (1u << kbits) - 1u;
    uint32_t qn = 0;
    it_begin = wave_uni(it_begin);
    it_end = wave_uni(it_end);
    bn = wave_uni(bn);
    if (it_begin >= it_end) return;
    uint32_t i0 = wave_uni(find_seg(T.bpos, bn, it_begin));  // owner of the first item
    for (uint32_t base = it_begin; base < it_end; base += R) {
        uint32_t own[kWalk], p[kWalk], w[kWalk];
        bool valid[kWalk];
        uint32_t pre;  // owner of the round's last item
        // the starts of the two lists after i0 (bpos[bn] is the sentinel: reads stay in bpos[0..bn])
        const uint32_t s1 = T.bpos[i0 + 1 <= bn ? i0 + 1 : bn].y;
        const uint32_t s2 = i0 + 2 <= bn ? T.bpos[i0 + 2].y : 0xffffffffu;
        if (s2 >= base + R) {
            // at most one list starts inside the round: a lane's owner is i0 or i0 + 1
            const uint2 b0 = T.bpos[i0], b1 = T.bpos[i0 + 1 <= bn ? i0 + 1 : bn];
            const uint32_t d0 = b0.x - b0.y, d1 = b1.x - b1.y;  // position = item + d (mod 2^32)
            if (base + R <= it_end) {  // a full round: every lane loads, no mask is needed
#pragma unroll
                for (uint32_t j = 0; j < kWalk; ++j) {
                    const uint32_t it = base + 64 * j + lane;
                    const bool second = it >= s1;
                    own[j] = second ? i0 + 1 : i0;
                    p[j] = it + (second ? d1 : d0);
                    valid[j] = true;
                    w[j] = ldg(J.nbr + p[j]);
                }
            } else {
#pragma unroll
                for (uint32_t j = 0; j < kWalk; ++j) {
                    const uint32_t it = base + 64 * j + lane;
                    const bool second = it >= s1;
                    own[j] = second ? i0 + 1 : i0;
                    p[j] = it + (second ? d1 : d0);
                    valid[j] = it < it_end;
                    w[j] = valid[j] ? ldg(J.nbr + p[j]) : 0u;
                }
            }
            pre = s1 < base + R ? i0 + 1 : i0;
        } else {
        static_assert(kWalk == 4, "one 32-bit word of marks per lane");
        ((uint32_t*)V.mark)[lane] = 0u;
        wave_sync();
        // lists after i0 start after `base`; the ones starting inside the round are marked.  List
        // starts increase, so once a candidate window's first list starts after the round, no
        // later one starts inside it.
#pragma unroll
        for (uint32_t j = 0; j < kWalk; ++j) {
            const uint32_t first = i0 + 1 + 64 * j;
            if (first >= bn || T.bpos[first].y >= base + R) break;
            const uint32_t idx = first + lane;
            if (idx < bn) {
                const uint32_t st = T.bpos[idx].y;
                if (st < base + R) V.mark[st - base] = 1;
            }
        }
        wave_sync();
        pre = i0;
#pragma unroll
        for (uint32_t j = 0; j < kWalk; ++j) {
            const uint32_t f = V.mark[64 * j + lane];
            const uint64_t bal = __ballot(f != 0);
            own[j] = pre + lanes_below(bal) + f;
            pre += (uint32_t)__popcll(bal);
        }
        // pre is now the owner of the round's last item
#pragma unroll
        for (uint32_t j = 0; j < kWalk; ++j) {
            const uint32_t it = base + 64 * j + lane;
            valid[j] = it < it_end;
            const uint2 bp = T.bpos[own[j]];
            p[j] = bp.x + (it - bp.y);
            w[j] = valid[j] ? ldg(J.nbr + p[j]) : 0u;
        }
        }
        // the earlier rounds' whole batches of 64 hits are drained while this round's
        // neighbour loads are in flight (one wait covers both); the rest (fewer than 64) stays
        if (qn >= 64) {
            wave_sync();
            const uint32_t full = qn & ~63u, rem = qn - full;
            drain_hits<ETA>(J, T, V, a, wbase, full);
            if (rem) {
                uint32_t v = 0, pp = 0;
                if (lane < rem) {
                    v = V.qv[full + lane];
                    pp = V.qp[full + lane];
                }
                wave_sync();
                if (lane < rem) {
                    V.qv[lane] = v;
                    V.qp[lane] = pp;
                }
                wave_sync();
            }
            qn = rem;
        }
        // first probe of every window: a 2-slot bucket; a miss goes on only past a full bucket
        uint32_t bk[kWalk], pos[kWalk];
        bool hit[kWalk], more[kWalk];
        uint2 kk[kWalk];
#pragma unroll
        for (uint32_t j = 0; j < kWalk; ++j) {
            bk[j] = (w[j] * kHashMul) >> (32 - kbits);
            kk[j] = *(const uint2*)(T.hkey + 2 * bk[j]);
        }
#pragma unroll
        for (uint32_t j = 0; j < kWalk; ++j) {
            const uint32_t key = w[j] + 1u;
            const bool m0 = kk[j].x == key, m1 = kk[j].y == key;
            hit[j] = valid[j] && (m0 || m1);
            pos[j] = 2 * bk[j] + (m1 ? 1u : 0u);
            more[j] = valid[j] && !(m0 || m1) && kk[j].y != 0u;
        }
#pragma unroll
        for (uint32_t j = 0; j < kWalk; ++j) {
            const uint32_t key = w[j] + 1u;
            uint32_t b = bk[j];
            while (more[j]) {
                b = (b + 1u) & bmask;
                const uint2 k2 = *(const uint2*)(T.hkey + 2 * b);
                if (k2.x == key || k2.y == key) {
                    hit[j] = true;
                    pos[j] = 2 * b + (k2.y == key ? 1u : 0u);
                    more[j] = false;
                } else {
                    more[j] = k2.y != 0u;
                }
            }
        }
#pragma unroll
        for (uint32_t j = 0; j < kWalk; ++j) {
            const uint64_t hm = __ballot(hit[j]);
            if (hit[j]) {
                const uint32_t q = qn + lanes_below(hm);
                V.qv[q] = own[j] | (pos[j] << 16);
                V.qp[q] = p[j];
            }
            qn += (uint32_t)__popcll(hm);
        }
        // owner of the next round's first item
        const uint32_t nx = pre + 1;
        i0 = (nx < bn && T.bpos[nx].y <= base + R) ? nx : pre;
        wave_sync();
    }
    if (qn) {
        wave_sync();
        drain_hits<ETA>(J, T, V, a, wbase, qn);
    }
}

// Count every triangle whose lowest-ranked node is a.  The team is the workgroup (BLOCK) or
// this wavefront.  a's list is hashed into LDS in chunks of DW entries (W side); for each W
// chunk the lists of all of a's out-neighbours are walked in chunks of DB entries (B side).
// (s, d): offset and length of a's list; (r0, rn): offset and length of a's reverse list.
template <bool BLOCK, bool ETA>
__device__ void count_apex(const JobRegs& J, const TeamView& T, const WaveView& V, uint32_t a, uint32_t s,
                           uint32_t d, uint32_t r0, uint32_t rn) {
    const uint32_t nt = BLOCK ? blockDim.x : 64;
    const uint32_t tid = BLOCK ? threadIdx.x : lane_id();
    const uint32_t nw = nt >> 6, wid = BLOCK ? (threadIdx.x >> 6) : 0;
    const uint32_t nbtot = d + rn;
    const uint32_t G = J.G;
    for (uint32_t ws = 0; ws < d; ws += T.DW) {
        const uint32_t wn = (d - ws) < T.DW ? (d - ws) : T.DW;
        // the whole table (sized for DW keys) is used whatever wn is: a sparser table ends more
        // probes at their first bucket
        const uint32_t slots = pow2_at_least(T.tf * T.DW), kbits = log2u(slots) - 1;
        for (uint32_t i = tid; i < slots; i += nt) T.hkey[i] = 0;
        team_sync<BLOCK>();
        for (uint32_t i = tid; i < wn; i += nt) {
            const uint32_t w = ldg(J.nbr + s + ws + i);
            T.ew[i] = w;
            T.et[i] = ldg(J.tim + s + ws + i);
            uint64_t lo, hi;
            load_slots(J.tab, J.gs, s + ws + i, lo, hi);
            store_row(T.wslot, J.gs, i, lo, hi);
            for (uint32_t g = 0; g < G; ++g) T.cntw[g * T.DW + i] = 0;
            if (ETA)
                for (uint32_t g = 0; g < G; ++g) T.ewe[g * T.DW + i] = 0;
            hash_insert(T.hkey, T.hidx, kbits, w, i);
        }
        team_sync<BLOCK>();
        // B entries: first a's own pairs a -> b whose out(b) is not longer than out(a) (walk
        // out(b)), then the reverse pairs y -> a with out(y) shorter than out(a) (walk out(y)):
        // every triangle is found once, from its lowest pair, walking the shorter list
        for (uint32_t bs = 0; bs < nbtot; bs += T.DB) {
            const uint32_t braw = (nbtot - bs) < T.DB ? (nbtot - bs) : T.DB;
            // stage the lists to walk in this chunk: compact by a scan of "walked", then scan
            // their lengths
            uint32_t nb = 0, items = 0;
            for (uint32_t c0 = 0; c0 < braw; c0 += nt) {
                const uint32_t i = c0 + tid;
                uint32_t b = 0, bo = 0, bd = 0, tb = 0, pab = 0;
                const uint32_t e = bs + i;  // B entry index
                if (i < braw) {
                    if (e < d) {
                        pab = s + e;
                        if (e >= ws && e < ws + wn) {  // staged as a W entry of this chunk
                            b = T.ew[e - ws];
                            tb = T.et[e - ws];
                        } else {
                            b = ldg(J.nbr + pab);
                            tb = ldg(J.tim + pab);
                        }
                        bo = ldg(J.off + b);
                        bd = ldg(J.off + b + 1) - bo;
                        if (bd > d) bd = 0;  // out(a) is shorter: counted at b
                    } else {
                        const uint32_t q = r0 + (e - d);
                        const uint4 r = J.rrec[q];
                        b = r.x;
                        tb = r.y;
                        bo = r.z;
                        bd = r.w;
                        pab = ldg(J.rpos + q);
                    }
                }
                uint32_t tot_nb, tot_items;
                const uint32_t pos = nb + team_excl_scan<BLOCK>(bd ? 1u : 0u, T.red, tot_nb);
                const uint32_t sc = items + team_excl_scan<BLOCK>(bd, T.red, tot_items);
                if (bd) {
                    T.eb[pos] = b;
                    T.etb[pos] = tb;
                    T.bpos[pos] = make_uint2(bo, sc);
                    if (ETA) T.epos[pos] = pab;
                    // an own pair {a, b} is also a W entry when it falls in the current W chunk
                    const bool staged = e >= ws && e < ws + wn;
                    uint64_t lo = 0, hi = 0;
                    if (staged) lds_row(T.wslot, J.gs, e - ws, lo, hi);
                    else load_slots(J.tab, J.gs, pab, lo, hi);
                    store_row(T.bslot, J.gs, pos, lo, hi);
                    for (uint32_t g = 0; g < G; ++g) T.cntb[g * T.DB + pos] = 0;
                    if (ETA)
                        for (uint32_t g = 0; g < G; ++g) T.ebe[g * T.DB + pos] = 0;
                }
                nb += tot_nb;
                items += tot_items;
            }
            if (tid == 0) T.bpos[nb] = make_uint2(0u, items);
            team_sync<BLOCK>();
            if (nb) {
                // each wavefront of the team walks one contiguous range of windows
                const uint32_t nwin = (items + 63) / 64;
                const uint32_t per = (nwin + nw - 1) / nw;
                const uint32_t w0 = wid * per, w1 = (w0 + per) < nwin ? (w0 + per) : nwin;
                const uint32_t ib = w0 * 64, ie = (w1 * 64) < items ? (w1 * 64) : items;
                if (w0 < w1) walk_items<ETA>(J, T, V, a, s + ws, kbits, nb, ib, ie);
            }
            team_sync<BLOCK>();
            if (!J.per_proc) {
                for (uint32_t x = tid; x < G * nb; x += nt) {
                    const uint32_t g = x / nb, i = x - g * nb;
                    const uint32_t v = T.cntb[g * T.DB + i];
                    if (v) add64(J.local + (uint64_t)g * J.n + T.eb[i], v);
                }
            }
            if (ETA && J.pairs) {
                // this B chunk's pair counts of the staged entries: at most one per W entry for a
                // B entry and one per B list for a W entry, so 16 bits each cannot overflow
                for (uint32_t x = tid; x < G * nb; x += nt) {
                    const uint32_t g = x / nb, i = x - g * nb;
                    const uint32_t v = T.ebe[g * T.DB + i];
                    if (v) flush_pair(J, g, T.epos[i], v);
                }
                for (uint32_t x = tid; x < G * wn; x += nt) {
                    const uint32_t g = x / wn, i = x - g * wn;
                    const uint32_t v = T.ewe[g * T.DW + i];
                    if (v) {
                        flush_pair(J, g, s + ws + i, v);
                        T.ewe[g * T.DW + i] = 0;
                    }
                }
            }
            team_sync<BLOCK>();
        }
        if (!J.per_proc) {
            // flush the w-side counts; their sum per group is a's own count for this chunk.  A W
            // entry gains at most one per list walked against it, so that sum is at most
            // wn * nbtot: a light unit's is below 2^32 and one 32-bit pass sums it.  A team of a
            // heavy unit always takes the three-piece sum (a few instructions per unit there), so
            // every graph with heavy and light units runs both forms.
            const bool narrow = !BLOCK && (uint64_t)wn * nbtot < (1ull << 32);
            for (uint32_t g = 0; g < G; ++g) {
                uint64_t part = 0;
                for (uint32_t i = tid; i < wn; i += nt) {
                    const uint32_t v = T.cntw[g * T.DW + i];
                    if (v) {
                        add64(J.local + (uint64_t)g * J.n + T.ew[i], v);
                        part += v;
                    }
                }
                const uint64_t tot = team_sum64<BLOCK>(part, T.red, narrow);
                if (tid == 0 && tot) add64(J.local + (uint64_t)g * J.n + a, tot);
            }
        }
        team_sync<BLOCK>();
    }
}

__device__ void flush_hist(const JobRegs& J, const WaveView& V, int cur) {
    if (cur < 0 || !J.use_hist) return;
    flush_hist_now(J, V);
}

// ======================================================================= setup / zero ====

__global__ void k_write_ctrl(uint8_t* ctrl, BatchHeader hdr, JobDev job) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        *(BatchHeader*)ctrl = hdr;
        *(JobDev*)(ctrl + sizeof(BatchHeader)) = job;
    }
}

// Per job: its units split into heavy units (out-degree above wave_cap) and light tiles, and
// its offsets in both queues.  One block: a thread per job finds the split by binary search
// over the job's apex order, then thread 0 forms the offsets from the counts in LDS.
__global__ void __launch_bounds__(1024) k_setup(BatchHeader* hdr, JobDev* jobs) {
    __shared__ uint32_t cnt[2][1024];  // heavy units and light tiles of the chunk's jobs
    const uint32_t nj = hdr->njobs, cap = hdr->wave_cap, lt = hdr->light_tile;
    uint32_t hp = 0, lp = 0;  // running prefixes (thread 0)
    for (uint32_t j0 = 0; j0 < nj; j0 += blockDim.x) {
        const uint32_t j = j0 + threadIdx.x;
        if (j < nj) {
            JobDev& J = jobs[j];
            // units are sorted by key = max(list length, reverse-list length >> REPT_REV_SHIFT), at
            // most n - 1, descending: the ones above `cap` (a workgroup each) form a prefix
            uint32_t lo = 0, hi = J.unit1;  // first index whose key <= cap (unit1 <= num_apex)
            while (lo < hi) {
                const uint32_t mid = (lo + hi) >> 1;
                const uint32_t a = J.apex[mid];
                const uint32_t d = J.off[a + 1] - J.off[a], r = (J.roff[a + 1] - J.roff[a]) >> REPT_REV_SHIFT;
                const uint32_t k = d > r ? d : r;
                const uint32_t key = k < J.n - 1 ? k : J.n - 1;
                if (key > cap) lo = mid + 1; else hi = mid;
            }
            const uint32_t u0 = J.unit0, u1 = J.unit1;
            const uint32_t hend = u1 < lo ? u1 : lo;
            const uint32_t nh = hend > u0 ? hend - u0 : 0;
            const uint32_t tiles = (u1 - u0 - nh + lt - 1) / lt;
            J.n_heavy = nh;
            J.light_tiles = tiles;
            cnt[0][threadIdx.x] = nh;
            cnt[1][threadIdx.x] = tiles;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            const uint32_t m = (nj - j0) < blockDim.x ? (nj - j0) : blockDim.x;
            for (uint32_t i = 0; i < m; ++i) {
                jobs[j0 + i].heavy_prefix = hp;
                jobs[j0 + i].light_prefix = lp;
                hp += cnt[0][i];
                lp += cnt[1][i];
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        hdr->heavy_total = hp;
        hdr->light_total = lp;
        for (uint32_t q = 0; q < kQueues; ++q) {
            hdr->queues[q * kQueueStride + kLightQueue] = 0;
            hdr->queues[q * kQueueStride + kHeavyQueue] = 0;
        }
    }
}

// clear the outputs of jobs that overwrite: grid (X, njobs)
__global__ void k_zero(const BatchHeader* hdr, const JobDev* jobs) {
    const JobDev& J = jobs[blockIdx.y];
    if (J.accumulate) return;
    const uint64_t nglob = J.c, nloc = (uint64_t)J.rows * J.n;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nglob + nloc; i += stride) {
        if (i < nglob) J.global[i] = 0;
        else J.local[i - nglob] = 0;
    }
}

// Slot table of each job whose launch writes it: tab[p * gs + k] = h_k of the edge stored at
// position p, i.e. {b, nbr[p]} for the node b whose list holds p (Section III-A's hash, one
// independent function per group as in Section III-B).  Grid (X, njobs) of 256 threads.  A
// workgroup takes FILL_CHUNK consecutive positions (so a range of long lists is spread over
// many workgroups), finds the nodes owning its first and last positions, stages the offsets of
// that node range in LDS, FILL_NODES at a time, and hashes one position per thread (coalesced),
// finding each position's node by binary search over the staged offsets.
constexpr uint32_t FILL_CHUNK = 4096;
constexpr uint32_t FILL_NODES = 1024;

// the node whose list holds position p (the largest b < n with off[b] <= p), for p < off[n]:
// each round samples the candidate node range at 256 evenly spaced nodes, one per thread, and
// keeps the interval between the last sample at or below p and the next
__device__ uint32_t fill_owner(const uint32_t* off, uint32_t n, uint32_t p) {
    uint32_t L = 0, R = n;  // off[L] <= p < off[R]
    while (R - L > 1) {
        const uint32_t step = (R - L + 255u) / 256u;
        const uint32_t b = L + threadIdx.x * step;
        const uint32_t k = (uint32_t)__syncthreads_count(b < R && ldg(off + b) <= p);  // >= 1
        const uint32_t L2 = L + (k - 1u) * step;
        R = (L2 + step) < R ? (L2 + step) : R;
        L = L2;
    }
    return L;
}

__global__ void __launch_bounds__(256) k_fill(const JobDev* __restrict__ jobs) {
    __shared__ uint32_t so[FILL_NODES + 1];
    const JobDev& J = jobs[blockIdx.y];
    if (!J.fill) return;
    const uint32_t G = J.G, gs = J.gs, m = J.m, n = J.n;
    const uint32_t* __restrict__ off = J.off;
    const uint32_t* __restrict__ nbr = J.nbr;
    uint16_t* __restrict__ tab = J.tab;
    uint64_t cf[4 * REPT_GMAX];  // coefficients read once (the table stores cannot change them)
#pragma unroll
    for (uint32_t i = 0; i < 4 * REPT_GMAX; ++i) cf[i] = i < 4 * G ? J.hp[i] : 0;
    const uint32_t Es = ldg(off + n);
    for (uint64_t c0 = (uint64_t)blockIdx.x * FILL_CHUNK; c0 < Es; c0 += (uint64_t)gridDim.x * FILL_CHUNK) {
        const uint32_t p0 = (uint32_t)c0, p1 = (c0 + FILL_CHUNK) < Es ? (uint32_t)(c0 + FILL_CHUNK) : Es;
        const uint32_t bf = fill_owner(off, n, p0), bl = fill_owner(off, n, p1 - 1u);
        for (uint32_t w0 = bf; w0 <= bl; w0 += FILL_NODES) {
            const uint32_t cnt = (bl + 1u - w0) < FILL_NODES ? (bl + 1u - w0) : FILL_NODES;
            __syncthreads();  // the previous window's offsets are no longer read
            for (uint32_t i = threadIdx.x; i <= cnt; i += 256u) so[i] = ldg(off + w0 + i);
            __syncthreads();
            const uint32_t q0 = so[0] > p0 ? so[0] : p0, q1 = so[cnt] < p1 ? so[cnt] : p1;
            for (uint32_t p = q0 + threadIdx.x; p < q1; p += 256u) {
                uint32_t lo = 0, hi = cnt;  // so[lo] <= p < so[hi]
                while (hi - lo > 1) {
                    const uint32_t mid = (lo + hi) >> 1;
                    if (so[mid] <= p) lo = mid; else hi = mid;
                }
                const uint32_t b = w0 + lo, w = ldg(nbr + p);
                uint32_t wd[4] = {0u, 0u, 0u, 0u};
                if (J.mask) {  // parallel MASCOT: bit g = processor g keeps the edge (h_g = 0)
#pragma unroll
                    for (uint32_t g = 0; g < REPT_GMAX; ++g)
                        if (g < G) wd[0] |= (slot_of(cf + 4 * g, m, b, w) == 0u ? 1u : 0u) << g;
                } else {
#pragma unroll
                    for (uint32_t g = 0; g < REPT_GMAX; ++g)
                        if (g < G) wd[g >> 1] |= slot_of(cf + 4 * g, m, b, w) << (16 * (g & 1));
                }
                if (gs == 1) tab[p] = (uint16_t)wd[0];
                else if (gs == 2) ((uint32_t*)tab)[p] = wd[0];
                else if (gs == 4) ((uint2*)tab)[p] = make_uint2(wd[0], wd[1]);
                else ((uint4*)tab)[p] = make_uint4(wd[0], wd[1], wd[2], wd[3]);
            }
        }
    }
}

// Algorithm 2's triangle-pair counts from the per-edge counters (Section III-B).  For a stored
// edge g of processor i (group k, slot h_k(g)): s = semi-triangles of i with g as a non-last
// edge, L = those with g as the last edge.  The definition of eta^(i) counts C(s, 2) pairs at
// g; Algorithm 2 as printed, whose counter starts at |N| when g is inserted, counts
// s L + C(s, 2).  Both go to eta[0][i], eta[1][i]; each edge's share also goes to both of its
// endpoints in eta_v[0][.], eta_v[1][.] (summed over processors).  Work split as in k_fill.
constexpr uint32_t ETA_LDS_PROCS = 512;  // processors accumulated in LDS per workgroup
constexpr uint32_t ETA_HASH = 1024;      // neighbour shares aggregated per workgroup (open addressing)
constexpr uint32_t ETA_PROBES = 16;      // probes before a share goes to global memory directly
__global__ void __launch_bounds__(256) k_eta(const uint32_t* __restrict__ off, const uint32_t* __restrict__ nbr,
                                             uint32_t n, const uint16_t* __restrict__ tab, uint32_t gs, uint32_t G,
                                             uint32_t m, uint32_t c, const uint32_t* __restrict__ pairs, uint32_t es,
                                             uint32_t proc0, uint32_t stride,
                                             int64_t* __restrict__ eta, int64_t* __restrict__ eta_v) {
    __shared__ uint32_t so[FILL_NODES + 1];
    __shared__ unsigned long long acc[2][ETA_LDS_PROCS];
    __shared__ unsigned long long own[2][FILL_NODES];  // shares of the owners in the node window
    __shared__ uint32_t hkey[ETA_HASH];                 // neighbour id + 1, 0 = empty
    __shared__ unsigned long long hval[2][ETA_HASH];
    const bool in_lds = c <= ETA_LDS_PROCS;
    for (uint32_t i = threadIdx.x; i < ETA_LDS_PROCS; i += 256u) acc[0][i] = acc[1][i] = 0ull;
    for (uint32_t i = threadIdx.x; i < ETA_HASH; i += 256u) {
        hkey[i] = 0u;
        hval[0][i] = hval[1][i] = 0ull;
    }
    const uint32_t Es = ldg(off + n);
    for (uint64_t c0 = (uint64_t)blockIdx.x * FILL_CHUNK; c0 < Es; c0 += (uint64_t)gridDim.x * FILL_CHUNK) {
        const uint32_t p0 = (uint32_t)c0, p1 = (c0 + FILL_CHUNK) < Es ? (uint32_t)(c0 + FILL_CHUNK) : Es;
        const uint32_t bf = fill_owner(off, n, p0), bl = fill_owner(off, n, p1 - 1u);
        for (uint32_t w0 = bf; w0 <= bl; w0 += FILL_NODES) {
            const uint32_t cnt = (bl + 1u - w0) < FILL_NODES ? (bl + 1u - w0) : FILL_NODES;
            __syncthreads();
            for (uint32_t i = threadIdx.x; i <= cnt; i += 256u) so[i] = ldg(off + w0 + i);
            for (uint32_t i = threadIdx.x; i < cnt; i += 256u) own[0][i] = own[1][i] = 0ull;
            __syncthreads();
            const uint32_t q0 = so[0] > p0 ? so[0] : p0, q1 = so[cnt] < p1 ? so[cnt] : p1;
            for (uint32_t p = q0 + threadIdx.x; p < q1; p += 256u) {
                unsigned long long fd = 0, fl = 0;
                for (uint32_t k = 0; k < G; ++k) {
                    const uint64_t w2 = ldg((const uint64_t*)pairs + (uint64_t)k * es + p);  // (s, L)
                    const uint32_t sx = (uint32_t)w2, ly = (uint32_t)(w2 >> 32);
                    const uint32_t slot = ldg(tab + (uint64_t)p * gs + k);
                    // an edge counts only for an active processor (inactive slots stay at zero)
                    if (sx == 0 || k * m + slot >= c) continue;
                    const unsigned long long d = (unsigned long long)sx * (sx - 1u) / 2u;
                    const unsigned long long l = d + (unsigned long long)sx * ly;
                    const uint32_t proc = k * m + slot;
                    if (in_lds) {
                        atomicAdd(&acc[0][proc], d);
                        atomicAdd(&acc[1][proc], l);
                    } else {
                        atomicAdd((unsigned long long*)eta + proc0 + proc, d);
                        atomicAdd((unsigned long long*)eta + stride + proc0 + proc, l);
                    }
                    fd += d;
                    fl += l;
                }
                if (eta_v && (fd | fl)) {
                    uint32_t lo = 0, hi = cnt;  // so[lo] <= p < so[hi]
                    while (hi - lo > 1) {
                        const uint32_t mid = (lo + hi) >> 1;
                        if (so[mid] <= p) lo = mid; else hi = mid;
                    }
                    atomicAdd(&own[0][lo], fd);  // the owner a = w0 + lo
                    atomicAdd(&own[1][lo], fl);
                    // the neighbour b: its slot in the workgroup's table, or global memory
                    const uint32_t b = ldg(nbr + p), key = b + 1u;
                    uint32_t h = (b * kHashMul) >> (32 - 10), probes = 0;
                    bool done = false;
                    for (; probes < ETA_PROBES; ++probes, h = (h + 1u) & (ETA_HASH - 1u)) {
                        const uint32_t cur = hkey[h];
                        if (cur == key || (cur == 0u && atomicCAS(&hkey[h], 0u, key) == 0u) || hkey[h] == key) {
                            atomicAdd(&hval[0][h], fd);
                            atomicAdd(&hval[1][h], fl);
                            done = true;
                            break;
                        }
                    }
                    if (!done) {
                        atomicAdd((unsigned long long*)eta_v + b, fd);
                        atomicAdd((unsigned long long*)eta_v + n + b, fl);
                    }
                }
            }
            __syncthreads();
            if (eta_v) {
                for (uint32_t i = threadIdx.x; i < cnt; i += 256u) {
                    if (own[0][i]) atomicAdd((unsigned long long*)eta_v + w0 + i, own[0][i]);
                    if (own[1][i]) atomicAdd((unsigned long long*)eta_v + n + w0 + i, own[1][i]);
                }
            }
        }
        // the neighbour shares of this run of positions
        __syncthreads();
        if (eta_v) {
            for (uint32_t i = threadIdx.x; i < ETA_HASH; i += 256u) {
                const uint32_t key = hkey[i];
                if (key) {
                    if (hval[0][i]) atomicAdd((unsigned long long*)eta_v + (key - 1u), hval[0][i]);
                    if (hval[1][i]) atomicAdd((unsigned long long*)eta_v + n + (key - 1u), hval[1][i]);
                    hkey[i] = 0u;
                    hval[0][i] = hval[1][i] = 0ull;
                }
            }
        }
    }
    __syncthreads();
    if (in_lds) {
        for (uint32_t i = threadIdx.x; i < c; i += 256u) {
            if (acc[0][i]) atomicAdd((unsigned long long*)eta + proc0 + i, acc[0][i]);
            if (acc[1][i]) atomicAdd((unsigned long long*)eta + stride + proc0 + i, acc[1][i]);
        }
    }
}

// zero n 32-bit words (a kernel rather than a memset, so the sequence stays capture-safe)
__global__ void k_zero_u32(uint32_t* p, uint64_t words) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

// ======================================================================= count kernel ====

// Claim the next tile of a phase's queue (counters at ctr[q * kQueueStride]).  The caller starts
// at its own sub-queue `q` with `left` = kQueues and moves on to the next sub-queue when one is
// exhausted; returns `total` once it has found every sub-queue exhausted.
__device__ uint32_t claim_tile(uint32_t* ctr, uint32_t total, uint32_t& q, uint32_t& left) {
    while (left) {
        const uint32_t cnt = total > q ? (total - q + kQueues - 1u) / kQueues : 0u;  // tiles of sub-queue q
        if (cnt) {
            const uint32_t k = atomicAdd(&ctr[q * kQueueStride], 1u);
            if (k < cnt) return q + kQueues * k;
        }
        q = (q + 1u) % kQueues;
        --left;
    }
    return total;
}

// ETA: the form that also counts Algorithm 2's per-edge pair counters for jobs that ask for
// them (a separate instance, so the plain kernel's registers are not spent on them)
// phases: 1 the heavy phase, 2 the light phase, 3 both (one launch)
template <bool ETA>
__global__ void __launch_bounds__(1024) k_count(BatchHeader* hdr, const JobDev* __restrict__ jobs, uint32_t phases) {
    extern __shared__ __align__(16) uint8_t lds[];
    const uint32_t lane = lane_id(), wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const uint32_t DL = hdr->wave_cap, DW = hdr->block_cap, DB = hdr->b_chunk;
    const uint32_t GM = hdr->G_max, HC = hdr->hist_c, njobs = hdr->njobs;
    const uint32_t LT = hdr->light_table, HT = hdr->heavy_table, DLB = hdr->light_b, RW = hdr->gs_max;
    const Layout L =
        count_layout(nw, DL, DW, DB, GM, RW, HC, LT, HT, DLB, ETA, (phases & 1u) != 0, (phases & 2u) != 0);
    const WaveView V = wave_view(lds + wid * L.misc.bytes, L.misc);
    uint8_t* uni = lds + L.union_off;
    __shared__ uint32_t s_tile;

    for (uint32_t i = lane; i < HC; i += 64) V.hist[i] = 0;
    if (lane == 0) *V.hits = 0;
    JobRegs J;
    int cur = -1;

    // phase 1: long lists, one apex per workgroup
    if (phases & 1u) {
        const TeamView T = team_view(uni, L.heavy, DW, DB, HT);
        const uint32_t total = hdr->heavy_total;
        uint32_t q = blockIdx.x % kQueues, left = kQueues;  // used by thread 0
        for (;;) {
            if (threadIdx.x == 0) s_tile = claim_tile(hdr->queues + kHeavyQueue, total, q, left);
            __syncthreads();
            const uint32_t tile = s_tile;
            __syncthreads();
            if (tile >= total) break;
            const uint32_t j = find_job(jobs, njobs, tile, true);
            if ((int)j != cur) {
                flush_hist(J, V, cur);
                load_job(jobs + j, HC, J);
                cur = (int)j;
            }
            __syncthreads();
            const uint32_t a = J.apex[jobs[j].unit0 + (tile - jobs[j].heavy_prefix)];
            const uint32_t s0 = J.off[a], r0 = J.roff[a];
            count_apex<true, ETA>(J, T, V, a, s0, J.off[a + 1] - s0, r0, J.roff[a + 1] - r0);
        }
    }
    __syncthreads();  // the union area changes owners

    // phase 2: short lists, one apex per wavefront
    if (phases & 2u) {
        const TeamView T = team_view(uni + wid * L.light.bytes, L.light, DL, DLB, LT);
        const uint32_t total = hdr->light_total, tile_len = hdr->light_tile;
        uint32_t q = (blockIdx.x * nw + wid) % kQueues, left = kQueues;  // used by lane 0
        for (;;) {
            uint32_t tile = 0;
            if (lane == 0) tile = claim_tile(hdr->queues + kLightQueue, total, q, left);
            tile = lane_val(tile, 0);
            if (tile >= total) break;
            const uint32_t j = find_job(jobs, njobs, tile, false);
            if ((int)j != cur) {
                flush_hist(J, V, cur);
                load_job(jobs + j, HC, J);
                cur = (int)j;
                wave_sync();
            }
            const JobDev& JD = jobs[j];
            const uint32_t ub = JD.unit0 + JD.n_heavy + (tile - JD.light_prefix) * tile_len;
            const uint32_t ue = (ub + tile_len) < JD.unit1 ? (ub + tile_len) : JD.unit1;
            // the tile's apexes and their list bounds, loaded together (lane i: unit ub + i), then
            // handed to the unit loop in scalar registers
            uint32_t ta = 0, ts = 0, td = 0, tr = 0, trn = 0;
            if (ub + lane < ue) {
                ta = ldg(J.apex + ub + lane);
                ts = ldg(J.off + ta);
                td = ldg(J.off + ta + 1) - ts;
                tr = ldg(J.roff + ta);
                trn = ldg(J.roff + ta + 1) - tr;
            }
            for (uint32_t u = 0; u < ue - ub; ++u)
                count_apex<false, ETA>(J, T, V, lane_val(ta, u), lane_val(ts, u), lane_val(td, u), lane_val(tr, u),
                                       lane_val(trn, u));
        }
    }
    flush_hist(J, V, cur);
}

// ======================================================================= hash slots ======

struct HashParams {
    uint64_t hp[4 * REPT_GMAX];
};

__global__ void k_slots(HashParams P, uint32_t G, uint32_t m, const uint2* __restrict__ edges, uint64_t E,
                        uint32_t* __restrict__ slots) {
    for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < E;
         t += (uint64_t)gridDim.x * blockDim.x) {
        const uint2 e = edges[t];
        for (uint32_t g = 0; g < G; ++g) slots[(uint64_t)g * E + t] = slot_of(P.hp + 4 * g, m, e.x, e.y);
    }
}

// sums[v] = sum over the rows of local[r][v] (exact int64).  Each thread reads every row at its
// own v before writing sums[v], so sums may be local's first row.
__global__ void k_reduce_rows(const int64_t* local, uint32_t rows, uint32_t n, int64_t* sums) {
    for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        int64_t acc = 0;
        for (uint32_t r = 0; r < rows; ++r) acc += local[(uint64_t)r * n + v];
        sums[v] = acc;
    }
}

bool g_attr_set = false;

// Second stream of the current device for the light-phase launch, and the fork and join
// events around it (created on first use, default priority, kept for the process).  One
// enqueue sequence at a time: the events are re-recorded by every launch.
struct AuxStream {
    int device = -1;
    hipStream_t stream = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
};
std::mutex g_aux_mu;
AuxStream g_aux[16];
hipError_t aux_for_current(AuxStream** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= 16) return hipErrorInvalidDevice;
    AuxStream& a = g_aux[dev];
    if (a.device != dev) {
        if ((e = hipStreamCreateWithFlags(&a.stream, hipStreamNonBlocking)) != hipSuccess) return e;
        if ((e = hipEventCreateWithFlags(&a.fork, hipEventDisableTiming)) != hipSuccess) return e;
        if ((e = hipEventCreateWithFlags(&a.join, hipEventDisableTiming)) != hipSuccess) return e;
        a.device = dev;
    }
    *out = &a;
    return hipSuccess;
}

hipError_t report(hipError_t e, const char* what) {
    if (e != hipSuccess) fprintf(stderr, "rept: %s failed: %s\n", what, hipGetErrorString(e));
    return e;
}

hipError_t set_attrs() {
    if (g_attr_set) return hipSuccess;
    // the kernel's static LDS (a few bytes) and the dynamic part share the CU's 160 KB
    hipError_t e = hipFuncSetAttribute((const void*)k_count<false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       160 * 1024 - 256);
    if (e != hipSuccess) return report(e, "hipFuncSetAttribute(k_count)");
    e = hipFuncSetAttribute((const void*)k_count<true>, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024 - 256);
    if (e != hipSuccess) return report(e, "hipFuncSetAttribute(k_count, pair counters)");
    g_attr_set = true;
    return hipSuccess;
}

hipError_t launch_common(uint8_t* ws, const BatchHeader& h, hipStream_t s) {
    (void)hipGetLastError();  // launch errors below are this call's own
    hipError_t e = set_attrs();
    if (e != hipSuccess) return e;
    BatchHeader* hdr = (BatchHeader*)ws;
    JobDev* jobs = (JobDev*)(ws + sizeof(BatchHeader));
    hipLaunchKernelGGL(k_setup, dim3(1), dim3(1024), 0, s, hdr, jobs);
    if (h.any_zero) {
        uint64_t blocks = (h.zero_words + 255) / 256;
        if (blocks > 1024) blocks = 1024;
        if (blocks < 1) blocks = 1;
        hipLaunchKernelGGL(k_zero, dim3((uint32_t)blocks, h.njobs), dim3(256), 0, s, hdr, jobs);
    }
    if (h.any_fill) {
        uint64_t blocks = (h.fill_edges + FILL_CHUNK - 1) / FILL_CHUNK;
        if (blocks > 8192) blocks = 8192;
        if (blocks < 1) blocks = 1;
        hipLaunchKernelGGL(k_fill, dim3((uint32_t)blocks, h.njobs), dim3(256), 0, s, jobs);
    }
    // heavy and light phases in one launch, or the light phase in a launch of its own (a
    // light-only workgroup needs no heavy team area, so more wavefronts fit per CU)
    // (split: the light launch on a second stream, forked after the setup kernels and joined
    // back, so that it runs beside the heavy launch as workgroups free the CUs)
    const uint32_t first = h.split ? 1u : 3u;
    std::unique_lock<std::mutex> lk(g_aux_mu, std::defer_lock);
    AuxStream* aux = nullptr;
    hipStream_t ls = s;
    if (h.split && h.split_streams) {
        lk.lock();
        if ((e = aux_for_current(&aux)) != hipSuccess) return report(e, "second stream");
        if ((e = hipEventRecord(aux->fork, s)) != hipSuccess) return report(e, "fork event");
        if ((e = hipStreamWaitEvent(aux->stream, aux->fork, 0)) != hipSuccess) return report(e, "fork wait");
        ls = aux->stream;
    }
    if (h.any_eta) hipLaunchKernelGGL(k_count<true>, dim3(h.blocks), dim3(h.threads), h.lds_bytes, s, hdr, jobs, first);
    else hipLaunchKernelGGL(k_count<false>, dim3(h.blocks), dim3(h.threads), h.lds_bytes, s, hdr, jobs, first);
    if (h.split) {
        if (h.any_eta)
            hipLaunchKernelGGL(k_count<true>, dim3(h.light_blocks), dim3(h.light_threads), h.light_lds, ls, hdr, jobs,
                               2u);
        else
            hipLaunchKernelGGL(k_count<false>, dim3(h.light_blocks), dim3(h.light_threads), h.light_lds, ls, hdr, jobs,
                               2u);
    }
    if ((e = hipGetLastError()) != hipSuccess) return report(e, "counting kernel launch");
    if (aux) {
        if ((e = hipEventRecord(aux->join, aux->stream)) != hipSuccess) return report(e, "join event");
        if ((e = hipStreamWaitEvent(s, aux->join, 0)) != hipSuccess) return report(e, "join wait");
    }
    return hipSuccess;
}

}  // namespace

uint32_t rept_count_lds(uint32_t threads, uint32_t wave_cap, uint32_t block_cap, uint32_t b_chunk, uint32_t G,
                        uint32_t gs, uint32_t hist_c, uint32_t light_table, uint32_t heavy_table, uint32_t light_b,
                        bool eta, bool heavy, bool light) {
    return count_layout(threads / 64, wave_cap, block_cap, b_chunk, G, gs, hist_c, light_table, heavy_table, light_b,
                        eta, heavy, light).total;
}

uint32_t rept_count_blocks_per_cu(uint32_t threads, uint32_t lds_bytes, bool eta) {
    if (set_attrs() != hipSuccess) return 0;
    int nb = 0;
    const void* fn = eta ? (const void*)k_count<true> : (const void*)k_count<false>;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, (int)threads, (size_t)lds_bytes);
    if (e != hipSuccess) {
        (void)report(e, "hipOccupancyMaxActiveBlocksPerMultiprocessor(k_count)");
        (void)hipGetLastError();
        return 0;
    }
    return nb > 0 ? (uint32_t)nb : 0u;
}

hipError_t rept_launch_batch(void* ws, const BatchHeader& h, hipStream_t s) {
    return launch_common((uint8_t*)ws, h, s);
}

hipError_t rept_launch_single(uint8_t* ctrl, const BatchHeader& hdr, const JobDev& job, hipStream_t s) {
    hipLaunchKernelGGL(k_write_ctrl, dim3(1), dim3(64), 0, s, ctrl, hdr, job);
    return launch_common(ctrl, hdr, s);
}

hipError_t rept_launch_reduce(const int64_t* local, uint32_t rows, uint32_t n, int64_t* sums, hipStream_t s) {
    (void)hipGetLastError();
    uint32_t blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_reduce_rows, dim3(blocks), dim3(256), 0, s, local, rows, n, sums);
    return hipGetLastError();
}

hipError_t rept_launch_zero(void* p, uint64_t bytes, hipStream_t s) {
    (void)hipGetLastError();
    const uint64_t words = bytes / 4;
    uint64_t blocks = (words + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_zero_u32, dim3((uint32_t)blocks), dim3(256), 0, s, (uint32_t*)p, words);
    return hipGetLastError();
}

hipError_t rept_launch_eta(const rept_graph* g, const JobDev& d, int64_t* eta, int64_t* eta_v, uint32_t proc0,
                           uint32_t stride, hipStream_t s) {
    (void)hipGetLastError();
    uint64_t blocks = (g->E + FILL_CHUNK - 1) / FILL_CHUNK;
    if (blocks > 8192) blocks = 8192;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_eta, dim3((uint32_t)blocks), dim3(256), 0, s, g->off, g->nbr, g->n, (const uint16_t*)d.tab,
                       d.gs, d.G, d.m, d.c, (const uint32_t*)d.pairs, d.es, proc0, stride, eta, eta_v);
    return hipGetLastError();
}

hipError_t rept_launch_slots(const uint64_t* hp, uint32_t G, uint32_t m, const uint32_t* edges, uint64_t E,
                             uint32_t* slots, hipStream_t s) {
    HashParams P{};
    for (uint32_t i = 0; i < 4 * G && i < 4 * REPT_GMAX; ++i) P.hp[i] = hp[i];
    uint64_t blocks = (E + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_slots, dim3((uint32_t)blocks), dim3(256), 0, s, P, G, m, (const uint2*)edges, E, slots);
    return hipGetLastError();
}
