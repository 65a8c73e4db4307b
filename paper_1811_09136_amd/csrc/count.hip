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
// Kernels.  k_heavy: one workgroup per apex with a long list (adjacency chunks staged in LDS);
// k_light: one wavefront per apex with a short list.  Both are persistent and drain a device
// work queue over all jobs of a batch.  Local counts are aggregated per list entry in LDS and
// global counts per processor in an LDS histogram before the 64-bit global atomics.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.h"

namespace {

constexpr uint32_t kHashMul = 0x9E3779B1u;  // table index: Fibonacci hashing of the node id
constexpr uint64_t kP61 = (1ull << 61) - 1;  // Mersenne prime of the edge hash

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint32_t o = __shfl_up(v, d, 64);
        if (lane >= d) v += o;
    }
    return v;
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

// ---- LDS layouts (shared by host sizing and device carving) ----
struct LightLayout {
    uint32_t coef, hkey, hidx, ew, et, boff, bscan, slot, cnt, acnt, hist, team;
};
__host__ __device__ inline LightLayout light_layout(uint32_t D, uint32_t G, uint32_t HC) {
    LightLayout L;
    const uint32_t H = pow2_at_least(2 * D);
    uint32_t p = 0;
    L.coef = p; p = up16(p + 8 * 4 * REPT_GMAX);
    L.hkey = p; p = up16(p + 4 * H);
    L.hidx = p; p = up16(p + 2 * H);
    L.ew = p; p = up16(p + 4 * D);
    L.et = p; p = up16(p + 4 * D);
    L.boff = p; p = up16(p + 4 * D);
    L.bscan = p; p = up16(p + 4 * (D + 1));
    L.slot = p; p = up16(p + 2 * G * D);
    L.cnt = p; p = up16(p + 4 * G * D);
    L.acnt = p; p = up16(p + 4 * REPT_GMAX);
    L.hist = p; p = up16(p + 4 * HC);
    L.team = p;
    return L;
}

struct HeavyLayout {
    uint32_t coef, hkey, hidx, ew, et, wslot, cntw, eb, etb, boff, bscan, bslot, cntb, acnt, hist, misc, total;
};
__host__ __device__ inline HeavyLayout heavy_layout(uint32_t D, uint32_t G, uint32_t HC) {
    HeavyLayout L;
    const uint32_t H = pow2_at_least(2 * D);
    uint32_t p = 0;
    L.coef = p; p = up16(p + 8 * 4 * REPT_GMAX);
    L.hkey = p; p = up16(p + 4 * H);
    L.hidx = p; p = up16(p + 2 * H);
    L.ew = p; p = up16(p + 4 * D);
    L.et = p; p = up16(p + 4 * D);
    L.wslot = p; p = up16(p + 2 * G * D);
    L.cntw = p; p = up16(p + 4 * G * D);
    L.eb = p; p = up16(p + 4 * D);
    L.etb = p; p = up16(p + 4 * D);
    L.boff = p; p = up16(p + 4 * D);
    L.bscan = p; p = up16(p + 4 * (D + 1));
    L.bslot = p; p = up16(p + 2 * G * D);
    L.cntb = p; p = up16(p + 4 * G * D);
    L.acnt = p; p = up16(p + 4 * REPT_GMAX);
    L.hist = p; p = up16(p + 4 * HC);
    L.misc = p; p = up16(p + 4 * 64);
    L.total = p;
    return L;
}

// ---- per-job constants held while a team works on that job ----
struct JobRegs {
    const uint32_t* off;
    const uint32_t* nbr;
    const uint32_t* tim;
    const uint32_t* apex;
    int64_t* global;
    int64_t* local;
    uint32_t n, m, c, G, per_proc, t0, t1, last_ck;
};

__device__ inline void load_job(const JobDev* __restrict__ j, JobRegs& r) {
    r.off = j->off;
    r.nbr = j->nbr;
    r.tim = j->tim;
    r.apex = j->apex;
    r.global = j->global;
    r.local = j->local;
    r.n = j->n;
    r.m = j->m;
    r.c = j->c;
    r.G = j->G;
    r.per_proc = j->per_proc;
    r.t0 = j->t0;
    r.t1 = j->t1;
    r.last_ck = j->c - (j->G - 1) * j->m;
}

// ---- edge hash: degree-3 polynomial over GF(2^61 - 1), Horner form ----
__device__ __forceinline__ uint64_t fold61(uint64_t r) {  // r < 2^62 -> [0, p)
    r = (r & kP61) + (r >> 61);
    return r >= kP61 ? r - kP61 : r;
}
__device__ __forceinline__ uint64_t mulmod61(uint64_t a, uint64_t b) {  // a, b < 2^61
    const uint64_t lo = a * b;
    const uint64_t hi = __umul64hi(a, b);  // product < 2^122
    return fold61((lo & kP61) + ((hi << 3) | (lo >> 61)));
}
// slot of the undirected edge {x, y} for the group whose coefficients are c4[0..3]
__device__ __forceinline__ uint32_t slot_of(const uint64_t* c4, uint32_t m, uint32_t x, uint32_t y) {
    const uint32_t lo = x < y ? x : y, hi = x < y ? y : x;
    const uint64_t key = ((uint64_t)lo << 32) | hi;  // < 2^61 - 1 for ids below 2^29
    uint64_t h = c4[3];
    h = fold61(mulmod61(h, key) + c4[2]);
    h = fold61(mulmod61(h, key) + c4[1]);
    h = fold61(mulmod61(h, key) + c4[0]);
    return (uint32_t)__umul64hi(h << 3, (uint64_t)m);
}

// Attribute the triangle (a, b, w) with edge times t_ab, t_aw, t_bw.  The first two edges by
// time are looked up (apex edges: staged slots s_ab(g), s_aw(g)) or hashed ({b, w}); for
// every group whose slots agree on an active processor, sink(g, processor) is called.
template <typename SAB, typename SAW, typename Sink>
__device__ __forceinline__ void attribute(const JobRegs& J, const uint64_t* coef, uint32_t b, uint32_t w,
                                          uint32_t tab, uint32_t taw, uint32_t tbw, SAB&& s_ab, SAW&& s_aw,
                                          Sink&& sink) {
    // which edge arrived last: 0 = {a,b}, 1 = {a,w}, 2 = {b,w} (arrival times are distinct)
    const uint32_t last = (tab > taw && tab > tbw) ? 0u : (taw > tbw ? 1u : 2u);
    const uint32_t tl = last == 0 ? tab : (last == 1 ? taw : tbw);
    if (tl < J.t0 || tl >= J.t1) return;
    for (uint32_t g = 0; g < J.G; ++g) {
        {
            uint32_t s1, s2;
            if (last == 2) {
                s1 = s_ab(g);
                s2 = s_aw(g);
            } else {
                s1 = last == 0 ? s_aw(g) : s_ab(g);
                s2 = slot_of(coef + 4 * g, J.m, b, w);
            }
            const uint32_t ck = (g + 1 < J.G) ? J.m : J.last_ck;
            if (s1 == s2 && s1 < ck) sink(g, g * J.m + s1);
        }
    }
}

__device__ __forceinline__ void add64(int64_t* p, uint64_t v) {
    atomicAdd((unsigned long long*)p, (unsigned long long)v);
}

__device__ __forceinline__ void hash_insert(uint32_t* hkey, uint16_t* hidx, uint32_t bits, uint32_t w,
                                            uint32_t i) {
    const uint32_t mask = (1u << bits) - 1u;
    uint32_t h = (w * kHashMul) >> (32 - bits);
    for (;;) {
        uint32_t old = atomicCAS(&hkey[h], 0u, w + 1u);
        if (old == 0u) {
            hidx[h] = (uint16_t)i;
            return;
        }
        h = (h + 1u) & mask;
    }
}

__device__ __forceinline__ int hash_find(const uint32_t* hkey, const uint16_t* hidx, uint32_t bits, uint32_t w) {
    const uint32_t mask = (1u << bits) - 1u;
    uint32_t h = (w * kHashMul) >> (32 - bits);
    for (;;) {
        uint32_t k = hkey[h];
        if (k == w + 1u) return hidx[h];
        if (k == 0u) return -1;
        h = (h + 1u) & mask;
    }
}

// largest i in [0, cnt) with scan[i] <= it, given scan[0] <= it < scan[cnt]
__device__ __forceinline__ uint32_t find_seg(const uint32_t* scan, uint32_t cnt, uint32_t it) {
    uint32_t lo = 0, hi = cnt;
    while (hi - lo > 1) {
        uint32_t mid = (lo + hi) >> 1;
        if (scan[mid] <= it) lo = mid; else hi = mid;
    }
    return lo;
}

// find the job owning queue position `tile` (largest j with prefix[j] <= tile)
__device__ __forceinline__ uint32_t find_job(const JobDev* jobs, uint32_t njobs, uint32_t tile, bool heavy) {
    uint32_t lo = 0, hi = njobs;
    while (hi - lo > 1) {
        uint32_t mid = (lo + hi) >> 1;
        uint32_t p = heavy ? jobs[mid].heavy_prefix : jobs[mid].light_prefix;
        if (p <= tile) lo = mid; else hi = mid;
    }
    return lo;
}

// ======================================================================= setup / zero ====

__global__ void k_write_ctrl(uint8_t* ctrl, BatchHeader hdr, JobDev job) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        *(BatchHeader*)ctrl = hdr;
        *(JobDev*)(ctrl + sizeof(BatchHeader)) = job;
    }
}

__global__ void k_setup(BatchHeader* hdr, JobDev* jobs) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const uint32_t nj = hdr->njobs, cap = hdr->wave_cap, lt = hdr->light_tile;
    uint32_t hp = 0, lp = 0;
    for (uint32_t j = 0; j < nj; ++j) {
        JobDev& J = jobs[j];
        // apexes are sorted by out-degree, descending: the ones above `cap` form a prefix
        uint32_t lo = 0, hi = J.unit1;  // first index whose out-degree <= cap (unit1 <= num_apex)
        while (lo < hi) {
            uint32_t mid = (lo + hi) >> 1;
            uint32_t a = J.apex[mid];
            if (J.off[a + 1] - J.off[a] > cap) lo = mid + 1; else hi = mid;
        }
        const uint32_t hb = lo;
        const uint32_t u0 = J.unit0, u1 = J.unit1;
        const uint32_t hend = u1 < hb ? u1 : hb;
        J.n_heavy = hend > u0 ? hend - u0 : 0;
        const uint32_t lunits = u1 - u0 - J.n_heavy;
        J.light_tiles = (lunits + lt - 1) / lt;
        J.heavy_prefix = hp;
        J.light_prefix = lp;
        hp += J.n_heavy;
        lp += J.light_tiles;
    }
    hdr->heavy_total = hp;
    hdr->light_total = lp;
    hdr->q_heavy = 0;
    hdr->q_light = 0;
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

// ======================================================================= light kernel ====

__global__ void __launch_bounds__(256) k_light(BatchHeader* hdr, const JobDev* __restrict__ jobs) {
    extern __shared__ __align__(16) uint8_t lds[];
    const uint32_t lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const uint32_t D = hdr->wave_cap, GM = hdr->G_max, HC = hdr->hist_c;
    const uint32_t njobs = hdr->njobs, total = hdr->light_total, tile_len = hdr->light_tile;
    const LightLayout L = light_layout(D, GM, HC);
    uint8_t* base = lds + wid * L.team;
    uint64_t* coef = (uint64_t*)(base + L.coef);
    uint32_t* hkey = (uint32_t*)(base + L.hkey);
    uint16_t* hidx = (uint16_t*)(base + L.hidx);
    uint32_t* ew = (uint32_t*)(base + L.ew);
    uint32_t* et = (uint32_t*)(base + L.et);
    uint32_t* boff = (uint32_t*)(base + L.boff);
    uint32_t* bscan = (uint32_t*)(base + L.bscan);
    uint16_t* eslot = (uint16_t*)(base + L.slot);
    uint32_t* cnt = (uint32_t*)(base + L.cnt);
    uint32_t* acnt = (uint32_t*)(base + L.acnt);
    uint32_t* hist = (uint32_t*)(base + L.hist);

    for (uint32_t i = lane; i < HC; i += 64) hist[i] = 0;
    wave_sync();

    JobRegs J;
    int cur = -1;
    uint64_t since_flush = 0;

    auto flush_hist = [&]() {
        if (cur >= 0 && HC && J.c <= HC) {  // jobs with c > HC bypass the histogram
            wave_sync();
            for (uint32_t p = lane; p < J.c; p += 64) {
                uint32_t v = hist[p];
                if (v) {
                    add64(J.global + p, v);
                    hist[p] = 0;
                }
            }
            wave_sync();
        }
        since_flush = 0;
    };

    for (;;) {
        uint32_t tile = 0;
        if (lane == 0) tile = atomicAdd(&hdr->q_light, 1u);
        tile = __shfl(tile, 0, 64);
        if (tile >= total) break;
        const uint32_t j = find_job(jobs, njobs, tile, false);
        if ((int)j != cur) {
            flush_hist();
            load_job(jobs + j, J);
            if (lane < 4 * REPT_GMAX) coef[lane] = jobs[j].hp[lane];
            cur = (int)j;
            wave_sync();
        }
        const JobDev& JD = jobs[j];
        const uint32_t ub = JD.unit0 + JD.n_heavy + (tile - JD.light_prefix) * tile_len;
        uint32_t ue = ub + tile_len;
        if (ue > JD.unit1) ue = JD.unit1;
        const bool use_hist = HC != 0 && J.c <= HC;

        for (uint32_t u = ub; u < ue; ++u) {
            const uint32_t a = J.apex[u];
            const uint32_t s = J.off[a], d = J.off[a + 1] - s;
            const uint32_t bits = log2u(pow2_at_least(2 * d));
            const uint32_t Ha = 1u << bits;
            for (uint32_t i = lane; i < Ha; i += 64) hkey[i] = 0;
            if (!J.per_proc) {
                for (uint32_t g = 0; g < J.G; ++g)
                    for (uint32_t i = lane; i < d; i += 64) cnt[g * D + i] = 0;
                if (lane < REPT_GMAX) acnt[lane] = 0;
            }
            wave_sync();
            // stage a's list: ids, times, slots of the edges {a, x}, hash table, list scan
            uint32_t run = 0;
            for (uint32_t c0 = 0; c0 < d; c0 += 64) {
                const uint32_t i = c0 + lane;
                uint32_t bd = 0;
                if (i < d) {
                    const uint32_t w = J.nbr[s + i];
                    ew[i] = w;
                    et[i] = J.tim[s + i];
                    const uint32_t bo = J.off[w];
                    bd = J.off[w + 1] - bo;
                    boff[i] = bo;
                    for (uint32_t g = 0; g < J.G; ++g) eslot[g * D + i] = (uint16_t)slot_of(coef + 4 * g, J.m, a, w);
                    hash_insert(hkey, hidx, bits, w, i);
                }
                const uint32_t inc = wave_incl_scan(bd);
                if (i < d) bscan[i] = run + inc - bd;
                run += __shfl(inc, 63, 64);
            }
            if (lane == 0) bscan[d] = run;
            wave_sync();
            const uint32_t T = run;
            for (uint32_t b0 = 0; b0 < T; b0 += 64) {
                const uint32_t it = b0 + lane;
                if (it < T) {
                    const uint32_t i = find_seg(bscan, d, it);
                    const uint32_t p = boff[i] + (it - bscan[i]);
                    const uint32_t w = J.nbr[p];
                    const int k = hash_find(hkey, hidx, bits, w);
                    if (k >= 0) {
                        const uint32_t b = ew[i];
                        attribute(
                            J, coef, b, w, et[i], et[k], J.tim[p], [&](uint32_t g) { return (uint32_t)eslot[g * D + i]; },
                            [&](uint32_t g) { return (uint32_t)eslot[g * D + k]; },
                            [&](uint32_t g, uint32_t proc) {
                                if (use_hist) atomicAdd(&hist[proc], 1u);
                                else add64(J.global + proc, 1);
                                if (J.per_proc) {
                                    int64_t* row = J.local + (uint64_t)proc * J.n;
                                    add64(row + a, 1);
                                    add64(row + b, 1);
                                    add64(row + w, 1);
                                } else {
                                    atomicAdd(&acnt[g], 1u);
                                    atomicAdd(&cnt[g * D + i], 1u);
                                    atomicAdd(&cnt[g * D + k], 1u);
                                }
                            });
                    }
                }
            }
            wave_sync();
            if (!J.per_proc) {
                for (uint32_t g = 0; g < J.G; ++g) {
                    int64_t* row = J.local + (uint64_t)g * J.n;
                    for (uint32_t i = lane; i < d; i += 64) {
                        const uint32_t v = cnt[g * D + i];
                        if (v) add64(row + ew[i], v);
                    }
                }
                if (lane < J.G) {
                    const uint32_t v = acnt[lane];
                    if (v) add64(J.local + (uint64_t)lane * J.n + a, v);
                }
            }
            wave_sync();
            since_flush += T;
            if (since_flush > (1ull << 30)) flush_hist();
        }
    }
    flush_hist();
}

// ======================================================================= heavy kernel ====

__device__ uint32_t block_excl_scan(uint32_t v, uint32_t* wsum, uint32_t& total) {
    const uint32_t lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const uint32_t inc = wave_incl_scan(v);
    if (lane == 63) wsum[wid] = inc;
    __syncthreads();
    uint32_t pre = 0, tot = 0;
    for (uint32_t w = 0; w < nw; ++w) {
        const uint32_t x = wsum[w];
        if (w < wid) pre += x;
        tot += x;
    }
    __syncthreads();
    total = tot;
    return pre + inc - v;
}

__global__ void __launch_bounds__(1024) k_heavy(BatchHeader* hdr, const JobDev* __restrict__ jobs) {
    extern __shared__ __align__(16) uint8_t lds[];
    const uint32_t tid = threadIdx.x, nt = blockDim.x;
    const uint32_t D = hdr->block_cap, GM = hdr->G_max, HC = hdr->hist_c;
    const uint32_t njobs = hdr->njobs, total = hdr->heavy_total;
    const HeavyLayout L = heavy_layout(D, GM, HC);
    uint64_t* coef = (uint64_t*)(lds + L.coef);
    uint32_t* hkey = (uint32_t*)(lds + L.hkey);
    uint16_t* hidx = (uint16_t*)(lds + L.hidx);
    uint32_t* ew = (uint32_t*)(lds + L.ew);
    uint32_t* et = (uint32_t*)(lds + L.et);
    uint16_t* wslot = (uint16_t*)(lds + L.wslot);
    uint32_t* cntw = (uint32_t*)(lds + L.cntw);
    uint32_t* eb = (uint32_t*)(lds + L.eb);
    uint32_t* etb = (uint32_t*)(lds + L.etb);
    uint32_t* boff = (uint32_t*)(lds + L.boff);
    uint32_t* bscan = (uint32_t*)(lds + L.bscan);
    uint16_t* bslot = (uint16_t*)(lds + L.bslot);
    uint32_t* cntb = (uint32_t*)(lds + L.cntb);
    uint32_t* acnt = (uint32_t*)(lds + L.acnt);
    uint32_t* hist = (uint32_t*)(lds + L.hist);
    uint32_t* misc = (uint32_t*)(lds + L.misc);  // [0]: tile, [16..31]: wave sums

    for (uint32_t i = tid; i < HC; i += nt) hist[i] = 0;
    __syncthreads();

    JobRegs J;
    int cur = -1;
    uint64_t since_flush = 0;
    auto flush_hist = [&]() {
        if (cur >= 0 && HC && J.c <= HC) {  // jobs with c > HC bypass the histogram
            __syncthreads();
            for (uint32_t p = tid; p < J.c; p += nt) {
                const uint32_t v = hist[p];
                if (v) {
                    add64(J.global + p, v);
                    hist[p] = 0;
                }
            }
            __syncthreads();
        }
        since_flush = 0;
    };

    for (;;) {
        if (tid == 0) misc[0] = atomicAdd(&hdr->q_heavy, 1u);
        __syncthreads();
        const uint32_t tile = misc[0];
        __syncthreads();
        if (tile >= total) break;
        const uint32_t j = find_job(jobs, njobs, tile, true);
        if ((int)j != cur) {
            flush_hist();
            load_job(jobs + j, J);
            if (tid < 4 * REPT_GMAX) coef[tid] = jobs[j].hp[tid];
            cur = (int)j;
            __syncthreads();
        }
        const bool use_hist = HC != 0 && J.c <= HC;
        const uint32_t a = J.apex[jobs[j].unit0 + (tile - jobs[j].heavy_prefix)];
        const uint32_t s = J.off[a], d = J.off[a + 1] - s;
        if (tid < REPT_GMAX) acnt[tid] = 0;

        for (uint32_t ws = 0; ws < d; ws += D) {
            const uint32_t wn = (d - ws) < D ? (d - ws) : D;
            const uint32_t bits = log2u(pow2_at_least(2 * wn));
            const uint32_t Ha = 1u << bits;
            for (uint32_t i = tid; i < Ha; i += nt) hkey[i] = 0;
            if (!J.per_proc)
                for (uint32_t x = tid; x < J.G * wn; x += nt) cntw[(x / wn) * D + (x % wn)] = 0;
            __syncthreads();
            for (uint32_t i = tid; i < wn; i += nt) {
                const uint32_t w = J.nbr[s + ws + i];
                ew[i] = w;
                et[i] = J.tim[s + ws + i];
                for (uint32_t g = 0; g < J.G; ++g) wslot[g * D + i] = (uint16_t)slot_of(coef + 4 * g, J.m, a, w);
                hash_insert(hkey, hidx, bits, w, i);
            }
            __syncthreads();
            for (uint32_t bs = 0; bs < d; bs += D) {
                const uint32_t bn = (d - bs) < D ? (d - bs) : D;
                uint32_t run = 0;
                for (uint32_t c0 = 0; c0 < bn; c0 += nt) {
                    const uint32_t i = c0 + tid;
                    uint32_t bd = 0;
                    if (i < bn) {
                        const uint32_t b = J.nbr[s + bs + i];
                        eb[i] = b;
                        etb[i] = J.tim[s + bs + i];
                        const uint32_t bo = J.off[b];
                        bd = J.off[b + 1] - bo;
                        boff[i] = bo;
                        for (uint32_t g = 0; g < J.G; ++g) {
                            bslot[g * D + i] = (uint16_t)slot_of(coef + 4 * g, J.m, a, b);
                            if (!J.per_proc) cntb[g * D + i] = 0;
                        }
                    }
                    uint32_t tot;
                    const uint32_t ex = block_excl_scan(bd, misc + 16, tot);
                    if (i < bn) bscan[i] = run + ex;
                    run += tot;
                }
                if (tid == 0) bscan[bn] = run;
                __syncthreads();
                const uint32_t T = run;
                for (uint32_t b0 = 0; b0 < T; b0 += nt) {
                    const uint32_t it = b0 + tid;
                    if (it < T) {
                        const uint32_t i = find_seg(bscan, bn, it);
                        const uint32_t p = boff[i] + (it - bscan[i]);
                        const uint32_t w = J.nbr[p];
                        const int k = hash_find(hkey, hidx, bits, w);
                        if (k >= 0) {
                            const uint32_t b = eb[i];
                            attribute(
                                J, coef, b, w, etb[i], et[k], J.tim[p],
                                [&](uint32_t g) { return (uint32_t)bslot[g * D + i]; },
                                [&](uint32_t g) { return (uint32_t)wslot[g * D + k]; },
                                [&](uint32_t g, uint32_t proc) {
                                    if (use_hist) atomicAdd(&hist[proc], 1u);
                                    else add64(J.global + proc, 1);
                                    if (J.per_proc) {
                                        int64_t* row = J.local + (uint64_t)proc * J.n;
                                        add64(row + a, 1);
                                        add64(row + b, 1);
                                        add64(row + w, 1);
                                    } else {
                                        atomicAdd(&acnt[g], 1u);
                                        atomicAdd(&cntb[g * D + i], 1u);
                                        atomicAdd(&cntw[g * D + k], 1u);
                                    }
                                });
                        }
                    }
                }
                __syncthreads();
                if (!J.per_proc) {
                    for (uint32_t x = tid; x < J.G * bn; x += nt) {
                        const uint32_t g = x / bn, i = x % bn;
                        const uint32_t v = cntb[g * D + i];
                        if (v) add64(J.local + (uint64_t)g * J.n + eb[i], v);
                    }
                }
                __syncthreads();
                since_flush += T;
                if (since_flush > (1ull << 30)) flush_hist();
            }
            if (!J.per_proc) {
                for (uint32_t x = tid; x < J.G * wn; x += nt) {
                    const uint32_t g = x / wn, i = x % wn;
                    const uint32_t v = cntw[g * D + i];
                    if (v) add64(J.local + (uint64_t)g * J.n + ew[i], v);
                }
                if (tid < J.G) {  // a's own count, flushed per chunk to stay within 32 bits
                    const uint32_t v = acnt[tid];
                    if (v) add64(J.local + (uint64_t)tid * J.n + a, v);
                }
            }
            __syncthreads();
            if (tid < REPT_GMAX) acnt[tid] = 0;
        }
        __syncthreads();
    }
    flush_hist();
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

bool g_attr_set = false;

hipError_t set_attrs() {
    if (g_attr_set) return hipSuccess;
    hipError_t e = hipFuncSetAttribute((const void*)k_light, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute((const void*)k_heavy, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
    g_attr_set = true;
    return hipSuccess;
}

hipError_t launch_common(uint8_t* ws, const BatchHeader& h, hipStream_t s) {
    hipError_t e = set_attrs();
    if (e != hipSuccess) return e;
    BatchHeader* hdr = (BatchHeader*)ws;
    JobDev* jobs = (JobDev*)(ws + sizeof(BatchHeader));
    hipLaunchKernelGGL(k_setup, dim3(1), dim3(64), 0, s, hdr, jobs);
    if (h.any_zero) {
        uint64_t blocks = (h.zero_words + 255) / 256;
        if (blocks > 1024) blocks = 1024;
        if (blocks < 1) blocks = 1;
        hipLaunchKernelGGL(k_zero, dim3((uint32_t)blocks, h.njobs), dim3(256), 0, s, hdr, jobs);
    }
    hipLaunchKernelGGL(k_heavy, dim3(h.heavy_blocks), dim3(h.heavy_threads), h.heavy_lds, s, hdr, jobs);
    hipLaunchKernelGGL(k_light, dim3(h.light_blocks), dim3(256), h.light_lds, s, hdr, jobs);
    return hipGetLastError();
}

}  // namespace

uint32_t rept_light_lds(uint32_t wave_cap, uint32_t G, uint32_t hist_c) {
    return 4 * light_layout(wave_cap, G, hist_c).team;
}

uint32_t rept_heavy_lds(uint32_t block_cap, uint32_t G, uint32_t hist_c) {
    return heavy_layout(block_cap, G, hist_c).total;
}

hipError_t rept_launch_batch(void* ws, const BatchHeader& h, hipStream_t s) {
    return launch_common((uint8_t*)ws, h, s);
}

hipError_t rept_launch_single(uint8_t* ctrl, const BatchHeader& hdr, const JobDev& job, hipStream_t s) {
    hipLaunchKernelGGL(k_write_ctrl, dim3(1), dim3(64), 0, s, ctrl, hdr, job);
    return launch_common(ctrl, hdr, s);
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
