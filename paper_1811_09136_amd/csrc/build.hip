// Graph build for the counting pass: validation, degree orientation, and the oriented
// adjacency (neighbour id + arrival time) grouped by lower-ranked endpoint and sorted by
// neighbour id.
//
// The stream positions are the arrival times of Section II; the validation enforces the
// simple undirected graph the paper assumes.  Orientation is this library's device layout
// (not part of the paper): each undirected edge is stored once, at its endpoint of lower
// rank (degree, id), so that every triangle is reachable from exactly one apex and every
// adjacency segment is short (at most sqrt(2E) entries).
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "common.h"

namespace {

constexpr int SCAN_THREADS = 256;
constexpr int SCAN_ITEMS = 16;
constexpr int SCAN_TILE = SCAN_THREADS * SCAN_ITEMS;
constexpr int MEDIUM_MAX = 4096;  // segments sorted in LDS by one workgroup
constexpr int WAVE_MAX = 1024;    // segments sorted in registers by one wavefront each
constexpr int SMALL_MAX = 64;     // segments sorted in registers, several per wavefront

__device__ __forceinline__ bool rank_less(uint32_t x, uint32_t dx, uint32_t y, uint32_t dy) {
    return dx < dy || (dx == dy && x < y);
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

// exclusive scan of one value per thread over a 256-thread block; returns the block total
__device__ uint32_t block_excl_scan256(uint32_t v, uint32_t& total) {
    __shared__ uint32_t wsum[SCAN_THREADS / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    uint32_t inc = wave_incl_scan(v);
    if (lane == 63) wsum[wid] = inc;
    __syncthreads();
    uint32_t base = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < SCAN_THREADS / 64; ++w) {
        if (w < wid) base += wsum[w];
        tot += wsum[w];
    }
    __syncthreads();
    total = tot;
    return base + inc - v;
}

template <typename T>
__device__ T block_reduce_sum256(T v) {
    __shared__ T red[SCAN_THREADS / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    if (lane == 0) red[wid] = v;
    __syncthreads();
    T s = 0;
    if (threadIdx.x == 0)
        for (int w = 0; w < SCAN_THREADS / 64; ++w) s += red[w];
    __syncthreads();
    return s;  // valid in thread 0
}

// ---------------------------------------------------------------- exclusive scan (u32) ----

__global__ void __launch_bounds__(SCAN_THREADS) k_scan_reduce(const uint32_t* __restrict__ in, uint64_t N,
                                                               uint32_t* __restrict__ part) {
    const uint64_t base = (uint64_t)blockIdx.x * SCAN_TILE;
    uint32_t s = 0;
    for (int r = 0; r < SCAN_ITEMS; ++r) {
        uint64_t i = base + (uint64_t)r * SCAN_THREADS + threadIdx.x;
        if (i < N) s += in[i];
    }
    uint32_t t = block_reduce_sum256<uint32_t>(s);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

__global__ void __launch_bounds__(1024) k_scan_top(uint32_t* part, uint32_t nparts) {
    __shared__ uint32_t wsum[16];
    __shared__ uint32_t carry;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (uint32_t base = 0; base < nparts; base += 1024) {
        uint32_t i = base + threadIdx.x;
        uint32_t v = i < nparts ? part[i] : 0;
        uint32_t inc = wave_incl_scan(v);
        if (lane == 63) wsum[wid] = inc;
        __syncthreads();
        uint32_t pre = 0, tot = 0;
        for (int w = 0; w < 16; ++w) {
            if (w < wid) pre += wsum[w];
            tot += wsum[w];
        }
        uint32_t c = carry;
        if (i < nparts) part[i] = c + pre + inc - v;
        __syncthreads();
        if (threadIdx.x == 0) carry = c + tot;
        __syncthreads();
    }
}

// out[i] = sum of in[0..i), out[N] = total
__global__ void __launch_bounds__(SCAN_THREADS) k_scan_down(const uint32_t* __restrict__ in, uint64_t N,
                                                             const uint32_t* __restrict__ part,
                                                             uint32_t* __restrict__ out) {
    const uint64_t base = (uint64_t)blockIdx.x * SCAN_TILE + (uint64_t)threadIdx.x * SCAN_ITEMS;
    uint32_t v[SCAN_ITEMS];
    uint32_t s = 0;
#pragma unroll
    for (int r = 0; r < SCAN_ITEMS; ++r) {
        uint64_t i = base + r;
        v[r] = i < N ? in[i] : 0;
        s += v[r];
    }
    uint32_t total;
    uint32_t pre = block_excl_scan256(s, total) + part[blockIdx.x];
#pragma unroll
    for (int r = 0; r < SCAN_ITEMS; ++r) {
        uint64_t i = base + r;
        if (i < N) out[i] = pre;
        pre += v[r];
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == SCAN_THREADS - 1) out[N] = pre;
}

// ---------------------------------------------------------------- build kernels ----------

__global__ void k_fill_u32(uint32_t* p, uint64_t count, uint32_t v) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// ---- degrees without global atomics: endpoints are partitioned into buckets of 2^shift
// consecutive ids (at most DEG_BUCKETS buckets, one LDS histogram per workgroup), then each
// bucket is counted by one workgroup in LDS.  Hub ids therefore never contend in memory.
constexpr uint32_t DEG_BUCKETS = 4096;
constexpr uint32_t DEG_SUB = 8192;  // ids counted per LDS pass

// per-workgroup bucket histogram of the endpoints of its edge range, with the range and
// self-loop checks of the stream (invalid edges contribute nothing)
__global__ void __launch_bounds__(1024) k_deg_hist(const uint2* __restrict__ edges, uint64_t E, uint32_t n,
                                                   uint32_t shift, uint32_t NB, uint64_t per_block,
                                                   uint32_t* __restrict__ bhist, BuildStats* st) {
    __shared__ uint32_t h[DEG_BUCKETS];
    for (uint32_t i = threadIdx.x; i < NB; i += blockDim.x) h[i] = 0;
    __syncthreads();
    const uint64_t e0 = (uint64_t)blockIdx.x * per_block;
    const uint64_t e1 = (e0 + per_block) < E ? (e0 + per_block) : E;
    uint32_t bad = 0;
    for (uint64_t t = e0 + threadIdx.x; t < e1; t += blockDim.x) {
        const uint2 e = edges[t];
        if (e.x >= n || e.y >= n) {
            bad |= RF_RANGE;
            continue;
        }
        if (e.x == e.y) {
            bad |= RF_SELFLOOP;
            continue;
        }
        atomicAdd(&h[e.x >> shift], 1u);
        atomicAdd(&h[e.y >> shift], 1u);
    }
    if (bad) atomicOr(&st->flags, bad);
    __syncthreads();
    for (uint32_t b = threadIdx.x; b < NB; b += blockDim.x) bhist[(uint64_t)b * gridDim.x + blockIdx.x] = h[b];
}

// write every valid endpoint id into its bucket's range (order within a bucket is free)
__global__ void __launch_bounds__(1024) k_deg_scatter(const uint2* __restrict__ edges, uint64_t E, uint32_t n,
                                                      uint32_t shift, uint32_t NB, uint64_t per_block,
                                                      const uint32_t* __restrict__ boff, uint32_t* __restrict__ part) {
    __shared__ uint32_t base[DEG_BUCKETS];
    for (uint32_t b = threadIdx.x; b < NB; b += blockDim.x) base[b] = boff[(uint64_t)b * gridDim.x + blockIdx.x];
    __syncthreads();
    const uint64_t e0 = (uint64_t)blockIdx.x * per_block;
    const uint64_t e1 = (e0 + per_block) < E ? (e0 + per_block) : E;
    for (uint64_t t = e0 + threadIdx.x; t < e1; t += blockDim.x) {
        const uint2 e = edges[t];
        if (e.x >= n || e.y >= n || e.x == e.y) continue;
        part[atomicAdd(&base[e.x >> shift], 1u)] = e.x;
        part[atomicAdd(&base[e.y >> shift], 1u)] = e.y;
    }
}

// Second pass of the endpoint partition: the first pass wrote the endpoints by super-bucket
// (at most 64 of them, so each workgroup's writes formed few, long runs); ranges of that output
// are partitioned again by the final bucket.  A range lies in one or two super-buckets, so a
// workgroup again writes few runs, and the scattered writes stay close to whole lines.
// `ntot`: the number of endpoints (the first pass's scan total).
__global__ void __launch_bounds__(1024) k_ids_hist(const uint32_t* __restrict__ ids, const uint32_t* __restrict__ ntot,
                                                   uint32_t shift, uint32_t NB, uint64_t per_block,
                                                   uint32_t* __restrict__ bhist) {
    __shared__ uint32_t h[DEG_BUCKETS];
    for (uint32_t i = threadIdx.x; i < NB; i += blockDim.x) h[i] = 0;
    __syncthreads();
    const uint64_t N = *ntot;
    const uint64_t e0 = (uint64_t)blockIdx.x * per_block;
    const uint64_t e1 = (e0 + per_block) < N ? (e0 + per_block) : N;
    for (uint64_t i = e0 + threadIdx.x; i < e1; i += blockDim.x) atomicAdd(&h[ids[i] >> shift], 1u);
    __syncthreads();
    for (uint32_t b = threadIdx.x; b < NB; b += blockDim.x) bhist[(uint64_t)b * gridDim.x + blockIdx.x] = h[b];
}

__global__ void __launch_bounds__(1024) k_ids_scatter(const uint32_t* __restrict__ ids, const uint32_t* __restrict__ ntot,
                                                      uint32_t shift, uint32_t NB, uint64_t per_block,
                                                      const uint32_t* __restrict__ boff, uint32_t* __restrict__ out) {
    __shared__ uint32_t base[DEG_BUCKETS];
    for (uint32_t b = threadIdx.x; b < NB; b += blockDim.x) base[b] = boff[(uint64_t)b * gridDim.x + blockIdx.x];
    __syncthreads();
    const uint64_t N = *ntot;
    const uint64_t e0 = (uint64_t)blockIdx.x * per_block;
    const uint64_t e1 = (e0 + per_block) < N ? (e0 + per_block) : N;
    for (uint64_t i = e0 + threadIdx.x; i < e1; i += blockDim.x) {
        const uint32_t x = ids[i];
        out[atomicAdd(&base[x >> shift], 1u)] = x;
    }
}

// Workgroups take fixed slices of the partitioned endpoints (so a bucket full of hubs is
// shared by many workgroups); within a slice each bucket's part is counted in LDS and added
// to the degrees with one atomic per distinct id.  `deg` must be zero on entry.
constexpr uint32_t DEG_SLICE = 65536;
__global__ void __launch_bounds__(1024) k_deg_count(const uint32_t* __restrict__ part,
                                                    const uint32_t* __restrict__ boff, uint32_t nblk, uint32_t NB,
                                                    uint32_t shift, uint32_t n, uint32_t* __restrict__ deg) {
    __shared__ uint32_t cnt[DEG_SUB];
    const uint32_t total = boff[(uint64_t)NB * nblk];
    const uint64_t span = (uint64_t)1 << shift;
    for (uint64_t s0 = (uint64_t)blockIdx.x * DEG_SLICE; s0 < total; s0 += (uint64_t)gridDim.x * DEG_SLICE) {
        const uint64_t s1 = (s0 + DEG_SLICE) < total ? (s0 + DEG_SLICE) : total;
        const uint32_t b_first = part[s0] >> shift, b_last = part[s1 - 1] >> shift;
        for (uint32_t b = b_first; b <= b_last; ++b) {
            const uint64_t start = boff[(uint64_t)b * nblk];
            const uint64_t end = (b + 1 < NB) ? boff[(uint64_t)(b + 1) * nblk] : total;
            const uint64_t lo = start > s0 ? start : s0, hi = end < s1 ? end : s1;
            if (lo >= hi) continue;
            const uint64_t v0 = (uint64_t)b << shift;
            for (uint64_t r0 = 0; r0 < span && v0 + r0 < n; r0 += DEG_SUB) {
                for (uint32_t i = threadIdx.x; i < DEG_SUB; i += blockDim.x) cnt[i] = 0;
                __syncthreads();
                for (uint64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
                    const uint64_t x = (uint64_t)part[i] - v0 - r0;
                    if (x < DEG_SUB) atomicAdd(&cnt[x], 1u);
                }
                __syncthreads();
                for (uint32_t i = threadIdx.x; i < DEG_SUB; i += blockDim.x) {
                    const uint64_t v = v0 + r0 + i;
                    if (cnt[i] && v < n) atomicAdd(&deg[v], cnt[i]);
                }
                __syncthreads();
            }
        }
    }
}

// Reverse-list counters per target on the shard path (graphs whose buckets are wider than
// DEG_SUB ids): REV_SHARDS shards (by source mod REV_SHARDS), so a hub's increments spread over
// that many addresses.
constexpr uint32_t REV_SHARDS = 8;

// an invalid edge's orientation
constexpr uint32_t NO_EDGE = 0xffffffffu;

// an oriented entry in the partition by the bucket of its lower endpoint: (a, b, t), 12 bytes
struct OEntry {
    uint32_t a, b, t;
};
// the node by whose bucket a partition entry is placed: a of an oriented entry, the target b
// (first word) of a reverse pair
__device__ __forceinline__ uint32_t entry_key(const OEntry& e) { return e.a; }
__device__ __forceinline__ uint32_t entry_key(const uint4& e) { return e.x; }

__global__ void k_copy_u32(const uint32_t* __restrict__ src, uint64_t count, uint32_t* __restrict__ dst) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (uint64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

// ---- out-degrees without global atomics: each edge is oriented from its lower- to its
// higher-ranked endpoint and partitioned by the bucket of that lower endpoint a (buckets of
// 2^shift ids, as for the degrees), and the out-degrees are counted per bucket in LDS.  (A
// placement per bucket with LDS cursors was tried too: the densest bucket, the top-degree
// nodes, held 18 times the mean of entries, and one workgroup placing it took 5.5 ms.)

// orientation ab[t] = (a, b) of every edge (NO_EDGE for an invalid one) and the per-workgroup
// histogram of the lower endpoints' buckets
__global__ void __launch_bounds__(1024) k_orient_hist(const uint2* __restrict__ edges, uint64_t E, uint32_t n,
                                                      const uint32_t* __restrict__ deg, uint32_t shift, uint32_t NB,
                                                      uint64_t per_block, uint2* __restrict__ ab,
                                                      uint32_t* __restrict__ bhist) {
    __shared__ uint32_t h[DEG_BUCKETS];
    for (uint32_t i = threadIdx.x; i < NB; i += blockDim.x) h[i] = 0;
    __syncthreads();
    const uint64_t e0 = (uint64_t)blockIdx.x * per_block;
    const uint64_t e1 = (e0 + per_block) < E ? (e0 + per_block) : E;
    for (uint64_t t = e0 + threadIdx.x; t < e1; t += blockDim.x) {
        const uint2 e = edges[t];
        if (e.x >= n || e.y >= n || e.x == e.y) {
            ab[t] = make_uint2(NO_EDGE, NO_EDGE);
            continue;
        }
        const bool xa = rank_less(e.x, deg[e.x], e.y, deg[e.y]);
        const uint32_t a = xa ? e.x : e.y, b = xa ? e.y : e.x;
        ab[t] = make_uint2(a, b);
        atomicAdd(&h[a >> shift], 1u);
    }
    __syncthreads();
    for (uint32_t b = threadIdx.x; b < NB; b += blockDim.x) bhist[(uint64_t)b * gridDim.x + blockIdx.x] = h[b];
}

// the oriented entries (a, b, t) in bucket order of a (order within a bucket is free)
__global__ void __launch_bounds__(1024) k_orient_part(const uint2* __restrict__ ab, uint64_t E, uint32_t shift,
                                                      uint32_t NB, uint64_t per_block,
                                                      const uint32_t* __restrict__ boff, OEntry* __restrict__ opart) {
    __shared__ uint32_t base[DEG_BUCKETS];
    for (uint32_t b = threadIdx.x; b < NB; b += blockDim.x) base[b] = boff[(uint64_t)b * gridDim.x + blockIdx.x];
    __syncthreads();
    const uint64_t e0 = (uint64_t)blockIdx.x * per_block;
    const uint64_t e1 = (e0 + per_block) < E ? (e0 + per_block) : E;
    for (uint64_t t = e0 + threadIdx.x; t < e1; t += blockDim.x) {
        const uint2 e = ab[t];
        if (e.x == NO_EDGE) continue;
        opart[atomicAdd(&base[e.x >> shift], 1u)] = OEntry{e.x, e.y, (uint32_t)t};
    }
}

// out-degrees: workgroups take fixed slices of the partition and count each bucket's part of
// the slice in LDS, one atomic per distinct node (`dout` zero on entry)
__global__ void __launch_bounds__(1024) k_out_count(const OEntry* __restrict__ opart,
                                                    const uint32_t* __restrict__ boff, uint32_t nblk, uint32_t NB,
                                                    uint32_t shift, uint32_t n, uint32_t* __restrict__ dout) {
    __shared__ uint32_t cnt[DEG_SUB];
    const uint32_t total = boff[(uint64_t)NB * nblk];
    const uint64_t span = (uint64_t)1 << shift;
    for (uint64_t s0 = (uint64_t)blockIdx.x * DEG_SLICE; s0 < total; s0 += (uint64_t)gridDim.x * DEG_SLICE) {
        const uint64_t s1 = (s0 + DEG_SLICE) < total ? (s0 + DEG_SLICE) : total;
        const uint32_t b_first = opart[s0].a >> shift, b_last = opart[s1 - 1].a >> shift;
        for (uint32_t b = b_first; b <= b_last; ++b) {
            const uint64_t start = boff[(uint64_t)b * nblk];
            const uint64_t end = (b + 1 < NB) ? boff[(uint64_t)(b + 1) * nblk] : total;
            const uint64_t lo = start > s0 ? start : s0, hi = end < s1 ? end : s1;
            if (lo >= hi) continue;
            const uint64_t v0 = (uint64_t)b << shift;
            for (uint64_t r0 = 0; r0 < span && v0 + r0 < n; r0 += DEG_SUB) {
                for (uint32_t i = threadIdx.x; i < DEG_SUB; i += blockDim.x) cnt[i] = 0;
                __syncthreads();
                for (uint64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
                    const uint64_t x = (uint64_t)opart[i].a - v0 - r0;
                    if (x < DEG_SUB) atomicAdd(&cnt[x], 1u);
                }
                __syncthreads();
                for (uint32_t i = threadIdx.x; i < DEG_SUB; i += blockDim.x) {
                    const uint64_t v = v0 + r0 + i;
                    if (cnt[i] && v < n) atomicAdd(&dout[v], cnt[i]);
                }
                __syncthreads();
            }
        }
    }
}

// ---- placement by slices: each bucket's part of the partition is cut into slices of
// SLICE_ENTRIES entries, one workgroup each (the densest bucket, the top-degree nodes, holds many
// times the mean).  A slice counts its entries per node of its bucket in LDS; a pass per node
// sums those counts into the out-degree and, after the scan, turns them into the node's base in
// each slice (its segment start plus its entries in the bucket's earlier slices); a slice then
// places its entries with LDS cursors from those bases.  Needs a bucket span of at most DEG_SUB
// ids (n <= 2^25).
// (R-MAT scale 24 build: 45.6-46.0 ms at 32768 entries, 45.9 at 65536, 46.9 at 16384, 48.4 at
// 8192: fewer slices per bucket write fewer per-slice counts and interleave less in each
// node's segment)
constexpr uint32_t SLICE_ENTRIES = 32768;

// slice_off[b] = first slice of bucket b (slice_off[NB] = the number of slices); one workgroup
__global__ void __launch_bounds__(1024) k_slice_plan(const uint32_t* __restrict__ boff, uint32_t nblk, uint32_t NB,
                                                     uint32_t* __restrict__ slice_off) {
    __shared__ uint32_t cnt[DEG_BUCKETS];
    const uint32_t total = boff[(uint64_t)NB * nblk];
    for (uint32_t b = threadIdx.x; b < NB; b += blockDim.x) {
        const uint32_t lo = boff[(uint64_t)b * nblk], hi = (b + 1 < NB) ? boff[(uint64_t)(b + 1) * nblk] : total;
        cnt[b] = (hi - lo + SLICE_ENTRIES - 1) / SLICE_ENTRIES;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t run = 0;
        for (uint32_t b = 0; b < NB; ++b) {
            slice_off[b] = run;
            run += cnt[b];
        }
        slice_off[NB] = run;
    }
}

// the slice of workgroup s: its bucket b and entry range [lo, hi); false past the last slice
__device__ __forceinline__ bool slice_of(uint32_t s, const uint32_t* __restrict__ slice_off,
                                         const uint32_t* __restrict__ boff, uint32_t nblk, uint32_t NB, uint32_t& b,
                                         uint64_t& lo, uint64_t& hi) {
    if (s >= slice_off[NB]) return false;
    uint32_t l = 0, h = NB;  // last bucket with slice_off[b] <= s
    while (h - l > 1) {
        const uint32_t mid = (l + h) >> 1;
        if (slice_off[mid] <= s) l = mid; else h = mid;
    }
    while (l + 1 < NB && slice_off[l + 1] <= s) ++l;  // skip buckets without slices
    b = l;
    const uint32_t total = boff[(uint64_t)NB * nblk];
    const uint64_t b0 = boff[(uint64_t)b * nblk], b1 = (b + 1 < NB) ? boff[(uint64_t)(b + 1) * nblk] : total;
    lo = b0 + (uint64_t)(s - slice_off[b]) * SLICE_ENTRIES;
    hi = (lo + SLICE_ENTRIES) < b1 ? (lo + SLICE_ENTRIES) : b1;
    return true;
}

// per slice, its entries per node of its bucket: scnt[s][i] for node (b << shift) + i
template <typename T>
__global__ void __launch_bounds__(1024) k_slice_count(const T* __restrict__ opart,
                                                      const uint32_t* __restrict__ boff, uint32_t nblk, uint32_t NB,
                                                      uint32_t shift, const uint32_t* __restrict__ slice_off,
                                                      uint32_t* __restrict__ scount) {
    __shared__ uint32_t cnt[DEG_SUB];
    uint32_t b;
    uint64_t lo, hi;
    if (!slice_of(blockIdx.x, slice_off, boff, nblk, NB, b, lo, hi)) return;
    const uint32_t span = 1u << shift, v0 = b << shift;
    for (uint32_t i = threadIdx.x; i < span; i += blockDim.x) cnt[i] = 0;
    __syncthreads();
    for (uint64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) atomicAdd(&cnt[entry_key(opart[i]) - v0], 1u);
    __syncthreads();
    uint32_t* out = scount + (uint64_t)blockIdx.x * span;
    for (uint32_t i = threadIdx.x; i < span; i += blockDim.x) out[i] = cnt[i];
}

// dout[v] = the entries of v over its bucket's slices
__global__ void k_slice_dout(const uint32_t* __restrict__ scount, const uint32_t* __restrict__ slice_off,
                             uint32_t shift, uint32_t n, uint32_t* __restrict__ dout) {
    for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        const uint32_t b = v >> shift, i = v - (b << shift), span = 1u << shift;
        uint32_t d = 0;
        for (uint32_t s = slice_off[b]; s < slice_off[b + 1]; ++s) d += scount[(uint64_t)s * span + i];
        dout[v] = d;
    }
}

// scount[s][i] <- the position of node v's first entry of slice s in v's segment
__global__ void k_slice_base(uint32_t* __restrict__ scount, const uint32_t* __restrict__ slice_off,
                             uint32_t shift, uint32_t n, const uint32_t* __restrict__ off) {
    for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        const uint32_t b = v >> shift, i = v - (b << shift), span = 1u << shift;
        uint32_t run = off[v];
        for (uint32_t s = slice_off[b]; s < slice_off[b + 1]; ++s) {
            uint32_t* c = scount + (uint64_t)s * span + i;
            const uint32_t k = *c;
            *c = run;
            run += k;
        }
    }
}

constexpr uint32_t PLACE_UNROLL = 4;
// place the slice's entries in their segments (as k_scatter below, with LDS cursors); with
// `rcnt`, also count the reverse pairs per target shard (the shard path of the reverse lists)
constexpr uint32_t REV_BIT = 0x80000000u;
__global__ void __launch_bounds__(1024) k_slice_place(const OEntry* __restrict__ opart,
                                                      const uint32_t* __restrict__ boff, uint32_t nblk, uint32_t NB,
                                                      uint32_t shift, const uint32_t* __restrict__ slice_off,
                                                      const uint32_t* __restrict__ sbase,
                                                      const uint32_t* __restrict__ dout,
                                                      unsigned long long* __restrict__ packed,
                                                      uint32_t* __restrict__ rcnt, BuildStats* st) {
    __shared__ uint32_t cur[DEG_SUB];
    uint32_t b;
    uint64_t lo, hi;
    if (!slice_of(blockIdx.x, slice_off, boff, nblk, NB, b, lo, hi)) return;
    const uint32_t span = 1u << shift, v0 = b << shift;
    const uint32_t* base = sbase + (uint64_t)blockIdx.x * span;
    for (uint32_t i = threadIdx.x; i < span; i += blockDim.x) cur[i] = base[i];
    __syncthreads();
    unsigned long long work = 0;
    // PLACE_UNROLL entries per thread per step, one block stride apart: their loads, cursor
    // atomics and scattered stores are in flight together
    const uint64_t stride = blockDim.x;
    for (uint64_t i0 = lo + threadIdx.x; i0 < hi; i0 += PLACE_UNROLL * stride) {
        OEntry e[PLACE_UNROLL];
        uint32_t pos[PLACE_UNROLL], da[PLACE_UNROLL], db[PLACE_UNROLL];
#pragma unroll
        for (uint32_t u = 0; u < PLACE_UNROLL; ++u) {
            const uint64_t i = i0 + u * stride;
            e[u] = i < hi ? opart[i] : OEntry{v0, v0, 0u};
        }
#pragma unroll
        for (uint32_t u = 0; u < PLACE_UNROLL; ++u) {
            const bool ok = i0 + u * stride < hi;
            pos[u] = ok ? atomicAdd(&cur[e[u].a - v0], 1u) : 0u;
            da[u] = ok ? dout[e[u].a] : 0u;
            db[u] = ok ? dout[e[u].b] : 0u;
        }
#pragma unroll
        for (uint32_t u = 0; u < PLACE_UNROLL; ++u) {
            if (i0 + u * stride >= hi) continue;
            // the counting pass walks the shorter out-list of the pair (see emit_rev)
            const bool rev = da[u] < db[u];
            packed[pos[u]] = ((unsigned long long)e[u].b << 32) | (rev ? REV_BIT : 0u) | e[u].t;
            work += db[u] <= da[u] ? db[u] : da[u];
            if (rev && rcnt) atomicAdd(&rcnt[(uint64_t)e[u].b * REV_SHARDS + (e[u].a % REV_SHARDS)], 1u);
        }
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) work += __shfl_xor(work, d, 64);
    if ((threadIdx.x & 63) == 0 && work) atomicAdd(&st->work, work);
}

// ---- reverse lists by a bucketed transpose (bucket spans of at most DEG_SUB ids): after the
// segment sorts, which mark each reverse pair's source at its adjacency position p, the pairs are
// partitioned by the id bucket of their target b, counted per target in LDS by the placement
// slices above, and placed with LDS cursors: one scan gives roff, and no global atomic touches a
// target's counter.

// per workgroup, the histogram of the target buckets of the reverse pairs in its range of
// adjacency positions (positions past off[n], the placed entries, are never read)
__global__ void __launch_bounds__(1024) k_rev_hist(const uint32_t* __restrict__ rsrc, const uint32_t* __restrict__ nbr,
                                                   const uint32_t* __restrict__ off, uint32_t n, uint32_t shift,
                                                   uint32_t NB, uint64_t per_block, uint32_t* __restrict__ bhist) {
    __shared__ uint32_t h[DEG_BUCKETS];
    for (uint32_t i = threadIdx.x; i < NB; i += blockDim.x) h[i] = 0;
    __syncthreads();
    const uint64_t total = off[n];
    const uint64_t e0 = (uint64_t)blockIdx.x * per_block;
    const uint64_t e1 = (e0 + per_block) < total ? (e0 + per_block) : total;
    for (uint64_t q = e0 + threadIdx.x; q < e1; q += blockDim.x)
        if (rsrc[q] != NO_EDGE) atomicAdd(&h[nbr[q] >> shift], 1u);
    __syncthreads();
    for (uint32_t b = threadIdx.x; b < NB; b += blockDim.x) bhist[(uint64_t)b * gridDim.x + blockIdx.x] = h[b];
}

// the reverse pairs (b, a, t, p) in bucket order of b (order within a bucket is free)
__global__ void __launch_bounds__(1024) k_rev_part(const uint32_t* __restrict__ rsrc, const uint32_t* __restrict__ nbr,
                                                   const uint32_t* __restrict__ tim, const uint32_t* __restrict__ off,
                                                   uint32_t n, uint32_t shift, uint32_t NB, uint64_t per_block,
                                                   const uint32_t* __restrict__ boff, uint4* __restrict__ rpart) {
    __shared__ uint32_t base[DEG_BUCKETS];
    for (uint32_t b = threadIdx.x; b < NB; b += blockDim.x) base[b] = boff[(uint64_t)b * gridDim.x + blockIdx.x];
    __syncthreads();
    const uint64_t total = off[n];
    const uint64_t e0 = (uint64_t)blockIdx.x * per_block;
    const uint64_t e1 = (e0 + per_block) < total ? (e0 + per_block) : total;
    for (uint64_t q = e0 + threadIdx.x; q < e1; q += blockDim.x) {
        const uint32_t a = rsrc[q];
        if (a == NO_EDGE) continue;
        const uint32_t b = nbr[q];
        rpart[atomicAdd(&base[b >> shift], 1u)] = make_uint4(b, a, tim[q], (uint32_t)q);
    }
}

// place the slice's reverse pairs in their targets' lists: the record (a, t, offset and length of
// out(a)) and the pair's adjacency position
__global__ void __launch_bounds__(1024) k_rev_place(const uint4* __restrict__ rpart, const uint32_t* __restrict__ boff,
                                                    uint32_t nblk, uint32_t NB, uint32_t shift,
                                                    const uint32_t* __restrict__ slice_off,
                                                    const uint32_t* __restrict__ sbase, const uint32_t* __restrict__ off,
                                                    uint4* __restrict__ rrec, uint32_t* __restrict__ rpos) {
    __shared__ uint32_t cur[DEG_SUB];
    uint32_t b;
    uint64_t lo, hi;
    if (!slice_of(blockIdx.x, slice_off, boff, nblk, NB, b, lo, hi)) return;
    const uint32_t span = 1u << shift, v0 = b << shift;
    const uint32_t* base = sbase + (uint64_t)blockIdx.x * span;
    for (uint32_t i = threadIdx.x; i < span; i += blockDim.x) cur[i] = base[i];
    __syncthreads();
    const uint64_t stride = blockDim.x;
    for (uint64_t i0 = lo + threadIdx.x; i0 < hi; i0 += PLACE_UNROLL * stride) {
        uint4 e[PLACE_UNROLL];
        uint32_t q[PLACE_UNROLL], s[PLACE_UNROLL], d[PLACE_UNROLL];
#pragma unroll
        for (uint32_t u = 0; u < PLACE_UNROLL; ++u) {
            const uint64_t i = i0 + u * stride;
            e[u] = i < hi ? rpart[i] : make_uint4(v0, 0u, 0u, 0u);
        }
#pragma unroll
        for (uint32_t u = 0; u < PLACE_UNROLL; ++u) {
            const bool ok = i0 + u * stride < hi;
            q[u] = ok ? atomicAdd(&cur[e[u].x - v0], 1u) : 0u;
            s[u] = ok ? off[e[u].y] : 0u;
            d[u] = ok ? off[e[u].y + 1] - s[u] : 0u;
        }
#pragma unroll
        for (uint32_t u = 0; u < PLACE_UNROLL; ++u) {
            if (i0 + u * stride >= hi) continue;
            rrec[q[u]] = make_uint4(e[u].y, e[u].z, s[u], d[u]);
            rpos[q[u]] = e[u].w;
        }
    }
}

// The placement pass takes EDGE_UNROLL edges per thread per step, one grid stride apart, so the
// independent scattered loads and atomics of those edges are in flight together.
constexpr uint32_t EDGE_UNROLL = 4;
// place every oriented entry in its apex segment (unordered within the segment) as
// b << 32 | rev << 31 | t, where rev marks a reverse pair (out(a) shorter than out(b); the
// stream position t is below 2^31, and rev, a function of b within a's segment, leaves the
// order by (b, t) unchanged), and count the reverse pairs per target shard.  cursor[a] starts
// at off[a].
__global__ void __launch_bounds__(SCAN_THREADS) k_scatter(const uint2* __restrict__ ab, uint64_t E,
                                                          const uint32_t* __restrict__ dout, uint32_t* cursor,
                                                          unsigned long long* __restrict__ packed,
                                                          uint32_t* __restrict__ rcnt, BuildStats* st) {
    unsigned long long work = 0;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t t0 = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t0 < E; t0 += EDGE_UNROLL * stride) {
        uint2 e[EDGE_UNROLL];
        uint32_t pos[EDGE_UNROLL], da[EDGE_UNROLL], db[EDGE_UNROLL];
#pragma unroll
        for (uint32_t u = 0; u < EDGE_UNROLL; ++u) {
            const uint64_t t = t0 + u * stride;
            e[u] = t < E ? ab[t] : make_uint2(NO_EDGE, NO_EDGE);
        }
#pragma unroll
        for (uint32_t u = 0; u < EDGE_UNROLL; ++u) {
            const bool ok = e[u].x != NO_EDGE;
            pos[u] = ok ? atomicAdd(&cursor[e[u].x], 1u) : 0u;
            // the counting pass walks the shorter out-list of the pair (see emit_rev)
            da[u] = ok ? dout[e[u].x] : 0u;
            db[u] = ok ? dout[e[u].y] : 0u;
        }
#pragma unroll
        for (uint32_t u = 0; u < EDGE_UNROLL; ++u) {
            if (e[u].x == NO_EDGE) continue;
            const uint32_t a = e[u].x, b = e[u].y;
            const bool rev = da[u] < db[u];
            packed[pos[u]] = ((unsigned long long)b << 32) | (rev ? REV_BIT : 0u) | (uint32_t)(t0 + u * stride);
            work += db[u] <= da[u] ? db[u] : da[u];
            if (rev) atomicAdd(&rcnt[(uint64_t)b * REV_SHARDS + (a % REV_SHARDS)], 1u);
        }
    }
    unsigned long long s = block_reduce_sum256<unsigned long long>(work);
    if (threadIdx.x == 0 && s) atomicAdd(&st->work, s);
}

// Reverse lists.  The counting pass finds a triangle from its lowest-ranked oriented pair
// a -> b by walking the shorter of out(a), out(b) against a hash of the other.  Pairs with
// out(a) shorter are counted at b: rev(b) lists them.  A record carries what the counting pass
// stages for the pair -- a, the arrival time of a-b, the offset and length of a's list -- and
// the position of b in a's list.  They are built by the bucketed transpose (k_rev_hist,
// k_rev_part, k_rev_place) or, on the shard path, cut into REV_SHARDS shards per target:
// k_scatter counts each shard, a scan gives the shard starts, and the segment sorts, which know
// each entry's final position, write the records (emit_rev).

// roff[b] = start of b's first shard (roff[n] = the number of pairs)
__global__ void k_rev_roff(const uint32_t* __restrict__ sofs, uint32_t n, uint32_t* __restrict__ roff,
                           BuildStats* st) {
    for (uint32_t b = blockIdx.x * blockDim.x + threadIdx.x; b <= n; b += gridDim.x * blockDim.x) {
        roff[b] = sofs[(uint64_t)b * REV_SHARDS];
        if (b == n) st->num_rev = roff[b];
    }
}

// Out-degrees below APEX_LDS_BINS are histogrammed per workgroup in LDS (the common small
// out-degrees would otherwise hammer a few global counters); each workgroup covers one
// contiguous node range.
constexpr uint32_t APEX_LDS_BINS = 4096;

__device__ __forceinline__ void node_range(uint32_t n, uint32_t& a0, uint32_t& a1) {
    const uint32_t per = (n + gridDim.x - 1) / gridDim.x;
    a0 = blockIdx.x * per;
    a1 = a0 + per < n ? a0 + per : n;
    if (a0 > n) a0 = n;
}

// classify segments by size (sort path: `medium` lists the wavefront class from its front and the
// workgroup class from its back), and the statistics of the oriented graph
// unit order key of node a (REPT_REV_SHIFT), at most n - 1; units are ordered by it, descending,
// and the counting pass gives a workgroup to the units whose key exceeds its wavefront cap
__device__ __forceinline__ uint32_t unit_key(const uint32_t* __restrict__ off, const uint32_t* __restrict__ roff,
                                             uint32_t n, uint32_t a) {
    const uint32_t d = off[a + 1] - off[a], r = (roff[a + 1] - roff[a]) >> REPT_REV_SHIFT;
    const uint32_t k = d > r ? d : r;
    return k < n - 1 ? k : n - 1;
}

__global__ void __launch_bounds__(SCAN_THREADS) k_classify(const uint32_t* __restrict__ off, uint32_t n,
                                                           uint32_t* medium, uint32_t* large, BuildStats* st) {
    __shared__ uint32_t cnt[3], base[3];
    if (threadIdx.x < 3) cnt[threadIdx.x] = 0;
    __syncthreads();
    uint32_t a0, a1;
    node_range(n, a0, a1);
    unsigned long long sq = 0;
    uint32_t mx = 0, napex = 0;
    for (uint32_t a = a0 + threadIdx.x; a < a1; a += blockDim.x) {
        const uint32_t d = off[a + 1] - off[a];
        sq += (unsigned long long)d * d;
        mx = d > mx ? d : mx;
        if (d >= 2) ++napex;
        if (d > WAVE_MAX && d <= MEDIUM_MAX) atomicAdd(&cnt[0], 1u);
        if (d > MEDIUM_MAX) atomicAdd(&cnt[1], 1u);
        if (d > SMALL_MAX && d <= WAVE_MAX) atomicAdd(&cnt[2], 1u);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        base[0] = cnt[0] ? atomicAdd(&st->n_medium, cnt[0]) : 0;
        base[1] = cnt[1] ? atomicAdd(&st->n_large, cnt[1]) : 0;
        base[2] = cnt[2] ? atomicAdd(&st->n_wave, cnt[2]) : 0;
    }
    __syncthreads();
    for (uint32_t a = a0 + threadIdx.x; a < a1; a += blockDim.x) {
        const uint32_t d = off[a + 1] - off[a];
        if (d > WAVE_MAX && d <= MEDIUM_MAX) medium[n - 1 - atomicAdd(&base[0], 1u)] = a;
        if (d > MEDIUM_MAX) large[atomicAdd(&base[1], 1u)] = a;
        if (d > SMALL_MAX && d <= WAVE_MAX) medium[atomicAdd(&base[2], 1u)] = a;
    }
    unsigned long long s = block_reduce_sum256<unsigned long long>(sq);
    uint32_t na = block_reduce_sum256<uint32_t>(napex);
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        uint32_t o = __shfl_xor(mx, d, 64);
        mx = o > mx ? o : mx;
    }
    if ((threadIdx.x & 63) == 0 && mx) atomicMax(&st->max_out, mx);
    if (threadIdx.x == 0) {
        if (s) atomicAdd(&st->sum_out_sq, s);
        if (na) atomicAdd(&st->num_apex, na);
    }
}

// histogram apexes by unit key for the descending unit order (bucket n-1-key); needs the reverse
// lists' offsets, and records their total
__global__ void __launch_bounds__(SCAN_THREADS) k_apex_hist(const uint32_t* __restrict__ off,
                                                            const uint32_t* __restrict__ roff, uint32_t n,
                                                            uint32_t* ahist, BuildStats* st) {
    __shared__ uint32_t h[APEX_LDS_BINS];
    for (uint32_t i = threadIdx.x; i < APEX_LDS_BINS; i += blockDim.x) h[i] = 0;
    __syncthreads();
    uint32_t a0, a1;
    node_range(n, a0, a1);
    for (uint32_t a = a0 + threadIdx.x; a < a1; a += blockDim.x) {
        const uint32_t d = off[a + 1] - off[a];
        if (d >= 2) {
            const uint32_t k = unit_key(off, roff, n, a);
            if (k < APEX_LDS_BINS) atomicAdd(&h[k], 1u);
            else atomicAdd(&ahist[n - 1 - k], 1u);
        }
    }
    __syncthreads();
    for (uint32_t d = threadIdx.x; d < APEX_LDS_BINS; d += blockDim.x)
        if (h[d]) atomicAdd(&ahist[n - 1 - d], h[d]);
    if (blockIdx.x == 0 && threadIdx.x == 0) st->num_rev = roff[n];
}

// place apexes in out-degree-descending order: reserve each bin's range once per workgroup
__global__ void __launch_bounds__(SCAN_THREADS) k_apex_scatter(const uint32_t* __restrict__ off,
                                                               const uint32_t* __restrict__ roff, uint32_t n,
                                                               const uint32_t* __restrict__ aoff, uint32_t* acur,
                                                               uint32_t* apex) {
    __shared__ uint32_t h[APEX_LDS_BINS];
    for (uint32_t i = threadIdx.x; i < APEX_LDS_BINS; i += blockDim.x) h[i] = 0;
    __syncthreads();
    uint32_t a0, a1;
    node_range(n, a0, a1);
    for (uint32_t a = a0 + threadIdx.x; a < a1; a += blockDim.x) {
        const uint32_t d = off[a + 1] - off[a];
        if (d < 2) continue;
        const uint32_t k = unit_key(off, roff, n, a);
        if (k < APEX_LDS_BINS) atomicAdd(&h[k], 1u);
    }
    __syncthreads();
    for (uint32_t k = threadIdx.x; k < APEX_LDS_BINS; k += blockDim.x)
        if (h[k]) h[k] = aoff[n - 1 - k] + atomicAdd(&acur[n - 1 - k], h[k]);
    __syncthreads();
    for (uint32_t a = a0 + threadIdx.x; a < a1; a += blockDim.x) {
        const uint32_t d = off[a + 1] - off[a];
        if (d < 2) continue;
        const uint32_t k = unit_key(off, roff, n, a);
        const uint32_t pos = k < APEX_LDS_BINS ? atomicAdd(&h[k], 1u)
                                               : aoff[n - 1 - k] + atomicAdd(&acur[n - 1 - k], 1u);
        apex[pos] = a;
    }
}

// Where the sorts emit the entry (b, t) at position s + i of a's list (length d), a reverse pair
// (out(a) shorter than out(b)) also goes either to its reverse record, in the next free slot of
// b's shard (shard path), or, with `src`, is marked at its position for the bucketed transpose
// below: src[s + i] = a for a reverse pair, NO_EDGE otherwise.
struct RevOut {
    uint32_t* cur;  // per target shard, from the shard's start
    uint4* rrec;
    uint32_t* rpos;
    uint32_t* src;  // null on the shard path
};
__device__ __forceinline__ void emit_rev(const RevOut& R, uint32_t a, uint32_t s, uint32_t d, uint32_t i, uint32_t b,
                                         uint32_t t) {
    const uint64_t sh = (uint64_t)b * REV_SHARDS + (a % REV_SHARDS);
    const uint32_t q = atomicAdd(&R.cur[sh], 1u);
    R.rrec[q] = make_uint4(a, t, s, d);
    R.rpos[q] = s + i;
}

__device__ __forceinline__ void emit_sorted(unsigned long long v, uint32_t idx, uint32_t a, uint32_t seg, uint32_t d,
                                            uint32_t* nbr, uint32_t* tim, const RevOut& R) {
    if (idx < d) {
        const uint32_t b = (uint32_t)(v >> 32), t = (uint32_t)v & ~REV_BIT;
        const bool rev = ((uint32_t)v & REV_BIT) != 0;
        nbr[seg + idx] = b;
        tim[seg + idx] = t;
        if (R.src) R.src[seg + idx] = rev ? a : NO_EDGE;
        else if (rev) emit_rev(R, a, seg, d, idx, b, t);
    }
}

// Bitonic network over aligned groups of G lanes: each group sorts its G values ascending
// (the partner lane ^ j of every step stays inside the group).  i: the value's index in the
// sequence being sorted (lane for one value per lane).
template <int G>
__device__ __forceinline__ unsigned long long group_sort(unsigned long long v, uint32_t i) {
#pragma unroll
    for (int k = 2; k <= G; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j >= 1; j >>= 1) {
            const unsigned long long o = __shfl_xor(v, j, 64);
            const bool up = (i & k) == 0, lower = (i & j) == 0;
            v = (lower == up) ? (o < v ? o : v) : (o > v ? o : v);
        }
    }
    return v;
}

// Segments of 1..64 entries.  A wavefront takes 64 consecutive nodes at a time (one coalesced
// load of their offsets) and sorts their segments in aligned lane groups of 8, 16, 32 or 64
// lanes (the smallest that holds the segment), 64 / G segments per pass, so a short segment
// costs a short network and shares it with others.
template <int G>
__device__ __forceinline__ void sort_class(bool in, uint32_t s, uint32_t d, uint32_t a0, int lane,
                                           const unsigned long long* __restrict__ packed, uint32_t* __restrict__ nbr,
                                           uint32_t* __restrict__ tim, const RevOut& R, uint32_t& dup) {
    constexpr int per = 64 / G;
    const int grp = lane / G;
    const uint32_t li = (uint32_t)(lane % G);
    unsigned long long mask = __ballot(in);
    while (mask) {
        unsigned long long m = mask;  // this group's segment: the grp-th node left in the mask
        for (int k = 0; k < grp; ++k) m &= m - 1;
        const int src = m ? __builtin_ctzll(m) : 0;
        // every lane takes part in both shuffles: a lane left out would not supply its own values
        const uint32_t gs = __shfl(s, src, 64), gd0 = __shfl(d, src, 64);
        const uint32_t gd = m ? gd0 : 0u;
        unsigned long long v = li < gd ? packed[gs + li] : ~0ull;
        v = group_sort<G>(v, li);
        const unsigned long long prev = __shfl_up(v, 1, 64);
        if (li > 0 && li < gd && (prev >> 32) == (v >> 32)) dup = 1;
        emit_sorted(v, li, a0 + (uint32_t)src, gs, gd, nbr, tim, R);
#pragma unroll
        for (int k = 0; k < per; ++k) mask &= mask - 1;  // the segments of this pass are done
    }
}

__global__ void __launch_bounds__(256) k_sort_small(const uint32_t* __restrict__ off, uint32_t n,
                                                    const unsigned long long* __restrict__ packed,
                                                    uint32_t* __restrict__ nbr, uint32_t* __restrict__ tim,
                                                    RevOut R, BuildStats* st) {
    const int lane = threadIdx.x & 63;
    const uint64_t waves = (uint64_t)gridDim.x * (blockDim.x >> 6);
    uint32_t dup = 0;
    for (uint64_t a0 = ((uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) * 64; a0 < n; a0 += waves * 64) {
        const uint64_t a = a0 + lane;
        uint32_t s = 0, d = 0;
        if (a < n) {
            s = off[a];
            d = off[a + 1] - s;
        }
        sort_class<8>(d >= 1 && d <= 8, s, d, (uint32_t)a0, lane, packed, nbr, tim, R, dup);
        sort_class<16>(d > 8 && d <= 16, s, d, (uint32_t)a0, lane, packed, nbr, tim, R, dup);
        sort_class<32>(d > 16 && d <= 32, s, d, (uint32_t)a0, lane, packed, nbr, tim, R, dup);
        sort_class<64>(d > 32 && d <= 64, s, d, (uint32_t)a0, lane, packed, nbr, tim, R, dup);
    }
    if (dup) atomicOr(&st->flags, RF_DUP);
}

// Segments of 65..1024 entries: one wavefront each, K values per lane (value i = r * 64 + lane in
// register r), bitonic network in registers: steps with j < 64 exchange across lanes, steps with
// j >= 64 between registers of one lane.  No barriers.
template <int K>
__device__ __forceinline__ void wave_sort(const unsigned long long* __restrict__ src, uint32_t a, uint32_t s,
                                          uint32_t d, int lane, uint32_t* __restrict__ nbr,
                                          uint32_t* __restrict__ tim, const RevOut& R, uint32_t& dup) {
    unsigned long long v[K];
#pragma unroll
    for (int r = 0; r < K; ++r) {
        const uint32_t i = (uint32_t)(r * 64 + lane);
        v[r] = i < d ? src[i] : ~0ull;
    }
    // fully unrolled: every register index is a constant (an index computed at run time would
    // put the array in scratch memory)
#pragma unroll
    for (int k = 2; k <= 64 * K; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j >= 1; j >>= 1) {
            if (j >= 64) {
                const int jr = j >> 6;
#pragma unroll
                for (int r = 0; r < K; ++r) {
                    if (r & jr) continue;
                    const int r2 = r | jr;
                    const bool up = (((uint32_t)(r * 64 + lane)) & (uint32_t)k) == 0;
                    const unsigned long long x = v[r], y = v[r2];
                    const bool sw = (x > y) == up;
                    v[r] = sw ? y : x;
                    v[r2] = sw ? x : y;
                }
            } else {
#pragma unroll
                for (int r = 0; r < K; ++r) {
                    const unsigned long long o = __shfl_xor(v[r], j, 64);
                    const uint32_t i = (uint32_t)(r * 64 + lane);
                    const bool up = (i & (uint32_t)k) == 0, lower = (i & (uint32_t)j) == 0;
                    v[r] = (lower == up) ? (o < v[r] ? o : v[r]) : (o > v[r] ? o : v[r]);
                }
            }
        }
    }
#pragma unroll
    for (int r = 0; r < K; ++r) {
        const uint32_t i = (uint32_t)(r * 64 + lane);
        unsigned long long prev = __shfl_up(v[r], 1, 64);
        if (r > 0) {
            const unsigned long long last = __shfl(v[r - 1], 63, 64);
            if (lane == 0) prev = last;
        }
        if (i > 0 && i < d && (prev >> 32) == (v[r] >> 32)) dup = 1;
        emit_sorted(v[r], i, a, s, d, nbr, tim, R);
    }
}

__global__ void __launch_bounds__(256) k_sort_wave(const uint32_t* __restrict__ off, const uint32_t* __restrict__ list,
                                                   const unsigned long long* __restrict__ packed,
                                                   uint32_t* __restrict__ nbr, uint32_t* __restrict__ tim,
                                                   RevOut R, BuildStats* st) {
    const int lane = threadIdx.x & 63;
    const uint32_t waves = gridDim.x * (blockDim.x >> 6);
    const uint32_t cnt = st->n_wave;
    uint32_t dup = 0;
    for (uint32_t q = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); q < cnt; q += waves) {
        const uint32_t a = list[q];
        const uint32_t s = off[a], d = off[a + 1] - s;
        if (d <= 128) wave_sort<2>(packed + s, a, s, d, lane, nbr, tim, R, dup);
        else if (d <= 256) wave_sort<4>(packed + s, a, s, d, lane, nbr, tim, R, dup);
        else if (d <= 512) wave_sort<8>(packed + s, a, s, d, lane, nbr, tim, R, dup);
        else wave_sort<16>(packed + s, a, s, d, lane, nbr, tim, R, dup);
    }
    if (dup) atomicOr(&st->flags, RF_DUP);
}

// segments of 1025..4096 entries: one workgroup, bitonic sort in LDS (their nodes are listed
// from the back of `list`, which holds n entries)
__global__ void __launch_bounds__(512) k_sort_medium(const uint32_t* __restrict__ off, const uint32_t* __restrict__ list,
                                                     uint32_t n, const unsigned long long* __restrict__ packed,
                                                     uint32_t* __restrict__ nbr, uint32_t* __restrict__ tim,
                                                     RevOut R, BuildStats* st) {
    __shared__ unsigned long long buf[MEDIUM_MAX];
    const uint32_t cnt = st->n_medium;
    for (uint32_t q = blockIdx.x; q < cnt; q += gridDim.x) {
        const uint32_t a = list[n - 1 - q];
        const uint32_t s = off[a], d = off[a + 1] - s;
        uint32_t P = 128;
        while (P < d) P <<= 1;
        for (uint32_t i = threadIdx.x; i < P; i += blockDim.x) buf[i] = i < d ? packed[s + i] : ~0ull;
        __syncthreads();
        for (uint32_t k = 2; k <= P; k <<= 1) {
            for (uint32_t j = k >> 1; j >= 1; j >>= 1) {
                for (uint32_t i = threadIdx.x; i < P; i += blockDim.x) {
                    uint32_t l = i ^ j;
                    if (l > i) {
                        unsigned long long x = buf[i], y = buf[l];
                        bool up = (i & k) == 0;
                        if ((x > y) == up) {
                            buf[i] = y;
                            buf[l] = x;
                        }
                    }
                }
                __syncthreads();
            }
        }
        uint32_t dup = 0;
        for (uint32_t i = threadIdx.x; i < d; i += blockDim.x) {
            unsigned long long v = buf[i];
            if (i > 0 && (buf[i - 1] >> 32) == (v >> 32)) dup = 1;
            emit_sorted(v, i, a, s, d, nbr, tim, R);
        }
        if (dup) atomicOr(&st->flags, RF_DUP);
        __syncthreads();
    }
}

// segments above 4096 entries: one wavefront, stable LSD radix sort (8-bit digits of the
// neighbour id) ping-ponging between `packed` and `alt` over the segment's own range
__global__ void __launch_bounds__(64) k_sort_large(const uint32_t* __restrict__ off, const uint32_t* __restrict__ list,
                                                   unsigned long long* packed, unsigned long long* alt,
                                                   uint32_t id_bits, uint32_t* __restrict__ nbr,
                                                   uint32_t* __restrict__ tim, RevOut R, BuildStats* st) {
    __shared__ uint32_t base[256];
    const int lane = threadIdx.x;
    const uint32_t cnt = st->n_large;
    const uint32_t passes = (id_bits + 7) / 8;
    for (uint32_t q = blockIdx.x; q < cnt; q += gridDim.x) {
        const uint32_t a = list[q];
        const uint32_t s = off[a], d = off[a + 1] - s;
        unsigned long long* src = packed + s;
        unsigned long long* dst = alt + s;
        for (uint32_t pass = 0; pass < passes; ++pass) {
            const uint32_t shift = 32 + 8 * pass;
            for (int b = lane; b < 256; b += 64) base[b] = 0;
            __syncthreads();
            for (uint32_t i = lane; i < d; i += 64) atomicAdd(&base[(uint32_t)(src[i] >> shift) & 255u], 1u);
            __syncthreads();
            if (lane == 0) {
                uint32_t run = 0;
                for (int b = 0; b < 256; ++b) {
                    uint32_t c = base[b];
                    base[b] = run;
                    run += c;
                }
            }
            __syncthreads();
            for (uint32_t c0 = 0; c0 < d; c0 += 64) {
                const uint32_t i = c0 + lane;
                const bool valid = i < d;
                unsigned long long v = valid ? src[i] : 0ull;
                uint32_t dig = (uint32_t)(v >> shift) & 255u;
                unsigned long long peers = __ballot(valid);
                for (int bit = 0; bit < 8; ++bit) {
                    unsigned long long bb = __ballot(valid && ((dig >> bit) & 1u));
                    peers &= ((dig >> bit) & 1u) ? bb : ~bb;
                }
                const unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
                uint32_t rank = __popcll(peers & lt);
                uint32_t pos = valid ? base[dig] + rank : 0;
                __syncthreads();
                if (valid) {
                    dst[pos] = v;
                    int last = 63 - __clzll(peers);
                    if (lane == last) base[dig] += __popcll(peers);
                }
                __syncthreads();
            }
            unsigned long long* tmp = src;
            src = dst;
            dst = tmp;
        }
        uint32_t dup = 0;
        for (uint32_t i = lane; i < d; i += 64) {
            unsigned long long v = src[i];
            if (i > 0 && (src[i - 1] >> 32) == (v >> 32)) dup = 1;
            emit_sorted(v, i, a, s, d, nbr, tim, R);
        }
        if (dup) atomicOr(&st->flags, RF_DUP);
        __syncthreads();
    }
}

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Layout {
    size_t ctrl, off, nbr, tim, apex, roff, rrec, rpos, total;
};
struct ScratchLayout {
    size_t stats, deg, dout, cursor, ahist, aoff, part, packed, alt, opart, slice_off, scount, medium, large, bhist,
        bscan, scnt, sofs, total;
};

// partition of endpoints for the degree count: buckets of 2^shift ids, NB <= DEG_BUCKETS of
// them, nblk workgroups each covering per_block edges
struct DegPlan {
    uint32_t shift, NB, nblk;
    uint64_t per_block;
};
DegPlan deg_plan(uint32_t n, uint64_t E) {
    DegPlan D;
    uint32_t bits = 1;
    while (bits < 32 && ((uint64_t)1 << bits) < (uint64_t)n) ++bits;
    D.shift = bits > 24 ? bits - 12 : 12;
    D.NB = (uint32_t)(((uint64_t)n + ((uint64_t)1 << D.shift) - 1) >> D.shift);
    uint64_t nb = (E + 8191) / 8192;
    D.nblk = (uint32_t)(nb < 1 ? 1 : (nb > 2048 ? 2048 : nb));
    D.per_block = (E + D.nblk - 1) / D.nblk;
    if (D.per_block == 0) D.per_block = 1;
    return D;
}

Layout persistent_layout(uint32_t n, uint64_t E) {
    Layout L;
    size_t p = 0;
    L.ctrl = p;
    p += align256(REPT_CTRL_BYTES);
    L.off = p;
    p += align256(((size_t)n + 1) * 4);
    L.nbr = p;
    p += align256((size_t)E * 4);
    L.tim = p;
    p += align256((size_t)E * 4);
    L.apex = p;
    p += align256((size_t)n * 4);
    L.roff = p;
    p += align256(((size_t)n + 1) * 4);
    L.rrec = p;
    p += align256((size_t)E * 16);
    L.rpos = p;
    p += align256((size_t)E * 4);
    L.total = p;
    return L;
}

ScratchLayout scratch_layout(uint32_t n, uint64_t E) {
    ScratchLayout S;
    size_t p = 0;
    const DegPlan D = deg_plan(n, E);
    // per-target shard counters of the reverse pairs only where the reverse lists are built
    // with shard cursors (buckets wider than DEG_SUB ids); the transpose needs none
    const bool sliced = D.shift <= 13;
    const size_t nhist = (size_t)D.NB * D.nblk, nshard = sliced ? 0 : (size_t)n * REV_SHARDS;
    size_t scan_max = nhist > nshard ? nhist : nshard;
    scan_max = (scan_max > (size_t)n ? scan_max : (size_t)n) + 1;  // the scans over nodes too
    const size_t nparts = (scan_max + SCAN_TILE - 1) / SCAN_TILE + 1;
    S.stats = p;
    p += align256(sizeof(BuildStats));
    S.deg = p;
    p += align256((size_t)n * 4);
    S.dout = p;
    p += align256((size_t)n * 4);
    S.cursor = p;
    p += align256((size_t)n * 4);
    S.ahist = p;
    p += align256((size_t)n * 4);
    S.aoff = p;
    p += align256(((size_t)n + 1) * 4);
    S.part = p;
    p += align256(nparts * 4);
    S.packed = p;
    p += align256((size_t)E * 8);
    S.alt = p;
    p += align256((size_t)E * 8);
    S.opart = p;  // oriented entries (a, b, t), 12 bytes, partitioned by the bucket of a; later the
                  // reverse marks (4 bytes per edge)
    p += align256((size_t)E * 16);
    // placement slices (bucket spans of at most DEG_SUB ids): their offsets per bucket and their
    // per-node counts, then bases
    const uint64_t smax = sliced ? (E + SLICE_ENTRIES - 1) / SLICE_ENTRIES + D.NB : 0;
    S.slice_off = p;
    p += align256(((size_t)D.NB + 1) * 4);
    S.scount = p;
    p += align256((size_t)smax * ((size_t)1 << D.shift) * 4);
    S.medium = p;
    p += align256((size_t)n * 4);
    S.large = p;
    p += align256((size_t)n * 4);
    S.bhist = p;
    p += align256(nhist * 4);
    S.bscan = p;
    p += align256((nhist + 1) * 4);
    S.scnt = p;  // reverse-list shard counters (then cursors)
    p += align256(nshard * 4);
    S.sofs = p;  // their exclusive scan
    p += align256((nshard + 1) * 4);
    S.total = p;
    return S;
}

hipError_t scan_u32(const uint32_t* in, uint64_t N, uint32_t* part, uint32_t* out, hipStream_t s) {
    const uint32_t nb = (uint32_t)((N + SCAN_TILE - 1) / SCAN_TILE);
    const uint32_t nbl = nb ? nb : 1;
    hipLaunchKernelGGL(k_scan_reduce, dim3(nbl), dim3(SCAN_THREADS), 0, s, in, N, part);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, s, part, nbl);
    hipLaunchKernelGGL(k_scan_down, dim3(nbl), dim3(SCAN_THREADS), 0, s, in, N, part, out);
    return hipGetLastError();
}

uint32_t grid_for(uint64_t items, uint32_t threads, uint32_t cap) {
    uint64_t g = (items + threads - 1) / threads;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (uint32_t)g;
}

}  // namespace

// Where a host-resident stream is staged in the persistent buffer: the reverse records' region
// (16 bytes per edge), which the build writes only in the segment sorts, after every pass that
// reads the stream.
size_t rept_host_stage_offset(uint32_t n, uint64_t E) { return persistent_layout(n, E).rrec; }

void rept_sizes_impl(uint32_t n, uint64_t E, size_t* persistent, size_t* scratch) {
    *persistent = persistent_layout(n, E).total;
    *scratch = scratch_layout(n, E).total;
}

rept_status rept_build_impl(uint32_t n, const uint32_t* edges, uint64_t E, void* persistent,
                            size_t persistent_bytes, void* scratch, size_t scratch_bytes,
                            hipStream_t s, rept_graph** out) {
    const Layout L = persistent_layout(n, E);
    const ScratchLayout S = scratch_layout(n, E);
    if (persistent_bytes < L.total || scratch_bytes < S.total) return REPT_ENOMEM;
    uint8_t* P = (uint8_t*)persistent;
    uint8_t* X = (uint8_t*)scratch;
    uint32_t* off = (uint32_t*)(P + L.off);
    uint32_t* nbr = (uint32_t*)(P + L.nbr);
    uint32_t* tim = (uint32_t*)(P + L.tim);
    uint32_t* apex = (uint32_t*)(P + L.apex);
    uint32_t* roff = (uint32_t*)(P + L.roff);
    uint4* rrec = (uint4*)(P + L.rrec);
    uint32_t* rpos = (uint32_t*)(P + L.rpos);
    BuildStats* st = (BuildStats*)(X + S.stats);
    uint32_t* deg = (uint32_t*)(X + S.deg);
    uint32_t* dout = (uint32_t*)(X + S.dout);
    uint32_t* cursor = (uint32_t*)(X + S.cursor);
    uint32_t* ahist = (uint32_t*)(X + S.ahist);
    uint32_t* aoff = (uint32_t*)(X + S.aoff);
    uint32_t* part = (uint32_t*)(X + S.part);
    unsigned long long* packed = (unsigned long long*)(X + S.packed);
    unsigned long long* alt = (unsigned long long*)(X + S.alt);
    OEntry* opart = (OEntry*)(X + S.opart);
    uint32_t* slice_off = (uint32_t*)(X + S.slice_off);
    uint32_t* scount = (uint32_t*)(X + S.scount);
    uint32_t* medium = (uint32_t*)(X + S.medium);
    uint32_t* large = (uint32_t*)(X + S.large);
    uint32_t* bhist = (uint32_t*)(X + S.bhist);
    uint32_t* bscan = (uint32_t*)(X + S.bscan);
    uint32_t* scnt = (uint32_t*)(X + S.scnt);
    uint32_t* sofs = (uint32_t*)(X + S.sofs);
    const uint2* e2 = (const uint2*)edges;

    const uint32_t cus = rept_num_cus();
    const uint32_t cap = cus ? cus * 16 : 4096;
    const uint32_t gE = grid_for(E, 256, cap), gN = grid_for(n, 256, cap);
    const uint32_t gA = grid_for(n, 2048, 512);  // node-range kernels with LDS histograms
    const DegPlan D = deg_plan(n, E);

    // clear counters (fill kernels rather than memsets, so the sequence is capture-safe)
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, s, (uint32_t*)st,
                       (uint64_t)(sizeof(BuildStats) / 4), 0u);
    hipLaunchKernelGGL(k_fill_u32, dim3(gN), dim3(256), 0, s, dout, (uint64_t)n, 0u);
    hipLaunchKernelGGL(k_fill_u32, dim3(gN), dim3(256), 0, s, ahist, (uint64_t)n, 0u);

    // degrees: partition endpoints by id bucket (reusing `packed` as the partition), count in LDS.
    // With many buckets the partition takes two passes: by super-buckets of 64 buckets into `alt`
    // (free until the orientation), then by bucket.  R-MAT scale 24 (4096 buckets): 5.2 ms for
    // both passes against 7.4 ms for one, whose 4096 runs per workgroup wrote 10.2 GB for 2.1 GB
    // of ids; the 1M/20M power-law graph (245 buckets) stays faster in one pass.
    uint32_t* ends = (uint32_t*)packed;
    if (D.NB >= 1024) {
        const uint32_t sshift = D.shift + 6;
        const uint32_t NB1 = (uint32_t)(((uint64_t)n + ((uint64_t)1 << sshift) - 1) >> sshift);
        uint32_t* ends1 = (uint32_t*)alt;
        hipLaunchKernelGGL(k_deg_hist, dim3(D.nblk), dim3(1024), 0, s, e2, E, n, sshift, NB1, D.per_block, bhist,
                           st);
        if (scan_u32(bhist, (uint64_t)NB1 * D.nblk, part, bscan, s) != hipSuccess) return REPT_EDEVICE;
        hipLaunchKernelGGL(k_deg_scatter, dim3(D.nblk), dim3(1024), 0, s, e2, E, n, sshift, NB1, D.per_block, bscan,
                           ends1);
        // the endpoint count (the first scan's total) is kept for the second pass, whose scan
        // reuses the first one's array
        hipLaunchKernelGGL(k_copy_u32, dim3(1), dim3(64), 0, s, bscan + (uint64_t)NB1 * D.nblk, (uint64_t)1,
                           &st->n_ends);
        uint64_t per2 = (2 * E + D.nblk - 1) / D.nblk;
        if (per2 == 0) per2 = 1;
        hipLaunchKernelGGL(k_ids_hist, dim3(D.nblk), dim3(1024), 0, s, ends1, &st->n_ends, D.shift, D.NB, per2,
                           bhist);
        if (scan_u32(bhist, (uint64_t)D.NB * D.nblk, part, bscan, s) != hipSuccess) return REPT_EDEVICE;
        hipLaunchKernelGGL(k_ids_scatter, dim3(D.nblk), dim3(1024), 0, s, ends1, &st->n_ends, D.shift, D.NB, per2,
                           bscan, ends);
    } else {
        hipLaunchKernelGGL(k_deg_hist, dim3(D.nblk), dim3(1024), 0, s, e2, E, n, D.shift, D.NB, D.per_block, bhist,
                           st);
        if (scan_u32(bhist, (uint64_t)D.NB * D.nblk, part, bscan, s) != hipSuccess) return REPT_EDEVICE;
        hipLaunchKernelGGL(k_deg_scatter, dim3(D.nblk), dim3(1024), 0, s, e2, E, n, D.shift, D.NB, D.per_block,
                           bscan, ends);
    }
    hipLaunchKernelGGL(k_fill_u32, dim3(gN), dim3(256), 0, s, deg, (uint64_t)n, 0u);
    hipLaunchKernelGGL(k_deg_count, dim3(grid_for(2 * E, DEG_SLICE, 4096)), dim3(1024), 0, s, ends, bscan, D.nblk,
                       D.NB, D.shift, n, deg);

    // orientation of every edge into `alt` (free until the large-segment sort), partitioned by
    // the bucket of its lower endpoint into `opart`, whose out-degrees are counted per bucket
    // with LDS counters (the degree partition's buckets); then the placement in the segments
    uint2* ab = (uint2*)alt;
    hipLaunchKernelGGL(k_orient_hist, dim3(D.nblk), dim3(1024), 0, s, e2, E, n, deg, D.shift, D.NB, D.per_block,
                       ab, bhist);
    if (scan_u32(bhist, (uint64_t)D.NB * D.nblk, part, bscan, s) != hipSuccess) return REPT_EDEVICE;
    hipLaunchKernelGGL(k_orient_part, dim3(D.nblk), dim3(1024), 0, s, ab, E, D.shift, D.NB, D.per_block, bscan,
                       opart);
    const uint64_t nsh = (uint64_t)n * REV_SHARDS;
    const uint32_t gS = grid_for(nsh, 256, cap);
    const bool sliced = D.shift <= 13;
    const uint64_t smax = (E + SLICE_ENTRIES - 1) / SLICE_ENTRIES + D.NB;
    if (sliced) {  // placement by slices of the partition, LDS cursors
        hipLaunchKernelGGL(k_slice_plan, dim3(1), dim3(1024), 0, s, bscan, D.nblk, D.NB, slice_off);
        hipLaunchKernelGGL(k_slice_count<OEntry>, dim3((uint32_t)smax), dim3(1024), 0, s, (const OEntry*)opart, bscan,
                           D.nblk, D.NB,
                           D.shift, slice_off, scount);
        hipLaunchKernelGGL(k_slice_dout, dim3(gN), dim3(256), 0, s, scount, slice_off, D.shift, n, dout);
        if (scan_u32(dout, n, part, off, s) != hipSuccess) return REPT_EDEVICE;
        hipLaunchKernelGGL(k_slice_base, dim3(gN), dim3(256), 0, s, scount, slice_off, D.shift, n, off);
        hipLaunchKernelGGL(k_slice_place, dim3((uint32_t)smax), dim3(1024), 0, s, opart, bscan, D.nblk, D.NB,
                           D.shift, slice_off, scount, dout, packed, (uint32_t*)nullptr, st);
    } else {  // wider buckets: out-degrees per bucket in LDS, placement by global cursors
        hipLaunchKernelGGL(k_fill_u32, dim3(gN), dim3(256), 0, s, dout, (uint64_t)n, 0u);
        hipLaunchKernelGGL(k_out_count, dim3(grid_for(E, DEG_SLICE, 4096)), dim3(1024), 0, s, opart, bscan, D.nblk,
                           D.NB, D.shift, n, dout);
        if (scan_u32(dout, n, part, off, s) != hipSuccess) return REPT_EDEVICE;
        hipLaunchKernelGGL(k_fill_u32, dim3(gS), dim3(256), 0, s, scnt, nsh, 0u);
        hipLaunchKernelGGL(k_copy_u32, dim3(gN), dim3(256), 0, s, off, (uint64_t)n, cursor);
        hipLaunchKernelGGL(k_scatter, dim3(gE), dim3(256), 0, s, ab, E, dout, cursor, packed, scnt, st);
    }
    // Reverse lists.  Sliced: the sorts mark each reverse pair's source at its adjacency position
    // (in the partition's space, free after the placement) and a bucketed transpose builds the
    // lists below.  Otherwise: shard starts from k_scatter's counts, and the sorts place the
    // records with shard cursors.
    uint32_t* rsrc = (uint32_t*)opart;
    RevOut RO{nullptr, rrec, rpos, rsrc};
    if (!sliced) {
        if (scan_u32(scnt, nsh, part, sofs, s) != hipSuccess) return REPT_EDEVICE;
        hipLaunchKernelGGL(k_rev_roff, dim3(gN), dim3(256), 0, s, sofs, n, roff, st);
        hipLaunchKernelGGL(k_copy_u32, dim3(gS), dim3(256), 0, s, sofs, nsh, scnt);  // shard cursors
        RO = RevOut{scnt, rrec, rpos, nullptr};
    }
    hipLaunchKernelGGL(k_classify, dim3(gA), dim3(256), 0, s, off, n, medium, large, st);
    hipLaunchKernelGGL(k_sort_small, dim3(grid_for((uint64_t)n, 256, cap)), dim3(256), 0, s, off, n, packed, nbr,
                       tim, RO, st);
    hipLaunchKernelGGL(k_sort_wave, dim3(cus ? cus * 8 : 2048), dim3(256), 0, s, off, medium, packed, nbr, tim,
                       RO, st);
    hipLaunchKernelGGL(k_sort_medium, dim3(cus ? cus * 4 : 1024), dim3(512), 0, s, off, medium, n, packed, nbr,
                       tim, RO, st);
    uint32_t id_bits = 1;
    while (id_bits < 32 && ((uint64_t)1 << id_bits) < (uint64_t)n) ++id_bits;
    hipLaunchKernelGGL(k_sort_large, dim3(cus ? cus : 256), dim3(64), 0, s, off, large, packed, alt, id_bits,
                       nbr, tim, RO, st);
    if (sliced) {
        // the reverse pairs (b, a, t, p) partitioned by the bucket of b into the sort buffers
        // (`packed` and `alt`, 16 bytes per edge together, free after the sorts)
        uint4* rpart = (uint4*)packed;
        uint32_t* rcnt = cursor;
        hipLaunchKernelGGL(k_rev_hist, dim3(D.nblk), dim3(1024), 0, s, rsrc, nbr, off, n, D.shift, D.NB,
                           D.per_block, bhist);
        if (scan_u32(bhist, (uint64_t)D.NB * D.nblk, part, bscan, s) != hipSuccess) return REPT_EDEVICE;
        hipLaunchKernelGGL(k_rev_part, dim3(D.nblk), dim3(1024), 0, s, rsrc, nbr, tim, off, n, D.shift, D.NB,
                           D.per_block, bscan, rpart);
        hipLaunchKernelGGL(k_slice_plan, dim3(1), dim3(1024), 0, s, bscan, D.nblk, D.NB, slice_off);
        hipLaunchKernelGGL(k_slice_count<uint4>, dim3((uint32_t)smax), dim3(1024), 0, s, (const uint4*)rpart, bscan,
                           D.nblk, D.NB, D.shift, slice_off, scount);
        hipLaunchKernelGGL(k_slice_dout, dim3(gN), dim3(256), 0, s, scount, slice_off, D.shift, n, rcnt);
        if (scan_u32(rcnt, n, part, roff, s) != hipSuccess) return REPT_EDEVICE;
        hipLaunchKernelGGL(k_slice_base, dim3(gN), dim3(256), 0, s, scount, slice_off, D.shift, n, roff);
        hipLaunchKernelGGL(k_rev_place, dim3((uint32_t)smax), dim3(1024), 0, s, (const uint4*)rpart, bscan, D.nblk,
                           D.NB, D.shift, slice_off, scount, off, rrec, rpos);
    }
    hipLaunchKernelGGL(k_apex_hist, dim3(gA), dim3(256), 0, s, off, roff, n, ahist, st);
    if (scan_u32(ahist, n, part, aoff, s) != hipSuccess) return REPT_EDEVICE;
    hipLaunchKernelGGL(k_fill_u32, dim3(gN), dim3(256), 0, s, cursor, (uint64_t)n, 0u);
    hipLaunchKernelGGL(k_apex_scatter, dim3(gA), dim3(256), 0, s, off, roff, n, aoff, cursor, apex);
    if (hipGetLastError() != hipSuccess) return REPT_EDEVICE;

    BuildStats hs;
    if (hipMemcpyAsync(&hs, st, sizeof(hs), hipMemcpyDeviceToHost, s) != hipSuccess) return REPT_EDEVICE;
    if (hipStreamSynchronize(s) != hipSuccess) return REPT_EDEVICE;
    if (hs.flags & RF_RANGE) return REPT_ERANGE;
    if (hs.flags & RF_SELFLOOP) return REPT_ESELFLOOP;
    if (hs.flags & RF_DUP) return REPT_EDUP;

    rept_graph* g = (rept_graph*)calloc(1, sizeof(rept_graph));
    if (!g) return REPT_ENOMEM;
    g->magic = REPT_MAGIC;
    g->n = n;
    g->E = E;
    g->ctrl = P + L.ctrl;
    g->off = off;
    g->nbr = nbr;
    g->tim = tim;
    g->apex = apex;
    g->roff = roff;
    g->rrec = rrec;
    g->rpos = rpos;
    g->num_apex = hs.num_apex;
    g->max_out = hs.max_out;
    g->num_rev = hs.num_rev;
    g->work = hs.work;
    g->sum_out_sq = hs.sum_out_sq;
    *out = g;
    return REPT_OK;
}
