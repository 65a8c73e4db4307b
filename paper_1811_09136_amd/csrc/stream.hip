// Incremental streaming (Section II: the stream arrives over time; REPT's sets are built on the
// fly): the stream is taken in chunks, and after every chunk the counters hold Algorithm 1's
// updates of every edge seen so far.
//
// State on the device: the whole adjacency of the edges seen so far, both directions, as one
// array of keys (x << 32 | y) sorted by (x, y) with the arrival time of each edge beside it,
// and the node offsets into it.  An append:
//   1. turns the chunk into keys (both directions, times T .. T+W-1) and checks ids and
//      self-loops;
//   2. sorts the chunk's keys (a stable LSD radix sort of 8-bit digits over the key bits that can
//      be set);
//   3. checks for an unordered pair twice in the chunk or already in the adjacency (binary
//      search in the node's sorted list), and finds each node's run in the sorted chunk;
//   4. after the host has read the validation word (the one synchronisation), merges the chunk
//      into the adjacency: every old and every new entry computes its merged position by one
//      binary search in the other side's run of the same node, so the merge is one pass;
//   5. counts the chunk's edges: for the edge (u, v) at time t, the entries w of the shorter of
//      the two lists that arrived before t are searched in the other list (arrived before t as
//      well); each common neighbour is a triangle whose last edge is (u, v), and every group
//      whose hash puts {u, w} and {v, w} in the same active slot adds it to that processor's
//      counters (Algorithm 1's UpdateTriangleCNT).  The work is one item per (edge, entry of
//      its shorter list), spread evenly over the grid through an inclusive scan of the lengths.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.h"
#include "edge_hash.h"

namespace {

constexpr uint32_t kThreads = 256;
constexpr uint32_t kHist = 1024;  // processors aggregated in LDS by the counting kernel

__device__ __forceinline__ uint32_t hi32(uint64_t k) { return (uint32_t)(k >> 32); }
__device__ __forceinline__ uint32_t lo32(uint64_t k) { return (uint32_t)k; }

// first index in [lo, hi) with key >= x (keys sorted ascending)
__device__ __forceinline__ uint64_t lower_bound64(const uint64_t* __restrict__ k, uint64_t lo, uint64_t hi,
                                                  uint64_t x) {
    while (lo < hi) {
        const uint64_t mid = (lo + hi) >> 1;
        if (k[mid] < x) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// 1. chunk edges -> keys of both directions, times; invalid ids are flagged and replaced by
// node 0 so that every later index stays in range (the append is refused anyway)
__global__ void __launch_bounds__(kThreads) k_inc_keys(const uint2* __restrict__ edges, uint64_t W, uint32_t n,
                                                       uint32_t T, uint64_t* __restrict__ key,
                                                       uint32_t* __restrict__ tim, uint32_t* __restrict__ flags) {
    uint32_t f = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < W; i += (uint64_t)gridDim.x * blockDim.x) {
        uint2 e = edges[i];
        if (e.x >= n || e.y >= n) {
            f |= RF_RANGE;
            e = make_uint2(0u, 0u);
        } else if (e.x == e.y) {
            f |= RF_SELFLOOP;
        }
        key[2 * i] = ((uint64_t)e.x << 32) | e.y;
        key[2 * i + 1] = ((uint64_t)e.y << 32) | e.x;
        tim[2 * i] = tim[2 * i + 1] = T + (uint32_t)i;
    }
    if (f) atomicOr(flags, f);
}

// 3a. a pair twice in the sorted chunk, or already in the adjacency
__global__ void __launch_bounds__(kThreads) k_inc_check(const uint64_t* __restrict__ ck, uint64_t N2,
                                                        const uint64_t* __restrict__ akey,
                                                        const uint32_t* __restrict__ off,
                                                        uint32_t* __restrict__ flags) {
    uint32_t f = 0;
    for (uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; p < N2; p += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t k = ck[p];
        if (p && ck[p - 1] == k) f |= RF_DUP;
        const uint32_t x = hi32(k);
        const uint64_t s = off[x], e = off[x + 1];
        const uint64_t j = lower_bound64(akey, s, e, k);
        if (j < e && akey[j] == k) f |= RF_DUP;
    }
    if (f) atomicOr(flags, f);
}

// 3b. coff[x] = first chunk position with node >= x, for x in [0, n]
__global__ void __launch_bounds__(kThreads) k_inc_coff(const uint64_t* __restrict__ ck, uint64_t N2, uint32_t n,
                                                       uint32_t* __restrict__ coff) {
    for (uint64_t x = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; x <= n; x += (uint64_t)gridDim.x * blockDim.x)
        coff[x] = (uint32_t)lower_bound64(ck, 0, N2, x << 32);
}

// 4a. old entries move up by the number of chunk entries of their node with a smaller key
__global__ void __launch_bounds__(kThreads) k_inc_merge_old(const uint64_t* __restrict__ akey,
                                                            const uint32_t* __restrict__ atim, uint64_t N,
                                                            const uint32_t* __restrict__ off,
                                                            const uint32_t* __restrict__ coff,
                                                            const uint64_t* __restrict__ ck,
                                                            uint64_t* __restrict__ okey, uint32_t* __restrict__ otim) {
    for (uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; p < N; p += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t k = akey[p];
        const uint32_t x = hi32(k);
        const uint64_t r = lower_bound64(ck, coff[x], coff[x + 1], k) - coff[x];
        const uint64_t q = p + coff[x] + r;  // off[x] + coff[x] + (p - off[x]) + r
        okey[q] = k;
        otim[q] = atim[p];
    }
}

// 4b. chunk entries land after the old entries of their node with a smaller key
__global__ void __launch_bounds__(kThreads) k_inc_merge_new(const uint64_t* __restrict__ ck,
                                                            const uint32_t* __restrict__ ct, uint64_t N2,
                                                            const uint32_t* __restrict__ off,
                                                            const uint64_t* __restrict__ akey,
                                                            uint64_t* __restrict__ okey, uint32_t* __restrict__ otim) {
    for (uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; p < N2; p += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t k = ck[p];
        const uint32_t x = hi32(k);
        const uint64_t r = lower_bound64(akey, off[x], off[x + 1], k) - off[x];
        const uint64_t q = off[x] + p + r;  // off[x] + coff[x] + (p - coff[x]) + r
        okey[q] = k;
        otim[q] = ct[p];
    }
}

// 4c. merged offsets: off[x] += coff[x]
__global__ void __launch_bounds__(kThreads) k_inc_off(uint32_t* __restrict__ off, const uint32_t* __restrict__ coff,
                                                      uint32_t n) {
    for (uint64_t x = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; x <= n; x += (uint64_t)gridDim.x * blockDim.x)
        off[x] += coff[x];
}

// 5a. items per chunk entry: the shorter list's length for the entry (u, v) with u < v (each
// chunk edge once), 0 for the other direction
__global__ void __launch_bounds__(kThreads) k_inc_lens(const uint64_t* __restrict__ ck, uint64_t N2,
                                                       const uint32_t* __restrict__ off, uint64_t* __restrict__ len) {
    for (uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; p < N2; p += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t k = ck[p];
        const uint32_t u = hi32(k), v = lo32(k);
        uint64_t l = 0;
        if (u < v) {
            const uint32_t du = off[u + 1] - off[u], dv = off[v + 1] - off[v];
            l = du < dv ? du : dv;
        }
        len[p] = l;
    }
}

// first p in [lo, hi) with end[p] > i (end ascending)
__device__ __forceinline__ uint64_t upper_item(const uint64_t* __restrict__ end, uint64_t lo, uint64_t hi, uint64_t i) {
    while (lo < hi) {
        const uint64_t mid = (lo + hi) >> 1;
        if (end[mid] <= i) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// 5b. the count: item i belongs to the chunk entry p with end[p - 1] <= i < end[p].  A workgroup
// takes kRun consecutive items; the slice of `end` they fall in is staged in LDS when it is
// short enough (entries without items, the reverse direction of each edge, also sit in it),
// so that each item finds its entry there.
constexpr uint32_t kRun = 4096;    // items per workgroup run (16 per thread)
constexpr uint32_t kStage = 4096;  // entries of `end` staged per run, at most
__global__ void __launch_bounds__(kThreads) k_inc_count(IncCount a) {
    __shared__ unsigned int hist[kHist];
    __shared__ uint64_t s_end[kStage];
    __shared__ uint64_t s_lo, s_hi;
    const bool use_hist = a.c <= kHist;
    for (uint32_t i = threadIdx.x; i < kHist; i += blockDim.x) hist[i] = 0u;
    const uint64_t total = a.N2 ? a.end[a.N2 - 1] : 0;
    // items counted into the histogram since its last flush: each item adds at most one to a
    // processor's counter, so flushing once this reaches 2^31 keeps every counter below 2^32
    uint64_t since = 0;
    for (uint64_t i0 = (uint64_t)blockIdx.x * kRun; i0 < total; i0 += (uint64_t)gridDim.x * kRun) {
        const uint64_t i1 = (i0 + kRun) < total ? (i0 + kRun) : total;
        if (use_hist && since + (i1 - i0) > (1ull << 31)) {  // uniform over the workgroup
            __syncthreads();
            for (uint32_t i = threadIdx.x; i < a.c; i += blockDim.x) {
                if (hist[i]) atomicAdd((unsigned long long*)a.global + i, (unsigned long long)hist[i]);
                hist[i] = 0u;
            }
            since = 0;
        }
        since += i1 - i0;
        __syncthreads();  // the previous run's readers of s_end are done (and the flush's)
        if (threadIdx.x == 0) {
            s_lo = upper_item(a.end, 0, a.N2, i0);
            s_hi = upper_item(a.end, s_lo, a.N2, i1 - 1) + 1;  // entries [lo, hi) hold the run
        }
        __syncthreads();
        const uint64_t plo = s_lo, phi = s_hi;
        const bool staged = phi - plo <= kStage;
        if (staged)
            for (uint64_t k = threadIdx.x; k < phi - plo; k += blockDim.x) s_end[k] = a.end[plo + k];
        __syncthreads();
        for (uint64_t i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
            uint64_t p;
            if (staged) {
                uint32_t lo = 0, hi = (uint32_t)(phi - plo);
                while (lo < hi) {
                    const uint32_t mid = (lo + hi) >> 1;
                    if (s_end[mid] <= i) lo = mid + 1;
                    else hi = mid;
                }
                p = plo + lo;
            } else {
                p = upper_item(a.end, plo, phi, i);
            }
            const uint64_t k = a.ck[p];
            const uint32_t t = a.ct[p];
            const uint32_t u = hi32(k), v = lo32(k);
            const uint32_t su = a.off[u], du = a.off[u + 1] - su, sv = a.off[v], dv = a.off[v + 1] - sv;
            const uint64_t before = p ? (staged && p > plo ? s_end[p - 1 - plo] : a.end[p - 1]) : 0;
            const uint64_t j = i - before;
            // A: the shorter list (ties: u's), B: the other
            const bool au = du <= dv;
            const uint32_t sa = au ? su : sv;
            const uint32_t sb = au ? sv : su, db = au ? dv : du, b = au ? v : u;
            const uint32_t ta = a.tim[sa + j];
            if (ta >= t) continue;  // {x, w} arrived at or after (u, v): not yet in any set
            const uint32_t w = lo32(a.key[sa + j]);
            const uint64_t want = ((uint64_t)b << 32) | w;
            const uint64_t q = lower_bound64(a.key, sb, (uint64_t)sb + db, want);
            if (q >= (uint64_t)sb + db || a.key[q] != want || a.tim[q] >= t) continue;
            // triangle {u, v, w} with last edge (u, v): per group, the processor that stored both
            // {u, w} and {v, w}, if one did
            for (uint32_t g = 0; g < a.G; ++g) {
                const uint64_t* c4 = a.hp + 4 * g;
                const uint32_t s1 = rept_hash::slot_of(c4, a.m, u, w);
                const uint32_t s2 = rept_hash::slot_of(c4, a.m, v, w);
                const uint32_t active = (g + 1 < a.G) ? a.ck_full : a.last_ck;
                if (s1 != s2 || s1 >= active) continue;
                const uint32_t proc = g * a.pstride + s1;
                if (use_hist) atomicAdd(&hist[proc], 1u);
                else atomicAdd((unsigned long long*)a.global + proc, 1ull);
                int64_t* row = a.local + (uint64_t)(a.per_proc ? proc : g) * a.n;
                atomicAdd((unsigned long long*)row + u, 1ull);
                atomicAdd((unsigned long long*)row + v, 1ull);
                atomicAdd((unsigned long long*)row + w, 1ull);
            }
        }
    }
    if (use_hist) {
        __syncthreads();
        for (uint32_t i = threadIdx.x; i < a.c; i += blockDim.x)
            if (hist[i]) atomicAdd((unsigned long long*)a.global + i, (unsigned long long)hist[i]);
    }
}

__global__ void k_inc_zero64(uint64_t* p, uint64_t words) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = 0ull;
}

uint32_t grid_of(uint64_t items, uint32_t cap) {
    uint64_t b = (items + kThreads - 1) / kThreads;
    if (b > cap) b = cap;
    return b ? (uint32_t)b : 1u;
}

// ---- scans: a tile of SC_TILE items per block (256 threads x 16), the tiles' sums scanned by one
// block, then each tile scanned again from its base
constexpr uint32_t SC_ITEMS = 16;
constexpr uint32_t SC_TILE = kThreads * SC_ITEMS;

template <typename T>
__device__ T block_excl_scan(T v, T& total) {  // 256 threads
    __shared__ T ws[kThreads / 64];
    const uint32_t lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    T inc = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const T o = __shfl_up(inc, d, 64);
        if ((int)lane >= d) inc += o;
    }
    if (lane == 63) ws[w] = inc;
    __syncthreads();
    T base = 0, tot = 0;
#pragma unroll
    for (uint32_t i = 0; i < kThreads / 64; ++i) {
        if (i < w) base += ws[i];
        tot += ws[i];
    }
    __syncthreads();
    total = tot;
    return base + inc - v;
}

template <typename T>
__global__ void __launch_bounds__(kThreads) k_scan_sums(const T* __restrict__ in, uint64_t N, T* __restrict__ part) {
    const uint64_t b0 = (uint64_t)blockIdx.x * SC_TILE;
    T s = 0;
    for (uint32_t r = 0; r < SC_ITEMS; ++r) {
        const uint64_t i = b0 + (uint64_t)r * kThreads + threadIdx.x;
        if (i < N) s += in[i];
    }
    T tot;
    (void)block_excl_scan<T>(s, tot);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// exclusive scan of the tiles' sums in place (one block)
template <typename T>
__global__ void __launch_bounds__(kThreads) k_scan_parts(T* part, uint32_t nparts) {
    __shared__ T carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (uint32_t b = 0; b < nparts; b += kThreads) {
        const uint32_t i = b + threadIdx.x;
        const T v = i < nparts ? part[i] : 0;
        T tot;
        const T ex = block_excl_scan<T>(v, tot);
        const T c = carry;
        if (i < nparts) part[i] = c + ex;
        __syncthreads();
        if (threadIdx.x == 0) carry = c + tot;
        __syncthreads();
    }
}

// out[i] = sum of in[0..i] (INCL) or in[0..i) (exclusive), each thread 16 consecutive items
template <typename T, bool INCL>
__global__ void __launch_bounds__(kThreads) k_scan_items(const T* __restrict__ in, uint64_t N,
                                                         const T* __restrict__ part, T* __restrict__ out) {
    const uint64_t b0 = (uint64_t)blockIdx.x * SC_TILE + (uint64_t)threadIdx.x * SC_ITEMS;
    T v[SC_ITEMS];
    T s = 0;
#pragma unroll
    for (uint32_t r = 0; r < SC_ITEMS; ++r) {
        const uint64_t i = b0 + r;
        v[r] = i < N ? in[i] : 0;
        s += v[r];
    }
    T tot;
    T run = block_excl_scan<T>(s, tot) + part[blockIdx.x];
#pragma unroll
    for (uint32_t r = 0; r < SC_ITEMS; ++r) {
        const uint64_t i = b0 + r;
        if (INCL) run += v[r];
        if (i < N) out[i] = run;
        if (!INCL) run += v[r];
    }
}

template <typename T, bool INCL>
hipError_t scan_items(const T* in, uint64_t N, T* part, T* out, hipStream_t s) {
    const uint64_t nb = (N + SC_TILE - 1) / SC_TILE;
    if (nb == 0) return hipSuccess;
    hipLaunchKernelGGL(k_scan_sums<T>, dim3((uint32_t)nb), dim3(kThreads), 0, s, in, N, part);
    hipLaunchKernelGGL(k_scan_parts<T>, dim3(1), dim3(kThreads), 0, s, part, (uint32_t)nb);
    hipLaunchKernelGGL((k_scan_items<T, INCL>), dim3((uint32_t)nb), dim3(kThreads), 0, s, in, N, part, out);
    return hipGetLastError();
}

// ---- stable LSD radix sort of (key, time) pairs: one 8-bit digit per pass.  A block takes a
// tile of RS_TILE pairs, each of its four wavefronts a contiguous quarter; the pass counts the
// digits per tile, scans the counts digit-major (all tiles' 0s, then all tiles' 1s, ...), and
// scatters each tile stably: a wavefront ranks its lanes among the lanes of the same digit
// (eight ballots) and keeps a running base per digit, seeded from the tile's base plus the
// counts of the wavefronts before it.
constexpr uint32_t RS_TILE = 4096;
constexpr uint32_t RS_WAVE = RS_TILE / (kThreads / 64);

__global__ void __launch_bounds__(kThreads) k_rs_hist(const uint64_t* __restrict__ keys, uint64_t N, uint32_t shift,
                                                      uint32_t nb, uint32_t* __restrict__ hist) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const uint64_t b0 = (uint64_t)blockIdx.x * RS_TILE, b1 = (b0 + RS_TILE) < N ? (b0 + RS_TILE) : N;
    for (uint64_t i = b0 + threadIdx.x; i < b1; i += kThreads) atomicAdd(&h[(uint32_t)(keys[i] >> shift) & 255u], 1u);
    __syncthreads();
    hist[(uint64_t)threadIdx.x * nb + blockIdx.x] = h[threadIdx.x];
}

__global__ void __launch_bounds__(kThreads) k_rs_scatter(const uint64_t* __restrict__ kin, const uint32_t* __restrict__ vin,
                                                         uint64_t N, uint32_t shift, uint32_t nb,
                                                         const uint32_t* __restrict__ offs, uint64_t* __restrict__ kout,
                                                         uint32_t* __restrict__ vout) {
    __shared__ uint32_t wc[kThreads / 64][256];  // per wavefront: digit counts, then running bases
    const uint32_t lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (uint32_t i = threadIdx.x; i < (kThreads / 64) * 256; i += kThreads) (&wc[0][0])[i] = 0;
    __syncthreads();
    const uint64_t t0 = (uint64_t)blockIdx.x * RS_TILE + (uint64_t)w * RS_WAVE;
    const uint64_t t1 = (t0 + RS_WAVE) < N ? (t0 + RS_WAVE) : N;
    for (uint64_t c0 = t0; c0 < t1; c0 += 64) {
        const uint64_t i = c0 + lane;
        if (i < t1) atomicAdd(&wc[w][(uint32_t)(kin[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    {  // thread d: the bases of digit d for the four wavefronts of this tile
        const uint32_t d = threadIdx.x;
        uint32_t run = offs[(uint64_t)d * nb + blockIdx.x];
        for (uint32_t v = 0; v < kThreads / 64; ++v) {
            const uint32_t c = wc[v][d];
            wc[v][d] = run;
            run += c;
        }
    }
    __syncthreads();
    const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
    for (uint64_t c0 = t0; c0 < t1; c0 += 64) {
        const uint64_t i = c0 + lane;
        const bool valid = i < t1;
        const uint64_t k = valid ? kin[i] : 0ull;
        const uint32_t t = valid ? vin[i] : 0u;
        const uint32_t dig = (uint32_t)(k >> shift) & 255u;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int bit = 0; bit < 8; ++bit) {
            const uint64_t bb = __ballot(valid && ((dig >> bit) & 1u));
            peers &= ((dig >> bit) & 1u) ? bb : ~bb;
        }
        const uint32_t pos = wc[w][dig] + (uint32_t)__popcll(peers & below);
        if (valid) {
            kout[pos] = k;
            vout[pos] = t;
            // the highest lane of the digit advances its base (after every lane has read it)
            if ((int)lane == 63 - __clzll(peers)) wc[w][dig] += (uint32_t)__popcll(peers);
        }
    }
}

__global__ void k_copy_pairs(const uint64_t* __restrict__ ks, const uint32_t* __restrict__ vs, uint64_t N,
                             uint64_t* __restrict__ kd, uint32_t* __restrict__ vd) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (uint64_t)gridDim.x * blockDim.x) {
        kd[i] = ks[i];
        vd[i] = vs[i];
    }
}

// temporary storage of the sort and the scans: the digit counts and their scan, then the scans'
// tile sums
struct SortTemp {
    size_t hist, offs, part, total;
};
SortTemp sort_temp(uint64_t N) {
    SortTemp T;
    const uint64_t nb = (N + RS_TILE - 1) / RS_TILE;
    const uint64_t nh = 256 * (nb ? nb : 1);
    const uint64_t parts = (nh + SC_TILE - 1) / SC_TILE + (N + SC_TILE - 1) / SC_TILE + 2;
    size_t p = 0;
    T.hist = p; p = (p + 4 * nh + 255) & ~(size_t)255;
    T.offs = p; p = (p + 4 * (nh + 1) + 255) & ~(size_t)255;
    T.part = p; p = (p + 8 * parts + 255) & ~(size_t)255;
    T.total = p;
    return T;
}

// sorts (ka, ta) by the key bits below end_bit that can be set (ids below 2^(end_bit - 32) on
// both halves), the result in (kb, tb); (ka, ta) is overwritten
hipError_t radix_sort_keys(void* temp, uint64_t N, uint32_t end_bit, uint64_t* ka, uint32_t* ta, uint64_t* kb,
                           uint32_t* tb, hipStream_t s) {
    if (N == 0) return hipSuccess;
    const SortTemp L = sort_temp(N);
    uint32_t* hist = (uint32_t*)((uint8_t*)temp + L.hist);
    uint32_t* offs = (uint32_t*)((uint8_t*)temp + L.offs);
    uint32_t* part = (uint32_t*)((uint8_t*)temp + L.part);
    const uint32_t nb = (uint32_t)((N + RS_TILE - 1) / RS_TILE);
    const uint32_t id_bits = end_bit - 32;
    uint64_t *src_k = ka, *dst_k = kb;
    uint32_t *src_t = ta, *dst_t = tb;
    for (uint32_t half = 0; half < 2; ++half) {  // y (bits 0..), then x (bits 32..)
        for (uint32_t b = 0; b < id_bits; b += 8) {
            const uint32_t shift = 32 * half + b;
            hipLaunchKernelGGL(k_rs_hist, dim3(nb), dim3(kThreads), 0, s, src_k, N, shift, nb, hist);
            hipError_t e = scan_items<uint32_t, false>(hist, (uint64_t)256 * nb, part, offs, s);
            if (e != hipSuccess) return e;
            hipLaunchKernelGGL(k_rs_scatter, dim3(nb), dim3(kThreads), 0, s, src_k, src_t, N, shift, nb, offs, dst_k,
                               dst_t);
            uint64_t* tk = src_k; src_k = dst_k; dst_k = tk;
            uint32_t* tt = src_t; src_t = dst_t; dst_t = tt;
        }
    }
    if (src_k != kb)
        hipLaunchKernelGGL(k_copy_pairs, dim3(grid_of(N, 8192)), dim3(kThreads), 0, s, src_k, src_t, N, kb, tb);
    return hipGetLastError();
}

}  // namespace

// ---------------------------------------------------------------------------- launchers ----

size_t rept_inc_sort_temp_bytes(uint64_t entries, uint32_t end_bit) {
    (void)end_bit;
    return sort_temp(entries).total;
}

hipError_t rept_inc_zero64(void* p, uint64_t words, hipStream_t s) {
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_inc_zero64, dim3(grid_of(words, 4096)), dim3(kThreads), 0, s, (uint64_t*)p, words);
    return hipGetLastError();
}

hipError_t rept_inc_prepare(const IncState& st, const uint32_t* edges, uint64_t W, hipStream_t s) {
    (void)hipGetLastError();
    const uint64_t N2 = 2 * W;
    hipLaunchKernelGGL(k_inc_zero64, dim3(1), dim3(64), 0, s, (uint64_t*)st.flags, (uint64_t)1);
    hipLaunchKernelGGL(k_inc_keys, dim3(grid_of(W, 8192)), dim3(kThreads), 0, s, (const uint2*)edges, W, st.n,
                       (uint32_t)st.T, st.ckey_a, st.ctim_a, st.flags);
    hipError_t e = radix_sort_keys(st.temp, N2, st.end_bit, st.ckey_a, st.ctim_a, st.ckey_b, st.ctim_b, s);
    if (e != hipSuccess) return e;
    const uint64_t* akey = st.key[st.cur];
    hipLaunchKernelGGL(k_inc_check, dim3(grid_of(N2, 8192)), dim3(kThreads), 0, s, st.ckey_b, N2, akey, st.off,
                       st.flags);
    hipLaunchKernelGGL(k_inc_coff, dim3(grid_of((uint64_t)st.n + 1, 8192)), dim3(kThreads), 0, s, st.ckey_b, N2,
                       st.n, st.coff);
    return hipGetLastError();
}

hipError_t rept_inc_merge(IncState& st, uint64_t W, hipStream_t s) {
    (void)hipGetLastError();
    const uint64_t N2 = 2 * W, N = 2 * st.T;
    const int nxt = st.cur ^ 1;
    hipLaunchKernelGGL(k_inc_merge_old, dim3(grid_of(N, 8192)), dim3(kThreads), 0, s, st.key[st.cur], st.tim[st.cur],
                       N, st.off, st.coff, st.ckey_b, st.key[nxt], st.tim[nxt]);
    hipLaunchKernelGGL(k_inc_merge_new, dim3(grid_of(N2, 8192)), dim3(kThreads), 0, s, st.ckey_b, st.ctim_b, N2,
                       st.off, st.key[st.cur], st.key[nxt], st.tim[nxt]);
    hipLaunchKernelGGL(k_inc_off, dim3(grid_of((uint64_t)st.n + 1, 8192)), dim3(kThreads), 0, s, st.off, st.coff,
                       st.n);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    st.cur = nxt;
    st.T += W;
    // the chunk's work items: one per entry of the shorter endpoint list of each chunk edge
    uint64_t* len = st.ckey_a;  // free after the sort
    hipLaunchKernelGGL(k_inc_lens, dim3(grid_of(N2, 8192)), dim3(kThreads), 0, s, st.ckey_b, N2, st.off, len);
    return scan_items<uint64_t, true>(len, N2, (uint64_t*)((uint8_t*)st.temp + sort_temp(N2).part), st.end, s);
}

hipError_t rept_inc_count(const IncState& st, uint64_t W, const IncCount& base, hipStream_t s) {
    (void)hipGetLastError();
    const uint64_t N2 = 2 * W;
    IncCount a = base;
    a.key = st.key[st.cur];
    a.tim = st.tim[st.cur];
    a.off = st.off;
    a.ck = st.ckey_b;
    a.ct = st.ctim_b;
    a.end = st.end;
    a.N2 = N2;
    hipLaunchKernelGGL(k_inc_count, dim3(st.count_blocks), dim3(kThreads), 0, s, a);
    return hipGetLastError();
}
