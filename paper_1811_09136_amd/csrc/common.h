// Internal declarations shared by the build, count and C-ABI translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rept.h"

#define REPT_GMAX 8           // hash groups handled by one launch (c <= 8*m)
// a unit's order key is max(list length, reverse-list length >> REPT_REV_SHIFT): a long reverse
// list is many lists to walk even under a short own list
#define REPT_REV_SHIFT 3
#define REPT_HIST_CAP 1024    // processors aggregated in LDS; larger c uses direct atomics
#define REPT_CTRL_BYTES 4096  // control block at the head of a graph's persistent buffer
#define REPT_MAGIC 0x52455054u

// validation flags written by the build kernels
#define RF_RANGE 1u
#define RF_SELFLOOP 2u
#define RF_DUP 4u

// Build statistics, written by the build kernels into scratch and read once by the host.
struct BuildStats {
    uint32_t flags;
    uint32_t num_apex;
    uint32_t max_out;
    uint32_t n_medium;  // segments sorted by a workgroup in LDS
    uint32_t n_large;   // segments sorted by a workgroup in global memory
    uint32_t num_rev;   // pairs in the reverse lists
    uint32_t n_wave;    // segments sorted in registers by one wavefront each
    uint32_t n_ends;    // endpoints of the valid edges (the degree partition's length)
    unsigned long long work;        // sum over oriented edges a->b of min(outdeg(a), outdeg(b))
    unsigned long long sum_out_sq;  // sum over nodes of outdeg^2
};

// Host handle (opaque to callers).
struct rept_graph {
    uint32_t magic;
    uint32_t n;
    uint64_t E;
    uint8_t* ctrl;       // device control block (REPT_CTRL_BYTES) for single-job launches
    const uint32_t* off; // [n+1] oriented adjacency offsets
    const uint32_t* nbr; // [E] higher-ranked neighbour ids, sorted within each segment
    const uint32_t* tim; // [E] arrival time of that edge
    const uint32_t* apex;// [num_apex] nodes with outdeg >= 2, by outdeg descending
    const uint32_t* roff;  // [n+1] reverse lists: pairs a -> b with outdeg(a) < outdeg(b), at b
    const uint4* rrec;     // [.] (a, arrival time of a-b, offset of a's list, length of a's list)
    const uint32_t* rpos;  // [.] position of b in a's list
    uint32_t num_apex;
    uint32_t max_out;
    uint32_t num_rev;
    uint64_t work;
    uint64_t sum_out_sq;
};

// Device-side job descriptor.
struct JobDev {
    const uint32_t* off;
    const uint32_t* nbr;
    const uint32_t* tim;
    const uint32_t* apex;
    const uint32_t* roff;
    const uint4* rrec;
    const uint32_t* rpos;
    int64_t* global;
    int64_t* local;
    uint64_t hp[4 * REPT_GMAX];  // polynomial hash coefficients (a0, a1, a2, a3) per group
    uint32_t n, m, c, G;
    uint32_t rows;       // local rows: G or c
    uint32_t per_proc;   // 1: local rows are processors
    uint32_t accumulate; // 1: do not zero the outputs first
    uint32_t t0, t1;     // window [t0, t1)
    uint32_t unit0, unit1;       // apex range [unit0, unit1)
    uint32_t n_heavy;            // apexes of the range with outdeg > wave_cap (set by setup)
    uint32_t light_tiles;        // set by setup
    uint32_t heavy_prefix;       // exclusive prefix of heavy units over jobs (set by setup)
    uint32_t light_prefix;       // exclusive prefix of light tiles over jobs (set by setup)
    uint32_t gs;                 // slots per stored edge in the slot table (G padded: 1, 2, 4, 8)
    uint16_t* tab;               // slot table [E][gs]: h_k of the edge stored at each position
    uint32_t fill;               // 1: the launch (re)writes the slot table first
    uint32_t es;                 // stored edges (rows of the pair counters)
    uint32_t* pairs;             // Algorithm 2 pair counters [G][es][2] (s, L), or null
    uint32_t ck, last_ck;        // active slots of a full group and of the last group
    uint32_t pstride;            // processor of slot j of group k: k * pstride + j
    uint32_t mask;               // 1: the table holds keep masks (parallel MASCOT), gs = 1
};

// Work queues of the counting kernel: each phase's tiles are split over kQueues interleaved
// sub-queues (tile t is the (t / kQueues)-th of sub-queue t % kQueues) whose counters sit on
// separate 128-byte lines, so claims spread over kQueues addresses instead of one.
constexpr uint32_t kQueues = 16;
constexpr uint32_t kQueueStride = 32;  // words per counter line
constexpr uint32_t kLightQueue = 0;    // word of the light phase's counter within a line
constexpr uint32_t kHeavyQueue = 16;   // word of the heavy phase's counter within a line

// Batch header, followed in memory by JobDev[njobs].
struct alignas(128) BatchHeader {
    uint32_t njobs;
    uint32_t wave_cap;     // apexes with out-degree <= wave_cap are counted by one wavefront
    uint32_t block_cap;    // adjacency entries staged per hash-table chunk by a workgroup
    uint32_t b_chunk;      // neighbour lists staged per chunk by a workgroup
    uint32_t blocks;       // persistent grid size
    uint32_t threads;      // workgroup size (multiple of 64, <= 1024)
    uint32_t light_tile;   // apexes per light queue tile
    uint32_t hist_c;       // processors aggregated in LDS (0: direct atomics)
    uint32_t G_max;        // max groups over jobs (LDS counter rows)
    uint32_t lds_bytes;    // dynamic LDS bytes per workgroup
    uint32_t heavy_total;  // set by setup
    uint32_t light_total;  // set by setup
    uint32_t any_zero;     // some job overwrites its outputs
    uint32_t light_table;  // hash slots per key, at least, in the light phase (2 or 4)
    uint64_t zero_words;   // max words to clear over jobs
    uint32_t any_fill;     // some job's slot table is written by this launch
    uint32_t fill_edges;   // largest stream length over those jobs (bounds their stored edges)
    uint32_t any_eta;      // some job counts Algorithm 2's pair counters (the kernel's second form)
    uint32_t split;          // 1: the light phase is a launch of its own (shape below)
    uint32_t light_threads;  // its workgroup size
    uint32_t light_blocks;   // its grid
    uint32_t light_lds;      // its dynamic LDS bytes (no heavy team area)
    uint32_t split_streams;  // 1: that launch runs on a second stream, beside the heavy one
    uint32_t heavy_table;    // hash slots per key, at least, in the heavy phase (2 or 4)
    uint32_t light_b;        // neighbour lists staged per chunk by a light-phase wavefront
    uint32_t gs_max;         // slots per staged row in LDS: the widest slot-table row over jobs
    uint32_t queues[kQueues * kQueueStride];  // sub-queue counters, reset by setup
};

static_assert(sizeof(BatchHeader) % 16 == 0, "header alignment");
static_assert(sizeof(JobDev) % 16 == 0, "job alignment");
static_assert(sizeof(BatchHeader) + sizeof(JobDev) <= REPT_CTRL_BYTES, "control block size");

// ---- build (build.hip) ----
size_t rept_host_stage_offset(uint32_t n, uint64_t E);
rept_status rept_build_impl(uint32_t n, const uint32_t* edges, uint64_t E, void* persistent,
                            size_t persistent_bytes, void* scratch, size_t scratch_bytes,
                            hipStream_t stream, rept_graph** out);
void rept_sizes_impl(uint32_t n, uint64_t E, size_t* persistent, size_t* scratch);

// ---- count (count.hip) ----
// Launch setup + zero + heavy + light kernels for a batch already in device memory.
hipError_t rept_launch_batch(void* ws, const BatchHeader& host_hdr, hipStream_t stream);
hipError_t rept_launch_single(uint8_t* ctrl, const BatchHeader& hdr, const JobDev& job,
                              hipStream_t stream);
// slots per stored edge in a slot table for G groups (1, 2, 4 or 8)
inline uint32_t rept_slot_stride(uint32_t G) { return G <= 1 ? 1u : (G <= 2 ? 2u : (G <= 4 ? 4u : 8u)); }
hipError_t rept_launch_zero(void* p, uint64_t bytes, hipStream_t stream);
// Algorithm 2's pair counts of one launch's processors, added to eta[r][proc0 + i] (rows of
// `stride` = c entries) and to eta_v
hipError_t rept_launch_eta(const rept_graph* g, const JobDev& d, int64_t* eta, int64_t* eta_v, uint32_t proc0,
                           uint32_t stride, hipStream_t stream);
hipError_t rept_launch_reduce(const int64_t* local, uint32_t rows, uint32_t n, int64_t* sums, hipStream_t stream);
hipError_t rept_launch_slots(const uint64_t* hp, uint32_t G, uint32_t m, const uint32_t* edges,
                             uint64_t E, uint32_t* slots, hipStream_t stream);
// LDS bytes of the counting kernel for a launch shape (eta: the form with Algorithm 2's counters;
// heavy / light: the launch runs the heavy / light phase; a launch running both shares one LDS
// region between the heavy team area and the wavefronts' light areas)
uint32_t rept_count_lds(uint32_t threads, uint32_t wave_cap, uint32_t block_cap, uint32_t b_chunk, uint32_t G,
                        uint32_t gs, uint32_t hist_c, uint32_t light_table, uint32_t heavy_table, uint32_t light_b,
                        bool eta, bool heavy = true, bool light = true);
// resident workgroups per CU of the counting kernel for a launch shape (0 if unknown)
uint32_t rept_count_blocks_per_cu(uint32_t threads, uint32_t lds_bytes, bool eta);
uint32_t rept_num_cus();

// ---- incremental streaming (stream.hip) ------------------------------------------------------
// Device state of an incrementally built stream: the adjacency of the edges seen so far, both
// directions, keys (x << 32 | y) sorted ascending with arrival times beside them (double
// buffered: the merge writes the other copy), node offsets, and the chunk work space.
struct IncState {
    uint32_t n;
    uint32_t end_bit;  // radix-sort bits of a key: 32 + bit length of n - 1
    uint64_t T;        // edges appended so far
    int cur;           // the current adjacency copy
    uint64_t* key[2];
    uint32_t* tim[2];
    uint32_t* off;   // [n + 1] offsets into the current copy
    uint32_t* coff;  // [n + 1] first position of each node's run in the sorted chunk
    uint64_t *ckey_a, *ckey_b;  // chunk keys before / after the sort (a: item lengths later)
    uint32_t *ctim_a, *ctim_b;
    uint64_t* end;      // inclusive scan of the item lengths
    uint32_t* flags;    // validation word (RF_*)
    void* temp;         // temporary storage of the chunk sort and the scans
    size_t temp_bytes;
    uint32_t count_blocks;
};
// Arguments of the per-edge counting kernel
struct IncCount {
    const uint64_t* key;
    const uint32_t* tim;
    const uint32_t* off;
    const uint64_t* ck;  // sorted chunk keys
    const uint32_t* ct;  // their times
    const uint64_t* end;
    uint64_t N2;
    int64_t* global;
    int64_t* local;
    uint32_t n, m, c, G;
    uint32_t ck_full, last_ck, pstride, per_proc;  // processor map as in JobDev
    uint64_t hp[4 * REPT_GMAX];
};
// temporary bytes for sorting `entries` keys of end_bit bits and scanning as many lengths (the
// library's own radix sort and scans; 0 on failure)
size_t rept_inc_sort_temp_bytes(uint64_t entries, uint32_t end_bit);
hipError_t rept_inc_zero64(void* p, uint64_t words, hipStream_t stream);
// steps 1-3 of an append (keys, sort, validation, chunk runs); the state is not changed
hipError_t rept_inc_prepare(const IncState& st, const uint32_t* edges, uint64_t W, hipStream_t stream);
// step 4: merge the chunk into the adjacency and scan the chunk's work items (one per entry of
// the shorter list of each chunk edge's endpoints; the total is st.end[2W - 1]); advances st.cur
// and st.T
hipError_t rept_inc_merge(IncState& st, uint64_t W, hipStream_t stream);
// step 5: count each chunk edge against the edges that arrived before it (after rept_inc_merge)
hipError_t rept_inc_count(const IncState& st, uint64_t W, const IncCount& base, hipStream_t stream);
