// Device-side definitions shared by the CAFS kernels for gfx950.
//
// Dispatch happens on the device.  Every call enqueues one fixed sequence of
// kernels; the first kernels write their decisions (path, engine, table sizes,
// sizes of intermediate arrays) into a Ctrl block in the workspace, and every
// later kernel reads it and returns at once when its branch is not taken.  The
// host never waits for the GPU, and the sequence can be captured in a graph.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/cafs.h"

namespace cafs {

// ---- constants of the method (CAFS paper) ---------------------------------
constexpr uint32_t kSamples = 1024;            // s, strided samples (Sec. 4.3)
constexpr uint32_t kFreqSlotsLog2 = 12;        // FreqSet of 4096 slots (Sec. 4.3)
constexpr uint64_t kSmallN = 2048;             // Table dispatcher: N < 2048 -> fallback
constexpr uint64_t kTinyK = 8;                 // Table dispatcher: K^ <= 8 and u <= 8
constexpr uint64_t kPhi = 0x9E3779B97F4A7C15ull;  // Eq. hash multiplier
constexpr uint32_t kBucketCap = 4;             // keys per 64-bit bucket (Sec. 4.2)
constexpr uint32_t kBucketCap32 = 8;           // keys per 32-bit bucket (Sec. 4.2)
constexpr uint32_t kMaxBucketCap = 8;

// ---- GPU design constants (not from the paper) ----------------------------
constexpr uint64_t kEmpty = ~0ull;             // empty-slot marker of the GPU hash tables;
                                               // keys equal to it are counted apart
constexpr uint32_t kMonoPrefix = 1u << 13;     // elements the pre kernel checks for order
constexpr int kCountThreads = 1024;            // hash-count workgroup
constexpr uint32_t kLdsSlots = 13568;          // per-workgroup LDS table (159 KiB with 32-bit counts)
constexpr uint32_t kRleProbePairs = 16;        // run-length path for a batch when this many of the 64 pairs of its
                                              // first slice hold two equal elements
constexpr uint32_t kRleMinMerged = 16;         // and, per slice, when its 128 elements merge at least this many
constexpr uint64_t kLdsWideMinKhat = 1800;     // buckets of 4 keys from this estimate up, of 2 below
constexpr uint32_t kLdsWindow = 2;             // buckets probed before an element is deferred
constexpr uint32_t kLdsProbeBuckets = 8;       // buckets probed in the deferred pass before the global table
constexpr uint32_t kMaxCountBlocks = 1024;     // workgroups of one hash count
constexpr uint32_t kGlobalProbe = 16;          // global probe limit: a key not found or placed by then spills
constexpr uint32_t kClosedProbe = 4;           // the same once the table has reached its load limit
constexpr uint32_t kSpillBelow = 4;            // a closed table's flush spills counts below this unprobed
constexpr uint32_t kGlobalProbeCheck = 4;      // a long probe looks at the overflow flag every this many slots
constexpr uint32_t kMaxPartLog2 = 4;           // hash partitions of the column before the count: at most 16
constexpr uint32_t kMaxParts = 1u << kMaxPartLog2;
constexpr uint64_t kTableSlotsPerKey = 32;     // default: global table slots per estimated key
constexpr uint64_t kPartKeys = 6000;           // default: distinct keys per partition the estimate aims at
                                               // (no partitions up to twice that)
constexpr uint32_t kScatterThreads = 1024;     // partition scatter workgroup
constexpr uint32_t kScatterChunk = kScatterThreads * 8;  // elements staged per step
constexpr uint32_t kXcds = 8;                  // accelerator dies
constexpr uint32_t kSpillFracDiv = 4;          // the radix engine takes over when the spill passes N / this
constexpr uint32_t kMinTableLog2 = 12;         // smallest global table (4096 slots)
// Engine planning from a larger sample, for long columns whose estimate shows a
// heavy tail (many singletons among the 1024 samples): the hash count's geometry
// then follows Chao1 over kSamples2 strided samples (the reported estimate, path
// and table M stay the paper's).
constexpr uint64_t kReplanMinN = 1ull << 22;
constexpr uint32_t kReplanMinF1 = 128;
constexpr uint32_t kSamples2 = 65536;
constexpr uint32_t kSamples2Block = 4096;      // samples per workgroup of the larger sample
constexpr uint32_t kSamples2Threads = 1024;    // threads per workgroup of the larger sample
constexpr uint32_t kSample2LdsLog2 = 13;       // its LDS set: 2 * kSamples2Block slots
constexpr uint32_t kSample2SlotsLog2 = 18;     // hash set of the large sample (load <= 1/4)
constexpr uint32_t kMaxTableLog2 = 22;         // largest global table (4M slots, 64 MiB)
constexpr uint32_t kTableFloorLog2 = 16;       // global table never smaller (64K slots) when the workspace allows
constexpr uint32_t kRankMax = 32768;           // K ordered by ranking (larger K: pair radix sort)
constexpr uint32_t kRankKeysPerBlock = 64;     // keys ranked by one workgroup (16 waves)
constexpr uint32_t kRankKeysPerWave = 4;       // keys ranked by one wave, held in registers
constexpr uint32_t kRankTile = 8192;           // keys staged in LDS at a time while ranking
constexpr uint32_t kRankBudgetLog2 = 24;       // compares per ranking workgroup before a pair sort wins
constexpr uint32_t kRankBudgetBatchLog2 = 20;  // the same in a batch, where total work counts more than latency
constexpr uint32_t kGuardLdsBuckets = 16384;   // guard bucket counts kept in LDS up to this M
constexpr int kRadixThreads = 256;             // key-value radix pass workgroup (4 waves)
constexpr int kRadixKeysThreads = 512;         // keys-only radix pass workgroup (8 waves)
constexpr int kRadixItems = 16;                // keys per thread per tile
constexpr uint32_t kRadixTile = kRadixThreads * kRadixItems;  // 4096 keys per tile
constexpr uint32_t kRleTile = 4096;            // elements per run-detection tile
constexpr uint32_t kGuardChunk = 4096;         // elements per first-occurrence chunk
constexpr uint32_t kGuardLdsKeys = 2048;       // contested keys resolved in LDS

enum Path : int32_t { P_MONOTONE = 0, P_SMALL_N = 1, P_TINY = 2, P_HIGH_K = 3, P_MAIN = 4, P_GUARD = 5 };
// Report flags (what ran on the GPU; the oracle does not model them).
constexpr uint32_t kFlagOverflow = 1u;  // the radix engine sorted the column instead of the count
constexpr uint32_t kFlagGuardFirst = 2u;  // the guard needed the first-occurrence pass
constexpr uint32_t kFlagSpill = 4u;     // keys went to the spill list, which was sorted and folded
enum Engine : uint32_t { E_NONE = 0, E_TINY = 1, E_HASH = 2, E_RADIX = 3 };

// Look-back status word of the radix passes: two flag bits over a 62-bit value.
constexpr uint64_t kStatAgg = 1ull << 62;
constexpr uint64_t kStatInc = 2ull << 62;
constexpr uint64_t kStatMask = (1ull << 62) - 1;

// One LSD radix job (the fallback sort of the keys, or the sort of the distinct
// (key, count) pairs when K is too large for the single-workgroup order kernel).
struct RadixJob {
    const uint64_t* src_k;
    const uint64_t* src_v;
    uint64_t* dst_k;
    uint64_t* dst_v;
    uint64_t* tmp_k;
    uint64_t* tmp_v;
    uint64_t n;
    uint32_t has_vals;
    uint32_t n_active;                // passes whose digit is not constant
    uint32_t digit[8];                // digit index of each active pass, in order
    const uint64_t* ps_k[8];          // source of active pass i
    const uint64_t* ps_v[8];
    uint64_t* pd_k[8];                // destination of active pass i
    uint64_t* pd_v[8];
    uint32_t copy_mode;               // after the passes: 0 nothing, 1 copy src->dst, 2 tmp->dst
    uint32_t src_ew, dst_ew;          // element bytes of src and dst (tmp always holds 8-byte keys)
    uint32_t ps_w[8], pd_w[8];        // element bytes of each active pass's source and destination
};

// Decisions and counters of one call, in device memory (workspace).
struct Ctrl {
    // monotone check
    uint32_t inversion;
    uint32_t mono_full;               // the full order check is still needed
    uint32_t mono_done;               // workgroups of the full order check that finished
    // Chao1 estimate
    uint64_t k_hat, u, f1, f2, n_samples, stride;
    uint32_t saturated;
    uint32_t n_tiny;                  // distinct sampled keys kept for the tiny branch (<= 8)
    uint64_t tiny_keys[8];            // sorted in the dtype's order
    // plan
    int32_t path;
    uint32_t engine;
    uint32_t tiny_miss;
    uint32_t flags;                   // report flags
    uint64_t table_M;                 // Eq. Msize
    uint32_t cap_log2;                // GPU global table size (log2 slots)
    uint32_t cap_limit;               // claimed slots allowed; keys arriving later spill
    uint32_t part_log2;               // hash partitions of the count workgroups (log2)
    uint32_t replan;                  // plan the count again from the larger sample
    uint32_t s2done;
    uint32_t lds_wide;                // LDS buckets of 4 keys (else 2)
    // tiny count: each key's counter on a line of its own (every workgroup adds to them)
    alignas(128) uint64_t tiny_cnt[8][16];
    // hash count.  Words that many workgroups update atomically, or poll while
    // others update them, each get a 128-byte line of their own: a read of a line
    // under atomic traffic waits behind it.
    alignas(128) uint32_t overflow;
    alignas(128) uint32_t claimed;
    alignas(128) uint32_t closed;     // the global table reached its load limit (written once)
    alignas(128) uint64_t ecount;     // elements equal to kEmpty
    alignas(128) uint64_t nspill;     // (key, count) pairs on the spill list
    uint64_t spill_limit;             // past this many the radix engine takes over
    // partition buckets in pbuf: bucket q is [pbase[q], pbase[q + 1]); the overflow
    // area after the last bucket, [pbase[P], pbase[P + 1]), takes what a full bucket
    // cannot (its keys are of any partition)
    uint64_t pbase[kMaxParts + 2];
    alignas(128) uint32_t pfill[kMaxParts + 1][32];  // elements sent to each bucket and the overflow area
    // where the sorted column is when the radix engine ran (the output, or scratch
    // when sorting in place on the main path, copied out after the guard)
    uint64_t* sorted;
    uint32_t sorted_ew;               // element bytes of `sorted`
    uint32_t deferred_copy;
    uint32_t pad0;
    // dense (key, count) arrays
    uint64_t K;
    uint32_t emit_main;               // dense arrays from the tiny branch or the rank order
    uint32_t dense_ready;
    uint32_t pair_sort;               // the pairs are radix sorted, then folded and scanned
    const uint64_t* fold_k;           // the sorted pairs the fold reads
    const uint64_t* fold_v;
    uint32_t radix_on;
    uint32_t guard_on;
    // radix
    RadixJob rj;
    uint64_t hist[8][256];
    alignas(128) uint32_t hist_done;
    alignas(128) uint32_t tile_ctr[8];  // (each pass's tiles are claimed from its own counter)
    // run-length pass over a sorted column
    alignas(128) uint32_t rle_done;
    uint32_t rle_on;
    // guard
    uint32_t guard_general;           // bucket counts must be built from the dense pairs
    uint32_t guard_rounds;            // too many contested keys for one workgroup
    uint32_t gidx_log2;               // hash index of the contested keys (0: binary search)
    alignas(128) uint64_t n_contested;
    uint64_t n_cbuckets;              // buckets holding more than four distinct keys
    alignas(128) uint64_t buckets_done;  // of those, buckets whose first four keys are known
    alignas(128) uint64_t found;
    alignas(128) uint32_t chunk_ctr;
    alignas(128) uint32_t guard_done;
    uint64_t spill;
    // key-value variant: payload placement by rank digits (count paths)
    uint32_t kv_on;
    uint32_t kv_passes;               // 8-bit digits of the largest rank (0 when K = 1)
    uint32_t kv_slots_log2;           // rank lookup table size
    uint32_t kv_mode;                 // lookup: 0 table in LDS, 1 table in memory, 2 binary search
};

// Everything a kernel needs to know about the call; passed by value.
struct Args {
    const uint64_t* in;
    uint64_t* out;
    uint64_t n;
    uint64_t flip;                    // 1<<63 for int64 and float64, 1<<31 for int32, 0 for unsigned
    uint64_t fneg;                    // all ones for float64, 0 otherwise (see okey)
    uint32_t ew;                      // element bytes of the column: 8, or 4 for 32-bit keys
    uint32_t cap;                     // keys per bucket of the paper's table (4, or 8 for 32-bit keys)
    void* uniq_out;                   // 32-bit keys: the caller's distinct-key array (uniq is internal)
    uint32_t in_head;                 // 1 if in is 8- but not 16-byte aligned
    uint32_t out_head;
    uint32_t want_report;
    uint32_t want_counts;
    cafs_report_t* report;
    Ctrl* c;
    // dense arrays (capacity n): user arrays when given, else workspace
    uint64_t* uniq;
    uint64_t* cnt;
    uint64_t* off;                    // n + 1 entries
    // GPU hash table
    uint64_t* gkeys;
    uint64_t* gcnt;
    uint32_t* claimed;
    uint32_t cap_ws_log2;             // largest table the workspace holds
    // radix scratch (n keys; the pair sort uses the dead hash table instead); during
    // the hash count it holds the deferred elements, one region per workgroup
    uint64_t* tmp_k;
    uint64_t* status;                 // 2 slots of status_slot words
    uint64_t status_slot;
    // guard scratch
    uint32_t* dcount;                 // m_ws entries
    uint32_t* bmin;                   // 4 * m_ws entries
    uint32_t* first_idx;              // n entries
    uint32_t* clist;                  // n entries: indices of contested keys
    uint32_t* bfound;                 // m_ws entries: contested keys seen per bucket
    uint64_t m_ws;
    uint32_t rank_blocks;             // workgroups of this column's ranking kernel
    uint32_t rank_budget_log2;        // compares per ranking workgroup allowed
    uint32_t row_blocks;              // workgroups of the row emit's sweep
    uint64_t table_mul;               // odd multiplier of the count tables' hash (kPhi unless seeded)
    // count geometry (tunable): distinct keys per hash partition the estimate aims
    // at, and the estimate per partition from which LDS buckets hold 4 keys
    uint64_t part_keys;
    uint64_t wide_min;
    uint64_t table_slots;             // global table slots per estimated key (rounded up to a power of two)
    // run-length scratch
    uint64_t* rle_tile;               // per-tile run counts
    uint64_t* psum;                   // 2 * kMaxCountBlocks: head counts and count sums of the fold's chunks
    // spill list: (key, count) pairs, n entries each
    uint64_t* spill_k;
    uint64_t* spill_v;
    // the column scattered into hash-partition buckets (pbuf_elems entries in all)
    uint64_t* pbuf;
    uint64_t pbuf_elems;
    // key-value variant: one 64-bit payload per key (null for a keys-only sort)
    const uint64_t* vin;
    uint64_t* vout;
    uint32_t kv_tab_log2;             // largest rank lookup table the workspace holds (16-byte slots)
};

// Block table of a batched launch: block b works on column col[b] as block
// b - first[col[b]] of count[col[b]] blocks given to that column.
// The radix jobs of a batch (built on the device once the histograms have planned
// them): for each kind (0 keys-only, 1 key-value) the columns and the first item of
// each (an item is a tile of kRadixTile keys), and one item counter per pass.  The
// arrays follow the struct: cols[kind][cap], then start[kind][cap + 1].
struct RadixList {
    uint32_t total[2];
    uint32_t ncols[2];
    uint32_t cap;
    uint32_t pad[3];
    uint32_t next[2][8];
};
constexpr uint32_t kNoCol = 0xFFFFFFFFu;
__host__ __device__ inline size_t radix_list_bytes(uint32_t cap) {
    return sizeof(RadixList) + 4ull * (2ull * cap + 2ull * (cap + 1ull));
}
__device__ __forceinline__ uint32_t* radix_list_cols(RadixList* R, uint32_t kind) {
    return reinterpret_cast<uint32_t*>(R + 1) + (size_t)kind * R->cap;
}
__device__ __forceinline__ const uint32_t* radix_list_cols(const RadixList* R, uint32_t kind) {
    return reinterpret_cast<const uint32_t*>(R + 1) + (size_t)kind * R->cap;
}
__device__ __forceinline__ uint32_t* radix_list_start(RadixList* R, uint32_t kind) {
    return reinterpret_cast<uint32_t*>(R + 1) + 2ull * R->cap + (size_t)kind * (R->cap + 1ull);
}
__device__ __forceinline__ const uint32_t* radix_list_start(const RadixList* R, uint32_t kind) {
    return reinterpret_cast<const uint32_t*>(R + 1) + 2ull * R->cap + (size_t)kind * (R->cap + 1ull);
}

struct BatchGrid {
    const Args* args;
    const uint32_t* col;
    const uint32_t* first;
    const uint32_t* count;
};

// Every kernel body is a device function of (call arguments, block id, block
// count); this emits the single-column kernel k_NAME over the launch grid and
// the batched kernel kb_NAME over a block table.
#define CAFS_KERNELS0(NAME, T)                                                         \
    __global__ __launch_bounds__(T) void k_##NAME(Args a) { NAME##_body(a, blockIdx.x, gridDim.x); } \
    __global__ __launch_bounds__(T) void kb_##NAME(BatchGrid g) {                     \
        const uint32_t col = g.col[blockIdx.x];                                        \
        NAME##_body(g.args[col], blockIdx.x - g.first[col], g.count[col]);             \
    }
#define CAFS_KERNELS1(NAME, T, XT, XN)                                                 \
    __global__ __launch_bounds__(T) void k_##NAME(Args a, XT XN) {                     \
        NAME##_body(a, XN, blockIdx.x, gridDim.x);                                     \
    }                                                                                  \
    __global__ __launch_bounds__(T) void kb_##NAME(BatchGrid g, XT XN) {              \
        const uint32_t col = g.col[blockIdx.x];                                        \
        NAME##_body(g.args[col], XN, blockIdx.x - g.first[col], g.count[col]);         \
    }

// ---- helpers ---------------------------------------------------------------

// Pointers reach the kernels inside structs, so the compiler sees them as generic
// (flat) pointers.  Flat accesses also count against the LDS wait counter, which
// makes every LDS wait in a loop wait for the loads in flight too; the hot loops
// access memory through these global-address-space views instead.
#define CAFS_GLOBAL __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ CAFS_GLOBAL T* gp(T* p) { return (CAFS_GLOBAL T*)p; }
template <class T>
__device__ __forceinline__ T g_add(T* p, T v) {
    return __hip_atomic_fetch_add(gp(p), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Returns the value found (== expected when the exchange happened).
template <class T>
__device__ __forceinline__ T g_cas(T* p, T expected, T desired) {
    __hip_atomic_compare_exchange_strong(gp(p), &expected, desired, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT);
    return expected;
}
template <class T>
__device__ __forceinline__ T g_load(const T* p) {
    return __hip_atomic_load(gp(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Element i of a column of `ew`-byte keys, as the 64-bit value the kernels work on
// (a 32-bit key zero-extended), and the converse store.
__device__ __forceinline__ uint64_t load_key(const uint64_t* p, uint64_t i, uint32_t ew) {
    return ew == 4 ? (uint64_t)gp(reinterpret_cast<const uint32_t*>(p))[i] : gp(p)[i];
}
__device__ __forceinline__ void store_key(uint64_t* p, uint64_t i, uint64_t v, uint32_t ew) {
    if (ew == 4) gp(reinterpret_cast<uint32_t*>(p))[i] = (uint32_t)v;
    else gp(p)[i] = v;
}

// Order key: the unsigned integer whose order is the column's order.  int64: bit 63
// flipped; int32 (zero-extended): bit 31 flipped; uint64 and uint32: the bits
// themselves; float64 in IEEE 754 totalOrder (-NaN <
// -inf < ... < -0 < +0 < ... < +inf < +NaN): bit 63 flipped for a clear sign bit,
// every bit flipped for a set one.  Equality stays on the raw bits.
__device__ __forceinline__ uint64_t okey(uint64_t x, uint64_t flip, uint64_t fneg) {
    return x ^ (flip | (fneg & (uint64_t)((int64_t)x >> 63)));
}
// Inverse of okey (a float64 key with bit 63 set came from a clear sign bit).
__device__ __forceinline__ uint64_t okey_inv(uint64_t k, uint64_t flip, uint64_t fneg) {
    return k ^ (flip | (fneg & ~(uint64_t)((int64_t)k >> 63)));
}

// Multiplicative hash of Eq. hash: top `bits` bits of x * phi mod 2^64.
__device__ __forceinline__ uint32_t phi_hash(uint64_t x, uint32_t bits) {
    return (uint32_t)((x * kPhi) >> (64 - bits));
}

// Multiply-shift with another odd multiplier `mul` (the count tables' hash; kPhi
// gives Eq. hash), in full and on 32-bit halves for bits <= 32.
__device__ __forceinline__ uint32_t mul_hash(uint64_t x, uint32_t bits, uint64_t mul) {
    return (uint32_t)((x * mul) >> (64 - bits));
}
__device__ __forceinline__ uint32_t mul_hash32(uint64_t x, uint32_t bits, uint64_t mul) {
    const uint32_t lo = (uint32_t)x, hi = (uint32_t)(x >> 32);
    const uint32_t mlo = (uint32_t)mul, mhi = (uint32_t)(mul >> 32);
    const uint32_t top = __umulhi(lo, mlo) + lo * mhi + hi * mlo;
    return top >> (32 - bits);
}

// The same hash on 32-bit halves, for bits <= 32: only the high word of the
// low 64 bits of the product is needed, which takes three 32-bit multiplies.
__device__ __forceinline__ uint32_t phi_hash32(uint64_t x, uint32_t bits) {
    const uint32_t lo = (uint32_t)x, hi = (uint32_t)(x >> 32);
    const uint32_t plo = (uint32_t)kPhi, phi = (uint32_t)(kPhi >> 32);
    const uint32_t top = __umulhi(lo, plo) + lo * phi + hi * plo;
    return top >> (32 - bits);
}

__device__ __forceinline__ uint64_t bit_ceil64(uint64_t v) {
    if (v <= 1) return 1;
    return 1ull << (64 - __clzll(v - 1));
}

__device__ __forceinline__ uint32_t log2_pow2(uint64_t p) { return 63 - __clzll(p); }

template <class T>
__device__ __forceinline__ T atomic_load_agent(const T* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T>
__device__ __forceinline__ void atomic_store_agent(T* p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// Sum over the wave (64 lanes).
__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Exclusive prefix sum over a workgroup of `nthreads` (multiple of 64) threads.
// `scratch` holds one entry per wave.  Returns the exclusive prefix; *total gets
// the sum over the workgroup.  Must be called by every thread.
template <typename T>
__device__ __forceinline__ T block_exclusive_scan(T v, T* scratch, T* total) {
    const int lane = __lane_id();
    const int wave = threadIdx.x >> 6;
    const int nwaves = (blockDim.x + 63) >> 6;
    T incl = v;
    for (int o = 1; o < 64; o <<= 1) {
        T t = __shfl_up(incl, o, 64);
        if (lane >= o) incl += t;
    }
    if (lane == 63) scratch[wave] = incl;
    __syncthreads();
    if (threadIdx.x == 0) {
        T run = 0;
        for (int w = 0; w < nwaves; ++w) {
            T t = scratch[w];
            scratch[w] = run;
            run += t;
        }
        scratch[nwaves] = run;
    }
    __syncthreads();
    T res = scratch[wave] + incl - v;
    *total = scratch[nwaves];
    __syncthreads();
    return res;
}

}  // namespace cafs
