// Count stage: tiny count, hash count, compaction and order of the distinct keys.
#pragma once
#include "cafs_dev.h"

namespace cafs {

typedef unsigned long long u64x2 __attribute__((ext_vector_type(2)));

// The column is walked in 16-byte "pairs".  When the base pointer is 8- but not
// 16-byte aligned (head = 1), pair 0 holds only element 0 and pair p >= 1 holds
// elements 2p-1 and 2p, which start on a 16-byte boundary.
__device__ __forceinline__ uint64_t num_pairs(uint64_t n, uint32_t head) { return (n + head + 1) / 2; }

__device__ __forceinline__ void load_pair(const uint64_t* __restrict__ x, uint64_t n, uint32_t head,
                                          uint64_t p, uint64_t& v0, uint64_t& v1, bool& ok0, bool& ok1) {
    const int64_t e0 = (int64_t)(2 * p) - (int64_t)head;
    ok0 = e0 >= 0 && (uint64_t)e0 < n;
    ok1 = (uint64_t)(e0 + 1) < n;
    if (ok0 && ok1) {
        const u64x2 w = *reinterpret_cast<const u64x2*>(x + e0);
        v0 = w.x;
        v1 = w.y;
    } else {
        v0 = ok0 ? x[e0] : 0;
        v1 = ok1 ? x[e0 + 1] : 0;
    }
}

// ---------------------------------------------------------------------------
// Phase 2: initialise the global table (tiny and hash engines) and run the
// tiny count (Sec. 4.4): one counter per sampled key, every element compared
// with every key, branch-free.  Each lane keeps its own eight counters in
// registers (a compare and an add per key and element) and the wave sums them
// once at the end, so the loop costs two vector instructions per key and element
// and nothing waits on a cross-lane result.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void phase2_body(const Args& a, uint32_t bid, uint32_t nblk) {
    Ctrl* c = a.c;
    const uint32_t engine = c->engine;
    if (engine != E_TINY && engine != E_HASH) return;
    const uint64_t gtid = (uint64_t)bid * blockDim.x + threadIdx.x;
    const uint64_t gstride = (uint64_t)nblk * blockDim.x;
    const uint64_t cap = 1ull << c->cap_log2;
    for (uint64_t i = gtid; i < cap; i += gstride) {
        a.gkeys[i] = kEmpty;
        a.gcnt[i] = 0;
    }
    if (engine != E_TINY) return;
    const uint32_t nk = c->n_tiny;
    uint64_t key[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) key[j] = c->tiny_keys[j];
    // absent keys compare against a key no element can match below: the slot of a
    // missing key gets key[0] again and its counter is dropped
#pragma unroll
    for (int j = 1; j < 8; ++j) key[j] = j < (int)nk ? key[j] : key[0];
    uint32_t cnt[8] = {0, 0, 0, 0, 0, 0, 0, 0};  // per lane: a lane sees < 2^32 elements
    const uint32_t lane = __lane_id();
    if (a.ew == 4) {
        // 32-bit keys: each wave reads 64 * 16 consecutive keys per batch, one 4-byte
        // load per lane and key (coalesced), the next batch's loads in flight
        constexpr int UE = 16;
        const CAFS_GLOBAL uint32_t* in32 = gp(reinterpret_cast<const uint32_t*>(a.in));
        const uint64_t n = a.n;
        const uint64_t step = gstride / 64 * 64 * UE;
        uint64_t eb = gtid / 64 * 64 * UE;
        uint32_t v32[UE];
        auto load32 = [&](uint64_t b) {
#pragma unroll
            for (int u = 0; u < UE; ++u) {
                const uint64_t e = b + (uint64_t)u * 64 + lane;
                v32[u] = e < n ? in32[e] : 0u;
            }
        };
        if (eb < n) load32(eb);
        while (eb < n) {
            uint32_t x32[UE];
#pragma unroll
            for (int u = 0; u < UE; ++u) x32[u] = v32[u];
            const uint64_t cur = eb;
            eb += step;
            if (eb < n) load32(eb);
#pragma unroll
            for (int u = 0; u < UE; ++u) {
                const bool ok = cur + (uint64_t)u * 64 + lane < n;
#pragma unroll
                for (int j = 0; j < 8; ++j) cnt[j] += (ok && (uint64_t)x32[u] == key[j]) ? 1u : 0u;
            }
        }
    } else {
    const uint32_t head = a.in_head;
    const uint64_t P = num_pairs(a.n, head);
    const uint64_t Pf = (a.n + head) / 2;
    constexpr int U = 4;  // pairs per lane per batch; the next batch's loads are in flight while one is counted
    const uint64_t waves_total = gstride / 64;
    const uint64_t wave_id = gtid / 64;
    const uint64_t step = waves_total * 64 * U;
    const CAFS_GLOBAL uint64_t* in = gp(a.in);
    uint64_t v[2 * U];
    uint32_t okm = 0;
    auto load = [&](uint64_t pb) {
        if (pb >= head && pb + 64 * U <= Pf) {
            const CAFS_GLOBAL u64x2* src = reinterpret_cast<const CAFS_GLOBAL u64x2*>(in + 2 * (pb + lane) - head);
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const u64x2 w = src[u * 64];
                v[2 * u] = w.x;
                v[2 * u + 1] = w.y;
            }
            okm = (1u << (2 * U)) - 1;
        } else {
            okm = 0;
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const uint64_t p = pb + (uint64_t)u * 64 + lane;
                bool o0 = false, o1 = false;
                v[2 * u] = v[2 * u + 1] = 0;
                if (p < P) load_pair(a.in, a.n, head, p, v[2 * u], v[2 * u + 1], o0, o1);
                okm |= (o0 ? 1u : 0u) << (2 * u);
                okm |= (o1 ? 1u : 0u) << (2 * u + 1);
            }
        }
    };
    uint64_t pb = wave_id * 64 * U;
    if (pb < P) load(pb);
    while (pb < P) {
        uint64_t x[2 * U];
#pragma unroll
        for (int e = 0; e < 2 * U; ++e) x[e] = v[e];
        const uint32_t m = okm;
        pb += step;
        if (pb < P) load(pb);
        if (m == (1u << (2 * U)) - 1) {
#pragma unroll
            for (int e = 0; e < 2 * U; ++e)
#pragma unroll
                for (int j = 0; j < 8; ++j) cnt[j] += x[e] == key[j] ? 1u : 0u;
        } else {
#pragma unroll
            for (int e = 0; e < 2 * U; ++e)
#pragma unroll
                for (int j = 0; j < 8; ++j) cnt[j] += (((m >> e) & 1u) && x[e] == key[j]) ? 1u : 0u;
        }
    }
    }
    // one device-scope update per key and workgroup (per wave, thousands of them
    // queued on the same lines)
    __shared__ uint32_t s_cnt[8];
    if (threadIdx.x < 8) s_cnt[threadIdx.x] = 0;
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const uint32_t w = wave_sum_u32(cnt[j]);
        if (lane == 0 && j < (int)nk && w) atomicAdd(&s_cnt[j], w);
    }
    __syncthreads();
    if (threadIdx.x < nk && s_cnt[threadIdx.x])
        atomicAdd((unsigned long long*)&c->tiny_cnt[threadIdx.x][0], (unsigned long long)s_cnt[threadIdx.x]);
}
CAFS_KERNELS0(phase2, 256)

// Switch to the radix engine (the spill grew past its limit, Sec. 4.5's guard aside:
// sorting the spilled pairs would cost more than sorting the column).  In place, the
// radix engine then sorts into scratch so that the guard can still read the input.
__device__ __noinline__ void set_overflow(Ctrl* c, uint32_t inplace, uint64_t* tmp_k, uint64_t* uniq) {
    if (atomicExch(&c->overflow, 1u) == 0) {
        if (inplace) {
            c->rj.dst_k = tmp_k;
            c->rj.dst_ew = 8;
            c->rj.tmp_k = uniq;
            c->sorted = tmp_k;
            c->sorted_ew = 8;
            c->deferred_copy = 1;
        }
        atomicExch(&c->radix_on, 1u);
        atomicExch(&c->guard_on, 1u);
        atomicExch(&c->guard_general, 1u);
        atomicOr(&c->flags, kFlagOverflow);
    }
}

// The global (key, count) table of one column, and its spill list.
struct GTable {
    Ctrl* c;
    uint64_t* keys;
    unsigned long long* cnt;
    uint32_t* claimed;
    uint64_t* tmp_k;
    uint64_t* uniq;
    uint64_t* spill_k;
    uint64_t* spill_v;
    uint64_t spill_cap;  // entries of the spill list (n)
    uint32_t inplace;
    uint64_t mul;  // the count tables' hash multiplier
};

__device__ __forceinline__ GTable gtable(const Args& a) {
    GTable t;
    t.c = a.c;
    t.keys = a.gkeys;
    t.cnt = reinterpret_cast<unsigned long long*>(a.gcnt);
    t.claimed = a.claimed;
    t.tmp_k = a.tmp_k;
    t.uniq = a.uniq;
    t.spill_k = a.spill_k;
    t.spill_v = a.spill_v;
    t.spill_cap = a.n;
    t.inplace = a.in == a.out;
    t.mul = a.table_mul;
    return t;
}

// Insert (v, cnt) into the global open-addressing table (linear probing from the
// multiply-shift slot).  A slot is claimed by CAS from kEmpty and never freed.  New
// keys are placed only while `may_claim` (the table is below its load limit, read
// by the wave beforehand, so the limit is approximate); after that the table is
// closed: a lookup stops after kClosedProbe slots, otherwise after kGlobalProbe,
// and a key not found by then goes to the spill list with its count.  A key may
// then be counted in the table and on the list, which the fold of the order stage
// sums.
// Returns the slot claimed for a new key, kNoSlot when the count was added to a
// key already there, kFail when the caller must spill (v, cnt).  The caller lists
// claimed slots with list_claims, so that compaction reads K entries, not the table.
constexpr uint32_t kNoSlot = 0xFFFFFFFFu;
constexpr uint32_t kFail = 0xFFFFFFFEu;

// The overflow flag, read by one lane and broadcast: an agent-scope load misses the
// XCD's L2 and goes to memory, and every lane of the GPU reading the same word
// queues on one line.  Called with every lane of the wave active.
__device__ __forceinline__ uint32_t wave_overflow(const Ctrl* c) {
    uint32_t ov = 0;
    if (__lane_id() == 0) ov = g_load(&c->overflow);
    return __builtin_amdgcn_readfirstlane(ov);
}

// Whether the wave may still place new keys in the global table (one lane reads the
// closed flag, which list_claims raises once the claimed count passes the load
// limit; the count's own line is under constant atomic traffic, and a read of it
// waits behind that).  Called with every lane of the wave active.
__device__ __forceinline__ bool wave_may_claim(const Ctrl* c) {
    uint32_t cl = 0;
    if (__lane_id() == 0) cl = g_load(&c->closed);
    return __builtin_amdgcn_readfirstlane(cl) == 0;
}

__device__ __forceinline__ uint32_t global_insert(const GTable& t, uint64_t v, uint64_t cnt, bool may_claim) {
    Ctrl* c = t.c;
    const uint32_t lg = c->cap_log2;
    const uint64_t mask = (1ull << lg) - 1;
    uint64_t h = mul_hash(v, lg, t.mul);
    const uint32_t limit = may_claim ? kGlobalProbe : kClosedProbe;
    for (uint32_t pr = 0; pr < limit; ++pr) {
        if (pr % kGlobalProbeCheck == kGlobalProbeCheck - 1 && g_load(&c->overflow)) return kNoSlot;
        uint64_t k = g_load(&t.keys[h]);
        if (k == kEmpty) {
            if (!may_claim) return kFail;  // v is not in the table (slots fill in probe order)
            k = g_cas(&t.keys[h], kEmpty, v);
            if (k == kEmpty) {
                g_add(&t.cnt[h], (unsigned long long)cnt);
                return (uint32_t)h;
            }
        }
        if (k == v) {
            g_add(&t.cnt[h], (unsigned long long)cnt);
            return kNoSlot;
        }
        h = (h + 1) & mask;
    }
    return kFail;
}

// Lists the slots the lanes of a wave claimed (kNoSlot or kFail: none) in the
// claimed-slot list, with one update of the shared counter per wave (one per claim
// would serialise on its address).  The list has room for every slot of the table.
// Called by every lane of the wave.
__device__ __forceinline__ void list_claims(const GTable& t, uint32_t h) {
    const bool mine = h < kFail;
    const uint64_t m = __ballot(mine);
    if (m == 0) return;
    const uint32_t leader = (uint32_t)__builtin_ctzll(m);
    uint32_t base = 0;
    if (__lane_id() == leader) {
        const uint32_t k = (uint32_t)__popcll(m);
        base = g_add(&t.c->claimed, k);
        const uint32_t lim = t.c->cap_limit;
        if (base < lim && base + k >= lim) __hip_atomic_store(gp(&t.c->closed), 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    base = __shfl(base, leader, 64);
    if (!mine) return;
    const uint32_t idx =
        base + __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
    if (idx < (1u << t.c->cap_log2)) gp(t.claimed)[idx] = h;
}

// Appends (key, cnt) of the lanes with `mine` to the spill list (Alg. 4's spill),
// one update of the shared counter per wave.  Each pair stands for elements no
// other pair holds, so the list never needs more than n entries.  When the list
// grows past its limit the radix engine takes the column over.  Called by every
// lane of the wave.
__device__ __forceinline__ void spill_pairs(const GTable& t, bool mine, uint64_t key, uint64_t cnt) {
    const uint64_t m = __ballot(mine);
    if (m == 0) return;
    Ctrl* c = t.c;
    const uint32_t leader = (uint32_t)__builtin_ctzll(m);
    uint64_t base = 0;
    if (__lane_id() == leader) {
        const uint64_t nm = (uint64_t)__popcll(m);
        base = g_add(&c->nspill, nm);
        if (base == 0) atomicOr(&c->flags, kFlagSpill);
        if (base + nm > c->spill_limit) set_overflow(c, t.inplace, t.tmp_k, t.uniq);
    }
    base = __shfl(base, leader, 64);
    if (!mine) return;
    const uint64_t idx =
        base + __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
    if (idx < t.spill_cap) {
        gp(t.spill_k)[idx] = key;
        gp(t.spill_v)[idx] = cnt;
    }
}

// spill_pairs for F pairs per lane at once (bit u of `mine` selects pair u): one
// update of the shared counter for all of them.  Called by every lane of the wave.
template <int F>
__device__ __forceinline__ void spill_pairs_n(const GTable& t, uint32_t mine, const uint64_t (&key)[F],
                                              const uint64_t (&cnt)[F]) {
    uint64_t bal[F];
    uint32_t tot = 0;
#pragma unroll
    for (int u = 0; u < F; ++u) {
        bal[u] = __ballot((mine >> u) & 1u);
        tot += (uint32_t)__popcll(bal[u]);
    }
    if (tot == 0) return;
    Ctrl* c = t.c;
    uint64_t base = 0;
    if (__lane_id() == 0) {
        base = g_add(&c->nspill, (uint64_t)tot);
        if (base == 0) atomicOr(&c->flags, kFlagSpill);
        if (base + tot > c->spill_limit) set_overflow(c, t.inplace, t.tmp_k, t.uniq);
    }
    uint64_t run = __shfl(base, 0, 64);
#pragma unroll
    for (int u = 0; u < F; ++u) {
        const uint64_t idx = run + __builtin_amdgcn_mbcnt_hi((uint32_t)(bal[u] >> 32),
                                                             __builtin_amdgcn_mbcnt_lo((uint32_t)bal[u], 0u));
        if (((mine >> u) & 1u) && idx < t.spill_cap) {
            gp(t.spill_k)[idx] = key[u];
            gp(t.spill_v)[idx] = cnt[u];
        }
        run += (uint64_t)__popcll(bal[u]);
    }
}

// Global insert of element u of each lane where bit u of `mine` is set (count
// add[u] when `use_add`, else 1), spilling what finds no room.  Once the table is
// closed these go to the spill list without probing it (the elements that reach
// here are the rare keys, which the closed table mostly lacks).  Called by every
// lane of the wave.
template <int F>
__device__ __forceinline__ void insert_or_spill_n(const GTable& t, uint32_t mine, const uint64_t (&key)[F],
                                                  const uint32_t (&add)[F], bool use_add) {
    const bool may = wave_may_claim(t.c);
    uint64_t cnt[F];
    uint32_t spill = 0;
#pragma unroll
    for (int u = 0; u < F; ++u) {
        cnt[u] = use_add ? add[u] : 1u;
        const bool m = (mine >> u) & 1u;
        uint32_t h = kNoSlot;
        if (m) h = may ? global_insert(t, key[u], cnt[u], true) : kFail;
        list_claims(t, h);
        spill |= (h == kFail) ? (1u << u) : 0u;
    }
    spill_pairs_n<F>(t, spill, key, cnt);
}

// ---------------------------------------------------------------------------
// Hash count (main path, Sec. 4.4).  The paper's hot loop updates a bucket of four
// 64-bit keys on one cache line (Sec. 4.2, Alg. 1).  Here each workgroup owns a
// table of kLdsSlots keys with 32-bit counters in LDS, cut into buckets of W keys:
// W = 4 (3392 buckets, like the paper's) when the estimate per partition is
// large, W = 2 (6784 buckets) below the geometry's threshold, where a bucket
// rarely overflows and a lookup then takes one 16-byte LDS load instead of two
// (LDS load instructions are what the loop pays for).  An element hashes to a
// bucket (multiply-shift, reduced to the bucket count by a multiply), reads its W
// keys with 16-byte LDS loads and compares them with the element, the GPU analogue
// of the paper's cmpeq + movemask + tzcnt; on a match it adds to that slot's
// counter with an LDS atomic.  Within a bucket occupied slots form a prefix and a
// key is stored in the first bucket, in probe order, that had room for it, so a
// lookup can stop at the first bucket with a free slot.  Lookups cover the home
// bucket and, when that one is full, the next one (the window), as straight-line
// code for the eight keys a thread holds while the loads of its next eight keys
// are in flight.  A key absent from a window with room is inserted by a 64-bit
// LDS CAS on the first free slot.
//
// Hash partitions.  One LDS table holds about 10^4 keys, so for a larger estimate
// the column is first scattered into P = 2^p buckets by the top p bits of each
// element's 32-bit hash (part_scatter), and each workgroup counts a range of one
// bucket, whose keys are a P-th of the column's: the bits below the partition bits
// pick the LDS bucket.  (Masking the other partitions' elements inside one pass
// instead costs the LDS instructions of every element in every workgroup.)
//
// Beyond the table (Alg. 4's spill).  An element whose window is full is deferred:
// the wave appends it to its workgroup's region of a scratch array (bounded), and a
// second pass counts the deferred elements with a fresh table.  What finds no room
// there either, or no room in the region, goes to the global table directly.  At
// the end each workgroup flushes its occupied slots to the global table.  The global
// table takes new keys up to its load limit; a key that finds no room there goes,
// with its count, to the spill list of (key, count) pairs, which the order stage
// sorts and folds with the table's pairs.  Only a spill past N / kSpillFracDiv
// hands the column to the radix engine (overflow).  Elements equal to the empty
// marker are counted in registers.
//
// The first pass also resolves the tiny branch: if the tiny counters sum to N the
// column is tiny and the dense arrays are written here; otherwise the element set
// has an unsampled value and the main path runs with the same estimate (Sec. 4.4).
// ---------------------------------------------------------------------------
template <uint32_t W>
struct LdsGeo {
    static constexpr uint32_t kBuckets = kLdsSlots / W;
    static_assert(kBuckets * W == kLdsSlots, "whole buckets");
};

// Bucket of a key from the bits of its 32-bit hash below the partition bits
// (`hb` = hash << partition bits).
template <uint32_t W>
__device__ __forceinline__ uint32_t lds_bucket(uint32_t hb) {
    return (uint32_t)(((uint64_t)hb * LdsGeo<W>::kBuckets) >> 32);
}

template <uint32_t W>
__device__ __forceinline__ uint32_t next_bucket(uint32_t b) {
    return (b + 1 == LdsGeo<W>::kBuckets) ? 0 : b + 1;
}

// Find or claim a slot for x within `window` buckets from its home bucket and add
// `add` to its counter.  Returns false when those buckets are full without x.
template <uint32_t W>
__device__ __forceinline__ bool lds_insert(uint64_t* skeys, uint32_t* scnt, uint64_t x, uint32_t hb, uint32_t add,
                                           uint32_t window) {
    uint32_t b = lds_bucket<W>(hb);
    for (uint32_t pr = 0; pr < window; ++pr) {
        const uint32_t base = b * W;
        for (uint32_t s = 0; s < W; ++s) {
            uint64_t k = __hip_atomic_load(&skeys[base + s], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            if (k == kEmpty) {
                k = atomicCAS((unsigned long long*)&skeys[base + s], (unsigned long long)kEmpty,
                              (unsigned long long)x);
                if (k == kEmpty) k = x;  // claimed; otherwise k is the key that took the slot
            }
            if (k == x) {
                atomicAdd(&scnt[s * LdsGeo<W>::kBuckets + b], add);
                return true;
            }
        }
        b = next_bucket<W>(b);
    }
    return false;
}

// Slot of x among the W keys of a bucket, or -1; `full` tells whether the last
// slot is taken (then x may sit in a later bucket).
template <uint32_t W>
__device__ __forceinline__ int match_bucket(const uint64_t* skeys, uint32_t b, uint64_t x, bool& full) {
    const u64x2 lo = *reinterpret_cast<const u64x2*>(skeys + b * W);
    if constexpr (W == 2) {
        full = lo.y != kEmpty;
        return lo.x == x ? 0 : lo.y == x ? 1 : -1;
    } else {
        static_assert(W == 4, "buckets of 2 or 4 keys");
        const u64x2 hi = *reinterpret_cast<const u64x2*>(skeys + b * W + 2);
        full = hi.y != kEmpty;
        return lo.x == x ? 0 : lo.y == x ? 1 : hi.x == x ? 2 : hi.y == x ? 3 : -1;
    }
}

// Counts the elements of x selected by `want_m` in the LDS table, one after the
// other (the loads of the next batch are in flight meanwhile); returns the mask of
// those whose window was full (not counted).  The top `pl` bits of a key's 32-bit
// multiply-shift hash name its partition (the same for every key of the range),
// the bits below them its LDS bucket.  (`part` is unused: the ranges hold one
// partition each.)
template <int NE, uint32_t W>
__device__ __forceinline__ uint32_t count_batch(uint64_t* __restrict__ skeys, uint32_t* __restrict__ scnt,
                                                uint32_t* __restrict__ sink, const uint64_t (&x)[NE], uint64_t mul,
                                                uint32_t pl, uint32_t part, uint32_t want_m,
                                                const uint32_t (&add)[NE]) {
    uint32_t ins = 0, dfr = 0;
#pragma unroll
    for (int e = 0; e < NE; ++e) {
        const bool want = (want_m >> e) & 1u;
        uint32_t b = lds_bucket<W>(mul_hash32(x[e], 32, mul) << pl);
        bool full;
        int m = match_bucket<W>(skeys, b, x[e], full);
        if (m < 0 && full) {  // home bucket full without x: x may be in the next one
            b = next_bucket<W>(b);
            m = match_bucket<W>(skeys, b, x[e], full);
        }
        const bool hit = want && m >= 0;
        // counters are slot-major (slot s of bucket b at s * buckets + b) so that
        // the first slots of many buckets spread over the LDS banks; lanes without a
        // hit add to their own sink word, off the counters (equal addresses in one
        // instruction serialise)
        atomicAdd(hit ? &scnt[m * LdsGeo<W>::kBuckets + b] : &sink[__lane_id()], add[e]);
        const bool miss = want && !hit;
        ins |= (miss && !full) ? (1u << e) : 0u;
        dfr |= (miss && full) ? (1u << e) : 0u;
    }
    if (ins) {
#pragma unroll
        for (int e = 0; e < NE; ++e)
            if (((ins >> e) & 1u) && !lds_insert<W>(skeys, scnt, x[e], mul_hash32(x[e], 32, mul) << pl, add[e],
                                                    kLdsWindow))
                dfr |= 1u << e;
    }
    return dfr;
}

// 64-bit value of the previous lane (lane 0: 0), by a whole-wave DPP shift (no LDS
// traffic).  Every lane of the wave must be active.
__device__ __forceinline__ uint64_t wave_shr1(uint64_t v) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)v, 0x138, 0xF, 0xF, false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(v >> 32), 0x138, 0xF, 0xF, false);
    return ((uint64_t)hi << 32) | lo;
}

// Run-length injection (the main path's RLE pass, Sec. 4.4): a run of r equal
// consecutive elements takes one table update of r instead of r updates of 1.  Pair
// u of lane i holds elements 2p and 2p+1 of pair p = (batch base) + u * blockDim +
// thread, so the 64 lanes of a wave hold 128 consecutive elements per u.  An element
// heads a run unless it equals the element before it in that slice (lane i's first
// element follows lane i-1's second, taken by a lane shift); a head gets the
// distance to the next head (or to the slice's end) as its count, the others get 0.
// Runs that cross a slice boundary are cut there.  The batch is first probed on
// its first slice: unless kRleProbePairs of its 64 pairs hold two equal elements
// (random columns rarely have any) every element counts 1 and nothing more is spent.
// Otherwise a slice takes the path when it is fully in range and at least
// kRleMinMerged of its elements merge.  Every test is wave-uniform.  Returns whether
// any slice of the batch took the path.
template <int NE>
__device__ __forceinline__ bool run_lengths(const uint64_t (&x)[NE], uint32_t want, uint32_t (&add)[NE]) {
    const uint32_t lane = __lane_id();
    bool any = false;
#pragma unroll
    for (int e = 0; e < NE; ++e) add[e] = 1u;
    if ((uint32_t)__popcll(__ballot((want & 3u) == 3u && x[0] == x[1])) < kRleProbePairs) return false;
#pragma unroll
    for (int u = 0; u < NE / 2; ++u) {
        if (__ballot(((want >> (2 * u)) & 3u) != 3u) != 0) continue;
        const uint64_t a = x[2 * u], b = x[2 * u + 1];
        const uint64_t prev = wave_shr1(b);
        const bool ha = lane == 0 || a != prev;
        const bool hb = b != a;
        const uint64_t he = __ballot(ha), ho = __ballot(hb);
        if (128u - (uint32_t)__popcll(he) - (uint32_t)__popcll(ho) < kRleMinMerged) continue;
        const uint64_t later = lane == 63 ? 0ull : (he | ho) & (~0ull << (lane + 1));
        const uint32_t j = later ? (uint32_t)__builtin_ctzll(later) : 64u;
        const uint32_t nxt = j == 64u ? 128u : 2u * j + (((he >> (j & 63u)) & 1ull) ? 0u : 1u);
        add[2 * u] = ha ? (hb ? 1u : nxt - 2u * lane) : 0u;
        add[2 * u + 1] = hb ? nxt - (2u * lane + 1u) : 0u;
        any = true;
    }
    return any;
}

// Each range of a workgroup's region of the deferred-element scratch (tmp_k) holds
// 2 ceil(pairs / nblk) elements (tmp_k has room for n + 2 + 2 * kMaxCountBlocks
// keys); deferrals past it go to the global table directly.
__device__ __forceinline__ uint64_t pairs_per_block(uint64_t P, uint32_t nblk) { return (P + nblk - 1) / nblk; }

// Stable match of equal partition numbers (pl bits) across the wave: the lanes
// (within `act`) whose partition equals this lane's.
__device__ __forceinline__ uint64_t match_part(uint32_t q, uint32_t pl, uint64_t act) {
    uint64_t peers = act;
    for (uint32_t b = 0; b < pl; ++b) {
        const bool bit = (q >> b) & 1u;
        const uint64_t m = __ballot(bit);
        peers &= bit ? m : ~m;
    }
    return peers;
}

template <uint32_t W>
__device__ __forceinline__ void flush_table(const GTable& t, const uint64_t* skeys, const uint32_t* scnt) {
    constexpr uint32_t S = kLdsSlots, B = LdsGeo<W>::kBuckets;
    // once the table has overflowed (the radix engine takes over) the flush is moot;
    // each wave looks before every group of inserts
    // four slots per thread at a time: their home slots in the global table are read
    // together, and a key already there (most are, after the first workgroups) gets
    // its count added directly; the rest take the probing insert, and what finds no
    // room in the global table goes to the spill list with its count
    // Once the table is closed (at its load limit) it takes no new keys, and a
    // small count most likely belongs to one of the rare keys that it lacks: such
    // entries go to the spill list without probing (if the key is in the table after
    // all, the fold sums both).
    const uint32_t lg = t.c->cap_log2;
    constexpr int F = 4;
    for (uint32_t i0 = threadIdx.x; i0 < S; i0 += F * blockDim.x) {  // uniform over each wave
        if (wave_overflow(t.c)) return;
        const bool may = wave_may_claim(t.c);
        uint32_t cn[F], h[F], cl[F];
        uint64_t key[F], k[F], cv[F];
        uint32_t spill = 0;
#pragma unroll
        for (int u = 0; u < F; ++u) {
            const uint32_t i = i0 + u * blockDim.x;
            cn[u] = i < S ? scnt[i] : 0u;  // slot i / B of bucket i % B; never 0 once claimed
            key[u] = cn[u] ? skeys[(i % B) * W + i / B] : 0;
            h[u] = mul_hash(key[u], lg, t.mul);
            cv[u] = cn[u];
        }
#pragma unroll
        for (int u = 0; u < F; ++u) k[u] = cn[u] ? g_load(&t.keys[h[u]]) : kEmpty;
#pragma unroll
        for (int u = 0; u < F; ++u) {
            cl[u] = kNoSlot;
            if (!cn[u]) continue;
            if (k[u] == key[u]) g_add(&t.cnt[h[u]], (unsigned long long)cn[u]);
            else if (!may && cn[u] < kSpillBelow) cl[u] = kFail;
            else cl[u] = global_insert(t, key[u], cn[u], may);
            spill |= (cl[u] == kFail) ? (1u << u) : 0u;
        }
#pragma unroll
        for (int u = 0; u < F; ++u) list_claims(t, cl[u]);  // (the loop is uniform over each wave)
        spill_pairs_n<F>(t, spill, key, cv);
    }
}

// Workgroup-uniform read of the overflow flag: thread 0 reads it into LDS between
// two barriers.  Called by every thread of the workgroup.
__device__ __forceinline__ bool block_overflow(const Ctrl* c, uint32_t* s_flag) {
    __syncthreads();
    if (threadIdx.x == 0) *s_flag = g_load(&c->overflow);
    __syncthreads();
    return *s_flag != 0;
}

// Partition scatter (before the count, when the plan has partitions): the column
// in chunks of kScatterChunk elements; each chunk's elements are ranked within their
// partition (a wave matches equal partitions by ballots and takes one LDS counter
// update per partition), staged in LDS in partition order, given a place in each
// bucket by one atomic per partition and chunk, and written out as runs of
// consecutive elements.  A bucket holds a sixteenth more than its planned share
// plus a chunk; elements past it go to the overflow area (a reservation per
// partition and chunk), and past that to the spill list.
__device__ __forceinline__ void part_scatter_body(const Args& a, uint32_t bid, uint32_t nblk) {
    Ctrl* c = a.c;
    if (c->engine != E_HASH || c->part_log2 == 0) return;
    const uint32_t pl = c->part_log2;
    const uint32_t P = 1u << pl;
    const uint64_t mul = a.table_mul;
    const GTable t = gtable(a);
    const uint64_t n = a.n;
    CAFS_GLOBAL uint64_t* pbuf = gp(a.pbuf);
    __shared__ uint64_t stage[kScatterChunk];
    __shared__ uint32_t lcnt[kMaxParts];
    __shared__ uint32_t loff[kMaxParts];
    __shared__ uint64_t gbase[kMaxParts];
    __shared__ uint64_t pb0[kMaxParts + 2];   // the bucket bounds
    __shared__ uint32_t ofirst[kMaxParts];    // first chunk-local index of a bucket that overflows
    __shared__ uint64_t obase[kMaxParts];     // its place in the overflow area
    if (threadIdx.x < P + 2) pb0[threadIdx.x] = c->pbase[threadIdx.x];
    const uint32_t tid = threadIdx.x, lane = __lane_id();
    const uint64_t lt = (1ull << lane) - 1;
    const uint64_t chunks = (n + kScatterChunk - 1) / kScatterChunk;
    constexpr int U = kScatterChunk / kScatterThreads;
    for (uint64_t ch = bid; ch < chunks; ch += nblk) {  // uniform
        if (tid < kMaxParts) lcnt[tid] = 0;
        __syncthreads();
        const uint64_t base = ch * kScatterChunk;
        uint64_t x[U];
        uint32_t q[U], r[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint64_t i = base + (uint64_t)u * kScatterThreads + tid;
            x[u] = i < n ? load_key(a.in, i, a.ew) : 0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const bool ok = base + (uint64_t)u * kScatterThreads + tid < n;
            q[u] = mul_hash32(x[u], 32, mul) >> (32 - pl);
            const uint64_t peers = match_part(q[u], pl, __ballot(ok));
            const uint32_t leader = peers ? (uint32_t)__builtin_ctzll(peers) : 0u;
            uint32_t rb = 0;
            if (ok && lane == leader) rb = atomicAdd(&lcnt[q[u]], (uint32_t)__popcll(peers));
            rb = __shfl(rb, (int)leader, 64);
            r[u] = rb + (uint32_t)__popcll(peers & lt);
        }
        __syncthreads();
        if (tid == 0) {
            uint32_t run = 0;
            for (uint32_t qq = 0; qq < (1u << pl); ++qq) {
                loff[qq] = run;
                run += lcnt[qq];
            }
        }
        if (tid < P) {
            const uint32_t lc = lcnt[tid];
            const uint64_t g = lc ? atomicAdd(&c->pfill[tid][0], lc) : 0u;
            const uint64_t cap = pb0[tid + 1] - pb0[tid];
            gbase[tid] = g;
            // elements past the bucket's capacity go to the overflow area
            const uint64_t fit = g >= cap ? 0 : (cap - g < lc ? cap - g : lc);
            ofirst[tid] = (uint32_t)fit;
            obase[tid] = fit < lc ? atomicAdd(&c->pfill[kMaxParts][0], (uint32_t)(lc - fit)) : 0u;
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (base + (uint64_t)u * kScatterThreads + tid < n) stage[loff[q[u]] + r[u]] = x[u];
        __syncthreads();
        const uint32_t cnt = (uint32_t)(n - base < kScatterChunk ? n - base : kScatterChunk);
#pragma unroll
        for (int u = 0; u < U; ++u) {  // uniform: every lane takes part in the spill's ballot
            const uint32_t i = (uint32_t)u * kScatterThreads + tid;
            const bool ok = i < cnt;
            const uint64_t v = ok ? stage[i] : 0;
            const uint32_t qq = mul_hash32(v, 32, mul) >> (32 - pl);
            const uint32_t li = ok ? i - loff[qq] : 0u;
            const bool in_bucket = li < ofirst[qq];
            const uint64_t odst = obase[qq] + (li - ofirst[qq]);
            const bool in_over = !in_bucket && odst < pb0[P + 1] - pb0[P];
            if (ok && in_bucket) pbuf[pb0[qq] + gbase[qq] + li] = v;
            if (ok && in_over) pbuf[pb0[P] + odst] = v;
            spill_pairs(t, ok && !in_bucket && !in_over, v, 1);
        }
        __syncthreads();
    }
}
CAFS_KERNELS0(part_scatter, kScatterThreads)

template <uint32_t W, uint32_t EW>
__device__ __forceinline__ void count_range(const Args& a, const GTable& t, uint64_t* skeys, uint32_t* scnt,
                                            uint32_t& s_ndef, uint32_t* s_sink, uint32_t* s_flag,
                                            const uint64_t* src, uint64_t n, uint32_t head, uint64_t p_begin,
                                            uint64_t p_end, uint32_t pl, CAFS_GLOBAL uint64_t* region,
                                            uint32_t region_cap);

template <uint32_t W, bool PARTS, uint32_t EW>
__device__ __forceinline__ void count_items(const Args& a, uint32_t bid, uint32_t nblk, uint64_t* skeys, uint32_t* scnt,
                                            uint32_t& s_ndef, uint32_t& s_flag, uint32_t* s_sink);

// Instances chosen once at the top of the kernel: the count without partitions
// (PARTS false: the partition bits are the constant 0 in its hot loop) over a column
// of EW-byte keys, and the count over the partition buckets (which hold 64-bit
// keys).  The first also resolves the tiny branch (a tiny plan has no partitions).
template <bool PARTS, uint32_t EW>
__device__ __forceinline__ void hash_count_impl(const Args& a, uint32_t bid, uint32_t nblk, uint64_t* skeys,
                                                uint32_t* scnt, uint32_t& s_ndef, uint32_t& s_flag, uint32_t* s_sink) {
    Ctrl* c = a.c;
    const uint32_t engine = c->engine;
    if (engine == E_TINY) {
        const uint32_t nk = c->n_tiny;
        uint64_t tot = 0;
        for (uint32_t j = 0; j < nk; ++j) tot += c->tiny_cnt[j][0];
        if (tot == a.n) {
            if (bid == 0 && threadIdx.x == 0) {
                uint64_t run = 0;
                for (uint32_t j = 0; j < nk; ++j) {
                    a.uniq[j] = c->tiny_keys[j];
                    a.cnt[j] = c->tiny_cnt[j][0];
                    a.off[j] = run;
                    run += c->tiny_cnt[j][0];
                }
                a.off[nk] = run;
                c->K = nk;
                c->dense_ready = 1;
                c->emit_main = 1;
            }
            return;
        }
        if (bid == 0 && threadIdx.x == 0) {
            c->tiny_miss = 1;
            c->path = P_MAIN;
            c->engine = E_HASH;
        }
    } else if (engine != E_HASH) {
        return;
    }

    if (c->lds_wide) count_items<4, PARTS, EW>(a, bid, nblk, skeys, scnt, s_ndef, s_flag, s_sink);
    else count_items<2, PARTS, EW>(a, bid, nblk, skeys, scnt, s_ndef, s_flag, s_sink);
}

// The contents of the partition buckets and the overflow area, taken as one
// sequence (each part's length rounded up to even, so that pairs stay aligned),
// split evenly over the items in multiples of 64 elements: item `it` counts its
// share, one contiguous range of a part at a time, each range with a cleared LDS
// table and its deferrals at the same place in tmp_k as the range in pbuf.
template <uint32_t W>
__device__ __forceinline__ void count_parts(const Args& a, const GTable& t, uint64_t* skeys, uint32_t* scnt,
                                            uint32_t& s_ndef, uint32_t& s_flag, uint32_t* s_sink, uint32_t it,
                                            uint32_t items, uint32_t pl) {
    Ctrl* c = a.c;
    const uint32_t P = 1u << pl;
    // (each part's length is read again where it is needed: an array indexed by
    // the part would live in scratch memory)
    auto part_len = [&](uint32_t q) -> uint64_t {
        const uint64_t cap = c->pbase[q + 1] - c->pbase[q];
        const uint64_t fill = c->pfill[q == P ? kMaxParts : q][0];
        return fill < cap ? fill : cap;
    };
    uint64_t total = 0;
    for (uint32_t q = 0; q <= P; ++q) total += (part_len(q) + 1) & ~1ull;
    const uint64_t per = ((total + items - 1) / items + 63) & ~63ull;
    const uint64_t v0 = (uint64_t)it * per, v1 = v0 + per < total ? v0 + per : total;
    uint64_t f = 0;  // start of part q in the sequence
    for (uint32_t q = 0; q <= P && f < v1; ++q) {
        const uint64_t lq = part_len(q);
        const uint64_t lv = (lq + 1) & ~1ull;
        const uint64_t s0 = v0 > f ? v0 - f : 0, s1 = v1 - f < lv ? v1 - f : lv;
        if (s0 < s1) {
            const uint64_t base = c->pbase[q];  // a multiple of 32 elements
            CAFS_GLOBAL uint64_t* region = gp(a.tmp_k) + base + s0;
            for (uint32_t i = threadIdx.x; i < kLdsSlots; i += blockDim.x) {
                skeys[i] = kEmpty;
                scnt[i] = 0;
            }
            if (threadIdx.x == 0) s_ndef = 0;
            __syncthreads();
            count_range<W, 8>(a, t, skeys, scnt, s_ndef, s_sink, &s_flag, a.pbuf + base, lq, 0, s0 / 2, s1 / 2,
                              pl, region, (uint32_t)(s1 - s0));
            __syncthreads();
        }
        f += lv;
    }
}

// This workgroup's work items with LDS buckets of W keys.
template <uint32_t W, bool PARTS, uint32_t EW>
__device__ __forceinline__ void count_items(const Args& a, uint32_t bid, uint32_t nblk, uint64_t* skeys, uint32_t* scnt,
                                            uint32_t& s_ndef, uint32_t& s_flag, uint32_t* s_sink) {
    Ctrl* c = a.c;
    constexpr uint32_t S = kLdsSlots;
    const GTable t = gtable(a);
    const uint64_t n = a.n;
    const uint32_t pl = PARTS ? c->part_log2 : 0u;
    const uint32_t items = nblk;
    for (uint32_t it = bid; it < items; it += nblk) {  // uniform over the workgroup
        const uint64_t* src;
        uint64_t ns, pb, pe, roff;  // roff: where the item's deferral region starts in tmp_k
        uint32_t head;
        if (!PARTS && EW == 4) {
            // ranges of quads: quad q holds elements 4q - head .. 4q - head + 3 (head:
            // the column's offset in its first 16 bytes, in keys), read by one
            // 16-byte load when all four are in the column
            src = a.in;
            ns = n;
            head = (uint32_t)((reinterpret_cast<uintptr_t>(a.in) >> 2) & 3u);
            const uint64_t Q = (n + head + 3) / 4, QS = (Q + nblk - 1) / nblk;
            pb = (uint64_t)it * QS < Q ? (uint64_t)it * QS : Q;
            pe = pb + QS < Q ? pb + QS : Q;
            roff = 4 * pb;
        } else if (!PARTS) {
            src = a.in;
            ns = n;
            head = a.in_head;
            const uint64_t P = num_pairs(n, head), PS = pairs_per_block(P, nblk);
            pb = (uint64_t)it * PS < P ? (uint64_t)it * PS : P;
            pe = pb + PS < P ? pb + PS : P;
            roff = 2 * pb;
        } else {
            count_parts<W>(a, t, skeys, scnt, s_ndef, s_flag, s_sink, it, items, pl);
            continue;
        }
        // the region holds every element of the item (tmp_k covers the column and
        // every bucket), so a deferral always finds room
        CAFS_GLOBAL uint64_t* region = gp(a.tmp_k) + roff;
        const uint32_t region_cap = (uint32_t)((EW == 4 ? 4 : 2) * (pe - pb));
        for (uint32_t i = threadIdx.x; i < S; i += blockDim.x) {
            skeys[i] = kEmpty;
            scnt[i] = 0;
        }
        if (threadIdx.x == 0) s_ndef = 0;
        __syncthreads();
        count_range<W, EW>(a, t, skeys, scnt, s_ndef, s_sink, &s_flag, src, ns, head, pb, pe, pl, region, region_cap);
        __syncthreads();
    }
}

// The count over pairs [p_begin, p_end) of src[0..n) (head: src is 8- but not
// 16-byte aligned), or for EW = 4 (32-bit keys) over elements [p_begin, p_end),
// with buckets of W keys (the LDS table is cleared): the first pass with its
// deferrals, the flush, the second pass over the deferred elements and its flush.
// Called by every thread of the workgroup.
template <uint32_t W, uint32_t EW>
__device__ __forceinline__ void count_range(const Args& a, const GTable& t, uint64_t* skeys, uint32_t* scnt,
                                            uint32_t& s_ndef, uint32_t* s_sink, uint32_t* s_flag,
                                            const uint64_t* src_, uint64_t n, uint32_t head, uint64_t p_begin,
                                            uint64_t p_end, uint32_t pl, CAFS_GLOBAL uint64_t* region,
                                            uint32_t region_cap) {
    constexpr uint32_t S = kLdsSlots;
    Ctrl* c = a.c;
    const CAFS_GLOBAL uint64_t* in = gp(src_);
    const uint32_t lane = __lane_id();
    const uint64_t mul = t.mul;
    uint32_t ecnt = 0;
    // pairs [head, Pf) hold two in-range elements; for EW = 4, quads [first, Qf)
    // hold four
    const uint64_t Pf = EW == 4 ? (n + head) / 4 : (n + head) / 2;
    const uint64_t p_full = p_end < Pf ? p_end : Pf;
    const uint64_t p_first = EW == 4 ? (head ? 1u : 0u) : head;
    constexpr int U = EW == 4 ? 2 : 4;   // 16-byte groups per thread per step
    constexpr int NE = 8;
    const uint64_t span = (uint64_t)blockDim.x * U;  // groups
    uint64_t base = p_begin;
    uint64_t v[NE];
    uint32_t okm = 0;  // bit e: element e of the batch is in range
    auto load = [&](uint64_t b) {
        if constexpr (EW == 4) {
            // 32-bit keys, zero-extended: quad q = b + u * blockDim + thread
            const CAFS_GLOBAL uint32_t* in32 = reinterpret_cast<const CAFS_GLOBAL uint32_t*>(in);
            if (b >= p_first && b + span <= p_full) {
                // interior batch: every quad is four aligned in-range elements
                const CAFS_GLOBAL u64x2* src =
                    reinterpret_cast<const CAFS_GLOBAL u64x2*>(in32 + 4 * (b + threadIdx.x) - head);
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const u64x2 w = src[(uint64_t)u * blockDim.x];
                    v[4 * u] = w.x & 0xFFFFFFFFull;
                    v[4 * u + 1] = w.x >> 32;
                    v[4 * u + 2] = w.y & 0xFFFFFFFFull;
                    v[4 * u + 3] = w.y >> 32;
                }
                okm = (1u << NE) - 1;
            } else {
                okm = 0;
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const uint64_t q = b + (uint64_t)u * blockDim.x + threadIdx.x;
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const int64_t e = (int64_t)(4 * q + j) - (int64_t)head;
                        const bool o = q < p_end && e >= 0 && (uint64_t)e < n;
                        v[4 * u + j] = o ? (uint64_t)in32[e] : 0;
                        okm |= (o ? 1u : 0u) << (4 * u + j);
                    }
                }
            }
            return;
        }
        if (b >= head && b + span <= p_full) {
            // interior batch: every pair is two aligned in-range elements
            const CAFS_GLOBAL u64x2* src = reinterpret_cast<const CAFS_GLOBAL u64x2*>(in + 2 * (b + threadIdx.x) - head);
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const u64x2 w = src[(uint64_t)u * blockDim.x];
                v[2 * u] = w.x;
                v[2 * u + 1] = w.y;
            }
            okm = (1u << NE) - 1;
        } else {
            okm = 0;
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const uint64_t p = b + (uint64_t)u * blockDim.x + threadIdx.x;
                const int64_t e0 = (int64_t)(2 * p) - (int64_t)head;
                const bool o0 = p < p_end && e0 >= 0 && (uint64_t)e0 < n;
                const bool o1 = p < p_end && (uint64_t)(e0 + 1) < n;
                v[2 * u] = o0 ? in[e0] : 0;
                v[2 * u + 1] = o1 ? in[e0 + 1] : 0;
                okm |= (o0 ? 1u : 0u) << (2 * u);
                okm |= (o1 ? 1u : 0u) << (2 * u + 1);
            }
        }
    };
    if (base < p_end) load(base);
    uint32_t iter = 0;
    while (base < p_end) {  // uniform over each wave
        // every eighth batch: stop when the count has been handed to the radix engine
        // (the flag's load overlaps this batch; lane 0 loads it, the wave reads it from
        // lane 0 after the batch)
        const bool check = (++iter & 7) == 0;
        const uint32_t handed = (check && __lane_id() == 0) ? g_load(&c->overflow) : 0u;
        uint64_t x[NE];
#pragma unroll
        for (int e = 0; e < NE; ++e) x[e] = v[e];
        uint32_t want = okm;
        const uint64_t next = base + span;
        if (next < p_end) load(next);  // next batch in flight while this one is counted
#pragma unroll
        for (int e = 0; e < NE; ++e) {
            const bool is_empty_key = ((want >> e) & 1u) && x[e] == kEmpty;
            ecnt += is_empty_key ? 1u : 0u;
            want &= is_empty_key ? ~(1u << e) : ~0u;
        }
        uint32_t add[NE];
        // (run detection follows the pair layout of 64-bit keys)
        const bool rle = EW == 8 && run_lengths<NE>(x, want, add);
        if (rle) {
            // merged elements are counted by their run's head
#pragma unroll
            for (int e = 0; e < NE; ++e) want &= add[e] ? ~0u : ~(1u << e);
            const uint32_t dfr = count_batch<NE, W>(skeys, scnt, s_sink, x, mul, pl, 0u, want, add);
            // a deferred head stands for its whole run: that many copies go to the region
#pragma unroll
            for (int e = 0; e < NE; ++e) {
                if ((dfr >> e) & 1u) {
                    const uint32_t at = atomicAdd(&s_ndef, add[e]);
                    for (uint32_t r = 0; r < add[e]; ++r) region[at + r] = x[e];
                }
            }
            base = next;
            if (__builtin_amdgcn_readfirstlane(handed)) break;
            continue;
        }
        uint32_t ones[NE];
#pragma unroll
        for (int e = 0; e < NE; ++e) ones[e] = 1u;
        const uint32_t dfr = count_batch<NE, W>(skeys, scnt, s_sink, x, mul, pl, 0u, want, ones);
        if (__ballot(dfr != 0)) {
            // append the deferred elements: one LDS reservation per wave, then each
            // element's place from the ballot of its batch position
            uint64_t bal[NE];
            uint32_t tot = 0;
#pragma unroll
            for (int e = 0; e < NE; ++e) {
                bal[e] = __ballot((dfr >> e) & 1u);
                tot += (uint32_t)__popcll(bal[e]);
            }
            uint32_t at0 = 0;
            if (lane == 0) at0 = atomicAdd(&s_ndef, tot);
            uint32_t run = __shfl(at0, 0, 64);
#pragma unroll
            for (int e = 0; e < NE; ++e) {
                const uint32_t below = __builtin_amdgcn_mbcnt_hi(
                    (uint32_t)(bal[e] >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bal[e], 0u));
                if ((dfr >> e) & 1u) region[run + below] = x[e];
                run += (uint32_t)__popcll(bal[e]);
            }
        }
        base = next;
        if (__builtin_amdgcn_readfirstlane(handed)) break;  // lane 0's load (every lane is active)
    }
    const uint32_t wsum = wave_sum_u32(ecnt);
    if (lane == 0 && wsum) g_add(&c->ecount, (uint64_t)wsum);
    if (block_overflow(c, s_flag)) return;  // (uniform: every thread read the same word)
    flush_table<W>(t, skeys, scnt);
    // Second pass over the deferred elements, with the table cleared (the keys that
    // found no room are few) and a longer probe; what still finds no room goes to the
    // global table.
    if (block_overflow(c, s_flag)) return;
    const uint32_t d = s_ndef;  // uniform: read after the barrier (at most region_cap)
    if (d == 0) return;
    for (uint32_t i = threadIdx.x; i < S; i += blockDim.x) {
        skeys[i] = kEmpty;
        scnt[i] = 0;
    }
    __syncthreads();
    constexpr int D = 4;  // elements per thread per step
    for (uint32_t i0 = 0; i0 < d; i0 += D * blockDim.x) {  // uniform
        uint64_t xd[D];
        uint32_t want = 0;
#pragma unroll
        for (int u = 0; u < D; ++u) {
            const uint32_t i = i0 + u * blockDim.x + threadIdx.x;
            xd[u] = i < d ? region[i] : 0;
            want |= (i < d ? 1u : 0u) << u;
        }
        uint32_t ones[D];
#pragma unroll
        for (int u = 0; u < D; ++u) ones[u] = 1u;
        const uint32_t dfr = count_batch<D, W>(skeys, scnt, s_sink, xd, mul, pl, 0u, want, ones);
        uint32_t left = 0;
        if (dfr) {
#pragma unroll
            for (int u = 0; u < D; ++u)
                if (((dfr >> u) & 1u) &&
                    !lds_insert<W>(skeys, scnt, xd[u], mul_hash32(xd[u], 32, mul) << pl, 1u, kLdsProbeBuckets))
                    left |= 1u << u;
        }
        if (__ballot(left != 0) && !wave_overflow(c)) {
            uint32_t ones[D];
#pragma unroll
            for (int u = 0; u < D; ++u) ones[u] = 1u;
            insert_or_spill_n<D>(t, left, xd, ones, false);
        }
    }
    if (block_overflow(c, s_flag)) return;
    flush_table<W>(t, skeys, scnt);
}
// One kernel per variant (the 64-bit and 32-bit columns without partitions, chosen
// by the host from the dtype, and the partitioned count, which returns at once
// unless the plan has partitions), so that each is register-allocated alone: the
// partitioned variant needs more registers than the others and would otherwise
// make the common count loop spill.  The batched kernels take the same split, each
// launched over the whole block table; a column's workgroups leave every launch
// but the one of its variant at once.
template <bool PARTS, uint32_t EW>
__device__ __forceinline__ void hash_count_variant(const Args& a, uint32_t bid, uint32_t nblk) {
    __shared__ __attribute__((aligned(16))) uint64_t skeys[kLdsSlots];
    __shared__ uint32_t scnt[kLdsSlots];
    __shared__ uint32_t s_ndef;
    __shared__ uint32_t s_flag;
    __shared__ uint32_t s_sink[64];
    if ((a.c->part_log2 != 0) != PARTS) return;
    hash_count_impl<PARTS, EW>(a, bid, nblk, skeys, scnt, s_ndef, s_flag, s_sink);
}
__global__ __launch_bounds__(kCountThreads) void k_hash_count(Args a) {
    hash_count_variant<false, 8>(a, blockIdx.x, gridDim.x);
}
__global__ __launch_bounds__(kCountThreads) void k_hash_count32(Args a) {
    hash_count_variant<false, 4>(a, blockIdx.x, gridDim.x);
}
__global__ __launch_bounds__(kCountThreads) void k_hash_count_parts(Args a) {
    hash_count_variant<true, 8>(a, blockIdx.x, gridDim.x);
}
template <bool PARTS, uint32_t EW>
__device__ __forceinline__ void hash_count_batch(const BatchGrid& g) {
    const uint32_t col = g.col[blockIdx.x];
    const Args& a = g.args[col];
    if (!PARTS && a.ew != EW) return;
    hash_count_variant<PARTS, EW>(a, blockIdx.x - g.first[col], g.count[col]);
}
__global__ __launch_bounds__(kCountThreads) void kb_hash_count(BatchGrid g) { hash_count_batch<false, 8>(g); }
__global__ __launch_bounds__(kCountThreads) void kb_hash_count32(BatchGrid g) { hash_count_batch<false, 4>(g); }
__global__ __launch_bounds__(kCountThreads) void kb_hash_count_parts(BatchGrid g) { hash_count_batch<true, 8>(g); }

// ---------------------------------------------------------------------------
// Order of the distinct keys (Alg. 4, steps "collect non-empty bucket slots" and
// "sort pairs by key").  For K <= kRankMax each key's place is its rank, the number
// of distinct keys below it (keys are distinct, so ranks are a permutation).  Every
// workgroup ranks 64 keys, 16 threads per key, against all K keys staged through
// LDS, and writes (key, count) to its place in the dense arrays: K^2 compares spread
// over the whole GPU instead of a sorting network in one workgroup.
// ---------------------------------------------------------------------------
// Ranking costs K^2 compares over the column's ranking workgroups; beyond
// kRankMax keys, or a budget per workgroup, the pairs are radix sorted instead.
__device__ __forceinline__ bool rank_ok(const Args& a, uint32_t K) {
    return K <= kRankMax && (uint64_t)K * K <= ((uint64_t)a.rank_blocks << a.rank_budget_log2);
}

__device__ __forceinline__ uint64_t table_key(const Args& a, uint32_t idx, uint32_t claimed) {
    return idx < claimed ? gp(a.gkeys)[gp(a.claimed)[idx]] : kEmpty;
}

// Gather of the (key, count) pairs for the radix engine in pair mode (too many to rank):
// the dense arrays are sorted in place, with the dead hash table as scratch
// (K <= table size).  All workgroups of the ranking launch share the gather.
__device__ __forceinline__ void gather_pairs(const Args& a, Ctrl* c, uint32_t claimed, uint64_t ecount, uint32_t K,
                                             uint32_t bid, uint32_t nblk) {
    for (uint64_t i = (uint64_t)bid * blockDim.x + threadIdx.x; i < claimed; i += (uint64_t)nblk * blockDim.x) {
        const uint32_t h = gp(a.claimed)[i];
        gp(a.uniq)[i] = gp(a.gkeys)[h];
        gp(a.cnt)[i] = gp(a.gcnt)[h];
    }
    if (bid == 0 && threadIdx.x == 0) {
        if (ecount) { a.uniq[claimed] = kEmpty; a.cnt[claimed] = ecount; }
        RadixJob& j = c->rj;
        j.src_k = a.uniq; j.src_v = a.cnt;
        j.dst_k = a.uniq; j.dst_v = a.cnt;
        j.tmp_k = a.gkeys; j.tmp_v = a.gcnt;
        j.n = K;
        j.has_vals = 1;
        j.src_ew = 8; j.dst_ew = 8;
        c->fold_k = a.uniq;
        c->fold_v = a.cnt;
        c->pair_sort = 1;
        c->radix_on = 1;
        c->guard_on = (c->path == P_MAIN);
        c->guard_general = c->guard_on;
    }
}

// Alg. 4 with a spill: the table's pairs (and the empty marker's) are appended to the
// spill list, and the radix engine sorts all of them by key; the fold then sums equal
// neighbours (a key may sit in the table and on the list, and on the list several
// times) into the dense arrays.  The spill list has room for them: every pair holds
// elements no other pair holds.
__device__ __forceinline__ void gather_spill(const Args& a, Ctrl* c, uint32_t claimed, uint64_t ecount,
                                             uint64_t nspill, uint32_t bid, uint32_t nblk) {
    CAFS_GLOBAL uint64_t* sk = gp(a.spill_k) + nspill;
    CAFS_GLOBAL uint64_t* sv = gp(a.spill_v) + nspill;
    for (uint64_t i = (uint64_t)bid * blockDim.x + threadIdx.x; i < claimed; i += (uint64_t)nblk * blockDim.x) {
        const uint32_t h = gp(a.claimed)[i];
        sk[i] = gp(a.gkeys)[h];
        sv[i] = gp(a.gcnt)[h];
    }
    if (bid == 0 && threadIdx.x == 0) {
        if (ecount) { sk[claimed] = kEmpty; sv[claimed] = ecount; }
        RadixJob& j = c->rj;
        j.src_k = a.spill_k; j.src_v = a.spill_v;
        j.dst_k = a.spill_k; j.dst_v = a.spill_v;
        j.tmp_k = a.tmp_k; j.tmp_v = a.off;  // (the offsets are written by the fold, after the sort)
        j.n = nspill + claimed + (ecount ? 1u : 0u);
        j.has_vals = 1;
        j.src_ew = 8; j.dst_ew = 8;
        c->fold_k = a.spill_k;
        c->fold_v = a.spill_v;
        c->pair_sort = 1;
        c->radix_on = 1;
        c->guard_on = (c->path == P_MAIN);
        c->guard_general = c->guard_on;
    }
}

// Run offsets of the ranked pairs and the spill guard's bucket check (one
// workgroup).  If no bucket of the paper's table (M buckets, Eq. hash)
// receives more than four distinct keys, nothing spills (Alg. 1) and the guard is
// settled here.  `bc` holds kGuardLdsBuckets 32-bit words of LDS.
__device__ __forceinline__ void offsets_and_guard_check(const Args& a, Ctrl* c, uint32_t K, uint32_t* bc) {
    const uint32_t tid = threadIdx.x;
    // exclusive scan of the counts -> run offsets; each thread takes a contiguous chunk
    __shared__ uint64_t scan_tmp[17];
    const CAFS_GLOBAL uint64_t* cnt = gp(a.cnt);
    const uint32_t per = (K + blockDim.x - 1) / blockDim.x;
    const uint32_t b0 = tid * per < K ? tid * per : K;
    const uint32_t b1 = b0 + per < K ? b0 + per : K;
    uint64_t local = 0;
    for (uint32_t i = b0; i < b1; ++i) local += cnt[i];
    uint64_t total;
    uint64_t run = block_exclusive_scan<uint64_t>(local, scan_tmp, &total);
    for (uint32_t i = b0; i < b1; ++i) {
        gp(a.off)[i] = run;
        run += cnt[i];
    }
    if (tid == 0) {
        a.off[K] = total;
        c->K = K;
        c->dense_ready = 1;
        c->emit_main = 1;
    }
    // guard check on the paper's M buckets (main path only): count the distinct keys
    // of each bucket in LDS and list the keys of buckets holding more than four
    if (c->path != P_MAIN) return;
    const uint64_t M = c->table_M;
    if (M > kGuardLdsBuckets) {
        if (tid == 0) { c->guard_on = 1; c->guard_general = 1; }
        return;
    }
    const CAFS_GLOBAL uint64_t* uq = gp(a.uniq);
    __shared__ uint32_t s_nc, s_nb;
    const uint32_t lg = log2_pow2(M);
    for (uint32_t i = tid; i < M; i += blockDim.x) bc[i] = 0;
    if (tid == 0) { s_nc = 0; s_nb = 0; }
    __syncthreads();
    for (uint32_t i = tid; i < K; i += blockDim.x) atomicAdd(&bc[phi_hash32(uq[i], lg)], 1u);
    __syncthreads();
    uint32_t over = 0, over_b = 0;
    const uint32_t cap = a.cap;
    for (uint32_t i = tid; i < K; i += blockDim.x) over += bc[phi_hash32(uq[i], lg)] > cap;
    for (uint32_t i = tid; i < M; i += blockDim.x) over_b += bc[i] > cap;
    over = wave_sum_u32(over);
    over_b = wave_sum_u32(over_b);
    if (__lane_id() == 0 && over) atomicAdd(&s_nc, over);
    if (__lane_id() == 0 && over_b) atomicAdd(&s_nb, over_b);
    __syncthreads();
    const uint32_t nc = s_nc;
    if (nc > kGuardLdsKeys) {
        // too many for the one-workgroup resolution: the general kernels recount
        if (tid == 0) { c->guard_on = 1; c->guard_general = 1; }
        return;
    }
    __syncthreads();
    if (tid == 0) s_nc = 0;
    __syncthreads();
    for (uint32_t i = tid; i < K; i += blockDim.x)
        if (bc[phi_hash32(uq[i], lg)] > cap) a.clist[atomicAdd(&s_nc, 1u)] = i;
    if (tid == 0) {
        c->n_contested = nc;
        c->n_cbuckets = s_nb;
        c->guard_on = nc > 0;
    }
}

__device__ __forceinline__ void rank_body(const Args& a, uint32_t bid, uint32_t nblk) {
    Ctrl* c = a.c;
    if (c->engine != E_HASH || c->overflow || c->dense_ready) return;
    const uint32_t claimed = c->claimed;
    const uint64_t ecount = c->ecount;
    const uint64_t nspill = c->nspill;
    if (nspill) {
        // (the pairs never outnumber the elements; the radix engine would take over
        // if they did)
        if (nspill + claimed + 1 > a.n) {
            if (bid == 0 && threadIdx.x == 0) set_overflow(c, a.in == a.out, a.tmp_k, a.uniq);
            return;
        }
        gather_spill(a, c, claimed, ecount, nspill, bid, nblk);
        return;
    }
    const uint32_t K = claimed + (ecount > 0 ? 1u : 0u);
    if (!rank_ok(a, K)) {
        gather_pairs(a, c, claimed, ecount, K, bid, nblk);
        return;
    }
    if ((uint64_t)bid * kRankKeysPerBlock >= K) return;
    const uint64_t flip = a.flip, fneg = a.fneg;
    __shared__ uint64_t sk[kRankTile];
    // each wave ranks kRankKeysPerWave keys held in registers: its 64 lanes read the
    // staged keys once between them and compare each with all of the wave's keys, so
    // the LDS reads per key ranked are K / 64 wave loads
    constexpr uint32_t Q = kRankKeysPerWave;
    static_assert(Q * 16 == kRankKeysPerBlock, "16 waves of 1024 threads");
    const uint32_t wave = threadIdx.x >> 6, lane = __lane_id();
    for (uint32_t i0 = bid * kRankKeysPerBlock; i0 < K; i0 += nblk * kRankKeysPerBlock) {  // uniform
        uint64_t ki[Q];
        uint32_t r[Q];
#pragma unroll
        for (uint32_t q = 0; q < Q; ++q) {
            const uint32_t i = i0 + wave * Q + q;
            ki[q] = okey(i < K ? table_key(a, i, claimed) : 0, flip, fneg);
            r[q] = 0;
        }
        for (uint32_t j0 = 0; j0 < K; j0 += kRankTile) {
            const uint32_t jn = K - j0 < kRankTile ? K - j0 : kRankTile;
            __syncthreads();
            for (uint32_t j = threadIdx.x; j < jn; j += blockDim.x) sk[j] = okey(table_key(a, j0 + j, claimed), flip, fneg);
            __syncthreads();
            for (uint32_t j = lane; j < jn; j += 64) {
                const uint64_t v = sk[j];
#pragma unroll
                for (uint32_t q = 0; q < Q; ++q) r[q] += v < ki[q] ? 1u : 0u;
            }
        }
#pragma unroll
        for (uint32_t q = 0; q < Q; ++q) r[q] = wave_sum_u32(r[q]);
        // lane q writes key q of the wave (the keys are distinct, so the ranks are)
        uint32_t rq = r[0];
        uint64_t kq = ki[0];
#pragma unroll
        for (uint32_t q = 1; q < Q; ++q) {
            rq = lane == q ? r[q] : rq;
            kq = lane == q ? ki[q] : kq;
        }
        const uint32_t i = i0 + wave * Q + lane;
        if (lane < Q && i < K) {
            gp(a.uniq)[rq] = okey_inv(kq, flip, fneg);
            gp(a.cnt)[rq] = i < claimed ? gp(a.gcnt)[gp(a.claimed)[i]] : ecount;
        }
    }
}
CAFS_KERNELS0(rank, 1024)

// After the ranking: run offsets and the guard's bucket check, or the gather for a
// pair sort when K is too large to rank.  One workgroup.
__device__ __forceinline__ void compact_order_body(const Args& a, uint32_t bid, uint32_t nblk) {
    Ctrl* c = a.c;
    if (c->engine != E_HASH || c->overflow || c->dense_ready || c->pair_sort) return;
    const uint32_t claimed = c->claimed;
    const uint64_t ecount = c->ecount;
    const uint32_t K = claimed + (ecount > 0 ? 1u : 0u);
    if (!rank_ok(a, K)) return;  // gathered for the pair sort by the ranking launch
    __shared__ uint32_t bc[kGuardLdsBuckets];
    offsets_and_guard_check(a, c, K, bc);
}
CAFS_KERNELS0(compact_order, 1024)

// Fold and scan of the sorted pairs after a pair sort (Alg. 4: fold equal
// neighbours, then the running offset of each key), in two launches over the same
// grid.  Pair i heads a run when its key differs from pair i - 1's; each run becomes
// one distinct key whose count is the sum of the run's counts and whose offset is the
// sum of the counts before it.  Launch 1: each workgroup counts the heads of its
// chunk and sums its counts.  Launch 2: each workgroup adds the totals of the chunks
// before its own, scans its chunk, and the thread holding a head sums its run (which
// may reach into the next chunks) and writes the key, count and offset.  Without a
// spill the keys are distinct (every pair heads its run) and the pairs are folded in
// place.
__device__ __forceinline__ uint64_t scan_chunk(uint64_t T, uint32_t nblk) { return (T + nblk - 1) / nblk; }

__device__ __forceinline__ bool is_head(const CAFS_GLOBAL uint64_t* fk, uint64_t i) {
    return i == 0 || fk[i] != fk[i - 1];
}

__device__ __forceinline__ void fold_sums_body(const Args& a, uint32_t bid, uint32_t nblk) {
    Ctrl* c = a.c;
    if (!c->pair_sort || c->overflow) return;
    const uint64_t T = c->rj.n;
    const CAFS_GLOBAL uint64_t* fk = gp(c->fold_k);
    const CAFS_GLOBAL uint64_t* fv = gp(c->fold_v);
    const uint64_t ch = scan_chunk(T, nblk);
    const uint64_t b = (uint64_t)bid * ch < T ? (uint64_t)bid * ch : T;
    const uint64_t e = b + ch < T ? b + ch : T;
    uint64_t heads = 0, sum = 0;
    for (uint64_t i = b + threadIdx.x; i < e; i += blockDim.x) {
        heads += is_head(fk, i) ? 1u : 0u;
        sum += fv[i];
    }
    __shared__ uint64_t s_h, s_v;
    if (threadIdx.x == 0) { s_h = 0; s_v = 0; }
    __syncthreads();
    heads = wave_sum_u64(heads);
    sum = wave_sum_u64(sum);
    if (__lane_id() == 0) {
        if (heads) atomicAdd((unsigned long long*)&s_h, (unsigned long long)heads);
        if (sum) atomicAdd((unsigned long long*)&s_v, (unsigned long long)sum);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        gp(a.psum)[bid] = s_h;
        gp(a.psum)[kMaxCountBlocks + bid] = s_v;
    }
}
CAFS_KERNELS0(fold_sums, 1024)

__device__ __forceinline__ void fold_write_body(const Args& a, uint32_t bid, uint32_t nblk) {
    Ctrl* c = a.c;
    if (!c->pair_sort || c->overflow) return;
    __shared__ uint64_t scan_h[17], scan_v[17];
    __shared__ uint64_t s_bh, s_bv;
    const uint64_t T = c->rj.n;
    const CAFS_GLOBAL uint64_t* fk = gp(c->fold_k);
    const CAFS_GLOBAL uint64_t* fv = gp(c->fold_v);
    const uint64_t ch = scan_chunk(T, nblk);
    uint64_t bh = 0, bv = 0;
    for (uint32_t w = threadIdx.x; w < bid; w += blockDim.x) {
        bh += gp(a.psum)[w];
        bv += gp(a.psum)[kMaxCountBlocks + w];
    }
    if (threadIdx.x == 0) { s_bh = 0; s_bv = 0; }
    __syncthreads();
    bh = wave_sum_u64(bh);
    bv = wave_sum_u64(bv);
    if (__lane_id() == 0) {
        if (bh) atomicAdd((unsigned long long*)&s_bh, (unsigned long long)bh);
        if (bv) atomicAdd((unsigned long long*)&s_bv, (unsigned long long)bv);
    }
    __syncthreads();
    const uint64_t cb = (uint64_t)bid * ch < T ? (uint64_t)bid * ch : T;
    const uint64_t ce = cb + ch < T ? cb + ch : T;
    const uint64_t len = ce - cb;
    const uint64_t per = (len + blockDim.x - 1) / blockDim.x;
    const uint64_t b0 = cb + (threadIdx.x * per < len ? threadIdx.x * per : len);
    const uint64_t b1 = b0 + per < ce ? b0 + per : ce;
    uint64_t lh = 0, lv = 0;
    for (uint64_t i = b0; i < b1; ++i) {
        lh += is_head(fk, i) ? 1u : 0u;
        lv += fv[i];
    }
    uint64_t th, tv;
    uint64_t j = s_bh + block_exclusive_scan<uint64_t>(lh, scan_h, &th);
    uint64_t pos = s_bv + block_exclusive_scan<uint64_t>(lv, scan_v, &tv);
    // (in place there is no spill: every pair is its own run and is written back
    // where it was, so a read by a neighbour sees the same value either way)
    for (uint64_t i = b0; i < b1; ++i) {
        const uint64_t k = fk[i];
        const uint64_t v = fv[i];
        if (is_head(fk, i)) {
            uint64_t sum = v;
            for (uint64_t i2 = i + 1; i2 < T && fk[i2] == k; ++i2) sum += fv[i2];
            gp(a.uniq)[j] = k;
            gp(a.cnt)[j] = sum;
            gp(a.off)[j] = pos;
            ++j;
        }
        pos += v;
    }
    if (threadIdx.x == 0 && bid == nblk - 1) {
        const uint64_t K = s_bh + th;
        a.off[K] = s_bv + tv;
        c->K = K;
        c->dense_ready = 1;  // read by the next launch (the emit), after this grid ends
    }
}
CAFS_KERNELS0(fold_write, 1024)

}  // namespace cafs
