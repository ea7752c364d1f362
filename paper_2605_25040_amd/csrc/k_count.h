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
// with every key.  The GPU form of the paper's eight branchless counters is a
// wave ballot: v_cmp_eq_u64 gives a 64-lane mask per key whose population count
// is added to a wave-uniform (scalar) counter.
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
    uint32_t cnt[8] = {0, 0, 0, 0, 0, 0, 0, 0};  // per wave, fits: a wave sees < 2^32 elements
    const uint32_t head = a.in_head;
    const uint64_t P = num_pairs(a.n, head);
    const uint64_t Pf = (a.n + head) / 2;
    constexpr int U = 8;  // pairs in flight per lane
    // every lane of a wave runs the same iterations so that each ballot sees the whole wave
    const uint64_t waves_total = gstride / 64;
    const uint64_t wave_id = gtid / 64;
    const uint32_t lane = __lane_id();
    for (uint64_t pb = wave_id * 64 * U; pb < P; pb += waves_total * 64 * U) {
        uint64_t v[2 * U];
        uint32_t okm = 0;
        if (pb >= head && pb + 64 * U <= Pf) {
            const u64x2* src = reinterpret_cast<const u64x2*>(a.in + 2 * (pb + lane) - head);
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const u64x2 w = src[u * 64];
                v[2 * u] = w.x;
                v[2 * u + 1] = w.y;
            }
            okm = (1u << (2 * U)) - 1;
        } else {
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
#pragma unroll
        for (int e = 0; e < 2 * U; ++e) {
            const bool in = (okm >> e) & 1u;
#pragma unroll
            for (int j = 0; j < 8; ++j)
                if (j < (int)nk) cnt[j] += (uint32_t)__popcll(__ballot(in && v[e] == key[j]));
        }
    }
    if (lane == 0) {
        for (uint32_t j = 0; j < nk; ++j)
            if (cnt[j]) atomicAdd((unsigned long long*)&c->tiny_cnt[j], (unsigned long long)cnt[j]);
    }
}
CAFS_KERNELS0(phase2, 256)

// Switch to the radix engine after the global table overflowed.  In place, the
// radix engine then sorts into scratch so that the guard can still read the input.
__device__ __noinline__ void set_overflow(Ctrl* c, uint32_t inplace, uint64_t* tmp_k, uint64_t* uniq) {
    if (atomicExch(&c->overflow, 1u) == 0) {
        if (inplace) {
            c->rj.dst_k = tmp_k;
            c->rj.tmp_k = uniq;
            c->sorted = tmp_k;
            c->deferred_copy = 1;
        }
        atomicExch(&c->radix_on, 1u);
        atomicExch(&c->guard_on, 1u);
        atomicExch(&c->guard_general, 1u);
        atomicOr(&c->flags, 1u);
    }
}

// The global (key, count) table of one column.
struct GTable {
    Ctrl* c;
    uint64_t* keys;
    unsigned long long* cnt;
    uint32_t* claimed;
    uint64_t* tmp_k;
    uint64_t* uniq;
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
    t.inplace = a.in == a.out;
    t.mul = a.table_mul;
    return t;
}

// Insert (v, cnt) into the global open-addressing table (linear probing, Eq. hash
// slot).  A slot is claimed by CAS from kEmpty and never freed, so a key is either
// in the table or (after an overflow) the whole table is abandoned for the radix
// engine.  Returns the slot claimed for a new key (kNoSlot otherwise); the caller
// lists claimed slots with list_claims, so that compaction reads K entries, not the
// table.
constexpr uint32_t kNoSlot = 0xFFFFFFFFu;

// The overflow flag, read by one lane and broadcast: an agent-scope load misses the
// XCD's L2 and goes to memory, and every lane of the GPU reading the same word
// queues on one line.  Called with every lane of the wave active.
__device__ __forceinline__ uint32_t wave_overflow(const Ctrl* c) {
    uint32_t ov = 0;
    if (__lane_id() == 0) ov = g_load(&c->overflow);
    return __builtin_amdgcn_readfirstlane(ov);
}

// The caller checks the overflow flag (per wave) before it inserts; a long probe
// looks again every kGlobalProbeCheck slots, so that inserts under way stop soon
// after the table passed its load limit (they would otherwise keep claiming slots
// and probe ever longer).
__device__ __forceinline__ uint32_t global_insert(const GTable& t, uint64_t v, uint64_t cnt) {
    Ctrl* c = t.c;
    const uint32_t lg = c->cap_log2;
    const uint64_t mask = (1ull << lg) - 1;
    uint64_t h = mul_hash(v, lg, t.mul);
    for (uint32_t pr = 0; pr < kGlobalProbe; ++pr) {
        if (pr % kGlobalProbeCheck == kGlobalProbeCheck - 1 && g_load(&c->overflow)) return kNoSlot;
        uint64_t k = g_load(&t.keys[h]);
        if (k == kEmpty) {
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
    set_overflow(c, t.inplace, t.tmp_k, t.uniq);
    return kNoSlot;
}

// Lists the slots the lanes of a wave claimed (kNoSlot: none) in the claimed-slot
// list, with one update of the shared counter per wave (one per claim would
// serialise on its address).  Past the table's load limit the radix engine takes
// over.  Called by every lane of the wave.
__device__ __forceinline__ void list_claims(const GTable& t, uint32_t h) {
    const uint64_t m = __ballot(h != kNoSlot);
    if (m == 0) return;
    const uint32_t leader = (uint32_t)__builtin_ctzll(m);
    uint32_t base = 0;
    if (__lane_id() == leader) base = g_add(&t.c->claimed, (uint32_t)__popcll(m));
    base = __shfl(base, leader, 64);
    if (h == kNoSlot) return;
    const uint32_t idx =
        base + __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
    if (idx >= t.c->cap_limit) set_overflow(t.c, t.inplace, t.tmp_k, t.uniq);
    else gp(t.claimed)[idx] = h;
}

// ---------------------------------------------------------------------------
// Hash count (main path, Sec. 4.4).  The paper's hot loop updates a bucket of four
// 64-bit keys on one cache line (Sec. 4.2, Alg. 1).  Here each workgroup owns a
// table of kLdsSlots keys with 32-bit counters in LDS, cut into buckets of W keys:
// W = 4 (3392 buckets, like the paper's) when the estimate is large, W = 2 (6784
// buckets) below kLdsWideMinKhat, where a bucket rarely overflows and a lookup
// then takes one 16-byte LDS load instead of two (LDS load instructions are what
// the loop pays for; measured crossover near K = 1800 at N = 2^28).  An element
// hashes to a bucket (Eq. hash, reduced to the bucket count by a multiply), reads
// its W keys with 16-byte LDS loads and compares them with the element, the GPU
// analogue of the paper's cmpeq + movemask + tzcnt; on a match it adds 1 to that
// slot's counter with an LDS atomic.  Within a bucket occupied slots form a
// prefix and a key is stored in the first bucket, in probe order, that had room
// for it, so a lookup can stop at the first bucket with a free slot.  Lookups cover the home
// bucket and, when that one is full, the next one (the window), as straight-line
// code for the eight keys a thread holds while the loads of its next eight keys
// are in flight.  A key absent from a window with room is inserted by a 64-bit
// LDS CAS on the first free slot.  An element whose window is full is deferred:
// the wave appends it to its workgroup's region of a scratch array, and a second
// pass counts the deferred elements with a fresh table.  Deferring keeps the
// rare long probes out of the wave-wide lockstep of the hot loop.  At the end
// each workgroup flushes its occupied slots to the global table (Eq. hash slot,
// linear probing).  Elements equal to the empty marker are counted in registers.
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

template <uint32_t W>
__device__ __forceinline__ uint32_t lds_bucket(uint64_t x, uint64_t mul) {
    return (uint32_t)(((uint64_t)mul_hash32(x, 32, mul) * LdsGeo<W>::kBuckets) >> 32);
}

template <uint32_t W>
__device__ __forceinline__ uint32_t next_bucket(uint32_t b) {
    return (b + 1 == LdsGeo<W>::kBuckets) ? 0 : b + 1;
}

// Find or claim a slot for x within `window` buckets from its home bucket and add
// `add` to its counter.  Returns false when those buckets are full without x.
template <uint32_t W>
__device__ __forceinline__ bool lds_insert(uint64_t* skeys, uint32_t* scnt, uint64_t x, uint32_t add,
                                           uint32_t window, uint64_t mul) {
    uint32_t b = lds_bucket<W>(x, mul);
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

// Counts the elements of x selected by `want` in the LDS table, one after the
// other (the loads of the next batch are in flight meanwhile); returns the mask of
// those whose window was full (not counted).
template <int NE, uint32_t W>
__device__ __forceinline__ uint32_t count_batch(uint64_t* __restrict__ skeys, uint32_t* __restrict__ scnt,
                                                uint32_t* __restrict__ sink, const uint64_t (&x)[NE],
                                                uint32_t want_m, uint64_t mul, const uint32_t (&add)[NE]) {
    uint32_t ins = 0, dfr = 0;
#pragma unroll
    for (int e = 0; e < NE; ++e) {
        const bool want = (want_m >> e) & 1u;
        uint32_t b = lds_bucket<W>(x[e], mul);
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
            if (((ins >> e) & 1u) && !lds_insert<W>(skeys, scnt, x[e], add[e], kLdsWindow, mul)) dfr |= 1u << e;
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

// Each workgroup of the first pass reads one contiguous range of ceil(P / nblk)
// pairs; its region of the deferred-element scratch (tmp_k) holds that many pairs,
// so it never fills up (tmp_k has room for n + 2 + 2 * kMaxCountBlocks keys).
__device__ __forceinline__ uint64_t pairs_per_block(uint64_t P, uint32_t nblk) { return (P + nblk - 1) / nblk; }

template <uint32_t W>
__device__ __forceinline__ void flush_table(const GTable& t, const uint64_t* skeys, const uint32_t* scnt) {
    constexpr uint32_t S = kLdsSlots, B = LdsGeo<W>::kBuckets;
    // once the table has overflowed (the radix engine takes over) the flush is moot;
    // each wave looks before every group of inserts
    // four slots per thread at a time: their home slots in the global table are read
    // together, and a key already there (most are, after the first workgroups) gets
    // its count added directly; the rest take the probing insert
    const uint32_t lg = t.c->cap_log2;
    constexpr int F = 4;
    for (uint32_t i0 = threadIdx.x; i0 < S; i0 += F * blockDim.x) {  // uniform over each wave
        if (wave_overflow(t.c)) return;
        uint32_t cn[F], h[F], cl[F];
        uint64_t key[F], k[F];
#pragma unroll
        for (int u = 0; u < F; ++u) {
            const uint32_t i = i0 + u * blockDim.x;
            cn[u] = i < S ? scnt[i] : 0u;  // slot i / B of bucket i % B; never 0 once claimed
            key[u] = cn[u] ? skeys[(i % B) * W + i / B] : 0;
            h[u] = mul_hash(key[u], lg, t.mul);
        }
#pragma unroll
        for (int u = 0; u < F; ++u) k[u] = cn[u] ? g_load(&t.keys[h[u]]) : kEmpty;
#pragma unroll
        for (int u = 0; u < F; ++u) {
            cl[u] = kNoSlot;
            if (!cn[u]) continue;
            if (k[u] == key[u]) g_add(&t.cnt[h[u]], (unsigned long long)cn[u]);
            else cl[u] = global_insert(t, key[u], cn[u]);
        }
#pragma unroll
        for (int u = 0; u < F; ++u) list_claims(t, cl[u]);  // (the loop is uniform over each wave)
    }
}

template <uint32_t W>
__device__ __forceinline__ void hash_count_table(const Args& a, uint32_t bid, uint32_t nblk, uint64_t* skeys,
                                                 uint32_t* scnt, uint32_t& s_ndef, uint32_t* s_sink);

__device__ __forceinline__ void hash_count_body(const Args& a, uint32_t bid, uint32_t nblk) {
    Ctrl* c = a.c;
    const uint32_t engine = c->engine;
    if (engine == E_TINY) {
        const uint32_t nk = c->n_tiny;
        uint64_t tot = 0;
        for (uint32_t j = 0; j < nk; ++j) tot += c->tiny_cnt[j];
        if (tot == a.n) {
            if (bid == 0 && threadIdx.x == 0) {
                uint64_t run = 0;
                for (uint32_t j = 0; j < nk; ++j) {
                    a.uniq[j] = c->tiny_keys[j];
                    a.cnt[j] = c->tiny_cnt[j];
                    a.off[j] = run;
                    run += c->tiny_cnt[j];
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

    constexpr uint32_t S = kLdsSlots;
    __shared__ __attribute__((aligned(16))) uint64_t skeys[S];
    __shared__ uint32_t scnt[S];
    __shared__ uint32_t s_ndef;
    __shared__ uint32_t s_sink[64];  // target of the atomics of lanes without a hit
    for (uint32_t i = threadIdx.x; i < S; i += blockDim.x) {
        skeys[i] = kEmpty;
        scnt[i] = 0;
    }
    if (threadIdx.x == 0) s_ndef = 0;
    __syncthreads();
    if (c->k_hat < kLdsWideMinKhat) hash_count_table<2>(a, bid, nblk, skeys, scnt, s_ndef, s_sink);
    else hash_count_table<4>(a, bid, nblk, skeys, scnt, s_ndef, s_sink);
}

// The count over one workgroup's range with buckets of W keys (the table in LDS
// is cleared).
template <uint32_t W>
__device__ __forceinline__ void hash_count_table(const Args& a, uint32_t bid, uint32_t nblk, uint64_t* skeys,
                                                 uint32_t* scnt, uint32_t& s_ndef, uint32_t* s_sink) {
    constexpr uint32_t S = kLdsSlots;
    Ctrl* c = a.c;
    const GTable t = gtable(a);
    const uint64_t n = a.n;
    const CAFS_GLOBAL uint64_t* in = gp(a.in);
    const uint32_t lane = __lane_id();
    uint32_t ecnt = 0;
    const uint32_t head = a.in_head;
    const uint64_t P = num_pairs(n, head);
    const uint64_t Pf = (n + head) / 2;  // pairs [head, Pf) hold two in-range elements
    const uint64_t PP = pairs_per_block(P, nblk);
    const uint64_t p_end = (uint64_t)(bid + 1) * PP < P ? (uint64_t)(bid + 1) * PP : P;
    const uint64_t p_full = p_end < Pf ? p_end : Pf;
    CAFS_GLOBAL uint64_t* region = gp(a.tmp_k) + (uint64_t)bid * 2 * PP;
    constexpr int U = 4;                 // pairs per thread per step
    constexpr int NE = 2 * U;
    const uint64_t span = (uint64_t)blockDim.x * U;
    uint64_t base = (uint64_t)bid * PP;
    uint64_t v[NE];
    uint32_t okm = 0;  // bit e: element e of the batch is in range
    auto load = [&](uint64_t b) {
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
        // (the flag's load overlaps this batch), or hand it over when a quarter of the
        // elements so far found no room (K far beyond the table)
        const bool check = (++iter & 7) == 0;
        // (lane 0 loads the flag; the wave reads it from lane 0 after the batch)
        const uint32_t handed = (check && __lane_id() == 0) ? g_load(&c->overflow) : 0u;
        if (check) {
            const uint64_t seen = 2 * (base - (uint64_t)bid * PP);
            if (4ull * s_ndef > seen && seen > 2 * PP / 8) {
                if (lane == 0) set_overflow(c, t.inplace, t.tmp_k, t.uniq);
                break;
            }
        }
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
        const bool rle = run_lengths<NE>(x, want, add);
        if (rle) {
            // merged elements are counted by their run's head
#pragma unroll
            for (int e = 0; e < NE; ++e) want &= add[e] ? ~0u : ~(1u << e);
            const uint32_t dfr = count_batch<NE, W>(skeys, scnt, s_sink, x, want, t.mul, add);
            // a deferred head stands for its whole run: that many copies go to the region
            // (the region has room for every element of the workgroup's range)
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
        const uint32_t dfr = count_batch<NE, W>(skeys, scnt, s_sink, x, want, t.mul, ones);
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
    __syncthreads();
    flush_table<W>(t, skeys, scnt);
    const uint32_t wsum = wave_sum_u32(ecnt);
    if (lane == 0 && wsum) g_add(&c->ecount, (uint64_t)wsum);
    // Second pass over this workgroup's deferred elements, with the table cleared
    // (the keys that found no room are few) and a longer probe; what still finds no
    // room goes to the global table.
    const uint32_t d = s_ndef;  // uniform: read after the barrier
    if (d == 0 || wave_overflow(c)) return;  // (d is uniform)
    __syncthreads();  // (the workgroup reads back only its own region)
    for (uint32_t i = threadIdx.x; i < S; i += blockDim.x) {
        skeys[i] = kEmpty;
        scnt[i] = 0;
    }
    __syncthreads();
    if (threadIdx.x == 0) s_ndef = 0;  // now: elements that found no room in the second table either
    __syncthreads();
    constexpr int D = 4;  // elements per thread per step
    for (uint32_t i0 = 0; i0 < d; i0 += D * blockDim.x) {
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
        const uint32_t dfr = count_batch<D, W>(skeys, scnt, s_sink, xd, want, t.mul, ones);
        uint32_t cl[D];
#pragma unroll
        for (int u = 0; u < D; ++u) cl[u] = kNoSlot;
        const uint32_t ov = wave_overflow(c);
        if (dfr && !ov) {
#pragma unroll
            for (int u = 0; u < D; ++u) {
                if (((dfr >> u) & 1u) && !lds_insert<W>(skeys, scnt, xd[u], 1u, kLdsProbeBuckets, t.mul)) {
                    atomicAdd(&s_ndef, 1u);
                    cl[u] = global_insert(t, xd[u], 1);
                }
            }
        }
#pragma unroll
        for (int u = 0; u < D; ++u) list_claims(t, cl[u]);
        // too many keys even for a second table: per-element global inserts would cost
        // more than sorting, so the radix engine takes over (the count is read between
        // two barriers, so every thread takes the same decision)
        __syncthreads();
        const bool stop = 64ull * s_ndef > 2 * PP;
        __syncthreads();
        if (stop) {
            if (threadIdx.x == 0) set_overflow(c, t.inplace, t.tmp_k, t.uniq);
            break;
        }
    }
    __syncthreads();
    flush_table<W>(t, skeys, scnt);
}
CAFS_KERNELS0(hash_count, kCountThreads)

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
        c->K = K;
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
    for (uint32_t i = tid; i < K; i += blockDim.x) over += bc[phi_hash32(uq[i], lg)] > kBucketCap;
    for (uint32_t i = tid; i < M; i += blockDim.x) over_b += bc[i] > kBucketCap;
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
        if (bc[phi_hash32(uq[i], lg)] > kBucketCap) a.clist[atomicAdd(&s_nc, 1u)] = i;
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
    const uint32_t K = claimed + (ecount > 0 ? 1u : 0u);
    if (!rank_ok(a, K)) {
        gather_pairs(a, c, claimed, ecount, K, bid, nblk);
        return;
    }
    if ((uint64_t)bid * kRankKeysPerBlock >= K) return;
    const uint64_t flip = a.flip, fneg = a.fneg;
    __shared__ uint64_t sk[kRankTile];
    const uint32_t part = threadIdx.x % 16;
    for (uint32_t i0 = bid * kRankKeysPerBlock; i0 < K; i0 += nblk * kRankKeysPerBlock) {  // uniform
        const uint32_t i = i0 + threadIdx.x / 16;
        const bool have = i < K;
        const uint64_t ki = okey(have ? table_key(a, i, claimed) : 0, flip, fneg);
        uint32_t r = 0;
        for (uint32_t j0 = 0; j0 < K; j0 += kRankTile) {
            const uint32_t jn = K - j0 < kRankTile ? K - j0 : kRankTile;
            __syncthreads();
            for (uint32_t j = threadIdx.x; j < jn; j += blockDim.x) sk[j] = okey(table_key(a, j0 + j, claimed), flip, fneg);
            __syncthreads();
            for (uint32_t j = part; j < jn; j += 16) r += sk[j] < ki ? 1u : 0u;
        }
        r += __shfl_xor(r, 8, 16);
        r += __shfl_xor(r, 4, 16);
        r += __shfl_xor(r, 2, 16);
        r += __shfl_xor(r, 1, 16);
        if (have && part == 0) {
            gp(a.uniq)[r] = okey_inv(ki, flip, fneg);
            gp(a.cnt)[r] = i < claimed ? gp(a.gcnt)[gp(a.claimed)[i]] : ecount;
        }
    }
}
CAFS_KERNELS0(rank, 1024)

// After the ranking: run offsets and the guard's bucket check, or the gather for a
// pair sort when K is too large to rank.  One workgroup.
__device__ __forceinline__ void compact_order_body(const Args& a, uint32_t bid, uint32_t nblk) {
    Ctrl* c = a.c;
    if (c->engine != E_HASH || c->overflow || c->dense_ready) return;
    const uint32_t claimed = c->claimed;
    const uint64_t ecount = c->ecount;
    const uint32_t K = claimed + (ecount > 0 ? 1u : 0u);
    if (!rank_ok(a, K)) return;  // gathered for the pair sort by the ranking launch
    __shared__ uint32_t bc[kGuardLdsBuckets];
    offsets_and_guard_check(a, c, K, bc);
}
CAFS_KERNELS0(compact_order, 1024)

// Exclusive scan of the sorted counts after a pair sort, in two launches over the
// same grid: each workgroup sums its chunk of the counts, then each adds the sums
// of the chunks before its own and scans its chunk.
__device__ __forceinline__ uint64_t scan_chunk(uint64_t K, uint32_t nblk) { return (K + nblk - 1) / nblk; }

__device__ __forceinline__ void pair_sums_body(const Args& a, uint32_t bid, uint32_t nblk) {
    Ctrl* c = a.c;
    if (!c->pair_sort || c->overflow) return;
    const uint64_t K = c->K;
    const uint64_t ch = scan_chunk(K, nblk);
    const uint64_t b = (uint64_t)bid * ch < K ? (uint64_t)bid * ch : K;
    const uint64_t e = b + ch < K ? b + ch : K;
    uint64_t local = 0;
    for (uint64_t i = b + threadIdx.x; i < e; i += blockDim.x) local += gp(a.cnt)[i];
    __shared__ uint64_t s_sum;
    if (threadIdx.x == 0) s_sum = 0;
    __syncthreads();
    local = wave_sum_u64(local);
    if (__lane_id() == 0 && local) atomicAdd((unsigned long long*)&s_sum, (unsigned long long)local);
    __syncthreads();
    if (threadIdx.x == 0) gp(a.psum)[bid] = s_sum;
}
CAFS_KERNELS0(pair_sums, 1024)

__device__ __forceinline__ void pair_scan_body(const Args& a, uint32_t bid, uint32_t nblk) {
    Ctrl* c = a.c;
    if (!c->pair_sort || c->overflow) return;
    __shared__ uint64_t scan_tmp[17];
    __shared__ uint64_t s_base;
    const uint64_t K = c->K;
    const uint64_t ch = scan_chunk(K, nblk);
    uint64_t before = 0;
    for (uint32_t w = threadIdx.x; w < bid; w += blockDim.x) before += gp(a.psum)[w];
    if (threadIdx.x == 0) s_base = 0;
    __syncthreads();
    before = wave_sum_u64(before);
    if (__lane_id() == 0 && before) atomicAdd((unsigned long long*)&s_base, (unsigned long long)before);
    __syncthreads();
    const uint64_t cb = (uint64_t)bid * ch < K ? (uint64_t)bid * ch : K;
    const uint64_t ce = cb + ch < K ? cb + ch : K;
    const uint64_t len = ce - cb;
    const uint64_t per = (len + blockDim.x - 1) / blockDim.x;
    const uint64_t b0 = cb + (threadIdx.x * per < len ? threadIdx.x * per : len);
    const uint64_t b1 = b0 + per < ce ? b0 + per : ce;
    const CAFS_GLOBAL uint64_t* cnt = gp(a.cnt);
    uint64_t local = 0;
    for (uint64_t i = b0; i < b1; ++i) local += cnt[i];
    uint64_t total;
    uint64_t run = s_base + block_exclusive_scan<uint64_t>(local, scan_tmp, &total);
    for (uint64_t i = b0; i < b1; ++i) {
        gp(a.off)[i] = run;
        run += cnt[i];
    }
    if (threadIdx.x == 0 && bid == nblk - 1) {
        a.off[K] = s_base + total;
        c->dense_ready = 1;  // read by the next launch (the emit), after this grid ends
    }
}
CAFS_KERNELS0(pair_scan, 1024)

}  // namespace cafs
