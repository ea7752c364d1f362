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

__device__ __noinline__ void set_overflow(const Args& a, Ctrl* c) {
    if (atomicExch(&c->overflow, 1u) == 0) {
        if (a.in == a.out) {  // see the dispatcher: keep the input for the guard
            c->rj.dst_k = a.tmp_k;
            c->rj.tmp_k = a.uniq;
            c->sorted = a.tmp_k;
            c->deferred_copy = 1;
        }
        atomicExch(&c->radix_on, 1u);
        atomicExch(&c->guard_on, 1u);
        atomicExch(&c->guard_general, 1u);
        atomicOr(&c->flags, 1u);
    }
}

// Insert (v, cnt) into the global open-addressing table (linear probing, Eq. hash
// slot).  A slot is claimed by CAS from kEmpty and never freed, so a key is either
// in the table or (after an overflow) the whole table is abandoned for the radix
// engine.  Claimed slots are listed so that compaction reads K entries, not the table.
__device__ __forceinline__ void global_insert(const Args& a, Ctrl* c, uint64_t v, uint64_t cnt) {
    if (atomic_load_agent(&c->overflow)) return;
    const uint32_t lg = c->cap_log2;
    const uint64_t mask = (1ull << lg) - 1;
    uint64_t h = phi_hash(v, lg);
    for (uint32_t pr = 0; pr < kGlobalProbe; ++pr) {
        uint64_t k = atomic_load_agent(&a.gkeys[h]);
        if (k == kEmpty) {
            const unsigned long long old =
                atomicCAS((unsigned long long*)&a.gkeys[h], (unsigned long long)kEmpty, (unsigned long long)v);
            if (old == kEmpty) {
                const uint32_t idx = atomicAdd(&c->claimed, 1u);
                if (idx >= c->cap_limit) { set_overflow(a, c); return; }
                a.claimed[idx] = (uint32_t)h;
                atomicAdd((unsigned long long*)&a.gcnt[h], (unsigned long long)cnt);
                return;
            }
            k = old;
        }
        if (k == v) {
            atomicAdd((unsigned long long*)&a.gcnt[h], (unsigned long long)cnt);
            return;
        }
        h = (h + 1) & mask;
    }
    set_overflow(a, c);
}

// ---------------------------------------------------------------------------
// Hash count (main path, Sec. 4.4).  The paper's hot loop updates a bucket of four
// 64-bit keys on one cache line (Sec. 4.2, Alg. 1).  Here each workgroup owns a
// table of 3072 such buckets in LDS (12288 keys with 32-bit counters).  An element
// hashes to a bucket (Eq. hash, reduced to 3072 by a multiply), reads its four keys
// with two 16-byte LDS loads and compares them with the element, the GPU analogue
// of the paper's cmpeq + movemask + tzcnt; on a match it adds 1 to that slot's
// counter with an LDS atomic.  Within a bucket occupied slots form a prefix and a
// key is stored in the first bucket, in probe order, that had room for it, so a
// lookup can stop at the first bucket with a free slot.  The fast path covers the
// home bucket and, when that one is full, the next bucket, as straight-line code
// for the eight keys a thread holds while the loads of its next eight keys are in
// flight.  Other keys take the slow path: claim the first free slot of the first
// bucket with room by a 64-bit LDS CAS, and after kLdsProbeBuckets full buckets go
// to the global table.  At the end each workgroup flushes its occupied slots to
// the global table.  Elements equal to the empty marker are counted in registers.
//
// This kernel also resolves the tiny branch: if the tiny counters sum to N the
// column is tiny and the dense arrays are written here; otherwise the element set
// has an unsampled value and the main path runs with the same estimate (Sec. 4.4).
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t lds_bucket(uint64_t x) {
    return (uint32_t)(((uint64_t)phi_hash32(x, 32) * kLdsBuckets) >> 32);
}

__device__ __forceinline__ void lds_insert_slow(const Args& a, Ctrl* c, uint64_t* skeys, uint32_t* scnt, uint64_t x) {
    uint32_t b = lds_bucket(x);
    for (uint32_t pr = 0; pr < kLdsProbeBuckets; ++pr) {
        const uint32_t base = b * kLdsBucketSlots;
        for (uint32_t s = 0; s < kLdsBucketSlots; ++s) {
            const uint64_t k = skeys[base + s];
            if (k == x) { atomicAdd(&scnt[s * kLdsBuckets + b], 1u); return; }
            if (k == kEmpty) {
                const unsigned long long old = atomicCAS((unsigned long long*)&skeys[base + s],
                                                         (unsigned long long)kEmpty, (unsigned long long)x);
                if (old == kEmpty || old == x) { atomicAdd(&scnt[s * kLdsBuckets + b], 1u); return; }
                // another key took the slot: the next slot may be free
            }
        }
        b = (b + 1 == kLdsBuckets) ? 0 : b + 1;
    }
    global_insert(a, c, x, 1);
}

// Slot of x among the four keys of a bucket, or -1; `full` tells whether the last
// slot is taken (then x may sit in a later bucket).
__device__ __forceinline__ int match4(const uint64_t* skeys, uint32_t b, uint64_t x, bool& full) {
    const u64x2 lo = *reinterpret_cast<const u64x2*>(skeys + b * kLdsBucketSlots);
    const u64x2 hi = *reinterpret_cast<const u64x2*>(skeys + b * kLdsBucketSlots + 2);
    full = hi.y != kEmpty;
    return lo.x == x ? 0 : lo.y == x ? 1 : hi.x == x ? 2 : hi.y == x ? 3 : -1;
}

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

    constexpr uint32_t S = kLdsBuckets * kLdsBucketSlots;
    __shared__ __attribute__((aligned(16))) uint64_t skeys[S];
    __shared__ uint32_t scnt[S];
    for (uint32_t i = threadIdx.x; i < S; i += blockDim.x) {
        skeys[i] = kEmpty;
        scnt[i] = 0;
    }
    __syncthreads();

    uint32_t ecnt = 0;
    const uint32_t head = a.in_head;
    const uint64_t P = num_pairs(a.n, head);
    const uint64_t Pf = (a.n + head) / 2;  // pairs [head, Pf) hold two in-range elements
    constexpr int U = 4;                   // pairs per thread per step
    const uint64_t span = (uint64_t)blockDim.x * U;
    const uint64_t step = (uint64_t)nblk * span;
    uint64_t base = (uint64_t)bid * span;
    uint64_t v[2 * U];
    uint32_t okm = 0;  // bit e: element e of the batch is in range
    auto load = [&](uint64_t b) {
        if (b >= head && b + span <= Pf) {
            // interior batch: every pair is two aligned in-range elements
            const u64x2* src = reinterpret_cast<const u64x2*>(a.in + 2 * (b + threadIdx.x) - head);
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const u64x2 w = src[(uint64_t)u * blockDim.x];
                v[2 * u] = w.x;
                v[2 * u + 1] = w.y;
            }
            okm = (1u << (2 * U)) - 1;
        } else {
            okm = 0;
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const uint64_t p = b + (uint64_t)u * blockDim.x + threadIdx.x;
                bool o0 = false, o1 = false;
                v[2 * u] = v[2 * u + 1] = 0;
                if (p < P) load_pair(a.in, a.n, head, p, v[2 * u], v[2 * u + 1], o0, o1);
                okm |= (o0 ? 1u : 0u) << (2 * u);
                okm |= (o1 ? 1u : 0u) << (2 * u + 1);
            }
        }
    };
    if (base < P) load(base);
    while (base < P) {
        uint64_t x[2 * U];
#pragma unroll
        for (int e = 0; e < 2 * U; ++e) x[e] = v[e];
        const uint32_t xok = okm;
        const uint64_t next = base + step;
        if (next < P) load(next);  // next batch in flight while this one is counted
        uint32_t pend = 0;
#pragma unroll
        for (int e = 0; e < 2 * U; ++e) {
            const bool in = (xok >> e) & 1u;
            const bool is_empty_key = x[e] == kEmpty;
            ecnt += (in && is_empty_key) ? 1u : 0u;
            const bool want = in && !is_empty_key;
            uint32_t b = lds_bucket(x[e]);
            bool full;
            int m = match4(skeys, b, x[e], full);
            if (m < 0 && full) {  // home bucket full without x: x may be in the next one
                b = (b + 1 == kLdsBuckets) ? 0 : b + 1;
                m = match4(skeys, b, x[e], full);
            }
            const bool hit = want && m >= 0;
            // counters are slot-major (slot s of bucket b at s * 3072 + b) so that the
            // first slots of many buckets spread over the LDS banks; a miss adds 0
            atomicAdd(&scnt[(m < 0 ? 0 : m) * kLdsBuckets + b], hit ? 1u : 0u);
            pend |= (want && !hit) ? (1u << e) : 0u;
        }
        if (pend) {
#pragma unroll 1
            for (int e = 0; e < 2 * U; ++e)
                if (pend & (1u << e)) lds_insert_slow(a, c, skeys, scnt, x[e]);
        }
        base = next;
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < S; i += blockDim.x) {
        const uint32_t cn = scnt[i];  // slot i / 3072 of bucket i % 3072; never 0 once claimed
        if (cn) global_insert(a, c, skeys[(i % kLdsBuckets) * kLdsBucketSlots + i / kLdsBuckets], cn);
    }
    const uint32_t wsum = wave_sum_u32(ecnt);
    if (__lane_id() == 0 && wsum) atomicAdd((unsigned long long*)&c->ecount, (unsigned long long)wsum);
}
CAFS_KERNELS0(hash_count, kCountThreads)

// ---------------------------------------------------------------------------
// Compaction and order (Alg. 4, steps "collect non-empty bucket slots", "sort
// pairs by key").  One workgroup.  For K <= 8192 the (key, count) pairs are
// sorted in LDS by a bitonic network and their counts scanned into run offsets;
// larger K goes to the radix engine in pair mode.  With the sorted pairs at hand
// this kernel also checks the spill guard's buckets: if no bucket of the paper's
// table (M buckets, Eq. hash) receives more than 4 distinct keys, nothing spills
// (Alg. 1) and the guard is settled here.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void compact_order_body(const Args& a, uint32_t bid, uint32_t nblk) {
    Ctrl* c = a.c;
    if (c->engine != E_HASH || c->overflow || c->dense_ready) return;
    const uint32_t claimed = c->claimed;
    const uint64_t ecount = c->ecount;
    const uint32_t K = claimed + (ecount > 0 ? 1u : 0u);
    const uint64_t flip = a.flip;
    const uint32_t tid = threadIdx.x;
    if (K > kOrderMax) {
        // gather the pairs into the dense arrays and sort them there, in place, with
        // the radix engine; the hash table is dead after the gather and serves as
        // the radix scratch (K <= table size)
        for (uint32_t i = tid; i < claimed; i += blockDim.x) {
            const uint32_t h = a.claimed[i];
            a.uniq[i] = a.gkeys[h];
            a.cnt[i] = a.gcnt[h];
        }
        if (tid == 0) {
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
        return;
    }
    __shared__ uint64_t sk[kOrderMax];
    __shared__ uint64_t sv[kOrderMax];
    __shared__ uint64_t scan_tmp[17];
    uint32_t P = 64;
    while (P < K) P <<= 1;
    for (uint32_t i = tid; i < P; i += blockDim.x) {
        if (i < claimed) {
            const uint32_t h = a.claimed[i];
            sk[i] = a.gkeys[h] ^ flip;
            sv[i] = a.gcnt[h];
        } else if (i < K) {
            sk[i] = kEmpty ^ flip;
            sv[i] = ecount;
        } else {
            sk[i] = ~0ull;  // padding sorts last: ties with a real key are broken by count 0
            sv[i] = 0;
        }
    }
    __syncthreads();
    // bitonic sort of (key, count) by key ascending; equal keys only occur between a
    // real key and padding, and the real key (count >= 1) goes first
    for (uint32_t kk = 2; kk <= P; kk <<= 1) {
        for (uint32_t jj = kk >> 1; jj > 0; jj >>= 1) {
            for (uint32_t i = tid; i < P; i += blockDim.x) {
                const uint32_t l = i ^ jj;
                if (l > i) {
                    const uint64_t ki = sk[i], kl = sk[l];
                    const uint64_t vi = sv[i], vl = sv[l];
                    const bool i_gt = (ki > kl) || (ki == kl && vi < vl);
                    const bool up = (i & kk) == 0;
                    if (up == i_gt) {
                        sk[i] = kl; sk[l] = ki;
                        sv[i] = vl; sv[l] = vi;
                    }
                }
            }
            __syncthreads();
        }
    }
    // exclusive scan of the counts -> run offsets; each thread takes a contiguous chunk
    const uint32_t per = (K + blockDim.x - 1) / blockDim.x;
    const uint32_t b0 = tid * per < K ? tid * per : K;
    const uint32_t b1 = b0 + per < K ? b0 + per : K;
    uint64_t local = 0;
    for (uint32_t i = b0; i < b1; ++i) local += sv[i];
    uint64_t total;
    uint64_t run = block_exclusive_scan<uint64_t>(local, scan_tmp, &total);
    for (uint32_t i = b0; i < b1; ++i) {
        a.uniq[i] = sk[i] ^ flip;
        a.cnt[i] = sv[i];
        a.off[i] = run;
        run += sv[i];
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
    __shared__ uint32_t s_nc;
    __syncthreads();
    uint32_t* bc = reinterpret_cast<uint32_t*>(sv);  // reuse: M <= 16384 u32 counters
    const uint32_t lg = log2_pow2(M);
    for (uint32_t i = tid; i < M; i += blockDim.x) bc[i] = 0;
    if (tid == 0) s_nc = 0;
    __syncthreads();
    for (uint32_t i = tid; i < K; i += blockDim.x) atomicAdd(&bc[phi_hash32(sk[i] ^ flip, lg)], 1u);
    __syncthreads();
    __shared__ uint32_t s_nb;
    if (tid == 0) s_nb = 0;
    __syncthreads();
    uint32_t over = 0, over_b = 0;
    for (uint32_t i = tid; i < K; i += blockDim.x) over += bc[phi_hash32(sk[i] ^ flip, lg)] > kBucketCap;
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
        if (bc[phi_hash32(sk[i] ^ flip, lg)] > kBucketCap) a.clist[atomicAdd(&s_nc, 1u)] = i;
    if (tid == 0) {
        c->n_contested = nc;
        c->n_cbuckets = s_nb;
        c->guard_on = nc > 0;
    }
}
CAFS_KERNELS0(compact_order, 1024)

// Exclusive scan of the sorted counts after a pair sort (K > 8192).  One workgroup.
__device__ __forceinline__ void pair_scan_body(const Args& a, uint32_t bid, uint32_t nblk) {
    Ctrl* c = a.c;
    if (!c->pair_sort || c->overflow) return;
    __shared__ uint64_t scan_tmp[17];
    const uint64_t K = c->K;
    const uint64_t per = (K + blockDim.x - 1) / blockDim.x;
    const uint64_t b0 = threadIdx.x * per < K ? threadIdx.x * per : K;
    const uint64_t b1 = b0 + per < K ? b0 + per : K;
    uint64_t local = 0;
    for (uint64_t i = b0; i < b1; ++i) local += a.cnt[i];
    uint64_t total;
    uint64_t run = block_exclusive_scan<uint64_t>(local, scan_tmp, &total);
    for (uint64_t i = b0; i < b1; ++i) {
        a.off[i] = run;
        run += a.cnt[i];
    }
    if (threadIdx.x == 0) {
        a.off[K] = total;
        c->dense_ready = 1;
    }
}
CAFS_KERNELS0(pair_scan, 1024)

}  // namespace cafs
