// Exact spill of the paper's bucket table, computed from the (key, count) pairs.
//
// In Alg. 1 a bucket never evicts and its counters only grow, so a bucket keeps
// the first cap distinct keys that hash to it (Eq. hash over M buckets, Eq. Msize;
// cap = 4 for 64-bit keys, 8 for 32-bit keys) in order of first occurrence, and
// every occurrence of any later key of that bucket goes to the spill (counted in
// elements; the RLE step of Sec. 4.4 does not change that count).  Hence
//     |spill| = sum over buckets with more than cap distinct keys of the counts of
//               the keys whose first occurrence is not among the bucket's first cap.
// The guard of Alg. 4 fires when |spill| > N/2 (tested as 2 |spill| > N).
//
// The GPU computes it in these steps, all skipped when no bucket is over-full:
//   (the order kernel counts the buckets in LDS and lists the keys of over-full,
//    "contested", buckets when K <= 8192, M <= 16384 and at most 2048 are contested;
//    otherwise the three general kernels below do it from the dense pairs)
//   k_guard_prep    clear bucket counters and the cap per-bucket minima (general)
//   k_guard_bucket  distinct keys per bucket (general)
//   k_guard_mark    list the contested keys (general); reset their first occurrences
//   k_guard_first   first occurrence of each contested key: one pass over the
//                   input in increasing chunks that stops once every contested
//                   key has been seen (later chunks cannot hold a first occurrence)
//   k_guard_resolve at most 2048 contested keys: rank them by first occurrence
//                   within their bucket in LDS and sum the spilled counts
//   k_guard_round   otherwise, r = 0..cap-1: the r-th smallest first occurrence per bucket
//   k_guard_final   and the sum of the counts of keys later than the cap-th
#pragma once
#include "cafs_dev.h"

namespace cafs {

constexpr uint32_t kNoIndex = 0xFFFFFFFFu;

__device__ __forceinline__ bool guard_active(const Ctrl* c) {
    return c->guard_on && c->path == P_MAIN;
}

// The bucket counting kernels run only when the order kernel could not count the
// buckets itself (pairs from the radix engine or the pair sort, or M too large).
__device__ __forceinline__ bool guard_general(const Ctrl* c) {
    return c->guard_on && c->guard_general && c->path == P_MAIN;
}

// In general mode the contested keys are found from the input through a hash
// index (key -> position in the dense keys, verified against them) kept in the
// radix scratch, sized for all K keys; 0 when the scratch still holds the sorted
// column (in place after the radix engine) or is too small: then binary search.
__device__ __forceinline__ uint32_t guard_index_log2(const Args& a, const Ctrl* c) {
    if (c->deferred_copy) return 0;
    const uint32_t lg = log2_pow2(bit_ceil64(2 * c->K > 64 ? 2 * c->K : 64));
    return (1ull << lg) <= 2 * (a.n + 2) ? lg : 0;  // the scratch holds 2 (n + 2) 32-bit words
}

__device__ __forceinline__ uint32_t* guard_index(const Args& a) { return reinterpret_cast<uint32_t*>(a.tmp_k); }

__device__ __forceinline__ void guard_prep_body(const Args& a, uint32_t bid, uint32_t nblk) {
    Ctrl* c = a.c;
    if (!guard_general(c)) return;
    const uint64_t M = c->table_M;
    const uint64_t gtid = (uint64_t)bid * blockDim.x + threadIdx.x;
    const uint64_t gstride = (uint64_t)nblk * blockDim.x;
    for (uint64_t i = gtid; i < M; i += gstride) {
        a.dcount[i] = 0;
        for (uint32_t r = 0; r < a.cap; ++r) a.bmin[r * a.m_ws + i] = kNoIndex;
    }
    const uint32_t lg = guard_index_log2(a, c);
    if (gtid == 0) c->gidx_log2 = lg;
    if (lg) {
        CAFS_GLOBAL uint32_t* tab = gp(guard_index(a));
        for (uint64_t i = gtid; i < (1ull << lg); i += gstride) tab[i] = kNoIndex;
    }
}
CAFS_KERNELS0(guard_prep, 256)

__device__ __forceinline__ void guard_bucket_body(const Args& a, uint32_t bid, uint32_t nblk) {
    const Ctrl* c = a.c;
    if (!guard_general(c)) return;
    const uint64_t K = c->K;
    const uint32_t lg = log2_pow2(c->table_M);
    const uint64_t gtid = (uint64_t)bid * blockDim.x + threadIdx.x;
    const uint64_t gstride = (uint64_t)nblk * blockDim.x;
    for (uint64_t j = gtid; j < K; j += gstride) atomicAdd(&a.dcount[phi_hash(a.uniq[j], lg)], 1u);
}
CAFS_KERNELS0(guard_bucket, 256)

// Lists the contested keys (general mode) and resets their first-occurrence
// minima.
__device__ __forceinline__ void guard_mark_body(const Args& a, uint32_t bid, uint32_t nblk) {
    Ctrl* c = a.c;
    if (!guard_active(c)) return;
    const uint64_t gtid = (uint64_t)bid * blockDim.x + threadIdx.x;
    const uint64_t gstride = (uint64_t)nblk * blockDim.x;
    const uint64_t M = c->table_M;
    uint32_t nb = 0;
    for (uint64_t b = gtid; b < M; b += gstride) {
        a.bfound[b] = 0;
        if (c->guard_general) nb += a.dcount[b] > a.cap;
    }
    nb = wave_sum_u32(nb);
    if (__lane_id() == 0 && nb) atomicAdd((unsigned long long*)&c->n_cbuckets, (unsigned long long)nb);
    if (c->guard_general) {
        const uint64_t K = c->K;
        const uint32_t lg = log2_pow2(c->table_M);
        const uint32_t glg = c->gidx_log2;
        uint32_t* tab = guard_index(a);
        for (uint64_t j = gtid; j < K; j += gstride) {
            const bool cont = a.dcount[phi_hash(a.uniq[j], lg)] > a.cap;
            // list places: one update of the shared counter per wave (one per key
            // serialised on its address)
            const uint64_t m = __ballot(cont);
            if (m == 0) continue;
            const uint32_t leader = (uint32_t)__builtin_ctzll(m);
            uint32_t base = 0;
            if (__lane_id() == leader)
                base = (uint32_t)atomicAdd((unsigned long long*)&c->n_contested, (unsigned long long)__popcll(m));
            base = __shfl(base, leader, 64);
            if (!cont) continue;
            a.first_idx[j] = kNoIndex;
            a.clist[base + __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u))] =
                (uint32_t)j;
            if (glg) {  // index the contested key: linear probing on 32-bit slots
                uint64_t h = phi_hash(a.uniq[j], glg);
                while (atomicCAS(&tab[h], kNoIndex, (uint32_t)j) != kNoIndex) h = (h + 1) & ((1ull << glg) - 1);
            }
        }
    } else {
        const uint64_t nc = c->n_contested;
        for (uint64_t li = gtid; li < nc; li += gstride) a.first_idx[a.clist[li]] = kNoIndex;
    }
}
CAFS_KERNELS0(guard_mark, 256)

// Position of key v in the sorted distinct keys (it is present).
__device__ __forceinline__ uint64_t find_key(const uint64_t* uq, uint64_t K, uint64_t v, uint64_t flip,
                                             uint64_t fneg) {
    uint64_t lo = 0, hi = K - 1;
    const uint64_t ov = okey(v, flip, fneg);
    while (lo < hi) {
        const uint64_t mid = lo + (hi - lo) / 2;
        if (okey(uq[mid], flip, fneg) < ov) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// Position of contested key v through the hash index (it is present), probing
// from slot h on.
__device__ __forceinline__ uint64_t index_probe(const Args& a, uint32_t glg, uint64_t v, uint64_t h) {
    const CAFS_GLOBAL uint32_t* tab = gp(guard_index(a));
    const CAFS_GLOBAL uint64_t* uq = gp(a.uniq);
    while (true) {
        const uint32_t j = tab[h];
        if (j == kNoIndex || uq[j] == v) return j;  // kNoIndex is unreachable for a contested key
        h = (h + 1) & ((1ull << glg) - 1);
    }
}

__device__ __forceinline__ uint64_t index_find(const Args& a, uint32_t glg, uint64_t v) {
    return index_probe(a, glg, v, phi_hash(v, glg));
}

// First occurrences of the contested keys.  Chunks of the input are claimed in
// increasing order and every claimed chunk is finished, so the minima found so far
// are exact for every key seen in a claimed chunk.  A workgroup stops claiming
// once every contested bucket has seen cap of its keys: a key first seen in a
// later chunk occurs after those and cannot be among the bucket's first cap,
// so its first occurrence (left at the maximum) does not change the spill.  With at
// most kGuardLdsKeys contested keys each workgroup keeps them in an LDS hash table
// with per-key minima that it merges into the global minima after each chunk;
// otherwise each element of a contested bucket is located through the hash index
// of the contested keys (binary search when there is none).  With kPhased (the
// batched kernel, where a column has few workgroups and each one's chain of
// dependent loads sets the launch's length) each lookup step of the general mode
// is taken for all of a thread's elements before the next step, so that their
// loads are in flight together; the single-column kernel keeps the element-wise
// loop, which shares the memory system better with the emit running beside it.
template <bool kPhased>
__device__ __forceinline__ void guard_first_body(const Args& a, uint32_t bid, uint32_t nblk) {
    Ctrl* c = a.c;
    if (c->path != P_MAIN || !c->guard_on) return;
    const uint64_t nc = c->n_contested;
    if (nc == 0) return;
    const uint64_t n = a.n;
    const uint64_t K = c->K;
    const uint64_t M = c->table_M;
    const uint32_t lg = log2_pow2(M);
    const uint64_t flip = a.flip;
    const uint32_t glg = c->guard_general ? c->gidx_log2 : 0;
    const uint64_t chunks = (n + kGuardChunk - 1) / kGuardChunk;
    constexpr uint32_t TS = 2 * kGuardLdsKeys;  // LDS table slots
    __shared__ uint64_t tkey[TS];
    __shared__ uint16_t tidx[TS];
    __shared__ uint32_t lmin[kGuardLdsKeys];
    __shared__ uint32_t lsent[kGuardLdsKeys];
    __shared__ uint32_t bflag[kGuardLdsBuckets / 32];  // contested-bucket bitmap when M is small
    __shared__ uint32_t s_chunk, s_stop;
    const bool small = nc <= kGuardLdsKeys;
    const bool bits = small && M <= kGuardLdsBuckets;  // bitmap built with the LDS table
    if (small) {
        for (uint32_t i = threadIdx.x; i < TS; i += blockDim.x) tkey[i] = kEmpty;
        for (uint32_t i = threadIdx.x; i < nc; i += blockDim.x) { lmin[i] = kNoIndex; lsent[i] = kNoIndex; }
        if (bits)
            for (uint32_t i = threadIdx.x; i < kGuardLdsBuckets / 32; i += blockDim.x) bflag[i] = 0;
        __syncthreads();
        for (uint32_t li = threadIdx.x; li < nc; li += blockDim.x) {
            const uint64_t key = a.uniq[a.clist[li]];
            if (bits) {
                const uint32_t b = phi_hash32(key, lg);
                atomicOr(&bflag[b >> 5], 1u << (b & 31));
            }
            // keys are distinct, so claiming the first empty slot never races with an equal key
            uint32_t h = phi_hash32(key, 12);
            while (true) {
                const unsigned long long old =
                    atomicCAS((unsigned long long*)&tkey[h], (unsigned long long)kEmpty, (unsigned long long)key);
                if (old == kEmpty) { tidx[h] = (uint16_t)li; break; }
                h = (h + 1) & (TS - 1);
            }
        }
        __syncthreads();
    }
    // Every key of a contested bucket is contested.  The LDS table cannot hold a key
    // equal to its empty marker; such a key takes the binary-search path.
    while (true) {
        if (threadIdx.x == 0) {
            s_stop = atomic_load_agent(&c->buckets_done) >= c->n_cbuckets;
            s_chunk = s_stop ? 0 : atomicAdd(&c->chunk_ctr, 1u);
        }
        __syncthreads();
        const uint64_t ch = s_chunk;
        const bool stop = s_stop || ch >= chunks;
        __syncthreads();
        if (stop) break;
        const uint64_t b0 = ch * kGuardChunk;
        const uint64_t e0 = (b0 + kGuardChunk < n) ? b0 + kGuardChunk : n;
        uint32_t newly = 0;
        // the chunk's elements are loaded first (all in flight), then looked up; a
        // key whose first position is already known to be earlier is skipped before
        // the atomic (a frequent key would otherwise serialise on one address; a
        // stale read is only ever larger, so the skip is safe)
        constexpr uint32_t PER = kGuardChunk / 256;  // workgroups of 256 threads
        uint64_t vv[PER];
#pragma unroll
        for (uint32_t u = 0; u < PER; ++u) {
            const uint64_t i = b0 + threadIdx.x + (uint64_t)u * blockDim.x;
            vv[u] = i < e0 ? load_key(a.in, i, a.ew) : 0;
        }
        if (kPhased && !small) {
            const CAFS_GLOBAL uint32_t* tab = gp(guard_index(a));
            const uint64_t imask = glg ? (1ull << glg) - 1 : 0;
            uint32_t bb[PER], dc[PER], jt[PER];
#pragma unroll
            for (uint32_t u = 0; u < PER; ++u) {
                const uint64_t i = b0 + threadIdx.x + (uint64_t)u * blockDim.x;
                bb[u] = phi_hash32(vv[u], lg);
                dc[u] = i < e0 ? a.dcount[bb[u]] : 0u;
            }
            if (glg) {
#pragma unroll
                for (uint32_t u = 0; u < PER; ++u) jt[u] = dc[u] > a.cap ? tab[phi_hash(vv[u], glg)] : kNoIndex;
                uint64_t kk[PER];
#pragma unroll
                for (uint32_t u = 0; u < PER; ++u) kk[u] = jt[u] != kNoIndex ? a.uniq[jt[u]] : 0;
#pragma unroll
                for (uint32_t u = 0; u < PER; ++u)
                    if (jt[u] != kNoIndex && kk[u] != vv[u])  // not in its home slot: probe on
                        jt[u] = (uint32_t)index_probe(a, glg, vv[u], (phi_hash(vv[u], glg) + 1) & imask);
            } else {
#pragma unroll
                for (uint32_t u = 0; u < PER; ++u)
                    jt[u] = dc[u] > a.cap ? (uint32_t)find_key(a.uniq, K, vv[u], flip, a.fneg) : kNoIndex;
            }
            uint32_t fi[PER];
#pragma unroll
            for (uint32_t u = 0; u < PER; ++u) fi[u] = jt[u] < K ? g_load(&a.first_idx[jt[u]]) : 0u;
#pragma unroll
            for (uint32_t u = 0; u < PER; ++u) {
                const uint64_t i = b0 + threadIdx.x + (uint64_t)u * blockDim.x;
                if (jt[u] >= K || fi[u] <= (uint32_t)i) continue;
                const uint32_t old = atomicMin(&a.first_idx[jt[u]], (uint32_t)i);
                if (old == kNoIndex && atomicAdd(&a.bfound[bb[u]], 1u) == a.cap - 1) ++newly;
            }
        } else {
#pragma unroll
        for (uint32_t u = 0; u < PER; ++u) {
            const uint64_t i = b0 + threadIdx.x + (uint64_t)u * blockDim.x;
            if (i >= e0) continue;
            const uint64_t v = vv[u];
            const uint32_t b = phi_hash32(v, lg);
            const bool cont = bits ? ((bflag[b >> 5] >> (b & 31)) & 1u) : (a.dcount[b] > a.cap);
            if (!cont) continue;
            if (small && v != kEmpty) {
                uint32_t h = phi_hash32(v, 12);
                while (true) {
                    const uint64_t tk = tkey[h];
                    if (tk == v) {
                        const uint32_t li = tidx[h];
                        if (lmin[li] > (uint32_t)i) atomicMin(&lmin[li], (uint32_t)i);
                        break;
                    }
                    if (tk == kEmpty) break;  // unreachable: contested keys are all in the table
                    h = (h + 1) & (TS - 1);
                }
            } else if (bits || a.dcount[b] > a.cap) {
                const uint64_t jj = glg ? index_find(a, glg, v) : find_key(a.uniq, K, v, flip, a.fneg);
                if (jj >= K) continue;  // not reached: every key of a contested bucket is indexed
                if (g_load(&a.first_idx[jj]) <= (uint32_t)i) continue;
                const uint32_t old = atomicMin(&a.first_idx[jj], (uint32_t)i);
                if (old == kNoIndex && atomicAdd(&a.bfound[b], 1u) == a.cap - 1) ++newly;
            }
        }
        }
        if (small) {
            __syncthreads();
            for (uint32_t li = threadIdx.x; li < nc; li += blockDim.x) {
                const uint32_t m = lmin[li];
                if (m < lsent[li]) {
                    lsent[li] = m;
                    const uint32_t j = a.clist[li];
                    const uint32_t old = atomicMin(&a.first_idx[j], m);
                    if (old == kNoIndex && atomicAdd(&a.bfound[phi_hash32(a.uniq[j], lg)], 1u) == a.cap - 1)
                        ++newly;
                }
            }
        }
        newly = wave_sum_u32(newly);  // buckets that now know cap keys
        if (__lane_id() == 0 && newly)
            atomicAdd((unsigned long long*)&c->buckets_done, (unsigned long long)newly);
        __syncthreads();
    }
}
__global__ __launch_bounds__(256) void k_guard_first(Args a) { guard_first_body<false>(a, blockIdx.x, gridDim.x); }
__global__ __launch_bounds__(256) void kb_guard_first(BatchGrid g) {
    const uint32_t col = g.col[blockIdx.x];
    guard_first_body<true>(g.args[col], blockIdx.x - g.first[col], g.count[col]);
}

// Rank of each contested key within its bucket by first occurrence, for at most
// kGuardLdsKeys contested keys: sort (bucket, first occurrence) in LDS; position p
// is past the bucket's first cap keys (cap = 4, or 8 for 32-bit keys) exactly when
// position p - cap holds the same bucket.  The spill is the sum of those keys'
// counts.  One workgroup.
__device__ __forceinline__ void guard_resolve_body(const Args& a, uint32_t bid, uint32_t nblk) {
    Ctrl* c = a.c;
    if (c->path != P_MAIN || !c->guard_on) return;
    const uint64_t nc = c->n_contested;
    if (nc == 0) return;
    if (nc > kGuardLdsKeys) {
        if (threadIdx.x == 0) c->guard_rounds = 1;
        return;
    }
    __shared__ uint64_t sk[kGuardLdsKeys];
    __shared__ uint64_t sv[kGuardLdsKeys];
    __shared__ unsigned long long s_spill;
    const uint32_t lg = log2_pow2(c->table_M);
    uint32_t P = 64;
    while (P < nc) P <<= 1;
    for (uint32_t i = threadIdx.x; i < P; i += blockDim.x) {
        if (i < nc) {
            const uint32_t j = a.clist[i];
            sk[i] = ((uint64_t)phi_hash32(a.uniq[j], lg) << 32) | a.first_idx[j];
            sv[i] = a.cnt[j];
        } else {
            sk[i] = ~0ull;
            sv[i] = 0;
        }
    }
    if (threadIdx.x == 0) s_spill = 0;
    __syncthreads();
    // keys are distinct (distinct first occurrences), padding sorts last
    for (uint32_t kk = 2; kk <= P; kk <<= 1) {
        for (uint32_t jj = kk >> 1; jj > 0; jj >>= 1) {
            for (uint32_t i = threadIdx.x; i < P; i += blockDim.x) {
                const uint32_t l = i ^ jj;
                if (l > i) {
                    const uint64_t ki = sk[i], kl = sk[l];
                    const bool up = (i & kk) == 0;
                    if (up == (ki > kl)) {
                        sk[i] = kl; sk[l] = ki;
                        const uint64_t t = sv[i]; sv[i] = sv[l]; sv[l] = t;
                    }
                }
            }
            __syncthreads();
        }
    }
    unsigned long long local = 0;
    for (uint32_t p = threadIdx.x; p < nc; p += blockDim.x)
        if (p >= a.cap && (sk[p - a.cap] >> 32) == (sk[p] >> 32)) local += sv[p];
    local = wave_sum_u64(local);
    if (__lane_id() == 0 && local) atomicAdd(&s_spill, local);
    __syncthreads();
    if (threadIdx.x == 0) {
        c->spill = s_spill;
        c->flags |= 2u;
        if (2 * s_spill > a.n) c->path = P_GUARD;
    }
}
CAFS_KERNELS0(guard_resolve, 1024)

// Round r (r < cap, one launch each): the r-th smallest first occurrence per bucket.
__device__ __forceinline__ void guard_round_body(const Args& a, uint32_t r, uint32_t bid, uint32_t nblk) {
    const Ctrl* c = a.c;
    if (!guard_active(c) || !c->guard_rounds || r >= a.cap) return;
    // The rounds run in general mode only, where the contested list holds every key
    // of an over-full bucket: walk it (not all K keys), four keys per thread with
    // their loads in flight together.
    const uint64_t nc = c->n_contested;
    const uint32_t lg = log2_pow2(c->table_M);
    const uint64_t gtid = (uint64_t)bid * blockDim.x + threadIdx.x;
    const uint64_t gstride = (uint64_t)nblk * blockDim.x;
    constexpr uint32_t U = 4;
    for (uint64_t l0 = gtid; l0 < nc; l0 += U * gstride) {
        uint32_t j[U], b[U], f[U], pm[U];
#pragma unroll
        for (uint32_t u = 0; u < U; ++u) j[u] = l0 + u * gstride < nc ? a.clist[l0 + u * gstride] : 0u;
#pragma unroll
        for (uint32_t u = 0; u < U; ++u) {
            const bool in = l0 + u * gstride < nc;
            b[u] = in ? phi_hash(a.uniq[j[u]], lg) : 0u;
            f[u] = in ? a.first_idx[j[u]] : 0u;
        }
#pragma unroll
        for (uint32_t u = 0; u < U; ++u) pm[u] = (r > 0 && l0 + u * gstride < nc) ? a.bmin[(r - 1) * a.m_ws + b[u]] : 0u;
#pragma unroll
        for (uint32_t u = 0; u < U; ++u)
            if (l0 + u * gstride < nc && (r == 0 || f[u] > pm[u])) atomicMin(&a.bmin[r * a.m_ws + b[u]], f[u]);
    }
}
CAFS_KERNELS1(guard_round, 256, uint32_t, r)

__device__ __forceinline__ void guard_final_body(const Args& a, uint32_t bid, uint32_t nblk) {
    Ctrl* c = a.c;
    if (!guard_active(c) || !c->guard_rounds) return;
    __shared__ uint32_t s_last;
    const uint32_t lg = log2_pow2(c->table_M);
    const uint64_t gtid = (uint64_t)bid * blockDim.x + threadIdx.x;
    const uint64_t gstride = (uint64_t)nblk * blockDim.x;
    // (the contested list, as in the rounds)
    const uint64_t nc = c->n_contested;
    constexpr uint32_t U = 4;
    uint64_t local = 0;
    for (uint64_t l0 = gtid; l0 < nc; l0 += U * gstride) {
        uint32_t j[U], b[U], f[U], m4[U];
#pragma unroll
        for (uint32_t u = 0; u < U; ++u) j[u] = l0 + u * gstride < nc ? a.clist[l0 + u * gstride] : 0u;
#pragma unroll
        for (uint32_t u = 0; u < U; ++u) {
            const bool in = l0 + u * gstride < nc;
            b[u] = in ? phi_hash(a.uniq[j[u]], lg) : 0u;
            f[u] = in ? a.first_idx[j[u]] : 0u;
        }
#pragma unroll
        for (uint32_t u = 0; u < U; ++u) m4[u] = l0 + u * gstride < nc ? a.bmin[(a.cap - 1) * a.m_ws + b[u]] : kNoIndex;
#pragma unroll
        for (uint32_t u = 0; u < U; ++u)
            if (l0 + u * gstride < nc && f[u] > m4[u]) local += a.cnt[j[u]];
    }
    local = wave_sum_u64(local);
    if (__lane_id() == 0 && local) atomicAdd((unsigned long long*)&c->spill, (unsigned long long)local);
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) s_last = (atomicAdd(&c->guard_done, 1u) == nblk - 1);
    __syncthreads();
    if (!s_last || threadIdx.x != 0) return;
    __threadfence();
    const uint64_t spill = atomic_load_agent(&c->spill);
    if (c->n_contested) c->flags |= 2u;
    if (2 * spill > a.n) c->path = P_GUARD;
}
CAFS_KERNELS0(guard_final, 256)

}  // namespace cafs
