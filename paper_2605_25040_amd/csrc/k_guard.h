// Exact spill of the paper's bucket table, computed from the (key, count) pairs.
//
// In Alg. 1 a bucket never evicts and its counters only grow, so a bucket keeps
// the first four distinct keys that hash to it (Eq. hash over M buckets, Eq.
// Msize) in order of first occurrence, and every occurrence of any later key of
// that bucket goes to the spill (counted in elements; the RLE step of Sec. 4.4
// does not change that count).  Hence
//     |spill| = sum over buckets with more than 4 distinct keys of the counts of
//               the keys whose first occurrence is not among the bucket's first four.
// The guard of Alg. 4 fires when |spill| > N/2 (tested as 2 |spill| > N).
//
// The GPU computes it in these steps, all skipped when no bucket is over-full:
//   k_guard_prep    clear bucket counters and the four per-bucket minima
//   k_guard_bucket  distinct keys per bucket
//   k_guard_mark    count the keys of over-full ("contested") buckets
//   k_guard_first   first occurrence of each contested key: one pass over the
//                   input in increasing chunks that stops once every contested
//                   key has been seen (later chunks cannot hold a first occurrence)
//   k_guard_round   r = 0..3: the r-th smallest first occurrence of each bucket
//   k_guard_final   sum the counts of keys later than the 4th, decide the path
#pragma once
#include "cafs_dev.h"

namespace cafs {

constexpr uint32_t kNoIndex = 0xFFFFFFFFu;

__device__ __forceinline__ bool guard_active(const Ctrl* c) {
    return c->guard_on && c->path == P_MAIN;
}

__global__ __launch_bounds__(256) void k_guard_prep(Args a) {
    const Ctrl* c = a.c;
    if (!guard_active(c)) return;
    const uint64_t M = c->table_M;
    const uint64_t gtid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t gstride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = gtid; i < M; i += gstride) {
        a.dcount[i] = 0;
        for (int r = 0; r < 4; ++r) a.bmin[r * a.m_ws + i] = kNoIndex;
    }
}

__global__ __launch_bounds__(256) void k_guard_bucket(Args a) {
    const Ctrl* c = a.c;
    if (!guard_active(c)) return;
    const uint64_t K = c->K;
    const uint32_t lg = log2_pow2(c->table_M);
    const uint64_t gtid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t gstride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t j = gtid; j < K; j += gstride) atomicAdd(&a.dcount[phi_hash(a.uniq[j], lg)], 1u);
}

__global__ __launch_bounds__(256) void k_guard_mark(Args a) {
    Ctrl* c = a.c;
    if (!guard_active(c)) return;
    const uint64_t K = c->K;
    const uint32_t lg = log2_pow2(c->table_M);
    const uint64_t gtid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t gstride = (uint64_t)gridDim.x * blockDim.x;
    uint32_t local = 0;
    for (uint64_t j = gtid; j < K; j += gstride) {
        a.first_idx[j] = kNoIndex;
        local += a.dcount[phi_hash(a.uniq[j], lg)] > kBucketCap;
    }
    local = wave_sum_u32(local);
    if (__lane_id() == 0 && local) atomicAdd((unsigned long long*)&c->n_contested, (unsigned long long)local);
}

// Position of key v in the sorted distinct keys (it is present).
__device__ __forceinline__ uint64_t find_key(const uint64_t* uq, uint64_t K, uint64_t v, uint64_t flip) {
    uint64_t lo = 0, hi = K - 1;
    const uint64_t ov = v ^ flip;
    while (lo < hi) {
        const uint64_t mid = lo + (hi - lo) / 2;
        if ((uq[mid] ^ flip) < ov) lo = mid + 1; else hi = mid;
    }
    return lo;
}

__global__ __launch_bounds__(256) void k_guard_first(Args a) {
    Ctrl* c = a.c;
    if (!guard_active(c)) return;
    const uint64_t nc = c->n_contested;
    if (nc == 0) return;
    const uint64_t n = a.n;
    const uint64_t K = c->K;
    const uint32_t lg = log2_pow2(c->table_M);
    const uint64_t chunks = (n + kGuardChunk - 1) / kGuardChunk;
    __shared__ uint32_t s_chunk;
    __shared__ uint32_t s_stop;
    while (true) {
        if (threadIdx.x == 0) {
            s_stop = atomic_load_agent(&c->found) >= nc;
            s_chunk = s_stop ? 0 : atomicAdd(&c->chunk_ctr, 1u);
        }
        __syncthreads();
        const uint64_t ch = s_chunk;
        const bool stop = s_stop || ch >= chunks;
        __syncthreads();
        if (stop) break;
        const uint64_t b = ch * kGuardChunk;
        const uint64_t e = (b + kGuardChunk < n) ? b + kGuardChunk : n;
        uint32_t newly = 0;
        for (uint64_t i = b + threadIdx.x; i < e; i += blockDim.x) {
            const uint64_t v = a.in[i];
            if (a.dcount[phi_hash(v, lg)] > kBucketCap) {
                const uint64_t jj = find_key(a.uniq, K, v, a.flip);
                const uint32_t old = atomicMin(&a.first_idx[jj], (uint32_t)i);
                newly += (old == kNoIndex);
            }
        }
        newly = wave_sum_u32(newly);
        if (__lane_id() == 0 && newly) atomicAdd((unsigned long long*)&c->found, (unsigned long long)newly);
    }
}

__global__ __launch_bounds__(256) void k_guard_round(Args a, uint32_t r) {
    const Ctrl* c = a.c;
    if (!guard_active(c) || c->n_contested == 0) return;
    const uint64_t K = c->K;
    const uint32_t lg = log2_pow2(c->table_M);
    const uint64_t gtid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t gstride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t j = gtid; j < K; j += gstride) {
        const uint32_t b = phi_hash(a.uniq[j], lg);
        if (a.dcount[b] <= kBucketCap) continue;
        const uint32_t f = a.first_idx[j];
        if (r == 0 || f > a.bmin[(r - 1) * a.m_ws + b]) atomicMin(&a.bmin[r * a.m_ws + b], f);
    }
}

__global__ __launch_bounds__(256) void k_guard_final(Args a) {
    Ctrl* c = a.c;
    if (!guard_active(c)) return;
    __shared__ uint32_t s_last;
    const uint64_t K = c->K;
    const uint32_t lg = log2_pow2(c->table_M);
    const uint64_t gtid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t gstride = (uint64_t)gridDim.x * blockDim.x;
    uint64_t local = 0;
    if (c->n_contested) {
        for (uint64_t j = gtid; j < K; j += gstride) {
            const uint32_t b = phi_hash(a.uniq[j], lg);
            if (a.dcount[b] > kBucketCap && a.first_idx[j] > a.bmin[3 * a.m_ws + b]) local += a.cnt[j];
        }
    }
    local = wave_sum_u64(local);
    if (__lane_id() == 0 && local) atomicAdd((unsigned long long*)&c->spill, (unsigned long long)local);
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) s_last = (atomicAdd(&c->guard_done, 1u) == gridDim.x - 1);
    __syncthreads();
    if (!s_last || threadIdx.x != 0) return;
    __threadfence();
    const uint64_t spill = atomic_load_agent(&c->spill);
    if (c->n_contested) c->flags |= 2u;
    if (2 * spill > a.n) c->path = P_GUARD;
}

}  // namespace cafs
