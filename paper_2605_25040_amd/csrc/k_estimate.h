// Estimate, order check, plan and report kernels.
#pragma once
#include "cafs_dev.h"

namespace cafs {

// Chao1 over strided samples (Sec. 4.3, Alg. 2, Eq. chao1), one workgroup.
//   stride = max(1, floor(N/1024)), samples at 0, stride, ... below min(N, 1024*stride),
//   i.e. min(N, 1024) samples; a 4096-slot open-addressing FreqSet in LDS counts them;
//   u, f1, f2 are read from the slot counters; K^ = N when u = 1024, else
//   u + floor(f1^2 / (2 (f2 + 1))).
// The FreqSet uses kEmpty as its empty marker; samples equal to kEmpty are counted
// in a separate LDS counter, which acts as one more slot.  When u <= 8 the distinct
// sampled keys are returned too, sorted in the dtype's order (tiny branch).
// Every thread must call it, passing the sample it loaded (chao1_sample) so that
// the load's latency overlaps other work; thread 0's outputs are the results.
struct Chao1Result {
    uint64_t k_hat, u, f1, f2, n_samples, stride;
    uint32_t saturated, n_small;
    uint64_t small[8];
};

// Sample threadIdx.x of the column of `ew`-byte keys (0 when there is none):
// element tid * stride.
__device__ __forceinline__ uint64_t chao1_sample(const uint64_t* x, uint64_t n, uint32_t ew) {
    const uint64_t stride = n / kSamples > 1 ? n / kSamples : 1;
    const uint64_t ns = n < kSamples ? n : kSamples;
    return threadIdx.x < ns ? load_key(x, threadIdx.x * stride, ew) : 0;
}

__device__ void chao1_block(uint64_t v_mine, uint64_t n, uint64_t flip, uint64_t fneg, Chao1Result* res) {
    __shared__ uint64_t fkeys[1u << kFreqSlotsLog2];
    __shared__ uint32_t fcnt[1u << kFreqSlotsLog2];
    __shared__ uint32_t s_e, s_u, s_f1, s_f2, s_ns;
    __shared__ uint64_t s_small[9];
    const uint32_t tid = threadIdx.x;
    const uint32_t slots = 1u << kFreqSlotsLog2;
    for (uint32_t i = tid; i < slots; i += blockDim.x) {
        fkeys[i] = kEmpty;
        fcnt[i] = 0;
    }
    if (tid == 0) { s_e = 0; s_u = 0; s_f1 = 0; s_f2 = 0; s_ns = 0; }
    __syncthreads();
    const uint64_t stride = n / kSamples > 1 ? n / kSamples : 1;
    const uint64_t ns = n < kSamples ? n : kSamples;
    // one sample per thread (blockDim.x >= kSamples)
    if (tid < ns) {
        const uint64_t v = v_mine;
        if (v == kEmpty) {
            atomicAdd(&s_e, 1u);
        } else {
            uint32_t h = phi_hash(v, kFreqSlotsLog2);
            while (true) {
                const uint64_t k = fkeys[h];
                if (k == v) { atomicAdd(&fcnt[h], 1u); break; }
                if (k == kEmpty) {
                    const unsigned long long old =
                        atomicCAS((unsigned long long*)&fkeys[h], (unsigned long long)kEmpty,
                                  (unsigned long long)v);
                    if (old == kEmpty || old == v) { atomicAdd(&fcnt[h], 1u); break; }
                }
                h = (h + 1) & (slots - 1);
            }
        }
    }
    __syncthreads();
    uint32_t lu = 0, l1 = 0, l2 = 0;
    for (uint32_t i = tid; i < slots; i += blockDim.x) {
        const uint32_t cn = fcnt[i];
        lu += cn > 0;
        l1 += cn == 1;
        l2 += cn == 2;
    }
    lu = wave_sum_u32(lu); l1 = wave_sum_u32(l1); l2 = wave_sum_u32(l2);
    if (__lane_id() == 0) {
        atomicAdd(&s_u, lu); atomicAdd(&s_f1, l1); atomicAdd(&s_f2, l2);
    }
    __syncthreads();
    uint32_t u = s_u + (s_e > 0);
    if (u <= kTinyK) {
        for (uint32_t i = tid; i < slots; i += blockDim.x)
            if (fcnt[i] > 0) s_small[atomicAdd(&s_ns, 1u)] = fkeys[i];
        __syncthreads();
        if (tid == 0 && s_e > 0) s_small[s_ns++] = kEmpty;
    }
    __syncthreads();
    if (tid == 0) {
        const uint64_t f1 = s_f1 + (s_e == 1);
        const uint64_t f2 = s_f2 + (s_e == 2);
        res->u = u;
        res->f1 = f1;
        res->f2 = f2;
        res->n_samples = ns;
        res->stride = stride;
        res->saturated = (u == kSamples);
        res->k_hat = res->saturated ? n : u + (f1 * f1) / (2 * (f2 + 1));
        uint32_t m = (u <= kTinyK) ? s_ns : 0;
        // insertion sort of at most 8 keys in the dtype's order
        for (uint32_t i = 0; i < m; ++i) {
            uint64_t v = s_small[i];
            uint32_t j = i;
            while (j > 0 && okey(s_small[j - 1], flip, fneg) > okey(v, flip, fneg)) { s_small[j] = s_small[j - 1]; --j; }
            s_small[j] = v;
        }
        res->n_small = m;
        for (uint32_t i = 0; i < m; ++i) res->small[i] = s_small[i];
    }
}

// Eq. Msize: M = bit_ceil(8 K^ / cap) clamped to [8, bit_ceil(N / cap)], cap = 4 for
// 64-bit keys and 8 for 32-bit keys.
__device__ __forceinline__ uint64_t paper_table_M(uint64_t k_hat, uint64_t n, uint32_t cap) {
    uint64_t m = bit_ceil64(8 * k_hat / cap);
    const uint64_t hi = bit_ceil64(n / cap);
    if (m > hi) m = hi;
    if (m < 8) m = 8;
    return m;
}

// Partition buckets: each a sixteenth more than its share of the column plus a
// scatter chunk, rounded to 32 elements (256 bytes); the rest of pbuf is the
// overflow area.  Shares are even, or `mass` (sampled elements per partition,
// summing to `total`) when given.  False when the buckets do not fit.
__device__ bool set_buckets(const Args& a, Ctrl* c, uint32_t pl, const uint32_t* mass, uint64_t total = 0) {
    const uint32_t P = 1u << pl;
    uint64_t at = 0;
    for (uint32_t q = 0; q < P; ++q) {
        const uint64_t share = mass ? (uint64_t)((double)a.n * mass[q] / (double)total) : (a.n >> pl);
        const uint64_t cap = (share + share / 16 + kScatterChunk + 31) / 32 * 32;
        c->pbase[q] = at;
        at += cap;
    }
    c->pbase[P] = at;
    if (at + a.n / 32 > a.pbuf_elems) return false;
    c->pbase[P + 1] = a.pbuf_elems / 32 * 32;
    return true;
}

// The hash count's geometry for an estimate kh of K: partitions of about part_keys
// estimated keys each (at most 2^kMaxPartLog2), LDS buckets of 4 keys when a
// partition's share reaches wide_min, a global table of table_slots kh slots (half
// of them may be claimed; keys past that spill).  Returns the engine: the radix
// engine when kh is more than the partitions' LDS tables or the global table hold
// (the estimate is close to K for flat frequencies, and there most elements of the
// keys beyond would spill).
__device__ uint32_t plan_count(const Args& a, Ctrl* c, uint64_t kh, uint32_t engine) {
    const uint64_t n = a.n;
    // (no partitions up to twice part_keys: one LDS table holds that many keys, and
    // partitions cost a scatter pass over the column)
    const uint64_t parts = kh <= 2 * a.part_keys ? 1 : (kh + a.part_keys - 1) / a.part_keys;
    uint32_t pl = parts <= 1 ? 0u : log2_pow2(bit_ceil64(parts));
    if (pl > kMaxPartLog2) pl = kMaxPartLog2;
    if (pl && !set_buckets(a, c, pl, nullptr)) pl = 0;
    c->part_log2 = pl;
    c->lds_wide = (kh >> pl) >= a.wide_min ? 1u : 0u;
    uint32_t lg = log2_pow2(bit_ceil64(a.table_slots * kh));
    if (lg < kMinTableLog2) lg = kMinTableLog2;
    const uint32_t floor_lg = kTableFloorLog2 < a.cap_ws_log2 ? kTableFloorLog2 : a.cap_ws_log2;
    if (lg < floor_lg) lg = floor_lg;
    if (lg > a.cap_ws_log2) lg = a.cap_ws_log2;
    if (kh > (a.part_keys << (kMaxPartLog2 + 1)) || 2 * kh > (1ull << a.cap_ws_log2)) engine = E_RADIX;
    c->cap_log2 = lg;
    c->cap_limit = (uint32_t)((1ull << lg) / 2);  // linear probing stays short up to half load
    return engine;
}

// Engine-dependent state: which later stages run, and the radix job (the column,
// or scratch when sorting in place on the main path).
__device__ void plan_engine_state(const Args& a, Ctrl* c, int32_t path, uint32_t engine) {
    c->engine = engine;
    c->radix_on = (engine == E_RADIX);
    c->guard_on = (path == P_MAIN && engine == E_RADIX);
    c->guard_general = c->guard_on;
    RadixJob& j = c->rj;
    j.src_k = a.in; j.src_v = a.vin;
    j.dst_k = a.out; j.dst_v = a.vout;
    j.tmp_k = a.tmp_k; j.tmp_v = a.spill_v;  // (the spill list is not used when the radix engine sorts the column)
    j.n = a.n;
    j.has_vals = a.vin ? 1u : 0u;
    j.n_active = 0;
    j.copy_mode = 0;
    j.src_ew = a.ew;
    j.dst_ew = a.ew;
    c->sorted = a.out;
    c->sorted_ew = a.ew;
    c->deferred_copy = 0;
    if (path == P_MAIN && engine == E_RADIX && a.in == a.out) {
        // in place on the main path: the guard still reads the input after the sort,
        // so sort into scratch (ping-pong with the dense key array, written later)
        j.dst_k = a.tmp_k;
        j.dst_ew = 8;
        j.tmp_k = a.uniq;
        c->sorted = a.tmp_k;
        c->sorted_ew = 8;
        c->deferred_copy = 1;
    }
}


// Dispatcher (Alg. 3): picks the path and the engine and resets the counters
// of the later stages.  Called by every thread of one workgroup once the order
// check is settled: by the pre kernel when its prefix already shows an inversion
// (or covers the column), else by the last workgroup of the full order check.
__device__ void plan_block(const Args& a) {
    Ctrl* c = a.c;
    const uint64_t n = a.n;
    for (uint32_t i = threadIdx.x; i < 8 * 256; i += blockDim.x) (&c->hist[0][0])[i] = 0;
    if (threadIdx.x != 0) return;
    const bool mono = (n <= 1) || !c->inversion;
    int32_t path;
    uint32_t engine;
    if (mono) { path = P_MONOTONE; engine = E_NONE; }
    else if (n < kSmallN) { path = P_SMALL_N; engine = E_RADIX; }
    else if (c->k_hat <= kTinyK && c->u <= kTinyK) { path = P_TINY; engine = E_TINY; }
    else if (2 * c->k_hat > n) { path = P_HIGH_K; engine = E_RADIX; }
    else { path = P_MAIN; engine = E_HASH; }
    c->table_M = 0;
    c->cap_log2 = kMinTableLog2;
    c->part_log2 = 0;
    c->lds_wide = 0;
    if (path == P_TINY || path == P_MAIN) {
        c->table_M = paper_table_M(c->k_hat, n, a.cap);
        engine = plan_count(a, c, c->k_hat, engine);
    }
    c->nspill = 0;
    c->spill_limit = n / kSpillFracDiv;
    for (uint32_t q = 0; q <= kMaxParts; ++q) c->pfill[q][0] = 0;
    c->path = path;
    c->engine = engine;
    c->tiny_miss = 0;
    c->flags = 0;
    for (int j = 0; j < 8; ++j) { c->tiny_cnt[j][0] = 0; c->tile_ctr[j] = 0; }
    c->overflow = 0;
    c->claimed = 0;
    c->closed = 0;
    c->ecount = 0;
    c->K = 0;
    c->emit_main = 0;
    c->dense_ready = 0;
    c->pair_sort = 0;
    c->guard_rounds = 0;
    c->hist_done = 0;
    c->rle_done = 0;
    c->rle_on = 0;
    c->n_contested = 0;
    c->gidx_log2 = 0;
    c->n_cbuckets = 0;
    c->buckets_done = 0;
    c->found = 0;
    c->chunk_ctr = 0;
    c->guard_done = 0;
    c->spill = 0;
    // (not after a full order check: the set is cleared beside that check)
    c->replan = (path == P_MAIN && engine == E_HASH && n >= kReplanMinN && c->f1 >= kReplanMinF1 && !c->mono_full)
                    ? 1u : 0u;
    c->s2done = 0;
    plan_engine_state(a, c, path, engine);
}

// First kernel of a sort: order check of a prefix and the Chao1 estimate.
__device__ __forceinline__ void pre_body(const Args& a, uint32_t bid, uint32_t nblk) {
    Ctrl* c = a.c;
    __shared__ uint32_t s_inv;
    __shared__ Chao1Result s_res;
    // the sample and the order-check prefix are loaded together, so that their
    // latencies overlap
    const uint64_t v_sample = chao1_sample(a.in, a.n, a.ew);
    if (threadIdx.x == 0) s_inv = 0;
    __syncthreads();
    const uint64_t lim = a.n < kMonoPrefix ? a.n : kMonoPrefix;
    uint32_t inv = 0;
    constexpr uint32_t kPer = kMonoPrefix / 1024;  // elements per thread (blockDim.x = 1024)
    uint64_t pv[kPer + 1];
#pragma unroll
    for (uint32_t k = 0; k <= kPer; ++k) {
        const uint64_t i = (uint64_t)threadIdx.x * kPer + k;
        pv[k] = i < lim ? okey(load_key(a.in, i, a.ew), a.flip, a.fneg) : 0;
    }
#pragma unroll
    for (uint32_t k = 0; k < kPer; ++k) {
        const uint64_t i = (uint64_t)threadIdx.x * kPer + k;
        inv |= (i + 1 < lim && pv[k] > pv[k + 1]) ? 1u : 0u;
    }
    if (inv) s_inv = 1;
    chao1_block(v_sample, a.n, a.flip, a.fneg, &s_res);  // contains __syncthreads
    const bool settled = s_inv || a.n <= kMonoPrefix;
    if (threadIdx.x == 0) {
        c->inversion = s_inv;
        c->mono_full = settled ? 0u : 1u;
        c->mono_done = 0;
        c->k_hat = s_res.k_hat; c->u = s_res.u; c->f1 = s_res.f1; c->f2 = s_res.f2;
        c->n_samples = s_res.n_samples; c->stride = s_res.stride;
        c->saturated = s_res.saturated;
        c->n_tiny = s_res.n_small;
        for (uint32_t i = 0; i < 8; ++i) c->tiny_keys[i] = i < s_res.n_small ? s_res.small[i] : 0;
    }
    if (settled) {
        __syncthreads();
        plan_block(a);
    }
}
CAFS_KERNELS0(pre, 1024)

// Standalone estimate (cafs_estimate) of a column of `ew`-byte keys.
__global__ __launch_bounds__(1024) void k_estimate_only(const uint64_t* x, uint64_t n, uint32_t ew,
                                                        cafs_estimate_t* out) {
    __shared__ Chao1Result s_res;
    chao1_block(chao1_sample(x, n, ew), n, 0, 0, &s_res);
    if (threadIdx.x == 0) {
        cafs_estimate_t e;
        e.k_hat = s_res.k_hat; e.u = s_res.u; e.f1 = s_res.f1; e.f2 = s_res.f2;
        e.n_samples = s_res.n_samples; e.stride = s_res.stride;
        e.saturated = s_res.saturated; e.pad = 0;
        *out = e;
    }
}

// The larger sample (engine planning for long heavy-tailed columns) is counted in
// a hash set in the deferral scratch, free until the count: keys at tmp_k[0, S),
// 32-bit counts after them.  The full order check's workgroups clear it when the
// prefix already settled the order (the only case that plans from that sample).
__device__ __forceinline__ uint32_t* sample2_counts(const Args& a) {
    return reinterpret_cast<uint32_t*>(a.tmp_k + (1ull << kSample2SlotsLog2));
}
// Rows of the per-workgroup sums (3 + kMaxParts words each), after the counts.
__device__ __forceinline__ uint32_t* sample2_rows(const Args& a) {
    return sample2_counts(a) + (1u << kSample2SlotsLog2);
}
__device__ __forceinline__ void sample2_clear(const Args& a, uint32_t bid, uint32_t nblk) {
    const uint32_t S = 1u << kSample2SlotsLog2;
    uint32_t* cnt = sample2_counts(a);
    for (uint32_t i = bid * blockDim.x + threadIdx.x; i < S; i += nblk * blockDim.x) {
        gp(a.tmp_k)[i] = kEmpty;
        gp(cnt)[i] = 0;
    }
}

// Full order check, only when the prefix was in order (IsMonotone, Alg. 3).  Exits
// early once any workgroup has found an inversion.
__device__ __forceinline__ void mono_full_body(const Args& a, uint32_t bid, uint32_t nblk) {
    Ctrl* c = a.c;
    if (!c->mono_full) {
        if (c->replan) sample2_clear(a, bid, nblk);
        return;
    }
    const uint64_t n = a.n;
    const uint64_t chunk = 256 * 16;
    __shared__ uint32_t s_stop, s_last;
    for (uint64_t base = (uint64_t)bid * chunk; base + 1 < n; base += (uint64_t)nblk * chunk) {
        if (threadIdx.x == 0) s_stop = atomic_load_agent(&c->inversion);
        __syncthreads();
        if (s_stop) break;
        uint32_t inv = 0;
        const uint64_t end = (base + chunk < n - 1) ? base + chunk : n - 1;  // pairs (i, i+1), i < end
        for (uint64_t i = base + threadIdx.x; i < end; i += 256)
            inv |= okey(load_key(a.in, i, a.ew), a.flip, a.fneg) > okey(load_key(a.in, i + 1, a.ew), a.flip, a.fneg);
        if (__any(inv) && __lane_id() == 0) atomicOr(&c->inversion, 1u);
        __syncthreads();
    }
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) s_last = (atomicAdd(&c->mono_done, 1u) == nblk - 1);
    __syncthreads();
    if (!s_last) return;
    __threadfence();
    if (threadIdx.x == 0) c->inversion = atomic_load_agent(&c->inversion);
    __syncthreads();
    plan_block(a);
}
CAFS_KERNELS0(mono_full, 256)

// Writes the caller's report.  One thread.
__device__ __forceinline__ void finalize_body(const Args& a, uint32_t bid, uint32_t nblk) {
    if (threadIdx.x != 0 || !a.want_report) return;
    const Ctrl* c = a.c;
    cafs_report_t r;
    const bool sampled = !(c->path == P_MONOTONE || c->path == P_SMALL_N);
    r.est.k_hat = sampled ? c->k_hat : 0;
    r.est.u = sampled ? c->u : 0;
    r.est.f1 = sampled ? c->f1 : 0;
    r.est.f2 = sampled ? c->f2 : 0;
    r.est.n_samples = sampled ? c->n_samples : 0;
    r.est.stride = sampled ? c->stride : 0;
    r.est.saturated = sampled ? c->saturated : 0;
    r.est.pad = 0;
    r.path = c->path;
    r.tiny_miss = (int32_t)c->tiny_miss;
    const bool main_path = (c->path == P_MAIN || c->path == P_GUARD);
    r.table_M = main_path ? c->table_M : 0;
    r.spill_elems = main_path ? c->spill : 0;
    r.k_exact = c->K;
    r.engine = c->engine;
    r.flags = c->flags;
    *a.report = r;
}
CAFS_KERNELS0(finalize, 64)

// kSamples2Block samples per workgroup (kSamples2 / kSamples2Block workgroups, so
// that a heavy key's set slot takes few same-address updates), merged in LDS first (a heavy key takes one
// update of the shared set per workgroup instead of one per sample), then added to
// the set, each thread's updates issued together.  Chao1's u, f1 and f2 of the
// whole sample are kept as they grow: an add that takes a slot's count from o to
// o + m changes u by [o = 0], f1 by [o + m = 1] - [o = 1] and f2 by
// [o + m = 2] - [o = 2], and these changes telescope along each slot's chain of
// adds to its final count whatever the order of the adds.  Each workgroup stores
// its changes and its sampled elements per partition in its own row; the last
// workgroup sums the rows and plans the hash count for that estimate when it is
// above the paper's, with the partition buckets sized by the sampled elements of
// each partition (a few heavy keys can make one partition far larger than an even
// share).
__device__ __forceinline__ void sample2_body(const Args& a, uint32_t bid, uint32_t nblk) {
    Ctrl* c = a.c;
    if (!c->replan) return;
    constexpr uint32_t LS = 2 * kSamples2Block;  // LDS set (load <= 1/2)
    constexpr uint32_t R = 3 + kMaxParts;        // u, f1, f2 changes; sampled elements per 16 partitions
    constexpr uint32_t SPT = kSamples2Block / kSamples2Threads;  // samples per thread
    constexpr uint32_t PER = LS / kSamples2Threads;              // set slots per thread
    __shared__ uint64_t lk[LS];
    __shared__ uint32_t lc[LS];
    __shared__ uint32_t s_acc[R];
    __shared__ uint32_t s_last;
    for (uint32_t i = threadIdx.x; i < LS; i += blockDim.x) {
        lk[i] = kEmpty;
        lc[i] = 0;
    }
    if (threadIdx.x < R) s_acc[threadIdx.x] = 0;
    __syncthreads();
    const uint64_t stride = a.n / kSamples2;
    uint64_t sv[SPT];
#pragma unroll
    for (uint32_t j = 0; j < SPT; ++j)  // (grid * kSamples2Block == kSamples2)
        sv[j] = load_key(a.in, (uint64_t)(bid * kSamples2Block + j * kSamples2Threads + threadIdx.x) * stride, a.ew);
#pragma unroll
    for (uint32_t j = 0; j < SPT; ++j) {
        const uint64_t v = sv[j];
        if (v == kEmpty) continue;  // (planning only: that one key is left out)
        uint32_t h = phi_hash(v, kSample2LdsLog2);
        for (uint32_t probe = 0; probe < LS; ++probe) {
            // a slot that already holds the key takes the add alone (a heavy key's
            // samples would otherwise queue twice on one LDS address)
            const uint64_t k = lk[h];
            if (k == v) {
                atomicAdd(&lc[h], 1u);
                break;
            }
            if (k == kEmpty) {
                const unsigned long long old =
                    atomicCAS((unsigned long long*)&lk[h], (unsigned long long)kEmpty, (unsigned long long)v);
                if (old == kEmpty || old == v) {
                    atomicAdd(&lc[h], 1u);
                    break;
                }
            }
            h = (h + 1) & (LS - 1);
        }
    }
    __syncthreads();
    const uint32_t mask = (1u << kSample2SlotsLog2) - 1;
    uint32_t* cnt = sample2_counts(a);
    uint64_t key[PER];
    uint32_t cn[PER], slot[PER];
    uint64_t found[PER];
#pragma unroll
    for (uint32_t j = 0; j < PER; ++j) {
        const uint32_t i = threadIdx.x + j * blockDim.x;
        cn[j] = lc[i];
        key[j] = lk[i];
        slot[j] = phi_hash(key[j], kSample2SlotsLog2);
        if (cn[j]) atomicAdd(&s_acc[3 + (mul_hash32(key[j], 32, a.table_mul) >> (32 - kMaxPartLog2))], cn[j]);
    }
    // a slot that already holds the key (the heavy keys, after the first workgroup)
    // is taken without a compare-and-swap: same-address atomics of every workgroup
    // would queue on it
#pragma unroll
    for (uint32_t j = 0; j < PER; ++j) found[j] = cn[j] ? g_load(&a.tmp_k[slot[j]]) : kEmpty;
#pragma unroll
    for (uint32_t j = 0; j < PER; ++j)
        if (cn[j] && found[j] != key[j]) found[j] = g_cas(&a.tmp_k[slot[j]], kEmpty, key[j]);
#pragma unroll
    for (uint32_t j = 0; j < PER; ++j)
        if (found[j] == key[j]) found[j] = kEmpty;  // (the slot is the key's: no probe)
#pragma unroll
    for (uint32_t j = 0; j < PER; ++j) {
        // another key holds the home slot (rare at this load): probe on
        for (uint32_t probe = 1; cn[j] && found[j] != kEmpty && found[j] != key[j] && probe <= mask; ++probe) {
            slot[j] = (slot[j] + 1) & mask;
            found[j] = g_cas(&a.tmp_k[slot[j]], kEmpty, key[j]);
        }
    }
    uint32_t o[PER];
#pragma unroll
    for (uint32_t j = 0; j < PER; ++j) o[j] = cn[j] ? g_add(&cnt[slot[j]], cn[j]) : 0u;
    int32_t du = 0, d1 = 0, d2 = 0;
#pragma unroll
    for (uint32_t j = 0; j < PER; ++j) {
        if (!cn[j]) continue;
        du += o[j] == 0;
        d1 += (int32_t)(o[j] + cn[j] == 1) - (int32_t)(o[j] == 1);
        d2 += (int32_t)(o[j] + cn[j] == 2) - (int32_t)(o[j] == 2);
    }
    du = (int32_t)wave_sum_u32((uint32_t)du);
    d1 = (int32_t)wave_sum_u32((uint32_t)d1);
    d2 = (int32_t)wave_sum_u32((uint32_t)d2);
    if (__lane_id() == 0) {
        atomicAdd(&s_acc[0], (uint32_t)du);
        atomicAdd(&s_acc[1], (uint32_t)d1);
        atomicAdd(&s_acc[2], (uint32_t)d2);
    }
    __syncthreads();
    // (the changes are added modulo 2^32; the totals are counts, so they come out right)
    uint32_t* rows = sample2_rows(a);
    if (threadIdx.x < R) {
        gp(rows)[bid * R + threadIdx.x] = s_acc[threadIdx.x];
        __threadfence();  // (only the row's writers release it: a fence waits for the wave's stores)
    }
    __syncthreads();
    if (threadIdx.x == 0) s_last = (atomicAdd(&c->s2done, 1u) == nblk - 1);
    __syncthreads();
    if (!s_last) return;
    __threadfence();
    // the rows' words, one device-scope load per thread (loads of one thread, one
    // after the other, would each wait on memory)
    if (threadIdx.x < R) s_acc[threadIdx.x] = 0;
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < nblk * R; i += blockDim.x) atomicAdd(&s_acc[i % R], atomic_load_agent(&rows[i]));
    __syncthreads();
    if (threadIdx.x != 0) return;
    const uint64_t u = s_acc[0], f1 = s_acc[1], f2 = s_acc[2];
    const uint64_t k2 = u >= kSamples2 ? a.n : u + (f1 * f1) / (2 * (f2 + 1));
    if (k2 <= c->k_hat) return;
    const uint32_t engine = plan_count(a, c, k2, E_HASH);
    plan_engine_state(a, c, c->path, engine);
    const uint32_t pl = c->part_log2;
    if (engine != E_HASH || pl == 0) return;
    uint32_t mass[kMaxParts];
    uint64_t total = 0;
    const uint32_t span = 1u << (kMaxPartLog2 - pl);  // 16-partition cells per partition
    for (uint32_t q = 0; q < (1u << pl); ++q) {
        mass[q] = 0;
        for (uint32_t j = 0; j < span; ++j) mass[q] += s_acc[3 + q * span + j];
        total += mass[q];
    }
    if (total > 0 && !set_buckets(a, c, pl, mass, total)) set_buckets(a, c, pl, nullptr);
}
CAFS_KERNELS0(sample2, kSamples2Threads)

// Report of an empty column (n = 0): path MONOTONE, everything else zero.
__global__ void k_report_empty(cafs_report_t* r) {
    if (threadIdx.x != 0) return;
    cafs_report_t z = {};
    z.path = P_MONOTONE;
    *r = z;
}

}  // namespace cafs
