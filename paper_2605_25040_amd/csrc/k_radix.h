// LSD radix sort with 8-bit digits (the fallback engine of the dispatcher, and the
// sort of the distinct (key, count) pairs when K is large).
//
// Structure (after Adinets and Merrill's single-pass "onesweep" radix sort):
//   k_radix_hist   one read of the keys builds the histograms of all eight digits;
//                  the last workgroup to finish scans them into digit bases and
//                  plans the passes, skipping digits on which every key agrees.
//   k_radix_pass   one launch per active digit.  Tiles (8192 keys keys-only, 4096
//                  key-value) are claimed in
//                  order from an atomic counter; each tile ranks its keys stably
//                  per wave (8-ballot match), publishes its digit counts, finds
//                  its global offsets by decoupled look-back over the tiles before
//                  it, reorders the tile in LDS by digit and writes it out in
//                  runs.  Claiming tiles in order means a tile only ever waits for
//                  tiles already held by running workgroups.
//   kbl_radix_pass a batch's pass: a fixed grid takes the tiles of every column's
//                  job from a list built on the device (kb_radix_list).
//   k_radix_copy   final copy when the passes end in the scratch buffer.
// Digits are taken from the order key (okey), so int64 and float64 columns sort
// in their own order.
#pragma once
#include "cafs_dev.h"

namespace cafs {

__device__ __forceinline__ uint32_t digit_of(uint64_t key, uint64_t flip, uint64_t fneg, uint32_t d) {
    return (uint32_t)((okey(key, flip, fneg) >> (8 * d)) & 255u);
}

__device__ __forceinline__ void radix_hist_body(const Args& a, uint32_t bid, uint32_t nblk) {
    Ctrl* c = a.c;
    if (!c->radix_on) return;
    const RadixJob& j = c->rj;
    const uint64_t n = j.n;
    const uint64_t* src = j.src_k;
    const uint32_t sw = j.src_ew;
    const uint64_t flip = a.flip, fneg = a.fneg;
    __shared__ uint32_t lh[8][256];
    __shared__ uint32_t s_last;
    for (uint32_t i = threadIdx.x; i < 8 * 256; i += blockDim.x) (&lh[0][0])[i] = 0;
    // clear the look-back status words of the first pass
    const uint64_t tiles = (n + kRadixTile - 1) / kRadixTile;
    const uint64_t gtid = (uint64_t)bid * blockDim.x + threadIdx.x;
    const uint64_t gstride = (uint64_t)nblk * blockDim.x;
    for (uint64_t i = gtid; i < tiles * 256; i += gstride) a.status[i] = 0;
    __syncthreads();
    const uint32_t lane = __lane_id();
    constexpr int U = 4;  // loads in flight per thread
    const uint64_t iters = (n + gstride * U - 1) / (gstride * U);
    for (uint64_t it = 0; it < iters; ++it) {
        uint64_t vv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint64_t i = (it * U + u) * gstride + gtid;
            vv[u] = i < n ? load_key(src, i, sw) : 0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
        const uint64_t v = vv[u];
        const bool ok = (it * U + u) * gstride + gtid < n;
        const uint64_t act = __ballot(ok);
        if (act == 0) continue;
        for (uint32_t d = 0; d < 8; ++d) {
            const uint32_t dg = digit_of(v, flip, fneg, d);
            // lane 0's digit, read as a scalar (no cross-lane LDS instruction); if lane
            // 0 is out of range and its digit differs, the lanes take the per-lane atomics
            const uint32_t first = __builtin_amdgcn_readfirstlane(dg);
            const uint64_t same = __ballot(ok && dg == first);
            if (same == act) {
                // wave-uniform digit: one atomic for the wave (skewed and low-K data)
                if (lane == (uint32_t)(__ffsll((unsigned long long)act) - 1))
                    atomicAdd(&lh[d][dg], (uint32_t)__popcll(act));
            } else if (ok) {
                atomicAdd(&lh[d][dg], 1u);
            }
        }
        }
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < 8 * 256; i += blockDim.x) {
        const uint32_t h = (&lh[0][0])[i];
        if (h) atomicAdd((unsigned long long*)&(&c->hist[0][0])[i], (unsigned long long)h);
    }
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) s_last = (atomicAdd(&c->hist_done, 1u) == nblk - 1);
    __syncthreads();
    if (!s_last) return;
    __threadfence();
    // last workgroup: digit bases (exclusive scans) and the pass plan.  Each of the
    // 256 threads loads 8 consecutive bins of one digit at once (read one after the
    // other, the device-scope loads took most of a millisecond) and 32 lanes scan
    // each digit in registers.
    __shared__ uint32_t s_active[8];
    {
        const uint32_t d = threadIdx.x >> 5, q = threadIdx.x & 31;  // blockDim.x == 256
        uint64_t h[8];
#pragma unroll
        for (uint32_t j = 0; j < 8; ++j) h[j] = atomic_load_agent(&c->hist[d][q * 8 + j]);
        uint64_t loc = 0;
        bool constant = false;
#pragma unroll
        for (uint32_t j = 0; j < 8; ++j) {
            constant |= (h[j] == n);
            loc += h[j];
        }
        uint64_t inc = loc;
#pragma unroll
        for (uint32_t o = 1; o < 32; o <<= 1) {
            const uint64_t t = __shfl_up(inc, o, 32);
            if (q >= o) inc += t;
        }
        uint64_t run = inc - loc;
#pragma unroll
        for (uint32_t j = 0; j < 8; ++j) {
            c->hist[d][q * 8 + j] = run;
            run += h[j];
        }
        const uint64_t cm = __ballot(constant);  // this digit's 32 lanes are one half of the wave
        if (q == 0) s_active[d] = ((cm >> (threadIdx.x & 32)) & 0xFFFFFFFFull) == 0 && n > 0 ? 1u : 0u;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        RadixJob& jw = c->rj;
        uint32_t np = 0;
        for (uint32_t d = 0; d < 8; ++d)
            if (s_active[d]) jw.digit[np++] = d;
        jw.n_active = np;
        const bool inplace = (jw.src_k == jw.dst_k);
        // ping-pong so that the last pass lands in dst; when sorting in place with an
        // odd number of passes the first pass must not write dst, so all passes shift
        // by one and a final copy moves the result from tmp to dst
        const uint32_t shift = (inplace && (np & 1u)) ? 1u : 0u;
        const uint64_t* ck = jw.src_k;
        const uint64_t* cv = jw.src_v;
        uint32_t cw = jw.src_ew;
        for (uint32_t i = 0; i < np; ++i) {
            const bool to_dst = ((np - 1 - i + shift) % 2) == 0;
            jw.ps_k[i] = ck; jw.ps_v[i] = cv; jw.ps_w[i] = cw;
            jw.pd_k[i] = to_dst ? jw.dst_k : jw.tmp_k;
            jw.pd_v[i] = to_dst ? jw.dst_v : jw.tmp_v;
            jw.pd_w[i] = to_dst ? jw.dst_ew : 8u;  // the scratch holds 8-byte keys
            ck = jw.pd_k[i]; cv = jw.pd_v[i]; cw = jw.pd_w[i];
        }
        if (np == 0) jw.copy_mode = inplace ? 0u : 1u;
        else jw.copy_mode = shift ? 2u : 0u;
    }
}
CAFS_KERNELS0(radix_hist, 256)

// Stable match of equal 8-bit digits across the wave: the lanes (within `act`)
// whose digit equals this lane's digit.
__device__ __forceinline__ uint64_t match_digit(uint32_t dg, uint64_t act) {
    uint64_t peers = act;
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        const bool bit = (dg >> b) & 1u;
        const uint64_t m = __ballot(bit);
        peers &= bit ? m : ~m;
    }
    return peers;
}

// LDS of one radix pass workgroup of THREADS threads (tiles of 16 keys per thread):
// each kernel declares the arrays itself (one array per variable keeps the layout
// the pass was tuned with) and hands the tile function their addresses.
template <bool VALS, uint32_t THREADS>
struct RadixLds {
    static constexpr uint32_t NW = THREADS / 64;
    static constexpr uint32_t TILE = THREADS * kRadixItems;
    uint64_t* lk;
    uint64_t* lv;
    uint32_t (*wcnt)[256];
    uint32_t* toff;
    uint64_t* gofs;
    uint64_t* sbase;  // the pass digit's global bases of the column
    uint32_t* scan_tmp;
};
#define CAFS_RADIX_LDS(VALS, THREADS, NAME)                                            \
    __shared__ uint64_t NAME##_lk[RadixLds<VALS, THREADS>::TILE];                     \
    __shared__ uint64_t NAME##_lv[VALS ? RadixLds<VALS, THREADS>::TILE : 1];          \
    __shared__ uint32_t NAME##_wcnt[RadixLds<VALS, THREADS>::NW][256];                \
    __shared__ uint32_t NAME##_toff[256];                                             \
    __shared__ uint64_t NAME##_gofs[256];                                             \
    __shared__ uint32_t NAME##_scan[RadixLds<VALS, THREADS>::NW + 1];                 \
    __shared__ uint64_t NAME##_sbase[256];                                            \
    const RadixLds<VALS, THREADS> NAME{NAME##_lk, NAME##_lv, NAME##_wcnt, NAME##_toff, \
                                       NAME##_gofs, NAME##_sbase, NAME##_scan};

// One tile t of a column's LSD pass (with its values when VALS): stable ranks within
// the tile by wave matching, the tile's digit offsets by decoupled look-back over the
// tiles before it, a reorder through LDS and a scatter of digit runs.  On entry
// L.wcnt is zero, L.sbase holds the column's digit bases for this pass and the
// workgroup is synchronised; on return it is synchronised again.  Called by every
// thread of the workgroup.
// A column's pass, read once per workgroup and column: the job's sizes, the pass's
// digit, source, destination and look-back words.
struct RadixPassView {
    uint64_t n, flip, fneg;
    uint32_t d, skw, dkw;
    const uint64_t* sk;
    const uint64_t* sv;
    uint64_t* dk;
    uint64_t* dv;
    uint64_t* status;
};
__device__ __forceinline__ RadixPassView radix_view(const Args& a, const RadixJob& j, uint32_t pass) {
    RadixPassView v;
    v.n = j.n;
    v.flip = a.flip;
    v.fneg = a.fneg;
    v.d = j.digit[pass];
    v.sk = j.ps_k[pass];
    v.sv = j.ps_v[pass];
    v.dk = j.pd_k[pass];
    v.dv = j.pd_v[pass];
    v.skw = j.ps_w[pass];
    v.dkw = j.pd_w[pass];
    v.status = a.status + (pass & 1u) * a.status_slot;
    return v;
}

template <bool VALS, uint32_t THREADS>
__device__ __forceinline__ void radix_tile(const RadixPassView& P, uint64_t t, const RadixLds<VALS, THREADS>& L) {
    constexpr uint32_t NW = RadixLds<VALS, THREADS>::NW;
    constexpr uint32_t TILE = RadixLds<VALS, THREADS>::TILE;
    const uint64_t n = P.n;
    const uint32_t d = P.d;
    const uint64_t flip = P.flip, fneg = P.fneg;
    const uint64_t* sk = P.sk;
    const CAFS_GLOBAL uint64_t* __restrict__ sv = gp(P.sv);
    uint64_t* dk = P.dk;
    CAFS_GLOBAL uint64_t* __restrict__ dv = gp(P.dv);
    const uint32_t skw = P.skw, dkw = P.dkw;
    uint64_t* status = P.status;
    const uint32_t tid = threadIdx.x;
    const uint32_t lane = __lane_id();
    const uint32_t wave = tid >> 6;
    const uint64_t lt_mask = (1ull << lane) - 1;
    const uint64_t base = t * TILE;
    // load: wave w owns positions base + w*64*16 + i*64 + lane, i = 0..15 (in order)
    uint64_t key[kRadixItems];
    uint64_t val[VALS ? kRadixItems : 1];
    uint32_t rank2[kRadixItems / 2];  // two 16-bit ranks per register
    uint32_t okm = 0;  // bit i: item i is in range (digits are recomputed from the keys)
#pragma unroll
    for (int i = 0; i < kRadixItems; ++i) {
        const uint64_t pos = base + (uint64_t)wave * (64 * kRadixItems) + (uint64_t)i * 64 + lane;
        const bool ok = pos < n;
        key[i] = ok ? load_key(sk, pos, skw) : 0;
        if constexpr (VALS) val[i] = ok ? sv[pos] : 0;
        okm |= (ok ? 1u : 0u) << i;
    }
    // stable rank within the wave, item by item
#pragma unroll
    for (int i = 0; i < kRadixItems; ++i) {
        const bool ok = (okm >> i) & 1u;
        const uint32_t dg = digit_of(key[i], flip, fneg, d);
        const uint64_t act = __ballot(ok);
        const uint64_t peers = match_digit(dg, act);
        uint32_t before = 0;
        if (ok) before = L.wcnt[wave][dg];
        const uint32_t rk = before + (uint32_t)__popcll(peers & lt_mask);
        if (i & 1) rank2[i >> 1] |= rk << 16; else rank2[i >> 1] = rk;
        const bool leader = ok && ((peers & lt_mask) == 0);
        if (leader) L.wcnt[wave][dg] = before + (uint32_t)__popcll(peers);
    }
    __syncthreads();
    // per digit: tile total and per-wave exclusive prefix
    uint32_t run = 0;  // this thread's digit: count in the tile (threads past 256: none)
    if (tid < 256) {
        const uint32_t dd = tid;  // one digit per thread
#pragma unroll
        for (uint32_t w = 0; w < NW; ++w) {
            const uint32_t cw = L.wcnt[w][dd];
            L.wcnt[w][dd] = run;
            run += cw;
        }
        // publish this tile's aggregate, then look back for the exclusive prefix
        CAFS_GLOBAL uint64_t* st = gp(status) + t * 256 + dd;
        uint64_t excl = 0;
        if (t == 0) {
            __hip_atomic_store(st, kStatInc | (uint64_t)run, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            __hip_atomic_store(st, kStatAgg | (uint64_t)run, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            uint64_t tt = t - 1;
            while (true) {
                const uint64_t* sp = status + tt * 256 + dd;
                uint64_t s = g_load(sp);
                while ((s & (kStatAgg | kStatInc)) == 0) {
                    __builtin_amdgcn_s_sleep(1);
                    s = g_load(sp);
                }
                excl += s & kStatMask;
                if (s & kStatInc) break;
                --tt;
            }
            __hip_atomic_store(st, kStatInc | (excl + run), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        L.gofs[dd] = L.sbase[dd] + excl;
    }
    // tile-local digit offsets
    {
        uint32_t total;
        const uint32_t ex = block_exclusive_scan<uint32_t>(run, L.scan_tmp, &total);
        if (tid < 256) L.toff[tid] = ex;
        __syncthreads();
        if (tid < 256) L.gofs[tid] -= ex;  // global position = gofs[digit] + local position
    }
    __syncthreads();
    // reorder the tile in LDS by digit (stable)
#pragma unroll
    for (int i = 0; i < kRadixItems; ++i) {
        if ((okm >> i) & 1u) {
            const uint32_t dg = digit_of(key[i], flip, fneg, d);
            const uint32_t q = L.toff[dg] + L.wcnt[wave][dg] + ((rank2[i >> 1] >> (16 * (i & 1))) & 0xFFFFu);
            if (q < TILE) {  // always true when the ranks are consistent
                L.lk[q] = key[i];
                if constexpr (VALS) L.lv[q] = val[i];
            }
        }
    }
    __syncthreads();
    const uint32_t cnt = (uint32_t)((n - base) < TILE ? (n - base) : TILE);
    for (uint32_t q = tid; q < cnt; q += blockDim.x) {
        const uint64_t k = L.lk[q];
        const uint64_t g = L.gofs[digit_of(k, flip, fneg, d)] + q;
        if (g < n) {  // always true when the look-back prefixes are consistent
            store_key(dk, g, k, dkw);
            if constexpr (VALS) dv[g] = L.lv[q];
        }
    }
    __syncthreads();
}

// One LSD pass of a column by the workgroups of its launch: tiles are claimed in
// order from the pass's counter (a tile only ever waits for tiles held by running
// workgroups).  Keys-only and key-value passes are separate kernels so that the
// keys-only one keeps fewer registers and less LDS.  The single-column keys-only
// pass takes 512 threads (tiles of 8192 keys: digit runs of 32 keys on average, so
// fewer partly written cache lines, and half the look-backs); key-value passes take
// 256.
template <bool VALS, uint32_t THREADS>
__device__ __forceinline__ void radix_pass_impl(const Args& a, uint32_t pass, uint32_t bid, uint32_t nblk) {
    constexpr uint32_t TILE = RadixLds<VALS, THREADS>::TILE;
    Ctrl* c = a.c;
    if (!c->radix_on) return;
    const RadixJob& j = c->rj;
    if ((j.has_vals != 0) != VALS || pass >= j.n_active) return;
    const uint64_t tiles = (j.n + TILE - 1) / TILE;  // (the status words are sized for kRadixTile)
    CAFS_GLOBAL uint64_t* status_next = gp(a.status) + ((pass + 1) & 1u) * a.status_slot;
    CAFS_RADIX_LDS(VALS, THREADS, L)
    __shared__ uint32_t s_tile;
    for (uint32_t i = threadIdx.x; i < 256; i += blockDim.x) L.sbase[i] = c->hist[j.digit[pass]][i];
    // clear the status words the next pass will use (the previous pass is done with them)
    {
        const uint64_t gtid = (uint64_t)bid * blockDim.x + threadIdx.x;
        const uint64_t gstride = (uint64_t)nblk * blockDim.x;
        if (pass + 1 < j.n_active)
            for (uint64_t i = gtid; i < tiles * 256; i += gstride) status_next[i] = 0;
    }
    const RadixPassView P = radix_view(a, j, pass);
    while (true) {
        if (threadIdx.x == 0) s_tile = atomicAdd(&c->tile_ctr[pass], 1u);
        for (uint32_t i = threadIdx.x; i < RadixLds<VALS, THREADS>::NW * 256; i += blockDim.x) (&L.wcnt[0][0])[i] = 0;
        __syncthreads();
        const uint64_t t = s_tile;
        if (t >= tiles) break;
        radix_tile<VALS, THREADS>(P, t, L);
    }
}

// Persistent pass of a batch: a fixed grid works through every column's tiles of
// one kind (keys-only or key-value) as one list of items in column order, claimed
// from one counter per pass (so a column's tiles are claimed in order, and a tile
// only waits for tiles held by running workgroups).  The grid does not depend on
// the number of columns: a batched launch over every column's blocks spends most of
// its time starting and ending the blocks of columns that have no radix job.
template <bool VALS>
__device__ __forceinline__ void radix_pass_list(const Args* args, RadixList* R, uint32_t pass) {
    constexpr uint32_t THREADS = kRadixThreads;
    constexpr uint32_t kind = VALS ? 1u : 0u;
    CAFS_RADIX_LDS(VALS, THREADS, L)
    __shared__ uint32_t s_col;
    __shared__ uint64_t s_t;
    const uint32_t total = R->total[kind];
    const uint32_t ncols = R->ncols[kind];
    const uint32_t* cols = radix_list_cols(R, kind);
    const uint32_t* start = radix_list_start(R, kind);
    uint32_t cur = kNoCol;  // column whose digit bases L.sbase holds (uniform)
    while (true) {
        if (threadIdx.x == 0) {
            const uint32_t item = atomicAdd(&R->next[kind][pass], 1u);
            uint32_t col = kNoCol;
            uint64_t t = 0;
            if (item < total) {
                // the last list entry whose first item is at or before this one
                uint32_t lo = 0, hi = ncols;
                while (hi - lo > 1) {
                    const uint32_t mid = (lo + hi) / 2;
                    if (start[mid] <= item) lo = mid; else hi = mid;
                }
                col = cols[lo];
                t = item - start[lo];
            }
            s_col = col;
            s_t = t;
        }
        for (uint32_t i = threadIdx.x; i < RadixLds<VALS, THREADS>::NW * 256; i += blockDim.x) (&L.wcnt[0][0])[i] = 0;
        __syncthreads();
        const uint32_t col = s_col;
        const uint64_t t = s_t;
        if (col == kNoCol) break;
        const Args& a = args[col];
        const RadixJob& j = a.c->rj;
        if (pass >= j.n_active) {  // (uniform: a constant digit needs no pass)
            __syncthreads();
            continue;
        }
        if (col != cur) {
            for (uint32_t i = threadIdx.x; i < 256; i += blockDim.x) L.sbase[i] = a.c->hist[j.digit[pass]][i];
            cur = col;
        }
        // this tile's status words for the next pass (the previous pass is done with them)
        if (pass + 1 < j.n_active && threadIdx.x < 256)
            (gp(a.status) + ((pass + 1) & 1u) * a.status_slot)[t * 256 + threadIdx.x] = 0;
        __syncthreads();
        radix_tile<VALS, THREADS>(radix_view(a, j, pass), t, L);
    }
}

// The radix jobs of a batch, listed once the histograms have planned them: one
// workgroup scans the columns in chunks, and each kind's entries (column, first
// item) are placed by block scans in column order.
__device__ __forceinline__ void radix_list_body(const Args* args, uint32_t n_cols, RadixList* R) {
    __shared__ uint32_t scan_tmp[17];
    uint32_t run_c[2] = {0, 0}, run_t[2] = {0, 0};
    for (uint32_t c0 = 0; c0 < n_cols; c0 += blockDim.x) {  // uniform
        const uint32_t col = c0 + threadIdx.x;
        uint32_t kind = 2, tiles = 0;
        if (col < n_cols) {
            const Ctrl* c = args[col].c;
            if (c->radix_on) {
                const uint64_t n = c->rj.n;
                tiles = (uint32_t)((n + kRadixTile - 1) / kRadixTile);
                kind = tiles ? (c->rj.has_vals ? 1u : 0u) : 2u;
            }
        }
        for (uint32_t k = 0; k < 2; ++k) {
            const uint32_t is = kind == k ? 1u : 0u;
            uint32_t tot_c, tot_t;
            const uint32_t ec = block_exclusive_scan<uint32_t>(is, scan_tmp, &tot_c);
            const uint32_t et = block_exclusive_scan<uint32_t>(is ? tiles : 0u, scan_tmp, &tot_t);
            if (is) {
                radix_list_cols(R, k)[run_c[k] + ec] = col;
                radix_list_start(R, k)[run_c[k] + ec] = run_t[k] + et;
            }
            run_c[k] += tot_c;
            run_t[k] += tot_t;
        }
    }
    if (threadIdx.x == 0) {
        for (uint32_t k = 0; k < 2; ++k) {
            R->ncols[k] = run_c[k];
            R->total[k] = run_t[k];
            radix_list_start(R, k)[run_c[k]] = run_t[k];
            for (uint32_t p = 0; p < 8; ++p) R->next[k][p] = 0;
        }
    }
}
__global__ __launch_bounds__(1024) void kb_radix_list(const Args* args, uint32_t n_cols, RadixList* R) {
    radix_list_body(args, n_cols, R);
}
__global__ __launch_bounds__(kRadixThreads) void kbl_radix_pass(const Args* args, RadixList* R, uint32_t pass) {
    radix_pass_list<false>(args, R, pass);
}
__global__ __launch_bounds__(kRadixThreads) void kbl_radix_pass_kv(const Args* args, RadixList* R, uint32_t pass) {
    radix_pass_list<true>(args, R, pass);
}

// (the keys-only pass asks for four waves per SIMD, two workgroups per CU, which
// its LDS allows: at most 128 registers)
__global__ __launch_bounds__(kRadixKeysThreads, 4) void k_radix_pass(Args a, uint32_t pass) {
    radix_pass_impl<false, kRadixKeysThreads>(a, pass, blockIdx.x, gridDim.x);
}
__global__ __launch_bounds__(kRadixThreads) void k_radix_pass_kv(Args a, uint32_t pass) {
    radix_pass_impl<true, kRadixThreads>(a, pass, blockIdx.x, gridDim.x);
}

__device__ __forceinline__ void radix_copy_body(const Args& a, uint32_t bid, uint32_t nblk) {
    Ctrl* c = a.c;
    if (!c->radix_on) return;
    const RadixJob& j = c->rj;
    if (j.copy_mode == 0) return;
    const uint64_t* sk = j.copy_mode == 1 ? j.src_k : j.tmp_k;
    const CAFS_GLOBAL uint64_t* sv = gp(j.copy_mode == 1 ? j.src_v : j.tmp_v);
    const uint32_t skw = j.copy_mode == 1 ? j.src_ew : 8u;
    uint64_t* dk = j.dst_k;
    CAFS_GLOBAL uint64_t* dv = gp(j.dst_v);
    const bool vals = j.has_vals != 0;
    const uint64_t n = j.n;
    const uint64_t gtid = (uint64_t)bid * blockDim.x + threadIdx.x;
    const uint64_t gstride = (uint64_t)nblk * blockDim.x;
    for (uint64_t i = gtid; i < n; i += gstride) {
        store_key(dk, i, load_key(sk, i, skw), j.dst_ew);
        if (vals) dv[i] = sv[i];
    }
}
CAFS_KERNELS0(radix_copy, 256)

}  // namespace cafs
