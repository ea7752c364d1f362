// Emit stage (Alg. 4: fill each key count times, in key order) and the run-length
// pass that recovers (key, count) pairs from an already sorted column.
#pragma once
#include "cafs_dev.h"
#include "k_count.h"

namespace cafs {

constexpr uint32_t kEmitPairsPerThread = 8;
constexpr uint32_t kEmitThreads = 256;
constexpr uint64_t kEmitTilePairs = (uint64_t)kEmitPairsPerThread * kEmitThreads;  // 2048 pairs
constexpr uint32_t kEmitLdsRuns = 512;  // small LDS footprint leaves room for the side stream

// Largest j in [lo, hi] with off[j] <= e (off is nondecreasing, off[lo] <= e).
template <typename OffT>
__device__ __forceinline__ uint64_t run_of(const OffT* off, uint64_t lo, uint64_t hi, uint64_t e) {
    while (lo < hi) {
        const uint64_t mid = lo + (hi - lo + 1) / 2;
        if ((uint64_t)off[mid] <= e) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ void store_pair(uint64_t* __restrict__ y, uint64_t n, uint32_t head, uint64_t p,
                                           uint64_t v0, uint64_t v1) {
    const int64_t e0 = (int64_t)(2 * p) - (int64_t)head;
    const bool ok0 = e0 >= 0 && (uint64_t)e0 < n;
    const bool ok1 = (uint64_t)(e0 + 1) < n;
    if (ok0 && ok1) {
        u64x2 w;
        w.x = v0;
        w.y = v1;
        __builtin_nontemporal_store(w, reinterpret_cast<u64x2*>(y + e0));
    } else {
        if (ok0) y[e0] = v0;
        if (ok1) y[e0 + 1] = v1;
    }
}

// Output tiles of 4096 elements; each tile finds the runs it covers by binary
// search in the run offsets.  A tile inside one run is a plain fill; otherwise the
// tile's offsets and keys are staged in LDS and each element searches there.
// `after_pair_sort` selects the instance: one runs on the caller's stream right
// after the single-workgroup order kernel (or the tiny branch), the other on the
// side stream after the pair sort; exactly one of them has work.
// The tile loop works on caller-provided LDS: kEmitLdsRuns + 1 offsets, kEmitLdsRuns
// keys and two words for the tile's run range.
__device__ __forceinline__ void emit_tiles(const Args& a, uint32_t bid, uint32_t nblk, uint64_t* s_off,
                                           uint64_t* s_key, uint64_t* s_j) {
    Ctrl* c = a.c;
    const uint64_t n = a.n;
    const uint64_t K = c->K;
    const uint32_t head = a.out_head;
    const uint64_t P = num_pairs(n, head);
    const uint64_t tiles = (P + kEmitTilePairs - 1) / kEmitTilePairs;
    const uint64_t* __restrict__ off = a.off;
    const uint64_t* __restrict__ uq = a.uniq;
    for (uint64_t t = bid; t < tiles; t += nblk) {
        const uint64_t p0 = t * kEmitTilePairs;
        const uint64_t p1 = (p0 + kEmitTilePairs < P) ? p0 + kEmitTilePairs : P;
        const int64_t e_lo_s = (int64_t)(2 * p0) - (int64_t)head;
        const uint64_t e_lo = e_lo_s < 0 ? 0 : (uint64_t)e_lo_s;
        const uint64_t e_hi = (2 * p1 - head < n) ? 2 * p1 - head : n;  // exclusive
        if (threadIdx.x == 0) {
            const uint64_t j0 = run_of(off, 0, K - 1, e_lo);
            s_j[0] = j0;
            s_j[1] = run_of(off, j0, K - 1, e_hi - 1);
        }
        __syncthreads();
        const uint64_t j0 = s_j[0], j1 = s_j[1];
        if (j0 == j1) {
            const uint64_t v = uq[j0];
            for (uint64_t p = p0 + threadIdx.x; p < p1; p += blockDim.x) store_pair(a.out, n, head, p, v, v);
        } else if (j1 - j0 + 1 <= kEmitLdsRuns) {
            const uint32_t R = (uint32_t)(j1 - j0 + 1);
            for (uint32_t i = threadIdx.x; i <= R; i += blockDim.x) s_off[i] = off[j0 + i];
            for (uint32_t i = threadIdx.x; i < R; i += blockDim.x) s_key[i] = uq[j0 + i];
            __syncthreads();
            for (uint64_t p = p0 + threadIdx.x; p < p1; p += blockDim.x) {
                const int64_t e0s = (int64_t)(2 * p) - (int64_t)head;
                const uint64_t e0 = e0s < 0 ? 0 : (uint64_t)e0s;
                const uint64_t r0 = run_of(s_off, 0, R - 1, e0);
                // the second element (e0s + 1, not e0 + 1 when the pair starts before the column)
                const uint64_t r1 = (r0 + 1 < R && (int64_t)s_off[r0 + 1] <= e0s + 1) ? r0 + 1 : r0;
                store_pair(a.out, n, head, p, s_key[r0], s_key[r1]);
            }
        } else {
            for (uint64_t p = p0 + threadIdx.x; p < p1; p += blockDim.x) {
                const int64_t e0s = (int64_t)(2 * p) - (int64_t)head;
                const uint64_t e0 = e0s < 0 ? 0 : (uint64_t)e0s;
                const uint64_t r0 = run_of(off, j0, j1, e0);
                const uint64_t r1 = (r0 + 1 <= j1 && (int64_t)off[r0 + 1] <= e0s + 1) ? r0 + 1 : r0;
                store_pair(a.out, n, head, p, uq[r0], uq[r1]);
            }
        }
        __syncthreads();
    }
}
// The tile emit for 32-bit keys: the same tiles counted in elements (4096 per
// tile), each element stored as 4 bytes (a wave writes 256 consecutive bytes per
// store instruction).
__device__ __forceinline__ void emit_tiles32(const Args& a, uint32_t bid, uint32_t nblk, uint64_t* s_off,
                                             uint64_t* s_key, uint64_t* s_j) {
    Ctrl* c = a.c;
    const uint64_t n = a.n;
    const uint64_t K = c->K;
    constexpr uint64_t T = 2 * kEmitTilePairs;
    const uint64_t tiles = (n + T - 1) / T;
    const uint64_t* __restrict__ off = a.off;
    const uint64_t* __restrict__ uq = a.uniq;
    CAFS_GLOBAL uint32_t* y = gp(reinterpret_cast<uint32_t*>(a.out));
    for (uint64_t t = bid; t < tiles; t += nblk) {
        const uint64_t e_lo = t * T;
        const uint64_t e_hi = e_lo + T < n ? e_lo + T : n;  // exclusive
        if (threadIdx.x == 0) {
            const uint64_t j0 = run_of(off, 0, K - 1, e_lo);
            s_j[0] = j0;
            s_j[1] = run_of(off, j0, K - 1, e_hi - 1);
        }
        __syncthreads();
        const uint64_t j0 = s_j[0], j1 = s_j[1];
        if (j0 == j1) {
            const uint32_t v = (uint32_t)uq[j0];
            for (uint64_t e = e_lo + threadIdx.x; e < e_hi; e += blockDim.x) y[e] = v;
        } else if (j1 - j0 + 1 <= kEmitLdsRuns) {
            const uint32_t R = (uint32_t)(j1 - j0 + 1);
            for (uint32_t i = threadIdx.x; i <= R; i += blockDim.x) s_off[i] = off[j0 + i];
            for (uint32_t i = threadIdx.x; i < R; i += blockDim.x) s_key[i] = uq[j0 + i];
            __syncthreads();
            for (uint64_t e = e_lo + threadIdx.x; e < e_hi; e += blockDim.x) y[e] = (uint32_t)s_key[run_of(s_off, 0, R - 1, e)];
        } else {
            for (uint64_t e = e_lo + threadIdx.x; e < e_hi; e += blockDim.x) y[e] = (uint32_t)uq[run_of(off, j0, j1, e)];
        }
        __syncthreads();
    }
}

// `mode`: 0 main instance (batched launches, which have no row emit), 1 after the
// pair sort.
__device__ __forceinline__ void emit_body(const Args& a, uint32_t mode, uint32_t bid, uint32_t nblk) {
    Ctrl* c = a.c;
    if (mode == 1 ? !(c->pair_sort && c->dense_ready && !c->overflow) : !c->emit_main) return;
    __shared__ uint64_t s_j[2];
    __shared__ uint64_t s_off[kEmitLdsRuns + 1];
    __shared__ uint64_t s_key[kEmitLdsRuns];
    if (a.ew == 4) emit_tiles32(a, bid, nblk, s_off, s_key, s_j);
    else emit_tiles(a, bid, nblk, s_off, s_key, s_j);
}
CAFS_KERNELS1(emit, kEmitThreads, uint32_t, mode)

// Row emit, the main instance of a single-column call (K <= kRankMax).  HBM takes writes
// fastest when few regions are written at a time (measured on MI355X: about 6.3
// TB/s when 256 workgroups sweep the output in rows, whether as one sweep or as up
// to 32 sweeps over separate segments, against 5.2-5.8 TB/s when each workgroup
// streams its own tiles or chunk).  The output is cut into segments of about
// R runs each (segment i starts at the 4 KB-aligned group at or before the first
// element of run i * R); each segment gets workgroups in
// proportion to its groups, and they sweep it in rows of (workgroups * blockDim)
// groups, each writing blockDim consecutive groups of every row, kEmitRowsUnroll
// rows per step.  A group is the 16 bytes of one store: two 64-bit keys or four
// 32-bit keys.  A workgroup stages its segment's runs in LDS (offsets relative
// to the segment start) with an index of the run holding every 2^s-th position of
// the segment (at most kEmitIdxSlots entries); an element's run is that entry's
// run, or a short binary search when run boundaries fall inside the span.
constexpr uint32_t kEmitRowsMaxK = 4088;   // runs one workgroup stages (64 KB of LDS with the index; one
                                           // workgroup per CU leaves room for the side stream's kernels)
constexpr uint32_t kEmitIdxSlots = 4096;
constexpr uint32_t kEmitAlignPairs = 256;  // segment starts: multiples of 4 KB of output
// runs starting in a segment: kEmitRowsMaxK - G * kEmitAlignPairs for groups of G keys
// per 16-byte store (2 for 64-bit keys, 4 for 32-bit keys); the fewest is for G = 4
constexpr uint32_t kEmitSegRunsMin = kEmitRowsMaxK - 4 * kEmitAlignPairs;
constexpr uint32_t kEmitMaxSegs = (kRankMax + kEmitSegRunsMin - 1) / kEmitSegRunsMin;  // segments for K <= kRankMax
constexpr uint32_t kEmitRowsThreads = 256;
constexpr int kEmitRowsUnroll = 8;

// Run of position e: largest j with soff[j] <= e, between the runs at the index
// positions around e.
__device__ __forceinline__ uint32_t run_in(const uint32_t* sidx, const uint32_t* soff, uint32_t s, uint32_t e) {
    const uint32_t q = e >> s;
    uint32_t lo = sidx[q], hi = sidx[q + 1];
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (soff[mid] <= e) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Largest j in [lo, hi] with off[j] <= e (off[lo] <= e), by one whole wave: each
// round probes 64 evenly spaced offsets at once and keeps the span between the last
// one at or below e and the next (the predicate is monotone in j).  Every lane gets
// the answer.
__device__ __forceinline__ uint64_t wave_run_of(const uint64_t* off, uint64_t lo, uint64_t hi, uint64_t e) {
    const uint32_t lane = __lane_id();
    while (true) {
        const uint64_t span = hi - lo + 1;
        const uint64_t step = span <= 64 ? 1 : (span + 63) / 64;
        const uint64_t j = lo + lane * step;
        const bool ok = j <= hi && gp(off)[j] <= e;
        const uint64_t m = __ballot(ok);  // a prefix of the lanes, lane 0 always set
        const uint64_t at = lo + (uint64_t)(63 - __builtin_clzll(m)) * step;
        if (step == 1) return at;
        lo = at;
        hi = at + step - 1 < hi ? at + step - 1 : hi;
    }
}

__device__ __forceinline__ bool rows_take(const Args& a, const Ctrl* c) {
    return c->K >= 1 && c->K <= kRankMax;  // (columns hold fewer than 2^32 keys)
}

// LDS of the row emit.
struct EmitRowsLds {
    uint32_t soff[kEmitRowsMaxK + 1];
    uint64_t skey[kEmitRowsMaxK];
    uint32_t sidx[kEmitIdxSlots + 2];
    uint32_t swave[kEmitRowsThreads / 64];
    uint64_t s_rng[2];
    uint64_t s_pb[kEmitMaxSegs + 1];  // first group of each segment, and the group count
    uint32_t s_seg[3];
};

// Four 32-bit keys of group p (elements 4p - head .. 4p - head + 3): one 16-byte
// store when all four are in the column.
__device__ __forceinline__ void store_quad(uint64_t* __restrict__ y64, uint64_t n, uint32_t head, uint64_t p,
                                           const uint32_t* v) {
    uint32_t* y = reinterpret_cast<uint32_t*>(y64);
    const int64_t e0 = (int64_t)(4 * p) - (int64_t)head;
    if (e0 >= 0 && (uint64_t)e0 + 3 < n) {
        u64x2 w;
        w.x = (uint64_t)v[0] | ((uint64_t)v[1] << 32);
        w.y = (uint64_t)v[2] | ((uint64_t)v[3] << 32);
        __builtin_nontemporal_store(w, reinterpret_cast<u64x2*>(y + e0));
    } else {
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (e0 + j >= 0 && (uint64_t)(e0 + j) < n) y[e0 + j] = v[j];
    }
}

template <uint32_t G>
__device__ __forceinline__ void emit_rows_impl(const Args& a, uint32_t bid, uint32_t nblk, EmitRowsLds& L) {
    Ctrl* c = a.c;
    const uint64_t n = a.n;
    const uint64_t K64 = c->K;
    uint32_t* soff = L.soff;
    uint64_t* skey = L.skey;
    uint32_t* sidx = L.sidx;
    uint32_t* swave = L.swave;
    uint64_t* s_rng = L.s_rng;
    uint64_t* s_pb = L.s_pb;
    uint32_t* s_seg = L.s_seg;
    if (!rows_take(a, c) || bid >= a.row_blocks) return;  // the sweep takes row_blocks workgroups
    nblk = a.row_blocks < nblk ? a.row_blocks : nblk;
    const uint32_t K = (uint32_t)K64;
    // slots of the first group before element 0 (the output's offset in its 16 bytes)
    const uint32_t head = G == 2 ? a.out_head : (uint32_t)((reinterpret_cast<uintptr_t>(a.out) >> 2) & 3u);
    const uint64_t P = (n + head + G - 1) / G;  // groups
    const uint32_t tid = threadIdx.x;
    const CAFS_GLOBAL uint64_t* off = gp(a.off);
    const CAFS_GLOBAL uint64_t* uq = gp(a.uniq);
    // segments by run count: segment i starts at the group holding the first element
    // of run i * R, so it holds runs i * R - 1 .. (i + 1) * R - 1 at most
    // (rounded down to a multiple of kEmitAlignPairs groups, so that the stores stay
    // aligned to whole cache lines; the rounding adds at most G * kEmitAlignPairs - 1
    // elements, so at most that many runs, in front)
    constexpr uint32_t R = kEmitRowsMaxK - G * kEmitAlignPairs;  // runs starting in a segment
    uint32_t S = (K + R - 1) / R;
    if (S > nblk) S = 1;  // (tiny grids) one segment, searched in global memory below
    if (tid < S)
        s_pb[tid + 1] = tid + 1 == S ? P : (off[(tid + 1) * R] + head) / G / kEmitAlignPairs * kEmitAlignPairs;
    if (tid == 0) s_pb[0] = 0;
    __syncthreads();
    if (tid == 0) {
        // workgroups per segment in proportion to its groups, at least one each
        uint32_t acc = 0;
        s_seg[0] = S;  // none
        for (uint32_t i = 0; i < S; ++i) {
            const uint64_t pairs = s_pb[i + 1] - s_pb[i];
            const uint32_t g = 1 + (uint32_t)((uint64_t)(nblk - S) * pairs / P);
            if (bid < acc + g) {
                s_seg[0] = i;
                s_seg[1] = bid - acc;
                s_seg[2] = g;
                break;
            }
            acc += g;
        }
    }
    __syncthreads();
    const uint32_t seg = s_seg[0];
    if (seg >= S) return;
    const uint32_t w = s_seg[1], gper = s_seg[2];
    const uint64_t sp0 = s_pb[seg], sp1 = s_pb[seg + 1];
    if (sp0 >= sp1) return;
    // the segment's elements [e_first, e_last] and the runs holding them
    const int64_t ef_s = (int64_t)(G * sp0) - (int64_t)head;
    const uint64_t e_first = ef_s < 0 ? 0 : (uint64_t)ef_s;
    const uint64_t el_s = G * sp1 - 1 - head;
    const uint64_t e_last = el_s < n - 1 ? el_s : n - 1;
    if (S == 1) {  // the whole column
        if (tid == 0) {
            s_rng[0] = 0;
            s_rng[1] = K - 1;
        }
    } else if (tid < 128) {
        // the segment starts at most 2 * kEmitAlignPairs - 1 elements before run
        // i * R, so its first run is at most that many runs before; it ends at most
        // 2 * kEmitAlignPairs elements before run (i + 1) * R, so its last run is at
        // most that many runs before that one (wave 0 finds the first, wave 1 the last)
        constexpr uint32_t back = G * kEmitAlignPairs;
        if (tid < 64) {
            const uint32_t a1 = seg * R, a0 = a1 > back ? a1 - back : 0u;
            const uint64_t jl = wave_run_of(a.off, a0, a1, e_first);
            if (tid == 0) s_rng[0] = jl;
        } else {
            const uint32_t b1 = seg + 1 == S ? K - 1 : (seg + 1) * R - 1;
            const uint32_t a0 = seg * R > back ? seg * R - back : 0u;  // at or below the first run
            const uint32_t b0 = b1 > back && b1 - back > a0 ? b1 - back : a0;
            const uint64_t jh = wave_run_of(a.off, b0, b1, e_last);
            if (tid == 64) s_rng[1] = jh;
        }
    }
    __syncthreads();
    const uint32_t j_lo = (uint32_t)s_rng[0], j_hi = (uint32_t)s_rng[1];
    const uint32_t Ks = j_hi - j_lo + 1;
    const uint64_t row = (uint64_t)gper * blockDim.x;
    if (Ks > kEmitRowsMaxK) {
        // too many runs to stage (one segment on a tiny grid): each pair searches the
        // global offsets
        for (uint64_t p = sp0 + (uint64_t)w * blockDim.x + tid; p < sp1; p += row) {
            const int64_t e0s = (int64_t)(G * p) - (int64_t)head;
            if constexpr (G == 2) {
                const uint64_t e0 = e0s < 0 ? 0 : (uint64_t)e0s;
                const uint64_t r0 = run_of(a.off, j_lo, j_hi, e0);
                const uint64_t r1 = (r0 + 1 <= j_hi && (int64_t)off[r0 + 1] <= e0s + 1) ? r0 + 1 : r0;
                store_pair(a.out, n, head, p, uq[r0], uq[r1]);
            } else {
                uint32_t v[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int64_t e = e0s + j;
                    const uint64_t ec = e < 0 ? 0 : ((uint64_t)e < n ? (uint64_t)e : n - 1);
                    v[j] = (uint32_t)uq[run_of(a.off, j_lo, j_hi, ec)];
                }
                store_quad(a.out, n, head, p, v);
            }
        }
        return;
    }
    const uint32_t len = (uint32_t)(e_last - e_first + 1);  // positions below are relative to e_first
    uint32_t s = 0;  // smallest shift with ceil(len / 2^s) <= kEmitIdxSlots
    while ((((uint64_t)len + (1ull << s) - 1) >> s) > kEmitIdxSlots) ++s;
    const uint32_t qn = (uint32_t)(((uint64_t)len + (1ull << s) - 1) >> s);  // index entries inside the segment
    // stage the runs; each run marks the first index entry it holds (runs hold
    // disjoint entry ranges), and a running maximum over the entries fills in the
    // rest: entry q gets the last run starting at or before position q * 2^s
    for (uint32_t q = tid; q < kEmitIdxSlots + 2; q += blockDim.x) sidx[q] = 0;
    __syncthreads();
    for (uint32_t r = tid; r < Ks; r += blockDim.x) {
        const uint64_t g0 = off[j_lo + r];
        const uint32_t o0 = g0 > e_first ? (uint32_t)(g0 - e_first) : 0u;
        const uint32_t o1 = r + 1 < Ks ? (uint32_t)(off[j_lo + r + 1] - e_first) : len;
        soff[r] = o0;
        skey[r] = uq[j_lo + r];
        const uint32_t q0 = (uint32_t)(((uint64_t)o0 + (1ull << s) - 1) >> s);
        const uint32_t q1 = (uint32_t)(((uint64_t)o1 + (1ull << s) - 1) >> s);
        if (q0 < q1) sidx[q0] = r;
    }
    if (tid == 0) soff[Ks] = len;
    __syncthreads();
    // inclusive max-scan of sidx[0, qn): each thread a contiguous chunk
    constexpr uint32_t kPer = kEmitIdxSlots / kEmitRowsThreads;
    static_assert(kPer * kEmitRowsThreads == kEmitIdxSlots, "index chunks");
    uint32_t loc = 0;
#pragma unroll
    for (uint32_t k = 0; k < kPer; ++k) {
        const uint32_t v = sidx[tid * kPer + k];
        loc = v > loc ? v : loc;
    }
    uint32_t inc = loc;  // inclusive max over the wave's threads up to this one
    const uint32_t lane = __lane_id();
#pragma unroll
    for (uint32_t d = 1; d < 64; d <<= 1) {
        const uint32_t o = __shfl_up(inc, d, 64);
        if (lane >= d) inc = o > inc ? o : inc;
    }
    if (lane == 63) swave[tid / 64] = inc;
    __syncthreads();
    uint32_t run = __shfl_up(inc, 1, 64);  // max over the earlier threads of the wave
    if (lane == 0) run = 0;
    for (uint32_t v = 0; v < tid / 64; ++v) run = swave[v] > run ? swave[v] : run;
#pragma unroll
    for (uint32_t k = 0; k < kPer; ++k) {
        const uint32_t q = tid * kPer + k;
        const uint32_t v = sidx[q];
        run = v > run ? v : run;
        sidx[q] = q < qn ? run : Ks - 1;  // entries past the segment point at its last run
    }
    if (tid == 0) { sidx[kEmitIdxSlots] = Ks - 1; sidx[kEmitIdxSlots + 1] = Ks - 1; }
    __syncthreads();

    constexpr int U = kEmitRowsUnroll;
    if constexpr (G == 2) {
        constexpr int U = kEmitRowsUnroll;
        // U rows per step.  Fast case: the index span of the element holds at most one
        // run boundary (hi <= lo + 1), so the pair's keys follow from that boundary's
        // offset and the keys of runs lo and lo + 1: two LDS round trips for all U rows,
        // no loop.  Spans with more boundaries take a binary search.
        for (uint64_t p = sp0 + (uint64_t)w * blockDim.x + tid; p < sp1; p += U * row) {
            int64_t e0s[U];  // first element of the pair, relative to e_first (-1: before the column)
            uint32_t e0[U], lo[U], hi[U];
    #pragma unroll
            for (int u = 0; u < U; ++u) {
                const uint64_t pu = p + u * row;
                e0s[u] = (int64_t)(2 * pu) - (int64_t)head - (int64_t)e_first;
                e0[u] = (pu < sp1 && e0s[u] > 0) ? (uint32_t)e0s[u] : 0u;
                const uint32_t q = e0[u] >> s;
                lo[u] = sidx[q];
                hi[u] = sidx[q + 1];
            }
            uint32_t nb[U];
            uint64_t k0[U], k1[U];
            bool slow = false;
    #pragma unroll
            for (int u = 0; u < U; ++u) {
                nb[u] = soff[lo[u] + 1];
                k0[u] = skey[lo[u]];
                k1[u] = skey[lo[u] + 1 < Ks ? lo[u] + 1 : lo[u]];
                slow |= hi[u] > lo[u] + 1;
            }
            if (slow) {
    #pragma unroll
                for (int u = 0; u < U; ++u) {
                    if (hi[u] <= lo[u] + 1) continue;
                    uint32_t l = lo[u], h = hi[u];
                    while (l < h) {
                        const uint32_t mid = (l + h + 1) >> 1;
                        if (soff[mid] <= e0[u]) l = mid; else h = mid - 1;
                    }
                    // as in the fast case, from the run holding the first element
                    nb[u] = soff[l + 1];
                    k0[u] = skey[l];
                    k1[u] = skey[l + 1 < Ks ? l + 1 : l];
                }
            }
    #pragma unroll
            for (int u = 0; u < U; ++u) {
                const uint64_t v0 = (int64_t)e0[u] >= (int64_t)nb[u] ? k1[u] : k0[u];
                const uint64_t v1 = e0s[u] + 1 >= (int64_t)nb[u] ? k1[u] : k0[u];
                if (p + u * row < sp1) store_pair(a.out, n, head, p + u * row, v0, v1);
            }
        }
    } else {
        // groups of four 32-bit keys: the index spans around the first and the last
        // element of the group; at most one run boundary between them is the fast
        // case, otherwise each element searches
        for (uint64_t p = sp0 + (uint64_t)w * blockDim.x + tid; p < sp1; p += U * row) {
            int64_t e0s[U];
            uint32_t e0[U], lo[U], hi[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const uint64_t pu = p + u * row;
                e0s[u] = (int64_t)(4 * pu) - (int64_t)head - (int64_t)e_first;
                e0[u] = (pu < sp1 && e0s[u] > 0) ? (uint32_t)e0s[u] : 0u;
                const uint32_t q3 = (e0[u] + 3) >> s;
                lo[u] = sidx[e0[u] >> s];
                hi[u] = sidx[(q3 < qn ? q3 : qn) + 1];  // (entries from qn on hold the last run)
            }
            uint32_t nb[U];
            uint64_t k0[U], k1[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                nb[u] = soff[lo[u] + 1];
                k0[u] = skey[lo[u]];
                k1[u] = skey[lo[u] + 1 < Ks ? lo[u] + 1 : lo[u]];
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (p + u * row >= sp1) continue;
                uint32_t v[4];
                if (hi[u] <= lo[u] + 1) {
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const int64_t e = e0s[u] + j;
                        v[j] = (uint32_t)(e >= (int64_t)nb[u] ? k1[u] : k0[u]);
                    }
                } else {
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const int64_t e = e0s[u] + j;
                        const uint32_t ec = e < 0 ? 0u : (e < (int64_t)len ? (uint32_t)e : len - 1);
                        v[j] = (uint32_t)skey[run_in(sidx, soff, s, ec)];
                    }
                }
                store_quad(a.out, n, head, p + u * row, v);
            }
        }
    }
}
__device__ __forceinline__ void emit_rows_body(const Args& a, uint32_t bid, uint32_t nblk) {
    if (!a.c->emit_main) return;
    __shared__ EmitRowsLds L;
    if (a.ew == 4) emit_rows_impl<4>(a, bid, nblk, L);
    else emit_rows_impl<2>(a, bid, nblk, L);
}
CAFS_KERNELS0(emit_rows, kEmitRowsThreads)

// Monotone input: the output is the input.
__device__ __forceinline__ void copy_mono_body(const Args& a, uint32_t bid, uint32_t nblk) {
    Ctrl* c = a.c;
    if (c->path != P_MONOTONE || a.in == a.out) return;
    const uint64_t gtid = (uint64_t)bid * blockDim.x + threadIdx.x;
    const uint64_t gstride = (uint64_t)nblk * blockDim.x;
    for (uint64_t i = gtid; i < a.n; i += gstride) store_key(a.out, i, load_key(a.in, i, a.ew), a.ew);
}
CAFS_KERNELS0(copy_mono, 256)

// Run-length pass over the sorted output, needed when the column was not counted
// (monotone input, radix engine) but the report needs K, or the counts or the
// guard need the (key, count) pairs.  The first pass alone gives K; the pairs are
// written only when they are needed.
__device__ __forceinline__ bool rle_needed(const Args& a, const Ctrl* c) {
    if (c->dense_ready && !c->overflow) return false;
    return a.want_report || a.want_counts || (c->path == P_MAIN);
}
__device__ __forceinline__ bool rle_pairs_needed(const Args& a, const Ctrl* c) {
    if (c->dense_ready && !c->overflow) return false;
    return a.want_counts || (c->path == P_MAIN);
}

// Pass 1: runs starting in each tile; the last workgroup scans the tile counts.
__device__ __forceinline__ void rle_count_body(const Args& a, uint32_t bid, uint32_t nblk) {
    Ctrl* c = a.c;
    if (!rle_needed(a, c)) return;
    const uint64_t n = a.n;
    const uint64_t* y = c->sorted;
    const uint32_t yw = c->sorted_ew;
    const uint64_t tiles = (n + kRleTile - 1) / kRleTile;
    __shared__ uint32_t s_cnt;
    __shared__ uint32_t s_last;
    __shared__ uint64_t scan_tmp[8];
    for (uint64_t t = bid; t < tiles; t += nblk) {
        if (threadIdx.x == 0) s_cnt = 0;
        __syncthreads();
        const uint64_t b = t * kRleTile;
        const uint64_t e = (b + kRleTile < n) ? b + kRleTile : n;
        uint32_t local = 0;
        constexpr uint32_t G = kRleTile / 256;  // elements per thread, loads all in flight
        uint64_t cur[G], prv[G];
#pragma unroll
        for (uint32_t u = 0; u < G; ++u) {
            const uint64_t i = b + (uint64_t)u * blockDim.x + threadIdx.x;
            cur[u] = i < e ? load_key(y, i, yw) : 0;
            prv[u] = (i < e && i > 0) ? load_key(y, i - 1, yw) : ~cur[u];  // element 0 starts a run
        }
#pragma unroll
        for (uint32_t u = 0; u < G; ++u) {
            const uint64_t i = b + (uint64_t)u * blockDim.x + threadIdx.x;
            local += (i < e && cur[u] != prv[u]) ? 1u : 0u;
        }
        local = wave_sum_u32(local);
        if (__lane_id() == 0) atomicAdd(&s_cnt, local);
        __syncthreads();
        if (threadIdx.x == 0) a.rle_tile[t] = s_cnt;
        __syncthreads();
    }
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) s_last = (atomicAdd(&c->rle_done, 1u) == nblk - 1);
    __syncthreads();
    if (!s_last) return;
    __threadfence();
    // exclusive scan of the tile counts (one workgroup, contiguous chunks per thread)
    const uint64_t per = (tiles + blockDim.x - 1) / blockDim.x;
    const uint64_t b0 = threadIdx.x * per < tiles ? threadIdx.x * per : tiles;
    const uint64_t b1 = b0 + per < tiles ? b0 + per : tiles;
    // (loads in groups of 8 in flight: one after the other, device-scope loads
    // queue for microseconds each)
    constexpr uint32_t G = 8;
    uint64_t local = 0;
    for (uint64_t i = b0; i < b1; i += G) {
        uint64_t v[G];
#pragma unroll
        for (uint32_t u = 0; u < G; ++u) v[u] = i + u < b1 ? atomic_load_agent(&a.rle_tile[i + u]) : 0;
#pragma unroll
        for (uint32_t u = 0; u < G; ++u) local += v[u];
    }
    uint64_t total;
    uint64_t run = block_exclusive_scan<uint64_t>(local, scan_tmp, &total);
    for (uint64_t i = b0; i < b1; i += G) {
        uint64_t v[G];
#pragma unroll
        for (uint32_t u = 0; u < G; ++u) v[u] = i + u < b1 ? atomic_load_agent(&a.rle_tile[i + u]) : 0;
#pragma unroll
        for (uint32_t u = 0; u < G; ++u) {
            if (i + u < b1) a.rle_tile[i + u] = run;
            run += v[u];
        }
    }
    if (threadIdx.x == 0) c->K = total;
}
CAFS_KERNELS0(rle_count, 256)

// Pass 2: write each run's key and start position (its offset).  A tile is staged
// in LDS with coalesced loads; each thread flags the run starts among 16
// consecutive elements, a block scan places them, and the tile's runs are written
// back with coalesced stores (their places in the output are consecutive).
__device__ __forceinline__ void rle_write_body(const Args& a, uint32_t bid, uint32_t nblk) {
    Ctrl* c = a.c;
    if (!rle_pairs_needed(a, c)) return;
    const uint64_t n = a.n;
    const uint64_t* y = c->sorted;
    const uint32_t yw = c->sorted_ew;
    CAFS_GLOBAL uint64_t* __restrict__ uq = gp(a.uniq);
    CAFS_GLOBAL uint64_t* __restrict__ off = gp(a.off);
    const uint64_t tiles = (n + kRleTile - 1) / kRleTile;
    constexpr uint32_t per = kRleTile / 256;  // contiguous elements per thread
    __shared__ uint64_t sy[kRleTile + 1];     // sy[i + 1] = y[b + i]; sy[0] = y[b - 1]
    __shared__ uint16_t spos[kRleTile];       // tile-relative start of each run
    __shared__ uint32_t scan_tmp[8];
    for (uint64_t t = bid; t < tiles; t += nblk) {
        const uint64_t b = t * kRleTile;
        const uint32_t cnt = (uint32_t)(n - b < kRleTile ? n - b : kRleTile);
        for (uint32_t i = threadIdx.x; i < cnt; i += blockDim.x) sy[i + 1] = load_key(y, b + i, yw);
        if (threadIdx.x == 0) sy[0] = b > 0 ? load_key(y, b - 1, yw) : ~load_key(y, 0, yw);  // element 0 starts a run
        __syncthreads();
        const uint32_t l0 = threadIdx.x * per;
        uint32_t flags = 0;
#pragma unroll
        for (uint32_t k = 0; k < per; ++k) {
            const uint32_t i = l0 + k;
            flags |= (i < cnt && sy[i + 1] != sy[i]) ? (1u << k) : 0u;
        }
        uint32_t total;
        const uint32_t ex = block_exclusive_scan<uint32_t>((uint32_t)__popc(flags), scan_tmp, &total);
        // the staged keys are read before the barrier and the runs written after it
        uint64_t keys[per];
#pragma unroll
        for (uint32_t k = 0; k < per; ++k) keys[k] = sy[l0 + k + 1];
        __syncthreads();
        uint32_t j = ex;
#pragma unroll
        for (uint32_t k = 0; k < per; ++k) {
            if ((flags >> k) & 1u) {
                sy[j] = keys[k];
                spos[j] = (uint16_t)(l0 + k);
                ++j;
            }
        }
        __syncthreads();
        const uint64_t j0 = a.rle_tile[t];
        for (uint32_t r = threadIdx.x; r < total; r += blockDim.x) {
            uq[j0 + r] = sy[r];
            off[j0 + r] = b + spos[r];
        }
        __syncthreads();
    }
    if (bid == 0 && threadIdx.x == 0) a.off[c->K] = n;
}
CAFS_KERNELS0(rle_write, 256)

// Pass 3: counts from consecutive offsets; marks the pairs ready for the guard.
__device__ __forceinline__ void rle_counts_body(const Args& a, uint32_t bid, uint32_t nblk) {
    Ctrl* c = a.c;
    if (!rle_pairs_needed(a, c)) return;
    const uint64_t K = c->K;
    const uint64_t gtid = (uint64_t)bid * blockDim.x + threadIdx.x;
    const uint64_t gstride = (uint64_t)nblk * blockDim.x;
    for (uint64_t jj = gtid; jj < K; jj += gstride) a.cnt[jj] = a.off[jj + 1] - a.off[jj];
}
CAFS_KERNELS0(rle_counts, 256)

// In-place main-path sort by the radix engine: the sorted column waited in
// scratch until the guard had read the input.
__device__ __forceinline__ void copy_deferred_body(const Args& a, uint32_t bid, uint32_t nblk) {
    const Ctrl* c = a.c;
    if (!c->deferred_copy) return;
    const uint64_t* src = c->sorted;
    const uint32_t sw = c->sorted_ew;
    const uint64_t gtid = (uint64_t)bid * blockDim.x + threadIdx.x;
    const uint64_t gstride = (uint64_t)nblk * blockDim.x;
    for (uint64_t i = gtid; i < a.n; i += gstride) store_key(a.out, i, load_key(src, i, sw), a.ew);
}
CAFS_KERNELS0(copy_deferred, 256)

// 32-bit keys: the distinct keys, kept as 64-bit values in the workspace, into the
// caller's 32-bit array.
__device__ __forceinline__ void uniq_out_body(const Args& a, uint32_t bid, uint32_t nblk) {
    if (a.ew != 4 || !a.uniq_out) return;
    const uint64_t K = a.c->K;
    const uint64_t gtid = (uint64_t)bid * blockDim.x + threadIdx.x;
    const uint64_t gstride = (uint64_t)nblk * blockDim.x;
    CAFS_GLOBAL uint32_t* dst = gp(static_cast<uint32_t*>(a.uniq_out));
    for (uint64_t j = gtid; j < K; j += gstride) dst[j] = (uint32_t)gp(a.uniq)[j];
}
CAFS_KERNELS0(uniq_out, 256)

}  // namespace cafs
