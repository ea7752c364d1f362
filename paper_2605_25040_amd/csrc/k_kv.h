// Key-value variant: one 64-bit payload per key.  The keys come out as in the
// keys-only sort; each payload lands at its key's position, equal keys in input
// order (a stable sort by key).
//
// On the count paths the sorted keys are written by the run expansion as usual, and
// the payloads are placed by an LSD sort of (rank, payload) on the digits of the
// rank, the key's position among the distinct keys: one pass of 8-bit digits per
// byte of K - 1 (one for K <= 256, two for K <= 65536) instead of the radix
// engine's passes over the keys' 64 bits.  A digit's histogram over the whole
// column is a sum of the dense counts.
//
// Each pass is reduce-then-scan over a fixed split of the column into chunks (one
// workgroup each), so that no workgroup waits for another:
//   kv_up     per chunk, the histogram of the pass's digit (the first pass also
//             looks every key's rank up in a hash table built from the distinct
//             keys and writes the ranks as 32-bit words);
//   kv_scan   one workgroup turns the chunk histograms into each chunk's starting
//             position per digit (exclusive prefix over the chunks plus the digit's
//             global base);
//   kv_down   each workgroup walks its chunk in tiles, in order: the stable rank of
//             every element within its digit (wave ballots), then each element is
//             written at its chunk's running position for its digit.
// On the radix engine's paths (high K, short columns, a spill past its limit) the
// payloads travel with the keys through the key-value radix passes; a monotone
// column's payloads are copied.
#pragma once
#include "cafs_dev.h"
#include "k_radix.h"

namespace cafs {

constexpr uint32_t kKvThreads = 256;
constexpr uint32_t kKvItems = 16;                        // elements per thread per tile
constexpr uint32_t kKvTile = kKvThreads * kKvItems;      // 4096
constexpr uint32_t kKvLdsSlotsLog2 = 11;                 // lookup tables this small are read from LDS
constexpr uint32_t kKvMinSlotsLog2 = 6;
constexpr uint32_t kKvMaxChunks = 1024;
constexpr uint32_t kKvUnitsPerChunk = 4;                 // upsweep workgroups per placement workgroup
constexpr uint32_t kKvUpItems = 8;                       // keys per thread in flight in the first upsweep
constexpr uint32_t kKvTagEmpty = 0;                      // tags hold rank + 1

// One slot of the rank lookup table: a distinct key and its rank + 1 (0: empty).
struct alignas(16) KvSlot {
    uint64_t key;
    uint32_t tag;
    uint32_t pad;
};

// The column is split into `units` equal runs of tiles (the last one short or
// empty), one per upsweep workgroup; a placement workgroup takes kKvUnitsPerChunk
// consecutive units (a chunk).
__host__ __device__ inline uint64_t kv_unit_tiles(uint64_t n, uint32_t units) {
    const uint64_t tiles = (n + kKvTile - 1) / kKvTile;
    return (tiles + units - 1) / units;
}

// The scratch of the payload placement, all in workspace regions the count no
// longer needs: ranks (32-bit) and payloads ping-pong between two buffers each; the
// lookup table; the chunk histograms.
__device__ __forceinline__ uint32_t* kv_r(const Args& a, uint32_t i) { return (i & 1u) ? a.first_idx : a.clist; }
__device__ __forceinline__ uint64_t* kv_v(const Args& a, uint32_t i) { return (i & 1u) ? a.tmp_k : a.spill_v; }
__device__ __forceinline__ KvSlot* kv_table(const Args& a) { return reinterpret_cast<KvSlot*>(a.pbuf); }
__device__ __forceinline__ uint32_t* kv_part(const Args& a) { return reinterpret_cast<uint32_t*>(a.status); }

// Plan the payload placement after the count: active only on the count paths
// (tiny, main, guard) with dense arrays.
__device__ __forceinline__ void kv_setup_body(const Args& a, uint32_t, uint32_t) {
    if (threadIdx.x != 0 || !a.vin) return;
    Ctrl* c = a.c;
    c->kv_on = 0;
    if (c->path == P_MONOTONE || c->engine == E_RADIX || c->overflow || !c->dense_ready) return;
    const uint64_t K = c->K;
    uint32_t P = 0;
    for (uint64_t r = K > 0 ? K - 1 : 0; r; r >>= 8) ++P;
    // load at most 1/2
    uint32_t lg = log2_pow2(bit_ceil64(2 * K));
    if (lg < kKvMinSlotsLog2) lg = kKvMinSlotsLog2;
    const uint32_t mode = lg <= kKvLdsSlotsLog2 ? 0u : (lg <= a.kv_tab_log2 ? 1u : 2u);
    c->kv_passes = P;
    c->kv_slots_log2 = lg;
    c->kv_mode = mode;
    for (uint32_t p = 0; p < 4; ++p)
        for (uint32_t b = 0; b < 256; ++b) c->hist[p][b] = 0;
    c->hist_done = 0;
    c->kv_on = 1;
}
CAFS_KERNELS0(kv_setup, 64)

// Clear the lookup table.
__device__ __forceinline__ void kv_clear_body(const Args& a, uint32_t bid, uint32_t nblk) {
    if (!a.vin) return;
    const Ctrl* c = a.c;
    if (!c->kv_on || c->kv_passes == 0 || c->kv_mode == 2) return;
    const uint64_t gtid = (uint64_t)bid * blockDim.x + threadIdx.x;
    const uint64_t gstride = (uint64_t)nblk * blockDim.x;
    const uint64_t slots = 1ull << c->kv_slots_log2;
    for (uint64_t i = gtid; i < slots; i += gstride) gp(&kv_table(a)[i].tag)[0] = kKvTagEmpty;
}
CAFS_KERNELS0(kv_clear, 256)

// Insert every distinct key with its rank (linear probing; the keys are distinct,
// so an insert takes the first free slot), and add each rank's count to the
// histogram of each of its digits; the last workgroup turns the histograms into
// the digit bases of every pass.
__device__ __forceinline__ void kv_build_body(const Args& a, uint32_t bid, uint32_t nblk) {
    if (!a.vin) return;
    Ctrl* c = a.c;
    if (!c->kv_on || c->kv_passes == 0) return;
    const uint32_t P = c->kv_passes;
    const uint64_t K = c->K;
    const uint32_t lg = c->kv_slots_log2;
    const uint64_t mask = (1ull << lg) - 1;
    const bool table = c->kv_mode < 2;
    __shared__ uint32_t lh[4][256];
    __shared__ uint32_t s_last;
    __shared__ uint64_t scan_tmp[8];
    for (uint32_t i = threadIdx.x; i < 4 * 256; i += blockDim.x) (&lh[0][0])[i] = 0;
    __syncthreads();
    const uint64_t gtid = (uint64_t)bid * blockDim.x + threadIdx.x;
    const uint64_t gstride = (uint64_t)nblk * blockDim.x;
    for (uint64_t r = gtid; r < K; r += gstride) {
        if (table) {
            const uint64_t key = a.uniq[r];
            uint64_t h = mul_hash32(key, lg, a.table_mul);
            for (uint64_t probe = 0; probe <= mask; ++probe) {
                if (g_cas(&kv_table(a)[h].tag, kKvTagEmpty, (uint32_t)(r + 1)) == kKvTagEmpty) {
                    gp(&kv_table(a)[h].key)[0] = key;
                    break;
                }
                h = (h + 1) & mask;
            }
        }
        const uint32_t cnt = (uint32_t)a.cnt[r];
        for (uint32_t p = 0; p < P; ++p) atomicAdd(&lh[p][(r >> (8 * p)) & 255u], cnt);
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < P * 256; i += blockDim.x) {
        const uint32_t h = (&lh[0][0])[i];
        if (h) atomicAdd((unsigned long long*)&(&c->hist[0][0])[i], (unsigned long long)h);
    }
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) s_last = (atomicAdd(&c->hist_done, 1u) == nblk - 1);
    __syncthreads();
    if (!s_last) return;
    __threadfence();
    for (uint32_t p = 0; p < P; ++p) {  // blockDim.x == 256: one bin per thread
        const uint64_t h = atomic_load_agent(&c->hist[p][threadIdx.x]);
        uint64_t total;
        const uint64_t ex = block_exclusive_scan<uint64_t>(h, scan_tmp, &total);
        c->hist[p][threadIdx.x] = ex;
    }
}
CAFS_KERNELS0(kv_build, 256)

// Slot i of a table in memory (two 8-byte loads of one 16-byte slot).
__device__ __forceinline__ KvSlot kv_slot_global(const KvSlot* tab, uint64_t i) {
    const CAFS_GLOBAL uint64_t* p = gp(reinterpret_cast<const uint64_t*>(tab)) + 2 * i;
    KvSlot s;
    s.key = p[0];
    s.tag = (uint32_t)p[1];
    s.pad = 0;
    return s;
}

// Ranks of a thread's keys.  The first probe of every key is issued before any is
// checked; keys that miss it (a collision in a table at load <= 1/2) probe on.
template <bool LDS, uint32_t NI>
__device__ __forceinline__ void kv_lookup_items(const Args& a, const KvSlot* tab, uint32_t lg, const uint64_t* key,
                                                uint32_t* rk, uint32_t okm) {
    const uint32_t mask = (1u << lg) - 1;
    uint32_t h[NI];
    KvSlot s[NI];
#pragma unroll
    for (int i = 0; i < (int)NI; ++i) {
        h[i] = mul_hash32(key[i], lg, a.table_mul);
        s[i] = LDS ? tab[h[i]] : kv_slot_global(tab, h[i]);
    }
#pragma unroll
    for (int i = 0; i < (int)NI; ++i) {
        uint32_t r = 0;
        if ((okm >> i) & 1u) {
            KvSlot t = s[i];
            uint32_t hh = h[i];
            for (uint32_t probe = 0; probe <= mask; ++probe) {
                if (t.tag == kKvTagEmpty) break;  // not reached: every key is a distinct key
                if (t.key == key[i]) {
                    r = t.tag - 1;
                    break;
                }
                hh = (hh + 1) & mask;
                t = LDS ? tab[hh] : kv_slot_global(tab, hh);
            }
        }
        rk[i] = r;
    }
}

// Rank by binary search of the dense keys (ordered by order key), for tables that
// would not fit the workspace.
__device__ __forceinline__ uint32_t kv_bsearch(const Args& a, uint64_t key, uint64_t K) {
    const uint64_t ok = okey(key, a.flip, a.fneg);
    uint64_t lo = 0, hi = K;
    while (lo < hi) {
        const uint64_t mid = (lo + hi) >> 1;
        if (okey(gp(a.uniq)[mid], a.flip, a.fneg) < ok) lo = mid + 1;
        else hi = mid;
    }
    return (uint32_t)lo;
}

// Lanes (within `act`) whose digit equals this lane's, comparing the low `nbits`
// bits (the digit's other bits are zero).
__device__ __forceinline__ uint64_t kv_match(uint32_t dg, uint64_t act, uint32_t nbits) {
    uint64_t peers = act;
    for (uint32_t b = 0; b < nbits; ++b) {
        const bool bit = (dg >> b) & 1u;
        const uint64_t m = __ballot(bit);
        peers &= bit ? m : ~m;
    }
    return peers;
}

// Bits the digits of a pass can take: all 8, except in the top pass, whose digits
// are at most (K - 1) >> 8 * pass.
__device__ __forceinline__ uint32_t kv_digit_bits(const Ctrl* c, uint32_t pass) {
    if (pass + 1 < c->kv_passes) return 8u;
    const uint32_t top = (uint32_t)(((c->K - 1) >> (8 * pass)) & 255u);
    return top ? 32u - __clz(top) : 0u;
}

// Digit counts of one wave's item.  Digits of at most 4 bits: matched by ballots,
// one LDS add per distinct digit.  Wider digits: one LDS add for the wave when
// every active lane has the same digit, else one per lane (adds without return;
// lanes with equal digits serialize in the LDS, which costs less than 8 ballots).
__device__ __forceinline__ void kv_count_digit(uint32_t* lh_wave, uint32_t dg, bool ok, uint32_t lane,
                                               uint32_t nbits) {
    const uint64_t act = __ballot(ok);
    if (act == 0) return;
    if (nbits <= 4) {
        const uint64_t peers = kv_match(dg, act, nbits);
        if (ok && (peers & ((1ull << lane) - 1)) == 0) atomicAdd(&lh_wave[dg], (uint32_t)__popcll(peers));
        return;
    }
    const int leader = __ffsll((unsigned long long)act) - 1;
    const uint32_t first = __shfl(dg, leader, 64);
    if (__ballot(ok && dg == first) == act) {
        if ((int)lane == leader) atomicAdd(&lh_wave[dg], (uint32_t)__popcll(act));
    } else if (ok) {
        atomicAdd(&lh_wave[dg], 1u);
    }
}

// Elements [e0, e1) of run `bid` of `nblk` runs of `per` units each.
__device__ __forceinline__ void kv_range(uint64_t n, uint32_t bid, uint32_t nblk, uint32_t per, uint64_t& e0,
                                         uint64_t& e1) {
    const uint64_t span = kv_unit_tiles(n, nblk * per) * per * kKvTile;
    e0 = (uint64_t)bid * span;
    e1 = e0 + span < n ? e0 + span : n;
    if (e0 > n) e0 = n;
}

// First pass, upsweep: every key's rank by lookup, written as a 32-bit word, and
// the unit's histogram of the rank's low digit.  Two instances: the lookup table
// copied into LDS (small K), or probed in memory / a binary search (larger K).
template <bool LDS_TABLE>
__device__ __forceinline__ void kv_up0_impl(const Args& a, uint32_t bid, uint32_t nblk) {
    if (!a.vin) return;
    const Ctrl* c = a.c;
    if (!c->kv_on || c->kv_passes == 0 || (c->kv_mode == 0) != LDS_TABLE) return;
    const uint64_t n = a.n;
    const uint32_t mode = c->kv_mode, lg = c->kv_slots_log2;
    const uint64_t K = c->K;
    const uint32_t nbits = kv_digit_bits(c, 0);
    __shared__ KvSlot s_tab[LDS_TABLE ? (1u << kKvLdsSlotsLog2) : 1];
    __shared__ uint32_t lh[kKvThreads / 64][256];
    const uint32_t tid = threadIdx.x, lane = __lane_id(), wave = tid >> 6;
    for (uint32_t i = tid; i < (kKvThreads / 64) * 256; i += blockDim.x) (&lh[0][0])[i] = 0;
    if (LDS_TABLE)
        for (uint32_t i = tid; i < (1u << lg); i += blockDim.x) s_tab[i] = kv_slot_global(kv_table(a), i);
    __syncthreads();
    uint64_t e0, e1;
    kv_range(n, bid, nblk, 1, e0, e1);
    CAFS_GLOBAL uint32_t* __restrict__ wr = gp(kv_r(a, 0));
    constexpr uint32_t STEP = kKvThreads * kKvUpItems;
    // the next step's keys are loaded before this step is worked on
    uint64_t key[kKvUpItems], nkey[kKvUpItems];
    uint32_t okm = 0, nokm = 0;
    auto load = [&](uint64_t base, uint64_t* k, uint32_t& m) {
        m = 0;
#pragma unroll
        for (int i = 0; i < (int)kKvUpItems; ++i) {
            const uint64_t pos = base + (uint64_t)i * kKvThreads + tid;
            const bool ok = pos < e1;
            k[i] = ok ? load_key(a.in, pos, a.ew) : 0;
            m |= (ok ? 1u : 0u) << i;
        }
    };
    if (e0 < e1) load(e0, key, okm);
    for (uint64_t base = e0; base < e1; base += STEP) {
        if (base + STEP < e1) load(base + STEP, nkey, nokm);
        uint32_t rk[kKvUpItems];
        if (LDS_TABLE) {
            kv_lookup_items<true, kKvUpItems>(a, s_tab, lg, key, rk, okm);
        } else if (mode == 1) {
            kv_lookup_items<false, kKvUpItems>(a, kv_table(a), lg, key, rk, okm);
        } else {
#pragma unroll
            for (int i = 0; i < (int)kKvUpItems; ++i) rk[i] = ((okm >> i) & 1u) ? kv_bsearch(a, key[i], K) : 0u;
        }
#pragma unroll
        for (int i = 0; i < (int)kKvUpItems; ++i) {
            const uint64_t pos = base + (uint64_t)i * kKvThreads + tid;
            if ((okm >> i) & 1u) wr[pos] = rk[i];
            kv_count_digit(lh[wave], rk[i] & 255u, (okm >> i) & 1u, lane, nbits);
        }
#pragma unroll
        for (int i = 0; i < (int)kKvUpItems; ++i) key[i] = nkey[i];
        okm = nokm;
    }
    __syncthreads();
    uint32_t s = 0;
#pragma unroll
    for (uint32_t w = 0; w < kKvThreads / 64; ++w) s += lh[w][tid];
    gp(kv_part(a))[(uint64_t)bid * 256 + tid] = s;
}
__device__ __forceinline__ void kv_up0_lds_body(const Args& a, uint32_t bid, uint32_t nblk) {
    kv_up0_impl<true>(a, bid, nblk);
}
__device__ __forceinline__ void kv_up0_mem_body(const Args& a, uint32_t bid, uint32_t nblk) {
    kv_up0_impl<false>(a, bid, nblk);
}
CAFS_KERNELS0(kv_up0_lds, kKvThreads)
CAFS_KERNELS0(kv_up0_mem, kKvThreads)

// Later passes, upsweep: the chunk's histogram of the pass's digit of the ranks
// the previous pass wrote (16-byte loads of four ranks).
__device__ __forceinline__ void kv_up_body(const Args& a, uint32_t pass, uint32_t bid, uint32_t nblk) {
    if (!a.vin) return;
    const Ctrl* c = a.c;
    if (!c->kv_on || pass == 0 || pass >= c->kv_passes) return;
    const uint64_t n = a.n;
    const uint32_t shift = 8 * pass;
    const uint32_t nbits = kv_digit_bits(c, pass);
    __shared__ uint32_t lh[kKvThreads / 64][256];
    const uint32_t tid = threadIdx.x, lane = __lane_id(), wave = tid >> 6;
    for (uint32_t i = tid; i < (kKvThreads / 64) * 256; i += blockDim.x) (&lh[0][0])[i] = 0;
    __syncthreads();
    uint64_t e0, e1;
    kv_range(n, bid, nblk, 1, e0, e1);
    const CAFS_GLOBAL uint32_t* __restrict__ sr = gp(kv_r(a, pass));
    const CAFS_GLOBAL uint64_t* __restrict__ sr8 = reinterpret_cast<const CAFS_GLOBAL uint64_t*>(sr);
    constexpr uint32_t V = kKvItems / 4;  // four ranks (16 bytes) per load per thread and tile
    uint4 q[V], nq[V];
    uint32_t okm = 0, nokm = 0;
    auto load = [&](uint64_t base, uint4* q, uint32_t& okm) {
        okm = 0;
#pragma unroll
        for (uint32_t i = 0; i < V; ++i) {
            const uint64_t pos = base + 4 * ((uint64_t)i * kKvThreads + tid);  // (chunks start at tile edges)
            if (pos + 4 <= e1) {
                const uint64_t lo = sr8[pos >> 1], hi = sr8[(pos >> 1) + 1];
                q[i].x = (uint32_t)lo;
                q[i].y = (uint32_t)(lo >> 32);
                q[i].z = (uint32_t)hi;
                q[i].w = (uint32_t)(hi >> 32);
                okm |= 15u << (4 * i);
            } else {
                q[i].x = pos < e1 ? sr[pos] : 0u;
                q[i].y = pos + 1 < e1 ? sr[pos + 1] : 0u;
                q[i].z = pos + 2 < e1 ? sr[pos + 2] : 0u;
                q[i].w = 0u;
                okm |= (uint32_t)((pos < e1) | ((pos + 1 < e1) << 1) | ((pos + 2 < e1) << 2)) << (4 * i);
            }
        }
    };
    if (e0 < e1) load(e0, q, okm);
    for (uint64_t base = e0; base < e1; base += kKvTile) {
        if (base + kKvTile < e1) load(base + kKvTile, nq, nokm);
#pragma unroll
        for (uint32_t i = 0; i < V; ++i) {
            kv_count_digit(lh[wave], (q[i].x >> shift) & 255u, (okm >> (4 * i)) & 1u, lane, nbits);
            kv_count_digit(lh[wave], (q[i].y >> shift) & 255u, (okm >> (4 * i + 1)) & 1u, lane, nbits);
            kv_count_digit(lh[wave], (q[i].z >> shift) & 255u, (okm >> (4 * i + 2)) & 1u, lane, nbits);
            kv_count_digit(lh[wave], (q[i].w >> shift) & 255u, (okm >> (4 * i + 3)) & 1u, lane, nbits);
        }
#pragma unroll
        for (uint32_t i = 0; i < V; ++i) q[i] = nq[i];
        okm = nokm;
    }
    __syncthreads();
    uint32_t s = 0;
#pragma unroll
    for (uint32_t w = 0; w < kKvThreads / 64; ++w) s += lh[w][tid];
    gp(kv_part(a))[(uint64_t)bid * 256 + tid] = s;
}
CAFS_KERNELS1(kv_up, kKvThreads, uint32_t, pass)

// Unit histograms -> each unit's first position per digit: exclusive prefix over
// the units, plus the digit's global base.  One workgroup of 1024 threads per
// digit; each thread takes up to four consecutive units.
__device__ __forceinline__ void kv_scan_body(const Args& a, uint32_t pass, uint32_t units) {
    if (!a.vin) return;
    const Ctrl* c = a.c;
    if (!c->kv_on || pass >= c->kv_passes) return;
    CAFS_GLOBAL uint32_t* part = gp(kv_part(a));
    const uint32_t d = blockIdx.x;
    const uint32_t per = (units + blockDim.x - 1) / blockDim.x;  // <= 4
    const uint32_t u0 = threadIdx.x * per;
    uint32_t v[4];
    uint32_t s = 0;
#pragma unroll
    for (uint32_t j = 0; j < 4; ++j) {
        v[j] = (j < per && u0 + j < units) ? part[(uint64_t)(u0 + j) * 256 + d] : 0u;
        s += v[j];
    }
    __shared__ uint32_t scan_tmp[17];
    uint32_t total;
    uint32_t run = (uint32_t)c->hist[pass][d] + block_exclusive_scan<uint32_t>(s, scan_tmp, &total);
#pragma unroll
    for (uint32_t j = 0; j < 4; ++j)
        if (j < per && u0 + j < units) {
            part[(uint64_t)(u0 + j) * 256 + d] = run;
            run += v[j];
        }
}
__global__ __launch_bounds__(1024) void k_kv_scan(Args a, uint32_t pass, uint32_t units) {
    kv_scan_body(a, pass, units);
}

// One placement pass: each workgroup walks its chunk's tiles in order.  Per tile:
// the stable rank of every element within its digit (wave ballots), a reorder of
// the tile by digit in LDS, and writes of each digit's run at the chunk's running
// position for that digit (stable: within a digit, positions follow element order).
// The last pass writes only the payloads, to the output.
struct KvDownLds {
    uint64_t lv[kKvTile];             // the tile's payloads, reordered by digit
    uint32_t lx[kKvTile];             // their ranks (last pass: their digits)
    uint32_t wcnt[kKvThreads / 64][256];
    uint32_t run[256];
    uint32_t toff[256];
    uint32_t gofs[256];
    uint32_t scan_tmp[8];
};

template <bool LAST>
__device__ __forceinline__ void kv_down_impl(const Args& a, uint32_t pass, uint32_t bid, uint32_t nblk,
                                             KvDownLds& L) {
    const uint64_t n = a.n;
    const uint32_t tid = threadIdx.x, lane = __lane_id(), wave = tid >> 6;
    const uint32_t shift = 8 * pass;
    const CAFS_GLOBAL uint32_t* __restrict__ sr = gp(kv_r(a, pass));
    const CAFS_GLOBAL uint64_t* __restrict__ sv = gp(pass == 0 ? a.vin : kv_v(a, pass));
    CAFS_GLOBAL uint32_t* __restrict__ dr = gp(kv_r(a, pass + 1));
    CAFS_GLOBAL uint64_t* __restrict__ dv = gp(LAST ? a.vout : kv_v(a, pass + 1));
    uint64_t* lv = L.lv;
    uint32_t* lx = L.lx;
    uint32_t (*wcnt)[256] = L.wcnt;
    uint32_t* run = L.run;
    uint32_t* toff = L.toff;
    uint32_t* gofs = L.gofs;
    run[tid] = gp(kv_part(a))[(uint64_t)bid * kKvUnitsPerChunk * 256 + tid];  // blockDim.x == 256
    uint64_t e0, e1;
    kv_range(n, bid, nblk, kKvUnitsPerChunk, e0, e1);
    const uint64_t lt_mask = (1ull << lane) - 1;
    const uint32_t nbits = kv_digit_bits(a.c, pass);
    // wave w owns elements base + w*1024 + i*64 + lane: element order is (w, i, lane).
    // The next tile is loaded before this tile is worked on.
    uint32_t rk[kKvItems], nrk[kKvItems];
    uint64_t val[kKvItems], nval[kKvItems];
    uint32_t okm = 0, nokm = 0;
    auto load = [&](uint64_t base, uint32_t* r, uint64_t* v, uint32_t& m) {
        m = 0;
#pragma unroll
        for (int i = 0; i < (int)kKvItems; ++i) {
            const uint64_t pos = base + (uint64_t)wave * (64 * kKvItems) + (uint64_t)i * 64 + lane;
            const bool ok = pos < e1;
            r[i] = ok ? sr[pos] : 0u;
            v[i] = ok ? sv[pos] : 0;
            m |= (ok ? 1u : 0u) << i;
        }
    };
    if (e0 < e1) load(e0, rk, val, okm);
    for (uint64_t base = e0; base < e1; base += kKvTile) {
        for (uint32_t i = tid; i < (kKvThreads / 64) * 256; i += blockDim.x) (&wcnt[0][0])[i] = 0;
        if (base + kKvTile < e1) load(base + kKvTile, nrk, nval, nokm);
        uint32_t rank2[kKvItems / 2];
        __syncthreads();  // wcnt cleared
#pragma unroll
        for (int i = 0; i < (int)kKvItems; ++i) {
            const bool ok = (okm >> i) & 1u;
            const uint32_t dg = (rk[i] >> shift) & 255u;
            const uint64_t act = __ballot(ok);
            const uint64_t peers = kv_match(dg, act, nbits);
            uint32_t before = 0;
            if (ok) before = wcnt[wave][dg];
            const uint32_t r = before + (uint32_t)__popcll(peers & lt_mask);
            if (i & 1) rank2[i >> 1] |= r << 16; else rank2[i >> 1] = r;
            const bool leader = ok && ((peers & lt_mask) == 0);
            if (leader) wcnt[wave][dg] = before + (uint32_t)__popcll(peers);
        }
        __syncthreads();
        // per digit (thread = digit): exclusive prefix over the waves; the tile's
        // digit offsets; where the digit's run goes in the output
        uint32_t tot = 0;
#pragma unroll
        for (uint32_t w = 0; w < kKvThreads / 64; ++w) {
            const uint32_t cw = wcnt[w][tid];
            wcnt[w][tid] = tot;
            tot += cw;
        }
        {
            uint32_t total;
            const uint32_t ex = block_exclusive_scan<uint32_t>(tot, L.scan_tmp, &total);
            toff[tid] = ex;
            gofs[tid] = run[tid] - ex;  // (mod 2^32: a slot q of digit d goes to gofs[d] + q)
            run[tid] += tot;
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < (int)kKvItems; ++i) {
            if ((okm >> i) & 1u) {
                const uint32_t dg = (rk[i] >> shift) & 255u;
                const uint32_t q = toff[dg] + wcnt[wave][dg] + ((rank2[i >> 1] >> (16 * (i & 1))) & 0xFFFFu);
                if (q < kKvTile) {  // always true when the ranks are consistent
                    lv[q] = val[i];
                    lx[q] = LAST ? dg : rk[i];
                }
            }
        }
        __syncthreads();
        const uint32_t cnt = (uint32_t)((e1 - base) < kKvTile ? (e1 - base) : kKvTile);
        for (uint32_t q = tid; q < cnt; q += blockDim.x) {
            const uint32_t r = lx[q];
            const uint32_t dg = LAST ? r : ((r >> shift) & 255u);
            const uint64_t g = (uint32_t)(gofs[dg] + q);
            if (g < n) {  // always true when the histograms are consistent
                dv[g] = lv[q];
                if constexpr (!LAST) dr[g] = r;
            }
        }
#pragma unroll
        for (int i = 0; i < (int)kKvItems; ++i) {
            rk[i] = nrk[i];
            val[i] = nval[i];
        }
        okm = nokm;
        __syncthreads();  // LDS is reused by the next tile
    }
}
__device__ __forceinline__ void kv_down_body(const Args& a, uint32_t pass, uint32_t bid, uint32_t nblk) {
    if (!a.vin) return;
    const Ctrl* c = a.c;
    if (!c->kv_on) return;
    const uint32_t P = c->kv_passes;
    if (P == 0) {  // a single distinct key: the stable order is the input order
        if (pass == 0) {
            const uint64_t gtid = (uint64_t)bid * blockDim.x + threadIdx.x;
            const uint64_t gstride = (uint64_t)nblk * blockDim.x;
            for (uint64_t i = gtid; i < a.n; i += gstride) gp(a.vout)[i] = gp(a.vin)[i];
        }
        return;
    }
    if (pass >= P) return;
    __shared__ KvDownLds L;
    if (pass + 1 == P) kv_down_impl<true>(a, pass, bid, nblk, L);
    else kv_down_impl<false>(a, pass, bid, nblk, L);
}
CAFS_KERNELS1(kv_down, kKvThreads, uint32_t, pass)

// Payloads of a monotone column: already in place order.
__device__ __forceinline__ void kv_copy_mono_body(const Args& a, uint32_t bid, uint32_t nblk) {
    if (!a.vin) return;
    const Ctrl* c = a.c;
    if (c->path != P_MONOTONE) return;
    const uint64_t gtid = (uint64_t)bid * blockDim.x + threadIdx.x;
    const uint64_t gstride = (uint64_t)nblk * blockDim.x;
    for (uint64_t i = gtid; i < a.n; i += gstride) gp(a.vout)[i] = gp(a.vin)[i];
}
CAFS_KERNELS0(kv_copy_mono, 256)

}  // namespace cafs
