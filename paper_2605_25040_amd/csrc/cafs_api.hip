// C ABI of the CAFS hot path (declared in include/cafs.h).
//
// The host side only validates arguments, lays out the caller's workspace and
// enqueues a fixed sequence of kernels; every decision of the dispatcher is
// taken on the device (see cafs_dev.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <deque>
#include <map>
#include <mutex>
#include <unordered_map>
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "cafs_dev.h"
#include "k_count.h"
#include "k_emit.h"
#include "k_estimate.h"
#include "k_guard.h"
#include "k_kv.h"
#include "k_radix.h"

struct cafs_ctx {
    int device;
    int cus;
    hipStream_t side;       // default-priority stream for the branches that overlap the emit
    hipEvent_t fork, join;  // side stream starts after the order kernel; the report waits for it
    void* staging;          // pinned host buffer for the block tables of batched calls
    size_t staging_bytes;
    hipEvent_t staged;      // the last upload from `staging` has been consumed
    bool staged_pending;
    std::vector<void*> captured_staging;  // staging buffers referenced by captured graphs
    uint64_t batch_per_block;       // batched launch: elements per block of the general kernels
    uint64_t batch_per_hash_block;  // and of the hash count
    uint64_t table_mul;             // odd multiplier of the count tables' hash
    void* scratch;                  // this device's address of the static workspace (cafs_sort_noalloc)
    uint64_t part_keys;             // count geometry: estimated keys per hash partition
    uint64_t wide_min;              // and the estimate per partition from which LDS buckets hold 4 keys
    uint64_t table_slots;           // global table slots per estimated key
    bool timing;
    std::vector<hipEvent_t> pool;                 // free events
    std::vector<std::vector<hipEvent_t>> calls;   // CAFS_N_STAGES + 1 events per recorded call
};

namespace {

thread_local std::string g_last_error;

cafs_status_t hip_fail(hipError_t e, const char* where) {
    g_last_error = std::string(where) + ": " + hipGetErrorString(e);
    return CAFS_EHIP;
}

constexpr size_t kAlign = 256;

constexpr size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

constexpr uint64_t bit_ceil_host(uint64_t v) {
    uint64_t p = 1;
    while (p < v) p <<= 1;
    return p;
}

constexpr uint32_t log2_host(uint64_t p) {
    uint32_t m = 0;
    while ((1ull << m) < p) ++m;
    return m;
}

// Workspace of one column of n keys.  Regions are 256-byte aligned.
struct Layout {
    size_t ctrl, gkeys, gcnt, claimed, uniq, cnt, off, tmp_k, psum, status, dcount, bfound, bmin, clist, first, rle_tile,
        spill_k, spill_v, pbuf;
    uint64_t pbuf_elems;
    size_t total;
    uint32_t cap_log2;
    uint64_t status_slot;
    uint64_t m_ws;
};

constexpr Layout make_layout(uint64_t n) {
    Layout L{};
    const uint64_t nn = n > 0 ? n : 1;
    // the global table never needs more than bit_ceil(n) slots (K <= n); the device
    // picks a smaller one from the estimate
    uint32_t lg = log2_host(bit_ceil_host(std::max<uint64_t>(nn, 1ull << cafs::kMinTableLog2)));
    lg = std::min<uint32_t>(std::max<uint32_t>(lg, cafs::kMinTableLog2), cafs::kMaxTableLog2);
    L.cap_log2 = lg;
    const uint64_t cap = 1ull << lg;
    L.m_ws = std::max<uint64_t>(8, bit_ceil_host(nn / cafs::kBucketCap));
    const uint64_t radix_max = std::max<uint64_t>(nn, cap);
    const uint64_t tiles = (radix_max + cafs::kRadixTile - 1) / cafs::kRadixTile;
    L.status_slot = tiles * 256;
    const uint64_t rle_tiles = (nn + cafs::kRleTile - 1) / cafs::kRleTile;
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t at = o; o = align_up(o + bytes); return at; };
    L.ctrl = take(sizeof(cafs::Ctrl));
    L.gkeys = take(cap * 8);
    L.gcnt = take(cap * 8);
    L.claimed = take(cap * 4);
    L.uniq = take(nn * 8);
    L.cnt = take(nn * 8);
    L.off = take((nn + 1) * 8);
    // radix scratch; also the hash count's deferral regions, one per item at the
    // item's place in the column or in the partition buckets
    L.pbuf_elems = nn + nn / 8 + cafs::kMaxParts * (cafs::kScatterChunk + 32);
    L.tmp_k = take(std::max<uint64_t>(nn + 2 + 2 * cafs::kMaxCountBlocks, L.pbuf_elems) * 8);
    L.psum = take(2 * cafs::kMaxCountBlocks * 8);
    L.status = take(2 * L.status_slot * 8);
    L.dcount = take(L.m_ws * 4);
    L.bfound = take(L.m_ws * 4);
    L.bmin = take(L.m_ws * 4 * cafs::kMaxBucketCap);  // the guard rounds' minima: cap per bucket
    L.clist = take(nn * 4);
    L.first = take(nn * 4);
    L.rle_tile = take(rle_tiles * 8);
    L.spill_k = take(nn * 8);
    L.spill_v = take(nn * 8);
    // partition buckets: an eighth more than the column plus a scatter chunk per bucket
    L.pbuf = take(L.pbuf_elems * 8);
    L.total = o;
    return L;
}

template <class T>
T* at(void* ws, size_t off) { return reinterpret_cast<T*>(static_cast<char*>(ws) + off); }

// Workspace of the allocation-free entry point: one column of up to CAFS_NOALLOC_MAX_N
// keys, in a file-scope device array.  Each GPU the library runs on holds its own
// copy until the process ends.  Host code never passes the array's name to a kernel
// (on the host it is only a stand-in for the symbol): each device's address is
// looked up once, with hipGetSymbolAddress, when the first context on that device is
// created, and only that address is used.
constexpr size_t kNoAllocWsBytes = make_layout(CAFS_NOALLOC_MAX_N).total;

}  // namespace

static __device__ __align__(256) unsigned char scratch[kNoAllocWsBytes];

namespace {

std::mutex g_scratch_mu;
std::vector<void*> g_scratch_ptr;  // per device, nullptr until looked up

// Called with `device` current.
cafs_status_t scratch_address(int device, int n_devices, void** out) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if ((int)g_scratch_ptr.size() < n_devices) g_scratch_ptr.resize(n_devices, nullptr);
    if (!g_scratch_ptr[device]) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p || reinterpret_cast<uintptr_t>(p) % kAlign) {
            g_last_error = "static workspace: unexpected address";
            return CAFS_EHIP;
        }
        g_scratch_ptr[device] = p;
    }
    *out = g_scratch_ptr[device];
    return CAFS_OK;
}

bool overlaps(const void* a, const void* b, uint64_t n, uint32_t ew) {
    const uintptr_t x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
    const uintptr_t bytes = n * ew;
    return x != y && x < y + bytes && y < x + bytes;
}

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        int cur = 0;
        if (hipGetDevice(&cur) == hipSuccess && cur != dev) {
            prev = cur;
            (void)hipSetDevice(dev);
        }
    }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

uint32_t grid_for(uint64_t work_items, uint64_t per_block, uint32_t cap) {
    uint64_t g = (work_items + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (uint32_t)g;
}

// The radix engine: digit histograms, up to eight passes (keys only, or key-value
// pairs when `pairs` may be needed), and the final copy.  Passes of constant
// digits and the variant without work return at once.
cafs_status_t launch_radix(const cafs::Args& a, uint64_t n_max, int cus, hipStream_t s, bool pairs) {
    const uint64_t tiles = (n_max + cafs::kRadixTile - 1) / cafs::kRadixTile;
    const uint32_t g_hist = grid_for(n_max, 256 * 16, cus * 4);
    cafs::k_radix_hist<<<g_hist, 256, 0, s>>>(a);
    // resident workgroups per CU (LDS): two keys-only (tiles of twice kRadixTile),
    // two key-value
    const uint32_t g_keys = grid_for(tiles / 2 + 1, 1, cus * 2), g_kv = grid_for(tiles, 1, cus * 2);
    for (uint32_t p = 0; p < 8; ++p) {
        cafs::k_radix_pass<<<g_keys, cafs::kRadixKeysThreads, 0, s>>>(a, p);
        if (pairs) cafs::k_radix_pass_kv<<<g_kv, cafs::kRadixThreads, 0, s>>>(a, p);
    }
    cafs::k_radix_copy<<<grid_for(n_max, 256 * 8, cus * 4), 256, 0, s>>>(a);
    return CAFS_OK;
}

// Workgroups of the single-column ranking kernel.
uint32_t rank_grid(uint64_t n) {
    return grid_for(std::min<uint64_t>(n, cafs::kRankMax), cafs::kRankKeysPerBlock, 1u << 16);
}

// Workgroups of the single-column hash count: one per CU (the LDS table takes the
// CU), fewer for short columns; a multiple of 8 * 16 or a power of two, so that
// the work items of every partition count divide evenly.
uint32_t count_grid(uint64_t n, int cus) {
    uint32_t g = grid_for(n, cafs::kCountThreads * 8, std::min<uint32_t>(cus, cafs::kMaxCountBlocks));
    const uint32_t q = cafs::kXcds << cafs::kMaxPartLog2;
    if (g >= q) return g / q * q;
    uint32_t p = 1;
    while (2 * p <= g) p *= 2;
    return p;
}

bool dtype_ok(cafs_dtype_t dt) {
    return dt == CAFS_I64 || dt == CAFS_U64 || dt == CAFS_F64 || dt == CAFS_I32 || dt == CAFS_U32;
}

uint32_t elem_bytes(cafs_dtype_t dt) { return (dt == CAFS_I32 || dt == CAFS_U32) ? 4u : 8u; }

cafs::Args make_args(const cafs_ctx* ctx, const Layout& L, const void* in, void* out, uint64_t n, cafs_dtype_t dt,
                     void* uniq, uint64_t* counts, cafs_report_t* report, void* ws) {
    cafs::Args a{};
    a.in = static_cast<const uint64_t*>(in);
    a.out = static_cast<uint64_t*>(out);
    a.n = n;
    a.flip = (dt == CAFS_I64 || dt == CAFS_F64) ? (1ull << 63) : dt == CAFS_I32 ? (1ull << 31) : 0ull;
    a.ew = elem_bytes(dt);
    a.cap = a.ew == 4 ? cafs::kBucketCap32 : cafs::kBucketCap;
    a.fneg = (dt == CAFS_F64) ? ~0ull : 0ull;
    // (the pair layout of 64-bit keys; 32-bit keys are accessed one by one)
    a.in_head = (a.ew == 8 && reinterpret_cast<uintptr_t>(in) % 16) ? 1u : 0u;
    a.out_head = (a.ew == 8 && reinterpret_cast<uintptr_t>(out) % 16) ? 1u : 0u;
    a.want_report = report != nullptr;
    a.want_counts = (uniq != nullptr) || (counts != nullptr);
    a.report = report;
    a.c = at<cafs::Ctrl>(ws, L.ctrl);
    // 32-bit keys: the distinct keys are built as 64-bit values in the workspace and
    // copied into the caller's array at the end
    a.uniq = (uniq && a.ew == 8) ? static_cast<uint64_t*>(uniq) : at<uint64_t>(ws, L.uniq);
    a.uniq_out = a.ew == 4 ? uniq : nullptr;
    a.cnt = counts ? counts : at<uint64_t>(ws, L.cnt);
    a.off = at<uint64_t>(ws, L.off);
    a.gkeys = at<uint64_t>(ws, L.gkeys);
    a.gcnt = at<uint64_t>(ws, L.gcnt);
    a.claimed = at<uint32_t>(ws, L.claimed);
    a.cap_ws_log2 = L.cap_log2;
    a.tmp_k = at<uint64_t>(ws, L.tmp_k);
    a.status = at<uint64_t>(ws, L.status);
    a.status_slot = L.status_slot;
    a.dcount = at<uint32_t>(ws, L.dcount);
    a.bmin = at<uint32_t>(ws, L.bmin);
    a.first_idx = at<uint32_t>(ws, L.first);
    a.clist = at<uint32_t>(ws, L.clist);
    a.bfound = at<uint32_t>(ws, L.bfound);
    a.m_ws = L.m_ws;
    a.rle_tile = at<uint64_t>(ws, L.rle_tile);
    a.psum = at<uint64_t>(ws, L.psum);
    a.spill_k = at<uint64_t>(ws, L.spill_k);
    a.spill_v = at<uint64_t>(ws, L.spill_v);
    a.pbuf = at<uint64_t>(ws, L.pbuf);
    a.pbuf_elems = L.pbuf_elems;
    a.kv_tab_log2 = log2_host(L.pbuf_elems / 2 + 1);  // (floor: pbuf_elems / 2 16-byte slots fit)
    a.part_keys = ctx ? ctx->part_keys : cafs::kPartKeys;
    a.wide_min = ctx ? ctx->wide_min : cafs::kLdsWideMinKhat;
    a.table_slots = ctx ? ctx->table_slots : cafs::kTableSlotsPerKey;
    a.rank_blocks = rank_grid(n);
    a.rank_budget_log2 = cafs::kRankBudgetLog2;
    a.row_blocks = ctx ? (uint32_t)ctx->cus : 256u;
    a.table_mul = ctx ? ctx->table_mul : cafs::kPhi;
    return a;
}

cafs_status_t check_buffers(const void* in, const void* out, uint64_t n, uint32_t ew) {
    if (n >= (1ull << 32)) return CAFS_EINVAL;
    if (n > 0 && (!in || !out)) return CAFS_EINVAL;
    if ((reinterpret_cast<uintptr_t>(in) | reinterpret_cast<uintptr_t>(out)) % ew) return CAFS_EINVAL;
    if (overlaps(in, out, n, ew)) return CAFS_EINVAL;
    return CAFS_OK;
}

// Byte ranges [a, a + na) and [b, b + nb) share a byte.
bool ranges_meet(const void* a, uint64_t na, const void* b, uint64_t nb) {
    const uintptr_t x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
    return na > 0 && nb > 0 && x < y + nb && y < x + na;
}

cafs_status_t sort_impl(cafs_ctx_t* ctx, const void* in, void* out, uint64_t n, cafs_dtype_t dt, void* uniq,
                        uint64_t* counts, cafs_report_t* report, void* ws, size_t ws_bytes, void* stream,
                        bool may_time = true, const uint64_t* vin = nullptr, uint64_t* vout = nullptr) {
    if (!ctx) return CAFS_EINVAL;
    if (!dtype_ok(dt)) return CAFS_EINVAL;
    cafs_status_t st = check_buffers(in, out, n, elem_bytes(dt));
    if (st != CAFS_OK) return st;
    if ((uniq || counts) && !report) return CAFS_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    DeviceGuard dg(ctx->device);
    if (n == 0) {
        if (report) cafs::k_report_empty<<<1, 64, 0, s>>>(report);
        hipError_t e = hipGetLastError();
        return e == hipSuccess ? CAFS_OK : hip_fail(e, "launch");
    }
    const Layout L = make_layout(n);
    if (!ws || ws_bytes < L.total || reinterpret_cast<uintptr_t>(ws) % kAlign) return CAFS_EWORKSPACE;
    cafs::Args a = make_args(ctx, L, in, out, n, dt, uniq, counts, report, ws);
    a.vin = vin;
    a.vout = vout;
    const bool kv = vin != nullptr;
    const int cus = ctx->cus;
    std::vector<hipEvent_t> evs;
    if (ctx->timing && may_time) {
        for (int i = 0; i <= CAFS_N_STAGES; ++i) {
            hipEvent_t e;
            if (!ctx->pool.empty()) {
                e = ctx->pool.back();
                ctx->pool.pop_back();
            } else if (hipEventCreate(&e) != hipSuccess) {
                return hip_fail(hipGetLastError(), "hipEventCreate");
            }
            evs.push_back(e);
        }
    }
    auto mark = [&](int i) {
        if (!evs.empty()) (void)hipEventRecord(evs[i], s);
    };
    const uint64_t cap_ws = 1ull << L.cap_log2;
    (void)hipGetLastError();  // clear any stale error so the check below is ours
    mark(0);
    cafs::k_pre<<<1, 1024, 0, s>>>(a);
    if (n > cafs::kMonoPrefix) cafs::k_mono_full<<<grid_for(n, 256 * 16, cus * 4), 256, 0, s>>>(a);
    if (n >= cafs::kReplanMinN)  // heavy-tailed estimates: the count's geometry from a larger sample
        cafs::k_sample2<<<cafs::kSamples2 / cafs::kSamples2Block, cafs::kSamples2Threads, 0, s>>>(a);
    const bool countable = n >= cafs::kSmallN;  // tiny and main need N >= 2048
    if (countable)
        cafs::k_phase2<<<grid_for(std::max<uint64_t>(n / 2, cap_ws), 256 * 4, cus * 4), 256, 0, s>>>(a);
    if (countable)
        cafs::k_part_scatter<<<grid_for(n, cafs::kScatterChunk * 4, cus * 2), cafs::kScatterThreads, 0, s>>>(a);
    mark(1);  // (the count stage brackets the hash count kernel alone)
    const uint32_t g_count = count_grid(n, cus);
    if (countable) {
        if (a.ew == 4) cafs::k_hash_count32<<<g_count, cafs::kCountThreads, 0, s>>>(a);
        else cafs::k_hash_count<<<g_count, cafs::kCountThreads, 0, s>>>(a);
        // partitions need an estimate above twice part_keys, at most N / 2 on the
        // main path, or the larger sample's estimate
        if (n > 4 * a.part_keys || n >= cafs::kReplanMinN)
            cafs::k_hash_count_parts<<<g_count, cafs::kCountThreads, 0, s>>>(a);
    }
    mark(2);
    if (countable) {
        cafs::k_rank<<<a.rank_blocks, 1024, 0, s>>>(a);
        cafs::k_compact_order<<<1, 1024, 0, s>>>(a);
    }
    // Fork: the branches that are idle on the common path (radix engine and pair
    // sort with their own emit, monotone copy, run-length pass, guard resolution)
    // run on the side stream and overlap the emit on the caller's stream.
    // In place, the guard's first-occurrence pass reads the input that the emit
    // overwrites, so then the emit waits for the side stream.
    hipStream_t s2 = ctx->side;
    const bool inplace = (in == out);
    (void)hipEventRecord(ctx->fork, s);
    (void)hipStreamWaitEvent(s2, ctx->fork, 0);
    mark(3);  // (after the fork record, so that the emit stage brackets the row emit only)
    // four workgroups per CU saturate the write bandwidth and leave CU slots free
    // for the side stream
    const uint32_t g_emit = grid_for(n, 2 * cafs::kEmitTilePairs, cus * 4);
    if (countable && !inplace) cafs::k_emit_rows<<<std::min<uint32_t>(g_emit, cus), cafs::kEmitRowsThreads, 0, s>>>(a);
    mark(4);
    // (K > 32768 is emitted by the tile emit after the pair sort on the side stream)
    launch_radix(a, std::max<uint64_t>(n, countable ? cap_ws : 0), cus, s2, countable || kv);
    if (countable) {
        // (a spill can reach the pair sort at any N)
        const uint32_t g_scan = std::min<uint32_t>(cus * 2, cafs::kMaxCountBlocks);
        cafs::k_fold_sums<<<g_scan, 1024, 0, s2>>>(a);
        cafs::k_fold_write<<<g_scan, 1024, 0, s2>>>(a);
    }
    cafs::k_copy_mono<<<grid_for(n, 256 * 8, cus * 4), 256, 0, s2>>>(a);
    if (kv) cafs::k_kv_copy_mono<<<grid_for(n, 256 * 8, cus * 4), 256, 0, s2>>>(a);
    const uint32_t g_rle = grid_for(n, cafs::kRleTile, cus * 4);
    cafs::k_rle_count<<<g_rle, 256, 0, s2>>>(a);
    cafs::k_rle_write<<<g_rle, 256, 0, s2>>>(a);
    cafs::k_rle_counts<<<grid_for(n, 256 * 8, cus * 4), 256, 0, s2>>>(a);
    if (countable) {
        const uint32_t g = grid_for(n, 256 * 64, cus * 2);
        cafs::k_guard_prep<<<grid_for(L.m_ws, 256 * 8, cus * 4), 256, 0, s2>>>(a);
        cafs::k_guard_bucket<<<g, 256, 0, s2>>>(a);
        cafs::k_guard_mark<<<g, 256, 0, s2>>>(a);
        // (two workgroups per CU: each one's chunk loop is a chain of dependent loads)
        cafs::k_guard_first<<<grid_for(n, cafs::kGuardChunk, cus * 2), 256, 0, s2>>>(a);
        cafs::k_guard_resolve<<<1, 1024, 0, s2>>>(a);
        for (uint32_t r = 0; r < a.cap; ++r) cafs::k_guard_round<<<g, 256, 0, s2>>>(a, r);
        cafs::k_guard_final<<<g, 256, 0, s2>>>(a);
        // outputs written after the guard: it reads the input, which an in-place sort overwrites
        cafs::k_copy_deferred<<<grid_for(n, 256 * 8, cus * 4), 256, 0, s2>>>(a);
        cafs::k_emit<<<g_emit, cafs::kEmitThreads, 0, s2>>>(a, 1u);
    }
    (void)hipEventRecord(ctx->join, s2);
    (void)hipStreamWaitEvent(s, ctx->join, 0);
    if (countable && inplace)
        cafs::k_emit_rows<<<std::min<uint32_t>(g_emit, cus), cafs::kEmitRowsThreads, 0, s>>>(a);
    if (kv && countable) {
        // payload placement on the count paths (the kernels return at once elsewhere):
        // `units` upsweep workgroups, kKvUnitsPerChunk of them per placement workgroup
        const uint64_t tiles = (n + cafs::kKvTile - 1) / cafs::kKvTile;
        const uint64_t want = (tiles + cafs::kKvUnitsPerChunk - 1) / cafs::kKvUnitsPerChunk;
        const uint32_t chunks =
            (uint32_t)std::min<uint64_t>(want, std::min<uint32_t>((uint32_t)cus * 2, cafs::kKvMaxChunks));
        const uint32_t units = chunks * cafs::kKvUnitsPerChunk;
        cafs::k_kv_setup<<<1, 64, 0, s>>>(a);
        cafs::k_kv_clear<<<grid_for(n, 256 * 8, cus * 4), 256, 0, s>>>(a);
        cafs::k_kv_build<<<grid_for(n, 256 * 4, cus * 2), 256, 0, s>>>(a);
        for (uint32_t p = 0; p < 4; ++p) {
            if (p == 0) {
                cafs::k_kv_up0_lds<<<units, cafs::kKvThreads, 0, s>>>(a);
                cafs::k_kv_up0_mem<<<units, cafs::kKvThreads, 0, s>>>(a);
            } else {
                cafs::k_kv_up<<<units, cafs::kKvThreads, 0, s>>>(a, p);
            }
            cafs::k_kv_scan<<<256, 1024, 0, s>>>(a, p, units);
            cafs::k_kv_down<<<chunks, cafs::kKvThreads, 0, s>>>(a, p);
        }
    }
    if (a.uniq_out) cafs::k_uniq_out<<<grid_for(n, 256 * 8, cus * 4), 256, 0, s>>>(a);
    cafs::k_finalize<<<1, 64, 0, s>>>(a);
    mark(5);
    if (!evs.empty()) ctx->calls.push_back(evs);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? CAFS_OK : hip_fail(e, "launch");
}

__global__ void k_radix_setup(cafs::Args a) {
    if (threadIdx.x != 0) return;
    cafs::Ctrl* c = a.c;
    for (int d = 0; d < 8; ++d) {
        c->tile_ctr[d] = 0;
        for (int b = 0; b < 256; ++b) c->hist[d][b] = 0;
    }
    c->hist_done = 0;
    c->radix_on = 1;
    cafs::RadixJob& j = c->rj;
    j.src_k = a.in; j.src_v = nullptr;
    j.dst_k = a.out; j.dst_v = nullptr;
    j.tmp_k = a.tmp_k; j.tmp_v = nullptr;
    j.n = a.n;
    j.has_vals = 0;
    j.n_active = 0;
    j.copy_mode = 0;
    j.src_ew = a.ew;
    j.dst_ew = a.ew;
}

}  // namespace

extern "C" {

cafs_status_t cafs_ctx_create(cafs_ctx_t** ctx, int device) {
    if (!ctx) return CAFS_EINVAL;
    *ctx = nullptr;
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceCount");
    if (device < 0 || device >= count) return CAFS_EINVAL;
    int cus = 0;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
    if (e != hipSuccess) return hip_fail(e, "hipDeviceGetAttribute");
    cafs_ctx_t* c = new (std::nothrow) cafs_ctx_t;
    if (!c) return CAFS_ENOMEM;
    c->device = device;
    c->cus = cus > 0 ? cus : 1;
    c->timing = false;
    c->staging = nullptr;
    c->staging_bytes = 0;
    c->staged_pending = false;
    c->batch_per_block = 1ull << 16;
    c->batch_per_hash_block = 1ull << 18;
    c->table_mul = cafs::kPhi;
    c->scratch = nullptr;
    c->part_keys = cafs::kPartKeys;
    c->wide_min = cafs::kLdsWideMinKhat;
    c->table_slots = cafs::kTableSlotsPerKey;
    {
        DeviceGuard dg(device);
        cafs_status_t st = scratch_address(device, count, &c->scratch);
        if (st != CAFS_OK) {
            delete c;
            return st;
        }
        e = hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&c->fork, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&c->join, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&c->staged, hipEventDisableTiming);
        if (e != hipSuccess) {
            delete c;
            return hip_fail(e, "side stream");
        }
    }
    *ctx = c;
    return CAFS_OK;
}

void cafs_ctx_destroy(cafs_ctx_t* ctx) {
    if (!ctx) return;
    for (auto& call : ctx->calls)
        for (hipEvent_t e : call) (void)hipEventDestroy(e);
    for (hipEvent_t e : ctx->pool) (void)hipEventDestroy(e);
    {
        DeviceGuard dg(ctx->device);
        (void)hipEventDestroy(ctx->fork);
        (void)hipEventDestroy(ctx->join);
        if (ctx->staged_pending) (void)hipEventSynchronize(ctx->staged);
        (void)hipEventDestroy(ctx->staged);
        if (ctx->staging) (void)hipHostFree(ctx->staging);
        for (void* p : ctx->captured_staging) (void)hipHostFree(p);
        (void)hipStreamDestroy(ctx->side);
    }
    delete ctx;
}

cafs_status_t cafs_ctx_enable_timing(cafs_ctx_t* ctx, int enable) {
    if (!ctx) return CAFS_EINVAL;
    ctx->timing = enable != 0;
    return CAFS_OK;
}

cafs_status_t cafs_ctx_stage_ms(cafs_ctx_t* ctx, float* h_ms, int n_stages, int* h_calls) {
    if (!ctx || (n_stages > 0 && !h_ms) || n_stages < 0 || n_stages > CAFS_N_STAGES) return CAFS_EINVAL;
    DeviceGuard dg(ctx->device);
    for (int i = 0; i < n_stages; ++i) h_ms[i] = 0.f;
    cafs_status_t st = CAFS_OK;
    for (auto& call : ctx->calls) {
        hipError_t e = hipEventSynchronize(call.back());
        if (e != hipSuccess && st == CAFS_OK) st = hip_fail(e, "hipEventSynchronize");
        for (int i = 0; i < n_stages && st == CAFS_OK; ++i) {
            float ms = 0.f;
            e = hipEventElapsedTime(&ms, call[i], call[i + 1]);
            if (e != hipSuccess) st = hip_fail(e, "hipEventElapsedTime");
            h_ms[i] += ms;
        }
        for (hipEvent_t ev : call) ctx->pool.push_back(ev);
    }
    if (h_calls) *h_calls = (int)ctx->calls.size();
    ctx->calls.clear();
    return st;
}

size_t cafs_workspace_bytes(uint64_t n, cafs_dtype_t dtype) {
    (void)dtype;
    return make_layout(n).total;
}

cafs_status_t cafs_estimate(cafs_ctx_t* ctx, const void* d_keys, uint64_t n, cafs_dtype_t dtype,
                            cafs_estimate_t* d_out, void* stream) {
    if (!ctx || !d_out || (n > 0 && !d_keys) || !dtype_ok(dtype)) return CAFS_EINVAL;
    if (reinterpret_cast<uintptr_t>(d_keys) % elem_bytes(dtype)) return CAFS_EINVAL;
    if (n >= (1ull << 32)) return CAFS_EINVAL;
    DeviceGuard dg(ctx->device);
    (void)hipGetLastError();
    cafs::k_estimate_only<<<1, 1024, 0, static_cast<hipStream_t>(stream)>>>(static_cast<const uint64_t*>(d_keys), n,
                                                                            elem_bytes(dtype), d_out);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? CAFS_OK : hip_fail(e, "launch");
}

cafs_status_t cafs_sort_kv(cafs_ctx_t* ctx, const void* d_keys_in, void* d_keys_out, const uint64_t* d_vals_in,
                           uint64_t* d_vals_out, uint64_t n, cafs_dtype_t dtype, void* d_uniq, uint64_t* d_counts,
                           cafs_report_t* d_report, void* d_ws, size_t ws_bytes, void* stream) {
    if (!ctx || !dtype_ok(dtype)) return CAFS_EINVAL;
    const uint32_t ew = elem_bytes(dtype);
    cafs_status_t st = check_buffers(d_keys_in, d_keys_out, n, ew);
    if (st != CAFS_OK) return st;
    if (n > 0) {
        if (!d_vals_in || !d_vals_out) return CAFS_EINVAL;
        if ((reinterpret_cast<uintptr_t>(d_vals_in) | reinterpret_cast<uintptr_t>(d_vals_out)) % 8) return CAFS_EINVAL;
        // no output may share a byte with another buffer (the keys are read again
        // after the sorted keys are written); the inputs are only read
        const uint64_t kb = n * ew, vb = n * 8;
        if (ranges_meet(d_keys_in, kb, d_keys_out, kb) || ranges_meet(d_vals_in, vb, d_vals_out, vb) ||
            ranges_meet(d_keys_in, kb, d_vals_out, vb) || ranges_meet(d_keys_out, kb, d_vals_in, vb) ||
            ranges_meet(d_keys_out, kb, d_vals_out, vb))
            return CAFS_EINVAL;
    }
    if (n == 0) return sort_impl(ctx, d_keys_in, d_keys_out, n, dtype, d_uniq, d_counts, d_report, d_ws, ws_bytes,
                                 stream);
    return sort_impl(ctx, d_keys_in, d_keys_out, n, dtype, d_uniq, d_counts, d_report, d_ws, ws_bytes, stream, true,
                     d_vals_in, d_vals_out);
}

cafs_status_t cafs_sort_i64(cafs_ctx_t* ctx, const int64_t* d_in, int64_t* d_out, uint64_t n, int64_t* d_uniq,
                            uint64_t* d_counts, cafs_report_t* d_report, void* d_ws, size_t ws_bytes, void* stream) {
    return sort_impl(ctx, d_in, d_out, n, CAFS_I64, d_uniq, d_counts, d_report, d_ws, ws_bytes, stream);
}

cafs_status_t cafs_sort_u64(cafs_ctx_t* ctx, const uint64_t* d_in, uint64_t* d_out, uint64_t n, uint64_t* d_uniq,
                            uint64_t* d_counts, cafs_report_t* d_report, void* d_ws, size_t ws_bytes, void* stream) {
    return sort_impl(ctx, d_in, d_out, n, CAFS_U64, d_uniq, d_counts, d_report, d_ws, ws_bytes, stream);
}

cafs_status_t cafs_sort_f64(cafs_ctx_t* ctx, const double* d_in, double* d_out, uint64_t n, double* d_uniq,
                            uint64_t* d_counts, cafs_report_t* d_report, void* d_ws, size_t ws_bytes, void* stream) {
    return sort_impl(ctx, d_in, d_out, n, CAFS_F64, d_uniq, d_counts, d_report, d_ws, ws_bytes, stream);
}

cafs_status_t cafs_sort_i32(cafs_ctx_t* ctx, const int32_t* d_in, int32_t* d_out, uint64_t n, int32_t* d_uniq,
                            uint64_t* d_counts, cafs_report_t* d_report, void* d_ws, size_t ws_bytes, void* stream) {
    return sort_impl(ctx, d_in, d_out, n, CAFS_I32, d_uniq, d_counts, d_report, d_ws, ws_bytes, stream);
}

cafs_status_t cafs_sort_u32(cafs_ctx_t* ctx, const uint32_t* d_in, uint32_t* d_out, uint64_t n, uint32_t* d_uniq,
                            uint64_t* d_counts, cafs_report_t* d_report, void* d_ws, size_t ws_bytes, void* stream) {
    return sort_impl(ctx, d_in, d_out, n, CAFS_U32, d_uniq, d_counts, d_report, d_ws, ws_bytes, stream);
}

cafs_status_t cafs_sort_noalloc(cafs_ctx_t* ctx, const void* d_in, void* d_out, uint64_t n, cafs_dtype_t dtype,
                                void* d_uniq, uint64_t* d_counts, cafs_report_t* d_report, void* stream) {
    if (!ctx) return CAFS_EINVAL;
    if (n > CAFS_NOALLOC_MAX_N) {
        g_last_error = "cafs_sort_noalloc: n exceeds CAFS_NOALLOC_MAX_N";
        return CAFS_EINVAL;
    }
    return sort_impl(ctx, d_in, d_out, n, dtype, d_uniq, d_counts, d_report, ctx->scratch, kNoAllocWsBytes, stream,
                     false);
}

cafs_status_t cafs_radix_sort(cafs_ctx_t* ctx, const void* d_in, void* d_out, uint64_t n, cafs_dtype_t dtype,
                              void* d_ws, size_t ws_bytes, void* stream) {
    if (!ctx) return CAFS_EINVAL;
    if (!dtype_ok(dtype)) return CAFS_EINVAL;
    cafs_status_t st = check_buffers(d_in, d_out, n, elem_bytes(dtype));
    if (st != CAFS_OK) return st;
    if (n == 0) return CAFS_OK;
    const Layout L = make_layout(n);
    if (!d_ws || ws_bytes < L.total || reinterpret_cast<uintptr_t>(d_ws) % kAlign) return CAFS_EWORKSPACE;
    DeviceGuard dg(ctx->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const cafs::Args a = make_args(ctx, L, d_in, d_out, n, dtype, nullptr, nullptr, nullptr, d_ws);
    (void)hipGetLastError();
    k_radix_setup<<<1, 64, 0, s>>>(a);
    launch_radix(a, n, ctx->cus, s, false);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? CAFS_OK : hip_fail(e, "launch");
}

// ---- batched calls ----------------------------------------------------------
// A batched call launches every kernel once for the whole batch; each block works
// on one column through a block table.  The device header of a batch holds the
// per-column call arguments and three block tables (one block per column; the
// general kernels; the hash count); it is built on the host in pinned memory and
// uploaded with one asynchronous copy.  Each column has its own single-column
// workspace.

}  // extern "C"

namespace {

constexpr uint32_t kBatchMaxBlocks = 64;  // per column and kernel

struct BatchShape {
    std::vector<uint32_t> bp, bh;  // blocks per column: general kernels, hash count
    uint32_t total_p = 0, total_h = 0;
    size_t off_args = 0, off_m1 = 0, off_mp = 0, off_mh = 0, off_rl = 0, header = 0;
};

uint32_t blocks_for(uint64_t n, uint64_t per) {
    uint64_t b = (n + per - 1) / per;
    return (uint32_t)std::min<uint64_t>(std::max<uint64_t>(b, 1), kBatchMaxBlocks);
}

// Header layout; its size is bounded by header_bound(n_cols) whatever the tuning.
BatchShape shape_batch(const uint64_t* ns, uint32_t n_cols, uint64_t per_block, uint64_t per_hash_block) {
    BatchShape P;
    P.bp.resize(n_cols);
    P.bh.resize(n_cols);
    for (uint32_t i = 0; i < n_cols; ++i) {
        P.bp[i] = blocks_for(ns[i], per_block);
        P.bh[i] = blocks_for(ns[i], per_hash_block);
        P.total_p += P.bp[i];
        P.total_h += P.bh[i];
    }
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t at = o; o = align_up(o + bytes); return at; };
    P.off_args = take(sizeof(cafs::Args) * (size_t)n_cols);
    P.off_m1 = take(4ull * (n_cols + 2ull * n_cols));   // col[total], first[n_cols], count[n_cols]
    P.off_mp = take(4ull * (P.total_p + 2ull * n_cols));
    P.off_mh = take(4ull * (P.total_h + 2ull * n_cols));
    P.off_rl = take(cafs::radix_list_bytes(n_cols));  // (filled on the device, after its capacity)
    P.header = o;
    return P;
}

size_t header_bound(uint32_t n_cols) {
    return align_up(sizeof(cafs::Args) * (size_t)n_cols) + 3 * align_up(4ull * (kBatchMaxBlocks + 2ull) * n_cols) +
           align_up(cafs::radix_list_bytes(n_cols));
}

void fill_table(uint32_t* dst, uint32_t n_cols, const std::vector<uint32_t>* per_col, uint32_t total) {
    uint32_t* col = dst;
    uint32_t* first = dst + total;
    uint32_t* count = first + n_cols;
    uint32_t b = 0;
    for (uint32_t c = 0; c < n_cols; ++c) {
        const uint32_t k = per_col ? (*per_col)[c] : 1u;
        first[c] = b;
        count[c] = k;
        for (uint32_t j = 0; j < k; ++j) col[b++] = c;
    }
}

cafs::BatchGrid grid_at(void* hdr, const BatchShape& P, size_t off, uint32_t total, uint32_t n_cols) {
    cafs::BatchGrid g;
    g.args = at<cafs::Args>(hdr, P.off_args);
    g.col = at<uint32_t>(hdr, off);
    g.first = g.col + total;
    g.count = g.first + n_cols;
    return g;
}

cafs_status_t check_columns(const cafs_column_t* cols, uint32_t n_cols, std::vector<uint64_t>& ns) {
    ns.resize(n_cols);
    for (uint32_t i = 0; i < n_cols; ++i) {
        const cafs_column_t& col = cols[i];
        if (col.flags != 0 || !dtype_ok((cafs_dtype_t)col.dtype)) return CAFS_EINVAL;
        cafs_status_t st = check_buffers(col.d_in, col.d_out, col.n, elem_bytes((cafs_dtype_t)col.dtype));
        if (st != CAFS_OK) return st;
        if ((col.d_uniq || col.d_counts) && !col.d_report) return CAFS_EINVAL;
        ns[i] = col.n;
    }
    return CAFS_OK;
}

// Enqueues one batch.  col_ws[i] is column i's workspace (make_layout(n_i).total
// bytes, 256-byte aligned); hdr_dev receives the header, staged through hdr_host
// (pinned, at least P.header bytes, not reused before this upload has run).
// A second stream with its fork and join events: the batch's partitioned count runs
// there beside the other count variants.
struct SideLane {
    hipStream_t s;
    hipEvent_t fork, join;
};

cafs_status_t launch_batch(const cafs_ctx_t* ctx, const cafs_column_t* cols, uint32_t n_cols, void* const* col_ws,
                           const BatchShape& P, void* hdr_dev, void* hdr_host, hipStream_t s, const SideLane& side) {
    char* h = static_cast<char*>(hdr_host);
    cafs::Args* args = reinterpret_cast<cafs::Args*>(h + P.off_args);
    for (uint32_t i = 0; i < n_cols; ++i) {
        const cafs_column_t& col = cols[i];
        args[i] = make_args(ctx, make_layout(col.n), col.d_in, col.d_out, col.n, (cafs_dtype_t)col.dtype,
                            col.d_uniq, col.d_counts, col.d_report, col_ws[i]);
        args[i].rank_blocks = P.bp[i];  // the ranking kernel runs over the general block table
        args[i].rank_budget_log2 = cafs::kRankBudgetBatchLog2;
        args[i].row_blocks = P.bp[i];
    }
    fill_table(reinterpret_cast<uint32_t*>(h + P.off_m1), n_cols, nullptr, n_cols);
    fill_table(reinterpret_cast<uint32_t*>(h + P.off_mp), n_cols, &P.bp, P.total_p);
    fill_table(reinterpret_cast<uint32_t*>(h + P.off_mh), n_cols, &P.bh, P.total_h);
    {
        cafs::RadixList* rl = reinterpret_cast<cafs::RadixList*>(h + P.off_rl);
        std::memset(rl, 0, sizeof(cafs::RadixList));
        rl->cap = n_cols;
    }
    (void)hipGetLastError();
    hipError_t e = hipMemcpyAsync(hdr_dev, hdr_host, P.header, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync");
    const cafs::BatchGrid g1 = grid_at(hdr_dev, P, P.off_m1, n_cols, n_cols);
    const cafs::BatchGrid gp = grid_at(hdr_dev, P, P.off_mp, P.total_p, n_cols);
    const cafs::BatchGrid gh = grid_at(hdr_dev, P, P.off_mh, P.total_h, n_cols);
    const uint32_t C = n_cols, TP = P.total_p, TH = P.total_h;
    cafs::kb_pre<<<C, 1024, 0, s>>>(g1);
    cafs::kb_mono_full<<<TP, 256, 0, s>>>(gp);
    cafs::kb_phase2<<<TP, 256, 0, s>>>(gp);
    cafs::kb_part_scatter<<<TP, cafs::kScatterThreads, 0, s>>>(gp);
    // the count variants present in the batch (partitions need an estimate above
    // twice part_keys, at most N / 2 on the main path)
    bool any32 = false, any64 = false, any_parts = false;
    for (uint32_t i = 0; i < n_cols; ++i) {
        (elem_bytes((cafs_dtype_t)cols[i].dtype) == 4 ? any32 : any64) = true;
        any_parts |= cols[i].n > 4 * args[i].part_keys;
    }
    // (a column's workgroups leave every variant's launch but one at once, so the
    // partitioned count overlaps the others on the side stream)
    if (any_parts) {
        (void)hipEventRecord(side.fork, s);
        (void)hipStreamWaitEvent(side.s, side.fork, 0);
        cafs::kb_hash_count_parts<<<TH, cafs::kCountThreads, 0, side.s>>>(gh);
        (void)hipEventRecord(side.join, side.s);
    }
    if (any64) cafs::kb_hash_count<<<TH, cafs::kCountThreads, 0, s>>>(gh);
    if (any32) cafs::kb_hash_count32<<<TH, cafs::kCountThreads, 0, s>>>(gh);
    if (any_parts) (void)hipStreamWaitEvent(s, side.join, 0);
    cafs::kb_rank<<<TP, 1024, 0, s>>>(gp);
    cafs::kb_compact_order<<<C, 1024, 0, s>>>(g1);
    cafs::kb_radix_hist<<<TP, 256, 0, s>>>(gp);
    // the radix jobs as one list per kind, worked through by fixed grids; a column's
    // job is keys-only or key-value, so the two chains of passes (different columns)
    // run side by side
    cafs::RadixList* rl = at<cafs::RadixList>(hdr_dev, P.off_rl);
    cafs::kb_radix_list<<<1, 1024, 0, s>>>(g1.args, n_cols, rl);
    (void)hipEventRecord(side.fork, s);
    (void)hipStreamWaitEvent(side.s, side.fork, 0);
    for (uint32_t p = 0; p < 8; ++p) {
        cafs::kbl_radix_pass<<<ctx->cus * 3, cafs::kRadixThreads, 0, s>>>(g1.args, rl, p);
        cafs::kbl_radix_pass_kv<<<ctx->cus * 2, cafs::kRadixThreads, 0, side.s>>>(g1.args, rl, p);
    }
    (void)hipEventRecord(side.join, side.s);
    (void)hipStreamWaitEvent(s, side.join, 0);
    cafs::kb_radix_copy<<<TP, 256, 0, s>>>(gp);
    cafs::kb_fold_sums<<<TP, 1024, 0, s>>>(gp);
    cafs::kb_fold_write<<<TP, 1024, 0, s>>>(gp);
    cafs::kb_copy_mono<<<TP, 256, 0, s>>>(gp);
    cafs::kb_rle_count<<<TP, 256, 0, s>>>(gp);
    cafs::kb_rle_write<<<TP, 256, 0, s>>>(gp);
    cafs::kb_rle_counts<<<TP, 256, 0, s>>>(gp);
    cafs::kb_guard_prep<<<TP, 256, 0, s>>>(gp);
    cafs::kb_guard_bucket<<<TP, 256, 0, s>>>(gp);
    cafs::kb_guard_mark<<<TP, 256, 0, s>>>(gp);
    cafs::kb_guard_first<<<TP, 256, 0, s>>>(gp);
    cafs::kb_guard_resolve<<<C, 1024, 0, s>>>(g1);
    for (uint32_t r = 0; r < cafs::kMaxBucketCap; ++r) cafs::kb_guard_round<<<TP, 256, 0, s>>>(gp, r);
    cafs::kb_guard_final<<<TP, 256, 0, s>>>(gp);
    // outputs written after the guard: it reads the input, which an in-place sort overwrites
    cafs::kb_copy_deferred<<<TP, 256, 0, s>>>(gp);
    cafs::kb_emit<<<TP, cafs::kEmitThreads, 0, s>>>(gp, 1u);
    cafs::kb_emit<<<TP, cafs::kEmitThreads, 0, s>>>(gp, 0u);
    cafs::kb_uniq_out<<<TP, 256, 0, s>>>(gp);
    cafs::kb_finalize<<<C, 64, 0, s>>>(g1);
    e = hipGetLastError();
    return e == hipSuccess ? CAFS_OK : hip_fail(e, "launch");
}

// Column workspaces of a contiguous batched workspace: header bound, then columns.
size_t batch_ws_layout(const uint64_t* ns, uint32_t n_cols, std::vector<size_t>* offs) {
    size_t o = align_up(header_bound(n_cols));
    if (offs) offs->resize(n_cols);
    for (uint32_t i = 0; i < n_cols; ++i) {
        if (offs) (*offs)[i] = o;
        o = align_up(o + make_layout(ns[i]).total);
    }
    return o;
}

}  // namespace

extern "C" {

size_t cafs_batched_workspace_bytes(const uint64_t* h_ns, uint32_t n_cols) {
    if (n_cols > 0 && !h_ns) return 0;
    return batch_ws_layout(h_ns, n_cols, nullptr);
}

cafs_status_t cafs_ctx_set_batch_tuning(cafs_ctx_t* ctx, uint64_t elems_per_block, uint64_t elems_per_hash_block) {
    if (!ctx || elems_per_block == 0 || elems_per_hash_block == 0) return CAFS_EINVAL;
    ctx->batch_per_block = elems_per_block;
    ctx->batch_per_hash_block = elems_per_hash_block;
    return CAFS_OK;
}

cafs_status_t cafs_ctx_set_count_geometry(cafs_ctx_t* ctx, uint64_t part_keys, uint64_t wide_min, uint64_t table_slots) {
    if (!ctx || part_keys < 256 || table_slots < 2 || table_slots > 256) return CAFS_EINVAL;
    ctx->part_keys = part_keys;
    ctx->wide_min = wide_min;
    ctx->table_slots = table_slots;
    return CAFS_OK;
}

cafs_status_t cafs_ctx_set_hash_seed(cafs_ctx_t* ctx, uint64_t seed) {
    if (!ctx) return CAFS_EINVAL;
    if (seed == 0) {
        ctx->table_mul = cafs::kPhi;
        return CAFS_OK;
    }
    // SplitMix64 output for the seed (Steele, Lea and Flood), made odd
    uint64_t z = seed + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    ctx->table_mul = z | 1ull;
    return CAFS_OK;
}

cafs_status_t cafs_sort_batched(cafs_ctx_t* ctx, const cafs_column_t* h_cols, uint32_t n_cols, void* d_ws,
                                size_t ws_bytes, void* stream) {
    if (!ctx || (n_cols > 0 && !h_cols)) return CAFS_EINVAL;
    if (n_cols == 0) return CAFS_OK;
    std::vector<uint64_t> ns;
    cafs_status_t st = check_columns(h_cols, n_cols, ns);
    if (st != CAFS_OK) return st;
    std::vector<size_t> offs;
    const size_t need = batch_ws_layout(ns.data(), n_cols, &offs);
    if (!d_ws || ws_bytes < need || reinterpret_cast<uintptr_t>(d_ws) % kAlign) return CAFS_EWORKSPACE;
    DeviceGuard dg(ctx->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const BatchShape P = shape_batch(ns.data(), n_cols, ctx->batch_per_block, ctx->batch_per_hash_block);
    std::vector<void*> col_ws(n_cols);
    for (uint32_t i = 0; i < n_cols; ++i) col_ws[i] = static_cast<char*>(d_ws) + offs[i];
    // Staging: a capture records the copy from the staging buffer into the graph, so a
    // captured call hands the context's staging buffer over to the graph (no host
    // allocation is allowed while capturing) and the next uncaptured call makes a new one.
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    (void)hipStreamIsCapturing(s, &cap);
    void* host = nullptr;
    if (cap != hipStreamCaptureStatusNone) {
        // No event query here: it is not allowed while capturing.  The caller has
        // synchronized after the last uncaptured batched call (documented).
        ctx->staged_pending = false;
        if (!ctx->staging || ctx->staging_bytes < P.header) {
            g_last_error = "capture: make an uncaptured batched call of this batch first";
            return CAFS_EUNSUPPORTED;
        }
        host = ctx->staging;
        ctx->captured_staging.push_back(host);
        ctx->staging = nullptr;
        ctx->staging_bytes = 0;
    } else {
        if (ctx->staged_pending) {
            hipError_t e = hipEventSynchronize(ctx->staged);  // the previous upload has been read
            if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
            ctx->staged_pending = false;
        }
        if (ctx->staging_bytes < P.header) {
            if (ctx->staging) (void)hipHostFree(ctx->staging);
            ctx->staging = nullptr;
            ctx->staging_bytes = 0;
            hipError_t e = hipHostMalloc(&ctx->staging, P.header, hipHostMallocDefault);
            if (e != hipSuccess) return hip_fail(e, "hipHostMalloc");
            ctx->staging_bytes = P.header;
        }
        host = ctx->staging;
    }
    st = launch_batch(ctx, h_cols, n_cols, col_ws.data(), P, d_ws, host, s, SideLane{ctx->side, ctx->fork, ctx->join});
    if (st != CAFS_OK) return st;
    if (cap == hipStreamCaptureStatusNone) {
        hipError_t e = hipEventRecord(ctx->staged, s);
        if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
        ctx->staged_pending = true;
    }
    return CAFS_OK;
}

cafs_status_t cafs_autotune_batched(cafs_ctx_t* ctx, const cafs_column_t* h_cols, uint32_t n_cols, void* d_ws,
                                    size_t ws_bytes, void* stream, double* h_best_ms) {
    if (!ctx || n_cols == 0 || !h_cols) return CAFS_EINVAL;
    DeviceGuard dg(ctx->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return hip_fail(hipGetLastError(), "hipEventCreate");
    cafs_status_t st = CAFS_OK;
    // one candidate: a warm-up run, then the faster of two timed runs
    auto time_batch = [&](double* out_ms) {
        float best = 1e30f;
        for (int rep = 0; rep < 3 && st == CAFS_OK; ++rep) {
            (void)hipEventRecord(e0, s);
            st = cafs_sort_batched(ctx, h_cols, n_cols, d_ws, ws_bytes, stream);
            (void)hipEventRecord(e1, s);
            hipError_t e = hipEventSynchronize(e1);
            if (e != hipSuccess && st == CAFS_OK) st = hip_fail(e, "hipEventSynchronize");
            float ms = 0.f;
            if (st == CAFS_OK && rep > 0 && hipEventElapsedTime(&ms, e0, e1) == hipSuccess) best = std::min(best, ms);
        }
        *out_ms = best;
    };
    double best = 1e30;
    // stage 1: workgroups per column (elements per block of the general kernels and of
    // the hash count)
    // (few elements per block give a long column of a batch more workgroups; many
    // give fewer idle launches to the short ones)
    const uint64_t per[] = {1ull << 13, 1ull << 14, 1ull << 15, 1ull << 16, 1ull << 17};
    const uint64_t per_h[] = {1ull << 15, 1ull << 16, 1ull << 17, 1ull << 18, 1ull << 19};
    uint64_t bp = ctx->batch_per_block, bh = ctx->batch_per_hash_block;
    for (uint64_t p : per) {
        for (uint64_t q : per_h) {
            ctx->batch_per_block = p;
            ctx->batch_per_hash_block = q;
            double ms;
            time_batch(&ms);
            if (st != CAFS_OK) break;
            if (ms < best) { best = ms; bp = p; bh = q; }
        }
        if (st != CAFS_OK) break;
    }
    ctx->batch_per_block = bp;
    ctx->batch_per_hash_block = bh;
    // stages 2-4: the count geometry, one parameter at a time with the others at their
    // best so far (partition size, LDS bucket width threshold, global table size)
    const uint64_t part_c[] = {4500, 6000, 9000};
    const uint64_t wide_c[] = {1200, 1800, 2600};
    const uint64_t slots_c[] = {16, 32, 64};
    uint64_t* params[] = {&ctx->part_keys, &ctx->wide_min, &ctx->table_slots};
    const uint64_t* cands[] = {part_c, wide_c, slots_c};
    for (int g = 0; g < 3 && st == CAFS_OK; ++g) {
        uint64_t keep = *params[g];
        for (int i = 0; i < 3 && st == CAFS_OK; ++i) {
            *params[g] = cands[g][i];
            double ms;
            time_batch(&ms);
            if (st == CAFS_OK && ms < best) { best = ms; keep = cands[g][i]; }
        }
        *params[g] = keep;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (h_best_ms) *h_best_ms = best;
    return st;
}

cafs_status_t cafs_ctx_get_tuning(cafs_ctx_t* ctx, uint64_t* h_vals, uint32_t n) {
    if (!ctx || (n > 0 && !h_vals)) return CAFS_EINVAL;
    const uint64_t v[] = {ctx->batch_per_block, ctx->batch_per_hash_block, ctx->part_keys, ctx->wide_min,
                          ctx->table_slots};
    for (uint32_t i = 0; i < n && i < sizeof(v) / sizeof(v[0]); ++i) h_vals[i] = v[i];
    return CAFS_OK;
}

// ---- serving -------------------------------------------------------------------
// Continuous batching: requests reserve memory in one device arena of the HBM
// budget (admission), are submitted once their input is ready, and every call to
// cafs_server_poll launches the queued requests as batches on the free streams
// and collects the batches that finished.  Requests arriving while other batches
// run join the next batch on another stream, so their work overlaps on the GPU.

struct cafs_server {
    cafs_ctx_t* ctx;
    char* arena = nullptr;
    size_t arena_bytes = 0;
    std::map<size_t, size_t> free_blocks;  // offset -> size, coalesced
    size_t used = 0, high_water = 0;
    struct Req {
        uint64_t n = 0;
        int32_t dtype = 0;
        size_t off = 0, bytes = 0;
        cafs_column_t col{};
        void* ws = nullptr;
        hipEvent_t ready = nullptr;
        int state = 0;  // 0 reserved, 1 queued, 2 running, 3 finished
    };
    std::unordered_map<uint64_t, Req> reqs;
    std::deque<uint64_t> queue;
    std::deque<uint64_t> finished;
    struct Slot {
        hipStream_t s = nullptr;
        hipStream_t side = nullptr;  // the slot's second stream (partitioned count)
        hipEvent_t fork = nullptr, join = nullptr;
        hipEvent_t done = nullptr;
        void* hdr_dev = nullptr;
        void* hdr_host = nullptr;
        std::vector<uint64_t> tickets;
        bool busy = false;
    };
    std::vector<Slot> slots;
    std::vector<hipEvent_t> events;
    uint32_t max_batch = 0;
    uint64_t next_ticket = 1;
    uint64_t n_batches = 0, n_launched = 0, n_refused = 0, max_busy = 0;
};

}  // extern "C"

namespace {

bool arena_alloc(cafs_server* sv, size_t bytes, size_t* off) {
    for (auto it = sv->free_blocks.begin(); it != sv->free_blocks.end(); ++it) {
        if (it->second >= bytes) {
            *off = it->first;
            const size_t rest = it->second - bytes;
            const size_t at2 = it->first + bytes;
            sv->free_blocks.erase(it);
            if (rest) sv->free_blocks[at2] = rest;
            sv->used += bytes;
            sv->high_water = std::max(sv->high_water, sv->used);
            return true;
        }
    }
    return false;
}

void arena_free(cafs_server* sv, size_t off, size_t bytes) {
    sv->used -= bytes;
    auto it = sv->free_blocks.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != sv->free_blocks.end() && it->first + it->second == nx->first) {
        it->second += nx->second;
        sv->free_blocks.erase(nx);
    }
    if (it != sv->free_blocks.begin()) {
        auto pv = std::prev(it);
        if (pv->first + pv->second == it->first) {
            pv->second += it->second;
            sv->free_blocks.erase(it);
        }
    }
}

}  // namespace

extern "C" {

cafs_status_t cafs_server_create(cafs_ctx_t* ctx, size_t hbm_budget, uint32_t n_streams, uint32_t max_batch,
                                 cafs_server_t** out) {
    if (!ctx || !out || n_streams == 0 || max_batch == 0 || hbm_budget < (1u << 20)) return CAFS_EINVAL;
    *out = nullptr;
    DeviceGuard dg(ctx->device);
    cafs_server_t* sv = new (std::nothrow) cafs_server_t;
    if (!sv) return CAFS_ENOMEM;
    sv->ctx = ctx;
    sv->max_batch = max_batch;
    sv->arena_bytes = hbm_budget / kAlign * kAlign;
    hipError_t e = hipMalloc(reinterpret_cast<void**>(&sv->arena), sv->arena_bytes);
    if (e != hipSuccess) {
        delete sv;
        return hip_fail(e, "hipMalloc arena");
    }
    sv->free_blocks[0] = sv->arena_bytes;
    sv->slots.resize(n_streams);
    const size_t hb = header_bound(max_batch);
    for (auto& sl : sv->slots) {
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&sl.s, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&sl.side, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.fork, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.join, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming);
        if (e == hipSuccess) e = hipMalloc(&sl.hdr_dev, hb);
        if (e == hipSuccess) e = hipHostMalloc(&sl.hdr_host, hb, hipHostMallocDefault);
    }
    *out = sv;
    if (e != hipSuccess) {
        cafs_status_t st = hip_fail(e, "server streams");
        cafs_server_destroy(sv);
        *out = nullptr;
        return st;
    }
    return CAFS_OK;
}

void cafs_server_destroy(cafs_server_t* sv) {
    if (!sv) return;
    DeviceGuard dg(sv->ctx->device);
    for (auto& sl : sv->slots) {
        if (sl.s) (void)hipStreamSynchronize(sl.s);
        if (sl.side) (void)hipStreamSynchronize(sl.side);
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.fork) (void)hipEventDestroy(sl.fork);
        if (sl.join) (void)hipEventDestroy(sl.join);
        if (sl.hdr_dev) (void)hipFree(sl.hdr_dev);
        if (sl.hdr_host) (void)hipHostFree(sl.hdr_host);
        if (sl.side) (void)hipStreamDestroy(sl.side);
        if (sl.s) (void)hipStreamDestroy(sl.s);
    }
    for (auto& kv : sv->reqs)
        if (kv.second.ready) (void)hipEventDestroy(kv.second.ready);
    for (hipEvent_t e : sv->events) (void)hipEventDestroy(e);
    if (sv->arena) (void)hipFree(sv->arena);
    delete sv;
}

cafs_status_t cafs_server_reserve(cafs_server_t* sv, uint64_t n, int32_t dtype, uint64_t* h_ticket, void** h_d_in,
                                  void** h_d_out, cafs_report_t** h_d_report) {
    if (!sv || !h_ticket || n >= (1ull << 32) || !dtype_ok((cafs_dtype_t)dtype)) return CAFS_EINVAL;
    const uint64_t eb = elem_bytes((cafs_dtype_t)dtype);
    const bool bufs = h_d_in && h_d_out && h_d_report;
    const size_t data = bufs ? 2 * align_up(n * eb) + align_up(sizeof(cafs_report_t)) : 0;
    const size_t bytes = data + align_up(make_layout(n).total);
    size_t off = 0;
    if (!arena_alloc(sv, bytes, &off)) {
        ++sv->n_refused;
        return CAFS_EBUSY;
    }
    cafs_server::Req r;
    r.n = n;
    r.dtype = dtype;
    r.off = off;
    r.bytes = bytes;
    char* base = sv->arena + off;
    r.col.n = n;
    r.col.dtype = dtype;
    if (bufs) {
        r.col.d_in = base;
        r.col.d_out = base + align_up(n * eb);
        r.col.d_report = reinterpret_cast<cafs_report_t*>(base + 2 * align_up(n * eb));
        *h_d_in = const_cast<void*>(r.col.d_in);
        *h_d_out = r.col.d_out;
        *h_d_report = r.col.d_report;
    }
    r.ws = base + data;
    const uint64_t t = sv->next_ticket++;
    sv->reqs[t] = r;
    *h_ticket = t;
    return CAFS_OK;
}

cafs_status_t cafs_server_submit(cafs_server_t* sv, uint64_t ticket, const cafs_column_t* col, void* ready_stream) {
    if (!sv) return CAFS_EINVAL;
    auto it = sv->reqs.find(ticket);
    if (it == sv->reqs.end() || it->second.state != 0) return CAFS_EINVAL;
    cafs_server::Req& r = it->second;
    if (col) {
        if (col->n != r.n || col->dtype != r.dtype || col->flags != 0) return CAFS_EINVAL;
        cafs_status_t st = check_buffers(col->d_in, col->d_out, col->n, elem_bytes((cafs_dtype_t)col->dtype));
        if (st != CAFS_OK) return st;
        if ((col->d_uniq || col->d_counts) && !col->d_report) return CAFS_EINVAL;
        r.col = *col;
    } else if (r.n > 0 && !r.col.d_in) {
        return CAFS_EINVAL;
    }
    DeviceGuard dg(sv->ctx->device);
    if (!sv->events.empty()) {
        r.ready = sv->events.back();
        sv->events.pop_back();
    } else {
        hipError_t e = hipEventCreateWithFlags(&r.ready, hipEventDisableTiming);
        if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
    }
    hipError_t e = hipEventRecord(r.ready, static_cast<hipStream_t>(ready_stream));
    if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
    r.state = 1;
    sv->queue.push_back(ticket);
    return CAFS_OK;
}

cafs_status_t cafs_server_poll(cafs_server_t* sv, uint64_t* h_tickets, uint32_t cap, uint32_t* h_n) {
    if (!sv || !h_n || (cap > 0 && !h_tickets)) return CAFS_EINVAL;
    DeviceGuard dg(sv->ctx->device);
    uint64_t busy = 0;
    for (auto& sl : sv->slots) {
        if (!sl.busy) continue;
        const hipError_t q = hipEventQuery(sl.done);
        if (q == hipErrorNotReady) { ++busy; continue; }
        if (q != hipSuccess) return hip_fail(q, "hipEventQuery");
        for (uint64_t t : sl.tickets) {
            sv->reqs[t].state = 3;
            sv->finished.push_back(t);
        }
        sl.tickets.clear();
        sl.busy = false;
    }
    for (auto& sl : sv->slots) {
        if (sl.busy || sv->queue.empty()) continue;
        const uint32_t m = (uint32_t)std::min<size_t>(sv->queue.size(), sv->max_batch);
        std::vector<cafs_column_t> cols(m);
        std::vector<void*> ws(m);
        std::vector<uint64_t> ns(m);
        sl.tickets.assign(sv->queue.begin(), sv->queue.begin() + m);
        sv->queue.erase(sv->queue.begin(), sv->queue.begin() + m);
        for (uint32_t i = 0; i < m; ++i) {
            cafs_server::Req& r = sv->reqs[sl.tickets[i]];
            hipError_t e = hipStreamWaitEvent(sl.s, r.ready, 0);
            if (e != hipSuccess) return hip_fail(e, "hipStreamWaitEvent");
            cols[i] = r.col;
            ws[i] = r.ws;
            ns[i] = r.n;
            r.state = 2;
        }
        const BatchShape P = shape_batch(ns.data(), m, sv->ctx->batch_per_block, sv->ctx->batch_per_hash_block);
        cafs_status_t st = launch_batch(sv->ctx, cols.data(), m, ws.data(), P, sl.hdr_dev, sl.hdr_host, sl.s,
                                        SideLane{sl.side, sl.fork, sl.join});
        if (st != CAFS_OK) return st;
        hipError_t e = hipEventRecord(sl.done, sl.s);
        if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
        sl.busy = true;
        ++busy;
        ++sv->n_batches;
        sv->n_launched += m;
    }
    sv->max_busy = std::max(sv->max_busy, busy);
    uint32_t k = 0;
    while (k < cap && !sv->finished.empty()) {
        h_tickets[k++] = sv->finished.front();
        sv->finished.pop_front();
    }
    *h_n = k;
    return CAFS_OK;
}

cafs_status_t cafs_server_release(cafs_server_t* sv, uint64_t ticket) {
    if (!sv) return CAFS_EINVAL;
    auto it = sv->reqs.find(ticket);
    if (it == sv->reqs.end() || (it->second.state != 3 && it->second.state != 0)) return CAFS_EINVAL;
    arena_free(sv, it->second.off, it->second.bytes);
    if (it->second.ready) sv->events.push_back(it->second.ready);
    sv->reqs.erase(it);
    return CAFS_OK;
}

cafs_status_t cafs_server_stats(cafs_server_t* sv, uint64_t* h_stats, uint32_t n) {
    if (!sv || (n > 0 && !h_stats)) return CAFS_EINVAL;
    const uint64_t v[] = {sv->n_batches, sv->n_launched, sv->n_refused, sv->max_busy, sv->high_water, sv->used,
                          (uint64_t)sv->queue.size()};
    for (uint32_t i = 0; i < n && i < sizeof(v) / sizeof(v[0]); ++i) h_stats[i] = v[i];
    return CAFS_OK;
}

const char* cafs_status_str(cafs_status_t status) {
    switch (status) {
    case CAFS_OK: return "ok";
    case CAFS_EINVAL: return "invalid argument";
    case CAFS_EWORKSPACE: return "workspace too small or misaligned";
    case CAFS_EHIP: return "HIP error";
    case CAFS_EUNSUPPORTED: return "unsupported";
    case CAFS_ENOMEM: return "out of host memory";
    case CAFS_EBUSY: return "not enough room in the server's memory budget now";
    }
    return "unknown status";
}

const char* cafs_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
