// Device twin of the column generator and the serving load driver (benchmark
// and test infrastructure; not part of the sort library, which it only calls
// through its C ABI).
//
// Generator: the same SplitMix64 counter stream and palettes as cafs_gen.c, so a
// uniform column generated here equals the host one bit for bit.  Zipf(s) ranks
// come from inverting the continuous power law x^-s on [1, K+1] (the host
// generator instead inverts the exact discrete CDF from a table); the serving
// load draws tens of millions of requests, too many for per-request tables.
//
// Load driver: replays a trace of request arrival times in real time.  An arrived
// request reserves memory in the server (admission under the HBM budget; a
// refused request waits, in arrival order), gets its input generated on a
// producer stream, and is submitted; the driver polls the server continuously
// and stamps each request when the host sees it finished.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdint>
#include <deque>
#include <unordered_map>
#include <vector>

#include "../include/cafs.h"

namespace {

constexpr uint64_t kGolden = 0x9E3779B97F4A7C15ull;
typedef unsigned long long u64x2 __attribute__((ext_vector_type(2)));

__host__ __device__ inline uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
__host__ __device__ inline uint64_t splitmix(uint64_t seed, uint64_t i) { return mix64(seed + (i + 1) * kGolden); }
__host__ __device__ inline uint64_t palette_seed(uint64_t seed) { return mix64(seed ^ 0x50616C6574746521ull); }
__host__ __device__ inline uint64_t stream_seed(uint64_t seed) { return mix64(seed ^ 0x5069636B73537472ull); }

__device__ inline uint64_t palette_value(int palette, uint64_t sp, uint64_t r) {
    if (palette == 1) return r;
    if (palette == 2) return splitmix(sp, 0) + (splitmix(sp, 1) | 1ull) * r;
    return mix64(sp + r);
}

// dist 0: uniform ranks (as the host); dist 1: continuous power-law ranks.
__global__ void gen_kernel(uint64_t* out, uint64_t n, uint64_t K, int dist, double s, int palette, uint64_t seed) {
    const uint64_t ss = stream_seed(seed), sp = palette_seed(seed);
    const double a = 1.0 - s;
    const double top = (std::fabs(a) < 1e-12) ? std::log((double)K + 1.0) : std::pow((double)K + 1.0, a) - 1.0;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t z = splitmix(ss, i);
        uint64_t r;
        if (K >= n && dist == 0) {
            r = i;
        } else if (dist == 0) {
            r = __umul64hi(z, K);
        } else {
            const double u = (double)(z >> 11) * (1.0 / 9007199254740992.0);
            const double x = (std::fabs(a) < 1e-12) ? std::exp(u * top) : std::pow(u * top + 1.0, 1.0 / a);
            const double f = std::floor(x) - 1.0;
            r = f < 0.0 ? 0 : (f >= (double)K ? K - 1 : (uint64_t)f);
        }
        out[i] = palette_value(palette, sp, r);
    }
}

// Plain copy with 16-byte loads and 16-byte nontemporal stores (the access shape of
// the sort's streaming kernels); a kernel of known traffic for scaling hardware
// byte counters.
__global__ void copy_kernel(const u64x2* __restrict__ src, u64x2* __restrict__ dst, uint64_t n2) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n2; i += (uint64_t)gridDim.x * blockDim.x)
        __builtin_nontemporal_store(src[i], &dst[i]);
}

double now_s() {
    using clk = std::chrono::steady_clock;
    static const clk::time_point t0 = clk::now();
    return std::chrono::duration<double>(clk::now() - t0).count();
}

}  // namespace

extern "C" {

// Fills d_out[0..n) on `stream`; returns 0 or a HIP error code.
int gen_column_dev(void* d_out, uint64_t n, uint64_t K, int dist, double s, int palette, uint64_t seed, void* stream) {
    if (n == 0) return 0;
    if (K == 0) return -1;
    const uint64_t blocks = std::min<uint64_t>((n + 255) / 256, 4096);
    gen_kernel<<<(unsigned)blocks, 256, 0, static_cast<hipStream_t>(stream)>>>(static_cast<uint64_t*>(d_out), n, K,
                                                                               dist, s, palette, seed);
    return (int)hipGetLastError();
}

// Copies bytes (a multiple of 16; both pointers 16-byte aligned) on `stream`.
int copy_dev(void* d_dst, const void* d_src, uint64_t bytes, void* stream) {
    if (bytes % 16 || reinterpret_cast<uintptr_t>(d_dst) % 16 || reinterpret_cast<uintptr_t>(d_src) % 16) return -1;
    const uint64_t n2 = bytes / 16;
    if (n2 == 0) return 0;
    const uint64_t blocks = std::min<uint64_t>((n2 + 255) / 256, 8192);
    copy_kernel<<<(unsigned)blocks, 256, 0, static_cast<hipStream_t>(stream)>>>(
        static_cast<const u64x2*>(d_src), static_cast<u64x2*>(d_dst), n2);
    return (int)hipGetLastError();
}

// Real-time replay of a request trace through a CAFS server.
//   arrival[i] (seconds from the start), n[i], k[i], seed[i]: the requests, in
//   arrival order; every request is an int64 column with power-law (s) ranks.
// Outputs per request: t_admit (memory reserved and input generation enqueued),
// t_done (the host saw it finished), path and k_exact from its report.
// stats[0..10): wall seconds, keys sorted, server counters (7), max waiting.
// Returns 0, or the failing cafs_status_t / HIP error.
int serve_replay(int device, const double* arrival, const uint64_t* n, const uint64_t* k, const uint64_t* seed,
                 uint64_t n_req, double zipf_s, uint64_t budget, uint32_t n_streams, uint32_t max_batch,
                 double* t_admit, double* t_done, int32_t* path, uint64_t* k_exact, double* stats) {
    hipSetDevice(device);
    cafs_ctx_t* ctx = nullptr;
    int rc = cafs_ctx_create(&ctx, device);
    if (rc) return rc;
    cafs_server_t* sv = nullptr;
    rc = cafs_server_create(ctx, budget, n_streams, max_batch, &sv);
    if (rc) { cafs_ctx_destroy(ctx); return rc; }
    hipStream_t producer, reporter;
    hipStreamCreateWithFlags(&producer, hipStreamNonBlocking);
    hipStreamCreateWithFlags(&reporter, hipStreamNonBlocking);
    cafs_report_t* h_rep = nullptr;
    hipHostMalloc(reinterpret_cast<void**>(&h_rep), sizeof(cafs_report_t) * 4096, hipHostMallocDefault);
    struct Live { uint64_t idx; cafs_report_t* d_rep; };
    std::unordered_map<uint64_t, Live> live;
    std::deque<uint64_t> waiting;
    std::vector<uint64_t> fin(4096);
    uint64_t next = 0, done = 0, keys = 0, max_wait = 0;
    const double t0 = now_s();
    while (done < n_req && rc == 0) {
        const double t = now_s() - t0;
        while (next < n_req && arrival[next] <= t) waiting.push_back(next++);
        max_wait = std::max<uint64_t>(max_wait, waiting.size());
        while (!waiting.empty()) {
            const uint64_t i = waiting.front();
            uint64_t ticket = 0;
            void *din = nullptr, *dout = nullptr;
            cafs_report_t* drep = nullptr;
            const int r = cafs_server_reserve(sv, n[i], CAFS_I64, &ticket, &din, &dout, &drep);
            if (r == CAFS_EBUSY && live.empty()) { rc = CAFS_ENOMEM; break; }  // can never fit the budget
            if (r == CAFS_EBUSY) break;  // admission waits for memory, in arrival order
            if (r) { rc = r; break; }
            t_admit[i] = now_s() - t0;
            rc = gen_column_dev(din, n[i], k[i], 1, zipf_s, 0, seed[i], producer);
            if (rc) break;
            rc = cafs_server_submit(sv, ticket, nullptr, producer);
            if (rc) break;
            live[ticket] = Live{i, drep};
            waiting.pop_front();
        }
        uint32_t m = 0;
        if (rc == 0) rc = cafs_server_poll(sv, fin.data(), (uint32_t)fin.size(), &m);
        if (m) {
            const double td = now_s() - t0;
            // reports of the finished requests, then their memory goes back
            for (uint32_t j = 0; j < m; ++j)
                hipMemcpyAsync(&h_rep[j], live[fin[j]].d_rep, sizeof(cafs_report_t), hipMemcpyDeviceToHost, reporter);
            hipStreamSynchronize(reporter);
            for (uint32_t j = 0; j < m && rc == 0; ++j) {
                const Live L = live[fin[j]];
                t_done[L.idx] = td;
                path[L.idx] = h_rep[j].path;
                k_exact[L.idx] = h_rep[j].k_exact;
                keys += n[L.idx];
                live.erase(fin[j]);
                rc = cafs_server_release(sv, fin[j]);
                ++done;
            }
        }
    }
    const double wall = now_s() - t0;
    uint64_t st[7] = {0};
    cafs_server_stats(sv, st, 7);
    if (stats) {
        stats[0] = wall;
        stats[1] = (double)keys;
        for (int i = 0; i < 7; ++i) stats[2 + i] = (double)st[i];
        stats[9] = (double)max_wait;
    }
    hipStreamSynchronize(producer);
    cafs_server_destroy(sv);
    hipHostFree(h_rep);
    hipStreamDestroy(producer);
    hipStreamDestroy(reporter);
    cafs_ctx_destroy(ctx);
    return rc;
}

// The same trace served one request at a time, in arrival order: each request's
// input is generated, sorted with a plain single-column call and waited for before
// the next one starts (the baseline of the serving loop).  Outputs per request:
// t_done (seconds from the start).  stats[0..2): wall seconds, keys sorted.
// Returns 0, or the failing cafs_status_t / HIP error.
int serve_fifo(int device, const double* arrival, const uint64_t* n, const uint64_t* k, const uint64_t* seed,
               uint64_t n_req, double zipf_s, double* t_done, double* stats) {
    hipSetDevice(device);
    cafs_ctx_t* ctx = nullptr;
    int rc = cafs_ctx_create(&ctx, device);
    if (rc) return rc;
    uint64_t n_max = 1;
    for (uint64_t i = 0; i < n_req; ++i) n_max = std::max<uint64_t>(n_max, n[i]);
    hipStream_t s;
    hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    void *din = nullptr, *dout = nullptr, *drep = nullptr, *dws = nullptr;
    const size_t ws_bytes = cafs_workspace_bytes(n_max, CAFS_I64);
    hipError_t e = hipMalloc(&din, n_max * 8);
    if (e == hipSuccess) e = hipMalloc(&dout, n_max * 8);
    if (e == hipSuccess) e = hipMalloc(&drep, sizeof(cafs_report_t));
    if (e == hipSuccess) e = hipMalloc(&dws, ws_bytes);
    if (e != hipSuccess) rc = (int)e;
    uint64_t keys = 0;
    const double t0 = now_s();
    for (uint64_t i = 0; i < n_req && rc == 0; ++i) {
        while (now_s() - t0 < arrival[i]) {
        }
        rc = gen_column_dev(din, n[i], k[i], 1, zipf_s, 0, seed[i], s);
        if (rc == 0)
            rc = cafs_sort_i64(ctx, static_cast<const int64_t*>(din), static_cast<int64_t*>(dout), n[i], nullptr,
                               nullptr, static_cast<cafs_report_t*>(drep), dws, ws_bytes, s);
        if (rc == 0) rc = (int)hipStreamSynchronize(s);
        t_done[i] = now_s() - t0;
        keys += n[i];
    }
    if (stats) {
        stats[0] = now_s() - t0;
        stats[1] = (double)keys;
    }
    hipFree(din);
    hipFree(dout);
    hipFree(drep);
    hipFree(dws);
    hipStreamDestroy(s);
    cafs_ctx_destroy(ctx);
    return rc;
}

}  // extern "C"
