// CAFS reference oracle -- TEST INFRASTRUCTURE ONLY.
//
// A plain, slow, single-threaded CPU implementation of what the cache-aware
// frequency sort (CAFS, "A Cache-Aware Frequency Sort for Low-Cardinality
// Integer Data on x86-64") computes.  Only the test suite, the smoke check and
// the benchmark's CPU-baseline leg may load this library.  It shares no code,
// header, table or constant generator with the GPU library: every constant it
// uses is retyped here from the paper.
//
// What is exact and what is a heuristic:
//   * the sorted output and the (key, count) multiset have plain definitions
//     (Sec. 3.1: a nondecreasing permutation; K = number of distinct keys), so
//     the oracle writes those definitions out with an ordered map;
//   * the cardinality estimate (Alg. 2, Eq. chao1), the dispatcher (Alg. 3,
//     Table dispatcher), the tiny-count verification (Sec. 4.4) and the spill
//     guard (Alg. 1, Eq. hash, Eq. Msize, Alg. 4) are heuristics, so they are
//     followed step by step in the paper's order.
//
// Readings of points the paper leaves open (listed in the design notes):
//   Chao1 uses unsigned 64-bit floor division; the sample loop bound is
//   exclusive; saturation means u == 1024 literally; tiny needs K^ <= 8 and
//   u <= 8; 2K^ == N stays on the main path; monotone is tested before the
//   N < 2048 cut; a tiny miss continues on the main path with the same K^ and
//   no high-K re-test; the spill is counted in elements; the guard fires iff
//   2*spill > N; M is clamped to [8, bit_ceil(N/4)] with integer N/4.
//
// Parity status: every function here is pinned by the CPU tests (library
// sort, library stable argsort for the key-value sort, brute force over small
// alphabets, closed forms of Eq. chao1, Eq. hash
// and Eq. Msize with the paper's worked sizes, crafted bucket collisions with
// hand-derived spill counts, a Poisson check of the bucket model).  The float64
// order (TotalF64) is pinned to the IEEE 754 totalOrder of signed zeros,
// infinities, subnormals and NaNs of both signs, and to numpy's sort on ordinary
// values.

#include <cstdint>
#include <cstring>
#include <map>
#include <set>
#include <vector>
#include <algorithm>

namespace {

// Path labels, in the order the dispatcher of Alg. 3 tests them.
enum OraclePath : int32_t {
    O_MONOTONE = 0,  // trivial bypass on already-sorted input
    O_SMALL_N  = 1,  // N < 2048: fallback sort, no sampling
    O_TINY     = 2,  // K^ <= 8 and u <= 8 and the sample keys cover the input
    O_HIGH_K   = 3,  // 2 K^ > N: high-entropy fallback
    O_MAIN     = 4,  // hash-count main path, guard did not fire
    O_GUARD    = 5,  // main path ran, spill guard fired (|spill| > N/2)
};

constexpr uint64_t kSamples      = 1024;                 // s, Sec. 4.3
constexpr uint64_t kSmallN       = 2048;                 // Table dispatcher
constexpr uint64_t kTinyK        = 8;                    // Table dispatcher
constexpr uint64_t kBucketCap    = 4;                    // 64-bit keys per bucket, Sec. 4.2
constexpr uint64_t kBucketCap32  = 8;                    // 32-bit keys per bucket, Sec. 4.2
constexpr uint64_t kLoadMul      = 8;                    // Eq. Msize numerator
constexpr uint64_t kMinBuckets   = 8;                    // Eq. Msize lower clamp
constexpr uint64_t kInvGolden    = 0x9E3779B97F4A7C15ull;  // Eq. hash multiplier

uint64_t bit_ceil_u64(uint64_t v) {
    // Smallest power of two >= v (bit_ceil(0) == 1, as in C++20).
    uint64_t p = 1;
    while (p < v) p <<= 1;
    return p;
}

unsigned log2_pow2(uint64_t p) {
    unsigned m = 0;
    while ((uint64_t(1) << m) < p) ++m;
    return m;
}

// Problem definition (Sec. 3.1): the output is the input's multiset in
// nondecreasing order.  Written as count-then-emit over an ordered map: the map
// iterates keys in T's order (signed for int64, unsigned for uint64).
template <class T>
void sort_by_map(const T* x, uint64_t n, T* y) {
    std::map<T, uint64_t> m;
    for (uint64_t i = 0; i < n; ++i) ++m[x[i]];
    uint64_t p = 0;
    for (const auto& kv : m)
        for (uint64_t c = 0; c < kv.second; ++c) y[p++] = kv.first;
}

// Key-value variant (a payload per key, for the post-group-by sort the paper names
// as an integration target, Sec. Future directions): the keys come out as in the
// keys-only sort and each payload goes with its key; equal keys keep their input
// order (a stable sort).  Written out as a map from each key to the list of its
// payloads in input order, emitted in key order.
template <class T>
void sort_kv_by_map(const T* x, const uint64_t* v, uint64_t n, T* y, uint64_t* w) {
    std::map<T, std::vector<uint64_t>> m;
    for (uint64_t i = 0; i < n; ++i) m[x[i]].push_back(v[i]);
    uint64_t p = 0;
    for (const auto& kv : m)
        for (uint64_t val : kv.second) {
            y[p] = kv.first;
            w[p] = val;
            ++p;
        }
}

template <class T>
uint64_t counts_by_map(const T* x, uint64_t n, T* uniq, uint64_t* counts) {
    std::map<T, uint64_t> m;
    for (uint64_t i = 0; i < n; ++i) ++m[x[i]];
    uint64_t j = 0;
    for (const auto& kv : m) {
        if (uniq) uniq[j] = kv.first;
        if (counts) counts[j] = kv.second;
        ++j;
    }
    return j;
}

template <class T>
uint64_t distinct_count(const T* x, uint64_t n) {
    std::set<T> s(x, x + n);
    return s.size();
}

// IsMonotone (Alg. 3): nondecreasing in T's order.
template <class T>
bool is_monotone(const T* x, uint64_t n) {
    for (uint64_t i = 0; i + 1 < n; ++i)
        if (x[i + 1] < x[i]) return false;
    return true;
}

// IEEE 754 double in totalOrder (IEEE 754-2008, Sec. 5.10), held as its bit
// pattern: a set sign bit orders before a clear one; among values with a clear
// sign bit a larger pattern is a larger value (+0 < subnormals < normals < +inf <
// NaNs by payload), among values with a set sign bit a larger pattern is a
// smaller value.  Two doubles are equal exactly when their patterns are, so -0
// and +0 are distinct keys, as are NaNs with different payloads.  This is the
// floating-point variant through the bit pattern that the paper names as future
// work (Sec. Future directions).
struct TotalF64 {
    uint64_t bits;
    bool operator<(const TotalF64& o) const {
        const bool na = (bits >> 63) != 0, nb = (o.bits >> 63) != 0;
        if (na != nb) return na;
        return na ? bits > o.bits : bits < o.bits;
    }
};
static_assert(sizeof(TotalF64) == 8, "same layout as the column");

std::vector<TotalF64> as_total(const uint64_t* x, uint64_t n) {
    std::vector<TotalF64> v(n);
    if (n) std::memcpy(v.data(), x, n * sizeof(uint64_t));
    return v;
}

struct Estimate {
    uint64_t k_hat, u, f1, f2, n_samples, stride, saturated;
    std::vector<uint64_t> sample_keys;  // distinct sampled values (bit patterns)
};

// Chao1 over strided samples (Alg. 2, Eq. chao1).  Equality is on the raw
// 64-bit pattern, so the result does not depend on signedness.  The paper's
// FreqSet is an open-addressing table; u, f1 and f2 depend only on the sample
// multiset, so an ordered map stands in for it here.
Estimate chao1(const uint64_t* x, uint64_t n) {
    Estimate e{};
    e.stride = std::max<uint64_t>(1, n / kSamples);
    const uint64_t end = std::min<uint64_t>(n, kSamples * e.stride);
    std::map<uint64_t, uint64_t> freq;
    for (uint64_t i = 0; i < end; i += e.stride) {
        ++freq[x[i]];
        ++e.n_samples;
    }
    e.u = freq.size();
    for (const auto& kv : freq) {
        if (kv.second == 1) ++e.f1;
        if (kv.second == 2) ++e.f2;
        e.sample_keys.push_back(kv.first);
    }
    if (e.u == kSamples) {
        e.saturated = 1;
        e.k_hat = n;  // saturated: high-entropy input
    } else {
        e.k_hat = e.u + (e.f1 * e.f1) / (2 * (e.f2 + 1));
    }
    return e;
}

// Eq. Msize, clamped to [8, bit_ceil(N/cap)]: cap = 4 for 64-bit keys, 8 for
// 32-bit keys (a bucket of one cache line holds that many keys, Sec. 4.2).
uint64_t table_buckets(uint64_t k_hat, uint64_t n, uint64_t cap) {
    uint64_t m = bit_ceil_u64(kLoadMul * k_hat / cap);
    m = std::min<uint64_t>(m, bit_ceil_u64(n / cap));
    m = std::max<uint64_t>(m, kMinBuckets);
    return m;
}

// Eq. hash: top log2(M) bits of the 64-bit product with the inverse golden ratio.
uint64_t bucket_of(uint64_t v, uint64_t M) {
    const unsigned m = log2_pow2(M);
    return (v * kInvGolden) >> (64 - m);
}

// The main hot loop of Sec. 4.4 with its RLE step, driving the bucket update of
// Alg. 1 literally.  Each bucket is an ordered list of at most four keys (a slot
// is claimed once and never freed because counters only grow).  A run of r equal
// neighbours is one update(v, r); when the bucket is full and does not hold v,
// the run goes to the spill, counted in elements.  Returns |spill|.
uint64_t simulate_spill(const uint64_t* x, uint64_t n, uint64_t M, uint64_t cap) {
    std::vector<std::vector<uint64_t>> buckets(M);
    uint64_t spill = 0;
    uint64_t i = 0;
    while (i < n) {
        const uint64_t v = x[i];
        uint64_t r = 1;
        while (i + r < n && x[i + r] == v) ++r;  // extend the run
        std::vector<uint64_t>& b = buckets[bucket_of(v, M)];
        const bool hit = std::find(b.begin(), b.end(), v) != b.end();
        if (!hit) {
            if (b.size() < cap) b.push_back(v);  // claim an empty slot
            else spill += r;                              // full bucket: spill
        }
        i += r;
    }
    return spill;
}

// The 64-bit values the estimate, the hash and the spill simulation see for a column
// of 32-bit keys: each key's 32-bit pattern, zero-extended.
template <class T>
std::vector<uint64_t> widen32(const T* x, uint64_t n) {
    std::vector<uint64_t> b(n);
    for (uint64_t i = 0; i < n; ++i) {
        uint32_t u;
        std::memcpy(&u, &x[i], sizeof(u));
        b[i] = u;
    }
    return b;
}

struct Report {
    Estimate est;
    int32_t path;
    int32_t tiny_miss;
    uint64_t table_M, spill_elems, k_exact;
};

// Dispatcher (Alg. 3) with the tiny-count verification of Sec. 4.4 and the
// reconstruction guard of Alg. 4.  `x` gives the column's order, `bits` the same
// elements as 64-bit patterns (equality, the estimate, the tiny check and the spill
// act on the patterns).
template <class T>
Report dispatch(const T* x, const uint64_t* bits, uint64_t n, uint64_t cap) {
    Report r{};
    r.k_exact = distinct_count(x, n);
    if (is_monotone(x, n)) { r.path = O_MONOTONE; return r; }
    if (n < kSmallN) { r.path = O_SMALL_N; return r; }
    r.est = chao1(bits, n);
    bool to_main = false;
    if (r.est.k_hat <= kTinyK && r.est.u <= kTinyK) {
        // TinyCount: one counter per sampled key, then the check sum(c_j) == N.
        std::vector<uint64_t> c(r.est.sample_keys.size(), 0);
        for (uint64_t i = 0; i < n; ++i)
            for (size_t j = 0; j < c.size(); ++j)
                if (bits[i] == r.est.sample_keys[j]) ++c[j];
        uint64_t total = 0;
        for (uint64_t cj : c) total += cj;
        if (total == n) { r.path = O_TINY; return r; }
        r.tiny_miss = 1;  // an unsampled value exists: fall into the main path
        to_main = true;
    }
    if (!to_main && 2 * r.est.k_hat > n) { r.path = O_HIGH_K; return r; }
    r.table_M = table_buckets(r.est.k_hat, n, cap);
    r.spill_elems = simulate_spill(bits, n, r.table_M, cap);
    r.path = (2 * r.spill_elems > n) ? O_GUARD : O_MAIN;  // |spill| > N/2
    return r;
}

// Flattened report, in this order:
//   0 k_hat, 1 u, 2 f1, 3 f2, 4 n_samples, 5 stride, 6 saturated,
//   7 path, 8 tiny_miss, 9 table_M, 10 spill_elems, 11 k_exact
void flatten(const Report& r, uint64_t* out) {
    out[0] = r.est.k_hat; out[1] = r.est.u; out[2] = r.est.f1; out[3] = r.est.f2;
    out[4] = r.est.n_samples; out[5] = r.est.stride; out[6] = r.est.saturated;
    out[7] = uint64_t(r.path); out[8] = uint64_t(r.tiny_miss);
    out[9] = r.table_M; out[10] = r.spill_elems; out[11] = r.k_exact;
}

}  // namespace

extern "C" {

void oracle_sort_i64(const int64_t* x, uint64_t n, int64_t* y) { sort_by_map(x, n, y); }
void oracle_sort_u64(const uint64_t* x, uint64_t n, uint64_t* y) { sort_by_map(x, n, y); }

// A plain comparison sort of a copy (std::sort, one thread): the reference point
// the paper times its sorts against, reported beside the oracle's own time.
void oracle_std_sort_i64(const int64_t* x, uint64_t n, int64_t* y) {
    std::memcpy(y, x, n * sizeof(int64_t));
    std::sort(y, y + n);
}

uint64_t oracle_counts_i64(const int64_t* x, uint64_t n, int64_t* uniq, uint64_t* counts) {
    return counts_by_map(x, n, uniq, counts);
}
uint64_t oracle_counts_u64(const uint64_t* x, uint64_t n, uint64_t* uniq, uint64_t* counts) {
    return counts_by_map(x, n, uniq, counts);
}

int oracle_is_monotone_i64(const int64_t* x, uint64_t n) { return is_monotone(x, n) ? 1 : 0; }
int oracle_is_monotone_u64(const uint64_t* x, uint64_t n) { return is_monotone(x, n) ? 1 : 0; }

// out[0..6] = k_hat, u, f1, f2, n_samples, stride, saturated.
void oracle_estimate(const uint64_t* x, uint64_t n, uint64_t* out) {
    const Estimate e = chao1(x, n);
    out[0] = e.k_hat; out[1] = e.u; out[2] = e.f1; out[3] = e.f2;
    out[4] = e.n_samples; out[5] = e.stride; out[6] = e.saturated;
}

uint64_t oracle_table_M(uint64_t k_hat, uint64_t n) { return table_buckets(k_hat, n, kBucketCap); }
uint64_t oracle_table_M32(uint64_t k_hat, uint64_t n) { return table_buckets(k_hat, n, kBucketCap32); }
uint64_t oracle_hash(uint64_t v, uint64_t M) { return bucket_of(v, M); }
uint64_t oracle_spill(const uint64_t* x, uint64_t n, uint64_t M) { return simulate_spill(x, n, M, kBucketCap); }
uint64_t oracle_spill32(const uint64_t* x, uint64_t n, uint64_t M) { return simulate_spill(x, n, M, kBucketCap32); }

void oracle_report_i64(const int64_t* x, uint64_t n, uint64_t* out) {
    std::vector<uint64_t> bits(n);
    if (n) std::memcpy(bits.data(), x, n * sizeof(uint64_t));
    flatten(dispatch(x, bits.data(), n, kBucketCap), out);
}
// float64 entry points: the bit patterns are copied into TotalF64 objects (and
// back), so that no storage is read through a type it does not hold.
void oracle_report_f64(const uint64_t* x, uint64_t n, uint64_t* out) {
    const std::vector<TotalF64> v = as_total(x, n);
    flatten(dispatch(v.data(), x, n, kBucketCap), out);
}
void oracle_sort_f64(const uint64_t* x, uint64_t n, uint64_t* y) {
    const std::vector<TotalF64> v = as_total(x, n);
    std::vector<TotalF64> w(n);
    sort_by_map(v.data(), n, w.data());
    if (n) std::memcpy(y, w.data(), n * sizeof(uint64_t));
}
uint64_t oracle_counts_f64(const uint64_t* x, uint64_t n, uint64_t* uniq, uint64_t* counts) {
    const std::vector<TotalF64> v = as_total(x, n);
    std::vector<TotalF64> u(uniq ? n : 0);
    const uint64_t k = counts_by_map(v.data(), n, uniq ? u.data() : nullptr, counts);
    if (uniq && k) std::memcpy(uniq, u.data(), k * sizeof(uint64_t));
    return k;
}
int oracle_is_monotone_f64(const uint64_t* x, uint64_t n) {
    const std::vector<TotalF64> v = as_total(x, n);
    return is_monotone(v.data(), n) ? 1 : 0;
}
void oracle_report_u64(const uint64_t* x, uint64_t n, uint64_t* out) { flatten(dispatch(x, x, n, kBucketCap), out); }

// Key-value sorts (stable; payloads are opaque 64-bit words).
void oracle_sort_kv_i64(const int64_t* x, const uint64_t* v, uint64_t n, int64_t* y, uint64_t* w) {
    sort_kv_by_map(x, v, n, y, w);
}
void oracle_sort_kv_u64(const uint64_t* x, const uint64_t* v, uint64_t n, uint64_t* y, uint64_t* w) {
    sort_kv_by_map(x, v, n, y, w);
}
void oracle_sort_kv_f64(const uint64_t* x, const uint64_t* v, uint64_t n, uint64_t* y, uint64_t* w) {
    const std::vector<TotalF64> a = as_total(x, n);
    std::vector<TotalF64> b(n);
    sort_kv_by_map(a.data(), v, n, b.data(), w);
    if (n) std::memcpy(y, b.data(), n * sizeof(uint64_t));
}
void oracle_sort_kv_i32(const int32_t* x, const uint64_t* v, uint64_t n, int32_t* y, uint64_t* w) {
    sort_kv_by_map(x, v, n, y, w);
}
void oracle_sort_kv_u32(const uint32_t* x, const uint64_t* v, uint64_t n, uint32_t* y, uint64_t* w) {
    sort_kv_by_map(x, v, n, y, w);
}

// 32-bit keys (the paper's int32 specialization, Sec. 4.2, and its unsigned twin).
// Equality, the estimate, the tiny check and the spill simulation act on each key's
// 32-bit pattern zero-extended to 64 bits (Eq. hash on that value); the order is the
// key type's; M and the spill use buckets of 8 keys.
void oracle_sort_i32(const int32_t* x, uint64_t n, int32_t* y) { sort_by_map(x, n, y); }
void oracle_sort_u32(const uint32_t* x, uint64_t n, uint32_t* y) { sort_by_map(x, n, y); }
uint64_t oracle_counts_i32(const int32_t* x, uint64_t n, int32_t* uniq, uint64_t* counts) {
    return counts_by_map(x, n, uniq, counts);
}
uint64_t oracle_counts_u32(const uint32_t* x, uint64_t n, uint32_t* uniq, uint64_t* counts) {
    return counts_by_map(x, n, uniq, counts);
}
int oracle_is_monotone_i32(const int32_t* x, uint64_t n) { return is_monotone(x, n) ? 1 : 0; }
int oracle_is_monotone_u32(const uint32_t* x, uint64_t n) { return is_monotone(x, n) ? 1 : 0; }
void oracle_report_i32(const int32_t* x, uint64_t n, uint64_t* out) {
    const std::vector<uint64_t> bits = widen32(x, n);
    flatten(dispatch(x, bits.data(), n, kBucketCap32), out);
}
void oracle_report_u32(const uint32_t* x, uint64_t n, uint64_t* out) {
    const std::vector<uint64_t> bits = widen32(x, n);
    flatten(dispatch(x, bits.data(), n, kBucketCap32), out);
}

}  // extern "C"
