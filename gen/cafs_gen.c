/* Seeded synthetic column generator shared by the tests, the oracle checks and
 * the benchmark.  It holds none of the sort's arithmetic: it only draws keys.
 *
 * Random numbers come from SplitMix64 (Steele, Lea and Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014) used in counter form: output i
 * of the stream with seed S is the SplitMix64 finaliser applied to
 * S + (i + 1) * 0x9E3779B97F4A7C15, so any element can be drawn independently
 * and in parallel.
 *
 * A column is defined by (n, K, distribution, palette, seed):
 *   palette  0: K distinct pseudo-random 64-bit values  v_r = mix(Sp + r)
 *               (the finaliser is a bijection, so the values are distinct);
 *            1: dictionary codes                        v_r = r;
 *            2: arithmetic progression a + b*r, odd b   (the paper's grid, Sec. 6.1).
 *   dist     0: uniform ranks  r_i = floor(z_i * K / 2^64);
 *            1: Zipf(s) ranks  r_i = min{ r : cdf[r] > u_i }, u_i = (z_i >> 11) 2^-53,
 *               cdf = normalised prefix sums of (r+1)^-s with cdf[K-1] = 1;
 *            2: sorted by group: uniform ranks, then the column is ordered by rank;
 *            3: runs: run lengths uniform in [1, 2L-1] with L = max(1, n/(4K)),
 *               each run one uniform rank;
 *            4: almost sorted: the sorted-by-group column with n/100 random
 *               position swaps.
 *   K >= n with dist 0 or 1: x_i = v_i, i.e. n distinct values in palette order.
 * The element seed convention is seed = 42 + N + K (Sec. 6.1), plus 2^32 * rep
 * and 2^40 * column or request id, applied by the caller.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define GOLDEN 0x9E3779B97F4A7C15ull

uint64_t gen_mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

uint64_t gen_splitmix(uint64_t seed, uint64_t i) { return gen_mix64(seed + (i + 1) * GOLDEN); }

static uint64_t palette_seed(uint64_t seed) { return gen_mix64(seed ^ 0x50616C6574746521ull); }
static uint64_t stream_seed(uint64_t seed) { return gen_mix64(seed ^ 0x5069636B73537472ull); }
static uint64_t shuffle_seed(uint64_t seed) { return gen_mix64(seed ^ 0x5377617073537770ull); }

static uint64_t mulhi64(uint64_t a, uint64_t b) {
    return (uint64_t)(((unsigned __int128)a * (unsigned __int128)b) >> 64);
}

uint64_t gen_palette_value(int palette, uint64_t seed, uint64_t r) {
    const uint64_t sp = palette_seed(seed);
    switch (palette) {
    case 1: return r;
    case 2: {
        const uint64_t a = gen_splitmix(sp, 0);
        const uint64_t b = gen_splitmix(sp, 1) | 1ull;
        return a + b * r;
    }
    default: return gen_mix64(sp + r);
    }
}

/* cdf[0..K-1] for Zipf(s); returns 0 on allocation failure. */
int gen_zipf_cdf(double* cdf, uint64_t K, double s) {
    double total = 0.0;
    for (uint64_t r = 0; r < K; ++r) {
        total += pow((double)(r + 1), -s);
        cdf[r] = total;
    }
    for (uint64_t r = 0; r < K; ++r) cdf[r] /= total;
    if (K) cdf[K - 1] = 1.0;
    return 1;
}

static uint64_t zipf_rank(const double* cdf, uint64_t K, uint64_t z) {
    const double u = (double)(z >> 11) * (1.0 / 9007199254740992.0);
    uint64_t lo = 0, hi = K - 1; /* smallest r with cdf[r] > u; cdf[K-1] = 1 > u */
    while (lo < hi) {
        const uint64_t mid = lo + (hi - lo) / 2;
        if (cdf[mid] > u) hi = mid; else lo = mid + 1;
    }
    return lo;
}

static int cmp_u64(const void* a, const void* b) {
    const uint64_t x = *(const uint64_t*)a, y = *(const uint64_t*)b;
    return (x > y) - (x < y);
}

/* Fills out[0..n-1].  Returns 0 on success, -1 on bad arguments. */
int gen_column(uint64_t* out, uint64_t n, uint64_t K, int dist, double s, int palette,
               uint64_t seed) {
    if (K == 0 && n > 0) return -1;
    const uint64_t ss = stream_seed(seed);
    if ((dist == 0 || dist == 1) && K >= n) {
#pragma omp parallel for schedule(static)
        for (long long i = 0; i < (long long)n; ++i)
            out[i] = gen_palette_value(palette, seed, (uint64_t)i);
        return 0;
    }
    if (dist == 1) {
        double* cdf = (double*)malloc(sizeof(double) * K);
        if (!cdf) return -1;
        gen_zipf_cdf(cdf, K, s);
#pragma omp parallel for schedule(static)
        for (long long i = 0; i < (long long)n; ++i)
            out[i] = gen_palette_value(palette, seed, zipf_rank(cdf, K, gen_splitmix(ss, (uint64_t)i)));
        free(cdf);
        return 0;
    }
    if (dist == 0 || dist == 2 || dist == 4) {
        if (dist == 0) {
#pragma omp parallel for schedule(static)
            for (long long i = 0; i < (long long)n; ++i)
                out[i] = gen_palette_value(palette, seed, mulhi64(gen_splitmix(ss, (uint64_t)i), K));
            return 0;
        }
        /* sorted by group: ranks drawn uniformly, grouped by rank */
        uint64_t* ranks = (uint64_t*)malloc(sizeof(uint64_t) * (n ? n : 1));
        if (!ranks) return -1;
#pragma omp parallel for schedule(static)
        for (long long i = 0; i < (long long)n; ++i) ranks[i] = mulhi64(gen_splitmix(ss, (uint64_t)i), K);
        qsort(ranks, n, sizeof(uint64_t), cmp_u64);
#pragma omp parallel for schedule(static)
        for (long long i = 0; i < (long long)n; ++i) out[i] = gen_palette_value(palette, seed, ranks[i]);
        free(ranks);
        if (dist == 4 && n > 1) {
            const uint64_t sw = shuffle_seed(seed);
            for (uint64_t t = 0; t < n / 100; ++t) {
                const uint64_t a = mulhi64(gen_splitmix(sw, 2 * t), n);
                const uint64_t b = mulhi64(gen_splitmix(sw, 2 * t + 1), n);
                const uint64_t tmp = out[a]; out[a] = out[b]; out[b] = tmp;
            }
        }
        return 0;
    }
    if (dist == 3) {
        const uint64_t L = (n / (4 * K)) > 1 ? n / (4 * K) : 1;
        uint64_t i = 0, run = 0;
        while (i < n) {
            const uint64_t len = 1 + mulhi64(gen_splitmix(ss, 2 * run), 2 * L - 1);
            const uint64_t v = gen_palette_value(palette, seed, mulhi64(gen_splitmix(ss, 2 * run + 1), K));
            for (uint64_t j = 0; j < len && i < n; ++j) out[i++] = v;
            ++run;
        }
        return 0;
    }
    return -1;
}
