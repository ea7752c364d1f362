/*
 * cafs.h -- C ABI of the MI355X (gfx950) CAFS hot path.
 *
 * CAFS ("A Cache-Aware Frequency Sort for Low-Cardinality Integer Data on
 * x86-64") sorts a column of N 64-bit integers whose number of distinct values
 * K is much smaller than N by counting and emitting instead of comparing.  This
 * library runs every stage of that method on one GPU:
 *   estimate  Chao1 over 1024 strided samples           (Sec. 4.3, Alg. 2, Eq. chao1)
 *   dispatch  monotone / N < 2048 / tiny / 2K^ > N / main (Sec. 4.4, Alg. 3, Table dispatcher)
 *   count     tiny-count or hash-count                    (Sec. 4.4)
 *   guard     spill guard |spill| > N/2                   (Sec. 4.5, Alg. 4, Alg. 1, Eq. hash, Eq. Msize)
 *   order     sort of the K distinct (key, count) pairs   (Sec. 4.5, Alg. 4)
 *   emit      expansion of the pairs into the output      (Sec. 4.5, Alg. 4)
 *   fallback  LSD radix sort for the high-entropy branches (Table dispatcher; the
 *             paper's fallback is a comparison sort, any correct sort gives the
 *             same output because the sorted multiset is unique, Sec. 3.1).
 *
 * Conventions for every entry point:
 *   - Pointers prefixed d_ are device pointers (hipMalloc'd or equivalent) on the
 *     context's device; h_ pointers are host memory.  The caller owns every
 *     buffer it passes; the library frees nothing it did not allocate.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *     Calls only enqueue work on it and return; no call synchronises the host,
 *     except cafs_ctx_create.  Outputs (sorted keys, counts, reports) are valid
 *     once the stream has reached the enqueued work.
 *   - Errors are returned as cafs_status_t and never thrown.  On any error
 *     nothing has been enqueued, except CAFS_EHIP, which reports a failed
 *     launch; cafs_last_error() then holds the HIP error string.
 *   - Keys are 64-bit, or 32-bit for CAFS_I32 and CAFS_U32 (the paper's int32
 *     specialization, Sec. 4.2: its bucket holds eight keys, so Eq. Msize and the
 *     spill guard use cap = 8; equality, the estimate and the hashes act on the
 *     32-bit pattern zero-extended to 64 bits; column, output and distinct-key
 *     arrays hold 4-byte keys, counts stay 64-bit).  CAFS_I64 and CAFS_I32 order
 *     keys as signed integers, CAFS_U64 and CAFS_U32 as unsigned, CAFS_F64 as IEEE
 *     754 doubles in totalOrder (-NaN < -inf < ...
 *     < -0 < +0 < ... < +inf < +NaN; NaNs by payload: the floating-point variant
 *     through the bit pattern that the paper lists as future work, Sec. Future
 *     directions); equality (used by the estimate, the counts and the guard's
 *     buckets) is on the raw 64-bit pattern, so -0 and +0 are distinct keys and
 *     so are NaNs with different payloads.
 *   - N must be below 2^32 (CAFS_EINVAL otherwise).  Positions, run offsets and
 *     the per-workgroup counters are 32-bit where that saves registers or LDS;
 *     with its workspace (about 47 bytes per key, cafs_workspace_bytes) and its
 *     input and output, a column of 2^32 keys would fill nearly all of a 288 GB GPU.
 */
#ifndef CAFS_H
#define CAFS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    CAFS_OK = 0,
    CAFS_EINVAL = -1,       /* bad argument: NULL pointer with n > 0, unknown dtype,
                               partially overlapping in/out, n >= 2^32, counts
                               requested without a report */
    CAFS_EWORKSPACE = -2,   /* ws_bytes < cafs_workspace_bytes(n) or d_ws misaligned */
    CAFS_EHIP = -3,         /* a HIP call or launch failed; see cafs_last_error() */
    CAFS_EUNSUPPORTED = -4, /* feature not available on this device */
    CAFS_ENOMEM = -5,       /* host allocation failed */
    CAFS_EBUSY = -6         /* server: the request does not fit the memory budget now */
} cafs_status_t;

typedef enum { CAFS_I64 = 0, CAFS_U64 = 1, CAFS_F64 = 2, CAFS_I32 = 3, CAFS_U32 = 4 } cafs_dtype_t;

/* Branch chosen by the dispatcher (Alg. 3), in the order it tests them. */
typedef enum {
    CAFS_PATH_MONOTONE = 0, /* input already nondecreasing: output = input */
    CAFS_PATH_SMALL_N = 1,  /* N < 2048: fallback sort without sampling */
    CAFS_PATH_TINY = 2,     /* K^ <= 8 and u <= 8 and the sampled keys cover the input */
    CAFS_PATH_HIGH_K = 3,   /* 2 K^ > N: fallback sort */
    CAFS_PATH_MAIN = 4,     /* hash-count main path; the spill guard did not fire */
    CAFS_PATH_GUARD = 5     /* main path whose spill exceeded N/2 (Alg. 4) */
} cafs_path_t;

/* What actually ran on the GPU (the label above follows the paper). */
typedef enum {
    CAFS_ENGINE_NONE = 0,  /* copy only (monotone input) */
    CAFS_ENGINE_TINY = 1,  /* wave-ballot tiny count + emit */
    CAFS_ENGINE_HASH = 2,  /* LDS/global hash count + order + emit */
    CAFS_ENGINE_RADIX = 3  /* LSD radix sort of the keys */
} cafs_engine_t;

/* Chao1 estimate over strided samples (Alg. 2, Eq. chao1):
 *   stride = max(1, floor(N/1024)); samples x[0], x[stride], ... while the index
 *   is below min(N, 1024*stride), so n_samples = min(N, 1024);
 *   u = distinct sampled values, f1 / f2 = values seen once / twice;
 *   saturated = (u == 1024); k_hat = saturated ? N : u + floor(f1^2 / (2 (f2+1)))
 *   in unsigned 64-bit arithmetic. */
typedef struct {
    uint64_t k_hat, u, f1, f2, n_samples, stride;
    uint32_t saturated, pad;
} cafs_estimate_t;

/* Per-call report.  est is zero on the MONOTONE and SMALL_N paths (the
 * dispatcher returns before sampling).  table_M (Eq. Msize, cap 4 for 64-bit
 * keys) and spill_elems (elements that the paper's bucket table of Alg. 1 would
 * send to the spill, counted in elements) are set on MAIN and GUARD only.
 * k_exact is the exact number of distinct keys.  engine is a cafs_engine_t.
 * flags: bit 0 = the GPU hash table overflowed and the radix engine sorted the
 * column instead; bit 1 = the guard needed the first-occurrence pass; bit 2 =
 * some keys went to the spill list, which was sorted and folded.
 * Every field up to k_exact is a function of the column alone.  engine and flags
 * describe what ran: which keys claim a slot of the global table first is
 * decided by timing, so a column near the table's limits can take the spill
 * list, or the radix engine, on one call and not on the next (the sorted output,
 * counts and the fields above are the same either way). */
typedef struct {
    cafs_estimate_t est;
    int32_t path;
    int32_t tiny_miss; /* 1 if the tiny branch was chosen but an unsampled value exists */
    uint64_t table_M;
    uint64_t spill_elems;
    uint64_t k_exact;
    uint32_t engine;
    uint32_t flags;
} cafs_report_t;

typedef struct cafs_ctx cafs_ctx_t;

/* Creates a context on `device` (queries its compute-unit count; synchronous).
 * Returns CAFS_EINVAL for a NULL ctx, CAFS_EHIP if the device is unusable. */
cafs_status_t cafs_ctx_create(cafs_ctx_t** ctx, int device);
void cafs_ctx_destroy(cafs_ctx_t* ctx);

/* Per-stage timing.  While enabled, every cafs_sort_i64/u64/f64 call on the context
 * records HIP events on its stream at the stage boundaries:
 *   0 pre    order check, Chao1 estimate, dispatch, table
 *            initialisation, tiny count, and the hash-partition
 *            scatter of columns estimated above 12000 keys (Alg. 2, Alg. 3, Sec. 4.4)
 *   1 count  hash count with run-length injection, and its pass over
 *            deferred elements (one kernel)                (Sec. 4.4)
 *   2 order  ranking of up to 32768 distinct keys, run offsets and the guard's
 *            bucket check, or the gather for a pair sort   (Alg. 4)
 *   3 emit   run expansion on the caller's stream: the row emit kernel (Alg. 4)
 *   4 tail   the rest until the report is written: the tile emit (K > 32768),
 *            the row emit of in-place calls (after the guard), the radix engine, the
 *            larger pair sort and its emit, the monotone copy, the run-length
 *            pass and the guard run on a side stream of the context, forked
 *            after stage 2, and count here as far as they outlast the emit.
 * Calls on one context share its side stream.
 * cafs_ctx_stage_ms waits for the recorded events, writes into h_ms[0..n_stages)
 * the summed milliseconds of each stage over every call recorded since the last
 * read, stores the number of calls in *h_calls, and forgets them.  Enabling
 * adds one event record per stage boundary to each call. */
#define CAFS_N_STAGES 5
cafs_status_t cafs_ctx_enable_timing(cafs_ctx_t* ctx, int enable);
cafs_status_t cafs_ctx_stage_ms(cafs_ctx_t* ctx, float* h_ms, int n_stages, int* h_calls);

/* Upper bound on the device workspace of one cafs_sort_i64/u64 call of n keys
 * (the same for both dtypes); depends on n only.  The workspace must be
 * 256-byte aligned and is used as scratch: its contents on entry do not matter. */
size_t cafs_workspace_bytes(uint64_t n, cafs_dtype_t dtype);

/* Chao1 estimate of the distinct-value count of d_keys[0..n) (Alg. 2).
 * Writes one cafs_estimate_t to device memory d_out.  Uses no workspace.
 * dtype names the column's key type (CAFS_I64, CAFS_U64 or CAFS_F64; anything
 * else is CAFS_EINVAL); the estimate compares keys by their 64-bit patterns only,
 * so its result is the same for every dtype.  n = 0 gives the all-zero estimate
 * with stride 1. */
cafs_status_t cafs_estimate(cafs_ctx_t* ctx, const void* d_keys, uint64_t n, cafs_dtype_t dtype,
                            cafs_estimate_t* d_out, void* stream);

/* Sorts d_in[0..n) into d_out[0..n) (nondecreasing in the dtype's order) along
 * the dispatcher of Alg. 3.  d_in == d_out (in place) is allowed; any other
 * overlap is CAFS_EINVAL.  Both must be 8-byte aligned.
 *   d_uniq, d_counts  optional (may be NULL), device arrays with room for n
 *                     entries: the distinct keys in order and their counts
 *                     (uint64); K = report.k_exact entries are written.  If
 *                     either is given, d_report must be given too.
 *   d_report          optional device cafs_report_t.
 *   d_ws, ws_bytes    device workspace of at least cafs_workspace_bytes(n).
 * Dispatch happens on the device: the call enqueues a fixed sequence of kernels
 * whose branches not taken exit at once, so it never waits for the GPU and can
 * be captured in a HIP graph. */
cafs_status_t cafs_sort_i64(cafs_ctx_t* ctx, const int64_t* d_in, int64_t* d_out, uint64_t n,
                            int64_t* d_uniq, uint64_t* d_counts, cafs_report_t* d_report,
                            void* d_ws, size_t ws_bytes, void* stream);
cafs_status_t cafs_sort_u64(cafs_ctx_t* ctx, const uint64_t* d_in, uint64_t* d_out, uint64_t n,
                            uint64_t* d_uniq, uint64_t* d_counts, cafs_report_t* d_report,
                            void* d_ws, size_t ws_bytes, void* stream);
/* 32-bit keys (CAFS_I32, CAFS_U32): the same call on 4-byte keys, which must be
 * 4-byte aligned; d_uniq receives 4-byte keys, d_counts 64-bit counts; the report's
 * table_M and spill_elems follow the paper's 32-bit bucket of eight keys.  The
 * workspace is cafs_workspace_bytes(n) as for 64-bit keys. */
cafs_status_t cafs_sort_i32(cafs_ctx_t* ctx, const int32_t* d_in, int32_t* d_out, uint64_t n,
                            int32_t* d_uniq, uint64_t* d_counts, cafs_report_t* d_report,
                            void* d_ws, size_t ws_bytes, void* stream);
cafs_status_t cafs_sort_u32(cafs_ctx_t* ctx, const uint32_t* d_in, uint32_t* d_out, uint64_t n,
                            uint32_t* d_uniq, uint64_t* d_counts, cafs_report_t* d_report,
                            void* d_ws, size_t ws_bytes, void* stream);
/* Doubles in totalOrder (CAFS_F64); d_uniq receives the distinct values. */
cafs_status_t cafs_sort_f64(cafs_ctx_t* ctx, const double* d_in, double* d_out, uint64_t n,
                            double* d_uniq, uint64_t* d_counts, cafs_report_t* d_report,
                            void* d_ws, size_t ws_bytes, void* stream);

/* Key-value sort: keys of any dtype with one opaque 64-bit payload each (a row id
 * or a value), for the post-group-by sort of a query engine that the paper names as
 * an integration target (Sec. Future directions).
 *   d_keys_in   n keys of `dtype` (device, 4- or 8-byte aligned by width)
 *   d_keys_out  n keys: the keys in the dtype's order, as cafs_sort_* writes them
 *   d_vals_in   n payloads (device, 8-byte aligned)
 *   d_vals_out  n payloads: each input payload at its key's output position; equal
 *               keys keep their input order (the sort is stable)
 * d_uniq, d_counts, d_report, d_ws and ws_bytes (cafs_workspace_bytes(n)) as for
 * cafs_sort_*; the report is the keys-only report of the same keys.  Neither output
 * may share a byte with another of the four buffers (no in-place sort; the two
 * inputs may overlap, they are only read): CAFS_EINVAL otherwise, as for
 * null buffers with n > 0, misalignment, n >= 2^32 or an unknown dtype; nothing is
 * enqueued then.  On the count paths the payloads are placed by a stable sort on
 * the digits of each key's rank among the distinct keys (one pass of 8-bit digits
 * per byte of K - 1); on the radix engine's paths they move with the keys. */
cafs_status_t cafs_sort_kv(cafs_ctx_t* ctx, const void* d_keys_in, void* d_keys_out,
                           const uint64_t* d_vals_in, uint64_t* d_vals_out, uint64_t n,
                           cafs_dtype_t dtype, void* d_uniq, uint64_t* d_counts,
                           cafs_report_t* d_report, void* d_ws, size_t ws_bytes, void* stream);

/* For callers that cannot allocate device memory or pass a workspace (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation): the
 * sort of cafs_sort_i64 / _u64 / _f64 (dtype selects which) with the same buffer
 * rules, outputs and report, but without a workspace argument.  Its workspace is a
 * static device array sized for CAFS_NOALLOC_MAX_N keys
 * (cafs_workspace_bytes(CAFS_NOALLOC_MAX_N) bytes, about 92 MiB), one copy per
 * GPU, held from the library's load until the process ends; its address is looked
 * up when the first context on the device is created.  The call allocates nothing
 * (no hipMalloc, no events; stage timing does not apply).  n > CAFS_NOALLOC_MAX_N is
 * CAFS_EINVAL.  Every call on one GPU shares that array: calls that overlap on a GPU
 * (on different streams, or different contexts, without ordering between them) race
 * and give wrong results.  The array needs no clearing: every call writes what it
 * reads (its contents on entry do not matter, as for a caller's workspace). */
#define CAFS_NOALLOC_MAX_N (1u << 20)
cafs_status_t cafs_sort_noalloc(cafs_ctx_t* ctx, const void* d_in, void* d_out, uint64_t n, cafs_dtype_t dtype,
                                void* d_uniq, uint64_t* d_counts, cafs_report_t* d_report, void* stream);

/* The fallback engine on its own: LSD radix sort with 8-bit digits and decoupled
 * look-back (digits on which every key agrees are skipped).  It is the GPU
 * baseline the CAFS path is measured against.  Same buffer rules as above;
 * uses cafs_workspace_bytes(n) of workspace. */
cafs_status_t cafs_radix_sort(cafs_ctx_t* ctx, const void* d_in, void* d_out, uint64_t n,
                              cafs_dtype_t dtype, void* d_ws, size_t ws_bytes, void* stream);

/* One column of a batched call. */
typedef struct {
    const void* d_in;
    void* d_out;
    uint64_t n;
    int32_t dtype;          /* cafs_dtype_t */
    int32_t flags;          /* reserved, must be 0 */
    void* d_uniq;           /* optional, room for n keys */
    uint64_t* d_counts;     /* optional, room for n counts */
    cafs_report_t* d_report;/* optional (required if d_uniq or d_counts is set) */
} cafs_column_t;

/* Workspace for a batched call over the given column lengths. */
size_t cafs_batched_workspace_bytes(const uint64_t* h_ns, uint32_t n_cols);

/* Sorts n_cols independent columns; each column's outputs are identical to a
 * cafs_sort_* call on it.  Every kernel is launched once for the whole batch
 * (each block works on one column), so the launch count does not grow with
 * n_cols.  h_cols is read before the call returns.  A call on a stream that is
 * not capturing waits on the host until the previous batched call of the context
 * has read its staged header (an early, small copy).  The call may be captured
 * in a HIP graph: the header is staged in a pinned host buffer that the graph
 * keeps (freed with the context).  Capturing needs an earlier uncaptured batched
 * call of a batch at least as large on this context (else CAFS_EUNSUPPORTED,
 * nothing enqueued), and the caller must have synchronized with that call's
 * stream before capturing: a capture cannot query the GPU. */
cafs_status_t cafs_sort_batched(cafs_ctx_t* ctx, const cafs_column_t* h_cols, uint32_t n_cols,
                                void* d_ws, size_t ws_bytes, void* stream);

/* Block sizing of batched launches: each column gets ceil(n / elems_per_block)
 * blocks (at most 64) in the general kernels and ceil(n / elems_per_hash_block)
 * in the hash count.  Affects speed only.  Defaults 65536 and 262144; the
 * autotuner (cafs_autotune_batched) picks them by timing. */
cafs_status_t cafs_ctx_set_batch_tuning(cafs_ctx_t* ctx, uint64_t elems_per_block, uint64_t elems_per_hash_block);

/* Geometry of the hash count (affects speed only; outputs and reports do not depend
 * on it).  part_keys: estimated distinct keys per hash partition (the column is
 * scattered into up to 16 partition buckets when the estimate exceeds twice this;
 * at least 256).  wide_min: the estimate per partition from which the LDS table's
 * buckets hold 4 keys instead of 2.  table_slots: global table slots per estimated
 * key (2 to 256; half the slots may be claimed, keys past that go to the spill
 * list).  Defaults 6000, 1800 and 32; cafs_autotune_batched tunes them for a
 * batch.  Applies to calls enqueued afterwards on the context.  CAFS_EINVAL for a
 * null context or values out of range. */
cafs_status_t cafs_ctx_set_count_geometry(cafs_ctx_t* ctx, uint64_t part_keys, uint64_t wide_min, uint64_t table_slots);

/* Seeds the hash of the GPU's count tables (the per-workgroup LDS tables and the
 * global table), against the deterministic-collision attack of a fixed hash (Sec.
 * Limitations; a randomised seed is named in Sec. Future directions).  The hash is
 * multiply-shift: seed 0 (the default) keeps the multiplier of Eq. hash; any other
 * seed selects the odd multiplier (SplitMix64 output of the seed) | 1, a member of
 * the universal multiply-shift family, so that keys chosen to collide under one
 * multiplier spread under another.  Sorted output, counts and report do not depend
 * on the seed: the spill guard keeps Eq. hash, since the report follows the paper's
 * bucket table (Alg. 1).  Affects calls enqueued after it on this context (single,
 * batched and served).  CAFS_EINVAL for a null context. */
cafs_status_t cafs_ctx_set_hash_seed(cafs_ctx_t* ctx, uint64_t seed);

/* Autotuner of batched calls: times the batch (synchronously; per candidate a
 * warm-up run and the faster of two timed runs) and keeps the fastest settings in
 * the context.  First the workgroups per column (2^15..2^18 elements per block of
 * the general kernels, 2^17..2^20 of the hash count, all 16 pairs), then the count
 * geometry of cafs_ctx_set_count_geometry one parameter at a time (keys per
 * partition 4500/6000/9000, 4-key LDS buckets from an estimate per partition of
 * 1200/1800/2600, 16/32/64 global table slots per estimated key).  The batch is
 * sorted many times, so in-place columns are timed as already sorted after the
 * first run.  *h_best_ms receives the best batch time. */
cafs_status_t cafs_autotune_batched(cafs_ctx_t* ctx, const cafs_column_t* h_cols, uint32_t n_cols, void* d_ws,
                                    size_t ws_bytes, void* stream, double* h_best_ms);

/* The context's tuning, into h_vals[0..n): elements per block of the batched
 * general kernels and of the batched hash count, keys per partition, the 4-key
 * bucket threshold and global table slots per estimated key. */
cafs_status_t cafs_ctx_get_tuning(cafs_ctx_t* ctx, uint64_t* h_vals, uint32_t n);

/* ---- Serving: continuous batching under an HBM budget ------------------------
 * A server owns one device arena of hbm_budget bytes (allocated at create) and
 * n_streams streams.  A request first reserves arena memory for its workspace
 * (and, when all three pointers are given, for its input, output and report):
 * that is admission, refused with CAFS_EBUSY while the budget is used up.  Once
 * its input is ready on `ready_stream` it is submitted.  cafs_server_poll
 * launches queued requests as batches (at most max_batch columns each, in
 * submission order) on streams whose previous batch has finished, and returns the
 * tickets of finished requests, whose outputs and reports are then valid.
 * Requests submitted while batches run go into the next batch on another stream,
 * so their work overlaps on the GPU.  Each request's results are identical to a
 * cafs_sort_* call on it.  A server is used from one host thread; the context's
 * batch tuning applies.  Memory goes back to the arena with cafs_server_release. */
typedef struct cafs_server cafs_server_t;
cafs_status_t cafs_server_create(cafs_ctx_t* ctx, size_t hbm_budget, uint32_t n_streams, uint32_t max_batch,
                                 cafs_server_t** out);
void cafs_server_destroy(cafs_server_t* sv);  /* waits for running batches */
cafs_status_t cafs_server_reserve(cafs_server_t* sv, uint64_t n, int32_t dtype, uint64_t* h_ticket,
                                  void** h_d_in, void** h_d_out, cafs_report_t** h_d_report);
/* col = NULL sorts the reserved buffers; otherwise col (same n and dtype) names
 * the caller's buffers and only the workspace comes from the arena. */
cafs_status_t cafs_server_submit(cafs_server_t* sv, uint64_t ticket, const cafs_column_t* col, void* ready_stream);
cafs_status_t cafs_server_poll(cafs_server_t* sv, uint64_t* h_tickets, uint32_t cap, uint32_t* h_n);
/* Returns the memory of a finished (or never submitted) request to the arena. */
cafs_status_t cafs_server_release(cafs_server_t* sv, uint64_t ticket);
/* h_stats[0..n): batches launched, requests launched, reservations refused,
 * most batches running at once, arena high-water bytes, arena bytes in use,
 * requests queued. */
cafs_status_t cafs_server_stats(cafs_server_t* sv, uint64_t* h_stats, uint32_t n);

const char* cafs_status_str(cafs_status_t status);
/* Detail of the last CAFS_EHIP on the calling thread ("" if none). */
const char* cafs_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* CAFS_H */
