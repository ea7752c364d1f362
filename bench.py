#!/usr/bin/env python3
"""Throughput of the CAFS hot path on one MI355X.

A step is one cafs_sort_i64 call over the HBM-scale column: N = 2^28 int64 keys,
K = 1000 distinct random 64-bit values with Zipf(1.0) frequencies (seed
42 + N + K).  The input is resident in HBM before the timed region; the report
(estimate, path, K, spill) is produced in every step.  Prints one JSON line.

Beside the CAFS number it times the library's own LSD radix sort (the GPU
baseline) on the same input, the dominant kernel's achieved HBM bandwidth from
HIP events recorded around it inside the timed region, and the CPU oracle on a
bounded prefix of the same column.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E peak
WORKLOADS = {
    # name: (n, k, dist, s, palette)
    "hbm_scale_column": (1 << 28, 1000, "zipf", 1.0, "random"),
    "plain_single_column": (1_000_000, 200, "uniform", 1.1, "random"),
    # the count loop as the table fills (hardware counter runs of the hash count)
    "hbm_k1000_uniform": (1 << 28, 1000, "uniform", 1.1, "random"),
    "hbm_k4000_uniform": (1 << 28, 4000, "uniform", 1.1, "random"),
    "hbm_k10000_uniform": (1 << 28, 10_000, "uniform", 1.1, "random"),
    # the tiny branch beside the main path at the dispatcher sweep's length
    "sweep_tiny_k8": (30_000_000, 8, "uniform", 1.1, "random"),
    "sweep_main_k200": (30_000_000, 200, "uniform", 1.1, "random"),
    # a heavy-tailed column of the sweep whose count geometry follows the larger sample
    "sweep_main_zipf11_k130000": (30_000_000, 130_000, "zipf", 1.1, "random"),
}
# algorithmic bytes per key of each single-kernel stage
STAGE_BYTES_PER_KEY = {"count": 8.0, "emit": 8.0}
STAGE_KERNEL = {"count": "k_hash_count", "emit": "k_emit_rows"}
KERNEL_SOURCES = ["paper_2605_25040_amd/csrc/cafs_dev.h", "paper_2605_25040_amd/csrc/k_count.h",
                  "paper_2605_25040_amd/csrc/k_emit.h", "paper_2605_25040_amd/csrc/cafs_api.hip"]


def progress(msg):
    """A progress line on stderr (the bench line itself is the only stdout output)."""
    sys.stderr.write("bench: %s (%.0f s)\n" % (msg, time.time() - _T0))
    sys.stderr.flush()


_T0 = time.time()


def sources_hash():
    """Hash of the kernel sources' code: line comments, trailing blanks and empty
    lines are left out, so that an edit of the comments keeps the counter runs valid."""
    import re
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "r") as f:
            for line in f:
                code = re.sub(r"//.*$", "", line).rstrip()
                if code:
                    h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]


def measured_traffic(kernel, n):
    """HBM bytes per launch from committed rocprofv3 counter runs, or None when
    absent or taken on different kernel sources."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        t = json.load(open(path))
    except ValueError:
        return None
    e = t.get(kernel)
    if not e or e.get("sources_hash") != sources_hash() or e.get("n") != n:
        return None
    return e.get("bytes_per_launch")


def _cpu_model():
    """Model name of the host CPU (first /proc/cpuinfo entry), or None."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(x_np, seconds_hint):
    import numpy as np

    import oracle
    m = min(x_np.size, 1 << 25)
    sample = np.ascontiguousarray(x_np[:m])
    best = None
    for _ in range(2):  # the paper's protocol: minimum of two runs
        t0 = time.perf_counter()
        oracle.sort(sample)
        dt = time.perf_counter() - t0
        best = dt if best is None else min(best, dt)
    # a plain std::sort of the same sample, one thread, beside it
    best_std = None
    for _ in range(2):
        t0 = time.perf_counter()
        oracle.std_sort_i64(sample)
        dt = time.perf_counter() - t0
        best_std = dt if best_std is None else min(best_std, dt)
    host = {"cpu_model": _cpu_model(), "nproc": os.cpu_count()}
    return {"value": m / best / 1e9, "unit": "Gkeys/s", "cores": 1, "kind": "oracle", "host": host,
            "sample": "first %d keys of the same column (std::map count + emit, single thread, min of 2 runs, %.2f s each)"
                      % (m, best),
            "std_sort": {"value": m / best_std / 1e9, "unit": "Gkeys/s", "cores": 1,
                         "sample": "the same keys, std::sort of a copy, single thread, min of 2 runs, %.2f s each"
                                   % best_std}}


def pct(a, q):
    import numpy as np
    return float(np.percentile(np.asarray(a), q))


def bench_batched(ctx, n_cols=4096, total=1 << 28, reps=50, seq_reps=1):
    """One batched call over n_cols columns vs the same columns sorted by
    sequential single-column calls on one stream."""
    import numpy as np
    import torch

    import gen
    import paper_2605_25040_amd as cafs
    spec = gen.batch_spec(n_cols, seed=2026, total=total)
    ns = [c["n"] for c in spec]
    total_keys = int(sum(ns))
    flat = np.empty(total_keys, dtype=np.int64)
    offs = np.concatenate([[0], np.cumsum(ns)])
    for i, c in enumerate(spec):
        gen.column(c["n"], c["k"], dist=c["dist"], s=c["s"], seed=c["seed"], dtype=np.int64,
                   out=flat[offs[i]:offs[i + 1]].view(np.uint64))
    dev = torch.device("cuda", 0)
    x = torch.from_numpy(flat).to(dev)
    y = torch.empty_like(x)
    reps_t = torch.zeros(n_cols, cafs.report_size(), dtype=torch.uint8, device=dev)
    cols = [{"in": x[offs[i]:offs[i + 1]], "out": y[offs[i]:offs[i + 1]], "report": reps_t[i]}
            for i in range(n_cols)]
    ws = torch.empty(ctx.batched_workspace_bytes(ns), dtype=torch.uint8, device=dev)
    tuned_ms = ctx.autotune_batched(cols, ws=ws)
    tuning = ctx.tuning()
    for _ in range(2):
        ctx.sort_batched(cols, ws=ws)
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for e0, e1 in evs:
        e0.record()
        ctx.sort_batched(cols, ws=ws)
        e1.record()
    torch.cuda.synchronize()
    lat = [e0.elapsed_time(e1) for e0, e1 in evs]
    y_eager, rep_eager = y.clone(), reps_t.clone()
    # graph-captured batched call, replayed
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        ctx.sort_batched(cols, ws=ws)
        torch.cuda.synchronize()
        with torch.cuda.graph(g, stream=s):
            ctx.sort_batched(cols, ws=ws)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    gevs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for e0, e1 in gevs:
        e0.record()
        g.replay()
        e1.record()
    torch.cuda.synchronize()
    glat = [e0.elapsed_time(e1) for e0, e1 in gevs]
    # replays == eager call: the sorted columns and every report field the paper
    # defines (the engine and flags words after them record what ran, which can
    # differ between calls on the same input)
    nfix = cafs.report_fixed_bytes()
    ok_graph = bool(torch.equal(y, y_eager) and torch.equal(reps_t[:, :nfix], rep_eager[:, :nfix]))
    diag_same = bool(torch.equal(reps_t[:, nfix:], rep_eager[:, nfix:]))
    # sequential single-column calls on one stream (the baseline of the batched pattern)
    lib, h = ctx._lib, ctx._h
    sws = ctx.workspace(ctx.workspace_bytes(max(ns)))
    stream = torch.cuda.current_stream(dev).cuda_stream
    seq = []
    for _ in range(seq_reps + 1):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for c in cols:
            rc = lib.cafs_sort_i64(h, c["in"].data_ptr(), c["out"].data_ptr(), c["in"].numel(), None, None,
                                   c["report"].data_ptr(), sws.data_ptr(), sws.numel(), stream)
            assert rc == 0
        e1.record()
        torch.cuda.synchronize()
        seq.append(e0.elapsed_time(e1))
    seq_ms = min(seq[1:])
    p50 = pct(lat, 50)
    del x, y, ws, g
    torch.cuda.empty_cache()
    return {"columns": n_cols, "keys": total_keys, "p50_ms": round(p50, 3), "p99_ms": round(pct(lat, 99), 3),
            "gkeys_s": round(total_keys / p50 / 1e6, 2),
            "graph_p50_ms": round(pct(glat, 50), 3), "graph_p99_ms": round(pct(glat, 99), 3),
            "sequential_ms": round(seq_ms, 3), "vs_sequential": round(seq_ms / p50, 2), "graph_ok": ok_graph, "graph_diag_same": diag_same,
            "tuning": tuning, "tuned_ms": round(tuned_ms, 3)}


def bench_structured(ctx, n=1 << 28, steps=10):
    """Columns made of runs of equal keys (mean run length n / (4K), random 64-bit
    values), where the count's run-length injection merges elements: Gkeys/s per
    column shape, inputs resident."""
    import numpy as np
    import torch

    import gen
    import paper_2605_25040_amd as cafs
    res = {}
    for dist, k in (("runs", 64), ("runs", 10_000)):
        h = gen.column(n, k, dist=dist, palette="random", dtype=np.int64)
        x = torch.from_numpy(h).to("cuda")
        del h
        out = torch.empty_like(x)
        ws = ctx.workspace(ctx.workspace_bytes(n))
        for _ in range(2):
            _, rep, _, _ = ctx.sort(x, out=out, ws=ws)
        torch.cuda.synchronize()
        r = cafs.parse_report(rep)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            ctx.sort(x, out=out, ws=ws)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        res["%s_k%d" % (dist, k)] = {"n": n, "ms": round(ms, 4), "gkeys_s": round(n / ms / 1e6, 2),
                                     "path": r["path"], "k_exact": r["k_exact"]}
        del x, out, ws
        ctx._ws = None
        torch.cuda.empty_cache()
    return res


def bench_variants(ctx, n=1 << 28, k=1000, steps=10):
    """The headline column shape (N = 2^28, K = 1000, Zipf(1.0)) as float64 keys
    (IEEE 754 totalOrder; a palette of normal doubles over the same rank stream), as
    int64 keys through a context with a seeded count-table hash, as int64 keys with
    int64 row-id payloads (key-value sort), and as int32 keys."""
    import numpy as np
    import torch

    import gen
    import paper_2605_25040_amd as cafs

    def timed(x, unsigned=False):
        out = torch.empty_like(x)
        ws = ctx.workspace(ctx.workspace_bytes(n))
        for _ in range(2):
            _, rep, _, _ = ctx.sort(x, unsigned=unsigned, out=out, ws=ws)
        torch.cuda.synchronize()
        r = cafs.parse_report(rep)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            ctx.sort(x, unsigned=unsigned, out=out, ws=ws)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        del out
        return {"n": n, "ms": round(ms, 4), "gkeys_s": round(n / ms / 1e6, 2), "path": r["path"],
                "k_exact": r["k_exact"]}

    def timed_kv(keys, steps_kv=5):
        """Key-value sort with row-id payloads; torch's stable sort with a gather of
        the payloads is timed beside it (the library way to do the same)."""
        vals = torch.arange(n, dtype=torch.int64, device="cuda")
        ko, vo = torch.empty_like(keys), torch.empty_like(vals)
        ws = ctx.workspace(ctx.workspace_bytes(n))
        for _ in range(2):
            _, _, rep, _, _ = ctx.sort_kv(keys, vals, out_keys=ko, out_vals=vo, ws=ws)
        torch.cuda.synchronize()
        r = cafs.parse_report(rep)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps_kv):
            ctx.sort_kv(keys, vals, out_keys=ko, out_vals=vo, ws=ws)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps_kv
        del ko, vo
        sk, idx = torch.sort(keys, stable=True)
        _ = vals[idx]
        del sk, idx, _
        torch.cuda.synchronize()
        e0.record()
        for _ in range(2):
            sk, idx = torch.sort(keys, stable=True)
            g = vals[idx]
            del sk, idx, g
        e1.record()
        torch.cuda.synchronize()
        t_ms = e0.elapsed_time(e1) / 2
        del vals
        torch.cuda.empty_cache()
        return {"n": n, "ms": round(ms, 4), "gkeys_s": round(n / ms / 1e6, 2), "path": r["path"],
                "k_exact": r["k_exact"], "payload": "int64 row ids",
                "torch_stable_sort_gather_ms": round(t_ms, 4), "vs_torch": round(t_ms / ms, 2)}

    res = {}
    codes = torch.empty(n, dtype=torch.int64, device="cuda")
    gen.column_device(codes, k, dist="zipf", s=1.0, palette="codes")
    pal = torch.from_numpy(np.random.default_rng(7).normal(size=k) * 1e3).to("cuda")
    x = pal[codes]
    del codes
    res["float64_k%d" % k] = timed(x)
    del x
    x = torch.empty(n, dtype=torch.int64, device="cuda")
    gen.column_device(x, k, dist="zipf", s=1.0, palette="random")
    ctx.set_hash_seed(0x5EED)
    try:
        res["seeded_hash_k%d" % k] = timed(x)
    finally:
        ctx.set_hash_seed(0)
    res["key_value_k%d" % k] = timed_kv(x)
    # 32-bit keys: the low halves of the same values (K stays 1000)
    x32 = (x & 0xFFFFFFFF).to(torch.int32)
    del x
    torch.cuda.empty_cache()
    res["int32_k%d" % k] = timed(x32)
    del x32
    ctx._ws = None
    torch.cuda.empty_cache()
    return res


def bench_serving(seconds, rate=10_000, budget=64 << 30, fifo_seconds=2.0):
    """Real-time Poisson replay through the server, then the first fifo_seconds of
    the same trace served one request at a time with plain calls (the baseline)."""
    import numpy as np

    import gen
    arrival, n, k, seeds = gen.serving_trace(rate=rate, seconds=seconds)
    res = gen.serve_replay(arrival, n, k, seeds, budget=budget, n_streams=4, max_batch=1024)
    lat = (res["t_done"] - arrival) * 1e3
    st = res["stats"]
    paths = np.bincount(res["path"], minlength=6).tolist()
    m = int(np.searchsorted(arrival, min(fifo_seconds, seconds)))
    fifo = gen.serve_fifo(arrival[:m], n[:m], k[:m], seeds[:m])
    flat = (fifo["t_done"] - arrival[:m]) * 1e3
    fifo_gk = fifo["stats"]["keys"] / fifo["stats"]["wall_s"] / 1e9
    server_gk = st["keys"] / st["wall_s"] / 1e9
    return {"seconds": seconds, "rate_req_s": rate, "requests": int(arrival.size),
            "fifo": {"requests": m, "gkeys_s": round(fifo_gk, 2), "served_req_s": round(m / fifo["stats"]["wall_s"], 1),
                     "p50_ms": round(pct(flat, 50), 3), "p99_ms": round(pct(flat, 99), 3)},
            "vs_fifo": round(server_gk / fifo_gk, 2),
            "served_req_s": round(arrival.size / st["wall_s"], 1),
            "gkeys_s": round(st["keys"] / st["wall_s"] / 1e9, 2),
            "p50_ms": round(pct(lat, 50), 3), "p99_ms": round(pct(lat, 99), 3), "p999_ms": round(pct(lat, 99.9), 3),
            "batches": int(st["batches"]), "max_streams_busy": int(st["max_busy_streams"]),
            "admission_refusals": int(st["refused"]), "arena_high_water_gb": round(st["arena_high_water"] / 2**30, 2),
            "paths": dict(zip(("MONOTONE", "SMALL_N", "TINY", "HIGH_K", "MAIN", "GUARD"), paths))}


SWEEP_N = 30_000_000
SWEEP_KS = (4, 8, 200, 10_000, 130_000, 670_000, 3_000_000, 30_000_000)


def run_sweep(seeds=3, steps=5, warmup=2):
    """The dispatcher sweep (N = 3e7; K in SWEEP_KS; uniform and Zipf(1.1); seeds
    42 + N + K + 2^32 rep), the plain column and the u64 dictionary-code variant of
    the HBM-scale column.  Every config is checked against the oracle's report
    (all fields) and for order on the device; prints one JSON object per config and
    a markdown table at the end."""
    import numpy as np
    import torch

    import gen
    import oracle
    import paper_2605_25040_amd as cafs
    dev = torch.device("cuda", 0)
    ctx = cafs.Context(0)
    cfgs = [("plain", 1_000_000, 200, "uniform", 1.1, "random", "i64", 0)]
    for dist in ("uniform", "zipf"):
        for k in SWEEP_KS:
            for rep in range(seeds):
                cfgs.append(("sweep", SWEEP_N, k, dist, 1.1, "random", "i64", rep))
    cfgs.append(("hbm_codes_u64", 1 << 28, 1000, "zipf", 1.0, "codes", "u64", 0))
    rows = []
    # the oracle's reports are computed on host threads (the library call releases
    # the GIL) while the GPU runs the next configs
    from concurrent.futures import ThreadPoolExecutor
    pool = ThreadPoolExecutor(max_workers=8)
    pending = []
    flush = torch.empty(1 << 27, dtype=torch.int64, device=dev)  # 1 GiB, written before each cold call
    for name, n, k, dist, s, pal, dt, rep in cfgs:
        seed = gen.default_seed(n, k, rep)
        x_np = gen.column(n, k, dist=dist, s=s, palette=pal, seed=seed, dtype=np.uint64)
        unsigned = dt == "u64"
        x = torch.from_numpy(x_np.view(np.int64)).to(dev)
        out = torch.empty_like(x)
        ws = ctx.workspace(ctx.workspace_bytes(n))
        rep_t = torch.zeros(cafs.report_size(), dtype=torch.uint8, device=dev)
        fn = ctx._lib.cafs_sort_u64 if unsigned else ctx._lib.cafs_sort_i64
        stream = torch.cuda.current_stream(dev).cuda_stream

        def step():
            rc = fn(ctx._h, x.data_ptr(), out.data_ptr(), n, None, None, rep_t.data_ptr(), ws.data_ptr(),
                    ws.numel(), stream)
            if rc != 0:
                raise RuntimeError("sort failed: %d" % rc)
        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            step()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        # cold: the 256 MB last-level cache (MALL) is flushed by writing a 1 GiB buffer
        # before each call, which is timed on its own
        cold = []
        for _ in range(steps):
            flush.fill_(1)
            c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            c0.record()
            step()
            c1.record()
            torch.cuda.synchronize()
            cold.append(c0.elapsed_time(c1))
        ms_cold = float(np.median(cold))
        r = cafs.parse_report(rep_t)
        o = out if not unsigned else (out ^ (-(2 ** 63)))  # unsigned order as signed order
        ordered = bool((o[1:] >= o[:-1]).all())
        if n <= 50_000_000:
            fut = pool.submit(oracle.report, x_np, np.uint64 if unsigned else np.int64)
            fields_of = (lambda r=r, fut=fut: [f for f in oracle.REPORT_FIELDS if r[f] != fut.result()[f]])
        else:
            est = oracle.estimate(x_np)
            fields_of = (lambda r=r, est=est: [f for f in est if r[f] != est[f]])
        row = {"config": name, "n": n, "k": k, "dist": dist if dist == "uniform" else "zipf(%s)" % s,
               "values": pal, "dtype": dt, "seed": seed, "ms": round(ms, 4), "ms_cold": round(ms_cold, 4),
               "gkeys_s": round(n / ms / 1e6, 2),
               "hbm_frac": round(16.0 * n / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4), "path": r["path"],
               "k_hat": r["k_hat"], "k_exact": r["k_exact"], "spill": r["spill_elems"],
               "ordered": ordered}
        pending.append((row, fields_of))
        print("%s n=%d k=%d %s: %.3f ms, %s" % (name, n, k, dist, ms, r["path"]), flush=True)
        del x, out, ws
        ctx._ws = None
        torch.cuda.empty_cache()
    for row, fields_of in pending:
        row["report_mismatch"] = fields_of()
        print(json.dumps(row), flush=True)
        rows.append(row)
    pool.shutdown()
    print("| config | N | K | freq | values | path | K^ | K | spill | ms | ms cold | Gkeys/s | % HBM | checked |")
    print("|---|---|---|---|---|---|---|---|---|---|---|---|---|---|")
    for r in rows:
        print("| %s | %d | %d | %s | %s %s | %s | %d | %d | %d | %.3f | %.3f | %.1f | %.1f | %s |" % (
            r["config"], r["n"], r["k"], r["dist"], r["values"], r["dtype"], r["path"], r["k_hat"], r["k_exact"],
            r["spill"], r["ms"], r["ms_cold"], r["gkeys_s"], 100 * r["hbm_frac"],
            "ok" if r["ordered"] and not r["report_mismatch"] else "MISMATCH %s" % r["report_mismatch"]))
    return rows


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="hbm_scale_column", choices=sorted(WORKLOADS))
    ap.add_argument("--radix-steps", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--serve-sustained-rate", type=float, default=7000.0,
                    help="second serving replay at this rate (req/s; 0: skip), one the GPU sustains")
    ap.add_argument("--serve-sustained-seconds", type=float, default=20.0)
    ap.add_argument("--no-structured", action="store_true",
                    help="skip the run-shaped, float64 and seeded-hash columns")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run one plain device copy of the input (counter calibration under a profiler)")
    ap.add_argument("--sweep", action="store_true",
                    help="run the dispatcher sweep (checked against the oracle) instead of the bench line")
    ap.add_argument("--serve-seconds", type=float, default=60.0,
                    help="length of the Poisson serving replay at 10^4 req/s (the configured workload); 0 skips "
                         "both serving replays")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        sys.stderr.write("bench.py runs on one GPU only: the library has no multi-GPU path "
                         "(a column would shard by an all-gather of the per-GPU (key, count) tables).  "
                         "Use --gpus 1.\n")
        sys.exit(2)

    if args.sweep:
        run_sweep()
        return

    import numpy as np
    import torch

    import gen
    import paper_2605_25040_amd as cafs

    n, k, dist, s, pal = WORKLOADS[args.workload]
    x_np = gen.column(n, k, dist=dist, s=s, palette=pal, dtype=np.int64)
    dev = torch.device("cuda", 0)
    x = torch.from_numpy(x_np).to(dev)
    ctx = cafs.Context(0)
    ws = ctx.workspace(ctx.workspace_bytes(n))
    out = torch.empty_like(x)
    rep = torch.zeros(cafs.report_size(), dtype=torch.uint8, device=dev)
    lib, h = ctx._lib, ctx._h

    def step():
        rc = lib.cafs_sort_i64(h, x.data_ptr(), out.data_ptr(), n, None, None, rep.data_ptr(), ws.data_ptr(),
                               ws.numel(), torch.cuda.current_stream(dev).cuda_stream)
        if rc != 0:
            raise RuntimeError("cafs_sort_i64 failed: %d" % rc)

    # one checked call (outside the timed region): the sorted output element by
    # element, the distinct keys and their counts, and every report field against
    # the oracle, whose three passes run in host threads meanwhile
    import concurrent.futures as cf

    import oracle
    pool = cf.ThreadPoolExecutor(max_workers=3)
    f_sort = pool.submit(oracle.sort, x_np, np.int64)
    f_counts = pool.submit(oracle.counts, x_np, np.int64)
    f_rep = pool.submit(oracle.report, x_np, np.int64)
    uq_chk = torch.empty_like(x)
    ct_chk = torch.empty_like(x)
    rc = lib.cafs_sort_i64(h, x.data_ptr(), out.data_ptr(), n, uq_chk.data_ptr(), ct_chk.data_ptr(), rep.data_ptr(),
                           ws.data_ptr(), ws.numel(), torch.cuda.current_stream(dev).cuda_stream)
    assert rc == 0, rc
    torch.cuda.synchronize()
    r = cafs.parse_report(rep)
    kx = r["k_exact"]
    got_out = out.cpu().numpy()
    got_uq = uq_chk[:kx].cpu().numpy()
    got_ct = ct_chk[:kx].cpu().numpy().view(np.uint64)
    del uq_chk, ct_chk
    assert np.array_equal(got_out, f_sort.result()), "sorted output differs from the oracle"
    want_uq, want_ct = f_counts.result()
    assert np.array_equal(got_uq, want_uq) and np.array_equal(got_ct, want_ct), "counts differ from the oracle"
    for f, v in f_rep.result().items():
        assert r[f] == v, ("report field", f, r[f], v)
    pool.shutdown()
    del got_out
    progress("checked call matches the oracle")

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # timed region: K steps, nothing else on the stream
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(args.steps):
        step()
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / args.steps
    value = n / (ms * 1e-3) / 1e9
    # per-step distribution: an event pair around each call
    pairs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
             for _ in range(args.steps)]
    for e0, e1 in pairs:
        e0.record()
        step()
        e1.record()
    torch.cuda.synchronize()
    per_step = [e0.elapsed_time(e1) for e0, e1 in pairs]
    # practical peak: a plain device copy of the column (2 x 8 B per key moved)
    cp = []
    for _ in range(3):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        gen.copy_device(out, x, torch.cuda.current_stream(dev).cuda_stream)
        e1.record()
        torch.cuda.synchronize()
        cp.append(e0.elapsed_time(e1))
    copy_gbs = 16.0 * n / (min(cp) * 1e-3) / 1e9
    # per-stage times (HIP events the library records on the stream the kernels run
    # on, at the stage boundaries) over the same number of steps, in a second loop so
    # that the events do not add to the timed region
    ctx.enable_timing(True)
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    ctx.enable_timing(False)
    stages, calls = ctx.stage_ms()
    stage_avg = {kk: v / max(calls, 1) for kk, v in stages.items()}

    if args.calibrate_copy:
        # a plain copy kernel of known size (n * 8 bytes read and written, 16-byte
        # accesses like the sort's kernels) for scaling hardware byte counters
        gen.copy_device(out, x, torch.cuda.current_stream(dev).cuda_stream)
        torch.cuda.synchronize()

    # dominant single-kernel stage and its roofline
    dom = max(STAGE_BYTES_PER_KEY, key=lambda st: stage_avg[st])
    dom_bytes = STAGE_BYTES_PER_KEY[dom] * n
    achieved = dom_bytes / (stage_avg[dom] * 1e-3) / 1e9
    traffic = measured_traffic(STAGE_KERNEL[dom], n)
    roofline = {"bound": "hbm", "kernel": STAGE_KERNEL[dom], "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic, "bytes_per_launch": dom_bytes, "launch_ms": round(stage_avg[dom], 4)}
    # both single-kernel stages, whichever is longer in this run
    per_kernel = {STAGE_KERNEL[st]: {"ms": round(stage_avg[st], 4),
                                     "gbs": round(STAGE_BYTES_PER_KEY[st] * n / (stage_avg[st] * 1e-3) / 1e9, 1)}
                  for st in STAGE_BYTES_PER_KEY}

    # the GPU radix baseline on the same input
    for _ in range(2):
        ctx.radix_sort(x, out=out, ws=ws)
    torch.cuda.synchronize()
    ev0.record()
    for _ in range(args.radix_steps):
        ctx.radix_sort(x, out=out, ws=ws)
    ev1.record()
    torch.cuda.synchronize()
    radix_ms = ev0.elapsed_time(ev1) / args.radix_steps
    radix_value = n / (radix_ms * 1e-3) / 1e9

    line = {
        "metric": "Gkeys/s int64 sort at K<<N (HBM-scale column), % HBM peak, vs GPU radix",
        "value": round(value, 3),
        "unit": "Gkeys/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64",
        "data": "synthetic",
        "config": {"workload": args.workload, "n": n, "k": k, "freq": "%s(%s)" % (dist, s) if dist == "zipf" else dist,
                   "values": "distinct random 64-bit" if pal == "random" else pal, "seed": "42+N+K",
                   "path": r["path"], "k_hat": r["k_hat"], "k_exact": r["k_exact"]},
        "hbm_frac_path": round(16.0 * n / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "step_ms": {"median": round(pct(per_step, 50), 4), "min": round(min(per_step), 4),
                    "p90": round(pct(per_step, 90), 4)},
        "copy_peak": {"gbs": round(copy_gbs, 1), "path_frac_of_copy": round(16.0 * n / (ms * 1e-3) / 1e9 / copy_gbs, 4)},
        "stages_ms": {kk: round(v, 4) for kk, v in stage_avg.items()},
        "radix_baseline": {"value": round(radix_value, 3), "unit": "Gkeys/s", "ms": round(radix_ms, 4)},
        "vs_radix": round(value / radix_value, 2),
        "roofline": roofline,
        "kernels": per_kernel,
    }
    del x, out, ws
    ctx._ws = None
    torch.cuda.empty_cache()
    progress("headline timed")
    if not args.no_structured:
        line["structured"] = bench_structured(ctx)
        line["variants"] = bench_variants(ctx)
        progress("structured columns and variants timed")
    if not args.no_batched:
        line["batched"] = bench_batched(ctx)
        progress("batched workload timed")
    if args.serve_seconds > 0:
        line["serving"] = bench_serving(args.serve_seconds)
        progress("serving replay at 10^4 req/s done")
        if args.serve_sustained_rate > 0:
            # the same request law at a rate the GPU sustains: request latency without
            # the queue that grows at 10^4 req/s
            line["serving_sustained"] = bench_serving(args.serve_sustained_seconds, rate=args.serve_sustained_rate,
                                                      fifo_seconds=0.5)
            progress("sustained serving replay done")
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(x_np, 20)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
