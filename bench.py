#!/usr/bin/env python3
"""Benchmark of the Benelux-pair search on one MI355X.

A step is one whole search: radicals sieved for every x of the workload, keys
generated, the hash-partitioned exact join over all passes, verification and the
sorted pair list.  The headline workload is the plain search up to N = 2^36, both
kinds.  Prints ONE JSON line (rank 0, N = 1 GPU).

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--log2n 36]
                  [--batched] [--served SECONDS] [--no-cpu]
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, 8 TB/s
VALU_PEAK_INT_OPS = 256 * 64 * 2.4e9  # 256 CUs x 64 lanes/clk x 2.4 GHz (32-bit integer lane-ops/s)
# Algorithmic 32-bit integer ops per sieved integer: 9 to reduce the factor 2 of a
# 64-bit x (add, count trailing zeros, shift), 1.6 for the odd prime-power divisions
# (0.273 per integer, 6 ops each), 0.9 for the per-segment first-multiple offsets,
# 6 for the member test, 2.7 to build the entries of the kept 10.7% (key, hash,
# packing) and 1.1 to rank them for the first partition.
SIEVE_OPS_PER_INT = 21.0
ENTRY_BYTES = 12
CALIB_BYTES = 4 << 30
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_plain_2p36.json")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2506_01099_amd", "csrc", f) for f in ("bx_kernels.h", "bx_device.h")]


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--log2n", type=int, default=36)
    ap.add_argument("--no-batched", action="store_true", help="skip the 4096-query batched workload")
    ap.add_argument("--served", type=float, default=60.0,
                    help="seconds of the served trace to replay (0 = skip; 60 = all 12,000 requests)")
    ap.add_argument("--tuning", default=os.path.join(ROOT, "paper_2506_01099_amd", "tuning_gfx950.json"),
                    help="autotuner result to load for the batched and served runs (if present)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-unpruned", action="store_true",
                    help="skip the comparison run with the member test off")
    ap.add_argument("--no-ablation", action="store_true",
                    help="skip the sort-join ablation run")
    ap.add_argument("--no-paper-schedule", action="store_true",
                    help="skip the paper's own designs at 2^32 (Algorithm 3's chunk schedule, Algorithm 2's whole-range sort)")
    ap.add_argument("--calib", action="store_true",
                    help="first copy 4 GiB with a plain copy kernel (reference for HBM counters)")
    ap.add_argument("--parse-counters", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="turn two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE) into " + TRAFFIC_FILE)
    ap.add_argument("--cpu-sample-log2", type=int, default=22)
    ap.add_argument("--only-served", type=float, default=0.0, metavar="SECONDS",
                    help="run only the served trace for SECONDS (no FIFO replay), for a kernel trace of that workload")
    ap.add_argument("--trace-overlap", metavar="TRACE_DIR",
                    help="device time during which kernels of two or more streams ran at once, from a "
                         "rocprofv3 --kernel-trace output directory")
    ap.add_argument("--autotune", action="store_true",
                    help="run the autotuner on the 4096-query batched workload and write its result to --tuning")
    ap.add_argument("--only-batched", action="store_true",
                    help="run only the 4096-query batched workload (--warmup + --steps launches of its graph), "
                         "for a kernel trace of that workload")
    return ap.parse_args()


def cpu_model():
    """The host CPU as /proc/cpuinfo names it: model name, family, model and stepping."""
    info = {}
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if ":" not in line:
                    if info:
                        break
                    continue
                k, v = (t.strip() for t in line.split(":", 1))
                if k in ("vendor_id", "model name", "cpu family", "model", "stepping", "cpu MHz") and k not in info:
                    info[k] = v
    except OSError:
        return None
    return (f"{info.get('model name', '?')} (vendor {info.get('vendor_id', '?')}, family {info.get('cpu family', '?')}, "
            f"model {info.get('model', '?')}, stepping {info.get('stepping', '?')}, {info.get('cpu MHz', '?')} MHz)")


def host_threads():
    """Threads for the oracle: the CPU share given to this process (OMP_NUM_THREADS when the
    environment sets it, as it does for one GPU's share of a shared host), else every core of
    the process's affinity mask."""
    aff = len(os.sched_getaffinity(0))
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit() and int(env) > 0:
        return min(aff, int(env)), aff
    return aff, aff


def cpu_baseline(N, log2_sample):
    import oracle

    S = 1 << log2_sample
    a = max(1, N - S)
    threads, host_cpus = host_threads()
    t0 = time.perf_counter()
    pairs, t_rad, t_join = oracle.search_range_timed(a, N + 1, 3, threads)
    dt = time.perf_counter() - t0
    return {"value": (N + 1 - a) / dt, "unit": "integers/s", "cores": threads, "kind": "oracle",
            "cpu_model": cpu_model(), "host_cpus_in_affinity": host_cpus,
            "os_cpu_count": os.cpu_count(), "omp_num_threads": os.environ.get("OMP_NUM_THREADS"),
            "sample": f"oracle.search_range over x in [{a}, {N + 1}) ({N + 1 - a} integers at magnitude 2^{int(math.log2(N))}); "
                      f"radicals {t_rad:.2f} s on {threads} threads, hash-map join {t_join:.2f} s on 1 thread",
            "seconds": dt}


def kernel_source_hash():
    import hashlib

    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def calib_copy():
    """A plain device-to-device copy of CALIB_BYTES (reference kernel for the counters)."""
    import torch

    src = torch.empty(CALIB_BYTES // 8, dtype=torch.int64, device="cuda")
    dst = torch.empty_like(src)
    src.fill_(1)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


def parse_counters(fetch_dir, write_dir):
    """Per-kernel HBM bytes per launch from FETCH_SIZE / WRITE_SIZE (KiB per dispatch), scaled
    by the factor that maps the calibration copy's counters onto its known bytes."""
    import csv
    import glob

    def load(d, counter):
        files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
        per = {}
        for f in files:
            for r in csv.DictReader(open(f)):
                if r.get("Counter_Name") != counter:
                    continue
                name = r["Kernel_Name"]
                per.setdefault(name, []).append(float(r["Counter_Value"]))
        return per

    fetch, write = load(fetch_dir, "FETCH_SIZE"), load(write_dir, "WRITE_SIZE")

    def pick(per, key):
        vals = [v for k, lst in per.items() if key in k for v in lst]
        return sum(vals) / len(vals) if vals else None

    copy_key = "copy"  # torch's elementwise copy kernel
    f_copy = max((max(l) for k, l in fetch.items() if copy_key in k.lower()), default=None)
    w_copy = max((max(l) for k, l in write.items() if copy_key in k.lower()), default=None)
    f_scale = CALIB_BYTES / (f_copy * 1024) if f_copy else None
    w_scale = CALIB_BYTES / (w_copy * 1024) if w_copy else None
    out = {"source_hash": kernel_source_hash(), "calib_bytes": CALIB_BYTES,
           "fetch_scale": f_scale, "write_scale": w_scale, "kernels": {}}
    for k, keys in (("sieve", ("k_sieve<",)), ("partition", ("k_partition<",)), ("join", ("k_join<", "k_join_c<"))):
        key = next((kk for kk in keys if any(kk in name for name in fetch)), keys[0])
        f, w = pick(fetch, key), pick(write, key)
        if f is None or w is None or not f_scale or not w_scale:
            continue
        out["kernels"][k] = {"fetch_bytes_per_launch": f * 1024 * f_scale,
                             "write_bytes_per_launch": w * 1024 * w_scale,
                             "launches": len([v for kk, l in fetch.items() if key in kk for v in l])}
    with open(TRAFFIC_FILE, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out))


def load_traffic():
    """Measured HBM bytes per launch with the launches per search they were taken over, or
    nothing when the kernels changed since the counters were taken."""
    if not os.path.exists(TRAFFIC_FILE):
        return {}
    t = json.load(open(TRAFFIC_FILE))
    if t.get("source_hash") != kernel_source_hash():
        return {}
    return {k: (v["fetch_bytes_per_launch"] + v["write_bytes_per_launch"], v["launches"])
            for k, v in t.get("kernels", {}).items()}


def traffic_of(traffic, kernel, launches, steps):
    """Counter bytes per launch, only if the counters saw as many launches per search as this run
    (a different plan moves different bytes per launch)."""
    tr = traffic.get(kernel)
    return tr[0] if tr and tr[1] * steps == launches else None


def run_plain(bx, N, steps, warmup, warm_s=None):
    for i in range(warmup):
        log(f"warmup {i + 1}/{warmup}: search N=2^{int(math.log2(N))}")
        t0 = time.perf_counter()
        bx.search(N)
        if warm_s is not None:
            st = bx.stats()
            warm_s.append({"seconds": time.perf_counter() - t0, "kernel_ms": st["kernel_ms"]})
    import torch

    torch.cuda.synchronize()
    per_step = []
    agg = None
    t0 = time.perf_counter()
    for i in range(steps):
        ts = time.perf_counter()
        pairs = bx.search(N)
        st = bx.stats()
        per_step.append(time.perf_counter() - ts)
        log(f"step {i + 1}/{steps}: {per_step[-1]:.3f} s, {len(pairs)} pairs, kernel ms {st['kernel_ms']}")
        if agg is None:
            agg = {k: dict(v) if isinstance(v, dict) else v for k, v in st.items()}
        else:
            for k in ("sieve", "partition", "join", "verify"):
                agg["kernel_ms"][k] += st["kernel_ms"][k]
                agg["launches"][k] += st["launches"][k]
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    return pairs, total, per_step, agg


def roofline_from(agg, n_ints_per_step, entries_per_step, steps, traffic):
    ms = agg["kernel_ms"]
    l2 = agg.get("l2_entry_bytes") or ENTRY_BYTES  # second-level entry: 12 B, or an 8 B compact word
    ln = agg["launches"]
    kinds = {k: ms[k] for k in ("sieve", "partition", "join")}
    dominant = max(kinds, key=kinds.get)
    out = {}
    # Sieve: ALU-bound.  Algorithmic ops per launch = ops per integer x integers per launch.
    if ln["sieve"]:
        avg_ms = ms["sieve"] / ln["sieve"]
        ints_per_launch = n_ints_per_step * steps / ln["sieve"]
        ach = SIEVE_OPS_PER_INT * ints_per_launch / (avg_ms * 1e-3) / 1e12
        out["sieve"] = {"bound": "alu", "achieved": ach, "peak": VALU_PEAK_INT_OPS / 1e12, "unit": "Tops/s",
                        "frac": ach / (VALU_PEAK_INT_OPS / 1e12), "traffic": traffic_of(traffic, "sieve", ln["sieve"], steps),
                        "avg_launch_ms": avg_ms, "integers_per_launch": ints_per_launch}
    # Partition: HBM-bound, a 12 B read and a 12 B (or 8 B compact) write per
    # entry (the entries the sieve wrote: the integers that pass the member test).
    if ln["partition"]:
        avg_ms = ms["partition"] / ln["partition"]
        b = (ENTRY_BYTES + l2) * entries_per_step * steps / ln["partition"]
        ach = b / (avg_ms * 1e-3) / 1e9
        out["partition"] = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                            "frac": ach / HBM_PEAK_GBS, "traffic": traffic_of(traffic, "partition", ln["partition"], steps),
                            "avg_launch_ms": avg_ms,
                            "bytes_per_launch": b}
    if ln["join"]:
        avg_ms = ms["join"] / ln["join"]
        b = l2 * entries_per_step * steps / ln["join"]
        ach = b / (avg_ms * 1e-3) / 1e9
        out["join"] = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": ach / HBM_PEAK_GBS, "traffic": traffic_of(traffic, "join", ln["join"], steps),
                       "avg_launch_ms": avg_ms,
                       "bytes_per_launch": b}
    # The join as a whole (second scatter + LDS join) against 24 B per key (the
    # sieve's 12 B entry read and its second-level copy written), whatever the
    # second-level format, over the join kernels' time.
    if ln["partition"] and ln["join"]:
        t = (ms["partition"] + ms["join"]) * 1e-3
        ach = 2 * ENTRY_BYTES * entries_per_step * steps / t / 1e9
        out["join_total"] = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                             "frac": ach / HBM_PEAK_GBS}
    return dominant, out


def main():
    args = parse()
    if args.parse_counters:
        parse_counters(*args.parse_counters)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU path (passes or range "
              "shares per GPU, one all-to-all of first-level buckets) is a design, not built", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2506_01099_amd import Benelux

    if args.trace_overlap:
        print(json.dumps(trace_overlap(args.trace_overlap)))
        return
    if args.autotune:
        from paper_2506_01099_amd import Benelux
        from paper_2506_01099_amd.inputs import batched_queries

        bx = Benelux(device=0)
        a, b = batched_queries()
        log(f"autotuning on {a.size} batched queries ...")
        bx.autotune(a, b, reps=2, path=args.tuning)
        bx.close()
        print(open(args.tuning).read().strip(), flush=True)
        return
    if args.only_batched:
        run_batched_only(args)
        return
    if args.only_served > 0:
        from paper_2506_01099_amd import Benelux

        bx = Benelux(device=0)
        if os.path.exists(args.tuning):
            bx.load_tuning(args.tuning)
        out = run_served(bx, args.only_served, fifo=False)
        bx.close()
        print(json.dumps(out), flush=True)
        return
    N = 1 << args.log2n
    if args.calib:
        calib_copy()
    # Cold start, outside the timed steps: the context builds its prime tables
    # (primes up to 2^21 and the prime powers up to 2^42) and uploads them once;
    # the HIP runtime is brought up first so that its start-up is not counted.
    torch.zeros(1, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    bx = Benelux(device=0)
    t_create = time.perf_counter() - t0
    warm_s = []
    pairs, total, per_step, agg = run_plain(bx, N, args.steps, args.warmup, warm_s)
    ms_step = total / args.steps * 1e3
    value = N / (total / args.steps)
    dominant, roof = roofline_from(agg, N, agg["entries"], args.steps,
                                   load_traffic() if args.log2n == 36 else {})
    line = {
        "metric": "integers sieved+joined/s at N=2^36 (both kinds), %HBM roofline; batched vs plain",
        "value": value,
        "unit": "integers/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic: the integers 1..N themselves (no dataset)",
        "config": {"workload": f"plain search N=2^{args.log2n}, both kinds, hash-partitioned passes",
                   "N": N, "member_test": True, "passes": agg["passes"], "b1_bits": agg["b1_bits"], "b2_bits": agg["b2_bits"],
                   "second_level_entry_bytes": agg.get("l2_entry_bytes"),
                   "seg_len": agg["seg_len"], "tile": agg["tile"], "parallelism": "single GPU"},
        "pairs_found": len(pairs),
        "roofline": dict(roof[dominant], kernel=dominant),
        "roofline_kernels": roof,
        "kernel_ms_per_step": {k: v / args.steps for k, v in agg["kernel_ms"].items()},
        "step_seconds": per_step,
        "entries_per_step": agg["entries"],
        "cold_start": {"context_create_s": t_create, "first_search_s": warm_s[0]["seconds"] if warm_s else None,
                       "first_search_kernel_ms": warm_s[0]["kernel_ms"] if warm_s else None},
    }
    if not args.no_unpruned:
        # The same search with every integer entered into the join (member test
        # off): the pair list is identical, the join moves ~3.5x more entries.
        log("same search without the member test ...")
        bx.set_option("prune", 0)
        try:
            p0, total0, per0, agg0 = run_plain(bx, N, 1, 1)
        finally:
            bx.set_option("prune", 1)
        if p0 != pairs:
            raise SystemExit("pair lists differ with and without the member test")
        line["without_member_test"] = {"integers_per_s": N / total0, "ms_per_step": total0 * 1e3,
                                       "passes": agg0["passes"], "entries_per_step": agg0["entries"],
                                       "kernel_ms_per_step": agg0["kernel_ms"]}
    if not args.no_ablation:
        # The same search with the sort join per partition instead of the LDS
        # hash join (Algorithm 2 per partition); the pair list must not change.
        log("same search with the sort join ...")
        bx.set_option("join", 1)
        try:
            p1, total1, per1, agg1 = run_plain(bx, N, 1, 1)
        finally:
            bx.set_option("join", 0)
        if p1 != pairs:
            raise SystemExit("pair lists differ between the hash join and the sort join")
        line["sort_join_ablation"] = {"integers_per_s": N / total1, "ms_per_step": total1 * 1e3,
                                      "join_ms": agg1["kernel_ms"]["join"],
                                      "hash_join_ms": line["kernel_ms_per_step"]["join"]}
    if not args.no_paper_schedule:
        # The paper's own design (Algorithm 3: chunks of 2^27 overlapping by one, a table of
        # 2^29 slots per chunk, every earlier chunk sieved again) on this GPU at 2^32, beside
        # the hash-partitioned passes on the same range; the pair lists must agree.
        log("paper schedule (Algorithm 3) at 2^32 ...")
        N32 = 1 << 32
        t0 = time.perf_counter()
        p_hash = bx.search(N32)
        t_hash = time.perf_counter() - t0
        bx.set_option("schedule", 1)
        try:
            t0 = time.perf_counter()
            p_a3 = bx.search(N32)
            t_a3 = time.perf_counter() - t0
            st_a3 = bx.stats()
        finally:
            bx.set_option("schedule", 0)
        if p_a3 != p_hash:
            raise SystemExit("pair lists differ between Algorithm 3's schedule and the hash-partitioned passes")
        line["paper_schedule_2p32"] = {"seconds": t_a3, "integers_per_s": N32 / t_a3, "chunks": st_a3["passes"],
                                       "chunk": 1 << 27, "table_slots": 1 << 29,
                                       "radicals_ms": st_a3["kernel_ms"]["radicals"],
                                       "insert_probe_ms": st_a3["kernel_ms"]["join"],
                                       "hash_partitioned_seconds": t_hash, "pairs": len(p_a3)}
        # Algorithm 2 (the whole range's list sorted once, runs of equal keys) on the same range.
        log("whole-range sort (Algorithm 2) at 2^32 ...")
        bx.set_option("schedule", 2)
        try:
            bx.search(N32)  # warm: allocates the list
            t0 = time.perf_counter()
            p_a2 = bx.search(N32)
            t_a2 = time.perf_counter() - t0
            st_a2 = bx.stats()
        finally:
            bx.set_option("schedule", 0)
        if p_a2 != p_hash:
            raise SystemExit("pair lists differ between Algorithm 2 and the hash-partitioned passes")
        line["whole_range_sort_2p32"] = {"seconds": t_a2, "integers_per_s": N32 / t_a2, "entries": st_a2["entries"],
                                         "sort_passes": st_a2["passes"],
                                         "radicals_ms": st_a2["kernel_ms"]["radicals"],
                                         "keys_ms": st_a2["kernel_ms"]["sieve"],
                                         "sort_ms": st_a2["kernel_ms"]["partition"],
                                         "runs_ms": st_a2["kernel_ms"]["join"],
                                         "hash_partitioned_seconds": t_hash, "pairs": len(p_a2)}
    if not args.no_batched or args.served > 0:
        if os.path.exists(args.tuning):
            bx.load_tuning(args.tuning)
            line["tuning"] = open(args.tuning).read().strip()
    if not args.no_batched:
        log("batched workload ...")
        line["batched"] = run_batched(bx)
    if args.served > 0:
        log(f"served trace ({args.served:.0f} s) ...")
        line["served"] = run_served(bx, args.served)
    if not args.no_cpu:
        log("cpu baseline (oracle) ...")
        line["cpu_baseline"] = cpu_baseline(N, args.cpu_sample_log2)
    bx.close()
    print(json.dumps(line), flush=True)


def run_batched(bx):
    import numpy as np

    from paper_2506_01099_amd.inputs import batched_queries

    a, b = batched_queries()
    total_L = int((b - a).sum())
    bx.search_batch(a, b)  # warm
    t0 = time.perf_counter()
    res = bx.search_batch(a, b)
    t_batch = time.perf_counter() - t0
    st = bx.stats()
    # plain single range of the same total length at offset 2^40
    lo = 1 << 40
    t0 = time.perf_counter()
    bx.search_range(lo, lo + total_L)
    t_plain = time.perf_counter() - t0
    # a sample of the queries one by one through the plain range path
    idx = np.arange(0, a.size, 16)
    t0 = time.perf_counter()
    for i in idx:
        bx.search_range(int(a[i]), int(b[i]))
    t_seq_sample = time.perf_counter() - t0
    L_sample = int((b[idx] - a[idx]).sum())
    return {"queries": int(a.size), "integers": total_L, "seconds": t_batch,
            "integers_per_s": total_L / t_batch, "pairs": int(sum(len(r) for r in res)),
            "plain_contiguous_integers_per_s": total_L / t_plain,
            "one_by_one_integers_per_s": L_sample / t_seq_sample, "one_by_one_sample_queries": int(idx.size),
            "kernel_ms": st["kernel_ms"], "passes": st["passes"]}


def run_batched_only(args):
    from paper_2506_01099_amd import Benelux
    from paper_2506_01099_amd.inputs import batched_queries

    bx = Benelux(device=0)
    if os.path.exists(args.tuning):
        bx.load_tuning(args.tuning)
    a, b = batched_queries()
    total_L = int((b - a).sum())
    for i in range(args.warmup):
        log(f"warmup {i + 1}/{args.warmup}: batch of {a.size} queries")
        bx.search_batch(a, b)
    times = []
    for i in range(args.steps):
        t0 = time.perf_counter()
        bx.search_batch(a, b)
        times.append(time.perf_counter() - t0)
        log(f"step {i + 1}/{args.steps}: {times[-1] * 1e3:.2f} ms")
    st = bx.stats()
    bx.close()
    print(json.dumps({"workload": f"batched: {a.size} range queries, {total_L} integers", "steps": args.steps,
                      "ms_per_batch": [t * 1e3 for t in times], "integers_per_s": total_L / min(times),
                      "graph_ms": st["graph_ms"], "passes": st["passes"]}), flush=True)


def trace_overlap(d):
    """From a kernel trace: the device time with at least one kernel running (busy)
    and the part of it with kernels of two or more streams running at once."""
    import csv
    import glob

    rows = []
    for f in glob.glob(os.path.join(d, "**", "*kernel_trace.csv"), recursive=True):
        for r in csv.DictReader(open(f)):
            stream = (r.get("Stream_Id"), r.get("Queue_Id"))
            rows.append((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), stream))
    # Sweep over start/end events: per stream the number of running kernels.
    ev = sorted([(t0, 1, st) for t0, t1, st in rows] + [(t1, -1, st) for t0, t1, st in rows],
                key=lambda e: (e[0], e[1]))
    running, busy, overlap, last = {}, 0, 0, None
    for t, delta, st in ev:
        if last is not None:
            active = sum(1 for v in running.values() if v > 0)
            if active >= 1:
                busy += t - last
            if active >= 2:
                overlap += t - last
        running[st] = running.get(st, 0) + delta
        last = t
    streams = sorted({str(st) for _, _, st in rows})
    return {"kernels": len(rows), "streams": streams, "busy_ms": busy / 1e6, "overlap_ms": overlap / 1e6,
            "overlap_frac_of_busy": overlap / busy if busy else None}


def run_served(bx, seconds, fifo=True, budget_bytes=200 << 30, max_inflight=2):
    """Replays the served trace (its first `seconds`, or all of it) through the serving
    calls.  A submitter thread submits each request at its arrival time; latency is the
    library's completion time minus the arrival time, and the submit lag (the library's
    submit time minus the arrival time) is reported beside it."""
    import threading

    import numpy as np

    from paper_2506_01099_amd import Server
    from paper_2506_01099_amd.inputs import served_trace

    t, a, b = served_trace(n=12000)
    keep = t < seconds
    t, a, b = t[keep], a[keep], b[keep]
    srv = Server(bx, budget_bytes=budget_bytes, max_inflight=max_inflight)
    tickets = [None] * t.size
    submitted = threading.Semaphore(0)
    t_start = srv.now() + 0.05

    def submitter():
        for i in range(t.size):
            while True:
                wait = t_start + t[i] - srv.now()
                if wait <= 0:
                    break
                time.sleep(wait if wait < 0.002 else wait - 0.001)
            tickets[i] = srv.submit(int(a[i]), int(b[i]))
            submitted.release()

    th = threading.Thread(target=submitter, daemon=True)
    th.start()
    lat, lag, svc, n_pairs = [], [], [], 0
    pending = []
    n_sub = 0
    while len(lat) < t.size:
        while submitted.acquire(blocking=False):
            pending.append(n_sub)
            n_sub += 1
        still = []
        for i in pending:
            if srv.poll(tickets[i]):
                pairs, ts, td = srv.take(tickets[i])
                arr = t_start + t[i]
                lat.append(td - arr)
                lag.append(ts - arr)
                svc.append(td - ts)
                n_pairs += len(pairs)
            else:
                still.append(i)
        pending = still
        time.sleep(0.0002)
    th.join()
    t_end = srv.now()
    info = srv.info()
    srv.stop()
    lat, lag, svc = np.array(lat), np.array(lag), np.array(svc)
    total_L = int((b - a).sum())
    pc = lambda v, q: float(np.percentile(v, q) * 1e3)
    out = {"requests": int(t.size), "integers": total_L, "wall_s": t_end - t_start,
           "integers_per_s": total_L / (t_end - t_start), "p50_ms": pc(lat, 50), "p99_ms": pc(lat, 99),
           "submit_lag_p50_ms": pc(lag, 50), "submit_lag_p99_ms": pc(lag, 99),
           "service_p50_ms": pc(svc, 50), "service_p99_ms": pc(svc, 99), "pairs": n_pairs,
           "budget_bytes": budget_bytes, "lanes": max_inflight, "admission": info}
    if fifo:
        out["fifo_plain"] = run_fifo(bx, t, a, b)
    return out


def run_fifo(bx, t, a, b):
    """The same trace on the plain range path, FIFO, one request at a time: each
    search starts at its arrival or when the previous one ends, whichever is later.
    Per-kernel event timing is off, as on the serving lanes."""
    import numpy as np

    lat = []
    n_pairs = 0
    bx.set_option("timing", 0)
    try:
        t_start = time.perf_counter()
        for i in range(t.size):
            wait = t_start + t[i] - time.perf_counter()
            if wait > 0:
                time.sleep(wait)
            n_pairs += len(bx.search_range(int(a[i]), int(b[i])))
            lat.append(time.perf_counter() - (t_start + t[i]))
        wall = time.perf_counter() - t_start
    finally:
        bx.set_option("timing", 1)
    lat = np.array(lat)
    return {"requests": int(t.size), "wall_s": wall, "integers_per_s": int((b - a).sum()) / wall,
            "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "pairs": n_pairs}


if __name__ == "__main__":
    main()
