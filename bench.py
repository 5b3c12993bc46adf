#!/usr/bin/env python3
"""On-device parse throughput of the single-pass GPU parser on one MI355X.

Workload: a 1 GiB synthetic numeric CSV (whole records up to 2^30 bytes,
~8.3M records x 18 columns, ~130 B per record: 4 integer ids, 2 timestamps,
8 two-decimal floats, 4 short strings), parsed with the 4-state quote-aware
CSV DFA into record offsets, field offsets, column ids and 18 typed columns.
The input is resident in HBM before timing starts; outputs and workspace are
preallocated. One step = one pp_parse call (all stages of the path).

Prints one JSON line. ``value`` is the parse rate in GB/s of input (10^9 B/s,
the paper's unit); ``roofline`` prices the dominant kernel's input+output
bytes against the 8 TB/s HBM peak; ``copy_kernel_gbs`` is the library's own
16-byte streaming copy over as many bytes (the practical ceiling);
``cpu_baseline`` is the sequential oracle on the host, timed on the same
buffer. ``--workload`` selects the other configurations (c1 latency, c3 text-
heavy CSV, c4 batched, c5 serving).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


KERNEL_SOURCES = ["paper_1905_13415_amd/csrc/tile.h", "paper_1905_13415_amd/csrc/parse.hip",
                  "paper_1905_13415_amd/csrc/convert.h", "paper_1905_13415_amd/csrc/convert_fast.h"]
# HBM byte counters of the dominant kernel per plain workload, from committed
# rocprofv3 counter runs (not measured in this process)
TRAFFIC_FILES = {"c2": "profiles/parse_tiles_c2_1GiB_traffic.json",
                 "c3": "profiles/parse_tiles_c3_2GiB_traffic.json",
                 "utf16": "profiles/parse_tiles_utf16_2GiB_traffic.json"}
METRIC = "on-device parse GB/s & % of HBM roofline; batched/serving vs plain; p50/p99 latency"


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload):
    """HBM bytes per launch of the dominant kernel from the committed
    counter runs (FETCH_SIZE, WRITE_SIZE, each scaled by a plain copy's
    reading), or None when the kernel sources changed since they were taken."""
    path = TRAFFIC_FILES.get(workload)
    if not path:
        return None
    try:
        with open(os.path.join(ROOT, path)) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("source_sha256") != kernel_source_hash():
        return None
    return t["fetch_bytes"] + t["write_bytes"]


def host_cpu():
    """CPU model and the number of cores visible to this process."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    return {"cpu_model": model, "nproc": avail, "cpu_count": os.cpu_count()}


def output_bytes(R, F, types):
    """Algorithmic output bytes: what the method must write."""
    b = (R + 1) * 8 + (F + 1) * 8 + F * 4
    for ty in types:
        if ty == 5:  # SKIP
            continue
        b += R * 9  # value + valid byte
        if ty == 4:  # STRING: span end
            b += R * 8
    return b


def copy_ceiling_gbs(nbytes, dev, stream):
    """Read+write GB/s of the library's 16-byte streaming copy kernel over
    nbytes (half read, half written): the practical HBM ceiling."""
    import torch

    import paper_1905_13415_amd as pp
    half = max(nbytes // 2 // 256 * 256, 1 << 20)
    src = torch.empty(half, dtype=torch.uint8, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3):
        pp.copy(dst, src, stream=stream)
    c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    c0.record(stream)
    for _ in range(10):
        pp.copy(dst, src, stream=stream)
    c1.record(stream)
    torch.cuda.synchronize()
    gbs = 2 * half * 10 / (c0.elapsed_time(c1) / 1e3) / 1e9
    del src, dst
    return gbs


PLAIN = {
    "c2": {"nbytes": 1 << 30, "schema": "SCHEMA_C2",
           "data": "synthetic (seeded numeric CSV shaped like the NYC taxi trips; no dataset used)",
           "workload": "c2: 1 GiB numeric CSV, 18 columns (4 int64, 2 timestamp, 8 float64, 4 string), "
                       "~130 B/record, csv4 DFA, plain single-buffer launch"},
    "c3": {"nbytes": 1 << 31, "schema": "SCHEMA_C3",
           "data": "synthetic (seeded text-heavy CSV shaped like the yelp reviews; no dataset used)",
           "workload": "c3: 2 GiB text-heavy CSV, 9 columns (3 id strings, 3 int64, 1 date, 2 quoted free-text "
                       "strings with embedded delimiters, LF and doubled quotes), ~700 B/record, csv4 DFA, "
                       "plain single-buffer launch"},
}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--nbytes", type=int, default=0, help="input size of c2/c3 (0: the workload's own)")
    ap.add_argument("--bytes-per-thread", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile-steps", type=int, default=0,
                    help="only run this many launches (for rocprofv3), no JSON")
    ap.add_argument("--workload", choices=["c1", "c2", "c3", "c4", "c5", "stream", "utf16"], default="c2",
                    help="c1: 10,000-record RFC-4180 CSV, latency of one plain launch; "
                         "c2: 1 GiB numeric CSV, plain launch (default); "
                         "c3: 2 GiB text-heavy quoted CSV, plain launch; "
                         "c4: 4,096 mixed-dialect buffers, batched launch against plain launches; "
                         "c5: request loop over pinned host inputs, p50/p99 latency; "
                         "stream: the 2 GiB text-heavy CSV end to end from pinned host memory in partitions; "
                         "utf16: the 1 GiB numeric CSV as UTF-16LE text (2 GiB), pp_parse_utf16")
    ap.add_argument("--stream-partition", type=int, default=256 << 20, help="stream: partition bytes")
    ap.add_argument("--c5-requests", type=int, default=2000)
    ap.add_argument("--c5-pool-bytes", type=int, default=1 << 30,
                    help="size of the pinned log text that c5 requests are cut from")
    ap.add_argument("--c5-budget", type=int, default=32 << 30, help="server device budget, bytes")
    ap.add_argument("--c5-copy-streams", type=int, default=4, help="server host-to-device copy streams")
    ap.add_argument("--c4-max-bytes", type=int, default=64 << 20,
                    help="upper bound of the c4 buffer sizes (8 MiB gives the ~4 GB variant)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: measures one GPU; --gpus {args.gpus} is not supported "
              f"(across GPUs the parse would shard by byte range with one small all-gather)",
              file=sys.stderr)
        sys.exit(2)
    if args.workload == "c1":
        return bench_c1(args)
    if args.workload == "c4":
        return bench_c4(args)
    if args.workload == "c5":
        return bench_c5(args)
    if args.workload == "stream":
        return bench_stream(args)
    if args.workload == "utf16":
        return bench_utf16(args)
    return bench_plain(args)


def bench_plain(args):
    """One plain launch over a resident buffer (c2 or c3); one step = one
    pp_parse call, every stage of the path."""
    import torch

    import datagen
    import paper_1905_13415_amd as pp
    from datagen import dialects as D

    wl = PLAIN[args.workload]
    nbytes = args.nbytes or wl["nbytes"]
    t0 = time.time()
    g = datagen.c2(nbytes=nbytes) if args.workload == "c2" else datagen.c3(nbytes=nbytes)
    types = getattr(D, wl["schema"]).types
    dfa = D.csv4()
    n = len(g.data)
    R = g.nrecords
    F = g.nrecords * g.ncols
    print(f"[bench] generated {n} bytes, {R} records in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)

    dev = torch.device("cuda:0")
    d_in = torch.from_numpy(g.data).to(dev)
    opts = pp.options(args.bytes_per_thread, 0) if args.bytes_per_thread else None
    out = pp.alloc_outputs(types, R, F, device=dev)
    ws = torch.empty(pp.workspace_size(n, opts), dtype=torch.uint8, device=dev)
    call = pp.Call(d_in, n, dfa, types, out, ws, opts)
    stream = torch.cuda.current_stream()

    if args.profile_steps:
        for _ in range(args.profile_steps):
            call.launch(stream)
        torch.cuda.synchronize()
        # reference for the HBM byte counters: one streaming copy of exactly 2^30 bytes
        src = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        pp.copy(dst, src, stream=stream)
        torch.cuda.synchronize()
        print("[bench] profile launches done (plus one 1 GiB streaming copy)", file=sys.stderr, flush=True)
        return

    for _ in range(args.warmup):
        call.launch(stream)
    torch.cuda.synchronize()
    res = out.result_dict()
    if res["status"] != pp.RESULT_OK or res["num_records"] != R or res["num_fields"] != F:
        print(f"[bench] unexpected result {res}", file=sys.stderr)
        sys.exit(1)

    # timed region: K launches bracketed by synchronisation, HIP events on the
    # launch stream around every call (a call is the init kernel, a few
    # microseconds, and the parse kernel)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    for a, b in evs:
        a.record(stream)
        call.launch(stream)
        b.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    per = sorted(a.elapsed_time(b) for a, b in evs)  # ms
    ms_mean = sum(per) / len(per)
    ms_med = per[len(per) // 2]

    outb = output_bytes(R, F, types)
    total_b = n + outb
    copy_gbs = copy_ceiling_gbs(total_b, dev, stream)

    in_gbs = n / (ms_mean / 1e3) / 1e9
    inout_gbs = total_b / (ms_mean / 1e3) / 1e9
    default_size = nbytes == wl["nbytes"] and not args.bytes_per_thread
    line = {
        "metric": METRIC,
        "value": round(in_gbs, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall * 1e3 / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": wl["data"],
        "config": {
            "workload": wl["workload"],
            "bytes": n, "records": R, "fields": F,
            "bytes_per_thread": args.bytes_per_thread or 64, "block_threads": 512 if not args.bytes_per_thread else 256,
        },
        "kernel_ms": {"mean": round(ms_mean, 4), "median": round(ms_med, 4), "min": round(per[0], 4),
                      "max": round(per[-1], 4), "p10": round(per[len(per) // 10], 4),
                      "p90": round(per[min(len(per) - 1, (9 * len(per)) // 10)], 4)},
        "input_gbs": round(in_gbs, 2),
        "in_out_gbs": round(inout_gbs, 2),
        "output_bytes": outb,
        "copy_kernel_gbs": round(copy_gbs, 1),
        "frac_of_copy_kernel": round(inout_gbs / copy_gbs, 4),
        "roofline": {
            "bound": "hbm",
            "achieved": round(inout_gbs, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(inout_gbs / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic(args.workload) if default_size else None,
            "timing": "HIP events on the launch stream around each call, mean over the timed steps",
            "traffic_source": TRAFFIC_FILES.get(args.workload) if default_size else None,
        },
    }
    tr = line["roofline"]["traffic"]
    # the measured bytes at this run's time: what the HBM actually moved
    line["roofline"]["traffic_frac"] = round(tr / (ms_mean / 1e3) / 1e9 / HBM_PEAK_GBS, 4) if tr else None

    if not args.no_cpu_baseline:
        import oracle
        t = time.perf_counter()
        ref = oracle.parse(g.data, dfa, types, cap_records=R, cap_fields=F)
        cpu_s = time.perf_counter() - t
        assert ref.num_records == R
        line["cpu_baseline"] = dict({"value": round(n / cpu_s / 1e9, 4), "unit": "GB/s", "cores": 1,
                                     "kind": "oracle",
                                     "sample": f"the whole {n}-byte workload, one sequential oracle parse "
                                               f"({cpu_s:.1f} s, outputs preallocated)"}, **host_cpu())
    print(json.dumps(line), flush=True)


def bench_c1(args):
    """Latency of one plain launch on the small quoted workload (10,000
    records x 8 columns, ~1.34 MB, 20% of strings quoted with embedded
    delimiters, newlines and doubled quotes): a handful of tiles, so the time
    is one tile's pipeline plus launch overhead, not bandwidth."""
    import torch

    import datagen
    import paper_1905_13415_amd as pp
    from datagen import dialects as D

    g = datagen.c1()
    types = list(D.SCHEMA_C1.types)
    dfa = D.csv4()
    n = len(g.data)
    R, F = g.nrecords, g.nrecords * g.ncols
    dev = torch.device("cuda:0")
    d_in = torch.from_numpy(g.data).to(dev)
    out = pp.alloc_outputs(types, R, F, device=dev)
    # launch shape from the autotuner: the input is a few dozen default
    # tiles, so smaller tiles can spread it over more of the chip
    best, tune = pp.autotune_parse(d_in, dfa, types, out, reps=10)
    ws = torch.empty(pp.workspace_size(n, best), dtype=torch.uint8, device=dev)
    call = pp.Call(d_in, n, dfa, types, out, ws, opts=best)
    stream = torch.cuda.current_stream()
    steps = max(args.steps, 50)
    for _ in range(max(args.warmup, 5)):
        call.launch(stream)
    torch.cuda.synchronize()
    res = out.result_dict()
    if res["status"] != pp.RESULT_OK or res["num_records"] != R or res["num_fields"] != F:
        print(f"[bench] unexpected result {res}", file=sys.stderr)
        sys.exit(1)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    for a, b in evs:
        a.record(stream)
        call.launch(stream)
        b.record(stream)
        b.synchronize()  # one call at a time: latency, not throughput
    wall = time.perf_counter() - wall0
    per = sorted(a.elapsed_time(b) * 1e3 for a, b in evs)  # us
    med = per[len(per) // 2]
    outb = output_bytes(R, F, types)
    line = {
        "metric": METRIC,
        "value": round(n / (med / 1e6) / 1e9, 3),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": max(args.warmup, 5),
        "ms_per_step": round(wall * 1e3 / steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic (seeded RFC-4180-style CSV; no dataset used)",
        "config": {"workload": "c1: 10,000 records x 8 columns (2 int64, 2 float64, 1 timestamp, 3 strings, "
                               "20% quoted with embedded commas, LF and doubled quotes), csv4 DFA, one plain launch",
                   "bytes": n, "records": R, "fields": F,
                   "block_threads": best.block_threads, "bytes_per_thread": best.bytes_per_thread},
        "autotune_us_per_shape": {f"{o.block_threads}x{o.bytes_per_thread}": round(m * 1e3, 2)
                                  for o, m in zip(pp.shapes(), tune["ms"]) if m >= 0},
        "latency_us": {"p50": round(med, 2), "p10": round(per[len(per) // 10], 2),
                       "p90": round(per[(9 * len(per)) // 10], 2), "min": round(per[0], 2)},
        "in_out_gbs": round((n + outb) / (med / 1e6) / 1e9, 2),
        "output_bytes": outb,
        "roofline": {"bound": "hbm", "achieved": round((n + outb) / (med / 1e6) / 1e9, 2), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round((n + outb) / (med / 1e6) / 1e9 / HBM_PEAK_GBS, 5),
                     "traffic": None},
    }
    if not args.no_cpu_baseline:
        import oracle
        reps = 20
        t = time.perf_counter()
        for _ in range(reps):
            oracle.parse(g.data, dfa, types, cap_records=R, cap_fields=F)
        cpu_s = (time.perf_counter() - t) / reps
        line["cpu_baseline"] = dict({"value": round(n / cpu_s / 1e9, 4), "unit": "GB/s", "cores": 1,
                                     "kind": "oracle",
                                     "sample": f"the whole {n}-byte workload, {reps} sequential oracle parses "
                                               f"({cpu_s * 1e3:.2f} ms each)"}, **host_cpu())
    print(json.dumps(line), flush=True)


def bench_c4(args):
    """4,096 independent buffers (sizes log-uniform from 1 KiB to 64 MiB, 18
    dialects: 3- to 8-state DFAs x comma/tab/pipe) parsed by one captured
    batched launch, against the same buffers parsed by one pp_parse call
    each, serialised on one stream. One step = the whole batch."""
    import numpy as np
    import torch

    import datagen
    import paper_1905_13415_amd as pp
    from datagen import dialects as D

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    dfas = datagen.c4_dialects()
    plan = datagen.c4_plan(hi=args.c4_max_bytes)
    t0 = time.time()
    gens = [datagen.c4_buffer(spec) for spec in plan]
    sizes = [len(g.data) for g in gens]
    total = sum(sizes)
    print(f"[bench] generated {len(gens)} buffers, {total} bytes in {time.time() - t0:.1f}s",
          file=sys.stderr, flush=True)

    # one device arena for the inputs, each buffer 256-byte aligned
    offs, off = [], 0
    for n in sizes:
        offs.append(off)
        off += (n + 255) // 256 * 256
    arena = torch.empty(max(off, 1), dtype=torch.uint8, device=dev)
    for g, o in zip(gens, offs):
        if len(g.data):
            arena[o:o + len(g.data)].copy_(torch.from_numpy(g.data))
    items, calls, expect, outb = [], [], [], 0
    ws = torch.empty(max(pp.workspace_size(max(sizes), None), 1), dtype=torch.uint8, device=dev)
    for spec, g, o in zip(plan, gens, offs):
        types = list(D.SCHEMA_LOG12.types if spec.kind == datagen.K_LOG else D.SCHEMA_C1.types)
        R, F = g.nrecords, g.nrecords * g.ncols
        d_in = arena[o:o + len(g.data)]
        out = pp.alloc_outputs(types, R, F, device=dev)
        items.append((d_in, spec.dialect, types, out))
        calls.append(pp.Call(d_in, len(g.data), dfas[spec.dialect], types, out, ws))
        expect.append((R, F))
        outb += output_bytes(R, F, types)
    torch.cuda.synchronize()
    print(f"[bench] inputs resident, outputs allocated ({outb} output bytes)", file=sys.stderr, flush=True)

    def check(tag):
        res = torch.stack([it[3].result for it in items]).cpu().numpy()
        for i, (R, F) in enumerate(expect):
            if res[i, 0] != pp.RESULT_OK or res[i, 1] != R or res[i, 2] != F:
                print(f"[bench] {tag}: buffer {i} unexpected result {res[i].tolist()}", file=sys.stderr)
                sys.exit(1)

    # launch shape (bytes per thread, block threads) from the autotuner
    t0 = time.time()
    best, tune = pp.autotune_batch(dfas, items, reps=2)
    print(f"[bench] autotuned shape {best.block_threads}x{best.bytes_per_thread} in {time.time() - t0:.1f}s "
          f"({tune['ms']} ms per shape)", file=sys.stderr, flush=True)
    batch = pp.Batch(dfas, items, opts=best)
    batch.capture()
    if args.profile_steps:
        for _ in range(args.profile_steps):
            batch.replay(stream)
        for c in calls:
            c.launch(stream)
        torch.cuda.synchronize()
        check("profile")
        print("[bench] profile replays and plain launches done", file=sys.stderr, flush=True)
        return

    def timed(fn, steps):
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(steps)]
        host = []
        torch.cuda.synchronize()
        for a, b in evs:
            h0 = time.perf_counter()
            a.record(stream)
            fn()
            b.record(stream)
            host.append(time.perf_counter() - h0)
        torch.cuda.synchronize()
        per = sorted(a.elapsed_time(b) for a, b in evs)
        return per, sum(host) / len(host) * 1e3

    for _ in range(args.warmup):
        batch.replay(stream)
    torch.cuda.synchronize()
    check("batched")
    # keep every 64th buffer's batched outputs to compare with the plain launches
    sample = list(range(0, len(items), 64))
    kept = {i: (items[i][3].field_offsets.clone(), [v.clone() for v in items[i][3].values if v is not None])
            for i in sample}
    wall0 = time.perf_counter()
    b_per, b_host = timed(lambda: batch.replay(stream), args.steps)
    wall = time.perf_counter() - wall0

    def plain_pass():
        for c in calls:
            c.launch(stream)

    plain_pass()
    torch.cuda.synchronize()
    check("plain")
    for i in sample:
        fo, vals = kept[i]
        same = torch.equal(fo, items[i][3].field_offsets) and all(
            torch.equal(a.view(torch.int64), b.view(torch.int64))
            for a, b in zip(vals, [v for v in items[i][3].values if v is not None]))
        if not same:
            print(f"[bench] buffer {i}: batched and plain outputs differ", file=sys.stderr)
            sys.exit(1)
    p_steps = max(3, min(args.steps, 10))
    p_per, p_host = timed(plain_pass, p_steps)
    # the plain launches without the host's pace: queue them all behind a
    # spin kernel longer than their enqueue, time from the end of the spin
    c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    c0.record(stream)
    torch.cuda._sleep(1_000_000)
    c1.record(stream)
    torch.cuda.synchronize()
    ticks_per_ms = 1_000_000 / c0.elapsed_time(c1)
    torch.cuda._sleep(int(ticks_per_ms * (1.5 * p_host + 50)))
    c0.record(stream)
    h0 = time.perf_counter()
    plain_pass()
    enq_ms = (time.perf_counter() - h0) * 1e3
    c1.record(stream)
    torch.cuda.synchronize()
    p_queued = c0.elapsed_time(c1)

    b_ms = sum(b_per) / len(b_per)
    p_ms = sum(p_per) / len(p_per)
    in_gbs = total / (b_ms / 1e3) / 1e9
    inout_gbs = (total + outb) / (b_ms / 1e3) / 1e9
    line = {
        "metric": METRIC,
        "value": round(in_gbs, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall * 1e3 / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic (seeded mixed-type records in 18 dialects; no dataset used)",
        "config": {
            "workload": f"c4: {len(items)} buffers, sizes log-uniform in [1 KiB, {args.c4_max_bytes >> 20} MiB], "
                        "18 dialects (3- to 8-state DFAs x comma/tab/pipe), one captured batched launch",
            "bytes": total, "buffers": len(items), "work_items": batch.num_tiles,
            "block_threads": best.block_threads, "bytes_per_thread": best.bytes_per_thread,
        },
        "autotune_ms_per_shape": {f"{o.block_threads}x{o.bytes_per_thread}": m
                                  for o, m in zip(pp.shapes(), tune["ms"])},
        "batched_ms": {"mean": round(b_ms, 4), "median": round(b_per[len(b_per) // 2], 4),
                       "min": round(b_per[0], 4), "max": round(b_per[-1], 4), "host_enqueue_ms": round(b_host, 4)},
        "plain_ms": {"mean": round(p_ms, 4), "median": round(p_per[len(p_per) // 2], 4),
                     "min": round(p_per[0], 4), "max": round(p_per[-1], 4), "host_enqueue_ms": round(p_host, 4),
                     "launches": 2 * len(calls),
                     "prequeued_ms": round(p_queued, 4), "prequeued_enqueue_ms": round(enq_ms, 4)},
        "plain_gbs": round(total / (p_ms / 1e3) / 1e9, 2),
        "batched_speedup_vs_plain": round(p_ms / b_ms, 3),
        "batched_speedup_vs_prequeued_plain": round(p_queued / b_ms, 3),
        "input_gbs": round(in_gbs, 2),
        "in_out_gbs": round(inout_gbs, 2),
        "output_bytes": outb,
        "roofline": {
            "bound": "hbm",
            "achieved": round(inout_gbs, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(inout_gbs / HBM_PEAK_GBS, 4),
            "traffic": None,
        },
    }
    if not args.no_cpu_baseline:
        import oracle
        from concurrent.futures import ThreadPoolExecutor
        # bounded sample: buffers in plan order until ~2 GB
        pick, acc = [], 0
        for i in range(len(gens)):
            if acc >= 2_000_000_000:
                break
            pick.append(i)
            acc += sizes[i]

        def one(i):
            return oracle.parse(gens[i].data, dfas[plan[i].dialect], items[i][2],
                                cap_records=expect[i][0], cap_fields=expect[i][1])

        t = time.perf_counter()
        for i in pick:
            one(i)
        cpu1 = time.perf_counter() - t
        # a pool over every core this process may use, at most 16 (a one-GPU
        # share of the host)
        cores = min(16, host_cpu()["nproc"])
        t = time.perf_counter()
        with ThreadPoolExecutor(cores) as ex:
            list(ex.map(one, pick))
        cpun = time.perf_counter() - t
        line["cpu_baseline"] = dict({"value": round(acc / cpu1 / 1e9, 4), "unit": "GB/s", "cores": 1,
                                     "kind": "oracle",
                                     "sample": f"the first {len(pick)} buffers of the batch ({acc} bytes), "
                                               f"sequential oracle, one thread ({cpu1:.1f} s)",
                                     "pool": {"value": round(acc / cpun / 1e9, 4), "cores": cores,
                                              "note": "same sample, one buffer per task"}}, **host_cpu())
    batch.close()
    print(json.dumps(line), flush=True)


def bench_c5(args):
    """Serving: requests cut at record boundaries from a pinned extended-log
    text (6-state DFA, 12 columns), sizes log-uniform in [4 KiB, 256 MiB],
    Poisson arrivals at offered loads of 0.5, 0.8 and 1.0 times the serial
    capacity, served by the request loop (continuous batching, copies
    overlapped with parsing) and, on the same trace, by the loop restricted to
    one request at a time (copy, then parse, no overlap). Latency is arrival
    to the end of the request's parse on the device."""
    import numpy as np
    import torch

    import datagen
    import paper_1905_13415_amd as pp
    from datagen import dialects as D

    dfa = D.log6()
    types = list(D.SCHEMA_LOG12.types)
    t0 = time.time()
    g = datagen.log(datagen.SEED_BASE + 4, args.c5_pool_bytes)
    data = g.data
    ends = np.flatnonzero(data == 10) + 1  # no LF inside a log record: every LF ends one
    starts = np.concatenate([[0], ends[:-1]])
    pool = torch.empty(len(data), dtype=torch.uint8).pin_memory()
    pool.numpy()[:] = data
    rng = np.random.default_rng(datagen.SEED_BASE + 4)
    N = args.c5_requests
    sizes = np.exp(rng.uniform(np.log(4096), np.log(256 << 20), size=N)).astype(np.int64)
    reqs = []
    for sz in sizes:
        last_ok = int(np.searchsorted(starts, len(data) - sz, side="right")) - 1
        i = int(rng.integers(0, max(last_ok, 0) + 1))
        j = int(np.searchsorted(ends, starts[i] + sz, side="left"))
        j = min(j, len(ends) - 1)
        a, b = int(starts[i]), int(ends[j])
        reqs.append((pool[a:b], j - i + 1))
    total = sum(int(r[0].numel()) for r in reqs)
    print(f"[bench] pool {len(data)} bytes, {N} requests, {total} bytes in {time.time() - t0:.1f}s",
          file=sys.stderr, flush=True)

    # pinned host -> device copy rate, the bound of this form
    dev = torch.device("cuda:0")
    dst = torch.empty(256 << 20, dtype=torch.uint8, device=dev)
    dst.copy_(pool[:256 << 20], non_blocking=True)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(4):
        dst.copy_(pool[:256 << 20], non_blocking=True)
    e1.record()
    torch.cuda.synchronize()
    h2d_gbs = 4 * (256 << 20) / (e0.elapsed_time(e1) / 1e3) / 1e9
    del dst

    def run(arrivals_ns, serial):
        if serial:
            srv = pp.Server([dfa], args.c5_budget, max_slots=1, copy_streams=1, compute_streams=1)
        else:
            srv = pp.Server([dfa], args.c5_budget, max_slots=256, copy_streams=args.c5_copy_streams,
                            compute_streams=2)
        lat, first, last = [], None, 0
        i = done = 0
        base = time.monotonic_ns() + 2_000_000
        while done < N:
            now = time.monotonic_ns()
            while i < N and base + arrivals_ns[i] <= now:
                t, R = reqs[i]
                srv.submit(t, 0, types, R, 12 * R)
                i += 1
            for c in srv.poll():
                if c.result["status"] != pp.RESULT_OK:
                    print(f"[bench] request {c.id}: {c.result}", file=sys.stderr)
                    sys.exit(1)
                lat.append(c.latency_ns)
                first = c.t_arrival_ns if first is None else min(first, c.t_arrival_ns)
                last = max(last, c.t_parse_done_ns)
                srv.release(c.id)
                done += 1
            if i >= N:
                srv.wait(500)
        st = srv.stats()
        srv.close()
        lat = np.sort(np.array(lat)) / 1e6
        return {"p50_ms": round(float(np.percentile(lat, 50)), 3),
                "p99_ms": round(float(np.percentile(lat, 99)), 3),
                "mean_ms": round(float(lat.mean()), 3),
                "sustained_gbs": round(total / ((last - first) / 1e9) / 1e9, 2),
                "batches": st["batches"], "max_batch": st["max_batch"]}

    zero = np.zeros(N, dtype=np.int64)
    closed_serial = run(zero, True)  # everything queued at once, one at a time
    service_ns = (total / (closed_serial["sustained_gbs"] * 1e9)) * 1e9 / N
    closed = run(zero, False)
    loads = {}
    for rho in (0.5, 0.8, 1.0):
        gaps = rng.exponential(service_ns / rho, size=N)
        arr = np.cumsum(gaps).astype(np.int64) - int(gaps[0])
        loads[str(rho)] = {"overlapped": run(arr, False), "serial": run(arr, True)}
        print(f"[bench] load {rho}: {loads[str(rho)]}", file=sys.stderr, flush=True)
    line = {
        "metric": METRIC,
        "value": closed["sustained_gbs"],
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": N,
        "warmup": 0,
        "ms_per_step": round(total / (closed["sustained_gbs"] * 1e9) * 1e3 / N, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic (seeded extended-log text; no dataset used)",
        "config": {
            "workload": f"c5: {N} requests cut from a {len(data)}-byte pinned log text, sizes log-uniform in "
                        "[4 KiB, 256 MiB], log6 DFA, 12 columns, request loop with continuous batching",
            "bytes": total, "budget_bytes": args.c5_budget, "copy_streams": args.c5_copy_streams,
        },
        "saturated": {"overlapped": closed, "serial": closed_serial},
        "serial_service_ms": round(service_ns / 1e6, 4),
        "poisson": loads,
        "pcie_h2d_gbs": round(h2d_gbs, 2),
        "roofline": {"bound": "pcie", "achieved": closed["sustained_gbs"], "peak": round(h2d_gbs, 2),
                     "unit": "GB/s", "frac": round(closed["sustained_gbs"] / h2d_gbs, 4), "traffic": None},
    }
    print(json.dumps(line), flush=True)


def bench_utf16(args):
    """The 1 GiB numeric CSV widened to UTF-16LE (2 GiB, one code unit per
    character), resident in HBM, parsed by pp_parse_utf16 (the one tile
    launch, narrowing the code units as it stages each tile). One step = one
    call."""
    import ctypes

    import numpy as np
    import torch

    import datagen
    import paper_1905_13415_amd as pp
    from datagen import dialects as D

    g = datagen.c2()
    types = list(D.SCHEMA_C2.types)
    dfa = D.csv4()
    units = g.data.astype(np.uint16)
    n_units, R = len(units), g.nrecords
    F = R * g.ncols
    dev = torch.device("cuda:0")
    d_in = torch.from_numpy(units.view(np.int16)).to(dev)
    out = pp.alloc_outputs(types, R, F, device=dev)
    L = pp.lib()
    ws = torch.empty(int(L.pp_workspace_size_utf16(n_units, None)), dtype=torch.uint8, device=dev)
    call = pp.Call(d_in, n_units, dfa, types, out, ws, None)
    stream = torch.cuda.current_stream()

    def launch():
        rc = L.pp_parse_utf16(d_in.data_ptr(), n_units, ctypes.byref(call.dfa), ctypes.byref(call.schema),
                              ctypes.byref(call.outs), ws.data_ptr(), ws.numel(), None,
                              ctypes.c_void_p(stream.cuda_stream))
        if rc != pp.PP_OK:
            raise pp.PpError(f"pp_parse_utf16: {rc}")

    if args.profile_steps:
        for _ in range(args.profile_steps):
            launch()
        torch.cuda.synchronize()
        src = torch.empty(1 << 30, dtype=torch.uint8, device=dev)  # the byte counters' reference copy
        dst = torch.empty_like(src)
        pp.copy(dst, src, stream=stream)
        torch.cuda.synchronize()
        print("[bench] profile launches done (plus one 1 GiB streaming copy)", file=sys.stderr, flush=True)
        return
    for _ in range(args.warmup):
        launch()
    torch.cuda.synchronize()
    res = out.result_dict()
    if res["status"] != pp.RESULT_OK or res["num_records"] != R or res["num_fields"] != F:
        print(f"[bench] unexpected result {res}", file=sys.stderr)
        sys.exit(1)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    for a, b in evs:
        a.record(stream)
        launch()
        b.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    per = sorted(a.elapsed_time(b) for a, b in evs)
    ms = sum(per) / len(per)
    nb = 2 * n_units
    outb = output_bytes(R, F, types)
    line = {
        "metric": METRIC, "value": round(nb / (ms / 1e3) / 1e9, 2), "unit": "GB/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(wall * 1e3 / args.steps, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u16",
        "data": "synthetic (the seeded numeric CSV, one UTF-16 code unit per character; no dataset used)",
        "config": {"workload": "utf16: the 1 GiB numeric CSV (c2) as UTF-16LE text, 2 GiB, 18 columns, csv4 DFA, "
                               "pp_parse_utf16 on a resident buffer", "bytes": nb, "records": R, "fields": F},
        "kernel_ms": {"mean": round(ms, 4), "median": round(per[len(per) // 2], 4), "min": round(per[0], 4),
                      "max": round(per[-1], 4)},
        "output_bytes": outb,
        "roofline": {"bound": "hbm", "achieved": round((nb + outb) / (ms / 1e3) / 1e9, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round((nb + outb) / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic("utf16"),
                     "timing": "HIP events on the launch stream around each call, mean over the timed steps",
                     "traffic_source": TRAFFIC_FILES["utf16"]},
    }
    tr = line["roofline"]["traffic"]
    line["roofline"]["traffic_frac"] = round(tr / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4) if tr else None
    if not args.no_cpu_baseline:
        import oracle
        t = time.perf_counter()
        ref = oracle.parse(units.view(np.uint8), dfa, types, cap_records=R, cap_fields=F, utf16=True)
        cpu_s = time.perf_counter() - t
        assert ref.num_records == R
        line["cpu_baseline"] = dict({"value": round(nb / cpu_s / 1e9, 4), "unit": "GB/s", "cores": 1, "kind": "oracle",
                                     "sample": f"the whole {nb}-byte workload, one sequential oracle parse "
                                               f"({cpu_s:.1f} s, outputs preallocated)"}, **host_cpu())
    print(json.dumps(line), flush=True)


def bench_stream(args):
    """End to end (Sec. 4.4): the 2 GiB text-heavy CSV in pinned host memory,
    parsed by pp_stream_parse in partitions (transfer, parse and return of
    the columns overlapped on three streams) into pinned host arrays. One
    step = the whole input, host to host. Against: the same input copied to
    the device in one transfer, parsed by one pp_parse call, and its outputs
    copied back, one after the other."""
    import numpy as np
    import torch

    import datagen
    import paper_1905_13415_amd as pp
    from datagen import dialects as D

    g = datagen.c3()
    types = list(D.SCHEMA_C3.types)
    dfa = D.csv4()
    n, R = len(g.data), g.nrecords
    F = R * g.ncols
    h_in = torch.empty(n, dtype=torch.uint8).pin_memory()
    h_in.numpy()[:] = g.data
    out = pp.alloc_host_outputs(types, R, F, pin=True)
    st = pp.Stream(dfa, types, partition_bytes=args.stream_partition, max_record_bytes=1 << 20)
    for _ in range(max(args.warmup, 1)):
        st.parse(h_in, out)
    if out.result["status"] != pp.RESULT_OK or out.result["num_records"] != R:
        print(f"[bench] unexpected stream result {out.result}", file=sys.stderr)
        sys.exit(1)
    steps = max(1, min(args.steps, 5))
    walls = []
    for _ in range(steps):
        t0 = time.perf_counter()
        st.parse(h_in, out)
        walls.append(time.perf_counter() - t0)
    stats = out.stats
    st.close()
    wall = sorted(walls)[len(walls) // 2]

    # the same work without overlap: one transfer in, one parse, transfers out
    dev = torch.device("cuda:0")
    d_in = torch.empty(n, dtype=torch.uint8, device=dev)
    dout = pp.alloc_outputs(types, R, F, device=dev)
    ws = torch.empty(pp.workspace_size(n), dtype=torch.uint8, device=dev)
    call = pp.Call(d_in, n, dfa, types, dout, ws)
    s = torch.cuda.current_stream()

    def serial():
        d_in.copy_(h_in, non_blocking=True)
        call.launch(s)
        for hd, dd in ((out.record_offsets, dout.record_offsets), (out.field_offsets, dout.field_offsets),
                       (out.column_ids, dout.column_ids)):
            hd[:dd.numel()].copy_(dd, non_blocking=True)
        for c in range(len(types)):
            for hd, dd in ((out.values[c], dout.values[c]), (out.valid[c], dout.valid[c]),
                           (out.str_end[c], dout.str_end[c])):
                if hd is not None:
                    hd[:dd.numel()].copy_(dd, non_blocking=True)
        torch.cuda.synchronize()
    serial()
    sw = []
    for _ in range(steps):
        t0 = time.perf_counter()
        serial()
        sw.append(time.perf_counter() - t0)
    swall = sorted(sw)[len(sw) // 2]
    # pinned transfer rates for context
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    d_in.copy_(h_in, non_blocking=True)
    e1.record(s)
    torch.cuda.synchronize()
    h2d = n / (e0.elapsed_time(e1) / 1e3) / 1e9
    e0.record(s)
    h_in.copy_(d_in, non_blocking=True)
    e1.record(s)
    torch.cuda.synchronize()
    d2h = n / (e0.elapsed_time(e1) / 1e3) / 1e9
    outb = output_bytes(R, F, types)
    line = {
        "metric": METRIC,
        "value": round(n / wall / 1e9, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": max(args.warmup, 1),
        "ms_per_step": round(wall * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic (seeded text-heavy CSV shaped like the yelp reviews; no dataset used)",
        "config": {"workload": "stream: the 2 GiB text-heavy CSV (c3) end to end from pinned host memory to pinned "
                               "host arrays, pp_stream_parse in partitions",
                   "bytes": n, "records": R, "fields": F, "partition_bytes": args.stream_partition,
                   "output_bytes": outb},
        "stream_stats": stats,
        "serial_ms": round(swall * 1e3, 3),
        "serial_gbs": round(n / swall / 1e9, 2),
        "speedup_vs_serial": round(swall / wall, 3),
        "pcie_h2d_gbs": round(h2d, 2),
        "pcie_d2h_gbs": round(d2h, 2),
        "roofline": {"bound": "pcie", "achieved": round(n / wall / 1e9, 2), "peak": round(h2d, 2), "unit": "GB/s",
                     "frac": round(n / wall / 1e9 / h2d, 4), "traffic": None},
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
