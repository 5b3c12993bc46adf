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
bytes against the 8 TB/s HBM peak; ``cpu_baseline`` is the sequential oracle
on the host, timed on the same buffer.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--nbytes", type=int, default=1 << 30)
    ap.add_argument("--bytes-per-thread", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile-steps", type=int, default=0,
                    help="only run this many launches (for rocprofv3), no JSON")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU; --gpus {args.gpus} is not supported "
              f"(the parse shards by byte range with one small all-gather; see DESIGN.md)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import datagen
    import paper_1905_13415_amd as pp
    from datagen import dialects as D

    t0 = time.time()
    g = datagen.c2(nbytes=args.nbytes)
    types = D.SCHEMA_C2.types
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
        # reference for the HBM byte counters: one device copy of exactly 2^30 bytes
        src = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print("[bench] profile launches done (plus one 1 GiB device copy)", file=sys.stderr, flush=True)
        return

    for _ in range(args.warmup):
        call.launch(stream)
    torch.cuda.synchronize()
    res = out.result_dict()
    if res["status"] != pp.RESULT_OK or res["num_records"] != R or res["num_fields"] != F:
        print(f"[bench] unexpected result {res}", file=sys.stderr)
        sys.exit(1)

    # timed region: K launches bracketed by synchronisation, HIP events on the
    # launch stream around every call
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

    # practical ceiling: a device-to-device copy of the same number of bytes
    outb = output_bytes(R, F, types)
    total_b = n + outb
    src = torch.empty(total_b // 2, dtype=torch.uint8, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    c0.record(stream)
    for _ in range(10):
        dst.copy_(src)
    c1.record(stream)
    torch.cuda.synchronize()
    copy_gbs = 2 * src.numel() * 10 / (c0.elapsed_time(c1) / 1e3) / 1e9
    del src, dst

    in_gbs = n / (ms_mean / 1e3) / 1e9
    inout_gbs = total_b / (ms_mean / 1e3) / 1e9
    line = {
        "metric": "on-device parse GB/s & % of HBM roofline; batched/serving vs plain; p50/p99 latency",
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
        "data": "synthetic (seeded numeric CSV shaped like the NYC taxi trips; no dataset used)",
        "config": {
            "workload": "c2: 1 GiB numeric CSV, 18 columns (4 int64, 2 timestamp, 8 float64, 4 string), "
                        "~130 B/record, csv4 DFA, plain single-buffer launch",
            "bytes": n, "records": R, "fields": F,
            "bytes_per_thread": args.bytes_per_thread or 64, "block_threads": 512 if not args.bytes_per_thread else 256,
        },
        "kernel_ms": {"mean": round(ms_mean, 4), "median": round(ms_med, 4), "min": round(per[0], 4),
                      "max": round(per[-1], 4)},
        "input_gbs": round(in_gbs, 2),
        "in_out_gbs": round(inout_gbs, 2),
        "output_bytes": outb,
        "d2d_copy_gbs": round(copy_gbs, 1),
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
        t = time.perf_counter()
        ref = oracle.parse(g.data, dfa, types, cap_records=R, cap_fields=F)
        cpu_s = time.perf_counter() - t
        assert ref.num_records == R
        line["cpu_baseline"] = {"value": round(n / cpu_s / 1e9, 4), "unit": "GB/s", "cores": 1,
                                "kind": "oracle",
                                "sample": f"the whole {n}-byte workload, one sequential oracle parse "
                                          f"({cpu_s:.1f} s, outputs preallocated)"}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
