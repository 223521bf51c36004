#!/usr/bin/env python3
"""Concurrency of several crowds on one GPU, from a rocprofv3 kernel trace.

Usage (on the GPU machine):
    rocprofv3 --kernel-trace --output-format csv -d OUT -o run -- \\
        python3 bench.py --workload c3 --scan 4x512 --steps 2 --warmup 1
    python3 bench_overlap.py OUT > profiles/c3_crowd_overlap.md

Reads every *kernel_trace.csv under OUT and groups the dispatches by HIP stream (each crowd
launches on its own streams).  The window analysed is the interval in which every busy
stream (one with at least 20 dispatches) has started and none has finished: the sweeps of
all crowds, after the crowds were set up one after another.  Reported: the time during which
0, 1, 2, ... streams have a kernel running, the busy time of each stream, and the share of
the GPU-busy time during which kernels of two or more streams run at once.
"""
import csv
import glob
import os
import sys


def load(run_dir):
    files = glob.glob(os.path.join(run_dir, "**", "*kernel_trace.csv"), recursive=True)
    if not files:
        raise SystemExit("no kernel_trace.csv under %s" % run_dir)
    rows = []
    for f in files:
        with open(f, newline="") as fh:
            for r in csv.DictReader(fh):
                key = r.get("Stream_Id") or r.get("Queue_Id") or "0"
                rows.append((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), key, r["Kernel_Name"]))
    rows.sort()
    return rows


def main():
    rows = load(sys.argv[1])
    n = len(rows)
    per = {}
    for s_, e_, key, _ in rows:
        per.setdefault(key, []).append((s_, e_))
    busy_streams = [k for k, v in per.items() if len(v) >= 20]
    t0 = max(min(s_ for s_, _ in per[k]) for k in busy_streams)
    t1 = min(max(e_ for _, e_ in per[k]) for k in busy_streams)
    part = [(max(s_, t0), min(e_, t1), key, name) for s_, e_, key, name in rows if e_ > t0 and s_ < t1]
    events = []
    busy = {}
    for s, e, key, _ in part:
        events.append((s, 1, key))
        events.append((e, -1, key))
        busy[key] = busy.get(key, 0) + (e - s)
    events.sort()
    active = {}
    level_time = {}
    last = t0
    for t, d, key in events:
        lev = sum(1 for v in active.values() if v > 0)
        level_time[lev] = level_time.get(lev, 0) + (t - last)
        last = t
        active[key] = active.get(key, 0) + d
    span = t1 - t0
    gpu_busy = span - level_time.get(0, 0)
    multi = sum(v for k, v in level_time.items() if k >= 2)
    print("# Crowd concurrency from a kernel trace\n")
    print("Command: %s\n" % " ".join(sys.argv))
    print("Dispatches analysed: %d of %d (streams %s), span %.3f ms.\n"
          % (len(part), n, ", ".join(sorted(busy_streams)), span / 1e6))
    print("| streams with a kernel running | time (ms) | share of span |")
    print("|---|---|---|")
    for lev in sorted(level_time):
        print("| %d | %.3f | %.1f %% |" % (lev, level_time[lev] / 1e6, 100.0 * level_time[lev] / span))
    print("\n| stream | dispatches | busy (ms) |")
    print("|---|---|---|")
    for key in sorted(busy):
        cnt = sum(1 for r in part if r[2] == key)
        print("| %s | %d | %.3f |" % (key, cnt, busy[key] / 1e6))
    print("\nGPU busy %.3f ms of %.3f ms; two or more streams at once during %.1f %% of the busy time."
          % (gpu_busy / 1e6, span / 1e6, 100.0 * multi / max(gpu_busy, 1)))


if __name__ == "__main__":
    main()
