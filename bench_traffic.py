#!/usr/bin/env python3
"""HBM traffic of the gather and update kernels from two rocprofv3 counter runs of bench.py.

Usage (on the GPU machine, each run in its own process):
    rocprofv3 --pmc FETCH_SIZE --output-format csv -d OUT/fetch -o run -- \\
        python3 bench.py --steps 2 --warmup 1 --fp64-steps 0 --no-cpu --calibrate-copy
    rocprofv3 --pmc WRITE_SIZE --output-format csv -d OUT/write -o run -- \\
        python3 bench.py --steps 2 --warmup 1 --fp64-steps 0 --no-cpu --calibrate-copy
    python3 bench_traffic.py OUT/fetch OUT/write c4 > profiles/k_prop_vgl_c4_traffic.json

FETCH_SIZE and WRITE_SIZE are read per dispatch in KiB.  The library's plain
copy kernel (cq::k_copy16, 1 GiB read + 1 GiB written, launched once by
--calibrate-copy) gives the factor between counter readings and bytes; the
per-launch averages of the gather (k_prop_vgl_wave), of the update
(k_flush_mfma_batch, "update"), of the FP64 Sherman-Morrison update
(k_flush_vec<double>, "sm") and of the virtual-move kernel (k_virtual,
"virtual") are scaled by it.  The output records the source
hash of the kernels, so bench.py uses the figures only while they are unchanged.
"""
import csv
import glob
import json
import os
import sys

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)


def per_kernel(run_dir, counter):
    files = glob.glob(os.path.join(run_dir, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise SystemExit("no counter_collection.csv under %s" % run_dir)
    sums, counts = {}, {}
    for f in files:
        with open(f, newline="") as fh:
            for row in csv.DictReader(fh):
                if row.get("Counter_Name") != counter:
                    continue
                name = row["Kernel_Name"]
                # one value per dispatch (sum over dimensions of the same dispatch)
                key = (name, row.get("Dispatch_Id"))
                sums[key] = sums.get(key, 0.0) + float(row["Counter_Value"])
    out = {}
    for (name, _), val in sums.items():
        s, c = out.get(name, (0.0, 0))
        out[name] = (s + val, c + 1)
    return {k: (s / c, c) for k, (s, c) in out.items()}


def pick(table, needle):
    hits = [(k, v) for k, v in table.items() if needle in k]
    if not hits:
        raise SystemExit("kernel %s not found in counters" % needle)
    return hits[0][1]


def main():
    fetch_dir, write_dir, workload = sys.argv[1], sys.argv[2], sys.argv[3]
    from bench import kernel_source_hash
    fetch = per_kernel(fetch_dir, "FETCH_SIZE")
    write = per_kernel(write_dir, "WRITE_SIZE")
    copy_bytes = float(1 << 30)
    cf, _ = pick(fetch, "k_copy16")
    cw, _ = pick(write, "k_copy16")
    sf, sw = copy_bytes / (cf * 1024.0), copy_bytes / (cw * 1024.0)
    gf, nf = pick(fetch, "k_prop_vgl_wave<float")
    gw, nw = pick(write, "k_prop_vgl_wave<float")
    fb, wb = gf * 1024.0 * sf, gw * 1024.0 * sw
    uf, unf = pick(fetch, "k_flush_mfma_batch")
    uw, unw = pick(write, "k_flush_mfma_batch")
    ufb, uwb = uf * 1024.0 * sf, uw * 1024.0 * sw
    update = dict(kernel="k_flush_mfma_batch", launches=[unf, unw], fetch_kib_per_launch=uf,
                  write_kib_per_launch=uw, fetch_bytes_per_launch=ufb, write_bytes_per_launch=uwb,
                  traffic_bytes_per_launch=ufb + uwb)
    extra = {}
    for key, needle in (("sm", "k_flush_vec<double"), ("virtual", "k_virtual")):
        if any(needle in k for k in fetch) and any(needle in k for k in write):
            xf, xnf = pick(fetch, needle)
            xw, xnw = pick(write, needle)
            extra[key] = dict(kernel=needle, launches=[xnf, xnw], fetch_kib_per_launch=xf, write_kib_per_launch=xw,
                              fetch_bytes_per_launch=xf * 1024.0 * sf, write_bytes_per_launch=xw * 1024.0 * sw,
                              traffic_bytes_per_launch=xf * 1024.0 * sf + xw * 1024.0 * sw)
    rec = dict(kernel="k_prop_vgl_wave", workload=workload, launches=[nf, nw],
               fetch_kib_per_launch=gf, write_kib_per_launch=gw,
               copy_fetch_kib=cf, copy_write_kib=cw, scale_fetch=sf, scale_write=sw,
               fetch_bytes_per_launch=fb, write_bytes_per_launch=wb, traffic_bytes_per_launch=fb + wb,
               update=update, source_sha256=kernel_source_hash(), **extra,
               command="rocprofv3 --pmc FETCH_SIZE|WRITE_SIZE --output-format csv -d DIR -o run -- "
                       "python3 bench.py --steps 2 --warmup 1 --fp64-steps 0 --no-cpu --alone-steps 0 --calibrate-copy; "
                       "python3 bench_traffic.py FETCH_DIR WRITE_DIR %s" % workload)
    print(json.dumps(rec, indent=1))


if __name__ == "__main__":
    main()
