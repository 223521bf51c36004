#!/usr/bin/env python3
"""Benchmark of the batched particle-by-particle VMC move on one MI355X.

A step is one sweep: every electron of every walker proposes one move (propose,
B-spline VGL, ratio, Jastrow, Metropolis, inverse update), then the local
energy; the FP64 recompute of the inverses runs every `recompute_every` sweeps
inside the timed steps.  Default workload: 1024 + 1024 electrons, L = 32 bohr,
96^3 FP32 B-spline table (3.62 GB), Pade J2, 128 walkers, delayed rank 32,
recompute every 32 sweeps, mixed precision; the same workload in FP64 is timed
for the mixed-vs-FP64 comparison.  Inputs are synthetic and seeded.

Prints ONE JSON line on stdout (progress goes to stderr).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
FP32_PEAK_TFLOPS = 157.3       # MI355X dense FP32 (vector = MFMA)
METRIC = "electron moves/sec at 1 GPU (mixed vs FP64 GPU) + B-spline HBM GB/s, update MFMA %"


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=32)
    ap.add_argument("--warmup", type=int, default=4)
    ap.add_argument("--workload", default="c4")
    ap.add_argument("--fp64-steps", type=int, default=2, help="sweeps of the FP64 comparison run (0: skip)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-moves", type=int, default=512, help="moves per walker in the CPU baseline sample")
    ap.add_argument("--delay", type=int, default=None, help="override the delay rank")
    ap.add_argument("--eager", action="store_true", help="launch kernels eagerly instead of replaying a graph")
    return ap.parse_args()


def make_system(cq, wl, elem_bytes):
    from synth import J2_A_ANTI, J2_A_PAR, J2_B
    s = cq.System(wl.n, wl.L)
    s.fill_philox(wl.seed, elem_bytes, wl.G)
    if wl.use_j2:
        s.load_j2(J2_A_PAR, J2_A_ANTI, J2_B)
    return s


def run_gpu(cq, wl, precision, delay, recompute, steps, warmup, timing_kinds, use_graph):
    """Time `steps` sweeps over `wl.crowds` crowds (one stream each); returns a result dict."""
    from synth import start_positions
    system = make_system(cq, wl, 4 if precision == "mixed" else 8)
    crowds = []
    for ci in range(wl.crowds):
        c = cq.Crowd(system, wl.walkers, precision=precision, delay_rank=delay, recompute_every=recompute,
                     seed=wl.seed, first_uid=ci * wl.walkers, use_graph=use_graph)
        c.set_positions(start_positions(wl.seed, wl.walkers, wl.n_e, wl.L, first_walker=ci * wl.walkers))
        crowds.append(c)
    log("  %s: %d crowd(s) x %d walkers set up" % (precision, wl.crowds, wl.walkers))
    for c in crowds:
        c.run_vmc(warmup, wl.sigma)
    for c in crowds:
        c.synchronize()
    for c in crowds:
        c.set_timing(timing_kinds)
    t0 = time.perf_counter()
    for c in crowds:
        c.run_vmc(steps, wl.sigma)
    for c in crowds:
        c.synchronize()
    t1 = time.perf_counter()
    kt = {}
    for k in timing_kinds:
        ms, n = 0.0, 0
        for c in crowds:
            a, b = c.kernel_timing(k)
            ms += a
            n += b
        kt[k] = (ms, n)
    acc = sum(int(c.acceptance()[0].sum()) for c in crowds)
    prop = sum(int(c.acceptance()[1].sum()) for c in crowds)
    el = np.concatenate([c.local_energy() for c in crowds])
    for c in crowds:
        c.set_timing(())
        c.close()
    system.close()
    moves = wl.crowds * wl.walkers * wl.n_e * steps
    return dict(seconds=t1 - t0, moves=moves, moves_per_s=moves / (t1 - t0), kernels=kt,
                acceptance=acc / max(prop, 1), e_mean=float(el.mean()), finite=bool(np.isfinite(el).all()))


def cpu_baseline(wl, moves_per_walker):
    """The FP64 oracle (OpenMP over walkers) on a bounded sample of the same workload."""
    import oracle as orc
    from synth import J2_A_ANTI, J2_A_PAR, J2_B, start_positions
    threads = min(os.cpu_count() or 1, 16)
    walkers = threads
    s = orc.System(wl.n, wl.n, wl.L, G=wl.G, n_orb=wl.n, orb_kind=orc.ORB_SEEDED, coef_seed=wl.seed,
                   coef_fp32=True, use_j2=wl.use_j2, j2_a_par=J2_A_PAR, j2_a_anti=J2_A_ANTI, j2_b=J2_B,
                   seed=wl.seed)
    R0 = start_positions(wl.seed, walkers, wl.n_e, wl.L)
    t0 = time.perf_counter()
    orc.setup(s, R0, n_threads=threads)
    t1 = time.perf_counter()
    orc.vmc(s, R0, 1, sigma=wl.sigma, max_moves=moves_per_walker, n_threads=threads)
    t2 = time.perf_counter()
    move_s = (t2 - t1) - (t1 - t0)  # the run repeats the set-up; count the moves only
    return dict(value=walkers * moves_per_walker / move_s, unit="moves/s", cores=threads, kind="oracle",
                sample="%d walkers x first %d electron moves of sweep 0 (%s), FP64 scalar C + OpenMP, "
                       "set-up time (%.1f s) subtracted" % (walkers, moves_per_walker, wl.name, t1 - t0),
                seconds=round(t2 - t0, 1))


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: every box here has one MI355X, and the walker-parallel path "
              "is not sharded across GPUs in this build (see DESIGN.md for how it would shard).",
              file=sys.stderr)
        sys.exit(2)
    import paper_2209_14487_amd as cq
    from synth import WORKLOADS
    wl = WORKLOADS[args.workload]
    delay = args.delay if args.delay is not None else wl.delay_rank
    log("workload %s: N=%d per spin, W=%d x %d crowd(s), G=%d, k=%d, recompute every %d"
        % (wl.name, wl.n, wl.walkers, wl.crowds, wl.G, delay, wl.recompute_every))

    kinds = ["vgl", "update"]
    mixed = run_gpu(cq, wl, "mixed", delay, wl.recompute_every, args.steps, args.warmup, kinds, not args.eager)
    log("  mixed: %.3f s for %d sweeps, %.3e moves/s, acceptance %.3f"
        % (mixed["seconds"], args.steps, mixed["moves_per_s"], mixed["acceptance"]))
    # eager-launch pass with events on every kernel class: device time per kernel class
    ev = run_gpu(cq, wl, "mixed", delay, wl.recompute_every, max(2, args.steps // 4), 1,
                 ["vgl", "resolve", "update", "energy", "inverse"], False)

    n, W, s_c, s = wl.n, wl.walkers * wl.crowds, 4, 4
    kinfo = {}
    for k, (ms, cnt) in ev["kernels"].items():
        kinfo[k] = dict(ms_total=round(ms, 3), launches=cnt, us_per_launch=round(1e3 * ms / max(cnt, 1), 3),
                        share=round(ms / (1e3 * ev["seconds"]), 4))
    # B-spline VGL kernel (per launch: every walker gathers 64 stencil points x N orbitals,
    # reads its inverse column and writes the proposal's 5 orbital rows and the column)
    vgl_ms, vgl_n = mixed["kernels"]["vgl"]
    vgl_bytes = W * (64 * n * s_c + n * s + 6 * n * s)
    vgl_gbs = vgl_bytes / (vgl_ms / vgl_n * 1e-3) / 1e9
    # update kernel (per launch: every walker reads and writes its N x N inverse once and streams
    # the window's k rows and k columns; 4 N^2 k flops executed)
    up_ms, up_n = mixed["kernels"]["update"]
    up_bytes = W * (2 * n * n * s + 2 * delay * n * s)
    up_flops = W * 4.0 * n * n * delay
    up_t = up_ms / max(up_n, 1) * 1e-3
    roof_vgl = dict(bound="hbm", achieved=round(vgl_gbs, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(vgl_gbs / HBM_PEAK_GBS, 4), traffic=None, kernel="k_vgl_move",
                    us_per_launch=round(vgl_ms / vgl_n * 1e3, 3), bytes_per_launch=vgl_bytes)
    roof_up = dict(bound="mfma", achieved=round(up_flops / up_t / 1e12, 2), peak=FP32_PEAK_TFLOPS,
                   unit="TFLOP/s", frac=round(up_flops / up_t / 1e12 / FP32_PEAK_TFLOPS, 4),
                   hbm_gbs=round(up_bytes / up_t / 1e9, 1), kernel="k_flush (+k_finalize)",
                   us_per_launch=round(up_t * 1e6, 3))

    out = dict(metric=METRIC, value=round(mixed["moves_per_s"], 1), unit="moves/s", n_gpus=1, steps=args.steps,
               warmup=args.warmup, ms_per_step=round(1e3 * mixed["seconds"] / args.steps, 3),
               higher_is_better=True, scaling="weak", vs_baseline=None, dtype="f32",
               data="synthetic (seeded Philox B-spline coefficients, uniform starting positions)",
               config=dict(workload="%s: %d+%d electrons, L=%g bohr, %d^3 FP32 B-spline table (%.2f GB), Pade J2, "
                                    "%d crowd(s) x %d walkers, delayed rank %d, FP64 recompute every %d sweeps"
                                    % (wl.name, n, n, wl.L, wl.G, wl.table_bytes(4) / 1e9, wl.crowds, wl.walkers,
                                       delay, wl.recompute_every),
                           precision="mixed", launch="eager" if args.eager else "hipGraph per sweep"),
               roofline=roof_vgl if vgl_ms >= up_ms else roof_up,
               roofline_spline=roof_vgl, roofline_update=roof_up, kernels=kinfo,
               acceptance=round(mixed["acceptance"], 4), e_mean=mixed["e_mean"])
    if args.fp64_steps > 0:
        f64 = run_gpu(cq, wl, "fp64", delay, 0, args.fp64_steps, 1, [], not args.eager)
        log("  fp64: %.3e moves/s" % f64["moves_per_s"])
        out["fp64_moves_per_s"] = round(f64["moves_per_s"], 1)
        out["mixed_over_fp64"] = round(mixed["moves_per_s"] / f64["moves_per_s"], 3)
    if not args.no_cpu:
        log("  cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_moves)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
