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
    ap.add_argument("--workload", default="c4",
                    help="c1..c6, or inverse (the FP64 recompute alone on the C4 matrices)")
    ap.add_argument("--fp64-steps", type=int, default=2, help="sweeps of the FP64 comparison run (0: skip)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-moves", type=int, default=2048, help="moves per walker in the CPU baseline sample")
    ap.add_argument("--time-kernels", default="vgl,update",
                    help="kernel kinds bracketed by HIP events in the timed run (comma separated, from "
                         "propose, vgl, resolve, update, energy, inverse); the events add launches to the "
                         "timed region, so by default only the two roofline kernels are bracketed")
    ap.add_argument("--delay", type=int, default=None, help="override the delay rank")
    ap.add_argument("--alone-steps", type=int, default=4,
                    help="sweeps of a one-stream run that times the gather and the update alone (0: skip)")
    ap.add_argument("--eager", action="store_true", help="skip the extra hipGraph replay run")
    ap.add_argument("--path", default="auto", choices=["auto", "multi", "window", "batch"],
                    help="mapping of the moves to the GPU")
    ap.add_argument("--sm-steps", type=int, default=1,
                    help="sweeps of the FP64 Sherman-Morrison (k = 1) run that measures the SM update's "
                         "HBM GB/s (0: skip)")
    ap.add_argument("--cpu-one-core-moves", type=int, default=1024,
                    help="moves of the one-core CPU oracle figure (0: skip)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first copy 1 GiB with the library's plain copy kernel (counter calibration runs)")
    ap.add_argument("--virtual-points", type=int, default=12,
                    help="quadrature points per electron of the timed virtual-move launch (0: skip)")
    ap.add_argument("--tiles", default="",
                    help="launch shapes of the batched path, Q,G[,U] (candidates per round, gather workgroups per CU "
                         "beside the update, FP64 update kernel 1 vector / 2 matrix cores); default: the built-in rules")
    ap.add_argument("--tile-cache", default="",
                    help="JSON tile cache: take the shapes from it, or tune them (2 sweeps per candidate, before "
                         "the warm-up) and add them to it")
    ap.add_argument("--scan", default="",
                    help="crowd/walker scan instead of the bench line: comma-separated CROWDSxWALKERS pairs "
                         "(e.g. 1x512,2x512,4x512); each is timed over --steps sweeps after --warmup, graph replay")
    return ap.parse_args()


def run_virtual(cq, wl, nq, launches=3):
    """Ratio-only virtual moves of every electron of every walker to nq icosahedral points of
    radius 0.5 bohr (mixed precision, set-up state), timed with HIP events on the crowd's stream.
    Algorithmic bytes per point: the 64 stencil rows of the value-only spline, 64 N 4 B."""
    from synth import icosahedron_offsets, start_positions
    system = make_system(cq, wl, 4)
    W = wl.walkers
    c = cq.Crowd(system, W, precision="mixed", delay_rank=wl.delay_rank, seed=wl.seed)
    c.set_positions(start_positions(wl.seed, W, wl.n_e, wl.L))
    off = np.vstack([icosahedron_offsets(0.5), icosahedron_offsets(0.25)])[:nq]
    out = cq.DeviceArray(shape=(W, wl.n_e, nq), dtype=np.float64)
    c.virtual_ratios(off, out=(out, None, None))  # warm-up
    c.synchronize()
    c.set_timing(("virtual",))
    for _ in range(launches):
        c.virtual_ratios(off, out=(out, None, None))
    c.synchronize()
    ms, cnt = c.kernel_timing("virtual")
    c.set_timing(())
    ratios = out.numpy()
    c.close()
    system.close()
    out.free()
    t = 1e-3 * ms / cnt
    points = W * wl.n_e * nq
    bytes_alg = points * 64 * wl.n * 4
    gbs = bytes_alg / t / 1e9
    return dict(bound="hbm", achieved=round(gbs, 1), peak=HBM_PEAK_GBS, unit="GB/s", frac=round(gbs / HBM_PEAK_GBS, 4),
                traffic=None, kernel="k_virtual", us_per_launch=round(t * 1e6, 3), points_per_launch=points,
                bytes_per_launch=bytes_alg, points_per_s=round(points / t, 1), finite=bool(np.isfinite(ratios).all()),
                note="value-only spline at %d points around every electron (radius 0.5 and 0.25 bohr) and the "
                     "dot with its inverse column, plus the Jastrow sums; algorithmic bytes = 64 N 4 B per "
                     "point (neighbouring points share stencil rows, so cache reuse can take the figure past "
                     "HBM speed)" % nq)


# Complex (twisted) orbitals in the triclinic cell: 64 + 64 electrons, 24^3 complex FP64 table
# (14 MB), Pade J2, twist (0.11, -0.07, 0.05) 1/bohr, 512 walkers, sigma 0.5.
C6 = dict(n=64, G=24, walkers=512, sigma=0.5, seed=1006, twist=(0.11, -0.07, 0.05))


def complex_leg(cq, args, precision):
    """Timed sweeps of the C6 system with one table precision: (moves/s, roofline dict, acceptance,
    E_L [W], R0)."""
    from synth import J2_A_ANTI, J2_A_PAR, J2_B, TRICLINIC, cell_positions, complex_table
    c6 = C6
    n, W, G = c6["n"], c6["walkers"], c6["G"]
    ne = 2 * n
    table = complex_table(c6["seed"], G, n)
    cb = 16 if precision == "fp64" else 8  # bytes per coefficient
    g = cq.ComplexSystem(n, TRICLINIC, c6["twist"])
    g.load_table(table if cb == 16 else table.astype(np.complex64))
    g.load_j2(J2_A_PAR, J2_A_ANTI, J2_B)
    R0 = cell_positions(c6["seed"], W, ne, TRICLINIC)
    crowd = cq.ComplexCrowd(g, W, seed=c6["seed"], precision=precision)
    crowd.set_positions(R0)
    crowd.run_vmc(args.warmup, c6["sigma"])
    crowd.synchronize()
    acc0, prop0 = (x.sum() for x in crowd.acceptance())
    crowd.set_timing(True)
    t0 = time.perf_counter()
    crowd.run_vmc(args.steps, c6["sigma"])
    crowd.synchronize()
    t1 = time.perf_counter()
    ms, launches = crowd.timing()
    acc1, prop1 = (x.sum() for x in crowd.acceptance())
    el = crowd.local_energy()
    crowd.close()
    g.close()
    moves = int(prop1 - prop0)
    accepted = int(acc1 - acc0)
    t_launch = 1e-3 * ms / max(launches, 1)
    bytes_launch = (moves * (64 * n * cb + n * 16) + accepted * (2 * n * n * 16 + 5 * n * 16)) / max(launches, 1)
    gbs = bytes_launch / t_launch / 1e9
    roof = dict(bound="hbm", achieved=round(gbs, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(gbs / HBM_PEAK_GBS, 4), traffic=None, kernel="k_csweep",
                us_per_launch=round(t_launch * 1e6, 3), bytes_per_launch=int(bytes_launch),
                moves_per_launch=moves // max(launches, 1),
                note="one launch = one sweep of every walker (one workgroup each); the table and most "
                     "inverses stay in the caches, so the chain of dependent moves, not HBM, bounds the kernel")
    return moves / (t1 - t0), t1 - t0, roof, accepted / max(moves, 1), el, R0


def run_complex(cq, args):
    """The complex-orbital path: moves/s over timed sweeps (one sweep-kernel launch each, HIP events
    around every launch) and the kernel's algorithmic bytes per launch: per move 64 stencil rows of
    N complex coefficients and the inverse row of the ratio, per accepted move one read and one
    write of the N x N complex inverse and the five new orbital rows.  The headline reads the
    complex128 table; `coef32` reads the complex64 table with the same FP64 arithmetic."""
    from synth import J2_A_ANTI, J2_A_PAR, J2_B, TRICLINIC, complex_table
    c6 = C6
    n, W, G = c6["n"], c6["walkers"], c6["G"]
    ne = 2 * n
    rate, secs, roof, acc, el, R0 = complex_leg(cq, args, "fp64")
    rate32, _, roof32, _, el32, _ = complex_leg(cq, args, "mixed")
    out = dict(metric="electron moves/sec at 1 GPU, complex orbitals with a twist in a triclinic cell (FP64)",
               value=round(rate, 1), unit="moves/s", n_gpus=1, steps=args.steps, warmup=args.warmup,
               ms_per_step=round(1e3 * secs / args.steps, 3), higher_is_better=True, scaling="weak",
               vs_baseline=None, dtype="f64",
               data="synthetic (seeded complex B-spline coefficients, uniform fractional starting positions)",
               config=dict(workload="c6: %d+%d electrons, triclinic cell (volume %.0f bohr^3), %d^3 complex FP64 "
                                    "table (%.3f GB), twist %s, Pade J2, %d walkers, Sherman-Morrison"
                                    % (n, n, abs(np.linalg.det(TRICLINIC)), G, G ** 3 * n * 16 / 1e9,
                                       list(c6["twist"]), W)),
               roofline=roof, acceptance=round(acc, 4), e_mean=float(np.mean(el.real)),
               e_imag_mean=float(np.mean(el.imag)),
               coef32=dict(moves_per_s=round(rate32, 1), roofline=roof32, e_mean=float(np.mean(el32.real)),
                           note="complex64 coefficients (half the spline bytes), every sum and the inverses FP64"))
    if not args.no_cpu:
        from oracle import complex_oracle as co
        o = co.CSystem(n, TRICLINIC, np.array(c6["twist"]), table=complex_table(c6["seed"], G, n), use_j2=True,
                       j2_a_par=J2_A_PAR, j2_a_anti=J2_A_ANTI, j2_b=J2_B, seed=c6["seed"])
        tc = time.perf_counter()
        co.vmc(o, R0[:2], 1, sigma=c6["sigma"])
        dt = time.perf_counter() - tc
        out["cpu_baseline"] = dict(value=round(2 * ne / dt, 2), unit="moves/s", cores=1, kind="oracle",
                                   sample="walkers 0 and 1, one sweep each (%d moves each, set-up and local energy included), "
                                          "numpy FP64 complex oracle, one thread" % ne, seconds=round(dt, 2))
    log("  complex: %.3e moves/s, k_csweep %.1f us per launch, %.0f GB/s algorithmic, acceptance %.3f; "
        "complex64 table %.3e moves/s, %.1f us per launch"
        % (out["value"], roof["us_per_launch"], roof["achieved"], out["acceptance"], rate32, roof32["us_per_launch"]))
    print(json.dumps(out), flush=True)


def run_inverse(cq, args):
    """The FP64 recompute alone: cq_slater_inverse (the recompute's kernels) on the 2W Slater
    matrices of a workload's system (C4: 256 matrices of N = 1024, stored in FP32 as in the mixed
    crowd), seeded diagonally dominated entries, `steps` timed calls after `warmup`.  The call is
    synchronous and allocates its workspace, so the wall time per call is an upper bound of the
    kernels' time; the roofline counts 2 N^3 flops per matrix against the FP64 peak."""
    from synth import WORKLOADS
    wl = WORKLOADS["c4" if args.workload == "inverse" else args.workload]
    n, nmat = wl.n, 2 * wl.walkers
    rng = np.random.default_rng(wl.seed)
    A = rng.uniform(-1, 1, (nmat, n, n)).astype(np.float32)
    A += np.float32(n ** 0.5) * np.eye(n, dtype=np.float32)[None]
    tA, tM = cq.DeviceArray(A), cq.DeviceArray(shape=A.shape, dtype=np.float32)
    tl, ts = cq.DeviceArray(shape=(nmat,), dtype=np.float64), cq.DeviceArray(shape=(nmat,), dtype=np.int32)
    for _ in range(args.warmup):
        cq.slater_inverse(tA, tM, tl, ts)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        cq.slater_inverse(tA, tM, tl, ts)
    secs = (time.perf_counter() - t0) / args.steps
    ld = tl.numpy()
    ref = np.linalg.slogdet(A[0].astype(np.float64))[1]
    tflops = 2.0 * n ** 3 * nmat / secs / 1e12
    out = dict(metric="FP64 batched Slater inversion (the periodic recompute)", value=round(1e3 * secs, 3),
               unit="ms per call", higher_is_better=False, n_gpus=1, steps=args.steps, warmup=args.warmup,
               dtype="f64", data="synthetic (seeded uniform entries plus sqrt(N) on the diagonal)",
               config=dict(workload="%s recompute: %d matrices of N = %d, FP32 storage, FP64 arithmetic"
                                    % (wl.name, nmat, n)),
               roofline=dict(bound="mfma", achieved=round(tflops, 2), peak=78.6, unit="TFLOP/s",
                             frac=round(tflops / 78.6, 4), traffic=None,
                             note="2 N^3 flops per matrix over the wall time of a synchronous call"),
               logdet_check=abs(float(ld[0]) - float(ref)))
    log("  inverse: %.2f ms per call, %.1f TFLOP/s" % (1e3 * secs, tflops))
    print(json.dumps(out), flush=True)


def run_scan(cq, args):
    """Moves/s over crowds x walkers per crowd on one GPU (the workload's system, its delay rank and
    recompute period): crowds are independent streams launched from one host thread, each replaying
    its captured sweep graph, so they overlap on the GPU (the paper's crowds over threads, Alg. 4)."""
    import dataclasses
    from synth import WORKLOADS
    base = WORKLOADS[args.workload]
    delay = args.delay if args.delay is not None else base.delay_rank
    rows = []
    for pair in args.scan.split(","):
        nc, nw = (int(x) for x in pair.lower().split("x"))
        wl = dataclasses.replace(base, crowds=nc, walkers=nw)
        r = run_gpu(cq, wl, "mixed", delay, wl.recompute_every, args.steps, args.warmup, [], True, path=args.path)
        rows.append(dict(crowds=nc, walkers_per_crowd=nw, walkers=nc * nw, moves_per_s=round(r["moves_per_s"], 1),
                         ms_per_sweep=round(1e3 * r["seconds"] / args.steps, 3), acceptance=round(r["acceptance"], 4)))
        log("  scan %d crowd(s) x %d walkers: %.3e moves/s" % (nc, nw, r["moves_per_s"]))
    out = dict(metric="electron moves/sec at 1 GPU over crowds x walkers per crowd", unit="moves/s",
               higher_is_better=True, dtype="f32", n_gpus=1, steps=args.steps, warmup=args.warmup,
               data="synthetic (seeded Philox B-spline coefficients, uniform starting positions)",
               config=dict(workload="%s: %d+%d electrons, L=%g bohr, %d^3 FP32 table, Pade J2, delayed rank %d, "
                                    "FP64 recompute every %d sweeps, mixed precision, graph replay"
                                    % (base.name, base.n, base.n, base.L, base.G, delay, base.recompute_every)),
               scan=rows)
    print(json.dumps(out), flush=True)


def make_system(cq, wl, elem_bytes):
    from synth import J2_A_ANTI, J2_A_PAR, J2_B
    s = cq.System(wl.n, wl.L)
    s.fill_philox(wl.seed, elem_bytes, wl.G)
    if wl.use_j2:
        s.load_j2(J2_A_PAR, J2_A_ANTI, J2_B)
    return s


def run_gpu(cq, wl, precision, delay, recompute, steps, warmup, timing_kinds, use_graph, path="auto",
            graph_steps=0, streams=2, tiles=None, tile_cache=None):
    """Time `steps` sweeps over `wl.crowds` crowds (one stream each); returns a result dict.

    With timing_kinds, HIP events bracket every launch of those kernel kinds on each crowd's
    stream during the timed sweeps (launches are then eager).  graph_steps > 0 adds a second
    timed run of that many sweeps replaying the captured sweep graph, no events."""
    from synth import start_positions
    system = make_system(cq, wl, 4 if precision == "mixed" else 8)
    crowds = []
    for ci in range(wl.crowds):
        c = cq.Crowd(system, wl.walkers, precision=precision, delay_rank=delay, recompute_every=recompute,
                     seed=wl.seed, first_uid=ci * wl.walkers, use_graph=use_graph, path=path, streams=streams)
        c.set_positions(start_positions(wl.seed, wl.walkers, wl.n_e, wl.L, first_walker=ci * wl.walkers))
        if tiles:
            c.set_tiles(*tiles)
        elif tile_cache:
            t, hit = c.autotune_tiles(2, tile_cache)
            log("  tiles %s (%s)" % (t, "from the cache" if hit else "tuned"))
        crowds.append(c)
    log("  %s: %d crowd(s) x %d walkers set up, tiles %s" % (precision, wl.crowds, wl.walkers, crowds[0].tiles()))
    for c in crowds:
        c.run_vmc(warmup, wl.sigma)
    for c in crowds:
        c.synchronize()
    acc0 = sum(int(c.acceptance()[0].sum()) for c in crowds)
    rec0 = sum(c.drift()[2] for c in crowds)
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
    k_used = crowds[0].delay_rank()
    path_used = crowds[0].path()
    tiles_used = crowds[0].tiles()
    el = np.concatenate([c.local_energy() for c in crowds])
    # FP64 recomputes that fell inside the timed sweeps, and their device time
    n_rec = sum(c.drift()[2] for c in crowds) - rec0
    rec_ms_in = kt["inverse"][0] if "inverse" in kt else 0.0
    rec_ms = None
    if recompute > 0:
        # one recompute of every crowd, timed alone (the recomputes of the timed sweeps are too
        # when there were any): device time per recompute of the whole crowd set
        for c in crowds:
            c.set_timing(("inverse",))
        for c in crowds:
            c.recompute()
        rec_ms = sum(c.kernel_timing("inverse")[0] for c in crowds)
    for c in crowds:
        c.set_timing(())
    graph_s = None
    if graph_steps > 0:
        for c in crowds:
            c.run_vmc(1, wl.sigma)  # captures the graph
        for c in crowds:
            c.synchronize()
        g0 = time.perf_counter()
        for c in crowds:
            c.run_vmc(graph_steps, wl.sigma)
        for c in crowds:
            c.synchronize()
        graph_s = time.perf_counter() - g0
    for c in crowds:
        c.close()
    system.close()
    moves = wl.crowds * wl.walkers * wl.n_e * steps
    # whole-job time: the timed sweeps with exactly steps / recompute_every recomputes in them
    # (the recomputes that fell inside are taken out and the amortised share put in)
    seconds = t1 - t0
    if recompute > 0 and rec_ms is not None:
        seconds = seconds - 1e-3 * rec_ms_in + (steps / recompute) * 1e-3 * rec_ms
    out = dict(seconds=seconds, wall_seconds=t1 - t0, moves=moves, moves_per_s=moves / seconds,
               wall_moves_per_s=moves / (t1 - t0), kernels=kt, delay_rank=k_used, path=path_used, tiles=tiles_used,
               accepted_timed=acc - acc0, acceptance=acc / max(prop, 1), e_mean=float(el.mean()),
               finite=bool(np.isfinite(el).all()), recomputes_in_timed=n_rec, recompute_ms=rec_ms,
               recompute_ms_in_timed=rec_ms_in)
    if graph_s is not None:
        out["graph_moves_per_s"] = wl.crowds * wl.walkers * wl.n_e * graph_steps / graph_s
    return out


def rooflines(res, n, W, steps, traffic, s_c=4, s=4):
    """(spline roofline, update roofline) from one run's HIP-event kernel times.

    B-spline VGL of the round's proposals (k_prop_vgl_wave, or k_prop_vgl when N has fewer than
    64 orbital groups of 16 bytes): per proposal 64 stencil points x N
    orbitals read from the table and the 5 rows written; one launch = the round's proposals.
    Rank-k inverse update (k_flush_mfma_batch): per walker-spin window with r accepted moves it
    reads and writes the N x N inverse once and does 4 N^2 r useful flops; r summed over the run,
    divided by all of its launches (rounds where no walker has a move left included)."""
    vgl_ms, vgl_n = res["kernels"]["vgl"]
    sweep_path = res.get("path") == "sweep"  # one launch per sweep does the gather of every move
    props_per_launch = W * n * 2 * steps / max(vgl_n, 1)
    vgl_bytes = props_per_launch * (64 * n * s_c + 5 * n * s)
    vgl_t = vgl_ms / max(vgl_n, 1) * 1e-3
    vgl_gbs = vgl_bytes / vgl_t / 1e9
    up_ms, up_n = res["kernels"]["update"]
    up_t = up_ms / max(up_n, 1) * 1e-3
    r_per_launch = res["accepted_timed"] / max(up_n, 1)
    up_flops = 4.0 * n * n * r_per_launch
    traffic = traffic or {}
    roof_vgl = dict(bound="hbm", achieved=round(vgl_gbs, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(vgl_gbs / HBM_PEAK_GBS, 4), traffic=traffic.get("vgl"),
                    kernel="k_sweep" if sweep_path else ("k_prop_vgl_wave" if n * s_c // 16 >= 64 else "k_prop_vgl"),
                    us_per_launch=round(vgl_t * 1e6, 3), bytes_per_launch=int(vgl_bytes),
                    proposals_per_launch=int(props_per_launch))
    if up_n == 0:  # the whole-sweep path applies its updates inside k_sweep
        return roof_vgl, dict(bound="mfma", achieved=0.0, peak=FP32_PEAK_TFLOPS, unit="TFLOP/s", frac=0.0,
                              traffic=None, kernel="k_sweep", note="Sherman-Morrison updates inside k_sweep")
    roof_up = dict(bound="mfma", achieved=round(up_flops / up_t / 1e12, 2), peak=FP32_PEAK_TFLOPS,
                   unit="TFLOP/s", frac=round(up_flops / up_t / 1e12 / FP32_PEAK_TFLOPS, 4),
                   traffic=traffic.get("update"), kernel="k_flush_mfma_batch",
                   us_per_launch=round(up_t * 1e6, 3), accepted_per_launch=round(r_per_launch, 2))
    return roof_vgl, roof_up


def roofline_sm(res, n, s):
    """HBM roofline of the Sherman-Morrison update (k = 1, k_flush_vec): per accepted move one read
    and one write of the N x N inverse (2 N^2 s bytes), plus the move's value row and column read
    and its 5 orbital rows copied (12 N s); accepted moves of the timed sweeps over the launches."""
    ms, cnt = res["kernels"]["update"]
    t = ms / max(cnt, 1) * 1e-3
    acc_per_launch = res["accepted_timed"] / max(cnt, 1)
    byts = acc_per_launch * (2.0 * n * n * s + 12.0 * n * s)
    gbs = byts / t / 1e9
    return dict(bound="hbm", achieved=round(gbs, 1), peak=HBM_PEAK_GBS, unit="GB/s", frac=round(gbs / HBM_PEAK_GBS, 4),
                traffic=None, kernel="k_flush_vec (FP64, k = 1)", us_per_launch=round(t * 1e6, 3),
                accepted_per_launch=round(acc_per_launch, 2), bytes_per_launch=int(byts), launches=cnt)


def kernel_source_hash():
    """SHA-256 of the sources the gather and update kernels are built from."""
    import hashlib
    h = hashlib.sha256()
    for f in ("k_batch.hip", "k_flush_mfma.hip", "k_update.hip", "k_virtual.hip", "cq_device.h", "cq_internal.h",
              "cq_stencil.h", "cq_jastrow.h"):
        with open(os.path.join(ROOT, "paper_2209_14487_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload):
    """HBM bytes per launch of k_prop_vgl and of k_flush_mfma_batch ({"vgl": B, "update": B})
    from the committed counter summary, or None when the summary is missing or was taken on
    a different kernel source."""
    path = os.path.join(ROOT, "profiles", "k_prop_vgl_%s_traffic.json" % workload)
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("source_sha256") != kernel_source_hash():
        return None
    return dict(vgl=rec.get("traffic_bytes_per_launch"), update=(rec.get("update") or {}).get("traffic_bytes_per_launch"),
                sm=(rec.get("sm") or {}).get("traffic_bytes_per_launch"),
                virtual=(rec.get("virtual") or {}).get("traffic_bytes_per_launch"))


def host_cpu():
    """(threads the oracle may use, logical CPUs of the host, CPU model)."""
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    env = os.environ.get("OMP_NUM_THREADS", "")
    threads = min(avail, int(env)) if env.isdigit() and int(env) > 0 else avail
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return threads, os.cpu_count() or 1, model


def cpu_baseline(wl, moves_per_walker, cq=None, one_core_moves=1024):
    """The FP64 oracle (OpenMP over walkers, one walker per thread) on a bounded sample of the same
    workload, on every core this process may use, and on one core.  With the GPU library given, the
    same walkers also run on the GPU in mixed precision along the oracle's decisions, and the errors
    of the GPU's ratios, log|det| and local energies against the oracle are reported."""
    import oracle as orc
    from synth import J2_A_ANTI, J2_A_PAR, J2_B, start_positions
    threads, host_cpus, model = host_cpu()
    walkers = threads
    s = orc.System(wl.n, wl.n, wl.L, G=wl.G, n_orb=wl.n, orb_kind=orc.ORB_SEEDED, coef_seed=wl.seed,
                   coef_fp32=True, use_j2=wl.use_j2, j2_a_par=J2_A_PAR, j2_a_anti=J2_A_ANTI, j2_b=J2_B,
                   seed=wl.seed)
    R0 = start_positions(wl.seed, walkers, wl.n_e, wl.L)
    t0 = time.perf_counter()
    res = orc.vmc(s, R0, 1, sigma=wl.sigma, max_moves=moves_per_walker, n_threads=threads)
    t1 = time.perf_counter()
    # the walkers run side by side, one per thread: the slowest one's sweep time (its
    # set-up excluded, timed inside the oracle) is the time of the moves
    move_s = float(np.max(res.t_moves))
    out = dict(value=walkers * min(moves_per_walker, wl.n_e) / move_s, unit="moves/s", cores=threads, kind="oracle",
               sample="%d walkers x first %d electron moves of sweep 0 (%s), FP64 scalar C + OpenMP, "
                      "timed after each walker's set-up" % (walkers, min(moves_per_walker, wl.n_e), wl.name),
               seconds=round(t1 - t0, 1), move_seconds=round(move_s, 2), host_logical_cpus=host_cpus,
               cpu_model=model)
    if one_core_moves > 0:
        r1 = orc.vmc(s, R0[:1], 1, sigma=wl.sigma, max_moves=one_core_moves, n_threads=1)
        m1 = min(one_core_moves, wl.n_e)
        out["one_core"] = dict(value=round(m1 / float(r1.t_moves[0]), 1), unit="moves/s",
                               sample="walker 0, first %d moves of sweep 0, one thread" % m1)
    if cq is not None:
        out["errors_vs_oracle"] = gpu_errors(cq, wl, s, R0, res, min(moves_per_walker, wl.n_e))
    return out


def gpu_errors(cq, wl, o, R0, ref, moves):
    """Mixed-precision GPU chain of the sampled walkers along the oracle's decisions (forced-decision
    mode, the workload's delay rank and path): relative errors of the ratios against the FP64
    oracle, and of log|det| and E_L at the end of the sweep when the sample covers it."""
    from oracle import fp32_chain
    W = R0.shape[0]
    system = make_system(cq, wl, 4)
    c = cq.Crowd(system, W, precision="mixed", delay_rank=wl.delay_rank, recompute_every=wl.recompute_every,
                 seed=wl.seed, use_graph=False)
    c.set_positions(R0)
    forced = np.full((1, wl.n_e, W), 2, np.uint8)
    forced[0, :moves] = ref.acc[0, :moves]
    c.record(1)
    c.set_forced(forced)
    c.run_vmc(1, wl.sigma)
    rec = c.records()
    ld, _ = c.logdet()
    el = c.local_energy()
    c.close()
    system.close()
    st = fp32_chain.ratio_error_stats(rec["rho"][0, :moves], ref.rho[0, :moves])
    out = dict(walkers=W, moves_per_walker=moves, ratio_rel=dict((k, float("%.3g" % v)) for k, v in st.items()),
               note="mixed-precision GPU chain along the FP64 oracle's decisions; relative ratio errors over all "
                    "moves (max over |rho| >= 1e-3)")
    if moves == wl.n_e:
        lrel = np.abs(ld - ref.logdet[0]) / np.maximum(1.0, np.abs(ref.logdet[0]))
        erel = np.abs(el - ref.eloc[0]) / np.maximum(1.0, np.abs(ref.eloc[0]))
        out["logdet_rel_max"] = float("%.3g" % lrel.max())
        out["eloc_rel_median"] = float("%.3g" % np.median(erel))
        out["eloc_rel_max"] = float("%.3g" % erel.max())
        out["eloc_bias"] = float("%.3g" % np.mean(el - ref.eloc[0]))
    return out


def run_c5(cq, args):
    """C5: DMC (tau = 0.01) on three systems at once (S1/S2/S3: 32, 256, 1024 electrons per spin;
    target populations 2000, 500, 64), mixed precision, as ONE crowd of the three systems: per spin
    block and window step one launch of the move kernel serves the walkers of all three systems
    (largest first) and one launch their updates.  Compared with the same generations in FP64, one
    system after another (per-system launches), and with three mixed crowds on three streams
    driven by three host threads.  Moves per second over all systems (accepted + rejected
    drift-diffusion moves of the populations that moved)."""
    import threading
    from synth import WORKLOADS, start_positions
    systems = [WORKLOADS[k] for k in ("c5s1", "c5s2", "c5s3")]
    tau, warm, gens, k = 0.01, args.warmup, args.steps, 32

    # one crowd of three systems, mixed; FP64 recompute after every generation
    sys_m = [make_system(cq, wl, 4) for wl in systems]
    counts = [wl.walkers for wl in systems]
    grp = cq.Crowd(sys_m, counts, precision="mixed", delay_rank=k, recompute_every=1, seed=1005,
                   max_walkers=sum(4 * w + 64 for w in counts), path="window")
    grp.set_positions([start_positions(wl.seed, wl.walkers, wl.n_e, wl.L) for wl in systems])
    grp.run_vmc(4, 0.5)  # equilibrate in VMC before the first DMC generation
    el = grp.local_energy()
    offs = np.cumsum([0] + counts)
    e0 = [float(np.mean(el[offs[i]:offs[i + 1]])) for i in range(3)]
    targets = [wl.dmc_target for wl in systems]
    grp.run_dmc_systems(warm, tau, e_trial=e0, n_target=targets)
    grp.synchronize()
    m0 = grp.dmc_moves()[1]
    grp.set_timing(("vgl", "update"))
    t0 = time.perf_counter()
    h = grp.run_dmc_systems(gens, tau, n_target=targets)
    t1 = time.perf_counter()
    moves = grp.dmc_moves()[1] - m0
    kv, nv = grp.kernel_timing("vgl")
    ku, nu = grp.kernel_timing("update")
    grp.close()
    for s in sys_m:
        s.close()
    one = moves / (t1 - t0)
    log("  c5 mixed, one crowd of three systems: %.3e moves/s over %.2f s" % (one, t1 - t0))

    def separate(precision, concurrent):
        out = {"ready": threading.Barrier(3 if concurrent else 1)}

        def run(wl):
            s = make_system(cq, wl, 4 if precision == "mixed" else 8)
            c = cq.Crowd(s, wl.walkers, precision=precision, delay_rank=min(k, wl.n), seed=wl.seed,
                         max_walkers=4 * wl.walkers + 64, path="window",
                         recompute_every=1 if precision == "mixed" else 0)
            c.set_positions(start_positions(wl.seed, wl.walkers, wl.n_e, wl.L))
            c.run_vmc(4, wl.sigma)
            c.run_dmc(warm, tau, float(np.mean(c.local_energy())), n_target=wl.dmc_target)
            out["ready"].wait()
            m1 = c.dmc_moves()[1]
            a = time.perf_counter()
            c.run_dmc(gens, tau, float("nan"), n_target=wl.dmc_target)
            b = time.perf_counter()
            out[wl.name] = dict(seconds=b - a, moves=c.dmc_moves()[1] - m1, t0=a, t1=b)
            c.close()
            s.close()
        if concurrent:
            ths = [threading.Thread(target=run, args=(wl,)) for wl in systems]
            for t in ths:
                t.start()
            for t in ths:
                t.join()
        else:
            for wl in systems:
                run(wl)
        return {wl.name: out[wl.name] for wl in systems}

    f64 = separate("fp64", False)
    f64_rate = sum(v["moves"] for v in f64.values()) / sum(v["seconds"] for v in f64.values())
    log("  c5 fp64, per-system launches one system after another: %.3e moves/s" % f64_rate)
    three = separate("mixed", True)
    span = max(v["t1"] for v in three.values()) - min(v["t0"] for v in three.values())
    three_rate = sum(v["moves"] for v in three.values()) / span
    log("  c5 mixed, three crowds on three streams: %.3e moves/s" % three_rate)
    res = dict(metric="DMC electron moves/sec at 1 GPU, three systems in one crowd (mixed) vs per-system FP64",
               value=round(one, 1), unit="moves/s", n_gpus=1, steps=gens, warmup=warm,
               ms_per_step=round(1e3 * (t1 - t0) / max(gens, 1), 3), higher_is_better=True, scaling="weak",
               vs_baseline=None, dtype="f32", data="synthetic (seeded Philox B-spline coefficients, uniform starts)",
               config=dict(workload="c5: DMC tau=0.01, S1 32+32 e L=10 G=48 target 2000, S2 256+256 e L=20 G=64 "
                                    "target 500, S3 1024+1024 e L=32 G=96 target 64; mixed with an FP64 recompute "
                                    "after every generation; one crowd of the three systems, delayed rank 32, "
                                    "one move launch and one update launch per window step for all systems"),
               populations=[[int(x) for x in h[:, i, 0]] for i in range(3)],
               e_t=[float(h[-1, i, 3]) for i in range(3)],
               kernels=dict(vgl=dict(ms_total=round(kv, 3), launches=nv), update=dict(ms_total=round(ku, 3), launches=nu)),
               fp64_per_system_moves_per_s=round(f64_rate, 1),
               mixed_one_crowd_over_fp64_per_system=round(one / f64_rate, 3),
               mixed_three_crowds_three_streams_moves_per_s=round(three_rate, 1))
    print(json.dumps(res), flush=True)


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the walker-parallel path is not sharded across GPUs "
              "(walkers are independent; each GPU would run its own crowds on its own copy of the "
              "orbital table, with a few FP64 sums all-reduced per generation).",
              file=sys.stderr)
        sys.exit(2)
    import paper_2209_14487_amd as cq
    from synth import WORKLOADS
    if args.workload == "c5":
        run_c5(cq, args)
        return
    if args.workload == "c6":
        run_complex(cq, args)
        return
    if args.workload == "inverse":
        run_inverse(cq, args)
        return
    if args.scan:
        run_scan(cq, args)
        return
    wl = WORKLOADS[args.workload]
    delay = args.delay if args.delay is not None else wl.delay_rank
    log("workload %s: N=%d per spin, W=%d x %d crowd(s), G=%d, k=%d, recompute every %d"
        % (wl.name, wl.n, wl.walkers, wl.crowds, wl.G, delay, wl.recompute_every))

    if args.calibrate_copy:
        src = cq.DeviceArray(np.ones(1 << 30, np.uint8))
        dst = cq.DeviceArray(shape=(1 << 30,), dtype=np.uint8)
        cq.device_copy(dst.ptr, src.ptr, 1 << 30)
        src.free()
        dst.free()
        log("  copied 1 GiB with cq_device_copy (calibration)")
    kinds = [k for k in args.time_kernels.split(",") if k]
    # the rooflines need the gather and the update; the recompute's device time is taken out
    # of the timed sweeps and its amortised share put back (events only on recompute launches)
    for k in ("vgl", "update", "inverse"):
        if k not in kinds:
            kinds.append(k)
    tiles = tuple(int(x) for x in args.tiles.split(",")) if args.tiles else None
    mixed = run_gpu(cq, wl, "mixed", delay, wl.recompute_every, args.steps, args.warmup, kinds, not args.eager,
                    path=args.path, graph_steps=0 if args.eager else max(2, args.steps // 4), tiles=tiles,
                    tile_cache=args.tile_cache or None)
    log("  mixed: %.3f s for %d sweeps (%.3f s wall, %d recompute(s) inside), %.3e moves/s, acceptance %.3f"
        % (mixed["seconds"], args.steps, mixed["wall_seconds"], mixed["recomputes_in_timed"],
           mixed["moves_per_s"], mixed["acceptance"]))

    n, W = wl.n, wl.walkers * wl.crowds
    kinfo = {}
    for k, (ms, cnt) in mixed["kernels"].items():
        kinfo[k] = dict(ms_total=round(ms, 3), launches=cnt, us_per_launch=round(1e3 * ms / max(cnt, 1), 3),
                        share=round(ms / (1e3 * mixed["seconds"]), 4))
    if delay == 0:
        delay = mixed["delay_rank"]
        log("  autotuned delay rank: %d" % delay)
    windows_per_sweep = 2 * ((n + delay - 1) // delay)
    traffic = measured_traffic(wl.name)
    roof_vgl, roof_up = rooflines(mixed, n, W, args.steps, traffic)
    vgl_ms, up_ms = mixed["kernels"]["vgl"][0], mixed["kernels"]["update"][0]
    dominant = roof_vgl if vgl_ms >= up_ms else roof_up
    out = dict(metric=METRIC, value=round(mixed["moves_per_s"], 1), unit="moves/s", n_gpus=1, steps=args.steps,
               warmup=args.warmup, ms_per_step=round(1e3 * mixed["seconds"] / args.steps, 3),
               higher_is_better=True, scaling="weak", vs_baseline=None, dtype="f32",
               data="synthetic (seeded Philox B-spline coefficients, uniform starting positions)",
               config=dict(workload="%s: %d+%d electrons, L=%g bohr, %d^3 FP32 B-spline table (%.2f GB), Pade J2, "
                                    "%d crowd(s) x %d walkers, delayed rank %d, FP64 recompute every %d sweeps"
                                    % (wl.name, n, n, wl.L, wl.G, wl.table_bytes(4) / 1e9, wl.crowds, wl.walkers,
                                       delay, wl.recompute_every),
                           precision="mixed", path=mixed["path"], tiles=mixed["tiles"],
                           launch="eager launches; HIP events around every launch of %s in the timed region" % "/".join(kinds)),
               roofline=dominant, roofline_spline=roof_vgl, roofline_update=roof_up, kernels=kinfo,
               windows_per_sweep=windows_per_sweep,
               acceptance=round(mixed["acceptance"], 4), e_mean=mixed["e_mean"],
               recompute=dict(every=wl.recompute_every, ms_per_recompute=mixed["recompute_ms"] and round(mixed["recompute_ms"], 3),
                              in_timed_region=mixed["recomputes_in_timed"],
                              ms_in_timed_region=round(mixed["recompute_ms_in_timed"], 3),
                              wall_seconds_timed=round(mixed["wall_seconds"], 4),
                              wall_moves_per_s=round(mixed["wall_moves_per_s"], 1),
                              note="value and ms_per_step count steps/every recomputes of the whole crowd: the "
                                   "device time of the recomputes that fell inside the timed sweeps is replaced "
                                   "by that share of one timed recompute"))
    if "graph_moves_per_s" in mixed:
        out["graph_moves_per_s"] = round(mixed["graph_moves_per_s"], 1)
    if args.alone_steps > 0 and mixed["path"] == "batch":
        # the same kernels with the GPU to themselves: one stream, every kernel in order
        alone = run_gpu(cq, wl, "mixed", delay, 0, args.alone_steps, 1, ["vgl", "update"], False,
                        path=args.path, streams=1, tiles=(mixed["tiles"]["candidates"], 0))
        a_vgl, a_up = rooflines(alone, n, W, args.alone_steps, None)
        log("  alone: k_prop_vgl %.0f GB/s, update %.1f TFLOP/s" % (a_vgl["achieved"], a_up["achieved"]))
        out["alone"] = dict(moves_per_s=round(alone["moves_per_s"], 1), steps=args.alone_steps,
                            roofline_spline=a_vgl, roofline_update=a_up,
                            note="one stream, no kernel beside another; context for the roofline above, "
                                 "which is measured in the timed region where gather and update share the GPU")
    if args.fp64_steps > 0:
        f64 = run_gpu(cq, wl, "fp64", delay, 0, args.fp64_steps, 1, [], not args.eager, path=args.path, tiles=tiles)
        log("  fp64: %.3e moves/s" % f64["moves_per_s"])
        out["fp64_moves_per_s"] = round(f64["moves_per_s"], 1)
        out["fp64_tiles"] = f64["tiles"]
        # both sides replay the captured sweep graph (no events), so launch overheads match
        ref = mixed.get("graph_moves_per_s", mixed["moves_per_s"])
        out["mixed_over_fp64"] = round(ref / f64["moves_per_s"], 3)
    if args.sm_steps > 0 and mixed["path"] == "batch":
        # Sherman-Morrison (k = 1) in FP64: the wave-reduced dot products and rank-1 update of
        # k_flush_vec, judged by HBM GB/s
        sm = run_gpu(cq, wl, "fp64", 1, 0, args.sm_steps, 0, ["update"], False, path=args.path)
        out["roofline_sm"] = roofline_sm(sm, n, 8)
        out["roofline_sm"]["traffic"] = (traffic or {}).get("sm")
        log("  SM update (FP64, k = 1): %.0f GB/s" % out["roofline_sm"]["achieved"])
    if args.virtual_points > 0:
        out["roofline_virtual"] = run_virtual(cq, wl, args.virtual_points)
        out["roofline_virtual"]["traffic"] = (traffic or {}).get("virtual")
        log("  virtual moves: %.0f GB/s (algorithmic), %.3e points/s" % (out["roofline_virtual"]["achieved"],
                                                                        out["roofline_virtual"]["points_per_s"]))
    if not args.no_cpu:
        log("  cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_moves, cq, args.cpu_one_core_moves)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
