"""GPU parity of the batched particle-by-particle VMC move against the FP64 CPU oracle.

Every test calls the HIP library through the C ABI (paper_2209_14487_amd) and
compares with ``oracle`` on the same seeded inputs and random streams.

Tolerances: FP64 path, ratios / log|det| / E_L within 1e-10 relative and identical
accept/reject decisions except at near-ties |P - u| < 1e-6.  Mixed path (FP32
table, FP32 inverse), run in forced-decision mode on the oracle's trajectory: the
relative ratio errors against the FP64 oracle are compared with those of the
rounding model ``oracle.fp32_chain`` replaying the same walkers along the same
decisions with the inverse and the orbital rows stored in FP32 and the updates applied
as the path applies them (delayed rank-k windows in FP32, FP64 sums of the ratio
products, the same recompute schedule).  The
model's errors are what an FP32 inverse costs on these matrices (at N = 1024,
cond(A) ~ 1e4, they exceed 1e-4 for a few percent of the moves whatever the
kernels do); the GPU's median and 99th percentile must stay within twice the
model's, its 99.9th percentile and maximum within three times.  The percentiles are
over every move; the maximum is over moves with |rho| >= 0.1: the relative error of a
dot product is bounded by its condition number sum_j |u_j c_j| / |rho|, which grows
without bound as rho -> 0, so below that floor the largest error of one chain says
nothing about another chain that groups its sums differently (the GPU's rank-k
updates against the model's rank-1 steps).
log|det| within 1e-4 of max(1, |log|det||).
"""
import json

import numpy as np
import pytest

import oracle as orc
import paper_2209_14487_amd as cq
from oracle import fp32_chain
from synth import J2_A_ANTI, J2_A_PAR, J2_B, planewave_table, start_positions

pytestmark = pytest.mark.gpu

NEAR_TIE = 1e-6


def make_pair(n, L, G, move_seed, table=None, coef_seed=None, j2=True, fp64=True, fp32=False):
    """The same system on both sides: GPU cq.System and oracle System."""
    g = cq.System(n, L)
    if table is not None:
        if fp64:
            g.load_table(np.asarray(table, np.float64))
        if fp32:
            g.load_table(np.asarray(table, np.float32))
        o = orc.System(n, n, L, G=G, n_orb=n, orb_kind=orc.ORB_TABLE, table=table, use_j2=j2, seed=move_seed)
    else:
        if fp64:
            g.fill_philox(coef_seed, 8, G)
        if fp32:
            g.fill_philox(coef_seed, 4, G)
        o = orc.System(n, n, L, G=G, n_orb=n, orb_kind=orc.ORB_SEEDED, coef_seed=coef_seed, use_j2=j2,
                       seed=move_seed)
    if j2:
        g.load_j2(J2_A_PAR, J2_A_ANTI, J2_B)
        o.j2_a_par, o.j2_a_anti, o.j2_b = J2_A_PAR, J2_A_ANTI, J2_B
    return g, o


def run_gpu(crowd, R0, sweeps, sigma, first_step=0, forced=None):
    crowd.set_positions(R0, first_step)
    crowd.record(sweeps)
    if forced is not None:
        crowd.set_forced(forced)
    ld = np.zeros((sweeps, crowd.W, 2))
    sg = np.zeros((sweeps, crowd.W, 2), np.int32)
    el = np.zeros((sweeps, crowd.W))
    for s in range(sweeps):
        crowd.run_vmc(1, sigma)
        ld[s], sg[s] = crowd.logdet()
        el[s] = crowd.local_energy()
    rec = crowd.records()
    rec.update(logdet=ld, sign=sg, eloc=el, R=crowd.positions())
    return rec


# GPU statistic <= factor x the same statistic of the FP32 rounding model
EMU_FACTOR = dict(median=2.0, p99=2.0, p999=3.0, max=3.0)
MAX_FLOOR = 0.1  # the maximum is taken over moves with |rho| >= this


def emulated_rho(o, R0, acc, uids=None, n_moves=None, recompute_every=0, sigma=0.5, k=1, path="batch"):
    """Ratios of the FP32 rounding model for walkers R0 along decisions acc [S][Ne][W], with the
    coefficient table rounded to FP32 as the mixed path stores it and the updates applied as
    the path applies them: windows of k accepted moves (batched path) or of k proposals."""
    import dataclasses
    o = dataclasses.replace(o, coef_fp32=True)
    W = R0.shape[0]
    uids = range(W) if uids is None else uids
    close = "accepts" if path == "batch" else "proposals"
    # the whole-sweep path applies each accepted move at once (Sherman-Morrison in FP64 from
    # the FP32-stored values, stored back in FP32)
    window, arith = (0, "fp64") if path == "sweep" else (k, "fp32")
    return np.stack([fp32_chain.replay(o, R0[i], int(u), acc[:, :, i], n_moves=n_moves, sigma=sigma,
                                       recompute_every=recompute_every, window=window, close_after=close,
                                       arith=arith)
                     for i, u in enumerate(uids)], axis=-1)


def mixed_ratio_check(gpu_rho, ref_rho, emu_rho, label):
    """GPU ratio errors against the FP64 oracle, bounded by the rounding model's on the same moves."""
    g = fp32_chain.ratio_error_stats(gpu_rho, ref_rho, floor=MAX_FLOOR)
    e = fp32_chain.ratio_error_stats(emu_rho, ref_rho, floor=MAX_FLOOR)
    print("%s: ratio rel err GPU %s | FP32 model %s" % (
        label, " ".join("%s=%.2e" % (k, g[k]) for k in EMU_FACTOR), " ".join("%s=%.2e" % (k, e[k]) for k in EMU_FACTOR)))
    assert g["n"] == e["n"]
    for k, f in EMU_FACTOR.items():
        assert g[k] <= f * e[k], (k, g, e)
    return g, e


def own_decision_check(gpu_prob, ref_prob, ref_u, ref_acc, emu_stats, max_frac):
    """The GPU's own decisions (P_gpu > u) differ from the oracle's only where |P - u| / P lies
    within twice the ratio-error bound (P carries rho squared), and rarely."""
    own = gpu_prob > ref_u
    mism = own != ref_acc.astype(bool)
    gap = np.abs(ref_prob[mism] - ref_u[mism]) / np.maximum(ref_prob[mism], 1e-300)
    lim = 2.0 * EMU_FACTOR["max"] * emu_stats["max"] + 1e-6
    print("   own decisions differing: %d of %d, max |P-u|/P there %.2e (bound %.2e)"
          % (mism.sum(), mism.size, gap.max() if mism.any() else 0.0, lim))
    assert mism.sum() <= max_frac * mism.size
    assert np.all(gap <= lim)


def first_divergence(acc_a, acc_b):
    """Per walker: flat (sweep, electron) index of the first differing decision, or None."""
    S, ne, W = acc_a.shape
    out = []
    for w in range(W):
        d = np.nonzero(acc_a[:, :, w].ravel() != acc_b[:, :, w].ravel())[0]
        out.append(int(d[0]) if len(d) else None)
    return out


def compare_fp64(gpu, ref, sweeps, ne, tol=1e-10):
    div = first_divergence(gpu["acc"], ref.acc)
    W = len(div)
    n_div = 0
    for w, d in enumerate(div):
        lim = sweeps * ne if d is None else d
        if d is not None:
            n_div += 1
            s, e = divmod(d, ne)
            assert abs(ref.prob[s, e, w] - ref.u[s, e, w]) < NEAR_TIE, "decision differs away from a near-tie"
        for key in ("rho", "dlnj", "prob"):
            a = gpu[key][:, :, w].ravel()[:lim]
            b = getattr(ref, key)[:, :, w].ravel()[:lim]
            assert np.all(np.abs(a - b) <= tol * np.maximum(1.0, np.abs(b))), key
        full = lim // ne  # sweeps completed before any divergence
        if full:
            a, b = gpu["logdet"][:full, w], ref.logdet[:full, w]
            assert np.all(np.abs(a - b) <= tol * np.maximum(1.0, np.abs(b)))
            assert np.array_equal(gpu["sign"][:full, w], ref.sign[:full, w])
            a, b = gpu["eloc"][:full, w], ref.eloc[:full, w]
            assert np.all(np.abs(a - b) <= tol * np.maximum(1.0, np.abs(b)))
    assert n_div <= max(1, W // 20)
    return div


PATHS = ["multi", "window", "batch"]
ALL_PATHS = PATHS + ["sweep"]  # the whole-sweep path runs delay rank 1 only


def rank_for(path, k):
    return 1 if path == "sweep" else k


@pytest.mark.parametrize("path", ALL_PATHS)
def test_c1_fp64_sherman_morrison_matches_oracle(path):
    """C1: 4+4 electrons, L=5, 16^3 plane-wave spline, 16 walkers, 200 sweeps, FP64, SM."""
    n, L, G, W, S = 4, 5.0, 16, 16, 200
    g, o = make_pair(n, L, G, 1001, table=planewave_table(G, L), j2=False)
    R0 = start_positions(1001, W, 2 * n, L)
    crowd = cq.Crowd(g, W, precision="fp64", delay_rank=1, seed=1001, path=path)
    gpu = run_gpu(crowd, R0, S, 0.5)
    ref = orc.vmc(o, R0, S, sigma=0.5)
    div = compare_fp64(gpu, ref, S, 2 * n)
    # E_L equals 12 pi^2 / 25 up to the O(h^2) spline error (about 1 % at G = 16)
    e0 = 12 * np.pi ** 2 / 25
    assert np.all(np.abs(gpu["eloc"] / e0 - 1) < 0.05)
    assert 0.2 < gpu["acc"].mean() < 0.95
    if all(d is None for d in div):
        assert np.allclose(gpu["R"], ref.R, atol=1e-12)
    crowd.close()


@pytest.mark.parametrize("k,path", [(k, p) for p in PATHS for k in (1, 4, 8, 32)] + [(1, "sweep")])
def test_c2_shape_fp64_delayed_ranks_match_oracle(k, path):
    """C2 shapes (32+32, L=10, 48^3 seeded table, Pade J2) on 61 walkers (ragged against the
    8-XCD mapping): Sherman-Morrison and rank-k delayed updates reproduce the oracle chain."""
    n, L, G, W, S = 32, 10.0, 48, 61, 4
    g, o = make_pair(n, L, G, 1002, coef_seed=1002)
    R0 = start_positions(1002, W, 2 * n, L)
    crowd = cq.Crowd(g, W, precision="fp64", delay_rank=k, seed=1002, path=path)
    gpu = run_gpu(crowd, R0, S, 0.5)
    ref = orc.vmc(o, R0, S, sigma=0.5, want_ainv=True)
    div = compare_fp64(gpu, ref, S, 2 * n)
    ok = [w for w, d in enumerate(div) if d is None]
    inv = crowd.inverse()
    for w in ok:
        assert np.abs(inv[w] - ref.ainv[w]).max() <= 1e-9 * np.abs(ref.ainv[w]).max()
    crowd.close()


@pytest.mark.parametrize("k,recompute,path", [(1, 2, "window"), (8, 2, "window"), (32, 0, "window"),
                                              (8, 2, "multi"), (1, 2, "batch"), (8, 2, "batch"),
                                              (32, 0, "batch"), (1, 2, "sweep"), (1, 0, "sweep")])
def test_c2_mixed_precision_on_oracle_trajectory(k, recompute, path):
    """C2 mixed precision (FP32 table, FP32 inverse and dots, FP64 log|det| and sums) follows
    the oracle's decisions; its own ratios stay within 1e-4 relative of the FP64 oracle, its
    own decisions differ only where |P - u| is within that error, and log|det| stays within
    1e-4 of max(1, |log|det||) across periodic FP64 recomputes."""
    n, L, G, W, S = 32, 10.0, 48, 40, 6
    g, o = make_pair(n, L, G, 1002, coef_seed=1002, fp64=False, fp32=True)
    R0 = start_positions(1002, W, 2 * n, L)
    ref = orc.vmc(o, R0, S, sigma=0.5)
    crowd = cq.Crowd(g, W, precision="mixed", delay_rank=k, recompute_every=recompute, seed=1002, path=path)
    gpu = run_gpu(crowd, R0, S, 0.5, forced=ref.acc)
    emu = emulated_rho(o, R0, ref.acc, recompute_every=recompute, k=k, path=path)
    _, es = mixed_ratio_check(gpu["rho"], ref.rho, emu, "C2 mixed k=%d recompute=%d %s" % (k, recompute, path))
    own_decision_check(gpu["prob"], ref.prob, ref.u, ref.acc, es, 1e-3)
    err = np.abs(gpu["logdet"] - ref.logdet) / np.maximum(1.0, np.abs(ref.logdet))
    eerr = np.abs(gpu["eloc"] - ref.eloc) / np.maximum(1.0, np.abs(ref.eloc))
    print("   log|det| max err %.2e, E_L max rel err %.2e (median %.2e)" % (err.max(), eerr.max(), np.median(eerr)))
    assert err.max() < 1e-4, err.max()
    assert np.array_equal(gpu["sign"], ref.sign)
    assert np.median(eerr) < 1e-5 and eerr.max() < 1e-2
    assert np.allclose(gpu["R"], ref.R, atol=1e-12)
    crowd.close()


@pytest.mark.parametrize("path", ALL_PATHS)
def test_crowd_partition_is_bit_identical(path):
    """Splitting the walkers into crowds changes nothing (paper Sec. III: crowd size 1 is the
    per-walker driver, one crowd is the whole-population batch): FP64 results per walker are
    bit-identical for 1 x 24, 8 + 16 and 24 x 1 walkers."""
    n, L, G, W, S = 32, 10.0, 48, 24, 2
    g, _ = make_pair(n, L, G, 7, coef_seed=1002)
    R0 = start_positions(1002, W, 2 * n, L)

    def run(parts):
        out_R, out_ld, out_el = [], [], []
        lo = 0
        for p in parts:
            c = cq.Crowd(g, p, precision="fp64", delay_rank=rank_for(path, 4), seed=7, first_uid=lo, path=path)
            c.set_positions(R0[lo:lo + p])
            c.run_vmc(S, 0.5)
            out_R.append(c.positions())
            out_ld.append(c.logdet()[0])
            out_el.append(c.local_energy())
            c.close()
            lo += p
        return np.concatenate(out_R), np.concatenate(out_ld), np.concatenate(out_el)

    a = run([24])
    b = run([8, 16])
    c = run([1] * 24)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    for x, y in zip(a, c):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("path", ALL_PATHS)
def test_graph_replay_equals_eager_launches(path):
    """The sweep captured once as a hipGraph and replayed gives the eager result bit for bit."""
    n, L, G, W, S = 32, 10.0, 48, 16, 3
    g, _ = make_pair(n, L, G, 9, coef_seed=1002, fp64=False, fp32=True)
    R0 = start_positions(1002, W, 2 * n, L)
    res = []
    for use_graph in (False, True):
        c = cq.Crowd(g, W, precision="mixed", delay_rank=rank_for(path, 8), recompute_every=2, seed=9,
                     use_graph=use_graph, path=path)
        c.set_positions(R0)
        for _ in range(S):
            c.run_vmc(1, 0.5)
            c.synchronize()
        res.append((c.positions(), c.logdet()[0], c.local_energy(), c.acceptance()[0]))
        c.close()
    for x, y in zip(*res):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("precision,k,path", [("fp64", 1, "multi"), ("fp64", 16, "multi"), ("mixed", 32, "multi"),
                                              ("fp64", 16, "window"), ("mixed", 32, "window"),
                                              ("fp64", 1, "batch"), ("fp64", 32, "batch"), ("mixed", 32, "batch")])
def test_n256_blocked_inverse_and_multichunk_sweep(precision, k, path):
    """C3 system size (256+256, L=20, 64^3): blocked FP64 Gauss-Jordan set-up, multi-workgroup
    orbital chunks and one full sweep, on 3 walkers."""
    n, L, G, W, S = 256, 20.0, 64, 3, 1
    g, o = make_pair(n, L, G, 1003, coef_seed=1003, fp64=precision == "fp64", fp32=precision == "mixed")
    R0 = start_positions(1003, W, 2 * n, L)
    ld0, sg0, el0, ai0 = orc.setup(o, R0)
    crowd = cq.Crowd(g, W, precision=precision, delay_rank=k, seed=1003, path=path)
    crowd.set_positions(R0)
    ld, sg = crowd.logdet()
    tol = 1e-10 if precision == "fp64" else 1e-4
    assert np.all(np.abs(ld - ld0) <= tol * np.maximum(1, np.abs(ld0)))
    assert np.array_equal(sg, sg0)
    inv = crowd.inverse()
    itol = 1e-9 if precision == "fp64" else 2e-3
    for w in range(W):
        assert np.abs(inv[w] - ai0[w]).max() <= itol * np.abs(ai0[w]).max()
    el = crowd.local_energy()
    assert np.all(np.abs(el - el0) <= (1e-9 if precision == "fp64" else 1e-3) * np.maximum(1, np.abs(el0)))
    ref = orc.vmc(o, R0, S, sigma=0.5)
    if precision == "fp64":
        gpu = run_gpu(crowd, R0, S, 0.5)
        compare_fp64(gpu, ref, S, 2 * n)
    else:
        gpu = run_gpu(crowd, R0, S, 0.5, forced=ref.acc)
        mixed_ratio_check(gpu["rho"], ref.rho, emulated_rho(o, R0, ref.acc, k=k, path=path),
                          "N=256 mixed k=%d %s" % (k, path))
    crowd.close()


@pytest.mark.parametrize("sigma,k", [(0.01, 8), (0.01, 32), (0.5, 16)])
def test_batch_rounds_at_extreme_acceptance(sigma, k):
    """Batched path at high acceptance (0.9 at sigma = 0.01: every round closes its window after
    exactly k accepted moves, so a spin block needs nearly all of its N / k rounds) and with
    windows cut short (k = 16 at 0.43 acceptance: the 32 candidates of a spin block run out
    before 16 are accepted): FP64 against the oracle, all decisions, ratios and energies."""
    n, L, G, W, S = 32, 10.0, 48, 24, 2
    g, o = make_pair(n, L, G, 1002, coef_seed=1002)
    R0 = start_positions(1002, W, 2 * n, L)
    crowd = cq.Crowd(g, W, precision="fp64", delay_rank=k, seed=1002, path="batch")
    gpu = run_gpu(crowd, R0, S, sigma)
    ref = orc.vmc(o, R0, S, sigma=sigma)
    compare_fp64(gpu, ref, S, 2 * n)
    acc = gpu["acc"].mean()
    print("   sigma %.2f k %d: acceptance %.3f" % (sigma, k, acc))
    assert (acc > 0.85) if sigma < 0.1 else (acc < 0.6)
    crowd.close()


@pytest.mark.parametrize("precision,n,L,G,W,S,k,plan", [("fp64", 32, 10.0, 48, 24, 3, 8, 1),
                                                         ("fp64", 32, 10.0, 48, 24, 3, 4, 3),
                                                         ("mixed", 32, 10.0, 48, 24, 3, 8, 1),
                                                         ("fp64", 256, 20.0, 64, 3, 1, 32, 1)])
def test_round_plan_tail_kernel_keeps_the_chain(precision, n, L, G, W, S, k, plan):
    """Batched path with fewer rounds per spin block than the walkers need (a fixed plan):
    the tail kernel moves every electron left, one move at a time, and the chain is the
    oracle's (FP64: ratios, log|det|, E_L within the parity bar, decisions except near-ties;
    mixed: on the oracle's trajectory within the FP32 rounding model)."""
    fp32 = precision == "mixed"
    g, o = make_pair(n, L, G, 1006, coef_seed=1006, fp64=not fp32, fp32=fp32)
    R0 = start_positions(1006, W, 2 * n, L)
    ref = orc.vmc(o, R0, S, sigma=0.5)
    crowd = cq.Crowd(g, W, precision=precision, delay_rank=k, recompute_every=2 if fp32 else 0, seed=1006,
                     path="batch")
    crowd.set_round_plan(plan)
    assert list(crowd.round_plan()) == [plan, plan]
    if fp32:
        gpu = run_gpu(crowd, R0, S, 0.5, forced=ref.acc)
        emu = emulated_rho(o, R0, ref.acc, recompute_every=2, k=k, path="batch")
        mixed_ratio_check(gpu["rho"], ref.rho, emu, "tail kernel mixed k=%d plan=%d" % (k, plan))
    elif S == 1 and n >= 256:
        # about a hundred Sherman-Morrison steps per spin block on each side (the oracle's and
        # the tail kernel's): the arbiter decides where the two chains have drifted apart
        gpu = run_gpu(crowd, R0, S, 0.5)
        arbitrated_fp64_check(gpu, ref, o, R0, range(W), range(W), 2 * n)
    else:
        gpu = run_gpu(crowd, R0, S, 0.5)
        compare_fp64(gpu, ref, S, 2 * n)
    crowd.close()


def test_round_plan_is_learned_and_keeps_the_chain():
    """The default plan: the first sweep runs all N / k rounds of each spin block, later ones
    as many as were needed plus a margin (fewer than N / k at this acceptance: 64 electrons per
    spin at k = 4 take about 8 of the 16 rounds); the chain over those sweeps is the oracle's."""
    n, L, G, W, S, k = 64, 12.0, 48, 16, 5, 4
    g, o = make_pair(n, L, G, 1007, coef_seed=1007)
    R0 = start_positions(1007, W, 2 * n, L)
    crowd = cq.Crowd(g, W, precision="fp64", delay_rank=k, seed=1007, path="batch")
    assert list(crowd.round_plan()) == [n // k, n // k]
    gpu = run_gpu(crowd, R0, S, 0.5)
    plan = crowd.round_plan()
    print("   learned plan", plan.tolist(), "of", n // k)
    assert np.all(plan < n // k) and np.all(plan >= 1)
    ref = orc.vmc(o, R0, S, sigma=0.5)
    # five sweeps of rank-4 and Sherman-Morrison steps on both sides: the arbiter decides where the
    # two FP64 chains have drifted apart by more than the parity bar
    arbitrated_fp64_check(gpu, ref, o, R0, range(W), range(W), S * 2 * n)
    crowd.close()



def test_round_plan_of_each_spin_comes_from_its_own_report():
    """Each spin block's plan is learned from that block's own report: a report of the up block
    alone never sets the down block's plan (which once read the down block's empty fields and
    planned 2 rounds, leaving most of that block to the tail kernel).  After a few sweeps both
    plans cover the rounds the blocks need (about half of N / k at this acceptance), and new
    launch shapes restart the plan."""
    n, L, G, W, k = 64, 12.0, 48, 16, 4
    g, _ = make_pair(n, L, G, 1012, coef_seed=1012)
    R0 = start_positions(1012, W, 2 * n, L)
    crowd = cq.Crowd(g, W, precision="fp64", delay_rank=k, seed=1012, path="batch")
    crowd.set_positions(R0)
    for _ in range(4):
        crowd.run_vmc(1, 0.5)
    crowd.synchronize()
    plan = crowd.round_plan()
    print("   plan", plan.tolist(), "of", n // k)
    assert np.all(plan >= 6) and np.all(plan <= n // k)
    crowd.set_tiles(candidates=8)
    assert list(crowd.round_plan()) == [n // k, n // k]
    crowd.run_vmc(3, 0.5)
    crowd.synchronize()
    plan = crowd.round_plan()
    assert np.all(plan >= 6) and np.all(plan <= n // k)
    crowd.close()
    g.close()

def test_singular_start_is_reported():
    """Two same-spin electrons at one position make A singular: CQ_ESINGULAR names the walker."""
    n, L, G, W = 4, 5.0, 16, 3
    g, _ = make_pair(n, L, G, 1, table=planewave_table(G, L), j2=False)
    R0 = start_positions(1001, W, 2 * n, L)
    R0[1, 2] = R0[1, 0]
    crowd = cq.Crowd(g, W, precision="fp64", seed=1)
    with pytest.raises(cq.CqError) as ei:
        crowd.set_positions(R0)
    assert ei.value.status == cq.CQ_ESINGULAR
    assert "walker 1" in str(ei.value)
    with pytest.raises(cq.CqError) as ei:
        crowd.run_vmc(1, 0.5)
    assert ei.value.status == cq.CQ_ESTATE
    crowd.close()


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_recompute_reports_the_drift_of_the_kept_log_det(precision):
    """cq_crowd_recompute's max_drift and cq_crowd_get_drift's per-walker record are
    |log|det| kept by the update chain - log|det| of the fresh inversion| (the drift the
    periodic FP64 recompute removes).  The fresh value is pinned to the oracle's LU of the
    orbital rows at the crowd's final positions (FP32-evaluated rows in mixed precision, as
    the path stores them), and the kept value is the chain's: so the drift is that of the
    chain, about 1e-6..1e-4 in mixed precision and at rounding level in FP64."""
    n, L, G, W, S, seed = 32, 10.0, 48, 16, 6, 1002
    fp32 = precision == "mixed"
    g, o = make_pair(n, L, G, seed, coef_seed=seed, fp64=not fp32, fp32=fp32)
    crowd = cq.Crowd(g, W, precision=precision, delay_rank=8, recompute_every=0, seed=seed, path="batch")
    crowd.set_positions(start_positions(seed, W, 2 * n, L))
    crowd.run_vmc(S, 0.5)
    kept, _ = crowd.logdet()
    R = crowd.positions()
    max_drift = crowd.recompute()
    fresh, _ = crowd.logdet()
    last, m, k = crowd.drift()
    crowd.close()
    g.close()
    vgl = orc.orbital_vgl_f32 if fp32 else orc.orbital_vgl
    ref = np.zeros((W, 2))
    for w in range(W):
        for s in range(2):
            A = np.array([vgl(o, R[w, s * n + i], n)[0] for i in range(n)])
            ref[w, s] = orc.lu_inverse(A)[1]
    # the fresh log|det| is the oracle's: FP64 inversion of the same rows (in mixed precision the
    # GPU's FP32 rows sum the 64 stencil terms in another order than the oracle's FP32 model, and
    # those last-bit differences move log|det| by up to a few 1e-6: the mixed log|det| bar)
    tol = 1e-4 if fp32 else 1e-10
    assert np.all(np.abs(fresh - ref) <= tol * np.maximum(1.0, np.abs(ref)))
    drift = np.abs(kept - fresh)
    assert np.allclose(last, drift, rtol=0, atol=1e-15)
    assert max_drift == pytest.approx(drift.max(), rel=0, abs=1e-15)
    assert m == pytest.approx(drift.max(), rel=0, abs=1e-15) and k == 1
    if fp32:
        assert 1e-8 < drift.max() < 1e-3
    else:
        assert drift.max() < 1e-10


@pytest.mark.parametrize("precision,n,L,G,W,S", [("fp64", 4, 5.0, 16, 9, 3), ("mixed", 8, 6.0, 24, 9, 3),
                                                  ("fp64", 64, 12.0, 48, 5, 2), ("mixed", 64, 12.0, 48, 5, 2)])
def test_sweep_path_sizes(precision, n, L, G, W, S):
    """Whole-sweep path at its edges: one orbital group (N = 4 FP64, N = 8 FP32: a quad of
    lanes per group), and the largest N = 64 (both inverses fill 64 KB of LDS in FP64).  FP64
    matches the oracle's chain; mixed precision follows the oracle's decisions within the FP32
    rounding model (Sherman-Morrison steps in FP64 from FP32-stored values), with the FP64
    recompute after every sweep (without it the FP32 ratio errors of a sweep's ~100 accepted
    moves at N = 64 add up in log|det| past the 1e-4 bar)."""
    fp32 = precision == "mixed"
    g, o = make_pair(n, L, G, 1005, coef_seed=1005, fp64=not fp32, fp32=fp32)
    R0 = start_positions(1005, W, 2 * n, L)
    ref = orc.vmc(o, R0, S, sigma=0.5)
    crowd = cq.Crowd(g, W, precision=precision, delay_rank=1, recompute_every=1 if fp32 else 0, seed=1005,
                     path="sweep")
    if fp32:
        gpu = run_gpu(crowd, R0, S, 0.5, forced=ref.acc)
        emu = emulated_rho(o, R0, ref.acc, recompute_every=1, path="sweep")
        mixed_ratio_check(gpu["rho"], ref.rho, emu, "sweep N=%d mixed" % n)
        err = np.abs(gpu["logdet"] - ref.logdet) / np.maximum(1.0, np.abs(ref.logdet))
        assert err.max() < 1e-4, err.max()
    else:
        gpu = run_gpu(crowd, R0, S, 0.5)
        compare_fp64(gpu, ref, S, 2 * n)
    crowd.close()


def test_sweep_path_limits():
    """The whole-sweep path refuses what it cannot hold (N > 64, a delay rank above 1) with
    CQ_EINVAL; the automatic choice takes it for small N at delay rank 0 or 1 and the batched
    path otherwise."""
    for n, k in ((68, 1), (32, 4)):
        g = cq.System(n, 10.0)
        g.fill_philox(1, 8, 16)
        with pytest.raises(cq.CqError) as ei:
            cq.Crowd(g, 2, precision="fp64", delay_rank=k, seed=1, path="sweep")
        assert ei.value.status == cq.CQ_EINVAL
        g.close()
    g = cq.System(32, 10.0)
    g.fill_philox(1, 8, 16)
    for k, path in ((1, "sweep"), (0, "sweep"), (8, "batch")):
        c = cq.Crowd(g, 2, precision="fp64", delay_rank=k, seed=1)
        assert c.path() == path
        if path == "sweep":  # nothing to tune: the delay rank is 1 and no sweep runs
            c.set_positions(start_positions(1, 2, 64, 10.0))
            assert c.autotune(1) == 1 and c.acceptance()[1].sum() == 0
        c.close()
    g.close()


def test_paths_agree():
    """The per-move multi-workgroup path, the walker-resident window path, the batched-window
    path and the whole-sweep path compute the same chain: identical decisions, and ratios,
    log|det| and energies within the FP64 parity bar (their sums are grouped differently, so
    they agree to rounding, not bit for bit)."""
    n, L, G, W, S = 32, 10.0, 48, 20, 3
    g, _ = make_pair(n, L, G, 1002, coef_seed=1002)
    R0 = start_positions(1002, W, 2 * n, L)
    out = []
    for path in ALL_PATHS:
        c = cq.Crowd(g, W, precision="fp64", delay_rank=rank_for(path, 8), seed=1002, path=path)
        out.append(run_gpu(c, R0, S, 0.5))
        c.close()
    b = out[0]
    for a in out[1:]:
        assert np.array_equal(a["acc"], b["acc"])
        assert np.all(np.abs(a["rho"] - b["rho"]) <= 1e-10 * np.maximum(1.0, np.abs(b["rho"])))
        assert np.all(np.abs(a["logdet"] - b["logdet"]) <= 1e-10 * np.maximum(1.0, np.abs(b["logdet"])))
        assert np.all(np.abs(a["eloc"] - b["eloc"]) <= 1e-10 * np.maximum(1.0, np.abs(b["eloc"])))


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("n,L,G,W,S", [(32, 10.0, 48, 16, 2), (256, 20.0, 64, 4, 1)])
def test_one_stream_schedule_is_bit_identical(precision, n, L, G, W, S):
    """The batched path computes the same chain bit for bit whether the next round's gather
    and Jastrow sums run on a second stream beside the current round (default) or every kernel
    runs in order on one stream."""
    g, _ = make_pair(n, L, G, 1003, coef_seed=1003, fp64=precision == "fp64", fp32=precision == "mixed")
    R0 = start_positions(1003, W, 2 * n, L)
    res = []
    for streams in (2, 1):
        c = cq.Crowd(g, W, precision=precision, delay_rank=16, seed=1003, path="batch", streams=streams)
        res.append(run_gpu(c, R0, S, 0.5))
        c.close()
    for key in ("rho", "dlnj", "prob", "acc", "logdet", "sign", "eloc", "R"):
        assert np.array_equal(res[0][key], res[1][key]), key


def test_autotuned_delay_rank_keeps_the_chain():
    """delay_rank = 0: the first run times sweeps at k = 1, 2, 4, ..., 32 and keeps the fastest;
    the tuning sweeps are ordinary sweeps, so the chain still matches the FP64 oracle."""
    n, L, G, W, S = 32, 10.0, 48, 16, 1
    g, o = make_pair(n, L, G, 1002, coef_seed=1002)
    R0 = start_positions(1002, W, 2 * n, L)
    crowd = cq.Crowd(g, W, precision="fp64", delay_rank=0, seed=1002, path="batch")
    crowd.set_positions(R0)
    k = crowd.autotune(1)
    assert k in (1, 2, 4, 8, 16, 32) and crowd.delay_rank() == k
    tuned_sweeps = 6  # one per candidate
    crowd.record(S)
    crowd.run_vmc(S, 0.5)
    ref = orc.vmc(o, R0, tuned_sweeps + S, sigma=0.5)
    rec = crowd.records()
    assert np.array_equal(rec["acc"][0], ref.acc[tuned_sweeps])
    assert np.all(np.abs(rec["rho"][0] - ref.rho[tuned_sweeps]) <= 1e-10 * np.maximum(1.0, np.abs(ref.rho[tuned_sweeps])))
    crowd.close()



def test_tile_autotune_keeps_the_chain_and_uses_its_cache(tmp_path):
    """cq_crowd_autotune_tiles times every pair (Q, gather workgroups per CU) with one untimed
    and one timed sweep each; those are ordinary sweeps of the chain, so the chain after tuning
    is still the FP64 oracle's.  The choice goes into the JSON cache, and a second crowd with
    the same key takes it from there without running a sweep."""
    n, L, G, W, S, k, seed = 32, 10.0, 48, 8, 1, 4, 1011
    g, o = make_pair(n, L, G, seed, coef_seed=seed)
    R0 = start_positions(seed, W, 2 * n, L)
    cache = str(tmp_path / "tiles.json")
    crowd = cq.Crowd(g, W, precision="fp64", delay_rank=k, seed=seed, path="batch")
    assert crowd.tiles()["candidates"] == 12  # min(88, 3 k, N)
    crowd.set_positions(R0)
    t, hit = crowd.autotune_tiles(1, cache)
    assert not hit and t["candidates"] in (6, 8, 12) and t["gather_blocks_per_cu"] in (1, 2, 3)
    assert t["update_kernel"] in (1, 2)
    assert crowd.tiles() == t
    # Q in {6, 8, 12} x {1, 2, 3} workgroups per CU x {vector, matrix-core} FP64 update, 1 + 1 sweeps each
    tuned_sweeps = 3 * 3 * 2 * 2
    crowd.record(S)
    crowd.run_vmc(S, 0.5)
    ref = orc.vmc(o, R0, tuned_sweeps + S, sigma=0.5)
    rec = crowd.records()
    assert np.array_equal(rec["acc"][0], ref.acc[tuned_sweeps])
    for key in ("rho", "dlnj", "prob"):
        b = getattr(ref, key)[tuned_sweeps]
        assert np.all(np.abs(rec[key][0] - b) <= 1e-10 * np.maximum(1.0, np.abs(b))), key
    entry = json.load(open(cache))[-1]
    assert (entry["n"], entry["walkers"], entry["precision"], entry["delay_rank"]) == (n, W, "fp64", k)
    assert (entry["candidates"], entry["gather_blocks_per_cu"], entry["update_kernel"]) == (
        t["candidates"], t["gather_blocks_per_cu"], t["update_kernel"])
    crowd.close()
    # the same key again: from the cache, no sweep run (the chain starts at sweep 0)
    crowd = cq.Crowd(g, W, precision="fp64", delay_rank=k, seed=seed, path="batch")
    crowd.set_positions(R0)
    t2, hit = crowd.autotune_tiles(1, cache)
    assert hit and t2 == t and crowd.tiles() == t
    crowd.record(S)
    crowd.run_vmc(S, 0.5)
    rec = crowd.records()
    assert np.array_equal(rec["acc"][0], ref.acc[0])
    assert np.all(np.abs(rec["rho"][0] - ref.rho[0]) <= 1e-10 * np.maximum(1.0, np.abs(ref.rho[0])))
    # shapes out of range are refused and change nothing; other paths report none
    for bad in (dict(candidates=3), dict(candidates=13), dict(gather_blocks_per_cu=9), dict(update_kernel=3)):
        with pytest.raises(cq.CqError) as ei:
            crowd.set_tiles(**bad)
        assert ei.value.status == cq.CQ_EINVAL
    assert crowd.tiles() == t
    crowd.close()
    sweep = cq.Crowd(g, W, precision="fp64", seed=seed, path="sweep")
    sweep.set_positions(R0)
    none = dict(candidates=0, gather_blocks_per_cu=0, update_kernel=0)
    assert sweep.tiles() == none
    assert sweep.autotune_tiles(1, cache) == (none, False)
    sweep.close()
    g.close()


@pytest.mark.parametrize("n,L,G,W,S,k", [(32, 10.0, 48, 16, 2, 8), (64, 12.0, 48, 8, 2, 4), (256, 20.0, 64, 3, 1, 32)])
def test_fp64_matrix_core_update_keeps_the_chain(n, L, G, W, S, k):
    """The FP64 rank-k update on the matrix cores (update_kernel = 2: strips of 16 rows of the
    inverse, both products on v_mfma_f64_16x16x4f64, forward substitution in move order) follows
    the oracle's chain like the vector one: decisions, ratios and ln J changes within 1e-10 (or,
    where the two FP64 update chains have parted by more, of the refined ratio)."""
    seed = 1013
    g, o = make_pair(n, L, G, seed, coef_seed=seed)
    R0 = start_positions(seed, W, 2 * n, L)
    crowd = cq.Crowd(g, W, precision="fp64", delay_rank=k, seed=seed, path="batch")
    crowd.set_tiles(update_kernel=2)
    assert crowd.tiles()["update_kernel"] == 2
    gpu = run_gpu(crowd, R0, S, 0.5)
    ref = orc.vmc(o, R0, S, sigma=0.5)
    arbitrated_fp64_check(gpu, ref, o, R0, range(W), range(W), S * 2 * n)
    if np.array_equal(gpu["acc"], ref.acc):  # the same chain throughout: log|det| and E_L of its end
        assert np.all(np.abs(gpu["logdet"][-1] - ref.logdet[-1]) <= 1e-9 * np.maximum(1.0, np.abs(ref.logdet[-1])))
        assert np.all(np.abs(gpu["eloc"][-1] - ref.eloc[-1]) <= 1e-8 * np.maximum(1.0, np.abs(ref.eloc[-1])))
    crowd.close()
    g.close()

# Full C4 size: 1024 + 1024 electrons, L = 32, 96^3 seeded table, Pade J2, a crowd of 128
# walkers, delayed rank 32 on the batched path.  The oracle follows three sampled walkers
# (first, interior, last of the crowd) through the whole up-spin block and the first 256
# moves of the down-spin block; the other walkers run alongside, as in the timed sweep.
C4_N, C4_L, C4_G, C4_W = 1024, 32.0, 96, 128
C4_SAMPLE = [0, 77, 127]
C4_MOVES = C4_N + 256


def c4_reference(o, R0):
    return orc.vmc(o, R0[C4_SAMPLE], 1, sigma=0.5, uids=np.array(C4_SAMPLE, np.uint32), max_moves=C4_MOVES,
                   n_threads=len(C4_SAMPLE))


def exact_ratios(o, R0w, uid, acc, moves, sigma=0.5):
    """Determinant ratios at the given moves (flat index sweep * Ne + electron, from sweep 0) of
    one walker from a fresh, refined solve of the current matrix (oracle.row_ratio_refined),
    replaying the oracle's decisions acc (flat) and its proposal stream r' = wrap(r_e + sigma z);
    A is kept by row replacement, with no inverse."""
    n, L = o.n_up, o.L
    ne = 2 * n
    want = set(int(k) for k in moves)
    out, R, A = {}, np.array(R0w, dtype=np.float64), [None, None]
    for m in range(max(want) + 1):
        if m not in want and not acc[m]:
            continue
        sweep, e = divmod(m, ne)
        sp, i = divmod(e, n)
        rnew = np.mod(R[e] + sigma * orc.gauss3(o.seed, uid, sweep, e), L)
        phi = orc.orbital_vgl(o, rnew, n)[0]
        if m in want:
            if A[sp] is None:
                A[sp] = np.array([orc.orbital_vgl(o, R[sp * n + j], n)[0] for j in range(n)])
            out[m] = orc.row_ratio_refined(A[sp], i, phi)
        if acc[m]:
            R[e] = rnew
            if A[sp] is not None:
                A[sp][i] = phi
    return out


def arbitrated_fp64_check(gpu, ref, o, R0, walkers, uids, moves, tol=1e-10, label=""):
    """The first `moves` moves (flat over sweeps) of the given walkers (columns of ref): identical
    decisions except at near-ties, Jastrow changes within tol, and ratios within tol relative of
    the oracle's; where a long FP64 update chain (the oracle's Sherman-Morrison steps, or the
    GPU's) has drifted more than tol, the arbiter is the ratio from a fresh, refined solve of the
    current matrix, and the GPU value must be within tol of it there."""
    rel = lambda a, b: np.abs(a - b) / np.maximum(1.0, np.abs(b))
    flat = lambda x, col: x[:, :, col].ravel()[:moves]
    for i, w in enumerate(walkers):
        acc_g, acc_r = flat(gpu["acc"], w), flat(ref.acc, i)
        d = np.nonzero(acc_g != acc_r)[0]
        lim = moves if len(d) == 0 else int(d[0])
        if len(d):
            assert abs(flat(ref.prob, i)[lim] - flat(ref.u, i)[lim]) < NEAR_TIE, "decision differs away from a near-tie"
        dj_g, dj_r = flat(gpu["dlnj"], w)[:lim], flat(ref.dlnj, i)[:lim]
        assert np.all(rel(dj_g, dj_r) <= tol), (w, "dlnj")
        rho_g, rho_r = flat(gpu["rho"], w)[:lim], flat(ref.rho, i)[:lim]
        pr_g, pr_r = flat(gpu["prob"], w)[:lim], flat(ref.prob, i)[:lim]
        off = np.nonzero((rel(rho_g, rho_r) > tol) | (rel(pr_g, pr_r) > tol))[0]
        msg = "   %swalker %d: %d moves (%d accepted), rho max diff from the oracle %.2e, %d beyond %.0e" % (
            label, w, lim, int(acc_r[:lim].sum()), rel(rho_g, rho_r).max(), len(off), tol)
        if len(off):
            ex = exact_ratios(o, R0[w], int(uids[i]), acc_r, off)
            x = np.array([ex[k] for k in off])
            eg, eo = rel(rho_g[off], x), rel(rho_r[off], x)
            msg += "; there: GPU - exact max %.2e, oracle - exact max %.2e" % (eg.max(), eo.max())
            print(msg)
            assert np.all(eg <= tol), (w, off[eg > tol])
            assert np.all(rel(pr_g[off], x * x * np.exp(2.0 * dj_r[off])) <= 2 * tol), w
        else:
            print(msg)


def test_c4_full_size_fp64_sampled_walkers_match_oracle():
    """At full C4 size the FP64 batched path reproduces the oracle's chain for the sampled walkers:
    identical decisions (except at near-ties), Jastrow changes within 1e-10, and ratios and
    acceptance probabilities within 1e-10 relative, across every round and window flush of a spin
    block and the spin boundary.  At N = 1024 (cond(A) ~ 1e4) the oracle's own chain of a few
    hundred Sherman-Morrison updates drifts up to a few 1e-10 from the true ratio, so where the two
    chains differ by more than 1e-10 the arbiter is the ratio from a fresh, refined solve of the
    current matrix: the GPU value must be within 1e-10 of it there."""
    g, o = make_pair(C4_N, C4_L, C4_G, 1004, coef_seed=1004)
    R0 = start_positions(1004, C4_W, 2 * C4_N, C4_L)
    crowd = cq.Crowd(g, C4_W, precision="fp64", delay_rank=32, seed=1004, path="batch")
    gpu = run_gpu(crowd, R0, 1, 0.5)
    crowd.close()
    g.close()
    ref = c4_reference(o, R0)
    arbitrated_fp64_check(gpu, ref, o, R0, C4_SAMPLE, C4_SAMPLE, C4_MOVES)


def test_c4_full_size_mixed_bench_configuration_on_oracle_trajectory():
    """The timed configuration at full C4 size (FP32 table, inverse and update GEMMs; FP64
    set-up, log|det| and energy sums; delayed rank 32, FP64 recompute every 32 sweeps, batched
    path, eager launches with HIP-event timing on): set-up log|det|, sign and E_L of the sampled
    walkers match the oracle, and along the oracle's decisions their ratios stay within the
    mixed-precision bar.  The other walkers take their own decisions (flag 2)."""
    g, o = make_pair(C4_N, C4_L, C4_G, 1004, coef_seed=1004, fp64=False, fp32=True)
    R0 = start_positions(1004, C4_W, 2 * C4_N, C4_L)
    ld0, sg0, el0, _ = orc.setup(o, R0[C4_SAMPLE], n_threads=len(C4_SAMPLE))
    ref = c4_reference(o, R0)
    forced = np.full((1, 2 * C4_N, C4_W), 2, np.uint8)
    for i, w in enumerate(C4_SAMPLE):
        forced[0, :C4_MOVES, w] = ref.acc[0, :C4_MOVES, i]
    crowd = cq.Crowd(g, C4_W, precision="mixed", delay_rank=32, recompute_every=32, seed=1004, path="batch")
    crowd.set_timing(["propose", "vgl", "resolve", "update", "energy", "inverse"])
    crowd.set_positions(R0)
    ld, sg = crowd.logdet()
    el = crowd.local_energy()
    lerr = np.abs(ld[C4_SAMPLE] - ld0) / np.maximum(1.0, np.abs(ld0))
    eerr = np.abs(el[C4_SAMPLE] - el0) / np.maximum(1.0, np.abs(el0))
    print("   set-up: log|det| max err %.2e, E_L max rel err %.2e" % (lerr.max(), eerr.max()))
    assert lerr.max() < 1e-4 and np.array_equal(sg[C4_SAMPLE], sg0)
    assert eerr.max() < 1e-3
    gpu = run_gpu(crowd, R0, 1, 0.5, forced=forced)
    crowd.close()
    g.close()
    assert np.array_equal(gpu["acc"][0, :C4_MOVES][:, C4_SAMPLE], ref.acc[0, :C4_MOVES])
    emu = emulated_rho(o, R0[C4_SAMPLE], ref.acc, uids=C4_SAMPLE, n_moves=C4_MOVES, k=32, path="batch")
    _, es = mixed_ratio_check(gpu["rho"][0, :C4_MOVES][:, C4_SAMPLE], ref.rho[0, :C4_MOVES],
                              emu[0, :C4_MOVES], "C4 mixed k=32 batch")
    own_decision_check(gpu["prob"][0, :C4_MOVES][:, C4_SAMPLE], ref.prob[0, :C4_MOVES], ref.u[0, :C4_MOVES],
                       ref.acc[0, :C4_MOVES], es, 5e-3)
    assert np.all(np.isfinite(gpu["logdet"])) and np.all(np.isfinite(gpu["eloc"]))
    acc = gpu["acc"].mean()
    print("   crowd acceptance %.3f" % acc)
    assert 0.2 < acc < 0.6
