"""GPU parity of the DMC generation (drift-diffusion moves, branching, trial energy) against
the FP64 CPU oracle on the same seeded inputs and random streams.

The drift-diffusion step amplifies rounding: near a node the drift grows like the inverse
distance, so two FP64 runs that round differently part ways move by move (a one-ulp change of
the starting positions moves the oracle's own ratios by 3.8e-7 after four generations at
N = 32 and by 2.7e-6 after two at N = 256).  So:

* small systems over a few generations (N <= 32): the population, the sum of branching weights,
  the weighted mean energy and the trial energy agree with the oracle within 1e-10 relative,
  the final uids exactly, local energies within 1e-9, positions within 1e-8;
* at the S2 / S3 sizes the GPU's own records are checked on the GPU's own trajectory, each
  ratio, proposal and acceptance probability against its definition (``dmc_replay``), and the
  generation sums against the oracle within ten times what a one-ulp start changes in the
  oracle's own;
* mixed precision (FP32 table, inverse and orbital rows; FP64 weights, sums and trial energy)
  runs in parity mode, following the oracle's decisions and branching multiplicities, and its
  ratio errors on its own trajectory are bounded by those of the FP32 rounding model
  (``oracle.fp32_chain.replay_dmc``) along the same proposals and decisions.

A decision that falls within 1e-6 of its uniform, or a branching weight within 1e-9 of an
integer boundary, could legitimately differ; the seeds used here have none.
"""
import numpy as np
import pytest

import oracle as orc
import paper_2209_14487_amd as cq
from oracle import fp32_chain
from synth import J2_A_ANTI, J2_A_PAR, J2_B, start_positions
from dmc_replay import periodic_abs, trajectory_checks

pytestmark = pytest.mark.gpu


def make_pair(n, L, G, seed, fp64=True, fp32=False):
    g = cq.System(n, L)
    if fp64:
        g.fill_philox(seed, 8, G)
    if fp32:
        g.fill_philox(seed, 4, G)
    g.load_j2(J2_A_PAR, J2_A_ANTI, J2_B)
    o = orc.System(n, n, L, G=G, n_orb=n, orb_kind=orc.ORB_SEEDED, coef_seed=seed, use_j2=True,
                   j2_a_par=J2_A_PAR, j2_a_anti=J2_A_ANTI, j2_b=J2_B, seed=seed)
    return g, o


def periodic_diff(a, b, L):
    """Largest |a - b| over coordinates, taken modulo the box (a position at x = L - 1e-15 and
    one at x = 0 are the same point; the wrap can land on either side of the seam)."""
    d = np.asarray(a) - np.asarray(b)
    d -= L * np.round(d / L)
    return float(np.abs(d).max())


def rel(a, b):
    return np.abs(np.asarray(a) - np.asarray(b)) / np.maximum(1.0, np.abs(np.asarray(b)))


@pytest.mark.parametrize("n,k", [(8, 1), (32, 8), (32, 32)])
def test_dmc_generations_match_oracle(n, k):
    L, G, W, gens, tau, seed = 10.0, 48, 24, 4, 0.01, 1005
    g, o = make_pair(n, L, G, seed)
    R0 = start_positions(seed, W, 2 * n, L)
    _, _, el0, _ = orc.setup(o, R0)
    e_trial = float(np.mean(el0))
    cap = 4 * W + 16
    ref = orc.dmc(o, R0, gens, tau, e_trial, n_target=W, max_pop=cap)
    crowd = cq.Crowd(g, W, precision="fp64", delay_rank=k, seed=seed, max_walkers=cap, path="window")
    crowd.set_positions(R0)
    hist = crowd.run_dmc(gens, tau, e_trial, n_target=W)
    print("   pop", hist[:, 0].astype(int).tolist(), "oracle", ref.pop.tolist())
    assert np.array_equal(hist[:, 0].astype(int), ref.pop)
    assert np.all(rel(hist[:, 1], ref.wsum) < 1e-10)
    assert np.all(rel(hist[:, 2], ref.e_est) < 1e-10)
    assert np.all(rel(hist[:, 3], ref.e_t) < 1e-10)
    assert crowd.W == len(ref.uids)
    assert np.array_equal(crowd.uids(), ref.uids)
    # the drift tau v enters every position; near a node |v| is large and the window-corrected
    # gradient dot products lose a few more digits than the ratio, so positions get 1e-8
    dR = periodic_diff(crowd.positions(), ref.R, L)
    print("   max position difference %.2e" % dR)
    assert dR < 1e-8
    assert np.all(rel(crowd.local_energy(), ref.eloc) < 1e-9)
    crowd.close()
    g.close()


def test_dmc_population_branches_and_survives():
    """A longer FP64 run at a larger time step: walkers are born and die (the population
    changes), and the result still follows the oracle generation by generation."""
    n, L, G, W, gens, tau, seed = 8, 10.0, 48, 32, 8, 0.05, 1005
    g, o = make_pair(n, L, G, seed)
    R0 = start_positions(seed + 1, W, 2 * n, L)
    _, _, el0, _ = orc.setup(o, R0)
    e_trial = float(np.mean(el0))
    cap = 4 * W + 16
    ref = orc.dmc(o, R0, gens, tau, e_trial, n_target=W, max_pop=cap)
    crowd = cq.Crowd(g, W, precision="fp64", delay_rank=4, seed=seed, max_walkers=cap, path="window")
    crowd.set_positions(R0)
    hist = crowd.run_dmc(gens, tau, e_trial, n_target=W)
    print("   pop", hist[:, 0].astype(int).tolist())
    assert len(set(ref.pop.tolist())) > 1, "population never changed: the test would not exercise branching"
    assert np.array_equal(hist[:, 0].astype(int), ref.pop)
    assert np.all(rel(hist[:, 3], ref.e_t) < 1e-10)
    assert np.array_equal(crowd.uids(), ref.uids)
    crowd.close()
    g.close()


def run_pair_fp64(n, L, G, W, gens, tau, seed, k, n_threads=0, forced=False):
    """One FP64 DMC run of the same population on the GPU and in the oracle, both recording
    (forced: the GPU follows the oracle's decisions and branching multiplicities)."""
    g, o = make_pair(n, L, G, seed)
    R0 = start_positions(seed, W, 2 * n, L)
    _, _, el0, _ = orc.setup(o, R0, n_threads=n_threads)
    e_trial = float(np.mean(el0))
    cap = 4 * W + 16
    ref = orc.dmc(o, R0, gens, tau, e_trial, n_target=W, max_pop=cap, record=True, n_threads=n_threads)
    crowd = cq.Crowd(g, W, precision="fp64", delay_rank=k, seed=seed, max_walkers=cap, path="window")
    crowd.set_positions(R0)
    crowd.record(gens)
    if forced:
        crowd.set_forced(ref.rec["acc"])
        crowd.set_forced_branching(ref.rec["mult"])
    hist = crowd.run_dmc(gens, tau, e_trial, n_target=W)
    rec = crowd.records(all_slots=True)
    return g, o, crowd, ref, hist, rec


def rounding_envelope(o, R0, gens, tau, e_trial, W, cap, n_threads=0):
    """How far the oracle's own DMC chain moves under a rounding-level change: the same run from
    starting positions one ulp away (the drift-diffusion step amplifies any such difference near
    nodes, generation after generation).  Returns that run."""
    return orc.dmc(o, np.nextafter(R0, np.inf), gens, tau, e_trial, n_target=W, max_pop=cap, record=True,
                   n_threads=n_threads)


@pytest.mark.parametrize("n,L,G,W,gens,k,stride,forced", [(256, 20.0, 64, 6, 2, 8, 3, False),
                                                           (1024, 32.0, 96, 8, 1, 32, 193, True)])
def test_dmc_fp64_at_c5_system_sizes(n, L, G, W, gens, k, stride, forced):
    """FP64 DMC at the S2 and S3 system sizes of the batched uneven workload (256 + 256 electrons
    on a 64^3 grid, 1024 + 1024 on 96^3, delay ranks 8 and 32), where the walker-resident move
    kernel takes several passes over the orbitals per thread.

    The drift-diffusion chain amplifies rounding: a one-ulp change of the starting positions moves
    the oracle's own ratios by up to 2.7e-6 within two generations at N = 256.  So the GPU's ratios
    are checked where they are defined, on the GPU's own trajectory: at sampled moves (every
    stride-th) each recorded ratio equals det A'/det A of the current matrix (refined solve) within
    1e-10 relative (1e-9 at N = 1024, where the FP64 update chains themselves drift by a few
    1e-10 over a thousand updates), each recorded proposal equals wrap(r + tau v + sqrt(tau) z)
    with the drift v of the current configuration within 1e-9 relative to max(1, |v|), and each
    acceptance probability its Green's-function form within 1e-9.  The decisions, populations and
    uids are the oracle's (at N = 1024, where over 16384 moves a few dozen decisions sit close
    enough to their uniforms for the two runs' diverging positions to flip them, the GPU follows
    the oracle's decisions and multiplicities); the generation's weight sum, E_est and E_T lie
    within 1e-10 relative of the oracle's, or within ten times the change that the one-ulp start
    makes to the oracle's own values."""
    tau, seed = 0.01, 1006 if n == 256 else 1007
    g, o, crowd, ref, hist, rec = run_pair_fp64(n, L, G, W, gens, tau, seed, k, n_threads=W, forced=forced)
    live = np.isfinite(ref.rec["rho"])
    d = np.nonzero(rec["acc"][live] != ref.rec["acc"][live])[0]
    print("   pop", hist[:, 0].astype(int).tolist(), "oracle", ref.pop.tolist(), "decisions differing", len(d))
    assert len(d) == 0 or np.all(np.abs(ref.rec["prob"][live][d] - ref.rec["u"][live][d]) < 1e-6)
    assert np.array_equal(hist[:, 0].astype(int), ref.pop)
    assert np.array_equal(crowd.uids(), ref.uids)
    R0 = start_positions(seed, W, 2 * n, L)
    pick = lambda gg, e, slot: (e + 7 * slot + gg) % stride == 0
    t = trajectory_checks(o, R0, np.arange(W), rec["acc"], rec["rnew"], ref.rec["mult"], tau, pick)
    m = np.isfinite(t["ratio"])
    rerr = np.abs(rec["rho"][m] - t["ratio"][m]) / np.maximum(1.0, np.abs(t["ratio"][m]))
    # drift error |v_gpu - v| = |r'_gpu - r'| / tau, relative to max(1, |v|)
    derr = np.linalg.norm(periodic_abs(rec["rnew"][m] - t["prop"][m], L), axis=-1) / tau / np.maximum(
        1.0, t["vabs"][m])
    perr = np.abs(rec["prob"][m] - t["prob"][m]) / np.maximum(1.0, np.abs(t["prob"][m]))
    print("   %d sampled moves: max error against the definitions: ratio %.2e, drift %.2e, probability %.2e"
          % (m.sum(), rerr.max(), derr.max(), perr.max()))
    tol = 1e-10 if n <= 256 else 1e-9
    assert m.sum() >= 40 and rerr.max() < tol
    assert derr.max() < 1e-9 and perr.max() < 1e-9
    env = rounding_envelope(o, R0, gens, tau, float(np.mean(orc.setup(o, R0, n_threads=W)[2])), W, 4 * W + 16,
                            n_threads=W)
    for q, (x, y, z) in {"wsum": (hist[:, 1], ref.wsum, env.wsum), "E_est": (hist[:, 2], ref.e_est, env.e_est),
                         "E_T": (hist[:, 3], ref.e_t, env.e_t)}.items():
        err, spread = np.abs(x - y), np.abs(z - y)
        print("   %s: GPU - oracle %s, one-ulp start %s" % (q, np.array2string(err, precision=2),
                                                           np.array2string(spread, precision=2)))
        assert np.all(err <= np.maximum(1e-10 * np.abs(y), 10.0 * spread))
    acc, prop = crowd.dmc_moves()
    assert prop == sum([W] + list(ref.pop[:-1])) * 2 * n and acc == int(ref.rec["acc"][live].sum())
    crowd.close()
    g.close()


@pytest.mark.parametrize("n,L,G,W,gens,k,rc,stride,sums", [(32, 10.0, 48, 24, 3, 8, 0, 1, True),
                                                           (256, 20.0, 64, 6, 2, 8, 1, 3, False)])
def test_dmc_mixed_precision_follows_oracle(n, L, G, W, gens, k, rc, stride, sums):
    """Mixed-precision DMC in parity mode at the S1 and S2 system sizes (S2 with the FP64
    recompute after every generation): the GPU follows the FP64 oracle's decisions and
    multiplicities, so the populations match walker for walker.  Its proposals follow its own
    (FP32-derived) drift, so its ratios are checked on its own trajectory: against det A'/det A
    of the current matrix in FP64 (the definition), their relative errors stay within factors
    2 (median, p99) and 3 (p99.9, max over |rho| >= 0.1) of those of the FP32 rounding model
    (``oracle.fp32_chain.replay_dmc``, windows of k proposals as the GPU kernel uses them)
    replayed along the same proposals, decisions, multiplicities and recomputes.  The generation's weight sum, E_est and E_T (FP64 sums of
    FP32-derived local energies) stay within 1e-4 relative of the oracle's."""
    tau, seed = 0.01, 1005
    g, o = make_pair(n, L, G, seed, fp64=False, fp32=True)
    R0 = start_positions(seed, W, 2 * n, L)
    _, _, el0, _ = orc.setup(o, R0)
    e_trial = float(np.mean(el0))
    cap = 4 * W + 16
    ref = orc.dmc(o, R0, gens, tau, e_trial, n_target=W, max_pop=cap, record=True)
    crowd = cq.Crowd(g, W, precision="mixed", delay_rank=k, recompute_every=rc, seed=seed, max_walkers=cap,
                     path="window")
    crowd.set_positions(R0)
    crowd.record(gens)
    crowd.set_forced(ref.rec["acc"])
    crowd.set_forced_branching(ref.rec["mult"])
    hist = crowd.run_dmc(gens, tau, e_trial, n_target=W)
    rec = crowd.records(all_slots=True)
    assert np.array_equal(hist[:, 0].astype(int), ref.pop)
    assert np.array_equal(crowd.uids(), ref.uids)
    live = np.isfinite(ref.rec["rho"])
    assert np.array_equal(rec["acc"][live], ref.rec["acc"][live])
    import dataclasses
    o32 = dataclasses.replace(o, coef_fp32=True)
    pick = lambda gg, e, slot: (e + 7 * slot + gg) % stride == 0
    fr = trajectory_checks(o32, R0, np.arange(W), rec["acc"], rec["rnew"], ref.rec["mult"], tau, pick,
                           with_drift=False)["ratio"]
    emu = fp32_chain.replay_dmc(o32, R0, np.arange(W), rec["acc"], ref.rec["mult"], tau, rnew=rec["rnew"],
                                recompute_every=rc, window=k)
    m = np.isfinite(fr)
    gs = fp32_chain.ratio_error_stats(rec["rho"][m], fr[m], floor=0.1)
    es = fp32_chain.ratio_error_stats(emu["rho"][m], fr[m], floor=0.1)
    print("   %d moves; ratio rel err GPU %s | FP32 model %s" % (m.sum(),
        " ".join("%s=%.2e" % (q, gs[q]) for q in ("median", "p99", "p999", "max")),
        " ".join("%s=%.2e" % (q, es[q]) for q in ("median", "p99", "p999", "max"))))
    factor = dict(median=2.0, p99=2.0, p999=3.0, max=3.0)
    for q, f in factor.items():
        assert gs[q] <= f * es[q], (q, gs, es)
    werr, eerr, terr = rel(hist[:, 1], ref.wsum), rel(hist[:, 2], ref.e_est), rel(hist[:, 3], ref.e_t)
    print("   weight sum err %.2e, E_est err %.2e, E_T err %.2e" % (werr.max(), eerr.max(), terr.max()))
    if sums:
        assert werr.max() < 1e-4 and eerr.max() < 1e-4 and terr.max() < 1e-4
    el = crowd.local_energy()
    el64 = orc.setup(o32, crowd.positions(), n_threads=8)[2]
    lerr = rel(el, el64)
    print("   final E_L against FP64 at the GPU's positions: max rel err %.2e" % lerr.max())
    assert np.all(np.isfinite(el)) and lerr.max() < 1e-3
    crowd.close()
    g.close()


def test_dmc_mixed_precision_recompute_keeps_logdet():
    """Mixed DMC with the periodic FP64 recompute every 2 generations: log|det| carried through
    branching stays within 1e-4 of max(1, |log|det||) of a fresh FP64 recompute, the recomputes
    are counted and their drift recorded."""
    n, L, G, W, gens, tau, seed = 32, 10.0, 48, 24, 5, 0.01, 1005
    g, o = make_pair(n, L, G, seed, fp64=False, fp32=True)
    R0 = start_positions(seed, W, 2 * n, L)
    _, _, el0, _ = orc.setup(o, R0)
    crowd = cq.Crowd(g, W, precision="mixed", delay_rank=8, recompute_every=2, seed=seed, max_walkers=4 * W + 16,
                     path="window")
    crowd.set_positions(R0)
    crowd.run_dmc(gens, tau, float(np.mean(el0)), n_target=W)
    _, dmax, nrec = crowd.drift()
    assert nrec == gens // 2
    ld0, _ = crowd.logdet()
    d = crowd.recompute()
    ld1, _ = crowd.logdet()
    err = np.abs(ld0 - ld1) / np.maximum(1.0, np.abs(ld1))
    print("   in-run recomputes %d, max drift %.2e; drift at the final recompute %.2e" % (nrec, dmax, d))
    assert err.max() < 1e-4 and abs(d - np.abs(ld0 - ld1).max()) <= 1e-12 * max(1.0, d)
    assert np.isfinite(dmax) and dmax < 1e-2
    crowd.close()
    g.close()
