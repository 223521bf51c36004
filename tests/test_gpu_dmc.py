"""GPU parity of the DMC generation (drift-diffusion moves, branching, trial energy) against
the FP64 CPU oracle on the same seeded inputs and random streams.

FP64: per generation the population, the sum of branching weights, the weighted mean energy and
the trial energy agree within 1e-10 relative; the final walkers agree too: uids in population
order exactly, local energies within 1e-9 relative, positions within 1e-8 (the drift step
tau v amplifies the rounding of the gradient near nodes).  A decision that falls within 1e-6 of its uniform, or
a branching weight within 1e-9 of an integer boundary, could legitimately differ; the seeds used
here have none.
"""
import numpy as np
import pytest

import oracle as orc
import paper_2209_14487_amd as cq
from synth import J2_A_ANTI, J2_A_PAR, J2_B, start_positions

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


def test_dmc_mixed_precision_runs():
    """Mixed precision (FP32 table and inverse, FP64 weights and sums): finite energies, a live
    population, trial energy within 2 % of the FP64 oracle's after 3 generations (a single
    decision that flips at the FP32 rounding level moves one walker's energy a lot on these rough
    random orbitals, so this is a smoke bound, not a parity bound)."""
    n, L, G, W, gens, tau, seed = 32, 10.0, 48, 32, 3, 0.01, 1005
    g, o = make_pair(n, L, G, seed, fp64=False, fp32=True)
    R0 = start_positions(seed, W, 2 * n, L)
    _, _, el0, _ = orc.setup(o, R0)
    e_trial = float(np.mean(el0))
    ref = orc.dmc(o, R0, gens, tau, e_trial, n_target=W, max_pop=4 * W + 16)
    crowd = cq.Crowd(g, W, precision="mixed", delay_rank=8, seed=seed, max_walkers=4 * W + 16)
    crowd.set_positions(R0)
    hist = crowd.run_dmc(gens, tau, e_trial, n_target=W)
    assert np.all(np.isfinite(hist))
    assert hist[-1, 0] > W // 2
    assert np.all(np.isfinite(crowd.local_energy()))
    assert np.all(rel(hist[:, 3], ref.e_t) < 2e-2)
    crowd.close()
    g.close()
