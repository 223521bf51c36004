"""Crowds of several systems (the batched uneven workload): the walkers of systems with different
electron counts moved by the same launches in DMC.

* The group's DMC equals, bit for bit, the same systems run as separate crowds (same seeds, uids,
  delay ranks and recompute schedule): populations, uids, positions, local energies, log|det| and
  the generation history, in FP64 and in mixed precision (where every system's N is a multiple of
  32, so the update runs on the matrix cores).  The shared launches change where each walker's
  work runs, not what it computes.
* In FP64 the group follows the per-system oracle runs generation by generation (systems of 8 and
  32 electrons per spin over two generations, where the drift-diffusion chains have not yet parted
  by more than 1e-10): populations and uids exactly, weight sums, E_est and E_T within 1e-10.
"""
import numpy as np
import pytest

import oracle as orc
import paper_2209_14487_amd as cq
from synth import J2_A_ANTI, J2_A_PAR, J2_B, start_positions

pytestmark = pytest.mark.gpu


def make(n, L, G, seed, eb):
    g = cq.System(n, L)
    g.fill_philox(seed, eb, G)
    g.load_j2(J2_A_PAR, J2_A_ANTI, J2_B)
    return g


def caps(counts, max_walkers):
    total = sum(counts)
    return [-(-max_walkers * w // total) for w in counts]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_group_dmc_equals_separate_crowds(precision):
    eb = 8 if precision == "fp64" else 4
    spec = [(32, 10.0, 48, 24), (64, 12.0, 48, 8), (256, 20.0, 64, 4)]  # (N, L, G, walkers)
    seed, gens, tau, k, rc = 1105, 3, 0.01, 16, (1 if precision == "mixed" else 0)
    systems = [make(n, L, G, seed + i, eb) for i, (n, L, G, _) in enumerate(spec)]
    counts = [w for (_, _, _, w) in spec]
    R0 = [start_positions(seed + i, w, 2 * n, L) for i, (n, L, _, w) in enumerate(spec)]
    mw = 4 * sum(counts) + 64
    grp = cq.Crowd(systems, counts, precision=precision, delay_rank=k, recompute_every=rc, seed=seed,
                   max_walkers=mw, path="window")
    grp.set_positions(R0)
    el0 = grp.local_energy()
    e_trial = [float(np.mean(el0[sum(counts[:i]):sum(counts[:i + 1])])) for i in range(len(spec))]
    hist = grp.run_dmc_systems(gens, tau, e_trial=e_trial)
    print("   group populations", hist[:, :, 0].astype(int).tolist())
    cp = caps(counts, mw)
    uid0 = np.cumsum([0] + [max(w, c) for w, c in zip(counts, cp)])[:-1]
    sep = []
    for i, (n, L, G, w) in enumerate(spec):
        c = cq.Crowd(systems[i], w, precision=precision, delay_rank=min(k, n), recompute_every=rc, seed=seed,
                     first_uid=int(uid0[i]), max_walkers=cp[i], path="window")
        c.set_positions(R0[i])
        h = c.run_dmc(gens, tau, e_trial[i], n_target=w)
        assert np.array_equal(h, hist[:, i, :]), (i, h, hist[:, i, :])
        sep.append(c)
    assert np.array_equal(np.concatenate([c.uids() for c in sep]), grp.uids())
    for a, b in zip(grp.positions(), [c.positions() for c in sep]):
        assert np.array_equal(a, b)
    assert np.array_equal(grp.local_energy(), np.concatenate([c.local_energy() for c in sep]))
    assert np.array_equal(grp.logdet()[0], np.concatenate([c.logdet()[0] for c in sep]))
    acc, prop = grp.dmc_moves()
    assert prop == sum(c.dmc_moves()[1] for c in sep) and acc == sum(c.dmc_moves()[0] for c in sep)
    for c in sep:
        c.close()
    grp.close()
    for g in systems:
        g.close()


def test_group_dmc_fp64_follows_per_system_oracle():
    spec = [(8, 6.0, 16, 20), (32, 10.0, 48, 12)]
    seed, gens, tau = 1205, 2, 0.01
    systems, refs, R0, e_trial = [], [], [], []
    for i, (n, L, G, w) in enumerate(spec):
        systems.append(make(n, L, G, seed + i, 8))
        o = orc.System(n, n, L, G=G, n_orb=n, orb_kind=orc.ORB_SEEDED, coef_seed=seed + i, use_j2=True,
                       j2_a_par=J2_A_PAR, j2_a_anti=J2_A_ANTI, j2_b=J2_B, seed=seed)
        R = start_positions(seed + i, w, 2 * n, L)
        R0.append(R)
        et = float(np.mean(orc.setup(o, R)[2]))
        e_trial.append(et)
        refs.append((o, R, et))
    counts = [w for (_, _, _, w) in spec]
    mw = 4 * sum(counts) + 64
    cp = caps(counts, mw)
    uid0 = np.cumsum([0] + [max(w, c) for w, c in zip(counts, cp)])[:-1]
    grp = cq.Crowd(systems, counts, precision="fp64", delay_rank=8, seed=seed, max_walkers=mw, path="window")
    grp.set_positions(R0)
    hist = grp.run_dmc_systems(gens, tau, e_trial=e_trial)
    uids = grp.uids()
    off = 0
    for i, ((o, R, et), w) in enumerate(zip(refs, counts)):
        ref = orc.dmc(o, R, gens, tau, et, n_target=w, max_pop=cp[i], uids=np.arange(w) + uid0[i])
        print("   system %d: pop %s oracle %s" % (i, hist[:, i, 0].astype(int).tolist(), ref.pop.tolist()))
        assert np.array_equal(hist[:, i, 0].astype(int), ref.pop)
        for q, r in ((1, ref.wsum), (2, ref.e_est), (3, ref.e_t)):
            assert np.all(np.abs(hist[:, i, q] - r) <= 1e-10 * np.maximum(1.0, np.abs(r))), (i, q)
        assert np.array_equal(uids[off:off + len(ref.uids)], ref.uids)
        off += len(ref.uids)
    grp.close()
    for g in systems:
        g.close()
