"""GPU parity of the complex-orbital path (Bloch orbitals with a twist in a triclinic cell,
cq_csystem / cq_ccrowd) against the complex FP64 oracle (oracle/complex_oracle.py, pinned in
test_complex_oracle_pins: plane-wave eigenstates, Marsden reproduction, finite differences
of the Cartesian derivatives and of Psi, determinant ratios, slogdet).

FP64 on both sides: set-up log|det|, phase, inverses and the complex E_L within 1e-10
(relative to max(1, |value|)); over VMC sweeps identical decisions except at near-ties, and
complex ratios, ln J changes, acceptance probabilities, log|det|, phase and E_L within 1e-10.
The mixed crowds read complex64 coefficients and do every sum in FP64; the oracle takes the
same coefficients (the complex64 table widened to complex128), so the same 1e-10 bar holds.
"""
import numpy as np
import pytest

import paper_2209_14487_amd as cq
from oracle import complex_oracle as co
from synth import TRICLINIC, cell_positions, complex_table

pytestmark = pytest.mark.gpu

TWIST = np.array([0.11, -0.07, 0.05])
NEAR_TIE = 1e-6


def rel(a, b):
    return np.abs(np.asarray(a) - np.asarray(b)) / np.maximum(1.0, np.abs(np.asarray(b)))


def pair(n, G, seed, lattice=TRICLINIC, twist=TWIST, j2=True, precision="fp64"):
    table = complex_table(seed, G, n)
    if precision == "mixed":
        table = table.astype(np.complex64)
    g = cq.ComplexSystem(n, lattice, twist)
    g.load_table(table)
    o = co.CSystem(n, lattice, twist, table=table.astype(np.complex128), use_j2=j2, seed=seed)
    if j2:
        g.load_j2(o.j2_a_par, o.j2_a_anti, o.j2_b)
    return g, o


def phase_diff(a, b):
    return np.abs(np.exp(1j * np.asarray(a)) - np.exp(1j * np.asarray(b)))


@pytest.mark.parametrize("n,G,W,precision", [(4, 8, 6, "fp64"), (32, 16, 8, "fp64"), (33, 10, 3, "fp64"),
                                             (64, 12, 4, "fp64"), (96, 10, 2, "fp64"), (32, 16, 8, "mixed"),
                                             (96, 10, 2, "mixed")])
def test_setup_matches_oracle(n, G, W, precision):
    seed = 1500 + n
    g, o = pair(n, G, seed, precision=precision)
    R0 = cell_positions(seed, W, 2 * n, TRICLINIC)
    crowd = cq.ComplexCrowd(g, W, seed=seed, precision=precision)
    crowd.set_positions(R0)
    ld, ph = crowd.logdet()
    el = crowd.local_energy()
    for w in range(W):
        ainv, ld0, ph0, el0 = co.setup(o, R0[w])
        assert np.all(rel(ld[w], ld0) < 1e-10), w
        assert np.all(phase_diff(ph[w], ph0) < 1e-10), w
        assert rel(el[w], el0) < 1e-10, (w, el[w], el0)
        for spin in range(2):
            inv = crowd.inverse(w, spin)
            assert np.abs(inv - ainv[spin]).max() < 1e-10 * max(1.0, np.abs(ainv[spin]).max())
    crowd.close()
    g.close()


@pytest.mark.parametrize("n,G,W,S,sigma,twisted,precision", [
    (4, 8, 8, 4, 1.0, True, "fp64"), (32, 16, 6, 2, 0.5, True, "fp64"), (32, 16, 4, 2, 0.5, False, "fp64"),
    (33, 10, 3, 1, 0.5, True, "fp64"), (64, 12, 3, 1, 0.4, True, "fp64"), (96, 10, 2, 1, 0.4, True, "fp64"),
    (32, 16, 6, 2, 0.5, True, "mixed"), (64, 12, 3, 1, 0.4, True, "mixed")])
def test_vmc_chain_matches_oracle(n, G, W, S, sigma, twisted, precision):
    seed = 1600 + n
    g, o = pair(n, G, seed, twist=TWIST if twisted else np.zeros(3), precision=precision)
    R0 = cell_positions(seed, W, 2 * n, TRICLINIC)
    crowd = cq.ComplexCrowd(g, W, seed=seed, precision=precision)
    crowd.set_positions(R0)
    crowd.record(S)
    ld = np.zeros((S, W, 2))
    ph = np.zeros((S, W, 2))
    el = np.zeros((S, W), np.complex128)
    for s in range(S):
        crowd.run_vmc(1, sigma)
        ld[s], ph[s] = crowd.logdet()
        el[s] = crowd.local_energy()
    rec = crowd.records()
    ref = co.vmc(o, R0, S, sigma=sigma)
    ne = 2 * n
    acc_rate = ref.acc.mean()
    print("   N=%d acceptance %.3f" % (n, acc_rate))
    assert 0.05 < acc_rate < 0.95
    for w in range(W):
        a_g = rec["acc"][:, :, w].ravel()
        a_r = ref.acc[:, :, w].ravel()
        d = np.nonzero(a_g != a_r)[0]
        lim = S * ne if len(d) == 0 else int(d[0])
        if len(d):
            s, e = divmod(lim, ne)
            assert abs(ref.prob[s, e, w] - ref.u[s, e, w]) < NEAR_TIE, "decision differs away from a near-tie"
        for key in ("rho", "dlnj", "prob"):
            a = rec[key][:, :, w].ravel()[:lim]
            b = getattr(ref, key)[:, :, w].ravel()[:lim]
            assert np.all(rel(a, b) <= 1e-10), (w, key, rel(a, b).max())
        full = lim // ne
        for s in range(full):
            assert np.all(rel(ld[s, w], ref.logdet[s, w]) < 1e-10), (w, s)
            assert np.all(phase_diff(ph[s, w], ref.phase[s, w]) < 1e-10), (w, s)
            assert rel(el[s, w], ref.eloc[s, w]) < 1e-10, (w, s, el[s, w], ref.eloc[s, w])
        if len(d) == 0:
            assert np.abs(crowd.positions()[w] - ref.R[w]).max() < 1e-12 * np.abs(TRICLINIC).max()
    acc, prop = crowd.acceptance()
    assert np.all(prop == S * ne)
    # the FP64 recompute agrees with the kept log|det| (Sherman-Morrison drift only)
    assert crowd.recompute() < 1e-9
    crowd.close()
    g.close()


def test_complex_path_arguments():
    """Bad cells, twists, tables and positions are refused; a singular start names the walker."""
    with pytest.raises(cq.CqError) as ei:
        cq.ComplexSystem(4, np.array([[1.0, 0, 0], [2.0, 0, 0], [0, 0, 1.0]]))
    assert ei.value.status == cq.CQ_EINVAL
    with pytest.raises(cq.CqError) as ei:
        cq.ComplexSystem(4, TRICLINIC, (0.0, np.nan, 0.0))
    assert ei.value.status == cq.CQ_EINVAL
    with pytest.raises(cq.CqError) as ei:
        cq.ComplexSystem(513, TRICLINIC)
    assert ei.value.status == cq.CQ_EINVAL
    g = cq.ComplexSystem(4, TRICLINIC, TWIST)
    with pytest.raises(cq.CqError) as ei:
        cq.ComplexCrowd(g, 2)  # no table yet
    assert ei.value.status == cq.CQ_EINVAL
    g.load_table(complex_table(1, 8, 4).astype(np.complex64))
    with pytest.raises(cq.CqError) as ei:
        cq.ComplexCrowd(g, 2, precision="fp64")  # only the complex64 table
    assert ei.value.status == cq.CQ_EINVAL
    with pytest.raises(cq.CqError) as ei:
        g.load_table(complex_table(1, 10, 4))  # a second table on another grid
    assert ei.value.status == cq.CQ_EINVAL
    with pytest.raises(cq.CqError) as ei:
        g.load_table(complex_table(1, 8, 5))
    assert ei.value.status == cq.CQ_EINVAL
    g.load_table(complex_table(1, 8, 4))
    crowd = cq.ComplexCrowd(g, 2, seed=1)
    with pytest.raises(cq.CqError) as ei:
        crowd.run_vmc(1, 0.5)
    assert ei.value.status == cq.CQ_ESTATE
    R0 = cell_positions(1, 2, 8, TRICLINIC)
    R0[1, 1] = R0[1, 0]  # two up electrons at one point: A is singular
    with pytest.raises(cq.CqError) as ei:
        crowd.set_positions(R0)
    assert ei.value.status == cq.CQ_ESINGULAR and "walker 1" in str(ei.value)
    crowd.close()
    g.close()
