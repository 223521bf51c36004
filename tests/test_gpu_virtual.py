"""GPU parity of the ratio-only virtual moves (cq_crowd_virtual_ratios: the wavefunction ratios
at quadrature points around every electron, the non-local shape of the local-energy step of
Alg. 1) against the FP64 oracle on the same configurations.

FP64: ratio, rho_D and dlnJ within 1e-10 relative (of max(1, |x|)), at set-up and after VMC
sweeps (the GPU's inverse is then its update chain, the oracle's a fresh LU: they agree to the
chain's rounding), for one and several orbital passes per thread (N = 32, 256, 1024).
Mixed precision (FP32 table and inverse, FP64 sums of the products): the relative ratio errors
at set-up stay within factors 2 (median, p99) and 3 (p99.9, max over |rho| >= 0.1) of those of
the rounding model on the same state (rows evaluated in FP32 arithmetic, the FP64 inverse of
those rows stored in FP32, the products summed in FP64), and dlnJ within the FP32 bound of the
FP64 value: 2 (Ne - 1) pair terms, each formed in FP32 with about four roundings of a value
below max(a)/b, give at most 8 (Ne - 1) 2^-24 max(a)/b.
"""
import dataclasses

import numpy as np
import pytest

import oracle as orc
import paper_2209_14487_amd as cq
from oracle import fp32_chain
from synth import J2_A_ANTI, J2_A_PAR, J2_B, icosahedron_offsets, start_positions

pytestmark = pytest.mark.gpu


def pair(n, L, G, seed, eb):
    g = cq.System(n, L)
    g.fill_philox(seed, eb, G)
    g.load_j2(J2_A_PAR, J2_A_ANTI, J2_B)
    o = orc.System(n, n, L, G=G, n_orb=n, orb_kind=orc.ORB_SEEDED, coef_seed=seed, use_j2=True,
                   j2_a_par=J2_A_PAR, j2_a_anti=J2_A_ANTI, j2_b=J2_B, seed=seed, coef_fp32=(eb == 4))
    return g, o


def rel(a, b):
    return np.abs(a - b) / np.maximum(1.0, np.abs(b))


@pytest.mark.parametrize("n,L,G,W,sweeps", [(32, 10.0, 48, 16, 0), (32, 10.0, 48, 16, 3), (256, 20.0, 64, 3, 1),
                                            (1024, 32.0, 96, 2, 0)])
def test_virtual_ratios_fp64_match_oracle(n, L, G, W, sweeps):
    seed = 1002
    g, o = pair(n, L, G, seed, 8)
    R0 = start_positions(seed, W, 2 * n, L)
    crowd = cq.Crowd(g, W, precision="fp64", delay_rank=8, seed=seed, path="batch")
    crowd.set_positions(R0)
    if sweeps:
        crowd.run_vmc(sweeps, 0.5)
    R = crowd.positions()
    off = np.vstack([icosahedron_offsets(0.5), [[0.0, 0.0, 0.0]]])  # the last point: r_e itself
    got = crowd.virtual_ratios(off)
    ref = orc.virtual_ratios(o, R, off, n_threads=8)
    errs = [rel(a, b).max() for a, b in zip(got, ref)]
    print("   N=%d after %d sweeps: max rel err ratio %.2e rho %.2e dlnJ %.2e" % (n, sweeps, *errs))
    assert max(errs) < 1e-10
    # the point r_e itself: rho_D = 1 and dlnJ = 0 (the current row against its own inverse column)
    assert np.abs(got[1][:, :, -1] - 1.0).max() < 1e-9 and np.abs(got[2][:, :, -1]).max() < 1e-12
    crowd.close()
    g.close()


@pytest.mark.parametrize("n,L,G,W", [(32, 10.0, 48, 8), (256, 20.0, 64, 2)])
def test_virtual_ratios_mixed_within_fp32_rounding(n, L, G, W):
    seed = 1003
    g, o = pair(n, L, G, seed, 4)
    R0 = start_positions(seed, W, 2 * n, L)
    crowd = cq.Crowd(g, W, precision="mixed", delay_rank=8, seed=seed, path="batch")
    crowd.set_positions(R0)
    off = icosahedron_offsets(0.5)
    got = crowd.virtual_ratios(off)
    ref = orc.virtual_ratios(o, R0, off, n_threads=8)
    # the rounding model on the same state
    emu = np.zeros_like(ref[1])
    for w in range(W):
        for sp in range(2):
            rows = np.array([orc.orbital_vgl_f32(o, R0[w, sp * n + i], n)[0] for i in range(n)])
            inv = np.linalg.inv(rows).astype(np.float32).astype(np.float64)  # inv[j][i] = (A^-1)[j][i]
            for i in range(n):
                e = sp * n + i
                for q in range(off.shape[0]):
                    rq = np.mod(R0[w, e] + off[q], L)
                    emu[w, e, q] = float(orc.orbital_vgl_f32(o, rq, n)[0] @ inv[:, i])
    gs = fp32_chain.ratio_error_stats(got[1], ref[1], floor=0.1)
    es = fp32_chain.ratio_error_stats(emu, ref[1], floor=0.1)
    print("   N=%d rho_D rel err GPU %s | model %s" % (n, " ".join("%s=%.2e" % (q, gs[q]) for q in ("median", "p99", "p999", "max")),
                                                     " ".join("%s=%.2e" % (q, es[q]) for q in ("median", "p99", "p999", "max"))))
    for q, f in dict(median=2.0, p99=2.0, p999=3.0, max=3.0).items():
        assert gs[q] <= f * es[q], (q, gs, es)
    jbound = 8 * (2 * n - 1) * 2.0 ** -24 * max(J2_A_PAR, J2_A_ANTI) / J2_B
    jerr = np.abs(got[2] - ref[2]).max()
    print("   dlnJ max abs err %.2e (bound %.2e)" % (jerr, jbound))
    assert jerr <= jbound
    assert np.allclose(got[0], got[1] * np.exp(got[2]), rtol=1e-12)
    crowd.close()
    g.close()
