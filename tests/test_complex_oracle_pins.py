"""Pins of the complex-orbital oracle (oracle/complex_oracle.py) against what the mathematics
fixes, independently of the oracle's own formulas (CPU only):

* analytic plane waves with a twist in a triclinic cell are kinetic eigenfunctions: E_L is
  sum |q_j|^2 / 2 exactly, with no imaginary part;
* the spline reproduces tensor-product cubics (Marsden) in fractional coordinates;
* the Cartesian gradient and Laplacian (full Hessian through the cell metric, twist phase)
  agree with finite differences of the orbital values;
* in a cubic cell, with no twist and a real table, the orbitals are the real oracle's;
* the minimum image is a lattice translate inside the half cell;
* the chain's Sherman-Morrison ratios equal ratios of two determinants and full pair sums,
  and its log|det| and phase equal slogdet of the final matrices;
* the complex local energy equals -1/2 sum lap Psi / Psi by finite differences of Psi.
"""
import numpy as np
import pytest

import oracle as orc
from oracle import complex_oracle as co
from synth import TRICLINIC, cell_positions, complex_table, planewave_table, start_positions

TWIST = np.array([0.11, -0.07, 0.05])


def rel(a, b):
    return np.abs(np.asarray(a) - np.asarray(b)) / np.maximum(1.0, np.abs(np.asarray(b)))


def interior_positions(seed, k, lattice, G, lo=0.2, hi=0.8):
    """Points whose fractional grid coordinate is at least 0.2 of a cell from a knot on every
    axis (and away from the cell's faces), so that finite differences stay on one polynomial
    piece of the spline."""
    rng = np.random.default_rng(seed)
    i = rng.integers(1, G - 2, size=(k, 3))
    t = rng.uniform(lo, hi, size=(k, 3))
    return ((i + t) / G) @ lattice


def test_plane_waves_with_a_twist_in_a_triclinic_cell_are_eigenstates():
    waves = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, -1]])
    sys = co.CSystem(4, TRICLINIC, TWIST, waves=waves)
    q = 2 * np.pi * waves @ np.linalg.inv(TRICLINIC).T + TWIST
    e0 = 2 * 0.5 * np.sum(q * q)  # both spins
    R = cell_positions(3, 3, 8, TRICLINIC)
    for w in range(3):
        el = co.setup(sys, R[w])[3]
        assert abs(el.real - e0) < 1e-10 * e0 and abs(el.imag) < 1e-10 * e0


def test_spline_reproduces_tensor_product_cubics():
    G, n = 12, 2
    rng = np.random.default_rng(5)
    # per axis and orbital a complex cubic in the grid coordinate x = f G
    P = rng.normal(size=(3, n, 4)) + 1j * rng.normal(size=(3, n, 4))  # coefficients of x^0..x^3
    poly = lambda c, x: c[0] + c[1] * x + c[2] * x ** 2 + c[3] * x ** 3
    dpoly = lambda c, x: c[1] + 2 * c[2] * x + 3 * c[3] * x ** 2
    d2poly = lambda c, x: 2 * c[2] + 6 * c[3] * x
    q = np.arange(G, dtype=np.float64)
    # Marsden: control value p(q) - p''(q) / 6 reproduces the cubic p (unit knot spacing)
    ctrl = np.array([[poly(P[a, j], q) - d2poly(P[a, j], q) / 6.0 for j in range(n)] for a in range(3)])
    table = np.einsum("jx,jy,jz->xyzj", ctrl[0], ctrl[1], ctrl[2])
    sys = co.CSystem(n, TRICLINIC, table=table)
    for r in interior_positions(9, 6, TRICLINIC, G):
        f = r @ np.linalg.inv(TRICLINIC)
        x = f * G
        s, gf, H = co.periodic_part(sys, r)
        for j in range(n):
            vals = [poly(P[a, j], x[a]) for a in range(3)]
            d1 = [dpoly(P[a, j], x[a]) * G for a in range(3)]
            d2 = [d2poly(P[a, j], x[a]) * G * G for a in range(3)]
            assert abs(s[j] - vals[0] * vals[1] * vals[2]) < 1e-11 * abs(s[j])
            for a in range(3):
                o = [vals[0], vals[1], vals[2]]
                o[a] = d1[a]
                assert abs(gf[j, a] - o[0] * o[1] * o[2]) < 1e-10 * np.abs(gf[j]).max()
                for b in range(3):
                    o = [vals[0], vals[1], vals[2]]
                    if a == b:
                        o[a] = d2[a]
                    else:
                        o[a], o[b] = d1[a], d1[b]
                    assert abs(H[j, a, b] - o[0] * o[1] * o[2]) < 1e-10 * np.abs(H[j]).max()


def test_cartesian_derivatives_match_finite_differences():
    G, n = 10, 3
    sys = co.CSystem(n, TRICLINIC, TWIST, table=complex_table(21, G, n))
    h = 2e-3
    for r in interior_positions(4, 5, TRICLINIC, G):
        v, g, l = co.orbitals(sys, r)
        lap_fd = np.zeros(n, np.complex128)
        for c in range(3):
            e = np.zeros(3)
            e[c] = h
            f = {m: co.orbitals(sys, r + m * e)[0] for m in (-2, -1, 1, 2)}
            d1 = (-f[2] + 8 * f[1] - 8 * f[-1] + f[-2]) / (12 * h)
            d2 = (-f[2] + 16 * f[1] - 30 * v + 16 * f[-1] - f[-2]) / (12 * h * h)
            assert np.all(np.abs(d1 - g[:, c]) < 1e-7 * np.abs(g).max()), c
            lap_fd += d2
        assert np.all(np.abs(lap_fd - l) < 1e-6 * np.abs(l).max())


def test_cubic_cell_without_twist_is_the_real_oracle():
    G, L, n = 16, 5.0, 4
    table = planewave_table(G, L)
    sys = co.CSystem(n, L * np.eye(3), table=table.astype(np.complex128))
    osys = orc.System(n, n, L, G=G, n_orb=n, orb_kind=orc.ORB_TABLE, table=table)
    for r in start_positions(8, 1, 6, L)[0]:
        v, g, l = co.orbitals(sys, r)
        v0, g0, l0 = orc.orbital_vgl(osys, r)
        assert np.all(np.abs(v.imag) == 0) and np.all(np.abs(g.imag) == 0) and np.all(np.abs(l.imag) == 0)
        assert np.all(rel(v.real, v0) < 1e-13) and np.all(rel(g.real, g0) < 1e-12) and np.all(rel(l.real, l0) < 1e-12)


def test_minimum_image_is_a_lattice_translate_in_the_half_cell():
    sys = co.CSystem(1, TRICLINIC)
    rng = np.random.default_rng(2)
    for d in rng.uniform(-30.0, 30.0, size=(200, 3)):
        m = co.min_image(sys, d)
        k = (d - m) @ np.linalg.inv(TRICLINIC)
        assert np.all(np.abs(k - np.rint(k)) < 1e-12)
        assert np.all(np.abs(m @ np.linalg.inv(TRICLINIC)) <= 0.5 + 1e-12)


def test_chain_ratios_equal_determinant_ratios():
    n, G, W, S, seed = 4, 8, 2, 2, 31
    sys = co.CSystem(n, TRICLINIC, TWIST, table=complex_table(seed, G, n), use_j2=True, seed=seed)
    R0 = cell_positions(seed, W, 2 * n, TRICLINIC)
    res = co.vmc(sys, R0, S, sigma=1.2)
    assert 0.05 < res.acc.mean() < 0.95
    for w in range(W):
        R = R0[w].copy()
        for s in range(S):
            for e in range(2 * n):
                z = orc.gauss3(seed, w, s, e)
                rp = co.wrap(sys, R[e] + 1.2 * z)
                rho, dj = co.direct_ratio(sys, R, e, rp)
                assert abs(res.rho[s, e, w] - rho) < 1e-10 * max(1.0, abs(rho))
                assert abs(res.dlnj[s, e, w] - dj) < 1e-12 * max(1.0, abs(dj))
                if res.acc[s, e, w]:
                    R[e] = rp
            for spin in range(2):
                sgn, lab = np.linalg.slogdet(co.slater(sys, R, spin)[0])
                assert abs(res.logdet[s, w, spin] - lab) < 1e-10 * max(1.0, abs(lab))
                assert abs(np.exp(1j * res.phase[s, w, spin]) - sgn) < 1e-10
        assert np.allclose(res.R[w], R, rtol=0, atol=0)


def test_complex_local_energy_matches_finite_differences():
    n, G, seed = 3, 8, 41
    sys = co.CSystem(n, TRICLINIC, TWIST, table=complex_table(seed, G, n), use_j2=True, seed=seed)
    R = interior_positions(seed, 2 * n, TRICLINIC, G, lo=0.3, hi=0.7)
    el = co.setup(sys, R)[3]
    h = 1e-3

    def psi_ratio(R1):  # Psi(R1) / Psi(R)
        out = np.exp(co.lnj(sys, R1) - co.lnj(sys, R))
        for spin in range(2):
            s0, l0 = np.linalg.slogdet(co.slater(sys, R, spin)[0])
            s1, l1 = np.linalg.slogdet(co.slater(sys, R1, spin)[0])
            out *= (s1 / s0) * np.exp(l1 - l0)
        return out

    lap = 0.0
    for i in range(2 * n):
        for c in range(3):
            f = {}
            for m in (-2, -1, 1, 2):
                R1 = R.copy()
                R1[i, c] += m * h
                f[m] = psi_ratio(R1)
            lap += (-f[2] + 16 * f[1] - 30.0 + 16 * f[-1] - f[-2]) / (12 * h * h)
    el_fd = -0.5 * lap
    print("   E_L", el, "finite differences", el_fd)
    assert abs(el - el_fd) < 1e-5 * max(1.0, abs(el))
