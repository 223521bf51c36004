"""Pins of the FP64 CPU oracle against what the mathematics fixes (CPU only).

Each test checks the oracle against something other than itself: published
known-answer vectors, closed forms, invariants, a textbook library routine, or
the brute-force second reference in ``oracle/direct.py``.
"""
import os

import numpy as np
import pytest

import oracle as orc
from oracle.direct import Direct, spline_vgl
from synth import planewave_table, start_positions

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _golden_numbers(name):
    vals = []
    for line in open(os.path.join(GOLD, name)):
        line = line.strip()
        if line and not line.startswith("#"):
            vals.append(line.split())
    return vals


# ---------------------------------------------------------------- Philox / RNG

def test_philox_known_answers():
    """Philox4x32-10 reproduces the published Random123 known-answer vectors."""
    rows = _golden_numbers("philox4x32_10_kat.txt")
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        assert orc.philox4x32_10(v[0:4], v[4:6]) == v[6:10]


def test_uniform53_endpoints():
    assert orc.uniform53(0, 0) == 0.0
    assert orc.uniform53(0xFFFFFFFF, 0xFFFFFFFF) == 1.0 - 2.0 ** -53
    # only the top 53 bits count: the low 11 bits of the low word are dropped
    assert orc.uniform53(0x7FF, 0) == 0.0
    assert orc.uniform53(0x800, 0) == 2.0 ** -53


def test_gaussian_moments():
    z = np.array([orc.gauss3(7, uid, 3, e) for uid in range(40) for e in range(100)])
    assert abs(z.mean()) < 0.04
    assert abs(z.var() - 1.0) < 0.05
    # components are independent
    assert abs(np.corrcoef(z.T)[0, 1]) < 0.05 and abs(np.corrcoef(z.T)[0, 2]) < 0.05


def test_coefficients_in_range_and_fp32_rounding():
    c = np.array([orc.coef(1002, i) for i in range(5000)])
    assert c.min() >= -1.0 and c.max() < 1.0
    assert abs(c.mean()) < 0.05
    # the FP32 table holds the round-to-nearest value of the FP64 coefficient
    sys64 = orc.System(1, 1, 10.0, G=4, n_orb=2, orb_kind=orc.ORB_SEEDED, coef_seed=1002)
    sys32 = orc.System(1, 1, 10.0, G=4, n_orb=2, orb_kind=orc.ORB_SEEDED, coef_seed=1002, coef_fp32=True)
    # at a grid node the value is (c_{i-1} + 4 c_i + c_{i+1}) / 6 per axis; compare both paths
    r = np.array([2.5, 5.0, 7.5])
    v64, _, _ = orc.orbital_vgl(sys64, r)
    v32, _, _ = orc.orbital_vgl(sys32, r)
    assert np.all(np.abs(v64 - v32) < 1e-7) and np.any(v64 != v32)


# ------------------------------------------------------------------- splines

def _cubic_reproduction_table(G, L, coeffs):
    """Per-axis control values c_j = p(x_j) - (h^2/6) p''(x_j) reproduce a cubic p exactly
    (Marsden identity); the 3-D table is the tensor product for p = px(x) py(y) pz(z)."""
    h = L / G
    x = np.arange(G) * h
    tab = np.zeros((G, G, G, len(coeffs)))
    for n, (cx, cy, cz) in enumerate(coeffs):
        ax = []
        for c in (cx, cy, cz):
            p = np.polynomial.Polynomial(c)
            ax.append(p(x) - h * h / 6.0 * p.deriv(2)(x))
        tab[..., n] = ax[0][:, None, None] * ax[1][None, :, None] * ax[2][None, None, :]
    return tab


def _poly_vgl(coeffs, r):
    v, g, l = [], [], []
    for cx, cy, cz in coeffs:
        P = [np.polynomial.Polynomial(c) for c in (cx, cy, cz)]
        f = [P[a](r[a]) for a in range(3)]
        d1 = [P[a].deriv(1)(r[a]) for a in range(3)]
        d2 = [P[a].deriv(2)(r[a]) for a in range(3)]
        v.append(f[0] * f[1] * f[2])
        g.append([d1[0] * f[1] * f[2], f[0] * d1[1] * f[2], f[0] * f[1] * d1[2]])
        l.append(d2[0] * f[1] * f[2] + f[0] * d2[1] * f[2] + f[0] * f[1] * d2[2])
    return np.array(v), np.array(g), np.array(l)


def test_spline_cubic_reproduction():
    """P1: cubic polynomials are reproduced exactly (value, gradient, Laplacian)."""
    G, L = 12, 6.0
    h = L / G
    rng = np.random.default_rng(1)
    coeffs = [tuple(rng.uniform(-1, 1, 4) for _ in range(3)) for _ in range(5)]
    tab = _cubic_reproduction_table(G, L, coeffs)
    s = orc.System(1, 1, L, G=G, n_orb=5, orb_kind=orc.ORB_TABLE, table=tab)
    for _ in range(30):
        # keep the 4-point stencil (i-1 .. i+2) inside the grid: no wrap
        r = rng.uniform(h, (G - 2) * h - 1e-9, 3)
        v, g, l = orc.orbital_vgl(s, r)
        ve, ge, le = _poly_vgl(coeffs, r)
        scale = 1.0 + np.abs(ve).max()
        assert np.allclose(v, ve, atol=1e-12 * scale, rtol=0)
        assert np.allclose(g, ge, atol=1e-11 * scale, rtol=0)
        assert np.allclose(l, le, atol=1e-10 * scale, rtol=0)


def test_spline_partition_of_unity():
    """P2: constant coefficients give a constant orbital, zero gradient and Laplacian."""
    G, L = 8, 4.0
    tab = np.full((G, G, G, 3), 0.0)
    tab[..., 0] = 1.0
    tab[..., 1] = -2.5
    tab[..., 2] = 0.125
    s = orc.System(1, 1, L, G=G, n_orb=3, orb_kind=orc.ORB_TABLE, table=tab)
    rng = np.random.default_rng(2)
    for r in list(rng.uniform(-3 * L, 3 * L, (20, 3))) + [np.array([L, 0.0, L - 1e-15]), np.zeros(3)]:
        v, g, l = orc.orbital_vgl(s, r)
        assert np.allclose(v, [1.0, -2.5, 0.125], atol=1e-14)
        assert np.abs(g).max() < 1e-13 and np.abs(l).max() < 1e-12


def test_spline_prefilter_interpolates_nodes():
    """P3: the closed-form prefilter makes the spline interpolate the plane waves at nodes,
    and the per-orbital -S''/S at nodes exceeds k^2 by the printed closed-form excess."""
    L = 5.0
    excess = [float(x) for x in _golden_numbers("planewave_c1_energy.txt")[1]]
    for G, exc in zip((16, 32, 64), excess):
        tab = planewave_table(G, L)
        s = orc.System(1, 1, L, G=G, n_orb=4, orb_kind=orc.ORB_TABLE, table=tab)
        h = L / G
        k = 2 * np.pi / L
        for (i, j, m) in [(0, 0, 0), (3, 5, 7), (G - 1, 1, G // 2)]:
            r = np.array([i * h, j * h, m * h])
            v, g, l = orc.orbital_vgl(s, r)
            f = np.array([1.0, np.cos(k * r[0]), np.sin(k * r[0]), np.cos(k * r[1])])
            assert np.allclose(v, f, atol=1e-13)
            # -S''/S = k^2 (1 + excess) wherever S != 0
            for n in (1, 2, 3):
                if abs(v[n]) > 0.1:
                    assert abs(-l[n] / v[n] / k ** 2 - 1.0 - exc) < 2e-6
        # gradient and Laplacian are consistent with finite differences of the value
        r = np.array([0.3, 1.7, 4.1])
        d = 1e-5
        v0, g0, l0 = orc.orbital_vgl(s, r)
        lap_fd = np.zeros(4)
        for c in range(3):
            e = np.zeros(3); e[c] = d
            vp, _, _ = orc.orbital_vgl(s, r + e)
            vm, _, _ = orc.orbital_vgl(s, r - e)
            assert np.allclose((vp - vm) / (2 * d), g0[:, c], atol=1e-7)
            lap_fd += (vp - 2 * v0 + vm) / d ** 2
        assert np.allclose(lap_fd, l0, atol=2e-4)


def test_spline_matches_basis_matrix_form():
    """The oracle's expanded polynomial weights agree with the basis-matrix form on random,
    wrapping inputs (two independent codings of the same definition)."""
    G, L = 7, 3.5
    rng = np.random.default_rng(3)
    tab = rng.uniform(-1, 1, (G, G, G, 6))
    s = orc.System(1, 1, L, G=G, n_orb=6, orb_kind=orc.ORB_TABLE, table=tab)
    pts = list(rng.uniform(-L, 2 * L, (40, 3))) + [np.array([L, L, L]), np.array([0.0, L - 1e-14, 1e-300])]
    for r in pts:
        v, g, l = orc.orbital_vgl(s, r)
        v2, g2, l2 = spline_vgl(tab, L, r)
        assert np.allclose(v, v2, atol=1e-13) and np.allclose(g, g2, atol=1e-12)
        assert np.allclose(l, l2, atol=1e-10)


def test_seeded_table_matches_materialised_table():
    """orb_kind=seeded evaluates coefficient idx = ((ix G + iy) G + iz) n_orb + n on the fly."""
    G, L, n = 5, 2.0, 3
    tab = np.array([orc.coef(99, i) for i in range(G ** 3 * n)]).reshape(G, G, G, n)
    s1 = orc.System(1, 1, L, G=G, n_orb=n, orb_kind=orc.ORB_SEEDED, coef_seed=99)
    s2 = orc.System(1, 1, L, G=G, n_orb=n, orb_kind=orc.ORB_TABLE, table=tab)
    for r in np.random.default_rng(4).uniform(0, L, (10, 3)):
        a = orc.orbital_vgl(s1, r)
        b = orc.orbital_vgl(s2, r)
        for x, y in zip(a, b):
            assert np.array_equal(x, y)


# ------------------------------------------------------------------------ LU

def test_lu_inverse_logdet_sign():
    rng = np.random.default_rng(5)
    for n in (1, 2, 5, 20, 64):
        A = rng.standard_normal((n, n))
        inv, ld, sg = orc.lu_inverse(A)
        s_np, ld_np = np.linalg.slogdet(A)
        assert abs(ld - ld_np) < 1e-11 * max(1, abs(ld_np))
        assert sg == int(s_np)
        assert np.abs(A @ inv - np.eye(n)).max() < 1e-10
    # permutation matrix: |det| = 1, sign = parity
    P = np.eye(4)[[1, 0, 3, 2]]
    inv, ld, sg = orc.lu_inverse(P)
    assert ld == 0.0 and sg == 1 and np.array_equal(inv, P.T)
    P = np.eye(3)[[1, 2, 0]]
    assert orc.lu_inverse(P)[2] == 1
    P = np.eye(3)[[1, 0, 2]]
    assert orc.lu_inverse(P)[2] == -1
    with pytest.raises(ZeroDivisionError):
        orc.lu_inverse(np.array([[1.0, 2.0], [2.0, 4.0]]))


# ------------------------------------------------------- chain vs brute force

# one-body Jastrow centres for the pins (a1 < 0: the electrons are drawn to them)
J1_IONS = np.array([[0.7, 1.1, 2.9], [3.1, 2.6, 0.4], [1.9, 3.7, 1.6]])
J1_A, J1_B = -0.8, 1.3


def _tiny_system(n, G=8, L=4.0, j2=True, seed=11, j1=False):
    tab = np.random.default_rng(seed).uniform(-1, 1, (G, G, G, n))
    ions = J1_IONS if j1 else None
    s = orc.System(n, n, L, G=G, n_orb=n, orb_kind=orc.ORB_TABLE, table=tab, use_j2=j2, seed=seed, ions=ions,
                   j1_a=J1_A, j1_b=J1_B)
    d = Direct(n, n, L, table=tab, use_j2=j2, seed=seed, ions=ions, j1_a=J1_A, j1_b=J1_B)
    return s, d


def _exact_solve(A, b):
    """Gauss-Jordan elimination in exact rational arithmetic (the float entries converted exactly)."""
    from fractions import Fraction
    n = len(b)
    M = [[Fraction(float(A[r][c])) for c in range(n)] + [Fraction(float(b[r]))] for r in range(n)]
    for c in range(n):
        p = next(r for r in range(c, n) if M[r][c] != 0)
        M[c], M[p] = M[p], M[c]
        for r in range(n):
            if r != c and M[r][c] != 0:
                f = M[r][c] / M[c][c]
                M[r] = [x - f * y for x, y in zip(M[r], M[c])]
    return [M[r][n] / M[r][r] for r in range(n)]


def test_refined_row_ratio_matches_exact_rational_value():
    """The refined ratio phi . A^-1 e_i equals the exact rational value for the float matrix to
    1e-13 relative even at cond(A) ~ 1e7 (a 6 x 6 Hilbert matrix), where a plain FP64 solve
    is off by orders of magnitude more; on a well-conditioned random matrix it is exact to 1e-15."""
    from fractions import Fraction
    n = 6
    H = 1.0 / (np.arange(n)[:, None] + np.arange(n)[None, :] + 1.0)
    phi = np.random.default_rng(3).uniform(-1, 1, n)
    for A in (H, np.random.default_rng(4).standard_normal((n, n))):
        for i in (0, 3, n - 1):
            e = np.zeros(n)
            e[i] = 1.0
            x = _exact_solve(A, e)
            exact = float(sum(Fraction(float(p)) * xi for p, xi in zip(phi, x)))
            got = orc.row_ratio_refined(A, i, phi)
            assert abs(got - exact) <= 1e-13 * abs(exact), (i, got, exact)
            col = orc.column_refined(A, i)
            xe = np.array([float(xi) for xi in x])
            assert np.abs(col - xe).max() <= 1e-13 * np.abs(xe).max()
            if A is H:
                plain = float(phi @ np.linalg.solve(A, e))
                assert abs(plain - exact) > 10 * abs(got - exact)


def test_det_ratio_refined_matches_direct_determinants():
    """det_ratio_refined builds A from the orbitals (rows = electrons of the moved electron's spin)
    and equals det(A')/det(A) from two LU determinants, for electrons of both spins."""
    s, d = _tiny_system(3)
    R = start_positions(91, 1, 6, s.L)[0]
    rng = np.random.default_rng(9)
    for e in range(6):
        rnew = np.mod(R[e] + rng.normal(0, 0.5, 3), s.L)
        R2 = R.copy()
        R2[e] = rnew
        sp = 0 if e < 3 else 1
        s1, l1 = np.linalg.slogdet(d.matrices(R)[sp])
        s2, l2 = np.linalg.slogdet(d.matrices(R2)[sp])
        ref = s1 * s2 * np.exp(l2 - l1)
        assert abs(orc.det_ratio_refined(s, R, e, rnew) - ref) <= 1e-12 * max(1.0, abs(ref))


@pytest.mark.parametrize("n,j2,j1", [(1, True, False), (2, False, False), (3, True, False), (2, False, True),
                                     (3, True, True)])
def test_vmc_chain_matches_direct_determinants(n, j2, j1):
    """P4 / P7 / P10: Sherman-Morrison ratios equal det(A')/det(A) from two LUs, the Jastrow
    ratio equals the brute-force difference of full pair (and one-body) sums, the accept
    sequence is the same, and the accumulated log|det| equals slogdet of the final matrices."""
    s, d = _tiny_system(n, j2=j2, j1=j1)
    R0 = start_positions(77, 3, 2 * n, s.L)
    sweeps = 6
    res = orc.vmc(s, R0, sweeps, sigma=0.6)
    for w in range(3):
        ref = d.vmc(R0[w], sweeps, sigma=0.6, uid=w)
        assert np.array_equal(res.acc[:, :, w], ref["acc"])
        assert np.allclose(res.rho[:, :, w], ref["rho"], rtol=1e-10, atol=1e-13)
        assert np.allclose(res.dlnj[:, :, w], ref["dlnj"], rtol=1e-12, atol=1e-13)
        assert np.allclose(res.logdet[:, w, :], ref["logdet"], rtol=1e-10, atol=1e-10)
        assert np.array_equal(res.sign[:, w, :], ref["sign"].astype(np.int32))
        assert np.allclose(res.R[w], ref["R"], atol=1e-14)
    assert 0.2 < res.acc.mean() < 0.95
    if n > 1:
        # the chains cross nodes, so both determinant signs occur
        assert (res.sign == -1).any() and (res.sign == 1).any()


def test_inverse_after_sweeps_matches_direct_inverse():
    """P5: after several sweeps of Sherman-Morrison updates the kept inverse equals inv(A)."""
    n = 6
    s, d = _tiny_system(n, G=10, L=5.0, j2=True, seed=12)
    R0 = start_positions(78, 2, 2 * n, s.L)
    res = orc.vmc(s, R0, 4, sigma=0.5, want_ainv=True)
    assert res.acc.sum() > 10
    for w in range(2):
        mats = d.matrices(res.R[w])
        for sp in range(2):
            ref = np.linalg.inv(mats[sp])
            err = np.abs(res.ainv[w, sp] - ref).max() / np.abs(ref).max()
            assert err < 1e-11


@pytest.mark.parametrize("j1", [False, True])
def test_local_energy_matches_finite_differences(j1):
    """Local energy: the kinetic local energy formula agrees with -1/2 sum lap Psi / Psi by finite
    differences of the directly evaluated wavefunction (splines + J2, and the one-body Jastrow)."""
    n = 2
    s, d = _tiny_system(n, G=8, L=4.0, j2=True, seed=13, j1=j1)
    R0 = start_positions(79, 3, 2 * n, s.L)
    res = orc.vmc(s, R0, 2, sigma=0.5)
    for w in range(3):
        e_fd = d.eloc_fd(res.R[w])
        assert abs(res.eloc[-1, w] - e_fd) < 2e-5 * max(1.0, abs(e_fd))


def test_planewave_local_energy_is_exact_constant():
    """P8: with analytic plane-wave orbitals E_L = sum k_j^2 / 2 = 12 pi^2 / 25 for every walker
    and every sweep."""
    e0 = float(_golden_numbers("planewave_c1_energy.txt")[0][0])
    s = orc.System(4, 4, 5.0, n_orb=4, orb_kind=orc.ORB_PLANEWAVE, seed=1001)
    R0 = start_positions(1001, 8, 8, 5.0)
    res = orc.vmc(s, R0, 5, sigma=0.5)
    assert np.all(np.abs(res.eloc - e0) < 1e-11 * e0)
    ld, sg, el, _ = orc.setup(s, R0)
    assert np.all(np.abs(el - e0) < 1e-11 * e0)
    # and the brute-force finite-difference energy agrees with it
    d = Direct(4, 4, 5.0, planewave=True)
    assert abs(d.eloc_fd(res.R[0]) - e0) < 1e-5


def test_spline_local_energy_converges_as_h2():
    """P9: with the prefiltered spline the local energy approaches 12 pi^2 / 25 as O(h^2):
    about 1 % off at G=16 and about 4x closer at G=32."""
    e0 = float(_golden_numbers("planewave_c1_energy.txt")[0][0])
    R0 = start_positions(1001, 16, 8, 5.0)
    errs = []
    for G in (16, 32):
        s = orc.System(4, 4, 5.0, G=G, n_orb=4, orb_kind=orc.ORB_TABLE, table=planewave_table(G, 5.0),
                       seed=1001)
        res = orc.vmc(s, R0, 3, sigma=0.5)
        errs.append(np.median(np.abs(res.eloc / e0 - 1.0)))
    assert 1e-3 < errs[0] < 5e-2
    assert 2.5 < errs[0] / errs[1] < 6.5


def test_two_electron_jastrow_closed_form():
    """P10: one up and one down electron, constant orbital: E_L = -(u'' + 2u'/r + u'^2) with
    u' = a/(1+br)^2, u'' = -2ab/(1+br)^3 (a = 0.5, b = 1) for r < L/2."""
    G, L = 4, 10.0
    tab = np.ones((G, G, G, 1))
    s = orc.System(1, 1, L, G=G, n_orb=1, orb_kind=orc.ORB_TABLE, table=tab, use_j2=True, seed=5)
    a, b = 0.5, 1.0
    for r in (0.3, 1.0, 2.2, 4.9):
        R = np.array([[[1.0, 2.0, 3.0], [1.0 + r, 2.0, 3.0]]])
        _, _, el, _ = orc.setup(s, R)
        up = a / (1 + b * r) ** 2
        upp = -2 * a * b / (1 + b * r) ** 3
        assert abs(el[0] - (-(upp + 2 * up / r + up * up))) < 1e-13
        # ln J of the pair is u(r) = a r / (1 + b r)
        assert abs(orc.lnj(s, R[0]) - a * r / (1 + b * r)) < 1e-15
    # minimum image: a separation of L - r is the same pair at distance r
    R1 = np.array([[0.5, 0.5, 0.5], [0.5 + L - 1.5, 0.5, 0.5]])
    assert abs(orc.lnj(s, R1) - a * 1.5 / 2.5) < 1e-14


def test_one_body_jastrow_closed_form():
    """One-body Jastrow, one centre, one up and one down electron, constant orbital, no pair term:
    ln J = sum_i u1(r_i) with u1 = a r / (1 + b r), and E_L = sum_i -1/2 (u1'' + 2 u1'/r_i + u1'^2)
    with u1' = a/(1+br)^2, u1'' = -2ab/(1+br)^3, for distances below L/2; a centre seen through the
    box boundary counts at its minimum-image distance."""
    G, L = 4, 10.0
    tab = np.ones((G, G, G, 1))
    a, b = -1.2, 0.7
    ion = np.array([[2.0, 5.0, 5.0]])
    s = orc.System(1, 1, L, G=G, n_orb=1, orb_kind=orc.ORB_TABLE, table=tab, use_j2=False, seed=5, ions=ion,
                   j1_a=a, j1_b=b)

    def parts(r):
        up = a / (1 + b * r) ** 2
        upp = -2 * a * b / (1 + b * r) ** 3
        return a * r / (1 + b * r), -0.5 * (upp + 2 * up / r + up * up)

    for r1, r2 in ((0.4, 3.0), (1.5, 4.6), (2.7, 0.9)):
        R = np.array([[[2.0 + r1, 5.0, 5.0], [2.0, 5.0 - r2, 5.0]]])
        _, _, el, _ = orc.setup(s, R)
        (l1, e1), (l2, e2) = parts(r1), parts(r2)
        assert abs(el[0] - (e1 + e2)) < 1e-13
        assert abs(orc.lnj(s, R[0]) - (l1 + l2)) < 1e-15
    # through the boundary: x = 2 - 1.5 + L sits 1.5 from the centre
    R = np.array([[2.0 - 1.5 + L, 5.0, 5.0], [2.0, 5.0, 5.0 + 0.8]])
    assert abs(orc.lnj(s, R) - (parts(1.5)[0] + parts(0.8)[0])) < 1e-14


def test_metropolis_always_accepts_when_ratio_is_one():
    """P11: constant orbital, no Jastrow: P = 1 so every move is accepted and the trajectory is
    the wrapped Gaussian walk r <- wrap(r + sigma z) of the generator alone."""
    G, L = 4, 3.0
    s = orc.System(1, 1, L, G=G, n_orb=1, orb_kind=orc.ORB_TABLE, table=np.full((G, G, G, 1), 0.7),
                   seed=31)
    R0 = start_positions(5, 2, 2, L)
    res = orc.vmc(s, R0, 25, sigma=0.9, uids=[10, 11], first_step=100)
    assert res.acc.all()
    assert np.allclose(res.prob, 1.0, atol=1e-15)
    for w, uid in enumerate((10, 11)):
        R = R0[w].copy()
        for sw in range(25):
            for e in range(2):
                R[e] = R[e] + 0.9 * orc.gauss3(31, uid, 100 + sw, e)
                R[e] -= L * np.floor(R[e] / L)
        assert np.allclose(res.R[w], R, atol=1e-12)


def test_walker_subsets_and_partial_sweeps_are_consistent():
    """Walkers are independent: a subset run (by uid) reproduces the full run's records, and a
    partial first sweep reproduces its prefix."""
    s, _ = _tiny_system(3, j2=True, seed=14)
    R0 = start_positions(80, 5, 6, s.L)
    full = orc.vmc(s, R0, 2)
    sub = orc.vmc(s, R0[[1, 3]], 2, uids=[1, 3])
    assert np.array_equal(sub.acc, full.acc[:, :, [1, 3]])
    assert np.array_equal(sub.rho, full.rho[:, :, [1, 3]])
    part = orc.vmc(s, R0, 1, max_moves=4)
    assert np.array_equal(part.rho[0, :4], full.rho[0, :4])
    assert np.isnan(part.rho[0, 4:]).all()


# ----------------------------------------------------------------------- DMC

def test_dmc_eigenstate_population_is_constant():
    """P13: for the analytic plane-wave eigenstate with E_T = E0 every branching weight is 1,
    the population never changes and the energy estimate is E0."""
    e0 = float(_golden_numbers("planewave_c1_energy.txt")[0][0])
    s = orc.System(4, 4, 5.0, n_orb=4, orb_kind=orc.ORB_PLANEWAVE, seed=9)
    R0 = start_positions(9, 12, 8, 5.0)
    res = orc.dmc(s, R0, 6, tau=0.01, e_trial=e0, n_target=12)
    assert np.all(res.pop == 12)
    assert np.allclose(res.wsum, 12.0, atol=1e-10)
    assert np.allclose(res.e_est, e0, atol=1e-10)
    assert np.allclose(res.e_t, e0, atol=1e-10)
    assert np.array_equal(res.uids, np.arange(12))
    assert res.n_acc > 0.9 * res.n_prop


def test_dmc_without_drift_is_a_gaussian_walk():
    """With a constant orbital and no Jastrow the drift is zero and P = 1: the DMC move is the
    wrapped Gaussian walk with standard deviation sqrt(tau)."""
    G, L, tau = 4, 3.0, 0.04
    s = orc.System(1, 1, L, G=G, n_orb=1, orb_kind=orc.ORB_TABLE, table=np.full((G, G, G, 1), 1.3),
                   seed=41)
    R0 = start_positions(6, 3, 2, L)
    res = orc.dmc(s, R0, 5, tau=tau, e_trial=0.0, n_target=3)
    assert res.n_acc == res.n_prop == 5 * 3 * 2
    assert np.all(res.pop == 3)
    for w in range(3):
        R = R0[w].copy()
        for g in range(5):
            for e in range(2):
                R[e] = R[e] + np.sqrt(tau) * orc.gauss3(41, w, g, e)
                R[e] -= L * np.floor(R[e] / L)
        assert np.allclose(res.R[w], R, atol=1e-12)


def test_dmc_branching_bookkeeping():
    """Branching multiplicities follow floor(w + u_b) capped at 3, children inherit the parent's
    configuration in population order, copy 0 keeps the parent's uid."""
    s, _ = _tiny_system(2, j2=True, seed=15)
    R0 = start_positions(81, 20, 4, s.L)
    res = orc.dmc(s, R0, 3, tau=0.05, e_trial=0.0, n_target=20)
    assert res.pop[-1] == len(res.uids) > 0
    # every final walker descends from an original uid or is a hashed child uid
    assert len(set(res.uids.tolist())) == len(res.uids)
    # the trial energy update: E_T = E_est - ln(N/N_target)/tau
    assert np.allclose(res.e_t, res.e_est - np.log(res.pop / 20.0) / 0.05, atol=1e-12)


@pytest.mark.parametrize("j1", [False, True])
def test_dmc_drift_matches_finite_differences(j1):
    """The DMC drift grad ln|Psi_T| (determinant part from the inverse column and gradient row,
    plus the Jastrow gradient, one-body terms included) agrees with central differences of the
    direct ln|Psi|."""
    n = 3
    s, d = _tiny_system(n, G=8, L=4.0, j2=True, seed=16, j1=j1)
    R = start_positions(82, 1, 2 * n, s.L)[0]
    for e in range(2 * n):
        v = orc.drift(s, R, e)
        assert np.allclose(v, d.drift_fd(R, e), atol=2e-6 * (1 + np.abs(v).max()))


def test_dmc_acceptance_detailed_balance():
    """Importance-sampled Metropolis-Hastings obeys detailed balance with respect to |Psi_T|^2:
    the acceptance of a move and of its exact reverse multiply to one,
    P(r -> r') P(r' -> r) = 1, for any displacement (Reynolds et al. 1982)."""
    n = 3
    s, _ = _tiny_system(n, G=8, L=4.0, j2=True, seed=17)
    R = start_positions(83, 1, 2 * n, s.L)[0]
    rng = np.random.default_rng(7)
    for tau in (0.01, 0.1):
        for e in range(2 * n):
            delta = rng.normal(0, np.sqrt(tau), 3) + tau * orc.drift(s, R, e)
            p_f, rho_f = orc.dmc_move_prob(s, R, e, delta, tau)
            R2 = R.copy()
            R2[e] = R[e] + delta
            R2[e] -= s.L * np.floor(R2[e] / s.L)
            p_b, rho_b = orc.dmc_move_prob(s, R2, e, -delta, tau)
            assert abs(p_f * p_b - 1.0) < 1e-9
            assert abs(rho_f * rho_b - 1.0) < 1e-9
            # and it is not trivially 1 in each direction
            assert abs(p_f - 1.0) > 1e-6


def test_dmc_branching_multiplicity_cap():
    """With the weight forced above 3 (E_T far above a constant E_L, large tau) every walker
    branches into exactly 3 copies: m = min(3, floor(w + u)), w = exp(tau ecut)."""
    e0 = float(_golden_numbers("planewave_c1_energy.txt")[0][0])
    s = orc.System(4, 4, 5.0, n_orb=4, orb_kind=orc.ORB_PLANEWAVE, seed=19)
    R0 = start_positions(19, 12, 8, 5.0)
    tau = 4.0
    ecut = 0.2 * np.sqrt(8 / tau)
    assert np.exp(tau * ecut) > 3.0
    res = orc.dmc(s, R0, 1, tau=tau, e_trial=e0 + 100.0, n_target=12, max_pop=64)
    assert res.pop[0] == 36
    assert np.allclose(res.wsum[0], 12 * np.exp(tau * ecut), rtol=1e-12)
    # children follow their parent: copies 0, 1, 2 of walker w sit at 3w, 3w+1, 3w+2
    assert np.array_equal(res.uids[::3], np.arange(12))
    assert np.array_equal(res.R[1::3], res.R[::3])
    assert res.uids[1] == orc.child_uid(19, 0, 0, 1)


def test_dmc_reweighting_averages_old_and_new_clipped_energies():
    """The branching weight of a generation is exp(-tau ((E_c(old) + E_c(new)) / 2 - E_T)) with
    both local energies clipped to E_T +- 0.2 sqrt(Ne / tau).  The generation's moves are replayed
    here with the per-move functions (drift, Green's-function acceptance), the two local energies
    of every walker come from finite differences of the directly evaluated wavefunction, and the
    weights, their sum, the weighted energy, the multiplicities floor(w + u_b) (capped at 3), the
    children's configurations and the new trial energy are formed by hand from them."""
    # analytic plane-wave orbitals with the Pade J2: E_L varies smoothly with the positions, so
    # most energies stay inside the clip window (a random spline table spreads them over tens of Ha)
    n, W, tau = 4, 12, 0.05
    s = orc.System(n, n, 5.0, n_orb=n, orb_kind=orc.ORB_PLANEWAVE, use_j2=True, seed=18)
    d = Direct(n, n, 5.0, planewave=True, use_j2=True, seed=18)
    R0 = start_positions(84, W, 2 * n, s.L)
    e_old = np.array([d.eloc_fd(R0[w]) for w in range(W)])
    e_t = float(np.median(e_old))
    ecut = 0.2 * np.sqrt(2 * n / tau)
    res = orc.dmc(s, R0, 1, tau=tau, e_trial=e_t, n_target=W, max_pop=64)
    R1 = R0.copy()
    for w in range(W):
        for e in range(2 * n):
            v = orc.drift(s, R1[w], e)
            delta = tau * v + np.sqrt(tau) * orc.gauss3(18, w, 0, e)
            p, rho = orc.dmc_move_prob(s, R1[w], e, delta, tau)
            if rho > 0.0 and orc.accept_uniform(18, w, 0, e) < p:
                R1[w, e] = R1[w, e] + delta
                R1[w, e] -= s.L * np.floor(R1[w, e] / s.L)
    e_new = np.array([d.eloc_fd(R1[w]) for w in range(W)])
    eo = np.clip(e_old, e_t - ecut, e_t + ecut)
    en = np.clip(e_new, e_t - ecut, e_t + ecut)
    # the case under test: energies that moved, inside the clip window on both sides
    free = (np.abs(e_old - e_t) < ecut) & (np.abs(e_new - e_t) < ecut) & (np.abs(e_new - e_old) > 0.05)
    assert free.sum() >= 3
    wt = np.exp(-tau * (0.5 * (eo + en) - e_t))
    mult = np.minimum(3, np.floor(wt + np.array([orc.branch_uniform(18, w, 0) for w in range(W)]))).astype(int)
    assert res.pop[0] == mult.sum()
    assert abs(res.wsum[0] - wt.sum()) < 1e-6 * wt.sum()
    e_est = (wt * e_new).sum() / wt.sum()
    assert abs(res.e_est[0] - e_est) < 1e-5 * max(1.0, abs(e_est))
    assert abs(res.e_t[0] - (e_est - np.log(mult.sum() / W) / tau)) < 1e-5 * max(1.0, abs(e_est))
    assert np.allclose(res.R, np.repeat(R1, mult, axis=0), atol=1e-12)
    # a weight from the new energy alone would be off by far more than the tolerance above
    wt_new_only = np.exp(-tau * (en - e_t))
    assert abs(wt_new_only.sum() - wt.sum()) > 1e-3 * wt.sum()


# ---------------------------------------------------- FP32 rounding model

def test_fp32_chain_model_without_rounding_is_the_oracle_chain():
    """The rounding model of the mixed-precision chain, with nothing rounded, replays the FP64
    oracle's Sherman-Morrison chain along its decisions: the same ratios to 1e-12, across
    accepted updates, both spin blocks, several sweeps and a periodic recompute (which changes
    nothing in exact arithmetic), with the updates applied move by move or as delayed rank-k
    windows (the same inverse in exact arithmetic)."""
    from oracle import fp32_chain
    n = 3
    s, _ = _tiny_system(n, j2=True, seed=21)
    R0 = start_positions(85, 2, 2 * n, s.L)
    ref = orc.vmc(s, R0, 4, sigma=0.6)
    assert ref.acc.mean() > 0.2
    for w in range(2):
        for k in (0, 2, 3):  # Sherman-Morrison steps, delayed windows of 2 and 3 accepted moves
            rho = fp32_chain.replay(s, R0[w], w, ref.acc[:, :, w], sigma=0.6, recompute_every=2, storage="fp64",
                                    window=k)
            assert np.allclose(rho, ref.rho[:, :, w], rtol=1e-12, atol=1e-14), k


def test_fp32_chain_model_rounds_to_single_precision():
    """With FP32 storage the model's ratios differ from the FP64 chain by FP32 rounding: on a
    well-conditioned 4 x 4 system every relative error is below 1e-5, and the typical one is of
    the order of the FP32 unit round-off (2^-24 = 6e-8), neither zero nor larger; the error is
    the same whether the update is formed in FP32 or in FP64 from the stored values, to that
    order."""
    from oracle import fp32_chain
    n = 4
    s, _ = _tiny_system(n, j2=True, seed=22)
    R0 = start_positions(86, 3, 2 * n, s.L)
    ref = orc.vmc(s, R0, 3, sigma=0.5)
    for arith in ("fp32", "fp64"):
        rel = []
        for w in range(3):
            rho = fp32_chain.replay(s, R0[w], w, ref.acc[:, :, w], sigma=0.5, storage="fp32", arith=arith)
            big = np.abs(ref.rho[:, :, w]) > 0.05
            rel.append((np.abs(rho - ref.rho[:, :, w]) / np.abs(ref.rho[:, :, w]))[big])
        rel = np.concatenate(rel)
        assert rel.max() < 1e-5, (arith, rel.max())
        assert 1e-9 < np.median(rel) < 2e-6, (arith, np.median(rel))
    st = fp32_chain.ratio_error_stats(rho, ref.rho[:, :, 2])
    assert st["n"] == 3 * 2 * n and st["median"] <= st["p99"] <= st["p999"]


def test_fp32_chain_dmc_model_without_rounding_is_the_oracle_chain():
    """The DMC variant of the rounding model, with nothing rounded, replays the oracle's DMC
    population along its decisions and multiplicities: the same ratios and acceptance
    probabilities (drift, Green's function, Jastrow) for every walker slot of every generation,
    across branching; the oracle's records are consistent (decisions from rho > 0 and u < P,
    multiplicities summing to the next population)."""
    from oracle import fp32_chain
    n, W, gens, tau = 2, 6, 3, 0.2
    s, _ = _tiny_system(n, j2=True, seed=23)
    R0 = start_positions(87, W, 2 * n, s.L)
    _, _, el0, _ = orc.setup(s, R0)
    cap = 4 * W + 16
    ref = orc.dmc(s, R0, gens, tau, float(np.mean(el0)), n_target=W, max_pop=cap, record=True)
    rec = ref.rec
    pops = [W] + list(ref.pop[:-1])
    assert len(set(ref.pop.tolist())) > 1
    for g in range(gens):
        live = pops[g]
        assert rec["mult"][g, :live].sum() == ref.pop[g]
        own = (rec["rho"][g, :, :live] > 0) & (rec["u"][g, :, :live] < rec["prob"][g, :, :live])
        assert np.array_equal(own, rec["acc"][g, :, :live].astype(bool))
    live = np.isfinite(rec["rho"])
    for k in (0, 1, 2):  # move by move, or delayed windows of 1 and 2 proposals
        model = fp32_chain.replay_dmc(s, R0, np.arange(W), rec["acc"], rec["mult"], tau, storage="fp64", window=k)
        assert np.array_equal(live, np.isfinite(model["rho"]))
        assert np.allclose(model["rho"][live], rec["rho"][live], rtol=1e-10, atol=1e-13), k
        assert np.allclose(model["prob"][live], rec["prob"][live], rtol=1e-9, atol=1e-13), k
    # along the oracle's own proposals the model reproduces its ratios without forming the drift
    model = fp32_chain.replay_dmc(s, R0, np.arange(W), rec["acc"], rec["mult"], tau, storage="fp64", window=2,
                                  rnew=rec["rnew"])
    assert np.allclose(model["rho"][live], rec["rho"][live], rtol=1e-10, atol=1e-13)


def test_dmc_records_equal_the_definitions_on_their_trajectory():
    """Along the oracle's own DMC trajectory (its decisions, proposals and branching), every
    recorded ratio equals det A'/det A of the current matrix from a refined solve, and every
    proposal equals wrap(r + tau v + sqrt(tau) z) with the drift v = grad ln|Psi| of the current
    configuration, and every acceptance probability equals the Green's-function form with the
    drift at the proposal: the Sherman-Morrison chain, the drift from the kept inverse column, the
    proposal formula and the acceptance are each pinned to their definitions (a wrong sign or a
    dropped term in the drift or the Green's function, or a stale column, fails)."""
    from dmc_replay import periodic_abs, trajectory_checks
    n, L, G, W, gens, tau, seed = 8, 6.0, 16, 4, 2, 0.05, 1205
    s = orc.System(n, n, L, G=G, n_orb=n, orb_kind=orc.ORB_SEEDED, coef_seed=seed, use_j2=True,
                   j2_a_par=0.25, j2_a_anti=0.5, j2_b=1.0, seed=seed)
    R0 = start_positions(seed, W, 2 * n, L)
    et = float(np.mean(orc.setup(s, R0)[2]))
    ref = orc.dmc(s, R0, gens, tau, et, n_target=W, max_pop=4 * W + 16, record=True)
    t = trajectory_checks(s, R0, np.arange(W), ref.rec["acc"], ref.rec["rnew"], ref.rec["mult"], tau,
                          lambda g, e, slot: True)
    m = np.isfinite(t["ratio"]) & np.isfinite(ref.rec["rho"])
    assert m.sum() == sum([W] + list(ref.pop[:-1])) * 2 * n
    rerr = np.abs(ref.rec["rho"][m] - t["ratio"][m]) / np.maximum(1.0, np.abs(t["ratio"][m]))
    derr = np.linalg.norm(periodic_abs(ref.rec["rnew"][m] - t["prop"][m], L), axis=-1) / tau / np.maximum(
        1.0, t["vabs"][m])
    perr = np.abs(ref.rec["prob"][m] - t["prob"][m]) / np.maximum(1.0, np.abs(t["prob"][m]))
    assert rerr.max() < 1e-11 and derr.max() < 1e-11 and perr.max() < 1e-10, (rerr.max(), derr.max(), perr.max())


def test_fp32_spline_is_the_spline_within_single_precision_rounding():
    """The binary32 evaluation of the spline (the rounding model's copy of the mixed path's
    arithmetic) equals the FP64 spline on the same binary32 coefficients to within the
    rounding of a 64-term binary32 sum: every value, gradient and Laplacian within
    64 * 2^-24 of the sum of the magnitudes of its terms (bounded here by 64 * max|c| * the
    largest weight), typically far below, and not identical (it does round)."""
    import dataclasses
    s = orc.System(16, 16, 7.0, G=12, n_orb=16, orb_kind=orc.ORB_SEEDED, coef_seed=44, use_j2=False, seed=44)
    s = dataclasses.replace(s, coef_fp32=True)
    rng = np.random.default_rng(5)
    h = 7.0 / 12
    scale = [1.0, 1.0 / h, 1.0 / h, 1.0 / h, 3 * 4.0 / h ** 2]  # bounds of the weights' magnitudes per output
    worst = 0.0
    for _ in range(20):
        r = rng.uniform(0, 7.0, 3)
        a = orc.orbital_vgl(s, r)
        b = orc.orbital_vgl_f32(s, r)
        outs_a = [a[0], a[1][:, 0], a[1][:, 1], a[1][:, 2], a[2]]
        outs_b = [b[0], b[1][:, 0], b[1][:, 1], b[1][:, 2], b[2]]
        for q in range(5):
            err = np.abs(outs_a[q] - outs_b[q]).max()
            assert err <= 64 * 2.0 ** -24 * 64 * scale[q], (q, err)
            worst = max(worst, err / scale[q])
    assert worst > 0.0


# ---------------------------------------------------- virtual moves (ratio only)

def test_virtual_ratios_are_wavefunction_ratios():
    """Every virtual-move ratio equals Psi(R with r_e -> r_q) / Psi(R) from two direct evaluations
    of the wavefunction (LU determinants of both spin blocks and the full pair sum of the
    Jastrow), for electrons of both spins, with a point that crosses the periodic boundary."""
    from synth import icosahedron_offsets
    n = 3
    s, d = _tiny_system(n, j2=True, seed=31)
    R = start_positions(95, 2, 2 * n, s.L)
    R[0, 1] = [s.L - 0.05, 0.3, 1.1]  # its points near +x wrap across the box edge
    off = np.vstack([icosahedron_offsets(0.4), [[0.2, -0.1, 0.05]]])
    ratio, rho, dlnj = orc.virtual_ratios(s, R, off)
    assert np.allclose(ratio, rho * np.exp(dlnj), rtol=1e-14)
    for w in range(2):
        s0, l0 = d.log_psi(R[w])
        for e in range(2 * n):
            for q in range(off.shape[0]):
                R2 = R[w].copy()
                R2[e] = np.mod(R2[e] + off[q], s.L)
                s1, l1 = d.log_psi(R2)
                ref = s0 * s1 * np.exp(l1 - l0)
                assert abs(ratio[w, e, q] - ref) <= 1e-11 * max(1.0, abs(ref)), (w, e, q, ratio[w, e, q], ref)


def test_virtual_ratios_spherical_mean_of_plane_waves():
    """For analytic plane-wave orbitals {1, cos kx, sin kx, cos ky} (no Jastrow) the ratio of a
    virtual move of electron e to r_e + d n is sum_j phi_j(r_e + d n) (A^-1)_{j,e}; its spherical
    mean over n is sum_j sinc(k_j d) phi_j(r_e) (A^-1)_{j,e}, and summed over the electrons of a
    spin block the trace identity leaves sum_j sinc(k_j d): with the 12-point icosahedral rule
    (exact to degree 5) sum_e mean_q(ratio_eq) = sum_j sinc(k_j d) up to O((k d)^6)."""
    from synth import icosahedron_offsets
    n, L = 4, 5.0
    s = orc.System(n, n, L, G=16, n_orb=n, orb_kind=orc.ORB_PLANEWAVE, use_j2=False, seed=1)
    R = start_positions(96, 3, 2 * n, L)
    k = 2 * np.pi / L
    for dd in (0.3, 0.15):
        ratio, _, _ = orc.virtual_ratios(s, R, icosahedron_offsets(dd))
        per_spin = ratio.mean(axis=2).reshape(3, 2, n).sum(axis=2)  # [W][spin]
        exact = 1.0 + 3.0 * np.sin(k * dd) / (k * dd)
        tol = 2.0 * n * (k * dd) ** 6 / 5040.0
        assert np.all(np.abs(per_spin - exact) <= tol), (dd, per_spin, exact)
        # and not trivially: the d^2 term is resolved
        assert np.all(np.abs(per_spin - 4.0) > 100 * tol)


# ---------------------------------------------------- Ewald electron-electron energy

# Madelung constant of a simple cubic lattice of unit charges in a uniform neutralising background
# (the Wigner-crystal value of Nijboer and de Wette, Physica 23 (1957) 309): one charge per cubic cell
# of edge L has the Coulomb energy -XI_SC / (2 L).
XI_SC = 2.837297479480620


def test_ewald_one_electron_is_the_madelung_energy():
    """One electron per periodic cell: V = -xi_sc / (2 L) wherever it sits and whatever the splitting
    parameter (a missing self or background term, or a wrong 2 pi / Omega, changes the value)."""
    for L in (5.0, 7.0):
        s = orc.System(1, 0, L)
        for r in ([0.0, 0.0, 0.0], [1.0, 2.0, 3.0], [L - 1e-9, 0.5 * L, 0.1]):
            for a in (3.0 / L, 6.0 / L, 9.0 / L):
                v = orc.ewald_energy(s, np.array([r]), a)
                assert abs(v * L + XI_SC / 2) < 1e-12, (L, r, a, v)


def test_ewald_energy_is_independent_of_the_splitting_and_homogeneous():
    """For 8 electrons anywhere in the box the Ewald sum does not depend on alpha (the real-space
    and reciprocal parts trade terms exactly), does not change under a common translation, and
    scales as 1/lambda when the box and the positions are scaled by lambda."""
    L = 7.0
    s = orc.System(4, 4, L)
    R = np.random.default_rng(1).uniform(0, L, (8, 3))
    vals = [orc.ewald_energy(s, R, a / L) for a in (2.5, 4.0, 6.0, 9.0)]
    assert max(vals) - min(vals) < 1e-12 * abs(vals[0])
    shifted = np.mod(R + np.array([1.3, -2.2, 0.4]), L)
    assert abs(orc.ewald_energy(s, shifted) - vals[0]) < 1e-12 * abs(vals[0])
    s2 = orc.System(4, 4, 2.0 * L)
    assert abs(2.0 * orc.ewald_energy(s2, 2.0 * R) - vals[0]) < 1e-12 * abs(vals[0])
    # two electrons far closer than the box: the Coulomb 1/r dominates and sets the sign and size
    R2 = R.copy()
    R2[1] = R2[0] + [1e-3, 0.0, 0.0]
    assert orc.ewald_energy(s, R2) - vals[0] > 900.0
