"""Complex (twisted) orbitals in a general periodic cell: a plain FP64 reference.

TEST INFRASTRUCTURE ONLY: imported by ``tests/`` (and nothing in the HIP library or its
binding).  Numpy, complex128, one walker and one move at a time, in the order of the
paper's Alg. 1 (propose, ratio, accept or reject, update; local energy after the sweep).

Wavefunction (the paper gives none; the textbook Slater-Jastrow form with Bloch orbitals):

    Psi(R) = det A_up det A_dn exp(sum_{i<j} u(|r_i - r_j|)),   A[i][j] = phi_j(r_i)
    phi_j(r) = exp(i k.r) s_j(f),   f = r L^-1 (fractional coordinates; L has the lattice
                                     vectors as rows, r = f L)

s_j is a periodic uniform cubic B-spline over a G^3 grid in f with complex coefficients
(control point q of an axis at f = q / G), k the twist.  Positions are kept wrapped into
the cell, f - floor(f), and phi is evaluated at the wrapped position (|Psi| and every ratio of
derivatives are unchanged by the wrap; the phase of Psi follows the wrapped coordinates).
Derivatives in Cartesian coordinates come from the fractional ones through L^-1:

    grad_r s = L^-1 grad_f s,      lap_r s = sum_ab (L^-T L^-1)_ab d2 s / df_a df_b

(the full Hessian in f: the metric of a non-orthogonal cell couples the axes), and the twist
adds  grad phi = e^{ik.r} (grad s + i k s),  lap phi = e^{ik.r} (lap s + 2 i k.grad s - |k|^2 s).
The pair Jastrow u(r) = a r / (1 + b r) takes the minimum image in fractional coordinates,
d - rint(d L^-1) L.  A move is accepted when u_acc < |rho_D|^2 exp(2 dlnJ); the local energy
E_L = -1/2 sum_i lap_i Psi / Psi is complex (its real part is the estimator), assembled as
-1/2 sum_i [l_i + lap_i U + |grad_i U|^2 + 2 g_i . grad_i U] with g_i, l_i the determinant's
gradient and Laplacian ratios.  The move random numbers are the real oracle's (Philox
counters (uid, step, e)).

``waves`` instead of a table gives analytic plane waves phi_j = exp(i (2 pi L^-1 m_j + k).r)
(integer m_j), exact eigenfunctions of the kinetic operator, for pins.
"""
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

from . import oracle as _o

# uniform cubic B-spline basis: [b0 b1 b2 b3](t) = [t^3 t^2 t 1] @ MB
MB = np.array([[-1.0, 3.0, -3.0, 1.0],
               [3.0, -6.0, 3.0, 0.0],
               [-3.0, 0.0, 3.0, 0.0],
               [1.0, 4.0, 1.0, 0.0]]) / 6.0


@dataclass
class CSystem:
    n: int                                  # electrons per spin = orbitals
    lattice: np.ndarray                     # [3][3], rows a_1, a_2, a_3 (bohr)
    twist: np.ndarray = field(default_factory=lambda: np.zeros(3))  # Cartesian k (1/bohr)
    table: Optional[np.ndarray] = None      # [G][G][G][n] complex128
    waves: Optional[np.ndarray] = None      # [n][3] integers (analytic plane waves)
    use_j2: bool = False
    j2_a_par: float = 0.25
    j2_a_anti: float = 0.5
    j2_b: float = 1.0
    seed: int = 0

    def __post_init__(self):
        self.lattice = np.asarray(self.lattice, dtype=np.float64)
        self.twist = np.asarray(self.twist, dtype=np.float64)
        self.linv = np.linalg.inv(self.lattice)

    @property
    def n_e(self):
        return 2 * self.n


def wrap(sys: CSystem, r):
    f = np.asarray(r, dtype=np.float64) @ sys.linv
    return (f - np.floor(f)) @ sys.lattice


def min_image(sys: CSystem, d):
    f = np.asarray(d, dtype=np.float64) @ sys.linv
    return (f - np.rint(f)) @ sys.lattice


def _axis(fa, G):
    """Grid points, weights and their first and second derivatives along one fractional axis."""
    u = fa * G
    i = int(np.floor(u))
    t = u - i
    pw = np.array([t ** 3, t ** 2, t, 1.0])
    d1 = np.array([3 * t ** 2, 2 * t, 1.0, 0.0]) * G
    d2 = np.array([6 * t, 2.0, 0.0, 0.0]) * G * G
    idx = (i - 1 + np.arange(4)) % G
    return idx, pw @ MB, d1 @ MB, d2 @ MB


def periodic_part(sys: CSystem, r):
    """(s [n], grad_f s [n][3], Hessian_f s [n][3][3]) of the spline at the wrapped r."""
    f = wrap(sys, r) @ sys.linv
    f = f - np.floor(f)
    G = sys.table.shape[0]
    ax = [_axis(f[a], G) for a in range(3)]
    C = sys.table[np.ix_(ax[0][0], ax[1][0], ax[2][0])]  # [4][4][4][n]
    w = [[ax[a][1], ax[a][2], ax[a][3]] for a in range(3)]  # per axis: value, d1, d2 weights

    def contract(order):  # order[a] = derivative order along axis a
        return np.einsum("x,y,z,xyzn->n", w[0][order[0]], w[1][order[1]], w[2][order[2]], C)

    s = contract((0, 0, 0))
    gf = np.stack([contract((1, 0, 0)), contract((0, 1, 0)), contract((0, 0, 1))], axis=1)
    H = np.empty((sys.n, 3, 3), np.complex128)
    for a in range(3):
        for b in range(3):
            o = [0, 0, 0]
            o[a] += 1
            o[b] += 1
            H[:, a, b] = contract(tuple(o))
    return s, gf, H


def orbitals(sys: CSystem, r):
    """(phi [n], grad phi [n][3], lap phi [n]) at r (wrapped into the cell), complex."""
    rw = wrap(sys, r)
    k = sys.twist
    if sys.waves is not None:
        q = 2.0 * np.pi * np.asarray(sys.waves, dtype=np.float64) @ sys.linv.T + k  # [n][3]
        v = np.exp(1j * (q @ rw))
        return v, 1j * q * v[:, None], -np.sum(q * q, axis=1) * v
    s, gf, H = periodic_part(sys, rw)
    gs = gf @ sys.linv.T                       # grad_r s = L^-1 grad_f s
    metric = sys.linv.T @ sys.linv             # (L^-T L^-1)_ab
    ls = np.einsum("ab,nab->n", metric, H)
    ph = np.exp(1j * (k @ rw))
    v = ph * s
    g = ph[..., None] * (gs + 1j * k[None, :] * s[:, None])
    l = ph * (ls + 2j * (gs @ k) - (k @ k) * s)
    return v, g, l


def _pade(sys, same_spin, r):
    a = sys.j2_a_par if same_spin else sys.j2_a_anti
    b = sys.j2_b
    u = a * r / (1.0 + b * r)
    du = a / (1.0 + b * r) ** 2
    d2u = -2.0 * a * b / (1.0 + b * r) ** 3
    return u, du, d2u


def lnj(sys: CSystem, R):
    if not sys.use_j2:
        return 0.0
    R = np.asarray(R, dtype=np.float64)
    tot = 0.0
    for i in range(sys.n_e):
        for j in range(i + 1, sys.n_e):
            d = min_image(sys, R[i] - R[j])
            tot += _pade(sys, (i < sys.n) == (j < sys.n), np.sqrt(d @ d))[0]
    return tot


def j2_move(sys: CSystem, R, e, rnew):
    """ln J(R') - ln J(R) for moving electron e to rnew, over its pair terms."""
    if not sys.use_j2:
        return 0.0
    dj = 0.0
    for m in range(sys.n_e):
        if m == e:
            continue
        same = (m < sys.n) == (e < sys.n)
        d1 = min_image(sys, rnew - R[m])
        d0 = min_image(sys, R[e] - R[m])
        dj += _pade(sys, same, np.sqrt(d1 @ d1))[0] - _pade(sys, same, np.sqrt(d0 @ d0))[0]
    return dj


def j2_grad_lap(sys: CSystem, R, i):
    """(grad_i U [3], lap_i U) of the pair Jastrow."""
    g = np.zeros(3)
    lap = 0.0
    if not sys.use_j2:
        return g, lap
    for m in range(sys.n_e):
        if m == i:
            continue
        d = min_image(sys, R[i] - R[m])
        r = np.sqrt(d @ d)
        _, du, d2u = _pade(sys, (m < sys.n) == (i < sys.n), r)
        g += du * d / r
        lap += d2u + 2.0 * du / r
    return g, lap


def slater(sys: CSystem, R, spin):
    """(A, grad rows [n][n][3], Laplacian rows [n][n]) of one spin: row i = electron i."""
    lo = spin * sys.n
    rows = [orbitals(sys, R[lo + i]) for i in range(sys.n)]
    return (np.array([r[0] for r in rows]), np.array([r[1] for r in rows]), np.array([r[2] for r in rows]))


def local_energy(sys: CSystem, R, ainv):
    """Complex kinetic E_L from the inverses ainv[spin] (A^-1, row j orbital, column i electron)."""
    R = np.asarray(R, dtype=np.float64)
    el = 0.0 + 0.0j
    for spin in range(2):
        _, Gr, Lr = slater(sys, R, spin)
        for i in range(sys.n):
            e = spin * sys.n + i
            g = Gr[i].T @ ainv[spin][:, i]   # sum_j grad phi_j(r_i) (A^-1)_ji
            l = Lr[i] @ ainv[spin][:, i]
            gu, lu = j2_grad_lap(sys, R, e)
            el += -0.5 * (l + lu + gu @ gu + 2.0 * (g @ gu))
    return el


def setup(sys: CSystem, R):
    """(A^-1 per spin, log|det| [2], phase [2], E_L) at R."""
    ainv, ld, ph = [], np.zeros(2), np.zeros(2)
    for spin in range(2):
        A = slater(sys, R, spin)[0]
        sgn, lab = np.linalg.slogdet(A)
        ainv.append(np.linalg.inv(A))
        ld[spin], ph[spin] = lab, np.angle(sgn)
    return ainv, ld, ph, local_energy(sys, R, ainv)


@dataclass
class CVmcResult:
    rho: np.ndarray      # [S][Ne][W] complex
    dlnj: np.ndarray     # [S][Ne][W]
    prob: np.ndarray
    u: np.ndarray
    acc: np.ndarray      # uint8
    logdet: np.ndarray   # [S][W][2] after each sweep
    phase: np.ndarray    # [S][W][2] in (-pi, pi]
    eloc: np.ndarray     # [S][W] complex
    R: np.ndarray        # [W][Ne][3]


def wrap_angle(x):
    return float(np.angle(np.exp(1j * x)))


def vmc(sys: CSystem, R0, n_sweeps, sigma=0.5, uids=None, first_step=0) -> CVmcResult:
    """VMC sweeps of Alg. 1 for every walker of R0 ([W][Ne][3]): electron e of walker w at
    sweep s proposes wrap(r_e + sigma z), z from Philox counter (uid, first_step + s, e),
    and the Slater inverse follows each acceptance by a Sherman-Morrison update."""
    R0 = np.asarray(R0, dtype=np.float64)
    W, ne = R0.shape[0], R0.shape[1]
    assert ne == sys.n_e
    uids = np.arange(W, dtype=np.uint32) if uids is None else np.asarray(uids, dtype=np.uint32)
    shp = (n_sweeps, ne, W)
    res = CVmcResult(np.zeros(shp, np.complex128), np.zeros(shp), np.zeros(shp), np.zeros(shp),
                     np.zeros(shp, np.uint8), np.zeros((n_sweeps, W, 2)), np.zeros((n_sweeps, W, 2)),
                     np.zeros((n_sweeps, W), np.complex128), np.zeros_like(R0))
    n = sys.n
    for w in range(W):
        R = R0[w].copy()
        ainv, ld, ph, _ = setup(sys, R)
        A = [slater(sys, R, s)[0] for s in range(2)]
        uid = int(uids[w])
        for s in range(n_sweeps):
            step = first_step + s
            for e in range(ne):
                spin, a = divmod(e, n)
                z = _o.gauss3(sys.seed, uid, step, e)
                rp = wrap(sys, R[e] + sigma * z)
                u = orbitals(sys, rp)[0]
                rho = u @ ainv[spin][:, a]
                dj = j2_move(sys, R, e, rp)
                prob = abs(rho) ** 2 * np.exp(2.0 * dj)
                ua = _o.accept_uniform(sys.seed, uid, step, e)
                acc = ua < prob
                res.rho[s, e, w], res.dlnj[s, e, w], res.prob[s, e, w] = rho, dj, prob
                res.u[s, e, w], res.acc[s, e, w] = ua, acc
                if acc:
                    Ai = ainv[spin]
                    ea = np.zeros(n)
                    ea[a] = 1.0
                    ainv[spin] = Ai - np.outer(Ai[:, a], u @ Ai - ea) / rho
                    A[spin][a] = u
                    R[e] = rp
                    ld[spin] += np.log(abs(rho))
                    ph[spin] = wrap_angle(ph[spin] + np.angle(rho))
            res.logdet[s, w], res.phase[s, w] = ld, ph
            res.eloc[s, w] = local_energy(sys, R, ainv)
        res.R[w] = R
    return res


def direct_ratio(sys: CSystem, R, e, rnew):
    """Psi(R') / Psi(R) for moving electron e to rnew from two determinants (slogdet) and two
    full pair sums: no inverse, no update (a second route for pins)."""
    R = np.asarray(R, dtype=np.float64)
    spin = e // sys.n
    A0 = slater(sys, R, spin)[0]
    R1 = R.copy()
    R1[e] = rnew
    A1 = slater(sys, R1, spin)[0]
    s0, l0 = np.linalg.slogdet(A0)
    s1, l1 = np.linalg.slogdet(A1)
    return (s1 / s0) * np.exp(l1 - l0), lnj(sys, R1) - lnj(sys, R)
