"""ctypes wrapper of the FP64 CPU oracle (``qmc_oracle.c``).

TEST INFRASTRUCTURE ONLY.  Nothing in the HIP library or its binding imports
this module.  Functions follow the paper's Alg. 1 (VMC: the sweep loop; DMC: the
whole generation loop including reweight/branch and the trial-energy update);
the wavefunction pieces are textbook definitions named in the C source.
"""
import ctypes
import os
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

from . import build_oracle

_lib = None


def lib():
    """Load (building first if needed) the oracle shared library."""
    global _lib
    if _lib is None:
        path = build_oracle.build(force=False)
        L = ctypes.CDLL(path)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        dp = ctypes.c_void_p
        L.or_philox4x32_10.argtypes = [u32p, u32p, u32p]
        L.or_uniform53.argtypes = [ctypes.c_uint32, ctypes.c_uint32]
        L.or_uniform53.restype = ctypes.c_double
        L.or_gauss3.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, dp]
        L.or_accept_uniform.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32]
        L.or_accept_uniform.restype = ctypes.c_double
        L.or_branch_uniform.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32]
        L.or_branch_uniform.restype = ctypes.c_double
        L.or_child_uid.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32]
        L.or_child_uid.restype = ctypes.c_uint32
        L.or_coef.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        L.or_coef.restype = ctypes.c_double
        L.or_orbital_vgl.argtypes = [ctypes.POINTER(OrSystem), dp, ctypes.c_int, dp, dp, dp]
        L.or_orbital_vgl_f32.argtypes = [ctypes.POINTER(OrSystem), dp, ctypes.c_int, dp, dp, dp]
        L.or_lnj.argtypes = [ctypes.POINTER(OrSystem), dp]
        L.or_lnj.restype = ctypes.c_double
        L.or_lu_inverse.argtypes = [ctypes.c_int, dp, dp, dp, dp]
        L.or_lu_inverse.restype = ctypes.c_int
        L.or_local_energy.argtypes = [ctypes.POINTER(OrSystem), dp, dp, dp, dp, dp, dp, dp]
        L.or_local_energy.restype = ctypes.c_double
        L.or_vmc.argtypes = [ctypes.POINTER(OrSystem), ctypes.c_int, dp, dp, ctypes.c_int,
                             ctypes.c_uint32, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                             dp, dp, dp, dp, dp, dp, dp, dp, dp, dp, dp, dp]
        L.or_vmc.restype = ctypes.c_int
        L.or_setup.argtypes = [ctypes.POINTER(OrSystem), ctypes.c_int, dp, ctypes.c_int, dp, dp, dp, dp]
        L.or_setup.restype = ctypes.c_int
        L.or_dmc.argtypes = [ctypes.POINTER(OrSystem), ctypes.c_int, dp, dp, ctypes.c_int,
                             ctypes.c_uint32, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                             ctypes.c_int, ctypes.c_int, dp, dp, dp, dp, dp, dp, dp, dp,
                             dp, dp, dp, dp, dp, dp]
        L.or_dmc.restype = ctypes.c_int
        L.or_j2_terms.argtypes = [ctypes.POINTER(OrSystem), dp, ctypes.c_int, dp, dp, dp]
        L.or_drift.argtypes = [ctypes.POINTER(OrSystem), dp, ctypes.c_int, dp]
        L.or_drift.restype = ctypes.c_int
        L.or_dmc_move_prob.argtypes = [ctypes.POINTER(OrSystem), dp, ctypes.c_int, dp, ctypes.c_double, dp, dp]
        L.or_dmc_move_prob.restype = ctypes.c_int
        L.or_virtual_ratios.argtypes = [ctypes.POINTER(OrSystem), ctypes.c_int, dp, ctypes.c_int, dp,
                                        ctypes.c_int, dp, dp, dp]
        L.or_virtual_ratios.restype = ctypes.c_int
        L.or_ewald_energy.argtypes = [ctypes.POINTER(OrSystem), dp, ctypes.c_double]
        L.or_ewald_energy.restype = ctypes.c_double
        _lib = L
    return _lib


class OrSystem(ctypes.Structure):
    _fields_ = [
        ("n_up", ctypes.c_int), ("n_dn", ctypes.c_int),
        ("L", ctypes.c_double),
        ("G", ctypes.c_int), ("n_orb", ctypes.c_int),
        ("orb_kind", ctypes.c_int),
        ("table", ctypes.c_void_p),
        ("coef_seed", ctypes.c_uint64),
        ("coef_fp32", ctypes.c_int),
        ("use_j2", ctypes.c_int),
        ("j2_a_par", ctypes.c_double), ("j2_a_anti", ctypes.c_double), ("j2_b", ctypes.c_double),
        ("seed", ctypes.c_uint64),
        ("use_coulomb", ctypes.c_int),
        ("n_ions", ctypes.c_int),
        ("ions", ctypes.c_void_p),
        ("j1_a", ctypes.c_double), ("j1_b", ctypes.c_double),
    ]


ORB_TABLE, ORB_SEEDED, ORB_PLANEWAVE = 0, 1, 2


@dataclass
class System:
    """One electronic system: box, orbitals, Jastrow and the move-RNG key."""
    n_up: int
    n_dn: int
    L: float
    G: int = 0
    n_orb: int = 0
    orb_kind: int = ORB_SEEDED
    table: Optional[np.ndarray] = None
    coef_seed: int = 0
    coef_fp32: bool = False
    use_j2: bool = False
    j2_a_par: float = 0.25
    j2_a_anti: float = 0.5
    j2_b: float = 1.0
    seed: int = 0
    use_coulomb: bool = False
    ions: Optional[np.ndarray] = None   # [n_ions][3] one-body Jastrow centres, or None
    j1_a: float = -1.0
    j1_b: float = 1.0
    _c: OrSystem = field(default=None, repr=False)

    @property
    def n_e(self) -> int:
        return self.n_up + self.n_dn

    def c(self) -> OrSystem:
        if self.table is not None:
            self.table = np.ascontiguousarray(self.table, dtype=np.float64)
        if self.ions is not None:
            self.ions = np.ascontiguousarray(self.ions, dtype=np.float64).reshape(-1, 3)
        self._c = OrSystem(self.n_up, self.n_dn, float(self.L), int(self.G), int(self.n_orb),
                           int(self.orb_kind),
                           self.table.ctypes.data if self.table is not None else None,
                           int(self.coef_seed), int(self.coef_fp32), int(self.use_j2),
                           float(self.j2_a_par), float(self.j2_a_anti), float(self.j2_b),
                           int(self.seed), int(self.use_coulomb),
                           0 if self.ions is None else int(self.ions.shape[0]),
                           self.ions.ctypes.data if self.ions is not None else None,
                           float(self.j1_a), float(self.j1_b))
        return self._c


def _p(a):
    return None if a is None else a.ctypes.data


def philox4x32_10(ctr, key):
    """Philox4x32-10 of one 128-bit counter under a 64-bit key."""
    c = (ctypes.c_uint32 * 4)(*[int(x) & 0xFFFFFFFF for x in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(x) & 0xFFFFFFFF for x in key])
    o = (ctypes.c_uint32 * 4)()
    lib().or_philox4x32_10(c, k, o)
    return [o[i] for i in range(4)]


def uniform53(lo, hi):
    return lib().or_uniform53(lo, hi)


def gauss3(seed, uid, step, e):
    z = np.zeros(3)
    lib().or_gauss3(seed, uid, step, e, z.ctypes.data)
    return z


def accept_uniform(seed, uid, step, e):
    return lib().or_accept_uniform(seed, uid, step, e)


def branch_uniform(seed, uid, step):
    return lib().or_branch_uniform(seed, uid, step)


def child_uid(seed, uid, step, copy):
    return lib().or_child_uid(seed, uid, step, copy)


def coef(seed, idx):
    return lib().or_coef(seed, idx)


def orbital_vgl(sys: System, r, norb=None):
    """(v[n], g[n,3], lap[n]) of orbitals 0..norb-1 at r."""
    norb = sys.n_orb if norb is None else norb
    r = np.ascontiguousarray(r, dtype=np.float64)
    v = np.zeros(norb)
    g = np.zeros((norb, 3))
    l = np.zeros(norb)
    cs = sys.c()
    lib().or_orbital_vgl(ctypes.byref(cs), r.ctypes.data, norb, v.ctypes.data, g.ctypes.data, l.ctypes.data)
    return v, g, l


def orbital_vgl_f32(sys: System, r, norb=None):
    """The spline of ``orbital_vgl`` evaluated in binary32 arithmetic (weights and sums; the
    mixed-precision path's arithmetic, used by the rounding model ``fp32_chain``)."""
    norb = sys.n_orb if norb is None else norb
    r = np.ascontiguousarray(r, dtype=np.float64)
    v = np.zeros(norb)
    g = np.zeros((norb, 3))
    l = np.zeros(norb)
    cs = sys.c()
    lib().or_orbital_vgl_f32(ctypes.byref(cs), r.ctypes.data, norb, v.ctypes.data, g.ctypes.data, l.ctypes.data)
    return v, g, l


def lnj(sys: System, R):
    R = np.ascontiguousarray(R, dtype=np.float64)
    cs = sys.c()
    return lib().or_lnj(ctypes.byref(cs), R.ctypes.data)


def lu_inverse(A):
    """(A^-1, log|det A|, sign det A) by LU with partial pivoting."""
    A = np.ascontiguousarray(A, dtype=np.float64)
    n = A.shape[0]
    inv = np.zeros_like(A)
    ld = ctypes.c_double()
    sg = ctypes.c_int()
    st = lib().or_lu_inverse(n, A.ctypes.data, inv.ctypes.data, ctypes.addressof(ld), ctypes.addressof(sg))
    if st != 0:
        raise ZeroDivisionError("singular matrix")
    return inv, ld.value, sg.value


def column_refined(A, i):
    """Column i of A^-1 (the solution of A x = e_i) from an LU solve refined twice with residuals
    e_i - A x formed in extended precision (numpy longdouble): good to a few ulp times
    (1 + eps cond(A)), independently of how A was reached."""
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[0]
    b = np.zeros(n)
    b[i] = 1.0
    Al = A.astype(np.longdouble)
    x = np.linalg.solve(A, b)
    for _ in range(2):
        r = (b.astype(np.longdouble) - Al @ x.astype(np.longdouble)).astype(np.float64)
        x = x + np.linalg.solve(A, r)
    return x


def row_ratio_refined(A, i, phi):
    """det A' / det A where A' is A with row i replaced by phi, by its definition phi . A^-1 e_i
    (the determinant part of the ratio step of Alg. 1).  A^-1 e_i comes from ``column_refined``
    and the final dot is taken in extended precision, so the value is good to a few ulp times
    (1 + eps cond(A)): an arbiter for a long FP64 update chain, whose error grows with each
    rank-1 or rank-k step."""
    x = column_refined(A, i)
    return float(np.asarray(phi, dtype=np.float64).astype(np.longdouble) @ x.astype(np.longdouble))


def det_ratio_refined(sys: System, R, e, rnew):
    """Slater-determinant ratio det A(R') / det A(R) for moving electron e to rnew, with A rebuilt
    from the orbitals at R (no update chain) and the ratio from ``row_ratio_refined``."""
    R = np.asarray(R, dtype=np.float64)
    lo, n = (0, sys.n_up) if e < sys.n_up else (sys.n_up, sys.n_dn)
    A = np.array([orbital_vgl(sys, R[lo + i], n)[0] for i in range(n)])
    return row_ratio_refined(A, e - lo, orbital_vgl(sys, rnew, n)[0])


def local_energy(sys: System, R, Ainv_up, Ainv_dn, G_up, G_dn, L_up, L_dn):
    """Kinetic local energy from inverses, gradient rows ([n][n][3]) and Laplacian rows."""
    arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (R, Ainv_up, Ainv_dn, G_up, G_dn, L_up, L_dn)]
    cs = sys.c()
    return lib().or_local_energy(ctypes.byref(cs), *[a.ctypes.data for a in arrs])


@dataclass
class VmcResult:
    rho: np.ndarray      # [S][Ne][W]
    dlnj: np.ndarray
    prob: np.ndarray
    u: np.ndarray
    acc: np.ndarray      # uint8
    logdet: np.ndarray   # [S][W][2]
    sign: np.ndarray     # [S][W][2]
    eloc: np.ndarray     # [S][W]
    R: np.ndarray        # [W][Ne][3]
    n_acc: np.ndarray    # [W]
    ainv: Optional[np.ndarray]  # [W][2][n][n] (A^-1 per spin, row j orbital / col i electron)
    t_moves: Optional[np.ndarray] = None  # [W] wall seconds of each walker's sweeps after set-up


def vmc(sys: System, R0, n_sweeps, sigma=0.5, uids=None, first_step=0, max_moves=0,
        n_threads=0, want_ainv=False) -> VmcResult:
    """Run VMC sweeps (the sweep loop of Alg. 1) for every walker of R0 ([W][Ne][3])."""
    R0 = np.ascontiguousarray(R0, dtype=np.float64)
    W, ne = R0.shape[0], R0.shape[1]
    assert ne == sys.n_e
    uids = np.arange(W, dtype=np.uint32) if uids is None else np.ascontiguousarray(uids, dtype=np.uint32)
    shp = (n_sweeps, ne, W)
    res = VmcResult(np.full(shp, np.nan), np.full(shp, np.nan), np.full(shp, np.nan), np.full(shp, np.nan),
                    np.zeros(shp, np.uint8), np.full((n_sweeps, W, 2), np.nan),
                    np.zeros((n_sweeps, W, 2), np.int32), np.full((n_sweeps, W), np.nan),
                    np.zeros_like(R0), np.zeros(W, np.int64),
                    np.zeros((W, sys.n_up * sys.n_up + sys.n_dn * sys.n_dn)) if want_ainv else None,
                    np.zeros(W))
    cs = sys.c()
    st = lib().or_vmc(ctypes.byref(cs), W, uids.ctypes.data, R0.ctypes.data, n_sweeps, first_step,
                      sigma, max_moves, n_threads,
                      res.rho.ctypes.data, res.dlnj.ctypes.data, res.prob.ctypes.data, res.u.ctypes.data,
                      res.acc.ctypes.data, res.logdet.ctypes.data, res.sign.ctypes.data,
                      res.eloc.ctypes.data, res.R.ctypes.data, res.n_acc.ctypes.data, _p(res.ainv),
                      res.t_moves.ctypes.data)
    if st != 0:
        raise ZeroDivisionError("singular starting configuration")
    if want_ainv:
        n = sys.n_up
        assert sys.n_up == sys.n_dn
        res.ainv = res.ainv.reshape(W, 2, n, n)
    return res


def setup(sys: System, R0, n_threads=0):
    """Initial (log|det| [W][2], sign [W][2], E_L [W], A^-1 [W][2][n][n])."""
    R0 = np.ascontiguousarray(R0, dtype=np.float64)
    W = R0.shape[0]
    ld = np.zeros((W, 2))
    sg = np.zeros((W, 2), np.int32)
    el = np.zeros(W)
    n = sys.n_up
    ai = np.zeros((W, 2, n, n))
    cs = sys.c()
    st = lib().or_setup(ctypes.byref(cs), W, R0.ctypes.data, n_threads, ld.ctypes.data, sg.ctypes.data,
                        el.ctypes.data, ai.ctypes.data)
    if st != 0:
        raise ZeroDivisionError("singular starting configuration")
    return ld, sg, el, ai


def j2_terms(sys: System, R, e, r):
    """(grad ln J of electron e placed at r, ln J(R') - ln J(R) for the move of e to r)."""
    R = np.ascontiguousarray(R, dtype=np.float64)
    r = np.ascontiguousarray(r, dtype=np.float64)
    g = np.zeros(3)
    d = ctypes.c_double()
    cs = sys.c()
    lib().or_j2_terms(ctypes.byref(cs), R.ctypes.data, e, r.ctypes.data, g.ctypes.data, ctypes.addressof(d))
    return g, d.value


def drift(sys: System, R, e):
    """grad ln|Psi_T| with respect to electron e at configuration R ([Ne][3])."""
    R = np.ascontiguousarray(R, dtype=np.float64)
    v = np.zeros(3)
    cs = sys.c()
    if lib().or_drift(ctypes.byref(cs), R.ctypes.data, e, v.ctypes.data) != 0:
        raise ZeroDivisionError("singular configuration")
    return v


def dmc_move_prob(sys: System, R, e, delta, tau):
    """(P, rho_D) of the DMC move of electron e by the displacement delta from configuration R."""
    R = np.ascontiguousarray(R, dtype=np.float64)
    d = np.ascontiguousarray(delta, dtype=np.float64)
    p = ctypes.c_double()
    r = ctypes.c_double()
    cs = sys.c()
    if lib().or_dmc_move_prob(ctypes.byref(cs), R.ctypes.data, e, d.ctypes.data, tau,
                              ctypes.addressof(p), ctypes.addressof(r)) != 0:
        raise ZeroDivisionError("singular configuration")
    return p.value, r.value


@dataclass
class DmcResult:
    pop: np.ndarray       # [gen]
    wsum: np.ndarray      # [gen] sum of branching weights
    e_est: np.ndarray     # [gen] weighted mean local energy
    e_t: np.ndarray       # [gen] trial energy after the update
    n_acc: int
    n_prop: int
    uids: np.ndarray      # final population
    R: np.ndarray
    eloc: np.ndarray
    rec: Optional[dict] = None  # per-move rho, prob, u, acc [gen][Ne][max_pop], rnew [gen][Ne][max_pop][3];
                                # mult [gen][max_pop]


def dmc(sys: System, R0, n_gen, tau, e_trial, n_target=None, max_pop=None, uids=None,
        first_step=0, n_threads=0, record=False) -> DmcResult:
    """Run DMC generations (Alg. 1 including reweighting and branching) on one system's population.
    record=True also returns every move's rho_D, P, u, decision and proposed position and every
    branching multiplicity, indexed by the walker's position in its generation's population."""
    R0 = np.ascontiguousarray(R0, dtype=np.float64)
    W, ne = R0.shape[0], R0.shape[1]
    n_target = W if n_target is None else n_target
    max_pop = 4 * W + 16 if max_pop is None else max_pop
    uids = np.arange(W, dtype=np.uint32) if uids is None else np.ascontiguousarray(uids, dtype=np.uint32)
    pop = np.zeros(n_gen, np.int32)
    wsum = np.zeros(n_gen)
    eest = np.zeros(n_gen)
    et = np.zeros(n_gen)
    counts = np.zeros(2, np.int64)
    uo = np.zeros(max_pop, np.uint32)
    Ro = np.zeros((max_pop, ne, 3))
    eo = np.zeros(max_pop)
    rec = None
    if record:
        shp = (n_gen, ne, max_pop)
        rec = dict(rho=np.full(shp, np.nan), prob=np.full(shp, np.nan), u=np.full(shp, np.nan),
                   acc=np.zeros(shp, np.uint8), mult=np.zeros((n_gen, max_pop), np.int32),
                   rnew=np.full(shp + (3,), np.nan))
    cs = sys.c()
    n = lib().or_dmc(ctypes.byref(cs), W, uids.ctypes.data, R0.ctypes.data, n_gen, first_step, tau,
                     e_trial, n_target, max_pop, n_threads, pop.ctypes.data, wsum.ctypes.data,
                     eest.ctypes.data, et.ctypes.data, counts.ctypes.data, uo.ctypes.data, Ro.ctypes.data,
                     eo.ctypes.data, *([_p(rec[k]) for k in ("rho", "prob", "u", "acc", "mult", "rnew")] if rec
                                       else [None] * 6))
    if n < 0:
        raise RuntimeError("oracle DMC failed with status %d" % n)
    return DmcResult(pop, wsum, eest, et, int(counts[0]), int(counts[1]), uo[:n].copy(), Ro[:n].copy(),
                     eo[:n].copy(), rec)


def virtual_ratios(sys: System, R0, offsets, n_threads=0):
    """Virtual moves of every electron of every walker to r_e + offsets[q] (the ratio-only
    evaluations of the local-energy step of Alg. 1): (ratio, rho_D, dlnJ), each [W][Ne][n_q],
    with ratio = Psi(R with r_e -> r_q) / Psi(R) = rho_D exp(dlnJ) at the set-up state."""
    R0 = np.ascontiguousarray(R0, dtype=np.float64)
    off = np.ascontiguousarray(offsets, dtype=np.float64).reshape(-1, 3)
    W, ne, nq = R0.shape[0], R0.shape[1], off.shape[0]
    out = [np.zeros((W, ne, nq)) for _ in range(3)]
    cs = sys.c()
    if lib().or_virtual_ratios(ctypes.byref(cs), W, R0.ctypes.data, nq, off.ctypes.data, n_threads,
                               *[o.ctypes.data for o in out]) != 0:
        raise ZeroDivisionError("singular configuration")
    return tuple(out)


def ewald_energy(sys: System, R, alpha=None):
    """Electron-electron Coulomb energy of one configuration R [Ne][3] in the periodic box with a
    uniform neutralising background (Ewald summation with splitting parameter alpha, default
    6 / L; the value does not depend on alpha)."""
    R = np.ascontiguousarray(R, dtype=np.float64)
    cs = sys.c()
    return lib().or_ewald_energy(ctypes.byref(cs), R.ctypes.data, 6.0 / sys.L if alpha is None else alpha)
