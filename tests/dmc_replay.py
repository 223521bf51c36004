"""Replay of a DMC trajectory with the oracle's definitions (test helper, CPU only).

Drift-diffusion moves amplify rounding (near a node the drift grows like the inverse
distance), so two FP64 runs that round differently part ways after a few hundred moves.
A run's ratios and proposals are therefore checked on that run's own trajectory: its
decisions, proposals and branching multiplicities are replayed with fresh orbital rows,
and at sampled moves the ratio and the proposal are formed from their definitions."""
import numpy as np

import oracle as orc


def periodic_abs(d, L):
    """|d| per coordinate taken modulo the box edge L."""
    d = np.asarray(d, dtype=np.float64)
    return np.abs(d - L * np.round(d / L))


def trajectory_checks(o, R0, uids, acc, rnew, mult, tau, pick, first_step=0, with_drift=True):
    """Replay a DMC population along a run's own decisions acc [gens][Ne][cap], proposals rnew
    [gens][Ne][cap][3] and multiplicities mult [gens][cap] with the oracle's orbitals, and at the
    moves where pick(g, e, slot) holds evaluate from the definitions, with x = A^-1 e_i of the
    current matrix by a refined solve (``oracle.column_refined``):
      ratio  det A' / det A = phi(r') . x,
      prop   the drift-diffusion proposal wrap(r_e + tau v + sqrt(tau) z) with the drift
             v = grad ln|Psi| at r_e = sum_j grad phi_j(r_e) x_j + grad ln J (``oracle.j2_terms``),
             z from the counter generator;
      prob   the acceptance probability rho^2 exp(2 dlnJ) exp(-(|d + tau v'|^2 - |d - tau v|^2)
             / (2 tau)) with d = tau v + sqrt(tau) z and v' = sum_j grad phi_j(r') x_j / rho +
             grad ln J at r'.
    Returns dict(ratio, prop, vabs, prob) of arrays [gens][Ne][cap](, 3), vabs = |v|, NaN where
    not picked (prop, vabs and prob only with_drift)."""
    gens, ne, cap = acc.shape
    n = ne // 2
    L = o.L
    pop = []
    for w in range(R0.shape[0]):
        R = np.array(R0[w], dtype=np.float64)
        A = [np.array([orc.orbital_vgl(o, R[sp * n + i], n)[0] for i in range(n)]) for sp in range(2)]
        pop.append((R, A))
    ids = [int(u) for u in uids]
    ratio = np.full((gens, ne, cap), np.nan)
    prop = np.full((gens, ne, cap, 3), np.nan)
    vabs = np.full((gens, ne, cap), np.nan)
    prob = np.full((gens, ne, cap), np.nan)
    for g in range(gens):
        step = first_step + g
        for slot, (R, A) in enumerate(pop):
            for e in range(ne):
                sp, i = divmod(e, n)
                rn = np.asarray(rnew[g, e, slot], dtype=np.float64)
                phi, gphi, _ = orc.orbital_vgl(o, rn, n)
                if pick(g, e, slot):
                    x = orc.column_refined(A[sp], i)
                    rho = float(phi.astype(np.longdouble) @ x.astype(np.longdouble))
                    ratio[g, e, slot] = rho
                    if with_drift:
                        jg, _ = orc.j2_terms(o, R, e, R[e])
                        v = orc.orbital_vgl(o, R[e], n)[1].T @ x + jg
                        d = tau * v + np.sqrt(tau) * orc.gauss3(o.seed, ids[slot], step, e)
                        r = R[e] + d
                        prop[g, e, slot] = r - L * np.floor(r / L)
                        vabs[g, e, slot] = np.linalg.norm(v)
                        jg2, dlnj = orc.j2_terms(o, R, e, rn)
                        vn = gphi.T @ x / rho + jg2
                        prob[g, e, slot] = rho * rho * np.exp(2.0 * dlnj) * np.exp(
                            -(np.sum((d + tau * vn) ** 2) - np.sum((d - tau * v) ** 2)) / (2.0 * tau))
                if acc[g, e, slot]:
                    A[sp][i] = phi
                    R[e] = rn
            print("   replayed generation %d walker %d" % (g, slot), flush=True)
        nxt, nid = [], []
        for slot, (R, A) in enumerate(pop):
            for c in range(int(mult[g, slot])):
                nxt.append((R.copy(), [x.copy() for x in A]))
                nid.append(ids[slot] if c == 0 else orc.child_uid(o.seed, ids[slot], step, c))
        pop, ids = nxt, nid
    return dict(ratio=ratio, prop=prop, vabs=vabs, prob=prob)
