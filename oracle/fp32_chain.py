"""Rounding model of the mixed-precision VMC chain (test infrastructure only).

TEST INFRASTRUCTURE ONLY: used by ``tests/`` (and the error report of
``bench.py``'s ``cpu_baseline`` leg) to say how large the ratio errors of a
chain that keeps its Slater inverses in FP32 must be, independently of any GPU
code.  It shares nothing with the HIP library.

The chain is the one of the paper's Alg. 1 (propose, ratio, accept, update the
walker's inverse after an acceptance), replayed along given decisions (normally
the FP64 oracle's), with the storage precision of the mixed path:

* orbital rows (spline values at the electrons and at the proposals) are rounded
  to FP32, as the mixed path stores them;
* the inverse is formed in FP64 from the FP32 rows and rounded to FP32, at the
  start and at every periodic recompute;
* the ratio rho_D = u . c_e is the FP64 sum of the exact products of the
  FP32-stored row u and inverse column c_e;
* an accepted move applies the Sherman-Morrison update
  A^-1 <- A^-1 - c_e (u^T A^-1 - e_i^T) / rho_D with FP32 operands and FP32
  arithmetic (``arith="fp32"``, numpy float32 products and sums), or in FP64
  from the FP32-stored values, rounded to FP32 afterwards (``arith="fp64"``).

With ``storage="fp64"`` nothing is rounded, and the chain is the FP64 oracle's
Sherman-Morrison chain term by term (pinned in ``tests/test_oracle_pins.py``).
"""
import numpy as np

from . import oracle as _o


def _f32(x):
    return np.asarray(x, dtype=np.float64).astype(np.float32)


def replay(sys, R0w, uid, acc, n_moves=None, sigma=0.5, first_step=0, recompute_every=0,
           storage="fp32", arith="fp32"):
    """Ratios of one walker's chain along the decisions ``acc`` ([sweeps][Ne], 1 = accept).

    Returns rho [sweeps][Ne] (NaN past n_moves moves of the first sweep, as the oracle's
    ``max_moves``).  recompute_every > 0 recomputes both inverses (FP64 from the stored
    rows, then stored) after every that many sweeps, as the mixed path does."""
    acc = np.asarray(acc)
    S, ne = acc.shape
    n = sys.n_up
    assert sys.n_dn == n and ne == 2 * n
    lp = storage == "fp32"
    store = _f32 if lp else (lambda x: np.asarray(x, dtype=np.float64))
    R = np.array(R0w, dtype=np.float64)
    A = [np.array([store(_o.orbital_vgl(sys, R[sp * n + i], n)[0]) for i in range(n)]) for sp in range(2)]

    def inverse(M):
        return store(np.linalg.inv(np.asarray(M, dtype=np.float64)))

    Ai = [inverse(A[0]), inverse(A[1])]   # Ai[sp][j][i] = (A^-1)[j][i]
    rho = np.full((S, ne), np.nan)
    total = S * ne if n_moves is None else n_moves
    done = 0
    for s in range(S):
        step = first_step + s
        for e in range(ne):
            if done >= total:
                return rho
            sp, i = divmod(e, n)
            rn = R[e] + sigma * _o.gauss3(sys.seed, uid, step, e)
            rn = rn - sys.L * np.floor(rn / sys.L)
            u = store(_o.orbital_vgl(sys, rn, n)[0])
            c = Ai[sp][:, i]
            r = float(np.dot(u.astype(np.float64), c.astype(np.float64)))
            rho[s, e] = r
            if acc[s, e]:
                if lp and arith == "fp32":
                    wrow = u @ Ai[sp]                       # float32 products and sums
                    wrow[i] -= np.float32(1.0)
                    Ai[sp] = Ai[sp] - np.outer(c, wrow / np.float32(r))
                else:
                    M = Ai[sp].astype(np.float64)
                    wrow = u.astype(np.float64) @ M
                    wrow[i] -= 1.0
                    Ai[sp] = store(M - np.outer(M[:, i], wrow) / r)
                A[sp][i] = u
                R[e] = rn
            done += 1
        if recompute_every > 0 and (s + 1) % recompute_every == 0:
            Ai = [inverse(A[0]), inverse(A[1])]
    return rho


def ratio_error_stats(rho, ref, floor=1e-3):
    """Relative error |rho - ref| / |ref| of every recorded move: median, 99th and 99.9th
    percentiles over all moves, and the maximum over moves with |ref| >= floor (the relative
    error of a dot product is unbounded as its value goes to zero)."""
    rho = np.asarray(rho, dtype=np.float64).ravel()
    ref = np.asarray(ref, dtype=np.float64).ravel()
    ok = np.isfinite(rho) & np.isfinite(ref) & (ref != 0.0)
    rel = np.abs(rho[ok] - ref[ok]) / np.abs(ref[ok])
    big = np.abs(ref[ok]) >= floor
    return dict(n=int(ok.sum()), median=float(np.median(rel)), p99=float(np.quantile(rel, 0.99)),
                p999=float(np.quantile(rel, 0.999)), max=float(rel[big].max()) if big.any() else 0.0)


def replay_dmc(sys, R0, uids, acc, mult, tau, first_step=0, storage="fp32"):
    """Ratios and acceptance probabilities of a DMC population's chain (drift-diffusion moves with
    the Green's-function acceptance, then branching; the generation loop of Alg. 1) along the
    decisions acc [gens][Ne][cap] and multiplicities mult [gens][cap] of a reference run, with the
    inverse, the value rows and the gradient rows stored in FP32 (``storage="fp32"``) or nothing
    rounded (``storage="fp64"``).  Drifts are the FP64 sums of the stored gradient rows times the
    stored inverse column plus the Jastrow gradient; the update is the FP32 Sherman-Morrison step
    of ``replay``.  Children copy their parent's stored state; copy 0 keeps the uid, copy c >= 1
    takes the counter-generator uid.  Returns dict(rho, prob) [gens][Ne][cap] (NaN where no
    walker)."""
    acc = np.asarray(acc)
    mult = np.asarray(mult)
    gens, ne, cap = acc.shape
    n = sys.n_up
    lp = storage == "fp32"
    store = _f32 if lp else (lambda x: np.asarray(x, dtype=np.float64))

    def new_state(R):
        R = np.array(R, dtype=np.float64)
        A, Gr = [], []
        for sp in range(2):
            rows = [_o.orbital_vgl(sys, R[sp * n + i], n) for i in range(n)]
            A.append(np.array([store(r[0]) for r in rows]))
            Gr.append(np.array([store(r[1]) for r in rows]))
        Ai = [store(np.linalg.inv(A[sp].astype(np.float64))) for sp in range(2)]
        return dict(R=R, A=A, G=Gr, Ai=Ai)

    pop = [new_state(R0[w]) for w in range(R0.shape[0])]
    ids = [int(u) for u in uids]
    rho_out = np.full((gens, ne, cap), np.nan)
    prob_out = np.full((gens, ne, cap), np.nan)
    st = np.sqrt(tau)
    for g in range(gens):
        step = first_step + g
        for slot, w in enumerate(pop):
            R = w["R"]
            for e in range(ne):
                sp, i = divmod(e, n)
                c = w["Ai"][sp][:, i].astype(np.float64)
                jg, _ = _o.j2_terms(sys, R, e, R[e])
                v = w["G"][sp][i].astype(np.float64).T @ c + jg
                delta = tau * v + st * _o.gauss3(sys.seed, ids[slot], step, e)
                rn = R[e] + delta
                rn = rn - sys.L * np.floor(rn / sys.L)
                val, grad, _ = _o.orbital_vgl(sys, rn, n)
                u, gu = store(val), store(grad)
                r = float(u.astype(np.float64) @ c)
                jg2, dlnj = _o.j2_terms(sys, R, e, rn)
                vn = gu.astype(np.float64).T @ c / r + jg2
                fwd = np.sum((delta - tau * v) ** 2)
                bwd = np.sum((delta + tau * vn) ** 2)
                p = r * r * np.exp(2.0 * dlnj) * np.exp(-(bwd - fwd) / (2.0 * tau))
                rho_out[g, e, slot] = r
                prob_out[g, e, slot] = p
                if acc[g, e, slot]:
                    Ai = w["Ai"][sp]
                    if lp:
                        wrow = u @ Ai
                        wrow[i] -= np.float32(1.0)
                        w["Ai"][sp] = Ai - np.outer(Ai[:, i], wrow / np.float32(r))
                    else:
                        wrow = u @ Ai
                        wrow[i] -= 1.0
                        w["Ai"][sp] = Ai - np.outer(Ai[:, i], wrow) / r
                    w["A"][sp][i] = u
                    w["G"][sp][i] = gu
                    R[e] = rn
        nxt, nid = [], []
        for slot, w in enumerate(pop):
            for k in range(int(mult[g, slot])):
                nxt.append(dict(R=w["R"].copy(), A=[a.copy() for a in w["A"]], G=[x.copy() for x in w["G"]],
                                Ai=[a.copy() for a in w["Ai"]]))
                nid.append(ids[slot] if k == 0 else _o.child_uid(sys.seed, ids[slot], step, k))
        pop, ids = nxt, nid
    return dict(rho=rho_out, prob=prob_out)
