"""Rounding model of the mixed-precision VMC chain (test infrastructure only).

TEST INFRASTRUCTURE ONLY: used by ``tests/`` (and the error report of
``bench.py``'s ``cpu_baseline`` leg) to say how large the ratio errors of a
chain that keeps its Slater inverses in FP32 must be, independently of any GPU
code.  It shares nothing with the HIP library.

The chain is the one of the paper's Alg. 1 (propose, ratio, accept, update the
walker's inverse after an acceptance), replayed along given decisions (normally
the FP64 oracle's), with the storage precision of the mixed path:

* orbital rows (spline values at the electrons and at the proposals) are evaluated
  in FP32 arithmetic (``oracle.orbital_vgl_f32``: FP32 weights, FP32 sums of the 64
  stencil terms) and stored in FP32, as the mixed path forms and stores them;
* the inverse is formed in FP64 from the FP32 rows and rounded to FP32, at the
  start and at every periodic recompute;
* the ratio rho_D = u . c_e is the FP64 sum of the exact products of the
  FP32-stored row u and inverse column c_e;
* an accepted move applies the Sherman-Morrison update
  A^-1 <- A^-1 - c_e (u^T A^-1 - e_i^T) / rho_D with FP32 operands and FP32
  arithmetic (``arith="fp32"``, numpy float32 products and sums), or in FP64
  from the FP32-stored values, rounded to FP32 afterwards (``arith="fp64"``).

With ``window=k`` the accepted moves are applied as delayed rank-k updates, the form
the GPU paths use (McDaniel et al.'s delayed update written as a forward recurrence in
move order):

* the moves of a window see the inverse stored at its start; the ratio of a move is
  formed with the current column c_e = c0_e - sum_m beta_m c_m of the moves accepted
  so far in the window (VMC: in FP64 from the stored values; DMC: the columns kept in
  FP32, as the walker-resident kernel keeps them);
* when the window closes (k accepted moves in VMC, k proposals in DMC, or the end of
  the spin block) the inverse is updated once: with U the accepted rows, C their
  columns (stored in FP32), Y = U A^-1 - E (FP32 products and sums, the sums over the
  orbital index in order, as a matrix core accumulates them), L the window
  triangle (rho on the diagonal, u_m . c_j below it, FP64) and B = L^-1 Y (FP64,
  stored in FP32): A^-1 <- A^-1 - C B in FP32, the k terms added into the stored
  inverse one after another (the inverse is the matrix cores' accumulator).

With ``storage="fp64"`` nothing is rounded, and the chain is the FP64 oracle's
Sherman-Morrison chain term by term (pinned in ``tests/test_oracle_pins.py``).
"""
import numpy as np

from . import oracle as _o


def _f32(x):
    return np.asarray(x, dtype=np.float64).astype(np.float32)


def _window_update(Ai, us, cs, rhos, Gw, els):
    """Apply a window's accepted moves to the stored inverse Ai (Ai[j][i] = (A^-1)[j][i], FP32 or
    FP64, the arithmetic of the products follows it) in one rank-k step: A^-1 <- A^-1 - C B,
    B = L^-1 (U A^-1 - E), L lower triangular with the move ratios on the diagonal and
    Gw[m][j] = u_m . c_j below it."""
    k = len(us)
    if k == 0:
        return Ai
    dt = Ai.dtype
    U = np.array(us, dtype=dt)                         # [k][n]
    C = np.array(cs, dtype=np.float64).astype(dt).T    # [n][k], columns stored
    if dt == np.float32:
        # products and sums in FP32, the sum over the orbital index taken in order (a matrix-core
        # product accumulates its K dimension step by step, not pairwise as a CPU BLAS does)
        Yf = np.zeros((k, Ai.shape[1]), np.float32)
        for j in range(Ai.shape[0]):
            Yf += U[:, j:j + 1] * Ai[j:j + 1, :]
        Y = Yf.astype(np.float64)
    else:
        Y = U @ Ai
    for m, e in enumerate(els):
        Y[m, e] -= 1.0
    Lw = np.zeros((k, k))
    for m in range(k):
        Lw[m, m] = rhos[m]
        Lw[m, :m] = Gw[m][:m]
    B = np.linalg.solve(Lw, Y).astype(dt)             # forward substitution in FP64, stored
    if dt == np.float32:
        # the matrix cores accumulate the k terms into the stored inverse one by one
        out = Ai.copy()
        for m in range(k):
            out -= np.outer(C[:, m], B[m])
        return out
    return Ai - C @ B


def replay(sys, R0w, uid, acc, n_moves=None, sigma=0.5, first_step=0, recompute_every=0,
           storage="fp32", arith="fp32", window=0, close_after="accepts"):
    """Ratios of one walker's chain along the decisions ``acc`` ([sweeps][Ne], 1 = accept).

    Returns rho [sweeps][Ne] (NaN past n_moves moves of the first sweep, as the oracle's
    ``max_moves``).  recompute_every > 0 recomputes both inverses (FP64 from the stored
    rows, then stored) after every that many sweeps, as the mixed path does.  window = k >= 1
    applies the accepted moves as delayed rank-k updates; a window closes after k accepted
    moves (close_after="accepts") or k proposals ("proposals"), and at the end of a spin
    block."""
    acc = np.asarray(acc)
    S, ne = acc.shape
    n = sys.n_up
    assert sys.n_dn == n and ne == 2 * n
    lp = storage == "fp32"
    store = _f32 if lp else (lambda x: np.asarray(x, dtype=np.float64))
    vgl = _o.orbital_vgl_f32 if lp else _o.orbital_vgl
    R = np.array(R0w, dtype=np.float64)
    A = [np.array([store(vgl(sys, R[sp * n + i], n)[0]) for i in range(n)]) for sp in range(2)]

    def inverse(M):
        return store(np.linalg.inv(np.asarray(M, dtype=np.float64)))

    Ai = [inverse(A[0]), inverse(A[1])]   # Ai[sp][j][i] = (A^-1)[j][i]
    rho = np.full((S, ne), np.nan)
    total = S * ne if n_moves is None else n_moves
    done = 0
    win = None  # open window: (FP64 working inverse, rows, columns, ratios, triangle, electrons)

    def close(sp):
        nonlocal win
        if win is not None:
            Ai[sp] = _window_update(Ai[sp], *win[1:])
            win = None

    for s in range(S):
        step = first_step + s
        for e in range(ne):
            if done >= total:
                return rho
            sp, i = divmod(e, n)
            if window and i == 0 and sp == 1:
                close(0)
            rn = R[e] + sigma * _o.gauss3(sys.seed, uid, step, e)
            rn = rn - sys.L * np.floor(rn / sys.L)
            u = store(vgl(sys, rn, n)[0])
            if window:
                if win is None:
                    win = (Ai[sp].astype(np.float64), [], [], [], [], [])
                Aw = win[0]
                c = Aw[:, i].copy()
                r = float(np.dot(u.astype(np.float64), c))
            else:
                c = Ai[sp][:, i]
                r = float(np.dot(u.astype(np.float64), c.astype(np.float64)))
            rho[s, e] = r
            if acc[s, e]:
                if window:
                    Aw, us, cs, rs, Gw, els = win
                    Gw.append([float(u.astype(np.float64) @ cj) for cj in cs] + [0.0])
                    us.append(u)
                    cs.append(c)
                    rs.append(r)
                    els.append(i)
                    wrow = u.astype(np.float64) @ Aw
                    wrow[i] -= 1.0
                    win = (Aw - np.outer(c, wrow) / r, us, cs, rs, Gw, els)
                    if close_after == "accepts" and len(us) == window:
                        close(sp)
                elif lp and arith == "fp32":
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
            if window and close_after == "proposals" and (i + 1) % window == 0:
                close(sp)
            done += 1
        if window:
            close(1)
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


def replay_dmc(sys, R0, uids, acc, mult, tau, first_step=0, storage="fp32", rnew=None, recompute_every=0,
               window=0):
    """Ratios and acceptance probabilities of a DMC population's chain (drift-diffusion moves with
    the Green's-function acceptance, then branching; the generation loop of Alg. 1) along the
    decisions acc [gens][Ne][cap] and multiplicities mult [gens][cap] of a reference run, with the
    inverse, the value rows and the gradient rows stored in FP32 (``storage="fp32"``) or nothing
    rounded (``storage="fp64"``).  Drifts are the FP64 sums of the stored gradient rows times the
    stored inverse column plus the Jastrow gradient; the update is the FP32 Sherman-Morrison step
    of ``replay``.  Children copy their parent's stored state; copy 0 keeps the uid, copy c >= 1
    takes the counter-generator uid.  rnew [gens][Ne][cap][3] (optional): the proposals to take
    instead of the chain's own drift-diffusion step (the trajectory of another run, so that both
    are compared at the same positions; prob is then not formed).  recompute_every > 0: both
    inverses are formed again in FP64 from the stored rows and stored after every that many
    generations (before the branching).  window = k >= 1: delayed rank-k updates over windows of
    k proposals (the columns of a window's moves kept in the storage precision, their
    products with the rows in it and summed in FP64).  Returns dict(rho, prob) [gens][Ne][cap]
    (NaN where no walker)."""
    acc = np.asarray(acc)
    mult = np.asarray(mult)
    gens, ne, cap = acc.shape
    n = sys.n_up
    lp = storage == "fp32"
    store = _f32 if lp else (lambda x: np.asarray(x, dtype=np.float64))
    vgl = _o.orbital_vgl_f32 if lp else _o.orbital_vgl

    def new_state(R):
        R = np.array(R, dtype=np.float64)
        A, Gr = [], []
        for sp in range(2):
            rows = [vgl(sys, R[sp * n + i], n) for i in range(n)]
            A.append(np.array([store(r[0]) for r in rows]))
            Gr.append(np.array([store(r[1]) for r in rows]))
        Ai = [store(np.linalg.inv(A[sp].astype(np.float64))) for sp in range(2)]
        return dict(R=R, A=A, G=Gr, Ai=Ai)

    pop = [new_state(R0[w]) for w in range(R0.shape[0])]
    ids = [int(u) for u in uids]
    rho_out = np.full((gens, ne, cap), np.nan)
    prob_out = np.full((gens, ne, cap), np.nan)
    st = np.sqrt(tau)
    dt = np.float32 if lp else np.float64

    def dot(a, b):
        # products in the storage precision, summed in FP64
        return float((np.asarray(a, dtype=dt) * np.asarray(b, dtype=dt)).astype(np.float64).sum())

    for g in range(gens):
        step = first_step + g
        for slot, w in enumerate(pop):
            R = w["R"]
            win = None  # (rows, columns, ratios, triangle, electrons) of the open window
            for e in range(ne):
                sp, i = divmod(e, n)
                if window and i % window == 0:
                    if win is not None:
                        w["Ai"][1 - sp if i == 0 else sp] = _window_update(w["Ai"][1 - sp if i == 0 else sp], *win)
                    win = ([], [], [], [], [])
                if window:
                    us, cs, rs, Gw, els = win
                    c0 = w["Ai"][sp][:, i]
                    beta = []
                    for m in range(len(us)):
                        beta.append((dot(us[m], c0) - sum(beta[j] * Gw[m][j] for j in range(m))) / rs[m])
                    gr = w["G"][sp][i]
                    gc = np.array([dot(gr[:, k], c0) - sum(b * dot(gr[:, k], cm) for b, cm in zip(beta, cs))
                                   for k in range(3)])
                else:
                    c = w["Ai"][sp][:, i].astype(np.float64)
                    gc = w["G"][sp][i].astype(np.float64).T @ c
                if rnew is None:
                    jg, _ = _o.j2_terms(sys, R, e, R[e])
                    v = gc + jg
                    delta = tau * v + st * _o.gauss3(sys.seed, ids[slot], step, e)
                    rn = R[e] + delta
                    rn = rn - sys.L * np.floor(rn / sys.L)
                else:
                    rn = np.asarray(rnew[g, e, slot], dtype=np.float64)
                val, grad, _ = vgl(sys, rn, n)
                u, gu = store(val), store(grad)
                if window:
                    xs = [dot(u, cm) for cm in cs]
                    r = dot(u, c0) - sum(b * x for b, x in zip(beta, xs))
                    gun = np.array([dot(gu[:, k], c0) - sum(b * dot(gu[:, k], cm) for b, cm in zip(beta, cs))
                                    for k in range(3)])
                else:
                    r = float(u.astype(np.float64) @ c)
                    gun = gu.astype(np.float64).T @ c
                rho_out[g, e, slot] = r
                if rnew is None:
                    jg2, dlnj = _o.j2_terms(sys, R, e, rn)
                    vn = gun / r + jg2
                    fwd = np.sum((delta - tau * v) ** 2)
                    bwd = np.sum((delta + tau * vn) ** 2)
                    prob_out[g, e, slot] = r * r * np.exp(2.0 * dlnj) * np.exp(-(bwd - fwd) / (2.0 * tau))
                if acc[g, e, slot]:
                    if window:
                        cn = np.asarray(c0, dtype=dt).copy()
                        for b, cm in zip(beta, cs):
                            cn = cn - dt(b) * np.asarray(cm, dtype=dt)
                        Gw.append(xs + [0.0])
                        us.append(u)
                        cs.append(cn)
                        rs.append(r)
                        els.append(i)
                    else:
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
            if window and win is not None:
                w["Ai"][1] = _window_update(w["Ai"][1], *win)
        if recompute_every > 0 and (g + 1) % recompute_every == 0:
            for w in pop:
                w["Ai"] = [store(np.linalg.inv(w["A"][sp].astype(np.float64))) for sp in range(2)]
        nxt, nid = [], []
        for slot, w in enumerate(pop):
            for k in range(int(mult[g, slot])):
                nxt.append(dict(R=w["R"].copy(), A=[a.copy() for a in w["A"]], G=[x.copy() for x in w["G"]],
                                Ai=[a.copy() for a in w["Ai"]]))
                nid.append(ids[slot] if k == 0 else _o.child_uid(sys.seed, ids[slot], step, k))
        pop, ids = nxt, nid
    return dict(rho=rho_out, prob=prob_out)
