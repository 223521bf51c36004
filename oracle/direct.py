"""Second, brute-force FP64 reference for tiny systems (N <= 8 per spin).

TEST INFRASTRUCTURE ONLY.  It re-derives the VMC chain of the paper's Alg. 1
(propose, ratio, accept/reject, local energy) by the most direct
route available, so that the C oracle can be pinned against it:

* orbitals: the uniform cubic B-spline in its basis-matrix form
  (1/6)[t^3 t^2 t 1] M, evaluated with numpy (the C oracle uses the expanded
  polynomials instead);
* ratio: det(A')/det(A) from two LU determinants (numpy.linalg.slogdet), no
  inverse and no Sherman-Morrison update;
* Jastrow: ln J(R') - ln J(R) from two full pair sums;
* local energy: -1/2 sum_i lap_i Psi / Psi by central finite differences of
  the directly evaluated Psi.

The move random numbers come from the oracle's Philox (pinned separately by
published known-answer vectors).
"""
import numpy as np

from . import oracle as _o

# uniform cubic B-spline basis matrix: [b0 b1 b2 b3] = (1/6) [t^3 t^2 t 1] @ MB
MB = np.array([[-1.0, 3.0, -3.0, 1.0],
               [3.0, -6.0, 3.0, 0.0],
               [-3.0, 0.0, 3.0, 0.0],
               [1.0, 4.0, 1.0, 0.0]]) / 6.0


def _axis(x, L, G):
    h = L / G
    x = x - L * np.floor(x / L)
    s = x / h
    i = int(np.floor(s))
    t = s - i
    i %= G
    pw = np.array([t ** 3, t ** 2, t, 1.0])
    d1 = np.array([3 * t ** 2, 2 * t, 1.0, 0.0]) / h
    d2 = np.array([6 * t, 2.0, 0.0, 0.0]) / h ** 2
    idx = (i - 1 + np.arange(4)) % G
    return idx, pw @ MB, d1 @ MB, d2 @ MB


def spline_vgl(table, L, r):
    """Value [n], gradient [n,3] and Laplacian [n] of a periodic cubic B-spline table [G,G,G,n]."""
    G = table.shape[0]
    ix, bx, dbx, d2bx = _axis(r[0], L, G)
    iy, by, dby, d2by = _axis(r[1], L, G)
    iz, bz, dbz, d2bz = _axis(r[2], L, G)
    P = table[np.ix_(ix, iy, iz)]  # [4,4,4,n]
    v = np.einsum("a,b,c,abcn->n", bx, by, bz, P)
    gx = np.einsum("a,b,c,abcn->n", dbx, by, bz, P)
    gy = np.einsum("a,b,c,abcn->n", bx, dby, bz, P)
    gz = np.einsum("a,b,c,abcn->n", bx, by, dbz, P)
    lap = (np.einsum("a,b,c,abcn->n", d2bx, by, bz, P) + np.einsum("a,b,c,abcn->n", bx, d2by, bz, P)
           + np.einsum("a,b,c,abcn->n", bx, by, d2bz, P))
    return v, np.stack([gx, gy, gz], axis=1), lap


def planewave_vgl(L, r, n):
    """Analytic {1, cos kx, sin kx, cos ky}, k = 2 pi / L (first n of them)."""
    k = 2 * np.pi / L
    x, y = r[0], r[1]
    v = np.array([1.0, np.cos(k * x), np.sin(k * x), np.cos(k * y)])[:n]
    g = np.array([[0, 0, 0], [-k * np.sin(k * x), 0, 0], [k * np.cos(k * x), 0, 0],
                  [0, -k * np.sin(k * y), 0]], dtype=float)[:n]
    lap = -k * k * np.array([0.0, np.cos(k * x), np.sin(k * x), np.cos(k * y)])[:n]
    return v, g, lap


class Direct:
    """Psi_T(R) = det A_up det A_dn exp(sum_{i<j} u(r_ij)), evaluated directly."""

    def __init__(self, n_up, n_dn, L, table=None, planewave=False, use_j2=False,
                 a_par=0.25, a_anti=0.5, b=1.0, seed=0, ions=None, j1_a=-1.0, j1_b=1.0):
        self.n_up, self.n_dn, self.L = n_up, n_dn, L
        self.table = table
        self.planewave = planewave
        self.use_j2 = use_j2
        self.a_par, self.a_anti, self.b = a_par, a_anti, b
        self.seed = seed
        self.ions = None if ions is None else np.asarray(ions, dtype=np.float64).reshape(-1, 3)
        self.j1_a, self.j1_b = j1_a, j1_b

    @property
    def n_e(self):
        return self.n_up + self.n_dn

    def orbitals(self, r, n):
        if self.planewave:
            return planewave_vgl(self.L, r, n)
        v, g, l = spline_vgl(self.table, self.L, r)
        return v[:n], g[:n], l[:n]

    def matrices(self, R):
        out = []
        for sp, (lo, n) in enumerate(((0, self.n_up), (self.n_up, self.n_dn))):
            out.append(np.array([self.orbitals(R[lo + i], n)[0] for i in range(n)]))
        return out

    def lnj(self, R):
        """ln J: the Pade pairs (if any) plus the one-body terms a1 r / (1 + b1 r) of every
        electron with every centre (minimum image)."""
        s = 0.0
        if self.use_j2:
            for i in range(self.n_e):
                for j in range(i + 1, self.n_e):
                    d = R[i] - R[j]
                    d = d - self.L * np.rint(d / self.L)
                    r = np.sqrt(d @ d)
                    a = self.a_par if (i < self.n_up) == (j < self.n_up) else self.a_anti
                    s += a * r / (1 + self.b * r)
        if self.ions is not None:
            for i in range(self.n_e):
                d = R[i][None, :] - self.ions
                d = d - self.L * np.rint(d / self.L)
                r = np.sqrt((d * d).sum(axis=1))
                s += float(np.sum(self.j1_a * r / (1 + self.j1_b * r)))
        return s

    def log_psi(self, R):
        """(sign, ln|Psi|) with the determinants from LU (numpy.linalg.slogdet)."""
        sg, ld = 1.0, 0.0
        for A in self.matrices(R):
            s, l = np.linalg.slogdet(A)
            sg *= s
            ld += l
        return sg, ld + self.lnj(R)

    def slogdets(self, R):
        return [np.linalg.slogdet(A) for A in self.matrices(R)]

    def eloc_fd(self, R, h=2e-4):
        """-1/2 sum_i lap_i Psi / Psi by central second differences."""
        s0, l0 = self.log_psi(R)
        tot = 0.0
        for i in range(self.n_e):
            for c in range(3):
                Rp = R.copy(); Rp[i, c] += h
                Rm = R.copy(); Rm[i, c] -= h
                sp_, lp = self.log_psi(Rp)
                sm_, lm = self.log_psi(Rm)
                tot += (sp_ * s0 * np.exp(lp - l0) - 2.0 + sm_ * s0 * np.exp(lm - l0)) / h ** 2
        return -0.5 * tot

    def vmc(self, R0, n_sweeps, sigma=0.5, uid=0, first_step=0):
        """One walker's VMC chain: per-move (rho_D, dlnJ, P, accept) and per-sweep ln|det|."""
        R = np.array(R0, dtype=float)
        ne = self.n_e
        rho = np.zeros((n_sweeps, ne)); dl = np.zeros((n_sweeps, ne)); pr = np.zeros((n_sweeps, ne))
        acc = np.zeros((n_sweeps, ne), np.uint8)
        logdet = np.zeros((n_sweeps, 2))
        sign = np.zeros((n_sweeps, 2))
        for s in range(n_sweeps):
            step = first_step + s
            for e in range(ne):
                z = _o.gauss3(self.seed, uid, step, e)
                rn = R[e] + sigma * z
                rn = rn - self.L * np.floor(rn / self.L)
                Rn = R.copy(); Rn[e] = rn
                d_old = self.slogdets(R)
                d_new = self.slogdets(Rn)
                sp = 0 if e < self.n_up else 1
                r_d = d_new[sp][0] * d_old[sp][0] * np.exp(d_new[sp][1] - d_old[sp][1])
                dlnj = self.lnj(Rn) - self.lnj(R)
                p = r_d * r_d * np.exp(2 * dlnj)
                u = _o.accept_uniform(self.seed, uid, step, e)
                a = u < p
                rho[s, e], dl[s, e], pr[s, e], acc[s, e] = r_d, dlnj, p, a
                if a:
                    R = Rn
            logdet[s] = [d[1] for d in self.slogdets(R)]
            sign[s] = [d[0] for d in self.slogdets(R)]
        return dict(rho=rho, dlnj=dl, prob=pr, acc=acc, logdet=logdet, sign=sign, R=R)

    def drift_fd(self, R, e, h=1e-6):
        """grad_e ln|Psi| by central first differences."""
        g = np.zeros(3)
        for c in range(3):
            Rp = R.copy(); Rp[e, c] += h
            Rm = R.copy(); Rm[e, c] -= h
            g[c] = (self.log_psi(Rp)[1] - self.log_psi(Rm)[1]) / (2 * h)
        return g
