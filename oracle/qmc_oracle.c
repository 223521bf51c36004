/*
 * qmc_oracle.c -- plain FP64 CPU oracle for the particle-by-particle QMC move
 * of Luo, Doak and Kent, "A High-Performance Design for Hierarchical
 * Parallelism in the QMCPACK Monte Carlo code" (arXiv 2209.14487).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
 * CPU-baseline leg of the benchmark load this library.  It shares no code,
 * header, table or generator with the HIP library, and the HIP library never
 * loads it.
 *
 * What is computed, and where it is defined:
 *   - the loop structure is the paper's Alg. 1 (walkers -> particles; for each
 *     particle: propose, ratio, derivatives, accept/reject; then the local
 *     energy; reweight/branch and the trial-energy update for DMC).  Walkers are spread over OpenMP threads, the pattern
 *     of the paper's multi-threaded CPU driver (Alg. 2).
 *   - the paper does not define the wavefunction or the update formulas; those
 *     are textbook mathematics: uniform cubic B-splines (de Boor), a product of
 *     one Slater determinant per spin, a two-body Pade Jastrow factor and a
 *     one-body Pade factor around fixed centres, the
 *     Sherman-Morrison rank-1 update of the inverse, LU with partial pivoting,
 *     importance-sampled DMC (Reynolds, Ceperley, Alder, Lester 1982) and the
 *     Philox4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw, SC'11).
 *
 * Everything is double precision and scalar.  The only deliberate "fast path"
 * is none: every move evaluates every orbital at every stencil point.
 *
 * Conventions (notation of the paper where it has one):
 *   R = {r_1 ... r_Ne}, electrons 0..N-1 are spin up, N..2N-1 spin down.
 *   A_sigma[i][j] = phi_j(r_i)  (row = electron of that spin, column = orbital)
 *   Ainv_sigma = (A_sigma)^-1 stored row-major: Ainv[j][i].
 *   rho = Psi_T(R')/Psi_T(R) = rho_D * exp(dlnJ).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_PI 3.14159265358979323846

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon et al., SC'11, "Parallel random numbers: as easy as  */
/* 1, 2, 3"): ten rounds of two 32x32->64 multiplies, key bumped by the       */
/* Weyl constants between rounds.                                            */
/* ------------------------------------------------------------------------ */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)M0 * (uint64_t)x0;
        uint64_t p1 = (uint64_t)M1 * (uint64_t)x2;
        uint32_t y0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
        uint32_t y1 = (uint32_t)p1;
        uint32_t y2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
        uint32_t y3 = (uint32_t)p0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
        k0 += W0; k1 += W1;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* 53-bit uniform in [0,1) from two 32-bit words: ((hi:lo) >> 11) * 2^-53. */
double or_uniform53(uint32_t lo, uint32_t hi)
{
    uint64_t v = ((uint64_t)hi << 32) | (uint64_t)lo;
    return (double)(v >> 11) * (1.0 / 9007199254740992.0);
}

static void philox_block(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                         uint32_t out[4])
{
    uint32_t ctr[4] = {c0, c1, c2, c3};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    or_philox4x32_10(ctr, key, out);
}

/* Box-Muller pair from two uniforms: sqrt(-2 ln(1-u0)) * (cos, sin)(2 pi u1). */
static void box_muller(double u0, double u1, double* z0, double* z1)
{
    double rad = sqrt(-2.0 * log(1.0 - u0));
    *z0 = rad * cos(2.0 * OR_PI * u1);
    *z1 = rad * sin(2.0 * OR_PI * u1);
}

/* Gaussian 3-vector for move (uid, step, electron): block 0 gives (z_x, z_y),
   block 1 gives z_z (first member of its pair). */
void or_gauss3(uint64_t seed, uint32_t uid, uint32_t step, uint32_t e, double z[3])
{
    uint32_t o[4];
    double unused;
    philox_block(seed, uid, step, e, 0u, o);
    box_muller(or_uniform53(o[0], o[1]), or_uniform53(o[2], o[3]), &z[0], &z[1]);
    philox_block(seed, uid, step, e, 1u, o);
    box_muller(or_uniform53(o[0], o[1]), or_uniform53(o[2], o[3]), &z[2], &unused);
}

/* Metropolis uniform for move (uid, step, electron): block 2, words 0-1. */
double or_accept_uniform(uint64_t seed, uint32_t uid, uint32_t step, uint32_t e)
{
    uint32_t o[4];
    philox_block(seed, uid, step, e, 2u, o);
    return or_uniform53(o[0], o[1]);
}

/* Branching uniform of walker uid at generation step (DMC): block 3 of the
   counter (uid, step, 0xFFFFFFFF). */
double or_branch_uniform(uint64_t seed, uint32_t uid, uint32_t step)
{
    uint32_t o[4];
    philox_block(seed, uid, step, 0xFFFFFFFFu, 3u, o);
    return or_uniform53(o[0], o[1]);
}

/* uid of the copy-th child (copy >= 1) of walker uid born at generation step. */
uint32_t or_child_uid(uint64_t seed, uint32_t uid, uint32_t step, uint32_t copy)
{
    uint32_t o[4];
    philox_block(seed, uid, step, copy, 4u, o);
    return o[0];
}

/* Seeded spline coefficient with linear index idx: 2u - 1 in [-1, 1). */
double or_coef(uint64_t seed, uint64_t idx)
{
    uint32_t o[4];
    philox_block(seed, (uint32_t)idx, (uint32_t)(idx >> 32), 0xC0EFu, 0u, o);
    return 2.0 * or_uniform53(o[0], o[1]) - 1.0;
}

/* ------------------------------------------------------------------------ */
/* System description (mirrored field by field by the Python wrapper).       */
/* ------------------------------------------------------------------------ */
typedef struct {
    int n_up, n_dn;       /* electrons per spin; each spin uses orbitals 0..n_sigma-1 */
    double L;             /* cubic box edge (bohr) */
    int G;                /* spline grid points per dimension */
    int n_orb;            /* orbitals in the table */
    int orb_kind;         /* 0: table given, 1: coefficients from seed, 2: analytic plane waves */
    const double* table;  /* [G][G][G][n_orb] when orb_kind == 0 */
    uint64_t coef_seed;   /* key of the coefficient generator when orb_kind == 1 */
    int coef_fp32;        /* round every coefficient to binary32 before use */
    int use_j2;
    double j2_a_par, j2_a_anti, j2_b;
    uint64_t seed;        /* key of the move generator */
    int use_coulomb;      /* add the Ewald electron-electron energy to E_L */
    int n_ions;           /* one-body Jastrow centres (0: no one-body Jastrow) */
    const double* ions;   /* [n_ions][3] */
    double j1_a, j1_b;    /* u1(r) = a r / (1 + b r) */
} or_system;

static double coef_at(const or_system* s, int ix, int iy, int iz, int n)
{
    uint64_t idx = (((uint64_t)ix * s->G + iy) * s->G + iz) * (uint64_t)s->n_orb + n;
    double c = (s->orb_kind == 0) ? s->table[idx] : or_coef(s->coef_seed, idx);
    if (s->coef_fp32) c = (double)(float)c;
    return c;
}

/* Uniform cubic B-spline weights of one axis (de Boor), for the four control
   points i-1, i, i+1, i+2 around fractional offset t in [0,1):
   value  b  = ((1-t)^3, 3t^3-6t^2+4, -3t^3+3t^2+3t+1, t^3) / 6
   first  b' = (-(1-t)^2, 3t^2-4t, -3t^2+2t+1, t^2) / (2h)
   second b''= (1-t, 3t-2, -3t+1, t) / h^2                                   */
static void bspline_axis(double x, double h, int G, int* i0, double b[4], double db[4], double d2b[4])
{
    double s = x / h;
    double fl = floor(s);
    double t = s - fl;
    int i = ((int)fl) % G;
    if (i < 0) i += G;
    *i0 = i;
    double u = 1.0 - t;
    b[0] = u * u * u / 6.0;
    b[1] = (3.0 * t * t * t - 6.0 * t * t + 4.0) / 6.0;
    b[2] = (-3.0 * t * t * t + 3.0 * t * t + 3.0 * t + 1.0) / 6.0;
    b[3] = t * t * t / 6.0;
    db[0] = -u * u / (2.0 * h);
    db[1] = (3.0 * t * t - 4.0 * t) / (2.0 * h);
    db[2] = (-3.0 * t * t + 2.0 * t + 1.0) / (2.0 * h);
    db[3] = t * t / (2.0 * h);
    d2b[0] = u / (h * h);
    d2b[1] = (3.0 * t - 2.0) / (h * h);
    d2b[2] = (-3.0 * t + 1.0) / (h * h);
    d2b[3] = t / (h * h);
}

/* Periodic wrap of one coordinate into [0, L): x - L floor(x/L). */
static double wrap(double x, double L) { return x - L * floor(x / L); }

/* Orbital value, gradient and Laplacian of orbitals 0..norb-1 at r.
   v[n], g[3n+c], lap[n]. */
void or_orbital_vgl(const or_system* s, const double r[3], int norb, double* v, double* g, double* lap)
{
    if (s->orb_kind == 2) {
        /* analytic plane waves {1, cos(kx), sin(kx), cos(ky)}, k = 2 pi / L */
        double k = 2.0 * OR_PI / s->L;
        double x = r[0], y = r[1];
        for (int n = 0; n < norb; ++n) {
            v[n] = 0; g[3 * n] = g[3 * n + 1] = g[3 * n + 2] = 0; lap[n] = 0;
            switch (n) {
            case 0: v[n] = 1.0; break;
            case 1: v[n] = cos(k * x); g[3 * n] = -k * sin(k * x); lap[n] = -k * k * cos(k * x); break;
            case 2: v[n] = sin(k * x); g[3 * n] = k * cos(k * x); lap[n] = -k * k * sin(k * x); break;
            case 3: v[n] = cos(k * y); g[3 * n + 1] = -k * sin(k * y); lap[n] = -k * k * cos(k * y); break;
            default: break;
            }
        }
        return;
    }
    const int G = s->G;
    const double h = s->L / G;
    int ix, iy, iz;
    double bx[4], dbx[4], d2bx[4], by[4], dby[4], d2by[4], bz[4], dbz[4], d2bz[4];
    bspline_axis(wrap(r[0], s->L), h, G, &ix, bx, dbx, d2bx);
    bspline_axis(wrap(r[1], s->L), h, G, &iy, by, dby, d2by);
    bspline_axis(wrap(r[2], s->L), h, G, &iz, bz, dbz, d2bz);
    for (int n = 0; n < norb; ++n) {
        v[n] = 0; g[3 * n] = g[3 * n + 1] = g[3 * n + 2] = 0; lap[n] = 0;
    }
    for (int a = 0; a < 4; ++a) {
        int jx = (ix + a - 1 + G) % G;
        for (int b = 0; b < 4; ++b) {
            int jy = (iy + b - 1 + G) % G;
            for (int c = 0; c < 4; ++c) {
                int jz = (iz + c - 1 + G) % G;
                double wv = bx[a] * by[b] * bz[c];
                double wgx = dbx[a] * by[b] * bz[c];
                double wgy = bx[a] * dby[b] * bz[c];
                double wgz = bx[a] * by[b] * dbz[c];
                double wl = d2bx[a] * by[b] * bz[c] + bx[a] * d2by[b] * bz[c] + bx[a] * by[b] * d2bz[c];
                for (int n = 0; n < norb; ++n) {
                    double p = coef_at(s, jx, jy, jz, n);
                    v[n] += wv * p;
                    g[3 * n] += wgx * p;
                    g[3 * n + 1] += wgy * p;
                    g[3 * n + 2] += wgz * p;
                    lap[n] += wl * p;
                }
            }
        }
    }
}

/* The same spline evaluated in the arithmetic of the mixed-precision path:  */
/* the per-axis weights (FP64, as above) are rounded to binary32, the 3-D    */
/* weights are binary32 products, and the 64 terms are summed in binary32     */
/* with fused multiply-adds, 16 at a time along each x-plane, the four plane  */
/* sums then added pairwise ((p0 + p1) + (p2 + p3)).  Coefficients are        */
/* rounded to binary32.  Used only by the rounding model of the mixed chain;  */
/* v[n], g[3n+c], lap[n] receive the binary32 results.                       */
void or_orbital_vgl_f32(const or_system* s, const double r[3], int norb, double* v, double* g, double* lap)
{
    const int G = s->G;
    const double h = s->L / G;
    int i0[3];
    float b[3][4], d1[3][4], d2[3][4];
    for (int ax = 0; ax < 3; ++ax) {
        double bd[4], d1d[4], d2d[4];
        bspline_axis(wrap(r[ax], s->L), h, G, &i0[ax], bd, d1d, d2d);
        for (int k = 0; k < 4; ++k) {
            b[ax][k] = (float)bd[k];
            d1[ax][k] = (float)d1d[k];
            d2[ax][k] = (float)d2d[k];
        }
    }
    for (int n = 0; n < norb; ++n) {
        float pl[4][5];
        for (int a = 0; a < 4; ++a) {
            int jx = (i0[0] + a - 1 + G) % G;
            float acc[5] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
            for (int bb = 0; bb < 4; ++bb) {
                int jy = (i0[1] + bb - 1 + G) % G;
                for (int c = 0; c < 4; ++c) {
                    int jz = (i0[2] + c - 1 + G) % G;
                    float p = (float)coef_at(s, jx, jy, jz, n);
                    float w[5];
                    w[0] = b[0][a] * b[1][bb] * b[2][c];
                    w[1] = d1[0][a] * b[1][bb] * b[2][c];
                    w[2] = b[0][a] * d1[1][bb] * b[2][c];
                    w[3] = b[0][a] * b[1][bb] * d1[2][c];
                    w[4] = d2[0][a] * b[1][bb] * b[2][c] + b[0][a] * d2[1][bb] * b[2][c] +
                           b[0][a] * b[1][bb] * d2[2][c];
                    for (int q = 0; q < 5; ++q) acc[q] = fmaf(w[q], p, acc[q]);
                }
            }
            for (int q = 0; q < 5; ++q) pl[a][q] = acc[q];
        }
        float o[5];
        for (int q = 0; q < 5; ++q) o[q] = (pl[0][q] + pl[1][q]) + (pl[2][q] + pl[3][q]);
        v[n] = o[0];
        g[3 * n] = o[1];
        g[3 * n + 1] = o[2];
        g[3 * n + 2] = o[3];
        lap[n] = o[4];
    }
}

/* ------------------------------------------------------------------------ */
/* Two-body Pade Jastrow: ln J = + sum_{i<j} u(r_ij), u(r) = a r / (1 + b r), */
/* a = a_par for equal spins, a_anti for opposite spins; minimum-image        */
/* distance d - L * nearbyint(d / L) per component (half to even).            */
/* ------------------------------------------------------------------------ */
static void min_image(const double* ri, const double* rj, double L, double d[3])
{
    for (int c = 0; c < 3; ++c) {
        double x = ri[c] - rj[c];
        d[c] = x - L * nearbyint(x / L);
    }
}

static int spin_of(const or_system* s, int e) { return e < s->n_up ? 0 : 1; }

static double pade_a(const or_system* s, int e, int m)
{
    return spin_of(s, e) == spin_of(s, m) ? s->j2_a_par : s->j2_a_anti;
}

/* u(r), u'(r), u''(r) */
static void pade(double a, double b, double r, double* u, double* du, double* d2u)
{
    double q = 1.0 + b * r;
    *u = a * r / q;
    *du = a / (q * q);
    *d2u = -2.0 * a * b / (q * q * q);
}

/* One-body Pade Jastrow: ln J1 = + sum_i sum_I u1(|r_i - R_I|), u1(r) = a r / (1 + b r)
   with the same Pade form as the pairs and its own a, b; minimum-image distance to each
   centre R_I.  u1 of one electron at r summed over the centres, with its gradient
   sum u1'(d) d/|d| and Laplacian sum u1'' + 2 u1'/d. */
static double j1_at(const or_system* s, const double* r, double grad[3], double* lap)
{
    double sum = 0.0;
    for (int I = 0; I < s->n_ions; ++I) {
        double d[3], u, du, d2u;
        min_image(r, &s->ions[3 * I], s->L, d);
        double rr = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        pade(s->j1_a, s->j1_b, rr, &u, &du, &d2u);
        sum += u;
        if (grad)
            for (int c = 0; c < 3; ++c) grad[c] += du * d[c] / rr;
        if (lap) *lap += d2u + 2.0 * du / rr;
    }
    return sum;
}

/* Full ln J of a configuration (used by the tests as brute force): the pairs, then
   the one-body terms. */
double or_lnj(const or_system* s, const double* R)
{
    int ne = s->n_up + s->n_dn;
    double sum = 0;
    if (s->use_j2)
        for (int i = 0; i < ne; ++i)
            for (int j = i + 1; j < ne; ++j) {
                double d[3], u, du, d2u;
                min_image(&R[3 * i], &R[3 * j], s->L, d);
                pade(pade_a(s, i, j), s->j2_b, sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]), &u, &du, &d2u);
                sum += u;
            }
    for (int i = 0; i < ne; ++i) sum += j1_at(s, &R[3 * i], NULL, NULL);
    return sum;
}

/* Gradient and Laplacian of ln J with respect to electron e at position re,
   all other electrons at R.  grad = sum_m u'(d) d/|d|, lap = sum_m u'' + 2u'/d,
   then the one-body terms of e at re. */
static void j2_grad_lap(const or_system* s, const double* R, int e, const double* re,
                        double grad[3], double* lap)
{
    int ne = s->n_up + s->n_dn;
    grad[0] = grad[1] = grad[2] = 0; *lap = 0;
    j1_at(s, re, grad, lap);
    if (!s->use_j2) return;
    for (int m = 0; m < ne; ++m) {
        if (m == e) continue;
        double d[3], u, du, d2u;
        min_image(re, &R[3 * m], s->L, d);
        double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        pade(pade_a(s, e, m), s->j2_b, r, &u, &du, &d2u);
        for (int c = 0; c < 3; ++c) grad[c] += du * d[c] / r;
        *lap += d2u + 2.0 * du / r;
    }
}

/* ln J(R') - ln J(R) when electron e moves from R[e] to rnew: the one-body change,
   then the pairs. */
static double j2_delta(const or_system* s, const double* R, int e, const double* rnew)
{
    int ne = s->n_up + s->n_dn;
    double sum = j1_at(s, rnew, NULL, NULL) - j1_at(s, &R[3 * e], NULL, NULL);
    if (!s->use_j2) return sum;
    for (int m = 0; m < ne; ++m) {
        if (m == e) continue;
        double d[3], u1, u0, du, d2u;
        min_image(rnew, &R[3 * m], s->L, d);
        pade(pade_a(s, e, m), s->j2_b, sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]), &u1, &du, &d2u);
        min_image(&R[3 * e], &R[3 * m], s->L, d);
        pade(pade_a(s, e, m), s->j2_b, sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]), &u0, &du, &d2u);
        sum += u1 - u0;
    }
    return sum;
}

/* Test entry point: the Jastrow gradient of electron e placed at r (the other
   electrons at R), and ln J(R') - ln J(R) for the move of e from R[e] to r. */
void or_j2_terms(const or_system* s, const double* R, int e, const double r[3], double grad[3], double* dlnj)
{
    double lap;
    j2_grad_lap(s, R, e, r, grad, &lap);
    *dlnj = j2_delta(s, R, e, r);
}

/* ------------------------------------------------------------------------ */
/* LU with partial pivoting (Golub & Van Loan, Alg. 3.4.1; ties -> lowest row */
/* index), then the inverse by solving A X = I column by column.             */
/* Returns 0, or -1 when a pivot is exactly zero.                             */
/* ------------------------------------------------------------------------ */
int or_lu_inverse(int n, const double* A, double* Ainv, double* logdet, int* sign)
{
    double* LU = (double*)malloc(sizeof(double) * (size_t)n * n);
    int* perm = (int*)malloc(sizeof(int) * (size_t)n);
    double* y = (double*)malloc(sizeof(double) * (size_t)n);
    memcpy(LU, A, sizeof(double) * (size_t)n * n);
    for (int i = 0; i < n; ++i) perm[i] = i;
    int sgn = 1;
    double ld = 0;
    int status = 0;
    for (int k = 0; k < n; ++k) {
        int p = k;
        double best = fabs(LU[(size_t)k * n + k]);
        for (int i = k + 1; i < n; ++i) {
            double v = fabs(LU[(size_t)i * n + k]);
            if (v > best) { best = v; p = i; }
        }
        if (best == 0.0) { status = -1; break; }
        if (p != k) {
            for (int j = 0; j < n; ++j) {
                double t = LU[(size_t)k * n + j];
                LU[(size_t)k * n + j] = LU[(size_t)p * n + j];
                LU[(size_t)p * n + j] = t;
            }
            int t = perm[k]; perm[k] = perm[p]; perm[p] = t;
            sgn = -sgn;
        }
        double piv = LU[(size_t)k * n + k];
        if (piv < 0) sgn = -sgn;
        ld += log(fabs(piv));
        for (int i = k + 1; i < n; ++i) {
            double l = LU[(size_t)i * n + k] / piv;
            LU[(size_t)i * n + k] = l;
            for (int j = k + 1; j < n; ++j) LU[(size_t)i * n + j] -= l * LU[(size_t)k * n + j];
        }
    }
    if (status == 0) {
        /* P A = L U: column c of A^-1 solves L U x = P e_c */
        for (int c = 0; c < n; ++c) {
            for (int i = 0; i < n; ++i) {
                double v = (perm[i] == c) ? 1.0 : 0.0;
                for (int j = 0; j < i; ++j) v -= LU[(size_t)i * n + j] * y[j];
                y[i] = v;
            }
            for (int i = n - 1; i >= 0; --i) {
                double v = y[i];
                for (int j = i + 1; j < n; ++j) v -= LU[(size_t)i * n + j] * Ainv[(size_t)j * n + c];
                Ainv[(size_t)i * n + c] = v / LU[(size_t)i * n + i];
            }
        }
        *logdet = ld;
        *sign = sgn;
    }
    free(LU); free(perm); free(y);
    return status;
}

/* ------------------------------------------------------------------------ */
/* Kinetic local energy (Alg. 1's local-energy step, H = kinetic only):      */
/*   E_L = -1/2 sum_i [ l_i + lap_i U + |grad_i U|^2 + 2 g_i . grad_i U ]     */
/*   g_i = sum_j grad phi_j(r_i) Ainv[j][i],  l_i = sum_j lap phi_j(r_i) Ainv[j][i] */
/* Ainv[s], Gm[s] ([N][N][3]) and Lm[s] ([N][N]) are per spin.               */
/* ------------------------------------------------------------------------ */
/* ------------------------------------------------------------------------ */
/* Electron-electron Coulomb energy of one configuration in the periodic box */
/* with a uniform neutralising background (Ewald summation; charges -1,     */
/* Omega = L^3, N = Ne):                                                      */
/*   V = 1/2 sum_{i,j} sum'_n erfc(alpha |r_ij + n L|) / |r_ij + n L|         */
/*     + (2 pi / Omega) sum_{k != 0} exp(-k^2 / (4 alpha^2)) / k^2 |rho_k|^2   */
/*     - alpha N / sqrt(pi) - pi N^2 / (2 alpha^2 Omega),                     */
/* rho_k = sum_i exp(i k . r_i), k = 2 pi n / L; the prime drops n = 0 when  */
/* i = j.  The value does not depend on alpha; the image and k shells are   */
/* taken until the terms fall below 1e-18 of the leading ones.              */
/* ------------------------------------------------------------------------ */
double or_ewald_energy(const or_system* s, const double* R, double alpha)
{
    const int N = s->n_up + s->n_dn;
    const double L = s->L, omega = L * L * L;
    const int nr = (int)ceil(6.5 / (alpha * L)) + 1;        /* image shells: alpha r >= 6.5 beyond */
    const int nk = (int)ceil(13.0 * alpha * L / (2.0 * OR_PI)) + 1;  /* k shells: k / (2 alpha) >= 6.5 */
    double real = 0.0;
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j)
            for (int a = -nr; a <= nr; ++a)
                for (int b = -nr; b <= nr; ++b)
                    for (int c = -nr; c <= nr; ++c) {
                        if (i == j && a == 0 && b == 0 && c == 0) continue;
                        double d[3] = {R[3 * i] - R[3 * j] + a * L, R[3 * i + 1] - R[3 * j + 1] + b * L,
                                       R[3 * i + 2] - R[3 * j + 2] + c * L};
                        double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
                        real += 0.5 * erfc(alpha * r) / r;
                    }
    double recip = 0.0;
    for (int a = -nk; a <= nk; ++a)
        for (int b = -nk; b <= nk; ++b)
            for (int c = -nk; c <= nk; ++c) {
                if (a == 0 && b == 0 && c == 0) continue;
                double k[3] = {2.0 * OR_PI * a / L, 2.0 * OR_PI * b / L, 2.0 * OR_PI * c / L};
                double k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
                double re = 0.0, im = 0.0;
                for (int i = 0; i < N; ++i) {
                    double ph = k[0] * R[3 * i] + k[1] * R[3 * i + 1] + k[2] * R[3 * i + 2];
                    re += cos(ph);
                    im += sin(ph);
                }
                recip += exp(-k2 / (4.0 * alpha * alpha)) / k2 * (re * re + im * im);
            }
    recip *= 2.0 * OR_PI / omega;
    return real + recip - alpha * N / sqrt(OR_PI) - OR_PI * (double)N * N / (2.0 * alpha * alpha * omega);
}

double or_local_energy(const or_system* s, const double* R,
                       const double* Ainv_up, const double* Ainv_dn,
                       const double* G_up, const double* G_dn,
                       const double* L_up, const double* L_dn)
{
    const double* Ai[2] = {Ainv_up, Ainv_dn};
    const double* Gm[2] = {G_up, G_dn};
    const double* Lm[2] = {L_up, L_dn};
    int nsp[2] = {s->n_up, s->n_dn};
    double sum = 0;
    for (int sp = 0; sp < 2; ++sp) {
        int n = nsp[sp];
        for (int i = 0; i < n; ++i) {
            int e = sp * s->n_up + i;
            double g[3] = {0, 0, 0}, l = 0;
            for (int j = 0; j < n; ++j) {
                double a = Ai[sp][(size_t)j * n + i];
                for (int c = 0; c < 3; ++c) g[c] += Gm[sp][((size_t)i * n + j) * 3 + c] * a;
                l += Lm[sp][(size_t)i * n + j] * a;
            }
            double gu[3], lu;
            j2_grad_lap(s, R, e, &R[3 * e], gu, &lu);
            sum += l + lu + gu[0] * gu[0] + gu[1] * gu[1] + gu[2] * gu[2]
                 + 2.0 * (g[0] * gu[0] + g[1] * gu[1] + g[2] * gu[2]);
        }
    }
    double e = -0.5 * sum;
    if (s->use_coulomb) e += or_ewald_energy(s, R, 6.0 / s->L);
    return e;
}

/* ------------------------------------------------------------------------ */
/* Walker state                                                              */
/* ------------------------------------------------------------------------ */
typedef struct {
    double* R;            /* [Ne][3] */
    double* A[2];         /* [n][n]    A[i][j] = phi_j(r_i) */
    double* Gm[2];        /* [n][n][3] */
    double* Lm[2];        /* [n][n]    */
    double* Ainv[2];      /* [n][n]    Ainv[j][i] */
    double logdet[2];
    int sign[2];
    double eloc;
    uint32_t uid;
    int64_t n_acc, n_prop;
} walker;

static void walker_alloc(const or_system* s, walker* w)
{
    int ne = s->n_up + s->n_dn;
    int nsp[2] = {s->n_up, s->n_dn};
    w->R = (double*)calloc((size_t)ne * 3, sizeof(double));
    for (int sp = 0; sp < 2; ++sp) {
        size_t nn = (size_t)nsp[sp] * nsp[sp];
        w->A[sp] = (double*)calloc(nn, sizeof(double));
        w->Gm[sp] = (double*)calloc(nn * 3, sizeof(double));
        w->Lm[sp] = (double*)calloc(nn, sizeof(double));
        w->Ainv[sp] = (double*)calloc(nn, sizeof(double));
    }
}

static void walker_free(walker* w)
{
    free(w->R);
    for (int sp = 0; sp < 2; ++sp) {
        free(w->A[sp]); free(w->Gm[sp]); free(w->Lm[sp]); free(w->Ainv[sp]);
    }
}

static void walker_copy(const or_system* s, walker* dst, const walker* src)
{
    int ne = s->n_up + s->n_dn;
    int nsp[2] = {s->n_up, s->n_dn};
    memcpy(dst->R, src->R, sizeof(double) * (size_t)ne * 3);
    for (int sp = 0; sp < 2; ++sp) {
        size_t nn = (size_t)nsp[sp] * nsp[sp];
        memcpy(dst->A[sp], src->A[sp], nn * sizeof(double));
        memcpy(dst->Gm[sp], src->Gm[sp], nn * 3 * sizeof(double));
        memcpy(dst->Lm[sp], src->Lm[sp], nn * sizeof(double));
        memcpy(dst->Ainv[sp], src->Ainv[sp], nn * sizeof(double));
        dst->logdet[sp] = src->logdet[sp];
        dst->sign[sp] = src->sign[sp];
    }
    dst->eloc = src->eloc;
    dst->uid = src->uid;
    dst->n_acc = src->n_acc;
    dst->n_prop = src->n_prop;
}

static double walker_eloc(const or_system* s, const walker* w)
{
    return or_local_energy(s, w->R, w->Ainv[0], w->Ainv[1], w->Gm[0], w->Gm[1], w->Lm[0], w->Lm[1]);
}

/* Fill the rows of A, G, L from the positions, then LU -> Ainv, log|det|. */
static int walker_setup(const or_system* s, walker* w)
{
    int nsp[2] = {s->n_up, s->n_dn};
    int nmax = s->n_up > s->n_dn ? s->n_up : s->n_dn;
    double* v = (double*)malloc(sizeof(double) * nmax);
    double* g = (double*)malloc(sizeof(double) * 3 * nmax);
    double* l = (double*)malloc(sizeof(double) * nmax);
    int status = 0;
    for (int sp = 0; sp < 2; ++sp) {
        int n = nsp[sp];
        for (int i = 0; i < n; ++i) {
            int e = sp * s->n_up + i;
            or_orbital_vgl(s, &w->R[3 * e], n, v, g, l);
            for (int j = 0; j < n; ++j) {
                w->A[sp][(size_t)i * n + j] = v[j];
                for (int c = 0; c < 3; ++c) w->Gm[sp][((size_t)i * n + j) * 3 + c] = g[3 * j + c];
                w->Lm[sp][(size_t)i * n + j] = l[j];
            }
        }
        if (or_lu_inverse(n, w->A[sp], w->Ainv[sp], &w->logdet[sp], &w->sign[sp]) != 0) status = -1;
    }
    free(v); free(g); free(l);
    w->eloc = status == 0 ? walker_eloc(s, w) : NAN;
    return status;
}

/* Sherman-Morrison: row i of A replaced by v (rho_D = v . Ainv[:,i]):
   Ainv' = Ainv - Ainv[:,i] (v^T Ainv - e_i^T) / rho_D                       */
static void sm_update(int n, double* Ainv, int i, const double* v, double rho, double* col, double* w)
{
    for (int j = 0; j < n; ++j) col[j] = Ainv[(size_t)j * n + i];
    for (int k = 0; k < n; ++k) {
        double s = 0;
        for (int j = 0; j < n; ++j) s += v[j] * Ainv[(size_t)j * n + k];
        w[k] = s - (k == i ? 1.0 : 0.0);
    }
    for (int j = 0; j < n; ++j)
        for (int k = 0; k < n; ++k) Ainv[(size_t)j * n + k] -= col[j] * w[k] / rho;
}

/* Per-move record written by the drivers (optional). */
typedef struct {
    double* rho_d;   /* determinant ratio rho_D */
    double* dlnj;    /* ln J(R') - ln J(R) */
    double* prob;    /* acceptance probability before comparison (may exceed 1) */
    double* uacc;    /* uniform drawn for the comparison */
    uint8_t* acc;    /* 1 accepted, 0 rejected */
} or_records;

typedef struct {
    double *v, *g, *l, *col, *w;
} scratch;

static void scratch_alloc(scratch* t, int nmax)
{
    t->v = (double*)malloc(sizeof(double) * nmax);
    t->g = (double*)malloc(sizeof(double) * 3 * nmax);
    t->l = (double*)malloc(sizeof(double) * nmax);
    t->col = (double*)malloc(sizeof(double) * nmax);
    t->w = (double*)malloc(sizeof(double) * nmax);
}

static void scratch_free(scratch* t) { free(t->v); free(t->g); free(t->l); free(t->col); free(t->w); }

/* Apply an accepted move of electron e to r' with orbital row (v, g, l). */
static void accept_move(const or_system* s, walker* w, int e, const double rnew[3], double rho,
                        scratch* t)
{
    int sp = spin_of(s, e);
    int n = sp == 0 ? s->n_up : s->n_dn;
    int i = e - sp * s->n_up;
    sm_update(n, w->Ainv[sp], i, t->v, rho, t->col, t->w);
    for (int j = 0; j < n; ++j) {
        w->A[sp][(size_t)i * n + j] = t->v[j];
        for (int c = 0; c < 3; ++c) w->Gm[sp][((size_t)i * n + j) * 3 + c] = t->g[3 * j + c];
        w->Lm[sp][(size_t)i * n + j] = t->l[j];
    }
    for (int c = 0; c < 3; ++c) w->R[3 * e + c] = rnew[c];
    w->logdet[sp] += log(fabs(rho));
    if (rho < 0) w->sign[sp] = -w->sign[sp];
}

/* Determinant ratio and gradient of ln D at the new position for electron e,
   orbital row t->v / t->g already evaluated at r'. */
static double det_ratio(const or_system* s, const walker* w, int e, const scratch* t, double gd[3])
{
    int sp = spin_of(s, e);
    int n = sp == 0 ? s->n_up : s->n_dn;
    int i = e - sp * s->n_up;
    double rho = 0;
    gd[0] = gd[1] = gd[2] = 0;
    for (int j = 0; j < n; ++j) {
        double a = w->Ainv[sp][(size_t)j * n + i];
        rho += t->v[j] * a;
        for (int c = 0; c < 3; ++c) gd[c] += t->g[3 * j + c] * a;
    }
    for (int c = 0; c < 3; ++c) gd[c] /= rho;
    return rho;
}

/* grad ln|Psi| for electron e at its current position (determinant + J2). */
static void drift_current(const or_system* s, const walker* w, int e, double v[3])
{
    int sp = spin_of(s, e);
    int n = sp == 0 ? s->n_up : s->n_dn;
    int i = e - sp * s->n_up;
    double gd[3] = {0, 0, 0}, gj[3], lj;
    for (int j = 0; j < n; ++j) {
        double a = w->Ainv[sp][(size_t)j * n + i];
        for (int c = 0; c < 3; ++c) gd[c] += w->Gm[sp][((size_t)i * n + j) * 3 + c] * a;
    }
    j2_grad_lap(s, w->R, e, &w->R[3 * e], gj, &lj);
    for (int c = 0; c < 3; ++c) v[c] = gd[c] + gj[c];
}

/* Wall-clock seconds (monotonic), for the sweep timing of or_vmc only.      */
static double wall_seconds(void)
{
    struct timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

/* ------------------------------------------------------------------------ */
/* VMC: the sweep loop of Alg. 1 for a set of walkers, Gaussian proposals    */
/* r' = wrap(r_e + sigma z), acceptance min(1, rho_D^2 exp(2 dlnJ)).          */
/* Records are indexed [(sweep * Ne + e) * W + walker].                      */
/* max_moves > 0 stops the first sweep after that many electron moves.       */
/* t_moves_out (optional, [W]): wall seconds each walker spent in its sweeps */
/* after its set-up.                                                          */
/* Returns 0, or -1 if a starting configuration is singular.                 */
/* ------------------------------------------------------------------------ */
int or_vmc(const or_system* s, int n_walkers, const uint32_t* uids, const double* R0,
           int n_sweeps, uint32_t first_step, double sigma, int max_moves, int n_threads,
           double* rec_rho, double* rec_dlnj, double* rec_prob, double* rec_u, uint8_t* rec_acc,
           double* logdet_out, int* sign_out, double* eloc_out,
           double* R_out, int64_t* n_acc_out, double* ainv_out, double* t_moves_out)
{
    const int ne = s->n_up + s->n_dn;
    const int nmax = s->n_up > s->n_dn ? s->n_up : s->n_dn;
    int status = 0;
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 1) reduction(min : status)
#endif
    for (int iw = 0; iw < n_walkers; ++iw) {
        walker w;
        scratch t;
        walker_alloc(s, &w);
        scratch_alloc(&t, nmax);
        w.uid = uids[iw];
        w.n_acc = w.n_prop = 0;
        memcpy(w.R, &R0[(size_t)iw * ne * 3], sizeof(double) * ne * 3);
        if (walker_setup(s, &w) != 0) {
            status = -1;
        } else {
            const double tm0 = wall_seconds();
            int moves_done = 0;
            for (int sw = 0; sw < n_sweeps; ++sw) {
                uint32_t step = first_step + (uint32_t)sw;
                int stop = 0;
                for (int e = 0; e < ne; ++e) {
                    if (max_moves > 0 && moves_done >= max_moves) { stop = 1; break; }
                    int sp = spin_of(s, e);
                    int n = sp == 0 ? s->n_up : s->n_dn;
                    double z[3], rnew[3], gd[3];
                    /* propose */
                    or_gauss3(s->seed, w.uid, step, (uint32_t)e, z);
                    for (int c = 0; c < 3; ++c) rnew[c] = wrap(w.R[3 * e + c] + sigma * z[c], s->L);
                    /* ratio and derivatives at r' */
                    or_orbital_vgl(s, rnew, n, t.v, t.g, t.l);
                    double rho = det_ratio(s, &w, e, &t, gd);
                    double dlnj = j2_delta(s, w.R, e, rnew);
                    /* accept / reject */
                    double prob = rho * rho * exp(2.0 * dlnj);
                    double u = or_accept_uniform(s->seed, w.uid, step, (uint32_t)e);
                    int acc = u < prob;
                    size_t ri = ((size_t)sw * ne + e) * n_walkers + iw;
                    if (rec_rho) rec_rho[ri] = rho;
                    if (rec_dlnj) rec_dlnj[ri] = dlnj;
                    if (rec_prob) rec_prob[ri] = prob;
                    if (rec_u) rec_u[ri] = u;
                    if (rec_acc) rec_acc[ri] = (uint8_t)acc;
                    w.n_prop++;
                    if (acc) {
                        w.n_acc++;
                        accept_move(s, &w, e, rnew, rho, &t);
                    }
                    moves_done++;
                }
                /* local energy */
                w.eloc = walker_eloc(s, &w);
                if (logdet_out) {
                    logdet_out[((size_t)sw * n_walkers + iw) * 2 + 0] = w.logdet[0];
                    logdet_out[((size_t)sw * n_walkers + iw) * 2 + 1] = w.logdet[1];
                }
                if (sign_out) {
                    sign_out[((size_t)sw * n_walkers + iw) * 2 + 0] = w.sign[0];
                    sign_out[((size_t)sw * n_walkers + iw) * 2 + 1] = w.sign[1];
                }
                if (eloc_out) eloc_out[(size_t)sw * n_walkers + iw] = w.eloc;
                if (stop) break;
            }
            if (t_moves_out) t_moves_out[iw] = wall_seconds() - tm0;
            if (R_out) memcpy(&R_out[(size_t)iw * ne * 3], w.R, sizeof(double) * ne * 3);
            if (n_acc_out) n_acc_out[iw] = w.n_acc;
            if (ainv_out) {
                size_t off = 0;
                for (int sp = 0; sp < 2; ++sp) {
                    int n = sp == 0 ? s->n_up : s->n_dn;
                    memcpy(&ainv_out[(size_t)iw * (s->n_up * s->n_up + s->n_dn * s->n_dn) + off],
                           w.Ainv[sp], sizeof(double) * n * n);
                    off += (size_t)n * n;
                }
            }
        }
        scratch_free(&t);
        walker_free(&w);
    }
    return status;
}

/* ------------------------------------------------------------------------ */
/* Virtual moves (the ratio-only evaluations of the local-energy step of     */
/* Alg. 1, Sec. II-A: a non-local energy term needs Psi at points around an  */
/* electron, without moving it).  For every walker (configuration R, set up */
/* from scratch), electron e and point q:                                    */
/*   r_q = wrap(r_e + offsets[q]),                                          */
/*   rho_D = sum_j phi_j(r_q) (A^-1)_{j,i}   (i: e's row in its spin block), */
/*   dlnJ = sum_{m != e} [u(|r_q - r_m|) - u(|r_e - r_m|)],                   */
/*   ratio = Psi(R with r_e -> r_q) / Psi(R) = rho_D exp(dlnJ).              */
/* Outputs [W][Ne][n_q] (any may be NULL).  Returns -1 if a configuration is */
/* singular.                                                                 */
/* ------------------------------------------------------------------------ */
int or_virtual_ratios(const or_system* s, int n_walkers, const double* R0, int n_q, const double* offsets,
                      int n_threads, double* ratio_out, double* rho_out, double* dlnj_out)
{
    const int ne = s->n_up + s->n_dn;
    const int nmax = s->n_up > s->n_dn ? s->n_up : s->n_dn;
    int status = 0;
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 1) reduction(min : status)
#endif
    for (int iw = 0; iw < n_walkers; ++iw) {
        walker w;
        walker_alloc(s, &w);
        memcpy(w.R, &R0[(size_t)iw * ne * 3], sizeof(double) * ne * 3);
        if (walker_setup(s, &w) != 0) {
            status = -1;
            walker_free(&w);
            continue;
        }
        double* v = (double*)malloc(sizeof(double) * nmax);
        double* g = (double*)malloc(sizeof(double) * 3 * nmax);
        double* l = (double*)malloc(sizeof(double) * nmax);
        for (int e = 0; e < ne; ++e) {
            int sp = spin_of(s, e);
            int n = sp == 0 ? s->n_up : s->n_dn;
            int i = e - sp * s->n_up;
            for (int q = 0; q < n_q; ++q) {
                double rq[3];
                for (int c = 0; c < 3; ++c) rq[c] = wrap(w.R[3 * e + c] + offsets[3 * q + c], s->L);
                or_orbital_vgl(s, rq, n, v, g, l);
                double rho = 0;
                for (int j = 0; j < n; ++j) rho += v[j] * w.Ainv[sp][(size_t)j * n + i];
                double dj = j2_delta(s, w.R, e, rq);
                size_t o = ((size_t)iw * ne + e) * n_q + q;
                if (ratio_out) ratio_out[o] = rho * exp(dj);
                if (rho_out) rho_out[o] = rho;
                if (dlnj_out) dlnj_out[o] = dj;
            }
        }
        free(v); free(g); free(l);
        walker_free(&w);
    }
    return status;
}

/* Initial state only: A, G, L, Ainv, log|det|, sign and E_L for each walker. */
int or_setup(const or_system* s, int n_walkers, const double* R0, int n_threads,
             double* logdet_out, int* sign_out, double* eloc_out, double* ainv_out)
{
    const int ne = s->n_up + s->n_dn;
    int status = 0;
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 1) reduction(min : status)
#endif
    for (int iw = 0; iw < n_walkers; ++iw) {
        walker w;
        walker_alloc(s, &w);
        memcpy(w.R, &R0[(size_t)iw * ne * 3], sizeof(double) * ne * 3);
        if (walker_setup(s, &w) != 0) status = -1;
        if (logdet_out) { logdet_out[2 * iw] = w.logdet[0]; logdet_out[2 * iw + 1] = w.logdet[1]; }
        if (sign_out) { sign_out[2 * iw] = w.sign[0]; sign_out[2 * iw + 1] = w.sign[1]; }
        if (eloc_out) eloc_out[iw] = w.eloc;
        if (ainv_out) {
            size_t off = 0;
            for (int sp = 0; sp < 2; ++sp) {
                int n = sp == 0 ? s->n_up : s->n_dn;
                memcpy(&ainv_out[(size_t)iw * (s->n_up * s->n_up + s->n_dn * s->n_dn) + off],
                       w.Ainv[sp], sizeof(double) * n * n);
                off += (size_t)n * n;
            }
        }
        walker_free(&w);
    }
    return status;
}


/* DMC acceptance probability of moving electron e by the displacement delta
   (r' = wrap(r_e + delta)); v = drift at r_e, v' = drift at r':
   P = rho_D^2 exp(2 dlnJ) exp(-(|delta + tau v'|^2 - |delta - tau v|^2) / (2 tau)).
   Leaves the orbital row at r' in t and r', rho_D in rnew, *rho_out. */
static double dmc_move_prob(const or_system* s, const walker* w, int e, const double delta[3],
                            double tau, scratch* t, double rnew[3], double* rho_out)
{
    int sp = spin_of(s, e);
    int n = sp == 0 ? s->n_up : s->n_dn;
    double v[3], gd[3], gj[3], lj, vnew[3];
    drift_current(s, w, e, v);
    for (int c = 0; c < 3; ++c) rnew[c] = wrap(w->R[3 * e + c] + delta[c], s->L);
    or_orbital_vgl(s, rnew, n, t->v, t->g, t->l);
    double rho = det_ratio(s, w, e, t, gd);
    double dlnj = j2_delta(s, w->R, e, rnew);
    j2_grad_lap(s, w->R, e, rnew, gj, &lj);
    double fwd = 0, bwd = 0;
    for (int c = 0; c < 3; ++c) {
        vnew[c] = gd[c] + gj[c];
        double f = delta[c] - tau * v[c];
        double b = delta[c] + tau * vnew[c];
        fwd += f * f;
        bwd += b * b;
    }
    *rho_out = rho;
    return rho * rho * exp(2.0 * dlnj) * exp(-(bwd - fwd) / (2.0 * tau));
}

/* Test entry points for one configuration R of one walker: the drift
   grad ln|Psi| of electron e, and the DMC acceptance probability of moving it
   by delta (rho_D returned through rho_out).  Return -1 if R is singular. */
int or_drift(const or_system* s, const double* R, int e, double v[3])
{
    walker w;
    walker_alloc(s, &w);
    memcpy(w.R, R, sizeof(double) * 3 * (s->n_up + s->n_dn));
    int st = walker_setup(s, &w);
    if (st == 0) drift_current(s, &w, e, v);
    walker_free(&w);
    return st;
}

int or_dmc_move_prob(const or_system* s, const double* R, int e, const double delta[3], double tau,
                     double* prob, double* rho_out)
{
    int nmax = s->n_up > s->n_dn ? s->n_up : s->n_dn;
    walker w;
    scratch t;
    double rnew[3];
    walker_alloc(s, &w);
    scratch_alloc(&t, nmax);
    memcpy(w.R, R, sizeof(double) * 3 * (s->n_up + s->n_dn));
    int st = walker_setup(s, &w);
    if (st == 0) *prob = dmc_move_prob(s, &w, e, delta, tau, &t, rnew, rho_out);
    scratch_free(&t);
    walker_free(&w);
    return st;
}

/* ------------------------------------------------------------------------ */
/* DMC: Alg. 1 with drift-diffusion proposals, reweighting and branching.    */
/* Per move (electron e, current drift v = grad ln|Psi| at r_e):             */
/*   Delta = tau v + sqrt(tau) z,  r' = wrap(r_e + Delta)                    */
/*   P = rho_D^2 exp(2 dlnJ) * exp(-(|Delta + tau v'|^2 - |Delta - tau v|^2) */
/*       / (2 tau)),  v' = grad ln|Psi| at r'; moves with rho_D <= 0 (node    */
/*   crossings) are rejected.                                                */
/* Per generation, for the whole population of this system:                 */
/*   E_c = E_L clipped to [E_T - ecut, E_T + ecut], ecut = 0.2 sqrt(Ne/tau)   */
/*   w = exp(-tau ((E_c(old) + E_c(new))/2 - E_T)), m = min(3, floor(w + u_b))*/
/*   E_est = sum w E_L(new) / sum w,  E_T <- E_est - ln(N_w / N_target) / tau   */
/* Children follow their parent in population order; copy 0 keeps the       */
/* parent's uid.  Returns the final population size, -1 on a singular start, */
/* -2 if the population dies out or exceeds max_pop.                         */
/* Optional records (any may be NULL): per move rho_D, P, u and the decision */
/* at [(gen * Ne + e) * max_pop + walker] (walker = position in the          */
/* generation's population), the proposed position r' at the same index     */
/* times 3, and the multiplicities at [gen * max_pop + w].                   */
/* ------------------------------------------------------------------------ */
int or_dmc(const or_system* s, int n_walkers, const uint32_t* uids, const double* R0,
           int n_gen, uint32_t first_step, double tau, double e_trial, int n_target, int max_pop,
           int n_threads,
           int* pop_out, double* wsum_out, double* eest_out, double* et_out,
           int64_t* counts_out, uint32_t* uids_out, double* R_out, double* eloc_out,
           double* rec_rho, double* rec_prob, double* rec_u, uint8_t* rec_acc, int* mult_out,
           double* rec_rnew)
{
    const int ne = s->n_up + s->n_dn;
    const int nmax = s->n_up > s->n_dn ? s->n_up : s->n_dn;
    const double ecut = 0.2 * sqrt((double)ne / tau);
    const double sqrt_tau = sqrt(tau);
    int pop = n_walkers;
    walker* ws = (walker*)calloc((size_t)max_pop, sizeof(walker));
    double* e_old = (double*)calloc((size_t)max_pop, sizeof(double));
    int status = 0;
    int64_t n_acc = 0, n_prop = 0;
    if (n_walkers > max_pop) { free(ws); free(e_old); return -2; }
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 1) reduction(min : status)
#endif
    for (int iw = 0; iw < pop; ++iw) {
        walker_alloc(s, &ws[iw]);
        ws[iw].uid = uids[iw];
        memcpy(ws[iw].R, &R0[(size_t)iw * ne * 3], sizeof(double) * ne * 3);
        if (walker_setup(s, &ws[iw]) != 0) status = -1;
        e_old[iw] = ws[iw].eloc;
    }
    double e_t = e_trial;
    for (int gen = 0; gen < n_gen && status == 0; ++gen) {
        uint32_t step = first_step + (uint32_t)gen;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : n_acc, n_prop)
#endif
        for (int iw = 0; iw < pop; ++iw) {
            walker* w = &ws[iw];
            scratch t;
            scratch_alloc(&t, nmax);
            for (int e = 0; e < ne; ++e) {
                double v[3], z[3], delta[3], rnew[3], rho;
                drift_current(s, w, e, v);
                or_gauss3(s->seed, w->uid, step, (uint32_t)e, z);
                for (int c = 0; c < 3; ++c) delta[c] = tau * v[c] + sqrt_tau * z[c];
                double prob = dmc_move_prob(s, w, e, delta, tau, &t, rnew, &rho);
                double u = or_accept_uniform(s->seed, w->uid, step, (uint32_t)e);
                int acc = (rho > 0.0) && (u < prob);
                size_t ri = ((size_t)gen * ne + e) * max_pop + iw;
                if (rec_rho) rec_rho[ri] = rho;
                if (rec_prob) rec_prob[ri] = prob;
                if (rec_u) rec_u[ri] = u;
                if (rec_acc) rec_acc[ri] = (uint8_t)acc;
                if (rec_rnew) memcpy(&rec_rnew[3 * ri], rnew, sizeof(double) * 3);
                n_prop++;
                if (acc) {
                    n_acc++;
                    accept_move(s, w, e, rnew, rho, &t);
                }
            }
            w->eloc = walker_eloc(s, w);
            scratch_free(&t);
        }
        /* reweight and branch */
        double wsum = 0, wesum = 0;
        int* mult = (int*)malloc(sizeof(int) * (size_t)pop);
        int new_pop = 0;
        for (int iw = 0; iw < pop; ++iw) {
            double eo = fmin(fmax(e_old[iw], e_t - ecut), e_t + ecut);
            double en = fmin(fmax(ws[iw].eloc, e_t - ecut), e_t + ecut);
            double wt = exp(-tau * (0.5 * (eo + en) - e_t));
            wsum += wt;
            wesum += wt * ws[iw].eloc;
            double ub = or_branch_uniform(s->seed, ws[iw].uid, step);
            int m = (int)floor(wt + ub);
            if (m > 3) m = 3;
            mult[iw] = m;
            if (mult_out) mult_out[(size_t)gen * max_pop + iw] = m;
            new_pop += m;
        }
        if (new_pop == 0 || new_pop > max_pop) {
            free(mult);
            status = -2;
            break;
        }
        walker* nws = (walker*)calloc((size_t)max_pop, sizeof(walker));
        double* ne_old = (double*)calloc((size_t)max_pop, sizeof(double));
        int k = 0;
        for (int iw = 0; iw < pop; ++iw) {
            for (int c = 0; c < mult[iw]; ++c) {
                walker_alloc(s, &nws[k]);
                walker_copy(s, &nws[k], &ws[iw]);
                if (c > 0) nws[k].uid = or_child_uid(s->seed, ws[iw].uid, step, (uint32_t)c);
                ne_old[k] = ws[iw].eloc;
                ++k;
            }
        }
        for (int iw = 0; iw < pop; ++iw) walker_free(&ws[iw]);
        free(ws);
        free(e_old);
        ws = nws;
        e_old = ne_old;
        free(mult);
        /* trial energy */
        double e_est = wesum / wsum;
        e_t = e_est - log((double)new_pop / (double)n_target) / tau;
        pop = new_pop;
        if (pop_out) pop_out[gen] = pop;
        if (wsum_out) wsum_out[gen] = wsum;
        if (eest_out) eest_out[gen] = e_est;
        if (et_out) et_out[gen] = e_t;
    }
    if (counts_out) { counts_out[0] = n_acc; counts_out[1] = n_prop; }
    for (int iw = 0; iw < pop; ++iw) {
        if (status == 0) {
            if (uids_out) uids_out[iw] = ws[iw].uid;
            if (R_out) memcpy(&R_out[(size_t)iw * ne * 3], ws[iw].R, sizeof(double) * ne * 3);
            if (eloc_out) eloc_out[iw] = ws[iw].eloc;
        }
        walker_free(&ws[iw]);
    }
    free(ws);
    free(e_old);
    return status == 0 ? pop : status;
}
