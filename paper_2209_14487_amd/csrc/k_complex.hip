// Kernels of the complex-orbital path (Bloch orbitals with a twist in a general cell):
// set-up rows, Gauss-Jordan inverse with log|det| and phase, one VMC sweep per launch
// (the propose, ratio, accept and update steps of Alg. 1 for every electron in order,
// one workgroup per walker, a Sherman-Morrison update of the walker's inverse in place
// after each acceptance), and the complex local energy.  Everything is FP64.
//
// A spline evaluation takes 64 stencil points of the complex table (16 bytes per
// orbital, coalesced along the orbital index; in the sweep kernel one thread per orbital
// and x-plane of the stencil when 4 N fits the workgroup, the four planes' sums then added
// in order, else one thread per orbital) with five real weights per point: the value weight, the three Cartesian gradient weights
// L^-1 (d/df_a) and the Laplacian weight sum_ab (L^-T L^-1)_ab d2/df_a df_b, so that the
// cell's metric (including its off-diagonal Hessian terms) costs nothing per orbital.  The
// twist multiplies the periodic part by exp(i k.r) and shifts the derivatives.
#include "cq_complex.h"
#include "cq_device.h"
#include "cq_internal.h"

namespace cq {

namespace {

__device__ __forceinline__ double2 cmul(double2 a, double2 b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__device__ __forceinline__ double2 cdiv(double2 a, double2 b)
{
    const double d = b.x * b.x + b.y * b.y;
    return make_double2((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
}

// f = r L^-1
__device__ __forceinline__ void frac_of(const CView& v, const double r[3], double f[3])
{
#pragma unroll
    for (int a = 0; a < 3; ++a) f[a] = r[0] * v.linv[a] + r[1] * v.linv[3 + a] + r[2] * v.linv[6 + a];
}

// r = f L
__device__ __forceinline__ void cart_of(const CView& v, const double f[3], double r[3])
{
#pragma unroll
    for (int c = 0; c < 3; ++c) r[c] = f[0] * v.lat[c] + f[1] * v.lat[3 + c] + f[2] * v.lat[6 + c];
}

__device__ __forceinline__ void wrap_cell(const CView& v, const double r[3], double out[3])
{
    double f[3];
    frac_of(v, r, f);
#pragma unroll
    for (int a = 0; a < 3; ++a) f[a] -= floor(f[a]);
    cart_of(v, f, out);
}

// minimum image in fractional coordinates: d - rint(d L^-1) L
__device__ __forceinline__ double cell_distance(const CView& v, const double* ri, const double* rj, double d[3])
{
    double d0[3] = {ri[0] - rj[0], ri[1] - rj[1], ri[2] - rj[2]}, f[3];
    frac_of(v, d0, f);
#pragma unroll
    for (int a = 0; a < 3; ++a) f[a] -= rint(f[a]);
    cart_of(v, f, d);
    return sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
}

// cubic B-spline weights of control points i0-1 .. i0+2 along a fractional axis (grid G),
// and their first and second derivatives with respect to f
struct FAxis {
    int i0;
    double b[4], d1[4], d2[4];
};

__device__ __forceinline__ FAxis frac_axis(double f, int G)
{
    FAxis r;
    const double s = (f - floor(f)) * G;
    const double fl = floor(s);
    int i = ((int)fl) % G;
    if (i < 0) i += G;
    r.i0 = i;
    const double t = s - fl, u = 1.0 - t, t2 = t * t, t3 = t2 * t;
    const double sixth = 1.0 / 6.0, hg = 0.5 * G, g2 = (double)G * G;
    r.b[0] = u * u * u * sixth;
    r.b[1] = (3.0 * t3 - 6.0 * t2 + 4.0) * sixth;
    r.b[2] = (-3.0 * t3 + 3.0 * t2 + 3.0 * t + 1.0) * sixth;
    r.b[3] = t3 * sixth;
    r.d1[0] = -u * u * hg;
    r.d1[1] = (3.0 * t2 - 4.0 * t) * hg;
    r.d1[2] = (-3.0 * t2 + 2.0 * t + 1.0) * hg;
    r.d1[3] = t2 * hg;
    r.d2[0] = u * g2;
    r.d2[1] = (3.0 * t - 2.0) * g2;
    r.d2[2] = (-3.0 * t + 1.0) * g2;
    r.d2[3] = t * g2;
    return r;
}

// Stencil entry of lane l (point 16 x + 4 y + z) at the wrapped position r: table offset
// and the five weights (value, Cartesian gradient, Laplacian through the metric).
__device__ __forceinline__ void cstencil(const CView& v, const double r[3], int l, size_t* sidx, double* sw)
{
    double f[3];
    frac_of(v, r, f);
    const FAxis ax = frac_axis(f[0], v.G), ay = frac_axis(f[1], v.G), az = frac_axis(f[2], v.G);
    const int p = l >> 4, q = (l >> 2) & 3, s = l & 3, G = v.G;
    const double bx = ax.b[p], dx = ax.d1[p], ddx = ax.d2[p];
    const double by = ay.b[q], dy = ay.d1[q], ddy = ay.d2[q];
    const double bz = az.b[s], dz = az.d1[s], ddz = az.d2[s];
    const double gf[3] = {dx * by * bz, bx * dy * bz, bx * by * dz};
    const double* m = v.metric;
    const double lap = m[0] * (ddx * by * bz) + m[1] * (bx * ddy * bz) + m[2] * (bx * by * ddz) +
                       2.0 * (m[3] * (dx * dy * bz) + m[4] * (dx * by * dz) + m[5] * (bx * dy * dz));
    const int jx = (ax.i0 + p + G - 1) % G, jy = (ay.i0 + q + G - 1) % G, jz = (az.i0 + s + G - 1) % G;
    sidx[l] = (((size_t)jx * G + jy) * G + jz) * (size_t)v.n_orb;
    sw[l * 5 + 0] = bx * by * bz;
#pragma unroll
    for (int c = 0; c < 3; ++c) sw[l * 5 + 1 + c] = v.linv[c * 3] * gf[0] + v.linv[c * 3 + 1] * gf[1] + v.linv[c * 3 + 2] * gf[2];
    sw[l * 5 + 4] = lap;
}

// The twisted rows from the periodic part's sums acc[5] (value, gradient, Laplacian):
// phi = ph s, grad phi = ph (grad s + i k s), lap phi = ph (lap s + 2 i k.grad s - k^2 s).
__device__ __forceinline__ void twist_rows(const CView& v, double2 ph, const double2 acc[5], double2 out[5])
{
    const double2 s = acc[0];
    out[0] = cmul(ph, s);
    double2 kg = make_double2(0.0, 0.0);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        out[1 + c] = cmul(ph, make_double2(acc[1 + c].x - v.k[c] * s.y, acc[1 + c].y + v.k[c] * s.x));
        kg.x += v.k[c] * acc[1 + c].x;
        kg.y += v.k[c] * acc[1 + c].y;
    }
    out[4] = cmul(ph, make_double2(acc[4].x - 2.0 * kg.y - v.k2 * s.x, acc[4].y + 2.0 * kg.x - v.k2 * s.y));
}

// Coefficient i of the table (complex64 tables are widened to FP64).
template <bool F32>
__device__ __forceinline__ double2 coef(const CView& v, size_t i)
{
    if constexpr (F32) {
        const float2 c = v.table32[i];
        return make_double2((double)c.x, (double)c.y);
    } else {
        return v.table[i];
    }
}

// Value, gradient and Laplacian of orbital j at the stencil's position (twist phase ph =
// exp(i k.r)), into out[5].
template <bool F32>
__device__ __forceinline__ void corbital(const CView& v, const size_t* sidx, const double* sw, double2 ph, int j,
                                         double2 out[5])
{
    double2 acc[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) acc[k] = make_double2(0.0, 0.0);
#pragma unroll 16
    for (int q = 0; q < 64; ++q) {
        const double2 c = coef<F32>(v, sidx[q] + j);
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            acc[k].x += sw[q * 5 + k] * c.x;
            acc[k].y += sw[q * 5 + k] * c.y;
        }
    }
    twist_rows(v, ph, acc, out);
}

__device__ __forceinline__ double2 twist_phase(const CView& v, const double r[3])
{
    const double th = v.k[0] * r[0] + v.k[1] * r[1] + v.k[2] * r[2];
    return make_double2(cos(th), sin(th));
}

// Three sums over the workgroup in a fixed order (each wave's, then the waves in index
// order); every thread gets them.
__device__ __forceinline__ void cblock_sum3(double& a, double& b, double& c, double (*red)[kBlock / 64], int lane,
                                            int wave, int nw)
{
    a = wave_sum(a);
    b = wave_sum(b);
    c = wave_sum(c);
    __syncthreads();
    if (lane == 0) {
        red[0][wave] = a;
        red[1][wave] = b;
        red[2][wave] = c;
    }
    __syncthreads();
    a = b = c = 0.0;
    for (int q = 0; q < nw; ++q) {
        a += red[0][q];
        b += red[1][q];
        c += red[2][q];
    }
}

constexpr int kRowBatch = 4;  // rows of the inverse one wave updates with their loads in flight together

}  // namespace

// Orbital rows of electron e of walker w at its (wrapped) position: one workgroup each.
template <bool F32>
__global__ __launch_bounds__(kBlock) void k_csetup_rows(CView v)
{
    __shared__ size_t s_idx[64];
    __shared__ double s_w[64 * 5];
    __shared__ double s_r[3];
    const int w = blockIdx.x / v.ne, e = blockIdx.x % v.ne;
    if (w >= v.W) return;
    const int tid = threadIdx.x, n = v.n;
    if (tid < 64) {
        double r[3];
        wrap_cell(v, v.R + ((size_t)w * v.ne + e) * 3, r);
        cstencil(v, r, tid, s_idx, s_w);
        if (tid < 3) s_r[tid] = r[tid];
    }
    __syncthreads();
    const double r[3] = {s_r[0], s_r[1], s_r[2]};
    const double2 ph = twist_phase(v, r);
    const int spin = e >= n, a = e - spin * n;
    double2* dst = v.VGL + (((size_t)w * 2 + spin) * n + a) * 5 * (size_t)n;
    for (int j = tid; j < n; j += blockDim.x) {
        double2 o[5];
        corbital<F32>(v, s_idx, s_w, ph, j, o);
#pragma unroll
        for (int k = 0; k < 5; ++k) dst[(size_t)k * n + j] = o[k];
    }
}

// Gauss-Jordan inverse with partial pivoting (largest modulus, lowest row on ties) of the
// value rows A[i][j] = phi_j(r_i) of one walker and spin, in the workspace [A | I]; the
// inverse is written transposed (M[a][j] = (A^-1)[j][a]), log|det| = sum log|pivot| and the
// phase = sum arg(pivot) + pi per row swap, wrapped to [-pi, pi].  A pivot of modulus at
// most n eps max|A_ij| (numerically singular) or not finite sets status bit 0 of the walker
// and leaves M unchanged.
__global__ __launch_bounds__(kBlock) void k_cinverse(CView v)
{
    __shared__ double2 s_col[kCMaxN];
    __shared__ double s_best[kBlock / 64];
    __shared__ int s_bi[kBlock / 64];
    __shared__ int s_piv, s_bad;
    __shared__ double s_tiny;
    const int w = blockIdx.x >> 1, spin = blockIdx.x & 1;
    if (w >= v.W) return;
    const int n = v.n, n2 = 2 * n, tid = threadIdx.x, nt = blockDim.x, lane = tid & 63, wave = tid >> 6;
    const int nw = nt >> 6;
    double2* aug = v.work + ((size_t)w * 2 + spin) * n * (size_t)n2;
    const double2* rows = v.VGL + ((size_t)w * 2 + spin) * n * 5 * (size_t)n;
    double amax = 0.0;
    for (size_t idx = tid; idx < (size_t)n * n2; idx += nt) {
        const int i = (int)(idx / n2), j = (int)(idx % n2);
        const double2 x = j < n ? rows[(size_t)i * 5 * n + j] : make_double2(j - n == i ? 1.0 : 0.0, 0.0);
        aug[idx] = x;
        if (j < n) amax = fmax(amax, hypot(x.x, x.y));
    }
    for (int off = 32; off >= 1; off >>= 1) amax = fmax(amax, __shfl_xor(amax, off));
    if (lane == 0) s_best[wave] = amax;
    __syncthreads();
    if (tid == 0) {
        double m = s_best[0];
        for (int q = 1; q < nw; ++q) m = fmax(m, s_best[q]);
        s_tiny = n * 2.220446049250313e-16 * m;
        s_bad = 0;
    }
    double ld = 0.0, ph = 0.0;
    __syncthreads();
    for (int c = 0; c < n; ++c) {
        // pivot: largest modulus in column c at or below row c
        double best = -1.0;
        int bi = n;
        for (int r = c + tid; r < n; r += nt) {
            const double2 x = aug[(size_t)r * n2 + c];
            const double m = hypot(x.x, x.y);
            if (m > best) {
                best = m;
                bi = r;
            }
        }
        for (int off = 32; off >= 1; off >>= 1) {
            const double ob = __shfl_xor(best, off);
            const int oi = __shfl_xor(bi, off);
            if (ob > best || (ob == best && oi < bi)) {
                best = ob;
                bi = oi;
            }
        }
        if (lane == 0) {
            s_best[wave] = best;
            s_bi[wave] = bi;
        }
        __syncthreads();
        if (tid == 0) {
            double b = s_best[0];
            int p = s_bi[0];
            for (int q = 1; q < nw; ++q)
                if (s_best[q] > b || (s_best[q] == b && s_bi[q] < p)) {
                    b = s_best[q];
                    p = s_bi[q];
                }
            s_piv = p;
            if (!(b > s_tiny) || !isfinite(b) || p >= n) s_bad = 1;
        }
        __syncthreads();
        if (s_bad) break;
        const int p = s_piv;
        if (p != c)
            for (int j = tid; j < n2; j += nt) {
                const double2 t = aug[(size_t)c * n2 + j];
                aug[(size_t)c * n2 + j] = aug[(size_t)p * n2 + j];
                aug[(size_t)p * n2 + j] = t;
            }
        __syncthreads();
        const double2 pv = aug[(size_t)c * n2 + c];
        if (tid == 0) {
            ld += log(hypot(pv.x, pv.y));
            ph += atan2(pv.y, pv.x) + (p != c ? M_PI : 0.0);
        }
        __syncthreads();  // every thread has read the pivot before the row changes
        for (int j = c + tid; j < n2; j += nt) aug[(size_t)c * n2 + j] = cdiv(aug[(size_t)c * n2 + j], pv);
        for (int r = tid; r < n; r += nt) s_col[r] = aug[(size_t)r * n2 + c];
        __syncthreads();
        const int width = n2 - c - 1;
        for (size_t idx = tid; idx < (size_t)n * width; idx += nt) {
            const int r = (int)(idx / width), j = c + 1 + (int)(idx % width);
            if (r == c) continue;
            const double2 f = s_col[r], x = aug[(size_t)c * n2 + j];
            double2& y = aug[(size_t)r * n2 + j];
            y.x -= f.x * x.x - f.y * x.y;
            y.y -= f.x * x.y + f.y * x.x;
        }
        __syncthreads();
    }
    if (s_bad) {
        if (tid == 0) atomicOr(&v.status[w], 1);
        return;
    }
    double2* M = v.M + ((size_t)w * 2 + spin) * n * (size_t)n;
    for (size_t idx = tid; idx < (size_t)n * n; idx += nt) {
        const int a = (int)(idx / n), j = (int)(idx % n);
        M[idx] = aug[(size_t)j * n2 + n + a];
    }
    if (tid == 0) {
        v.logdet[w * 2 + spin] = ld;
        v.phase[w * 2 + spin] = remainder(ph, 2.0 * M_PI);
    }
}

// One VMC sweep of walker w (one workgroup): electron e in order proposes
// r' = wrap(r_e + sigma z), takes rho = sum_j phi_j(r') (A^-1)_{j a} and the pair-Jastrow
// change, accepts when u < |rho|^2 exp(2 dlnJ), and on acceptance updates the inverse by
// Sherman-Morrison, M[b] -= ((u . M[b]) - delta_ab) / rho M_old[a], copies the rows, moves
// the electron and adds log|rho| and arg rho to log|det| and the phase.
template <bool F32>
__global__ __launch_bounds__(kBlock) void k_csweep(CView v)
{
    extern __shared__ double2 cs_lds[];  // u [5][n], c0 [n], then (4 n <= threads) the planes' sums [4][5][n]
    __shared__ size_t s_idx[64];
    __shared__ double s_w[64 * 5];
    __shared__ double s_red[3][kBlock / 64];
    __shared__ double s_rp[3];
    const int w = blockIdx.x;
    if (w >= v.W) return;
    const int n = v.n, ne = v.ne, tid = threadIdx.x, nt = blockDim.x, lane = tid & 63, wave = tid >> 6;
    const int nw = nt >> 6;
    double2* u = cs_lds;
    double2* c0 = cs_lds + (size_t)5 * n;
    double* Rw = v.R + (size_t)w * ne * 3;
    const uint32_t uid = v.uid[w];
    const bool rec = v.rec_sweep < v.rec_cap;
    for (int e = 0; e < ne; ++e) {
        const int spin = e >= n, a = e - spin * n;
        double2* M = v.M + ((size_t)w * 2 + spin) * n * (size_t)n;
        __syncthreads();  // the previous move's readers of the stencil, rows, c0 and R are done
        if (wave == 0) {
            double z[3], r1[3], rp[3];
            gauss3(v.seed, uid, v.step, (uint32_t)e, z);
#pragma unroll
            for (int c = 0; c < 3; ++c) r1[c] = Rw[(size_t)e * 3 + c] + v.sigma * z[c];
            wrap_cell(v, r1, rp);
            cstencil(v, rp, lane, s_idx, s_w);
            if (lane < 3) s_rp[lane] = rp[lane];
        }
        __syncthreads();
        const double rp[3] = {s_rp[0], s_rp[1], s_rp[2]};
        const double re[3] = {Rw[(size_t)e * 3], Rw[(size_t)e * 3 + 1], Rw[(size_t)e * 3 + 2]};
        const double2 ph = twist_phase(v, rp);
        if (4 * n <= nt) {
            // one x-plane of the stencil (16 points) per item, the planes' sums added in order
            double2* part = c0 + n;  // [4][5][n]
            if (tid < 4 * n) {
                const int p = tid / n, j = tid % n;
                double2 acc[5];
#pragma unroll
                for (int k = 0; k < 5; ++k) acc[k] = make_double2(0.0, 0.0);
                double2 cq[16];
#pragma unroll
                for (int q = 0; q < 16; ++q) cq[q] = coef<F32>(v, s_idx[p * 16 + q] + j);
#pragma unroll
                for (int q = 0; q < 16; ++q)
#pragma unroll
                    for (int k = 0; k < 5; ++k) {
                        acc[k].x += s_w[(p * 16 + q) * 5 + k] * cq[q].x;
                        acc[k].y += s_w[(p * 16 + q) * 5 + k] * cq[q].y;
                    }
#pragma unroll
                for (int k = 0; k < 5; ++k) part[((size_t)p * 5 + k) * n + j] = acc[k];
            }
            __syncthreads();
            for (int j = tid; j < n; j += nt) {
                double2 acc[5];
#pragma unroll
                for (int k = 0; k < 5; ++k) {
                    acc[k] = part[(size_t)k * n + j];
                    for (int p = 1; p < 4; ++p) {
                        acc[k].x += part[((size_t)p * 5 + k) * n + j].x;
                        acc[k].y += part[((size_t)p * 5 + k) * n + j].y;
                    }
                }
                double2 o[5];
                twist_rows(v, ph, acc, o);
#pragma unroll
                for (int k = 0; k < 5; ++k) u[(size_t)k * n + j] = o[k];
            }
        } else {
            for (int j = tid; j < n; j += nt) {
                double2 o[5];
                corbital<F32>(v, s_idx, s_w, ph, j, o);
#pragma unroll
                for (int k = 0; k < 5; ++k) u[(size_t)k * n + j] = o[k];
            }
        }
        __syncthreads();
        double rx = 0.0, ry = 0.0, dj = 0.0;
        for (int j = tid; j < n; j += nt) {
            const double2 p = cmul(u[j], M[(size_t)a * n + j]);
            rx += p.x;
            ry += p.y;
        }
        if (v.use_j2)
            for (int m = tid; m < ne; m += nt) {
                if (m == e) continue;
                const double aa = ((m >= n) == (spin != 0)) ? v.a_par : v.a_anti;
                double d[3], u1, u0, du, d2u;
                pade(aa, v.b, cell_distance(v, rp, Rw + (size_t)m * 3, d), u1, du, d2u);
                pade(aa, v.b, cell_distance(v, re, Rw + (size_t)m * 3, d), u0, du, d2u);
                dj += u1 - u0;
            }
        cblock_sum3(rx, ry, dj, s_red, lane, wave, nw);
        const double2 rho = make_double2(rx, ry);
        const double prob = (rx * rx + ry * ry) * exp(2.0 * dj);
        const bool acc = accept_uniform(v.seed, uid, v.step, (uint32_t)e) < prob;
        if (tid == 0) {
            if (rec) {
                const size_t ri = ((size_t)v.rec_sweep * ne + e) * v.W + w;
                v.rec_rho[ri] = rho;
                v.rec_dlnj[ri] = dj;
                v.rec_prob[ri] = prob;
                v.rec_acc[ri] = (uint8_t)acc;
            }
            v.nprop[w] += 1;
        }
        if (!acc) continue;
        for (int j = tid; j < n; j += nt) c0[j] = M[(size_t)a * n + j];
        __syncthreads();  // the old column is in LDS before any row changes
        const double2 irho = cdiv(make_double2(1.0, 0.0), rho);
        // rows b0 .. b0 + kRowBatch - 1 per wave and pass: every row's loads are issued
        // before any of them is used, and its dot and update are those of a row alone
        constexpr int RB = kRowBatch;
        for (int b0 = wave * RB; b0 < n; b0 += nw * RB) {
            double xr[RB], xi[RB];
#pragma unroll
            for (int r = 0; r < RB; ++r) xr[r] = xi[r] = 0.0;
            for (int j = lane; j < n; j += 64) {
                const double2 uj = u[j];
                double2 m[RB];
#pragma unroll
                for (int r = 0; r < RB; ++r)
                    m[r] = b0 + r < n ? M[(size_t)(b0 + r) * n + j] : make_double2(0.0, 0.0);
#pragma unroll
                for (int r = 0; r < RB; ++r) {
                    const double2 p = cmul(uj, m[r]);
                    xr[r] += p.x;
                    xi[r] += p.y;
                }
            }
            double2 beta[RB];
#pragma unroll
            for (int r = 0; r < RB; ++r)
                beta[r] = cmul(make_double2(wave_sum(xr[r]) - (b0 + r == a ? 1.0 : 0.0), wave_sum(xi[r])), irho);
            for (int j = lane; j < n; j += 64) {
                const double2 c = c0[j];
                double2 m[RB];
#pragma unroll
                for (int r = 0; r < RB; ++r)
                    m[r] = b0 + r < n ? M[(size_t)(b0 + r) * n + j] : make_double2(0.0, 0.0);
#pragma unroll
                for (int r = 0; r < RB; ++r) {
                    if (b0 + r < n) {
                        const double2 q = cmul(beta[r], c);
                        M[(size_t)(b0 + r) * n + j] = make_double2(m[r].x - q.x, m[r].y - q.y);
                    }
                }
            }
        }
        double2* dst = v.VGL + (((size_t)w * 2 + spin) * n + a) * 5 * (size_t)n;
        for (int i = tid; i < 5 * n; i += nt) dst[i] = u[i];
        if (tid == 0) {
            v.logdet[w * 2 + spin] += 0.5 * log(rx * rx + ry * ry);
            v.phase[w * 2 + spin] = remainder(v.phase[w * 2 + spin] + atan2(ry, rx), 2.0 * M_PI);
            v.nacc[w] += 1;
        }
        if (tid < 3) Rw[(size_t)e * 3 + tid] = rp[tid];
    }
}

// Complex kinetic local energy of walker w: -1/2 sum_i [l_i + lap_i U + |grad_i U|^2 +
// 2 g_i . grad_i U], g_i = sum_j grad phi_j(r_i) (A^-1)_{j i}, l_i likewise with the
// Laplacian rows; one wave per electron, the electrons summed in order.
__global__ __launch_bounds__(kBlock) void k_cenergy(CView v)
{
    __shared__ double2 s_part[2 * kCMaxN];
    const int w = blockIdx.x;
    if (w >= v.W) return;
    const int n = v.n, ne = v.ne, tid = threadIdx.x, nt = blockDim.x, lane = tid & 63, wave = tid >> 6;
    const int nw = nt >> 6;
    const double* Rw = v.R + (size_t)w * ne * 3;
    for (int ei = wave; ei < ne; ei += nw) {
        const int spin = ei >= n, a = ei - spin * n;
        const double2* Mr = v.M + (((size_t)w * 2 + spin) * n + a) * n;
        const double2* rows = v.VGL + (((size_t)w * 2 + spin) * n + a) * 5 * (size_t)n;
        double s[8] = {0, 0, 0, 0, 0, 0, 0, 0};  // g x y z, l: real and imaginary
        for (int j = lane; j < n; j += 64) {
            const double2 m = Mr[j];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const double2 p = cmul(rows[(size_t)(1 + k) * n + j], m);
                s[2 * k] += p.x;
                s[2 * k + 1] += p.y;
            }
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) s[k] = wave_sum(s[k]);
        double gu[3] = {0.0, 0.0, 0.0}, lu = 0.0;
        if (v.use_j2)
            for (int m = lane; m < ne; m += 64) {
                if (m == ei) continue;
                const double aa = ((m >= n) == (spin != 0)) ? v.a_par : v.a_anti;
                double d[3], uu, du, d2u;
                const double r = cell_distance(v, Rw + (size_t)ei * 3, Rw + (size_t)m * 3, d);
                pade(aa, v.b, r, uu, du, d2u);
#pragma unroll
                for (int c = 0; c < 3; ++c) gu[c] += du * d[c] / r;
                lu += d2u + 2.0 * du / r;
            }
#pragma unroll
        for (int c = 0; c < 3; ++c) gu[c] = wave_sum(gu[c]);
        lu = wave_sum(lu);
        if (lane == 0) {
            const double gg = gu[0] * gu[0] + gu[1] * gu[1] + gu[2] * gu[2];
            const double dr = s[0] * gu[0] + s[2] * gu[1] + s[4] * gu[2];
            const double di = s[1] * gu[0] + s[3] * gu[1] + s[5] * gu[2];
            s_part[ei] = make_double2(-0.5 * (s[6] + lu + gg + 2.0 * dr), -0.5 * (s[7] + 2.0 * di));
        }
    }
    __syncthreads();
    if (tid == 0) {
        double2 t = make_double2(0.0, 0.0);
        for (int i = 0; i < ne; ++i) {
            t.x += s_part[i].x;
            t.y += s_part[i].y;
        }
        v.eloc[w] = t;
    }
}

void launch_csetup_rows(const CView& v, hipStream_t s)
{
    if (v.table32)
        hipLaunchKernelGGL(k_csetup_rows<true>, dim3(v.W * v.ne), dim3(kBlock), 0, s, v);
    else
        hipLaunchKernelGGL(k_csetup_rows<false>, dim3(v.W * v.ne), dim3(kBlock), 0, s, v);
}

void launch_cinverse(const CView& v, hipStream_t s)
{
    hipLaunchKernelGGL(k_cinverse, dim3(2 * v.W), dim3(kBlock), 0, s, v);
}

void launch_csweep(const CView& v, hipStream_t s)
{
    const size_t lds = sizeof(double2) * (4 * v.n <= kBlock ? 26 : 6) * (size_t)v.n;
    static bool opted = false;  // the dynamic LDS of the largest N, for both kernels
    if (!opted) {
        for (const void* f : {(const void*)k_csweep<true>, (const void*)k_csweep<false>})
            (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)(sizeof(double2) * 6 * kCMaxN));
        opted = true;
    }
    if (v.table32)
        hipLaunchKernelGGL(k_csweep<true>, dim3(v.W), dim3(kBlock), lds, s, v);
    else
        hipLaunchKernelGGL(k_csweep<false>, dim3(v.W), dim3(kBlock), lds, s, v);
}

void launch_cenergy(const CView& v, hipStream_t s)
{
    hipLaunchKernelGGL(k_cenergy, dim3(v.W), dim3(kBlock), 0, s, v);
}

}  // namespace cq
