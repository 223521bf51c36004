// Virtual moves: the ratio-only wavefunction evaluations of the local-energy step
// (Alg. 1; the energy is the expensive part of a step, Sec. II-A).  A non-local
// energy term needs Psi at quadrature points around an electron without moving
// it: for walker w, electron e (row i of its spin block) and point q,
//     r_q   = wrap(r_e + offset_q),
//     rho_D = sum_j phi_j(r_q) (A^-1)_{j,i} = phi(r_q) . M[i]      (value-only spline)
//     dlnJ  = sum_{m != e} [u(|r_q - r_m|) - u(|r_e - r_m|)],
//     ratio = rho_D exp(dlnJ).
// One workgroup per (walker, electron), its blocks of one walker on one XCD.  The
// inverse column M[i] stays in registers (VEC orbitals per thread) for all points
// of the electron.  Per point: 64 threads form the stencil (offsets and value
// weights) in LDS, then every thread gathers its orbitals' 64 coefficients in 16-byte
// loads, forms phi_j in T (the path's precision) and adds phi_j (A^-1)_{j,i} in FP64.
// The Jastrow sums run over the electrons (one per thread per pass) with the pair
// terms in T and FP64 sums; the terms at r_e are the same for every point and are
// summed once.  Sums over threads: wave sums, then waves in a fixed order.
#include "cq_device.h"
#include "cq_internal.h"
#include "cq_jastrow.h"

namespace cq {

namespace {

__device__ __forceinline__ double vblock_sum(double x, double* red, int lane, int wave, int nw)
{
    x = wave_sum(x);
    __syncthreads();
    if (lane == 0) red[wave] = x;
    __syncthreads();
    double s = 0.0;
    for (int q = 0; q < nw; ++q) s += red[q];
    return s;
}

template <typename T>
__device__ __forceinline__ T pade_u(T a, T b, T r)
{
    return a * r / ((T)1 + b * r);
}

template <typename T>
__device__ __forceinline__ T pair_dist(const double* ri, const double* rj, double L)
{
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        double x = ri[c] - rj[c];
        x -= L * rint(x / L);
        s += x * x;
    }
    return (T)sqrt(s);
}

}  // namespace

template <typename T, int PASSES>
__global__ __launch_bounds__(kBlock) void k_virtual(CrowdView<T> v, const double* __restrict__ offsets, int nq,
                                                    double* ratio, double* rho_out, double* dlnj_out)
{
    constexpr int VEC = 16 / sizeof(T);
    __shared__ size_t s_idx[64];
    __shared__ T s_w[64];
    __shared__ double s_red[kBlock / 64];
    __shared__ double s_rq[3];
    const int n = v.n, ne = v.ne, G = v.G;
    int w, e;
    xcd_map(blockIdx.x, ne, w, e);
    if (w >= v.W) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = kBlock / 64;
    const int spin = e >= n, i = e - spin * n;
    const double* Rw = v.R + (size_t)w * ne * 3;
    const double re[3] = {Rw[3 * e], Rw[3 * e + 1], Rw[3 * e + 2]};
    // the inverse column of e: VEC consecutive orbitals per thread and pass
    const T* Mi = v.M + (((size_t)w * 2 + spin) * n + i) * (size_t)n;
    T col[PASSES][VEC];
#pragma unroll
    for (int p = 0; p < PASSES; ++p) {
        const int j0 = (p * kBlock + tid) * VEC;
        if (j0 < n) {
            load16(Mi + j0, col[p]);
        } else {
#pragma unroll
            for (int t = 0; t < VEC; ++t) col[p][t] = (T)0;
        }
    }
    // Jastrow terms at r_e, common to every point
    const T L_T = (T)v.L;
    (void)L_T;
    double j_old = 0.0;
    const bool jas = v.use_j2 || v.n_ions;
    if (jas) {
        for (int m = tid; v.use_j2 && m < ne; m += kBlock) {
            if (m == e) continue;
            const T a = (T)(((m >= n) == (spin != 0)) ? v.a_par : v.a_anti);
            j_old += (double)pade_u<T>(a, (T)v.b, pair_dist<T>(re, Rw + 3 * m, v.L));
        }
        double g[3] = {0.0, 0.0, 0.0}, lap = 0.0;  // one-body terms (FP64), centres over the threads
        if (v.n_ions) j_old += j1_at(v, re, tid, kBlock, g, lap);
        j_old = vblock_sum(j_old, s_red, lane, wave, nw);
    }
    for (int q = 0; q < nq; ++q) {
        if (tid < 64) {
            double rq[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) rq[c] = wrap_box(re[c] + offsets[3 * q + c], v.L);
            const AxisW<T> ax = axis_weights<T>(rq[0], v.L, G);
            const AxisW<T> ay = axis_weights<T>(rq[1], v.L, G);
            const AxisW<T> az = axis_weights<T>(rq[2], v.L, G);
            const int px = tid >> 4, py = (tid >> 2) & 3, pz = tid & 3;
            const int jx = (ax.i0 + px + G - 1) % G, jy = (ay.i0 + py + G - 1) % G, jz = (az.i0 + pz + G - 1) % G;
            s_idx[tid] = (((size_t)jx * G + jy) * G + jz) * (size_t)v.n_orb;
            s_w[tid] = ax.b[px] * ay.b[py] * az.b[pz];
            if (tid < 3) s_rq[tid] = rq[tid];
        }
        __syncthreads();
        double part = 0.0;
#pragma unroll
        for (int p = 0; p < PASSES; ++p) {
            const int j0 = (p * kBlock + tid) * VEC;
            if (j0 < n) {
                T acc[VEC];
#pragma unroll
                for (int t = 0; t < VEC; ++t) acc[t] = (T)0;
#pragma unroll 4
                for (int s0 = 0; s0 < 64; s0 += 16) {
                    T vals[16][VEC];
#pragma unroll
                    for (int s = 0; s < 16; ++s) load16(v.table + s_idx[s0 + s] + j0, vals[s]);
#pragma unroll
                    for (int s = 0; s < 16; ++s) {
                        const T ws = s_w[s0 + s];
#pragma unroll
                        for (int t = 0; t < VEC; ++t) acc[t] += ws * vals[s][t];
                    }
                }
#pragma unroll
                for (int t = 0; t < VEC; ++t) part += (double)acc[t] * (double)col[p][t];
            }
        }
        const double rho = vblock_sum(part, s_red, lane, wave, nw);
        double dj = 0.0;
        if (jas) {
            const double rq[3] = {s_rq[0], s_rq[1], s_rq[2]};
            double jn = 0.0;
            for (int m = tid; v.use_j2 && m < ne; m += kBlock) {
                if (m == e) continue;
                const T a = (T)(((m >= n) == (spin != 0)) ? v.a_par : v.a_anti);
                jn += (double)pade_u<T>(a, (T)v.b, pair_dist<T>(rq, Rw + 3 * m, v.L));
            }
            double g[3] = {0.0, 0.0, 0.0}, lap = 0.0;
            if (v.n_ions) jn += j1_at(v, rq, tid, kBlock, g, lap);
            dj = vblock_sum(jn, s_red, lane, wave, nw) - j_old;
        }
        if (tid == 0) {
            const size_t o = ((size_t)w * ne + e) * nq + q;
            if (ratio) ratio[o] = rho * exp(dj);
            if (rho_out) rho_out[o] = rho;
            if (dlnj_out) dlnj_out[o] = dj;
        }
        __syncthreads();  // the next point's stencil overwrites s_idx / s_w
    }
}

template <typename T>
void launch_virtual(const CrowdView<T>& v, const double* offsets, int nq, double* ratio, double* rho, double* dlnj,
                    hipStream_t s)
{
    constexpr int VEC = 16 / sizeof(T);
    const int passes = (v.n + kBlock * VEC - 1) / (kBlock * VEC);
    const dim3 grid(xcd_grid(v.W, v.ne)), block(kBlock);
    if (passes <= 1)
        hipLaunchKernelGGL((k_virtual<T, 1>), grid, block, 0, s, v, offsets, nq, ratio, rho, dlnj);
    else if (passes == 2)
        hipLaunchKernelGGL((k_virtual<T, 2>), grid, block, 0, s, v, offsets, nq, ratio, rho, dlnj);
    else
        hipLaunchKernelGGL((k_virtual<T, 4>), grid, block, 0, s, v, offsets, nq, ratio, rho, dlnj);
}

template void launch_virtual<float>(const CrowdView<float>&, const double*, int, double*, double*, double*,
                                    hipStream_t);
template void launch_virtual<double>(const CrowdView<double>&, const double*, int, double*, double*, double*,
                                     hipStream_t);

}  // namespace cq
