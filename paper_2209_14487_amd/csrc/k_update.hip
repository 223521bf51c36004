// Inverse update and local energy kernels.
//
// k_flush_vec   applies the accepted moves m = 0 .. cnt-1 of one window to the
//               inverse in one read and one write of M = (A^-1)^T.  Move m
//               replaced row e_m of A by u_m with ratio rho_m; c_m is the inverse
//               column of e_m just before move m.  For every row a of M
//               (a column of A^-1) the moves act in order as rank-1 updates:
//                 p_m  = M[a] . u_m                        (rank-k product)
//                 b_m  = (p_m - sum_{j<m} b_j (u_m . c_j) - delta(a, e_m)) / rho_m
//                 M[a] -= sum_m b_m c_m                     (rank-k product)
//               k = 1 is Sherman-Morrison; for k > 1 this is the Woodbury update
//               with the k x k window matrix factorised in move order, which
//               keeps the rounding of a sequence of Sherman-Morrison steps.
//               Each wave keeps RPW rows in registers and streams the window rows.
// k_energy_*    kinetic local energy (the local-energy step of Alg. 1):
//                 E_L = -1/2 sum_i [l_i + lap_i U + |grad_i U|^2 + 2 g_i . grad_i U]
//               g_i = sum_j grad phi_j(r_i) A^-1_ji is the dot of gradient row i
//               with row i of M (likewise l_i); FP64 sums over electrons.
#include <algorithm>

#include "cq_device.h"
#include "cq_internal.h"
#include "cq_jastrow.h"

namespace cq {

constexpr int kRowsPerWave = 4;
constexpr int kRowsPerBlock = 4 * kRowsPerWave;

template <typename T, int EPL>
__device__ __forceinline__ void flush_vec_body(const CrowdView<T>& v, int spin, const int w, const int strip)
{
    constexpr int VEC = 16 / sizeof(T);
    constexpr int NV = EPL / VEC;  // 16-byte vectors per lane per row
    __shared__ double gG[kMaxDelay][kMaxDelay + 1];
    __shared__ double grho[kMaxDelay];
    __shared__ int wel[kMaxDelay];
    __shared__ int wsl[kMaxDelay];
    __shared__ double pq[4][kRowsPerWave][kMaxDelay];
    __shared__ double xs[4][kRowsPerWave][kMaxDelay];
    const int n = v.n, K = v.K;
    const int nstrip = (n + kRowsPerBlock - 1) / kRowsPerBlock;
    if (w >= v.W) return;
    int cnt = v.cnt[(size_t)2 * v.W + w];  // final size of the window
    if (cnt > K) cnt = K;
    if (cnt <= 0) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int i = tid; i < cnt * cnt; i += kBlock) {
        const int r = i / cnt, c = i % cnt;
        gG[r][c] = c < r ? v.wG[((size_t)w * K + r) * K + c] : 0.0;
    }
    if (tid < cnt) {
        wel[tid] = v.welec[(size_t)w * K + tid];
        grho[tid] = v.wrho[(size_t)w * K + tid];
        const int sl = v.wslot[(size_t)w * K + tid];
        if (sl < 0 || sl >= v.QR) atomicOr(&v.status[w], 2);
        wsl[tid] = sl < 0 || sl >= v.QR ? 0 : sl;
    }

    // copy the accepted orbital rows of the window into the A, G, L rows
    __syncthreads();
    for (int mm = strip; mm < cnt; mm += nstrip) {
        const int ea = wel[mm];
        if (ea < 0 || ea >= n) {  // never written: bookkeeping error, flagged, row left alone
            if (tid == 0) atomicOr(&v.status[w], 2);
            continue;
        }
        const T* src = v.stage + ((size_t)w * v.QR + wsl[mm]) * 5 * (size_t)n;
        T* dst = v.VGL + (((size_t)w * 2 + spin) * n + ea) * 5 * (size_t)n;
        for (int i = tid; i < 5 * n; i += kBlock) dst[i] = src[i];
    }
    __syncthreads();

    const int r0 = strip * kRowsPerBlock + wave * kRowsPerWave;
    T* Mbase = v.M + ((size_t)w * 2 + spin) * n * (size_t)n;
    T mr[kRowsPerWave][EPL];
#pragma unroll
    for (int q = 0; q < kRowsPerWave; ++q)
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            const int j = (i * 64 + lane) * VEC;
            if (r0 + q < n && j < n) {
                load16(Mbase + (size_t)(r0 + q) * n + j, &mr[q][i * VEC]);
            } else {
#pragma unroll
                for (int t = 0; t < VEC; ++t) mr[q][i * VEC + t] = (T)0;
            }
        }
    // p[q][m] = M[r] . u_m
    for (int mm = 0; mm < cnt; ++mm) {
        T u[EPL];
        const T* up = v.stage + (((size_t)w * v.QR + wsl[mm]) * 5 + 0) * n;
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            const int j = (i * 64 + lane) * VEC;
            if (j < n) {
                load16(up + j, &u[i * VEC]);
            } else {
#pragma unroll
                for (int t = 0; t < VEC; ++t) u[i * VEC + t] = (T)0;
            }
        }
#pragma unroll
        for (int q = 0; q < kRowsPerWave; ++q) {
            T s = (T)0;
#pragma unroll
            for (int i = 0; i < EPL; ++i) s += mr[q][i] * u[i];
            s = wave_sum(s);
            if (lane == 0) pq[wave][q][mm] = (double)s;
        }
    }
    __syncthreads();
    // b[q][m]: forward substitution in move order, one lane per row
    if (lane < kRowsPerWave) {
        const int q = lane, r = r0 + q;
        for (int mm = 0; mm < cnt; ++mm) {
            double t = pq[wave][q][mm] - (r == wel[mm] ? 1.0 : 0.0);
            for (int j = 0; j < mm; ++j) t -= xs[wave][q][j] * gG[mm][j];
            xs[wave][q][mm] = t / grho[mm];
        }
    }
    __syncthreads();
    // M[r] -= sum_m b[q][m] c_m
    for (int mm = 0; mm < cnt; ++mm) {
        T cm[EPL];
        const T* cp = v.Cbuf + ((size_t)w * K + mm) * n;
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            const int j = (i * 64 + lane) * VEC;
            if (j < n) {
                load16(cp + j, &cm[i * VEC]);
            } else {
#pragma unroll
                for (int t = 0; t < VEC; ++t) cm[i * VEC + t] = (T)0;
            }
        }
#pragma unroll
        for (int q = 0; q < kRowsPerWave; ++q) {
            const T x = (T)xs[wave][q][mm];
#pragma unroll
            for (int i = 0; i < EPL; ++i) mr[q][i] -= x * cm[i];
        }
    }
#pragma unroll
    for (int q = 0; q < kRowsPerWave; ++q)
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            const int j = (i * 64 + lane) * VEC;
            if (r0 + q < n && j < n) store16(Mbase + (size_t)(r0 + q) * n + j, &mr[q][i * VEC]);
        }
}

template <typename T, int EPL>
__global__ __launch_bounds__(kBlock) void k_flush_vec(CrowdView<T> v, int spin)
{
    int w, strip;
    xcd_map(blockIdx.x, (v.n + kRowsPerBlock - 1) / kRowsPerBlock, w, strip);
    flush_vec_body<T, EPL>(v, spin, w, strip);
}

// Several systems in one launch: item i = (system, walker, strip of 16 rows); persistent.  EPL
// covers the largest system; the smaller ones leave the lanes past their N idle.
template <typename T, int EPL>
__global__ __launch_bounds__(kBlock) void k_flush_vec_multi(const CrowdView<T>* __restrict__ views,
                                                            const int4* __restrict__ items, int n_items, int spin)
{
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        const int4 item = items[it];
        flush_vec_body<T, EPL>(views[item.x], spin, item.y, item.z);
        __syncthreads();  // the next item reuses the shared memory
    }
}

template <typename T>
void launch_flush_vec_multi(const CrowdView<T>* views, const int4* strips, int n_strips, int max_n, int spin, int grid,
                            hipStream_t s)
{
    constexpr int VEC = 16 / sizeof(T);
    const int per_lane = (max_n + 63) / 64;
    const dim3 g(std::min(n_strips, grid)), b(kBlock);
    if (per_lane <= VEC)
        hipLaunchKernelGGL((k_flush_vec_multi<T, VEC>), g, b, 0, s, views, strips, n_strips, spin);
    else if (per_lane <= 4)
        hipLaunchKernelGGL((k_flush_vec_multi<T, 4>), g, b, 0, s, views, strips, n_strips, spin);
    else if (per_lane <= 8)
        hipLaunchKernelGGL((k_flush_vec_multi<T, 8>), g, b, 0, s, views, strips, n_strips, spin);
    else if (per_lane <= 16)
        hipLaunchKernelGGL((k_flush_vec_multi<T, 16>), g, b, 0, s, views, strips, n_strips, spin);
    else
        hipLaunchKernelGGL((k_flush_vec_multi<T, 32>), g, b, 0, s, views, strips, n_strips, spin);
}

template <typename T>
void launch_flush(const CrowdView<T>& v, int spin, hipStream_t s, bool linv_ready)
{
    if constexpr (sizeof(T) == 4) {
        if (flush_mfma_fits(v.n)) {
            launch_flush_mfma(v, spin, s, linv_ready);
            return;
        }
    } else {
        // the batched path (its windows come with linv_ready), when its shapes ask for the
        // FP64 matrix cores
        if (linv_ready && v.upd_mfma && flush_f64_mfma_fits(v.n)) {
            launch_flush_f64_mfma(v, spin, s);
            return;
        }
    }
    constexpr int VEC = 16 / sizeof(T);
    const int nstrip = (v.n + kRowsPerBlock - 1) / kRowsPerBlock;
    const dim3 grid(xcd_grid(v.W, nstrip)), block(kBlock);
    const int per_lane = (v.n + 63) / 64;
    if (per_lane <= VEC)
        hipLaunchKernelGGL((k_flush_vec<T, VEC>), grid, block, 0, s, v, spin);
    else if (per_lane <= 4)
        hipLaunchKernelGGL((k_flush_vec<T, 4>), grid, block, 0, s, v, spin);
    else if (per_lane <= 8)
        hipLaunchKernelGGL((k_flush_vec<T, 8>), grid, block, 0, s, v, spin);
    else if (per_lane <= 16)
        hipLaunchKernelGGL((k_flush_vec<T, 16>), grid, block, 0, s, v, spin);
    else
        hipLaunchKernelGGL((k_flush_vec<T, 32>), grid, block, 0, s, v, spin);
}

// One wave per (walker, electron): this electron's contribution to sum_i [...].
// The determinant part streams the electron's inverse row and its gradient and
// Laplacian rows (four iterations of loads in flight per lane).  The Jastrow part
// sums the Pade pair terms over the other electrons: coordinate differences in
// FP64, each term in the precision of the path (FP32 in mixed precision, like
// the ratios), the sums in FP64.
template <typename T>
__device__ __forceinline__ void j2_energy_terms(T a, T b, T L, T iL, const double* re, const double* rm, T& gx,
                                                T& gy, T& gz, T& lap)
{
    T d[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        T x = (T)(re[c] - rm[c]);
        if constexpr (sizeof(T) == 8)
            x -= L * rint(x / L);
        else
            x -= L * rintf(x * iL);
        d[c] = x;
    }
    const T r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    const T iq = (T)1 / ((T)1 + b * r);
    const T du = a * iq * iq, d2u = (T)-2 * a * b * iq * iq * iq;
    const T f = du / r;
    gx = f * d[0];
    gy = f * d[1];
    gz = f * d[2];
    lap = d2u + (T)2 * f;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_energy_rows(CrowdView<T> v)
{
    constexpr int VEC = 16 / sizeof(T);
    constexpr int UNR = 4;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const long long gw = (long long)blockIdx.x * 4 + wave;
    if (gw >= (long long)v.W * v.ne) return;
    const int w = (int)(gw / v.ne), e = (int)(gw % v.ne);
    const int n = v.n, spin = e >= n, a = e - spin * n;
    const T* mrow = v.M + (((size_t)w * 2 + spin) * n + a) * (size_t)n;
    const T* vg = v.VGL + (((size_t)w * 2 + spin) * n + a) * 5 * (size_t)n;
    T s[4] = {(T)0, (T)0, (T)0, (T)0};
    for (int j0 = lane * VEC; j0 < n; j0 += UNR * 64 * VEC) {
        T m[UNR][VEC], x[UNR][4][VEC];
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
            const int j = j0 + u * 64 * VEC;
            if (j < n) {
                load16(mrow + j, m[u]);
#pragma unroll
                for (int k = 0; k < 4; ++k) load16(vg + (size_t)(k + 1) * n + j, x[u][k]);
            } else {
#pragma unroll
                for (int i = 0; i < VEC; ++i) {
                    m[u][i] = (T)0;
#pragma unroll
                    for (int k = 0; k < 4; ++k) x[u][k][i] = (T)0;
                }
            }
        }
#pragma unroll
        for (int u = 0; u < UNR; ++u)
#pragma unroll
            for (int k = 0; k < 4; ++k)
#pragma unroll
                for (int i = 0; i < VEC; ++i) s[k] += x[u][k][i] * m[u][i];
    }
    double g[3], l;
#pragma unroll
    for (int k = 0; k < 3; ++k) g[k] = (double)wave_sum(s[k]);
    l = (double)wave_sum(s[3]);
    double gu[3] = {0.0, 0.0, 0.0}, lu = 0.0;
    if (v.use_j2) {
        const double* Rw = v.R + (size_t)w * v.ne * 3;
        const double re[3] = {Rw[(size_t)e * 3], Rw[(size_t)e * 3 + 1], Rw[(size_t)e * 3 + 2]};
        const T L = (T)v.L, iL = (T)(1.0 / v.L), b = (T)v.b;
        const T a_same = (T)v.a_par, a_other = (T)v.a_anti;
        // the positions of 4 partners per lane are loaded together (one round trip per
        // 256 partners); the terms are summed in the order m = lane, lane + 64, ...
        constexpr int PU = 4;
        for (int m0 = lane; m0 < v.ne; m0 += PU * 64) {
            double rm[PU][3];
#pragma unroll
            for (int u = 0; u < PU; ++u) {
                const int m = m0 + 64 * u, mc = m < v.ne ? m : lane;
#pragma unroll
                for (int c = 0; c < 3; ++c) rm[u][c] = Rw[(size_t)mc * 3 + c];
            }
#pragma unroll
            for (int u = 0; u < PU; ++u) {
                const int m = m0 + 64 * u;
                if (m < v.ne) {
                    const T aa = ((m >= n) == (spin != 0)) ? a_same : a_other;
                    T gx, gy, gz, lp;
                    j2_energy_terms<T>(aa, b, L, iL, re, rm[u], gx, gy, gz, lp);
                    const bool self = m == e;  // the electron's own pair term is not a term
                    gu[0] += self ? 0.0 : (double)gx;
                    gu[1] += self ? 0.0 : (double)gy;
                    gu[2] += self ? 0.0 : (double)gz;
                    lu += self ? 0.0 : (double)lp;
                }
            }
        }
    }
    if (v.n_ions) {  // one-body terms of the electron, the centres over the lanes
        const double* re = v.R + ((size_t)w * v.ne + e) * 3;
        const double r3[3] = {re[0], re[1], re[2]};
        (void)j1_at(v, r3, lane, 64, gu, lu);
    }
    if (v.use_j2 || v.n_ions) {
#pragma unroll
        for (int k = 0; k < 3; ++k) gu[k] = wave_sum(gu[k]);
        lu = wave_sum(lu);
    }
    if (lane == 0)
        v.elpart[gw] = l + lu + gu[0] * gu[0] + gu[1] * gu[1] + gu[2] * gu[2]
                       + 2.0 * (g[0] * gu[0] + g[1] * gu[1] + g[2] * gu[2]);
}

// Fixed-order FP64 sum over electrons: one wave per walker.
__global__ __launch_bounds__(kBlock) void k_energy_sum(const double* __restrict__ elpart, double* __restrict__ eloc,
                                                       int W, int ne)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int w = blockIdx.x * 4 + wave;
    if (w >= W) return;
    double s = 0.0;
    for (int e = lane; e < ne; e += 64) s += elpart[(size_t)w * ne + e];
    s = wave_sum(s);
    if (lane == 0) eloc[w] = -0.5 * s;
}

template <typename T>
void launch_energy(const CrowdView<T>& v, hipStream_t s)
{
    const long long waves = (long long)v.W * v.ne;
    hipLaunchKernelGGL(k_energy_rows<T>, dim3((unsigned)((waves + 3) / 4)), dim3(kBlock), 0, s, v);
    hipLaunchKernelGGL(k_energy_sum, dim3((v.W + 3) / 4), dim3(kBlock), 0, s, v.elpart, v.eloc, v.W, v.ne);
}

template void launch_flush<float>(const CrowdView<float>&, int, hipStream_t, bool);
template void launch_flush_vec_multi<float>(const CrowdView<float>*, const int4*, int, int, int, int, hipStream_t);
template void launch_flush_vec_multi<double>(const CrowdView<double>*, const int4*, int, int, int, int, hipStream_t);
template void launch_flush<double>(const CrowdView<double>&, int, hipStream_t, bool);
template void launch_energy<float>(const CrowdView<float>&, hipStream_t);
template void launch_energy<double>(const CrowdView<double>&, hipStream_t);

}  // namespace cq
