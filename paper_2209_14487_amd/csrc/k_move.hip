// Per-move kernels of the batched particle-by-particle move (paper Alg. 1
// L5-L9 applied to every walker of a crowd in lock-step, Alg. 3/4):
//
//   k_vgl_move   L5 propose + L7/L8 B-spline value/gradient/Laplacian at r' for
//                one orbital chunk, the chunk's partial dot products with the
//                inverse column and the delayed-update window, and a slice of
//                the Jastrow difference / gradient.  Grid: walkers x chunks.
//   k_resolve    L7 ratio (column corrected for the window's accepted moves),
//                L9 Metropolis decision, window bookkeeping.  One wave per walker.
//   k_finalize   brings the inverse column of the window's last accepted move up
//                to date before the window is applied to the inverse.
//
// Orbital tables are [G][G][G][n_orb] with the orbital index fastest, so the 64
// stencil points of one walker are 64 contiguous runs of n_orb elements (16
// runs of 4 consecutive z-points): each lane loads 16 bytes per point,
// coalesced along orbitals.  Four waves split the 4 x-planes of the stencil;
// their partial sums meet in LDS in a fixed order (bit-reproducible results,
// independent of how walkers are grouped into crowds).
#include "cq_device.h"
#include "cq_internal.h"

namespace cq {

template <typename T>
__global__ void k_fill_philox(T* __restrict__ table, uint64_t seed, size_t count)
{
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) {
        uint32_t o[4];
        philox_block(seed, (uint32_t)i, (uint32_t)(i >> 32), 0xC0EFu, 0u, o);
        const double c = 2.0 * uniform53(o[0], o[1]) - 1.0;
        table[i] = (T)c;
    }
}

template <typename T>
void launch_fill_philox(T* table, uint64_t seed, size_t count, hipStream_t s)
{
    const int blocks = 4096;
    hipLaunchKernelGGL(k_fill_philox<T>, dim3(blocks), dim3(kBlock), 0, s, table, seed, count);
}

// x-plane weight (value, first, second derivative) of stencil plane a = 0..3.
template <typename T>
__device__ __forceinline__ void pick_plane(const AxisW<T>& ax, int a, T& b, T& d1, T& d2)
{
    b = ax.b[0]; d1 = ax.d1[0]; d2 = ax.d2[0];
    if (a == 1) { b = ax.b[1]; d1 = ax.d1[1]; d2 = ax.d2[1]; }
    if (a == 2) { b = ax.b[2]; d1 = ax.d1[2]; d2 = ax.d2[2]; }
    if (a == 3) { b = ax.b[3]; d1 = ax.d1[3]; d2 = ax.d2[3]; }
}

// Value, gradient and Laplacian of orbitals [c*CH, c*CH + CH) at r, left in
// row[5][CH] (LDS).  All 256 threads of the block must call it.
template <typename T>
__device__ __forceinline__ void spline_chunk(const T* __restrict__ table, int G, int n_orb, int n, double L,
                                             const double r[3], int c, T* red /*[4][5][CH]*/,
                                             T* row /*[5][CH]*/)
{
    constexpr int VEC = 16 / sizeof(T);
    constexpr int CH = 64 * VEC;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const AxisW<T> ax = axis_weights<T>(r[0], L, G);
    const AxisW<T> ay = axis_weights<T>(r[1], L, G);
    const AxisW<T> az = axis_weights<T>(r[2], L, G);
    T bxa, dxa, d2xa;
    pick_plane(ax, wave, bxa, dxa, d2xa);
    const int j0 = c * CH + lane * VEC;
    T acc[5][VEC];
#pragma unroll
    for (int k = 0; k < 5; ++k)
#pragma unroll
        for (int i = 0; i < VEC; ++i) acc[k][i] = (T)0;
    if (j0 < n) {
        const int jx = (ax.i0 + wave + G - 1) % G;
        int jy[4], jz[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            jy[q] = (ay.i0 + q + G - 1) % G;
            jz[q] = (az.i0 + q + G - 1) % G;
        }
        T vals[16][VEC];
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const size_t pt = ((size_t)jx * G + jy[q >> 2]) * G + jz[q & 3];
            load16(table + pt * n_orb + j0, vals[q]);
        }
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int bb = q >> 2, cc = q & 3;
            const T yz = ay.b[bb] * az.b[cc];
            const T wv = bxa * yz;
            const T wgx = dxa * yz;
            const T wgy = bxa * ay.d1[bb] * az.b[cc];
            const T wgz = bxa * ay.b[bb] * az.d1[cc];
            const T wl = d2xa * yz + bxa * (ay.d2[bb] * az.b[cc] + ay.b[bb] * az.d2[cc]);
#pragma unroll
            for (int i = 0; i < VEC; ++i) {
                const T p = vals[q][i];
                acc[0][i] += wv * p;
                acc[1][i] += wgx * p;
                acc[2][i] += wgy * p;
                acc[3][i] += wgz * p;
                acc[4][i] += wl * p;
            }
        }
    }
#pragma unroll
    for (int k = 0; k < 5; ++k)
#pragma unroll
        for (int i = 0; i < VEC; ++i) red[(wave * 5 + k) * CH + lane * VEC + i] = acc[k][i];
    __syncthreads();
    if (threadIdx.x < CH) {
        const int t = threadIdx.x;
#pragma unroll
        for (int k = 0; k < 5; ++k)
            row[k * CH + t] = ((red[(0 * 5 + k) * CH + t] + red[(1 * 5 + k) * CH + t]) + red[(2 * 5 + k) * CH + t])
                              + red[(3 * 5 + k) * CH + t];
    }
    __syncthreads();
}

// Orbital rows of every electron at its current position (setup).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_setup_vgl(CrowdView<T> v)
{
    constexpr int VEC = 16 / sizeof(T);
    constexpr int CH = 64 * VEC;
    __shared__ T red[4 * 5 * CH];
    __shared__ T row[5 * CH];
    const int C = (v.n + CH - 1) / CH;
    int w, part;
    xcd_map(blockIdx.x, v.ne * C, w, part);
    if (w >= v.W) return;
    const int e = part / C, c = part % C;
    const int spin = e >= v.n, a = e - spin * v.n;
    double r[3];
    for (int k = 0; k < 3; ++k) r[k] = v.R[((size_t)w * v.ne + e) * 3 + k];
    spline_chunk<T>(v.table, v.G, v.n_orb, v.n, v.L, r, c, red, row);
    const int t = threadIdx.x;
    const int j = c * CH + t;
    if (t < CH && j < v.n) {
        T* dst = v.VGL + (((size_t)w * 2 + spin) * v.n + a) * 5 * (size_t)v.n;
        for (int k = 0; k < 5; ++k) dst[(size_t)k * v.n + j] = row[k * CH + t];
    }
}

template <typename T>
void launch_setup_vgl(const CrowdView<T>& v, hipStream_t s)
{
    constexpr int CH = chunk_orbitals<T>();
    const int C = (v.n + CH - 1) / CH;
    hipLaunchKernelGGL(k_setup_vgl<T>, dim3(xcd_grid(v.W, v.ne * C)), dim3(kBlock), 0, s, v);
}

// One move of electron e for every walker: propose, orbital chunk VGL, partial
// dots, Jastrow slice.  reset = 1 starts a new update window.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_vgl_move(CrowdView<T> v, int e, int reset)
{
    constexpr int VEC = 16 / sizeof(T);
    constexpr int CH = 64 * VEC;
    __shared__ T red[4 * 5 * CH];
    __shared__ T row[5 * CH];
    __shared__ double jred[4][4];
    const int C = (v.n + CH - 1) / CH;
    int w, c;
    xcd_map(blockIdx.x, C, w, c);
    if (w >= v.W) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int n = v.n, K = v.K, NP = part_stride(K);
    const int spin = e >= n, a = e - spin * n;
    const int cnt = reset ? 0 : v.cnt[w];
    const int pend = reset ? -1 : v.pend[w];
    const uint32_t step = v.prm->step;

    // L5: propose r' = wrap(r_e + sigma z)
    double re[3], rp[3], z[3];
    for (int k = 0; k < 3; ++k) re[k] = v.R[((size_t)w * v.ne + e) * 3 + k];
    gauss3(v.seed, v.uid[w], step, (uint32_t)e, z);
    const double sigma = v.prm->sigma;
    for (int k = 0; k < 3; ++k) rp[k] = wrap_box(re[k] + sigma * z[k], v.L);
    if (c == 0 && tid < 3) v.rnew[(size_t)w * 3 + tid] = rp[tid];

    // L7-L8: orbital values, gradients, Laplacians of this chunk at r'
    spline_chunk<T>(v.table, v.G, v.n_orb, n, v.L, rp, c, red, row);

    const int j0 = c * CH + lane * VEC;
    const bool valid = j0 < n;
    double* P = v.part + ((size_t)w * C + c) * NP;
    T m[VEC], rv[5][VEC];
#pragma unroll
    for (int i = 0; i < VEC; ++i) m[i] = (T)0;
    if (valid) load16(v.M + (((size_t)w * 2 + spin) * n + a) * (size_t)n + j0, m);
#pragma unroll
    for (int k = 0; k < 5; ++k)
#pragma unroll
        for (int i = 0; i < VEC; ++i) rv[k][i] = row[k * CH + lane * VEC + i];
    if (valid) {
        // pending window slot: the proposal's orbital rows and the old inverse column c0_e
        if (wave == 0) store16(v.Cbuf + ((size_t)w * K + cnt) * n + j0, m);
        for (int k = wave; k < 5; k += 4) store16(v.stage + (((size_t)w * K + cnt) * 5 + k) * n + j0, rv[k]);
    }
    // dot products of the ratio: products in T, sums in FP64
    if (wave == 0) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            double s = 0.0;
#pragma unroll
            for (int i = 0; i < VEC; ++i) s += (double)(rv[k][i] * m[i]);
            s = wave_sum(s);
            if (lane == 0) P[k] = s;
        }
    }
    for (int nn = wave; nn < cnt; nn += 4) {
        T cn[VEC], un[VEC];
#pragma unroll
        for (int i = 0; i < VEC; ++i) { cn[i] = (T)0; un[i] = (T)0; }
        if (valid) {
            load16(v.Cbuf + ((size_t)w * K + nn) * n + j0, cn);
            load16(v.stage + (((size_t)w * K + nn) * 5 + 0) * n + j0, un);
            if (nn == pend) {
                // the previous move was accepted: its column still holds c0; apply the
                // window's earlier moves, c = c0 - sum_m beta_m c_m (this chunk only)
                for (int mm = 0; mm < pend; ++mm) {
                    T cm[VEC];
                    load16(v.Cbuf + ((size_t)w * K + mm) * n + j0, cm);
                    const T bm = (T)v.beta[(size_t)w * K + mm];
#pragma unroll
                    for (int i = 0; i < VEC; ++i) cn[i] -= bm * cm[i];
                }
                store16(v.Cbuf + ((size_t)w * K + nn) * n + j0, cn);
            }
        }
        double s[5];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            s[k] = 0.0;
#pragma unroll
            for (int i = 0; i < VEC; ++i) s[k] += (double)(rv[k][i] * cn[i]);
        }
        s[4] = 0.0;
#pragma unroll
        for (int i = 0; i < VEC; ++i) s[4] += (double)(m[i] * un[i]);
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            const double t = wave_sum(s[k]);
            if (lane == 0) P[4 + 5 * nn + k] = t;
        }
    }

    // Jastrow: this workgroup's slice of the other electrons
    double jv[4] = {0.0, 0.0, 0.0, 0.0};
    if (v.use_j2) {
        const int per = (v.ne + C - 1) / C;
        const int lo = c * per, hi = min(v.ne, lo + per);
        for (int mm = lo + tid; mm < hi; mm += kBlock) {
            if (mm == e) continue;
            const double* rm = v.R + ((size_t)w * v.ne + mm) * 3;
            const double aa = ((mm >= n) == (spin != 0)) ? v.a_par : v.a_anti;
            double d1[3], d0[3], u1, du1, dd1, u0, du0, dd0;
            min_image(rp, rm, v.L, d1);
            min_image(re, rm, v.L, d0);
            const double r1 = sqrt(d1[0] * d1[0] + d1[1] * d1[1] + d1[2] * d1[2]);
            const double r0 = sqrt(d0[0] * d0[0] + d0[1] * d0[1] + d0[2] * d0[2]);
            pade(aa, v.b, r1, u1, du1, dd1);
            pade(aa, v.b, r0, u0, du0, dd0);
            jv[0] += u1 - u0;
            const double f = du1 / r1;
            jv[1] += f * d1[0];
            jv[2] += f * d1[1];
            jv[3] += f * d1[2];
        }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) jv[k] = wave_sum(jv[k]);
    if (lane == 0)
        for (int k = 0; k < 4; ++k) jred[wave][k] = jv[k];
    __syncthreads();
    if (tid < 4) P[part_j2(K) + tid] = ((jred[0][tid] + jred[1][tid]) + jred[2][tid]) + jred[3][tid];
}

template <typename T>
void launch_vgl_move(const CrowdView<T>& v, int e, int reset, hipStream_t s)
{
    constexpr int CH = chunk_orbitals<T>();
    const int C = (v.n + CH - 1) / CH;
    hipLaunchKernelGGL(k_vgl_move<T>, dim3(xcd_grid(v.W, C)), dim3(kBlock), 0, s, v, e, reset);
}

// Ratio, decision and window bookkeeping of the move of electron e; one wave
// per walker.  The window's accepted moves m = 0 .. cnt-1 (rows u_m, columns
// c_m taken just before move m, ratios rho_m) act on the old column c0_e of e
// as a sequence of rank-1 updates:
//   c_e = c0_e - sum_m beta_m c_m,  beta_m = (u_m . c0_e - sum_{j<m} beta_j u_m . c_j) / rho_m
// (forward substitution with wG[m][j] = u_m . c_j), so
//   rho_D = u . c0_e - sum_m beta_m (u . c_m)
// and grad ln D(r') follows the same way from grad u.  This applies the window's
// updates in order, as Sherman-Morrison would, and is as accurate; it avoids the
// explicit inverse of the k x k window matrix, whose conditioning degrades when a
// small ratio enters the window.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_resolve(CrowdView<T> v, int e, int reset)
{
    __shared__ double vals[4][part_stride(kMaxDelay)];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int w = blockIdx.x * 4 + wave;
    const bool active = w < v.W;
    constexpr int CH = chunk_orbitals<T>();
    const int n = v.n, K = v.K, NP = part_stride(K), J2 = part_j2(K);
    const int C = (n + CH - 1) / CH;
    const int spin = e >= n, a = e - spin * n;
    const int cnt = active ? (reset ? 0 : v.cnt[w]) : 0;
    if (active) {
        for (int i = lane; i < NP; i += 64) {
            double s = 0.0;
            if (i < 4 + 5 * cnt || i >= J2)
                for (int c = 0; c < C; ++c) s += v.part[((size_t)w * C + c) * NP + i];
            vals[wave][i] = s;
        }
    }
    __syncthreads();
    if (!active) return;  // no block-wide barrier below this point
    const double* V = vals[wave];
    const double* wG = v.wG + (size_t)w * K * K;
    const double* wrho = v.wrho + (size_t)w * K;
    // forward substitution: lane i carries t_i = y_i - sum_{j<m} beta_j wG[i][j]
    // and keeps beta_i once its turn comes
    double t = lane < cnt ? V[4 + 5 * lane + 4] : 0.0;
    double my_beta = 0.0;
    for (int mm = 0; mm < cnt; ++mm) {
        const double bm = __shfl(t, mm, 64) / wrho[mm];
        if (lane == mm) my_beta = bm;
        if (lane > mm && lane < cnt) t -= bm * wG[lane * K + mm];
    }
    double r[4] = {0.0, 0.0, 0.0, 0.0};
    if (lane < cnt) {
#pragma unroll
        for (int k = 0; k < 4; ++k) r[k] = my_beta * V[4 + 5 * lane + k];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) r[k] = wave_sum(r[k]);
    const double rho = V[0] - r[0];
    double gd[3] = {(V[1] - r[1]) / rho, (V[2] - r[2]) / rho, (V[3] - r[3]) / rho};
    (void)gd;
    const double dlnj = V[J2];
    const double prob = rho * rho * exp(2.0 * dlnj);
    const uint32_t step = v.prm->step;
    const double u = accept_uniform(v.seed, v.uid[w], step, (uint32_t)e);
    int acc = u < prob;
    const int rs = v.prm->rec_sweep;
    const size_t ri = ((size_t)rs * v.ne + e) * v.W + w;
    if (v.forced && rs < v.prm->forced_cap) acc = v.forced[ri] != 0;
    if (lane == 0 && rs < v.prm->rec_cap) {
        v.rec_rho[ri] = rho;
        v.rec_dlnj[ri] = dlnj;
        v.rec_prob[ri] = prob;
        v.rec_acc[ri] = (uint8_t)acc;
    }
    if (acc) {
        if (lane < cnt) {
            v.beta[(size_t)w * K + lane] = my_beta;
            v.wG[((size_t)w * K + cnt) * K + lane] = V[4 + 5 * lane];  // u . c_lane
        }
        if (lane == 0) {
            v.wrho[(size_t)w * K + cnt] = rho;
            v.welec[(size_t)w * K + cnt] = a;
            v.cnt[w] = cnt + 1;
            v.pend[w] = cnt;
            for (int k = 0; k < 3; ++k) v.R[((size_t)w * v.ne + e) * 3 + k] = v.rnew[(size_t)w * 3 + k];
            v.logdet[w * 2 + spin] += log(fabs(rho));
            if (rho < 0.0) v.sign[w * 2 + spin] = -v.sign[w * 2 + spin];
            v.nacc[w] += 1;
        }
    } else if (lane == 0) {
        v.cnt[w] = cnt;
        v.pend[w] = -1;
    }
    if (lane == 0) v.nprop[w] += 1;
}

// End of a window: bring the last accepted move's column up to date (one chunk
// of orbitals per workgroup), so that the update sees every c_m.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_finalize(CrowdView<T> v)
{
    constexpr int VEC = 16 / sizeof(T);
    constexpr int CH = 64 * VEC;
    const int C = (v.n + CH - 1) / CH;
    int w, c;
    xcd_map(blockIdx.x, C, w, c);
    if (w >= v.W) return;
    const int p = v.pend[w];
    if (p <= 0) return;  // nothing pending, or the first move of the window (c = c0)
    const int K = v.K, n = v.n;
    const int j0 = c * CH + threadIdx.x * VEC;
    if (threadIdx.x >= 64 || j0 >= n) return;
    T cn[VEC];
    load16(v.Cbuf + ((size_t)w * K + p) * n + j0, cn);
    for (int mm = 0; mm < p; ++mm) {
        T cm[VEC];
        load16(v.Cbuf + ((size_t)w * K + mm) * n + j0, cm);
        const T bm = (T)v.beta[(size_t)w * K + mm];
#pragma unroll
        for (int i = 0; i < VEC; ++i) cn[i] -= bm * cm[i];
    }
    store16(v.Cbuf + ((size_t)w * K + p) * n + j0, cn);
}

template <typename T>
void launch_finalize(const CrowdView<T>& v, hipStream_t s)
{
    constexpr int CH = chunk_orbitals<T>();
    const int C = (v.n + CH - 1) / CH;
    hipLaunchKernelGGL(k_finalize<T>, dim3(xcd_grid(v.W, C)), dim3(64), 0, s, v);
}

template <typename T>
void launch_resolve(const CrowdView<T>& v, int e, int reset, hipStream_t s)
{
    hipLaunchKernelGGL(k_resolve<T>, dim3((v.W + 3) / 4), dim3(kBlock), 0, s, v, e, reset);
}

__global__ void k_sweep_end(Params* prm)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        prm->step += 1;
        prm->rec_sweep += 1;
    }
}

void launch_sweep_end(Params* prm, hipStream_t s)
{
    hipLaunchKernelGGL(k_sweep_end, dim3(1), dim3(64), 0, s, prm);
}

// Grid-stride 16-byte copy (reference kernel for traffic-counter calibration).
__global__ __launch_bounds__(kBlock) void k_copy16(float4* __restrict__ dst, const float4* __restrict__ src,
                                                   size_t n16)
{
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride) dst[i] = src[i];
}

void launch_copy(void* dst, const void* src, size_t bytes, hipStream_t s)
{
    hipLaunchKernelGGL(k_copy16, dim3(4096), dim3(kBlock), 0, s, (float4*)dst, (const float4*)src, bytes / 16);
}

template void launch_fill_philox<float>(float*, uint64_t, size_t, hipStream_t);
template void launch_fill_philox<double>(double*, uint64_t, size_t, hipStream_t);
template void launch_setup_vgl<float>(const CrowdView<float>&, hipStream_t);
template void launch_setup_vgl<double>(const CrowdView<double>&, hipStream_t);
template void launch_vgl_move<float>(const CrowdView<float>&, int, int, hipStream_t);
template void launch_vgl_move<double>(const CrowdView<double>&, int, int, hipStream_t);
template void launch_resolve<float>(const CrowdView<float>&, int, int, hipStream_t);
template void launch_resolve<double>(const CrowdView<double>&, int, int, hipStream_t);
template void launch_finalize<float>(const CrowdView<float>&, hipStream_t);
template void launch_finalize<double>(const CrowdView<double>&, hipStream_t);

}  // namespace cq
