// The tail of a spin block of the batched path.  A spin block of N electrons needs
// at most N / k rounds (every round advances a walker by at least k electrons), but
// at the usual acceptance about a third of them: the rest would find every walker
// done.  So the sweep runs only the rounds that recent sweeps needed, plus a margin,
// and then this kernel finishes any walker that still has electrons left, one
// workgroup per walker and one move at a time (the propose, ratio and accept steps
// of Alg. 1 with a Sherman-Morrison update of the walker's inverse in place).  It
// computes the same chain as the rounds would have (same proposals and uniforms,
// decisions to rounding), so the plan affects the speed only.  A walker without
// electrons left returns at once.
//
// Per move e of electron a (M[b] = A^-1 e_b, the walker's inverse after the last
// round's update):
//   u = phi(r'), grad, Laplacian at r' = wrap(r_e + sigma z)
//   rho = u . M[a] (exact products, FP64 sum), dlnJ (pairs and one-body terms)
//   accept if u_e < rho^2 exp(2 dlnJ); then M[b] -= ((u . M[b]) - delta_ab) / rho M_old[a]
//   (FP64 from the stored values, stored in T), rows into the walker's VGL matrix.
// k_plan_report then hands the host the number of rounds the block's walkers had
// candidates in, and whether this kernel had work, in pinned host memory.
#include "cq_device.h"
#include "cq_internal.h"
#include "cq_jastrow.h"
#include "cq_stencil.h"

namespace cq {

namespace {

__device__ __forceinline__ double lo_block_sum(double x, double* red, int lane, int wave)
{
    x = wave_sum(x);
    __syncthreads();
    if (lane == 0) red[wave] = x;
    __syncthreads();
    return ((red[0] + red[1]) + red[2]) + red[3];
}

}  // namespace

template <typename T>
__global__ __launch_bounds__(kBlock) void k_leftover(CrowdView<T> v, int spin)
{
    constexpr int VEC = 16 / sizeof(T);
    extern __shared__ unsigned char lo_lds[];  // u rows [5][N] in T, then c0 [N] in FP64
    __shared__ size_t s_idx[64];
    __shared__ T s_w[64 * 5];
    __shared__ double s_red[kBlock / 64];
    __shared__ double s_rp[3];
    const int w = blockIdx.x;
    if (w >= v.W) return;
    const int n = v.n, ne = v.ne, groups = n / VEC;
    const int dec = v.cur[2 * w];
    if (dec >= n) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    T* u = reinterpret_cast<T*>(lo_lds);
    double* c0 = reinterpret_cast<double*>(u + (size_t)5 * n);
    if (tid == 0) v.left[spin] = 1;
    T* M = v.M + ((size_t)w * 2 + spin) * n * (size_t)n;
    double* Rw = v.R + (size_t)w * ne * 3;
    const uint32_t step = v.prm->step, uid = v.uid[w];
    const int rs = v.prm->rec_sweep;
    const double sigma = v.prm->sigma;
    for (int a = dec; a < n; ++a) {
        const int e = spin * n + a;
        __syncthreads();  // the previous move's readers of the stencil, rows and c0 are done
        if (wave == 0) {
            double z[3], rp[3];
            gauss3(v.seed, uid, step, (uint32_t)e, z);
#pragma unroll
            for (int k = 0; k < 3; ++k) rp[k] = wrap_box(Rw[(size_t)e * 3 + k] + sigma * z[k], v.L);
            stencil_entry<T>(v, rp, lane, s_idx, s_w);
            if (lane < 3) s_rp[lane] = rp[lane];
        }
        __syncthreads();
        const double rp[3] = {s_rp[0], s_rp[1], s_rp[2]};
        const double re[3] = {Rw[(size_t)e * 3], Rw[(size_t)e * 3 + 1], Rw[(size_t)e * 3 + 2]};
        // value, gradient, Laplacian rows at r' (one orbital group of 16 bytes per thread and pass)
        for (int g = tid; g < groups; g += kBlock) {
            const int j0 = g * VEC;
            T acc[5][VEC];
#pragma unroll
            for (int k = 0; k < 5; ++k)
#pragma unroll
                for (int i = 0; i < VEC; ++i) acc[k][i] = (T)0;
#pragma unroll 1
            for (int x = 0; x < 4; ++x) {
                T vals[16][VEC];
#pragma unroll
                for (int q = 0; q < 16; ++q) load16(v.table + s_idx[x * 16 + q] + j0, vals[q]);
#pragma unroll
                for (int q = 0; q < 16; ++q) {
                    const T* wq = s_w + (x * 16 + q) * 5;
#pragma unroll
                    for (int k = 0; k < 5; ++k)
#pragma unroll
                        for (int i = 0; i < VEC; ++i) acc[k][i] += wq[k] * vals[q][i];
                }
            }
#pragma unroll
            for (int k = 0; k < 5; ++k)
#pragma unroll
                for (int i = 0; i < VEC; ++i) u[(size_t)k * n + j0 + i] = acc[k][i];
        }
        __syncthreads();
        // ratio and Jastrow difference
        double rho = 0.0, dj = 0.0;
        for (int j = tid; j < n; j += kBlock) rho += (double)u[j] * (double)M[(size_t)a * n + j];
        if (v.use_j2)
            for (int m = tid; m < ne; m += kBlock) {
                if (m == e) continue;
                const double aa = ((m >= n) == (spin != 0)) ? v.a_par : v.a_anti;
                double d1[3], d0[3], u1, u0, du, d2u;
                min_image(rp, Rw + (size_t)m * 3, v.L, d1);
                min_image(re, Rw + (size_t)m * 3, v.L, d0);
                pade(aa, v.b, sqrt(d1[0] * d1[0] + d1[1] * d1[1] + d1[2] * d1[2]), u1, du, d2u);
                pade(aa, v.b, sqrt(d0[0] * d0[0] + d0[1] * d0[1] + d0[2] * d0[2]), u0, du, d2u);
                dj += u1 - u0;
            }
        if (v.n_ions) dj += j1_delta(v, rp, re, tid, kBlock);
        rho = lo_block_sum(rho, s_red, lane, wave);
        dj = lo_block_sum(dj, s_red, lane, wave);
        const double prob = rho * rho * exp(2.0 * dj);
        int acc = accept_uniform(v.seed, uid, step, (uint32_t)e) < prob;
        const size_t ri = ((size_t)rs * ne + e) * v.Wcap + w;
        if (v.forced && rs < v.prm->forced_cap && v.forced[ri] < 2) acc = v.forced[ri] != 0;
        if (tid == 0) {
            if (rs < v.prm->rec_cap) {
                v.rec_rho[ri] = rho;
                v.rec_dlnj[ri] = dj;
                v.rec_prob[ri] = prob;
                v.rec_acc[ri] = (uint8_t)acc;
            }
            v.nprop[w] += 1;
        }
        if (!acc) continue;
        for (int j = tid; j < n; j += kBlock) c0[j] = (double)M[(size_t)a * n + j];
        __syncthreads();  // every thread sees the old column before any row changes
        // Sherman-Morrison, one row per wave pass
        const double irho = 1.0 / rho;
        for (int b = wave; b < n; b += kBlock / 64) {
            T* Mb = M + (size_t)b * n;
            double x = 0.0;
            for (int j = lane; j < n; j += 64) x += (double)u[j] * (double)Mb[j];
            x = wave_sum(x);
            const double beta = (x - (b == a ? 1.0 : 0.0)) * irho;
            for (int j = lane; j < n; j += 64) Mb[j] = (T)((double)Mb[j] - beta * c0[j]);
        }
        T* dst = v.VGL + (((size_t)w * 2 + spin) * n + a) * 5 * (size_t)n;
        for (int i = tid; i < 5 * n; i += kBlock) dst[i] = u[i];
        if (tid == 0) {
            v.logdet[w * 2 + spin] += log(fabs(rho));
            if (rho < 0.0) v.sign[w * 2 + spin] = -v.sign[w * 2 + spin];
            v.nacc[w] += 1;
        }
        if (tid < 3) Rw[(size_t)e * 3 + tid] = rp[tid];
        // the next move's readers of R and M come after the barrier at the top of the loop
    }
    if (tid == 0) v.cur[2 * w] = n;
}

// The block's plan record for the host (pinned memory): out[1 + 2 spin] = rounds in which
// some walker had candidates, out[2 + 2 spin] = whether k_leftover had work; bit `spin` of
// out[0] is set once that spin's record has been written (the host clears out[0] when the
// plan restarts, so a spin's fields are read only after a record of its own).
__global__ void k_plan_report(const int* used, const int* left, int spin, int* out)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        out[1 + 2 * spin] = used[spin];
        out[2 + 2 * spin] = left[spin];
        __threadfence_system();
        out[0] = out[0] | (1 << spin);
    }
}

template <typename T>
void launch_leftover(const CrowdView<T>& v, int spin, int* host_report, bool run, hipStream_t s)
{
    if (run) {
        const size_t lds = sizeof(T) * 5 * (size_t)v.n + sizeof(double) * (size_t)v.n;
        static size_t opted = 64 * 1024;  // dynamic LDS opted in to (per type)
        if (lds > opted) {
            (void)hipFuncSetAttribute((const void*)k_leftover<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                      (int)lds);
            opted = lds;
        }
        hipLaunchKernelGGL(k_leftover<T>, dim3(v.W), dim3(kBlock), lds, s, v, spin);
    }
    if (host_report) hipLaunchKernelGGL(k_plan_report, dim3(1), dim3(64), 0, s, v.used, v.left, spin, host_report);
}

template void launch_leftover<float>(const CrowdView<float>&, int, int*, bool, hipStream_t);
template void launch_leftover<double>(const CrowdView<double>&, int, int*, bool, hipStream_t);

}  // namespace cq
