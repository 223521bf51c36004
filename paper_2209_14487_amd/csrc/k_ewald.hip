// Electron-electron Coulomb energy of every walker (the potential part of the
// local energy of Alg. 1), for the periodic box with a uniform neutralising
// background, by Ewald summation (charges -1, Omega = L^3, N = Ne):
//   V = sum_{i<j} erfc(alpha r_ij) / r_ij                       (minimum image)
//     + (4 pi / Omega) sum_{k in half space} exp(-k^2/4alpha^2)/k^2 |rho_k|^2
//     - alpha N / sqrt(pi) - pi N^2 / (2 alpha^2 Omega),
// rho_k = sum_i exp(i k . r_i), k = 2 pi n / L, |n| <= nmax.  alpha L = 10.1 puts
// every image beyond the nearest below 1e-12 of its pair's term (erfc(5.05)), and
// the k shells stop where exp(-k^2/4alpha^2) falls below 1e-13 (n^2 <= 18^2).
// FP64 throughout, whatever the precision of the crowd.
//   k_ewald_phase   exp(i 2 pi m x / L) for m = 0 .. nmax and each axis of each
//                   electron (negative m are the conjugates);
//   k_ewald_recip   W x P blocks: each thread sums rho_k for 4 wavevectors over
//                   all electrons, tiles of 32 electrons' phase tables in LDS,
//                   rho_k = e_x e_y e_z (two complex products per electron);
//   k_ewald_real    W x P blocks over the pairs (i < j), one row i per thread pass;
//   k_ewald_finish  the parts of each walker in a fixed order, added to E_L.
#include "cq_device.h"
#include "cq_internal.h"

namespace cq {

namespace {

constexpr int kTile = 32;   // electrons per LDS tile of phase tables
constexpr int kKPT = 4;     // wavevectors per thread

__device__ __forceinline__ double ewald_block_sum(double x, double* red)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    x = wave_sum(x);
    if (lane == 0) red[wave] = x;
    __syncthreads();
    double s = 0.0;
    for (int q = 0; q < nw; ++q) s += red[q];
    return s;
}

}  // namespace

__global__ __launch_bounds__(kBlock) void k_ewald_phase(EwaldView e)
{
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (size_t)e.W * e.ne) return;
    const int m1 = e.nmax + 1;
    const double* r = e.R + 3 * t;
    double2* out = e.phase + t * 3 * m1;
    for (int ax = 0; ax < 3; ++ax) {
        const double th = 2.0 * kPi * r[ax] / e.L;
        for (int m = 0; m < m1; ++m) {
            double sn, cs;
            sincos(th * m, &sn, &cs);
            out[ax * m1 + m] = make_double2(cs, sn);
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_ewald_recip(EwaldView e)
{
    extern __shared__ double2 tab[];  // [kTile][3][nmax + 1]
    __shared__ double red[kBlock / 64];
    const int w = blockIdx.x / e.pk, p = blockIdx.x % e.pk;
    if (w >= e.W) return;
    const int m1 = e.nmax + 1, tid = threadIdx.x;
    int kx[kKPT], ky[kKPT], kz[kKPT];
    double re[kKPT], im[kKPT], f[kKPT];
#pragma unroll
    for (int q = 0; q < kKPT; ++q) {
        const int k = (p * kKPT + q) * kBlock + tid;
        const bool live = k < e.nk;
        const int4 v = live ? e.kvec[k] : make_int4(0, 0, 0, 0);
        kx[q] = v.x;
        ky[q] = v.y;
        kz[q] = v.z;
        f[q] = live ? e.kfac[k] : 0.0;
        re[q] = 0.0;
        im[q] = 0.0;
    }
    const double2* src = e.phase + (size_t)w * e.ne * 3 * m1;
    for (int i0 = 0; i0 < e.ne; i0 += kTile) {
        const int cnt = min(kTile, e.ne - i0);
        __syncthreads();
        for (int idx = tid; idx < cnt * 3 * m1; idx += kBlock) tab[idx] = src[(size_t)i0 * 3 * m1 + idx];
        __syncthreads();
        for (int i = 0; i < cnt; ++i) {
            const double2* ti = tab + i * 3 * m1;
#pragma unroll
            for (int q = 0; q < kKPT; ++q) {
                double2 a = ti[abs(kx[q])], b = ti[m1 + abs(ky[q])], c = ti[2 * m1 + abs(kz[q])];
                if (kx[q] < 0) a.y = -a.y;
                if (ky[q] < 0) b.y = -b.y;
                if (kz[q] < 0) c.y = -c.y;
                const double abr = a.x * b.x - a.y * b.y, abi = a.x * b.y + a.y * b.x;
                re[q] += abr * c.x - abi * c.y;
                im[q] += abr * c.y + abi * c.x;
            }
        }
    }
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < kKPT; ++q) s += f[q] * (re[q] * re[q] + im[q] * im[q]);
    s = ewald_block_sum(s, red);
    if (tid == 0) e.part[(size_t)w * (e.pk + e.pr) + p] = s;
}

__global__ __launch_bounds__(kBlock) void k_ewald_real(EwaldView e)
{
    __shared__ double red[kBlock / 64];
    const int w = blockIdx.x / e.pr, p = blockIdx.x % e.pr;
    if (w >= e.W) return;
    const double* R = e.R + (size_t)w * e.ne * 3;
    const double L = e.L, a = e.alpha;
    double s = 0.0;
    for (int i = p; i < e.ne; i += e.pr) {
        const double xi = R[3 * i], yi = R[3 * i + 1], zi = R[3 * i + 2];
        for (int j = i + 1 + threadIdx.x; j < e.ne; j += kBlock) {
            double d[3] = {xi - R[3 * j], yi - R[3 * j + 1], zi - R[3 * j + 2]};
#pragma unroll
            for (int c = 0; c < 3; ++c) d[c] -= L * rint(d[c] / L);
            const double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
            s += erfc(a * r) / r;
        }
    }
    s = ewald_block_sum(s, red);
    if (threadIdx.x == 0) e.part[(size_t)w * (e.pk + e.pr) + e.pk + p] = s;
}

__global__ __launch_bounds__(kBlock) void k_ewald_finish(EwaldView e, double* eloc)
{
    const int w = blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= e.W) return;
    const double* pt = e.part + (size_t)w * (e.pk + e.pr);
    double rec = 0.0, real = 0.0;
    for (int p = 0; p < e.pk; ++p) rec += pt[p];
    for (int p = 0; p < e.pr; ++p) real += pt[e.pk + p];
    const double N = (double)e.ne, omega = e.L * e.L * e.L;
    const double v = real + (4.0 * kPi / omega) * rec - e.alpha * N / sqrt(kPi) -
                     kPi * N * N / (2.0 * e.alpha * e.alpha * omega);
    eloc[w] += v;
}

void launch_ewald(const EwaldView& e, double* eloc, hipStream_t s)
{
    const size_t n = (size_t)e.W * e.ne;
    hipLaunchKernelGGL(k_ewald_phase, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, e);
    const size_t lds = sizeof(double2) * kTile * 3 * (e.nmax + 1);
    hipLaunchKernelGGL(k_ewald_recip, dim3(e.W * e.pk), dim3(kBlock), lds, s, e);
    hipLaunchKernelGGL(k_ewald_real, dim3(e.W * e.pr), dim3(kBlock), 0, s, e);
    hipLaunchKernelGGL(k_ewald_finish, dim3((e.W + kBlock - 1) / kBlock), dim3(kBlock), 0, s, e, eloc);
}

int ewald_wavevectors_per_block() { return kKPT * kBlock; }

}  // namespace cq
