// FP64 rank-k inverse update of the batched path on the FP64 matrix cores
// (v_mfma_f64_16x16x4f64), N % 16 == 0, N <= 1024.
//
// The same update as k_flush_vec: with u_m the accepted rows, c_m the columns just before
// move m, rho_m the ratios and G[m][j] = u_m . c_j, every row a of M = (A^-1)^T gets
//     x_m = M[a] . u_m                                          (GEMM 1, X = M U^T)
//     b_m = (x_m - delta(a, e_m) - sum_{j<m} b_j G[m][j]) / rho_m  (forward substitution)
//     M[a] -= sum_m b_m c_m                                     (GEMM 2, M -= B C)
// One workgroup owns a strip of 16 rows of M, so M is read and written once.  The strip
// lives in registers as 16 x 16 tiles of M^T in the accumulator layout of the FP64 MFMA
// (lane l holds D[l / 16 + 4 v][l % 16], v = 0..3): element v of a tile is at the same time
// the B operand of GEMM 1's k-step v (lane l supplies B[l / 16][l % 16]) and a part of the
// accumulator of GEMM 2, so neither product moves the strip.  The strip is loaded and stored
// in whole rows (coalesced) and transposed through LDS one tile per wave at a time.  Each of
// the 8 waves holds every 8th tile; GEMM 1 partial sums of the waves are added in a fixed
// order in LDS, and the forward substitution runs in move order per row, in FP64, as in
// k_flush_vec (a sequence of Sherman-Morrison steps).
#include "cq_device.h"
#include "cq_internal.h"

namespace cq {

namespace {

typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr int kF64Waves = 8;
constexpr int kF64Threads = 64 * kF64Waves;
constexpr int kF64Tiles = 8;  // 16-column tiles per wave: N <= 8 x 8 x 16

}  // namespace

__global__ __launch_bounds__(kF64Threads) void k_flush_f64_mfma(CrowdView<double> v, int spin)
{
    __shared__ double sT[kF64Waves][16][17];  // per wave: one 16 x 16 tile in transit
    __shared__ double sX[kF64Waves][32][17];  // per wave: partial X^T[m][i]
    __shared__ double sY[16][33];             // x[i][m] - delta(row0 + i, e_m)
    __shared__ double sG[32][33];             // G[m][j], j < m
    __shared__ double sB[16][33];             // b[i][m] (zero past the window's moves)
    __shared__ double sR[32];                 // rho_m
    __shared__ int wel[32], wsl[32];
    const int n = v.n, K = v.K;
    const int ntile = n / 16, nstrip = n / 16;
    int w, strip;
    xcd_map(blockIdx.x, nstrip, w, strip);
    if (w >= v.W) return;
    int cnt = v.cnt[(size_t)2 * v.W + w];
    if (cnt > K) cnt = K;
    if (cnt <= 0) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int r16 = lane & 15, q4 = lane >> 4;
    if (tid < 32) {
        const bool live = tid < cnt;
        int e = live ? v.welec[(size_t)w * K + tid] : -1;
        int sl = live ? v.wslot[(size_t)w * K + tid] : 0;
        if (live && (sl < 0 || sl >= v.QR)) {
            atomicOr(&v.status[w], 2);
            sl = 0;
        }
        wel[tid] = e;
        wsl[tid] = sl;
        sR[tid] = live ? v.wrho[(size_t)w * K + tid] : 1.0;
    }
    for (int idx = tid; idx < 32 * 32; idx += kF64Threads) {
        const int r = idx >> 5, c = idx & 31;
        sG[r][c] = (r < cnt && c < r) ? v.wG[((size_t)w * K + r) * K + c] : 0.0;
    }
    __syncthreads();

    // the accepted orbital rows of the window go to the A, G, L rows (one strip's share)
    for (int mm = strip; mm < cnt; mm += nstrip) {
        const int ea = wel[mm];
        if (ea < 0 || ea >= n) {
            if (tid == 0) atomicOr(&v.status[w], 2);
            continue;
        }
        const double* src = v.stage + ((size_t)w * v.QR + wsl[mm]) * 5 * (size_t)n;
        double* dst = v.VGL + (((size_t)w * 2 + spin) * n + ea) * 5 * (size_t)n;
        for (int i = tid; i < 5 * n; i += kF64Threads) dst[i] = src[i];
    }

    // the strip: row loads of 16 columns (4 rows per load), transposed through LDS into
    // D[k][i] = M[row0 + i][16 t + k]
    const int row0 = strip * 16;
    double* Mb = v.M + (((size_t)w * 2 + spin) * n + row0) * (size_t)n;
    f64x4 acc[kF64Tiles];
#pragma unroll
    for (int tt = 0; tt < kF64Tiles; ++tt) {
        const int t = wave + kF64Waves * tt;
        acc[tt] = f64x4{0.0, 0.0, 0.0, 0.0};
        if (t < ntile) {
            double x[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) x[j] = Mb[(size_t)(4 * j + q4) * n + 16 * t + r16];
#pragma unroll
            for (int j = 0; j < 4; ++j) sT[wave][4 * j + q4][r16] = x[j];
        }
        __syncthreads();
        if (t < ntile)
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[tt][q] = sT[wave][r16][q4 + 4 * q];
        __syncthreads();
    }

    // GEMM 1: X^T[m][i] = sum_k u_m[k] M^T[k][i], moves m = 16 mb + r16 supply A
    f64x4 xacc[2] = {f64x4{0.0, 0.0, 0.0, 0.0}, f64x4{0.0, 0.0, 0.0, 0.0}};
    const double* urow[2];
    bool ulive[2];
#pragma unroll
    for (int mb = 0; mb < 2; ++mb) {
        const int m = 16 * mb + r16;
        ulive[mb] = m < cnt;
        urow[mb] = v.stage + ((size_t)w * v.QR + wsl[ulive[mb] ? m : 0]) * 5 * (size_t)n;
    }
#pragma unroll
    for (int tt = 0; tt < kF64Tiles; ++tt) {
        const int t = wave + kF64Waves * tt;
        if (t < ntile) {
            double a[2][4];
#pragma unroll
            for (int mb = 0; mb < 2; ++mb)
#pragma unroll
                for (int q = 0; q < 4; ++q) a[mb][q] = ulive[mb] ? urow[mb][16 * t + 4 * q + q4] : 0.0;
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int mb = 0; mb < 2; ++mb)
                    xacc[mb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[mb][q], acc[tt][q], xacc[mb], 0, 0, 0);
        }
    }
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int q = 0; q < 4; ++q) sX[wave][16 * mb + q4 + 4 * q][r16] = xacc[mb][q];
    __syncthreads();

    // y[i][m] = x[i][m] - delta(row0 + i, e_m), the waves' partial sums in wave order
    for (int idx = tid; idx < 16 * 32; idx += kF64Threads) {
        const int i = idx >> 5, m = idx & 31;
        double x = 0.0;
#pragma unroll
        for (int q = 0; q < kF64Waves; ++q) x += sX[q][m][i];
        sY[i][m] = m < cnt ? x - (row0 + i == wel[m] ? 1.0 : 0.0) : 0.0;
    }
    __syncthreads();
    // forward substitution in move order, one thread per strip row
    if (tid < 16) {
        const int i = tid;
        for (int m = 0; m < 32; ++m) {
            double b = 0.0;
            if (m < cnt) {
                double t = sY[i][m];
                for (int j = 0; j < m; ++j) t -= sB[i][j] * sG[m][j];
                b = t / sR[m];
            }
            sB[i][m] = b;
        }
    }
    __syncthreads();

    // GEMM 2: M^T[k][i] -= sum_m c_m[k] b[i][m], moves m = 4 s + q4 per step
    double nb[8];
#pragma unroll
    for (int s = 0; s < 8; ++s) nb[s] = -sB[r16][4 * s + q4];
    const double* Cw = v.Cbuf + (size_t)w * K * n;
#pragma unroll
    for (int tt = 0; tt < kF64Tiles; ++tt) {
        const int t = wave + kF64Waves * tt;
        if (t < ntile) {
            double a[8];
#pragma unroll
            for (int s = 0; s < 8; ++s) {
                const int m = 4 * s + q4;
                a[s] = m < cnt ? Cw[(size_t)m * n + 16 * t + r16] : 0.0;
            }
#pragma unroll
            for (int s = 0; s < 8; ++s) acc[tt] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[s], nb[s], acc[tt], 0, 0, 0);
        }
    }

    // store: transposed back through LDS, written in row segments of 16 columns
#pragma unroll
    for (int tt = 0; tt < kF64Tiles; ++tt) {
        const int t = wave + kF64Waves * tt;
        if (t < ntile)
#pragma unroll
            for (int q = 0; q < 4; ++q) sT[wave][r16][q4 + 4 * q] = acc[tt][q];
        __syncthreads();
        if (t < ntile)
#pragma unroll
            for (int j = 0; j < 4; ++j) Mb[(size_t)(4 * j + q4) * n + 16 * t + r16] = sT[wave][4 * j + q4][r16];
        __syncthreads();
    }
}

bool flush_f64_mfma_fits(int n) { return n % 16 == 0 && n <= kF64Waves * kF64Tiles * 16; }

void launch_flush_f64_mfma(const CrowdView<double>& v, int spin, hipStream_t s)
{
    hipLaunchKernelGGL(k_flush_f64_mfma, dim3(xcd_grid(v.W, v.n / 16)), dim3(kF64Threads), 0, s, v, spin);
}

}  // namespace cq
