// Rank-k inverse update on the FP32 matrix cores (mixed precision, N % 32 == 0,
// N <= 1024).
//
// Same update as k_flush_vec: with u_m the accepted rows, c_m the columns just
// before move m, rho_m the ratios and G[m][j] = u_m . c_j, every row a of
// M = (A^-1)^T gets
//     x_m = M[a] . u_m                                   (GEMM 1, X = M U^T)
//     b_m = (x_m - sum_{j<m} b_j G[m][j] - delta(a, e_m)) / rho_m
//     M[a] -= sum_m b_m c_m                              (GEMM 2, M -= B C)
// The forward substitution is the same for every row: with L lower triangular,
// L[m][j] = G[m][j] (j < m), L[m][m] = rho_m, it is b = L^-1 y, y_m = x_m -
// delta(a, e_m).  k_window_linv forms L^-1 once per walker (FP64, one lane per
// column), so the strip's 32 rows are solved in parallel.
// One workgroup owns a strip of 32 rows of M for the whole update, so M is read
// and written once.  The strip stays in registers as 32 x 32 tiles of M^T in the
// accumulator layout of v_mfma_f32_32x32x2f32 (lane l holds strip row l % 32 and
// the 16 columns 8 (v / 4) + 4 (l / 32) + v % 4 of the tile).  That layout is at
// the same time the B operand of GEMM 1 (the two k values of step v are the
// columns of half 0 and half 1) and the accumulator of GEMM 2, so neither product
// moves the strip.  Each of the 8 waves holds every 8th tile; GEMM 1 partial
// sums of the waves are added in a fixed order in LDS.
#include <algorithm>

#include "cq_device.h"
#include "cq_internal.h"

namespace cq {

typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kFlushWaves = 8;                    // waves per workgroup (two workgroups per CU)
constexpr int kFlushThreads = 64 * kFlushWaves;
constexpr int kStripTiles = 4;                    // 32-column tiles per wave (N <= 8 * 4 * 32)

// Window and per-move paths: the window's columns are read from the row buffer
// Cbuf.  Two workgroups per CU (four waves per SIMD): one's operand and HBM
// latency hides behind the other's MFMAs.
__device__ __forceinline__ void flush_mfma_body(const CrowdView<float>& v, int spin, const int w, const int strip)
{
    __shared__ float sX[kFlushWaves][32][33];  // per wave: partial X^T[m][i]
    __shared__ float sB[32][33];      // -b[i][m] (FP32 operand of GEMM 2)
    __shared__ double sY[32][33];     // x[i][j] - delta(row0 + i, e_j)
    __shared__ double sL[32][33];     // L^-1
    __shared__ int wel[32], wsl[32];
    const int n = v.n, K = v.K;
    const int ntile = n / 32, nstrip = n / 32;
    if (w >= v.W) return;
    int cnt = v.cnt[(size_t)2 * v.W + w];
    if (cnt > K) cnt = K;
    if (cnt <= 0) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int h = lane >> 5, l32 = lane & 31;
    if (tid < cnt) {
        wel[tid] = v.welec[(size_t)w * K + tid];
        const int sl = v.wslot[(size_t)w * K + tid];
        if (sl < 0 || sl >= v.QR) atomicOr(&v.status[w], 2);
        wsl[tid] = sl < 0 || sl >= v.QR ? 0 : sl;
    }
    __syncthreads();

    // the accepted orbital rows of the window go to the A, G, L rows
    for (int mm = strip; mm < cnt; mm += nstrip) {
        const int ea = wel[mm];
        if (ea < 0 || ea >= n) {
            if (tid == 0) atomicOr(&v.status[w], 2);
            continue;
        }
        const float* src = v.stage + ((size_t)w * v.QR + wsl[mm]) * 5 * (size_t)n;
        float* dst = v.VGL + (((size_t)w * 2 + spin) * n + ea) * 5 * (size_t)n;
        for (int i = tid * 4; i < 5 * n; i += kFlushThreads * 4) {
            float x[4];
            load16(src + i, x);
            store16(dst + i, x);
        }
    }

    const int row0 = strip * 32;
    float* Mb = v.M + (((size_t)w * 2 + spin) * n + row0) * (size_t)n;
    f32x16 mt[kStripTiles];
#pragma unroll
    for (int tt = 0; tt < kStripTiles; ++tt) {
        const int t = wave + kFlushWaves * tt;
#pragma unroll
        for (int q = 0; q < 16; ++q) mt[tt][q] = 0.0f;
        if (t < ntile) {
            const float* src = Mb + (size_t)l32 * n + t * 32 + 4 * h;
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                float x[4];
                load16(src + 8 * g, x);
#pragma unroll
                for (int q = 0; q < 4; ++q) mt[tt][4 * g + q] = x[q];
            }
        }
    }

    // GEMM 1: X^T[m][i] = sum_k u_m[k] M[row0 + i][k] over this wave's tiles.  The
    // second workgroup on the CU covers the operand latency, so there is no register
    // double buffer here.
    f32x16 xacc;
#pragma unroll
    for (int q = 0; q < 16; ++q) xacc[q] = 0.0f;
    const float* urow = v.stage + ((size_t)w * v.QR + wsl[l32 < cnt ? l32 : 0]) * 5 * (size_t)n;
    const bool urow_live = l32 < cnt;
#pragma unroll
    for (int tt = 0; tt < kStripTiles; ++tt) {
        const int t = wave + kFlushWaves * tt;
        if (t < ntile) {
            float u[16];
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                float x[4];
                load16(urow + t * 32 + 8 * g + 4 * h, x);
#pragma unroll
                for (int q = 0; q < 4; ++q) u[4 * g + q] = urow_live ? x[q] : 0.0f;
            }
#pragma unroll
            for (int q = 0; q < 16; ++q) xacc = __builtin_amdgcn_mfma_f32_32x32x2f32(u[q], mt[tt][q], xacc, 0, 0, 0);
        }
        __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int q = 0; q < 16; ++q) sX[wave][8 * (q >> 2) + 4 * h + (q & 3)][l32] = xacc[q];
    __syncthreads();

    // y[i][j] = x[i][j] - delta(row0 + i, e_j) in FP64, then
    // b[i][m] = sum_j Linv[m][j] y[i][j] (Linv and y zero-padded to 32 x 32)
    for (int idx = tid; idx < 32 * 32; idx += kFlushThreads) {
        const int i = idx >> 5, j = idx & 31;
        double x = 0.0;
#pragma unroll
        for (int q = 0; q < kFlushWaves; ++q) x += (double)sX[q][j][i];
        sY[i][j] = j < cnt ? x - (row0 + i == wel[j] ? 1.0 : 0.0) : 0.0;
        sL[i][j] = (i < cnt && j <= i) ? v.wlinv[((size_t)w * K + i) * K + j] : 0.0;
    }
    __syncthreads();
    {
        constexpr int MPT = 32 * 32 / kFlushThreads;  // moves of one row per thread
        const int i = tid / (32 / MPT), m0 = (tid % (32 / MPT)) * MPT;
        double b[MPT];
#pragma unroll
        for (int r = 0; r < MPT; ++r) b[r] = 0.0;
#pragma unroll
        for (int j = 0; j < 32; ++j) {
            const double y = sY[i][j];
#pragma unroll
            for (int r = 0; r < MPT; ++r) b[r] = fma(sL[m0 + r][j], y, b[r]);
        }
#pragma unroll
        for (int r = 0; r < MPT; ++r) sB[i][m0 + r] = -(float)b[r];  // GEMM 2 subtracts
    }
    __syncthreads();

    // GEMM 2: M^T[k][i] -= sum_m c_m[k] b[i][m], moves m = 16 h + q, one load per step
    const float* Cw = v.Cbuf + (size_t)w * K * n;
    auto fetch = [&](int t, float (&a)[16]) {
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int m = 16 * h + q;
            const float c = Cw[(size_t)(m < cnt ? m : 0) * n + t * 32 + l32];
            a[q] = m < cnt ? c : 0.0f;
        }
    };
    float nb[16];  // -b[l32][16 h + q], the same for every tile
#pragma unroll
    for (int q = 0; q < 16; ++q) nb[q] = sB[l32][16 * h + q];
#pragma unroll
    for (int tt = 0; tt < kStripTiles; ++tt) {
        const int t = wave + kFlushWaves * tt;
        if (t < ntile) {
            float a[16];
            fetch(t, a);
            // operands past cnt are zero (Ct and b are zero-padded), so all 16 steps run
#pragma unroll
            for (int q = 0; q < 16; ++q) mt[tt] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[q], nb[q], mt[tt], 0, 0, 0);
        }
        __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int tt = 0; tt < kStripTiles; ++tt) {
        const int t = wave + kFlushWaves * tt;
        if (t < ntile) {
            float* dst = Mb + (size_t)l32 * n + t * 32 + 4 * h;
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                float x[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) x[q] = mt[tt][4 * g + q];
                store16(dst + 8 * g, x);
            }
        }
    }
}

__global__ __launch_bounds__(kFlushThreads) __attribute__((amdgpu_waves_per_eu(4))) void k_flush_mfma(CrowdView<float> v, int spin)
{
    int w, strip;
    xcd_map(blockIdx.x, v.n / 32, w, strip);
    flush_mfma_body(v, spin, w, strip);
}

// Several systems in one launch: item i = (system, walker, strip of 32 rows); persistent.
__global__ __launch_bounds__(kFlushThreads) __attribute__((amdgpu_waves_per_eu(4))) void k_flush_mfma_multi(
    const CrowdView<float>* __restrict__ views, const int4* __restrict__ items, int n_items, int spin)
{
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        const int4 item = items[it];
        flush_mfma_body(views[item.x], spin, item.y, item.z);
        __syncthreads();  // the next item reuses the shared memory
    }
}

// Batched path: the window's accepted value rows come packed in v.ub and its
// columns transposed in v.ct (both written by the column kernel, which has also
// moved the accepted orbital rows), so a strip's loads need no indirection.  Two
// workgroups of 8 waves (4 tiles each) per CU: one's loads are in flight while the
// other runs its MFMAs.
constexpr int kBatchWaves = 8;
constexpr int kBatchThreads = 64 * kBatchWaves;
constexpr int kBatchTiles = 4;

__global__ __launch_bounds__(kBatchThreads) __attribute__((amdgpu_waves_per_eu(4))) void k_flush_mfma_batch(
    CrowdView<float> v, int spin)
{
    __shared__ float sX[kBatchWaves][32][33];  // per wave: partial X^T[m][i]
    __shared__ float sB[32][33];      // -b[i][m] (FP32 operand of GEMM 2)
    __shared__ double sY[32][33];     // x[i][j] - delta(row0 + i, e_j)
    __shared__ double sL[32][33];     // L^-1
    __shared__ int wel[32];
    const int n = v.n, K = v.K;
    const int ntile = n / 32, nstrip = n / 32;
    int w, strip;
    xcd_map(blockIdx.x, nstrip, w, strip);
    if (w >= v.W) return;
    int cnt = v.cnt[(size_t)2 * v.W + w];
    if (cnt > K) cnt = K;
    if (cnt <= 0) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int h = lane >> 5, l32 = lane & 31;
    if (tid < 32) wel[tid] = tid < cnt ? v.welec[(size_t)w * K + tid] : -1;
    __syncthreads();

    const int row0 = strip * 32;
    float* Mb = v.M + (((size_t)w * 2 + spin) * n + row0) * (size_t)n;
    f32x16 mt[kBatchTiles];
#pragma unroll
    for (int tt = 0; tt < kBatchTiles; ++tt) {
        const int t = wave + kBatchWaves * tt;
#pragma unroll
        for (int q = 0; q < 16; ++q) mt[tt][q] = 0.0f;
        if (t < ntile) {
            const float* src = Mb + (size_t)l32 * n + t * 32 + 4 * h;
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                float x[4];
                load16(src + 8 * g, x);
#pragma unroll
                for (int q = 0; q < 4; ++q) mt[tt][4 * g + q] = x[q];
            }
        }
    }

    // GEMM 1: X^T[m][i] = sum_k u_m[k] M[row0 + i][k] over this wave's tiles.  The
    // second workgroup on the CU covers the operand latency, so there is no register
    // double buffer here.
    f32x16 xacc;
#pragma unroll
    for (int q = 0; q < 16; ++q) xacc[q] = 0.0f;
    const float* urow = v.ub + ((size_t)w * kMaxDelay + l32) * n;
    const bool urow_live = l32 < cnt;
#pragma unroll
    for (int tt = 0; tt < kBatchTiles; ++tt) {
        const int t = wave + kBatchWaves * tt;
        if (t < ntile) {
            float u[16];
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                float x[4];
                load16(urow + t * 32 + 8 * g + 4 * h, x);
#pragma unroll
                for (int q = 0; q < 4; ++q) u[4 * g + q] = urow_live ? x[q] : 0.0f;
            }
#pragma unroll
            for (int q = 0; q < 16; ++q) xacc = __builtin_amdgcn_mfma_f32_32x32x2f32(u[q], mt[tt][q], xacc, 0, 0, 0);
        }
        __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int q = 0; q < 16; ++q) sX[wave][8 * (q >> 2) + 4 * h + (q & 3)][l32] = xacc[q];
    __syncthreads();

    // y[i][j] = x[i][j] - delta(row0 + i, e_j) in FP64, then
    // b[i][m] = sum_j Linv[m][j] y[i][j] (Linv and y zero-padded to 32 x 32)
    for (int idx = tid; idx < 32 * 32; idx += kBatchThreads) {
        const int i = idx >> 5, j = idx & 31;
        double x = 0.0;
#pragma unroll
        for (int q = 0; q < kBatchWaves; ++q) x += (double)sX[q][j][i];
        sY[i][j] = j < cnt ? x - (row0 + i == wel[j] ? 1.0 : 0.0) : 0.0;
        sL[i][j] = (i < cnt && j <= i) ? v.wlinv[((size_t)w * K + i) * K + j] : 0.0;
    }
    __syncthreads();
    {
        constexpr int MPT = 32 * 32 / kBatchThreads;  // moves of one row per thread
        const int i = tid / (32 / MPT), m0 = (tid % (32 / MPT)) * MPT;
        double b[MPT];
#pragma unroll
        for (int r = 0; r < MPT; ++r) b[r] = 0.0;
#pragma unroll
        for (int j = 0; j < 32; ++j) {
            const double y = sY[i][j];
#pragma unroll
            for (int r = 0; r < MPT; ++r) b[r] = fma(sL[m0 + r][j], y, b[r]);
        }
#pragma unroll
        for (int r = 0; r < MPT; ++r) sB[i][m0 + r] = -(float)b[r];  // GEMM 2 subtracts
    }
    __syncthreads();

    // GEMM 2: M^T[k][i] -= sum_m c_m[k] b[i][m], moves m = 16 h + q, operands Ct[k][m]
    // (32 per row, zero past cnt), 4 vector loads per tile
    const float* Ct = v.ct + ((size_t)w * n) * kMaxDelay;
    auto fetch = [&](int t, float (&a)[16]) {
        const float* src = Ct + (size_t)(t * 32 + l32) * kMaxDelay + 16 * h;
#pragma unroll
        for (int g = 0; g < 4; ++g) load16(src + 4 * g, &a[4 * g]);
    };
    float nb[16];  // -b[l32][16 h + q], the same for every tile
#pragma unroll
    for (int q = 0; q < 16; ++q) nb[q] = sB[l32][16 * h + q];
#pragma unroll
    for (int tt = 0; tt < kBatchTiles; ++tt) {
        const int t = wave + kBatchWaves * tt;
        if (t < ntile) {
            float a[16];
            fetch(t, a);
            // operands past cnt are zero (Ct and b are zero-padded), so all 16 steps run
#pragma unroll
            for (int q = 0; q < 16; ++q) mt[tt] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[q], nb[q], mt[tt], 0, 0, 0);
        }
        __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int tt = 0; tt < kBatchTiles; ++tt) {
        const int t = wave + kBatchWaves * tt;
        if (t < ntile) {
            float* dst = Mb + (size_t)l32 * n + t * 32 + 4 * h;
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                float x[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) x[q] = mt[tt][4 * g + q];
                store16(dst + 8 * g, x);
            }
        }
    }
}

// L^-1 of each walker's window (lower triangular, FP64): lane j forms column j
// by forward substitution down the rows.
__device__ __forceinline__ void window_linv_body(const CrowdView<float>& v, const int w)
{
    __shared__ double sL[32][33];
    __shared__ double sX[32][33];
    const int K = v.K, lane = threadIdx.x;
    int cnt = v.cnt[(size_t)2 * v.W + w];
    if (cnt > K) cnt = K;
    if (cnt <= 0) return;
    for (int idx = lane; idx < cnt * cnt; idx += 64) {
        const int r = idx / cnt, c = idx % cnt;
        sL[r][c] = c < r ? v.wG[((size_t)w * K + r) * K + c] : (c == r ? v.wrho[(size_t)w * K + r] : 0.0);
    }
    __syncthreads();
    if (lane < cnt) {
        const int j = lane;
        for (int m = 0; m < cnt; ++m) {
            double t = m == j ? 1.0 : 0.0;
            for (int q = j; q < m; ++q) t -= sL[m][q] * sX[q][j];
            sX[m][j] = m < j ? 0.0 : t / sL[m][m];
        }
    }
    __syncthreads();
    for (int idx = lane; idx < cnt * cnt; idx += 64) {
        const int r = idx / cnt, c = idx % cnt;
        v.wlinv[((size_t)w * K + r) * K + c] = sX[r][c];
    }
}

__global__ __launch_bounds__(64) void k_window_linv(CrowdView<float> v) { window_linv_body(v, blockIdx.x); }

__global__ __launch_bounds__(64) void k_window_linv_multi(const CrowdView<float>* __restrict__ views,
                                                          const int2* __restrict__ items, int n_items)
{
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        const int2 item = items[it];
        window_linv_body(views[item.x], item.y);
        __syncthreads();
    }
}

void launch_flush_mfma_multi(const CrowdView<float>* views, const int2* walkers, int n_walkers, const int4* strips,
                             int n_strips, int spin, int grid, hipStream_t s)
{
    hipLaunchKernelGGL(k_window_linv_multi, dim3(std::min(n_walkers, 4 * grid)), dim3(64), 0, s, views, walkers,
                       n_walkers);
    hipLaunchKernelGGL(k_flush_mfma_multi, dim3(std::min(n_strips, grid)), dim3(kFlushThreads), 0, s, views, strips,
                       n_strips, spin);
}

bool flush_mfma_fits(int n)
{
    return n % 32 == 0 && n <= kFlushWaves * kStripTiles * 32 && n <= kBatchWaves * kBatchTiles * 32;
}

void launch_flush_mfma(const CrowdView<float>& v, int spin, hipStream_t s, bool linv_ready)
{
    const int nstrip = v.n / 32;
    if (!linv_ready) hipLaunchKernelGGL(k_window_linv, dim3(v.W), dim3(64), 0, s, v);
    if (v.ct && v.ub)
        hipLaunchKernelGGL(k_flush_mfma_batch, dim3(xcd_grid(v.W, nstrip)), dim3(kBatchThreads), 0, s, v, spin);
    else
        hipLaunchKernelGGL(k_flush_mfma, dim3(xcd_grid(v.W, nstrip)), dim3(kFlushThreads), 0, s, v, spin);
}

}  // namespace cq
