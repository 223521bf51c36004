// FP64 inversion of the Slater matrices: at set-up and for the periodic
// recompute that removes the drift of the updated (FP32 in the mixed path)
// inverses.  Also produces log|det| and the sign.
//
// Method: in-place Gauss-Jordan "sweeps" with partial pivoting and no
// physical row exchanges, applied to B = A^T (so the result is (A^T)^-1 =
// (A^-1)^T = M directly).  The sweep of column k at pivot row p = pi(k) (the
// largest |B[i][k]| among rows not yet used) is
//   B[i][j] -= B[i][k] B[p][j] / piv  (i != p, j != k),   B[p][j] /= piv,
//   B[i][k]  = -B[i][k] / piv,                            B[p][k]  = 1 / piv.
// After all n sweeps, S[pi(k)][j] = M[k][pi(j)], so M[k][c] = S[pi(k)][pi^-1(c)];
// det A = det B = sign(pi) prod piv.  A pivot with |piv| <= n eps max|A_ij| (or
// not finite) marks the matrix numerically singular.
//
// n <= 64: one workgroup per matrix with the matrix in LDS (k_gj_small).
// n  > 64: blocked.  A panel of b columns is swept by one workgroup per matrix
// (k_gj_panel, panel in LDS); the same b sweeps act on every other column as the
// rank-b update  S[i][j] = [i not a pivot of the panel] S[i][j]
//                          + sum_q P[i][q] S_old[pi(k0+q)][j]
// with P the swept panel (k_gj_update), 2 n^3 flops in all.
#include "cq_device.h"
#include "cq_internal.h"

namespace cq {

constexpr int kSmallN = 64;

// argmax of |value| over the block (ties -> lowest index); returns in *best_i.
__device__ __forceinline__ void wave_argmax(double& val, int& idx)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const double ov = __shfl_xor(val, off, 64);
        const int oi = __shfl_xor(idx, off, 64);
        if (ov > val || (ov == val && oi < idx)) {
            val = ov;
            idx = oi;
        }
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_gj_small(CrowdView<T> v)
{
    __shared__ double S[kSmallN][kSmallN + 1];
    __shared__ double colk[kSmallN], rowp[kSmallN];
    __shared__ int used[kSmallN], piv_row[kSmallN], inv_perm[kSmallN];
    __shared__ double s_piv;
    __shared__ int s_p;
    const int mat = blockIdx.x, w = mat >> 1, spin = mat & 1;
    const int n = v.n, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const T* A = v.VGL + ((size_t)w * 2 + spin) * n * 5 * (size_t)n;
    __shared__ double smax[4];
    double amax = 0.0;
    for (int idx = tid; idx < n * n; idx += kBlock) {
        const int i = idx / n, j = idx % n;  // A[i][j] = phi_j(r_i)
        const double a = (double)A[(size_t)i * 5 * n + j];
        S[j][i] = a;
        amax = fmax(amax, fabs(a));
    }
    for (int off = 32; off >= 1; off >>= 1) amax = fmax(amax, __shfl_xor(amax, off, 64));
    if (lane == 0) smax[wave] = amax;
    if (tid < n) used[tid] = 0;
    __syncthreads();
    const double tiny = n * 2.220446049250313e-16 * fmax(fmax(smax[0], smax[1]), fmax(smax[2], smax[3]));
    double logabs = 0.0;
    int negs = 0, bad = 0;
    for (int k = 0; k < n; ++k) {
        if (wave == 0) {
            double best = -1.0;
            int bi = n;
            for (int i = lane; i < n; i += 64)
                if (!used[i]) {
                    const double val = fabs(S[i][k]);
                    if (val > best) { best = val; bi = i; }
                }
            wave_argmax(best, bi);
            if (lane == 0) {
                if (bi >= n)  // every candidate is NaN: take the first unused row, flagged below
                    for (int i = n - 1; i >= 0; --i)
                        if (!used[i]) bi = i;
                s_p = bi;
                s_piv = S[bi][k];
                used[bi] = 1;
                piv_row[k] = bi;
            }
        }
        __syncthreads();
        const int p = s_p;
        const double piv = s_piv;
        if (!(fabs(piv) > tiny) || !isfinite(piv)) bad = 1;
        logabs += log(fabs(piv));
        negs += piv < 0.0;
        if (tid < n) {
            colk[tid] = S[tid][k];
            rowp[tid] = S[p][tid];
        }
        __syncthreads();
        const double ipiv = 1.0 / piv;
        for (int idx = tid; idx < n * n; idx += kBlock) {
            const int i = idx / n, j = idx % n;
            double val;
            if (i == p)
                val = (j == k) ? ipiv : rowp[j] * ipiv;
            else if (j == k)
                val = -colk[i] * ipiv;
            else
                val = S[i][j] - colk[i] * rowp[j] * ipiv;
            S[i][j] = val;
        }
        __syncthreads();
    }
    if (tid < n) inv_perm[piv_row[tid]] = tid;
    __syncthreads();
    T* M = v.M + ((size_t)w * 2 + spin) * n * (size_t)n;
    for (int idx = tid; idx < n * n; idx += kBlock) {
        const int k = idx / n, c = idx % n;
        M[idx] = (T)S[piv_row[k]][inv_perm[c]];
    }
    if (tid == 0) {
        // sign of the permutation k -> pi(k) from its cycle decomposition
        int parity = 0;
        for (int i = 0; i < n; ++i) used[i] = 0;
        for (int i = 0; i < n; ++i) {
            if (used[i]) continue;
            int len = 0;
            for (int j = i; !used[j]; j = piv_row[j]) { used[j] = 1; ++len; }
            parity ^= (len - 1) & 1;
        }
        const int sgn = ((negs + parity) & 1) ? -1 : 1;
        const double old = v.logdet[w * 2 + spin];
        v.drift[w * 2 + spin] = fabs(old - logabs);
        v.logdet[w * 2 + spin] = logabs;
        v.sign[w * 2 + spin] = sgn;
        if (bad) atomicOr(&v.status[w], 1);
    }
}

// ---------------------------------------------------------------- blocked

template <typename T>
__global__ __launch_bounds__(kBlock) void k_gj_load(CrowdView<T> v, double* __restrict__ S,
                                                     unsigned long long* __restrict__ scale)
{
    // S[mat][j][i] = A[i][j] through a 64 x 64 LDS tile; scale[mat] = max |A_ij|
    // (non-negative doubles order like their bit patterns)
    __shared__ double tile[64][65];
    __shared__ double wmax[4];
    const int n = v.n, tiles = (n + 63) / 64;
    const int mat = blockIdx.x / (tiles * tiles), t = blockIdx.x % (tiles * tiles);
    const int ti = t / tiles, tj = t % tiles;
    const int w = mat >> 1, spin = mat & 1;
    const T* A = v.VGL + ((size_t)w * 2 + spin) * n * 5 * (size_t)n;
    double amax = 0.0;
    for (int idx = threadIdx.x; idx < 64 * 64; idx += kBlock) {
        const int r = idx / 64, c = idx % 64;
        const int i = ti * 64 + r, j = tj * 64 + c;
        const double a = (i < n && j < n) ? (double)A[(size_t)i * 5 * n + j] : 0.0;
        tile[r][c] = a;
        amax = fmax(amax, fabs(a));
    }
    for (int off = 32; off >= 1; off >>= 1) amax = fmax(amax, __shfl_xor(amax, off, 64));
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = amax;
    __syncthreads();
    if (threadIdx.x == 0) {
        const double m = fmax(fmax(wmax[0], wmax[1]), fmax(wmax[2], wmax[3]));
        atomicMax(&scale[mat], (unsigned long long)__double_as_longlong(m));
    }
    double* Sm = S + (size_t)mat * n * n;
    for (int idx = threadIdx.x; idx < 64 * 64; idx += kBlock) {
        const int r = idx / 64, c = idx % 64;  // output row j = tj*64 + r, column i = ti*64 + c
        const int j = tj * 64 + r, i = ti * 64 + c;
        if (i < n && j < n) Sm[(size_t)j * n + i] = tile[c][r];
    }
}

// Sweep the b panel columns k0 .. k0+b-1 of every matrix (one workgroup per
// matrix, panel and row-use flags in LDS), record the pivots, copy the old
// pivot rows.
__global__ __launch_bounds__(kBlock) void k_gj_panel(double* __restrict__ S, double* __restrict__ PR,
                                                      int* __restrict__ pivrow, int* __restrict__ rowstate,
                                                      double* __restrict__ logabs, int* __restrict__ negs,
                                                      int* __restrict__ status,
                                                      const unsigned long long* __restrict__ scale, int n, int b,
                                                      int k0, int panel)
{
    extern __shared__ double sh[];
    double* P = sh;                    // [n][b]
    double* colk = P + (size_t)n * b;  // [n]
    int* used = (int*)(colk + n);      // [n]
    __shared__ double rowp[64];
    __shared__ double wbest[4];
    __shared__ int wbi[4];
    __shared__ int pivs[64];
    __shared__ double s_piv;
    const int mat = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    double* Sm = S + (size_t)mat * n * n;
    int* rs = rowstate + (size_t)mat * n;
    for (int idx = tid; idx < n * b; idx += kBlock) {
        const int i = idx / b, q = idx % b;
        P[idx] = Sm[(size_t)i * n + k0 + q];
    }
    for (int i = tid; i < n; i += kBlock) used[i] = rs[i];
    __syncthreads();
    const double tiny = n * 2.220446049250313e-16 * __longlong_as_double((long long)scale[mat]);
    double la = 0.0;
    int ng = 0, bad = 0;
    for (int q = 0; q < b; ++q) {
        double best = -1.0;
        int bi = n;
        for (int i = tid; i < n; i += kBlock)
            if (used[i] == 0) {
                const double val = fabs(P[i * b + q]);
                if (val > best) { best = val; bi = i; }
            }
        wave_argmax(best, bi);
        if (lane == 0) { wbest[wave] = best; wbi[wave] = bi; }
        __syncthreads();
        if (tid == 0) {
            double bb = wbest[0];
            int ii = wbi[0];
            for (int x = 1; x < 4; ++x)
                if (wbest[x] > bb || (wbest[x] == bb && wbi[x] < ii)) { bb = wbest[x]; ii = wbi[x]; }
            if (ii >= n)  // every candidate is NaN: take the first unused row, flagged below
                for (int i = n - 1; i >= 0; --i)
                    if (used[i] == 0) ii = i;
            pivs[q] = ii;
            s_piv = P[ii * b + q];
            used[ii] = panel + 1;
        }
        __syncthreads();
        const int p = pivs[q];
        const double piv = s_piv;
        if (!(fabs(piv) > tiny) || !isfinite(piv)) bad = 1;
        la += log(fabs(piv));
        ng += piv < 0.0;
        for (int i = tid; i < n; i += kBlock) colk[i] = P[i * b + q];
        if (tid < b) rowp[tid] = P[p * b + tid];
        __syncthreads();
        const double ipiv = 1.0 / piv;
        for (int idx = tid; idx < n * b; idx += kBlock) {
            const int i = idx / b, j = idx % b;
            double val;
            if (i == p)
                val = (j == q) ? ipiv : rowp[j] * ipiv;
            else if (j == q)
                val = -colk[i] * ipiv;
            else
                val = P[idx] - colk[i] * rowp[j] * ipiv;
            P[idx] = val;
        }
        __syncthreads();
    }
    // old pivot rows (all columns; the panel columns of PR are not used)
    for (int q = 0; q < b; ++q) {
        const int p = pivs[q];
        for (int j = tid; j < n; j += kBlock) PR[((size_t)mat * b + q) * n + j] = Sm[(size_t)p * n + j];
    }
    __syncthreads();
    for (int idx = tid; idx < n * b; idx += kBlock) {
        const int i = idx / b, q = idx % b;
        Sm[(size_t)i * n + k0 + q] = P[idx];
    }
    for (int i = tid; i < n; i += kBlock) rs[i] = used[i];
    if (tid < b) pivrow[(size_t)mat * n + k0 + tid] = pivs[tid];
    if (tid == 0) {
        logabs[mat] += la;
        negs[mat] += ng;
        if (bad) status[mat] = 1;
    }
}

// Rank-b update of all non-panel columns: 64 x 64 output tile per workgroup.
__global__ __launch_bounds__(kBlock) void k_gj_update(double* __restrict__ S, const double* __restrict__ PR,
                                                       const int* __restrict__ rowstate, int n, int b, int k0,
                                                       int panel)
{
    __shared__ double Pt[64][33];   // panel rows i0..i0+63, q < b (b <= 32)
    __shared__ double Rt[32][65];   // pivot rows q < b, columns j0..j0+63
    const int tiles = (n + 63) / 64;
    const int mat = blockIdx.x / (tiles * tiles), t = blockIdx.x % (tiles * tiles);
    const int i0 = (t / tiles) * 64, j0 = (t % tiles) * 64;
    double* Sm = S + (size_t)mat * n * n;
    const int* rs = rowstate + (size_t)mat * n;
    const int tid = threadIdx.x;
    for (int idx = tid; idx < 64 * b; idx += kBlock) {
        const int r = idx / b, q = idx % b;
        Pt[r][q] = (i0 + r < n) ? Sm[(size_t)(i0 + r) * n + k0 + q] : 0.0;
    }
    for (int idx = tid; idx < b * 64; idx += kBlock) {
        const int q = idx / 64, c = idx % 64;
        Rt[q][c] = (j0 + c < n) ? PR[((size_t)mat * b + q) * n + j0 + c] : 0.0;
    }
    __syncthreads();
    // thread owns a 4 x 4 block: rows i0 + ty*4 + a, columns j0 + tx + 16 c
    const int ty = tid / 16, tx = tid % 16;
    double acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[a][c] = 0.0;
    for (int q = 0; q < b; ++q) {
        double pa[4], rc[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) pa[a] = Pt[ty * 4 + a][q];
#pragma unroll
        for (int c = 0; c < 4; ++c) rc[c] = Rt[q][tx + 16 * c];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int c = 0; c < 4; ++c) acc[a][c] += pa[a] * rc[c];
    }
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        const int i = i0 + ty * 4 + a;
        if (i >= n) continue;
        const bool pivot_row = rs[i] == panel + 1;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int j = j0 + tx + 16 * c;
            if (j >= n || (j >= k0 && j < k0 + b)) continue;
            const size_t o = (size_t)i * n + j;
            Sm[o] = (pivot_row ? 0.0 : Sm[o]) + acc[a][c];
        }
    }
}

// M[k][c] = S[pi(k)][pi^-1(c)], log|det|, sign, drift, status; one workgroup per matrix.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_gj_finish(CrowdView<T> v, const double* __restrict__ S,
                                                       const int* __restrict__ pivrow, int* __restrict__ rowstate,
                                                       const double* __restrict__ logabs,
                                                       const int* __restrict__ negs, const int* __restrict__ mstatus)
{
    extern __shared__ double rowbuf[];   // [n]
    int* inv_perm = (int*)(rowbuf + v.n);  // [n]
    const int mat = blockIdx.x, w = mat >> 1, spin = mat & 1, n = v.n, tid = threadIdx.x;
    const int* pr = pivrow + (size_t)mat * n;
    for (int k = tid; k < n; k += kBlock) inv_perm[pr[k]] = k;
    __syncthreads();
    const double* Sm = S + (size_t)mat * n * n;
    T* M = v.M + ((size_t)w * 2 + spin) * n * (size_t)n;
    for (int k = 0; k < n; ++k) {
        const double* src = Sm + (size_t)pr[k] * n;
        for (int j = tid; j < n; j += kBlock) rowbuf[j] = src[j];
        __syncthreads();
        for (int c = tid; c < n; c += kBlock) M[(size_t)k * n + c] = (T)rowbuf[inv_perm[c]];
        __syncthreads();
    }
    if (tid == 0) {
        int* seen = rowstate + (size_t)mat * n;  // reused as scratch: zero it
        for (int i = 0; i < n; ++i) seen[i] = 0;
        int parity = 0;
        for (int i = 0; i < n; ++i) {
            if (seen[i]) continue;
            int len = 0;
            for (int j = i; !seen[j]; j = pr[j]) { seen[j] = 1; ++len; }
            parity ^= (len - 1) & 1;
        }
        for (int i = 0; i < n; ++i) seen[i] = 0;
        const int sgn = ((negs[mat] + parity) & 1) ? -1 : 1;
        const double old = v.logdet[w * 2 + spin];
        v.drift[w * 2 + spin] = fabs(old - logabs[mat]);
        v.logdet[w * 2 + spin] = logabs[mat];
        v.sign[w * 2 + spin] = sgn;
        if (mstatus[mat]) atomicOr(&v.status[w], 1);
    }
}

__global__ void k_gj_reset(int* rowstate, double* logabs, int* negs, int* mstatus, unsigned long long* scale,
                           int nmat, int n)
{
    const size_t total = (size_t)nmat * n;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x)
        rowstate[i] = 0;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < (size_t)nmat; i += (size_t)gridDim.x * blockDim.x) {
        logabs[i] = 0.0;
        negs[i] = 0;
        mstatus[i] = 0;
        scale[i] = 0ull;
    }
}

int panel_width(int n) { return n > 1024 ? 8 : 16; }

size_t inverse_work_bytes(int nmat, int n)
{
    if (n <= kSmallN) return 0;
    const int b = panel_width(n);
    return (size_t)nmat * n * n * sizeof(double) + (size_t)nmat * b * n * sizeof(double)
           + (size_t)nmat * n * sizeof(int) * 2 + (size_t)nmat * (sizeof(double) + 2 * sizeof(int)) + 4096;
}

template <typename T>
void launch_inverse(const CrowdView<T>& v, const InvWork& wk, hipStream_t s)
{
    const int nmat = v.W * 2, n = v.n;
    if (n <= kSmallN) {
        hipLaunchKernelGGL(k_gj_small<T>, dim3(nmat), dim3(kBlock), 0, s, v);
        return;
    }
    const int tiles = (n + 63) / 64;
    int* rowstate = wk.pivrow + (size_t)nmat * n;
    int* mstatus = wk.negs + nmat;
    unsigned long long* scale = (unsigned long long*)(wk.logabs + nmat);
    hipLaunchKernelGGL(k_gj_reset, dim3(256), dim3(kBlock), 0, s, rowstate, wk.logabs, wk.negs, mstatus, scale,
                       nmat, n);
    hipLaunchKernelGGL(k_gj_load<T>, dim3(nmat * tiles * tiles), dim3(kBlock), 0, s, v, wk.S, scale);
    // panel width: the n x b panel plus a column and the row flags must fit in LDS
    const int bmax = panel_width(n);
    const size_t panel_lds = ((size_t)n * bmax + n) * sizeof(double) + (size_t)n * sizeof(int);
    (void)hipFuncSetAttribute((const void*)k_gj_panel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)panel_lds);
    for (int k0 = 0, panel = 0; k0 < n; k0 += bmax, ++panel) {
        const int b = min(bmax, n - k0);  // the last panel may be narrower
        hipLaunchKernelGGL(k_gj_panel, dim3(nmat), dim3(kBlock), panel_lds, s, wk.S, wk.PR, wk.pivrow, rowstate,
                           wk.logabs, wk.negs, mstatus, scale, n, b, k0, panel);
        hipLaunchKernelGGL(k_gj_update, dim3(nmat * tiles * tiles), dim3(kBlock), 0, s, wk.S, wk.PR, rowstate, n, b,
                           k0, panel);
    }
    const size_t fin_lds = (size_t)n * sizeof(double) + (size_t)n * sizeof(int);
    hipLaunchKernelGGL(k_gj_finish<T>, dim3(nmat), dim3(kBlock), fin_lds, s, v, wk.S, wk.pivrow, rowstate, wk.logabs,
                       wk.negs, mstatus);
}

template void launch_inverse<float>(const CrowdView<float>&, const InvWork&, hipStream_t);
template void launch_inverse<double>(const CrowdView<double>&, const InvWork&, hipStream_t);

}  // namespace cq
