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
// n  > 64: blocked on two levels.  A panel of b columns is swept by one workgroup
// per matrix (k_gj_panel, panel in registers); the same b sweeps act on every other
// column as the rank-b update
//     S[i][j] = [i not a pivot of the panel] S[i][j] + sum_q P[i][q] S_old[pi(k0+q)][j]
// with P the swept panel.  A block of B = 8b columns is swept panel by panel,
// each panel's update applied to the block's own columns only; the block's
// columns then hold the multipliers of all its B sweeps, and one rank-B update
// with the block's old pivot rows (k_gj_update) brings every other column up
// to date.  So the whole matrix is read and written n/B times, not n/b times;
// 2 n^3 flops in all.  S has a row stride of n + 16 doubles (s_ld).
#include "cq_device.h"
#include "cq_internal.h"

namespace cq {

constexpr int kSmallN = 64;

// argmax of |value| over the block (ties -> lowest index); returns in *best_i.
// One step of an argmax over lanes through a DPP lane pattern (no LDS): the larger value,
// the lower index on ties; every lane of the pattern has a source lane.
template <int CTRL>
__device__ __forceinline__ void argmax_dpp(double& val, int& idx)
{
    const long long bits = __double_as_longlong(val);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)bits, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(bits >> 32), CTRL, 0xF, 0xF, false);
    const int oi = __builtin_amdgcn_update_dpp(0, idx, CTRL, 0xF, 0xF, false);
    const double ov = __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
    if (ov > val || (ov == val && oi < idx)) {
        val = ov;
        idx = oi;
    }
}

// argmax over each row of 16 lanes, the result in all 16: quad_perm [1,0,3,2] and [2,3,0,1]
// combine the lanes of a quad, row_half_mirror the quads of a half row, row_mirror the halves
__device__ __forceinline__ void row_argmax(double& val, int& idx)
{
    argmax_dpp<0xB1>(val, idx);
    argmax_dpp<0x4E>(val, idx);
    argmax_dpp<0x141>(val, idx);
    argmax_dpp<0x140>(val, idx);
}

// argmax over the wave, the same result in every lane: rows by DPP, then the four rows'
// results read as wave-uniform values and combined in row order
__device__ __forceinline__ void wave_argmax_dpp(double& val, int& idx)
{
    row_argmax(val, idx);
    const long long bits = __double_as_longlong(val);
    double bv = 0.0;
    int bi = 0;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int lo = __builtin_amdgcn_readlane((int)bits, 16 * r);
        const int hi = __builtin_amdgcn_readlane((int)(bits >> 32), 16 * r);
        const int oi = __builtin_amdgcn_readlane(idx, 16 * r);
        const double ov = __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
        if (r == 0 || ov > bv || (ov == bv && oi < bi)) {
            bv = ov;
            bi = oi;
        }
    }
    val = bv;
    idx = bi;
}

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
    const T* A = v.VGL + ((size_t)w * 2 + spin) * n * (size_t)v.arow;
    __shared__ double smax[4];
    double amax = 0.0;
    for (int idx = tid; idx < n * n; idx += kBlock) {
        const int i = idx / n, j = idx % n;  // A[i][j] = phi_j(r_i)
        const double a = (double)A[(size_t)i * v.arow + j];
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
        const double d = fabs(old - logabs);
        v.drift[w * 2 + spin] = d;
        if (v.drift_max) atomicMax(v.drift_max, (unsigned long long)__double_as_longlong(isfinite(d) ? d : INFINITY));
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
    const T* A = v.VGL + ((size_t)w * 2 + spin) * n * (size_t)v.arow;
    double amax = 0.0;
    for (int idx = threadIdx.x; idx < 64 * 64; idx += kBlock) {
        const int r = idx / 64, c = idx % 64;
        const int i = ti * 64 + r, j = tj * 64 + c;
        const double a = (i < n && j < n) ? (double)A[(size_t)i * v.arow + j] : 0.0;
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
    double* Sm = S + (size_t)mat * n * s_ld(n);
    for (int idx = threadIdx.x; idx < 64 * 64; idx += kBlock) {
        const int r = idx / 64, c = idx % 64;  // output row j = tj*64 + r, column i = ti*64 + c
        const int j = tj * 64 + r, i = ti * 64 + c;
        if (i < n && j < n) Sm[(size_t)j * s_ld(n) + i] = tile[c][r];
    }
}

// Sweep the b panel columns k0 .. k0+b-1 of every matrix (b <= BP; one workgroup per
// matrix), record the pivots, copy the old pivot rows.  The panel lives in registers:
// thread t of TH holds rows t, t + TH, ... (R of them) with their b panel columns, so a sweep
// is a wave argmax, one barrier and a rank-1 update of the thread's own rows.  Each
// wave hands its candidate pivot row to the others through LDS with its argmax, and
// the LDS slots alternate with the parity of the sweep, so one barrier per sweep is
// enough.  Pivot choice: the largest |B[i][k]| among the unused rows, the lowest index
// on ties; rows whose entry is NaN rank below every number, so a column of NaNs still
// takes the first unused row (and is flagged).
// The old pivot rows go to rows pr0 .. pr0+b-1 of the matrix's pr_rows-row block of PR.
template <int TH, int R, int BP>
__global__ __launch_bounds__(TH) void k_gj_panel(double* __restrict__ S, double* __restrict__ PR,
                                                             int* __restrict__ pivrow, int* __restrict__ rowstate,
                                                             double* __restrict__ logabs, int* __restrict__ negs,
                                                             int* __restrict__ status,
                                                             const unsigned long long* __restrict__ scale, int n,
                                                             int b, int k0, int panel, int pr_rows, int pr0)
{
    constexpr int kPanelThreads = TH, kPanelWaves = TH / 64;
    __shared__ double wrow[2][kPanelWaves][BP];  // each wave's candidate pivot row
    __shared__ double wval[2][kPanelWaves];
    __shared__ int widx[2][kPanelWaves];
    __shared__ int pivs[BP];
    __shared__ double spiv[BP], slog[BP];
    const int mat = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    double* Sm = S + (size_t)mat * n * s_ld(n);
    int* rs = rowstate + (size_t)mat * n;
    // the panel is read and written in whole row segments (a wave covers 64 / BP rows per
    // access) and handed to the row-per-thread layout through LDS
    extern __shared__ double ptile[];  // [R TH][BP + 1]
    constexpr int LD = BP + 1;
    static_assert((R * BP) % 8 == 0, "panel loads");
#pragma unroll
    for (int h = 0; h < R * BP; h += 8) {  // 8 loads in flight per thread
        double y[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int idx = tid + (h + u) * kPanelThreads, row = idx / BP, col = idx % BP;
            y[u] = (row < n && col < b) ? Sm[(size_t)row * s_ld(n) + k0 + col] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int idx = tid + (h + u) * kPanelThreads;
            ptile[(idx / BP) * LD + idx % BP] = y[u];
        }
    }
    __syncthreads();
    double x[R][BP];
    int used[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int i = tid + r * kPanelThreads;
        used[r] = i < n ? rs[i] : 1;
#pragma unroll
        for (int j = 0; j < BP; ++j) x[r][j] = ptile[i * LD + j];
    }
    const double tiny = n * 2.220446049250313e-16 * __longlong_as_double((long long)scale[mat]);
    int ng = 0, bad = 0;
#pragma unroll
    for (int q = 0; q < BP; ++q) {
        if (q >= b) continue;  // b is uniform; a constant trip count keeps the loop fully unrolled
        const int par = q & 1;
        double best = -1.0;
        int bi = n;
#pragma unroll
        for (int r = 0; r < R; ++r)
            if (used[r] == 0) {
                const double a = fabs(x[r][q]);
                const double key = a == a ? a : -0.5;
                if (key > best) {
                    best = key;
                    bi = tid + r * kPanelThreads;
                }
            }
        wave_argmax_dpp(best, bi);
#pragma unroll
        for (int r = 0; r < R; ++r)
            if (tid + r * kPanelThreads == bi)
#pragma unroll
                for (int j = 0; j < BP; ++j) wrow[par][wave][j] = x[r][j];
        if (lane == 0) {
            wval[par][wave] = best;
            widx[par][wave] = bi;
        }
        __syncthreads();
        // every lane takes one wave's candidate (a row of lanes repeats them when there are
        // fewer than 16 waves) and the row argmax combines them, the same result in every lane;
        // some row is always unused, since a matrix has n rows and n sweeps
        static_assert(kPanelWaves <= 16 && (kPanelWaves & (kPanelWaves - 1)) == 0, "candidate rows");
        double bb = wval[par][lane & (kPanelWaves - 1)];
        int p = widx[par][lane & (kPanelWaves - 1)];
        row_argmax(bb, p);
        const int ww = (p % kPanelThreads) >> 6;  // the wave holding row p sent it
        const double* rowp = wrow[par][ww];  // read from LDS where used (broadcast)
        const double piv = rowp[q];
        if (tid == 0) {  // the logarithms are taken after the sweeps, off their chain
            if (!(fabs(piv) > tiny) || !isfinite(piv)) bad = 1;
            spiv[q] = piv;
            ng += piv < 0.0;
        }
        const double ipiv = 1.0 / piv;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (tid + r * kPanelThreads == p) {
#pragma unroll
                for (int j = 0; j < BP; ++j) x[r][j] = (j == q) ? ipiv : rowp[j] * ipiv;
                used[r] = panel + 1;
            } else {
                const double c = x[r][q];
#pragma unroll
                for (int j = 0; j < BP; ++j) x[r][j] = (j == q) ? -c * ipiv : x[r][j] - c * rowp[j] * ipiv;
            }
        }
        if (tid == 0) pivs[q] = p;
    }
    // the swept panel back to the LDS tile (the registers are free from here on)
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int i = tid + r * kPanelThreads;
#pragma unroll
        for (int j = 0; j < BP; ++j) ptile[i * LD + j] = x[r][j];
        if (i < n) rs[i] = used[r];
    }
    __syncthreads();
    if (tid < b) slog[tid] = log(fabs(spiv[tid]));
    // old pivot rows (all columns; the panel columns of PR are not used)
    for (int i0 = 0; i0 < n * b; i0 += 8 * kPanelThreads) {  // 8 loads in flight per thread
        double y[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int idx = i0 + u * kPanelThreads + tid;
            y[u] = idx < n * b ? Sm[(size_t)pivs[idx / n] * s_ld(n) + idx % n] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int idx = i0 + u * kPanelThreads + tid;
            if (idx < n * b) PR[((size_t)mat * pr_rows + pr0 + idx / n) * n + idx % n] = y[u];
        }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < R * BP; ++u) {
        const int idx = tid + u * kPanelThreads, row = idx / BP, col = idx % BP;
        if (row < n && col < b) Sm[(size_t)row * s_ld(n) + k0 + col] = ptile[row * LD + col];
    }
    if (tid < b) pivrow[(size_t)mat * n + k0 + tid] = pivs[tid];
    if (tid == 0) {
        double la = 0.0;
        for (int q = 0; q < b; ++q) la += slog[q];  // in sweep order
        logabs[mat] += la;
        negs[mat] += ng;
        if (bad) status[mat] = 1;
    }
}

// Rank-b update of the columns j in [jlo, jhi) outside [xlo, xhi), for the column tiles
// jt0 .. jt0+njt-1: 64 x 64 output tile per workgroup (4 waves), the b multipliers and
// old pivot rows staged through LDS KC at a time (the next chunk's loads in flight during
// the current chunk's products; small chunks leave room for 4 workgroups per CU).  The
// multipliers are S's columns k0 .. k0+b-1, the old pivot rows are rows pr0 .. pr0+b-1 of
// PR's pr_rows-row block, and the pivot rows of the update are the rows whose state lies
// in (plo, phi] (state = panel index + 1).  The tiles of one matrix run on one XCD, so
// the operands they share stay in that XCD's L2.
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <int KC>
__global__ __launch_bounds__(kBlock) void k_gj_update(double* __restrict__ S, const double* __restrict__ PR,
                                                       const int* __restrict__ rowstate, int nmat, int n, int b,
                                                       int k0, int pr_rows, int pr0, int plo, int phi, int jt0,
                                                       int njt, int jlo, int jhi, int xlo, int xhi)
{
    __shared__ double Pt[64][KC + 1];  // multiplier rows i0..i0+63, one chunk of q
    // one chunk of old pivot rows, columns j0..j0+63; a row stride of 80 doubles puts the
    // four q rows of an operand read in two halves of the LDS banks (65 gave 4-way conflicts)
    __shared__ double Rt[KC][80];
    const int tiles = (n + 63) / 64;
    int mat, t;
    xcd_map(blockIdx.x, tiles * njt, mat, t);
    if (mat >= nmat) return;
    const int i0 = (t / njt) * 64, j0 = (jt0 + t % njt) * 64;
    double* Sm = S + (size_t)mat * n * s_ld(n);
    const int* rs = rowstate + (size_t)mat * n;
    const int tid = threadIdx.x;
    // FP64 matrix cores (v_mfma_f64_16x16x4f64): wave wv owns the 32 x 32 quarter
    // (rows 32 (wv / 2), columns 32 (wv % 2)) as 2 x 2 blocks of 16 x 16.  Lane l
    // supplies A[l % 16][l / 16] and B[l / 16][l % 16] of a step of 4 q values and
    // holds D[l / 16 + 4 v][l % 16]; operands past b are zero.
    const int lane = tid & 63, wv = tid >> 6;
    const int r16 = lane & 15, q4 = lane >> 4;
    const int wi = (wv >> 1) * 32, wj = (wv & 1) * 32;
    constexpr int U = 64 * KC / kBlock;
    static_assert(U * kBlock == 64 * KC, "chunk loads");
    double xp[U], xr[U];
    auto load_chunk = [&](int kc) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int idx = tid + u * kBlock;
            const int r = idx / KC, q = idx % KC, qr = idx / 64, c = idx % 64;
            xp[u] = (kc + q < b && i0 + r < n) ? Sm[(size_t)(i0 + r) * s_ld(n) + k0 + kc + q] : 0.0;
            xr[u] = (kc + qr < b && j0 + c < n) ? PR[((size_t)mat * pr_rows + pr0 + kc + qr) * n + j0 + c] : 0.0;
        }
    };
    f64x4 acc[2][2];
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) acc[bi][bj] = f64x4{0.0, 0.0, 0.0, 0.0};
    auto stage = [&](bool first) {
        if (!first) __syncthreads();  // the previous chunk's products are done with the LDS
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int idx = tid + u * kBlock;
            Pt[idx / KC][idx % KC] = xp[u];
            Rt[idx / 64][idx % 64] = xr[u];
        }
        __syncthreads();
    };
    auto products = [&]() {
#pragma unroll
        for (int q0 = 0; q0 < KC; q0 += 4) {
            const double a0 = Pt[wi + r16][q0 + q4], a1 = Pt[wi + 16 + r16][q0 + q4];
            const double b0 = Rt[q0 + q4][wj + r16], b1 = Rt[q0 + q4][wj + 16 + r16];
            acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
            acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
            acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
            acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
        }
    };
    // every chunk but the last: the next chunk's loads in flight during the products
    const int nch = (b + KC - 1) / KC;
    load_chunk(0);
    for (int c = 0; c + 1 < nch; ++c) {
        stage(c == 0);
        load_chunk((c + 1) * KC);
        products();
    }
    stage(nch == 1);
    // the tile's old values, in flight during the last chunk's products
    double old[2][2][4];
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int i = i0 + wi + 16 * bi + q4 + 4 * v;
#pragma unroll
            for (int bj = 0; bj < 2; ++bj) {
                const int j = j0 + wj + 16 * bj + r16;
                const bool live = i < n && j < n && j >= jlo && j < jhi && !(j >= xlo && j < xhi);
                old[bi][bj][v] = live ? Sm[(size_t)i * s_ld(n) + j] : 0.0;
            }
        }
    products();
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int i = i0 + wi + 16 * bi + q4 + 4 * v;
            if (i >= n) continue;
            const bool pivot_row = rs[i] > plo && rs[i] <= phi;
#pragma unroll
            for (int bj = 0; bj < 2; ++bj) {
                const int j = j0 + wj + 16 * bj + r16;
                if (j >= n || j < jlo || j >= jhi || (j >= xlo && j < xhi)) continue;
                Sm[(size_t)i * s_ld(n) + j] = (pivot_row ? 0.0 : old[bi][bj][v]) + acc[bi][bj][v];
            }
        }
}

// M[k][c] = S[pi(k)][pi^-1(c)] for kFinRows rows k per workgroup (reads gathered within a row of
// S, writes coalesced); the first workgroup of each matrix also forms log|det|, the sign (the
// parity of pi counted as the parity of its inversions, in parallel from LDS), the drift and the
// status.
constexpr int kFinRows = 16;

template <typename T>
__global__ __launch_bounds__(kBlock) void k_gj_finish(CrowdView<T> v, const double* __restrict__ S,
                                                       const int* __restrict__ pivrow,
                                                       const double* __restrict__ logabs,
                                                       const int* __restrict__ negs, const int* __restrict__ mstatus)
{
    extern __shared__ int fin_sh[];
    int* inv_perm = fin_sh;     // [n]
    int* prl = fin_sh + v.n;    // [n]
    __shared__ int wpar[kBlock / 64];
    const int n = v.n, tid = threadIdx.x, parts = (n + kFinRows - 1) / kFinRows;
    const int mat = blockIdx.x / parts, part = blockIdx.x % parts, w = mat >> 1, spin = mat & 1;
    const int* pr = pivrow + (size_t)mat * n;
    for (int k = tid; k < n; k += kBlock) {
        const int p = pr[k];
        prl[k] = p;
        inv_perm[p] = k;
    }
    __syncthreads();
    const double* Sm = S + (size_t)mat * n * s_ld(n);
    T* M = v.M + ((size_t)w * 2 + spin) * n * (size_t)n;
    // two rows at a time, every load of both in flight before the stores (n <= 8 kBlock)
    for (int kk = 0; kk < kFinRows; kk += 2) {
        double x[2][8];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int k = part * kFinRows + kk + h;
            const double* src = Sm + (size_t)prl[k < n ? k : 0] * s_ld(n);
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int c = tid + u * kBlock;
                x[h][u] = (k < n && c < n) ? src[inv_perm[c]] : 0.0;
            }
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int k = part * kFinRows + kk + h;
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int c = tid + u * kBlock;
                if (k < n && c < n) M[(size_t)k * n + c] = (T)x[h][u];
            }
        }
    }
    if (part != 0) return;
    int par = 0;
    for (int i = tid; i < n; i += kBlock) {
        const int pi = prl[i];
        for (int j = i + 1; j < n; ++j) par ^= prl[j] < pi;
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) par ^= __shfl_xor(par, off, 64);
    if ((tid & 63) == 0) wpar[tid >> 6] = par;
    __syncthreads();
    if (tid == 0) {
        int parity = 0;
        for (int x = 0; x < kBlock / 64; ++x) parity ^= wpar[x];
        const int sgn = ((negs[mat] + parity) & 1) ? -1 : 1;
        const double old = v.logdet[w * 2 + spin];
        const double d = fabs(old - logabs[mat]);
        v.drift[w * 2 + spin] = d;
        if (v.drift_max) atomicMax(v.drift_max, (unsigned long long)__double_as_longlong(isfinite(d) ? d : INFINITY));
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
static size_t panel_lds(int th, int r, int bp) { return (size_t)th * r * (bp + 1) * sizeof(double); }
int block_width(int n) { return 8 * panel_width(n); }

size_t inverse_work_bytes(int nmat, int n)
{
    if (n <= kSmallN) return 0;
    const int B = block_width(n);
    return (size_t)nmat * n * s_ld(n) * sizeof(double) + (size_t)nmat * B * n * sizeof(double)
           + (size_t)nmat * n * sizeof(int) * 2 + (size_t)nmat * (sizeof(double) + 2 * sizeof(int)) + 4096;
}

template <typename T>
void launch_inverse(const CrowdView<T>& v, const InvWork& wk, hipStream_t s, int nmat)
{
    if (nmat < 0) nmat = v.W * 2;
    const int n = v.n;
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
    const int bmax = panel_width(n);
    const int B = block_width(n), per_block = B / bmax;
    static bool panel_attr = false;  // the panels' LDS tiles exceed the default 64 KB
    if (!panel_attr) {
        (void)hipFuncSetAttribute((const void*)k_gj_panel<512, 1, 16>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)panel_lds(512, 1, 16));
        (void)hipFuncSetAttribute((const void*)k_gj_panel<1024, 1, 16>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)panel_lds(1024, 1, 16));
        (void)hipFuncSetAttribute((const void*)k_gj_panel<1024, 2, 8>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)panel_lds(1024, 2, 8));
        panel_attr = true;
    }
    static_assert(kBlock == 256, "update tiles");
    const int mat_groups = ((nmat + 7) / 8) * 8;  // update grids: the tiles of a matrix on one XCD
    for (int K0 = 0, blk = 0; K0 < n; K0 += B, ++blk) {
        const int Bw = min(B, n - K0);  // the last block may be narrower
        const int plo = blk * per_block;
        int np = 0;
        for (int k0 = K0; k0 < K0 + Bw; k0 += bmax, ++np) {
            const int b = min(bmax, K0 + Bw - k0), panel = plo + np;
            if (n <= 512)
                hipLaunchKernelGGL((k_gj_panel<512, 1, 16>), dim3(nmat), dim3(512), panel_lds(512, 1, 16), s, wk.S,
                                   wk.PR, wk.pivrow, rowstate, wk.logabs, wk.negs, mstatus, scale, n, b, k0, panel, B,
                                   np * bmax);
            else if (n <= 1024)
                hipLaunchKernelGGL((k_gj_panel<1024, 1, 16>), dim3(nmat), dim3(1024), panel_lds(1024, 1, 16), s,
                                   wk.S, wk.PR, wk.pivrow, rowstate, wk.logabs, wk.negs, mstatus, scale, n, b, k0,
                                   panel, B, np * bmax);
            else
                hipLaunchKernelGGL((k_gj_panel<1024, 2, 8>), dim3(nmat), dim3(1024), panel_lds(1024, 2, 8), s, wk.S,
                                   wk.PR, wk.pivrow, rowstate, wk.logabs, wk.negs, mstatus, scale, n, b, k0, panel,
                                   B, np * bmax);
            if (Bw > b) {  // the panel's sweeps on the rest of the block
                const int jt0 = K0 / 64, njt = (K0 + Bw - 1) / 64 - jt0 + 1;
                hipLaunchKernelGGL(k_gj_update<16>, dim3(mat_groups * tiles * njt), dim3(kBlock), 0, s, wk.S, wk.PR,
                                   rowstate, nmat, n, b, k0, B, np * bmax, panel, panel + 1, jt0, njt, K0, K0 + Bw,
                                   k0, k0 + b);
            }
        }
        if (n > Bw)  // the block's sweeps on every other column, as one rank-Bw update
            hipLaunchKernelGGL(k_gj_update<16>, dim3(mat_groups * tiles * tiles), dim3(kBlock), 0, s, wk.S, wk.PR,
                               rowstate, nmat, n, Bw, K0, B, 0, plo, plo + np, 0, tiles, 0, n, K0, K0 + Bw);
    }
    const size_t fin_lds = (size_t)2 * n * sizeof(int);
    hipLaunchKernelGGL(k_gj_finish<T>, dim3(nmat * ((n + kFinRows - 1) / kFinRows)), dim3(kBlock), fin_lds, s, v, wk.S,
                       wk.pivrow, wk.logabs, wk.negs, mstatus);
}

template void launch_inverse<float>(const CrowdView<float>&, const InvWork&, hipStream_t, int);
template void launch_inverse<double>(const CrowdView<double>&, const InvWork&, hipStream_t, int);

}  // namespace cq
