// Per-move kernels of the batched particle-by-particle move (the propose, ratio,
// derivative and accept steps of Alg. 1 applied to every walker of a crowd in
// lock-step, Alg. 3/4):
//
//   k_move       one launch per move e: B-spline value/gradient/Laplacian
//                at the proposal r'_e for one orbital chunk, the chunk's partial
//                dot products with the inverse column and the delayed-update
//                window, a slice of the Jastrow sums; fused with the ratio and
//                decision of the previous move and the proposal of the
//                next one.  Grid: walkers x chunks.
//
// Orbital tables are [G][G][G][n_orb] with the orbital index fastest, so the 64
// stencil points of one walker are 64 contiguous runs of n_orb elements (16
// runs of 4 consecutive z-points): each lane loads 16 bytes per point,
// coalesced along orbitals.  Four waves split the 4 x-planes of the stencil;
// their partial sums meet in LDS in a fixed order (bit-reproducible results,
// independent of how walkers are grouped into crowds).
#include <algorithm>

#include "cq_device.h"
#include "cq_internal.h"
#include "cq_jastrow.h"

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

// Ratio and decision of move `prev` of walker w, by one wave.  The window's
// accepted moves m = 0 .. cnt-1 (rows u_m, columns c_m taken just before move m,
// ratios rho_m) act on the old column c0_e of e as a sequence of rank-1 updates:
//   c_e = c0_e - sum_m beta_m c_m,  beta_m = (u_m . c0_e - sum_{j<m} beta_j u_m . c_j) / rho_m
// (forward substitution with wG[m][j] = u_m . c_j), so
//   rho_D = u . c0_e - sum_m beta_m (u . c_m).
// This applies the window's updates in order, as Sherman-Morrison would, and is as
// accurate; it avoids the explicit inverse of the k x k window matrix, whose
// conditioning degrades when a small ratio enters the window.
// Leaves beta in sbeta[0 .. cnt-1]; returns the decision (lane-uniform).  When
// `owner` is set the wave also writes the walker's state (position, log|det|,
// sign, counters, window bookkeeping and the per-move records).
template <typename T>
__device__ int resolve_wave(const CrowdView<T>& v, int w, int prev, int cnt, bool owner, double* sbeta,
                            double* sG /*[kMaxDelay][kMaxDelay]*/)
{
    constexpr int CH = chunk_orbitals<T>();
    constexpr int kMaxChunks = 2048 / CH;
    const int lane = threadIdx.x & 63;
    const int n = v.n, K = v.K, NP = part_stride(K), J2 = part_j2(K);
    const int C = (n + CH - 1) / CH;
    const int spin = prev >= n, a = prev - spin * n;
    const double* part = v.part + (size_t)(prev & 1) * v.W * C * NP + (size_t)w * C * NP;
    // every load first (partials over chunks in a fixed order, window rows, ratios)
    double x_l = 0.0, y_l = 0.0, d0 = 0.0, dj = 0.0;
    const bool mine = lane < cnt;
#pragma unroll
    for (int c = 0; c < kMaxChunks; ++c) {
        if (c < C) {
            const double* pc = part + (size_t)c * NP;
            d0 += pc[0];
            dj += pc[J2];
            if (mine) {
                x_l += pc[4 + 5 * lane];      // u . c_lane
                y_l += pc[4 + 5 * lane + 4];  // u_lane . c0
            }
        }
    }
    const double* wG = v.wG + (size_t)w * K * K;
#pragma unroll
    for (int r = 0; r < kMaxDelay * kMaxDelay / 64; ++r) {
        const int idx = lane + 64 * r, i = idx / kMaxDelay, j = idx % kMaxDelay;
        if (i < cnt && j < i) sG[idx] = wG[i * K + j];
    }
    const double rinv = mine ? 1.0 / v.wrho[(size_t)w * K + lane] : 0.0;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    // forward substitution: lane i carries t_i = y_i - sum_{j<m} beta_j wG[i][j]
    double t = y_l, my_beta = 0.0;
    for (int mm = 0; mm < cnt; ++mm) {
        const double bm = dpp::lane(t, mm) * dpp::lane(rinv, mm);
        if (lane == mm) my_beta = bm;
        if (lane > mm && mine) t -= bm * sG[lane * kMaxDelay + mm];
    }
    if (mine) sbeta[lane] = my_beta;
    const double r0 = wave_sum(mine ? my_beta * x_l : 0.0);
    const double rho = d0 - r0;
    const double prob = rho * rho * exp(2.0 * dj);
    const uint32_t step = v.prm->step;
    const double u = accept_uniform(v.seed, v.uid[w], step, (uint32_t)prev);
    int acc = u < prob;
    const int rs = v.prm->rec_sweep;
    const size_t ri = ((size_t)rs * v.ne + prev) * v.Wcap + w;
    if (v.forced && rs < v.prm->forced_cap && v.forced[ri] < 2) acc = v.forced[ri] != 0;
    if (owner) {
        if (lane == 0 && rs < v.prm->rec_cap) {
            v.rec_rho[ri] = rho;
            v.rec_dlnj[ri] = dj;
            v.rec_prob[ri] = prob;
            v.rec_acc[ri] = (uint8_t)acc;
        }
        if (acc) {
            if (mine) {
                v.beta[(size_t)w * K + lane] = my_beta;
                v.wG[((size_t)w * K + cnt) * K + lane] = x_l;  // u . c_lane
            }
            if (lane == 0) {
                v.wrho[(size_t)w * K + cnt] = rho;
                v.welec[(size_t)w * K + cnt] = a;
                v.wslot[(size_t)w * K + cnt] = cnt;
                const double* rp = v.rnew + ((size_t)(prev & 3) * v.W + w) * 3;
                for (int k = 0; k < 3; ++k) v.R[((size_t)w * v.ne + prev) * 3 + k] = rp[k];
                v.logdet[w * 2 + spin] += log(fabs(rho));
                if (rho < 0.0) v.sign[w * 2 + spin] = -v.sign[w * 2 + spin];
                v.nacc[w] += 1;
            }
        }
        if (lane == 0) v.nprop[w] += 1;
    }
    return acc;
}

// The proposal of move e at the current step: r' = wrap(r_e + sigma z).
template <typename T>
__device__ __forceinline__ void propose(const CrowdView<T>& v, int w, int e, uint32_t step, double rp[3])
{
    double z[3];
    gauss3(v.seed, v.uid[w], step, (uint32_t)e, z);
    const double sigma = v.prm->sigma;
    for (int k = 0; k < 3; ++k) rp[k] = wrap_box(v.R[((size_t)w * v.ne + e) * 3 + k] + sigma * z[k], v.L);
}

// One kernel per move, grid = walkers x orbital chunks.  Workgroup (w, c):
//   1. loads the proposal r'_e (made one kernel earlier: it does not depend on
//      the previous decision) and issues the B-spline gather of its chunk;
//   2. while that is in flight, resolves move `prev` (ratio, decision) from the
//      previous kernel's partial sums -- every workgroup of the walker computes the
//      same result, chunk 0 writes the state;
//   3. brings the column of `prev` up to date if it was accepted (its chunk),
//      finishes the value/gradient/Laplacian, the dots with the inverse column
//      and the window, a slice of the Jastrow sums, and writes its partials;
//   4. chunk 0 makes the proposal of the next move.
// e = -1: only steps 2-3 (end of a window).  prev = -1: nothing to resolve.
// Partial sums and the window count seen by a move alternate between two
// buffers by move parity (cnt[e & 1][w]) and proposals rotate over four, so no
// buffer is read and written by one launch; the final count of a window goes to
// cnt[2][w] for the update.  Counts read back are range-checked: a count outside
// 0 .. k-1 sets bit 2 of status[w] and is clamped, so no slot index can leave
// its buffer.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_move(CrowdView<T> v, int e, int prev, int reset)
{
    constexpr int VEC = 16 / sizeof(T);
    constexpr int CH = 64 * VEC;
    __shared__ T red[4 * 5 * CH];
    __shared__ T row[5 * CH];
    __shared__ double jred[4][4];
    __shared__ double sbeta[kMaxDelay];
    __shared__ double sG[kMaxDelay * kMaxDelay];
    __shared__ int s_acc;
    const int C = (v.n + CH - 1) / CH;
    int w, c;
    xcd_map(blockIdx.x, C, w, c);
    if (w >= v.W) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int n = v.n, K = v.K, NP = part_stride(K);
    int cnt0 = reset || prev < 0 ? 0 : v.cnt[(size_t)(prev & 1) * v.W + w];
    if (cnt0 < 0 || cnt0 >= K) {
        if (tid == 0) atomicOr(&v.status[w], 2);
        cnt0 = cnt0 < 0 ? 0 : K - 1;
    }
    const int j0 = c * CH + lane * VEC;
    const bool valid = j0 < n;

    // 1. proposal and gather of this chunk
    double rp[3] = {0.0, 0.0, 0.0};
    T vals[16][VEC];
    AxisW<T> ax, ay, az;
    if (e >= 0) {
        const double* rq = v.rnew + ((size_t)(e & 3) * v.W + w) * 3;
        rp[0] = rq[0]; rp[1] = rq[1]; rp[2] = rq[2];
        ax = axis_weights<T>(rp[0], v.L, v.G);
        ay = axis_weights<T>(rp[1], v.L, v.G);
        az = axis_weights<T>(rp[2], v.L, v.G);
        if (valid) {
            const int G = v.G;
            const int jx = (ax.i0 + wave + G - 1) % G;
            int jy[4], jz[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                jy[q] = (ay.i0 + q + G - 1) % G;
                jz[q] = (az.i0 + q + G - 1) % G;
            }
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const size_t pt = ((size_t)jx * G + jy[q >> 2]) * G + jz[q & 3];
                load16(v.table + pt * v.n_orb + j0, vals[q]);
            }
        }
    }

    // 2. resolve the previous move
    int acc = 0;
    if (prev >= 0) {
        if (wave == 0) {
            const int a = resolve_wave<T>(v, w, prev, cnt0, c == 0, sbeta, sG);
            if (lane == 0) s_acc = a;
        }
        __syncthreads();
        acc = s_acc;
    }
    int cnt = cnt0 + acc;  // window size seen by move e (or the final size when e = -1)
    if (c == 0 && tid == 0) v.cnt[(size_t)(e < 0 ? 2 : (e & 1)) * v.W + w] = cnt;
    if (e >= 0 && cnt >= K) {  // a move never sees a full window
        if (tid == 0) atomicOr(&v.status[w], 2);
        cnt = K - 1;
    }

    // 3a. the accepted previous move's column: c = c0 - sum_m beta_m c_m (this chunk)
    if (acc && cnt0 > 0 && valid && wave == (cnt0 & 3)) {
        T cn[VEC];
        load16(v.Cbuf + ((size_t)w * K + cnt0) * n + j0, cn);
        for (int mm = 0; mm < cnt0; ++mm) {
            T cm[VEC];
            load16(v.Cbuf + ((size_t)w * K + mm) * n + j0, cm);
            const T bm = (T)sbeta[mm];
#pragma unroll
            for (int i = 0; i < VEC; ++i) cn[i] -= bm * cm[i];
        }
        store16(v.Cbuf + ((size_t)w * K + cnt0) * n + j0, cn);
    }
    if (e < 0) return;

    const int spin = e >= n, a = e - spin * n;
    double* P = v.part + (size_t)(e & 1) * v.W * C * NP + ((size_t)w * C + c) * NP;

    // 3b. value, gradient, Laplacian of the chunk
    {
        T bxa, dxa, d2xa;
        pick_plane(ax, wave, bxa, dxa, d2xa);
        T accv[5][VEC];
#pragma unroll
        for (int k = 0; k < 5; ++k)
#pragma unroll
            for (int i = 0; i < VEC; ++i) accv[k][i] = (T)0;
        if (valid) {
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
                    accv[0][i] += wv * p;
                    accv[1][i] += wgx * p;
                    accv[2][i] += wgy * p;
                    accv[3][i] += wgz * p;
                    accv[4][i] += wl * p;
                }
            }
        }
#pragma unroll
        for (int k = 0; k < 5; ++k)
#pragma unroll
            for (int i = 0; i < VEC; ++i) red[(wave * 5 + k) * CH + lane * VEC + i] = accv[k][i];
    }
    __syncthreads();
    if (tid < CH) {
#pragma unroll
        for (int k = 0; k < 5; ++k)
            row[k * CH + tid] = ((red[(0 * 5 + k) * CH + tid] + red[(1 * 5 + k) * CH + tid]) +
                                 red[(2 * 5 + k) * CH + tid]) + red[(3 * 5 + k) * CH + tid];
    }
    __syncthreads();

    // 3c. dots with the old column c0_e and with the window
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
        for (int k = wave; k < 5; k += 4) store16(v.stage + (((size_t)w * v.QR + cnt) * 5 + k) * n + j0, rv[k]);
    }
    // products in T, sums in FP64.  The Metropolis step needs u . c0_e and, per
    // window slot, u . c_m and u_m . c0_e; every wave takes the slots m = wave
    // (mod 4), loads them all, then reduces.
    {
        double d = 0.0;
#pragma unroll
        for (int i = 0; i < VEC; ++i) d += (double)(rv[0][i] * m[i]);
        d = wave_sum(d);
        if (wave == 0 && lane == 0) P[0] = d;
    }
    constexpr int kSlots = kMaxDelay / 4;
#pragma unroll
    for (int half = 0; half < 2; ++half) {
        T cn[kSlots / 2][VEC], un[kSlots / 2][VEC];
#pragma unroll
        for (int q = 0; q < kSlots / 2; ++q) {
            const int nn = wave + 4 * (q + half * kSlots / 2);
#pragma unroll
            for (int i = 0; i < VEC; ++i) { cn[q][i] = (T)0; un[q][i] = (T)0; }
            if (nn < cnt && valid) {
                load16(v.Cbuf + ((size_t)w * K + nn) * n + j0, cn[q]);
                load16(v.stage + (((size_t)w * v.QR + nn) * 5 + 0) * n + j0, un[q]);
            }
        }
#pragma unroll
        for (int q = 0; q < kSlots / 2; ++q) {
            const int nn = wave + 4 * (q + half * kSlots / 2);
            if (nn < cnt) {  // wave-uniform
                double x = 0.0, y = 0.0;
#pragma unroll
                for (int i = 0; i < VEC; ++i) {
                    x += (double)(rv[0][i] * cn[q][i]);
                    y += (double)(m[i] * un[q][i]);
                }
                x = wave_sum(x);
                y = wave_sum(y);
                if (lane == 0) {
                    P[4 + 5 * nn] = x;
                    P[4 + 5 * nn + 4] = y;
                }
            }
        }
    }

    // 3d. Jastrow: this workgroup's slice of the other electrons (the previous
    // move's electron sits at its proposal if that was accepted)
    double jv[4] = {0.0, 0.0, 0.0, 0.0};
    if (v.use_j2) {
        double re[3];
        for (int k = 0; k < 3; ++k) re[k] = v.R[((size_t)w * v.ne + e) * 3 + k];
        const double* rprev = v.rnew + ((size_t)((prev < 0 ? 0 : prev) & 3) * v.W + w) * 3;
        const int per = (v.ne + C - 1) / C;
        const int lo = c * per, hi = min(v.ne, lo + per);
        for (int mm = lo + tid; mm < hi; mm += kBlock) {
            if (mm == e) continue;
            const double* rm = (acc && mm == prev) ? rprev : v.R + ((size_t)w * v.ne + mm) * 3;
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
    if (v.n_ions && c == 0) {  // one-body terms in the first chunk, centres over the threads
        double re[3], g[3] = {0.0, 0.0, 0.0}, lap = 0.0;
        for (int k = 0; k < 3; ++k) re[k] = v.R[((size_t)w * v.ne + e) * 3 + k];
        jv[0] += j1_delta(v, rp, re, tid, kBlock);
        (void)j1_at(v, rp, tid, kBlock, g, lap);
        jv[1] += g[0];
        jv[2] += g[1];
        jv[3] += g[2];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) jv[k] = wave_sum(jv[k]);
    if (lane == 0)
        for (int k = 0; k < 4; ++k) jred[wave][k] = jv[k];
    __syncthreads();
    if (tid < 4) P[part_j2(K) + tid] = ((jred[0][tid] + jred[1][tid]) + jred[2][tid]) + jred[3][tid];

    // 4. the next move's proposal (electron e+1, or electron 0 of the next sweep)
    if (c == 0 && tid == 0) {
        const bool wrapn = e + 1 == v.ne;
        double rn[3];
        propose(v, w, wrapn ? 0 : e + 1, v.prm->step + (wrapn ? 1u : 0u), rn);
        double* dst = v.rnew + ((size_t)((e + 1) & 3) * v.W + w) * 3;
        dst[0] = rn[0]; dst[1] = rn[1]; dst[2] = rn[2];
    }
}

template <typename T>
void launch_move(const CrowdView<T>& v, int e, int prev, int reset, hipStream_t s)
{
    constexpr int CH = chunk_orbitals<T>();
    const int C = (v.n + CH - 1) / CH;
    hipLaunchKernelGGL(k_move<T>, dim3(xcd_grid(v.W, C)), dim3(kBlock), 0, s, v, e, prev, reset);
}

// Proposal of electron 0 at the current step (start of a run).
template <typename T>
__global__ void k_first_proposal(CrowdView<T> v)
{
    const int w = blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= v.W) return;
    double rn[3];
    propose(v, w, 0, v.prm->step, rn);
    double* dst = v.rnew + (size_t)w * 3;  // slot 0
    dst[0] = rn[0]; dst[1] = rn[1]; dst[2] = rn[2];
}

template <typename T>
void launch_first_proposal(const CrowdView<T>& v, hipStream_t s)
{
    hipLaunchKernelGGL(k_first_proposal<T>, dim3((v.W + 63) / 64), dim3(64), 0, s, v);
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

// Zero fill of count 32-bit words (a kernel rather than a memset node, so that work a
// caller captures into a graph replays it correctly).
__global__ __launch_bounds__(kBlock) void k_zero32(uint32_t* p, size_t count)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

void launch_zero(void* p, size_t bytes, hipStream_t s)
{
    const size_t count = bytes / 4;
    if (count == 0) return;
    const size_t blocks = std::min<size_t>(1024, (count + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_zero32, dim3((unsigned)blocks), dim3(kBlock), 0, s, (uint32_t*)p, count);
}

template void launch_fill_philox<float>(float*, uint64_t, size_t, hipStream_t);
template void launch_fill_philox<double>(double*, uint64_t, size_t, hipStream_t);
template void launch_setup_vgl<float>(const CrowdView<float>&, hipStream_t);
template void launch_setup_vgl<double>(const CrowdView<double>&, hipStream_t);
template void launch_move<float>(const CrowdView<float>&, int, int, int, hipStream_t);
template void launch_move<double>(const CrowdView<double>&, int, int, int, hipStream_t);
template void launch_first_proposal<float>(const CrowdView<float>&, hipStream_t);
template void launch_first_proposal<double>(const CrowdView<double>&, hipStream_t);

}  // namespace cq
