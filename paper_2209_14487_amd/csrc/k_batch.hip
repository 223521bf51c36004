// Batched VMC moves with delayed updates of k accepted moves.
//
// A VMC proposal r'_e = r_e + sigma z (Sec. II, Metropolis sampling with
// Gaussian moves, no drift) depends only on electron e's own position, and e has
// not moved yet in the sweep when its turn comes.  So the proposals of many
// upcoming moves are known before any of them is decided, and their orbital rows
// (the wavefunction evaluation of Alg. 1: B-spline value, gradient, Laplacian) can be evaluated in one
// wide, fully parallel gather launch over all walkers.  The sequential part
// (the ratio and accept steps of Alg. 1: ratios, Jastrow, Metropolis, in electron order) then works on
// small matrices only.
//
// Per walker and spin block, electrons are taken in order.  A round looks at the
// next Q candidates [dec, dec + Q) (evaluated ones are kept in a ring of 2Q stage
// slots, slot = electron mod 2Q) and decides them in order until k moves have been
// accepted or the candidates run out; the k (or fewer) accepted moves are then
// applied to the inverse in one rank-k update (delayed update).  With
//     P[i][j] = u_i . c0_j      (u_i: value row of candidate i, c0_j: inverse
//                                column of candidate j's electron, round start)
// the determinant ratio of candidate m after the accepted set S of the round is
// the Schur complement det(P[S+m, S+m]) / det(P[S, S]), evaluated in move order:
//     c_a     column of the a-th accepted electron just before its move
//             = sum_i T[a][i] c0_i
//     x_a     = u_m . c_a      = sum_i T[a][i] P[m][i]
//     beta_a  = (P[s_a][m] - sum_{j<a} beta_j G[a][j]) / rho_a
//     rho_m   = P[m][m] - sum_a beta_a x_a
//     accepted: T[cnt] = e_m - sum_a beta_a T[a], G[cnt][a] = x_a, rho_cnt = rho_m.
// The Jastrow difference of a candidate is summed over all electrons when it is
// evaluated; every later accepted move adds the change of its pair term.
//
// The orbital rows of an electron depend on nothing but its own proposal, so
// the gather runs ahead: from the end of round r-1's column kernel, through
// round r's P, decisions, columns and update, the gather fills the ring up to
// 2Q electrons past round r's first candidate (the furthest round r+1 can
// reach), on a second stream.  Its range is fixed by the cursors of round r-1,
// and it writes only ring slots of electrons that round r-1 (or an earlier
// round) decided, so it shares no data with round r.  The Jastrow sums need
// the positions after round r and are formed separately once round r is
// decided, next to round r's inverse update.
//
// k_stencils    proposals and stencils of the electrons in the gather range
// k_prop_vgl_wave / k_prop_vgl   gather + VGL of the same electrons (N >= 64 orbital
//               groups of 16 bytes / smaller N)
// k_jd          Jastrow sums of a round's new candidates
// k_pmat        P of every walker's candidates (FP64 sums of exact products)
// k_decide      one workgroup per walker: the decisions, the window for the
//               update kernel (accepted rows by slot, rho, G, L^-1, and T with
//               c_a = sum_i T[a][i] c0_i), the cursors and the Jastrow sums of the
//               candidates left for later
// k_cols        the columns c_a of the accepted moves
#include <algorithm>

#include "cq_device.h"
#include "cq_internal.h"
#include "cq_jastrow.h"
#include "cq_stencil.h"

namespace cq {

template <typename T>
__device__ __forceinline__ double pair_j2(const CrowdView<T>& v, double a, const double* x, const double* y)
{
    double d[3];
    min_image(x, y, v.L, d);
    double u, du, d2u;
    pade(a, v.b, sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]), u, du, d2u);
    return u;
}

// Gather layout for small N (fewer than 64 orbital groups of 16 bytes): 4
// proposals per workgroup, `groups` consecutive threads each.
constexpr int kVglSmallPP = 4;

inline int vgl_groups(int n, int elem_bytes) { return n / (16 / elem_bytes); }

inline int vgl_small_threads(int n, int elem_bytes)
{
    return ((kVglSmallPP * vgl_groups(n, elem_bytes) + 63) / 64) * 64;
}

// Electron t of walker w's gather range [look[par][w][0], look[par][w][1])
// (within the spin block); par is the parity of the round the range is for.
__device__ __forceinline__ bool gather_electron(const int* look, int par, int W, int w, int t, int& a)
{
    const int* L = look + ((size_t)par * W + w) * 2;
    a = L[0] + t;
    return a < L[1];
}

// Proposals and stencils of the electrons in the gather range, one wave per
// electron (lane = stencil entry), so that the gather workgroups start loading at
// once.  A range never holds more than Q electrons.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_stencils(CrowdView<T> v, int spin, int par)
{
    const int n = v.n, Q = v.Q, QR = v.QR;
    const int pi = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (pi >= v.W * Q) return;
    int a = 0;
    if (!gather_electron(v.look, par, v.W, pi / Q, pi % Q, a)) return;
    const int w = pi / Q, e = spin * n + a, slot = a % QR;
    const size_t ps = (size_t)w * QR + slot;
    double z[3], rp[3];
    gauss3(v.seed, v.uid[w], v.prm->step, (uint32_t)e, z);
    const double sigma = v.prm->sigma;
    for (int k = 0; k < 3; ++k) rp[k] = wrap_box(v.R[((size_t)w * v.ne + e) * 3 + k] + sigma * z[k], v.L);
    stencil_entry<T>(v, rp, lane, v.sidx + ps * 64, (T*)v.swt + ps * 64 * 5);
    if (lane < 3) v.rprop[ps * 3 + lane] = rp[lane];
}

// Gather + value/gradient/Laplacian of the electrons in the gather range, for
// N whose orbital groups (16 bytes each) fill whole waves (groups >= 64).  Every
// wave takes one slice of 64 groups of one proposal at a time, so the stencil
// (64 table offsets and 320 weights) is the same for all its lanes and is read with
// scalar loads: no LDS and no barrier.  Lane l of the slice owns one group, and
// each x-plane's 16 table loads (16 bytes per lane) are issued together before any
// of its sums, so that a wave keeps 16 KB in flight.  Work items (proposal,
// slice) go round-robin over the waves of a persistent grid (a few workgroups per
// CU), so that the decision, column and update kernels of the current round still
// find room on every CU while it runs.
// The stencils and the gather ranges are read through constant-address-space
// pointers (scalar loads).

template <typename T>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(5))) void k_prop_vgl_wave(CrowdView<T> v,
                                                                                                  int spin, int par)
{
    constexpr int VEC = 16 / sizeof(T);
    const int n = v.n, Q = v.Q, QR = v.QR, groups = n / VEC;
    const int slices = (groups + 63) >> 6;
    const int nitem = v.W * Q * slices;
    const int lane = threadIdx.x & 63;
    const int wave0 = __builtin_amdgcn_readfirstlane(blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6));
    const int nwave = gridDim.x * (kBlock / 64);
    const cptr<int> look = as_const(v.look);
    const cptr<size_t> sidx_all = as_const(v.sidx);
    const cptr<T> swt_all = as_const((const T*)v.swt);
    for (int item = wave0; item < nitem; item += nwave) {
        const int pi = item / slices, sl = item - pi * slices;
        const int w = pi / Q, t = pi - w * Q;
        const cptr<int> lk = look + ((size_t)par * v.W + w) * 2;  // gather range of this round
        const int a = lk[0] + t;
        if (a >= lk[1]) continue;
        const int g = sl * 64 + lane;
        const size_t ps = (size_t)w * QR + a % QR;
        const cptr<size_t> sidx = sidx_all + ps * 64;
        const cptr<T> sw = swt_all + ps * 64 * 5;
        const uint32_t lane_off = (uint32_t)(g < groups ? g : 0) * (uint32_t)(VEC * sizeof(T));
        T acc[5][VEC];
#pragma unroll
        for (int k = 0; k < 5; ++k)
#pragma unroll
            for (int i = 0; i < VEC; ++i) acc[k][i] = (T)0;
#pragma unroll 1
        for (int x = 0; x < 4; ++x) {
            T vals[16][VEC];
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const char* base = reinterpret_cast<const char*>(v.table + sidx[x * 16 + q]);
                load16(reinterpret_cast<const T*>(base + lane_off), vals[q]);
            }
            // keeps the sums (and the scheduler's interleaving of them) behind the loads
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const cptr<T> wq = sw + (x * 16 + q) * 5;
                const T wv = wq[0], wgx = wq[1], wgy = wq[2], wgz = wq[3], wl = wq[4];
#pragma unroll
                for (int i = 0; i < VEC; ++i) {
                    acc[0][i] += wv * vals[q][i];
                    acc[1][i] += wgx * vals[q][i];
                    acc[2][i] += wgy * vals[q][i];
                    acc[3][i] += wgz * vals[q][i];
                    acc[4][i] += wl * vals[q][i];
                }
            }
        }
        if (g < groups) {
            T* dst = v.stage + ps * 5 * (size_t)n + (size_t)g * VEC;
#pragma unroll
            for (int k = 0; k < 5; ++k) store16(dst + (size_t)k * n, acc[k]);
        }
    }
}

// The same for small N (groups < 64): up to 4 proposals per workgroup, `groups`
// consecutive threads per proposal, stencils staged in LDS.
template <typename T>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(6))) void k_prop_vgl(CrowdView<T> v, int spin,
                                                                                           int pp, int par)
{
    constexpr int VEC = 16 / sizeof(T);
    // dynamic LDS sized for pp proposals: stencil offsets, weights, flags
    extern __shared__ size_t vgl_lds[];
    size_t(*s_idx)[64] = reinterpret_cast<size_t(*)[64]>(vgl_lds);
    T(*s_w)[64 * 5] = reinterpret_cast<T(*)[64 * 5]>(vgl_lds + (size_t)pp * 64);
    int* s_ok = reinterpret_cast<int*>(&s_w[pp][0]);
    const int n = v.n, Q = v.Q, QR = v.QR, groups = n / VEC;
    const int nprop = v.W * Q;
    const int nt = blockDim.x, tid = threadIdx.x;
    const int p = tid / groups, t0 = tid % groups;  // proposal of the chunk, group
    const int nchunk = (nprop + pp - 1) / pp;

    for (int chunk = blockIdx.x; chunk < nchunk; chunk += gridDim.x) {
        const int first = chunk * pp;
        __syncthreads();  // the previous chunk's readers of the stencils are done
        // stencils of this chunk's proposals into LDS
        if (tid < pp) {
            const int pi = first + tid;
            int a = 0;
            s_ok[tid] = pi < nprop && gather_electron(v.look, par, v.W, pi / Q, pi % Q, a);
        }
        __syncthreads();
        for (int idx = tid; idx < pp * 64; idx += nt) {
            const int pq = idx >> 6, l = idx & 63, pi = first + pq;
            if (!s_ok[pq]) continue;
            int a = 0;
            gather_electron(v.look, par, v.W, pi / Q, pi % Q, a);
            const size_t ps = (size_t)(pi / Q) * QR + a % QR;
            s_idx[pq][l] = v.sidx[ps * 64 + l];
            const T* sw = (const T*)v.swt + (ps * 64 + l) * 5;
#pragma unroll
            for (int k = 0; k < 5; ++k) s_w[pq][l * 5 + k] = sw[k];
        }
        __syncthreads();

        const int pi = first + p;
        if (!(p < pp && pi < nprop && s_ok[p])) continue;
        int a = 0;
        gather_electron(v.look, par, v.W, pi / Q, pi % Q, a);
        const int w = pi / Q, slot = a % QR;
        T* dst = v.stage + ((size_t)w * QR + slot) * 5 * (size_t)n;
        const size_t* sidx = s_idx[p];
        const T* sw = s_w[p];
        {
            const int j0 = t0 * VEC;
            T acc[5][VEC];
#pragma unroll
            for (int k = 0; k < 5; ++k)
#pragma unroll
                for (int i = 0; i < VEC; ++i) acc[k][i] = (T)0;
#pragma unroll 1
            for (int x = 0; x < 4; ++x) {
                T vals[16][VEC];
#pragma unroll
                for (int q = 0; q < 16; ++q) load16(v.table + sidx[x * 16 + q] + j0, vals[q]);
#pragma unroll
                for (int q = 0; q < 16; ++q) {
                    const T* wq = sw + (x * 16 + q) * 5;
                    const T wv = wq[0], wgx = wq[1], wgy = wq[2], wgz = wq[3], wl = wq[4];
#pragma unroll
                    for (int i = 0; i < VEC; ++i) {
                        acc[0][i] += wv * vals[q][i];
                        acc[1][i] += wgx * vals[q][i];
                        acc[2][i] += wgy * vals[q][i];
                        acc[3][i] += wgz * vals[q][i];
                        acc[4][i] += wl * vals[q][i];
                    }
                }
            }
#pragma unroll
            for (int k = 0; k < 5; ++k) store16(dst + (size_t)k * n + j0, acc[k]);
        }
    }
}

// Jastrow sums of a round's new candidates [ev, min(dec + Q, n)) against the
// positions after the previous round:
//     dlnJ_e = sum_{i != e} u(|r'_e - r_i|) - u(|r_e - r_i|)
//              + sum_I u1(|r'_e - R_I|) - u1(|r_e - R_I|)     (one-body terms, FP64).
// The coordinate differences are taken in FP64 and each pair term in the
// precision of the path (FP32 terms in mixed precision, like the ratios); the
// sums are FP64.  One workgroup per walker and group of kJdCand candidates;
// thread t takes the electrons i = t, t + kBlock, ...; the partial sums are
// added in a fixed order.
constexpr int kJdCand = 8;

template <typename T>
__device__ __forceinline__ T jd_term(T a, T b, T L, T iL, const double* x, const double* y)
{
    T r2 = (T)0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        T d = (T)(x[c] - y[c]);
        if constexpr (sizeof(T) == 8)
            d -= L * rint(d / L);
        else
            d -= L * rintf(d * iL);
        r2 += d * d;
    }
    const T r = sqrt(r2);
    return a * r / ((T)1 + b * r);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_jd(CrowdView<T> v, int spin)
{
    __shared__ double s_rp[kJdCand][3], s_re[kJdCand][3];
    __shared__ double s_part[kJdCand][kBlock / 64];
    const int n = v.n, Q = v.Q, QR = v.QR, ne = v.ne;
    const int per = (Q + kJdCand - 1) / kJdCand;
    const int w = blockIdx.x / per, c0 = (blockIdx.x % per) * kJdCand;
    const int dec = v.cur[2 * w], ev = v.cur[2 * w + 1];
    const int end = dec + Q < n ? dec + Q : n;
    const int a0 = ev + c0;
    if (a0 >= end) return;
    const int nc = end - a0 < kJdCand ? end - a0 : kJdCand;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const double* Rw = v.R + (size_t)w * ne * 3;
    if (!v.use_j2 && !v.n_ions) {
        if (tid < nc) v.jd[(size_t)w * QR + (a0 + tid) % QR] = 0.0;
        return;
    }
    if (tid < kJdCand * 3) {
        const int c = tid / 3, k = tid % 3;
        const int a = a0 + (c < nc ? c : 0);
        s_rp[c][k] = v.rprop[((size_t)w * QR + a % QR) * 3 + k];
        s_re[c][k] = Rw[((size_t)spin * n + a) * 3 + k];
    }
    __syncthreads();
    const T L = (T)v.L, iL = (T)(1.0 / v.L), b = (T)v.b;
    double dj[kJdCand];
#pragma unroll
    for (int c = 0; c < kJdCand; ++c) dj[c] = 0.0;
    const int self = spin * n + a0;
    for (int i = tid; v.use_j2 && i < ne; i += kBlock) {
        const double ri[3] = {Rw[(size_t)i * 3], Rw[(size_t)i * 3 + 1], Rw[(size_t)i * 3 + 2]};
        const T aa = (T)(((i >= n) == (spin != 0)) ? v.a_par : v.a_anti);
#pragma unroll
        for (int c = 0; c < kJdCand; ++c) {
            const T d = jd_term<T>(aa, b, L, iL, s_rp[c], ri) - jd_term<T>(aa, b, L, iL, s_re[c], ri);
            dj[c] += i == self + c ? 0.0 : (double)d;  // the candidate's own electron is not a pair
        }
    }
    // one-body terms (FP64), the centres shared out over the threads
#pragma unroll
    for (int c = 0; c < kJdCand; ++c)
        if (v.n_ions) dj[c] += j1_delta(v, s_rp[c], s_re[c], tid, kBlock);
#pragma unroll
    for (int c = 0; c < kJdCand; ++c) {
        const double t = wave_sum(dj[c]);
        if (lane == 0) s_part[c][wave] = t;
    }
    __syncthreads();
    if (tid < nc) {
        double sum = 0.0;
#pragma unroll
        for (int q = 0; q < kBlock / 64; ++q) sum += s_part[tid][q];
        v.jd[(size_t)w * QR + (a0 + tid) % QR] = sum;
    }
}

// P of one walker's candidates in 16 x 16 blocks on the FP64 matrix cores
// (v_mfma_f64_16x16x4f64): the stored T values are widened to FP64, so every
// product is exact and the sums are FP64.  Operand layout: lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16]; the result is D[l / 16 + 4 v][l % 16].
// The 4 k values of a step are taken as k0 + VEC q + s (q = l / 16, s = step
// within a 16-byte load), the same on both operands.  The 4 waves of a
// workgroup take alternate k chunks; their partial blocks are added in order.  A
// workgroup covers kPTJ blocks of one block row, which share the row operand: the
// launch has a third of the workgroups that one block each would need, and each
// does three times the work between its loads and its stores.
typedef double f64x4 __attribute__((ext_vector_type(4)));
constexpr int kPB = 16;   // block edge
constexpr int kPTJ = 3;   // column blocks per workgroup (when a block row has that many)

template <typename T, int TJ>  // TJ column blocks per workgroup, sharing the row operand
__global__ __launch_bounds__(kBlock) void k_pmat(CrowdView<T> v, int spin)
{
    constexpr int VEC = 16 / sizeof(T);
    constexpr int KC = 4 * VEC;  // k values per chunk
    __shared__ double sP[4][TJ][kPB][kPB + 1];
    const int Q = v.Q, n = v.n;
    const int nb = (Q + kPB - 1) / kPB, nbg = (nb + TJ - 1) / TJ;
    int w, blk;  // a walker's tiles share one XCD, so its rows are fetched into one L2
    xcd_map(blockIdx.x, nb * nbg, w, blk);
    if (w >= v.W) return;
    const int bi = blk / nbg, bj0 = (blk % nbg) * TJ;
    const int dec = v.cur[2 * w];
    const int nc = (dec + Q < n ? dec + Q : n) - dec;
    if (bi * kPB >= nc || bj0 * kPB >= nc) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int r = lane & 15, q = lane >> 4;
    const int ci = bi * kPB + r;
    const T* urow = v.stage + ((size_t)w * v.QR + (dec + (ci < nc ? ci : 0)) % v.QR) * 5 * (size_t)n;
    const T* crow[TJ];
    bool c_live[TJ];
#pragma unroll
    for (int tj = 0; tj < TJ; ++tj) {
        const int cj = (bj0 + tj) * kPB + r;
        c_live[tj] = cj < nc;
        crow[tj] = v.M + (((size_t)w * 2 + spin) * n + dec + (cj < nc ? cj : 0)) * (size_t)n;
    }
    f64x4 acc[TJ];
#pragma unroll
    for (int tj = 0; tj < TJ; ++tj) acc[tj] = f64x4{0.0, 0.0, 0.0, 0.0};
    // 4 chunks of loads in flight per lane.  Addresses past the end (k >= n) or of
    // rows past the candidates are clamped to valid ones and the values zeroed, so
    // no branch splits a batch.
    constexpr int NB = 4;
    const bool u_live = ci < nc;
    for (int k00 = wave * KC; k00 < n; k00 += NB * 4 * KC) {
        T u[NB][VEC], c[TJ][NB][VEC];
#pragma unroll
        for (int it = 0; it < NB; ++it) {
            const int kk = k00 + it * 4 * KC + VEC * q;
            const int kc = kk < n ? kk : 0;
            load16(urow + kc, u[it]);
#pragma unroll
            for (int tj = 0; tj < TJ; ++tj) load16(crow[tj] + kc, c[tj][it]);
        }
#pragma unroll
        for (int it = 0; it < NB; ++it) {
            const bool in = k00 + it * 4 * KC + VEC * q < n;
#pragma unroll
            for (int s2 = 0; s2 < VEC; ++s2) {
                const double a = in && u_live ? (double)u[it][s2] : 0.0;
#pragma unroll
                for (int tj = 0; tj < TJ; ++tj)
                    acc[tj] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, in && c_live[tj] ? (double)c[tj][it][s2] : 0.0,
                                                                   acc[tj], 0, 0, 0);
            }
        }
    }
#pragma unroll
    for (int tj = 0; tj < TJ; ++tj)
#pragma unroll
        for (int t = 0; t < 4; ++t) sP[wave][tj][q + 4 * t][r] = acc[tj][t];
    __syncthreads();
    double* P = v.pmat + (size_t)w * Q * Q;
    for (int idx = tid; idx < TJ * kPB * kPB; idx += kBlock) {
        const int tj = idx / (kPB * kPB), i = (idx / kPB) % kPB, j = idx % kPB;
        const double sum = ((sP[0][tj][i][j] + sP[1][tj][i][j]) + sP[2][tj][i][j]) + sP[3][tj][i][j];
        const int gi = bi * kPB + i, gj = (bj0 + tj) * kPB + j;
        if (gi < nc && gj < nc) P[(size_t)gi * Q + gj] = sum;
    }
}

// Jastrow pair-term change for candidate (r_old -> r_new) when another electron
// moved from o to q.
template <typename T>
__device__ __forceinline__ double pair_change(const CrowdView<T>& v, const double* rn, const double* ro,
                                              const double* q, const double* o)
{
    return (pair_j2(v, v.a_par, rn, q) - pair_j2(v, v.a_par, rn, o)) -
           (pair_j2(v, v.a_par, ro, q) - pair_j2(v, v.a_par, ro, o));
}

// Decision kernel.  Everything the sequential loop reads sits in LDS (dynamic,
// about 146 KB at Q = 88): P, the Jastrow pair changes of every candidate pair,
// the rows X[a][i] = u_i . c_a and B[a][i] = beta_a(i) of every accepted move a
// against every candidate i, and the running ratio and Jastrow sum of every
// candidate.  An acceptance adds one row of X and of B (O(accepted) per
// candidate); T and L^-1 of the window follow from these rows once the decisions
// are made, as the inverses of two triangles, so the loop carries neither.
struct DecideLds {
    static constexpr int QM = kMaxCand, D = kMaxDelay;
    double P[QM][QM + 1];
    double PC[QM * (QM - 1) / 2];  // Jastrow change of candidate m when s (< m) moves, at m(m-1)/2 + s
    double X[D][QM + 1];           // X[a][i] = u_i . c_a: candidate i against accepted move a
    double B[D][QM + 1];           // B[a][i] = beta_a(i), component a of L^-1 y(i)
    double u[QM], jd[QM];
    double rho[QM], dj[QM];        // running Schur complement and Jastrow sum of each candidate
    double racc[D];                // Schur complements of the accepted moves
    double rold[QM][3], rnew[QM][3];
    int slot[D];
    int cnt, ndec;
};

// par: parity of the round within the spin block.  Besides the round's window the
// kernel writes the gather range of round r+2: from the end of round r+1's range
// to 2Q past round r+1's first candidate.
// Gather workgroups per CU when it runs beside the round being decided and applied
// (the rest of each CU stays free for those kernels: one workgroup of the wave-sliced
// gather, 4 waves of 92 registers, leaves room for an update workgroup of 8 waves of
// 124 registers and for the decision and column kernels), and when it runs alone.
constexpr int kVglBlocksPerCU = 3;
constexpr int kVglWaveBlocksPerCU = 1;
constexpr int kVglBlocksPerCUAlone = 8;

template <typename T>
__global__ __launch_bounds__(kBlock) void k_decide(CrowdView<T> v, int spin, int par, int round)
{
    extern __shared__ unsigned char dsm[];
    DecideLds& S = *reinterpret_cast<DecideLds*>(dsm);
    const int w = blockIdx.x;
    const int n = v.n, K = v.K, Q = v.Q;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int dec = v.cur[2 * w];
    const int nc = (dec + Q < n ? dec + Q : n) - dec;
    const int e0 = spin * n + dec;
    // run parameters in registers: the loop below stores to global memory, so loads
    // through v.prm inside it could not be hoisted and would cost a round trip each
    const int rs = v.prm->rec_sweep;
    const uint32_t step = v.prm->step;
    const bool recording = rs < v.prm->rec_cap;
    const bool forcing = v.forced && rs < v.prm->forced_cap;
    auto next_range = [&](int dec_next) {  // gather range of round r+2
        const int lo = v.look[((size_t)(par ^ 1) * v.W + w) * 2 + 1];
        const int hi = dec_next + 2 * Q < n ? dec_next + 2 * Q : n;
        int* L = v.look + ((size_t)par * v.W + w) * 2;
        L[0] = lo;
        L[1] = hi > lo ? hi : lo;
    };
    if (nc <= 0) {  // this walker's spin block is done
        if (tid == 0) {
            v.cnt[(size_t)2 * v.W + w] = 0;
            next_range(dec);
        }
        return;
    }
    if (tid == 0) atomicMax(&v.used[spin], round + 1);  // rounds the block has needed so far
    // candidates: P, uniforms, Jastrow sums, positions
    // P (nc x nc, row stride Q): wave v loads rows 22v..22v+21 with the lanes along
    // the columns, all rows of a column batch in flight together
    const double* Pw = v.pmat + (size_t)w * Q * Q;
    {
        constexpr int RPW = DecideLds::QM / 4;
        static_assert(DecideLds::QM % 4 == 0 && DecideLds::QM <= 128 && kBlock == 256, "P rows per wave");
#pragma unroll
        for (int half = 0; half < 2; ++half) {
            const int j = lane + 64 * half;
            if (j < nc) {
                double x[RPW];
#pragma unroll
                for (int r = 0; r < RPW; ++r) {
                    const int i = wave * RPW + r;
                    x[r] = i < nc ? Pw[(size_t)i * Q + j] : 0.0;
                }
#pragma unroll
                for (int r = 0; r < RPW; ++r) {
                    const int i = wave * RPW + r;
                    if (i < nc) S.P[i][j] = x[r];
                }
            }
        }
    }
    if (tid < nc) {
        const int slot = (dec + tid) % v.QR;
        S.u[tid] = accept_uniform(v.seed, v.uid[w], step, (uint32_t)(e0 + tid));
        S.jd[tid] = v.jd[(size_t)w * v.QR + slot];
        for (int k = 0; k < 3; ++k) {
            S.rold[tid][k] = v.R[((size_t)w * v.ne + e0 + tid) * 3 + k];
            S.rnew[tid][k] = v.rprop[((size_t)w * v.QR + slot) * 3 + k];
        }
    }
    __syncthreads();
    // rows of X and B start at zero: the sums over accepted moves below run over whole
    // groups of 8 rows, and the rows past the accepted count must contribute nothing
    for (int idx = tid; idx < DecideLds::D * (DecideLds::QM + 1); idx += kBlock) {
        (&S.X[0][0])[idx] = 0.0;
        (&S.B[0][0])[idx] = 0.0;
    }
    if (tid < nc) {
        S.rho[tid] = S.P[tid][tid];
        S.dj[tid] = S.jd[tid];
    }
    // Jastrow pair changes of all candidate pairs (s < m)
    for (int idx = tid; idx < nc * nc; idx += kBlock) {
        const int m = idx / nc, sx = idx % nc;
        if (sx < m)
            S.PC[m * (m - 1) / 2 + sx] = v.use_j2 ? pair_change(v, S.rnew[m], S.rold[m], S.rnew[sx], S.rold[sx]) : 0.0;
    }
    __syncthreads();

    // Decisions in electron order (wave 0, lane <-> candidate).  Candidate i's ratio
    // and Jastrow sum are rho_i and dj_i, brought up to date by every acceptance of an
    // earlier candidate m (the a-th accepted move) for all later candidates at once:
    //     X[a][i] = P[i][m] - sum_{b<a} beta_b(m) X[b][i]
    //     B[a][i] = (P[m][i] - sum_{t<a} X[t][m] B[t][i]) / rho_m
    //     rho_i  -= B[a][i] X[a][i],    dj_i += PC(i, m).
    // Every candidate past the last acceptance is then tested at once (lanes), and a
    // ballot gives the next acceptance: the candidates before it are rejected with the
    // ratios they had, since nothing changed them in between.  A rejection costs no
    // serial step, an acceptance one pass of O(accepted) per lane.
    if (wave == 0) {
        int cnt = 0, first = 0, macc = -1, ndec = 0;
        double xa = 0.0, ba = 0.0, rinv = 0.0;  // lane a: X[a][m], beta_a(m) of the last acceptance m
        for (;;) {
            const bool deciding = cnt < K;
            bool found = false;
            int next = nc;
            double rnext = 0.0;
            for (int base = first; base < nc; base += 64) {
                const int i = base + lane;
                const bool valid = i < nc;
                const int ic = valid ? i : first;
                double r = S.rho[ic], d = S.dj[ic];
                if (macc >= 0) {  // row cnt-1 of X and B, for the acceptance of candidate macc
                    const int row = cnt - 1;
                    double xc = S.P[ic][macc], bc = S.P[macc][ic];
                    for (int a0 = 0; a0 < row; a0 += 8) {
#pragma unroll
                        for (int q = 0; q < 8; ++q) {  // rows past row are zero, so are their coefficients
                            xc -= dpp::lane(ba, a0 + q) * S.X[a0 + q][ic];
                            bc -= dpp::lane(xa, a0 + q) * S.B[a0 + q][ic];
                        }
                    }
                    bc *= rinv;
                    r -= bc * xc;
                    d += S.PC[ic * (ic - 1) / 2 + macc];
                    if (valid) {
                        S.X[row][i] = xc;
                        S.B[row][i] = bc;
                        S.rho[i] = r;
                        S.dj[i] = d;
                    }
                }
                if (deciding && !found) {
                    const double prob = r * r * exp(2.0 * d);
                    int acc = S.u[ic] < prob;
                    const size_t ri = ((size_t)rs * v.ne + e0 + ic) * v.Wcap + w;
                    if (forcing && v.forced[ri] < 2) acc = v.forced[ri] != 0;
                    const uint64_t hit = __builtin_amdgcn_ballot_w64(valid && acc);
                    const int lim = hit ? base + __builtin_ctzll(hit) : nc;  // candidates decided here: i <= lim
                    if (recording && valid && i <= lim) {
                        v.rec_rho[ri] = r;
                        v.rec_dlnj[ri] = d;
                        v.rec_prob[ri] = prob;
                        v.rec_acc[ri] = (uint8_t)acc;
                    }
                    if (hit) {
                        found = true;
                        next = lim;
                        rnext = dpp::lane(r, __builtin_ctzll(hit));
                    }
                }
            }
            if (!deciding) {  // the update pass of the last acceptance the window holds
                ndec = first;
                break;
            }
            if (!found) {  // the rest rejected
                ndec = nc;
                break;
            }
            // acceptance of candidate next: its coefficients against the earlier accepted
            // moves, read after this wave's stores of the pass above
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
            __builtin_amdgcn_wave_barrier();
            xa = lane < cnt ? S.X[lane][next] : 0.0;
            ba = lane < cnt ? S.B[lane][next] : 0.0;
            if (lane == 0) {
                S.racc[cnt] = rnext;
                S.slot[cnt] = next;
            }
            rinv = 1.0 / rnext;
            macc = next;
            first = next + 1;
            ++cnt;
        }
        if (lane == 0) {
            v.nacc[w] += cnt;
            v.nprop[w] += ndec;
            S.cnt = cnt;
            S.ndec = ndec;
        }
    }
    __syncthreads();
    const int cnt = S.cnt, ndec = S.ndec;

    // the window for the update kernels, the accepted positions, the cursors
    if (tid < cnt) {
        const int a = dec + S.slot[tid];
        v.welec[(size_t)w * K + tid] = a;
        v.wslot[(size_t)w * K + tid] = a % v.QR;
        for (int k = 0; k < 3; ++k) v.R[((size_t)w * v.ne + spin * n + a) * 3 + k] = S.rnew[S.slot[tid]][k];
    }
    if (wave < 2) {
        // L^-1 (wave 0) and T (wave 1) of the window by forward substitution, column j
        // in lane j:  L[c][t] = X[t][s_c] (t < c), L[c][c] = rho_c, so that
        //     Linv[c][j] = (delta_cj - sum_{t<c} L[c][t] Linv[t][j]) / rho_c;
        // T inverts the unit lower triangle U[c][a] = beta_a(s_c) = B[a][s_c] (a < c).
        const bool lower = wave == 0;
        const double rv = lower && lane < cnt ? 1.0 / S.racc[lane] : 1.0;
        double col[kMaxDelay];
#pragma unroll
        for (int c = 0; c < kMaxDelay; ++c) {
            col[c] = 0.0;
            if (c < cnt) {
                const int sc = S.slot[c];
                double sum = 0.0;
#pragma unroll
                for (int t = 0; t < c; ++t) sum += (lower ? S.X[t][sc] : S.B[t][sc]) * col[t];
                col[c] = ((c == lane ? 1.0 : 0.0) - sum) * dpp::lane(rv, c);
            }
        }
        double* out = (lower ? v.wlinv : v.tmat) + (size_t)w * K * K;
        if (lane < cnt)
#pragma unroll
            for (int c = 0; c < kMaxDelay; ++c)
                if (c < cnt) out[(size_t)c * K + lane] = col[c];
    } else if (wave == 2) {  // G[c][a] = u_{s_c} . c_a (a < c) and the ratios of the window
        for (int idx = lane; idx < cnt * cnt; idx += 64) {
            const int c = idx / cnt, a = idx % cnt;
            if (a < c) v.wG[((size_t)w * K + c) * K + a] = S.X[a][S.slot[c]];
        }
        if (lane < cnt) v.wrho[(size_t)w * K + lane] = S.racc[lane];
    } else {  // log |det| and sign, summed in acceptance order
        const double rc = lane < cnt ? S.racc[lane] : 1.0;
        const double lg = log(fabs(rc));
        const uint64_t neg = __builtin_amdgcn_ballot_w64(rc < 0.0);
        // the lane reads run in every lane: inside a one-lane branch the compiler may
        // move the computation of lg there too, and the other lanes would not hold it
        double ld = v.logdet[w * 2 + spin];
#pragma unroll
        for (int c = 0; c < kMaxDelay; ++c)
            if (c < cnt) ld += dpp::lane(lg, c);
        if (lane == 0) {
            v.logdet[w * 2 + spin] = ld;
            if (__builtin_popcountll(neg) & 1) v.sign[w * 2 + spin] = -v.sign[w * 2 + spin];
        }
    }
    if (tid == 0) {
        v.cnt[(size_t)2 * v.W + w] = cnt;
        v.cur[2 * w] = dec + ndec;
        v.cur[2 * w + 1] = dec + nc;
        v.cur[2 * v.W + w] = dec;  // start of this round's candidates, for the column kernel
        next_range(dec + ndec);
    }
    // Jastrow sums of the candidates left for later rounds, with this round's moves
    if (v.use_j2 && tid >= ndec && tid < nc) v.jd[(size_t)w * v.QR + (dec + tid) % v.QR] = S.dj[tid];
}

// Columns of the accepted moves: c_a = sum_{j<=a} T[a][j] c0_{s_j} for a < cnt,
// c0_{s_j} the start column of the j-th accepted move's electron (FP64 sums of
// exact products, rounded to T).  One thread per orbital.  For the matrix-core
// update the kernel also packs the accepted value rows (ub), so that the update
// kernel's loads need no indirection.  The kernel sits between the decisions and
// the update while the gather of the next round streams beside it, so every
// global round trip is long: the count, T and the window are loaded in one batch,
// then all accepted rows at once.
template <typename T>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4))) void k_cols(CrowdView<T> v, int spin)
{
    constexpr int D = kMaxDelay, TL = D * D / kBlock;
    static_assert(D * D % kBlock == 0, "T tile per thread");
    __shared__ __align__(16) double s_T[D][D];
    __shared__ __align__(16) int s_row[D];
    __shared__ __align__(16) int s_slot[D];
    const int n = v.n, K = v.K;
    const int nlb = (n + kBlock - 1) / kBlock;
    int w, part;  // a walker's blocks share one XCD
    xcd_map(blockIdx.x, nlb, w, part);
    if (w >= v.W) return;
    const int tid = threadIdx.x, l = part * kBlock + tid;
    // first batch: the count, T (K x K) and the window's electrons and slots; what
    // lies past the count is replaced once the loads are back (T by zeros, so the
    // sums below need no bounds)
    const int cnt = v.cnt[(size_t)2 * v.W + w];
    double tv[TL];
#pragma unroll
    for (int q = 0; q < TL; ++q) {
        const int idx = q * kBlock + tid, a = idx / D, j = idx % D;
        tv[q] = a < K && j < K ? v.tmat[((size_t)w * K + a) * K + j] : 0.0;
    }
    int e = 0, sl = 0;
    if (tid < K) {
        e = v.welec[(size_t)w * K + tid];
        sl = v.wslot[(size_t)w * K + tid];
    }
    if (cnt <= 0 || cnt > K) return;
#pragma unroll
    for (int q = 0; q < TL; ++q) {
        const int idx = q * kBlock + tid, a = idx / D, j = idx % D;
        s_T[j][a] = a < cnt && j < cnt ? tv[q] : 0.0;  // transposed: s_T[j][a] = T[a][j]
    }
    if (tid < D) {
        if (tid < cnt && (e < 0 || e >= n || sl < 0 || sl >= v.QR)) atomicOr(&v.status[w], 2);
        s_row[tid] = tid < cnt && e >= 0 && e < n ? e : 0;
        s_slot[tid] = tid < cnt && sl >= 0 && sl < v.QR ? sl : 0;
    }
    __syncthreads();
    if (l >= n) return;
    // second batch: the accepted value rows (for ub) and start columns
    const T* Mw = v.M + ((size_t)w * 2 + spin) * n * (size_t)n + l;
    const bool pack = sizeof(T) == 4 && v.ub != nullptr;
    // Rows past the count are loaded too (row 0, slot 0: one cached line per thread),
    // so that no branch splits the batch; their T entries are zero.  Value rows
    // first: they are stored while the columns are in flight.
    T c[D], x[D];
    if (pack) {
#pragma unroll
        for (int j = 0; j < D; ++j) x[j] = v.stage[((size_t)w * v.QR + s_slot[j]) * 5 * (size_t)n + l];
    } else {
#pragma unroll
        for (int j = 0; j < D; ++j) x[j] = (T)0;
    }
#pragma unroll
    for (int j = 0; j < D; ++j) c[j] = Mw[(size_t)s_row[j] * n];
    if constexpr (sizeof(T) == 4) {
        if (pack)
#pragma unroll
            for (int a = 0; a < D; ++a)
                if (a < cnt) v.ub[((size_t)w * D + a) * n + l] = x[a];
    }
    // c_a for 4 accepted moves at a time (one 16-byte store of ct); T is read
    // transposed, 4 consecutive moves per LDS load
    auto group = [&](int g, double acc[4]) {
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[q] = 0.0;
#pragma unroll
        for (int h = 0; h < D / 8; ++h) {
            if (8 * h < cnt) {
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const int j = 8 * h + q;
                    const double cj = (double)c[j];
                    const double2 t01 = *reinterpret_cast<const double2*>(&s_T[j][4 * g]);
                    const double2 t23 = *reinterpret_cast<const double2*>(&s_T[j][4 * g + 2]);
                    acc[0] = fma(t01.x, cj, acc[0]);
                    acc[1] = fma(t01.y, cj, acc[1]);
                    acc[2] = fma(t23.x, cj, acc[2]);
                    acc[3] = fma(t23.y, cj, acc[3]);
                }
            }
        }
    };
    if constexpr (sizeof(T) == 4) {
        if (v.ct) {  // transposed for the matrix-core update: 32 per row, zeros past cnt
            float* dst = v.ct + ((size_t)w * n + l) * D;
#pragma unroll 1
            for (int g = 0; g < D / 4; ++g) {
                double acc[4] = {0.0, 0.0, 0.0, 0.0};
                if (4 * g < cnt) group(g, acc);
                float y[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) y[q] = 4 * g + q < cnt ? (float)acc[q] : 0.0f;
                store16(dst + 4 * g, y);
            }
            return;
        }
    }
    T* Cw = v.Cbuf + (size_t)w * K * n;
#pragma unroll 1
    for (int g = 0; g < D / 4; ++g) {
        if (4 * g < cnt) {
            double acc[4];
            group(g, acc);
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (4 * g + q < cnt) Cw[(size_t)(4 * g + q) * n + l] = (T)acc[q];
        }
    }
}

// Start of a spin block: cursors at 0, gather ranges [0, Q) for round 0 and
// [Q, 2Q) for round 1 (clipped to N).
// The accepted orbital rows of the window (value, gradient, Laplacian) go into the
// walker's matrices: one thread per orbital, for the matrix-core path (the vector
// update copies them itself).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_rows(CrowdView<T> v, int spin)
{
    constexpr int D = kMaxDelay, RB = 8;  // accepted rows per batch of loads
    __shared__ __align__(16) int s_e[D];
    __shared__ __align__(16) int s_sl[D];
    const int n = v.n, K = v.K;
    const int nlb = (n + kBlock - 1) / kBlock;
    int w, part;  // a walker's blocks share one XCD
    xcd_map(blockIdx.x, nlb, w, part);
    if (w >= v.W) return;
    const int tid = threadIdx.x, l = part * kBlock + tid;
    // the window's electrons and slots in one batch (entries past the count or out of
    // range are marked; bad entries are reported by the column kernel)
    int cnt = v.cnt[(size_t)2 * v.W + w];
    int e = -1, sl = -1;
    if (tid < K) {
        e = v.welec[(size_t)w * K + tid];
        sl = v.wslot[(size_t)w * K + tid];
    }
    if (cnt > K) cnt = K;
    if (cnt <= 0) return;
    if (tid < D) {
        const bool ok = tid < cnt && e >= 0 && e < n && sl >= 0 && sl < v.QR;
        s_e[tid] = ok ? e : -1;
        s_sl[tid] = ok ? sl : 0;
    }
    __syncthreads();
    if (l >= n) return;
    // RB accepted rows (5 RB loads) in flight per thread
    for (int a0 = 0; a0 < cnt; a0 += RB) {
        T x[RB][5];
#pragma unroll
        for (int q = 0; q < RB; ++q) {
            const int a = (a0 + q) & (D - 1);
            const T* src = v.stage + ((size_t)w * v.QR + s_sl[a]) * 5 * (size_t)n + l;
#pragma unroll
            for (int p = 0; p < 5; ++p) x[q][p] = src[(size_t)p * n];
        }
#pragma unroll
        for (int q = 0; q < RB; ++q) {
            const int a = a0 + q, ea = s_e[a & (D - 1)];
            if (a >= cnt || ea < 0) continue;
            T* dst = v.VGL + (((size_t)w * 2 + spin) * n + ea) * 5 * (size_t)n + l;
#pragma unroll
            for (int p = 0; p < 5; ++p) dst[(size_t)p * n] = x[q][p];
        }
    }
}

__global__ void k_cursor_reset(int* cur, int* look, int* used, int* left, int spin, int W, int Q, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < 2 * W) cur[i] = 0;
    if (i == 0) {
        used[spin] = 0;
        left[spin] = 0;
    }
    if (i < W) {
        const int q1 = Q < n ? Q : n, q2 = 2 * Q < n ? 2 * Q : n;
        look[(size_t)i * 2] = 0;
        look[(size_t)i * 2 + 1] = q1;
        look[((size_t)W + i) * 2] = q1;
        look[((size_t)W + i) * 2 + 1] = q2;
    }
}

int batch_rounds(int n, int K) { return (n + K - 1) / K; }

// Candidates per round: about k / acceptance for acceptance near 0.35, so that
// a round usually closes on k accepted moves rather than on running out.
int batch_candidates(int n, int K)
{
    int q = 3 * K;
    if (q > kMaxCand) q = kMaxCand;
    if (q < 2) q = 2;
    return q < n ? q : n;
}

template <typename T>
void launch_batch_stencils(const CrowdView<T>& v, int spin, int par, bool block_start, hipStream_t s)
{
    if (block_start)
        hipLaunchKernelGGL(k_cursor_reset, dim3((2 * v.W + 255) / 256), dim3(256), 0, s, v.cur, v.look, v.used, v.left,
                           spin, v.W, v.Q, v.n);
    hipLaunchKernelGGL(k_stencils<T>, dim3((v.W * v.Q + kBlock / 64 - 1) / (kBlock / 64)), dim3(kBlock), 0, s, v, spin,
                       par);
}

int device_cu_count()
{
    static int cus = 0;
    if (!cus) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
            cus = 256;
    }
    return cus;
}

int batch_vgl_blocks_per_cu(int n, int elem_bytes, int request)
{
    if (request > 0) return request;
    return vgl_groups(n, elem_bytes) >= 64 ? kVglWaveBlocksPerCU : kVglBlocksPerCU;
}

template <typename T>
void launch_batch_vgl(const CrowdView<T>& v, int spin, int par, bool beside, hipStream_t s)
{
    const int groups = vgl_groups(v.n, sizeof(T));
    const int per_cu = beside ? batch_vgl_blocks_per_cu(v.n, sizeof(T), v.vgl_wg) : kVglBlocksPerCUAlone;
    if (groups >= 64) {
        const int items = v.W * v.Q * ((groups + 63) / 64);
        const int nb = std::min((items + kBlock / 64 - 1) / (kBlock / 64), per_cu * device_cu_count());
        hipLaunchKernelGGL(k_prop_vgl_wave<T>, dim3(nb), dim3(kBlock), 0, s, v, spin, par);
        return;
    }
    const int pp = kVglSmallPP;
    const int nchunk = (v.W * v.Q + pp - 1) / pp;
    const int nb = std::min(nchunk, per_cu * device_cu_count());
    const size_t lds = (size_t)pp * (64 * sizeof(size_t) + 64 * 5 * sizeof(T)) + 4 * sizeof(int);
    hipLaunchKernelGGL(k_prop_vgl<T>, dim3(nb), dim3(vgl_small_threads(v.n, sizeof(T))), lds, s, v, spin, pp, par);
}

template <typename T>
void launch_batch_jd(const CrowdView<T>& v, int spin, hipStream_t s)
{
    const int per = (v.Q + kJdCand - 1) / kJdCand;
    hipLaunchKernelGGL(k_jd<T>, dim3(v.W * per), dim3(kBlock), 0, s, v, spin);
}

template <typename T>
void launch_batch_rows(const CrowdView<T>& v, int spin, hipStream_t s)
{
    if (!v.ub) return;
    hipLaunchKernelGGL(k_rows<T>, dim3(xcd_grid(v.W, (v.n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, v, spin);
}

template <typename T>
void launch_batch_pmat(const CrowdView<T>& v, int spin, hipStream_t s)
{
    const int pb = (v.Q + kPB - 1) / kPB;
    if (pb >= kPTJ)  // a block row of at least kPTJ blocks: kPTJ per workgroup
        hipLaunchKernelGGL((k_pmat<T, kPTJ>), dim3(xcd_grid(v.W, pb * ((pb + kPTJ - 1) / kPTJ))), dim3(kBlock), 0, s, v,
                           spin);
    else
        hipLaunchKernelGGL((k_pmat<T, 1>), dim3(xcd_grid(v.W, pb * pb)), dim3(kBlock), 0, s, v, spin);
}

template <typename T>
void launch_batch_decide(const CrowdView<T>& v, int spin, int par, int round, hipStream_t s)
{
    static bool lds_set = false;  // opt in to more than 64 KB of LDS, once per type
    if (!lds_set) {
        (void)hipFuncSetAttribute((const void*)k_decide<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)sizeof(DecideLds));
        lds_set = true;
    }
    hipLaunchKernelGGL(k_decide<T>, dim3(v.W), dim3(kBlock), sizeof(DecideLds), s, v, spin, par, round);
}

template <typename T>
void launch_batch_cols(const CrowdView<T>& v, int spin, hipStream_t s)
{
    hipLaunchKernelGGL(k_cols<T>, dim3(xcd_grid(v.W, (v.n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, v, spin);
}

template void launch_batch_stencils<float>(const CrowdView<float>&, int, int, bool, hipStream_t);
template void launch_batch_stencils<double>(const CrowdView<double>&, int, int, bool, hipStream_t);
template void launch_batch_vgl<float>(const CrowdView<float>&, int, int, bool, hipStream_t);
template void launch_batch_vgl<double>(const CrowdView<double>&, int, int, bool, hipStream_t);
template void launch_batch_jd<float>(const CrowdView<float>&, int, hipStream_t);
template void launch_batch_jd<double>(const CrowdView<double>&, int, hipStream_t);
template void launch_batch_rows<float>(const CrowdView<float>&, int, hipStream_t);
template void launch_batch_rows<double>(const CrowdView<double>&, int, hipStream_t);
template void launch_batch_pmat<float>(const CrowdView<float>&, int, hipStream_t);
template void launch_batch_pmat<double>(const CrowdView<double>&, int, hipStream_t);
template void launch_batch_cols<float>(const CrowdView<float>&, int, hipStream_t);
template void launch_batch_cols<double>(const CrowdView<double>&, int, hipStream_t);
template void launch_batch_decide<float>(const CrowdView<float>&, int, int, int, hipStream_t);
template void launch_batch_decide<double>(const CrowdView<double>&, int, int, int, hipStream_t);

}  // namespace cq
