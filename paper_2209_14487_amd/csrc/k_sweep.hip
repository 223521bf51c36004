// Whole-sweep kernel for small N: one workgroup per walker runs every move of a
// VMC sweep (both spin blocks, electrons in order) in one launch: the propose,
// ratio and accept steps of Alg. 1 and, after each accepted move, the
// Sherman-Morrison update of the walker's inverse (delay rank 1).  The walker's
// two inverses and positions stay in LDS for the whole sweep, so a sweep costs
// one launch instead of a handful per move; that is what limits small systems
// (N = 32 and below), where a move's arithmetic is a few microseconds.
//
// Per move e of spin s, electron a (M = rows of the inverse, M[b] = A^-1 e_b):
//   r'      = wrap(r_e + sigma z)                 (Philox stream of the move)
//   u       = phi(r'), grad, Laplacian            (tricubic B-spline, 64 points)
//   rho     = u . M[a]                            (exact products, FP64 sum)
//   dlnJ    = sum_{m != e} u(|r' - r_m|) - u(|r_e - r_m|)   (FP64)
//             + sum_I u1(|r' - R_I|) - u1(|r_e - R_I|)   (one-body terms)
//   accept  if u_e < rho^2 exp(2 dlnJ)
//   update  M[b] <- M[b] - ((u . M[b]) - delta_ab) / rho * M_old[a]   for every b
//           (FP64 from the stored values, then stored in T)
// A VMC proposal depends only on its own electron, which has not moved yet in the
// sweep when its turn comes, so the kernel takes the moves in blocks: first the
// proposals, uniforms and orbital rows of a whole block, in parallel (each wave
// gathers up to 4 proposals at once: lanes = (proposal, orbital group of 16 bytes,
// stencil x-plane), the 4 planes of a group summed by DPP quad swaps), then the
// decisions in electron order.  Every wave forms the same ratio and Jastrow sums,
// so a rejected move needs no barrier; an accepted one updates the inverse one
// row per wave pass between two barriers.  The accepted orbital rows go to the
// walker's VGL rows in global memory (the local energy and the recompute read
// them); the inverses and positions go back at the end of the sweep.
#include "cq_device.h"
#include "cq_internal.h"
#include "cq_jastrow.h"
#include "cq_stencil.h"

namespace cq {

namespace {

template <int CTRL, typename T>
__device__ __forceinline__ T quad_add(T x)
{
    return x + dpp::mov<CTRL>(x);
}

}  // namespace

// Proposals gathered together by one wave: as many as its 64 lanes hold at 4 x-planes x
// (N / VEC) orbital groups each, at most 4.
constexpr int kSweepPerWave = 4;
// LDS for the orbital rows of a block of proposals
constexpr int kSweepRowBytes = 64 * 1024;

__host__ __device__ inline int sweep_per_wave(int n, int elem_bytes)
{
    const int items = 4 * (n / (16 / elem_bytes));
    return items >= 64 ? 1 : (64 / items < kSweepPerWave ? 64 / items : kSweepPerWave);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_sweep(CrowdView<T> v, int B)
{
    constexpr int VEC = 16 / sizeof(T);
    constexpr int NW = kBlock / 64;
    // M [2][N][N] and rows [B][5][N] in T, then per wave and proposal gathered at once the
    // stencil: offsets [NW][per_wave][64] and weights [NW][per_wave][64 * 5]
    extern __shared__ unsigned char sweep_lds[];
    __shared__ double s_R[2 * kSweepMaxN][3];
    __shared__ double s_rp[2 * kSweepMaxN][3];  // proposals of the block's moves
    __shared__ double s_u[2 * kSweepMaxN];      // their Metropolis uniforms
    T* Msh = reinterpret_cast<T*>(sweep_lds);
    const int w = blockIdx.x;
    if (w >= v.W) return;
    const int n = v.n, ne = v.ne, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    T* rows = Msh + (size_t)2 * n * n;
    const int groups = n / VEC, items = 4 * groups;  // items of one proposal
    const int per_wave = sweep_per_wave(n, sizeof(T));
    size_t* st_idx = reinterpret_cast<size_t*>(rows + (size_t)B * 5 * n) + (size_t)wave * per_wave * 64;
    T* st_w = reinterpret_cast<T*>(reinterpret_cast<size_t*>(rows + (size_t)B * 5 * n) + (size_t)NW * per_wave * 64) +
              (size_t)wave * per_wave * 64 * 5;
    const int passes = (items + 63) / 64;
    T* Mg = v.M + (size_t)w * 2 * n * n;
    for (int i = tid; i < 2 * n * n; i += kBlock) Msh[i] = Mg[i];
    for (int i = tid; i < ne * 3; i += kBlock) s_R[i / 3][i % 3] = v.R[(size_t)w * ne * 3 + i];

    const uint32_t step = v.prm->step, uid = v.uid[w];
    const int rs = v.prm->rec_sweep;
    const double sigma = v.prm->sigma;
    double ld[2] = {0.0, 0.0};
    int flip[2] = {0, 0};
    long long nacc = 0;
    for (int e0 = 0; e0 < ne; e0 += B) {
        const int nb = min(B, ne - e0);
        __syncthreads();  // the previous block's rows and proposals are no longer read
        // proposals (an electron has not moved yet in the sweep when its turn comes, so every
        // proposal of the block is known now) and the uniforms, one move per thread
        if (tid < nb) {
            const int e = e0 + tid;
            double z[3];
            gauss3(v.seed, uid, step, (uint32_t)e, z);
#pragma unroll
            for (int k = 0; k < 3; ++k) s_rp[tid][k] = wrap_box(s_R[e][k] + sigma * z[k], v.L);
            s_u[tid] = accept_uniform(v.seed, uid, step, (uint32_t)e);
        }
        __syncthreads();
        // orbital rows of the block's proposals: wave `wave` takes per_wave of them at a time,
        // their stencils in its own LDS, lane = (proposal, group, x-plane)
        for (int m0 = wave * per_wave; m0 < nb; m0 += NW * per_wave) {
            for (int i = 0; i < per_wave; ++i)
                if (m0 + i < nb) stencil_entry<T>(v, s_rp[m0 + i], lane, st_idx + i * 64, st_w + i * 64 * 5);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            for (int pass = 0; pass < passes; ++pass) {
                const int item = lane + 64 * pass, i = item / items, r = item - i * items;
                const bool live = i < per_wave && m0 + i < nb;
                const int g = r >> 2, p = r & 3, j0 = g * VEC;
                T acc[5][VEC];
#pragma unroll
                for (int k = 0; k < 5; ++k)
#pragma unroll
                    for (int q = 0; q < VEC; ++q) acc[k][q] = (T)0;
                if (live) {
                    const size_t* sidx = st_idx + i * 64;
                    const T* sw = st_w + i * 64 * 5;
                    T vals[16][VEC];
#pragma unroll
                    for (int q = 0; q < 16; ++q) load16(v.table + sidx[p * 16 + q] + j0, vals[q]);
#pragma unroll
                    for (int q = 0; q < 16; ++q) {
                        const T* wq = sw + (p * 16 + q) * 5;
#pragma unroll
                        for (int k = 0; k < 5; ++k)
#pragma unroll
                            for (int c = 0; c < VEC; ++c) acc[k][c] += wq[k] * vals[q][c];
                    }
                }
                // the 4 x-planes of a group are the 4 lanes of a quad
#pragma unroll
                for (int k = 0; k < 5; ++k)
#pragma unroll
                    for (int c = 0; c < VEC; ++c) {
                        T x = quad_add<dpp::kQuadXor1>(acc[k][c]);
                        acc[k][c] = quad_add<dpp::kQuadXor2>(x);
                    }
                if (live && p == 0) {
                    T* row = rows + (size_t)(m0 + i) * 5 * n;
#pragma unroll
                    for (int k = 0; k < 5; ++k)
#pragma unroll
                        for (int c = 0; c < VEC; ++c) row[k * n + j0 + c] = acc[k][c];
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();  // the next proposals' stencils overwrite this wave's
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
        __syncthreads();
        // the decisions in electron order.  Every wave forms the same ratio and Jastrow sums
        // (same lanes, same order), so all of them know the decision without a barrier; only
        // an accepted move changes shared state.
        for (int m = 0; m < nb; ++m) {
            const int e = e0 + m, spin = e >= n, a = e - spin * n;
            T* M = Msh + (size_t)spin * n * n;
            const T* u = rows + (size_t)m * 5 * n;
            const double rp[3] = {s_rp[m][0], s_rp[m][1], s_rp[m][2]};
            const double c0 = lane < n ? (double)M[(size_t)a * n + lane] : 0.0;
            const double u0 = lane < n ? (double)u[lane] : 0.0;
            const double rho = wave_sum(u0 * c0);
            double dj = 0.0;
            if (v.use_j2) {
                for (int o = lane; o < ne; o += 64) {
                    if (o == e) continue;
                    const double aa = ((o >= n) == (spin != 0)) ? v.a_par : v.a_anti;
                    double d1[3], d0[3], u1, u0j, du, d2u;
                    min_image(rp, s_R[o], v.L, d1);
                    min_image(s_R[e], s_R[o], v.L, d0);
                    pade(aa, v.b, sqrt(d1[0] * d1[0] + d1[1] * d1[1] + d1[2] * d1[2]), u1, du, d2u);
                    pade(aa, v.b, sqrt(d0[0] * d0[0] + d0[1] * d0[1] + d0[2] * d0[2]), u0j, du, d2u);
                    dj += u1 - u0j;
                }
            }
            if (v.n_ions) dj += j1_delta(v, rp, s_R[e], lane, 64);
            if (v.use_j2 || v.n_ions) dj = wave_sum(dj);
            const double prob = rho * rho * exp(2.0 * dj);
            int acc = s_u[m] < prob;
            const size_t ri = ((size_t)rs * ne + e) * v.Wcap + w;
            if (v.forced && rs < v.prm->forced_cap && v.forced[ri] < 2) acc = v.forced[ri] != 0;
            if (tid == 0 && rs < v.prm->rec_cap) {
                v.rec_rho[ri] = rho;
                v.rec_dlnj[ri] = dj;
                v.rec_prob[ri] = prob;
                v.rec_acc[ri] = (uint8_t)acc;
            }
            if (!acc) continue;
            __syncthreads();  // every wave holds the old column c0 before any row changes
            // Sherman-Morrison: M[b] -= ((u . M[b]) - delta_ab) / rho * c0, one row per wave pass
            const double irho = 1.0 / rho;
            for (int b = wave; b < n; b += NW) {
                const double mb = lane < n ? (double)M[(size_t)b * n + lane] : 0.0;
                const double x = wave_sum(u0 * mb);
                const double beta = (x - (b == a ? 1.0 : 0.0)) * irho;
                if (lane < n) M[(size_t)b * n + lane] = (T)(mb - beta * c0);
            }
            // the accepted rows, the position and the log|det| bookkeeping
            T* dst = v.VGL + (((size_t)w * 2 + spin) * n + a) * 5 * (size_t)n;
            for (int i = tid; i < 5 * n; i += kBlock) dst[i] = u[i];
            if (tid == 0) {
                ld[spin] += log(fabs(rho));
                if (rho < 0.0) flip[spin] ^= 1;
                nacc += 1;
            }
            if (tid < 3) s_R[e][tid] = rp[tid];
            __syncthreads();  // updated rows and position are seen by the next move
        }
    }

    __syncthreads();
    for (int i = tid; i < 2 * n * n; i += kBlock) Mg[i] = Msh[i];
    for (int i = tid; i < ne * 3; i += kBlock) v.R[(size_t)w * ne * 3 + i] = s_R[i / 3][i % 3];
    if (tid == 0) {
        for (int s = 0; s < 2; ++s) {
            v.logdet[w * 2 + s] += ld[s];
            if (flip[s]) v.sign[w * 2 + s] = -v.sign[w * 2 + s];
        }
        v.nacc[w] += nacc;
        v.nprop[w] += ne;
    }
}

// Moves per block: as many as the row budget holds (all of them for N <= 32 in FP32).
inline int sweep_block(int n, int ne, int elem_bytes)
{
    const int b = kSweepRowBytes / (5 * n * elem_bytes);
    return b >= ne ? ne : (b < 1 ? 1 : b);
}

template <typename T>
void launch_sweep(const CrowdView<T>& v, hipStream_t s)
{
    const int B = sweep_block(v.n, v.ne, sizeof(T));
    const int pw = sweep_per_wave(v.n, sizeof(T));
    const size_t lds = sizeof(T) * (2 * (size_t)v.n * v.n + (size_t)B * 5 * v.n) +
                       (size_t)(kBlock / 64) * pw * 64 * (sizeof(size_t) + 5 * sizeof(T));
    static size_t opted = 64 * 1024;  // dynamic LDS the kernel has been opted in to (per type)
    if (lds > opted) {
        (void)hipFuncSetAttribute((const void*)k_sweep<T>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        opted = lds;
    }
    hipLaunchKernelGGL(k_sweep<T>, dim3(v.W), dim3(kBlock), lds, s, v, B);
}

template void launch_sweep<float>(const CrowdView<float>&, hipStream_t);
template void launch_sweep<double>(const CrowdView<double>&, hipStream_t);

}  // namespace cq
