// Walker-resident window kernel: one workgroup per walker performs the k
// consecutive moves of one update window (the per-particle steps of Alg. 1 for k
// particles),
// keeping the window's bookkeeping in LDS and synchronising only inside the
// workgroup.  The window's accepted moves are left in global memory for the
// rank-k update kernel that follows.
//
// Work split for one move: item (g, p) = (orbital group of 16 bytes, stencil
// x-plane p); the 4 planes of a group sit in 4 consecutive lanes and are summed
// with two DPP quad swaps.  The lanes of a quad then share the window dots:
// lane p takes the window slots m = p (mod 4).
#include "cq_device.h"
#include "cq_internal.h"
#include "cq_jastrow.h"

namespace cq {

namespace {

template <int CTRL, typename T>
__device__ __forceinline__ T quad_add(T x)
{
    return x + dpp::mov<CTRL>(x);
}

}  // namespace

// Partial-sum slots reduced over the workgroup for one move: u . c0, the
// Jastrow difference, then u . c_m and u_m . c0 for m < cnt.
constexpr int kWinVals = 2 + 2 * kMaxDelay;

// Stencil of the proposal r' for one move, shared by the workgroup: for stencil
// point q of x-plane p (index 16 p + q), the table offset of the point and its
// five weights (value, d/dx, d/dy, d/dz, Laplacian).  One wave fills it, lane l
// taking (p, q) = (l / 16, l % 16).
template <typename T>
__device__ __forceinline__ void stencil_lane(const CrowdView<T>& v, const double rp[3], int l, size_t* sidx,
                                             T* sw)
{
    const int G = v.G;
    const AxisW<T> ax = axis_weights<T>(rp[0], v.L, G);
    const AxisW<T> ay = axis_weights<T>(rp[1], v.L, G);
    const AxisW<T> az = axis_weights<T>(rp[2], v.L, G);
    const int p = l >> 4, q = l & 15, bb = q >> 2, cc = q & 3;
    T bx = ax.b[0], dx = ax.d1[0], d2x = ax.d2[0];
    if (p == 1) { bx = ax.b[1]; dx = ax.d1[1]; d2x = ax.d2[1]; }
    if (p == 2) { bx = ax.b[2]; dx = ax.d1[2]; d2x = ax.d2[2]; }
    if (p == 3) { bx = ax.b[3]; dx = ax.d1[3]; d2x = ax.d2[3]; }
    T by = ay.b[0], dy = ay.d1[0], d2y = ay.d2[0];
    if (bb == 1) { by = ay.b[1]; dy = ay.d1[1]; d2y = ay.d2[1]; }
    if (bb == 2) { by = ay.b[2]; dy = ay.d1[2]; d2y = ay.d2[2]; }
    if (bb == 3) { by = ay.b[3]; dy = ay.d1[3]; d2y = ay.d2[3]; }
    T bz = az.b[0], dz = az.d1[0], d2z = az.d2[0];
    if (cc == 1) { bz = az.b[1]; dz = az.d1[1]; d2z = az.d2[1]; }
    if (cc == 2) { bz = az.b[2]; dz = az.d1[2]; d2z = az.d2[2]; }
    if (cc == 3) { bz = az.b[3]; dz = az.d1[3]; d2z = az.d2[3]; }
    const int jx = (ax.i0 + p + G - 1) % G, jy = (ay.i0 + bb + G - 1) % G, jz = (az.i0 + cc + G - 1) % G;
    sidx[l] = (((size_t)jx * G + jy) * G + jz) * (size_t)v.n_orb;
    sw[l * 5 + 0] = bx * by * bz;
    sw[l * 5 + 1] = dx * by * bz;
    sw[l * 5 + 2] = bx * dy * bz;
    sw[l * 5 + 3] = bx * by * dz;
    sw[l * 5 + 4] = d2x * by * bz + bx * d2y * bz + bx * by * d2z;
}

template <typename T>
__global__ __launch_bounds__(512) void k_window(CrowdView<T> v, int e0, int nmoves)
{
    constexpr int VEC = 16 / sizeof(T);
    __shared__ double s_red[8][kWinVals];
    __shared__ double s_sum[kWinVals];
    __shared__ double s_G[kMaxDelay][kMaxDelay + 1];  // u_m . c_j, j < m
    __shared__ double s_rho[kMaxDelay], s_beta[kMaxDelay];
    __shared__ int s_wel[kMaxDelay];
    __shared__ double s_rp[2][3];
    __shared__ size_t s_idx[2][64];
    __shared__ T s_w[2][64 * 5];
    __shared__ int s_acc;

    const int w = blockIdx.x;
    const int nt = blockDim.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = nt >> 6;
    const int n = v.n, K = v.K;
    const int spin = e0 >= n;
    const int groups = n / VEC, items = 4 * groups;
    const int rounds = (items + nt - 1) / nt;
    const uint32_t step = v.prm->step;
    const int rs = v.prm->rec_sweep;
    const double sigma = v.prm->sigma;
    const bool recording = rs < v.prm->rec_cap, forcing = v.forced && rs < v.prm->forced_cap;
    const T* Mspin = v.M + ((size_t)w * 2 + spin) * n * (size_t)n;
    T* stage = v.stage + (size_t)w * v.QR * 5 * n;
    T* Cb = v.Cbuf + (size_t)w * K * n;
    const int prop_wave = nw > 1 ? 1 : 0;  // the wave that prepares the next move's stencil

    if (wave == 0) {
        double rp[3], z[3];
        gauss3(v.seed, v.uid[w], step, (uint32_t)e0, z);
        for (int k = 0; k < 3; ++k) rp[k] = wrap_box(v.R[((size_t)w * v.ne + e0) * 3 + k] + sigma * z[k], v.L);
        stencil_lane<T>(v, rp, lane, s_idx[0], s_w[0]);
        if (lane == 0) { s_rp[0][0] = rp[0]; s_rp[0][1] = rp[1]; s_rp[0][2] = rp[2]; }
    }
    __syncthreads();

    int cnt = 0;
    for (int mv = 0; mv < nmoves; ++mv) {
        const int e = e0 + mv, a = e - spin * n, buf = mv & 1;
        const double rp[3] = {s_rp[buf][0], s_rp[buf][1], s_rp[buf][2]};
        // this lane's partial sums: d0 (plane 0), dJ, and (x, y) of its slots m = p, p+4, ...
        double d0 = 0.0, dj = 0.0;
        double xs[kMaxDelay / 4], ys[kMaxDelay / 4];
#pragma unroll
        for (int q = 0; q < kMaxDelay / 4; ++q) { xs[q] = 0.0; ys[q] = 0.0; }
        for (int r = 0; r < rounds; ++r) {
            const int item = tid + r * nt;
            const int g = item >> 2, p = item & 3;
            const bool valid = g < groups;
            const int j0 = valid ? g * VEC : 0;  // invalid items read group 0 and discard it
            T c0[VEC];
            load16(Mspin + (size_t)a * n + j0, c0);
            T vals[16][VEC];
#pragma unroll
            for (int q = 0; q < 16; ++q) load16(v.table + s_idx[buf][p * 16 + q] + j0, vals[q]);
            T acc[5][VEC];
#pragma unroll
            for (int k = 0; k < 5; ++k)
#pragma unroll
                for (int i = 0; i < VEC; ++i) acc[k][i] = (T)0;
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const T* wq = &s_w[buf][(p * 16 + q) * 5];
                const T wv = wq[0], wgx = wq[1], wgy = wq[2], wgz = wq[3], wl = wq[4];
#pragma unroll
                for (int i = 0; i < VEC; ++i) {
                    const T x = valid ? vals[q][i] : (T)0;
                    acc[0][i] += wv * x;
                    acc[1][i] += wgx * x;
                    acc[2][i] += wgy * x;
                    acc[3][i] += wgz * x;
                    acc[4][i] += wl * x;
                }
            }
            // sum the 4 planes of the group across the quad: every lane of it gets the total
#pragma unroll
            for (int k = 0; k < 5; ++k)
#pragma unroll
                for (int i = 0; i < VEC; ++i) {
                    acc[k][i] = quad_add<dpp::kQuadXor1>(acc[k][i]);
                    acc[k][i] = quad_add<dpp::kQuadXor2>(acc[k][i]);
                }
            if (valid) {
                if (p == 0) {
                    store16(Cb + (size_t)cnt * n + j0, c0);  // pending slot: old column
                    double s = 0.0;
#pragma unroll
                    for (int i = 0; i < VEC; ++i) s += (double)(acc[0][i] * c0[i]);
                    d0 += s;
                }
                // pending slot: the proposal's orbital rows, one component per lane of the quad
                T* dst = stage + (size_t)cnt * 5 * n + j0;
                if (p == 0) {
                    store16(dst, acc[0]);
                    store16(dst + 4 * (size_t)n, acc[4]);
                }
                if (p == 1) store16(dst + 1 * (size_t)n, acc[1]);
                if (p == 2) store16(dst + 2 * (size_t)n, acc[2]);
                if (p == 3) store16(dst + 3 * (size_t)n, acc[3]);
                // window dots of this lane's slots, loaded 4 at a time (indices clamped
                // into the buffer, unused slots masked)
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    if (16 * h >= cnt) break;  // slots 16.. only matter past 16 accepted moves
                    T cm[4][VEC], um[4][VEC];
#pragma unroll
                    for (int qq = 0; qq < 4; ++qq) {
                        const int ms = min(p + 4 * (qq + 4 * h), K - 1);
                        load16(Cb + (size_t)ms * n + j0, cm[qq]);
                        load16(stage + ((size_t)ms * 5) * n + j0, um[qq]);
                    }
#pragma unroll
                    for (int qq = 0; qq < 4; ++qq) {
                        double sx = 0.0, sy = 0.0;
#pragma unroll
                        for (int i = 0; i < VEC; ++i) {
                            sx += (double)(acc[0][i] * cm[qq][i]);
                            sy += (double)(um[qq][i] * c0[i]);
                        }
                        const bool used = p + 4 * (qq + 4 * h) < cnt;
                        xs[qq + 4 * h] += used ? sx : 0.0;
                        ys[qq + 4 * h] += used ? sy : 0.0;
                    }
                }
            }
        }
        // Jastrow difference over the other electrons (positions loaded 4 at a time)
        if (v.use_j2) {
            double re[3];
            for (int k = 0; k < 3; ++k) re[k] = v.R[((size_t)w * v.ne + e) * 3 + k];
            for (int t0 = 0; t0 * nt < v.ne; t0 += 4) {
                double rm[4][3];
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int mm = min(tid + (t0 + t) * nt, v.ne - 1);
#pragma unroll
                    for (int k = 0; k < 3; ++k) rm[t][k] = v.R[((size_t)w * v.ne + mm) * 3 + k];
                }
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int mm = tid + (t0 + t) * nt;
                    if (mm < v.ne && mm != e) {
                        const double aa = ((mm >= n) == (spin != 0)) ? v.a_par : v.a_anti;
                        double d1[3], dd[3], u1, u0, du, d2u;
                        min_image(rp, rm[t], v.L, d1);
                        min_image(re, rm[t], v.L, dd);
                        pade(aa, v.b, sqrt(d1[0] * d1[0] + d1[1] * d1[1] + d1[2] * d1[2]), u1, du, d2u);
                        pade(aa, v.b, sqrt(dd[0] * dd[0] + dd[1] * dd[1] + dd[2] * dd[2]), u0, du, d2u);
                        dj += u1 - u0;
                    }
                }
            }
        }
        if (v.n_ions) {  // one-body terms, the centres shared out over the threads
            double re[3];
            for (int k = 0; k < 3; ++k) re[k] = v.R[((size_t)w * v.ne + e) * 3 + k];
            dj += j1_delta(v, rp, re, tid, nt);
        }
        // the next move's proposal and stencil (electron e+1 has not moved in this window)
        if (wave == prop_wave && mv + 1 < nmoves) {
            double rn[3], z[3];
            gauss3(v.seed, v.uid[w], step, (uint32_t)(e + 1), z);
            for (int k = 0; k < 3; ++k) rn[k] = wrap_box(v.R[((size_t)w * v.ne + e + 1) * 3 + k] + sigma * z[k], v.L);
            stencil_lane<T>(v, rn, lane, s_idx[buf ^ 1], s_w[buf ^ 1]);
            if (lane == 0) { s_rp[buf ^ 1][0] = rn[0]; s_rp[buf ^ 1][1] = rn[1]; s_rp[buf ^ 1][2] = rn[2]; }
        }
        // workgroup sums in a fixed order: waves, then the 4 lane classes of the slots
        {
            const double t0 = wave_sum(d0), t1 = wave_sum(dj);
            if (lane == 0) { s_red[wave][0] = t0; s_red[wave][1] = t1; }
#pragma unroll
            for (int q = 0; q < kMaxDelay / 4; ++q) {
                if (4 * q >= cnt) break;  // wave-uniform
#pragma unroll
                for (int p = 0; p < 4; ++p) {
                    const int m = p + 4 * q;
                    const bool own = (lane & 3) == p;
                    const double tx = wave_sum(own ? xs[q] : 0.0);
                    const double ty = wave_sum(own ? ys[q] : 0.0);
                    if (lane == 0 && m < cnt) {
                        s_red[wave][2 + m] = tx;
                        s_red[wave][2 + kMaxDelay + m] = ty;
                    }
                }
            }
        }
        __syncthreads();
        // ratio and decision (wave 0)
        if (wave == 0) {
            for (int i = lane; i < kWinVals; i += 64) {
                const bool need = i < 2 || (i >= 2 && i < 2 + cnt) || (i >= 2 + kMaxDelay && i < 2 + kMaxDelay + cnt);
                double s = 0.0;
                if (need)
                    for (int ww = 0; ww < nw; ++ww) s += s_red[ww][i];
                s_sum[i] = s;
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
            const bool mine = lane < cnt;
            const double x_l = mine ? s_sum[2 + lane] : 0.0;
            const double rinv = mine ? 1.0 / s_rho[lane] : 0.0;
            double t = mine ? s_sum[2 + kMaxDelay + lane] : 0.0, my_beta = 0.0;
            for (int mm = 0; mm < cnt; ++mm) {
                const double bm = dpp::lane(t, mm) * dpp::lane(rinv, mm);
                if (lane == mm) my_beta = bm;
                if (lane > mm && mine) t -= bm * s_G[lane][mm];
            }
            const double rho = s_sum[0] - wave_sum(mine ? my_beta * x_l : 0.0);
            const double dlnj = s_sum[1];
            const double prob = rho * rho * exp(2.0 * dlnj);
            const double u = accept_uniform(v.seed, v.uid[w], step, (uint32_t)e);
            int acc = u < prob;
            const size_t ri = ((size_t)rs * v.ne + e) * v.Wcap + w;
            if (forcing && v.forced[ri] < 2) acc = v.forced[ri] != 0;
            if (lane == 0 && recording) {
                v.rec_rho[ri] = rho;
                v.rec_dlnj[ri] = dlnj;
                v.rec_prob[ri] = prob;
                v.rec_acc[ri] = (uint8_t)acc;
            }
            if (acc) {
                if (mine) {
                    s_beta[lane] = my_beta;
                    s_G[cnt][lane] = x_l;  // u . c_lane
                }
                if (lane == 0) {
                    s_rho[cnt] = rho;
                    s_wel[cnt] = a;
                    for (int k = 0; k < 3; ++k) v.R[((size_t)w * v.ne + e) * 3 + k] = rp[k];
                    v.logdet[w * 2 + spin] += log(fabs(rho));
                    if (rho < 0.0) v.sign[w * 2 + spin] = -v.sign[w * 2 + spin];
                    v.nacc[w] += 1;
                }
            }
            if (lane == 0) {
                v.nprop[w] += 1;
                s_acc = acc;
            }
        }
        __syncthreads();
        if (s_acc) {
            // the accepted move's column: c = c0 - sum_m beta_m c_m (slots loaded in
            // batches of 8, indices clamped into the buffer, unused ones masked)
            for (int g = tid; g < groups; g += nt) {
                const int j0 = g * VEC;
                T cn[VEC];
                load16(Cb + (size_t)cnt * n + j0, cn);
#pragma unroll
                for (int b8 = 0; b8 < kMaxDelay; b8 += 8) {
                    if (b8 >= cnt) break;
                    T cmv[8][VEC];
#pragma unroll
                    for (int q = 0; q < 8; ++q) load16(Cb + (size_t)min(b8 + q, K - 1) * n + j0, cmv[q]);
#pragma unroll
                    for (int q = 0; q < 8; ++q) {
                        if (b8 + q >= cnt) break;  // unused slots may hold anything (even NaN): skip, never scale by 0
                        const T bm = (T)s_beta[b8 + q];
#pragma unroll
                        for (int i = 0; i < VEC; ++i) cn[i] -= bm * cmv[q][i];
                    }
                }
                store16(Cb + (size_t)cnt * n + j0, cn);
            }
            ++cnt;
        }
        __syncthreads();
    }
    // hand the window to the update kernel
    if (tid < cnt) {
        v.welec[(size_t)w * K + tid] = s_wel[tid];
        v.wslot[(size_t)w * K + tid] = tid;
        v.wrho[(size_t)w * K + tid] = s_rho[tid];
    }
    for (int idx = tid; idx < cnt * cnt; idx += nt) {
        const int i = idx / cnt, j = idx % cnt;
        if (j < i) v.wG[((size_t)w * K + i) * K + j] = s_G[i][j];
    }
    if (tid == 0) v.cnt[(size_t)2 * v.W + w] = cnt;
}

int window_threads(int n, int elem_bytes)
{
    const int items = 4 * n / (16 / elem_bytes);
    int nt = ((items + 63) / 64) * 64;
    return nt > 512 ? 512 : nt;
}

template <typename T>
void launch_window(const CrowdView<T>& v, int e0, int nmoves, hipStream_t s)
{
    hipLaunchKernelGGL(k_window<T>, dim3(v.W), dim3(window_threads(v.n, sizeof(T))), 0, s, v, e0, nmoves);
}

template void launch_window<float>(const CrowdView<float>&, int, int, hipStream_t);
template void launch_window<double>(const CrowdView<double>&, int, int, hipStream_t);

}  // namespace cq
