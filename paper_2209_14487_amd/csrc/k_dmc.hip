// Diffusion Monte Carlo: drift-diffusion moves and branching (paper Alg. 1 with
// its proposal read as a drift-diffusion step, then reweighting / branching).
//
// A DMC proposal moves electron e by
//     delta = tau v(r_e) + sqrt(tau) z,      v = grad ln|Psi| at the current r_e,
// and is accepted with the Metropolis-Hastings probability of the drifted
// Gaussian transition (Green's function) times |Psi'/Psi|^2:
//     P = rho_D^2 exp(2 dlnJ) exp(-(|delta + tau v'|^2 - |delta - tau v|^2) / (2 tau)),
// v' = grad ln|Psi| at r'; moves that change the sign of the determinant are
// rejected (fixed node).  The drift depends on the inverse column of e after
// every earlier move, so DMC proposals cannot be evaluated ahead of time: this
// kernel runs one walker per workgroup and its k moves in order, like the
// walker-resident VMC window kernel, with two phases per move.
//   A  drift at r_e: g_e . c_e with the window-corrected column
//      c_e = c0_e - sum_m beta_m c_m (beta from the accepted rows u_m against
//      c0_e), plus the Jastrow gradient; then the proposal and its stencil.
//   B  orbital rows at r', ratio rho = u . c_e, drift at r' = (grad u . c_e) /
//      rho plus the Jastrow gradient at r', the acceptance, and on acceptance
//      the new column for the window.
// Window dot products are taken one wave per window slot over full rows; the
// row vectors of the move sit in LDS.
//
// Branching after every generation (all walkers of the crowd's population):
//   E_c = E_L clipped to [E_T - ecut, E_T + ecut], ecut = 0.2 sqrt(Ne / tau)
//   w = exp(-tau ((E_c(old) + E_c(new)) / 2 - E_T)),  m = min(3, floor(w + u_b))
//   E_est = sum w E_L / sum w,  E_T <- E_est - ln(N_new / N_target) / tau
// Children follow their parent in population order; copy 0 keeps the parent's
// uid, copy c >= 1 gets Philox(uid, step, c, block 4) word 0.  The sums and the
// prefix sum run in population order (one thread), as the definition reads.
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

// Stencil of position rp for lane l (entry 16 x + 4 y + z): table offset and the
// five weights, into LDS.
template <typename T>
__device__ __forceinline__ void dmc_stencil(const CrowdView<T>& v, const double rp[3], int l, size_t* sidx, T* sw)
{
    const int G = v.G;
    const AxisW<T> ax = axis_weights<T>(rp[0], v.L, G);
    const AxisW<T> ay = axis_weights<T>(rp[1], v.L, G);
    const AxisW<T> az = axis_weights<T>(rp[2], v.L, G);
    const int p = l >> 4, yy = (l >> 2) & 3, zz = l & 3;
    T bx = ax.b[0], dx = ax.d1[0], d2x = ax.d2[0];
    if (p == 1) { bx = ax.b[1]; dx = ax.d1[1]; d2x = ax.d2[1]; }
    if (p == 2) { bx = ax.b[2]; dx = ax.d1[2]; d2x = ax.d2[2]; }
    if (p == 3) { bx = ax.b[3]; dx = ax.d1[3]; d2x = ax.d2[3]; }
    T by = ay.b[0], dy = ay.d1[0], d2y = ay.d2[0];
    if (yy == 1) { by = ay.b[1]; dy = ay.d1[1]; d2y = ay.d2[1]; }
    if (yy == 2) { by = ay.b[2]; dy = ay.d1[2]; d2y = ay.d2[2]; }
    if (yy == 3) { by = ay.b[3]; dy = ay.d1[3]; d2y = ay.d2[3]; }
    T bz = az.b[0], dz = az.d1[0], d2z = az.d2[0];
    if (zz == 1) { bz = az.b[1]; dz = az.d1[1]; d2z = az.d2[1]; }
    if (zz == 2) { bz = az.b[2]; dz = az.d1[2]; d2z = az.d2[2]; }
    if (zz == 3) { bz = az.b[3]; dz = az.d1[3]; d2z = az.d2[3]; }
    const int jx = (ax.i0 + p + G - 1) % G, jy = (ay.i0 + yy + G - 1) % G, jz = (az.i0 + zz + G - 1) % G;
    sidx[l] = (((size_t)jx * G + jy) * G + jz) * (size_t)v.n_orb;
    sw[l * 5 + 0] = bx * by * bz;
    sw[l * 5 + 1] = dx * by * bz;
    sw[l * 5 + 2] = bx * dy * bz;
    sw[l * 5 + 3] = bx * by * dz;
    sw[l * 5 + 4] = d2x * by * bz + bx * d2y * bz + bx * by * d2z;
}

// Jastrow gradient of electron e at position r against the current positions of
// the other electrons and the one-body centres, and (with r0) the difference
// ln J(r) - ln J(r0); this thread's share of the electrons and centres (tid, tid + nt, ...).
template <typename T>
__device__ __forceinline__ void j2_part(const CrowdView<T>& v, int w, int e, const double r[3], const double* r0,
                                        int tid, int nt, double g[3], double& dj)
{
    const int spin = e >= v.n;
    if (v.n_ions) {
        double lap = 0.0;
        (void)j1_at(v, r, tid, nt, g, lap);
        if (r0) dj += j1_delta(v, r, r0, tid, nt);
    }
    for (int m = tid; v.use_j2 && m < v.ne; m += nt) {
        if (m == e) continue;
        const double* rm = v.R + ((size_t)w * v.ne + m) * 3;
        const double aa = ((m >= v.n) == (spin != 0)) ? v.a_par : v.a_anti;
        double d[3], u, du, d2u;
        min_image(r, rm, v.L, d);
        const double rr = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        pade(aa, v.b, rr, u, du, d2u);
#pragma unroll
        for (int c = 0; c < 3; ++c) g[c] += du * d[c] / rr;
        if (r0) {
            double d0[3], u0;
            min_image(r0, rm, v.L, d0);
            pade(aa, v.b, sqrt(d0[0] * d0[0] + d0[1] * d0[1] + d0[2] * d0[2]), u0, du, d2u);
            dj += u - u0;
        }
    }
}

// Sum of a value over the workgroup in a fixed order (waves, then wave index);
// every thread gets the total.  `slot` picks one of 8 LDS columns.
__device__ __forceinline__ double block_sum(double x, double (*red)[8], int slot, int lane, int wave, int nw)
{
    x = wave_sum(x);
    if (lane == 0) red[wave][slot] = x;
    __syncthreads();
    double s = 0.0;
    for (int q = 0; q < nw; ++q) s += red[q][slot];
    return s;
}

}  // namespace

// The moves of one window of walker w (any system: every size comes from the view).
template <typename T>
__device__ __forceinline__ void window_dmc_body(const CrowdView<T>& v, const int w, int e0, int nmoves)
{
    constexpr int VEC = 16 / sizeof(T);
    constexpr int D = kMaxDelay;
    extern __shared__ unsigned char dsm[];
    const int n = v.n, K = v.K;
    T* s_c0 = reinterpret_cast<T*>(dsm);  // [N] inverse column of e at window start
    T* s_g = s_c0 + n;                     // [3][N] gradient rows of e at r_e
    T* s_u = s_g + 3 * (size_t)n;          // [4][N] value and gradient rows at r'
    __shared__ double s_y[D], s_gm[D][3], s_x[D], s_xg[D][3], s_d[4];
    __shared__ double s_red[kBlock / 64][8];
    __shared__ double s_G[D][D + 1], s_rho[D], s_beta[D];
    __shared__ int s_wel[D];
    __shared__ double s_rp[3], s_delta[3], s_v[3], s_jg[4];
    __shared__ size_t s_idx[64];
    __shared__ T s_w[64 * 5];
    __shared__ int s_acc;

    if (w >= v.W) return;
    const int nt = blockDim.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = nt >> 6;
    const int spin = e0 >= n;
    const int groups = n / VEC, items = 4 * groups;
    const uint32_t step = v.prm->step;
    const double tau = v.prm->tau, sqrt_tau = sqrt(tau);
    // parity mode: the generation's records and forced decisions (walker stride Wcap)
    const int rs = v.prm->rec_sweep;
    const bool recording = rs < v.prm->rec_cap, forcing = v.forced && rs < v.prm->forced_cap;
    const T* Mspin = v.M + ((size_t)w * 2 + spin) * n * (size_t)n;
    const T* VGLspin = v.VGL + ((size_t)w * 2 + spin) * n * 5 * (size_t)n;
    T* stage = v.stage + (size_t)w * v.QR * 5 * n;
    T* Cb = v.Cbuf + (size_t)w * K * n;

    int cnt = 0;
    for (int mv = 0; mv < nmoves; ++mv) {
        const int e = e0 + mv, a = e - spin * n;
        double re[3];
        for (int k = 0; k < 3; ++k) re[k] = v.R[((size_t)w * v.ne + e) * 3 + k];

        // ---- phase A: drift at r_e
        for (int j = tid * VEC; j < n; j += nt * VEC) {
            T x[VEC];
            load16(Mspin + (size_t)a * n + j, x);
#pragma unroll
            for (int i = 0; i < VEC; ++i) s_c0[j + i] = x[i];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                load16(VGLspin + ((size_t)a * 5 + 1 + k) * n + j, x);
#pragma unroll
                for (int i = 0; i < VEC; ++i) s_g[(size_t)k * n + j + i] = x[i];
            }
        }
        double jg[3] = {0.0, 0.0, 0.0}, dummy = 0.0;
        if (v.use_j2 || v.n_ions) j2_part(v, w, e, re, nullptr, tid, nt, jg, dummy);
        __syncthreads();
        // window dots, one wave per slot: y_m = u_m . c0, gm_k = g_k . c_m
        for (int m = wave; m < cnt; m += nw) {
            const T* um = stage + (size_t)m * 5 * n;
            const T* cm = Cb + (size_t)m * n;
            double y = 0.0, g0 = 0.0, g1 = 0.0, g2 = 0.0;
            for (int j = lane * VEC; j < n; j += 64 * VEC) {
                T uv[VEC], cv[VEC];
                load16(um + j, uv);
                load16(cm + j, cv);
#pragma unroll
                for (int i = 0; i < VEC; ++i) {
                    y += (double)(uv[i] * s_c0[j + i]);
                    g0 += (double)(s_g[j + i] * cv[i]);
                    g1 += (double)(s_g[(size_t)n + j + i] * cv[i]);
                    g2 += (double)(s_g[2 * (size_t)n + j + i] * cv[i]);
                }
            }
            y = wave_sum(y);
            g0 = wave_sum(g0);
            g1 = wave_sum(g1);
            g2 = wave_sum(g2);
            if (lane == 0) {
                s_y[m] = y;
                s_gm[m][0] = g0;
                s_gm[m][1] = g1;
                s_gm[m][2] = g2;
            }
        }
        if (wave == nw - 1) {  // g_k . c0
            double g0 = 0.0, g1 = 0.0, g2 = 0.0;
            for (int j = lane; j < n; j += 64) {
                g0 += (double)(s_g[j] * s_c0[j]);
                g1 += (double)(s_g[(size_t)n + j] * s_c0[j]);
                g2 += (double)(s_g[2 * (size_t)n + j] * s_c0[j]);
            }
            g0 = wave_sum(g0);
            g1 = wave_sum(g1);
            g2 = wave_sum(g2);
            if (lane == 0) {
                s_d[0] = g0;
                s_d[1] = g1;
                s_d[2] = g2;
            }
        }
        jg[0] = block_sum(jg[0], s_red, 0, lane, wave, nw);
        jg[1] = block_sum(jg[1], s_red, 1, lane, wave, nw);
        jg[2] = block_sum(jg[2], s_red, 2, lane, wave, nw);
        // beta, the drift and the proposal (wave 0), its stencil
        if (wave == 0) {
            const bool mine = lane < cnt;
            const double rinv = mine ? 1.0 / s_rho[lane] : 0.0;
            double t = mine ? s_y[lane] : 0.0, my_beta = 0.0;
            for (int mm = 0; mm < cnt; ++mm) {
                const double bm = dpp::lane(t, mm) * dpp::lane(rinv, mm);
                if (lane == mm) my_beta = bm;
                if (lane > mm && mine) t -= bm * s_G[lane][mm];
            }
            double vd[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) vd[k] = s_d[k] - wave_sum(mine ? my_beta * s_gm[lane][k] : 0.0) + jg[k];
            double z[3], rp[3], dl[3];
            gauss3(v.seed, v.uid[w], step, (uint32_t)e, z);
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                dl[k] = tau * vd[k] + sqrt_tau * z[k];
                rp[k] = wrap_box(re[k] + dl[k], v.L);
            }
            dmc_stencil<T>(v, rp, lane, s_idx, s_w);
            if (mine) s_beta[lane] = my_beta;
            if (lane < 3) {
                s_rp[lane] = rp[lane];
                s_delta[lane] = dl[lane];
                s_v[lane] = vd[lane];
            }
        }
        __syncthreads();

        // ---- phase B: orbital rows at r', ratio, drift at r', acceptance
        const double rp[3] = {s_rp[0], s_rp[1], s_rp[2]};
        const int rounds = (items + nt - 1) / nt;
        for (int r = 0; r < rounds; ++r) {  // every lane takes part (quad sums)
            const int item = tid + r * nt;
            const int g = item >> 2, p = item & 3;
            const bool valid = g < groups;
            const int j0 = valid ? g * VEC : 0;
            T vals[16][VEC];
#pragma unroll
            for (int q = 0; q < 16; ++q) load16(v.table + s_idx[p * 16 + q] + j0, vals[q]);
            T acc[5][VEC];
#pragma unroll
            for (int k = 0; k < 5; ++k)
#pragma unroll
                for (int i = 0; i < VEC; ++i) acc[k][i] = (T)0;
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const T* wq = &s_w[(p * 16 + q) * 5];
#pragma unroll
                for (int i = 0; i < VEC; ++i) {
                    const T x = valid ? vals[q][i] : (T)0;
#pragma unroll
                    for (int k = 0; k < 5; ++k) acc[k][i] += wq[k] * x;
                }
            }
#pragma unroll
            for (int k = 0; k < 5; ++k)
#pragma unroll
                for (int i = 0; i < VEC; ++i) {
                    acc[k][i] = quad_add<dpp::kQuadXor1>(acc[k][i]);
                    acc[k][i] = quad_add<dpp::kQuadXor2>(acc[k][i]);
                }
            if (valid) {
                // pending slot: the proposal's rows, one component per lane of the quad
                T* dst = stage + (size_t)cnt * 5 * n + j0;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    if (k != p) continue;
                    store16(dst + (size_t)k * n, acc[k]);
#pragma unroll
                    for (int i = 0; i < VEC; ++i) s_u[(size_t)k * n + j0 + i] = acc[k][i];
                }
                if (p == 0) store16(dst + 4 * (size_t)n, acc[4]);
            }
        }
        double jg2[3] = {0.0, 0.0, 0.0}, dj = 0.0;
        if (v.use_j2 || v.n_ions) j2_part(v, w, e, rp, re, tid, nt, jg2, dj);
        __syncthreads();
        // window dots, one wave per slot: x_m = u . c_m, xg_k = grad_k u . c_m
        for (int m = wave; m < cnt; m += nw) {
            const T* cm = Cb + (size_t)m * n;
            double x0 = 0.0, x1 = 0.0, x2 = 0.0, x3 = 0.0;
            for (int j = lane * VEC; j < n; j += 64 * VEC) {
                T cv[VEC];
                load16(cm + j, cv);
#pragma unroll
                for (int i = 0; i < VEC; ++i) {
                    x0 += (double)(s_u[j + i] * cv[i]);
                    x1 += (double)(s_u[(size_t)n + j + i] * cv[i]);
                    x2 += (double)(s_u[2 * (size_t)n + j + i] * cv[i]);
                    x3 += (double)(s_u[3 * (size_t)n + j + i] * cv[i]);
                }
            }
            x0 = wave_sum(x0);
            x1 = wave_sum(x1);
            x2 = wave_sum(x2);
            x3 = wave_sum(x3);
            if (lane == 0) {
                s_x[m] = x0;
                s_xg[m][0] = x1;
                s_xg[m][1] = x2;
                s_xg[m][2] = x3;
            }
        }
        if (wave == nw - 1) {  // u . c0 and grad u . c0
            double d0 = 0.0, d1 = 0.0, d2 = 0.0, d3 = 0.0;
            for (int j = lane; j < n; j += 64) {
                d0 += (double)(s_u[j] * s_c0[j]);
                d1 += (double)(s_u[(size_t)n + j] * s_c0[j]);
                d2 += (double)(s_u[2 * (size_t)n + j] * s_c0[j]);
                d3 += (double)(s_u[3 * (size_t)n + j] * s_c0[j]);
            }
            d0 = wave_sum(d0);
            d1 = wave_sum(d1);
            d2 = wave_sum(d2);
            d3 = wave_sum(d3);
            if (lane == 0) {
                s_d[0] = d0;
                s_d[1] = d1;
                s_d[2] = d2;
                s_d[3] = d3;
            }
        }
        jg2[0] = block_sum(jg2[0], s_red, 3, lane, wave, nw);
        jg2[1] = block_sum(jg2[1], s_red, 4, lane, wave, nw);
        jg2[2] = block_sum(jg2[2], s_red, 5, lane, wave, nw);
        dj = block_sum(dj, s_red, 6, lane, wave, nw);
        if (wave == 0) {
            const bool mine = lane < cnt;
            const double b = mine ? s_beta[lane] : 0.0;
            const double rho = s_d[0] - wave_sum(b * (mine ? s_x[lane] : 0.0));
            double fwd = 0.0, bwd = 0.0;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const double gnum = s_d[1 + k] - wave_sum(b * (mine ? s_xg[lane][k] : 0.0));
                const double vn = gnum / rho + jg2[k];
                const double f = s_delta[k] - tau * s_v[k];
                const double bb = s_delta[k] + tau * vn;
                fwd += f * f;
                bwd += bb * bb;
            }
            const double prob = rho * rho * exp(2.0 * dj) * exp(-(bwd - fwd) / (2.0 * tau));
            const double u = accept_uniform(v.seed, v.uid[w], step, (uint32_t)e);
            int acc = rho > 0.0 && u < prob;
            const size_t ri = ((size_t)rs * v.ne + e) * v.Wcap + w;
            if (forcing && v.forced[ri] < 2) acc = v.forced[ri] != 0;
            if (recording && lane == 0) {
                v.rec_rho[ri] = rho;
                v.rec_dlnj[ri] = dj;
                v.rec_prob[ri] = prob;
                v.rec_acc[ri] = (uint8_t)acc;
                for (int k = 0; k < 3; ++k) v.rec_rnew[3 * ri + k] = rp[k];
            }
            if (acc) {
                if (mine) s_G[cnt][lane] = s_x[lane];
                if (lane == 0) {
                    s_rho[cnt] = rho;
                    s_wel[cnt] = a;
                    for (int k = 0; k < 3; ++k) v.R[((size_t)w * v.ne + e) * 3 + k] = rp[k];
                    v.logdet[w * 2 + spin] += log(fabs(rho));
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
            // the accepted move's column: c = c0 - sum_m beta_m c_m
            for (int j = tid * VEC; j < n; j += nt * VEC) {
                T cn[VEC];
#pragma unroll
                for (int i = 0; i < VEC; ++i) cn[i] = s_c0[j + i];
                for (int m = 0; m < cnt; ++m) {
                    T cm[VEC];
                    load16(Cb + (size_t)m * n + j, cm);
                    const T bm = (T)s_beta[m];
#pragma unroll
                    for (int i = 0; i < VEC; ++i) cn[i] -= bm * cm[i];
                }
                store16(Cb + (size_t)cnt * n + j, cn);
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

template <typename T>
__global__ __launch_bounds__(kBlock) void k_window_dmc(CrowdView<T> v, int e0, int nmoves)
{
    window_dmc_body<T>(v, blockIdx.x, e0, nmoves);
}

// Walkers of several systems in one launch: item i = (system, walker), window j of spin
// block `spin` (systems whose blocks have fewer windows skip it).  Persistent: the grid
// strides over the items, which come largest system first, so the long windows start first
// and the short ones fill in behind them.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_window_dmc_multi(const CrowdView<T>* __restrict__ views,
                                                             const int2* __restrict__ items, int n_items, int spin,
                                                             int j)
{
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        const int2 item = items[it];
        const CrowdView<T> v = views[item.x];
        const int a0 = j * v.K;
        if (a0 < v.n) window_dmc_body<T>(v, item.y, spin * v.n + a0, min(v.K, v.n - a0));
        __syncthreads();  // the next item reuses the shared memory
    }
}

template <typename T>
void launch_window_dmc_multi(const CrowdView<T>* views, const int2* items, int n_items, int max_n, int spin, int j,
                             int grid, hipStream_t s)
{
    const size_t lds = 8 * (size_t)max_n * sizeof(T);
    static bool lds_set = false;
    if (!lds_set) {
        (void)hipFuncSetAttribute((const void*)k_window_dmc_multi<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)(8 * 2048 * sizeof(T)));
        lds_set = true;
    }
    hipLaunchKernelGGL(k_window_dmc_multi<T>, dim3(grid), dim3(kBlock), lds, s, views, items, n_items, spin, j);
}

template <typename T>
void launch_window_dmc(const CrowdView<T>& v, int e0, int nmoves, hipStream_t s)
{
    const size_t lds = 8 * (size_t)v.n * sizeof(T);
    static bool lds_set = false;
    if (!lds_set) {
        (void)hipFuncSetAttribute((const void*)k_window_dmc<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)(8 * 2048 * sizeof(T)));
        lds_set = true;
    }
    hipLaunchKernelGGL(k_window_dmc<T>, dim3(v.W), dim3(kBlock), lds, s, v, e0, nmoves);
}

// ---- branching

__device__ __forceinline__ double branch_uniform(uint64_t seed, uint32_t uid, uint32_t step)
{
    uint32_t o[4];
    philox_block(seed, uid, step, 0xFFFFFFFFu, 3u, o);
    return uniform53(o[0], o[1]);
}

__device__ __forceinline__ uint32_t child_uid(uint64_t seed, uint32_t uid, uint32_t step, uint32_t copy)
{
    uint32_t o[4];
    philox_block(seed, uid, step, copy, 4u, o);
    return o[0];
}

// weights and multiplicities, one thread per walker
__global__ __launch_bounds__(kBlock) void k_dmc_weights(DmcView d, const double* eloc, const double* eold,
                                                        const uint32_t* uid, const Params* prm)
{
    const int w = blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= d.pop) return;
    const double tau = prm->tau, et = d.state->e_t;
    const double lo = et - d.ecut, hi = et + d.ecut;
    const double eo = fmin(fmax(eold[w], lo), hi);
    const double en = fmin(fmax(eloc[w], lo), hi);
    const double wt = exp(-tau * (0.5 * (eo + en) - et));
    const double ub = branch_uniform(d.seed, uid[w], prm->step);
    int m = (int)floor(wt + ub);
    if (m > 3) m = 3;
    // parity mode: the given multiplicity (the population then follows the reference's)
    if (d.forced_mult && prm->rec_sweep < prm->mult_cap) m = d.forced_mult[(size_t)prm->rec_sweep * d.cap + w];
    d.wt[w] = wt;
    d.mult[w] = m;
}

// sums and prefix sum in population order (one thread), the trial energy, history
__global__ void k_dmc_sums(DmcView d, const double* eloc, long long* nacc, long long* nprop, const Params* prm, int gen)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double wsum = 0.0, wesum = 0.0;
    int off = 0;
    long long na = 0, np = 0;
    for (int w = 0; w < d.pop; ++w) {
        wsum += d.wt[w];
        wesum += d.wt[w] * eloc[w];
        d.off[w] = off;
        off += d.mult[w];
        na += nacc[w];
        np += nprop[w];
    }
    DmcState* st = d.state;
    st->nacc += na;
    st->nprop += np;
    st->new_pop = off;
    if (off == 0 || off > d.cap) {
        st->status = 1;
        return;
    }
    const double e_est = wesum / wsum;
    const double et = e_est - log((double)off / (double)d.n_target) / prm->tau;
    st->e_t = et;
    double* h = d.history + (size_t)gen * 4;
    h[0] = (double)off;
    h[1] = wsum;
    h[2] = e_est;
    h[3] = et;
}

// copies of walker w (grid: walkers x chunks); copy 0 keeps the uid
template <typename T>
__global__ __launch_bounds__(kBlock) void k_dmc_copy(DmcView d, WalkerArrays<T> src, WalkerArrays<T> dst, int n,
                                                     int ne, const Params* prm)
{
    const int w = blockIdx.x / d.chunks, chunk = blockIdx.x % d.chunks;
    if (w >= d.pop || d.state->status) return;
    const int m = d.mult[w], o = d.off[w];
    const size_t nM = 2 * (size_t)n * n, nV = 2 * (size_t)n * 5 * n;
    const size_t stride = (size_t)d.chunks * blockDim.x;
    for (int c = 0; c < m; ++c) {
        const int t = o + c;
        if (t >= d.cap) return;
        for (size_t i = (size_t)chunk * blockDim.x + threadIdx.x; i < nM; i += stride)
            dst.M[(size_t)t * nM + i] = src.M[(size_t)w * nM + i];
        for (size_t i = (size_t)chunk * blockDim.x + threadIdx.x; i < nV; i += stride)
            dst.VGL[(size_t)t * nV + i] = src.VGL[(size_t)w * nV + i];
        if (chunk == 0) {
            for (int i = threadIdx.x; i < ne * 3; i += blockDim.x)
                dst.R[(size_t)t * ne * 3 + i] = src.R[(size_t)w * ne * 3 + i];
            if (threadIdx.x == 0) {
                dst.logdet[2 * t] = src.logdet[2 * w];
                dst.logdet[2 * t + 1] = src.logdet[2 * w + 1];
                dst.sign[2 * t] = src.sign[2 * w];
                dst.sign[2 * t + 1] = src.sign[2 * w + 1];
                dst.eloc[t] = src.eloc[w];
                dst.eold[t] = src.eloc[w];
                dst.uid[t] = c == 0 ? src.uid[w] : child_uid(d.seed, src.uid[w], prm->step, (uint32_t)c);
                dst.nacc[t] = 0;
                dst.nprop[t] = 0;
            }
        }
    }
}

template <typename T>
void launch_dmc_branch(const DmcView& d, const WalkerArrays<T>& src, const WalkerArrays<T>& dst, int n, int ne,
                       const Params* prm, int gen, hipStream_t s)
{
    hipLaunchKernelGGL(k_dmc_weights, dim3((d.pop + kBlock - 1) / kBlock), dim3(kBlock), 0, s, d, src.eloc, src.eold,
                       src.uid, prm);
    hipLaunchKernelGGL(k_dmc_sums, dim3(1), dim3(64), 0, s, d, src.eloc, src.nacc, src.nprop, prm, gen);
    hipLaunchKernelGGL(k_dmc_copy<T>, dim3(d.pop * d.chunks), dim3(kBlock), 0, s, d, src, dst, n, ne, prm);
}

template void launch_window_dmc<float>(const CrowdView<float>&, int, int, hipStream_t);
template void launch_window_dmc_multi<float>(const CrowdView<float>*, const int2*, int, int, int, int, int,
                                             hipStream_t);
template void launch_window_dmc_multi<double>(const CrowdView<double>*, const int2*, int, int, int, int, int,
                                              hipStream_t);
template void launch_window_dmc<double>(const CrowdView<double>&, int, int, hipStream_t);
template void launch_dmc_branch<float>(const DmcView&, const WalkerArrays<float>&, const WalkerArrays<float>&, int, int,
                                       const Params*, int, hipStream_t);
template void launch_dmc_branch<double>(const DmcView&, const WalkerArrays<double>&, const WalkerArrays<double>&, int,
                                        int, const Params*, int, hipStream_t);

}  // namespace cq
