// One-body Pade Jastrow of the kernels: ln J1 = + sum_i sum_I u1(|r_i - R_I|),
// u1(r) = a r / (1 + b r), minimum-image distance to each fixed centre R_I, in FP64
// whatever the precision of the path.  Each helper takes the centres
// I = i0, i0 + stride, ..., so that the threads of a sum share them out.
#pragma once
#include "cq_device.h"
#include "cq_internal.h"

namespace cq {

// u1 of an electron at r summed over the centres, with its gradient
// sum u1'(d) d/|d| and Laplacian sum u1'' + 2 u1'/d added to g and lap.
template <typename T>
__device__ __forceinline__ double j1_at(const CrowdView<T>& v, const double r[3], int i0, int stride, double g[3],
                                        double& lap)
{
    double sum = 0.0;
    for (int I = i0; I < v.n_ions; I += stride) {
        double d[3], u, du, d2u;
        min_image(r, v.ions + 3 * I, v.L, d);
        const double rr = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        pade(v.j1_a, v.j1_b, rr, u, du, d2u);
        sum += u;
#pragma unroll
        for (int c = 0; c < 3; ++c) g[c] += du * d[c] / rr;
        lap += d2u + 2.0 * du / rr;
    }
    return sum;
}

// The change of sum_I u1 when an electron moves from r0 to r1.
template <typename T>
__device__ __forceinline__ double j1_delta(const CrowdView<T>& v, const double r1[3], const double r0[3], int i0,
                                           int stride)
{
    double s = 0.0;
    for (int I = i0; I < v.n_ions; I += stride) {
        double d[3], u1, u0, du, d2u;
        min_image(r1, v.ions + 3 * I, v.L, d);
        pade(v.j1_a, v.j1_b, sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]), u1, du, d2u);
        min_image(r0, v.ions + 3 * I, v.L, d);
        pade(v.j1_a, v.j1_b, sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]), u0, du, d2u);
        s += u1 - u0;
    }
    return s;
}

}  // namespace cq
