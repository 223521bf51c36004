// Stencil of a B-spline evaluation, shared by the batched gather and the
// whole-sweep kernel.
#pragma once
#include "cq_device.h"
#include "cq_internal.h"

namespace cq {

// Stencil of one proposal (table offsets and the five weights of the 64 points,
// index 16 x + 4 y + z); lane l of a wave fills entry l.
template <typename T>
__device__ __forceinline__ void stencil_entry(const CrowdView<T>& v, const double rp[3], int l, size_t* sidx,
                                              T* sw)
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

}  // namespace cq
