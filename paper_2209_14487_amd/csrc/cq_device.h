// Device helpers of the crowd QMC kernels (gfx950, wave64).
//
// Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) with key =
// (seed low, seed high).  Streams are addressed by 128-bit counters:
//   move Gaussians   (uid, step, electron, 0|1)   Box-Muller pairs
//   Metropolis u     (uid, step, electron, 2)
//   spline coefs     (idx low, idx high, 0xC0EF, 0)
// The 53-bit uniform of two words (w0, w1) is ((w1:w0) >> 11) * 2^-53.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cq {

constexpr double kPi = 3.14159265358979323846;

__device__ __forceinline__ void philox4x32_10(uint32_t& x0, uint32_t& x1, uint32_t& x2, uint32_t& x3,
                                              uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t lo0 = 0xD2511F53u * x0;
        const uint32_t hi0 = __umulhi(0xD2511F53u, x0);
        const uint32_t lo1 = 0xCD9E8D57u * x2;
        const uint32_t hi1 = __umulhi(0xCD9E8D57u, x2);
        const uint32_t y0 = hi1 ^ x1 ^ k0;
        const uint32_t y2 = hi0 ^ x3 ^ k1;
        x0 = y0;
        x1 = lo1;
        x2 = y2;
        x3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

__device__ __forceinline__ double uniform53(uint32_t lo, uint32_t hi)
{
    const uint64_t v = ((uint64_t)hi << 32) | (uint64_t)lo;
    return (double)(v >> 11) * (1.0 / 9007199254740992.0);
}

__device__ __forceinline__ void philox_block(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                             uint32_t o[4])
{
    uint32_t x0 = c0, x1 = c1, x2 = c2, x3 = c3;
    philox4x32_10(x0, x1, x2, x3, (uint32_t)seed, (uint32_t)(seed >> 32));
    o[0] = x0; o[1] = x1; o[2] = x2; o[3] = x3;
}

// Gaussian 3-vector of move (uid, step, e): Box-Muller of blocks 0 (x, y) and 1 (z).
__device__ __forceinline__ void gauss3(uint64_t seed, uint32_t uid, uint32_t step, uint32_t e, double z[3])
{
    uint32_t o[4];
    philox_block(seed, uid, step, e, 0u, o);
    double u0 = uniform53(o[0], o[1]), u1 = uniform53(o[2], o[3]);
    double rad = sqrt(-2.0 * log(1.0 - u0));
    z[0] = rad * cos(2.0 * kPi * u1);
    z[1] = rad * sin(2.0 * kPi * u1);
    philox_block(seed, uid, step, e, 1u, o);
    u0 = uniform53(o[0], o[1]);
    u1 = uniform53(o[2], o[3]);
    z[2] = sqrt(-2.0 * log(1.0 - u0)) * cos(2.0 * kPi * u1);
}

__device__ __forceinline__ double accept_uniform(uint64_t seed, uint32_t uid, uint32_t step, uint32_t e)
{
    uint32_t o[4];
    philox_block(seed, uid, step, e, 2u, o);
    return uniform53(o[0], o[1]);
}

__device__ __forceinline__ double wrap_box(double x, double L) { return x - L * floor(x / L); }

// Per-axis cubic B-spline stencil: control points i0-1 .. i0+2 (mod G) and the
// value / first / second derivative weights at fractional offset t.  The
// integer cell, t and the weights are formed in FP64; the weights are stored in T.
template <typename T>
struct AxisW {
    int i0;
    T b[4], d1[4], d2[4];
};

// Per-axis weights of the cubic B-spline at x: cell index i0 and the weights of
// control points i0-1 .. i0+2 for the value, first and second derivative.  The
// polynomials are evaluated in FP64 and each weight is rounded to T once, so that
// an FP32 weight carries an independent half-ulp error (an FP32 factor 1/6 shared
// by every weight would bias all orbital values alike, and an ill-conditioned
// Slater matrix amplifies such a correlated error several times more than
// independent roundings).
template <typename T>
__device__ __forceinline__ AxisW<T> axis_weights(double x, double L, int G)
{
    AxisW<T> r;
    const double h = L / G;
    const double s = wrap_box(x, L) / h;
    const double fl = floor(s);
    int i = ((int)fl) % G;
    if (i < 0) i += G;
    r.i0 = i;
    const double t = s - fl;
    const double u = 1.0 - t;
    const double t2 = t * t, t3 = t2 * t;
    const double sixth = 1.0 / 6.0;
    r.b[0] = (T)(u * u * u * sixth);
    r.b[1] = (T)((3.0 * t3 - 6.0 * t2 + 4.0) * sixth);
    r.b[2] = (T)((-3.0 * t3 + 3.0 * t2 + 3.0 * t + 1.0) * sixth);
    r.b[3] = (T)(t3 * sixth);
    const double ih2 = 1.0 / (h * h);
    const double half_ih = 0.5 / h;
    r.d1[0] = (T)(-u * u * half_ih);
    r.d1[1] = (T)((3.0 * t2 - 4.0 * t) * half_ih);
    r.d1[2] = (T)((-3.0 * t2 + 2.0 * t + 1.0) * half_ih);
    r.d1[3] = (T)(t2 * half_ih);
    r.d2[0] = (T)(u * ih2);
    r.d2[1] = (T)((3.0 * t - 2.0) * ih2);
    r.d2[2] = (T)((-3.0 * t + 1.0) * ih2);
    r.d2[3] = (T)(t * ih2);
    return r;
}

// Pade two-body term u(r) = a r / (1 + b r) with u' and u''.
__device__ __forceinline__ void pade(double a, double b, double r, double& u, double& du, double& d2u)
{
    const double q = 1.0 + b * r;
    const double iq = 1.0 / q;
    u = a * r * iq;
    du = a * iq * iq;
    d2u = -2.0 * a * b * iq * iq * iq;
}

__device__ __forceinline__ void min_image(const double* ri, const double* rj, double L, double d[3])
{
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double x = ri[c] - rj[c];
        d[c] = x - L * rint(x / L);
    }
}

// Sum over the 64 lanes of a wave; every lane gets the same total.  Within each
// row of 16 lanes the partner values come from DPP lane swizzles (quad
// permutations for distances 1 and 2, half-row and row mirrors for 4 and 8), so
// no LDS traffic is needed; the four row sums are then read as scalars and added
// in a fixed order, (row0 + row1) + (row2 + row3).
namespace dpp {
constexpr int kQuadXor1 = 0xB1;      // quad_perm [1,0,3,2]
constexpr int kQuadXor2 = 0x4E;      // quad_perm [2,3,0,1]
constexpr int kHalfMirror = 0x141;   // row_half_mirror
constexpr int kMirror = 0x140;       // row_mirror
template <int CTRL>
__device__ __forceinline__ float mov(float x)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double mov(double x)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float lane(float x, int l)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), l));
}
__device__ __forceinline__ double lane(double x, int l)
{
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(x), l),
                            __builtin_amdgcn_readlane(__double2loint(x), l));
}
}  // namespace dpp

template <typename T>
__device__ __forceinline__ T wave_sum(T v)
{
    v += dpp::mov<dpp::kQuadXor1>(v);
    v += dpp::mov<dpp::kQuadXor2>(v);
    v += dpp::mov<dpp::kHalfMirror>(v);
    v += dpp::mov<dpp::kMirror>(v);
    return (dpp::lane(v, 0) + dpp::lane(v, 16)) + (dpp::lane(v, 32) + dpp::lane(v, 48));
}

// Block-to-(walker, part) mapping that keeps all workgroups of one walker on the
// same XCD (workgroups are dispatched to the 8 XCDs round-robin by block id), so
// a walker's rows, window and positions stay in one L2.
__device__ __forceinline__ void xcd_map(int bid, int per_walker, int& w, int& part)
{
    const int xcd = bid & 7, loc = bid >> 3;
    w = (loc / per_walker) * 8 + xcd;
    part = loc % per_walker;
}

inline int xcd_grid(int W, int per_walker) { return ((W + 7) / 8) * 8 * per_walker; }

// Pointer into the constant address space: it marks memory as read-only for the
// kernel's duration, and loads through it at a wave-uniform address become scalar
// loads.
template <typename T>
using cptr = const __attribute__((address_space(4))) T*;

template <typename T>
__device__ __forceinline__ cptr<T> as_const(const T* p)
{
    return (cptr<T>)p;
}

template <typename T>
struct Vec16;  // 16-byte vector of T
template <>
struct Vec16<float> {
    using type = float4;
    static constexpr int n = 4;
};
template <>
struct Vec16<double> {
    using type = double2;
    static constexpr int n = 2;
};

template <typename T>
__device__ __forceinline__ void load16(const T* p, T out[16 / sizeof(T)])
{
    using V = typename Vec16<T>::type;
    const V v = *reinterpret_cast<const V*>(p);
    if constexpr (sizeof(T) == 4) {
        out[0] = v.x; out[1] = v.y; out[2] = v.z; out[3] = v.w;
    } else {
        out[0] = v.x; out[1] = v.y;
    }
}

template <typename T>
__device__ __forceinline__ void store16(T* p, const T in[16 / sizeof(T)])
{
    using V = typename Vec16<T>::type;
    V v;
    if constexpr (sizeof(T) == 4) {
        v.x = in[0]; v.y = in[1]; v.z = in[2]; v.w = in[3];
    } else {
        v.x = in[0]; v.y = in[1];
    }
    *reinterpret_cast<V*>(p) = v;
}

}  // namespace cq
