// Complex (twisted) orbitals in a general periodic cell: the device view of a crowd and
// the launchers of its kernels (k_complex.hip).  FP64 throughout; complex numbers are
// double2 (x = real, y = imaginary).
//
//   phi_j(r) = exp(i k.r) s_j(f),  f = r L^-1 (fractional coordinates; L has the lattice
//   vectors as rows), s_j a periodic cubic B-spline over a G^3 grid in f with complex
//   coefficients.  Cartesian derivatives: grad s = L^-1 grad_f s, lap s = sum_ab
//   (L^-T L^-1)_ab d2s/df_a df_b (the full Hessian in f); the twist adds
//   grad phi = e^{ik.r} (grad s + i k s), lap phi = e^{ik.r} (lap s + 2 i k.grad s - k^2 s).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace cq {

constexpr int kCMaxN = 512;  // electrons per spin on the complex path

struct CView {
    int W, n, ne, G, n_orb;
    double lat[9];     // rows a_1, a_2, a_3
    double linv[9];    // L^-1: f = r L^-1
    double metric[6];  // (L^-T L^-1): xx, yy, zz, xy, xz, yz
    double k[3], k2;   // twist and |k|^2
    const double2* table;    // [G][G][G][n_orb] complex128 coefficients, or
    const float2* table32;   // complex64 coefficients (the other pointer is null); the sums are FP64
    double* R;             // [W][ne][3]
    double2* M;            // [W][2][n][n]: M[a][j] = (A^-1)[j][a]
    double2* VGL;          // [W][2][n][5][n]: value, gradient x y z, Laplacian rows of phi
    double* logdet;        // [W][2]
    double* phase;         // [W][2] in (-pi, pi]
    double2* eloc;         // [W]
    long long* nacc;       // [W]
    long long* nprop;      // [W]
    const uint32_t* uid;   // [W]
    int* status;           // [W]: bit 0 singular or non-finite pivot
    double2* work;         // [W][2][n][2n] Gauss-Jordan workspace
    int use_j2;
    double a_par, a_anti, b;
    uint64_t seed;
    uint32_t step;
    double sigma;
    int rec_sweep, rec_cap;  // records of sweep rec_sweep are kept while rec_sweep < rec_cap
    double2* rec_rho;        // [rec_cap][ne][W]
    double* rec_dlnj;
    double* rec_prob;
    uint8_t* rec_acc;
};

void launch_csetup_rows(const CView& v, hipStream_t s);   // orbital rows of every electron
void launch_cinverse(const CView& v, hipStream_t s);      // A^-1, log|det| and phase per spin
void launch_csweep(const CView& v, hipStream_t s);        // one VMC sweep of every walker
void launch_cenergy(const CView& v, hipStream_t s);       // complex local energy per walker

}  // namespace cq
