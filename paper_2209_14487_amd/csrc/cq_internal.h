// Internal declarations shared by the C ABI (capi.cpp) and the kernel files.
//
// Device layout of one crowd (W walkers, N electrons per spin, Ne = 2N,
// T = float for the mixed path and double for the FP64 path, K = delay rank):
//   R      double [W][Ne][3]          positions
//   M      T      [W][2][N][N]        M[w][s][a][j] = (A_s^-1)[j][a]: row a is the
//                                     inverse column of electron a, contiguous
//   VGL    T      [W][2][N][5][N]     rows of A (value), grad x/y/z and Laplacian of
//                                     every orbital j at electron a
//   logdet double [W][2], sign int [W][2], nacc/nprop int64 [W], eloc double [W]
//   window (accepted moves m = 0 .. cnt-1 of the current k proposals):
//           welec int [W][K]    electron (within its spin) of move m
//           wslot int [W][K]    stage slot holding the rows of move m
//           stage T [W][Q][5][N] orbital rows (+ gradients, Laplacian) of proposals:
//                               per-move paths (Q = K): slot m = accepted move m,
//                               slot cnt the pending proposal; batched path: ring
//                               of Q candidates, slot = electron mod Q
//           Cbuf  T [W][K][N]   inverse column c_m of electron e_m just before
//                               move m (slot cnt: the old column, pending)
//           wrho  double [W][K] determinant ratio of move m
//           wG    double [W][K][K] wG[m][j] = u_m . c_j (j < m)
//           beta  double [W][K], pend int [W]: coefficients of the last accepted
//                               move, whose column still has to be brought up to date
//   part   double [2][W][C][NP]       per-workgroup partial sums of a move (by move parity)
//   rnew   double [4][W][3]           proposals, slot e % 4 holds move e's
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "cq.h"

namespace cq {

constexpr int kMaxDelay = 32;
constexpr int kMaxCand = 88;   // candidates per round of the batched path
constexpr int kBlock = 256;
constexpr int kSweepMaxN = 64;
constexpr int kMaxIons = 64;    // centres of the one-body Jastrow  // largest N of the whole-sweep path (both inverses in LDS)

// Partial-sum slots of one move workgroup: 4 determinant dots, 5 per window
// slot, then the Jastrow difference and gradient.
__host__ __device__ constexpr int part_stride(int K) { return 4 + 5 * K + 4; }
__host__ __device__ constexpr int part_j2(int K) { return 4 + 5 * K; }

template <typename T>
__host__ __device__ constexpr int chunk_orbitals() { return 64 * (16 / (int)sizeof(T)); }

// Device-resident scalars read by every kernel, so that a captured sweep graph
// stays valid from one sweep to the next.
struct Params {
    uint32_t step;       // Philox step of the current sweep
    int32_t rec_sweep;   // index of the current sweep in the record / forced buffers
    int32_t rec_cap;     // record capacity in sweeps (0 = off)
    int32_t forced_cap;  // forced-decision capacity in sweeps (0 = off)
    int32_t mult_cap;    // forced branching multiplicities, in generations (0 = off)
    double sigma;        // VMC step
    double tau;          // DMC time step
};

template <typename T>
struct CrowdView {
    int W, n, ne, K;
    int arow;            // row stride of the value rows in VGL read by the inversion (5 N in a crowd)
    int Wcap;            // walker capacity: the walker stride of the record and forced-decision buffers
    int Q;               // candidates per round (batched path), else K
    int vgl_wg;          // gather workgroups per CU beside the update (batched path; 0: built-in rule)
    int upd_mfma;        // FP64 batched path: the rank-k update on the FP64 matrix cores
    int QR;              // stage slots per walker: K, or the candidate ring of the batched path (2 Q,
                         // so a round's new candidates never reuse a slot the previous window's
                         // update still reads)
    int G, n_orb;
    double L;
    const T* table;
    double* R;
    T* M;
    T* VGL;
    double* logdet;
    int* sign;
    long long* nacc;
    long long* nprop;
    double* eloc;
    double* elpart;
    int* cnt;            // [3][W] window count seen by the last move of each parity; [2]: final
    int* welec;
    int* wslot;          // [W][K] stage slot of accepted move m
    T* stage;
    T* Cbuf;
    float* ct;           // [W][N][32] columns transposed (Ct[k][m]) for the matrix-core update, or null
    float* ub;           // [W][32][N] the window's accepted value rows, packed (set with ct), or null
    double* wrho;
    double* wG;
    double* wlinv;       // [W][K][K] inverse of the window's triangle (G below, rho on the diagonal)
    double* beta;
    int* pend;
    double* part;
    double* rnew;
    double* jd;          // [W][Q] Jastrow difference of the candidate in ring slot q
    double* rprop;       // [W][Q][3] its proposed position
    size_t* sidx;        // [W][Q][64] table offsets of its stencil points
    void* swt;           // [W][Q][64][5] T: their value, gradient and Laplacian weights
    double* pmat;        // [W][Q][Q] P of the current round's candidates
    double* tmat;        // [W][K][K] T: accepted columns in the basis of their own start columns
    int* cur;            // [W][2] next electron to decide, end of the evaluated candidates;
                         // then [W] first candidate of the last round
    int* look;           // [2][W][2] gather range of the rounds of each parity
    int* used;           // [2] rounds of the current spin block in which some walker had candidates
    int* left;           // [2] whether the block's tail kernel had electrons to move
    const uint32_t* uid;
    uint64_t seed;
    int use_j2;
    double a_par, a_anti, b;
    const double* ions;  // [n_ions][3] centres of the one-body Jastrow (n_ions = 0: none)
    int n_ions;
    double j1_a, j1_b;
    Params* prm;
    double* rec_rho;
    double* rec_dlnj;
    double* rec_prob;
    uint8_t* rec_acc;
    double* rec_rnew;    // DMC moves: the proposed position [rec][Ne][Wcap][3], or null
    const uint8_t* forced;
    int* status;         // [W] bit 0: singular / not finite at the last inversion; bit 1: window
                         // bookkeeping out of range (internal error)
    double* drift;       // [W][2] |log|det| kept - recomputed| at the last inversion
    unsigned long long* drift_max;  // largest drift of any inversion since the positions were set (FP64
                                    // bit pattern: non-negative doubles order like their patterns)
};

// DMC population state on the device.
struct DmcState {
    double e_t;       // trial energy
    int new_pop;      // population after the last branching
    int status;       // 1: population died out or exceeded the capacity
    long long nacc;   // accepted / proposed moves over all generations
    long long nprop;
};

// Branching buffers of one crowd.
struct DmcView {
    DmcState* state;
    double* wt;       // [cap] weights of the generation
    int* mult;        // [cap] multiplicities
    int* off;         // [cap] first child index
    double* history;  // [n_gen][4] population, sum of weights, E_est, E_T
    const int* forced_mult;  // parity mode: [generations][cap] multiplicities to follow, or null
    int pop, cap, n_target, chunks;
    double ecut;
    uint64_t seed;
};

// The per-walker arrays that branching copies (one of two buffer sets).
template <typename T>
struct WalkerArrays {
    double* R;
    T* M;
    T* VGL;
    double* logdet;
    int* sign;
    double* eloc;
    double* eold;     // E_L at the start of the generation
    uint32_t* uid;
    long long* nacc;
    long long* nprop;
};

// Ewald electron-electron energy of a crowd's walkers (FP64).
struct EwaldView {
    int W, ne, nmax, nk, pk, pr;  // walkers, electrons, largest |n| component, half-space
                                  // wavevectors, blocks per walker for the k sum and the pairs
    double L, alpha;
    const double* R;              // [W][Ne][3]
    const int4* kvec;             // [nk] (nx, ny, nz, 0), the half space of 0 < n^2 <= nmax^2
    const double* kfac;           // [nk] exp(-k^2 / 4 alpha^2) / k^2
    double2* phase;               // [W][Ne][3][nmax + 1] exp(i 2 pi m x / L)
    double* part;                 // [W][pk + pr] block sums
};

// FP64 Gauss-Jordan workspace for matrices too large for LDS.
struct InvWork {
    double* S;        // [nmat][N][N]
    double* PR;       // [nmat][B][N] pivot rows of the current block of B = 4b columns (before its update)
    int* pivrow;      // [nmat][N] pivot row of column k
    double* logabs;   // [nmat] log|det|, followed by [nmat] max|A_ij| (as 64-bit patterns)
    int* negs;        // [nmat] number of negative pivots
    int b;            // panel width
};

template <typename T> void launch_fill_philox(T* table, uint64_t seed, size_t count, hipStream_t s);
template <typename T> void launch_setup_vgl(const CrowdView<T>& v, hipStream_t s);
template <typename T> void launch_move(const CrowdView<T>& v, int e, int prev, int reset, hipStream_t s);
template <typename T> void launch_first_proposal(const CrowdView<T>& v, hipStream_t s);
template <typename T> void launch_window(const CrowdView<T>& v, int e0, int nmoves, hipStream_t s);
int window_threads(int n, int elem_bytes);
template <typename T>
void launch_batch_stencils(const CrowdView<T>& v, int spin, int par, bool block_start, hipStream_t s);
template <typename T> void launch_batch_vgl(const CrowdView<T>& v, int spin, int par, bool beside, hipStream_t s);
// workgroups per CU of the gather launched beside the update: the request, else the built-in rule
int batch_vgl_blocks_per_cu(int n, int elem_bytes, int request);
template <typename T> void launch_batch_jd(const CrowdView<T>& v, int spin, hipStream_t s);
template <typename T> void launch_batch_pmat(const CrowdView<T>& v, int spin, hipStream_t s);
template <typename T> void launch_batch_rows(const CrowdView<T>& v, int spin, hipStream_t s);
int device_cu_count();
template <typename T> void launch_sweep(const CrowdView<T>& v, hipStream_t s);
template <typename T> void launch_batch_decide(const CrowdView<T>& v, int spin, int par, int round, hipStream_t s);
template <typename T> void launch_batch_cols(const CrowdView<T>& v, int spin, hipStream_t s);
// tail of a spin block after the planned rounds (run), and the plan record for the host
template <typename T> void launch_leftover(const CrowdView<T>& v, int spin, int* host_report, bool run,
                                           hipStream_t s);
int batch_rounds(int n, int K);      // rounds per spin block (enough when every move is accepted)
int batch_candidates(int n, int K);  // candidates per round, Q
// linv_ready: the window's L^-1 is already in wlinv (the batched path forms it)
template <typename T> void launch_flush(const CrowdView<T>& v, int spin, hipStream_t s, bool linv_ready = false);
bool flush_mfma_fits(int n);  // the FP32 matrix-core update handles this N
bool flush_f64_mfma_fits(int n);  // the FP64 matrix-core update of the batched path handles this N
void launch_flush_f64_mfma(const CrowdView<double>& v, int spin, hipStream_t s);
void launch_flush_mfma(const CrowdView<float>& v, int spin, hipStream_t s, bool linv_ready);
template <typename T> void launch_energy(const CrowdView<T>& v, hipStream_t s);
// nmat < 0: the 2 W matrices of the view; else matrices 0 .. nmat-1 (matrix m at (m / 2, m % 2))
template <typename T> void launch_inverse(const CrowdView<T>& v, const InvWork& wk, hipStream_t s, int nmat = -1);
void launch_sweep_end(Params* prm, hipStream_t s);
template <typename T> void launch_window_dmc(const CrowdView<T>& v, int e0, int nmoves, hipStream_t s);
// Walkers of several systems in one launch (device views, one (system, walker) item each; window
// step j of spin block `spin`; persistent grid)
template <typename T>
void launch_window_dmc_multi(const CrowdView<T>* views, const int2* items, int n_items, int max_n, int spin, int j,
                             int grid, hipStream_t s);
// The window updates of several systems in one launch: L^-1 per (system, walker) item, then the
// strips of 32 rows (FP32 matrix cores) or 16 rows (vector path), one (system, walker, strip) item each
void launch_flush_mfma_multi(const CrowdView<float>* views, const int2* walkers, int n_walkers, const int4* strips,
                             int n_strips, int spin, int grid, hipStream_t s);
template <typename T>
void launch_flush_vec_multi(const CrowdView<T>* views, const int4* strips, int n_strips, int max_n, int spin, int grid,
                            hipStream_t s);
template <typename T>
void launch_dmc_branch(const DmcView& d, const WalkerArrays<T>& src, const WalkerArrays<T>& dst, int n, int ne,
                       const Params* prm, int gen, hipStream_t s);
template <typename T>
void launch_virtual(const CrowdView<T>& v, const double* offsets, int nq, double* ratio, double* rho, double* dlnj,
                    hipStream_t s);
void launch_ewald(const EwaldView& e, double* eloc, hipStream_t s);  // adds V_ee to eloc
int ewald_wavevectors_per_block();
void launch_copy(void* dst, const void* src, size_t bytes, hipStream_t s);
void launch_zero(void* p, size_t bytes, hipStream_t s);  // bytes: a multiple of 4
size_t inverse_work_bytes(int nmat, int n);
// Batched inversion of caller-held matrices (the C ABI's cq_slater_inverse and its variant on
// the library's static workspace): bytes of workspace it needs, argument checks, the inversion.
size_t slater_work_bytes(int n, int nmat);
// Sets the thread-local message of cq_last_error and returns s.
cq_status report_error(cq_status s, const char* msg);
cq_status check_slater_args(const void* A, int elem_bytes, int n, int nmat, const void* Minv, const double* logdet,
                            const int* sign);
template <typename T>
cq_status slater_inverse_impl(const T* A, int n, int nmat, T* Minv, double* logdet, int* sign, hipStream_t st,
                              unsigned char* work);
int panel_width(int n);  // columns per panel of the blocked inversion
// Row stride (doubles) of the blocked inversion's work matrix S: n plus a pad, so that the rows
// of a column panel do not all start at the same offset of a power-of-two stride (measured at
// n = 1024: the panel sweep takes 96 us with a pad of 16, 129 us with none, 149 us with 8).
__host__ __device__ inline int s_ld(int n) { return n + 16; }
int block_width(int n);  // columns per block (4 panels) of the blocked inversion

}  // namespace cq
