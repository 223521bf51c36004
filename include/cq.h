/*
 * cq.h -- C ABI of the crowd-of-walkers particle-by-particle QMC move on
 * MI355X (gfx950).
 *
 * The library implements the batched particle-by-particle move of Luo, Doak
 * and Kent, "A High-Performance Design for Hierarchical Parallelism in the
 * QMCPACK Monte Carlo code" (arXiv 2209.14487): for every walker of a crowd
 * (Sec. III, a subset of the walkers that moves through the algorithm in
 * lock-step, driven by one host thread) and for every particle in turn, the
 * per-particle steps of Alg. 1 -- propose a move, evaluate the wavefunction
 * ratio and the derivatives at the new position, accept or reject -- followed
 * by the local energy (Alg. 1).  The calls are the paper's batched "multi-walker" API
 * (Sec. III): one call advances every walker of the crowd.
 *
 * Wavefunction (not specified by the paper; textbook definitions):
 *   Psi_T(R) = det A_up det A_dn exp(sum_{i<j} u(r_ij)),
 *   A_sigma[i][j] = phi_j(r_i) with phi_j a periodic uniform cubic B-spline on a
 *   G^3 grid over a cubic box of edge L, and u(r) = a r / (1 + b r) (two-body
 *   Pade Jastrow, a depends on equal/opposite spins, minimum-image distance).
 *
 * Conventions shared by every call:
 *   - Status codes only; nothing is thrown across the ABI.  On a non-OK status
 *     cq_last_error() returns a thread-local message.
 *   - Invalid sizes or pointers give CQ_EINVAL before anything is allocated.
 *   - Host arrays passed in are copied; host arrays passed out are owned by the
 *     caller.  Device buffers allocated by the library are owned by it.
 *   - run_* calls are asynchronous on the crowd's HIP stream; get_* calls
 *     synchronise that stream first.
 *   - A crowd is driven by one host thread at a time; distinct crowds may be
 *     driven concurrently from different threads (the paper's crowds over host
 *     threads, Alg. 4).
 *   - Electrons 0..N-1 are spin up, N..2N-1 spin down; n_up == n_dn == N.
 *   - Positions are FP64, [walker][electron][xyz], row-major.
 */
#ifndef CQ_H
#define CQ_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    CQ_OK = 0,
    CQ_EINVAL = 1,     /* invalid argument or size */
    CQ_ENOMEM = 2,     /* device or host allocation failed */
    CQ_EDEVICE = 3,    /* HIP runtime error (message says which call) */
    CQ_ESINGULAR = 4,  /* a Slater matrix was singular or not finite (message names the walker) */
    CQ_ESTATE = 5,     /* call made in the wrong state (e.g. run before positions are set) */
    CQ_EIO = 6         /* a file could not be read or written (the tile cache) */
} cq_status;

typedef enum { CQ_FP64 = 0, CQ_MIXED = 1 } cq_precision;

/* Kernel classes whose device time can be measured with cq_crowd_get_kernel_timing. */
typedef enum {
    CQ_KERNEL_VGL = 0,      /* B-spline VGL at the proposals: per move fused with the ratio, Jastrow
                               and the previous decision (MULTI), per window with all its moves
                               (WINDOW), or for the electrons of a round's gather range (BATCH) */
    CQ_KERNEL_RESOLVE = 1,  /* decisions: of a window's last move (MULTI), of a round's moves with
                               the products they need (BATCH) */
    CQ_KERNEL_UPDATE = 2,   /* Sherman-Morrison / delayed rank-k inverse update */
    CQ_KERNEL_ENERGY = 3,   /* local energy */
    CQ_KERNEL_INVERSE = 4,  /* FP64 Gauss-Jordan inversion (initial and periodic recompute) */
    CQ_KERNEL_PROPOSE = 5,  /* proposals and stencils of a round's gather range, and the Jastrow
                               sums of its new candidates (BATCH) */
    CQ_KERNEL_VIRTUAL = 6,  /* ratio-only virtual moves (cq_crowd_virtual_ratios) */
    CQ_KERNEL_COUNT = 7
} cq_kernel_kind;

/* Mapping of the moves to the GPU.  All paths compute the same Markov chain
   (same proposals, uniforms and decisions); their sums are grouped differently,
   so results agree to rounding, and each path is bit-reproducible on its own
   (independent of how walkers form crowds).
   CQ_PATH_MULTI:   one kernel launch per move, several workgroups per walker (one
                    per chunk of orbitals), the previous move decided inside the
                    next launch; uses every CU even for few walkers.
   CQ_PATH_WINDOW:  one workgroup per walker runs all k moves of an update window
                    in one launch (decisions and window bookkeeping stay in the
                    workgroup); far fewer launches, one CU per walker.
   CQ_PATH_BATCH:   the k proposals of a window are evaluated in one launch over
                    all walkers (a VMC proposal depends only on its own electron,
                    which has not moved yet), then one workgroup per walker
                    decides the window's moves in order from the k x k products of
                    proposal rows and inverse columns.
   CQ_PATH_SWEEP:   one workgroup per walker runs every move of a sweep in one
                    launch, the walker's inverses in LDS, a Sherman-Morrison update
                    after each accepted move (delay rank 1).  For small systems,
                    where launches would dominate: N <= 64 and N a multiple of 4.
   CQ_PATH_AUTO:    CQ_PATH_SWEEP when it applies and the delay rank is 0 or 1,
                    else CQ_PATH_BATCH. */
typedef enum {
    CQ_PATH_AUTO = 0,
    CQ_PATH_MULTI = 1,
    CQ_PATH_WINDOW = 2,
    CQ_PATH_BATCH = 3,
    CQ_PATH_SWEEP = 4
} cq_kernel_path;

typedef struct cq_system cq_system;  /* orbitals + Jastrow + box + electron counts (opaque) */
typedef struct cq_crowd cq_crowd;    /* walkers moved in lock-step (opaque) */

/* ---------------------------------------------------------------- systems */

/* Create an empty system of n_up + n_dn electrons in a cubic box of edge box_L
   (bohr).  Requires n_up == n_dn >= 1, box_L > 0. */
cq_status cq_system_create(int n_up, int n_dn, double box_L, cq_system** out);

/* Load B-spline coefficients, layout [gx][gy][gz][n_orb] row-major (orbital
   index fastest), elem_bytes 4 (FP32) or 8 (FP64), gx == gy == gz >= 4,
   n_orb == n_up.  coefs_on_device = 0: host array, copied to the device.
   coefs_on_device = 1: a device buffer that the system BORROWS (e.g. a torch
   tensor); it must stay alive and unchanged while the system exists.
   The FP32 table drives the mixed-precision path, the FP64 table the FP64 path;
   a system may hold both (load twice). */
cq_status cq_system_load_bspline(cq_system* sys, const void* coefs, int elem_bytes, int gx, int gy, int gz,
                                 int n_orb, int coefs_on_device);

/* Generate a seeded coefficient table on the device (owned by the system):
   coefficient with linear index idx = ((ix G + iy) G + iz) n_orb + n is
   2 u - 1, u the 53-bit uniform of Philox4x32-10 (Salmon et al. SC'11) with key
   (seed low, seed high) and counter (idx low, idx high, 0xC0EF, 0), u =
   ((w1:w0) >> 11) 2^-53.  elem_bytes 4 stores the FP64 value rounded to
   nearest FP32.  Synthetic stand-in for fitted orbitals of any size. */
cq_status cq_system_fill_bspline_philox(cq_system* sys, uint64_t seed, int elem_bytes, int grid, int n_orb);

/* Two-body Pade Jastrow u(r) = a r / (1 + b r): a_par for equal spins,
   a_anti for opposite spins.  Without this call the Jastrow factor is 1. */
cq_status cq_system_load_pade_j2(cq_system* sys, double a_par, double a_anti, double b);

/* One-body Pade Jastrow around fixed centres (the electron-ion factor of a Slater-Jastrow
   wavefunction, part of the local-energy step of Alg. 1):
     ln J1 = + sum_i sum_I u1(|r_i - R_I|),  u1(r) = a r / (1 + b r),
   minimum-image distances.  centres: host array [n_centres][3] (bohr), copied;
   0 <= n_centres <= 64 (0 removes the factor); a finite, b >= 0.  It enters every
   move's ratio, the DMC drift and the local energy, in FP64 in both precisions.  Call it
   before creating crowds of the system.  Errors: CQ_EINVAL (bad arguments, nothing
   changed), CQ_EDEVICE. */
cq_status cq_system_load_pade_j1(cq_system* sys, const double* centres, int n_centres, double a, double b);

/* Add the electron-electron Coulomb energy to the local energy (enable = 1; 0 removes it):
   the electrons (charge -1) in the periodic box with a uniform neutralising background, by
   Ewald summation,
     V = sum_{i<j} erfc(alpha r_ij) / r_ij + (2 pi / L^3) sum_{k != 0} exp(-k^2/4alpha^2) / k^2
         |sum_i exp(i k.r_i)|^2 - alpha Ne / sqrt(pi) - pi Ne^2 / (2 alpha^2 L^3),
   minimum-image pairs, alpha L = 10.1 and k = 2 pi n / L with n^2 <= 18^2 (each left-out term
   below about 1e-12 of its kind), in FP64 for every precision; one electron per cell gives the
   Madelung energy -2.8372975 / (2 L).  Crowds created afterwards include it in E_L (and so in
   the DMC weights and energies); the kinetic part is unchanged.  Errors: CQ_EINVAL, CQ_ENOMEM. */
cq_status cq_system_set_coulomb(cq_system* sys, int enable);

void cq_system_destroy(cq_system* sys);

/* ----------------------------------------------------------------- crowds */

typedef struct {
    int precision;        /* cq_precision: CQ_MIXED uses the FP32 table and FP32 inverses,
                             FP64 for log|det|, the recompute and every sum over walkers */
    int delay_rank;       /* k: 1 = Sherman-Morrison after every accepted move, 2..32 = delayed
                             rank-k update (the batched path closes a window after k accepted
                             moves, the per-move paths after k proposals); 0 = autotune: the
                             first run_vmc (or cq_crowd_autotune) times sweeps at k = 1, 2, 4,
                             ..., min(32, n_up) and keeps the fastest (the whole-sweep path
                             always uses k = 1) */
    int recompute_every;  /* sweeps between FP64 recomputes of the inverses (0 = never) */
    uint64_t seed;        /* Philox key of the move random numbers */
    uint32_t first_uid;   /* walker w of this crowd has uid first_uid + w (random streams) */
    void* hip_stream;     /* borrowed hipStream_t to run on, or NULL: the crowd makes its own */
    int use_graph;        /* 1: capture one sweep as a hipGraph and replay it */
    int kernel_path;      /* how the moves are mapped to the GPU (cq_kernel_path) */
    int max_walkers;      /* capacity for a DMC population (0: the initial walker count); the
                             per-walker buffers are sized for it */
    int streams;          /* batched path: 2 (or 0) runs the next round's gather on a second
                             stream beside the current round's decisions and update; 1 runs
                             every kernel in order on one stream (each then has the GPU alone) */
} cq_crowd_desc;

/* Create a crowd of walkers_per_system[s] walkers of each system s.  Allocates every device
   buffer up front (CQ_ENOMEM if the device cannot hold them).
   Several systems (n_systems > 1, the batched uneven workload): the walkers of every system
   share the crowd's stream and are ordered system by system in every per-walker array (walker
   uids continue from one system to the next); the descriptor applies to every system (delay
   rank capped at each system's N); max_walkers > 0 is the capacity over all systems, shared
   out in proportion to walkers_per_system.  cq_crowd_run_dmc_systems moves the walkers of all
   systems with the same launches (per spin block and window step, one launch of the
   walker-resident move kernel over every system's walkers, largest system first, and one update
   launch over their strips), then runs each system's energy and branching; VMC sweeps run system
   after system.  The parity-mode calls (forced decisions and branching, move records) take
   crowds of one system. */
cq_status cq_crowd_create(const cq_system* const* systems, const int* walkers_per_system, int n_systems,
                          const cq_crowd_desc* desc, cq_crowd** out);

/* Set positions R [W][Ne][3] (host, or device when on_device = 1), then
   evaluate every orbital at every electron, invert both Slater matrices in
   FP64 (Gauss-Jordan with partial pivoting) and compute log|det|, sign and the
   local energy.  CQ_ESINGULAR if a matrix is singular.  Resets the sweep
   counter to first_step. */
cq_status cq_crowd_set_positions(cq_crowd* c, const double* R, int on_device, uint32_t first_step);

/* The VMC sweep of Alg. 1, n_sweeps times: each electron in index order proposes
   r' = wrap(r + sigma z), z ~ N(0, I_3) from Philox counter (uid, step, e, 0/1),
   accepts iff u < rho_D^2 exp(2 dlnJ) with u from counter (uid, step, e, 2), and
   updates the inverse.  The local energy is evaluated after every sweep.
   Asynchronous. */
cq_status cq_crowd_run_vmc(cq_crowd* c, int n_sweeps, double sigma);

/* Recompute every inverse and log|det| from the current rows in FP64 now.
   If max_drift is non-NULL it receives max |log|det| kept - log|det| recomputed|
   over walkers and spins.  Synchronous.  CQ_ESINGULAR if a matrix is singular or
   not finite (the message names the walker). */
cq_status cq_crowd_recompute(cq_crowd* c, double* max_drift);

/* Drift record of the FP64 recomputes (the periodic ones inside run_vmc / run_dmc,
   every recompute_every sweeps or generations, and cq_crowd_recompute):
   last [W][2] (may be NULL): |log|det| kept - log|det| recomputed| at the last
   inversion of each walker and spin; max_drift (may be NULL): the largest drift of
   any recompute since the positions were set (+inf if one was not finite);
   n_recomputes (may be NULL): how many recomputes ran since then.  Synchronises
   the crowd's stream. */
cq_status cq_crowd_get_drift(cq_crowd* c, double* last, double* max_drift, int* n_recomputes);

/* The get calls below synchronise the crowd's stream, copy to caller-owned host
   memory and then report any error the asynchronous run left on the device:
   CQ_ESINGULAR when a recompute inside run_vmc / run_dmc met a singular or
   non-finite matrix, CQ_ESTATE when the update-window bookkeeping went out of range
   (an internal error); the message names the walker.  The data are copied either
   way. */

/* log|det A_sigma| [W][2] (FP64) and sign [W][2] (+1/-1). */
cq_status cq_crowd_get_logdet(cq_crowd* c, double* logdet, int* sign);
/* accepted and proposed single-electron moves per walker [W] since set_positions. */
cq_status cq_crowd_get_acceptance(cq_crowd* c, int64_t* accepted, int64_t* proposed);
/* kinetic local energy -1/2 sum_i lap_i Psi / Psi per walker [W] after the last sweep. */
cq_status cq_crowd_get_local_energy(cq_crowd* c, double* e_l);
/* positions [W][Ne][3] (several systems: each system's block [W_s][Ne_s][3] in turn);
   n_walkers_per_system (may be NULL) receives the walker count of every system. */
cq_status cq_crowd_get_positions(cq_crowd* c, double* R, int* n_walkers_per_system);
/* the kept inverses as FP64 [W][2][N][N], element [w][s][j][i] = (A_s^-1)[j][i]. */
cq_status cq_crowd_get_inverse(cq_crowd* c, double* ainv);

/* Parity-mode buffers are indexed by walker slot with the walker capacity
   Wcap = max(initial walkers, max_walkers) as stride: [sweep or generation][e][Wcap]
   (under DMC the slot is the walker's position in the generation's population).

   The crowd follows the given decisions flags[sweep][e][Wcap] (1 accept, 0
   reject, 2 or more: the walker's own decision) for the next n_sweeps VMC sweeps
   or DMC generations instead of its own, while still recording its own
   probability.  flags = NULL switches it off. */
cq_status cq_crowd_set_forced_decisions(cq_crowd* c, const uint8_t* flags, int n_sweeps);
/* DMC parity mode: the branching of the next n_generations generations gives
   walker slot w the multiplicity mult[generation][Wcap] (0..3) instead of
   floor(w + u_b), so the population follows a reference run; the weights, their
   sums and E_T are still the crowd's own.  mult = NULL switches it off.
   CQ_EINVAL for a multiplicity outside 0..3. */
cq_status cq_crowd_set_forced_branching(cq_crowd* c, const int* mult, int n_generations);
/* Record per-move rho_D, dlnJ, P and the decision for the next n_sweeps sweeps or
   generations (0 switches recording off). */
cq_status cq_crowd_record_moves(cq_crowd* c, int n_sweeps);
/* Copy the records out: arrays [n_sweeps][Ne][Wcap]; any pointer may be NULL. */
cq_status cq_crowd_get_move_records(cq_crowd* c, double* rho, double* dlnj, double* prob, uint8_t* acc);
/* The proposed positions r' of the recorded DMC moves, [n_sweeps][Ne][Wcap][3] (FP64): the
   state that a drift-diffusion proposal depends on (the drift at the electron's position) is
   the crowd's own, so a check of its ratios takes the positions from here.  Entries that no DMC
   move wrote (VMC sweeps, empty walker slots) are NaN.  CQ_ESTATE if recording is off. */
cq_status cq_crowd_get_move_proposals(cq_crowd* c, double* rnew);
/* Drift-diffusion moves accepted and proposed over every DMC generation the crowd
   has run (the populations that moved, before their branching). */
cq_status cq_crowd_get_dmc_moves(cq_crowd* c, int64_t* accepted, int64_t* proposed);

/* Delay-rank autotuning for a crowd created with delay_rank = 0: time
   sweeps_per_candidate sweeps (eager launches, HIP events) at every candidate
   k = 1, 2, 4, ..., min(32, n_up) and keep the fastest; *chosen_k (may be NULL)
   receives it.  The timed sweeps are ordinary sweeps of the chain (they advance
   the positions and the random-number step).  run_vmc calls it with one sweep
   per candidate when the crowd has not been tuned.  On the whole-sweep path
   (CQ_PATH_SWEEP) nothing is timed and k stays 1.  Errors: CQ_EINVAL,
   CQ_ESTATE (positions not set). */
cq_status cq_crowd_autotune(cq_crowd* c, int sweeps_per_candidate, int* chosen_k);

/* The delay rank in use (after autotuning, the chosen one). */
cq_status cq_crowd_get_delay_rank(cq_crowd* c, int* k);

/* Rounds per spin block of the batched path.  A spin block of N electrons needs at most
   N / k rounds (delay rank k), but at ordinary acceptance far fewer; by default each sweep
   runs as many as recent sweeps needed plus a margin (learned from a report the device
   writes after each block, without synchronising), and a tail kernel then finishes, one
   move at a time, any walker with electrons left.  rounds = 0: that default; rounds >= 1:
   exactly that many (at most N / k) before the tail kernel, for callers that know their
   acceptance and for tests of the tail.  The chain is the same either way (decisions to
   rounding); only the speed changes.  Errors: CQ_EINVAL. */
cq_status cq_crowd_set_round_plan(cq_crowd* c, int rounds);
/* The planned rounds of each spin block [2] (0 on the other paths). */
cq_status cq_crowd_get_round_plan(cq_crowd* c, int* rounds);

/* Launch shapes of the batched path (the crowd batching of Sec. III; the paper's drivers
   fix theirs per kernel, Sec. II-D).  Neither changes the chain (same proposals and
   uniforms, decisions to rounding), only the speed:
     candidates            Q, the upcoming proposals whose orbital rows one round evaluates
                           per walker; from the delay rank k (or 2, if larger) up to the
                           value the crowd was created with, min(88, 3 k_max, N); 0 = that
                           default.  A round examines at most Q candidates and closes after
                           k acceptances, so Q >= k keeps N / k rounds enough for a block.
     gather_blocks_per_cu  workgroups per compute unit of the persistent orbital gather
                           while it runs beside the decisions and the update (two-stream
                           schedule), 1..8; 0 = the built-in rule (1 for the wave-sliced
                           gather at N >= 256 in FP32 / 128 in FP64, else 3).
     update_kernel         the rank-k update of an FP64 crowd: 1 = vector units (k_flush_vec),
                           2 = FP64 matrix cores (strips of 16 rows, N % 16 == 0 and N <= 1024;
                           otherwise the vector units); 0 = the default, vector units.  FP32
                           crowds always take the FP32 matrix-core update when N % 32 == 0 (the
                           field is ignored). */
typedef struct cq_tiles {
    int candidates;
    int gather_blocks_per_cu;
    int update_kernel;
} cq_tiles;

/* Set the launch shapes (values as above; 0 keeps a field's default).  Takes effect from
   the next sweep (a captured sweep graph is rebuilt).  Other paths accept and ignore them.
   Errors: CQ_EINVAL (out of range; nothing changes). */
cq_status cq_crowd_set_tiles(cq_crowd* c, const cq_tiles* t);
/* The launch shapes in use, defaults resolved (candidates = Q; gather_blocks_per_cu and
   update_kernel (1 vector units, 2 matrix cores) as launched). */
cq_status cq_crowd_get_tiles(cq_crowd* c, cq_tiles* t);

/* Tile autotuning for the batched path.  With cache_path non-NULL and an entry in it for
   this device (architecture name and compute-unit count), N, walkers, precision and delay
   rank, apply that entry and time nothing (*from_cache = 1).  Otherwise time
   sweeps_per_candidate sweeps (eager launches, HIP events, after one untimed sweep that
   learns the round plan) for every candidate: Q in {1.5 k, 2 k, default} within the
   limits above, gather workgroups per CU in {1, 2, 3} and, for an FP64 crowd whose N the
   matrix-core update takes, both update kernels; keep the fastest and, with
   cache_path, append it to the cache (*from_cache = 0).  Every timed sweep is an ordinary
   sweep of the chain.  On other paths nothing is timed and the defaults stay.  chosen and
   from_cache may be NULL.  Errors: CQ_EINVAL, CQ_ESTATE (positions not set), CQ_EIO (the
   cache cannot be written). */
cq_status cq_crowd_autotune_tiles(cq_crowd* c, int sweeps_per_candidate, const char* cache_path, cq_tiles* chosen,
                                  int* from_cache);

/* The tile cache (host only, no GPU call).  A JSON file: an array with one object per line,
   {"device": "...", "n": N, "walkers": W, "precision": "mixed"|"fp64", "delay_rank": k,
   "candidates": Q, "gather_blocks_per_cu": g, "update_kernel": u, "ms_per_sweep": t}
   (an entry without update_kernel reads as 0).  Lookup returns the last
   entry that matches every key (*found = 0 and *out untouched if none, or if the file does
   not exist); lines that do not parse are skipped.  Store appends an entry (creating the
   file), keeping the file a valid JSON array.  device: at most 127 bytes, no '"' or '\'.
   Errors: CQ_EINVAL, CQ_EIO. */
cq_status cq_tile_cache_find(const char* path, const char* device, int n, int walkers, int precision, int delay_rank,
                             cq_tiles* out, int* found);
cq_status cq_tile_cache_store(const char* path, const char* device, int n, int walkers, int precision, int delay_rank,
                              const cq_tiles* t, double ms_per_sweep);

/* The kernel path in use (cq_kernel_path; CQ_PATH_AUTO resolved at creation; for a
   crowd of several systems, the first system's). */
cq_status cq_crowd_get_path(cq_crowd* c, int* path);

/* Diffusion Monte Carlo (paper Alg. 1 with a drift-diffusion proposal and
   reweighting / branching; Sec. II-A).  Runs n_generations
   generations of the crowd's population at time step tau: per generation one
   sweep of drift-diffusion moves (Metropolis-Hastings with the drifted Gaussian
   Green's function; moves that cross a node are rejected), the local energy,
   then branching:
     E_c = E_L clipped to E_T +- 0.2 sqrt(Ne / tau),
     w = exp(-tau ((E_c,old + E_c,new) / 2 - E_T)),  m = min(3, floor(w + u_b)),
     E_est = sum w E_L / sum w,  E_T <- E_est - ln(N / n_target) / tau.
   Children follow their parent in population order; copy 0 keeps the parent's
   uid, copy c >= 1 gets a new one from the counter generator.  e_trial: the
   starting E_T (NaN: continue with the current one).  history (may be NULL):
   host array [n_generations][4] of population, sum of weights, E_est and E_T
   after each generation.  Moves use the walker-resident per-move kernel
   whatever the crowd's kernel path.  Synchronous: the population size is read
   back after every generation.  Errors: CQ_EINVAL (bad arguments), CQ_ESTATE
   (positions not set, or the population died out or outgrew max_walkers; the
   crowd then keeps the last complete generation). */
cq_status cq_crowd_run_dmc(cq_crowd* c, int n_generations, double tau, double e_trial, int n_target,
                           double* history);

/* Virtual moves: the ratio-only wavefunction evaluations of the local-energy step of Alg. 1
   (the energy evaluation is the expensive part of a step, Sec. II-A; a non-local energy term
   needs Psi at quadrature points around an electron without moving it).  For every walker w,
   electron e (row i of its spin block) and point q of the current state:
     r_q = wrap(r_e + offsets[q]),  rho_D = sum_j phi_j(r_q) (A^-1)_{j,i},
     dlnJ = sum_{m != e} [u(|r_q - r_m|) - u(|r_e - r_m|)],  ratio = rho_D exp(dlnJ),
   with phi in the crowd's precision (FP32 table in mixed precision, the products with the
   inverse column summed in FP64) and the Jastrow pair terms likewise.  offsets: host array
   [n_q][3] (bohr), 1 <= n_q <= 64.  ratio, rho, dlnj: [W][Ne][n_q] FP64, any may be NULL;
   out_on_device = 0: host arrays, the call synchronises; 1: device buffers owned by the
   caller, the call is asynchronous on the crowd's stream.  Nothing in the crowd changes.
   Errors: CQ_EINVAL, CQ_ESTATE (positions not set). */
cq_status cq_crowd_virtual_ratios(cq_crowd* c, const double* offsets, int n_q, double* ratio, double* rho,
                                  double* dlnj, int out_on_device);

/* DMC generations of every system of the crowd (one or several), as cq_crowd_run_dmc does for
   one: e_trial [n_systems] starting trial energies (NULL or NaN entries: continue with the
   current ones), n_target [n_systems] target populations (NULL: the starting walker counts),
   history (may be NULL) [n_generations][n_systems][4] of population, sum of weights, E_est and
   E_T.  With several systems, each generation moves the walkers of all systems with the same
   launches (see cq_crowd_create), then branches each system's population on its own.
   Synchronous.  Errors as cq_crowd_run_dmc (CQ_ESTATE names the system). */
cq_status cq_crowd_run_dmc_systems(cq_crowd* c, int n_generations, double tau, const double* e_trial,
                                   const int* n_target, double* history);

/* Current number of walkers (changes under DMC branching). */
cq_status cq_crowd_get_population(cq_crowd* c, int* n_walkers);

/* uids of the current walkers, [n_walkers]. */
cq_status cq_crowd_get_uids(cq_crowd* c, uint32_t* uids);

/* Record HIP events on the crowd's stream around every launch of the kernel
   kinds in kind_mask (bit 1 << cq_kernel_kind; 0 switches timing off) and read
   back the summed device time in ms and the launch count of one kind since the
   last set call.  While timing is on, sweeps are launched eagerly (no graph).
   Up to 65536 launches per kind are timed between set calls. */
cq_status cq_crowd_set_kernel_timing(cq_crowd* c, int kind_mask);
cq_status cq_crowd_get_kernel_timing(cq_crowd* c, int kind, double* total_ms, int64_t* launches);

/* Wait for all work queued on the crowd's stream. */
cq_status cq_crowd_synchronize(cq_crowd* c);

void cq_crowd_destroy(cq_crowd* c);

/* ------------------------------------------- complex orbitals, general cells */

/* Bloch orbitals with a twist in a general (triclinic) periodic cell: the same move of
   Alg. 1 with complex orbitals and determinants.  FP64 throughout.
     phi_j(r) = exp(i k.r) s_j(f),  f = r L^-1 (fractional coordinates; L [3][3] holds the
     lattice vectors as rows, r = f L), s_j a periodic uniform cubic B-spline over a G^3 grid
     in f with complex coefficients (control point q of an axis at f = q / G).
   Cartesian derivatives come through L^-1 (gradient) and the metric L^-T L^-1 with the full
   Hessian in f (Laplacian); the twist adds i k s to the gradient and 2 i k.grad s - k^2 s to
   the Laplacian.  Positions are kept wrapped into the cell, f - floor(f), and phi is taken at
   the wrapped position (|Psi| and every ratio of derivatives are unaffected; the phase of Psi
   follows the wrapped coordinates).  The pair Jastrow takes the minimum image in fractional
   coordinates, d - rint(d L^-1) L.  A move is accepted when u < |rho_D|^2 exp(2 dlnJ), the
   Slater inverses follow each acceptance by a Sherman-Morrison update (delay rank 1), and the
   kinetic local energy -1/2 sum_i lap_i Psi / Psi is complex (its real part is the estimator).
   Random numbers as for cq_crowd_run_vmc: Philox counters (uid, step, e, 0..2).  VMC only. */
typedef struct cq_csystem cq_csystem;  /* complex orbitals + cell + twist + Jastrow (opaque) */
typedef struct cq_ccrowd cq_ccrowd;    /* walkers of a complex system (opaque) */

/* n electrons per spin (1..512), lattice [3][3] (rows, bohr; non-degenerate), twist [3]
   (Cartesian, 1/bohr; NULL = 0).  Errors: CQ_EINVAL. */
cq_status cq_csystem_create(int n, const double* lattice, const double* twist, cq_csystem** out);
/* Complex coefficients [G][G][G][n_orb] (interleaved real, imaginary; orbital index
   fastest): elem_bytes 16 (complex128, for CQ_FP64 crowds) or 8 (complex64, for CQ_MIXED
   crowds); a system may hold both, on one grid.  Grid G >= 4, n_orb == n.
   coefs_on_device = 0: host array, copied; 1: a device buffer the system borrows (it must
   outlive the system).  Errors: CQ_EINVAL, CQ_ENOMEM. */
cq_status cq_csystem_load_bspline(cq_csystem* sys, const void* coefs, int elem_bytes, int grid, int n_orb,
                                  int coefs_on_device);
/* Pade pair Jastrow u(r) = a r / (1 + b r) (a_par equal spins, a_anti opposite). */
cq_status cq_csystem_load_pade_j2(cq_csystem* sys, double a_par, double a_anti, double b);
void cq_csystem_destroy(cq_csystem* sys);

/* A crowd of `walkers` walkers (uids first_uid + w) on a borrowed hipStream_t or its own
   (hip_stream NULL).  precision CQ_FP64 reads the complex128 table; CQ_MIXED reads the
   complex64 table (half the spline bytes), every sum, row, inverse and energy staying FP64.
   Device buffers: inverses and orbital rows, 16 (2 n^2 + 10 n^2) bytes per walker, plus a
   Gauss-Jordan workspace of 64 n^2 bytes.  Errors: CQ_EINVAL (no table of that precision),
   CQ_ENOMEM, CQ_EDEVICE. */
cq_status cq_ccrowd_create(const cq_csystem* sys, int walkers, int precision, uint64_t seed, uint32_t first_uid,
                           void* hip_stream, cq_ccrowd** out);
/* Positions R [W][2n][3] (host), then the orbital rows of every electron, both inverses
   (Gauss-Jordan with partial pivoting by modulus), log|det|, phase and E_L.  Resets the
   counters; the next sweep uses step first_step.  Errors: CQ_EINVAL, CQ_ESINGULAR (names the
   walker). */
cq_status cq_ccrowd_set_positions(cq_ccrowd* c, const double* R, uint32_t first_step);
/* n_sweeps sweeps (one kernel launch each, every walker at once, each electron in index order)
   and the local energy after each; asynchronous.  Errors: CQ_EINVAL, CQ_ESTATE. */
cq_status cq_ccrowd_run_vmc(cq_ccrowd* c, int n_sweeps, double sigma);
/* Fresh inverses, log|det| and phase from the current orbital rows (FP64 recompute);
   *max_drift (may be NULL) = max |log|det| kept - log|det| fresh| over walkers and spins. */
cq_status cq_ccrowd_recompute(cq_ccrowd* c, double* max_drift);
/* log|det| [W][2] and phase [W][2] (radians in [-pi, pi]). */
cq_status cq_ccrowd_get_logdet(cq_ccrowd* c, double* logdet, double* phase);
/* E_L [W][2] (real, imaginary). */
cq_status cq_ccrowd_get_local_energy(cq_ccrowd* c, double* el);
cq_status cq_ccrowd_get_positions(cq_ccrowd* c, double* R);
cq_status cq_ccrowd_get_acceptance(cq_ccrowd* c, int64_t* accepted, int64_t* proposed);
/* A^-1 of one walker and spin, [n][n][2] (row j orbital, column i electron; real, imaginary). */
cq_status cq_ccrowd_get_inverse(cq_ccrowd* c, int walker, int spin, double* out);
/* Keep the ratio rho [S][2n][W][2], ln J change, acceptance probability and decision of
   every move of the next n_sweeps sweeps (0: stop recording).  get_move_records copies them
   out (CQ_ESTATE when recording is off). */
cq_status cq_ccrowd_record_moves(cq_ccrowd* c, int n_sweeps);
cq_status cq_ccrowd_get_move_records(cq_ccrowd* c, double* rho, double* dlnj, double* prob, uint8_t* acc);
/* HIP events around every launch of the sweep kernel while on (set_timing also clears the
   record); get_timing returns their total device time (ms) and count, then clears them. */
cq_status cq_ccrowd_set_timing(cq_ccrowd* c, int on);
cq_status cq_ccrowd_get_timing(cq_ccrowd* c, double* ms, int64_t* launches);
cq_status cq_ccrowd_synchronize(cq_ccrowd* c);
void cq_ccrowd_destroy(cq_ccrowd* c);

/* ------------------------------------------------------------ batched inverse */

/* The FP64 recompute of the Slater inverses (Gauss-Jordan with partial pivoting,
   the same kernels as the periodic recompute of a crowd) for matrices the caller
   holds, e.g. walkers that arrive from elsewhere with positions only.
   A     device [nmat][n][n], row-major, A[m][i][j] = phi_j(r_i) (elem_bytes 4: FP32,
         8: FP64; promoted to FP64 for the elimination);
   Minv  device [nmat][n][n] of the same element type: Minv[m][a][j] = (A_m^-1)[j][a],
         so row a is the inverse column of electron a (the crowds' layout);
   logdet, sign  device [nmat]: log|det A_m| (FP64) and its sign (+1/-1).
   All pointers are device pointers owned by the caller; A is only read.  The
   library allocates a workspace of about nmat n (n + 144) 8 bytes for 64 < n <= 1024
   (nmat n (n + 80) 8 bytes above) for the duration of the call.  Runs on hip_stream (NULL: the null stream) and
   returns when the results are written.  Errors: CQ_EINVAL (NULL pointer,
   elem_bytes not 4 or 8, n outside 1..2048, nmat < 1), CQ_ENOMEM (workspace),
   CQ_ESINGULAR (a pivot at or below n eps max|A_ij| or not finite; the message
   names the pair of matrices 2w, 2w+1 holding it). */
cq_status cq_slater_inverse(const void* A, int elem_bytes, int n, int nmat, void* Minv, double* logdet, int* sign,
                            void* hip_stream);

/* Size of the library's static inversion workspace (bytes, per GPU). */
#define CQ_STATIC_WORK_BYTES ((uint64_t)64 << 20)

/* cq_slater_inverse without any allocation, for callers that cannot allocate device
   memory (work recorded under graph capture, tight serving loops, harnesses that forbid
   hipMalloc).  Same arguments, results and errors as cq_slater_inverse, computed by the
   same kernels, but the workspace is a static device array of CQ_STATIC_WORK_BYTES
   bytes that the library holds on each GPU it runs on until the process ends (looked up
   at the first call on a device); the call makes no hipMalloc, hipFree or other
   allocating call.  The workspace needed is about nmat n (n + 144) 8 bytes for
   64 < n <= 1024, nmat n (n + 80) 8 bytes above (nmat (4 + 8) bytes for n <= 64):
   CQ_EINVAL names the size when it exceeds the array (64 MiB holds, e.g., 7 matrices of
   n = 1024 or 81 of n = 256).  Every call on one
   GPU shares that GPU's array: calls that overlap on one GPU (several host threads, or
   streams without ordering between them) race; serialise them.  Returns when the
   results are written. */
cq_status cq_slater_inverse_static(const void* A, int elem_bytes, int n, int nmat, void* Minv, double* logdet,
                                   int* sign, void* hip_stream);

/* Plain streaming device-to-device copy of `bytes` bytes (multiple of 16,
   16-byte aligned pointers) with a library kernel on `hip_stream` (NULL: the
   null stream), synchronous.  Its hardware traffic counters give the scale
   factor between counter readings and bytes moved. */
cq_status cq_device_copy(void* dst, const void* src, uint64_t bytes, void* hip_stream);

/* Thread-local message of the last non-OK status ("" if none). */
const char* cq_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* CQ_H */
