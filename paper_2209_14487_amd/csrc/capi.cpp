// C ABI and crowd runtime: device buffers, the per-sweep launch sequence
// (optionally captured once as a hipGraph and replayed), the FP64 recompute
// schedule, parity-mode buffers and per-kernel event timing.
//
// One sweep (the VMC sweep of Alg. 1 over all walkers of the crowd in lock-step,
// the batched form of Alg. 3/4) is, for e = 0 .. Ne-1:
//   k_move(e, resolving e-1)  [-> k_move(resolve e only) -> k_flush(spin) at the
//   end of a window]
// then the local energy and the step counter.  Windows cover k consecutive
// electrons of one spin and never span spins or sweeps.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "cq.h"
#include "cq_host.h"
#include "cq_internal.h"

namespace {

thread_local std::string g_err;

cq_status fail(cq_status s, const std::string& msg)
{
    g_err = msg;
    return s;
}

#define HIP_TRY(x)                                                                                   \
    do {                                                                                             \
        hipError_t e_ = (x);                                                                         \
        if (e_ != hipSuccess) return fail(CQ_EDEVICE, std::string(#x) + ": " + hipGetErrorString(e_)); \
    } while (0)

constexpr int kEventCap = 1 << 16;  // timed launches kept per kernel kind between reads

}  // namespace

cq_status cq::host_fail(cq_status s, const std::string& msg) { return fail(s, msg); }

struct cq_system {
    int n_up = 0, n_dn = 0;
    double L = 0.0;
    int G = 0, n_orb = 0;
    void* table[2] = {nullptr, nullptr};  // [0] FP32, [1] FP64
    bool owned[2] = {false, false};
    int use_j2 = 0;
    double a_par = 0.0, a_anti = 0.0, b = 1.0;
    // one-body Jastrow (cq_system_load_pade_j1): centres on the device
    double* ions = nullptr;
    int n_ions = 0;
    double j1_a = 0.0, j1_b = 1.0;
    // Ewald electron-electron energy in E_L (cq_system_set_coulomb)
    int coulomb = 0, nmax = 0, nk = 0;
    double alpha = 0.0;
    int4* kvec = nullptr;
    double* kfac = nullptr;
};

struct cq_crowd {
    const cq_system* sys = nullptr;
    int W = 0, n = 0, ne = 0, K = 1, Q = 1, QR = 1, prec = CQ_MIXED, recompute_every = 0, use_graph = 0;
    int Wcap = 0;  // capacity of the per-walker buffers (DMC populations)
    int Kcap = 1;  // largest delay rank the window buffers hold
    // batched path: candidate buffers hold Qcap per walker; q_req (0: the default rule) and
    // vgl_wg (gather workgroups per CU beside the update, 0: built-in) are cq_crowd_set_tiles'
    int Qcap = 1, q_req = 0, vgl_wg = 0, upd_kernel = 0;
    bool autotune = false, tuned = false;
    int path = CQ_PATH_WINDOW;
    uint64_t seed = 0;
    uint32_t first_uid = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    // second stream of the batched path: the gather for round r+2 runs on it while round
    // r+1 is decided and applied on `stream`, then round r+2's Jastrow sums.  Events per
    // round: first gather done (ev_fork, at a spin block's start), decided (ev_dec),
    // columns (or update) done (ev_cols), gathered (ev_gat).
    hipStream_t stream2 = nullptr;
    std::vector<hipEvent_t> ev_fork, ev_dec, ev_cols, ev_gat;
    std::vector<void*> allocs;
    // device state
    double* R = nullptr;
    void* M = nullptr;
    void* VGL = nullptr;
    double* logdet = nullptr;
    int* sign = nullptr;
    long long* nacc = nullptr;
    long long* nprop = nullptr;
    double* eloc = nullptr;
    double* eold = nullptr;
    // DMC: the second set of per-walker buffers (allocated on first use) and branching state
    struct {
        double* R = nullptr;
        void* M = nullptr;
        void* VGL = nullptr;
        double* logdet = nullptr;
        int* sign = nullptr;
        double* eloc = nullptr;
        double* eold = nullptr;
        uint32_t* uid = nullptr;
        long long* nacc = nullptr;
        long long* nprop = nullptr;
    } alt;
    bool have_alt = false;
    // virtual moves: quadrature offsets and (host-output case) result staging
    double* voff = nullptr;
    int voff_cap = 0;
    double* vout = nullptr;
    size_t vout_cap = 0;
    cq::DmcState* dmc_state = nullptr;
    double* dmc_wt = nullptr;
    int* dmc_mult = nullptr;
    int* dmc_off = nullptr;
    double* dmc_hist = nullptr;
    int dmc_hist_cap = 0;
    double* elpart = nullptr;
    int* cnt = nullptr;
    int* welec = nullptr;
    int* wslot = nullptr;
    void* stage = nullptr;
    void* Cbuf = nullptr;
    float* ct = nullptr;
    float* ub = nullptr;
    double* wrho = nullptr;
    double* wG = nullptr;
    double* wlinv = nullptr;
    double* beta = nullptr;
    int* pend = nullptr;
    double* part = nullptr;
    double* rnew = nullptr;
    double* jd = nullptr;
    double* rprop = nullptr;
    size_t* sidx = nullptr;
    void* swt = nullptr;
    double* pmat = nullptr;
    double* tmat = nullptr;
    int* cur = nullptr;
    int* look = nullptr;
    // planned rounds per spin block of the batched path: learned from the rounds recent
    // sweeps needed (pinned report written by the device), or fixed by the caller
    int* used = nullptr;
    int* left = nullptr;
    int* hplan = nullptr;  // pinned host [5]: valid, used/left of spin 0, used/left of spin 1
    int plan[2] = {-1, -1};
    int plan_fixed = 0;
    uint32_t* uid = nullptr;
    cq::Params* prm = nullptr;
    int* status = nullptr;
    double* drift = nullptr;
    unsigned long long* drift_max = nullptr;  // [1]: largest in-run drift since set_positions
    int n_recomputes = 0;                     // in-run recomputes since set_positions
    cq::InvWork inv{};
    // parity mode
    int rec_cap = 0;
    double* rec_rho = nullptr;
    double* rec_dlnj = nullptr;
    double* rec_prob = nullptr;
    uint8_t* rec_acc = nullptr;
    double* rec_rnew = nullptr;  // [rec_cap][Ne][Wcap][3] proposals of DMC moves
    int forced_cap = 0;
    uint8_t* forced = nullptr;
    int mult_cap = 0;
    int* forced_mult = nullptr;  // [generations][Wcap] branching multiplicities to follow
    // several systems: one crowd per system, all on this crowd's stream, and the device views
    // and work lists of the launches that serve the walkers of every system at once
    std::vector<cq_crowd*> subs;
    void* gviews = nullptr;                 // CrowdView<T> [systems]
    int2* gwalk = nullptr;                  // (system, walker) items of each window step
    int4* gstrip = nullptr;                 // (system, walker, strip) items of each window step
    size_t gwalk_cap = 0, gstrip_cap = 0;
    std::vector<int2> hwalk;                // host copies (kept until the next generation's copy)
    std::vector<int4> hstrip;
    std::vector<unsigned char> hviews;
    int n_cu = 0;
    // Ewald buffers (systems with the Coulomb energy)
    double2* ew_phase = nullptr;
    double* ew_part = nullptr;
    // host state
    cq::Params hp{};
    bool ready = false;
    int since_recompute = 0;
    hipGraphExec_t gexec = nullptr;
    // first failing event / wait call while a sweep is enqueued (the enqueue helpers are
    // void, so they keep it here and the calling entry point reports it)
    hipError_t enq_err = hipSuccess;
    // timing
    int timing_mask = 0;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev[CQ_KERNEL_COUNT];
    size_t ev_used[CQ_KERNEL_COUNT] = {};
};

namespace {

template <typename T>
cq::CrowdView<T> view(const cq_crowd* c)
{
    cq::CrowdView<T> v{};
    v.W = c->W;
    v.arow = 5 * c->n;
    v.Wcap = c->Wcap;
    v.n = c->n;
    v.ne = c->ne;
    v.K = c->K;
    v.Q = c->Q;
    v.QR = c->QR;
    v.vgl_wg = c->vgl_wg;
    v.upd_mfma = c->upd_kernel == 2;
    v.G = c->sys->G;
    v.n_orb = c->sys->n_orb;
    v.L = c->sys->L;
    v.table = (const T*)c->sys->table[sizeof(T) == 8 ? 1 : 0];
    v.R = c->R;
    v.M = (T*)c->M;
    v.VGL = (T*)c->VGL;
    v.logdet = c->logdet;
    v.sign = c->sign;
    v.nacc = c->nacc;
    v.nprop = c->nprop;
    v.eloc = c->eloc;
    v.elpart = c->elpart;
    v.cnt = c->cnt;
    v.welec = c->welec;
    v.wslot = c->wslot;
    v.stage = (T*)c->stage;
    v.Cbuf = (T*)c->Cbuf;
    // the batched path hands the matrix-core update its columns transposed
    v.ct = (sizeof(T) == 4 && c->path == CQ_PATH_BATCH && cq::flush_mfma_fits(c->n)) ? c->ct : nullptr;
    v.ub = v.ct ? c->ub : nullptr;
    v.wrho = c->wrho;
    v.wG = c->wG;
    v.wlinv = c->wlinv;
    v.beta = c->beta;
    v.pend = c->pend;
    v.part = c->part;
    v.rnew = c->rnew;
    v.jd = c->jd;
    v.rprop = c->rprop;
    v.sidx = c->sidx;
    v.swt = c->swt;
    v.pmat = c->pmat;
    v.tmat = c->tmat;
    v.cur = c->cur;
    v.look = c->look;
    v.used = c->used;
    v.left = c->left;
    v.uid = c->uid;
    v.seed = c->seed;
    v.use_j2 = c->sys->use_j2;
    v.a_par = c->sys->a_par;
    v.a_anti = c->sys->a_anti;
    v.b = c->sys->b;
    v.ions = c->sys->ions;
    v.n_ions = c->sys->n_ions;
    v.j1_a = c->sys->j1_a;
    v.j1_b = c->sys->j1_b;
    v.prm = c->prm;
    v.rec_rho = c->rec_rho;
    v.rec_dlnj = c->rec_dlnj;
    v.rec_prob = c->rec_prob;
    v.rec_acc = c->rec_acc;
    v.rec_rnew = c->rec_rnew;
    v.forced = c->forced;
    v.status = c->status;
    v.drift = c->drift;
    v.drift_max = c->drift_max;
    return v;
}

// The local energy of every walker: the kinetic part, plus the Ewald electron-electron energy
// when the system has it.
template <typename T>
void local_energy(cq_crowd* c, const cq::CrowdView<T>& v, hipStream_t st)
{
    cq::launch_energy<T>(v, st);
    const cq_system* s = c->sys;
    if (s && s->coulomb && c->ew_phase) {
        cq::EwaldView e{};
        e.W = c->W;
        e.ne = c->ne;
        e.nmax = s->nmax;
        e.nk = s->nk;
        e.pk = (s->nk + cq::ewald_wavevectors_per_block() - 1) / cq::ewald_wavevectors_per_block();
        e.pr = 8;
        e.L = s->L;
        e.alpha = s->alpha;
        e.R = c->R;
        e.kvec = s->kvec;
        e.kfac = s->kfac;
        e.phase = c->ew_phase;
        e.part = c->ew_part;
        cq::launch_ewald(e, c->eloc, st);
    }
}

cq_status dev_alloc(cq_crowd* c, void** p, size_t bytes)
{
    if (bytes == 0) bytes = 16;
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(CQ_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed: " + hipGetErrorString(e));
    }
    c->allocs.push_back(*p);
    return CQ_OK;
}

void timed_begin(cq_crowd* c, int kind, hipStream_t st = nullptr)
{
    if (!(c->timing_mask >> kind & 1) || c->ev_used[kind] >= (size_t)kEventCap) return;
    auto& pool = c->ev[kind];
    if (c->ev_used[kind] == pool.size()) {
        hipEvent_t a, b;
        if (hipEventCreate(&a) != hipSuccess) return;
        if (hipEventCreate(&b) != hipSuccess) { (void)hipEventDestroy(a); return; }
        pool.push_back({a, b});
    }
    const hipError_t e = hipEventRecord(pool[c->ev_used[kind]].first, st ? st : c->stream);
    if (e != hipSuccess && c->enq_err == hipSuccess) c->enq_err = e;
}

void timed_end(cq_crowd* c, int kind, hipStream_t st = nullptr)
{
    if (!(c->timing_mask >> kind & 1) || c->ev_used[kind] >= (size_t)kEventCap || c->ev_used[kind] >= c->ev[kind].size())
        return;
    const hipError_t e = hipEventRecord(c->ev[kind][c->ev_used[kind]].second, st ? st : c->stream);
    if (e != hipSuccess && c->enq_err == hipSuccess) c->enq_err = e;
    c->ev_used[kind]++;
}

// Rounds a margin above the most any recent sweep needed absorb the sweep-to-sweep
// spread; when the tail kernel still had work, the plan grows by more.
constexpr int kPlanMargin = 2;

int planned_rounds(const cq_crowd* c, int spin, int rounds)
{
    const int p = c->plan_fixed > 0 ? c->plan_fixed : c->plan[spin];
    return p > 0 && p < rounds ? p : rounds;
}

// Candidates per round for the current delay rank: the requested Q (cq_crowd_set_tiles) or
// the default rule, at least min(k, N) (so N / k rounds finish a block) and at most the
// buffers' Qcap.
int min_candidates(const cq_crowd* c) { return std::min(std::max(c->K, 2), c->n); }

void apply_q(cq_crowd* c)
{
    if (c->path != CQ_PATH_BATCH) {
        c->Q = c->QR = c->K;
        return;
    }
    int q = c->q_req > 0 ? c->q_req : cq::batch_candidates(c->n, c->K);
    q = std::min(std::max(q, min_candidates(c)), c->Qcap);
    c->Q = q;
    c->QR = 2 * q;
}

void reset_plan(cq_crowd* c)
{
    c->plan[0] = c->plan[1] = -1;
    if (c->hplan) c->hplan[0] = 0;
}

// Take the latest report of the rounds each spin block needed (written by the device into
// pinned memory after the block; no synchronisation, a report a sweep or two old does as
// well).  The first report sets the plan; later ones only grow it, so that a captured sweep
// graph is rebuilt rarely.  Returns whether the plan changed.
bool update_plan(cq_crowd* c)
{
    if (!c->hplan || c->path != CQ_PATH_BATCH || c->plan_fixed > 0) return false;
    const volatile int* h = c->hplan;
    const int have = h[0];  // bit s: spin s has reported since the plan restarted
    if (!have) return false;
    const int rounds = cq::batch_rounds(c->n, c->K);
    bool changed = false;
    for (int s = 0; s < 2; ++s) {
        if (!((have >> s) & 1)) continue;
        const int used = h[1 + 2 * s], left = h[2 + 2 * s];
        int want = used + kPlanMargin;
        if (left) want = std::max(want, (c->plan[s] > 0 ? c->plan[s] : used) + 2 * kPlanMargin);
        want = std::max(1, std::min(want, rounds));
        const int p = c->plan[s] < 0 ? want : std::max(c->plan[s], want);
        if (p != c->plan[s]) {
            c->plan[s] = p;
            changed = true;
        }
    }
    return changed;
}

template <typename T>
void enqueue_sweep(cq_crowd* c)
{
    const cq::CrowdView<T> v = view<T>(c);
    const int n = c->n, K = c->K;
    if (c->path == CQ_PATH_BATCH) {
        // Rounds of both spin blocks in order.  On stream: P(r), decide(r), cols(r),
        // update(r), P(r+1), ...  On stream2, two rounds ahead: gather(r+2) as soon as
        // cols(r) is done (update(r) too when the update reads the stage ring), then
        // jd(r+2) and the row copy of round r+1 once decide(r+1) is done; P(r+2) waits
        // for them.  So the gather runs beside the whole of round r+1: P, decisions,
        // columns and update.
        //   gather(r+2)'s range, fixed by decide(r), lies in [d + Q, d + 2Q) with d the
        //   first candidate of round r+1; its ring slots (electron mod 2Q) are those of
        //   electrons decided in round r or before, whose readers (P, decide, cols, the
        //   row copy and a stage-reading update of those rounds) have finished, and are
        //   disjoint from round r+1's candidates [d, d + Q).
        //   jd(r+2) reads the positions decide(r+1) wrote and the proposals of gather(r+2).
        //   The row copy of round r+1 reads the window decide(r+2) overwrites; P(r+2)
        //   orders them.
        // A spin block starts with gather(0) and jd(0) on stream, then gather(1) on
        // stream2 (its range is set by the cursor reset).
        const int rounds = cq::batch_rounds(n, K), total = 2 * rounds;
        const bool overlap = c->stream2 != nullptr && (int)c->ev_gat.size() >= total;
        auto gather = [&](int q, hipStream_t st) {
            const int spin = q / rounds, r = q % rounds;
            timed_begin(c, CQ_KERNEL_PROPOSE, st);
            cq::launch_batch_stencils<T>(v, spin, r & 1, r == 0, st);
            timed_end(c, CQ_KERNEL_PROPOSE, st);
            timed_begin(c, CQ_KERNEL_VGL, st);
            cq::launch_batch_vgl<T>(v, spin, r & 1, overlap, st);
            timed_end(c, CQ_KERNEL_VGL, st);
        };
        auto jastrow = [&](int q, hipStream_t st) {
            timed_begin(c, CQ_KERNEL_PROPOSE, st);
            cq::launch_batch_jd<T>(v, q / rounds, st);
            timed_end(c, CQ_KERNEL_PROPOSE, st);
        };
        hipStream_t s1 = c->stream, s2 = c->stream2;
        auto keep = [&](hipError_t e) {
            if (e != hipSuccess && c->enq_err == hipSuccess) c->enq_err = e;
        };
        // the vector update reads the accepted rows from the stage ring; the matrix-core
        // update reads them packed by the column kernel
        const bool update_reads_stage = v.ub == nullptr;
        for (int spin = 0; spin < 2; ++spin) {
            // R planned rounds (the rest of the block's N / k would find every walker done,
            // at the usual acceptance); the tail kernel finishes any walker left over
            const int R = planned_rounds(c, spin, rounds);
            const int q0 = spin * rounds;
            gather(q0, s1);
            jastrow(q0, s1);
            if (overlap && R > 1) {
                keep(hipEventRecord(c->ev_fork[q0], s1));
                keep(hipStreamWaitEvent(s2, c->ev_fork[q0], 0));
                gather(q0 + 1, s2);
            }
            for (int r = 0; r < R; ++r) {
                const int q = q0 + r;
                const bool next = r + 1 < R, ahead = overlap && r + 2 < R;
                if (overlap && r > 0) keep(hipStreamWaitEvent(s1, c->ev_gat[q], 0));
                timed_begin(c, CQ_KERNEL_RESOLVE);
                cq::launch_batch_pmat<T>(v, spin, s1);
                cq::launch_batch_decide<T>(v, spin, r & 1, r, s1);
                if (overlap && next) keep(hipEventRecord(c->ev_dec[q], s1));
                cq::launch_batch_cols<T>(v, spin, s1);
                timed_end(c, CQ_KERNEL_RESOLVE);
                if (ahead && !update_reads_stage) keep(hipEventRecord(c->ev_cols[q], s1));
                if (overlap && next) {
                    keep(hipStreamWaitEvent(s2, c->ev_dec[q], 0));
                    jastrow(q + 1, s2);
                    cq::launch_batch_rows<T>(v, spin, s2);
                    keep(hipEventRecord(c->ev_gat[q + 1], s2));
                } else {
                    cq::launch_batch_rows<T>(v, spin, s1);
                }
                timed_begin(c, CQ_KERNEL_UPDATE);
                cq::launch_flush<T>(v, spin, s1, true);
                timed_end(c, CQ_KERNEL_UPDATE);
                if (ahead) {
                    if (update_reads_stage) keep(hipEventRecord(c->ev_cols[q], s1));
                    keep(hipStreamWaitEvent(s2, c->ev_cols[q], 0));
                    gather(q + 2, s2);
                }
                if (!overlap && next) {
                    gather(q + 1, s1);
                    jastrow(q + 1, s1);
                }
            }
            timed_begin(c, CQ_KERNEL_RESOLVE);
            cq::launch_leftover<T>(v, spin, c->hplan, R < rounds, s1);
            timed_end(c, CQ_KERNEL_RESOLVE);
        }
        timed_begin(c, CQ_KERNEL_ENERGY);
        local_energy<T>(c, v, c->stream);
        timed_end(c, CQ_KERNEL_ENERGY);
        cq::launch_sweep_end(c->prm, c->stream);
        return;
    }
    if (c->path == CQ_PATH_SWEEP) {
        timed_begin(c, CQ_KERNEL_VGL);
        cq::launch_sweep<T>(v, c->stream);
        timed_end(c, CQ_KERNEL_VGL);
        timed_begin(c, CQ_KERNEL_ENERGY);
        local_energy<T>(c, v, c->stream);
        timed_end(c, CQ_KERNEL_ENERGY);
        cq::launch_sweep_end(c->prm, c->stream);
        return;
    }
    if (c->path == CQ_PATH_WINDOW) {
        for (int spin = 0; spin < 2; ++spin)
            for (int a0 = 0; a0 < n; a0 += K) {
                timed_begin(c, CQ_KERNEL_VGL);
                cq::launch_window<T>(v, spin * n + a0, std::min(K, n - a0), c->stream);
                timed_end(c, CQ_KERNEL_VGL);
                timed_begin(c, CQ_KERNEL_UPDATE);
                cq::launch_flush<T>(v, spin, c->stream);
                timed_end(c, CQ_KERNEL_UPDATE);
            }
        timed_begin(c, CQ_KERNEL_ENERGY);
        local_energy<T>(c, v, c->stream);
        timed_end(c, CQ_KERNEL_ENERGY);
        cq::launch_sweep_end(c->prm, c->stream);
        return;
    }
    for (int e = 0; e < c->ne; ++e) {
        const int spin = e / n, a = e % n;
        const int reset = (a % K) == 0;
        timed_begin(c, CQ_KERNEL_VGL);
        cq::launch_move<T>(v, e, reset ? -1 : e - 1, reset, c->stream);
        timed_end(c, CQ_KERNEL_VGL);
        if ((a + 1) % K == 0 || a == n - 1) {
            // end of the window: decide its last move, then apply the window
            timed_begin(c, CQ_KERNEL_RESOLVE);
            cq::launch_move<T>(v, -1, e, 0, c->stream);
            timed_end(c, CQ_KERNEL_RESOLVE);
            timed_begin(c, CQ_KERNEL_UPDATE);
            cq::launch_flush<T>(v, spin, c->stream);
            timed_end(c, CQ_KERNEL_UPDATE);
        }
    }
    timed_begin(c, CQ_KERNEL_ENERGY);
    local_energy<T>(c, v, c->stream);
    timed_end(c, CQ_KERNEL_ENERGY);
    cq::launch_sweep_end(c->prm, c->stream);
}

template <typename T>
void enqueue_inverse(cq_crowd* c)
{
    timed_begin(c, CQ_KERNEL_INVERSE);
    cq::launch_inverse<T>(view<T>(c), c->inv, c->stream);
    timed_end(c, CQ_KERNEL_INVERSE);
}

void sweep(cq_crowd* c)
{
    if (c->prec == CQ_FP64)
        enqueue_sweep<double>(c);
    else
        enqueue_sweep<float>(c);
}

void inverse(cq_crowd* c)
{
    if (c->prec == CQ_FP64)
        enqueue_inverse<double>(c);
    else
        enqueue_inverse<float>(c);
}

// The first error of the launches and event calls enqueued since the last check.
cq_status enqueue_status(cq_crowd* c, const char* where)
{
    hipError_t e = c->enq_err;
    c->enq_err = hipSuccess;
    const hipError_t l = hipGetLastError();
    if (e == hipSuccess) e = l;
    if (e != hipSuccess) return fail(CQ_EDEVICE, std::string(where) + ": " + hipGetErrorString(e));
    return CQ_OK;
}

cq_status push_params(cq_crowd* c)
{
    HIP_TRY(hipStreamSynchronize(c->stream));
    HIP_TRY(hipMemcpy(c->prm, &c->hp, sizeof(cq::Params), hipMemcpyHostToDevice));
    return CQ_OK;
}

void drop_graph(cq_crowd* c)
{
    if (c->gexec) {
        (void)hipGraphExecDestroy(c->gexec);
        c->gexec = nullptr;
    }
}

cq_status build_graph(cq_crowd* c)
{
    hipGraph_t g = nullptr;
    HIP_TRY(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    sweep(c);
    const hipError_t eq = c->enq_err;
    c->enq_err = hipSuccess;
    hipError_t e = hipStreamEndCapture(c->stream, &g);
    if (e == hipSuccess && eq != hipSuccess) {
        (void)hipGraphDestroy(g);
        return fail(CQ_EDEVICE, std::string("sweep capture: ") + hipGetErrorString(eq));
    }
    if (e != hipSuccess) return fail(CQ_EDEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    e = hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        c->gexec = nullptr;
        return fail(CQ_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    }
    return CQ_OK;
}

cq_status check_singular(cq_crowd* c, const char* where)
{
    std::vector<int> st(c->W);
    HIP_TRY(hipStreamSynchronize(c->stream));
    HIP_TRY(hipMemcpy(st.data(), c->status, sizeof(int) * c->W, hipMemcpyDeviceToHost));
    for (int w = 0; w < c->W; ++w) {
        if (st[w] & 2)
            return fail(CQ_ESTATE, std::string(where) + ": update-window bookkeeping out of range for walker " +
                                       std::to_string(w) + " (internal error)");
        if (st[w] & 1)
            return fail(CQ_ESINGULAR, std::string(where) + ": Slater matrix of walker " + std::to_string(w) +
                                          " is singular or not finite");
    }
    return CQ_OK;
}

template <typename T>
cq_status setup_state(cq_crowd* c)
{
    const cq::CrowdView<T> v = view<T>(c);
    HIP_TRY(hipMemsetAsync(c->logdet, 0, sizeof(double) * 2 * c->W, c->stream));
    HIP_TRY(hipMemsetAsync(c->sign, 0, sizeof(int) * 2 * c->W, c->stream));
    HIP_TRY(hipMemsetAsync(c->nacc, 0, sizeof(long long) * c->W, c->stream));
    HIP_TRY(hipMemsetAsync(c->nprop, 0, sizeof(long long) * c->W, c->stream));
    HIP_TRY(hipMemsetAsync(c->cnt, 0, sizeof(int) * 3 * c->Wcap, c->stream));
    HIP_TRY(hipMemsetAsync(c->welec, 0, sizeof(int) * c->Wcap * c->K, c->stream));
    HIP_TRY(hipMemsetAsync(c->wslot, 0, sizeof(int) * c->Wcap * c->K, c->stream));
    // window slots are read (masked) before they are first written: start them at 0; every
    // walker slot up to the capacity, since DMC branching fills slots past the initial count
    const size_t es = c->prec == CQ_FP64 ? 8 : 4;
    HIP_TRY(hipMemsetAsync(c->stage, 0, es * c->Wcap * c->QR * 5 * c->n, c->stream));
    HIP_TRY(hipMemsetAsync(c->cur, 0, sizeof(int) * 3 * c->Wcap, c->stream));
    HIP_TRY(hipMemsetAsync(c->look, 0, sizeof(int) * 4 * c->Wcap, c->stream));
    HIP_TRY(hipMemsetAsync(c->Cbuf, 0, es * c->Wcap * c->K * c->n, c->stream));
    HIP_TRY(hipMemsetAsync(c->status, 0, sizeof(int) * c->Wcap, c->stream));
    cq::launch_setup_vgl<T>(v, c->stream);
    HIP_TRY(hipGetLastError());
    enqueue_inverse<T>(c);
    HIP_TRY(hipGetLastError());
    // the set-up inversion is no recompute: the drift record starts after it
    HIP_TRY(hipMemsetAsync(c->drift_max, 0, sizeof(unsigned long long), c->stream));
    c->n_recomputes = 0;
    local_energy<T>(c, v, c->stream);
    HIP_TRY(hipGetLastError());
    return check_singular(c, "set_positions");
}

template <typename T>
cq::WalkerArrays<T> walker_arrays(cq_crowd* c, bool alt)
{
    if (alt)
        return {c->alt.R, (T*)c->alt.M, (T*)c->alt.VGL, c->alt.logdet, c->alt.sign, c->alt.eloc, c->alt.eold,
                c->alt.uid, c->alt.nacc, c->alt.nprop};
    return {c->R, (T*)c->M, (T*)c->VGL, c->logdet, c->sign, c->eloc, c->eold, c->uid, c->nacc, c->nprop};
}

cq_status ensure_dmc(cq_crowd* c, int n_gen)
{
    if (!c->have_alt) {
        const size_t Wc = (size_t)c->Wcap, n = c->n, ne = c->ne;
        const size_t es = c->prec == CQ_FP64 ? 8 : 4;
        struct {
            void** p;
            size_t bytes;
        } plan[] = {
            {(void**)&c->alt.R, sizeof(double) * Wc * ne * 3},
            {&c->alt.M, es * Wc * 2 * n * n},
            {&c->alt.VGL, es * Wc * 2 * n * 5 * n},
            {(void**)&c->alt.logdet, sizeof(double) * Wc * 2},
            {(void**)&c->alt.sign, sizeof(int) * Wc * 2},
            {(void**)&c->alt.eloc, sizeof(double) * Wc},
            {(void**)&c->alt.eold, sizeof(double) * Wc},
            {(void**)&c->alt.uid, sizeof(uint32_t) * Wc},
            {(void**)&c->alt.nacc, sizeof(long long) * Wc},
            {(void**)&c->alt.nprop, sizeof(long long) * Wc},
            {(void**)&c->dmc_state, sizeof(cq::DmcState)},
            {(void**)&c->dmc_wt, sizeof(double) * Wc},
            {(void**)&c->dmc_mult, sizeof(int) * Wc},
            {(void**)&c->dmc_off, sizeof(int) * Wc},
        };
        for (auto& e : plan) {
            cq_status st = dev_alloc(c, e.p, e.bytes);
            if (st != CQ_OK) return st;
        }
        cq::DmcState st0{};
        HIP_TRY(hipMemcpy(c->dmc_state, &st0, sizeof(st0), hipMemcpyHostToDevice));
        c->have_alt = true;
    }
    if (n_gen > c->dmc_hist_cap) {
        if (c->dmc_hist) (void)hipFree(c->dmc_hist);
        c->dmc_hist = nullptr;
        c->dmc_hist_cap = 0;
        HIP_TRY(hipMalloc(&c->dmc_hist, sizeof(double) * 4 * (size_t)n_gen));
        c->dmc_hist_cap = n_gen;
    }
    return CQ_OK;
}

template <typename T>
void dmc_moves(cq_crowd* c)
{
    cq::CrowdView<T> v = view<T>(c);
    v.ct = nullptr;  // the per-move kernel leaves the window's columns in row layout
    v.ub = nullptr;
    const int n = c->n, K = c->K;
    for (int spin = 0; spin < 2; ++spin)
        for (int a0 = 0; a0 < n; a0 += K) {
            timed_begin(c, CQ_KERNEL_VGL);
            cq::launch_window_dmc<T>(v, spin * n + a0, std::min(K, n - a0), c->stream);
            timed_end(c, CQ_KERNEL_VGL);
            timed_begin(c, CQ_KERNEL_UPDATE);
            cq::launch_flush<T>(v, spin, c->stream, false);
            timed_end(c, CQ_KERNEL_UPDATE);
        }
}

// The moves of one generation for the walkers of every system of a group: per spin block and
// window step j, ONE launch of the walker-resident move kernel over the walkers of all systems
// that have a window j (largest system first) and ONE update launch over their strips.
template <typename T>
cq_status group_moves(cq_crowd* g)
{
    const int S = (int)g->subs.size();
    std::vector<cq::CrowdView<T>> hv(S);
    int max_n = 0, max_win = 0;
    bool mfma = sizeof(T) == 4;
    for (int s = 0; s < S; ++s) {
        cq_crowd* c = g->subs[s];
        hv[s] = view<T>(c);
        hv[s].ct = nullptr;
        hv[s].ub = nullptr;
        max_n = std::max(max_n, c->n);
        max_win = std::max(max_win, (c->n + c->K - 1) / c->K);
        mfma = mfma && cq::flush_mfma_fits(c->n);
    }
    // systems in order of decreasing N: the longest windows are handed out first
    std::vector<int> order(S);
    for (int s = 0; s < S; ++s) order[s] = s;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return g->subs[a]->n > g->subs[b]->n; });
    const int rows = mfma ? 32 : 16;  // rows per update workgroup
    g->hwalk.clear();
    g->hstrip.clear();
    std::vector<size_t> woff(max_win + 1), soff(max_win + 1);
    for (int j = 0; j < max_win; ++j) {
        woff[j] = g->hwalk.size();
        soff[j] = g->hstrip.size();
        for (int s : order) {
            cq_crowd* c = g->subs[s];
            if (j * c->K >= c->n) continue;
            const int strips = (c->n + rows - 1) / rows;
            for (int w = 0; w < c->W; ++w) g->hwalk.push_back(make_int2(s, w));
            for (int w = 0; w < c->W; ++w)
                for (int t = 0; t < strips; ++t) g->hstrip.push_back(make_int4(s, w, t, 0));
        }
    }
    woff[max_win] = g->hwalk.size();
    soff[max_win] = g->hstrip.size();
    const size_t vb = sizeof(cq::CrowdView<T>) * S;
    if (!g->gviews) {
        if (hipMalloc(&g->gviews, sizeof(cq::CrowdView<double>) * S + sizeof(cq::CrowdView<float>) * S) !=
            hipSuccess) {
            (void)hipGetLastError();
            return fail(CQ_ENOMEM, "group views");
        }
    }
    if (g->hwalk.size() > g->gwalk_cap) {
        if (g->gwalk) HIP_TRY(hipFree(g->gwalk));
        g->gwalk = nullptr;
        g->gwalk_cap = 0;
        const size_t cap = g->hwalk.size() * 2;
        if (hipMalloc((void**)&g->gwalk, sizeof(int2) * cap) != hipSuccess) {
            (void)hipGetLastError();
            return fail(CQ_ENOMEM, "group walker items");
        }
        g->gwalk_cap = cap;
    }
    if (g->hstrip.size() > g->gstrip_cap) {
        if (g->gstrip) HIP_TRY(hipFree(g->gstrip));
        g->gstrip = nullptr;
        g->gstrip_cap = 0;
        const size_t cap = g->hstrip.size() * 2;
        if (hipMalloc((void**)&g->gstrip, sizeof(int4) * cap) != hipSuccess) {
            (void)hipGetLastError();
            return fail(CQ_ENOMEM, "group strip items");
        }
        g->gstrip_cap = cap;
    }
    g->hviews.assign((const unsigned char*)hv.data(), (const unsigned char*)hv.data() + vb);
    HIP_TRY(hipMemcpyAsync(g->gviews, g->hviews.data(), vb, hipMemcpyHostToDevice, g->stream));
    HIP_TRY(hipMemcpyAsync(g->gwalk, g->hwalk.data(), sizeof(int2) * g->hwalk.size(), hipMemcpyHostToDevice,
                           g->stream));
    HIP_TRY(hipMemcpyAsync(g->gstrip, g->hstrip.data(), sizeof(int4) * g->hstrip.size(), hipMemcpyHostToDevice,
                           g->stream));
    const cq::CrowdView<T>* dv = (const cq::CrowdView<T>*)g->gviews;
    const int cus = g->n_cu > 0 ? g->n_cu : 256;
    for (int spin = 0; spin < 2; ++spin)
        for (int j = 0; j < max_win; ++j) {
            const int nw = (int)(woff[j + 1] - woff[j]), ns = (int)(soff[j + 1] - soff[j]);
            timed_begin(g, CQ_KERNEL_VGL);
            cq::launch_window_dmc_multi<T>(dv, g->gwalk + woff[j], nw, max_n, spin, j, std::min(nw, 4 * cus),
                                           g->stream);
            timed_end(g, CQ_KERNEL_VGL);
            timed_begin(g, CQ_KERNEL_UPDATE);
            if constexpr (sizeof(T) == 4) {
                if (mfma)
                    cq::launch_flush_mfma_multi((const cq::CrowdView<float>*)dv, g->gwalk + woff[j], nw,
                                                g->gstrip + soff[j], ns, spin, 2 * cus, g->stream);
                else
                    cq::launch_flush_vec_multi<T>(dv, g->gstrip + soff[j], ns, max_n, spin, 4 * cus, g->stream);
            } else {
                cq::launch_flush_vec_multi<T>(dv, g->gstrip + soff[j], ns, max_n, spin, 4 * cus, g->stream);
            }
            timed_end(g, CQ_KERNEL_UPDATE);
        }
    return CQ_OK;
}

// After the moves of a generation: the periodic FP64 recompute, the local energy and the
// branching of one system's population.
template <typename T>
void dmc_post(cq_crowd* c, int gen, int n_target, double tau, bool recompute)
{
    cq::CrowdView<T> v = view<T>(c);
    const int n = c->n;
    // the periodic FP64 recompute, before the energy and the branching read the inverses
    if (recompute) enqueue_inverse<T>(c);
    timed_begin(c, CQ_KERNEL_ENERGY);
    local_energy<T>(c, v, c->stream);
    timed_end(c, CQ_KERNEL_ENERGY);
    cq::DmcView d{};
    d.state = c->dmc_state;
    d.wt = c->dmc_wt;
    d.mult = c->dmc_mult;
    d.off = c->dmc_off;
    d.history = c->dmc_hist;
    d.forced_mult = c->mult_cap > 0 ? c->forced_mult : nullptr;
    d.pop = c->W;
    d.cap = c->Wcap;
    d.n_target = n_target;
    const size_t nV = 2 * (size_t)n * 5 * n;
    d.chunks = (int)std::min<size_t>(256, std::max<size_t>(1, nV / (256 * 256)));
    d.ecut = 0.2 * std::sqrt((double)c->ne / tau);
    d.seed = c->seed;
    cq::launch_dmc_branch<T>(d, walker_arrays<T>(c, false), walker_arrays<T>(c, true), n, c->ne, c->prm, gen,
                             c->stream);
    cq::launch_sweep_end(c->prm, c->stream);
}

void swap_walker_sets(cq_crowd* c)
{
    std::swap(c->R, c->alt.R);
    std::swap(c->M, c->alt.M);
    std::swap(c->VGL, c->alt.VGL);
    std::swap(c->logdet, c->alt.logdet);
    std::swap(c->sign, c->alt.sign);
    std::swap(c->eloc, c->alt.eloc);
    std::swap(c->eold, c->alt.eold);
    std::swap(c->uid, c->alt.uid);
    std::swap(c->nacc, c->alt.nacc);
    std::swap(c->nprop, c->alt.nprop);
}

}  // namespace

extern "C" {

const char* cq_last_error(void) { return g_err.c_str(); }

cq_status cq_system_create(int n_up, int n_dn, double box_L, cq_system** out)
{
    if (!out) return fail(CQ_EINVAL, "out is NULL");
    *out = nullptr;
    if (n_up < 1 || n_dn != n_up) return fail(CQ_EINVAL, "need n_up == n_dn >= 1");
    if (n_up % 4 != 0) return fail(CQ_EINVAL, "electrons per spin must be a multiple of 4");
    if (n_up > 2048) return fail(CQ_EINVAL, "at most 2048 electrons per spin");
    if (!(box_L > 0.0) || !std::isfinite(box_L)) return fail(CQ_EINVAL, "box_L must be positive and finite");
    cq_system* s = new (std::nothrow) cq_system();
    if (!s) return fail(CQ_ENOMEM, "host allocation failed");
    s->n_up = n_up;
    s->n_dn = n_dn;
    s->L = box_L;
    *out = s;
    return CQ_OK;
}

static cq_status check_table_shape(cq_system* s, int elem_bytes, int gx, int gy, int gz, int n_orb)
{
    if (!s) return fail(CQ_EINVAL, "system is NULL");
    if (elem_bytes != 4 && elem_bytes != 8) return fail(CQ_EINVAL, "elem_bytes must be 4 or 8");
    if (gx != gy || gy != gz || gx < 4) return fail(CQ_EINVAL, "grid must be cubic with at least 4 points");
    if (n_orb != s->n_up) return fail(CQ_EINVAL, "n_orb must equal the electrons per spin");
    if (s->G != 0 && s->G != gx) return fail(CQ_EINVAL, "grid differs from the table already loaded");
    return CQ_OK;
}

cq_status cq_system_load_bspline(cq_system* s, const void* coefs, int elem_bytes, int gx, int gy, int gz, int n_orb,
                                 int coefs_on_device)
{
    cq_status st = check_table_shape(s, elem_bytes, gx, gy, gz, n_orb);
    if (st != CQ_OK) return st;
    if (!coefs) return fail(CQ_EINVAL, "coefs is NULL");
    const int slot = elem_bytes == 8 ? 1 : 0;
    const size_t bytes = (size_t)gx * gx * gx * n_orb * elem_bytes;
    if (s->owned[slot]) HIP_TRY(hipFree(s->table[slot]));
    s->table[slot] = nullptr;
    s->owned[slot] = false;
    if (coefs_on_device) {
        s->table[slot] = const_cast<void*>(coefs);
    } else {
        void* p = nullptr;
        hipError_t e = hipMalloc(&p, bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return fail(CQ_ENOMEM, "hipMalloc of the coefficient table failed");
        }
        e = hipMemcpy(p, coefs, bytes, hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            (void)hipFree(p);
            return fail(CQ_EDEVICE, std::string("hipMemcpy table: ") + hipGetErrorString(e));
        }
        s->table[slot] = p;
        s->owned[slot] = true;
    }
    s->G = gx;
    s->n_orb = n_orb;
    return CQ_OK;
}

cq_status cq_system_fill_bspline_philox(cq_system* s, uint64_t seed, int elem_bytes, int grid, int n_orb)
{
    cq_status st = check_table_shape(s, elem_bytes, grid, grid, grid, n_orb);
    if (st != CQ_OK) return st;
    const int slot = elem_bytes == 8 ? 1 : 0;
    const size_t count = (size_t)grid * grid * grid * n_orb;
    if (s->owned[slot]) HIP_TRY(hipFree(s->table[slot]));
    s->table[slot] = nullptr;
    s->owned[slot] = false;
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, count * elem_bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(CQ_ENOMEM, "hipMalloc of the coefficient table failed");
    }
    if (elem_bytes == 4)
        cq::launch_fill_philox<float>((float*)p, seed, count, nullptr);
    else
        cq::launch_fill_philox<double>((double*)p, seed, count, nullptr);
    e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipGetLastError();
    if (e != hipSuccess) {
        (void)hipFree(p);
        return fail(CQ_EDEVICE, std::string("coefficient fill: ") + hipGetErrorString(e));
    }
    s->table[slot] = p;
    s->owned[slot] = true;
    s->G = grid;
    s->n_orb = n_orb;
    return CQ_OK;
}

cq_status cq_system_load_pade_j2(cq_system* s, double a_par, double a_anti, double b)
{
    if (!s) return fail(CQ_EINVAL, "system is NULL");
    if (!std::isfinite(a_par) || !std::isfinite(a_anti) || !(b >= 0.0) || !std::isfinite(b))
        return fail(CQ_EINVAL, "Jastrow parameters must be finite, b >= 0");
    s->use_j2 = 1;
    s->a_par = a_par;
    s->a_anti = a_anti;
    s->b = b;
    return CQ_OK;
}

cq_status cq_system_load_pade_j1(cq_system* s, const double* centres, int n_centres, double a, double b)
{
    if (!s) return fail(CQ_EINVAL, "system is NULL");
    if (n_centres < 0 || n_centres > cq::kMaxIons)
        return fail(CQ_EINVAL, "n_centres must be 0.." + std::to_string(cq::kMaxIons));
    if (n_centres > 0 && !centres) return fail(CQ_EINVAL, "centres is NULL");
    if (!std::isfinite(a) || !(b >= 0.0) || !std::isfinite(b))
        return fail(CQ_EINVAL, "Jastrow parameters must be finite, b >= 0");
    for (int i = 0; i < 3 * n_centres; ++i)
        if (!std::isfinite(centres[i])) return fail(CQ_EINVAL, "centre coordinates must be finite");
    if (n_centres == 0) {
        s->n_ions = 0;
        return CQ_OK;
    }
    double* d = nullptr;
    HIP_TRY(hipMalloc(&d, sizeof(double) * 3 * n_centres));
    const hipError_t e = hipMemcpy(d, centres, sizeof(double) * 3 * n_centres, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(d);
        return fail(CQ_EDEVICE, std::string("hipMemcpy: ") + hipGetErrorString(e));
    }
    if (s->ions) (void)hipFree(s->ions);
    s->ions = d;
    s->n_ions = n_centres;
    s->j1_a = a;
    s->j1_b = b;
    return CQ_OK;
}

cq_status cq_system_set_coulomb(cq_system* s, int enable)
{
    if (!s) return fail(CQ_EINVAL, "system is NULL");
    if (!enable) {
        s->coulomb = 0;
        return CQ_OK;
    }
    if (!s->kvec) {
        // alpha L = 10.1: beyond the nearest image every pair term is below erfc(5.05) = 8e-13 of it;
        // wavevectors with n^2 <= 18^2, where exp(-k^2 / 4 alpha^2) has fallen to 1e-13
        const int nmax = 18;
        const double L = s->L, alpha = 10.1 / L;
        std::vector<int4> kv;
        std::vector<double> kf;
        for (int a = 0; a <= nmax; ++a)
            for (int b = -nmax; b <= nmax; ++b)
                for (int c = -nmax; c <= nmax; ++c) {
                    const bool half = a > 0 || (a == 0 && (b > 0 || (b == 0 && c > 0)));
                    if (!half || a * a + b * b + c * c > nmax * nmax) continue;
                    const double k2 = (4.0 * M_PI * M_PI / (L * L)) * (double)(a * a + b * b + c * c);
                    kv.push_back(make_int4(a, b, c, 0));
                    kf.push_back(std::exp(-k2 / (4.0 * alpha * alpha)) / k2);
                }
        if (hipMalloc((void**)&s->kvec, sizeof(int4) * kv.size()) != hipSuccess ||
            hipMalloc((void**)&s->kfac, sizeof(double) * kf.size()) != hipSuccess) {
            (void)hipGetLastError();
            return fail(CQ_ENOMEM, "Ewald wavevectors");
        }
        HIP_TRY(hipMemcpy(s->kvec, kv.data(), sizeof(int4) * kv.size(), hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(s->kfac, kf.data(), sizeof(double) * kf.size(), hipMemcpyHostToDevice));
        s->nmax = nmax;
        s->nk = (int)kv.size();
        s->alpha = alpha;
    }
    s->coulomb = 1;
    return CQ_OK;
}

void cq_system_destroy(cq_system* s)
{
    if (!s) return;
    if (s->kvec) (void)hipFree(s->kvec);
    if (s->kfac) (void)hipFree(s->kfac);
    if (s->ions) (void)hipFree(s->ions);
    for (int i = 0; i < 2; ++i)
        if (s->owned[i]) (void)hipFree(s->table[i]);
    delete s;
}

void cq_crowd_destroy(cq_crowd* c)
{
    if (!c) return;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    for (cq_crowd* sub : c->subs) cq_crowd_destroy(sub);
    if (c->gviews) (void)hipFree(c->gviews);
    if (c->gwalk) (void)hipFree(c->gwalk);
    if (c->gstrip) (void)hipFree(c->gstrip);
    drop_graph(c);
    for (int k = 0; k < CQ_KERNEL_COUNT; ++k)
        for (auto& p : c->ev[k]) {
            (void)hipEventDestroy(p.first);
            (void)hipEventDestroy(p.second);
        }
    for (void* p : c->allocs) (void)hipFree(p);
    if (c->dmc_hist) (void)hipFree(c->dmc_hist);
    if (c->rec_rho) (void)hipFree(c->rec_rho);
    if (c->rec_dlnj) (void)hipFree(c->rec_dlnj);
    if (c->rec_prob) (void)hipFree(c->rec_prob);
    if (c->rec_acc) (void)hipFree(c->rec_acc);
    if (c->rec_rnew) (void)hipFree(c->rec_rnew);
    if (c->voff) (void)hipFree(c->voff);
    if (c->vout) (void)hipFree(c->vout);
    if (c->forced) (void)hipFree(c->forced);
    if (c->forced_mult) (void)hipFree(c->forced_mult);
    if (c->hplan) (void)hipHostFree(c->hplan);
    for (auto* evs : {&c->ev_fork, &c->ev_dec, &c->ev_cols, &c->ev_gat})
        for (hipEvent_t e : *evs) (void)hipEventDestroy(e);
    if (c->stream2) (void)hipStreamDestroy(c->stream2);
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

cq_status cq_crowd_create(const cq_system* const* systems, const int* walkers_per_system, int n_systems,
                          const cq_crowd_desc* desc, cq_crowd** out)
{
    if (!out) return fail(CQ_EINVAL, "out is NULL");
    *out = nullptr;
    if (!systems || !walkers_per_system || !desc) return fail(CQ_EINVAL, "NULL argument");
    if (n_systems < 1) return fail(CQ_EINVAL, "n_systems must be >= 1");
    if (n_systems > 1) {
        // one crowd per system on a shared stream; walker uids continue from system to system
        int total = 0;
        if (desc->precision != CQ_FP64 && desc->precision != CQ_MIXED) return fail(CQ_EINVAL, "unknown precision");
        for (int k = 0; k < n_systems; ++k) {
            if (!systems[k]) return fail(CQ_EINVAL, "system is NULL");
            if (walkers_per_system[k] < 1) return fail(CQ_EINVAL, "need at least one walker per system");
            if (!systems[k]->table[desc->precision == CQ_FP64 ? 1 : 0])
                return fail(CQ_EINVAL, "system " + std::to_string(k) +
                                           (desc->precision == CQ_FP64 ? " has no FP64 table" : " has no FP32 table"));
            total += walkers_per_system[k];
        }
        if (desc->max_walkers < 0) return fail(CQ_EINVAL, "max_walkers must be >= 0");
        cq_crowd* g = new (std::nothrow) cq_crowd();
        if (!g) return fail(CQ_ENOMEM, "host allocation failed");
        g->W = total;
        g->prec = desc->precision;
        if (desc->hip_stream) {
            g->stream = (hipStream_t)desc->hip_stream;
        } else {
            if (hipStreamCreateWithFlags(&g->stream, hipStreamNonBlocking) != hipSuccess) {
                delete g;
                return fail(CQ_EDEVICE, "hipStreamCreate failed");
            }
            g->own_stream = true;
        }
        int dev = 0;
        if (hipGetDevice(&dev) == hipSuccess)
            (void)hipDeviceGetAttribute(&g->n_cu, hipDeviceAttributeMultiprocessorCount, dev);
        uint32_t uid = desc->first_uid;
        for (int k = 0; k < n_systems; ++k) {
            cq_crowd_desc d = *desc;
            d.hip_stream = g->stream;
            d.first_uid = uid;
            if (d.delay_rank > systems[k]->n_up) d.delay_rank = systems[k]->n_up;
            // the walker capacity is shared out in proportion to the starting walkers
            d.max_walkers = desc->max_walkers > 0
                                ? (int)(((int64_t)desc->max_walkers * walkers_per_system[k] + total - 1) / total)
                                : 0;
            cq_crowd* sub = nullptr;
            cq_status st = cq_crowd_create(&systems[k], &walkers_per_system[k], 1, &d, &sub);
            if (st != CQ_OK) {
                cq_crowd_destroy(g);
                return st;
            }
            g->subs.push_back(sub);
            uid += (uint32_t)std::max(walkers_per_system[k], d.max_walkers);
        }
        g->n = g->subs[0]->n;
        g->ne = g->subs[0]->ne;
        g->K = g->subs[0]->K;
        *out = g;
        return CQ_OK;
    }
    const cq_system* s = systems[0];
    if (!s) return fail(CQ_EINVAL, "system is NULL");
    const int W = walkers_per_system[0];
    if (W < 1) return fail(CQ_EINVAL, "need at least one walker");
    if (desc->precision != CQ_FP64 && desc->precision != CQ_MIXED) return fail(CQ_EINVAL, "unknown precision");
    if (!s->table[desc->precision == CQ_FP64 ? 1 : 0])
        return fail(CQ_EINVAL, desc->precision == CQ_FP64 ? "system has no FP64 table" : "system has no FP32 table");
    int K = desc->delay_rank == 0 ? std::min(32, s->n_up) : desc->delay_rank;
    if (K < 1 || K > cq::kMaxDelay) return fail(CQ_EINVAL, "delay_rank must be 0..32");
    if (desc->recompute_every < 0) return fail(CQ_EINVAL, "recompute_every must be >= 0");
    if (desc->kernel_path < CQ_PATH_AUTO || desc->kernel_path > CQ_PATH_SWEEP)
        return fail(CQ_EINVAL, "unknown kernel_path");
    // the whole-sweep path: N <= 64 (both inverses in LDS), N % 4 == 0, delay rank 1;
    // the automatic choice for such systems unless a delay rank above 1 is asked for
    const bool sweep_fits = s->n_up <= cq::kSweepMaxN && s->n_up % 4 == 0;
    const bool sweep_k = desc->delay_rank == 0 || desc->delay_rank == 1;
    if (desc->kernel_path == CQ_PATH_SWEEP && !(sweep_fits && sweep_k))
        return fail(CQ_EINVAL, "the whole-sweep path needs N <= 64, N a multiple of 4 and delay rank 0 or 1");
    const int path = desc->kernel_path != CQ_PATH_AUTO ? desc->kernel_path
                                                        : (sweep_fits && sweep_k ? CQ_PATH_SWEEP : CQ_PATH_BATCH);
    if (path == CQ_PATH_SWEEP) K = 1;

    if (desc->max_walkers < 0) return fail(CQ_EINVAL, "max_walkers must be >= 0");
    if (desc->streams < 0 || desc->streams > 2) return fail(CQ_EINVAL, "streams must be 0, 1 or 2");
    cq_crowd* c = new (std::nothrow) cq_crowd();
    if (!c) return fail(CQ_ENOMEM, "host allocation failed");
    c->sys = s;
    c->W = W;
    c->Wcap = std::max(W, desc->max_walkers);
    c->n = s->n_up;
    c->ne = 2 * s->n_up;
    c->K = K;
    c->Kcap = K;
    c->autotune = desc->delay_rank == 0 && path != CQ_PATH_SWEEP;
    c->prec = desc->precision;
    c->recompute_every = desc->recompute_every;
    c->use_graph = desc->use_graph;
    c->path = path;
    c->Q = c->path == CQ_PATH_BATCH ? cq::batch_candidates(c->n, K) : K;
    c->QR = c->path == CQ_PATH_BATCH ? 2 * c->Q : c->Q;
    c->Qcap = c->Q;  // the candidate buffers below are sized for it
    c->seed = desc->seed;
    c->first_uid = desc->first_uid;
    if (desc->hip_stream) {
        c->stream = (hipStream_t)desc->hip_stream;
    } else {
        if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
            delete c;
            return fail(CQ_EDEVICE, "hipStreamCreate failed");
        }
        c->own_stream = true;
    }
    if (c->path == CQ_PATH_BATCH && desc->streams != 1) {
        // default priority, like the crowd's own stream
        if (hipStreamCreateWithFlags(&c->stream2, hipStreamNonBlocking) == hipSuccess) {
            const int total = 2 * cq::batch_rounds(c->n, 1) + 2;  // enough for any delay rank
            bool ok = true;
            for (auto* evs : {&c->ev_fork, &c->ev_dec, &c->ev_cols, &c->ev_gat})
                for (int i = 0; ok && i < total; ++i) {
                    hipEvent_t e;
                    ok = hipEventCreateWithFlags(&e, hipEventDisableTiming) == hipSuccess;
                    if (ok) evs->push_back(e);
                }
            if (!ok) (void)hipGetLastError();
        } else {
            (void)hipGetLastError();
            c->stream2 = nullptr;
        }
    }
    if (c->path == CQ_PATH_BATCH) {  // the device's report of the rounds each spin block needed
        if (hipHostMalloc((void**)&c->hplan, 5 * sizeof(int), hipHostMallocCoherent | hipHostMallocMapped) != hipSuccess) {
            (void)hipGetLastError();
            c->hplan = nullptr;  // no report: every sweep runs all N / k rounds
        } else {
            for (int i = 0; i < 5; ++i) c->hplan[i] = 0;
        }
    }
    const size_t es = c->prec == CQ_FP64 ? 8 : 4;
    const size_t n = c->n, ne = c->ne;
    constexpr int CHf = cq::chunk_orbitals<float>(), CHd = cq::chunk_orbitals<double>();
    const int C = (int)((n + (es == 8 ? CHd : CHf) - 1) / (es == 8 ? CHd : CHf));
    const size_t Wc = (size_t)c->Wcap;
    struct {
        void** p;
        size_t bytes;
    } plan[] = {
        {(void**)&c->R, sizeof(double) * Wc * ne * 3},
        {&c->M, es * Wc * 2 * n * n},
        {&c->VGL, es * Wc * 2 * n * 5 * n},
        {(void**)&c->logdet, sizeof(double) * Wc * 2},
        {(void**)&c->sign, sizeof(int) * Wc * 2},
        {(void**)&c->nacc, sizeof(long long) * Wc},
        {(void**)&c->nprop, sizeof(long long) * Wc},
        {(void**)&c->eloc, sizeof(double) * Wc},
        {(void**)&c->eold, sizeof(double) * Wc},
        {(void**)&c->elpart, sizeof(double) * Wc * ne},
        {(void**)&c->cnt, sizeof(int) * 3 * Wc},
        {(void**)&c->welec, sizeof(int) * Wc * K},
        {(void**)&c->wslot, sizeof(int) * Wc * K},
        {(void**)&c->jd, sizeof(double) * Wc * c->QR},
        {(void**)&c->rprop, sizeof(double) * Wc * c->QR * 3},
        {(void**)&c->sidx, sizeof(size_t) * Wc * c->QR * 64},
        {&c->swt, es * Wc * c->QR * 64 * 5},
        {(void**)&c->pmat, sizeof(double) * Wc * c->Q * c->Q},
        {(void**)&c->tmat, sizeof(double) * Wc * K * K},
        {(void**)&c->cur, sizeof(int) * Wc * 3},
        {(void**)&c->look, sizeof(int) * Wc * 4},
        {(void**)&c->used, sizeof(int) * 2},
        {(void**)&c->left, sizeof(int) * 2},
        {&c->stage, es * Wc * c->QR * 5 * n},
        {&c->Cbuf, es * Wc * K * n},
        {(void**)&c->ct, sizeof(float) * Wc * n * cq::kMaxDelay},
        {(void**)&c->ub, sizeof(float) * Wc * n * cq::kMaxDelay},
        {(void**)&c->wrho, sizeof(double) * Wc * K},
        {(void**)&c->wG, sizeof(double) * Wc * K * K},
        {(void**)&c->wlinv, sizeof(double) * Wc * K * K},
        {(void**)&c->beta, sizeof(double) * Wc * K},
        {(void**)&c->pend, sizeof(int) * Wc},
        {(void**)&c->part, sizeof(double) * 2 * Wc * C * cq::part_stride(K)},
        {(void**)&c->rnew, sizeof(double) * 4 * Wc * 3},
        {(void**)&c->uid, sizeof(uint32_t) * Wc},
        {(void**)&c->prm, sizeof(cq::Params)},
        {(void**)&c->status, sizeof(int) * Wc},
        {(void**)&c->drift, sizeof(double) * Wc * 2},
        {(void**)&c->drift_max, sizeof(unsigned long long)},
    };
    for (auto& e : plan) {
        cq_status st = dev_alloc(c, e.p, e.bytes);
        if (st != CQ_OK) {
            std::string msg = g_err;
            cq_crowd_destroy(c);
            return fail(st, msg);
        }
    }
    const size_t invb = cq::inverse_work_bytes(2 * c->Wcap, (int)n);
    if (invb) {
        const int nmat = 2 * c->Wcap, b = cq::panel_width((int)n);
        void *S, *PR, *piv, *la, *ng;
        cq_status st = dev_alloc(c, &S, sizeof(double) * nmat * n * cq::s_ld((int)n));
        if (st == CQ_OK) st = dev_alloc(c, &PR, sizeof(double) * nmat * cq::block_width((int)n) * n);
        if (st == CQ_OK) st = dev_alloc(c, &piv, sizeof(int) * nmat * n * 2);
        if (st == CQ_OK) st = dev_alloc(c, &la, sizeof(double) * nmat * 2);  // log|det| and max|A| per matrix
        if (st == CQ_OK) st = dev_alloc(c, &ng, sizeof(int) * nmat * 2);
        if (st != CQ_OK) {
            std::string msg = g_err;
            cq_crowd_destroy(c);
            return fail(st, msg);
        }
        c->inv.S = (double*)S;
        c->inv.PR = (double*)PR;
        c->inv.pivrow = (int*)piv;
        c->inv.logabs = (double*)la;
        c->inv.negs = (int*)ng;
        c->inv.b = b;
    }
    if (s->coulomb) {
        const int pk = (s->nk + cq::ewald_wavevectors_per_block() - 1) / cq::ewald_wavevectors_per_block();
        cq_status st = dev_alloc(c, (void**)&c->ew_phase, sizeof(double2) * Wc * ne * 3 * (s->nmax + 1));
        if (st == CQ_OK) st = dev_alloc(c, (void**)&c->ew_part, sizeof(double) * Wc * (pk + 8));
        if (st != CQ_OK) {
            std::string msg = g_err;
            cq_crowd_destroy(c);
            return fail(st, msg);
        }
    }
    std::vector<uint32_t> uids(W);
    for (int w = 0; w < W; ++w) uids[w] = desc->first_uid + (uint32_t)w;
    hipError_t e = hipMemcpy(c->uid, uids.data(), sizeof(uint32_t) * W, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        cq_crowd_destroy(c);
        return fail(CQ_EDEVICE, std::string("hipMemcpy uids: ") + hipGetErrorString(e));
    }
    c->hp = cq::Params{};
    c->hp.sigma = 0.5;
    e = hipMemcpy(c->prm, &c->hp, sizeof(cq::Params), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        cq_crowd_destroy(c);
        return fail(CQ_EDEVICE, std::string("hipMemcpy params: ") + hipGetErrorString(e));
    }
    *out = c;
    return CQ_OK;
}

cq_status cq_crowd_set_positions(cq_crowd* c, const double* R, int on_device, uint32_t first_step)
{
    if (!c || !R) return fail(CQ_EINVAL, "NULL argument");
    if (!c->subs.empty()) {
        size_t off = 0;
        for (cq_crowd* sub : c->subs) {
            cq_status st = cq_crowd_set_positions(sub, R + off, on_device, first_step);
            if (st != CQ_OK) return st;
            off += (size_t)sub->W * sub->ne * 3;
        }
        c->ready = true;
        return CQ_OK;
    }
    const size_t bytes = sizeof(double) * c->W * c->ne * 3;
    HIP_TRY(hipStreamSynchronize(c->stream));
    HIP_TRY(hipMemcpy(c->R, R, bytes, on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice));
    c->hp.step = first_step;
    c->hp.rec_sweep = 0;
    cq_status st = push_params(c);
    if (st != CQ_OK) return st;
    c->ready = false;
    c->since_recompute = 0;
    st = c->prec == CQ_FP64 ? setup_state<double>(c) : setup_state<float>(c);
    if (st != CQ_OK) return st;
    HIP_TRY(hipMemcpyAsync(c->eold, c->eloc, sizeof(double) * c->W, hipMemcpyDeviceToDevice, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    c->ready = true;
    return CQ_OK;
}

// Delay-rank autotuning: time `sweeps` eager sweeps at every k in {1, 2, 4, ..., Kcap}
// (powers of two below Kcap, then Kcap itself)
// (the window buffers are sized for Kcap) and keep the fastest.  The timed sweeps are
// ordinary sweeps of the chain.
static cq_status autotune_k(cq_crowd* c, int sweeps, int* chosen)
{
    if (c->path == CQ_PATH_SWEEP) {  // delay rank 1 by construction
        c->tuned = true;
        if (chosen) *chosen = c->K;
        return CQ_OK;
    }
    hipEvent_t a, b;
    HIP_TRY(hipEventCreate(&a));
    if (hipEventCreate(&b) != hipSuccess) {
        (void)hipEventDestroy(a);
        return fail(CQ_EDEVICE, "hipEventCreate failed");
    }
    int best_k = c->K;
    float best_ms = 0.0f;
    std::vector<int> cands;
    for (int k = 1; k < c->Kcap; k *= 2) cands.push_back(k);
    cands.push_back(c->Kcap);
    for (int k : cands) {
        c->K = k;
        apply_q(c);
        drop_graph(c);
        reset_plan(c);  // the previous candidate's sweeps have completed (event synchronised)
        if (c->path == CQ_PATH_MULTI) {
            if (c->prec == CQ_FP64)
                cq::launch_first_proposal<double>(view<double>(c), c->stream);
            else
                cq::launch_first_proposal<float>(view<float>(c), c->stream);
        }
        hipError_t er = hipEventRecord(a, c->stream);
        for (int s = 0; s < sweeps; ++s) {
            sweep(c);
            c->hp.step += 1;
            c->hp.rec_sweep += 1;
        }
        if (er == hipSuccess) er = hipEventRecord(b, c->stream);
        if (er == hipSuccess) er = hipEventSynchronize(b);
        cq_status es = enqueue_status(c, "autotune sweep");
        if (er != hipSuccess || es != CQ_OK) {
            (void)hipEventDestroy(a);
            (void)hipEventDestroy(b);
            return es != CQ_OK ? es : fail(CQ_EDEVICE, std::string("autotune events: ") + hipGetErrorString(er));
        }
        float ms = 0.0f;
        HIP_TRY(hipEventElapsedTime(&ms, a, b));
        if (best_ms == 0.0f || ms < best_ms) {
            best_ms = ms;
            best_k = k;
        }
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    c->K = best_k;
    apply_q(c);
    drop_graph(c);
    reset_plan(c);
    c->tuned = true;
    if (chosen) *chosen = best_k;
    return check_singular(c, "autotune");
}

cq_status cq_crowd_autotune(cq_crowd* c, int sweeps_per_candidate, int* chosen_k)
{
    if (!c) return fail(CQ_EINVAL, "crowd is NULL");
    if (!c->subs.empty()) {
        for (cq_crowd* sub : c->subs) {
            cq_status st = cq_crowd_autotune(sub, sweeps_per_candidate, nullptr);
            if (st != CQ_OK) return st;
        }
        if (chosen_k) *chosen_k = c->subs[0]->K;
        return CQ_OK;
    }
    if (sweeps_per_candidate < 1) return fail(CQ_EINVAL, "sweeps_per_candidate must be >= 1");
    if (!c->ready) return fail(CQ_ESTATE, "set positions before autotuning");
    return autotune_k(c, sweeps_per_candidate, chosen_k);
}

cq_status cq_crowd_run_vmc(cq_crowd* c, int n_sweeps, double sigma)
{
    if (!c) return fail(CQ_EINVAL, "crowd is NULL");
    if (!c->subs.empty()) {
        for (cq_crowd* sub : c->subs) {
            cq_status st = cq_crowd_run_vmc(sub, n_sweeps, sigma);
            if (st != CQ_OK) return st;
        }
        return CQ_OK;
    }
    if (n_sweeps < 0 || !(sigma > 0.0) || !std::isfinite(sigma)) return fail(CQ_EINVAL, "bad n_sweeps or sigma");
    if (!c->ready) return fail(CQ_ESTATE, "set positions before running");
    if (sigma != c->hp.sigma) {
        c->hp.sigma = sigma;
        cq_status st = push_params(c);
        if (st != CQ_OK) return st;
    }
    if (c->autotune && !c->tuned && n_sweeps > 0) {
        cq_status st = autotune_k(c, 1, nullptr);
        if (st != CQ_OK) return st;
    }
    // proposal of the first move (each move kernel makes the next one's)
    if (c->path == CQ_PATH_MULTI) {
        if (c->prec == CQ_FP64)
            cq::launch_first_proposal<double>(view<double>(c), c->stream);
        else
            cq::launch_first_proposal<float>(view<float>(c), c->stream);
    }
    for (int s = 0; s < n_sweeps; ++s) {
        if (update_plan(c)) drop_graph(c);
        if (c->use_graph && !c->timing_mask) {
            if (!c->gexec) {
                cq_status st = build_graph(c);
                if (st != CQ_OK) return st;
            }
            HIP_TRY(hipGraphLaunch(c->gexec, c->stream));
        } else {
            sweep(c);
        }
        c->hp.step += 1;
        c->hp.rec_sweep += 1;
        if (c->recompute_every > 0 && ++c->since_recompute >= c->recompute_every) {
            // singular or non-finite pivots set the walker's status bit, which the next
            // synchronising call reports; the drift goes into the crowd's drift record
            inverse(c);
            c->since_recompute = 0;
            c->n_recomputes++;
        }
    }
    return enqueue_status(c, "run_vmc");
}

}  // extern "C"

namespace {

// DMC generations of one crowd, or of every system of a group (the walkers of all systems
// moved by the same launches, then each system's energy and branching).  e_trial and
// n_target per system (e_trial NaN: continue with the current E_T); history [gen][S][4].
cq_status run_dmc_set(cq_crowd* owner, const std::vector<cq_crowd*>& set, int n_generations, double tau,
                      const double* e_trial, const int* n_target, double* history)
{
    const int S = (int)set.size();
    for (int s = 0; s < S; ++s) {
        cq_crowd* c = set[s];
        if (!c->ready) return fail(CQ_ESTATE, "set positions before running");
        if (n_target[s] < 1) return fail(CQ_EINVAL, "n_target must be >= 1");
    }
    if (n_generations == 0) return CQ_OK;
    for (int s = 0; s < S; ++s) {
        cq_crowd* c = set[s];
        cq_status st = ensure_dmc(c, n_generations);
        if (st != CQ_OK) return st;
        c->hp.tau = tau;
        st = push_params(c);
        if (st != CQ_OK) return st;
        cq::DmcState ds{};
        HIP_TRY(hipMemcpy(&ds, c->dmc_state, sizeof(ds), hipMemcpyDeviceToHost));
        if (e_trial && std::isfinite(e_trial[s])) ds.e_t = e_trial[s];
        ds.status = 0;
        HIP_TRY(hipMemcpy(c->dmc_state, &ds, sizeof(ds), hipMemcpyHostToDevice));
        drop_graph(c);  // walker buffers and the population change from here on
        // the generation sums count the moves each walker made since the last branching: clear
        // the counters the walkers bring from VMC sweeps (children of a branching start at zero)
        HIP_TRY(hipMemsetAsync(c->nacc, 0, sizeof(long long) * c->W, c->stream));
        HIP_TRY(hipMemsetAsync(c->nprop, 0, sizeof(long long) * c->W, c->stream));
    }
    const bool fp64 = owner->prec == CQ_FP64;
    for (int gen = 0; gen < n_generations; ++gen) {
        if (S == 1) {
            if (fp64)
                dmc_moves<double>(set[0]);
            else
                dmc_moves<float>(set[0]);
        } else {
            cq_status st = fp64 ? group_moves<double>(owner) : group_moves<float>(owner);
            if (st != CQ_OK) return st;
        }
        for (int s = 0; s < S; ++s) {
            cq_crowd* c = set[s];
            const bool rc = c->recompute_every > 0 && ++c->since_recompute >= c->recompute_every;
            if (rc) {
                c->since_recompute = 0;
                c->n_recomputes++;
            }
            if (fp64)
                dmc_post<double>(c, gen, n_target[s], tau, rc);
            else
                dmc_post<float>(c, gen, n_target[s], tau, rc);
        }
        cq_status es = enqueue_status(owner, "run_dmc");
        if (es != CQ_OK) return es;
        HIP_TRY(hipStreamSynchronize(owner->stream));
        for (int s = 0; s < S; ++s) {
            cq_crowd* c = set[s];
            cq::DmcState ds{};
            HIP_TRY(hipStreamSynchronize(c->stream));
            HIP_TRY(hipMemcpy(&ds, c->dmc_state, sizeof(ds), hipMemcpyDeviceToHost));
            c->hp.step += 1;
            c->hp.rec_sweep += 1;
            if (ds.status) {
                if (history)
                    for (int g2 = 0; g2 < gen; ++g2)
                        HIP_TRY(hipMemcpy(history + ((size_t)g2 * S + s) * 4, c->dmc_hist + (size_t)g2 * 4,
                                          sizeof(double) * 4, hipMemcpyDeviceToHost));
                return fail(CQ_ESTATE, "DMC population " + std::to_string(ds.new_pop) +
                                           (ds.new_pop == 0 ? " died out" : " exceeds max_walkers") +
                                           (S > 1 ? " in system " + std::to_string(s) : std::string()) +
                                           " at generation " + std::to_string(gen));
            }
            cq_status cs = check_singular(c, "run_dmc");
            if (cs != CQ_OK) return cs;
            swap_walker_sets(c);
            c->W = ds.new_pop;
        }
        if (S > 1) {
            int tot = 0;
            for (cq_crowd* c : set) tot += c->W;
            owner->W = tot;
        }
    }
    if (history)
        for (int s = 0; s < S; ++s)
            for (int g2 = 0; g2 < n_generations; ++g2)
                HIP_TRY(hipMemcpy(history + ((size_t)g2 * S + s) * 4, set[s]->dmc_hist + (size_t)g2 * 4,
                                  sizeof(double) * 4, hipMemcpyDeviceToHost));
    return CQ_OK;
}

}  // namespace

extern "C" {

cq_status cq_crowd_run_dmc(cq_crowd* c, int n_generations, double tau, double e_trial, int n_target,
                           double* history)
{
    if (!c) return fail(CQ_EINVAL, "crowd is NULL");
    if (!c->subs.empty()) return fail(CQ_EINVAL, "a crowd of several systems runs DMC with cq_crowd_run_dmc_systems");
    if (n_generations < 0 || !(tau > 0.0) || !std::isfinite(tau) || n_target < 1)
        return fail(CQ_EINVAL, "bad n_generations, tau or n_target");
    return run_dmc_set(c, {c}, n_generations, tau, &e_trial, &n_target, history);
}

cq_status cq_crowd_run_dmc_systems(cq_crowd* c, int n_generations, double tau, const double* e_trial,
                                   const int* n_target, double* history)
{
    if (!c) return fail(CQ_EINVAL, "crowd is NULL");
    if (n_generations < 0 || !(tau > 0.0) || !std::isfinite(tau)) return fail(CQ_EINVAL, "bad n_generations or tau");
    std::vector<cq_crowd*> set = c->subs.empty() ? std::vector<cq_crowd*>{c} : c->subs;
    std::vector<int> tgt(set.size());
    for (size_t s = 0; s < set.size(); ++s) tgt[s] = n_target ? n_target[s] : set[s]->W;
    return run_dmc_set(c, set, n_generations, tau, e_trial, tgt.data(), history);
}

cq_status cq_crowd_set_round_plan(cq_crowd* c, int rounds)
{
    if (!c) return fail(CQ_EINVAL, "crowd is NULL");
    if (rounds < 0) return fail(CQ_EINVAL, "rounds must be >= 0");
    if (!c->subs.empty()) {
        for (cq_crowd* sub : c->subs) {
            cq_status st = cq_crowd_set_round_plan(sub, rounds);
            if (st != CQ_OK) return st;
        }
        return CQ_OK;
    }
    c->plan_fixed = rounds;
    drop_graph(c);
    return CQ_OK;
}

cq_status cq_crowd_get_round_plan(cq_crowd* c, int* rounds)
{
    if (!c || !rounds) return fail(CQ_EINVAL, "NULL argument");
    cq_crowd* x = c->subs.empty() ? c : c->subs[0];
    if (x->path != CQ_PATH_BATCH) {
        rounds[0] = rounds[1] = 0;
        return CQ_OK;
    }
    if (update_plan(x)) drop_graph(x);  // a captured sweep holds the old plan's rounds
    const int all = cq::batch_rounds(x->n, x->K);
    for (int s = 0; s < 2; ++s) rounds[s] = planned_rounds(x, s, all);
    return CQ_OK;
}

cq_status cq_crowd_get_path(cq_crowd* c, int* path)
{
    if (!c || !path) return fail(CQ_EINVAL, "NULL argument");
    *path = c->subs.empty() ? c->path : c->subs[0]->path;
    return CQ_OK;
}

cq_status cq_crowd_set_tiles(cq_crowd* c, const cq_tiles* t)
{
    if (!c || !t) return fail(CQ_EINVAL, "NULL argument");
    if (!c->subs.empty()) {
        for (cq_crowd* sub : c->subs) {
            cq_status st = cq_crowd_set_tiles(sub, t);
            if (st != CQ_OK) return st;
        }
        return CQ_OK;
    }
    if (t->gather_blocks_per_cu < 0 || t->gather_blocks_per_cu > 8)
        return fail(CQ_EINVAL, "gather_blocks_per_cu must be 0..8");
    if (t->update_kernel < 0 || t->update_kernel > 2) return fail(CQ_EINVAL, "update_kernel must be 0..2");
    if (t->candidates < 0) return fail(CQ_EINVAL, "candidates must be >= 0");
    if (c->path != CQ_PATH_BATCH) return CQ_OK;
    if (t->candidates > 0 && (t->candidates < min_candidates(c) || t->candidates > c->Qcap))
        return fail(CQ_EINVAL, "candidates must lie in [" + std::to_string(min_candidates(c)) + ", " +
                                   std::to_string(c->Qcap) + "] at this delay rank");
    // rounds per block depend on Q: restart the plan once no report of the old shapes is due
    HIP_TRY(hipStreamSynchronize(c->stream));
    c->q_req = t->candidates;
    c->vgl_wg = t->gather_blocks_per_cu;
    c->upd_kernel = t->update_kernel;
    apply_q(c);
    drop_graph(c);
    reset_plan(c);
    return CQ_OK;
}

cq_status cq_crowd_get_tiles(cq_crowd* c, cq_tiles* t)
{
    if (!c || !t) return fail(CQ_EINVAL, "NULL argument");
    cq_crowd* x = c->subs.empty() ? c : c->subs[0];
    if (x->path != CQ_PATH_BATCH) {
        t->candidates = 0;
        t->gather_blocks_per_cu = 0;
        t->update_kernel = 0;
        return CQ_OK;
    }
    t->candidates = x->Q;
    t->gather_blocks_per_cu = cq::batch_vgl_blocks_per_cu(x->n, x->prec == CQ_FP64 ? 8 : 4, x->vgl_wg);
    t->update_kernel = (x->prec == CQ_FP64 ? x->upd_kernel == 2 && cq::flush_f64_mfma_fits(x->n)
                                            : cq::flush_mfma_fits(x->n)) ? 2 : 1;
    return CQ_OK;
}

}  // extern "C"

namespace {

// "<architecture>/<compute units>cu" of the current device, the tile cache's device key
cq_status device_key(std::string* key)
{
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, dev));
    std::string arch;
    for (const char* p = prop.gcnArchName; *p && arch.size() < 100; ++p)
        if (*p != '"' && *p != '\\' && (unsigned char)*p >= 0x20) arch.push_back(*p);
    *key = (arch.empty() ? std::string("unknown") : arch) + "/" + std::to_string(prop.multiProcessorCount) + "cu";
    return CQ_OK;
}

// Time `sweeps` eager sweeps of the chain (after one untimed sweep that learns the round
// plan for the current shapes); *ms per sweep.
cq_status time_sweeps(cq_crowd* c, int sweeps, hipEvent_t a, hipEvent_t b, float* ms)
{
    auto one = [&]() {
        if (update_plan(c)) drop_graph(c);
        sweep(c);
        c->hp.step += 1;
        c->hp.rec_sweep += 1;
    };
    one();
    HIP_TRY(hipStreamSynchronize(c->stream));  // the plan report of that sweep is in
    cq_status es = enqueue_status(c, "tile autotune sweep");
    if (es != CQ_OK) return es;
    (void)update_plan(c);
    HIP_TRY(hipEventRecord(a, c->stream));
    for (int s = 0; s < sweeps; ++s) {
        sweep(c);
        c->hp.step += 1;
        c->hp.rec_sweep += 1;
    }
    HIP_TRY(hipEventRecord(b, c->stream));
    HIP_TRY(hipEventSynchronize(b));
    es = enqueue_status(c, "tile autotune sweep");
    if (es != CQ_OK) return es;
    float t = 0.0f;
    HIP_TRY(hipEventElapsedTime(&t, a, b));
    *ms = t / sweeps;
    return CQ_OK;
}

cq_status autotune_tiles(cq_crowd* c, int sweeps, const char* cache, cq_tiles* chosen, int* from_cache)
{
    if (from_cache) *from_cache = 0;
    if (c->path != CQ_PATH_BATCH) return chosen ? cq_crowd_get_tiles(c, chosen) : CQ_OK;
    if (c->autotune && !c->tuned) {  // the delay rank is part of the key: choose it first
        cq_status st = autotune_k(c, 1, nullptr);
        if (st != CQ_OK) return st;
    }
    std::string dev;
    cq_status st = device_key(&dev);
    if (st != CQ_OK) return st;
    if (cache) {
        cq_tiles t{};
        int found = 0;
        st = cq_tile_cache_find(cache, dev.c_str(), c->n, c->W, c->prec, c->K, &t, &found);
        if (st != CQ_OK) return st;
        if (found && cq_crowd_set_tiles(c, &t) == CQ_OK) {
            if (from_cache) *from_cache = 1;
            return chosen ? cq_crowd_get_tiles(c, chosen) : CQ_OK;
        }
    }
    // candidates: Q in {1.5 k, 2 k, default}, gather workgroups per CU in {1, 2, 3}
    std::vector<int> qs;
    const int qdef = std::min(std::max(cq::batch_candidates(c->n, c->K), min_candidates(c)), c->Qcap);
    for (int q : {(3 * c->K + 1) / 2, 2 * c->K, qdef}) {
        q = std::min(std::max(q, min_candidates(c)), c->Qcap);
        if (std::find(qs.begin(), qs.end(), q) == qs.end()) qs.push_back(q);
    }
    hipEvent_t a, b;
    HIP_TRY(hipEventCreate(&a));
    if (hipEventCreate(&b) != hipSuccess) {
        (void)hipEventDestroy(a);
        return fail(CQ_EDEVICE, "hipEventCreate failed");
    }
    // the FP64 update kernels: vector units, and the matrix cores when they take this N
    std::vector<int> uks{1};
    if (c->prec == CQ_FP64 && cq::flush_f64_mfma_fits(c->n)) uks.push_back(2);
    cq_tiles best{0, 0, 0};
    float best_ms = 0.0f;
    for (int q : qs)
        for (int g = 1; g <= 3 && st == CQ_OK; ++g)
            for (int uk : uks) {
                if (st != CQ_OK) break;
                const cq_tiles t{q, g, c->prec == CQ_FP64 ? uk : 0};
                st = cq_crowd_set_tiles(c, &t);
                float ms = 0.0f;
                if (st == CQ_OK) st = time_sweeps(c, sweeps, a, b, &ms);
                if (st == CQ_OK && (best_ms == 0.0f || ms < best_ms)) {
                    best_ms = ms;
                    best = t;
                }
            }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (st != CQ_OK) return st;
    st = cq_crowd_set_tiles(c, &best);
    if (st != CQ_OK) return st;
    if (cache) {
        st = cq_tile_cache_store(cache, dev.c_str(), c->n, c->W, c->prec, c->K, &best, best_ms);
        if (st != CQ_OK) return st;
    }
    if (chosen) *chosen = best;
    return check_singular(c, "tile autotune");
}

}  // namespace

extern "C" {

cq_status cq_crowd_autotune_tiles(cq_crowd* c, int sweeps_per_candidate, const char* cache_path, cq_tiles* chosen,
                                  int* from_cache)
{
    if (!c) return fail(CQ_EINVAL, "crowd is NULL");
    if (sweeps_per_candidate < 1) return fail(CQ_EINVAL, "sweeps_per_candidate must be >= 1");
    if (!c->subs.empty()) {
        for (cq_crowd* sub : c->subs) {
            cq_status st = cq_crowd_autotune_tiles(sub, sweeps_per_candidate, cache_path, nullptr, from_cache);
            if (st != CQ_OK) return st;
        }
        return chosen ? cq_crowd_get_tiles(c, chosen) : CQ_OK;
    }
    if (!c->ready) return fail(CQ_ESTATE, "set positions before autotuning");
    return autotune_tiles(c, sweeps_per_candidate, cache_path, chosen, from_cache);
}

cq_status cq_crowd_get_delay_rank(cq_crowd* c, int* k)
{
    if (!c || !k) return fail(CQ_EINVAL, "NULL argument");
    if (!c->subs.empty()) {
        *k = c->subs[0]->K;
        return CQ_OK;
    }
    *k = c->K;
    return CQ_OK;
}

cq_status cq_crowd_get_population(cq_crowd* c, int* n_walkers)
{
    if (!c || !n_walkers) return fail(CQ_EINVAL, "NULL argument");
    if (!c->subs.empty()) {
        int tot = 0;
        for (cq_crowd* sub : c->subs) tot += sub->W;
        *n_walkers = tot;
        return CQ_OK;
    }
    *n_walkers = c->W;
    return CQ_OK;
}

cq_status cq_crowd_recompute(cq_crowd* c, double* max_drift)
{
    if (!c) return fail(CQ_EINVAL, "crowd is NULL");
    if (!c->subs.empty()) {
        double m = 0.0;
        for (cq_crowd* sub : c->subs) {
            double d = 0.0;
            cq_status st = cq_crowd_recompute(sub, max_drift ? &d : nullptr);
            if (st != CQ_OK) return st;
            m = std::max(m, d);
        }
        if (max_drift) *max_drift = m;
        return CQ_OK;
    }
    if (!c->ready) return fail(CQ_ESTATE, "set positions before recomputing");
    inverse(c);
    HIP_TRY(hipGetLastError());
    c->since_recompute = 0;
    c->n_recomputes++;
    cq_status st = check_singular(c, "recompute");
    if (st != CQ_OK) return st;
    if (max_drift) {
        std::vector<double> d(2 * c->W);
        HIP_TRY(hipMemcpy(d.data(), c->drift, sizeof(double) * 2 * c->W, hipMemcpyDeviceToHost));
        double m = 0.0;
        for (double x : d) m = std::max(m, x);
        *max_drift = m;
    }
    return CQ_OK;
}

static cq_status copy_out(cq_crowd* c, void* dst, const void* src, size_t bytes)
{
    if (!c) return fail(CQ_EINVAL, "crowd is NULL");
    if (!dst) return CQ_OK;
    HIP_TRY(hipStreamSynchronize(c->stream));
    HIP_TRY(hipMemcpy(dst, src, bytes, hipMemcpyDeviceToHost));
    return CQ_OK;
}

// Every get call ends here: the walkers' status bits (a singular or non-finite matrix at
// an in-run recompute, window bookkeeping out of range) become the call's status, so an
// error inside an asynchronous run surfaces at the first synchronising call after it.
static cq_status got(cq_crowd* c, cq_status st, const char* where)
{
    if (st != CQ_OK) return st;
    return check_singular(c, where);
}

cq_status cq_crowd_virtual_ratios(cq_crowd* c, const double* offsets, int n_q, double* ratio, double* rho,
                                  double* dlnj, int out_on_device)
{
    if (!c || !offsets) return fail(CQ_EINVAL, "NULL argument");
    if (!c->subs.empty()) {
        size_t off = 0;
        for (cq_crowd* sub : c->subs) {
            cq_status st = cq_crowd_virtual_ratios(sub, offsets, n_q, ratio ? ratio + off : nullptr,
                                                   rho ? rho + off : nullptr, dlnj ? dlnj + off : nullptr,
                                                   out_on_device);
            if (st != CQ_OK) return st;
            off += (size_t)sub->W * sub->ne * n_q;
        }
        return CQ_OK;
    }
    if (n_q < 1 || n_q > 64) return fail(CQ_EINVAL, "n_q must be 1..64");
    if (!c->ready) return fail(CQ_ESTATE, "positions not set");
    HIP_TRY(hipStreamSynchronize(c->stream));
    if (n_q > c->voff_cap) {
        if (c->voff) HIP_TRY(hipFree(c->voff));
        c->voff = nullptr;
        c->voff_cap = 0;
        if (hipMalloc((void**)&c->voff, sizeof(double) * 3 * 64) != hipSuccess) {
            (void)hipGetLastError();
            return fail(CQ_ENOMEM, "virtual-move offsets");
        }
        c->voff_cap = 64;
    }
    HIP_TRY(hipMemcpy(c->voff, offsets, sizeof(double) * 3 * (size_t)n_q, hipMemcpyHostToDevice));
    const size_t cnt = (size_t)c->W * c->ne * n_q;
    double* d[3] = {ratio, rho, dlnj};
    if (!out_on_device) {
        // staging for the host outputs, kept for later calls
        if (3 * cnt > c->vout_cap) {
            if (c->vout) HIP_TRY(hipFree(c->vout));
            c->vout = nullptr;
            c->vout_cap = 0;
            if (hipMalloc((void**)&c->vout, sizeof(double) * 3 * cnt) != hipSuccess) {
                (void)hipGetLastError();
                return fail(CQ_ENOMEM, "virtual-move outputs");
            }
            c->vout_cap = 3 * cnt;
        }
        for (int k = 0; k < 3; ++k) d[k] = d[k] ? c->vout + k * cnt : nullptr;
    }
    timed_begin(c, CQ_KERNEL_VIRTUAL);
    if (c->prec == CQ_FP64)
        cq::launch_virtual<double>(view<double>(c), c->voff, n_q, d[0], d[1], d[2], c->stream);
    else
        cq::launch_virtual<float>(view<float>(c), c->voff, n_q, d[0], d[1], d[2], c->stream);
    timed_end(c, CQ_KERNEL_VIRTUAL);
    HIP_TRY(hipGetLastError());
    if (!out_on_device) {
        double* h[3] = {ratio, rho, dlnj};
        for (int k = 0; k < 3; ++k) {
            cq_status st = copy_out(c, h[k], d[k], sizeof(double) * cnt);
            if (st != CQ_OK) return st;
        }
        return got(c, CQ_OK, "virtual_ratios");
    }
    return CQ_OK;
}


cq_status cq_crowd_get_logdet(cq_crowd* c, double* logdet, int* sign)
{
    if (!c) return fail(CQ_EINVAL, "crowd is NULL");
    if (!c->subs.empty()) {
        size_t off = 0;
        for (cq_crowd* sub : c->subs) {
            cq_status st = cq_crowd_get_logdet(sub, logdet ? logdet + 2 * off : nullptr, sign ? sign + 2 * off : nullptr);
            if (st != CQ_OK) return st;
            off += sub->W;
        }
        return CQ_OK;
    }
    cq_status st = copy_out(c, logdet, c->logdet, sizeof(double) * 2 * c->W);
    if (st != CQ_OK) return st;
    return got(c, copy_out(c, sign, c->sign, sizeof(int) * 2 * c->W), "get_logdet");
}

cq_status cq_crowd_get_acceptance(cq_crowd* c, int64_t* accepted, int64_t* proposed)
{
    if (!c) return fail(CQ_EINVAL, "crowd is NULL");
    if (!c->subs.empty()) {
        size_t off = 0;
        for (cq_crowd* sub : c->subs) {
            cq_status st = cq_crowd_get_acceptance(sub, accepted ? accepted + off : nullptr,
                                                   proposed ? proposed + off : nullptr);
            if (st != CQ_OK) return st;
            off += sub->W;
        }
        return CQ_OK;
    }
    cq_status st = copy_out(c, accepted, c->nacc, sizeof(int64_t) * c->W);
    if (st != CQ_OK) return st;
    return got(c, copy_out(c, proposed, c->nprop, sizeof(int64_t) * c->W), "get_acceptance");
}

cq_status cq_crowd_get_local_energy(cq_crowd* c, double* e_l)
{
    if (!c) return fail(CQ_EINVAL, "crowd is NULL");
    if (!c->subs.empty()) {
        size_t off = 0;
        for (cq_crowd* sub : c->subs) {
            cq_status st = cq_crowd_get_local_energy(sub, e_l ? e_l + off : nullptr);
            if (st != CQ_OK) return st;
            off += sub->W;
        }
        return CQ_OK;
    }
    return got(c, copy_out(c, e_l, c->eloc, sizeof(double) * c->W), "get_local_energy");
}

cq_status cq_crowd_get_positions(cq_crowd* c, double* R, int* n_walkers_per_system)
{
    if (!c) return fail(CQ_EINVAL, "crowd is NULL");
    if (!c->subs.empty()) {
        size_t off = 0;
        for (size_t k = 0; k < c->subs.size(); ++k) {
            cq_crowd* sub = c->subs[k];
            cq_status st = cq_crowd_get_positions(sub, R ? R + off : nullptr, nullptr);
            if (st != CQ_OK) return st;
            if (n_walkers_per_system) n_walkers_per_system[k] = sub->W;
            off += (size_t)sub->W * sub->ne * 3;
        }
        return CQ_OK;
    }
    if (n_walkers_per_system) n_walkers_per_system[0] = c->W;
    return got(c, copy_out(c, R, c->R, sizeof(double) * c->W * c->ne * 3), "get_positions");
}

cq_status cq_crowd_get_drift(cq_crowd* c, double* last, double* max_drift, int* n_recomputes)
{
    if (!c) return fail(CQ_EINVAL, "crowd is NULL");
    if (!c->subs.empty()) {
        size_t off = 0;
        double m = 0.0;
        int nr = 0;
        for (cq_crowd* sub : c->subs) {
            double dm = 0.0;
            int k = 0;
            cq_status st = cq_crowd_get_drift(sub, last ? last + 2 * off : nullptr, &dm, &k);
            if (st != CQ_OK) return st;
            m = std::max(m, dm);
            nr = std::max(nr, k);
            off += sub->W;
        }
        if (max_drift) *max_drift = m;
        if (n_recomputes) *n_recomputes = nr;
        return CQ_OK;
    }
    cq_status st = copy_out(c, last, c->drift, sizeof(double) * 2 * c->W);
    if (st != CQ_OK) return st;
    unsigned long long bits = 0;
    st = copy_out(c, &bits, c->drift_max, sizeof(bits));
    if (st != CQ_OK) return st;
    double m;
    std::memcpy(&m, &bits, sizeof(m));
    if (max_drift) *max_drift = m;
    if (n_recomputes) *n_recomputes = c->n_recomputes;
    return got(c, CQ_OK, "get_drift");
}

cq_status cq_crowd_get_uids(cq_crowd* c, uint32_t* uids)
{
    if (!c) return fail(CQ_EINVAL, "crowd is NULL");
    if (!c->subs.empty()) {
        size_t off = 0;
        for (cq_crowd* sub : c->subs) {
            cq_status st = cq_crowd_get_uids(sub, uids ? uids + off : nullptr);
            if (st != CQ_OK) return st;
            off += sub->W;
        }
        return CQ_OK;
    }
    return got(c, copy_out(c, uids, c->uid, sizeof(uint32_t) * c->W), "get_uids");
}

cq_status cq_crowd_get_inverse(cq_crowd* c, double* ainv)
{
    if (!c) return fail(CQ_EINVAL, "crowd is NULL");
    if (!c->subs.empty()) {
        size_t off = 0;
        for (cq_crowd* sub : c->subs) {
            cq_status st = cq_crowd_get_inverse(sub, ainv ? ainv + off : nullptr);
            if (st != CQ_OK) return st;
            off += (size_t)sub->W * 2 * sub->n * sub->n;
        }
        return CQ_OK;
    }
    if (!ainv) return CQ_OK;
    const size_t n = c->n, cnt = (size_t)c->W * 2 * n * n;
    const size_t es = c->prec == CQ_FP64 ? 8 : 4;
    std::vector<unsigned char> raw(cnt * es);
    cq_status st = got(c, copy_out(c, raw.data(), c->M, cnt * es), "get_inverse");
    if (st != CQ_OK) return st;
    for (size_t m = 0; m < (size_t)c->W * 2; ++m)
        for (size_t i = 0; i < n; ++i)
            for (size_t j = 0; j < n; ++j) {
                const size_t src = (m * n + i) * n + j;  // M[i][j] = A^-1[j][i]
                ainv[(m * n + j) * n + i] = es == 8 ? ((const double*)raw.data())[src]
                                                    : (double)((const float*)raw.data())[src];
            }
    return CQ_OK;
}

cq_status cq_crowd_set_forced_decisions(cq_crowd* c, const uint8_t* flags, int n_sweeps)
{
    if (!c) return fail(CQ_EINVAL, "crowd is NULL");
    if (!c->subs.empty()) return fail(CQ_EINVAL, "parity mode works on crowds of one system");
    if (flags && n_sweeps < 1) return fail(CQ_EINVAL, "n_sweeps must be >= 1");
    HIP_TRY(hipStreamSynchronize(c->stream));
    if (c->forced) {
        HIP_TRY(hipFree(c->forced));
        c->forced = nullptr;
    }
    c->forced_cap = 0;
    if (flags) {
        const size_t bytes = (size_t)n_sweeps * c->ne * c->Wcap;
        if (hipMalloc((void**)&c->forced, bytes) != hipSuccess) {
            (void)hipGetLastError();
            c->forced = nullptr;
            return fail(CQ_ENOMEM, "forced-decision buffer");
        }
        HIP_TRY(hipMemcpy(c->forced, flags, bytes, hipMemcpyHostToDevice));
        c->forced_cap = n_sweeps;
    }
    c->hp.forced_cap = c->forced_cap;
    c->hp.rec_sweep = 0;
    drop_graph(c);
    return push_params(c);
}

cq_status cq_crowd_set_forced_branching(cq_crowd* c, const int* mult, int n_generations)
{
    if (!c) return fail(CQ_EINVAL, "crowd is NULL");
    if (!c->subs.empty()) return fail(CQ_EINVAL, "parity mode works on crowds of one system");
    if (mult && n_generations < 1) return fail(CQ_EINVAL, "n_generations must be >= 1");
    HIP_TRY(hipStreamSynchronize(c->stream));
    if (c->forced_mult) {
        HIP_TRY(hipFree(c->forced_mult));
        c->forced_mult = nullptr;
    }
    c->mult_cap = 0;
    if (mult) {
        const size_t cnt = (size_t)n_generations * c->Wcap;
        for (size_t i = 0; i < cnt; ++i)
            if (mult[i] < 0 || mult[i] > 3) return fail(CQ_EINVAL, "multiplicities must be 0..3");
        if (hipMalloc((void**)&c->forced_mult, cnt * sizeof(int)) != hipSuccess) {
            (void)hipGetLastError();
            c->forced_mult = nullptr;
            return fail(CQ_ENOMEM, "forced-multiplicity buffer");
        }
        HIP_TRY(hipMemcpy(c->forced_mult, mult, cnt * sizeof(int), hipMemcpyHostToDevice));
        c->mult_cap = n_generations;
    }
    c->hp.mult_cap = c->mult_cap;
    c->hp.rec_sweep = 0;
    drop_graph(c);
    return push_params(c);
}

cq_status cq_crowd_get_dmc_moves(cq_crowd* c, int64_t* accepted, int64_t* proposed)
{
    if (!c) return fail(CQ_EINVAL, "crowd is NULL");
    if (!c->subs.empty()) {
        int64_t a = 0, b = 0;
        for (cq_crowd* sub : c->subs) {
            int64_t x = 0, y = 0;
            cq_status st = cq_crowd_get_dmc_moves(sub, &x, &y);
            if (st != CQ_OK) return st;
            a += x;
            b += y;
        }
        if (accepted) *accepted = a;
        if (proposed) *proposed = b;
        return CQ_OK;
    }
    if (!c->have_alt) {
        if (accepted) *accepted = 0;
        if (proposed) *proposed = 0;
        return CQ_OK;
    }
    cq::DmcState ds{};
    cq_status st = copy_out(c, &ds, c->dmc_state, sizeof(ds));
    if (st != CQ_OK) return st;
    if (accepted) *accepted = ds.nacc;
    if (proposed) *proposed = ds.nprop;
    return CQ_OK;
}

cq_status cq_crowd_record_moves(cq_crowd* c, int n_sweeps)
{
    if (!c) return fail(CQ_EINVAL, "crowd is NULL");
    if (!c->subs.empty()) return fail(CQ_EINVAL, "parity mode works on crowds of one system");
    if (n_sweeps < 0) return fail(CQ_EINVAL, "n_sweeps must be >= 0");
    HIP_TRY(hipStreamSynchronize(c->stream));
    for (void** p : {(void**)&c->rec_rho, (void**)&c->rec_dlnj, (void**)&c->rec_prob, (void**)&c->rec_acc,
                     (void**)&c->rec_rnew})
        if (*p) {
            HIP_TRY(hipFree(*p));
            *p = nullptr;
        }
    c->rec_cap = 0;
    if (n_sweeps > 0) {
        const size_t cnt = (size_t)n_sweeps * c->ne * c->Wcap;
        bool ok = hipMalloc((void**)&c->rec_rho, cnt * 8) == hipSuccess;
        ok = ok && hipMalloc((void**)&c->rec_dlnj, cnt * 8) == hipSuccess;
        ok = ok && hipMalloc((void**)&c->rec_prob, cnt * 8) == hipSuccess;
        ok = ok && hipMalloc((void**)&c->rec_acc, cnt) == hipSuccess;
        ok = ok && hipMalloc((void**)&c->rec_rnew, cnt * 24) == hipSuccess;
        if (!ok) {
            (void)hipGetLastError();
            return fail(CQ_ENOMEM, "record buffers");
        }
        // proposals are recorded by DMC moves only: the rest reads as NaN (all bits set)
        HIP_TRY(hipMemset(c->rec_rnew, 0xFF, cnt * 24));
        c->rec_cap = n_sweeps;
    }
    c->hp.rec_cap = c->rec_cap;
    c->hp.rec_sweep = 0;
    drop_graph(c);
    return push_params(c);
}

cq_status cq_crowd_get_move_records(cq_crowd* c, double* rho, double* dlnj, double* prob, uint8_t* acc)
{
    if (!c) return fail(CQ_EINVAL, "crowd is NULL");
    if (!c->subs.empty()) return fail(CQ_EINVAL, "parity mode works on crowds of one system");
    if (c->rec_cap == 0) return fail(CQ_ESTATE, "recording is off");
    const size_t cnt = (size_t)c->rec_cap * c->ne * c->Wcap;
    cq_status st = copy_out(c, rho, c->rec_rho, cnt * 8);
    if (st == CQ_OK) st = copy_out(c, dlnj, c->rec_dlnj, cnt * 8);
    if (st == CQ_OK) st = copy_out(c, prob, c->rec_prob, cnt * 8);
    if (st == CQ_OK) st = copy_out(c, acc, c->rec_acc, cnt);
    return got(c, st, "get_move_records");
}

cq_status cq_crowd_get_move_proposals(cq_crowd* c, double* rnew)
{
    if (!c || !rnew) return fail(CQ_EINVAL, "NULL argument");
    if (!c->subs.empty()) return fail(CQ_EINVAL, "parity mode works on crowds of one system");
    if (c->rec_cap == 0) return fail(CQ_ESTATE, "recording is off");
    const size_t cnt = (size_t)c->rec_cap * c->ne * c->Wcap;
    return got(c, copy_out(c, rnew, c->rec_rnew, cnt * 24), "get_move_proposals");
}

cq_status cq_crowd_set_kernel_timing(cq_crowd* c, int kind_mask)
{
    if (!c) return fail(CQ_EINVAL, "crowd is NULL");
    for (cq_crowd* sub : c->subs) {
        cq_status st = cq_crowd_set_kernel_timing(sub, kind_mask);
        if (st != CQ_OK) return st;
    }
    if (kind_mask < 0 || kind_mask >= (1 << CQ_KERNEL_COUNT)) return fail(CQ_EINVAL, "bad kernel kind mask");
    HIP_TRY(hipStreamSynchronize(c->stream));
    c->timing_mask = kind_mask;
    for (int k = 0; k < CQ_KERNEL_COUNT; ++k) c->ev_used[k] = 0;
    return CQ_OK;
}

cq_status cq_crowd_get_kernel_timing(cq_crowd* c, int kind, double* total_ms, int64_t* launches)
{
    if (!c) return fail(CQ_EINVAL, "crowd is NULL");
    if (kind < 0 || kind >= CQ_KERNEL_COUNT) return fail(CQ_EINVAL, "unknown kernel kind");
    HIP_TRY(hipStreamSynchronize(c->stream));
    double tot = 0.0;
    for (size_t i = 0; i < c->ev_used[kind]; ++i) {
        float ms = 0.0f;
        HIP_TRY(hipEventElapsedTime(&ms, c->ev[kind][i].first, c->ev[kind][i].second));
        tot += ms;
    }
    int64_t cnt = (int64_t)c->ev_used[kind];
    for (cq_crowd* sub : c->subs) {  // a group's per-system launches (energy, branching, recompute)
        double ms = 0.0;
        int64_t k = 0;
        cq_status st = cq_crowd_get_kernel_timing(sub, kind, &ms, &k);
        if (st != CQ_OK) return st;
        tot += ms;
        cnt += k;
    }
    if (total_ms) *total_ms = tot;
    if (launches) *launches = cnt;
    return CQ_OK;
}

}  // extern "C"

namespace cq {

cq_status report_error(cq_status s, const char* msg) { return fail(s, msg); }

// Workspace of one batched inversion of nmat n x n matrices: the blocked Gauss-Jordan buffers
// (n > 64 only), then the per-pair status words and per-matrix drift the kernels write.
size_t slater_work_bytes(int n, int nmat)
{
    const size_t pairs = ((size_t)nmat + 1) / 2;
    size_t b = cq::inverse_work_bytes(nmat, n);
    return ((b + 255) / 256) * 256 + pairs * sizeof(int) + (size_t)nmat * sizeof(double) + 256;
}

// The inversion proper on a caller-provided workspace of slater_work_bytes(n, nmat) bytes (256-byte
// aligned); no allocation on any path but the error message of a failure.
template <typename T>
cq_status slater_inverse_impl(const T* A, int n, int nmat, T* Minv, double* logdet, int* sign, hipStream_t st,
                              unsigned char* work)
{
    const int pairs = (nmat + 1) / 2;
    size_t off = 0;
    cq::InvWork wk{};
    if (n > 64) {
        const int B = cq::block_width(n);
        wk.S = (double*)(work + off);
        off += sizeof(double) * (size_t)nmat * n * cq::s_ld(n);
        wk.PR = (double*)(work + off);
        off += sizeof(double) * (size_t)nmat * B * n;
        wk.pivrow = (int*)(work + off);
        off += sizeof(int) * (size_t)nmat * n * 2;
        off = (off + 15) / 16 * 16;
        wk.logabs = (double*)(work + off);
        off += sizeof(double) * (size_t)nmat * 2;
        wk.negs = (int*)(work + off);
        off += sizeof(int) * (size_t)nmat * 2;
        wk.b = cq::panel_width(n);
    }
    off = (off + 255) / 256 * 256;
    int* status = (int*)(work + off);
    off += sizeof(int) * (size_t)pairs;
    off = (off + 15) / 16 * 16;
    double* drift = (double*)(work + off);
    cq::CrowdView<T> v{};
    v.W = pairs;
    v.n = n;
    v.ne = 2 * n;
    v.arow = n;
    v.VGL = const_cast<T*>(A);
    v.M = Minv;
    v.logdet = logdet;
    v.sign = sign;
    v.status = status;
    v.drift = drift;
    v.drift_max = nullptr;
    cq::launch_zero(status, sizeof(int) * (size_t)pairs, st);
    // the kernels read the previous log|det| for a drift figure that this call does not report
    cq::launch_zero(logdet, sizeof(double) * (size_t)nmat, st);
    cq::launch_inverse<T>(v, wk, st, nmat);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(st));
    int hs[256];
    for (int w0 = 0; w0 < pairs; w0 += 256) {
        const int cnt = pairs - w0 < 256 ? pairs - w0 : 256;
        HIP_TRY(hipMemcpy(hs, status + w0, sizeof(int) * (size_t)cnt, hipMemcpyDeviceToHost));
        for (int q = 0; q < cnt; ++q)
            if (hs[q] & 1) {
                const int w = w0 + q;
                return fail(CQ_ESINGULAR, "matrix " + std::to_string(2 * w) +
                                              (2 * w + 1 < nmat ? " or " + std::to_string(2 * w + 1) : std::string()) +
                                              " is singular or not finite");
            }
    }
    return CQ_OK;
}

template cq_status slater_inverse_impl<float>(const float*, int, int, float*, double*, int*, hipStream_t,
                                              unsigned char*);
template cq_status slater_inverse_impl<double>(const double*, int, int, double*, double*, int*, hipStream_t,
                                               unsigned char*);

cq_status check_slater_args(const void* A, int elem_bytes, int n, int nmat, const void* Minv, const double* logdet,
                            const int* sign)
{
    if (!A || !Minv || !logdet || !sign) return fail(CQ_EINVAL, "NULL argument");
    if (elem_bytes != 4 && elem_bytes != 8) return fail(CQ_EINVAL, "elem_bytes must be 4 or 8");
    if (n < 1 || n > 2048) return fail(CQ_EINVAL, "n must be 1..2048");
    if (nmat < 1) return fail(CQ_EINVAL, "nmat must be >= 1");
    if ((size_t)nmat * n * n > (size_t)1 << 34) return fail(CQ_EINVAL, "batch too large");
    return CQ_OK;
}

}  // namespace cq

extern "C" {

cq_status cq_slater_inverse(const void* A, int elem_bytes, int n, int nmat, void* Minv, double* logdet, int* sign,
                            void* hip_stream)
{
    cq_status st = cq::check_slater_args(A, elem_bytes, n, nmat, Minv, logdet, sign);
    if (st != CQ_OK) return st;
    void* work = nullptr;
    const size_t bytes = cq::slater_work_bytes(n, nmat);
    if (hipMalloc(&work, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return fail(CQ_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes of inversion workspace failed");
    }
    hipStream_t s = (hipStream_t)hip_stream;
    st = elem_bytes == 4 ? cq::slater_inverse_impl<float>((const float*)A, n, nmat, (float*)Minv, logdet, sign, s,
                                                      (unsigned char*)work)
                         : cq::slater_inverse_impl<double>((const double*)A, n, nmat, (double*)Minv, logdet, sign, s,
                                                       (unsigned char*)work);
    (void)hipStreamSynchronize(s);
    (void)hipFree(work);
    return st;
}

cq_status cq_device_copy(void* dst, const void* src, uint64_t bytes, void* hip_stream)
{
    if (!dst || !src || bytes % 16 || ((uintptr_t)dst | (uintptr_t)src) % 16)
        return fail(CQ_EINVAL, "copy needs 16-byte aligned pointers and a multiple of 16 bytes");
    cq::launch_copy(dst, src, (size_t)bytes, (hipStream_t)hip_stream);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize((hipStream_t)hip_stream));
    return CQ_OK;
}

cq_status cq_crowd_synchronize(cq_crowd* c)
{
    if (!c) return fail(CQ_EINVAL, "crowd is NULL");
    for (cq_crowd* sub : c->subs) {
        cq_status st = cq_crowd_synchronize(sub);
        if (st != CQ_OK) return st;
    }
    if (!c->subs.empty()) return CQ_OK;
    HIP_TRY(hipStreamSynchronize(c->stream));
    HIP_TRY(hipGetLastError());
    return check_singular(c, "synchronize");
}

}  // extern "C"
