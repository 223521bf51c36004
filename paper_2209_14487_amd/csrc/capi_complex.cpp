// C ABI of the complex-orbital path: systems with a general cell, a twist and a complex
// B-spline table, and crowds of walkers moved by one sweep kernel per sweep (the VMC
// sweep of Alg. 1, every walker of the crowd at once, one workgroup per walker).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "cq.h"
#include "cq_complex.h"
#include "cq_host.h"

struct cq_csystem {
    int n = 0;
    double lat[9] = {}, linv[9] = {}, metric[6] = {}, k[3] = {};
    int G = 0, n_orb = 0;
    double2* table = nullptr;  // complex128 coefficients
    float2* table32 = nullptr;  // complex64 coefficients (a system may hold both, of one grid)
    bool owned = false, owned32 = false;
    int use_j2 = 0;
    double a_par = 0.0, a_anti = 0.0, b = 1.0;
};

struct cq_ccrowd {
    const cq_csystem* sys = nullptr;
    int W = 0, n = 0, ne = 0, prec = CQ_FP64;
    uint64_t seed = 0;
    uint32_t first_uid = 0, step = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false, ready = false;
    double* R = nullptr;
    double2* M = nullptr;
    double2* VGL = nullptr;
    double* logdet = nullptr;
    double* phase = nullptr;
    double2* eloc = nullptr;
    long long* nacc = nullptr;
    long long* nprop = nullptr;
    uint32_t* uid = nullptr;
    int* status = nullptr;
    double2* work = nullptr;
    int rec_cap = 0, rec_sweep = 0;
    double2* rec_rho = nullptr;
    double* rec_dlnj = nullptr;
    double* rec_prob = nullptr;
    uint8_t* rec_acc = nullptr;
    // HIP events around every sweep-kernel launch while timing is on
    bool timing = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
    size_t ev_used = 0;
};

namespace {

using cq::host_fail;

#define CHIP_TRY(x)                                                                                        \
    do {                                                                                                   \
        hipError_t e_ = (x);                                                                               \
        if (e_ != hipSuccess) return host_fail(CQ_EDEVICE, std::string(#x) + ": " + hipGetErrorString(e_)); \
    } while (0)

cq::CView cview(const cq_ccrowd* c)
{
    const cq_csystem* s = c->sys;
    cq::CView v{};
    v.W = c->W;
    v.n = c->n;
    v.ne = c->ne;
    v.G = s->G;
    v.n_orb = s->n_orb;
    std::memcpy(v.lat, s->lat, sizeof v.lat);
    std::memcpy(v.linv, s->linv, sizeof v.linv);
    std::memcpy(v.metric, s->metric, sizeof v.metric);
    std::memcpy(v.k, s->k, sizeof v.k);
    v.k2 = s->k[0] * s->k[0] + s->k[1] * s->k[1] + s->k[2] * s->k[2];
    v.table = c->prec == CQ_FP64 ? s->table : nullptr;
    v.table32 = c->prec == CQ_FP64 ? nullptr : s->table32;
    v.R = c->R;
    v.M = c->M;
    v.VGL = c->VGL;
    v.logdet = c->logdet;
    v.phase = c->phase;
    v.eloc = c->eloc;
    v.nacc = c->nacc;
    v.nprop = c->nprop;
    v.uid = c->uid;
    v.status = c->status;
    v.work = c->work;
    v.use_j2 = s->use_j2;
    v.a_par = s->a_par;
    v.a_anti = s->a_anti;
    v.b = s->b;
    v.seed = c->seed;
    v.step = c->step;
    v.rec_sweep = c->rec_sweep;
    v.rec_cap = c->rec_cap;
    v.rec_rho = c->rec_rho;
    v.rec_dlnj = c->rec_dlnj;
    v.rec_prob = c->rec_prob;
    v.rec_acc = c->rec_acc;
    return v;
}

cq_status launched(const char* what)
{
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? CQ_OK : host_fail(CQ_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

// Zero or non-finite pivots flagged by the inversion name the first such walker.
cq_status check_status(cq_ccrowd* c, const char* what)
{
    CHIP_TRY(hipStreamSynchronize(c->stream));
    std::vector<int> st(c->W);
    CHIP_TRY(hipMemcpy(st.data(), c->status, sizeof(int) * c->W, hipMemcpyDeviceToHost));
    for (int w = 0; w < c->W; ++w)
        if (st[w]) return host_fail(CQ_ESINGULAR, std::string(what) + ": walker " + std::to_string(w) +
                                                     " has a singular or non-finite Slater matrix");
    return CQ_OK;
}

void free_records(cq_ccrowd* c)
{
    for (void* p : {(void*)c->rec_rho, (void*)c->rec_dlnj, (void*)c->rec_prob, (void*)c->rec_acc})
        if (p) (void)hipFree(p);
    c->rec_rho = nullptr;
    c->rec_dlnj = c->rec_prob = nullptr;
    c->rec_acc = nullptr;
    c->rec_cap = c->rec_sweep = 0;
}

}  // namespace

extern "C" {

cq_status cq_csystem_create(int n, const double* lattice, const double* twist, cq_csystem** out)
{
    if (!out || !lattice) return host_fail(CQ_EINVAL, "NULL argument");
    *out = nullptr;
    if (n < 1 || n > cq::kCMaxN) return host_fail(CQ_EINVAL, "n must be 1.." + std::to_string(cq::kCMaxN));
    for (int i = 0; i < 9; ++i)
        if (!std::isfinite(lattice[i])) return host_fail(CQ_EINVAL, "lattice must be finite");
    double k[3] = {0.0, 0.0, 0.0};
    if (twist)
        for (int i = 0; i < 3; ++i) {
            if (!std::isfinite(twist[i])) return host_fail(CQ_EINVAL, "twist must be finite");
            k[i] = twist[i];
        }
    const double* L = lattice;
    // cofactors: L^-1 = adj(L) / det(L)
    const double c00 = L[4] * L[8] - L[5] * L[7], c01 = L[5] * L[6] - L[3] * L[8], c02 = L[3] * L[7] - L[4] * L[6];
    const double det = L[0] * c00 + L[1] * c01 + L[2] * c02;
    double scale = 0.0;
    for (int i = 0; i < 9; ++i) scale = std::fmax(scale, std::fabs(L[i]));
    if (!(std::fabs(det) > 1e-9 * scale * scale * scale)) return host_fail(CQ_EINVAL, "lattice vectors are degenerate");
    auto* s = new cq_csystem;
    s->n = n;
    std::memcpy(s->lat, L, sizeof s->lat);
    std::memcpy(s->k, k, sizeof s->k);
    double* Li = s->linv;
    Li[0] = c00 / det;
    Li[3] = c01 / det;
    Li[6] = c02 / det;
    Li[1] = (L[2] * L[7] - L[1] * L[8]) / det;
    Li[4] = (L[0] * L[8] - L[2] * L[6]) / det;
    Li[7] = (L[1] * L[6] - L[0] * L[7]) / det;
    Li[2] = (L[1] * L[5] - L[2] * L[4]) / det;
    Li[5] = (L[2] * L[3] - L[0] * L[5]) / det;
    Li[8] = (L[0] * L[4] - L[1] * L[3]) / det;
    // metric (L^-T L^-1)_ab = sum_c Li[c][a] Li[c][b]
    auto m = [&](int a, int b) { return Li[a] * Li[b] + Li[3 + a] * Li[3 + b] + Li[6 + a] * Li[6 + b]; };
    s->metric[0] = m(0, 0);
    s->metric[1] = m(1, 1);
    s->metric[2] = m(2, 2);
    s->metric[3] = m(0, 1);
    s->metric[4] = m(0, 2);
    s->metric[5] = m(1, 2);
    *out = s;
    return CQ_OK;
}

cq_status cq_csystem_load_bspline(cq_csystem* s, const void* coefs, int elem_bytes, int grid, int n_orb,
                                  int coefs_on_device)
{
    if (!s || !coefs) return host_fail(CQ_EINVAL, "NULL argument");
    if (elem_bytes != 8 && elem_bytes != 16) return host_fail(CQ_EINVAL, "elem_bytes must be 8 or 16");
    if (grid < 4 || grid > 1024) return host_fail(CQ_EINVAL, "grid must be 4..1024");
    if (n_orb != s->n) return host_fail(CQ_EINVAL, "n_orb must equal n");
    if ((s->table || s->table32) && grid != s->G) return host_fail(CQ_EINVAL, "both tables must share one grid");
    void** slot = elem_bytes == 16 ? (void**)&s->table : (void**)&s->table32;
    bool& owned = elem_bytes == 16 ? s->owned : s->owned32;
    if (owned && *slot) (void)hipFree(*slot);
    *slot = nullptr;
    owned = false;
    const size_t bytes = (size_t)elem_bytes * grid * grid * grid * n_orb;
    if (coefs_on_device) {
        *slot = const_cast<void*>(coefs);
    } else {
        if (hipMalloc(slot, bytes) != hipSuccess) {
            (void)hipGetLastError();
            *slot = nullptr;
            return host_fail(CQ_ENOMEM, "complex table");
        }
        owned = true;
        CHIP_TRY(hipMemcpy(*slot, coefs, bytes, hipMemcpyHostToDevice));
    }
    s->G = grid;
    s->n_orb = n_orb;
    return CQ_OK;
}

cq_status cq_csystem_load_pade_j2(cq_csystem* s, double a_par, double a_anti, double b)
{
    if (!s) return host_fail(CQ_EINVAL, "system is NULL");
    if (!std::isfinite(a_par) || !std::isfinite(a_anti) || !(b >= 0.0) || !std::isfinite(b))
        return host_fail(CQ_EINVAL, "Jastrow parameters must be finite, b >= 0");
    s->use_j2 = 1;
    s->a_par = a_par;
    s->a_anti = a_anti;
    s->b = b;
    return CQ_OK;
}

void cq_csystem_destroy(cq_csystem* s)
{
    if (!s) return;
    if (s->owned && s->table) (void)hipFree(s->table);
    if (s->owned32 && s->table32) (void)hipFree(s->table32);
    delete s;
}

void cq_ccrowd_destroy(cq_ccrowd* c)
{
    if (!c) return;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    free_records(c);
    for (auto& p : c->ev) {
        (void)hipEventDestroy(p.first);
        (void)hipEventDestroy(p.second);
    }
    for (void* p : {(void*)c->R, (void*)c->M, (void*)c->VGL, (void*)c->logdet, (void*)c->phase, (void*)c->eloc,
                    (void*)c->nacc, (void*)c->nprop, (void*)c->uid, (void*)c->status, (void*)c->work})
        if (p) (void)hipFree(p);
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

cq_status cq_ccrowd_create(const cq_csystem* s, int walkers, int precision, uint64_t seed, uint32_t first_uid,
                           void* hip_stream, cq_ccrowd** out)
{
    if (!s || !out) return host_fail(CQ_EINVAL, "NULL argument");
    *out = nullptr;
    if (walkers < 1) return host_fail(CQ_EINVAL, "walkers must be >= 1");
    if (precision != CQ_FP64 && precision != CQ_MIXED) return host_fail(CQ_EINVAL, "bad precision");
    if (precision == CQ_FP64 && !s->table) return host_fail(CQ_EINVAL, "the system has no complex128 table");
    if (precision == CQ_MIXED && !s->table32) return host_fail(CQ_EINVAL, "the system has no complex64 table");
    auto* c = new cq_ccrowd;
    c->sys = s;
    c->prec = precision;
    c->W = walkers;
    c->n = s->n;
    c->ne = 2 * s->n;
    c->seed = seed;
    c->first_uid = first_uid;
    if (hip_stream) {
        c->stream = (hipStream_t)hip_stream;
    } else {
        if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
            (void)hipGetLastError();
            c->stream = nullptr;
            delete c;
            return host_fail(CQ_EDEVICE, "hipStreamCreate failed");
        }
        c->own_stream = true;
    }
    const size_t W = walkers, n = c->n, ne = c->ne;
    struct {
        void** p;
        size_t bytes;
    } plan[] = {
        {(void**)&c->R, sizeof(double) * W * ne * 3},
        {(void**)&c->M, sizeof(double2) * W * 2 * n * n},
        {(void**)&c->VGL, sizeof(double2) * W * 2 * n * 5 * n},
        {(void**)&c->logdet, sizeof(double) * W * 2},
        {(void**)&c->phase, sizeof(double) * W * 2},
        {(void**)&c->eloc, sizeof(double2) * W},
        {(void**)&c->nacc, sizeof(long long) * W},
        {(void**)&c->nprop, sizeof(long long) * W},
        {(void**)&c->uid, sizeof(uint32_t) * W},
        {(void**)&c->status, sizeof(int) * W},
        {(void**)&c->work, sizeof(double2) * W * 2 * n * 2 * n},
    };
    for (auto& e : plan)
        if (hipMalloc(e.p, e.bytes) != hipSuccess) {
            (void)hipGetLastError();
            *e.p = nullptr;
            cq_ccrowd_destroy(c);
            return host_fail(CQ_ENOMEM, "complex crowd buffers");
        }
    std::vector<uint32_t> uids(W);
    for (size_t w = 0; w < W; ++w) uids[w] = first_uid + (uint32_t)w;
    if (hipMemcpy(c->uid, uids.data(), sizeof(uint32_t) * W, hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipGetLastError();
        cq_ccrowd_destroy(c);
        return host_fail(CQ_EDEVICE, "uid upload");
    }
    *out = c;
    return CQ_OK;
}

cq_status cq_ccrowd_set_positions(cq_ccrowd* c, const double* R, uint32_t first_step)
{
    if (!c || !R) return host_fail(CQ_EINVAL, "NULL argument");
    const size_t cnt = (size_t)c->W * c->ne * 3;
    for (size_t i = 0; i < cnt; ++i)
        if (!std::isfinite(R[i])) return host_fail(CQ_EINVAL, "positions must be finite");
    c->ready = false;
    CHIP_TRY(hipMemcpyAsync(c->R, R, sizeof(double) * cnt, hipMemcpyHostToDevice, c->stream));
    CHIP_TRY(hipMemsetAsync(c->status, 0, sizeof(int) * c->W, c->stream));
    CHIP_TRY(hipMemsetAsync(c->nacc, 0, sizeof(long long) * c->W, c->stream));
    CHIP_TRY(hipMemsetAsync(c->nprop, 0, sizeof(long long) * c->W, c->stream));
    c->step = first_step;
    const cq::CView v = cview(c);
    cq::launch_csetup_rows(v, c->stream);
    cq::launch_cinverse(v, c->stream);
    cq::launch_cenergy(v, c->stream);
    cq_status st = launched("complex set-up");
    if (st != CQ_OK) return st;
    st = check_status(c, "set_positions");
    if (st != CQ_OK) return st;
    c->ready = true;
    return CQ_OK;
}

cq_status cq_ccrowd_run_vmc(cq_ccrowd* c, int n_sweeps, double sigma)
{
    if (!c) return host_fail(CQ_EINVAL, "crowd is NULL");
    if (n_sweeps < 0 || !(sigma > 0.0) || !std::isfinite(sigma)) return host_fail(CQ_EINVAL, "bad n_sweeps or sigma");
    if (!c->ready) return host_fail(CQ_ESTATE, "set positions before running");
    for (int s = 0; s < n_sweeps; ++s) {
        cq::CView v = cview(c);
        v.sigma = sigma;
        std::pair<hipEvent_t, hipEvent_t>* e = nullptr;
        if (c->timing) {
            if (c->ev_used == c->ev.size()) {
                std::pair<hipEvent_t, hipEvent_t> p{};
                CHIP_TRY(hipEventCreate(&p.first));
                if (hipEventCreate(&p.second) != hipSuccess) {
                    (void)hipEventDestroy(p.first);
                    return host_fail(CQ_EDEVICE, "hipEventCreate failed");
                }
                c->ev.push_back(p);
            }
            e = &c->ev[c->ev_used++];
            CHIP_TRY(hipEventRecord(e->first, c->stream));
        }
        cq::launch_csweep(v, c->stream);
        if (e) CHIP_TRY(hipEventRecord(e->second, c->stream));
        cq::launch_cenergy(v, c->stream);
        c->step += 1;
        c->rec_sweep += 1;
    }
    return launched("complex sweep");
}

cq_status cq_ccrowd_recompute(cq_ccrowd* c, double* max_drift)
{
    if (!c) return host_fail(CQ_EINVAL, "crowd is NULL");
    if (!c->ready) return host_fail(CQ_ESTATE, "set positions first");
    std::vector<double> before(2 * (size_t)c->W), after(2 * (size_t)c->W);
    CHIP_TRY(hipStreamSynchronize(c->stream));
    CHIP_TRY(hipMemcpy(before.data(), c->logdet, sizeof(double) * 2 * c->W, hipMemcpyDeviceToHost));
    const cq::CView v = cview(c);
    cq::launch_cinverse(v, c->stream);
    cq::launch_cenergy(v, c->stream);
    cq_status st = launched("complex recompute");
    if (st != CQ_OK) return st;
    st = check_status(c, "recompute");
    if (st != CQ_OK) return st;
    CHIP_TRY(hipMemcpy(after.data(), c->logdet, sizeof(double) * 2 * c->W, hipMemcpyDeviceToHost));
    double d = 0.0;
    for (size_t i = 0; i < before.size(); ++i) d = std::fmax(d, std::fabs(before[i] - after[i]));
    if (max_drift) *max_drift = d;
    return CQ_OK;
}

cq_status cq_ccrowd_get_logdet(cq_ccrowd* c, double* logdet, double* phase)
{
    if (!c || !logdet || !phase) return host_fail(CQ_EINVAL, "NULL argument");
    CHIP_TRY(hipStreamSynchronize(c->stream));
    CHIP_TRY(hipMemcpy(logdet, c->logdet, sizeof(double) * 2 * c->W, hipMemcpyDeviceToHost));
    CHIP_TRY(hipMemcpy(phase, c->phase, sizeof(double) * 2 * c->W, hipMemcpyDeviceToHost));
    return CQ_OK;
}

cq_status cq_ccrowd_get_local_energy(cq_ccrowd* c, double* el)
{
    if (!c || !el) return host_fail(CQ_EINVAL, "NULL argument");
    CHIP_TRY(hipStreamSynchronize(c->stream));
    CHIP_TRY(hipMemcpy(el, c->eloc, sizeof(double2) * c->W, hipMemcpyDeviceToHost));
    return CQ_OK;
}

cq_status cq_ccrowd_get_positions(cq_ccrowd* c, double* R)
{
    if (!c || !R) return host_fail(CQ_EINVAL, "NULL argument");
    CHIP_TRY(hipStreamSynchronize(c->stream));
    CHIP_TRY(hipMemcpy(R, c->R, sizeof(double) * (size_t)c->W * c->ne * 3, hipMemcpyDeviceToHost));
    return CQ_OK;
}

cq_status cq_ccrowd_get_acceptance(cq_ccrowd* c, int64_t* accepted, int64_t* proposed)
{
    if (!c || !accepted || !proposed) return host_fail(CQ_EINVAL, "NULL argument");
    CHIP_TRY(hipStreamSynchronize(c->stream));
    CHIP_TRY(hipMemcpy(accepted, c->nacc, sizeof(long long) * c->W, hipMemcpyDeviceToHost));
    CHIP_TRY(hipMemcpy(proposed, c->nprop, sizeof(long long) * c->W, hipMemcpyDeviceToHost));
    return CQ_OK;
}

cq_status cq_ccrowd_get_inverse(cq_ccrowd* c, int walker, int spin, double* out)
{
    if (!c || !out) return host_fail(CQ_EINVAL, "NULL argument");
    if (walker < 0 || walker >= c->W || spin < 0 || spin > 1) return host_fail(CQ_EINVAL, "bad walker or spin");
    const size_t n = c->n;
    std::vector<double2> m(n * n);
    CHIP_TRY(hipStreamSynchronize(c->stream));
    CHIP_TRY(hipMemcpy(m.data(), c->M + ((size_t)walker * 2 + spin) * n * n, sizeof(double2) * n * n,
                       hipMemcpyDeviceToHost));
    for (size_t a = 0; a < n; ++a)  // (A^-1)[j][a] = M[a][j]
        for (size_t j = 0; j < n; ++j) {
            out[2 * (j * n + a)] = m[a * n + j].x;
            out[2 * (j * n + a) + 1] = m[a * n + j].y;
        }
    return CQ_OK;
}

cq_status cq_ccrowd_record_moves(cq_ccrowd* c, int n_sweeps)
{
    if (!c) return host_fail(CQ_EINVAL, "crowd is NULL");
    if (n_sweeps < 0) return host_fail(CQ_EINVAL, "n_sweeps must be >= 0");
    CHIP_TRY(hipStreamSynchronize(c->stream));
    free_records(c);
    if (n_sweeps == 0) return CQ_OK;
    const size_t cnt = (size_t)n_sweeps * c->ne * c->W;
    bool ok = hipMalloc((void**)&c->rec_rho, cnt * sizeof(double2)) == hipSuccess;
    ok = ok && hipMalloc((void**)&c->rec_dlnj, cnt * 8) == hipSuccess;
    ok = ok && hipMalloc((void**)&c->rec_prob, cnt * 8) == hipSuccess;
    ok = ok && hipMalloc((void**)&c->rec_acc, cnt) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        free_records(c);
        return host_fail(CQ_ENOMEM, "record buffers");
    }
    c->rec_cap = n_sweeps;
    c->rec_sweep = 0;
    return CQ_OK;
}

cq_status cq_ccrowd_get_move_records(cq_ccrowd* c, double* rho, double* dlnj, double* prob, uint8_t* acc)
{
    if (!c || !rho || !dlnj || !prob || !acc) return host_fail(CQ_EINVAL, "NULL argument");
    if (!c->rec_cap) return host_fail(CQ_ESTATE, "recording is off");
    const size_t cnt = (size_t)c->rec_cap * c->ne * c->W;
    CHIP_TRY(hipStreamSynchronize(c->stream));
    CHIP_TRY(hipMemcpy(rho, c->rec_rho, cnt * sizeof(double2), hipMemcpyDeviceToHost));
    CHIP_TRY(hipMemcpy(dlnj, c->rec_dlnj, cnt * 8, hipMemcpyDeviceToHost));
    CHIP_TRY(hipMemcpy(prob, c->rec_prob, cnt * 8, hipMemcpyDeviceToHost));
    CHIP_TRY(hipMemcpy(acc, c->rec_acc, cnt, hipMemcpyDeviceToHost));
    return CQ_OK;
}

cq_status cq_ccrowd_set_timing(cq_ccrowd* c, int on)
{
    if (!c) return host_fail(CQ_EINVAL, "crowd is NULL");
    c->timing = on != 0;
    c->ev_used = 0;
    return CQ_OK;
}

cq_status cq_ccrowd_get_timing(cq_ccrowd* c, double* ms, int64_t* launches)
{
    if (!c || !ms || !launches) return host_fail(CQ_EINVAL, "NULL argument");
    CHIP_TRY(hipStreamSynchronize(c->stream));
    double t = 0.0;
    for (size_t i = 0; i < c->ev_used; ++i) {
        float x = 0.0f;
        CHIP_TRY(hipEventElapsedTime(&x, c->ev[i].first, c->ev[i].second));
        t += x;
    }
    *ms = t;
    *launches = (int64_t)c->ev_used;
    c->ev_used = 0;
    return CQ_OK;
}

cq_status cq_ccrowd_synchronize(cq_ccrowd* c)
{
    if (!c) return host_fail(CQ_EINVAL, "crowd is NULL");
    CHIP_TRY(hipStreamSynchronize(c->stream));
    return CQ_OK;
}

}  // extern "C"
