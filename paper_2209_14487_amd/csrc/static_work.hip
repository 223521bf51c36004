// The batched FP64 Slater inverse on a workspace that the library holds in a
// file-scope device array, for callers that cannot allocate device memory.
//
// The array `scratch` exists once per GPU the library runs on and lives until the
// process ends.  Host code never passes the array's name to a kernel or a copy (in
// host code it names a host-side stand-in, not device memory): at the first call on
// a device, with that device current, its device address is looked up with
// hipGetSymbolAddress and kept per device, and only that address is used.
//
// Every call on one GPU shares that GPU's array, which keeps the previous call's
// contents; the inversion clears the words it needs (status, log|det|) with a fill
// kernel before use.  Calls that overlap on one GPU (from several host threads, or on
// several streams without ordering between them) race on the array.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "cq.h"
#include "cq_internal.h"

namespace {

constexpr size_t kStaticWorkBytes = (size_t)CQ_STATIC_WORK_BYTES;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kStaticWorkBytes];

std::mutex g_lookup;
void* g_work[kMaxDevices] = {};  // device address of `scratch` on each device, once looked up

// Device address of this device's array (looked up on the first call on the device).
cq_status work_address(void** out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return cq::report_error(CQ_EDEVICE, (std::string("hipGetDevice: ") + hipGetErrorString(e)).c_str());
    if (dev < 0 || dev >= kMaxDevices) return cq::report_error(CQ_EDEVICE, "device index out of range");
    std::lock_guard<std::mutex> lock(g_lookup);
    if (!g_work[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return cq::report_error(CQ_EDEVICE,
                                    (std::string("hipGetSymbolAddress of the static workspace: ") + hipGetErrorString(e)).c_str());
        g_work[dev] = p;
    }
    *out = g_work[dev];
    return CQ_OK;
}

}  // namespace

extern "C" {

cq_status cq_slater_inverse_static(const void* A, int elem_bytes, int n, int nmat, void* Minv, double* logdet,
                                   int* sign, void* hip_stream)
{
    cq_status st = cq::check_slater_args(A, elem_bytes, n, nmat, Minv, logdet, sign);
    if (st != CQ_OK) return st;
    const size_t need = cq::slater_work_bytes(n, nmat);
    if (need > kStaticWorkBytes)
        return cq::report_error(CQ_EINVAL, ("the inversion needs " + std::to_string(need) +
                                            " bytes of workspace, more than the static workspace's " +
                                            std::to_string(kStaticWorkBytes))
                                               .c_str());
    void* work = nullptr;
    st = work_address(&work);
    if (st != CQ_OK) return st;
    hipStream_t s = (hipStream_t)hip_stream;
    return elem_bytes == 4 ? cq::slater_inverse_impl<float>((const float*)A, n, nmat, (float*)Minv, logdet, sign, s,
                                                            (unsigned char*)work)
                           : cq::slater_inverse_impl<double>((const double*)A, n, nmat, (double*)Minv, logdet, sign,
                                                             s, (unsigned char*)work);
}

}  // extern "C"
