// frkc2_step_noalloc: frkc2_step for callers that cannot allocate device
// memory (code under HIP graph capture, tight serving loops, harnesses that
// forbid hipMalloc). The workspace frkc2_step takes from the caller (two
// complex state buffers, reduction partials and the stepsize table) comes
// instead from a file-scope device array of fixed size, one per GPU, held
// until the process ends.
//
// In host code the array's name is a host-side stand-in, not a device
// address, so it is never passed to a kernel or a copy: the device address is
// taken once per device with hipGetSymbolAddress (with that device current)
// and kept per device.
#include <hip/hip_runtime.h>

#include <mutex>

#include "internal.h"

namespace frkc2 {
namespace {

constexpr int kMaxDevices = 64;

// 2 x 32 MiB of complex state (2^21 values) plus the 64 KiB of partials and
// stepsizes a workspace of frkc2_step carries.
constexpr size_t kNoAllocBytes = (size_t)FRKC2_NOALLOC_MAX_VALUES * 32 + ((size_t)64 << 10);

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};

// Device address of this device's copy of the array (looked up on the first
// call on the device).
int scratch_ptr(void **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        set_error("frkc2_step_noalloc: hipGetDevice: HIP error %d (%s)", (int)e,
                  hipGetErrorString(e));
        return FRKC2_EHIP;
    }
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("frkc2_step_noalloc: device %d beyond the %d the library tracks", dev,
                  kMaxDevices);
        return FRKC2_EINVAL;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            set_error("frkc2_step_noalloc: hipGetSymbolAddress: HIP error %d (%s)", (int)e,
                      hipGetErrorString(e));
            return FRKC2_EHIP;
        }
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return FRKC2_OK;
}

}  // namespace
}  // namespace frkc2

using namespace frkc2;

extern "C" int frkc2_step_noalloc(const frkc2_grid *g, double *w, const double *D, double T,
                                  double cfl, int s, double nu, int nsteps, hipStream_t st,
                                  frkc2_step_stats *stats)
{
    KGrid kg;
    const int vrc = step_validate(g, w, D, T, cfl, s, nu, nsteps, kg);
    if (vrc < 0) return vrc;
    const size_t need = step_workspace_bytes(kg.nstate());
    if (need > kNoAllocBytes) {
        set_error("frkc2_step_noalloc: a state of %lld values needs %zu bytes of scratch; the "
                  "static scratch holds %zu (at most %lld values)",
                  kg.nstate(), need, kNoAllocBytes, (long long)FRKC2_NOALLOC_MAX_VALUES);
        return FRKC2_ENOMEM;
    }
    void *ws = nullptr;
    const int rc = scratch_ptr(&ws);
    if (rc < 0) return rc;
    return step_core(g, w, D, T, cfl, s, nu, nsteps, ws, kNoAllocBytes, st, stats);
}
