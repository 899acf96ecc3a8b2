// noalloc.hip -- lbm_step_record without any allocation, for callers that
// cannot allocate device memory (code under HIP graph capture, tight serving
// loops, harnesses that forbid hipMalloc).
//
// lbm_step_record keeps its per-step particle records in device memory the
// library allocates (and grows).  Here they go through `scratch`, a fixed
// array of LBM_NOALLOC_REC_DOUBLES doubles in the module's device data: each
// GPU the library runs on holds its own copy until the process ends.  Host
// code must never pass the symbol itself to a kernel (its host-side name is
// not a device address); the address comes from hipGetSymbolAddress, taken
// once per device on the first call there, with that device current, and
// kept in `g_scratch`.  Every context on one GPU shares that GPU's copy, so
// calls that overlap in time on one GPU race; the records of a call are
// fully written by its own steps before they are read, so nothing has to be
// cleared between calls.
#include <mutex>
#include <string>

#include "ctx.h"

using namespace lbm;

static __device__ __align__(256) double scratch[LBM_NOALLOC_REC_DOUBLES];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
double *g_scratch[MAX_DEVICES]; // device address of `scratch` per device; NULL until looked up

// The device address of this device's `scratch` (the device is current).
double *scratch_on(int device, hipError_t &e)
{
    e = hipSuccess;
    if (device < 0 || device >= MAX_DEVICES) {
        e = hipErrorInvalidDevice;
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch[device]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return nullptr;
        g_scratch[device] = (double *)ptr;
    }
    return g_scratch[device];
}

} // namespace

extern "C" int lbm_step_record_noalloc(lbm_ctx *c, int64_t nsteps, double *host_rec)
{
    if (!c) return LBM_EINVAL;
    if (nsteps < 0 || (nsteps > 0 && !host_rec)) return c->err = "bad arguments", LBM_EINVAL;
    const int64_t per_step = (int64_t)std::max(c->np, 1) * REC_STRIDE;
    if (nsteps > (int64_t)LBM_NOALLOC_REC_DOUBLES / per_step)
        return c->err = "nsteps x particles x 20 doubles exceed the static record array of " +
                        std::to_string(LBM_NOALLOC_REC_DOUBLES) + " doubles",
               LBM_EINVAL;
    if (c->prof) return c->err = "profiling creates events: switch it off for the no-allocation call", LBM_ESTATE;
    hipError_t e = hipSetDevice(c->device);
    double *rec = e == hipSuccess ? scratch_on(c->device, e) : nullptr;
    if (!rec) return c->err = std::string("static record array: ") + hipGetErrorString(e), LBM_EDEVICE;
    int rc = step_impl(c, nsteps, rec);
    if (rc) return rc;
    if (nsteps > 0 && c->np > 0) {
        // the 14 leading values of every 20-double record, straight into host_rec
        e = hipMemcpy2DAsync(host_rec, 14 * sizeof(double), rec, REC_STRIDE * sizeof(double), 14 * sizeof(double),
                             (size_t)nsteps * c->np, hipMemcpyDeviceToHost, c->stream);
        if (e != hipSuccess) return c->err = std::string("record copy: ") + hipGetErrorString(e), LBM_EDEVICE;
    }
    e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return c->err = std::string("hipStreamSynchronize: ") + hipGetErrorString(e), LBM_EDEVICE;
    return lbm_sync(c);
}
