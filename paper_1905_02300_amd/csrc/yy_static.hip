// yy_static.hip -- yy_step_static: the time step of yy_step for callers
// that cannot allocate device memory (code under HIP graph capture, tight
// serving loops, harnesses that forbid allocation).  The step's scratch
// arrays -- the residual/correction buffer, the Thomas scratch, the norm
// partial sums and the mass-flux partials -- live in one file-scope static
// device array instead of the caller's workspace, so a grid whose scratch
// fits the array steps without any allocation by the library or the
// caller beyond the shell's own state.
#include <mutex>

#include "../../include/yy.h"
#include "yy_internal.h"

using namespace yy;

// One copy per GPU the library runs on, held until the process ends.
static __device__ __align__(256) double scratch[STATIC_SCRATCH_BYTES / 8];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex scratch_mu;
char *scratch_ptr[MAX_DEVICES];      // device address of `scratch` per device

// Device address of the static scratch on the current device, looked up
// once per device (with that device current).  In host code the name
// `scratch` is only a host-side handle; kernels get this address.
int scratch_on_current(char **out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) return YY_ERR_HIP;
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_ptr[dev]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return YY_ERR_HIP;
        scratch_ptr[dev] = (char *)ptr;
    }
    *out = scratch_ptr[dev];
    return YY_OK;
}

}  // namespace

extern "C" int yy_step_static(yy_shell *s, int32_t n_schwarz, hipStream_t stream)
{
    if (!s || n_schwarz < 1 || n_schwarz > 64) return YY_ERR_ARG;
    char *ptr = nullptr;
    const int rc = scratch_on_current(&ptr);
    if (rc != YY_OK) return rc;
    return step_with_scratch(s, n_schwarz, ptr, STATIC_SCRATCH_BYTES, stream);
}
