// iblb_get_fields_noalloc: iblb_get_fields staged through a fixed device
// array instead of a buffer allocated per call.
#include "iblb.h"
#include "iblb_internal.h"

#include <hip/hip_runtime.h>

#include <mutex>

namespace {

constexpr long long kMaxNodes = IBLB_NOALLOC_MAX_NODES;
constexpr int kMaxDevices = 64;

// rho [n] then u [3][n] of the last call on this device.  Host code never
// uses this name for memory: it takes the device address that
// hipGetSymbolAddress gives for each device (scratch_at below).
static __device__ __align__(256) double scratch[4 * kMaxNodes];

std::mutex scratch_mu;
bool scratch_tried[kMaxDevices];
double *scratch_at[kMaxDevices];

double *scratch_of(int device)
{
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(scratch_mu);
    return scratch_at[device];
}

}  // namespace

namespace iblb {

void noalloc_setup(int device)
{
    if (device < 0 || device >= kMaxDevices) return;
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (scratch_tried[device]) return;
    scratch_tried[device] = true;
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) == hipSuccess && p)
        scratch_at[device] = (double *)p;
    else
        (void)hipGetLastError();  // leave no sticky error for the caller's next call
}

}  // namespace iblb

int iblb_get_fields_noalloc(iblb_ctx *c, double *rho, double *u)
{
    if (!c || !rho || !u) return IBLB_E_INVAL;
    const long long n = iblb::ctx_fluid_nodes(c);
    if (n > kMaxNodes)
        return iblb::ctx_fail(c, IBLB_E_INVAL,
                              "lattice has more fluid nodes than the allocation-free staging array holds "
                              "(IBLB_NOALLOC_MAX_NODES)");
    double *p = scratch_of(iblb::ctx_device(c));
    if (!p) return iblb::ctx_fail(c, IBLB_E_DEVICE, "allocation-free staging array not available on this device");
    return iblb::get_fields_staged(c, p, rho, u);
}
