// <Z_q> readout that allocates nothing: for callers that cannot allocate
// device memory (code under HIP graph capture, tight serving loops).  The
// partial sums live in one fixed device array per GPU instead of the
// handle's growable scratch buffer.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/qops.h"
#include "kernels.hpp"
#include "runtime.hpp"

using namespace qops;

// 2^11 partial records of at most 35 doubles plus the 35 final sums (n <= 34),
// rounded up: 576 KiB per GPU, held until the process ends.
#define QOPS_NOALLOC_SCRATCH_DOUBLES (72 * 1024)

static __device__ __align__(256) double scratch[QOPS_NOALLOC_SCRATCH_DOUBLES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_dev[kMaxDevices] = {};   // device address of `scratch` on each GPU

// Device address of this GPU's copy of `scratch`, looked up once per device
// with that device current.  The host-side name `scratch` is only a stand-in
// for the symbol and must never be passed to a kernel or a copy.
int32_t scratch_address(int device, double** out)
{
    if (device < 0 || device >= kMaxDevices) return set_error(QOPS_UNSUPPORTED, "device index beyond 63");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[device]) {
        int cur = 0;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
        if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return hip_fail(e, "hipSetDevice");
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != device) (void)hipSetDevice(cur);
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p) return set_error(QOPS_HIP_ERROR, "hipGetSymbolAddress(scratch) returned null");
        g_scratch_dev[device] = static_cast<double*>(p);
    }
    *out = g_scratch_dev[device];
    return QOPS_OK;
}

}  // namespace

extern "C" int32_t qops_expect_z_noalloc(qops_sim* h, double* out_dev)
{
    if (!h || !out_dev) return set_error(QOPS_INVALID_ARG, "null argument");
    const size_t need = zsum_bounded_scratch_doubles(h->n);
    if (need > QOPS_NOALLOC_SCRATCH_DOUBLES)
        return set_error(QOPS_UNSUPPORTED, "state too large for the fixed readout scratch");
    double* sc = nullptr;
    int32_t rc = scratch_address(h->device, &sc);
    if (rc) return rc;
    hipError_t e = launch_expect_z_bounded(h->prec, h->state, h->n, h->l2p.data(), sc, out_dev, h->stream);
    if (e != hipSuccess) return hip_fail(e, "expect_z_noalloc");
    return QOPS_OK;
}
