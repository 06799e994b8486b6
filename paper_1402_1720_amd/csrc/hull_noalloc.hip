// hull_fbp_noalloc: the FDK hull with its workspace in a fixed device array
// of the library, for callers that cannot allocate device memory or pass a
// workspace (code under stream capture, tight serving loops, harnesses that
// forbid allocation). The kernels are those of hull_fbp; only where the bin
// sums, counts, filtered projections, per-angle trig and backprojection
// footprints live differs.
//
// Each device that runs the library holds its own copy of the array for the
// life of the process. In host code `scratch` names a host-side stand-in, not
// device memory: its device address is looked up once per device with
// hipGetSymbolAddress (with that device current) and only that address is
// handed to kernels.
#include <hip/hip_runtime.h>

#include <mutex>

#include "hull_runtime.h"
#include "hullmi.h"

namespace hullmi {
namespace {

static __device__ __align__(256) unsigned char scratch[HULLMI_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's copy of `scratch`.
int scratch_on_current_device(void **out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        (void)hipGetLastError();
        return HULL_EDEVICE;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
            (void)hipGetLastError();
            return HULL_EDEVICE;
        }
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return HULL_OK;
}

}  // namespace
}  // namespace hullmi

using namespace hullmi;

extern "C" {

int hull_fbp_noalloc(const hullmi_histories *hist, const hullmi_grid *grid,
                     const hullmi_fbp_params *fbp, float *image, uint8_t *mask, void *stream)
{
    if (!hist || !grid || !fbp) return HULL_EINVAL;
    hullmi_job j{};
    j.op = HULL_OP_FBP;
    j.hist = *hist;
    j.grid = *grid;
    j.fbp = *fbp;
    j.image = image;
    j.fbp_mask = mask;
    if (job_check(j) != HULL_OK) return HULL_EINVAL;
    const size_t need = job_ws_bytes(j);
    if (need == (size_t)-1 || need > (size_t)HULLMI_NOALLOC_SCRATCH_BYTES) return HULL_EINVAL;
    void *ws = nullptr;
    const int rc = scratch_on_current_device(&ws);
    if (rc != HULL_OK) return rc;
    return job_run(j, ws, (size_t)HULLMI_NOALLOC_SCRATCH_BYTES, reinterpret_cast<hipStream_t>(stream),
                   CountOpts{});
}

}  // extern "C"
