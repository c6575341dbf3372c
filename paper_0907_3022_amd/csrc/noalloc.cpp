// Allocation-free region sum: the transmission-type observable of Sect. 3.1
// (sum of |psi_i|^2 over a masked region) for callers that cannot allocate
// device memory, e.g. inside a captured HIP graph or a serving loop.  The
// per-block partial sums live in a fixed device array of this file instead
// of a context's scratch buffer; the kernels are those of chebtd_region_sum,
// so both give bit-identical results.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <string>

#include "internal.h"

namespace chebtd {
int fail(Ctx *c, int code, const std::string &msg);
}  // namespace chebtd

using namespace chebtd;

namespace {

// Result pair first, then two doubles per block of the region kernel.
constexpr int64_t kResultDoubles = 32;  // 256 B, keeps the partials aligned
constexpr int64_t kMaxBlocks = kReduceBlocks;  // reduce_blocks(n) <= kReduceBlocks for every n
constexpr int64_t kScratchDoubles = kResultDoubles + 2 * kMaxBlocks;

// One copy per GPU, held until the process ends.  Host code never passes
// this name to a kernel: it is a host-side stand-in, not a device address.
static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
double *g_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per
// device; null (and *err set) if the lookup fails.
double *scratch_on_current_device(hipError_t *err)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        *err = e;
        return nullptr;
    }
    if (dev < 0 || dev >= kMaxDevices) {
        *err = hipErrorInvalidDevice;
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            *err = e != hipSuccess ? e : hipErrorInvalidSymbol;
            return nullptr;
        }
        g_ptr[dev] = static_cast<double *>(p);
    }
    return g_ptr[dev];
}

}  // namespace

extern "C" {

int chebtd_region_sum_noalloc(const double *psi_dev, const uint8_t *mask_dev, int64_t n, double *out_dev,
                              void *hip_stream)
{
    if (!psi_dev || !mask_dev || !out_dev)
        return fail(nullptr, CHEBTD_E_ARG, "chebtd_region_sum_noalloc: null pointer");
    if (n < 1 || n > CHEBTD_NOALLOC_MAX_SITES)
        return fail(nullptr, CHEBTD_E_ARG,
                    "chebtd_region_sum_noalloc: n = " + std::to_string(n) + " outside [1, " +
                        std::to_string((long long)CHEBTD_NOALLOC_MAX_SITES) + "]");
    hipError_t e = hipSuccess;
    double *base = scratch_on_current_device(&e);
    if (!base)
        return fail(nullptr, CHEBTD_E_HIP,
                    std::string("chebtd_region_sum_noalloc: device scratch lookup: ") + hipGetErrorString(e));
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    // every block writes its partial pair before the final sum reads it, and
    // the final sum writes both result doubles: nothing needs clearing
    double *res = base, *partials = base + kResultDoubles;
    e = launch_region(s, reinterpret_cast<const double2 *>(psi_dev), mask_dev, n, partials, res);
    if (e == hipSuccess) e = hipMemcpyAsync(out_dev, res, sizeof(double), hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess)
        return fail(nullptr, CHEBTD_E_HIP,
                    std::string("chebtd_region_sum_noalloc: ") + hipGetErrorString(e));
    return CHEBTD_OK;
}

}  // extern "C"
