// The no-allocation entry point: RK3 steps of Couette instances whose only device memory
// is the caller's state and a fixed scratch array of this library (for callers that
// cannot call hipMalloc).  The array is a file-scope device variable; its device address
// is taken once per device, with that device current, on the first call there, and only
// that address is handed to the copies and kernels (in host code the array's name is a
// host-side stand-in, not a device address).
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/vlb.h"

struct vlb_batch;

namespace vlb {
vlb_status set_error(vlb_status s, const char* fmt, ...);
vlb_status couette_noalloc_plan(int B, const vlb_couette_desc* descs, vlb_batch** out, size_t* bytes);
vlb_status couette_noalloc_run(vlb_batch* b, double* F, long nsteps, double* resid, hipStream_t stream,
                               char* scratch);
}  // namespace vlb

namespace {

constexpr size_t kScratchBytes = VLB_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

// stage buffers, moment sums, residual partials, tables, descriptors and block lists of
// one call; each GPU holds its own copy until the process ends
static __device__ __align__(256) char scratch[kScratchBytes];

std::mutex g_mu;
char* g_scratch[kMaxDevices] = {};

}  // namespace

extern "C" vlb_status vlb_couette_step_noalloc(int B, const vlb_couette_desc* descs, double* F, long nsteps,
                                               double* resid, void* hip_stream) {
    if (B < 1 || !descs || !F || nsteps < 1)
        return vlb::set_error(VLB_EINVAL, "need B >= 1, descriptors, a device state and nsteps >= 1");
    vlb_batch* b = nullptr;
    size_t need = 0;
    vlb_status st = vlb::couette_noalloc_plan(B, descs, &b, &need);
    if (st != VLB_OK) return st;
    if (need > kScratchBytes) {
        vlb_batch_destroy(b);
        return vlb::set_error(VLB_ENOMEM, "the instances need %zu bytes of device scratch; the no-allocation entry "
                              "point holds %zu", need, kScratchBytes);
    }
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        vlb_batch_destroy(b);
        return vlb::set_error(VLB_EDEVICE, "no usable current device (%s)", hipGetErrorString(e));
    }
    char* ptr = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_mu);
        if (!g_scratch[dev]) {
            void* p = nullptr;
            e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
            if (e != hipSuccess || !p) {
                vlb_batch_destroy(b);
                return vlb::set_error(VLB_EDEVICE, "hipGetSymbolAddress of the scratch array failed on device %d: %s",
                                      dev, hipGetErrorString(e));
            }
            g_scratch[dev] = static_cast<char*>(p);
        }
        ptr = g_scratch[dev];
    }
    st = vlb::couette_noalloc_run(b, F, nsteps, resid, static_cast<hipStream_t>(hip_stream), ptr);
    vlb_batch_destroy(b);
    return st;
}
