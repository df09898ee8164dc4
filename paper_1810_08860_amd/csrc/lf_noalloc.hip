// Allocation-free render entry point (lf_render_noalloc, include/lf.h).
//
// lf_render keeps its per-launch scratch -- the per-(eye, view) records of
// the set-up kernel, the per-tile candidate lists and counts of the culling
// kernel -- in a context buffer grown with hipMalloc. Callers that may not
// allocate (code under stream capture, tight serving loops) use this variant:
// the same kernels, with that scratch in a fixed file-scope device array of
// kScratchBytes, one copy per GPU the library runs on, held until the process
// ends. Host code never passes the array's name to a kernel (in host code it
// is a stand-in, not a device address): the device address of each GPU's
// copy is looked up once per device with hipGetSymbolAddress and kept.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/lf.h"
#include "lf_internal.h"

namespace {

// 16 MiB: a stereo pair of 2160 x 2160 eyes (36,450 tiles of 16 x 16 at
// 260 bytes each, plus 2 x 1024 eye-view records of 96 bytes) needs 9.2 MiB.
constexpr size_t kScratchBytes = (size_t)16 << 20;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) char scratch[kScratchBytes];

std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};

// Device address of the current device's copy of `scratch` (looked up once
// per device, with that device current).
int scratch_ptr(int dev, void **out) {
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            char msg[256];
            snprintf(msg, sizeof msg, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
            return lf::fail_msg(LF_EHIP, msg);
        }
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return LF_OK;
}

}  // namespace

extern "C" {

int lf_render_noalloc(lf_ctx *c, const lf_eye *eyes, int32_t n_eyes, double hfov_deg, const int32_t *res,
                      float *out_rgb, float *out_wsum, uint8_t *out_count, void *hip_stream) {
    if (!c) return lf::fail_msg(LF_EINVAL, "NULL context");
    int dev = -1, ctx_dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
        return lf::fail_msg(LF_EHIP, "no current HIP device (or device index beyond 63)");
    ctx_dev = lf::ctx_device(c);
    if (dev != ctx_dev) return lf::fail_msg(LF_EINVAL, "the current device is not the context's device");
    void *p = nullptr;
    const int rc = scratch_ptr(dev, &p);
    if (rc) return rc;
    return lf::render_fixed_scratch(c, eyes, n_eyes, hfov_deg, res, out_rgb, out_wsum, out_count, p, kScratchBytes,
                                    (hipStream_t)hip_stream);
}

}  // extern "C"
