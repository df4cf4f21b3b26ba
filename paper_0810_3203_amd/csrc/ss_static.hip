// zx_mul_ss_static: the Schoenhage-Strassen product of zx_mul_ss (Sect. 5.1)
// run from a fixed device array instead of a caller workspace, for callers
// that may not allocate device memory.  The array holds the product's two
// cell arrays and the descriptors of its three transform plans; the kernels
// are those of zx_mul_ss.  Each device the library runs on holds one copy of
// the array for the life of the process; calls that overlap on one device
// share it and race.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <mutex>

#include "../../include/tft.h"
#include "kernels.hpp"
#include "ss.hpp"

namespace {

static __device__ __align__(256) unsigned char scratch[TFT_STATIC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};

// Device address of the current device's copy of scratch, looked up once per
// device with that device current.
int scratch_ptr(void **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return tft::device_error(e, "zx_mul_ss_static: hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return tft::set_error(TFT_E_UNSUPPORTED, "zx_mul_ss_static: device index");
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return tft::device_error(e, "zx_mul_ss_static: hipGetSymbolAddress");
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return TFT_OK;
}

}  // namespace

extern "C" int zx_mul_ss_static(const uint32_t *g, uint64_t len_g, uint32_t g_limbs, const uint32_t *h,
                                uint64_t len_h, uint32_t h_limbs, uint32_t *out, uint32_t out_limbs,
                                const tft_ss_params *params, void *stream) {
    if (!g || !h || !out) return TFT_E_ARG;
    uint64_t need = 0;
    int st = tft::ss_scratch_bytes(len_g, g_limbs, len_h, h_limbs, out_limbs, params, &need);
    if (st) return st;
    if (need > TFT_STATIC_SCRATCH_BYTES) {
        char msg[160];
        std::snprintf(msg, sizeof msg, "zx_mul_ss_static: needs %llu bytes of scratch, the limit is %llu",
                      (unsigned long long)need, (unsigned long long)TFT_STATIC_SCRATCH_BYTES);
        return tft::set_error(TFT_E_WORKSPACE, msg);
    }
    void *p = nullptr;
    st = scratch_ptr(&p);
    if (st) return st;
    return tft::ss_scratch_run(g, len_g, g_limbs, h, len_h, h_limbs, out, out_limbs, params, p,
                               TFT_STATIC_SCRATCH_BYTES, static_cast<hipStream_t>(stream));
}
