// Allocation-free form of the batched SCV call: the same kernels and launch
// order as kdefft_scv_batch, with the workspace (per-candidate parameter
// blocks and per-item partial sums) taken from a fixed device array instead
// of a caller buffer.
//
// The array is a file-scope __device__ variable: each GPU the library runs on
// holds its own copy for the rest of the process.  In host code its name is
// not a device address, so the address is looked up once per device with
// hipGetSymbolAddress (with that device current) and only that address is
// handed to the kernels.
#include <hip/hip_runtime.h>

#include <mutex>

#include "internal.h"

static __device__ __align__(256) unsigned char scratch[KDEFFT_NOALLOC_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};

// Device address of this device's scratch array (looked up on first use).
int scratch_for_current_device(void** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return kdefft::set_error(KDEFFT_E_HIP, hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return kdefft::set_error(KDEFFT_E_HIP, "device index out of range");
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return kdefft::set_error(KDEFFT_E_HIP, e != hipSuccess ? hipGetErrorString(e) : "scratch address is NULL");
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return KDEFFT_OK;
}

}  // namespace

extern "C" int kdefft_scv_batch_noalloc(const kdefft_dataset* ds_host, int n_ds, const int64_t* h_offsets_host,
                                        const double* vechL, double* obj, double* grad, int32_t* status,
                                        void* stream) {
    if (!obj) return kdefft::set_error(KDEFFT_E_ARG, "obj is NULL");
    size_t need = 0;
    int rc = kdefft::scv_batch_ws_need(ds_host, n_ds, h_offsets_host, &need);
    if (rc) return rc;
    if (need > (size_t)KDEFFT_NOALLOC_BYTES)
        return kdefft::set_error(KDEFFT_E_WORKSPACE,
                                 "batch needs more workspace than the fixed scratch of KDEFFT_NOALLOC_BYTES bytes "
                                 "(fewer candidates per call, or kdefft_scv_batch with a caller workspace)");
    void* ws = nullptr;
    rc = scratch_for_current_device(&ws);
    if (rc) return rc;
    return kdefft_scv_batch(ds_host, n_ds, h_offsets_host, vechL, obj, grad, status, ws,
                            (size_t)KDEFFT_NOALLOC_BYTES, stream);
}
