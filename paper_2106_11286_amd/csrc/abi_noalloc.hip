// abi_noalloc.hip -- mc_measure_buffers_static: the from-scratch measurement
// of caller spin buffers with its partial sums in a static device array, for
// callers that cannot allocate (code under HIP graph capture, tight serving
// loops).  Host code and the array share this translation unit: the array has
// internal linkage, and its device address is looked up once per device.
#include <hip/hip_runtime.h>

#include <mutex>

#include "abi_internal.h"

using namespace mcabi;

namespace {

// FP64 partial sums of the measurement workgroups, [MEASURE_BLOCKS][8]
// (64 KiB).  Every GPU the library runs on holds its own copy until the
// process ends.  In host code this name is a host-side stand-in: only the
// address from hipGetSymbolAddress may reach a kernel or a copy.
static __device__ __align__(256) double scratch[MEASURE_BLOCKS * 8];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_scratch_dev[kMaxDevices]; // device address of `scratch`, per device

// The device address of this device's `scratch` (looked up on the first call
// on the device, with that device current).
mc_status scratch_address(void **out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        return fail(MC_E_DEVICE, "no current HIP device");
    }
    if (dev < 0 || dev >= kMaxDevices)
        return fail(MC_E_DEVICE, "device %d outside the %d the library tracks", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return fail(MC_E_DEVICE, "static scratch of device %d: %s", dev,
                        hipGetErrorString(e));
        }
        g_scratch_dev[dev] = p;
    }
    *out = g_scratch_dev[dev];
    return MC_OK;
}

} // namespace

extern "C" {

mc_status mc_measure_buffers_static(const mc_replica_desc *d, mc_precision prec,
                                    const mc_spin_buffers *bufs, double *record_dev,
                                    void *hip_stream)
{
    mc_status s = check_measure_args(d, prec, bufs, record_dev);
    if (s != MC_OK) return s;
    RepDev R;
    fill_repdev(*d, *bufs, R);
    const uint32_t blocks = measure_blocks(R);
    // every workgroup writes its own slots before the finishing workgroup
    // reads them, so nothing in the array needs clearing between calls
    if ((uint64_t)blocks * 8u * sizeof(double) > sizeof(scratch))
        return fail(MC_E_UNSUPPORTED, "measurement needs %llu bytes of partials, the static "
                                      "scratch holds %llu",
                    (unsigned long long)blocks * 8u * sizeof(double),
                    (unsigned long long)sizeof(scratch));
    void *ptr = nullptr;
    if ((s = scratch_address(&ptr)) != MC_OK) return s;
    const hipError_t e = launch_measure_direct(prec == MC_F64, d->kind, &R, (double *)ptr, blocks,
                                               0.0, record_dev, (hipStream_t)hip_stream);
    if (e != hipSuccess) return fail(MC_E_DEVICE, "measure launch: %s", hipGetErrorString(e));
    return MC_OK;
}

} // extern "C"
