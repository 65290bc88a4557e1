// kernels_fused.hip -- the fused simple-cubic sweep (kernel 9) and the swap of
// the two state buffer sets that follows each of its launches.
#include <mutex>

#include "launch.hpp"
#include "sc_fused.hpp"

namespace mc {

// 1024 threads only for one FP32 position per lane (128 registers)
template <typename T, bool MEASURE, int PP>
__global__ void __launch_bounds__((PP == 1 && sizeof(T) == 4) ? 1024 : 512) k_sc_fused(PassLaunch P)
{
    uint32_t item;
    if (!logical_item(P, item)) return;
    sc_fused_body<T, MEASURE, PP>(P, item, *P.tctr_dev + P.t_off);
}

// After a fused sweep the second buffer set holds the current state.
__global__ void __launch_bounds__(64) k_swap_state(RepDev *reps, uint32_t n)
{
    const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    RepDev &R = reps[r];
    void *a = R.sx, *b = R.sy, *c = R.sz;
    R.sx = R.ax;
    R.sy = R.ay;
    R.sz = R.az;
    R.ax = a;
    R.ay = b;
    R.az = c;
}

// FP32: one to three positions per lane; FP64: one (more would not fit 256
// registers, checked on the host)
template <typename T, bool MEASURE>
static hipError_t fused_dispatch(const PassLaunch &p, hipStream_t st)
{
    const dim3 g(((p.n_blocks + 7u) >> 3) << 3), b((unsigned)p.tile.tx);
    switch (p.lds_positions) {
    case 1: hipLaunchKernelGGL((k_sc_fused<T, MEASURE, 1>), g, b, p.lds_bytes, st, p); break;
    case 2:
        if constexpr (sizeof(T) == 4) {
            hipLaunchKernelGGL((k_sc_fused<T, MEASURE, 2>), g, b, p.lds_bytes, st, p);
            break;
        } else {
            return hipErrorInvalidValue;
        }
    case 3:
        if constexpr (sizeof(T) == 4) {
            hipLaunchKernelGGL((k_sc_fused<T, MEASURE, 3>), g, b, p.lds_bytes, st, p);
            break;
        } else {
            return hipErrorInvalidValue;
        }
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_fused(bool f64, bool measure, const PassLaunch &p, hipStream_t st)
{
    if (p.n_blocks == 0) return hipSuccess;
    if ((p.tile.tx != 256 && p.tile.tx != 512 && p.tile.tx != 1024) || p.tile.ty < 1 ||
        (p.tile.tx == 1024 && (p.lds_positions != 1 || f64)) || (f64 && p.lds_positions != 1))
        return hipErrorInvalidValue;
    if (f64)
        return measure ? fused_dispatch<double, true>(p, st) : fused_dispatch<double, false>(p, st);
    return measure ? fused_dispatch<float, true>(p, st) : fused_dispatch<float, false>(p, st);
}

hipError_t launch_swap_state(RepDev *reps_dev, uint32_t n_reps, hipStream_t st)
{
    hipLaunchKernelGGL(k_swap_state, dim3((n_reps + 63u) / 64u), dim3(64), 0, st, reps_dev, n_reps);
    return hipGetLastError();
}

template <typename T, bool MEASURE>
static hipError_t fused_allow_one(uint32_t bytes)
{
    const void *f[3] = {(const void *)&k_sc_fused<T, MEASURE, 1>, nullptr, nullptr};
    if constexpr (sizeof(T) == 4) {
        f[1] = (const void *)&k_sc_fused<T, MEASURE, 2>;
        f[2] = (const void *)&k_sc_fused<T, MEASURE, 3>;
    }
    for (const void *fn : f) {
        if (!fn) continue;
        const hipError_t e =
            hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// The allowance is per kernel (and device), shared by every handle: it is
// only ever raised, so a handle with a smaller tile never takes away what
// another one's launches need.
hipError_t fused_allow(bool f64, uint32_t bytes)
{
    static std::mutex mu;
    static uint32_t allowed[64][2]; // per device and precision
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    uint32_t &a = allowed[dev][f64 ? 1 : 0];
    if (bytes <= a) return hipSuccess;
    e = f64 ? fused_allow_one<double, false>(bytes) : fused_allow_one<float, false>(bytes);
    if (e == hipSuccess)
        e = f64 ? fused_allow_one<double, true>(bytes) : fused_allow_one<float, true>(bytes);
    if (e == hipSuccess) a = bytes;
    return e;
}

} // namespace mc
