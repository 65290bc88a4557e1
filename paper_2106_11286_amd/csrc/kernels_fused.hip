// kernels_fused.hip -- the fused simple-cubic sweep (kernel 9) and the swap of
// the two state buffer sets that follows each of its launches.
#include "launch.hpp"
#include "sc_fused.hpp"

namespace mc {

template <typename T, bool MEASURE>
__global__ void __launch_bounds__(256) k_sc_fused(PassLaunch P)
{
    uint32_t item;
    if (!logical_item(P, item)) return;
    sc_fused_body<T, MEASURE>(P, item, *P.tctr_dev + P.t_off);
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

hipError_t launch_fused(bool f64, bool measure, const PassLaunch &p, hipStream_t st)
{
    if (p.n_blocks == 0) return hipSuccess;
    if (p.tile.tx != 256 || p.tile.ty < 1) return hipErrorInvalidValue;
    const dim3 g(((p.n_blocks + 7u) >> 3) << 3), b(256);
    if (f64) {
        if (measure)
            hipLaunchKernelGGL((k_sc_fused<double, true>), g, b, p.lds_bytes, st, p);
        else
            hipLaunchKernelGGL((k_sc_fused<double, false>), g, b, p.lds_bytes, st, p);
    } else {
        if (measure)
            hipLaunchKernelGGL((k_sc_fused<float, true>), g, b, p.lds_bytes, st, p);
        else
            hipLaunchKernelGGL((k_sc_fused<float, false>), g, b, p.lds_bytes, st, p);
    }
    return hipGetLastError();
}

hipError_t launch_swap_state(RepDev *reps_dev, uint32_t n_reps, hipStream_t st)
{
    hipLaunchKernelGGL(k_swap_state, dim3((n_reps + 63u) / 64u), dim3(64), 0, st, reps_dev, n_reps);
    return hipGetLastError();
}

hipError_t fused_allow(bool f64, uint32_t bytes)
{
    const void *f[2];
    if (f64) {
        f[0] = (const void *)&k_sc_fused<double, false>;
        f[1] = (const void *)&k_sc_fused<double, true>;
    } else {
        f[0] = (const void *)&k_sc_fused<float, false>;
        f[1] = (const void *)&k_sc_fused<float, true>;
    }
    for (const void *fn : f) {
        const hipError_t e =
            hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

} // namespace mc
