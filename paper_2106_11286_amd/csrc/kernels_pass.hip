// kernels_pass.hip -- one launch per colour pass: the pass kernels of every
// scheme and their launchers.
#include "basis_bodies.hpp"
#include "sc_bodies.hpp"
#include "sc_lband.hpp"

namespace mc {

// ---------------------------------------------------------------------------
// Pass kernels: one workgroup per work item, sweep counter from the device.
// ---------------------------------------------------------------------------
template <typename T, bool MEASURE, int MODE>
__global__ void __launch_bounds__(256) k_sc_tile(PassLaunch P, int colour)
{
    uint32_t item;
    if (!logical_item(P, item)) return;
    sc_tile_body<T, MEASURE, MODE>(P, colour, item, *P.tctr_dev + P.t_off);
}

template <typename T, bool MEASURE, int MODE, int RY>
__global__ void __launch_bounds__(256) k_sc_strip(PassLaunch P, int colour)
{
    uint32_t item;
    if (!logical_item(P, item)) return;
    sc_strip_body<T, MEASURE, MODE, RY>(P, colour, item, *P.tctr_dev + P.t_off);
}

template <typename T, bool MEASURE, int MODE, int RY>
__global__ void __launch_bounds__(256) k_sc_band(PassLaunch P, int colour)
{
    uint32_t item;
    if (!logical_item(P, item)) return;
    sc_band_body<T, MEASURE, MODE, RY>(P, colour, item, *P.tctr_dev + P.t_off);
}

template <typename T, bool MEASURE, int MODE, int RY>
__global__ void __launch_bounds__(256) k_sc_pair(PassLaunch P, int colour)
{
    uint32_t item;
    if (!logical_item(P, item)) return;
    sc_pair_body<T, MEASURE, MODE, RY>(P, colour, item, *P.tctr_dev + P.t_off);
}

template <typename T, bool MEASURE, int MODE, int RY>
__global__ void __launch_bounds__(256) k_sc_pband(PassLaunch P, int colour)
{
    uint32_t item;
    if (!logical_item(P, item)) return;
    sc_pband_body<T, MEASURE, MODE, RY>(P, colour, item, *P.tctr_dev + P.t_off);
}

template <typename T, bool MEASURE, int MODE, int PP>
__global__ void __launch_bounds__(256) k_sc_lband(PassLaunch P, int colour)
{
    uint32_t item;
    if (!logical_item(P, item)) return;
    sc_lband_body<T, MEASURE, MODE, PP>(P, colour, item, *P.tctr_dev + P.t_off);
}

template <int KIND, int B, typename T, bool MEASURE, int MODE>
__global__ void __launch_bounds__(256) k_basis_strip(PassLaunch P)
{
    uint32_t item;
    if (!logical_item(P, item)) return;
    basis_strip_body<KIND, B, T, MEASURE, MODE>(P, item, *P.tctr_dev + P.t_off);
}

template <int KIND, int B, typename T, bool MEASURE, int MODE>
__global__ void __launch_bounds__(256) k_basis_pass(PassLaunch P)
{
    uint32_t item;
    if (!logical_item(P, item)) return;
    basis_body<KIND, B, T, MEASURE, MODE>(P, item, *P.tctr_dev + P.t_off);
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
static dim3 pass_grid(const PassLaunch &p) { return dim3(((p.n_blocks + 7u) >> 3) << 3); }

template <typename T, bool MEASURE, int MODE>
static hipError_t sc_launch(int colour, const PassLaunch &p, hipStream_t st)
{
    if (p.tile.kernel == KERNEL_BAND) {
        const dim3 g = pass_grid(p), b(p.tile.tx);
        switch (p.tile.ty) {
        case 2: hipLaunchKernelGGL((k_sc_band<T, MEASURE, MODE, 2>), g, b, 0, st, p, colour); break;
        case 4: hipLaunchKernelGGL((k_sc_band<T, MEASURE, MODE, 4>), g, b, 0, st, p, colour); break;
        default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    if (p.tile.kernel == KERNEL_PBAND) {
        const dim3 g = pass_grid(p), b(p.tile.tx);
        switch (p.tile.ty) {
        case 2: hipLaunchKernelGGL((k_sc_pband<T, MEASURE, MODE, 2>), g, b, 0, st, p, colour); break;
        case 4:
            // four-row bands in FP64 need more than 256 registers (refused on the host)
            if constexpr (sizeof(T) == 4) {
                hipLaunchKernelGGL((k_sc_pband<T, MEASURE, MODE, 4>), g, b, 0, st, p, colour);
                break;
            } else {
                return hipErrorInvalidValue;
            }
        default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    if (p.tile.kernel == KERNEL_LBAND) {
        const dim3 g = pass_grid(p), b(p.tile.tx);
        switch (p.lds_positions) {
        case 1: hipLaunchKernelGGL((k_sc_lband<T, MEASURE, MODE, 1>), g, b, p.lds_bytes, st, p, colour); break;
        case 2: hipLaunchKernelGGL((k_sc_lband<T, MEASURE, MODE, 2>), g, b, p.lds_bytes, st, p, colour); break;
        default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    if (p.tile.kernel == KERNEL_PAIR) {
        const dim3 g = pass_grid(p), b(p.tile.tx);
        switch (p.tile.ty) {
        case 1: hipLaunchKernelGGL((k_sc_pair<T, MEASURE, MODE, 1>), g, b, 0, st, p, colour); break;
        case 2: hipLaunchKernelGGL((k_sc_pair<T, MEASURE, MODE, 2>), g, b, 0, st, p, colour); break;
        case 4: hipLaunchKernelGGL((k_sc_pair<T, MEASURE, MODE, 4>), g, b, 0, st, p, colour); break;
        default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    if (p.tile.kernel == KERNEL_STRIP) {
        const dim3 g = pass_grid(p), b(p.tile.tx);
        switch (p.tile.ty) {
        case 1: hipLaunchKernelGGL((k_sc_strip<T, MEASURE, MODE, 1>), g, b, 0, st, p, colour); break;
        case 2: hipLaunchKernelGGL((k_sc_strip<T, MEASURE, MODE, 2>), g, b, 0, st, p, colour); break;
        case 4: hipLaunchKernelGGL((k_sc_strip<T, MEASURE, MODE, 4>), g, b, 0, st, p, colour); break;
        case 8: hipLaunchKernelGGL((k_sc_strip<T, MEASURE, MODE, 8>), g, b, 0, st, p, colour); break;
        default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    const int threads = ((p.tile.tx * p.tile.ty + 63) / 64) * 64;
    hipLaunchKernelGGL((k_sc_tile<T, MEASURE, MODE>), pass_grid(p), dim3(threads), 0, st, p,
                       colour);
    return hipGetLastError();
}

template <int KIND, typename T, bool MEASURE, int MODE>
static hipError_t basis_launch(int colour, const PassLaunch &p, hipStream_t st)
{
    const int threads = ((p.tile.tx * p.tile.ty + 63) / 64) * 64;
    const dim3 g = pass_grid(p), b(threads);
    if (p.tile.kernel == KERNEL_BSTRIP) {
        switch (colour) {
        case 0: hipLaunchKernelGGL((k_basis_strip<KIND, 0, T, MEASURE, MODE>), g, b, 0, st, p); break;
        case 1: hipLaunchKernelGGL((k_basis_strip<KIND, 1, T, MEASURE, MODE>), g, b, 0, st, p); break;
        case 2:
            if constexpr (KIND == FCC) hipLaunchKernelGGL((k_basis_strip<KIND, 2, T, MEASURE, MODE>), g, b, 0, st, p);
            break;
        case 3:
            if constexpr (KIND == FCC) hipLaunchKernelGGL((k_basis_strip<KIND, 3, T, MEASURE, MODE>), g, b, 0, st, p);
            break;
        default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    switch (colour) {
    case 0: hipLaunchKernelGGL((k_basis_pass<KIND, 0, T, MEASURE, MODE>), g, b, 0, st, p); break;
    case 1: hipLaunchKernelGGL((k_basis_pass<KIND, 1, T, MEASURE, MODE>), g, b, 0, st, p); break;
    case 2:
        if constexpr (KIND == FCC) hipLaunchKernelGGL((k_basis_pass<KIND, 2, T, MEASURE, MODE>), g, b, 0, st, p);
        break;
    case 3:
        if constexpr (KIND == FCC) hipLaunchKernelGGL((k_basis_pass<KIND, 3, T, MEASURE, MODE>), g, b, 0, st, p);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T, bool MEASURE, int MODE>
static hipError_t pass_dispatch(int kind, int colour, const PassLaunch &p, hipStream_t st)
{
    switch (kind) {
    case SC: return sc_launch<T, MEASURE, MODE>(colour, p, st);
    case BCC: return basis_launch<BCC, T, MEASURE, MODE>(colour, p, st);
    case FCC: return basis_launch<FCC, T, MEASURE, MODE>(colour, p, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_pass(int kind, bool f64, int colour, bool measure, int mode, const PassLaunch &p,
                       hipStream_t st)
{
    if (p.n_blocks == 0) return hipSuccess;
    if (mode == 2 && (!p.dbg_dh || !p.dbg_acc)) return hipErrorInvalidValue;
    if (kind != SC && p.tile.kernel == KERNEL_BPAIR)
        return launch_basis_pair(kind, f64, colour, measure, mode, p, st);
    if (mode == 1) {
        return f64 ? pass_dispatch<double, true, 1>(kind, colour, p, st)
                   : pass_dispatch<float, true, 1>(kind, colour, p, st);
    }
    if (mode == 2) {
        if (!p.dbg_dh || !p.dbg_acc) return hipErrorInvalidValue;
        return f64 ? pass_dispatch<double, false, 2>(kind, colour, p, st)
                   : pass_dispatch<float, false, 2>(kind, colour, p, st);
    }
    if (f64)
        return measure ? pass_dispatch<double, true, 0>(kind, colour, p, st)
                       : pass_dispatch<double, false, 0>(kind, colour, p, st);
    return measure ? pass_dispatch<float, true, 0>(kind, colour, p, st)
                   : pass_dispatch<float, false, 0>(kind, colour, p, st);
}

} // namespace mc
