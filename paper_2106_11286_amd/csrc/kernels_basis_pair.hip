// kernels_basis_pair.hip -- pass kernels of the basis pair scheme (bcc and fcc
// lattices with an even number of cells per row) and their launcher.
#include "basis_bodies.hpp"

namespace mc {

template <int KIND, int B, typename T, bool MEASURE, int MODE, int RY>
__global__ void __launch_bounds__(256) k_basis_pair(PassLaunch P)
{
    uint32_t item;
    if (!logical_item(P, item)) return;
    basis_pair_body<KIND, B, T, MEASURE, MODE, RY>(P, item, *P.tctr_dev + P.t_off);
}

template <int KIND, typename T, bool MEASURE, int MODE, int RY>
static hipError_t bpair_colour(int colour, const PassLaunch &p, hipStream_t st)
{
    // a multiple of 8 workgroups (logical_item deals them to the XCDs)
    const dim3 g(((p.n_blocks + 7u) >> 3) << 3), b(p.tile.tx);
    switch (colour) {
    case 0: hipLaunchKernelGGL((k_basis_pair<KIND, 0, T, MEASURE, MODE, RY>), g, b, 0, st, p); break;
    case 1: hipLaunchKernelGGL((k_basis_pair<KIND, 1, T, MEASURE, MODE, RY>), g, b, 0, st, p); break;
    case 2:
        if constexpr (KIND == FCC) {
            hipLaunchKernelGGL((k_basis_pair<KIND, 2, T, MEASURE, MODE, RY>), g, b, 0, st, p);
            break;
        }
        return hipErrorInvalidValue;
    case 3:
        if constexpr (KIND == FCC) {
            hipLaunchKernelGGL((k_basis_pair<KIND, 3, T, MEASURE, MODE, RY>), g, b, 0, st, p);
            break;
        }
        return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T, bool MEASURE, int MODE>
static hipError_t bpair_dispatch(int kind, int colour, const PassLaunch &p, hipStream_t st)
{
    if (kind == BCC) {
        if (p.tile.ty == 1) return bpair_colour<BCC, T, MEASURE, MODE, 1>(colour, p, st);
        if (p.tile.ty == 2) return bpair_colour<BCC, T, MEASURE, MODE, 2>(colour, p, st);
    } else if (kind == FCC) {
        if (p.tile.ty == 1) return bpair_colour<FCC, T, MEASURE, MODE, 1>(colour, p, st);
        if (p.tile.ty == 2) return bpair_colour<FCC, T, MEASURE, MODE, 2>(colour, p, st);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_basis_pair(int kind, bool f64, int colour, bool measure, int mode,
                             const PassLaunch &p, hipStream_t st)
{
    if (mode == 1)
        return f64 ? bpair_dispatch<double, true, 1>(kind, colour, p, st)
                   : bpair_dispatch<float, true, 1>(kind, colour, p, st);
    if (mode == 2)
        return f64 ? bpair_dispatch<double, false, 2>(kind, colour, p, st)
                   : bpair_dispatch<float, false, 2>(kind, colour, p, st);
    if (f64)
        return measure ? bpair_dispatch<double, true, 0>(kind, colour, p, st)
                       : bpair_dispatch<double, false, 0>(kind, colour, p, st);
    return measure ? bpair_dispatch<float, true, 0>(kind, colour, p, st)
                   : bpair_dispatch<float, false, 0>(kind, colour, p, st);
}

} // namespace mc
