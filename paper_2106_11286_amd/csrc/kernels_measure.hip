// kernels_measure.hip -- observables of a spin state computed from scratch,
// for checking the fused reduction of the pass kernels.
//
// Independent of the pass code on purpose: sites are enumerated in canonical
// order, the storage index is derived from the layout rule, nearest
// neighbours come from a table of bond vectors in half-cell units (each bond
// counted once, from the end that sees it along a "forward" vector), and
// every product is formed in FP64.  Eq. (1) of arXiv:2106.11286 gives the
// energy (E_exch = -J sum_bonds S_i.S_j, E_anis = -K sum_i (S_i.e)^2), Eq. (2)
// the magnetisation sum.
#include <hip/hip_runtime.h>

#include "launch.hpp"

namespace mc {

namespace {

// Forward bond vectors (half-cell units): the first nonzero component is
// positive, so every unordered nearest-neighbour pair is met once.
__constant__ int8_t kFwdSC[3][3] = {{2, 0, 0}, {0, 2, 0}, {0, 0, 2}};
__constant__ int8_t kFwdBCC[4][3] = {{1, 1, 1}, {1, 1, -1}, {1, -1, 1}, {1, -1, -1}};
__constant__ int8_t kFwdFCC[6][3] = {{1, 1, 0}, {1, -1, 0}, {1, 0, 1},
                                     {1, 0, -1}, {0, 1, 1}, {0, 1, -1}};
// Basis offsets (half-cell units) of the conventional cell.
__constant__ int8_t kBasisFCC[4][3] = {{0, 0, 0}, {1, 1, 0}, {1, 0, 1}, {0, 1, 1}};

struct Geo {
    int kind, nb, Lx, Ly, Lz;
    uint32_t pmask, n_cells;
    int sphere;
    double r2x4;
};

__device__ __forceinline__ void basis_offset(const Geo &g, int b, int &ox, int &oy, int &oz)
{
    if (g.kind == FCC) {
        ox = kBasisFCC[b][0];
        oy = kBasisFCC[b][1];
        oz = kBasisFCC[b][2];
    } else {
        ox = oy = oz = (g.kind == BCC && b == 1) ? 1 : 0;
    }
}

// Basis index of a half-cell parity pattern, or -1 if no site sits there.
__device__ __forceinline__ int basis_of(const Geo &g, int px, int py, int pz)
{
    for (int b = 0; b < g.nb; ++b) {
        int ox, oy, oz;
        basis_offset(g, b, ox, oy, oz);
        if (ox == px && oy == py && oz == pz) return b;
    }
    return -1;
}

__device__ __forceinline__ bool inside(const Geo &g, int qx, int qy, int qz)
{
    if (!g.sphere) return true;
    const double dx = qx - g.Lx, dy = qy - g.Ly, dz = qz - g.Lz;
    return dx * dx + dy * dy + dz * dz <= g.r2x4;
}

// Storage index of site (x, y, z, b) in the library layout.
__device__ __forceinline__ uint32_t storage(const Geo &g, int x, int y, int z, int b)
{
    const uint32_t cell = (uint32_t)(z * g.Ly + y) * (uint32_t)g.Lx + (uint32_t)x;
    if (g.kind == SC) return (uint32_t)((x + y + z) & 1) * (g.n_cells / 2u) + (cell >> 1);
    return (uint32_t)b * g.n_cells + cell;
}

// Wrap one coordinate of a half-cell position; false across an open face.
__device__ __forceinline__ bool wrap(int &q, int L, bool periodic)
{
    if (q >= 0 && q < 2 * L) return true;
    if (!periodic) return false;
    q = q < 0 ? q + 2 * L : q - 2 * L;
    return true;
}

} // namespace

template <typename T>
__global__ void __launch_bounds__(256)
k_measure_direct(RepDev R, int kind, double *__restrict__ partials)
{
    Geo g;
    g.kind = kind;
    g.nb = kind == SC ? 1 : (kind == BCC ? 2 : 4);
    g.Lx = R.Lx;
    g.Ly = R.Ly;
    g.Lz = R.Lz;
    g.pmask = R.pmask;
    g.n_cells = (uint32_t)R.Lx * (uint32_t)R.Ly * (uint32_t)R.Lz;
    g.sphere = R.sphere;
    g.r2x4 = R.r2x4;
    const T *sx = (const T *)R.sx, *sy = (const T *)R.sy, *sz = (const T *)R.sz;
    const double ex = R.e[0], ey = R.e[1], ez = R.e[2];
    const int n_fwd = kind == SC ? 3 : (kind == BCC ? 4 : 6);
    const uint32_t n = R.n_box;
    const uint32_t s0 = (uint32_t)(((uint64_t)n * blockIdx.x) / gridDim.x);
    const uint32_t s1 = (uint32_t)(((uint64_t)n * (blockIdx.x + 1)) / gridDim.x);
    double m_x = 0, m_y = 0, m_z = 0, pe2 = 0, bond = 0, cnt = 0;
    for (uint32_t s = s0 + threadIdx.x; s < s1; s += blockDim.x) {
        const int b = (int)(s % (uint32_t)g.nb);
        const uint32_t cell = s / (uint32_t)g.nb;
        const int x = (int)(cell % (uint32_t)g.Lx);
        const int y = (int)((cell / (uint32_t)g.Lx) % (uint32_t)g.Ly);
        const int z = (int)(cell / ((uint32_t)g.Lx * (uint32_t)g.Ly));
        int ox, oy, oz;
        basis_offset(g, b, ox, oy, oz);
        const int qx = 2 * x + ox, qy = 2 * y + oy, qz = 2 * z + oz;
        if (!inside(g, qx, qy, qz)) continue;
        const uint32_t i = storage(g, x, y, z, b);
        const double ax = (double)sx[i], ay = (double)sy[i], az = (double)sz[i];
        m_x += ax;
        m_y += ay;
        m_z += az;
        const double pe = ax * ex + ay * ey + az * ez;
        pe2 += pe * pe;
        cnt += 1.0;
        for (int k = 0; k < n_fwd; ++k) {
            int dx, dy, dz;
            if (kind == SC) {
                dx = kFwdSC[k][0]; dy = kFwdSC[k][1]; dz = kFwdSC[k][2];
            } else if (kind == BCC) {
                dx = kFwdBCC[k][0]; dy = kFwdBCC[k][1]; dz = kFwdBCC[k][2];
            } else {
                dx = kFwdFCC[k][0]; dy = kFwdFCC[k][1]; dz = kFwdFCC[k][2];
            }
            int px = qx + dx, py = qy + dy, pz = qz + dz;
            if (!wrap(px, g.Lx, g.pmask & 1u) || !wrap(py, g.Ly, g.pmask & 2u) ||
                !wrap(pz, g.Lz, g.pmask & 4u))
                continue;
            // an unoccupied neighbour (outside the sphere) has no bond
            if (!inside(g, px, py, pz)) continue;
            const int b2 = basis_of(g, px & 1, py & 1, pz & 1);
            const uint32_t j = storage(g, px >> 1, py >> 1, pz >> 1, b2);
            bond += ax * (double)sx[j] + ay * (double)sy[j] + az * (double)sz[j];
        }
    }
    // fixed-order block reduction: wave butterflies, then the waves in order
    __shared__ double red[4][6];
    double v[6] = {m_x, m_y, m_z, pe2, bond, cnt};
#pragma unroll
    for (int q = 0; q < 6; ++q)
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) v[q] += __shfl_xor(v[q], o, 64);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0)
#pragma unroll
        for (int q = 0; q < 6; ++q) red[wave][q] = v[q];
    __syncthreads();
    if (threadIdx.x < 6) {
        double a = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) a += red[w][threadIdx.x];
        partials[(size_t)blockIdx.x * 8 + threadIdx.x] = a;
    }
}

// Sum the block partials in block order into one record (FP64): M sums,
// E_exch, E_anis, occupied count in the accepted-count slot.
__global__ void __launch_bounds__(64)
k_measure_finish(const double *__restrict__ partials, uint32_t n_blocks, double J, double K,
                 double sweep, double *__restrict__ record)
{
    __shared__ double out[6];
    const uint32_t q = threadIdx.x;
    if (q < 6) {
        double a = 0.0;
        for (uint32_t b = 0; b < n_blocks; ++b) a += partials[(size_t)b * 8 + q];
        out[q] = a;
    }
    __syncthreads();
    if (q != 0) return;
    record[R_MX] = out[0];
    record[R_MY] = out[1];
    record[R_MZ] = out[2];
    record[R_EEX] = -J * out[4];
    record[R_EAN] = -K * out[3];
    record[R_NACC] = out[5];
    record[R_SWEEP] = sweep;
    record[7] = 0.0;
}

hipError_t launch_measure_direct(bool f64, int kind, const RepDev *rep_host, double *partials,
                                 uint32_t n_blocks, double sweep, double *record, hipStream_t st)
{
    if (n_blocks == 0 || n_blocks > MEASURE_BLOCKS) return hipErrorInvalidValue;
    if (f64)
        hipLaunchKernelGGL((k_measure_direct<double>), dim3(n_blocks), dim3(256), 0, st,
                           *rep_host, kind, partials);
    else
        hipLaunchKernelGGL((k_measure_direct<float>), dim3(n_blocks), dim3(256), 0, st,
                           *rep_host, kind, partials);
    hipLaunchKernelGGL(k_measure_finish, dim3(1), dim3(64), 0, st, partials, n_blocks,
                       rep_host->J, rep_host->K, sweep, record);
    return hipGetLastError();
}

} // namespace mc
