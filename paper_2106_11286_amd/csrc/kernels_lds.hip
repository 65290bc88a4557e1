// kernels_lds.hip -- whole sweeps of small lattices held in one workgroup's
// LDS.
#include <mutex>

#include "device_common.hpp"

namespace mc {

// ---------------------------------------------------------------------------
// Small lattices held in LDS: one workgroup per replica copies the replica's
// three component planes into LDS, runs n whole sweeps there (colour passes
// separated by workgroup barriers, so no other workgroup is involved and no
// device-scope synchronisation is needed), optionally writes one record per
// sweep, and copies the planes back.  The site updates are the same
// arithmetic, in the same order, as the pass kernels, so the chain is
// bitwise the same.
// ---------------------------------------------------------------------------
template <typename T> using lptr = __attribute__((address_space(3))) T *;

// Division by a divisor fixed for the launch (a lattice edge d >= 1):
// floor(n / d) = mulhi(n, ceil(2^32 / d)), exact while n d < 2^32, which the
// site indices of a lattice held in LDS (n below its few thousand box sites)
// always satisfy.  Replaces the integer division sequence in the site loop.
struct FastDiv {
    uint32_t d, m;
};
__device__ __forceinline__ FastDiv fast_div(uint32_t d)
{
    return FastDiv{d, d <= 1u ? 0u : (uint32_t)((0x100000000ull + d - 1u) / d)};
}
__device__ __forceinline__ uint32_t div_of(uint32_t n, FastDiv f)
{
    return f.d <= 1u ? n : __umulhi(n, f.m);
}

// Block reduction for up to 1024 threads into out[0..Q_N) (LDS); fixed order.
__device__ __forceinline__ void block_reduce_1024(double (&a)[Q_N], double *out)
{
    __shared__ double red[16][Q_N];
#pragma unroll
    for (int q = 0; q < Q_N; ++q) {
        double v = a[q];
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
        a[q] = v;
    }
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int n_waves = (blockDim.x + 63) >> 6;
    if (lane == 0) {
#pragma unroll
        for (int q = 0; q < Q_N; ++q) red[wave][q] = a[q];
    }
    __syncthreads();
    if (threadIdx.x < Q_N) {
        double v = 0.0;
        for (int w = 0; w < n_waves; ++w) v += red[w][threadIdx.x];
        out[threadIdx.x] = v;
    }
    __syncthreads();
}

template <typename T, int KIND, bool MEASURE>
__global__ void __launch_bounds__(1024) k_lds_sweeps(LdsLaunch L)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char lds_raw[];
    __shared__ double s_rec[Q_N];
    constexpr int NB = basis_count(KIND);
    constexpr int NC = KIND == SC ? 2 : NB;
    const RepDev &R = L.reps_dev[blockIdx.x];
    const int Lx = R.Lx, Ly = R.Ly, Lz = R.Lz, Lxh = R.Lxh;
    const uint32_t n_box = R.n_box, plane = R.plane, rid = R.rid;
    const gptr<T> gx = as_global<T>(R.sx), gy = as_global<T>(R.sy), gz = as_global<T>(R.sz);
    const T J = (T)R.J, K = (T)R.K, ex = (T)R.e[0], ey = (T)R.e[1], ez = (T)R.e[2];
    const T beta = (T)R.beta;
    const bool greedy = R.greedy != 0;
    const bool px = R.pmask & 1u, py = R.pmask & 2u, pz = R.pmask & 4u;
    const double Kd = R.K, Jd = R.J;
    const uint32_t t0 = *L.tctr_dev;
    const FastDiv f_row = fast_div((uint32_t)(KIND == SC ? Lxh : Lx)), f_y = fast_div((uint32_t)Ly);
    const lptr<T> lx = (lptr<T>)(lptr<unsigned char>)lds_raw;
    const lptr<T> ly = lx + n_box, lz = ly + n_box;
    for (uint32_t i = threadIdx.x; i < n_box; i += blockDim.x) {
        lx[i] = gx[i];
        ly[i] = gy[i];
        lz[i] = gz[i];
    }
    __syncthreads();
    for (uint32_t sw = 0; sw < L.n_sweeps; ++sw) {
        const uint32_t t = t0 + sw;
        double acc[Q_N] = {0, 0, 0, 0, 0, 0};
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            for (uint32_t k = threadIdx.x; k < plane; k += blockDim.x) {
                T hx, hy, hz, sh_x, sh_y, sh_z;
                uint32_t i, s;
                if constexpr (KIND == SC) {
                    const uint32_t row = div_of(k, f_row);
                    const int xh = (int)(k - row * (uint32_t)Lxh);
                    const uint32_t zz = div_of(row, f_y);
                    const int y = (int)(row - zz * (uint32_t)Ly), z = (int)zz;
                    const int p = (c + y + z) & 1;
                    if (!occupied(R, 2 * xh + p, y, z, 0, 0, 0)) continue;
                    sc_site_field<T>(lx, ly, lz, c ? 0u : plane, Lxh, Ly, Lz, px, py, pz, xh, y,
                                     z, p, hx, hy, hz);
                    i = (c ? plane : 0u) + k;
                    s = row * (uint32_t)Lx + 2u * (uint32_t)xh + (uint32_t)p;
                } else {
                    const uint32_t r2 = div_of(k, f_row);
                    const int x = (int)(k - r2 * (uint32_t)Lx);
                    const uint32_t zz = div_of(r2, f_y);
                    const int y = (int)(r2 - zz * (uint32_t)Ly), z = (int)zz;
                    if (!occupied(R, x, y, z, basis2(KIND, c, 0), basis2(KIND, c, 1),
                                  basis2(KIND, c, 2)))
                        continue;
                    switch (c) {
                    case 0:
                        basis_site_field<KIND, 0, T>(lx, ly, lz, plane, Lx, Ly, Lz, px, py, pz, x,
                                                     y, z, hx, hy, hz, sh_x, sh_y, sh_z);
                        break;
                    case 1:
                        basis_site_field<KIND, 1, T>(lx, ly, lz, plane, Lx, Ly, Lz, px, py, pz, x,
                                                     y, z, hx, hy, hz, sh_x, sh_y, sh_z);
                        break;
                    case 2:
                        basis_site_field<KIND, (NB > 2 ? 2 : 0), T>(lx, ly, lz, plane, Lx, Ly, Lz,
                                                                    px, py, pz, x, y, z, hx, hy,
                                                                    hz, sh_x, sh_y, sh_z);
                        break;
                    default:
                        basis_site_field<KIND, (NB > 3 ? 3 : 0), T>(lx, ly, lz, plane, Lx, Ly, Lz,
                                                                    px, py, pz, x, y, z, hx, hy,
                                                                    hz, sh_x, sh_y, sh_z);
                        break;
                    }
                    i = (uint32_t)c * plane + k;
                    s = k * NB + (uint32_t)c;
                }
                hx *= J;
                hy *= J;
                hz *= J;
                T sx = lx[i], sy = ly[i], sz = lz[i];
                T dH;
                const bool a = metropolis<T>(sx, sy, sz, hx, hy, hz, s, rid, t, L.seed_lo,
                                             L.seed_hi, K, ex, ey, ez, beta, greedy, dH);
                if (a) {
                    lx[i] = sx;
                    ly[i] = sy;
                    lz[i] = sz;
                }
                if (MEASURE) {
                    if constexpr (KIND == SC)
                        observe<T>(acc, sx, sy, sz, ex, ey, ez, c == 1, hx, hy, hz, 1.0);
                    else
                        observe<T>(acc, sx, sy, sz, ex, ey, ez, true, sh_x, sh_y, sh_z, Jd);
                    acc[Q_NACC] += a ? 1.0 : 0.0;
                }
            }
            __syncthreads();
        }
        if (MEASURE) {
            block_reduce_1024(acc, s_rec);
            if (threadIdx.x == 0) {
                double *rec = L.records +
                              ((size_t)((L.slot0 + sw) % L.ring) * L.n_reps + blockIdx.x) * NR;
                rec[R_MX] = s_rec[Q_MX];
                rec[R_MY] = s_rec[Q_MY];
                rec[R_MZ] = s_rec[Q_MZ];
                rec[R_EEX] = -s_rec[Q_SH];
                rec[R_EAN] = -Kd * s_rec[Q_PE2];
                rec[R_NACC] = s_rec[Q_NACC];
                rec[R_SWEEP] = (double)t + 1.0;
                rec[7] = 0.0;
            }
        }
    }
    for (uint32_t i = threadIdx.x; i < n_box; i += blockDim.x) {
        gx[i] = lx[i];
        gy[i] = ly[i];
        gz[i] = lz[i];
    }
}

template <typename T, bool MEASURE>
static hipError_t lds_dispatch(int kind, const LdsLaunch &L, int threads, hipStream_t st)
{
    const dim3 g(L.n_reps), b(threads);
    if (kind == SC)
        hipLaunchKernelGGL((k_lds_sweeps<T, SC, MEASURE>), g, b, L.lds_bytes, st, L);
    else if (kind == BCC)
        hipLaunchKernelGGL((k_lds_sweeps<T, BCC, MEASURE>), g, b, L.lds_bytes, st, L);
    else
        hipLaunchKernelGGL((k_lds_sweeps<T, FCC, MEASURE>), g, b, L.lds_bytes, st, L);
    return hipGetLastError();
}

hipError_t launch_lds(int kind, bool f64, bool measure, const LdsLaunch &L, int threads,
                      hipStream_t st)
{
    if (L.n_reps == 0 || L.n_sweeps == 0) return hipSuccess;
    if (threads < 64 || threads > 1024 || threads % 64) return hipErrorInvalidValue;
    if (f64)
        return measure ? lds_dispatch<double, true>(kind, L, threads, st)
                       : lds_dispatch<double, false>(kind, L, threads, st);
    return measure ? lds_dispatch<float, true>(kind, L, threads, st)
                   : lds_dispatch<float, false>(kind, L, threads, st);
}

template <typename T> static hipError_t lds_allow_kind(int kind, uint32_t bytes)
{
    const void *f[2];
    if (kind == SC) {
        f[0] = (const void *)&k_lds_sweeps<T, SC, false>;
        f[1] = (const void *)&k_lds_sweeps<T, SC, true>;
    } else if (kind == BCC) {
        f[0] = (const void *)&k_lds_sweeps<T, BCC, false>;
        f[1] = (const void *)&k_lds_sweeps<T, BCC, true>;
    } else {
        f[0] = (const void *)&k_lds_sweeps<T, FCC, false>;
        f[1] = (const void *)&k_lds_sweeps<T, FCC, true>;
    }
    for (const void *fn : f) {
        const hipError_t e =
            hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// The allowance is per kernel (and device), shared by every handle: it is
// only ever raised, so a handle with a smaller lattice never takes away what
// another one's launches need.
hipError_t lds_allow(int kind, bool f64, uint32_t bytes)
{
    static std::mutex mu;
    static uint32_t allowed[64][3][2]; // per device, lattice kind and precision
    if (kind < 0 || kind > 2) return hipErrorInvalidValue;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    uint32_t &a = allowed[dev][kind][f64 ? 1 : 0];
    if (bytes <= a) return hipSuccess;
    e = f64 ? lds_allow_kind<double>(kind, bytes) : lds_allow_kind<float>(kind, bytes);
    if (e == hipSuccess) a = bytes;
    return e;
}

} // namespace mc
