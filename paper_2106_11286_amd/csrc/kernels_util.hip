// kernels_util.hip -- initial state, layout conversion, the observable
// finalise, counters, fills and the memory-pattern probe.
#include "device_common.hpp"

namespace mc {

// ---------------------------------------------------------------------------
// Initial state and layout conversion (one replica per launch).
// ---------------------------------------------------------------------------
struct SiteCoord {
    int x, y, z, b;
    uint32_t s; // canonical index
};

__device__ __forceinline__ SiteCoord decode(const RepDev &R, int kind, uint32_t i)
{
    SiteCoord c;
    const uint32_t colour = i / R.plane, j = i - colour * R.plane;
    if (kind == SC) {
        const uint32_t xh = j % (uint32_t)R.Lxh, r = j / (uint32_t)R.Lxh;
        c.y = (int)(r % (uint32_t)R.Ly);
        c.z = (int)(r / (uint32_t)R.Ly);
        c.x = 2 * (int)xh + (int)((colour + c.y + c.z) & 1u);
        c.b = 0;
        c.s = (uint32_t)(c.z * R.Ly + c.y) * (uint32_t)R.Lx + c.x;
    } else {
        c.x = (int)(j % (uint32_t)R.Lx);
        const uint32_t r = j / (uint32_t)R.Lx;
        c.y = (int)(r % (uint32_t)R.Ly);
        c.z = (int)(r / (uint32_t)R.Ly);
        c.b = (int)colour;
        c.s = j * (uint32_t)basis_count(kind) + colour;
    }
    return c;
}

__device__ __forceinline__ bool occupied_site(const RepDev &R, int kind, const SiteCoord &c)
{
    int bx = 0, by = 0, bz = 0;
    if (kind == BCC) bx = by = bz = c.b;
    if (kind == FCC) {
        bx = c.b == 1 || c.b == 2;
        by = c.b == 1 || c.b == 3;
        bz = c.b == 2 || c.b == 3;
    }
    return occupied(R, c.x, c.y, c.z, bx, by, bz);
}

template <typename T>
__global__ void __launch_bounds__(256)
k_init(RepDev R, int kind, int mode, uint32_t k0, uint32_t k1)
{
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < R.n_box;
         i += gridDim.x * blockDim.x) {
        const SiteCoord c = decode(R, kind, i);
        T vx = 0, vy = 0, vz = 0;
        if (occupied_site(R, kind, c)) {
            if (mode == 1) {
                vx = (T)R.e[0];
                vy = (T)R.e[1];
                vz = (T)R.e[2];
            } else {
                const Words w = philox10(c.s, R.rid, 0u, 1u, k0, k1);
                sphere_point(uniform23<T>(w.w0), uniform23<T>(w.w1), vx, vy, vz);
            }
        }
        ((T *)R.sx)[i] = vx;
        ((T *)R.sy)[i] = vy;
        ((T *)R.sz)[i] = vz;
    }
}

template <typename T>
__global__ void __launch_bounds__(256)
k_layout(RepDev R, int kind, int to_natural, T *nx, T *ny, T *nz)
{
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < R.n_box;
         i += gridDim.x * blockDim.x) {
        const SiteCoord c = decode(R, kind, i);
        T *px = (T *)R.sx, *py = (T *)R.sy, *pz = (T *)R.sz;
        if (to_natural) {
            nx[c.s] = px[i];
            ny[c.s] = py[i];
            nz[c.s] = pz[i];
        } else {
            px[i] = nx[c.s];
            py[i] = ny[c.s];
            pz[i] = nz[c.s];
        }
    }
}

// ---------------------------------------------------------------------------
// Finalise, two launches: FIN_BLOCKS blocks per replica each sum a contiguous
// share of the replica's partial slots (all passes) into a stage slot; then
// one workgroup per replica sums the stage slots in index order and writes
// the FP64 record.  The launch boundary orders the two steps, so no block
// waits for, or publishes to, another; the result depends only on the work
// list.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256)
k_finalize_stage(const RepDev *__restrict__ reps, int n_colours,
                 const double *__restrict__ partials, uint32_t n_items,
                 double *__restrict__ stage)
{
    const uint32_t r = blockIdx.x / FIN_BLOCKS, j = blockIdx.x % FIN_BLOCKS;
    const RepDev &R = reps[r];
    const uint32_t n = R.item_end - R.item_begin;
    const uint32_t b0 = R.item_begin + (uint32_t)(((uint64_t)n * j) / FIN_BLOCKS);
    const uint32_t b1 = R.item_begin + (uint32_t)(((uint64_t)n * (j + 1)) / FIN_BLOCKS);
    double a[Q_N] = {0, 0, 0, 0, 0, 0};
    for (int c = 0; c < n_colours; ++c)
        for (uint32_t it = b0 + threadIdx.x; it < b1; it += blockDim.x) {
            const double *p = partials + ((size_t)c * n_items + it) * NQ;
#pragma unroll
            for (int q = 0; q < Q_N; ++q) a[q] += p[q];
        }
    block_store_partials(a, stage + ((size_t)r * FIN_BLOCKS + j) * NQ);
}

__global__ void __launch_bounds__(64)
k_finalize_record(const RepDev *__restrict__ reps, const uint32_t *__restrict__ tctr,
                  uint32_t t_off, const double *__restrict__ stage, double *__restrict__ records)
{
    // lane q sums observable q over the stage slots in slot order; all its
    // loads are issued before the first add
    __shared__ double out[Q_N];
    const uint32_t r = blockIdx.x, q = threadIdx.x;
    const double *st = stage + (size_t)r * FIN_BLOCKS * NQ;
    if (q < (uint32_t)Q_N) {
        double v[FIN_BLOCKS];
#pragma unroll
        for (uint32_t b = 0; b < FIN_BLOCKS; ++b) v[b] = st[b * NQ + q];
        double sum = 0.0;
#pragma unroll
        for (uint32_t b = 0; b < FIN_BLOCKS; ++b) sum += v[b];
        out[q] = sum;
    }
    __syncthreads();
    if (q != 0) return;
    double *rec = records + (size_t)r * NR;
    rec[R_MX] = out[Q_MX];
    rec[R_MY] = out[Q_MY];
    rec[R_MZ] = out[Q_MZ];
    rec[R_EEX] = -out[Q_SH];
    rec[R_EAN] = -reps[r].K * out[Q_PE2];
    rec[R_NACC] = out[Q_NACC];
    rec[R_SWEEP] = (double)(*tctr + t_off) + 1.0;
    rec[7] = 0.0;
}

__global__ void k_advance(uint32_t *tctr, uint32_t n)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *tctr += n;
}

__global__ void k_set_counter(uint32_t *tctr, uint32_t v)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *tctr = v;
}

__global__ void k_fill_zero(double *p, uint64_t n)
{
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = 0.0;
}

// ---------------------------------------------------------------------------
// Memory-pattern probe: the HBM streams of one colour pass without its
// arithmetic.  Three component arrays of 2 P elements; the first half is read
// and written in place, the second half read (24 B read and 12 B written per
// FP32 element of the first half), two elements per lane per access.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) k_stream_probe(T *x, T *y, T *z, uint64_t P)
{
    const uint64_t n2 = P / 2; // element pairs per half
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n2;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t a = 2 * i, b = P + 2 * i;
        const T x0 = x[a] + x[b], x1 = x[a + 1] + x[b + 1];
        const T y0 = y[a] + y[b], y1 = y[a + 1] + y[b + 1];
        const T z0 = z[a] + z[b], z1 = z[a + 1] + z[b + 1];
        x[a] = x0;
        x[a + 1] = x1;
        y[a] = y0;
        y[a + 1] = y1;
        z[a] = z0;
        z[a + 1] = z1;
    }
}

static unsigned grid_for(uint32_t n)
{
    uint32_t g = (n + 255) / 256;
    return g < 8192 ? (g ? g : 1) : 8192;
}

hipError_t launch_init(bool f64, int kind, const RepDev *rep_host, int mode, uint32_t seed_lo,
                       uint32_t seed_hi, hipStream_t st)
{
    const unsigned g = grid_for(rep_host->n_box);
    if (f64)
        hipLaunchKernelGGL((k_init<double>), dim3(g), dim3(256), 0, st, *rep_host, kind, mode,
                           seed_lo, seed_hi);
    else
        hipLaunchKernelGGL((k_init<float>), dim3(g), dim3(256), 0, st, *rep_host, kind, mode,
                           seed_lo, seed_hi);
    return hipGetLastError();
}

hipError_t launch_layout(bool f64, int kind, const RepDev *rep_host, bool to_natural, void *nx,
                         void *ny, void *nz, hipStream_t st)
{
    const unsigned g = grid_for(rep_host->n_box);
    if (f64)
        hipLaunchKernelGGL((k_layout<double>), dim3(g), dim3(256), 0, st, *rep_host, kind,
                           (int)to_natural, (double *)nx, (double *)ny, (double *)nz);
    else
        hipLaunchKernelGGL((k_layout<float>), dim3(g), dim3(256), 0, st, *rep_host, kind,
                           (int)to_natural, (float *)nx, (float *)ny, (float *)nz);
    return hipGetLastError();
}

hipError_t launch_finalize(const RepDev *reps_dev, int n_reps, int n_colours,
                           const double *partials_dev, uint32_t n_items,
                           const uint32_t *tctr_dev, uint32_t t_off, double *records_dev,
                           double *stage_dev, hipStream_t st)
{
    hipLaunchKernelGGL(k_finalize_stage, dim3(n_reps * FIN_BLOCKS), dim3(256), 0, st, reps_dev,
                       n_colours, partials_dev, n_items, stage_dev);
    hipLaunchKernelGGL(k_finalize_record, dim3(n_reps), dim3(64), 0, st, reps_dev, tctr_dev, t_off,
                       stage_dev, records_dev);
    return hipGetLastError();
}

__global__ void k_zero_u32(uint32_t *p, uint32_t n)
{
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        p[i] = 0u;
}

hipError_t launch_zero_u32(uint32_t *p, uint32_t n, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero_u32, dim3((n + 255) / 256 < 1024 ? (n + 255) / 256 : 1024), dim3(256),
                       0, st, p, n);
    return hipGetLastError();
}

// Replica exchange (one workgroup; the pairs of a round are disjoint, so
// each thread owns the slots it writes).  Counter (k, 0, t, 2) keys the
// uniform of pair k after t sweeps.
__global__ void __launch_bounds__(256) k_exchange(ExchangeLaunch L)
{
    const uint32_t rnd = *L.round, t = *L.tctr_dev;
    __syncthreads();
    for (uint32_t k = 2u * threadIdx.x + (rnd & 1u); k + 1u < L.n; k += 2u * blockDim.x) {
        const uint32_t i = L.rep_at[k], j = L.rep_at[k + 1u];
        const double *ri = L.records + (size_t)i * NR, *rj = L.records + (size_t)j * NR;
        const double Ei = ri[R_EEX] + ri[R_EAN], Ej = rj[R_EEX] + rj[R_EAN];
        const double delta = (L.beta[k] - L.beta[k + 1u]) * (Ei - Ej);
        bool acc = delta >= 0.0;
        if (!acc) {
            const Words w = philox10(k, 0u, t, 2u, L.seed_lo, L.seed_hi);
            acc = uniform23<double>(w.w0) < exp(delta);
        }
        L.attempted[k] += 1u;
        if (acc) {
            L.accepted[k] += 1u;
            L.rep_at[k] = j;
            L.rep_at[k + 1u] = i;
            L.reps_dev[i].beta = L.beta[k + 1u];
            L.reps_dev[j].beta = L.beta[k];
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) *L.round = rnd + 1u;
}

hipError_t launch_exchange(const ExchangeLaunch &L, hipStream_t st)
{
    hipLaunchKernelGGL(k_exchange, dim3(1), dim3(256), 0, st, L);
    return hipGetLastError();
}

__global__ void k_xcd_probe(uint32_t *out, uint32_t n)
{
    if (threadIdx.x == 0 && blockIdx.x < n) out[blockIdx.x] = xcd_id();
}

hipError_t launch_xcd_probe(uint32_t *out, uint32_t n, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_xcd_probe, dim3(n), dim3(64), 0, st, out, n);
    return hipGetLastError();
}

hipError_t launch_advance(uint32_t *tctr_dev, uint32_t n, hipStream_t st)
{
    hipLaunchKernelGGL(k_advance, dim3(1), dim3(64), 0, st, tctr_dev, n);
    return hipGetLastError();
}

hipError_t launch_set_counter(uint32_t *tctr_dev, uint32_t v, hipStream_t st)
{
    hipLaunchKernelGGL(k_set_counter, dim3(1), dim3(64), 0, st, tctr_dev, v);
    return hipGetLastError();
}

hipError_t launch_fill_zero(double *p, uint64_t n, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    const unsigned g = grid_for((uint32_t)(n < 0xFFFFFFFFull ? n : 0xFFFFFFFFull));
    hipLaunchKernelGGL(k_fill_zero, dim3(g), dim3(256), 0, st, p, n);
    return hipGetLastError();
}

hipError_t launch_stream_probe(bool f64, void *x, void *y, void *z, uint64_t P, uint32_t grid,
                               hipStream_t st)
{
    if (grid == 0 || P < 2) return hipErrorInvalidValue;
    if (f64)
        hipLaunchKernelGGL(k_stream_probe<double>, dim3(grid), dim3(256), 0, st, (double *)x,
                           (double *)y, (double *)z, P);
    else
        hipLaunchKernelGGL(k_stream_probe<float>, dim3(grid), dim3(256), 0, st, (float *)x,
                           (float *)y, (float *)z, P);
    return hipGetLastError();
}

} // namespace mc
