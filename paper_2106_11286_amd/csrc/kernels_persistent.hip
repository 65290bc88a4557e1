// kernels_persistent.hip -- n sweeps of every replica in one launch, work units
// claimed in order, per-replica phase release.
#include "basis_bodies.hpp"
#include "sc_bodies.hpp"

namespace mc {

// ---------------------------------------------------------------------------
// Persistent batched sweeps (see PersistLaunch).  Memory ordering: a unit's
// stores are released (agent scope) before its completion is counted; the
// workgroup that completes a replica's pass acquires, reduces the pass's
// partial sums if the sweep is measured, then releases the next phase; a
// waiting unit acquires before reading spins.
// ---------------------------------------------------------------------------
template <typename T, bool MEASURE, int KIND, int KERNEL, int RY>
__device__ __forceinline__ void unit_body(const PassLaunch &P, int c, uint32_t item, uint32_t t)
{
    if constexpr (KIND == SC) {
        if constexpr (KERNEL == KERNEL_STRIP) sc_strip_body<T, MEASURE, 0, RY>(P, c, item, t);
        else if constexpr (KERNEL == KERNEL_BAND) sc_band_body<T, MEASURE, 0, RY>(P, c, item, t);
        else if constexpr (KERNEL == KERNEL_PAIR) sc_pair_body<T, MEASURE, 0, RY>(P, c, item, t);
        else if constexpr (KERNEL == KERNEL_PBAND) sc_pband_body<T, MEASURE, 0, RY>(P, c, item, t);
        else sc_tile_body<T, MEASURE, 0>(P, c, item, t);
    } else {
        switch (c) {
        case 0: basis_body<KIND, 0, T, MEASURE, 0>(P, item, t); break;
        case 1: basis_body<KIND, 1, T, MEASURE, 0>(P, item, t); break;
        case 2:
            if constexpr (KIND == FCC) basis_body<KIND, 2, T, MEASURE, 0>(P, item, t);
            break;
        default:
            if constexpr (KIND == FCC) basis_body<KIND, 3, T, MEASURE, 0>(P, item, t);
            break;
        }
    }
}

template <typename T, bool MEASURE, int KIND, int KERNEL, int RY>
__global__ void __launch_bounds__(256) k_persistent(PassLaunch P, PersistLaunch A)
{
    __shared__ uint32_t s_unit, s_flag;
    __shared__ double s_rec[NQ];
    uint32_t *const hdr = A.state, *const done = A.state + 4, *const ready = A.state + 4 + A.n_reps;
    const uint32_t n_items = P.n_items;
    const uint32_t per_sweep = A.n_colours * n_items;
    const uint32_t total = A.n_sweeps * per_sweep;
    const uint32_t t0 = *P.tctr_dev + P.t_off;
    for (;;) {
        if (threadIdx.x == 0) {
            uint32_t u = __hip_atomic_fetch_add(&hdr[0], 1u, __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_AGENT);
            if (__hip_atomic_load(&hdr[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) u = total;
            s_unit = u;
        }
        __syncthreads();
        const uint32_t u = s_unit;
        if (u >= total) break;
        const uint32_t sw = u / per_sweep, rem = u - sw * per_sweep;
        const uint32_t c = rem / n_items, item = rem - c * n_items;
        const uint32_t r = P.work_dev[item].rep;
        const uint32_t phase = sw * A.n_colours + c;
        if (threadIdx.x == 0) {
            // poll with plain (relaxed) loads; the acquire fence below, once
            // the phase is released, orders the unit's reads after it
            uint32_t ok = 1;
            for (uint32_t spins = 0;
                 __hip_atomic_load(&ready[r], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < phase;
                 ++spins) {
                if (spins >= A.spin_limit ||
                    __hip_atomic_load(&hdr[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                    ok = 0;
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
            }
            if (!ok) {
                __hip_atomic_store(&hdr[2], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&hdr[1], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            s_flag = ok;
        }
        __syncthreads();
        if (!s_flag) break;
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        unit_body<T, MEASURE, KIND, KERNEL, RY>(P, (int)c, item, t0 + sw);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __syncthreads();
        if (threadIdx.x == 0) {
            const RepDev &R = P.reps_dev[r];
            const uint32_t n_r = R.item_end - R.item_begin;
            // every wave released its stores above; the count itself needs
            // no ordering of its own
            const uint32_t old = __hip_atomic_fetch_add(&done[r], 1u, __ATOMIC_RELAXED,
                                                        __HIP_MEMORY_SCOPE_AGENT);
            s_flag = (old + 1u == (phase + 1u) * n_r);
        }
        __syncthreads();
        if (s_flag) { // this unit completed replica r's phase
            if (MEASURE && c == A.n_colours - 1) {
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                const RepDev &R = P.reps_dev[r];
                double a[Q_N] = {0, 0, 0, 0, 0, 0};
                for (uint32_t cc = 0; cc < A.n_colours; ++cc)
                    for (uint32_t it = R.item_begin + threadIdx.x; it < R.item_end; it += blockDim.x) {
                        const double *p = P.partials_dev + ((size_t)cc * n_items + it) * NQ;
#pragma unroll
                        for (int q = 0; q < Q_N; ++q) a[q] += p[q];
                    }
                block_store_partials(a, s_rec);
                __syncthreads();
                if (threadIdx.x == 0) {
                    double *rec = A.records + ((size_t)((A.slot0 + sw) % A.ring) * A.n_reps + r) * NR;
                    rec[R_MX] = s_rec[Q_MX];
                    rec[R_MY] = s_rec[Q_MY];
                    rec[R_MZ] = s_rec[Q_MZ];
                    rec[R_EEX] = -s_rec[Q_SH];
                    rec[R_EAN] = -R.K * s_rec[Q_PE2];
                    rec[R_NACC] = s_rec[Q_NACC];
                    rec[R_SWEEP] = (double)(t0 + sw) + 1.0;
                    rec[7] = 0.0;
                }
            }
            if (threadIdx.x == 0) {
                // the other units of this phase released their stores before
                // counting; acquire them, then release the next phase
                __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
                __hip_atomic_store(&ready[r], phase + 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        __syncthreads();
    }
}

template <typename T, bool MEASURE>
static hipError_t persist_dispatch(int kind, const PassLaunch &p, const PersistLaunch &a,
                                   hipStream_t st)
{
    // at most one phase of every replica (n_items units in all) can run at a
    // time; workgroups beyond twice that would only wait
    const uint64_t total = (uint64_t)a.n_sweeps * a.n_colours * p.n_items;
    uint64_t cap = 2ull * p.n_items;
    if (cap > 2048) cap = 2048;
    const unsigned grid = (unsigned)(total < cap ? total : cap);
    if (grid == 0) return hipSuccess;
    // tx x ty threads for the tile-shaped kernels (a persistent unit of a bcc
    // or fcc lattice runs the tile body on the same tile), tx for the others
    const bool tile_shaped = p.tile.kernel == KERNEL_TILE || p.tile.kernel == KERNEL_BSTRIP;
    const int threads = tile_shaped ? ((p.tile.tx * p.tile.ty + 63) / 64) * 64 : p.tile.tx;
    const dim3 g(grid), b(threads);
    if (kind == BCC) {
        hipLaunchKernelGGL((k_persistent<T, MEASURE, BCC, KERNEL_TILE, 1>), g, b, 0, st, p, a);
    } else if (kind == FCC) {
        hipLaunchKernelGGL((k_persistent<T, MEASURE, FCC, KERNEL_TILE, 1>), g, b, 0, st, p, a);
    } else if (p.tile.kernel == KERNEL_TILE) {
        hipLaunchKernelGGL((k_persistent<T, MEASURE, SC, KERNEL_TILE, 1>), g, b, 0, st, p, a);
    } else if (p.tile.kernel == KERNEL_STRIP && p.tile.ty == 2) {
        hipLaunchKernelGGL((k_persistent<T, MEASURE, SC, KERNEL_STRIP, 2>), g, b, 0, st, p, a);
    } else if (p.tile.kernel == KERNEL_STRIP && p.tile.ty == 4) {
        hipLaunchKernelGGL((k_persistent<T, MEASURE, SC, KERNEL_STRIP, 4>), g, b, 0, st, p, a);
    } else if (p.tile.kernel == KERNEL_PBAND && p.tile.ty == 2) {
        hipLaunchKernelGGL((k_persistent<T, MEASURE, SC, KERNEL_PBAND, 2>), g, b, 0, st, p, a);
    } else if (p.tile.kernel == KERNEL_PAIR && p.tile.ty == 1) {
        hipLaunchKernelGGL((k_persistent<T, MEASURE, SC, KERNEL_PAIR, 1>), g, b, 0, st, p, a);
    } else if (p.tile.kernel == KERNEL_PAIR && p.tile.ty == 2) {
        hipLaunchKernelGGL((k_persistent<T, MEASURE, SC, KERNEL_PAIR, 2>), g, b, 0, st, p, a);
    } else if (p.tile.kernel == KERNEL_BAND && p.tile.ty == 2) {
        hipLaunchKernelGGL((k_persistent<T, MEASURE, SC, KERNEL_BAND, 2>), g, b, 0, st, p, a);
    } else if (p.tile.kernel == KERNEL_BAND && p.tile.ty == 4) {
        hipLaunchKernelGGL((k_persistent<T, MEASURE, SC, KERNEL_BAND, 4>), g, b, 0, st, p, a);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_persistent(int kind, bool f64, bool measure, const PassLaunch &p,
                             const PersistLaunch &a, hipStream_t st)
{
    if ((uint64_t)a.n_sweeps * a.n_colours * p.n_items >= 0xFFFFFFFFull) return hipErrorInvalidValue;
    if (f64)
        return measure ? persist_dispatch<double, true>(kind, p, a, st)
                       : persist_dispatch<double, false>(kind, p, a, st);
    return measure ? persist_dispatch<float, true>(kind, p, a, st)
                   : persist_dispatch<float, false>(kind, p, a, st);
}

} // namespace mc
