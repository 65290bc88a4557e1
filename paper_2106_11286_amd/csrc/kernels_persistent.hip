// kernels_persistent.hip -- n sweeps of every replica in one launch, work units
// claimed in order, per-replica phase release.
#include "basis_bodies.hpp"
#include "sc_bodies.hpp"

namespace mc {

// ---------------------------------------------------------------------------
// Persistent batched sweeps (see PersistLaunch).  Units are claimed in order
// from one queue (n_queues == 1) or from one queue per XCD (n_queues == 8,
// every replica of queue g swept only by workgroups running on XCD g).
//
// Memory ordering.  A waiting unit polls its replica's phase flag, then
// acquires (agent scope: its L1 is invalidated) before reading spins.  With
// one queue a unit's stores are released at agent scope (the XCD's L2 is
// written back) before its completion is counted, and the workgroup that
// completes a replica's pass acquires and releases again before it publishes
// the next phase.  With a queue per XCD every reader and writer of a replica
// shares one L2, so a unit only waits until its stores have reached that L2
// (vmcnt 0, the compiler's own release for workgroups split over the CUs of
// one XCD) before counting; nothing is written back during the launch.
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
    } else if constexpr (KERNEL == KERNEL_BPAIR) {
        switch (c) {
        case 0: basis_pair_body<KIND, 0, T, MEASURE, 0, RY>(P, item, t); break;
        case 1: basis_pair_body<KIND, 1, T, MEASURE, 0, RY>(P, item, t); break;
        case 2:
            if constexpr (KIND == FCC) basis_pair_body<KIND, 2, T, MEASURE, 0, RY>(P, item, t);
            break;
        default:
            if constexpr (KIND == FCC) basis_pair_body<KIND, 3, T, MEASURE, 0, RY>(P, item, t);
            break;
        }
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

// s_waitcnt immediate with vmcnt = 0 and expcnt, lgkmcnt left at their maxima
constexpr int WAIT_VMCNT0 = 0x0F70;

template <typename T, bool MEASURE, int KIND, int KERNEL, int RY>
__global__ void __launch_bounds__(256) k_persistent(PassLaunch P, PersistLaunch A)
{
    __shared__ uint32_t s_unit, s_flag;
    __shared__ double s_rec[NQ];
    uint32_t *const hdr = A.state;
    uint32_t *const done = A.state + PERSIST_HDR, *const ready = done + A.n_reps;
    const bool per_xcd = A.n_queues > 1;
    const uint32_t g = per_xcd ? xcd_id() : 0u;
    uint32_t *const claim = hdr + PS_CLAIM + g;
    // queue g: the items q_items[q_off[g] .. q_off[g+1]) (all items when NULL)
    const uint32_t q_begin = per_xcd ? A.q_off[g] : 0u;
    const uint32_t n_items = per_xcd ? A.q_off[g + 1] - q_begin : P.n_items;
    const uint32_t per_sweep = A.n_colours * n_items;
    const uint32_t total = A.n_sweeps * per_sweep;
    const uint32_t t0 = *P.tctr_dev + P.t_off;
    for (;;) {
        if (threadIdx.x == 0) {
            uint32_t u = __hip_atomic_fetch_add(claim, 1u, __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_AGENT);
            if (__hip_atomic_load(&hdr[PS_ABORT], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
                u = total;
            s_unit = u;
        }
        __syncthreads();
        const uint32_t u = s_unit;
        if (u >= total) break;
        const uint32_t sw = u / per_sweep, rem = u - sw * per_sweep;
        const uint32_t c = rem / n_items, local = rem - c * n_items;
        const uint32_t item = per_xcd ? A.q_items[q_begin + local] : local;
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
                    __hip_atomic_load(&hdr[PS_ABORT], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                    ok = 0;
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
            }
            if (!ok) {
                __hip_atomic_store(&hdr[PS_TRIPPED], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&hdr[PS_ABORT], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            s_flag = ok;
        }
        __syncthreads();
        if (!s_flag) break;
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        unit_body<T, MEASURE, KIND, KERNEL, RY>(P, (int)c, item, t0 + sw);
        if (per_xcd) {
            // the fence keeps the stores above it; the wait lets them reach the L2
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            __builtin_amdgcn_s_waitcnt(WAIT_VMCNT0);
        } else {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        }
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
                        const double *p = P.partials_dev + ((size_t)cc * P.n_items + it) * NQ;
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
                // one queue: the other units of this phase released their
                // stores (agent scope) before counting; acquire them and
                // release them on to the next phase's readers.  Per-XCD
                // queues: they are already in the L2 every reader uses.
                if (!per_xcd) __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
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
    // time; workgroups beyond twice that would only wait.  Per-XCD queues:
    // a multiple of 8 workgroups, dispatched to the XCDs in turn, sized for
    // the largest queue.
    const uint64_t total = (uint64_t)a.n_sweeps * a.n_colours * p.n_items;
    unsigned grid;
    if (a.n_queues > 1) {
        uint64_t per = 2ull * a.max_queue_items;
        if (per > 256) per = 256;
        grid = (unsigned)(8 * per);
        if (total == 0) grid = 0;
    } else {
        uint64_t cap = 2ull * p.n_items;
        if (cap > 2048) cap = 2048;
        grid = (unsigned)(total < cap ? total : cap);
    }
    if (grid == 0) return hipSuccess;
    // tx x ty threads for the tile-shaped kernels (a persistent unit of a bcc
    // or fcc lattice runs the tile body on the same tile), tx for the others
    const bool tile_shaped = p.tile.kernel == KERNEL_TILE || p.tile.kernel == KERNEL_BSTRIP;
    const int threads = tile_shaped ? ((p.tile.tx * p.tile.ty + 63) / 64) * 64 : p.tile.tx;
    const dim3 g(grid), b(threads);
    if (kind != SC && p.tile.kernel == KERNEL_BPAIR) {
        const dim3 bp(p.tile.tx);
        if (kind == BCC && p.tile.ty == 1)
            hipLaunchKernelGGL((k_persistent<T, MEASURE, BCC, KERNEL_BPAIR, 1>), g, bp, 0, st, p, a);
        else if (kind == BCC && p.tile.ty == 2)
            hipLaunchKernelGGL((k_persistent<T, MEASURE, BCC, KERNEL_BPAIR, 2>), g, bp, 0, st, p, a);
        else if (kind == FCC && p.tile.ty == 1)
            hipLaunchKernelGGL((k_persistent<T, MEASURE, FCC, KERNEL_BPAIR, 1>), g, bp, 0, st, p, a);
        else if (kind == FCC && p.tile.ty == 2)
            hipLaunchKernelGGL((k_persistent<T, MEASURE, FCC, KERNEL_BPAIR, 2>), g, bp, 0, st, p, a);
        else
            return hipErrorInvalidValue;
    } else if (kind == BCC) {
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

// One thread: the launch before it (same stream) has ended.
__global__ void k_persist_check(PersistLaunch A, uint32_t n_items)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    uint32_t *const hdr = A.state;
    if (hdr[PS_TRIPPED]) hdr[PS_STICKY_WATCHDOG] = 1u;
    for (uint32_t g = 0; g < A.n_queues; ++g) {
        const uint32_t n_g = A.n_queues > 1 ? A.q_off[g + 1] - A.q_off[g] : n_items;
        if (hdr[PS_CLAIM + g] < A.n_sweeps * A.n_colours * n_g) hdr[PS_STICKY_UNDRAINED] = 1u;
    }
}

hipError_t launch_persist_check(const PersistLaunch &a, uint32_t n_items, hipStream_t st)
{
    hipLaunchKernelGGL(k_persist_check, dim3(1), dim3(64), 0, st, a, n_items);
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
