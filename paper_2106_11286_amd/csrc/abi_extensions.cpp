// abi_extensions.cpp -- beyond the colour sweep: replica exchange between
// neighbouring temperatures (mc_exchange_*) and the paper's block scheme as a
// comparison kernel (mc_block_*).
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <vector>

#include "abi_internal.h"

using namespace mcabi;

namespace mcabi {

// Device pointers of the replica-exchange table (scratch, off_exchange).
struct XchgPtrs {
    double *beta;
    uint64_t *attempted, *accepted;
    uint32_t *rep_at, *round;
};
XchgPtrs xchg_ptrs(const mc_sim *h)
{
    char *b = h->scratch + h->lay.off_exchange;
    const size_t n = (size_t)h->n_reps;
    return {(double *)b, (uint64_t *)(b + 8 * n), (uint64_t *)(b + 16 * n),
            (uint32_t *)(b + 24 * n), (uint32_t *)(b + 28 * n)};
}

mc_status xchg_pull(mc_sim *h)
{
    if (!h->xchg_active) return MC_OK;
    std::vector<uint32_t> rep_at(h->n_reps);
    HIP_TRY(hipStreamSynchronize(h->stream));
    HIP_TRY(hipMemcpy(rep_at.data(), xchg_ptrs(h).rep_at, sizeof(uint32_t) * h->n_reps,
                      hipMemcpyDeviceToHost));
    for (int k = 0; k < h->n_reps; ++k) {
        const uint32_t r = rep_at[k];
        if (r >= (uint32_t)h->n_reps) return fail(MC_E_DEVICE, "exchange table corrupted");
        h->desc[r].T = h->xchg_T[k];
        set_temperature(h->reps[r], h->xchg_T[k]);
    }
    return MC_OK;
}

// Identical lattices and couplings (all but T and replica_id).
bool same_system(const mc_replica_desc &a, const mc_replica_desc &b)
{
    return a.kind == b.kind && a.Lx == b.Lx && a.Ly == b.Ly && a.Lz == b.Lz &&
           a.periodic_mask == b.periodic_mask && a.sphere_radius == b.sphere_radius &&
           a.J == b.J && a.K == b.K && a.e[0] == b.e[0] && a.e[1] == b.e[1] && a.e[2] == b.e[2];
}

} // namespace mcabi

extern "C" {

mc_status mc_exchange_init(mc_sim *h)
{
    if (!alive(h)) return fail(MC_E_STATE, "invalid or destroyed handle");
    const int n = h->n_reps;
    if (n < 2) return fail(MC_E_ARG, "replica exchange needs at least 2 replicas");
    for (int r = 0; r < n; ++r) {
        if (!same_system(h->desc[r], h->desc[0]))
            return fail(MC_E_ARG, "replica %d: exchange needs replicas that differ only in T and "
                                  "replica_id", r);
        const double T = h->desc[r].T;
        if (!(T > 0.0) || !std::isfinite(T))
            return fail(MC_E_ARG, "replica %d: exchange needs 0 < T < inf (T = %g)", r, T);
    }
    HIP_TRY(hipStreamSynchronize(h->stream));
    std::vector<int> order(n);
    for (int r = 0; r < n; ++r) order[r] = r;
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return h->desc[a].T < h->desc[b].T; });
    h->xchg_T.resize(n);
    h->xchg_beta.resize(n);
    h->xchg_rep_host.resize(n);
    for (int k = 0; k < n; ++k) {
        h->xchg_T[k] = h->desc[order[k]].T;
        h->xchg_beta[k] = 1.0 / h->xchg_T[k];
        h->xchg_rep_host[k] = (uint32_t)order[k];
    }
    const XchgPtrs x = xchg_ptrs(h);
    HIP_TRY(hipMemcpyAsync(x.beta, h->xchg_beta.data(), sizeof(double) * n, hipMemcpyHostToDevice,
                           h->stream));
    HIP_TRY(hipMemcpyAsync(x.rep_at, h->xchg_rep_host.data(), sizeof(uint32_t) * n,
                           hipMemcpyHostToDevice, h->stream));
    HIP_TRY(launch_zero_u32((uint32_t *)x.attempted, 4u * (uint32_t)n, h->stream));
    HIP_TRY(launch_zero_u32(x.round, 1u, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    h->xchg_active = true;
    return MC_OK;
}

mc_status mc_exchange_sweep(mc_sim *h, uint32_t n_rounds, uint32_t sweeps_per_round,
                            uint32_t flags)
{
    if (!alive(h)) return fail(MC_E_STATE, "invalid or destroyed handle");
    if (!h->xchg_active) return fail(MC_E_STATE, "replica exchange not initialised (mc_exchange_init)");
    if (flags & ~MC_PERSISTENT) return fail(MC_E_ARG, "unknown flags 0x%x", flags);
    if (sweeps_per_round < 1) return fail(MC_E_ARG, "sweeps_per_round must be >= 1");
    if (h->t + (uint64_t)n_rounds * sweeps_per_round > 0xFFFFFFFFull)
        return fail(MC_E_STATE, "sweep counter would exceed 2^32-1");
    const XchgPtrs x = xchg_ptrs(h);
    for (uint32_t k = 0; k < n_rounds; ++k) {
        mc_status st;
        if (flags & MC_PERSISTENT) {
            // one launch per round: every sweep measured (the records are a
            // by-product; the chain does not depend on them)
            if ((st = mc_sweep(h, sweeps_per_round, MC_MEASURE | flags)) != MC_OK) return st;
        } else {
            if (sweeps_per_round > 1 && (st = mc_sweep(h, sweeps_per_round - 1, flags)) != MC_OK)
                return st;
            if ((st = mc_sweep(h, 1, MC_MEASURE | flags)) != MC_OK) return st;
        }
        ExchangeLaunch L;
        L.reps_dev = h->reps_dev;
        L.records = h->records + (size_t)h->last_slot * h->n_reps * NR;
        L.beta = x.beta;
        L.rep_at = x.rep_at;
        L.round = x.round;
        L.attempted = x.attempted;
        L.accepted = x.accepted;
        L.tctr_dev = h->tctr;
        L.n = (uint32_t)h->n_reps;
        L.seed_lo = (uint32_t)h->seed;
        L.seed_hi = (uint32_t)(h->seed >> 32);
        HIP_TRY(launch_exchange(L, h->stream));
    }
    return MC_OK;
}

mc_status mc_exchange_state(mc_sim *h, int32_t *replica_at_slot, double *T_slot,
                            uint64_t *attempted, uint64_t *accepted, uint64_t *rounds)
{
    if (!alive(h)) return fail(MC_E_STATE, "invalid or destroyed handle");
    if (!h->xchg_active) return fail(MC_E_STATE, "replica exchange not initialised (mc_exchange_init)");
    HIP_TRY(hipStreamSynchronize(h->stream));
    mc_status st = check_persistent(h);
    if (st != MC_OK) return st;
    const int n = h->n_reps;
    const XchgPtrs x = xchg_ptrs(h);
    std::vector<uint32_t> rep_at(n);
    std::vector<uint64_t> att(n), acc(n);
    uint32_t rnd = 0;
    HIP_TRY(hipMemcpy(rep_at.data(), x.rep_at, sizeof(uint32_t) * n, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(att.data(), x.attempted, sizeof(uint64_t) * n, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(acc.data(), x.accepted, sizeof(uint64_t) * n, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(&rnd, x.round, sizeof rnd, hipMemcpyDeviceToHost));
    for (int k = 0; k < n; ++k) {
        if (replica_at_slot) replica_at_slot[k] = (int32_t)rep_at[k];
        if (T_slot) T_slot[k] = h->xchg_T[k];
        if (k + 1 < n) {
            if (attempted) attempted[k] = att[k];
            if (accepted) accepted[k] = acc[k];
        }
    }
    if (rounds) *rounds = rnd;
    return xchg_pull(h);
}

mc_status mc_block_workspace(const mc_sim *h, uint32_t n, uint64_t *bytes)
{
    if (!alive(h)) return fail(MC_E_STATE, "invalid or destroyed handle");
    if (!bytes) return fail(MC_E_ARG, "bytes is NULL");
    if (n < 1) return fail(MC_E_ARG, "n (sites per block) must be >= 1");
    uint64_t nb = 0;
    for (const RepDev &R : h->reps) nb = std::max<uint64_t>(nb, (R.n_box + n - 1) / n);
    const uint64_t esz = h->prec == MC_F64 ? 8 : 4;
    *bytes = 256 + align_up(4 * nb, 256) + 3 * esz * nb;
    return MC_OK;
}

mc_status mc_block_steps(mc_sim *h, uint32_t n, uint32_t step0, uint32_t n_steps, uint32_t flags,
                         void *work, uint64_t work_bytes)
{
    if (!alive(h)) return fail(MC_E_STATE, "invalid or destroyed handle");
    if (h->kind != MC_SC) return fail(MC_E_UNSUPPORTED, "the block scheme is built for sc lattices");
    if (flags & ~(MC_BLOCK_CONFLICTS | MC_BLOCK_RESET))
        return fail(MC_E_ARG, "unknown flags 0x%x", flags);
    uint64_t need = 0;
    mc_status st = mc_block_workspace(h, n, &need);
    if (st != MC_OK) return st;
    if (!work || reinterpret_cast<uintptr_t>(work) % 256)
        return fail(MC_E_BUFFER, "block workspace is NULL or not 256-byte aligned");
    if (work_bytes < need)
        return fail(MC_E_BUFFER, "block workspace has %llu bytes, %llu needed",
                    (unsigned long long)work_bytes, (unsigned long long)need);
    if ((uint64_t)step0 + n_steps > 0xFFFFFFFFull) return fail(MC_E_ARG, "step counter would exceed 2^32-1");
    uint64_t nb_max = 0;
    for (const RepDev &R : h->reps) nb_max = std::max<uint64_t>(nb_max, (R.n_box + n - 1) / n);
    char *w = (char *)work;
    BlockLaunch B;
    B.n = n;
    B.seed_lo = (uint32_t)h->seed;
    B.seed_hi = (uint32_t)(h->seed >> 32);
    B.count_conflicts = (flags & MC_BLOCK_CONFLICTS) ? 1 : 0;
    B.counts = (unsigned long long *)w;
    B.stage_idx = (uint32_t *)(w + 256);
    B.stage_spin = w + 256 + align_up(4 * nb_max, 256);
    if ((st = xchg_pull(h)) != MC_OK) return st; // current temperatures into h->reps
    if (flags & MC_BLOCK_RESET) HIP_TRY(launch_zero_u32((uint32_t *)w, 6, h->stream));
    for (uint32_t j = 0; j < n_steps; ++j)
        for (int r = 0; r < h->n_reps; ++r) {
            B.rep = h->reps[r];
            B.n_blocks = (uint32_t)((h->reps[r].n_box + n - 1) / n);
            B.step = step0 + j;
            HIP_TRY(launch_block_step(h->prec == MC_F64, B, h->stream));
        }
    return MC_OK;
}

mc_status mc_block_counts(mc_sim *h, void *work, uint64_t counts[3])
{
    if (!alive(h)) return fail(MC_E_STATE, "invalid or destroyed handle");
    if (!work || !counts) return fail(MC_E_ARG, "work or counts is NULL");
    HIP_TRY(hipStreamSynchronize(h->stream));
    HIP_TRY(hipMemcpy(counts, work, 3 * sizeof(uint64_t), hipMemcpyDeviceToHost));
    HIP_TRY(launch_zero_u32((uint32_t *)work, 6, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    return MC_OK;
}

} // extern "C"
