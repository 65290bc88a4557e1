// launch.hpp -- host-callable launchers of the device kernels (kernels_*.hip).
#pragma once

#include <hip/hip_runtime_api.h>
#include <stdint.h>

#include "mc_internal.hpp"

namespace mc {

// Everything a pass launch needs; device pointers point into the scratch.
struct PassLaunch {
    const RepDev *reps_dev;   // [n_reps]
    const WorkItem *work_dev; // [n_items]
    uint32_t item_base;       // first work item of this launch
    uint32_t n_blocks;        // work items in this launch
    uint32_t n_items;         // items in the whole work list (partials stride)
    const uint32_t *tctr_dev; // sweep counter t (device)
    uint32_t t_off;           // added to t
    uint32_t seed_lo, seed_hi;
    Tile tile;
    double *partials_dev;     // [n_colours][n_items][NQ]
    void *dbg_dh;             // debug: per-site dH (or null)
    uint8_t *dbg_acc;         // debug: per-site decision (or null)
    uint32_t lds_bytes;       // dynamic LDS of the LDS-staged pass kernel
    int32_t lds_positions;    // its (row, pair) positions per lane (1 or 2)
};

// mode: 0 = Metropolis update, 1 = observables of the current state only,
//       2 = update writing per-site dH and decisions to p.dbg_dh / p.dbg_acc
hipError_t launch_pass(int kind, bool f64, int colour, bool measure, int mode,
                       const PassLaunch &p, hipStream_t st);
// The basis pair kernels (bcc, fcc; called by launch_pass for that tile).
hipError_t launch_basis_pair(int kind, bool f64, int colour, bool measure, int mode,
                             const PassLaunch &p, hipStream_t st);

hipError_t launch_init(bool f64, int kind, const RepDev *rep_host, int mode, uint32_t seed_lo,
                       uint32_t seed_hi, hipStream_t st);

hipError_t launch_layout(bool f64, int kind, const RepDev *rep_host, bool to_natural, void *nx,
                         void *ny, void *nz, hipStream_t st);

// Reduce partials of every pass into one record per replica (two launches).
// stage_dev holds n_reps * FIN_BLOCKS * NQ doubles.
hipError_t launch_finalize(const RepDev *reps_dev, int n_reps, int n_colours,
                           const double *partials_dev, uint32_t n_items,
                           const uint32_t *tctr_dev, uint32_t t_off, double *records_dev,
                           double *stage_dev, hipStream_t st);
hipError_t launch_zero_u32(uint32_t *p, uint32_t n, hipStream_t st);

// One persistent launch that runs n_sweeps sweeps of every replica.  Work units
// (sweep, colour, item) are handed out in that order by an atomic counter; a
// unit waits until its replica has finished the previous colour pass (or
// sweep), so replicas advance independently and no grid-wide barrier is
// needed.  State layout (uint32, zeroed before every launch):
//   [0] next unit, [1] abort, [2] watchdog tripped, [3] unused,
//   [4 .. 4+n_reps) items done per replica, [4+n_reps .. 4+2 n_reps) phases released.
struct PersistLaunch {
    uint32_t *state;      // PERSIST_HDR header words, then done[n_reps], ready[n_reps]
    uint32_t n_sweeps, n_colours, n_reps;
    uint32_t spin_limit;  // bounded wait: spins of ~0.1 us before the watchdog trips
    double *records;      // ring [ring][n_reps][NR]
    uint32_t ring, slot0; // record slot of sweep s = (slot0 + s) % ring
    // 1: one queue of all items in order; 8: queue g holds the items
    // q_items[q_off[g] .. q_off[g+1]) and is served by XCD g only
    uint32_t n_queues, max_queue_items;
    const uint32_t *q_off, *q_items;
};
// Header words.  Sticky (kept across launches until the host reads them):
// a launch's bounded wait gave up; a launch left a queue undrained.  Per
// launch (cleared before each): abort, wait gave up, claim counter of queue g.
constexpr uint32_t PS_STICKY_WATCHDOG = 0, PS_STICKY_UNDRAINED = 1, PS_ABORT = 2, PS_TRIPPED = 3,
                   PS_CLAIM = 4, PERSIST_HDR = 12;
inline uint32_t persist_state_words(int n_reps) { return PERSIST_HDR + 2u * (uint32_t)n_reps; }

hipError_t launch_persistent(int kind, bool f64, bool measure, const PassLaunch &p,
                             const PersistLaunch &a, hipStream_t st);
// After a persistent launch over n_items items: fold its watchdog flag into
// the sticky word and flag any queue whose units were not all claimed.
hipError_t launch_persist_check(const PersistLaunch &a, uint32_t n_items, hipStream_t st);

// Whole sweeps of small replicas in LDS: one workgroup per replica (every
// replica's three planes, lds_bytes in all, fit one workgroup's LDS).
struct LdsLaunch {
    const RepDev *reps_dev;
    uint32_t n_reps, n_sweeps;
    const uint32_t *tctr_dev; // sweep counter t of the first sweep
    uint32_t seed_lo, seed_hi;
    double *records;          // ring [ring][n_reps][NR] (measured launches)
    uint32_t ring, slot0;
    uint32_t lds_bytes;       // dynamic LDS per workgroup
};
hipError_t launch_lds(int kind, bool f64, bool measure, const LdsLaunch &L, int threads,
                      hipStream_t st);
// Allow the LDS kernels of one lattice kind and precision `bytes` of dynamic LDS.
hipError_t lds_allow(int kind, bool f64, uint32_t bytes);

// The fused simple-cubic sweep (kernel 9): both colours of one sweep in one
// launch, from each replica's current buffer set (sx, sy, sz) into its second
// set (ax, ay, az), measured or not; p.lds_bytes of dynamic LDS.
hipError_t launch_fused(bool f64, bool measure, const PassLaunch &p, hipStream_t st);
// Swap every replica's two buffer sets in the device descriptors (after a
// fused sweep: the second set holds the current state).
hipError_t launch_swap_state(RepDev *reps_dev, uint32_t n_reps, hipStream_t st);
// Allow the fused kernel `bytes` of dynamic LDS.
hipError_t fused_allow(bool f64, uint32_t bytes);

// The HBM streams of a colour pass without its arithmetic (see mc_stream_probe).
hipError_t launch_stream_probe(bool f64, void *x, void *y, void *z, uint64_t P, uint32_t grid,
                               hipStream_t st);
// Replica exchange between neighbouring temperature slots (one workgroup):
// slot k holds replica rep_at[k] at inverse temperature beta[k]; the round's
// pairs (k, k+1), k = round mod 2 + 2m, compare the total energies of the
// records at `records` ([n_reps][NR], the last measured sweep) and, when
// accepted, swap rep_at[k], rep_at[k+1] and the two replicas' beta in reps_dev.
struct ExchangeLaunch {
    RepDev *reps_dev;
    const double *records;
    const double *beta;       // [n] per slot
    uint32_t *rep_at;         // [n]
    uint32_t *round;          // rounds done (incremented by the launch)
    uint64_t *attempted, *accepted; // [n] per pair (k, k+1)
    const uint32_t *tctr_dev; // sweeps done
    uint32_t n, seed_lo, seed_hi;
};
hipError_t launch_exchange(const ExchangeLaunch &L, hipStream_t st);

// One synchronous step of the block scheme on one sc replica: block k of n
// consecutive canonical sites picks a site from Philox counter
// (k, rid, step, 3); staged moves are written by a second launch.
struct BlockLaunch {
    RepDev rep;
    uint32_t n, n_blocks, step, seed_lo, seed_hi;
    int count_conflicts;
    uint32_t *stage_idx;            // [n_blocks] storage index of the accepted move, or ~0
    void *stage_spin;               // [n_blocks][3] of the precision's type
    unsigned long long *counts;     // attempts, accepted, conflicts (accumulated)
};
hipError_t launch_block_step(bool f64, const BlockLaunch &B, hipStream_t st);

// Observables of one replica's current state from scratch (independent of
// the pass kernels): n_blocks (<= MEASURE_BLOCKS) workgroups write FP64
// partials [n_blocks][8], then one workgroup sums them in block order into
// record[NR] (M sums, E_exch, E_anis, occupied count in the R_NACC slot,
// `sweep` in R_SWEEP).
constexpr uint32_t MEASURE_BLOCKS = 1024;
hipError_t launch_measure_direct(bool f64, int kind, const RepDev *rep_host, double *partials,
                                 uint32_t n_blocks, double sweep, double *record, hipStream_t st);

// XCC_ID of workgroups 0..n-1 (thread 0 of each writes one word).
hipError_t launch_xcd_probe(uint32_t *out, uint32_t n, hipStream_t st);
hipError_t launch_advance(uint32_t *tctr_dev, uint32_t n, hipStream_t st);
hipError_t launch_set_counter(uint32_t *tctr_dev, uint32_t v, hipStream_t st);
hipError_t launch_fill_zero(double *p, uint64_t n, hipStream_t st);

} // namespace mc
