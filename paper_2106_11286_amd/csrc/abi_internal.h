// abi_internal.h -- host-side declarations shared by the translation units of
// the runtime behind the C ABI: the handle, the scratch layout and the helpers
// that more than one unit uses (abi.cpp: handle, plan, sweeps, schedule;
// abi_tune.cpp: autotuner; abi_stats.cpp: series statistics;
// abi_extensions.cpp: replica exchange and the block scheme).
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstdint>
#include <map>
#include <string>
#include <utility>
#include <vector>

#include "launch.hpp"
#include "mc_internal.hpp"
#include "mcheis.h"

using namespace mc;

namespace mcabi {

extern thread_local std::string g_err;
// Set the thread's error message and return the status.
mc_status fail(mc_status s, const char *fmt, ...);

#define HIP_TRY(expr)                                                                    \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess)                                                            \
            return fail(MC_E_DEVICE, "%s: %s (%s:%d)", #expr, hipGetErrorString(e_),     \
                        __FILE__, __LINE__);                                             \
    } while (0)

constexpr uint32_t kRing = 256;       // observable records kept per replica
// LDS kept back from the dynamic allocation of the LDS kernel for its static
// arrays (reduction slots).
constexpr uint32_t kLdsReserve = 2048;
constexpr uint32_t kTargetItems = 8192; // work items aimed for per pass
constexpr uint32_t kGraphChunk = 64;  // sweeps per captured graph

struct ScratchLayout {
    uint64_t off_ctr, off_reps, off_work, off_partials, off_records, off_stage,
        off_persist, off_queues, off_exchange, off_measure, total;
};

// Words of the persistent-queue region: 16 queue offsets, then every item
// index once (at least 64 words: it also takes the XCD probe's output).
inline uint64_t queue_words(uint64_t n_items) { return 16 + std::max<uint64_t>(n_items, 64); }

uint64_t align_up(uint64_t v, uint64_t a);
int row_len(const mc_replica_desc &d);
int pow2_at_least(int v);
uint64_t xy_tiles(const mc_replica_desc &d, const Tile &t);
bool persistent_supported(const Tile &t);
void set_temperature(RepDev &R, double T);

} // namespace mcabi

struct mc_sim {
    int32_t n_reps = 0, kind = 0, n_colours = 0;
    mc_precision prec = MC_F32;
    uint64_t seed = 0;
    std::vector<mc_replica_desc> desc;
    std::vector<RepDev> reps;
    std::vector<uint64_t> n_occ;
    std::vector<WorkItem> work;
    Tile tile{};      // kernel of whole sweeps
    Tile pass_tile{}; // kernel of single passes (= tile unless tile is the LDS kernel)
    uint32_t lds_max = 0; // dynamic LDS a workgroup may use on this device (bytes)
    std::string device_key; // the device as the autotuner's cache sees it
    hipStream_t stream = nullptr;
    char *scratch = nullptr;
    uint64_t scratch_bytes = 0;
    mcabi::ScratchLayout lay{};
    uint32_t *tctr = nullptr;
    RepDev *reps_dev = nullptr;
    WorkItem *work_dev = nullptr;
    double *partials = nullptr;
    double *records = nullptr;
    double *stage = nullptr;    // finalise stage slots
    uint32_t *pstate = nullptr; // persistent-launch counters
    uint32_t *queues_dev = nullptr; // queue offsets [16], then queue items
    // replica exchange (mc_exchange_*): device table in scratch, host ladder
    bool xchg_active = false;
    std::vector<double> xchg_T, xchg_beta; // per slot
    std::vector<uint32_t> xchg_rep_host;   // upload staging
    uint32_t spin_limit = 1u << 24;
    bool persist_used = false;
    bool tuned_persistent = false;  // launch mode chosen by mc_autotune(MC_TUNED_LAUNCH)
    int persist_mode = MC_PERSIST_AUTO;
    bool xcd_ok = false;            // workgroups are dealt to 8 XCDs in turn
    uint32_t n_queues = 1, max_queue_items = 0;
    std::vector<uint32_t> q_host;   // queue table as uploaded (offsets [16], items)
    double *host_rec = nullptr; // pinned, (kRing + 1) * n_reps * NR
    uint64_t t = 0;             // sweeps done
    uint64_t n_measured = 0;
    int64_t last_slot = -1;
    std::map<std::pair<uint32_t, uint32_t>, hipGraphExec_t> graphs;
    uint32_t magic = 0x4d434831u;
};

namespace mcabi {

bool alive(const mc_sim *h);
void fill_repdev(const mc_replica_desc &d, const mc_spin_buffers &b, RepDev &R);
// Workgroups of a from-scratch measurement of one replica (<= MEASURE_BLOCKS).
uint32_t measure_blocks(const RepDev &R);
// Arguments of a from-scratch measurement of caller buffers.
mc_status check_measure_args(const mc_replica_desc *d, mc_precision prec,
                             const mc_spin_buffers *bufs, const double *record_dev);
bool lds_fits(const mc_sim *h);
// A simple-cubic handle with a replica cut to a sphere (tile and LDS kernels only).
bool sc_sphere(const mc_sim *h);
mc_status check_persistent(mc_sim *h);
// While replica exchange is active the device descriptors hold each
// replica's current temperature; copy it into the host descriptors.
mc_status xchg_pull(mc_sim *h);

} // namespace mcabi
