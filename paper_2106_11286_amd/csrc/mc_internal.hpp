// mc_internal.hpp -- structures shared by the host runtime (abi.cpp) and the
// device kernels (kernels_*.hip).  Plain-old-data only: copied verbatim into the
// caller's scratch buffer.
#pragma once

#include <stdint.h>

namespace mc {

enum Kind : int32_t { SC = 0, BCC = 1, FCC = 2 };

// Per-replica descriptor as the kernels see it (lives in device scratch).
struct alignas(16) RepDev {
    void *sx, *sy, *sz;       // colour-major planes (library layout): the current state
    void *ax, *ay, *az;       // second buffer set the fused sweep writes (null if none)
    int32_t Lx, Ly, Lz;       // cells
    int32_t Lxh;              // sc: Lx/2 (packed row length); basis kinds: Lx
    uint32_t pmask;           // periodic axes
    uint32_t rid;             // replica id (Philox counter word 1)
    uint32_t n_box;           // sites in the box (all colours)
    uint32_t plane;           // elements per colour (sc: N/2, basis: Lx*Ly*Lz)
    double J, K;
    double e[3];              // unit easy axis
    double beta;              // 1/T (0 for T = +inf)
    int32_t greedy;           // T == 0
    int32_t sphere;           // 1 if a sphere mask applies
    double r2x4;              // 4 R^2 (half-cell units squared)
    uint32_t item_begin, item_end; // this replica's range in the work list
};

// One workgroup's work: replica and the origin of its tile.
struct alignas(16) WorkItem {
    uint32_t rep;
    int32_t x0, y0, z0;
};

// Observable slots accumulated per workgroup and pass (FP64).
enum : int { Q_MX = 0, Q_MY, Q_MZ, Q_PE2, Q_SH, Q_NACC, Q_N };
constexpr int NQ = 8; // padded slot width (doubles)

// Workgroups per replica in the first stage of the observable finalise.
constexpr uint32_t FIN_BLOCKS = 32;

// Record written by the finalise kernel (FP64), per replica per measured sweep.
enum : int { R_MX = 0, R_MY, R_MZ, R_EEX, R_EAN, R_NACC, R_SWEEP, R_N };
constexpr int NR = 8;

// Kernel variants of a colour pass.
enum : int32_t {
    KERNEL_TILE = 0,  // one site per thread per plane, tx x ty threads (any lattice kind)
    KERNEL_STRIP = 1, // sc only: tx threads along a row (multiple of 64), ty rows per thread
    KERNEL_BAND = 2,  // sc only: tx threads over (band, column) positions, ty (even) rows per band
    KERNEL_LDS = 3,   // whole sweeps in LDS, one workgroup of tx threads per replica (small lattices)
    KERNEL_PAIR = 4,  // sc only, even packed rows: as KERNEL_STRIP with two columns per thread
    KERNEL_PBAND = 5, // sc only, even packed rows: as KERNEL_BAND with two columns per thread
    KERNEL_BSTRIP = 6, // bcc / fcc: tx (multiple of 64) lanes along x, ty rows, planes in registers
    KERNEL_BPAIR = 7,  // bcc / fcc, even Lx: tx threads over (band, pair) positions, ty rows per band
    KERNEL_LBAND = 8,  // sc only, 16-byte rows: tiles of ty whole rows, rows staged through LDS
    KERNEL_FUSED = 9,  // sc only, even packed rows: both colours in one launch, tiles of ty
                       // whole rows (tx = 256 threads), next state into the second buffer set
};

// LDS elements of one stage of the LDS-staged band kernel for tiles of br rows
// of lxh packed columns: the other colour's rows y0-1 .. y0+br and the own
// colour's rows, three components each (two stages are held).
// Chunks of 16 bytes per component of a staged buffer of `rows` rows of lxh
// elements of esz bytes, padded to a multiple of 64 (one wave's copy).
constexpr uint32_t lband_comp_chunks(int rows, int lxh, int esz)
{
    return ((uint32_t)rows * (uint32_t)lxh * (uint32_t)esz / 16u + 63u) / 64u * 64u;
}
// Bytes of dynamic LDS of a workgroup (two stages of other and own rows).
constexpr uint32_t lband_lds_bytes(int br, int lxh, int esz)
{
    return 2u * 3u * 16u * (lband_comp_chunks(br + 2, lxh, esz) + lband_comp_chunks(br, lxh, esz));
}
// Dynamic LDS of the fused sweep kernel: two planes of new colour-0 spins,
// rows y0-1 .. y0+br of lxh packed columns, three components.
constexpr uint32_t fused_lds_bytes(int br, int lxh, int esz)
{
    return 6u * (uint32_t)(br + 2) * (uint32_t)lxh * (uint32_t)esz;
}
// (row, pair) positions per lane of the fused sweep kernel (tx threads).
constexpr int fused_positions(int br, int lxh, int tx)
{
    return ((br + 2) * (lxh / 2) + tx - 1) / tx;
}
// Copy slots per lane and buffer (chunk groups of 64 over 4 waves).
constexpr int LBAND_SLOTS = 6;
constexpr int lband_slots_needed(int rows, int lxh, int esz, int n_waves)
{
    return (int)((3u * lband_comp_chunks(rows, lxh, esz) / 64u + (uint32_t)n_waves - 1) / (uint32_t)n_waves);
}

// Tile of one workgroup: tx row columns x ty rows x zc planes, and the kernel
// that maps it onto threads.
struct Tile {
    int32_t kernel, tx, ty, zc;
};

} // namespace mc
