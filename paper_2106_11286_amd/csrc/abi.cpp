// abi.cpp -- host runtime behind the C ABI (include/mcheis.h): argument and
// buffer validation, the colouring/tiling plan, the scratch layout, sweep
// scheduling with HIP graph replay and persistent launches, observable
// records and the temperature schedule.  The autotuner, the series
// statistics and the extensions (replica exchange, block scheme) live in
// abi_tune.cpp, abi_stats.cpp and abi_extensions.cpp.
//
// The library allocates no spin or scratch memory: the caller owns both (in
// practice as framework tensors) and the stream.  The only allocation it makes
// is a small pinned host ring for observable records.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <new>
#include <string>
#include <vector>

#include "abi_internal.h"

namespace mcabi {

thread_local std::string g_err;

mc_status fail(mc_status s, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

int n_basis(int kind) { return kind == SC ? 1 : (kind == BCC ? 2 : 4); }
int n_colours_of(int kind) { return kind == SC ? 2 : n_basis(kind); }

uint64_t align_up(uint64_t v, uint64_t a) { return (v + a - 1) / a * a; }

mc_status check_desc(const mc_replica_desc &d, int idx)
{
    if (d.kind < MC_SC || d.kind > MC_FCC)
        return fail(MC_E_ARG, "replica %d: unknown lattice kind %d", idx, d.kind);
    if (d.Lx < 1 || d.Ly < 1 || d.Lz < 1)
        return fail(MC_E_ARG, "replica %d: lengths must be >= 1 (got %d %d %d)", idx, d.Lx,
                    d.Ly, d.Lz);
    if (d.periodic_mask > 7u) return fail(MC_E_ARG, "replica %d: periodic_mask > 7", idx);
    if (!(d.T >= 0.0)) return fail(MC_E_ARG, "replica %d: T must be >= 0 (got %g)", idx, d.T);
    if (!std::isfinite(d.J) || !std::isfinite(d.K))
        return fail(MC_E_ARG, "replica %d: J and K must be finite", idx);
    const double en = std::sqrt(d.e[0] * d.e[0] + d.e[1] * d.e[1] + d.e[2] * d.e[2]);
    if (!(en > 0.0) || !std::isfinite(en))
        return fail(MC_E_ARG, "replica %d: easy axis must be nonzero and finite", idx);
    if (std::isnan(d.sphere_radius)) return fail(MC_E_ARG, "replica %d: sphere_radius is NaN", idx);
    const double nbox = (double)d.Lx * d.Ly * d.Lz * n_basis(d.kind);
    if (nbox >= 2147483647.0)
        return fail(MC_E_UNSUPPORTED, "replica %d: box of %.0f sites exceeds 2^31", idx, nbox);
    if (d.kind == MC_SC) {
        if (d.Lx % 2)
            return fail(MC_E_UNSUPPORTED, "replica %d: simple cubic needs even Lx (colour packing)",
                        idx);
        const int L[3] = {d.Lx, d.Ly, d.Lz};
        for (int a = 0; a < 3; ++a)
            if ((d.periodic_mask >> a & 1u) && (L[a] % 2))
                return fail(MC_E_UNSUPPORTED,
                            "replica %d: simple cubic with odd periodic length on axis %d cannot "
                            "be two-coloured",
                            idx, a);
    }
    return MC_OK;
}

uint64_t box_sites(const mc_replica_desc &d)
{
    return (uint64_t)d.Lx * d.Ly * d.Lz * n_basis(d.kind);
}

bool site_occupied(const mc_replica_desc &d, int x, int y, int z, int b)
{
    if (!(d.sphere_radius > 0.0)) return true;
    static const int B2[3][4][3] = {{{0, 0, 0}},
                                    {{0, 0, 0}, {1, 1, 1}},
                                    {{0, 0, 0}, {1, 1, 0}, {1, 0, 1}, {0, 1, 1}}};
    const int64_t qx = 2 * (int64_t)x + B2[d.kind][b][0] - d.Lx;
    const int64_t qy = 2 * (int64_t)y + B2[d.kind][b][1] - d.Ly;
    const int64_t qz = 2 * (int64_t)z + B2[d.kind][b][2] - d.Lz;
    return (double)(qx * qx + qy * qy + qz * qz) <= 4.0 * d.sphere_radius * d.sphere_radius;
}

uint64_t count_occupied(const mc_replica_desc &d)
{
    if (!(d.sphere_radius > 0.0)) return box_sites(d);
    uint64_t n = 0;
    const int nb = n_basis(d.kind);
    for (int z = 0; z < d.Lz; ++z)
        for (int y = 0; y < d.Ly; ++y)
            for (int x = 0; x < d.Lx; ++x)
                for (int b = 0; b < nb; ++b) n += site_occupied(d, x, y, z, b);
    return n;
}

int row_len(const mc_replica_desc &d) { return d.kind == MC_SC ? d.Lx / 2 : d.Lx; }

int pow2_at_least(int v)
{
    int p = 1;
    while (p < v) p <<= 1;
    return p;
}

// Workgroup tiles covering one z plane of a replica.
uint64_t xy_tiles(const mc_replica_desc &d, const Tile &t)
{
    if (t.kernel == KERNEL_BAND || t.kernel == KERNEL_PBAND || t.kernel == KERNEL_BPAIR) {
        const int cols = t.kernel == KERNEL_BAND ? row_len(d) : row_len(d) / 2;
        const uint64_t F = (uint64_t)((d.Ly + t.ty - 1) / t.ty) * cols;
        return (F + t.tx - 1) / t.tx;
    }
    if (t.kernel == KERNEL_LBAND || t.kernel == KERNEL_FUSED)
        return (uint64_t)((d.Ly + t.ty - 1) / t.ty);
    const int wx = t.kernel == KERNEL_PAIR ? 2 * t.tx : t.tx; // packed columns per tile
    return (uint64_t)((row_len(d) + wx - 1) / wx) * ((d.Ly + t.ty - 1) / t.ty);
}

// Planes per workgroup so that a pass has about kTargetItems workgroups.
int z_chunk(const mc_replica_desc *reps, int n, const Tile &t)
{
    uint64_t cols = 0, planes = 0;
    for (int r = 0; r < n; ++r) {
        cols += xy_tiles(reps[r], t) * reps[r].Lz;
        planes = std::max<uint64_t>(planes, reps[r].Lz);
    }
    const uint64_t zc = (cols + kTargetItems - 1) / kTargetItems;
    return (int)std::max<uint64_t>(1, std::min<uint64_t>(zc, planes));
}

// Whether the LDS-staged band kernel takes every replica (rows a multiple of
// 16 bytes, a workgroup's rows within two positions per thread, its LDS and
// copy slots within the limits) with tiles that fill one workgroup.
bool lband_default(const mc_replica_desc *reps, int n, size_t esz, int W)
{
    for (int r = 0; r < n; ++r)
        if ((uint64_t)row_len(reps[r]) * esz % 16u) return false;
    const int ty = std::max(1, std::min(64, 256 / std::max(1, W / 2)));
    return (ty * (W / 2) + 255) / 256 <= 2 && lband_lds_bytes(ty, W, (int)esz) <= 61440u &&
           lband_slots_needed(ty + 2, W, (int)esz, 4) <= LBAND_SLOTS;
}

// Default pass kernel and tile for replicas whose spins have `esz`-byte
// elements.
Tile default_tile(const mc_replica_desc *reps, int n, size_t esz)
{
    int W = 1, Ly = 1, Wmin = 1 << 30;
    for (int r = 0; r < n; ++r) {
        W = std::max(W, row_len(reps[r]));
        Wmin = std::min(Wmin, row_len(reps[r]));
        Ly = std::max(Ly, reps[r].Ly);
    }
    Tile t;
    bool sphere = false; // only the tile kernel masks unoccupied simple-cubic sites
    for (int r = 0; r < n; ++r) sphere |= reps[r].kind == MC_SC && reps[r].sphere_radius > 0.0;
    bool fits = !sphere; // the strip kernel addresses each component array with 32-bit offsets
    for (int r = 0; r < n; ++r) fits &= box_sites(reps[r]) * esz <= 0xFFFFFFFFull;
    bool even = true; // every row holds an even number of packed columns (sc) or cells
    for (int r = 0; r < n; ++r) even &= row_len(reps[r]) % 2 == 0;
    if (reps[0].kind == MC_SC && fits && even && Wmin >= 96) {
        // long rows: two columns per thread, 2 rows per thread, whole rows
        // (up to 512 columns) per workgroup
        t.kernel = KERNEL_PAIR;
        t.tx = std::min(256, ((W + 1) / 2 + 63) / 64 * 64);
        t.ty = 2;
    } else if (reps[0].kind == MC_SC && fits) {
        // bands of 2 rows, (band, column) positions dealt to 256 threads
        t.kernel = KERNEL_BAND;
        t.tx = 256;
        t.ty = 2;
    } else if (reps[0].kind == MC_SC && !sphere && lband_default(reps, n, esz, W)) {
        // arrays beyond the 32-bit offsets of the buffer kernels: whole rows
        // staged through LDS, 64-bit addresses
        t.kernel = KERNEL_LBAND;
        t.tx = 256;
        t.ty = std::max(1, std::min(64, 256 / std::max(1, W / 2)));
    } else if (reps[0].kind != MC_SC && fits && even) {
        // bcc / fcc: bands of cell pairs (fcc keeps one row per band: three
        // other bases' rows in registers)
        t.kernel = KERNEL_BPAIR;
        t.tx = 256;
        t.ty = reps[0].kind == MC_FCC ? 1 : 2;
    } else {
        t.kernel = KERNEL_TILE;
        t.tx = std::min(64, pow2_at_least(W));
        t.ty = std::min(256 / t.tx, pow2_at_least(Ly));
    }
    t.zc = z_chunk(reps, n, t);
    return t;
}

mc_status check_tile(const Tile &t, int kind, uint64_t max_component_bytes, bool f64)
{
    if (t.kernel == KERNEL_BAND) {
        if (kind != MC_SC) return fail(MC_E_ARG, "the band kernel is for simple cubic lattices");
        if (max_component_bytes > 0xFFFFFFFFull)
            return fail(MC_E_UNSUPPORTED, "band kernel: a spin component array exceeds 4 GiB");
        if (t.tx < 64 || t.tx > 256 || t.tx % 64)
            return fail(MC_E_ARG, "band tile: tx must be 64, 128, 192 or 256 (got %d)", t.tx);
        if (t.ty != 2 && t.ty != 4)
            return fail(MC_E_ARG, "band tile: ty (rows per band) must be 2 or 4");
    } else if (t.kernel == KERNEL_PBAND) {
        if (kind != MC_SC) return fail(MC_E_ARG, "the band-pair kernel is for simple cubic lattices");
        if (max_component_bytes > 0xFFFFFFFFull)
            return fail(MC_E_UNSUPPORTED, "band-pair kernel: a spin component array exceeds 4 GiB");
        if (t.tx < 64 || t.tx > 256 || t.tx % 64)
            return fail(MC_E_ARG, "band-pair tile: tx must be 64, 128, 192 or 256 (got %d)", t.tx);
        if (t.ty != 2 && t.ty != 4)
            return fail(MC_E_ARG, "band-pair tile: ty (rows per band) must be 2 or 4");
        if (f64 && t.ty == 4)
            return fail(MC_E_UNSUPPORTED, "band-pair tile: FP64 takes bands of 2 rows (4-row bands "
                                          "need more than the 256 registers of a lane)");
    } else if (t.kernel == KERNEL_PAIR) {
        if (kind != MC_SC) return fail(MC_E_ARG, "the pair kernel is for simple cubic lattices");
        if (max_component_bytes > 0xFFFFFFFFull)
            return fail(MC_E_UNSUPPORTED, "pair kernel: a spin component array exceeds 4 GiB");
        if (t.tx < 64 || t.tx > 256 || t.tx % 64)
            return fail(MC_E_ARG, "pair tile: tx must be 64, 128, 192 or 256 (got %d)", t.tx);
        if (t.ty != 1 && t.ty != 2 && t.ty != 4)
            return fail(MC_E_ARG, "pair tile: ty (rows per thread) must be 1, 2 or 4");
    } else if (t.kernel == KERNEL_STRIP) {
        if (kind != MC_SC) return fail(MC_E_ARG, "the strip kernel is for simple cubic lattices");
        if (max_component_bytes > 0xFFFFFFFFull)
            return fail(MC_E_UNSUPPORTED, "strip kernel: a spin component array exceeds 4 GiB");
        if (t.tx < 64 || t.tx > 256 || t.tx % 64)
            return fail(MC_E_ARG, "strip tile: tx must be 64, 128, 192 or 256 (got %d)", t.tx);
        if (t.ty != 1 && t.ty != 2 && t.ty != 4 && t.ty != 8)
            return fail(MC_E_ARG, "strip tile: ty (rows per thread) must be 1, 2, 4 or 8");
    } else if (t.kernel == KERNEL_BPAIR) {
        if (kind == MC_SC) return fail(MC_E_ARG, "the basis pair kernel is for bcc and fcc lattices");
        if (max_component_bytes > 0xFFFFFFFFull)
            return fail(MC_E_UNSUPPORTED, "basis pair kernel: a spin component array exceeds 4 GiB");
        if (t.tx < 64 || t.tx > 256 || t.tx % 64)
            return fail(MC_E_ARG, "basis pair tile: tx must be 64, 128, 192 or 256 (got %d)", t.tx);
        if (t.ty != 1 && t.ty != 2)
            return fail(MC_E_ARG, "basis pair tile: ty (rows per band) must be 1 or 2");
    } else if (t.kernel == KERNEL_BSTRIP) {
        if (kind == MC_SC) return fail(MC_E_ARG, "the basis strip kernel is for bcc and fcc lattices");
        if (t.tx < 64 || t.tx > 256 || t.tx % 64 || t.ty < 1 || t.tx * t.ty > 256)
            return fail(MC_E_ARG, "basis strip tile: tx must be 64, 128, 192 or 256 and tx*ty <= 256");
    } else if (t.kernel == KERNEL_LBAND) {
        if (kind != MC_SC) return fail(MC_E_ARG, "the LDS-staged band kernel is for simple cubic lattices");
        if (t.tx != 256) return fail(MC_E_ARG, "LDS-staged band tile: tx must be 256 (got %d)", t.tx);
        if (t.ty < 1 || t.ty > 64)
            return fail(MC_E_ARG, "LDS-staged band tile: ty (rows per tile) must be in [1, 64]");
        (void)max_component_bytes;
    } else if (t.kernel == KERNEL_FUSED) {
        if (kind != MC_SC) return fail(MC_E_ARG, "the fused sweep kernel is for simple cubic lattices");
        if (max_component_bytes > 0xFFFFFFFFull)
            return fail(MC_E_UNSUPPORTED, "fused sweep kernel: a spin component array exceeds 4 GiB");
        if (t.tx != 256 && t.tx != 512 && t.tx != 1024)
            return fail(MC_E_ARG, "fused sweep tile: tx must be 256, 512 or 1024 (got %d)", t.tx);
        if (t.ty < 1 || t.ty > 64)
            return fail(MC_E_ARG, "fused sweep tile: ty (rows per tile) must be in [1, 64]");
    } else if (t.kernel == KERNEL_TILE) {
        if (t.tx < 1 || t.ty < 1 || t.tx * t.ty > 256)
            return fail(MC_E_ARG, "tile %d x %d invalid (need >= 1 and tx*ty <= 256)", t.tx, t.ty);
    } else {
        return fail(MC_E_ARG, "unknown kernel %d", t.kernel);
    }
    if (t.zc < 1) return fail(MC_E_ARG, "zc must be >= 1");
    return MC_OK;
}

// minimum of q^2 for q in [lo, hi]
int64_t min_sq(int64_t lo, int64_t hi)
{
    if (lo <= 0 && hi >= 0) return 0;
    const int64_t a = lo > 0 ? lo : -hi;
    return a * a;
}

// Tiles of every replica in (z, x, y) order (y fastest, so that tiles sharing
// halo rows are adjacent); fully unoccupied tiles dropped.
void make_work(const mc_replica_desc *reps, int n, const Tile &t, std::vector<WorkItem> &work,
               std::vector<uint32_t> &begin, std::vector<uint32_t> &end)
{
    work.clear();
    begin.assign(n, 0);
    end.assign(n, 0);
    for (int r = 0; r < n; ++r) {
        const mc_replica_desc &d = reps[r];
        begin[r] = (uint32_t)work.size();
        const int W = row_len(d);
        const bool sc = d.kind == MC_SC;
        if (t.kernel == KERNEL_BAND || t.kernel == KERNEL_PBAND || t.kernel == KERNEL_BPAIR) {
            const int rows = t.ty;
            const int cols = t.kernel == KERNEL_BAND ? W : W / 2; // positions per row
            const int F = (d.Ly + rows - 1) / rows * cols;
            for (int z0 = 0; z0 < d.Lz; z0 += t.zc)
                for (int f0 = 0; f0 < F; f0 += t.tx) {
                    if (d.sphere_radius > 0.0) {
                        const int y0 = f0 / cols * rows;
                        const int y1 = std::min(d.Ly, ((f0 + t.tx - 1) / cols + 1) * rows) - 1;
                        const int cz1 = std::min(d.Lz, z0 + t.zc) - 1;
                        const int64_t m = min_sq(-d.Lx, d.Lx - 1) +
                                          min_sq(2 * y0 - d.Ly, 2 * y1 + 1 - d.Ly) +
                                          min_sq(2 * z0 - d.Lz, 2 * cz1 + 1 - d.Lz);
                        if ((double)m > 4.0 * d.sphere_radius * d.sphere_radius) continue;
                    }
                    work.push_back(WorkItem{(uint32_t)r, f0, 0, z0});
                }
            end[r] = (uint32_t)work.size();
            continue;
        }
        if (t.kernel == KERNEL_LBAND || t.kernel == KERNEL_FUSED) { // whole rows: tiles of ty rows
            for (int z0 = 0; z0 < d.Lz; z0 += t.zc)
                for (int y0 = 0; y0 < d.Ly; y0 += t.ty) work.push_back(WorkItem{(uint32_t)r, 0, y0, z0});
            end[r] = (uint32_t)work.size();
            continue;
        }
        const int wx = t.kernel == KERNEL_PAIR ? 2 * t.tx : t.tx; // packed columns per tile
        for (int z0 = 0; z0 < d.Lz; z0 += t.zc)
            for (int x0 = 0; x0 < W; x0 += wx)
                for (int y0 = 0; y0 < d.Ly; y0 += t.ty) {
                    if (d.sphere_radius > 0.0) {
                        // cells covered, then half-unit site positions relative to the centre
                        const int cx0 = sc ? 2 * x0 : x0;
                        const int cx1 = sc ? std::min(d.Lx, 2 * (x0 + wx)) - 1
                                           : std::min(d.Lx, x0 + wx) - 1;
                        const int cy1 = std::min(d.Ly, y0 + t.ty) - 1;
                        const int cz1 = std::min(d.Lz, z0 + t.zc) - 1;
                        const int64_t m = min_sq(2 * cx0 - d.Lx, 2 * cx1 + 1 - d.Lx) +
                                          min_sq(2 * y0 - d.Ly, 2 * cy1 + 1 - d.Ly) +
                                          min_sq(2 * z0 - d.Lz, 2 * cz1 + 1 - d.Lz);
                        if ((double)m > 4.0 * d.sphere_radius * d.sphere_radius) continue;
                    }
                    work.push_back(WorkItem{(uint32_t)r, x0, y0, z0});
                }
        end[r] = (uint32_t)work.size();
    }
}

ScratchLayout scratch_layout(int n_reps, uint64_t n_items, int n_colours)
{
    ScratchLayout L;
    uint64_t o = 0;
    L.off_ctr = o;
    o += 256;
    L.off_reps = o;
    o = align_up(o + sizeof(RepDev) * n_reps, 256);
    // replica exchange: beta[n], attempted[n], accepted[n] (8 bytes each),
    // rep_at[n], round; placed before every region that depends on the work
    // list, so a tile change does not move it
    L.off_exchange = o;
    o = align_up(o + 24ull * n_reps + 4ull * n_reps + 4, 256);
    L.off_work = o;
    o = align_up(o + sizeof(WorkItem) * std::max<uint64_t>(n_items, 1), 256);
    L.off_partials = o;
    o = align_up(o + sizeof(double) * NQ * n_colours * std::max<uint64_t>(n_items, 1), 256);
    L.off_records = o;
    // ring of records plus one slot for from-scratch measurements
    o = align_up(o + sizeof(double) * NR * n_reps * (kRing + 1), 256);
    L.off_stage = o;
    o = align_up(o + sizeof(double) * NQ * FIN_BLOCKS * n_reps, 256);
    L.off_persist = o;
    o = align_up(o + sizeof(uint32_t) * persist_state_words(n_reps), 256);
    L.off_queues = o;
    o = align_up(o + sizeof(uint32_t) * queue_words(n_items), 256);
    // partials of the from-scratch measurement (mc_measure_state)
    L.off_measure = o;
    o = align_up(o + sizeof(double) * 8 * MEASURE_BLOCKS, 256);
    L.total = o;
    return L;
}

mc_status check_device_buffer(const void *p, uint64_t bytes, const char *what, int rep)
{
    if (!p) return fail(MC_E_BUFFER, "replica %d: %s is NULL", rep, what);
    if (reinterpret_cast<uintptr_t>(p) % 16)
        return fail(MC_E_BUFFER, "replica %d: %s is not 16-byte aligned", rep, what);
    hipPointerAttribute_t attr;
    std::memset(&attr, 0, sizeof attr);
    hipError_t e = hipPointerGetAttributes(&attr, p);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(MC_E_BUFFER, "replica %d: %s is not HIP memory (%s)", rep, what,
                    hipGetErrorString(e));
    }
    if (attr.type != hipMemoryTypeDevice)
        return fail(MC_E_BUFFER, "replica %d: %s is not device memory", rep, what);
    hipDeviceptr_t base = nullptr;
    size_t size = 0;
    e = hipMemGetAddressRange(&base, &size, (hipDeviceptr_t)p);
    if (e == hipSuccess && base) {
        const uint64_t avail = (uint64_t)((const char *)base + size - (const char *)p);
        if (avail < bytes)
            return fail(MC_E_BUFFER, "replica %d: %s holds %llu bytes, %llu needed", rep, what,
                        (unsigned long long)avail, (unsigned long long)bytes);
    } else {
        (void)hipGetLastError();
    }
    return MC_OK;
}

} // namespace mcabi


namespace mcabi {

bool alive(const mc_sim *h) { return h && h->magic == 0x4d434831u; }

PassLaunch pass_args(mc_sim *h, uint32_t item_base, uint32_t n_blocks, uint32_t t_off)
{
    PassLaunch p;
    p.reps_dev = h->reps_dev;
    p.work_dev = h->work_dev;
    p.item_base = item_base;
    p.n_blocks = n_blocks;
    p.n_items = (uint32_t)h->work.size();
    p.tctr_dev = h->tctr;
    p.t_off = t_off;
    p.seed_lo = (uint32_t)h->seed;
    p.seed_hi = (uint32_t)(h->seed >> 32);
    p.tile = h->pass_tile;
    p.partials_dev = h->partials;
    p.dbg_dh = nullptr;
    p.dbg_acc = nullptr;
    p.lds_bytes = 0;
    p.lds_positions = 0;
    if (p.tile.kernel == KERNEL_LBAND) {
        int w = 1;
        for (const auto &d : h->desc) w = std::max(w, row_len(d));
        const int esz = h->prec == MC_F64 ? 8 : 4;
        p.lds_bytes = lband_lds_bytes(p.tile.ty, w, esz);
        p.lds_positions = (p.tile.ty * (w / 2) + p.tile.tx - 1) / p.tile.tx;
    }
    if (p.tile.kernel == KERNEL_FUSED) {
        int w = 1;
        for (const auto &d : h->desc) w = std::max(w, row_len(d));
        p.lds_bytes = fused_lds_bytes(p.tile.ty, w, h->prec == MC_F64 ? 8 : 4);
        p.lds_positions = fused_positions(p.tile.ty, w, p.tile.tx);
    }
    return p;
}

// LDS bytes the LDS kernel needs: three component planes of the largest replica.
uint64_t lds_need(const mc_sim *h)
{
    const uint64_t esz = h->prec == MC_F64 ? sizeof(double) : sizeof(float);
    uint64_t m = 0;
    for (const RepDev &R : h->reps) m = std::max<uint64_t>(m, 3ull * R.n_box * esz);
    return m;
}

bool sc_sphere(const mc_sim *h)
{
    if (h->kind != MC_SC) return false;
    for (const auto &d : h->desc)
        if (d.sphere_radius > 0.0) return true;
    return false;
}

bool lds_fits(const mc_sim *h) { return h->lds_max > 0 && lds_need(h) <= h->lds_max; }

// Threads of the default LDS tile: one per site of a colour, 64 .. 1024.
int lds_threads(const mc_sim *h)
{
    uint32_t m = 64;
    for (const RepDev &R : h->reps) m = std::max<uint32_t>(m, R.plane);
    return (int)std::min<uint32_t>(1024, (m + 63) / 64 * 64);
}

// n whole sweeps of every replica by the LDS kernel, then the counter advance.
mc_status enqueue_lds(mc_sim *h, uint32_t n, bool measure, uint32_t slot0)
{
    LdsLaunch L;
    L.reps_dev = h->reps_dev;
    L.n_reps = (uint32_t)h->n_reps;
    L.n_sweeps = n;
    L.tctr_dev = h->tctr;
    L.seed_lo = (uint32_t)h->seed;
    L.seed_hi = (uint32_t)(h->seed >> 32);
    L.records = h->records;
    L.ring = kRing;
    L.slot0 = slot0;
    L.lds_bytes = (uint32_t)lds_need(h);
    HIP_TRY(launch_lds(h->kind, h->prec == MC_F64, measure, L, h->tile.tx, h->stream));
    HIP_TRY(launch_advance(h->tctr, n, h->stream));
    return MC_OK;
}

// Enqueue n sweeps (passes, optional finalise into ring slots slot0.., then
// the counter advance).  Pure launches: safe inside stream capture.
mc_status enqueue_sweeps(mc_sim *h, uint32_t n, bool measure, uint32_t slot0)
{
    if (h->tile.kernel == KERNEL_LDS) return enqueue_lds(h, n, measure, slot0);
    const bool f64 = h->prec == MC_F64;
    const uint32_t n_items = (uint32_t)h->work.size();
    const bool fused = h->tile.kernel == KERNEL_FUSED;
    for (uint32_t i = 0; i < n; ++i) {
        const PassLaunch p = pass_args(h, 0, n_items, i);
        if (fused) {
            HIP_TRY(launch_fused(f64, measure, p, h->stream));
            HIP_TRY(launch_swap_state(h->reps_dev, (uint32_t)h->n_reps, h->stream));
        } else {
            for (int c = 0; c < h->n_colours; ++c)
                HIP_TRY(launch_pass(h->kind, f64, c, measure, 0, p, h->stream));
        }
        if (measure) {
            const uint32_t slot = (slot0 + i) % kRing;
            HIP_TRY(launch_finalize(h->reps_dev, h->n_reps, h->n_colours, h->partials, n_items,
                                    h->tctr, i, h->records + (size_t)slot * h->n_reps * NR,
                                    h->stage, h->stream));
        }
    }
    HIP_TRY(launch_advance(h->tctr, n, h->stream));
    return MC_OK;
}

// Whether the device deals workgroups to its eight XCDs in turn (workgroup b
// on XCD b mod 8), checked once per device with a 64-workgroup launch that
// records each workgroup's XCD.  `buf` holds at least 64 words.
bool device_deals_xcds(mc_sim *h, uint32_t *buf)
{
    static std::mutex mu;
    static signed char known[64];
    static bool init = false;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) {
        (void)hipGetLastError();
        return false;
    }
    std::lock_guard<std::mutex> lock(mu);
    if (!init) {
        std::memset(known, -1, sizeof known);
        init = true;
    }
    if (known[dev] >= 0) return known[dev] == 1;
    uint32_t v[64];
    bool ok = launch_xcd_probe(buf, 64, h->stream) == hipSuccess &&
              hipMemcpyAsync(v, buf, sizeof v, hipMemcpyDeviceToHost, h->stream) == hipSuccess &&
              hipStreamSynchronize(h->stream) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        return false; // not cached: a later handle checks again
    }
    for (uint32_t b = 0; b < 64; ++b) ok = ok && v[b] == b % 8;
    known[dev] = ok ? 1 : 0;
    return ok;
}

// Deal the replicas to the persistent-launch queues (see
// mc_set_persistent_mode) and upload the queue table.  Asynchronous on the
// handle's stream; h->q_host stays alive until the next call.
mc_status plan_queues(mc_sim *h)
{
    const int n = h->n_reps;
    std::vector<uint64_t> load(n);
    uint64_t sum = 0;
    for (int r = 0; r < n; ++r) {
        load[r] = h->reps[r].item_end - h->reps[r].item_begin;
        sum += load[r];
    }
    std::vector<int> order(n), home(n, 0);
    for (int r = 0; r < n; ++r) order[r] = r;
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return load[a] > load[b]; });
    uint64_t q_load[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int r : order) {
        int g = 0;
        for (int k = 1; k < 8; ++k)
            if (q_load[k] < q_load[g]) g = k;
        home[r] = g;
        q_load[g] += load[r];
    }
    const uint64_t max_load = *std::max_element(q_load, q_load + 8);
    bool xcd = false;
    if (h->persist_mode == MC_PERSIST_XCD) xcd = true;
    else if (h->persist_mode == MC_PERSIST_AUTO)
        xcd = h->xcd_ok && n >= 8 && 8 * max_load * 4 <= sum * 5; // max <= 1.25 x mean
    h->n_queues = xcd ? 8 : 1;
    h->max_queue_items = xcd ? (uint32_t)max_load : (uint32_t)sum;
    h->q_host.assign(16 + h->work.size(), 0u);
    uint32_t pos = 0;
    for (int g = 0; g < 8; ++g) {
        h->q_host[g] = pos;
        for (int r = 0; r < n; ++r)
            if (home[r] == g)
                for (uint32_t it = h->reps[r].item_begin; it < h->reps[r].item_end; ++it)
                    h->q_host[16 + pos++] = it;
    }
    h->q_host[8] = pos;
    HIP_TRY(hipMemcpyAsync(h->queues_dev, h->q_host.data(), sizeof(uint32_t) * h->q_host.size(),
                           hipMemcpyHostToDevice, h->stream));
    return MC_OK;
}

// Tile shapes the persistent kernel is instantiated for.
bool persistent_supported(const Tile &t)
{
    if (t.kernel == KERNEL_LBAND || t.kernel == KERNEL_FUSED) return false;
    if (t.kernel == KERNEL_PAIR) return t.ty == 1 || t.ty == 2;
    if (t.kernel == KERNEL_PBAND) return t.ty == 2;
    if (t.kernel == KERNEL_BPAIR) return t.ty == 1 || t.ty == 2;
    return t.kernel != KERNEL_STRIP || t.ty == 2 || t.ty == 4;
}

// A persistent call with the LDS kernel is an LDS launch (already one launch
// for all n sweeps, with no device-scope synchronisation).

// n sweeps as one persistent launch (preceded by a counter reset, followed by
// the counter advance).  Pure launches: safe inside stream capture.
mc_status enqueue_persistent(mc_sim *h, uint32_t n, bool measure, uint32_t slot0)
{
    if (h->tile.kernel == KERNEL_LDS) return enqueue_lds(h, n, measure, slot0);
    if (!persistent_supported(h->tile))
        return fail(MC_E_UNSUPPORTED, "persistent sweeps: no kernel for this tile (%d rows "
                                      "per thread); use strips of 2 or 4 rows, pairs of 1 or "
                                      "2 rows, or another kernel", h->tile.ty);
    const uint32_t n_items = (uint32_t)h->work.size();
    if ((uint64_t)n * h->n_colours * n_items >= 0xFFFFFFFFull)
        return fail(MC_E_ARG, "persistent launch of %u sweeps exceeds 2^32 work units", n);
    PersistLaunch a;
    a.state = h->pstate;
    a.n_sweeps = n;
    a.n_colours = (uint32_t)h->n_colours;
    a.n_reps = (uint32_t)h->n_reps;
    a.spin_limit = h->spin_limit;
    a.records = h->records;
    a.ring = kRing;
    a.slot0 = slot0;
    a.n_queues = h->n_queues;
    a.max_queue_items = h->max_queue_items;
    a.q_off = h->queues_dev;
    a.q_items = h->queues_dev + 16;
    // clear the per-launch words (the sticky ones stay until read)
    HIP_TRY(launch_zero_u32(h->pstate + PS_ABORT, persist_state_words(h->n_reps) - PS_ABORT,
                            h->stream));
    HIP_TRY(launch_persistent(h->kind, h->prec == MC_F64, measure, pass_args(h, 0, n_items, 0), a,
                              h->stream));
    HIP_TRY(launch_persist_check(a, n_items, h->stream));
    HIP_TRY(launch_advance(h->tctr, n, h->stream));
    h->persist_used = true;
    return MC_OK;
}

// After a synchronisation: report a persistent launch whose bounded wait gave
// up (the spins of that call are then incomplete).
mc_status check_persistent(mc_sim *h)
{
    if (!h->persist_used) return MC_OK;
    uint32_t hdr[2] = {0, 0};
    HIP_TRY(hipMemcpy(hdr, h->pstate, sizeof hdr, hipMemcpyDeviceToHost));
    h->persist_used = false;
    if (hdr[PS_STICKY_WATCHDOG] || hdr[PS_STICKY_UNDRAINED]) {
        HIP_TRY(launch_zero_u32(h->pstate, 2, h->stream));
        HIP_TRY(hipStreamSynchronize(h->stream));
    }
    if (hdr[PS_STICKY_WATCHDOG])
        return fail(MC_E_DEVICE, "persistent sweep: a wait for a replica's previous pass exceeded "
                                 "%u spins; the state of that call is incomplete",
                    h->spin_limit);
    if (hdr[PS_STICKY_UNDRAINED])
        return fail(MC_E_DEVICE, "persistent sweep: a work queue was left with unclaimed units "
                                 "(no workgroup ran on its XCD); the state of that call is "
                                 "incomplete");
    return MC_OK;
}

void record_to_obs(const mc_sim *h, const double *rec, int r, mc_obs *o)
{
    const double N = (double)h->n_occ[r];
    o->sweep = (uint64_t)rec[R_SWEEP];
    o->n_sites = h->n_occ[r];
    o->n_accepted = (uint64_t)rec[R_NACC];
    for (int a = 0; a < 3; ++a) o->M[a] = rec[R_MX + a] / N;
    o->absM = std::sqrt(o->M[0] * o->M[0] + o->M[1] * o->M[1] + o->M[2] * o->M[2]);
    o->E_exch = rec[R_EEX];
    o->E_anis = rec[R_EAN];
    o->E = o->E_exch + o->E_anis;
}

void set_temperature(RepDev &R, double T)
{
    R.greedy = T == 0.0;
    R.beta = (T > 0.0 && std::isfinite(T)) ? 1.0 / T : 0.0;
}

void fill_repdev(const mc_replica_desc &d, const mc_spin_buffers &b, RepDev &R)
{
    std::memset(&R, 0, sizeof R);
    R.sx = b.sx;
    R.sy = b.sy;
    R.sz = b.sz;
    R.Lx = d.Lx;
    R.Ly = d.Ly;
    R.Lz = d.Lz;
    R.Lxh = row_len(d);
    R.pmask = d.periodic_mask;
    R.rid = d.replica_id;
    R.n_box = (uint32_t)box_sites(d);
    R.plane = d.kind == MC_SC ? R.n_box / 2 : (uint32_t)d.Lx * d.Ly * d.Lz;
    R.J = d.J;
    R.K = d.K;
    const double en = std::sqrt(d.e[0] * d.e[0] + d.e[1] * d.e[1] + d.e[2] * d.e[2]);
    for (int a = 0; a < 3; ++a) R.e[a] = d.e[a] / en;
    set_temperature(R, d.T);
    R.sphere = d.sphere_radius > 0.0;
    R.r2x4 = 4.0 * d.sphere_radius * d.sphere_radius;
}

static_assert(sizeof(double) * 8 * MEASURE_BLOCKS <= MC_MEASURE_WORKSPACE_BYTES,
              "measurement partials exceed the documented workspace");

uint32_t measure_blocks(const RepDev &R)
{
    const uint64_t want = (R.n_box + 2047ull) / 2048ull;
    return (uint32_t)std::min<uint64_t>(MEASURE_BLOCKS, std::max<uint64_t>(1, want));
}

mc_status check_measure_args(const mc_replica_desc *d, mc_precision prec,
                             const mc_spin_buffers *bufs, const double *record_dev)
{
    if (!d || !bufs || !record_dev) return fail(MC_E_ARG, "NULL argument");
    if (prec != MC_F32 && prec != MC_F64) return fail(MC_E_ARG, "unknown precision %d", (int)prec);
    mc_status s = check_desc(*d, 0);
    if (s != MC_OK) return s;
    const uint64_t need = box_sites(*d);
    if (bufs->capacity_sites < need)
        return fail(MC_E_BUFFER, "capacity %llu < %llu sites",
                    (unsigned long long)bufs->capacity_sites, (unsigned long long)need);
    const size_t esz = prec == MC_F64 ? sizeof(double) : sizeof(float);
    const void *pl[3] = {bufs->sx, bufs->sy, bufs->sz};
    const char *nm[3] = {"sx", "sy", "sz"};
    for (int a = 0; a < 3; ++a)
        if ((s = check_device_buffer(pl[a], need * esz, nm[a], 0)) != MC_OK) return s;
    if (reinterpret_cast<uintptr_t>(record_dev) % 8)
        return fail(MC_E_BUFFER, "record is not 8-byte aligned");
    return check_device_buffer(record_dev, sizeof(double) * NR, "record", 0);
}

mc_status upload_reps(mc_sim *h)
{
    {
        mc_status s = xchg_pull(h);
        if (s != MC_OK) return s;
    }
    HIP_TRY(hipMemcpyAsync(h->reps_dev, h->reps.data(), sizeof(RepDev) * h->n_reps,
                           hipMemcpyHostToDevice, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    return MC_OK;
}


// The host copies of the replica descriptors follow the device ones: after an
// odd number of fused sweeps the two buffer sets have traded places.
void note_sweeps(mc_sim *h, uint64_t n)
{
    if (h->tile.kernel != KERNEL_FUSED || !(n & 1u)) return;
    for (RepDev &R : h->reps) {
        std::swap(R.sx, R.ax);
        std::swap(R.sy, R.ay);
        std::swap(R.sz, R.az);
    }
}

mc_status run_chunk(mc_sim *h, uint32_t n, bool measure, uint32_t slot0, bool persistent)
{
    if (n == 0) return MC_OK;
    if (!h->stream) {
        const mc_status s = persistent ? enqueue_persistent(h, n, measure, slot0)
                                       : enqueue_sweeps(h, n, measure, slot0);
        if (s == MC_OK) note_sweeps(h, n);
        return s;
    }
    // replay a captured graph of n sweeps; graphs bake the ring slots, so a
    // measured graph is keyed by its first slot too (callers use slot 0)
    const std::pair<uint32_t, uint32_t> key(n | (persistent ? 0x80000000u : 0u),
                                            measure ? 1u + slot0 : 0u);
    auto it = h->graphs.find(key);
    if (it == h->graphs.end()) {
        HIP_TRY(hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
        mc_status s = persistent ? enqueue_persistent(h, n, measure, slot0)
                                 : enqueue_sweeps(h, n, measure, slot0);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(h->stream, &g);
        if (s != MC_OK) {
            if (g) (void)hipGraphDestroy(g);
            return s;
        }
        if (e != hipSuccess) return fail(MC_E_DEVICE, "graph capture: %s", hipGetErrorString(e));
        hipGraphExec_t ex = nullptr;
        e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) return fail(MC_E_DEVICE, "graph instantiate: %s", hipGetErrorString(e));
        it = h->graphs.emplace(key, ex).first;
    }
    HIP_TRY(hipGraphLaunch(it->second, h->stream));
    note_sweeps(h, n);
    // the LDS kernel keeps no counters that a watchdog could trip
    if (persistent && h->tile.kernel != KERNEL_LDS) h->persist_used = true;
    return MC_OK;
}

} // namespace mcabi

using namespace mcabi;

extern "C" {

const char *mc_last_error(void) { return g_err.c_str(); }

const char *mc_version(void) { return "mcheis 0.1 (gfx950)"; }

mc_status mc_stream_probe(mc_precision prec, void *x, void *y, void *z, uint64_t half_elems,
                          uint32_t grid, uint32_t reps, void *hip_stream, double *ms)
{
    if (prec != MC_F32 && prec != MC_F64) return fail(MC_E_ARG, "unknown precision %d", (int)prec);
    if (!ms) return fail(MC_E_ARG, "ms is NULL");
    if (half_elems < 2 || half_elems % 2)
        return fail(MC_E_ARG, "half_elems must be even and >= 2");
    if (grid < 1 || grid > (1u << 20)) return fail(MC_E_ARG, "grid must be in [1, 2^20]");
    if (reps < 1) return fail(MC_E_ARG, "reps must be >= 1");
    const uint64_t bytes = 2 * half_elems * (prec == MC_F64 ? sizeof(double) : sizeof(float));
    void *pl[3] = {x, y, z};
    const char *nm[3] = {"x", "y", "z"};
    for (int a = 0; a < 3; ++a) {
        mc_status s = check_device_buffer(pl[a], bytes, nm[a], -1);
        if (s != MC_OK) return s;
    }
    hipStream_t st = (hipStream_t)hip_stream;
    const bool f64 = prec == MC_F64;
    HIP_TRY(launch_stream_probe(f64, x, y, z, half_elems, grid, st));
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    hipError_t err = hipEventRecord(e0, st);
    for (uint32_t r = 0; r < reps && err == hipSuccess; ++r)
        err = launch_stream_probe(f64, x, y, z, half_elems, grid, st);
    if (err == hipSuccess) err = hipEventRecord(e1, st);
    if (err == hipSuccess) err = hipEventSynchronize(e1);
    float t = 0.f;
    if (err == hipSuccess) err = hipEventElapsedTime(&t, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (err != hipSuccess) return fail(MC_E_DEVICE, "stream probe: %s", hipGetErrorString(err));
    *ms = (double)t / reps;
    return MC_OK;
}

mc_status mc_required_sites(const mc_replica_desc *d, uint64_t *sites)
{
    if (!d || !sites) return fail(MC_E_ARG, "NULL argument");
    mc_status s = check_desc(*d, 0);
    if (s != MC_OK) return s;
    *sites = box_sites(*d);
    return MC_OK;
}

mc_status mc_occupied_sites(const mc_replica_desc *d, uint64_t *n)
{
    if (!d || !n) return fail(MC_E_ARG, "NULL argument");
    mc_status s = check_desc(*d, 0);
    if (s != MC_OK) return s;
    *n = count_occupied(*d);
    return MC_OK;
}

mc_status mc_required_scratch(const mc_replica_desc *reps, int32_t n_reps, uint64_t *bytes)
{
    if (!reps || !bytes) return fail(MC_E_ARG, "NULL argument");
    if (n_reps < 1) return fail(MC_E_ARG, "n_reps must be >= 1");
    for (int r = 0; r < n_reps; ++r) {
        mc_status s = check_desc(reps[r], r);
        if (s != MC_OK) return s;
        if (reps[r].kind != reps[0].kind)
            return fail(MC_E_ARG, "replica %d: all replicas must share one lattice kind", r);
    }
    // the precision is not known here: the larger of the two default layouts
    uint64_t need = 0;
    for (size_t esz : {sizeof(float), sizeof(double)}) {
        const Tile t = default_tile(reps, n_reps, esz);
        std::vector<WorkItem> work;
        std::vector<uint32_t> b, e;
        make_work(reps, n_reps, t, work, b, e);
        need = std::max(need, scratch_layout(n_reps, work.size(), n_colours_of(reps[0].kind)).total);
    }
    *bytes = need;
    return MC_OK;
}

mc_status mc_init_lattice(const mc_replica_desc *reps, int32_t n_reps, mc_precision prec,
                          uint64_t seed, mc_init_mode init, const mc_spin_buffers *bufs,
                          void *scratch, uint64_t scratch_bytes, void *hip_stream, mc_sim **out)
{
    if (!out) return fail(MC_E_ARG, "out is NULL");
    *out = nullptr;
    if (!reps || !bufs) return fail(MC_E_ARG, "reps or bufs is NULL");
    if (n_reps < 1) return fail(MC_E_ARG, "n_reps must be >= 1");
    if (prec != MC_F32 && prec != MC_F64) return fail(MC_E_ARG, "unknown precision %d", (int)prec);
    if (init < MC_INIT_RANDOM || init > MC_INIT_USER)
        return fail(MC_E_ARG, "unknown init mode %d", (int)init);
    for (int r = 0; r < n_reps; ++r) {
        mc_status s = check_desc(reps[r], r);
        if (s != MC_OK) return s;
        if (reps[r].kind != reps[0].kind)
            return fail(MC_E_ARG, "replica %d: all replicas must share one lattice kind", r);
    }
    int dev_count = 0;
    if (hipGetDeviceCount(&dev_count) != hipSuccess || dev_count < 1) {
        (void)hipGetLastError();
        return fail(MC_E_DEVICE, "no HIP device available");
    }
    const size_t esz = prec == MC_F64 ? sizeof(double) : sizeof(float);
    for (int r = 0; r < n_reps; ++r) {
        const uint64_t need = box_sites(reps[r]);
        if (bufs[r].capacity_sites < need)
            return fail(MC_E_BUFFER, "replica %d: capacity %llu < %llu sites", r,
                        (unsigned long long)bufs[r].capacity_sites, (unsigned long long)need);
        const void *pl[3] = {bufs[r].sx, bufs[r].sy, bufs[r].sz};
        const char *nm[3] = {"sx", "sy", "sz"};
        for (int a = 0; a < 3; ++a) {
            mc_status s = check_device_buffer(pl[a], need * esz, nm[a], r);
            if (s != MC_OK) return s;
        }
    }
    mc_sim *h = new (std::nothrow) mc_sim();
    if (!h) return fail(MC_E_ARG, "out of host memory");
    h->n_reps = n_reps;
    h->kind = reps[0].kind;
    h->n_colours = n_colours_of(h->kind);
    h->prec = prec;
    h->seed = seed;
    h->stream = (hipStream_t)hip_stream;
    h->desc.assign(reps, reps + n_reps);
    h->tile = default_tile(reps, n_reps, esz);
    h->pass_tile = h->tile;
    std::vector<uint32_t> b, e;
    make_work(reps, n_reps, h->pass_tile, h->work, b, e);
    h->lay = scratch_layout(n_reps, h->work.size(), h->n_colours);
    auto cleanup = [&](mc_status s) {
        mc_destroy(h);
        return s;
    };
    if (!scratch) return cleanup(fail(MC_E_BUFFER, "scratch is NULL"));
    if (reinterpret_cast<uintptr_t>(scratch) % 256)
        return cleanup(fail(MC_E_BUFFER, "scratch must be 256-byte aligned"));
    if (scratch_bytes < h->lay.total)
        return cleanup(fail(MC_E_BUFFER, "scratch has %llu bytes, %llu needed",
                            (unsigned long long)scratch_bytes, (unsigned long long)h->lay.total));
    {
        mc_status s = check_device_buffer(scratch, h->lay.total, "scratch", -1);
        if (s != MC_OK) return cleanup(s);
    }
    h->scratch = (char *)scratch;
    h->scratch_bytes = scratch_bytes;
    h->tctr = (uint32_t *)(h->scratch + h->lay.off_ctr);
    h->reps_dev = (RepDev *)(h->scratch + h->lay.off_reps);
    h->work_dev = (WorkItem *)(h->scratch + h->lay.off_work);
    h->partials = (double *)(h->scratch + h->lay.off_partials);
    h->records = (double *)(h->scratch + h->lay.off_records);
    h->stage = (double *)(h->scratch + h->lay.off_stage);
    h->pstate = (uint32_t *)(h->scratch + h->lay.off_persist);
    h->queues_dev = (uint32_t *)(h->scratch + h->lay.off_queues);

    h->reps.resize(n_reps);
    h->n_occ.resize(n_reps);
    for (int r = 0; r < n_reps; ++r) {
        const mc_replica_desc &d = reps[r];
        RepDev &R = h->reps[r];
        fill_repdev(d, bufs[r], R);
        R.item_begin = b[r];
        R.item_end = e[r];
        h->n_occ[r] = count_occupied(d);
        if (h->n_occ[r] == 0) return cleanup(fail(MC_E_ARG, "replica %d has no occupied site", r));
    }
    if (hipHostMalloc((void **)&h->host_rec, sizeof(double) * NR * n_reps * (kRing + 1),
                      hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        h->host_rec = nullptr;
        return cleanup(fail(MC_E_DEVICE, "pinned host allocation failed"));
    }
    h->xcd_ok = device_deals_xcds(h, h->queues_dev);
    mc_status s;
    if ((s = plan_queues(h)) != MC_OK) return cleanup(s);
    if ((s = upload_reps(h)) != MC_OK) return cleanup(s);
    if (hipMemcpyAsync(h->work_dev, h->work.data(), sizeof(WorkItem) * h->work.size(),
                       hipMemcpyHostToDevice, h->stream) != hipSuccess ||
        launch_set_counter(h->tctr, 0u, h->stream) != hipSuccess ||
        launch_zero_u32(h->pstate, persist_state_words(n_reps), h->stream) != hipSuccess)
        return cleanup(fail(MC_E_DEVICE, "upload failed: %s", hipGetErrorString(hipGetLastError())));
    if (init != MC_INIT_USER) {
        for (int r = 0; r < n_reps; ++r) {
            hipError_t er = launch_init(prec == MC_F64, h->kind, &h->reps[r],
                                        init == MC_INIT_ALIGNED ? 1 : 0, (uint32_t)seed,
                                        (uint32_t)(seed >> 32), h->stream);
            if (er != hipSuccess)
                return cleanup(fail(MC_E_DEVICE, "init launch: %s", hipGetErrorString(er)));
        }
    }
    if (hipStreamSynchronize(h->stream) != hipSuccess)
        return cleanup(fail(MC_E_DEVICE, "init: %s", hipGetErrorString(hipGetLastError())));
    // the device as the autotuner's cache sees it (architecture, compute
    // units, XCDs: a partition mode changes the last two)
    {
        int dev = 0, n_xcd = 0;
        hipDeviceProp_t prop;
        std::memset(&prop, 0, sizeof prop);
        if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) {
            if (hipDeviceGetAttribute(&n_xcd, hipDeviceAttributeNumberOfXccs, dev) != hipSuccess)
                n_xcd = 0;
            char key[160];
            if (mc_tune_device_key(prop.gcnArchName, prop.multiProcessorCount, n_xcd, key,
                                   sizeof key) == MC_OK)
                h->device_key = key;
        }
        (void)hipGetLastError();
        if (h->device_key.empty()) h->device_key = "unknown-device";
    }
    // lattices whose state fits one workgroup's LDS run whole sweeps there
    {
        int dev = 0, lds = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) ==
                hipSuccess &&
            lds > (int)kLdsReserve)
            h->lds_max = (uint32_t)lds - kLdsReserve;
        (void)hipGetLastError();
        if (lds_fits(h) && lds_allow(h->kind, prec == MC_F64, (uint32_t)lds_need(h)) == hipSuccess)
            h->tile = Tile{KERNEL_LDS, lds_threads(h), 1, 1};
        (void)hipGetLastError();
    }
    *out = h;
    return MC_OK;
}

mc_status mc_sweep(mc_sim *h, uint32_t n_sweeps, uint32_t flags)
{
    if (!alive(h)) return fail(MC_E_STATE, "invalid or destroyed handle");
    if (flags & ~(MC_MEASURE | MC_PERSISTENT | MC_TUNED_LAUNCH))
        return fail(MC_E_ARG, "unknown flags 0x%x", flags);
    if ((flags & MC_PERSISTENT) && (flags & MC_TUNED_LAUNCH))
        return fail(MC_E_ARG, "MC_PERSISTENT and MC_TUNED_LAUNCH exclude each other");
    if ((flags & MC_TUNED_LAUNCH) && h->tuned_persistent) flags |= MC_PERSISTENT;
    if (n_sweeps == 0) return MC_OK;
    if (h->t + n_sweeps > 0xFFFFFFFFull) return fail(MC_E_STATE, "sweep counter would exceed 2^32-1");
    const bool measure = flags & MC_MEASURE;
    const uint32_t slot0 = (uint32_t)(h->n_measured % kRing);
    mc_status s = (flags & MC_PERSISTENT) ? enqueue_persistent(h, n_sweeps, measure, slot0)
                                          : enqueue_sweeps(h, n_sweeps, measure, slot0);
    if (s != MC_OK) return s;
    note_sweeps(h, n_sweeps);
    h->t += n_sweeps;
    if (measure) {
        h->n_measured += n_sweeps;
        h->last_slot = (int64_t)((slot0 + n_sweeps - 1) % kRing);
    }
    return MC_OK;
}

mc_status mc_sweep_timed(mc_sim *h, uint32_t n_sweeps, uint32_t flags, double *pass_ms_avg,
                         double *total_ms)
{
    if (!alive(h)) return fail(MC_E_STATE, "invalid or destroyed handle");
    if (flags & ~MC_MEASURE) return fail(MC_E_ARG, "unknown flags 0x%x", flags);
    if (!pass_ms_avg || !total_ms) return fail(MC_E_ARG, "NULL out-pointer");
    if (n_sweeps == 0) return fail(MC_E_ARG, "n_sweeps must be >= 1");
    if (h->t + n_sweeps > 0xFFFFFFFFull) return fail(MC_E_STATE, "sweep counter would exceed 2^32-1");
    const bool measure = flags & MC_MEASURE;
    if (h->tile.kernel == KERNEL_LDS) {
        // whole sweeps in one launch: the pass time reported is the average
        // share of a colour pass
        hipEvent_t e0, e1;
        HIP_TRY(hipEventCreate(&e0));
        HIP_TRY(hipEventCreate(&e1));
        const uint32_t slot0 = (uint32_t)(h->n_measured % kRing);
        hipError_t err = hipEventRecord(e0, h->stream);
        mc_status st = err == hipSuccess ? enqueue_lds(h, n_sweeps, measure, slot0) : MC_OK;
        if (err == hipSuccess && st == MC_OK) err = hipEventRecord(e1, h->stream);
        if (err == hipSuccess && st == MC_OK) err = hipEventSynchronize(e1);
        float ms = 0.f;
        if (err == hipSuccess && st == MC_OK) err = hipEventElapsedTime(&ms, e0, e1);
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (st != MC_OK) return st;
        if (err != hipSuccess) return fail(MC_E_DEVICE, "timed sweeps: %s", hipGetErrorString(err));
        h->t += n_sweeps;
        if (measure) {
            h->n_measured += n_sweeps;
            h->last_slot = (int64_t)((slot0 + n_sweeps - 1) % kRing);
        }
        *total_ms = ms;
        *pass_ms_avg = ms / (double)(n_sweeps * (uint32_t)h->n_colours);
        return MC_OK;
    }
    const bool f64 = h->prec == MC_F64;
    const uint32_t n_items = (uint32_t)h->work.size();
    const bool fused = h->tile.kernel == KERNEL_FUSED; // one launch per sweep
    const uint32_t per_sweep = fused ? 1u : (uint32_t)h->n_colours;
    const uint32_t n_pass = n_sweeps * per_sweep;
    std::vector<hipEvent_t> ev(2 * (size_t)n_pass + 2, nullptr);
    for (auto &e : ev) HIP_TRY(hipEventCreate(&e));
    auto release = [&]() {
        for (auto &e : ev)
            if (e) (void)hipEventDestroy(e);
    };
    const uint32_t slot0 = (uint32_t)(h->n_measured % kRing);
    hipError_t err = hipEventRecord(ev[2 * n_pass], h->stream);
    for (uint32_t i = 0; i < n_sweeps && err == hipSuccess; ++i) {
        const PassLaunch p = pass_args(h, 0, n_items, i);
        for (uint32_t c = 0; c < per_sweep && err == hipSuccess; ++c) {
            const uint32_t k = i * per_sweep + c;
            err = hipEventRecord(ev[2 * k], h->stream);
            if (err == hipSuccess)
                err = fused ? launch_fused(f64, measure, p, h->stream)
                            : launch_pass(h->kind, f64, (int)c, measure, 0, p, h->stream);
            if (err == hipSuccess) err = hipEventRecord(ev[2 * k + 1], h->stream);
            if (err == hipSuccess && fused)
                err = launch_swap_state(h->reps_dev, (uint32_t)h->n_reps, h->stream);
        }
        if (measure && err == hipSuccess)
            err = launch_finalize(h->reps_dev, h->n_reps, h->n_colours, h->partials, n_items,
                                  h->tctr, i,
                                  h->records + (size_t)((slot0 + i) % kRing) * h->n_reps * NR,
                                  h->stage, h->stream);
    }
    if (err == hipSuccess) err = launch_advance(h->tctr, n_sweeps, h->stream);
    if (err == hipSuccess) err = hipEventRecord(ev[2 * n_pass + 1], h->stream);
    if (err == hipSuccess) err = hipEventSynchronize(ev[2 * n_pass + 1]);
    if (err != hipSuccess) {
        release();
        return fail(MC_E_DEVICE, "timed sweep: %s", hipGetErrorString(err));
    }
    double sum = 0.0;
    for (uint32_t k = 0; k < n_pass; ++k) {
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, ev[2 * k], ev[2 * k + 1]);
        sum += ms;
    }
    float tot = 0.f;
    (void)hipEventElapsedTime(&tot, ev[2 * n_pass], ev[2 * n_pass + 1]);
    release();
    *pass_ms_avg = sum / n_pass;
    *total_ms = tot;
    note_sweeps(h, n_sweeps);
    h->t += n_sweeps;
    if (measure) {
        h->n_measured += n_sweeps;
        h->last_slot = (int64_t)((slot0 + n_sweeps - 1) % kRing);
    }
    return MC_OK;
}

mc_status mc_observables(mc_sim *h, mc_obs *out, int32_t n_reps)
{
    if (!alive(h)) return fail(MC_E_STATE, "invalid or destroyed handle");
    if (!out) return fail(MC_E_ARG, "out is NULL");
    if (n_reps != h->n_reps) return fail(MC_E_ARG, "n_reps %d != handle's %d", n_reps, h->n_reps);
    if (h->last_slot < 0) return fail(MC_E_STATE, "no measured sweep yet");
    HIP_TRY(hipStreamSynchronize(h->stream));
    mc_status ps = check_persistent(h);
    if (ps != MC_OK) return ps;
    const size_t sz = sizeof(double) * NR * h->n_reps;
    HIP_TRY(hipMemcpyAsync(h->host_rec, h->records + (size_t)h->last_slot * h->n_reps * NR, sz,
                           hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    for (int r = 0; r < h->n_reps; ++r) record_to_obs(h, h->host_rec + (size_t)r * NR, r, &out[r]);
    return MC_OK;
}

mc_status mc_measure_state(mc_sim *h, mc_obs *out, int32_t n_reps)
{
    if (!alive(h)) return fail(MC_E_STATE, "invalid or destroyed handle");
    if (!out) return fail(MC_E_ARG, "out is NULL");
    if (n_reps != h->n_reps) return fail(MC_E_ARG, "n_reps %d != handle's %d", n_reps, h->n_reps);
    HIP_TRY(hipStreamSynchronize(h->stream));
    mc_status ps = check_persistent(h);
    if (ps != MC_OK) return ps;
    const bool f64 = h->prec == MC_F64;
    double *partials = (double *)(h->scratch + h->lay.off_measure);
    double *dst = h->records + (size_t)kRing * h->n_reps * NR;
    for (int r = 0; r < h->n_reps; ++r) {
        HIP_TRY(launch_measure_direct(f64, h->kind, &h->reps[r], partials,
                                      measure_blocks(h->reps[r]), (double)h->t,
                                      dst + (size_t)r * NR, h->stream));
    }
    HIP_TRY(hipMemcpyAsync(h->host_rec, dst, sizeof(double) * NR * h->n_reps,
                           hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    for (int r = 0; r < h->n_reps; ++r) {
        const double counted = h->host_rec[(size_t)r * NR + R_NACC];
        if (counted != (double)h->n_occ[r])
            return fail(MC_E_DEVICE, "replica %d: the measurement visited %.0f occupied sites, "
                                     "the lattice has %llu", r, counted,
                        (unsigned long long)h->n_occ[r]);
        record_to_obs(h, h->host_rec + (size_t)r * NR, r, &out[r]);
        out[r].sweep = h->t;
        out[r].n_accepted = 0;
    }
    return MC_OK;
}

mc_status mc_measure_buffers(const mc_replica_desc *d, mc_precision prec,
                             const mc_spin_buffers *bufs, void *workspace,
                             uint64_t workspace_bytes, double *record_dev, void *hip_stream)
{
    mc_status s = check_measure_args(d, prec, bufs, record_dev);
    if (s != MC_OK) return s;
    if (!workspace) return fail(MC_E_BUFFER, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(workspace) % 256)
        return fail(MC_E_BUFFER, "workspace must be 256-byte aligned");
    if (workspace_bytes < MC_MEASURE_WORKSPACE_BYTES)
        return fail(MC_E_BUFFER, "workspace has %llu bytes, %llu needed",
                    (unsigned long long)workspace_bytes,
                    (unsigned long long)MC_MEASURE_WORKSPACE_BYTES);
    if ((s = check_device_buffer(workspace, MC_MEASURE_WORKSPACE_BYTES, "workspace", 0)) != MC_OK)
        return s;
    RepDev R;
    fill_repdev(*d, *bufs, R);
    const hipError_t e = launch_measure_direct(prec == MC_F64, d->kind, &R, (double *)workspace,
                                               measure_blocks(R), 0.0, record_dev,
                                               (hipStream_t)hip_stream);
    if (e != hipSuccess) return fail(MC_E_DEVICE, "measure launch: %s", hipGetErrorString(e));
    return MC_OK;
}

mc_status mc_set_temperatures(mc_sim *h, const double *T, int32_t n_reps)
{
    if (!alive(h)) return fail(MC_E_STATE, "invalid or destroyed handle");
    if (!T) return fail(MC_E_ARG, "T is NULL");
    if (n_reps != h->n_reps) return fail(MC_E_ARG, "n_reps %d != handle's %d", n_reps, h->n_reps);
    for (int r = 0; r < n_reps; ++r)
        if (!(T[r] >= 0.0)) return fail(MC_E_ARG, "replica %d: T must be >= 0", r);
    HIP_TRY(hipStreamSynchronize(h->stream));
    h->xchg_active = false; // explicit temperatures end replica exchange
    for (int r = 0; r < n_reps; ++r) {
        h->desc[r].T = T[r];
        set_temperature(h->reps[r], T[r]);
    }
    return upload_reps(h);
}

mc_status mc_run_schedule(mc_sim *h, const mc_schedule *s, mc_obs *series, uint64_t capacity,
                          uint64_t *n_written)
{
    if (!alive(h)) return fail(MC_E_STATE, "invalid or destroyed handle");
    if (!s || !s->T) return fail(MC_E_ARG, "schedule or its T is NULL");
    if (s->n_T < 1 || s->measure_every < 1) return fail(MC_E_ARG, "n_T and measure_every must be >= 1");
    if (s->flags & ~(MC_PERSISTENT | MC_TUNED_LAUNCH))
        return fail(MC_E_ARG, "unknown schedule flags 0x%x", s->flags);
    if ((s->flags & MC_PERSISTENT) && (s->flags & MC_TUNED_LAUNCH))
        return fail(MC_E_ARG, "MC_PERSISTENT and MC_TUNED_LAUNCH exclude each other");
    const bool persistent = (s->flags & MC_PERSISTENT) != 0 ||
                            ((s->flags & MC_TUNED_LAUNCH) && h->tuned_persistent);
    const uint64_t per_step = s->n_meas / s->measure_every;
    const uint64_t need = (uint64_t)s->n_T * per_step * h->n_reps;
    if (need > 0 && !series) return fail(MC_E_ARG, "series is NULL");
    if (capacity < need)
        return fail(MC_E_ARG, "series capacity %llu < %llu", (unsigned long long)capacity,
                    (unsigned long long)need);
    const uint64_t total_sweeps = (uint64_t)s->n_T * ((uint64_t)s->n_equil + s->n_meas);
    if (h->t + total_sweeps > 0xFFFFFFFFull) return fail(MC_E_STATE, "sweep counter would exceed 2^32-1");
    for (int64_t i = 0; i < (int64_t)s->n_T * h->n_reps; ++i)
        if (!(s->T[i] >= 0.0)) return fail(MC_E_ARG, "schedule T[%lld] must be >= 0", (long long)i);
    uint64_t written = 0;
    for (int step = 0; step < s->n_T; ++step) {
        mc_status st = mc_set_temperatures(h, s->T + (size_t)step * h->n_reps, h->n_reps);
        if (st != MC_OK) return st;
        for (uint32_t done = 0; done < s->n_equil;) {
            const uint32_t k = std::min(kGraphChunk, s->n_equil - done);
            if ((st = run_chunk(h, k, false, 0, persistent)) != MC_OK) return st;
            done += k;
            h->t += k;
        }
        uint32_t meas_idx = 0;
        for (uint32_t done = 0; done < s->n_meas;) {
            const uint32_t k = std::min(kGraphChunk, s->n_meas - done);
            if ((st = run_chunk(h, k, true, 0, persistent)) != MC_OK) return st;
            h->t += k;
            h->n_measured += k;
            h->last_slot = k - 1;
            const size_t sz = sizeof(double) * NR * h->n_reps * k;
            HIP_TRY(hipMemcpyAsync(h->host_rec, h->records, sz, hipMemcpyDeviceToHost, h->stream));
            HIP_TRY(hipStreamSynchronize(h->stream));
            if ((st = check_persistent(h)) != MC_OK) return st;
            for (uint32_t j = 0; j < k; ++j, ++meas_idx) {
                if ((meas_idx + 1) % s->measure_every) continue;
                for (int r = 0; r < h->n_reps; ++r)
                    record_to_obs(h, h->host_rec + ((size_t)j * h->n_reps + r) * NR, r,
                                  &series[written++]);
            }
            done += k;
        }
    }
    HIP_TRY(hipStreamSynchronize(h->stream));
    mc_status fin = check_persistent(h);
    if (fin != MC_OK) return fin;
    if (n_written) *n_written = written;
    return MC_OK;
}

mc_status mc_set_persistent_mode(mc_sim *h, mc_persist_mode mode)
{
    if (!alive(h)) return fail(MC_E_STATE, "invalid or destroyed handle");
    if (mode != MC_PERSIST_AUTO && mode != MC_PERSIST_GLOBAL && mode != MC_PERSIST_XCD)
        return fail(MC_E_ARG, "unknown persistent mode %d", (int)mode);
    if (mode == MC_PERSIST_XCD && !h->xcd_ok)
        return fail(MC_E_UNSUPPORTED, "per-XCD queues: this device does not deal workgroups to "
                                      "eight XCDs in turn");
    HIP_TRY(hipStreamSynchronize(h->stream));
    for (auto &kv : h->graphs) (void)hipGraphExecDestroy(kv.second);
    h->graphs.clear();
    h->persist_mode = mode;
    mc_status st = plan_queues(h);
    if (st != MC_OK) return st;
    HIP_TRY(hipStreamSynchronize(h->stream));
    return MC_OK;
}

mc_status mc_get_persistent_queues(const mc_sim *h, int32_t *n_queues)
{
    if (!alive(h)) return fail(MC_E_STATE, "invalid or destroyed handle");
    if (!n_queues) return fail(MC_E_ARG, "n_queues is NULL");
    *n_queues = (int32_t)h->n_queues;
    return MC_OK;
}

mc_status mc_set_watchdog(mc_sim *h, uint32_t spins)
{
    if (!alive(h)) return fail(MC_E_STATE, "invalid or destroyed handle");
    HIP_TRY(hipStreamSynchronize(h->stream)); // no captured graph may be in flight
    h->spin_limit = spins;
    for (auto &kv : h->graphs) (void)hipGraphExecDestroy(kv.second);
    h->graphs.clear();
    return MC_OK;
}

mc_status mc_synchronize(mc_sim *h)
{
    if (!alive(h)) return fail(MC_E_STATE, "invalid or destroyed handle");
    HIP_TRY(hipStreamSynchronize(h->stream));
    return check_persistent(h);
}

mc_status mc_debug_pass(mc_sim *h, int32_t colour, void *const *dh, void *const *accepted)
{
    if (!alive(h)) return fail(MC_E_STATE, "invalid or destroyed handle");
    if (colour < 0 || colour >= h->n_colours)
        return fail(MC_E_ARG, "colour %d out of range [0, %d)", colour, h->n_colours);
    if (!dh || !accepted) return fail(MC_E_ARG, "dh or accepted is NULL");
    if (h->pass_tile.kernel == KERNEL_FUSED)
        return fail(MC_E_UNSUPPORTED, "the fused sweep kernel has no single colour pass; set "
                                      "another tile for debug passes");
    const size_t esz = h->prec == MC_F64 ? sizeof(double) : sizeof(float);
    for (int r = 0; r < h->n_reps; ++r) {
        mc_status s = check_device_buffer(dh[r], h->reps[r].n_box * esz, "dh", r);
        if (s != MC_OK) return s;
        s = check_device_buffer(accepted[r], h->reps[r].n_box, "accepted", r);
        if (s != MC_OK) return s;
    }
    for (int r = 0; r < h->n_reps; ++r) {
        const RepDev &R = h->reps[r];
        PassLaunch p = pass_args(h, R.item_begin, R.item_end - R.item_begin, 0);
        p.dbg_dh = dh[r];
        p.dbg_acc = (uint8_t *)accepted[r];
        HIP_TRY(launch_pass(h->kind, h->prec == MC_F64, colour, false, 2, p, h->stream));
    }
    HIP_TRY(hipStreamSynchronize(h->stream));
    return MC_OK;
}

mc_status mc_layout_copy(mc_sim *h, int32_t replica, int32_t to_natural, void *nx, void *ny,
                         void *nz)
{
    if (!alive(h)) return fail(MC_E_STATE, "invalid or destroyed handle");
    if (replica < 0 || replica >= h->n_reps) return fail(MC_E_ARG, "replica %d out of range", replica);
    const size_t esz = h->prec == MC_F64 ? sizeof(double) : sizeof(float);
    void *pl[3] = {nx, ny, nz};
    for (int a = 0; a < 3; ++a) {
        mc_status s = check_device_buffer(pl[a], h->reps[replica].n_box * esz, "natural plane", replica);
        if (s != MC_OK) return s;
    }
    HIP_TRY(launch_layout(h->prec == MC_F64, h->kind, &h->reps[replica], to_natural != 0, nx, ny,
                          nz, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    return MC_OK;
}

mc_status mc_set_second_buffers(mc_sim *h, const mc_spin_buffers *bufs)
{
    if (!alive(h)) return fail(MC_E_STATE, "invalid or destroyed handle");
    if (!bufs) return fail(MC_E_ARG, "bufs is NULL");
    const size_t esz = h->prec == MC_F64 ? sizeof(double) : sizeof(float);
    for (int r = 0; r < h->n_reps; ++r) {
        const RepDev &R = h->reps[r];
        if (bufs[r].capacity_sites < R.n_box)
            return fail(MC_E_BUFFER, "replica %d: capacity %llu < %u sites", r,
                        (unsigned long long)bufs[r].capacity_sites, R.n_box);
        const void *pl[3] = {bufs[r].sx, bufs[r].sy, bufs[r].sz};
        const char *nm[3] = {"sx", "sy", "sz"};
        for (int a = 0; a < 3; ++a) {
            mc_status st = check_device_buffer(pl[a], (uint64_t)R.n_box * esz, nm[a], r);
            if (st != MC_OK) return st;
            const char *p0 = (const char *)pl[a], *p1 = p0 + (uint64_t)R.n_box * esz;
            const void *cur[3] = {R.sx, R.sy, R.sz};
            for (int b = 0; b < 3; ++b) {
                const char *q0 = (const char *)cur[b], *q1 = q0 + (uint64_t)R.n_box * esz;
                if (p0 < q1 && q0 < p1)
                    return fail(MC_E_BUFFER, "replica %d: second %s overlaps the current state",
                                r, nm[a]);
            }
        }
    }
    if (h->tile.kernel == KERNEL_FUSED) HIP_TRY(hipStreamSynchronize(h->stream));
    for (int r = 0; r < h->n_reps; ++r) {
        h->reps[r].ax = bufs[r].sx;
        h->reps[r].ay = bufs[r].sy;
        h->reps[r].az = bufs[r].sz;
    }
    return upload_reps(h);
}

mc_status mc_get_state_buffers(const mc_sim *h, int32_t replica, mc_spin_buffers *out)
{
    if (!alive(h)) return fail(MC_E_STATE, "invalid or destroyed handle");
    if (!out) return fail(MC_E_ARG, "out is NULL");
    if (replica < 0 || replica >= h->n_reps)
        return fail(MC_E_ARG, "replica %d out of range [0, %d)", replica, h->n_reps);
    const RepDev &R = h->reps[replica];
    out->sx = R.sx;
    out->sy = R.sy;
    out->sz = R.sz;
    out->capacity_sites = R.n_box;
    return MC_OK;
}

mc_status mc_set_tile(mc_sim *h, int32_t kernel, int32_t tx, int32_t ty, int32_t zc)
{
    if (!alive(h)) return fail(MC_E_STATE, "invalid or destroyed handle");
    if (kernel == KERNEL_LDS) {
        if (tx < 64 || tx > 1024 || tx % 64)
            return fail(MC_E_ARG, "LDS tile: tx (threads per replica) must be a multiple of 64 "
                                  "in [64, 1024] (got %d)", tx);
        if (!lds_fits(h))
            return fail(MC_E_UNSUPPORTED, "LDS kernel: a replica needs %llu bytes of LDS, a "
                                          "workgroup may use %u",
                        (unsigned long long)lds_need(h), h->lds_max);
        HIP_TRY(hipStreamSynchronize(h->stream));
        HIP_TRY(lds_allow(h->kind, h->prec == MC_F64, (uint32_t)lds_need(h)));
        for (auto &kv : h->graphs) (void)hipGraphExecDestroy(kv.second);
        h->graphs.clear();
        h->tile = Tile{KERNEL_LDS, tx, 1, 1};
        h->tuned_persistent = false; // a tile set by hand runs per pass under MC_TUNED_LAUNCH
        return MC_OK;
    }
    Tile t{kernel, tx, ty, zc};
    uint64_t max_bytes = 0;
    for (const RepDev &R : h->reps)
        max_bytes = std::max<uint64_t>(max_bytes, (uint64_t)R.n_box *
                                                      (h->prec == MC_F64 ? 8u : 4u));
    mc_status st = check_tile(t, h->kind, max_bytes, h->prec == MC_F64);
    if (st != MC_OK) return st;
    if (kernel == KERNEL_LBAND) {
        const uint32_t esz = h->prec == MC_F64 ? 8u : 4u;
        int w = 1;
        for (int r = 0; r < h->n_reps; ++r) {
            const int lxh = row_len(h->desc[r]);
            if ((uint32_t)lxh * esz % 16u)
                return fail(MC_E_UNSUPPORTED, "LDS-staged band kernel: replica %d has rows of %u "
                                              "bytes, not a multiple of 16", r, (uint32_t)lxh * esz);
            w = std::max(w, lxh);
        }
        if ((ty * (w / 2) + tx - 1) / tx > 2)
            return fail(MC_E_UNSUPPORTED, "LDS-staged band kernel: %d rows of %d pairs exceed two "
                                          "positions per thread", ty, w / 2);
        const uint64_t lds = lband_lds_bytes(ty, w, (int)esz);
        if (lds > 61440) // 60 KiB of dynamic LDS, the rest of 64 KiB for the reductions
            return fail(MC_E_UNSUPPORTED, "LDS-staged band kernel: %d rows of %d columns need %llu "
                                          "bytes of LDS (limit 61440)", ty, w, (unsigned long long)lds);
        if (lband_slots_needed(ty + 2, w, (int)esz, tx / 64) > LBAND_SLOTS)
            return fail(MC_E_UNSUPPORTED, "LDS-staged band kernel: %d rows of %d columns need more "
                                          "than %d copies per lane", ty + 2, w, LBAND_SLOTS);
    }
    if (kernel == KERNEL_FUSED) {
        for (int r = 0; r < h->n_reps; ++r)
            if (!h->reps[r].ax || !h->reps[r].ay || !h->reps[r].az)
                return fail(MC_E_STATE, "fused sweep kernel: replica %d has no second buffer set "
                                        "(mc_set_second_buffers)", r);
        int w = 1;
        for (int r = 0; r < h->n_reps; ++r) w = std::max(w, row_len(h->desc[r]));
        const bool f64 = h->prec == MC_F64;
        if (f64 && tx == 1024)
            return fail(MC_E_UNSUPPORTED, "fused sweep kernel: FP64 tiles take 256 or 512 threads");
        // FP64 keeps one position per lane, FP32 at most three (more would need
        // more than the 256 registers of a lane); 1024 threads: one
        const int max_pos = (tx == 1024 || f64) ? 1 : 3;
        if (fused_positions(ty, w, tx) > max_pos)
            return fail(MC_E_UNSUPPORTED, "fused sweep kernel: %d rows of %d columns exceed %d "
                                          "(row, pair) position%s per thread of %d", ty + 2, w,
                        max_pos, max_pos > 1 ? "s" : "", tx);
        const uint32_t lds = fused_lds_bytes(ty, w, h->prec == MC_F64 ? 8 : 4);
        if (lds > h->lds_max)
            return fail(MC_E_UNSUPPORTED, "fused sweep kernel: %d rows of %d columns need %u bytes "
                                          "of LDS, a workgroup may use %u", ty, w, lds, h->lds_max);
    }
    if (kernel != KERNEL_TILE && sc_sphere(h))
        return fail(MC_E_UNSUPPORTED, "a simple-cubic lattice cut to a sphere runs on the tile "
                                      "kernel (0) or the LDS kernel (3) only");
    if (kernel == KERNEL_PAIR || kernel == KERNEL_PBAND || kernel == KERNEL_BPAIR ||
        kernel == KERNEL_FUSED)
        for (int r = 0; r < h->n_reps; ++r)
            if (row_len(h->desc[r]) % 2)
                return fail(MC_E_UNSUPPORTED, "pair kernels: replica %d has an odd number (%d) of "
                                              "%s per row", r, row_len(h->desc[r]),
                            h->kind == MC_SC ? "packed columns" : "cells");
    std::vector<WorkItem> work;
    std::vector<uint32_t> b, e;
    make_work(h->desc.data(), h->n_reps, t, work, b, e);
    const ScratchLayout lay = scratch_layout(h->n_reps, work.size(), h->n_colours);
    if (lay.total > h->scratch_bytes)
        return fail(MC_E_BUFFER, "tile %d x %d x %d needs %llu scratch bytes, handle has %llu", tx,
                    ty, zc, (unsigned long long)lay.total, (unsigned long long)h->scratch_bytes);
    HIP_TRY(hipStreamSynchronize(h->stream));
    // a deferred persistent-launch error lives in the state words that move
    if ((st = check_persistent(h)) != MC_OK) return st;
    if (kernel == KERNEL_FUSED) {
        int w = 1;
        for (int r = 0; r < h->n_reps; ++r) w = std::max(w, row_len(h->desc[r]));
        HIP_TRY(fused_allow(h->prec == MC_F64, fused_lds_bytes(ty, w, h->prec == MC_F64 ? 8 : 4)));
    }
    for (auto &kv : h->graphs) (void)hipGraphExecDestroy(kv.second);
    h->graphs.clear();
    h->tile = t;
    h->pass_tile = t;
    h->tuned_persistent = false;
    h->work.swap(work);
    h->lay = lay;
    h->reps_dev = (RepDev *)(h->scratch + lay.off_reps);
    h->work_dev = (WorkItem *)(h->scratch + lay.off_work);
    h->partials = (double *)(h->scratch + lay.off_partials);
    h->records = (double *)(h->scratch + lay.off_records);
    h->stage = (double *)(h->scratch + lay.off_stage);
    h->pstate = (uint32_t *)(h->scratch + lay.off_persist);
    h->queues_dev = (uint32_t *)(h->scratch + lay.off_queues);
    h->last_slot = -1;
    HIP_TRY(launch_zero_u32(h->pstate, persist_state_words(h->n_reps), h->stream));
    for (int r = 0; r < h->n_reps; ++r) {
        h->reps[r].item_begin = b[r];
        h->reps[r].item_end = e[r];
    }
    HIP_TRY(hipMemcpyAsync(h->work_dev, h->work.data(), sizeof(WorkItem) * h->work.size(),
                           hipMemcpyHostToDevice, h->stream));
    if ((st = plan_queues(h)) != MC_OK) return st;
    return upload_reps(h);
}

mc_status mc_get_tile(const mc_sim *h, int32_t *kernel, int32_t *tx, int32_t *ty, int32_t *zc,
                      uint64_t *n_items)
{
    if (!alive(h)) return fail(MC_E_STATE, "invalid or destroyed handle");
    if (kernel) *kernel = h->tile.kernel;
    if (tx) *tx = h->tile.tx;
    if (ty) *ty = h->tile.ty;
    if (zc) *zc = h->tile.zc;
    if (n_items) *n_items = h->work.size();
    return MC_OK;
}

mc_status mc_get_sweep(const mc_sim *h, uint64_t *t)
{
    if (!alive(h)) return fail(MC_E_STATE, "invalid or destroyed handle");
    if (!t) return fail(MC_E_ARG, "t is NULL");
    *t = h->t;
    return MC_OK;
}

mc_status mc_set_sweep(mc_sim *h, uint64_t t)
{
    if (!alive(h)) return fail(MC_E_STATE, "invalid or destroyed handle");
    if (t > 0xFFFFFFFFull) return fail(MC_E_ARG, "sweep counter must be < 2^32");
    HIP_TRY(launch_set_counter(h->tctr, (uint32_t)t, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    h->t = t;
    return MC_OK;
}

mc_status mc_num_colours(const mc_sim *h, int32_t *n)
{
    if (!alive(h)) return fail(MC_E_STATE, "invalid or destroyed handle");
    if (!n) return fail(MC_E_ARG, "NULL argument");
    *n = h->n_colours;
    return MC_OK;
}

void mc_destroy(mc_sim *h)
{
    if (!alive(h)) return;
    if (h->stream || h->scratch) (void)hipStreamSynchronize(h->stream);
    for (auto &kv : h->graphs) (void)hipGraphExecDestroy(kv.second);
    h->graphs.clear();
    if (h->host_rec) (void)hipHostFree(h->host_rec);
    h->magic = 0;
    delete h;
}

} // extern "C"
