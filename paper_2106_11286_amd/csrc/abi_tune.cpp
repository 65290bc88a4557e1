// abi_tune.cpp -- the autotuner: candidate kernels and tile shapes timed on
// the handle's own lattices, with a text cache keyed by the lattice shapes.
#include <algorithm>
#include <cstdint>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "abi_internal.h"

using namespace mcabi;

namespace {

// Candidate shapes for the autotuner: each kernel family with a few tile
// widths, rows per thread and plane chunks aimed at 2k .. 24k workgroups.
std::vector<Tile> tile_candidates(const mc_sim *h)
{
    int W = 1, Ly = 1;
    for (const auto &d : h->desc) {
        W = std::max(W, row_len(d));
        Ly = std::max(Ly, d.Ly);
    }
    std::vector<Tile> base;
    if (h->kind == MC_SC && !sc_sphere(h)) {
        const int whole = std::min(256, (W + 63) / 64 * 64);
        for (int ry : {1, 2, 4}) {
            base.push_back(Tile{KERNEL_STRIP, whole, ry, 1});
            if (whole > 64) base.push_back(Tile{KERNEL_STRIP, 64, ry, 1});
        }
        for (int ry : {2, 4}) base.push_back(Tile{KERNEL_BAND, 256, ry, 1});
        bool even = true;
        for (const auto &d : h->desc) even &= row_len(d) % 2 == 0;
        if (even) {
            const int pairs = std::min(256, ((W + 1) / 2 + 63) / 64 * 64);
            for (int ry : {1, 2, 4}) base.push_back(Tile{KERNEL_PAIR, pairs, ry, 1});
            base.push_back(Tile{KERNEL_PBAND, 256, 2, 1});
            if (h->prec != MC_F64) base.push_back(Tile{KERNEL_PBAND, 256, 4, 1});
            // LDS-staged rows: tiles of whole rows that fill a workgroup once or
            // twice (mc_set_tile refuses the shapes that do not fit)
            const int np = std::max(1, W / 2);
            for (int rows : {256 / np, 512 / np})
                if (rows >= 1) base.push_back(Tile{KERNEL_LBAND, 256, std::min(rows, 64), 1});
            base.push_back(Tile{KERNEL_PBAND, 128, 2, 1});
            // the fused sweep, when every replica has its second buffer set
            bool second = true;
            for (const RepDev &R : h->reps) second &= R.ax && R.ay && R.az;
            if (second) {
                base.push_back(Tile{KERNEL_FUSED, 1024, 6, 1});
                base.push_back(Tile{KERNEL_FUSED, 512, 8, 1});
                base.push_back(Tile{KERNEL_FUSED, 256, 4, 1});
                base.push_back(Tile{KERNEL_FUSED, 256, 2, 1});
            }
        }
    }
    for (int tx : {64, 32, 16, 8}) {
        if (tx > 2 * pow2_at_least(W) && tx > 8) continue;
        const int ty = std::min(256 / tx, pow2_at_least(Ly));
        base.push_back(Tile{KERNEL_TILE, tx, ty, 1});
    }
    if (h->kind != MC_SC) {
        for (int tx : {64, 128, 256}) {
            if (tx > 64 && tx / 2 >= W) continue;
            base.push_back(Tile{KERNEL_BSTRIP, tx, 256 / tx, 1});
            if (tx <= 128) base.push_back(Tile{KERNEL_BSTRIP, tx, 1, 1});
        }
        bool even = true;
        for (const auto &d : h->desc) even &= d.Lx % 2 == 0;
        if (even)
            for (int ry : {1, 2}) {
                base.push_back(Tile{KERNEL_BPAIR, 256, ry, 1});
                base.push_back(Tile{KERNEL_BPAIR, 128, ry, 1});
            }
    }
    std::vector<Tile> out;
    if (lds_fits(h))
        for (int threads : {256, 512, 1024}) out.push_back(Tile{KERNEL_LDS, threads, 1, 1});
    for (Tile t : base) {
        uint64_t cols = 0;
        int planes = 1;
        for (const auto &d : h->desc) {
            cols += xy_tiles(d, t) * d.Lz;
            planes = std::max(planes, d.Lz);
        }
        int last = -1;
        for (uint64_t target : {2048ull, 4096ull, 8192ull, 16384ull, 24576ull}) {
            const int zc = (int)std::max<uint64_t>(1, std::min<uint64_t>((cols + target - 1) / target, planes));
            if (zc == last) continue;
            last = zc;
            t.zc = zc;
            out.push_back(t);
        }
    }
    return out;
}

std::string tune_key(const mc_sim *h, uint32_t flags)
{
    uint64_t hash = 1469598103934665603ull; // FNV-1a over the lattice shapes
    for (const auto &d : h->desc) {
        const int32_t v[5] = {d.kind, d.Lx, d.Ly, d.Lz, (int32_t)d.periodic_mask};
        for (int i = 0; i < 5; ++i)
            for (int b = 0; b < 4; ++b) {
                hash ^= (uint64_t)((v[i] >> (8 * b)) & 0xff);
                hash *= 1099511628211ull;
            }
        const uint64_t r = (uint64_t)std::llround(d.sphere_radius * 1024.0);
        for (int b = 0; b < 8; ++b) {
            hash ^= (r >> (8 * b)) & 0xff;
            hash *= 1099511628211ull;
        }
    }
    std::ostringstream k;
    k << h->device_key << "/kind" << h->kind << "/prec" << (int)h->prec << "/flags" << flags
      << "/reps" << h->n_reps;
    if (flags & (MC_PERSISTENT | MC_TUNED_LAUNCH)) k << "/queues" << h->persist_mode;
    k << "/" << std::hex << hash;
    return k.str();
}

} // namespace

extern "C" {

mc_status mc_get_tuned_launch(const mc_sim *h, int32_t *persistent)
{
    if (!alive(h)) return fail(MC_E_STATE, "invalid or destroyed handle");
    if (!persistent) return fail(MC_E_ARG, "persistent is NULL");
    *persistent = h->tuned_persistent ? 1 : 0;
    return MC_OK;
}

mc_status mc_tune_device_key(const char *arch, int32_t n_cu, int32_t n_xcd, char *out,
                             uint64_t capacity)
{
    if (!arch || !out) return fail(MC_E_ARG, "arch and out must not be NULL");
    if (n_cu < 0 || n_xcd < 0) return fail(MC_E_ARG, "negative unit count");
    std::string a;
    for (const char *c = arch; *c; ++c) // no separators of the cache's text format
        a.push_back((*c == ' ' || *c == '/' || *c == '\t' || *c == '\n') ? '_' : *c);
    std::ostringstream k;
    k << (a.empty() ? "unknown" : a) << "-cu" << n_cu << "-xcd" << n_xcd;
    const std::string s = k.str();
    if (capacity < s.size() + 1)
        return fail(MC_E_ARG, "key needs %llu bytes, capacity %llu",
                    (unsigned long long)(s.size() + 1), (unsigned long long)capacity);
    std::memcpy(out, s.c_str(), s.size() + 1);
    return MC_OK;
}

mc_status mc_autotune(mc_sim *h, uint32_t trial_sweeps, uint32_t flags, const char *cache_path,
                      int32_t *kernel, int32_t *tx, int32_t *ty, int32_t *zc)
{
    if (!alive(h)) return fail(MC_E_STATE, "invalid or destroyed handle");
    if (flags & ~(MC_MEASURE | MC_PERSISTENT | MC_TUNED_LAUNCH))
        return fail(MC_E_ARG, "unknown flags 0x%x", flags);
    if ((flags & MC_PERSISTENT) && (flags & MC_TUNED_LAUNCH))
        return fail(MC_E_ARG, "MC_PERSISTENT and MC_TUNED_LAUNCH exclude each other");
    const bool tune_launch = (flags & MC_TUNED_LAUNCH) != 0;
    if (trial_sweeps < 1) return fail(MC_E_ARG, "trial_sweeps must be >= 1");
    const std::string key = tune_key(h, flags);
    Tile best = h->tile;
    bool best_pers = false;
    bool found = false;
    if (cache_path) {
        std::ifstream in(cache_path);
        std::string line;
        while (std::getline(in, line)) {
            std::istringstream ls(line);
            std::string k;
            Tile t;
            double ms;
            int pers = 0;
            if (ls >> k >> t.kernel >> t.tx >> t.ty >> t.zc >> ms && k == key) {
                if (!(ls >> pers)) pers = 0;
                best = t;
                best_pers = tune_launch && pers == 1;
                found = true;
            }
        }
    }
    if (found) {
        mc_status st = mc_set_tile(h, best.kernel, best.tx, best.ty, best.zc);
        if (st != MC_OK) found = false; // stale entry: tune again
    }
    if (!found) {
        hipEvent_t e0, e1;
        HIP_TRY(hipEventCreate(&e0));
        HIP_TRY(hipEventCreate(&e1));
        double best_ms = 1e300;
        for (const Tile &t : tile_candidates(h)) {
            if ((flags & MC_PERSISTENT) && !persistent_supported(t)) continue;
            if (mc_set_tile(h, t.kernel, t.tx, t.ty, t.zc) != MC_OK) continue; // e.g. too big
            // launch modes to time: as asked, or (MC_TUNED_LAUNCH) both
            for (int mode = 0; mode < 2; ++mode) {
                uint32_t f = flags & ~MC_TUNED_LAUNCH;
                if (mode == 1) {
                    if (!tune_launch || !persistent_supported(t) || t.kernel == KERNEL_LDS) break;
                    f |= MC_PERSISTENT;
                }
                mc_status st = mc_sweep(h, 1, f);
                if (st == MC_OK) st = mc_synchronize(h);
                if (st != MC_OK) {
                    (void)hipEventDestroy(e0);
                    (void)hipEventDestroy(e1);
                    return st;
                }
                (void)hipEventRecord(e0, h->stream);
                st = mc_sweep(h, trial_sweeps, f);
                (void)hipEventRecord(e1, h->stream);
                if (st == MC_OK) st = mc_synchronize(h);
                if (st != MC_OK) {
                    (void)hipEventDestroy(e0);
                    (void)hipEventDestroy(e1);
                    return st;
                }
                float ms = 0.f;
                (void)hipEventElapsedTime(&ms, e0, e1);
                if (ms < best_ms) {
                    best_ms = ms;
                    best = t;
                    best_pers = mode == 1;
                }
            }
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        mc_status st = mc_set_tile(h, best.kernel, best.tx, best.ty, best.zc);
        if (st != MC_OK) return st;
        if (cache_path) {
            std::ofstream out(cache_path, std::ios::app);
            if (out) {
                out << key << " " << best.kernel << " " << best.tx << " " << best.ty << " "
                    << best.zc << " " << best_ms / trial_sweeps;
                if (tune_launch) out << " " << (best_pers ? 1 : 0);
                out << "\n";
            }
        }
    }
    if (tune_launch) h->tuned_persistent = best_pers;
    if (kernel) *kernel = h->tile.kernel;
    if (tx) *tx = h->tile.tx;
    if (ty) *ty = h->tile.ty;
    if (zc) *zc = h->tile.zc;
    return MC_OK;
}

} // extern "C"
