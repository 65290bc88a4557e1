// sc_lband.hpp -- simple-cubic colour pass with LDS-staged rows (kernel 8).
//
// A workgroup owns a tile of BR whole rows and a chunk of planes.  Plane by
// plane, the rows it needs are copied from HBM into LDS by the asynchronous
// global-to-LDS loads of gfx950 (16 bytes per lane, no registers held while in
// flight): the other colour's rows y0-1 .. y0+BR of the next plane and the own
// colour's rows of the current plane are fetched a full step ahead into the
// idle half of two double buffers, while the workgroup computes on the other
// half.  The neighbour field is read from LDS (rows y-1, y, y+1 and the
// column beyond the pair, with the periodic wrap inside the staged row), so
// no lane shifts and no per-lane prefetch registers are needed; the only
// state carried in registers across planes is the partial field of each site
// (-z, -y, -x, +x, +y, summed in that order) and the other colour's row of the
// previous plane (-z), as in the band-pair kernel.  The sums and the update
// are the same arithmetic in the same order as every other simple-cubic
// kernel, so the chain is bitwise the same.
//
// Stage n (n = z0-1 .. z1) holds the other colour of plane n and the own
// colour of plane n-1; it completes the sites of plane n-1 (+z term) and
// starts the partial fields of plane n.  One workgroup barrier per stage.
#pragma once

#include "device_common.hpp"

namespace mc {

template <typename T, bool MEASURE, int MODE, int PP>
__device__ __forceinline__ void sc_lband_body(const PassLaunch &P, int colour, uint32_t item,
                                              uint32_t t)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char lband_lds[];
    const WorkItem w = P.work_dev[item];
    const RepDev &R = P.reps_dev[w.rep];
    const int Ly = R.Ly, Lz = R.Lz, Lxh = R.Lxh, Lx = R.Lx;
    const uint32_t rid = R.rid;
    const int BR = P.tile.ty;
    const int NP = Lxh >> 1;
    const int y0 = w.y0;
    const uint32_t plane = R.plane;
    const uint32_t own = colour ? plane : 0u, oth = colour ? 0u : plane;
    const T J = (T)R.J, K = (T)R.K, ex = (T)R.e[0], ey = (T)R.e[1], ez = (T)R.e[2];
    const T beta = (T)R.beta;
    const bool greedy = R.greedy != 0;
    const bool px = R.pmask & 1u, py = R.pmask & 2u, pz = R.pmask & 4u;
    const gptr<T> gx = as_global<T>(R.sx), gy = as_global<T>(R.sy), gz = as_global<T>(R.sz);
    const int z0 = w.z0, z1 = min(w.z0 + P.tile.zc, Lz);

    // Copies of 16-byte chunks (rows are whole, 16-byte aligned and a multiple
    // of 16 bytes long; checked on the host).  A staged buffer holds, per
    // component, the rows' chunks padded to a multiple of 64 (one wave's copy
    // instruction never straddles two components): element (comp, row k, col)
    // at comp * cs * CH + k * Lxh + col, cs = lband_comp_chunks(rows, Lxh, T).
    // Each lane's source offsets within a plane are fixed for the whole tile
    // and computed once: slot j of the lane is chunk group g = wave + j n_waves.
    constexpr int CH = 16 / (int)sizeof(T); // elements per chunk
    typedef __attribute__((address_space(3))) T lds_t;
    lds_t *const lds = (lds_t *)(__attribute__((address_space(3))) unsigned char *)lband_lds;
    const int row_chunks = Lxh / CH;
    const uint32_t cs_o = lband_comp_chunks(BR + 2, Lxh, (int)sizeof(T));
    const uint32_t cs_w = lband_comp_chunks(BR, Lxh, (int)sizeof(T));
    // stage buffers: oth(b) = other rows, own(b) = own rows, b = 0, 1
    auto oth_buf = [&](unsigned b) __attribute__((always_inline)) { return lds + b * (3 * cs_o * CH); };
    auto own_buf = [&](unsigned b) __attribute__((always_inline)) {
        return lds + 6 * cs_o * CH + b * (3 * cs_w * CH);
    };
    // the wave index is uniform over the wave: say so, so the copy bookkeeping
    // stays scalar
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    const int n_waves = (int)(blockDim.x >> 6);
    struct Slots {
        uint32_t off[LBAND_SLOTS]; // element offset within a plane; ~0u: nothing to copy
        int n;                     // slots of this wave
    };
    // rows ybase .. ybase+n_rows-1 (wrapped on a periodic y axis, skipped
    // beyond an open face)
    auto make_slots = [&](int ybase, int n_rows, uint32_t cs) __attribute__((always_inline)) {
        Slots sl;
        const int gpc = (int)(cs / 64u); // chunk groups per component
        const int total = 3 * gpc;
        sl.n = 0;
#pragma unroll
        for (int j = 0; j < LBAND_SLOTS; ++j) {
            const int g = wave + j * n_waves;
            sl.off[j] = ~0u;
            if (g >= total) continue;
            sl.n = j + 1;
            const int cc = (g % gpc) * 64 + lane;
            if (cc >= n_rows * row_chunks) continue;
            const int k = cc / row_chunks, col = (cc - k * row_chunks) * CH;
            int y = ybase + k;
            if (y < 0 || y >= Ly) {
                if (!py) continue;
                y = y < 0 ? y + Ly : y - Ly;
            }
            sl.off[j] = (uint32_t)y * (uint32_t)Lxh + (uint32_t)col;
        }
        return sl;
    };
    const Slots sl_o = make_slots(y0 - 1, BR + 2, cs_o);
    const Slots sl_w = make_slots(y0, BR, cs_w);
    const uint32_t plane_elems = (uint32_t)Ly * (uint32_t)Lxh;
    auto stage = [&](lds_t *dst, const Slots sl, uint32_t cs, uint32_t cbase, int n)
        __attribute__((always_inline)) {
        const int gpc = (int)(cs / 64u);
        const uint32_t pbase = cbase + (uint32_t)n * plane_elems;
        const gptr<T> base[3] = {gx + pbase, gy + pbase, gz + pbase};
#pragma unroll
        for (int comp = 0; comp < 3; ++comp)
#pragma unroll
            for (int j = 0; j < LBAND_SLOTS; ++j) {
                const int g = wave + j * n_waves; // uniform over the wave
                if (j < sl.n && g >= comp * gpc && g < (comp + 1) * gpc && sl.off[j] != ~0u)
                    __builtin_amdgcn_global_load_lds(
                        (const void *)(base[comp] + sl.off[j]),
                        (__attribute__((address_space(3))) void *)(dst + (uint32_t)g * 64u * CH),
                        16, 0, 0);
            }
    };
    // stage n's buffers: other rows of plane n in oth_buf[(n + 2) & 1], own rows
    // of plane n in own_buf[n & 1] (read at stage n + 1)
    auto stage_other = [&](int n) __attribute__((always_inline)) {
        lds_t *dst = oth_buf((unsigned)(n + 2) & 1u);
        if (n < 0 || n >= Lz) {
            if (!pz) return; // an open z face: the plane reads as zero
            n = n < 0 ? n + Lz : n - Lz;
        }
        stage(dst, sl_o, cs_o, oth, n);
    };
    auto stage_own = [&](int n) __attribute__((always_inline)) {
        // rows past Ly (a ragged last tile) hold no site; they wrap or are skipped
        stage(own_buf((unsigned)n & 1u), sl_w, cs_w, own, n);
    };

    // this lane's positions: (row r, pair j) = divmod(q, NP), q = tid + 256 i
    int prow[PP], pxa[PP];
    bool pval[PP];
#pragma unroll
    for (int i = 0; i < PP; ++i) {
        const int q = (int)threadIdx.x + (int)blockDim.x * i;
        pval[i] = q < BR * NP;
        const int qq = pval[i] ? q : 0;
        prow[i] = qq / NP;
        pxa[i] = 2 * (qq - prow[i] * NP);
    }
    // the other colour's column beyond the pair (wrapped; -1 across an open face)
    auto beyond = [&](int xa, int p) __attribute__((always_inline)) -> int {
        if (p == 0) return xa > 0 ? xa - 1 : (px ? Lxh - 1 : -1);
        return xa + 2 < Lxh ? xa + 2 : (px ? 0 : -1);
    };
    // other-colour row k (0 .. BR+1, i.e. y0-1+k) exists on this plane
    auto row_ok = [&](int k) __attribute__((always_inline)) -> bool {
        const int y = y0 - 1 + k;
        return py || (y >= 0 && y < Ly);
    };

    double acc[Q_N] = {0, 0, 0, 0, 0, 0};
    uint32_t n_acc = 0;
    Row2<T> part[PP], mid[PP];
    const Row2<T> zero = {T(0), T(0), T(0), T(0), T(0), T(0)};

    auto site = [&](T &sx, T &sy, T &sz, T hx, T hy, T hz, uint32_t s, bool live,
                    uint32_t i) __attribute__((always_inline)) -> bool {
        hx *= J;
        hy *= J;
        hz *= J;
        bool a = false;
        if (MODE != 1) {
            T dH;
            a = metropolis<T>(sx, sy, sz, hx, hy, hz, s, rid, t, P.seed_lo, P.seed_hi, K, ex, ey,
                              ez, beta, greedy, dH);
            if (MODE == 2 && live) {
                ((T *)P.dbg_dh)[i] = dH;
                P.dbg_acc[i] = a ? 1 : 0;
            }
        }
        if (MEASURE && live) {
            observe<T>(acc, sx, sy, sz, ex, ey, ez, colour == 1, hx, hy, hz, 1.0);
            n_acc += a ? 1u : 0u;
        }
        return a;
    };

    auto read_pair = [&](const lds_t *b, uint32_t cs, int k, int xa) __attribute__((always_inline)) {
        Row2<T> v;
        const uint32_t o = (uint32_t)k * Lxh + xa;
        cs *= CH;
        v.xa = b[o];
        v.xb = b[o + 1];
        v.ya = b[cs + o];
        v.yb = b[cs + o + 1];
        v.za = b[2 * cs + o];
        v.zb = b[2 * cs + o + 1];
        return v;
    };

    const int n_first = z0 - 1, n_last = z1;
    stage_other(n_first);
    for (int n = n_first; n <= n_last; ++n) {
        __builtin_amdgcn_s_waitcnt(0); // this wave's copies (and stores) are done
        __syncthreads();               // ... and every wave's
        if (n < n_last) stage_other(n + 1);
        if (n >= z0 && n < z1) stage_own(n);
        const bool plane_ok = pz || (n >= 0 && n < Lz);
        const lds_t *ob = oth_buf((unsigned)(n + 2) & 1u);
        const lds_t *wb = own_buf((unsigned)(n + 1) & 1u); // own rows of plane n-1
#pragma unroll
        for (int i = 0; i < PP; ++i) {
            const int r = prow[i], xa = pxa[i];
            const int y = y0 + r;
            const bool live = pval[i] && y < Ly;
            // this plane's other-colour rows y (for the +z term and -z of n+1)
            Row2<T> c = (plane_ok && row_ok(r + 1)) ? read_pair(ob, cs_o, r + 1, xa) : zero;
            if (n >= z0 + 1) {
                // complete the sites of plane n-1
                const int z = n - 1;
                const int p = (colour + y + z) & 1;
                Row2<T> me = read_pair(wb, cs_w, r, xa);
                const T hxa = part[i].xa + c.xa, hya = part[i].ya + c.ya, hza = part[i].za + c.za;
                const T hxb = part[i].xb + c.xb, hyb = part[i].yb + c.yb, hzb = part[i].zb + c.zb;
                const uint32_t s0 = (uint32_t)(z * Ly + y) * (uint32_t)Lx + 2u * xa + p;
                const uint32_t i0 = own + (uint32_t)(z * Ly + y) * Lxh + xa;
                const bool aa = site(me.xa, me.ya, me.za, hxa, hya, hza, s0, live, i0);
                const bool ab = site(me.xb, me.yb, me.zb, hxb, hyb, hzb, s0 + 2u, live, i0 + 1u);
                if (MODE != 1 && live && (aa || ab)) {
                    typedef T v2 __attribute__((ext_vector_type(2)));
                    v2 vx, vy, vz;
                    vx.x = me.xa; vx.y = me.xb;
                    vy.x = me.ya; vy.y = me.yb;
                    vz.x = me.za; vz.y = me.zb;
                    *(gptr<v2>)(gx + i0) = vx;
                    *(gptr<v2>)(gy + i0) = vy;
                    *(gptr<v2>)(gz + i0) = vz;
                }
            }
            if (n >= z0 && n < z1) {
                // partial fields of plane n: -z (previous plane), -y, -x, +x, +y
                const int p = (colour + y + n) & 1;
                const Row2<T> dn = (plane_ok && row_ok(r)) ? read_pair(ob, cs_o, r, xa) : zero;
                const Row2<T> up = (plane_ok && row_ok(r + 2)) ? read_pair(ob, cs_o, r + 2, xa) : zero;
                const int xo = beyond(xa, p);
                Vec3<T> nb = {T(0), T(0), T(0)};
                if (plane_ok && row_ok(r + 1) && xo >= 0) {
                    const uint32_t o = (uint32_t)(r + 1) * Lxh + xo, cs = cs_o * CH;
                    nb = {ob[o], ob[cs + o], ob[2 * cs + o]};
                }
                const Vec3<T> la = p ? Vec3<T>{c.xa, c.ya, c.za} : nb;
                const Vec3<T> ha = p ? Vec3<T>{c.xb, c.yb, c.zb} : Vec3<T>{c.xa, c.ya, c.za};
                const Vec3<T> lb = p ? Vec3<T>{c.xb, c.yb, c.zb} : Vec3<T>{c.xa, c.ya, c.za};
                const Vec3<T> hb = p ? nb : Vec3<T>{c.xb, c.yb, c.zb};
                const Row2<T> &m = mid[i];
                part[i].xa = m.xa + dn.xa + la.x + ha.x + up.xa;
                part[i].ya = m.ya + dn.ya + la.y + ha.y + up.ya;
                part[i].za = m.za + dn.za + la.z + ha.z + up.za;
                part[i].xb = m.xb + dn.xb + lb.x + hb.x + up.xb;
                part[i].yb = m.yb + dn.yb + lb.y + hb.y + up.yb;
                part[i].zb = m.zb + dn.zb + lb.z + hb.z + up.zb;
            }
            mid[i] = c;
        }
    }
    if (MEASURE) {
        acc[Q_NACC] = (double)n_acc;
        block_store_partials(acc, P.partials_dev + ((size_t)colour * P.n_items + item) * NQ);
    }
}

} // namespace mc
