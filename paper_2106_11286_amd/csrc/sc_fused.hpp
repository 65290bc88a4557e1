// sc_fused.hpp -- simple-cubic fused sweep (kernel 9): both colours of one
// sweep in a single launch that reads every spin of the current state once
// and writes every spin of the next state once (24 bytes per update in FP32,
// against 36 for two colour passes).
//
// A sweep updates colour 0, then colour 1 against colour 0's new spins (the
// checkerboard decomposition of the Monte Carlo paragraph).  A workgroup owns
// a tile of BR whole rows and zc planes and walks it plane by plane: plane n's
// colour-0 sites are updated first, then plane n-1's colour-1 sites, whose six
// colour-0 neighbours (planes n-2, n-1, n) are all new by then.  Colour 1 in
// the tile's edge rows and end planes needs new colour-0 spins one row and one
// plane outside the tile; the workgroup computes those itself.  An update is a
// function of the old spins around it and of its Philox numbers, which are
// keyed by site and sweep, so these copies are bitwise the values the owning
// tile writes.  Neighbouring tiles run concurrently, so the sweep cannot work
// in place: it reads the current state and writes the next one into the
// replica's second buffer set (ax, ay, az); a one-thread launch afterwards
// swaps the two sets in the replica descriptors.  Field sums and the update
// are the same arithmetic in the same order (-z, -y, -x, +x, +y, +z) as in
// every other simple-cubic kernel, so the chain is bitwise the two-pass chain.
//
// Colour-1 old spins are read straight from the current state (the halo rows
// and planes come from the caches); new colour-0 spins of the rows y0-1 ..
// y0+BR of the last three planes live in LDS (three slots, rotated), which is
// where colour 1 reads its neighbours.
#pragma once

#include "device_common.hpp"

namespace mc {

template <typename T, bool MEASURE>
__device__ __forceinline__ void sc_fused_body(const PassLaunch &P, uint32_t item, uint32_t t)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char fused_lds[];
    typedef __attribute__((address_space(3))) T lds_t;
    lds_t *const lds = (lds_t *)(__attribute__((address_space(3))) unsigned char *)fused_lds;

    // every descriptor field is read before the first store (scalar loads)
    const WorkItem w = P.work_dev[item];
    const RepDev &R = P.reps_dev[w.rep];
    const int Ly = R.Ly, Lz = R.Lz, Lxh = R.Lxh, Lx = R.Lx;
    void *const src_x = R.sx, *const src_y = R.sy, *const src_z = R.sz;
    void *const dst_x = R.ax, *const dst_y = R.ay, *const dst_z = R.az;
    const uint32_t rid = R.rid;
    const uint32_t plane = R.plane; // elements per colour
    const T J = (T)R.J, K = (T)R.K, ex = (T)R.e[0], ey = (T)R.e[1], ez = (T)R.e[2];
    const T beta = (T)R.beta;
    const bool greedy = R.greedy != 0;
    const bool px = R.pmask & 1u, py = R.pmask & 2u, pz = R.pmask & 4u;
    const int BR = P.tile.ty;
    const int NP = Lxh >> 1; // pairs per row
    const int y0 = w.y0, z0 = w.z0, z1 = min(w.z0 + P.tile.zc, Lz);
    const PlaneRs<T> src = {plane_rsrc<T>(src_x, 0, R.n_box), plane_rsrc<T>(src_y, 0, R.n_box),
                            plane_rsrc<T>(src_z, 0, R.n_box)};
    const PlaneRs<T> dst = {plane_rsrc<T>(dst_x, 0, R.n_box), plane_rsrc<T>(dst_y, 0, R.n_box),
                            plane_rsrc<T>(dst_z, 0, R.n_box)};
    constexpr uint32_t ES = (uint32_t)sizeof(T);
    const uint32_t row_bytes = (uint32_t)Lxh * ES;
    const uint32_t zplane_b = (uint32_t)Ly * row_bytes;
    const uint32_t c1_b = plane * ES; // byte offset of colour 1

    // LDS slot s (0..2), component c, row k (0 .. BR+1 = y0-1 .. y0+BR), column j
    const uint32_t slot_elems = 3u * (uint32_t)(BR + 2) * (uint32_t)Lxh;
    const uint32_t comp_elems = (uint32_t)(BR + 2) * (uint32_t)Lxh;
    auto lds_at = [&](uint32_t s, int k, int j) __attribute__((always_inline)) {
        return s * slot_elems + (uint32_t)k * (uint32_t)Lxh + (uint32_t)j;
    };

    double acc0[Q_N] = {0, 0, 0, 0, 0, 0}, acc1[Q_N] = {0, 0, 0, 0, 0, 0};
    uint32_t n_acc0 = 0, n_acc1 = 0;
    const Row2<T> zero = {T(0), T(0), T(0), T(0), T(0), T(0)};

    // wrapped coordinate along an axis of length L (periodic) or -1 (absent)
    auto wrap = [](int v, int L, bool per) __attribute__((always_inline)) -> int {
        if (v >= 0 && v < L) return v;
        if (!per) return -1;
        return v < 0 ? v + L : v - L;
    };
    auto load_pair = [&](const PlaneRs<T> &q, uint32_t off_b) __attribute__((always_inline)) {
        Row2<T> v;
        buf_load2(q.x, off_b, 0u, v.xa, v.xb);
        buf_load2(q.y, off_b, 0u, v.ya, v.yb);
        buf_load2(q.z, off_b, 0u, v.za, v.zb);
        return v;
    };
    auto load_one = [&](const PlaneRs<T> &q, uint32_t off_b) __attribute__((always_inline)) {
        return Vec3<T>{buf_load(q.x, off_b, 0u, T()), buf_load(q.y, off_b, 0u, T()),
                       buf_load(q.z, off_b, 0u, T())};
    };
    auto lds_pair = [&](uint32_t o) __attribute__((always_inline)) {
        return Row2<T>{lds[o], lds[comp_elems + o], lds[2u * comp_elems + o],
                       lds[o + 1u], lds[comp_elems + o + 1u], lds[2u * comp_elems + o + 1u]};
    };
    auto lds_one = [&](uint32_t o) __attribute__((always_inline)) {
        return Vec3<T>{lds[o], lds[comp_elems + o], lds[2u * comp_elems + o]};
    };
    // the Metropolis attempt of one site (field h without J)
    auto attempt = [&](T &sx, T &sy, T &sz, T &hx, T &hy, T &hz, uint32_t s)
        __attribute__((always_inline)) -> bool {
        hx *= J;
        hy *= J;
        hz *= J;
        T dH;
        return metropolis<T>(sx, sy, sz, hx, hy, hz, s, rid, t, P.seed_lo, P.seed_hi, K, ex, ey,
                             ez, beta, greedy, dH);
    };
    // field of the pair (columns a, b) from the other colour: -z, -y, the
    // in-row neighbours (c: the pair's own columns, nb: the column beyond on
    // the side of parity p), +y, +z
    auto field = [&](const Row2<T> &m, const Row2<T> &dn, const Row2<T> &c, const Vec3<T> &nb,
                     const Row2<T> &up, const Row2<T> &top, int p, Row2<T> &h)
        __attribute__((always_inline)) {
        const Vec3<T> la = p ? Vec3<T>{c.xa, c.ya, c.za} : nb;
        const Vec3<T> ha = p ? Vec3<T>{c.xb, c.yb, c.zb} : Vec3<T>{c.xa, c.ya, c.za};
        const Vec3<T> lb = p ? Vec3<T>{c.xb, c.yb, c.zb} : Vec3<T>{c.xa, c.ya, c.za};
        const Vec3<T> hb = p ? nb : Vec3<T>{c.xb, c.yb, c.zb};
        h.xa = m.xa + dn.xa + la.x + ha.x + up.xa + top.xa;
        h.ya = m.ya + dn.ya + la.y + ha.y + up.ya + top.ya;
        h.za = m.za + dn.za + la.z + ha.z + up.za + top.za;
        h.xb = m.xb + dn.xb + lb.x + hb.x + up.xb + top.xb;
        h.yb = m.yb + dn.yb + lb.y + hb.y + up.yb + top.yb;
        h.zb = m.zb + dn.zb + lb.z + hb.z + up.zb + top.zb;
    };

    // Colour 0 of plane n (z0-1 <= n <= z1) on rows y0-1 .. y0+BR into slot s:
    // new spins of rows that exist, zeros for rows and planes beyond open faces.
    auto colour0 = [&](int n, uint32_t s) __attribute__((always_inline)) {
        const int nz = wrap(n, Lz, pz);
        const int nzm = nz < 0 ? -1 : wrap(nz - 1, Lz, pz);
        const int nzp = nz < 0 ? -1 : wrap(nz + 1, Lz, pz);
        const bool inner_plane = n >= z0 && n < z1;
        const int n_pos = (BR + 2) * NP;
        for (int q = (int)threadIdx.x; q < n_pos; q += (int)blockDim.x) {
            const int k = q / NP;
            const int ja = 2 * (q - k * NP);
            const int yv = y0 - 1 + k;
            const int y = wrap(yv, Ly, py);
            Row2<T> v = zero;
            if (nz >= 0 && y >= 0) {
                const int ym = wrap(y - 1, Ly, py), yp = wrap(y + 1, Ly, py);
                const int p = (y + nz) & 1;
                const uint32_t col_b = (uint32_t)ja * ES;
                const uint32_t in_plane = c1_b + (uint32_t)nz * zplane_b;
                const Row2<T> m = nzm >= 0
                    ? load_pair(src, c1_b + (uint32_t)nzm * zplane_b + (uint32_t)y * row_bytes + col_b)
                    : zero;
                const Row2<T> dn =
                    ym >= 0 ? load_pair(src, in_plane + (uint32_t)ym * row_bytes + col_b) : zero;
                const Row2<T> c = load_pair(src, in_plane + (uint32_t)y * row_bytes + col_b);
                const int jb = p ? (ja + 2 < Lxh ? ja + 2 : (px ? 0 : -1))
                                 : (ja > 0 ? ja - 1 : (px ? Lxh - 1 : -1));
                const Vec3<T> nb = jb >= 0
                    ? load_one(src, in_plane + (uint32_t)y * row_bytes + (uint32_t)jb * ES)
                    : Vec3<T>{T(0), T(0), T(0)};
                const Row2<T> up =
                    yp >= 0 ? load_pair(src, in_plane + (uint32_t)yp * row_bytes + col_b) : zero;
                const Row2<T> top = nzp >= 0
                    ? load_pair(src, c1_b + (uint32_t)nzp * zplane_b + (uint32_t)y * row_bytes + col_b)
                    : zero;
                const uint32_t own_b = (uint32_t)nz * zplane_b + (uint32_t)y * row_bytes + col_b;
                v = load_pair(src, own_b);
                Row2<T> h;
                field(m, dn, c, nb, up, top, p, h);
                const uint32_t s0 = (uint32_t)(nz * Ly + y) * (uint32_t)Lx + 2u * (uint32_t)ja + (uint32_t)p;
                const bool aa = attempt(v.xa, v.ya, v.za, h.xa, h.ya, h.za, s0);
                const bool ab = attempt(v.xb, v.yb, v.zb, h.xb, h.yb, h.zb, s0 + 2u);
                if (inner_plane && k >= 1 && k <= BR && yv < Ly) {
                    buf_store2(v.xa, v.xb, dst.x, own_b, 0u);
                    buf_store2(v.ya, v.yb, dst.y, own_b, 0u);
                    buf_store2(v.za, v.zb, dst.z, own_b, 0u);
                    if (MEASURE) {
                        observe<T>(acc0, v.xa, v.ya, v.za, ex, ey, ez, false, h.xa, h.ya, h.za, 1.0);
                        observe<T>(acc0, v.xb, v.yb, v.zb, ex, ey, ez, false, h.xb, h.yb, h.zb, 1.0);
                        n_acc0 += (aa ? 1u : 0u) + (ab ? 1u : 0u);
                    }
                }
            }
            const uint32_t o = lds_at(s, k, ja);
            lds[o] = v.xa;
            lds[o + 1u] = v.xb;
            lds[comp_elems + o] = v.ya;
            lds[comp_elems + o + 1u] = v.yb;
            lds[2u * comp_elems + o] = v.za;
            lds[2u * comp_elems + o + 1u] = v.zb;
        }
    };

    // Colour 1 of plane m (z0 <= m < z1), rows y0 .. y0+BR-1, from the new
    // colour-0 spins of planes m-1, m, m+1 in slots sm, s, sp.
    auto colour1 = [&](int m, uint32_t sm, uint32_t s, uint32_t sp) __attribute__((always_inline)) {
        const int n_pos = BR * NP;
        for (int q = (int)threadIdx.x; q < n_pos; q += (int)blockDim.x) {
            const int k = q / NP;
            const int ja = 2 * (q - k * NP);
            const int y = y0 + k;
            if (y >= Ly) continue; // a ragged last tile
            const int p = (y + m + 1) & 1;
            const Row2<T> mm = lds_pair(lds_at(sm, k + 1, ja));
            const Row2<T> dn = lds_pair(lds_at(s, k, ja));
            const Row2<T> c = lds_pair(lds_at(s, k + 1, ja));
            const int jb = p ? (ja + 2 < Lxh ? ja + 2 : (px ? 0 : -1))
                             : (ja > 0 ? ja - 1 : (px ? Lxh - 1 : -1));
            const Vec3<T> nb = jb >= 0 ? lds_one(lds_at(s, k + 1, jb)) : Vec3<T>{T(0), T(0), T(0)};
            const Row2<T> up = lds_pair(lds_at(s, k + 2, ja));
            const Row2<T> top = lds_pair(lds_at(sp, k + 1, ja));
            const uint32_t own_b = c1_b + (uint32_t)m * zplane_b + (uint32_t)y * row_bytes +
                                   (uint32_t)ja * ES;
            Row2<T> v = load_pair(src, own_b);
            Row2<T> h;
            field(mm, dn, c, nb, up, top, p, h);
            const uint32_t s0 = (uint32_t)(m * Ly + y) * (uint32_t)Lx + 2u * (uint32_t)ja + (uint32_t)p;
            const bool aa = attempt(v.xa, v.ya, v.za, h.xa, h.ya, h.za, s0);
            const bool ab = attempt(v.xb, v.yb, v.zb, h.xb, h.yb, h.zb, s0 + 2u);
            buf_store2(v.xa, v.xb, dst.x, own_b, 0u);
            buf_store2(v.ya, v.yb, dst.y, own_b, 0u);
            buf_store2(v.za, v.zb, dst.z, own_b, 0u);
            if (MEASURE) {
                observe<T>(acc1, v.xa, v.ya, v.za, ex, ey, ez, true, h.xa, h.ya, h.za, 1.0);
                observe<T>(acc1, v.xb, v.yb, v.zb, ex, ey, ez, true, h.xb, h.yb, h.zb, 1.0);
                n_acc1 += (aa ? 1u : 0u) + (ab ? 1u : 0u);
            }
        }
    };

    // slots rotate: plane n in slot (n - z0 + 1) mod 3
    uint32_t s_prev2 = 1u, s_prev = 2u, s_cur = 0u; // slots of planes n-2, n-1, n
    for (int n = z0 - 1; n <= z1; ++n) {
        colour0(n, s_cur);
        __syncthreads(); // plane n's new colour 0 is in LDS
        if (n - 1 >= z0) colour1(n - 1, s_prev2, s_prev, s_cur);
        __syncthreads(); // slot of plane n-2 is free for plane n+1
        const uint32_t nx = s_prev2;
        s_prev2 = s_prev;
        s_prev = s_cur;
        s_cur = nx;
    }

    if (MEASURE) {
        acc0[Q_NACC] = (double)n_acc0;
        acc1[Q_NACC] = (double)n_acc1;
        block_store_partials(acc0, P.partials_dev + (size_t)item * NQ);
        __syncthreads(); // the reduction's LDS is reused
        block_store_partials(acc1, P.partials_dev + ((size_t)P.n_items + item) * NQ);
    }
}

} // namespace mc
