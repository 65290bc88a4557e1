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
// Work of a lane: PP (1 .. 3) fixed (row, pair) positions of the tile's rows y0-1 ..
// y0+BR, the same on every plane.  Across planes a lane keeps in registers
// the old colour-1 pair of its own row on planes n-1 and n (the -z and
// in-row terms of plane n's colour 0, the +z term of plane n-1's), and the
// new colour-0 pair of planes n-1 and n, which are the -z and +z terms of
// colour 1 at the same site; only the in-plane (row and column) neighbours
// of colour 1 come from other lanes, through two LDS slots of new colour-0
// rows.  One workgroup barrier per plane.
#pragma once

#include "device_common.hpp"

namespace mc {

template <typename T, bool MEASURE, int PP>
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

    // LDS slot s (0, 1), component c, row k (0 .. BR+1 = y0-1 .. y0+BR), column j
    const uint32_t comp_elems = (uint32_t)(BR + 2) * (uint32_t)Lxh;
    const uint32_t slot_elems = 3u * comp_elems;

    // wrapped coordinate along an axis of length L (periodic) or -1 (absent)
    auto wrap = [](int v, int L, bool per) __attribute__((always_inline)) -> int {
        if (v >= 0 && v < L) return v;
        if (!per) return -1;
        return v < 0 ? v + L : v - L;
    };

    // this lane's positions: row k, pair column ja, wrapped row y and its
    // neighbours (-1: absent), byte offsets within a plane, the columns beyond
    // the pair on either side (-1: absent)
    int pk[PP], pja[PP], py_[PP];
    bool pval[PP], pinner[PP];
    uint32_t roff[PP], roff_m[PP], roff_p[PP], boff_l[PP], boff_r[PP];
    bool has_m[PP], has_p[PP], has_l[PP], has_r[PP];
#pragma unroll
    for (int i = 0; i < PP; ++i) {
        const int q = (int)threadIdx.x + (int)blockDim.x * i;
        const int n_pos = (BR + 2) * NP;
        const int qq = q < n_pos ? q : 0;
        const int k = qq / NP;
        const int ja = 2 * (qq - k * NP);
        const int yv = y0 - 1 + k;
        const int y = wrap(yv, Ly, py);
        pk[i] = k;
        pja[i] = ja;
        py_[i] = y;
        pval[i] = q < n_pos && y >= 0;
        // a site of the tile itself (colour 1 is updated here, colour 0 stored)
        pinner[i] = q < n_pos && k >= 1 && k <= BR && yv < Ly;
        const int ym = y >= 0 ? wrap(y - 1, Ly, py) : -1;
        const int yp = y >= 0 ? wrap(y + 1, Ly, py) : -1;
        const int jl = ja > 0 ? ja - 1 : (px ? Lxh - 1 : -1);
        const int jr = ja + 2 < Lxh ? ja + 2 : (px ? 0 : -1);
        const uint32_t yy = (uint32_t)(y >= 0 ? y : 0);
        roff[i] = yy * row_bytes + (uint32_t)ja * ES;
        roff_m[i] = (uint32_t)(ym >= 0 ? ym : 0) * row_bytes + (uint32_t)ja * ES;
        roff_p[i] = (uint32_t)(yp >= 0 ? yp : 0) * row_bytes + (uint32_t)ja * ES;
        boff_l[i] = yy * row_bytes + (uint32_t)(jl >= 0 ? jl : 0) * ES;
        boff_r[i] = yy * row_bytes + (uint32_t)(jr >= 0 ? jr : 0) * ES;
        has_m[i] = ym >= 0;
        has_p[i] = yp >= 0;
        has_l[i] = jl >= 0;
        has_r[i] = jr >= 0;
    }

    double acc0[Q_N] = {0, 0, 0, 0, 0, 0}, acc1[Q_N] = {0, 0, 0, 0, 0, 0};
    uint32_t n_acc0 = 0, n_acc1 = 0;
    const Row2<T> zero = {T(0), T(0), T(0), T(0), T(0), T(0)};
    const Vec3<T> zero3 = {T(0), T(0), T(0)};

    auto load_pair = [&](uint32_t off_b) __attribute__((always_inline)) {
        Row2<T> v;
        buf_load2(src.x, off_b, 0u, v.xa, v.xb);
        buf_load2(src.y, off_b, 0u, v.ya, v.yb);
        buf_load2(src.z, off_b, 0u, v.za, v.zb);
        return v;
    };
    auto load_one = [&](uint32_t off_b) __attribute__((always_inline)) {
        return Vec3<T>{buf_load(src.x, off_b, 0u, T()), buf_load(src.y, off_b, 0u, T()),
                       buf_load(src.z, off_b, 0u, T())};
    };
    auto lds_pair = [&](uint32_t o) __attribute__((always_inline)) {
        return Row2<T>{lds[o], lds[comp_elems + o], lds[2u * comp_elems + o],
                       lds[o + 1u], lds[comp_elems + o + 1u], lds[2u * comp_elems + o + 1u]};
    };
    auto lds_one = [&](uint32_t o) __attribute__((always_inline)) {
        return Vec3<T>{lds[o], lds[comp_elems + o], lds[2u * comp_elems + o]};
    };
    // the Metropolis attempt of one site (field h without J; J applied here)
    auto attempt = [&](T &sx, T &sy, T &sz, T &hx, T &hy, T &hz, uint32_t s)
        __attribute__((always_inline)) -> bool {
        hx *= J;
        hy *= J;
        hz *= J;
        T dH;
        return metropolis<T>(sx, sy, sz, hx, hy, hz, s, rid, t, P.seed_lo, P.seed_hi, K, ex, ey,
                             ez, beta, greedy, dH);
    };
    // -z, -y, -x, +x, +y of the pair (columns a, b): c is the other colour's
    // pair in the same columns, nb its column beyond on the side of parity p
    // (p = 0: x-1 of column a is nb, x+1 is c.a; x-1 of column b is c.a, x+1 is
    // c.b; p = 1: c.a, c.b and c.b, nb).  Component-wise selects keep every
    // value in registers.
    auto partial = [&](const Row2<T> &m, const Row2<T> &dn, const Row2<T> &c, const Vec3<T> &nb,
                       const Row2<T> &up, int p) __attribute__((always_inline)) {
        const bool q = p != 0;
        Row2<T> h;
        h.xa = m.xa + dn.xa + (q ? c.xa : nb.x) + (q ? c.xb : c.xa) + up.xa;
        h.ya = m.ya + dn.ya + (q ? c.ya : nb.y) + (q ? c.yb : c.ya) + up.ya;
        h.za = m.za + dn.za + (q ? c.za : nb.z) + (q ? c.zb : c.za) + up.za;
        h.xb = m.xb + dn.xb + (q ? c.xb : c.xa) + (q ? nb.x : c.xb) + up.xb;
        h.yb = m.yb + dn.yb + (q ? c.yb : c.ya) + (q ? nb.y : c.yb) + up.yb;
        h.zb = m.zb + dn.zb + (q ? c.zb : c.za) + (q ? nb.z : c.zb) + up.zb;
        return h;
    };

    // old colour 1 of the lane's own rows on planes n-1 (m1) and n (c1); new
    // colour 0 of planes n-1 (prev0) and n (cur0); partial field of colour 1
    // on plane n-1 (part1)
    Row2<T> m1[PP], c1[PP], prev0[PP], part1[PP];
    auto c1_row = [&](int n, int i) __attribute__((always_inline)) {
        const int nz = wrap(n, Lz, pz);
        if (nz < 0 || !pval[i]) return zero;
        return load_pair(c1_b + (uint32_t)nz * zplane_b + roff[i]);
    };
#pragma unroll
    for (int i = 0; i < PP; ++i) {
        m1[i] = c1_row(z0 - 2, i);
        c1[i] = c1_row(z0 - 1, i);
        prev0[i] = zero;
        part1[i] = zero;
    }

    for (int n = z0 - 1; n <= z1; ++n) {
        const int nz = wrap(n, Lz, pz);
        const int nzp = wrap(n + 1, Lz, pz); // plane n+1 (exists even when n does not)
        const bool inner_plane = n >= z0 && n < z1;
        const uint32_t slot = (uint32_t)(n & 1) * slot_elems;
        const uint32_t in_plane = c1_b + (uint32_t)(nz >= 0 ? nz : 0) * zplane_b;
        const uint32_t own_plane = (uint32_t)(nz >= 0 ? nz : 0) * zplane_b;
        Row2<T> top[PP], cur0[PP];
        // colour 0 of plane n on every position of rows y0-1 .. y0+BR
#pragma unroll
        for (int i = 0; i < PP; ++i) {
            const bool live = pval[i] && nz >= 0;
            top[i] = (pval[i] && nzp >= 0) ? load_pair(c1_b + (uint32_t)nzp * zplane_b + roff[i])
                                           : zero;
            // new colour 0 (zero where the row or the plane does not exist)
            T vxa = T(0), vya = T(0), vza = T(0), vxb = T(0), vyb = T(0), vzb = T(0);
            if (live) {
                const int y = py_[i], ja = pja[i];
                const int p = (y + nz) & 1;
                const Row2<T> dn = has_m[i] ? load_pair(in_plane + roff_m[i]) : zero;
                const Row2<T> up = has_p[i] ? load_pair(in_plane + roff_p[i]) : zero;
                const bool hb = p ? has_r[i] : has_l[i];
                const Vec3<T> nb = hb ? load_one(in_plane + (p ? boff_r[i] : boff_l[i])) : zero3;
                const Row2<T> o = load_pair(own_plane + roff[i]);
                vxa = o.xa;
                vya = o.ya;
                vza = o.za;
                vxb = o.xb;
                vyb = o.yb;
                vzb = o.zb;
                const Row2<T> pf = partial(m1[i], dn, c1[i], nb, up, p);
                T hxa = pf.xa + top[i].xa, hya = pf.ya + top[i].ya, hza = pf.za + top[i].za;
                T hxb = pf.xb + top[i].xb, hyb = pf.yb + top[i].yb, hzb = pf.zb + top[i].zb;
                const uint32_t s0 = (uint32_t)(nz * Ly + y) * (uint32_t)Lx + 2u * (uint32_t)ja + (uint32_t)p;
                const bool aa = attempt(vxa, vya, vza, hxa, hya, hza, s0);
                const bool ab = attempt(vxb, vyb, vzb, hxb, hyb, hzb, s0 + 2u);
                if (inner_plane && pinner[i]) {
                    buf_store2(vxa, vxb, dst.x, own_plane + roff[i], 0u);
                    buf_store2(vya, vyb, dst.y, own_plane + roff[i], 0u);
                    buf_store2(vza, vzb, dst.z, own_plane + roff[i], 0u);
                    if (MEASURE) {
                        observe<T>(acc0, vxa, vya, vza, ex, ey, ez, false, hxa, hya, hza, 1.0);
                        observe<T>(acc0, vxb, vyb, vzb, ex, ey, ez, false, hxb, hyb, hzb, 1.0);
                        n_acc0 += (aa ? 1u : 0u) + (ab ? 1u : 0u);
                    }
                }
            }
            const Row2<T> v = {vxa, vya, vza, vxb, vyb, vzb};
            cur0[i] = v;
            if ((int)threadIdx.x + (int)blockDim.x * i < (BR + 2) * NP) {
                const uint32_t o = slot + (uint32_t)pk[i] * (uint32_t)Lxh + (uint32_t)pja[i];
                lds[o] = v.xa;
                lds[o + 1u] = v.xb;
                lds[comp_elems + o] = v.ya;
                lds[comp_elems + o + 1u] = v.yb;
                lds[2u * comp_elems + o] = v.za;
                lds[2u * comp_elems + o + 1u] = v.zb;
            }
        }
        __syncthreads(); // plane n's new colour 0 is in LDS slot n & 1

        // colour 1 of plane n-1: partial field (formed last plane) + new colour 0 above
        if (n - 1 >= z0) {
            const int zm = n - 1;
#pragma unroll
            for (int i = 0; i < PP; ++i) {
                if (!pinner[i]) continue;
                const int y = py_[i], ja = pja[i];
                const int p = (y + zm + 1) & 1;
                // old colour 1 of plane n-1 on the own row, and its field
                T vxa = m1[i].xa, vya = m1[i].ya, vza = m1[i].za;
                T vxb = m1[i].xb, vyb = m1[i].yb, vzb = m1[i].zb;
                T hxa = part1[i].xa + cur0[i].xa, hya = part1[i].ya + cur0[i].ya,
                  hza = part1[i].za + cur0[i].za;
                T hxb = part1[i].xb + cur0[i].xb, hyb = part1[i].yb + cur0[i].yb,
                  hzb = part1[i].zb + cur0[i].zb;
                const uint32_t s0 = (uint32_t)(zm * Ly + y) * (uint32_t)Lx + 2u * (uint32_t)ja + (uint32_t)p;
                const bool aa = attempt(vxa, vya, vza, hxa, hya, hza, s0);
                const bool ab = attempt(vxb, vyb, vzb, hxb, hyb, hzb, s0 + 2u);
                const uint32_t o1 = c1_b + (uint32_t)zm * zplane_b + roff[i];
                buf_store2(vxa, vxb, dst.x, o1, 0u);
                buf_store2(vya, vyb, dst.y, o1, 0u);
                buf_store2(vza, vzb, dst.z, o1, 0u);
                if (MEASURE) {
                    observe<T>(acc1, vxa, vya, vza, ex, ey, ez, true, hxa, hya, hza, 1.0);
                    observe<T>(acc1, vxb, vyb, vzb, ex, ey, ez, true, hxb, hyb, hzb, 1.0);
                    n_acc1 += (aa ? 1u : 0u) + (ab ? 1u : 0u);
                }
            }
        }
        // partial field of colour 1 on plane n: -z (new colour 0 of plane n-1,
        // this lane's own), then the in-plane neighbours from the slot
        if (inner_plane) {
#pragma unroll
            for (int i = 0; i < PP; ++i) {
                if (!pinner[i]) continue;
                const int y = py_[i], ja = pja[i], k = pk[i];
                const int p = (y + n + 1) & 1;
                const uint32_t o = slot + (uint32_t)k * (uint32_t)Lxh + (uint32_t)ja;
                const Row2<T> dn = lds_pair(o - (uint32_t)Lxh);
                const Row2<T> c = lds_pair(o);
                const Row2<T> up = lds_pair(o + (uint32_t)Lxh);
                const bool hb = p ? has_r[i] : has_l[i];
                const int jb = p ? (ja + 2 < Lxh ? ja + 2 : 0) : (ja > 0 ? ja - 1 : Lxh - 1);
                const Vec3<T> nb = hb ? lds_one(slot + (uint32_t)k * (uint32_t)Lxh + (uint32_t)jb) : zero3;
                part1[i] = partial(prev0[i], dn, c, nb, up, p);
            }
        }
#pragma unroll
        for (int i = 0; i < PP; ++i) {
            prev0[i] = cur0[i];
            m1[i] = c1[i];
            c1[i] = top[i];
        }
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
