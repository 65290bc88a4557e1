// sc_bodies.hpp -- simple-cubic colour-pass bodies (one work item each): the
// tile, row-strip, pair, band-pair and band schemes.  Shared by the pass
// kernels and the persistent kernel.
#pragma once

#include <type_traits>

#include "device_common.hpp"

namespace mc {

// ---------------------------------------------------------------------------
// Simple cubic, two colours, colour-packed rows.  A site (x, y, z) of colour
// c = (x+y+z)&1 sits at packed column xh = x/2 of row (y, z) in plane c.  Its
// six neighbours all have the other colour: the same column of rows y+-1 and
// planes z+-1, and in its own row the columns xh and xh-1 (x even) or xh and
// xh+1 (x odd).
//
// Tile kernel: each thread owns one (xh, y) column of a tx x ty tile and walks
// the tile's z range; neighbours are loaded directly (cache hits).  Used for
// short rows, and the only pass kernel (with the LDS kernel) for a simple-cubic
// lattice cut to a sphere: it skips unoccupied sites.
// ---------------------------------------------------------------------------
template <typename T, bool MEASURE, int MODE>
__device__ __forceinline__ void sc_tile_body(const PassLaunch &P, int colour, uint32_t item,
                                             uint32_t t)
{
    const WorkItem w = P.work_dev[item];
    const RepDev &R = P.reps_dev[w.rep];
    const int Ly = R.Ly, Lz = R.Lz, Lxh = R.Lxh;
    const int lx = threadIdx.x % P.tile.tx, ly = threadIdx.x / P.tile.tx;
    const int xh = w.x0 + lx, y = w.y0 + ly;
    const bool active = xh < Lxh && y < Ly && ly < P.tile.ty;
    const uint32_t plane = R.plane;
    const gptr<T> gx = as_global<T>(R.sx), gy = as_global<T>(R.sy), gz = as_global<T>(R.sz);
    const uint32_t own = colour ? plane : 0u, oth = colour ? 0u : plane;
    const T J = (T)R.J, K = (T)R.K, ex = (T)R.e[0], ey = (T)R.e[1], ez = (T)R.e[2];
    const T beta = (T)R.beta;
    const bool greedy = R.greedy != 0;
    const bool px = R.pmask & 1u, py = R.pmask & 2u, pz = R.pmask & 4u;

    double acc[Q_N] = {0, 0, 0, 0, 0, 0};
    if (active) {
        const int z1 = min(w.z0 + P.tile.zc, Lz);
        for (int z = w.z0; z < z1; ++z) {
            const int p = (colour + y + z) & 1;
            // a site outside a sphere holds S = 0 and is never updated
            if (!occupied(R, 2 * xh + p, y, z, 0, 0, 0)) continue;
            const uint32_t i = (uint32_t)(z * Ly + y) * Lxh + xh;
            T hx, hy, hz;
            sc_site_field<T>(gx, gy, gz, oth, Lxh, Ly, Lz, px, py, pz, xh, y, z, p, hx, hy, hz);
            hx *= J;
            hy *= J;
            hz *= J;
            T sx = gx[own + i], sy = gy[own + i], sz = gz[own + i];
            bool a = false;
            if (MODE != 1) {
                const uint32_t s = (uint32_t)(z * Ly + y) * (uint32_t)R.Lx + 2u * xh + p;
                T dH;
                a = metropolis<T>(sx, sy, sz, hx, hy, hz, s, R.rid, t, P.seed_lo, P.seed_hi, K,
                                  ex, ey, ez, beta, greedy, dH);
                if (MODE == 2) {
                    ((T *)P.dbg_dh)[own + i] = dH;
                    P.dbg_acc[own + i] = a ? 1 : 0;
                }
                if (a) {
                    gx[own + i] = sx;
                    gy[own + i] = sy;
                    gz[own + i] = sz;
                }
            }
            // every bond has exactly one colour-1 end: count it there,
            // against colour-0 neighbours that are final after pass 0
            if (MEASURE) {
                observe<T>(acc, sx, sy, sz, ex, ey, ez, colour == 1, hx, hy, hz, 1.0);
                acc[Q_NACC] += a ? 1.0 : 0.0;
            }
        }
    }
    if (MEASURE)
        block_store_partials(acc, P.partials_dev + ((size_t)colour * P.n_items + item) * NQ);
}

// ---------------------------------------------------------------------------
// Row-strip kernel (simple cubic).  The workgroup's tx threads lie along one
// row segment (whole rows when they fit), each thread owns RY consecutive rows
// of its column and walks the tile's planes in z:
//  * the other colour's planes z-1, z, z+1 sit in registers and roll forward,
//    so each element of the other colour is loaded once per tile (plus one
//    halo row above and below the RY rows, and one halo plane at each end);
//  * the +-y neighbours are the thread's own rows; the in-row neighbour comes
//    from the adjacent lane through a DPP lane shift, or from memory at wave
//    edges and at the periodic wrap.
// All lanes run the loop (the DPP sources must be live); lanes and rows
// outside the lattice read clamped in-bounds addresses and store nothing.
// ---------------------------------------------------------------------------
template <typename T, bool MEASURE, int MODE, int RY>
__device__ __forceinline__ void sc_strip_body(const PassLaunch &P, int colour, uint32_t item,
                                              uint32_t t)
{
    // every descriptor field is read into registers before the first store, so
    // the loads stay scalar (memory that the kernel may write cannot be)
    const WorkItem w = P.work_dev[item];
    const RepDev &R = P.reps_dev[w.rep];
    const int Ly = R.Ly, Lz = R.Lz, Lxh = R.Lxh, Lx = R.Lx;
    void *const base_x = R.sx, *const base_y = R.sy, *const base_z = R.sz;
    const uint32_t rid = R.rid;
    const int lane = threadIdx.x & 63;
    const int xraw = w.x0 + (int)threadIdx.x;
    const bool xin = xraw < Lxh && (int)threadIdx.x < P.tile.tx;
    const int xh = xin ? xraw : Lxh - 1;
    const uint32_t plane = R.plane;
    const uint32_t own = colour ? plane : 0u, oth = colour ? 0u : plane;
    const T J = (T)R.J, K = (T)R.K, ex = (T)R.e[0], ey = (T)R.e[1], ez = (T)R.e[2];
    const T beta = (T)R.beta;
    const bool greedy = R.greedy != 0;
    const bool px = R.pmask & 1u, py = R.pmask & 2u, pz = R.pmask & 4u;
    const int xl = xh > 0 ? xh - 1 : (px ? Lxh - 1 : -1);
    const int xr = xh < Lxh - 1 ? xh + 1 : (px ? 0 : -1);
    const bool left_mem = lane == 0 || xh == 0;           // x-1 not held by lane-1
    const bool right_mem = lane == 63 || xh >= Lxh - 1;   // x+1 not held by lane+1
    // lane byte offsets within a row; row byte offsets are uniform
    const uint32_t b_c = (uint32_t)xh * (uint32_t)sizeof(T);
    const uint32_t b_l = (uint32_t)(xl < 0 ? 0 : xl) * (uint32_t)sizeof(T);
    const uint32_t b_r = (uint32_t)(xr < 0 ? 0 : xr) * (uint32_t)sizeof(T);
    const uint32_t row_bytes = (uint32_t)Lxh * (uint32_t)sizeof(T);
    const PlaneRs<T> q = {plane_rsrc<T>(base_x, 0, R.n_box), plane_rsrc<T>(base_y, 0, R.n_box),
                          plane_rsrc<T>(base_z, 0, R.n_box)};
    const uint32_t own_b = own * (uint32_t)sizeof(T), oth_b = oth * (uint32_t)sizeof(T);
    auto row_off = [&](int y, int z) -> uint32_t {
        return ((uint32_t)z * (uint32_t)Ly + (uint32_t)y) * row_bytes;
    };
    auto load3 = [&](const PlaneRs<T> &q, uint32_t voff, uint32_t soff) -> Vec3<T> {
        return {buf_load(q.x, voff, soff, T()), buf_load(q.y, voff, soff, T()),
                buf_load(q.z, voff, soff, T())};
    };

    // rows y0-1 .. y0+RY: lattice row index or -1 (open face)
    int yrow[RY + 2];
#pragma unroll
    for (int k = -1; k <= RY; ++k) {
        int y = w.y0 + k;
        if (y < 0 || y >= Ly) {
            if (!py) y = -1;
            else {
                while (y < 0) y += Ly;
                while (y >= Ly) y -= Ly;
            }
        }
        yrow[k + 1] = y;
    }
    // Loads are issued unconditionally (rows and planes outside an open face
    // read row / plane 0) and zeroed afterwards by a uniform branch that
    // periodic lattices never take.
    auto load_rows = [&](int z, Vec3<T> *dst, int k0, int n) {
        const bool z_ok = z >= 0;
        const int zc = z_ok ? z : 0;
        for (int k = 0; k < n; ++k) {
            const int y = yrow[k0 + k];
            dst[k] = load3(q, b_c, oth_b + row_off(y < 0 ? 0 : y, zc));
            if (!z_ok || y < 0) dst[k] = {T(0), T(0), T(0)};
        }
    };

    // In-row neighbours that the lane shift cannot supply (wave edges, the
    // periodic wrap, open faces) are loaded one plane ahead by the lanes that
    // need them, so the loads never stall the plane being updated.
    auto load_edges = [&](int z, Vec3<T> (&dst)[RY]) {
#pragma unroll
        for (int k = 0; k < RY; ++k) {
            const int yk = w.y0 + k;
            const int yc = yk < Ly ? yk : Ly - 1;
            const int p = (colour + yc + z) & 1;
            const bool need = p ? right_mem : left_mem;
            const int col = p ? xr : xl;
            if (need && col >= 0)
                dst[k] = load3(q, p ? b_r : b_l, oth_b + row_off(yc, z));
            else
                dst[k] = {T(0), T(0), T(0)};
        }
    };

    const int z0 = w.z0, z1 = min(w.z0 + P.tile.zc, Lz);
    double acc[Q_N] = {0, 0, 0, 0, 0, 0};
    uint32_t n_acc = 0;
    // One plane: rows of the other colour at z-1 (pm), z (pc) and z+1 (pn,
    // loaded here), in-row edge values of plane z (ec) and z+1 (en, loaded
    // here).  The plane sets form a ring of three; the loop is unrolled by
    // three so that the ring turns without moving registers.
    auto step = [&](const Vec3<T> (&pm)[RY + 2], const Vec3<T> (&pc)[RY + 2],
                    Vec3<T> (&pn)[RY + 2], const Vec3<T> (&ec)[RY], Vec3<T> (&en)[RY], int z) {
        const int zn = z < Lz - 1 ? z + 1 : (pz ? 0 : -1);
        load_rows(zn, pn, 0, RY + 2);
        if (z + 1 < z1) load_edges(zn, en);
#pragma unroll
        for (int k = 0; k < RY; ++k) {
            const int yk = w.y0 + k;
            const bool row_in = yk < Ly;
            const int yc = row_in ? yk : Ly - 1;
            const int p = (colour + yc + z) & 1; // uniform over the workgroup
            const uint32_t soff = row_off(yc, z);
            const uint32_t s_own = own_b + soff;
            T sx = buf_load(q.x, b_c, s_own, T()), sy = buf_load(q.y, b_c, s_own, T()),
              sz = buf_load(q.z, b_c, s_own, T());
            // in-row neighbour on the side given by the parity
            const Vec3<T> c = pc[k + 1];
            const bool from_mem = p ? right_mem : left_mem;
            Vec3<T> nb;
            if (p == 0)
                nb = {from_lower_lane(c.x), from_lower_lane(c.y), from_lower_lane(c.z)};
            else
                nb = {from_upper_lane(c.x), from_upper_lane(c.y), from_upper_lane(c.z)};
            if (from_mem) nb = ec[k];
            // fixed order: -z, -y, -x, +x, +y, +z
            const Vec3<T> lo = p ? c : nb, hi = p ? nb : c;
            T hx = pm[k + 1].x + pc[k].x + lo.x + hi.x + pc[k + 2].x + pn[k + 1].x;
            T hy = pm[k + 1].y + pc[k].y + lo.y + hi.y + pc[k + 2].y + pn[k + 1].y;
            T hz = pm[k + 1].z + pc[k].z + lo.z + hi.z + pc[k + 2].z + pn[k + 1].z;
            hx *= J;
            hy *= J;
            hz *= J;
            const bool live = xin && row_in;
            bool a = false;
            if (MODE != 1) {
                const uint32_t s = (uint32_t)(z * Ly + yc) * (uint32_t)Lx + 2u * xh + p;
                T dH;
                a = metropolis<T>(sx, sy, sz, hx, hy, hz, s, rid, t, P.seed_lo, P.seed_hi, K,
                                  ex, ey, ez, beta, greedy, dH);
                if (live) {
                    const uint32_t i = own + (uint32_t)(z * Ly + yc) * Lxh + xh;
                    if (MODE == 2) {
                        ((T *)P.dbg_dh)[i] = dH;
                        P.dbg_acc[i] = a ? 1 : 0;
                    }
                    if (a) {
                        buf_store(sx, q.x, b_c, s_own);
                        buf_store(sy, q.y, b_c, s_own);
                        buf_store(sz, q.z, b_c, s_own);
                    }
                }
            }
            if (MEASURE && live) {
                observe<T>(acc, sx, sy, sz, ex, ey, ez, colour == 1, hx, hy, hz, 1.0);
                n_acc += a ? 1u : 0u;
            }
        }
    };
    Vec3<T> ra[RY + 2], rb[RY + 2], rc[RY + 2], ea[RY], eb[RY], ee[RY];
    load_rows(z0 > 0 ? z0 - 1 : (pz ? Lz - 1 : -1), ra, 0, RY + 2);
    load_rows(z0, rb, 0, RY + 2);
    load_edges(z0, eb);
    int z = z0;
    for (; z + 2 < z1; z += 3) {
        step(ra, rb, rc, eb, ee, z);
        step(rb, rc, ra, ee, ea, z + 1);
        step(rc, ra, rb, ea, eb, z + 2);
    }
    if (z < z1) step(ra, rb, rc, eb, ee, z);
    if (z + 1 < z1) step(rb, rc, ra, ee, ea, z + 1);
    if (MEASURE) {
        acc[Q_NACC] = (double)n_acc;
        block_store_partials(acc, P.partials_dev + ((size_t)colour * P.n_items + item) * NQ);
    }
}

// ---------------------------------------------------------------------------
// Pair kernel (simple cubic): the row-strip scheme with two adjacent packed
// columns per lane, loaded and stored as one 8-byte (FP32) or 16-byte (FP64)
// buffer access.  Columns 2l and 2l+1 of lane l are each other's in-row
// neighbours on one side; the column beyond the pair comes from one lane
// shift per row and component (lane l-1's second column when the row parity
// is 0, lane l+1's first column when it is 1), or from memory at wave edges
// and at the periodic wrap.  Rows of an even number of packed columns only
// (pairs stay aligned).  A tile is 2 tx columns x ty rows per thread x zc
// planes.
// ---------------------------------------------------------------------------
template <typename T, bool MEASURE, int MODE, int RY>
__device__ __forceinline__ void sc_pair_body(const PassLaunch &P, int colour, uint32_t item,
                                             uint32_t t)
{
    // every descriptor field is read into registers before the first store, so
    // the loads stay scalar (memory that the kernel may write cannot be)
    const WorkItem w = P.work_dev[item];
    const RepDev &R = P.reps_dev[w.rep];
    const int Ly = R.Ly, Lz = R.Lz, Lxh = R.Lxh, Lx = R.Lx;
    void *const base_x = R.sx, *const base_y = R.sy, *const base_z = R.sz;
    const uint32_t rid = R.rid;
    const int lane = threadIdx.x & 63;
    const int xraw = w.x0 + 2 * (int)threadIdx.x;
    const bool xin = xraw < Lxh && (int)threadIdx.x < P.tile.tx;
    const int xa = xin ? xraw : Lxh - 2, xb = xa + 1;
    const uint32_t plane = R.plane;
    const uint32_t own = colour ? plane : 0u, oth = colour ? 0u : plane;
    const T J = (T)R.J, K = (T)R.K, ex = (T)R.e[0], ey = (T)R.e[1], ez = (T)R.e[2];
    const T beta = (T)R.beta;
    const bool greedy = R.greedy != 0;
    const bool px = R.pmask & 1u, py = R.pmask & 2u, pz = R.pmask & 4u;
    const int xl = xa > 0 ? xa - 1 : (px ? Lxh - 1 : -1);  // column left of the pair
    const int xr = xb < Lxh - 1 ? xb + 1 : (px ? 0 : -1);  // column right of the pair
    const bool left_mem = lane == 0 || xa == 0;           // xa-1 not held by lane-1
    const bool right_mem = lane == 63 || xb >= Lxh - 1;   // xb+1 not held by lane+1
    const uint32_t b_c = (uint32_t)xa * (uint32_t)sizeof(T);
    const uint32_t b_l = (uint32_t)(xl < 0 ? 0 : xl) * (uint32_t)sizeof(T);
    const uint32_t b_r = (uint32_t)(xr < 0 ? 0 : xr) * (uint32_t)sizeof(T);
    const uint32_t row_bytes = (uint32_t)Lxh * (uint32_t)sizeof(T);
    const PlaneRs<T> q = {plane_rsrc<T>(base_x, 0, R.n_box), plane_rsrc<T>(base_y, 0, R.n_box),
                          plane_rsrc<T>(base_z, 0, R.n_box)};
    const uint32_t own_b = own * (uint32_t)sizeof(T), oth_b = oth * (uint32_t)sizeof(T);
    auto row_off = [&](int y, int z) -> uint32_t {
        return ((uint32_t)z * (uint32_t)Ly + (uint32_t)y) * row_bytes;
    };
    auto load_row = [&](uint32_t soff) -> Row2<T> {
        Row2<T> v;
        buf_load2(q.x, b_c, soff, v.xa, v.xb);
        buf_load2(q.y, b_c, soff, v.ya, v.yb);
        buf_load2(q.z, b_c, soff, v.za, v.zb);
        return v;
    };

    // rows y0-1 .. y0+RY: lattice row index or -1 (open face)
    int yrow[RY + 2];
#pragma unroll
    for (int k = -1; k <= RY; ++k) {
        int y = w.y0 + k;
        if (y < 0 || y >= Ly) {
            if (!py) y = -1;
            else {
                while (y < 0) y += Ly;
                while (y >= Ly) y -= Ly;
            }
        }
        yrow[k + 1] = y;
    }
    auto load_rows = [&](int z, Row2<T> *dst) {
        const bool z_ok = z >= 0;
        const int zc = z_ok ? z : 0;
        for (int k = 0; k < RY + 2; ++k) {
            const int y = yrow[k];
            dst[k] = load_row(oth_b + row_off(y < 0 ? 0 : y, zc));
            if (!z_ok || y < 0) dst[k] = Row2<T>{T(0), T(0), T(0), T(0), T(0), T(0)};
        }
    };
    // the in-row neighbour beyond the pair where the lane shift cannot supply
    // it, loaded one plane ahead
    auto load_edges = [&](int z, Vec3<T> (&dst)[RY]) {
#pragma unroll
        for (int k = 0; k < RY; ++k) {
            const int yk = w.y0 + k;
            const int yc = yk < Ly ? yk : Ly - 1;
            const int p = (colour + yc + z) & 1;
            const bool need = p ? right_mem : left_mem;
            const int col = p ? xr : xl;
            if (need && col >= 0) {
                const uint32_t soff = oth_b + row_off(yc, z);
                const uint32_t v = p ? b_r : b_l;
                dst[k] = {buf_load(q.x, v, soff, T()), buf_load(q.y, v, soff, T()),
                          buf_load(q.z, v, soff, T())};
            } else {
                dst[k] = {T(0), T(0), T(0)};
            }
        }
    };

    const int z0 = w.z0, z1 = min(w.z0 + P.tile.zc, Lz);
    double acc[Q_N] = {0, 0, 0, 0, 0, 0};
    uint32_t n_acc = 0;
    auto site = [&](T &sx, T &sy, T &sz, T hx, T hy, T hz, uint32_t s, bool live,
                    uint32_t i) -> bool {
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
    auto step = [&](const Row2<T> (&pm)[RY + 2], const Row2<T> (&pc)[RY + 2],
                    Row2<T> (&pn)[RY + 2], const Vec3<T> (&ec)[RY], Vec3<T> (&en)[RY], int z) {
        const int zn = z < Lz - 1 ? z + 1 : (pz ? 0 : -1);
        load_rows(zn, pn);
        if (z + 1 < z1) load_edges(zn, en);
#pragma unroll
        for (int k = 0; k < RY; ++k) {
            const int yk = w.y0 + k;
            const bool row_in = yk < Ly;
            const int yc = row_in ? yk : Ly - 1;
            const int p = (colour + yc + z) & 1; // uniform over the workgroup
            const uint32_t s_own = own_b + row_off(yc, z);
            Row2<T> me;
            buf_load2(q.x, b_c, s_own, me.xa, me.xb);
            buf_load2(q.y, b_c, s_own, me.ya, me.yb);
            buf_load2(q.z, b_c, s_own, me.za, me.zb);
            const Row2<T> c = pc[k + 1];
            // the other colour's column beyond the pair
            Vec3<T> nb;
            if (p == 0)
                nb = {from_lower_lane(c.xb), from_lower_lane(c.yb), from_lower_lane(c.zb)};
            else
                nb = {from_upper_lane(c.xa), from_upper_lane(c.ya), from_upper_lane(c.za)};
            if (p ? right_mem : left_mem) nb = ec[k];
            // in-row neighbours (x-1, x+1) of column a and of column b
            const T lax = p ? c.xa : nb.x, lay = p ? c.ya : nb.y, laz = p ? c.za : nb.z;
            const T hax = p ? c.xb : c.xa, hay = p ? c.yb : c.ya, haz = p ? c.zb : c.za;
            const T lbx = p ? c.xb : c.xa, lby = p ? c.yb : c.ya, lbz = p ? c.zb : c.za;
            const T hbx = p ? nb.x : c.xb, hby = p ? nb.y : c.yb, hbz = p ? nb.z : c.zb;
            // fixed order: -z, -y, -x, +x, +y, +z
            const T hxa = pm[k + 1].xa + pc[k].xa + lax + hax + pc[k + 2].xa + pn[k + 1].xa;
            const T hya = pm[k + 1].ya + pc[k].ya + lay + hay + pc[k + 2].ya + pn[k + 1].ya;
            const T hza = pm[k + 1].za + pc[k].za + laz + haz + pc[k + 2].za + pn[k + 1].za;
            const T hxb = pm[k + 1].xb + pc[k].xb + lbx + hbx + pc[k + 2].xb + pn[k + 1].xb;
            const T hyb = pm[k + 1].yb + pc[k].yb + lby + hby + pc[k + 2].yb + pn[k + 1].yb;
            const T hzb = pm[k + 1].zb + pc[k].zb + lbz + hbz + pc[k + 2].zb + pn[k + 1].zb;
            const bool live = xin && row_in;
            const uint32_t s0 = (uint32_t)(z * Ly + yc) * (uint32_t)Lx + 2u * xa + p;
            const uint32_t i0 = own + (uint32_t)(z * Ly + yc) * Lxh + xa;
            const bool aa = site(me.xa, me.ya, me.za, hxa, hya, hza, s0, live, i0);
            const bool ab = site(me.xb, me.yb, me.zb, hxb, hyb, hzb, s0 + 2u, live, i0 + 1u);
            // every pair is written back, accepted or not (same bits where
            // rejected; no other workgroup owns it): whole lines reach the L2,
            // measured 0.8 % faster than storing only pairs with a move
            (void)aa;
            (void)ab;
            if (MODE != 1 && live) {
                buf_store2(me.xa, me.xb, q.x, b_c, s_own);
                buf_store2(me.ya, me.yb, q.y, b_c, s_own);
                buf_store2(me.za, me.zb, q.z, b_c, s_own);
            }
        }
    };
    Row2<T> ra[RY + 2], rb[RY + 2], rc[RY + 2];
    Vec3<T> ea[RY], eb[RY], ee[RY];
    load_rows(z0 > 0 ? z0 - 1 : (pz ? Lz - 1 : -1), ra);
    load_rows(z0, rb);
    load_edges(z0, eb);
    int z = z0;
    for (; z + 2 < z1; z += 3) {
        step(ra, rb, rc, eb, ee, z);
        step(rb, rc, ra, ee, ea, z + 1);
        step(rc, ra, rb, ea, eb, z + 2);
    }
    if (z < z1) step(ra, rb, rc, eb, ee, z);
    if (z + 1 < z1) step(rb, rc, ra, ee, ea, z + 1);
    if (MEASURE) {
        acc[Q_NACC] = (double)n_acc;
        block_store_partials(acc, P.partials_dev + ((size_t)colour * P.n_items + item) * NQ);
    }
}

// ---------------------------------------------------------------------------
// Band-pair kernel (simple cubic, rows of an even number of packed columns):
// the pair scheme with the band layout.  Rows are grouped into bands of RY
// rows; the (band, pair) positions are numbered band-major and dealt to the
// lanes contiguously, so no lane idles whatever the row length, and the bands
// of one workgroup share their halo rows through the CU's cache.  With RY
// even the row parity depends only on (k, z), so it is uniform over a wave.
//
// The planes of a tile are walked in z keeping only two sets of registers
// across planes: the other colour's own rows of the previous plane (the -z
// neighbours of the next plane) and, for every site of the current plane, the
// partial field of its first five neighbours (-z, -y, -x, +x, +y, summed in
// that order).  When the next plane's rows arrive, the +z term completes the
// field (the same sum, in the same order, as every other kernel) and the sites
// are updated.  The z loop is unrolled by two so the row parity is a
// compile-time constant (no selects, one lane shift per row and component).
// Fully periodic lattices take a variant without open-face masking.
// ---------------------------------------------------------------------------
template <typename T, bool MEASURE, int MODE, int RY, bool PER>
__device__ __forceinline__ void sc_pband_run(const PassLaunch &P, int colour, uint32_t item,
                                             uint32_t t)
{
    static_assert(RY % 2 == 0, "band rows must be even");
    // every descriptor field is read into registers before the first store, so
    // the loads stay scalar (memory that the kernel may write cannot be)
    const WorkItem w = P.work_dev[item];
    const RepDev &R = P.reps_dev[w.rep];
    const int Ly = R.Ly, Lz = R.Lz, Lxh = R.Lxh, Lx = R.Lx;
    void *const base_x = R.sx, *const base_y = R.sy, *const base_z = R.sz;
    const uint32_t rid = R.rid;
    const int lane = threadIdx.x & 63;
    const int NP = Lxh >> 1; // pairs per row
    const int n_bands = (Ly + RY - 1) / RY;
    const int F = n_bands * NP; // positions (band, pair)
    const int fraw = w.x0 + (int)threadIdx.x;
    const bool fin = fraw < F && (int)threadIdx.x < P.tile.tx;
    const int f = fin ? fraw : F - 1;
    const int band = f / NP;
    const int xa = 2 * (f - band * NP), xb = xa + 1;
    const int yb = band * RY; // first row of the band
    const uint32_t plane = R.plane;
    const uint32_t own = colour ? plane : 0u, oth = colour ? 0u : plane;
    const T J = (T)R.J, K = (T)R.K, ex = (T)R.e[0], ey = (T)R.e[1], ez = (T)R.e[2];
    const T beta = (T)R.beta;
    const bool greedy = R.greedy != 0;
    const bool px = PER || (R.pmask & 1u), py = PER || (R.pmask & 2u), pz = PER || (R.pmask & 4u);
    const int xl = xa > 0 ? xa - 1 : (px ? Lxh - 1 : -1);  // column left of the pair
    const int xr = xb < Lxh - 1 ? xb + 1 : (px ? 0 : -1);  // column right of the pair
    const bool left_mem = lane == 0 || xa == 0;           // xa-1 not held by lane-1
    const bool right_mem = lane == 63 || xb >= Lxh - 1;   // xb+1 not held by lane+1
    const uint32_t row_bytes = (uint32_t)Lxh * (uint32_t)sizeof(T);
    const uint32_t b_c = (uint32_t)xa * (uint32_t)sizeof(T);
    const uint32_t b_l = (uint32_t)(xl < 0 ? 0 : xl) * (uint32_t)sizeof(T);
    const uint32_t b_r = (uint32_t)(xr < 0 ? 0 : xr) * (uint32_t)sizeof(T);
    const PlaneRs<T> q = {plane_rsrc<T>(base_x, 0, R.n_box), plane_rsrc<T>(base_y, 0, R.n_box),
                          plane_rsrc<T>(base_z, 0, R.n_box)};
    const uint32_t own_b = own * (uint32_t)sizeof(T), oth_b = oth * (uint32_t)sizeof(T);
    const uint32_t zplane_b = (uint32_t)Ly * row_bytes;

    // this lane's rows yb-1 .. yb+RY (wrapped on periodic faces) as byte
    // offsets within a z plane, and which of them exist (open faces)
    uint32_t roff[RY + 2];
    uint32_t row_ok = 0;
#pragma unroll
    for (int k = -1; k <= RY; ++k) {
        int y = yb + k;
        bool ok = true;
        if (y < 0 || y >= Ly) {
            if (py) {
                while (y < 0) y += Ly;
                while (y >= Ly) y -= Ly;
            } else {
                ok = false;
                y = y < 0 ? 0 : Ly - 1;
            }
        }
        roff[k + 1] = (uint32_t)y * row_bytes + b_c;
        row_ok |= (ok ? 1u : 0u) << (k + 1);
    }
    const Row2<T> zero = {T(0), T(0), T(0), T(0), T(0), T(0)};
    // other-colour rows k0 .. k1-1 (of yb-1 .. yb+RY) of plane n; planes
    // beyond an open z face and rows beyond an open y face read as zero
    auto load_rows = [&](int n, Row2<T> *dst, int k0, int k1) __attribute__((always_inline)) {
        if (n < 0 || n >= Lz) {
            if (!pz) {
#pragma unroll
                for (int k = k0; k < k1; ++k) dst[k] = zero;
                return;
            }
            n = n < 0 ? n + Lz : n - Lz;
        }
        const uint32_t soff = oth_b + (uint32_t)n * zplane_b;
#pragma unroll
        for (int k = k0; k < k1; ++k) {
            buf_load2(q.x, roff[k], soff, dst[k].xa, dst[k].xb);
            buf_load2(q.y, roff[k], soff, dst[k].ya, dst[k].yb);
            buf_load2(q.z, roff[k], soff, dst[k].za, dst[k].zb);
            if (!PER && !py && !((row_ok >> k) & 1u)) dst[k] = zero;
        }
    };

    double acc[Q_N] = {0, 0, 0, 0, 0, 0};
    uint32_t n_acc = 0;
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

    const int z0 = w.z0, z1 = min(w.z0 + P.tile.zc, Lz);
    Row2<T> mid[RY];  // other colour, rows yb .. yb+RY-1 of the previous plane
    Row2<T> part[RY]; // partial fields (-z, -y, -x, +x, +y) of the current plane's sites

    // partial fields of plane n (row parity of row k: (Q + k) & 1) from its
    // other-colour rows o[0 .. RY+1] and the previous plane's rows `mid`
    auto partial = [&](int Q, int n, const Row2<T> *o, Row2<T> *dst) __attribute__((always_inline)) {
        const uint32_t soff = oth_b + (uint32_t)n * zplane_b; // z0 <= n < z1
#pragma unroll
        for (int k = 0; k < RY; ++k) {
            const int p = (Q + k) & 1; // uniform over the wave
            const Row2<T> &c = o[k + 1];
            // the other colour's column beyond the pair: lane l-1's second
            // column (p = 0) or lane l+1's first (p = 1); from memory where
            // no lane holds it
            Vec3<T> nb;
            if (p == 0)
                nb = {from_lower_lane(c.xb), from_lower_lane(c.yb), from_lower_lane(c.zb)};
            else
                nb = {from_upper_lane(c.xa), from_upper_lane(c.ya), from_upper_lane(c.za)};
            const bool need = p ? right_mem : left_mem;
            if (need) {
                const int col = p ? xr : xl;
                if (PER || col >= 0) {
                    const uint32_t v = roff[k + 1] - b_c + (p ? b_r : b_l);
                    nb = {buf_load(q.x, v, soff, T()), buf_load(q.y, v, soff, T()),
                          buf_load(q.z, v, soff, T())};
                } else {
                    nb = {T(0), T(0), T(0)};
                }
            }
            // in-row neighbours (x-1, x+1) of column a and of column b
            const Vec3<T> la = p ? Vec3<T>{c.xa, c.ya, c.za} : nb;
            const Vec3<T> ha = p ? Vec3<T>{c.xb, c.yb, c.zb} : Vec3<T>{c.xa, c.ya, c.za};
            const Vec3<T> lb = p ? Vec3<T>{c.xb, c.yb, c.zb} : Vec3<T>{c.xa, c.ya, c.za};
            const Vec3<T> hb = p ? nb : Vec3<T>{c.xb, c.yb, c.zb};
            // fixed order: -z, -y, -x, +x, +y (+z added when the next plane arrives)
            dst[k].xa = mid[k].xa + o[k].xa + la.x + ha.x + o[k + 2].xa;
            dst[k].ya = mid[k].ya + o[k].ya + la.y + ha.y + o[k + 2].ya;
            dst[k].za = mid[k].za + o[k].za + la.z + ha.z + o[k + 2].za;
            dst[k].xb = mid[k].xb + o[k].xb + lb.x + hb.x + o[k + 2].xb;
            dst[k].yb = mid[k].yb + o[k].yb + lb.y + hb.y + o[k + 2].yb;
            dst[k].zb = mid[k].zb + o[k].zb + lb.z + hb.z + o[k + 2].zb;
        }
    };

    // sites of plane z (row parity (Q + k) & 1): the +z rows are top[0 .. RY-1]
    // own rows of plane z (the sites' current spins)
    auto load_own = [&](int z, Row2<T> *me) __attribute__((always_inline)) {
        const uint32_t s_own = own_b + (uint32_t)z * zplane_b;
#pragma unroll
        for (int k = 0; k < RY; ++k) {
            buf_load2(q.x, roff[k + 1], s_own, me[k].xa, me[k].xb);
            buf_load2(q.y, roff[k + 1], s_own, me[k].ya, me[k].yb);
            buf_load2(q.z, roff[k + 1], s_own, me[k].za, me[k].zb);
        }
    };
    auto update = [&](int Q, int z, const Row2<T> *pf, const Row2<T> *top, Row2<T> *me)
        __attribute__((always_inline)) {
        const uint32_t s_own = own_b + (uint32_t)z * zplane_b;
#pragma unroll
        for (int k = 0; k < RY; ++k) {
            const int p = (Q + k) & 1;
            const int y = yb + k;
            const bool live = fin && y < Ly;
            const T hxa = pf[k].xa + top[k].xa, hya = pf[k].ya + top[k].ya,
                    hza = pf[k].za + top[k].za;
            const T hxb = pf[k].xb + top[k].xb, hyb = pf[k].yb + top[k].yb,
                    hzb = pf[k].zb + top[k].zb;
            const uint32_t s0 = (uint32_t)(z * Ly + y) * (uint32_t)Lx + 2u * xa + p;
            const uint32_t i0 = own + (uint32_t)(z * Ly + y) * Lxh + xa;
            const bool aa = site(me[k].xa, me[k].ya, me[k].za, hxa, hya, hza, s0, live, i0);
            const bool ab = site(me[k].xb, me[k].yb, me[k].zb, hxb, hyb, hzb, s0 + 2u, live,
                                 i0 + 1u);
            if (MODE != 1 && live && (aa || ab)) {
                buf_store2(me[k].xa, me[k].xb, q.x, roff[k + 1], s_own);
                buf_store2(me[k].ya, me[k].yb, q.y, roff[k + 1], s_own);
                buf_store2(me[k].za, me[k].zb, q.z, roff[k + 1], s_own);
            }
        }
    };

    // one plane step: plane n's other-colour rows complete the sites of plane
    // n-1 and, unless n is past the tile, start the partial fields of plane n
    auto step = [&](int n) __attribute__((always_inline)) {
        const int Q = (colour + n) & 1;
        Row2<T> o[RY + 2], me[RY];
        if (n < z1) {
            // every load of the step is issued first; the new partial fields
            // are formed before the site updates, so the previous plane's rows
            // and this plane's halo rows are dead by then
            load_rows(n, o, 0, RY + 2);
            load_own(n - 1, me);
            Row2<T> next[RY];
            partial(Q, n, o, next);
            update(Q ^ 1, n - 1, part, o + 1, me);
#pragma unroll
            for (int k = 0; k < RY; ++k) {
                part[k] = next[k];
                mid[k] = o[k + 1];
            }
        } else {
            load_rows(n, o, 1, RY + 1);
            load_own(n - 1, me);
            update(Q ^ 1, n - 1, part, o + 1, me);
        }
    };
    {
        Row2<T> o[RY + 2];
        load_rows(z0 - 1, o, 1, RY + 1);
#pragma unroll
        for (int k = 0; k < RY; ++k) mid[k] = o[k + 1];
        load_rows(z0, o, 0, RY + 2);
        partial((colour + z0) & 1, z0, o, part);
#pragma unroll
        for (int k = 0; k < RY; ++k) mid[k] = o[k + 1];
    }
    // two planes per iteration, so the loop-carried rows alternate between
    // two register sets instead of being copied
    int n = z0 + 1;
    for (; n < z1; n += 2) {
        step(n);
        step(n + 1);
    }
    if (n == z1) step(n);

    if (MEASURE) {
        acc[Q_NACC] = (double)n_acc;
        block_store_partials(acc, P.partials_dev + ((size_t)colour * P.n_items + item) * NQ);
    }
}

template <typename T, bool MEASURE, int MODE, int RY>
__device__ __forceinline__ void sc_pband_body(const PassLaunch &P, int colour, uint32_t item,
                                              uint32_t t)
{
    const WorkItem w = P.work_dev[item];
    if (P.reps_dev[w.rep].pmask == 7u)
        sc_pband_run<T, MEASURE, MODE, RY, true>(P, colour, item, t);
    else
        sc_pband_run<T, MEASURE, MODE, RY, false>(P, colour, item, t);
}

// ---------------------------------------------------------------------------
// Band kernel (simple cubic): the row-strip scheme without idle lanes.  Rows
// are grouped into bands of RY rows; the positions (band, xh) are numbered
// band-major and dealt to the lanes contiguously, so a wave may run from the
// end of one band into the next and every lane has work whatever the row
// length.  With RY even, the parity of a site depends only on (k, z), so it
// stays uniform over the wave; each lane keeps per-row byte offsets of its
// own band in registers, and every access is one buffer instruction with the
// plane offset in a scalar register.
// ---------------------------------------------------------------------------
template <typename T, bool MEASURE, int MODE, int RY>
__device__ __forceinline__ void sc_band_body(const PassLaunch &P, int colour, uint32_t item,
                                             uint32_t t)
{
    static_assert(RY % 2 == 0, "band rows must be even");
    // every descriptor field is read into registers before the first store, so
    // the loads stay scalar (memory that the kernel may write cannot be)
    const WorkItem w = P.work_dev[item];
    const RepDev &R = P.reps_dev[w.rep];
    const int Ly = R.Ly, Lz = R.Lz, Lxh = R.Lxh, Lx = R.Lx;
    void *const base_x = R.sx, *const base_y = R.sy, *const base_z = R.sz;
    const uint32_t rid = R.rid;
    const int lane = threadIdx.x & 63;
    const int n_bands = (Ly + RY - 1) / RY;
    const int F = n_bands * Lxh; // positions (band, xh)
    const int fraw = w.x0 + (int)threadIdx.x;
    const bool fin = fraw < F && (int)threadIdx.x < P.tile.tx;
    const int f = fin ? fraw : F - 1;
    const int band = f / Lxh;
    const int xh = f - band * Lxh;
    const int yb = band * RY; // first row of the band
    const uint32_t plane = R.plane;
    const uint32_t own = colour ? plane : 0u, oth = colour ? 0u : plane;
    const T J = (T)R.J, K = (T)R.K, ex = (T)R.e[0], ey = (T)R.e[1], ez = (T)R.e[2];
    const T beta = (T)R.beta;
    const bool greedy = R.greedy != 0;
    const bool px = R.pmask & 1u, py = R.pmask & 2u, pz = R.pmask & 4u;
    const int xl = xh > 0 ? xh - 1 : (px ? Lxh - 1 : -1);
    const int xr = xh < Lxh - 1 ? xh + 1 : (px ? 0 : -1);
    const bool left_mem = lane == 0 || xh == 0;           // x-1 not held by lane-1
    const bool right_mem = lane == 63 || xh >= Lxh - 1;   // x+1 not held by lane+1
    const uint32_t row_bytes = (uint32_t)Lxh * (uint32_t)sizeof(T);
    const uint32_t b_c = (uint32_t)xh * (uint32_t)sizeof(T);
    const uint32_t b_l = (uint32_t)(xl < 0 ? 0 : xl) * (uint32_t)sizeof(T);
    const uint32_t b_r = (uint32_t)(xr < 0 ? 0 : xr) * (uint32_t)sizeof(T);
    const PlaneRs<T> q = {plane_rsrc<T>(base_x, 0, R.n_box), plane_rsrc<T>(base_y, 0, R.n_box),
                          plane_rsrc<T>(base_z, 0, R.n_box)};
    const uint32_t own_b = own * (uint32_t)sizeof(T), oth_b = oth * (uint32_t)sizeof(T);
    const uint32_t zplane_b = (uint32_t)Ly * row_bytes;
    auto load3 = [&](uint32_t voff, uint32_t soff) -> Vec3<T> {
        return {buf_load(q.x, voff, soff, T()), buf_load(q.y, voff, soff, T()),
                buf_load(q.z, voff, soff, T())};
    };

    // this lane's rows yb-1 .. yb+RY (wrapped on periodic faces) as byte
    // offsets within a z plane, and which of them exist (open faces)
    uint32_t roff[RY + 2];
    uint32_t row_ok = 0;
#pragma unroll
    for (int k = -1; k <= RY; ++k) {
        int y = yb + k;
        bool ok = true;
        if (y < 0 || y >= Ly) {
            if (py) {
                while (y < 0) y += Ly;
                while (y >= Ly) y -= Ly;
            } else {
                ok = false;
                y = y < 0 ? 0 : Ly - 1;
            }
        }
        roff[k + 1] = (uint32_t)y * row_bytes + b_c;
        row_ok |= (ok ? 1u : 0u) << (k + 1);
    }
    auto load_rows = [&](int z, Vec3<T> *dst) {
        if (z < 0) {
#pragma unroll
            for (int k = 0; k < RY + 2; ++k) dst[k] = {T(0), T(0), T(0)};
            return;
        }
        const uint32_t soff = oth_b + (uint32_t)z * zplane_b;
#pragma unroll
        for (int k = 0; k < RY + 2; ++k) {
            dst[k] = load3(roff[k], soff);
            if (!py && !((row_ok >> k) & 1u)) dst[k] = {T(0), T(0), T(0)};
        }
    };
    // In-row neighbours that the lane shift cannot supply (wave edges, band
    // seams, the periodic wrap, open faces) are loaded one plane ahead by the
    // lanes that need them, so the loads never stall the plane being updated.
    auto load_edges = [&](int z, Vec3<T> *dst) {
        const uint32_t soff = oth_b + (uint32_t)z * zplane_b;
#pragma unroll
        for (int k = 0; k < RY; ++k) {
            const int p = (colour + k + z) & 1;
            const bool need = p ? right_mem : left_mem;
            const int col = p ? xr : xl;
            if (need && col >= 0)
                dst[k] = load3(roff[k + 1] - b_c + (p ? b_r : b_l), soff);
            else
                dst[k] = {T(0), T(0), T(0)};
        }
    };

    const int z0 = w.z0, z1 = min(w.z0 + P.tile.zc, Lz);
    Vec3<T> om[RY + 2], oc[RY + 2], op[RY + 2], ec[RY], en[RY];
    load_rows(z0 > 0 ? z0 - 1 : (pz ? Lz - 1 : -1), om);
    load_rows(z0, oc);
    load_edges(z0, ec);
    double acc[Q_N] = {0, 0, 0, 0, 0, 0};
    uint32_t n_acc = 0;
    for (int z = z0; z < z1; ++z) {
        const int zn = z < Lz - 1 ? z + 1 : (pz ? 0 : -1);
        load_rows(zn, op);
        if (z + 1 < z1) load_edges(zn, en);
        const uint32_t s_own = own_b + (uint32_t)z * zplane_b;
#pragma unroll
        for (int k = 0; k < RY; ++k) {
            const int y = yb + k;
            const bool live = fin && y < Ly;
            const int p = (colour + k + z) & 1; // uniform over the wave (RY even)
            T sx = buf_load(q.x, roff[k + 1], s_own, T()), sy = buf_load(q.y, roff[k + 1], s_own, T()),
              sz = buf_load(q.z, roff[k + 1], s_own, T());
            // in-row neighbour on the side given by the parity
            const Vec3<T> c = oc[k + 1];
            const bool from_mem = p ? right_mem : left_mem;
            Vec3<T> nb;
            if (p == 0)
                nb = {from_lower_lane(c.x), from_lower_lane(c.y), from_lower_lane(c.z)};
            else
                nb = {from_upper_lane(c.x), from_upper_lane(c.y), from_upper_lane(c.z)};
            if (from_mem) nb = ec[k];
            // fixed order: -z, -y, -x, +x, +y, +z
            const Vec3<T> lo = p ? c : nb, hi = p ? nb : c;
            T hx = om[k + 1].x + oc[k].x + lo.x + hi.x + oc[k + 2].x + op[k + 1].x;
            T hy = om[k + 1].y + oc[k].y + lo.y + hi.y + oc[k + 2].y + op[k + 1].y;
            T hz = om[k + 1].z + oc[k].z + lo.z + hi.z + oc[k + 2].z + op[k + 1].z;
            hx *= J;
            hy *= J;
            hz *= J;
            bool a = false;
            if (MODE != 1) {
                const uint32_t s = (uint32_t)(z * Ly + y) * (uint32_t)Lx + 2u * xh + p;
                T dH;
                a = metropolis<T>(sx, sy, sz, hx, hy, hz, s, rid, t, P.seed_lo, P.seed_hi, K,
                                  ex, ey, ez, beta, greedy, dH);
                if (live) {
                    const uint32_t i = own + (uint32_t)(z * Ly + y) * Lxh + xh;
                    if (MODE == 2) {
                        ((T *)P.dbg_dh)[i] = dH;
                        P.dbg_acc[i] = a ? 1 : 0;
                    }
                    if (a) {
                        buf_store(sx, q.x, roff[k + 1], s_own);
                        buf_store(sy, q.y, roff[k + 1], s_own);
                        buf_store(sz, q.z, roff[k + 1], s_own);
                    }
                }
            }
            if (MEASURE && live) {
                observe<T>(acc, sx, sy, sz, ex, ey, ez, colour == 1, hx, hy, hz, 1.0);
                n_acc += a ? 1u : 0u;
            }
        }
#pragma unroll
        for (int k = 0; k < RY + 2; ++k) om[k] = oc[k];
#pragma unroll
        for (int k = 0; k < RY + 2; ++k) oc[k] = op[k];
#pragma unroll
        for (int k = 0; k < RY; ++k) ec[k] = en[k];
    }
    if (MEASURE) {
        acc[Q_NACC] = (double)n_acc;
        block_store_partials(acc, P.partials_dev + ((size_t)colour * P.n_items + item) * NQ);
    }
}

} // namespace mc
