// basis_bodies.hpp -- bcc / fcc colour-pass bodies (one work item each): the
// tile scheme and the register-streaming strip scheme.  Shared by the pass
// kernels and the persistent kernel.
#pragma once

#include "device_common.hpp"

namespace mc {

// ---------------------------------------------------------------------------
// bcc / fcc: colour = basis site B, one dense plane per basis site.  The
// neighbours of a B site in basis b2 sit at cell offsets o with o_a = 0 on
// axes where the two basis vectors agree and o_a in {0, -sign(d_a)} where
// they differ (d = basis(b2) - basis(B), half-cell units): 4 cells per other
// basis for fcc, 8 for bcc.  Unoccupied sites hold zero, so the field sum is
// branch-free inside the box.
// ---------------------------------------------------------------------------
template <int KIND, int B, typename T, bool MEASURE, int MODE>
__device__ __forceinline__ void basis_body(const PassLaunch &P, uint32_t item, uint32_t t)
{
    constexpr int NB = basis_count(KIND);
    const WorkItem w = P.work_dev[item];
    const RepDev &R = P.reps_dev[w.rep];
    const int Lx = R.Lx, Ly = R.Ly, Lz = R.Lz;
    const int lx = threadIdx.x % P.tile.tx, ly = threadIdx.x / P.tile.tx;
    const int x = w.x0 + lx, y = w.y0 + ly;
    const bool active = x < Lx && y < Ly && ly < P.tile.ty;
    const uint32_t plane = R.plane;
    const gptr<T> gx = as_global<T>(R.sx), gy = as_global<T>(R.sy), gz = as_global<T>(R.sz);
    const T J = (T)R.J, K = (T)R.K, ex = (T)R.e[0], ey = (T)R.e[1], ez = (T)R.e[2];
    const double Jd = R.J;
    const T beta = (T)R.beta;
    const bool greedy = R.greedy != 0;
    const bool pxm = R.pmask & 1u, pym = R.pmask & 2u, pzm = R.pmask & 4u;
    constexpr int bx = basis2(KIND, B, 0), by = basis2(KIND, B, 1), bz = basis2(KIND, B, 2);

    double acc[Q_N] = {0, 0, 0, 0, 0, 0};
    if (active) {
        const int z1 = min(w.z0 + P.tile.zc, Lz);
        for (int z = w.z0; z < z1; ++z) {
            if (!occupied(R, x, y, z, bx, by, bz)) continue;
            const uint32_t cell = (uint32_t)(z * Ly + y) * Lx + x;
            T hx, hy, hz, lx_, ly_, lz_;
            basis_site_field<KIND, B, T>(gx, gy, gz, plane, Lx, Ly, Lz, pxm, pym, pzm, x, y, z,
                                         hx, hy, hz, lx_, ly_, lz_);
            hx *= J;
            hy *= J;
            hz *= J;
            const uint32_t i = (uint32_t)B * plane + cell;
            T sx = gx[i], sy = gy[i], sz = gz[i];
            bool a = false;
            if (MODE != 1) {
                const uint32_t s = cell * NB + B;
                T dH;
                a = metropolis<T>(sx, sy, sz, hx, hy, hz, s, R.rid, t, P.seed_lo, P.seed_hi, K,
                                  ex, ey, ez, beta, greedy, dH);
                if (MODE == 2) {
                    ((T *)P.dbg_dh)[i] = dH;
                    P.dbg_acc[i] = a ? 1 : 0;
                }
                if (a) {
                    gx[i] = sx;
                    gy[i] = sy;
                    gz[i] = sz;
                }
            }
            // bonds to lower colours, whose spins are final after their pass
            if (MEASURE) {
                observe<T>(acc, sx, sy, sz, ex, ey, ez, true, lx_, ly_, lz_, Jd);
                acc[Q_NACC] += a ? 1.0 : 0.0;
            }
        }
    }
    if (MEASURE)
        block_store_partials(acc, P.partials_dev + ((size_t)B * P.n_items + item) * NQ);
}

// ---------------------------------------------------------------------------
// Basis-lattice strip kernel (bcc / fcc): lanes along x (tx a multiple of 64,
// so a wave never straddles rows), one row per thread, walking the tile's
// planes in z.  For each other basis site b2, with d = basis(b2) - basis(B)
// in half-cell units, the neighbour cells are (x - ix dx, y - iy dy,
// z - iz dz): the rows y and y - dy of planes z and z - dz sit in registers
// (one new plane per step: the other one rolls over from the previous
// step), and the cell x - dx comes from the adjacent lane by a DPP lane
// shift, or from memory at wave edges and at the periodic wrap.  The sums
// follow basis_site_field's order exactly.
// ---------------------------------------------------------------------------
template <int KIND, int B, typename T, bool MEASURE, int MODE>
__device__ __forceinline__ void basis_strip_body(const PassLaunch &P, uint32_t item, uint32_t t)
{
    constexpr int NB = basis_count(KIND);
    constexpr int bx = basis2(KIND, B, 0), by = basis2(KIND, B, 1), bz = basis2(KIND, B, 2);
    const WorkItem w = P.work_dev[item];
    const RepDev &R = P.reps_dev[w.rep];
    const int Lx = R.Lx, Ly = R.Ly, Lz = R.Lz;
    const int lane = threadIdx.x & 63;
    const int lxi = threadIdx.x % P.tile.tx, lyi = threadIdx.x / P.tile.tx;
    const int xraw = w.x0 + lxi, yraw = w.y0 + lyi;
    const bool row_live = yraw < Ly && lyi < P.tile.ty;
    const bool live_x = xraw < Lx;
    const int x = live_x ? xraw : Lx - 1; // lanes past the row end mirror its last cell
    const int y = row_live ? yraw : Ly - 1;
    const uint32_t plane = R.plane;
    const gptr<T> gx = as_global<T>(R.sx), gy = as_global<T>(R.sy), gz = as_global<T>(R.sz);
    const T J = (T)R.J, K = (T)R.K, ex = (T)R.e[0], ey = (T)R.e[1], ez = (T)R.e[2];
    const double Jd = R.J;
    const T beta = (T)R.beta;
    const bool greedy = R.greedy != 0;
    const bool pxm = R.pmask & 1u, pym = R.pmask & 2u, pzm = R.pmask & 4u;
    auto wrap = [](int v, int L, bool per, bool &ok) {
        if (v < 0) { v += L; ok &= per; }
        if (v >= L) { v -= L; ok &= per; }
        return v;
    };
    auto ld = [&](uint32_t b2, int cx, int cy, int cz, bool ok) -> Vec3<T> {
        if (!ok) return {T(0), T(0), T(0)};
        const uint32_t j = b2 * plane + (uint32_t)(cz * Ly + cy) * Lx + cx;
        return {gx[j], gy[j], gz[j]};
    };

    // per other basis site: registers [iz][iy] and the row / column geometry
    Vec3<T> V[NB][2][2];
    const int z0 = w.z0, z1 = min(w.z0 + P.tile.zc, Lz);
#pragma unroll
    for (int b2 = 0; b2 < NB; ++b2) {
        if (b2 == B) continue;
        const int dy = basis2(KIND, b2, 1) - by, dz = basis2(KIND, b2, 2) - bz;
        bool oky0 = true, oky1 = true;
        const int y0r = y, y1r = wrap(y - dy, Ly, pym, oky1);
        // before the loop: the plane that the first step rolls over
        if (dz > 0) {
            bool okz = true;
            const int cz = wrap(z0 - 1, Lz, pzm, okz);
            V[b2][0][0] = ld(b2, x, y0r, cz, okz && oky0);
            if (dy) V[b2][0][1] = ld(b2, x, y1r, cz, okz && oky1);
        } else if (dz < 0) {
            V[b2][1][0] = ld(b2, x, y0r, z0, oky0);
            if (dy) V[b2][1][1] = ld(b2, x, y1r, z0, oky1);
        }
    }

    double acc[Q_N] = {0, 0, 0, 0, 0, 0};
    for (int z = z0; z < z1; ++z) {
        T hx = 0, hy = 0, hz = 0, lx_ = 0, ly_ = 0, lz_ = 0;
#pragma unroll
        for (int b2 = 0; b2 < NB; ++b2) {
            if (b2 == B) continue;
            const int dx = basis2(KIND, b2, 0) - bx;
            const int dy = basis2(KIND, b2, 1) - by;
            const int dz = basis2(KIND, b2, 2) - bz;
            bool oky1 = true;
            const int y1r = wrap(y - dy, Ly, pym, oky1);
            // roll the planes and load the new one
            if (dz > 0) { // planes z (iz 0) and z-1 (iz 1)
                V[b2][1][0] = V[b2][0][0];
                if (dy) V[b2][1][1] = V[b2][0][1];
                V[b2][0][0] = ld(b2, x, y, z, true);
                if (dy) V[b2][0][1] = ld(b2, x, y1r, z, oky1);
            } else if (dz < 0) { // planes z (iz 0) and z+1 (iz 1)
                bool okz = true;
                const int cz = wrap(z + 1, Lz, pzm, okz);
                V[b2][0][0] = V[b2][1][0];
                if (dy) V[b2][0][1] = V[b2][1][1];
                V[b2][1][0] = ld(b2, x, y, cz, okz);
                if (dy) V[b2][1][1] = ld(b2, x, y1r, cz, okz && oky1);
            } else {
                V[b2][0][0] = ld(b2, x, y, z, true);
                if (dy) V[b2][0][1] = ld(b2, x, y1r, z, oky1);
            }
            // the column x - dx: lane shift, or memory at wave edges and the wrap
            bool okx = true;
            const int xs = wrap(x - dx, Lx, pxm, okx);
            const bool from_mem = dx > 0 ? (lane == 0 || x == 0) : (lane == 63 || x >= Lx - 1);
            const int noz = dz ? 2 : 1, noy = dy ? 2 : 1, nox = dx ? 2 : 1;
            T ax = 0, ay = 0, az = 0;
#pragma unroll
            for (int iz = 0; iz < noz; ++iz) {
                bool okz = true;
                const int cz = wrap(z - iz * dz, Lz, pzm, okz);
#pragma unroll
                for (int iy = 0; iy < noy; ++iy) {
                    const bool oky = iy ? oky1 : true;
                    const Vec3<T> v = V[b2][iz][iy];
#pragma unroll
                    for (int ix = 0; ix < nox; ++ix) {
                        if (ix == 0) {
                            if (okz && oky) {
                                ax += v.x;
                                ay += v.y;
                                az += v.z;
                            }
                        } else {
                            Vec3<T> s;
                            if (dx > 0)
                                s = {from_lower_lane(v.x), from_lower_lane(v.y), from_lower_lane(v.z)};
                            else
                                s = {from_upper_lane(v.x), from_upper_lane(v.y), from_upper_lane(v.z)};
                            if (from_mem) s = ld(b2, xs, iy ? y1r : y, cz, okx && okz && oky);
                            if (okz && oky && okx) {
                                ax += s.x;
                                ay += s.y;
                                az += s.z;
                            }
                        }
                    }
                }
            }
            hx += ax;
            hy += ay;
            hz += az;
            if (b2 < B) {
                lx_ += ax;
                ly_ += ay;
                lz_ += az;
            }
        }
        const bool live = live_x && row_live && occupied(R, x, y, z, bx, by, bz);
        if (!live) continue;
        hx *= J;
        hy *= J;
        hz *= J;
        const uint32_t cell = (uint32_t)(z * Ly + y) * Lx + x;
        const uint32_t i = (uint32_t)B * plane + cell;
        T sx = gx[i], sy = gy[i], sz = gz[i];
        bool a = false;
        if (MODE != 1) {
            const uint32_t s = cell * NB + B;
            T dH;
            a = metropolis<T>(sx, sy, sz, hx, hy, hz, s, R.rid, t, P.seed_lo, P.seed_hi, K, ex, ey,
                              ez, beta, greedy, dH);
            if (MODE == 2) {
                ((T *)P.dbg_dh)[i] = dH;
                P.dbg_acc[i] = a ? 1 : 0;
            }
            if (a) {
                gx[i] = sx;
                gy[i] = sy;
                gz[i] = sz;
            }
        }
        if (MEASURE) {
            observe<T>(acc, sx, sy, sz, ex, ey, ez, true, lx_, ly_, lz_, Jd);
            acc[Q_NACC] += a ? 1.0 : 0.0;
        }
    }
    if (MEASURE)
        block_store_partials(acc, P.partials_dev + ((size_t)B * P.n_items + item) * NQ);
}

// ---------------------------------------------------------------------------
// Basis pair kernel (bcc, fcc; Lx even): two cells (2p, 2p+1) of basis B per
// lane and RY rows per lane.  Positions (band of RY rows, pair p) numbered
// band-major are dealt to the lanes contiguously, so every lane has work
// whatever the row length and the lanes of one wave may hold different rows:
// row offsets are per lane, the basis and plane offsets scalar, and every
// access is one buffer instruction (8 bytes per component for FP32, 16 for
// FP64).  For each other basis b2 (offset d = b2 - B in half cells) the rows
// y - dy of the band and the planes z, z - dz sit in registers and roll along
// z; the column x - dx is the pair's own other cell or the neighbouring
// lane's (DPP), or, at wave edges, row ends and the periodic wrap, a word
// loaded with the row.  Missing neighbours (open faces) load as zero, which
// adds exactly nothing to the partial sums (they start at +0 and cannot
// become -0).  The field is summed in the order of basis_site_field, so the
// Markov chain is the tile kernel's, bitwise.
// ---------------------------------------------------------------------------
template <int KIND, int B, typename T, bool MEASURE, int MODE, int RY>
__device__ __forceinline__ void basis_pair_body(const PassLaunch &P, uint32_t item, uint32_t t)
{
    constexpr int NB = basis_count(KIND);
    constexpr int bx = basis2(KIND, B, 0), by = basis2(KIND, B, 1), bz = basis2(KIND, B, 2);
    // every descriptor field is read into registers before the first store, so
    // the loads stay scalar (memory that the kernel may write cannot be)
    const WorkItem w = P.work_dev[item];
    const RepDev &R = P.reps_dev[w.rep];
    const int Lx = R.Lx, Ly = R.Ly, Lz = R.Lz;
    void *const base_x = R.sx, *const base_y = R.sy, *const base_z = R.sz;
    const uint32_t n_box = R.n_box, plane = R.plane, rid = R.rid;
    const T J = (T)R.J, K = (T)R.K, ex = (T)R.e[0], ey = (T)R.e[1], ez = (T)R.e[2];
    const double Jd = R.J;
    const T beta = (T)R.beta;
    const bool greedy = R.greedy != 0;
    const bool px = R.pmask & 1u, py = R.pmask & 2u, pz = R.pmask & 4u;
    const bool sphere = R.sphere;
    const double r2x4 = R.r2x4;
    const int lane = threadIdx.x & 63;
    const int NPR = Lx >> 1; // pairs per row
    const int n_bands = (Ly + RY - 1) / RY;
    const int F = n_bands * NPR; // positions (band, pair)
    const int fraw = w.x0 + (int)threadIdx.x;
    const bool fin = fraw < F && (int)threadIdx.x < P.tile.tx;
    const int f = fin ? fraw : F - 1;
    const int band = f / NPR;
    const int xa = 2 * (f - band * NPR), xb = xa + 1;
    const int yb = band * RY; // first row of the band
    const int xl = xa > 0 ? xa - 1 : (px ? Lx - 1 : -1); // column left of the pair
    const int xr = xb < Lx - 1 ? xb + 1 : (px ? 0 : -1); // column right of the pair
    const bool left_mem = lane == 0 || xa == 0;         // xa-1 not held by lane-1
    const bool right_mem = lane == 63 || xb >= Lx - 1;  // xb+1 not held by lane+1
    const uint32_t esz = (uint32_t)sizeof(T);
    const uint32_t row_bytes = (uint32_t)Lx * esz, zplane_b = (uint32_t)Ly * row_bytes;
    const uint32_t basis_b = plane * esz;
    const uint32_t b_c = (uint32_t)xa * esz;
    const uint32_t b_l = (uint32_t)(xl < 0 ? 0 : xl) * esz;
    const uint32_t b_r = (uint32_t)(xr < 0 ? 0 : xr) * esz;
    const PlaneRs<T> q = {plane_rsrc<T>(base_x, 0, n_box), plane_rsrc<T>(base_y, 0, n_box),
                          plane_rsrc<T>(base_z, 0, n_box)};
    // this lane's rows yb-1 .. yb+RY (wrapped on periodic faces) as byte
    // offsets of column xa within a plane, and which of them exist
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
    auto occ = [&](int x, int y, int z) -> bool {
        if (!sphere) return true;
        const int qx = 2 * x + bx - Lx, qy = 2 * y + by - Ly, qz = 2 * z + bz - Lz;
        return (double)(qx * qx + qy * qy + qz * qz) <= r2x4;
    };

    // other basis b2: [b2][slot][window row]; slot 0 = plane z, slot 1 =
    // plane z - dz; window row j = row yb - max(dy, 0) + j
    Row2<T> V[NB][2][RY + 1];
    Vec3<T> E[NB][2][RY + 1]; // the column x - dx where it comes from memory
    auto load_plane = [&](int b2, int dx, int dy, int cz, bool okz, Row2<T> *dst, Vec3<T> *edst) {
        const int j0 = dy > 0 ? 1 : 0;
        const int nrow = RY + (dy != 0 ? 1 : 0);
        const uint32_t soff = (uint32_t)b2 * basis_b + (uint32_t)(okz ? cz : 0) * zplane_b;
#pragma unroll
        for (int j = 0; j < nrow; ++j) {
            const int k = j - j0; // row yb + k
            const bool ok = okz && ((row_ok >> (k + 1)) & 1u);
            Row2<T> v;
            buf_load2(q.x, roff[k + 1], soff, v.xa, v.xb);
            buf_load2(q.y, roff[k + 1], soff, v.ya, v.yb);
            buf_load2(q.z, roff[k + 1], soff, v.za, v.zb);
            if (!ok) v = Row2<T>{T(0), T(0), T(0), T(0), T(0), T(0)};
            dst[j] = v;
            if (dx != 0) {
                const bool need = dx > 0 ? (left_mem && xl >= 0) : (right_mem && xr >= 0);
                Vec3<T> e = {T(0), T(0), T(0)};
                if (need && ok) {
                    const uint32_t vo = roff[k + 1] - b_c + (dx > 0 ? b_l : b_r);
                    e = {buf_load(q.x, vo, soff, T()), buf_load(q.y, vo, soff, T()),
                         buf_load(q.z, vo, soff, T())};
                }
                edst[j] = e;
            }
        }
    };
    const int z0 = w.z0, z1 = min(w.z0 + P.tile.zc, Lz);
    // before the loop: the plane that the first step rolls over
#pragma unroll
    for (int b2 = 0; b2 < NB; ++b2) {
        if (b2 == B) continue;
        const int dx = basis2(KIND, b2, 0) - bx, dy = basis2(KIND, b2, 1) - by;
        const int dz = basis2(KIND, b2, 2) - bz;
        if (dz > 0) {
            const int cz = z0 > 0 ? z0 - 1 : (pz ? Lz - 1 : -1);
            load_plane(b2, dx, dy, cz, cz >= 0, V[b2][0], E[b2][0]);
        } else if (dz < 0) {
            load_plane(b2, dx, dy, z0, true, V[b2][1], E[b2][1]);
        }
    }

    double acc[Q_N] = {0, 0, 0, 0, 0, 0};
    auto site = [&](T &sx, T &sy, T &sz, T hx, T hy, T hz, T lx_, T ly_, T lz_, uint32_t cell,
                    bool live, uint32_t i) -> bool {
        hx *= J;
        hy *= J;
        hz *= J;
        bool a = false;
        if (MODE != 1 && live) {
            const uint32_t s = cell * NB + B;
            T dH;
            a = metropolis<T>(sx, sy, sz, hx, hy, hz, s, rid, t, P.seed_lo, P.seed_hi, K, ex, ey,
                              ez, beta, greedy, dH);
            if (MODE == 2) {
                ((T *)P.dbg_dh)[i] = dH;
                P.dbg_acc[i] = a ? 1 : 0;
            }
        }
        if (MEASURE && live) {
            observe<T>(acc, sx, sy, sz, ex, ey, ez, true, lx_, ly_, lz_, Jd);
            acc[Q_NACC] += a ? 1.0 : 0.0;
        }
        return a;
    };

    for (int z = z0; z < z1; ++z) {
        // roll the planes and load the new one
#pragma unroll
        for (int b2 = 0; b2 < NB; ++b2) {
            if (b2 == B) continue;
            const int dx = basis2(KIND, b2, 0) - bx, dy = basis2(KIND, b2, 1) - by;
            const int dz = basis2(KIND, b2, 2) - bz;
            if (dz > 0) { // slot 0 = z, slot 1 = z - 1
#pragma unroll
                for (int j = 0; j < RY + 1; ++j) {
                    V[b2][1][j] = V[b2][0][j];
                    E[b2][1][j] = E[b2][0][j];
                }
                load_plane(b2, dx, dy, z, true, V[b2][0], E[b2][0]);
            } else if (dz < 0) { // slot 0 = z, slot 1 = z + 1
#pragma unroll
                for (int j = 0; j < RY + 1; ++j) {
                    V[b2][0][j] = V[b2][1][j];
                    E[b2][0][j] = E[b2][1][j];
                }
                const int cz = z < Lz - 1 ? z + 1 : (pz ? 0 : -1);
                load_plane(b2, dx, dy, cz, cz >= 0, V[b2][1], E[b2][1]);
            } else {
                load_plane(b2, dx, dy, z, true, V[b2][0], E[b2][0]);
            }
        }
        const uint32_t s_own = (uint32_t)B * basis_b + (uint32_t)z * zplane_b;
#pragma unroll
        for (int k = 0; k < RY; ++k) {
            const int y = yb + k;
            Row2<T> me;
            buf_load2(q.x, roff[k + 1], s_own, me.xa, me.xb);
            buf_load2(q.y, roff[k + 1], s_own, me.ya, me.yb);
            buf_load2(q.z, roff[k + 1], s_own, me.za, me.zb);
            T hxa = 0, hya = 0, hza = 0, hxb = 0, hyb = 0, hzb = 0;
            T lxa = 0, lya = 0, lza = 0, lxb = 0, lyb = 0, lzb = 0;
#pragma unroll
            for (int b2 = 0; b2 < NB; ++b2) {
                if (b2 == B) continue;
                const int dx = basis2(KIND, b2, 0) - bx, dy = basis2(KIND, b2, 1) - by;
                const int dz = basis2(KIND, b2, 2) - bz;
                const int j0 = dy > 0 ? 1 : 0;
                T aax = 0, aay = 0, aaz = 0, abx = 0, aby = 0, abz = 0;
#pragma unroll
                for (int iz = 0; iz < (dz ? 2 : 1); ++iz) {
#pragma unroll
                    for (int iy = 0; iy < (dy ? 2 : 1); ++iy) {
                        const int j = k - iy * dy + j0;
                        const Row2<T> v = V[b2][iz][j];
                        // column x of each cell
                        aax += v.xa;
                        aay += v.ya;
                        aaz += v.za;
                        abx += v.xb;
                        aby += v.yb;
                        abz += v.zb;
                        if (dx > 0) { // column x - 1: a <- lane-1's b (or memory), b <- a
                            Vec3<T> n = {from_lower_lane(v.xb), from_lower_lane(v.yb),
                                         from_lower_lane(v.zb)};
                            if (left_mem) n = E[b2][iz][j];
                            aax += n.x;
                            aay += n.y;
                            aaz += n.z;
                            abx += v.xa;
                            aby += v.ya;
                            abz += v.za;
                        } else if (dx < 0) { // column x + 1: a <- b, b <- lane+1's a (or memory)
                            Vec3<T> n = {from_upper_lane(v.xa), from_upper_lane(v.ya),
                                         from_upper_lane(v.za)};
                            if (right_mem) n = E[b2][iz][j];
                            aax += v.xb;
                            aay += v.yb;
                            aaz += v.zb;
                            abx += n.x;
                            aby += n.y;
                            abz += n.z;
                        }
                    }
                }
                hxa += aax;
                hya += aay;
                hza += aaz;
                hxb += abx;
                hyb += aby;
                hzb += abz;
                if (b2 < B) {
                    lxa += aax;
                    lya += aay;
                    lza += aaz;
                    lxb += abx;
                    lyb += aby;
                    lzb += abz;
                }
            }
            const bool row_live = fin && y < Ly;
            const bool live_a = row_live && occ(xa, y, z), live_b = row_live && occ(xb, y, z);
            const uint32_t cell = (uint32_t)(z * Ly + y) * (uint32_t)Lx + (uint32_t)xa;
            const uint32_t i0 = (uint32_t)B * plane + cell;
            const bool aa = site(me.xa, me.ya, me.za, hxa, hya, hza, lxa, lya, lza, cell, live_a, i0);
            const bool ab = site(me.xb, me.yb, me.zb, hxb, hyb, hzb, lxb, lyb, lzb, cell + 1u,
                                 live_b, i0 + 1u);
            // every pair of an existing row is written back, accepted or not
            // (same bits where rejected or unoccupied; no other workgroup owns
            // it): whole lines reach the L2, measured 2 % faster on bcc
            (void)aa;
            (void)ab;
            if (MODE != 1 && row_live) {
                buf_store2(me.xa, me.xb, q.x, roff[k + 1], s_own);
                buf_store2(me.ya, me.yb, q.y, roff[k + 1], s_own);
                buf_store2(me.za, me.zb, q.z, roff[k + 1], s_own);
            }
        }
    }
    if (MEASURE)
        block_store_partials(acc, P.partials_dev + ((size_t)B * P.n_items + item) * NQ);
}

} // namespace mc
