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
            if (MEASURE)
                accumulate<T>(acc, sx, sy, sz, ex, ey, ez, J * (sx * lx_ + sy * ly_ + sz * lz_),
                              a);
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
        if (MEASURE)
            accumulate<T>(acc, sx, sy, sz, ex, ey, ez, J * (sx * lx_ + sy * ly_ + sz * lz_), a);
    }
    if (MEASURE)
        block_store_partials(acc, P.partials_dev + ((size_t)B * P.n_items + item) * NQ);
}

} // namespace mc
