// kernels.hip -- CDNA4 (gfx950) kernels of the colour-sweep Metropolis method
// for the anisotropic classical Heisenberg model, Eq. (1) of arXiv:2106.11286:
//     H = -J sum_<ij> S_i.S_j - K sum_i (S_i.e)^2.
//
// One launch = one colour pass: every occupied site of one sublattice colour
// gets one Metropolis attempt (propose uniformly on the sphere; accept if
// dH <= 0 or P <= exp(-beta dH), the rule of the paper's Monte Carlo
// paragraph).  No bond joins two sites of one colour, so all sites of a pass
// are independent and the result does not depend on tiling or thread order.
//
// Memory: spins are structure-of-arrays planes (x, y, z components) in the
// working precision, colour-major, so a pass reads its own colour and the
// other colour(s) as dense, coalesced rows.  Random numbers are computed in
// registers from a counter-based generator (no state in memory).  Observables
// (magnetisation, Eq. (2), and both energy terms) are reduced in FP64 inside
// the pass from values that are final after it, so measuring adds no spin
// traffic.
#include <hip/hip_runtime.h>

#include "launch.hpp"
#include "mc_internal.hpp"

namespace mc {

// Spin planes are plain device allocations: address them as global memory so
// loads take a scalar base plus a 32-bit vector offset.
template <typename T> using gptr = __attribute__((address_space(1))) T *;
template <typename T> __device__ __forceinline__ gptr<T> as_global(void *p)
{
    return (gptr<T>)(p);
}

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds, each with two
// 32x32 -> 64-bit products (one v_mad_u64_u32 each); the high halves are mixed
// with the other counter words and the key, which is bumped by the Weyl
// increments between rounds.
// ---------------------------------------------------------------------------
struct Words {
    uint32_t w0, w1, w2, w3;
};

__device__ __forceinline__ Words philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                          uint32_t k0, uint32_t k1)
{
    constexpr uint32_t kMulA = 0xD2511F53u, kMulB = 0xCD9E8D57u;
    constexpr uint32_t kWeylA = 0x9E3779B9u, kWeylB = 0xBB67AE85u;
    // The key is uniform: keep its schedule in scalar registers computed per
    // call, instead of 20 hoisted loop invariants that would crowd out the
    // sweep kernels' other scalar state.
    asm volatile("" : "+s"(k0), "+s"(k1));
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t pa = (uint64_t)kMulA * c0;
        const uint64_t pb = (uint64_t)kMulB * c2;
        const uint32_t n0 = (uint32_t)(pb >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(pa >> 32) ^ c3 ^ k1;
        c0 = n0;
        c1 = (uint32_t)pb;
        c2 = n2;
        c3 = (uint32_t)pa;
        k0 += kWeylA;
        k1 += kWeylB;
    }
    return {c0, c1, c2, c3};
}

// u = (k + 1/2) 2^-23 from the top 23 bits: exact in binary32 and binary64.
template <typename T> __device__ __forceinline__ T uniform23(uint32_t w);
template <> __device__ __forceinline__ float uniform23<float>(uint32_t w)
{
    return __uint2float_rn(w >> 9) * 0x1p-23f + 0x1p-24f;
}
template <> __device__ __forceinline__ double uniform23<double>(uint32_t w)
{
    return __uint2double_rn(w >> 9) * 0x1p-23 + 0x1p-24;
}

// Uniform point on the unit sphere: z uniform on [-1,1], azimuth 2 pi u1.
// FP32 uses the hardware sine/cosine, which take their argument in
// revolutions (no range reduction), and the hardware square root.
__device__ __forceinline__ void sphere_point(float u0, float u1, float &x, float &y, float &z)
{
    z = 2.0f * u0 - 1.0f;
    const float r = __builtin_amdgcn_sqrtf(1.0f - z * z);
    x = r * __builtin_amdgcn_cosf(u1);
    y = r * __builtin_amdgcn_sinf(u1);
}
__device__ __forceinline__ void sphere_point(double u0, double u1, double &x, double &y, double &z)
{
    z = 2.0 * u0 - 1.0;
    const double r = sqrt(1.0 - z * z);
    double s, c;
    sincospi(2.0 * u1, &s, &c);
    x = r * c;
    y = r * s;
}

__device__ __forceinline__ float fast_exp(float v) { return __expf(v); }
__device__ __forceinline__ double fast_exp(double v) { return exp(v); }
__device__ __forceinline__ float inv_norm(float v) { return __builtin_amdgcn_rsqf(v); }
__device__ __forceinline__ double inv_norm(double v) { return 1.0 / sqrt(v); }

// Lane shifts inside a wave64 (DPP): value of lane i-1 / lane i+1.  Lanes
// without a source keep their own value.
__device__ __forceinline__ float from_lower_lane(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(v), __float_as_int(v),
                                                      0x138, 0xf, 0xf, false));
}
__device__ __forceinline__ float from_upper_lane(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(v), __float_as_int(v),
                                                      0x130, 0xf, 0xf, false));
}
__device__ __forceinline__ double from_lower_lane(double v)
{
    const int lo = __double2loint(v), hi = __double2hiint(v);
    return __hiloint2double(__builtin_amdgcn_update_dpp(hi, hi, 0x138, 0xf, 0xf, false),
                            __builtin_amdgcn_update_dpp(lo, lo, 0x138, 0xf, 0xf, false));
}
__device__ __forceinline__ double from_upper_lane(double v)
{
    const int lo = __double2loint(v), hi = __double2hiint(v);
    return __hiloint2double(__builtin_amdgcn_update_dpp(hi, hi, 0x130, 0xf, 0xf, false),
                            __builtin_amdgcn_update_dpp(lo, lo, 0x130, 0xf, 0xf, false));
}

// Basis positions of the conventional cubic cell, in half-cell units.
__host__ __device__ constexpr int basis_count(int kind) { return kind == SC ? 1 : (kind == BCC ? 2 : 4); }
__host__ __device__ constexpr int basis2(int kind, int b, int axis)
{
    // fcc: (0,0,0) (1,1,0) (1,0,1) (0,1,1); bcc: (0,0,0) (1,1,1)
    return kind == FCC ? ((b == 0) ? 0 : (b == 1 ? (axis != 2) : (b == 2 ? (axis != 1) : (axis != 0))))
                       : (kind == BCC ? (b == 1 ? 1 : 0) : 0);
}

// Exact sphere occupancy (half-cell units are integers).
__device__ __forceinline__ bool occupied(const RepDev &R, int x, int y, int z, int bx, int by,
                                         int bz)
{
    if (!R.sphere) return true;
    const int qx = 2 * x + bx - R.Lx, qy = 2 * y + by - R.Ly, qz = 2 * z + bz - R.Lz;
    return (double)(qx * qx + qy * qy + qz * qz) <= R.r2x4;
}

// Logical work item of this workgroup.  Workgroups are dealt to the XCDs in
// turn, so consecutive dispatch indices land on different L2 caches; the
// mapping below gives each XCD a contiguous run of the work list, whose
// neighbouring tiles share halo rows.  Returns false for padding workgroups.
__device__ __forceinline__ bool logical_item(const PassLaunch &P, uint32_t &item)
{
    const uint32_t q = (P.n_blocks + 7u) >> 3;
    const uint32_t b = blockIdx.x;
    const uint32_t l = (b & 7u) * q + (b >> 3);
    item = P.item_base + l;
    return l < P.n_blocks;
}

// ---------------------------------------------------------------------------
// Block reduction of Q_N doubles (fixed order: wave butterflies, then waves in
// index order), written to one partial slot.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void block_store_partials(double (&a)[Q_N], double *dst)
{
    __shared__ double red[4][Q_N];
#pragma unroll
    for (int q = 0; q < Q_N; ++q) {
        double v = a[q];
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
        a[q] = v;
    }
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int n_waves = (blockDim.x + 63) >> 6;
    if (lane == 0) {
#pragma unroll
        for (int q = 0; q < Q_N; ++q) red[wave][q] = a[q];
    }
    __syncthreads();
    if (threadIdx.x < Q_N) {
        double s = 0.0;
        for (int w = 0; w < n_waves; ++w) s += red[w][threadIdx.x];
        dst[threadIdx.x] = s;
    }
    if (threadIdx.x >= Q_N && threadIdx.x < NQ) dst[threadIdx.x] = 0.0;
}

// One Metropolis attempt at a site with local field h (J already applied).
// Returns the final spin in (sx, sy, sz).  Canonical site s keys the stream.
template <typename T>
__device__ __forceinline__ bool metropolis(T &sx, T &sy, T &sz, T hx, T hy, T hz, uint32_t s,
                                           uint32_t rid, uint32_t t, uint32_t k0, uint32_t k1,
                                           T K, T ex, T ey, T ez, T beta, bool greedy, T &dH)
{
    const Words w = philox10(s, rid, t, 0u, k0, k1);
    T nx, ny, nz;
    sphere_point(uniform23<T>(w.w0), uniform23<T>(w.w1), nx, ny, nz);
    const T P = uniform23<T>(w.w2);
    const T dx = nx - sx, dy = ny - sy, dz = nz - sz;
    const T pn = nx * ex + ny * ey + nz * ez;
    const T po = sx * ex + sy * ey + sz * ez;
    // Eq. (1): dH = -h.(S'-S) - K[(S'.e)^2 - (S.e)^2]
    dH = -(hx * dx + hy * dy + hz * dz) - K * ((pn - po) * (pn + po));
    const bool acc = (dH <= T(0)) || (!greedy && P <= fast_exp(-beta * dH));
    if (acc) {
        const T inv = inv_norm(nx * nx + ny * ny + nz * nz);
        sx = nx * inv;
        sy = ny * inv;
        sz = nz * inv;
    }
    return acc;
}

// FP64 accumulation of the observables of one final spin.  sh is the spin
// dotted with the field of its already-final neighbours (J applied); pass 0
// of a bipartite lattice contributes none.
template <typename T>
__device__ __forceinline__ void accumulate(double (&acc)[Q_N], T sx, T sy, T sz, T ex, T ey, T ez,
                                           T sh, bool accepted)
{
    acc[Q_MX] += (double)sx;
    acc[Q_MY] += (double)sy;
    acc[Q_MZ] += (double)sz;
    const double pe = (double)sx * (double)ex + (double)sy * (double)ey + (double)sz * (double)ez;
    acc[Q_PE2] += pe * pe;
    acc[Q_SH] += (double)sh;
    acc[Q_NACC] += accepted ? 1.0 : 0.0;
}

// ---------------------------------------------------------------------------
// Simple cubic, two colours, colour-packed rows.  A site (x, y, z) of colour
// c = (x+y+z)&1 sits at packed column xh = x/2 of row (y, z) in plane c.  Its
// six neighbours all have the other colour: the same column of rows y+-1 and
// planes z+-1, and in its own row the columns xh and xh-1 (x even) or xh and
// xh+1 (x odd).
//
// Tile kernel: each thread owns one (xh, y) column of a tx x ty tile and walks
// the tile's z range; neighbours are loaded directly (cache hits).  Used for
// short rows.
// ---------------------------------------------------------------------------
// Field of the six neighbours of a simple-cubic site (J not applied), summed
// in the fixed order -z, -y, -x, +x, +y, +z over the other colour's plane at
// element offset oth.  P is a global or an LDS pointer; missing neighbours
// across open faces contribute nothing.
template <typename T, typename P>
__device__ __forceinline__ void sc_site_field(P gx, P gy, P gz, uint32_t oth, int Lxh, int Ly,
                                              int Lz, bool px, bool py, bool pz, int xh, int y,
                                              int z, int p, T &hx, T &hy, T &hz)
{
    const int ym = y > 0 ? y - 1 : (py ? Ly - 1 : -1);
    const int yp = y < Ly - 1 ? y + 1 : (py ? 0 : -1);
    const int xm = xh > 0 ? xh - 1 : (px ? Lxh - 1 : -1);
    const int xp = xh < Lxh - 1 ? xh + 1 : (px ? 0 : -1);
    const int zm = z > 0 ? z - 1 : (pz ? Lz - 1 : -1);
    const int zp = z < Lz - 1 ? z + 1 : (pz ? 0 : -1);
    hx = 0;
    hy = 0;
    hz = 0;
    auto add = [&](int valid, uint32_t j) {
        if (valid) {
            hx += gx[oth + j];
            hy += gy[oth + j];
            hz += gz[oth + j];
        }
    };
    add(zm >= 0, (uint32_t)(zm * Ly + y) * Lxh + xh);
    add(ym >= 0, (uint32_t)(z * Ly + ym) * Lxh + xh);
    const int xl = p ? xh : xm; // x-1
    const int xr = p ? xp : xh; // x+1
    const uint32_t row = (uint32_t)(z * Ly + y) * Lxh;
    add(xl >= 0, row + xl);
    add(xr >= 0, row + xr);
    add(yp >= 0, (uint32_t)(z * Ly + yp) * Lxh + xh);
    add(zp >= 0, (uint32_t)(zp * Ly + y) * Lxh + xh);
}

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
            if (MEASURE)
                accumulate<T>(acc, sx, sy, sz, ex, ey, ez,
                              colour == 1 ? sx * hx + sy * hy + sz * hz : T(0), a);
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
template <typename T> struct Vec3 {
    T x, y, z;
};

// Raw buffer access: a resource per spin component holds the array's base and
// size in scalar registers; an access is one instruction with the lane's byte
// offset in a vector register and the row's byte offset in a scalar register
// (no per-lane 64-bit address arithmetic).  A component array must stay below
// 4 GiB (checked on the host).
using rsrc_t = __amdgpu_buffer_rsrc_t;
constexpr int kRsrcWord3 = 0x00020000; // raw dword access, gfx9-family descriptor

template <typename T>
__device__ __forceinline__ rsrc_t plane_rsrc(void *comp, uint32_t elem_off, uint32_t n_elems)
{
    return __builtin_amdgcn_make_buffer_rsrc((char *)comp + (size_t)elem_off * sizeof(T), (short)0,
                                             (int)(n_elems * (uint32_t)sizeof(T)), kRsrcWord3);
}
__device__ __forceinline__ float buf_load(rsrc_t r, uint32_t voff, uint32_t soff, float)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
__device__ __forceinline__ double buf_load(rsrc_t r, uint32_t voff, uint32_t soff, double)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
__device__ __forceinline__ void buf_store(float v, rsrc_t r, uint32_t voff, uint32_t soff)
{
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, voff, soff, 0);
}
__device__ __forceinline__ void buf_store(double v, rsrc_t r, uint32_t voff, uint32_t soff)
{
    typedef uint32_t v2u __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(v2u, v), r, voff, soff, 0);
}
template <typename T> struct PlaneRs {
    rsrc_t x, y, z;
};

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
                acc[Q_MX] += (double)sx;
                acc[Q_MY] += (double)sy;
                acc[Q_MZ] += (double)sz;
                const double pe = (double)(sx * ex + sy * ey + sz * ez);
                acc[Q_PE2] += pe * pe;
                if (colour == 1) acc[Q_SH] += (double)(sx * hx + sy * hy + sz * hz);
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
template <typename T> struct Row2 {
    T xa, ya, za, xb, yb, zb; // components of the pair's columns a = 2l, b = 2l+1
};
__device__ __forceinline__ void buf_load2(rsrc_t r, uint32_t voff, uint32_t soff, float &a, float &b)
{
    typedef uint32_t v2u __attribute__((ext_vector_type(2)));
    const v2u v = __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0);
    // elements go through scalars first: a bit cast applied directly to a
    // vector element reads the vector's first element
    const uint32_t lo = v.x, hi = v.y;
    a = __uint_as_float(lo);
    b = __uint_as_float(hi);
}
__device__ __forceinline__ void buf_load2(rsrc_t r, uint32_t voff, uint32_t soff, double &a,
                                          double &b)
{
    typedef uint32_t v4u __attribute__((ext_vector_type(4)));
    const v4u v = __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0);
    a = __hiloint2double((int)v.y, (int)v.x);
    b = __hiloint2double((int)v.w, (int)v.z);
}
__device__ __forceinline__ void buf_store2(float a, float b, rsrc_t r, uint32_t voff, uint32_t soff)
{
    typedef uint32_t v2u __attribute__((ext_vector_type(2)));
    v2u v;
    v.x = __builtin_bit_cast(uint32_t, a);
    v.y = __builtin_bit_cast(uint32_t, b);
    __builtin_amdgcn_raw_buffer_store_b64(v, r, voff, soff, 0);
}
__device__ __forceinline__ void buf_store2(double a, double b, rsrc_t r, uint32_t voff,
                                           uint32_t soff)
{
    typedef uint32_t v4u __attribute__((ext_vector_type(4)));
    v4u v;
    v.x = (uint32_t)__double2loint(a);
    v.y = (uint32_t)__double2hiint(a);
    v.z = (uint32_t)__double2loint(b);
    v.w = (uint32_t)__double2hiint(b);
    __builtin_amdgcn_raw_buffer_store_b128(v, r, voff, soff, 0);
}

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
            acc[Q_MX] += (double)sx;
            acc[Q_MY] += (double)sy;
            acc[Q_MZ] += (double)sz;
            const double pe = (double)(sx * ex + sy * ey + sz * ez);
            acc[Q_PE2] += pe * pe;
            if (colour == 1) acc[Q_SH] += (double)(sx * hx + sy * hy + sz * hz);
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
            // a pair with one accepted move rewrites the other column's
            // unchanged value (same bits; no other workgroup owns it)
            if (MODE != 1 && live && (aa || ab)) {
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
// ---------------------------------------------------------------------------
template <typename T, bool MEASURE, int MODE, int RY>
__device__ __forceinline__ void sc_pband_body(const PassLaunch &P, int colour, uint32_t item,
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
    const bool px = R.pmask & 1u, py = R.pmask & 2u, pz = R.pmask & 4u;
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
    auto load_rows = [&](int z, Row2<T> *dst) {
        if (z < 0) {
#pragma unroll
            for (int k = 0; k < RY + 2; ++k) dst[k] = Row2<T>{T(0), T(0), T(0), T(0), T(0), T(0)};
            return;
        }
        const uint32_t soff = oth_b + (uint32_t)z * zplane_b;
#pragma unroll
        for (int k = 0; k < RY + 2; ++k) {
            buf_load2(q.x, roff[k], soff, dst[k].xa, dst[k].xb);
            buf_load2(q.y, roff[k], soff, dst[k].ya, dst[k].yb);
            buf_load2(q.z, roff[k], soff, dst[k].za, dst[k].zb);
            if (!py && !((row_ok >> k) & 1u)) dst[k] = Row2<T>{T(0), T(0), T(0), T(0), T(0), T(0)};
        }
    };
    // the in-row neighbour beyond the pair where the lane shift cannot supply
    // it (wave edges, band seams, the periodic wrap, open faces), loaded one
    // plane ahead
    auto load_edges = [&](int z, Vec3<T> *dst) {
        const uint32_t soff = oth_b + (uint32_t)z * zplane_b;
#pragma unroll
        for (int k = 0; k < RY; ++k) {
            const int p = (colour + k + z) & 1;
            const bool need = p ? right_mem : left_mem;
            const int col = p ? xr : xl;
            if (need && col >= 0) {
                const uint32_t v = roff[k + 1] - b_c + (p ? b_r : b_l);
                dst[k] = {buf_load(q.x, v, soff, T()), buf_load(q.y, v, soff, T()),
                          buf_load(q.z, v, soff, T())};
            } else {
                dst[k] = {T(0), T(0), T(0)};
            }
        }
    };

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
            acc[Q_MX] += (double)sx;
            acc[Q_MY] += (double)sy;
            acc[Q_MZ] += (double)sz;
            const double pe = (double)(sx * ex + sy * ey + sz * ez);
            acc[Q_PE2] += pe * pe;
            if (colour == 1) acc[Q_SH] += (double)(sx * hx + sy * hy + sz * hz);
            n_acc += a ? 1u : 0u;
        }
        return a;
    };

    const int z0 = w.z0, z1 = min(w.z0 + P.tile.zc, Lz);
    Row2<T> om[RY + 2], oc[RY + 2], op[RY + 2];
    Vec3<T> ec[RY], en[RY];
    load_rows(z0 > 0 ? z0 - 1 : (pz ? Lz - 1 : -1), om);
    load_rows(z0, oc);
    load_edges(z0, ec);
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
            Row2<T> me;
            buf_load2(q.x, roff[k + 1], s_own, me.xa, me.xb);
            buf_load2(q.y, roff[k + 1], s_own, me.ya, me.yb);
            buf_load2(q.z, roff[k + 1], s_own, me.za, me.zb);
            const Row2<T> c = oc[k + 1];
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
            const T hxa = om[k + 1].xa + oc[k].xa + lax + hax + oc[k + 2].xa + op[k + 1].xa;
            const T hya = om[k + 1].ya + oc[k].ya + lay + hay + oc[k + 2].ya + op[k + 1].ya;
            const T hza = om[k + 1].za + oc[k].za + laz + haz + oc[k + 2].za + op[k + 1].za;
            const T hxb = om[k + 1].xb + oc[k].xb + lbx + hbx + oc[k + 2].xb + op[k + 1].xb;
            const T hyb = om[k + 1].yb + oc[k].yb + lby + hby + oc[k + 2].yb + op[k + 1].yb;
            const T hzb = om[k + 1].zb + oc[k].zb + lbz + hbz + oc[k + 2].zb + op[k + 1].zb;
            const uint32_t s0 = (uint32_t)(z * Ly + y) * (uint32_t)Lx + 2u * xa + p;
            const uint32_t i0 = own + (uint32_t)(z * Ly + y) * Lxh + xa;
            const bool aa = site(me.xa, me.ya, me.za, hxa, hya, hza, s0, live, i0);
            const bool ab = site(me.xb, me.yb, me.zb, hxb, hyb, hzb, s0 + 2u, live, i0 + 1u);
            if (MODE != 1 && live && (aa || ab)) {
                buf_store2(me.xa, me.xb, q.x, roff[k + 1], s_own);
                buf_store2(me.ya, me.yb, q.y, roff[k + 1], s_own);
                buf_store2(me.za, me.zb, q.z, roff[k + 1], s_own);
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
                acc[Q_MX] += (double)sx;
                acc[Q_MY] += (double)sy;
                acc[Q_MZ] += (double)sz;
                const double pe = (double)(sx * ex + sy * ey + sz * ez);
                acc[Q_PE2] += pe * pe;
                if (colour == 1) acc[Q_SH] += (double)(sx * hx + sy * hy + sz * hz);
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

// ---------------------------------------------------------------------------
// bcc / fcc: colour = basis site B, one dense plane per basis site.  The
// neighbours of a B site in basis b2 sit at cell offsets o with o_a = 0 on
// axes where the two basis vectors agree and o_a in {0, -sign(d_a)} where
// they differ (d = basis(b2) - basis(B), half-cell units): 4 cells per other
// basis for fcc, 8 for bcc.  Unoccupied sites hold zero, so the field sum is
// branch-free inside the box.
// ---------------------------------------------------------------------------
// Field at basis site B of cell (x, y, z) (J not applied): hx.. over all
// neighbours, lx_.. over the neighbours of lower colour (basis index < B).
// Other basis sites b2 ascending; per b2 the 2 to 8 candidate cells in the
// fixed (iz, iy, ix) order, summed first, then added.  P is a global or an
// LDS pointer; plane = cells per basis plane.
template <int KIND, int B, typename T, typename P>
__device__ __forceinline__ void basis_site_field(P gx, P gy, P gz, uint32_t plane, int Lx, int Ly,
                                                 int Lz, bool pxm, bool pym, bool pzm, int x,
                                                 int y, int z, T &hx, T &hy, T &hz, T &lx_,
                                                 T &ly_, T &lz_)
{
    constexpr int NB = basis_count(KIND);
    constexpr int bx = basis2(KIND, B, 0), by = basis2(KIND, B, 1), bz = basis2(KIND, B, 2);
    hx = 0;
    hy = 0;
    hz = 0;
    lx_ = 0;
    ly_ = 0;
    lz_ = 0;
#pragma unroll
    for (int b2 = 0; b2 < NB; ++b2) {
        if (b2 == B) continue;
        const int dx = basis2(KIND, b2, 0) - bx;
        const int dy = basis2(KIND, b2, 1) - by;
        const int dz = basis2(KIND, b2, 2) - bz;
        const int nox = dx ? 2 : 1, noy = dy ? 2 : 1, noz = dz ? 2 : 1;
        T ax = 0, ay = 0, az = 0;
#pragma unroll
        for (int iz = 0; iz < noz; ++iz)
#pragma unroll
            for (int iy = 0; iy < noy; ++iy)
#pragma unroll
                for (int ix = 0; ix < nox; ++ix) {
                    int cx = x - ix * dx, cy = y - iy * dy, cz = z - iz * dz;
                    bool ok = true;
                    if (cx < 0) { cx += Lx; ok &= pxm; }
                    if (cx >= Lx) { cx -= Lx; ok &= pxm; }
                    if (cy < 0) { cy += Ly; ok &= pym; }
                    if (cy >= Ly) { cy -= Ly; ok &= pym; }
                    if (cz < 0) { cz += Lz; ok &= pzm; }
                    if (cz >= Lz) { cz -= Lz; ok &= pzm; }
                    if (ok) {
                        const uint32_t j = (uint32_t)b2 * plane + (uint32_t)(cz * Ly + cy) * Lx + cx;
                        ax += gx[j];
                        ay += gy[j];
                        az += gz[j];
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
}

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

// ---------------------------------------------------------------------------
// Pass kernels: one workgroup per work item, sweep counter from the device.
// ---------------------------------------------------------------------------
template <typename T, bool MEASURE, int MODE>
__global__ void __launch_bounds__(256) k_sc_tile(PassLaunch P, int colour)
{
    uint32_t item;
    if (!logical_item(P, item)) return;
    sc_tile_body<T, MEASURE, MODE>(P, colour, item, *P.tctr_dev + P.t_off);
}

template <typename T, bool MEASURE, int MODE, int RY>
__global__ void __launch_bounds__(256) k_sc_strip(PassLaunch P, int colour)
{
    uint32_t item;
    if (!logical_item(P, item)) return;
    sc_strip_body<T, MEASURE, MODE, RY>(P, colour, item, *P.tctr_dev + P.t_off);
}

template <typename T, bool MEASURE, int MODE, int RY>
__global__ void __launch_bounds__(256) k_sc_band(PassLaunch P, int colour)
{
    uint32_t item;
    if (!logical_item(P, item)) return;
    sc_band_body<T, MEASURE, MODE, RY>(P, colour, item, *P.tctr_dev + P.t_off);
}

template <typename T, bool MEASURE, int MODE, int RY>
__global__ void __launch_bounds__(256) k_sc_pair(PassLaunch P, int colour)
{
    uint32_t item;
    if (!logical_item(P, item)) return;
    sc_pair_body<T, MEASURE, MODE, RY>(P, colour, item, *P.tctr_dev + P.t_off);
}

template <typename T, bool MEASURE, int MODE, int RY>
__global__ void __launch_bounds__(256) k_sc_pband(PassLaunch P, int colour)
{
    uint32_t item;
    if (!logical_item(P, item)) return;
    sc_pband_body<T, MEASURE, MODE, RY>(P, colour, item, *P.tctr_dev + P.t_off);
}

template <int KIND, int B, typename T, bool MEASURE, int MODE>
__global__ void __launch_bounds__(256) k_basis_strip(PassLaunch P)
{
    uint32_t item;
    if (!logical_item(P, item)) return;
    basis_strip_body<KIND, B, T, MEASURE, MODE>(P, item, *P.tctr_dev + P.t_off);
}

template <int KIND, int B, typename T, bool MEASURE, int MODE>
__global__ void __launch_bounds__(256) k_basis_pass(PassLaunch P)
{
    uint32_t item;
    if (!logical_item(P, item)) return;
    basis_body<KIND, B, T, MEASURE, MODE>(P, item, *P.tctr_dev + P.t_off);
}

// ---------------------------------------------------------------------------
// Persistent batched sweeps (see PersistLaunch).  Memory ordering: a unit's
// stores are released (agent scope) before its completion is counted; the
// workgroup that completes a replica's pass acquires, reduces the pass's
// partial sums if the sweep is measured, then releases the next phase; a
// waiting unit acquires before reading spins.
// ---------------------------------------------------------------------------
template <typename T, bool MEASURE, int KIND, int KERNEL, int RY>
__device__ __forceinline__ void unit_body(const PassLaunch &P, int c, uint32_t item, uint32_t t)
{
    if constexpr (KIND == SC) {
        if constexpr (KERNEL == KERNEL_STRIP) sc_strip_body<T, MEASURE, 0, RY>(P, c, item, t);
        else if constexpr (KERNEL == KERNEL_BAND) sc_band_body<T, MEASURE, 0, RY>(P, c, item, t);
        else if constexpr (KERNEL == KERNEL_PAIR) sc_pair_body<T, MEASURE, 0, RY>(P, c, item, t);
        else if constexpr (KERNEL == KERNEL_PBAND) sc_pband_body<T, MEASURE, 0, RY>(P, c, item, t);
        else sc_tile_body<T, MEASURE, 0>(P, c, item, t);
    } else {
        switch (c) {
        case 0: basis_body<KIND, 0, T, MEASURE, 0>(P, item, t); break;
        case 1: basis_body<KIND, 1, T, MEASURE, 0>(P, item, t); break;
        case 2:
            if constexpr (KIND == FCC) basis_body<KIND, 2, T, MEASURE, 0>(P, item, t);
            break;
        default:
            if constexpr (KIND == FCC) basis_body<KIND, 3, T, MEASURE, 0>(P, item, t);
            break;
        }
    }
}

template <typename T, bool MEASURE, int KIND, int KERNEL, int RY>
__global__ void __launch_bounds__(256) k_persistent(PassLaunch P, PersistLaunch A)
{
    __shared__ uint32_t s_unit, s_flag;
    __shared__ double s_rec[NQ];
    uint32_t *const hdr = A.state, *const done = A.state + 4, *const ready = A.state + 4 + A.n_reps;
    const uint32_t n_items = P.n_items;
    const uint32_t per_sweep = A.n_colours * n_items;
    const uint32_t total = A.n_sweeps * per_sweep;
    const uint32_t t0 = *P.tctr_dev + P.t_off;
    for (;;) {
        if (threadIdx.x == 0) {
            uint32_t u = __hip_atomic_fetch_add(&hdr[0], 1u, __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_AGENT);
            if (__hip_atomic_load(&hdr[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) u = total;
            s_unit = u;
        }
        __syncthreads();
        const uint32_t u = s_unit;
        if (u >= total) break;
        const uint32_t sw = u / per_sweep, rem = u - sw * per_sweep;
        const uint32_t c = rem / n_items, item = rem - c * n_items;
        const uint32_t r = P.work_dev[item].rep;
        const uint32_t phase = sw * A.n_colours + c;
        if (threadIdx.x == 0) {
            // poll with plain (relaxed) loads; the acquire fence below, once
            // the phase is released, orders the unit's reads after it
            uint32_t ok = 1;
            for (uint32_t spins = 0;
                 __hip_atomic_load(&ready[r], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < phase;
                 ++spins) {
                if (spins >= A.spin_limit ||
                    __hip_atomic_load(&hdr[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                    ok = 0;
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
            }
            if (!ok) {
                __hip_atomic_store(&hdr[2], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&hdr[1], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            s_flag = ok;
        }
        __syncthreads();
        if (!s_flag) break;
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        unit_body<T, MEASURE, KIND, KERNEL, RY>(P, (int)c, item, t0 + sw);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __syncthreads();
        if (threadIdx.x == 0) {
            const RepDev &R = P.reps_dev[r];
            const uint32_t n_r = R.item_end - R.item_begin;
            // every wave released its stores above; the count itself needs
            // no ordering of its own
            const uint32_t old = __hip_atomic_fetch_add(&done[r], 1u, __ATOMIC_RELAXED,
                                                        __HIP_MEMORY_SCOPE_AGENT);
            s_flag = (old + 1u == (phase + 1u) * n_r);
        }
        __syncthreads();
        if (s_flag) { // this unit completed replica r's phase
            if (MEASURE && c == A.n_colours - 1) {
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                const RepDev &R = P.reps_dev[r];
                double a[Q_N] = {0, 0, 0, 0, 0, 0};
                for (uint32_t cc = 0; cc < A.n_colours; ++cc)
                    for (uint32_t it = R.item_begin + threadIdx.x; it < R.item_end; it += blockDim.x) {
                        const double *p = P.partials_dev + ((size_t)cc * n_items + it) * NQ;
#pragma unroll
                        for (int q = 0; q < Q_N; ++q) a[q] += p[q];
                    }
                block_store_partials(a, s_rec);
                __syncthreads();
                if (threadIdx.x == 0) {
                    double *rec = A.records + ((size_t)((A.slot0 + sw) % A.ring) * A.n_reps + r) * NR;
                    rec[R_MX] = s_rec[Q_MX];
                    rec[R_MY] = s_rec[Q_MY];
                    rec[R_MZ] = s_rec[Q_MZ];
                    rec[R_EEX] = -s_rec[Q_SH];
                    rec[R_EAN] = -R.K * s_rec[Q_PE2];
                    rec[R_NACC] = s_rec[Q_NACC];
                    rec[R_SWEEP] = (double)(t0 + sw) + 1.0;
                    rec[7] = 0.0;
                }
            }
            if (threadIdx.x == 0) {
                // the other units of this phase released their stores before
                // counting; acquire them, then release the next phase
                __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
                __hip_atomic_store(&ready[r], phase + 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Small lattices held in LDS: one workgroup per replica copies the replica's
// three component planes into LDS, runs n whole sweeps there (colour passes
// separated by workgroup barriers, so no other workgroup is involved and no
// device-scope synchronisation is needed), optionally writes one record per
// sweep, and copies the planes back.  The site updates are the same
// arithmetic, in the same order, as the pass kernels, so the chain is
// bitwise the same.
// ---------------------------------------------------------------------------
template <typename T> using lptr = __attribute__((address_space(3))) T *;

// Block reduction for up to 1024 threads into out[0..Q_N) (LDS); fixed order.
__device__ __forceinline__ void block_reduce_1024(double (&a)[Q_N], double *out)
{
    __shared__ double red[16][Q_N];
#pragma unroll
    for (int q = 0; q < Q_N; ++q) {
        double v = a[q];
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
        a[q] = v;
    }
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int n_waves = (blockDim.x + 63) >> 6;
    if (lane == 0) {
#pragma unroll
        for (int q = 0; q < Q_N; ++q) red[wave][q] = a[q];
    }
    __syncthreads();
    if (threadIdx.x < Q_N) {
        double v = 0.0;
        for (int w = 0; w < n_waves; ++w) v += red[w][threadIdx.x];
        out[threadIdx.x] = v;
    }
    __syncthreads();
}

template <typename T, int KIND, bool MEASURE>
__global__ void __launch_bounds__(1024) k_lds_sweeps(LdsLaunch L)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char lds_raw[];
    __shared__ double s_rec[Q_N];
    constexpr int NB = basis_count(KIND);
    constexpr int NC = KIND == SC ? 2 : NB;
    const RepDev &R = L.reps_dev[blockIdx.x];
    const int Lx = R.Lx, Ly = R.Ly, Lz = R.Lz, Lxh = R.Lxh;
    const uint32_t n_box = R.n_box, plane = R.plane, rid = R.rid;
    const gptr<T> gx = as_global<T>(R.sx), gy = as_global<T>(R.sy), gz = as_global<T>(R.sz);
    const T J = (T)R.J, K = (T)R.K, ex = (T)R.e[0], ey = (T)R.e[1], ez = (T)R.e[2];
    const T beta = (T)R.beta;
    const bool greedy = R.greedy != 0;
    const bool px = R.pmask & 1u, py = R.pmask & 2u, pz = R.pmask & 4u;
    const double Kd = R.K;
    const uint32_t t0 = *L.tctr_dev;
    const lptr<T> lx = (lptr<T>)(lptr<unsigned char>)lds_raw;
    const lptr<T> ly = lx + n_box, lz = ly + n_box;
    for (uint32_t i = threadIdx.x; i < n_box; i += blockDim.x) {
        lx[i] = gx[i];
        ly[i] = gy[i];
        lz[i] = gz[i];
    }
    __syncthreads();
    for (uint32_t sw = 0; sw < L.n_sweeps; ++sw) {
        const uint32_t t = t0 + sw;
        double acc[Q_N] = {0, 0, 0, 0, 0, 0};
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            for (uint32_t k = threadIdx.x; k < plane; k += blockDim.x) {
                T hx, hy, hz, sh_x, sh_y, sh_z;
                uint32_t i, s;
                if constexpr (KIND == SC) {
                    const int xh = (int)(k % (uint32_t)Lxh);
                    const uint32_t row = k / (uint32_t)Lxh;
                    const int y = (int)(row % (uint32_t)Ly), z = (int)(row / (uint32_t)Ly);
                    const int p = (c + y + z) & 1;
                    sc_site_field<T>(lx, ly, lz, c ? 0u : plane, Lxh, Ly, Lz, px, py, pz, xh, y,
                                     z, p, hx, hy, hz);
                    i = (c ? plane : 0u) + k;
                    s = row * (uint32_t)Lx + 2u * (uint32_t)xh + (uint32_t)p;
                } else {
                    const int x = (int)(k % (uint32_t)Lx);
                    const uint32_t r2 = k / (uint32_t)Lx;
                    const int y = (int)(r2 % (uint32_t)Ly), z = (int)(r2 / (uint32_t)Ly);
                    if (!occupied(R, x, y, z, basis2(KIND, c, 0), basis2(KIND, c, 1),
                                  basis2(KIND, c, 2)))
                        continue;
                    switch (c) {
                    case 0:
                        basis_site_field<KIND, 0, T>(lx, ly, lz, plane, Lx, Ly, Lz, px, py, pz, x,
                                                     y, z, hx, hy, hz, sh_x, sh_y, sh_z);
                        break;
                    case 1:
                        basis_site_field<KIND, 1, T>(lx, ly, lz, plane, Lx, Ly, Lz, px, py, pz, x,
                                                     y, z, hx, hy, hz, sh_x, sh_y, sh_z);
                        break;
                    case 2:
                        basis_site_field<KIND, (NB > 2 ? 2 : 0), T>(lx, ly, lz, plane, Lx, Ly, Lz,
                                                                    px, py, pz, x, y, z, hx, hy,
                                                                    hz, sh_x, sh_y, sh_z);
                        break;
                    default:
                        basis_site_field<KIND, (NB > 3 ? 3 : 0), T>(lx, ly, lz, plane, Lx, Ly, Lz,
                                                                    px, py, pz, x, y, z, hx, hy,
                                                                    hz, sh_x, sh_y, sh_z);
                        break;
                    }
                    i = (uint32_t)c * plane + k;
                    s = k * NB + (uint32_t)c;
                }
                hx *= J;
                hy *= J;
                hz *= J;
                T sx = lx[i], sy = ly[i], sz = lz[i];
                T dH;
                const bool a = metropolis<T>(sx, sy, sz, hx, hy, hz, s, rid, t, L.seed_lo,
                                             L.seed_hi, K, ex, ey, ez, beta, greedy, dH);
                if (a) {
                    lx[i] = sx;
                    ly[i] = sy;
                    lz[i] = sz;
                }
                if (MEASURE) {
                    T sh;
                    if constexpr (KIND == SC) sh = c == 1 ? sx * hx + sy * hy + sz * hz : T(0);
                    else sh = J * (sx * sh_x + sy * sh_y + sz * sh_z);
                    accumulate<T>(acc, sx, sy, sz, ex, ey, ez, sh, a);
                }
            }
            __syncthreads();
        }
        if (MEASURE) {
            block_reduce_1024(acc, s_rec);
            if (threadIdx.x == 0) {
                double *rec = L.records +
                              ((size_t)((L.slot0 + sw) % L.ring) * L.n_reps + blockIdx.x) * NR;
                rec[R_MX] = s_rec[Q_MX];
                rec[R_MY] = s_rec[Q_MY];
                rec[R_MZ] = s_rec[Q_MZ];
                rec[R_EEX] = -s_rec[Q_SH];
                rec[R_EAN] = -Kd * s_rec[Q_PE2];
                rec[R_NACC] = s_rec[Q_NACC];
                rec[R_SWEEP] = (double)t + 1.0;
                rec[7] = 0.0;
            }
        }
    }
    for (uint32_t i = threadIdx.x; i < n_box; i += blockDim.x) {
        gx[i] = lx[i];
        gy[i] = ly[i];
        gz[i] = lz[i];
    }
}

// ---------------------------------------------------------------------------
// Initial state and layout conversion (one replica per launch).
// ---------------------------------------------------------------------------
struct SiteCoord {
    int x, y, z, b;
    uint32_t s; // canonical index
};

__device__ __forceinline__ SiteCoord decode(const RepDev &R, int kind, uint32_t i)
{
    SiteCoord c;
    const uint32_t colour = i / R.plane, j = i - colour * R.plane;
    if (kind == SC) {
        const uint32_t xh = j % (uint32_t)R.Lxh, r = j / (uint32_t)R.Lxh;
        c.y = (int)(r % (uint32_t)R.Ly);
        c.z = (int)(r / (uint32_t)R.Ly);
        c.x = 2 * (int)xh + (int)((colour + c.y + c.z) & 1u);
        c.b = 0;
        c.s = (uint32_t)(c.z * R.Ly + c.y) * (uint32_t)R.Lx + c.x;
    } else {
        c.x = (int)(j % (uint32_t)R.Lx);
        const uint32_t r = j / (uint32_t)R.Lx;
        c.y = (int)(r % (uint32_t)R.Ly);
        c.z = (int)(r / (uint32_t)R.Ly);
        c.b = (int)colour;
        c.s = j * (uint32_t)basis_count(kind) + colour;
    }
    return c;
}

__device__ __forceinline__ bool occupied_site(const RepDev &R, int kind, const SiteCoord &c)
{
    int bx = 0, by = 0, bz = 0;
    if (kind == BCC) bx = by = bz = c.b;
    if (kind == FCC) {
        bx = c.b == 1 || c.b == 2;
        by = c.b == 1 || c.b == 3;
        bz = c.b == 2 || c.b == 3;
    }
    return occupied(R, c.x, c.y, c.z, bx, by, bz);
}

template <typename T>
__global__ void __launch_bounds__(256)
k_init(RepDev R, int kind, int mode, uint32_t k0, uint32_t k1)
{
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < R.n_box;
         i += gridDim.x * blockDim.x) {
        const SiteCoord c = decode(R, kind, i);
        T vx = 0, vy = 0, vz = 0;
        if (occupied_site(R, kind, c)) {
            if (mode == 1) {
                vx = (T)R.e[0];
                vy = (T)R.e[1];
                vz = (T)R.e[2];
            } else {
                const Words w = philox10(c.s, R.rid, 0u, 1u, k0, k1);
                sphere_point(uniform23<T>(w.w0), uniform23<T>(w.w1), vx, vy, vz);
            }
        }
        ((T *)R.sx)[i] = vx;
        ((T *)R.sy)[i] = vy;
        ((T *)R.sz)[i] = vz;
    }
}

template <typename T>
__global__ void __launch_bounds__(256)
k_layout(RepDev R, int kind, int to_natural, T *nx, T *ny, T *nz)
{
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < R.n_box;
         i += gridDim.x * blockDim.x) {
        const SiteCoord c = decode(R, kind, i);
        T *px = (T *)R.sx, *py = (T *)R.sy, *pz = (T *)R.sz;
        if (to_natural) {
            nx[c.s] = px[i];
            ny[c.s] = py[i];
            nz[c.s] = pz[i];
        } else {
            px[i] = nx[c.s];
            py[i] = ny[c.s];
            pz[i] = nz[c.s];
        }
    }
}

// ---------------------------------------------------------------------------
// Finalise: FIN_BLOCKS blocks per replica each sum a contiguous share of the
// replica's partial slots (all passes) into a stage slot; the last block to
// finish (counted with an agent-scope atomic) sums the stage slots in index
// order and writes the FP64 record, then re-arms the counter.  The result
// depends only on the work list, not on block timing.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256)
k_finalize(const RepDev *__restrict__ reps, int n_colours, const double *__restrict__ partials,
           uint32_t n_items, const uint32_t *__restrict__ tctr, uint32_t t_off,
           double *__restrict__ records, double *__restrict__ stage, uint32_t *__restrict__ count)
{
    const uint32_t r = blockIdx.x / FIN_BLOCKS, j = blockIdx.x % FIN_BLOCKS;
    const RepDev &R = reps[r];
    const uint32_t n = R.item_end - R.item_begin;
    const uint32_t b0 = R.item_begin + (uint32_t)(((uint64_t)n * j) / FIN_BLOCKS);
    const uint32_t b1 = R.item_begin + (uint32_t)(((uint64_t)n * (j + 1)) / FIN_BLOCKS);
    double a[Q_N] = {0, 0, 0, 0, 0, 0};
    for (int c = 0; c < n_colours; ++c)
        for (uint32_t it = b0 + threadIdx.x; it < b1; it += blockDim.x) {
            const double *p = partials + ((size_t)c * n_items + it) * NQ;
#pragma unroll
            for (int q = 0; q < Q_N; ++q) a[q] += p[q];
        }
    double *slot = stage + ((size_t)r * FIN_BLOCKS + j) * NQ;
    block_store_partials(a, slot);
    __shared__ uint32_t last;
    __threadfence(); // the stage slot is visible device-wide before it is counted
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t done = __hip_atomic_fetch_add(&count[r], 1u, __ATOMIC_ACQ_REL,
                                                     __HIP_MEMORY_SCOPE_AGENT);
        last = done == FIN_BLOCKS - 1;
    }
    __syncthreads();
    if (!last) return;
    if (threadIdx.x == 0) {
        __atomic_thread_fence(__ATOMIC_ACQUIRE);
        double out[Q_N] = {0, 0, 0, 0, 0, 0};
        const double *st = stage + (size_t)r * FIN_BLOCKS * NQ;
        for (uint32_t b = 0; b < FIN_BLOCKS; ++b)
#pragma unroll
            for (int q = 0; q < Q_N; ++q)
                out[q] += __hip_atomic_load(&st[b * NQ + q], __ATOMIC_RELAXED,
                                            __HIP_MEMORY_SCOPE_AGENT);
        double *rec = records + (size_t)r * NR;
        rec[R_MX] = out[Q_MX];
        rec[R_MY] = out[Q_MY];
        rec[R_MZ] = out[Q_MZ];
        rec[R_EEX] = -out[Q_SH];
        rec[R_EAN] = -R.K * out[Q_PE2];
        rec[R_NACC] = out[Q_NACC];
        rec[R_SWEEP] = (double)(*tctr + t_off) + 1.0;
        rec[7] = 0.0;
        __hip_atomic_store(&count[r], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

__global__ void k_advance(uint32_t *tctr, uint32_t n)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *tctr += n;
}

__global__ void k_set_counter(uint32_t *tctr, uint32_t v)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *tctr = v;
}

__global__ void k_fill_zero(double *p, uint64_t n)
{
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = 0.0;
}

// ---------------------------------------------------------------------------
// Memory-pattern probe: the HBM streams of one colour pass without its
// arithmetic.  Three component arrays of 2 P elements; the first half is read
// and written in place, the second half read (24 B read and 12 B written per
// FP32 element of the first half), two elements per lane per access.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) k_stream_probe(T *x, T *y, T *z, uint64_t P)
{
    const uint64_t n2 = P / 2; // element pairs per half
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n2;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t a = 2 * i, b = P + 2 * i;
        const T x0 = x[a] + x[b], x1 = x[a + 1] + x[b + 1];
        const T y0 = y[a] + y[b], y1 = y[a + 1] + y[b + 1];
        const T z0 = z[a] + z[b], z1 = z[a + 1] + z[b + 1];
        x[a] = x0;
        x[a + 1] = x1;
        y[a] = y0;
        y[a + 1] = y1;
        z[a] = z0;
        z[a + 1] = z1;
    }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
static dim3 pass_grid(const PassLaunch &p) { return dim3(((p.n_blocks + 7u) >> 3) << 3); }

template <typename T, bool MEASURE, int MODE>
static hipError_t sc_launch(int colour, const PassLaunch &p, hipStream_t st)
{
    if (p.tile.kernel == KERNEL_BAND) {
        const dim3 g = pass_grid(p), b(p.tile.tx);
        switch (p.tile.ty) {
        case 2: hipLaunchKernelGGL((k_sc_band<T, MEASURE, MODE, 2>), g, b, 0, st, p, colour); break;
        case 4: hipLaunchKernelGGL((k_sc_band<T, MEASURE, MODE, 4>), g, b, 0, st, p, colour); break;
        default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    if (p.tile.kernel == KERNEL_PBAND) {
        const dim3 g = pass_grid(p), b(p.tile.tx);
        switch (p.tile.ty) {
        case 2: hipLaunchKernelGGL((k_sc_pband<T, MEASURE, MODE, 2>), g, b, 0, st, p, colour); break;
        case 4: hipLaunchKernelGGL((k_sc_pband<T, MEASURE, MODE, 4>), g, b, 0, st, p, colour); break;
        default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    if (p.tile.kernel == KERNEL_PAIR) {
        const dim3 g = pass_grid(p), b(p.tile.tx);
        switch (p.tile.ty) {
        case 1: hipLaunchKernelGGL((k_sc_pair<T, MEASURE, MODE, 1>), g, b, 0, st, p, colour); break;
        case 2: hipLaunchKernelGGL((k_sc_pair<T, MEASURE, MODE, 2>), g, b, 0, st, p, colour); break;
        case 4: hipLaunchKernelGGL((k_sc_pair<T, MEASURE, MODE, 4>), g, b, 0, st, p, colour); break;
        default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    if (p.tile.kernel == KERNEL_STRIP) {
        const dim3 g = pass_grid(p), b(p.tile.tx);
        switch (p.tile.ty) {
        case 1: hipLaunchKernelGGL((k_sc_strip<T, MEASURE, MODE, 1>), g, b, 0, st, p, colour); break;
        case 2: hipLaunchKernelGGL((k_sc_strip<T, MEASURE, MODE, 2>), g, b, 0, st, p, colour); break;
        case 4: hipLaunchKernelGGL((k_sc_strip<T, MEASURE, MODE, 4>), g, b, 0, st, p, colour); break;
        case 8: hipLaunchKernelGGL((k_sc_strip<T, MEASURE, MODE, 8>), g, b, 0, st, p, colour); break;
        default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    const int threads = ((p.tile.tx * p.tile.ty + 63) / 64) * 64;
    hipLaunchKernelGGL((k_sc_tile<T, MEASURE, MODE>), pass_grid(p), dim3(threads), 0, st, p,
                       colour);
    return hipGetLastError();
}

template <int KIND, typename T, bool MEASURE, int MODE>
static hipError_t basis_launch(int colour, const PassLaunch &p, hipStream_t st)
{
    const int threads = ((p.tile.tx * p.tile.ty + 63) / 64) * 64;
    const dim3 g = pass_grid(p), b(threads);
    if (p.tile.kernel == KERNEL_BSTRIP) {
        switch (colour) {
        case 0: hipLaunchKernelGGL((k_basis_strip<KIND, 0, T, MEASURE, MODE>), g, b, 0, st, p); break;
        case 1: hipLaunchKernelGGL((k_basis_strip<KIND, 1, T, MEASURE, MODE>), g, b, 0, st, p); break;
        case 2:
            if constexpr (KIND == FCC) hipLaunchKernelGGL((k_basis_strip<KIND, 2, T, MEASURE, MODE>), g, b, 0, st, p);
            break;
        case 3:
            if constexpr (KIND == FCC) hipLaunchKernelGGL((k_basis_strip<KIND, 3, T, MEASURE, MODE>), g, b, 0, st, p);
            break;
        default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    switch (colour) {
    case 0: hipLaunchKernelGGL((k_basis_pass<KIND, 0, T, MEASURE, MODE>), g, b, 0, st, p); break;
    case 1: hipLaunchKernelGGL((k_basis_pass<KIND, 1, T, MEASURE, MODE>), g, b, 0, st, p); break;
    case 2:
        if constexpr (KIND == FCC) hipLaunchKernelGGL((k_basis_pass<KIND, 2, T, MEASURE, MODE>), g, b, 0, st, p);
        break;
    case 3:
        if constexpr (KIND == FCC) hipLaunchKernelGGL((k_basis_pass<KIND, 3, T, MEASURE, MODE>), g, b, 0, st, p);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T, bool MEASURE, int MODE>
static hipError_t pass_dispatch(int kind, int colour, const PassLaunch &p, hipStream_t st)
{
    switch (kind) {
    case SC: return sc_launch<T, MEASURE, MODE>(colour, p, st);
    case BCC: return basis_launch<BCC, T, MEASURE, MODE>(colour, p, st);
    case FCC: return basis_launch<FCC, T, MEASURE, MODE>(colour, p, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_pass(int kind, bool f64, int colour, bool measure, int mode, const PassLaunch &p,
                       hipStream_t st)
{
    if (p.n_blocks == 0) return hipSuccess;
    if (mode == 1) {
        return f64 ? pass_dispatch<double, true, 1>(kind, colour, p, st)
                   : pass_dispatch<float, true, 1>(kind, colour, p, st);
    }
    if (mode == 2) {
        if (!p.dbg_dh || !p.dbg_acc) return hipErrorInvalidValue;
        return f64 ? pass_dispatch<double, false, 2>(kind, colour, p, st)
                   : pass_dispatch<float, false, 2>(kind, colour, p, st);
    }
    if (f64)
        return measure ? pass_dispatch<double, true, 0>(kind, colour, p, st)
                       : pass_dispatch<double, false, 0>(kind, colour, p, st);
    return measure ? pass_dispatch<float, true, 0>(kind, colour, p, st)
                   : pass_dispatch<float, false, 0>(kind, colour, p, st);
}

static unsigned grid_for(uint32_t n)
{
    uint32_t g = (n + 255) / 256;
    return g < 8192 ? (g ? g : 1) : 8192;
}

hipError_t launch_init(bool f64, int kind, const RepDev *rep_host, int mode, uint32_t seed_lo,
                       uint32_t seed_hi, hipStream_t st)
{
    const unsigned g = grid_for(rep_host->n_box);
    if (f64)
        hipLaunchKernelGGL((k_init<double>), dim3(g), dim3(256), 0, st, *rep_host, kind, mode,
                           seed_lo, seed_hi);
    else
        hipLaunchKernelGGL((k_init<float>), dim3(g), dim3(256), 0, st, *rep_host, kind, mode,
                           seed_lo, seed_hi);
    return hipGetLastError();
}

hipError_t launch_layout(bool f64, int kind, const RepDev *rep_host, bool to_natural, void *nx,
                         void *ny, void *nz, hipStream_t st)
{
    const unsigned g = grid_for(rep_host->n_box);
    if (f64)
        hipLaunchKernelGGL((k_layout<double>), dim3(g), dim3(256), 0, st, *rep_host, kind,
                           (int)to_natural, (double *)nx, (double *)ny, (double *)nz);
    else
        hipLaunchKernelGGL((k_layout<float>), dim3(g), dim3(256), 0, st, *rep_host, kind,
                           (int)to_natural, (float *)nx, (float *)ny, (float *)nz);
    return hipGetLastError();
}

hipError_t launch_finalize(const RepDev *reps_dev, int n_reps, int n_colours,
                           const double *partials_dev, uint32_t n_items,
                           const uint32_t *tctr_dev, uint32_t t_off, double *records_dev,
                           double *stage_dev, uint32_t *count_dev, hipStream_t st)
{
    hipLaunchKernelGGL(k_finalize, dim3(n_reps * FIN_BLOCKS), dim3(256), 0, st, reps_dev,
                       n_colours, partials_dev, n_items, tctr_dev, t_off, records_dev, stage_dev,
                       count_dev);
    return hipGetLastError();
}

__global__ void k_zero_u32(uint32_t *p, uint32_t n)
{
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        p[i] = 0u;
}

hipError_t launch_zero_u32(uint32_t *p, uint32_t n, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero_u32, dim3((n + 255) / 256 < 1024 ? (n + 255) / 256 : 1024), dim3(256),
                       0, st, p, n);
    return hipGetLastError();
}

template <typename T, bool MEASURE>
static hipError_t persist_dispatch(int kind, const PassLaunch &p, const PersistLaunch &a,
                                   hipStream_t st)
{
    // at most one phase of every replica (n_items units in all) can run at a
    // time; workgroups beyond twice that would only wait
    const uint64_t total = (uint64_t)a.n_sweeps * a.n_colours * p.n_items;
    uint64_t cap = 2ull * p.n_items;
    if (cap > 2048) cap = 2048;
    const unsigned grid = (unsigned)(total < cap ? total : cap);
    if (grid == 0) return hipSuccess;
    // tx x ty threads for the tile-shaped kernels (a persistent unit of a bcc
    // or fcc lattice runs the tile body on the same tile), tx for the others
    const bool tile_shaped = p.tile.kernel == KERNEL_TILE || p.tile.kernel == KERNEL_BSTRIP;
    const int threads = tile_shaped ? ((p.tile.tx * p.tile.ty + 63) / 64) * 64 : p.tile.tx;
    const dim3 g(grid), b(threads);
    if (kind == BCC) {
        hipLaunchKernelGGL((k_persistent<T, MEASURE, BCC, KERNEL_TILE, 1>), g, b, 0, st, p, a);
    } else if (kind == FCC) {
        hipLaunchKernelGGL((k_persistent<T, MEASURE, FCC, KERNEL_TILE, 1>), g, b, 0, st, p, a);
    } else if (p.tile.kernel == KERNEL_TILE) {
        hipLaunchKernelGGL((k_persistent<T, MEASURE, SC, KERNEL_TILE, 1>), g, b, 0, st, p, a);
    } else if (p.tile.kernel == KERNEL_STRIP && p.tile.ty == 2) {
        hipLaunchKernelGGL((k_persistent<T, MEASURE, SC, KERNEL_STRIP, 2>), g, b, 0, st, p, a);
    } else if (p.tile.kernel == KERNEL_STRIP && p.tile.ty == 4) {
        hipLaunchKernelGGL((k_persistent<T, MEASURE, SC, KERNEL_STRIP, 4>), g, b, 0, st, p, a);
    } else if (p.tile.kernel == KERNEL_PBAND && p.tile.ty == 2) {
        hipLaunchKernelGGL((k_persistent<T, MEASURE, SC, KERNEL_PBAND, 2>), g, b, 0, st, p, a);
    } else if (p.tile.kernel == KERNEL_PAIR && p.tile.ty == 1) {
        hipLaunchKernelGGL((k_persistent<T, MEASURE, SC, KERNEL_PAIR, 1>), g, b, 0, st, p, a);
    } else if (p.tile.kernel == KERNEL_PAIR && p.tile.ty == 2) {
        hipLaunchKernelGGL((k_persistent<T, MEASURE, SC, KERNEL_PAIR, 2>), g, b, 0, st, p, a);
    } else if (p.tile.kernel == KERNEL_BAND && p.tile.ty == 2) {
        hipLaunchKernelGGL((k_persistent<T, MEASURE, SC, KERNEL_BAND, 2>), g, b, 0, st, p, a);
    } else if (p.tile.kernel == KERNEL_BAND && p.tile.ty == 4) {
        hipLaunchKernelGGL((k_persistent<T, MEASURE, SC, KERNEL_BAND, 4>), g, b, 0, st, p, a);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T, bool MEASURE>
static hipError_t lds_dispatch(int kind, const LdsLaunch &L, int threads, hipStream_t st)
{
    const dim3 g(L.n_reps), b(threads);
    if (kind == SC)
        hipLaunchKernelGGL((k_lds_sweeps<T, SC, MEASURE>), g, b, L.lds_bytes, st, L);
    else if (kind == BCC)
        hipLaunchKernelGGL((k_lds_sweeps<T, BCC, MEASURE>), g, b, L.lds_bytes, st, L);
    else
        hipLaunchKernelGGL((k_lds_sweeps<T, FCC, MEASURE>), g, b, L.lds_bytes, st, L);
    return hipGetLastError();
}

hipError_t launch_lds(int kind, bool f64, bool measure, const LdsLaunch &L, int threads,
                      hipStream_t st)
{
    if (L.n_reps == 0 || L.n_sweeps == 0) return hipSuccess;
    if (threads < 64 || threads > 1024 || threads % 64) return hipErrorInvalidValue;
    if (f64)
        return measure ? lds_dispatch<double, true>(kind, L, threads, st)
                       : lds_dispatch<double, false>(kind, L, threads, st);
    return measure ? lds_dispatch<float, true>(kind, L, threads, st)
                   : lds_dispatch<float, false>(kind, L, threads, st);
}

template <typename T> static hipError_t lds_allow_kind(int kind, uint32_t bytes)
{
    const void *f[2];
    if (kind == SC) {
        f[0] = (const void *)&k_lds_sweeps<T, SC, false>;
        f[1] = (const void *)&k_lds_sweeps<T, SC, true>;
    } else if (kind == BCC) {
        f[0] = (const void *)&k_lds_sweeps<T, BCC, false>;
        f[1] = (const void *)&k_lds_sweeps<T, BCC, true>;
    } else {
        f[0] = (const void *)&k_lds_sweeps<T, FCC, false>;
        f[1] = (const void *)&k_lds_sweeps<T, FCC, true>;
    }
    for (const void *fn : f) {
        const hipError_t e =
            hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t lds_allow(int kind, bool f64, uint32_t bytes)
{
    return f64 ? lds_allow_kind<double>(kind, bytes) : lds_allow_kind<float>(kind, bytes);
}

hipError_t launch_persistent(int kind, bool f64, bool measure, const PassLaunch &p,
                             const PersistLaunch &a, hipStream_t st)
{
    if ((uint64_t)a.n_sweeps * a.n_colours * p.n_items >= 0xFFFFFFFFull) return hipErrorInvalidValue;
    if (f64)
        return measure ? persist_dispatch<double, true>(kind, p, a, st)
                       : persist_dispatch<double, false>(kind, p, a, st);
    return measure ? persist_dispatch<float, true>(kind, p, a, st)
                   : persist_dispatch<float, false>(kind, p, a, st);
}

hipError_t launch_advance(uint32_t *tctr_dev, uint32_t n, hipStream_t st)
{
    hipLaunchKernelGGL(k_advance, dim3(1), dim3(64), 0, st, tctr_dev, n);
    return hipGetLastError();
}

hipError_t launch_set_counter(uint32_t *tctr_dev, uint32_t v, hipStream_t st)
{
    hipLaunchKernelGGL(k_set_counter, dim3(1), dim3(64), 0, st, tctr_dev, v);
    return hipGetLastError();
}

hipError_t launch_fill_zero(double *p, uint64_t n, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    const unsigned g = grid_for((uint32_t)(n < 0xFFFFFFFFull ? n : 0xFFFFFFFFull));
    hipLaunchKernelGGL(k_fill_zero, dim3(g), dim3(256), 0, st, p, n);
    return hipGetLastError();
}

hipError_t launch_stream_probe(bool f64, void *x, void *y, void *z, uint64_t P, uint32_t grid,
                               hipStream_t st)
{
    if (grid == 0 || P < 2) return hipErrorInvalidValue;
    if (f64)
        hipLaunchKernelGGL(k_stream_probe<double>, dim3(grid), dim3(256), 0, st, (double *)x,
                           (double *)y, (double *)z, P);
    else
        hipLaunchKernelGGL(k_stream_probe<float>, dim3(grid), dim3(256), 0, st, (float *)x,
                           (float *)y, (float *)z, P);
    return hipGetLastError();
}

} // namespace mc
