// device_common.hpp -- device helpers shared by the CDNA4 (gfx950) kernels of the
// colour-sweep Metropolis method
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
#pragma once

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
// increments between rounds.  A three-way XOR of varying words is one CDNA4
// v_bitop3_b32 (truth table 0x96), which the compiler does not form from two
// XORs itself.  Plain XORs stay where the words can be uniform (the replica
// and sweep words of a colour pass's counter, and what the first round makes
// of them), so that their part runs in scalar instructions.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c)
{
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

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
        const uint32_t n0 = r <= 1 ? (uint32_t)(pb >> 32) ^ c1 ^ k0 : xor3((uint32_t)(pb >> 32), c1, k0);
        const uint32_t n2 = r <= 2 ? (uint32_t)(pa >> 32) ^ c3 ^ k1 : xor3((uint32_t)(pa >> 32), c3, k1);
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

// The XCD (0..7) the calling wave runs on (hardware register XCC_ID).
__device__ __forceinline__ uint32_t xcd_id()
{
    uint32_t v;
    asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID)" : "=s"(v));
    return v & 7u;
}

// ---------------------------------------------------------------------------
// Block reduction of Q_N doubles (fixed order: wave butterflies, then waves in
// index order), written to one partial slot.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void block_store_partials(double (&a)[Q_N], double *dst)
{
    __shared__ double red[16][Q_N]; // up to 1024 threads
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

// One Metropolis attempt with local field h (J already applied) from the
// words w of its Philox block: proposal from w0, w1, acceptance uniform from
// w2.  Returns the final spin in (sx, sy, sz).
template <typename T>
__device__ __forceinline__ bool metropolis_words(const Words &w, T &sx, T &sy, T &sz, T hx, T hy,
                                                 T hz, T K, T ex, T ey, T ez, T beta, bool greedy,
                                                 T &dH)
{
    T nx, ny, nz;
    sphere_point(uniform23<T>(w.w0), uniform23<T>(w.w1), nx, ny, nz);
    const T P = uniform23<T>(w.w2);
    const T dx = nx - sx, dy = ny - sy, dz = nz - sz;
    const T pn = nx * ex + ny * ey + nz * ez;
    const T po = sx * ex + sy * ey + sz * ez;
    // Eq. (1): dH = -h.(S'-S) - K[(S'.e)^2 - (S.e)^2]
    dH = -(hx * dx + hy * dy + hz * dz) - K * ((pn - po) * (pn + po));
    // Non-short-circuit: both comparisons stay lane masks, combined with the
    // uniform greedy flag by scalar mask operations.
    const bool acc = (dH <= T(0)) | ((P <= fast_exp(-beta * dH)) & !greedy);
    if (acc) {
        const T inv = inv_norm(nx * nx + ny * ny + nz * nz);
        sx = nx * inv;
        sy = ny * inv;
        sz = nz * inv;
    }
    return acc;
}

// The attempt of a colour pass: canonical site s, replica rid and sweep t key
// the stream (counter (s, rid, t, 0)).
template <typename T>
__device__ __forceinline__ bool metropolis(T &sx, T &sy, T &sz, T hx, T hy, T hz, uint32_t s,
                                           uint32_t rid, uint32_t t, uint32_t k0, uint32_t k1,
                                           T K, T ex, T ey, T ez, T beta, bool greedy, T &dH)
{
    const Words w = philox10(s, rid, t, 0u, k0, k1);
    return metropolis_words<T>(w, sx, sy, sz, hx, hy, hz, K, ex, ey, ez, beta, greedy, dH);
}

// FP64 observables of one final spin: its components (Eq. (2)), (S.e)^2 and,
// for a site that closes bonds, S dotted with the field h of its
// already-final neighbours scaled by jscale (1 when h has J applied, J when
// it has not).  The products are formed from FP64 operands, so every kernel
// adds the same per-site values and records differ between kernels only by
// the FP64 summation order.
template <typename T>
__device__ __forceinline__ void observe(double (&acc)[Q_N], T sx, T sy, T sz, T ex, T ey, T ez,
                                        bool bonds, T hx, T hy, T hz, double jscale)
{
    const double dx = (double)sx, dy = (double)sy, dz = (double)sz;
    acc[Q_MX] += dx;
    acc[Q_MY] += dy;
    acc[Q_MZ] += dz;
    const double pe = dx * (double)ex + dy * (double)ey + dz * (double)ez;
    acc[Q_PE2] += pe * pe;
    if (bonds) acc[Q_SH] += jscale * (dx * (double)hx + dy * (double)hy + dz * (double)hz);
}

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

// The descriptor is uniform by construction; its fields are passed through
// readfirstlane so the compiler keeps it in scalar registers on every path
// (a descriptor it believes divergent turns each access into a loop).
template <typename T>
__device__ __forceinline__ rsrc_t plane_rsrc(void *comp, uint32_t elem_off, uint32_t n_elems)
{
    const uint64_t a = (uint64_t)(uintptr_t)comp + (uint64_t)elem_off * sizeof(T);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)a);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
    const uint32_t bytes = __builtin_amdgcn_readfirstlane(n_elems * (uint32_t)sizeof(T));
    return __builtin_amdgcn_make_buffer_rsrc((void *)(uintptr_t)(((uint64_t)hi << 32) | lo),
                                             (short)0, (int)bytes, kRsrcWord3);
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

} // namespace mc
