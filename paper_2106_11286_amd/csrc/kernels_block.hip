// kernels_block.hip -- the paper's block scheme in synchronous form, for
// comparison with the colour sweep (simple cubic).  A step is two launches:
// every block of n consecutive canonical sites picks one site and computes its
// attempt from the state before the step, staging the accepted spin; then the
// staged moves are written.
#include "device_common.hpp"

namespace mc {

__device__ __forceinline__ uint32_t block_pick(uint32_t k, uint32_t n, uint32_t n_box,
                                               uint32_t rid, uint32_t step, uint32_t k0,
                                               uint32_t k1, Words &w)
{
    const uint32_t m = min(n, n_box - k * n);
    w = philox10(k, rid, step, 3u, k0, k1);
    return k * n + (uint32_t)(((uint64_t)w.w3 * m) >> 32);
}

// Colour-packed storage index of canonical sc site (x, y, z).
__device__ __forceinline__ uint32_t sc_store(int x, int y, int z, int Lx, int Ly, uint32_t plane)
{
    const uint32_t c = (uint32_t)(x + y + z) & 1u;
    return c * plane + (((uint32_t)(z * Ly + y) * (uint32_t)Lx + (uint32_t)x) >> 1);
}

template <typename T>
__global__ void __launch_bounds__(256) k_block_propose(BlockLaunch B)
{
    const RepDev &R = B.rep;
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t att = 0, acc = 0, conf = 0;
    if (k < B.n_blocks) {
        const int Lx = R.Lx, Ly = R.Ly, Lz = R.Lz;
        Words w;
        const uint32_t s = block_pick(k, B.n, R.n_box, R.rid, B.step, B.seed_lo, B.seed_hi, w);
        const int x = (int)(s % (uint32_t)Lx), y = (int)((s / (uint32_t)Lx) % (uint32_t)Ly);
        const int z = (int)(s / ((uint32_t)Lx * (uint32_t)Ly));
        uint32_t out = 0xFFFFFFFFu;
        if (occupied(R, x, y, z, 0, 0, 0)) {
            att = 1;
            const T *gx = (const T *)R.sx, *gy = (const T *)R.sy, *gz = (const T *)R.sz;
            const bool px = R.pmask & 1u, py = R.pmask & 2u, pz = R.pmask & 4u;
            // neighbours -x, +x, -y, +y, -z, +z (missing across open faces)
            int q[6][3] = {{x - 1, y, z}, {x + 1, y, z}, {x, y - 1, z},
                           {x, y + 1, z}, {x, y, z - 1}, {x, y, z + 1}};
            T hx = 0, hy = 0, hz = 0;
#pragma unroll
            for (int j = 0; j < 6; ++j) {
                int &a = q[j][0], &b = q[j][1], &c = q[j][2];
                bool ok = true;
                if (a < 0) { a += Lx; ok &= px; }
                if (a >= Lx) { a -= Lx; ok &= px; }
                if (b < 0) { b += Ly; ok &= py; }
                if (b >= Ly) { b -= Ly; ok &= py; }
                if (c < 0) { c += Lz; ok &= pz; }
                if (c >= Lz) { c -= Lz; ok &= pz; }
                if (!ok || !occupied(R, a, b, c, 0, 0, 0)) {
                    a = -1;
                    continue;
                }
                const uint32_t i = sc_store(a, b, c, Lx, Ly, R.plane);
                hx += gx[i];
                hy += gy[i];
                hz += gz[i];
                if (B.count_conflicts && !conf) {
                    const uint32_t qs = ((uint32_t)(c * Ly + b) * (uint32_t)Lx) + (uint32_t)a;
                    Words w2;
                    if (block_pick(qs / B.n, B.n, R.n_box, R.rid, B.step, B.seed_lo, B.seed_hi,
                                   w2) == qs)
                        conf = 1;
                }
            }
            const T J = (T)R.J;
            hx *= J;
            hy *= J;
            hz *= J;
            const uint32_t i = sc_store(x, y, z, Lx, Ly, R.plane);
            T sx = gx[i], sy = gy[i], sz = gz[i];
            T dH;
            if (metropolis_words<T>(w, sx, sy, sz, hx, hy, hz, (T)R.K, (T)R.e[0], (T)R.e[1],
                                    (T)R.e[2], (T)R.beta, R.greedy != 0, dH)) {
                acc = 1;
                out = i;
                T *st = (T *)B.stage_spin + 3 * (size_t)k;
                st[0] = sx;
                st[1] = sy;
                st[2] = sz;
            }
        }
        B.stage_idx[k] = out;
    }
    // counts: wave sums, then one atomic per wave
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        att += __shfl_xor(att, o, 64);
        acc += __shfl_xor(acc, o, 64);
        conf += __shfl_xor(conf, o, 64);
    }
    if ((threadIdx.x & 63) == 0 && att) {
        atomicAdd(B.counts + 0, (unsigned long long)att);
        atomicAdd(B.counts + 1, (unsigned long long)acc);
        atomicAdd(B.counts + 2, (unsigned long long)conf);
    }
}

template <typename T>
__global__ void __launch_bounds__(256) k_block_apply(BlockLaunch B)
{
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= B.n_blocks) return;
    const uint32_t i = B.stage_idx[k];
    if (i == 0xFFFFFFFFu) return;
    const T *st = (const T *)B.stage_spin + 3 * (size_t)k;
    ((T *)B.rep.sx)[i] = st[0];
    ((T *)B.rep.sy)[i] = st[1];
    ((T *)B.rep.sz)[i] = st[2];
}

hipError_t launch_block_step(bool f64, const BlockLaunch &B, hipStream_t st)
{
    if (B.n_blocks == 0) return hipSuccess;
    const dim3 g((B.n_blocks + 255) / 256), b(256);
    if (f64) {
        hipLaunchKernelGGL(k_block_propose<double>, g, b, 0, st, B);
        hipLaunchKernelGGL(k_block_apply<double>, g, b, 0, st, B);
    } else {
        hipLaunchKernelGGL(k_block_propose<float>, g, b, 0, st, B);
        hipLaunchKernelGGL(k_block_apply<float>, g, b, 0, st, B);
    }
    return hipGetLastError();
}

} // namespace mc
