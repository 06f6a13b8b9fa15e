// common.cuh -- device helpers shared by the kernel translation units.
#pragma once

#include "hsf_internal.h"

namespace hsf {

// Value of the lane to the left (x - 1) and to the right (x + 1) within the wavefront
// (wave_shr:1 / wave_shl:1 data-parallel moves); lane 0 (left) and lane 63 (right) receive
// 0, as does a lane whose source lane is inactive.
__device__ __forceinline__ float from_left(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x138, 0xf, 0xf, false));
}
__device__ __forceinline__ float from_right(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x130, 0xf, 0xf, false));
}
__device__ __forceinline__ double from_left(double v)
{
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, 0x138, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x138, 0xf, 0xf, false);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double from_right(double v)
{
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, 0x130, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x130, 0xf, 0xf, false);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}

// Periodic wrap of an index that is at most one step outside [0, L).
__device__ __forceinline__ int wrap1(int i, int L) { return i < 0 ? i + L : (i >= L ? i - L : i); }

// Work item (tile or site block) of this block.  Blocks are dealt to the chip's eight
// XCDs round robin (block b runs on XCD b mod 8), each with its own L2; this bijection
// gives every XCD a contiguous range of work items, so neighbouring tiles, whose halos
// overlap, share an L2.  Partial results are indexed by the work item.
__device__ __forceinline__ int plan_block()
{
    const int n = (int)gridDim.x, q = n >> 3, rr = n & 7, xcd = (int)blockIdx.x & 7, slot = (int)blockIdx.x >> 3;
    return xcd * q + (xcd < rr ? xcd : rr) + slot;
}

// Q and ln Q of a replica from the sum over its sites of the stored G_N (the stored
// propagators carry the per-step factors 2^-e_s), and whether Q left the range.
__device__ __forceinline__ void q_from_sum(double gsum, double V, const int *scale_e, int N, double &q, double &ln_q,
                                           bool &bad)
{
    q = gsum / V;
    int cum = 0;
    for (int s = 0; s < N; ++s) cum += scale_e[s];
    ln_q = log(q) + cum * 0.69314718055994530942;
    bad = !isfinite(q) || q <= 0.0;
}

// Replica and local site of the calling thread in a site plan.
struct SiteRef {
    int r;
    long long i;
};

__device__ __forceinline__ SiteRef site_ref(const int *blk_rep, const int *blk_first)
{
    SiteRef s;
    const int pb = plan_block();
    s.r = blk_rep[pb];
    s.i = (long long)(pb - blk_first[s.r]) * kBlock + threadIdx.x;
    return s;
}

// Deterministic block sum (fixed shuffle tree inside each 64-lane wavefront, then
// the four wavefront sums in order).  Every thread must call it; the result is
// valid in thread 0.
__device__ __forceinline__ double block_sum(double v)
{
    __shared__ double ws[kBlock / 64];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) ws[wid] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < kBlock / 64; ++k) t += ws[k];
    }
    __syncthreads();
    return t;
}

// Block sums of NV values at once, each bit for bit block_sum's (the same shuffle tree
// and the same order over the wavefronts), with one barrier pair for all of them.  Every
// thread must call it; the results are valid in thread 0.
template <int NV>
__device__ __forceinline__ void block_sums(double (&v)[NV])
{
    __shared__ double ws[NV][kBlock / 64];
#pragma unroll
    for (int q = 0; q < NV; ++q)
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v[q] += __shfl_down(v[q], o, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0)
#pragma unroll
        for (int q = 0; q < NV; ++q) ws[q][wid] = v[q];
    __syncthreads();
    if (threadIdx.x == 0)
#pragma unroll
        for (int q = 0; q < NV; ++q) {
            double t = 0.0;
#pragma unroll
            for (int k = 0; k < kBlock / 64; ++k) t += ws[q][k];
            v[q] = t;
        }
    __syncthreads();
}

// 27-point linkage stencil at (x, y, z): weights by the number of non-zero offset
// components, summed per class (centre, 6 faces, 12 edges, 8 corners).
template <typename real>
__device__ __forceinline__ real stencil27(const real *__restrict__ f, int x, int y, int z, int Lx,
                                          int Ly, int Lz, real c0, real c1, real c2, real c3)
{
    const int xm = wrap1(x - 1, Lx), xp = wrap1(x + 1, Lx);
    const int ym = wrap1(y - 1, Ly), yp = wrap1(y + 1, Ly);
    const int zm = wrap1(z - 1, Lz), zp = wrap1(z + 1, Lz);
    auto row = [&](int yy, int zz, real &ctr, real &side) {
        const real *p = f + ((long long)zz * Ly + yy) * Lx;
        ctr = p[x];
        side = p[xm] + p[xp];
    };
    real a, s, s0, s1, s2, s3;
    row(y, z, a, s);
    s0 = a;
    s1 = s;
    s2 = 0;
    s3 = 0;
    // rows with exactly one of (dy, dz) non-zero
    row(ym, z, a, s); s1 += a; s2 += s;
    row(yp, z, a, s); s1 += a; s2 += s;
    row(y, zm, a, s); s1 += a; s2 += s;
    row(y, zp, a, s); s1 += a; s2 += s;
    // rows with both non-zero
    row(ym, zm, a, s); s2 += a; s3 += s;
    row(ym, zp, a, s); s2 += a; s3 += s;
    row(yp, zm, a, s); s2 += a; s3 += s;
    row(yp, zp, a, s); s2 += a; s3 += s;
    return c0 * s0 + c1 * s1 + c2 * s2 + c3 * s3;
}

}  // namespace hsf
