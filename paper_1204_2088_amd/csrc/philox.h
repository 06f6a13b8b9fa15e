// philox.h -- counter-based random numbers for the thermal noise (device side).
//
// Philox4x64 with 10 rounds (Salmon, Moraes, Dror and Shaw, "Parallel random numbers:
// as easy as 1, 2, 3", SC11): each round takes the 128-bit products of counter words 0
// and 2 with two fixed odd multipliers; the new words are the high halves xored with
// words 1 / 3 and the round key, and the low halves.  The key advances by two Weyl
// increments between rounds.  Stateless: any (counter, key) can be drawn by any thread.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace hsf {

struct U64x4 {
    uint64_t v[4];
};

__device__ __forceinline__ U64x4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3, uint64_t k0,
                                               uint64_t k1)
{
    constexpr uint64_t kM0 = 0xD2E7470EE14C6C93ULL, kM1 = 0xCA5A826395121157ULL;
    constexpr uint64_t kW0 = 0x9E3779B97F4A7C15ULL, kW1 = 0xBB67AE8584CAA73BULL;
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint64_t h0 = __umul64hi(kM0, c0), l0 = kM0 * c0;
        const uint64_t h1 = __umul64hi(kM1, c2), l1 = kM1 * c2;
        const uint64_t n0 = h1 ^ c1 ^ k0, n2 = h0 ^ c3 ^ k1;
        c0 = n0;
        c1 = l1;
        c2 = n2;
        c3 = l0;
        k0 += kW0;
        k1 += kW1;
    }
    return U64x4{{c0, c1, c2, c3}};
}

// Four standard normal numbers of counter (site, step, purpose, 0) under key (seed, rep):
// two Box-Muller pairs, radius from u1 = (top 53 bits + 1) 2^-53 in (0, 1], angle
// 2 pi u2 with u2 = (top 53 bits) 2^-53 in [0, 1).
__device__ __forceinline__ void normals4(uint64_t seed, uint64_t rep, uint64_t site, uint64_t step,
                                         uint64_t purpose, double z[4])
{
    const U64x4 r = philox4x64_10(site, step, purpose, 0ULL, seed, rep);
    constexpr double kTwoM53 = 1.0 / 9007199254740992.0;
#pragma unroll
    for (int p = 0; p < 2; ++p) {
        const double u1 = (double)((r.v[2 * p] >> 11) + 1ULL) * kTwoM53;
        const double u2 = (double)(r.v[2 * p + 1] >> 11) * kTwoM53;
        const double rad = sqrt(-2.0 * log(u1));
        double sn, cs;
        sincospi(2.0 * u2, &sn, &cs);   // sin and cos of 2 pi u2, without a rounded 2 pi
        z[2 * p] = rad * cs;
        z[2 * p + 1] = rad * sn;
    }
}

}  // namespace hsf
