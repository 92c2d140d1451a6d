// qt_rng.h -- counter-based random numbers of the trajectory kernels (device).
//
// Philox-4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two 32x32->64 multiplies
// (multipliers 0xD2511F53, 0xCD9E8D57) with the key bumped by the Weyl constants 0x9E3779B9,
// 0xBB67AE85 between rounds.  Counters: quantum jumps use (trajectory, event, 0); Wiener increments
// use (trajectory, step, 1 + pair), two standard normals per call by the Box-Muller transform.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qt {

__device__ __forceinline__ void philox10(uint32_t c[4], uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c[1] ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c[3] ^ k1;
        c[1] = (uint32_t)p1;
        c[3] = (uint32_t)p0;
        c[0] = n0;
        c[2] = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

// Uniform double in (0, 1) from 27 + 26 bits of two words, offset by half a unit of 2^-53.
__device__ __forceinline__ double u01(uint32_t hi, uint32_t lo)
{
    return ((double)(hi >> 5) * 67108864.0 + (double)(lo >> 6) + 0.5) * (1.0 / 9007199254740992.0);
}

// Standard normals 2*pair and 2*pair + 1 of a trajectory's step (Box-Muller: radius from the first
// uniform, angle from the second; cos for the even one, sin for the odd one).
__device__ __forceinline__ void wiener_normals(uint64_t seed, uint64_t traj, uint32_t step, uint32_t pair, double *z0,
                                               double *z1)
{
    uint32_t c[4] = {(uint32_t)traj, (uint32_t)(traj >> 32), step, 1u + pair};
    philox10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
    const double r = sqrt(-2.0 * log(u01(c[0], c[1])));
    const double th = 6.283185307179586476925286766559 * u01(c[2], c[3]);
    *z0 = r * cos(th);
    *z1 = r * sin(th);
}

}  // namespace qt
