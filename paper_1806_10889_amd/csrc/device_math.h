// device_math.h -- device numerics of the SSA on gfx950: the counter-based
// random stream, the two uniforms per event and the project's log.
//
// Philox4x32-10 is the counter-based generator of Salmon, Moraes, Dror and
// Shaw ("Parallel random numbers: as easy as 1, 2, 3", SC'11): four 32-bit
// words, ten rounds of two 32x32->64 products (v_mad_u64_u32 on CDNA), the
// high halves xored into the other words together with the round key, the
// key bumped by the Weyl increments between rounds.
//
// plog(x), x in [2^-53, 1]: log m = 2 atanh((m-1)/(m+1)) summed as an odd
// series in s = (m-1)/(m+1) after folding m into (sqrt2/2, sqrt2], and
// k ln2 added back with ln2 split into a head and a tail (argument reduction
// as in J.-M. Muller, "Elementary Functions").  Every step is an IEEE
// binary64 operation in a fixed order; fma only where written.
#pragma once

#ifndef __HIPCC_RTC__
#include <hip/hip_runtime.h>
#include <stdint.h>
#else
// runtime compilation: the fixed-width integer types live in __hip_internal
using __hip_internal::int8_t;
using __hip_internal::int32_t;
using __hip_internal::int64_t;
using __hip_internal::uint8_t;
using __hip_internal::uint16_t;
using __hip_internal::uint32_t;
using __hip_internal::uint64_t;
#endif

namespace tdev {

struct Words4 {
    uint32_t w0, w1, w2, w3;
};

__device__ __forceinline__ Words4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2,
                                                uint32_t c3, uint32_t k0, uint32_t k1)
{
    constexpr uint32_t kMulA = 0xD2511F53u, kMulB = 0xCD9E8D57u;
    constexpr uint32_t kWeylA = 0x9E3779B9u, kWeylB = 0xBB67AE85u;
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint64_t pa = (uint64_t)kMulA * c0;
        const uint64_t pb = (uint64_t)kMulB * c2;
        const uint32_t n0 = (uint32_t)(pb >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(pa >> 32) ^ c3 ^ k1;
        c1 = (uint32_t)pb;
        c3 = (uint32_t)pa;
        c0 = n0;
        c2 = n2;
        k0 += kWeylA;
        k1 += kWeylB;
    }
    return Words4{c0, c1, c2, c3};
}

// U1 in (0, 1] from words (w0:w1), U2 in [0, 1) from (w2:w3), 53 bits each.
__device__ __forceinline__ void two_uniforms(const Words4 &w, double &u1, double &u2)
{
    const uint64_t hiA = (((uint64_t)w.w0 << 32) | w.w1) >> 11;
    const uint64_t hiB = (((uint64_t)w.w2 << 32) | w.w3) >> 11;
    u1 = (double)(hiA + 1u) * 0x1p-53;
    u2 = (double)hiB * 0x1p-53;
}

// p z + c as the three-operand FMA, so that a coefficient held in a register
// is read in place (the two-operand form overwrites its addend, and a
// coefficient kept for the next call is copied first); the same single
// rounding as fma.
__device__ __forceinline__ double fma3(double p, double z, double c)
{
    double r;
    asm("v_fma_f64 %0, %1, %2, %3" : "=v"(r) : "v"(p), "v"(z), "v"(c));
    return r;
}

// One Horner step of plog: the compiler's fma, or fma3 (same bits).  fma3
// pays where a draw is made at every event (one lane per cell); in the row
// kernel's batched draws the compiler's form schedules better.
template <bool FMA3>
__device__ __forceinline__ double horner_step(double p, double z, double c)
{
    return FMA3 ? fma3(p, z, c) : __builtin_fma(p, z, c);
}

template <bool FMA3 = false>
__device__ __forceinline__ double plog(double x)
{
    // x = m 2^k with m in [1, 2): exponent and mantissa fields (x is normal)
    const uint64_t bits = (uint64_t)__double_as_longlong(x);
    int k = (int)((bits >> 52) & 0x7FFu) - 1023;
    double m = __longlong_as_double((long long)((bits & 0x000FFFFFFFFFFFFFull) |
                                                0x3FF0000000000000ull));
    if (m > 1.4142135623730951) {   // RN(sqrt 2)
        m = m * 0.5;
        k = k + 1;
    }
    const double f = m - 1.0;
    const double s = f / (2.0 + f);
    const double z = s * s;
    // Horner over 2/(2l+3), l = 11 down to 0
    double p = 2.0 / 25.0;
    p = horner_step<FMA3>(p, z, 2.0 / 23.0);
    p = horner_step<FMA3>(p, z, 2.0 / 21.0);
    p = horner_step<FMA3>(p, z, 2.0 / 19.0);
    p = horner_step<FMA3>(p, z, 2.0 / 17.0);
    p = horner_step<FMA3>(p, z, 2.0 / 15.0);
    p = horner_step<FMA3>(p, z, 2.0 / 13.0);
    p = horner_step<FMA3>(p, z, 2.0 / 11.0);
    p = horner_step<FMA3>(p, z, 2.0 / 9.0);
    p = horner_step<FMA3>(p, z, 2.0 / 7.0);
    p = horner_step<FMA3>(p, z, 2.0 / 5.0);
    p = horner_step<FMA3>(p, z, 2.0 / 3.0);
    const double q = __builtin_fma(s * z, p, 2.0 * s);
    const double dk = (double)k;
    return __builtin_fma(dk, 0x1.62e42fefa39efp-1, __builtin_fma(dk, 0x1.abc9e3b39803fp-56, q));
}

}  // namespace tdev
