// Device helpers shared by the sampling kernels (gfx950 only).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pbit_types.h"

namespace pbit {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

// Philox4x32-10 block function (Salmon, Moraes, Dror, Shaw, "Parallel random
// numbers: as easy as 1, 2, 3", SC'11): ten rounds of two 32x32->64 products
// with the Weyl key schedule.  The counter's third word is the replica, fixed
// for a lane, so its first-round product m2 = 0xCD9E8D57 * c2 is passed in.
// a ^ b ^ k in one instruction (gfx950 three-input bitwise op, truth table
// 0x96); k is a key word, uniform across the wave, so it is read as a scalar.
__device__ __forceinline__ uint32_t xor3_key(uint32_t a, uint32_t b, uint32_t k)
{
    uint32_t r;
    asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x96" : "=v"(r) : "v"(a), "v"(b), "s"(k));
    return r;
}

__device__ __forceinline__ void philox_block(uint32_t c0, uint32_t c1, uint64_t m2, uint32_t c3,
                                             uint32_t k0, uint32_t k1, uint32_t out[4])
{
    const uint64_t m0 = (uint64_t)0xD2511F53u * c0;
    uint32_t x0 = xor3_key((uint32_t)(m2 >> 32), c1, k0);
    uint32_t x1 = (uint32_t)m2;
    uint32_t x2 = xor3_key((uint32_t)(m0 >> 32), c3, k1);
    uint32_t x3 = (uint32_t)m0;
#pragma unroll
    for (int rd = 1; rd < 10; ++rd) {
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
        const uint64_t p0 = (uint64_t)0xD2511F53u * x0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * x2;
        const uint32_t y0 = xor3_key((uint32_t)(p1 >> 32), x1, k0);
        const uint32_t y2 = xor3_key((uint32_t)(p0 >> 32), x3, k1);
        x1 = (uint32_t)p1;
        x3 = (uint32_t)p0;
        x0 = y0;
        x2 = y2;
    }
    out[0] = x0;
    out[1] = x1;
    out[2] = x2;
    out[3] = x3;
}

// min(max(v, lo), hi) for lo <= hi: one v_med3_i32 on the device.
__host__ __device__ __forceinline__ int32_t med3_i32(int32_t v, int32_t lo, int32_t hi)
{
#if defined(__HIP_DEVICE_COMPILE__)
    int32_t r;
    asm volatile("v_med3_i32 %0, %1, %2, %3" : "=v"(r) : "v"(v), "v"(lo), "v"(hi));
    return r;
#else
    return v < lo ? lo : (v > hi ? hi : v);
#endif
}

// Threshold index clamp(floor((Z*B + 2^(S-1)) / 2^S), -2304, 2304) for a
// field carried as Z' = 2^u Z with S' = S + u >= 34 (the host picks u), without
// a 128-bit product: Z*B = zh*B*2^32 + zl*B, so
//   hi = floor((Z*B + 2^(S'-1)) / 2^32) = zh*B + (zl*B >> 32) + 2^(S'-33)
// and the index is floor(hi / 2^(S'-32)).  The high word of hi is clamped first
// so that the shifted value fits 32 bits while every out-of-range value still
// lands beyond +-2304; then one 64-bit shift and one clamp finish it.
__host__ __device__ __forceinline__ int32_t theta_index(int64_t Z, int32_t B, int32_t ish, int64_t irnd,
                                               int32_t hclo, int32_t hchi)
{
    const uint64_t lo = (uint64_t)(uint32_t)Z * (uint64_t)(uint32_t)B;
    const int64_t hi = (int64_t)(int32_t)(Z >> 32) * (int64_t)B + (int64_t)(lo >> 32) + irnd;
    const int32_t H = med3_i32((int32_t)(hi >> 32), hclo, hchi);
    const int64_t hc = (int64_t)(((uint64_t)(uint32_t)H << 32) | (uint64_t)(uint32_t)hi);
    int32_t q = (int32_t)(hc >> ish);
    q = q < -kThetaHalf ? -kThetaHalf : q;
    q = q > kThetaHalf ? kThetaHalf : q;
    return q;
}

// hi = floor((Z*B + 2^(S'-1)) / 2^32) for a field carried as Z' = 2^u Z (the
// first step of theta_index, exact for |Z| < 2^62, 0 <= B < 2^31).
__host__ __device__ __forceinline__ int64_t field_hi(int64_t Z, int32_t B, int64_t irnd)
{
    const uint64_t lo = (uint64_t)(uint32_t)Z * (uint64_t)(uint32_t)B;
    return (int64_t)(int32_t)(Z >> 32) * (int64_t)B + (int64_t)(lo >> 32) + irnd;
}

// Threshold on the carried field itself.  With n = 2 j* - 1 (j* the table
// position of the draw) the split kernels' decision
//   [floor(Z B_t / 2^32) >= j* 2^ish - 2^(ish-1)] = [Z B_t >= n 2^E]
// (E = ish + 31) is [Z >= Zt] with Zt = ceil(n 2^E / B_t) for B_t > 0; when
// B_t = 0 it is [n < 0].  Since |Z| < 2^62, a threshold beyond +-2^62 acts as
// +-2^62.  Zt = n A + ceil(n rho / B_t) with A = floor(2^E / B_t), rho = 2^E
// mod B_t (|n rho / B_t| < 2^14); the last term is estimated in double and
// fixed by one exact check (0 <= q B_t - n rho < B_t), the double's error
// being below 2^-38.  The whole result is exact.
__host__ __device__ __forceinline__ int64_t field_threshold(int32_t n, const ZtSweep &z)
{
    constexpr int64_t kSat = (int64_t)1 << 62;
    if (z.sat) return n < 0 ? -kSat : kSat;
    const int64_t nr = (int64_t)n * z.rho;
    int32_t q = (int32_t)ceil((double)n * z.rb);
    const int64_t e = (int64_t)q * z.bt - nr;
    q += e < 0 ? 1 : (e >= (int64_t)z.bt ? -1 : 0);
    // |n A| >= (2^31 + 2^16) 2^31 - 2^45 > 2^62 once |n a_hi| exceeds 2^31 + 2^16;
    // below that n A + q stays under 2^63
    const int64_t hp = (int64_t)n * z.a_hi;
    constexpr int64_t lim = ((int64_t)1 << 31) + ((int64_t)1 << 16);
    const int64_t hc = hp > lim ? lim : (hp < -lim ? -lim : hp);  // (clamped: no overflow below)
    const int64_t zt = hc * ((int64_t)1 << 31) + (int64_t)n * z.a_lo + q;
    if (hp > lim || zt > kSat) return kSat;
    if (hp < -lim || zt < -kSat) return -kSat;
    return zt;
}

// field_threshold for a sweep with fast = 1 (A < 2^48, no saturation): the
// double estimate v of n rho / B_t is within 2^-37 of the exact value, so
// ceil(v) is exact unless v lies within 2^-30 of an integer; such draws (and
// only they) set *near and must be redone with field_threshold.
__host__ __device__ __forceinline__ int64_t field_threshold_fast(int32_t n, const ZtSweep &z, bool *near)
{
    const double v = (double)n * z.rb;
    const double c = ceil(v);
    *near = fabs(v - rint(v)) < 0x1p-30;
    const int32_t hp = n * z.a_hi;
    return (int64_t)hp * ((int64_t)1 << 31) + (int64_t)n * z.a_lo + (int64_t)(int32_t)c;
}

// Threshold on field_hi equivalent to a threshold index: for -2304 < js <= 2304,
// [clamp(floor(hi / 2^ish), +-2304) >= js] = [hi >= js 2^ish], and since
// |hi| < 2^62 a product that would not fit is saturated to +-2^62.
__host__ __device__ __forceinline__ int64_t index_threshold(int js, int ish)
{
    const int aj = js < 0 ? -js : js;
    // |js| < 2^12, so the product fits whenever ish <= 50; above that the
    // 32-bit shift count 62 - ish stays in 0..11
    const bool fits = ish <= 50 || (aj >> (62 - ish)) == 0;
    const int64_t sat = js > 0 ? ((int64_t)1 << 62) : (js < 0 ? -((int64_t)1 << 62) : 0);
    return fits ? (int64_t)js * ((int64_t)1 << ish) : sat;
}

// 24-bit signed multiply (-add) on the vector ALU.  The instructions read only
// the low 24 bits of each operand, so values known to lie in [-2^23, 2^23) need
// no sign extension first (which __mul24 spells out for arbitrary ints).
__device__ __forceinline__ int32_t mul_i24(int32_t a, int32_t b)
{
    int32_t r;
    asm("v_mul_i32_i24 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}

__device__ __forceinline__ int32_t mad_i24(int32_t a, int32_t b, int32_t c)
{
    int32_t r;
    asm("v_mad_i32_i24 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}

// Four 0/1 bytes of a word -> four bits.
__device__ __forceinline__ uint32_t bytes_to_nibble(uint32_t v)
{
    return (v | (v >> 7) | (v >> 14) | (v >> 21)) & 0xFu;
}

__device__ __forceinline__ void swap_halves(uint32_t &a, uint32_t &b)
{
    // lanes 32..63 of a trade places with lanes 0..31 of b
    auto s = __builtin_amdgcn_permlane32_swap(a, b, false, false);
    a = s[0];
    b = s[1];
}

}  // namespace pbit
