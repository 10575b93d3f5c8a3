// Host check of the sampling kernels' threshold-index arithmetic: compares
// theta_index (the same inline function the GPU kernels call) with the plain
// definition clamp(floor((Z*B + 2^(S-1)) / 2^S), -2304, 2304) evaluated in
// 128-bit integers, over random and boundary inputs.  Prints the number of
// mismatches and exits nonzero if there is any.
#include <cstdio>
#include <cstdint>
#include <algorithm>
#include <random>
#include <vector>

#include "../paper_2501_04971_amd/csrc/device_common.h"

typedef __int128 i128;

static int32_t reference(int64_t Z, int32_t B, int S)
{
    i128 v = (i128)Z * B + ((i128)1 << (S - 1));
    i128 d = (i128)1 << S;
    i128 q = v / d;
    if (v % d != 0 && v < 0) q -= 1;
    if (q > 2304) q = 2304;
    if (q < -2304) q = -2304;
    return (int32_t)q;
}

// Per-sweep constants as the instance compiler builds them: A = floor(2^E / B)
// split into 31-bit limbs, rho = 2^E mod B, rho / B as a double; saturated when
// B = 0 or A >= 2^62.
static pbit::ZtSweep sweep_constants(int32_t B, int E)
{
    pbit::ZtSweep z{};
    if (B <= 0) {
        z.sat = 1;
        return z;
    }
    const unsigned __int128 A = ((unsigned __int128)1 << E) / (unsigned)B;
    if (A >= ((unsigned __int128)1 << 62)) {
        z.sat = 1;
        return z;
    }
    const unsigned __int128 rho = ((unsigned __int128)1 << E) % (unsigned)B;
    z.a_hi = (int32_t)(A >> 31);
    z.a_lo = (int32_t)(A & 0x7FFFFFFFu);
    z.rho = (int32_t)rho;
    z.bt = B;
    z.rb = (double)(int32_t)rho / (double)B;
    z.fast = A < ((unsigned __int128)1 << 48) ? 1 : 0;
    return z;
}

int main()
{
    std::mt19937_64 rng(12345);
    long bad = 0, total = 0;
    for (int S = 34; S <= 94; ++S) {
        const int ish = S - 32;
        const int64_t irnd = (int64_t)1 << (S - 33);
        const int32_t hclo = ish <= 31 ? -(int32_t)(1u << (ish - 1)) : INT32_MIN;
        const int32_t hchi = ish <= 31 ? (int32_t)((1u << (ish - 1)) - 1u) : INT32_MAX;
        for (int it = 0; it < 20000; ++it) {
            const int32_t B = it == 0 ? 0 : it == 1 ? INT32_MAX : (int32_t)(rng() >> 33);
            int64_t Z;
            const int mode = it % 4;
            if (mode == 0) {
                Z = (int64_t)(rng() >> 2) * ((rng() & 1) ? 1 : -1);            // |Z| < 2^62
            } else if (mode == 1) {
                Z = (int64_t)(rng() >> (2 + rng() % 60)) * ((rng() & 1) ? 1 : -1);
            } else {
                // near the saturation boundary and the rounding midpoints
                if (B == 0) continue;
                const long double target = (mode == 2 ? 2304.5L : (long double)((int)(rng() % 4609) - 2304) + 0.5L) *
                                           ((rng() & 1) ? 1 : -1);
                const long double z = target * powl(2.0L, S) / (long double)B;
                if (fabsl(z) > 4.0e18L) continue;
                Z = (int64_t)z + (int64_t)(rng() % 5) - 2;
            }
            ++total;
            if (pbit::theta_index(Z, B, ish, irnd, hclo, hchi) != reference(Z, B, S)) {
                if (bad < 10) std::printf("mismatch S=%d Z=%lld B=%d\n", S, (long long)Z, B);
                ++bad;
            }
        }
    }
    // The split kernel's decision: with Theta non-decreasing, Theta[-2304] = 0
    // and Theta[2304] = 2^24, [u < Theta[idx]] = [field_hi >= index_threshold(j*)]
    // with j* = min{ j : Theta[j] > u }.
    std::vector<int32_t> th(4609);
    for (int j = -2304; j <= 2304; ++j)
        th[j + 2304] = (int32_t)llroundl(16777216.0L * (1.0L + tanhl((long double)j / 256.0L)) / 2.0L);
    th[0] = 0;
    th[4608] = 1 << 24;
    long bad2 = 0, total2 = 0;
    for (int S = 34; S <= 94; ++S) {
        const int ish = S - 32;
        const int64_t irnd = (int64_t)1 << (S - 33);
        const int32_t hclo = ish <= 31 ? -(int32_t)(1u << (ish - 1)) : INT32_MIN;
        const int32_t hchi = ish <= 31 ? (int32_t)((1u << (ish - 1)) - 1u) : INT32_MAX;
        for (int it = 0; it < 20000; ++it) {
            const int32_t B = it == 0 ? 0 : (int32_t)(rng() >> 33);
            const int64_t Z = (int64_t)(rng() >> (2 + rng() % 60)) * ((rng() & 1) ? 1 : -1);
            uint32_t u = (uint32_t)(rng() >> 40);
            if (it % 7 == 0) u = (uint32_t)th[rng() % 4609] - (uint32_t)(rng() % 2);  // on table steps
            u &= 0xFFFFFFu;
            const int q = pbit::theta_index(Z, B, ish, irnd, hclo, hchi);
            const bool ref = u < (uint32_t)th[q + 2304];
            const int p = (int)(std::upper_bound(th.begin(), th.end(), (int32_t)u) - th.begin()) - 1;
            const bool got = pbit::field_hi(Z, B, irnd) >= pbit::index_threshold(p + 1 - 2304, ish);
            // the same decision as a threshold on the field itself
            const bool got_z = Z >= pbit::field_threshold(2 * (p + 1 - 2304) - 1, sweep_constants(B, ish + 31));
            ++total2;
            if (ref != got || ref != got_z) {
                if (bad2 < 10) std::printf("split mismatch S=%d Z=%lld B=%d u=%u\n", S, (long long)Z, B, u);
                ++bad2;
            }
        }
    }
    // The field threshold itself against its definition ceil(n 2^E / B) in
    // 128-bit integers (clamped to +-2^62; the sign of n when B = 0), and the
    // decision it stands for, [floor(Z B / 2^32) >= n 2^(E-32)], at and around it.
    long bad3 = 0, total3 = 0;
    const i128 sat = (i128)1 << 62;
    for (int S = 34; S <= 94; ++S) {
        const int E = S - 1;
        for (int it = 0; it < 4000; ++it) {
            const int32_t B = it == 0 ? 0 : it == 1 ? 1 : it == 2 ? INT32_MAX : (int32_t)(rng() >> (33 + rng() % 31));
            const int32_t n = 2 * ((int32_t)(rng() % 4609) - 2304) - 1;
            const pbit::ZtSweep z = sweep_constants(B, E);
            const int64_t got = pbit::field_threshold(n, z);
            i128 want;
            if (B == 0) {
                want = n < 0 ? -sat : sat;
            } else {
                const i128 num = (i128)n * ((i128)1 << E);  // |n| < 2^14, E <= 93: fits
                i128 q = num / B;
                if (num % B != 0 && num > 0) q += 1;  // ceil (C division truncates)
                want = q > sat ? sat : (q < -sat ? -sat : q);
            }
            if (z.fast) {
                // the short form agrees wherever it does not ask for the exact one
                bool near = false;
                const int64_t quick = pbit::field_threshold_fast(n, z, &near);
                ++total3;
                if (!near && quick != got) {
                    if (bad3 < 10) std::printf("short form mismatch S=%d B=%d n=%d\n", S, B, n);
                    ++bad3;
                }
            }
            ++total3;
            if ((i128)got != want) {
                if (bad3 < 10) std::printf("field threshold mismatch S=%d B=%d n=%d\n", S, B, n);
                ++bad3;
                continue;
            }
            for (int dz = -2; dz <= 2; ++dz) {
                i128 Zc = want + dz;
                if (dz == 2) Zc = (i128)(int64_t)(rng() >> (2 + rng() % 60)) * ((rng() & 1) ? 1 : -1);
                if (Zc >= sat || Zc <= -sat) continue;
                const int64_t Z = (int64_t)Zc;
                const i128 prod = (i128)Z * B;
                i128 fl = prod >> 32;  // floor
                const bool ref = fl >= (i128)n * ((i128)1 << (E - 32));
                ++total3;
                if (ref != (Z >= got)) {
                    if (bad3 < 10) std::printf("field decision mismatch S=%d B=%d n=%d Z=%lld\n", S, B, n, (long long)Z);
                    ++bad3;
                }
            }
        }
    }
    std::printf("checked %ld cases, %ld mismatches; split form %ld cases, %ld mismatches; field threshold %ld cases, "
                "%ld mismatches\n", total, bad, total2, bad2, total3, bad3);
    return bad || bad2 || bad3 ? 1 : 0;
}
